"""Writes the oracle's values on sampled rows of the large sheets, for the GPU parity tests:

  sheet64k_rows.txt   U = M F + M_C T on 256 rows and the centred RFD drift on 64 rows of the
                      65,536-sphere sheet (area fraction 0.4, heights in [1.1a, 2.5a]);
  sheet256k_rows.txt  U = M F + M_C T on 1,024 rows of the 262,144-sphere sheet (heights in
                      [1.1a, 2.0a]).

Inputs are the seeded workloads of paper_1612_00474_amd.workloads (seed 0): positions, forces
and torques, W~.  Rows are drawn by numpy.random.default_rng(9) without replacement, the last
sphere (ragged last tile) always included.  Calls the oracle only (matrix-free direct sums,
Sec. II.B; the RFD of Sec. II.A), over a pool of worker processes:

    python tests/golden/make_sheet_rows.py [--workers 8] [--only sheet64k|sheet256k]
"""
import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import mobility, stochastic  # noqa: E402
from paper_1612_00474_amd import workloads as wl  # noqa: E402


def sample_rows(n, k, seed=9):
    rows = np.random.default_rng(seed).choice(n, k, replace=False)
    rows[0] = n - 1
    return rows


def fingerprint(inp):
    """Sums of the inputs, to detect a change of the input generator."""
    return {key: float(np.sum(inp[key])) for key in ("pos", "force", "torque", "w_tilde")}


def write(path, name, inp, sections, note):
    with open(path, "w") as f:
        f.write(f"# {note}\n# written by tests/golden/make_sheet_rows.py (oracle only)\n")
        f.write(f"workload {name}\n")
        for key, v in fingerprint(inp).items():
            f.write(f"sum_{key} {v!r}\n")
        for tag, rows, vals in sections:
            for r, v in zip(rows, vals):
                f.write(f"{tag} {int(r)} " + " ".join(repr(float(x)) for x in v) + "\n")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=8)
    ap.add_argument("--only", default=None)
    args = ap.parse_args()
    if args.only in (None, "sheet64k"):
        w = wl.WORKLOADS["sheet64k_mixed"]
        inp = wl.make_inputs(w, 0)
        t0 = time.time()
        ru = sample_rows(w.n, 256)
        u = mobility.matvec(inp["pos"], inp["force"], inp["torque"], rows=ru,
                            workers=args.workers)
        rd = sample_rows(w.n, 64, seed=13)
        d = stochastic.rfd(inp["pos"], inp["w_tilde"], w.delta, rows=rd, workers=args.workers)
        write(os.path.join(HERE, "sheet64k_rows.txt"), w.name, inp,
              [("u", ru, u), ("drift", rd, d)],
              f"65,536-sphere sheet: U = M F + M_C T on 256 rows, centred RFD drift "
              f"(delta = {w.delta}, kT = 1) with W~ on 64 rows")
        print(f"sheet64k: {time.time() - t0:.0f} s")
    if args.only in (None, "sheet256k"):
        w = wl.WORKLOADS["sheet256k_mixed"]
        inp = wl.make_inputs(w, 0)
        t0 = time.time()
        ru = sample_rows(w.n, 1024)
        u = mobility.matvec(inp["pos"], inp["force"], inp["torque"], rows=ru,
                            workers=args.workers)
        write(os.path.join(HERE, "sheet256k_rows.txt"), w.name, inp, [("u", ru, u)],
              "262,144-sphere sheet: U = M F + M_C T on 1,024 rows")
        print(f"sheet256k: {time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()
