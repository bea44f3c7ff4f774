"""Lanczos iteration counts against N: with the wall, with the wall and the block-diagonal
preconditioner, and in free space.

Sec. II.C: with the wall, hydrodynamic interactions in a sedimented sheet are screened
(far field ~ 1/r^3) and the number of Lanczos iterations for M^{1/2} W at a fixed relative
tolerance does not grow with N; in free space (unscreened 1/r interactions) it does.  This
driver measures both on the synthetic sheets (area fraction 0.4, heights uniform in
[1.1, 2.5]) for several N and tolerances, with the same noise vector in every mode.  Sec. II.C
also reports that a block-diagonal preconditioner (wall self-terms) gives only a very small
improvement; the second mode measures that.  ``--recipe sedimented`` uses instead the
configuration of the paper's convergence study (area fraction 0.25, heights with an
exponential profile of mean 1.6a, no overlaps; ``workloads.sedimented_sheet``):

    python -m paper_1612_00474_amd.lanczos_scan [--sizes 1024 4096 16384 65536] [--recipe sedimented]

Prints one JSON line per (N, mode) and a final summary line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--sizes", type=int, nargs="+", default=[1024, 4096, 16384, 65536])
    ap.add_argument("--tols", type=float, nargs="+", default=[1e-3, 1e-5])
    ap.add_argument("--precision", default="mixed")
    ap.add_argument("--recipe", choices=["sheet", "sedimented"], default="sheet")
    args = ap.parse_args()

    import numpy as np
    import torch

    from paper_1612_00474_amd import Context
    from paper_1612_00474_amd import workloads as wl

    torch.cuda.init()
    wall = Context(0)
    modes = {"wall": (wall, False), "wall + block-diagonal preconditioner": (wall, True),
             "free space": (Context(0, wall=False), False)}
    rows = []
    for n in args.sizes:
        host = wl.sheet(n, seed=0) if args.recipe == "sheet" else wl.sedimented_sheet(n, seed=0)
        pos = torch.as_tensor(host).cuda()
        w = torch.as_tensor(np.random.default_rng(1).standard_normal((n, 3))).cuda()
        for mode, (ctx, precond) in modes.items():
            row = {"n": n, "mode": mode, "recipe": args.recipe, "precision": args.precision}
            for tol in args.tols:
                g, it, eps, st = ctx.lanczos(pos, w, tol, max_iter=64, precision=args.precision,
                                             allow_noconv=True, precond=precond)
                row[f"m@{tol:g}"] = int(it)
                row[f"eps@{tol:g}"] = float(eps)
            rows.append(row)
            print(json.dumps(row), flush=True)
    for ctx, _ in modes.values():
        if ctx.h:
            ctx.close()
    print(json.dumps({"summary": {f"{r['mode']} N={r['n']}": {k: v for k, v in r.items()
                                                               if k.startswith("m@")}
                                  for r in rows}}))


if __name__ == "__main__":
    main()
