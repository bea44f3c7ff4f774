"""Kernel profiling driver (run under rocprofv3).

On one synthetic sheet of N spheres, launches one plain device-to-device copy of known size
(to calibrate the HBM byte counters FETCH_SIZE / WRITE_SIZE against a kernel whose traffic is
known) followed by `--reps` launches of every whole-system pair-kernel variant the tuner may
pick (the symmetric kernel at 1, 2 and 4 targets per lane, force only and with a torque, both
precisions; the shape is set explicitly, so every counter pass sees the same kernels), of the
multi-vector kernel (four vectors per launch) and of the steric force kernel.  Only the
dispatches after the copy count:

    rocprofv3 --kernel-trace --stats -d OUT -o run -- python -m paper_1612_00474_amd.profile_kernels
    rocprofv3 --pmc FETCH_SIZE -d OUT -o fetch -- python -m paper_1612_00474_amd.profile_kernels
    rocprofv3 --pmc WRITE_SIZE -d OUT -o write -- python -m paper_1612_00474_amd.profile_kernels

Prints one JSON line with the copy size and the pair-kernel launches made.
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
    ap.add_argument("--n", type=int, default=65536)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--copy-mib", type=int, default=512)
    args = ap.parse_args()

    import numpy as np
    import torch

    from paper_1612_00474_amd import Context
    from paper_1612_00474_amd import workloads as wl

    torch.cuda.init()
    pos = torch.as_tensor(wl.sheet(args.n, seed=0)).cuda()
    rng = np.random.default_rng(0)
    F = torch.as_tensor(rng.standard_normal((args.n, 3))).cuda()
    T = torch.as_tensor(rng.standard_normal((args.n, 3))).cuda()
    ctx = Context(0)
    torch.cuda.synchronize()

    nelem = args.copy_mib * (1 << 20) // 8
    src = torch.ones(nelem, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()

    launches = []
    for precision in ("mixed", "fp64"):
        for tpt in (1, 2, 4):
            ctx.set_tuning(precision, tpt=tpt, symmetric=1)
            for torque in (None, T):
                for _ in range(args.reps):
                    ctx.matvec(pos, F, torque, precision)
                launches.append({"precision": precision, "tpt": tpt, "torque": torque is not None,
                                 "reps": args.reps})
    FF = torch.as_tensor(rng.standard_normal((4, args.n, 3))).cuda()
    for precision in ("mixed", "fp64"):
        for _ in range(args.reps):
            ctx.matvec_multi(pos, FF, precision)
        launches.append({"precision": precision, "multi_vector": 4, "reps": args.reps})
    for _ in range(args.reps):
        ctx.forces(pos, f_grav_z=-1.0, u0=1.0, b=0.1)
    launches.append({"kernel": "steric", "reps": args.reps})
    torch.cuda.synchronize()
    ctx.close()
    print(json.dumps({"copy_bytes": nelem * 8, "n": args.n, "launches": launches}))


if __name__ == "__main__":
    main()
