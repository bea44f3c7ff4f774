"""Writes periodic_not_spd.txt: a crowded pseudo-periodic configuration whose truncated image
sum M (App. B: minimum image plus the eight neighbour cells) is indefinite, a noise vector w,
and what the oracle's Lanczos (Sec. II.C) does on it: the iteration at which a Ritz value first
falls below -1e-12 times the largest.  Calls the oracle only:

    python tests/golden/make_periodic_not_spd.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import lanczos, mobility  # noqa: E402


def ritz_min_ratio(M, w, m):
    """Smallest / largest Ritz value after m plain Lanczos steps (full re-orthogonalisation)."""
    V = [w / np.linalg.norm(w)]
    al, be = [], []
    for k in range(m):
        u = M @ V[-1]
        al.append(V[-1] @ u)
        Vm = np.array(V)
        u = u - Vm.T @ (Vm @ u)
        u = u - Vm.T @ (Vm @ u)
        if k + 1 < m:
            be.append(np.linalg.norm(u))
            V.append(u / be[-1])
    T = np.diag(al) + np.diag(be, 1) + np.diag(be, -1)
    lam = np.linalg.eigvalsh(T)
    return lam[0] / lam[-1]


def main():
    rng = np.random.default_rng(2024)
    for trial in range(2000):
        n = int(rng.integers(12, 22))
        L = float(rng.uniform(3.5, 5.0))
        pos = np.column_stack([rng.uniform(0, L, n), rng.uniform(0, L, n),
                               rng.uniform(1.0, 2.5, n)])
        M, _ = mobility.dense(pos, box=(L, L))
        lam = np.linalg.eigvalsh(M)
        if lam[0] / lam[-1] > -1e-3:
            continue
        w = rng.standard_normal(3 * n)
        g, m, eps, status = lanczos.lanczos_sqrt(lambda v: M @ v, w, 1e-300, 64)
        if status != "notspd" or m < 3:
            continue
        # a clean crossing: clearly positive one iteration before, clearly negative at m
        before, at = ritz_min_ratio(M, w, m - 1), ritz_min_ratio(M, w, m)
        if before < 1e-6 or at > -1e-6:
            continue
        break
    else:
        raise SystemExit("no configuration found")
    out = os.path.join(HERE, "periodic_not_spd.txt")
    with open(out, "w") as f:
        f.write("# Crowded pseudo-periodic configuration (App. B image set) whose truncated image sum\n")
        f.write("# is indefinite; written by tests/golden/make_periodic_not_spd.py (oracle only).\n")
        f.write(f"# lambda_min / lambda_max of the dense oracle M: {lam[0] / lam[-1]:.6e}\n")
        f.write(f"# oracle Lanczos (tol 1e-300, max 64 iterations): status notspd at m = {m}\n")
        f.write(f"# smallest / largest Ritz value at m - 1: {before:.3e}, at m: {at:.3e}\n")
        f.write(f"box {L!r} {L!r}\n")
        f.write(f"notspd_m {m}\n")
        for i in range(n):
            f.write("pos " + " ".join(repr(float(x)) for x in pos[i]) + "\n")
        for i in range(n):
            f.write("w " + " ".join(repr(float(x)) for x in w[3 * i:3 * i + 3]) + "\n")
    print(f"wrote {out}: n = {n}, L = {L:.3f}, lambda ratio {lam[0] / lam[-1]:.3e}, m = {m}")


if __name__ == "__main__":
    main()
