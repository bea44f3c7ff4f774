"""Benchmark: Rotne-Prager-Blake Brownian dynamics steps at N = 65,536 on one MI355X.

One "step" is one stochastic Adams-Bashforth step of the full hot path (paper, Sec. II):
steric + gravity forces, the deterministic product u = M F + M_C T, the Lanczos Brownian
increment M^{1/2} W (tolerance 1e-3), the centred random finite difference (two products)
and the update.  Positions and noise are synthetic and resident on the GPU before the
timed region starts (a uniform sheet at area fraction 0.4, heights in [1.1, 2.5]; noise
drawn on the device from Philox).

Prints ONE JSON line.  ``value`` is the pair interactions evaluated per second over the
timed steps (every product counts N^2 ordered pairs); ``steps_per_s`` the step rate.
The ``roofline`` object prices the dominant kernel (the float32 pair kernel) against the
float32 vector-ALU peak; ``cpu_baseline`` times the FP64 CPU oracle on a sample of rows.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic operation count of one ordered pair (the closed form evaluated by the pair
# kernel: add/sub/mul = 1, FMA = 2, rsqrt = 1; the two separations x_i - x_j, y_i - y_j and
# the three accumulations are included; float32 hi/lo reconstruction, Kahan compensation,
# index math, selects and branches are not).  Far branch (|r| >= 2a), i.e. all but the few
# overlapping pairs.
FLOPS_PER_PAIR_FORCE = 106   # source carries a force only (Lanczos and RFD products)
FLOPS_PER_PAIR_TORQUE = 147  # source carries a force and a torque (deterministic product)
PEAK_FP32_TFLOPS = 157.3     # 256 CU x 128 FP32 lanes x 2 (FMA) x 2.4 GHz
PEAK_FP64_TFLOPS = 78.6
KIND_FP64_FORCE, KIND_FP64_TORQUE, KIND_MIXED_FORCE, KIND_MIXED_TORQUE = 0, 1, 2, 3
KIND_MULTI_FP64, KIND_MULTI_MIXED = 8, 10   # multi-vector kernel (pairs counted per vector)


PROFILED_N = 65536   # sheet size of the committed counter summary


def kernel_source_hash() -> str:
    """sha256[:16] of the pair-kernel sources with comments and blank lines removed (so that
    editing a comment does not void the recorded counters)."""
    import hashlib
    import re
    csrc = os.path.join(ROOT, "paper_1612_00474_amd", "csrc")
    h = hashlib.sha256()
    for name in ("matvec.hip", "multi.hip", "pair_common.h", "pair_tensor.h"):
        with open(os.path.join(csrc, name)) as f:
            for line in f:
                code = re.sub(r"//.*$", "", line).strip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


class ClockSampler:
    """Samples the GPU shader clock (the active level of the sysfs pp_dpm_sclk table) from a
    background thread while the timed steps run; best effort, empty where it is not readable."""

    def __init__(self, period=0.05):
        import glob
        import threading
        self.paths = sorted(glob.glob("/sys/class/drm/card*/device/pp_dpm_sclk"))
        self.period = period
        self.mhz = []
        self._stop = threading.Event()
        self._thread = threading.Thread(target=self._run, daemon=True)

    def _read(self):
        for path in self.paths:
            try:
                with open(path) as f:
                    for line in f:
                        if line.rstrip().endswith("*"):
                            return float(line.split(":")[1].strip().split("Mhz")[0].split("MHz")[0])
            except (OSError, ValueError, IndexError):
                continue
        return None

    def _run(self):
        while not self._stop.is_set():
            v = self._read()
            if v is not None:
                self.mhz.append(v)
            self._stop.wait(self.period)

    def __enter__(self):
        if self.paths:
            self._thread.start()
        return self

    def __exit__(self, *exc):
        self._stop.set()
        if self._thread.is_alive():
            self._thread.join()

    def summary(self):
        if not self.mhz:
            return None
        v = sorted(self.mhz)
        return {"sclk_mhz_median": v[len(v) // 2], "sclk_mhz_min": v[0], "sclk_mhz_max": v[-1],
                "samples": len(v), "source": "pp_dpm_sclk during the timed steps"}


def measured_traffic(kernel: str, n: int = PROFILED_N):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary, or None
    when the kernel sources changed since the counters were taken or `n` is another size."""
    if n != PROFILED_N:
        return None
    current = kernel_source_hash()
    path = os.path.join(ROOT, "profiles", "pair_kernels_sheet64k_hbm_traffic.md")
    try:
        with open(path) as f:
            for line in f:
                parts = line.rstrip("\n").split("\t")
                if len(parts) == 3 and parts[0] == kernel and parts[2] == current:
                    return float(parts[1])
    except OSError:
        pass
    return None


def force_kernel_name(prec: str, shape: dict) -> str:
    """rocprofv3 name of the pair kernel that a force-only product launches with `shape`."""
    kind = "mixed" if prec == "mixed" else "f64"
    # template arguments: (targets per lane, torque, wall, periodic) for the symmetric kernel,
    # (torque, targets per lane, wall, periodic) for the ordered one
    if shape["symmetric"]:
        return f"pair_kernel_{kind}_sym<{shape['tpt']}, false, true, false>"
    return f"pair_kernel_{kind}<false, {shape['tpt']}, true, false>"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="sheet64k_mixed")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rows", type=int, default=48)
    return ap.parse_args()


def cpu_baseline(w, rows):
    """Time the FP64 oracle's matrix-free product on `rows` target rows (all N sources); for a
    batch, on rows of its first system, sized to about the same number of pairs."""
    import numpy as np
    from oracle import mobility
    from paper_1612_00474_amd import workloads as wl
    if w.nsys > 1:
        pos_b, offs = wl.make_batch(w, 0)
        n = int(offs[1])
        pos = pos_b[:n]
        rng = np.random.default_rng(0)
        force, torque = rng.standard_normal((n, 3)), rng.standard_normal((n, 3))
        rows = min(n, max(1, rows * 65536 // n))
        what = f"system 0 of the batch (N = {n})"
    else:
        inp = wl.make_inputs(w, 0)
        pos, force, torque, n = inp["pos"], inp["force"], inp["torque"], w.n
        rows = min(n, max(1, rows * 65536 // n))
        what = f"{n} sources"
    sel = np.arange(rows)
    mobility.matvec(pos[:64], force[:64], torque[:64])   # warm the tensors
    t0 = time.perf_counter()
    mobility.matvec(pos, force, torque, rows=sel)
    dt = time.perf_counter() - t0
    pairs = rows * n
    return {"value": pairs / dt, "unit": "pair-interactions/s", "cores": 1, "kind": "oracle",
            "sample": f"{rows} target rows x {what}, one product M F + M_C T "
                      f"({pairs:.3e} pairs, {dt:.1f} s, single process)"}


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE={world}): "
              "the library has no multi-GPU path.", file=sys.stderr)
        sys.exit(2)

    from paper_1612_00474_amd import workloads as wl
    w = wl.WORKLOADS[args.workload]

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(w, args.cpu_rows)   # before the GPU is touched

    import numpy as np
    import torch
    from paper_1612_00474_amd import Context, StepState

    torch.cuda.init()
    ctx = Context(0, a=w.a, eta=w.eta, kT=w.kT)
    if w.nsys > 1:
        return bench_batched(args, w, ctx, cpu)
    inp = wl.make_inputs(w, 0)
    pos0 = torch.as_tensor(inp["pos"]).cuda()
    F = torch.as_tensor(inp["force"]).cuda()
    T = torch.as_tensor(inp["torque"]).cuda()
    prec = w.precision
    step_kw = dict(dt=w.dt, delta=w.delta, lanczos_tol=w.lanczos_tol, lanczos_max_iter=64,
                   rfd_precision="fp64", f_grav_z=w.f_grav_z, torque=w.torque,
                   steric_u0=w.steric_u0, steric_b=w.steric_b, seed=0, precision=prec)

    # ---- launch shapes from the tuner (timed on this configuration, cached per size) -------
    shapes = {prec_: ctx.autotune(pos0, None, prec_)[0] for prec_ in ("mixed", "fp64")}

    # ---- kernel-only product throughput, mixed and float64 (pair kernel, HIP events) ----
    def kernel_rate(precision, reps=3):
        ctx.matvec(pos0, F, T, precision)
        torch.cuda.synchronize()
        ctx.timing(True)
        ctx.timing_read()
        for _ in range(reps):
            ctx.matvec(pos0, F, T, precision)
        ms, launches, pairs = ctx.timing_read()
        ctx.timing(False)
        return pairs / (ms * 1e-3), ms / launches

    mixed_rate, mixed_ms = kernel_rate("mixed")
    f64_rate, f64_ms = kernel_rate("fp64")

    # ---- multi-vector product: four force vectors of this configuration per launch -------
    FF = torch.as_tensor(np.random.default_rng(7).standard_normal((4, w.n, 3))).cuda()

    def multi_rate(precision, reps=3):
        kind = KIND_MULTI_MIXED if precision == "mixed" else KIND_MULTI_FP64
        one = KIND_MIXED_FORCE if precision == "mixed" else KIND_FP64_FORCE
        ctx.matvec_multi(pos0, FF, precision)
        torch.cuda.synchronize()
        ctx.timing(True)
        ctx.timing_read()
        for _ in range(reps):
            ctx.matvec_multi(pos0, FF, precision)
            ctx.matvec(pos0, FF[0], None, precision)
        ms, launches, pairs = ctx.timing_read(kind)
        ms1, launches1, pairs1 = ctx.timing_read(one)
        ctx.timing(False)
        rate, rate1 = pairs / (ms * 1e-3), pairs1 / (ms1 * 1e-3)
        return {"vector_pairs_per_s": rate, "ms_per_launch": ms / launches,
                "single_vector_pairs_per_s": rate1, "speedup_per_vector": rate / rate1}

    multi = {"vectors_per_launch": 4, "mixed": multi_rate("mixed"), "fp64": multi_rate("fp64")}

    # ---- pseudo-periodic product: the same sheet in a box of its own side, each pair taken
    # with the minimum image and its eight neighbours (nine image pairs per ordered pair) -----
    pctx = Context(0, a=w.a, eta=w.eta, kT=w.kT, box=(w.side, w.side))

    def periodic_rate(precision, reps=2):
        pctx.matvec(pos0, F, None, precision)
        torch.cuda.synchronize()
        pctx.timing(True)
        pctx.timing_read()
        for _ in range(reps):
            pctx.matvec(pos0, F, None, precision)
        ms, launches, pairs = pctx.timing_read()
        pctx.timing(False)
        rate = 9.0 * pairs / (ms * 1e-3)
        # logical count: 106 flop per ordered image pair, although the kernel evaluates each
        # unordered pair's coefficients once and the image-independent terms once per pair
        return {"ms_per_launch": ms / launches, "image_pairs_per_s": rate,
                "tflops_logical": FLOPS_PER_PAIR_FORCE * rate / 1e12}

    periodic = {"box": [w.side, w.side], "images_per_pair": 9, "force_only": True,
                "mixed": periodic_rate("mixed"), "fp64": periodic_rate("fp64")}
    pctx.close()

    # ---- time steps ----------------------------------------------------------------------
    state = StepState(pos0.clone())
    iters = []
    for _ in range(args.warmup):
        iters.append(ctx.sab_step(state, **step_kw)[0])
    torch.cuda.synchronize()
    ctx.timing(True)
    ctx.timing_read()
    with ClockSampler() as clocks:
        t0 = time.perf_counter()
        for _ in range(args.steps):
            iters.append(ctx.sab_step(state, **step_kw)[0])
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
    kinds = {}
    for name, kind, fpp in (("fp64_force", KIND_FP64_FORCE, FLOPS_PER_PAIR_FORCE),
                            ("fp64_torque", KIND_FP64_TORQUE, FLOPS_PER_PAIR_TORQUE),
                            ("mixed_force", KIND_MIXED_FORCE, FLOPS_PER_PAIR_FORCE),
                            ("mixed_torque", KIND_MIXED_TORQUE, FLOPS_PER_PAIR_TORQUE)):
        ms, k, pairs = ctx.timing_read(kind)
        if k:
            kinds[name] = {"launches": k, "ms_per_launch": ms / k,
                           "pairs_per_s": pairs / (ms * 1e-3),
                           "tflops": fpp * pairs / (ms * 1e-3) / 1e12}
    # the two-vector launch of each step: M F + M_C T together with the first Lanczos product
    for name, kind in (("fp64_two_vector", KIND_MULTI_FP64), ("mixed_two_vector", KIND_MULTI_MIXED)):
        ms, k, pairs = ctx.timing_read(kind)
        if k:
            kinds[name] = {"launches": k, "ms_per_launch": ms / k,
                           "vector_pairs_per_s": pairs / (ms * 1e-3)}
    ctx.timing(False)
    timed_iters = iters[args.warmup:]
    n = w.n
    products = sum(1 + m + 2 for m in timed_iters)
    step_pairs = products * float(n) * n
    value = step_pairs / elapsed

    if cpu is not None:
        # the oracle's step rate, extrapolated from its sampled product rate at the Lanczos
        # counts of the timed steps (products only; the O(N) work is left out)
        cpu["steps_per_s_extrapolated"] = cpu["value"] * len(timed_iters) / step_pairs
        cpu["steps_per_s_note"] = ("extrapolated: rate / ((1 + m + 2) N^2) at the GPU "
                                   "steps' Lanczos m, not timed")

    # dominant kernel: the pair kernel of the Lanczos products (most launches and most time)
    dom = kinds["mixed_force" if prec == "mixed" else "fp64_force"]
    peak = PEAK_FP32_TFLOPS if prec == "mixed" else PEAK_FP64_TFLOPS
    achieved = dom["tflops"]
    line = {
        "metric": "RPB matvec pair-interactions/s + BD steps/s at N=65,536, FP32-mixed vs FP64",
        "value": value,
        "unit": "pair-interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "steps_per_s": args.steps / elapsed,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "n": n, "area_fraction": 0.4, "z_range": [w.z_lo, w.z_hi],
                   "scheme": "stochastic Adams-Bashforth", "dt": w.dt, "rfd_delta": w.delta,
                   "lanczos_tol": w.lanczos_tol, "precision": prec, "rfd_precision": "fp64",
                   "parallelism": "single GPU"},
        "lanczos_iters": timed_iters,
        "launch_shapes": shapes,
        "matvec_kernel_pairs_per_s": {"mixed": mixed_rate, "fp64": f64_rate,
                                      "mixed_over_fp64": mixed_rate / f64_rate,
                                      "ms_per_launch": {"mixed": mixed_ms, "fp64": f64_ms}},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak,
                     "traffic": measured_traffic(force_kernel_name(prec, shapes[prec]), n),
                     "kernel": f"{force_kernel_name(prec, shapes[prec])}, force-only "
                               f"products ({FLOPS_PER_PAIR_FORCE} flop/pair x {n}^2 pairs/launch)",
                     "ms_per_launch": dom["ms_per_launch"], "launches": dom["launches"]},
        "pair_kernels": kinds,
        "multi_vector_product": multi,
        "periodic_product": periodic,
        "gpu_clock": clocks.summary(),
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))
    ctx.close()


def bench_batched(args, w, ctx, cpu):
    """Batched suspensions: one persistent launch per product, steps replayed from a hipGraph."""
    import numpy as np
    import torch
    from paper_1612_00474_amd import workloads as wl

    pos_np, offs = wl.make_batch(w, 0)
    sizes = np.diff(offs)
    n = int(offs[-1])
    sum_sq = float(np.sum(sizes.astype(np.float64) ** 2))
    pos0 = torch.as_tensor(pos_np).cuda()
    F = torch.as_tensor(np.random.default_rng(0).standard_normal((n, 3))).cuda()
    shapes = {prec_: ctx.autotune(pos0, offs, prec_)[0] for prec_ in ("mixed", "fp64")}

    def kernel_rate(precision, reps=5):
        ctx.matvec_batched(pos0, offs, F, None, precision)
        torch.cuda.synchronize()
        ctx.timing(True)
        ctx.timing_read()
        for _ in range(reps):
            ctx.matvec_batched(pos0, offs, F, None, precision)
        ms, k, pairs = ctx.timing_read()
        ctx.timing(False)
        return {"pairs_per_s": pairs / (ms * 1e-3), "ms_per_launch": ms / k,
                "tflops": FLOPS_PER_PAIR_FORCE * pairs / (ms * 1e-3) / 1e12}

    rates = {"mixed": kernel_rate("mixed"), "fp64": kernel_rate("fp64")}
    budget = 16
    kw = dict(dt=w.dt, delta=w.delta, lanczos_tol=w.lanczos_tol, lanczos_max_iter=budget,
              rfd_precision="fp64", f_grav_z=w.f_grav_z, torque=w.torque, steric_u0=w.steric_u0,
              steric_b=w.steric_b, seed=0, precision=w.precision)
    P = pos0.clone()
    U = torch.zeros_like(P)
    graph = ctx.step_graph(P, U, offs, 0, False, **kw)
    for _ in range(args.warmup):
        graph.launch()
    torch.cuda.synchronize()
    with ClockSampler() as clocks:
        t0 = time.perf_counter()
        for _ in range(args.steps):
            graph.launch()
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
    step, iters, eps, _ = graph.status()
    graph.close()
    # eager batched steps (host reads the Lanczos flags every iteration) for comparison
    Pe = pos0.clone()
    Ue = torch.zeros_like(Pe)
    ctx.sab_step_batched(Pe, Ue, offs, 0, False, **kw)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for k in range(args.steps):
        ctx.sab_step_batched(Pe, Ue, offs, k + 1, True, **kw)
    torch.cuda.synchronize()
    eager = time.perf_counter() - t1
    pairs_step = float(np.sum(sizes.astype(np.float64) ** 2 * (3 + iters)))
    dom = rates["mixed" if w.precision == "mixed" else "fp64"]
    peak = PEAK_FP32_TFLOPS if w.precision == "mixed" else PEAK_FP64_TFLOPS
    line = {
        "metric": "RPB matvec pair-interactions/s + BD steps/s, batched suspensions",
        "value": pairs_step * args.steps / elapsed,
        "unit": "pair-interactions/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "steps_per_s": args.steps / elapsed,
        "eager_steps_per_s": args.steps / eager,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if w.precision == "mixed" else "f64", "data": "synthetic",
        "config": {"workload": w.name, "nsys": int(w.nsys), "n_total": n,
                   "sizes": [int(x) for x in sizes], "sum_n_squared": sum_sq,
                   "precision": w.precision, "rfd_precision": "fp64",
                   "lanczos_tol": w.lanczos_tol, "lanczos_budget": budget,
                   "graph": "one hipGraph launch per step", "parallelism": "single GPU"},
        "lanczos_iters_last_step": [int(x) for x in iters],
        "launch_shapes": shapes,
        "batched_kernel": rates,
        "gpu_clock": clocks.summary(),
        "roofline": {"bound": "alu", "achieved": dom["tflops"], "peak": peak, "unit": "TFLOP/s",
                     "frac": dom["tflops"] / peak, "traffic": None,
                     "kernel": f"batched pair kernel, force-only, {FLOPS_PER_PAIR_FORCE} flop/pair x "
                               f"sum N_s^2 = {sum_sq:.4e} pairs/launch",
                     "ms_per_launch": dom["ms_per_launch"]},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))
    ctx.close()


if __name__ == "__main__":
    main()
