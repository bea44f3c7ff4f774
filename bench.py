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
float32 vector-ALU peak with the operation count of the algorithm it runs (one evaluation
per unordered pair, applied in both directions); the logical count (every ordered pair
charged in full) and the arithmetic the hardware counters saw issued sit beside it.
``batched`` times the 64-system mixed batch (one hipGraph launch per step), ``fp64_sheet16k``
and ``fp64_sheet256`` the float64 steps at N = 16,384 and N = 256 (eager and graph-captured).
``cpu_baseline`` times the FP64 CPU oracle over the host's cores on bounded samples.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# ---- operation counts (add/sub/mul = 1, FMA = 2, rsqrt = 1; float32 hi/lo reconstruction,
# Kahan compensation, index math, selects and branches excluded; far branch |r| >= 2a, i.e.
# all but the few overlapping pairs) ----------------------------------------------------------
# Ordered pair (target i, source j) of the closed form, separations and accumulation included:
FLOP_ORD_FORCE = 106     # source carries a force only (Lanczos and RFD products)
FLOP_ORD_TORQUE = 147    # force and torque (deterministic product)
# Symmetric kernel, per unordered pair {i, j}: the separations (2), the pair's coefficients
# once (75: geometry and unbounded part 19, wall part 56), then per vector both directions of
# the force application (2 x 20) and, with torques, both coupling directions (77).
FLOP_SEP, FLOP_COEF, FLOP_APPLY, FLOP_TORQUE_APPLY = 2, 75, 40, 77
FLOP_SYM_FORCE = FLOP_SEP + FLOP_COEF + FLOP_APPLY                     # 117
FLOP_SYM_TORQUE = FLOP_SYM_FORCE + FLOP_TORQUE_APPLY                   # 194

PEAK_FP32_TFLOPS = 157.3     # 256 CU x 2.4 GHz x 256 FP32 flop per CU per clock
PEAK_FP64_TFLOPS = 78.6
KIND_FP64_FORCE, KIND_FP64_TORQUE, KIND_MIXED_FORCE, KIND_MIXED_TORQUE = 0, 1, 2, 3
KIND_BATCHED = 4
KIND_MULTI_FP64, KIND_MULTI_MIXED = 8, 10   # multi-vector kernel (pairs counted per vector)

PROFILED_N = 65536   # sheet size of the committed counter summaries


def sym_flops(nvec=1, torque=False):
    """Operations of the symmetric kernel per unordered pair for `nvec` source vectors."""
    return FLOP_SEP + FLOP_COEF + FLOP_APPLY * nvec + (FLOP_TORQUE_APPLY if torque else 0)


def alg_flops(sizes, symmetric, torque=False, nvec=1):
    """Algorithmic operations of one product over systems of the given sizes: the symmetric
    kernel evaluates N(N+1)/2 unordered pairs (self pairs included), the ordered one N^2."""
    if symmetric:
        return sum(n * (n + 1) / 2.0 for n in sizes) * sym_flops(nvec, torque)
    return sum(float(n) * n for n in sizes) * nvec * (FLOP_ORD_TORQUE if torque else FLOP_ORD_FORCE)


def kernel_source_hash() -> str:
    """sha256[:16] of the pair-kernel sources, comments and blank lines removed (the key of the
    committed counter summaries)."""
    from paper_1612_00474_amd.profile_summary import kernel_source_hash as h
    return h()


def counter_record(fname: str, kernel: str, n: int = PROFILED_N):
    """The per-launch figure recorded for `kernel` in the machine-readable block of a committed
    counter summary (tab-separated: kernel, value, source hash), or None when the pair-kernel
    sources changed since the counters were taken or `n` is another size."""
    if n != PROFILED_N:
        return None
    current = kernel_source_hash()
    try:
        with open(os.path.join(ROOT, "profiles", fname)) as f:
            for line in f:
                parts = line.rstrip("\n").split("\t")
                if len(parts) == 3 and parts[0] == kernel and parts[2] == current:
                    return float(parts[1])
    except OSError:
        pass
    return None


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
    ap.add_argument("--no-extra", action="store_true",
                    help="headline workload only (no batched / float64 sub-benchmarks)")
    ap.add_argument("--cpu-rows", type=int, default=24, help="C3 sample rows per CPU worker")
    ap.add_argument("--steps-only", action="store_true",
                    help="time the steps only (no product, multi-vector or periodic rates): "
                         "for kernel traces of the step")
    return ap.parse_args()


# ---- CPU oracle baseline -------------------------------------------------------------------

def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_workers():
    """Host cores this process may use, at most 16 (one GPU's share of a box)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_baseline(w, rows_per_worker):
    """The FP64 oracle, as it stands, on the host's cores (a pool of forked workers, each taking
    a block of target rows against all sources):
      - the headline workload's product M F + M_C T on a bounded sample of target rows;
      - the 16,384-sphere float64 sheet's product on a sample of rows, with its product and
        step times extrapolated from that rate (labelled);
      - one whole oracle step of the 256-sphere case (dense matrices, Lanczos at 1e-6, centred
        RFD), measured."""
    import numpy as np
    from oracle import integrator, mobility
    from paper_1612_00474_amd import workloads as wl
    workers = cpu_workers()
    out = {"unit": "pair-interactions/s", "cores": workers, "cpu_model": cpu_model(),
           "kind": "oracle"}

    def sample(inp, n, rows):
        sel = np.arange(rows)
        t0 = time.perf_counter()
        mobility.matvec(inp["pos"], inp["force"], inp["torque"], rows=sel, workers=workers)
        dt = time.perf_counter() - t0
        return rows * n / dt, dt

    if w.nsys > 1:
        pos_b, offs = wl.make_batch(w, 0)
        n = int(offs[1])
        rng = np.random.default_rng(0)
        inp = {"pos": pos_b[:n], "force": rng.standard_normal((n, 3)),
               "torque": rng.standard_normal((n, 3))}
        what = f"system 0 of the batch (N = {n})"
    else:
        inp, n = wl.make_inputs(w, 0), w.n
        what = f"all {n} sources"
    mobility.matvec(inp["pos"][:64], inp["force"][:64], inp["torque"][:64])   # compile tensors
    rows = min(n, rows_per_worker * workers)
    rate, dt = sample(inp, n, rows)
    out["value"] = rate
    out["sample"] = (f"{rows} target rows x {what}, one product M F + M_C T ({rows * n:.3e} "
                     f"pairs, {dt:.1f} s on {workers} worker processes)")

    c2 = wl.WORKLOADS["sheet16k_fp64"]
    inp2 = wl.make_inputs(c2, 0)
    rate2, dt2 = sample(inp2, c2.n, min(c2.n, 16 * workers))
    t_product = float(c2.n) * c2.n / rate2
    out["sheet16k_fp64"] = {
        "pairs_per_s": rate2, "sample_rows": min(c2.n, 16 * workers), "sample_s": dt2,
        "product_s_extrapolated": t_product,
        # a step takes 1 + m + 2 products; m = 11 at tolerance 1e-3 on this sheet (GPU runs)
        "steps_per_s_extrapolated": 1.0 / ((1 + 11 + 2) * t_product),
        "note": "extrapolated from the sampled product rate: (1 + m + 2) products per step at "
                "m = 11, O(N) work left out; not timed"}

    c1 = wl.WORKLOADS["sheet256_rsa"]
    inp1 = wl.make_inputs(c1, 0)
    t0 = time.perf_counter()
    _, _, m1, _, _ = integrator.step(inp1["pos"], None, inp1["w"], inp1["w_tilde"], dt=c1.dt,
                                     delta=c1.delta, lanczos_tol=c1.lanczos_tol)
    t1 = time.perf_counter() - t0
    out["sheet256_step"] = {"n": c1.n, "s_per_step": t1, "steps_per_s": 1.0 / t1,
                            "lanczos_iters": int(m1), "lanczos_tol": c1.lanczos_tol,
                            "note": "one whole oracle step, measured (single process: dense "
                                    "matrices and numpy products)"}
    return out


# ---- GPU pieces --------------------------------------------------------------------------

def read_kinds(ctx, shape_sym, sizes):
    """Per-kernel-variant timing records since the last read (alg = algorithmic TFLOP/s of the
    kernel as launched; logical = every ordered pair charged in full)."""
    kinds = {}
    for name, kind, torque, mixed in (("fp64_force", KIND_FP64_FORCE, False, False),
                                      ("fp64_torque", KIND_FP64_TORQUE, True, False),
                                      ("mixed_force", KIND_MIXED_FORCE, False, True),
                                      ("mixed_torque", KIND_MIXED_TORQUE, True, True)):
        ms, k, pairs = ctx.timing_read(kind)
        if k:
            s = shape_sym["mixed" if mixed else "fp64"]
            t = ms * 1e-3
            kinds[name] = {"launches": k, "ms_per_launch": ms / k, "pairs_per_s": pairs / t,
                           "tflops_alg": k * alg_flops(sizes, s, torque) / t / 1e12,
                           "tflops_logical": (FLOP_ORD_TORQUE if torque else FLOP_ORD_FORCE)
                           * pairs / t / 1e12}
    # the two-vector launch of each step: M F + M_C T together with the first Lanczos product
    for name, kind in (("fp64_two_vector", KIND_MULTI_FP64), ("mixed_two_vector", KIND_MULTI_MIXED)):
        ms, k, pairs = ctx.timing_read(kind)
        if k:
            t = ms * 1e-3
            kinds[name] = {"launches": k, "ms_per_launch": ms / k,
                           "vector_pairs_per_s": pairs / t,
                           "tflops_alg": k * alg_flops(sizes, True, True, 2) / t / 1e12}
    return kinds


def run_single_steps(ctx, w, pos0, steps, warmup, prec, timing=True):
    """`warmup` + `steps` SAB steps of one system; returns the timed figures.  With `timing`
    the pair kernels of the timed steps are bracketed by events (read back by read_kinds),
    which costs small systems some of their step rate."""
    import torch
    from paper_1612_00474_amd import StepState
    step_kw = dict(dt=w.dt, delta=w.delta, lanczos_tol=w.lanczos_tol, lanczos_max_iter=64,
                   rfd_precision="fp64", f_grav_z=w.f_grav_z, torque=w.torque,
                   steric_u0=w.steric_u0, steric_b=w.steric_b, seed=0, precision=prec)
    state = StepState(pos0.clone())
    iters = []
    for _ in range(warmup):
        iters.append(ctx.sab_step(state, **step_kw)[0])
    torch.cuda.synchronize()
    ctx.timing(timing)
    ctx.timing_read()
    with ClockSampler() as clocks:
        t0 = time.perf_counter()
        for _ in range(steps):
            iters.append(ctx.sab_step(state, **step_kw)[0])
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
    return elapsed, iters[warmup:], clocks.summary()


def run_batched(ctx, w, steps, warmup):
    """Batched suspensions: one persistent launch per product, steps replayed from a hipGraph.
    Returns a dict of figures (and the timed step work for the caller's `value`)."""
    import numpy as np
    import torch
    from paper_1612_00474_amd import workloads as wl

    pos_np, offs = wl.make_batch(w, 0)
    sizes = [int(x) for x in np.diff(offs)]
    n = int(offs[-1])
    sum_sq = float(np.sum(np.asarray(sizes, dtype=np.float64) ** 2))
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
        t = ms * 1e-3
        sym = bool(shapes[precision]["batch_symmetric"])
        return {"pairs_per_s": pairs / t, "ms_per_launch": ms / k,
                "tflops_alg": k * alg_flops(sizes, sym) / t / 1e12,
                "tflops_logical": FLOP_ORD_FORCE * pairs / t / 1e12}

    rates = {"mixed": kernel_rate("mixed"), "fp64": kernel_rate("fp64")}
    budget = 16
    kw = dict(dt=w.dt, delta=w.delta, lanczos_tol=w.lanczos_tol, lanczos_max_iter=budget,
              rfd_precision="fp64", f_grav_z=w.f_grav_z, torque=w.torque, steric_u0=w.steric_u0,
              steric_b=w.steric_b, seed=0, precision=w.precision)
    P = pos0.clone()
    U = torch.zeros_like(P)
    graph = ctx.step_graph(P, U, offs, 0, False, **kw)
    for _ in range(warmup):
        graph.launch()
    torch.cuda.synchronize()
    with ClockSampler() as clocks:
        t0 = time.perf_counter()
        for _ in range(steps):
            graph.launch()
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
    _, iters, _, _ = graph.status()
    graph.close()
    # eager batched steps (host reads the Lanczos flags every iteration) for comparison
    Pe = pos0.clone()
    Ue = torch.zeros_like(Pe)
    ctx.sab_step_batched(Pe, Ue, offs, 0, False, **kw)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for k in range(steps):
        ctx.sab_step_batched(Pe, Ue, offs, k + 1, True, **kw)
    torch.cuda.synchronize()
    eager = time.perf_counter() - t1
    pairs_step = float(np.sum(np.asarray(sizes, dtype=np.float64) ** 2 * (3 + iters)))
    dom = rates["mixed" if w.precision == "mixed" else "fp64"]
    peak = PEAK_FP32_TFLOPS if w.precision == "mixed" else PEAK_FP64_TFLOPS
    return {
        "workload": w.name, "nsys": int(w.nsys), "n_total": n, "sum_n_squared": sum_sq,
        "sizes": sizes, "precision": w.precision, "steps": steps, "warmup": warmup,
        "graph": "one hipGraph launch per step", "lanczos_budget": budget,
        "steps_per_s": steps / elapsed, "ms_per_step": 1e3 * elapsed / steps,
        "eager_steps_per_s": steps / eager,
        "pairs_per_s": pairs_step * steps / elapsed,
        "lanczos_iters_last_step": {"min": int(iters.min()), "median": float(np.median(iters)),
                                    "max": int(iters.max())},
        "launch_shapes": shapes, "batched_kernel": rates, "gpu_clock": clocks.summary(),
        "roofline": {"bound": "alu", "achieved": dom["tflops_alg"], "peak": peak,
                     "unit": "TFLOP/s", "frac": dom["tflops_alg"] / peak,
                     "kernel": "batched pair kernel, force-only",
                     "ms_per_launch": dom["ms_per_launch"],
                     "frac_logical": dom["tflops_logical"] / peak},
        "_elapsed": elapsed, "_pairs_step": pairs_step,
    }


def run_graph_steps(ctx, w, pos0, steps, warmup, budget):
    """The same single-system step captured in a hipGraph (the batched step with one system:
    device-side Lanczos stop, `budget` iterations enqueued, no host synchronisation)."""
    import numpy as np
    import torch
    kw = dict(dt=w.dt, delta=w.delta, lanczos_tol=w.lanczos_tol, lanczos_max_iter=budget,
              rfd_precision="fp64", f_grav_z=w.f_grav_z, torque=w.torque,
              steric_u0=w.steric_u0, steric_b=w.steric_b, seed=0, precision=w.precision)
    P = pos0.clone()
    U = torch.zeros_like(P)
    graph = ctx.step_graph(P, U, np.array([0, w.n], dtype=np.int64), 0, False, **kw)
    for _ in range(warmup):
        graph.launch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        graph.launch()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    _, iters, _, _ = graph.status()
    graph.close()
    return {"steps_per_s": steps / elapsed, "ms_per_step": 1e3 * elapsed / steps,
            "lanczos_budget": budget, "lanczos_iters_last_step": int(iters[0])}


def run_fp64_sheet(ctx_cls, name, steps, warmup, budget):
    """Float64 steps of one sheet (its own context and tuned shape): eager single-system steps
    (the host reads each Lanczos status) and the graph-captured step."""
    import torch
    from paper_1612_00474_amd import workloads as wl
    w = wl.WORKLOADS[name]
    inp = wl.make_inputs(w, 0)
    pos0 = torch.as_tensor(inp["pos"]).cuda()
    ctx = ctx_cls(0, a=w.a, eta=w.eta, kT=w.kT)
    shape = ctx.autotune(pos0, None, "fp64")[0]
    elapsed, iters, clocks = run_single_steps(ctx, w, pos0, steps, warmup, "fp64", timing=False)
    # the pair-kernel figures from a few more steps with the kernels bracketed by events
    run_single_steps(ctx, w, pos0, max(3, steps // 5), 0, "fp64", timing=True)
    kinds = read_kinds(ctx, {"fp64": bool(shape["symmetric"]), "mixed": True}, [w.n])
    ctx.timing(False)
    graph = run_graph_steps(ctx, w, pos0, steps, warmup, budget)
    ctx.close()
    dom = kinds.get("fp64_force")
    products = sum(1 + m + 2 for m in iters)
    return {"workload": w.name, "n": w.n, "precision": "fp64", "lanczos_tol": w.lanczos_tol,
            "steps": steps, "warmup": warmup,
            "steps_per_s": steps / elapsed, "ms_per_step": 1e3 * elapsed / steps,
            "pairs_per_s": products * float(w.n) ** 2 / elapsed, "lanczos_iters": iters,
            "graph": graph, "launch_shape": shape, "pair_kernels": kinds, "gpu_clock": clocks,
            "roofline": None if dom is None else {
                "bound": "alu", "achieved": dom["tflops_alg"], "peak": PEAK_FP64_TFLOPS,
                "unit": "TFLOP/s", "frac": dom["tflops_alg"] / PEAK_FP64_TFLOPS,
                "kernel": force_kernel_name("fp64", shape) + ", force-only products",
                "ms_per_launch": dom["ms_per_launch"]}}


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
        cpu = cpu_baseline(w, args.cpu_rows)   # before the GPU is touched (the pool forks)

    import numpy as np
    import torch
    from paper_1612_00474_amd import Context

    torch.cuda.init()
    ctx = Context(0, a=w.a, eta=w.eta, kT=w.kT)
    if w.nsys > 1:
        return bench_batched(args, w, ctx, cpu)
    inp = wl.make_inputs(w, 0)
    pos0 = torch.as_tensor(inp["pos"]).cuda()
    F = torch.as_tensor(inp["force"]).cuda()
    T = torch.as_tensor(inp["torque"]).cuda()
    prec = w.precision
    n = w.n

    # ---- launch shapes from the tuner (timed on this configuration, cached per size) -------
    shapes = {prec_: ctx.autotune(pos0, None, prec_)[0] for prec_ in ("mixed", "fp64")}
    sym = {p_: bool(s["symmetric"]) for p_, s in shapes.items()}

    if args.steps_only:
        elapsed, timed_iters, clock = run_single_steps(ctx, w, pos0, args.steps, args.warmup, prec,
                                                       timing=False)
        ctx.close()
        print(json.dumps({"workload": w.name, "steps": args.steps, "warmup": args.warmup,
                          "ms_per_step": 1e3 * elapsed / args.steps,
                          "steps_per_s": args.steps / elapsed, "lanczos_iters": timed_iters,
                          "launch_shapes": shapes, "gpu_clock": clock}))
        return

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
        t = ms * 1e-3
        return {"pairs_per_s": pairs / t, "ms_per_launch": ms / launches,
                "tflops_alg": launches * alg_flops([n], sym[precision], True) / t / 1e12}

    mv = {"mixed": kernel_rate("mixed"), "fp64": kernel_rate("fp64")}

    # ---- multi-vector product: four force vectors of this configuration per launch -------
    FF = torch.as_tensor(np.random.default_rng(7).standard_normal((4, n, 3))).cuda()

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
                "tflops_alg": launches * alg_flops([n], True, False, 4) / (ms * 1e-3) / 1e12,
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
        return {"ms_per_launch": ms / launches, "image_pairs_per_s": 9.0 * pairs / (ms * 1e-3)}

    periodic = {"box": [w.side, w.side], "images_per_pair": 9, "force_only": True,
                "mixed": periodic_rate("mixed"), "fp64": periodic_rate("fp64")}
    pctx.close()

    # ---- time steps ----------------------------------------------------------------------
    elapsed, timed_iters, clock = run_single_steps(ctx, w, pos0, args.steps, args.warmup, prec)
    kinds = read_kinds(ctx, sym, [n])
    ctx.timing(False)
    products = sum(1 + m + 2 for m in timed_iters)
    step_pairs = products * float(n) * n
    value = step_pairs / elapsed

    if cpu is not None:
        # the oracle's step rate at this size, extrapolated from its sampled product rate at the
        # Lanczos counts of the timed steps (products only; the O(N) work is left out)
        cpu["steps_per_s_extrapolated"] = cpu["value"] * len(timed_iters) / step_pairs
        cpu["steps_per_s_note"] = ("extrapolated: rate / ((1 + m + 2) N^2) at the GPU "
                                   "steps' Lanczos m, not timed")

    # dominant kernel: the pair kernel of the Lanczos products (most launches and most time)
    dom = kinds["mixed_force" if prec == "mixed" else "fp64_force"]
    peak = PEAK_FP32_TFLOPS if prec == "mixed" else PEAK_FP64_TFLOPS
    kname = force_kernel_name(prec, shapes[prec])
    issued = counter_record("pair_kernels_sheet64k_valu_counters.md", kname, n)
    issued_tflops = None if issued is None else issued / (dom["ms_per_launch"] * 1e-3) / 1e12
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
        "matvec_kernel_pairs_per_s": {"mixed": mv["mixed"]["pairs_per_s"],
                                      "fp64": mv["fp64"]["pairs_per_s"],
                                      "mixed_over_fp64": mv["mixed"]["pairs_per_s"]
                                      / mv["fp64"]["pairs_per_s"],
                                      "ms_per_launch": {"mixed": mv["mixed"]["ms_per_launch"],
                                                        "fp64": mv["fp64"]["ms_per_launch"]},
                                      "tflops_alg": {"mixed": mv["mixed"]["tflops_alg"],
                                                     "fp64": mv["fp64"]["tflops_alg"]}},
        "roofline": {
            "bound": "alu", "achieved": dom["tflops_alg"], "peak": peak, "unit": "TFLOP/s",
            "frac": dom["tflops_alg"] / peak,
            "traffic": counter_record("pair_kernels_sheet64k_hbm_traffic.md", kname, n),
            "kernel": f"{kname}, force-only products",
            "work": (f"{FLOP_SYM_FORCE} flop per unordered pair x N(N+1)/2 pairs per launch "
                     "(each pair's coefficients once, the force applied in both directions)"
                     if sym[prec] else f"{FLOP_ORD_FORCE} flop per ordered pair x N^2"),
            "ms_per_launch": dom["ms_per_launch"], "launches": dom["launches"],
            "logical": {"flop_per_ordered_pair": FLOP_ORD_FORCE, "achieved": dom["tflops_logical"],
                        "frac": dom["tflops_logical"] / peak,
                        "note": "every ordered pair charged the closed form in full; not "
                                "arithmetic the symmetric kernel performs"},
            "issued_frac": None if issued_tflops is None else issued_tflops / peak,
            "issued": None if issued is None else {
                "flop_per_launch": issued, "achieved": issued_tflops,
                "source": "profiles/pair_kernels_sheet64k_valu_counters.md (FMA = 2; MUL, ADD, "
                          "transcendental = 1; Kahan compensation and hi/lo reconstruction "
                          "included)"},
        },
        "pair_kernels": kinds,
        "multi_vector_product": multi,
        "periodic_product": periodic,
        "gpu_clock": clock,
    }
    ctx.close()
    if not args.no_extra:
        bw = wl.WORKLOADS["batch64_uneven_mixed"]
        bctx = Context(0, a=bw.a, eta=bw.eta, kT=bw.kT)
        b = run_batched(bctx, bw, max(args.steps, 10), args.warmup)
        bctx.close()
        b.pop("_elapsed")
        b.pop("_pairs_step")
        b.pop("sizes")
        line["batched"] = b
        line["fp64_sheet16k"] = run_fp64_sheet(Context, "sheet16k_fp64", max(args.steps, 10),
                                               args.warmup, 16)
        line["fp64_sheet256"] = run_fp64_sheet(Context, "sheet256_rsa", 50, 5, 32)
    line["cpu_baseline"] = cpu
    print(json.dumps(line))


def bench_batched(args, w, ctx, cpu):
    """--workload batch64_uneven(_mixed): the batched figures as the main line."""
    b = run_batched(ctx, w, args.steps, args.warmup)
    ctx.close()
    elapsed, pairs_step = b.pop("_elapsed"), b.pop("_pairs_step")
    line = {
        "metric": "RPB matvec pair-interactions/s + BD steps/s, batched suspensions",
        "value": pairs_step * args.steps / elapsed,
        "unit": "pair-interactions/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "steps_per_s": args.steps / elapsed,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if w.precision == "mixed" else "f64", "data": "synthetic",
        "config": {"workload": w.name, "nsys": int(w.nsys), "n_total": b["n_total"],
                   "sizes": b.pop("sizes"), "sum_n_squared": b["sum_n_squared"],
                   "precision": w.precision, "rfd_precision": "fp64",
                   "lanczos_tol": w.lanczos_tol, "lanczos_budget": b["lanczos_budget"],
                   "graph": "one hipGraph launch per step", "parallelism": "single GPU"},
        "roofline": b.pop("roofline"),
        "batched": b,
        "cpu_baseline": cpu,
    }
    line["roofline"]["traffic"] = None
    print(json.dumps(line))


if __name__ == "__main__":
    main()
