"""Benchmark: TT-roundings per second on one MI355X.

Workload: one TT-round of the sum of 20 random rank-10 TTs (order 8, mode
size 32, term j with every core scaled by 2**-j, input rank 200), at
delta = 1e-4 in FP32-bulk (headline value) and in FP64, plus FP64 at
delta = 1e-8.  Inputs are synthetic (seeded) and resident in HBM before the
timed region.  A step is one rounding; the timed region runs --steps of them
back to back on one stream, bracketed by device synchronisation.

Only results that meet the metric's condition count: after timing, the
relative error ||x - x~|| / ||x|| of the last result (computed on the GPU by
the library: the norm of the lazy sum x - x~) must be <= delta.

The roofline object describes the kernel with the largest share of device
time, measured with HIP events on the library's streams in a separate pass of
further roundings right after the timed region (the timed region runs with
the profiler off); its achieved rate is the algorithmic flops of its launches
divided by their summed duration.

Further lines: FP64 at 1e-4 and 1e-8 and FP32-bulk at 1e-8 (reported with the
accuracy it reaches, delta_eff), 256 uneven jobs in one batch, the 20-vector
MGS workload (LOO and kappa per step), CGS2 and TT-Gram on 50 order-6 vectors
under a rank guard, a serving sweep over offered request rates, TT-Householder,
the Section 4 experiment and randomized rounding.  The CPU legs time the FP64
oracle on bounded samples of the same workloads (all BLAS threads and one; a
process pool for the batch) and check the headline result and sampled serving
requests against it.
"""
from __future__ import annotations

import argparse
import ctypes as C
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {  # MI355X published peaks, TFLOP/s
    "fp64_vector": 78.6, "fp64_mfma": 78.6, "fp32_vector": 157.3, "fp32_mfma": 157.3,
}
KINDS = ["qr_factor_leaf", "qr_factor_node", "qr_apply", "svd_jacobi", "contraction_gemm", "tt_dot", "other"]


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    p.add_argument("--cpu-seconds", type=float, default=12.0)
    p.add_argument("--serving-requests", type=int, default=80, help="requests per offered-rate point of the serving sweep")
    p.add_argument("--order6-n64-all", action="store_true", help="CGS2 and Gram at all three deltas of the 50-vector order-6, n=64 workload")
    p.add_argument("--copy-calibration", action="store_true",
                   help="only run a plain 256 MiB device-to-device copy (reference for the HBM byte counters)")
    p.add_argument("--headline-only", action="store_true",
                   help="time only the headline configuration (for profiler runs); no FP64 side runs, no CPU baseline")
    p.add_argument("--householder-only", action="store_true",
                   help="only the TT-Householder measurement (for profiler runs); prints its JSON object")
    p.add_argument("--batched-only", action="store_true",
                   help="only the 256-job uneven batch (for profiler runs); prints its JSON object")
    p.add_argument("--randomized-only", action="store_true",
                   help="only the randomized-rounding measurement (for profiler runs); prints its JSON object")
    p.add_argument("--serving-only", action="store_true",
                   help="only the serving sweep (for profiler runs); prints its JSON object")
    p.add_argument("--order6-only", action="store_true",
                   help="only the order-6 experiment of the paper's workload (for profiler runs); prints its JSON object")
    p.add_argument("--order6-n64-guard", type=int, default=0,
                   help="with --order6-n64-only: the pre-round rank guard (default 1024; above it each non-Gram q "
                        "output is capped at 128M elements, 1 GB in FP64)")
    p.add_argument("--order6-complete", action="store_true",
                   help="only the order-6 experiment with every scheme run to m = 35 (several minutes)")
    p.add_argument("--order6-n64-only", action="store_true",
                   help="only the CGS2/Gram runs of the order-6, n=64 workload (for profiler runs); prints its JSON object")
    p.add_argument("--serving-qps", type=str, default="",
                   help="comma-separated offered rates of the serving sweep (default 3,6,9,15)")
    return p.parse_args()


def recorded_traffic(kernel, workload="graded_sum_r200"):
    """HBM bytes per launch of `kernel` on `workload` from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None when there is none or the QR source changed
    since it was taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path).read().splitlines():
        if ": " in line:
            k, v = line.split(": ", 1)
            kv[k.strip()] = v.strip()
    with open(os.path.join(ROOT, "paper_2211_08770_amd", "csrc", "qr.hip"), "rb") as f:
        src = hashlib.sha256(f.read()).hexdigest()[:16]
    if kv.get("kernel") != kernel or kv.get("source_sha256_prefix") != src:
        return None
    return int(kv["traffic_bytes_per_launch"])


def roofline_of(prof, bulk_fp32=True):
    """Roofline object of the kernel kind with the largest device time in a library profile: its
    algorithmic flops over its summed launch durations, against the MFMA peak of its precision."""
    name, p = max(prof.items(), key=lambda kv: kv[1]["ms"])
    achieved = p["flops"] / (p["ms"] * 1e-3) / 1e12 if p["ms"] > 0 else 0.0
    # FP32-bulk leaves are factored and applied on the FP32 MFMA (157.3 TF/s) and the component GEMMs
    # run there too; tree nodes are FP64 (78.6 TF/s) and the TT dots use the FP64 MFMA for either
    # dtype.  The apply kind mixes leaf and node tiles: it is priced at the FP32 peak, so its fraction
    # is a lower bound.  An FP64 workload runs every kind on the FP64 units.  The Jacobi SVD runs on
    # the vector ALU ("alu", FP64).
    alu = name in ("svd_jacobi", "other")
    if alu:
        peak = PEAK["fp64_vector"]
    else:
        fp32_kinds = ("qr_factor_leaf", "qr_apply", "contraction_gemm") if bulk_fp32 else ()
        peak = PEAK["fp32_mfma"] if name in fp32_kinds else PEAK["fp64_mfma"]
    return {"bound": "alu" if alu else "mfma", "achieved": round(achieved, 4), "peak": peak, "unit": "TFLOP/s",
            "frac": round(achieved / peak, 5), "traffic": None, "kernel": name,
            "avg_launch_ms": round(p["ms"] / max(p["launches"], 1), 5), "launches": p["launches"],
            "share_of_kernel_time": round(p["ms"] / sum(v["ms"] for v in prof.values()), 4)}


def profile_arrays(ctx):
    lib = ctx.lib
    lib.tt_ctx_profile.argtypes = [C.c_void_p, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_int64),
                                   C.POINTER(C.c_double), C.POINTER(C.c_double)]
    out = {}
    for k, name in enumerate(KINDS):
        ms, n, fl, by = C.c_double(), C.c_int64(), C.c_double(), C.c_double()
        lib.tt_ctx_profile(ctx.h, k, C.byref(ms), C.byref(n), C.byref(fl), C.byref(by))
        out[name] = {"ms": ms.value, "launches": n.value, "flops": fl.value, "bytes": by.value}
    return out


def run_config(tt, torch, dtype, delta, steps, warmup, profile_steps=0):
    """Time `steps` roundings of the graded sum (profiler off); then, when profile_steps > 0,
    run that many more with the library's per-launch HIP-event profiler on (not timed) for
    the per-kernel breakdown and the roofline object."""
    import numpy as np
    from paper_2211_08770_amd import synth
    npdt = np.float32 if dtype == torch.float32 else np.float64
    terms = synth.sum_of_graded_terms(dtype=npdt)
    x = [(a, tt.TT.from_cores(c, device="cuda", dtype=dtype)) for a, c in terms]
    ctx = tt._ctx()
    ctx.lib.tt_ctx_set_profiling.argtypes = [C.c_void_p, C.c_int]
    for _ in range(warmup):
        out = tt.round(x, delta)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        out = tt.round(x, delta)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = None
    if profile_steps > 0:
        ctx.lib.tt_ctx_set_profiling(ctx.h, 1)
        for _ in range(profile_steps):
            tt.round(x, delta)
        torch.cuda.synchronize()
        prof = profile_arrays(ctx)
        ctx.lib.tt_ctx_set_profiling(ctx.h, 0)
    # validity: ||x - x~|| / ||x|| on the GPU (norms of lazy sums by the right-to-left sweep)
    nx = tt.norm(x)
    nd = tt.norm(x + [(-1.0, out)])
    return {"rate": steps / dt, "ms": 1e3 * dt / steps, "ranks": out.r, "rel_err": nd / nx, "prof": prof,
            "delta_eff": tt.effective_delta(x, delta), "out": out, "profile_steps": profile_steps}


def run_batched(tt, torch, reps=3):
    """256 independent uneven roundings (orders 4-10, modes 16/32/64, ranks 8-128, FP32, delta 1e-5)
    in shared batched launches; value in roundings/s; validity: output ranks equal the caps and a
    sample of errors ||x - x~|| / ||x|| <= delta."""
    from paper_2211_08770_amd import synth
    jobs = synth.uneven_jobs()
    xs = [tt.TT.from_cores(c, device="cuda", dtype=torch.float32) for c, _ in jobs]
    tt.set_autotune(True)
    outs = tt.round_batched(xs, 1e-5)
    tt.set_autotune(False)
    # a one-element fill before and after the timed batches marks their window in a kernel trace
    # (the tuning launches above come before it)
    torch.full((1,), 2.5, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        outs = tt.round_batched(xs, 1e-5)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    torch.full((1,), 2.5, dtype=torch.float64, device="cuda")
    caps_ok = all(o.r == [1] + [min(R, n ** k, n ** (d - k)) for k in range(1, d)] + [1]
                  for o, (_, (d, n, R)) in zip(outs, jobs))
    errs = [tt.norm([(1.0, xs[i]), (-1.0, outs[i])]) / tt.norm(xs[i]) for i in range(0, len(xs), 16)]
    # one more batch with the library profiler on (not part of the rate): the dominant kernel kind
    # when many jobs share each launch
    ctx = tt._ctx()
    ctx.lib.tt_ctx_set_profiling.argtypes = [C.c_void_p, C.c_int]
    ctx.lib.tt_ctx_set_profiling(ctx.h, 1)
    tt.round_batched(xs, 1e-5)
    torch.cuda.synchronize()
    prof = profile_arrays(ctx)
    ctx.lib.tt_ctx_set_profiling(ctx.h, 0)
    roof = roofline_of(prof)
    roof["traffic"] = recorded_traffic(roof["kernel"], "batched_uneven_256")
    # the same batch planned at the rank bounds (tt_round_batched_async: no host synchronisation
    # before the final read-back); its ranks equal the bounds here, so the results are bitwise equal
    bnd = tt.round_batched(xs, 1e-5, plan="bounds")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        bnd = tt.round_batched(xs, 1e-5, plan="bounds")
    torch.cuda.synchronize()
    dtb = (time.perf_counter() - t0) / reps
    same = all(a.r == b.r and torch.equal(a.data, b.data) for a, b in zip(outs, bnd))
    # the same call captured once as a HIP graph and replayed (fixed buffers: a solver loop)
    br = tt.BatchRounder(xs, 1e-5)
    br.run()
    gres = br.results()
    t0 = time.perf_counter()
    for _ in range(reps):
        br.run()
    br.stream.synchronize()
    dtg = (time.perf_counter() - t0) / reps
    gres = br.results()
    same_graph = br.graph_count() == 1 and all(a.r == b.r and torch.equal(a.data, b.data)
                                               for a, b in zip(outs, gres))
    return {"value": round(len(xs) / dtg, 2), "unit": "TT-roundings/s", "jobs": len(xs),
            "ms_per_batch": round(1e3 * dtg, 3),
            "planning": "every left-to-right step planned at the rank bounds, cores compacted on the device, the "
                        "call captured once as a HIP graph and replayed on the same buffers (tt_ctx_set_graphs, "
                        "tt_round_batched_async)",
            "bound_planning_without_graph": {"value": round(len(xs) / dtb, 2), "ms_per_batch": round(1e3 * dtb, 3)},
            "host_planning": {"value": round(len(xs) / dt, 2), "ms_per_batch": round(1e3 * dt, 3),
                              "note": "tt_round_batched: the rank of every left-to-right step read back to plan the "
                                      "next; bitwise the same results"},
            "bitwise_equal_to_host_planning": same,
            "graph_replay": {"value": round(len(xs) / dtg, 2), "ms_per_batch": round(1e3 * dtg, 3),
                             "bitwise_equal_to_host_planning": same_graph,
                             "note": "the bound-planned call captured once as a HIP graph (tt_ctx_set_graphs) and "
                                     "replayed on the same buffers; no host planning per batch"},
            "roofline": roof,
            "roofline_note": "kernel kinds from one host-planned batch with the library profiler on (the same kernels)",
            "ranks_equal_caps": caps_ok, "max_sampled_rel_err": max(errs),
            "workload": "256 uneven jobs: d~U{4..10}, n~U{16,32,64}, rank~U{8..128}, N(0,1) FP32 cores, delta=1e-5"}


def blas_cores():
    try:
        from threadpoolctl import threadpool_info
        return int(max([i.get("num_threads", 1) for i in threadpool_info()] + [1]))
    except Exception:
        return os.cpu_count() or 1


def timed_loop(fn, seconds):
    """Run fn() until `seconds` have passed (at least once); returns (calls, elapsed s)."""
    n = 0
    t0 = time.perf_counter()
    while True:
        fn()
        n += 1
        if time.perf_counter() - t0 >= seconds:
            break
    return n, time.perf_counter() - t0


def at_threads(threads, fn):
    """fn() with the BLAS thread pools limited to `threads` (None: as configured)."""
    if threads is None:
        return fn()
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=threads):
        return fn()


def conditioned_dev(tt, torch, seed, m, d, n, r, kappa, dtype):
    """x_k = sum_{j<=k} c_kj t_j (private copies) with cond(Gram(x)) = kappa; the Gram matrix of
    the generators that fixes the c_kj is taken on the GPU (the oracle is not used here)."""
    import numpy as np
    from paper_2211_08770_amd import synth
    npdt = np.float32 if dtype == torch.float32 else np.float64
    t = synth.conditioned_terms(seed, m, d, n, r, dtype=npdt)
    dev = [tt.TT.from_cores(c, device="cuda", dtype=dtype) for c in t]
    Gt = tt.dot_batched([(dev[i], dev[j]) for i in range(m) for j in range(m)]).reshape(m, m)
    cm, M = synth.mixing_coefficients(0.5 * (Gt + Gt.T), seed, kappa)
    A = [[(float(cm[k, j]), tt.TT.from_cores(t[j], device="cuda", dtype=dtype)) for j in range(k + 1)]
         for k in range(m)]
    return A, t, cm, M


def oracle_conditioned(seed, m, d, n, r, kappa):
    """The same inputs built on the host with the oracle's Gram matrix of the generators."""
    import oracle
    from paper_2211_08770_amd import synth
    t = synth.conditioned_terms(seed, m, d, n, r)
    cm, M = synth.mixing_coefficients(oracle.gram_of(t), seed, kappa)
    return [[(float(cm[k, j]), [c.copy() for c in t[j]]) for j in range(k + 1)] for k in range(m)], M


MGS20 = dict(seed=10000, m=20, d=4, n=8, r=3, kappa=1e6, delta=1e-6)
MGS20_DESC = ("TT-MGS (Algorithm 2) of m=20 TT-vectors x_k = sum_{j<=k} c_kj t_j (private copies), t_j random rank-3 "
           "TTs of order 4, n=8, cond(Gram(x)) = 1e6, delta=1e-6, FP64")


def run_mgs_m20_order4(tt, torch, reps=5):
    """The 20-vector MGS workload: per-step LOO, kappa(A_k) (tt_cond), pre/post ranks, time per call."""
    w = MGS20
    A, _, _, M = conditioned_dev(tt, torch, w["seed"], w["m"], w["d"], w["n"], w["r"], w["kappa"], torch.float64)
    Q, R, loo, st = tt.orthogonalize("mgs", A, w["delta"])
    kap, _ = tt.cond(A)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        tt.orthogonalize("mgs", A, w["delta"], with_loo=False)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    return {"ms_per_call": round(1e3 * dt, 3), "rounds": st["rounds"], "loo": [float(v) for v in loo],
            "kappa": [float(v) for v in kap], "max_pre_rank": st["max_pre_rank"],
            "max_post_rank": st["max_post_rank"], "q_ranks": [max(q.r) for q in Q], "workload": MGS20_DESC}


def cpu_baseline_mgs_m20_order4(seconds=4.0):
    """The oracle's MGS on the same workload, end to end, at all BLAS threads and at one."""
    import oracle
    w = MGS20
    X, M = oracle_conditioned(w["seed"], w["m"], w["d"], w["n"], w["r"], w["kappa"])
    out = {}
    for label, th in (("all", None), ("1", 1)):
        n, dt = at_threads(th, lambda: timed_loop(lambda: oracle.mgs(X, w["delta"]), seconds))
        out[label] = {"ms_per_call": round(1e3 * dt / n, 2), "cores": blas_cores() if th is None else 1}
    res = oracle.mgs(X, w["delta"])
    return {"ms_per_call": out, "kind": "oracle", "loo": [float(v) for v in oracle.loo_curve(res.Q)],
            "kappa": [float(v) for v in oracle.cond_curve(X)],
            "sample": f"FP64 NumPy/LAPACK MGS calls on the same workload (about {seconds:.0f} s per thread setting)"}


ORDER6_N64 = dict(seed=20000, m=50, d=6, n=64, r=8, kappa=1e10, guard=1024)
ORDER6_N64_DESC = ("CGS2 and TT-Gram on m=50 TT-vectors of order 6, n=64, generating ranks 8, cond(Gram(x)) = 1e10, FP64, "
           "under a pre-round rank guard of 1024 (prefix up to the guard)")


def run_cgs2_gram_m50_order6(tt, torch, runs=(("gram", 1e-3), ("gram", 1e-5), ("gram", 1e-7), ("cgs2", 1e-5)), reps=1,
                guard=None, profile=True):
    """CGS2 and Gram on the 50 order-6 vectors under the rank guard (by default Gram at
    delta 1e-3/1e-5/1e-7 and CGS2 at 1e-5; --order6-n64-all adds CGS2 at 1e-3 and 1e-7, whose
    guarded prefixes take several seconds per call): vectors reached, time per call and per
    step (profiler off), and the dominant kernel's roofline from a separate profiled call."""
    w = dict(ORDER6_N64)
    if guard:
        w["guard"] = int(guard)
    # above a guard of 1024 the q outputs sized for the rank bounds (up to the guard at every
    # middle bond) would exceed the GPU's memory: each q gets 128M elements (1 GB) instead
    # (TT-Gram's outputs past the guard are never formed and the binding sizes them so)
    qcap = (128 << 20) if w["guard"] > 1024 else None
    A, _, _, M = conditioned_dev(tt, torch, w["seed"], w["m"], w["d"], w["n"], w["r"], w["kappa"], torch.float64)
    ctx = tt._ctx()
    ctx.lib.tt_ctx_set_profiling.argtypes = [C.c_void_p, C.c_int]
    out = {}
    for sch, delta in runs:
        if True:
            # one timed call (the guarded prefixes take seconds: launch and allocation warm-up
            # are a small part), then one profiled call
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                Q, R, _, st = tt.orthogonalize(sch, A, delta, rank_guard=w["guard"], with_loo=False,
                                               partial_on_guard=True, q_capacity=None if sch == "gram" else qcap)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / reps
            prof = {}
            if profile:
                ctx.lib.tt_ctx_set_profiling(ctx.h, 1)
                tt.orthogonalize(sch, A, delta, rank_guard=w["guard"], with_loo=False, partial_on_guard=True,
                                 q_capacity=None if sch == "gram" else qcap)
                torch.cuda.synchronize()
                prof = profile_arrays(ctx)
                ctx.lib.tt_ctx_set_profiling(ctx.h, 0)
            k = st["m_reached"]
            loo = tt.loo(Q)[0] if k > 0 else []
            out[f"{sch}_{delta:.0e}"] = {
                "m_reached": k, "ms_per_call": round(1e3 * dt, 3), "ms_per_step": round(1e3 * dt / max(k, 1), 3),
                "rounds": st["rounds"], "max_pre_rank": st["max_pre_rank"], "max_post_rank": st["max_post_rank"],
                "loo_at_m_reached": float(loo[-1]) if k > 0 else None,
                "flops": sum(v["flops"] for v in prof.values()) if prof else None,
                "bytes": sum(v["bytes"] for v in prof.values()) if prof else None,
                "roofline": roofline_of(prof, bulk_fp32=False) if prof else None}
            if guard:
                progress(f"order-6 n=64 {sch} {delta:.0e} (m = {k} in {dt:.1f} s)")
    desc = ORDER6_N64_DESC if w["guard"] == ORDER6_N64["guard"] else ORDER6_N64_DESC.replace(f"guard of {ORDER6_N64['guard']}", f"guard of {w['guard']}")
    return {"workload": desc, "runs": out}


def cpu_baseline_cgs2_m50_order6(m_prefix=8, delta=1e-5):
    """The oracle's CGS2 on the first m_prefix vectors of the same workload: time per step."""
    import oracle
    w = ORDER6_N64
    X, M = oracle_conditioned(w["seed"], w["m"], w["d"], w["n"], w["r"], w["kappa"])
    t0 = time.perf_counter()
    res = oracle.cgs2(X[:m_prefix], delta)
    dt = time.perf_counter() - t0
    return {"ms_per_step": round(1e3 * dt / m_prefix, 2), "cores": blas_cores(), "kind": "oracle",
            "sample": f"FP64 NumPy/LAPACK CGS2 on the first {m_prefix} vectors at delta={delta:g} ({dt:.1f} s)",
            "max_pre_rank": max(max(r) for r in res.pre_ranks)}


_POOL_JOBS = None


def _pool_init(seed, count):
    global _POOL_JOBS
    import numpy as np
    from paper_2211_08770_amd import synth
    from threadpoolctl import threadpool_limits
    threadpool_limits(limits=1)
    jobs = synth.uneven_jobs(seed=seed, njobs=count)     # the first `count` jobs of the batch
    _POOL_JOBS = [[c.astype(np.float64) for c in j[0]] for j in jobs]


def _pool_round(i):
    import oracle
    oracle.tt_round(_POOL_JOBS[i % len(_POOL_JOBS)], 1e-5)
    return i


def cpu_baseline_batched(seconds=10.0, sample_jobs=32):
    """The oracle on the 256-job uneven workload in a process pool (one BLAS thread per worker,
    as many workers as host cores): roundings/s over a bounded run on the first jobs."""
    import concurrent.futures as cf
    import multiprocessing as mp
    workers = min(os.cpu_count() or 1, 16)
    ctx = mp.get_context("spawn")
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=ctx, initializer=_pool_init,
                                initargs=(30000, sample_jobs)) as ex:
        list(ex.map(_pool_round, range(workers)))          # start-up and inputs, not timed
        done = 0
        t0 = time.perf_counter()
        i = 0
        while time.perf_counter() - t0 < seconds:
            list(ex.map(_pool_round, range(i, i + 2 * workers)))
            i += 2 * workers
            done += 2 * workers
        dt = time.perf_counter() - t0
    return {"value": round(done / dt, 2), "unit": "TT-roundings/s", "cores": workers, "kind": "oracle",
            "sample": f"{done} FP64 NumPy/LAPACK roundings of the first {sample_jobs} jobs of the same batch, "
                      f"{workers} worker processes with one BLAS thread each ({dt:.1f} s)"}


HH_WORKLOAD = dict(seed=10000, m=20, d=4, n=8, r=3, kappa=1e6, delta=1e-6)
HH_DESC = ("TT-Householder of m=20 TT-vectors x_k = sum_{j<=k} c_kj t_j (private copies), t_j random rank-3 TTs "
           "of order 4, n=8, cond(Gram(x)) = 1e6, delta=1e-6, FP64")


def run_householder(tt, torch, reps=5):
    """TT-Householder (Algorithms 6-8) on the m=20 order-4 workload; value in orthogonalizations/s."""
    from paper_2211_08770_amd import synth
    w = HH_WORKLOAD
    t = synth.conditioned_terms(w["seed"], w["m"], w["d"], w["n"], w["r"])
    dev = [tt.TT.from_cores(c, device="cuda", dtype=torch.float64) for c in t]
    m = w["m"]
    Gt = tt.dot_batched([(dev[i], dev[j]) for i in range(m) for j in range(m)]).reshape(m, m)
    cm, _ = synth.mixing_coefficients(0.5 * (Gt + Gt.T), w["seed"], w["kappa"])
    A = [[(float(cm[k, j]), tt.TT.from_cores(t[j], device="cuda", dtype=torch.float64)) for j in range(k + 1)]
         for k in range(m)]
    Q, R, loo, st = tt.orthogonalize("householder", A, w["delta"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        tt.orthogonalize("householder", A, w["delta"], with_loo=False)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    ctx = tt._ctx()
    ctx.lib.tt_ctx_set_profiling.argtypes = [C.c_void_p, C.c_int]
    ctx.lib.tt_ctx_set_profiling(ctx.h, 1)
    tt.orthogonalize("householder", A, w["delta"], with_loo=False)
    torch.cuda.synchronize()
    prof = profile_arrays(ctx)
    ctx.lib.tt_ctx_set_profiling(ctx.h, 0)
    busy = sum(v["ms"] for v in prof.values())
    return {"value": round(1.0 / dt, 3), "unit": "orthogonalizations/s", "ms_per_call": round(1e3 * dt, 3),
            "device_busy_ms": round(busy, 3), "rounds": st["rounds"], "max_loo": float(max(loo)),
            "max_pre_rank": st["max_pre_rank"], "max_post_rank": st["max_post_rank"],
            "roofline": roofline_of(prof, bulk_fp32=False), "workload": HH_DESC}


def cpu_baseline_householder(reps_seconds=10.0):
    """The oracle's TT-Householder on the same workload (its own FP64 Gram matrix of the generators)."""
    import numpy as np
    import oracle
    from paper_2211_08770_amd import synth
    w = HH_WORKLOAD
    t = synth.conditioned_terms(w["seed"], w["m"], w["d"], w["n"], w["r"])
    cm, _ = synth.mixing_coefficients(oracle.gram_of(t), w["seed"], w["kappa"])
    A = [[(float(cm[k, j]), [c.copy() for c in t[j]]) for j in range(k + 1)] for k in range(w["m"])]
    n = 0
    t0 = time.perf_counter()
    while True:
        oracle.householder(A, w["delta"])
        n += 1
        if time.perf_counter() - t0 >= reps_seconds:
            break
    dt = time.perf_counter() - t0
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    return {"value": n / dt, "unit": "orthogonalizations/s", "cores": int(cores), "kind": "oracle",
            "sample": f"{n} FP64 NumPy/LAPACK TT-Householder calls on the same workload ({dt:.1f} s)"}


RTO_DESC = ("randomized rounding (Randomize-then-Orthogonalize) of the headline lazy sum in FP64: Gaussian sketch "
            "TT of ranks 30 (seed 50001), then deterministic rounding at delta=1e-4")


def rto_inputs(tt, torch, np_mod):
    from paper_2211_08770_amd import synth
    terms = synth.sum_of_graded_terms(dtype=np_mod.float64)
    sk = synth.random_tt(synth.rng(50001), [32] * 8, [1] + [30] * 7 + [1])
    return terms, sk


def run_randomized(tt, torch, steps=10):
    """Randomized rounding of the graded sum (FP64): roundings/s, error, ranks."""
    import numpy as np
    terms, sk = rto_inputs(tt, torch, np)
    x = [(a, tt.TT.from_cores(c, device="cuda", dtype=torch.float64)) for a, c in terms]
    s_dev = tt.TT.from_cores(sk, device="cuda", dtype=torch.float64)
    out = tt.round_randomized(x, s_dev, 1e-4)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        out = tt.round_randomized(x, s_dev, 1e-4)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    nx = tt.norm(x)
    # one more call with the library profiler on (not part of the rate): the dominant kernel kind
    ctx = tt._ctx()
    ctx.lib.tt_ctx_set_profiling.argtypes = [C.c_void_p, C.c_int]
    ctx.lib.tt_ctx_set_profiling(ctx.h, 1)
    tt.round_randomized(x, s_dev, 1e-4)
    torch.cuda.synchronize()
    prof = profile_arrays(ctx)
    ctx.lib.tt_ctx_set_profiling(ctx.h, 0)
    return {"value": round(1.0 / dt, 3), "unit": "TT-roundings/s", "ms_per_step": round(1e3 * dt, 4),
            "rel_err": tt.norm(x + [(-1.0, out)]) / nx, "out_ranks": out.r,
            "roofline": roofline_of(prof, bulk_fp32=False), "workload": RTO_DESC}


def cpu_baseline_randomized(seconds=5.0):
    import numpy as np
    import oracle
    terms, sk = rto_inputs(None, None, np)
    n = 0
    t0 = time.perf_counter()
    while True:
        oracle.tt_round_rto(terms, sk, 1e-4)
        n += 1
        if time.perf_counter() - t0 >= seconds:
            break
    dt = time.perf_counter() - t0
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    return {"value": n / dt, "unit": "TT-roundings/s", "cores": int(cores), "kind": "oracle",
            "sample": f"{n} FP64 NumPy randomized roundings of the same sum with the same sketch ({dt:.1f} s)"}


PAPER_SCHEMES = ["cgs", "mgs", "cgs2", "mgs2", "gram", "householder"]
O6_CASES = {"cgs": (35, 0), "mgs": (35, 2048), "cgs2": (35, 2048), "mgs2": (35, 2048), "gram": (35, 0),
            "householder": (20, 8192)}
# every scheme to m = 35 (pre-round ranks up to about 16000; minutes per scheme)
O6_COMPLETE = {"cgs": (35, 0), "mgs": (35, 32768), "cgs2": (35, 32768), "mgs2": (35, 32768), "gram": (35, 0),
               "householder": (35, 32768)}
PAPER_DESC = ("Section 4 order-3 experiment: m=20 Krylov TT-vectors of the Dirichlet Laplacian (d=3, n=15; ones, "
              "-Delta_d, rank-one rounding, normalisation) generated on the GPU, then each scheme at delta=1e-5, FP64")


def run_paper_experiment(tt, torch, delta=1e-5, reps=3):
    """The paper's own workload: Krylov inputs, then the six schemes (time, LOO at k = m, TT storage of Q)."""
    ns, m = [15, 15, 15], 20
    tt.krylov_laplacian(ns, m)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        A = tt.krylov_laplacian(ns, m)
    torch.cuda.synchronize()
    gen_ms = 1e3 * (time.perf_counter() - t0) / reps
    full = 15 ** 3
    out = {"workload": PAPER_DESC, "inputs_ms": round(gen_ms, 3), "schemes": {}}
    for sch in PAPER_SCHEMES:
        try:
            Q, R, loo, st = tt.orthogonalize(sch, A, delta)
        except tt.TTError as e:
            out["schemes"][sch] = {"status": e.status}
            continue
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            tt.orthogonalize(sch, A, delta, with_loo=False)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / reps
        sizes = [sum(q.r[k] * q.n[k] * q.r[k + 1] for k in range(q.d)) for q in Q]
        out["schemes"][sch] = {"ms_per_call": round(ms, 3), "rounds": st["rounds"], "loo_at_m": float(loo[-1]),
                               "max_rank_q": max(max(q.r) for q in Q),
                               "compression_ratio_q": round(sum(sizes) / (m * full), 4),
                               "compression_ratio_q_last": round(sizes[-1] / full, 4),
                               "compression_gain_q": [round(g, 3) for g in st["gain"]]}
    out["order6"] = run_order6(tt, torch, delta)
    return out


def run_order6(tt, torch, delta=1e-5, complete=False):
    """The order-6 experiment (n = 15, m = 35): each scheme up to a pre-round rank guard (the
    completed prefix), beside the oracle's run of the same experiment (stored curves);
    complete=True runs every scheme to m = 35."""
    ns6, m6 = [15] * 6, 35
    A6 = tt.krylov_laplacian(ns6, m6)
    gold = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests", "golden", "order6_oracle.json")
    with open(gold) as f:
        ref6 = json.load(f)["schemes"]
    o6 = {}
    for sch, (mm, guard) in (O6_COMPLETE if complete else O6_CASES).items():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        try:
            Q, R, _, st = tt.orthogonalize(sch, A6[:mm], delta, rank_guard=guard, with_loo=False,
                                           partial_on_guard=True)
        except tt.TTError as e:
            o6[sch] = {"status": e.status, "oracle": ref6[sch].get("status", "completed")}
            continue
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        k = st["m_reached"]
        loo6 = tt.loo(Q)[0] if Q else []
        r = ref6[sch]
        o6[sch] = {"vectors": mm, "rank_guard": guard or None, "m_reached": k, "guard_hit": bool(st.get("guard")),
                   "seconds": round(sec, 3), "max_pre_rank": st["max_pre_rank"],
                   "loo_at_m_reached": float(loo6[-1]) if len(loo6) else None,
                   "oracle_loo_at_m_reached": r["loo"][k - 1] if k else None,
                   "max_rank_q": max(max(q.r) for q in Q) if Q else None,
                   "oracle_max_rank_q_prefix": max(max(v) for v in r["q_ranks"][:k]) if k else None}
        if complete:
            o6[sch]["loo"] = [float(v) for v in loo6]
            progress(f"order-6 {sch}")
    return {"workload": "d=6, n=15, m=35 Krylov TT-vectors, delta=1e-5, FP64; " +
                        ("every scheme to m = 35 (rank guard 32768)" if complete else
                         "each scheme up to its pre-round rank guard (CGS none, MGS/CGS2/MGS2 2048, "
                         "TT-Householder 8192 on the first 20 vectors)") +
                        "; the oracle's values from its stored run of the same experiment",
            "schemes": o6}


def cpu_baseline_paper_experiment(delta=1e-5):
    """The oracle on the same experiment (its own Krylov inputs), one call per scheme."""
    import oracle
    A = oracle.krylov_inputs([15, 15, 15], 20)
    res = {}
    t_all = 0.0
    for sch in PAPER_SCHEMES:
        t0 = time.perf_counter()
        try:
            oracle.orthogonalize(sch, A, delta)
            res[sch] = round(1e3 * (time.perf_counter() - t0), 1)
        except oracle.GramBreakdown:
            res[sch] = "breakdown"
        t_all += time.perf_counter() - t0
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    return {"ms_per_call": res, "cores": int(cores), "kind": "oracle",
            "sample": f"one FP64 NumPy/LAPACK call per scheme on the same experiment ({t_all:.1f} s)"}


SERVE_DESC = ("64 solvers, d~U{5..8}, n~U{32,64,128}, solver rank~U{4..32}, basis b0~U{10..39} (restart at 40), "
              "MGS2 FP32-bulk, delta=1e-6, 8 GiB admission budget")


def run_serving(torch, qps_points=(3.0, 6.0, 9.0, 15.0), nreq=500, keep_sample=0):
    """Poisson serving traces at several offered rates: MGS2 steps of 64 simulated TT-GMRES solvers
    against resident bases.  Per point: p50/p99 latency, throughput, engine steps; the saturation
    rate is the largest completed throughput.  keep_sample > 0 keeps that many finished requests
    (host copies of basis, w and result) for a check against the oracle in the CPU leg."""
    from paper_2211_08770_amd import serve
    points = []
    sample = []
    for qps in qps_points:
        solvers, g = serve.make_solvers(64, seed=40000, dtype=torch.float32)
        rep = serve.run_trace(solvers, g, qps=qps, nreq=nreq, delta=1e-6, keep_sample=keep_sample)
        sample += rep.pop("sample", [])
        points.append(rep)
    return {"points": points, "saturation_rps": round(max(p["throughput_rps"] for p in points), 2),
            "workload": SERVE_DESC, "_sample": sample}


def cpu_check_serving(sample):
    """Sampled finished requests against the oracle's MGS2 step on the same FP32 values upcast."""
    import numpy as np
    import oracle
    worst_q, worst_r = 0.0, 0.0
    for basis, w, q, r in sample:
        qref, cref = oracle.gs_step("mgs2", basis, w, 1e-6)
        diff = oracle.tt_sum([(1.0, q), (-1.0, qref)])
        G, _ = oracle.tt_orth_rl(diff)
        worst_q = max(worst_q, float(np.linalg.norm(G[0])))
        worst_r = max(worst_r, float(np.abs(r - cref).max() / oracle.tt_norm(w)))
    return {"requests_checked": len(sample), "max_q_diff": worst_q, "max_r_diff_rel": worst_r,
            "tolerance": 1e-5, "ok": bool(worst_q <= 1e-5 and worst_r <= 1e-5)}


def cpu_check_headline(out_cores):
    """The headline result against the oracle's rounding of the same sum (FP32 values upcast):
    difference norm and the error of each against the exact sum, relative to ||x||."""
    import numpy as np
    import oracle
    from paper_2211_08770_amd import synth
    terms = synth.sum_of_graded_terms(dtype=np.float32)
    x = oracle.tt_sum([(a, [c.astype(np.float64) for c in t]) for a, t in terms])
    ref = oracle.tt_round(x, 1e-4)
    nx = oracle.tt_norm(x)

    def dn(a, b):
        G, _ = oracle.tt_orth_rl(oracle.tt_sum([(1.0, a), (-1.0, b)]))
        return float(np.linalg.norm(G[0])) / nx
    return {"diff_vs_oracle_rounding": dn(out_cores, ref), "rel_err_exact": dn(out_cores, x),
            "oracle_rel_err_exact": dn(ref, x), "ranks_equal": oracle.tt_ranks(ref) == [c.shape[0] for c in out_cores] + [1]}


def cpu_baseline(seconds):
    import numpy as np
    import oracle
    from paper_2211_08770_amd import synth
    terms = synth.sum_of_graded_terms(dtype=np.float32)
    x = oracle.tt_sum([(a, [c.astype(np.float64) for c in t]) for a, t in terms])
    n = 0
    t0 = time.perf_counter()
    while True:
        oracle.tt_round(x, 1e-4)
        n += 1
        if time.perf_counter() - t0 >= seconds:
            break
    dt = time.perf_counter() - t0
    return {"value": n / dt, "unit": "TT-roundings/s", "cores": blas_cores(), "kind": "oracle",
            "sample": f"{n} FP64 NumPy/LAPACK roundings of the same 20-term sum at delta=1e-4 ({dt:.1f} s)"}


_T0 = time.perf_counter()


def progress(what):
    """One line per finished measurement on stderr (stdout carries only the JSON line)."""
    print(f"bench: {what} done at {time.perf_counter() - _T0:.1f} s", file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the library has no multi-GPU path.",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2211_08770_amd import tt
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.copy_calibration:
        src = torch.ones(256 << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": 2 * src.numel(), "launches": 3}))
        return
    import numpy as np
    torch.cuda.set_device(0)
    tt._load()
    if args.householder_only:
        print(json.dumps(run_householder(tt, torch)))
        return
    if args.randomized_only:
        print(json.dumps(run_randomized(tt, torch)))
        return
    if args.batched_only:
        print(json.dumps(run_batched(tt, torch)))
        return
    if args.order6_only or args.order6_complete:
        print(json.dumps(run_order6(tt, torch, complete=args.order6_complete)))
        return
    if args.order6_n64_only:
        kw = {"runs": [(a, b) for a in ("gram", "cgs2") for b in (1e-3, 1e-5, 1e-7)]} if args.order6_n64_all else {}
        if args.order6_n64_guard:
            kw.update(guard=args.order6_n64_guard, profile=False)
        print(json.dumps(run_cgs2_gram_m50_order6(tt, torch, **kw)))
        return
    if args.serving_only:
        kw = {"qps_points": tuple(float(v) for v in args.serving_qps.split(","))} if args.serving_qps else {}
        rep = run_serving(torch, nreq=args.serving_requests, **kw)
        rep.pop("_sample")
        print(json.dumps(rep))
        return
    pst = min(args.steps, 10)
    res32 = run_config(tt, torch, torch.float32, 1e-4, args.steps, args.warmup, profile_steps=pst)
    progress("headline FP32-bulk")
    if args.headline_only:
        res64 = res64b = res32b = None
    else:
        res64 = run_config(tt, torch, torch.float64, 1e-4, args.steps, args.warmup)
        res64b = run_config(tt, torch, torch.float64, 1e-8, max(args.steps // 2, 1), 1)
        res32b = run_config(tt, torch, torch.float32, 1e-8, max(args.steps // 2, 1), 1)
        progress("FP64 and delta 1e-8 lines")
    # dominant kernel of the headline configuration (from the separate profiled pass)
    prof = res32["prof"]
    roof = roofline_of(prof)
    roof["traffic"] = recorded_traffic(roof["kernel"])
    line = {
        "metric": "TT-roundings/sec, FP32-bulk vs FP64 at rel.err <= delta",
        "value": round(res32["rate"], 3) if res32["rel_err"] <= 1e-4 else 0.0,
        "unit": "TT-roundings/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(res32["ms"], 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 bulk (f64 R-tree, SVD, norms)", "data": "synthetic",
        "config": {"workload": "TT-round of a lazy sum of 20 rank-10 TTs, d=8, n=32, term j scaled 2^-j per core "
                               "(input rank 200), delta=1e-4",
                   "global_batch": 1, "seq_len": None, "parallelism": "none (1 GPU)"},
        "rel_err": res32["rel_err"], "out_ranks": res32["ranks"],
        "fp64": None if res64 is None else {
            "value": round(res64["rate"], 3), "ms_per_step": round(res64["ms"], 4), "rel_err": res64["rel_err"],
            "out_ranks": res64["ranks"], "fp32_bulk_speedup": round(res32["rate"] / res64["rate"], 3)},
        "fp64_delta_1e-8": None if res64b is None else {
            "value": round(res64b["rate"], 3), "ms_per_step": round(res64b["ms"], 4),
            "rel_err": res64b["rel_err"], "out_ranks": res64b["ranks"]},
        # FP32-bulk cannot meet rel.err <= 1e-8: not a rate at that accuracy; reported with what it achieves
        "fp32_bulk_delta_1e-8": None if res32b is None else {
            "value": "n/a", "achieved_rel_err": res32b["rel_err"], "delta_eff": res32b["delta_eff"],
            "roundings_per_s_at_delta_eff": round(res32b["rate"], 3), "out_ranks": res32b["ranks"]},
        "kernel_ms_per_step": {k: round(v["ms"] / pst, 4) for k, v in prof.items()},
        "kernel_profile": f"{pst} further roundings with the library's per-launch HIP-event profiler on (not timed)",
        "roofline": roof,
    }
    sample = []
    if not args.headline_only:
        line["batched_uneven"] = run_batched(tt, torch)
        progress("batched_uneven")
        line["mgs_m20_order4"] = run_mgs_m20_order4(tt, torch)
        progress("mgs_m20_order4")
        all_runs = {"runs": [(a, b) for a in ("gram", "cgs2") for b in (1e-3, 1e-5, 1e-7)]}
        line["cgs2_gram_m50_order6_guarded"] = run_cgs2_gram_m50_order6(
            tt, torch, **(all_runs if args.order6_n64_all else {}))
        progress("cgs2_gram_m50_order6_guarded")
        line["serving"] = run_serving(torch, nreq=args.serving_requests, keep_sample=0 if args.no_cpu else 2)
        sample = line["serving"].pop("_sample")
        progress("serving sweep")
        line["householder"] = run_householder(tt, torch)
        progress("householder")
        line["paper_experiment"] = run_paper_experiment(tt, torch)
        progress("paper_experiment")
        line["randomized"] = run_randomized(tt, torch)
        progress("randomized")
    if not args.no_cpu and not args.headline_only:
        # oracle legs (CPU): baselines timed on the host, and result checks against the oracle
        line["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
        progress("cpu_baseline")
        line["cpu_baseline_1thread"] = at_threads(1, lambda: cpu_baseline(args.cpu_seconds / 2))
        progress("cpu_baseline_1thread")
        line["oracle_check"] = cpu_check_headline([c.astype(np.float64) for c in res32["out"].numpy_cores()])
        progress("oracle_check")
        line["batched_uneven"]["cpu_baseline"] = cpu_baseline_batched()
        progress("batched_uneven cpu_baseline")
        line["mgs_m20_order4"]["cpu_baseline"] = cpu_baseline_mgs_m20_order4()
        progress("mgs_m20_order4 cpu_baseline")
        line["cgs2_gram_m50_order6_guarded"]["cpu_baseline"] = cpu_baseline_cgs2_m50_order6()
        progress("cgs2_gram_m50_order6_guarded cpu_baseline")
        line["serving"]["oracle_check"] = cpu_check_serving(sample)
        progress("serving oracle_check")
        line["householder"]["cpu_baseline"] = cpu_baseline_householder()
        progress("householder cpu_baseline")
        line["paper_experiment"]["cpu_baseline"] = cpu_baseline_paper_experiment()
        progress("paper_experiment cpu_baseline")
        line["randomized"]["cpu_baseline"] = cpu_baseline_randomized()
        progress("randomized cpu_baseline")
    print(json.dumps(line))

if __name__ == "__main__":
    main()
