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
time, measured live with HIP events on the library's stream during the timed
region; its achieved rate is the algorithmic flops of its launches divided by
their summed duration.  cpu_baseline times the FP64 CPU oracle on a bounded
sample of the same rounding.
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
    p.add_argument("--cpu-seconds", type=float, default=15.0)
    p.add_argument("--copy-calibration", action="store_true",
                   help="only run a plain 256 MiB device-to-device copy (reference for the HBM byte counters)")
    p.add_argument("--headline-only", action="store_true",
                   help="time only the headline configuration (for profiler runs); no FP64 side runs, no CPU baseline")
    p.add_argument("--householder-only", action="store_true",
                   help="only the TT-Householder measurement (for profiler runs); prints its JSON object")
    p.add_argument("--randomized-only", action="store_true",
                   help="only the randomized-rounding measurement (for profiler runs); prints its JSON object")
    return p.parse_args()


def recorded_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary (FETCH_SIZE + WRITE_SIZE,
    copy-calibrated), or None when there is none or the QR source changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_graded_sum_r200_traffic.txt")
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
    # FP32-bulk leaves are factored and applied on the FP32 MFMA (157.3 TF/s); tree nodes and the SVD are
    # FP64 (78.6 TF/s).  The apply kind mixes leaf and node tiles: it is priced at the FP32 peak, so its
    # fraction is a lower bound.  An FP64 workload runs every kind on the FP64 units.
    # The Jacobi SVD, the component GEMMs and the TT dots run on the vector ALU ("alu"; the
    # component GEMMs are FP32 in an FP32-bulk workload), the tile QR kernels on MFMA.
    alu = name in ("svd_jacobi", "contraction_gemm", "tt_dot", "other")
    if alu:
        peak = PEAK["fp32_vector"] if (bulk_fp32 and name == "contraction_gemm") else PEAK["fp64_vector"]
    else:
        fp32_kinds = ("qr_factor_leaf", "qr_apply") if bulk_fp32 else ()
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


def run_config(tt, torch, dtype, delta, steps, warmup, profile):
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
    if profile:
        ctx.lib.tt_ctx_set_profiling(ctx.h, 1)
    t0 = time.perf_counter()
    for _ in range(steps):
        out = tt.round(x, delta)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = profile_arrays(ctx) if profile else None
    if profile:
        ctx.lib.tt_ctx_set_profiling(ctx.h, 0)
    # validity: ||x - x~|| / ||x|| on the GPU (norms of lazy sums by the right-to-left sweep)
    nx = tt.norm(x)
    nd = tt.norm(x + [(-1.0, out)])
    return {"rate": steps / dt, "ms": 1e3 * dt / steps, "ranks": out.r, "rel_err": nd / nx, "prof": prof}


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
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        outs = tt.round_batched(xs, 1e-5)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
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
    return {"value": round(len(xs) / dt, 2), "unit": "TT-roundings/s", "jobs": len(xs), "ms_per_batch": round(1e3 * dt, 3),
            "roofline": roofline_of(prof),
            "ranks_equal_caps": caps_ok, "max_sampled_rel_err": max(errs),
            "workload": "256 uneven jobs: d~U{4..10}, n~U{16,32,64}, rank~U{8..128}, N(0,1) FP32 cores, delta=1e-5"}


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
                               "compression_ratio_q": round(sum(sizes) / (m * full), 4)}
    return out


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


def run_serving(torch, qps=100.0, nreq=150):
    """Poisson serving trace: MGS2 steps of 64 simulated TT-GMRES solvers against resident bases."""
    from paper_2211_08770_amd import serve
    solvers, g = serve.make_solvers(64, seed=40000, dtype=torch.float32)
    rep = serve.run_trace(solvers, g, qps=qps, nreq=nreq, delta=1e-6)
    rep["workload"] = ("64 solvers, d~U{5..8}, n~U{32,64,128}, solver rank~U{4..9}, basis b0~U{10..39} (restart at 40), "
                       "MGS2 FP32-bulk, delta=1e-6, 8 GiB admission budget")
    return rep


def cpu_baseline(seconds):
    import numpy as np
    import oracle
    from paper_2211_08770_amd import synth
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count() or 1
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
    return {"value": n / dt, "unit": "TT-roundings/s", "cores": int(cores), "kind": "oracle",
            "sample": f"{n} FP64 NumPy/LAPACK roundings of the same 20-term sum at delta=1e-4 ({dt:.1f} s)"}


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
    torch.cuda.set_device(0)
    tt._load()
    if args.householder_only:
        print(json.dumps(run_householder(tt, torch)))
        return
    if args.randomized_only:
        print(json.dumps(run_randomized(tt, torch)))
        return
    res32 = run_config(tt, torch, torch.float32, 1e-4, args.steps, args.warmup, profile=True)
    if args.headline_only:
        res64 = res64b = None
    else:
        res64 = run_config(tt, torch, torch.float64, 1e-4, args.steps, args.warmup, profile=False)
        res64b = run_config(tt, torch, torch.float64, 1e-8, max(args.steps // 2, 1), 1, profile=False)
    # dominant kernel of the headline configuration
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
            "out_ranks": res64["ranks"]},
        "fp64_delta_1e-8": None if res64b is None else {
            "value": round(res64b["rate"], 3), "ms_per_step": round(res64b["ms"], 4),
            "rel_err": res64b["rel_err"], "out_ranks": res64b["ranks"]},
        "kernel_ms_per_step": {k: round(v["ms"] / args.steps, 4) for k, v in prof.items()},
        "roofline": roof,
    }
    if not args.headline_only:
        line["batched_uneven"] = run_batched(tt, torch)
        line["serving"] = run_serving(torch)
        line["householder"] = run_householder(tt, torch)
        line["paper_experiment"] = run_paper_experiment(tt, torch)
        line["randomized"] = run_randomized(tt, torch)
    if not args.no_cpu and not args.headline_only:
        line["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
        line["householder"]["cpu_baseline"] = cpu_baseline_householder()
        line["paper_experiment"]["cpu_baseline"] = cpu_baseline_paper_experiment()
        line["randomized"]["cpu_baseline"] = cpu_baseline_randomized()
    print(json.dumps(line))


if __name__ == "__main__":
    main()
