"""Serving loop: Poisson arrivals of orthogonalization requests from simulated
TT-GMRES solvers, admitted by device-memory footprint and run by the
continuous-batching engine of the library (tt_engine_*).

Each solver keeps its orthonormal Krylov basis resident on the device.  A
request orthogonalizes a new vector against that basis with TT-MGS2
(Algorithm 4, one step); its result is appended to the basis (restart at
`bmax`).  A solver has at most one request in flight (its next Arnoldi step
needs the previous one); later arrivals for a busy solver wait in its queue.
Latency is measured from arrival to completion.  This module only schedules:
all arithmetic runs in the library.
"""
from __future__ import annotations

import collections
import time

import numpy as np
import torch

from . import synth, tt

__all__ = ["Solver", "make_solvers", "run_trace"]


class Solver:
    def __init__(self, spec, device, dtype):
        self.spec = spec
        self.dtype = dtype
        self.device = device
        self.basis = [tt.TT.from_cores(synth.serving_vector(None, spec, spec["firsts"][j]), device=device,
                                       dtype=dtype) for j in range(spec["b0"])]
        self.initial = list(self.basis)
        self.gram = np.eye(len(self.basis))
        self.busy = False
        self.queue = collections.deque()

    def nbytes(self):
        return sum(q.data.numel() * q.data.element_size() for q in self.basis)

    def append(self, q, gram_row):
        b = len(self.basis)
        if b + 1 >= self.spec["bmax"]:            # restart from the initial basis
            self.basis = list(self.initial)
            self.gram = np.eye(len(self.basis))
            return
        g = np.zeros((b + 1, b + 1))
        g[:b, :b] = self.gram
        g[b, :b] = g[:b, b] = gram_row
        g[b, b] = 1.0
        # (a result far below its rank bounds owns a packed buffer: a long trace does not
        # fill the device with bound-sized buffers)
        self.basis.append(q)
        self.gram = g


def make_solvers(nsolvers=64, seed=40000, device="cuda", dtype=torch.float32, **kw):
    g = synth.rng(seed)
    return [Solver(synth.serving_solver(g, dtype=np.float32 if dtype == torch.float32 else np.float64, **kw),
                   device, dtype) for _ in range(nsolvers)], g


def run_trace(solvers, g, qps=200.0, nreq=200, delta=1e-6, scheme="mgs2", budget_bytes=8 << 30,
              max_inflight=64, engine=None, keep_sample=0):
    """Replay nreq Poisson arrivals at `qps` (requests/s) over the solvers.

    Returns a dict with p50/p99 latency (ms) and throughput (requests/s) of
    the requests served, the counts of requests rejected at admission (a
    footprint above the budget, or, once every request has arrived and none is
    in flight, above the room the bases leave) and of
    requests whose step failed (breakdown, capacity: reported by the engine,
    neither served nor timed), the high-water mark of the device memory the
    loop holds (bases plus in-flight requests) and the engine steps taken.
    With keep_sample > 0, "sample" holds host copies (float64) of the basis,
    w, q and the R column of that many requests that completed, for checks.
    """
    kept = []
    eng = engine or tt.Engine()
    arrivals = np.cumsum(g.exponential(1.0 / qps, size=nreq))
    owners = g.integers(0, len(solvers), size=nreq)
    reqs = []
    for i in range(nreq):
        s = solvers[owners[i]]
        w = synth.serving_request(g, s.spec, min(len(s.basis), s.spec["b0"]))
        reqs.append((arrivals[i], owners[i], w))
    lat, rejected, failed, steps = [], 0, 0, 0
    inflight = {}                      # engine id -> (request index, solver, footprint)
    held = sum(s.nbytes() for s in solvers)
    high = held
    nxt = 0
    done = 0
    t0 = time.perf_counter()
    while done + failed + rejected < nreq:
        now = time.perf_counter() - t0
        while nxt < nreq and reqs[nxt][0] <= now:      # arrivals go to their solver's queue
            solvers[reqs[nxt][1]].queue.append(nxt)
            nxt += 1
        # admission: idle solvers with a queued request, while slots and memory allow
        blocked = []                                   # solvers whose queue head did not fit
        for s in solvers:
            if s.busy or not s.queue or len(inflight) >= max_inflight:
                continue
            i = s.queue[0]
            w = tt.TT.from_cores(synth.serving_vector(None, s.spec, reqs[i][2]), device=s.device, dtype=s.dtype)
            fp = eng.footprint(scheme, s.basis, w) + w.data.numel() * w.data.element_size()
            if fp > budget_bytes:
                s.queue.popleft()
                rejected += 1
                continue
            if held + fp > budget_bytes:
                blocked.append(s)
                continue
            s.queue.popleft()
            rid = eng.submit(scheme, s.basis, w, delta, basis_gram=s.gram)
            inflight[rid] = (i, s, fp, w)
            s.busy = True
            held += fp
            high = max(high, held)
        if inflight:
            out = eng.step()
            steps += 1
            tnow = time.perf_counter() - t0
            inflight_w = {rid: inflight[rid][3] for rid in out}
            for rid, (status, q, r, grow) in out.items():
                i, s, fp, _ = inflight.pop(rid)
                held -= fp
                s.busy = False
                if status != "TT_OK":
                    failed += 1
                    continue
                done += 1
                lat.append(tnow - reqs[i][0])
                if len(kept) < keep_sample:
                    kept.append((list(s.basis), inflight_w[rid], q, r))
                before = s.nbytes()
                s.append(q, grow)
                held += s.nbytes() - before
        elif nxt < nreq:
            time.sleep(max(0.0, min(reqs[nxt][0] - (time.perf_counter() - t0), 0.01)))
        else:
            # every request has arrived and none is in flight, so no finishing request will free
            # memory: a queue head that did not fit beside the bases in this pass never will.
            # Those are rejected (the requests behind them are tried in the next pass).
            for s in blocked:
                s.queue.popleft()
                rejected += 1
    wall = time.perf_counter() - t0
    lat_ms = np.array(lat) * 1e3
    host = lambda t: [c.astype(np.float64) for c in t.numpy_cores()]
    sample = [([host(b) for b in basis], host(w), host(q), np.array(r)) for basis, w, q, r in kept]
    return {"sample": sample, "qps_offered": qps, "requests": nreq, "completed": done, "rejected": rejected,
            "failed": failed,
            "p50_ms": float(np.percentile(lat_ms, 50)) if len(lat_ms) else None,
            "p99_ms": float(np.percentile(lat_ms, 99)) if len(lat_ms) else None,
            "throughput_rps": done / wall, "wall_s": wall, "engine_steps": steps,
            "hbm_high_water_bytes": int(high)}
