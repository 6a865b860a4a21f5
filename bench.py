#!/usr/bin/env python3
"""Batched rank-k update throughput of the incremental-SVD engine on one MI355X.

Workload (one "step" = one tick): 512 independent factor-model streams with
n ~ U{50..2000} columns, m ~ U{1000..50000} rows and rank k ~ U{8,16,32,64}
(clamped to n), five factors (variances 4, 2, 1, 0.5, 0.25, noise 0.1); each
tick appends one row to every stream.  The chosen form runs a tick as one
batched launch sequence over all streams with FP32 storage, projections and
rotations and an FP64 core; the plain form runs the same updates one stream
per launch sequence in FP64.  Both start from the same factors (the FP64
engine's TruncatedSVD of A_0; the FP32 engine is seeded with them) and apply
the same rows, so the FP32 result is compared with the FP64 one at the end.

Prints ONE JSON line on stdout; progress goes to stderr.
"""
import argparse
import ctypes
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np

METRIC = "batched rank-k updates/sec + p99 tick latency vs plain path at rel err ≤2e-5"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3
K_FACTORS = 5
SEED = 3
PROF_TICKS = 20      # extra profiled ticks (per-launch times) after the comparison
CPU_MAX_ROUNDS = 2000   # cap of the oracle baseline's rounds (its time budget ends it first)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def stream_params(nstreams, seed=SEED):
    """(m0, n0, k) per stream, drawn from Philox uniforms of the input generator."""
    from synth import uniforms
    u = uniforms(seed, 0xC3, 100, np.arange(nstreams), 3)
    n = 50 + np.floor(u[:, 0] * 1951).astype(np.int64)
    m = 1000 + np.floor(u[:, 1] * 49001).astype(np.int64)
    k = np.array([8, 16, 32, 64])[np.minimum(np.floor(u[:, 2] * 4).astype(np.int64), 3)]
    k = np.minimum(k, n)
    return [(int(a), int(b), int(c)) for a, b, c in zip(m, n, k)]


def rot_bytes(m, n, k, esz):
    # rotation of one row append: read + write U (m x k) and V (n x k), read x, write the A row
    return esz * (2 * m * k + 2 * n * k) + n * (esz + esz)


def rot_u_bytes(m, k, esz):
    # U's rotation in a row append: read + write U (m x k)
    return esz * 2 * m * k


def tick_bytes(m, n, k, esz, deferred=False):
    # whole row append: the projected basis V is read once more, x once more for the projection
    full = rot_bytes(m, n, k, esz) + esz * n * k + esz * n
    if not deferred:
        return full
    # deferred U: U is read and written once per explicit append, every m / (8 k)-th
    period = max(1, min(256, int(m) // (8 * k)))
    return full - rot_u_bytes(m, k, esz) + rot_u_bytes(m, k, esz) / period


CSRC = os.path.join(ROOT, "paper_2605_24514_amd", "csrc")
PMC_ROTATE = (os.path.join(ROOT, "profiles", "rotate_u_kc64_tick512_pmc.md"),
              [os.path.join(CSRC, f) for f in ("isvd_common.h", "isvd_update.h")])
PMC_CORE = (os.path.join(ROOT, "profiles", "core_chain_tick512_pmc.md"),
            [os.path.join(CSRC, f) for f in ("isvd_common.h", "isvd_update.h", "isvd_secular.h", "isvd_jacobi.h",
                                             "isvd_chain.h")])


def core_bytes(k):
    # deferred row append in the core: W and W^-1 (k x k, FP64) read and
    # written, V's (k + 1) x k FP32 rotation written
    return 32.0 * k * k + 4.0 * k * (k + 1)


def recorded_traffic_ratio(record, key):
    """HBM traffic / algorithmic bytes under `key` in a committed counter
    record, or None once the kernel sources differ from the profiled ones."""
    import hashlib
    path, sources = record
    try:
        text = open(path).read()
    except OSError:
        return None
    ratio = sha = None
    for line in text.splitlines():
        if line.startswith(key + ":"):
            ratio = float(line.split(":")[1])
        if line.startswith("kernel_source_sha256:"):
            sha = line.split(":")[1].strip()
    h = hashlib.sha256()
    for f in sources:
        h.update(open(f, "rb").read())
    return ratio if (ratio is not None and sha == h.hexdigest()) else None


def pctl(a, q):
    return float(np.percentile(np.asarray(a), q))


def cpu_baseline(params, seconds, torch):
    """Time the FP64 oracle's row append (Alg. A1, oracle.brand.row_append, as
    it stands) on a bounded sample of the workload, with A pre-reserved: each
    appended row is written into a preallocated m_cap x n array, as the GPU
    engine does, instead of the oracle engine loop's np.vstack of the dense A
    (which copies all of A on every append and would dominate the time)."""
    from threadpoolctl import threadpool_info
    from oracle import brand
    from synth import device as sdev
    sample = list(range(min(8, len(params))))
    rng = np.random.default_rng(0)
    states, rows, bufs = [], [], []
    for s in sample:
        m0, n0, k = params[s]
        A = torch.empty((m0, n0), dtype=torch.float64, device="cuda")
        sdev.rows_into(A, 0, m0, n0, SEED, s, K_FACTORS)
        Abuf = np.empty((m0 + CPU_MAX_ROUNDS, n0))
        Abuf[:m0] = A.cpu().numpy()
        del A
        U, _ = np.linalg.qr(rng.standard_normal((m0, k)))
        V, _ = np.linalg.qr(rng.standard_normal((n0, k)))
        sig = np.sort(rng.uniform(1.0, 100.0, k))[::-1]
        states.append([U, sig, V, m0, k])
        bufs.append(Abuf)
        R = torch.empty((64, n0), dtype=torch.float64, device="cuda")
        sdev.rows_into(R, m0, 64, n0, SEED, s, K_FACTORS)
        rows.append(R.cpu().numpy())
    done, t0 = 0, time.perf_counter()
    c0 = time.process_time()
    r = 0
    while True:
        for q, st in enumerate(states):
            U, sig, V, m, k = st
            x = rows[q][r % 64]
            bufs[q][m] = x
            U, sig, V, _ = brand.row_append(U, sig, V, x, k, 1e-10, cgs2=True)
            st[:] = [U, sig, V, m + 1, k]
            done += 1
        r += 1
        if time.perf_counter() - t0 > seconds or r >= CPU_MAX_ROUNDS:
            break
    wall = time.perf_counter() - t0
    cpu = time.process_time() - c0
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    mean_m = float(np.mean([params[s][0] for s in sample]))
    return {"value": done / wall, "unit": "updates/s", "cores": int(threads), "kind": "oracle",
            "sample": "%d row appends over the first %d streams of the workload (%d rounds, mean m %.0f; the 64 "
                      "generated rows of each stream appended in turn): the "
                      "FP64 oracle's Alg. A1 row append (oracle.brand.row_append, CGS2) with A pre-reserved "
                      "(each row written in place); started from random orthonormal factors of each stream's "
                      "shape (the update's cost does not depend on their values); cores = BLAS threads"
                      % (done, len(sample), r, mean_m),
            "wall_s": wall, "cpu_s": cpu, "nproc": os.cpu_count()}


def serve_main(args):
    """Serving run: streams of the batched workload's sizes arrive as requests
    (Poisson, mixed row / column / entry updates, per-stream policies) and are
    admitted under an HBM budget; prints one JSON line."""
    print(json.dumps(serve_run(args)), flush=True)


def serve_run(args):
    """The serving run of serve_main; returns its record."""
    import torch
    from paper_2605_24514_amd import isvd
    from synth import device as sdev, uniforms
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    N, L, rate = args.serve_streams, args.serve_lifetime, args.serve_rate
    params = stream_params(N, seed=7)
    u = uniforms(7, 0xC4, 101, np.arange(N), 1)[:, 0]
    pol_kind = np.minimum((u * 4).astype(int), 3)
    policies = [isvd.Policy(kind=isvd.POL_PERIODIC, period=500),
                isvd.Policy(kind=isvd.POL_ERROR, gamma=1.05, check_every=100, t_min=100),
                isvd.Policy(kind=isvd.POL_ANGLE, theta_max=1e-3, t_min=1),
                isvd.Policy(kind=isvd.POL_ADAPTIVE, tau=0.95, band=0.01, eta=0.5, k_min=1, period=500)]
    rng = np.random.default_rng(17)
    dev_stream = torch.cuda.Stream()
    eng = isvd.Engine()
    # released streams' blocks are reused by later admissions (no device-wide
    # wait per release, no allocation per admission)
    eng.set_block_cache(int(args.serve_cache_gb * 1e9))
    srv = isvd.Server(eng, hbm_budget=int(args.serve_budget_gb * 1e9), max_inflight=2, stream=dev_stream)
    log("serving: %d streams, lifetime %d, %.0f requests/s, budget %.0f GB" % (N, L, rate, args.serve_budget_gb))
    # Every stream's requests are drawn up front; its A0 (about 105 MB on
    # average, 428 GB for 4096 streams) is generated when the stream joins the
    # admission queue, and at most `window` streams wait in that queue with
    # their A0 in memory.  Requests of a stream that has not joined yet are
    # held here and submitted with their own arrival times when it joins, so
    # the admission order is that of a server that registered every stream at
    # once (the waits include generating A0 on the device).
    rows_pool, cols, reqs, arrivals, owner = [], [], [], [], []
    with torch.cuda.stream(dev_stream):
        for s, (m0, n0, k) in enumerate(params):
            R = torch.empty((16, n0 + L), dtype=torch.float32, device="cuda")
            sdev.rows_into(R, m0, 16, n0 + L, SEED, s, K_FACTORS)
            rows_pool.append(R)
            cols.append(torch.randn(m0 + L, dtype=torch.float32, device="cuda"))
            kinds = rng.choice([0, 1, 2], size=L, p=[0.7, 0.15, 0.15])
            t = np.cumsum(rng.exponential(N / rate, size=L))
            m, n = m0, n0
            for q in range(L):
                r = isvd.CRequest()
                r.kind = int(kinds[q])
                if r.kind == isvd.ROW:
                    r.payload = ctypes.c_void_p(R[q % 16].data_ptr())
                    r.len, r.dtype = n, isvd.DTYPE_F32
                    m += 1
                elif r.kind == isvd.COL:
                    r.payload = ctypes.c_void_p(cols[-1].data_ptr())
                    r.len, r.dtype = m, isvd.DTYPE_F32
                    n += 1
                else:
                    r.i, r.j, r.delta = int(rng.integers(m)), int(rng.integers(n)), float(rng.normal(0, 0.5))
                    r.dtype = isvd.DTYPE_F32
                reqs.append(r)
                arrivals.append(t[q])
                owner.append(s)
    torch.cuda.synchronize()
    order = np.argsort(np.asarray(arrivals), kind="stable")
    arr = np.asarray(arrivals)[order]
    own = np.asarray(owner, dtype=np.int64)[order]
    creq = (isvd.CRequest * len(order))(*[reqs[i] for i in order])
    raw = np.frombuffer(creq, dtype=np.dtype((np.void, ctypes.sizeof(isvd.CRequest))))
    total = len(order)
    del reqs
    ticket = np.full(N, -1, dtype=np.int64)
    window = args.serve_window
    # each stream's requests (positions in arrival order), for its join
    by_stream = np.split(np.argsort(own, kind="stable"), np.cumsum(np.bincount(own, minlength=N))[:-1])

    # A0 of the joining streams in a ring of `window` slots of the largest
    # size (a slot is reused only after its stream was admitted: at most
    # `window` streams wait with their A0; admission is in join order), each
    # generated on the server's stream without a wait, so that the server's
    # creation of the stream reads it in stream order
    slot_elems = max(m0 * n0 for (m0, n0, k) in params)
    with torch.cuda.stream(dev_stream):
        a0_pool = torch.empty((window, slot_elems), dtype=torch.float32, device="cuda")
        a0_gen = sdev.AsyncRows(max(p[0] for p in params), max(p[1] for p in params), K_FACTORS)

    def join(s):
        m0, n0, k = params[s]
        with torch.cuda.stream(dev_stream):
            A0 = a0_pool[s % window, :m0 * n0].view(m0, n0)
            a0_gen.rows_into(A0, 0, m0, n0, SEED, s, dev_stream.cuda_stream)
            ticket[s] = srv.add_stream(A0, min(k, n0), m_cap=m0 + L, n_cap=n0 + L, lifetime=L,
                                       policy=policies[int(pol_kind[s])], refresh_iters=1)

    def submit(idx):
        if len(idx) == 0:
            return
        g = np.ascontiguousarray(raw[idx])
        srv.submit_many(ticket[own[idx]], ctypes.cast(g.ctypes.data, ctypes.POINTER(isvd.CRequest)),
                        arr[idx] + t_start)

    log("serving: %d requests prepared" % total)
    t_start = srv.clock()
    pos, joined, ndone, done = 0, 0, 0, []
    last = time.perf_counter()
    hs = {"join": 0.0, "submit": 0.0, "step": 0.0, "poll": 0.0}   # the harness's own host seconds
    while ndone < total:
        h0 = time.perf_counter()
        while joined < N and srv.held_a0() < window:
            join(joined)
            # the requests that arrived before the stream joined
            mine = by_stream[joined]
            submit(mine[mine < pos])
            joined += 1
        h1 = time.perf_counter()
        now = srv.clock() - t_start
        hi = int(np.searchsorted(arr, now, side="right"))
        if hi > pos:
            idx = np.arange(pos, hi)
            submit(idx[ticket[own[idx]] >= 0])
            pos = hi
        h2 = time.perf_counter()
        srv.step()
        h3 = time.perf_counter()
        c = srv.poll_array()
        h4 = time.perf_counter()
        hs["join"] += h1 - h0
        hs["submit"] += h2 - h1
        hs["step"] += h3 - h2
        hs["poll"] += h4 - h3
        if len(c):
            done.append(c)
            ndone += len(c)
        if pos >= total and joined == N and srv.stats()["queued"] == 0:
            srv.drain()
            c = srv.poll_array()
            done.append(c)
            ndone += len(c)
        if time.perf_counter() - last > 10:
            last = time.perf_counter()
            log("  %d / %d requests done, %d streams joined, %s" % (ndone, total, joined, srv.stats()))
    wall = srv.clock() - t_start
    done = np.concatenate(done)
    ok = done[done["status"] == 0]
    lat = (ok["done_s"] - ok["arrival_s"]) * 1e3
    wait = np.maximum(0.0, ok["admit_s"] - ok["arrival_s"]) * 1e3
    served = (ok["done_s"] - np.maximum(ok["arrival_s"], ok["admit_s"])) * 1e3
    out = {"metric": "serving updates/s with p50/p99 arrival-to-completion latency (mixed requests, "
                     "per-stream policies, HBM-budget admission)",
           "value": round(len(ok) / wall, 1), "unit": "updates/s", "n_gpus": 1, "higher_is_better": True,
           "dtype": "f32", "data": "synthetic",
           "config": {"workload": "serving loop: %d factor-model streams (n~U{50..2000}, m~U{1000..50000}, "
                                  "k~U{8,16,32,64}), %d requests each, 70/15/15 row/column/entry, Poisson "
                                  "arrivals at %.0f/s aggregate, policies uniform over periodic 500 / error 1.05 / "
                                  "angle 1e-3 / adaptive 0.95, budget %.0f GB" % (N, L, rate, args.serve_budget_gb),
                      "streams": N, "lifetime": L},
           "requests": total, "completed_ok": len(ok), "wall_s": round(wall, 3),
           "latency_ms": {"p50": round(pctl(lat, 50), 3), "p99": round(pctl(lat, 99), 3)},
           "after_admission_ms": {"p50": round(pctl(served, 50), 3), "p99": round(pctl(served, 99), 3)},
           "admission_wait_ms": {"p50": round(pctl(wait, 50), 3), "p99": round(pctl(wait, 99), 3)}}
    st = srv.stats()
    out["server"] = {"ticks": st["ticks"], "requests_per_tick": round(st["tick_requests"] / max(st["ticks"], 1), 1),
                     "host_s": {"admission": round(st["host_admit_s"], 3), "tick_calls": round(st["host_tick_s"], 3),
                                "waits": round(st["host_wait_s"], 3), "releases": round(st["host_release_s"], 3)},
                     "harness_s": {q: round(v, 3) for q, v in hs.items()}}
    srv.close()
    eng.close()
    return out


def refresh_main(args):
    """Refresh run: TruncatedSVD(A_t, 64) of one 100000 x 2000 FP32 stream (20
    factors) by block subspace iteration; prints one JSON line with the time
    per refresh and the matrix-core rate of its A X / A^T Q products."""
    import torch
    from paper_2605_24514_amd import isvd
    from synth import device as sdev
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    m, n, k = 100000, 2000, 64
    iters = -1 if args.refresh_iters is None else args.refresh_iters
    st = torch.cuda.Stream()
    A0 = torch.empty((m, n), dtype=torch.float32, device="cuda")
    sdev.rows_into(A0, 0, m, n, SEED, 0, 20)
    torch.cuda.synchronize()
    with isvd.Engine() as eng:
        sid = eng.init(A0, k, "fp32", refresh_iters=iters, stream=st)
        for _ in range(args.warmup):
            eng.refresh(sid, stream=st)
        st.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ts = []
        for _ in range(args.steps):
            e0.record(st)
            eng.refresh(sid, stream=st)
            e1.record(st)
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
        met = eng.metrics(sid, exact=True, stream=st)
    b = min(n, k + max(8, k // 2), 96)
    ms = float(np.median(ts))
    if iters < 0:
        form = ("Gram form: G = A^T A on the FP64 matrix cores, Chebyshev-filtered subspace iteration with "
                "locking until every leading Ritz residual <= 1e-10 theta_1, block b = %d, then A L, CholQR2, "
                "FP64 Rayleigh-Ritz" % b)
        gram_flop = 1.0 * m * n * (n + 64)      # the upper 64 x 64 tiles of A^T A, 2 flops per product
        extra = {"gram_tflops_equivalent": round(gram_flop / (ms * 1e-3) / 1e12, 1),
                 "refresh_rounds": met["refresh_rounds"], "refresh_converged": met["refresh_converged"]}
    else:
        form = ("A form: block b = %d, %d subspace iterations, CholQR2 / FP64 Gram, FP64 Rayleigh-Ritz"
                % (b, iters))
        gemm_flop = 2.0 * m * n * b * (2 * iters + 1)      # iters x (A X, A^T Q) + final A X
        extra = {"gemm_equivalent_tflops": round(gemm_flop / (ms * 1e-3) / 1e12, 1)}
    out = {"metric": "refresh time: TruncatedSVD(A_t, k) of one stream", "value": round(ms, 3), "unit": "ms",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "higher_is_better": False, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": "one factor-model stream, A 100000 x 2000 FP32 (20 factors), k = 64, " + form},
           "ms_min": round(min(ts), 3), "ms_p99": round(pctl(ts, 99), 3),
           "frob_ratio": met["frob_ratio"], "frob_opt": met["frob_opt"], "ortho_U": met["ortho_U"],
           "ortho_V": met["ortho_V"]}
    out.update(extra)
    print(json.dumps(out), flush=True)


SWEEP_SEED = 2


def precision_sweep(args, torch, isvd, appends, log_prefix="sweep"):
    """The precision sweep on one stream: a 1,000,000 x 512 factor-model panel
    (40 factors), k = 128, `appends` row appends, in three forms started from
    the same FP64 initial factors: FP64 throughout; FP32 storage, projections
    and rotations with the FP64 core and re-orthogonalisation; BF16 matrix-core
    rotations (FP32 accumulation) with the angle-threshold refresh at 1e-3 rad
    (Section 3.3).  Each form's error against the FP64 form after the run
    (the FP64 engine itself is held to the oracle by the rank-128 and full-size
    parity tests), updates/s and per-append latency."""
    from synth import device as sdev
    from tests.parity import compare
    m0, n, nf, k = 1_000_000, 512, 40, 128
    T = appends
    st = torch.cuda.Stream()
    A0 = torch.empty((m0, n), dtype=torch.float64, device="cuda")
    sdev.rows_into(A0, 0, m0, n, SWEEP_SEED, 0, nf)
    rows = torch.empty((T, n), dtype=torch.float64, device="cuda")
    sdev.rows_into(rows, m0, T, n, SWEEP_SEED, 0, nf)
    rows32 = rows.to(torch.float32)
    torch.cuda.synchronize()
    out = {"workload": "one stream, A 1,000,000 x 512 (40 factors), k = 128, %d row appends" % T}
    with isvd.Engine() as e64, isvd.Engine() as e32, isvd.Engine() as eb:
        t0 = time.perf_counter()
        s64 = e64.init(A0, k, "fp64", m_cap=m0 + T, n_cap=n, stream=st)
        st.synchronize()
        init_ms = (time.perf_counter() - t0) * 1e3
        met0 = e64.metrics(s64, stream=st)
        U, S, V = e64.factors(s64, stream=st)
        A32 = A0.to(torch.float32)
        s32 = e32.init_from_factors(A32, U, S, V, "fp32", m_cap=m0 + T, n_cap=n, stream=st)
        pol = isvd.Policy(kind=isvd.POL_ANGLE, theta_max=1e-3, t_min=1)
        sb = eb.init_from_factors(A32, U, S, V, "bf16rot", m_cap=m0 + T, n_cap=n, policy=pol, stream=st)
        del A32, U, V
        st.synchronize()
        forms = []
        for name, eng, sid, pay in (("fp64", e64, s64, rows), ("fp32_core64", e32, s32, rows32),
                                    ("bf16rot_angle_refresh", eb, sb, rows32)):
            evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(T)]
            st.synchronize()
            w0 = time.perf_counter()
            for t in range(T):
                evs[t][0].record(st)
                eng.append_row(sid, pay[t], stream=st)
                evs[t][1].record(st)
            st.synchronize()
            wall = time.perf_counter() - w0
            lat = [a.elapsed_time(b) for a, b in evs]
            met = eng.metrics(sid, stream=st)
            forms.append((name, eng, sid, {"updates_per_s": round(T / wall, 1),
                                           "p50_update_ms": round(pctl(lat, 50), 4),
                                           "p99_update_ms": round(pctl(lat, 99), 4),
                                           "refreshes": int(met["n_refresh"])}))
            log("%s %s: %.1f appends/s, p50 %.3f ms, p99 %.3f ms, %d refreshes"
                % (log_prefix, name, T / wall, pctl(lat, 50), pctl(lat, 99), met["n_refresh"]))
        ref = e64.factors(s64, stream=st)
        for name, eng, sid, rec in forms:
            if name != "fp64":
                c = compare(eng.factors(sid, stream=st), ref)
                rec["error_vs_fp64"] = {q: float("%.3g" % c[q]) for q in
                                        ("recon", "sigma", "angle_U", "angle_V", "angle_U_full", "ortho_U")}
                rec["error_vs_fp64"]["angle_scope"] = int(c["angle_scope"])
            out[name] = rec
        out["init_ms_fp64"] = round(init_ms, 1)
        out["init_refresh_rounds"] = int(met0["refresh_rounds"])
    del A0, rows, rows32
    torch.cuda.synchronize()
    return out


def sweep_main(args):
    """Precision sweep run (one JSON line)."""
    import torch
    from paper_2605_24514_amd import isvd
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    res = precision_sweep(args, torch, isvd, args.sweep_appends)
    out = {"metric": "precision sweep: appends/s and error against FP64 per form", "value":
           res["fp32_core64"]["updates_per_s"], "unit": "updates/s", "n_gpus": 1, "steps": args.sweep_appends,
           "warmup": 0, "higher_is_better": True, "dtype": "f32", "data": "synthetic",
           "config": {"workload": res["workload"]}, "forms": res}
    print(json.dumps(out), flush=True)


C1_SEED = 1


def c0_main(args):
    """The 500 x 50 FP64 stream (5 factors, seed 0): 1000 row appends and 200
    rank-1 updates in the seeded interleaving, k = 10, periodic refresh every
    200 updates (six refreshes).  Per-update latency of the immediate-mode
    calls (one synchronised update at a time) against the same updates sent
    as one-request ticks, each form run on its own engine from A_0; prints
    one JSON line."""
    import torch
    from paper_2605_24514_amd import isvd
    from synth import FactorStream, event_schedule_c0, ROW
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    fs = FactorStream(seed=0, stream=0, n0=50, K=5)
    A0 = fs.initial(500)
    events = fs.materialize(event_schedule_c0(0, 0, 1000, 200), m0=500)
    st = torch.cuda.Stream()
    pays = [torch.tensor(ev.vec, dtype=torch.float64, device="cuda") if ev.kind == ROW else None for ev in events]
    torch.cuda.synchronize()
    pol = isvd.Policy(kind=isvd.POL_PERIODIC, period=200)
    forms = {}
    for form in ("immediate", "tick"):
        with isvd.Engine() as eng:
            sid = eng.init(A0, 10, "fp64", m_cap=1500, n_cap=50, oversample=64, policy=pol, stream=st)
            st.synchronize()
            lat, refresh_lat = [], []
            w0 = time.perf_counter()
            for ev, pay in zip(events, pays):
                a = time.perf_counter()
                if form == "immediate":
                    if ev.kind == ROW:
                        eng.append_row(sid, pay, stream=st)
                    else:
                        eng.update_entry(sid, ev.i, ev.j, ev.delta, stream=st)
                else:
                    if ev.kind == ROW:
                        eng.tick([(sid, isvd.ROW, pay)], stream=st)
                    else:
                        eng.tick([(sid, isvd.ENTRY, (ev.i, ev.j, ev.delta))], stream=st)
                st.synchronize()
                (refresh_lat if ev.t % 200 == 0 else lat).append((time.perf_counter() - a) * 1e3)
            wall = time.perf_counter() - w0
            met = eng.metrics(sid, stream=st)
            forms[form] = {"updates_per_s": round(len(events) / wall, 1), "p50_update_ms": round(pctl(lat, 50), 4),
                           "p99_update_ms": round(pctl(lat, 99), 4),
                           "refresh_tick_ms_mean": round(float(np.mean(refresh_lat)), 3),
                           "refreshes": int(met["n_refresh"])}
        log("C0 %s: %s" % (form, forms[form]))
    out = {"metric": "per-update latency of one FP64 stream, immediate calls against one-request ticks",
           "value": forms["immediate"]["updates_per_s"], "unit": "updates/s", "n_gpus": 1,
           "steps": len(events), "warmup": 0, "higher_is_better": True, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "one stream, A_0 500 x 50 (5 factors, seed 0), 1000 row appends + 200 "
                                  "rank-1 updates interleaved, k = 10, periodic refresh every 200"},
           "forms": forms,
           "note": "host-timed, a synchronisation after every update; parity with the oracle (<= 1e-10 at every "
                   "25th update, A bitwise) is tests/test_gpu_update.py"}
    print(json.dumps(out))


def c1_main(args):
    """The single large stream at spec: A_0 100000 x 2000 (20 factors), k = 64,
    FP32 storage with the FP64 core, T i.i.d. ticks of 80 % row appends, 10 %
    column appends and 10 % entry updates, and the error-threshold refresh
    (eq. error-refresh-rule) with gamma = 1.05 checked every 100 ticks (each
    check: E_inc from one residual pass over A, E_opt from the Gram-form
    TruncatedSVD of A_t, committed as the refresh when the policy fires).
    Immediate-mode updates (one stream); prints one JSON line with updates/s,
    per-update p50 / p99, the checks' and refreshes' counts and times, and the
    final frob_ratio and orthogonality."""
    import torch
    from paper_2605_24514_amd import isvd
    from synth import device as sdev, uniforms, FactorStream
    from synth.factor_model import P_EVENT, P_DELTA, normals
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    m0, n0, nf, k, T = 100_000, 2000, 20, 64, args.c1_ticks
    st = torch.cuda.Stream()
    A0 = torch.empty((m0, n0), dtype=torch.float32, device="cuda")
    sdev.rows_into(A0, 0, m0, n0, C1_SEED, 0, nf)
    # the schedule (i.i.d. kinds, entry positions and deltas from their own counters)
    u = uniforms(C1_SEED, 0, P_EVENT, np.arange(1, T + 1), 4)
    kinds = np.where(u[:, 0] < 0.8, 0, np.where(u[:, 0] < 0.9, 1, 2))
    nrow, ncol = int(np.sum(kinds == 0)), int(np.sum(kinds == 1))
    # factor-model payloads: row t of the panel over all the columns it may
    # meet (the first n_t entries are the row of the n_t-column panel), and
    # new asset columns y = F b_j + 0.1 eps over all rows they may meet, with
    # the loadings b_j of the column's index and the panel's own factors F
    fs = FactorStream(seed=C1_SEED, stream=0, n0=n0, K=nf)
    rows = torch.empty((max(nrow, 1), n0 + ncol), dtype=torch.float32, device="cuda")
    sdev.rows_into(rows, m0, max(nrow, 1), n0 + ncol, C1_SEED, 0, nf)
    F = torch.tensor(fs.factors(0, m0 + nrow), dtype=torch.float64, device="cuda")
    Bc = torch.tensor(fs.loadings(n0, n0 + max(ncol, 1)), dtype=torch.float64, device="cuda")
    g = torch.Generator(device="cuda").manual_seed(C1_SEED)
    cols = (F @ Bc.T).T.contiguous()
    cols += 0.1 * torch.randn(cols.shape, generator=g, device="cuda", dtype=torch.float64)
    cols = cols.to(torch.float32)
    del F, Bc
    deltas = 0.5 * normals(C1_SEED, 0, P_DELTA, np.arange(1, T + 1), 1)[:, 0]
    torch.cuda.synchronize()
    pol = isvd.Policy(kind=isvd.POL_ERROR, gamma=1.05, check_every=100, t_min=100)
    with isvd.Engine() as eng:
        t0 = time.perf_counter()
        sid = eng.init(A0, k, "fp32", m_cap=m0 + nrow, n_cap=n0 + ncol, policy=pol, stream=st)
        st.synchronize()
        init_s = time.perf_counter() - t0
        del A0
        m, n = m0, n0
        ri = ci = 0
        lat = []
        w0 = time.perf_counter()
        for t in range(T):
            a = time.perf_counter()
            if kinds[t] == 0:
                eng.append_row(sid, rows[ri, :n], stream=st)
                ri += 1
                m += 1
            elif kinds[t] == 1:
                eng.append_col(sid, cols[ci, :m], stream=st)
                ci += 1
                n += 1
            else:
                i = min(int(u[t, 2] * m), m - 1)
                j = min(int(u[t, 3] * n), n - 1)
                eng.update_entry(sid, i, j, float(deltas[t]), stream=st)
            if (t + 1) % 100 == 0 or t + 1 == T:
                st.synchronize()   # latency of a check tick includes its check
            lat.append((time.perf_counter() - a) * 1e3)
        st.synchronize()
        wall = time.perf_counter() - w0
        met = eng.metrics(sid, exact=True, stream=st)
    out = {"metric": "updates/s of one large stream with the error-threshold refresh", "value": round(T / wall, 1),
           "unit": "updates/s", "n_gpus": 1, "steps": T, "warmup": 0, "higher_is_better": True, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": "one stream, A_0 100000 x 2000 (20 factors), k = 64, %d i.i.d. ticks 80/10/10 "
                                  "row / column / entry, error-threshold refresh gamma = 1.05 every 100 ticks" % T},
           "p50_update_ms": round(pctl(lat, 50), 4), "p99_update_ms": round(pctl(lat, 99), 4),
           "max_update_ms": round(max(lat), 3), "refreshes": int(met["n_refresh"]),
           "checks": T // 100, "final_frob_ratio": met["frob_ratio"], "ortho_U": met["ortho_U"],
           "ortho_V": met["ortho_V"], "init_s": round(init_s, 2), "final_shape": [m, n],
           "note": "host-timed per update, a synchronisation at every check tick; the refresh decisions in this "
                   "regime are checked against the oracle at 6000 x 400 in tests/test_gpu_c1_policy.py"}
    print(json.dumps(out), flush=True)


def finance_main(args):
    """Finance readout (Section 5): a 60-asset returns stream (the paper's ETF
    universe size, synthetic five-factor returns in place of its price data),
    k = 5, FP32 storage.  Each streamed day: causal de-meaning of the day's
    returns on the GPU, the row append, and the equal-weight portfolio's
    volatility from the factors.  Also times the exact readout (volatility,
    risk and covariance errors against TruncatedSVD(A_t, k)) and the
    covariance kernel on a 2000-asset, k = 64 stream."""
    import torch
    from paper_2605_24514_amd import isvd
    from synth import FactorStream
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    n, k, t0, days = 60, 5, 1000, 640
    fs = FactorStream(seed=SEED, stream=0, n0=n, K=5)
    drift = 0.0005 * np.random.default_rng(SEED).standard_normal(n)
    r = torch.tensor(0.01 * fs.initial(t0 + days) + drift, dtype=torch.float32, device="cuda")
    w = np.full(n, 1.0 / n)
    st = torch.cuda.current_stream()
    with isvd.Engine() as eng:
        mu = torch.zeros(n, dtype=torch.float64, device="cuda")
        R0 = isvd.causal_center(r[:t0], mu, 0)
        sid = eng.init(R0, k, "fp32", m_cap=t0 + days, n_cap=n, oversample=64)
        eng.sync()
        x = torch.empty(n, dtype=torch.float32, device="cuda")
        lat = []
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        for d in range(days):
            a = time.perf_counter()
            isvd.causal_center(r[t0 + d], mu, t0 + d, out=x)
            eng.append_row(sid, x)
            vol = eng.risk(sid, w)["vol_inc"]
            lat.append((time.perf_counter() - a) * 1e3)
        wall = time.perf_counter() - w0
        ex = []
        for _ in range(max(3, args.steps // 10)):
            a = time.perf_counter()
            res = eng.risk(sid, w, exact=True)
            ex.append((time.perf_counter() - a) * 1e3)
    # covariance kernel at a 2000-asset universe
    nb, kb, mb = 2000, 64, 20000
    from synth import device as sdev
    Ab = torch.empty((mb, nb), dtype=torch.float32, device="cuda")
    sdev.rows_into(Ab, 0, mb, nb, SEED, 1, 20)
    with isvd.Engine() as eng:
        sidb = eng.init(Ab, kb, "fp32", refresh_iters=1)
        C = eng.covariance(sidb)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 20
        e0.record(st)
        for _ in range(reps):
            eng.covariance(sidb, out=C, stream=st)
        e1.record(st)
        e1.synchronize()
        cov_ms = e0.elapsed_time(e1) / reps
    cov_bytes = 8.0 * nb * nb + 4.0 * nb * kb
    cov_tf = 2.0 * nb * nb * kb / (cov_ms * 1e-3) / 1e12
    out = {"metric": "finance readout days/s (causal de-meaning + row append + portfolio volatility per day)",
           "value": round(days / wall, 1), "unit": "days/s", "n_gpus": 1, "steps": days, "warmup": 0,
           "higher_is_better": True, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "one returns stream of 60 assets (five-factor returns, daily scale, per-asset drift), "
                                  "1000 initial days then 640 streamed, k = 5, FP32 storage, FP64 core; equal-weight "
                                  "portfolio"},
           "day_ms_p50": round(pctl(lat, 50), 4), "day_ms_p99": round(pctl(lat, 99), 4),
           "last_vol_inc": vol,
           "exact_readout_ms_p50": round(pctl(ex, 50), 3),
           "exact_readout": {k2: (None if v != v else v) for k2, v in res.items()},
           "covariance_kernel": {"workload": "2000 assets, k = 64, 20000 rows, FP32 factors -> FP64 2000 x 2000",
                                 "ms": round(cov_ms, 4),
                                 "roofline": {"bound": "alu", "achieved": round(cov_tf, 2), "peak": FP64_PEAK_TFLOPS,
                                              "unit": "TFLOP/s", "frac": round(cov_tf / FP64_PEAK_TFLOPS, 4),
                                              "flops": 2.0 * nb * nb * kb,
                                              "hbm_gbs": round(cov_bytes / (cov_ms * 1e-3) / 1e9, 1)}}}
    print(json.dumps(out), flush=True)


def parse_args(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--streams", type=int, default=512)
    ap.add_argument("--refresh-iters", type=int, default=None,
                    help="subspace iterations of the A-form refresh (default: the Gram form with its stopping "
                         "rule in --refresh mode, 2 for the initial SVDs of the tick workload)")
    ap.add_argument("--compare-streams", type=int, default=32)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-pipeline", action="store_true", help="join every tick's U rotations before the next tick")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one plain 1 GiB device copy (reference for hardware byte counters)")
    ap.add_argument("--serve", action="store_true", help="run the serving loop instead of the batched tick")
    ap.add_argument("--refresh", action="store_true", help="time the refresh of one 100000 x 2000 stream instead")
    ap.add_argument("--finance", action="store_true", help="time the finance readout of a 60-asset returns stream")
    ap.add_argument("--c1", action="store_true",
                    help="run the single large stream (100000 x 2000, k = 64, error-threshold refresh) instead")
    ap.add_argument("--c1-ticks", type=int, default=10000)
    ap.add_argument("--c0", action="store_true",
                    help="per-update latency of the 500 x 50 FP64 stream: immediate calls against one-request ticks")
    ap.add_argument("--sweep", action="store_true",
                    help="run the precision sweep (1,000,000 x 512, k = 128) instead")
    ap.add_argument("--sweep-appends", type=int, default=5000)
    ap.add_argument("--sweep-default", type=int, default=300,
                    help="row appends of the shortened precision sweep added to the default line (0: none)")
    ap.add_argument("--explicit-u", action="store_true",
                    help="rotate U on every row append (no deferred U = U0 W)")
    ap.add_argument("--no-graphs", action="store_true", help="launch every tick from the host (no captured graph)")
    ap.add_argument("--no-explicit", action="store_true",
                    help="skip the explicit-U comparison that follows the deferred headline")
    ap.add_argument("--serve-streams", type=int, default=1024)
    ap.add_argument("--serve-lifetime", type=int, default=200)
    ap.add_argument("--serve-rate", type=float, default=200000.0)
    ap.add_argument("--serve-budget-gb", type=float, default=50.0)
    ap.add_argument("--serve-default", type=int, default=4096,
                    help="streams of the serving run added to the default line (0: none)")
    ap.add_argument("--serve-cache-gb", type=float, default=24.0,
                    help="device blocks of released streams kept for later admissions")
    ap.add_argument("--serve-window", type=int, default=32,
                    help="streams waiting for admission with their A0 in memory")
    return ap.parse_args(argv)


def main():
    args = parse_args()
    if args.serve and args.gpus == 1:
        serve_main(args)
        return
    if args.refresh and args.gpus == 1:
        refresh_main(args)
        return
    if args.finance and args.gpus == 1:
        finance_main(args)
        return
    if args.sweep and args.gpus == 1:
        sweep_main(args)
        return
    if args.c1 and args.gpus == 1:
        c1_main(args)
        return
    if args.c0 and args.gpus == 1:
        c0_main(args)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the streams are independent and would shard by stream across "
              "GPUs with no communication; runs on %d GPUs are not implemented" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2605_24514_amd import isvd
    from synth import device as sdev
    from tests.parity import compare

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev_stream = torch.cuda.Stream()
    sp = dev_stream.cuda_stream
    params = stream_params(args.streams)
    W, K = args.warmup, args.steps
    T = W + K
    # the explicit-U comparison runs W + K more ticks (plus a profiled pass)
    # on the same streams after the chosen form, with fresh rows
    TX = 0 if (args.explicit_u or args.no_explicit) else W + K
    T_pay = T + TX
    log("streams %d, ticks %d (+%d warmup)" % (len(params), K, W))

    eng64 = isvd.Engine()
    eng32 = isvd.Engine()
    sid64, sid32 = [], []
    t_init = time.perf_counter()
    mmax = max(p[0] for p in params)
    nmax = max(p[1] for p in params)
    tmp = torch.empty(mmax * nmax, dtype=torch.float64, device="cuda")
    with torch.cuda.stream(dev_stream):
        for s, (m0, n0, k) in enumerate(params):
            A0 = tmp[:m0 * n0].view(m0, n0)
            sdev.rows_into(A0, 0, m0, n0, SEED, s, K_FACTORS, hip_stream=sp)
            sid64.append(eng64.init(A0, k, "fp64", m_cap=m0 + T, n_cap=n0, refresh_iters=2 if args.refresh_iters is None else args.refresh_iters,
                                    stream=dev_stream))
            U, S, V = eng64.factors(sid64[-1], stream=dev_stream)
            sid32.append(eng32.init_from_factors(A0, U, S, V, "fp32", m_cap=m0 + T_pay + 2 * PROF_TICKS + 8, n_cap=n0,
                                                 stream=dev_stream))
            if s % 64 == 63:
                log("  init %d/%d streams (%.1fs)" % (s + 1, len(params), time.perf_counter() - t_init))
    del tmp
    torch.cuda.synchronize()
    init_s = time.perf_counter() - t_init
    # row payloads for every tick, resident in HBM before timing
    pay32, pay64 = [], []
    for s, (m0, n0, k) in enumerate(params):
        p64 = torch.empty((T_pay, n0), dtype=torch.float64, device="cuda")
        sdev.rows_into(p64, m0, T_pay, n0, SEED, s, K_FACTORS)
        pay64.append(p64)
        pay32.append(p64.to(torch.float32))
    torch.cuda.synchronize()
    reqs = [isvd.Engine.tick_requests([(sid32[s], isvd.ROW, pay32[s][t]) for s in range(len(params))])
            for t in range(T_pay)]
    log("init %.1fs; payloads ready" % init_s)

    # ---------------------------------------------------- chosen form: batched FP32
    eng32.set_pipelining(not args.no_pipeline)
    # Brand's deferred left basis U = U0 W for the row appends (explicit U
    # rotation every m / (8 k) appends, staggered over the streams)
    eng32.set_deferred_u(not args.explicit_u, stream=dev_stream)
    # deferred-U row-append ticks replay a captured HIP graph (captured during the warm-up)
    eng32.set_tick_graphs(not args.explicit_u and not args.no_graphs)
    tune = eng32.autotune(stream=dev_stream)
    log("rotation autotune (bucket: variant): %s" % {kc: v for kc, (v, _) in tune.items()})
    rot_lane = torch.cuda.ExternalStream(eng32.rotation_stream())

    def timed_ticks(first, deferred_form):
        """W warm-up and K timed ticks of requests reqs[first:]; per tick from
        an event on the caller's stream before it to events on both streams a
        tick can end on (the caller's stream; the rotation lane, where a
        pipelined explicit-U tick leaves its U rotations)."""
        for t in range(W):
            eng32.tick_raw(reqs[first + t], stream=dev_stream)
        eng32.sync(stream=dev_stream)
        torch.cuda.synchronize()
        evs = [tuple(torch.cuda.Event(enable_timing=True) for _ in range(3)) for _ in range(K)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        host_s = 0.0
        for q in range(K):
            evs[q][0].record(dev_stream)
            h0 = time.perf_counter()
            eng32.tick_raw(reqs[first + W + q], stream=dev_stream)
            host_s += time.perf_counter() - h0
            evs[q][1].record(dev_stream)
            evs[q][2].record(rot_lane)
        eng32.sync(stream=dev_stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        tick_ms = [max(a.elapsed_time(b), a.elapsed_time(c)) for a, b, c in evs]
        return wall, tick_ms, host_s / K

    wall, tick_ms, host_per_tick = timed_ticks(0, not args.explicit_u)
    value = len(params) * K / wall
    log("batched FP32: %.0f updates/s, tick latency p50 %.3f ms p99 %.3f ms; host %.3f ms per tick call"
        % (value, pctl(tick_ms, 50), pctl(tick_ms, 99), host_per_tick * 1e3))

    # ------------------------------------------------------- plain form: FP64, one stream per launch
    plain = None
    if not args.no_plain:
        ptick = []
        with torch.cuda.stream(dev_stream):
            for t in range(T):
                torch.cuda.synchronize()
                a = time.perf_counter()
                for s in range(len(params)):
                    eng64.append_row(sid64[s], pay64[s][t], stream=dev_stream)
                torch.cuda.synchronize()
                ptick.append((time.perf_counter() - a) * 1e3)
        pt = ptick[W:]
        plain = {"value": len(params) * len(pt) / (np.sum(pt) * 1e-3), "unit": "updates/s",
                 "p50_tick_ms": pctl(pt, 50), "p99_tick_ms": pctl(pt, 99), "dtype": "f64",
                 "form": "one stream per launch sequence, FP64, no batching"}
        log("plain FP64: %.0f updates/s, tick p50 %.2f ms p99 %.2f ms" % (plain["value"], plain["p50_tick_ms"],
                                                                           plain["p99_tick_ms"]))

    # ----------------------------------------------- accuracy of the FP32 result against FP64
    err = None
    if plain is not None and args.compare_streams > 0:
        pick = np.linspace(0, len(params) - 1, min(args.compare_streams, len(params))).astype(int)
        worst = {"recon": 0.0, "sigma": 0.0, "angle_U": 0.0, "angle_V": 0.0, "ortho_U": 0.0}
        for s in pick:
            c = compare(eng32.factors(sid32[s]), eng64.factors(sid64[s]))
            for key in worst:
                worst[key] = max(worst[key], c[key])
        err = {k: float("%.3g" % v) for k, v in worst.items()}
        err["streams_compared"] = int(len(pick))
        log("FP32 vs FP64 after %d ticks: %s" % (T, err))

    names = {0: "k_proj (pass 1)", 1: "k_proj (pass 2)", 2: "k_core", 3: "k_rotate_mfma_t (U)",
             4: "k_rotate_mfma_t (V)"}
    bucket = lambda k: 8 if k <= 8 else 16 if k <= 16 else 32 if k <= 32 else 64 if k <= 64 else 128

    def bound_of(byts, flops, flops_peak_tf, ms):
        """Roofline of one launch by the max(bytes / BW, flops / peak) rule."""
        t_b = byts / (HBM_PEAK_GBS * 1e9)
        t_f = flops / (flops_peak_tf * 1e12)
        if t_b >= t_f:
            ach = byts / (ms * 1e-3) / 1e9
            return {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(t_b / (ms * 1e-3), 5)}
        ach = flops / (ms * 1e-3) / 1e12
        return {"bound": "mfma", "achieved": round(ach, 3), "peak": flops_peak_tf, "unit": "TFLOP/s",
                "frac": round(t_f / (ms * 1e-3), 5)}

    def profile_pass(first, deferred_form, m_off):
        """PROF_TICKS more ticks with per-launch HIP events (requests
        reqs[first + q % K]); the dominant launch's roofline and the mean time
        per tick of each phase.  m_off: rows appended before the pass."""
        eng32.profile(True)
        for q in range(PROF_TICKS):
            eng32.tick_raw(reqs[first + q % K], stream=dev_stream)
        eng32.sync(stream=dev_stream)
        torch.cuda.synchronize()
        eng32.profile(False)
        prof = eng32.profile_read()
        by_launch = {}
        for r in prof:
            by_launch.setdefault((r["phase"], r["kc"]), []).append(r["ms"])
        phase_ms = {}
        for (ph, kc), v in by_launch.items():
            phase_ms.setdefault(ph, 0.0)
            phase_ms[ph] += float(np.sum(v)) / PROF_TICKS
        mid = m_off + (PROF_TICKS - 1) / 2.0
        if not deferred_form:
            # dominant kernel: the U rotation of the widest bucket (HBM-bound:
            # 16 flop/B at k = 64 against the FP32 balance of 19.7)
            kdom = max(kc for (ph, kc) in by_launch if ph == 3)
            dom_ms = float(np.mean(by_launch[(3, kdom)]))
            sel = [(m0, n0, k) for (m0, n0, k) in params if bucket(k) == kdom]
            dom_bytes = sum(rot_u_bytes(m0 + mid, k, 4) for (m0, n0, k) in sel)
            dom_flops = sum(2.0 * (m0 + mid) * k * k for (m0, n0, k) in sel)
            roof = bound_of(dom_bytes, dom_flops, FP32_PEAK_TFLOPS, dom_ms)
            dom_ratio = (recorded_traffic_ratio(PMC_ROTATE, "traffic_over_algorithmic_variant_%d" % tune[kdom][0])
                         if kdom in tune else None)
            roof.update({"traffic": (int(dom_ratio * dom_bytes) if dom_ratio is not None and kdom == 64 else None),
                         "traffic_note": "HBM bytes per launch: rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated, "
                                         "ratio to algorithmic bytes from profiles/rotate_u_kc64_tick512_pmc.md",
                         "kernel": "k_rotate_mfma_t<%d> (U rotation, variant %d)"
                                   % (kdom, tune[kdom][0] if kdom in tune else -1),
                         "launch_ms": round(dom_ms, 4), "bytes_per_launch": int(dom_bytes),
                         "flops_per_launch": dom_flops})
            return roof, phase_ms
        # deferred U: the longest launch of the tick (bucket 0: a merged
        # launch over every bucket)
        (ph, kdom) = max(by_launch, key=lambda key: float(np.mean(by_launch[key])))
        dom_ms = float(np.mean(by_launch[(ph, kdom)]))
        sel = [(m0, n0, k) for (m0, n0, k) in params if kdom == 0 or bucket(k) == kdom]
        what = "all buckets" if kdom == 0 else "bucket %d" % kdom
        if ph == 2:
            # the append core: its W update (W A and A^T W^-1, 4 k^3 flops per
            # append on the FP64 matrix cores) and its bytes (W, W^-1 read and
            # written, V's rotation written)
            flops = sum(4.0 * k ** 3 for (m0, n0, k) in sel)
            cbytes = sum(core_bytes(k) for (m0, n0, k) in sel)
            roof = bound_of(cbytes, flops, FP64_PEAK_TFLOPS, dom_ms)
            cratio = recorded_traffic_ratio(PMC_CORE, "traffic_over_algorithmic") if kdom == 0 else None
            roof.update({"traffic": int(cratio * cbytes) if cratio is not None else None,
                         "traffic_note": "HBM bytes per launch: rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated, "
                                         "ratio to algorithmic bytes from profiles/core_chain_tick512_pmc.md",
                         "kernel": ("k_core_chain (append cores of every bucket: secular SVD + deferred-U update, FP64)"
                                    if kdom == 0 else
                                    "k_core<float, %d> (append core: secular SVD + deferred-U update, FP64)" % kdom),
                         "launch_ms": round(dom_ms, 4), "flops_per_launch": flops, "bytes_per_launch": int(cbytes),
                         "note": "one workgroup per stream; bound by max(bytes / 8 TB/s, flops / FP64 matrix peak)"})
            return roof, phase_ms
        if ph == 4:
            byts = sum(4.0 * 2 * n0 * k + 8.0 * n0 for (m0, n0, k) in sel)
        elif ph == 3:
            byts = sum(rot_u_bytes(m0 + mid, k, 4) / max(1, min(256, int(m0 + mid) // (8 * k)))
                       for (m0, n0, k) in sel)
        else:
            byts = sum(4.0 * n0 * k + 4.0 * n0 for (m0, n0, k) in sel)
        roof = bound_of(byts, 0.0, FP32_PEAK_TFLOPS, dom_ms)
        chain_names = {0: "k_proj_chain<1>", 1: "k_proj_chain<2>", 3: "k_rotu_chain (U)",
                       4: "k_rotv_chain (V and the U plan)"}
        roof.update({"traffic": None, "kernel": "%s, %s" % (chain_names[ph] if kdom == 0 else names[ph], what),
                     "launch_ms": round(dom_ms, 4),
                     "bytes_per_launch": int(byts)})
        return roof, phase_ms

    # the host's own cost per tick call, with the device busy so that no call
    # waits for it: a bounded spin kernel first, then 6 ticks issued behind it
    # (re-using already-applied payloads: only the host side is of interest)
    torch.cuda.synchronize()
    with torch.cuda.stream(dev_stream):
        torch.cuda._sleep(200_000_000)
    h0 = time.perf_counter()
    for q in range(6):
        eng32.tick_raw(reqs[(W + q) % len(reqs)], stream=dev_stream)
    host_unthrottled = (time.perf_counter() - h0) / 6
    eng32.sync(stream=dev_stream)
    torch.cuda.synchronize()
    log("host cost per tick call with the device busy: %.3f ms" % (host_unthrottled * 1e3))
    deferred = not args.explicit_u
    roofline, phase_ms = profile_pass(W, deferred, W + K + 6)
    mid_all = W + (K - 1) / 2.0
    all_tick_bytes = sum(tick_bytes(m0 + mid_all, n0, k, 4, deferred) for (m0, n0, k) in params)

    # ---------------------------------------- the same streams with U rotated on every append
    explicit = None
    if TX:
        eng32.set_tick_graphs(False)
        eng32.set_deferred_u(False, stream=dev_stream)
        xwall, xtick_ms, xhost = timed_ticks(T, False)
        xvalue = len(params) * K / xwall
        base = T + PROF_TICKS
        xroof, xphase = profile_pass(T + W, False, base + W + K)
        xmid = base + W + (K - 1) / 2.0
        xbytes = sum(tick_bytes(m0 + xmid, n0, k, 4, False) for (m0, n0, k) in params)
        explicit = {"value": round(xvalue, 1), "unit": "updates/s", "ms_per_step": round(xwall / K * 1e3, 4),
                    "p50_tick_ms": round(pctl(xtick_ms, 50), 4), "p99_tick_ms": round(pctl(xtick_ms, 99), 4),
                    "host_ms_per_tick": round(xhost * 1e3, 4),
                    "tick_algorithmic_GBps": round(xbytes / (xwall / K) / 1e9, 1),
                    "phase_ms_per_tick": {["proj1", "proj2", "core", "rotate_U", "rotate_V"][p]: round(v, 4)
                                          for p, v in sorted(xphase.items())},
                    "roofline": xroof,
                    "form": "Alg. A1 as written: U = [[U, 0], [0, 1]] U_K on every append, same streams, "
                            "measured after the deferred form in the same run"}
        log("explicit U: %.0f updates/s, tick p50 %.3f ms p99 %.3f ms; U rotation %s"
            % (xvalue, pctl(xtick_ms, 50), pctl(xtick_ms, 99), xroof))
    tick_gbs = all_tick_bytes / (wall / K) / 1e9
    if args.calibrate_copy:
        src = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy: %d bytes read, %d bytes written" % (src.numel() * 4, dst.numel() * 4))
        del src, dst

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(params, args.cpu_seconds, torch)
        log("cpu oracle: %.1f updates/s on %d threads" % (cpu["value"], cpu["cores"]))

    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": round(wall / K * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "batched row-append tick over %d factor-model streams: n~U{50..2000}, "
                               "m~U{1000..50000}, k~U{8,16,32,64}, 5 factors; FP32 storage, FP64 core"
                               % len(params),
                   "streams": len(params), "rows_total": int(sum(p[0] for p in params)),
                   "cols_total": int(sum(p[1] for p in params)),
                   "tick": ("one replay of a captured HIP graph per tick" if not (args.explicit_u or args.no_graphs)
                            else "launched from the host"),
                   "left_basis": ("explicit: U rotated on every append" if args.explicit_u else
                                  "deferred U = U0 W (Brand), explicit rotation every m/(8k) appends per stream")},
        "p50_tick_ms": round(pctl(tick_ms, 50), 4),
        "p99_tick_ms": round(pctl(tick_ms, 99), 4),
        "host_ms_per_tick": round(host_per_tick * 1e3, 4),
        "host_ms_per_tick_device_busy": round(host_unthrottled * 1e3, 4),
        "plain_fp64": plain,
        "speedup_vs_plain": round(value / plain["value"], 2) if plain else None,
        "p99_vs_plain": round(plain["p99_tick_ms"] / pctl(tick_ms, 99), 2) if plain else None,
        "error_vs_fp64": err,
        "tick_algorithmic_GBps": round(tick_gbs, 1),
        "phase_ms_per_tick": {["proj1", "proj2", "core", "rotate_U", "rotate_V"][p]: round(v, 4)
                              for p, v in sorted(phase_ms.items())},
        "roofline": roofline,
        "explicit_u": explicit,
        "speedup_vs_plain_explicit_u": round(explicit["value"] / plain["value"], 2) if (plain and explicit) else None,
        "cpu_baseline": cpu,
        "init_s": round(init_s, 1),
    }
    eng32.close()
    eng64.close()
    del pay32, pay64, reqs
    torch.cuda.synchronize()
    if args.sweep_default > 0:
        # the precision sweep (1,000,000 x 512, k = 128), shortened; --sweep runs all 5000 appends
        out["precision_sweep"] = precision_sweep(args, torch, isvd, args.sweep_default)
    if args.serve_default > 0:
        # the serving workload at full size: 4096 streams, 200 GB, 200 k requests/s
        torch.cuda.empty_cache()
        sargs = argparse.Namespace(**vars(args))
        sargs.serve_streams, sargs.serve_budget_gb, sargs.serve_rate = args.serve_default, 200.0, 200000.0
        sargs.serve_lifetime = 200
        srec = serve_run(sargs)
        out["serving"] = {q: srec[q] for q in ("metric", "value", "unit", "config", "requests", "completed_ok",
                                               "wall_s", "latency_ms", "after_admission_ms", "admission_wait_ms",
                                               "server")}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
