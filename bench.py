"""Benchmark: full-pivot Gauss-Jordan inversion on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--extras]

One step = one whole inversion (every kernel of the path: copy-in, n
elimination steps with the fused pivot search, pivot/determinant record and
depivoting gather) of the headline workload: a single 4096 x 4096 FP64 matrix
with entries iid U[-1,1] plus 4 on the diagonal, already resident in HBM.

Prints ONE JSON line.  ``value`` is inversions per second; ``roofline`` is
for the dominant kernel (the per-step sweep), whose algorithmic traffic is
16 n^2 bytes per launch (each element of the n x n working array read once
and written once); its average duration comes from HIP events recorded
around the step launches on the library's stream.  ``cpu_baseline`` times the
FP64 oracle on the host over a bounded sample of the same input.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
PROFILES = os.path.join(ROOT, "profiles")


def _kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("big.hip", "gj_device.h"):
        with open(os.path.join(ROOT, "paper_1401_7962_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _traffic_per_launch(kernel_key: str):
    """HBM bytes per launch measured with rocprofv3 counters (FETCH_SIZE +
    WRITE_SIZE, scaled by a copy-kernel calibration) and stored under
    profiles/; None when missing or taken on a different kernel source."""
    path = os.path.join(PROFILES, "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        data = json.load(open(path))
        entry = data.get(kernel_key)
        if not entry or entry.get("source_hash") != _kernel_source_hash():
            return None
        return float(entry["bytes_per_launch"])
    except Exception:
        return None


def bench_headline(steps: int, warmup: int, n: int = 4096):
    import torch
    import paper_1401_7962_amd as gj
    from paper_1401_7962_amd import inputs

    dev = torch.device("cuda:0")
    A_h = inputs.single_dominant(n)
    A = torch.from_numpy(A_h).to(dev)
    X = torch.empty_like(A)
    ipiv = torch.empty(n, dtype=torch.int32, device=dev)
    jpiv = torch.empty(n, dtype=torch.int32, device=dev)
    res = torch.empty(gj.RESULT_BYTES, dtype=torch.uint8, device=dev)
    ws = torch.empty(gj.gj_workspace_size(gj.GJ_OP_INVERT, n), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * steps)]
    for e in ev:          # torch creates the underlying hipEvent_t on first record
        e.record(stream)

    for _ in range(warmup):
        gj.gj_invert(A, X, ipiv, jpiv, res, None, ws, stream)
    torch.cuda.synchronize()

    t0 = time.perf_counter()
    for s in range(steps):
        o = gj.make_opts(step_events=(ctypes_ptr(ev[2 * s]), ctypes_ptr(ev[2 * s + 1])))
        gj.gj_invert(A, X, ipiv, jpiv, res, o, ws, stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()

    step_ms = sum(ev[2 * s].elapsed_time(ev[2 * s + 1]) for s in range(steps)) / steps
    r = gj.results_to_dicts(res)[0]
    if r["code"] != gj.GJ_RES_OK:
        raise RuntimeError(f"inversion failed: {r}")
    # residual of the last result, computed on the GPU (independent of the path)
    Ar = A
    Xr = X
    R = Ar @ Xr - torch.eye(n, dtype=torch.float64, device=dev)
    resid = float(torch.linalg.norm(R) / (torch.linalg.norm(Ar) * torch.linalg.norm(Xr)))
    ms_per_inv = (t1 - t0) * 1e3 / steps
    per_launch_ms = step_ms / n
    alg_bytes = 16.0 * n * n
    achieved = alg_bytes / (per_launch_ms * 1e-3) / 1e9
    traffic = _traffic_per_launch(f"gj_big_step_f64_n{n}")
    return {
        "ms_per_inv": ms_per_inv,
        "value": 1e3 / ms_per_inv,
        "step_phase_ms": step_ms,
        "per_launch_us": per_launch_ms * 1e3,
        "achieved_gbs": achieved,
        "traffic": traffic,
        "resid": resid,
        "logabsdet": r["logabsdet"],
        "det_sign": r["det_sign"],
    }


def _events(n, stream):
    import torch
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(n)]
    for e in ev:
        e.record(stream)
    return ev


def bench_latency_small(reps: int = 200):
    """64 x 64 N(0,1) and the 3 x 3 Pascal matrix: microseconds per inversion,
    one inversion per replay of a captured HIP graph."""
    import torch
    import paper_1401_7962_amd as gj
    from paper_1401_7962_amd import inputs
    out = {}
    for name, A_h in (("normal64", inputs.single_normal(64)), ("pascal3", inputs.pascal(3))):
        n = A_h.shape[0]
        A = torch.from_numpy(A_h).cuda()
        X = torch.empty_like(A)
        ip = torch.empty(n, dtype=torch.int32, device="cuda")
        jp = torch.empty_like(ip)
        res = torch.empty(gj.RESULT_BYTES, dtype=torch.uint8, device="cuda")
        ws = torch.empty(256, dtype=torch.uint8, device="cuda")
        gj.gj_invert(A, X, ip, jp, res, None, ws)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            with torch.cuda.graph(g, stream=s):
                gj.gj_invert(A, X, ip, jp, res, None, ws, s)
        torch.cuda.synchronize()
        e0, e1 = _events(2, torch.cuda.current_stream())
        e0.record()
        for _ in range(reps):
            g.replay()
        e1.record()
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / reps
        r = gj.results_to_dicts(res)[0]
        out[name] = {"n": n, "us_per_inversion": round(us, 2), "code": r["code"], "det": r["det"]}
    return out


def _graph_time(call, reps):
    """Capture call(stream) once in a HIP graph, replay it ``reps`` times
    between events; returns the best milliseconds per replay."""
    import torch
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            call(s)
    torch.cuda.synchronize()
    cur = torch.cuda.current_stream()
    e = _events(2 * reps, cur)
    for k in range(reps):
        e[2 * k].record()
        g.replay()
        e[2 * k + 1].record()
    torch.cuda.synchronize()
    best = min(e[2 * k].elapsed_time(e[2 * k + 1]) for k in range(reps))
    del g
    return best


def bench_batch_conditioned(batch: int = 20_000, reps: int = 2):
    """20,000 matrices, n log-uniform in [32,512], U diag(s) V^T with cond
    log-uniform in [1e2,1e8]: FP32 elimination + FP64 Newton-Schulz +
    FP64 determinant for every member, against the plain FP64 elimination
    of the same batch; each timed as a replayed HIP graph."""
    import torch
    import paper_1401_7962_amd as gj
    from paper_1401_7962_amd import inputs
    t0 = time.perf_counter()
    sizes, offs, A, conds = inputs.batch_conditioned(batch, device="cuda")
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t0
    poff = np.zeros(batch, dtype=np.int64)
    poff[1:] = np.cumsum(sizes.astype(np.int64))[:-1]
    out = {"batch": batch, "input_generation_s": round(gen_s, 1)}
    # independent determinant reference on the same bytes: torch's LU slogdet
    lu_ref = np.empty(batch)
    for n in np.unique(sizes):
        n = int(n)
        idx = np.nonzero(sizes == n)[0]
        base = torch.from_numpy(offs[idx]).to(A.device)
        M = A[(base[:, None] + torch.arange(n * n, device=A.device)[None, :])].reshape(len(idx), n, n)
        lu_ref[idx] = torch.linalg.slogdet(M)[1].cpu().numpy()
        del M, base
    Xs = {}
    for name, prec in (("plain_fp64", gj.GJ_PREC_FP64), ("fp32_refined", gj.GJ_PREC_FP32_REFINED)):
        opts = gj.make_opts(precision=prec)
        X = torch.empty_like(A)
        ip = torch.empty(int(sizes.sum()), dtype=torch.int32, device="cuda")
        jp = torch.empty_like(ip)
        res = torch.empty(batch * gj.RESULT_BYTES, dtype=torch.uint8, device="cuda")
        ws = torch.empty(gj.gj_workspace_size(gj.GJ_OP_INVERT_BATCHED, batch, sizes, opts),
                         dtype=torch.uint8, device="cuda")
        gj.gj_invert_batched(sizes, offs, A, X, poff, ip, jp, res, opts, ws)   # uploads the plan
        torch.cuda.synchronize()
        reuse = gj.make_opts(precision=prec, flags=gj.GJ_FLAG_REUSE_PLAN)
        ms = _graph_time(lambda st: gj.gj_invert_batched(sizes, offs, A, X, poff, ip, jp, res, reuse,
                                                          ws, st), reps)
        del ws
        raw = np.frombuffer(res.cpu().numpy().tobytes(), dtype=np.uint8).reshape(batch, gj.RESULT_BYTES)
        codes = raw[:, 0:4].copy().view(np.int32)[:, 0]
        iters = raw[:, 12:16].copy().view(np.int32)[:, 0]
        logdet = raw[:, 40:48].copy().view(np.float64)[:, 0]
        cf = sizes * np.log(conds) / 2.0
        rel_det = np.abs(logdet - cf) / np.abs(cf)
        out[name] = {"ms": round(ms, 2), "inversions_per_s": round(batch / (ms * 1e-3), 1),
                     "codes": {str(c): int((codes == c).sum()) for c in np.unique(codes)},
                     "mean_refine_iters": float(iters.mean()),
                     "max_rel_logdet_err_vs_closed_form": float(rel_det.max()),
                     "max_rel_logdet_err_vs_lu_slogdet": float((np.abs(logdet - lu_ref) / np.abs(lu_ref)).max())}
        Xs[name] = X
    d = torch.linalg.norm(Xs["fp32_refined"] - Xs["plain_fp64"]) / torch.linalg.norm(Xs["plain_fp64"])
    out["refined_vs_plain_rel_frobenius_whole_batch"] = float(d)
    out["speedup_refined_over_plain"] = round(out["plain_fp64"]["ms"] / out["fp32_refined"]["ms"], 3)
    return out


def bench_batch_uneven(batch: int = 100_000, reps: int = 3):
    """100,000 FP64 matrices, n uniform in [8,128], 1% rank n-1: one persistent
    on-chip launch.  Reports inversions/s and FP64 FMA throughput (n^3 FMAs =
    2 n^3 flop per inversion)."""
    import torch
    import paper_1401_7962_amd as gj
    from paper_1401_7962_amd import inputs
    sizes, offs, packed, singular = inputs.batch_uneven(batch)
    A = torch.from_numpy(packed).cuda()
    del packed
    X = torch.empty_like(A)
    poff = np.zeros(batch, dtype=np.int64)
    poff[1:] = np.cumsum(sizes.astype(np.int64))[:-1]
    ip = torch.empty(int(sizes.sum()), dtype=torch.int32, device="cuda")
    jp = torch.empty_like(ip)
    res = torch.empty(batch * gj.RESULT_BYTES, dtype=torch.uint8, device="cuda")
    ws = torch.empty(gj.gj_workspace_size(gj.GJ_OP_INVERT_BATCHED, batch, sizes), dtype=torch.uint8,
                     device="cuda")
    gj.gj_invert_batched(sizes, offs, A, X, poff, ip, jp, res, None, ws)   # uploads the plan
    torch.cuda.synchronize()
    reuse = gj.make_opts(flags=gj.GJ_FLAG_REUSE_PLAN)
    ms = _graph_time(lambda st: gj.gj_invert_batched(sizes, offs, A, X, poff, ip, jp, res, reuse,
                                                      ws, st), reps)
    codes = np.frombuffer(res.cpu().numpy().tobytes(), dtype=np.int32).reshape(batch, 14)[:, 0]
    flops = 2.0 * float((sizes.astype(np.float64) ** 3).sum())
    return {
        "batch": batch,
        "ms": round(ms, 3),
        "inversions_per_s": round(batch / (ms * 1e-3), 1),
        "fp64_tflops": round(flops / (ms * 1e-3) / 1e12, 3),
        "frac_of_fp64_peak": round(flops / (ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS, 4),
        "singular_flagged": int((codes == 1).sum()),
        "singular_planted": int(len(singular)),
        "other_codes": int(((codes != 0) & (codes != 1)).sum()),
    }


def bench_conditioned_8192(n: int = 8192, reps: int = 2):
    """U diag(s) V^T, s log-spaced 1..1e6: plain FP64 elimination against FP32
    elimination + FP64 Newton-Schulz refinement, with the residual of each
    result and the refined result's distance from the plain FP64 result."""
    import torch
    import paper_1401_7962_amd as gj
    from paper_1401_7962_amd import inputs
    t0 = time.perf_counter()
    A = inputs.single_conditioned(n, device="cuda")   # Gaussian draws on the host, QR on the GPU
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t0
    out = {"n": n, "cond": 1e6, "input_generation_s": round(gen_s, 1),
           "closed_form_logabsdet": inputs.closed_form_logdet(n, 1e6)}
    Xs = {}
    stream = torch.cuda.current_stream()
    for name, prec, flags in (("plain_fp64", gj.GJ_PREC_FP64, 0),
                              ("fp32_refined", gj.GJ_PREC_FP32_REFINED, 0),
                              ("fp32_refined_accurate", gj.GJ_PREC_FP32_REFINED, gj.GJ_FLAG_ACCURATE)):
        opts = gj.make_opts(precision=prec, flags=flags)
        X = torch.empty_like(A)
        ip = torch.empty(n, dtype=torch.int32, device="cuda")
        jp = torch.empty_like(ip)
        res = torch.empty(gj.RESULT_BYTES, dtype=torch.uint8, device="cuda")
        ws = torch.empty(gj.gj_workspace_size(gj.GJ_OP_INVERT, n, None, opts), dtype=torch.uint8,
                         device="cuda")
        gj.gj_invert(A, X, ip, jp, res, opts, ws)
        torch.cuda.synchronize()
        e = _events(2 * reps, stream)
        for k in range(reps):
            e[2 * k].record()
            gj.gj_invert(A, X, ip, jp, res, opts, ws)
            e[2 * k + 1].record()
        torch.cuda.synchronize()
        ms = min(e[2 * k].elapsed_time(e[2 * k + 1]) for k in range(reps))
        r = gj.results_to_dicts(res)[0]
        del ws
        R = gj.gj_dgemm(A, X, gamma=1.0, alpha=-1.0)
        resid = float(torch.linalg.norm(R) / (torch.linalg.norm(A) * torch.linalg.norm(X)))
        del R
        out[name] = {"ms": round(ms, 1), "inversions_per_s": round(1e3 / ms, 4), "code": r["code"],
                     "refine_iters": r["refine_iters"], "logabsdet": r["logabsdet"],
                     "det_sign": r["det_sign"], "resid": resid}
        Xs[name] = X
    d = float(torch.linalg.norm(Xs["fp32_refined"] - Xs["plain_fp64"]) / torch.linalg.norm(Xs["plain_fp64"]))
    out["refined_vs_plain_rel_frobenius"] = d
    out["accurate_vs_refined_rel_frobenius"] = float(
        torch.linalg.norm(Xs["fp32_refined_accurate"] - Xs["fp32_refined"]) / torch.linalg.norm(Xs["fp32_refined"]))
    out["speedup_accurate_over_plain"] = round(out["plain_fp64"]["ms"] / out["fp32_refined_accurate"]["ms"], 3)
    out["speedup_refined_over_plain"] = round(out["plain_fp64"]["ms"] / out["fp32_refined"]["ms"], 3)
    # roofline of the refinement's dominant kernel: the Newton-Schulz product
    # X R (n x n x n, FP64 MFMA), timed alone with HIP events
    X, R = Xs["fp32_refined"], Xs["plain_fp64"]
    D = torch.empty_like(X)
    gj.gj_dgemm(X, R, D=D)
    torch.cuda.synchronize()
    e = _events(2 * reps, stream)
    for k in range(reps):
        e[2 * k].record()
        gj.gj_dgemm(X, R, D=D)
        e[2 * k + 1].record()
    torch.cuda.synchronize()
    gms = min(e[2 * k].elapsed_time(e[2 * k + 1]) for k in range(reps))
    tflops = 2.0 * n ** 3 / (gms * 1e-3) / 1e12
    out["mfma_roofline"] = {"bound": "mfma", "kernel": "gemm_f64_kernel (n x n x n)",
                            "ms": round(gms, 3), "achieved": round(tflops, 2),
                            "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                            "frac": round(tflops / FP64_PEAK_TFLOPS, 4)}
    return out


def bench_solve(n: int = 4096, m: int = 16, reps: int = 3):
    """A X = B with m right-hand sides by the elimination of [A | B] (eq. 2
    with D^0 = B), on the headline's 4096 input: time per solve, the step
    kernel's rate over the n (n + m) array, and the normwise residual."""
    import torch
    import paper_1401_7962_amd as gj
    from paper_1401_7962_amd import inputs
    A = torch.from_numpy(inputs.single_dominant(n)).to("cuda")
    B = torch.from_numpy(inputs.rng_for(0, 4242).standard_normal((n, m))).to("cuda")
    X = torch.empty((n, m), dtype=torch.float64, device="cuda")
    ip = torch.empty(n, dtype=torch.int32, device="cuda")
    jp = torch.empty_like(ip)
    res = torch.empty(gj.RESULT_BYTES, dtype=torch.uint8, device="cuda")
    ws = torch.empty(gj.gj_workspace_size(gj.GJ_OP_SOLVE, n, [m]), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    gj.gj_solve(A, B, X, ip, jp, res, None, ws)
    torch.cuda.synchronize()
    e = _events(4 * reps, stream)
    for k in range(reps):
        o = gj.make_opts(step_events=(ctypes_ptr(e[4 * k + 1]), ctypes_ptr(e[4 * k + 2])))
        e[4 * k].record()
        gj.gj_solve(A, B, X, ip, jp, res, o, ws)
        e[4 * k + 3].record()
    torch.cuda.synchronize()
    ms = min(e[4 * k].elapsed_time(e[4 * k + 3]) for k in range(reps))
    steps_ms = min(e[4 * k + 1].elapsed_time(e[4 * k + 2]) for k in range(reps))
    r = gj.results_to_dicts(res)[0]
    resid = float(torch.linalg.norm(A @ X - B) / (torch.linalg.norm(A) * torch.linalg.norm(X)
                                                  + torch.linalg.norm(B)))
    per_launch_us = steps_ms * 1e3 / n
    alg = 16.0 * n * (n + m)
    gbs = alg / (per_launch_us * 1e-6) / 1e9
    return {"n": n, "m": m, "ms": round(ms, 2), "solves_per_s": round(1e3 / ms, 3),
            "code": r["code"], "resid": resid, "per_launch_us": round(per_launch_us, 2),
            "alg_bytes_per_launch": int(alg), "achieved_gbs": round(gbs, 1),
            "frac_of_hbm_peak": round(gbs / HBM_PEAK_GBS, 4)}


def bench_blocked(sizes=(4096, 8192), reps: int = 3):
    """Delayed updates (GJ_FLAG_BLOCKED) against the unblocked elimination on
    the same input (the headline's at 4096, a diagonally weighted uniform one
    at 8192): time per inversion, the steps' algorithmic sweep bytes
    sum_k 16 (n - k0(k))^2 over the whole-inversion time, identical pivots,
    and the distance between the two inverses."""
    import torch
    import paper_1401_7962_amd as gj
    from paper_1401_7962_amd import inputs
    out = {}
    stream = torch.cuda.current_stream()
    for n in sizes:
        if n == 4096:
            A = torch.from_numpy(inputs.single_dominant(n)).to("cuda")
        else:
            A = torch.from_numpy(inputs.rng_for(0, 8800 + n).uniform(-1.0, 1.0, (n, n))).to("cuda")
            A.diagonal().add_(4.0)
        row = {}
        Xs, pivs = {}, {}
        for name, flags in (("unblocked", 0), ("blocked", gj.GJ_FLAG_BLOCKED)):
            o = gj.make_opts(flags=flags)
            X = torch.empty_like(A)
            ip = torch.empty(n, dtype=torch.int32, device="cuda")
            jp = torch.empty_like(ip)
            res = torch.empty(gj.RESULT_BYTES, dtype=torch.uint8, device="cuda")
            ws = torch.empty(gj.gj_workspace_size(gj.GJ_OP_INVERT, n, None, o), dtype=torch.uint8, device="cuda")
            gj.gj_invert(A, X, ip, jp, res, o, ws)
            torch.cuda.synchronize()
            e = _events(2 * reps, stream)
            for k in range(reps):
                e[2 * k].record()
                gj.gj_invert(A, X, ip, jp, res, o, ws)
                e[2 * k + 1].record()
            torch.cuda.synchronize()
            ms = min(e[2 * k].elapsed_time(e[2 * k + 1]) for k in range(reps))
            r = gj.results_to_dicts(res)[0]
            row[name] = {"ms": round(ms, 2), "inv_per_s": round(1e3 / ms, 3), "code": r["code"]}
            Xs[name], pivs[name] = X, (ip.clone(), jp.clone(), r["det_mant"], r["det_exp"], r["det_sign"])
            del ws
        nb = 256   # the library's panel width (steps per delayed update)
        sweep = sum(16.0 * (n - (k // nb) * nb) ** 2 for k in range(n))
        row["blocked"]["step_sweep_bytes"] = sweep
        row["blocked"]["sweep_gbs_over_total_time"] = round(sweep / (row["blocked"]["ms"] * 1e-3) / 1e9, 1)
        row["speedup_blocked_over_unblocked"] = round(row["unblocked"]["ms"] / row["blocked"]["ms"], 3)
        pu, pb = pivs["unblocked"], pivs["blocked"]
        row["same_pivots_and_det"] = bool(torch.equal(pu[0], pb[0]) and torch.equal(pu[1], pb[1])
                                          and pu[2:] == pb[2:])
        row["blocked_vs_unblocked_rel_frobenius"] = float(
            torch.linalg.norm(Xs["blocked"] - Xs["unblocked"]) / torch.linalg.norm(Xs["unblocked"]))
        out[str(n)] = row
        del Xs, A
        torch.cuda.empty_cache()
    return out


def bench_pivot_rules(n: int = 4096, n_growth: int = 512, reps: int = 2):
    """The three pivot rules on the GPU: time per inversion of the headline
    input, and the normwise residual ||A X - I||_F / (||A||_F ||X||_F) on a
    matrix where the program's signed rule takes tiny pivots (negative
    off-diagonal entries, a tiny positive diagonal)."""
    import torch
    import paper_1401_7962_amd as gj
    from paper_1401_7962_amd import inputs
    A = torch.from_numpy(inputs.single_dominant(n)).to("cuda")
    rng = inputs.rng_for(0, 4343)
    G = -np.abs(rng.standard_normal((n_growth, n_growth)))
    np.fill_diagonal(G, 1e-6)
    G = torch.from_numpy(G).to("cuda")
    stream = torch.cuda.current_stream()
    out = {"n": n, "growth_n": n_growth}
    for name, flags in (("full", 0), ("partial", gj.GJ_FLAG_PIVOT_PARTIAL),
                        ("program", gj.GJ_FLAG_PIVOT_PROGRAM)):
        o = gj.make_opts(flags=flags)
        X, ip, jp, res = gj.gj_invert(A, opts=o)
        torch.cuda.synchronize()
        e = _events(2 * reps, stream)
        for k in range(reps):
            e[2 * k].record()
            gj.gj_invert(A, X, ip, jp, res, o)
            e[2 * k + 1].record()
        torch.cuda.synchronize()
        ms = min(e[2 * k].elapsed_time(e[2 * k + 1]) for k in range(reps))
        Xg, _, _, rg = gj.gj_invert(G, opts=o)
        torch.cuda.synchronize()
        code = gj.results_to_dicts(rg)[0]["code"]
        resid = float(torch.linalg.norm(G @ Xg - torch.eye(n_growth, dtype=torch.float64, device="cuda"))
                      / (torch.linalg.norm(G) * torch.linalg.norm(Xg)))
        out[name] = {"ms": round(ms, 1), "growth_case_code": code, "growth_case_resid": resid}
    return out


def bench_accuracy_exact(n: int = 4096, span: int = 20, reps: int = 2):
    """Forward error against an exactly known inverse at the headline order:
    A = H D H^T with H Sylvester-Hadamard and D a diagonal of powers of two
    spanning 2^span (cond(A) = 2^span); A and A^-1 = H D^-1 H^T / n^2 are
    exact in FP64 (integer and dyadic sums below 2^53).  Plain FP64
    elimination, FP32 + FP64 Newton-Schulz, and the same with the
    accurate-residual updates."""
    import torch
    import paper_1401_7962_amd as gj
    from paper_1401_7962_amd import inputs
    H = torch.from_numpy(inputs.sylvester_hadamard(n)).to("cuda")
    rng = inputs.rng_for(0, 4444)
    e = rng.integers(0, span + 1, size=n)
    e[0], e[1] = 0, span
    d = torch.from_numpy(np.ldexp(1.0, e)).to("cuda")
    A = (H * d) @ H.T
    Ainv = (H / d) @ H.T / float(n * n)
    del H
    stream = torch.cuda.current_stream()
    out = {"n": n, "cond": 2.0 ** span}
    for name, prec, flags in (("plain_fp64", gj.GJ_PREC_FP64, 0),
                              ("fp32_refined", gj.GJ_PREC_FP32_REFINED, 0),
                              ("fp32_refined_accurate", gj.GJ_PREC_FP32_REFINED, gj.GJ_FLAG_ACCURATE)):
        o = gj.make_opts(precision=prec, flags=flags)
        X, ip, jp, res = gj.gj_invert(A, opts=o)
        torch.cuda.synchronize()
        ev = _events(2 * reps, stream)
        for k in range(reps):
            ev[2 * k].record()
            gj.gj_invert(A, X, ip, jp, res, o)
            ev[2 * k + 1].record()
        torch.cuda.synchronize()
        ms = min(ev[2 * k].elapsed_time(ev[2 * k + 1]) for k in range(reps))
        r = gj.results_to_dicts(res)[0]
        err = float(torch.linalg.norm(X - Ainv) / torch.linalg.norm(Ainv))
        out[name] = {"ms": round(ms, 1), "code": r["code"], "refine_iters": r["refine_iters"],
                     "rel_forward_error": err}
        del X
    return out


def ctypes_ptr(event):
    """hipEvent_t handle of a torch.cuda.Event."""
    return event.cuda_event


def cpu_baseline(n: int = 4096, sample_steps: int = 256):
    """The FP64 oracle (single-threaded C) on the same 4096 input for its
    first ``sample_steps`` steps; every step of the in-place elimination does
    the same n(n-1) updates, so the full inversion takes n/sample_steps times
    as long (the shrinking pivot search makes this a slight overestimate)."""
    import oracle
    from paper_1401_7962_amd import inputs
    A = inputs.single_dominant(n)
    t0 = time.perf_counter()
    oracle.gj_first_steps(A, sample_steps)
    dt = time.perf_counter() - t0
    full = dt * n / sample_steps
    return {
        "value": 1.0 / full,
        "unit": "inversions/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"first {sample_steps} of {n} elimination steps of the {n}x{n} input "
                  f"({dt:.1f} s), scaled by {n}/{sample_steps}",
    }


LEGS = {"latency_small": lambda: bench_latency_small(),
        "batch_uneven_100k": lambda: bench_batch_uneven(),
        "conditioned_8192": lambda: bench_conditioned_8192(),
        "batch_conditioned_20k": lambda: bench_batch_conditioned(),
        "solve_4096": lambda: bench_solve(),
        "pivot_rules": lambda: bench_pivot_rules(),
        "accuracy_exact_4096": lambda: bench_accuracy_exact(),
        "blocked": lambda: bench_blocked()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--headline-only", action="store_true",
                    help="skip the secondary workloads (latency, batch, refined 8192)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 512 MiB device copy, whose rocprofv3 FETCH_SIZE and "
                         "WRITE_SIZE calibrate the counters")
    ap.add_argument("--leg", choices=sorted(LEGS),
                    help="run one secondary workload alone and print its result (for profiling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: measures one GPU only (asked for --gpus {args.gpus}); "
              "the batched and single-matrix paths would shard by matrix or by row block across "
              "GPUs, but no multi-GPU run is implemented.",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1401_7962_amd as gj
    gj.load_library()
    torch.cuda.init()
    if args.leg:
        print(json.dumps({"leg": args.leg, **LEGS[args.leg]()}), flush=True)
        return

    if args.copy_calibration:
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(2):
            dst.copy_(src)
        torch.cuda.synchronize()
        print("copy calibration: 2 x 536870912-byte device copies", file=sys.stderr, flush=True)
    head = bench_headline(args.steps, args.warmup, args.n)
    out = {
        "metric": "inversions/s & HBM GB/s: FP64 plain vs FP32+FP64-refined, at 1e-12 rel error",
        "value": round(head["value"], 4),
        "unit": "inversions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_inv"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"single {args.n}x{args.n} FP64 matrix, U[-1,1] + 4I, plain full-pivot "
                        "Gauss-Jordan (inverse, pivots, determinant)",
            "n": args.n,
            "path": "streaming, one fused eq.15-sweep + pivot-search launch per step",
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "gj_big_step<double,256>",
            "achieved": round(head["achieved_gbs"], 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(head["achieved_gbs"] / HBM_PEAK_GBS, 4),
            "traffic": head["traffic"],
            "per_launch_us": round(head["per_launch_us"], 3),
            "alg_bytes_per_launch": 16 * args.n * args.n,
        },
        "checks": {"resid": head["resid"], "logabsdet": head["logabsdet"],
                   "det_sign": head["det_sign"]},
    }
    if not args.headline_only:
        extras = {}
        extras["latency_small"] = bench_latency_small()
        print("bench: small-matrix latency done", file=sys.stderr, flush=True)
        extras["batch_uneven_100k"] = bench_batch_uneven()
        print("bench: 100k batch done", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
        extras["conditioned_8192"] = bench_conditioned_8192()
        print("bench: 8192 plain vs refined done", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
        extras["batch_conditioned_20k"] = bench_batch_conditioned()
        print("bench: 20k refined batch done", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
        extras["solve_4096"] = bench_solve()
        print("bench: solve done", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
        extras["pivot_rules"] = bench_pivot_rules()
        print("bench: pivot rules done", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
        extras["accuracy_exact_4096"] = bench_accuracy_exact()
        print("bench: exact-inverse accuracy done", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
        extras["blocked"] = bench_blocked()
        print("bench: blocked elimination done", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
        out["extras"] = extras
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.n)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
