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


def host_info() -> dict:
    """CPU model and the cores this process may use (the oracle legs use all
    of them unless OMP_NUM_THREADS caps it)."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    import oracle
    return {"cpu_model": model, "cores_available": len(os.sched_getaffinity(0)),
            "oracle_threads": oracle.host_threads()}


def _oracle_sample_rate(A, all_steps: int, one_steps: int):
    """Inversions/s of the FP64 oracle on a square matrix, from the first
    steps of the run (every step does the same n(n-1) updates; the shrinking
    search makes the scaled time a slight overestimate): all host cores
    (OpenMP form, bitwise the serial oracle) and one core (serial oracle)."""
    import oracle
    n = A.shape[0]
    threads = oracle.host_threads()
    t0 = time.perf_counter()
    oracle.gj_invert_f64_par(A, threads, max_steps=min(all_steps, n))
    t_all = (time.perf_counter() - t0) * n / min(all_steps, n)
    t0 = time.perf_counter()
    oracle.gj_first_steps(A, min(one_steps, n))
    t_one = (time.perf_counter() - t0) * n / min(one_steps, n)
    return {"all_cores_s_per_inversion": t_all, "threads": threads,
            "one_core_s_per_inversion": t_one,
            "sample": f"first {min(all_steps, n)} (all cores) and {min(one_steps, n)} (one core) "
                      f"of {n} steps, scaled by n / steps"}


def _rel(a, b) -> float:
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


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
    # the metric's comparison on the same input: FP32 elimination + FP64
    # Newton-Schulz, against the plain result (which the tests hold bit for
    # bit to the FP64 oracle at this order)
    ro = gj.make_opts(precision=gj.GJ_PREC_FP32_REFINED)
    Xr = torch.empty_like(A)
    ipr = torch.empty_like(ipiv)
    jpr = torch.empty_like(jpiv)
    resr = torch.empty_like(res)
    wsr = torch.empty(gj.gj_workspace_size(gj.GJ_OP_INVERT, n, None, ro), dtype=torch.uint8, device=dev)
    gj.gj_invert(A, Xr, ipr, jpr, resr, ro, wsr, stream)
    torch.cuda.synchronize()
    evr = _events(2 * 3, stream)
    for k in range(3):
        evr[2 * k].record()
        gj.gj_invert(A, Xr, ipr, jpr, resr, ro, wsr, stream)
        evr[2 * k + 1].record()
    torch.cuda.synchronize()
    ref_ms = min(evr[2 * k].elapsed_time(evr[2 * k + 1]) for k in range(3))
    rr = gj.results_to_dicts(resr)[0]
    refined = {"ms_per_inv": round(ref_ms, 2), "inversions_per_s": round(1e3 / ref_ms, 4),
               "code": rr["code"], "refine_iters": rr["refine_iters"],
               "rel_frobenius_vs_fp64": float(torch.linalg.norm(Xr - X) / torch.linalg.norm(X)),
               "logabsdet_minus_fp64": rr["logabsdet"] - r["logabsdet"],
               "speedup_over_fp64": round(ms_per_inv / ref_ms, 3)}
    del wsr, Xr
    return {
        "refined": refined,
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
        import oracle
        t0 = time.perf_counter()
        for _ in range(20):
            Xo, io, jo, ro = oracle.gj_invert_f64(A_h)
        ous = (time.perf_counter() - t0) / 20 * 1e6
        same = (X.cpu().numpy().tobytes() == Xo.tobytes() and np.array_equal(ip.cpu().numpy(), io)
                and np.array_equal(jp.cpu().numpy(), jo) and r["det_mant"] == ro["det_mant"]
                and r["det_exp"] == ro["det_exp"])
        out[name] = {"n": n, "us_per_inversion": round(us, 2), "code": r["code"], "det": r["det"],
                     "bitwise_equal_to_oracle": bool(same),
                     "oracle_one_core_us_per_inversion": round(ous, 2)}
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
        # the streaming members' step launches, timed eagerly between events:
        # every launch reads and writes each active member's array once, so
        # the phase moves 2 esz sum(n^3) bytes (members above the on-chip
        # limit)
        ev = _events(2, torch.cuda.current_stream())
        so = gj.make_opts(precision=prec, flags=gj.GJ_FLAG_REUSE_PLAN,
                          step_events=(ctypes_ptr(ev[0]), ctypes_ptr(ev[1])))
        gj.gj_invert_batched(sizes, offs, A, X, poff, ip, jp, res, so, ws)
        torch.cuda.synchronize()
        steps_ms = ev[0].elapsed_time(ev[1])
        esz = 8 if prec == gj.GJ_PREC_FP64 else 4
        big = sizes[sizes > gj.gj_onchip_max_n()].astype(np.float64)
        step_bytes = 2.0 * esz * float((big ** 3).sum())
        gbs = step_bytes / (steps_ms * 1e-3) / 1e9
        del ws
        raw = np.frombuffer(res.cpu().numpy().tobytes(), dtype=np.uint8).reshape(batch, gj.RESULT_BYTES)
        codes = raw[:, 0:4].copy().view(np.int32)[:, 0]
        iters = raw[:, 12:16].copy().view(np.int32)[:, 0]
        logdet = raw[:, 40:48].copy().view(np.float64)[:, 0]
        cf = sizes * np.log(conds) / 2.0
        rel_det = np.abs(logdet - cf) / np.abs(cf)
        out[name] = {"ms": round(ms, 2), "inversions_per_s": round(batch / (ms * 1e-3), 1),
                     "streaming_steps_ms": round(steps_ms, 2),
                     "step_roofline": {"bound": "hbm",
                                       "kernel": "gj_big_step, batched (%s)" % ("FP64" if esz == 8 else "FP32"),
                                       "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                       "frac": round(gbs / HBM_PEAK_GBS, 4),
                                       "alg_bytes": step_bytes},
                     "codes": {str(c): int((codes == c).sum()) for c in np.unique(codes)},
                     "mean_refine_iters": float(iters.mean()),
                     "max_rel_logdet_err_vs_closed_form": float(rel_det.max()),
                     "max_rel_logdet_err_vs_lu_slogdet": float((np.abs(logdet - lu_ref) / np.abs(lu_ref)).max())}
        Xs[name] = X
    d = torch.linalg.norm(Xs["fp32_refined"] - Xs["plain_fp64"]) / torch.linalg.norm(Xs["plain_fp64"])
    out["refined_vs_plain_rel_frobenius_whole_batch"] = float(d)
    out["speedup_refined_over_plain"] = round(out["plain_fp64"]["ms"] / out["fp32_refined"]["ms"], 3)
    out["oracle"] = _batch_conditioned_oracle(sizes, offs, conds, A, Xs)
    return out


def _batch_conditioned_oracle(sizes, offs, conds, A, Xs, n_sample: int = 200, n_one: int = 24):
    """A stratified sample of the 20,000 members (sorted by order, then every
    (batch / n_sample)-th): the FP64 oracle on all host cores (and on one
    core for fewer of them), both scaled to the whole batch by sum n^3; the
    GPU's plain and refined inverses of the sample against the oracle's and
    against reference inverses (Newton steps with an exactly formed
    residual).  The refined bar (R-16): forward error <= 4 x the oracle's
    own + 1e-14, and 1e-12 against the oracle for cond <= 1e4."""
    import oracle
    batch = len(sizes)
    order = np.argsort(sizes.astype(np.int64) * 100 + np.log10(conds).astype(np.int64), kind="stable")
    pick = order[:: max(1, batch // n_sample)][:n_sample]
    mats = [A[int(offs[b]): int(offs[b]) + int(sizes[b]) ** 2].cpu().numpy() for b in pick]
    xg = {name: [X[int(offs[b]): int(offs[b]) + int(sizes[b]) ** 2].cpu().numpy() for b in pick]
          for name, X in Xs.items()}
    ns = sizes[pick].astype(np.int32)
    so = np.zeros(len(pick), dtype=np.int64)
    so[1:] = np.cumsum(ns.astype(np.int64) ** 2)[:-1]
    packed = np.concatenate(mats)
    t0 = time.perf_counter()
    Xo, _, _, _ = oracle.gj_invert_batched(ns, so, packed)
    t_all = time.perf_counter() - t0
    one = np.arange(0, len(pick), max(1, len(pick) // n_one))[:n_one]
    t0 = time.perf_counter()
    for i in one:
        oracle.gj_invert_f64(mats[i].reshape(int(ns[i]), int(ns[i])))
    t_one = time.perf_counter() - t0
    cube = sizes.astype(np.float64) ** 3
    scale_all = cube.sum() / (ns.astype(np.float64) ** 3).sum()
    scale_one = cube.sum() / (ns[one].astype(np.float64) ** 3).sum()
    worst = {"fp32_refined": 0.0, "plain_fp64": 0.0}
    max_vs_oracle_low_cond = 0.0
    max_err = {"fp32_refined": 0.0, "plain_fp64": 0.0, "fp64_oracle": 0.0}
    for i, b in enumerate(pick):
        n = int(ns[i])
        Ab = mats[i].reshape(n, n)
        Xob = Xo[so[i]: so[i] + n * n].reshape(n, n)
        T = oracle.inverse_truth(Ab, Xob)
        err_o = _rel(Xob, T)
        max_err["fp64_oracle"] = max(max_err["fp64_oracle"], err_o)
        for name in ("fp32_refined", "plain_fp64"):
            e = _rel(xg[name][i].reshape(n, n), T)
            max_err[name] = max(max_err[name], e)
            worst[name] = max(worst[name], e / (4 * err_o + 1e-14))
        if conds[b] <= 1e4:
            max_vs_oracle_low_cond = max(max_vs_oracle_low_cond,
                                         _rel(xg["fp32_refined"][i].reshape(n, n), Xob))
    return {"sample_members": int(len(pick)), "threads": oracle.host_threads(),
            "all_cores_inversions_per_s": round(batch / (t_all * scale_all), 1),
            "one_core_inversions_per_s": round(batch / (t_one * scale_one), 1),
            "sample": f"{len(pick)} members stratified by order and condition (all cores); "
                      f"{len(one)} of them on one core; scaled by sum n^3",
            "max_forward_error_vs_reference": max_err,
            "max_error_over_bar": worst,
            "max_refined_vs_oracle_cond_le_1e4": max_vs_oracle_low_cond}


def bench_batch_uneven(batch: int = 100_000, reps: int = 3, oracle_sample: int = 10000,
                       oracle_sample_one: int = 1000):
    """100,000 FP64 matrices, n uniform in [8,128], 1% rank n-1: the on-chip
    persistent launches (one per register-block class).  Reports
    inversions/s, the FP64 FMA rate against the FP64 vector peak (n^3 FMAs
    = 2 n^3 flop per inversion), and the FP64 oracle on a sample of the same
    members (all host cores, and one core), whose results the GPU's must
    equal bit for bit."""
    import torch
    import oracle
    import paper_1401_7962_amd as gj
    from paper_1401_7962_amd import inputs
    sizes, offs, packed, singular = inputs.batch_uneven(batch)
    A = torch.from_numpy(packed).cuda()
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
    tflops = flops / (ms * 1e-3) / 1e12
    # the oracle on the first members (a uniform draw of orders): all cores,
    # then one core on fewer; both scaled to the whole batch by sum n^3
    cube = sizes.astype(np.float64) ** 3
    m_all, m_one = min(oracle_sample, batch), min(oracle_sample_one, batch)
    span_all = int(offs[m_all - 1] + int(sizes[m_all - 1]) ** 2)
    t0 = time.perf_counter()
    Xo, io, jo, ro = oracle.gj_invert_batched(sizes[:m_all], offs[:m_all], packed[:span_all])
    t_all = (time.perf_counter() - t0) * cube.sum() / cube[:m_all].sum()
    span_one = int(offs[m_one - 1] + int(sizes[m_one - 1]) ** 2)
    t0 = time.perf_counter()
    oracle.gj_invert_batched(sizes[:m_one], offs[:m_one], packed[:span_one], nthreads=1)
    t_one = (time.perf_counter() - t0) * cube.sum() / cube[:m_one].sum()
    npiv = int(poff[m_all - 1] + sizes[m_all - 1])
    same = bool(X[:span_all].cpu().numpy().tobytes() == Xo[:span_all].tobytes()
                and np.array_equal(ip[:npiv].cpu().numpy(), io) and np.array_equal(jp[:npiv].cpu().numpy(), jo))
    return {
        "batch": batch,
        "ms": round(ms, 3),
        "inversions_per_s": round(batch / (ms * 1e-3), 1),
        "fp64_tflops": round(tflops, 3),
        "roofline": {"bound": "alu", "kernel": "gj_onchip_kernel (FP64, every class)",
                     "achieved": round(tflops, 3), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(tflops / FP64_PEAK_TFLOPS, 4),
                     "alg_flop": flops, "note": "n^3 fma per member; pivot-search compares not counted"},
        "singular_flagged": int((codes == 1).sum()),
        "singular_planted": int(len(singular)),
        "other_codes": int(((codes != 0) & (codes != 1)).sum()),
        "oracle": {"all_cores_inversions_per_s": round(batch / t_all, 1),
                   "one_core_inversions_per_s": round(batch / t_one, 1),
                   "threads": oracle.host_threads(),
                   "sample": f"first {m_all} members on all cores, first {m_one} on one core, "
                             "scaled by sum n^3",
                   "gpu_bitwise_equal_on_sample": same},
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
                              ("fp32_refined_accurate", gj.GJ_PREC_FP32_REFINED, gj.GJ_FLAG_ACCURATE),
                              ("plain_fp64_blocked", gj.GJ_PREC_FP64, gj.GJ_FLAG_BLOCKED),
                              ("fp32_refined_blocked", gj.GJ_PREC_FP32_REFINED, gj.GJ_FLAG_BLOCKED)):
        # the FP64 blocked elimination records no step events
        timed_steps = not (flags & gj.GJ_FLAG_BLOCKED and prec == gj.GJ_PREC_FP64)
        opts = gj.make_opts(precision=prec, flags=flags)
        X = torch.empty_like(A)
        ip = torch.empty(n, dtype=torch.int32, device="cuda")
        jp = torch.empty_like(ip)
        res = torch.empty(gj.RESULT_BYTES, dtype=torch.uint8, device="cuda")
        ws = torch.empty(gj.gj_workspace_size(gj.GJ_OP_INVERT, n, None, opts), dtype=torch.uint8,
                         device="cuda")
        gj.gj_invert(A, X, ip, jp, res, opts, ws)
        torch.cuda.synchronize()
        e = _events(4 * reps, stream)
        for k in range(reps):
            so = gj.make_opts(precision=prec, flags=flags,
                              step_events=(ctypes_ptr(e[4 * k + 1]), ctypes_ptr(e[4 * k + 2]))
                              if timed_steps else (None, None))
            e[4 * k].record()
            gj.gj_invert(A, X, ip, jp, res, so, ws)
            e[4 * k + 3].record()
        torch.cuda.synchronize()
        best = min(range(reps), key=lambda k: e[4 * k].elapsed_time(e[4 * k + 3]))
        ms = e[4 * best].elapsed_time(e[4 * best + 3])
        steps_ms = e[4 * best + 1].elapsed_time(e[4 * best + 2]) if timed_steps else None
        r = gj.results_to_dicts(res)[0]
        del ws
        R = gj.gj_dgemm(A, X, gamma=1.0, alpha=-1.0)
        resid = float(torch.linalg.norm(R) / (torch.linalg.norm(A) * torch.linalg.norm(X)))
        del R
        esz = 8 if prec == gj.GJ_PREC_FP64 else 4
        out[name] = {"ms": round(ms, 1), "inversions_per_s": round(1e3 / ms, 4), "code": r["code"],
                     "refine_iters": r["refine_iters"], "logabsdet": r["logabsdet"],
                     "det_sign": r["det_sign"], "resid": resid}
        if steps_ms is not None and not flags & gj.GJ_FLAG_BLOCKED:
            # the elimination's step kernel: each launch reads and writes the
            # whole n x n array once (16 n^2 B in FP64, 8 n^2 B in FP32)
            gbs = 2.0 * esz * n * n * n / (steps_ms * 1e-3) / 1e9
            out[name]["elimination_ms"] = round(steps_ms, 1)
            out[name]["step_roofline"] = {
                "bound": "hbm", "kernel": "gj_big_step (%s)" % ("FP64" if esz == 8 else "FP32"),
                "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(gbs / HBM_PEAK_GBS, 4), "alg_bytes_per_launch": 2 * esz * n * n,
                "per_launch_us": round(steps_ms * 1e3 / n, 2)}
        elif steps_ms is not None:
            # delayed updates: the steps sweep only the trailing block (order
            # n - k0 in the panel starting at k0); the products between panels
            # are inside the same interval
            nb = 256
            sweep = sum(2.0 * esz * (n - (k // nb) * nb) ** 2 for k in range(n))
            out[name]["elimination_ms"] = round(steps_ms, 1)
            out[name]["elimination_sweep_gbs"] = round(sweep / (steps_ms * 1e-3) / 1e9, 1)
        Xs[name] = X
        print(f"[conditioned_{n}] {name}: {ms:.1f} ms", file=sys.stderr, flush=True)
    d = float(torch.linalg.norm(Xs["fp32_refined"] - Xs["plain_fp64"]) / torch.linalg.norm(Xs["plain_fp64"]))
    out["refined_vs_plain_rel_frobenius"] = d
    out["accurate_vs_refined_rel_frobenius"] = float(
        torch.linalg.norm(Xs["fp32_refined_accurate"] - Xs["fp32_refined"]) / torch.linalg.norm(Xs["fp32_refined"]))
    out["speedup_accurate_over_plain"] = round(out["plain_fp64"]["ms"] / out["fp32_refined_accurate"]["ms"], 3)
    out["speedup_refined_over_plain"] = round(out["plain_fp64"]["ms"] / out["fp32_refined"]["ms"], 3)
    out["speedup_refined_blocked_over_plain_blocked"] = round(
        out["plain_fp64_blocked"]["ms"] / out["fp32_refined_blocked"]["ms"], 3)
    out["refined_blocked_vs_plain_rel_frobenius"] = float(
        torch.linalg.norm(Xs["fp32_refined_blocked"] - Xs["plain_fp64"]) / torch.linalg.norm(Xs["plain_fp64"]))
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
    del Xs, X, R, D, A
    torch.cuda.empty_cache()
    out["cross_check_2048"] = oracle_cross_check_2048()
    return out


def bench_gemm_f64(n: int = 8192, reps: int = 3):
    """The refinement's product alone: D = X R for n x n FP64 operands (the
    Newton-Schulz update X (I - A X) of the conditioned workload has this
    shape), timed with HIP events; for counter runs (MFMA busy cycles)."""
    import torch
    import paper_1401_7962_amd as gj
    g = torch.Generator(device="cuda")
    g.manual_seed(8192)
    X = torch.randn(n, n, dtype=torch.float64, device="cuda", generator=g)
    R = torch.randn(n, n, dtype=torch.float64, device="cuda", generator=g)
    D = torch.empty_like(X)
    gj.gj_dgemm(X, R, D=D)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e = _events(2 * reps, stream)
    for k in range(reps):
        e[2 * k].record()
        gj.gj_dgemm(X, R, D=D)
        e[2 * k + 1].record()
    torch.cuda.synchronize()
    gms = min(e[2 * k].elapsed_time(e[2 * k + 1]) for k in range(reps))
    tflops = 2.0 * n ** 3 / (gms * 1e-3) / 1e12
    return {"n": n, "calls": reps + 1, "ms": round(gms, 3),
            "roofline": {"bound": "mfma", "kernel": "gemm_f64_kernel (n x n x n)",
                         "achieved": round(tflops, 2), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": round(tflops / FP64_PEAK_TFLOPS, 4), "flop_per_call": 2.0 * n ** 3}}


def oracle_cross_check_2048(n: int = 2048, cond: float = 1e6):
    """The 2048 instance of the conditioned workload (seed offset 40, built on
    the host): the plain and refined GPU inverses against the FP64 oracle and
    against a reference inverse (Newton steps from the oracle's inverse with
    an exactly formed residual), with the oracle timed on all host cores and
    on one."""
    import torch
    import oracle
    import paper_1401_7962_amd as gj
    from paper_1401_7962_amd import inputs
    A_h = inputs.single_conditioned(n, cond, offset=40)
    A = torch.from_numpy(A_h).cuda()
    gpu = {}
    for name, prec in (("plain_fp64", gj.GJ_PREC_FP64), ("fp32_refined", gj.GJ_PREC_FP32_REFINED)):
        X, ip, jp, res = gj.gj_invert(A, opts=gj.make_opts(precision=prec))
        torch.cuda.synchronize()
        gpu[name] = (X.cpu().numpy(), ip.cpu().numpy(), jp.cpu().numpy(), gj.results_to_dicts(res)[0])
    t0 = time.perf_counter()
    Xo, io, jo, ro = oracle.gj_invert_f64_par(A_h)
    t_all = time.perf_counter() - t0
    t0 = time.perf_counter()
    Xt = oracle.inverse_truth(A_h, Xo)
    t_truth = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.gj_first_steps(A_h, 128)
    t_one = (time.perf_counter() - t0) * n / 128
    err_o = _rel(Xo, Xt)
    out = {"n": n, "cond": cond, "fp64_oracle_forward_error_vs_reference": err_o}
    for name, (Xg, ig, jg, r) in gpu.items():
        out[name] = {"code": r["code"], "refine_iters": r["refine_iters"],
                     "rel_frobenius_vs_fp64_oracle": _rel(Xg, Xo),
                     "rel_forward_error_vs_reference": _rel(Xg, Xt),
                     "logabsdet_minus_closed_form": r["logabsdet"] - inputs.closed_form_logdet(n, cond)}
    Xg, ig, jg, r = gpu["plain_fp64"]
    out["plain_fp64"]["bitwise_equal_to_oracle"] = bool(
        Xg.tobytes() == Xo.tobytes() and np.array_equal(ig, io) and np.array_equal(jg, jo)
        and r["det_mant"] == ro["det_mant"] and r["det_exp"] == ro["det_exp"])
    out["refined_error_over_oracle_error"] = out["fp32_refined"]["rel_forward_error_vs_reference"] / err_o
    out["oracle"] = {"all_cores_s": round(t_all, 2), "threads": oracle.host_threads(),
                     "one_core_s": round(t_one, 1), "reference_inverse_s": round(t_truth, 2),
                     "sample": "all cores: the whole inversion; one core: the first 128 of 2048 "
                               "steps, scaled by 16"}
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


def bench_single_orders(sizes=(256, 512, 1024, 2048), reps: int = 3):
    """One matrix of moderate order (the headline's input family): plain FP64
    and FP32 + FP64 refinement, ms per inversion and the elimination's us per
    step (HIP events around the step launches), with the FP64 result checked
    bit for bit against the oracle (its OpenMP form, bitwise the serial
    oracle) and the oracle's time on all host cores."""
    import torch
    import oracle
    import paper_1401_7962_amd as gj
    from paper_1401_7962_amd import inputs
    out = {}
    stream = torch.cuda.current_stream()
    for n in sizes:
        A_h = inputs.single_dominant(n)
        A = torch.from_numpy(A_h).to("cuda")
        row = {}
        for name, prec in (("plain_fp64", gj.GJ_PREC_FP64), ("fp32_refined", gj.GJ_PREC_FP32_REFINED)):
            o = gj.make_opts(precision=prec)
            X = torch.empty_like(A)
            ip = torch.empty(n, dtype=torch.int32, device="cuda")
            jp = torch.empty_like(ip)
            res = torch.empty(gj.RESULT_BYTES, dtype=torch.uint8, device="cuda")
            ws = torch.empty(gj.gj_workspace_size(gj.GJ_OP_INVERT, n, None, o), dtype=torch.uint8,
                             device="cuda")
            gj.gj_invert(A, X, ip, jp, res, o, ws)
            torch.cuda.synchronize()
            e = _events(4 * reps, stream)
            for k in range(reps):
                so = gj.make_opts(precision=prec,
                                  step_events=(ctypes_ptr(e[4 * k + 1]), ctypes_ptr(e[4 * k + 2])))
                e[4 * k].record()
                gj.gj_invert(A, X, ip, jp, res, so, ws)
                e[4 * k + 3].record()
            torch.cuda.synchronize()
            ms = min(e[4 * k].elapsed_time(e[4 * k + 3]) for k in range(reps))
            steps_ms = min(e[4 * k + 1].elapsed_time(e[4 * k + 2]) for k in range(reps))
            r = gj.results_to_dicts(res)[0]
            row[name] = {"ms": round(ms, 3), "us_per_step": round(steps_ms * 1e3 / n, 2),
                         "code": r["code"], "refine_iters": r["refine_iters"]}
            if prec == gj.GJ_PREC_FP64:
                t0 = time.perf_counter()
                Xo, io, jo, ro = oracle.gj_invert_f64_par(A_h)
                row["oracle_all_cores_ms"] = round((time.perf_counter() - t0) * 1e3, 1)
                row[name]["bitwise_equal_to_oracle"] = bool(
                    X.cpu().numpy().tobytes() == Xo.tobytes()
                    and np.array_equal(ip.cpu().numpy(), io) and np.array_equal(jp.cpu().numpy(), jo)
                    and r["det_mant"] == ro["det_mant"] and r["det_exp"] == ro["det_exp"])
            del ws
        out[str(n)] = row
    out["oracle_threads"] = oracle.host_threads()
    return out


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
                              ("fp32_refined_accurate", gj.GJ_PREC_FP32_REFINED, gj.GJ_FLAG_ACCURATE),
                              ("plain_fp64_blocked", gj.GJ_PREC_FP64, gj.GJ_FLAG_BLOCKED),
                              ("fp32_refined_blocked", gj.GJ_PREC_FP32_REFINED, gj.GJ_FLAG_BLOCKED)):
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


def cpu_baseline(n: int = 4096, all_steps: int = 512, one_steps: int = 64):
    """The FP64 oracle on the same 4096 input, timed on all host cores (its
    OpenMP form: each step's rows shared among threads, bitwise the serial
    oracle) and on one core (the serial oracle), each over the first steps
    of the run and scaled by n / steps (every step does the same n(n-1)
    updates; the shrinking search makes this a slight overestimate)."""
    from paper_1401_7962_amd import inputs
    A = inputs.single_dominant(n)
    r = _oracle_sample_rate(A, all_steps, one_steps)
    info = host_info()
    return {
        "value": round(1.0 / r["all_cores_s_per_inversion"], 5),
        "unit": "inversions/s",
        "cores": r["threads"],
        "kind": "oracle",
        "sample": r["sample"] + f" of the {n}x{n} input",
        "cpu_model": info["cpu_model"],
        "single_core": {"value": round(1.0 / r["one_core_s_per_inversion"], 5), "cores": 1},
    }


LEGS = {"latency_small": lambda: bench_latency_small(),
        "batch_uneven_100k": lambda: bench_batch_uneven(),
        "conditioned_8192": lambda: bench_conditioned_8192(),
        "batch_conditioned_20k": lambda: bench_batch_conditioned(),
        "solve_4096": lambda: bench_solve(),
        "pivot_rules": lambda: bench_pivot_rules(),
        "accuracy_exact_4096": lambda: bench_accuracy_exact(),
        "blocked": lambda: bench_blocked(),
        "single_orders": lambda: bench_single_orders(),
        "gemm_f64_8192": lambda: bench_gemm_f64()}


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
        "fp32_refined_same_input": head["refined"],
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
        extras["single_orders"] = bench_single_orders()
        print("bench: single matrices of moderate order done", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
        out["extras"] = extras
        out["host"] = host_info()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.n)
        print("bench: cpu baseline done", file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
