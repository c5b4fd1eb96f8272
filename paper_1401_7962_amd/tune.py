"""Autotuner for the streaming elimination's workgroup shape.

The streaming kernels give each workgroup R whole rows of the working array.
Small R means many workgroups with a high fixed cost each (they all reduce
the candidate list and read the pivot row); large R means few workgroups and
less memory-level parallelism.  This script times every admissible R for
each size bucket and precision on the GPU it runs on, then, with the best
R, the share of a step's work units left to the step kernel's counter (the
rest are taken by workgroup index; units from the counter let faster parts
of the chip sweep more rows, at the cost of a barrier per unit) and, where
no units go to the counter, fewer register chunks per thread (more threads
per row, so more loads in flight per row at the cost of more workgroup-wide
reductions).  The winners go to gj_tune.txt beside libgj.so, which the
library reads at its first call:

    big_rows <f32|f64> <n_min> <n_max> <R> <counted %> <chunks>

Buckets up to n = 1024 are timed as packed batches (about 128 MiB of
matrices, the batched use case); larger ones as single inversions.  FP64 is
timed through the plain elimination, FP32 through the refined path (its
elimination dominates for these sizes).

    python -m paper_1401_7962_amd.tune [--out FILE] [--quick]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
BUCKETS = [(129, 256), (257, 512), (513, 1024), (1025, 2048), (2049, 4096), (4097, 8192)]
CANDIDATES = [1, 2, 4, 8, 16, 32, 64]
COUNTED = [25, 37, 50]   # percent of a step's units from the counter (0: none)
CHUNKS = [4]             # register chunks per thread tried besides the default 8


def _time(fn, reps):
    import torch
    fn()
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    return best


def _workload(n, fp32, gj, inputs):
    """Return a zero-argument callable that runs the bucket's workload."""
    import torch
    prec = gj.GJ_PREC_FP32_REFINED if fp32 else gj.GJ_PREC_FP64
    if n <= 1024:
        batch = max(1, (128 << 20) // (n * n * 8))
        sizes = np.full(batch, n, dtype=np.int32)
        offs = np.arange(batch, dtype=np.int64) * n * n
        rng = inputs.rng_for(0, 9900 + n)
        A = torch.from_numpy(rng.uniform(-1, 1, batch * n * n)).cuda()
        for b in range(batch):   # diagonally weighted, like the single-matrix workload
            A[b * n * n: (b + 1) * n * n: n + 1] += 4.0
        opts = gj.make_opts(precision=prec)
        X = torch.empty_like(A)
        poff = np.arange(batch, dtype=np.int64) * n
        ip = torch.empty(batch * n, dtype=torch.int32, device="cuda")
        jp = torch.empty_like(ip)
        res = torch.empty(batch * gj.RESULT_BYTES, dtype=torch.uint8, device="cuda")
        state = {}

        def run():
            ws = state.get("ws")
            need = gj.gj_workspace_size(gj.GJ_OP_INVERT_BATCHED, batch, sizes, opts)
            if ws is None or ws.numel() < need:
                ws = state["ws"] = torch.empty(need, dtype=torch.uint8, device="cuda")
            gj.gj_invert_batched(sizes, offs, A, X, poff, ip, jp, res, opts, ws)
        return run
    A = torch.from_numpy(inputs.single_dominant(n)).cuda()
    opts = gj.make_opts(precision=prec)
    X = torch.empty_like(A)
    ip = torch.empty(n, dtype=torch.int32, device="cuda")
    jp = torch.empty_like(ip)
    res = torch.empty(gj.RESULT_BYTES, dtype=torch.uint8, device="cuda")
    state = {}

    def run():
        ws = state.get("ws")
        need = gj.gj_workspace_size(gj.GJ_OP_INVERT, n, None, opts)
        if ws is None or ws.numel() < need:
            ws = state["ws"] = torch.empty(need, dtype=torch.uint8, device="cuda")
        gj.gj_invert(A, X, ip, jp, res, opts, ws)
    return run


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(HERE, "gj_tune.txt"))
    ap.add_argument("--quick", action="store_true", help="one repetition per candidate")
    ap.add_argument("--max-n", type=int, default=8192)
    args = ap.parse_args(argv)
    sys.path.insert(0, os.path.dirname(HERE))
    import torch  # noqa: F401
    import paper_1401_7962_amd as gj
    from paper_1401_7962_amd import inputs
    gj.load_library()
    lines, report = [], []
    for fp32 in (False, True):
        for lo, hi in BUCKETS:
            if lo > args.max_n:
                continue
            n = hi
            run = _workload(n, fp32, gj, inputs)
            times = {}
            for R in CANDIDATES:
                os.environ["GJ_BIG_ROWS"] = str(R)
                ms = _time(run, 1 if args.quick or n >= 4096 else 2)
                times[R] = ms
                print(f"tune {'f32' if fp32 else 'f64'} n={n} R={R}: {ms:.2f} ms", flush=True)
            best = min(times, key=times.get)
            os.environ["GJ_BIG_ROWS"] = str(best)
            ctimes = {0: times[best]}
            for pct in COUNTED:
                os.environ["GJ_BIG_COUNTED"] = str(pct)
                ctimes[pct] = _time(run, 1 if args.quick or n >= 4096 else 2)
                print(f"tune {'f32' if fp32 else 'f64'} n={n} R={best} counted={pct}%: "
                      f"{ctimes[pct]:.2f} ms", flush=True)
            os.environ.pop("GJ_BIG_COUNTED", None)
            pct = min(ctimes, key=ctimes.get)
            if ctimes[pct] > 0.99 * ctimes[0]:   # keep the barrier-free sweep unless it clearly loses
                pct = 0
            chtimes = {8: times[best]}
            if pct == 0 and n > 1024:   # the counter needs all 8 chunks
                for ch in CHUNKS:
                    os.environ["GJ_BIG_CHUNKS"] = str(ch)
                    chtimes[ch] = _time(run, 1 if args.quick or n >= 4096 else 2)
                    print(f"tune {'f32' if fp32 else 'f64'} n={n} R={best} chunks={ch}: "
                          f"{chtimes[ch]:.2f} ms", flush=True)
                os.environ.pop("GJ_BIG_CHUNKS", None)
            os.environ.pop("GJ_BIG_ROWS", None)
            ch = min(chtimes, key=chtimes.get)
            if chtimes[ch] > 0.99 * chtimes[8]:
                ch = 8
            lines.append(f"big_rows {'f32' if fp32 else 'f64'} {lo} {hi} {best} {pct} {ch}")
            report.append({"prec": "f32" if fp32 else "f64", "bucket": [lo, hi], "n": n,
                           "ms": times, "best": best, "counted_ms": ctimes, "counted": pct,
                           "chunks_ms": chtimes, "chunks": ch})
            del run
            torch.cuda.empty_cache()
    with open(args.out, "w") as f:
        f.write("# streaming elimination: rows per workgroup, chosen by paper_1401_7962_amd/tune.py\n")
        f.write("# big_rows <precision> <n_min> <n_max> <rows> <counted %> [<chunks per thread>]\n")
        f.write("\n".join(lines) + "\n")
    print(json.dumps(report), flush=True)


if __name__ == "__main__":
    main()
