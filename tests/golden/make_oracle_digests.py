"""Write tests/golden/oracle_digests.json: what the FP64 oracle returns for
the large orders the benchmark runs, stored as SHA-256 digests so that the
GPU tests can compare bit for bit without running the oracle there.

Calls only ``oracle`` (the parallel form, which the CPU tests hold bitwise
equal to the serial oracle) and the seeded generators in
``paper_1401_7962_amd.inputs``.  Digests are of the raw little-endian bytes
in C order: X as float64 (n x n), ipiv and jpiv as int32.

    python tests/golden/make_oracle_digests.py            # every case
    python tests/golden/make_oracle_digests.py dominant_4096
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_1401_7962_amd import inputs  # noqa: E402

OUT = os.path.join(HERE, "oracle_digests.json")

# name -> (generator call as text, function building the input)
CASES = {
    # the headline workload: U[-1,1] + 4I at 4096
    "dominant_4096": ("inputs.single_dominant(4096)", lambda: inputs.single_dominant(4096)),
    # the largest plain order the benchmark runs, same recipe
    "dominant_8192": ("inputs.single_dominant(8192)", lambda: inputs.single_dominant(8192)),
    # a ragged order in the same size bucket as 8192
    "dominant_7777": ("inputs.single_dominant(7777, offset=77)",
                      lambda: inputs.single_dominant(7777, offset=77)),
}


def sha(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def digest(name: str) -> dict:
    call, make = CASES[name]
    A = make()
    n = A.shape[0]
    threads = oracle.host_threads()
    t0 = time.perf_counter()
    X, ipiv, jpiv, r = oracle.gj_invert_f64_par(A, threads)
    dt = time.perf_counter() - t0
    return {
        "input": call,
        "n": n,
        "sha256_A": sha(A.astype("<f8")),
        "sha256_X": sha(X.astype("<f8")),
        "sha256_ipiv": sha(ipiv.astype("<i4")),
        "sha256_jpiv": sha(jpiv.astype("<i4")),
        "code": int(r["code"]),
        "rank": int(r["rank"]),
        "det_sign": int(r["det_sign"]),
        "det_mant_hex": float(r["det_mant"]).hex(),
        "det_exp": int(r["det_exp"]),
        "logabsdet": float(r["logabsdet"]),
        "x_row0_first8_hex": [float(v).hex() for v in X[0, :8]],
        "oracle_seconds": round(dt, 1),
        "oracle_threads": threads,
    }


def main(names):
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for name in names:
        print(f"oracle: {name} ...", flush=True)
        data[name] = digest(name)
        print(f"oracle: {name} done in {data[name]['oracle_seconds']} s", flush=True)
        with open(OUT, "w") as fh:
            json.dump(data, fh, indent=1, sort_keys=True)
            fh.write("\n")


if __name__ == "__main__":
    main(sys.argv[1:] or list(CASES))
