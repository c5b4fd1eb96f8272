"""Drives the host side of libgj (argument checks, plan building, workspace
sizes, status strings) through ctypes, with no GPU call: loaded from a
library build whose host code carries AddressSanitizer and
UndefinedBehaviorSanitizer.  usage: python host_abi_driver.py <lib.so>"""
import ctypes
import sys

import numpy as np

lib = ctypes.CDLL(sys.argv[1])
P, I32, I64, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t


class Opts(ctypes.Structure):
    _fields_ = [("precision", I32), ("want_resid", I32), ("max_refine_iters", I32), ("flags", I32),
                ("zero_tol", ctypes.c_double), ("step_events", P * 2)]


def opts(prec=0, flags=0, resid=0):
    o = Opts()
    o.precision, o.flags, o.want_resid, o.max_refine_iters, o.zero_tol = prec, flags, resid, 10, -1.0
    return o


lib.gj_workspace_size.argtypes = [I32, I32, P, P]
lib.gj_workspace_size.restype = SZ
lib.gj_status_string.argtypes = [I32]
lib.gj_status_string.restype = ctypes.c_char_p
rng = np.random.default_rng(5)
# plans of many batches, both precisions, every option the batched call takes
for trial in range(40):
    batch = int(rng.integers(1, 400))
    sizes = rng.integers(1, 700 if trial % 4 else 4200, batch).astype(np.int32)
    for prec in (0, 1):
        o = opts(prec)
        lib.gj_workspace_size(2, batch, sizes.ctypes.data_as(P), ctypes.byref(o))
for n in list(range(1, 300)) + [1023, 1024, 1025, 4096, 8192, 16384, 16385]:
    for o in (opts(), opts(1), opts(0, 16), opts(1, 8), opts(0, 2), opts(0, 4), opts(0, 0, 1), opts(1, 0, 1)):
        lib.gj_workspace_size(0, n, None, ctypes.byref(o))
        lib.gj_workspace_size(1, n, None, ctypes.byref(o))
    m = np.array([max(1, n // 7)], dtype=np.int32)
    lib.gj_workspace_size(3, n, m.ctypes.data_as(P), None)
for code in list(range(-6, 2)) + [100, 101, 102, 103, 104]:
    lib.gj_status_string(code)
# argument checks that return before any HIP call
fake, A, X, ws = P(1 << 20), P(1 << 30), P(1 << 40), P(1 << 36)
lib.gj_invert.argtypes = [I32, P, I64, P, I64, P, P, P, P, P, SZ, P]
lib.gj_invert_batched.argtypes = [I32, P, P, P, P, P, P, P, P, P, P, SZ, P]
lib.gj_invert_noalloc.argtypes = [I32, P, I64, P, I64, P, P, P, P, P]
assert lib.gj_invert(0, A, 1, X, 1, fake, fake, fake, None, None, 0, None) == -1
assert lib.gj_invert(1000, A, 1000, X, 1000, fake, fake, fake, None, None, 0, None) == -2
assert lib.gj_invert_noalloc(5000, A, 5000, X, 5000, fake, fake, fake, None, None) == -4
n = np.array([4, 300, 70], dtype=np.int32)
off = np.array([0, 16, 16 + 90000], dtype=np.int64)
poff = np.array([0, 4, 304], dtype=np.int64)
reuse = opts(0, 1)
assert lib.gj_invert_batched(3, n.ctypes.data_as(P), off.ctypes.data_as(P), A, X, poff.ctypes.data_as(P),
                             fake, fake, fake, ctypes.byref(reuse), ws, 1 << 30, None) == -1
print("host driver: done")
