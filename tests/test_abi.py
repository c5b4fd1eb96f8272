"""The C-ABI library loads and exports every function include/gj.h declares;
argument checks reject bad calls before touching the GPU.  CPU only: no
compute call is made here."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import paper_1401_7962_amd as gj

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    text = open(os.path.join(ROOT, "include", "gj.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gj_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(gj.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return gj.load_library()


def test_header_lists_the_boundary():
    names = _header_functions()
    for f in ("gj_invert", "gj_invert_batched", "gj_det", "gj_solve", "gj_workspace_size",
              "gj_status_string"):
        assert f in names


def test_library_resolves_every_symbol_at_load():
    """RTLD_NOW: an undefined symbol fails here, not at the first call."""
    import torch  # noqa: F401  -- the HIP runtime the library binds to
    ctypes.CDLL(gj.LIB_PATH, mode=os.RTLD_NOW | os.RTLD_LOCAL)


def test_every_declared_symbol_is_exported(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", gj.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(line.split()[-1] for line in out.splitlines() if line.strip())
    for name in _header_functions():
        assert name in exported, name
        assert hasattr(lib, name)


def test_result_and_opts_layout():
    assert ctypes.sizeof(gj.gj_result) == 56
    assert gj.gj_result.det_mant.offset == 16 and gj.gj_result.resid.offset == 48
    assert ctypes.sizeof(gj.gj_opts) == 40


def test_status_strings(lib):
    for code in (0, -1, -2, -3, -4, 100, 101, 102, 103):
        assert gj.gj_status_string(code)
    assert gj.gj_status_string(-1).startswith("GJ_E_INVALID_ARG")


def test_workspace_size(lib):
    assert gj.gj_workspace_size(gj.GJ_OP_INVERT, 0) == 0
    assert gj.gj_workspace_size(gj.GJ_OP_INVERT, 64) >= 256           # on chip: no real workspace
    big = gj.gj_workspace_size(gj.GJ_OP_INVERT, 4096)
    assert big >= 4096 * 4096 * 8                                     # holds the working array
    assert gj.gj_workspace_size(gj.GJ_OP_INVERT, 20000) == 0         # beyond the supported order
    assert gj.gj_workspace_size(gj.GJ_OP_INVERT_BATCHED, 3, [5, 200, 64]) > 200 * 200 * 8
    assert gj.gj_workspace_size(gj.GJ_OP_INVERT_BATCHED, 2, [5, 0]) == 0
    bad = gj.make_opts(precision=7)
    assert gj.gj_workspace_size(gj.GJ_OP_INVERT, 64, None, bad) == 0
    # solve: m passed through the host-array argument; [A | B] is swept as one array
    sol = gj.gj_workspace_size(gj.GJ_OP_SOLVE, 4096, [16])
    assert sol >= 4096 * (4096 + 16) * 8
    assert gj.gj_workspace_size(gj.GJ_OP_SOLVE, 3, [1]) >= 256
    assert gj.gj_workspace_size(gj.GJ_OP_SOLVE, 4096, [0]) == 0
    assert gj.gj_workspace_size(gj.GJ_OP_SOLVE, 4096) == 0              # m missing
    assert gj.gj_workspace_size(gj.GJ_OP_SOLVE, 16000, [385]) == 0      # n + m beyond 16384
    fp32 = gj.make_opts(precision=gj.GJ_PREC_FP32_REFINED)
    assert gj.gj_workspace_size(gj.GJ_OP_SOLVE, 100, [2], fp32) == 0   # FP64 only
    # pivot rules: every order through the streaming kernels; FP64, single matrix only
    part = gj.make_opts(flags=gj.GJ_FLAG_PIVOT_PARTIAL)
    prog = gj.make_opts(flags=gj.GJ_FLAG_PIVOT_PROGRAM)
    assert gj.gj_workspace_size(gj.GJ_OP_INVERT, 64, None, part) > 64 * 64 * 8
    assert gj.gj_workspace_size(gj.GJ_OP_DET, 64, None, prog) > 64 * 64 * 8
    assert gj.gj_workspace_size(gj.GJ_OP_SOLVE, 64, [3], prog) > 64 * 67 * 8
    both = gj.make_opts(flags=gj.GJ_FLAG_PIVOT_PARTIAL | gj.GJ_FLAG_PIVOT_PROGRAM)
    assert gj.gj_workspace_size(gj.GJ_OP_INVERT, 64, None, both) == 0
    assert gj.gj_workspace_size(gj.GJ_OP_INVERT_BATCHED, 2, [5, 9], part) == 0
    p32 = gj.make_opts(precision=gj.GJ_PREC_FP32_REFINED, flags=gj.GJ_FLAG_PIVOT_PARTIAL)
    assert gj.gj_workspace_size(gj.GJ_OP_INVERT, 500, None, p32) == 0
    # accurate residuals: refined single matrices only; six more n^2 buffers
    acc = gj.make_opts(precision=gj.GJ_PREC_FP32_REFINED, flags=gj.GJ_FLAG_ACCURATE)
    ref = gj.make_opts(precision=gj.GJ_PREC_FP32_REFINED)
    assert (gj.gj_workspace_size(gj.GJ_OP_INVERT, 500, None, acc)
            >= gj.gj_workspace_size(gj.GJ_OP_INVERT, 500, None, ref) + 6 * 500 * 500 * 8)
    assert gj.gj_workspace_size(gj.GJ_OP_INVERT, 500, None, gj.make_opts(flags=gj.GJ_FLAG_ACCURATE)) == 0
    assert gj.gj_workspace_size(gj.GJ_OP_INVERT_BATCHED, 2, [5, 9], acc) == 0
    # delayed updates: two padded n x n arrays; orders up to 128 stay on chip (no workspace)
    blk = gj.make_opts(flags=gj.GJ_FLAG_BLOCKED)
    assert gj.gj_workspace_size(gj.GJ_OP_INVERT, 4096, None, blk) >= 2 * 4096 * 4096 * 8
    assert (gj.gj_workspace_size(gj.GJ_OP_INVERT, 64, None, blk)
            == gj.gj_workspace_size(gj.GJ_OP_INVERT, 64, None, gj.make_opts()))
    assert gj.gj_workspace_size(gj.GJ_OP_DET, 500, None, blk) == 0
    assert gj.gj_workspace_size(gj.GJ_OP_SOLVE, 500, [2], blk) == 0
    assert gj.gj_workspace_size(gj.GJ_OP_INVERT_BATCHED, 2, [5, 900], blk) == 0
    # the refined path's FP32 stage with delayed updates: two padded n x n FP32
    # arrays in place of the streaming one, the refinement's buffers as before
    rblk = gj.make_opts(precision=gj.GJ_PREC_FP32_REFINED, flags=gj.GJ_FLAG_BLOCKED)
    assert (gj.gj_workspace_size(gj.GJ_OP_INVERT, 4096, None, rblk)
            >= gj.gj_workspace_size(gj.GJ_OP_INVERT, 4096, None, ref) + 4096 * 4096 * 4)
    assert (gj.gj_workspace_size(gj.GJ_OP_INVERT, 100, None, rblk)
            == gj.gj_workspace_size(gj.GJ_OP_INVERT, 100, None, ref))
    assert gj.gj_workspace_size(gj.GJ_OP_INVERT_BATCHED, 2, [5, 900], rblk) == 0


def test_argument_checks_without_gpu(lib):
    P = ctypes.c_void_p
    fake = P(1 << 20)
    # n < 1, lda < n, NULL pointers and bad options are rejected synchronously
    assert lib.gj_invert(0, fake, 1, fake, 1, fake, fake, fake, None, None, 0, None) == gj.GJ_E_INVALID_ARG
    assert lib.gj_invert(4, fake, 3, fake, 4, fake, fake, fake, None, None, 0, None) == gj.GJ_E_INVALID_ARG
    assert lib.gj_invert(4, None, 4, fake, 4, fake, fake, fake, None, None, 0, None) == gj.GJ_E_INVALID_ARG
    o = gj.make_opts(flags=32)
    assert lib.gj_invert(4, fake, 4, P(1 << 24), 4, fake, fake, fake, ctypes.byref(o), None, 0,
                         None) == gj.GJ_E_INVALID_ARG
    # delayed updates: full search only; not for the determinant, solve or batches
    for bad in (gj.make_opts(flags=gj.GJ_FLAG_BLOCKED | gj.GJ_FLAG_PIVOT_PARTIAL),
                gj.make_opts(precision=gj.GJ_PREC_FP32_REFINED,
                             flags=gj.GJ_FLAG_BLOCKED | gj.GJ_FLAG_PIVOT_PROGRAM)):
        assert lib.gj_invert(4, fake, 4, P(1 << 24), 4, fake, fake, fake, ctypes.byref(bad), None, 0,
                             None) == gj.GJ_E_INVALID_ARG
    blk = gj.make_opts(flags=gj.GJ_FLAG_BLOCKED)
    assert lib.gj_det(300, P(1 << 30), 300, fake, fake, fake, ctypes.byref(blk), None, 0,
                      None) == gj.GJ_E_UNSUPPORTED
    assert lib.gj_solve(8, 2, P(1 << 30), 8, P(1 << 34), 2, P(1 << 38), 2, fake, fake, fake,
                        ctypes.byref(blk), None, 0, None) == gj.GJ_E_UNSUPPORTED
    assert lib.gj_invert(1000, P(1 << 30), 1000, P(1 << 40), 1000, fake, fake, fake, ctypes.byref(blk),
                         None, 0, None) == gj.GJ_E_WORKSPACE
    # X overlapping A
    assert lib.gj_invert(4, fake, 4, fake, 4, fake, fake, fake, None, None, 0, None) == gj.GJ_E_INVALID_ARG
    # large n needs a workspace
    assert lib.gj_invert(1000, P(1 << 30), 1000, P(1 << 40), 1000, fake, fake, fake, None, None, 0,
                         None) == gj.GJ_E_WORKSPACE
    assert lib.gj_det(0, fake, 1, fake, fake, fake, None, None, 0, None) == gj.GJ_E_INVALID_ARG
    # solve: m < 1, ldb < m, X over B, unsupported precision, missing workspace
    A, B, X = P(1 << 30), P(1 << 34), P(1 << 38)
    assert lib.gj_solve(8, 0, A, 8, B, 1, X, 1, fake, fake, fake, None, None, 0, None) == gj.GJ_E_INVALID_ARG
    assert lib.gj_solve(8, 2, A, 8, B, 1, X, 2, fake, fake, fake, None, None, 0, None) == gj.GJ_E_INVALID_ARG
    assert lib.gj_solve(8, 2, A, 8, B, 2, B, 2, fake, fake, fake, None, None, 0, None) == gj.GJ_E_INVALID_ARG
    o32 = gj.make_opts(precision=gj.GJ_PREC_FP32_REFINED)
    assert lib.gj_solve(8, 2, A, 8, B, 2, X, 2, fake, fake, fake, ctypes.byref(o32), None, 0,
                        None) == gj.GJ_E_UNSUPPORTED
    assert lib.gj_solve(16000, 385, A, 16000, B, 385, X, 385, fake, fake, fake, None, None, 0,
                        None) == gj.GJ_E_UNSUPPORTED
    assert lib.gj_solve(8, 2, A, 8, B, 2, X, 2, fake, fake, fake, None, None, 0, None) == gj.GJ_E_WORKSPACE
    # pivot rules: not both, not refined, not batched; a small order then needs a workspace
    both = gj.make_opts(flags=gj.GJ_FLAG_PIVOT_PARTIAL | gj.GJ_FLAG_PIVOT_PROGRAM)
    assert lib.gj_invert(8, A, 8, X, 8, fake, fake, fake, ctypes.byref(both), None, 0,
                         None) == gj.GJ_E_INVALID_ARG
    p32 = gj.make_opts(precision=gj.GJ_PREC_FP32_REFINED, flags=gj.GJ_FLAG_PIVOT_PROGRAM)
    assert lib.gj_invert(8, A, 8, X, 8, fake, fake, fake, ctypes.byref(p32), None, 0,
                         None) == gj.GJ_E_UNSUPPORTED
    part = gj.make_opts(flags=gj.GJ_FLAG_PIVOT_PARTIAL)
    assert lib.gj_invert(8, A, 8, X, 8, fake, fake, fake, ctypes.byref(part), None, 0,
                         None) == gj.GJ_E_WORKSPACE
    nb = np.array([4, 5], dtype=np.int32)
    ob = np.array([0, 16], dtype=np.int64)
    assert lib.gj_invert_batched(2, nb.ctypes.data_as(P), ob.ctypes.data_as(P), A, X,
                                 ob.ctypes.data_as(P), fake, fake, fake, ctypes.byref(part),
                                 P(1 << 28), 1 << 20, None) == gj.GJ_E_UNSUPPORTED
    n = np.array([4, 0], dtype=np.int32)
    off = np.zeros(2, dtype=np.int64)
    assert lib.gj_invert_batched(2, n.ctypes.data_as(P), off.ctypes.data_as(P), fake, P(1 << 24),
                                 off.ctypes.data_as(P), fake, fake, fake, None, P(1 << 28), 1 << 20,
                                 None) == gj.GJ_E_INVALID_ARG


def test_noalloc_and_batched_checks_without_gpu(lib):
    """Checks taken before any HIP call: gj_invert_noalloc refuses orders whose
    workspace exceeds its built-in array, and gj_invert_batched refuses A / X
    overlapping each other or the workspace, and a reused plan it never
    uploaded into that workspace."""
    P = ctypes.c_void_p
    fake = P(1 << 20)
    A, X = P(1 << 30), P(1 << 40)
    lib.gj_invert_noalloc.argtypes = [ctypes.c_int32, P, ctypes.c_int64, P, ctypes.c_int64, P, P,
                                      P, P, P]
    assert lib.gj_invert_noalloc(0, A, 1, X, 1, fake, fake, fake, None, None) == gj.GJ_E_INVALID_ARG
    assert lib.gj_invert_noalloc(4096, A, 4096, X, 4096, fake, fake, fake, None,
                                 None) == gj.GJ_E_UNSUPPORTED
    assert lib.gj_invert_noalloc(20000, A, 20000, X, 20000, fake, fake, fake, None,
                                 None) == gj.GJ_E_UNSUPPORTED
    assert gj.gj_workspace_size(gj.GJ_OP_INVERT, 2500) <= gj.NOALLOC_SCRATCH_BYTES
    n = np.array([4, 5], dtype=np.int32)
    off = np.array([0, 16], dtype=np.int64)
    poff = np.array([0, 4], dtype=np.int64)
    ws = P(1 << 36)
    # X starts inside A's span (A spans 16 + 25 elements)
    assert lib.gj_invert_batched(2, n.ctypes.data_as(P), off.ctypes.data_as(P), A,
                                 P((1 << 30) + 8 * 40), poff.ctypes.data_as(P), fake, fake, fake,
                                 None, ws, 1 << 20, None) == gj.GJ_E_INVALID_ARG
    # workspace over X
    assert lib.gj_invert_batched(2, n.ctypes.data_as(P), off.ctypes.data_as(P), A, X,
                                 poff.ctypes.data_as(P), fake, fake, fake, None, X, 1 << 20,
                                 None) == gj.GJ_E_INVALID_ARG
    reuse = gj.make_opts(flags=gj.GJ_FLAG_REUSE_PLAN)
    assert lib.gj_invert_batched(2, n.ctypes.data_as(P), off.ctypes.data_as(P), A, X,
                                 poff.ctypes.data_as(P), fake, fake, fake, ctypes.byref(reuse), ws,
                                 1 << 20, None) == gj.GJ_E_INVALID_ARG


def test_batch_plans_every_order(lib):
    """The host-side batch plans (plain and refined) over every order up to
    300, each on-chip task class included: they build without error and the
    workspace grows with the batch."""
    sizes = np.arange(1, 301, dtype=np.int32)
    for prec in (gj.GJ_PREC_FP64, gj.GJ_PREC_FP32_REFINED):
        o = gj.make_opts(precision=prec)
        full = gj.gj_workspace_size(gj.GJ_OP_INVERT_BATCHED, len(sizes), sizes, o)
        small = gj.gj_workspace_size(gj.GJ_OP_INVERT_BATCHED, 128, sizes[:128], o)
        assert 0 < small < full
        for n in range(1, 129):
            assert gj.gj_workspace_size(gj.GJ_OP_INVERT_BATCHED, 3, np.full(3, n, np.int32), o) > 0


def test_binding_refuses_without_library(tmp_path):
    with pytest.raises(gj.GJError):
        gj._lib_saved = gj._lib
        try:
            gj._lib = None
            gj.load_library(str(tmp_path / "missing.so"))
        finally:
            gj._lib = gj._lib_saved
