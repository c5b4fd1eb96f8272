"""Calls from several host threads at once, each on its own stream with its
own buffers and workspaces.  The batched call runs its one-matrix-per-
wavefront classes and the refined single-matrix call its FP64 fallback on the
device's one shared second stream, whose fork and join events a lock guards;
every result must equal the one a lone serial call produced, bit for bit."""
import threading

import numpy as np
import pytest

from paper_1401_7962_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gj():
    import torch  # noqa: F401
    import paper_1401_7962_amd as m
    m.load_library()
    return m


def test_threads_share_the_second_stream(gj):
    import torch
    rng = inputs.rng_for(0, 9100)
    sizes = np.array([8, 20, 33, 50, 64, 70, 100, 128, 140, 260], dtype=np.int32)
    mats = [rng.standard_normal((int(n), int(n))) for n in sizes]
    offs = np.zeros(len(sizes), dtype=np.int64)
    offs[1:] = np.cumsum(sizes.astype(np.int64) ** 2)[:-1]
    Ab = torch.from_numpy(np.concatenate([m.ravel() for m in mats])).cuda()
    As = torch.from_numpy(inputs.conditioned(260, 1e3, rng)).cuda()
    refined = gj.make_opts(precision=gj.GJ_PREC_FP32_REFINED)

    def run_once():
        Xb, ib, jb, rb, _ = gj.gj_invert_batched(sizes, offs, Ab)
        Xs, is_, js, rs = gj.gj_invert(As, opts=refined)
        return (Xb, ib, jb, rb, Xs, is_, js, rs)

    torch.cuda.synchronize()
    want = [t.cpu().numpy().copy() for t in run_once()]
    torch.cuda.synchronize()
    assert gj.results_to_dicts(torch.from_numpy(want[7]))[0]["code"] == 0

    failures = []

    def worker(k):
        try:
            st = torch.cuda.Stream()
            with torch.cuda.stream(st):
                for rep in range(4):
                    got = run_once()
                    st.synchronize()
                    for i, (a, b) in enumerate(zip(got, want)):
                        if a.cpu().numpy().tobytes() != b.tobytes():
                            failures.append(f"thread {k} call {rep} output {i} differs")
                            return
        except Exception as e:   # reported below, in the main thread
            failures.append(f"thread {k}: {e!r}")

    threads = [threading.Thread(target=worker, args=(k,)) for k in range(3)]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=90)
    assert not any(t.is_alive() for t in threads), "a worker thread did not finish"
    assert not failures, failures
