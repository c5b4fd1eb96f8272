"""The FP64 matrix-core product against NumPy's FP64 matmul (a library
primitive), with the bound K u |A||B| of any summation order."""
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


@pytest.mark.parametrize("M,N,K", [(16, 16, 4), (128, 128, 16), (1, 1, 1), (37, 91, 53),
                                   (128, 256, 512), (300, 200, 129), (1000, 64, 7), (512, 512, 512)])
def test_dgemm_shapes(gj, M, N, K):
    import torch
    rng = inputs.rng_for(0, 7000 + M + N + K)
    A, B, C = rng.standard_normal((M, K)), rng.standard_normal((K, N)), rng.standard_normal((M, N))
    for alpha, beta, gamma in ((1.0, 0.0, 0.0), (-1.0, 0.0, 1.0), (0.5, 1.0, 0.0), (-1.0, 1.0, 2.0)):
        Ad, Bd, Cd = (torch.from_numpy(x).to("cuda") for x in (A, B, C))
        D = gj.gj_dgemm(Ad, Bd, Cd, alpha=alpha, beta=beta, gamma=gamma)
        torch.cuda.synchronize()
        want = alpha * (A @ B) + beta * C + gamma * np.eye(M, N)
        bound = 4 * K * 2.0 ** -53 * (np.abs(A) @ np.abs(B)) + 1e-300
        assert np.all(np.abs(D.cpu().numpy() - want) <= bound + 4 * 2.0 ** -53 * np.abs(want)), (alpha, beta, gamma)


def test_dgemm_in_place(gj):
    import torch
    rng = inputs.rng_for(0, 7100)
    A, B, C = rng.standard_normal((200, 64)), rng.standard_normal((64, 200)), rng.standard_normal((200, 200))
    Cd = torch.from_numpy(C.copy()).to("cuda")
    gj.gj_dgemm(torch.from_numpy(A).to("cuda"), torch.from_numpy(B).to("cuda"), Cd, D=Cd,
                alpha=-1.0, beta=1.0)
    torch.cuda.synchronize()
    assert np.allclose(Cd.cpu().numpy(), C - A @ B, rtol=0, atol=1e-12)


@pytest.mark.parametrize("M,N,K", [(16, 16, 4), (128, 128, 16), (1, 1, 1), (37, 91, 53),
                                   (300, 200, 129), (512, 512, 512)])
def test_sgemm_shapes(gj, M, N, K):
    """The FP32 product (FP32 accumulation) against an FP64 NumPy product of
    the same FP32 operands, with the bound of FP32 summation in any order:
    it also pins the FP32 accumulator's lane layout (a wrong row map moves
    whole rows of the 16 x 16 blocks)."""
    import torch
    rng = inputs.rng_for(0, 7200 + M + N + K)
    A, B, C = (rng.standard_normal(s).astype(np.float32) for s in ((M, K), (K, N), (M, N)))
    for alpha, beta, gamma in ((1.0, 0.0, 0.0), (-1.0, 0.0, 1.0), (-1.0, 1.0, 2.0)):
        Ad, Bd, Cd = (torch.from_numpy(x).to("cuda") for x in (A, B, C))
        D = gj.gj_sgemm(Ad, Bd, Cd, alpha=alpha, beta=beta, gamma=gamma)
        torch.cuda.synchronize()
        A64, B64, C64 = A.astype(np.float64), B.astype(np.float64), C.astype(np.float64)
        want = alpha * (A64 @ B64) + beta * C64 + gamma * np.eye(M, N)
        u = 2.0 ** -24
        bound = (K + 4) * u * (np.abs(A64) @ np.abs(B64)) + 4 * u * (np.abs(C64) + np.abs(want)) + 1e-30
        assert np.all(np.abs(D.cpu().numpy().astype(np.float64) - want) <= bound), (alpha, beta, gamma)


def test_sgemm_rejects_wrong_dtype(gj):
    import torch
    A = torch.zeros((4, 4), dtype=torch.float64, device="cuda")
    with pytest.raises(gj.GJError):
        gj.gj_sgemm(A, A)
