"""GPU pivoted Cholesky decomposition (lrcc_cholesky) against the oracle."""
import numpy as np
import pytest

import lrcc_synth as S
from oracle import chol

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lrcc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_12914_amd as m
    return m


@pytest.mark.parametrize("n,rank,tau,decay", [(40, 12, 1e-10, 4.0), (300, 80, 1e-5, 6.0),
                                               (1500, 200, 1e-5, 16.0), (7, 7, 0.0, 2.0)])
def test_cholesky_matches_oracle(lrcc, n, rank, tau, decay):
    print(f"cholesky parity n={n} rank={rank} tau={tau}", flush=True)
    M = S.make_psd(np.random.default_rng(n), n, rank, decay)
    if tau == 0.0:
        M = M + np.eye(n)                      # full rank
    Lg, pg = lrcc.cholesky(torch.from_numpy(M).cuda(), tau)
    Lr, pr, dr = chol.pivoted_cholesky(M, tau)
    Lg = Lg.cpu().numpy()
    # the pivots are argmax decisions on FP64 values on both sides
    assert Lg.shape == Lr.shape and np.array_equal(pg, pr)
    assert np.abs(Lg - Lr).max() < 1e-12 * np.abs(Lr).max()
    R = M - Lg.T @ np.conj(Lg)
    assert np.real(np.diag(R)).max() <= max(tau, 1e-13 * np.abs(M).max())


def test_cholesky_cap_and_degenerate(lrcc):
    M = S.make_psd(np.random.default_rng(5), 64, 30)
    L, p = lrcc.cholesky(torch.from_numpy(M).cuda(), 0.0, max_vectors=10)
    Lr, pr, _ = chol.pivoted_cholesky(M, 0.0, max_vectors=10)
    assert L.shape[0] == 10 and np.array_equal(p, pr)
    assert np.abs(L.cpu().numpy() - Lr).max() < 1e-12 * np.abs(Lr).max()
    Z = torch.zeros((16, 16), dtype=torch.complex128).cuda()
    L, p = lrcc.cholesky(Z, 1e-8)
    assert L.shape == (0, 16) and len(p) == 0
    one = torch.full((1, 1), 4.0, dtype=torch.complex128).cuda()
    L, p = lrcc.cholesky(one, 1e-8)
    assert L.shape == (1, 1) and abs(complex(L[0, 0].item()) - 2.0) < 1e-15
    with pytest.raises(lrcc.LrccError):
        lrcc.cholesky(one, -1.0)
