"""Pins for the oracle's pivoted Cholesky decomposition (oracle/chol.py)."""
import numpy as np
import pytest

import lrcc_synth as S
from oracle import chol


def recon(L):
    return L.T @ np.conj(L)           # sum_q L_q L_q^H


@pytest.mark.parametrize("n,rank", [(30, 8), (64, 20)])
def test_exact_low_rank_is_recovered(n, rank):
    M = S.make_psd(np.random.default_rng(n), n, rank)
    L, piv, d = chol.pivoted_cholesky(M, 1e-12)
    assert L.shape[0] == rank
    assert np.abs(recon(L) - M).max() < 1e-12 * np.abs(M).max()
    assert d.max() <= 1e-12 and len(set(piv.tolist())) == rank


def test_full_rank_equals_library_cholesky_of_the_permuted_matrix():
    rng = np.random.default_rng(2)
    A = S.cn(rng, (9, 9))
    M = A @ np.conj(A.T) + np.eye(9)
    L, piv, d = chol.pivoted_cholesky(M, 0.0)
    assert L.shape[0] == 9
    C = np.linalg.cholesky(M[np.ix_(piv, piv)])       # M[piv][:, piv] = C C^H
    assert np.abs(L[:, piv].T - C).max() < 1e-12 * np.abs(C).max()


def test_stopping_rule_and_pivot_order():
    M = S.make_psd(np.random.default_rng(7), 50, 40, decay=3.0)
    tau = 1e-5
    L, piv, d = chol.pivoted_cholesky(M, tau)
    k = L.shape[0]
    assert 0 < k < 40
    assert d.max() <= tau                               # stopped below tau
    # one step earlier the largest remaining diagonal element was above tau
    Lm, _, dm = chol.pivoted_cholesky(M, tau, max_vectors=k - 1)
    assert dm.max() > tau and np.array_equal(Lm, L[:k - 1])
    # the first pivot is the largest diagonal element; pivots never repeat
    assert piv[0] == int(np.argmax(np.real(np.diag(M))))
    assert len(set(piv.tolist())) == k
    # the residual diagonal is what the vectors leave unexplained
    assert np.abs(np.real(np.diag(M - recon(L))) - d).max() < 1e-12 * np.abs(M).max()


def test_zero_matrix_and_cap():
    L, piv, d = chol.pivoted_cholesky(np.zeros((5, 5), complex), 1e-8)
    assert L.shape == (0, 5) and len(piv) == 0
    M = S.make_psd(np.random.default_rng(3), 20, 10)
    L, piv, d = chol.pivoted_cholesky(M, 0.0, max_vectors=4)
    assert L.shape[0] == 4
