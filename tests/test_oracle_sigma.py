"""Pins for the oracle's PPL product (oracle/ppl.py).

Each check is chosen so that a plausible slip (dropped partner term, wrong
sign in the antisymmetrisation, swapped index of L, lost factor 2) fails at
least one of them.
"""
import numpy as np
import pytest

import lrcc_synth as S
from oracle import ppl


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("o,v,P,herm", [(3, 6, 4, True), (3, 7, 3, False),
                                        (2, 5, 2, False)])
def test_definition_matches_bruteforce(o, v, P, herm):
    rng = np.random.default_rng(11 + v)
    L = S.make_L(rng, P, v, hermitian=herm)
    X = S.make_packed(rng, 2, o, v)
    ref = ppl.sigma_bruteforce(L, X, o, v)
    assert rel(ppl.sigma(L, X, o, v), ref) < 1e-13


@pytest.mark.parametrize("herm", [True, False])
def test_factored_identity(herm):
    rng = np.random.default_rng(3)
    o, v, P = 4, 13, 20
    L = S.make_L(rng, P, v, hermitian=herm)
    X = S.make_packed(rng, 3, o, v)
    assert rel(ppl.sigma_factored(L, X, o, v), ppl.sigma(L, X, o, v)) < 1e-13


def test_entries_match_definition():
    rng = np.random.default_rng(4)
    o, v, P = 4, 17, 12
    L = S.make_L(rng, P, v, hermitian=False)
    X = S.make_packed(rng, 2, o, v)
    full = ppl.sigma(L, X, o, v).reshape(-1, ppl.pairs(v)[0].size)
    rows = [0, 5, 11]
    pa, pb = ppl.pairs(v)
    ks = [0, 7, 40, len(pa) - 1]
    got = ppl.sigma_entries(L, X, v, rows, [(pa[k], pb[k]) for k in ks])
    assert rel(got, full[np.ix_(rows, ks)]) < 1e-13


def test_zero_L_gives_zero():
    rng = np.random.default_rng(5)
    X = S.make_packed(rng, 1, 3, 9)
    assert np.all(ppl.sigma(np.zeros((4, 9, 9), complex), X, 3, 9) == 0)


def test_rank_one_hermitian_vectors_cancel():
    # L^P = u u^H: <ab|cd> = u_a u*_c u_b u*_d = <ab|dc>, so <ab||cd> = 0.
    rng = np.random.default_rng(6)
    v, o = 10, 3
    L = np.stack([np.outer(u, np.conj(u)) for u in S.cn(rng, (3, v))])
    X = S.make_packed(rng, 2, o, v)
    s = ppl.sigma(L, X, o, v)
    scale = np.linalg.norm(L) ** 2 * np.linalg.norm(X)
    assert np.linalg.norm(s) < 1e-14 * scale


def test_diagonal_vectors_closed_form():
    # L^P = diag(lam^P): <ab||cd> = sum_P lam_a lam_b (d_ac d_bd - d_ad d_bc)
    # and the unrestricted sum gives sigma^ab = 2 sum_P lam_a lam_b X^ab.
    rng = np.random.default_rng(7)
    v, o, P = 11, 4, 5
    lam = S.cn(rng, (P, v))
    L = np.stack([np.diag(x) for x in lam])
    X = S.make_packed(rng, 2, o, v)
    pa, pb = ppl.pairs(v)
    expect = 2.0 * np.sum(lam[:, pa] * lam[:, pb], axis=0)[None, None, :] * X
    assert rel(ppl.sigma(L, X, o, v), expect) < 1e-14


def test_antisymmetric_and_symmetric_part_annihilated():
    rng = np.random.default_rng(8)
    v, P = 9, 6
    L = S.make_L(rng, P, v, hermitian=False)
    A = S.cn(rng, (3, v, v))
    Xa = A - np.swapaxes(A, 1, 2)
    Xs = A + np.swapaxes(A, 1, 2)
    sa = ppl.sigma_full(L, Xa)
    assert np.linalg.norm(sa + np.swapaxes(sa, 1, 2)) < 1e-13 * np.linalg.norm(sa)
    # a symmetric X is annihilated by the antisymmetrised integral
    assert np.linalg.norm(ppl.sigma_full(L, Xs)) < 1e-13 * np.linalg.norm(sa)


def test_linear_in_X_quadratic_in_L_pair_local():
    rng = np.random.default_rng(9)
    o, v, P = 4, 10, 7
    L = S.make_L(rng, P, v, hermitian=False)
    X1, X2 = S.make_packed(rng, 2, o, v), S.make_packed(rng, 2, o, v)
    a, g = 0.3 - 1.1j, 0.7 + 0.2j
    s = lambda LL, XX: ppl.sigma(LL, XX, o, v)
    assert rel(s(L, a * X1 + X2), a * s(L, X1) + s(L, X2)) < 1e-13
    assert rel(s(g * L, X1), g * g * s(L, X1)) < 1e-13
    # sigma_ij depends on X_ij only
    Y = X1.copy()
    Y[1, 2] += S.cn(rng, Y.shape[-1])
    d = s(L, Y) - s(L, X1)
    mask = np.zeros(d.shape[:2], bool)
    mask[1, 2] = True
    assert np.abs(d[~mask]).max() == 0.0 and np.abs(d[mask]).max() > 0


def test_hermitian_vectors_give_hermitian_operator():
    rng = np.random.default_rng(10)
    o, v, P = 3, 12, 9
    L = S.make_L(rng, P, v, hermitian=True)
    X, Y = S.make_packed(rng, 2, o, v), S.make_packed(rng, 2, o, v)
    lhs = np.vdot(Y, ppl.sigma(L, X, o, v))
    rhs = np.vdot(ppl.sigma(L, Y, o, v), X)
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)
    K = ppl.ladder_matrix(L, v)
    assert np.linalg.norm(K - np.conj(K.T)) < 1e-13 * np.linalg.norm(K)


def test_adjoint_identity_general_vectors():
    rng = np.random.default_rng(12)
    o, v, P = 3, 11, 6
    L = S.make_L(rng, P, v, hermitian=False)
    X, G = S.make_packed(rng, 2, o, v), S.make_packed(rng, 2, o, v)
    LH = np.conj(np.transpose(L, (0, 2, 1)))
    lhs = np.vdot(G, ppl.sigma(L, X, o, v))
    rhs = np.vdot(ppl.sigma(LH, G, o, v), X)
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)


def test_ladder_matrix_applies_sigma():
    rng = np.random.default_rng(13)
    o, v, P = 3, 8, 5
    L = S.make_L(rng, P, v, hermitian=False)
    X = S.make_packed(rng, 1, o, v)
    K = ppl.ladder_matrix(L, v)
    assert rel(np.einsum("pq,rmq->rmp", K, X), ppl.sigma(L, X, o, v)) < 1e-13


def test_pack_unpack_roundtrip_and_order():
    v = 6
    pa, pb = ppl.pairs(v)
    # row-major upper triangle: index of (a, b) is a(2v-a-1)/2 + (b-a-1)
    for k, (a, b) in enumerate(zip(pa, pb)):
        assert k == a * (2 * v - a - 1) // 2 + (b - a - 1)
    rng = np.random.default_rng(14)
    x = S.cn(rng, (2, len(pa)))
    f = ppl.unpack(x, v)
    assert np.all(f == -np.swapaxes(f, -1, -2))
    assert np.all(ppl.pack(f) == x)
