"""Pins for the oracle's vector-Jacobian products (oracle/grads.py).

sigma is linear in X and quadratic in L, so a central finite difference is
exact up to rounding; h = 1e-6 in complex128.
"""
import numpy as np
import pytest

import lrcc_synth as S
from oracle import grads, ppl


def _fd(f, x, E, h=1e-6):
    return (f(x + h * E) - f(x - h * E)) / (2 * h)


@pytest.mark.parametrize("o,v,P,herm", [(3, 7, 4, False), (6, 36, 144, True)])
def test_finite_differences(o, v, P, herm):
    rng = np.random.default_rng(v)
    L = S.make_L(rng, P, v, hermitian=herm)
    X, G = S.make_packed(rng, 1, o, v), S.make_packed(rng, 1, o, v)
    loss_L = lambda LL: np.real(np.vdot(G, ppl.sigma(LL, X, o, v)))
    loss_X = lambda XX: np.real(np.vdot(G, ppl.sigma(L, XX, o, v)))
    gL = grads.vjp_L(L, X, G, o, v)
    gX = grads.vjp_X(L, G, o, v)
    for _ in range(2):
        EL = S.cn(rng, L.shape)
        EX = S.cn(rng, X.shape)
        fdL, fdX = _fd(loss_L, L, EL), _fd(loss_X, X, EX)
        assert abs(fdL - np.real(np.vdot(gL, EL))) < 1e-8 * abs(fdL)
        assert abs(fdX - np.real(np.vdot(gX, EX))) < 1e-8 * abs(fdX)


def test_elementwise_fd_of_L():
    # each component: d loss / d Re L + i d loss / d Im L == Lbar
    rng = np.random.default_rng(2)
    o, v, P = 3, 5, 2
    L = S.make_L(rng, P, v, hermitian=False)
    X, G = S.make_packed(rng, 2, o, v), S.make_packed(rng, 2, o, v)
    loss = lambda LL: np.real(np.vdot(G, ppl.sigma(LL, X, o, v)))
    gL = grads.vjp_L(L, X, G, o, v)
    for idx in [(0, 0, 0), (1, 2, 4), (0, 4, 1)]:
        E = np.zeros_like(L)
        E[idx] = 1.0
        dre = _fd(loss, L, E)
        dim = _fd(loss, L, 1j * E)
        assert abs(complex(dre, dim) - gL[idx]) < 1e-8 * max(1.0, abs(gL[idx]))


def test_adjoint_routes_agree():
    rng = np.random.default_rng(3)
    o, v, P = 3, 9, 5
    L = S.make_L(rng, P, v, hermitian=False)
    G = S.make_packed(rng, 2, o, v)
    a, b = grads.vjp_X(L, G, o, v), grads.vjp_X_explicit(L, G, o, v)
    assert np.linalg.norm(a - b) < 1e-13 * np.linalg.norm(b)


def test_sampled_L_entries_match_full_gradient_and_fd():
    # the entry-by-entry gradient used at full sizes: against the whole
    # gradient and, independently, against finite differences per element
    rng = np.random.default_rng(4)
    o, v, P = 4, 9, 3
    L = S.make_L(rng, P, v, hermitian=False)
    X, G = S.make_packed(rng, 2, o, v), S.make_packed(rng, 2, o, v)
    pairs = [(0, 0), (3, 7), (8, 1), (5, 5)]
    got = grads.vjp_L_entries(L, X, G, v, pairs)
    full = grads.vjp_L(L, X, G, o, v)
    for k, (a, c) in enumerate(pairs):
        assert np.abs(got[:, k] - full[:, a, c]).max() < 1e-13 * np.abs(full).max()
    loss = lambda LL: np.real(np.vdot(G, ppl.sigma(LL, X, o, v)))
    for (Pi, a, c) in [(0, 3, 7), (2, 8, 1)]:
        E = np.zeros_like(L)
        E[Pi, a, c] = 1.0
        fd = complex(_fd(loss, L, E), _fd(loss, L, 1j * E))
        k = pairs.index((a, c))
        assert abs(fd - got[Pi, k]) < 1e-8 * max(1.0, abs(fd))


def test_packed_row_is_the_unpacked_row():
    rng = np.random.default_rng(5)
    n = 7
    Xp = S.cn(rng, (3, n * (n - 1) // 2))
    full = ppl.unpack(Xp, n)
    for p in range(n):
        assert np.array_equal(ppl.packed_row(Xp, n, p), full[:, p, :])
