"""Pins for the oracle's hole-hole ladder (oracle/hhl.py) and the model
Jacobian that includes it (oracle/response.py, coupled solves)."""
import numpy as np
import pytest

import lrcc_synth as S
from oracle import hhl, ppl, response

OMEGAS = [0.0, 0.0428, 0.0656, 0.0856]


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("herm", [True, False])
@pytest.mark.parametrize("o,v,P", [(4, 3, 3), (5, 4, 2)])
def test_definition_matches_bruteforce(o, v, P, herm):
    rng = np.random.default_rng(10 + o)
    Loo = S.make_L(rng, P, o, hermitian=herm)
    X = S.make_packed(rng, 2, o, v)
    ref = hhl.sigma_bruteforce(Loo, X, o, v)
    assert rel(hhl.sigma(Loo, X, o, v), ref) < 1e-14
    # the second route: 2 sum_P (L^P)^T X^ab L^P
    assert rel(hhl.sigma_factored(Loo, X, o, v), ref) < 1e-13
    # the packed matrix W applies it
    W = hhl.hh_matrix(Loo, o)
    assert rel(np.einsum("pq,rqa->rpa", W, X), ref) < 1e-13


def test_zero_and_rank_one_hermitian_vectors():
    rng = np.random.default_rng(3)
    o, v = 6, 5
    X = S.make_packed(rng, 1, o, v)
    assert np.abs(hhl.sigma(np.zeros((2, o, o), complex), X, o, v)).max() == 0.0
    # L^P = u u^H: <kl|ij> - <kl|ji> = u_k u_l (conj(u_i u_j) - conj(u_j u_i)) = 0
    Loo = np.stack([np.outer(u, np.conj(u)) for u in S.cn(rng, (3, o))])
    assert np.abs(hhl.sigma(Loo, X, o, v)).max() < 1e-13 * np.abs(Loo).max() ** 2


@pytest.mark.parametrize("herm", [True, False])
def test_matrix_symmetries(herm):
    rng = np.random.default_rng(5)
    o = 6
    Loo = S.make_L(rng, 4, o, hermitian=herm)
    W = hhl.hh_matrix(Loo, o)
    Wt = hhl.hh_matrix(np.ascontiguousarray(Loo.transpose(0, 2, 1)), o)
    assert np.abs(Wt - W.T).max() < 1e-14 * np.abs(W).max()   # W(L^T) = W(L)^T
    if herm:
        assert np.abs(W - np.conj(W.T)).max() < 1e-14 * np.abs(W).max()


@pytest.mark.parametrize("o,v,P", [(4, 12, 24), (5, 10, 16)])
def test_coupled_solves_agree(o, v, P):
    inst = S.make_instance(o, v, P, ncomp=3, seed=1, gamma=S.solve_gamma(v), hh=True)
    dense = response.solve_dense_coupled(inst.L, inst.eps, inst.mu, OMEGAS, o, v, inst.Loo)
    sos = response.solve_sos_coupled(inst.L, inst.eps, inst.mu, OMEGAS, o, v, inst.Loo)
    it = response.solve_iterative(inst.L, inst.eps, inst.mu, OMEGAS, o, v, tol=1e-10,
                                  Loo=inst.Loo)
    assert rel(sos["alpha"], dense["alpha"]) < 1e-12
    assert rel(it["alpha"], dense["alpha"]) < 1e-9
    # the dense X solves the coupled response equation
    X = dense["X"][2]
    R = response.apply_jacobian(inst.L, X, inst.eps, o, v, inst.Loo) - OMEGAS[2] * X \
        + response.rhs(inst.mu, o, v)
    assert np.linalg.norm(R) < 1e-12 * np.linalg.norm(response.rhs(inst.mu, o, v))
    # without the hole-hole ladder the whole-vector solve is the per-pair one
    d0 = response.solve_dense_coupled(inst.L, inst.eps, inst.mu, OMEGAS, o, v, None)
    d1 = response.solve_dense(inst.L, inst.eps, inst.mu, OMEGAS, o, v)
    assert rel(d0["alpha"], d1["alpha"]) < 1e-13
    # and the hole-hole ladder moves alpha by a few per cent here
    assert rel(dense["alpha"], d1["alpha"]) > 1e-3


@pytest.mark.parametrize("herm", [True, False])
def test_coupled_left_solve_and_full_response(herm):
    o, v, P = 4, 10, 16
    inst = S.make_instance(o, v, P, ncomp=2, seed=2, gamma=S.solve_gamma(v), hh=True,
                           hermitian=herm)
    left = response.solve_left_dense_coupled(inst.L, inst.eps, inst.mu, OMEGAS, o, v, inst.Loo)
    Lt = np.ascontiguousarray(inst.L.transpose(0, 2, 1))
    Loot = np.ascontiguousarray(inst.Loo.transpose(0, 2, 1))
    it = response.solve_iterative(Lt, inst.eps, np.conj(inst.mu), [-w for w in OMEGAS], o, v,
                                  tol=1e-11, Loo=Loot)
    assert rel(it["alpha"], left["alpha_left"]) < 1e-9
    full = response.response_full_dense(inst.L, inst.eps, inst.mu, OMEGAS, o, v, inst.Loo)
    if herm:  # both sum-over-states terms of the whole Hermitian A
        a = response.solve_sos_coupled(inst.L, inst.eps, inst.mu, OMEGAS, o, v, inst.Loo)
        m = response.solve_sos_coupled(inst.L, inst.eps, inst.mu, [-w for w in OMEGAS], o, v,
                                       inst.Loo)
        assert rel(full["alpha"], a["alpha"] + np.conj(m["alpha"])) < 1e-12
