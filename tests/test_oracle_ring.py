"""Pins of the ring-term oracle (oracle/ring.py): the Fock-space matrix
element of the normal-ordered two-electron operator between doubles, a
second route that never forms the integrals, Hermiticity and structure."""
import itertools

import numpy as np
import pytest

import lrcc_synth as S
from fock import Fock
from oracle import hhl, ppl, response, ring


def blocks(Lfull, o):
    return (Lfull[:, :o, o:], Lfull[:, o:, :o], Lfull[:, :o, :o], Lfull[:, o:, o:])


def test_ring_is_the_two_body_matrix_element():
    """<ij->ab| W_N |Psi_X> = 1/2 PPL + 1/2 HHL + RING for the normal-ordered
    two-electron operator W_N built in the Fock space of 6 spinors from one
    Hermitian decomposition L^P over all of them (the ladders carry the
    doubled convention of ppl.py / hhl.py, hence the halves)."""
    o, v, nchol = 3, 3, 4
    n = o + v
    rng = np.random.default_rng(5)
    Lfull = S.make_L(rng, nchol, n, 1.0, True)
    Lov, Lvo, Loo, Lvv = blocks(Lfull, o)
    F = Fock(o, v)
    V = F.two_body(Lfull)
    g = np.einsum("Ppr,Pqs->pqrs", Lfull, Lfull)
    gas = g - np.transpose(g, (0, 1, 3, 2))
    G = sum(gas[:, i, :, i] for i in range(o))        # normal-ordering one-body part
    WN = V - F.one_body(G) + 0.5 * np.trace(G[:o, :o]) * np.eye(1 << n)
    assert abs(np.vdot(F.ref, WN @ F.ref)) < 1e-14
    X = S.make_packed(rng, 1, o, v)
    psi = np.zeros(1 << n, np.complex128)
    pij = list(zip(*np.triu_indices(o, 1)))
    pab = list(zip(*np.triu_indices(v, 1)))
    for (p, (i, j)), (q, (a, b)) in itertools.product(enumerate(pij), enumerate(pab)):
        psi += X[0, p, q] * F.double(i, j, a, b)
    out = WN @ psi
    got = np.array([[np.vdot(F.double(i, j, a, b), out) for (a, b) in pab] for (i, j) in pij])
    want = (0.5 * ppl.sigma(Lvv, X, o, v) + 0.5 * hhl.sigma(Loo, X, o, v)
            + ring.sigma(Lov, Lvo, Loo, Lvv, X, o, v))[0]
    np.testing.assert_allclose(got, want, atol=1e-13)
    # the model Jacobian with both ladders and the ring term applies exactly
    # this block (zero orbital energies: no Fock-diagonal part)
    AX = response.apply_jacobian(Lvv, X, np.zeros(n), o, v, Loo, (Lov, Lvo))[0]
    np.testing.assert_allclose(AX, got, atol=1e-13)
    Am = response.full_matrix(Lvv, np.zeros(n), o, v, Loo, (Lov, Lvo))
    np.testing.assert_allclose(Am @ X[0].reshape(-1), got.reshape(-1), atol=1e-13)


@pytest.mark.parametrize("o,v,nchol,nrhs,herm", [(3, 5, 4, 2, True), (5, 9, 7, 1, False),
                                                 (2, 2, 3, 1, True)])
def test_factored_route(o, v, nchol, nrhs, herm):
    rng = np.random.default_rng(o * 10 + v)
    Lfull = S.make_L(rng, nchol, o + v, 1.0, herm)
    X = S.make_packed(rng, nrhs, o, v)
    a = ring.sigma(*blocks(Lfull, o), X, o, v)
    b = ring.sigma_factored(*blocks(Lfull, o), X, o, v)
    np.testing.assert_allclose(a, b, atol=1e-12 * np.abs(a).max())


def test_hermitian_operator():
    """With one Hermitian decomposition the ring operator on packed doubles is
    Hermitian (a block of the Hermitian W_N)."""
    o, v = 3, 4
    Lfull = S.make_L(np.random.default_rng(2), 5, o + v, 1.0, True)
    R = ring.ring_matrix(*blocks(Lfull, o), o, v)
    np.testing.assert_allclose(R, np.conj(R.T), atol=1e-13)


def test_single_vector_closed_form():
    """One vector that couples only occupied 0 with virtual 0 (L_0a = L_a0* =
    1 for a = 0, all else 0): <kb||cj> = delta_k0 delta_c0 delta_b0 delta_j0,
    so sigma_ij^ab = P(ij)P(ab) delta_j0 delta_b0 X_i0^a0."""
    o, v = 3, 3
    Lfull = np.zeros((1, o + v, o + v), np.complex128)
    Lfull[0, 0, o] = 1.0
    Lfull[0, o, 0] = 1.0
    X = S.make_packed(np.random.default_rng(1), 1, o, v)
    got = ring.sigma(*blocks(Lfull, o), X, o, v)
    Xf = ppl.unpack_doubles(X, o, v)[0]
    r = np.zeros((o, o, v, v), np.complex128)
    for i, a in itertools.product(range(o), range(v)):
        r[i, 0, a, 0] = Xf[i, 0, a, 0]
    s = r - r.transpose(1, 0, 2, 3) - r.transpose(0, 1, 3, 2) + r.transpose(1, 0, 3, 2)
    np.testing.assert_allclose(got[0], ring.pack_doubles(s[None])[0], atol=1e-15)


def test_linear_and_zero():
    o, v = 4, 5
    rng = np.random.default_rng(3)
    Lfull = S.make_L(rng, 6, o + v, 1.0, True)
    X, Y = S.make_packed(rng, 1, o, v), S.make_packed(rng, 1, o, v)
    bl = blocks(Lfull, o)
    np.testing.assert_allclose(ring.sigma(*bl, 2 * X - 1j * Y, o, v),
                               2 * ring.sigma(*bl, X, o, v) - 1j * ring.sigma(*bl, Y, o, v),
                               atol=1e-12)
    assert np.abs(ring.sigma(*blocks(0 * Lfull, o), X, o, v)).max() == 0


# --- the ring term inside the model Jacobian ---------------------------------

from oracle import response  # noqa: E402

OMEGAS = [0.0, 0.0656]


def ring_instance(herm=True, seed=3, o=4, v=8, nchol=12):
    return S.make_instance(o, v, nchol, ncomp=2, seed=seed, gamma=S.solve_gamma(v),
                           hermitian=herm, ring=True)


def test_jacobian_matrix_and_apply_agree():
    inst = ring_instance(herm=False)
    o, v = inst.o, inst.v
    rg = (inst.Lov, inst.Lvo)
    A = response.full_matrix(inst.L, inst.eps, o, v, inst.Loo, rg)
    X = S.make_packed(np.random.default_rng(8), 1, o, v)
    got = response.apply_jacobian(inst.L, X, inst.eps, o, v, inst.Loo, rg)
    np.testing.assert_allclose(got.reshape(-1), A @ X.reshape(-1), atol=1e-12)


def test_coupled_solves_with_ring():
    """Dense solve = sum over states (Hermitian A, eigen route); the
    iterative Jacobi+DIIS solve converges to it; the full response function
    equals alpha(w) + conj alpha(-w); and the ring term moves alpha."""
    inst = ring_instance()
    o, v = inst.o, inst.v
    rg = (inst.Lov, inst.Lvo)
    A = response.full_matrix(inst.L, inst.eps, o, v, inst.Loo, rg)
    np.testing.assert_allclose(A, np.conj(A.T), atol=1e-14)
    assert np.linalg.eigvalsh(A).min() > 0.3
    dense = response.solve_dense_coupled(inst.L, inst.eps, inst.mu, OMEGAS, o, v, inst.Loo, rg)
    sos = response.solve_sos_coupled(inst.L, inst.eps, inst.mu, OMEGAS, o, v, inst.Loo, rg)
    np.testing.assert_allclose(dense["alpha"], sos["alpha"], atol=1e-12)
    it = response.solve_iterative(inst.L, inst.eps, inst.mu, OMEGAS, o, v, tol=1e-10,
                                  Loo=inst.Loo, ring=rg)
    np.testing.assert_allclose(it["alpha"], dense["alpha"], atol=1e-9)
    full = response.response_full_dense(inst.L, inst.eps, inst.mu, OMEGAS, o, v, inst.Loo, rg)
    minus = response.solve_dense_coupled(inst.L, inst.eps, inst.mu, [-w for w in OMEGAS], o, v,
                                         inst.Loo, rg)
    np.testing.assert_allclose(full["alpha"], dense["alpha"] + np.conj(minus["alpha"]),
                               atol=1e-12)
    no_ring = response.solve_dense_coupled(inst.L, inst.eps, inst.mu, OMEGAS, o, v, inst.Loo)
    d = np.abs(no_ring["alpha"] - dense["alpha"]).max() / np.abs(dense["alpha"]).max()
    assert d > 1e-4
