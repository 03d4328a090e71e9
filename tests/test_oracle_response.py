"""Pins for the oracle's model response problem (oracle/response.py)."""
import numpy as np
import pytest

import lrcc_synth as S
from oracle import ppl, response

OMEGAS = [0.0, 0.0428, 0.0656, 0.0856]


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def test_rhs_and_denominators_by_loops():
    rng = np.random.default_rng(1)
    o, v = 4, 6
    mu = S.cn(rng, (2, o, v), 0.1)
    eps = np.concatenate([rng.uniform(-2, -0.5, o), rng.uniform(0.1, 5, v)])
    xi = response.rhs(mu, o, v)
    D = response.denominators(eps, o, v)
    ij = 0
    for i in range(o):
        for j in range(i + 1, o):
            ab = 0
            for a in range(v):
                for b in range(a + 1, v):
                    for x in range(2):
                        m = mu[x]
                        want = m[i, a] * m[j, b] - m[i, b] * m[j, a]
                        assert abs(xi[x, ij, ab] - want) <= 1e-15 * abs(m).max() ** 2
                    assert D[ij, ab] == (eps[o + a] + eps[o + b]) - (eps[i] + eps[j])
                    ab += 1
            ij += 1
    # the full doubles image is antisymmetric in i<->j and a<->b
    full = ppl.unpack_doubles(xi, o, v)
    assert np.all(full == -np.swapaxes(full, 1, 2))
    assert np.all(full == -np.swapaxes(full, 3, 4))


def _closed_form(xi, Deff, omegas):
    return np.stack([np.einsum("xpq,ypq->xy", np.conj(xi), xi / (Deff - w))
                     for w in omegas])


def test_no_ladder_is_diagonal_jacobian_limit():
    inst = S.make_instance(3, 10, 4, ncomp=3, seed=2)
    L0 = np.zeros_like(inst.L)
    xi = response.rhs(inst.mu, 3, 10)
    D = response.denominators(inst.eps, 3, 10)
    expect = _closed_form(xi, D, OMEGAS)
    for fn in (response.solve_dense, response.solve_sos):
        assert rel(fn(L0, inst.eps, inst.mu, OMEGAS, 3, 10)["alpha"], expect) < 1e-13
    it = response.solve_iterative(L0, inst.eps, inst.mu, OMEGAS, 3, 10)
    assert rel(it["alpha"], expect) < 1e-13
    assert np.all(it["iters"] == 0)      # the Jacobi start is already exact


def test_diagonal_vectors_closed_form_solve():
    rng = np.random.default_rng(3)
    o, v, P = 3, 9, 4
    lam = 0.2 * rng.standard_normal((P, v))          # real: Hermitian L^P
    L = np.stack([np.diag(x).astype(complex) for x in lam])
    inst = S.make_instance(o, v, 1, ncomp=2, seed=3)
    pa, pb = ppl.pairs(v)
    shift = 2.0 * np.sum(lam[:, pa] * lam[:, pb], axis=0)
    xi = response.rhs(inst.mu, o, v)
    D = response.denominators(inst.eps, o, v) + shift[None, :]
    expect = _closed_form(xi, D, OMEGAS)
    got = response.solve_iterative(L, inst.eps, inst.mu, OMEGAS, o, v, tol=1e-12)
    assert rel(got["alpha"], expect) < 1e-11
    assert rel(response.solve_sos(L, inst.eps, inst.mu, OMEGAS, o, v)["alpha"],
               expect) < 1e-13


@pytest.mark.parametrize("o,v,P", [(4, 24, 64), (5, 30, 120)])
def test_three_solves_agree(o, v, P):
    inst = S.make_instance(o, v, P, ncomp=3, seed=0, gamma=S.solve_gamma(v))
    dense = response.solve_dense(inst.L, inst.eps, inst.mu, OMEGAS, o, v)
    sos = response.solve_sos(inst.L, inst.eps, inst.mu, OMEGAS, o, v)
    it = response.solve_iterative(inst.L, inst.eps, inst.mu, OMEGAS, o, v, tol=1e-8)
    assert rel(sos["alpha"], dense["alpha"]) < 1e-12
    assert np.all(it["relres"] < 1e-8)
    assert rel(it["alpha"], dense["alpha"]) < 1e-7
    # the packed X of the dense solve satisfies the response equation
    X = dense["X"][1]
    R = response.apply_jacobian(inst.L, X, inst.eps, o, v) - OMEGAS[1] * X \
        + response.rhs(inst.mu, o, v)
    assert np.linalg.norm(R) < 1e-12 * np.linalg.norm(response.rhs(inst.mu, o, v))


def test_alpha_hermitian_positive_increasing():
    o, v, P = 4, 24, 64
    inst = S.make_instance(o, v, P, ncomp=3, seed=0, gamma=S.solve_gamma(v))
    a = response.solve_dense(inst.L, inst.eps, inst.mu, OMEGAS, o, v)["alpha"]
    herm = a - np.conj(np.transpose(a, (0, 2, 1)))
    assert np.abs(herm).max() < 1e-12 * np.abs(a).max()
    # with complex random dipoles alpha is Hermitian but not symmetric
    assert np.abs(a - np.transpose(a, (0, 2, 1))).max() > 1e-6 * np.abs(a).max()
    zz = a[:, 2, 2]
    assert np.all(np.abs(zz.imag) < 1e-14 * np.abs(zz))
    assert zz.real[0] > 0 and np.all(np.diff(zz.real) > 0)


def test_literal_generator_does_not_converge():
    # Unscaled vectors: |K| ~ 5v Eh exceeds the smallest gap, the shifted
    # Jacobian is indefinite and Jacobi+DIIS does not reach the tolerance.
    inst = S.make_instance(4, 24, 64, ncomp=1, seed=0, gamma=1.0)
    it = response.solve_iterative(inst.L, inst.eps, inst.mu, [0.0], 4, 24,
                                  max_iter=30)
    assert it["relres"].min() > 1e-3
    assert np.linalg.norm(ppl.ladder_matrix(inst.L, 24), 2) > 50.0


def test_diis_singular_subspace_detected():
    rng = np.random.default_rng(4)
    e = S.cn(rng, 50)
    assert response._diis_coefficients([e, 2 * e]) is None
    c = response._diis_coefficients([e, S.cn(rng, 50)])
    assert abs(np.sum(c) - 1) < 1e-14


# --- left-hand amplitudes and the full response function (Sec. 2.2) -------

@pytest.mark.parametrize("herm", [True, False])
def test_transposed_vectors_give_the_transposed_ladder(herm):
    # K(L^T) = K(L)^T: the left-hand solve runs the ladder on transposed
    # Cholesky vectors; pinned on the explicit packed matrices
    rng = np.random.default_rng(31)
    v = 9
    L = S.make_L(rng, 7, v, hermitian=herm)
    Lt = np.ascontiguousarray(L.transpose(0, 2, 1))
    K = ppl.ladder_matrix(L, v)
    assert np.abs(ppl.ladder_matrix(Lt, v) - K.T).max() < 1e-14 * np.abs(K).max()
    if herm:  # Hermitian vectors: K^T = conj(K), not K
        assert np.abs(K.T - np.conj(K)).max() < 1e-14 * np.abs(K).max()
        assert np.abs(K.T - K).max() > 1e-3 * np.abs(K).max()


@pytest.mark.parametrize("herm", [True, False])
def test_left_solve_routes_agree(herm):
    # exact per-pair LU of (A + w)^T against Jacobi + DIIS on the transposed
    # vectors with the conjugate dipoles (eta = conj xi) and -w
    o, v, P = 3, 12, 24
    inst = S.make_instance(o, v, P, ncomp=2, seed=4, gamma=S.solve_gamma(v), hermitian=herm)
    left = response.solve_left_dense(inst.L, inst.eps, inst.mu, OMEGAS, o, v)
    Lt = np.ascontiguousarray(inst.L.transpose(0, 2, 1))
    it = response.solve_iterative(Lt, inst.eps, np.conj(inst.mu), [-w for w in OMEGAS], o, v,
                                  tol=1e-11)
    assert rel(it["alpha"], left["alpha_left"]) < 1e-9
    # each Y solves its own equation: Y (A + w) = -eta, row by row
    et = response.eta(inst.mu, o, v)
    D = response.denominators(inst.eps, o, v)
    K = ppl.ladder_matrix(inst.L, v)
    for w, om in enumerate(OMEGAS):
        Y = left["Y"][w]                                   # [comp, ij, ab]
        lhs = np.einsum("xpa,ab->xpb", Y, K) + Y * (D + om)[None]
        assert np.linalg.norm(lhs + et) < 1e-12 * np.linalg.norm(et)


def test_left_amplitudes_of_a_hermitian_operator():
    # Hermitian K: (A + w)^T = conj(A + w), so Y(w) = conj X(-w)
    o, v, P = 3, 12, 24
    inst = S.make_instance(o, v, P, ncomp=2, seed=5, gamma=S.solve_gamma(v))
    left = response.solve_left_dense(inst.L, inst.eps, inst.mu, OMEGAS, o, v)
    right_m = response.solve_dense(inst.L, inst.eps, inst.mu, [-w for w in OMEGAS], o, v)
    assert rel(left["Y"], np.conj(right_m["X"])) < 1e-12


def test_full_response_is_both_sum_over_states_terms():
    # the combined right/left response against the eigen-decomposition form
    # with the -w and +w denominators of Eq. (sos)
    o, v, P = 4, 16, 40
    inst = S.make_instance(o, v, P, ncomp=3, seed=6, gamma=S.solve_gamma(v))
    full = response.response_full_dense(inst.L, inst.eps, inst.mu, OMEGAS, o, v)
    sos = response.solve_sos_full(inst.L, inst.eps, inst.mu, OMEGAS, o, v)
    assert rel(full["alpha"], sos["alpha"]) < 1e-12
    a = full["alpha"]
    # Hermitian in the components; the static value is twice the Hermitian
    # right-hand alpha's real part; the zz component rises with w
    assert np.abs(a - np.conj(np.transpose(a, (0, 2, 1)))).max() < 1e-13 * np.abs(a).max()
    a0 = response.solve_dense(inst.L, inst.eps, inst.mu, [0.0], o, v)["alpha"][0]
    assert rel(a[0], a0 + np.conj(a0)) < 1e-12
    assert np.all(np.diff(a[:, 2, 2].real) > 0)
