"""Pins of the FNS++ oracle (perturbation-sensitive natural spinors, Sec. 2.4,
with the diagonalisation, Fock transform and semicanonicalisation of Sec. 2.3).

The amplitude, perturbation and density formulas are checked against second
quantisation done by brute force: creation and annihilation operators as
matrices on the full Fock space of a few spinors (Jordan-Wigner signs), the
first-order wave function as a Fock-space vector, the commutator of the
perturbation with the doubles operator and the density as an expectation
value.  None of that shares an index convention with the einsum code.
"""
import itertools

import numpy as np
import pytest

import lrcc_synth
from fock import Fock
from oracle import fns


def full_operator(inst, x):
    """The Hermitian one-body matrix over all spinors from its stored blocks."""
    o, v = inst.o, inst.v
    M = np.zeros((o + v, o + v), np.complex128)
    M[:o, :o] = inst.A_oo[x]
    M[o:, o:] = inst.A_vv[x]
    M[o:, :o] = inst.A_ov[x].T          # <a|A|i>
    M[:o, o:] = np.conj(inst.A_ov[x])   # <i|A|a> = conj <a|A|i>
    return M


@pytest.fixture(scope="module")
def tiny():
    inst = lrcc_synth.make_fns_instance(3, 4, 5, ncomp=2, seed=7)
    return inst, Fock(3, 4)


# ---------------------------------------------------------------------------

def test_fock_machinery_reproduces_amplitudes(tiny):
    """<ij->ab| T2 |ref> = t_ij^ab for every antisymmetric t (checks the
    Fock-space construction the other pins rely on)."""
    inst, F = tiny
    t, _ = fns.mp2_amplitudes(inst.eps, inst.Lov)
    psi = F.t2_op(t) @ F.ref
    for i, j, a, b in itertools.product(range(3), range(3), range(4), range(4)):
        if i < j and a < b:
            assert np.vdot(F.double(i, j, a, b), psi) == pytest.approx(t[i, j, a, b], abs=1e-15)


def test_mp2_amplitudes_antisymmetric_and_first_order(tiny):
    """t is antisymmetric in both pairs, and H0 t = -V|ref> projected on the
    doubles: (e_a + e_b - e_i - e_j) t_ij^ab = -<ij||ab>, the first-order
    Rayleigh-Schroedinger equation with H0 = sum_p e_p a+_p a_p."""
    inst, F = tiny
    t, W = fns.mp2_amplitudes(inst.eps, inst.Lov)
    np.testing.assert_allclose(t, -np.transpose(t, (1, 0, 2, 3)), atol=1e-17)
    np.testing.assert_allclose(t, -np.transpose(t, (0, 1, 3, 2)), atol=1e-17)
    H0 = F.one_body(np.diag(inst.eps).astype(np.complex128))
    psi = F.t2_op(t) @ F.ref
    e0 = np.vdot(F.ref, H0 @ F.ref).real
    lhs = H0 @ psi - e0 * psi             # (H0 - E0) |Psi1>
    rhs = -(F.t2_op(W) @ F.ref)           # -(doubles part of V|ref>), V|ref> ~ 1/4 sum W |ij->ab>
    np.testing.assert_allclose(lhs, rhs, atol=1e-15)
    # a brute-force double loop for <ij|ab> on one element
    i, j, a, b = 0, 2, 1, 3
    direct = sum(inst.Lov[P, i, a] * inst.Lov[P, j, b] - inst.Lov[P, i, b] * inst.Lov[P, j, a]
                 for P in range(inst.nchol))
    assert W[i, j, a, b] == pytest.approx(direct, abs=1e-17)


def test_perturbation_doubles_is_the_commutator(tiny):
    """Ab_ij^ac = <ij->ac| [A, T2] |ref> with A the oo and vv blocks of the
    one-body operator (the ov coupling switched off)."""
    inst, F = tiny
    t, _ = fns.mp2_amplitudes(inst.eps, inst.Lov)
    o, v = 3, 4
    for x in range(2):
        M = full_operator(inst, x)
        M[:o, o:] = 0
        M[o:, :o] = 0
        A = F.one_body(M)
        T = F.t2_op(t)
        comm = (A @ T - T @ A) @ F.ref
        Ab = fns.perturbation_doubles(t, inst.A_vv[x], inst.A_oo[x])
        for i, j, a, c in itertools.product(range(o), range(o), range(v), range(v)):
            if i < j and a < c:
                assert np.vdot(F.double(i, j, a, c), comm) == pytest.approx(Ab[i, j, a, c],
                                                                             abs=1e-15)
        np.testing.assert_allclose(Ab, -np.transpose(Ab, (1, 0, 2, 3)), atol=1e-16)
        np.testing.assert_allclose(Ab, -np.transpose(Ab, (0, 1, 3, 2)), atol=1e-16)


def test_identity_perturbation_has_no_response():
    """A multiple of the identity commutes with everything: Ab = 0, and a
    shift of the operator by c*I leaves the doubles unchanged."""
    inst = lrcc_synth.make_fns_instance(4, 6, 8, ncomp=1, seed=3)
    t, _ = fns.mp2_amplitudes(inst.eps, inst.Lov)
    Z = fns.perturbation_doubles(t, 1.7 * np.eye(6), 1.7 * np.eye(4))
    assert np.max(np.abs(Z)) < 1e-16
    base = fns.perturbation_doubles(t, inst.A_vv[0], inst.A_oo[0])
    shifted = fns.perturbation_doubles(t, inst.A_vv[0] - 0.4j * np.eye(6),
                                       inst.A_oo[0] - 0.4j * np.eye(4))
    np.testing.assert_allclose(shifted, base, atol=1e-16)


def test_singles_numerator_is_the_operator_element(tiny):
    """t_i^a(A) (Hb_aa - Hb_ii + w) = <i->a| A |ref>."""
    inst, F = tiny
    t, W = fns.mp2_amplitudes(inst.eps, inst.Lov)
    hi, ha = fns.dressed_diagonals(inst.eps, t, W)
    A = F.one_body(full_operator(inst, 1))
    drive = A @ F.ref
    _, t1 = fns.perturbed_amplitudes(t, inst.A_ov[1], inst.A_vv[1], inst.A_oo[1], hi, ha, 0.3)
    for i, a in itertools.product(range(3), range(4)):
        num = t1[i, a] * (ha[a] - hi[i] + 0.3)
        assert num == pytest.approx(np.vdot(F.single(i, a), drive), abs=1e-15)


def test_density_is_the_expectation_value(tiny):
    """G_ab = <Psi1| a+_b a_a |Psi1> for the first-order wave function built
    from the perturbed doubles and singles (both index placement and the
    factor 1/2 of the doubles part)."""
    inst, F = tiny
    t, W = fns.mp2_amplitudes(inst.eps, inst.Lov)
    hi, ha = fns.dressed_diagonals(inst.eps, t, W)
    t2, t1 = fns.perturbed_amplitudes(t, inst.A_ov[0], inst.A_vv[0], inst.A_oo[0], hi, ha, 0.1)
    psi = F.t2_op(t2) @ F.ref
    for i, a in itertools.product(range(3), range(4)):
        psi = psi + t1[i, a] * F.single(i, a)
    G = fns.density(t2, t1)
    for a, b in itertools.product(range(4), range(4)):
        op = F.c[F.vir(b)] @ F.a[F.vir(a)]
        assert G[a, b] == pytest.approx(np.vdot(psi, op @ psi), abs=1e-16)
    np.testing.assert_allclose(G, np.conj(G.T), atol=1e-18)
    assert np.min(np.linalg.eigvalsh(G)) > -1e-16


def test_dressed_diagonals_sum_rule(tiny):
    """sum_i (Hb_ii - e_i) = -sum_a (Hb_aa - e_a) = 2 E2, where E2 is the
    second-order energy, summed over the doubly excited determinants K of the
    Fock space with their couplings <K|V|ref> and energies <K|H0|K>."""
    inst, F = tiny
    o = 3
    t, W = fns.mp2_amplitudes(inst.eps, inst.Lov)
    hi, ha = fns.dressed_diagonals(inst.eps, t, W)
    # E2 = sum over distinct doubles |<K|V|ref>|^2 / (E_ref - E_K); both the
    # coupling and the energy difference come from Fock-space vectors.
    H0 = F.one_body(np.diag(inst.eps).astype(np.complex128))
    vref = F.t2_op(W) @ F.ref
    e0 = np.vdot(F.ref, H0 @ F.ref).real
    E2 = 0.0
    for i, j, a, b in itertools.product(range(3), range(3), range(4), range(4)):
        if i < j and a < b:
            K = F.double(i, j, a, b)
            E2 += abs(np.vdot(K, vref)) ** 2 / (e0 - np.vdot(K, H0 @ K).real)
    assert E2 < 0
    assert np.sum(hi - inst.eps[:o]) == pytest.approx(2 * E2, rel=1e-13)
    assert np.sum(ha - inst.eps[o:]) == pytest.approx(-2 * E2, rel=1e-13)


def test_dressed_diagonals_two_active_occupied():
    """Only occupied spinors 0 and 1 couple: each is lowered by E2 and the
    others keep their energies."""
    inst = lrcc_synth.make_fns_instance(4, 5, 6, ncomp=1, seed=11)
    Lov = inst.Lov.copy()
    Lov[:, 2:, :] = 0
    t, W = fns.mp2_amplitudes(inst.eps, Lov)
    hi, ha = fns.dressed_diagonals(inst.eps, t, W)
    eo, ev = inst.eps[:4], inst.eps[4:]
    E2 = 0.0
    for a in range(5):
        for b in range(5):
            E2 += 0.5 * abs(W[0, 1, a, b]) ** 2 / (eo[0] + eo[1] - ev[a] - ev[b])
    assert hi[0] - inst.eps[0] == pytest.approx(E2, rel=1e-13)
    assert hi[1] - inst.eps[1] == pytest.approx(E2, rel=1e-13)
    np.testing.assert_array_equal(hi[2:], inst.eps[2:4])


def test_basis_without_truncation_recovers_the_orbital_energies():
    """Keeping every natural spinor makes B unitary: the semicanonical
    energies are the virtual energies, sorted, and |B| is a permutation."""
    inst = lrcc_synth.make_fns_instance(4, 7, 10, ncomp=3, seed=5)
    o = 4
    r = fns.fns_plus(inst.eps, inst.Lov, inst.A_ov, inst.A_vv, inst.A_oo, 0.0656, 0.0)
    assert r["keep"] == 7
    np.testing.assert_allclose(r["eps_new"], np.sort(inst.eps[o:]), atol=1e-12)  # eps * |F|
    P = np.abs(r["B"])
    # F spans about three decades: eigenvectors are exact to about 1e-13
    np.testing.assert_allclose(np.sort(P.ravel())[-7:], np.ones(7), atol=1e-11)
    np.testing.assert_allclose(P @ P.T, np.eye(7), atol=1e-11)


def test_truncated_basis_properties():
    """Truncation keeps the |n| > threshold spinors: B is orthonormal,
    semicanonical (B^H F B diagonal with the returned energies) and spans an
    invariant subspace of G holding the kept occupations; the average over
    components is the mean of the per-component densities."""
    inst = lrcc_synth.make_fns_instance(5, 12, 16, ncomp=3, seed=9)
    o = 5
    thr = 3e-3
    r = fns.fns_plus(inst.eps, inst.Lov, inst.A_ov, inst.A_vv, inst.A_oo, 0.0428, thr)
    n, k, B, G = r["n"], r["keep"], r["B"], r["G"]
    assert k == int(np.sum(np.abs(n) > thr)) and 0 < k < 12
    assert np.all(np.diff(np.abs(n)) <= 0)
    np.testing.assert_allclose(np.conj(B.T) @ B, np.eye(k), atol=1e-13)
    Fv = np.diag(inst.eps[o:])
    np.testing.assert_allclose(np.conj(B.T) @ Fv @ B, np.diag(r["eps_new"]), atol=1e-12)
    np.testing.assert_allclose(G @ B, B @ (np.conj(B.T) @ G @ B), atol=1e-15)
    np.testing.assert_allclose(np.sort(np.linalg.eigvalsh(np.conj(B.T) @ G @ B)),
                               np.sort(n[:k]), atol=1e-15)
    np.testing.assert_allclose(np.sort(np.linalg.eigvalsh(G)), np.sort(n), atol=1e-15)
    t, W = fns.mp2_amplitudes(inst.eps, inst.Lov)
    hi, ha = fns.dressed_diagonals(inst.eps, t, W)
    parts = [fns.density(*fns.perturbed_amplitudes(t, inst.A_ov[x], inst.A_vv[x],
                                                   inst.A_oo[x], hi, ha, 0.0428))
             for x in range(3)]
    np.testing.assert_allclose(G, sum(parts) / 3, atol=1e-18)


def test_transformed_vectors_give_the_transformed_ladder():
    """With a unitary B (no truncation) the ladder of the transformed
    vectors on the transformed doubles is the transformed ladder:
    sigma(B^H L B)[X_t] = B^T-side transform of sigma(L)[X] with
    X_t^{kl} = sum_ab conj(B_ak) conj(B_bl) X^{ab} (both virtual indices);
    the spectra of the Hermitian L^P are kept; and a truncated B keeps the
    integrals of the kept spinors."""
    from oracle import ppl
    inst = lrcc_synth.make_fns_instance(4, 9, 12, ncomp=2, seed=4)
    o, v = 4, 9
    r = fns.fns_plus(inst.eps, inst.Lov, inst.A_ov, inst.A_vv, inst.A_oo, 0.0, 0.0)
    B = r["B"]
    assert B.shape == (v, v)
    rng = np.random.default_rng(1)
    L = lrcc_synth.make_L(rng, 6, v, 1.0, True)
    Lt = fns.transform_vectors(B, L)
    for P in range(6):
        np.testing.assert_allclose(np.linalg.eigvalsh(Lt[P]), np.linalg.eigvalsh(L[P]),
                                   atol=1e-12)
    X = lrcc_synth.make_packed(rng, 2, o, v)
    Xf = ppl.unpack(X, v)                                   # [r, ij, a, b]
    Xt = np.einsum("ak,bl,rpab->rpkl", np.conj(B), np.conj(B), Xf)
    got = ppl.sigma(Lt, ppl.pack(Xt), o, v)
    sf = ppl.unpack(ppl.sigma(L, X, o, v), v)
    want = ppl.pack(np.einsum("ak,bl,rpab->rpkl", np.conj(B), np.conj(B), sf))
    np.testing.assert_allclose(got, want, atol=1e-12 * np.abs(want).max())
    # a truncated basis: the first k columns give the sub-block of the above
    k = 5
    np.testing.assert_allclose(fns.transform_vectors(B[:, :k], L), Lt[:, :k, :k], atol=1e-14)
    mu = inst.A_ov
    np.testing.assert_allclose(fns.transform_dipole(mu, B[:, :k]), (mu @ np.conj(B))[:, :, :k],
                               atol=1e-15)


def test_response_is_invariant_under_the_full_basis_change():
    """Keeping every natural spinor is a unitary change of the virtual basis
    that keeps the Fock block diagonal: the model's alpha (dense solve) is
    the same in both bases, which fixes how each input transforms (vectors
    B^H L B, dipole with conj(B), energies eps_new)."""
    from oracle import response
    o, v, nchol = 4, 14, 20
    inst = lrcc_synth.make_fns_instance(o, v, nchol, ncomp=3, seed=12)
    L = lrcc_synth.make_L(np.random.default_rng(13), nchol, v, lrcc_synth.solve_gamma(v), True)
    om = [0.0, 0.0656]
    full = response.solve_dense(L, inst.eps, inst.A_ov, om, o, v)["alpha"]
    r = fns.fns_plus(inst.eps, inst.Lov, inst.A_ov, inst.A_vv, inst.A_oo, 0.0656, 0.0)
    assert r["keep"] == v
    eps_t = np.concatenate([inst.eps[:o], r["eps_new"]])
    red = response.solve_dense(fns.transform_vectors(r["B"], L), eps_t,
                               fns.transform_dipole(inst.A_ov, r["B"]), om, o, v)["alpha"]
    np.testing.assert_allclose(red, full, atol=1e-10 * np.abs(full).max())
