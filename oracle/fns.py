"""Perturbation-sensitive frozen natural spinors (FNS++) of the virtual space.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Paper, Sec. 2.3 (natural spinors) and Sec. 2.4 (FNS++), written out for a
canonical Hartree-Fock reference (F diagonal: F_ii = e_i, F_aa = e_a):

  MP2 amplitudes       t_ij^ab = <ij||ab> / (e_i + e_j - e_a - e_b),
                       <ij|ab> = sum_P L^P_ia L^P_jb (ov Cholesky vectors),
                       <ij||ab> = <ij|ab> - <ij|ba>
  dressed diagonals    Hb_ii = e_i + 1/2 sum_{n,e,f} t_in^ef conj<in||ef>
                       Hb_aa = e_a - 1/2 sum_{m,n,f} t_mn^fa conj<mn||fa>
  perturbed doubles    Ab_ij^ac = P(a,c) sum_e t_ij^ec A_ae - P(i,j) sum_m t_mj^ac A_mi
                       t_ij^ac(A) = Ab_ij^ac / (Hb_aa + Hb_cc - Hb_ii - Hb_jj + w)
  perturbed singles    t_i^a(A) = A_ia / (Hb_aa - Hb_ii + w)
  density              G^A_ab = 1/2 sum_{i,j,c} t_ij^ac(A) conj t_ij^bc(A)
                                + sum_i t_i^a(A) conj t_i^b(A),
                       averaged over the perturbation's components
  natural spinors      G V = V diag(n); keep |n| > threshold (largest first)
  semicanonical        Ft = Vt^H diag(e_v) Vt = Z diag(et) Z^H;  B = Vt Z

with A_ae = <a|A|e> (vv block, A_vv[a, e]), A_mi = <m|A|i> (oo block,
A_oo[m, i]) and A_ia = <a|A|i> (the element that couples the reference to
the single excitation i -> a, stored A_ov[i, a]); P(p, q) f = f(p, q) - f(q, p).
G is the matrix of the density operator, G_ab = <Psi1| a+_b a_a |Psi1> for
|Psi1> = 1/4 sum t_ij^ac(A) |ij->ac> + sum t_i^a(A) |i->a>, so its
eigenvectors are the coefficients of the natural spinors.  Where the paper
leaves it open: one factor of each product of two amplitudes (or of an
amplitude and an integral) is conjugated, the singles numerator is the bare
element <a|A|i>, and the basis change is B = Vt Z (v x k; the printed order
has the wrong dimensions).
Plain NumPy (einsum, eigh), FP64.
"""
from __future__ import annotations

import numpy as np


def integrals_ov(Lov: np.ndarray) -> np.ndarray:
    """<ij||ab> for all i, j, a, b: [o, o, v, v]."""
    g = np.einsum("pia,pjb->ijab", Lov, Lov, optimize=True)           # <ij|ab>
    return g - np.transpose(g, (0, 1, 3, 2))


def mp2_amplitudes(eps: np.ndarray, Lov: np.ndarray):
    """(t [o, o, v, v], <ij||ab> [o, o, v, v]); the i = j and a = b entries vanish."""
    nchol, o, v = Lov.shape
    W = integrals_ov(Lov)
    eo, ev = eps[:o], eps[o:o + v]
    D = eo[:, None, None, None] + eo[None, :, None, None] - ev[None, None, :, None] \
        - ev[None, None, None, :]
    return W / D, W


def dressed_diagonals(eps, t, W):
    """(Hb_ii [o], Hb_aa [v])."""
    o = t.shape[0]
    hi = eps[:o] + 0.5 * np.einsum("inef,inef->i", t, np.conj(W), optimize=True).real
    ha = eps[o:] - 0.5 * np.einsum("mnfa,mnfa->a", t, np.conj(W), optimize=True).real
    return hi, ha


def perturbation_doubles(t, A_vv, A_oo):
    """Ab_ij^ac = P(a,c) sum_e t_ij^ec A_ae - P(i,j) sum_m t_mj^ac A_mi."""
    X = np.einsum("ijec,ae->ijac", t, A_vv, optimize=True)            # sum_e t_ij^ec A_ae
    Y = np.einsum("mjac,mi->ijac", t, A_oo, optimize=True)            # sum_m t_mj^ac A_mi
    return (X - np.transpose(X, (0, 1, 3, 2))) - (Y - np.transpose(Y, (1, 0, 2, 3)))


def perturbed_amplitudes(t, A_ov, A_vv, A_oo, hi, ha, omega):
    """(t2(A) [o, o, v, v], t1(A) [o, v]) for one perturbation component."""
    Ab = perturbation_doubles(t, A_vv, A_oo)
    den2 = ha[None, None, :, None] + ha[None, None, None, :] - hi[:, None, None, None] \
        - hi[None, :, None, None] + omega
    den1 = ha[None, :] - hi[:, None] + omega
    return Ab / den2, A_ov / den1


def density(t2A, t1A):
    """G_ab = 1/2 sum_{ijc} t_ij^ac conj t_ij^bc + sum_i t_i^a conj t_i^b."""
    return 0.5 * np.einsum("ijac,ijbc->ab", t2A, np.conj(t2A), optimize=True) \
        + np.einsum("ia,ib->ab", t1A, np.conj(t1A), optimize=True)


def fns_plus(eps, Lov, A_ov, A_vv, A_oo, omega, threshold):
    """Averaged FNS++ density and the truncated, semicanonical virtual basis.

    A_*: [ncomp, ...] component blocks.  Returns dict(n [v] occupation
    numbers, largest |n| first; keep = count with |n| > threshold;
    eps_new [keep]; B [v, keep]; G [v, v])."""
    o = Lov.shape[1]
    t, W = mp2_amplitudes(eps, Lov)
    hi, ha = dressed_diagonals(eps, t, W)
    ncomp = A_vv.shape[0]
    v = len(eps) - o
    G = np.zeros((v, v), np.complex128)   # no component: a zero density
    for x in range(ncomp):
        t2A, t1A = perturbed_amplitudes(t, A_ov[x], A_vv[x], A_oo[x], hi, ha, omega)
        G = G + density(t2A, t1A)
    if ncomp:
        G = G / ncomp
    n, V = np.linalg.eigh(G)
    order = np.argsort(-np.abs(n), kind="stable")
    n, V = n[order], V[:, order]
    keep = int(np.sum(np.abs(n) > threshold))
    Vt = V[:, :keep]
    Ft = np.conj(Vt.T) @ np.diag(eps[o:]) @ Vt
    et, Z = np.linalg.eigh(Ft)
    return dict(n=n, keep=keep, eps_new=et, B=Vt @ Z, G=G, hi=hi, ha=ha)


def hermitian_eigh(A):
    """Eigenvalues (ascending) and eigenvectors of a Hermitian matrix: the
    library routine (LAPACK zheevd through numpy) as the definition."""
    return np.linalg.eigh(A)


def transform_vectors(B, L):
    """Cholesky vectors in the new virtual basis: Lt^P = B^H L^P B (so that
    <ab|cd> = sum_P L_ac L_bd becomes the integrals over the columns of B)."""
    return np.einsum("ak,pab,bl->pkl", np.conj(B), L, B, optimize=True)


def transform_dipole(mu, B):
    """Occupied-virtual one-body block in the new basis.  mu[x, i, a] =
    <a|mu_x|i> carries the virtual in the bra, so with the new spinors
    phi~_l = sum_a phi_a B[a, l]: mu_t[x, i, l] = sum_a conj(B[a, l]) mu[x, i, a]."""
    return np.einsum("xia,al->xil", mu, np.conj(B), optimize=True)
