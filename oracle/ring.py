"""sigma_ring = RING(X): the particle-hole (ring) part of the doubles-doubles
Jacobian.

TEST INFRASTRUCTURE ONLY (see the package docstring).

With the ground-state amplitudes at zero (the model of the response
equations, Sec. 2.2), the two-electron part of <mu|[H, tau_nu]|Phi0> between
doubles has three pieces: the particle-particle ladder (ppl.py), the
hole-hole ladder (hhl.py) and the ring term written out here.  The integrals
come from the Cholesky vectors of one decomposition over all spinors
(Sec. 3), <pq|rs> = sum_P L^P_pr L^P_qs:

    <kb|cj>  = sum_P L^P_kc L^P_bj          (occupied-virtual, virtual-occupied)
    <kb|jc>  = sum_P L^P_kj L^P_bc          (occupied-occupied, virtual-virtual)
    <kb||cj> = <kb|cj> - <kb|jc>
    r_ij^ab  = sum_{k,c} <kb||cj> X_ik^ac
    sigma_ij^ab = r_ij^ab - r_ji^ab - r_ij^ba + r_ji^ba     (P(ij) P(ab))

The k, c sum is unrestricted and carries no extra factor: this is the matrix
element between determinants itself (pinned in the Fock space), unlike the
doubled ladder convention of ppl.py and hhl.py.  X and sigma are packed
doubles [nrhs, o(o-1)/2, v(v-1)/2].  FP64, plain NumPy.
"""
from __future__ import annotations

import numpy as np

from .ppl import pairs, unpack_doubles


def integrals_ph(Lov, Lvo, Loo, Lvv) -> np.ndarray:
    """M[k, b, c, j] = <kb||cj>."""
    direct = np.einsum("pkc,pbj->kbcj", Lov, Lvo, optimize=True)      # <kb|cj>
    exch = np.einsum("pkj,pbc->kbcj", Loo, Lvv, optimize=True)        # <kb|jc>
    return direct - exch


def pack_doubles(F: np.ndarray) -> np.ndarray:
    """[nrhs, o, o, v, v] -> packed [nrhs, npo, npv] (i < j, a < b)."""
    o, v = F.shape[1], F.shape[3]
    pi, pj = pairs(o)
    pa, pb = pairs(v)
    G = F[:, pi, pj]                       # [nrhs, npo, v, v]
    return G[:, :, pa, pb]


def sigma(Lov, Lvo, Loo, Lvv, X, o: int, v: int) -> np.ndarray:
    """Definition route: form <kb||cj>, contract, antisymmetrise."""
    Xf = unpack_doubles(X, o, v)                                      # [m, i, k, a, c]
    M = integrals_ph(Lov, Lvo, Loo, Lvv)
    r = np.einsum("kbcj,mikac->mijab", M, Xf, optimize=True)
    s = r - np.swapaxes(r, 1, 2) - np.swapaxes(r, 3, 4) + np.swapaxes(np.swapaxes(r, 1, 2), 3, 4)
    return pack_doubles(s)


def sigma_factored(Lov, Lvo, Loo, Lvv, X, o: int, v: int) -> np.ndarray:
    """Independent second route, vector by vector and never forming <kb||cj>:
    the direct part is an outer product per P, u^P_ia = sum_kc X_ik^ac L^P_kc
    times L^P_bj; the exchange part is X contracted with L^P_kj and L^P_bc."""
    Xf = unpack_doubles(X, o, v)
    r = np.zeros_like(Xf)
    for P in range(Lov.shape[0]):
        u = np.tensordot(Xf, Lov[P], axes=([2, 4], [0, 1]))           # [m, i, a]
        r += u[:, :, None, :, None] * Lvo[P].T[None, None, :, None, :]
        t = np.tensordot(Xf, Loo[P], axes=([2], [0]))                 # [m, i, a, c, j]
        t = np.tensordot(t, Lvv[P], axes=([3], [1]))                  # [m, i, a, j, b]
        r -= np.transpose(t, (0, 1, 3, 2, 4))
    s = r - np.swapaxes(r, 1, 2) - np.swapaxes(r, 3, 4) + np.swapaxes(np.swapaxes(r, 1, 2), 3, 4)
    return pack_doubles(s)


def ring_matrix(Lov, Lvo, Loo, Lvv, o: int, v: int, chunk: int = 256) -> np.ndarray:
    """The operator on packed doubles as an explicit matrix (small sizes):
    the definition route applied to the unit vectors, a chunk at a time."""
    npo, npv = o * (o - 1) // 2, v * (v - 1) // 2
    n = npo * npv
    R = np.zeros((n, n), np.complex128)
    for c0 in range(0, n, chunk):
        c1 = min(n, c0 + chunk)
        E = np.zeros((c1 - c0, n), np.complex128)
        E[np.arange(c1 - c0), np.arange(c0, c1)] = 1.0
        out = sigma(Lov, Lvo, Loo, Lvv, E.reshape(c1 - c0, npo, npv), o, v)
        R[:, c0:c1] = out.reshape(c1 - c0, n).T
    return R
