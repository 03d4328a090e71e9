"""Vector-Jacobian products of sigma = PPL(L, X) (FP64, CPU).

Convention (PyTorch's for complex tensors): for a real loss l and an
upstream gradient G = dl/dsigma, the gradient g of an input z satisfies
dl = Re <g, dz> = Re sum conj(g) dz.  sigma is linear in X and a
holomorphic quadratic in L.

dX: the adjoint of the packed linear map X -> sigma, applied to G.  With
K[(ab),(cd)] = 2 <ab||cd>, Xbar = K^H G.  Since conj(<ab||cd>[L]) equals
<cd||ab>[L^H] with (L^H)^P = (L^P)^H, this is sigma(L^H, G): the adjoint
is the same ladder with conjugate-transposed Cholesky vectors.

dL: differentiate sigma_ab = 2 sum_P sum_cd L^P_ac L^P_bd X^cd (antisymmetric
X, unrestricted sum).  With G extended to an antisymmetric matrix per row,
both factors contribute equally and
    Lbar^P = 2 sum_m G_m conj(L^P) X_m^H
where G_m, X_m are the full antisymmetric v x v matrices of row m = (r, ij).
"""
from __future__ import annotations

import numpy as np

from . import ppl


def vjp_X_explicit(L, G, o, v):
    """Xbar = K^H G with the packed ladder matrix built explicitly (small v)."""
    K = ppl.ladder_matrix(L, v)
    nrhs, npo, npv = G.shape
    return (G.reshape(-1, npv) @ np.conj(K)).reshape(nrhs, npo, npv)


def vjp_X(L, G, o, v):
    """Xbar = sigma(L^H, G), the adjoint ladder."""
    LH = np.conj(np.transpose(L, (0, 2, 1)))
    return ppl.sigma(LH, G, o, v)


def vjp_L(L, X, G, o, v):
    """Lbar^P = 2 sum_m G_m conj(L^P) X_m^H (full antisymmetric G_m, X_m)."""
    npv = X.shape[-1]
    Gf = ppl.unpack(G.reshape(-1, npv), v)       # [M, v, v]
    Xf = ppl.unpack(X.reshape(-1, npv), v)
    XH = np.conj(np.transpose(Xf, (0, 2, 1)))
    out = np.zeros_like(L)
    for P in range(L.shape[0]):
        out[P] = 2.0 * np.einsum("mab,bd,mdc->ac", Gf, np.conj(L[P]), XH)
    return out


def vjp_L_entries(L, X, G, v, ac_pairs):
    """Lbar^P_ac for every P and the chosen (a, c), one pair at a time from
    the definition above: Lbar^P_ac = 2 sum_m sum_{b,d} G_m[a,b]
    conj(L^P_bd) conj(X_m[c,d]).  Row a of every G_m and row c of every X_m
    are read straight from the packed arrays, so full-size checks need no
    unpacked copy.  Returns ``[nchol, len(ac_pairs)]``."""
    npv = X.shape[-1]
    Gm, Xm = G.reshape(-1, npv), X.reshape(-1, npv)
    Lc = np.conj(L).reshape(L.shape[0], v * v)
    out = np.zeros((L.shape[0], len(ac_pairs)), dtype=np.complex128)
    for k, (a, c) in enumerate(ac_pairs):
        Ga = ppl.packed_row(Gm, v, a)                 # [M, v]: G_m[a, b]
        Xc = ppl.packed_row(Xm, v, c)                 # [M, v]: X_m[c, d]
        Q = Ga.T @ np.conj(Xc)                        # [b, d]: sum_m G_m[a,b] conj X_m[c,d]
        out[:, k] = 2.0 * (Lc @ Q.reshape(v * v))
    return out
