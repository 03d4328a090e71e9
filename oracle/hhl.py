"""sigma_hh = HHL(X): the hole-hole-ladder part of the doubles-doubles Jacobian.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The occupied-occupied block of the same Cholesky decomposition gives the
integrals over occupied spinors; with no particle index they are of the kind
the paper forms explicitly (Sec. 3: only integrals with more than two
particle indices are rebuilt on the fly).  Definitions:

    <kl|ij>  = sum_P L^P_ki L^P_lj
    <kl||ij> = <kl|ij> - <kl|ji>
    sigma_ij^ab = sum_{k,l} <kl||ij> X_kl^ab      (unrestricted k, l sum)

The unrestricted sum (no 1/2) follows the factor convention of the
particle-particle ladder (ppl.py), so the two ladders enter the model
Jacobian on the same footing.  X and sigma are packed doubles as in ppl.py.
FP64, plain NumPy.
"""
from __future__ import annotations

import numpy as np

from .ppl import pack, pairs, unpack


def coulomb_oo(Loo: np.ndarray) -> np.ndarray:
    """V[k, l, i, j] = <kl|ij> = sum_P L^P_ki L^P_lj."""
    return np.einsum("pki,plj->klij", Loo, Loo)


def sigma(Loo: np.ndarray, X: np.ndarray, o: int, v: int) -> np.ndarray:
    """Definition route: antisymmetrise <kl|ij> in (i, j) and take the
    unrestricted k, l sum against the unpacked X for every packed (a, b)."""
    nrhs, npo, npv = X.shape
    V = coulomb_oo(Loo)
    Vas = V - np.transpose(V, (0, 1, 3, 2))                 # <kl||ij>
    # X_kl^ab with all k, l: unpack the occupied pair index of every (r, ab)
    Xr = np.transpose(X, (0, 2, 1)).reshape(nrhs * npv, npo)
    Xf = unpack(Xr, o)                                      # [r*ab, k, l]
    full = np.einsum("klij,mkl->mij", Vas, Xf)              # [r*ab, i, j]
    pi, pj = pairs(o)
    out = full[:, pi, pj].reshape(nrhs, npv, npo)
    return np.transpose(out, (0, 2, 1)).copy()


def sigma_factored(Loo: np.ndarray, X: np.ndarray, o: int, v: int) -> np.ndarray:
    """Independent second route: sigma^ab = 2 sum_P (L^P)^T X^ab L^P.

    For X antisymmetric in (k, l): sum_kl (L_ki L_lj - L_kj L_li) X_kl
    = 2 sum_kl L_ki X_kl L_lj.
    """
    nrhs, npo, npv = X.shape
    Xr = np.transpose(X, (0, 2, 1)).reshape(nrhs * npv, npo)
    Xf = unpack(Xr, o)                                      # [m, o, o]
    acc = np.zeros_like(Xf)
    for P in range(Loo.shape[0]):
        acc += Loo[P].T @ Xf @ Loo[P]
    out = pack(2.0 * acc).reshape(nrhs, npv, npo)
    return np.transpose(out, (0, 2, 1)).copy()


def sigma_bruteforce(Loo, X, o: int, v: int):
    """Pure-Python loops over explicit integrals, tiny sizes only."""
    nch = Loo.shape[0]
    V = [[[[sum(complex(Loo[P, k, i]) * complex(Loo[P, l, j]) for P in range(nch))
            for j in range(o)] for i in range(o)] for l in range(o)] for k in range(o)]
    pidx = {}
    n = 0
    for p in range(o):
        for q in range(p + 1, o):
            pidx[(p, q)] = n
            n += 1

    def xval(r, k, l, ab):
        if k == l:
            return 0.0
        if k < l:
            return complex(X[r, pidx[(k, l)], ab])
        return -complex(X[r, pidx[(l, k)], ab])

    nrhs, npo, npv = X.shape
    out = np.zeros(X.shape, dtype=np.complex128)
    for r in range(nrhs):
        for (i, j), ij in pidx.items():
            for ab in range(npv):
                s = 0.0
                for k in range(o):
                    for l in range(o):
                        s += (V[k][l][i][j] - V[k][l][j][i]) * xval(r, k, l, ab)
                out[r, ij, ab] = s
    return out


def hh_matrix(Loo: np.ndarray, o: int) -> np.ndarray:
    """W[(ij), (kl)] = 2 <kl||ij> on packed occupied pairs: sigma^ab = W X^ab.

    The factor 2 turns the unrestricted k, l sum into the packed k<l sum."""
    V = coulomb_oo(Loo)
    Vas = V - np.transpose(V, (0, 1, 3, 2))                 # <kl||ij> [k, l, i, j]
    pi, pj = pairs(o)
    # row (ij) = (pi[r], pj[r]), column (kl) = (pi[c], pj[c])
    return 2.0 * Vas[pi[None, :], pj[None, :], pi[:, None], pj[:, None]]
