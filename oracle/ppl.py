"""sigma = PPL(X): the particle-particle-ladder part of the Jacobian product.

Definitions (paper, Sec. 3 "Computational Details": integrals with more than
two particle indices are never stored but rebuilt from Cholesky vectors; the
antisymmetrised integral is the one used in the MP2 amplitudes of Sec. 2.3):

    <ab|cd>  = sum_P L^P_ac L^P_bd
    <ab||cd> = <ab|cd> - <ab|dc>
    sigma_ij^ab = sum_{c,d} <ab||cd> X_ij^cd        (unrestricted c, d sum)

X and sigma are doubles, antisymmetric in ij and in ab (Sec. 2.2, the T2
operator with its 1/4 prefactor), stored packed: ``[nrhs, o(o-1)/2, v(v-1)/2]``
with pairs p<q in row-major upper-triangular order.  The unrestricted c, d
sum is taken literally (no 1/2), so for antisymmetric X it equals twice the
restricted sum over c<d.

FP64 throughout.  Everything is plain NumPy; the only library primitives are
tensordot / matmul.
"""
from __future__ import annotations

import numpy as np


def pairs(n: int):
    """Row-major list of ordered pairs (p, q), p<q: index arrays (p, q)."""
    return np.triu_indices(n, 1)


def unpack(Xp: np.ndarray, n: int) -> np.ndarray:
    """Packed ``[..., n(n-1)/2]`` -> full antisymmetric ``[..., n, n]``."""
    p, q = pairs(n)
    full = np.zeros(Xp.shape[:-1] + (n, n), dtype=Xp.dtype)
    full[..., p, q] = Xp
    full[..., q, p] = -Xp
    return full


def pack(F: np.ndarray) -> np.ndarray:
    """Full ``[..., n, n]`` -> packed upper triangle ``[..., n(n-1)/2]``."""
    n = F.shape[-1]
    p, q = pairs(n)
    return F[..., p, q]


def packed_row(Xp: np.ndarray, n: int, p: int) -> np.ndarray:
    """Row p of the full antisymmetric matrix of every packed vector:
    ``[..., n(n-1)/2]`` -> ``[..., n]`` with F[p, q] = X(p, q) for q > p,
    -X(q, p) for q < p and 0 on the diagonal."""
    out = np.zeros(Xp.shape[:-1] + (n,), dtype=Xp.dtype)
    for q in range(n):
        if q > p:
            out[..., q] = Xp[..., p * (2 * n - p - 1) // 2 + (q - p - 1)]
        elif q < p:
            out[..., q] = -Xp[..., q * (2 * n - q - 1) // 2 + (p - q - 1)]
    return out


def unpack_doubles(X: np.ndarray, o: int, v: int) -> np.ndarray:
    """``[nrhs, npo, npv]`` -> ``[nrhs, o, o, v, v]`` antisymmetric in both."""
    Xv = unpack(X, v)                       # [nrhs, npo, v, v]
    Xv = np.moveaxis(Xv, 1, -1)             # [nrhs, v, v, npo]
    Xo = unpack(Xv, o)                      # [nrhs, v, v, o, o]
    return np.moveaxis(Xo, (1, 2), (3, 4))  # [nrhs, o, o, v, v]


def coulomb_ab(L: np.ndarray, a: int) -> np.ndarray:
    """<ab|cd> for one a and all b, c, d: ``[b, c, d]`` = sum_P L^P_ac L^P_bd."""
    g = np.tensordot(L[:, a, :], L, axes=([0], [0]))   # [c, b, d]
    return np.transpose(g, (1, 0, 2))


def sigma(L: np.ndarray, X: np.ndarray, o: int, v: int, a_range=None) -> np.ndarray:
    """Definition route.  L ``[nchol, v, v]``, X packed -> sigma packed.

    For each virtual a: build <ab|cd> for all b, c, d from the Cholesky
    vectors, antisymmetrise in (c, d), and contract the full c, d sum
    against the unpacked X.  Only b > a is kept (packed output).
    ``a_range=(a0, a1)`` evaluates only the rows a0 <= a < a1 (the others
    stay zero); used to time a bounded share of the work.
    """
    nrhs, npo, npv = X.shape
    M = nrhs * npo
    Xf = unpack(X.reshape(M, npv), v).reshape(M, v * v)     # X^{cd}, all c, d
    pa, pb = pairs(v)
    out = np.zeros((M, npv), dtype=np.complex128)
    a0, a1 = a_range if a_range is not None else (0, v - 1)
    for a in range(a0, min(a1, v - 1)):
        g = coulomb_ab(L, a)                     # <ab|cd>  [b, c, d]
        g_as = g - np.transpose(g, (0, 2, 1))   # <ab||cd> = <ab|cd> - <ab|dc>
        s_ab = Xf @ g_as.reshape(v, v * v).T     # sum_{c,d} <ab||cd> X^cd  [M, b]
        sel = pa == a
        out[:, sel] = s_ab[:, pb[sel]]
    return out.reshape(nrhs, npo, npv)


def sigma_full(L: np.ndarray, Xfull_m: np.ndarray) -> np.ndarray:
    """Definition route with every (a, b), including a >= b.

    ``Xfull_m`` is ``[M, v, v]`` (any matrix, not necessarily antisymmetric).
    Returns ``[M, v, v]``; used by the invariant tests.
    """
    M, v, _ = Xfull_m.shape
    out = np.zeros((M, v, v), dtype=np.complex128)
    Xf = Xfull_m.reshape(M, v * v)
    for a in range(v):
        g = coulomb_ab(L, a)
        g_as = g - np.transpose(g, (0, 2, 1))
        out[:, a, :] = Xf @ g_as.reshape(v, v * v).T
    return out


def sigma_factored(L: np.ndarray, X: np.ndarray, o: int, v: int) -> np.ndarray:
    """Independent second route: sigma_ij = 2 sum_P L^P X_ij (L^P)^T.

    Follows from the definition for antisymmetric X:
    sum_cd (<ab|cd> - <ab|dc>) X^cd = 2 sum_cd <ab|cd> X^cd
    = 2 sum_P sum_cd L^P_ac X^cd L^P_bd.
    """
    nrhs, npo, npv = X.shape
    Xf = unpack(X.reshape(-1, npv), v)                      # [M, v, v]
    acc = np.zeros_like(Xf)
    for P in range(L.shape[0]):
        acc += L[P] @ Xf @ L[P].T
    return pack(2.0 * acc).reshape(nrhs, npo, npv)


def sigma_bruteforce(L, X, o: int, v: int):
    """Explicit tensors in pure-Python loops, tiny sizes only (v <= 8).

    Builds V[a][b][c][d] = sum_P L^P_ac L^P_bd element by element, then
    <ab||cd> = V[a][b][c][d] - V[a][b][d][c], then the unrestricted sum.
    """
    L = [[[complex(L[P, a, c]) for c in range(v)] for a in range(v)]
         for P in range(len(L))]
    V = [[[[sum(LP[a][c] * LP[b][d] for LP in L) for d in range(v)]
           for c in range(v)] for b in range(v)] for a in range(v)]
    nrhs, npo, npv = X.shape
    out = np.zeros(X.shape, dtype=np.complex128)
    # index of pair (p, q), p<q, in row-major upper-triangular order
    pidx = {}
    k = 0
    for p in range(v):
        for q in range(p + 1, v):
            pidx[(p, q)] = k
            k += 1

    def xval(r, ij, c, d):
        if c == d:
            return 0.0
        if c < d:
            return complex(X[r, ij, pidx[(c, d)]])
        return -complex(X[r, ij, pidx[(d, c)]])

    for r in range(nrhs):
        for ij in range(npo):
            for (a, b), k in pidx.items():
                s = 0.0
                for c in range(v):
                    for d in range(v):
                        s += (V[a][b][c][d] - V[a][b][d][c]) * xval(r, ij, c, d)
                out[r, ij, k] = s
    return out


def sigma_entries(L: np.ndarray, X: np.ndarray, v: int, rows, ab_pairs):
    """sigma[m, (a,b)] for chosen flattened rows m = r*npo + ij and pairs.

    Entry by entry from the definition, for spot checks at sizes where the
    whole of sigma is too slow: for each (a, b) build <ab|cd> for all c, d,
    antisymmetrise, and take the unrestricted sum against X_m^{cd}.
    Returns ``[len(rows), len(ab_pairs)]``.
    """
    npv = X.shape[-1]
    Xm = unpack(X.reshape(-1, npv)[np.asarray(rows)], v)       # [R, v, v]
    out = np.zeros((len(rows), len(ab_pairs)), dtype=np.complex128)
    for k, (a, b) in enumerate(ab_pairs):
        g = L[:, a, :].T @ L[:, b, :]          # <ab|cd>  [c, d]
        g_as = g - g.T                         # <ab||cd>
        out[:, k] = np.einsum("cd,rcd->r", g_as, Xm)
    return out


def ladder_matrix(L: np.ndarray, v: int) -> np.ndarray:
    """K[(ab),(cd)] = 2 <ab||cd> on packed pairs: sigma = K X for one ij.

    The factor 2 turns the unrestricted c, d sum into the packed c<d sum.
    Size npv x npv; for the dense and sum-over-states solves.
    """
    pa, pb = pairs(v)
    npv = len(pa)
    K = np.zeros((npv, npv), dtype=np.complex128)
    for a in range(v - 1):
        g = coulomb_ab(L, a)
        g_as = g - np.transpose(g, (0, 2, 1))
        sel = np.nonzero(pa == a)[0]
        K[sel, :] = 2.0 * g_as[pb[sel]][:, pa, pb]
    return K
