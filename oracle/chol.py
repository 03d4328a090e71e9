"""Pivoted (single-step) Cholesky decomposition of a two-electron matrix.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 3 (computational details): the Cholesky vectors are formed by an
iterative procedure that stops once the largest diagonal element of the
(remaining) integral matrix is below the threshold tau.  For a Hermitian
positive semi-definite M (n x n), with d the diagonal of what is not yet
represented:

    repeat:  p = argmax_i d_i   (the first index of the largest value);
             stop if d_p <= tau (or max_vectors reached);
             l_i = (M_ip - sum_q L_q,i conj(L_q,p)) / sqrt(d_p)   for all i;
             append l;  d_i -= |l_i|^2

so that M - sum_q L_q L_q^H has every diagonal element <= tau at the end.
Plain NumPy, FP64.
"""
from __future__ import annotations

import numpy as np


def pivoted_cholesky(M: np.ndarray, tau: float, max_vectors: int | None = None):
    """Returns (L [k, n] complex, pivots [k] int, d [n] remaining diagonal)."""
    n = M.shape[0]
    kmax = n if max_vectors is None else min(max_vectors, n)
    d = np.real(np.diag(M)).astype(np.float64).copy()
    vecs, piv = [], []
    for _ in range(kmax):
        p = int(np.argmax(d))          # numpy returns the first of equal maxima
        if not d[p] > tau:
            break
        col = M[:, p].astype(np.complex128).copy()
        for lq in vecs:
            col -= lq * np.conj(lq[p])
        lnew = col / np.sqrt(d[p])
        vecs.append(lnew)
        piv.append(p)
        d = d - np.abs(lnew) ** 2
    L = np.array(vecs, dtype=np.complex128).reshape(len(vecs), n)
    return L, np.array(piv, dtype=np.int64), d
