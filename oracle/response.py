"""Model linear-response problem driven by the PPL product (FP64, CPU).

Paper, Sec. 2.2: the first-order right-hand amplitudes solve
X(omega) = (-A + omega I)^{-1} xi(omega), i.e. (A - omega) X = -xi, with A
the CC Jacobian.  Here A is the doubles-doubles block at T = 0 restricted
to the Fock diagonal plus the particle-particle ladder:

    (A X)_ij^ab = D_ij^ab X_ij^ab + sigma_ij^ab,
    D_ij^ab = e_a + e_b - e_i - e_j,

the same orbital-energy difference that forms the diagonal-Jacobian
denominators of the perturbation-sensitive amplitudes (Sec. 2.4).

Right-hand side (a reading; the paper defines xi only as the projection of
the similarity-transformed perturbation on the excited determinants): the
antisymmetric doubles image of the dipole ov block,

    xi_ij^ab = mu_ia mu_jb - mu_ib mu_ja.

Response function (Sec. 2.2, last equation, reduced to the right-hand
amplitudes of this model): alpha_xy(omega) = -<xi_x | X_y(omega)> with
<u|w> = sum over packed (r, i<j, a<b) of conj(u) w.

Three solves:
  solve_iterative -- Jacobi + DIIS on the packed vector, one subspace per RHS
  solve_dense     -- per occupied pair ij, an LU solve of the packed
                     (A_ij - omega) system (A is block diagonal in ij here)
  solve_sos       -- eigen-decomposition H = U diag(lam) U^H of the ladder
                     plus virtual energies, giving the sum-over-states form
                     of Eq. (sos) exactly (Hermitian L only)

Left-hand amplitudes and the full response function (Sec. 2.2): Y(omega)
solves Y (A + omega) = -(eta + F X).  In this model (T = 0, Lambda = 0, a
Hermitian one-body perturbation, doubles only) eta_nu = <Phi_0|V|nu> =
conj(xi_nu) and F = 0 (it would couple doubles to quadruples), so
(A + omega)^T Y^T = -eta.  The response function, with the symmetriser P
taken as f(A, B) + conj f(B, A) and the 1/2 of the paper,
    <<x; y>> = (f_xy + conj f_yx) / 2,  f_xy = sum Y_y xi_x + sum eta_x X_y,
and alpha_full = -<<x; y>>.  For Hermitian L, Y(omega) = conj X(-omega)
and alpha_full(omega) = alpha(omega) + conj alpha(-omega): both terms of
Eq. (sos).
  eta, solve_left_dense, response_full_dense, solve_sos_full
"""
from __future__ import annotations

import numpy as np

from . import hhl, ppl
from . import ring as ringterm


def rhs(mu: np.ndarray, o: int, v: int) -> np.ndarray:
    """xi[x, ij, ab] = mu_ia mu_jb - mu_ib mu_ja on packed pairs."""
    pi, pj = ppl.pairs(o)
    pa, pb = ppl.pairs(v)
    ncomp = mu.shape[0]
    xi = np.zeros((ncomp, len(pi), len(pa)), dtype=np.complex128)
    for x in range(ncomp):
        m = mu[x]
        xi[x] = (m[pi][:, pa] * m[pj][:, pb]) - (m[pi][:, pb] * m[pj][:, pa])
    return xi


def denominators(eps: np.ndarray, o: int, v: int) -> np.ndarray:
    """D[ij, ab] = e_a + e_b - e_i - e_j on packed pairs."""
    pi, pj = ppl.pairs(o)
    pa, pb = ppl.pairs(v)
    eo, ev = eps[:o], eps[o:o + v]
    return (ev[pa] + ev[pb])[None, :] - (eo[pi] + eo[pj])[:, None]


def two_body(L, X, o, v, Loo=None, ring=None):
    """The two-electron part of the model Jacobian applied to X.

    Particle-particle ladder alone: sigma(X) as ppl.py defines it (the
    literal unrestricted c, d sum).  With the hole-hole ladder (``Loo``) and
    optionally the ring term (``ring`` = (Lov, Lvo), which needs ``Loo``):
    the doubles-doubles block of the normal-ordered two-electron operator at
    T = 0 (Sec. 2.2), which in the doubled ladder convention of ppl.py and
    hhl.py is 1/2 PPL + 1/2 HHL (+ RING) -- pinned by the Fock-space matrix
    element in the tests.
    """
    S = ppl.sigma(L, X, o, v)
    if Loo is None:
        return S
    S = 0.5 * S + 0.5 * hhl.sigma(Loo, X, o, v)
    if ring is not None:
        S = S + ringterm.sigma(ring[0], ring[1], Loo, L, X, o, v)
    return S


def apply_jacobian(L, X, eps, o, v, Loo=None, ring=None):
    """(A X) = D o X + the two-electron part (two_body: the ladder alone, or
    the T = 0 doubles-doubles block with ``Loo`` and ``ring``)."""
    return denominators(eps, o, v)[None] * X + two_body(L, X, o, v, Loo, ring)


def _diis_coefficients(errs):
    """Pulay DIIS: minimise |sum c_k e_k| subject to sum c_k = 1.

    Solves the bordered system [[B, 1], [1^T, 0]] [c; l] = [0; 1] with
    B_kl = <e_k|e_l> divided by its largest diagonal entry (a common scale,
    which leaves c unchanged).  Returns None when B is numerically singular:
    condition number of the unit-diagonal form D^-1/2 B D^-1/2 above 1e14.
    """
    m = len(errs)
    B = np.array([[np.vdot(errs[k], errs[l]) for l in range(m)]
                  for k in range(m)])
    d = np.sqrt(np.real(np.diag(B)))
    if m > 1 and np.linalg.cond(B / np.outer(d, d)) > 1e14:
        return None
    A = np.zeros((m + 1, m + 1), dtype=np.complex128)
    A[:m, :m] = B / np.max(d) ** 2
    A[:m, m] = 1.0
    A[m, :m] = 1.0
    rhs_ = np.zeros(m + 1, dtype=np.complex128)
    rhs_[m] = 1.0
    return np.linalg.solve(A, rhs_)[:m]


def solve_iterative(L, eps, mu, omegas, o, v, tol=1e-8, max_iter=200,
                    diis_dim=8, sigma_fn=None, Loo=None, ring=None):
    """Jacobi + DIIS for every (omega, component) right-hand side.

    X0 = -xi / (D - omega).  Each iteration: R = -xi - (D - omega) X - sigma(X);
    stop when |R|_2 / |xi|_2 < tol; otherwise X~ = X + R / (D - omega),
    e = X~ - X, and X = sum_k c_k X~_k over the last ``diis_dim`` pairs.  If
    the DIIS matrix is singular, take the plain Jacobi step and restart the
    subspace.  All active right-hand sides share one sigma call per iteration.

    Returns dict(alpha [nomega, ncomp, ncomp], X [nomega, ncomp, npo, npv],
    iters [nomega, ncomp], relres [nomega, ncomp], n_sigma).
    """
    if sigma_fn is None:
        sigma_fn = lambda X: two_body(L, X, o, v, Loo, ring)  # noqa: E731
    xi = rhs(mu, o, v)
    D = denominators(eps, o, v)
    ncomp = xi.shape[0]
    nom = len(omegas)
    rhs_list = [(w, x) for w in range(nom) for x in range(ncomp)]
    n = len(rhs_list)
    b = np.stack([-xi[x] for (_, x) in rhs_list])
    Dw = np.stack([D - omegas[w] for (w, _) in rhs_list])
    bnorm = np.array([np.linalg.norm(xi[x]) for (_, x) in rhs_list])
    X = b / Dw
    hist = [[] for _ in range(n)]
    iters = np.zeros(n, dtype=int)
    relres = np.full(n, np.inf)
    active = np.ones(n, dtype=bool)
    n_sigma = 0
    for it in range(max_iter + 1):
        idx = np.nonzero(active)[0]
        if len(idx) == 0:
            break
        S = sigma_fn(X[idx])
        n_sigma += 1
        for k, r in enumerate(idx):
            R = b[r] - Dw[r] * X[r] - S[k]
            relres[r] = np.linalg.norm(R) / bnorm[r]
            if relres[r] < tol or it == max_iter:
                active[r] = False
                continue
            Xt = X[r] + R / Dw[r]
            hist[r].append((Xt, Xt - X[r]))
            if len(hist[r]) > diis_dim:
                hist[r].pop(0)
            c = _diis_coefficients([e for (_, e) in hist[r]])
            if c is None:
                X[r] = Xt
                hist[r] = [hist[r][-1]]
            else:
                X[r] = sum(ck * Xk for ck, (Xk, _) in zip(c, hist[r]))
            iters[r] = it + 1
    Xs = X.reshape(nom, ncomp, *X.shape[1:])
    alpha = np.zeros((nom, ncomp, ncomp), dtype=np.complex128)
    for w in range(nom):
        for x in range(ncomp):
            for y in range(ncomp):
                alpha[w, x, y] = -np.vdot(xi[x], Xs[w, y])
    return dict(alpha=alpha, X=Xs, iters=iters.reshape(nom, ncomp),
                relres=relres.reshape(nom, ncomp), n_sigma=n_sigma)


def solve_dense(L, eps, mu, omegas, o, v):
    """Exact solve: per occupied pair ij, LU of (diag(D_ij) + K - omega).

    K = 2 <ab||cd> on packed pairs (the ladder acting on one ij block).
    Returns dict(alpha, X) with the same shapes as ``solve_iterative``.
    """
    xi = rhs(mu, o, v)
    D = denominators(eps, o, v)
    K = ppl.ladder_matrix(L, v)
    ncomp, npo, npv = xi.shape
    X = np.zeros((len(omegas), ncomp, npo, npv), dtype=np.complex128)
    for w, om in enumerate(omegas):
        for ij in range(npo):
            Aij = K + np.diag(D[ij] - om)
            X[w, :, ij, :] = np.linalg.solve(Aij, -xi[:, ij, :].T).T
    alpha = -np.einsum("xpq,wypq->wxy", np.conj(xi), X)
    return dict(alpha=alpha, X=X)


def solve_sos(L, eps, mu, omegas, o, v):
    """Sum-over-states form (Eq. sos) of the same model, Hermitian L only.

    H = diag(e_a + e_b) + K = U diag(lam) U^H on packed virtual pairs; with
    s_ij = e_i + e_j the pair block of A - omega has eigenvalues
    lam_k - s_ij - omega, so
    alpha_xy(omega) = sum_ij sum_k conj(U^H xi_x,ij)_k (U^H xi_y,ij)_k
                                      / (lam_k - s_ij - omega).
    """
    xi = rhs(mu, o, v)
    pa, pb = ppl.pairs(v)
    pi, pj = ppl.pairs(o)
    eo, ev = eps[:o], eps[o:o + v]
    H = ppl.ladder_matrix(L, v) + np.diag(ev[pa] + ev[pb])
    lam, U = np.linalg.eigh(H)
    s = eo[pi] + eo[pj]
    proj = np.einsum("ka,xpa->xpk", np.conj(U.T), xi)   # (U^H xi)[x, ij, k]
    alpha = np.zeros((len(omegas), xi.shape[0], xi.shape[0]),
                     dtype=np.complex128)
    for w, om in enumerate(omegas):
        den = lam[None, :] - s[:, None] - om              # [ij, k]
        alpha[w] = np.einsum("xpk,ypk,pk->xy", np.conj(proj), proj, 1.0 / den)
    return dict(alpha=alpha, eigenvalues=lam)


def eta(mu: np.ndarray, o: int, v: int) -> np.ndarray:
    """Left-hand right-hand side of this model: eta = conj(xi)."""
    return np.conj(rhs(mu, o, v))


def solve_left_dense(L, eps, mu, omegas, o, v):
    """Exact left-hand solve: per occupied pair ij, LU of (A_ij + omega)^T.

    A_ij = diag(D_ij) + K on packed pairs (K the packed ladder matrix), so
    each column y = Y_ij^T solves (A_ij + omega)^T y = -eta_ij.  Returns
    dict(Y [nomega, ncomp, npo, npv], alpha_left [nomega, ncomp, ncomp]) with
    alpha_left_xy = -sum xi_x Y_y = -<eta_x | Y_y>.
    """
    xi = rhs(mu, o, v)
    et = np.conj(xi)
    D = denominators(eps, o, v)
    K = ppl.ladder_matrix(L, v)
    ncomp, npo, npv = xi.shape
    Y = np.zeros((len(omegas), ncomp, npo, npv), dtype=np.complex128)
    for w, om in enumerate(omegas):
        for ij in range(npo):
            Aij = K + np.diag(D[ij] + om)
            Y[w, :, ij, :] = np.linalg.solve(Aij.T, -et[:, ij, :].T).T
    alpha_left = -np.einsum("xpq,wypq->wxy", xi, Y)
    return dict(Y=Y, alpha_left=alpha_left)


def combine_full(alpha_right, alpha_left):
    """alpha_full = (s + s^H) / 2 per frequency, s = alpha_right + alpha_left
    (minus the response function (f_xy + conj f_yx) / 2, f = -s)."""
    s_ = alpha_right + alpha_left
    return 0.5 * (s_ + np.conj(np.transpose(s_, (0, 2, 1))))


def response_full_dense(L, eps, mu, omegas, o, v, Loo=None, ring=None):
    """Full response function from the exact right- and left-hand solves
    (per occupied pair, or on the whole vector with the hole-hole ladder and
    the ring term)."""
    if Loo is None:
        right = solve_dense(L, eps, mu, omegas, o, v)
        left = solve_left_dense(L, eps, mu, omegas, o, v)
    else:
        right = solve_dense_coupled(L, eps, mu, omegas, o, v, Loo, ring)
        left = solve_left_dense_coupled(L, eps, mu, omegas, o, v, Loo, ring)
    return dict(alpha=combine_full(right["alpha"], left["alpha_left"]), X=right["X"],
                Y=left["Y"])


def solve_sos_full(L, eps, mu, omegas, o, v):
    """Both terms of Eq. (sos) for this model (Hermitian L only):
    alpha_xy(omega) = sum_ij sum_k [conj(p_x) p_y / (lam_k - s_ij - omega)
                                    + p_x conj(p_y) / (lam_k - s_ij + omega)]
    with p = U^H xi (see solve_sos)."""
    xi = rhs(mu, o, v)
    pa, pb = ppl.pairs(v)
    pi, pj = ppl.pairs(o)
    eo, ev = eps[:o], eps[o:o + v]
    H = ppl.ladder_matrix(L, v) + np.diag(ev[pa] + ev[pb])
    lam, U = np.linalg.eigh(H)
    s = eo[pi] + eo[pj]
    proj = np.einsum("ka,xpa->xpk", np.conj(U.T), xi)
    alpha = np.zeros((len(omegas), xi.shape[0], xi.shape[0]), dtype=np.complex128)
    for w, om in enumerate(omegas):
        exc = lam[None, :] - s[:, None]                    # [ij, k]
        alpha[w] = (np.einsum("xpk,ypk,pk->xy", np.conj(proj), proj, 1.0 / (exc - om))
                    + np.einsum("xpk,ypk,pk->xy", proj, np.conj(proj), 1.0 / (exc + om)))
    return dict(alpha=alpha)



# --- the hole-hole ladder couples the occupied pairs ----------------------

def full_matrix(L, eps, o, v, Loo=None, ring=None):
    """A on the whole packed vector x[(ij, ab)] (ij major): diag(D) + I (x) K,
    or with the hole-hole ladder diag(D) + (I (x) K + W (x) I) / 2 (+ the ring
    matrix with ``ring`` = (Lov, Lvo)), as two_body.  Small sizes only."""
    K = ppl.ladder_matrix(L, v)
    npo, npv = o * (o - 1) // 2, K.shape[0]
    A = np.diag(denominators(eps, o, v).reshape(-1)).astype(np.complex128)
    if Loo is None:
        A += np.kron(np.eye(npo), K)
    else:
        A += 0.5 * np.kron(np.eye(npo), K) + 0.5 * np.kron(hhl.hh_matrix(Loo, o), np.eye(npv))
    if ring is not None:
        A += ringterm.ring_matrix(ring[0], ring[1], Loo, L, o, v)
    return A


def solve_dense_coupled(L, eps, mu, omegas, o, v, Loo=None, ring=None):
    """Exact right-hand solve on the whole vector: (A - w) x = -xi."""
    xi = rhs(mu, o, v)
    ncomp, npo, npv = xi.shape
    A = full_matrix(L, eps, o, v, Loo, ring)
    X = np.zeros((len(omegas), ncomp, npo, npv), dtype=np.complex128)
    for w, om in enumerate(omegas):
        sol = np.linalg.solve(A - om * np.eye(A.shape[0]), -xi.reshape(ncomp, -1).T)
        X[w] = sol.T.reshape(ncomp, npo, npv)
    alpha = -np.einsum("xpq,wypq->wxy", np.conj(xi), X)
    return dict(alpha=alpha, X=X)


def solve_left_dense_coupled(L, eps, mu, omegas, o, v, Loo=None, ring=None):
    """Exact left-hand solve on the whole vector: (A + w)^T y = -eta."""
    xi = rhs(mu, o, v)
    et = np.conj(xi)
    ncomp, npo, npv = xi.shape
    A = full_matrix(L, eps, o, v, Loo, ring)
    Y = np.zeros((len(omegas), ncomp, npo, npv), dtype=np.complex128)
    for w, om in enumerate(omegas):
        sol = np.linalg.solve((A + om * np.eye(A.shape[0])).T, -et.reshape(ncomp, -1).T)
        Y[w] = sol.T.reshape(ncomp, npo, npv)
    alpha_left = -np.einsum("xpq,wypq->wxy", xi, Y)
    return dict(Y=Y, alpha_left=alpha_left)


def solve_sos_coupled(L, eps, mu, omegas, o, v, Loo=None, ring=None):
    """Sum over states of the whole Hermitian A (Hermitian L and Loo):
    alpha_xy(w) = sum_k conj(p_x,k) p_y,k / (lam_k - w), p = U^H xi."""
    xi = rhs(mu, o, v)
    lam, U = np.linalg.eigh(full_matrix(L, eps, o, v, Loo, ring))
    proj = np.conj(U.T) @ xi.reshape(xi.shape[0], -1).T      # [k, comp]
    alpha = np.zeros((len(omegas), xi.shape[0], xi.shape[0]), dtype=np.complex128)
    for w, om in enumerate(omegas):
        alpha[w] = np.einsum("kx,ky,k->xy", np.conj(proj), proj, 1.0 / (lam - om))
    return dict(alpha=alpha, eigenvalues=lam)
