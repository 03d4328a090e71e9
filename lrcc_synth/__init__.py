"""Seeded synthetic inputs for the particle-particle-ladder (PPL) response path.

This module only draws random numbers.  It holds none of the method's
arithmetic: no integrals, no right-hand sides, no denominators.  Both the
FP64 CPU oracle and the GPU library are fed from here, so the two sides see
bit-identical inputs.

Recipe (stand-in for the paper's molecular workloads, whose integrals are not
available; shapes follow the systems of the paper's efficiency section and
its retained-virtual range of about 50--300 spinors):

* Cholesky vectors ``L[P, a, c]`` (complex, vv block):
  ``L^P = gamma * (G^P + G^P^H) / 2 * exp(-P / 16)`` with ``G ~ CN(0, 1)``.
  Each ``L^P`` is Hermitian in its pair index, which is what real
  Cholesky vectors of a Hermitian two-electron matrix look like in a Kramers-
  unrestricted spinor basis.
* Occupied spinor energies ``U(-2, -0.5)`` Eh, virtual ``U(0.1, 5)`` Eh.
* Dipole ov block ``mu[x, i, a] ~ CN(0, 0.1^2)``.
* A complex normal ``CN(0, s^2)`` draw is ``s * (x + i y) / sqrt(2)`` with
  ``x, y ~ N(0, 1)``, so ``E|z|^2 = s^2``.
* Draw order from ``numpy.random.default_rng(seed)``: G real part, G
  imaginary part (each ``[nchol, v, v]``), occupied energies, virtual
  energies, then per dipole component its real and imaginary part.
* Optionally (the hole-hole ladder), occupied-occupied Cholesky vectors
  ``Loo[P, k, i]`` of the same form over the occupied spinors, drawn last,
  scaled by ``solve_gamma(o)``.

Packed doubles for sigma-only runs are drawn directly in packed form
(``[nrhs, o(o-1)/2, v(v-1)/2]``, ``CN(0, 1)``); they stand for an amplitude
vector that is antisymmetric in ij and in ab, which the packed form encodes.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "CONFIGS",
    "Config",
    "cn",
    "make_L",
    "make_instance",
    "make_packed",
    "make_psd",
    "make_fns_instance",
    "make_hermitian",
    "FnsInstance",
    "npair",
    "solve_gamma",
    "ring_gamma",
]


def npair(n: int) -> int:
    """Number of strictly ordered pairs p<q among n indices."""
    return n * (n - 1) // 2


def cn(rng: np.random.Generator, shape, scale: float = 1.0) -> np.ndarray:
    """Complex normal CN(0, scale^2): real part drawn first, then imaginary."""
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return (scale / math.sqrt(2.0)) * (re + 1j * im)


def make_L(rng: np.random.Generator, nchol: int, v: int, gamma: float = 1.0,
           hermitian: bool = True) -> np.ndarray:
    """Cholesky vectors ``[nchol, v, v]`` complex128, decaying as exp(-P/16).

    With ``hermitian=False`` the symmetrisation is skipped (general complex
    vectors, used for adjoint tests where L has no structure).
    """
    g = cn(rng, (nchol, v, v))
    if hermitian:
        g = 0.5 * (g + np.conj(np.swapaxes(g, 1, 2)))
    decay = np.exp(-np.arange(nchol, dtype=np.float64) / 16.0)
    # C order [P][a][c] (the sum with the swapped view would otherwise come
    # back in the swapped layout, which slows every slice L[:, a, :] ~500x)
    return np.ascontiguousarray((gamma * decay)[:, None, None] * g)


def make_packed(rng: np.random.Generator, nrhs: int, o: int, v: int,
                scale: float = 1.0) -> np.ndarray:
    """Packed doubles ``[nrhs, o(o-1)/2, v(v-1)/2]`` complex128, CN(0, scale^2)."""
    return cn(rng, (nrhs, npair(o), npair(v)), scale)


def solve_gamma(v: int) -> float:
    """Scale applied to L for response solves: 1 / (3 sqrt(v)).

    The raw generator gives a ladder operator whose norm grows like 5v Eh,
    far above the smallest orbital-energy gap (about 1.2 Eh), which makes the
    model Jacobian indefinite.  With this scale the ladder part stays below
    the smallest gap and the shifted Jacobian is positive definite for the
    frequencies used here.
    """
    return 1.0 / (3.0 * math.sqrt(v))


@dataclass
class Instance:
    o: int
    v: int
    nchol: int
    L: np.ndarray      # [nchol, v, v] complex128
    eps: np.ndarray    # [o + v] float64, occupied first
    mu: np.ndarray     # [ncomp, o, v] complex128
    gamma: float
    Loo: np.ndarray = None  # [nchol, o, o] complex128 (hole-hole ladder), optional
    Lov: np.ndarray = None  # [nchol, o, v] complex128 (ring term), optional
    Lvo: np.ndarray = None  # [nchol, v, o] complex128 (ring term), optional


def ring_gamma(o: int, v: int) -> float:
    """Scale of the occupied-virtual vectors of the ring term: 1 / (6 sqrt(o v)),
    which keeps the ring operator's norm a fraction of the smallest gap."""
    return 1.0 / (6.0 * math.sqrt(max(o * v, 1)))


def make_instance(o: int, v: int, nchol: int, ncomp: int = 3, seed: int = 0,
                  gamma: float = 1.0, hermitian: bool = True, hh: bool = False,
                  ring: bool = False) -> Instance:
    """One synthetic LR instance, drawn in the documented order (``hh``: also
    the occupied-occupied vectors of the hole-hole ladder, drawn last;
    ``ring``: then the occupied-virtual vectors ``Lov[P] = CN(0, s^2)
    exp(-P / 16)``, s = ``ring_gamma(o, v)``, with ``Lvo[P] = Lov[P]^H``
    (one Hermitian decomposition) or, for ``hermitian=False``, an
    independent draw of the same form; ``ring`` implies ``hh``)."""
    rng = np.random.default_rng(seed)
    L = make_L(rng, nchol, v, gamma, hermitian)
    e_occ = rng.uniform(-2.0, -0.5, size=o)
    e_vir = rng.uniform(0.1, 5.0, size=v)
    mu = np.stack([cn(rng, (o, v), 0.1) for _ in range(ncomp)]) if ncomp else \
        np.zeros((0, o, v), np.complex128)
    hh = hh or ring
    Loo = make_L(rng, nchol, o, solve_gamma(o), hermitian) if hh else None
    Lov = Lvo = None
    if ring:
        decay = np.exp(-np.arange(nchol, dtype=np.float64) / 16.0)[:, None, None]
        Lov = cn(rng, (nchol, o, v), ring_gamma(o, v)) * decay
        if hermitian:
            Lvo = np.ascontiguousarray(np.conj(np.swapaxes(Lov, 1, 2)))
        else:
            Lvo = cn(rng, (nchol, v, o), ring_gamma(o, v)) * decay
    return Instance(o, v, nchol, L, np.concatenate([e_occ, e_vir]), mu, gamma, Loo, Lov, Lvo)


@dataclass
class Config:
    name: str
    o: int
    v: int
    nchol: int
    ncomp: int
    omegas: tuple
    seed: int = 0
    note: str = ""
    instances: list = field(default_factory=list)  # batched workload only

    @property
    def nrhs(self) -> int:
        return self.ncomp * len(self.omegas)


# The five workloads: a tiny oracle case, the FP64 baseline, the precision
# study, the uneven batch, and the large differentiation/scale case.
CONFIGS = {
    "tiny": Config("tiny", 4, 24, 64, 1, (0.0,), 0,
                   "o=4 v=24 Nchol=64, z only, omega=0"),
    "baseline": Config("baseline", 16, 160, 640, 3, (0.0, 0.0656), 0,
                       "o=16 v=160 Nchol=640, 3 components x 2 frequencies"),
    "precision": Config("precision", 24, 256, 1024, 1,
                        (0.0, 0.0428, 0.0656, 0.0856), 0,
                        "o=24 v=256 Nchol=1024, z x 4 frequencies"),
    "batch": Config("batch", 0, 0, 0, 3, (0.0, 0.0428, 0.0656, 0.0856), 0,
                    "8 instances o in {8..32}, v=10o, Nchol=4v, seeds 0..7",
                    instances=[(o, 10 * o, 40 * o, s) for s, o in
                               enumerate((8, 12, 16, 20, 24, 28, 32, 32))]),
    "scale": Config("scale", 40, 480, 2400, 1, (0.0,), 0,
                    "o=40 v=480 Nchol=2400, one RHS"),
    "gradcheck": Config("gradcheck", 6, 36, 144, 1, (0.0,), 0,
                        "o=6 v=36 Nchol=144 (Nchol = 4v)"),
}


def make_psd(rng: np.random.Generator, n: int, rank: int, decay: float = 4.0) -> np.ndarray:
    """Hermitian positive semi-definite ``[n, n]`` complex128 matrix of the
    given rank, M = B B^H with ``B[:, k] ~ CN(0, 1) exp(-k / decay)``: a
    stand-in for a two-electron integral matrix over index pairs (decaying
    spectrum, low numerical rank) for the pivoted Cholesky decomposition.
    Made exactly Hermitian (the upper triangle mirrored)."""
    B = cn(rng, (n, rank)) * np.exp(-np.arange(rank, dtype=np.float64) / decay)[None, :]
    M = B @ np.conj(B.T)
    iu = np.triu_indices(n, 1)
    M[(iu[1], iu[0])] = np.conj(M[iu])
    M[np.diag_indices(n)] = np.real(np.diag(M))
    return M


@dataclass
class FnsInstance:
    o: int
    v: int
    nchol: int
    eps: np.ndarray    # [o + v] float64, occupied first (canonical spinor energies)
    Lov: np.ndarray    # [nchol, o, v] complex128, Lov[P, i, a] = L^P_ia
    A_oo: np.ndarray   # [ncomp, o, o] complex128, A_oo[x, m, i] = <m|A_x|i>
    A_vv: np.ndarray   # [ncomp, v, v] complex128, A_vv[x, a, e] = <a|A_x|e>
    A_ov: np.ndarray   # [ncomp, o, v] complex128, A_ov[x, i, a] = <a|A_x|i>


def make_fns_instance(o: int, v: int, nchol: int, ncomp: int = 3, seed: int = 0,
                      lscale: float = 0.05, ascale: float = 0.1,
                      emax: float = 200.0) -> FnsInstance:
    """Inputs of the perturbation-sensitive natural-spinor density.

    Draw order from ``default_rng(seed)``: occupied energies ``U(-2, -0.5)``,
    virtual energies log-uniform on ``[0.1, emax]`` Eh (a relativistic basis
    reaches far up in energy), the occupied-virtual Cholesky vectors
    ``Lov[P, i, a] = CN(0, lscale^2) exp(-P / 16) / (1 + e_a)`` (real part
    then imaginary part of the whole ``[nchol, o, v]`` array; high virtuals
    couple weakly, so the occupation numbers decay over several decades and
    a 1e-5 threshold keeps roughly a third to two fifths of the virtuals),
    then per perturbation component a
    Hermitian one-body matrix over all ``o + v`` spinors,
    ``(G + G^H) / 2`` with ``G ~ CN(0, ascale^2)`` (a dipole-like operator),
    split into its occupied-occupied, virtual-virtual and virtual-occupied
    blocks.  The blocks are stored as ``A_oo[m, i] = <m|A|i>``,
    ``A_vv[a, e] = <a|A|e>`` and ``A_ov[i, a] = <a|A|i>``."""
    rng = np.random.default_rng(seed)
    e_occ = rng.uniform(-2.0, -0.5, size=o)
    e_vir = np.exp(rng.uniform(math.log(0.1), math.log(emax), size=v))
    decay = np.exp(-np.arange(nchol, dtype=np.float64) / 16.0)
    Lov = cn(rng, (nchol, o, v), lscale) * decay[:, None, None] / (1.0 + e_vir)[None, None, :]
    n = o + v
    A_oo = np.zeros((ncomp, o, o), np.complex128)
    A_vv = np.zeros((ncomp, v, v), np.complex128)
    A_ov = np.zeros((ncomp, o, v), np.complex128)
    for x in range(ncomp):
        g = cn(rng, (n, n), ascale)
        a = 0.5 * (g + np.conj(g.T))
        iu = np.triu_indices(n, 1)
        a[(iu[1], iu[0])] = np.conj(a[iu])
        a[np.diag_indices(n)] = np.real(np.diag(a))
        A_oo[x] = a[:o, :o]
        A_vv[x] = a[o:, o:]
        A_ov[x] = a[o:, :o].T
    return FnsInstance(o, v, nchol, np.concatenate([e_occ, e_vir]), Lov, A_oo, A_vv, A_ov)


def make_hermitian(rng: np.random.Generator, n: int, spectrum=None) -> np.ndarray:
    """Hermitian ``[n, n]`` complex128 matrix: ``(G + G^H) / 2`` with
    ``G ~ CN(0, 1)``; with ``spectrum`` (n real values) instead
    ``U diag(spectrum) U^H`` for the unitary factor ``U`` of the QR
    decomposition of a ``CN(0, 1)`` draw (repeated values give exactly
    degenerate eigenvalues).  Made exactly Hermitian (upper triangle
    mirrored, real diagonal)."""
    g = cn(rng, (n, n))
    if spectrum is None:
        a = 0.5 * (g + np.conj(g.T))
    else:
        q, _ = np.linalg.qr(g)
        a = (q * np.asarray(spectrum, dtype=np.float64)[None, :]) @ np.conj(q.T)
    iu = np.triu_indices(n, 1)
    a[(iu[1], iu[0])] = np.conj(a[iu])
    a[np.diag_indices(n)] = np.real(np.diag(a))
    return a
