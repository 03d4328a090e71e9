"""GPU FNS++ natural spinors (lrcc_fns_plus) and the Jacobi eigensolver
(lrcc_heev) against the oracle.

Tolerances: every step is FP64.  The amplitudes, dressed diagonals and the
density differ from the oracle only in summation order (GEMM blocking), so
they agree to a few ulps of the largest entry (checked at 1e-12 relative).
Jacobi eigenvalues are exact to about n * eps * |A| (absolute), checked at
1e-13 of |A|.  Eigenvectors and the basis B are unique up to column phases
and their error scales as eps * |A| / gap; B is compared after aligning each
column's phase, at 1e-9 (the synthetic spectra keep the gaps at the
threshold well above 1e-6 of the largest occupation).  The kept count is an
integer decision on FP64 values on both sides and must match exactly.
"""
import numpy as np
import pytest

import lrcc_synth as S
from oracle import fns

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lrcc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_12914_amd as m
    return m


def cuda(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def check_eigen(A, w, V, tol):
    nrm = max(np.abs(A).max(), 1e-300)
    assert np.all(np.diff(w) >= -tol * nrm)
    np.testing.assert_allclose(np.conj(V.T) @ V, np.eye(len(w)), atol=1e-12)
    assert np.abs(A @ V - V * w[None, :]).max() < tol * nrm * max(1, len(w))


@pytest.mark.parametrize("n", [1, 2, 3, 17, 64, 161, 300])
def test_heev_matches_oracle(lrcc, n):
    print(f"heev parity n={n}", flush=True)
    A = S.make_hermitian(np.random.default_rng(100 + n), n)
    w, V, sweeps = lrcc.heev(cuda(A))
    w, V = w.cpu().numpy(), V.cpu().numpy()
    wr, Vr = fns.hermitian_eigh(A)
    assert np.abs(w - wr).max() < 1e-13 * np.abs(A).max() * max(1, n) ** 0.5
    check_eigen(A, w, V, 1e-13)
    # eigenvectors of well-separated eigenvalues match up to a phase
    gaps = np.diff(wr)
    for k in range(n):
        g = min(gaps[k - 1] if k > 0 else np.inf, gaps[k] if k < n - 1 else np.inf)
        if g > 1e-3:
            ov = np.vdot(Vr[:, k], V[:, k])
            assert abs(abs(ov) - 1) < 1e-10
    assert 1 <= sweeps <= 30


@pytest.mark.parametrize("case", ["degenerate", "zero", "diagonal", "wide"])
def test_heev_special_matrices(lrcc, case):
    print(f"heev special {case}", flush=True)
    rng = np.random.default_rng(7)
    n = 40
    if case == "degenerate":
        A = S.make_hermitian(rng, n, spectrum=np.repeat([-1.0, 0.5, 2.0, 3.0], 10))
    elif case == "zero":
        A = np.zeros((n, n), np.complex128)
    elif case == "diagonal":
        A = np.diag(rng.uniform(-1, 1, n)).astype(np.complex128)
    else:  # eigenvalues spread over 12 decades
        A = S.make_hermitian(rng, n, spectrum=np.logspace(-12, 0, n))
    w, V, _ = lrcc.heev(cuda(A))
    w, V = w.cpu().numpy(), V.cpu().numpy()
    wr, _ = fns.hermitian_eigh(A)
    assert np.abs(w - wr).max() <= 1e-13 * max(np.abs(A).max(), 1e-300) * 8
    check_eigen(A, w, V, 1e-13)


def test_heev_values_only_and_empty(lrcc):
    A = S.make_hermitian(np.random.default_rng(3), 9)
    w, V, _ = lrcc.heev(cuda(A), vectors=False)
    assert V is None
    np.testing.assert_allclose(w.cpu().numpy(), fns.hermitian_eigh(A)[0], atol=1e-13 * 9)
    w, V, s = lrcc.heev(torch.zeros((0, 0), dtype=torch.complex128).cuda())
    assert w.numel() == 0 and s == 0


def run_both(lrcc, inst, omega, thr):
    g = lrcc.fns_plus(cuda(inst.eps), cuda(inst.Lov), cuda(inst.A_ov), cuda(inst.A_vv),
                      cuda(inst.A_oo), omega, thr)
    r = fns.fns_plus(inst.eps, inst.Lov, inst.A_ov, inst.A_vv, inst.A_oo, omega, thr)
    return g, r


def compare(g, r, inst):
    o = inst.o
    t, W = fns.mp2_amplitudes(inst.eps, inst.Lov)
    hi, ha = fns.dressed_diagonals(inst.eps, t, W)
    hb = g["hbar"].cpu().numpy()
    np.testing.assert_allclose(hb, np.concatenate([hi, ha]), rtol=1e-12, atol=1e-14)
    G = g["gamma"].cpu().numpy()
    gs = max(np.abs(r["G"]).max(), 1e-300)
    assert np.abs(G - r["G"]).max() < 1e-12 * gs
    occ = g["occ"].cpu().numpy()
    assert np.abs(occ - r["n"]).max() < 1e-13 * max(np.abs(r["n"]).max(), 1e-300) * 8
    assert g["keep"] == r["keep"]
    k = r["keep"]
    if k == 0:
        assert g["B"].shape == (inst.v, 0) and g["eps_new"].numel() == 0
        return
    en = g["eps_new"].cpu().numpy()
    assert np.abs(en - r["eps_new"]).max() < 1e-12 * np.abs(inst.eps[o:]).max()
    B, Br = g["B"].cpu().numpy(), r["B"]
    assert B.shape == Br.shape
    for c in range(k):
        ph = np.vdot(B[:, c], Br[:, c])
        B[:, c] *= ph / abs(ph)
    assert np.abs(B - Br).max() < 1e-9
    # the basis itself: orthonormal and semicanonical
    np.testing.assert_allclose(np.conj(B.T) @ B, np.eye(k), atol=1e-12)
    F = np.conj(B.T) @ np.diag(inst.eps[o:]) @ B
    assert np.abs(F - np.diag(en)).max() < 1e-12 * np.abs(inst.eps[o:]).max()


@pytest.mark.parametrize("o,v,nchol,ncomp,omega,thr", [
    (3, 7, 5, 1, 0.0, 1e-6),           # smaller than one tile
    (4, 33, 12, 3, 0.0656, 1e-5),      # one element past a 32-tile edge
    (5, 70, 40, 2, 0.0428, 1e-4),      # ragged tiles, two components
    (8, 64, 256, 3, 0.0656, 1e-5),     # whole tiles
])
def test_fns_matches_oracle(lrcc, o, v, nchol, ncomp, omega, thr):
    print(f"fns parity o={o} v={v} nchol={nchol} ncomp={ncomp} omega={omega}", flush=True)
    inst = S.make_fns_instance(o, v, nchol, ncomp, seed=o * 100 + v)
    g, r = run_both(lrcc, inst, omega, thr)
    assert 0 < r["keep"] < v
    compare(g, r, inst)


def test_fns_full_size(lrcc):
    """The workload of the ladder benchmark: o=16, v=160, Nchol=640, three
    dipole components, threshold 1e-5."""
    print("fns parity o=16 v=160 nchol=640", flush=True)
    inst = S.make_fns_instance(16, 160, 640, 3, seed=0)
    g, r = run_both(lrcc, inst, 0.0656, 1e-5)
    compare(g, r, inst)


@pytest.mark.parametrize("case", ["one_occupied", "no_occupied", "no_component",
                                  "keep_all", "keep_none", "one_virtual", "no_vectors"])
def test_fns_edge_cases(lrcc, case):
    print(f"fns edge {case}", flush=True)
    o, v, nchol, ncomp, thr = 4, 20, 10, 2, 1e-5
    if case == "one_occupied":
        o = 1
    elif case == "no_occupied":
        o = 0
    elif case == "no_component":
        ncomp = 0
    elif case == "keep_all":
        thr = 0.0
    elif case == "keep_none":
        thr = 1e3
    elif case == "one_virtual":
        v = 1
    elif case == "no_vectors":
        nchol = 0
    inst = S.make_fns_instance(o, v, nchol, ncomp, seed=21)
    g, r = run_both(lrcc, inst, 0.0656, thr)
    if case in ("no_occupied", "no_component", "keep_none"):
        assert r["keep"] == 0
    if case == "keep_all":
        assert r["keep"] == v
    compare(g, r, inst)


def test_fns_errors(lrcc):
    inst = S.make_fns_instance(3, 8, 4, 1, seed=1)
    args = [cuda(inst.eps), cuda(inst.Lov), cuda(inst.A_ov), cuda(inst.A_vv), cuda(inst.A_oo)]
    with pytest.raises(RuntimeError, match="threshold"):
        lrcc.fns_plus(*args, 0.0, -1.0)
    with pytest.raises(RuntimeError, match="omega"):
        lrcc.fns_plus(*args, float("nan"), 1e-5)
    with pytest.raises(ValueError):
        lrcc.fns_plus(args[0][:-1], *args[1:])


def test_fns_transform_matches_oracle(lrcc):
    inst = S.make_fns_instance(5, 40, 20, 3, seed=31)
    g = lrcc.fns_plus(cuda(inst.eps), cuda(inst.Lov), cuda(inst.A_ov), cuda(inst.A_vv),
                      cuda(inst.A_oo), 0.0656, 1e-5)
    B = g["B"]
    k = B.shape[1]
    assert 0 < k < 40
    L = S.make_L(np.random.default_rng(2), 24, 40, 1.0, True)
    Lt, mt = lrcc.fns_transform(B, cuda(L), cuda(inst.A_ov))
    Bn = B.cpu().numpy()
    Lr, mr = fns.transform_vectors(Bn, L), fns.transform_dipole(inst.A_ov, Bn)
    assert np.abs(Lt.cpu().numpy() - Lr).max() < 1e-12 * np.abs(Lr).max()
    assert np.abs(mt.cpu().numpy() - mr).max() < 1e-12 * np.abs(mr).max()
    Lt2, none = lrcc.fns_transform(B, cuda(L))
    assert none is None and torch.equal(Lt2, Lt)


def joint(o, v, nchol, seed):
    """FNS++ inputs plus particle-particle vectors over the same virtuals
    (solve scale), the dipole's virtual-occupied block as the response
    operator."""
    inst = S.make_fns_instance(o, v, nchol, 3, seed=seed)
    L = S.make_L(np.random.default_rng(seed + 1), nchol, v, S.solve_gamma(v), True)
    return inst, L


def test_solve_in_the_truncated_basis(lrcc):
    """alpha in the FNS++ basis: identical to the canonical one when every
    spinor is kept (a unitary change of the virtual basis that keeps the
    Fock block diagonal); after truncation it moves away gradually (this
    synthetic model's right-hand side spreads over all virtuals, so the
    error is larger than the paper's molecules show)."""
    o, v, nchol = 6, 48, 96
    inst, L = joint(o, v, nchol, 41)
    omegas = [0.0, 0.0656]
    eps, Lg, mu = cuda(inst.eps), cuda(L), cuda(inst.A_ov)
    a_full, _ = lrcc.solve(eps, Lg, mu, omegas, tol=1e-10)
    errs, keeps = [], []
    for thr in (0.0, 1e-7, 1e-5):
        print(f"solve in the FNS++ basis thr={thr}", flush=True)
        g = lrcc.fns_plus(eps, cuda(inst.Lov), mu, cuda(inst.A_vv), cuda(inst.A_oo), 0.0656,
                          thr)
        Lt, mt = lrcc.fns_transform(g["B"], Lg, mu)
        eps_t = torch.cat([eps[:o], g["eps_new"]]).contiguous()
        a_red, info = lrcc.solve(eps_t, Lt, mt, omegas, tol=1e-10)
        assert info["status"] == "LRCC_OK"
        errs.append(np.abs(a_red - a_full).max() / np.abs(a_full).max())
        keeps.append(g["keep"])
    assert keeps[0] == v and errs[0] < 1e-8
    assert v > keeps[1] > keeps[2] > 0
    assert errs[1] < errs[2] < 0.2
