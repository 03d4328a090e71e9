"""GPU ring term (lrcc_ring_sigma) against the oracle (oracle/ring.py).

FP64 throughout; the GPU forms the same integrals and products in another
summation order (GEMM blocking), so the bar is 1e-12 relative (Frobenius).
Inputs: one Hermitian decomposition L^P over all o + v spinors
(lrcc_synth.make_L), split into its four blocks, and packed CN(0, 1) doubles.
"""
import numpy as np
import pytest

import lrcc_synth as S
from oracle import ring

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lrcc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_12914_amd as m
    return m


def blocks(Lfull, o):
    return (np.ascontiguousarray(Lfull[:, :o, :o]), np.ascontiguousarray(Lfull[:, :o, o:]),
            np.ascontiguousarray(Lfull[:, o:, :o]), np.ascontiguousarray(Lfull[:, o:, o:]))


def run(lrcc, o, v, nchol, nrhs, herm=True, seed=0, gamma=1.0):
    rng = np.random.default_rng(seed)
    Lfull = S.make_L(rng, nchol, o + v, gamma, herm)
    X = S.make_packed(rng, nrhs, o, v)
    Loo, Lov, Lvo, Lvv = blocks(Lfull, o)
    g = lrcc.ring_sigma(*(torch.from_numpy(t).cuda() for t in (Loo, Lov, Lvo, Lvv, X)), o=o)
    return g.cpu().numpy(), (Loo, Lov, Lvo, Lvv), X


def rel(a, b):
    """The larger of two relative errors: the Frobenius-norm ratio and the
    element-wise ratio max|a - b| / max|b|, so that neither a spread-out
    error nor one concentrated in a few (possibly small) entries passes."""
    d = np.asarray(a) - np.asarray(b)
    fro = np.linalg.norm(d) / max(np.linalg.norm(b), 1e-300)
    mx = np.abs(d).max(initial=0.0) / max(np.abs(b).max(initial=0.0), 1e-300)
    return max(fro, mx)


@pytest.mark.parametrize("o,v,nchol,nrhs,herm", [
    (2, 2, 3, 1, True),          # one occupied and one virtual pair
    (3, 5, 4, 2, True),
    (5, 9, 7, 1, False),         # general complex vectors
    (6, 33, 20, 3, True),        # o v = 198: tiles over b past 32
    (8, 40, 64, 2, False),
    (33, 5, 9, 1, True),         # j-tiles past 32
])
def test_ring_matches_oracle(lrcc, o, v, nchol, nrhs, herm):
    print(f"ring parity o={o} v={v} nchol={nchol} nrhs={nrhs} herm={herm}", flush=True)
    g, (Loo, Lov, Lvo, Lvv), X = run(lrcc, o, v, nchol, nrhs, herm, seed=o * 100 + v)
    r = ring.sigma(Lov, Lvo, Loo, Lvv, X, o, v)
    assert rel(g, r) < 1e-12


def test_ring_full_size(lrcc):
    """o=16, v=160, Nchol=640 and 6 right-hand sides (the shapes of the ladder
    benchmark); vectors scaled by 1/(3 sqrt(v)) as in the solves."""
    print("ring parity o=16 v=160 nchol=640 nrhs=6", flush=True)
    g, (Loo, Lov, Lvo, Lvv), X = run(lrcc, 16, 160, 640, 6, True, seed=0,
                                     gamma=S.solve_gamma(160))
    r = ring.sigma(Lov, Lvo, Loo, Lvv, X, 16, 160)
    assert rel(g, r) < 1e-12


def test_ring_hermitian_operator(lrcc):
    """<Y, ring(X)> = <ring(Y), X> for a Hermitian decomposition (a property
    that holds at any size, checked on the GPU alone)."""
    o, v, nchol = 10, 50, 30
    rng = np.random.default_rng(4)
    Lfull = S.make_L(rng, nchol, o + v, 1.0, True)
    X, Y = S.make_packed(rng, 1, o, v), S.make_packed(rng, 1, o, v)
    bl = [torch.from_numpy(t).cuda() for t in blocks(Lfull, o)]
    RX = lrcc.ring_sigma(*bl, torch.from_numpy(X).cuda(), o=o).cpu().numpy()
    RY = lrcc.ring_sigma(*bl, torch.from_numpy(Y).cuda(), o=o).cpu().numpy()
    a, b = np.vdot(Y, RX), np.vdot(RY, X)
    assert abs(a - b) < 1e-12 * abs(a)


@pytest.mark.parametrize("case", ["one_occupied", "one_virtual", "no_rhs", "no_vectors"])
def test_ring_edge_cases(lrcc, case):
    o, v, nchol, nrhs = 4, 6, 5, 2
    if case == "one_occupied":
        o = 1
    elif case == "one_virtual":
        v = 1
    elif case == "no_rhs":
        nrhs = 0
    elif case == "no_vectors":
        nchol = 0
    g, (Loo, Lov, Lvo, Lvv), X = run(lrcc, o, v, nchol, nrhs, True, seed=9)
    r = ring.sigma(Lov, Lvo, Loo, Lvv, X, o, v)
    assert g.shape == r.shape
    if r.size:
        assert np.abs(g - r).max() <= 1e-12 * max(np.abs(r).max(), 1.0)


def test_ring_errors(lrcc):
    o, v = 300, 300   # o v > 65535
    z = torch.zeros((1, o, o), dtype=torch.complex128).cuda()
    X = torch.zeros((1, 2, 2), dtype=torch.complex128).cuda()
    with pytest.raises(RuntimeError, match="65535"):
        lrcc.lib()
        h = lrcc.handle(0)
        lrcc._check(lrcc.lib().lrcc_ring_sigma(h, o, v, 1, 1, lrcc._ptr(z), lrcc._ptr(z),
                                               lrcc._ptr(z), lrcc._ptr(z), lrcc._ptr(X),
                                               lrcc._ptr(X)), h)


# --- the ring term inside the response solve ---------------------------------

from oracle import response  # noqa: E402

OMEGAS = [0.0, 0.0428, 0.0656]


def dev_ring(inst):
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    return (t(inst.eps), t(inst.L), t(inst.mu)), dict(Loo=t(inst.Loo), Lov=t(inst.Lov),
                                                      Lvo=t(inst.Lvo))


@pytest.mark.parametrize("herm", [True, False])
@pytest.mark.parametrize("cmul", ["4m", "3m"])
@pytest.mark.parametrize("o,v,nchol", [(4, 24, 64), (6, 20, 40)])
def test_solve_with_ring(lrcc, o, v, nchol, cmul, herm):
    print(f"solve with ring o={o} v={v} nchol={nchol} {cmul} herm={herm}", flush=True)
    inst = S.make_instance(o, v, nchol, ncomp=3, seed=11, gamma=S.solve_gamma(v),
                           hermitian=herm, ring=True)
    args, kw = dev_ring(inst)
    rg = (inst.Lov, inst.Lvo)
    alpha, info = lrcc.solve(*args, OMEGAS, tol=1e-8, cmul=cmul, **kw)
    ref = response.solve_dense_coupled(inst.L, inst.eps, inst.mu, OMEGAS, o, v, inst.Loo, rg)
    assert info["status"] == "LRCC_OK" and info["final_relres"] < 1e-8
    assert rel(alpha, ref["alpha"]) < 1e-7
    no_ring = response.solve_dense_coupled(inst.L, inst.eps, inst.mu, OMEGAS, o, v, inst.Loo)
    assert rel(no_ring["alpha"], ref["alpha"]) > 1e-4
    full, finfo = lrcc.solve(*args, OMEGAS, tol=1e-8, cmul=cmul, response="full", **kw)
    fref = response.response_full_dense(inst.L, inst.eps, inst.mu, OMEGAS, o, v, inst.Loo, rg)
    assert finfo["status"] == "LRCC_OK"
    assert rel(full, fref["alpha"]) < 1e-7


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_refinement_with_ring(lrcc, prec):
    o, v, nchol = 5, 30, 60
    inst = S.make_instance(o, v, nchol, ncomp=2, seed=12, gamma=S.solve_gamma(v), ring=True)
    args, kw = dev_ring(inst)
    alpha, info = lrcc.solve(*args, OMEGAS[:2], prec=prec, tol=1e-8, inner_tol=1e-5, **kw)
    ref = response.solve_dense_coupled(inst.L, inst.eps, inst.mu, OMEGAS[:2], o, v, inst.Loo,
                                       (inst.Lov, inst.Lvo))
    assert info["status"] == "LRCC_OK"
    assert rel(alpha, ref["alpha"]) < 1e-7


def test_solve_ring_argument_errors(lrcc):
    inst = S.make_instance(3, 8, 10, ncomp=1, seed=13, gamma=S.solve_gamma(8), ring=True)
    args, kw = dev_ring(inst)
    with pytest.raises(ValueError):
        lrcc.solve(*args, [0.0], Loo=kw["Loo"], Lov=kw["Lov"])
    with pytest.raises(RuntimeError, match="L_oo"):
        lrcc.solve(*args, [0.0], Lov=kw["Lov"], Lvo=kw["Lvo"])


def test_solve_with_ring_full_size(lrcc):
    """The workload of the benchmark (o=16, v=160, Nchol=640, 3 components x
    2 frequencies) with both ladders and the ring term: converged by the
    solver's FP64 residual, and alpha Hermitian (alpha_xy = conj alpha_yx, a
    property of the Hermitian Jacobian at any size); the extra terms move
    alpha by more than the solve tolerance."""
    print("solve with ring o=16 v=160 nchol=640", flush=True)
    cfg = S.CONFIGS["baseline"]
    inst = S.make_instance(cfg.o, cfg.v, cfg.nchol, ncomp=cfg.ncomp, seed=cfg.seed,
                           gamma=S.solve_gamma(cfg.v), ring=True)
    args, kw = dev_ring(inst)
    om = list(cfg.omegas)
    alpha, info = lrcc.solve(*args, om, tol=1e-8, cmul="3m", **kw)
    assert info["status"] == "LRCC_OK" and info["final_relres"] < 1e-8
    herm = np.abs(alpha - np.conj(np.transpose(alpha, (0, 2, 1)))).max()
    assert herm < 1e-9 * np.abs(alpha).max()
    plain, _ = lrcc.solve(*args, om, tol=1e-8, cmul="3m")
    assert rel(plain, alpha) > 1e-4
