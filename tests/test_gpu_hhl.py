"""GPU hole-hole ladder (lrcc_hhl_sigma) and the solves whose model Jacobian
includes it, against the FP64 oracle (oracle/hhl.py, coupled solves)."""
import numpy as np
import pytest

import lrcc_synth as S
from oracle import hhl, response

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

OMEGAS = [0.0, 0.0428, 0.0656, 0.0856]


@pytest.fixture(scope="module")
def lrcc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_12914_amd as m
    return m


def rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


@pytest.mark.parametrize("herm", [True, False])
@pytest.mark.parametrize("o,v,nchol,nrhs,dtype", [(4, 24, 64, 1, torch.complex128),
                                                  (7, 13, 10, 3, torch.complex128),
                                                  (9, 10, 5, 2, torch.complex64),
                                                  (2, 9, 3, 2, torch.complex128),
                                                  (20, 17, 12, 1, torch.complex128)])
def test_hhl_sigma_matches_oracle(lrcc, o, v, nchol, nrhs, dtype, herm):
    # several 16-row pair tiles (o = 7: 21 pairs; o = 20: 190), ragged v,
    # one occupied pair (o = 2), complex64 storage
    print(f"hhl parity o={o} v={v} nchol={nchol} nrhs={nrhs} {dtype} herm={herm}", flush=True)
    rng = np.random.default_rng(50 + o)
    Loo = S.make_L(rng, nchol, o, hermitian=herm)
    X = S.make_packed(rng, nrhs, o, v)
    if dtype == torch.complex64:
        Loo, X = Loo.astype(np.complex64).astype(complex), X.astype(np.complex64).astype(complex)
    got = lrcc.hhl_sigma(torch.from_numpy(Loo).to(dtype).cuda(),
                         torch.from_numpy(X).to(dtype).cuda(), v=v).cpu().numpy()
    ref = hhl.sigma(Loo, X, o, v)
    assert rel(got, ref) < (1e-12 if dtype == torch.complex128 else 2e-6)


def test_hhl_sigma_empty(lrcc):
    X = np.zeros((2, 0, 6), np.complex128)                 # o = 1: no pairs
    out = lrcc.hhl_sigma(torch.zeros((3, 1, 1), dtype=torch.complex128).cuda(),
                         torch.from_numpy(X).cuda(), v=4)
    assert out.shape == (2, 0, 6)
    Loo = torch.zeros((0, 4, 4), dtype=torch.complex128).cuda()   # nchol = 0
    X = torch.from_numpy(S.make_packed(np.random.default_rng(1), 1, 4, 5)).cuda()
    assert float(torch.abs(lrcc.hhl_sigma(Loo, X, v=5)).max()) == 0.0


def dev(inst):
    return (torch.from_numpy(inst.eps).cuda(), torch.from_numpy(inst.L).cuda(),
            torch.from_numpy(inst.mu).cuda())


@pytest.mark.parametrize("herm", [True, False])
@pytest.mark.parametrize("cmul", ["4m", "3m"])
@pytest.mark.parametrize("o,v,nchol", [(4, 24, 64), (6, 20, 40)])
def test_solve_with_hole_hole_ladder(lrcc, o, v, nchol, cmul, herm):
    print(f"solve with hhl o={o} v={v} nchol={nchol} {cmul} herm={herm}", flush=True)
    inst = S.make_instance(o, v, nchol, ncomp=3, seed=9, gamma=S.solve_gamma(v), hh=True,
                           hermitian=herm)
    Loo = torch.from_numpy(inst.Loo).cuda()
    alpha, info = lrcc.solve(*dev(inst), OMEGAS, tol=1e-8, cmul=cmul, Loo=Loo)
    ref = response.solve_dense_coupled(inst.L, inst.eps, inst.mu, OMEGAS, o, v, inst.Loo)
    assert info["status"] == "LRCC_OK" and info["final_relres"] < 1e-8
    assert rel(alpha, ref["alpha"]) < 1e-7
    # the hole-hole ladder matters at this size: without it alpha differs
    plain = response.solve_dense(inst.L, inst.eps, inst.mu, OMEGAS, o, v)["alpha"]
    assert rel(plain, ref["alpha"]) > 1e-4
    full, finfo = lrcc.solve(*dev(inst), OMEGAS, tol=1e-8, cmul=cmul, Loo=Loo, response="full")
    fref = response.response_full_dense(inst.L, inst.eps, inst.mu, OMEGAS, o, v, inst.Loo)
    assert finfo["status"] == "LRCC_OK"
    assert rel(full, fref["alpha"]) < 1e-7


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_refinement_with_hole_hole_ladder(lrcc, prec):
    o, v, nchol = 5, 30, 60
    inst = S.make_instance(o, v, nchol, ncomp=2, seed=10, gamma=S.solve_gamma(v), hh=True)
    alpha, info = lrcc.solve(*dev(inst), OMEGAS[:2], prec=prec, tol=1e-8, inner_tol=1e-5,
                             Loo=torch.from_numpy(inst.Loo).cuda())
    ref = response.solve_dense_coupled(inst.L, inst.eps, inst.mu, OMEGAS[:2], o, v, inst.Loo)
    assert info["status"] == "LRCC_OK"
    assert rel(alpha, ref["alpha"]) < 1e-7
