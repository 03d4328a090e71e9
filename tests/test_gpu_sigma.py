"""GPU parity of the fused ladder kernel against the FP64 oracle, through the
C ABI (python binding -> liblrcc.so -> HIP kernels)."""
import numpy as np
import pytest

import lrcc_synth as S
from oracle import grads, ppl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def rel(a, b):
    """The larger of two relative errors: the Frobenius-norm ratio and the
    element-wise ratio max|a - b| / max|b|, so that neither a spread-out
    error nor one concentrated in a few (possibly small) entries passes."""
    d = np.asarray(a) - np.asarray(b)
    fro = np.linalg.norm(d) / max(np.linalg.norm(b), 1e-300)
    mx = np.abs(d).max(initial=0.0) / max(np.abs(b).max(initial=0.0), 1e-300)
    return max(fro, mx)


@pytest.fixture(scope="module")
def lrcc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_12914_amd as m
    return m


def dev(x, dtype=torch.complex128):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda").to(dtype)


def run(lrcc, L, X, prec="fp64", cmul="4m", dtype=torch.complex128):
    s = lrcc.ppl_sigma(dev(L, dtype), dev(X, dtype), prec=prec, cmul=cmul)
    torch.cuda.synchronize()
    return s.cpu().numpy().astype(np.complex128)


# (o, v, nchol, nrhs): several tiles, ragged virtual blocks (v not a
# multiple of 8), nchol not a multiple of the chunk, several RHS.  Each runs
# with Hermitian L^P (one integral build per tile pair, the mirror tile taken
# as its conjugate transpose) and with general complex L^P (both built).
SHAPES = [
    (4, 24, 64, 1),      # tiny workload
    (5, 44, 100, 3),     # ragged v
    (3, 37, 7, 2),       # short Cholesky index, odd v
    (6, 16, 33, 1),
    (2, 9, 16, 1),       # one full block plus a 1-wide tail
    (7, 2, 5, 2),        # a single virtual pair
]
CASES = [c + (h,) for c in SHAPES for h in (True, False)]


@pytest.mark.parametrize("o,v,nchol,nrhs,herm", CASES)
def test_fp64_matches_oracle(lrcc, o, v, nchol, nrhs, herm):
    print(f"fp64 parity o={o} v={v} nchol={nchol} nrhs={nrhs}", flush=True)
    rng = np.random.default_rng(100 + v)
    L = S.make_L(rng, nchol, v, hermitian=herm)
    X = S.make_packed(rng, nrhs, o, v)
    got = run(lrcc, L, X)
    ref = ppl.sigma(L, X, o, v)
    assert rel(got, ref) < 1e-10


@pytest.mark.parametrize("herm", [True, False])
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 2e-6)])
@pytest.mark.parametrize("o,v,nchol,nrhs", [(5, 44, 100, 3), (3, 37, 7, 2), (4, 24, 64, 1)])
def test_3m_matches_oracle(lrcc, prec, tol, o, v, nchol, nrhs, herm):
    print(f"3M {prec} parity o={o} v={v} nchol={nchol} nrhs={nrhs} herm={herm}", flush=True)
    rng = np.random.default_rng(400 + v)
    L = S.make_L(rng, nchol, v, hermitian=herm)
    X = S.make_packed(rng, nrhs, o, v)
    got = run(lrcc, L, X, prec=prec, cmul="3m")
    if prec == "fp32":
        L, X = L.astype(np.complex64).astype(complex), X.astype(np.complex64).astype(complex)
    assert rel(got, ppl.sigma(L, X, o, v)) < tol


def test_fp64_complex64_storage(lrcc):
    rng = np.random.default_rng(7)
    o, v, nchol = 4, 30, 40
    L = S.make_L(rng, nchol, v).astype(np.complex64)
    X = S.make_packed(rng, 2, o, v).astype(np.complex64)
    got = run(lrcc, L, X, dtype=torch.complex64)
    ref = ppl.sigma(L.astype(np.complex128), X.astype(np.complex128), o, v)
    assert rel(got, ref) < 1e-6       # only the final rounding to complex64


@pytest.mark.parametrize("herm", [True, False])
@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_fp32_matches_oracle(lrcc, dtype, herm):
    rng = np.random.default_rng(8)
    o, v, nchol = 5, 40, 160
    L = S.make_L(rng, nchol, v, hermitian=herm)
    X = S.make_packed(rng, 2, o, v)
    got = run(lrcc, L, X, prec="fp32", dtype=dtype)
    ref = ppl.sigma(L.astype(np.complex64).astype(np.complex128),
                    X.astype(np.complex64).astype(np.complex128), o, v)
    # FP32 products and sums over K = nchol and 64-slot tiles: ~ sqrt(K) * 2^-24
    assert rel(got, ref) < 2e-6


@pytest.mark.parametrize("herm", [True, False])
@pytest.mark.parametrize("o,v,nchol,nrhs,dtype", [(5, 44, 100, 3, torch.complex128),
                                                  (4, 24, 64, 1, torch.complex128),
                                                  (3, 37, 7, 2, torch.complex64),
                                                  (6, 96, 200, 2, torch.complex128)])
def test_bf16x3_matches_oracle(lrcc, o, v, nchol, nrhs, dtype, herm):
    print(f"bf16x3 parity o={o} v={v} nchol={nchol} nrhs={nrhs} herm={herm}", flush=True)
    rng = np.random.default_rng(200 + v)
    L = S.make_L(rng, nchol, v, hermitian=herm)
    X = S.make_packed(rng, nrhs, o, v)
    got = run(lrcc, L, X, prec="bf16x3", dtype=dtype)
    ref = ppl.sigma(L, X, o, v)
    # each real product keeps hi*hi + hi*lo + lo*hi of the bf16 split
    # (relative error about 2^-17 per product), sums in FP32; two chained
    # products (integral build, contraction): bound 2^-14 relative
    err = rel(got, ref)
    print(f"bf16x3 relative error {err:.2e}", flush=True)
    assert err < 6e-5


@pytest.mark.parametrize("herm", [True, False])
@pytest.mark.parametrize("limit", [1 << 20, 3 << 20])
def test_bf16x3_several_panels(lrcc, limit, herm):
    # a workspace limit far below the triangle's 14.8 MB (v = 44: 231 tile
    # pairs x 64 KB) splits the ladder into panels of one or a few rows; the
    # result must not depend on the split
    rng = np.random.default_rng(21)
    o, v, nchol = 5, 44, 70
    L = S.make_L(rng, nchol, v, hermitian=herm)
    X = S.make_packed(rng, 2, o, v)
    whole = run(lrcc, L, X, prec="bf16x3")
    lrcc.set_workspace_limit(limit)
    try:
        split = run(lrcc, L, X, prec="bf16x3")
    finally:
        lrcc.set_workspace_limit(0)
    ref = ppl.sigma(L, X, o, v)
    assert rel(split, ref) < 6e-5
    # the same products, summed in another order per panel: FP32 rounding only
    assert rel(split, whole) < 1e-6


@pytest.mark.parametrize("where", ["off-diagonal", "diagonal imaginary", "last element"])
def test_almost_hermitian_L_takes_the_general_path(lrcc, where):
    # one element of a Hermitian L breaks the symmetry: the device-side check
    # must see it (else the mirror tiles would be taken as conjugate
    # transposes and miss the change); a Hermitian call before and after on
    # the same handle checks that the flag is recomputed per call
    rng = np.random.default_rng(11)
    o, v, nchol = 4, 37, 24
    L = S.make_L(rng, nchol, v)
    X = S.make_packed(rng, 2, o, v)
    Lb = L.copy()
    if where == "off-diagonal":
        Lb[5, 3, 30] += 1e-3
    elif where == "diagonal imaginary":
        Lb[0, 17, 17] += 1e-3j
    else:
        Lb[-1, v - 1, v - 2] += 1e-3
    for Lx in (L, Lb, L):
        got = run(lrcc, Lx, X)
        assert rel(got, ppl.sigma(Lx, X, o, v)) < 1e-10


def test_empty_and_degenerate(lrcc):
    rng = np.random.default_rng(9)
    # nchol = 0: sigma is zero
    X = S.make_packed(rng, 2, 4, 12)
    L0 = np.zeros((0, 12, 12), np.complex128)
    s = lrcc.ppl_sigma(dev(L0), dev(X))
    assert float(torch.abs(s).max()) == 0.0
    # no occupied pairs / no virtual pairs / no rhs: empty outputs, no error
    for (o, v, nrhs) in [(1, 12, 2), (4, 1, 2), (4, 12, 0)]:
        L = S.make_L(rng, 5, v)
        X = np.zeros((nrhs, o * (o - 1) // 2, v * (v - 1) // 2), np.complex128)
        s = lrcc.ppl_sigma(dev(L), dev(X), o=o)
        assert s.shape == X.shape
    # sigma does not depend on L without occupied pairs, virtual pairs or
    # right-hand sides: the gradient is zero (written over a NaN-filled buffer)
    for cdt in (torch.complex128, torch.complex64):
        for (o, v, nrhs) in [(1, 12, 2), (4, 1, 2), (4, 12, 0)]:
            L = dev(S.make_L(rng, 5, v)).to(cdt)
            X = torch.zeros((nrhs, o * (o - 1) // 2, v * (v - 1) // 2), dtype=cdt,
                            device=L.device)
            dL = torch.full_like(L, float("nan"))
            h = lrcc.handle(0)
            lrcc._check(lrcc.lib().lrcc_ppl_sigma_adjoint(
                h, o, v, 5, nrhs, lrcc._ptr(L), lrcc._ptr(X), lrcc._ptr(X), None,
                lrcc._ptr(dL), lrcc._dtype_code(X), lrcc.PREC["fp64"], lrcc.CMUL["4m"]), h)
            torch.cuda.synchronize()
            assert int(torch.count_nonzero(dL)) == 0
    # rank-one Hermitian vectors cancel exactly in <ab||cd>
    v = 20
    L = np.stack([np.outer(u, np.conj(u)) for u in S.cn(rng, (3, v))])
    X = S.make_packed(rng, 1, 3, v)
    got = run(lrcc, L, X)
    assert np.linalg.norm(got) < 1e-13 * np.linalg.norm(L) ** 2 * np.linalg.norm(X)


def test_argument_errors_raise(lrcc):
    L = dev(S.make_L(np.random.default_rng(1), 4, 10))
    X = dev(S.make_packed(np.random.default_rng(2), 1, 3, 10))
    with pytest.raises(lrcc.LrccError) as e:
        lrcc.lib().lrcc_ppl_sigma  # noqa: B018
        lrcc._check(lrcc.lib().lrcc_ppl_sigma(lrcc.handle(0), 3, 10, 4, 1, lrcc._ptr(L),
                                              lrcc._ptr(X), lrcc._ptr(X), 0, 0, 0),
                    lrcc.handle(0))
    assert e.value.status == lrcc.ERR_ARG


def test_adjoint_dX_matches_oracle(lrcc):
    rng = np.random.default_rng(10)
    o, v, nchol = 4, 26, 48
    L = S.make_L(rng, nchol, v, hermitian=False)
    X, G = S.make_packed(rng, 2, o, v), S.make_packed(rng, 2, o, v)
    dX, _ = lrcc.ppl_sigma_adjoint(dev(L), dev(X), dev(G), want_dL=False)
    torch.cuda.synchronize()
    assert rel(dX.cpu().numpy(), grads.vjp_X(L, G, o, v)) < 1e-10


def test_baseline_size_sampled_entries(lrcc):
    # the FP64 baseline workload (o=16, v=160, Nchol=640, 6 RHS), checked on
    # sampled entries that the oracle computes one by one
    o, v, nchol, nrhs = 16, 160, 640, 6
    print(f"fp64 sampled parity o={o} v={v} nchol={nchol} nrhs={nrhs}", flush=True)
    rng = np.random.default_rng(0)
    L = S.make_L(rng, nchol, v)
    X = S.make_packed(rng, nrhs, o, v)
    got = run(lrcc, L, X).reshape(-1, X.shape[-1])
    rows, pairs, ks = sample(got.shape[0], v, 1)
    ref = ppl.sigma_entries(L, X, v, rows, pairs)
    assert rel(got[np.ix_(rows, ks)], ref) < 1e-10
    # invariants at full size: linearity in X and homogeneity in L
    got2 = run(lrcc, 2.0 * L, X).reshape(got.shape)
    assert rel(got2, 4.0 * got) < 1e-13


def sample(nrows, v, seed):
    # first, last and random rows and packed virtual pairs of a full-size run
    pa, pb = ppl.pairs(v)
    srng = np.random.default_rng(seed)
    ks = np.concatenate([[0, 1, len(pa) - 1], srng.choice(len(pa), 29, replace=False)])
    rows = np.concatenate([[0, nrows - 1], srng.choice(nrows, 14, replace=False)])
    return rows, [(pa[k], pb[k]) for k in ks], ks


# full workload sizes in the default launch configuration of each precision
# (the one bench.py times), Hermitian and general L, sampled entries
@pytest.mark.parametrize("workload,prec,herm", [("baseline", "fp64", False),
                                                ("baseline", "fp32", True),
                                                ("baseline", "bf16x3", True),
                                                ("baseline", "bf16x3", False),
                                                ("precision", "fp64", True),
                                                ("precision", "bf16x3", True)])
def test_workload_size_sampled_entries(lrcc, workload, prec, herm):
    cfg = S.CONFIGS[workload]
    o, v, nchol, nrhs = cfg.o, cfg.v, cfg.nchol, cfg.nrhs
    print(f"{prec} sampled parity {workload} herm={herm}", flush=True)
    rng = np.random.default_rng(2)
    L = S.make_L(rng, nchol, v, hermitian=herm)
    X = S.make_packed(rng, nrhs, o, v)
    got = run(lrcc, L, X, prec=prec).reshape(-1, X.shape[-1])
    rows, pairs, ks = sample(got.shape[0], v, 3)
    if prec == "fp32":  # FP32 arithmetic on the inputs rounded to FP32
        L, X = L.astype(np.complex64).astype(complex), X.astype(np.complex64).astype(complex)
    ref = ppl.sigma_entries(L, X, v, rows, pairs)
    tol = {"fp64": 1e-10, "fp32": 2e-6, "bf16x3": 6e-5}[prec]
    err = rel(got[np.ix_(rows, ks)], ref)
    print(f"{prec} {workload} sampled relative error {err:.2e}", flush=True)
    assert err < tol


@pytest.mark.parametrize("o,v,nchol,nrhs,herm", [(4, 26, 48, 2, False), (6, 36, 144, 1, True),
                                                 (3, 11, 5, 3, False)])
def test_dL_matches_oracle(lrcc, o, v, nchol, nrhs, herm):
    print(f"dL parity o={o} v={v} nchol={nchol} nrhs={nrhs}", flush=True)
    rng = np.random.default_rng(300 + v)
    L = S.make_L(rng, nchol, v, hermitian=herm)
    X, G = S.make_packed(rng, nrhs, o, v), S.make_packed(rng, nrhs, o, v)
    dX, dL = lrcc.ppl_sigma_adjoint(dev(L), dev(X), dev(G))
    torch.cuda.synchronize()
    assert rel(dL.cpu().numpy(), grads.vjp_L(L, X, G, o, v)) < 1e-10
    assert rel(dX.cpu().numpy(), grads.vjp_X(L, G, o, v)) < 1e-10
    # complex64 storage: FP32 GEMMs
    dX32, dL32 = lrcc.ppl_sigma_adjoint(dev(L, torch.complex64), dev(X, torch.complex64),
                                        dev(G, torch.complex64))
    torch.cuda.synchronize()
    assert rel(dL32.cpu().numpy().astype(np.complex128), grads.vjp_L(L, X, G, o, v)) < 1e-5


def test_autograd_function_and_finite_differences(lrcc):
    # o=6, v=36, Nchol=144: torch autograd through the hand-written backward,
    # checked against central finite differences of the GPU forward itself
    # (sigma is linear in X and quadratic in L, so h=1e-6 is exact up to
    # rounding) and against the oracle's gradients
    o, v, nchol = 6, 36, 144
    rng = np.random.default_rng(11)
    L = S.make_L(rng, nchol, v)
    X, G = S.make_packed(rng, 1, o, v), S.make_packed(rng, 1, o, v)
    Lt = dev(L).requires_grad_(True)
    Xt = dev(X).requires_grad_(True)
    s = lrcc.ppl(Lt, Xt)
    loss = torch.real(torch.sum(torch.conj(dev(G)) * s))
    loss.backward()
    gL, gX = Lt.grad.cpu().numpy(), Xt.grad.cpu().numpy()
    assert rel(gL, grads.vjp_L(L, X, G, o, v)) < 1e-10
    assert rel(gX, grads.vjp_X(L, G, o, v)) < 1e-10

    def f(LL, XX):
        out = lrcc.ppl_sigma(dev(LL), dev(XX))
        return float(torch.real(torch.sum(torch.conj(dev(G)) * out)))

    h = 1e-6
    for _ in range(2):
        EL, EX = S.cn(rng, L.shape), S.cn(rng, X.shape)
        fdL = (f(L + h * EL, X) - f(L - h * EL, X)) / (2 * h)
        fdX = (f(L, X + h * EX) - f(L, X - h * EX)) / (2 * h)
        assert abs(fdL - np.real(np.vdot(gL, EL))) < 1e-7 * abs(fdL)
        assert abs(fdX - np.real(np.vdot(gX, EX))) < 1e-7 * abs(fdX)


def test_autotune_cache_and_parity_after_tuning(lrcc, tmp_path):
    cache = str(tmp_path / "tune.txt")
    o, v, nchol, nrhs = 5, 44, 100, 3
    for prec in ("fp64", "fp32"):
        r = lrcc.autotune(o, v, nchol, nrhs, prec=prec, cache_path=cache)
        assert r["supertile"] in (2, 4, 8) and r["occupancy"] in (1, 2, 3, 4, 5)
        assert r["candidates"] >= 2 and r["ms"] > 0
        again = lrcc.autotune(o, v, nchol, nrhs, prec=prec, cache_path=cache)
        assert again["candidates"] == 0
        assert (again["supertile"], again["occupancy"]) == (r["supertile"], r["occupancy"])
    # bf16x3: one launch form, nothing timed
    r = lrcc.autotune(o, v, nchol, nrhs, prec="bf16x3", cache_path=cache)
    assert r["candidates"] == 0 and r["supertile"] == 4
    rng = np.random.default_rng(500)
    L = S.make_L(rng, nchol, v, hermitian=False)
    X = S.make_packed(rng, nrhs, o, v)
    assert rel(run(lrcc, L, X), ppl.sigma(L, X, o, v)) < 1e-10
    assert rel(run(lrcc, L, X, prec="fp32"),
               ppl.sigma(L.astype(np.complex64).astype(complex),
                         X.astype(np.complex64).astype(complex), o, v)) < 2e-6


@pytest.mark.parametrize("herm", [True, False])
@pytest.mark.parametrize("prec,cmul,variants", [("fp32", "4m", (2, 3, 4, 5, 1)),
                                                ("fp64", "4m", (3, 5, 1)),
                                                ("fp64", "3m", (5, 1)), ("fp32", "3m", (5, 1))])
def test_launch_variants(lrcc, tmp_path, prec, cmul, variants, herm):
    # force each launch variant of the fused kernel through a tuner cache
    # entry and check parity with it; 132 rows = 9 chunks of 16: whole rounds
    # for four and eight waves plus a chunk shared out column-block-wise
    ncu = torch.cuda.get_device_properties(0).multi_processor_count
    o, v, nchol, nrhs = 12, 36, 64, 2
    rng = np.random.default_rng(501)
    L = S.make_L(rng, nchol, v, hermitian=herm)
    X = S.make_packed(rng, nrhs, o, v)
    # reference on complex64-rounded inputs: FP32 arithmetic, or FP64
    # arithmetic on complex64 storage
    ref64 = ppl.sigma(L.astype(np.complex64).astype(complex),
                      X.astype(np.complex64).astype(complex), o, v)
    bars = {("fp32", torch.complex128): (ref64, 2e-6), ("fp32", torch.complex64): (ref64, 2e-6),
            ("fp64", torch.complex128): (ppl.sigma(L, X, o, v), 1e-10),
            ("fp64", torch.complex64): (ref64, 1e-6)}
    code = {"fp64": 0, "fp32": 1}[prec]
    ccode = {"4m": 0, "3m": 1}[cmul]
    for var in variants:
        print(f"{prec} {cmul} variant {var}", flush=True)
        cache = tmp_path / f"force{prec}{cmul}{var}.txt"
        cache.write_text(f"gfx950 {ncu} {o} {v} {nchol} {nrhs} {code} {ccode} 4 {var} 1.0\n")
        r = lrcc.autotune(o, v, nchol, nrhs, prec=prec, cmul=cmul, cache_path=str(cache))
        assert r["occupancy"] == var and r["candidates"] == 0
        for dtype in (torch.complex128, torch.complex64):
            ref, tol = bars[(prec, dtype)]
            assert rel(run(lrcc, L, X, prec=prec, cmul=cmul, dtype=dtype), ref) < tol


@pytest.mark.parametrize("dtype,tol", [(torch.complex128, 1e-10), (torch.complex64, 1e-5)])
@pytest.mark.parametrize("limit", [1 << 20, 4 << 20, 0])
def test_dL_panels(lrcc, dtype, tol, limit):
    # the gradient's R' panels: one block row per panel (a 1 MB limit), a
    # limit between one and two rows (4 MB: the workspace holds the first row
    # and the later panels, of shorter rows, must stay within it), or the
    # whole triangle at once; ragged v, rows not a multiple of 16, general L
    o, v, nchol, nrhs = 5, 29, 37, 2
    rng = np.random.default_rng(303)
    L = S.make_L(rng, nchol, v, hermitian=False)
    X, G = S.make_packed(rng, nrhs, o, v), S.make_packed(rng, nrhs, o, v)
    lrcc.set_workspace_limit(limit)
    try:
        _, dL = lrcc.ppl_sigma_adjoint(dev(L, dtype), dev(X, dtype), dev(G, dtype),
                                       want_dX=False)
        torch.cuda.synchronize()
    finally:
        lrcc.set_workspace_limit(0)
    ref = grads.vjp_L(L, X, G, o, v)
    if dtype == torch.complex64:
        ref = grads.vjp_L(L.astype(np.complex64).astype(complex),
                          X.astype(np.complex64).astype(complex),
                          G.astype(np.complex64).astype(complex), o, v)
    assert rel(dL.cpu().numpy().astype(np.complex128), ref) < tol
