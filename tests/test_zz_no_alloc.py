"""The allocation-free ladder entry point (lrcc_ppl_sigma_noalloc) against
lrcc_ppl_sigma, through the C ABI: two calls in a row on the shared static
scratch, the second with a smaller problem, in FP64 and FP32 arithmetic and
both complex forms; the oracle's bars (FP64 1e-10, FP32 2e-6 relative, as
the larger of the Frobenius and the element-wise max-abs ratio)."""
import ctypes

import numpy as np
import pytest

import lrcc_synth as S

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def rel(a, b):
    d = a - b
    fro = np.linalg.norm(d) / max(np.linalg.norm(b), 1e-300)
    mx = np.abs(d).max(initial=0.0) / max(np.abs(b).max(initial=0.0), 1e-300)
    return max(fro, mx)


@pytest.fixture(scope="module")
def lrcc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_12914_amd as m
    return m


def call(lrcc, fn, L, X, prec, cmul):
    out = torch.full_like(X, complex(np.nan, np.nan))   # every entry must be written
    nchol, v = L.shape[0], L.shape[1]
    o = lrcc._o_from_npo(X.shape[1])
    h = lrcc.handle(0)
    st = getattr(lrcc.lib(), fn)(h, o, v, nchol, X.shape[0], lrcc._ptr(L), lrcc._ptr(X),
                                 lrcc._ptr(out), lrcc._dtype_code(X), lrcc.PREC[prec],
                                 lrcc.CMUL[cmul])
    lrcc._check(st, h)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.complex128)


@pytest.mark.parametrize("prec,cmul,tol", [("fp64", "4m", 1e-10), ("fp64", "3m", 1e-10),
                                           ("fp32", "4m", 2e-6), ("fp32", "3m", 2e-6)])
@pytest.mark.parametrize("herm", [True, False])
def test_noalloc_matches_ppl_sigma_twice(lrcc, prec, cmul, tol, herm):
    # a larger problem (several block pairs, ragged v, nchol not a multiple of
    # the chunk), then a smaller one on the same scratch
    for (o, v, nchol, nrhs, seed) in [(6, 45, 70, 2, 1), (3, 13, 9, 1, 2)]:
        print(f"noalloc {prec} {cmul} herm={herm} o={o} v={v} nchol={nchol} nrhs={nrhs}",
              flush=True)
        rng = np.random.default_rng(seed)
        L = torch.from_numpy(S.make_L(rng, nchol, v, hermitian=herm)).cuda()
        X = torch.from_numpy(S.make_packed(rng, nrhs, o, v)).cuda()
        ref = call(lrcc, "lrcc_ppl_sigma", L, X, prec, cmul)
        got = call(lrcc, "lrcc_ppl_sigma_noalloc", L, X, prec, cmul)
        assert np.all(np.isfinite(got))
        assert rel(got, ref) < tol


def test_noalloc_limits(lrcc):
    rng = np.random.default_rng(3)
    L = torch.from_numpy(S.make_L(rng, 16, 20)).cuda()
    X = torch.from_numpy(S.make_packed(rng, 1, 3, 20)).cuda()
    out = torch.empty_like(X)
    with pytest.raises(lrcc.LrccError) as e:
        lrcc.ppl_sigma_noalloc(L, X, out, prec="bf16x3")
    assert e.value.status == lrcc.ERR_UNSUPPORTED
    # staged FP64 vectors alone: (480/8)^2 blocks x 2400 x 1 KB = 8.8 GB
    h = lrcc.handle(0)
    fake = ctypes.c_void_p(1 << 40)
    st = lrcc.lib().lrcc_ppl_sigma_noalloc(h, 40, 480, 2400, 1, fake,
                                           ctypes.c_void_p((1 << 40) + (1 << 36)),
                                           ctypes.c_void_p((1 << 40) + (1 << 38)), 0, 0, 0)
    assert st == lrcc.ERR_SHAPE
    # the entry point still works after the refusals
    lrcc.ppl_sigma_noalloc(L, X, out)
    ref = lrcc.ppl_sigma(L, X)
    torch.cuda.synchronize()
    assert rel(out.cpu().numpy(), ref.cpu().numpy()) < 1e-10
