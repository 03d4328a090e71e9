"""Parity at the scale workload (o=40, v=480, Nchol=2400, one right-hand
side), in the launch configuration bench.py times: the ladder in every
precision and complex form, the adjoint and the gradient with respect to L,
each on sampled entries that the FP64 oracle computes one by one.

Bars, each the larger of the Frobenius and the element-wise max-abs ratio
over the sampled entries: FP64 1e-10 (sums of ~1e6 FP64 products); bf16x3
6e-5 as at the smaller sizes (each real product keeps hi*hi + hi*lo + lo*hi,
about 2^-17 relative, two chained products); FP32 3e-5: with complex64
storage the FP32 ladder sums its tile partials in FP32 as well, and a K-term
FP32 sum has a typical relative error of sqrt(K) 2^-24, 3e-6 for the
Nchol = 2400 terms of an integral and again for the 1830 block-pair tiles
of an output slot, with a factor of 3 for the largest of ~300 entries.
"""
import numpy as np
import pytest

import lrcc_synth as S
from oracle import grads, ppl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

O, V, NCHOL, NRHS = 40, 480, 2400, 1


def rel(a, b):
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


@pytest.fixture(scope="module")
def inputs():
    print(f"drawing the scale workload o={O} v={V} nchol={NCHOL}", flush=True)
    rng = np.random.default_rng(7)
    L = S.make_L(rng, NCHOL, V)                  # Hermitian, as the benchmark
    X = S.make_packed(rng, NRHS, O, V)
    G = S.make_packed(rng, NRHS, O, V)
    pa, pb = ppl.pairs(V)
    srng = np.random.default_rng(8)
    ks = np.concatenate([[0, 1, len(pa) - 1], srng.choice(len(pa), 21, replace=False)])
    M = NRHS * O * (O - 1) // 2
    rows = np.concatenate([[0, M - 1], srng.choice(M, 10, replace=False)])
    out = dict(L=L, X=X, G=G, ks=ks, rows=rows, pairs=[(pa[k], pb[k]) for k in ks])
    # the inputs on the GPU, uploaded once per storage type
    out[torch.complex128] = tuple(torch.from_numpy(a).cuda() for a in (L, X, G))
    out[torch.complex64] = tuple(t.to(torch.complex64) for t in out[torch.complex128])
    return out


def on_gpu(inp, dtype):
    return inp[dtype]


def sampled(t, inp):
    s = t.cpu().numpy().astype(np.complex128).reshape(-1, inp["X"].shape[-1])
    return s[np.ix_(inp["rows"], inp["ks"])]


def rounded(inp):
    """The inputs rounded to complex64 (what the complex64 runs see), once."""
    if "r64" not in inp:
        inp["r64"] = tuple(a.astype(np.complex64).astype(np.complex128)
                           for a in (inp["L"], inp["X"], inp["G"]))
    return inp["r64"]


@pytest.mark.parametrize("prec,cmul,dtype", [("fp64", "3m", torch.complex128),
                                             ("fp64", "4m", torch.complex128),
                                             ("fp32", "4m", torch.complex64),
                                             ("bf16x3", "4m", torch.complex64)])
def test_scale_sigma_sampled_entries(lrcc, inputs, prec, cmul, dtype):
    print(f"scale sigma {prec} {cmul} {dtype}", flush=True)
    L, X = inputs["L"], inputs["X"]
    Ld, Xd, _ = on_gpu(inputs, dtype)
    got = sampled(lrcc.ppl_sigma(Ld, Xd, prec=prec, cmul=cmul), inputs)
    if dtype == torch.complex64:
        L, X, _ = rounded(inputs)
    ref = ppl.sigma_entries(L, X, V, inputs["rows"], inputs["pairs"])
    err = rel(got, ref)
    print(f"scale sigma {prec} {cmul}: sampled relative error {err:.2e}", flush=True)
    assert err < {"fp64": 1e-10, "fp32": 3e-5, "bf16x3": 6e-5}[prec]


def test_scale_adjoint_dX_sampled_entries(lrcc, inputs):
    print("scale adjoint dX (FP64)", flush=True)
    L, G = inputs["L"], inputs["G"]
    Ld, Xd, Gd = on_gpu(inputs, torch.complex128)
    dX, _ = lrcc.ppl_sigma_adjoint(Ld, Xd, Gd, want_dL=False)
    got = sampled(dX, inputs)
    del dX
    LH = np.ascontiguousarray(np.conj(np.transpose(L, (0, 2, 1))))  # C order: fast slices
    ref = ppl.sigma_entries(LH, G, V, inputs["rows"], inputs["pairs"])
    err = rel(got, ref)
    print(f"scale adjoint dX: sampled relative error {err:.2e}", flush=True)
    assert err < 1e-10


# complex64: FP32 arithmetic; an entry of dL sums v^2 = 230400 products of
# the R products with the vectors (and each R entry the 780 rows), a typical
# relative error of sqrt(v^2) 2^-24 = 3e-5, with a factor of 3 for the
# largest of the sampled entries
@pytest.mark.parametrize("dtype,tol", [(torch.complex128, 1e-10), (torch.complex64, 1e-4)])
def test_scale_dL_sampled_entries(lrcc, inputs, dtype, tol):
    print(f"scale dL {dtype}", flush=True)
    L, X, G = inputs["L"], inputs["X"], inputs["G"]
    Ld, Xd, Gd = on_gpu(inputs, dtype)
    _, dL = lrcc.ppl_sigma_adjoint(Ld, Xd, Gd, want_dX=False)
    acs = [(0, 0), (1, 479), (479, 0), (200, 201), (333, 17), (64, 64), (7, 300)]
    Ps = np.array([0, 1, 17, 400, 1999, NCHOL - 1])
    dLh = dL.cpu().numpy().astype(np.complex128)
    del dL
    got = np.stack([dLh[Ps, a, c] for (a, c) in acs], axis=1)
    if dtype == torch.complex64:
        L, X, G = rounded(inputs)
    ref = grads.vjp_L_entries(L, X, G, V, acs)[Ps]
    err = rel(got, ref)
    print(f"scale dL {dtype}: sampled relative error {err:.2e}", flush=True)
    assert err < tol
