"""Auxiliary solve and ladder features on the GPU: the deterministic
(atomic-free) ladder, warm starts with the final amplitudes returned, and
per-iteration metrics."""
import json

import numpy as np
import pytest

import lrcc_synth as S
from oracle import ppl, response

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

OMEGAS = [0.0, 0.0428, 0.0656]


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


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.mark.parametrize("prec,dtype,tol", [("fp64", torch.complex128, 1e-10),
                                            ("fp32", torch.complex128, 2e-6),
                                            ("fp32", torch.complex64, 2e-6),
                                            ("bf16x3", torch.complex128, 6e-5)])
@pytest.mark.parametrize("herm", [True, False])
def test_deterministic_sigma_is_reproducible(lrcc, prec, dtype, tol, herm):
    print(f"deterministic sigma {prec} {dtype} herm={herm}", flush=True)
    o, v, nchol, nrhs = 5, 44, 70, 3
    rng = np.random.default_rng(31)
    L = S.make_L(rng, nchol, v, hermitian=herm)
    X = S.make_packed(rng, nrhs, o, v)
    Ld, Xd = dev(L).to(dtype), dev(X).to(dtype)
    lrcc.set_deterministic(True)
    try:
        a = lrcc.ppl_sigma(Ld, Xd, prec=prec).cpu().numpy()
        b = lrcc.ppl_sigma(Ld, Xd, prec=prec).cpu().numpy()
    finally:
        lrcc.set_deterministic(False)
    assert np.array_equal(a.view(np.float64 if a.dtype == np.complex128 else np.float32),
                          b.view(np.float64 if b.dtype == np.complex128 else np.float32))
    if prec == "fp64" and dtype == torch.complex128:
        ref = ppl.sigma(L, X, o, v)
    else:
        ref = ppl.sigma(L.astype(np.complex64).astype(complex),
                        X.astype(np.complex64).astype(complex), o, v) if prec != "bf16x3" \
            else ppl.sigma(L, X, o, v)
    assert rel(a.astype(np.complex128), ref) < tol
    # the default kernels agree with it to rounding
    c = lrcc.ppl_sigma(Ld, Xd, prec=prec).cpu().numpy()
    assert rel(c.astype(np.complex128), a.astype(np.complex128)) < tol


def test_deterministic_solve_is_reproducible(lrcc):
    o, v = 4, 24
    inst = S.make_instance(o, v, 64, ncomp=2, seed=3, gamma=S.solve_gamma(v))
    args = (dev(inst.eps), dev(inst.L), dev(inst.mu), OMEGAS)
    a1, i1 = lrcc.solve(*args, deterministic=True)
    a2, i2 = lrcc.solve(*args, deterministic=True)
    assert np.array_equal(a1.view(np.float64), a2.view(np.float64))
    assert i1["n_sigma_fp64"] == i2["n_sigma_fp64"]
    exact = response.solve_dense(inst.L, inst.eps, inst.mu, OMEGAS, o, v)["alpha"]
    assert np.abs(a1 - exact).max() < 1e-7 * np.abs(exact).max()
    # the batched solve has no deterministic mode
    with pytest.raises(lrcc.LrccError):
        lrcc.solve_batched([{"eps": args[0], "L": args[1], "mu": args[2], "omegas": [0.0]}],
                           deterministic=True)


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_warm_start_from_converged_amplitudes(lrcc, prec):
    o, v = 5, 30
    inst = S.make_instance(o, v, 90, ncomp=2, seed=4, gamma=S.solve_gamma(v))
    args = (dev(inst.eps), dev(inst.L), dev(inst.mu), OMEGAS)
    shape = (len(OMEGAS), 2, o * (o - 1) // 2, v * (v - 1) // 2)
    xo = torch.zeros(shape, dtype=torch.complex128, device="cuda")
    a1, i1 = lrcc.solve(*args, prec=prec, x_out=xo)
    assert i1["status"] == "LRCC_OK"
    # alpha = -<xi_x | X_y> from the returned amplitudes
    xi = response.rhs(inst.mu, o, v)
    Xh = xo.cpu().numpy()
    a_from_x = -np.einsum("xpq,wypq->wxy", np.conj(xi), Xh)
    assert np.abs(a_from_x - a1).max() < 1e-12 * np.abs(a1).max()
    # restarting from them: converged at the start, the same alpha
    a2, i2 = lrcc.solve(*args, prec=prec, x0=xo)
    assert i2["status"] == "LRCC_OK" and i2["iters_max"] == 0 and i2["n_sigma_lowp"] == 0
    assert np.abs(a2 - a1).max() < 1e-9 * np.abs(a1).max()
    # a neighbouring frequency's amplitudes as the start of the next one
    x_prev = torch.zeros(shape, dtype=torch.complex128, device="cuda")
    x_prev[:] = xo[0:1]
    cold_a, cold = lrcc.solve(*args, prec=prec)
    warm_a, warm = lrcc.solve(*args, prec=prec, x0=x_prev)
    assert np.abs(warm_a - cold_a).max() < 1e-7 * np.abs(cold_a).max()
    if prec == "fp64":
        assert warm["iters_max"] <= cold["iters_max"]


def test_metrics_lines(lrcc, tmp_path):
    o, v = 4, 24
    inst = S.make_instance(o, v, 64, ncomp=1, seed=0, gamma=S.solve_gamma(v))
    path = tmp_path / "m.jsonl"
    args = (dev(inst.eps), dev(inst.L), dev(inst.mu), OMEGAS)
    a, info = lrcc.solve(*args, metrics_path=str(path))
    lines = [json.loads(x) for x in path.read_text().splitlines()]
    assert len(lines) == info["iters_max"] + 1
    assert [x["iter"] for x in lines] == list(range(len(lines)))
    assert all(x["side"] == "right" and x["phase"] == "fp64" for x in lines)
    assert all(len(x["relres"]) == len(OMEGAS) for x in lines)
    assert max(lines[-1]["relres"]) < 1e-8 and lines[0]["active"] == len(OMEGAS)
    assert all(b["ms"] >= a_["ms"] for a_, b in zip(lines, lines[1:]))
    # refinement: inner iterations and the outer FP64 residual of each sweep
    path2 = tmp_path / "r.jsonl"
    lrcc.solve(*args, prec="bf16x3", metrics_path=str(path2))
    phases = [json.loads(x)["phase"] for x in path2.read_text().splitlines()]
    assert "inner" in phases and phases[-1] in ("outer", "final")
    # full response: both sides
    path3 = tmp_path / "f.jsonl"
    lrcc.solve(*args, response="full", metrics_path=str(path3))
    sides = {json.loads(x)["side"] for x in path3.read_text().splitlines()}
    assert sides == {"right", "left"}
    with pytest.raises(lrcc.LrccError):
        lrcc.solve(*args, metrics_path=str(tmp_path / "no" / "such" / "dir" / "m.jsonl"))
