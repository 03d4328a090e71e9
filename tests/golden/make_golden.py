"""Write exact alpha(omega) of the model response problem, using only the
FP64 oracle.

    python tests/golden/make_golden.py                # every workload below
    python tests/golden/make_golden.py precision      # only the named ones

* tiny, baseline: the sum-over-states route (exact), cross-checked against
  the dense per-pair solve on the tiny case.
* precision (o=24, v=256, Nchol=1024, z, four frequencies): the packed
  ladder matrix has 32640^2 entries (17 GB), too large for the eigen route
  on this host, so the oracle's Jacobi + DIIS solve runs to a relative
  residual of 1e-11 with sigma applied as K X (K = oracle.ppl.ladder_matrix,
  pinned against the definition route of sigma).  The stored alpha is then
  within about 1e-11 relative of the exact one; the final residuals are
  stored beside it.

Inputs: lrcc_synth.make_instance(o, v, nchol, ncomp, seed=0,
gamma=1/(3 sqrt(v))) and the workload's frequencies.  Entries already in
the file and not named on the command line are kept as they are.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import lrcc_synth as S  # noqa: E402
from oracle import ppl, response  # noqa: E402

PATH = os.path.join(HERE, "alpha_exact.json")

WORKLOADS = {
    "tiny": dict(ncomp=3, omegas=[0.0, 0.0428, 0.0656, 0.0856], route="sos"),
    "baseline": dict(ncomp=3, omegas=[0.0, 0.0656], route="sos"),
    "precision": dict(ncomp=1, omegas=[0.0, 0.0428, 0.0656, 0.0856], route="iterative",
                      tol=1e-11),
}


def exact_sos(name, inst, omegas):
    o, v = inst.o, inst.v
    a = response.solve_sos(inst.L, inst.eps, inst.mu, omegas, o, v)["alpha"]
    if name == "tiny":
        d = response.solve_dense(inst.L, inst.eps, inst.mu, omegas, o, v)["alpha"]
        assert np.abs(a - d).max() < 1e-12 * np.abs(d).max()
    return a, {"route": "oracle.response.solve_sos (exact sum over states)"}


def exact_iterative(inst, omegas, tol):
    o, v = inst.o, inst.v
    t0 = time.time()
    K = ppl.ladder_matrix(inst.L, v)
    print(f"  ladder matrix {K.shape}: {time.time() - t0:.0f} s", flush=True)
    npv = K.shape[0]

    def sigma_fn(X):
        t1 = time.time()
        out = (X.reshape(-1, npv) @ K.T).reshape(X.shape)
        print(f"  sigma on {X.shape[0]} right-hand sides: {time.time() - t1:.0f} s",
              flush=True)
        return out

    r = response.solve_iterative(inst.L, inst.eps, inst.mu, omegas, o, v, tol=tol,
                                 max_iter=200, diis_dim=8, sigma_fn=sigma_fn)
    return r["alpha"], {
        "route": "oracle.response.solve_iterative (Jacobi + DIIS, 8 vectors) with "
                 "sigma = K X, K = oracle.ppl.ladder_matrix",
        "tol": tol, "relres": r["relres"].ravel().tolist(),
        "iters": r["iters"].ravel().tolist(), "n_sigma": int(r["n_sigma"])}


def main(names):
    out = {}
    if os.path.exists(PATH):
        with open(PATH) as f:
            out = json.load(f)
    for name in names:
        w = WORKLOADS[name]
        cfg = S.CONFIGS[name]
        o, v, nchol = cfg.o, cfg.v, cfg.nchol
        inst = S.make_instance(o, v, nchol, ncomp=w["ncomp"], seed=0,
                               gamma=S.solve_gamma(v))
        t0 = time.time()
        if w["route"] == "sos":
            a, meta = exact_sos(name, inst, w["omegas"])
        else:
            a, meta = exact_iterative(inst, w["omegas"], w["tol"])
        out[name] = {"o": o, "v": v, "nchol": nchol, "ncomp": w["ncomp"], "seed": 0,
                     "gamma": S.solve_gamma(v), "omegas": w["omegas"], **meta,
                     "seconds": round(time.time() - t0, 1),
                     "alpha_re": a.real.tolist(), "alpha_im": a.imag.tolist()}
        print(f"{name}: {time.time() - t0:.1f} s, alpha_zz = {a[:, -1, -1].real}", flush=True)
        with open(PATH, "w") as f:
            json.dump(out, f, indent=1)


if __name__ == "__main__":
    main(sys.argv[1:] or list(WORKLOADS))
