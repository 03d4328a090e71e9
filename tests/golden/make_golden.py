"""Write exact alpha(omega) of the model response problem for the tiny and
baseline workloads, using only the FP64 oracle (sum-over-states route,
cross-checked against the dense per-pair solve on the tiny case).

    python tests/golden/make_golden.py

Inputs: lrcc_synth.make_instance(o, v, nchol, ncomp=3, seed=0,
gamma=1/(3 sqrt(v))) and the workload's frequencies.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import lrcc_synth as S  # noqa: E402
from oracle import response  # noqa: E402


def main():
    out = {}
    for name, omegas in [("tiny", [0.0, 0.0428, 0.0656, 0.0856]),
                         ("baseline", [0.0, 0.0656])]:
        cfg = S.CONFIGS[name]
        o, v, nchol = cfg.o, cfg.v, cfg.nchol
        inst = S.make_instance(o, v, nchol, ncomp=3, seed=0, gamma=S.solve_gamma(v))
        t0 = time.time()
        a = response.solve_sos(inst.L, inst.eps, inst.mu, omegas, o, v)["alpha"]
        if name == "tiny":
            d = response.solve_dense(inst.L, inst.eps, inst.mu, omegas, o, v)["alpha"]
            assert np.abs(a - d).max() < 1e-12 * np.abs(d).max()
        out[name] = {"o": o, "v": v, "nchol": nchol, "ncomp": 3, "seed": 0,
                     "gamma": S.solve_gamma(v), "omegas": omegas,
                     "route": "oracle.response.solve_sos (exact sum over states)",
                     "alpha_re": a.real.tolist(), "alpha_im": a.imag.tolist()}
        print(f"{name}: {time.time() - t0:.1f} s, alpha_zz = {a[:, 2, 2].real}", flush=True)
    with open(os.path.join(HERE, "alpha_exact.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
