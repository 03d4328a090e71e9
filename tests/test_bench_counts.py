"""CPU checks of the work counts behind bench.py's rates.

The issued count (bench.issued_flops) is what roofline.issued_frac divides
by the kernel time; here it is pinned to the matrix-core instruction counter
of the FP64 3M ladder (SQ_INSTS_VALU_MFMA_MOPS_F64, 512 flop per unit) in
the committed counter summaries, at the baseline and the scale workload.
The method's count (bench.alg_flops) and the plain 4M count
(bench.flops_per_sigma) are checked against brute-force sums over the
packed pairs on small shapes."""
import os
import re

import pytest

import bench

HERE = os.path.dirname(os.path.abspath(__file__))
PROFILES = os.path.join(HERE, "..", "profiles")


def counter(profile, name):
    """Per-launch value of a counter from a summary table row '| name | value ...'."""
    text = open(os.path.join(PROFILES, profile)).read()
    m = re.search(r"^\| " + re.escape(name) + r" \| ([0-9.]+e[0-9]+)", text, re.M)
    assert m, f"{name} not in {profile}"
    return float(m.group(1))


@pytest.mark.parametrize("profile, shape", [
    ("k_ppl_3m_fp64_o16_v160_nchol640_sq_counters.md", (16, 160, 640, 6)),
    ("k_ppl_3m_fp64_o40_v480_nchol2400_sq_counters.md", (40, 480, 2400, 1)),
])
def test_issued_count_matches_the_mfma_counter(profile, shape):
    measured = counter(profile, "SQ_INSTS_VALU_MFMA_MOPS_F64") * 512
    counted = bench.issued_flops(*shape, prec="fp64", cmul="3m")
    # the summaries print the counter to three or four digits
    assert counted == pytest.approx(measured, rel=2e-3)


@pytest.mark.parametrize("o, v, nchol, nrhs", [(3, 5, 2, 1), (4, 7, 3, 2), (5, 9, 1, 3)])
def test_work_counts_by_brute_force(o, v, nchol, nrhs):
    pv = [(a, b) for a in range(v) for b in range(a + 1, v)]
    po = [(i, j) for i in range(o) for j in range(i + 1, o)]
    # integrals <ab||cd> for packed (ab) <= (cd): two Cholesky dot products each
    builds = sum(1 for p in range(len(pv)) for q in range(p, len(pv))) * 2 * nchol
    # contraction: every (ab, cd) pair for every row
    contract = nrhs * len(po) * len(pv) ** 2
    for cmul, per in (("3m", 6), ("4m", 8)):
        assert bench.alg_flops(o, v, nchol, nrhs, cmul) == per * (builds + contract)
    # no symmetry savings: every ordered pair built, 4M
    assert bench.flops_per_sigma(o, v, nchol, nrhs) == 8 * (len(pv) ** 2 * 2 * nchol + contract)


def test_headline_traffic_summary_describes_the_current_kernel():
    # bench.py reports roofline.traffic from the committed FETCH_SIZE /
    # WRITE_SIZE summary only while the kernel sources hash as they did when
    # the counters were taken; a kernel change must come with new counters
    t = bench.measured_traffic()
    assert t is not None and t > 0
