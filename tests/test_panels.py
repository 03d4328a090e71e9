"""CPU checks of the host-side panel plan of the gradient's workspace
(csrc/panels.hpp, compiled here with the host compiler): every panel fits in
the workspace the plan sizes, the panels cover the block rows in order, and
the workspace stays within the limit (or one row when a row is larger).

A regression test: the plan once sized the workspace from the first panel
but grew later panels (shorter rows, more of them) against the larger
limit, so at o=40, v=480, Nchol=2400 a fresh handle's gradient wrote up to
2.6 GB past its workspace."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_2604_12914_amd", "csrc")

DRIVER = r"""
#include <cstdio>
#include <cstdlib>
#include "panels.hpp"
int main(int argc, char** argv) {
  const int nbv = std::atoi(argv[1]);
  const size_t pb = std::strtoull(argv[2], nullptr, 10), cap = std::strtoull(argv[3], nullptr, 10);
  const lrcc::PanelPlan p = lrcc::plan_row_panels(nbv, pb, cap);
  std::printf("%zu\n", p.bytes);
  for (const auto& r : p.rows)
    std::printf("%d %d %zu\n", r.first, r.second, (size_t)lrcc::panel_pairs(nbv, r.first, r.second) * pb);
  return 0;
}
"""


@pytest.fixture(scope="module")
def planner(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no host C++ compiler")
    d = tmp_path_factory.mktemp("panels")
    src, exe = d / "driver.cpp", d / "driver"
    src.write_text(DRIVER)
    subprocess.run([gxx, "-std=c++17", "-O1", "-I", CSRC, str(src), "-o", str(exe)], check=True)

    def run(nbv, pair_bytes, cap):
        out = subprocess.run([str(exe), str(nbv), str(pair_bytes), str(cap)], check=True,
                             capture_output=True, text=True).stdout.split("\n")
        ws = int(out[0])
        rows = [tuple(int(x) for x in line.split()) for line in out[1:] if line.strip()]
        return ws, rows
    return run


def pairs(nbv, a0, a1):
    return sum(nbv - a for a in range(a0, a1))


@pytest.mark.parametrize("nbv", [1, 2, 4, 7, 20, 32, 60, 128])
@pytest.mark.parametrize("cap_rows", [0, 1, 1.5, 2.3, 7.9, 1000])
def test_every_panel_fits_the_workspace(planner, nbv, cap_rows):
    nbp = nbv * (nbv + 1) // 2
    pair_bytes = nbp * 65536                      # one FP64 tile per block pair of the triangle
    cap = int(cap_rows * nbv * pair_bytes)        # the limit, in units of the first row
    ws, rows = planner(nbv, pair_bytes, cap)
    assert rows[0][0] == 0 and rows[-1][1] == nbv
    for (a0, a1, b), (n0, _, _) in zip(rows, rows[1:] + [(nbv, nbv, 0)]):
        assert a1 > a0 and n0 == a1               # contiguous, at least one row each
        assert b == pairs(nbv, a0, a1) * pair_bytes
        assert b <= ws                            # the bug: later panels grew past ws
    assert ws == rows[0][2]                       # sized by the first (largest) panel
    assert ws <= max(cap, nbv * pair_bytes)       # within the limit, or one row


def test_scale_workload_plan(planner):
    # o=40, v=480, Nchol=2400 in FP64 with a 16 GiB limit: the workspace is
    # the first two rows and no later panel exceeds it
    nbv = 60
    pair_bytes = 1830 * 65536
    ws, rows = planner(nbv, pair_bytes, 16 << 30)
    assert ws == pairs(nbv, 0, 2) * pair_bytes
    assert max(b for _, _, b in rows) == ws
