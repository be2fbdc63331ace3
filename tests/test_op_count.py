"""The FP64 operation count per bulk 2D update that bench.py prices the bulk
kernel with is the count of the library's own point-wise templates
(tests/opcount/op_count.cpp instantiates them on the host with a counting
scalar type)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def counts(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no host C++ compiler")
    exe = tmp_path_factory.mktemp("opcount") / "op_count"
    subprocess.check_call([gxx, "-O1", "-std=c++17", "-I", os.path.join(HERE, "opcount"),
                           "-o", str(exe), os.path.join(HERE, "opcount", "op_count.cpp")])
    out = subprocess.check_output([str(exe)], text=True)
    return {k: float(v) for k, v in (line.split() for line in out.splitlines())}


def test_weno5_count_by_hand(counts):
    # smoothness indicators 12 + 9 + 12, squared shifted indicators 6,
    # unnormalised weights 6, candidate stencils 5 + 4 + 4, weighted sum 5,
    # normaliser 3, one division
    assert counts["weno5"] == 12 + 9 + 12 + 6 + 6 + 5 + 4 + 4 + 5 + 3 + 1


def test_update_count_composition(counts):
    face = 8 * counts["weno5"] + counts["hllc_star"]
    assert counts["face"] == face
    mean = 2 * face + counts["prim"] + 4 * (counts["update_component_stage0"]
                                           + 2 * counts["update_component"]) / 3
    assert counts["bulk_update_2d_rk3_mean"] == pytest.approx(mean, rel=1e-12)


def test_bench_constant_matches_count(counts):
    import bench
    assert bench.FLOPS_PER_BULK_UPDATE_2D == counts["bulk_update_2d_rk3_mean"]
