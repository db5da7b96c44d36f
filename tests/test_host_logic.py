"""Host-side logic that needs no GPU: the autotuner's candidate set, the
workload signature, and how bench.py ties HBM traffic to the profiled
kernel source."""
import os

import pytest

from paper_1311_0380_amd import synth


def uneven():
    # the module imports torch and the binding only for device work
    from paper_1311_0380_amd import uneven as u
    return u


@pytest.mark.parametrize("ne,nr", [(10000, 160000), (3000, 192000), (100, 800), (1, 5000),
                                   (50000, 50000), (7, 7000)])
def test_candidates_are_valid_shapes(ne, nr):
    cands = uneven().candidates(ne, nr)
    assert cands
    for c in cands:
        assert c["kernel"] == 1
        assert 1 <= c["events_per_chunk"] <= 256 or c["events_per_chunk"] == 0
        assert 0 <= c["blocks_per_cu"] <= 16
        assert c["schedule"] in (1, 2, 3)


def test_candidates_cover_every_schedule_on_the_uneven_workload():
    cands = uneven().candidates(10000, 160000)
    assert {c["schedule"] for c in cands} == {1, 2, 3}
    assert len({c["events_per_chunk"] for c in cands if c["schedule"] != 3}) >= 2


def test_workload_signature_groups_similar_batches():
    u = uneven()
    a = u.workload_signature(10000, 160000, 1100000)
    b = u.workload_signature(10001, 160100, 1100500)
    c = u.workload_signature(3000, 192000, 1920000)
    assert a == b and a != c


def test_traffic_follows_the_profiled_source(tmp_path, monkeypatch):
    import bench
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "fit_kernel_3000ev_hbm_counters.md").write_text(
        "| x | 1 |\n"
        f"kernel_sha256_prefix = {bench.kernel_source_hash()}\n"
        "traffic_bytes_per_pass = 12345\n")
    src = os.path.join(bench.ROOT, "paper_1311_0380_amd")
    (tmp_path / "paper_1311_0380_amd").symlink_to(src)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic() == 12345
    (prof / "fit_kernel_3000ev_hbm_counters.md").write_text(
        "kernel_sha256_prefix = 0000000000000000\ntraffic_bytes_per_pass = 12345\n")
    assert bench.measured_traffic() is None
    (prof / "fit_kernel_3000ev_hbm_counters.md").unlink()
    assert bench.measured_traffic() is None


def test_algorithmic_bytes_of_the_headline_batch():
    import bench
    b, _ = synth.cfg2()
    assert bench.algorithmic_bytes(b.n_events, b.n_roads, b.n_hits) == 13284326


GUARD_TEST = r"""
#include <cstdio>
#include <string>
#include "svt_submit_guard.h"
static std::string log_;
static int run(int fail_at, bool enqueue_before_fail) {
    // a submission: buffers acquired, then enqueues, failing at step fail_at
    auto g = svt::make_submit_guard([] { log_ += "S"; }, [] { log_ += "R"; });
    for (int step = 0; step < 3; ++step) {
        if (step == 1 && enqueue_before_fail) g.enqueuing();
        if (step == fail_at) return -1;     // an error return: the guard decides
    }
    g.submitted();
    return 0;
}
int main() {
    log_.clear(); run(0, true);  std::printf("%s|", log_.c_str());   // failed before enqueuing
    log_.clear(); run(2, true);  std::printf("%s|", log_.c_str());   // failed after enqueuing
    log_.clear(); run(2, false); std::printf("%s|", log_.c_str());   // failed, nothing enqueued
    log_.clear(); run(9, true);  std::printf("%s|", log_.c_str());   // submitted
    return 0;
}
"""


def test_failed_submission_waits_for_its_stream_before_releasing(tmp_path):
    """A submission that fails after enqueuing work waits for its stream
    (S) before its staging buffer goes back to the pool (R); one that fails
    before enqueuing releases at once; a submitted request releases nothing
    (its completion does)."""
    import shutil
    import subprocess
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no host C++ compiler")
    src = tmp_path / "guard.cc"
    src.write_text(GUARD_TEST)
    exe = tmp_path / "guard"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                       "paper_1311_0380_amd", "csrc")
    subprocess.run([gxx, "-std=c++17", "-O1", "-I", inc, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    assert out == "R|SR|R||"
