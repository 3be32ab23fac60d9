"""Host-side checks of bench.py: the one-GPU contract and the lookup of HBM
traffic from committed rocprofv3 summaries (taken only while the kernel's
source file is unchanged)."""
import hashlib
import os
import subprocess
import sys

import bench

CSRC = os.path.join(bench.ROOT, "paper_1811_05903_amd", "csrc")


def _summary(tmp_path, digest, name="steps_periodic.hip", traffic=123456.0):
    p = tmp_path / "summary.md"
    p.write_text("# rocprofv3 summary\n\ntraffic_bytes_per_launch: %.0f\n"
                 "source_sha256: %s  (%s)\n" % (traffic, digest, name))
    return str(p)


def test_traffic_taken_while_source_unchanged(tmp_path):
    src = os.path.join(CSRC, "steps_periodic.hip")
    digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
    assert bench.profile_traffic(_summary(tmp_path, digest)) == 123456.0


def test_traffic_dropped_after_source_change(tmp_path):
    assert bench.profile_traffic(_summary(tmp_path, "0" * 64)) is None
    assert bench.profile_traffic(_summary(tmp_path, "0" * 64, name="missing.hip")) is None
    assert bench.profile_traffic(str(tmp_path / "absent.md")) is None


def test_committed_summaries_name_their_source():
    # every committed summary carries a traffic figure and the digest of a
    # source file of the package
    prof = os.path.join(bench.ROOT, "profiles")
    names = [f for f in os.listdir(prof) if f.endswith(".md")]
    assert names
    for f in names:
        text = open(os.path.join(prof, f)).read()
        assert "traffic_bytes_per_launch:" in text, f
        line = [l for l in text.splitlines() if l.startswith("source_sha256:")]
        assert len(line) == 1, f
        name = line[0].split()[2].strip("()")
        assert os.path.exists(os.path.join(CSRC, name)), (f, name)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(bench.ROOT, "bench.py"),
                        "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_counter_figures_of_committed_summaries():
    # the headline kernels' summaries give the clock, the pipe or issue
    # figure and the executed flops that the bench line restates
    f64 = bench.counter_roofline(
        bench.profile_path("fp64", {"r": 1, "tj": 256, "variant": 30}, 3), 0.75)
    assert f64 is not None
    assert 2.0 < f64["clock_ghz"] < 2.5
    assert 0.0 < f64["fp64_pipe_busy"] <= 1.0
    assert 0.0 < f64["executed_flop_per_pair"] < 40.0
    assert abs(f64["frac_at_measured_clock"] - 0.75 * 2.4 / f64["clock_ghz"]) < 1e-12
    mixed = bench.counter_roofline(
        bench.profile_path("mixed", {"r": 4, "tj": 256, "variant": 10}, 3), 0.7)
    assert mixed is not None and 1.0 < mixed["valu_issue_vs_single"] < 2.0
    assert "fp64_pipe_busy" not in mixed
    assert bench.counter_roofline(
        bench.profile_path("fp64", {"r": 9, "tj": 256, "variant": 30}, 3), 0.7) is None
