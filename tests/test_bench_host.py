"""Host-side logic of bench.py (no GPU): the one-GPU refusal, the rule that
reports measured HBM traffic only for the kernel source it was taken on,
the algorithmic byte counts of the roofline, and the launch counts the
per-launch figures are divided by."""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1510_02237_amd import workloads as W  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"),
                        "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def _profile(tmp_path, value, sha):
    p = tmp_path / "traffic.md"
    p.write_text(f"# summary\n\ntraffic_bytes_per_point_step: {value}\n"
                 f"fine_hip_sha256_16: {sha}\n")
    return str(p)


def test_traffic_needs_the_current_kernel_source(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC_FILE",
                        _profile(tmp_path, 50.5, bench.fine_src_hash()))
    assert bench.measured_traffic() == 50.5
    monkeypatch.setattr(bench, "TRAFFIC_FILE",
                        _profile(tmp_path, 50.5, "0123456789abcdef"))
    assert bench.measured_traffic() is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.md"))
    assert bench.measured_traffic() is None


def test_committed_traffic_profile_is_well_formed():
    """The committed summary carries both machine-read lines, a per-point
    figure no smaller than the algorithmic 48 bytes, and a 16-digit hash."""
    txt = open(bench.TRAFFIC_FILE).read().splitlines()
    vals = dict(l.split(":", 1) for l in txt
                if l.startswith(("traffic_bytes_per_point_step:",
                                 "fine_hip_sha256_16:")))
    assert float(vals["traffic_bytes_per_point_step"]) >= bench.BYTES_PER_POINT_STEP
    h = vals["fine_hip_sha256_16"].strip()
    assert len(h) == 16 and int(h, 16) >= 0


def test_roofline_byte_counts():
    # one RK-3 step (one launch in either form) reads and writes the three
    # fields once: 2 * 3 * 8 bytes
    assert bench.BYTES_PER_POINT_STEP == 2 * 3 * 8


@pytest.mark.parametrize("kw,stage", [
    ({}, False), ({"V": 0.1}, True), ({"gamma": 1.0}, True),
    ({"fine_acoustic_order": 2}, True), ({"scheme": "rk3"}, True)])
def test_stage_form_rule(kw, stage):
    prob, _, _ = W.config("c2_512x256")
    assert bench.stage_form(dict(prob, **kw)) is stage


def test_launch_counts_of_the_benchmarked_workload():
    """512x256, P = 32 over T = 1 at fine CFL 0.2: 80 fine RK-3 steps and 8
    coarse steps per slice, one window."""
    prob, K, _ = W.config("c2_512x256")
    assert (prob["nx"], prob["nz"], prob["P"], K) == (512, 256, 32, 4)
    assert bench.ctx_nf(prob) == 80
    assert bench.ctx_ng(prob) == 8
    assert prob.get("windows", 1) == 1
    assert not bench.stage_form(prob)
