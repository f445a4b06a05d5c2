"""Host-side logic of bench.py (CPU): the one-GPU guard, the d = 3 streamed-byte
model of the roofline, and the rule that PMC traffic is reported only for the
kernel sources it was measured on."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2108_09463_amd import inputs  # noqa: E402
from paper_2108_09463_amd import llhmm as L  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_three_d_roofline_bytes():
    """Per cell and step: 120 bytes per stage, less 24 at a step's first stage
    (RK4P 456, HeunP 216); frac is the rate over 8 TB/s."""
    eps = 0.01
    boxes = []
    for n, integ in ((8, 2), (12, 1), (16, 2)):
        boxes.append(inputs.make_box(dim=3, n=n, order=2, bc=0, quantity=inputs.Q_FIELD, integrator=integ,
                                     n_steps=5 + n, eps=eps, alpha=0.3, mu=3 * eps, mu_box=3 * eps,
                                     eta=0.3 * eps ** 2, a_max=1.5, center=(0.1, 0.2, 0.3),
                                     macro_index=(0, 0, 0)))
    M, _, ig = L.llhmm_plan(boxes)
    per_step = {2: 4 * 120 - 24, 1: 2 * 120 - 24}
    want = sum(int(m) * b["n"] ** 3 * per_step[int(g)] for b, m, g in zip(boxes, M, ig))
    assert per_step == {2: 456, 1: 216}
    r = bench.hbm_roofline_3d(boxes, kernel_ms=2.0)
    assert r["bytes_per_launch"] == pytest.approx(want, rel=0, abs=0.5)
    assert r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert r["frac"] == pytest.approx(want / 2.0e-3 / 8.0e12, rel=1e-12)
    assert r["achieved"] == pytest.approx(want / 2.0e-3 / 1e9, rel=1e-12)


def test_three_d_roofline_bytes_fourth_order():
    """Fourth order also reads the three stored faces of each cell: 144 bytes
    per stage, less 24 at a step's first stage (RK4P 552 per step); the PMC
    traffic of the second-order kernel is not reported for it."""
    eps = 0.01
    boxes = [inputs.make_box(dim=3, n=n, order=4, bc=0, quantity=inputs.Q_FIELD, integrator=2,
                             n_steps=4 + n, eps=eps, alpha=0.3, mu=3 * eps, mu_box=3 * eps,
                             eta=0.3 * eps ** 2, a_max=1.5, center=(0.1, 0.2, 0.3), macro_index=(0, 0, 0))
             for n in (8, 16)]
    M, _, ig = L.llhmm_plan(boxes)
    assert all(int(g) == 2 for g in ig)
    want = sum(int(m) * b["n"] ** 3 * (4 * 144 - 24) for b, m in zip(boxes, M))
    r = bench.hbm_roofline_3d(boxes, kernel_ms=4.0)
    assert r["bytes_per_launch"] == pytest.approx(want, rel=0, abs=0.5)
    assert r["bytes_per_cell_stage"] == 144.0
    assert r["kernel"] == "k_micro3d_o4" and r["traffic"] is None
    assert r["frac"] == pytest.approx(want / 4.0e-3 / 8.0e12, rel=1e-12)


def test_three_d_roofline_is_valu_primary():
    """The d = 3 record's roofline is the VALU one (algorithmic flops over the
    FP64 peak); the streamed-byte figure rides along as secondary."""
    eps = 0.01
    boxes = [inputs.make_box(dim=3, n=8, order=2, bc=0, quantity=inputs.Q_FIELD, integrator=2,
                             n_steps=6, eps=eps, alpha=0.3, mu=3 * eps, mu_box=3 * eps,
                             eta=0.3 * eps ** 2, a_max=1.5, center=(0.1, 0.2, 0.3), macro_index=(0, 0, 0))]
    flops = bench.algorithmic_flops(boxes)
    M, _, _ = L.llhmm_plan(boxes)
    assert flops == 281 * int(M[0]) * 8 ** 3          # F = 4 * 33 + 149 for d = 3, order 2, RK4P
    valu = dict(bound="alu", achieved=flops / 1e-3 / 1e12, peak=bench.PEAK_FP64 / 1e12, unit="TFLOP/s",
                frac=flops / 1e-3 / bench.PEAK_FP64, traffic=None)
    roof = bench.three_d_roofline(dict(roofline=valu, kernel_ms=1.0), boxes)
    assert roof["bound"] == "alu" and roof["unit"] == "TFLOP/s"
    assert roof["frac"] == pytest.approx(flops / 1e-3 / 78.6e12, rel=1e-12)
    assert roof["streamed_hbm"]["bound"] == "hbm" and roof["kernel"] == "k_micro3d"


def test_traffic_reported_only_for_the_measured_sources(tmp_path, monkeypatch):
    src = tmp_path / "kernel.hip"
    src.write_text("// kernel v1\n")
    summary = tmp_path / "traffic.txt"
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "KERNEL_SOURCES", ["kernel.hip"])
    monkeypatch.setattr(bench, "TRAFFIC_FILES", {"fp32": "traffic.txt"})
    assert bench.measured_traffic("fp32") is None          # no summary yet
    h = bench.kernel_source_hash(["kernel.hip"])
    summary.write_text(f"HBM traffic\nkernel_sources_sha256_16: {h}\nhbm_bytes_per_launch: 12345\n")
    assert bench.measured_traffic("fp32") == 12345.0
    src.write_text("// kernel v2\n")                        # the kernel changed since
    assert bench.measured_traffic("fp32") is None
