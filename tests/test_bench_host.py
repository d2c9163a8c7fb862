"""Host-side pieces of bench.py (no GPU): the one-GPU contract, the roofline
bookkeeping, and the served-trace request builder."""

import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_roofline_bookkeeping():
    # a stage list of one plane pass and one GEMM: the longer one is the
    # dominant kernel, each fraction is achieved / peak of its bound, and the
    # one-wide FP32 figure is reported beside the plane pass
    shape = dict(npw=23976, nst=1007, nkb=512, n1=72, n2=72, n3=72, ext=36, block=128,
                 precision=1, plane_path=2, stick_path=1)
    stages = {"k2_plane": (0.170 * 20, 20), "calbec_gemm": (0.100 * 20, 20)}
    best, per = bench.roofline_for(stages, shape, 1, 128)
    assert best == "k2_plane"
    k2 = per["k2_plane"]
    assert k2["bound"] == "alu" and abs(k2["frac"] - k2["achieved"] / k2["peak"]) < 1e-12
    assert abs(k2["frac_one_wide_fp32"] - k2["achieved"] / k2["peak_one_wide_fp32"]) < 1e-12
    assert k2["peak_one_wide_fp32"] < k2["peak"]
    g = per["calbec_gemm"]
    flops = 8.0 * 128 * 512 * 23976
    assert g["bound"] == "mfma" and abs(g["achieved"] - flops / 100e-6 / 1e12) < 1e-9


def test_served_request_with_tables():
    r = dict(nat=8, ecutwfc=20.0, nk=2, seed=7)
    cells, psis = bench._make_request(r, device_beta=True)
    assert len(cells) == 2 and all(c.beta is None and c.projgen is not None for c in cells)
    assert all(p.shape == (c.nbnd, c.npw) for c, p in zip(cells, psis))
    cells_h, _ = bench._make_request(r, device_beta=False)
    assert all(c.beta is not None and c.projgen is None for c in cells_h)
    assert np.array_equal(cells[0].miller, cells_h[0].miller)
