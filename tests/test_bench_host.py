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
    # dominant kernel, each fraction is achieved / peak of its bound; the plane
    # pass is priced by its HBM bytes with its transform flops against the
    # one-wide vector peak beside them
    shape = dict(npw=23976, nst=1007, nkb=512, n1=72, n2=72, n3=72, ext=36, block=128,
                 precision=1, plane_path=2, stick_path=1, gamma=False)
    stages = {"k2_plane": (0.170 * 20, 20), "calbec_gemm": (0.100 * 20, 20)}
    best, per = bench.roofline_for(stages, shape, 1, 128)
    assert best == "k2_plane"
    k2 = per["k2_plane"]
    byts = 128 * 2 * 8 * 1007 * 72 + 4 * 72 ** 3
    assert k2["bound"] == "hbm" and abs(k2["achieved"] - byts / 170e-6 / 1e9) < 1e-6
    assert abs(k2["frac"] - k2["achieved"] / 8000.0) < 1e-12
    assert k2["alu_peak_one_wide"] == 78.6
    assert abs(k2["alu_frac"] - k2["alu_TFLOPs"] / 78.6) < 1e-12
    g = per["calbec_gemm"]
    flops = 8.0 * 128 * 512 * 23976
    assert g["bound"] == "mfma" and abs(g["achieved"] - flops / 100e-6 / 1e12) < 1e-9


def test_gamma_accounting():
    # Gamma launches transform band pairs and run real products over the half
    # sphere: half the plane-pass stick bytes and half the GEMM flops of a
    # complex launch with the same stored coefficient count
    shape = dict(npw=93225, nst=3809, nkb=6144, n1=160, n2=160, n3=168, ext=69, block=128,
                 gamma=True)
    cshape = dict(shape, gamma=False)
    v = 4 * 160 * 160 * 168
    kb = bench.algorithmic("k2_plane", shape, 1, 128)[1] - v
    kc = bench.algorithmic("k2_plane", cshape, 1, 128)[1] - v
    assert kb * 2 == kc
    assert bench.algorithmic("calbec_gemm", shape, 1, 128)[1] * 2 == \
        bench.algorithmic("calbec_gemm", cshape, 1, 128)[1]
    assert bench.transforms(shape, 127) == 64


def test_host_cpu_record():
    hc = bench.host_cpu()
    assert hc["affinity"] >= 1 and hc["cpu_count"] >= hc["affinity"]


def test_served_request_with_tables():
    r = dict(nat=8, ecutwfc=20.0, nk=2, seed=7)
    cells, psis = bench._make_request(r, device_beta=True)
    assert len(cells) == 2 and all(c.beta is None and c.projgen is not None for c in cells)
    assert all(p.shape == (c.nbnd, c.npw) for c, p in zip(cells, psis))
    cells_h, _ = bench._make_request(r, device_beta=False)
    assert all(c.beta is not None and c.projgen is None for c in cells_h)
    assert np.array_equal(cells[0].miller, cells_h[0].miller)
