"""GPU parity of H|psi> (qeh_apply_h through the C ABI) against the FP64 oracle.

Bars: FP64 form, per-band relative L2 <= 1e-12 and element-wise
|d| <= 1e-12 max|H psi|; mixed form (FP32 FFTs and projector GEMMs),
per-band relative L2 <= 1e-5.  Batch invariance (a band's result does not
depend on the other bands in its launch) is checked bitwise.
"""

import numpy as np
import pytest

import cellgen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _qeh():
    import paper_2104_10502_amd as q
    return q


def _rel_l2(a, b):
    return np.linalg.norm(a - b, axis=1) / np.linalg.norm(b, axis=1)


_CELLS = {}


def cell(name, **kw):
    key = (name, tuple(sorted(kw.items())))
    if key not in _CELLS:
        _CELLS[key] = cellgen.make_cell(name, **kw)
    return _CELLS[key]


def run(c, psi, precision, block, part=None):
    q = _qeh()
    ctx = q.Context.from_cell(c, precision=precision, block=block)
    d = torch.from_numpy(psi).cuda()
    out = ctx.apply_h(d, part=part)
    torch.cuda.synchronize()
    return out.cpu().numpy(), ctx


@pytest.mark.parametrize("prec", [0, 1])
def test_apply_h_c1(prec):
    c = cell("c1")
    psi = cellgen.make_psi0(c.npw, 16)
    print("case c1 prec", prec, flush=True)
    got, ctx = run(c, psi, prec, 16)
    ref = oracle.apply_h(c, psi)
    err = _rel_l2(got, ref)
    if prec == 0:
        assert err.max() < 1e-12, err.max()
        assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()
    else:
        assert err.max() < 1e-5, err.max()


@pytest.mark.parametrize("prec", [0, 1])
def test_apply_h_parts_c1(prec):
    c = cell("c1")
    psi = cellgen.make_psi0(c.npw, 5, seed=3)
    loc, _ = run(c, psi, prec, 4, part=0)
    nl, _ = run(c, psi, prec, 4, part=1)
    ref_loc = oracle.kinetic(c)[None, :] * psi + oracle.vloc_psi(c, psi)
    ref_nl = oracle.vnl_psi(c, psi)
    tol = 1e-12 if prec == 0 else 1e-5
    assert _rel_l2(loc, ref_loc).max() < tol
    assert _rel_l2(nl, ref_nl).max() < tol * 10


@pytest.mark.parametrize("prec", [0, 1])
def test_apply_h_c2_sampled(prec):
    # full C2 shape (72^3 box, 23976 plane waves, 512 projectors) on 6 bands,
    # launched in blocks of 4 (one full block and a ragged tail)
    c = cell("c2")
    psi = cellgen.make_psi0(c.npw, 6, seed=21)
    print("case c2 prec", prec, flush=True)
    got, ctx = run(c, psi, prec, 4)
    ref = oracle.apply_h(c, psi)
    err = _rel_l2(got, ref)
    assert err.max() < (1e-12 if prec == 0 else 1e-5), err.max()


def test_apply_h_anisotropic_radix7():
    # non-cubic cell, general k, s/p/d projectors, box with radix 7 and odd sizes
    c = cellgen.make_cell("t", lattice=np.diag([7.0, 8.0, 9.5]), frac=np.array(
        [[0.1, 0.2, 0.3], [0.6, 0.5, 0.9], [0.3, 0.8, 0.55]]), kpt=(0.11, -0.07, 0.23),
        ecutwfc=12.0, fft=(21, 25, 28), proj="s2pd", dfixed=False, nbnd=8)
    psi = cellgen.make_psi0(c.npw, 7, seed=5)
    ref = oracle.apply_h(c, psi)
    for prec in (0, 1):
        got, _ = run(c, psi, prec, 3)
        assert _rel_l2(got, ref).max() < (1e-12 if prec == 0 else 1e-5)


@pytest.mark.parametrize("prec", [0, 1])
def test_batch_invariance_bitwise(prec):
    c = cell("c1")
    psi = cellgen.make_psi0(c.npw, 9, seed=8)
    q = _qeh()
    ctx = q.Context.from_cell(c, precision=prec, block=16)
    d = torch.from_numpy(psi).cuda()
    full = ctx.apply_h(d).cpu().numpy()
    one = np.stack([ctx.apply_h(d[i:i + 1]).cpu().numpy()[0] for i in range(9)])
    assert np.array_equal(full, one)


def test_hermiticity_and_linearity_gpu():
    c = cell("c1")
    q = _qeh()
    ctx = q.Context.from_cell(c, precision=0, block=8)
    a = cellgen.make_psi0(c.npw, 2, seed=31)
    d = torch.from_numpy(a).cuda()
    h = ctx.apply_h(d).cpu().numpy()
    assert abs(np.vdot(a[0], h[1]) - np.conj(np.vdot(a[1], h[0]))) < 1e-13
    lin = ctx.apply_h(torch.from_numpy((0.5 - 2j) * a[:1] + 3j * a[1:2]).cuda()).cpu().numpy()
    assert np.abs(lin[0] - ((0.5 - 2j) * h[0] + 3j * h[1])).max() < 1e-13 * np.abs(h).max() * 10


@pytest.mark.parametrize("prec", [0, 1])
def test_apply_h_split_plane_path(prec, monkeypatch):
    # the HBM-staged plane path (used when a plane's column tile exceeds LDS),
    # forced on a small anisotropic cell with ragged column / row groups
    monkeypatch.setenv("QEH_FORCE_SPLIT_PLANE", "1")
    c = cellgen.make_cell("t", lattice=np.diag([9.0, 8.0, 9.5]), frac=np.array(
        [[0.1, 0.2, 0.3], [0.6, 0.5, 0.9]]), kpt=(0.11, -0.07, 0.23), ecutwfc=40.0,
        fft=(40, 35, 42), proj="s2pd", dfixed=False, nbnd=5)
    psi = cellgen.make_psi0(c.npw, 5, seed=6)
    got, ctx = run(c, psi, prec, 3)
    assert ctx.info()["plane_path"] == 1 and ctx.info()["ext"] > 16
    ref = oracle.apply_h(c, psi)
    assert _rel_l2(got, ref).max() < (1e-12 if prec == 0 else 1e-5)


@pytest.mark.parametrize("prec", [0, 1])
def test_apply_h_c2_bench_launch(prec):
    # the benchmark's launch configuration: all 128 bands in one block;
    # sampled bands against the oracle
    c = cell("c2")
    psi = cellgen.make_psi0(c.npw, 128, seed=10502)
    got, _ = run(c, psi, prec, 128)
    idx = [0, 57, 127]
    ref = oracle.apply_h(c, psi[idx])
    err = _rel_l2(got[idx], ref)
    assert err.max() < (1e-12 if prec == 0 else 1e-5), err


def test_plane_kernel_choice_c1(monkeypatch):
    # the mixed form of a cubic box with a compiled lane-pair size takes the
    # lane-pair plane kernel; QEH_PLANE_KERNEL=generic keeps the fused one
    c = cell("c1")
    q = _qeh()
    assert q.Context.from_cell(c, precision=1, block=4).info()["plane_path"] == 2
    assert q.Context.from_cell(c, precision=0, block=4).info()["plane_path"] == 0
    monkeypatch.setenv("QEH_PLANE_KERNEL", "generic")
    assert q.Context.from_cell(c, precision=1, block=4).info()["plane_path"] == 0


@pytest.mark.parametrize("kernel", ["pair", "generic"])
def test_apply_h_c1_mixed_plane_kernels(kernel, monkeypatch):
    if kernel == "generic":
        monkeypatch.setenv("QEH_PLANE_KERNEL", "generic")
    c = cell("c1")
    psi = cellgen.make_psi0(c.npw, 16, seed=41)
    got, ctx = run(c, psi, 1, 16)
    assert ctx.info()["plane_path"] == (2 if kernel == "pair" else 0)
    err = _rel_l2(got, oracle.apply_h(c, psi))
    assert err.max() < 1e-5, err.max()


@pytest.mark.parametrize("pb", [1, 3, 8])
def test_apply_h_pair_planes_per_workgroup(pb, monkeypatch):
    # bands per lane-pair workgroup 1, 3 and 8 on 7 bands in blocks of 5:
    # ragged band groups in both launches
    monkeypatch.setenv("QEH_PAIR_PLANES", str(pb))
    c = cell("c1")
    psi = cellgen.make_psi0(c.npw, 7, seed=42)
    got, ctx = run(c, psi, 1, 5)
    assert ctx.info()["plane_path"] == 2
    err = _rel_l2(got, oracle.apply_h(c, psi))
    assert err.max() < 1e-5, err.max()


def test_apply_h_pair_small_box_general_k():
    # N1 = N2 = 18 (in-lane length 9), non-cubic lattice, general k, s/p/d
    # projectors, odd x-extent 7
    c = cellgen.make_cell("t", lattice=np.diag([7.0, 7.0, 9.5]), frac=np.array(
        [[0.1, 0.2, 0.3], [0.6, 0.5, 0.9]]), kpt=(0.11, -0.07, 0.23), ecutwfc=12.0,
        fft=(18, 18, 28), proj="s2pd", dfixed=False, nbnd=8)
    psi = cellgen.make_psi0(c.npw, 6, seed=43)
    got, ctx = run(c, psi, 1, 4)
    assert ctx.info()["plane_path"] == 2 and ctx.info()["ext"] == 7
    err = _rel_l2(got, oracle.apply_h(c, psi))
    assert err.max() < 1e-5, err.max()


def test_pair_matches_generic_c2():
    # the two mixed plane kernels agree on the full C2 shape to FP32 rounding
    import os
    c = cell("c2")
    psi = cellgen.make_psi0(c.npw, 4, seed=44)
    a, ca = run(c, psi, 1, 4)
    os.environ["QEH_PLANE_KERNEL"] = "generic"
    try:
        b, cb = run(c, psi, 1, 4)
    finally:
        del os.environ["QEH_PLANE_KERNEL"]
    assert ca.info()["plane_path"] == 2 and cb.info()["plane_path"] == 0
    assert _rel_l2(a, b).max() < 2e-6


@pytest.mark.parametrize("kernel", ["pair", "generic"])
def test_apply_h_c1_mixed_stick_kernels(kernel, monkeypatch):
    # the lane-pair z transforms (K1 / K3) and the LDS-pass ones
    if kernel == "generic":
        monkeypatch.setenv("QEH_STICK_KERNEL", "generic")
    c = cell("c1")
    psi = cellgen.make_psi0(c.npw, 16, seed=45)
    got, ctx = run(c, psi, 1, 16)
    assert ctx.info()["stick_path"] == (1 if kernel == "pair" else 0)
    err = _rel_l2(got, oracle.apply_h(c, psi))
    assert err.max() < 1e-5, err.max()


def test_stick_path_choice():
    q = _qeh()
    c1 = cell("c1")
    assert q.Context.from_cell(c1, precision=1, block=4).info()["stick_path"] == 1
    assert q.Context.from_cell(c1, precision=0, block=4).info()["stick_path"] == 0
    # N3 = 30 has a compiled size, 21 x 25 planes do not: pair sticks with
    # generic planes (and the reverse on the radix-7 box 21 x 25 x 28), both
    # checked against the oracle
    for fft, sticks in (((21, 25, 30), 1), ((21, 25, 28), 0)):
        t = cellgen.make_cell("t", lattice=np.diag([7.0, 8.0, 9.5]), frac=np.array(
            [[0.1, 0.2, 0.3], [0.6, 0.5, 0.9]]), kpt=(0.11, -0.07, 0.23), ecutwfc=12.0,
            fft=fft, proj="s2pd", dfixed=False, nbnd=6)
        psi = cellgen.make_psi0(t.npw, 6, seed=47)
        got, ctx = run(t, psi, 1, 4)
        assert ctx.info()["stick_path"] == sticks and ctx.info()["plane_path"] == 0
        assert _rel_l2(got, oracle.apply_h(t, psi)).max() < 1e-5


def test_pair_sticks_match_generic_c2(monkeypatch):
    c = cell("c2")
    psi = cellgen.make_psi0(c.npw, 4, seed=46)
    a, ca = run(c, psi, 1, 4)
    monkeypatch.setenv("QEH_STICK_KERNEL", "generic")
    b, cb = run(c, psi, 1, 4)
    assert ca.info()["stick_path"] == 1 and cb.info()["stick_path"] == 0
    assert _rel_l2(a, b).max() < 2e-6


def test_apply_h_quad_fp64_small_box():
    # FP64 lane-quad plane kernel at N1 = N2 = 24 (6 points per lane), non-cubic
    # lattice, general k, s/p/d projectors; against the oracle at the FP64 bar
    c = cellgen.make_cell("t", lattice=np.diag([8.0, 8.0, 9.5]), frac=np.array(
        [[0.1, 0.2, 0.3], [0.6, 0.5, 0.9]]), kpt=(0.11, -0.07, 0.23), ecutwfc=14.0,
        fft=(24, 24, 28), proj="s2pd", dfixed=False, nbnd=6)
    psi = cellgen.make_psi0(c.npw, 6, seed=48)
    got, ctx = run(c, psi, 0, 4)
    assert ctx.info()["plane_path"] == 4
    ref = oracle.apply_h(c, psi)
    assert _rel_l2(got, ref).max() < 1e-12
    assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("pb", [1, 2])
def test_quad_matches_generic_fp64_c2(pb, monkeypatch):
    # the two FP64 plane kernels on the 72^3 cell, one and two bands per
    # lane-quad workgroup (5 bands: a ragged group)
    c = cell("c2")
    psi = cellgen.make_psi0(c.npw, 5, seed=49)
    monkeypatch.setenv("QEH_PAIR_PLANES", str(pb))
    a, ca = run(c, psi, 0, 5)
    monkeypatch.setenv("QEH_PLANE_KERNEL", "generic")
    b, cb = run(c, psi, 0, 5)
    assert ca.info()["plane_path"] == 4 and cb.info()["plane_path"] == 0
    assert _rel_l2(a, b).max() < 1e-13


@pytest.mark.parametrize("n", [96, 120])
def test_apply_h_quad_single_precision(n, monkeypatch):
    # single-precision lane-quad plane kernel (boxes above the lane-pair
    # sizes): N1 = N2 = n, N3 = 40, a non-cubic lattice, general k, s/p/d
    # projectors, 7 bands in blocks of 3 (ragged); against the oracle at the
    # mixed-form bar, and against the fused LDS-pass kernel
    c = cellgen.make_cell("t", lattice=np.diag([22.0, 22.0, 9.0]), frac=np.array(
        [[0.1, 0.2, 0.3], [0.6, 0.5, 0.9], [0.3, 0.8, 0.45]]), kpt=(0.11, -0.07, 0.23),
        ecutwfc=14.0, fft=(n, n, 40), proj="s2pd", dfixed=False, nbnd=7)
    psi = cellgen.make_psi0(c.npw, 7, seed=51)
    got, ctx = run(c, psi, 1, 3)
    assert ctx.info()["plane_path"] == 4
    ref = oracle.apply_h(c, psi)
    assert _rel_l2(got, ref).max() < 1e-5, _rel_l2(got, ref).max()
    monkeypatch.setenv("QEH_PLANE_KERNEL", "generic")
    gen, cg = run(c, psi, 1, 3)
    assert cg.info()["plane_path"] == 0
    assert _rel_l2(got, gen).max() < 1e-5
