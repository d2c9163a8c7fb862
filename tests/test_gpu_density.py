"""GPU parity of the charge density (qeh_density through the C ABI) against
the FP64 oracle.

Bars: FP64 form, max |d rho| <= 1e-12 max rho over the whole grid; mixed form
(FP32 transforms, FP64 sums), max |d rho| <= 1e-5 max rho.  Both plane
layouts of the context (lane-pair tables and digit-reversed tables), ragged
band blocks, the split plane path, the full 72^3 cell, and the quadrature
property at the benchmark's 128 bands.
"""

import numpy as np
import pytest

import cellgen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _q():
    import paper_2104_10502_amd as q
    return q


def _rho(c, psi, occ, prec, block):
    q = _q()
    ctx = q.Context.from_cell(c, precision=prec, block=block)
    out = ctx.density(torch.from_numpy(psi).cuda(), occ)
    torch.cuda.synchronize()
    return out.cpu().numpy(), ctx


def _check(got, ref, prec):
    tol = 1e-12 if prec == 0 else 1e-5
    err = np.abs(got - ref).max() / np.abs(ref).max()
    assert err < tol, err


@pytest.mark.parametrize("prec", [0, 1])
def test_density_c1(prec):
    c = cellgen.make_cell("c1")
    psi = cellgen.make_psi0(c.npw, 16, seed=81)
    occ = np.linspace(2.0, 0.1, 16)
    print("case density c1 prec", prec, flush=True)
    got, ctx = _rho(c, psi, occ, prec, 16)
    assert got.shape == (30, 30, 30)
    _check(got, oracle.density(c, psi, occ), prec)


@pytest.mark.parametrize("prec", [0, 1])
def test_density_ragged_blocks(prec):
    # 21 bands in blocks of 8 (two full blocks and a tail of 5, each block
    # summed onto the previous ones), weights of both signs
    c = cellgen.make_cell("c1")
    psi = cellgen.make_psi0(c.npw, 21, seed=82)
    occ = np.cos(np.arange(21.0))
    got, _ = _rho(c, psi, occ, prec, 8)
    _check(got, oracle.density(c, psi, occ), prec)


@pytest.mark.parametrize("env", [{}, {"QEH_DENSITY_KERNEL": "rows"},
                                 {"QEH_DENSITY_KERNEL": "generic"},
                                 {"QEH_PLANE_KERNEL": "generic"}])
def test_density_paths_mixed(env, monkeypatch):
    # the fused lane-pair plane pass (default at mixed C1), lane-pair rows after
    # the HBM column pass, LDS-pass rows, and a context with digit-reversed
    # plane tables: each against the oracle and against the default
    c = cellgen.make_cell("c1")
    psi = cellgen.make_psi0(c.npw, 5, seed=83)
    occ = [2.0, 2.0, 1.0, 1.0, 0.5]
    ref = oracle.density(c, psi, occ)
    a, _ = _rho(c, psi, occ, 1, 5)
    for k, v in env.items():
        monkeypatch.setenv(k, v)
    b, _ = _rho(c, psi, occ, 1, 5)
    _check(b, ref, 1)
    assert np.abs(a - b).max() < 2e-6 * np.abs(ref).max()


@pytest.mark.parametrize("prec", [0, 1])
def test_density_split_path_anisotropic(prec, monkeypatch):
    monkeypatch.setenv("QEH_FORCE_SPLIT_PLANE", "1")
    c = cellgen.make_cell("t", lattice=np.diag([9.0, 8.0, 9.5]), frac=np.array(
        [[0.1, 0.2, 0.3], [0.6, 0.5, 0.9]]), kpt=(0.11, -0.07, 0.23), ecutwfc=40.0,
        fft=(40, 35, 42), proj="s2pd", dfixed=False, nbnd=5)
    psi = cellgen.make_psi0(c.npw, 5, seed=84)
    occ = [2.0, 1.5, 1.0, 0.5, 0.25]
    got, ctx = _rho(c, psi, occ, prec, 3)
    assert ctx.info()["plane_path"] == 1
    _check(got, oracle.density(c, psi, occ), prec)


@pytest.mark.parametrize("prec", [0, 1])
def test_density_c2_full_grid(prec):
    c = cellgen.make_cell("c2")
    psi = cellgen.make_psi0(c.npw, 3, seed=85)
    occ = [2.0, 2.0, 2.0]
    print("case density c2 prec", prec, flush=True)
    got, _ = _rho(c, psi, occ, prec, 3)
    _check(got, oracle.density(c, psi, occ), prec)


@pytest.mark.parametrize("prec", [0, 1])
def test_density_c2_bench_quadrature(prec):
    # the benchmark configuration (128 bands in one block): the grid integral
    # equals the occupation sum (normalised bands), rho >= 0, and one sampled
    # band's density matches the oracle at the sampled z planes
    c = cellgen.make_cell("c2")
    psi = cellgen.make_psi0(c.npw, 128, seed=10502)
    occ = np.full(128, 2.0)
    got, ctx = _rho(c, psi, occ, prec, 128)
    n = np.prod(c.fft)
    total = oracle.cell_volume(c) / n * got.sum()
    assert abs(total - occ.sum()) < (1e-9 if prec == 0 else 1e-4) * occ.sum()
    assert got.min() >= 0.0
    one, _ = _rho(c, psi[57:58], [1.0], prec, 128)
    _check(one, oracle.density(c, psi[57:58], [1.0]), prec)


def test_density_zero_bands_and_errors():
    q = _q()
    c = cellgen.make_cell("c1")
    ctx = q.Context.from_cell(c, precision=0, block=4)
    empty = torch.zeros((0, c.npw), dtype=torch.complex128, device="cuda")
    out = torch.full((30, 30, 30), 7.0, dtype=torch.float64, device="cuda")
    ctx.density(empty, [], out=out)
    assert float(out.abs().max()) == 0.0
    psi = torch.from_numpy(cellgen.make_psi0(c.npw, 2, seed=1)).cuda()
    with pytest.raises(q.QehError):
        ctx.density(psi, [1.0, float("nan")])
    # a workspace shorter than qeh_density_plan's is rejected by the library
    import ctypes
    small = torch.empty(256, dtype=torch.uint8, device="cuda")
    occ = np.array([1.0, 1.0])
    st = q._lib.qeh_density(ctx._h, 2, ctypes.c_void_p(psi.data_ptr()), psi.stride(0),
                            occ.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                            ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(small.data_ptr()),
                            256)
    assert st == q.QEH_ERR_INVALID


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_density_row_kernels_agree_mixed(name, monkeypatch):
    # lane-pair rows (default in the mixed form at these boxes) and the
    # LDS-pass rows: both against the oracle, and against each other
    c = cellgen.make_cell(name)
    psi = cellgen.make_psi0(c.npw, 5, seed=86)
    occ = [2.0, 1.0, 1.0, 0.5, 0.25]
    a, _ = _rho(c, psi, occ, 1, 5)
    monkeypatch.setenv("QEH_DENSITY_KERNEL", "generic")
    b, _ = _rho(c, psi, occ, 1, 5)
    ref = oracle.density(c, psi, occ)
    _check(a, ref, 1)
    _check(b, ref, 1)
    assert np.abs(a - b).max() < 2e-6 * np.abs(ref).max()


@pytest.mark.parametrize("fft", [(32, 32, 32), (24, 24, 30)])
def test_density_fp64_fused_quad(fft, monkeypatch):
    # FP64 contexts on the lane-quad plane kernel take the fused lane-quad
    # density pass (11 bands: subgroups of 8 and 3); against the oracle and
    # against the unfused LDS-pass rows
    c = cellgen.make_cell("c1", fft=fft)
    psi = cellgen.make_psi0(c.npw, 11, seed=87)
    occ = np.linspace(2.0, 0.2, 11)
    a, ctx = _rho(c, psi, occ, 0, 11)
    assert ctx.info()["plane_path"] == 4
    ref = oracle.density(c, psi, occ)
    _check(a, ref, 0)
    monkeypatch.setenv("QEH_DENSITY_KERNEL", "generic")
    b, _ = _rho(c, psi, occ, 0, 11)
    _check(b, ref, 0)
