"""Full-size cells on the GPU, sampled bands against the FP64 oracle:

* the 256-atom jittered cell (135^3 box, 148 093 plane waves, 2048
  projectors), H applied in blocks of 64 bands;
* the 512-atom orthorhombic cell (160x160x168 box with radix 7, 186 449
  plane waves, 6144 s/p/d projectors), H applied in blocks of 128 bands;
  its FP64 planes exceed LDS and go through the split plane path.

Both cells are at k = 0 (the Gamma point), so each also runs on the Gamma
path: half the sphere stored, bands paired in the FFT (the sampled bands are
the two members of one pair and one band of another).

Bars: FP64 per-band relative L2 <= 1e-12, mixed <= 1e-5.  The oracle evaluates
a few bands of each launch one by one (dense per-axis DFTs of a few million
points).
"""

import numpy as np
import pytest

import cellgen
import oracle
from oracle import gamma

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _rel_l2(a, b):
    return np.linalg.norm(a - b, axis=1) / np.linalg.norm(b, axis=1)


@pytest.fixture(scope="module")
def c3():
    return cellgen.make_cell("c3")


@pytest.fixture(scope="module")
def c5():
    return cellgen.make_cell("c5")


def _check(c, nb, block, idx):
    import paper_2104_10502_amd as q
    psi = cellgen.make_psi0(c.npw, nb, seed=10502)
    ref = oracle.apply_h(c, psi[idx])
    d = torch.from_numpy(psi).cuda()
    for prec, tol in ((q.QEH_MIXED, 1e-5), (q.QEH_FP64, 1e-12)):
        ctx = q.Context.from_cell(c, precision=prec, block=block)
        print(c.name, "precision", prec, ctx.info(), flush=True)
        out = ctx.apply_h(d).cpu().numpy()
        err = _rel_l2(out[idx], ref)
        print("  rel L2", err, flush=True)
        assert err.max() < tol
        ctx.close()
        del out
        torch.cuda.empty_cache()


def test_apply_h_c3_sampled(c3):
    _check(c3, 64, 64, [0, 63])


def test_apply_h_c5_sampled(c5):
    _check(c5, 128, 128, [5, 127])


def _check_gamma(c, nb, block, idx):
    import paper_2104_10502_amd as q
    h = cellgen.gamma_half(c)
    psi = cellgen.make_psi0(h.npw, nb, seed=10503)
    psi[:, 0] = psi[:, 0].real
    ref = gamma.restrict(oracle.apply_h(c, gamma.expand(psi[idx])))
    d = torch.from_numpy(psi).cuda()
    for prec, tol in ((q.QEH_MIXED, 1e-5), (q.QEH_FP64, 1e-12)):
        ctx = q.Context.from_cell(h, precision=prec, block=block)
        print(c.name, "gamma precision", prec, ctx.info(), flush=True)
        out = ctx.apply_h(d).cpu().numpy()
        err = _rel_l2(out[idx], ref)
        print("  rel L2", err, flush=True)
        assert err.max() < tol
        ctx.close()
        del out
        torch.cuda.empty_cache()


def test_apply_h_c3_gamma_sampled(c3):
    _check_gamma(c3, 64, 64, [10, 11, 63])


def test_apply_h_c5_gamma_sampled(c5):
    _check_gamma(c5, 128, 128, [4, 5, 126])
