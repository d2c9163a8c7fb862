"""Wide single-precision projector tiles (128 bands x 128 or 256 projectors,
eight waves, 32 x 32 MFMA blocks) against the oracle, element by element.

The wide tiles run for QEH_MIXED contexts with >= 2048 projectors and a band
block of >= 128.  The cell here has 515 atoms with s + p projectors (2 060
projectors: a ragged last projector tile), ~3 900 plane waves (a ragged last
K slice) and 130 bands in blocks of 128 (a 2-band second block).  Both the
general-k form (three-product complex MFMA) and the Gamma forms (real
products) are checked, the nonlocal part alone and the whole H.
"""

import numpy as np
import pytest

import cellgen
import oracle
from oracle import gamma

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _q():
    import paper_2104_10502_amd as q
    return q


def _rel_l2(a, b):
    return np.linalg.norm(a - b, axis=1) / np.linalg.norm(b, axis=1)


def _many_projector_cell(k_zero):
    nat = 515
    a = (20.0 * nat) ** (1.0 / 3.0)
    frac = np.random.default_rng(4242).uniform(0.0, 1.0, size=(nat, 3))
    return cellgen.make_cell("serve", seed=4242, lattice=np.diag([a, a, a]), frac=frac,
                             kfrac=(0.0, 0.0, 0.0) if k_zero else (0.25, 0.25, 0.25),
                             ecutwfc=8.0, ecutrho=32.0, fft=None, proj="sp", dfixed=True,
                             nbnd=130, block=128)


@pytest.mark.parametrize("gamma_path", [False, True])
def test_wide_projector_tiles_vs_oracle(gamma_path):
    q = _q()
    c = _many_projector_cell(gamma_path)
    cell = cellgen.gamma_half(c) if gamma_path else c
    nb = 130
    psi = cellgen.make_psi0(cell.npw, nb, seed=77)
    if gamma_path:
        psi[:, 0] = psi[:, 0].real
        ref_h = gamma.restrict(oracle.apply_h(c, gamma.expand(psi)))
        ref_nl = gamma.restrict(oracle.vnl_psi(c, gamma.expand(psi)))
    else:
        ref_h = oracle.apply_h(c, psi)
        ref_nl = oracle.vnl_psi(c, psi)
    d = torch.from_numpy(psi).cuda()
    ctx = q.Context.from_cell(cell, precision=q.QEH_MIXED, block=128)
    info = ctx.info()
    print(c.name, "gamma" if gamma_path else "k", info, flush=True)
    assert info["wide_tiles"] == 1 and info["nkb"] == 2060
    nl = ctx.apply_h(d, part=1).cpu().numpy()
    h = ctx.apply_h(d).cpu().numpy()
    e_nl = _rel_l2(nl, ref_nl)
    e_h = _rel_l2(h, ref_h)
    print("  rel L2 nonlocal %.2e, H %.2e" % (e_nl.max(), e_h.max()), flush=True)
    assert e_nl.max() < 1e-5 and e_h.max() < 1e-5
    # the same bands in one block of 64 (64 x 64 tiles) agree to single
    # precision as well
    c64 = q.Context.from_cell(cell, precision=q.QEH_MIXED, block=64)
    assert c64.info()["wide_tiles"] == 0
    h64 = c64.apply_h(d).cpu().numpy()
    assert _rel_l2(h64, ref_h).max() < 1e-5
