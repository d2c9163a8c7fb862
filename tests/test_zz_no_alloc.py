"""qeh_beta_generate_static, the projector entry point that allocates nothing
(for callers that cannot allocate device memory): through the C ABI it must
give exactly the bits of qeh_beta_generate, call after call on the shared
static staging array, a larger input first and a smaller one after it, and
refuse inputs beyond the array with QEH_ERR_NOMEM."""

import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import cellgen  # noqa: E402

pytestmark = pytest.mark.gpu


def _q():
    import paper_2104_10502_amd as q
    return q


def _cells():
    big = cellgen.make_cell("c2", with_beta=False)                  # 64 atoms, 23 976 PW
    small = cellgen.random_served_cell(12, 25.0, 1, seed=3, with_beta=False)
    return big, small


@pytest.mark.parametrize("prec", [0, 1])
def test_static_matches_workspace_form_twice(prec):
    import torch
    q = _q()
    for cell in _cells():
        pg = cellgen.projgen_tables(cell)
        ref = q.generate_beta(cell.lattice, cell.kpt, cell.miller, cell.nproj, pg, precision=prec)
        # a padded output: columns beyond npw must stay untouched
        pad = torch.full((ref.shape[0], ref.shape[1] + 5), 7.0 + 1j, dtype=ref.dtype,
                         device=ref.device)
        got = q.generate_beta_static(cell.lattice, cell.kpt, cell.miller, cell.nproj, pg,
                                     precision=prec, out=pad)
        torch.cuda.synchronize()
        assert torch.equal(got[:, :cell.npw], ref), cell.name
        assert bool((got[:, cell.npw:] == (7.0 + 1j)).all())


def test_static_rejects_inputs_beyond_the_array():
    import torch
    q = _q()
    cell = cellgen.make_cell("c2", with_beta=False)
    pg = cellgen.projgen_tables(cell)
    # a sphere whose k+G staging alone exceeds the static array
    n = q.BETA_STATIC_BYTES // 24 + 1000
    reps = -(-n // cell.npw)
    miller = np.tile(cell.miller, (reps, 1))[:n]
    out = torch.empty((cell.nkb, n), dtype=torch.complex128, device="cuda")
    with pytest.raises(q.QehError) as ei:
        q.generate_beta_static(cell.lattice, cell.kpt, miller, cell.nproj, pg, out=out)
    assert ei.value.status == q.QEH_ERR_NOMEM
