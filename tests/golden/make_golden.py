"""Write the stored expected values under tests/golden/ from the FP64 oracle.

Calls only ``oracle`` and the seeded generator ``cellgen``; nothing from the
HIP library.  Usage: python tests/golden/make_golden.py [c2]
"""

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import cellgen  # noqa: E402
import oracle   # noqa: E402


def c2_eigs():
    cell = cellgen.make_cell("c2")
    nb = cell.nbnd
    psi0 = cellgen.make_psi0(cell.npw, nb, seed=10502)
    t = time.time()
    eps, psi, info = oracle.davidson(lambda x: oracle.apply_h(cell, x), psi0, oracle.hdiag(cell),
                                     rtol=1e-9, nvecx=4 * nb, maxiter=400)
    dt = time.time() - t
    assert info["converged"], info
    path = os.path.join(HERE, "c2_eigs.txt")
    with open(path, "w") as f:
        f.write("# C2 cell (64-atom diamond supercell a=20.52 bohr, k=(1/4,1/4,1/4) 2pi/a,\n")
        f.write("# ecutwfc 30 Ry, box 72^3, 512 projectors, seed 2104, psi0 seed 10502):\n")
        f.write("# lowest %d eigenvalues (Ry) from the FP64 oracle block Davidson,\n" % nb)
        f.write("# residual norms <= 1e-9; %d iterations, %d band applies, %.0f s.\n"
                % (info["iters"], info["band_applies"], dt))
        for e in eps:
            f.write("%.15e\n" % e)
    print("wrote", path, info["iters"], info["band_applies"], "%.0f s" % dt)


if __name__ == "__main__":
    which = sys.argv[1:] or ["c2"]
    if "c2" in which:
        c2_eigs()
