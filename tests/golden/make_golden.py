"""Write the stored expected values under tests/golden/ from the FP64 oracle.

Calls only ``oracle`` and the seeded generator ``cellgen``; nothing from the
HIP library.  Usage: python tests/golden/make_golden.py [c2] [c3] [c5] [served]

The 256- and 512-atom cells are solved for their lowest 64 and 32 bands only
(an oracle H application there takes seconds per band); the GPU solves all
512 / 1024 bands and its lowest ones are compared with these.
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


_CELL = None


def _vloc_band(x):
    return oracle.vloc_psi(_CELL, x[None, :])[0]


def _parallel_apply_h(cell, nproc):
    """oracle.apply_h with the local-potential term of each band computed in a
    separate forked worker (each band's transform is independent; the
    arithmetic per band is exactly apply_h's)."""
    import multiprocessing as mp
    global _CELL
    _CELL = cell
    pool = mp.get_context("fork").Pool(nproc)
    kin = oracle.kinetic(cell)

    def apply(x):
        x = np.atleast_2d(x)
        loc = np.array(pool.map(_vloc_band, list(x)))
        return kin[None, :] * x + loc + oracle.vnl_psi(cell, x)
    return apply, pool


def low_eigs(name: str, nb: int, header: str, nproc: int = 6):
    """Lowest nb eigenvalues of a Gamma cell, solved on the full complex sphere."""
    cell = cellgen.make_cell(name)
    psi0 = cellgen.make_psi0(cell.npw, nb, seed=10502)
    t = time.time()
    hd = oracle.hdiag(cell)
    apply, pool = _parallel_apply_h(cell, nproc)
    eps, psi, info = oracle.davidson(apply, psi0, hd, rtol=1e-9, nvecx=4 * nb, maxiter=400)
    pool.close()
    dt = time.time() - t
    assert info["converged"], info
    path = os.path.join(HERE, "%s_eigs.txt" % name)
    with open(path, "w") as f:
        f.write(header)
        f.write("# lowest %d eigenvalues (Ry) from the FP64 oracle block Davidson on the\n" % nb)
        f.write("# full complex sphere (psi0 seed 10502, nvecx %d), residual norms <= 1e-9;\n"
                % (4 * nb))
        f.write("# %d iterations, %d band applies, %.0f s.\n"
                % (info["iters"], info["band_applies"], dt))
        for e in eps:
            f.write("%.15e\n" % e)
    print("wrote", path, info["iters"], info["band_applies"], "%.0f s" % dt, flush=True)


# Served requests whose eigenvalues the serving test checks: (atoms, ecutwfc,
# k-points, cell seed), cells from the served-trace generator with host-built
# projectors (the s+p Gaussian form), nb = 2 atoms.
SERVED = [(128, 30.0, 1, 501), (64, 30.0, 2, 502), (96, 25.0, 2, 503), (40, 30.0, 3, 504),
          (16, 20.0, 4, 505)]


def served_eigs():
    import json
    out = []
    t = time.time()
    for nat, ecut, nk, seed in SERVED:
        ks = []
        for k in range(nk):
            cell = cellgen.random_served_cell(nat, ecut, k, seed)
            ks.append([float(x) for x in oracle.dense_eigs(cell, cell.nbnd)])
            print("served", nat, ecut, k, cell.npw, "%.0f s" % (time.time() - t), flush=True)
        out.append(dict(nat=nat, ecutwfc=ecut, nk=nk, seed=seed, eigs=ks))
    path = os.path.join(HERE, "served_eigs.json")
    with open(path, "w") as f:
        json.dump(dict(source="LAPACK eigenvalues of the FP64 oracle's dense H "
                              "(oracle.dense_eigs) of each k-point cell of "
                              "cellgen.random_served_cell(nat, ecutwfc, k, seed), host projectors",
                       requests=out), f, indent=1)
    print("wrote", path, "%.0f s" % (time.time() - t))


if __name__ == "__main__":
    which = sys.argv[1:] or ["c2"]
    if "c2" in which:
        c2_eigs()
    if "served" in which:
        served_eigs()
    if "c3" in which:
        low_eigs("c3", 64, "# 256-atom cell (cubic a=32.6 bohr, jittered FCC sites, k = 0, ecutwfc 40 Ry,\n"
                 "# box 135^3, 2048 projectors, seed 2104):\n")
    if "c5" in which:
        low_eigs("c5", 32, "# 512-atom cell (orthorhombic 40x40x42 bohr, diamond sites, k = 0,\n"
                 "# ecutwfc 30 Ry, box 160x160x168, 6144 s/p/d projectors, seed 2104):\n")
