"""Synthetic cells shaped like the paper's benchmark workloads.

The paper benchmarks pw.x on sixteen crystal structures of 250-1000 A^3 with
SSSP pseudopotentials (section "Evolution of the GPU-enabled version").  Those
structures and pseudopotentials are not available here, so these seeded cells
stand in for them: cubic / orthorhombic supercells with Gaussian model local
potentials and Gaussian-radial s/p/d projectors, sized to bracket the paper's
cells (tens to hundreds of atoms, tens of thousands to ~2e5 plane waves).

Conventions (Rydberg atomic units: lengths in bohr, energies in Ry, a plane
wave exp(i q.r) has kinetic energy |q|^2):

* ``lattice`` rows are a1, a2, a3; reciprocal rows b_i = 2 pi (A^-1)^T.
* ``miller`` is the (npw, 3) int32 list of (h, k, l) with |k + G|^2 <= ecutwfc,
  sorted lexicographically so that every (h, k) z-stick is one contiguous run
  of consecutive l.
* ``vloc`` is the real local potential on the FFT grid r_j = sum_i j_i/N_i a_i,
  shape (N3, N2, N1) with x fastest.
* ``beta`` is (nkb, npw) complex128, plane-wave index fastest, and already
  contains 1/sqrt(Omega) and the structure phase exp(-i (k+G).tau).
* ``qmat`` (optional, ``overlap=True``) holds per-atom q blocks of the overlap
  S = 1 + sum_ij |beta_i> q_ij <beta_j| in the layout of ``dmat``, one
  U[0.05, 0.5] value per (atom, channel) shared across m, drawn from the
  stream seeded with seed + 1 (q >= 0, so S is positive definite).
* ``dmat`` holds the per-atom Hermitian D blocks (nproj_a x nproj_a each,
  row-major) concatenated in atom order, complex128, in Ry.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

TWO_PI = 2.0 * math.pi

# Projector channel sets: list of (l, sigma) with beta_l(r) = r^l exp(-r^2/sigma).
PROJ_SETS = {
    "sp": [(0, 1.5), (1, 1.5)],                          # 4 per atom
    "2s2p": [(0, 1.5), (0, 0.75), (1, 1.5), (1, 0.75)],  # 8 per atom
    "s2pd": [(0, 1.5), (1, 1.5), (1, 0.75), (2, 1.5)],   # 12 per atom
}

# Model local potential v(r) = VLOC_AMP * exp(-r^2 / (2 VLOC_WIDTH^2)), Ry.
VLOC_AMP = -4.0
VLOC_WIDTH = 1.0
IMAGE_CUTOFF = 12.0   # bohr; the Gaussian tail beyond it is < 1e-30


@dataclass
class Cell:
    name: str
    lattice: np.ndarray
    fft: tuple
    kpt: np.ndarray
    ecutwfc: float
    ecutrho: float
    positions: np.ndarray
    miller: np.ndarray
    vloc: np.ndarray
    nproj: np.ndarray
    beta: np.ndarray
    dmat: np.ndarray
    nbnd: int
    block: int
    proj_set: str = "sp"
    meta: dict = field(default_factory=dict)
    # radial-table description of the projectors (see ``projgen_tables``);
    # when set, consumers may build beta from it instead of using ``beta``
    projgen: dict = None
    # True: a k = 0 cell stored over the half sphere (see ``gamma_half``)
    gamma: bool = False
    # per-atom Hermitian q blocks of the overlap S = 1 + sum |beta> q <beta|
    # (same layout as dmat); None: S = 1 (norm-conserving)
    qmat: np.ndarray = None

    @property
    def npw(self) -> int:
        return int(self.miller.shape[0])

    @property
    def nat(self) -> int:
        return int(self.positions.shape[0])

    @property
    def nkb(self) -> int:
        return int(self.nproj.sum())

    @property
    def omega(self) -> float:
        return float(abs(np.linalg.det(self.lattice)))

    @property
    def nfft(self) -> int:
        return int(self.fft[0] * self.fft[1] * self.fft[2])


# --------------------------------------------------------------------------
# lattice helpers


def reciprocal(lattice: np.ndarray) -> np.ndarray:
    """Rows b_i with a_i . b_j = 2 pi delta_ij."""
    return TWO_PI * np.linalg.inv(lattice).T


def is_5smooth(n: int) -> bool:
    for p in (2, 3, 5):
        while n % p == 0:
            n //= p
    return n == 1


def fft_box_min(lattice: np.ndarray, ecutrho: float) -> tuple:
    """Smallest 5-smooth N_i >= 2 floor(sqrt(ecutrho) |a_i| / 2 pi) + 1."""
    out = []
    for i in range(3):
        nmin = 2 * int(math.floor(math.sqrt(ecutrho) * np.linalg.norm(lattice[i]) / TWO_PI)) + 1
        n = nmin
        while not is_5smooth(n):
            n += 1
        out.append(n)
    return tuple(out)


def sphere_miller(lattice: np.ndarray, kpt: np.ndarray, ecutwfc: float) -> np.ndarray:
    """Miller indices of {G : |k+G|^2 <= ecutwfc}, lexicographic (h, k, l)."""
    b = reciprocal(lattice)
    kq = math.sqrt(ecutwfc) + float(np.linalg.norm(kpt))
    ms = [int(math.ceil(kq * np.linalg.norm(lattice[i]) / TWO_PI)) + 1 for i in range(3)]
    r = [np.arange(-m, m + 1) for m in ms]
    h, k, l = np.meshgrid(r[0], r[1], r[2], indexing="ij")
    m = np.stack([h.ravel(), k.ravel(), l.ravel()], axis=1)
    q = m @ b + kpt[None, :]
    q2 = np.einsum("ij,ij->i", q, q)
    sel = m[q2 <= ecutwfc]
    order = np.lexsort((sel[:, 2], sel[:, 1], sel[:, 0]))
    return np.ascontiguousarray(sel[order].astype(np.int32))


# --------------------------------------------------------------------------
# local potential


def _box_freqs(n: int) -> np.ndarray:
    return np.rint(np.fft.fftfreq(n) * n).astype(np.int64)


def vloc_fourier(lattice, fft, positions) -> np.ndarray:
    """Periodic sum of Gaussians evaluated through its Fourier series.

    V(r) = (1/Omega) sum_G vt(|G|) S(G) exp(i G.r) with
    vt(q) = A (2 pi w^2)^{3/2} exp(-q^2 w^2 / 2) and S(G) = sum_a exp(-i G.tau_a)
    (Poisson summation of the image sum).  The Gaussian is negligible beyond
    the box's G range, so sampling the series on the grid is exact to rounding.
    """
    n1, n2, n3 = fft
    b = reciprocal(lattice)
    omega = abs(np.linalg.det(lattice))
    f1, f2, f3 = _box_freqs(n1), _box_freqs(n2), _box_freqs(n3)
    m3, m2, m1 = np.meshgrid(f3, f2, f1, indexing="ij")
    g = (m1[..., None] * b[0] + m2[..., None] * b[1] + m3[..., None] * b[2])
    g2 = np.einsum("...i,...i->...", g, g)
    vt = VLOC_AMP * (TWO_PI * VLOC_WIDTH ** 2) ** 1.5 * np.exp(-0.5 * g2 * VLOC_WIDTH ** 2)
    # structure factor S(G) = sum_a exp(-i G.tau_a), G.tau = sum_i m_i (b_i.tau):
    # separable per axis, so S = sum_a e3[a,m3] e2[a,m2] e1[a,m1] (one contraction)
    pos = np.asarray(positions, dtype=np.float64)
    e1 = np.exp(-1j * np.outer(pos @ b[0], f1))     # (nat, n1)
    e2 = np.exp(-1j * np.outer(pos @ b[1], f2))
    e3 = np.exp(-1j * np.outer(pos @ b[2], f3))
    e21 = (e2[:, :, None] * e1[:, None, :]).reshape(pos.shape[0], -1)
    s = (e3.T @ e21).reshape(n3, n2, n1)
    c = vt * s / omega
    v = np.fft.ifftn(c) * (n1 * n2 * n3)
    return np.ascontiguousarray(v.real)


def vloc_image_sum(lattice, fft, positions, cutoff=IMAGE_CUTOFF) -> np.ndarray:
    """Direct real-space image sum of the same Gaussians (for small cells)."""
    n1, n2, n3 = fft
    j3, j2, j1 = np.meshgrid(np.arange(n3) / n3, np.arange(n2) / n2, np.arange(n1) / n1,
                             indexing="ij")
    frac = np.stack([j1, j2, j3], axis=-1)
    r = frac @ lattice
    v = np.zeros((n3, n2, n1))
    nr = [int(math.ceil(cutoff / np.linalg.norm(lattice[i]))) + 1 for i in range(3)]
    for tau in positions:
        for a in range(-nr[0], nr[0] + 1):
            for bb in range(-nr[1], nr[1] + 1):
                for c in range(-nr[2], nr[2] + 1):
                    shift = tau + a * lattice[0] + bb * lattice[1] + c * lattice[2]
                    d = r - shift
                    d2 = np.einsum("...i,...i->...", d, d)
                    mask = d2 <= cutoff * cutoff
                    v[mask] += VLOC_AMP * np.exp(-0.5 * d2[mask] / VLOC_WIDTH ** 2)
    return v


# --------------------------------------------------------------------------
# projectors


def radial_ft_closed(l: int, sigma: float, q: np.ndarray) -> np.ndarray:
    """F_l(q) = int_0^inf r^2 r^l exp(-r^2/sigma) j_l(q r) dr (closed form)."""
    return (math.sqrt(math.pi) * sigma ** (l + 1.5) / 2.0 ** (l + 2)) * q ** l \
        * np.exp(-sigma * q * q / 4.0)


def real_harmonics_poly(l: int, q: np.ndarray) -> np.ndarray:
    """q^l Y_lm(q_hat) for real harmonics, shape (2l+1, n)."""
    qx, qy, qz = q[:, 0], q[:, 1], q[:, 2]
    if l == 0:
        return np.full((1, q.shape[0]), 1.0 / math.sqrt(4 * math.pi))
    if l == 1:
        c = math.sqrt(3.0 / (4 * math.pi))
        return c * np.stack([qx, qy, qz])
    if l == 2:
        q2 = qx * qx + qy * qy + qz * qz
        c1 = math.sqrt(15.0 / (4 * math.pi))
        c2 = math.sqrt(5.0 / (16 * math.pi))
        c3 = math.sqrt(15.0 / (16 * math.pi))
        return np.stack([c1 * qx * qy, c1 * qy * qz, c1 * qz * qx,
                         c2 * (3 * qz * qz - q2), c3 * (qx * qx - qy * qy)])
    raise ValueError("l > 2 not supported")


def beta_matrix(lattice, kpt, miller, positions, proj_set: str) -> np.ndarray:
    """beta_i(k+G) for every projector i = (atom, channel, m); (nkb, npw) complex."""
    b = reciprocal(lattice)
    omega = abs(np.linalg.det(lattice))
    q = miller.astype(np.float64) @ b + kpt[None, :]
    qn = np.sqrt(np.einsum("ij,ij->i", q, q))
    chans = PROJ_SETS[proj_set]
    rows = []
    pref = 4.0 * math.pi / math.sqrt(omega)
    angular = {}
    radial = {}
    for (l, sig) in chans:
        if l not in angular:
            angular[l] = real_harmonics_poly(l, q)
        # F_l(q) / q^l: regular at q = 0
        radial[(l, sig)] = (math.sqrt(math.pi) * sig ** (l + 1.5) / 2.0 ** (l + 2)) \
            * np.exp(-sig * qn * qn / 4.0)
    nkb = len(positions) * sum(2 * l + 1 for l, _ in chans)
    out = np.empty((nkb, q.shape[0]), dtype=np.complex128)
    i = 0
    for tau in positions:
        phase = np.exp(-1j * (q @ tau))
        for (l, sig) in chans:
            base = pref * ((-1j) ** l) * radial[(l, sig)] * phase
            for m in range(2 * l + 1):
                out[i] = base * angular[l][m]
                i += 1
    del rows
    return out


def projgen_tables(cell, dq: float = 0.01) -> dict:
    """Pseudopotential data of the cell's projectors in tabulated form: one
    species, its radial channels (l, sigma) of ``PROJ_SETS[cell.proj_set]``,
    and for each channel the radial transform F(q) sampled at q = j dq, from 0
    to past sqrt(ecutwfc) (the largest |k+G| of the sphere) with three points
    to spare -- the form a pseudopotential file's radial functions take once
    transformed.  Returned as the dict the HIP binding takes as ``projgen``."""
    chans = PROJ_SETS[cell.proj_set]
    nq = int(math.ceil(math.sqrt(cell.ecutwfc) / dq)) + 4
    q = np.arange(nq) * dq
    tab = np.stack([radial_ft_closed(l, sig, q) for (l, sig) in chans])
    return dict(tau=np.ascontiguousarray(cell.positions, dtype=np.float64),
                ityp=np.zeros(cell.nat, dtype=np.int32),
                nchan=np.array([len(chans)], dtype=np.int32),
                lchan=np.array([l for (l, _) in chans], dtype=np.int32),
                dq=float(dq), tab=tab)


def gamma_half(cell: Cell) -> Cell:
    """The same k = 0 cell stored over half of the sphere, for real
    wavefunctions: the Miller list from (0,0,0) on (every G that follows
    (0,0,0) lexicographically; the others are their negatives), beta restricted
    to those columns, ``gamma=True``."""
    import dataclasses
    if np.any(np.asarray(cell.kpt) != 0.0):
        raise ValueError("gamma_half needs k = 0")
    i0 = int(np.flatnonzero((cell.miller == 0).all(axis=1))[0])
    beta = None if cell.beta is None else np.ascontiguousarray(cell.beta[:, i0:])
    return dataclasses.replace(cell, miller=np.ascontiguousarray(cell.miller[i0:]), beta=beta,
                               gamma=True)


def _dmat_blocks(nat: int, proj_set: str, dvals: np.ndarray) -> np.ndarray:
    """Diagonal D blocks: one value per (atom, channel) shared across m."""
    chans = PROJ_SETS[proj_set]
    blocks = []
    for a in range(nat):
        diag = []
        for c, (l, _) in enumerate(chans):
            diag += [dvals[a, c]] * (2 * l + 1)
        blocks.append(np.diag(np.array(diag, dtype=np.complex128)).ravel())
    return np.concatenate(blocks)


# --------------------------------------------------------------------------
# positions


def _fcc(n: int) -> np.ndarray:
    base = np.array([[0, 0, 0], [0, .5, .5], [.5, 0, .5], [.5, .5, 0]])
    cells = np.array([[i, j, k] for i in range(n) for j in range(n) for k in range(n)])
    return ((cells[:, None, :] + base[None, :, :]).reshape(-1, 3)) / n


def _diamond(n: int) -> np.ndarray:
    f = _fcc(n)
    return np.concatenate([f, f + 0.25 / n]) % 1.0


# --------------------------------------------------------------------------
# named configurations


def config_names():
    return ["c1", "c2", "c3", "c5"]


def _spec(name: str) -> dict:
    if name == "c1":
        a = 10.0
        return dict(lattice=np.diag([a, a, a]), fft=(30, 30, 30), kfrac=(0, 0, 0),
                    ecutwfc=20.0, ecutrho=80.0, frac=np.array([[0, 0, 0], [.5, .5, .5]]),
                    proj="sp", dfixed=True, nbnd=16, block=16)
    if name == "c2":
        a = 20.52
        return dict(lattice=np.diag([a, a, a]), fft=(72, 72, 72), kfrac=(.25, .25, .25),
                    ecutwfc=30.0, ecutrho=120.0, frac=_diamond(2), proj="2s2p",
                    dfixed=False, nbnd=128, block=128)
    if name == "c3":
        a = 32.6
        return dict(lattice=np.diag([a, a, a]), fft=(135, 135, 135), kfrac=(0, 0, 0),
                    ecutwfc=40.0, ecutrho=160.0, frac=_fcc(4), jitter=0.1, proj="2s2p",
                    dfixed=False, nbnd=512, block=64)
    if name == "c5":
        return dict(lattice=np.diag([40.0, 40.0, 42.0]), fft=(160, 160, 168), kfrac=(0, 0, 0),
                    ecutwfc=30.0, ecutrho=120.0, frac=_diamond(4), proj="s2pd",
                    dfixed=False, nbnd=1024, block=128)
    raise KeyError(name)


def make_cell(name: str, *, seed: int = 2104, with_beta: bool = True, **override) -> Cell:
    """Build a named cell.  ``override`` may replace any spec entry (e.g. fft,
    ecutwfc, nbnd, block, kfrac, lattice, frac, proj, vzero=True, nobeta=True,
    overlap=True for the q blocks of a non-identity overlap)."""
    spec = _spec(name) if name in ("c1", "c2", "c3", "c5") else {}
    spec.update(override)
    lattice = np.asarray(spec["lattice"], dtype=np.float64)
    rng = np.random.default_rng(seed)
    frac = np.asarray(spec["frac"], dtype=np.float64)
    pos = frac @ lattice
    if spec.get("jitter"):
        pos = pos + rng.normal(0.0, spec["jitter"], size=pos.shape)
    a0 = float(np.linalg.norm(lattice[0]))
    if "kpt" in spec:
        kpt = np.asarray(spec["kpt"], dtype=np.float64)
    else:
        kpt = np.asarray(spec.get("kfrac", (0, 0, 0)), dtype=np.float64) * (TWO_PI / a0)
    ecutrho = spec.get("ecutrho", 4.0 * spec["ecutwfc"])
    fft = tuple(spec["fft"]) if spec.get("fft") else fft_box_min(lattice, ecutrho)
    miller = sphere_miller(lattice, kpt, spec["ecutwfc"])
    proj = spec["proj"]
    nat = pos.shape[0]
    nchan = len(PROJ_SETS[proj])
    if spec.get("dfixed", True):
        dvals = np.tile(np.array([1.0, 0.5, 0.5, 0.25][:nchan]), (nat, 1))
    else:
        dvals = rng.uniform(0.2, 2.0, size=(nat, nchan))
    if spec.get("vzero"):
        vloc = np.zeros((fft[2], fft[1], fft[0]))
    elif "vloc" in spec:
        vloc = np.ascontiguousarray(spec["vloc"], dtype=np.float64)
    else:
        vloc = vloc_fourier(lattice, fft, pos)
    per_atom = sum(2 * l + 1 for l, _ in PROJ_SETS[proj])
    if spec.get("nobeta"):
        nproj = np.zeros(nat, dtype=np.int32)
        beta = np.zeros((0, miller.shape[0]), dtype=np.complex128)
        dmat = np.zeros(0, dtype=np.complex128)
    else:
        nproj = np.full(nat, per_atom, dtype=np.int32)
        beta = beta_matrix(lattice, kpt, miller, pos, proj) if with_beta else None
        dmat = _dmat_blocks(nat, proj, dvals)
    qmat = None
    if spec.get("overlap") and not spec.get("nobeta"):
        qvals = np.random.default_rng(seed + 1).uniform(0.05, 0.5, size=(nat, nchan))
        qmat = _dmat_blocks(nat, proj, qvals)
    return Cell(name=name, lattice=lattice, fft=fft, kpt=kpt,
                ecutwfc=float(spec["ecutwfc"]), ecutrho=float(ecutrho), positions=pos,
                miller=miller, vloc=vloc, nproj=nproj, beta=beta, dmat=dmat,
                nbnd=int(spec["nbnd"]), block=int(spec.get("block", spec["nbnd"])),
                proj_set=proj, meta=dict(seed=seed), qmat=qmat)


def make_psi0(npw: int, nb: int, seed: int = 10502) -> np.ndarray:
    """Starting bands: Re and Im iid N(0,1) from PCG64(seed), drawn band-major,
    each band scaled to unit 2-norm.  Shape (nb, npw) complex128."""
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((nb, npw, 2))
    psi = a[..., 0] + 1j * a[..., 1]
    psi /= np.linalg.norm(psi, axis=1, keepdims=True)
    return np.ascontiguousarray(psi)


# --------------------------------------------------------------------------
# served stream: random cubic cells


SERVE_KFRAC = [(.25, .25, .25), (.25, .25, -.25), (.25, -.25, .25), (-.25, .25, .25)]


def random_served_cell(nat: int, ecutwfc: float, kidx: int, seed: int,
                       with_beta: bool = True) -> Cell:
    """Random cubic cell at 8 atoms per 160 bohr^3, uniform random positions,
    the s+p Gaussian projector form, minimal 5-smooth box, nb = 2 nat
    (``with_beta=False`` skips building beta on the host)."""
    a = (20.0 * nat) ** (1.0 / 3.0)
    rng = np.random.default_rng(seed)
    frac = rng.uniform(0.0, 1.0, size=(nat, 3))
    cell = make_cell("serve", seed=seed, lattice=np.diag([a, a, a]), frac=frac,
                     kfrac=SERVE_KFRAC[kidx], ecutwfc=ecutwfc, ecutrho=4 * ecutwfc,
                     fft=None, proj="sp", dfixed=True, nbnd=2 * nat, block=2 * nat,
                     with_beta=with_beta)
    cell.name = f"serve_n{nat}_e{int(ecutwfc)}_k{kidx}"
    return cell


def served_trace(n_requests: int, rate: float = 20.0, seed: int = 2104,
                 nat_range=(8, 128), ecuts=(20.0, 25.0, 30.0), nk_range=(1, 4)):
    """Poisson arrival trace: list of dicts with t_arrive (s), nat, ecutwfc,
    nk and a per-request seed."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n_requests):
        t += rng.exponential(1.0 / rate)
        nat = int(rng.integers(nat_range[0], nat_range[1] + 1))
        ec = float(ecuts[int(rng.integers(0, len(ecuts)))])
        nk = int(rng.integers(nk_range[0], nk_range[1] + 1))
        out.append(dict(index=i, t_arrive=t, nat=nat, ecutwfc=ec, nk=nk,
                        seed=int(seed * 1000 + i)))
    return out
