"""Benchmark: H|psi> band-applies per second on one MI355X.

Headline workload: the 512-atom orthorhombic cell (40 x 40 x 42 bohr, diamond
sites, Gamma point, ecutwfc 30 Ry, 160 x 160 x 168 FFT box, 186 449 plane waves
on the full sphere, 93 225 stored on the Gamma half sphere, 6 144 s/p/d
projectors), 1 024 bands applied per step in launches of 128 on the Gamma
path (real wavefunctions: two bands per complex FFT, real projections).
Projectors are built on the device from radial tables; inputs are seeded
synthetic (Gaussian model pseudopotential), resident in HBM before timing.

A step = one full H|psi> (kinetic + local-potential FFT path + nonlocal
projectors) over all 1 024 bands; the timed steps run without
instrumentation.  ``value`` is the mixed form (FP32 FFTs and projector GEMMs,
FP64 psi / kinetic); the plain FP64 form is reported beside it.  Per-kernel
device times come from HIP events recorded on the context stream during a
second, equal set of steps; ``kernels`` prices each against the resource that
bounds it and ``roofline`` reports the dominant one.

Beside it: the same cell as a general complex k = 0 (full sphere), the 64-atom
cell (72^3 box, 128 bands, both forms, its charge density and projector
generation, and its k = 0 Gamma comparison), block-Davidson time to solution
on the 64-, 256- and 512-atom cells with eigenvalues held to the stored FP64
oracle values, a replay of the served request trace (``serve``), and
``cpu_baseline``: the FP64 oracle's H|psi> timed on a bounded band sample of
the headline cell on the host cores.

usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--serve SECONDS]
                      [--no-cpu] [--no-davidson] [--no-extras] [--no-cg]
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
MFMA_F32_TFLOPS = 157.3
MFMA_F64_TFLOPS = 78.6
# vector ALU: 256 CUs x 4 SIMDs x 16 lanes x FMA at 2.4 GHz = 78.6 TFLOP/s per
# instruction stream for FP32 and FP64 alike; the published FP32 figure
# (157.3) counts packed two-wide FP32, which every HIP source here is compiled
# without, so one-wide FP32 issue peaks at 78.6
VALU_F32_ONE_WIDE_TFLOPS = 78.6
VALU_F64_TFLOPS = 78.6
METRIC = "H|psi> band-applies/sec (FFT pts*bands/s) FP32 vs FP64; serve p50/p99 latency"
DENSITY_BSUB = 16   # bands per density subgroup (library constant)


def fft_flops(n):
    """Conventional flop count of a complex 1D transform of length n."""
    return 5.0 * n * np.log2(n)


def plane_flops(shape):
    """Flops of the pruned plane pass per transformed band and z plane: inverse
    and forward transforms of the N2 x rows and the x-extent y columns, and the
    real V(r) multiply (2 flops per point)."""
    n1, n2, ext = shape["n1"], shape["n2"], shape["ext"]
    return 2.0 * (n2 * fft_flops(n1) + ext * fft_flops(n2)) + 2.0 * n1 * n2


def transforms(shape, nb):
    """Complex 3D transforms per launch of nb bands (Gamma: one per band pair)."""
    return (nb + 1) // 2 if shape.get("gamma") else nb


def algorithmic(stage, shape, prec, nb):
    """Algorithmic amount of one launch of nb bands with the resource that
    bounds it: bytes for the stick passes, flops for the GEMMs.  The plane
    pass (k2_plane) is priced by its HBM bytes; its transform flops are
    reported beside them (plane_flops)."""
    npw, nst, nkb, n1, n2, n3 = (shape[k] for k in ("npw", "nst", "nkb", "n1", "n2", "n3"))
    c = 16 if prec == 0 else 8
    nfft = n1 * n2 * n3
    nt = transforms(shape, nb)
    gam = bool(shape.get("gamma"))
    npw_fft = 2 * npw - 1 if gam else npw
    if stage == "k1_scatter_zinv":
        # read psi (complex128) and the box map, write the sticks (+ the FP32
        # psi copy the single-precision beta^H psi reads, complex k only)
        if gam:
            return "hbm", nb * 16 * npw + nt * (4 * npw_fft + c * nst * n3)
        return "hbm", nb * (16 * npw + c * nst * n3 + 4 * npw + (8 * npw if prec else 0))
    if stage == "k2_plane":
        return "hbm", plane_bytes(shape, prec, nb)
    if stage == "k3_zfwd_gather":
        if gam:
            # K3 to the full-sphere pair buffer, then the unpack: read the buffer
            # at G and -G, psi, |G|^2; write H psi
            return "hbm", (nt * (c * nst * n3 + 4 * npw_fft + 2 * 16 * npw_fft) +
                           nb * 2 * 16 * npw + 8 * npw)
        return "hbm", nb * (c * nst * n3 + 16 * npw + 16 * npw + 4 * npw) + 8 * npw
    if stage in ("calbec_gemm", "addnl_gemm"):
        # complex: 8 flops per complex multiply-add; Gamma: real products over
        # the half sphere, 2 x (2 flops) per stored coefficient
        return "mfma", (4.0 if gam else 8.0) * nb * nkb * npw
    if stage == "dscale":
        return "hbm", nb * nkb * c * 2
    ext = shape["ext"]
    nsub = -(-nb // DENSITY_BSUB)
    if stage == "density_columns":   # read sticks, write inverse-y columns
        return "hbm", nb * c * (nst * n3 + ext * n2 * n3)
    if stage == "density_rows":      # read the columns, write the subgroup partial planes
        return "hbm", nb * c * ext * n2 * n3 + 8 * nsub * nfft
    if stage == "density_reduce":    # read the partial planes, write rho
        return "hbm", 8 * nsub * nfft + 8 * nfft
    raise KeyError(stage)


def plane_bytes(shape, prec, nb):
    """K2 algorithmic HBM bytes: read + write the sticks, V once per launch."""
    c = 16 if prec == 0 else 8
    return (transforms(shape, nb) * 2 * c * shape["nst"] * shape["n3"] +
            (c // 2) * shape["n1"] * shape["n2"] * shape["n3"])


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hpsi_c5_gamma_hbm_traffic.json")


# sources of the H|psi> kernels whose HBM counters are stored (the FFT
# passes, the projector GEMMs and D scaling, the Gamma unpack) and the headers
# they include
HPSI_SOURCES = ("cplx.h", "dav_kernels.hip", "fft_kernels.hip", "fft_reg.h", "gemm_kernels.hip",
                "qeh_internal.h")


def kernel_source_hash():
    """Hash of the H|psi> kernel sources; a stored counter measurement is used
    only while those kernels are unchanged."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2104_10502_amd", "csrc")
    for f in HPSI_SOURCES:
        h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:16]


def stored_traffic(kernel, prec, path=TRAFFIC_FILE):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE runs (scaled by the copy-kernel calibration), or None if absent
    or taken on other kernel sources."""
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    if rec.get("source_hash") != kernel_source_hash():
        return None
    k = rec.get("kernels", {}).get("%s/%s" % (kernel, "mixed" if prec else "fp64"))
    return None if k is None else k["bytes_per_launch"]


def time_projectors(q, torch, cell, reps=5):
    """Projectors of the benchmark cell built on the device from radial tables
    (wall time per qeh_beta_generate call, which includes its host-side
    validation and staging; the generator kernel's own time is in the kernel
    trace), and context set-up with host-built projectors (upload and host
    diag(H) sums) against device-built ones."""
    import cellgen
    pg = cellgen.projgen_tables(cell)
    out = {}
    for prec in (q.QEH_MIXED, q.QEH_FP64):
        name = "mixed" if prec else "fp64"
        b = q.generate_beta(cell.lattice, cell.kpt, cell.miller, cell.nproj, pg, precision=prec)
        del b
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            b = q.generate_beta(cell.lattice, cell.kpt, cell.miller, cell.nproj, pg,
                                precision=prec)
            del b
        torch.cuda.synchronize()
        gen_ms = (time.perf_counter() - t0) / reps * 1e3
        setup = {}
        for kind in ("host", "device"):
            t0 = time.perf_counter()
            ctx = q.Context.from_cell(cell, precision=prec, block=128,
                                      projgen=pg if kind == "device" else None)
            torch.cuda.synchronize()
            setup[kind] = (time.perf_counter() - t0) * 1e3
            ctx.close()
        out[name] = dict(generate_call_ms=gen_ms,
                         beta_bytes=cell.nkb * cell.npw * (8 if prec else 16),
                         ctx_create_ms_host_beta=setup["host"],
                         ctx_create_ms_device_beta=setup["device"])
    return out


def time_apply(q, torch, cell, prec, nb, steps, warmup, block=None, projgen=None):
    """Timed steps without instrumentation (the reported rate), then the same
    number of steps with per-stage HIP events (the kernel breakdown)."""
    import cellgen
    ctx = q.Context.from_cell(cell, precision=prec, block=block or nb, projgen=projgen)
    psi = torch.from_numpy(cellgen.make_psi0(cell.npw, nb, seed=10502)).cuda()
    if getattr(cell, "gamma", False):
        psi[:, 0].imag.zero_()   # real wavefunctions: psi(G = 0) real
    out = torch.empty_like(psi)
    for _ in range(warmup):
        ctx.apply_h(psi, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.apply_h(psi, out=out)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.profile(True)
    for _ in range(steps):
        ctx.apply_h(psi, out=out)
    stages = ctx.stage_times()
    ctx.profile(False)
    shape = ctx.info()
    shape["gamma"] = bool(getattr(cell, "gamma", False))
    ctx.close()
    del psi, out
    torch.cuda.empty_cache()
    return dt, stages, shape


def hpsi_leg(q, torch, cell, nb, steps, warmup, block=None, projgen=None, label=""):
    """Both precision forms of H|psi> on one cell: rate, per-kernel rooflines."""
    res = {}
    for prec in (q.QEH_MIXED, q.QEH_FP64):
        dt, stages, shape = time_apply(q, torch, cell, prec, nb, steps, warmup, block, projgen)
        blk = shape["block"]
        best, per = roofline_for(stages, shape, prec, blk)
        name = "mixed" if prec else "fp64"
        res[name] = dict(value=nb * steps / dt, unit="band-applies/s",
                         ms_per_step=dt / steps * 1e3,
                         fft_pts_bands_per_s=nb * steps / dt * cell.nfft,
                         dominant_kernel=best, kernels=per)
        print("# %s %s: %.3f ms/step, %.4g band-applies/s; kernels: %s" % (
            label, name, dt / steps * 1e3, nb * steps / dt,
            ", ".join("%s %.1f us (%.2f of %s peak)" % (k, v["avg_us"], v["frac"], v["bound"])
                      for k, v in per.items())), file=sys.stderr, flush=True)
    res["shape"] = shape
    return res


def time_gamma(q, torch, nb, steps, warmup):
    """The 64-atom cell moved to k = 0: H|psi> with complex wavefunctions over
    the full sphere against the Gamma-point path (real wavefunctions over half
    the sphere, two bands per complex FFT)."""
    import cellgen
    full = cellgen.make_cell("c2", kfrac=(0.0, 0.0, 0.0))
    half = cellgen.gamma_half(full)
    out = {}
    for prec in (q.QEH_MIXED, q.QEH_FP64):
        r = {}
        for kind, cell in (("complex", full), ("gamma", half)):
            dt, stages, _ = time_apply(q, torch, cell, prec, nb, steps, warmup)
            r[kind] = dict(band_applies_per_s=nb * steps / dt, ms_per_step=dt / steps * 1e3,
                           stage_us={k: v[0] / max(v[1], 1) * 1e3 for k, v in stages.items()
                                     if v[1]})
        r["speedup"] = r["gamma"]["band_applies_per_s"] / r["complex"]["band_applies_per_s"]
        out["mixed" if prec else "fp64"] = r
    out["npw_full"], out["npw_half"] = full.npw, half.npw
    return out


def golden_eigs(name):
    """Stored FP64 oracle eigenvalues of a named cell (tests/golden), or None."""
    path = os.path.join(ROOT, "tests", "golden", "%s_eigs.txt" % name)
    if not os.path.exists(path):
        return None
    return np.loadtxt(path)


def davidson_leg(q, torch, name, with_cg=True):
    """Block Davidson to converged eigenvalues on a named cell.  The 64-atom
    cell runs at its k-point (complex, 128 bands, basis up to 512 vectors); the
    256- and 512-atom Gamma cells run on the Gamma path with projectors built on
    the device (512 bands in launches of 64; 1024 in launches of 128).  Forms:
    mixed; FP64 to the mixed form's residual threshold (1e-5 Ry, equal
    accuracy); FP64 to 1e-8 Ry.  The mixed form runs single precision until
    its residuals stall, then H in FP64 until every FP64 residual is <= 1e-5 Ry.
    Eigenvalues are held to the stored FP64 oracle values (the lowest ones the
    oracle solved for)."""
    import cellgen
    if name == "c2":
        cell = cellgen.make_cell("c2")
        pg, nvecx = None, 4 * cell.nbnd
        full = cell
    else:
        full = cellgen.make_cell(name, with_beta=False)
        pg = cellgen.projgen_tables(full)
        cell, nvecx = cellgen.gamma_half(full), 0
    nb = full.nbnd
    psi0 = cellgen.make_psi0(cell.npw, nb, seed=10502)
    gold = golden_eigs(name)
    res = {}
    for label, prec, rtol in (("mixed", q.QEH_MIXED, 1e-8), ("fp64_1e-5", q.QEH_FP64, 1e-5),
                              ("fp64_1e-8", q.QEH_FP64, 1e-8)):
        ctx = q.Context.from_cell(cell, precision=prec, block=full.block, projgen=pg)
        # the mixed form finishes with H in FP64 through a context of the same
        # cell (built beside it: its set-up is outside the timed solve)
        c64 = q.Context.from_cell(cell, precision=q.QEH_FP64, block=full.block, projgen=pg) \
            if prec == q.QEH_MIXED else None
        p = torch.from_numpy(psi0).cuda()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        eig, info = ctx.davidson(p, nvecx=nvecx, rtol=rtol, allow_notconv=True, refine=c64)
        torch.cuda.synchronize()
        eig = np.sort(eig)
        r = dict(seconds=time.perf_counter() - t0, status=info["status"], iters=info["iters"],
                 refine_iters=info["refine_iters"],
                 band_applies=info["band_applies"], t_hpsi=info["t_hpsi"],
                 t_subspace=info["t_subspace"], resid_max=info["resid_max"],
                 eig_min=float(eig[0]), eig_max=float(eig[-1]))
        if gold is not None:
            m = min(len(gold), nb)
            r["max_err_vs_oracle_Ry"] = float(np.abs(eig[:m] - gold[:m]).max())
            r["oracle_bands_compared"] = m
        res[label] = r
        print("# davidson %s %s: %s" % (name, label, json.dumps(r)), file=sys.stderr, flush=True)
        ctx.close()
        if c64 is not None:
            c64.close()
        del p
        torch.cuda.empty_cache()
    res["npw_stored"], res["bands"], res["gamma"] = cell.npw, nb, name != "c2"
    basis = nvecx or 2 * nb
    res["subspace_solver"] = ("own HIP kernels (wide form), basis <= %d" % basis if basis <= 1024
                              else "rocSOLVER (basis <= %d > 1024)" % basis)
    if name == "c2" and with_cg:
        res["cg_fp64_1e-8"] = cg_leg(q, torch, cell, psi0, gold)
    return res


def cg_leg(q, torch, cell, psi0, gold):
    """The band-by-band conjugate-gradient solver on the same cell, start and
    residual threshold as Davidson's FP64 1e-8 Ry run (H applied one band at a
    time: the latency-bound comparison solver)."""
    ctx = q.Context.from_cell(cell, precision=q.QEH_FP64, block=cell.block)
    p = torch.from_numpy(psi0).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    eig, info = ctx.cg(p, rtol=1e-8, maxiter=400, allow_notconv=True)
    torch.cuda.synchronize()
    r = dict(seconds=time.perf_counter() - t0, status=info["status"], iters=info["iters"],
             notconv=info["notconv"], band_applies=info["band_applies"], t_hpsi=info["t_hpsi"],
             t_subspace=info["t_subspace"], resid_max=info["resid_max"])
    if gold is not None:
        m = min(len(gold), len(eig))
        r["max_err_vs_oracle_Ry"] = float(np.abs(np.sort(eig)[:m] - gold[:m]).max())
    print("# cg c2: %s" % json.dumps(r), file=sys.stderr, flush=True)
    ctx.close()
    del p
    torch.cuda.empty_cache()
    return r


def time_density(q, torch, cell, prec, nb, steps, warmup):
    """Charge density of nb bands (occupation 2 each): seconds for `steps`
    calls, per-stage device times, context shape."""
    ctx = q.Context.from_cell(cell, precision=prec, block=nb)
    psi = torch.from_numpy(__import__("cellgen").make_psi0(cell.npw, nb, seed=10502)).cuda()
    occ = np.full(nb, 2.0)
    info = ctx.info()
    rho = torch.empty((info["n3"], info["n2"], info["n1"]), dtype=torch.float64, device="cuda")
    work = torch.empty(ctx.density_plan(), dtype=torch.uint8, device="cuda")
    for _ in range(warmup):
        ctx.density(psi, occ, out=rho, work=work)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.density(psi, occ, out=rho, work=work)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.profile(True)
    for _ in range(steps):
        ctx.density(psi, occ, out=rho, work=work)
    stages = ctx.stage_times()
    ctx.profile(False)
    n = np.prod(cell.fft)
    integral = float(rho.sum()) * abs(np.linalg.det(cell.lattice)) / n
    ctx.close()
    return dt, stages, info, integral


def roofline_for(stages, shape, prec, nb):
    """Per-kernel achieved rate against its bound's peak; nb = bands per launch."""
    best = None
    per = {}
    for name, (ms, n) in stages.items():
        if n == 0:
            continue
        avg_s = ms / n * 1e-3
        bound, amount = algorithmic(name, shape, prec, nb)
        if bound == "hbm":
            achieved = amount / avg_s / 1e9
            peak, unit = HBM_PEAK_GBS, "GB/s"
        else:
            achieved = amount / avg_s / 1e12
            peak, unit = (MFMA_F64_TFLOPS if prec == 0 else MFMA_F32_TFLOPS), "TFLOP/s"
        per[name] = dict(avg_us=avg_s * 1e6, launches=n, bound=bound, achieved=achieved,
                         peak=peak, unit=unit, frac=achieved / peak, amount_per_launch=amount)
        if name == "k2_plane":
            # the plane pass also does the transform arithmetic: its flops against
            # the one-wide vector peak (packed FP32 is not emitted)
            tf = transforms(shape, nb) * shape["n3"] * plane_flops(shape) / avg_s / 1e12
            pk = VALU_F64_TFLOPS if prec == 0 else VALU_F32_ONE_WIDE_TFLOPS
            per[name].update(alu_TFLOPs=tf, alu_peak_one_wide=pk, alu_frac=tf / pk)
        if best is None or ms > stages[best][0]:
            best = name
    return best, per


def host_cpu():
    """Core counts and CPU model of the host (lscpu, else /proc/cpuinfo)."""
    import subprocess
    model = None
    try:
        r = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10)
        for ln in r.stdout.splitlines():
            if ln.startswith("Model name:"):
                model = ln.split(":", 1)[1].strip()
                break
    except (OSError, subprocess.SubprocessError):
        pass
    if model is None:
        try:
            for ln in open("/proc/cpuinfo"):
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
        except OSError:
            pass
    try:
        aff = len(os.sched_getaffinity(0))
    except AttributeError:
        aff = os.cpu_count()
    return dict(cpu_count=os.cpu_count(), affinity=aff, model=model)


def cpu_baseline(cell, budget_s=15.0):
    """The FP64 oracle's H|psi> on the full complex sphere of the headline cell,
    one band at a time, until budget_s has passed (at least one band)."""
    import oracle
    import cellgen
    hc = host_cpu()
    threads = int(os.environ.get("OMP_NUM_THREADS", hc["affinity"]))
    psi = cellgen.make_psi0(cell.npw, 8, seed=10502)
    done = 0
    t0 = time.perf_counter()
    while done < psi.shape[0]:
        oracle.apply_h(cell, psi[done:done + 1])
        done += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    return dict(value=done / dt, unit="band-applies/s", cores=min(hc["affinity"], threads),
                kind="oracle", cpu_model=hc["model"], cpu_count=hc["cpu_count"],
                affinity=hc["affinity"],
                sample="FP64 oracle apply_h (dense per-axis DFT, host-built projectors) on "
                       "%d band(s) of the 512-atom cell over its full complex sphere "
                       "(%d plane waves), %.1f s; projector construction untimed"
                       % (done, cell.npw, dt))


def _make_request(r, device_beta=True):
    """Cells and start vectors of one served request.  With device_beta the
    cells carry the projectors' radial tables and the library builds beta on
    the device; otherwise the host builds beta and the request carries it."""
    import dataclasses
    import cellgen
    cells = [cellgen.random_served_cell(r["nat"], r["ecutwfc"], k, r["seed"],
                                        with_beta=not device_beta) for k in range(r["nk"])]
    if device_beta:
        cells = [dataclasses.replace(c, projgen=cellgen.projgen_tables(c)) for c in cells]
    psis = [cellgen.make_psi0(c.npw, c.nbnd, seed=10502 + k) for k, c in enumerate(cells)]
    return cells, psis


def make_trace(duration, rate, seed=2104, device_beta=True):
    """Generate the served requests (host only; called before any GPU use, in a
    pool of spawned processes)."""
    import concurrent.futures as cf
    import functools
    import multiprocessing as mp
    import cellgen
    trace = [r for r in cellgen.served_trace(int(rate * duration * 2) + 10, rate=rate, seed=seed)
             if r["t_arrive"] <= duration]
    t_gen = time.perf_counter()
    # fork: this process has not touched the GPU yet, and a fork pool leaves no
    # resource-tracker process behind
    with cf.ProcessPoolExecutor(max_workers=min(16, os.cpu_count() or 4),
                                mp_context=mp.get_context("fork")) as ex:
        reqs = list(ex.map(functools.partial(_make_request, device_beta=device_beta), trace,
                           chunksize=4))
    return trace, reqs, time.perf_counter() - t_gen


def serve_bench(q, trace, reqs, t_gen, duration, rate, slots=8, arena_gib=96,
                device_beta=True):
    """Replay a Poisson trace of Davidson requests (random cubic cells, 8-128 atoms,
    ecutwfc in {20,25,30} Ry, 1-4 k-points, nb = 2 nat, mixed form) against the server."""
    srv = q.Server(int(arena_gib) << 30, max_slots=slots)
    # warm-up request (kernel loading, solver workspace queries), not measured
    w = _make_request(dict(nat=8, ecutwfc=20.0, nk=1, seed=1))
    tw = srv.submit(w[0], w[1], w[0][0].nbnd, precision=q.QEH_MIXED)
    while srv.poll(tw) is None:
        time.sleep(0.01)
    t0 = time.perf_counter()
    lag = 0.0
    tickets = []
    submit_s = []
    for r, (cells, psis) in zip(trace, reqs):
        delay = r["t_arrive"] - (time.perf_counter() - t0)
        if delay > 0:
            time.sleep(delay)
        else:
            lag = max(lag, -delay)
        ts = time.perf_counter()
        tickets.append(srv.submit(cells, psis, cells[0].nbnd, precision=q.QEH_MIXED))
        submit_s.append(time.perf_counter() - ts)
    res = {}
    t_note = time.perf_counter()
    while len(res) < len(tickets):
        for t in tickets:
            if t not in res:
                o = srv.poll(t)
                if o is not None:
                    res[t] = o
        if time.perf_counter() - t_note > 20.0:
            t_note = time.perf_counter()
            print("# serve: %d of %d requests done" % (len(res), len(tickets)), file=sys.stderr,
                  flush=True)
        time.sleep(0.005)
    st = srv.stats()
    srv.close()
    out = [res[t] for t in tickets]
    bad = sum(1 for o in out if o["status"] != 0)
    errors = sorted({"%d: %s" % (o["status"], o["error"]) for o in out if o["status"] != 0})
    lat = np.array([o["stamps"][3] - o["stamps"][0] for o in out])
    queue = np.array([o["stamps"][1] - o["stamps"][0] for o in out])
    arrive = min(o["stamps"][0] for o in out)
    finish = max(o["stamps"][3] for o in out)
    span = finish - arrive
    kpts = sum(len(o["eig"]) for o in out)
    run = sum(o["stamps"][3] - o["stamps"][2] for o in out)
    iters = [i["iters"] for o in out for i in o["info"]]
    return dict(requests=len(out), failed=bad, errors=errors[:5], rate_offered=rate,
                duration_s=duration,
                p50_latency_s=float(np.percentile(lat, 50)),
                p99_latency_s=float(np.percentile(lat, 99)),
                p50_queue_s=float(np.percentile(queue, 50)),
                solves_per_s=len(out) / span, kpoint_solves_per_s=kpts / span,
                mean_running_requests=run / span, peak_running_jobs=st["peak_running"],
                mean_davidson_iters=float(np.mean(iters)), max_davidson_iters=int(max(iters)),
                gpu_busy_fraction=st["busy_s"] / max(st["uptime_s"], 1e-9),
                max_submit_lag_s=lag, mean_submit_call_s=float(np.mean(submit_s)),
                max_submit_call_s=float(np.max(submit_s)), slots=slots, arena_gib=arena_gib,
                projectors="built on the device from radial tables" if device_beta
                else "built on the host, copied with the request",
                generation_s=t_gen)


def serve_child_main(a):
    """Served-trace leg (child process): trace on the host, wait for the
    parent's go, replay, print one JSON line."""
    served = make_trace(a.serve, a.serve_rate, device_beta=not a.serve_host_beta)
    print("# serve: trace of %d requests ready" % len(served[0]), file=sys.stderr, flush=True)
    print("ready", flush=True)
    if sys.stdin.readline().strip() != "go":
        return
    import paper_2104_10502_amd as q
    res = serve_bench(q, *served, duration=a.serve, rate=a.serve_rate, slots=a.serve_slots,
                      device_beta=not a.serve_host_beta)
    print(json.dumps(res), flush=True)


def run_serve_child(child, timeout_s=300.0):
    """Release the served-trace child and collect its result (or its failure)."""
    import subprocess
    try:
        out, _ = child.communicate("go\n", timeout=timeout_s)
    except subprocess.TimeoutExpired:
        child.kill()
        child.communicate()
        return {"error": "served-trace leg exceeded %.0f s" % timeout_s}
    lines = [ln for ln in (out or "").splitlines() if ln.startswith("{")]
    if child.returncode != 0 or not lines:
        return {"error": "served-trace leg ended with status %s" % child.returncode}
    return json.loads(lines[-1])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-davidson", action="store_true",
                    help="skip the Davidson time-to-solution legs")
    ap.add_argument("--davidson-cells", default="c2,c3,c5",
                    help="comma-separated cells of the Davidson legs (c2, c3, c5)")
    ap.add_argument("--no-cg", action="store_true",
                    help="skip the conjugate-gradient comparison beside the 64-atom Davidson leg")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the complex-k = 0 and 64-atom legs (density, projectors, Gamma)")
    ap.add_argument("--serve", type=float, default=5.0,
                    help="seconds of the served Poisson trace to replay (0 = skip)")
    ap.add_argument("--serve-rate", type=float, default=20.0)
    ap.add_argument("--serve-child", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--serve-slots", type=int, default=32)
    ap.add_argument("--serve-host-beta", action="store_true",
                    help="served requests carry host-built projectors instead of radial tables")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one plain 1 GiB device-to-device copy (the reference "
                         "kernel for scaling FETCH_SIZE / WRITE_SIZE counters)")
    a = ap.parse_args()
    if a.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % a.gpus, file=sys.stderr)
        sys.exit(2)
    if a.serve_child:
        serve_child_main(a)
        return
    # The served-trace leg runs in a child process, started here before this
    # process touches the GPU: it builds the trace on the host, then waits for
    # the parent's go (after the timed work) before it initialises its own
    # device context.  A failure there cannot take down this benchmark line.
    child = None
    if a.serve > 0:
        import subprocess
        env = dict(os.environ)
        # one hardware queue per job stream (up to 32 slots), so that jobs'
        # one-workgroup subspace solves run side by side instead of queueing
        # behind each other (HIP reads this at initialisation; its default is
        # 4, and values above 32 are not used here)
        env["GPU_MAX_HW_QUEUES"] = str(max(4, min(32, a.serve_slots)))
        child = subprocess.Popen(
            [sys.executable, os.path.abspath(__file__), "--serve-child", "--serve", str(a.serve),
             "--serve-rate", str(a.serve_rate), "--serve-slots", str(a.serve_slots)] +
            (["--serve-host-beta"] if a.serve_host_beta else []),
            stdin=subprocess.PIPE, stdout=subprocess.PIPE, env=env, text=True)
        # host-side trace generation uses all cores: let it finish before the
        # timed device work starts
        child.stdout.readline()
    import torch
    import cellgen
    import paper_2104_10502_amd as q

    # ---- headline: the 512-atom Gamma cell, 1024 bands in launches of 128
    c5full = cellgen.make_cell("c5", with_beta=False)
    pg5 = cellgen.projgen_tables(c5full)
    c5 = cellgen.gamma_half(c5full)
    nb = c5full.nbnd
    head = hpsi_leg(q, torch, c5, nb, a.steps, a.warmup, block=c5full.block, projgen=pg5,
                    label="512-atom Gamma")
    mixed, f64 = head["mixed"], head["fp64"]
    b = mixed["kernels"][mixed["dominant_kernel"]]
    shape = head["shape"]
    out = {
        "metric": METRIC,
        "value": mixed["value"],
        "unit": "band-applies/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": mixed["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (FFTs, V multiply, projector GEMMs) + f64 (psi, kinetic)",
        "data": "synthetic",
        "config": {"workload": "512-atom orthorhombic cell 40x40x42 bohr (diamond sites), "
                               "Gamma point on the real-wavefunction path, ecutwfc 30 Ry, "
                               "160x160x168 box, 6144 s/p/d projectors, 1024 bands per step "
                               "in launches of 128",
                   "bands_per_step": nb, "bands_per_launch": shape["block"],
                   "fft_points": c5full.nfft, "npw_full_sphere": c5full.npw,
                   "npw_stored": c5.npw, "nkb": c5full.nkb,
                   "projectors": "built on the device from radial tables"},
        "fft_pts_bands_per_s": mixed["fft_pts_bands_per_s"],
        "fp64_form": {k: f64[k] for k in ("value", "unit", "ms_per_step", "fft_pts_bands_per_s",
                                          "dominant_kernel", "kernels")},
        "mixed_over_fp64": mixed["value"] / f64["value"],
        "kernels": mixed["kernels"],
        "roofline": {"kernel": mixed["dominant_kernel"], "bound": b["bound"],
                     "achieved": b["achieved"], "peak": b["peak"], "unit": b["unit"],
                     "frac": b["frac"],
                     "traffic": stored_traffic(mixed["dominant_kernel"], q.QEH_MIXED)},
        "roofline_fft_path": {k: {kk: mixed["kernels"][k][kk] for kk in
                                  ("avg_us", "achieved", "peak", "unit", "frac")}
                              for k in ("k1_scatter_zinv", "k2_plane", "k3_zfwd_gather")
                              if k in mixed["kernels"]},
    }
    print("# headline: %s" % json.dumps({k: out[k] for k in ("value", "ms_per_step", "roofline")}),
          file=sys.stderr, flush=True)
    if not a.no_extras:
        # the same cell as a general complex k = 0 (full sphere), fewer steps
        ext = hpsi_leg(q, torch, c5full, nb, max(2, a.steps // 4), 1, block=c5full.block,
                       projgen=pg5, label="512-atom complex k=0")
        out["c5_complex_k0"] = {k: {kk: v[kk] for kk in ("value", "ms_per_step", "kernels")}
                                for k, v in ext.items() if k in ("mixed", "fp64")}
        out["c5_complex_k0"]["gamma_speedup_mixed"] = mixed["value"] / ext["mixed"]["value"]
        # the 64-atom cell at its k-point
        c2 = cellgen.make_cell("c2")
        r2 = hpsi_leg(q, torch, c2, 128, 20, 3, label="64-atom")
        out["c2"] = {k: {kk: v[kk] for kk in ("value", "ms_per_step", "fft_pts_bands_per_s",
                                                "kernels")}
                     for k, v in r2.items() if k in ("mixed", "fp64")}
        dens = {}
        for prec in (q.QEH_MIXED, q.QEH_FP64):
            dt, stages, shp, integral = time_density(q, torch, c2, prec, 128, 20, 3)
            _, per = roofline_for(stages, shp, prec, 128)
            dens["mixed" if prec else "fp64"] = dict(
                ms_per_call=dt / 20 * 1e3, band_densities_per_s=128 * 20 / dt,
                integral=integral, occupation_sum=2.0 * 128, kernels=per)
        out["c2"]["density"] = dens
        out["c2"]["gamma_point"] = time_gamma(q, torch, 128, 20, 3)
        out["c2"]["projectors"] = time_projectors(q, torch, c2)
        print("# 64-atom extras done", file=sys.stderr, flush=True)
    if not a.no_davidson:
        for name in [x for x in a.davidson_cells.split(",") if x in ("c2", "c3", "c5")]:
            out["davidson_%s" % name] = davidson_leg(q, torch, name, with_cg=not a.no_cg)
    if a.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if child is not None:
        out["serve"] = run_serve_child(child)
        print("# serve: %s" % json.dumps(out["serve"]), file=sys.stderr, flush=True)
    if not a.no_cpu:
        print("# cpu baseline: building the host projectors of the 512-atom cell",
              file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(cellgen.make_cell("c5"))
    print(json.dumps(out))


if __name__ == "__main__":
    main()
