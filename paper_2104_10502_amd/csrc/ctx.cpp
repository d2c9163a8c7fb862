// Context set-up and the H|psi> driver.
//
// Set-up (once per cell, untimed): validate the cell, build the z-stick table
// of the plane-wave sphere and the box positions (the "plane-wave generation
// and mapping to FFT grids" of the paper's Modules, section "Quantum-engine
// modules"), |k+G|^2 and diag(H), and copy V/N, beta and D into the caller's
// arena (the paper's device buffers are likewise preallocated and reused,
// section "Performance portability").
//
// apply_h: per band block, K1 -> K2 -> K3 (kinetic + local) then
// beta^H psi -> D scaling -> beta ps accumulated into hpsi, all on the
// context stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstdint>
#include <cstring>
#include <vector>

#include "qeh_internal.h"

namespace qeh {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

qeh_status hip_fail(hipError_t e, const char *what) {
  char buf[256];
  snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(e));
  set_error(buf);
  return QEH_ERR_DEVICE;
}

static qeh_status invalid(const std::string &m) {
  set_error(m);
  return QEH_ERR_INVALID;
}

FastDiv make_fastdiv(uint32_t d) {
  FastDiv f;
  f.d = d;
  f.s = 0;
  while ((1ull << f.s) < d) ++f.s;
  f.m = (uint32_t)(((1ull << 32) * ((1ull << f.s) - d)) / d + 1);
  return f;
}

bool make_fft_dim(int n, FftDim *d) {
  if (n < 1 || n > 1024) return false;
  int e[8] = {0};
  int r = n;
  const int primes[4] = {2, 3, 5, 7};
  for (int i = 0; i < 4; ++i)
    while (r % primes[i] == 0) {
      r /= primes[i];
      e[primes[i]]++;
    }
  if (r != 1) return false;
  std::vector<int> rad;
  int e2 = e[2];
  while (e2 >= 3) {
    if (e2 == 4) break;
    rad.push_back(8);
    e2 -= 3;
  }
  if (e2 == 4) {
    rad.push_back(4);
    rad.push_back(4);
  } else if (e2 == 2) {
    rad.push_back(4);
  } else if (e2 == 1) {
    rad.push_back(2);
  }
  for (int i = 0; i < e[3]; ++i) rad.push_back(3);
  for (int i = 0; i < e[5]; ++i) rad.push_back(5);
  for (int i = 0; i < e[7]; ++i) rad.push_back(7);
  if ((int)rad.size() > kMaxPass) return false;
  std::memset(d, 0, sizeof *d);
  d->n = n;
  d->npass = (int)rad.size();
  int span = 1;
  for (int p = 0; p < d->npass; ++p) {
    d->radix[p] = rad[p];
    d->span[p] = span;
    d->nbf_div[p] = make_fastdiv(n / rad[p]);
    d->span_div[p] = make_fastdiv(span);
    span *= rad[p];
  }
  return span == n;
}

int fft_digit_pos(const FftDim &d, int m) {
  int pos = 0, r = m;
  for (int p = d.npass - 1; p >= 0; --p) {
    const int q = r % d.radix[p];
    r /= d.radix[p];
    pos += q * d.span[p];
  }
  return pos;
}

namespace {

struct HostMaps {
  int nst = 0, hmin = 0, ext = 0;
  int npw_fft = 0;                  // G-vectors the FFT path places (the full sphere)
  std::vector<int> stick_off, stick_h, stick_k;
  std::vector<int> full;            // Gamma cells: the full sphere's Miller list
  const int *miller_fft = nullptr;  // Miller list of the FFT sphere (cell's or full)
};

inline int imod(int a, int n) {
  const int r = a % n;
  return r < 0 ? r + n : r;
}

qeh_status validate(const qeh_cell *c, HostMaps *hm) {
  if (!c) return invalid("cell is null");
  for (int i = 0; i < 3; ++i)
    if (c->fft[i] < 1 || c->fft[i] > 1024)
      return invalid("fft dimensions must be in [1, 1024]");
  FftDim t;
  for (int i = 0; i < 3; ++i)
    if (!make_fft_dim(c->fft[i], &t))
      return invalid("fft dimension " + std::to_string(c->fft[i]) +
                     " has a prime factor outside {2,3,5,7}");
  if (c->npw < 1 || !c->miller) return invalid("npw must be >= 1 with a Miller list");
  if (!c->vloc) return invalid("vloc is null");
  if (c->precision != QEH_FP64 && c->precision != QEH_MIXED)
    return invalid("precision must be QEH_FP64 or QEH_MIXED");
  if (c->block < 1) return invalid("block must be >= 1");
  if (c->nat < 0) return invalid("nat < 0");
  long nkb = 0, nd = 0;
  for (int a = 0; a < c->nat; ++a) {
    if (!c->nproj) return invalid("nproj is null");
    if (c->nproj[a] < 0 || c->nproj[a] > 256) return invalid("nproj per atom must be in [0,256]");
    nkb += c->nproj[a];
    nd += (long)c->nproj[a] * c->nproj[a];
  }
  if (nkb > 0 && !c->dmat) return invalid("dmat null with projectors");
  if (nkb > 0 && !c->beta && !c->projgen) return invalid("beta and projgen both null with projectors");
  for (int i = 0; i < 9; ++i)
    if (!std::isfinite(c->lattice[i])) return invalid("lattice not finite");
  for (int i = 0; i < 3; ++i)
    if (!std::isfinite(c->kpt[i])) return invalid("kpt not finite");
  if (c->gamma != 0 && c->gamma != 1) return invalid("gamma must be 0 or 1");
  // Gamma cells store the half sphere, (0,0,0) first; the FFT path places the
  // full sphere: the negated list reversed (all before (0,0,0)), then the half
  int npw_fft = c->npw;
  hm->full.clear();
  if (c->gamma) {
    if (c->kpt[0] != 0.0 || c->kpt[1] != 0.0 || c->kpt[2] != 0.0)
      return invalid("gamma cells need kpt = (0, 0, 0)");
    if (c->miller[0] != 0 || c->miller[1] != 0 || c->miller[2] != 0)
      return invalid("gamma cells list (0,0,0) first");
    npw_fft = 2 * c->npw - 1;
    hm->full.resize(3 * (size_t)npw_fft);
    for (int h = 1; h < c->npw; ++h)
      for (int i = 0; i < 3; ++i) hm->full[3 * (size_t)(c->npw - 1 - h) + i] = -c->miller[3 * h + i];
    for (int h = 0; h < c->npw; ++h)
      for (int i = 0; i < 3; ++i) hm->full[3 * (size_t)(c->npw - 1 + h) + i] = c->miller[3 * h + i];
  }
  hm->npw_fft = npw_fft;
  hm->miller_fft = c->gamma ? hm->full.data() : c->miller;
  // Miller list: lexicographic, sticks are contiguous runs, fits the box (for a
  // Gamma cell this also checks that the half list follows (0,0,0))
  const int *m = hm->miller_fft;
  int lo[3], hi[3];
  for (int i = 0; i < 3; ++i) lo[i] = hi[i] = m[i];
  hm->stick_off.clear();
  hm->stick_h.clear();
  hm->stick_k.clear();
  for (int g = 0; g < npw_fft; ++g) {
    const int *mg = m + 3 * g;
    for (int i = 0; i < 3; ++i) {
      lo[i] = std::min(lo[i], mg[i]);
      hi[i] = std::max(hi[i], mg[i]);
    }
    bool new_stick = g == 0;
    if (g > 0) {
      const int *mp = mg - 3;
      const bool inc = (mg[0] > mp[0]) || (mg[0] == mp[0] && mg[1] > mp[1]) ||
                       (mg[0] == mp[0] && mg[1] == mp[1] && mg[2] > mp[2]);
      if (!inc) return invalid("Miller list not strictly lexicographic at index " + std::to_string(g));
      new_stick = !(mg[0] == mp[0] && mg[1] == mp[1]);
      if (!new_stick && mg[2] != mp[2] + 1)
        return invalid("stick l values not contiguous at index " + std::to_string(g));
    }
    if (new_stick) {
      hm->stick_off.push_back(g);
      hm->stick_h.push_back(mg[0]);
      hm->stick_k.push_back(mg[1]);
    }
  }
  hm->stick_off.push_back(npw_fft);
  for (int i = 0; i < 3; ++i)
    if (hi[i] - lo[i] >= c->fft[i])
      return invalid("Miller index range exceeds the FFT box on axis " + std::to_string(i));
  hm->nst = (int)hm->stick_h.size();
  hm->hmin = lo[0];
  hm->ext = hi[0] - lo[0] + 1;
  // finiteness of the numeric inputs
  const long nfft = (long)c->fft[0] * c->fft[1] * c->fft[2];
  for (long i = 0; i < nfft; ++i)
    if (!std::isfinite(c->vloc[i])) {
      set_error("vloc has a non-finite value");
      return QEH_ERR_NUMERIC;
    }
  if (nkb > 0 && c->beta) {
    for (long i = 0; i < 2 * nkb * (long)c->npw; ++i)
      if (!std::isfinite(c->beta[i])) {
        set_error("beta has a non-finite value");
        return QEH_ERR_NUMERIC;
      }
  } else if (nkb > 0) {
    const qeh_status st = projgen_validate(c);
    if (st != QEH_OK) return st;
  }
  for (long i = 0; i < 2 * nd; ++i)
    if (!std::isfinite(c->dmat[i])) {
      set_error("dmat has a non-finite value");
      return QEH_ERR_NUMERIC;
    }
  if (c->qmat) {
    if (nkb == 0) return invalid("qmat given without projectors");
    for (long i = 0; i < 2 * nd; ++i)
      if (!std::isfinite(c->qmat[i])) {
        set_error("qmat has a non-finite value");
        return QEH_ERR_NUMERIC;
      }
    if (c->gamma)
      for (long i = 0; i < nd; ++i)
        if (c->qmat[2 * i + 1] != 0.0) return invalid("gamma cells need a real q");
  }
  if (c->gamma) {
    // real projectors: beta_i(G = 0) real, D real symmetric
    for (long i = 0; i < nd; ++i)
      if (c->dmat[2 * i + 1] != 0.0) return invalid("gamma cells need a real D");
    if (c->beta)
      for (long i = 0; i < nkb; ++i)
        if (c->beta[2 * i * (long)c->npw + 1] != 0.0)
          return invalid("gamma cells need beta_i(G = 0) real");
  }
  return QEH_OK;
}

// Arena layout, shared by plan and create.
struct Layout {
  size_t off_stick_off, off_gmap, off_tidx, off_tidx_dit, off_xin, off_kin, off_hdiag, off_vs,
      off_tw, off_beta, off_dmat, off_qmat, off_pj0, off_pnb, off_pdoff, off_chunk, off_sbuf, off_part,
      off_ps, off_big, off_colstart, off_psi32, off_pgen, off_gbuf;
  size_t total;
};

size_t bump(size_t *cur, size_t bytes) {
  const size_t o = *cur;
  *cur += (bytes + kAlign - 1) / kAlign * kAlign;
  return o;
}

struct Geometry {
  int nkb, nd, nchunk, nsplit, kchunk, plane_path, zpair, wide;
  FftDim dx, dy, dz;
  PlaneGeom pg;
  SplitGeom spg;
  StickGeom sg;
};

void geometry(const qeh_cell *c, const HostMaps &hm, Geometry *g) {
  g->nkb = 0;
  g->nd = 0;
  for (int a = 0; a < c->nat; ++a) {
    g->nkb += c->nproj[a];
    g->nd += c->nproj[a] * c->nproj[a];
  }
  make_fft_dim(c->fft[0], &g->dx);
  make_fft_dim(c->fft[1], &g->dy);
  make_fft_dim(c->fft[2], &g->dz);
  const int prec = c->precision;
  const size_t cs = prec == QEH_FP64 ? 16 : 8;
  const int n1 = c->fft[0], n2 = c->fft[1], n3 = c->fft[2];
  // sticks: z lines of odd stride; enough sticks per workgroup to fill ~48 KB
  g->sg.ldz = n3 | 1;
  int S = (int)(48 * 1024 / (cs * g->sg.ldz));
  S = std::max(1, std::min(64, S));
  g->sg.S = S;
  g->sg.lds_bytes = stick_lds_bytes(prec, n3, g->sg);
  g->sg.s_div = make_fastdiv(S);
  g->sg.slast_div = make_fastdiv(hm.nst % S ? hm.nst % S : S);
  // plane: x-extent columns of odd stride + a few full rows
  g->pg.ldT = n2 | 1;
  g->pg.ldR = n1 | 1;
  g->plane_path = 1;
  // rows per chunk: as many as fit in 80 KB (two workgroups per CU) keeping at
  // least min(N2, 16) rows, else as many as fit in the whole LDS
  const int rmin = std::min(n2, 16);
  for (int pass = 0; pass < 2 && g->plane_path; ++pass) {
    const size_t cap = pass == 0 ? (size_t)80 * 1024 : (size_t)kLdsMax;
    for (int rc = n2; rc >= (pass == 0 ? rmin : 1); --rc) {
      g->pg.rc = rc;
      g->pg.lds_bytes = plane_lds_bytes(prec, hm.ext, n1, n2, g->pg);
      if (g->pg.lds_bytes <= cap) {
        g->plane_path = 0;
        break;
      }
    }
  }
  // split path geometry (used when the column tile does not fit in LDS)
  {
    SplitGeom &q = g->spg;
    q.cg = std::min(16, hm.ext);
    q.rg = std::min(16, n2);
    q.ldl = q.rg | 1;
    q.lds_col = cs * ((size_t)q.cg * g->pg.ldT + n2);
    q.lds_row = cs * ((size_t)hm.ext * q.ldl + (size_t)q.rg * g->pg.ldR + n1) + 4 * (size_t)n1;
    q.cg_div = make_fastdiv(q.cg);
    q.cglast_div = make_fastdiv(hm.ext % q.cg ? hm.ext % q.cg : q.cg);
    q.rg_div = make_fastdiv(q.rg);
    q.rglast_div = make_fastdiv(n2 % q.rg ? n2 % q.rg : q.rg);
    // test hook: QEH_FORCE_SPLIT_PLANE=1 sends every plane through the split path
    const char *force = std::getenv("QEH_FORCE_SPLIT_PLANE");
    if (force && force[0] == '1') g->plane_path = 1;
    if (g->plane_path == 1) g->pg.rc = 1;   // unused by the split path
  }
  // tuning knob: QEH_PLANE_ROWS=n caps the rows per chunk of the fused plane
  // pass (fewer rows = less LDS per workgroup = more workgroups per CU)
  if (g->plane_path == 0) {
    const char *rows = std::getenv("QEH_PLANE_ROWS");
    const int cap = rows ? std::atoi(rows) : 0;
    if (cap > 0 && cap < g->pg.rc) {
      g->pg.rc = cap;
      g->pg.lds_bytes = plane_lds_bytes(prec, hm.ext, n1, n2, g->pg);
    }
  }
  // lane-pair kernel (N1 = N2 with a compiled form, single precision): pb bands
  // of one plane per workgroup, 2 by default (QEH_PAIR_PLANES=n overrides);
  // QEH_PLANE_KERNEL=generic keeps the fused kernel (comparison and test hook)
  g->pg.pb = 0;
  g->pg.lds_pair = 0;
  if (g->plane_path == 0 && pair_plane_supported(prec, n1, n2)) {
    const char *kern = std::getenv("QEH_PLANE_KERNEL");
    const bool generic = kern && std::strcmp(kern, "generic") == 0;
    const char *pbs = std::getenv("QEH_PAIR_PLANES");
    int pb = pbs ? std::atoi(pbs) : 2;
    pb = std::max(1, std::min(8, pb));
    while (pb > 1 && pair_plane_lds_bytes(prec, hm.ext, n2, pb) > (size_t)kLdsMax) --pb;
    if (!generic && pair_plane_lds_bytes(prec, hm.ext, n2, pb) <= (size_t)kLdsMax) {
      g->plane_path = 2;
      g->pg.pb = pb;
      g->pg.lds_pair = pair_plane_lds_bytes(prec, hm.ext, n2, pb);
    }
  }
  // lane-pair K1 / K3 (single precision, N3 with a compiled form);
  // QEH_STICK_KERNEL=generic keeps the LDS-pass kernels (test hook)
  g->zpair = 0;
  if (pair_z_supported(prec, n3) && pair_z_lds_bytes(n3) <= (size_t)kLdsMax) {
    const char *kern = std::getenv("QEH_STICK_KERNEL");
    if (!(kern && std::strcmp(kern, "generic") == 0)) g->zpair = 1;
  }
  // lane-quad kernel (N1 = N2 a compiled size: FP64 up to 72, single
  // precision above the lane-pair sizes): one band per workgroup by default
  // (QEH_PAIR_PLANES overrides); QEH_PLANE_KERNEL=generic keeps the fused
  // kernel
  if (g->plane_path == 0 && quad_plane_supported(prec, n1, n2)) {
    const char *kern = std::getenv("QEH_PLANE_KERNEL");
    const bool generic = kern && std::strcmp(kern, "generic") == 0;
    const char *pbs = std::getenv("QEH_PAIR_PLANES");
    int pb = pbs ? std::atoi(pbs) : 1;
    pb = std::max(1, std::min(8, pb));
    while (pb > 1 && quad_plane_lds_bytes(prec, hm.ext, n2, pb) > (size_t)kLdsMax) --pb;
    if (!generic && quad_plane_lds_bytes(prec, hm.ext, n2, pb) <= (size_t)kLdsMax) {
      g->plane_path = 4;
      g->pg.pb = pb;
      g->pg.lds_pair = quad_plane_lds_bytes(prec, hm.ext, n2, pb);
    }
  }
  g->pg.ext_div = make_fastdiv(hm.ext);
  g->pg.rc_div = make_fastdiv(g->pg.rc);
  g->pg.rlast_div = make_fastdiv(n2 % g->pg.rc ? n2 % g->pg.rc : g->pg.rc);
  // D-scaling chunks: whole atoms, <= 256 projectors each
  g->nchunk = 0;
  {
    int cur = 0;
    for (int a = 0; a < c->nat; ++a) {
      if (c->nproj[a] == 0) continue;
      if (cur == 0 || cur + c->nproj[a] > 256) {
        g->nchunk++;
        cur = 0;
      }
      cur += c->nproj[a];
    }
  }
  // split-K of beta^H psi: fixed chunks of >= 256 plane waves, enough
  // workgroups to fill the chip.  Single precision with >= 2048 projectors
  // and blocks of >= 128 bands takes the wide FP32 tiles (128 bands x 128
  // projectors, eight waves): at most two rounds of the workgroups resident
  // at once (256 CUs; one workgroup per CU, two for the Gamma product held to
  // 128 registers), since a third, nearly empty round costs as much as a full
  // one; otherwise 64 x 64 tiles (~4 workgroups per CU; measured faster than
  // 128 x 64 at 128 bands and 512 projectors).
  g->nsplit = 1;
  g->kchunk = c->npw;
  g->wide = c->precision == QEH_MIXED && c->block >= 128 && g->nkb >= 2048 ? 1 : 0;
  if (g->nkb > 0) {
    const int bm = g->wide ? 128 : 64;
    const int bn = g->wide ? 128 : 64;
    const int tiles = ((c->block + bm - 1) / bm) * ((g->nkb + bn - 1) / bn);
    const int resident = c->gamma ? 2 * 256 : 256;
    int ns = g->wide ? std::max(1, 2 * resident / tiles) : std::max(1, (1024 + tiles - 1) / tiles);
    ns = std::min(ns, std::max(1, c->npw / 256));
    int kc = (c->npw + ns - 1) / ns;
    kc = (kc + 15) / 16 * 16;
    g->kchunk = kc;
    g->nsplit = (c->npw + kc - 1) / kc;
  }
}

Layout layout(const qeh_cell *c, const HostMaps &hm, const Geometry &g) {
  Layout L;
  size_t cur = 0;
  const size_t cs = c->precision == QEH_FP64 ? 16 : 8;
  const size_t rs = c->precision == QEH_FP64 ? 8 : 4;
  const size_t nfft = (size_t)c->fft[0] * c->fft[1] * c->fft[2];
  L.off_stick_off = bump(&cur, 4 * (hm.nst + 1));
  L.off_gmap = bump(&cur, 4 * (size_t)hm.npw_fft);
  L.off_tidx = bump(&cur, 4 * (size_t)hm.nst);
  L.off_tidx_dit = bump(&cur, 4 * (size_t)hm.nst);
  L.off_xin = bump(&cur, 4 * (size_t)c->fft[0]);
  L.off_kin = bump(&cur, 8 * (size_t)c->npw);
  L.off_hdiag = bump(&cur, 8 * (size_t)c->npw);
  L.off_vs = bump(&cur, rs * nfft);
  L.off_tw = bump(&cur, cs * (size_t)(c->fft[0] + c->fft[1] + c->fft[2]));
  L.off_beta = bump(&cur, cs * (size_t)g.nkb * c->npw);
  L.off_dmat = bump(&cur, 16 * (size_t)g.nd);
  L.off_qmat = bump(&cur, c->qmat ? 16 * (size_t)g.nd : 0);
  L.off_pj0 = bump(&cur, 4 * (size_t)g.nkb);
  L.off_pnb = bump(&cur, 4 * (size_t)g.nkb);
  L.off_pdoff = bump(&cur, 4 * (size_t)g.nkb);
  L.off_chunk = bump(&cur, 4 * (size_t)(g.nchunk + 1));
  L.off_sbuf = bump(&cur, cs * (size_t)c->block * c->fft[2] * hm.nst);
  L.off_part = bump(&cur, cs * (size_t)g.nsplit * c->block * g.nkb);
  L.off_ps = bump(&cur, cs * (size_t)c->block * g.nkb);
  L.off_big = bump(&cur, g.plane_path == 1 ? cs * (size_t)c->block * c->fft[2] * hm.ext *
                                               c->fft[1]
                                         : 0);
  L.off_colstart = bump(&cur, 4 * (size_t)(hm.ext + 1));
  L.off_psi32 = bump(&cur, c->precision == QEH_MIXED ? 8 * (size_t)c->block * hm.npw_fft : 0);
  // projectors built on the device: the generator's staging area
  L.off_pgen = bump(&cur, g.nkb > 0 && !c->beta ? projgen_layout(c).total : 0);
  // Gamma: the full-sphere H of the band pairs (FP64), written by K3
  L.off_gbuf = bump(&cur, c->gamma ? 16 * (size_t)((c->block + 1) / 2) * hm.npw_fft : 0);
  L.total = cur;
  return L;
}

void reciprocal(const double *a, double *b) {
  // b rows: 2 pi (A^-1)^T, A rows a1 a2 a3
  const double det = a[0] * (a[4] * a[8] - a[5] * a[7]) - a[1] * (a[3] * a[8] - a[5] * a[6]) +
                     a[2] * (a[3] * a[7] - a[4] * a[6]);
  const double f = 2.0 * M_PI / det;
  // b1 = 2pi (a2 x a3) / det, etc.
  const double *a1 = a, *a2 = a + 3, *a3 = a + 6;
  auto cross = [](const double *u, const double *v, double *w) {
    w[0] = u[1] * v[2] - u[2] * v[1];
    w[1] = u[2] * v[0] - u[0] * v[2];
    w[2] = u[0] * v[1] - u[1] * v[0];
  };
  cross(a2, a3, b);
  cross(a3, a1, b + 3);
  cross(a1, a2, b + 6);
  for (int i = 0; i < 9; ++i) b[i] *= f;
}

}  // namespace
}  // namespace qeh

using namespace qeh;

extern "C" {

const char *qeh_status_str(qeh_status s) {
  switch (s) {
    case QEH_OK: return "ok";
    case QEH_ERR_INVALID: return "invalid argument";
    case QEH_ERR_NOMEM: return "arena or workspace too small";
    case QEH_ERR_NUMERIC: return "non-finite input";
    case QEH_ERR_CHOLESKY: return "overlap matrix not positive definite";
    case QEH_ERR_NOT_CONVERGED: return "not converged";
    case QEH_ERR_REJECTED: return "request rejected";
    case QEH_ERR_DEVICE: return "device error";
    case QEH_ERR_BUSY: return "busy";
    case QEH_RCI_APPLY_H: return "apply H to the request";
    default: return "unknown status";
  }
}

const char *qeh_last_error(void) { return g_last_error.c_str(); }

qeh_status qeh_ctx_plan(const qeh_cell *cell, size_t *arena_bytes) {
  if (!arena_bytes) return invalid("arena_bytes is null");
  HostMaps hm;
  qeh_status st = validate(cell, &hm);
  if (st != QEH_OK) return st;
  Geometry g;
  geometry(cell, hm, &g);
  if (g.plane_path != 0 && (g.spg.lds_col > (size_t)kLdsMax || g.spg.lds_row > (size_t)kLdsMax))
    return invalid("FFT plane too large for both plane paths");
  *arena_bytes = layout(cell, hm, g).total;
  return QEH_OK;
}

qeh_status qeh_ctx_create(const qeh_cell *cell, void *arena, size_t arena_bytes,
                          void *hip_stream, qeh_ctx **out) {
  if (!out) return invalid("out is null");
  *out = nullptr;
  HostMaps hm;
  qeh_status st = validate(cell, &hm);
  if (st != QEH_OK) return st;
  Geometry g;
  geometry(cell, hm, &g);
  if (g.plane_path != 0 && (g.spg.lds_col > (size_t)kLdsMax || g.spg.lds_row > (size_t)kLdsMax))
    return invalid("FFT plane too large for both plane paths");
  Layout L = layout(cell, hm, g);
  if (!arena) return invalid("arena is null");
  if (reinterpret_cast<uintptr_t>(arena) % kAlign) return invalid("arena not 256-byte aligned");
  if (arena_bytes < L.total) {
    set_error("arena has " + std::to_string(arena_bytes) + " bytes, plan needs " +
              std::to_string(L.total));
    return QEH_ERR_NOMEM;
  }
  qeh_ctx *c = new qeh_ctx();
  c->npw = cell->npw;
  c->npw_fft = hm.npw_fft;
  c->gamma = cell->gamma;
  c->nst = hm.nst;
  c->nkb = g.nkb;
  c->nat = cell->nat;
  c->n1 = cell->fft[0];
  c->n2 = cell->fft[1];
  c->n3 = cell->fft[2];
  c->ext = hm.ext;
  c->hmin = hm.hmin;
  c->block = cell->block;
  c->prec = cell->precision;
  c->plane_path = g.plane_path;
  c->zpair = g.zpair;
  c->nsplit = g.nsplit;
  c->wide = g.wide;
  c->kchunk = g.kchunk;
  c->nchunk = g.nchunk;
  c->dx = g.dx;
  c->dy = g.dy;
  c->dz = g.dz;
  c->pg = g.pg;
  c->spg = g.spg;
  c->sg = g.sg;
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  c->arena = reinterpret_cast<char *>(arena);
  c->arena_bytes = arena_bytes;
  char *A = c->arena;
  c->d.stick_off = reinterpret_cast<int *>(A + L.off_stick_off);
  c->d.gmap = reinterpret_cast<int *>(A + L.off_gmap);
  c->d.tidx = reinterpret_cast<int *>(A + L.off_tidx);
  c->d.tidx_dit = reinterpret_cast<int *>(A + L.off_tidx_dit);
  c->d.xin = reinterpret_cast<int *>(A + L.off_xin);
  c->d.kin = reinterpret_cast<double *>(A + L.off_kin);
  c->d.hdiag = reinterpret_cast<double *>(A + L.off_hdiag);
  c->d.vs = A + L.off_vs;
  c->d.tw = A + L.off_tw;
  c->d.beta = A + L.off_beta;
  c->d.dmat = reinterpret_cast<double2 *>(A + L.off_dmat);
  c->has_q = cell->qmat ? 1 : 0;
  c->d.qmat = cell->qmat ? reinterpret_cast<double2 *>(A + L.off_qmat) : nullptr;
  c->d.pj0 = reinterpret_cast<int *>(A + L.off_pj0);
  c->d.pnb = reinterpret_cast<int *>(A + L.off_pnb);
  c->d.pdoff = reinterpret_cast<int *>(A + L.off_pdoff);
  c->d.chunk = reinterpret_cast<int *>(A + L.off_chunk);
  c->d.sbuf = A + L.off_sbuf;
  c->d.part = A + L.off_part;
  c->d.ps = A + L.off_ps;
  c->d.big = g.plane_path == 1 ? A + L.off_big : nullptr;
  c->d.colstart = reinterpret_cast<int *>(A + L.off_colstart);
  c->d.psi32 = c->prec == QEH_MIXED ? reinterpret_cast<float2 *>(A + L.off_psi32) : nullptr;
  c->d.gbuf = c->gamma ? reinterpret_cast<double2 *>(A + L.off_gbuf) : nullptr;

  const int npw = cell->npw, n1 = c->n1, n2 = c->n2, n3 = c->n3;
  const size_t nfft = (size_t)n1 * n2 * n3;
  const bool f64 = c->prec == QEH_FP64;
  // ---- host-side maps
  std::vector<int> gmap(hm.npw_fft), tidx(hm.nst), tidx_dit(hm.nst), xin(n1, -1);
  const int *mf = hm.miller_fft;
  for (int s = 0; s < hm.nst; ++s) {
    for (int gg = hm.stick_off[s]; gg < hm.stick_off[s + 1]; ++gg)
      gmap[gg] = s * c->sg.ldz + (c->zpair ? imod(mf[3 * gg + 2], n3)
                                           : fft_digit_pos(c->dz, imod(mf[3 * gg + 2], n3)));
    const int ky = imod(hm.stick_k[s], n2);
    tidx_dit[s] = (hm.stick_h[s] - hm.hmin) * c->pg.ldT + fft_digit_pos(c->dy, ky);
    tidx[s] = (c->plane_path == 2 || c->plane_path == 4) ? (hm.stick_h[s] - hm.hmin) * c->pg.ldT + ky
                                                          : tidx_dit[s];
  }
  for (int cc = 0; cc < hm.ext; ++cc) xin[fft_digit_pos(c->dx, imod(hm.hmin + cc, n1))] = cc;
  std::vector<int> colstart(hm.ext + 1, hm.nst);
  for (int s2 = hm.nst - 1; s2 >= 0; --s2) colstart[hm.stick_h[s2] - hm.hmin] = s2;
  for (int cc = hm.ext - 1; cc >= 0; --cc) colstart[cc] = std::min(colstart[cc], colstart[cc + 1]);
  double b[9];
  reciprocal(cell->lattice, b);
  {
    const double *a = cell->lattice;
    c->omega = std::fabs(a[0] * (a[4] * a[8] - a[5] * a[7]) - a[1] * (a[3] * a[8] - a[5] * a[6]) +
                         a[2] * (a[3] * a[7] - a[4] * a[6]));
  }
  std::vector<double> kin(npw), hdiag(npw);
  double vsum = 0.0;
  for (size_t i = 0; i < nfft; ++i) vsum += cell->vloc[i];
  c->vmean = vsum / (double)nfft;
  for (int gg = 0; gg < npw; ++gg) {
    const int *m = cell->miller + 3 * gg;
    double q[3];
    for (int i = 0; i < 3; ++i)
      q[i] = cell->kpt[i] + m[0] * b[i] + m[1] * b[3 + i] + m[2] * b[6 + i];
    kin[gg] = q[0] * q[0] + q[1] * q[1] + q[2] * q[2];
    hdiag[gg] = kin[gg] + c->vmean;
  }
  std::vector<int> pj0(g.nkb), pnb(g.nkb), pdoff(g.nkb), chunk;
  {
    int i0 = 0, doff = 0, cur = 0;
    for (int a = 0; a < cell->nat; ++a) {
      const int n = cell->nproj[a];
      if (n == 0) continue;
      if (chunk.empty() || cur + n > 256) {
        chunk.push_back(i0);
        cur = 0;
      }
      cur += n;
      const double *D = cell->dmat + 2 * (size_t)doff;
      for (int i = 0; i < n; ++i) {
        pj0[i0 + i] = i0;
        pnb[i0 + i] = n;
        pdoff[i0 + i] = doff + i * n;
      }
      // nonlocal diagonal: sum_ij Re(beta_i D_ij conj(beta_j)) (on the device
      // when beta is built there)
      for (int gg = 0; gg < npw && cell->beta; ++gg) {
        double acc = 0.0;
        for (int i = 0; i < n; ++i) {
          const double *bi = cell->beta + 2 * ((size_t)(i0 + i) * npw + gg);
          for (int j = 0; j < n; ++j) {
            const double *bj = cell->beta + 2 * ((size_t)(i0 + j) * npw + gg);
            const double dr = D[2 * (i * n + j)], di = D[2 * (i * n + j) + 1];
            // beta_i * D_ij
            const double tr = bi[0] * dr - bi[1] * di, ti = bi[0] * di + bi[1] * dr;
            // * conj(beta_j), real part
            acc += tr * bj[0] + ti * bj[1];
          }
        }
        hdiag[gg] += acc;
      }
      i0 += n;
      doff += n * n;
    }
    chunk.push_back(i0);
  }
  // twiddles exp(-2 pi i t / n) for x, y, z
  const int ntw = n1 + n2 + n3;
  std::vector<double> tw64(2 * (size_t)ntw);
  c->tw_off[0] = 0;
  c->tw_off[1] = n1;
  c->tw_off[2] = n1 + n2;
  const int dims[3] = {n1, n2, n3};
  for (int d = 0; d < 3; ++d)
    for (int t = 0; t < dims[d]; ++t) {
      const double ang = 2.0 * M_PI * (double)t / (double)dims[d];
      tw64[2 * (c->tw_off[d] + t)] = std::cos(ang);
      tw64[2 * (c->tw_off[d] + t) + 1] = -std::sin(ang);
    }
  std::vector<double> vs64(nfft);
  for (size_t i = 0; i < nfft; ++i) vs64[i] = cell->vloc[i] / (double)nfft;

  // ---- uploads (synchronous on the stream before returning)
  hipStream_t s = c->stream;
  hipError_t e = hipSuccess;
  auto up = [&](void *dst, const void *src, size_t bytes) {
    if (e == hipSuccess && bytes) e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s);
  };
  up(c->d.stick_off, hm.stick_off.data(), 4 * hm.stick_off.size());
  up(c->d.gmap, gmap.data(), 4 * gmap.size());
  up(c->d.tidx, tidx.data(), 4 * tidx.size());
  up(c->d.tidx_dit, tidx_dit.data(), 4 * tidx_dit.size());
  up(c->d.xin, xin.data(), 4 * xin.size());
  up(c->d.colstart, colstart.data(), 4 * colstart.size());
  up(c->d.kin, kin.data(), 8 * kin.size());
  up(c->d.hdiag, hdiag.data(), 8 * hdiag.size());
  up(c->d.pj0, pj0.data(), 4 * pj0.size());
  up(c->d.pnb, pnb.data(), 4 * pnb.size());
  up(c->d.pdoff, pdoff.data(), 4 * pdoff.size());
  up(c->d.chunk, chunk.data(), 4 * chunk.size());
  up(c->d.dmat, cell->dmat, 16 * (size_t)g.nd);
  if (cell->qmat) up(c->d.qmat, cell->qmat, 16 * (size_t)g.nd);
  std::vector<float> f32;
  if (f64) {
    up(c->d.vs, vs64.data(), 8 * nfft);
    up(c->d.tw, tw64.data(), 16 * (size_t)ntw);
    if (cell->beta) up(c->d.beta, cell->beta, 16 * (size_t)g.nkb * npw);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
  } else {
    f32.resize(nfft);
    for (size_t i = 0; i < nfft; ++i) f32[i] = (float)vs64[i];
    up(c->d.vs, f32.data(), 4 * nfft);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    f32.resize(2 * (size_t)ntw);
    for (size_t i = 0; i < 2 * (size_t)ntw; ++i) f32[i] = (float)tw64[i];
    up(c->d.tw, f32.data(), 4 * f32.size());
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    // beta in slices of 16M complex to bound the host staging copy
    const size_t tot = cell->beta ? (size_t)g.nkb * npw : 0, sl = (size_t)1 << 24;
    for (size_t o = 0; o < tot && e == hipSuccess; o += sl) {
      const size_t nn = std::min(sl, tot - o);
      f32.resize(2 * nn);
      for (size_t i = 0; i < 2 * nn; ++i) f32[i] = (float)cell->beta[2 * o + i];
      up(reinterpret_cast<char *>(c->d.beta) + 8 * o, f32.data(), 8 * nn);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
    }
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    delete c;
    return hip_fail(e, "qeh_ctx_create upload");
  }
  if (g.nkb > 0 && !cell->beta) {
    // beta (context precision) and the nonlocal part of diag(H) on the device
    const qeh_status pst = projgen_run(cell, f64, c->d.beta, npw, A + L.off_pgen, s, c->d.dmat,
                                       c->d.hdiag);
    if (pst != QEH_OK) {
      delete c;
      return pst;
    }
  }
  *out = c;
  return QEH_OK;
}

qeh_status qeh_ctx_destroy(qeh_ctx *c) {
  if (!c) return QEH_OK;
  for (auto &ev : c->ev_pool) (void)hipEventDestroy(ev);
  delete c;
  return QEH_OK;
}

}  // extern "C"

namespace qeh {

// Stage timing: each recorded stage takes two events from a pool; totals are
// read back (after a stream sync) by qeh_ctx_stage_times.
struct StageGuard {
  qeh_ctx *c;
  int stage;
  int idx = -1;
  StageGuard(qeh_ctx *cc, int st) : c(cc), stage(st) {
    if (!c->prof) return;
    idx = (int)c->ev_recs.size();
    const size_t need = 2 * (size_t)(idx + 1);
    while (c->ev_pool.size() < need) {
      hipEvent_t ev;
      if (hipEventCreate(&ev) != hipSuccess) {
        idx = -1;
        return;
      }
      c->ev_pool.push_back(ev);
    }
    c->ev_recs.push_back(stage);
    (void)hipEventRecord(c->ev_pool[2 * idx], c->stream);
  }
  ~StageGuard() {
    if (idx >= 0) (void)hipEventRecord(c->ev_pool[2 * idx + 1], c->stream);
  }
};

qeh_status apply_block(qeh_ctx *c, int part, int nbk, const double2 *psi, int ldpsi,
                       double2 *hpsi, int ldh) {
  hipError_t e;
  const bool f64 = c->prec == QEH_FP64;
  if ((part == 0 || part == 2) && c->gamma) {
    // Gamma: bands 2p, 2p+1 go through one complex FFT as psi_2p + i psi_2p+1
    // over the full sphere (K1 reads the pairs from the stored halves; K3
    // writes the full-sphere result to gbuf), and are separated again with the
    // kinetic term added
    const int np = (nbk + 1) / 2;
    {
      StageGuard g(c, 0);
      e = launch_k1_gamma(c, nbk, psi, ldpsi, nullptr, 0, /*copy32=*/true);
    }
    if (e != hipSuccess) return hip_fail(e, "K1 launch");
    {
      StageGuard g(c, 1);
      e = launch_k2(c, np);
    }
    if (e != hipSuccess) return hip_fail(e, "K2 launch");
    {
      StageGuard g(c, 2);
      e = launch_k3(c, np, c->d.gbuf, c->npw_fft, c->d.gbuf, c->npw_fft, 0);
      if (e == hipSuccess)
        e = launch_gamma_unpack(c->d.gbuf, c->npw_fft, nbk, c->npw, psi, ldpsi, c->d.kin, hpsi,
                                ldh, c->stream);
    }
    if (e != hipSuccess) return hip_fail(e, "K3 launch");
  } else if (part == 0 || part == 2) {
    {
      StageGuard g(c, 0);
      e = launch_k1(c, nbk, psi, ldpsi);
    }
    if (e != hipSuccess) return hip_fail(e, "K1 launch");
    {
      StageGuard g(c, 1);
      e = launch_k2(c, nbk);
    }
    if (e != hipSuccess) return hip_fail(e, "K2 launch");
    {
      StageGuard g(c, 2);
      e = launch_k3(c, nbk, psi, ldpsi, hpsi, ldh, 1);
    }
    if (e != hipSuccess) return hip_fail(e, "K3 launch");
  }
  if ((part == 1 || part == 2) && c->nkb > 0) {
    GemmDesc g1{};
    // K1 has just written psi32 (the single-precision copy of the block)
    const bool use32 = !f64 && part == 2;
    g1.A = use32 ? static_cast<const void *>(c->d.psi32) : static_cast<const void *>(psi);
    g1.lda = use32 ? c->npw_fft : ldpsi;
    g1.ta = use32 ? T_F2 : T_D2;
    g1.tile = c->wide;
    g1.B = c->d.beta;
    g1.ldb = c->npw;
    g1.tb = f64 ? T_D2 : T_F2;
    g1.bmode = 0;
    g1.C = c->d.part;
    g1.ldc = c->nkb;
    g1.tc = f64 ? T_D2 : T_F2;
    g1.M = nbk;
    g1.N = c->nkb;
    g1.K = c->npw;
    g1.conjB = 1;
    g1.nsplit = c->nsplit;
    g1.kchunk = c->kchunk;
    g1.split_stride = (long)c->block * c->nkb;
    g1.prec = f64 ? G_F64 : G_F32;
    g1.rmode = c->gamma ? 1 : 0;   // Gamma: only the real part enters becp
    {
      StageGuard g(c, 3);
      e = launch_cgemm(g1, c->stream);
    }
    if (e != hipSuccess) return hip_fail(e, "beta^H psi launch");
    {
      StageGuard g(c, 4);
      e = launch_dscale(c, nbk, psi, ldpsi);
    }
    if (e != hipSuccess) return hip_fail(e, "D scaling launch");
    GemmDesc g3{};
    g3.A = c->d.ps;
    g3.lda = c->nkb;
    g3.ta = f64 ? T_D2 : c->gamma ? T_F1 : T_F2;   // single-precision Gamma: real ps
    g3.B = c->d.beta;
    g3.ldb = c->npw;
    g3.tb = f64 ? T_D2 : T_F2;
    g3.bmode = 1;
    g3.C = hpsi;
    g3.ldc = ldh;
    g3.tc = T_D2;
    g3.M = nbk;
    g3.N = c->npw;
    g3.K = c->nkb;
    g3.accumulate = part == 2 ? 1 : 0;
    g3.nsplit = 1;
    g3.kchunk = c->nkb;
    g3.prec = f64 ? G_F64 : G_F32;
    g3.rmode = c->gamma ? 2 : 0;   // Gamma: ps is real
    g3.tile = c->wide;
    {
      StageGuard g(c, 5);
      e = launch_cgemm(g3, c->stream);
    }
    if (e != hipSuccess) return hip_fail(e, "beta ps launch");
  } else if (part == 1) {
    // no projectors: the nonlocal part is zero
    for (int b = 0; b < nbk; ++b) {
      e = hipMemsetAsync(hpsi + (size_t)b * ldh, 0, 16 * (size_t)c->npw, c->stream);
      if (e != hipSuccess) return hip_fail(e, "memset");
    }
  }
  return QEH_OK;
}

qeh_status apply_h_impl(qeh_ctx *c, int part, int nb, const double *psi, int ldpsi,
                        double *hpsi, int ldh) {
  if (!c) return invalid("ctx is null");
  if (nb < 0) return invalid("nb < 0");
  if (nb == 0) return QEH_OK;
  if (!psi || !hpsi) return invalid("psi / hpsi null");
  if (ldpsi < c->npw || ldh < c->npw) return invalid("leading dimension < npw");
  if (psi == hpsi) return invalid("psi and hpsi must not overlap");
  const double2 *p = reinterpret_cast<const double2 *>(psi);
  double2 *h = reinterpret_cast<double2 *>(hpsi);
  for (int b0 = 0; b0 < nb; b0 += c->block) {
    const int nbk = std::min(c->block, nb - b0);
    qeh_status st = apply_block(c, part, nbk, p + (size_t)b0 * ldpsi, ldpsi,
                                h + (size_t)b0 * ldh, ldh);
    if (st != QEH_OK) return st;
  }
  return QEH_OK;
}

// S psi = psi + beta q beta^H psi, per block of the context's block size:
// copy psi, beta^H psi (split-K), q scaling (the D-scaling kernel with the q
// blocks), beta qs accumulated onto the copy.
qeh_status apply_s_impl(qeh_ctx *c, int nb, const double *psi, int ldpsi, double *spsi,
                        int ldsp) {
  if (!c) return invalid("ctx is null");
  if (nb < 0) return invalid("nb < 0");
  if (nb == 0) return QEH_OK;
  if (!psi || !spsi) return invalid("psi / spsi null");
  if (ldpsi < c->npw || ldsp < c->npw) return invalid("leading dimension < npw");
  if (psi == spsi) return invalid("psi and spsi must not overlap");
  const double2 *p = reinterpret_cast<const double2 *>(psi);
  double2 *o = reinterpret_cast<double2 *>(spsi);
  hipError_t e = launch_copy_rows(p, ldpsi, o, ldsp, c->npw, nb, c->stream);
  if (e != hipSuccess) return hip_fail(e, "S psi copy");
  if (!c->has_q || c->nkb == 0) return QEH_OK;
  const bool f64 = c->prec == QEH_FP64;
  for (int b0 = 0; b0 < nb; b0 += c->block) {
    const int nbk = std::min(c->block, nb - b0);
    const double2 *pb = p + (size_t)b0 * ldpsi;
    GemmDesc g1{};
    g1.A = pb;
    g1.lda = ldpsi;
    g1.ta = T_D2;
    g1.B = c->d.beta;
    g1.ldb = c->npw;
    g1.tb = f64 ? T_D2 : T_F2;
    g1.bmode = 0;
    g1.C = c->d.part;
    g1.ldc = c->nkb;
    g1.tc = f64 ? T_D2 : T_F2;
    g1.M = nbk;
    g1.N = c->nkb;
    g1.K = c->npw;
    g1.conjB = 1;
    g1.nsplit = c->nsplit;
    g1.kchunk = c->kchunk;
    g1.split_stride = (long)c->block * c->nkb;
    g1.prec = f64 ? G_F64 : G_F32;
    g1.rmode = c->gamma ? 1 : 0;
    g1.tile = c->wide;
    e = launch_cgemm(g1, c->stream);
    if (e == hipSuccess) e = launch_dscale(c, nbk, pb, ldpsi, c->d.qmat);
    if (e != hipSuccess) return hip_fail(e, "S psi projections");
    GemmDesc g3{};
    g3.A = c->d.ps;
    g3.lda = c->nkb;
    g3.ta = f64 ? T_D2 : c->gamma ? T_F1 : T_F2;   // single-precision Gamma: real ps
    g3.B = c->d.beta;
    g3.ldb = c->npw;
    g3.tb = f64 ? T_D2 : T_F2;
    g3.bmode = 1;
    g3.C = o + (size_t)b0 * ldsp;
    g3.ldc = ldsp;
    g3.tc = T_D2;
    g3.M = nbk;
    g3.N = c->npw;
    g3.K = c->nkb;
    g3.accumulate = 1;
    g3.nsplit = 1;
    g3.kchunk = c->nkb;
    g3.prec = f64 ? G_F64 : G_F32;
    g3.rmode = c->gamma ? 2 : 0;
    g3.tile = c->wide;
    e = launch_cgemm(g3, c->stream);
    if (e != hipSuccess) return hip_fail(e, "S psi product");
  }
  return QEH_OK;
}

// ---- charge density (charge density generation among the ported kernels,
// section "Evolution of the GPU-enabled version")
struct DensityWork {
  size_t big, partial, occ, zcol, pairs, total;
};

DensityWork density_work(const qeh_ctx *c, const DensityGeom &dg) {
  DensityWork w{};
  size_t cur = 0;
  const size_t cs = c->prec == QEH_FP64 ? 16 : 8;
  const size_t nfft = (size_t)c->n1 * c->n2 * c->n3;
  const int nsub = (c->block + dg.bsub - 1) / dg.bsub;
  w.big = bump(&cur, dg.fused ? 0 : cs * (size_t)c->block * c->n3 * c->ext * c->n2);
  w.partial = bump(&cur, 8 * (size_t)nsub * nfft);
  w.occ = bump(&cur, 8 * (size_t)c->block);
  w.zcol = bump(&cur, 8 * (size_t)c->n2);
  w.pairs = bump(&cur, c->gamma ? 8 * (size_t)c->block : 0);
  w.total = cur;
  return w;
}

qeh_status density_impl(qeh_ctx *c, int nb, const double *psi, int ldpsi, const double *occ,
                        double *rho, void *work, size_t work_bytes) {
  if (!c) return invalid("ctx is null");
  if (nb < 0) return invalid("nb < 0");
  if (!rho) return invalid("rho is null");
  if (nb > 0 && (!psi || !occ)) return invalid("psi / occ null");
  if (ldpsi < c->npw) return invalid("leading dimension < npw");
  DensityGeom dg{};
  if (!density_geometry(c, &dg)) return invalid("box too large for the density row kernel");
  const DensityWork w = density_work(c, dg);
  if (!work || work_bytes < w.total) return invalid("density work buffer too small");
  if ((reinterpret_cast<uintptr_t>(work) % kAlign) != 0)
    return invalid("density work buffer not 256-byte aligned");
  for (int b = 0; b < nb; ++b)
    if (!std::isfinite(occ[b])) return invalid("non-finite occupation");
  char *W = static_cast<char *>(work);
  double *occ_d = reinterpret_cast<double *>(W + w.occ);
  double *partial = reinterpret_cast<double *>(W + w.partial);
  const long npts = (long)c->n1 * c->n2 * c->n3;
  const double scale = 1.0 / c->omega;
  hipError_t e;
  if (nb == 0) {
    // no bands: rho = 0 (a kernel, not a memset)
    e = launch_density_reduce(partial, 0, npts, scale, rho, 0, c->stream);
    return e == hipSuccess ? QEH_OK : hip_fail(e, "density reduce launch");
  }
  const double2 *p = reinterpret_cast<const double2 *>(psi);
  // the zero column of the lane-pair rows (a kernel, not a memset)
  e = launch_fill_int(reinterpret_cast<int *>(W + w.zcol), 2 * c->n2, 0, c->stream);
  if (e != hipSuccess) return hip_fail(e, "density zero column");
  // Gamma: consecutive bands of equal occupation share one complex transform,
  // psi_a + i psi_b, whose |.|^2 is psi_a^2 + psi_b^2 (both real in real
  // space); a band without such a partner goes alone.  Each transform is one
  // "slot" with its occupation; without Gamma a slot is a band.
  std::vector<int2> slot_pair;
  std::vector<double> slot_occ;
  if (c->gamma) {
    for (int b = 0; b < nb;) {
      if (b + 1 < nb && occ[b] == occ[b + 1]) {
        slot_pair.push_back(make_int2(b, b + 1));
        b += 2;
      } else {
        slot_pair.push_back(make_int2(b, -1));
        b += 1;
      }
      slot_occ.push_back(occ[slot_pair.back().x]);
    }
  }
  const int nslots = c->gamma ? (int)slot_pair.size() : nb;
  const double *socc = c->gamma ? slot_occ.data() : occ;
  int2 *pairs_d = reinterpret_cast<int2 *>(W + w.pairs);
  for (int b0 = 0; b0 < nslots; b0 += c->block) {
    const int nbk = std::min(c->block, nslots - b0);
    // the previous block's kernels read occ_d (and the pair table); the copies
    // below are ordered after them on the same stream
    e = hipMemcpyAsync(occ_d, socc + b0, 8 * (size_t)nbk, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess && c->gamma)
      e = hipMemcpyAsync(pairs_d, slot_pair.data() + b0, 8 * (size_t)nbk, hipMemcpyHostToDevice,
                         c->stream);
    if (e != hipSuccess) return hip_fail(e, "occupation upload");
    {
      StageGuard g(c, 0);
      e = c->gamma ? launch_k1_gamma(c, nb, p, ldpsi, pairs_d, nbk)
                   : launch_k1(c, nbk, p + (size_t)b0 * ldpsi, ldpsi);
    }
    if (e != hipSuccess) return hip_fail(e, "K1 launch");
    if (dg.fused) {
      StageGuard g(c, 7);
      e = launch_density_plane(c, dg, nbk, occ_d, partial);
    } else {
      {
        StageGuard g(c, 6);
        e = launch_density_columns(c, nbk, W + w.big);
      }
      if (e != hipSuccess) return hip_fail(e, "density columns launch");
      StageGuard g(c, 7);
      e = launch_density_rows(c, dg, nbk, W + w.big, occ_d, partial, W + w.zcol);
    }
    if (e != hipSuccess) return hip_fail(e, "density rows launch");
    const int nsub = (nbk + dg.bsub - 1) / dg.bsub;
    {
      StageGuard g(c, 8);
      e = launch_density_reduce(partial, nsub, npts, scale, rho, b0 > 0 ? 1 : 0, c->stream);
    }
    if (e != hipSuccess) return hip_fail(e, "density reduce launch");
  }
  // occ is a caller's host array: the copies above must be complete on return
  e = hipStreamSynchronize(c->stream);
  return e == hipSuccess ? QEH_OK : hip_fail(e, "density sync");
}

}  // namespace qeh

extern "C" {

qeh_status qeh_apply_h(qeh_ctx *c, int nb, const double *psi, int ldpsi, double *hpsi,
                       int ldh) {
  return apply_h_impl(c, 2, nb, psi, ldpsi, hpsi, ldh);
}

qeh_status qeh_apply_s(qeh_ctx *c, int nb, const double *psi, int ldpsi, double *spsi,
                       int ldsp) {
  return apply_s_impl(c, nb, psi, ldpsi, spsi, ldsp);
}

qeh_status qeh_apply_h_part(qeh_ctx *c, int part, int nb, const double *psi, int ldpsi,
                            double *hpsi, int ldh) {
  if (part != 0 && part != 1) return invalid("part must be 0 (kinetic+local) or 1 (nonlocal)");
  return apply_h_impl(c, part, nb, psi, ldpsi, hpsi, ldh);
}

qeh_status qeh_density_plan(const qeh_ctx *c, size_t *work_bytes) {
  if (!c || !work_bytes) return invalid("null argument");
  DensityGeom dg{};
  if (!density_geometry(c, &dg)) return invalid("box too large for the density row kernel");
  *work_bytes = density_work(c, dg).total;
  return QEH_OK;
}

qeh_status qeh_density(qeh_ctx *c, int nb, const double *psi, int ldpsi, const double *occ,
                       double *rho, void *work, size_t work_bytes) {
  return density_impl(c, nb, psi, ldpsi, occ, rho, work, work_bytes);
}

qeh_status qeh_ctx_profile(qeh_ctx *c, int enable) {
  if (!c) return invalid("ctx is null");
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(e, "profile sync");
  c->prof = enable != 0;
  c->ev_recs.clear();
  for (int i = 0; i < QEH_NSTAGES; ++i) {
    c->stage_ms[i] = 0.0;
    c->stage_n[i] = 0;
  }
  return QEH_OK;
}

qeh_status qeh_ctx_stage_times(qeh_ctx *c, double *ms, long *launches, int nstages) {
  if (!c) return invalid("ctx is null");
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(e, "stage_times sync");
  for (size_t r = 0; r < c->ev_recs.size(); ++r) {
    float t = 0.f;
    e = hipEventElapsedTime(&t, c->ev_pool[2 * r], c->ev_pool[2 * r + 1]);
    if (e != hipSuccess) return hip_fail(e, "event elapsed");
    c->stage_ms[c->ev_recs[r]] += t;
    c->stage_n[c->ev_recs[r]] += 1;
  }
  c->ev_recs.clear();
  for (int i = 0; i < nstages && i < QEH_NSTAGES; ++i) {
    if (ms) ms[i] = c->stage_ms[i];
    if (launches) launches[i] = c->stage_n[i];
  }
  return QEH_OK;
}

qeh_status qeh_ctx_hdiag(const qeh_ctx *c, double *hdiag) {
  if (!c || !hdiag) return invalid("null argument");
  const hipError_t e = hipMemcpyAsync(hdiag, c->d.hdiag, 8 * (size_t)c->npw,
                                      hipMemcpyDeviceToDevice, c->stream);
  if (e != hipSuccess) return hip_fail(e, "hdiag copy");
  return QEH_OK;
}

qeh_status qeh_ctx_info(const qeh_ctx *c, long *out, int n) {
  if (!c || !out) return invalid("null argument");
  const long v[12] = {c->npw, c->nst, c->nkb, c->n1, c->n2, c->n3, c->ext, c->block, c->prec,
                      c->plane_path, c->zpair, c->wide};
  for (int i = 0; i < n && i < 12; ++i) out[i] = v[i];
  return QEH_OK;
}

}  // extern "C"
