// Local-potential path of H|psi>: sphere scatter + z transforms (K1), the
// per-plane 2D transforms with the V(r) multiply (K2), and z transforms +
// sphere gather + kinetic term (K3).
//
// The paper lists the local-potential and kinetic contributions among the
// Hamiltonian kernels ported to GPUs and builds its 3D FFT from 1D and 2D
// transforms (section "Evolution of the GPU-enabled version").  Here the 3D
// transform is pruned to the data that is non-zero or needed: only the z
// sticks touched by the plane-wave sphere are transformed along z, only the
// x-extent columns of each plane along y, and each plane row along x.
//
// Transforms are in-place mixed-radix (2,3,4,5,7,8) passes in LDS.  Inverse
// transforms use decimation in time, which wants digit-reversed input and
// yields natural order; forward transforms use decimation in frequency,
// natural in and digit-reversed out.  The permutations are folded into the
// scatter / gather index tables, so no explicit reordering pass exists.
#include <algorithm>
#include <cstdlib>
#include <cstring>

#include "cplx.h"
#include "fft_radix.h"
#include "fft_reg.h"
#include "qeh_internal.h"

namespace qeh {
namespace {

// ---------------------------------------------------------------- passes
// tw[t] = exp(-2 pi i t / n); the inverse uses the conjugate.

__device__ __forceinline__ uint32_t fdiv(uint32_t n, const FastDiv &f) {
  return (__umulhi(n, f.m) + n) >> f.s;
}

template <typename C, int R, bool INV, bool DIT>
__device__ __forceinline__ void radix_pass(C *buf, const FastDiv &lines, int ld, int n, int L,
                                           const FastDiv &nbfd, const FastDiv &Ld, const C *tw,
                                           int tid, int nthr) {
  const int nlines = (int)lines.d;
  const int nbf = n / R;
  const int total = nlines * nbf;
  const int tstep = n / (L * R);
  for (int t = tid; t < total; t += nthr) {
    // L == 1: neighbouring threads take neighbouring lines (odd line stride,
    // no LDS bank conflicts); otherwise neighbouring j within a line.
    int line, u;
    if (L == 1) {
      u = (int)fdiv(t, lines);
      line = t - u * nlines;
    } else {
      line = (int)fdiv(t, nbfd);
      u = t - line * nbf;
    }
    const int blk = (int)fdiv(u, Ld);
    const int j = u - blk * L;
    C *p = buf + line * ld + blk * (L * R) + j;
    C v[R];
#pragma unroll
    for (int q = 0; q < R; ++q) v[q] = p[q * L];
    if (DIT && L > 1) {
#pragma unroll
      for (int q = 1; q < R; ++q) {
        C w = tw[q * j * tstep];
        if (INV) w.y = -w.y;
        v[q] = cmul(v[q], w);
      }
    }
    dftR<C, R, INV>(v);
    if (!DIT && L > 1) {
#pragma unroll
      for (int q = 1; q < R; ++q) {
        C w = tw[q * j * tstep];
        if (INV) w.y = -w.y;
        v[q] = cmul(v[q], w);
      }
    }
#pragma unroll
    for (int q = 0; q < R; ++q) p[q * L] = v[q];
  }
}

template <typename C, bool INV, bool DIT>
__device__ __forceinline__ void one_pass(C *buf, const FastDiv &lines, int ld, const FftDim &d,
                                         int p, const C *tw, int tid, int nthr) {
  const int n = d.n, L = d.span[p];
#define QEH_PASS(RR)                                                                     \
  radix_pass<C, RR, INV, DIT>(buf, lines, ld, n, L, d.nbf_div[p], d.span_div[p], tw, tid, \
                              nthr)
  switch (d.radix[p]) {
    case 2: QEH_PASS(2); break;
    case 3: QEH_PASS(3); break;
    case 4: QEH_PASS(4); break;
    case 5: QEH_PASS(5); break;
    case 7: QEH_PASS(7); break;
    case 8: QEH_PASS(8); break;
    default: break;
  }
#undef QEH_PASS
}

// Inverse transform of the lines (stride ld), digit-reversed in, natural out.
template <typename C>
__device__ void fft_inv_dit(C *buf, const FastDiv &lines, int ld, const FftDim &d, const C *tw,
                            int tid, int nthr) {
  for (int p = 0; p < d.npass; ++p) {
    one_pass<C, true, true>(buf, lines, ld, d, p, tw, tid, nthr);
    __syncthreads();
  }
}

// Forward transform, natural in, digit-reversed out.
template <typename C>
__device__ void fft_fwd_dif(C *buf, const FastDiv &lines, int ld, const FftDim &d, const C *tw,
                            int tid, int nthr) {
  for (int p = d.npass - 1; p >= 0; --p) {
    one_pass<C, false, false>(buf, lines, ld, d, p, tw, tid, nthr);
    __syncthreads();
  }
}

constexpr int kNT = 256;

// ---------------------------------------------------------------- K1
// Gamma contexts (real wavefunctions, half sphere of nh stored coefficients):
// "band" p of a launch is the pair c = psi_a + i psi_b at full-sphere index f,
// where f < nh - 1 is -G of stored h = nh - 1 - f (read conjugated) and
// f >= nh - 1 is stored h = f - (nh - 1); the imaginary part at G = 0 is not
// referenced.  The rows (a, b) are (2p, 2p + 1), or pairs[p] when a pair table
// is given; a missing partner (b = nbk, or b < 0 in a table) is zero.
__device__ __forceinline__ double2 gamma_pair(const double2 *__restrict__ psi, int ldpsi, int p,
                                              int f, int nh, int nbk,
                                              const int2 *__restrict__ pairs) {
  int ia = 2 * p, ib = 2 * p + 1 < nbk ? 2 * p + 1 : -1;
  if (pairs) {
    const int2 t = pairs[p];
    ia = t.x;
    ib = t.y;
  }
  const bool neg = f < nh - 1;
  const int h = neg ? nh - 1 - f : f - (nh - 1);
  double2 va = psi[(size_t)ia * ldpsi + h];
  double2 vb = ib >= 0 ? psi[(size_t)ib * ldpsi + h] : make_double2(0.0, 0.0);
  if (h == 0) {
    va.y = 0.0;
    vb.y = 0.0;
  }
  if (neg) {
    va.y = -va.y;
    vb.y = -vb.y;
  }
  return make_double2(va.x - vb.y, va.y + vb.x);
}

// Single-precision copy of the two bands of Gamma pair p for the projector
// GEMM: the stored coefficients h = f - (nh - 1) of the +G half of the sphere
// indices f in [g0, g1), so each is written once.  psi32 rows have length npw.
__device__ __forceinline__ void gamma_pair_copy32(const double2 *__restrict__ psi, int ldpsi,
                                                  int p, int g0, int g1, int nh, int nbk,
                                                  const int2 *__restrict__ pairs,
                                                  float2 *__restrict__ psi32, int npw, int tid,
                                                  int nt) {
  int ia = 2 * p, ib = 2 * p + 1 < nbk ? 2 * p + 1 : -1;
  if (pairs) {
    const int2 t = pairs[p];
    ia = t.x;
    ib = t.y;
  }
  for (int g = max(g0, nh - 1) + tid; g < g1; g += nt) {
    const int h = g - (nh - 1);
    const double2 va = psi[(size_t)ia * ldpsi + h];
    psi32[(size_t)ia * npw + h] = make_float2((float)va.x, (float)va.y);
    if (ib >= 0) {
      const double2 vb = psi[(size_t)ib * ldpsi + h];
      psi32[(size_t)ib * npw + h] = make_float2((float)vb.x, (float)vb.y);
    }
  }
}

// One workgroup: S consecutive sticks of one band.  Their sphere runs are one
// contiguous range of psi (lexicographic Miller order), so the read is
// coalesced; the output rows [z][s0 .. s0+S) are contiguous too.  GAM: the
// Gamma band-pair reading above (nbk bands, nh stored coefficients).
template <typename C, bool GAM = false>
__global__ __launch_bounds__(kNT) void k1_scatter_zinv(
    const double2 *__restrict__ psi, int ldpsi, C *__restrict__ sbuf,
    const int *__restrict__ stick_off, const int *__restrict__ gmap,
    const C *__restrict__ twz, FftDim dz, int nst, int S, int ldz, FastDiv sdiv,
    FastDiv slast, float2 *__restrict__ psi32, int npw, int nbk, int nh,
    const int2 *__restrict__ pairs) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C *tile = reinterpret_cast<C *>(smem_raw);
  C *tw = tile + S * ldz;
  const int tid = threadIdx.x;
  const int b = blockIdx.y;
  const int s0 = blockIdx.x * S;
  const int ns = min(S, nst - s0);
  const int n3 = dz.n;
  for (int i = tid; i < n3; i += kNT) tw[i] = twz[i];
  const C zero = cmk<C>(0, 0);
  for (int i = tid; i < ns * ldz; i += kNT) tile[i] = zero;
  __syncthreads();
  const int g0 = stick_off[s0], g1 = stick_off[s0 + ns];
  const double2 *pb = psi + (size_t)b * ldpsi;
  const int base = s0 * ldz;
  // mixed form: also leave a single-precision copy of psi for the projector
  // GEMM (on Gamma contexts each stored coefficient of the pair's two bands,
  // written from the +G half of the full sphere, so once)
  if (GAM) {
    for (int g = g0 + tid; g < g1; g += kNT)
      tile[gmap[g] - base] = ccast<C>(gamma_pair(psi, ldpsi, b, g, nh, nbk, pairs));
    if (psi32) gamma_pair_copy32(psi, ldpsi, b, g0, g1, nh, nbk, pairs, psi32, npw, tid, kNT);
  } else if (psi32) {
    float2 *p32 = psi32 + (size_t)b * npw;
    for (int g = g0 + tid; g < g1; g += kNT) {
      const double2 v = pb[g];
      tile[gmap[g] - base] = ccast<C>(v);
      p32[g] = make_float2((float)v.x, (float)v.y);
    }
  } else {
    for (int g = g0 + tid; g < g1; g += kNT) tile[gmap[g] - base] = ccast<C>(pb[g]);
  }
  __syncthreads();
  fft_inv_dit<C>(tile, ns == S ? sdiv : slast, ldz, dz, tw, tid, kNT);
  C *out = sbuf + (size_t)b * n3 * nst + s0;
  for (int i = tid; i < ns * n3; i += kNT) {
    const int z = i / ns;
    const int s = i - z * ns;
    out[(size_t)z * nst + s] = tile[s * ldz + z];
  }
}

// ---------------------------------------------------------------- K3
template <typename C>
__global__ __launch_bounds__(kNT) void k3_zfwd_gather(
    const C *__restrict__ sbuf, const double2 *__restrict__ psi, int ldpsi,
    double2 *__restrict__ hpsi, int ldh, const double *__restrict__ kin,
    const int *__restrict__ stick_off, const int *__restrict__ gmap,
    const C *__restrict__ twz, FftDim dz, int nst, int S, int ldz, int add_kin, FastDiv sdiv,
    FastDiv slast) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C *tile = reinterpret_cast<C *>(smem_raw);
  C *tw = tile + S * ldz;
  const int tid = threadIdx.x;
  const int b = blockIdx.y;
  const int s0 = blockIdx.x * S;
  const int ns = min(S, nst - s0);
  const int n3 = dz.n;
  for (int i = tid; i < n3; i += kNT) tw[i] = twz[i];
  const C *in = sbuf + (size_t)b * n3 * nst + s0;
  for (int i = tid; i < ns * n3; i += kNT) {
    const int z = i / ns;
    const int s = i - z * ns;
    tile[s * ldz + z] = in[(size_t)z * nst + s];
  }
  __syncthreads();
  fft_fwd_dif<C>(tile, ns == S ? sdiv : slast, ldz, dz, tw, tid, kNT);
  const int g0 = stick_off[s0], g1 = stick_off[s0 + ns];
  const int base = s0 * ldz;
  const double2 *pb = psi + (size_t)b * ldpsi;
  double2 *hb = hpsi + (size_t)b * ldh;
  for (int g = g0 + tid; g < g1; g += kNT) {
    double2 r = ccast<double2>(tile[gmap[g] - base]);
    if (add_kin) {
      const double2 p = pb[g];
      const double k = kin[g];
      r.x += k * p.x;
      r.y += k * p.y;
    }
    hb[g] = r;
  }
}

// ---------------------------------------------------------------- K2
// Row operations of the plane pass.  A row line (length n = N1) lives in RB;
// the first inverse pass reads its input straight from the column tile T
// (xin[p] = column whose h-index sits at DIT input position p, or -1 for a
// zero), the last inverse pass is fused with the V multiply and the first
// forward pass (both touch the same R positions), and the last forward pass
// writes the x-extent outputs straight back into T.
template <typename C, int R, bool DIT, bool DIF, bool IN_T, bool OUT_T>
__device__ __forceinline__ void row_op(C *RB, int ldR, C *T, int ldT, int y0,
                                       const FastDiv &rows, const int *xin, int n, int L,
                                       const FastDiv &nbfd, const FastDiv &Ld, const C *tw,
                                       const typename real_of<C>::type *vrow, int tid,
                                       int nthr) {
  const int nr = (int)rows.d;
  const int nbf = n / R;
  const int total = nr * nbf;
  const int tstep = n / (L * R);
  const C zero = cmk<C>(0, 0);
  for (int t = tid; t < total; t += nthr) {
    int r, u;
    if (L == 1) {
      u = (int)fdiv(t, rows);
      r = t - u * nr;
    } else {
      r = (int)fdiv(t, nbfd);
      u = t - r * nbf;
    }
    const int blk = (int)fdiv(u, Ld);
    const int j = u - blk * L;
    const int p0 = blk * (L * R) + j;
    C v[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int pos = p0 + q * L;
      if (IN_T) {
        const int c = xin[pos];
        v[q] = c >= 0 ? T[c * ldT + y0 + r] : zero;
      } else {
        v[q] = RB[r * ldR + pos];
      }
    }
    if (DIT) {
      if (L > 1) {
#pragma unroll
        for (int q = 1; q < R; ++q) {
          C w = tw[q * j * tstep];
          w.y = -w.y;
          v[q] = cmul(v[q], w);
        }
      }
      dftR<C, R, true>(v);
    }
    if (DIT && DIF) {
      // natural x order here: multiply by V(r)/N of this row
#pragma unroll
      for (int q = 0; q < R; ++q) v[q] = cscale(v[q], vrow[r * n + p0 + q * L]);
    }
    if (DIF) {
      dftR<C, R, false>(v);
      if (L > 1) {
#pragma unroll
        for (int q = 1; q < R; ++q) v[q] = cmul(v[q], tw[q * j * tstep]);
      }
    }
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int pos = p0 + q * L;
      if (OUT_T) {
        const int c = xin[pos];
        if (c >= 0) T[c * ldT + y0 + r] = v[q];
      } else {
        RB[r * ldR + pos] = v[q];
      }
    }
  }
}

template <typename C, bool DIT, bool DIF, bool IN_T, bool OUT_T>
__device__ __forceinline__ void row_op_r(const FftDim &d, int p, C *RB, int ldR, C *T, int ldT,
                                         int y0, const FastDiv &rows, const int *xin,
                                         const C *tw, const typename real_of<C>::type *vrow,
                                         int tid, int nthr) {
#define QEH_ROW(RR)                                                                        \
  row_op<C, RR, DIT, DIF, IN_T, OUT_T>(RB, ldR, T, ldT, y0, rows, xin, d.n, d.span[p],    \
                                       d.nbf_div[p], d.span_div[p], tw, vrow, tid, nthr)
  switch (d.radix[p]) {
    case 2: QEH_ROW(2); break;
    case 3: QEH_ROW(3); break;
    case 4: QEH_ROW(4); break;
    case 5: QEH_ROW(5); break;
    case 7: QEH_ROW(7); break;
    case 8: QEH_ROW(8); break;
    default: break;
  }
#undef QEH_ROW
}

// Rows y0 .. y0+nr of the plane: x inverse, V multiply, x forward, in place
// on the column tile T.  Ends with a barrier.
template <typename C>
__device__ void row_phase(C *RB, int ldR, C *T, int ldT, int y0, const FastDiv &rows,
                          const int *xin, const FftDim &d, const C *tw,
                          const typename real_of<C>::type *vrow, int tid, int nthr) {
  const int m = d.npass;
  if (m == 1) {
    row_op_r<C, true, true, true, true>(d, 0, RB, ldR, T, ldT, y0, rows, xin, tw, vrow, tid,
                                        nthr);
    __syncthreads();
    return;
  }
  row_op_r<C, true, false, true, false>(d, 0, RB, ldR, T, ldT, y0, rows, xin, tw, vrow, tid,
                                        nthr);
  __syncthreads();
  for (int p = 1; p < m - 1; ++p) {
    row_op_r<C, true, false, false, false>(d, p, RB, ldR, T, ldT, y0, rows, xin, tw, vrow, tid,
                                           nthr);
    __syncthreads();
  }
  row_op_r<C, true, true, false, false>(d, m - 1, RB, ldR, T, ldT, y0, rows, xin, tw, vrow,
                                        tid, nthr);
  __syncthreads();
  for (int p = m - 2; p >= 1; --p) {
    row_op_r<C, false, true, false, false>(d, p, RB, ldR, T, ldT, y0, rows, xin, tw, vrow, tid,
                                           nthr);
    __syncthreads();
  }
  row_op_r<C, false, true, false, true>(d, 0, RB, ldR, T, ldT, y0, rows, xin, tw, vrow, tid,
                                        nthr);
  __syncthreads();
}

// One workgroup: one z-plane of one band.  T holds the x-extent columns of the
// plane (column c = h - hmin, y along the column); rc rows at a time are
// expanded to full x lines in RB for the x transforms and the V multiply.
// Workgroup ids are remapped so that each XCD (ids are dealt round-robin to
// the 8 XCDs) walks a contiguous range of (z, band) with band fastest: the
// bands of one plane share that plane's V in the XCD's L2.
constexpr int kPT = 512;   // plane workgroup: 8 waves

template <typename C>
__global__ __launch_bounds__(kPT) void k2_plane(
    C *__restrict__ sbuf, const typename real_of<C>::type *__restrict__ vs,
    const int *__restrict__ tidx, const int *__restrict__ xin_g,
    const C *__restrict__ twx_g, const C *__restrict__ twy_g, FftDim dx, FftDim dy,
    int nst, int n3, int ext, int ldT, int rc, int ldR, int nbk, int per_xcd, FastDiv extd,
    FastDiv rcd, FastDiv rlastd) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int n1 = dx.n, n2 = dy.n;
  C *T = reinterpret_cast<C *>(smem_raw);
  C *RB = T + ext * ldT;
  C *twx = RB + rc * ldR;
  C *twy = twx + n1;
  int *xin = reinterpret_cast<int *>(twy + n2);
  const int id = blockIdx.x;
  const int logical = (id & 7) * per_xcd + (id >> 3);
  if (logical >= nbk * n3) return;
  const int z = logical / nbk;
  const int b = logical - z * nbk;
  const int tid = threadIdx.x;
  const C zero = cmk<C>(0, 0);

  for (int i = tid; i < ext * ldT; i += kPT) T[i] = zero;
  for (int i = tid; i < n1; i += kPT) {
    twx[i] = twx_g[i];
    xin[i] = xin_g[i];
  }
  for (int i = tid; i < n2; i += kPT) twy[i] = twy_g[i];
  __syncthreads();
  C *plane = sbuf + ((size_t)b * n3 + z) * nst;
  for (int s = tid; s < nst; s += kPT) T[tidx[s]] = plane[s];
  __syncthreads();
  fft_inv_dit<C>(T, extd, ldT, dy, twy, tid, kPT);
  for (int y0 = 0; y0 < n2; y0 += rc) {
    const FastDiv &rows = (y0 + rc <= n2) ? rcd : rlastd;
    row_phase<C>(RB, ldR, T, ldT, y0, rows, xin, dx, twx, vs + ((size_t)z * n2 + y0) * n1, tid,
                 kPT);
  }
  fft_fwd_dif<C>(T, extd, ldT, dy, twy, tid, kPT);
  for (int s = tid; s < nst; s += kPT) plane[s] = T[tidx[s]];
}

// ---------------------------------------------------------------- K2, lane pairs
// Plane pass with every line transform held in registers, for boxes with
// N1 = N2 = N even and a compiled form of N.  Each line (a y column of the
// x-extent tile, or a full x row) belongs to two adjacent lanes that hold one
// half of it each (pair_inv / pair_fwd), so a transform costs one LDS load and
// one LDS store per point, with compile-time indices and twiddles.
// Rows: the x-extent column c = h - hmin sits at x position c instead of
// h mod N.  The shift multiplies the inverse row transform by
// exp(2 pi i hmin x / N) and the forward transform by its conjugate; V(r) is
// real, so the two phases cancel and the values returned on the columns are
// those of the unshifted transform.  Row positions c >= ext load from a zero
// slot and store to a per-thread discard slot, which keeps every lane on one
// path.  Column y positions are natural (tidx holds c*LD + (k mod N)).
// One workgroup: pb bands of one z plane (they read the same V rows), with the
// XCD-aware id remap of the fused kernel.
constexpr int kRT = 256;

// Register budget: three waves per SIMD (<= 168 VGPRs) keeps three 2-band
// workgroups resident per CU at N = 72 without spills, measured faster there
// than two waves per SIMD; N = 90 needs the two-wave budget to avoid spills.
template <typename C, int N>
__global__ __launch_bounds__(kRT) __attribute__((amdgpu_waves_per_eu(N < 90 ? 3 : 2))) void k2_plane_pair(
    C *__restrict__ sbuf, const typename real_of<C>::type *__restrict__ vs,
    const int *__restrict__ tidx, int nst, int n3, int ext, int pb, int nbk, int ngrp,
    int per_xcd) {
  using R = typename real_of<C>::type;
  constexpr int LD = N | 1, M = N / 2;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C *T = reinterpret_cast<C *>(smem_raw);
  const int id = blockIdx.x;
  const int logical = (id & 7) * per_xcd + (id >> 3);
  if (logical >= ngrp * n3) return;
  const int z = logical / ngrp;
  const int g = logical - z * ngrp;
  const int b0 = g * pb;
  const int np = min(pb, nbk - b0);
  const int tid = threadIdx.x;
  const int tile = ext * LD;
  const C *zslot = T + pb * tile;
  C *dslot = T + pb * tile + 1 + tid;
  const C zero = cmk<C>(0, 0);

  for (int i = tid; i < np * tile; i += kRT) T[i] = zero;
  if (tid == 0) T[pb * tile] = zero;
  __syncthreads();
  for (int p = 0; p < np; ++p) {
    const C *plane = sbuf + ((size_t)(b0 + p) * n3 + z) * nst;
    C *Tp = T + p * tile;
    for (int s = tid; s < nst; s += kRT) Tp[tidx[s]] = plane[s];
  }
  __syncthreads();

  // inverse y transforms of the np * ext columns
  for (int j = tid; j < 2 * np * ext; j += kRT) {
    const bool odd = j & 1;
    C *col = T + (j >> 1) * LD;
    C v[M];
#pragma unroll
    for (int n = 0; n < M; ++n) v[n] = col[2 * n + odd];
    regfft::pair_inv<C, N>(v, odd);
    C *out = col + (odd ? M : 0);
#pragma unroll
    for (int k = 0; k < M; ++k) out[k] = v[k];
  }
  __syncthreads();

  // rows: x inverse, V(r)/N, x forward
  for (int j = tid; j < 2 * np * N; j += kRT) {
    const bool odd = j & 1;
    const int r = j >> 1;
    const int p = r / N;
    const int y = r - p * N;
    C *row = T + p * tile + y;
    const int l = odd ? 1 : 0;
    C v[M];
#pragma unroll
    for (int n = 0; n < M; ++n) {
      const int c = 2 * n + l;
      const C *a = c < ext ? row + c * LD : zslot;
      v[n] = *a;
    }
    regfft::pair_inv<C, N>(v, odd);
    const R *vr = vs + ((size_t)z * N + y) * N + l * M;
#pragma unroll
    for (int x = 0; x < M; ++x) v[x] = cscale(v[x], vr[x]);
    regfft::pair_fwd<C, N>(v, odd);
#pragma unroll
    for (int m = 0; m < M; ++m) {
      const int c = 2 * m + l;
      C *a = c < ext ? row + c * LD : dslot;
      *a = v[m];
    }
  }
  __syncthreads();

  // forward y transforms
  for (int j = tid; j < 2 * np * ext; j += kRT) {
    const bool odd = j & 1;
    C *col = T + (j >> 1) * LD;
    const C *in = col + (odd ? M : 0);
    C v[M];
#pragma unroll
    for (int x = 0; x < M; ++x) v[x] = in[x];
    regfft::pair_fwd<C, N>(v, odd);
#pragma unroll
    for (int m = 0; m < M; ++m) col[2 * m + odd] = v[m];
  }
  __syncthreads();
  for (int p = 0; p < np; ++p) {
    C *plane = sbuf + ((size_t)(b0 + p) * n3 + z) * nst;
    const C *Tp = T + p * tile;
    for (int s = tid; s < nst; s += kRT) plane[s] = Tp[tidx[s]];
  }
}

// ---------------------------------------------------------------- density
// Charge density generation: rho(r) = (1/Omega) sum_b occ_b |psi_b(r)|^2.
// The bands reach real space along z and y through K1 and k2a (big holds the
// inverse-y columns of every plane); this kernel takes a group of rows of one
// z plane for a subgroup of bands: rows from big -> inverse x transforms ->
// sum over the subgroup's bands of occ_b |psi_b|^2, accumulated in double in
// band order, written as partial[sub][z][y][x].  density_reduce sums the
// subgroups in order, so every point has one fixed summation order.
constexpr int kDensityPPT = 8;   // grid points per thread of a row group

template <typename C>
__global__ __launch_bounds__(kNT) void k2d_rows_density(
    const C *__restrict__ big, const double *__restrict__ occ, double *__restrict__ partial,
    const int *__restrict__ xin_g, const C *__restrict__ twx_g, FftDim dx, int n2, int n3,
    int ext, int rg, int ldR, int ngroups, int nbk, int bsub, FastDiv rgd, FastDiv rglast) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int n1 = dx.n;
  C *RB = reinterpret_cast<C *>(smem_raw);
  C *twx = RB + rg * ldR;
  int *xin = reinterpret_cast<int *>(twx + n1);
  const int g = blockIdx.x % ngroups;
  const int z = (blockIdx.x / ngroups) % n3;
  const int sub = blockIdx.x / (ngroups * n3);
  const int y0 = g * rg;
  const int nr = min(rg, n2 - y0);
  const int b0 = sub * bsub;
  const int b1 = min(nbk, b0 + bsub);
  const int tid = threadIdx.x;
  const int npt = nr * n1;
  const C zero = cmk<C>(0, 0);
  for (int i = tid; i < n1; i += kNT) {
    twx[i] = twx_g[i];
    xin[i] = xin_g[i];
  }
  __syncthreads();
  // per-thread points: line buffer slot of each input (DIT position p of
  // row r) and of each output (natural x of row r); fixed for every band
  int lds_in[kDensityPPT], src[kDensityPPT], lds_out[kDensityPPT];
#pragma unroll
  for (int k = 0; k < kDensityPPT; ++k) {
    const int i = tid + k * kNT;
    lds_in[k] = -1;
    src[k] = -1;
    lds_out[k] = -1;
    if (i < npt) {
      const int p = i / nr, r = i - (i / nr) * nr;   // r fastest: y-contiguous reads
      const int c = xin[p];
      lds_in[k] = r * ldR + p;
      src[k] = c >= 0 ? c * n2 + y0 + r : -1;
      const int ro = i / n1, x = i - (i / n1) * n1;
      lds_out[k] = ro * ldR + x;
    }
  }
  double acc[kDensityPPT];
#pragma unroll
  for (int k = 0; k < kDensityPPT; ++k) acc[k] = 0.0;
  for (int b = b0; b < b1; ++b) {
    const C *col = big + ((size_t)b * n3 + z) * ext * n2;
#pragma unroll
    for (int k = 0; k < kDensityPPT; ++k)
      if (lds_in[k] >= 0) RB[lds_in[k]] = src[k] >= 0 ? col[src[k]] : zero;
    __syncthreads();
    fft_inv_dit<C>(RB, nr == rg ? rgd : rglast, ldR, dx, twx, tid, kNT);
    const double f = occ[b];
#pragma unroll
    for (int k = 0; k < kDensityPPT; ++k)
      if (lds_out[k] >= 0) {
        const C v = RB[lds_out[k]];
        const double re = static_cast<double>(v.x), im = static_cast<double>(v.y);
        acc[k] += f * (re * re + im * im);
      }
    __syncthreads();
  }
  double *out = partial + ((size_t)sub * n3 + z) * n2 * n1 + (size_t)y0 * n1;
#pragma unroll
  for (int k = 0; k < kDensityPPT; ++k) {
    const int i = tid + k * kNT;
    if (i < npt) out[i] = acc[k];
  }
}

// Density rows on lane pairs (mixed form, N1 = N a compiled size): one
// workgroup = one z plane x one subgroup of bands; the pair (y, l) loads row y
// of each band from big with the x-extent column c at x position c (the shift
// multiplies psi by a unit-modulus phase, which |psi|^2 does not see),
// transforms it in registers and keeps its N/2 points' occ_b |psi_b|^2 sums in
// double registers across the subgroup, in band order.
template <int N>
__global__ __launch_bounds__(kRT) __attribute__((amdgpu_waves_per_eu(2))) void k2d_rows_pair(
    const float2 *__restrict__ big, const double *__restrict__ occ, double *__restrict__ partial,
    const float2 *__restrict__ zcol, int n2, int n3, int ext, int nbk, int bsub) {
  constexpr int M = N / 2;
  const int z = blockIdx.x % n3;
  const int sub = blockIdx.x / n3;
  const int b0 = sub * bsub;
  const int b1 = min(nbk, b0 + bsub);
  const int j = threadIdx.x;
  if (j >= 2 * n2) return;   // no barriers below
  const bool odd = j & 1;
  const int y = j >> 1;
  const int l = odd ? 1 : 0;
  double acc[M];
#pragma unroll
  for (int k = 0; k < M; ++k) acc[k] = 0.0;
  for (int b = b0; b < b1; ++b) {
    const float2 *col = big + ((size_t)b * n3 + z) * ext * n2 + y;
    float2 v[M];
#pragma unroll
    for (int n = 0; n < M; ++n) {
      // positions beyond the x-extent read a zero column in the workspace
      const int c = 2 * n + l;
      const float2 *src = c < ext ? col + (size_t)c * n2 : zcol + y;
      v[n] = *src;
    }
    regfft::pair_inv<float2, N>(v, odd);
    const double f = occ[b];
#pragma unroll
    for (int k = 0; k < M; ++k) {
      const double re = v[k].x, im = v[k].y;
      acc[k] += f * (re * re + im * im);
    }
  }
  double *out = partial + (((size_t)sub * n3 + z) * n2 + y) * N + l * M;
#pragma unroll
  for (int k = 0; k < M; ++k) out[k] = acc[k];
}

// Fused density plane pass on lane pairs (mixed form, N1 = N2 = N a compiled
// size, lane-pair plane tables): one workgroup = one z plane x one subgroup of
// bands.  Per band: the plane's sticks into the LDS column tile (natural y),
// inverse y transforms of the x-extent columns, then the x rows, each held by
// the same pair (y, l) for every band, whose N/2 points accumulate
// occ_b |psi_b|^2 in double registers (the x shift of the rows is a unit-modulus
// phase).  No HBM round trip between the column and row transforms.
template <int N>
__global__ __launch_bounds__(kRT) __attribute__((amdgpu_waves_per_eu(2))) void k2d_plane_pair(
    const float2 *__restrict__ sbuf, const double *__restrict__ occ, double *__restrict__ partial,
    const int *__restrict__ tidx, int nst, int n3, int ext, int nbk, int bsub) {
  constexpr int LD = N | 1, M = N / 2;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  float2 *T = reinterpret_cast<float2 *>(smem_raw);
  const int tile = ext * LD;
  const float2 *zslot = T + tile;
  const int z = blockIdx.x % n3;
  const int sub = blockIdx.x / n3;
  const int b0 = sub * bsub;
  const int b1 = min(nbk, b0 + bsub);
  const int tid = threadIdx.x;
  const float2 zero = make_float2(0.f, 0.f);
  if (tid == 0) T[tile] = zero;
  const bool row_lane = tid < 2 * N;
  const bool odd = tid & 1;
  const int l = odd ? 1 : 0;
  const int y = tid >> 1;
  double acc[M];
#pragma unroll
  for (int k = 0; k < M; ++k) acc[k] = 0.0;
  for (int b = b0; b < b1; ++b) {
    for (int i = tid; i < tile; i += kRT) T[i] = zero;
    __syncthreads();
    const float2 *plane = sbuf + ((size_t)b * n3 + z) * nst;
    for (int s = tid; s < nst; s += kRT) T[tidx[s]] = plane[s];
    __syncthreads();
    for (int j = tid; j < 2 * ext; j += kRT) {
      const bool jodd = j & 1;
      float2 *col = T + (j >> 1) * LD;
      float2 v[M];
#pragma unroll
      for (int n = 0; n < M; ++n) v[n] = col[2 * n + jodd];
      regfft::pair_inv<float2, N>(v, jodd);
      float2 *out = col + (jodd ? M : 0);
#pragma unroll
      for (int k = 0; k < M; ++k) out[k] = v[k];
    }
    __syncthreads();
    if (row_lane) {
      const float2 *row = T + y;
      float2 v[M];
#pragma unroll
      for (int n = 0; n < M; ++n) {
        const int c = 2 * n + l;
        const float2 *a = c < ext ? row + c * LD : zslot;
        v[n] = *a;
      }
      regfft::pair_inv<float2, N>(v, odd);
      const double f = occ[b];
#pragma unroll
      for (int k = 0; k < M; ++k) {
        const double re = v[k].x, im = v[k].y;
        acc[k] += f * (re * re + im * im);
      }
    }
    __syncthreads();
  }
  if (row_lane) {
    double *out = partial + (((size_t)sub * n3 + z) * N + y) * N + l * M;
#pragma unroll
    for (int k = 0; k < M; ++k) out[k] = acc[k];
  }
}

// Fused density plane pass on lane quads (FP64 form, N1 = N2 = N a compiled
// lane-quad size, natural-y plane tables): as the lane-pair form above, with
// each column and row held by four lanes (quad_inv); 512 threads so that every
// row has its own quad ((y, q) = (tid / 4, tid % 4), 4 N <= 512).  The inverse
// leaves lane q with x positions k + (N/4) br(q), k < N/4; the x shift is a
// unit-modulus phase again.  The per-point sums live in LDS (each lane owns
// its N/4 entries; in registers they spilled at N = 72).
constexpr int kDQT = 512;

template <int N>
__global__ __launch_bounds__(kDQT) __attribute__((amdgpu_waves_per_eu(2))) void k2d_plane_quad(
    const double2 *__restrict__ sbuf, const double *__restrict__ occ,
    double *__restrict__ partial, const int *__restrict__ tidx, const double2 *__restrict__ tw_g,
    int nst, int n3, int ext, int nbk, int bsub) {
  constexpr int LD = N | 1, Q = N / 4;
  static_assert(4 * N <= kDQT, "one quad per row");
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double2 *T = reinterpret_cast<double2 *>(smem_raw);
  const int tile = ext * LD;
  const double2 *zslot = T + tile;
  double2 *twq = T + tile + 1;   // [4][Q]: row q holds W_N^{q k}
  double *acc = reinterpret_cast<double *>(twq + 4 * Q);   // [N][N] sums of the plane
  const int z = blockIdx.x % n3;
  const int sub = blockIdx.x / n3;
  const int b0 = sub * bsub;
  const int b1 = min(nbk, b0 + bsub);
  const int tid = threadIdx.x;
  const double2 zero = make_double2(0.0, 0.0);
  const int q = tid & 3;
  const int bq = ((q & 1) << 1) | (q >> 1);   // two-bit reversal of q
  const regfft::QuadLane<double> ql(q);
  const double2 *tw = twq + q * Q;
  const bool row_lane = tid < 4 * N;
  const int y = tid >> 2;
  if (tid == 0) T[tile] = zero;
  for (int i = tid; i < 4 * Q; i += kDQT) twq[i] = tw_g[((i / Q) * (i % Q)) % N];
  for (int i = tid; i < N * N; i += kDQT) acc[i] = 0.0;
  double *mine = acc + y * N + Q * bq;   // this lane's points (row lanes only)
  for (int b = b0; b < b1; ++b) {
    for (int i = tid; i < tile; i += kDQT) T[i] = zero;
    __syncthreads();
    const double2 *plane = sbuf + ((size_t)b * n3 + z) * nst;
    for (int s = tid; s < nst; s += kDQT) T[tidx[s]] = plane[s];
    __syncthreads();
    for (int j = tid; j < 4 * ext; j += kDQT) {
      double2 *col = T + (j >> 2) * LD;
      double2 v[Q];
#pragma unroll
      for (int n = 0; n < Q; ++n) v[n] = col[4 * n + q];
      regfft::quad_inv<double2, N>(v, tw, ql);
      double2 *out = col + Q * bq;
#pragma unroll
      for (int k = 0; k < Q; ++k) out[k] = v[k];
    }
    __syncthreads();
    if (row_lane) {
      const double2 *row = T + y;
      double2 v[Q];
#pragma unroll
      for (int n = 0; n < Q; ++n) {
        const int c = 4 * n + q;
        const double2 *a = c < ext ? row + c * LD : zslot;
        v[n] = *a;
      }
      regfft::quad_inv<double2, N>(v, tw, ql);
      const double f = occ[b];
#pragma unroll
      for (int k = 0; k < Q; ++k) mine[k] += f * (v[k].x * v[k].x + v[k].y * v[k].y);
    }
    __syncthreads();
  }
  double *out = partial + ((size_t)sub * n3 + z) * N * N;
  for (int i = tid; i < N * N; i += kDQT) out[i] = acc[i];
}

// rho[i] = (accumulate ? rho[i] : 0) + scale * sum_sub partial[sub][i], sub in order.
__global__ __launch_bounds__(256) void density_reduce(const double *__restrict__ partial,
                                                      int nsub, long npts, double scale,
                                                      double *__restrict__ rho, int accumulate) {
  for (long i = blockIdx.x * 256L + threadIdx.x; i < npts; i += (long)gridDim.x * 256) {
    double t = 0.0;
    for (int s = 0; s < nsub; ++s) t += partial[(size_t)s * npts + i];
    rho[i] = (accumulate ? rho[i] : 0.0) + scale * t;
  }
}

// ---------------------------------------------------------------- K2, lane quads / octets
// Register plane pass for N1 = N2 = N with a compiled form: each line belongs
// to L adjacent lanes holding N/L points each (L = 4: quad_inv / quad_fwd;
// L = 8, single precision: oct_inv / oct_fwd).  The inverse returns
// lane-bit-reversed blocks, which is the forward's input layout, so the row
// chain inverse -> V -> forward moves no data.  The x-extent shift of the rows
// and the zero / discard slots are those of the lane-pair kernel.  One band per
// workgroup by default.  FP64 (lane quads, N <= 72, 256 threads): the column
// tile is 42 KB at N = 72.  Single precision (the boxes above the lane-pair
// sizes, 512 threads): lane quads at N = 96, lane octets at N >= 120 (20 points
// per lane at N = 160, where quads need 40 and spill); at the 512-atom cell
// one workgroup (89 KB of column tile for its x-extent of 69) fills a CU.
template <int L> __device__ __forceinline__ int lane_rev(int o) {
  return L == 4 ? (((o & 1) << 1) | (o >> 1)) : (((o & 1) << 2) | (o & 2) | (o >> 2));
}

template <typename C, int N, int L> struct LineLanes;
template <typename C, int N> struct LineLanes<C, N, 4> {
  regfft::QuadLane<typename real_of<C>::type> ql;
  __device__ explicit LineLanes(int o) : ql(o) {}
  __device__ void inv(C *v, const C *tw) const { regfft::quad_inv<C, N>(v, tw, ql); }
  __device__ void fwd(C *v, const C *tw) const { regfft::quad_fwd<C, N>(v, tw, ql); }
};
template <int N> struct LineLanes<float2, N, 8> {
  regfft::OctLane ol;
  __device__ explicit LineLanes(int o) : ol(o) {}
  __device__ void inv(float2 *v, const float2 *tw) const { regfft::oct_inv<N>(v, tw, ol); }
  __device__ void fwd(float2 *v, const float2 *tw) const { regfft::oct_fwd<N>(v, tw, ol); }
};

template <typename C, int N, int NT, int L>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(
    NT > 256 ? 2 : (N < 48 ? 3 : 2)))) void k2_plane_lanes(
    C *__restrict__ sbuf, const typename real_of<C>::type *__restrict__ vs,
    const int *__restrict__ tidx, const C *__restrict__ tw_g, int nst, int n3, int ext, int pb,
    int nbk, int ngrp, int per_xcd) {
  using R = typename real_of<C>::type;
  constexpr int LD = N | 1, Q = N / L;
  static_assert(Q * L == N, "N must be a multiple of the lanes per line");
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C *T = reinterpret_cast<C *>(smem_raw);
  const int id = blockIdx.x;
  const int logical = (id & 7) * per_xcd + (id >> 3);
  if (logical >= ngrp * n3) return;
  const int z = logical / ngrp;
  const int g = logical - z * ngrp;
  const int b0 = g * pb;
  const int np = min(pb, nbk - b0);
  const int tid = threadIdx.x;
  const int tile = ext * LD;
  const C *zslot = T + pb * tile;
  C *dslot = T + pb * tile + 1 + tid;
  C *twl = T + pb * tile + 1 + NT;   // [L][Q]: row o holds W_N^{o k}
  const C zero = cmk<C>(0, 0);
  const int o = tid & (L - 1);
  const int bo = lane_rev<L>(o);
  const LineLanes<C, N, L> ln(o);
  const C *tw = twl + o * Q;

  for (int i = tid; i < np * tile; i += NT) T[i] = zero;
  if (tid == 0) T[pb * tile] = zero;
  for (int i = tid; i < L * Q; i += NT) twl[i] = tw_g[((i / Q) * (i % Q)) % N];
  __syncthreads();
  for (int p = 0; p < np; ++p) {
    const C *plane = sbuf + ((size_t)(b0 + p) * n3 + z) * nst;
    C *Tp = T + p * tile;
    for (int s = tid; s < nst; s += NT) Tp[tidx[s]] = plane[s];
  }
  __syncthreads();
  for (int j = tid; j < L * np * ext; j += NT) {
    C *col = T + (j / L) * LD;
    C v[Q];
#pragma unroll
    for (int n = 0; n < Q; ++n) v[n] = col[L * n + o];
    ln.inv(v, tw);
    C *out = col + Q * bo;
#pragma unroll
    for (int k = 0; k < Q; ++k) out[k] = v[k];
  }
  __syncthreads();
  for (int j = tid; j < L * np * N; j += NT) {
    const int r = j / L;
    const int p = r / N;
    const int y = r - p * N;
    C *row = T + p * tile + y;
    C v[Q];
#pragma unroll
    for (int n = 0; n < Q; ++n) {
      const int c = L * n + o;
      const C *a = c < ext ? row + c * LD : zslot;
      v[n] = *a;
    }
    ln.inv(v, tw);
    const R *vr = vs + ((size_t)z * N + y) * N + Q * bo;
#pragma unroll
    for (int k = 0; k < Q; ++k) v[k] = cscale(v[k], vr[k]);
    ln.fwd(v, tw);
#pragma unroll
    for (int m = 0; m < Q; ++m) {
      const int c = L * m + o;
      C *a = c < ext ? row + c * LD : dslot;
      *a = v[m];
    }
  }
  __syncthreads();
  for (int j = tid; j < L * np * ext; j += NT) {
    C *col = T + (j / L) * LD;
    const C *in = col + Q * bo;
    C v[Q];
#pragma unroll
    for (int x = 0; x < Q; ++x) v[x] = in[x];
    ln.fwd(v, tw);
#pragma unroll
    for (int m = 0; m < Q; ++m) col[L * m + o] = v[m];
  }
  __syncthreads();
  for (int p = 0; p < np; ++p) {
    C *plane = sbuf + ((size_t)(b0 + p) * n3 + z) * nst;
    const C *Tp = T + p * tile;
    for (int s = tid; s < nst; s += NT) plane[s] = Tp[tidx[s]];
  }
}

// threads of the lane-quad / lane-octet plane workgroup: 256 in FP64, 512 in
// single precision (two waves per SIMD)
constexpr int quad_plane_threads(bool fp64, int n) { return fp64 ? kRT : 512; }
// lanes per line: octets for the single-precision boxes of >= 120 points
constexpr int plane_lanes(bool fp64, int n) { return !fp64 && n >= 120 ? 8 : 4; }

// Box sizes with a compiled lane-quad kernel (double precision).
#define QEH_QUAD_SIZES(X) X(16) X(20) X(24) X(32) X(36) X(40) X(48) X(60) X(64) X(72)

// Box sizes with a compiled single-precision lane-quad kernel (above the
// lane-pair sizes).
#define QEH_QUAD32_SIZES(X) X(96) X(120) X(128) X(144) X(160)

// Box sizes with a compiled lane-pair kernel (single precision).
#define QEH_PAIR_SIZES(X) \
  X(16) X(18) X(20) X(24) X(30) X(32) X(36) X(40) X(48) X(50) X(54) X(60) X(64) X(72) X(80) X(90)
// ... and for the density kernels, whose per-point sums add registers (N = 90
// would spill)
#define QEH_DENSITY_PAIR_SIZES(X) \
  X(16) X(18) X(20) X(24) X(30) X(32) X(36) X(40) X(48) X(50) X(54) X(60) X(64) X(72) X(80)

// ---------------------------------------------------------------- K1 / K3, lane pairs
// Mixed form with N3 = N even and a compiled form of N: the z transforms held
// in registers by lane pairs (pair_inv / pair_fwd).  The sphere runs of S
// consecutive sticks are staged through LDS at natural z positions (gmap holds
// s*ldz + (l mod N3) for this path) so that the psi reads and H psi writes stay
// coalesced; each pair then loads its z line from LDS once.  K1 writes the
// transformed line straight to the plane-major stick buffer: the lanes of a
// wave hold consecutive sticks, so every store covers two runs of consecutive
// sticks.  K3 reads the same way, transforms forward, and stages the result
// for the sphere gather.
constexpr int kPairSticks = 64;   // 37 KB of LDS at N = 72: four workgroups per CU

template <int N, bool GAM = false>
__global__ __launch_bounds__(kNT) __attribute__((amdgpu_waves_per_eu(N < 90 ? 3 : 2))) void
k1_pair(const double2 *__restrict__ psi, int ldpsi, float2 *__restrict__ sbuf,
        const int *__restrict__ stick_off, const int *__restrict__ gmap, int nst,
        float2 *__restrict__ psi32, int npw, int nbk, int nh, const int2 *__restrict__ pairs) {
  constexpr int LD = N | 1, M = N / 2;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  float2 *tile = reinterpret_cast<float2 *>(smem_raw);
  const int tid = threadIdx.x;
  const int b = blockIdx.y;
  const int s0 = blockIdx.x * kPairSticks;
  const int ns = min(kPairSticks, nst - s0);
  const float2 zero = make_float2(0.f, 0.f);
  for (int i = tid; i < ns * LD; i += kNT) tile[i] = zero;
  __syncthreads();
  const int g0 = stick_off[s0], g1 = stick_off[s0 + ns];
  const int base = s0 * LD;
  for (int g = g0 + tid; g < g1; g += kNT) {
    const double2 v =
        GAM ? gamma_pair(psi, ldpsi, b, g, nh, nbk, pairs) : psi[(size_t)b * ldpsi + g];
    const float2 f = make_float2((float)v.x, (float)v.y);
    tile[gmap[g] - base] = f;
    if (!GAM) psi32[(size_t)b * npw + g] = f;
  }
  if (GAM && psi32) gamma_pair_copy32(psi, ldpsi, b, g0, g1, nh, nbk, pairs, psi32, npw, tid, kNT);
  __syncthreads();
  float2 *out = sbuf + (size_t)b * N * nst + s0;
  for (int j = tid; j < 2 * ns; j += kNT) {
    const bool odd = j & 1;
    const int st = j >> 1;
    const float2 *line = tile + st * LD;
    float2 v[M];
#pragma unroll
    for (int n = 0; n < M; ++n) v[n] = line[2 * n + odd];
    regfft::pair_inv<float2, N>(v, odd);
    float2 *o = out + (size_t)(odd ? M : 0) * nst + st;
#pragma unroll
    for (int k = 0; k < M; ++k) o[(size_t)k * nst] = v[k];
  }
}

template <int N>
__global__ __launch_bounds__(kNT) __attribute__((amdgpu_waves_per_eu(N < 90 ? 3 : 2))) void
k3_pair(const float2 *__restrict__ sbuf, const double2 *__restrict__ psi, int ldpsi,
        double2 *__restrict__ hpsi, int ldh, const double *__restrict__ kin,
        const int *__restrict__ stick_off, const int *__restrict__ gmap, int nst, int add_kin) {
  constexpr int LD = N | 1, M = N / 2;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  float2 *tile = reinterpret_cast<float2 *>(smem_raw);
  const int tid = threadIdx.x;
  const int b = blockIdx.y;
  const int s0 = blockIdx.x * kPairSticks;
  const int ns = min(kPairSticks, nst - s0);
  const float2 *in = sbuf + (size_t)b * N * nst + s0;
  for (int j = tid; j < 2 * ns; j += kNT) {
    const bool odd = j & 1;
    const int st = j >> 1;
    const float2 *ip = in + (size_t)(odd ? M : 0) * nst + st;
    float2 v[M];
#pragma unroll
    for (int x = 0; x < M; ++x) v[x] = ip[(size_t)x * nst];
    regfft::pair_fwd<float2, N>(v, odd);
    float2 *line = tile + st * LD;
#pragma unroll
    for (int m = 0; m < M; ++m) line[2 * m + odd] = v[m];
  }
  __syncthreads();
  const int g0 = stick_off[s0], g1 = stick_off[s0 + ns];
  const int base = s0 * LD;
  const double2 *pb = psi + (size_t)b * ldpsi;
  double2 *hb = hpsi + (size_t)b * ldh;
  for (int g = g0 + tid; g < g1; g += kNT) {
    double2 r = ccast<double2>(tile[gmap[g] - base]);
    if (add_kin) {
      const double2 p = pb[g];
      const double k = kin[g];
      r.x += k * p.x;
      r.y += k * p.y;
    }
    hb[g] = r;
  }
}

// ---------------------------------------------------------------- K2, split
// Planes whose column tile does not fit in LDS go through an HBM scratch
// big[b][z][c][y] (one x-extent column of N2 values after another):
//   k2a: a group of columns of one plane: sticks -> inverse y transforms -> big
//   k2b: a group of rows of one plane: big -> x inverse, V, x forward -> big
//   k2c: a group of columns: big -> forward y transforms -> sticks
// The transforms are the same device routines as in the fused kernel.
template <typename C>
__global__ __launch_bounds__(kNT) void k2a_columns_inv(
    const C *__restrict__ sbuf, C *__restrict__ big, const int *__restrict__ tidx,
    const int *__restrict__ colstart, const C *__restrict__ twy_g, FftDim dy, int nst, int n3,
    int ext, int ldT, int cg, int ngroups, FastDiv cgd, FastDiv cglast) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int n2 = dy.n;
  C *T = reinterpret_cast<C *>(smem_raw);
  C *twy = T + cg * ldT;
  const int g = blockIdx.x % ngroups;
  const int bz = blockIdx.x / ngroups;   // b * n3 + z
  const int c0 = g * cg;
  const int nc = min(cg, ext - c0);
  const int tid = threadIdx.x;
  const C zero = cmk<C>(0, 0);
  for (int i = tid; i < nc * ldT; i += kNT) T[i] = zero;
  for (int i = tid; i < n2; i += kNT) twy[i] = twy_g[i];
  __syncthreads();
  const C *plane = sbuf + (size_t)bz * nst;
  for (int s = colstart[c0] + tid; s < colstart[c0 + nc]; s += kNT)
    T[tidx[s] - c0 * ldT] = plane[s];
  __syncthreads();
  fft_inv_dit<C>(T, nc == cg ? cgd : cglast, ldT, dy, twy, tid, kNT);
  C *out = big + ((size_t)bz * ext + c0) * n2;
  for (int i = tid; i < nc * n2; i += kNT) {
    const int c = i / n2, y = i - (i / n2) * n2;
    out[i] = T[c * ldT + y];
  }
}

template <typename C>
__global__ __launch_bounds__(kNT) void k2b_rows(
    C *__restrict__ big, const typename real_of<C>::type *__restrict__ vs,
    const int *__restrict__ xin_g, const C *__restrict__ twx_g, FftDim dx, int n2, int n3,
    int ext, int rg, int ldl, int ldR, int ngroups, FastDiv rgd, FastDiv rglast) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int n1 = dx.n;
  C *Tl = reinterpret_cast<C *>(smem_raw);
  C *RB = Tl + ext * ldl;
  C *twx = RB + rg * ldR;
  int *xin = reinterpret_cast<int *>(twx + n1);
  const int g = blockIdx.x % ngroups;
  const int bz = blockIdx.x / ngroups;
  const int z = bz % n3;
  const int y0 = g * rg;
  const int nr = min(rg, n2 - y0);
  const int tid = threadIdx.x;
  for (int i = tid; i < n1; i += kNT) {
    twx[i] = twx_g[i];
    xin[i] = xin_g[i];
  }
  C *col = big + (size_t)bz * ext * n2;
  for (int i = tid; i < ext * nr; i += kNT) {
    const int c = i / nr, r = i - (i / nr) * nr;
    Tl[c * ldl + r] = col[(size_t)c * n2 + y0 + r];
  }
  __syncthreads();
  row_phase<C>(RB, ldR, Tl, ldl, 0, nr == rg ? rgd : rglast, xin, dx, twx,
               vs + ((size_t)z * n2 + y0) * n1, tid, kNT);
  for (int i = tid; i < ext * nr; i += kNT) {
    const int c = i / nr, r = i - (i / nr) * nr;
    col[(size_t)c * n2 + y0 + r] = Tl[c * ldl + r];
  }
}

template <typename C>
__global__ __launch_bounds__(kNT) void k2c_columns_fwd(
    C *__restrict__ sbuf, const C *__restrict__ big, const int *__restrict__ tidx,
    const int *__restrict__ colstart, const C *__restrict__ twy_g, FftDim dy, int nst, int n3,
    int ext, int ldT, int cg, int ngroups, FastDiv cgd, FastDiv cglast) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int n2 = dy.n;
  C *T = reinterpret_cast<C *>(smem_raw);
  C *twy = T + cg * ldT;
  const int g = blockIdx.x % ngroups;
  const int bz = blockIdx.x / ngroups;
  const int c0 = g * cg;
  const int nc = min(cg, ext - c0);
  const int tid = threadIdx.x;
  for (int i = tid; i < n2; i += kNT) twy[i] = twy_g[i];
  const C *in = big + ((size_t)bz * ext + c0) * n2;
  for (int i = tid; i < nc * n2; i += kNT) {
    const int c = i / n2, y = i - (i / n2) * n2;
    T[c * ldT + y] = in[i];
  }
  __syncthreads();
  fft_fwd_dif<C>(T, nc == cg ? cgd : cglast, ldT, dy, twy, tid, kNT);
  C *plane = sbuf + (size_t)bz * nst;
  for (int s = colstart[c0] + tid; s < colstart[c0 + nc]; s += kNT)
    plane[s] = T[tidx[s] - c0 * ldT];
}

template <typename K> void allow_lds(K kern, size_t bytes) {
  if (bytes > 64 * 1024)
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// GAM: nbk launch "bands" are Gamma band pairs of nb_gam bands (nh = npw), or
// the pairs of a table.
template <typename C, bool GAM>
hipError_t k1_impl(const qeh_ctx *c, int nbk, const double2 *psi, int ldpsi, int nb_gam,
                   const int2 *pairs, float2 *p32) {
  const C *tw = reinterpret_cast<const C *>(c->d.tw) + c->tw_off[2];
  dim3 grid((c->nst + c->sg.S - 1) / c->sg.S, nbk);
  allow_lds(k1_scatter_zinv<C, GAM>, c->sg.lds_bytes);
  hipLaunchKernelGGL((k1_scatter_zinv<C, GAM>), grid, dim3(kNT), c->sg.lds_bytes, c->stream,
                     psi, ldpsi, reinterpret_cast<C *>(c->d.sbuf), c->d.stick_off, c->d.gmap, tw,
                     c->dz, c->nst, c->sg.S, c->sg.ldz, c->sg.s_div, c->sg.slast_div,
                     p32, c->npw_fft, nb_gam, c->npw, pairs);
  return hipGetLastError();
}

template <typename C>
hipError_t k3_impl(const qeh_ctx *c, int nbk, const double2 *psi, int ldpsi, double2 *hpsi,
                   int ldh, int add_kin) {
  const C *tw = reinterpret_cast<const C *>(c->d.tw) + c->tw_off[2];
  dim3 grid((c->nst + c->sg.S - 1) / c->sg.S, nbk);
  allow_lds(k3_zfwd_gather<C>, c->sg.lds_bytes);
  hipLaunchKernelGGL(k3_zfwd_gather<C>, grid, dim3(kNT), c->sg.lds_bytes, c->stream,
                     reinterpret_cast<const C *>(c->d.sbuf), psi, ldpsi, hpsi, ldh, c->d.kin,
                     c->d.stick_off, c->d.gmap, tw, c->dz, c->nst, c->sg.S, c->sg.ldz, add_kin,
                     c->sg.s_div, c->sg.slast_div);
  return hipGetLastError();
}

template <typename C> hipError_t k2_split_impl(const qeh_ctx *c, int nbk) {
  using R = typename real_of<C>::type;
  const C *tw = reinterpret_cast<const C *>(c->d.tw);
  const SplitGeom &g = c->spg;
  C *big = reinterpret_cast<C *>(c->d.big);
  C *sb = reinterpret_cast<C *>(c->d.sbuf);
  const int ncg = (c->ext + g.cg - 1) / g.cg;
  const int nrg = (c->n2 + g.rg - 1) / g.rg;
  const unsigned planes = (unsigned)nbk * c->n3;
  allow_lds(k2a_columns_inv<C>, g.lds_col);
  hipLaunchKernelGGL(k2a_columns_inv<C>, dim3(planes * ncg), dim3(kNT), g.lds_col, c->stream, sb,
                     big, c->d.tidx, c->d.colstart, tw + c->tw_off[1], c->dy, c->nst, c->n3,
                     c->ext, c->pg.ldT, g.cg, ncg, g.cg_div, g.cglast_div);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  allow_lds(k2b_rows<C>, g.lds_row);
  hipLaunchKernelGGL(k2b_rows<C>, dim3(planes * nrg), dim3(kNT), g.lds_row, c->stream, big,
                     reinterpret_cast<const R *>(c->d.vs), c->d.xin, tw + c->tw_off[0], c->dx,
                     c->n2, c->n3, c->ext, g.rg, g.ldl, c->pg.ldR, nrg, g.rg_div, g.rglast_div);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  allow_lds(k2c_columns_fwd<C>, g.lds_col);
  hipLaunchKernelGGL(k2c_columns_fwd<C>, dim3(planes * ncg), dim3(kNT), g.lds_col, c->stream, sb,
                     big, c->d.tidx, c->d.colstart, tw + c->tw_off[1], c->dy, c->nst, c->n3,
                     c->ext, c->pg.ldT, g.cg, ncg, g.cg_div, g.cglast_div);
  return hipGetLastError();
}

template <typename C> hipError_t k2_impl(const qeh_ctx *c, int nbk) {
  using R = typename real_of<C>::type;
  const C *tw = reinterpret_cast<const C *>(c->d.tw);
  const int total = nbk * c->n3;
  const int per_xcd = (total + 7) / 8;
  allow_lds(k2_plane<C>, c->pg.lds_bytes);
  hipLaunchKernelGGL(k2_plane<C>, dim3(8 * per_xcd), dim3(kPT), c->pg.lds_bytes, c->stream,
                     reinterpret_cast<C *>(c->d.sbuf), reinterpret_cast<const R *>(c->d.vs),
                     c->d.tidx, c->d.xin, tw + c->tw_off[0], tw + c->tw_off[1], c->dx, c->dy,
                     c->nst, c->n3, c->ext, c->pg.ldT, c->pg.rc, c->pg.ldR, nbk, per_xcd,
                     c->pg.ext_div, c->pg.rc_div, c->pg.rlast_div);
  return hipGetLastError();
}

template <int N> hipError_t k2_pair_launch(const qeh_ctx *c, int nbk) {
  const int pb = c->pg.pb;
  const int ngrp = (nbk + pb - 1) / pb;
  const int per_xcd = (ngrp * c->n3 + 7) / 8;
  allow_lds(k2_plane_pair<float2, N>, c->pg.lds_pair);
  hipLaunchKernelGGL((k2_plane_pair<float2, N>), dim3(8 * per_xcd), dim3(kRT), c->pg.lds_pair,
                     c->stream, reinterpret_cast<float2 *>(c->d.sbuf),
                     reinterpret_cast<const float *>(c->d.vs), c->d.tidx, c->nst, c->n3, c->ext,
                     pb, nbk, ngrp, per_xcd);
  return hipGetLastError();
}

hipError_t k2_pair_impl(const qeh_ctx *c, int nbk) {
  switch (c->n1) {
#define QEH_PAIR_CASE(NN) \
  case NN: return k2_pair_launch<NN>(c, nbk);
    QEH_PAIR_SIZES(QEH_PAIR_CASE)
#undef QEH_PAIR_CASE
    default: return hipErrorInvalidValue;
  }
}

template <typename C> hipError_t density_columns_impl(const qeh_ctx *c, int nbk, void *big_v) {
  const C *tw = reinterpret_cast<const C *>(c->d.tw);
  const SplitGeom &g = c->spg;
  C *big = reinterpret_cast<C *>(big_v);
  const int ncg = (c->ext + g.cg - 1) / g.cg;
  const unsigned planes = (unsigned)nbk * c->n3;
  allow_lds(k2a_columns_inv<C>, g.lds_col);
  hipLaunchKernelGGL(k2a_columns_inv<C>, dim3(planes * ncg), dim3(kNT), g.lds_col, c->stream,
                     reinterpret_cast<const C *>(c->d.sbuf), big, c->d.tidx_dit, c->d.colstart,
                     tw + c->tw_off[1], c->dy, c->nst, c->n3, c->ext, c->pg.ldT, g.cg, ncg,
                     g.cg_div, g.cglast_div);
  return hipGetLastError();
}

template <int N>
hipError_t density_rows_pair_launch(const qeh_ctx *c, const DensityGeom &dg, int nbk,
                                    const void *big, const double *occ_d, double *partial,
                                    const void *zcol) {
  const int nsub = (nbk + dg.bsub - 1) / dg.bsub;
  hipLaunchKernelGGL(k2d_rows_pair<N>, dim3((unsigned)nsub * c->n3), dim3(kRT), 0, c->stream,
                     reinterpret_cast<const float2 *>(big), occ_d, partial,
                     reinterpret_cast<const float2 *>(zcol), c->n2, c->n3, c->ext, nbk, dg.bsub);
  return hipGetLastError();
}

template <int N>
hipError_t density_plane_pair_launch(const qeh_ctx *c, const DensityGeom &dg, int nbk,
                                     const double *occ_d, double *partial) {
  const int nsub = (nbk + dg.bsub - 1) / dg.bsub;
  const size_t lds = 8 * ((size_t)c->ext * (N | 1) + 1);
  allow_lds(k2d_plane_pair<N>, lds);
  hipLaunchKernelGGL(k2d_plane_pair<N>, dim3((unsigned)nsub * c->n3), dim3(kRT), lds, c->stream,
                     reinterpret_cast<const float2 *>(c->d.sbuf), occ_d, partial, c->d.tidx,
                     c->nst, c->n3, c->ext, nbk, dg.bsub);
  return hipGetLastError();
}

template <int N>
hipError_t density_plane_quad_launch(const qeh_ctx *c, const DensityGeom &dg, int nbk,
                                     const double *occ_d, double *partial) {
  const int nsub = (nbk + dg.bsub - 1) / dg.bsub;
  const size_t lds = 16 * ((size_t)c->ext * (N | 1) + 1 + N) + 8 * (size_t)N * N;
  allow_lds(k2d_plane_quad<N>, lds);
  hipLaunchKernelGGL(k2d_plane_quad<N>, dim3((unsigned)nsub * c->n3), dim3(kDQT), lds, c->stream,
                     reinterpret_cast<const double2 *>(c->d.sbuf), occ_d, partial, c->d.tidx,
                     reinterpret_cast<const double2 *>(c->d.tw) + c->tw_off[0], c->nst, c->n3,
                     c->ext, nbk, dg.bsub);
  return hipGetLastError();
}

template <typename C>
hipError_t density_rows_impl(const qeh_ctx *c, const DensityGeom &dg, int nbk, const void *big,
                             const double *occ_d, double *partial, const void *zcol) {
  if (dg.pair) {
    switch (c->n1) {
#define QEH_PAIR_CASE(NN) \
  case NN: return density_rows_pair_launch<NN>(c, dg, nbk, big, occ_d, partial, zcol);
      QEH_DENSITY_PAIR_SIZES(QEH_PAIR_CASE)
#undef QEH_PAIR_CASE
      default: return hipErrorInvalidValue;
    }
  }
  const C *tw = reinterpret_cast<const C *>(c->d.tw);
  const int nsub = (nbk + dg.bsub - 1) / dg.bsub;
  allow_lds(k2d_rows_density<C>, dg.lds);
  hipLaunchKernelGGL(k2d_rows_density<C>, dim3((unsigned)nsub * c->n3 * dg.ngroups), dim3(kNT),
                     dg.lds, c->stream, reinterpret_cast<const C *>(big), occ_d, partial,
                     c->d.xin, tw + c->tw_off[0], c->dx, c->n2, c->n3, c->ext, dg.rg,
                     c->pg.ldR, dg.ngroups, nbk, dg.bsub, dg.rg_div, dg.rglast_div);
  return hipGetLastError();
}

template <int N, bool GAM>
hipError_t k1_pair_launch(const qeh_ctx *c, int nbk, const double2 *psi, int ldpsi, int nb_gam,
                          const int2 *pairs, float2 *p32) {
  const size_t lds = 8 * (size_t)kPairSticks * (N | 1);
  allow_lds(k1_pair<N, GAM>, lds);
  hipLaunchKernelGGL((k1_pair<N, GAM>), dim3((c->nst + kPairSticks - 1) / kPairSticks, nbk),
                     dim3(kNT), lds, c->stream, psi, ldpsi, reinterpret_cast<float2 *>(c->d.sbuf),
                     c->d.stick_off, c->d.gmap, c->nst, p32, c->npw_fft, nb_gam, c->npw,
                     pairs);
  return hipGetLastError();
}

template <int N>
hipError_t k3_pair_launch(const qeh_ctx *c, int nbk, const double2 *psi, int ldpsi,
                          double2 *hpsi, int ldh, int add_kin) {
  const size_t lds = 8 * (size_t)kPairSticks * (N | 1);
  allow_lds(k3_pair<N>, lds);
  hipLaunchKernelGGL(k3_pair<N>, dim3((c->nst + kPairSticks - 1) / kPairSticks, nbk), dim3(kNT),
                     lds, c->stream, reinterpret_cast<const float2 *>(c->d.sbuf), psi, ldpsi,
                     hpsi, ldh, c->d.kin, c->d.stick_off, c->d.gmap, c->nst, add_kin);
  return hipGetLastError();
}

template <bool GAM>
hipError_t k1_pair_impl(const qeh_ctx *c, int nbk, const double2 *psi, int ldpsi, int nb_gam,
                        const int2 *pairs, float2 *p32) {
  switch (c->n3) {
#define QEH_PAIR_CASE(NN) \
  case NN: return k1_pair_launch<NN, GAM>(c, nbk, psi, ldpsi, nb_gam, pairs, p32);
    QEH_PAIR_SIZES(QEH_PAIR_CASE)
#undef QEH_PAIR_CASE
    default: return hipErrorInvalidValue;
  }
}

hipError_t k3_pair_impl(const qeh_ctx *c, int nbk, const double2 *psi, int ldpsi, double2 *hpsi,
                        int ldh, int add_kin) {
  switch (c->n3) {
#define QEH_PAIR_CASE(NN) \
  case NN: return k3_pair_launch<NN>(c, nbk, psi, ldpsi, hpsi, ldh, add_kin);
    QEH_PAIR_SIZES(QEH_PAIR_CASE)
#undef QEH_PAIR_CASE
    default: return hipErrorInvalidValue;
  }
}

template <typename C, int N> hipError_t k2_quad_launch(const qeh_ctx *c, int nbk) {
  using R = typename real_of<C>::type;
  constexpr int NT = quad_plane_threads(sizeof(R) == 8, N);
  constexpr int L = plane_lanes(sizeof(R) == 8, N);
  const int pb = c->pg.pb;
  const int ngrp = (nbk + pb - 1) / pb;
  const int per_xcd = (ngrp * c->n3 + 7) / 8;
  allow_lds(k2_plane_lanes<C, N, NT, L>, c->pg.lds_pair);
  hipLaunchKernelGGL((k2_plane_lanes<C, N, NT, L>), dim3(8 * per_xcd), dim3(NT), c->pg.lds_pair,
                     c->stream, reinterpret_cast<C *>(c->d.sbuf),
                     reinterpret_cast<const R *>(c->d.vs), c->d.tidx,
                     reinterpret_cast<const C *>(c->d.tw) + c->tw_off[0], c->nst, c->n3, c->ext,
                     pb, nbk, ngrp, per_xcd);
  return hipGetLastError();
}

hipError_t k2_quad_impl(const qeh_ctx *c, int nbk) {
  if (c->prec == QEH_FP64) {
    switch (c->n1) {
#define QEH_QUAD_CASE(NN) \
  case NN: return k2_quad_launch<double2, NN>(c, nbk);
      QEH_QUAD_SIZES(QEH_QUAD_CASE)
#undef QEH_QUAD_CASE
      default: return hipErrorInvalidValue;
    }
  }
  switch (c->n1) {
#define QEH_QUAD_CASE(NN) \
  case NN: return k2_quad_launch<float2, NN>(c, nbk);
    QEH_QUAD32_SIZES(QEH_QUAD_CASE)
#undef QEH_QUAD_CASE
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

size_t plane_lds_bytes(int prec, int ext, int n1, int n2, const PlaneGeom &g) {
  const size_t c = prec == QEH_FP64 ? 16 : 8;
  return c * ((size_t)ext * g.ldT + (size_t)g.rc * g.ldR + n1 + n2) + 4 * (size_t)n1;
}

bool density_geometry(const qeh_ctx *c, DensityGeom *dg) {
  const int n1 = c->n1, n2 = c->n2;
  const size_t cs = c->prec == QEH_FP64 ? 16 : 8;
  dg->bsub = 16;
  // lane-pair rows: mixed form, N1 a compiled size, one pair per row of a plane
  // (QEH_DENSITY_KERNEL=generic keeps the LDS-pass rows: test hook)
  const char *kern = std::getenv("QEH_DENSITY_KERNEL");
  dg->pair = pair_plane_supported(c->prec, n1, n1) && n1 <= 80 && 2 * n2 <= kRT &&
             !(kern && std::strcmp(kern, "generic") == 0);   // N1 = 90 would spill
  // fused plane pass: lane-pair plane tables (natural y) and a square plane;
  // in FP64 the lane-quad form on the lane-quad plane tables
  const bool unfused =
      kern && (std::strcmp(kern, "rows") == 0 || std::strcmp(kern, "generic") == 0);
  dg->fused = dg->pair && c->plane_path == 2 && n1 == n2 &&
              8 * ((size_t)c->ext * (n2 | 1) + 1) <= (size_t)kLdsMax && !unfused;
  dg->fused_quad = c->prec == QEH_FP64 && c->plane_path == 4 && n1 == n2 && 4 * n1 <= kDQT &&
                   quad_plane_supported(c->prec, n1, n2) &&
                   16 * ((size_t)c->ext * (n2 | 1) + 1 + n1) + 8 * (size_t)n1 * n1 <=
                       (size_t)kLdsMax &&
                   !unfused;
  if (dg->fused_quad) dg->fused = true;
  // the fused pass runs its bands one after another per workgroup: smaller
  // subgroups give more workgroups (measured: 8 bands 0.27 ms, 16 bands
  // 0.30 ms per 128-band density at the 72^3 cell)
  if (dg->fused) dg->bsub = 8;
  dg->rg = std::max(1, std::min(n2, kDensityPPT * kNT / n1));
  if ((size_t)dg->rg * n1 > (size_t)kDensityPPT * kNT) return false;
  dg->ngroups = (n2 + dg->rg - 1) / dg->rg;
  dg->rg_div = make_fastdiv(dg->rg);
  dg->rglast_div = make_fastdiv(n2 - (dg->ngroups - 1) * dg->rg);
  dg->lds = cs * ((size_t)dg->rg * c->pg.ldR + n1) + 4 * (size_t)n1;
  return dg->lds <= (size_t)kLdsMax && c->spg.lds_col <= (size_t)kLdsMax;
}

hipError_t launch_density_columns(const qeh_ctx *c, int nbk, void *big) {
  return c->prec == QEH_FP64 ? density_columns_impl<double2>(c, nbk, big)
                             : density_columns_impl<float2>(c, nbk, big);
}

hipError_t launch_density_plane(const qeh_ctx *c, const DensityGeom &dg, int nbk,
                                const double *occ_d, double *partial) {
  if (dg.fused_quad) {
    switch (c->n1) {
#define QEH_QUAD_CASE(NN) \
  case NN: return density_plane_quad_launch<NN>(c, dg, nbk, occ_d, partial);
      QEH_QUAD_SIZES(QEH_QUAD_CASE)
#undef QEH_QUAD_CASE
      default: return hipErrorInvalidValue;
    }
  }
  switch (c->n1) {
#define QEH_PAIR_CASE(NN) \
  case NN: return density_plane_pair_launch<NN>(c, dg, nbk, occ_d, partial);
    QEH_DENSITY_PAIR_SIZES(QEH_PAIR_CASE)
#undef QEH_PAIR_CASE
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_density_rows(const qeh_ctx *c, const DensityGeom &dg, int nbk, const void *big,
                               const double *occ_d, double *partial, const void *zcol) {
  return c->prec == QEH_FP64 ? density_rows_impl<double2>(c, dg, nbk, big, occ_d, partial, zcol)
                             : density_rows_impl<float2>(c, dg, nbk, big, occ_d, partial, zcol);
}

hipError_t launch_density_reduce(const double *partial, int nsub, long npts, double scale,
                                 double *rho, int accumulate, hipStream_t s) {
  const int blocks = (int)std::min<long>((npts + 255) / 256, 8192);
  hipLaunchKernelGGL(density_reduce, dim3(blocks), dim3(256), 0, s, partial, nsub, npts, scale,
                     rho, accumulate);
  return hipGetLastError();
}

bool pair_z_supported(int prec, int n3) { return pair_plane_supported(prec, n3, n3); }

bool quad_plane_supported(int prec, int n1, int n2) {
  if (n1 != n2) return false;
  if (prec == QEH_FP64) {
    switch (n1) {
#define QEH_QUAD_CASE(NN) \
  case NN: return true;
      QEH_QUAD_SIZES(QEH_QUAD_CASE)
#undef QEH_QUAD_CASE
      default: return false;
    }
  }
  switch (n1) {
#define QEH_QUAD_CASE(NN) \
  case NN: return true;
    QEH_QUAD32_SIZES(QEH_QUAD_CASE)
#undef QEH_QUAD_CASE
    default: return false;
  }
}

size_t quad_plane_lds_bytes(int prec, int ext, int n2, int pb) {
  const bool f64 = prec == QEH_FP64;
  const size_t c = f64 ? 16 : 8;
  // column tiles, zero slot, discard slots, the [4][N/4] twiddle table
  return c * ((size_t)pb * ext * (n2 | 1) + 1 + quad_plane_threads(f64, n2) + n2);
}

size_t pair_z_lds_bytes(int n3) { return 8 * (size_t)kPairSticks * (n3 | 1); }

bool pair_plane_supported(int prec, int n1, int n2) {
  if (prec != QEH_MIXED || n1 != n2) return false;
  switch (n1) {
#define QEH_PAIR_CASE(NN) \
  case NN: return true;
    QEH_PAIR_SIZES(QEH_PAIR_CASE)
#undef QEH_PAIR_CASE
    default: return false;
  }
}

size_t pair_plane_lds_bytes(int prec, int ext, int n2, int pb) {
  const size_t c = prec == QEH_FP64 ? 16 : 8;
  // column tiles, zero slot, discard slots
  return c * ((size_t)pb * ext * (n2 | 1) + 1 + kRT);
}

size_t stick_lds_bytes(int prec, int n3, const StickGeom &g) {
  const size_t c = prec == QEH_FP64 ? 16 : 8;
  return c * ((size_t)g.S * g.ldz + n3);
}

hipError_t launch_k1(const qeh_ctx *c, int nbk, const double2 *psi, int ldpsi) {
  // mixed form: K1 also leaves the single-precision copy of the block for the
  // projector GEMM
  float2 *p32 = c->prec == QEH_MIXED ? c->d.psi32 : nullptr;
  if (c->zpair) return k1_pair_impl<false>(c, nbk, psi, ldpsi, 0, nullptr, p32);
  return c->prec == QEH_FP64 ? k1_impl<double2, false>(c, nbk, psi, ldpsi, 0, nullptr, p32)
                             : k1_impl<float2, false>(c, nbk, psi, ldpsi, 0, nullptr, p32);
}

hipError_t launch_k1_gamma(const qeh_ctx *c, int nbk, const double2 *psi, int ldpsi,
                           const int2 *pairs, int npairs, bool copy32) {
  const int np = pairs ? npairs : (nbk + 1) / 2;
  // the single-precision copy only for a block of <= block bands in natural
  // pairs (its rows are the bands' indices)
  float2 *p32 = copy32 && !pairs && nbk <= c->block && c->prec == QEH_MIXED ? c->d.psi32 : nullptr;
  if (c->zpair) return k1_pair_impl<true>(c, np, psi, ldpsi, nbk, pairs, p32);
  return c->prec == QEH_FP64 ? k1_impl<double2, true>(c, np, psi, ldpsi, nbk, pairs, p32)
                             : k1_impl<float2, true>(c, np, psi, ldpsi, nbk, pairs, p32);
}

hipError_t launch_k2(const qeh_ctx *c, int nbk) {
  if (c->plane_path == 2) return k2_pair_impl(c, nbk);
  if (c->plane_path == 4) return k2_quad_impl(c, nbk);
  if (c->plane_path != 0)
    return c->prec == QEH_FP64 ? k2_split_impl<double2>(c, nbk) : k2_split_impl<float2>(c, nbk);
  return c->prec == QEH_FP64 ? k2_impl<double2>(c, nbk) : k2_impl<float2>(c, nbk);
}

hipError_t launch_k3(const qeh_ctx *c, int nbk, const double2 *psi, int ldpsi, double2 *hpsi,
                     int ldh, int add_kinetic) {
  if (c->zpair) return k3_pair_impl(c, nbk, psi, ldpsi, hpsi, ldh, add_kinetic);
  return c->prec == QEH_FP64 ? k3_impl<double2>(c, nbk, psi, ldpsi, hpsi, ldh, add_kinetic)
                             : k3_impl<float2>(c, nbk, psi, ldpsi, hpsi, ldh, add_kinetic);
}

}  // namespace qeh
