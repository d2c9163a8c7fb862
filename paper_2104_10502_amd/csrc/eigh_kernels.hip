// Dense Hermitian solver of the Davidson Rayleigh-Ritz step, written for the
// small reduced problems of block Davidson (n <= 2048): the paper solves this
// small generalized eigenproblem with a dense GPU solver (section "Evolution
// of the GPU-enabled version").  H y = eps S y for the lowest nb
// pairs, in deterministic kernels (fixed summation orders, no atomics on
// floating-point data):
//
//   chol_kernel     one workgroup: S = L L^H, right-looking, lower triangle
//                   (orders <= 64); cholp_kernel: one launch per 16-column
//                   panel over many workgroups (larger orders)
//   trsm_kernel     one wave per column, many workgroups: L X = B (forward),
//                   with B given or as the adjoint of a matrix, or L^H X = B
//                   (backward with the explicit L^H); A = L^-1 H L^-H by two
//                   of them, Y = L^-H Z by a third
//   tdstep_kernel   one launch per Householder step while the trailing block
//                   is larger than kTailN, one wave per column, many
//                   workgroups
//   tridiag_lds_kernel  one workgroup, trailing block in LDS: the last
//                   kTailN steps of the Householder reduction A = Q T Q^H, T
//                   real symmetric tridiagonal (d, e), reflectors kept in A
//   trieig_kernel   the nb lowest eigenpairs of T.  T is split where
//                   |e_k| <= eps ||T||; the global nb-th eigenvalue is
//                   bracketed by multisection of Sturm counts; every block's
//                   eigenvalues below it are found by multisection over many
//                   workgroups (first launch) and sorted (second launch, one
//                   workgroup); eigenvectors come from twisted
//                   factorizations of T_b - lambda I (one thread each), except
//                   for groups of numerically equal eigenvalues of one block
//                   (gap <= 1e-12 ||T||, as exact multiplets of A leave them:
//                   Householder does not split T there), which get inverse
//                   iteration from distinct start vectors through one pivoted
//                   LU of T_b - sigma I with Gram-Schmidt between the two
//                   sweeps; vectors of close eigenvalues of one block
//                   (gap <= 1e-5 ||T||) are re-orthogonalised in index order
//   backtr_kernel   one wave per column, many workgroups: Z = Q Z_T through
//                   the stored reflectors (staged in LDS, shared by a
//                   workgroup's waves)
//
// Storage: column-major double2 matrices with leading dimension ld.  A real
// symmetric pair (Gamma point) goes through the same kernels with zero
// imaginary parts, which stay zero.
#include <hip/hip_runtime.h>

#include "cplx.h"
#include "qeh_internal.h"

namespace qeh {
namespace {

constexpr int kET = 1024;            // threads of the one-workgroup kernels
constexpr int kEW = kET / 64;        // their waves
constexpr int kEMaxN = kEigMaxN;     // largest problem
constexpr int kSlots = kEMaxN / 64;  // register slots per lane at the largest order
constexpr int kCholMaxN = 512;       // largest order of the one-workgroup Cholesky (LDS panel)
constexpr double kEps = 2.220446049250313e-16;
constexpr double kTiny = 2.2250738585072014e-308;
constexpr double kDegRel = 1e-12;    // numerically equal eigenvalues (relative to ||T||)
constexpr double kCloseRel = 1e-5;   // close eigenvalues, re-orthogonalised

__device__ __forceinline__ double wave_sum(double v) {
  // fixed butterfly; lane 0's result is what callers use
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return __shfl(v, 0);
}

// Sum over the workgroup (NW waves), identical in every thread and from run
// to run.
// Two sums at once (red holds 2 NW doubles): the same orders as two calls of
// block_sum, one pair of barriers.
template <int NW> __device__ double2 block_sum2(double a, double b, double *red) {
  a = wave_sum(a);
  b = wave_sum(b);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    red[threadIdx.x >> 6] = a;
    red[NW + (threadIdx.x >> 6)] = b;
  }
  __syncthreads();
  double sa = 0.0, sb = 0.0;
  for (int i = 0; i < NW; ++i) sa += red[i];
  for (int i = 0; i < NW; ++i) sb += red[NW + i];
  return make_double2(sa, sb);
}

template <int NW = kEW> __device__ double block_sum(double v, double *red) {
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < NW; ++i) s += red[i];
  return s;
}

__device__ double block_max(double v, double *red) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = red[0];
  for (int i = 1; i < kEW; ++i) s = fmax(s, red[i]);
  return s;
}

__device__ double block_min(double v, double *red) {
  return -block_max(-v, red);
}

// ---------------------------------------------------------------- Cholesky
// S (n x n, lower triangle read) = L L^H in place (lower).  info = 0, or
// j + 1 if the leading (j+1) x (j+1) minor is not positive definite (or not
// finite); L is then incomplete.
//
// Right-looking by panels of kCB columns: the panel (rows jb..n-1) is
// factored in LDS, written back, and the trailing lower triangle gets one
// rank-kCB update, each element read and written once per panel (the row's
// panel entries in registers, the column's broadcast from LDS).
constexpr int kCB = 16;
constexpr int kCBP = kCB + 1;   // padded LDS row stride (bank spread)

__global__ __launch_bounds__(kET) void chol_kernel(double2 *S, long ld, int n, int *info) {
  __shared__ double2 P[kCholMaxN * kCBP];
  const int tid = threadIdx.x;
  for (int jb = 0; jb < n; jb += kCB) {
    const int b = min(kCB, n - jb), m = n - jb;
    for (int idx = tid; idx < m * kCB; idx += kET) {
      const int r = idx % m, c = idx / m;
      P[r * kCBP + c] = (c < b && r >= c) ? S[(jb + r) + (long)(jb + c) * ld] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    for (int c = 0; c < b; ++c) {
      const double ajj = P[c * kCBP + c].x;
      if (!(ajj > 0.0) || !isfinite(ajj)) {   // same value in every thread
        if (tid == 0) *info = jb + c + 1;
        return;
      }
      const double ljj = sqrt(ajj), rinv = 1.0 / ljj;
      __syncthreads();
      for (int r = c + tid; r < m; r += kET)
        P[r * kCBP + c] = r == c ? make_double2(ljj, 0.0) : cscale(P[r * kCBP + c], rinv);
      __syncthreads();
      const int w = b - c - 1;
      for (int idx = tid; idx < m * w; idx += kET) {
        const int r = idx % m, c2 = c + 1 + idx / m;
        if (r >= c2) P[r * kCBP + c2] = csub(P[r * kCBP + c2], cmulc(P[r * kCBP + c], P[c2 * kCBP + c]));
      }
      __syncthreads();
    }
    for (int idx = tid; idx < m * b; idx += kET) {
      const int r = idx % m, c = idx / m;
      if (r >= c) S[(jb + r) + (long)(jb + c) * ld] = P[r * kCBP + c];
    }
    const int mt = n - jb - b;
    if (mt > 0) {
      const int g = kET / mt;   // >= 2
      if (tid < g * mt) {
        const int r = tid % mt, grp = tid / mt;
        double2 pr[kCB];
#pragma unroll
        for (int c = 0; c < kCB; ++c) pr[c] = P[(b + r) * kCBP + c];
        double2 *row = S + (jb + b + r) + (long)(jb + b) * ld;
        for (int kk = grp; kk <= r; kk += g) {
          const double2 *pk = P + (b + kk) * kCBP;
          double2 acc = row[(long)kk * ld];
#pragma unroll
          for (int c = 0; c < kCB; ++c) acc = csub(acc, cmulc(pr[c], pk[c]));
          row[(long)kk * ld] = acc;
        }
      }
    }
    __syncthreads();
  }
  if (tid == 0) *info = 0;
}

// Blocked form over many workgroups, one launch per panel of kCB columns.
// Launch p (panel jb = p kCB): every workgroup factors the b x b diagonal
// block L11 itself (the same data and arithmetic in each, hence the same
// L11), forms the rows of L21 = A21 L11^-H that its kCT x kCT tile of the
// trailing lower triangle needs, and subtracts L21 L21^H from that tile.  The
// factored panel goes to a scratch panel (parity p & 1; L11 by tile (0, 0),
// the rows of L21 by the diagonal tiles) and launch p + 1, which reads
// neither, copies it into S: within a launch no workgroup writes what another
// reads.  The last panel (no trailing block) writes its L11 to S itself.
// Launch 0 sets info = 0; a panel that is not positive definite sets
// jb + c + 1, and every later launch returns at once.
constexpr int kCT = 32;   // trailing-update tile
constexpr int kCholOneWG = 64;   // orders left to the one-workgroup kernel

__global__ __launch_bounds__(256) void cholp_kernel(double2 *S, long ld, int n, int jb,
                                                    double2 *scr, int *info) {
  __shared__ double2 D[kCB * kCBP];          // diagonal block -> L11
  __shared__ double2 Lr[2][kCT * kCBP];      // panel rows of the tile's rows / columns
  const int tid = threadIdx.x;
  if (jb > 0 && *info != 0) return;
  if (jb == 0 && blockIdx.x == 0 && tid == 0) *info = 0;
  const int b = min(kCB, n - jb), m = n - jb, mt = m - b;
  const int pan = jb / kCB;
  double2 *cur = scr + (long)(pan & 1) * n * kCB;
  // the previous panel into S
  if (jb > 0) {
    const int jp = jb - kCB, mp = n - jp;
    const double2 *prev = scr + (long)((pan - 1) & 1) * n * kCB;
    for (int idx = blockIdx.x * 256 + tid; idx < mp * kCB; idx += gridDim.x * 256) {
      const int r = idx % mp, c = idx / mp;
      if (r >= c) S[(jp + r) + (long)(jp + c) * ld] = prev[r * kCB + c];
    }
  }
  for (int idx = tid; idx < kCB * kCB; idx += 256) {
    const int r = idx % kCB, c = idx / kCB;
    D[r * kCBP + c] = (r < b && c < b && r >= c) ? S[(jb + r) + (long)(jb + c) * ld]
                                                : make_double2(0.0, 0.0);
  }
  __syncthreads();
  for (int c = 0; c < b; ++c) {
    const double ajj = D[c * kCBP + c].x;
    if (!(ajj > 0.0) || !isfinite(ajj)) {   // same value in every workgroup
      if (blockIdx.x == 0 && tid == 0) *info = jb + c + 1;
      return;
    }
    const double ljj = sqrt(ajj), rinv = 1.0 / ljj;
    __syncthreads();
    if (tid >= c && tid < b)
      D[tid * kCBP + c] = tid == c ? make_double2(ljj, 0.0) : cscale(D[tid * kCBP + c], rinv);
    __syncthreads();
    const int w = b - c - 1;
    if (tid < b * w) {
      const int r = tid % b, c2 = c + 1 + tid / b;
      if (r >= c2) D[r * kCBP + c2] = csub(D[r * kCBP + c2], cmulc(D[r * kCBP + c], D[c2 * kCBP + c]));
    }
    __syncthreads();
  }
  if (mt == 0) {   // last panel
    if (blockIdx.x == 0)
      for (int idx = tid; idx < b * b; idx += 256) {
        const int r = idx % b, c = idx / b;
        if (r >= c) S[(jb + r) + (long)(jb + c) * ld] = D[r * kCBP + c];
      }
    return;
  }
  // this workgroup's tile (ti >= tj) of the trailing lower triangle
  const int x = blockIdx.x;
  int ti = (int)((sqrt(8.0 * x + 1.0) - 1.0) * 0.5);
  while (ti * (ti + 1) / 2 > x) --ti;
  while ((ti + 1) * (ti + 2) / 2 <= x) ++ti;
  const int tj = x - ti * (ti + 1) / 2;
  const int r0[2] = {ti * kCT, tj * kCT};   // rows of the trailing block
  // panel rows of the tile's rows and columns, then L21 = A21 L11^-H (one
  // thread per row, forward in the column index)
  for (int idx = tid; idx < 2 * kCT * kCB; idx += 256) {
    const int h = idx / (kCT * kCB), e = idx % (kCT * kCB);
    const int r = e % kCT, c = e / kCT;
    const int gr = r0[h] + r;
    Lr[h][r * kCBP + c] = (gr < mt && c < b) ? S[(jb + b + gr) + (long)(jb + c) * ld]
                                             : make_double2(0.0, 0.0);
  }
  __syncthreads();
  if (tid < 2 * kCT) {
    const int h = tid / kCT, r = tid % kCT;
    double2 *row = &Lr[h][r * kCBP];
    for (int c = 0; c < b; ++c) {
      double2 a = row[c];
      for (int c2 = 0; c2 < c; ++c2) a = csub(a, cmulc(row[c2], D[c * kCBP + c2]));
      row[c] = cscale(a, 1.0 / D[c * kCBP + c].x);
    }
  }
  __syncthreads();
  // the factored panel to the scratch panel
  if (ti == tj) {
    for (int idx = tid; idx < kCT * kCB; idx += 256) {
      const int r = idx % kCT, c = idx / kCT;
      if (r0[0] + r < mt) cur[(b + r0[0] + r) * kCB + c] = Lr[0][r * kCBP + c];
    }
    if (ti == 0)
      for (int idx = tid; idx < kCB * kCB; idx += 256) {
        const int r = idx % kCB, c = idx / kCB;
        cur[r * kCB + c] = D[r * kCBP + c];
      }
  }
  // tile -= L21(rows) L21(cols)^H
  for (int e = tid; e < kCT * kCT; e += 256) {
    const int r = e % kCT, k = e / kCT;
    const int gr = r0[0] + r, gk = r0[1] + k;
    if (gr >= mt || gk >= mt || gk > gr) continue;
    double2 *p = S + (jb + b + gr) + (long)(jb + b + gk) * ld;
    double2 acc = *p;
#pragma unroll
    for (int c = 0; c < kCB; ++c) acc = csub(acc, cmulc(Lr[0][r * kCBP + c], Lr[1][k * kCBP + c]));
    *p = acc;
  }
}

// ---------------------------------------------------------------- triangular solves
// One wave per right-hand side column j; the column's n <= 64 NS entries sit in
// registers (row s * 64 + lane in slot s).
//   MODE 0: L x = b,   L lower (T), b = B(:, j)
//   MODE 1: L x = b,   b = conj(M(j, :)) with M = B (column j of M^H)
//   MODE 2: U x = b,   U upper (T), b = B(:, j)   (backward)
// The diagonal of T is real (a Cholesky factor).
//
// By blocks of 64 rows (one slot): the diagonal block of T is staged in LDS
// (shared by the workgroup's four waves) and the block's 64 unknowns are
// solved there, a dependent chain through LDS and scalar lane reads; the
// slots on the far side then take the block's contribution, x_s -= T_sb x_b,
// whose T loads are independent of one another and stream from L2.  Each
// x_i still receives its terms T_ik x_k in the order of k.
__device__ __forceinline__ double lane_read(double v, int l) {
  // value of lane l (wave-uniform) of v, through the scalar unit
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// One block round: solve block (= slot) B, then the far side.  B is a
// template argument so that every slot index is a compile-time constant and
// x stays in registers.
template <int MODE, int B, int NS>
__device__ __forceinline__ void trsm_round(double2 (&x)[NS], const double2 *__restrict__ T,
                                           long ldt, int n, int lane, double2 (*Tb)[64],
                                           double *rd) {
  const int nbk = (n + 63) / 64;
  if (B >= nbk) return;   // uniform
  const int b0 = B * 64, bs = min(64, n - b0);
  __syncthreads();
  for (int idx = threadIdx.x; idx < 64 * 64; idx += 256) {
    const int r = idx & 63, c = idx >> 6;
    if (r < bs && c < bs) Tb[c][r] = T[(b0 + r) + (long)(b0 + c) * ldt];
  }
  if ((int)threadIdx.x < bs)
    rd[threadIdx.x] = 1.0 / T[(b0 + threadIdx.x) + (long)(b0 + threadIdx.x) * ldt].x;
  __syncthreads();
  // the block's unknowns
  if (MODE != 2) {
    for (int c = 0; c < bs; ++c) {
      const double2 xk = cscale(make_double2(lane_read(x[B].x, c), lane_read(x[B].y, c)), rd[c]);
      if (lane == c) x[B] = xk;
      else if (lane > c && lane < bs) x[B] = csub(x[B], cmul(Tb[c][lane], xk));
    }
  } else {
    for (int c = bs - 1; c >= 0; --c) {
      const double2 xk = cscale(make_double2(lane_read(x[B].x, c), lane_read(x[B].y, c)), rd[c]);
      if (lane == c) x[B] = xk;
      else if (lane < c) x[B] = csub(x[B], cmul(Tb[c][lane], xk));
    }
  }
  // the far side: x_s -= T(rows of s, columns of B) x_B
#pragma unroll
  for (int s2 = 0; s2 < NS; ++s2) {
    const bool far = MODE == 2 ? s2 < B : s2 > B;
    const int i = s2 * 64 + lane;
    if (far && s2 < nbk) {
      const double2 *tc = T + i + (long)b0 * ldt;
      double2 acc = x[s2];
      for (int c0 = 0; c0 < bs; c0 += 8) {
        double2 tv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u)
          tv[u] = i < n && c0 + u < bs ? tc[(long)(c0 + u) * ldt] : make_double2(0.0, 0.0);
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          if (c0 + u < bs) {
            const double2 xc = make_double2(lane_read(x[B].x, c0 + u), lane_read(x[B].y, c0 + u));
            acc = csub(acc, cmul(tv[u], xc));
          }
        }
      }
      if (i < n) x[s2] = acc;
    }
  }
}

// All block rounds, in solve order (forward for MODE 0 / 1, backward for 2).
template <int MODE, int NS, int Q>
__device__ __forceinline__ void trsm_rounds(double2 (&x)[NS], const double2 *__restrict__ T,
                                            long ldt, int n, int lane, double2 (*Tb)[64],
                                            double *rd) {
  if constexpr (Q < NS) {
    trsm_round<MODE, MODE == 2 ? NS - 1 - Q : Q, NS>(x, T, ldt, n, lane, Tb, rd);
    trsm_rounds<MODE, NS, Q + 1>(x, T, ldt, n, lane, Tb, rd);
  }
}

// NS register slots per lane (orders up to 64 NS).
template <int MODE, int NS>
__global__ __launch_bounds__(256) void trsm_kernel(const double2 *__restrict__ T, long ldt, int n,
                                                   const double2 *__restrict__ B, long ldb,
                                                   int ncol, double2 *__restrict__ X, long ldx) {
  __shared__ double2 Tb[64][64];   // diagonal block, column-major: Tb[c][r] = T(b0 + r, b0 + c)
  __shared__ double rd[64];        // reciprocals of its diagonal
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  const bool live = j < ncol;   // every wave stays for the barriers
  double2 x[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int i = s * 64 + lane;
    double2 v = make_double2(0.0, 0.0);
    if (live && i < n) {
      if (MODE == 1) {
        const double2 m = B[j + (long)i * ldb];
        v = make_double2(m.x, -m.y);
      } else {
        v = B[i + (long)j * ldb];
      }
    }
    x[s] = v;
  }
  trsm_rounds<MODE, NS, 0>(x, T, ldt, n, lane, Tb, rd);
  if (!live) return;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int i = s * 64 + lane;
    if (i < n) X[i + (long)j * ldx] = x[s];
  }
}

// ---------------------------------------------------------------- tridiagonalisation
// A (n x n Hermitian, full storage) = Q T Q^H, Q = H_0 ... H_{n-2},
// H_k = I - tau_k v_k v_k^H acting on rows k+1..n-1.  On return column k of A
// holds v_k in rows k+1..n-1 (v_k[k+1] = 1); tri = d[n] | e[n] | tau (double2)[n].
//
// Step k needs p = A22 v_k (A22 = rows / columns k+1..) and applies the
// rank-2 update A22 -= v w^H + w v^H.
//
// Householder vector of the column col[0..m) (col[0] the subdiagonal entry):
// tau, beta, and v written to col (v[0] = 1) and to vs.  Uniform in all NT
// threads of the workgroup.
template <int NT = kET>
__device__ void householder(double2 *col, int m, double2 *vs, double *red, double2 *t_out,
                            double *beta_out) {
  const int tid = threadIdx.x;
  // alpha is read before the barriers of the sum: thread 0 overwrites col[0]
  // with v[0] = 1 below, and a wave that read it only after the sum could
  // see that write
  const double2 alpha = col[0];
  double s = 0.0;
  for (int i = 1 + tid; i < m; i += NT) {
    const double2 v = col[i];
    s += v.x * v.x + v.y * v.y;
  }
  const double xn2 = block_sum<NT / 64>(s, red);
  double beta;
  double2 t = make_double2(0.0, 0.0), scale = make_double2(0.0, 0.0);
  if (xn2 == 0.0 && alpha.y == 0.0) {
    beta = alpha.x;
  } else {
    beta = -copysign(sqrt(alpha.x * alpha.x + alpha.y * alpha.y + xn2), alpha.x);
    t = make_double2((beta - alpha.x) / beta, -alpha.y / beta);
    const double2 ab = make_double2(alpha.x - beta, alpha.y);
    const double den = ab.x * ab.x + ab.y * ab.y;
    scale = make_double2(ab.x / den, -ab.y / den);   // 1 / (alpha - beta)
  }
  const bool refl = t.x != 0.0 || t.y != 0.0;
  for (int i = tid; i < m; i += NT) {
    const double2 v = i == 0 ? make_double2(1.0, 0.0) : (refl ? cmul(col[i], scale) : col[i]);
    vs[i] = v;
    col[i] = v;
  }
  *t_out = t;
  *beta_out = beta;
}

constexpr int kTU = 6;   // independent loads in flight per thread

// One pass over the m x m block U (columns 1..m-1, rows 1..m-1 of the
// trailing matrix of step k; element (i, j) at U[i + j*lda]):
//   if upd:  U(i, j) -= v_i conj(w_j) + w_i conj(v_j)   (stored back)
//   if vn:   part[grp * mm + (i - 1)] = sum over the thread's columns of U(i, j) vn_{j-1}
// Rows and columns 0 (column 0 was done separately) are skipped.
__device__ void fused_pass(double2 *U, long lda, int m, bool upd, const double2 *vs,
                           const double2 *ws, bool mv, const double2 *vn, double2 *part) {
  const int tid = threadIdx.x;
  const int mm = m - 1;
  if (mm <= 0) return;
  const int g = kET / mm;   // >= 1 (mm < kEMaxN)
  if (tid >= g * mm) return;
  const int r = tid % mm, grp = tid / mm;
  const int i = r + 1;
  const double2 vi = vs[i], wi = ws[i];
  double2 acc = make_double2(0.0, 0.0);
  int j = 1 + grp;
  for (; j + (kTU - 1) * g < m; j += kTU * g) {
    double2 a[kTU];
#pragma unroll
    for (int u = 0; u < kTU; ++u) a[u] = U[i + (long)(j + u * g) * lda];
#pragma unroll
    for (int u = 0; u < kTU; ++u) {
      const int jj = j + u * g;
      if (upd) {
        a[u] = csub(a[u], cadd(cmulc(vi, ws[jj]), cmulc(wi, vs[jj])));
        U[i + (long)jj * lda] = a[u];
      }
      if (mv) acc = cadd(acc, cmul(a[u], vn[jj - 1]));
    }
  }
  for (; j < m; j += g) {
    double2 a = U[i + (long)j * lda];
    if (upd) {
      a = csub(a, cadd(cmulc(vi, ws[j]), cmulc(wi, vs[j])));
      U[i + (long)j * lda] = a;
    }
    if (mv) acc = cadd(acc, cmul(a, vn[j - 1]));
  }
  if (mv) part[grp * mm + r] = acc;
}

// The whole reduction on one workgroup, the trailing matrix streamed from
// memory once per step (rank-2 update of step k fused with the product of
// step k+1): little device time in total, for solves that share the device.
__global__ __launch_bounds__(kET) void tridiag_kernel(double2 *A, long lda, int n, double *d,
                                                      double *e, double2 *tau,
                                                      const int *info_chol) {
  if (*info_chol != 0) return;
  __shared__ double2 vbuf[2][kEMaxN];   // v_k and v_{k+1}
  __shared__ double2 ps[kEMaxN];        // A22 v_k, then p, then w
  __shared__ double2 part[kET];
  __shared__ double red[kEW];
  const int tid = threadIdx.x;
  if (n == 1) {
    if (tid == 0) d[0] = A[0].x;
    return;
  }
  // step 0's reflector and its product A22 v_0 (a plain pass: no update)
  double2 t;
  double beta;
  householder(A + 1, n - 1, vbuf[0], red, &t, &beta);
  if (tid == 0) {
    d[0] = A[0].x;
    e[0] = beta;
    tau[0] = t;
  }
  __syncthreads();
  {
    // the pass skips row / column 0 of its block: hand it the whole A22 by
    // starting one row and column earlier (A11 corner of A)
    const int m = n - 1;
    // rows 0..m-1 of A22 times v: do row 0 and column 0 here too
    const double2 *a22 = A + lda + 1;
    const int g = kET / m;
    if (tid < g * m) {
      const int i = tid % m, grp = tid / m;
      double2 acc = make_double2(0.0, 0.0);
      int jj = grp;
      for (; jj + (kTU - 1) * g < m; jj += kTU * g) {
        double2 a[kTU];
#pragma unroll
        for (int u = 0; u < kTU; ++u) a[u] = a22[i + (long)(jj + u * g) * lda];
#pragma unroll
        for (int u = 0; u < kTU; ++u) acc = cadd(acc, cmul(a[u], vbuf[0][jj + u * g]));
      }
      for (; jj < m; jj += g) acc = cadd(acc, cmul(a22[i + (long)jj * lda], vbuf[0][jj]));
      part[tid] = acc;
    }
    __syncthreads();
    for (int i = tid; i < m; i += kET) {
      double2 acc = part[i];
      for (int q = 1; q < g; ++q) acc = cadd(acc, part[q * m + i]);
      ps[i] = acc;
    }
    __syncthreads();
  }
  int cur = 0;
  for (int k = 0; k + 1 < n; ++k) {
    const int m = n - k - 1;   // order of A22 of step k
    double2 *u = A + (long)(k + 1) * lda + (k + 1);   // A22 of step k, (0, 0) corner
    const double2 *vs = vbuf[cur];
    const bool refl = t.x != 0.0 || t.y != 0.0;
    if (refl) {
      // p = t A22 v, alpha2 = -1/2 t (p^H v), w = p + alpha2 v (in ps)
      double dr = 0.0, di = 0.0;
      for (int i = tid; i < m; i += kET) {
        const double2 p = cmul(t, ps[i]), v = vs[i];
        dr += p.x * v.x + p.y * v.y;
        di += p.x * v.y - p.y * v.x;
      }
      dr = block_sum(dr, red);
      di = block_sum(di, red);
      const double2 a2 = cscale(cmul(t, make_double2(dr, di)), -0.5);
      for (int i = tid; i < m; i += kET) ps[i] = cadd(cmul(t, ps[i]), cmul(a2, vs[i]));
      __syncthreads();
      // column 0 of A22 (column k+1 of A), rows 0..m-1
      for (int i = tid; i < m; i += kET)
        u[i] = csub(u[i], cadd(cmulc(vs[i], ps[0]), cmulc(ps[i], vs[0])));
      __syncthreads();
    }
    if (m == 1) {
      if (tid == 0) d[k + 1] = u[0].x;
      break;
    }
    // reflector of step k+1 from column k+1 below the diagonal
    double2 t1;
    double beta1;
    householder(u + 1, m - 1, vbuf[cur ^ 1], red, &t1, &beta1);
    if (tid == 0) {
      d[k + 1] = u[0].x;
      e[k + 1] = beta1;
      tau[k + 1] = t1;
    }
    __syncthreads();
    const bool refl1 = t1.x != 0.0 || t1.y != 0.0;
    // rest of step k's update fused with step k+1's product (rows / columns
    // 1..m-1 of this A22 are A22 of step k+1)
    fused_pass(u, lda, m, refl, vs, ps, refl1, vbuf[cur ^ 1], part);
    __syncthreads();
    if (refl1) {
      const int mm = m - 1, g = kET / mm;
      for (int i = tid; i < mm; i += kET) {
        double2 acc = part[i];
        for (int q = 1; q < g; ++q) acc = cadd(acc, part[q * mm + i]);
        ps[i] = acc;
      }
    }
    __syncthreads();
    t = t1;
    cur ^= 1;
  }
}

// The last orders of the reduction (m <= kTailN, the whole problem when it
// is that small): one workgroup with the trailing block in LDS, so nothing
// leaves LDS between steps.  Step k: reflector of column k, p = t A22 v
// (each thread a row and a quarter of the columns, partial sums added in a
// fixed order), alpha = -1/2 t (p^H v), w = p + alpha v, A22 -= v w^H + w v^H
// (both triangles).  On return the columns hold the reflectors as in the
// step kernel's part.
constexpr int kLT = 256;

// Leading steps of the same reduction while the trailing block is large: one
// launch per step over many workgroups, one wave per column of the trailing
// block (kSW columns per workgroup); tridiag_lds_kernel then reduces the last
// kTailN rows and columns as a problem of its own (after k0 steps the rest of
// the reduction is the reduction of the updated block A[k0:, k0:]).
//
// Launch k (k = -1 .. k0-1) applies step k's update A22 -= v w^H + w v^H
// (A22 = rows / columns k+1..n-1) to the columns its waves own, and forms
// step k+1's reflector v' (from column k+1) and product y' = A22' v' (A22' =
// rows / columns k+2..) for the next launch.  w needs the whole y of step k,
// and v' the updated column k+1: every workgroup forms both itself from the
// small vectors of the previous launch (the same arithmetic in each, hence
// the same values), so the launch boundary is the only synchronisation.  y'
// uses the Hermitian symmetry, (A22' v')_j = sum_i conj(A(i, j)) v'_i, so
// that a wave needs only its own column.  Launch -1 only forms v_0 and y_0.
// Scratch (double2, double-buffered by parity so that a launch never writes
// what it reads): vb[2][n] = v of a step, yb[2][n] = its y, cb[2][n] =
// column c of A (rows c..n-1) as the launch before left it, for c = k+1.
// Column k's reflector is written into A by the launch of step k, when no
// wave reads that column any more.
constexpr int kSW = 4;         // waves (columns) per workgroup of the step kernel
constexpr int kTailN = 64;     // order left to the one-workgroup kernel

template <int NS>   // register slots per lane: orders up to 64 NS
__global__ __launch_bounds__(64 * kSW) void tdstep_kernel(double2 *A, long lda, int n, int k,
                                                          int last, double *d, double *e,
                                                          double2 *tau, double2 *scr,
                                                          const int *info_chol) {
  if (*info_chol != 0) return;
  __shared__ double2 vs[NS * 64];   // v of step k
  __shared__ double2 ws[NS * 64];   // y of step k, then w
  __shared__ double2 cs[NS * 64];   // column k+1 (rows k+1..), then v' in cs[1..]
  __shared__ double red[2 * kSW];
  const int tid = threadIdx.x, lane = tid & 63;
  const int r0 = k + 1;            // first row / column of A22
  const int m = n - r0;            // its order
  double2 *vb = scr, *yb = scr + 2 * (long)n, *cb = scr + 4 * (long)n;
  const int col = blockIdx.x * kSW + (tid >> 6);   // this wave's column of A22
  const bool own = col < m;
  double2 *acol = A + (long)(r0 + col) * lda + r0;
  // the owned column first: its loads overlap the small vectors'
  double2 a[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int i = s * 64 + lane;
    a[s] = own && i < m ? acol[i] : make_double2(0.0, 0.0);
  }
  const double2 t = k >= 0 ? tau[k] : make_double2(0.0, 0.0);
  const bool refl = t.x != 0.0 || t.y != 0.0;
  const double2 *csrc = k >= 0 ? cb + (long)(r0 & 1) * n : A;
  for (int i = tid; i < m; i += 64 * kSW) {
    if (k >= 0) {
      vs[i] = vb[(long)(k & 1) * n + i];
      ws[i] = yb[(long)(k & 1) * n + i];
    }
    cs[i] = csrc[i];
  }
  __syncthreads();
  if (refl) {
    // p = t y, alpha = -1/2 t (p^H v), w = p + alpha v; then column k+1
    // less v w0^* + w v0^*.  Every thread forms w0 itself from y0 and v0,
    // read before the sum's barriers (thread 0 overwrites ws[0] with w0 below).
    const double2 y0 = ws[0], v0 = vs[0];
    double dr = 0.0, di = 0.0;
    for (int i = tid; i < m; i += 64 * kSW) {
      const double2 p = cmul(t, ws[i]), v = vs[i];
      dr += p.x * v.x + p.y * v.y;
      di += p.x * v.y - p.y * v.x;
    }
    const double2 pv = block_sum2<kSW>(dr, di, red);
    const double2 a2 = cscale(cmul(t, pv), -0.5);
    const double2 w0 = cadd(cmul(t, y0), cmul(a2, v0));
    for (int i = tid; i < m; i += 64 * kSW) {
      const double2 wi = cadd(cmul(t, ws[i]), cmul(a2, vs[i]));
      ws[i] = wi;
      cs[i] = csub(cs[i], cadd(cmulc(vs[i], w0), cmulc(wi, v0)));
    }
    __syncthreads();
  }
  double2 t1 = make_double2(0.0, 0.0);
  double beta1 = 0.0;
  if (!last) {
    householder<64 * kSW>(cs + 1, m - 1, cs + 1, red, &t1, &beta1);
    __syncthreads();
  }
  if (own) {
    if (refl) {
      const double2 vj = vs[col], wj = ws[col];
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const int i = s * 64 + lane;
        if (i < m) {
          a[s] = csub(a[s], cadd(cmulc(vs[i], wj), cmulc(ws[i], vj)));
          acol[i] = a[s];
        }
      }
    }
    if (!last && col >= 1) {
      double dr = 0.0, di = 0.0;   // conj(column) . v'
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const int i = s * 64 + lane;
        if (i >= 1 && i < m) {
          const double2 v = cs[i];
          dr += a[s].x * v.x + a[s].y * v.y;
          di += a[s].x * v.y - a[s].y * v.x;
        }
      }
      dr = wave_sum(dr);
      di = wave_sum(di);
      if (lane == 0) yb[(long)(r0 & 1) * n + col - 1] = make_double2(dr, di);
      if (col == 1) {
        double2 *cn = cb + (long)((r0 + 1) & 1) * n;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          const int i = s * 64 + lane;
          if (i >= 1 && i < m) cn[i - 1] = a[s];
        }
      }
    }
  }
  if (blockIdx.x == 0) {
    if (k >= 0)
      for (int i = tid; i < m; i += 64 * kSW) A[(long)k * lda + r0 + i] = vs[i];
    if (!last) {
      for (int i = tid; i + 1 < m; i += 64 * kSW) vb[(long)(r0 & 1) * n + i] = cs[1 + i];
      if (tid == 0) {
        d[r0] = cs[0].x;
        e[r0] = beta1;
        tau[r0] = t1;
      }
    }
  }
}

__global__ __launch_bounds__(kLT) void tridiag_lds_kernel(double2 *A, long lda, int m, double *d,
                                                          double *e, double2 *tau,
                                                          const int *info_chol) {
  if (*info_chol != 0) return;
  constexpr int G = kLT / kTailN;            // column groups of the product
  __shared__ double2 Al[kTailN][kTailN + 1];   // [column][row]
  __shared__ double2 vs[kTailN], ws[kTailN];
  __shared__ double2 part[G][kTailN];
  __shared__ double red[2 * (kLT / 64)];
  const int tid = threadIdx.x;
  for (int idx = tid; idx < m * m; idx += kLT) {
    const int r = idx % m, c = idx / m;
    Al[c][r] = A[r + (long)c * lda];
  }
  __syncthreads();
  for (int k = 0; k + 1 < m; ++k) {
    const int mm = m - k - 1;   // order of A22
    double2 t;
    double beta;
    householder<kLT>(&Al[k][k + 1], mm, vs, red, &t, &beta);
    if (tid == 0) {
      d[k] = Al[k][k].x;
      e[k] = beta;
      tau[k] = t;
    }
    __syncthreads();
    if (t.x == 0.0 && t.y == 0.0) continue;   // uniform
    {
      const int i = tid % kTailN, g = tid / kTailN;
      double2 acc = make_double2(0.0, 0.0);
      if (i < mm)
        for (int j = g; j < mm; j += G) acc = cadd(acc, cmul(Al[k + 1 + j][k + 1 + i], vs[j]));
      part[g][i] = acc;
    }
    __syncthreads();
    double dr = 0.0, di = 0.0;
    if (tid < mm) {
      double2 p = part[0][tid];
#pragma unroll
      for (int g = 1; g < G; ++g) p = cadd(p, part[g][tid]);
      p = cmul(t, p);
      ws[tid] = p;
      const double2 v = vs[tid];
      dr = p.x * v.x + p.y * v.y;
      di = p.x * v.y - p.y * v.x;
    }
    const double2 a2 = cscale(cmul(t, block_sum2<kLT / 64>(dr, di, red)), -0.5);
    if (tid < mm) ws[tid] = cadd(ws[tid], cmul(a2, vs[tid]));
    __syncthreads();
    for (int idx = tid; idx < mm * mm; idx += kLT) {
      const int i = idx % mm, j = idx / mm;
      double2 &a = Al[k + 1 + j][k + 1 + i];
      a = csub(a, cadd(cmulc(vs[i], ws[j]), cmulc(ws[i], vs[j])));
    }
    __syncthreads();
  }
  if (tid == 0) d[m - 1] = Al[m - 1][m - 1].x;
  for (int idx = tid; idx < m * m; idx += kLT) {
    const int r = idx % m, c = idx / m;
    A[r + (long)c * lda] = Al[c][r];
  }
}

// ---------------------------------------------------------------- tridiagonal eigenpairs
// Number of eigenvalues of the block [s, t) of T (split e) below x.
// 1/q from the hardware reciprocal estimate and two Newton steps (full
// double precision for |q| >= pivmin; the quotient e^2/q then stays below
// 1/DBL_MIN because pivmin >= DBL_MIN max(1, e^2))
__device__ __forceinline__ double recip(double q) {
  double r = __builtin_amdgcn_rcp(q);
  double e = fma(-q, r, 1.0);
  r = fma(r, e, r);
  e = fma(-q, r, 1.0);
  return fma(r, e, r);
}

// The recurrence is one dependent chain; its operands (LDS) are read a chunk
// of kSU steps ahead so that their latency stays off the chain.
constexpr int kSU = 8;
__device__ __forceinline__ int sturm_count(const double *d, const double *e2, int s, int t, double x,
                                           double pivmin) {
  int c = 0;
  double q = d[s] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  c += q < 0.0;
  int i = s + 1;
  double dn[kSU], en[kSU];
  if (i + kSU <= t) {
#pragma unroll
    for (int u = 0; u < kSU; ++u) {
      dn[u] = d[i + u];
      en[u] = e2[i - 1 + u];
    }
  }
  for (; i + kSU <= t; i += kSU) {
    double dc[kSU], ec[kSU];
#pragma unroll
    for (int u = 0; u < kSU; ++u) {
      dc[u] = dn[u];
      ec[u] = en[u];
    }
    if (i + 2 * kSU <= t) {
#pragma unroll
      for (int u = 0; u < kSU; ++u) {
        dn[u] = d[i + kSU + u];
        en[u] = e2[i + kSU - 1 + u];
      }
    }
#pragma unroll
    for (int u = 0; u < kSU; ++u) {
      q = dc[u] - x - ec[u] * recip(q);
      if (fabs(q) < pivmin) q = -pivmin;
      c += q < 0.0;
    }
  }
  for (; i < t; ++i) {
    q = d[i] - x - e2[i - 1] * recip(q);
    if (fabs(q) < pivmin) q = -pivmin;
    c += q < 0.0;
  }
  return c;
}

__device__ __forceinline__ double guard(double q, double pivmin) {
  return fabs(q) < pivmin ? -pivmin : q;
}

// deterministic start vector entry in [-1, 1) for row i of group member r
__device__ __forceinline__ double start_entry(int i, int r) {
  unsigned long long z = (unsigned long long)(i + 1) * 0x9E3779B97F4A7C15ull ^
                         (unsigned long long)(r + 1) * 0xC2B2AE3D27D4EB4Full;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

// Solve (T_b - sigma I) x = x in place with the pivoted LU (dl, dd, du, du2,
// piv) of length m; tiny pivots replaced by +-tiny.
__device__ void lu_solve(const double *dl, const double *dd, const double *du, const double *du2,
                         const double *piv, int m, double tiny, double *x) {
  for (int i = 0; i + 1 < m; ++i) {
    if (piv[i] != 0.0) {
      const double a = x[i], b = x[i + 1];
      x[i] = b;
      x[i + 1] = a - dl[i] * b;
    } else {
      x[i + 1] -= dl[i] * x[i];
    }
  }
  auto piv_d = [&](int i) {
    const double v = dd[i];
    return fabs(v) < tiny ? copysign(tiny, v) : v;
  };
  x[m - 1] /= piv_d(m - 1);
  if (m > 1) x[m - 2] = (x[m - 2] - du[m - 2] * x[m - 1]) / piv_d(m - 2);
  for (int i = m - 3; i >= 0; --i) x[i] = (x[i] - du[i] * x[i + 1] - du2[i] * x[i + 2]) / piv_d(i);
}

// Gram-Schmidt of the columns of one group (tasks g0 .. g0+cnt-1 in block
// order, Z columns zc[task]) by one wave: each column against the earlier
// ones, then normalised.
__device__ void wave_mgs(double *Z, int ldz, const int *zc, int g0, int cnt, int s, int t) {
  const int lane = threadIdx.x & 63;
  for (int r = 0; r < cnt; ++r) {
    double *zr = Z + (long)zc[g0 + r] * ldz;
    for (int rr = 0; rr < r; ++rr) {
      const double *zq = Z + (long)zc[g0 + rr] * ldz;
      double dp = 0.0;
      for (int i = s + lane; i < t; i += 64) dp += zq[i] * zr[i];
      dp = wave_sum(dp);
      for (int i = s + lane; i < t; i += 64) zr[i] -= dp * zq[i];
    }
    double nn = 0.0;
    for (int i = s + lane; i < t; i += 64) nn += zr[i] * zr[i];
    nn = wave_sum(nn);
    const double inv = nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
    for (int i = s + lane; i < t; i += 64) zr[i] *= inv;
  }
}

// The nb lowest eigenpairs of T (tri = d | e).  w[j] ascending, Z(:, j)
// (column-major, ldz >= n, real) orthonormal eigenvectors.  scr:
// eig_scratch_doubles(n) doubles.  info: 0, 1 (T not finite), 2 (fewer than
// nb eigenvalues found).  Two launches: PH = 0 over many workgroups finds the
// cut and the eigenvalues (each workgroup sets up T and the tasks itself, the
// same arithmetic in each, and bisects its share of the tasks), leaving the
// cut and the task eigenvalues in scr; PH = 1 (one workgroup) takes them and
// sorts, groups and forms the eigenvectors.
template <int PH, int KM>   // KM: largest order this instance takes (array sizes)
__global__ __launch_bounds__(kET) void trieig_kernel(const double *tri, int n, int nb, double *w,
                                                     double *Z, int ldz, double *scr, int *info,
                                                     const int *info_chol) {
  if (*info_chol != 0) return;
  if (PH == 1 && *info != 0) return;
  if (PH == 0 && blockIdx.x == 0 && threadIdx.x == 0) *info = 0;
  double *tlam_g = scr + 7L * n * n;   // task eigenvalues, then the cut
  double *xcut_g = tlam_g + KM;
  __shared__ double sd[KM], se[KM], se2[KM];
  __shared__ int bst[KM + 1];    // block starts
  __shared__ int bof[KM + 1];    // first task of each block
  __shared__ double tlam[KM];    // task eigenvalue
  __shared__ int tblk[KM], tpos[KM];   // task block, sorted position
  __shared__ int gdeg[KM], gclo[KM];   // first task of the task's degenerate / close group
  constexpr int kSK = KM > kET ? KM : kET;   // sort keys (tasks <= KM <= kSK)
  static_assert(KM <= 2 * kET, "the sort handles at most two keys per thread");
  __shared__ double key[kSK];
  __shared__ int kid[kSK];
  __shared__ double red[kEW];
  __shared__ int sh_i[4];            // nblk, ntask, first qualifying multisection point
  __shared__ double sh_d[2];         // multisection bracket
  const int tid = threadIdx.x;
  const int wid = tid >> 6, lane = tid & 63;
  for (int i = tid; i < n; i += kET) {
    sd[i] = tri[i];
    se[i] = i + 1 < n ? tri[n + i] : 0.0;
  }
  __syncthreads();
  double md = 0.0, me = 0.0;
  for (int i = tid; i < n; i += kET) {
    md = fmax(md, fabs(sd[i]));
    me = fmax(me, fabs(se[i]));
  }
  md = block_max(md, red);
  me = block_max(me, red);
  const double tnorm = md + 2.0 * me;
  if (!isfinite(tnorm) || nb < 1 || nb > n) {
    if (PH == 0 && blockIdx.x == 0 && tid == 0) *info = 1;
    return;
  }
  // split where |e| is negligible
  double e2max = 0.0;
  for (int i = tid; i < n; i += kET) {
    if (fabs(se[i]) <= kEps * tnorm) se[i] = 0.0;
    se2[i] = se[i] * se[i];
    e2max = fmax(e2max, se2[i]);
  }
  e2max = block_max(e2max, red);
  const double pivmin = kTiny * fmax(1.0, e2max);
  double lo = 1e300, hi = -1e300;
  for (int i = tid; i < n; i += kET) {
    const double r = fabs(se[i]) + (i > 0 ? fabs(se[i - 1]) : 0.0);
    lo = fmin(lo, sd[i] - r);
    hi = fmax(hi, sd[i] + r);
  }
  const double gl = block_min(lo, red) - 2.0 * kEps * tnorm - pivmin;
  const double gu = block_max(hi, red) + 2.0 * kEps * tnorm + pivmin;
  if (tid == 0) {
    int nbk = 0;
    bst[nbk++] = 0;
    for (int i = 0; i + 1 < n; ++i)
      if (se[i] == 0.0) bst[nbk++] = i + 1;
    bst[nbk] = n;
    sh_i[0] = nbk;
  }
  __syncthreads();
  const int nblk = sh_i[0];
  // bracket the nb-th eigenvalue: count(lo) <= nb - 1 < count(hi)
  if (tid == 0) {
    sh_d[0] = gl;
    sh_d[1] = gu;
  }
  __syncthreads();
  if (PH == 0) {
    // (stops once exactly nb eigenvalues lie below the upper end: the cut then
    // selects the nb wanted ones and nothing else)
    int cup = n;   // count at the upper end
    for (int round = 0; round < 8; ++round) {
      const double a = sh_d[0], b = sh_d[1];
      if (b - a <= 2.0 * kEps * tnorm || cup == nb) break;   // uniform
      const double x = a + (b - a) * (double)(tid + 1) / (double)(kET + 1);
      const int c = sturm_count(sd, se2, 0, n, x, pivmin);
      if (tid == 0) sh_i[2] = kET;
      __syncthreads();
      if (c > nb - 1) atomicMin(&sh_i[2], tid);   // first point above: order-free minimum
      __syncthreads();
      const int f = sh_i[2];
      if (tid == f) sh_i[3] = c;
      __syncthreads();
      if (f < kET) cup = sh_i[3];
      if (tid == 0) {
        const double xf = f < kET ? a + (b - a) * (double)(f + 1) / (double)(kET + 1) : b;
        const double xl = f > 0 ? a + (b - a) * (double)f / (double)(kET + 1) : a;
        sh_d[0] = xl;
        sh_d[1] = xf;
      }
      __syncthreads();
    }
  }
  const double xcut = PH == 0 ? sh_d[1] + 4.0 * kEps * tnorm + pivmin : *xcut_g;
  if (PH == 0 && blockIdx.x == 0 && tid == 0) *xcut_g = xcut;
  // eigenvalues of each block below the cut -> tasks
  for (int b = tid; b < nblk; b += kET) bof[b] = sturm_count(sd, se2, bst[b], bst[b + 1], xcut, pivmin);
  __syncthreads();
  if (tid == 0) {
    int acc = 0;
    for (int b = 0; b < nblk; ++b) {
      const int c = bof[b];
      bof[b] = acc;
      acc += c;
    }
    bof[nblk] = acc;
    sh_i[1] = acc;
  }
  __syncthreads();
  const int ntask = sh_i[1];
  if (ntask < nb || ntask > KM) {
    if (PH == 0 && blockIdx.x == 0 && tid == 0) *info = 2;
    return;
  }
  for (int b = tid; b < nblk; b += kET)
    for (int t = bof[b]; t < bof[b + 1]; ++t) tblk[t] = b;
  __syncthreads();
  if (PH == 0) {
    // Start brackets.  When T is one block (the usual case) a task's local
    // index is its global one, and one pass of kET Sturm counts over
    // [gl, xcut] gives every task a bracket 1/(kET + 1) of that range wide
    // (count at the lower end <= index < count at the upper end).
    if (nblk == 1) {
      kid[tid] = sturm_count(sd, se2, 0, n,
                             gl + (xcut - gl) * (double)(tid + 1) / (double)(kET + 1), pivmin);
      __syncthreads();
    }
    // Multisection, G lanes per task over all workgroups (the lanes of a
    // group adjacent in one wave; G a power of two <= 64): each round the
    // group's G points split the bracket into G + 1 parts and the first
    // point whose count exceeds the task's index becomes the upper end.
    // Every lane takes part in every round (one wave-wide ballot carries
    // the groups' comparisons), finished groups unchanged.
    const int gthreads = gridDim.x * kET;
    int G = 64;
    while (G > 1 && G * ntask > gthreads) G >>= 1;
    const int gt = blockIdx.x * kET + tid;
    // (more tasks than lanes, one lane each: rounds of gthreads tasks)
    for (int tb = 0; tb < ntask; tb += gthreads / G) {
    const int task = tb + gt / G, sub = gt % G;
    const bool real_task = task < ntask;
    const int b = real_task ? tblk[task] : 0;
    const int s = bst[b], t = bst[b + 1], loc = real_task ? task - bof[b] : 0;
    double a = gl, c = xcut;
    if (nblk == 1 && real_task) {
      int lo = 0, hi = kET;   // first point with count > loc (kET: none)
      while (lo < hi) {
        const int md = (lo + hi) >> 1;
        if (kid[md] > loc) hi = md;
        else lo = md + 1;
      }
      if (lo < kET) c = gl + (xcut - gl) * (double)(lo + 1) / (double)(kET + 1);
      if (lo > 0) a = gl + (xcut - gl) * (double)lo / (double)(kET + 1);
    }
    const int base = lane - sub;   // the group's first lane
    for (int it = 0; it < 160; ++it) {
      const double x0 = a + (c - a) / (double)(G + 1);
      const double xl = a + (c - a) * (double)G / (double)(G + 1);
      const bool act = real_task && c - a > 2.0 * kEps * tnorm && x0 > a && xl < c;
      if (!__any(act)) break;
      const double x = a + (c - a) * (double)(sub + 1) / (double)(G + 1);
      const unsigned long long above =
          __ballot(sturm_count(sd, se2, s, t, x, pivmin) > loc);
      // first point of the group above the index (G: none)
      const unsigned long long mine = (above >> base) & (G == 64 ? ~0ull : ((1ull << G) - 1));
      const int first = mine ? __builtin_ctzll(mine) : G;
      if (act) {
        const double na = first > 0 ? a + (c - a) * (double)first / (double)(G + 1) : a;
        const double nc = first < G ? a + (c - a) * (double)(first + 1) / (double)(G + 1) : c;
        a = na;
        c = nc;
      }
    }
    if (real_task && sub == 0) tlam_g[task] = 0.5 * (a + c);
    }
    return;
  }
  for (int i = tid; i < ntask; i += kET) tlam[i] = tlam_g[i];
  __syncthreads();
  // sort (value, task) pairs by value, task index breaking ties (bitonic over
  // KS keys, a power of two >= ntask)
  const int KS = ntask <= kET ? kET : kSK;
  for (int e = tid; e < KS; e += kET) {
    key[e] = e < ntask ? tlam[e] : INFINITY;
    kid[e] = e;
  }
  for (int e = tid; e < KM; e += kET) tpos[e] = nb;   // not selected unless sorted below nb
  __syncthreads();
  for (int size = 2; size <= KS; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int e = tid; e < KS; e += kET) {
        const int p = e ^ stride;
        if (p > e) {
          const bool up = (e & size) == 0;
          const double ka = key[e], kb = key[p];
          const int ia = kid[e], ib = kid[p];
          const bool gt = ka > kb || (ka == kb && ia > ib);
          if (gt == up) {
            key[e] = kb;
            key[p] = ka;
            kid[e] = ib;
            kid[p] = ia;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int e = tid; e < ntask; e += kET)
    if (kid[e] < ntask) tpos[kid[e]] = e;
  __syncthreads();
  // groups within a block among the selected tasks (tasks of one block are
  // consecutive and ascending)
  for (int task = tid; task < ntask; task += kET)
    if (tpos[task] < nb) {
      int g = task;
      while (g > bof[tblk[task]] && tpos[g - 1] < nb && tlam[g] - tlam[g - 1] <= kDegRel * tnorm)
        --g;
      gdeg[task] = g;
      g = task;
      while (g > bof[tblk[task]] && tpos[g - 1] < nb && tlam[g] - tlam[g - 1] <= kCloseRel * tnorm)
        --g;
      gclo[task] = g;
    }
  __syncthreads();
  const long ls = n;   // per-task scratch stride
  const long kTS = ls;                  // row stride of the pivot arrays (tasks <= n)
  double *twp = scr;                    // [n][task] D+ (top-down pivots)
  double *twm = scr + ls * ls;          // [n][task] D- (bottom-up pivots)
  double *lu = scr + 2 * ls * ls;       // [task][5 n] pivoted LU (group leaders)
  const double dtiny = kEps * tnorm;
  auto in_group = [&](int t) {   // selected task t is in a degenerate group of >= 2
    return gdeg[t] != t || (t + 1 < bof[tblk[t] + 1] && tpos[t + 1] < nb && gdeg[t + 1] == t);
  };
  // pass 1: twisted vectors (singletons); LU of the degenerate groups (leaders)
  for (int task = tid; task < ntask; task += kET) {
    if (tpos[task] >= nb) continue;
    const int b = tblk[task], s = bst[b], t = bst[b + 1], m = t - s;
    double *z = Z + (long)tpos[task] * ldz;
    const double lam = tlam[task];
    if (in_group(task))
      for (int i = 0; i < n; ++i)
        if (i < s || i >= t) z[i] = 0.0;
    if (!in_group(task)) {
      if (m == 1) {
        for (int i = 0; i < n; ++i) z[i] = i == s ? 1.0 : 0.0;
      } else {
        // pivots stored row-major over the tasks ([i][task]): the lanes of a
        // wave touch consecutive addresses at each step
        // (the top-down and bottom-up recurrences interleaved: two
        // independent chains)
        double *dp = twp + task, *dm = twm + task;
        double qp = sd[s] - lam, qm = sd[t - 1] - lam;
        dp[0] = qp;
        dm[(m - 1) * kTS] = qm;
        for (int i = 1; i < m; ++i) {
          const int j = m - 1 - i;
          qp = sd[s + i] - lam - se2[s + i - 1] / guard(qp, pivmin);
          qm = sd[s + j] - lam - se2[s + j] / guard(qm, pivmin);
          dp[i * kTS] = qp;
          dm[j * kTS] = qm;
        }
        int r = 0;
        double best = INFINITY;
#pragma unroll 8
        for (int i = 0; i < m; ++i) {
          const double gm = fabs(dp[i * kTS] + dm[i * kTS] - (sd[s + i] - lam));
          if (gm < best) {
            best = gm;
            r = i;
          }
        }
        // the unnormalised vector (entry r = 1) replaces the pivots it is
        // formed from (coalesced), and goes to Z once, normalised, with the
        // zeros outside the block (one strided pass)
        double zc = 1.0, nn = 1.0;
#pragma unroll 8
        for (int i = r - 1; i >= 0; --i) {
          zc = -se[s + i] / guard(dp[i * kTS], pivmin) * zc;
          dp[i * kTS] = zc;
          nn += zc * zc;
        }
        zc = 1.0;
#pragma unroll 8
        for (int i = r; i + 1 < m; ++i) {
          zc = -se[s + i] / guard(dm[(i + 1) * kTS], pivmin) * zc;
          dm[(i + 1) * kTS] = zc;
          nn += zc * zc;
        }
        const double inv = 1.0 / sqrt(nn);
#pragma unroll 8
        for (int i = 0; i < n; ++i) {
          const int li = i - s;
          const double v = li < 0 || li >= m ? 0.0 : li < r ? dp[li * kTS] : li == r ? 1.0 : dm[li * kTS];
          z[i] = v * inv;
        }
      }
    } else if (gdeg[task] == task) {
      // pivoted LU of T_b - lam I (LAPACK gttrf order)
      double *dl = lu + (long)task * 5 * ls, *dd = dl + ls, *du = dd + ls, *du2 = du + ls,
             *pv = du2 + ls;
      for (int i = 0; i < m; ++i) dd[i] = sd[s + i] - lam;
      for (int i = 0; i + 1 < m; ++i) {
        dl[i] = se[s + i];
        du[i] = se[s + i];
        pv[i] = 0.0;
      }
      for (int i = 0; i + 2 < m; ++i) du2[i] = 0.0;
      for (int i = 0; i + 1 < m; ++i) {
        if (fabs(dd[i]) >= fabs(dl[i])) {
          const double f = dd[i] != 0.0 ? dl[i] / dd[i] : 0.0;
          dl[i] = f;
          dd[i + 1] -= f * du[i];
        } else {
          const double f = dd[i] / dl[i];
          dd[i] = dl[i];
          dl[i] = f;
          const double tmp = du[i];
          du[i] = dd[i + 1];
          dd[i + 1] = tmp - f * dd[i + 1];
          if (i + 2 < m) {
            du2[i] = du[i + 1];
            du[i + 1] = -f * du[i + 1];
          }
          pv[i] = 1.0;
        }
      }
    }
  }
  __syncthreads();
  // passes 2-5: two sweeps of inverse iteration for the degenerate groups,
  // each followed by Gram-Schmidt within the group (one wave per group)
  for (int sweep = 0; sweep < 2; ++sweep) {
    for (int task = tid; task < ntask; task += kET) {
      if (tpos[task] >= nb || !in_group(task)) continue;
      const int b = tblk[task], s = bst[b], t = bst[b + 1], m = t - s;
      const int ld0 = gdeg[task];
      const double *dl = lu + (long)ld0 * 5 * ls, *dd = dl + ls, *du = dd + ls, *du2 = du + ls,
                   *pv = du2 + ls;
      double *z = Z + (long)tpos[task] * ldz + s;
      if (sweep == 0)
        for (int i = 0; i < m; ++i) z[i] = start_entry(i, task - ld0);
      lu_solve(dl, dd, du, du2, pv, m, dtiny, z);
      double nn = 0.0;
      for (int i = 0; i < m; ++i) nn += z[i] * z[i];
      const double inv = nn > 0.0 && isfinite(nn) ? 1.0 / sqrt(nn) : 0.0;
      for (int i = 0; i < m; ++i) z[i] *= inv;
    }
    __syncthreads();
    // group leaders, dealt to waves in task order
    for (int t0 = 0; t0 < ntask; ++t0) {
      if (t0 % kEW != wid || tpos[t0] >= nb || gdeg[t0] != t0 || !in_group(t0)) continue;
      int cnt = 1;
      while (t0 + cnt < bof[tblk[t0] + 1] && tpos[t0 + cnt] < nb && gdeg[t0 + cnt] == t0) ++cnt;
      wave_mgs(Z, ldz, tpos, t0, cnt, bst[tblk[t0]], bst[tblk[t0] + 1]);
    }
    __syncthreads();
  }
  // close groups: Gram-Schmidt in block order (one wave per group)
  for (int t0 = 0; t0 < ntask; ++t0) {
    if (t0 % kEW != wid || tpos[t0] >= nb || gclo[t0] != t0) continue;
    int cnt = 1;
    while (t0 + cnt < bof[tblk[t0] + 1] && tpos[t0 + cnt] < nb && gclo[t0 + cnt] == t0) ++cnt;
    if (cnt > 1) wave_mgs(Z, ldz, tpos, t0, cnt, bst[tblk[t0]], bst[tblk[t0] + 1]);
  }
  for (int task = tid; task < ntask; task += kET)
    if (tpos[task] < nb) w[tpos[task]] = tlam[task];
  (void)lane;
  if (tid == 0) *info = 0;
}

// ---------------------------------------------------------------- back-transformation
constexpr int kTK = 8;   // reflectors staged per chunk

// Zc(:, j) = Q Zt(:, j) = H_0 (H_1 ( ... H_{n-2} Zt(:, j))), one wave per
// column; the four waves of a workgroup share the reflectors, staged through
// LDS kTK at a time with the next chunk's loads in flight.
template <int NS>   // register slots per lane: orders up to 64 NS
__global__ __launch_bounds__(256) void backtr_kernel(const double2 *__restrict__ A, long lda, int n,
                                                     const double *__restrict__ tri,
                                                     const double *__restrict__ Zt, int ldz,
                                                     int nb, double2 *__restrict__ Zc, long ldc,
                                                     const int *info_chol, const int *info_eig) {
  if (*info_chol != 0 || *info_eig != 0) return;
  constexpr int TK = NS <= 16 ? kTK : 2;   // reflectors per chunk (LDS, registers)
  __shared__ double2 Vs[TK][NS * 64];
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  const bool live = j < nb;   // every wave stays for the barriers
  const double2 *tau = reinterpret_cast<const double2 *>(tri + 2 * n);
  double2 z[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int i = s * 64 + lane;
    z[s] = make_double2(live && i < n ? Zt[i + (long)j * ldz] : 0.0, 0.0);
  }
  // reflectors k = kl .. kh (rows > kl) in descending chunks, the next
  // chunk's loads in flight during the current one's reflectors
  constexpr int NPF = TK * NS * 64 / 256;
  double2 pf[NPF];
  auto fetch = [&](int kh) {
    const int kl = max(0, kh - TK + 1), rows = n - (kl + 1);
#pragma unroll
    for (int u = 0; u < NPF; ++u) {
      const int idx = threadIdx.x + u * 256;
      const int c = idx / rows, i = kl + 1 + idx % rows;
      pf[u] = idx < (kh - kl + 1) * rows ? A[i + (long)(kl + c) * lda] : make_double2(0.0, 0.0);
    }
  };
  const int top = n - 2;
  if (top >= 0) fetch(top);
  for (int kh = top; kh >= 0; kh -= TK) {
    const int kl = max(0, kh - TK + 1);
    __syncthreads();
    {
      const int rows = n - (kl + 1);
#pragma unroll
      for (int u = 0; u < NPF; ++u) {
        const int idx = threadIdx.x + u * 256;
        const int c = idx / rows, i = kl + 1 + idx % rows;
        if (idx < (kh - kl + 1) * rows) Vs[c][i] = pf[u];
      }
    }
    __syncthreads();
    if (kh - TK >= 0) fetch(kh - TK);
    for (int k = kh; k >= kl; --k) {
      const double2 t = tau[k];
      if (t.x == 0.0 && t.y == 0.0) continue;
      const double2 *v = Vs[k - kl];
      double dr = 0.0, di = 0.0;   // v^H z
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const int i = s * 64 + lane;
        if (i > k && i < n) {
          const double2 vi = v[i];
          dr += vi.x * z[s].x + vi.y * z[s].y;
          di += vi.x * z[s].y - vi.y * z[s].x;
        }
      }
      dr = wave_sum(dr);
      di = wave_sum(di);
      const double2 c = cmul(t, make_double2(dr, di));
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const int i = s * 64 + lane;
        if (i > k && i < n) z[s] = csub(z[s], cmul(c, v[i]));
      }
    }
  }
  if (!live) return;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int i = s * 64 + lane;
    if (i < n) Zc[i + (long)j * ldc] = z[s];
  }
}

}  // namespace

size_t eig_scratch_doubles(int n) { return (size_t)7 * n * n + kEMaxN + 8; }

hipError_t launch_chol(double2 *S, long ld, int n, int *info, double *scr, bool wide,
                       hipStream_t s) {
  if (n < 1 || n > kEMaxN) return hipErrorInvalidValue;
  if ((!wide || n <= kCholOneWG) && n <= kCholMaxN) {
    hipLaunchKernelGGL(chol_kernel, dim3(1), dim3(kET), 0, s, S, ld, n, info);
    return hipGetLastError();
  }
  double2 *w = reinterpret_cast<double2 *>(scr);
  for (int jb = 0; jb < n; jb += kCB) {
    const int mt = max(0, n - jb - kCB);
    const int t = (mt + kCT - 1) / kCT;
    hipLaunchKernelGGL(cholp_kernel, dim3(max(1, t * (t + 1) / 2)), dim3(256), 0, s, S, ld, n, jb,
                       w, info);
  }
  return hipGetLastError();
}

hipError_t launch_trsm(int mode, const double2 *T, long ldt, int n, const double2 *B, long ldb,
                       int ncol, double2 *X, long ldx, hipStream_t s) {
  if (n < 1 || n > kEMaxN || ncol < 1) return hipErrorInvalidValue;
  const dim3 grid((ncol + 3) / 4);
  auto go = [&](auto kern) {
    hipLaunchKernelGGL(kern, grid, dim3(256), 0, s, T, ldt, n, B, ldb, ncol, X, ldx);
  };
  if (n <= 512) {
    if (mode == 0) go(trsm_kernel<0, 8>);
    else if (mode == 1) go(trsm_kernel<1, 8>);
    else go(trsm_kernel<2, 8>);
  } else if (n <= 1024) {
    if (mode == 0) go(trsm_kernel<0, 16>);
    else if (mode == 1) go(trsm_kernel<1, 16>);
    else go(trsm_kernel<2, 16>);
  } else {
    if (mode == 0) go(trsm_kernel<0, 32>);
    else if (mode == 1) go(trsm_kernel<1, 32>);
    else go(trsm_kernel<2, 32>);
  }
  return hipGetLastError();
}

hipError_t launch_tridiag(double2 *A, long lda, int n, double *tri, double *scr,
                          const int *info_chol, bool wide, hipStream_t s) {
  if (n < 1 || n > kEMaxN) return hipErrorInvalidValue;
  double *d = tri, *e = tri + n;
  double2 *tau = reinterpret_cast<double2 *>(tri + 2 * n);
  if (!wide && n > kTailN && n <= kET) {   // (its row x column-group layout needs n <= kET)
    hipLaunchKernelGGL(tridiag_kernel, dim3(1), dim3(kET), 0, s, A, lda, n, d, e, tau, info_chol);
    return hipGetLastError();
  }
  const int k0 = n > kTailN ? n - kTailN : 0;   // steps taken by the step kernel
  if (k0 > 0) {
    double2 *w = reinterpret_cast<double2 *>(scr);
    for (int k = -1; k < k0; ++k) {
      const int m = n - k - 1;
      const dim3 grid((m + kSW - 1) / kSW), blk(64 * kSW);
      const int last = k == k0 - 1 ? 1 : 0;
      if (n <= 512)
        hipLaunchKernelGGL(tdstep_kernel<8>, grid, blk, 0, s, A, lda, n, k, last, d, e, tau, w,
                           info_chol);
      else if (n <= 1024)
        hipLaunchKernelGGL(tdstep_kernel<16>, grid, blk, 0, s, A, lda, n, k, last, d, e, tau, w,
                           info_chol);
      else
        hipLaunchKernelGGL(tdstep_kernel<32>, grid, blk, 0, s, A, lda, n, k, last, d, e, tau, w,
                           info_chol);
    }
  }
  hipLaunchKernelGGL(tridiag_lds_kernel, dim3(1), dim3(kLT), 0, s, A + k0 + (long)k0 * lda, lda,
                     n - k0, d + k0, e + k0, tau + k0, info_chol);
  return hipGetLastError();
}

hipError_t launch_trieig(const double *tri, int n, int nb, double *w, double *Z, int ldz,
                         double *scr, int *info, const int *info_chol, bool wide, hipStream_t s) {
  if (n < 1 || n > kEMaxN || nb < 1 || nb > n || ldz < n) return hipErrorInvalidValue;
  // eigenvalues on about 64 lanes per wanted one, then the vectors
  const int g = wide ? max(1, min(32, (nb * 64 + kET - 1) / kET)) : 1;
  // (instances sized for the order: the 2 048-task arrays measured 20% slower
  // on orders <= 512)
  auto go = [&](auto k0, auto k1) {
    hipLaunchKernelGGL(k0, dim3(g), dim3(kET), 0, s, tri, n, nb, w, Z, ldz, scr, info, info_chol);
    hipLaunchKernelGGL(k1, dim3(1), dim3(kET), 0, s, tri, n, nb, w, Z, ldz, scr, info, info_chol);
  };
  if (n <= 512) go(trieig_kernel<0, 512>, trieig_kernel<1, 512>);
  else if (n <= 1024) go(trieig_kernel<0, 1024>, trieig_kernel<1, 1024>);
  else go(trieig_kernel<0, kEMaxN>, trieig_kernel<1, kEMaxN>);
  return hipGetLastError();
}

hipError_t launch_backtr(const double2 *A, long lda, int n, const double *tri, const double *Zt,
                         int ldz, int nb, double2 *Zc, long ldc, const int *info_chol,
                         const int *info_eig, hipStream_t s) {
  if (n < 1 || n > kEMaxN || nb < 1) return hipErrorInvalidValue;
  const dim3 grid((nb + 3) / 4);
  if (n <= 512)
    hipLaunchKernelGGL(backtr_kernel<8>, grid, dim3(256), 0, s, A, lda, n, tri, Zt, ldz, nb, Zc,
                       ldc, info_chol, info_eig);
  else if (n <= 1024)
    hipLaunchKernelGGL(backtr_kernel<16>, grid, dim3(256), 0, s, A, lda, n, tri, Zt, ldz, nb, Zc,
                       ldc, info_chol, info_eig);
  else
    hipLaunchKernelGGL(backtr_kernel<32>, grid, dim3(256), 0, s, A, lda, n, tri, Zt, ldz, nb, Zc,
                       ldc, info_chol, info_eig);
  return hipGetLastError();
}

}  // namespace qeh
