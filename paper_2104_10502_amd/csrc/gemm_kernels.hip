// Complex matrix products on the MFMA units, and the D scaling of the
// projector coefficients.
//
// Uses: the pseudopotential contribution of H (becp = beta^H psi, ps = D becp,
// hpsi += beta ps), which the paper lists among the ported Hamiltonian
// kernels, and the Rayleigh-Ritz reductions / Ritz rotations of the Davidson
// solver, which the paper runs through GPU BLAS (section "Evolution of the
// GPU-enabled version").
//
// A complex product is three real MFMA products on planar (re, im) tiles
// (Gauss's three-multiplication form):
//   P1 += Ar Br,   P2 += Ai Bi,   P3 += (Ar + Ai)(Br + Bi),
//   Cr = P1 - P2,  Ci = P3 - P1 - P2.
// The operand sums are formed in registers after the LDS reads.  The form is
// normwise stable; its rounding error is a small constant multiple of that of
// the four-product form (Cr = Ar Br - Ai Bi, Ci = Ar Bi + Ai Br), and it issues
// a quarter fewer MFMAs.  The FP64 instances are held to three waves per SIMD
// (their third accumulator set would otherwise push them to two).
// Two cheaper forms serve the Gamma-point projections (RM = 1: only the real
// part of C is wanted, Cr = P1 - P2; RM = 2: A is real, Cr = sum Ar Br and
// Ci = sum Ar Bi): two MFMA products per step instead of three.
// WGM x WGN waves (64 * WGM * WGN threads); each wave owns a
// (BM/WGM) x (BN/WGN) block of C built from 16 x 16 x 4 MFMA tiles.  Long K is
// split into fixed chunks whose partial results are summed in double by a
// separate kernel in a fixed order (deterministic, no atomics).
#include <algorithm>

#include "cplx.h"
#include "qeh_internal.h"

namespace qeh {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

// Accumulator of one BS x BS block: BS = 16 (f32 or f64, k = 4 per
// instruction) or 32 (f32 only, k = 2 per instruction; on this chip the
// 32 x 32 f32 instruction sustains close to the matrix peak, the 16 x 16 one
// about 0.85 of it).
template <typename R, int BS> struct acc_of;
template <> struct acc_of<float, 16> { using type = floatx4; };
template <> struct acc_of<float, 32> { using type = floatx16; };
template <> struct acc_of<double, 16> { using type = doublex4; };

__device__ __forceinline__ void mfma(float a, float b, floatx4 &c) {
  c = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ void mfma(float a, float b, floatx16 &c) {
  c = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ void mfma(double a, double b, doublex4 &c) {
  c = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Operand load: element of type T (double2/float2) -> compute type R, conj.
template <typename R, typename T>
__device__ __forceinline__ void ld_elem(const T *p, bool valid, bool cj, R &re, R &im) {
  if (valid) {
    const T v = *p;
    re = static_cast<R>(v.x);
    im = cj ? -static_cast<R>(v.y) : static_cast<R>(v.y);
  } else {
    re = R(0);
    im = R(0);
  }
}

template <typename T> __device__ __forceinline__ T zero_of() {
  T z;
  z.x = 0;
  z.y = 0;
  return z;
}
template <> __device__ __forceinline__ float zero_of<float>() { return 0.f; }

// real and imaginary parts of an operand element (a real element: imaginary 0)
template <typename R, typename T> __device__ __forceinline__ R re_of(const T &v) {
  return static_cast<R>(v.x);
}
template <typename R, typename T> __device__ __forceinline__ R im_of(const T &v) {
  return static_cast<R>(v.y);
}
template <> __device__ __forceinline__ float re_of<float, float>(const float &v) { return v; }
template <> __device__ __forceinline__ float im_of<float, float>(const float &v) { return 0.f; }

// One workgroup: a BM x BN tile of C over the K slice [kbeg, kend).  Global
// tiles are prefetched into registers while the MFMAs consume the LDS copy of
// the previous slice (two LDS buffers, one barrier per slice).
template <typename R, typename TA, typename TB, typename TC, int BMODE, int BM, int BN, int BK,
          int RM, int WGM, int WGN, int BS, int WPE>
__global__ __launch_bounds__(64 * WGM * WGN)
__attribute__((amdgpu_waves_per_eu(WPE > 0 ? WPE : (sizeof(R) == 8 ? 3 : 1))))
void cgemm_kernel(
    const TA *__restrict__ A, long lda, const TB *__restrict__ B, long ldb, TC *__restrict__ C,
    long ldc, int M, int N, int K, int conjA, int conjB, int accumulate, int kchunk,
    long split_stride, int tiles_m, int tiles_n, int ntiles, int per_xcd) {
  using ACC = typename acc_of<R, BS>::type;
  constexpr int NACC = BS * BS / 64;   // accumulator entries per lane
  constexpr int KS = BS == 32 ? 2 : 4;   // k per instruction
  static_assert(BK % KS == 0, "K slice / instruction k mismatch");
  constexpr int kGT = 64 * WGM * WGN;
  constexpr int BKP = BK + 1;
  constexpr int TM = BM / (BS * WGM);
  constexpr int TN = BN / (BS * WGN);
  constexpr int NA = BM * BK / kGT;
  constexpr int NB = BN * BK / kGT;
  static_assert(TM * BS * WGM == BM && TN * BS * WGN == BN, "tile / wave mismatch");
  static_assert(NA * kGT == BM * BK && NB * kGT == BN * BK, "tile / thread mismatch");
  __shared__ R As[2][2][BM * BKP];   // [buffer][re, im]
  __shared__ R Bs[2][2][BN * BKP];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm0 = (wave / WGN) * (BM / WGM);
  const int wn0 = (wave % WGN) * (BN / WGN);
  // Workgroup ids are dealt round-robin to the 8 XCDs (each with its own L2);
  // the remap gives each XCD a contiguous run of (m tile fastest, n tile,
  // K slice), so tiles that read the same operand rows run on one XCD
  // back to back.
  const int id = blockIdx.x;
  const int logical = (id & 7) * per_xcd + (id >> 3);
  if (logical >= ntiles) return;
  const int mt = logical % tiles_m;
  const int nt = (logical / tiles_m) % tiles_n;
  const int kz = logical / (tiles_m * tiles_n);
  const int m0 = mt * BM;
  const int n0 = nt * BN;
  const int kbeg = kz * kchunk;
  const int kend = min(K, kbeg + kchunk);
  TC *Cz = C + (long)kz * split_stride;
  const R sa = conjA ? R(-1) : R(1);
  const R sb = conjB ? R(-1) : R(1);

  ACC p1[TM][TN], p2[TM][TN], p3[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int e = 0; e < NACC; ++e) {
        p1[i][j][e] = R(0);
        p2[i][j][e] = R(0);
        p3[i][j][e] = R(0);
      }

  // Global operand loads for one K slice into registers.
  auto gload = [&](int k0, TA *ra, TB *rb) {
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      const int e = tid + u * kGT;
      const int r = e / BK, k = e % BK;
      const int gm = m0 + r, gk = k0 + k;
      ra[u] = (gm < M && gk < kend) ? A[(long)gm * lda + gk] : zero_of<TA>();
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int e = tid + u * kGT;
      if (BMODE == 0) {
        const int r = e / BK, k = e % BK;
        const int gn = n0 + r, gk = k0 + k;
        rb[u] = (gn < N && gk < kend) ? B[(long)gn * ldb + gk] : zero_of<TB>();
      } else {
        const int k = e / BN, r = e % BN;
        const int gn = n0 + r, gk = k0 + k;
        rb[u] = (gn < N && gk < kend) ? B[(long)gk * ldb + gn] : zero_of<TB>();
      }
    }
  };
  auto sstore = [&](int buf, const TA *ra, const TB *rb) {
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      const int e = tid + u * kGT;
      const int r = e / BK, k = e % BK;
      As[buf][0][r * BKP + k] = re_of<R>(ra[u]);
      As[buf][1][r * BKP + k] = sa * im_of<R>(ra[u]);
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int e = tid + u * kGT;
      int r, k;
      if (BMODE == 0) {
        r = e / BK;
        k = e % BK;
      } else {
        k = e / BN;
        r = e % BN;
      }
      Bs[buf][0][r * BKP + k] = static_cast<R>(rb[u].x);
      Bs[buf][1][r * BKP + k] = sb * static_cast<R>(rb[u].y);
    }
  };

  const int lr = lane % BS;   // row (A) / column (B) inside a block
  const int lk = lane / BS;   // k inside a step of KS

  auto compute = [&](int buf) {
#pragma unroll
    for (int kk = 0; kk < BK; kk += KS) {
      R ar[TM], ai[TM], as[TM], br[TN], bi[TN], bs[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        const int off = (wm0 + i * BS + lr) * BKP + kk + lk;
        ar[i] = As[buf][0][off];
        ai[i] = As[buf][1][off];
        as[i] = ar[i] + ai[i];
      }
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int off = (wn0 + j * BS + lr) * BKP + kk + lk;
        br[j] = Bs[buf][0][off];
        bi[j] = Bs[buf][1][off];
        bs[j] = br[j] + bi[j];
      }
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          mfma(ar[i], br[j], p1[i][j]);
          if (RM == 2) {
            mfma(ar[i], bi[j], p2[i][j]);
          } else {
            mfma(ai[i], bi[j], p2[i][j]);
            if (RM == 0) mfma(as[i], bs[j], p3[i][j]);
          }
        }
    }
  };

  // one slice in flight: loaded during the MFMAs of the previous one
  TA ra[NA];
  TB rb[NB];
  if (kbeg < kend) {
    gload(kbeg, ra, rb);
    sstore(0, ra, rb);
  }
  __syncthreads();
  int buf = 0;
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    const bool more = k0 + BK < kend;
    if (more) gload(k0 + BK, ra, rb);
    compute(buf);
    if (more) sstore(buf ^ 1, ra, rb);
    __syncthreads();
    buf ^= 1;
  }

  // ---- epilogue.  Column lane%BS of each block.  16 x 16 blocks:
  // accumulator entry r holds row 4*(lane/16)+r for the f32 instruction but
  // row lane/16+4*r for the f64 one (the two lay out D differently); 32 x 32
  // f32 blocks: entry r holds row (r%4) + 8*(r/4) + 4*(lane/32).
  constexpr bool kF64 = sizeof(R) == 8;
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < NACC; ++r) {
        const int rw = BS == 32 ? (r % 4) + 8 * (r / 4) + 4 * lk : kF64 ? lk + 4 * r : 4 * lk + r;
        const int gm = m0 + wm0 + i * BS + rw;
        const int gn = n0 + wn0 + j * BS + lr;
        if (gm < M && gn < N) {
          TC *p = Cz + (long)gm * ldc + gn;
          using RC = typename real_of<TC>::type;
          const R cr = RM == 2 ? p1[i][j][r] : p1[i][j][r] - p2[i][j][r];
          const R ci = RM == 0   ? p3[i][j][r] - p1[i][j][r] - p2[i][j][r]
                       : RM == 2 ? p2[i][j][r]
                                 : R(0);
          if (accumulate) {
            TC v = *p;
            // the add happens in the result's precision
            v.x = v.x + static_cast<RC>(cr);
            v.y = v.y + static_cast<RC>(ci);
            *p = v;
          } else {
            TC v;
            v.x = static_cast<RC>(cr);
            v.y = static_cast<RC>(ci);
            *p = v;
          }
        }
      }
}

template <typename R, typename TA, typename TB, typename TC, int BMODE, int BM, int BN, int BK,
          int RM = 0, int WGM = 2, int WGN = 2, int BS = 16, int WPE = 0>
hipError_t run_tile(const GemmDesc &g, hipStream_t s) {
  const int tm = (g.M + BM - 1) / BM, tn = (g.N + BN - 1) / BN;
  const long total = (long)tm * tn * g.nsplit;
  if (total > (1L << 30)) return hipErrorInvalidValue;
  const int per_xcd = (int)((total + 7) / 8);
  const int kchunk = g.nsplit > 1 ? g.kchunk : g.K;
  hipLaunchKernelGGL((cgemm_kernel<R, TA, TB, TC, BMODE, BM, BN, BK, RM, WGM, WGN, BS, WPE>),
                     dim3(8 * per_xcd), dim3(64 * WGM * WGN), 0, s, reinterpret_cast<const TA *>(g.A), g.lda,
                     reinterpret_cast<const TB *>(g.B), g.ldb, reinterpret_cast<TC *>(g.C), g.ldc,
                     g.M, g.N, g.K, g.conjA, g.conjB, g.accumulate, kchunk, g.split_stride, tm, tn,
                     (int)total, per_xcd);
  return hipGetLastError();
}

// FP64: 64 x 64 tiles, K slices of 8 (16 x 16 blocks).  FP32: 64 x 64 tiles
// on four waves (16 x 16 blocks), or the wide tile for the large projector
// products: 128 x 128 on eight waves with 32 x 32 blocks (half the operand
// re-reads of 64 x 64, and the faster 32 x 32 instruction).
template <typename TA, typename TC, int BMODE>
hipError_t run_f32(const GemmDesc &g, hipStream_t s) {
  if (g.tile == 1) return run_tile<float, TA, float2, TC, BMODE, 128, 128, 16, 0, 2, 4, 32>(g, s);
  return run_tile<float, TA, float2, TC, BMODE, 64, 64, 16>(g, s);
}

template <typename TA, typename TC> hipError_t run_f32_b(const GemmDesc &g, hipStream_t s) {
  return g.bmode == 0 ? run_f32<TA, TC, 0>(g, s) : run_f32<TA, TC, 1>(g, s);
}

template <typename TA> hipError_t run_f32_c(const GemmDesc &g, hipStream_t s) {
  return g.tc == T_D2 ? run_f32_b<TA, double2>(g, s) : run_f32_b<TA, float2>(g, s);
}

template <typename TP, typename TC>
__global__ __launch_bounds__(256) void splitk_reduce_kernel(const TP *__restrict__ part,
                                                            long stride, int nsplit, int M, int N,
                                                            long ldp, TC *__restrict__ C, long ldc,
                                                            int accumulate) {
  const long total = (long)M * N;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < total;
       t += (long)gridDim.x * blockDim.x) {
    const int m = (int)(t / N), n = (int)(t % N);
    const TP *pp = part + (long)m * ldp + n;
    double sr = 0.0, si = 0.0;
    int s = 0;
    for (; s + 8 <= nsplit; s += 8) {   // split order kept; 8 loads in flight
      TP v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = pp[(long)(s + u) * stride];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        sr += static_cast<double>(v[u].x);
        si += static_cast<double>(v[u].y);
      }
    }
    for (; s < nsplit; ++s) {
      const TP v = pp[(long)s * stride];
      sr += static_cast<double>(v.x);
      si += static_cast<double>(v.y);
    }
    TC *p = C + (long)m * ldc + n;
    if (accumulate) {
      sr += static_cast<double>(p->x);
      si += static_cast<double>(p->y);
    }
    TC o;
    o.x = static_cast<typename real_of<TC>::type>(sr);
    o.y = static_cast<typename real_of<TC>::type>(si);
    *p = o;
  }
}

// ---------------------------------------------------------------- D scaling
// grid (chunk, band).  Chunk c covers whole atoms [p0, p1), p1 - p0 <= 256.
// Gamma contexts (gpsi set): the partials sum conj(beta) psi over the stored
// half sphere, and the full-sphere projection is real:
//   becp = 2 Re(sum) - beta(0) psi(0)   (G = 0 counted once; beta(0) real).
__device__ __forceinline__ void store_ps(double2 *ps, long i, double sr, double si) {
  ps[i] = make_double2(sr, si);
}
__device__ __forceinline__ void store_ps(float2 *ps, long i, double sr, double si) {
  ps[i] = make_float2((float)sr, (float)si);
}
// Gamma, single precision: ps is real, stored as one float per entry
__device__ __forceinline__ void store_ps(float *ps, long i, double sr, double) {
  ps[i] = (float)sr;
}

template <typename TP, typename TS>
__global__ __launch_bounds__(256) void dscale_kernel(
    const TP *__restrict__ part, long split_stride, int nsplit, int nkb, TS *__restrict__ ps,
    const double2 *__restrict__ dmat, const int *__restrict__ pj0, const int *__restrict__ pnb,
    const int *__restrict__ pdoff, const int *__restrict__ chunk,
    const double2 *__restrict__ gpsi, long ldpsi, const TP *__restrict__ gbeta, long ldb) {
  __shared__ double2 becp[256];
  const int p0 = chunk[blockIdx.x], p1 = chunk[blockIdx.x + 1];
  const int b = blockIdx.y;
  const int t = threadIdx.x;
  const int j = p0 + t;
  if (j < p1) {
    // partials summed in split order; loads issued eight at a time so that
    // several are in flight per thread
    const TP *pp = part + (long)b * nkb + j;
    double sr = 0.0, si = 0.0;
    int s = 0;
    for (; s + 8 <= nsplit; s += 8) {
      TP v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = pp[(long)(s + u) * split_stride];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        sr += static_cast<double>(v[u].x);
        si += static_cast<double>(v[u].y);
      }
    }
    for (; s < nsplit; ++s) {
      const TP v = pp[(long)s * split_stride];
      sr += static_cast<double>(v.x);
      si += static_cast<double>(v.y);
    }
    if (gpsi) {
      const double p0 = gpsi[(long)b * ldpsi].x;
      const double b0 = static_cast<double>(gbeta[(long)j * ldb].x);
      sr = 2.0 * sr - b0 * p0;
      si = 0.0;
    }
    becp[t] = make_double2(sr, si);
  }
  __syncthreads();
  if (j < p1) {
    const int j0 = pj0[j], nbk = pnb[j];
    const double2 *drow = dmat + pdoff[j];
    double sr = 0.0, si = 0.0;
    for (int q = 0; q < nbk; ++q) {
      const double2 d = drow[q];
      const double2 v = becp[j0 + q - p0];
      sr += d.x * v.x - d.y * v.y;
      si += d.x * v.y + d.y * v.x;
    }
    store_ps(ps, (long)b * nkb + j, sr, si);
  }
}

}  // namespace

// The Gamma-point forms: RM = 1 for beta^H psi (bmode 0, psi read in double,
// or its single-precision copy), RM = 2 for beta ps (bmode 1, A = ps real:
// complex storage in FP64, one float per entry in single precision;
// C = hpsi).  FP32 wide tiles (tile 1): beta^H psi from the single-precision
// copy on 128 x 128 held to 128 registers (four waves per SIMD, two
// workgroups per CU: 2.54 against 2.72 ms for 128 x 256 at the 512-atom
// cell), from psi in double on 128 x 256 (psi re-read once per 256
// projectors); beta ps on 128 x 128.
hipError_t launch_cgemm_real(const GemmDesc &g, hipStream_t s) {
  if (g.prec == G_F64) {
    if (g.ta != T_D2 || g.tb != T_D2 || g.tc != T_D2) return hipErrorInvalidValue;
    if (g.rmode == 1 && g.bmode == 0)
      return run_tile<double, double2, double2, double2, 0, 64, 64, 8, 1>(g, s);
    if (g.rmode == 2 && g.bmode == 1)
      return run_tile<double, double2, double2, double2, 1, 64, 64, 8, 2>(g, s);
    return hipErrorInvalidValue;
  }
  if (g.tb != T_F2) return hipErrorInvalidValue;
  if (g.rmode == 1 && g.bmode == 0 && g.ta == T_D2 && g.tc == T_F2)
    return g.tile == 1
               ? run_tile<float, double2, float2, float2, 0, 128, 256, 16, 1, 2, 4, 32>(g, s)
               : run_tile<float, double2, float2, float2, 0, 64, 64, 16, 1>(g, s);
  if (g.rmode == 1 && g.bmode == 0 && g.ta == T_F2 && g.tc == T_F2)
    return g.tile == 1
               ? run_tile<float, float2, float2, float2, 0, 128, 128, 16, 1, 2, 4, 32, 4>(g, s)
               : run_tile<float, float2, float2, float2, 0, 64, 64, 16, 1>(g, s);
  if (g.rmode == 2 && g.bmode == 1 && g.ta == T_F2 && g.tc == T_D2)
    return g.tile == 1
               ? run_tile<float, float2, float2, double2, 1, 128, 128, 16, 2, 2, 4, 32>(g, s)
               : run_tile<float, float2, float2, double2, 1, 64, 64, 16, 2>(g, s);
  if (g.rmode == 2 && g.bmode == 1 && g.ta == T_F1 && g.tc == T_D2)
    return g.tile == 1
               ? run_tile<float, float, float2, double2, 1, 128, 128, 16, 2, 2, 4, 32>(g, s)
               : run_tile<float, float, float2, double2, 1, 64, 64, 16, 2>(g, s);
  return hipErrorInvalidValue;
}

hipError_t launch_cgemm(const GemmDesc &g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0 || g.K <= 0) return hipSuccess;
  if (g.rmode != 0) return launch_cgemm_real(g, s);
  if (g.prec == G_F64) {
    if (g.ta != T_D2 || g.tb != T_D2 || g.tc != T_D2) return hipErrorInvalidValue;
    return g.bmode == 0 ? run_tile<double, double2, double2, double2, 0, 64, 64, 8>(g, s)
                        : run_tile<double, double2, double2, double2, 1, 64, 64, 8>(g, s);
  }
  if (g.tb != T_F2) return hipErrorInvalidValue;
  return g.ta == T_D2 ? run_f32_c<double2>(g, s) : run_f32_c<float2>(g, s);
}

hipError_t launch_splitk_reduce(const void *part, int tp, long stride, int nsplit, int M, int N,
                                long ldp, double2 *C, long ldc, int accumulate, hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  const long total = (long)M * N;
  const int blocks = (int)std::min<long>((total + 255) / 256, 4096);
  if (tp == T_D2)
    hipLaunchKernelGGL((splitk_reduce_kernel<double2, double2>), dim3(blocks), dim3(256), 0, s,
                       reinterpret_cast<const double2 *>(part), stride, nsplit, M, N, ldp, C, ldc,
                       accumulate);
  else
    hipLaunchKernelGGL((splitk_reduce_kernel<float2, double2>), dim3(blocks), dim3(256), 0, s,
                       reinterpret_cast<const float2 *>(part), stride, nsplit, M, N, ldp, C, ldc,
                       accumulate);
  return hipGetLastError();
}

hipError_t launch_dscale(const qeh_ctx *c, int nbk, const double2 *psi, long ldpsi,
                         const double2 *mat) {
  if (c->nkb == 0) return hipSuccess;
  if (!mat) mat = c->d.dmat;
  dim3 grid(c->nchunk, nbk);
  const long ss = (long)c->block * c->nkb;
  const double2 *gpsi = c->gamma ? psi : nullptr;
  if (c->prec == QEH_FP64) {
    hipLaunchKernelGGL((dscale_kernel<double2, double2>), grid, dim3(256), 0, c->stream,
                       reinterpret_cast<const double2 *>(c->d.part), ss, c->nsplit, c->nkb,
                       reinterpret_cast<double2 *>(c->d.ps), mat, c->d.pj0, c->d.pnb,
                       c->d.pdoff, c->d.chunk, gpsi, ldpsi,
                       reinterpret_cast<const double2 *>(c->d.beta), (long)c->npw);
  } else if (c->gamma) {
    // real ps, one float per entry: half the A operand of the beta ps product
    hipLaunchKernelGGL((dscale_kernel<float2, float>), grid, dim3(256), 0, c->stream,
                       reinterpret_cast<const float2 *>(c->d.part), ss, c->nsplit, c->nkb,
                       reinterpret_cast<float *>(c->d.ps), mat, c->d.pj0, c->d.pnb,
                       c->d.pdoff, c->d.chunk, gpsi, ldpsi,
                       reinterpret_cast<const float2 *>(c->d.beta), (long)c->npw);
  } else {
    hipLaunchKernelGGL((dscale_kernel<float2, float2>), grid, dim3(256), 0, c->stream,
                       reinterpret_cast<const float2 *>(c->d.part), ss, c->nsplit, c->nkb,
                       reinterpret_cast<float2 *>(c->d.ps), mat, c->d.pj0, c->d.pnb,
                       c->d.pdoff, c->d.chunk, gpsi, ldpsi,
                       reinterpret_cast<const float2 *>(c->d.beta), (long)c->npw);
  }
  return hipGetLastError();
}

}  // namespace qeh
