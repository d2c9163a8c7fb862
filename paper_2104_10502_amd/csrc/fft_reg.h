// Whole 1D transforms held in one thread's registers, for lengths known at
// compile time (natural order in and out).
//
// N = R * M with R the first radix from {8, 4, 2, 3, 5, 7}: the R sub-sequences
// x[r + R m] are transformed recursively (length M), multiplied by the
// twiddles W_N^{r k'}, and combined by R-point butterflies:
//   X[k' + M s] = sum_r W_R^{r s} W_N^{r k'} Y_r[k'].
// Every index is a compile-time constant after unrolling, so the arrays stay
// in registers and the twiddles are immediate constants (tables evaluated by
// constexpr trigonometry: Taylor series on the reduced angle).
#pragma once

#include "cplx.h"
#include "fft_radix.h"

namespace qeh {
namespace regfft {

constexpr double kPi = 3.14159265358979323846264338327950288;

// sin / cos of 2 pi m / n for integers m, n (angle reduced to [-pi, pi]).
constexpr double ce_sincos(long m, long n, bool want_sin) {
  long r = m % n;
  if (r < 0) r += n;
  if (2 * r > n) r -= n;
  const double x = 2.0 * kPi * (double)r / (double)n;
  double term = want_sin ? x : 1.0;
  double sum = term;
  const int start = want_sin ? 1 : 0;
  for (int i = 1; i < 30; ++i) {
    const int a = 2 * i - 1 + start, b = 2 * i + start;
    term *= -x * x / ((double)a * (double)b);
    sum += term;
  }
  return sum;
}

template <int N> struct Table {
  double re[N > 0 ? N : 1];
  double im[N > 0 ? N : 1];
};

// exp(-2 pi i m / N)
template <int N> constexpr Table<N> make_table() {
  Table<N> t{};
  for (int m = 0; m < N; ++m) {
    t.re[m] = ce_sincos(m, N, false);
    t.im[m] = -ce_sincos(m, N, true);
  }
  return t;
}

template <int N> struct Tw {
  static constexpr Table<N> t = make_table<N>();
};

constexpr int first_radix(int n) {
  return n % 8 == 0 ? 8 : n % 4 == 0 ? 4 : n % 2 == 0 ? 2 : n % 3 == 0 ? 3 : n % 5 == 0 ? 5 : 7;
}

template <typename C, int N, bool INV> struct Fft {
  static __host__ __device__ __forceinline__ void run(C *v) {
    constexpr int R = first_radix(N);
    constexpr int M = N / R;
    using Rl = typename real_of<C>::type;
    if constexpr (M == 1) {
      dftR<C, R, INV>(v);
    } else {
      C y[R][M];
#pragma unroll
      for (int r = 0; r < R; ++r) {
#pragma unroll
        for (int m = 0; m < M; ++m) y[r][m] = v[r + R * m];
        Fft<C, M, INV>::run(y[r]);
      }
#pragma unroll
      for (int k = 0; k < M; ++k) {
        C u[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int e = (r * k) % N;
          if (e == 0) {
            u[r] = y[r][k];
          } else {
            const Rl wr = static_cast<Rl>(Tw<N>::t.re[e]);
            const Rl wi = static_cast<Rl>(INV ? -Tw<N>::t.im[e] : Tw<N>::t.im[e]);
            u[r] = cmul(y[r][k], cmk<C>(wr, wi));
          }
        }
        dftR<C, R, INV>(u);
#pragma unroll
        for (int s = 0; s < R; ++s) v[k + M * s] = u[s];
      }
    }
  }
};

// ---------------------------------------------------------------- lane pairs
// A line of N = 2M points held by two adjacent lanes (lane parity l), M points
// each: the in-lane transforms of length M above plus one radix-2 stage across
// the pair, whose partner values arrive through a DPP swap of adjacent lanes.
// Both lanes of a pair must be active together.

__device__ __forceinline__ float lane_swap(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false));
}
__device__ __forceinline__ double lane_swap(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, 0xB1, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0xB1, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Lane 1 multiplies element k by W_N^{k} (conjugated for the inverse); the
// product is formed on both lanes and selected, which keeps the code free of
// divergent branches.
template <typename C, int N, bool INV>
__device__ __forceinline__ void pair_twiddle(C *v, bool odd) {
  using Rl = typename real_of<C>::type;
  constexpr int M = N / 2;
#pragma unroll
  for (int k = 1; k < M; ++k) {
    const Rl wr = static_cast<Rl>(Tw<N>::t.re[k]);
    const Rl wi = static_cast<Rl>(INV ? -Tw<N>::t.im[k] : Tw<N>::t.im[k]);
    const C t = cmul(v[k], cmk<C>(wr, wi));
    v[k] = odd ? t : v[k];
  }
}

// Radix-2 across the pair: lane 0 keeps own + partner, lane 1 partner - own.
template <typename C, int M>
__device__ __forceinline__ void pair_butterfly(C *v, bool odd) {
#pragma unroll
  for (int k = 0; k < M; ++k) {
    const C o = v[k];
    const C p = cmk<C>(lane_swap(o.x), lane_swap(o.y));
    v[k].x = odd ? p.x - o.x : p.x + o.x;
    v[k].y = odd ? p.y - o.y : p.y + o.y;
  }
}

// Inverse (+i) transform of length N: on entry lane l holds x[2n + l], n < M;
// on exit X[k + M l], k < M.
template <typename C, int N>
__device__ __forceinline__ void pair_inv(C *v, bool odd) {
  Fft<C, N / 2, true>::run(v);
  pair_twiddle<C, N, true>(v, odd);
  pair_butterfly<C, N / 2>(v, odd);
}

// Forward (-i) transform of length N: on entry lane l holds f[x + M l];
// on exit F[2m + l].
template <typename C, int N>
__device__ __forceinline__ void pair_fwd(C *v, bool odd) {
  pair_butterfly<C, N / 2>(v, odd);
  pair_twiddle<C, N, false>(v, odd);
  Fft<C, N / 2, false>::run(v);
}

// ---------------------------------------------------------------- lane quads
// A line of N = 4Q points held by four adjacent lanes (q = lane & 3), Q points
// each: in-lane transforms of length Q plus a 4-point transform across the
// quad, done as two radix-2 stages through DPP swaps (partner lane q ^ 2, then
// q ^ 1) with a quarter-turn rotation on lane 3 between them.  With br(q) the
// two-bit reversal of q:
//   quad_inv: lane q holds x[4n + q] (n < Q) -> X[k + Q br(q)] (k < Q);
//   quad_fwd: lane q holds f[x + Q br(q)]    -> F[4m + q].
// So the output of quad_inv is the input layout of quad_fwd.  All four lanes of
// a quad must be active together.

template <int CTRL> __device__ __forceinline__ float lane_perm(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL> __device__ __forceinline__ double lane_perm(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
constexpr int kDppXor1 = 0xB1;   // quad_perm [1, 0, 3, 2]
constexpr int kDppXor2 = 0x4E;   // quad_perm [2, 3, 0, 1]

// Per-lane constants of a quad, computed once: the signs of the two radix-2
// stages and the quarter-turn coefficients of lane 3.
template <typename Rl> struct QuadLane {
  Rl s1, s2;   // +1 / -1: own + partner or partner - own (partners q ^ 1, q ^ 2)
  Rl rc, rs;   // lane 3: (0, 1) (times +i; the forward uses -i); others (1, 0)
  __device__ explicit QuadLane(int q)
      : s1((q & 1) ? Rl(-1) : Rl(1)), s2((q & 2) ? Rl(-1) : Rl(1)),
        rc(q == 3 ? Rl(0) : Rl(1)), rs(q == 3 ? Rl(1) : Rl(0)) {}
};

// radix-2 across lanes q and q ^ mask: partner + sign * own
template <typename C, int Q, int CTRL>
__device__ __forceinline__ void quad_bfly(C *v, typename real_of<C>::type sgn) {
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    const C o = v[k];
    v[k].x = lane_perm<CTRL>(o.x) + sgn * o.x;
    v[k].y = lane_perm<CTRL>(o.y) + sgn * o.y;
  }
}

// lane 3 times +i (inverse) or -i (forward), as (rc + i rs) or its conjugate
template <typename C, int Q, bool INV>
__device__ __forceinline__ void quad_rotate(C *v, typename real_of<C>::type rc,
                                            typename real_of<C>::type rs) {
  const auto s = INV ? rs : -rs;
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    const C a = v[k];
    v[k].x = rc * a.x - s * a.y;
    v[k].y = s * a.x + rc * a.y;
  }
}

// element k times tw[k] (this lane's row W_N^{q k} of a table), conjugated for
// the inverse
template <typename C, int Q, bool INV>
__device__ __forceinline__ void quad_twiddle(C *v, const C *tw) {
#pragma unroll
  for (int k = 1; k < Q; ++k) v[k] = INV ? cmulc(v[k], tw[k]) : cmul(v[k], tw[k]);
}

// tw: this lane's table row, tw[k] = W_N^{q k} for k < Q (W_N = exp(-2 pi i / N))
template <typename C, int N>
__device__ __forceinline__ void quad_inv(C *v, const C *tw,
                                         const QuadLane<typename real_of<C>::type> &ql) {
  constexpr int Q = N / 4;
  Fft<C, Q, true>::run(v);
  quad_twiddle<C, Q, true>(v, tw);
  quad_bfly<C, Q, kDppXor2>(v, ql.s2);
  quad_rotate<C, Q, true>(v, ql.rc, ql.rs);
  quad_bfly<C, Q, kDppXor1>(v, ql.s1);
}

template <typename C, int N>
__device__ __forceinline__ void quad_fwd(C *v, const C *tw,
                                         const QuadLane<typename real_of<C>::type> &ql) {
  constexpr int Q = N / 4;
  quad_bfly<C, Q, kDppXor1>(v, ql.s1);
  quad_rotate<C, Q, false>(v, ql.rc, ql.rs);
  quad_bfly<C, Q, kDppXor2>(v, ql.s2);
  quad_twiddle<C, Q, false>(v, tw);
  Fft<C, Q, false>::run(v);
}

// ---------------------------------------------------------------- lane octets
// A line of N = 8Q points held by eight adjacent lanes (o = lane & 7), Q
// points each: in-lane transforms of length Q, a per-lane twiddle W_N^{o k},
// and the 8-point transform across the octet as three radix-2 stages: with
// partners o ^ 4 (a DPP shift by four lanes inside the 16-lane row, up or down
// by bit 2 of the lane), then o ^ 2 and o ^ 1 (quad permutations), and the
// eighth- and quarter-turn twiddles between them.  With br3(o) the three-bit
// reversal of o:
//   oct_inv: lane o holds x[8n + o] (n < Q) -> X[k + Q br3(o)] (k < Q);
//   oct_fwd: lane o holds f[x + Q br3(o)]    -> F[8m + o].
// Single precision only; all eight lanes of an octet must be active together.

constexpr int kDppShl4 = 0x104;   // lane i reads lane i + 4 (same row)
constexpr int kDppShr4 = 0x114;   // lane i reads lane i - 4 (same row)

__device__ __forceinline__ float lane_xor4(float v, bool hi) {
  const float up = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), kDppShl4, 0xF,
                                                              0xF, false));
  const float dn = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), kDppShr4, 0xF,
                                                              0xF, false));
  return hi ? dn : up;
}

// Per-lane constants of an octet: signs of the three radix-2 stages, the
// eighth-turn w8^{o & 3} of the lanes o >= 4 (after the o ^ 4 stage) and the
// quarter turn of the lanes o & 3 == 3 (after the o ^ 2 stage), as (cos, sin)
// of the inverse direction (the forward uses the conjugates).
struct OctLane {
  float s1, s2, s4;
  float ec, es;   // eighth turn: lanes o >= 4, angle 2 pi (o & 3) / 8; else (1, 0)
  float qc, qs;   // quarter turn: lanes with o & 3 == 3, (0, 1); else (1, 0)
  bool hi;        // bit 2 of the lane
  __device__ explicit OctLane(int o)
      : s1((o & 1) ? -1.f : 1.f), s2((o & 2) ? -1.f : 1.f), s4((o & 4) ? -1.f : 1.f),
        ec(1.f), es(0.f), qc((o & 3) == 3 ? 0.f : 1.f), qs((o & 3) == 3 ? 1.f : 0.f),
        hi((o & 4) != 0) {
    if (o & 4) {
      const int j = o & 3;   // cos / sin of 2 pi j / 8
      const float r = 0.70710678118654752440f;
      ec = j == 0 ? 1.f : j == 1 ? r : j == 2 ? 0.f : -r;
      es = j == 0 ? 0.f : j == 1 ? r : j == 2 ? 1.f : r;
    }
  }
};

// radix-2 across lanes o and o ^ 4: partner + sign * own
template <int Q> __device__ __forceinline__ void oct_bfly4(float2 *v, const OctLane &ol) {
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    const float2 a = v[k];
    v[k].x = lane_xor4(a.x, ol.hi) + ol.s4 * a.x;
    v[k].y = lane_xor4(a.y, ol.hi) + ol.s4 * a.y;
  }
}

// times (c + i s) for the inverse, (c - i s) for the forward
template <int Q, bool INV>
__device__ __forceinline__ void oct_rotate(float2 *v, float c, float s0) {
  const float s = INV ? s0 : -s0;
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    const float2 a = v[k];
    v[k].x = c * a.x - s * a.y;
    v[k].y = s * a.x + c * a.y;
  }
}

// tw: this lane's table row, tw[k] = W_N^{o k} for k < Q (W_N = exp(-2 pi i / N))
template <int N>
__device__ __forceinline__ void oct_inv(float2 *v, const float2 *tw, const OctLane &ol) {
  constexpr int Q = N / 8;
  Fft<float2, Q, true>::run(v);
  quad_twiddle<float2, Q, true>(v, tw);
  oct_bfly4<Q>(v, ol);
  oct_rotate<Q, true>(v, ol.ec, ol.es);
  quad_bfly<float2, Q, kDppXor2>(v, ol.s2);
  oct_rotate<Q, true>(v, ol.qc, ol.qs);
  quad_bfly<float2, Q, kDppXor1>(v, ol.s1);
}

template <int N>
__device__ __forceinline__ void oct_fwd(float2 *v, const float2 *tw, const OctLane &ol) {
  constexpr int Q = N / 8;
  quad_bfly<float2, Q, kDppXor1>(v, ol.s1);
  oct_rotate<Q, false>(v, ol.qc, ol.qs);
  quad_bfly<float2, Q, kDppXor2>(v, ol.s2);
  oct_rotate<Q, false>(v, ol.ec, ol.es);
  oct_bfly4<Q>(v, ol);
  quad_twiddle<float2, Q, false>(v, tw);
  Fft<float2, Q, false>::run(v);
}

}  // namespace regfft
}  // namespace qeh
