// Radix-2/3/4/5/7/8 DFT butterflies on registers (host and device).
// Sign convention: exp(+2 pi i/R) for INV, exp(-2 pi i/R) otherwise.
#pragma once

#include "cplx.h"

namespace qeh {


template <typename C, bool INV> __host__ __device__ __forceinline__ void dft2(C *v) {
  C a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}

template <typename C, bool INV> __host__ __device__ __forceinline__ void dft3(C *v) {
  using R = typename real_of<C>::type;
  const R s3 = R(0.86602540378443864676);
  C t1 = cadd(v[1], v[2]);
  C t2 = csub(v[1], v[2]);
  C m = cmk<C>(v[0].x - R(0.5) * t1.x, v[0].y - R(0.5) * t1.y);
  C r = mul_si<C, INV>(cscale(t2, s3));
  v[0] = cadd(v[0], t1);
  v[1] = cadd(m, r);
  v[2] = csub(m, r);
}

template <typename C, bool INV> __host__ __device__ __forceinline__ void dft4(C *v) {
  C a02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
  C a13 = cadd(v[1], v[3]), d13 = mul_si<C, INV>(csub(v[1], v[3]));
  v[0] = cadd(a02, a13);
  v[2] = csub(a02, a13);
  v[1] = cadd(d02, d13);
  v[3] = csub(d02, d13);
}

template <typename C, bool INV> __host__ __device__ __forceinline__ void dft5(C *v) {
  using R = typename real_of<C>::type;
  const R c1 = R(0.30901699437494742410), c2 = R(-0.80901699437494742410);
  const R s1 = R(0.95105651629515357212), s2 = R(0.58778525229247312917);
  C A = cadd(v[1], v[4]), B = cadd(v[2], v[3]);
  C Cd = csub(v[1], v[4]), D = csub(v[2], v[3]);
  C m1 = cmk<C>(v[0].x + c1 * A.x + c2 * B.x, v[0].y + c1 * A.y + c2 * B.y);
  C m2 = cmk<C>(v[0].x + c2 * A.x + c1 * B.x, v[0].y + c2 * A.y + c1 * B.y);
  C n1 = mul_si<C, INV>(cmk<C>(s1 * Cd.x + s2 * D.x, s1 * Cd.y + s2 * D.y));
  C n2 = mul_si<C, INV>(cmk<C>(s2 * Cd.x - s1 * D.x, s2 * Cd.y - s1 * D.y));
  v[0] = cadd(v[0], cadd(A, B));
  v[1] = cadd(m1, n1);
  v[4] = csub(m1, n1);
  v[2] = cadd(m2, n2);
  v[3] = csub(m2, n2);
}

template <typename C, bool INV> __host__ __device__ __forceinline__ void dft7(C *v) {
  using R = typename real_of<C>::type;
  // cos(2 pi m / 7), sin(2 pi m / 7), m = 1..3
  const R cs[3] = {R(0.62348980185873353053), R(-0.22252093395631440429),
                   R(-0.90096886790241912624)};
  const R sn[3] = {R(0.78183148246802980871), R(0.97492791218182360702),
                   R(0.43388373911755812048)};
  C sp[3], sm[3];
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    sp[q] = cadd(v[q + 1], v[6 - q]);
    sm[q] = csub(v[q + 1], v[6 - q]);
  }
  C x0 = v[0];
  C out[7];
  out[0] = cadd(x0, cadd(sp[0], cadd(sp[1], sp[2])));
#pragma unroll
  for (int k = 1; k <= 3; ++k) {
    C re = x0, im = cmk<C>(R(0), R(0));
#pragma unroll
    for (int q = 1; q <= 3; ++q) {
      const int m = (q * k) % 7;           // 1..6
      const R c = (m <= 3) ? cs[m - 1] : cs[7 - m - 1];
      const R s = (m <= 3) ? sn[m - 1] : -sn[7 - m - 1];
      re = cadd(re, cscale(sp[q - 1], c));
      im = cadd(im, cscale(sm[q - 1], s));
    }
    C rot = mul_si<C, INV>(im);
    out[k] = cadd(re, rot);
    out[7 - k] = csub(re, rot);
  }
#pragma unroll
  for (int k = 0; k < 7; ++k) v[k] = out[k];
}

template <typename C, bool INV> __host__ __device__ __forceinline__ void dft8(C *v) {
  using R = typename real_of<C>::type;
  const R h = R(0.70710678118654752440);
  C e[4] = {v[0], v[2], v[4], v[6]};
  C o[4] = {v[1], v[3], v[5], v[7]};
  dft4<C, INV>(e);
  dft4<C, INV>(o);
  // w^k o_k, w = exp(sign 2 pi i / 8)
  C w1 = cscale(cadd(o[1], mul_si<C, INV>(o[1])), h);
  C w2 = mul_si<C, INV>(o[2]);
  C w3 = cscale(csub(mul_si<C, INV>(o[3]), o[3]), h);
  v[0] = cadd(e[0], o[0]);
  v[4] = csub(e[0], o[0]);
  v[1] = cadd(e[1], w1);
  v[5] = csub(e[1], w1);
  v[2] = cadd(e[2], w2);
  v[6] = csub(e[2], w2);
  v[3] = cadd(e[3], w3);
  v[7] = csub(e[3], w3);
}

template <typename C, int R, bool INV> __host__ __device__ __forceinline__ void dftR(C *v) {
  if constexpr (R == 2) dft2<C, INV>(v);
  else if constexpr (R == 3) dft3<C, INV>(v);
  else if constexpr (R == 4) dft4<C, INV>(v);
  else if constexpr (R == 5) dft5<C, INV>(v);
  else if constexpr (R == 7) dft7<C, INV>(v);
  else if constexpr (R == 8) dft8<C, INV>(v);
}

}  // namespace qeh
