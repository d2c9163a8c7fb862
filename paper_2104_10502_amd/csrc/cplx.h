// Small complex helpers on HIP float2 / double2 (device code).
#pragma once

#include <hip/hip_runtime.h>

namespace qeh {

template <typename R> struct cplx_of;
template <> struct cplx_of<float> { using type = float2; };
template <> struct cplx_of<double> { using type = double2; };

template <typename C> struct real_of;
template <> struct real_of<float2> { using type = float; };
template <> struct real_of<double2> { using type = double; };

template <typename C>
__host__ __device__ __forceinline__ C cmk(typename real_of<C>::type a, typename real_of<C>::type b) {
  C r;
  r.x = a;
  r.y = b;
  return r;
}
template <typename C> __host__ __device__ __forceinline__ C cadd(C a, C b) { return cmk<C>(a.x + b.x, a.y + b.y); }
template <typename C> __host__ __device__ __forceinline__ C csub(C a, C b) { return cmk<C>(a.x - b.x, a.y - b.y); }
template <typename C> __host__ __device__ __forceinline__ C cmul(C a, C b) {
  return cmk<C>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
template <typename C> __host__ __device__ __forceinline__ C cmulc(C a, C b) {
  return cmk<C>(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
template <typename C>
__host__ __device__ __forceinline__ C cscale(C a, typename real_of<C>::type s) { return cmk<C>(a.x * s, a.y * s); }
// multiply by sign*i, sign = +1 (INV) or -1
template <typename C, bool INV> __host__ __device__ __forceinline__ C mul_si(C z) {
  return INV ? cmk<C>(-z.y, z.x) : cmk<C>(z.y, -z.x);
}
template <typename CD, typename CS> __host__ __device__ __forceinline__ CD ccast(CS a) {
  return cmk<CD>(static_cast<typename real_of<CD>::type>(a.x),
                 static_cast<typename real_of<CD>::type>(a.y));
}

}  // namespace qeh
