// Nonlocal projectors beta_i(k+G) built on the device from radial tables (the
// pseudopotential terms of the quantum-engine modules), and the nonlocal part
// of diag(H) summed from them.
//
// Generator: one thread per (G, atom); workgroups of 256 consecutive G of one
// atom (grid x = G chunks, y = atoms).  The thread forms q = k + G, |q|, the
// unit vector and the structure factor exp(-i q . tau_a) once, then for each
// radial channel of the atom's species interpolates F_c(|q|) from its table
// (cubic Lagrange through four points) and writes the 2l+1 harmonics.  Every
// write of a projector row is 64 consecutive complex values per wave, so the
// kernel streams nkb * npw complex values to HBM with nothing read back; the
// tables (a few KB) and the per-atom data stay in the caches.  Everything is
// computed in double; the single-precision form rounds at the store.
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "qeh_internal.h"

namespace qeh {
namespace {

constexpr int kBT = 256;

template <typename T2> __device__ __forceinline__ T2 mk2(double re, double im);
template <> __device__ __forceinline__ double2 mk2<double2>(double re, double im) {
  return make_double2(re, im);
}
template <> __device__ __forceinline__ float2 mk2<float2>(double re, double im) {
  return make_float2((float)re, (float)im);
}

template <typename T2>
__global__ __launch_bounds__(kBT) void beta_gen_kernel(
    const double *__restrict__ q, int npw, const int4 *__restrict__ atoms,
    const double *__restrict__ tau, const int *__restrict__ chan0,
    const int *__restrict__ lchan, const double *__restrict__ tab, int nq, double inv_dq,
    double pref, T2 *__restrict__ beta, long ldb) {
  const int g = blockIdx.x * kBT + threadIdx.x;
  if (g >= npw) return;
  const int a = blockIdx.y;
  const int4 at = atoms[a];   // species, first projector row, projectors, D offset
  const double qx = q[g], qy = q[npw + g], qz = q[2 * npw + g];
  const double qn = sqrt(qx * qx + qy * qy + qz * qz);
  const double inv = qn > 0.0 ? 1.0 / qn : 0.0;
  const double ux = qx * inv, uy = qy * inv, uz = qz * inv;
  double sn, cs;
  sincos(qx * tau[3 * a] + qy * tau[3 * a + 1] + qz * tau[3 * a + 2], &sn, &cs);
  // cubic Lagrange weights on table points j-1, j, j+1, j+2 at offset t from j
  const double x = qn * inv_dq;
  int j = (int)x;
  j = max(1, min(j, nq - 3));
  const double t = x - (double)j;
  const double tp = t + 1.0, tm = t - 1.0, tmm = t - 2.0;
  const double w0 = -t * tm * tmm * (1.0 / 6.0);
  const double w1 = tp * tm * tmm * 0.5;
  const double w2 = -tp * t * tmm * 0.5;
  const double w3 = tp * t * tm * (1.0 / 6.0);
  // real harmonics of the unit vector
  constexpr double kPi = 3.14159265358979323846;
  const double y0 = 0.5 / sqrt(kPi);                  // 1 / sqrt(4 pi)
  const double y1 = sqrt(3.0 / (4.0 * kPi));
  const double y2a = sqrt(15.0 / (4.0 * kPi));
  const double y2b = sqrt(5.0 / (16.0 * kPi));
  const double y2c = sqrt(15.0 / (16.0 * kPi));
  T2 *out = beta + (long)at.y * ldb + g;
  const int c1 = chan0[at.x + 1];
  for (int c = chan0[at.x]; c < c1; ++c) {
    const double *f = tab + (long)c * nq + (j - 1);
    const double F = pref * (w0 * f[0] + w1 * f[1] + w2 * f[2] + w3 * f[3]);
    // F exp(-i q.tau) (-i)^l
    double vr = F * cs, vi = -F * sn;
    const int l = lchan[c];
    if (l == 0) {
      out[0] = mk2<T2>(vr * y0, vi * y0);
      out += ldb;
    } else if (l == 1) {
      const double r = vi, i = -vr;   // times -i
      out[0] = mk2<T2>(r * y1 * ux, i * y1 * ux);
      out[ldb] = mk2<T2>(r * y1 * uy, i * y1 * uy);
      out[2 * ldb] = mk2<T2>(r * y1 * uz, i * y1 * uz);
      out += 3 * ldb;
    } else {
      vr = -vr;   // times (-i)^2
      vi = -vi;
      const double h[5] = {y2a * ux * uy, y2a * uy * uz, y2a * uz * ux,
                           y2b * (3.0 * uz * uz - 1.0), y2c * (ux * ux - uy * uy)};
#pragma unroll
      for (int m = 0; m < 5; ++m) out[m * ldb] = mk2<T2>(vr * h[m], vi * h[m]);
      out += 5 * ldb;
    }
  }
}

template <typename T2> __device__ __forceinline__ double2 ld2(const T2 *p);
template <> __device__ __forceinline__ double2 ld2<double2>(const double2 *p) { return *p; }
template <> __device__ __forceinline__ double2 ld2<float2>(const float2 *p) {
  const float2 v = *p;
  return make_double2(v.x, v.y);
}

// hdiag[G] += sum_a sum_ij Re(beta_i(G) D_ij conj(beta_j(G))).  A workgroup
// holds 64 consecutive G (one per lane) and kDW waves; wave w sums the atoms
// w, w + kDW, ... in order, and wave 0 adds the kDW partial sums in wave
// order, so the result does not depend on scheduling.  Spreading the atoms
// over the waves gives kDW times the workgroups' parallelism of a thread per G.
constexpr int kDW = 16;

template <typename T2>
__global__ __launch_bounds__(64 * kDW) void nl_diag_kernel(const T2 *__restrict__ beta, long ldb,
                                                           int npw, int nat,
                                                           const int4 *__restrict__ atoms,
                                                           const double2 *__restrict__ dmat,
                                                           double *__restrict__ hdiag) {
  __shared__ double part[kDW][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int g = blockIdx.x * 64 + lane;
  constexpr int kReg = 16;   // atoms with up to this many projectors: values in registers
  double acc = 0.0;
  if (g < npw) {
    for (int a = w; a < nat; a += kDW) {
      const int4 at = atoms[a];
      const int n = at.z;
      const T2 *b = beta + (long)at.y * ldb + g;
      const double2 *D = dmat + at.w;
      if (n <= kReg) {
        double2 v[kReg];
#pragma unroll
        for (int i = 0; i < kReg; ++i)
          v[i] = i < n ? ld2<T2>(b + (long)i * ldb) : make_double2(0.0, 0.0);
#pragma unroll
        for (int i = 0; i < kReg; ++i)
#pragma unroll
          for (int k = 0; k < kReg; ++k)
            if (i < n && k < n) {
              const double2 d = D[i * n + k];
              const double tr = v[i].x * d.x - v[i].y * d.y, ti = v[i].x * d.y + v[i].y * d.x;
              acc += tr * v[k].x + ti * v[k].y;
            }
      } else {
        for (int i = 0; i < n; ++i) {
          const double2 bi = ld2<T2>(b + (long)i * ldb);
          for (int k = 0; k < n; ++k) {
            const double2 d = D[i * n + k];
            const double2 bk = ld2<T2>(b + (long)k * ldb);
            const double tr = bi.x * d.x - bi.y * d.y, ti = bi.x * d.y + bi.y * d.x;
            acc += tr * bk.x + ti * bk.y;
          }
        }
      }
    }
  }
  part[w][lane] = acc;
  __syncthreads();
  if (w == 0 && g < npw) {
    double t = part[0][lane];
#pragma unroll
    for (int k = 1; k < kDW; ++k) t += part[k][lane];
    hdiag[g] += t;
  }
}

}  // namespace

hipError_t launch_beta_gen(bool f64, const double *q, int npw, int nat, const int4 *atoms,
                           const double *tau, const int *chan0, const int *lchan,
                           const double *tab, int nq, double dq, double pref, void *beta,
                           long ldb, hipStream_t s) {
  if (npw <= 0 || nat <= 0) return hipSuccess;
  const dim3 grid((npw + kBT - 1) / kBT, nat);
  if (f64)
    hipLaunchKernelGGL(beta_gen_kernel<double2>, grid, dim3(kBT), 0, s, q, npw, atoms, tau,
                       chan0, lchan, tab, nq, 1.0 / dq, pref, static_cast<double2 *>(beta),
                       ldb);
  else
    hipLaunchKernelGGL(beta_gen_kernel<float2>, grid, dim3(kBT), 0, s, q, npw, atoms, tau,
                       chan0, lchan, tab, nq, 1.0 / dq, pref, static_cast<float2 *>(beta),
                       ldb);
  return hipGetLastError();
}

hipError_t launch_nl_diag(bool f64, const void *beta, long ldb, int npw, int nat,
                          const int4 *atoms, const double2 *dmat, double *hdiag,
                          hipStream_t s) {
  if (npw <= 0 || nat <= 0) return hipSuccess;
  const dim3 grid((npw + 63) / 64);
  if (f64)
    hipLaunchKernelGGL(nl_diag_kernel<double2>, grid, dim3(64 * kDW), 0, s,
                       static_cast<const double2 *>(beta), ldb, npw, nat, atoms, dmat, hdiag);
  else
    hipLaunchKernelGGL(nl_diag_kernel<float2>, grid, dim3(64 * kDW), 0, s,
                       static_cast<const float2 *>(beta), ldb, npw, nat, atoms, dmat, hdiag);
  return hipGetLastError();
}

// Staging array of qeh_beta_generate_static (callers that cannot allocate):
// one per GPU, alive until the process ends.  Host code never passes the name
// itself to a kernel or a copy: it is a host-side stand-in, so each device's
// address is looked up once (with that device current) and kept.
static __device__ __align__(256) char scratch[QEH_BETA_STATIC_BYTES];

hipError_t beta_static_scratch(hipStream_t s, char **out) {
  static std::mutex mu;
  static std::vector<char *> ptr;   // per device, from hipGetSymbolAddress
  int dev = 0;
  hipError_t e = s ? hipStreamGetDevice(s, &dev) : hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(mu);
  if (dev >= (int)ptr.size()) ptr.resize(dev + 1, nullptr);
  if (!ptr[dev]) {
    int cur = 0;
    e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != dev && (e = hipSetDevice(dev)) != hipSuccess) return e;
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) {
      const hipError_t e2 = hipSetDevice(cur);
      if (e == hipSuccess) e = e2;
    }
    if (e != hipSuccess) return e;
    ptr[dev] = static_cast<char *>(p);
  }
  *out = ptr[dev];
  return hipSuccess;
}

}  // namespace qeh
