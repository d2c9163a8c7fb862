// Kernels of the band-by-band conjugate-gradient eigensolver (the paper's
// other iterative solver beside Davidson, section "Evolution of the
// GPU-enabled version").  The solver's scalars (Rayleigh quotient, inner
// products, the conjugation factor, the 2 x 2 line-minimisation rotation)
// live in a small device array `sc`: the vector kernels read them there and
// one single-thread kernel updates them, so an iteration needs the host only
// once, for the convergence test.  Every reduction runs in a fixed order
// (deterministic).
#include <algorithm>

#include "cplx.h"
#include "qeh_internal.h"

namespace qeh {
namespace {

constexpr int kCT = 256;

__device__ __forceinline__ double csum(double v, double *sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int s = kCT / 2; s > 0; s >>= 1) {
    if (t < s) sh[t] += sh[t + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// stage 1: block blockIdx.x of pair blockIdx.y sums conj(a) b over its chunk.
// Gamma vectors (half sphere, G = 0 first): the real inner product of the
// full-sphere vectors, sum_G w_G Re(conj(a_G) b_G) with w = 2 for G != 0.
__global__ __launch_bounds__(kCT) void cg_dot_partial(CgDots p, int npw, int gamma,
                                                      double *__restrict__ part) {
  __shared__ double sh[kCT];
  const int q = blockIdx.y;
  const double2 *a = p.a[q], *b = p.b[q];
  const int chunk = (npw + kCgDotBlocks - 1) / kCgDotBlocks;
  const int g0 = blockIdx.x * chunk, g1 = min(npw, g0 + chunk);
  double re = 0.0, im = 0.0;
  for (int g = g0 + threadIdx.x; g < g1; g += kCT) {
    const double2 u = a[g], v = b[g];
    const double w = (gamma && g > 0) ? 2.0 : 1.0;
    re += w * (u.x * v.x + u.y * v.y);
    im += w * (u.x * v.y - u.y * v.x);
  }
  re = csum(re, sh);
  im = csum(im, sh);
  if (threadIdx.x == 0) {
    double *o = part + 2 * ((long)q * kCgDotBlocks + blockIdx.x);
    o[0] = re;
    o[1] = gamma ? 0.0 : im;
  }
}

// stage 2: the partials of each pair summed in block order into sc[dst]
__global__ void cg_dot_final(CgDots p, const double *__restrict__ part, double *__restrict__ sc) {
  const int q = blockIdx.x;
  if (threadIdx.x != 0) return;
  double re = 0.0, im = 0.0;
  for (int k = 0; k < kCgDotBlocks; ++k) {
    re += part[2 * ((long)q * kCgDotBlocks + k)];
    im += part[2 * ((long)q * kCgDotBlocks + k) + 1];
  }
  sc[p.dst[q]] = re;
  sc[p.dst[q] + 1] = im;
}

// r = hx - lam x;  g = r / sqrt(1 + (h_G - lam)^2).  Gamma vectors: the
// imaginary part at G = 0 is set to zero (the coefficient is real), so the
// search directions and the updated band keep a real psi(0).
__global__ __launch_bounds__(kCT) void cg_resid(const double2 *__restrict__ x,
                                                const double2 *__restrict__ hx,
                                                const double *__restrict__ hdiag,
                                                const double *__restrict__ sc,
                                                double2 *__restrict__ r, double2 *__restrict__ g,
                                                int npw, int gamma) {
  const double lam = sc[kCgLam];
  for (int i = blockIdx.x * kCT + threadIdx.x; i < npw; i += gridDim.x * kCT) {
    const double2 a = x[i], h = hx[i];
    double2 ri = make_double2(h.x - lam * a.x, h.y - lam * a.y);
    if (gamma && i == 0) ri.y = 0.0;
    const double e = hdiag[i] - lam;
    const double w = 1.0 / sqrt(1.0 + e * e);
    r[i] = ri;
    g[i] = make_double2(w * ri.x, w * ri.y);
  }
}

// g -= sum_{j < m} coef_j X_j  (coef_j = <X_j|g>, in a fixed j order)
__global__ __launch_bounds__(kCT) void cg_project(double2 *__restrict__ g,
                                                  const double2 *__restrict__ X, long ldx,
                                                  const double2 *__restrict__ coef, int m,
                                                  int npw) {
  for (int i = blockIdx.x * kCT + threadIdx.x; i < npw; i += gridDim.x * kCT) {
    double2 v = g[i];
    for (int j = 0; j < m; ++j) {
      const double2 c = coef[j], xj = X[(long)j * ldx + i];
      v.x -= c.x * xj.x - c.y * xj.y;
      v.y -= c.x * xj.y + c.y * xj.x;
    }
    g[i] = v;
  }
}

// x *= sc[kCgInvX]
__global__ __launch_bounds__(kCT) void cg_scale(double2 *__restrict__ x,
                                                const double *__restrict__ sc, int npw) {
  const double s = sc[kCgInvX];
  for (int i = blockIdx.x * kCT + threadIdx.x; i < npw; i += gridDim.x * kCT) {
    const double2 a = x[i];
    x[i] = make_double2(s * a.x, s * a.y);
  }
}

// d = g + beta d (d = g when beta = 0: the previous band's d is not read);
// gp = g
__global__ __launch_bounds__(kCT) void cg_dir(const double2 *__restrict__ g,
                                              double2 *__restrict__ d, double2 *__restrict__ gp,
                                              const double *__restrict__ sc, int npw) {
  const double beta = sc[kCgBeta];
  for (int i = blockIdx.x * kCT + threadIdx.x; i < npw; i += gridDim.x * kCT) {
    const double2 a = g[i];
    if (beta != 0.0) {
      const double2 b = d[i];
      d[i] = make_double2(a.x + beta * b.x, a.y + beta * b.y);
    } else {
      d[i] = a;
    }
    gp[i] = a;
  }
}

// d -= <x|d> x;  dn = d / ||d||
__global__ __launch_bounds__(kCT) void cg_dnorm(double2 *__restrict__ d,
                                                const double2 *__restrict__ x,
                                                double2 *__restrict__ dn,
                                                const double *__restrict__ sc, int npw) {
  const double cr = sc[kCgXD], ci = sc[kCgXD + 1], s = sc[kCgInvD];
  for (int i = blockIdx.x * kCT + threadIdx.x; i < npw; i += gridDim.x * kCT) {
    const double2 a = d[i], u = x[i];
    const double2 v = make_double2(a.x - (cr * u.x - ci * u.y), a.y - (cr * u.y + ci * u.x));
    d[i] = v;
    dn[i] = make_double2(s * v.x, s * v.y);
  }
}

// x = c0 x + c1 dn;  hx = c0 hx + c1 hd  (c0 real, c1 complex)
__global__ __launch_bounds__(kCT) void cg_update(double2 *__restrict__ x, double2 *__restrict__ hx,
                                                 const double2 *__restrict__ dn,
                                                 const double2 *__restrict__ hd,
                                                 const double *__restrict__ sc, int npw) {
  const double c0 = sc[kCgC0], ar = sc[kCgC1], ai = sc[kCgC1 + 1];
  for (int i = blockIdx.x * kCT + threadIdx.x; i < npw; i += gridDim.x * kCT) {
    const double2 a = x[i], b = dn[i], h = hx[i], k = hd[i];
    x[i] = make_double2(c0 * a.x + ar * b.x - ai * b.y, c0 * a.y + ar * b.y + ai * b.x);
    hx[i] = make_double2(c0 * h.x + ar * k.x - ai * k.y, c0 * h.y + ar * k.y + ai * k.x);
  }
}

// The scalar steps, one thread.
//   phase 0 (band start): 1 / ||x||, first-iteration flag set;
//   phase 1: Polak-Ribiere factor beta = max(0, (gam - <g_prev|r>) / gam_prev)
//            (0 on a band's first iteration), gam_prev = gam;
//   phase 2: 1 / ||d - <x|d> x|| (0 when that vanishes);
//   phase 3: lower eigenpair of [[lam, b], [conj b, c]] over the orthonormal
//            pair (x, dn): eigenvector (c0 >= 0 real, c1), lam <- its value;
//            no move when the direction vanished.
__global__ void cg_scalar(double *__restrict__ sc, int phase) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (phase == 0) {
    const double n2 = sc[kCgXX];
    sc[kCgInvX] = n2 > 0.0 ? 1.0 / sqrt(n2) : 0.0;
    sc[kCgFirst] = 1.0;
    sc[kCgGamp] = 0.0;
  } else if (phase == 1) {
    const double gam = sc[kCgGam];
    double beta = 0.0;
    if (sc[kCgFirst] == 0.0 && sc[kCgGamp] != 0.0)
      beta = fmax(0.0, (gam - sc[kCgGpr]) / sc[kCgGamp]);
    sc[kCgBeta] = beta;
    sc[kCgGamp] = gam;
    sc[kCgFirst] = 0.0;
  } else if (phase == 2) {
    const double den = sc[kCgDD] - (sc[kCgXD] * sc[kCgXD] + sc[kCgXD + 1] * sc[kCgXD + 1]);
    sc[kCgInvD] = den > 0.0 ? 1.0 / sqrt(den) : 0.0;
  } else {
    if (sc[kCgInvD] == 0.0) {
      sc[kCgC0] = 1.0;
      sc[kCgC1] = 0.0;
      sc[kCgC1 + 1] = 0.0;
      return;
    }
    const double a = sc[kCgLam], br = sc[kCgB], bi = sc[kCgB + 1], c = sc[kCgC];
    const double bb = sqrt(br * br + bi * bi);
    const double h = 0.5 * (a - c);
    const double mu = 0.5 * (a + c) - sqrt(h * h + bb * bb);
    // (M - mu) v = 0: v = (c - mu, -conj b) or (b, mu - a), the longer one
    double v0r = c - mu, v0i = 0.0, v1r = -br, v1i = bi;
    const double n1 = (c - mu) * (c - mu) + bb * bb;
    const double n2 = bb * bb + (mu - a) * (mu - a);
    if (n2 > n1) {
      v0r = br;
      v0i = bi;
      v1r = mu - a;
      v1i = 0.0;
    }
    const double nn = sqrt(n1 > n2 ? n1 : n2);
    if (nn == 0.0) {
      sc[kCgC0] = 1.0;
      sc[kCgC1] = 0.0;
      sc[kCgC1 + 1] = 0.0;
      return;
    }
    v0r /= nn;
    v0i /= nn;
    v1r /= nn;
    v1i /= nn;
    // phase making c0 real and >= 0: multiply by conj(v0) / |v0|
    const double a0 = sqrt(v0r * v0r + v0i * v0i);
    double c1r, c1i, c0;
    if (a0 > 0.0) {
      const double pr = v0r / a0, pi = -v0i / a0;
      c0 = a0;
      c1r = v1r * pr - v1i * pi;
      c1i = v1r * pi + v1i * pr;
    } else {
      const double a1 = sqrt(v1r * v1r + v1i * v1i);
      c0 = 0.0;
      c1r = v1r / a1;
      c1i = v1i / a1;
    }
    sc[kCgC0] = c0;
    sc[kCgC1] = c1r;
    sc[kCgC1 + 1] = c1i;
    sc[kCgLam] = mu;
    sc[kCgLam + 1] = 0.0;
  }
}

int vec_blocks(int npw) { return std::max(1, std::min(2048, (npw + kCT - 1) / kCT)); }

}  // namespace

hipError_t launch_cg_dots(const CgDots &p, int npairs, int npw, int gamma, double *part,
                          double *sc, hipStream_t s) {
  if (npairs < 1 || npairs > kCgMaxDots) return hipErrorInvalidValue;
  hipLaunchKernelGGL(cg_dot_partial, dim3(kCgDotBlocks, npairs), dim3(kCT), 0, s, p, npw, gamma,
                     part);
  hipLaunchKernelGGL(cg_dot_final, dim3(npairs), dim3(64), 0, s, p, part, sc);
  return hipGetLastError();
}

hipError_t launch_cg_resid(const double2 *x, const double2 *hx, const double *hdiag,
                           const double *sc, double2 *r, double2 *g, int npw, int gamma,
                           hipStream_t s) {
  hipLaunchKernelGGL(cg_resid, dim3(vec_blocks(npw)), dim3(kCT), 0, s, x, hx, hdiag, sc, r, g,
                     npw, gamma);
  return hipGetLastError();
}

hipError_t launch_cg_project(double2 *g, const double2 *X, long ldx, const double2 *coef, int m,
                             int npw, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(cg_project, dim3(vec_blocks(npw)), dim3(kCT), 0, s, g, X, ldx, coef, m, npw);
  return hipGetLastError();
}

hipError_t launch_cg_scale(double2 *x, const double *sc, int npw, hipStream_t s) {
  hipLaunchKernelGGL(cg_scale, dim3(vec_blocks(npw)), dim3(kCT), 0, s, x, sc, npw);
  return hipGetLastError();
}

hipError_t launch_cg_dir(const double2 *g, double2 *d, double2 *gp, const double *sc, int npw,
                         hipStream_t s) {
  hipLaunchKernelGGL(cg_dir, dim3(vec_blocks(npw)), dim3(kCT), 0, s, g, d, gp, sc, npw);
  return hipGetLastError();
}

hipError_t launch_cg_dnorm(double2 *d, const double2 *x, double2 *dn, const double *sc, int npw,
                           hipStream_t s) {
  hipLaunchKernelGGL(cg_dnorm, dim3(vec_blocks(npw)), dim3(kCT), 0, s, d, x, dn, sc, npw);
  return hipGetLastError();
}

hipError_t launch_cg_update(double2 *x, double2 *hx, const double2 *dn, const double2 *hd,
                            const double *sc, int npw, hipStream_t s) {
  hipLaunchKernelGGL(cg_update, dim3(vec_blocks(npw)), dim3(kCT), 0, s, x, hx, dn, hd, sc, npw);
  return hipGetLastError();
}

hipError_t launch_cg_scalar(double *sc, int phase, hipStream_t s) {
  hipLaunchKernelGGL(cg_scalar, dim3(1), dim3(64), 0, s, sc, phase);
  return hipGetLastError();
}

}  // namespace qeh
