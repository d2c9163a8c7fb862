// Davidson helper kernels: residual norms, the diagonal preconditioner
// (listed among the GPU-ported kernels, section "Evolution of the
// GPU-enabled version"), and small reduced-matrix utilities.  All reductions
// run in a fixed order inside one workgroup per band (deterministic).
#include "cplx.h"
#include "qeh_internal.h"

namespace qeh {
namespace {

constexpr int kDT = 256;

__device__ __forceinline__ double block_sum(double v, double *sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int s = kDT / 2; s > 0; s >>= 1) {
    if (t < s) sh[t] += sh[t + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// Weight of stored coefficient g in a squared norm: 1, or for Gamma vectors
// (half sphere, G = 0 first) 2 for every G != 0, which stands for G and -G.
__device__ __forceinline__ double norm_weight(int g, int gamma) {
  return (gamma && g > 0) ? 2.0 : 1.0;
}

// one workgroup per band
__global__ __launch_bounds__(kDT) void resid_norms_kernel(const double2 *__restrict__ P,
                                                          const double2 *__restrict__ Q, long ld,
                                                          int npw, const double *__restrict__ eps,
                                                          double *__restrict__ norms, int gamma) {
  __shared__ double sh[kDT];
  const int b = blockIdx.x;
  const double e = eps[b];
  const double2 *p = P + (long)b * ld;
  const double2 *q = Q + (long)b * ld;
  double acc = 0.0;
  for (int g = threadIdx.x; g < npw; g += kDT) {
    const double2 a = p[g], h = q[g];
    const double rx = h.x - e * a.x, ry = h.y - e * a.y;
    acc += norm_weight(g, gamma) * (rx * rx + ry * ry);
  }
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) norms[b] = s;
}

__global__ __launch_bounds__(kDT) void precond_kernel(
    const double2 *__restrict__ P, const double2 *__restrict__ Q, long ld, int npw,
    const int *__restrict__ idx, const double *__restrict__ eps,
    const double *__restrict__ hdiag, double2 *__restrict__ V, long ldv, int gamma) {
  __shared__ double sh[kDT];
  const int j = blockIdx.x;
  const int b = idx[j];
  const double e = eps[b];
  const double2 *p = P + (long)b * ld;
  const double2 *q = Q + (long)b * ld;
  double2 *v = V + (long)j * ldv;
  double acc = 0.0;
  for (int g = threadIdx.x; g < npw; g += kDT) {
    const double2 a = p[g], h = q[g];
    const double x = hdiag[g] - e;
    const double w = 1.0 / sqrt(1.0 + x * x);
    const double rx = (h.x - e * a.x) * w, ry = (h.y - e * a.y) * w;
    v[g] = make_double2(rx, ry);
    acc += norm_weight(g, gamma) * (rx * rx + ry * ry);
  }
  const double s = block_sum(acc, sh);
  const double inv = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
  for (int g = threadIdx.x; g < npw; g += kDT) {
    const double2 a = v[g];
    v[g] = make_double2(a.x * inv, a.y * inv);
  }
}

__global__ void copy_rows_kernel(const double2 *__restrict__ src, long lds,
                                 double2 *__restrict__ dst, long ldd, int npw) {
  const int r = blockIdx.y;
  for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < npw; g += gridDim.x * blockDim.x)
    dst[(long)r * ldd + g] = src[(long)r * lds + g];
}

// col-major M(i,j) at M[i + j*ld].  For j in [n0,n1), i in [0,n0):
// M(j,i) = conj(M(i,j)).
__global__ void herm_fill_kernel(double2 *M, long ld, int n0, int n1) {
  const int j = n0 + blockIdx.y;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n0; i += gridDim.x * blockDim.x) {
    const double2 v = M[i + (long)j * ld];
    M[j + (long)i * ld] = make_double2(v.x, -v.y);
  }
}

__global__ void set_diag_kernel(double2 *M, long ld, int n, const double *d) {
  const int j = blockIdx.y;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    M[i + (long)j * ld] = make_double2(i == j ? (d ? d[i] : 1.0) : 0.0, 0.0);
}

__global__ void hermitise_copy_kernel(const double2 *src, long lds, double2 *dst, long ldd,
                                      int n) {
  const int j = blockIdx.y;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const double2 a = src[i + (long)j * lds];
    const double2 b = src[j + (long)i * lds];
    dst[i + (long)j * ldd] = make_double2(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
  }
}

__global__ void check_finite_kernel(const double *x, long n, int *flag) {
  int bad = 0;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
       i += (long)gridDim.x * blockDim.x)
    if (!isfinite(x[i])) bad = 1;
  if (bad) flag[0] = 1;   // plain store: any writer sets the same value
}

// From M (lower triangle valid, col-major ld): L = tril(M), LH = L^H.
__global__ void tril_and_adjoint_kernel(const double2 *M, double2 *L, double2 *LH, long ld,
                                        int n) {
  const int j = blockIdx.y;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const double2 a = i >= j ? M[i + (long)j * ld] : make_double2(0.0, 0.0);
    L[i + (long)j * ld] = a;
    LH[j + (long)i * ld] = make_double2(a.x, -a.y);
  }
}

__global__ void fill_int_kernel(int *p, int n, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// ---- Gamma point: two real bands per complex FFT ---------------------------
// K1 reads band pairs psi_2p + i psi_2p+1 straight from the half-sphere bands;
// the full-sphere result of K3 (2 nh - 1 entries: index f < nh - 1 is -G of
// stored h = nh - 1 - f, index f >= nh - 1 is stored h = f - (nh - 1)) is
// separated here.
// From C = F(V psi_a) + i F(V psi_b) on the full sphere: F(V psi_a)(G) =
// (C(G) + conj C(-G)) / 2, F(V psi_b)(G) = (C(G) - conj C(-G)) / (2i); plus
// the kinetic term.  Writes hpsi (overwrites).
__global__ void gamma_unpack_kernel(const double2 *__restrict__ hc, long ldc, int nbk, int nh,
                                    const double2 *__restrict__ psi, long ldpsi,
                                    const double *__restrict__ kin, double2 *__restrict__ hpsi,
                                    long ldh) {
  const int h = blockIdx.x * blockDim.x + threadIdx.x;
  const int p = blockIdx.y;
  if (h >= nh) return;
  const double2 cp = hc[(long)p * ldc + (nh - 1) + h];
  const double2 cm = hc[(long)p * ldc + (nh - 1) - h];
  const double k = kin[h];
  const int a = 2 * p, b = 2 * p + 1;
  {
    double2 v = psi[(long)a * ldpsi + h];
    if (h == 0) v.y = 0.0;
    hpsi[(long)a * ldh + h] =
        make_double2(0.5 * (cp.x + cm.x) + k * v.x, 0.5 * (cp.y - cm.y) + k * v.y);
  }
  if (b < nbk) {
    double2 v = psi[(long)b * ldpsi + h];
    if (h == 0) v.y = 0.0;
    hpsi[(long)b * ldh + h] =
        make_double2(0.5 * (cp.y + cm.y) + k * v.x, -0.5 * (cp.x - cm.x) + k * v.y);
  }
}

// Inner products of Gamma vectors from the half-sphere sums S(i, j) =
// sum_h conj(X_i[h]) Y_j[h]: <X_i|Y_j> = 2 Re S(i, j) - X_i[0] Y_j[0] (real
// parts at G = 0), stored with zero imaginary part.  M col-major (ld), rows
// i < nrow, columns j < ncol.
__global__ void gamma_inner_kernel(double2 *M, long ld, int nrow, const double2 *__restrict__ X,
                                   const double2 *__restrict__ Y, long npw) {
  const int j = blockIdx.y;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nrow; i += gridDim.x * blockDim.x) {
    const double2 v = M[i + (long)j * ld];
    M[i + (long)j * ld] =
        make_double2(2.0 * v.x - X[(long)i * npw].x * Y[(long)j * npw].x, 0.0);
  }
}

// n x n blocks (column-major, leading dimensions given): real part out, and a
// real matrix back in as complex with zero imaginary part.
__global__ void real_part_kernel(const double2 *__restrict__ M, long ld, double *__restrict__ R,
                                 long ldr, int n) {
  const int j = blockIdx.y;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    R[i + (long)j * ldr] = M[i + (long)j * ld].x;
}

__global__ void real_to_complex_kernel(const double *__restrict__ R, long ldr,
                                       double2 *__restrict__ M, long ld, int n) {
  const int j = blockIdx.y;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    M[i + (long)j * ld] = make_double2(R[i + (long)j * ldr], 0.0);
}

__global__ void zero_g0_imag_kernel(double2 *psi, long ldpsi, int nb) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < nb) psi[(long)b * ldpsi].y = 0.0;
}

}  // namespace

hipError_t launch_tril_adjoint(const double2 *M, double2 *L, double2 *LH, long ld, int n,
                               hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(tril_and_adjoint_kernel, dim3((n + 255) / 256, n), dim3(256), 0, s, M, L,
                     LH, ld, n);
  return hipGetLastError();
}

hipError_t launch_fill_int(int *p, int n, int v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_int_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_resid_norms(const double2 *P, const double2 *Q, long ld, int npw, int nb,
                              const double *eps, double *norms, int gamma, hipStream_t s) {
  if (nb <= 0) return hipSuccess;
  hipLaunchKernelGGL(resid_norms_kernel, dim3(nb), dim3(kDT), 0, s, P, Q, ld, npw, eps, norms,
                     gamma);
  return hipGetLastError();
}

hipError_t launch_precond(const double2 *P, const double2 *Q, long ld, int npw, const int *idx,
                          int nc, const double *eps, const double *hdiag, double2 *V, long ldv,
                          int gamma, hipStream_t s) {
  if (nc <= 0) return hipSuccess;
  hipLaunchKernelGGL(precond_kernel, dim3(nc), dim3(kDT), 0, s, P, Q, ld, npw, idx, eps, hdiag,
                     V, ldv, gamma);
  return hipGetLastError();
}

hipError_t launch_gamma_unpack(const double2 *hc, long ldc, int nbk, int nh, const double2 *psi,
                               long ldpsi, const double *kin, double2 *hpsi, long ldh,
                               hipStream_t s) {
  if (nbk <= 0) return hipSuccess;
  hipLaunchKernelGGL(gamma_unpack_kernel, dim3((nh + 255) / 256, (nbk + 1) / 2), dim3(256), 0, s,
                     hc, ldc, nbk, nh, psi, ldpsi, kin, hpsi, ldh);
  return hipGetLastError();
}

hipError_t launch_gamma_inner(double2 *M, long ld, int nrow, int ncol, const double2 *X,
                              const double2 *Y, long npw, hipStream_t s) {
  if (nrow <= 0 || ncol <= 0) return hipSuccess;
  hipLaunchKernelGGL(gamma_inner_kernel, dim3((nrow + 255) / 256, ncol), dim3(256), 0, s, M, ld,
                     nrow, X, Y, npw);
  return hipGetLastError();
}

hipError_t launch_real_part(const double2 *M, long ld, double *R, long ldr, int n,
                            hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(real_part_kernel, dim3((n + 255) / 256, n), dim3(256), 0, s, M, ld, R, ldr,
                     n);
  return hipGetLastError();
}

hipError_t launch_real_to_complex(const double *R, long ldr, double2 *M, long ld, int n,
                                  hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(real_to_complex_kernel, dim3((n + 255) / 256, n), dim3(256), 0, s, R, ldr, M,
                     ld, n);
  return hipGetLastError();
}

hipError_t launch_zero_g0_imag(double2 *psi, long ldpsi, int nb, hipStream_t s) {
  if (nb <= 0) return hipSuccess;
  hipLaunchKernelGGL(zero_g0_imag_kernel, dim3((nb + 255) / 256), dim3(256), 0, s, psi, ldpsi,
                     nb);
  return hipGetLastError();
}


hipError_t launch_copy_rows(const double2 *src, long lds, double2 *dst, long ldd, int npw,
                            int nrows, hipStream_t s) {
  if (nrows <= 0) return hipSuccess;
  const int gx = (npw + 255) / 256 < 64 ? (npw + 255) / 256 : 64;
  hipLaunchKernelGGL(copy_rows_kernel, dim3(gx, nrows), dim3(256), 0, s, src, lds, dst, ldd, npw);
  return hipGetLastError();
}

hipError_t launch_herm_fill(double2 *M, long ld, int n0, int n1, hipStream_t s) {
  if (n1 <= n0 || n0 <= 0) return hipSuccess;
  hipLaunchKernelGGL(herm_fill_kernel, dim3((n0 + 255) / 256, n1 - n0), dim3(256), 0, s, M, ld,
                     n0, n1);
  return hipGetLastError();
}

hipError_t launch_set_diag(double2 *M, long ld, int n, const double *d, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(set_diag_kernel, dim3((n + 255) / 256, n), dim3(256), 0, s, M, ld, n, d);
  return hipGetLastError();
}

hipError_t launch_hermitise_copy(const double2 *src, long lds, double2 *dst, long ldd, int n,
                                 hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(hermitise_copy_kernel, dim3((n + 255) / 256, n), dim3(256), 0, s, src, lds,
                     dst, ldd, n);
  return hipGetLastError();
}

hipError_t launch_check_finite(const double *x, long n, int *flag, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  long blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(check_finite_kernel, dim3((unsigned)blocks), dim3(256), 0, s, x, n, flag);
  return hipGetLastError();
}

}  // namespace qeh
