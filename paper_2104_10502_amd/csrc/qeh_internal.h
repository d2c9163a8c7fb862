// Internal declarations of the qeh library: context layout, FFT plans and the
// kernel launchers.  Not part of the public C ABI (include/qeh.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/qeh.h"

namespace qeh {

constexpr int kMaxPass = 8;
constexpr size_t kAlign = 256;
constexpr int kLdsMax = 160 * 1024;   // LDS per workgroup on gfx950

// Division by a fixed divisor d as q = (umulhi(n, m) + n) >> s, exact for
// n < 2^31 (round-up multiplier); built on the host, used in kernel index math.
struct FastDiv {
  uint32_t m, s, d;
};
FastDiv make_fastdiv(uint32_t d);

// One 1D mixed-radix transform of length n = prod radix[p].  Pass p combines
// radix[p] sub-transforms of length span[p] (span[0] = 1).  The decimation-
// in-time form takes digit-reversed input (element m at pos(m)) and returns
// natural order; the decimation-in-frequency form is its transpose.
struct FftDim {
  int n;
  int npass;
  int radix[kMaxPass];
  int span[kMaxPass];
  FastDiv nbf_div[kMaxPass];    // n / radix[p]
  FastDiv span_div[kMaxPass];   // span[p]
};

bool make_fft_dim(int n, FftDim *d);
// position of element m in the digit-reversed input of the DIT transform
int fft_digit_pos(const FftDim &d, int m);

// Plane-pass LDS geometry (elements of the working complex type).
struct PlaneGeom {
  int ldT;   // column stride of the x-extent column tile (>= N2, odd)
  int rc;    // rows processed together in the row phase
  int ldR;   // row stride of the row buffer (>= N1, odd)
  size_t lds_bytes;
  FastDiv ext_div, rc_div, rlast_div;   // ext, rc, rows of the last chunk
  int pb;            // lane-pair kernel: planes (bands of one z) per workgroup
  size_t lds_pair;   // lane-pair kernel: LDS bytes per workgroup
};

// Split plane path (planes too large for LDS): column groups of cg columns,
// row groups of rg rows (local column stride ldl).
struct SplitGeom {
  int cg, rg, ldl;
  size_t lds_col, lds_row;
  FastDiv cg_div, cglast_div, rg_div, rglast_div;
};

struct StickGeom {
  int ldz;   // z-line stride (>= N3, odd)
  int S;     // sticks per workgroup
  size_t lds_bytes;
  FastDiv s_div, slast_div;   // S, sticks of the last workgroup
};

// Device arrays of one context, all inside the caller's arena.
struct DevMaps {
  int *stick_off;    // [nst+1] first G of each stick
  int *gmap;         // [npw] s*ldz + digit-reversed z position (natural z for the
                     // lane-pair K1 / K3, whose ldz is N3 | 1 as well)
  int *tidx;         // [nst] plane-tile index c*ldT + pos_y(k mod N2); the lane-pair
                     // and lane-quad kernels take natural y (pos_y = identity)
  int *tidx_dit;     // [nst] the same with pos_y the y-DIT input position (always)
  int *xin;          // [N1] column c whose h sits at x-DIT input position p, or -1
  double *kin;       // [npw] |k+G|^2
  double *hdiag;     // [npw] diag(H)
  void *vs;          // [N3][N2][N1] V/N (double or float)
  void *tw;          // twiddles x | y | z (double2 or float2)
  void *beta;        // [nkb][npw] (double2 or float2)
  double2 *dmat;     // concatenated blocks
  double2 *qmat;     // overlap q blocks (same layout), or null
  int *pj0;          // [nkb] first projector of the atom block of i
  int *pnb;          // [nkb] size of that block
  int *pdoff;        // [nkb] offset of row i of its block in dmat
  int *chunk;        // [nchunk+1] atom-aligned projector ranges (<= 256 each)
  void *sbuf;        // [block][N3][nst] stick buffer (working complex type)
  void *part;        // [nsplit][block][nkb] split-K partials
  void *ps;          // [block][nkb] D * becp (working complex type; real floats on
                     // single-precision Gamma contexts)
  float2 *psi32;     // mixed form: [block][npw] single-precision copy of psi (K1)
  void *big;         // split plane path: [block][N3][ext][N2] (or null)
  double2 *gbuf;     // Gamma: [(block+1)/2][npw_fft] full-sphere H of band pairs (or null)
  int *colstart;     // [ext+1] first stick of each x-extent column
};

}  // namespace qeh

struct qeh_ctx {
  int npw = 0, nst = 0, nkb = 0, nat = 0;
  int npw_fft = 0;      // G-vectors of the FFT sphere (2 npw - 1 for Gamma cells, else npw)
  int gamma = 0;        // 1: real wavefunctions at k = 0, half sphere stored
  int has_q = 0;        // 1: overlap q blocks present (S != 1)
  int n1 = 0, n2 = 0, n3 = 0, ext = 0, hmin = 0;
  int block = 0, prec = 0;
  int plane_path = 0;   // 0 fused plane kernel, 1 split through HBM, 2 lane-pair kernel,
                        // 4 lane-quad kernel (FP64)
  int zpair = 0;        // 1: lane-pair K1 / K3 (gmap at natural z)
  int nsplit = 1, kchunk = 0;
  int wide = 0;         // 1: wide FP32 tiles for the projector products
  int nchunk = 0;
  qeh::FftDim dx{}, dy{}, dz{};
  qeh::PlaneGeom pg{};
  qeh::SplitGeom spg{};
  qeh::StickGeom sg{};
  int tw_off[3] = {0, 0, 0};
  hipStream_t stream = nullptr;
  qeh::DevMaps d{};
  char *arena = nullptr;
  size_t arena_bytes = 0;
  double vmean = 0.0;
  double omega = 0.0;   // cell volume
  // profiling
  bool prof = false;
  double stage_ms[QEH_NSTAGES] = {0};
  long stage_n[QEH_NSTAGES] = {0};
  std::vector<hipEvent_t> ev_pool;   // 2 events per recorded stage launch
  std::vector<int> ev_recs;          // stage id of each recorded launch
};

namespace qeh {

void set_error(const std::string &msg);
qeh_status hip_fail(hipError_t e, const char *what);

// ---- FFT path launchers (fft_kernels.hip) --------------------------------
// All take band count nbk (<= ctx block) and operate on the ctx stick buffer.
hipError_t launch_k1(const qeh_ctx *c, int nbk, const double2 *psi, int ldpsi);
// Gamma contexts: K1 of ceil(nbk/2) band pairs psi_2p + i psi_2p+1, read from
// the half-sphere bands (nbk rows, ldpsi) and expanded to the full sphere; with
// a device pair table, K1 of npairs pairs (rows pairs[p].x, pairs[p].y, the
// second < 0 for none).  copy32 (mixed form, natural pairs of a block of
// <= block bands): K1 also writes the block's single-precision copy psi32.
hipError_t launch_k1_gamma(const qeh_ctx *c, int nbk, const double2 *psi, int ldpsi,
                           const int2 *pairs = nullptr, int npairs = 0, bool copy32 = false);
hipError_t launch_k2(const qeh_ctx *c, int nbk);
hipError_t launch_k3(const qeh_ctx *c, int nbk, const double2 *psi, int ldpsi,
                     double2 *hpsi, int ldh, int add_kinetic);
size_t plane_lds_bytes(int prec, int ext, int n1, int n2, const PlaneGeom &g);
size_t stick_lds_bytes(int prec, int n3, const StickGeom &g);
// Lane-pair plane kernel: whether a compiled form exists for this precision and
// box, and its LDS bytes for pb planes of ext columns.
bool pair_plane_supported(int prec, int n1, int n2);
bool pair_z_supported(int prec, int n3);
bool quad_plane_supported(int prec, int n1, int n2);
size_t pair_z_lds_bytes(int n3);
size_t pair_plane_lds_bytes(int prec, int ext, int n2, int pb);
size_t quad_plane_lds_bytes(int prec, int ext, int n2, int pb);

// Charge density: row groups of rg rows, subgroups of bsub bands.
struct DensityGeom {
  int rg, ngroups, bsub;
  bool pair;    // lane-pair rows kernel (partial planes in the same layout)
  bool fused;   // fused plane kernel (lane pairs, or lane quads in FP64): no column
                // pass through HBM
  bool fused_quad;   // the FP64 lane-quad form of the fused kernel
  size_t lds;
  FastDiv rg_div, rglast_div;
};
bool density_geometry(const qeh_ctx *c, DensityGeom *dg);
// One block of nbk bands whose sticks K1 has written: inverse y columns into
// big, then partial[sub][z][y][x] = sum over subgroup sub of occ_b |psi_b|^2.
hipError_t launch_density_columns(const qeh_ctx *c, int nbk, void *big);
// zcol: N2 zero complex values (single precision), read by the lane-pair rows
// for positions beyond the x-extent
hipError_t launch_density_rows(const qeh_ctx *c, const DensityGeom &dg, int nbk, const void *big,
                               const double *occ_d, double *partial, const void *zcol);
// Fused form (dg.fused): sticks -> columns -> rows -> partial planes in one pass.
hipError_t launch_density_plane(const qeh_ctx *c, const DensityGeom &dg, int nbk,
                                const double *occ_d, double *partial);
hipError_t launch_density_reduce(const double *partial, int nsub, long npts, double scale,
                                 double *rho, int accumulate, hipStream_t s);

// ---- projectors built on the device (beta.cpp, beta_kernels.hip) -----------
// Workspace of the generator: k+G vectors [3][npw] (SoA), per-atom int4
// {species, first row, projectors, D offset}, positions [nat][3], channel
// offsets per species [nsp+1], l per channel, tables [channels][nq].
struct ProjgenLayout {
  size_t off_q, off_atom, off_tau, off_chan0, off_lchan, off_tab, total;
};
ProjgenLayout projgen_layout(const qeh_cell *c);   // c->projgen set
// Checks c->projgen against the cell (nproj per atom, table range over the
// sphere, finiteness); c's Miller list and lattice must already be valid.
qeh_status projgen_validate(const qeh_cell *c);
// Stages the generator inputs into work, writes beta (nkb rows of ldb complex,
// double2 if f64 else float2) and, when hdiag_dev is set, adds the nonlocal
// part of diag(H) (D blocks from dmat_dev); returns after the stream drained.
qeh_status projgen_run(const qeh_cell *c, bool f64, void *out, long ldb, char *work,
                       hipStream_t s, const double2 *dmat_dev, double *hdiag_dev);
hipError_t launch_beta_gen(bool f64, const double *q, int npw, int nat, const int4 *atoms,
                           const double *tau, const int *chan0, const int *lchan,
                           const double *tab, int nq, double dq, double pref, void *beta,
                           long ldb, hipStream_t s);
hipError_t launch_nl_diag(bool f64, const void *beta, long ldb, int npw, int nat,
                          const int4 *atoms, const double2 *dmat, double *hdiag,
                          hipStream_t s);
// Device address of the static staging array of qeh_beta_generate_static on
// the device of stream s (the current device when s is null); looked up once
// per device.
hipError_t beta_static_scratch(hipStream_t s, char **out);

// ---- complex GEMM launchers (gemm_kernels.hip) ----------------------------
// C[m][n] (+)= sum_k opA(A[m][k]) opB(B(k,n)), complex, MFMA.
//   A: element (m,k) at A[m*lda + k], conjugated if conjA.
//   B: bmode 0: element (k,n) at B[n*ldb + k] (conjugated if conjB);
//      bmode 1: element (k,n) at B[k*ldb + n].
//   Split-K: grid z = nsplit slices of kchunk; slice s writes
//      C + s*split_stride (accumulate must be 0 then).
enum GemmPrec { G_F64 = 0, G_F32 = 1 };
enum GemmType { T_D2 = 0, T_F2 = 1, T_F1 = 2 };   // operand storage (T_F1: real float)
struct GemmDesc {
  const void *A; long lda; int ta;
  const void *B; long ldb; int tb; int bmode;
  void *C; long ldc; int tc;
  int M, N, K;
  int conjA, conjB, accumulate;
  int nsplit, kchunk; long split_stride;
  int prec;
  int tile;   // FP32 tiles: 0 = 64 x 64; 1 = wide (128 x 128, Gamma beta^H psi 128 x 256)
  int rmode;  // 0 complex; 1 only Re(C) wanted (Im written 0); 2 A real (Im A ignored)
};
hipError_t launch_cgemm(const GemmDesc &g, hipStream_t s);

// ---- Davidson building blocks shared with the CG solver (davidson.cpp) ----
// out(i, j) = <X_i|Y_j> for i < nrow, j < ncol (col-major, ld), FP64 MFMA,
// split-K partials in `part` (16 * 32 * nrow * ncol bytes) summed in a fixed
// order; real inner products on Gamma contexts.
hipError_t reduce_cols(const qeh_ctx *c, const double2 *X, int nrow, const double2 *Y, int ncol,
                       double2 *out, int ld, double2 *part);
// rows b < nb: out_b = sum_j Y(j, b) X_j  (Y col-major ld, j < n)
hipError_t rotate(const qeh_ctx *c, const double2 *Y, int ld, int n, int nb, const double2 *X,
                  double2 *out);
constexpr int kReduceMaxSplit = 32;

// ---- conjugate-gradient solver kernels (cg_kernels.hip) ----
// Slots of the solver's device scalar array (doubles; complex values take two).
enum CgSlot {
  kCgLam = 0,     // Rayleigh quotient of the current band
  kCgRR = 2,      // <r|r>
  kCgGpr = 4,     // <g_prev|r>
  kCgGam = 6,     // <g|r>
  kCgGamp = 8,    // previous <g|r>
  kCgXD = 10,     // <x|d>
  kCgDD = 12,     // <d|d>
  kCgB = 14,      // <x|H dn>
  kCgC = 16,      // <dn|H dn>
  kCgBeta = 18,   // conjugation factor
  kCgC0 = 20,     // rotation of (x, dn): c0 (real)
  kCgC1 = 22,     //   and c1 (complex)
  kCgInvD = 24,   // 1 / ||d - <x|d> x||
  kCgXX = 26,     // <x|x> at a band's start
  kCgInvX = 28,   // 1 / ||x||
  kCgFirst = 30,  // 1 on a band's first iteration
  kCgSlots = 32
};
constexpr int kCgDotBlocks = 64;   // stage-1 blocks per inner product
constexpr int kCgMaxDots = 4;      // inner products per launch
struct CgDots {
  const double2 *a[kCgMaxDots];
  const double2 *b[kCgMaxDots];
  int dst[kCgMaxDots];   // slot of <a|b> (re, im)
};
// inner products <a_q|b_q> into sc[dst_q] (part: 2 * kCgDotBlocks * npairs doubles)
hipError_t launch_cg_dots(const CgDots &p, int npairs, int npw, int gamma, double *part,
                          double *sc, hipStream_t s);
hipError_t launch_cg_resid(const double2 *x, const double2 *hx, const double *hdiag,
                           const double *sc, double2 *r, double2 *g, int npw, int gamma,
                           hipStream_t s);
hipError_t launch_cg_project(double2 *g, const double2 *X, long ldx, const double2 *coef, int m,
                             int npw, hipStream_t s);
hipError_t launch_cg_scale(double2 *x, const double *sc, int npw, hipStream_t s);
hipError_t launch_cg_dir(const double2 *g, double2 *d, double2 *gp, const double *sc, int npw,
                         hipStream_t s);
hipError_t launch_cg_dnorm(double2 *d, const double2 *x, double2 *dn, const double *sc, int npw,
                           hipStream_t s);
hipError_t launch_cg_update(double2 *x, double2 *hx, const double2 *dn, const double2 *hd,
                            const double *sc, int npw, hipStream_t s);
hipError_t launch_cg_scalar(double *sc, int phase, hipStream_t s);

// C[m][n] (+)= sum_s part[s*stride + m*ldp + n], summed in double in split order.
hipError_t launch_splitk_reduce(const void *part, int tp, long stride, int nsplit, int M, int N,
                                long ldp, double2 *C, long ldc, int accumulate, hipStream_t s);

// Sum split-K partials (double2 or float2 partials, double accumulation) and
// apply the block-diagonal D: ps[b][i] = sum_j D_ij sum_s part[s][b][j].
// Gamma contexts: psi (ldpsi) are the block's bands, whose G = 0 values enter
// the real full-sphere projection (ignored otherwise).
// mat: the block-diagonal matrix applied (D, or the overlap's q; null = D).
hipError_t launch_dscale(const qeh_ctx *c, int nbk, const double2 *psi, long ldpsi,
                         const double2 *mat = nullptr);

// ---- dense Hermitian subspace solver (eigh_kernels.hip) --------------------
// Reduced problems up to kEigMaxN; column-major double2 matrices.
constexpr int kEigMaxN = 2048;
// Largest basis for which the Davidson's automatic choice takes the own solver:
// above it the one-stage Householder reduction streams the trailing matrix
// from HBM at every step (n = 2048: 86 ms per complex solve) and rocSOLVER's
// real solver of the Gamma path measured faster (512-atom cell: 12.8 against
// 13.6 s per Davidson run).
constexpr int kEigAutoMaxN = 1024;
// The solver's launchers take `wide`: true spreads each step over many
// workgroups (shortest time for one solve alone on the device), false keeps
// the Cholesky, the Householder reduction and the bisection on one workgroup
// each (least device time, for solves that share the device with others).
// S = L L^H in place (lower); info = 0 or the failing column + 1.  scr: 64 n
// doubles of scratch (the eigenpair scratch below is large enough and free).
hipError_t launch_chol(double2 *S, long ld, int n, int *info, double *scr, bool wide,
                       hipStream_t s);
// X = L^-1 B (mode 0, T = L lower), X = L^-1 M^H with B = M (mode 1), or
// X = U^-1 B (mode 2, T = U upper, backward); ncol columns, one wave each.
hipError_t launch_trsm(int mode, const double2 *T, long ldt, int n, const double2 *B, long ldb,
                       int ncol, double2 *X, long ldx, hipStream_t s);
// A = Q T Q^H (Householder, in place); tri = d[n] | e[n] | tau (double2)[n].
// scr: 12 n doubles of scratch (the multi-workgroup steps' vectors); the
// eigenpair scratch below is large enough and free at this point.
hipError_t launch_tridiag(double2 *A, long lda, int n, double *tri, double *scr,
                          const int *info_chol, bool wide, hipStream_t s);
// nb lowest eigenpairs of T: w[nb] ascending, Z (real, n x nb, ldz); scr holds
// eig_scratch_doubles(n) doubles; info 0 / nonzero on failure.
size_t eig_scratch_doubles(int n);
hipError_t launch_trieig(const double *tri, int n, int nb, double *w, double *Z, int ldz,
                         double *scr, int *info, const int *info_chol, bool wide, hipStream_t s);
// Zc = Q Zt (n x nb) through the reflectors stored in A by launch_tridiag.
hipError_t launch_backtr(const double2 *A, long lda, int n, const double *tri, const double *Zt,
                         int ldz, int nb, double2 *Zc, long ldc, const int *info_chol,
                         const int *info_eig, hipStream_t s);

// ---- Davidson helpers (dav_kernels.hip) ----------------------------------
// norms[b] = || Q_b - eps_b P_b ||^2 over npw (double), one launch; gamma = 1:
// half-sphere vectors, every G != 0 counted twice (G and -G).
hipError_t launch_resid_norms(const double2 *P, const double2 *Q, long ld, int npw,
                              int nb, const double *eps, double *norms, int gamma,
                              hipStream_t s);
// V[dst_b] = t / ||t||, t = (Q_b - eps_b P_b) / sqrt(1 + (h - eps_b)^2) for the
// listed bands b = idx[j], dst row j (norm as above).
hipError_t launch_precond(const double2 *P, const double2 *Q, long ld, int npw,
                          const int *idx, int nc, const double *eps, const double *hdiag,
                          double2 *V, long ldv, int gamma, hipStream_t s);
// Gamma point (real wavefunctions, half sphere of nh coefficients, G = 0 first):
// split the full-sphere result (2 nh - 1 entries, -G before G) of the local
// operator on band pairs psi_2p + i psi_2p+1 back into the two bands (+ kinetic
// term), writing hpsi.
hipError_t launch_gamma_unpack(const double2 *hc, long ldc, int nbk, int nh, const double2 *psi,
                               long ldpsi, const double *kin, double2 *hpsi, long ldh,
                               hipStream_t s);
// M(i, j) <- 2 Re M(i, j) - Re X_i[0] Re Y_j[0] (imaginary part zero): half-sphere
// sums turned into full-sphere inner products of real functions.
hipError_t launch_gamma_inner(double2 *M, long ld, int nrow, int ncol, const double2 *X,
                              const double2 *Y, long npw, hipStream_t s);
hipError_t launch_zero_g0_imag(double2 *psi, long ldpsi, int nb, hipStream_t s);
// n x n blocks, column-major: R = Re M, and M = R + 0 i.
hipError_t launch_real_part(const double2 *M, long ld, double *R, long ldr, int n,
                            hipStream_t s);
hipError_t launch_real_to_complex(const double *R, long ldr, double2 *M, long ld, int n,
                                  hipStream_t s);
// Copy rows; Hermitian fill; diag set etc.
hipError_t launch_copy_rows(const double2 *src, long lds, double2 *dst, long ldd, int npw,
                            int nrows, hipStream_t s);
// M[j][i] = conj(M[i][j]) for i in [0,n0), j in [n0,n1) (col-major, ld): fills
// the rows n0..n1 of the first n0 columns from the new columns.
hipError_t launch_herm_fill(double2 *M, long ld, int n0, int n1, hipStream_t s);
// M[0:n,0:n] = diag(d) (complex), or identity if d == null.
hipError_t launch_set_diag(double2 *M, long ld, int n, const double *d, hipStream_t s);
// dst (n x n, ldd) = (src + src^H)/2 (src n x n, lds), col-major.
hipError_t launch_hermitise_copy(const double2 *src, long lds, double2 *dst, long ldd, int n,
                                 hipStream_t s);
// L = lower triangle of M (zeros above), LH = L^H; all n x n col-major, ld.
hipError_t launch_tril_adjoint(const double2 *M, double2 *L, double2 *LH, long ld, int n,
                               hipStream_t s);
// p[0..n) = v (a kernel, not a memset, so the call can sit in captured graphs)
hipError_t launch_fill_int(int *p, int n, int v, hipStream_t s);
// finite check: flag[0] |= any non-finite in x[0..n) (doubles)
hipError_t launch_check_finite(const double *x, long n, int *flag, hipStream_t s);

}  // namespace qeh
