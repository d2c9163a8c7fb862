/*
 * qeh.h - plane-wave Kohn-Sham H|psi> and block-Davidson eigensolver on one
 * AMD MI355X (gfx950).  C ABI: plain pointers and sizes, no library types in
 * the arguments.
 *
 * The paper (Quantum ESPRESSO toward the exascale) asks its extracted
 * libraries to expose plain-array interfaces without structured arguments
 * (section "Domain-specific mathematical libraries"), to keep the iterative
 * solver separate from the Hamiltonian builder it calls (same section), and
 * lists the kernels ported to GPUs: local-potential, pseudopotential and
 * kinetic contributions to the Hamiltonian, the preconditioner, the overlap
 * operator (the identity for the norm-conserving form used here) and the
 * Davidson solver (section "Evolution of the GPU-enabled version").
 *
 * Units: Rydberg atomic units (lengths in bohr, energies in Ry).
 * Complex numbers: interleaved (re, im) pairs of double.
 * Bands: one band per row, psi[b * ldpsi + G], plane-wave index fastest.
 * Memory: the library never allocates device memory.  Device storage is an
 *   arena the caller allocates (size from the *_plan call) and keeps alive
 *   until the matching destroy.  Every host array passed in is copied before
 *   the call returns; the caller keeps ownership of everything it passes.
 * Errors: every call returns a qeh_status; nothing aborts.  qeh_last_error()
 *   gives a thread-local message for the last failing call on that thread.
 *   Errors of asynchronous device work surface at the next synchronising call.
 * Threads: a context is used by one thread at a time; its work is ordered on
 *   the HIP stream given at creation.
 */
#ifndef QEH_H
#define QEH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int qeh_status;
enum {
  QEH_OK = 0,
  QEH_ERR_INVALID = -1,        /* bad argument, shape or Miller list            */
  QEH_ERR_NOMEM = -2,          /* arena / workspace smaller than the plan       */
  QEH_ERR_NUMERIC = -3,        /* NaN or Inf in an input                        */
  QEH_ERR_CHOLESKY = -4,       /* overlap matrix not positive definite twice    */
  QEH_ERR_NOT_CONVERGED = -5,  /* Davidson hit maxiter (results still written)  */
  QEH_ERR_REJECTED = -6,       /* served request can never fit the budget       */
  QEH_ERR_DEVICE = -7,         /* a HIP call failed                             */
  QEH_ERR_BUSY = -8,           /* served request not finished yet               */
  QEH_RCI_APPLY_H = 1          /* qeh_dav_rci_step: apply H to the request      */
};

enum { QEH_FP64 = 0, QEH_MIXED = 1 };
/* QEH_FP64:  every step in double precision.
 * QEH_MIXED: FFTs, the V_loc multiply and the projector GEMMs in single
 *            precision with single-precision accumulation (long sums split
 *            into fixed chunks reduced in double); the kinetic term, psi,
 *            H psi and the whole Davidson subspace algebra in double.       */

/* Projectors built on the device from radial tables: the "calculation of
 * pseudopotential terms" of the quantum-engine modules (section
 * "Quantum-engine modules", item viii), done where the Hamiltonian lives.
 * Standard separable form; for projector i = (atom a of species s, radial
 * channel c of s with angular momentum l, real harmonic m) and q = k + G:
 *   beta_i(q) = 4 pi / sqrt(Omega) (-i)^l F_c(|q|) Y_lm(q/|q|) exp(-i q . tau_a),
 *   F_c(q)    = int_0^inf r^2 beta_c(r) j_l(q r) dr,
 * with F_c given as a table F_c(j dq), j < nq, and evaluated at |q| by the
 * cubic Lagrange polynomial through table points j-1 .. j+2 where
 * j = max(1, floor(|q| / dq)).  Real harmonics of the unit vector (x, y, z)
 * (all zero-argument values taken at (0, 0, 0) when q = 0), in this order:
 *   l = 0: 1/sqrt(4 pi);  l = 1: sqrt(3/(4 pi)) (x, y, z);
 *   l = 2: sqrt(15/(4 pi)) (xy, yz, zx), sqrt(5/(16 pi)) (3z^2 - 1),
 *          sqrt(15/(16 pi)) (x^2 - y^2).
 * Projector order: atoms in order; within an atom its species' channels in
 * order; within a channel m as listed.  nproj[a] must equal the sum of
 * 2 l + 1 over the channels of atom a's species.  All pointers are HOST
 * pointers. */
typedef struct {
  const double *tau;      /* [nat][3] cartesian atom positions (bohr)          */
  const int *ityp;        /* [nat] species of each atom, in [0, nsp)           */
  int nsp;                /* species (>= 1)                                    */
  const int *nchan;       /* [nsp] radial channels per species (>= 0)          */
  const int *lchan;       /* [sum nchan] l (0, 1 or 2) per channel, species by
                             species                                            */
  int nq;                 /* table points per channel (>= 4)                   */
  double dq;              /* table spacing (bohr^-1, > 0); every |k+G| of the
                             sphere must satisfy |k+G| <= (nq - 3) dq          */
  const double *tab;      /* [sum nchan][nq] F_c(j dq), same channel order     */
} qeh_projgen;

/* One cell at one k-point.  Every pointer is a HOST pointer, read during
 * qeh_ctx_plan / qeh_ctx_create only. */
typedef struct {
  double lattice[9];      /* rows a1, a2, a3 (bohr), row-major               */
  int fft[3];             /* N1, N2, N3; prime factors in {2,3,5,7}, <= 1024 */
  double kpt[3];          /* cartesian k (bohr^-1)                           */
  int npw;                /* plane waves in the sphere                       */
  const int *miller;      /* [npw][3] (h,k,l), lexicographic, each (h,k)
                             stick a contiguous run of consecutive l, and
                             max(m_i) - min(m_i) < N_i on every axis         */
  const double *vloc;     /* [N3][N2][N1] real local potential on the grid
                             r_j = sum_i j_i/N_i a_i (Ry), x fastest         */
  int nat;                /* atoms (may be 0)                                */
  const int *nproj;       /* [nat] projectors per atom                       */
  const double *beta;     /* complex [nkb][npw], nkb = sum nproj; includes
                             1/sqrt(Omega) and exp(-i(k+G).tau)              */
  const double *dmat;     /* complex: per-atom Hermitian nproj x nproj D
                             blocks (row-major), concatenated (Ry)           */
  int precision;          /* QEH_FP64 or QEH_MIXED                           */
  int block;              /* bands per H-application launch (>= 1)           */
  const qeh_projgen *projgen;   /* optional: when beta is NULL and there are
                             projectors, qeh_ctx_create builds beta on the
                             device from these tables (and diag(H) with it);
                             ignored when beta is given                        */
  int gamma;              /* 1: real wavefunctions at k = 0 (see below); 0: general k */
  const double *qmat;     /* optional, complex, layout of dmat: per-atom
                             Hermitian q blocks of the overlap
                             S = 1 + sum_ij |beta_i> q_ij <beta_j|; NULL: S = 1 */
} qeh_cell;

/* The overlap operator (listed among the GPU-ported kernels, section
 * "Evolution of the GPU-enabled version"; ultrasoft / PAW form): with qmat
 * set, a context applies S with qeh_apply_s, and qeh_davidson solves the
 * generalized problem H psi = eps S psi (basis V, H V and S V; reduced pair
 * V^H H V, V^H S V; residuals H psi - eps S psi; S-orthonormal Ritz vectors,
 * psi^H S psi = I).  S must be positive definite (q >= 0 suffices); Gamma
 * cells need real q blocks. */

/* Gamma-point cells (gamma = 1): the real-wavefunction case ("k = 0 only
 * sampling" of section "Evolution of the GPU-enabled version").  With
 * psi(r) real, psi(-G) = conj(psi(G)), so only half of the sphere is stored:
 *   kpt must be (0, 0, 0);
 *   miller lists the half sphere: (0,0,0) first, then every G of the sphere
 *     that follows (0,0,0) lexicographically (h > 0, or h = 0 and k > 0, or
 *     h = k = 0 and l > 0), in lexicographic order; npw counts these;
 *   psi, hpsi, beta rows and the Davidson vectors hold those npw coefficients;
 *     the imaginary part of psi(G = 0) is not referenced (qeh_davidson sets it
 *     to zero in psi_inout); beta_i(G = 0) must be real and D real symmetric
 *     (projectors real in real space);
 *   two bands share one complex 3D FFT (psi_a + i psi_b is transformed and
 *     the two results separated from the values at G and -G);
 *   inner products are 2 Re sum_G conj(a_G) b_G - a_0 b_0 over the stored
 *     half, so the subspace problem is real symmetric;
 *   qeh_density pairs consecutive bands of equal occupation into one complex
 *     transform (|psi_a + i psi_b|^2 = psi_a^2 + psi_b^2 for real functions);
 *     other bands go alone. */

typedef struct qeh_ctx qeh_ctx;

/* Device bytes the context needs for this cell (validates the cell). */
qeh_status qeh_ctx_plan(const qeh_cell *cell, size_t *arena_bytes);

/* Build the index maps on the host (stick table, box positions, |k+G|^2,
 * diag(H)), copy them, V/N, beta and D into the arena, and bind the context
 * to hip_stream (a hipStream_t; NULL = the null stream).  arena must be a
 * device pointer with 256-byte alignment and >= the planned size.  The
 * copies are complete when the call returns.  With beta NULL and projgen
 * set, beta is built on the device instead (as qeh_beta_generate, in the
 * context's precision) and the nonlocal part of diag(H) is summed from it
 * there; the plan then includes the generator's workspace. */
qeh_status qeh_ctx_create(const qeh_cell *cell, void *arena, size_t arena_bytes,
                          void *hip_stream, qeh_ctx **out);

qeh_status qeh_ctx_destroy(qeh_ctx *ctx);

/* H|psi> for nb bands: hpsi_b = |k+G|^2 psi_b + V_loc psi_b + beta D beta^H psi_b.
 * psi and hpsi are DEVICE pointers (complex, rows of length npw with leading
 * dimensions ldpsi, ldh >= npw, in complex elements); they must not overlap.
 * Enqueued on the context stream in launches of `block` bands; returns
 * without waiting.  Result is independent of how bands are grouped. */
qeh_status qeh_apply_h(qeh_ctx *ctx, int nb, const double *psi, int ldpsi,
                       double *hpsi, int ldh);

/* S psi for nb bands (same layout rules as qeh_apply_h): spsi = psi +
 * beta q beta^H psi, with beta^H psi and the product in the context's
 * precision (single precision in QEH_MIXED, accumulated onto the FP64 psi).
 * A context without qmat copies psi.  Enqueued on the context stream. */
qeh_status qeh_apply_s(qeh_ctx *ctx, int nb, const double *psi, int ldpsi, double *spsi,
                       int ldsp);

/* The three parts of H separately (same layout rules as qeh_apply_h):
 * part 0 = kinetic + local (the FFT path), part 1 = nonlocal only. */
qeh_status qeh_apply_h_part(qeh_ctx *ctx, int part, int nb, const double *psi,
                            int ldpsi, double *hpsi, int ldh);

/* Charge density of a set of bands: the charge density generation listed
 * among the GPU-ported kernels (section "Evolution of the GPU-enabled
 * version"), the step that follows the diagonalisation in the
 * self-consistency cycle.
 *   rho[(z * N2 + y) * N1 + x] = (1 / Omega) sum_b occ[b] |psi_b(r)|^2,
 *   psi_b(r) = sum_G psi_b(G) exp(i (k + G) . r),  r = x/N1 a1 + y/N2 a2 + z/N3 a3,
 * with Omega = |det(lattice)|.  For bands normalised to sum_G |psi(G)|^2 = 1,
 * (Omega / N) sum_r rho = sum_b occ[b].
 *   psi  : device, nb rows of npw complex values (row stride ldpsi >= npw),
 *          same layout as qeh_apply_h;
 *   occ  : host, nb finite weights (any sign);
 *   rho  : device, N1 N2 N3 doubles, overwritten (zero when nb = 0);
 *   work : device workspace of qeh_density_plan bytes, 256-byte aligned,
 *          owned by the caller.
 * Bands go through in blocks of the context's block size: K1 (sticks and
 * inverse z), inverse y columns into the workspace, then inverse x rows with
 * the occupation-weighted |psi|^2 summed in double in a fixed order (the
 * result does not depend on timing).  Contexts on the register plane
 * kernels (lane pairs in the mixed form, lane quads in FP64) run the y and x
 * transforms as one fused pass per z plane instead (no column workspace);
 * QEH_DENSITY_KERNEL=rows or =generic, read per call, selects the unfused
 * lane-pair rows or the LDS-pass rows (test hooks).  Precision: the
 * context's (the mixed form transforms in FP32 and sums in FP64).  Blocking: returns after the
 * device work of the call has finished.  Errors: QEH_ERR_INVALID for null
 * pointers, ldpsi < npw, a short or misaligned workspace, a non-finite
 * occupation, or a box whose rows exceed the row kernel (N1 > 2048). */
qeh_status qeh_density_plan(const qeh_ctx *ctx, size_t *work_bytes);
qeh_status qeh_density(qeh_ctx *ctx, int nb, const double *psi, int ldpsi,
                       const double *occ, double *rho, void *work, size_t work_bytes);

/* Projectors of cell->projgen for the sphere of cell (lattice, kpt, npw,
 * miller, nat, nproj; vloc, beta and dmat are not read), written on the
 * device: beta (DEVICE) holds nkb rows of ldb >= npw complex elements, row i
 * = projector i, as double pairs when precision is QEH_FP64 and as float
 * pairs (each value computed in double, then rounded) when QEH_MIXED.  work:
 * DEVICE workspace of qeh_beta_plan bytes, 256-byte aligned, caller-owned
 * (it receives the k+G vectors, positions and tables).  Work is ordered on
 * hip_stream (a hipStream_t, NULL = null stream); the call returns after it
 * has finished.  Errors: QEH_ERR_INVALID for a missing or inconsistent
 * projgen (species or l out of range, nproj not matching the channels, a
 * table too short for the sphere, dq <= 0, nq < 4), null pointers, ldb < npw
 * or a short / misaligned workspace; QEH_ERR_NUMERIC for a non-finite table
 * value or position. */
qeh_status qeh_beta_plan(const qeh_cell *cell, size_t *work_bytes);
qeh_status qeh_beta_generate(const qeh_cell *cell, int precision, void *beta, long ldb,
                             void *work, size_t work_bytes, void *hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * projectors as qeh_beta_generate (bitwise), with the generator's inputs
 * staged in a static device array of QEH_BETA_STATIC_BYTES per GPU instead
 * of a caller workspace.  The call allocates nothing (no hipMalloc, no
 * library allocation); the array is created with the library's code object on
 * each GPU it runs on and kept until the process ends.  The inputs it stages
 * are 24 npw + 40 nat + 4 (nsp + 1 + channels) + 8 channels nq bytes, each
 * field rounded up to 256 (qeh_beta_plan gives the figure): cells needing
 * more get QEH_ERR_NOMEM and must use qeh_beta_generate.  beta (DEVICE),
 * ldb, precision and hip_stream as for qeh_beta_generate (the array used is
 * the one on the stream's device); returns after the work has finished.
 * All calls on one GPU share its array: calls that overlap in time on the
 * same GPU (two host threads) race and must be serialised by the caller. */
#define QEH_BETA_STATIC_BYTES (8u << 20)
qeh_status qeh_beta_generate_static(const qeh_cell *cell, int precision, void *beta, long ldb,
                                    void *hip_stream);

/* Davidson options: nvecx = maximum basis size (>= 2 nb; 0 = 2 nb),
 * rtol = residual 2-norm threshold (Ry), maxiter = iterations (0 = 200),
 * subspace = solver of the reduced problem H_r y = eps S_r y:
 *   QEH_SUBSPACE_AUTO (0): the library's own when nvecx <= 1024, else rocSOLVER;
 *   QEH_SUBSPACE_OWN (1): the library's own HIP solver (nvecx <= 2048 only):
 *     Cholesky, triangular solves, Householder tridiagonalisation, bisection
 *     and inverse iteration, back-transformation; deterministic (fixed
 *     summation orders), no library calls; about a dozen launches per
 *     iteration, plus one per Householder step above order 64 and one per
 *     16-column Cholesky panel (the steps spread over many workgroups: the
 *     shortest time for one solve alone on the device; the request
 *     server's jobs keep them on one workgroup each);
 *   QEH_SUBSPACE_ROCSOLVER (2): rocSOLVER potrf / trtri / heevd (syevd for
 *     Gamma contexts) with the library's MFMA products around them.
 * In QEH_MIXED the residual threshold is thr = max(rtol, 1e-5), since
 * single precision limits how small the residual can get, and the solve runs
 * in two phases when refine is set:
 *   1. H applied in single precision (the context's form) until every band
 *      has ||r|| <= thr, or a residual that has not dropped by 10% in 3
 *      iterations, or a Ritz value that moved by <= 1e-8 Ry in one (the
 *      single-precision floor);
 *   2. the same basis with H V recomputed, and H applied from then on, in
 *      FP64 through refine
 *      (a QEH_FP64 context of the same cell: same Miller list, k, V,
 *      projectors and D, on the same HIP stream, with the same npw, box,
 *      projector count and Gamma flag) until every band has ||r|| <= thr,
 *      that residual computed in FP64; the eigenvalue error is then the
 *      FP64 form's at residual thr.
 * Without refine the mixed form stops at phase 1's rules, with the floor
 * accepted only while ||r|| <= 10 thr (3 iterations without a 10% drop) or
 * <= 100 thr (5 iterations, or a settled Ritz value); its eigenvalue error is
 * then bounded by ||r||^2 / gap with ||r|| up to 100 thr. */
enum { QEH_SUBSPACE_AUTO = 0, QEH_SUBSPACE_OWN = 1, QEH_SUBSPACE_ROCSOLVER = 2 };
typedef struct {
  int nvecx;
  double rtol;
  int maxiter;
  int subspace;
  qeh_ctx *refine;   /* QEH_MIXED solves only, may be NULL: see below */
} qeh_dav_opts;

typedef struct {
  int iters;              /* Rayleigh-Ritz steps taken                       */
  int notconv;            /* bands not converged at exit                     */
  int restarts;           /* basis restarts (including Cholesky recoveries)  */
  long band_applies;      /* bands passed through H                          */
  double resid_max;       /* max_i ||H psi_i - eps_i psi_i|| at exit         */
  double t_total;         /* wall seconds                                    */
  double t_hpsi;          /* seconds in H application (device events)        */
  double t_subspace;      /* seconds in reductions + subspace eigensolve     */
  int refine_iters;       /* of iters, those with H applied in FP64 through
                             qeh_dav_opts.refine (QEH_MIXED)                  */
} qeh_dav_info;

/* Device workspace bytes for qeh_davidson with nb bands. */
qeh_status qeh_davidson_plan(const qeh_ctx *ctx, int nb, const qeh_dav_opts *opts,
                             size_t *work_bytes);

/* Lowest nb eigenpairs of H by block Davidson, starting from psi_inout
 * (DEVICE, nb rows, ldpsi).  On return psi_inout holds orthonormal Ritz
 * vectors and eig (HOST, nb doubles) the ascending Ritz values.  Blocks
 * until done.  Returns QEH_ERR_NOT_CONVERGED (results written) at maxiter,
 * QEH_ERR_CHOLESKY if the overlap matrix fails twice in a row. */
qeh_status qeh_davidson(qeh_ctx *ctx, int nb, double *psi_inout, int ldpsi,
                        double *eig, const qeh_dav_opts *opts, void *work,
                        size_t work_bytes, qeh_dav_info *info);

/* Band-by-band preconditioned conjugate-gradient eigensolver, the paper's
 * other iterative solver of the Kohn-Sham problem beside Davidson (section
 * "Evolution of the GPU-enabled version"): the lowest nb eigenpairs of H (the
 * standard problem: a context with q blocks is rejected), starting from
 * psi_inout (DEVICE, nb rows, ldpsi >= npw).  Steps: Rayleigh-Ritz of the
 * starting block; then for each band in turn, conjugate-gradient minimisation
 * of the Rayleigh quotient with the Davidson preconditioner
 * 1 / sqrt(1 + (diag(H)_G - lam)^2), the search direction kept orthogonal to
 * the bands below (Polak-Ribiere conjugation, restarted when negative) and an
 * exact line minimisation over the current vector and the direction; a final
 * Rayleigh-Ritz of the block.  Band b stops when ||H x - lam x|| <= thr
 * (thr = rtol, or max(rtol, 1e-5) for QEH_MIXED) or after maxiter
 * iterations (QEH_ERR_NOT_CONVERGED, results written).  1 <= nb <= 2048 (the
 * block steps use the library's subspace solver).  H is applied one band at a
 * time, so the solver is latency-bound; Davidson is the throughput path.
 * On return psi_inout holds orthonormal Ritz vectors and eig (HOST, nb
 * doubles) their ascending values; info (may be NULL): iters = CG iterations
 * over all bands, notconv = bands stopped at maxiter, resid_max = the final
 * Ritz residual.  Blocks until done.  Errors: QEH_ERR_INVALID (sizes, nulls,
 * overlap context), QEH_ERR_NOMEM (short or misaligned work),
 * QEH_ERR_NUMERIC (non-finite input or residual), QEH_ERR_CHOLESKY. */
typedef struct {
  double rtol;    /* residual 2-norm threshold (Ry); 0 = 1e-8 */
  int maxiter;    /* iterations per band; 0 = 100 */
} qeh_cg_opts;
qeh_status qeh_cg_plan(const qeh_ctx *ctx, int nb, size_t *work_bytes);
qeh_status qeh_cg(qeh_ctx *ctx, int nb, double *psi_inout, int ldpsi, double *eig,
                  const qeh_cg_opts *opts, void *work, size_t work_bytes, qeh_dav_info *info);

/* Reverse-communication Davidson: the solver hands every H|psi> product to
 * the caller, who computes it with a Hamiltonian builder of its own and
 * passes the result back (the solver library's reverse communication
 * interface, section "Domain-specific mathematical libraries").  The same
 * solve as qeh_davidson, driven one step at a time:
 *   qeh_dav_rci_create binds the solve (arguments as qeh_davidson's; work is
 *     qeh_davidson_plan bytes; opts->refine must be NULL) and enqueues nothing;
 *   qeh_dav_rci_step enqueues work on the context's stream up to the next H
 *     product and returns QEH_RCI_APPLY_H with req filled: x (DEVICE, n bands
 *     of npw complex coefficients, interleaved re/im, leading dimension ld =
 *     npw, inside work: read only) and y (DEVICE, same layout, inside work:
 *     write only).  The caller writes H x into y, enqueued on the context's
 *     stream or finished before the next qeh_dav_rci_step (x is ready on that
 *     stream, not necessarily on the host), and calls qeh_dav_rci_step
 *     again.  It returns QEH_OK when the solve has converged (psi_inout, eig
 *     written), a negative status on failure (QEH_ERR_NOT_CONVERGED with the
 *     results written at maxiter); once ended, every further call returns
 *     that same status.  It blocks only where qeh_davidson waits for the
 *     stream (the per-iteration residual readback);
 *   qeh_dav_rci_destroy waits for the context's stream, fills info (may be
 *     NULL; t_hpsi = 0, the H time being the caller's) and frees the handle.
 * The context supplies the plane-wave set, the Gamma flag, diag(H) for the
 * preconditioner and, with q blocks set, the overlap S; its precision sets
 * the stop rule only (QEH_MIXED: qeh_davidson's single-precision rules
 * without refine).  A caller that serves each request with qeh_apply_h on the
 * same context gets qeh_davidson's results bit for bit.  One thread drives a
 * handle.  Errors: QEH_ERR_INVALID (nulls, refine set, and qeh_davidson's
 * argument checks), QEH_ERR_NOMEM (short work or no host memory for the
 * handle), QEH_ERR_DEVICE. */
typedef struct qeh_dav_rci qeh_dav_rci;
typedef struct {
  const double *x;
  double *y;
  int n;
  int ld;
} qeh_rci_request;
qeh_status qeh_dav_rci_create(qeh_ctx *ctx, int nb, double *psi_inout, int ldpsi,
                              double *eig, const qeh_dav_opts *opts, void *work,
                              size_t work_bytes, qeh_dav_rci **out);
qeh_status qeh_dav_rci_step(qeh_dav_rci *rci, qeh_rci_request *req);
qeh_status qeh_dav_rci_destroy(qeh_dav_rci *rci, qeh_dav_info *info);

/* The dense solver of the Rayleigh-Ritz step on its own (the generalized
 * Hermitian eigenproblem the paper solves with a dense GPU solver, section
 * "Evolution of the GPU-enabled version"): the nb lowest eigenpairs of
 * H y = eps S y, S positive definite, 1 <= nb <= n <= 2048.  H, S: DEVICE
 * complex n x n column-major with leading dimension ld >= n (Hermitian; only
 * (X + X^H) / 2 is used).  eig: DEVICE, nb doubles, ascending.  Y: DEVICE
 * complex n x nb column-major (ldy >= n), S-orthonormal eigenvectors
 * (Y^H S Y = I).  work: DEVICE, qeh_subspace_plan bytes, 256-byte aligned.
 * Runs on hip_stream (NULL = null stream) and returns after it finished.
 * The kernels are qeh_davidson's own subspace path: Cholesky, two triangular
 * solves for L^-1 H L^-H, Householder tridiagonalisation, bisection with
 * twisted-factorisation eigenvectors (inverse iteration with Gram-Schmidt
 * for numerically equal eigenvalues), back-transformation, a last triangular
 * solve; fixed summation orders, so repeated calls give the same bits.
 * Errors: QEH_ERR_INVALID (sizes, nulls), QEH_ERR_NOMEM (short or misaligned
 * work), QEH_ERR_CHOLESKY (S not positive definite), QEH_ERR_NUMERIC
 * (non-finite input). */
qeh_status qeh_subspace_plan(int n, int nb, size_t *work_bytes);
qeh_status qeh_subspace_eigh(int n, int nb, const double *H, const double *S, int ld,
                             double *eig, double *Y, int ldy, void *work, size_t work_bytes,
                             void *hip_stream);

/* Diagonal of H over the context's plane waves (npw doubles, the cell's G
 * order): |k+G|^2 + the mean of V(r) + sum over atoms of
 * sum_ij Re(beta_i(G) D_ij conj(beta_j(G))), the diagonal that the Davidson
 * preconditioner divides by (the preconditioner is among the kernels of the
 * GPU port, section "Evolution of the GPU-enabled version").  Built when the
 * context is created (the nonlocal sum on the device when the projectors come
 * from radial tables).  Copied to hdiag (DEVICE, npw doubles, caller-owned)
 * on the context stream; returns after enqueueing the copy.  Null arguments:
 * QEH_ERR_INVALID. */
qeh_status qeh_ctx_hdiag(const qeh_ctx *ctx, double *hdiag);

/* Per-stage device timing of H application and of the charge density (HIP
 * events on the context stream).  Stages: 0 scatter+z-FFT, 1 plane pass,
 * 2 z-FFT+gather+kinetic, 3 beta^H psi, 4 D scaling, 5 beta ps accumulate,
 * 6 density inverse y columns, 7 density inverse x rows + |psi|^2 sums (the
 * fused y + x pass when it runs; stage 6 then stays empty), 8 density
 * subgroup reduce (qeh_density's K1 counts as stage 0).  enable=1
 * starts recording (and clears totals); qeh_ctx_stage_times synchronises the
 * stream and returns total milliseconds and launch counts per stage. */
#define QEH_NSTAGES 9
qeh_status qeh_ctx_profile(qeh_ctx *ctx, int enable);
qeh_status qeh_ctx_stage_times(qeh_ctx *ctx, double *ms, long *launches, int nstages);

/* ---------------------------------------------------------------------------
 * Serving: continuous batching of Davidson solves.
 *
 * The paper expects exascale throughput to come from many independent
 * (high-throughput / ensemble) calculations and notes that oversubscribing a
 * GPU with several small runs pays off (sections "Outlook and conclusions"
 * and "Evolution of the GPU-enabled version").  A server owns a device arena
 * (the HBM budget) and max_slots HIP streams.  A request is a cell at nk
 * k-points with nb bands; each k-point is one job.  Requests are admitted
 * first-come first-served as soon as their whole footprint fits in the free
 * arena and nk slots are free (smaller later requests may pass a head request
 * that has waited < 0.25 s); every admitted job runs its Davidson on its own
 * stream, so work of different requests overlaps on the device.  A request
 * solved alone, repeated, gives the same bits; among concurrent requests the
 * low-order bits of some results can differ from run to run (mixed-form
 * eigenvalues by up to ~3e-5 Ry on the served trace), with a different
 * iteration count.
 * ------------------------------------------------------------------------- */
typedef struct qeh_server qeh_server;

/* arena: DEVICE memory (256-byte aligned) used for every admitted job; the
 * server never allocates device memory.  max_slots in [1, 64]; eight slots
 * already keep the device busy on served Davidson solves (their dense
 * eigensolver is launch-bound). */
qeh_status qeh_server_create(void *arena, size_t arena_bytes, int max_slots,
                             qeh_server **out);

/* Queue a request.  cells: nk HOST cell descriptors (same nb for all);
 * psi0: HOST complex start vectors, k-point after k-point, each nb x npw_k.
 * Everything is copied before return.  Returns QEH_ERR_REJECTED if the
 * request could never fit (footprint > arena or nk > max_slots).
 * Thread-safe. */
qeh_status qeh_submit(qeh_server *srv, const qeh_cell *cells, int nk, int nb,
                      const double *psi0, const qeh_dav_opts *opts, uint64_t *ticket);

/* Results of a finished request: eig (HOST, nk*nb, k-point-major), info
 * (HOST, nk entries, may be NULL), t_stamps[4] = arrive, admit, start,
 * finish (seconds since server creation; may be NULL).  Returns
 * QEH_ERR_BUSY while queued or running, QEH_ERR_INVALID for an unknown
 * ticket, otherwise the request's status; the request is forgotten after a
 * non-busy poll.  Thread-safe. */
qeh_status qeh_poll(qeh_server *srv, uint64_t ticket, double *eig, qeh_dav_info *info,
                    double *t_stamps);

/* Drop a request that has not been admitted yet (QEH_ERR_BUSY if it is
 * already running); a later poll returns QEH_ERR_REJECTED. */
qeh_status qeh_cancel(qeh_server *srv, uint64_t ticket);

/* out[0..n): queued requests, running jobs, finished requests, arena bytes in
 * use, arena bytes, peak running jobs, seconds with >= 1 job running,
 * seconds since creation. */
qeh_status qeh_server_stats(qeh_server *srv, double *out, int n);

/* Stops the server thread after the running jobs finish; queued requests
 * are dropped. */
qeh_status qeh_server_destroy(qeh_server *srv);

/* Shape facts of a context: [npw, nst, nkb, N1, N2, N3, x-extent, block,
 * precision, plane path (0 fused in one kernel, 1 split through HBM,
 * 2 lane-pair register kernel, 4 lane-quad register kernel), stick path
 * (0 LDS passes, 1 lane-pair register z transforms), projector tiles (0 the
 * 64 x 64 MFMA tiles, 1 the wide single-precision tiles: QEH_MIXED with
 * >= 2048 projectors and a block of >= 128 bands)].  out has room for n
 * values (up to 12).
 * The plane path is chosen by LDS fit and box shape: the lane-pair kernel
 * serves the mixed form when N1 = N2 is one of its compiled sizes (even,
 * 16..90), the lane-quad kernel the FP64 form when N1 = N2 is one of its
 * compiled sizes (multiples of 4, 16..72).  Environment variables read by qeh_ctx_plan / qeh_ctx_create:
 * QEH_FORCE_SPLIT_PLANE=1 forces the split path (a test hook);
 * QEH_STICK_KERNEL=generic keeps the LDS-pass z transforms where the lane-pair
 * ones would run (mixed form, N3 a compiled size; a test hook);
 * QEH_PLANE_KERNEL=generic keeps the fused kernel where a register one
 * would run (a test and comparison hook); QEH_PAIR_PLANES=n sets the bands per
 * register-kernel workgroup (default 2 lane-pair, 1 lane-quad); QEH_PLANE_ROWS=n caps the rows the fused
 * plane kernel expands at once (a tuning knob; fewer rows use less LDS). */
qeh_status qeh_ctx_info(const qeh_ctx *ctx, long *out, int n);

const char *qeh_status_str(qeh_status s);
const char *qeh_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* QEH_H */
