/*
 * jacobi.h -- C-ABI of libjacobi, an MI355X (gfx950) implementation of the
 * mixed-precision preconditioned Jacobi method of Zhang & Bai, "A mixed
 * precision preconditioned Jacobi method for the symmetric eigenvalue
 * problem" (arXiv 2211.03339).
 *
 * Conventions (all entry points):
 *  - Matrices are column-major FP64 (LAPACK layout): element (i,j) of X is
 *    X[i + j*ldx].  Matrix/vector pointers are DEVICE pointers (hipMalloc'd or
 *    a torch tensor's data pointer) unless an argument says "host".
 *  - `stream` is a hipStream_t passed as void*; NULL means the null stream.
 *    Every compute call is synchronous: it returns after the results are
 *    written.
 *  - Ownership: the caller owns every buffer it passes; the library never
 *    frees or retains them.  The library allocates its own device workspace
 *    (grow-only, kept until jac_release_workspace()).
 *  - Return codes (LAPACK style): 0 success; -i the i-th argument is invalid
 *    (counting from 1); +1 the iteration did not converge within max_sweeps
 *    (outputs hold the last iterate); +2 the input contains NaN or Inf;
 *    +3 modified Gram-Schmidt broke down (rank-deficient start);
 *    +4 HIP/device error.  jac_last_error() describes the last failure.
 *  - A (symmetric problems) must be exactly symmetric; both triangles are
 *    read.  A is never written.
 */
#ifndef JACOBI_H
#define JACOBI_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Start of the FP64 Jacobi iteration (Algorithm 4.1 of the paper vs its
 * Algorithm 3.2). */
typedef enum {
  JAC_PRECOND_NONE = 0, /* plain cyclic Jacobi from T = A, P = I (Algorithm 3.2) */
  JAC_PRECOND_FP32 = 1, /* FP32 eigensolve -> FP64 MGS -> T = Q^T A Q (Algorithm 4.1) */
  JAC_PRECOND_MLP = 2   /* learned warm start, FP32 solve as fallback */
} jac_precond_t;

/* How each sweep is carried out. */
typedef enum {
  JAC_VARIANT_AUTO = 0,
  JAC_VARIANT_ELEMENT = 1, /* n/2 disjoint 2x2 rotations per parallel step */
  JAC_VARIANT_BLOCKED = 2  /* 2b x 2b block rotations applied as GEMMs */
} jac_variant_t;

/* Solver of the low-precision step 1 (Algorithm 4.1 step 1; the paper uses a
 * LAPACK-style tridiagonal FP32 eigensolver there, Section 6 setup, and needs
 * only its backward stability, Lemma symeig). */
typedef enum {
  JAC_STAGE1_AUTO = 0,     /* tridiagonal for 16 <= n <= 4096, else Jacobi */
  JAC_STAGE1_JACOBI = 1,   /* FP32 cyclic Jacobi (the same sweep kernels in float), stopped at
                              fp32_tol ||A||_F: a truncated start (default fp32_tol 1e-4) */
  JAC_STAGE1_TRIDIAG = 2   /* FP32 Householder tridiagonalization, FP64 bisection and
                              twisted-factorization eigenvectors of T, FP32 back-transformation;
                              n <= 8192 (larger orders use Jacobi) */
} jac_stage1_t;

/* QR preconditioning of the one-sided SVD for m >> n (the remark after
 * Algorithm 5.2): A = Q_A B with Q_A (m x n) orthonormal -- two passes of block
 * MGS, so that Q_A is orthonormal to working precision -- and B = Q_A^T A
 * (n x n); the SVD B = U_B S V^T by the same method; U = Q_A U_B.  The sweeps
 * then work on n x n columns instead of m x n.  Needs m <= 32768 (block MGS). */
typedef enum {
  JAC_SVD_QR_AUTO = 0,  /* QR first when m >= 8 n, n >= 512 and m <= 8192 */
  JAC_SVD_QR_OFF = 1,
  JAC_SVD_QR_ON = 2
} jac_svd_qr_t;

/* Precision upsilon of step 1 (Algorithm 4.1; the paper's precision study,
 * Section 6.1).  FP16 and BF16: A is rounded to upsilon (FP16 after scaling by
 * a power of two near 1/||A||_F) before the step-1 eigensolver, and the
 * eigenvectors it returns are rounded to upsilon before step 2, so that the
 * start carries upsilon's accuracy; the eigensolver itself computes in FP32. */
typedef enum {
  JAC_PREC_FP32 = 0,
  JAC_PREC_FP16 = 1,
  JAC_PREC_BF16 = 2
} jac_prec_t;

struct jac_mlp;

typedef struct jac_opts {
  int precond;         /* jac_precond_t; default (zeroed struct) = NONE */
  int variant;         /* jac_variant_t */
  int block_b;         /* reserved, must be 0 (the blocked variant uses 2b = 64) */
  int max_sweeps;      /* FP64 sweeps; <= 0 means 64 */
  double fp32_tol;     /* FP32 stage stops at off(T32) <= fp32_tol ||A||_F; <= 0: default
                          (1e-4 for syev_jacobi_ex, 1e-6 for the Gram matrix of gesvd_jacobi_ex) */
  int fp32_max_sweeps; /* <= 0 means 30 */
  const struct jac_mlp* mlp;  /* JAC_PRECOND_MLP: the network */
  const float* theta;  /* JAC_PRECOND_MLP: device pointer to its input */
  double fallback_tol; /* MLP start rejected if off(Q^T A Q)_F / ||A||_F > this; <= 0: 1e-2 */
  int inner_sweeps;    /* blocked variant: cap on the sweeps of each 2b x 2b subproblem; <= 0: default */
  int profile;         /* nonzero: time every sweep launch with HIP events into jac_stats.kern_* */
  int stage1;          /* jac_stage1_t: solver of the FP32 step 1 (FP32 start and fallback) */
  int svd_qr;          /* jac_svd_qr_t: gesvd_jacobi_ex only */
  int stage1_prec;     /* jac_prec_t: precision of step 1 (syev with the FP32 start only) */
} jac_opts;

#define JAC_HIST 65
typedef struct jac_stats {
  int sweeps;              /* FP64 sweeps executed (SP) */
  int fp32_sweeps;         /* sweeps of the FP32 stage */
  long long rotations;     /* FP64 rotations applied (JU = rotations / (n(n-1)/2)) */
  long long fp32_rotations;
  int used_fallback;       /* MLP start rejected, FP32 start used */
  double nrmA;             /* ||A||_F */
  double off0;             /* ||off(T_0)||_F before the first FP64 sweep */
  double off_final;        /* ||off(T)||_F at return */
  double off_hist[JAC_HIST]; /* ||off(T)||_F before sweep 1, after sweep 1, ... */
  float stage_ms[8];       /* 0 low-precision start, 1 MGS, 2 Q^T A Q, 3 sweeps,
                              4 output, 5 total, 6 norm/checks */
  double step_ms;          /* HIP-event time of the FP64 sweep launches (rotation steps) */
  long long step_launches; /* number of FP64 step launches timed in step_ms */
  double fp32_step_ms;     /* same for the FP32 stage */
  long long fp32_step_launches;
  /* With opts.profile: per kernel class, summed HIP-event time, launch count and
   * work done.  Classes: 0 FP64 inner solve, 1 FP64 block update, 2 FP32 inner
   * solve, 3 FP32 block update, 4 FP64 element step, 5 FP32 element step,
   * 6 tridiagonal step 1: the reduction (one cooperative launch), 7 tridiagonal
   * step 1: bisection, eigenvectors of T and back-transformation.
   * Events bracket each run of consecutive launches of one class (the inner
   * launches of a block sweep, the steps of an element sweep), not each launch.
   * The inner-solve launches of block steps after the first also carry the
   * whole update (T tiles and V chunks) of the previous step; the block update
   * class is the full update of a sweep's last step.
   * kern_work of the inner and update classes: 64x64 T tiles (high 32 bits)
   * and 64-row V chunks (low 32 bits) updated in those launches; element
   * classes: steps. */
  double kern_ms[8];
  long long kern_launches[8];
  long long kern_work[8];
  double start_resid;      /* precond MLP: ||off(Q^T A Q)||_F / ||A||_F of the predicted start */
  int fp32_method;         /* step 1 that ran: 0 none, 1 FP32 Jacobi, 2 tridiagonal */
  int svd_qr_used;         /* gesvd: 1 when the QR-first form ran */
  float qr_ms;             /* gesvd QR first: time of A = Q_A B and U = Q_A U_B */
} jac_stats;

/* Symmetric eigendecomposition A = V diag(W) V^T by Algorithm 4.1
 * (preconditioned, FP32 start) with the library's choice of sweep variant.
 * A: n x n (lda >= max(1,n)), read only.  W: n eigenvalues, ascending.
 * V: n x n (leading dimension n), column i pairs with W[i].
 * tol: stop when ||off(T)||_F <= tol ||A||_F (tested before each sweep);
 * tol <= 0 selects the paper's 20 * 2^-53.  sweeps_out (host, may be NULL):
 * FP64 sweeps executed.  Preconditioned solves (and custom starts) need
 * n <= 32768, the row limit of step 2's block MGS (-2 otherwise); plain Jacobi
 * has no such limit. */
int syev_jacobi(const double* A, int n, int lda, double* W, double* V, double tol, int* sweeps_out);

/* As syev_jacobi with explicit options, leading dimension of V, statistics
 * (host pointer, may be NULL) and stream.  opts NULL = plain method. */
int syev_jacobi_ex(const double* A, int n, int lda, double* W, double* V, int ldv, double tol,
                   const jac_opts* opts, jac_stats* stats, void* stream);

/* For callers that cannot allocate device memory (code under stream capture,
 * serving loops, harnesses that forbid allocation): syev_jacobi_ex with the
 * library's pooled workspace replaced by a fixed device array of
 * JAC_NOALLOC_BYTES, one per device, held from the library's load until the
 * process ends.  The call allocates nothing (no device memory, no events):
 *  - opts NULL or precond NONE / FP32 (other starts return -8);
 *  - returns -2 ("n too large") when jac_workspace_bytes(n, opts) exceeds
 *    JAC_NOALLOC_BYTES (n <= 524 preconditioned, n <= 995 plain);
 *  - stats (may be NULL): sweeps, rotations, norms and the off history are
 *    filled; stage_ms, step_ms and kern_* stay zero (timing needs events);
 *  - the GEMMs of Q^T A Q run without split-K (same sums, other order than
 *    syev_jacobi_ex for small n).
 * Every call on a device uses that device's one array and leaves its contents
 * there; each call initialises what it reads.  Calls that overlap on one device
 * (other host threads, other streams) race and must be serialised by the
 * caller.  Synchronous like syev_jacobi_ex. */
#define JAC_NOALLOC_BYTES ((size_t)32 << 20)
int syev_jacobi_noalloc(const double* A, int n, int lda, double* W, double* V, int ldv, double tol,
                        const jac_opts* opts, jac_stats* stats, void* stream);

/* Resume / custom start (Algorithm 4.1 steps 2-4 from a given Q0): Q = MGS(Q0),
 * T = Q^T A Q, sweeps.  Q0: n x n, ldq >= n, read only. */
int syev_jacobi_warm(const double* A, int n, int lda, const double* Q0, int ldq, double* W, double* V,
                     int ldv, double tol, const jac_opts* opts, jac_stats* stats, void* stream);

/* Thin SVD A = U diag(S) V^T of an m x n matrix (m >= n, full column rank) by
 * the preconditioned one-sided Jacobi method (Algorithm 5.2): FP32 right
 * singular vectors (eigenvectors of the FP32 Gram A^T A), FP64 MGS, C = A Q,
 * V = Q, then one-sided sweeps (Lemma ortho-2c) on column pairs of C and V
 * until a sweep applies fewer than 2e-4 n(n-1)/2 rotations.  A pair is rotated
 * only when |c_i.c_j| > m tol ||c_i|| ||c_j||; tol <= 0 selects 2^-53.
 * A: m x n (lda >= m), read only.  S: n singular values, descending.
 * U: m x n (ldu >= m), u_j = c_j / s_j.  V: n x n (ldv >= n).
 * sweeps_out (host, may be NULL).  Takes the QR-first form (jac_svd_qr_t) when
 * m >= 8 n, n >= 512 and m <= 8192.  The preconditioned SVD needs n <= 32768 (-3). */
int gesvd_jacobi(const double* A, int m, int n, int lda, double* S, double* U, int ldu, double* V, int ldv,
                 double tol, int* sweeps_out);

/* As gesvd_jacobi with options (precond NONE = Algorithm 5.1 from C = A,
 * V = I), statistics (off_hist[s] = rotations applied in sweep s) and stream. */
int gesvd_jacobi_ex(const double* A, int m, int n, int lda, double* S, double* U, int ldu, double* V, int ldv,
                    double tol, const jac_opts* opts, jac_stats* stats, void* stream);

/* Batched symmetric eigendecompositions (blocked variant) of `batch` <= 65535
 * independent matrices of order n[i] in [1, 512].  Host arrays: n, A (device
 * pointers to column-major n[i] x n[i] inputs, read only), lda, W (device
 * pointers, n[i] eigenvalues ascending), V (device pointers, n[i] x n[i]
 * eigenvectors, leading dimension ldv[i]).  Device arrays (may be NULL):
 * sweeps[i] = FP64 sweeps until ||off(T)||_F <= tol ||A_i||_F first held
 * (max_sweeps when it never did), info[i] = 0 converged / 1 not converged
 * within max_sweeps.  tol <= 0 selects 20 * 2^-53.
 * Each matrix stops at its own convergence: its results do not depend on the
 * rest of the batch.  The solve is one graph launch on `stream` (built on the
 * first call with these sizes, pointers and options, replayed afterwards),
 * then a host check of the convergence flags: size classes with unconverged
 * matrices get further sweeps up to max_sweeps.  Synchronous. */
int syev_jacobi_batched(int batch, const int* n, const double* const* A, const int* lda, double* const* W,
                        double* const* V, const int* ldv, double tol, int* sweeps, int* info, void* stream);

/* Options of the batched path (NULL: all defaults). */
typedef struct jac_batched_opts {
  int precond;        /* JAC_PRECOND_NONE (plain, Algorithm 3.2) or JAC_PRECOND_FP32:
                         Algorithm 4.1 per matrix -- FP32 blocked Jacobi on fl32(A)
                         truncated at fp32_tol ||A||_F, the QR factor of its
                         eigenvectors (series passes; a matrix whose start they
                         cannot orthogonalise takes the plain start), T0 = Q^T A Q */
  double fp32_tol;    /* stop of the FP32 stage; <= 0: 1e-4 */
  int max_sweeps;     /* FP64 sweep cap including the top-up; 0: 60 (at most 1000) */
  int reserved;       /* must be 0 */
} jac_batched_opts;

/* Host statistics of one batched call. */
typedef struct jac_batched_stats {
  int topup_sweeps;   /* sweeps run after the graph (summed over size classes) */
  int series_failed;  /* JAC_PRECOND_FP32: matrices that fell back to the plain start */
  int graph_built;    /* 1 when this call captured a new graph */
  int classes;        /* size classes (orders rounded up to 64) */
} jac_batched_stats;

/* syev_jacobi_batched with options and statistics.  sweeps32 (device, may be
 * NULL): FP32 sweeps per matrix (0 without preconditioning).  Error -12: bad
 * option. */
int syev_jacobi_batched_ex(int batch, const int* n, const double* const* A, const int* lda, double* const* W,
                           double* const* V, const int* ldv, double tol, int* sweeps, int* info, int* sweeps32,
                           const jac_batched_opts* opts, jac_batched_stats* stats, void* stream);

/* Autotuner of the batched path: for every size class present in the batch,
 * runs up to 16 of the given matrices with each inner-sweep cap 1..4 (with the
 * options' preconditioning), takes the sweeps the samples needed in each
 * stage, times that configuration and keeps the fastest.  The block size 2b is
 * fixed at 64 (the width of the matrix-core tiles).  The table is used by
 * later batched calls in this process and written to the file named by the
 * environment variable JACOBI_TUNE_CACHE (read back at the first use in a
 * later process).  Synchronous. */
int jac_autotune_batched(int batch, const int* n, const double* const* A, const int* lda, double tol,
                         void* stream);
int jac_autotune_batched_ex(int batch, const int* n, const double* const* A, const int* lda, double tol,
                            const jac_batched_opts* opts, void* stream);

/* Host: the (inner-sweep cap, FP64 sweeps[, FP32 sweeps]) the batched path
 * uses for order n (1..512) without / with preconditioning. */
int jac_tune_entry(int n, int* inner_sweeps, int* sweeps);
int jac_tune_entry_ex(int n, int precond, int* inner_sweeps, int* sweeps, int* sweeps32);

/* Host: forget the tuned table of this process (the built-in defaults apply
 * until the autotuner runs again; the cache file is not read again). */
int jac_tune_clear(void);

/* ---- Learned warm start (a project addition; not in the paper) ------------
 * A three-layer perceptron theta (n_in values) -> hidden -> ReLU -> hidden ->
 * ReLU -> n^2 values, read as the column-major entries of an approximate
 * eigenvector matrix Z of A(theta).  With opts.precond = JAC_PRECOND_MLP,
 * syev_jacobi_ex uses Z in place of the FP32 eigensolve of Algorithm 4.1
 * step 1: Q = MGS(Z), T = Q^T A Q; if ||off(T)||_F / ||A||_F exceeds
 * opts.fallback_tol (default 1e-2) or MGS meets a zero column, the FP32 start
 * is computed and used instead (jac_stats.used_fallback = 1).
 * Every matrix product takes bfloat16 operands (round to nearest even from
 * FP32) and accumulates in FP32; biases, activations, gradients, FP32 master
 * weights and AdamW moments are FP32.  Parameters are packed row-major as
 * [W1 (hidden x n_in), b1, W2 (hidden x hidden), b2, W3 (n^2 x hidden), b3].
 * Activations are row-major (batch x features).  A handle owns its device
 * memory (about 16 bytes per parameter plus activations for max_batch rows);
 * calls that use one handle must not overlap (they share its buffers). */
enum { JAC_MLP_PARAMS = 0, JAC_MLP_GRADS = 1, JAC_MLP_MOMENT1 = 2, JAC_MLP_MOMENT2 = 3 };

/* New network on the current device: weights uniform in [-a, a] from
 * SplitMix64(seed, index) (a = sqrt(6/n_in), sqrt(6/hidden), sqrt(3/hidden)
 * per layer), biases and moments zero.  1 <= n_in <= 32, hidden a positive
 * multiple of 32, n^2 a multiple of 32, max_batch >= 1.  Errors: -1..-4 for
 * those arguments, -6 out NULL, 4 allocation failure. */
int jac_mlp_create(int n_in, int hidden, int n, int max_batch, unsigned long long seed, struct jac_mlp** out);
void jac_mlp_free(struct jac_mlp* net);
long long jac_mlp_num_params(const struct jac_mlp* net);
/* Shape and optimiser step count (host pointers, each may be NULL). */
int jac_mlp_shape(const struct jac_mlp* net, int* n_in, int* hidden, int* n, int* max_batch, long long* steps);
/* Copy one packed buffer (JAC_MLP_*) to / from host memory (num_params floats).
 * Synchronises the device.  Setting the parameters refreshes the bfloat16
 * weight copies; moments and step count are left as they are. */
int jac_mlp_get(const struct jac_mlp* net, int which, float* host);
int jac_mlp_set(struct jac_mlp* net, int which, const float* host);
/* AdamW hyper-parameters (defaults 0.9, 0.999, 1e-8) and step count t. */
int jac_mlp_set_adam(struct jac_mlp* net, float beta1, float beta2, float eps, long long steps);
/* Y (device, batch x n^2 FP32, row stride ldy >= n^2) = network(theta)
 * for theta (device, batch x n_in FP32, row-major), 0 <= batch <= max_batch. */
int jac_mlp_forward(struct jac_mlp* net, const float* theta, int batch, float* Y, int ldy, void* stream);
/* Z (device, column-major n x n FP64, ldz >= n) for one theta (device). */
int jac_mlp_predict(const struct jac_mlp* net, const float* theta, double* Z, int ldz, void* stream);
/* Mean squared error over batch x n^2 outputs against target (device,
 * bfloat16 bits, row stride ldt >= n^2) and its gradient, left in the handle
 * (JAC_MLP_GRADS).  loss: device float, may be NULL.  1 <= batch <= max_batch. */
int jac_mlp_grads(struct jac_mlp* net, const float* theta, const unsigned short* target, long long ldt, int batch,
                  float* loss, void* stream);
/* One AdamW step (decoupled weight decay) with the gradient in the handle:
 * t += 1, m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
 * p -= lr (m/(1-b1^t) / (sqrt(v/(1-b2^t)) + eps) + weight_decay p). */
int jac_mlp_adamw(struct jac_mlp* net, float lr, float weight_decay, void* stream);
/* jac_mlp_grads followed by jac_mlp_adamw. */
int jac_mlp_train_step(struct jac_mlp* net, const float* theta, const unsigned short* target, long long ldt,
                       int batch, float lr, float weight_decay, float* loss, void* stream);
/* Training targets from eigenvector matrices: for matrix c (device V +
 * c stride_v, column-major n x n, ldv >= n) every column is multiplied by the
 * sign of its entry of largest magnitude (the first one on ties) and its
 * column-major entries are written, rounded to bfloat16 from FP32, to
 * T + c ldt (device).  count <= 65535. */
int jac_mlp_pack_targets(const double* V, int n, int ldv, long long stride_v, int count, unsigned short* T,
                         long long ldt, void* stream);
/* The same with a choice of signs: sign_mode 0 as jac_mlp_pack_targets,
 * 1 the columns as given (for targets whose signs the caller has already
 * aligned).  Error -8: sign_mode not 0 or 1. */
int jac_mlp_pack_targets_ex(const double* V, int n, int ldv, long long stride_v, int count, unsigned short* T,
                            long long ldt, int sign_mode, void* stream);
/* Weights, AdamW moments, step count and hyper-parameters to / from a file
 * ("JACMLP01", int32 n_in, hidden, n, int64 t, float beta1, beta2, eps, then
 * the weights, first and second moments as num_params floats each).  Loading
 * checks the shape (6 on mismatch); 5 on an I/O error. */
int jac_mlp_save(const struct jac_mlp* net, const char* path);
int jac_mlp_load(struct jac_mlp* net, const char* path);

/* ---- Stages of the path, callable on their own --------------------------- */

/* Apply parallel round-robin steps r0 .. r0+nsteps-1 (Section 6.2 ordering,
 * step r pairs the indices of ring positions i and ne-1-i, ne = n rounded up
 * to even; see jac_round_robin_pairs) to the symmetric T (n x n, in place)
 * and the columns of V (n x n, in place; may be NULL).  Angles follow Lemma
 * offa-jr from T before each step; an entry with |t_pq| <= min(2^-53
 * sqrt|t_pp t_qq|, skip_abs) is set to zero without a rotation (Remark dc).
 * rotations (host, may be NULL) receives the number applied. */
int jac_parallel_steps(double* T, int n, int ldt, double* V, int ldv, int r0, int nsteps,
                       double skip_abs, long long* rotations, void* stream);

/* Host: index pairs (p[i] < q[i], i < ne/2) of step r of the round-robin
 * ordering for ne (even) indices. */
int jac_round_robin_pairs(int ne, int r, int* p, int* q);

/* FP64 modified Gram-Schmidt, in place: Q (m x n, m >= n, ldq >= m, m <= 32768)
 * becomes orthonormal with the column order and signs of the input
 * (Algorithm 4.1 step 2).  Returns +3 on a zero column. */
int jac_mgs(double* Q, int m, int n, int ldq, void* stream);

/* Step 2 as the pipeline runs it: Q (n x n, ldq >= n, in place) becomes the
 * orthonormal factor of its QR factorization with a positive R diagonal (the
 * factor MGS returns; Algorithm 4.1 step 2, Lemma MGS).  When ||Q^T Q - I||_F
 * <= 1e-3 it is evaluated as Q R^{-1} from a second-order series for R (four
 * FP64 GEMMs; error O(||Q^T Q - I||^3)), otherwise by block MGS.  method (host,
 * may be NULL): 1 series, 2 block MGS.  n <= 32768.  Returns +3 on a zero column. */
int jac_qr_orth(double* Q, int n, int ldq, int* method, void* stream);

/* T = Q^T A Q (Algorithm 4.1 step 3), FP64: upper triangle computed, mirrored.
 * A, Q, T: n x n. */
int jac_similarity(const double* A, int n, int lda, const double* Q, int ldq, double* T, int ldt,
                   void* stream);

/* Low-precision step 1 by the FP32 Jacobi stage (JAC_STAGE1_JACOBI): FP32
 * eigenvectors of A (demoted to FP32), stored in FP64.  Z: n x n (ldz >= n); W (may be NULL): FP32 eigenvalues promoted,
 * ascending, with Z's columns in the same order.  tol <= 0: default.
 * sweeps (host, may be NULL). */
int jac_eig_fp32(const double* A, int n, int lda, double* Z, int ldz, double* W, double tol,
                 int max_sweeps, int* sweeps, void* stream);

/* Parts of the tridiagonal step 1 (JAC_STAGE1_TRIDIAG), each as the pipeline
 * runs it:
 * jac_sytrd_f32: Householder tridiagonalization of fl32(A) in FP32 (A n x n
 *   FP64, lda): Q^T A Q = T with d (n), e (n - 1) holding T's FP32 entries in
 *   FP64, and the reflectors H_k = I - tau(k) u_k u_k^T, k < n - 2, as tau
 *   (FP32, n - 2) and U (FP32, n x (n - 2), ldu >= n; column k = u_k with
 *   u_k(k+1) = 1 and zeros above), Q = H_0 ... H_{n-3}.  One cooperative
 *   launch; returns 4 if the device cannot run it.  n <= 8192.
 * jac_tridiag_eig: eigenvalues w (FP64, ascending) of the symmetric
 *   tridiagonal (d, e) by bisection, and if Z is not NULL the eigenvectors
 *   (FP64, n x n, ldz) by twisted factorization.  All pointers device.
 * jac_tridiag_backtransform: Y <- H_0 ... H_{n-3} Y (Y FP64 n x n, ldy,
 *   computed in FP32) for reflectors as returned by jac_sytrd_f32.
 * jac_eig_fp32_tridiag: the whole step: Z (FP64, ldz) eigenvectors of fl32(A)
 *   in ascending order of W (FP64, may be NULL). */
int jac_sytrd_f32(const double* A, int n, int lda, double* d, double* e, float* tau, float* U, int ldu, void* stream);
int jac_tridiag_eig(const double* d, const double* e, int n, double* w, double* Z, int ldz, void* stream);
int jac_tridiag_backtransform(const float* U, int ldu, const float* tau, int n, double* Y, int ldy, void* stream);
int jac_eig_fp32_tridiag(const double* A, int n, int lda, double* Z, int ldz, double* W, void* stream);

/* C = alpha op(A) op(B) + beta C on the matrix cores (FP64 / FP32). */
int jac_gemm_f64(int transa, int transb, int m, int n, int k, double alpha, const double* A, int lda,
                 const double* B, int ldb, double beta, double* C, int ldc, void* stream);
int jac_gemm_f32(int transa, int transb, int m, int n, int k, float alpha, const float* A, int lda,
                 const float* B, int ldb, float beta, float* C, int ldc, void* stream);

/* ---- Housekeeping ---------------------------------------------------------- */

/* Device workspace bytes a call of order n with these options would use. */
size_t jac_workspace_bytes(int n, const jac_opts* opts);
/* Free the library's device workspace (after all calls have returned). */
void jac_release_workspace(void);
/* Text of the last error in this thread ("" if none). */
const char* jac_last_error(void);
/* Library version string. */
const char* jac_version(void);

#ifdef __cplusplus
}
#endif

#endif /* JACOBI_H */
