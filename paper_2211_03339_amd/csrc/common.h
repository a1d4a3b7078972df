// Internal declarations shared by the HIP sources of libjacobi.
// (Library-internal: nothing here is part of the C-ABI in include/jacobi.h.)
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

struct jac_mlp;

namespace jac {

// ---------------------------------------------------------------- errors
void set_error(const std::string& msg);
const char* last_error();

#define JAC_HIP(call)                                                          \
  do {                                                                         \
    hipError_t e_ = (call);                                                    \
    if (e_ != hipSuccess) {                                                    \
      ::jac::set_error(std::string(#call) + ": " + hipGetErrorString(e_));     \
      return 4;                                                                \
    }                                                                          \
  } while (0)

#define JAC_CHECK_LAUNCH() JAC_HIP(hipGetLastError())

// ---------------------------------------------------------------- profiling
// Optional kernel timing with HIP events recorded in the stream around runs of
// consecutive launches of one class (classes as in jac_stats.kern_*).  An
// event between every two launches would add its own cost to each launch, so
// a run of launches is timed as a whole and divided by its count.
struct Prof {
  bool on = false;
  std::vector<hipEvent_t> ev;
  int used = 0;
  struct Iv { int cls, e0, e1, count; };
  std::vector<Iv> ivs;
  double ms[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  long long launches[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  unsigned long long* work = nullptr;   // device counters [6]
  int mark(hipStream_t s);              // record an event, return its id (-1 if off)
  // count launches of class cls ran back to back between events e0 and e1
  void interval(int cls, int e0, int e1, int count = 1) {
    if (on && e0 >= 0 && e1 >= 0) ivs.push_back({cls, e0, e1, count});
  }
  int flush();                          // after the stream is synchronised
  ~Prof();
};

// ---------------------------------------------------------------- workspace
// Grow-only device scratch owned by the library (one pool per device).
void* workspace(size_t bytes);
void release_workspace();

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

struct Carve {
  char* base;
  size_t off = 0;
  explicit Carve(void* b) : base(static_cast<char*>(b)) {}
  template <typename T>
  T* take(size_t count) {
    off = align_up(off, 256);
    T* p = reinterpret_cast<T*>(base + off);
    off += count * sizeof(T);
    return p;
  }
};

// ---------------------------------------------------------------- types
template <typename T> struct Prec;
template <> struct Prec<double> {
  static constexpr double unit = 1.1102230246251565e-16;  // 2^-53
  static constexpr double bigmu = 1e150;
  static constexpr double tiny = 1e-150;
};
template <> struct Prec<float> {
  static constexpr float unit = 5.9604644775390625e-08f;  // 2^-24
  static constexpr float bigmu = 1e18f;
  static constexpr float tiny = 1e-18f;
};

// A 2x2 pair block: rows (top_k, bottom_k) x cols (top_l, bottom_l).
template <typename T> struct alignas(4 * sizeof(T)) Blk { T tt, tb, bt, bb; };
// Rotation of one pair in slot roles: new_top = x_t - s (x_b + tau x_t),
// new_bottom = x_b + s (x_t - tau x_b); diagonal pair: tt -= t tb, bb += t tb.
template <typename T> struct alignas(4 * sizeof(T)) Ang { T s, tau, t, applied; };

// Round-robin (circle method) in Brent-Luk slots.  There are ne (even)
// indices; slot s < h = ne/2 is ring position s, slot h + j is ring position
// ne-1-j, so step r pairs slot k with slot h+k.  Ring position 0 holds index
// 0; position p >= 1 holds index 1 + ((p - 1 + r) mod (ne - 1)).  Between
// steps the occupants of positions 1..ne-1 shift one position down (position
// 1 wraps to ne-1), which in slots is: top slots move down by one, bottom
// slots up by one, slot 1 -> h and slot ne-1 -> h-1.
struct RR {
  int ne, h;
  __host__ __device__ RR(int ne_) : ne(ne_), h(ne_ / 2) {}
  __host__ __device__ int ringpos(int s) const { return s < h ? s : ne - 1 - (s - h); }
  __host__ __device__ int index(int s, int r) const {
    int p = ringpos(s);
    return p == 0 ? 0 : 1 + (p - 1 + r) % (ne - 1);
  }
  __host__ __device__ int newslot(int s) const {
    if (s == 0) return 0;
    if (s == 1) return h;
    if (s < h) return s - 1;
    if (s == ne - 1) return h - 1;
    return s + 1;
  }
  __host__ __device__ int srcslot(int s) const {
    if (s == 0) return 0;
    if (s == h) return 1;
    if (s < h - 1) return s + 1;
    if (s == h - 1) return ne - 1;
    return s - 1;
  }
};

// Matrix-core operations.  v_mfma_f64_16x16x4f64 and v_mfma_f32_16x16x4f32
// take one A value (row lane % 16, k = lane / 16) and one B value (k = lane /
// 16, column lane % 16) per lane and accumulate four C values per lane in
// column lane % 16: accumulator r holds row 4 r + lane / 16 for FP64 and row
// 4 (lane / 16) + r for FP32 (measured on gfx950).
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <typename T> struct Mfma;
template <> struct Mfma<double> {
  typedef f64x4 acc_t;
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * r + (lane >> 4); }
  static __device__ __forceinline__ acc_t op(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};
template <> struct Mfma<float> {
  typedef f32x4 acc_t;
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
  static __device__ __forceinline__ acc_t op(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};

// Scalar helpers shared by the rotation kernels.
template <typename T> __device__ __forceinline__ T fmaT(T a, T b, T c);
template <> __device__ __forceinline__ double fmaT<double>(double a, double b, double c) { return __builtin_fma(a, b, c); }
template <> __device__ __forceinline__ float fmaT<float>(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
template <typename T> __device__ __forceinline__ T sqrtT(T a);
template <> __device__ __forceinline__ double sqrtT<double>(double a) { return __builtin_sqrt(a); }
template <> __device__ __forceinline__ float sqrtT<float>(float a) { return __builtin_sqrtf(a); }
template <typename T> __device__ __forceinline__ T absT(T a) { return a < T(0) ? -a : a; }

// (x, y) <- (x - s (y + tau x), y + s (x - tau y)): columns (or rows) i, j of
// J(i,j;c,s) applied from the right (left, transposed), tau = s / (1 + c).
template <typename T>
__device__ __forceinline__ void rot2(T& x, T& y, T s, T tau) {
  T nx = fmaT(-s, fmaT(tau, x, y), x);
  T ny = fmaT(s, fmaT(-tau, y, x), y);
  x = nx;
  y = ny;
}

// Angle of Lemma offa-jr for the pair whose "top" member holds index ip and
// "bottom" member index iq, from the entries tt (top,top), bb (bottom,bottom),
// tb.  The rotation is J(p, q) with p = min(ip, iq); the result is expressed in
// top/bottom roles (sign flipped when the top member is q).  Pairs with an
// index >= n (padding), and negligible t_pq (Remark dc: |t_pq| <= u
// sqrt|t_pp t_qq|, capped by skip_abs), give the identity.
// Negligibility of a pair (squared comparison, no square root):
//  symmetric problem (rel == 0): Remark dc, apq^2 <= min(u^2 |app aqq|, skip_abs^2);
//  one-sided SVD (rel > 0): columns already orthogonal to rel, i.e.
//  gamma^2 <= rel^2 alpha beta for the Gram entries (alpha, beta, gamma).
template <typename T>
__device__ __forceinline__ bool negligible2(T app, T aqq, T apq, T skip_abs, T rel) {
  if (apq == T(0)) return true;
  T lim2;
  if (rel > T(0)) {
    lim2 = rel * rel * absT(app * aqq);
  } else {
    lim2 = Prec<T>::unit * Prec<T>::unit * absT(app * aqq);
    T sk2 = skip_abs * skip_abs;
    if (sk2 < lim2) lim2 = sk2;
  }
  return apq * apq <= lim2;
}

template <typename T>
__device__ __forceinline__ Ang<T> make_angle(T tt, T bb, T tb, int ip, int iq, int n, T skip_abs, T rel = T(0)) {
  Ang<T> a{T(0), T(0), T(0), T(0)};
  if (ip >= n || iq >= n) return a;
  bool flip = ip > iq;
  T app = flip ? bb : tt, aqq = flip ? tt : bb, apq = tb;
  if (negligible2(app, aqq, apq, skip_abs, rel)) return a;
  // Lemma offa-jr: t = sign(mu) / (|mu| + sqrt(1 + mu^2)), mu = d / (2 apq),
  // d = aqq - app, written as t = sign(d) 2 apq / (|d| + sqrt(d^2 + 4 apq^2))
  // (t = 1 when d = 0).  Then c = 1/r, s = t/r, tau = s/(1+c) = t/(1+r) with
  // r = sqrt(1 + t^2).
  T d = aqq - app, t;
  T num = T(2) * apq;
  const T ad = absT(d), an = absT(num);
  if (d == T(0)) {
    t = T(1);
  } else if (ad > Prec<T>::bigmu || an > Prec<T>::bigmu || ad < Prec<T>::tiny || an < Prec<T>::tiny) {
    // magnitudes where d^2 + 4 apq^2 could overflow or underflow: the mu form
    T mu = d / num;
    if (absT(mu) > Prec<T>::bigmu) t = T(0.5) / mu;
    else t = mu >= T(0) ? T(1) / (mu + sqrtT(T(1) + mu * mu)) : T(1) / (mu - sqrtT(T(1) + mu * mu));
  } else {
    T rr = sqrtT(fmaT(d, d, num * num));
    t = (d > T(0) ? num : -num) / (absT(d) + rr);
  }
  T r = sqrtT(fmaT(t, t, T(1)));
  T c = T(1) / r;
  T s = t / r;
  T tau = t / (T(1) + r);
  (void)c;
  if (flip) { s = -s; tau = -tau; t = -t; }
  a.s = s; a.tau = tau; a.t = t; a.applied = T(1);
  return a;
}

// Packed upper triangle of pair blocks: block (k, l), k <= l.
__host__ __device__ inline long long bidx(int k, int l) { return (long long)l * (l + 1) / 2 + k; }

// ---------------------------------------------------------------- kernels
// Element-wise round-robin path (elem.hip).
template <typename T>
struct ElemState {
  int n, ne, h;
  long long nblk;
  Blk<T>* Tp[2];        // ping-pong packed T
  Ang<T>* A[2];         // ping-pong angles
  T* V;                 // n x n, leading dimension ldv, logical column order
  int ldv;
  T skip_abs;
  double* partial;      // off-norm partial sums (>= 1024)
  double* scalars;      // [0] off^2 result, [1] fro^2 result
  unsigned long long* rot;  // per-sweep applied-rotation counters
  int cur;              // which Tp / A holds the current step
  Prof* prof = nullptr;
  int cls = 4;
};

// Pack / angles at the slot layout of step r (r = 0 at sweep boundaries).
template <typename T>
int elem_pack(ElemState<T>& st, const double* Adense, int lda, int r, hipStream_t s);
template <typename T>
int elem_pack_from(ElemState<T>& st, const T* Adense, int lda, int r, hipStream_t s);
template <typename T>
int elem_init_angles(ElemState<T>& st, int r, hipStream_t s);
template <typename T>
int elem_steps(ElemState<T>& st, long long gstep0, int nsteps, hipStream_t s);
template <typename T>
int elem_offnorm2(ElemState<T>& st, hipStream_t s);  // result -> st.scalars[0]
template <typename T>
int elem_unpack_dense(const ElemState<T>& st, int r, T* D, int ldd, hipStream_t s);
template <typename T>
int elem_diag(const ElemState<T>& st, T* d, hipStream_t s);  // logical-order diagonal

// Per-matrix descriptor of the batched path.
template <typename T>
struct BDesc {
  T* Tm;                    // np x np, ldt = np
  T* V;                     // np x np, leading dimension ldv (rows >= n: the identity's, never touched)
  T* E;                     // (np / 64) pairs x 64 x 64
  int* ident;               // per pair
  unsigned long long* rot;  // applied rotations of this matrix
  const double* nrm2;       // ||A||_F^2 of this matrix (written before the sweeps)
  const int* conv;          // sweep at which the stop test first held, -1 before: the sweep
                            // kernels leave a matrix alone once it is >= 0
  int n, ldt, ldv;
  int s32;                  // FP32 sweeps the graph runs for this matrix's size class (0: none)
  double tol_n;             // tol / n: skip cap = tol_n * ||A||_F
};

// Blocked path (blocked.hip): in-place np x np T, blocks of b = blk_b2()/2.
template <typename T>
struct BlkState {
  int n, np;
  T* Tm;                // np x np, leading dimension ldt
  int ldt;
  T* V;                 // nvr x np, leading dimension ldv (pad columns zero)
  int ldv, nvr;
  T* W;                 // 2 x (np / blk_b2()) accumulated 2b x 2b rotations (E = W - I), by step parity
  int* ident;           // 2 x (np / blk_b2()) flags: W is exactly I
  int* tcount;          // per-tile reader counters of the merged launches (m (m - 1) / 2, >= 1; zero between launches)
  T skip_abs;
  double* partial;      // >= 1024
  double* scalars;      // [0] off^2
  unsigned long long* rot;  // applied rotations (cumulative)
  Prof* prof = nullptr; // optional timing; classes cls_inner / cls_update
  int cls_inner = 0, cls_update = 1;
};
int blk_np(int n);
int blk_b2();
template <typename T>
int blk_load(BlkState<T>& st, const void* A, bool a_is_double, int lda, hipStream_t s);
template <typename T>
int blk_offnorm2(BlkState<T>& st, hipStream_t s);
template <typename T>
int blk_sweep(BlkState<T>& st, int max_inner, hipStream_t s);
template <typename T>
int blk_diag(const BlkState<T>& st, T* d, hipStream_t s);
template <typename T>
int blk_sweep_batched(const BDesc<T>* desc, int count, int np, int max_nvr, int max_inner, hipStream_t s);

// Utilities (util.hip).
int fro2_f64(const double* A, int m, int n, int lda, double* partial, double* out, hipStream_t s);
// ||off(T)||_F^2 of a full n x n matrix (diagonal excluded).
int off2_f64(const double* T, int n, int ldt, double* partial, double* out, hipStream_t s);
// Learned start: Z (column-major, ldz) for one theta (device); order n of the network.
int mlp_predict_f64(const jac_mlp* net, const float* theta, double* Z, int ldz, hipStream_t s);
int mlp_order(const jac_mlp* net);
template <typename T>
int set_identity(T* V, int n, int ldv, hipStream_t s);
template <typename Tin, typename Tout>
int copy_convert(const Tin* A, int m, int n, int lda, Tout* B, int ldb, hipStream_t s);
template <typename T>
int sort_eigs(const T* d, const T* Vw, int n, int ldw, double* W, double* Vout, int ldv,
              int* rank, hipStream_t s);
int check_finite(const double* A, int m, int n, int lda, int* flag, hipStream_t s);
// X <- fl_p(X scale) / scale (p = JAC_PREC_FP16 / JAC_PREC_BF16; scale a power of two).
int round_lowp(double* X, int m, int n, int ldx, int prec, double scale, hipStream_t s);
int svd_finish(const double* C, int m, int ldc, const double* Vw, int n, int ldvw, double* sig, int* rank,
               double* S, double* U, int ldu, double* V, int ldv, hipStream_t s);

// One-sided Jacobi sweep (blocked.hip).
template <typename T>
int svd_sweep(T* C, int ldc, int mrows, T* V, int ldv, int n, int np, T* Ebuf, int* ident, T* Gpart, int gsplit,
              T rel, int max_inner, unsigned long long* rot, hipStream_t s);

// GEMM (gemm.hip): C = alpha * op(A) * op(B) + beta * C, column-major.  max_split = 1 keeps K
// whole (no split-K partial buffer, which is allocated on first need); 0 lets the GEMM choose.
// tri: zero structure the product may skip (square operands, m = n = k): kGemmBUpper, op(B)(kk, j) =
// 0 for kk > j; kGemmALower, op(A)(i, kk) = 0 for kk > i; kGemmCUpper, only C(i, j) with i <= j
// is wanted (tiles wholly below the diagonal are written as alpha * 0, i.e. beta C).
constexpr int kGemmBUpper = 1, kGemmALower = 2, kGemmCUpper = 4;
template <typename T>
int gemm(bool ta, bool tb, int m, int n, int k, T alpha, const T* A, int lda, const T* B, int ldb,
         T beta, T* C, int ldc, hipStream_t s, int max_split = 0, int tri = 0);
// count independent products C_z = alpha op(A_z) op(B_z) + beta C_z with A_z = A + z sA (and so on);
// state (device, may be NULL): product z runs only when state[z] <= state_max.
template <typename T>
int gemm_batched(bool ta, bool tb, int m, int n, int k, T alpha, const T* A, int lda, long long sA, const T* B,
                 int ldb, long long sB, T beta, T* C, int ldc, long long sC, int count, const int* state,
                 int state_max, hipStream_t s);

// Tridiagonal FP32 eigensolver (tridiag.hip): step 1 of Algorithm 4.1 through Householder
// tridiagonalization, bisection, twisted-factorization eigenvectors and the back-transformation.
size_t tridiag_bytes(int n);
bool tridiag_supported(int n);
template <typename TA>
int eig_tridiag_f32(const TA* A, int n, int lda, double* Z, int ldz, double* w_out, Carve& c, hipStream_t s,
                    bool no_split, Prof* prof = nullptr);
int tridiag_reduce_entry(const double* A, int n, int lda, double* d, double* e, float* tau, float* U, int ldu,
                         hipStream_t s);
int tridiag_eig_entry(const double* d, const double* e, int n, double* w, double* Z, int ldz, hipStream_t s);
int tridiag_backtransform_entry(const float* U, int ldu, const float* tau, int n, double* Y, int ldy, hipStream_t s);

// Step 2 for nearly orthonormal Z (orth.hip): Q = Z R^{-1} by passes of the second-order series;
// *used = 0 when ||Z^T Z - I||_F is too large for it (Z then holds Z S with S upper triangular, whose
// orthonormal QR factor is Z's: the caller finishes with block MGS).
constexpr double kSeriesMax = 0.1;      // ||Z^T Z - I||_F above which no pass is tried
constexpr double kSeriesOnePass = 2e-5; // a pass from ||E||_F below this is final: its error ||E||^3 < 1e-14
constexpr int kSeriesPasses = 3;
int orth_series_f64(double* Z, int n, int ldz, double* B1, double* B2, double* B3, double* B4, double* part,
                    double* scal, int* used, hipStream_t s, bool no_split);
// The same for count matrices of order np stored back to back (leading dimension np); per matrix
// state[z] ends as 2 (orthonormal) or 3 (the series did not apply); e2_first[z] = ||Z^T Z - I||_F^2
// of the start.  S1..S4: count np^2 doubles each.  A fixed list of launches (no host round trip).
int orth_series_batched(double* Z, int np, int count, double* S1, double* S2, double* S3, double* S4, int* state,
                        double* e2_first, hipStream_t s);

// Block modified Gram-Schmidt in place (mgs.hip).  Returns 0 or 3 on breakdown.  The panel kernel
// holds a panel's rows in registers: at most kMgsMaxRows rows (64 per thread, one-column panels
// above 16384 rows).  kMgsFastRows bounds the automatic QR-first SVD (measured faster only there).
constexpr int kMgsMaxRows = 32768;
constexpr int kMgsFastRows = 8192;
int mgs_f64(double* Q, int m, int n, int ldq, double* scratch, int* flag, hipStream_t s);
size_t mgs_scratch_elems(int m, int n);

}  // namespace jac
