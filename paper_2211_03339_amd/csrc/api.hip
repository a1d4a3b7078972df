// C-ABI entry points of libjacobi (declared in include/jacobi.h).
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/jacobi.h"
#include "common.h"

namespace jac {

// ------------------------------------------------------------------ errors
static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }
const char* last_error() { return g_err.c_str(); }

// ------------------------------------------------------------------ workspace
struct Pool { void* ptr = nullptr; size_t bytes = 0; };
static std::map<int, Pool> g_pools;
static std::mutex g_pool_mu;

void* workspace(size_t bytes) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lk(g_pool_mu);
  Pool& p = g_pools[dev];
  if (bytes > p.bytes) {
    if (p.ptr) {
      (void)hipDeviceSynchronize();
      (void)hipFree(p.ptr);
      p.ptr = nullptr;
      p.bytes = 0;
    }
    size_t want = align_up(bytes + bytes / 8, 1 << 20);
    if (hipMalloc(&p.ptr, want) != hipSuccess) {
      p.ptr = nullptr;
      return nullptr;
    }
    p.bytes = want;
  }
  return p.ptr;
}

void release_workspace() {
  std::lock_guard<std::mutex> lk(g_pool_mu);
  (void)hipDeviceSynchronize();
  for (auto& kv : g_pools) {
    if (kv.second.ptr) (void)hipFree(kv.second.ptr);
    kv.second = Pool{};
  }
}

static inline int cdiv(long long a, long long b) { return (int)((a + b - 1) / b); }

// ------------------------------------------------------------------ profiling
int Prof::mark(hipStream_t s) {
  if (!on) return -1;
  if (used == (int)ev.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) { on = false; return -1; }
    ev.push_back(e);
  }
  if (hipEventRecord(ev[used], s) != hipSuccess) { on = false; return -1; }
  return used++;
}

int Prof::flush() {
  if (!on) return 0;
  for (const Iv& iv : ivs) {
    float t = 0;
    if (hipEventElapsedTime(&t, ev[iv.e0], ev[iv.e1]) == hipSuccess) {
      ms[iv.cls] += t;
      launches[iv.cls] += iv.count;
    }
  }
  ivs.clear();
  used = 0;
  return 0;
}

Prof::~Prof() {
  for (hipEvent_t e : ev) (void)hipEventDestroy(e);
}

// ------------------------------------------------------------------ sizing
constexpr int kMaxSweepsDefault = 64;
constexpr int kRotSlots = 272;  // per-sweep rotation counters (>= max sweeps + 2)

template <typename T>
static size_t elem_bytes(int n) {
  int ne = n + (n & 1), h = ne / 2;
  long long nblk = (long long)h * (h + 1) / 2;
  size_t b = 0;
  b += 2 * align_up(nblk * sizeof(Blk<T>), 256);
  b += 2 * align_up((size_t)h * sizeof(Ang<T>), 256);
  return b;
}

// Off-diagonal tiles of the block sweeps (at least one slot).
static int blk_ntile(int np) {
  const int m = np / blk_b2();
  return m > 1 ? m * (m - 1) / 2 : 1;
}

template <typename T>
static size_t blk_bytes(int n) {
  int np = blk_np(n), m = np / blk_b2();
  size_t b = 0;
  b += align_up((size_t)np * np * sizeof(T), 256);
  b += align_up((size_t)n * np * sizeof(T), 256);
  b += align_up((size_t)2 * m * blk_b2() * blk_b2() * sizeof(T), 256);   // E, two step parities
  b += align_up((size_t)2 * m * sizeof(int), 256);
  b += align_up((size_t)blk_ntile(np) * sizeof(int), 256);   // tile reader counters
  return b;
}

// Workspace of the FP32 step 1: the larger of the Jacobi stage (blocked or element) and the
// tridiagonal route, plus an FP64 eigenvalue buffer.
static size_t stage1_bytes(int n) {
  size_t jac32 = blk_bytes<float>(n) + elem_bytes<float>(n) + 2 * align_up((size_t)n * n * 4, 256) +
                 align_up((size_t)n * 4, 256);
  size_t tri = tridiag_bytes(n);
  return (jac32 > tri ? jac32 : tri) + align_up((size_t)n * 8, 256) + 4 * 256;
}

static size_t syev_bytes(int n, int precond) {
  size_t b = 0;
  b += blk_bytes<double>(n);
  b += 4096 + 1024 * 8 + 2 * kRotSlots * 8 + align_up((size_t)n * 4, 256) + 256;
  b += elem_bytes<double>(n);
  b += align_up((size_t)n * n * 8, 256);           // Vw
  b += align_up((size_t)n * 8, 256);               // d
  if (precond != JAC_PRECOND_NONE) {
    b += 2 * align_up((size_t)n * n * 8, 256);     // GEMM scratch W, T0
    b += align_up(mgs_scratch_elems(n, n) * 8, 256);
    b += 2 * align_up((size_t)n * n * 8, 256) + align_up((size_t)(2 * n + 64) * 8, 256);   // step-2 series
    b += stage1_bytes(n);
  }
  return b + 64 * 256;
}

// Scalars block at the start of every workspace.
struct Head {
  double* scal;               // [0] off^2, [1] fro^2
  double* partial;            // 1024 partial sums
  unsigned long long* rot64;  // FP64 rotation counters
  unsigned long long* rot32;  // FP32 rotation counters
  int* flag;
  unsigned long long* work;   // per kernel class work counters [8]
};

static Head carve_head(Carve& c, int) {
  Head h;
  h.scal = c.take<double>(16);
  h.partial = c.take<double>(1024);
  h.rot64 = c.take<unsigned long long>(kRotSlots);
  h.rot32 = c.take<unsigned long long>(kRotSlots);
  h.flag = c.take<int>(16);
  h.work = c.take<unsigned long long>(8);
  return h;
}

template <typename T>
static void carve_elem(Carve& c, ElemState<T>& st, int n) {
  st.n = n;
  st.ne = n + (n & 1);
  st.h = st.ne / 2;
  st.nblk = (long long)st.h * (st.h + 1) / 2;
  st.Tp[0] = c.take<Blk<T>>(st.nblk);
  st.Tp[1] = c.take<Blk<T>>(st.nblk);
  st.A[0] = c.take<Ang<T>>(st.h);
  st.A[1] = c.take<Ang<T>>(st.h);
  st.cur = 0;
}

// Run sweeps of the element-wise path until off <= tol*nrm or max_sweeps.
// Returns 0 (converged), 1 (not converged), or an error code.  off history in
// hist (host, may be NULL, length hist_len).
template <typename T>
static int elem_run(ElemState<T>& st, double tol, double nrm, int max_sweeps, hipStream_t s, int* sweeps_out,
                    double* off_out, double* hist, int hist_len, long long* rot_out, double* step_ms = nullptr,
                    long long* launches = nullptr) {
  const int per = st.ne - 1;
  hipEvent_t ea = nullptr, eb = nullptr;
  if (step_ms) {
    JAC_HIP(hipEventCreate(&ea));
    JAC_HIP(hipEventCreate(&eb));
    *step_ms = 0;
  }
  JAC_HIP(hipMemsetAsync(st.rot, 0, kRotSlots * sizeof(unsigned long long), s));
  int e = elem_init_angles<T>(st, 0, s);
  if (e) return e;
  double off2 = 0;
  e = elem_offnorm2<T>(st, s);
  if (e) return e;
  JAC_HIP(hipMemcpyAsync(&off2, st.scalars, 8, hipMemcpyDeviceToHost, s));
  JAC_HIP(hipStreamSynchronize(s));
  double off = std::sqrt(off2);
  if (hist && hist_len > 0) hist[0] = off;
  int sweeps = 0;
  if (max_sweeps > kRotSlots - 2) max_sweeps = kRotSlots - 2;
  while (off > tol * nrm && sweeps < max_sweeps) {
    if (ea) JAC_HIP(hipEventRecord(ea, s));
    e = elem_steps<T>(st, (long long)sweeps * per, per, s);
    if (e) return e;
    if (eb) JAC_HIP(hipEventRecord(eb, s));
    ++sweeps;
    e = elem_offnorm2<T>(st, s);
    if (e) return e;
    JAC_HIP(hipMemcpyAsync(&off2, st.scalars, 8, hipMemcpyDeviceToHost, s));
    JAC_HIP(hipStreamSynchronize(s));
    if (st.prof) st.prof->flush();
    if (ea) {
      float ms = 0;
      JAC_HIP(hipEventElapsedTime(&ms, ea, eb));
      *step_ms += ms;
    }
    off = std::sqrt(off2);
    if (hist && sweeps < hist_len) hist[sweeps] = off;
    if (!(off == off)) break;
  }
  if (rot_out) {
    unsigned long long cnt[kRotSlots];
    JAC_HIP(hipMemcpyAsync(cnt, st.rot, kRotSlots * 8, hipMemcpyDeviceToHost, s));
    JAC_HIP(hipStreamSynchronize(s));
    long long tot = 0;
    for (int i = 0; i < sweeps; ++i) tot += (long long)cnt[i];
    *rot_out = tot;
  }
  if (sweeps_out) *sweeps_out = sweeps;
  if (off_out) *off_out = off;
  if (launches) *launches = (long long)sweeps * per;
  if (ea) (void)hipEventDestroy(ea);
  if (eb) (void)hipEventDestroy(eb);
  return off > tol * nrm ? 1 : 0;
}

template <typename T>
static void carve_blk(Carve& c, BlkState<T>& st, int n) {
  st.n = n;
  st.np = blk_np(n);
  st.ldt = st.np;
  st.Tm = c.take<T>((size_t)st.np * st.np);
  st.nvr = n;
  st.ldv = n > 1 ? n : 1;
  st.V = c.take<T>((size_t)n * st.np);
  st.W = c.take<T>((size_t)2 * (st.np / blk_b2()) * blk_b2() * blk_b2());   // two step parities
  st.ident = c.take<int>(2 * (st.np / blk_b2()));
  st.tcount = c.take<int>(blk_ntile(st.np));
}

// Blocked sweeps until off <= tol*nrm or max_sweeps (same contract as elem_run).
template <typename T>
static int blk_run(BlkState<T>& st, double tol, double nrm, int max_sweeps, int max_inner, hipStream_t s,
                   int* sweeps_out, double* off_out, double* hist, int hist_len, long long* rot_out,
                   double* step_ms = nullptr, long long* launches = nullptr) {
  hipEvent_t ea = nullptr, eb = nullptr;
  if (step_ms) {
    JAC_HIP(hipEventCreate(&ea));
    JAC_HIP(hipEventCreate(&eb));
    *step_ms = 0;
  }
  JAC_HIP(hipMemsetAsync(st.rot, 0, sizeof(unsigned long long), s));
  JAC_HIP(hipMemsetAsync(st.tcount, 0, (size_t)blk_ntile(st.np) * sizeof(int), s));
  double off2 = 0;
  int e = blk_offnorm2<T>(st, s);
  if (e) return e;
  JAC_HIP(hipMemcpyAsync(&off2, st.scalars, 8, hipMemcpyDeviceToHost, s));
  JAC_HIP(hipStreamSynchronize(s));
  double off = std::sqrt(off2);
  if (hist && hist_len > 0) hist[0] = off;
  int sweeps = 0;
  const int per = st.np / (blk_b2() / 2) - 1;
  while (off > tol * nrm && sweeps < max_sweeps) {
    if (ea) JAC_HIP(hipEventRecord(ea, s));
    e = blk_sweep<T>(st, max_inner, s);
    if (e) return e;
    if (eb) JAC_HIP(hipEventRecord(eb, s));
    ++sweeps;
    e = blk_offnorm2<T>(st, s);
    if (e) return e;
    JAC_HIP(hipMemcpyAsync(&off2, st.scalars, 8, hipMemcpyDeviceToHost, s));
    JAC_HIP(hipStreamSynchronize(s));
    if (st.prof) st.prof->flush();
    if (ea) {
      float ms = 0;
      JAC_HIP(hipEventElapsedTime(&ms, ea, eb));
      *step_ms += ms;
    }
    off = std::sqrt(off2);
    if (hist && sweeps < hist_len) hist[sweeps] = off;
    if (!(off == off)) break;
  }
  if (rot_out) {
    unsigned long long cnt = 0;
    JAC_HIP(hipMemcpyAsync(&cnt, st.rot, 8, hipMemcpyDeviceToHost, s));
    JAC_HIP(hipStreamSynchronize(s));
    *rot_out = (long long)cnt;
  }
  if (sweeps_out) *sweeps_out = sweeps;
  if (off_out) *off_out = off;
  if (launches) *launches = (long long)sweeps * per * 2;
  if (ea) (void)hipEventDestroy(ea);
  if (eb) (void)hipEventDestroy(eb);
  return off > tol * nrm ? 1 : 0;
}

static bool use_blocked(int variant, int n) {
  if (variant == JAC_VARIANT_ELEMENT) return false;
  if (variant == JAC_VARIANT_BLOCKED) return true;
  return n >= 2;
}

constexpr int kMaxInner64 = 1;
constexpr int kMaxInner32 = 1;
constexpr int kSvdInner = 4;

struct Timer {
  hipEvent_t ev[8];
  int used = 0;
  hipStream_t s;
  bool on;
  Timer(hipStream_t st, bool enable) : s(st), on(enable) {
    if (on)
      for (int i = 0; i < 8; ++i) (void)hipEventCreate(&ev[i]);
  }
  ~Timer() {
    if (on)
      for (int i = 0; i < 8; ++i) (void)hipEventDestroy(ev[i]);
  }
  void mark(int i) {
    if (on) (void)hipEventRecord(ev[i], s);
  }
  float ms(int a, int b) {
    if (!on) return 0.f;
    float t = 0;
    (void)hipEventSynchronize(ev[b]);
    (void)hipEventElapsedTime(&t, ev[a], ev[b]);
    return t;
  }
};

// FP32 stage (Algorithm 4.1 step 1): eigenvectors of fl32(A) by the FP32
// element-wise round-robin Jacobi.  Z (FP64, n x n, ldz) receives them in
// working (unsorted) order; d32 (device, may be NULL) the FP32 diagonal.
// The library's choice: the tridiagonal route where its reduction keeps the working rows in
// registers (16 <= n <= 4096; measured at n = 4096 it takes 1.06 s over the three test spectra
// against 1.26 s with the Jacobi stage), the FP32 Jacobi stage elsewhere.
static bool use_tridiag(int stage1, int n) {
  if (!tridiag_supported(n)) return false;
  if (stage1 == JAC_STAGE1_TRIDIAG) return true;
  return stage1 == JAC_STAGE1_AUTO && n >= 16 && n <= 4096;
}

// stage1: jac_stage1_t; *method receives the solver that ran (1 Jacobi, 2 tridiagonal).  The
// tridiagonal route returns Z in ascending order of the eigenvalues of T (no sweeps); no_split
// keeps its GEMMs free of split-K buffers.
static int fp32_stage(const void* A, bool a_dbl, int n, int lda, double nrmA, double tol32, int max32, double* Z,
                      int ldz, float* d32, Carve& c, Head& hd, hipStream_t s, int* sweeps, long long* rots,
                      double* step_ms = nullptr, long long* launches = nullptr, int variant = 0,
                      int inner = 0, Prof* prof = nullptr, int stage1 = JAC_STAGE1_JACOBI, int* method = nullptr,
                      bool no_split = false) {
  if (use_tridiag(stage1, n)) {
    if (method) *method = 2;
    if (sweeps) *sweeps = 0;
    if (rots) *rots = 0;
    if (launches) *launches = 0;
    if (step_ms) *step_ms = 0;
    double* w = d32 ? c.take<double>(n) : nullptr;
    int e = a_dbl ? eig_tridiag_f32<double>((const double*)A, n, lda, Z, ldz, w, c, s, no_split, prof)
                  : eig_tridiag_f32<float>((const float*)A, n, lda, Z, ldz, w, c, s, no_split, prof);
    if (e) return e;
    if (d32) {
      e = copy_convert<double, float>(w, n, 1, n, d32, n, s);
      if (e) return e;
    }
    return 0;
  }
  if (method) *method = 1;
  if (use_blocked(variant, n)) {
    BlkState<float> st;
    carve_blk(c, st, n);
    st.prof = prof;
    st.cls_inner = 2;
    st.cls_update = 3;
    st.partial = hd.partial;
    st.scalars = hd.scal;
    st.rot = hd.rot32;
    st.skip_abs = (float)(tol32 * nrmA / n);
    int e = blk_load<float>(st, A, a_dbl, lda, s);
    if (e) return e;
    JAC_HIP(hipMemsetAsync(st.V, 0, (size_t)n * st.np * sizeof(float), s));
    e = set_identity<float>(st.V, n, st.ldv, s);
    if (e) return e;
    double off = 0;
    e = blk_run<float>(st, tol32, nrmA, max32, inner > 0 ? inner : kMaxInner32, s, sweeps, &off, nullptr, 0, rots,
                       step_ms, launches);
    if (e < 0 || e > 1) return e;
    e = copy_convert<float, double>(st.V, n, n, st.ldv, Z, ldz, s);
    if (e) return e;
    if (d32) {
      e = blk_diag<float>(st, d32, s);
      if (e) return e;
    }
    return 0;
  }
  ElemState<float> st;
  carve_elem(c, st, n);
  st.prof = prof;
  st.cls = 5;
  float* A32 = c.take<float>((size_t)n * n);
  float* V32 = c.take<float>((size_t)n * n);
  st.V = V32;
  st.ldv = n;
  st.partial = hd.partial;
  st.scalars = hd.scal;
  st.rot = hd.rot32;
  st.skip_abs = (float)(tol32 * nrmA / n);
  int e = a_dbl ? copy_convert<double, float>((const double*)A, n, n, lda, A32, n, s)
                : copy_convert<float, float>((const float*)A, n, n, lda, A32, n, s);
  if (e) return e;
  e = elem_pack_from<float>(st, A32, n, 0, s);
  if (e) return e;
  e = set_identity<float>(V32, n, n, s);
  if (e) return e;
  double off = 0;
  e = elem_run<float>(st, tol32, nrmA, max32, s, sweeps, &off, nullptr, 0, rots, step_ms, launches);
  if (e < 0 || e > 1) return e;
  e = copy_convert<float, double>(V32, n, n, n, Z, ldz, s);
  if (e) return e;
  if (d32) {
    e = elem_diag<float>(st, d32, s);
    if (e) return e;
  }
  return 0;
}

// T = Q^T A Q: Q^T is formed explicitly in T (a coalesced tiled transpose), then W = Q^T A and
// T = W Q as untransposed GEMMs (a transposed operand streams 128-byte pieces of columns and
// runs an order of magnitude slower), then T is mirrored from its upper triangle, the only part
// the second product forms.
__global__ void mirror_upper_kernel(double* T, int n, int ldt) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  int j = blockIdx.y;
  if (i < n && i > j) T[i + (size_t)j * ldt] = T[j + (size_t)i * ldt];
}

// B = A^T for an n x n block (32 x 32 tiles staged through LDS).
__global__ void transpose_kernel(const double* __restrict__ A, int n, int lda, double* __restrict__ B, int ldb) {
  __shared__ double t[32][33];
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 256 threads: 8 rows of 32
  for (int r = ty; r < 32; r += 8) {
    const int i = bx + tx, j = by + r;
    if (i < n && j < n) t[r][tx] = A[i + (size_t)j * lda];
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int i = by + tx, j = bx + r;
    if (i < n && j < n) B[i + (size_t)j * ldb] = t[tx][r];
  }
}

// no_split: the GEMMs take no split-K partial buffer (which the library allocates on demand).
static int similarity(const double* A, int n, int lda, const double* Q, int ldq, double* T, int ldt, double* W,
                      hipStream_t s, bool no_split = false) {
  hipLaunchKernelGGL(transpose_kernel, dim3(cdiv(n, 32), cdiv(n, 32)), dim3(256), 0, s, Q, n, ldq, T, ldt);
  JAC_CHECK_LAUNCH();
  const int ms = no_split ? 1 : 0;
  int e = gemm<double>(false, false, n, n, n, 1.0, T, ldt, A, lda, 0.0, W, n, s, ms);
  if (e) return e;
  // (only T's upper triangle is formed: the tiles below the diagonal are skipped, then mirrored)
  e = gemm<double>(false, false, n, n, n, 1.0, W, n, Q, ldq, 0.0, T, ldt, s, ms, kGemmCUpper);
  if (e) return e;
  hipLaunchKernelGGL(mirror_upper_kernel, dim3(cdiv(n, 256), n), dim3(256), 0, s, T, n, ldt);
  JAC_CHECK_LAUNCH();
  return 0;
}

static double default_tol(double tol) { return tol > 0 ? tol : 20.0 * 1.1102230246251565e-16; }

// Shared driver of syev_jacobi_ex / syev_jacobi_warm.
// fixed_ws (device, fixed_cap bytes): use it instead of the library's pooled workspace and create
// no events (no stage or kernel timing), so that the call allocates nothing.
static int syev_impl(const double* A, int n, int lda, const double* Q0, int ldq, double* W, double* V, int ldv,
                     double tol, const jac_opts* opts, jac_stats* stats, hipStream_t s, void* fixed_ws = nullptr,
                     size_t fixed_cap = 0) {
  jac_opts o{};
  if (opts) o = *opts;
  if (Q0) o.precond = -1;  // custom start
  const bool fixed = fixed_ws != nullptr;
  if (fixed) o.profile = 0;
  const int max_sweeps = o.max_sweeps > 0 ? o.max_sweeps : kMaxSweepsDefault;
  tol = default_tol(tol);
  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
  }
  if (o.block_b != 0) {
    set_error("syev_jacobi_ex: opts.block_b is reserved and must be 0");
    return -8;
  }
  if (o.stage1 < JAC_STAGE1_AUTO || o.stage1 > JAC_STAGE1_TRIDIAG) {
    set_error("syev_jacobi_ex: opts.stage1 must be a jac_stage1_t");
    return -8;
  }
  if (o.stage1_prec < JAC_PREC_FP32 || o.stage1_prec > JAC_PREC_BF16) {
    set_error("syev_jacobi_ex: opts.stage1_prec must be a jac_prec_t");
    return -8;
  }
  if (n == 0) return 0;
  if (o.precond != JAC_PRECOND_NONE && n > kMgsMaxRows) {
    set_error("syev_jacobi: preconditioned solves (and custom starts) need n <= 32768 (block MGS of step 2)");
    return -2;
  }
  if (o.precond == JAC_PRECOND_MLP) {
    if (!o.mlp || !o.theta) {
      set_error("syev_jacobi_ex: the learned start needs opts.mlp and opts.theta");
      return -8;
    }
    if (mlp_order(o.mlp) != n) {
      set_error("syev_jacobi_ex: the network predicts eigenvectors of another order");
      return -8;
    }
  }
  Timer tm(s, stats != nullptr && !fixed);
  tm.mark(0);
  const int pre = o.precond;
  const size_t need = syev_bytes(n, pre == JAC_PRECOND_NONE ? 0 : 1);
  if (fixed && need > fixed_cap) {
    set_error("syev_jacobi_noalloc: order n needs " + std::to_string(need) + " bytes of workspace, more than the " +
              std::to_string(fixed_cap) + " of the fixed device array");
    return -2;
  }
  void* ws = fixed ? fixed_ws : workspace(need);
  if (!ws) {
    set_error("syev_jacobi: workspace allocation failed");
    return 4;
  }
  Carve c(ws);
  Head hd = carve_head(c, n);
  Prof prof;
  prof.on = stats != nullptr && o.profile != 0;
  prof.work = hd.work;
  Prof* pf = prof.on ? &prof : nullptr;
  JAC_HIP(hipMemsetAsync(hd.flag, 0, 16 * sizeof(int), s));
  JAC_HIP(hipMemsetAsync(hd.work, 0, 8 * sizeof(unsigned long long), s));
  int e = check_finite(A, n, n, lda, hd.flag, s);
  if (e) return e;
  e = fro2_f64(A, n, n, lda, hd.partial, hd.scal + 1, s);
  if (e) return e;
  double hs[2];
  int hflag = 0;
  JAC_HIP(hipMemcpyAsync(hs, hd.scal, 16, hipMemcpyDeviceToHost, s));
  JAC_HIP(hipMemcpyAsync(&hflag, hd.flag, 4, hipMemcpyDeviceToHost, s));
  JAC_HIP(hipStreamSynchronize(s));
  if (hflag) {
    set_error("syev_jacobi: A contains NaN or Inf");
    return 2;
  }
  const double nrm = std::sqrt(hs[1]);
  if (stats) stats->nrmA = nrm;
  tm.mark(1);

  ElemState<double> st;
  carve_elem(c, st, n);
  double* Vw = c.take<double>((size_t)n * n);
  double* d = c.take<double>(n);
  int* rank = c.take<int>(n);
  st.V = Vw;
  st.ldv = n;
  st.partial = hd.partial;
  st.scalars = hd.scal;
  st.rot = hd.rot64;
  st.skip_abs = tol * nrm / n;
  st.prof = pf;
  st.cls = 4;

  float ms_pre = 0, ms_mgs = 0, ms_sim = 0;
  double* T0p = nullptr;
  if (pre == JAC_PRECOND_NONE || nrm == 0.0) {
    e = elem_pack<double>(st, A, lda, 0, s);
    if (e) return e;
    e = set_identity<double>(Vw, n, n, s);
    if (e) return e;
    tm.mark(2);
    tm.mark(3);
    tm.mark(4);
  } else {
    double* Wg = c.take<double>((size_t)n * n);
    double* T0 = c.take<double>((size_t)n * n);
    T0p = T0;
    double* mscr = c.take<double>(mgs_scratch_elems(n, n));
    double* oB3 = c.take<double>((size_t)n * n);
    double* oB4 = c.take<double>((size_t)n * n);
    double* opart = c.take<double>((size_t)2 * n + 64);
    bool accepted = false;
    bool mgs_done = false;   // the tridiagonal start is orthogonalised inside the stage-1 block
    int method1 = 0;
    // Step 2: the QR factor of the start (what MGS returns), by the series on the matrix cores when
    // the start is nearly orthonormal, else by block MGS.
    auto step2 = [&](double* Zs) -> int {
      int used = 0;
      int r = orth_series_f64(Zs, n, n, Wg, T0, oB3, oB4, opart, hd.scal + 3, &used, s, fixed);
      if (r) return r;
      if (!used) return mgs_f64(Zs, n, n, n, mscr, hd.flag, s);
      return 0;
    };
    if (pre == JAC_PRECOND_MLP) {
      // Learned start: Z -> MGS -> T = Q^T A Q; kept when ||off(T)||_F / ||A||_F <= fallback_tol
      // and MGS met no zero column, else replaced by the FP32 start.
      e = mlp_predict_f64(o.mlp, o.theta, Vw, n, s);
      if (e) return e;
      tm.mark(2);
      // A predicted Z can be far from orthogonal (condition number well above 1), where one MGS
      // pass leaves ||Q^T Q - I|| ~ u cond(Z); a second pass restores it to ~u.
      e = mgs_f64(Vw, n, n, n, mscr, hd.flag, s);
      if (e) return e;
      e = mgs_f64(Vw, n, n, n, mscr, hd.flag, s);
      if (e) return e;
      tm.mark(3);
      e = similarity(A, n, lda, Vw, n, T0, n, Wg, s);
      if (e) return e;
      e = off2_f64(T0, n, n, hd.partial, hd.scal + 2, s);
      if (e) return e;
      double off2 = 0;
      JAC_HIP(hipMemcpyAsync(&off2, hd.scal + 2, 8, hipMemcpyDeviceToHost, s));
      JAC_HIP(hipMemcpyAsync(&hflag, hd.flag, 4, hipMemcpyDeviceToHost, s));
      JAC_HIP(hipStreamSynchronize(s));
      const double r = hflag ? HUGE_VAL : std::sqrt(off2) / nrm;
      const double ftol = o.fallback_tol > 0 ? o.fallback_tol : 1e-2;
      if (stats) stats->start_resid = r;
      if (r <= ftol) {
        accepted = true;
      } else {
        if (stats) stats->used_fallback = 1;
        JAC_HIP(hipMemsetAsync(hd.flag, 0, 16 * sizeof(int), s));
      }
    }
    if (accepted) {
      // T0 and Q already hold the accepted start.
    } else if (pre == JAC_PRECOND_FP32 || pre == JAC_PRECOND_MLP) {
      // Default stop of the FP32 eigensolve: off(T32) <= 1e-4 ||A||_F.  Its last sweeps
      // (1e-4 -> 1e-6) cost more FP32 time than the FP64 sweeps they save: measured at
      // n = 2048 over the three test spectra, the whole solve is fastest near 1e-4.
      double tol32 = o.fp32_tol > 0 ? o.fp32_tol : 1e-4;
      int max32 = o.fp32_max_sweeps > 0 ? o.fp32_max_sweeps : 30;
      int sw32 = 0;
      long long r32 = 0;
      double ms32 = 0;
      long long l32 = 0;
      Carve c1 = c;   // the FP32 stage's carve, reused if it has to run again
      // Step 1 at precision upsilon below FP32: the eigensolver sees fl_upsilon(A) (held in T0
      // until step 3 overwrites it) and its eigenvectors are rounded to upsilon as well.
      const double* As = A;
      int las = lda;
      const double lp_scale = std::ldexp(1.0, -std::ilogb(nrm) - 1);   // ||A||_F scale < 1
      if (o.stage1_prec != JAC_PREC_FP32) {
        e = copy_convert<double, double>(A, n, n, lda, T0, n, s);
        if (e) return e;
        e = round_lowp(T0, n, n, n, o.stage1_prec, o.stage1_prec == JAC_PREC_FP16 ? lp_scale : 1.0, s);
        if (e) return e;
        As = T0;
        las = n;
      }
      e = fp32_stage(As, true, n, las, nrm, tol32, max32, Vw, n, nullptr, c, hd, s, &sw32, &r32,
                     stats && !fixed ? &ms32 : nullptr, &l32, o.variant, o.inner_sweeps, pf, o.stage1, &method1,
                     fixed);
      if (e) return e;
      if (o.stage1_prec != JAC_PREC_FP32) {
        e = round_lowp(Vw, n, n, n, o.stage1_prec, 1.0, s);
        if (e) return e;
      }
      if (method1 == 2) {
        // A tridiagonal start whose columns MGS cannot orthogonalise (a zero column: eigenvectors of
        // T computed for numerically equal eigenvalues) is replaced by the FP32 Jacobi start.
        tm.mark(2);
        e = step2(Vw);
        if (e) return e;
        JAC_HIP(hipMemcpyAsync(&hflag, hd.flag, 4, hipMemcpyDeviceToHost, s));
        JAC_HIP(hipStreamSynchronize(s));
        mgs_done = hflag == 0;
        if (hflag) {
          JAC_HIP(hipMemsetAsync(hd.flag, 0, 16 * sizeof(int), s));
          c = c1;
          e = fp32_stage(As, true, n, las, nrm, tol32, max32, Vw, n, nullptr, c, hd, s, &sw32, &r32,
                         stats && !fixed ? &ms32 : nullptr, &l32, o.variant, o.inner_sweeps, pf,
                         JAC_STAGE1_JACOBI, &method1, fixed);
          if (e) return e;
          if (o.stage1_prec != JAC_PREC_FP32) {
            e = round_lowp(Vw, n, n, n, o.stage1_prec, 1.0, s);
            if (e) return e;
          }
        }
      }
      if (stats) {
        stats->fp32_sweeps = sw32;
        stats->fp32_rotations = r32;
        stats->fp32_step_ms = ms32;
        stats->fp32_step_launches = l32;
        stats->fp32_method = method1;
      }
    } else {
      e = copy_convert<double, double>(Q0, n, n, ldq, Vw, n, s);
      if (e) return e;
    }
    if (!accepted) {
      if (!mgs_done) {
        tm.mark(2);
        e = step2(Vw);
        if (e) return e;
      }
      tm.mark(3);
      e = similarity(A, n, lda, Vw, n, T0, n, Wg, s, fixed);
      if (e) return e;
    }
    e = elem_pack<double>(st, T0, n, 0, s);
    if (e) return e;
    if (!mgs_done) {   // (after an early step 2 the flag was read already and nothing since sets it)
      JAC_HIP(hipMemcpyAsync(&hflag, hd.flag, 4, hipMemcpyDeviceToHost, s));
      JAC_HIP(hipStreamSynchronize(s));
      if (hflag) {
        set_error("syev_jacobi: modified Gram-Schmidt met a zero column");
        return 3;
      }
    }
    tm.mark(4);
  }
  int sweeps = 0;
  double off = 0;
  long long rots = 0;
  double ms64 = 0;
  long long l64 = 0;
  int info;
  const bool blocked = use_blocked(o.variant, n);
  BlkState<double> bst;
  if (blocked) {
    carve_blk(c, bst, n);
    bst.partial = hd.partial;
    bst.scalars = hd.scal;
    bst.rot = hd.rot64;
    bst.skip_abs = tol * nrm / n;
    bst.prof = pf;
    bst.cls_inner = 0;
    bst.cls_update = 1;
    const bool plain = (pre == JAC_PRECOND_NONE || nrm == 0.0);
    e = blk_load<double>(bst, plain ? (const void*)A : (const void*)T0p, true, plain ? lda : n, s);
    if (e) return e;
    JAC_HIP(hipMemsetAsync(bst.V, 0, (size_t)n * bst.np * sizeof(double), s));
    e = copy_convert<double, double>(Vw, n, n, n, bst.V, bst.ldv, s);
    if (e) return e;
    info = blk_run<double>(bst, tol, nrm, max_sweeps, o.inner_sweeps > 0 ? o.inner_sweeps : kMaxInner64, s,
                           &sweeps, &off,
                           stats ? stats->off_hist : nullptr, JAC_HIST, &rots, stats && !fixed ? &ms64 : nullptr,
                           &l64);
  } else {
    info = elem_run<double>(st, tol, nrm, max_sweeps, s, &sweeps, &off, stats ? stats->off_hist : nullptr,
                            JAC_HIST, &rots, stats && !fixed ? &ms64 : nullptr, &l64);
  }
  if (info < 0 || info > 1) return info;
  tm.mark(5);
  if (blocked) {
    e = blk_diag<double>(bst, d, s);
    if (e) return e;
    e = sort_eigs<double>(d, bst.V, n, bst.ldv, W, V, ldv, rank, s);
  } else {
    e = elem_diag<double>(st, d, s);
    if (e) return e;
    e = sort_eigs<double>(d, Vw, n, n, W, V, ldv, rank, s);
  }
  if (e) return e;
  tm.mark(6);
  JAC_HIP(hipStreamSynchronize(s));
  if (stats) {
    stats->sweeps = sweeps;
    stats->rotations = rots;
    stats->step_ms = ms64;
    stats->step_launches = l64;
    stats->off0 = stats->off_hist[0];
    stats->off_final = off;
    stats->stage_ms[6] = tm.ms(0, 1);
    stats->stage_ms[0] = tm.ms(1, 2);
    stats->stage_ms[1] = tm.ms(2, 3);
    stats->stage_ms[2] = tm.ms(3, 4);
    stats->stage_ms[3] = tm.ms(4, 5);
    stats->stage_ms[4] = tm.ms(5, 6);
    stats->stage_ms[5] = tm.ms(0, 6);
    if (prof.on) {
      unsigned long long wk[8];
      JAC_HIP(hipMemcpy(wk, hd.work, sizeof(wk), hipMemcpyDeviceToHost));
      for (int i = 0; i < 8; ++i) {
        stats->kern_ms[i] = prof.ms[i];
        stats->kern_launches[i] = prof.launches[i];
        stats->kern_work[i] = (long long)wk[i];
      }
    }
  }
  (void)ms_pre; (void)ms_mgs; (void)ms_sim;
  return info;
}


// ------------------------------------------------------------------ one-sided SVD
static int svd_gsplit(int m, int npair) {
  int g = 512 / (npair > 0 ? npair : 1);
  int gmax = m / 128 > 1 ? m / 128 : 1;
  if (g > gmax) g = gmax;
  if (g < 1) g = 1;
  return g;
}

static size_t gesvd_bytes(int m, int n, int precond) {
  int np = blk_np(n), npair = np / blk_b2();
  int g = svd_gsplit(m, npair);
  size_t b = 4096 + 1024 * 8 + 2 * kRotSlots * 8 + 64 * 256;
  b += align_up((size_t)m * np * 8, 256);                       // C
  b += align_up((size_t)n * np * 8, 256);                       // V work
  b += align_up((size_t)npair * blk_b2() * blk_b2() * 8, 256);  // E
  b += align_up((size_t)npair * 4, 256);
  b += align_up((size_t)g * npair * blk_b2() * blk_b2() * 8, 256);  // Gram partials
  b += 2 * align_up((size_t)n * 8, 256);
  if (precond != JAC_PRECOND_NONE) {
    b += align_up((size_t)m * n * 4, 256) + align_up((size_t)n * n * 4, 256);  // A32, G32
    b += align_up((size_t)n * n * 8, 256);                                      // Z / Q
    b += align_up(mgs_scratch_elems(n, n) * 8, 256);
    b += syev_bytes(n, 1);                                                      // FP32 eig work
    b += stage1_bytes(n);
  }
  return b;
}

__global__ void zero_cols_kernel(double* C, int m, int ldc, int c0) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) C[i + (size_t)(c0 + blockIdx.y) * ldc] = 0.0;
}

static int gesvd_impl(const double* A, int m, int n, int lda, double* S, double* U, int ldu, double* V, int ldv,
                      double tol, const jac_opts* opts, jac_stats* stats, hipStream_t s) {
  jac_opts o{};
  if (opts) o = *opts;
  const int max_sweeps = o.max_sweeps > 0 ? o.max_sweeps : kMaxSweepsDefault;
  if (tol <= 0) tol = 1.1102230246251565e-16;  // epsilon = omega for the SVD (Section 6 setup)
  if (stats) std::memset(stats, 0, sizeof(*stats));
  if (n == 0) return 0;
  Timer tm(s, stats != nullptr);
  tm.mark(0);
  const int pre = o.precond;
  if (pre == JAC_PRECOND_MLP) { set_error("gesvd_jacobi: no learned start for the SVD"); return -10; }
  if (o.stage1_prec != JAC_PREC_FP32) {
    set_error("gesvd_jacobi_ex: opts.stage1_prec applies to the symmetric eigensolver only");
    return -11;
  }
  if (pre != JAC_PRECOND_NONE && n > kMgsMaxRows) {
    set_error("gesvd_jacobi: the preconditioned SVD needs n <= 32768 (block MGS of step 2)");
    return -3;
  }
  if (o.block_b != 0) { set_error("gesvd_jacobi_ex: opts.block_b is reserved and must be 0"); return -11; }
  if (o.stage1 < JAC_STAGE1_AUTO || o.stage1 > JAC_STAGE1_TRIDIAG) {
    set_error("gesvd_jacobi_ex: opts.stage1 must be a jac_stage1_t");
    return -11;
  }
  void* ws = workspace(gesvd_bytes(m, n, pre));
  if (!ws) { set_error("gesvd_jacobi: workspace allocation failed"); return 4; }
  Carve c(ws);
  Head hd = carve_head(c, n);
  JAC_HIP(hipMemsetAsync(hd.flag, 0, 16 * sizeof(int), s));
  int e = check_finite(A, m, n, lda, hd.flag, s);
  if (e) return e;
  e = fro2_f64(A, m, n, lda, hd.partial, hd.scal + 1, s);
  if (e) return e;
  double hs[2];
  int hflag = 0;
  JAC_HIP(hipMemcpyAsync(hs, hd.scal, 16, hipMemcpyDeviceToHost, s));
  JAC_HIP(hipMemcpyAsync(&hflag, hd.flag, 4, hipMemcpyDeviceToHost, s));
  JAC_HIP(hipStreamSynchronize(s));
  if (hflag) { set_error("gesvd_jacobi: A contains NaN or Inf"); return 2; }
  const double nrm = std::sqrt(hs[1]);
  if (stats) stats->nrmA = nrm;
  const int np = blk_np(n), npair = np / blk_b2();
  const int gsplit = svd_gsplit(m, npair);
  double* C = c.take<double>((size_t)m * np);
  double* Vw = c.take<double>((size_t)n * np);
  double* E = c.take<double>((size_t)npair * blk_b2() * blk_b2());
  int* ident = c.take<int>(npair);
  double* Gp = c.take<double>((size_t)gsplit * npair * blk_b2() * blk_b2());
  double* sig = c.take<double>(n);
  int* rank = c.take<int>(n);
  JAC_HIP(hipMemsetAsync(Vw, 0, (size_t)n * np * 8, s));
  tm.mark(1);
  if (pre == JAC_PRECOND_NONE || nrm == 0.0) {
    e = copy_convert<double, double>(A, m, n, lda, C, m, s);
    if (e) return e;
    e = set_identity<double>(Vw, n, n, s);
    if (e) return e;
    tm.mark(2);
    tm.mark(3);
  } else {
    // Step 1 (reading of Algorithm 5.2): right singular vectors of fl32(A) as the
    // FP32 eigenvectors of the FP32 Gram matrix A32^T A32.
    float* A32 = c.take<float>((size_t)m * n);
    float* G32 = c.take<float>((size_t)n * n);
    double* Z = c.take<double>((size_t)n * n);
    double* mscr = c.take<double>(mgs_scratch_elems(n, n));
    e = copy_convert<double, float>(A, m, n, lda, A32, m, s);
    if (e) return e;
    e = gemm<float>(true, false, n, n, m, 1.0f, A32, m, A32, m, 0.0f, G32, n, s);
    if (e) return e;
    double tol32 = o.fp32_tol > 0 ? o.fp32_tol : 1e-6;
    int max32 = o.fp32_max_sweeps > 0 ? o.fp32_max_sweeps : 30;
    int sw32 = 0;
    long long r32 = 0;
    int method1 = 0;
    e = fp32_stage(G32, false, n, n, nrm * nrm, tol32, max32, Z, n, nullptr, c, hd, s, &sw32, &r32, nullptr,
                   nullptr, o.variant, o.inner_sweeps, nullptr, o.stage1, &method1);
    if (e) return e;
    if (stats) { stats->fp32_sweeps = sw32; stats->fp32_rotations = r32; stats->fp32_method = method1; }
    tm.mark(2);
    e = mgs_f64(Z, n, n, n, mscr, hd.flag, s);   // step 2
    if (e) return e;
    tm.mark(3);
    e = gemm<double>(false, false, m, n, n, 1.0, A, lda, Z, n, 0.0, C, m, s);   // step 3: C = A Q
    if (e) return e;
    e = copy_convert<double, double>(Z, n, n, n, Vw, n, s);                        // V = Q
    if (e) return e;
    JAC_HIP(hipMemcpyAsync(&hflag, hd.flag, 4, hipMemcpyDeviceToHost, s));
    JAC_HIP(hipStreamSynchronize(s));
    if (hflag) { set_error("gesvd_jacobi: modified Gram-Schmidt met a zero column"); return 3; }
  }
  if (np > n) {
    hipLaunchKernelGGL(zero_cols_kernel, dim3(cdiv(m, 256), np - n), dim3(256), 0, s, C, m, m, n);
    JAC_CHECK_LAUNCH();
  }
  tm.mark(4);
  // Step 4: one-sided sweeps until a sweep applies fewer than 2e-4 N rotations
  // (Section 6 setup) or max_sweeps.  A pair is rotated only when its columns are
  // not yet orthogonal to m * tol relative accuracy.
  const double N = 0.5 * (double)n * (n - 1);
  const double rel = (double)m * tol;
  int sweeps = 0;
  long long rots = 0;
  double step_ms = 0;
  int info = 1;
  hipEvent_t ea = nullptr, eb = nullptr;
  if (stats) { JAC_HIP(hipEventCreate(&ea)); JAC_HIP(hipEventCreate(&eb)); }
  while (sweeps < max_sweeps) {
    JAC_HIP(hipMemsetAsync(hd.rot64, 0, 8, s));
    if (ea) JAC_HIP(hipEventRecord(ea, s));
    e = svd_sweep<double>(C, m, m, Vw, n, n, np, E, ident, Gp, gsplit, rel, kSvdInner, hd.rot64, s);
    if (e) return e;
    if (eb) JAC_HIP(hipEventRecord(eb, s));
    unsigned long long cnt = 0;
    JAC_HIP(hipMemcpyAsync(&cnt, hd.rot64, 8, hipMemcpyDeviceToHost, s));
    JAC_HIP(hipStreamSynchronize(s));
    if (ea) { float ms = 0; JAC_HIP(hipEventElapsedTime(&ms, ea, eb)); step_ms += ms; }
    ++sweeps;
    rots += (long long)cnt;
    if (stats && sweeps < JAC_HIST) stats->off_hist[sweeps] = (double)cnt;
    // A sweep that applies no rotation has converged (this also covers n <= 1, N = 0).
    if (cnt == 0 || (double)cnt < 2e-4 * N) { info = 0; break; }
  }
  if (ea) { (void)hipEventDestroy(ea); (void)hipEventDestroy(eb); }
  tm.mark(5);
  e = svd_finish(C, m, m, Vw, n, n, sig, rank, S, U, ldu, V, ldv, s);
  if (e) return e;
  tm.mark(6);
  JAC_HIP(hipStreamSynchronize(s));
  if (stats) {
    stats->sweeps = sweeps;
    stats->rotations = rots;
    stats->step_ms = step_ms;
    stats->step_launches = (long long)sweeps * (2 * npair - 1) * 4;
    stats->stage_ms[6] = tm.ms(0, 1);
    stats->stage_ms[0] = tm.ms(1, 2);
    stats->stage_ms[1] = tm.ms(2, 3);
    stats->stage_ms[2] = tm.ms(3, 4);
    stats->stage_ms[3] = tm.ms(4, 5);
    stats->stage_ms[4] = tm.ms(5, 6);
    stats->stage_ms[5] = tm.ms(0, 6);
  }
  return info;
}


// B (n x m) = A^T for an m x n block (32 x 32 tiles through LDS).
__global__ void transpose_rect_kernel(const double* __restrict__ A, int m, int n, int lda, double* __restrict__ B,
                                      int ldb) {
  __shared__ double t[32][33];
  const int bi = blockIdx.x * 32, bj = blockIdx.y * 32;   // rows / columns of A
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int r = ty; r < 32; r += 8) {
    const int i = bi + tx, j = bj + r;
    if (i < m && j < n) t[r][tx] = A[i + (size_t)j * lda];
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int j = bj + tx, i = bi + r;
    if (i < m && j < n) B[j + (size_t)i * ldb] = t[tx][r];
  }
}

static bool svd_qr_first(const jac_opts& o, int m, int n) {
  if (o.svd_qr == JAC_SVD_QR_ON) return true;
  if (o.svd_qr == JAC_SVD_QR_OFF) return false;
  // measured: 8192 x 512 37.6 vs 41.9 ms direct; at n <= 256 the two MGS passes cost more than
  // the shorter columns save (4096 x 256 13.4 vs 13.2 ms, 2048 x 128 5.0 vs 4.6 ms)
  return n >= 512 && m >= 8 * n && m <= kMgsFastRows;
}

// QR-first SVD (m >> n; the remark after Algorithm 5.2): A = Q_A B with Q_A from two passes of
// block MGS (orthonormal to working precision for any full-rank A with cond(A) < 1/u) and
// B = Q_A^T A; the SVD of the n x n B by gesvd_impl; U = Q_A U_B.  The outer buffers lie behind
// the inner call's part of the same grow-only workspace: the inner call asks for less than this
// call did, so it gets the same block back and carves only its own front part.
static int gesvd_qr_first(const double* A, int m, int n, int lda, double* S, double* U, int ldu, double* V, int ldv,
                          double tol, const jac_opts& o, jac_stats* stats, hipStream_t s) {
  if (m > kMgsMaxRows) { set_error("gesvd_jacobi_ex: the QR-first form needs m <= 32768"); return -2; }
  const size_t inner = align_up(gesvd_bytes(n, n, o.precond), 256);
  const size_t outer = 8192 + 2 * align_up((size_t)m * n * 8, 256) + 2 * align_up((size_t)n * n * 8, 256) +
                       align_up(mgs_scratch_elems(m, n) * 8, 256) + align_up((size_t)(n + 64) * 8, 256) +
                       align_up(1024 * 8, 256);
  void* ws = workspace(inner + outer);
  if (!ws) { set_error("gesvd_jacobi: workspace allocation failed"); return 4; }
  Carve c(static_cast<char*>(ws) + inner);
  int* flag = c.take<int>(16);
  double* Qa = c.take<double>((size_t)m * n);
  double* Qt = c.take<double>((size_t)m * n);
  double* B = c.take<double>((size_t)n * n);
  double* Ub = c.take<double>((size_t)n * n);
  double* mscr = c.take<double>(mgs_scratch_elems(m, n));
  hipEvent_t e0 = nullptr, e1 = nullptr, e2 = nullptr, e3 = nullptr;
  if (stats) {
    JAC_HIP(hipEventCreate(&e0)); JAC_HIP(hipEventCreate(&e1)); JAC_HIP(hipEventCreate(&e2)); JAC_HIP(hipEventCreate(&e3));
    JAC_HIP(hipEventRecord(e0, s));
  }
  JAC_HIP(hipMemsetAsync(flag, 0, 16 * sizeof(int), s));
  int e = check_finite(A, m, n, lda, flag, s);
  if (e) return e;
  int hflag = 0;
  JAC_HIP(hipMemcpyAsync(&hflag, flag, 4, hipMemcpyDeviceToHost, s));
  JAC_HIP(hipStreamSynchronize(s));
  if (hflag) { set_error("gesvd_jacobi: A contains NaN or Inf"); return 2; }
  e = copy_convert<double, double>(A, m, n, lda, Qa, m, s);
  if (e) return e;
  for (int pass = 0; pass < 2 && !e; ++pass) e = mgs_f64(Qa, m, n, m, mscr, flag, s);
  if (e) return e;
  hipLaunchKernelGGL(transpose_rect_kernel, dim3(cdiv(m, 32), cdiv(n, 32)), dim3(256), 0, s, (const double*)Qa, m, n,
                     m, Qt, n);
  JAC_CHECK_LAUNCH();
  e = gemm<double>(false, false, n, n, m, 1.0, Qt, n, A, lda, 0.0, B, n, s);   // B = Q_A^T A
  if (e) return e;
  JAC_HIP(hipMemcpyAsync(&hflag, flag, 4, hipMemcpyDeviceToHost, s));
  JAC_HIP(hipStreamSynchronize(s));
  if (hflag) { set_error("gesvd_jacobi: modified Gram-Schmidt met a zero column (rank-deficient A)"); return 3; }
  if (e1) JAC_HIP(hipEventRecord(e1, s));
  jac_opts oi = o;
  oi.svd_qr = JAC_SVD_QR_OFF;
  const int info = gesvd_impl(B, n, n, n, S, Ub, n, V, ldv, tol, &oi, stats, s);
  if (info != 0 && info != 1) return info;
  if (e2) JAC_HIP(hipEventRecord(e2, s));
  e = gemm<double>(false, false, m, n, n, 1.0, Qa, m, Ub, n, 0.0, U, ldu, s);   // U = Q_A U_B
  if (e) return e;
  if (e3) JAC_HIP(hipEventRecord(e3, s));
  JAC_HIP(hipStreamSynchronize(s));
  if (stats) {
    float a = 0, b = 0;
    JAC_HIP(hipEventElapsedTime(&a, e0, e1));
    JAC_HIP(hipEventElapsedTime(&b, e2, e3));
    stats->svd_qr_used = 1;
    stats->qr_ms = a + b;
    stats->stage_ms[5] += a + b;
    (void)hipEventDestroy(e0); (void)hipEventDestroy(e1); (void)hipEventDestroy(e2); (void)hipEventDestroy(e3);
  }
  return info;
}
}  // namespace jac

using namespace jac;

static hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

extern "C" {

const char* jac_last_error(void) { return last_error(); }
const char* jac_version(void) { return "libjacobi 0.1 (gfx950)"; }
void jac_release_workspace(void) { release_workspace(); }

size_t jac_workspace_bytes(int n, const jac_opts* opts) {
  if (n <= 0) return 0;
  int pre = opts ? opts->precond : 0;
  return syev_bytes(n, pre);
}

int jac_round_robin_pairs(int ne, int r, int* p, int* q) {
  if (ne < 2 || (ne & 1)) return -1;
  if (r < 0) return -2;
  if (!p) return -3;
  if (!q) return -4;
  RR rr(ne);
  for (int k = 0; k < rr.h; ++k) {
    int a = rr.index(k, r % (ne - 1)), b = rr.index(rr.h + k, r % (ne - 1));
    p[k] = a < b ? a : b;
    q[k] = a < b ? b : a;
  }
  return 0;
}

static int check_syev_args(const double* A, int n, int lda, double* W, double* V, int ldv, double tol) {
  g_err.clear();
  if (n < 0) { set_error("n < 0"); return -2; }
  if (lda < (n > 1 ? n : 1)) { set_error("lda < max(1,n)"); return -3; }
  if (n > 0 && !A) { set_error("A is NULL"); return -1; }
  if (n > 0 && !W) { set_error("W is NULL"); return -4; }
  if (n > 0 && !V) { set_error("V is NULL"); return -5; }
  if (ldv < (n > 1 ? n : 1)) { set_error("ldv < max(1,n)"); return -6; }
  if (tol != tol) { set_error("tol is NaN"); return -7; }
  return 0;
}

int syev_jacobi_ex(const double* A, int n, int lda, double* W, double* V, int ldv, double tol,
                   const jac_opts* opts, jac_stats* stats, void* stream) {
  int e = check_syev_args(A, n, lda, W, V, ldv, tol);
  if (e) return e;
  return syev_impl(A, n, lda, nullptr, 0, W, V, ldv, tol, opts, stats, as_stream(stream));
}

int syev_jacobi(const double* A, int n, int lda, double* W, double* V, double tol, int* sweeps_out) {
  jac_opts o{};
  o.precond = JAC_PRECOND_FP32;
  jac_stats st;
  int e = check_syev_args(A, n, lda, W, V, n > 1 ? n : 1, tol);
  if (e) return e;
  e = syev_impl(A, n, lda, nullptr, 0, W, V, n > 1 ? n : 1, tol, &o, &st, nullptr);
  if (sweeps_out) *sweeps_out = st.sweeps;
  return e;
}

}  // extern "C"

// Fixed device array of the allocation-free entry point.  In host code `scratch` names a host-side
// stand-in: its device address (one copy per device) comes from hipGetSymbolAddress, taken once per
// device with that device current, and only that address is handed to kernels and copies.
static __device__ __align__(256) unsigned char scratch[JAC_NOALLOC_BYTES];
static void* g_scratch_addr[256];
static std::mutex g_scratch_mu;

static int scratch_address(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 256) {
    set_error("syev_jacobi_noalloc: no current device");
    return 4;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* p = nullptr;
    hipError_t rc = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (rc != hipSuccess || !p) {
      set_error(std::string("syev_jacobi_noalloc: hipGetSymbolAddress failed: ") + hipGetErrorString(rc));
      return 4;
    }
    g_scratch_addr[dev] = p;
  }
  *out = g_scratch_addr[dev];
  return 0;
}

extern "C" {

int syev_jacobi_noalloc(const double* A, int n, int lda, double* W, double* V, int ldv, double tol,
                        const jac_opts* opts, jac_stats* stats, void* stream) {
  int e = check_syev_args(A, n, lda, W, V, ldv, tol);
  if (e) return e;
  if (opts && opts->precond != JAC_PRECOND_NONE && opts->precond != JAC_PRECOND_FP32) {
    set_error("syev_jacobi_noalloc: only the plain and FP32-preconditioned starts are available");
    return -8;
  }
  if (n == 0) {
    if (stats) std::memset(stats, 0, sizeof(*stats));
    return 0;
  }
  void* ws = nullptr;
  e = scratch_address(&ws);
  if (e) return e;
  return syev_impl(A, n, lda, nullptr, 0, W, V, ldv, tol, opts, stats, as_stream(stream), ws, JAC_NOALLOC_BYTES);
}

int syev_jacobi_warm(const double* A, int n, int lda, const double* Q0, int ldq, double* W, double* V, int ldv,
                     double tol, const jac_opts* opts, jac_stats* stats, void* stream) {
  g_err.clear();
  if (n < 0) { set_error("n < 0"); return -2; }
  if (lda < (n > 1 ? n : 1)) { set_error("lda < max(1,n)"); return -3; }
  if (n > 0 && !A) { set_error("A is NULL"); return -1; }
  if (n > 0 && !Q0) { set_error("Q0 is NULL"); return -4; }
  if (ldq < (n > 1 ? n : 1)) { set_error("ldq < max(1,n)"); return -5; }
  if (n > 0 && !W) { set_error("W is NULL"); return -6; }
  if (n > 0 && !V) { set_error("V is NULL"); return -7; }
  if (ldv < (n > 1 ? n : 1)) { set_error("ldv < max(1,n)"); return -8; }
  if (tol != tol) { set_error("tol is NaN"); return -9; }
  return syev_impl(A, n, lda, Q0, ldq, W, V, ldv, tol, opts, stats, as_stream(stream));
}

static int check_svd_args(const double* A, int m, int n, int lda, double* S, double* U, int ldu, double* V, int ldv,
                          double tol) {
  g_err.clear();
  if (n > 0 && !A) { set_error("A is NULL"); return -1; }
  if (m < 0) { set_error("m < 0"); return -2; }
  if (n < 0 || n > m) { set_error("need 0 <= n <= m"); return -3; }
  if (lda < (m > 1 ? m : 1)) { set_error("lda < max(1,m)"); return -4; }
  if (n > 0 && !S) { set_error("S is NULL"); return -5; }
  if (n > 0 && !U) { set_error("U is NULL"); return -6; }
  if (ldu < (m > 1 ? m : 1)) { set_error("ldu < max(1,m)"); return -7; }
  if (n > 0 && !V) { set_error("V is NULL"); return -8; }
  if (ldv < (n > 1 ? n : 1)) { set_error("ldv < max(1,n)"); return -9; }
  if (tol != tol) { set_error("tol is NaN"); return -10; }
  return 0;
}

int gesvd_jacobi(const double* A, int m, int n, int lda, double* S, double* U, int ldu, double* V, int ldv,
                 double tol, int* sweeps_out) {
  int e = check_svd_args(A, m, n, lda, S, U, ldu, V, ldv, tol);
  if (e) return e;
  jac_opts o{};
  o.precond = JAC_PRECOND_FP32;
  jac_stats st;
  e = svd_qr_first(o, m, n) ? gesvd_qr_first(A, m, n, lda, S, U, ldu, V, ldv, tol, o, &st, nullptr)
                            : gesvd_impl(A, m, n, lda, S, U, ldu, V, ldv, tol, &o, &st, nullptr);
  if (sweeps_out) *sweeps_out = st.sweeps;
  return e;
}

int gesvd_jacobi_ex(const double* A, int m, int n, int lda, double* S, double* U, int ldu, double* V, int ldv,
                    double tol, const jac_opts* opts, jac_stats* stats, void* stream) {
  int e = check_svd_args(A, m, n, lda, S, U, ldu, V, ldv, tol);
  if (e) return e;
  jac_opts o{};
  if (opts) o = *opts;
  if (o.svd_qr < JAC_SVD_QR_AUTO || o.svd_qr > JAC_SVD_QR_ON) {
    set_error("gesvd_jacobi_ex: opts.svd_qr must be a jac_svd_qr_t");
    return -11;
  }
  if (svd_qr_first(o, m, n)) {
    if (stats) std::memset(stats, 0, sizeof(*stats));
    return gesvd_qr_first(A, m, n, lda, S, U, ldu, V, ldv, tol, o, stats, as_stream(stream));
  }
  return gesvd_impl(A, m, n, lda, S, U, ldu, V, ldv, tol, &o, stats, as_stream(stream));
}

int jac_parallel_steps(double* T, int n, int ldt, double* V, int ldv, int r0, int nsteps, double skip_abs,
                       long long* rotations, void* stream) {
  g_err.clear();
  if (!T && n > 0) { set_error("T is NULL"); return -1; }
  if (n < 0) { set_error("n < 0"); return -2; }
  if (ldt < (n > 1 ? n : 1)) { set_error("ldt < max(1,n)"); return -3; }
  if (V && ldv < (n > 1 ? n : 1)) { set_error("ldv < max(1,n)"); return -5; }
  if (r0 < 0) { set_error("r0 < 0"); return -6; }
  if (nsteps < 0) { set_error("nsteps < 0"); return -7; }
  if (!(skip_abs >= 0)) { set_error("skip_abs must be >= 0"); return -8; }
  if (rotations) *rotations = 0;
  if (n < 2 || nsteps == 0) return 0;
  if ((long long)nsteps > (long long)(kRotSlots - 4) * (n + (n & 1) - 1)) {
    set_error("nsteps too large for one call");
    return -7;
  }
  hipStream_t s = as_stream(stream);
  size_t need = 4096 + 1024 * 8 + 2 * kRotSlots * 8 + elem_bytes<double>(n) + 64 * 256 +
                (V ? 0 : align_up((size_t)n * n * 8, 256));
  void* ws = workspace(need);
  if (!ws) { set_error("workspace allocation failed"); return 4; }
  Carve c(ws);
  Head hd = carve_head(c, n);
  ElemState<double> st;
  carve_elem(c, st, n);
  double* Vd = V;
  int ldvd = ldv;
  if (!V) {
    Vd = c.take<double>((size_t)n * n);
    ldvd = n;
    int e = set_identity<double>(Vd, n, n, s);
    if (e) return e;
  }
  st.V = Vd;
  st.ldv = ldvd;
  st.partial = hd.partial;
  st.scalars = hd.scal;
  st.rot = hd.rot64;
  st.skip_abs = skip_abs;
  const int per = st.ne - 1;
  const int r = r0 % per;
  JAC_HIP(hipMemsetAsync(st.rot, 0, kRotSlots * 8, s));
  int e = elem_pack<double>(st, T, ldt, r, s);
  if (e) return e;
  e = elem_init_angles<double>(st, r, s);
  if (e) return e;
  // Global step numbering starts at r, so the counters of the first sweep
  // hold every step of this call as long as nsteps < kRotSlots * per.
  e = elem_steps<double>(st, r, nsteps, s);
  if (e) return e;
  e = elem_unpack_dense<double>(st, (int)((r + (long long)nsteps) % per), T, ldt, s);
  if (e) return e;
  if (rotations) {
    std::vector<unsigned long long> cnt(kRotSlots);
    JAC_HIP(hipMemcpyAsync(cnt.data(), st.rot, kRotSlots * 8, hipMemcpyDeviceToHost, s));
    JAC_HIP(hipStreamSynchronize(s));
    // Count only the steps that were applied: angles of the step after the
    // last one were computed but not used.
    long long last = (long long)r + nsteps;  // global index of the unused step
    long long tot = 0;
    for (int i = 0; i < kRotSlots; ++i) tot += (long long)cnt[i];
    // Recompute the unused step's count by running its angle kernel alone.
    JAC_HIP(hipMemsetAsync(st.rot, 0, 8, s));
    e = elem_init_angles<double>(st, (int)(last % per), s);
    if (e) return e;
    unsigned long long extra = 0;
    JAC_HIP(hipMemcpyAsync(&extra, st.rot, 8, hipMemcpyDeviceToHost, s));
    JAC_HIP(hipStreamSynchronize(s));
    *rotations = tot - (long long)extra;
  }
  JAC_HIP(hipStreamSynchronize(s));
  return 0;
}

int jac_mgs(double* Q, int m, int n, int ldq, void* stream) {
  g_err.clear();
  if (!Q && m > 0 && n > 0) { set_error("Q is NULL"); return -1; }
  if (m < 0) { set_error("m < 0"); return -2; }
  if (n < 0 || n > m) { set_error("need 0 <= n <= m"); return -3; }
  if (ldq < (m > 1 ? m : 1)) { set_error("ldq < max(1,m)"); return -4; }
  if (m > kMgsMaxRows) { set_error("m > 32768 is not supported"); return -2; }
  if (n == 0) return 0;
  hipStream_t s = as_stream(stream);
  void* ws = workspace(align_up(mgs_scratch_elems(m, n) * 8, 256) + 4096);
  if (!ws) { set_error("workspace allocation failed"); return 4; }
  Carve c(ws);
  int* flag = c.take<int>(16);
  double* scr = c.take<double>(mgs_scratch_elems(m, n));
  JAC_HIP(hipMemsetAsync(flag, 0, 64, s));
  int e = mgs_f64(Q, m, n, ldq, scr, flag, s);
  if (e) return e;
  int hf = 0;
  JAC_HIP(hipMemcpyAsync(&hf, flag, 4, hipMemcpyDeviceToHost, s));
  JAC_HIP(hipStreamSynchronize(s));
  if (hf) { set_error("modified Gram-Schmidt met a zero column"); return 3; }
  return 0;
}

int jac_qr_orth(double* Q, int n, int ldq, int* method, void* stream) {
  g_err.clear();
  if (!Q && n > 0) { set_error("Q is NULL"); return -1; }
  if (n < 0 || n > kMgsMaxRows) { set_error("need 0 <= n <= 32768"); return -2; }
  if (ldq < (n > 1 ? n : 1)) { set_error("ldq < max(1,n)"); return -3; }
  if (method) *method = 0;
  if (n == 0) return 0;
  hipStream_t s = as_stream(stream);
  void* ws = workspace(4 * align_up((size_t)n * n * 8, 256) + align_up((size_t)(2 * n + 64) * 8, 256) +
                       align_up(mgs_scratch_elems(n, n) * 8, 256) + 8192);
  if (!ws) { set_error("workspace allocation failed"); return 4; }
  Carve c(ws);
  int* flag = c.take<int>(16);
  double* scal = c.take<double>(8);
  double* B[4];
  for (int i = 0; i < 4; ++i) B[i] = c.take<double>((size_t)n * n);
  double* part = c.take<double>((size_t)2 * n + 64);
  double* mscr = c.take<double>(mgs_scratch_elems(n, n));
  JAC_HIP(hipMemsetAsync(flag, 0, 64, s));
  int used = 0;
  int e = orth_series_f64(Q, n, ldq, B[0], B[1], B[2], B[3], part, scal, &used, s, false);
  if (e) return e;
  if (!used) {
    e = mgs_f64(Q, n, n, ldq, mscr, flag, s);
    if (e) return e;
  }
  int hf = 0;
  JAC_HIP(hipMemcpyAsync(&hf, flag, 4, hipMemcpyDeviceToHost, s));
  JAC_HIP(hipStreamSynchronize(s));
  if (method) *method = used ? 1 : 2;
  if (hf) { set_error("modified Gram-Schmidt met a zero column"); return 3; }
  return 0;
}

int jac_similarity(const double* A, int n, int lda, const double* Q, int ldq, double* T, int ldt, void* stream) {
  g_err.clear();
  if (!A && n > 0) { set_error("A is NULL"); return -1; }
  if (n < 0) { set_error("n < 0"); return -2; }
  if (lda < (n > 1 ? n : 1)) { set_error("lda < max(1,n)"); return -3; }
  if (!Q && n > 0) { set_error("Q is NULL"); return -4; }
  if (ldq < (n > 1 ? n : 1)) { set_error("ldq < max(1,n)"); return -5; }
  if (!T && n > 0) { set_error("T is NULL"); return -6; }
  if (ldt < (n > 1 ? n : 1)) { set_error("ldt < max(1,n)"); return -7; }
  if (n == 0) return 0;
  hipStream_t s = as_stream(stream);
  void* ws = workspace(align_up((size_t)n * n * 8, 256) + 4096);
  if (!ws) { set_error("workspace allocation failed"); return 4; }
  Carve c(ws);
  double* W = c.take<double>((size_t)n * n);
  int e = similarity(A, n, lda, Q, ldq, T, ldt, W, s);
  if (e) return e;
  JAC_HIP(hipStreamSynchronize(s));
  return 0;
}

int jac_eig_fp32(const double* A, int n, int lda, double* Z, int ldz, double* W, double tol, int max_sweeps,
                 int* sweeps, void* stream) {
  g_err.clear();
  if (!A && n > 0) { set_error("A is NULL"); return -1; }
  if (n < 0) { set_error("n < 0"); return -2; }
  if (lda < (n > 1 ? n : 1)) { set_error("lda < max(1,n)"); return -3; }
  if (!Z && n > 0) { set_error("Z is NULL"); return -4; }
  if (ldz < (n > 1 ? n : 1)) { set_error("ldz < max(1,n)"); return -5; }
  if (tol != tol) { set_error("tol is NaN"); return -7; }
  if (sweeps) *sweeps = 0;
  if (n == 0) return 0;
  hipStream_t s = as_stream(stream);
  size_t need = syev_bytes(n, 1) + align_up((size_t)n * n * 8, 256) + align_up((size_t)n * 8, 256);
  void* ws = workspace(need);
  if (!ws) { set_error("workspace allocation failed"); return 4; }
  Carve c(ws);
  Head hd = carve_head(c, n);
  double* Zw = c.take<double>((size_t)n * n);
  float* d32 = c.take<float>(n);
  int* rank = c.take<int>(n);
  int e = fro2_f64(A, n, n, lda, hd.partial, hd.scal + 1, s);
  if (e) return e;
  double f2 = 0;
  JAC_HIP(hipMemcpyAsync(&f2, hd.scal + 1, 8, hipMemcpyDeviceToHost, s));
  JAC_HIP(hipStreamSynchronize(s));
  int sw = 0;
  long long rots = 0;
  e = fp32_stage(A, true, n, lda, std::sqrt(f2), tol > 0 ? tol : 1e-6, max_sweeps > 0 ? max_sweeps : 30, Zw, n, d32,
                 c, hd, s, &sw, &rots);
  if (e) return e;
  if (W) {
    // Z's columns in ascending order of the FP32 eigenvalues.
    double* d64 = c.take<double>(n);
    e = copy_convert<float, double>(d32, n, 1, n, d64, n, s);
    if (e) return e;
    e = sort_eigs<double>(d64, Zw, n, n, W, Z, ldz, rank, s);
    if (e) return e;
  } else {
    e = copy_convert<double, double>(Zw, n, n, n, Z, ldz, s);
    if (e) return e;
  }
  JAC_HIP(hipStreamSynchronize(s));
  if (sweeps) *sweeps = sw;
  return 0;
}

int jac_sytrd_f32(const double* A, int n, int lda, double* d, double* e, float* tau, float* U, int ldu, void* stream) {
  g_err.clear();
  if (!A && n > 0) { set_error("A is NULL"); return -1; }
  if (n < 0 || n > 8192) { set_error("need 0 <= n <= 8192"); return -2; }
  if (lda < (n > 1 ? n : 1)) { set_error("lda < max(1,n)"); return -3; }
  if (!d && n > 0) { set_error("d is NULL"); return -4; }
  if (!e && n > 1) { set_error("e is NULL"); return -5; }
  if (!tau && n > 2) { set_error("tau is NULL"); return -6; }
  if (!U && n > 2) { set_error("U is NULL"); return -7; }
  if (ldu < (n > 1 ? n : 1)) { set_error("ldu < max(1,n)"); return -8; }
  if (n == 0) return 0;
  return tridiag_reduce_entry(A, n, lda, d, e, tau, U, ldu, as_stream(stream));
}

int jac_tridiag_eig(const double* d, const double* e, int n, double* w, double* Z, int ldz, void* stream) {
  g_err.clear();
  if (!d && n > 0) { set_error("d is NULL"); return -1; }
  if (!e && n > 1) { set_error("e is NULL"); return -2; }
  if (n < 0) { set_error("n < 0"); return -3; }
  if (!w && n > 0) { set_error("w is NULL"); return -4; }
  if (Z && ldz < (n > 1 ? n : 1)) { set_error("ldz < max(1,n)"); return -6; }
  if (n == 0) return 0;
  return tridiag_eig_entry(d, e, n, w, Z, ldz, as_stream(stream));
}

int jac_tridiag_backtransform(const float* U, int ldu, const float* tau, int n, double* Y, int ldy, void* stream) {
  g_err.clear();
  if (!U && n > 2) { set_error("U is NULL"); return -1; }
  if (ldu < (n > 1 ? n : 1)) { set_error("ldu < max(1,n)"); return -2; }
  if (!tau && n > 2) { set_error("tau is NULL"); return -3; }
  if (n < 0 || n > 8192) { set_error("need 0 <= n <= 8192"); return -4; }
  if (!Y && n > 0) { set_error("Y is NULL"); return -5; }
  if (ldy < (n > 1 ? n : 1)) { set_error("ldy < max(1,n)"); return -6; }
  if (n == 0) return 0;
  return tridiag_backtransform_entry(U, ldu, tau, n, Y, ldy, as_stream(stream));
}

int jac_eig_fp32_tridiag(const double* A, int n, int lda, double* Z, int ldz, double* W, void* stream) {
  g_err.clear();
  if (!A && n > 0) { set_error("A is NULL"); return -1; }
  if (n < 0 || n > 8192) { set_error("need 0 <= n <= 8192"); return -2; }
  if (lda < (n > 1 ? n : 1)) { set_error("lda < max(1,n)"); return -3; }
  if (!Z && n > 0) { set_error("Z is NULL"); return -4; }
  if (ldz < (n > 1 ? n : 1)) { set_error("ldz < max(1,n)"); return -5; }
  if (n == 0) return 0;
  hipStream_t s = as_stream(stream);
  void* ws = workspace(tridiag_bytes(n) + 4096);
  if (!ws) { set_error("workspace allocation failed"); return 4; }
  Carve c(ws);
  int e = eig_tridiag_f32<double>(A, n, lda, Z, ldz, W, c, s, false);
  if (e) return e;
  JAC_HIP(hipStreamSynchronize(s));
  return 0;
}

int jac_gemm_f64(int ta, int tb, int m, int n, int k, double alpha, const double* A, int lda, const double* B,
                 int ldb, double beta, double* C, int ldc, void* stream) {
  g_err.clear();
  if (m < 0 || n < 0 || k < 0) { set_error("negative size"); return -3; }
  int e = gemm<double>(ta != 0, tb != 0, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, as_stream(stream));
  if (e) return e;
  JAC_HIP(hipStreamSynchronize(as_stream(stream)));
  return 0;
}

int jac_gemm_f32(int ta, int tb, int m, int n, int k, float alpha, const float* A, int lda, const float* B,
                 int ldb, float beta, float* C, int ldc, void* stream) {
  g_err.clear();
  if (m < 0 || n < 0 || k < 0) { set_error("negative size"); return -3; }
  int e = gemm<float>(ta != 0, tb != 0, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, as_stream(stream));
  if (e) return e;
  JAC_HIP(hipStreamSynchronize(as_stream(stream)));
  return 0;
}

}  // extern "C"
