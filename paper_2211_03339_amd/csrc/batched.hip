// Batched path: thousands of independent symmetric eigenproblems of uneven
// order (n <= 512) in one graph launch plus a convergence check.
//
// Matrices are grouped by padded order np (a multiple of 64).  Each size class
// is stored back to back (T and V of np x np each; the padding of T is zero and
// that of V the identity, which no rotation ever touches) and advances through
// the block steps of the blocked Jacobi method in lockstep: every launch covers
// all matrices of the class (grid y = matrix).  Every matrix carries a
// convergence flag, set by the check after each sweep (the sweep at which
// ||off(T)||_F <= tol ||A||_F first held); the sweep kernels leave a flagged
// matrix alone, so a matrix stops exactly where it converged -- its result does
// not depend on the other matrices of the batch nor on how many sweeps its
// class runs.
//
// One call: a captured graph (cached, replayed while sizes, pointers and tuned
// values stay the same) holds the set-up, the optional preconditioning
// (Algorithm 4.1 steps 1-3 per matrix: FP32 blocked Jacobi sweeps on fl32(A)
// truncated at fp32_tol ||A||_F, the QR factor of the FP32 eigenvectors by the
// batched series passes of orth.hip, T0 = Q^T A Q by batched GEMMs) and each
// class's tuned number of FP64 sweeps.  The host then reads the flags; a class
// with unconverged matrices gets further sweeps (eager launches, checked after
// each) up to max_sweeps, and a last launch writes W ascending and V.  The
// graph is captured on a single stream: no forked branches, so no streams or
// events beyond the one capture stream.
//
// The sweep counts and the inner-sweep cap of each size class come from an
// autotuner (jac_autotune_batched*) that runs sample matrices of the class
// with every cap and keeps the fastest configuration, with the sweeps its
// samples needed; its table can be cached in the text file named by
// JACOBI_TUNE_CACHE.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "../../include/jacobi.h"
#include "common.h"

namespace jac {

struct TuneEntry { int inner, sweeps, sweeps32; };
static std::map<std::pair<int, int>, TuneEntry> g_tune;   // (np, precond) -> entry
static bool g_tune_loaded = false;
static std::mutex g_tune_mu;
constexpr int kMaxBatchN = 512, kMaxBatch = 65535;
constexpr int kDefaultInner = 2, kDefaultSweeps = 12, kDefaultSweepsPre = 4, kDefaultSweeps32 = 10;
constexpr int kDefaultMaxSweeps = 60;
constexpr double kDefaultFp32Tol = 1e-4;

static void load_tune_locked() {
  g_tune_loaded = true;
  const char* p = std::getenv("JACOBI_TUNE_CACHE");
  if (!p) return;
  std::ifstream f(p);
  int np, pre, inner, sweeps, sweeps32;
  while (f >> np >> pre >> inner >> sweeps >> sweeps32)
    if (np > 0 && inner > 0 && sweeps > 0 && sweeps32 >= 0) g_tune[{np, pre ? 1 : 0}] = {inner, sweeps, sweeps32};
}

static void save_tune_locked() {
  const char* p = std::getenv("JACOBI_TUNE_CACHE");
  if (!p) return;
  std::ofstream f(p);
  for (auto& kv : g_tune)
    f << kv.first.first << " " << kv.first.second << " " << kv.second.inner << " " << kv.second.sweeps << " "
      << kv.second.sweeps32 << "\n";
}

static TuneEntry tune_for(int np, int pre) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  if (!g_tune_loaded) load_tune_locked();
  auto it = g_tune.find({np, pre});
  if (it != g_tune.end()) return it->second;
  return pre ? TuneEntry{kDefaultInner, kDefaultSweepsPre, kDefaultSweeps32}
             : TuneEntry{kDefaultInner, kDefaultSweeps, 0};
}

static inline size_t al(size_t x) { return (x + 255) / 256 * 256; }
static inline int bcdiv(long long a, long long b) { return (int)((a + b - 1) / b); }

// ---------------------------------------------------------------- kernels
// T <- [A 0; 0 0] and V <- I (np x np each), rotation counter cleared.  grid (x, matrix).
__global__ void bat_load_kernel(const BDesc<double>* __restrict__ desc, const double* const* __restrict__ A,
                                const int* __restrict__ lda) {
  const BDesc<double> d = desc[blockIdx.y];
  const double* a = A[blockIdx.y];
  const int la = lda[blockIdx.y], np = d.ldt;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < (long long)np * np;
       e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e % np), j = (int)(e / np);
    d.Tm[e] = (i < d.n && j < d.n) ? a[i + (size_t)j * la] : 0.0;
    d.V[i + (size_t)j * d.ldv] = i == j ? 1.0 : 0.0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) *d.rot = 0;
}

// FP32 stage set-up: T32 <- fl32(T64) (= [A 0; 0 0]), V32 <- I.
__global__ void bat_load32_kernel(const BDesc<float>* __restrict__ d32, const BDesc<double>* __restrict__ d64) {
  const BDesc<float> d = d32[blockIdx.y];
  const double* t = d64[blockIdx.y].Tm;
  const int np = d.ldt;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < (long long)np * np;
       e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e % np), j = (int)(e / np);
    d.Tm[e] = (float)t[e];
    d.V[i + (size_t)j * d.ldv] = i == j ? 1.0f : 0.0f;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) *d.rot = 0;
}

// ||A||_F^2 from T = [A 0; 0 0] (one workgroup per matrix, fixed order).
__global__ __launch_bounds__(256) void bat_norm_kernel(const BDesc<double>* __restrict__ desc) {
  __shared__ double red[256];
  const BDesc<double> d = desc[blockIdx.x];
  const int np = d.ldt;
  double acc = 0.0;
  for (long long e = threadIdx.x; e < (long long)np * np; e += 256) acc += d.Tm[e] * d.Tm[e];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *const_cast<double*>(d.nrm2) = red[0];
}

// The stop test after `sweep` sweeps (sweep 0: of the start, which also resets the flag):
// conv = sweep when ||off(T)||_F <= tol ||A||_F first holds.  One workgroup per matrix.
template <typename T>
__global__ __launch_bounds__(256) void bat_check_kernel(const BDesc<T>* __restrict__ desc, int sweep, double tol) {
  __shared__ double red[256];
  const BDesc<T> d = desc[blockIdx.x];
  int* conv = const_cast<int*>(d.conv);
  if (sweep > 0 && *conv >= 0) return;
  const int np = d.ldt;
  double acc = 0.0;
  for (long long e = threadIdx.x; e < (long long)np * np; e += 256) {
    const int i = (int)(e % np), j = (int)(e / np);
    const double v = (double)d.Tm[e];
    if (i != j) acc += v * v;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *conv = sqrt(red[0]) <= tol * sqrt(*d.nrm2) ? sweep : -1;
}

// V64 <- V32 (the FP32 eigenvectors, padding included).
__global__ void bat_convert_kernel(const BDesc<float>* __restrict__ d32, const BDesc<double>* __restrict__ d64) {
  const float* v = d32[blockIdx.y].V;
  double* w = d64[blockIdx.y].V;
  const int np = d64[blockIdx.y].ldt;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < (long long)np * np;
       e += (long long)gridDim.x * blockDim.x)
    w[e] = (double)v[e];
}

// A start the series could not orthogonalise (state 3) is replaced by the plain start V = I.
__global__ void bat_restart_kernel(const BDesc<double>* __restrict__ desc, const int* __restrict__ state) {
  if (state[blockIdx.y] != 3) return;
  const BDesc<double> d = desc[blockIdx.y];
  const int np = d.ldt;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < (long long)np * np;
       e += (long long)gridDim.x * blockDim.x)
    d.V[e] = (e % np) == (e / np) ? 1.0 : 0.0;
}

// B_z = A_z^T for matrices stored back to back (np x np, 32 x 32 tiles through LDS).
__global__ void bat_transpose_kernel(const double* __restrict__ A, int np, double* __restrict__ B) {
  __shared__ double tl[32][33];
  const size_t off = (size_t)blockIdx.z * np * np;
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int r = ty; r < 32; r += 8) {
    const int i = bx + tx, j = by + r;
    if (i < np && j < np) tl[r][tx] = A[off + i + (size_t)j * np];
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int i = by + tx, j = bx + r;
    if (i < np && j < np) B[off + i + (size_t)j * np] = tl[tx][r];
  }
}

// T <- its upper triangle mirrored (T0 = Q^T A Q is symmetric in exact arithmetic).
__global__ void bat_mirror_kernel(double* __restrict__ T, int np) {
  const size_t off = (size_t)blockIdx.y * np * np;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < (long long)np * np;
       e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e % np), j = (int)(e / np);
    if (i > j) T[off + e] = T[off + j + (size_t)i * np];
  }
}

// Per matrix: W ascending with V's columns permuted alike; sweeps (the flag, or max_sweeps when the
// matrix did not converge), info (0 converged / 1 not) and the FP32 sweeps (the FP32 flag, or the
// class's FP32 sweep count when the FP32 stop was not reached).
__global__ void bat_finish_kernel(const BDesc<double>* __restrict__ desc, double* const* __restrict__ W,
                                  double* const* __restrict__ V, const int* __restrict__ ldv,
                                  const int* __restrict__ orig, const int* __restrict__ conv32, int max_sweeps,
                                  int* __restrict__ sweeps_out, int* __restrict__ info, int* __restrict__ sweeps32_out) {
  __shared__ int rank[kMaxBatchN];
  const BDesc<double> d = desc[blockIdx.x];
  const int n = d.n;
  double* w = W[blockIdx.x];
  double* v = V[blockIdx.x];
  const int lv = ldv[blockIdx.x];
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double di = d.Tm[i + (size_t)i * d.ldt];
    int rk = 0;
    for (int j = 0; j < n; ++j) {
      const double dj = d.Tm[j + (size_t)j * d.ldt];
      rk += (dj < di) || (dj == di && j < i);
    }
    rank[i] = rk;
    w[rk] = di;
  }
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    const int rk = rank[j];
    for (int row = threadIdx.x; row < n; row += blockDim.x) v[row + (size_t)rk * lv] = d.V[row + (size_t)j * d.ldv];
  }
  if (threadIdx.x == 0) {
    const int c = *d.conv, o = orig[blockIdx.x];
    if (info) info[o] = c < 0 ? 1 : 0;
    if (sweeps_out) sweeps_out[o] = c < 0 ? max_sweeps : c;
    if (sweeps32_out) sweeps32_out[o] = d.s32 == 0 ? 0 : (conv32[blockIdx.x] < 0 ? d.s32 : conv32[blockIdx.x]);
  }
}

// ---------------------------------------------------------------- plan
struct Cls {
  int np, off, cnt, maxn, inner, sweeps, sweeps32;
  double* T;   // cnt np x np, back to back
  double* V;
};

struct Plan {
  std::vector<uintptr_t> key;
  int batch = 0, pre = 0;
  double tol = 0, tol32 = 0;
  std::vector<Cls> cls;
  void* mem = nullptr;
  BDesc<double>* d_desc = nullptr;
  BDesc<float>* d_desc32 = nullptr;
  int *d_conv = nullptr, *d_conv32 = nullptr, *d_state = nullptr, *d_orig = nullptr, *d_ldv = nullptr;
  double* d_e2 = nullptr;
  double* const* d_W = nullptr;
  double* const* d_V = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<int> h_conv;
  ~Plan() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (mem) (void)hipFree(mem);
  }
};
static Plan* g_plan = nullptr;
static std::mutex g_plan_mu;

// The library's capture stream of the current device (created once, kept for the process).
static hipStream_t capture_stream() {
  static std::mutex mu;
  static std::map<int, hipStream_t> streams;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lk(mu);
  auto it = streams.find(dev);
  if (it != streams.end()) return it->second;
  hipStream_t s = nullptr;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return nullptr;
  streams[dev] = s;
  return s;
}

// One sweep of class C followed by its stop test after `sweep` sweeps.
static int class_sweep(const Plan& P, const Cls& C, int sweep, hipStream_t s) {
  int e = blk_sweep_batched<double>(P.d_desc + C.off, C.cnt, C.np, C.maxn, C.inner, s);
  if (e) return e;
  hipLaunchKernelGGL((bat_check_kernel<double>), dim3(C.cnt), dim3(256), 0, s,
                     (const BDesc<double>*)(P.d_desc + C.off), sweep, P.tol);
  JAC_CHECK_LAUNCH();
  return 0;
}

// The graph's work: set-up, per class the optional preconditioning and the tuned FP64 sweeps.
static int record_solve(const Plan& P, const double* const* d_A, const int* d_lda, double* S[4], hipStream_t s) {
  const int maxnp = P.cls.front().np;
  int gx = bcdiv((long long)maxnp * maxnp, 256);
  if (gx > 64) gx = 64;
  hipLaunchKernelGGL(bat_load_kernel, dim3(gx, P.batch), dim3(256), 0, s, (const BDesc<double>*)P.d_desc, d_A, d_lda);
  JAC_CHECK_LAUNCH();
  hipLaunchKernelGGL(bat_norm_kernel, dim3(P.batch), dim3(256), 0, s, (const BDesc<double>*)P.d_desc);
  JAC_CHECK_LAUNCH();
  for (const Cls& C : P.cls) {
    const BDesc<double>* dd = P.d_desc + C.off;
    int cx = bcdiv((long long)C.np * C.np, 256);
    if (cx > 64) cx = 64;
    const long long st = (long long)C.np * C.np;
    if (P.pre) {
      // Step 1: FP32 blocked Jacobi on fl32(A), truncated at tol32 ||A||_F.
      const BDesc<float>* d3 = P.d_desc32 + C.off;
      hipLaunchKernelGGL(bat_load32_kernel, dim3(cx, C.cnt), dim3(256), 0, s, d3, dd);
      JAC_CHECK_LAUNCH();
      hipLaunchKernelGGL((bat_check_kernel<float>), dim3(C.cnt), dim3(256), 0, s, d3, 0, P.tol32);
      JAC_CHECK_LAUNCH();
      for (int sw = 1; sw <= C.sweeps32; ++sw) {
        int e = blk_sweep_batched<float>(d3, C.cnt, C.np, C.maxn, C.inner, s);
        if (e) return e;
        hipLaunchKernelGGL((bat_check_kernel<float>), dim3(C.cnt), dim3(256), 0, s, d3, sw, P.tol32);
        JAC_CHECK_LAUNCH();
      }
      // Step 2: Q = the QR factor of the FP32 eigenvectors (series passes; plain start on failure).
      hipLaunchKernelGGL(bat_convert_kernel, dim3(cx, C.cnt), dim3(256), 0, s, d3, dd);
      JAC_CHECK_LAUNCH();
      int e = orth_series_batched(C.V, C.np, C.cnt, S[0], S[1], S[2], S[3], P.d_state + C.off, P.d_e2 + C.off, s);
      if (e) return e;
      hipLaunchKernelGGL(bat_restart_kernel, dim3(cx, C.cnt), dim3(256), 0, s, dd,
                         (const int*)(P.d_state + C.off));
      JAC_CHECK_LAUNCH();
      // Step 3: T0 = Q^T A Q as untransposed GEMMs (S1 = Q^T, S2 = Q^T A, T = S2 Q), mirrored.
      hipLaunchKernelGGL(bat_transpose_kernel, dim3(bcdiv(C.np, 32), bcdiv(C.np, 32), C.cnt), dim3(256), 0, s,
                         (const double*)C.V, C.np, S[0]);
      JAC_CHECK_LAUNCH();
      e = gemm_batched<double>(false, false, C.np, C.np, C.np, 1.0, S[0], C.np, st, C.T, C.np, st, 0.0, S[1], C.np,
                               st, C.cnt, nullptr, 0, s);
      if (e) return e;
      e = gemm_batched<double>(false, false, C.np, C.np, C.np, 1.0, S[1], C.np, st, C.V, C.np, st, 0.0, C.T, C.np,
                               st, C.cnt, nullptr, 0, s);
      if (e) return e;
      hipLaunchKernelGGL(bat_mirror_kernel, dim3(cx, C.cnt), dim3(256), 0, s, C.T, C.np);
      JAC_CHECK_LAUNCH();
    }
    // Step 4: FP64 sweeps with the stop test after each.
    hipLaunchKernelGGL((bat_check_kernel<double>), dim3(C.cnt), dim3(256), 0, s, dd, 0, P.tol);
    JAC_CHECK_LAUNCH();
    for (int sw = 1; sw <= C.sweeps; ++sw) {
      int e = class_sweep(P, C, sw, s);
      if (e) return e;
    }
  }
  return 0;
}

struct Force { int inner = 0, sweeps = 0, sweeps32 = 0; };

static int build_plan(Plan& P, int batch, const int* n_host, const double* const* A_host, const int* lda_host,
                      double* const* W_host, double* const* V_host, const int* ldv_host, double tol, int pre,
                      double tol32, int max_sweeps, const Force& f) {
  P.batch = batch;
  P.pre = pre;
  P.tol = tol;
  P.tol32 = tol32;
  // size classes, largest first
  std::vector<int> order(batch);
  for (int i = 0; i < batch; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return blk_np(n_host[a]) > blk_np(n_host[b]); });
  for (int k = 0; k < batch; ++k) {
    const int np = blk_np(n_host[order[k]]);
    if (P.cls.empty() || P.cls.back().np != np) {
      const TuneEntry t = tune_for(np, pre);
      const int sw = std::min(f.sweeps > 0 ? f.sweeps : t.sweeps, max_sweeps);
      P.cls.push_back({np, k, 0, 0, f.inner > 0 ? f.inner : t.inner, sw,
                       pre ? (f.sweeps32 > 0 ? f.sweeps32 : t.sweeps32) : 0, nullptr, nullptr});
    }
    P.cls.back().cnt++;
    P.cls.back().maxn = std::max(P.cls.back().maxn, n_host[order[k]]);
  }
  for (const Cls& C : P.cls)
    if (C.cnt > kMaxBatch) { set_error("batched: more than 65535 matrices of one size class"); return -1; }
  // memory
  size_t bytes = al(sizeof(BDesc<double>) * batch) + al(sizeof(BDesc<float>) * batch) + al(sizeof(void*) * batch) * 3 +
                 al(sizeof(int) * batch) * 6 + al(sizeof(double) * batch) * 2 + al(sizeof(unsigned long long) * batch) * 2;
  size_t scratch = 0;
  for (const Cls& C : P.cls) {
    const size_t sq = (size_t)C.np * C.np, m = C.np / 64;
    bytes += 2 * al(sq * 8 * C.cnt) + al(m * 64 * 64 * 8 * C.cnt) + al(m * 4 * C.cnt);
    scratch = std::max(scratch, sq * C.cnt);
  }
  if (pre) bytes += 4 * al(scratch * 8);
  if (hipMalloc(&P.mem, bytes) != hipSuccess) { set_error("batched: device allocation failed"); return 4; }
  Carve c(P.mem);
  P.d_desc = c.take<BDesc<double>>(batch);
  P.d_desc32 = c.take<BDesc<float>>(batch);
  const double** d_A = c.take<const double*>(batch);
  double** d_W = c.take<double*>(batch);
  double** d_V = c.take<double*>(batch);
  int* d_lda = c.take<int>(batch);
  P.d_ldv = c.take<int>(batch);
  P.d_orig = c.take<int>(batch);
  P.d_conv = c.take<int>(batch);
  P.d_conv32 = c.take<int>(batch);
  P.d_state = c.take<int>(batch);
  double* d_nrm2 = c.take<double>(batch);
  P.d_e2 = c.take<double>(batch);
  unsigned long long* d_rot = c.take<unsigned long long>(batch);
  unsigned long long* d_rot32 = c.take<unsigned long long>(batch);
  P.d_W = d_W;
  P.d_V = d_V;
  std::vector<BDesc<double>> h_desc(batch);
  std::vector<BDesc<float>> h_desc32(batch);
  std::vector<const double*> hA(batch);
  std::vector<double*> hW(batch), hV(batch);
  std::vector<int> hlda(batch), hldv(batch);
  for (Cls& C : P.cls) {
    const size_t sq = (size_t)C.np * C.np, m = C.np / 64;
    C.T = c.take<double>(sq * C.cnt);
    C.V = c.take<double>(sq * C.cnt);
    double* E = c.take<double>(m * 64 * 64 * C.cnt);
    int* ident = c.take<int>(m * C.cnt);
    for (int j = 0; j < C.cnt; ++j) {
      const int k = C.off + j, i = order[k], n = n_host[i];
      BDesc<double>& d = h_desc[k];
      d.Tm = C.T + sq * j;
      d.V = C.V + sq * j;
      d.E = E + m * 64 * 64 * j;
      d.ident = ident + m * j;
      d.rot = d_rot + k;
      d.nrm2 = d_nrm2 + k;
      d.conv = P.d_conv + k;
      d.n = n;
      d.ldt = C.np;
      d.ldv = C.np;
      d.s32 = C.sweeps32;
      d.tol_n = tol / n;
      BDesc<float>& d3 = h_desc32[k];
      d3.Tm = nullptr;
      d3.V = nullptr;
      d3.E = reinterpret_cast<float*>(d.E);
      d3.ident = d.ident;
      d3.rot = d_rot32 + k;
      d3.nrm2 = d.nrm2;
      d3.conv = P.d_conv32 + k;
      d3.n = n;
      d3.ldt = C.np;
      d3.ldv = C.np;
      d3.s32 = C.sweeps32;
      d3.tol_n = tol32 / n;
      hA[k] = A_host[i];
      hW[k] = W_host[i];
      hV[k] = V_host[i];
      hlda[k] = lda_host[i];
      hldv[k] = ldv_host[i];
    }
  }
  double* S[4] = {nullptr, nullptr, nullptr, nullptr};
  if (pre) {
    for (int i = 0; i < 4; ++i) S[i] = c.take<double>(scratch);
    // FP32 T and V of a class live in the series scratch (free until the FP32 stage is over).
    for (const Cls& C : P.cls)
      for (int j = 0; j < C.cnt; ++j) {
        const size_t sq = (size_t)C.np * C.np;
        h_desc32[C.off + j].Tm = reinterpret_cast<float*>(S[0]) + sq * j;
        h_desc32[C.off + j].V = reinterpret_cast<float*>(S[1]) + sq * j;
      }
  }
  JAC_HIP(hipMemcpy(P.d_desc, h_desc.data(), sizeof(BDesc<double>) * batch, hipMemcpyHostToDevice));
  JAC_HIP(hipMemcpy(P.d_desc32, h_desc32.data(), sizeof(BDesc<float>) * batch, hipMemcpyHostToDevice));
  JAC_HIP(hipMemcpy(d_A, hA.data(), sizeof(void*) * batch, hipMemcpyHostToDevice));
  JAC_HIP(hipMemcpy(d_W, hW.data(), sizeof(void*) * batch, hipMemcpyHostToDevice));
  JAC_HIP(hipMemcpy(d_V, hV.data(), sizeof(void*) * batch, hipMemcpyHostToDevice));
  JAC_HIP(hipMemcpy(d_lda, hlda.data(), sizeof(int) * batch, hipMemcpyHostToDevice));
  JAC_HIP(hipMemcpy(P.d_ldv, hldv.data(), sizeof(int) * batch, hipMemcpyHostToDevice));
  JAC_HIP(hipMemcpy(P.d_orig, order.data(), sizeof(int) * batch, hipMemcpyHostToDevice));
  P.h_conv.resize(batch);
  // capture on the library's stream (one stream, no branches)
  hipStream_t cs = capture_stream();
  if (!cs) { set_error("batched: capture stream creation failed"); return 4; }
  JAC_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
  int e = record_solve(P, d_A, d_lda, S, cs);
  hipGraph_t g = nullptr;
  const hipError_t ce = hipStreamEndCapture(cs, &g);
  if (e) { if (g) (void)hipGraphDestroy(g); return e; }
  if (ce != hipSuccess || !g) { set_error(std::string("batched: capture failed: ") + hipGetErrorString(ce)); return 4; }
  P.graph = g;
  JAC_HIP(hipGraphInstantiate(&P.exec, g, nullptr, nullptr, 0));
  return 0;
}

static std::vector<uintptr_t> make_key(int batch, const int* n_host, const double* const* A, const int* lda,
                                       double* const* W, double* const* V, const int* ldv, double tol, int pre,
                                       double tol32, int max_sweeps, const Force& f) {
  std::vector<uintptr_t> k;
  k.reserve(6 * (size_t)batch + 16);
  k.push_back((uintptr_t)batch);
  for (int i = 0; i < batch; ++i) {
    k.push_back((uintptr_t)n_host[i]);
    k.push_back((uintptr_t)A[i]);
    k.push_back((uintptr_t)lda[i]);
    k.push_back((uintptr_t)W[i]);
    k.push_back((uintptr_t)V[i]);
    k.push_back((uintptr_t)ldv[i]);
  }
  uint64_t tb, tb32;
  static_assert(sizeof(tb) == sizeof(tol), "");
  std::memcpy(&tb, &tol, 8);
  std::memcpy(&tb32, &tol32, 8);
  k.push_back((uintptr_t)tb);
  k.push_back((uintptr_t)pre);
  k.push_back((uintptr_t)tb32);
  k.push_back((uintptr_t)max_sweeps);
  k.push_back((uintptr_t)f.inner);
  k.push_back((uintptr_t)f.sweeps);
  k.push_back((uintptr_t)f.sweeps32);
  int dev = 0;
  (void)hipGetDevice(&dev);
  k.push_back((uintptr_t)dev);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (auto& kv : g_tune) {
    k.push_back(kv.first.first * 2 + kv.first.second);
    k.push_back(kv.second.inner);
    k.push_back(kv.second.sweeps);
    k.push_back(kv.second.sweeps32);
  }
  return k;
}

struct RunOut {
  int topup = 0;          // eager FP64 sweeps after the graph, summed over classes
  int built = 0;          // 1 when this call captured a new graph
  int classes = 0;
  std::vector<int> conv;  // per matrix (class order), if asked for
  std::vector<int> conv32;
  std::vector<int> state;
};

static int run_batched(int batch, const int* n_host, const double* const* A, const int* lda, double* const* W,
                       double* const* V, const int* ldv, double tol, int pre, double tol32, int max_sweeps,
                       int* sweeps_dev, int* info_dev, int* sweeps32_dev, hipStream_t s, const Force& f,
                       RunOut* out, bool want_flags) {
  std::vector<uintptr_t> key = make_key(batch, n_host, A, lda, W, V, ldv, tol, pre, tol32, max_sweeps, f);
  std::lock_guard<std::mutex> lk(g_plan_mu);
  if (!g_plan || g_plan->key != key) {
    if (g_plan) {
      JAC_HIP(hipDeviceSynchronize());
      delete g_plan;
      g_plan = nullptr;
    }
    Plan* P = new Plan();
    const int e = build_plan(*P, batch, n_host, A, lda, W, V, ldv, tol, pre, tol32, max_sweeps, f);
    if (e) { delete P; return e; }
    P->key = std::move(key);
    g_plan = P;
    if (out) out->built = 1;
  }
  Plan& P = *g_plan;
  if (out) out->classes = (int)P.cls.size();
  JAC_HIP(hipGraphLaunch(P.exec, s));
  // convergence check and top-up
  JAC_HIP(hipMemcpyAsync(P.h_conv.data(), P.d_conv, sizeof(int) * batch, hipMemcpyDeviceToHost, s));
  JAC_HIP(hipStreamSynchronize(s));
  for (const Cls& C : P.cls) {
    auto pending = [&]() {
      int u = 0;
      for (int j = 0; j < C.cnt; ++j) u += P.h_conv[C.off + j] < 0;
      return u;
    };
    for (int sw = C.sweeps + 1; sw <= max_sweeps && pending() > 0; ++sw) {
      const int e = class_sweep(P, C, sw, s);
      if (e) return e;
      if (out) out->topup++;
      JAC_HIP(hipMemcpyAsync(P.h_conv.data() + C.off, P.d_conv + C.off, sizeof(int) * C.cnt, hipMemcpyDeviceToHost,
                             s));
      JAC_HIP(hipStreamSynchronize(s));
    }
  }
  hipLaunchKernelGGL(bat_finish_kernel, dim3(batch), dim3(256), 0, s, (const BDesc<double>*)P.d_desc, P.d_W, P.d_V,
                     (const int*)P.d_ldv, (const int*)P.d_orig, (const int*)P.d_conv32, max_sweeps, sweeps_dev,
                     info_dev, sweeps32_dev);
  JAC_CHECK_LAUNCH();
  if (out && want_flags) {
    out->conv = P.h_conv;
    out->conv32.resize(batch);
    out->state.resize(batch);
    JAC_HIP(hipMemcpyAsync(out->conv32.data(), P.d_conv32, sizeof(int) * batch, hipMemcpyDeviceToHost, s));
    JAC_HIP(hipMemcpyAsync(out->state.data(), P.d_state, sizeof(int) * batch, hipMemcpyDeviceToHost, s));
  }
  JAC_HIP(hipStreamSynchronize(s));
  return 0;
}

}  // namespace jac

using namespace jac;

static int check_batched(int batch, const int* n_host, const double* const* A, const int* lda, double* const* W,
                         double* const* V, const int* ldv) {
  if (batch < 0) { set_error("batch < 0"); return -1; }
  if (batch == 0) return 0;
  if (batch > kMaxBatch) { set_error("batch > 65535"); return -1; }
  if (!n_host) { set_error("n is NULL"); return -2; }
  if (!A) { set_error("A is NULL"); return -3; }
  if (!lda) { set_error("lda is NULL"); return -4; }
  if (!W) { set_error("W is NULL"); return -5; }
  if (!V) { set_error("V is NULL"); return -6; }
  if (!ldv) { set_error("ldv is NULL"); return -7; }
  for (int i = 0; i < batch; ++i) {
    const int n = n_host[i];
    if (n < 1 || n > kMaxBatchN) { set_error("batched: every n must be in [1, 512]"); return -2; }
    if (lda[i] < n) { set_error("batched: lda[i] < n[i]"); return -4; }
    if (ldv[i] < n) { set_error("batched: ldv[i] < n[i]"); return -7; }
    if (!A[i] || !W[i] || !V[i]) { set_error("batched: NULL matrix pointer"); return -3; }
  }
  return 0;
}

// Options resolved: precond flag (0/1), FP32 stop, sweep cap.  Returns 0 or a negative code.
static int resolve_opts(const jac_batched_opts* o, int& pre, double& tol32, int& max_sweeps) {
  pre = 0;
  tol32 = kDefaultFp32Tol;
  max_sweeps = kDefaultMaxSweeps;
  if (!o) return 0;
  if (o->precond != JAC_PRECOND_NONE && o->precond != JAC_PRECOND_FP32) {
    set_error("batched: precond must be JAC_PRECOND_NONE or JAC_PRECOND_FP32");
    return -12;
  }
  if (o->reserved != 0) { set_error("jac_batched_opts.reserved must be 0"); return -12; }
  pre = o->precond == JAC_PRECOND_FP32;
  if (o->fp32_tol != o->fp32_tol) { set_error("fp32_tol is NaN"); return -12; }
  if (o->fp32_tol > 0) tol32 = o->fp32_tol;
  if (o->max_sweeps < 0 || o->max_sweeps > 1000) { set_error("max_sweeps must be in [0, 1000]"); return -12; }
  if (o->max_sweeps > 0) max_sweeps = o->max_sweeps;
  return 0;
}

static int autotune(int batch, const int* n_host, const double* const* A, const int* lda, double tol, int pre,
                    double tol32, hipStream_t s) {
  // up to 16 sample matrices of each size class
  std::map<int, std::vector<int>> byclass;
  for (int i = 0; i < batch; ++i) {
    auto& v = byclass[blk_np(n_host[i])];
    if (v.size() < 16) v.push_back(i);
  }
  for (auto& kv : byclass) {
    const std::vector<int>& idx = kv.second;
    const int cnt = (int)idx.size();
    std::vector<int> ns(cnt), ldas(cnt), ldvs(cnt);
    std::vector<const double*> As(cnt);
    std::vector<double*> Ws(cnt), Vs(cnt);
    size_t tot = 0;
    for (int k = 0; k < cnt; ++k) tot += (size_t)n_host[idx[k]] * (n_host[idx[k]] + 1);
    double* buf = nullptr;
    JAC_HIP(hipMalloc(&buf, tot * 8));
    size_t off = 0;
    for (int k = 0; k < cnt; ++k) {
      const int n = n_host[idx[k]];
      ns[k] = n; ldas[k] = lda[idx[k]]; ldvs[k] = n; As[k] = A[idx[k]];
      Ws[k] = buf + off; off += n;
      Vs[k] = buf + off; off += (size_t)n * n;
    }
    TuneEntry best = tune_for(kv.first, pre);
    float best_ms = 1e30f;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = 0;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
      set_error("autotune: event creation failed");
      rc = 4;
    }
    for (int inner = 1; inner <= 4 && !rc; ++inner) {
      // sweeps the samples need with this cap (a generous count in the graph, flags read back)
      Force f;
      f.inner = inner;
      f.sweeps = 40;
      f.sweeps32 = pre ? 40 : 0;
      RunOut out;
      rc = run_batched(cnt, ns.data(), As.data(), ldas.data(), Ws.data(), Vs.data(), ldvs.data(), tol, pre, tol32, 40,
                       nullptr, nullptr, nullptr, s, f, &out, true);
      if (rc) break;
      int need = 0, need32 = 0;
      bool ok = true;
      for (int k = 0; k < cnt; ++k) {
        ok &= out.conv[k] >= 0;
        need = std::max(need, out.conv[k]);
        need32 = std::max(need32, out.conv32[k] < 0 ? 40 : out.conv32[k]);
      }
      if (!ok) continue;
      f.sweeps = std::max(need, 1);
      f.sweeps32 = pre ? std::max(need32, 1) : 0;
      // time that configuration (graph built outside the timing)
      rc = run_batched(cnt, ns.data(), As.data(), ldas.data(), Ws.data(), Vs.data(), ldvs.data(), tol, pre, tol32, 40,
                       nullptr, nullptr, nullptr, s, f, nullptr, false);
      if (rc) break;
      if (hipEventRecord(e0, s) != hipSuccess) { rc = 4; break; }
      rc = run_batched(cnt, ns.data(), As.data(), ldas.data(), Ws.data(), Vs.data(), ldvs.data(), tol, pre, tol32, 40,
                       nullptr, nullptr, nullptr, s, f, nullptr, false);
      if (rc) break;
      float ms = 0;
      if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { rc = 4; break; }
      if (ms < best_ms) { best_ms = ms; best = {inner, f.sweeps, f.sweeps32}; }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(s);
    {
      std::lock_guard<std::mutex> lk(g_plan_mu);
      delete g_plan;     // its pointers were the temporary buffers
      g_plan = nullptr;
    }
    (void)hipFree(buf);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (!g_tune_loaded) load_tune_locked();
    g_tune[{kv.first, pre}] = best;
  }
  std::lock_guard<std::mutex> lk(g_tune_mu);
  save_tune_locked();
  return 0;
}

extern "C" {

int syev_jacobi_batched_ex(int batch, const int* n_host, const double* const* A, const int* lda, double* const* W,
                           double* const* V, const int* ldv, double tol, int* sweeps, int* info, int* sweeps32,
                           const jac_batched_opts* opts, jac_batched_stats* stats, void* stream) {
  if (stats) std::memset(stats, 0, sizeof(*stats));
  int e = check_batched(batch, n_host, A, lda, W, V, ldv);
  if (e || batch == 0) return e;
  if (tol != tol) { set_error("tol is NaN"); return -8; }
  if (tol <= 0) tol = 20.0 * 1.1102230246251565e-16;
  int pre = 0, max_sweeps = 0;
  double tol32 = 0;
  if ((e = resolve_opts(opts, pre, tol32, max_sweeps))) return e;
  RunOut out;
  e = run_batched(batch, n_host, A, lda, W, V, ldv, tol, pre, tol32, max_sweeps, sweeps, info, sweeps32,
                  reinterpret_cast<hipStream_t>(stream), Force(), &out, stats != nullptr && pre);
  if (e) return e;
  if (stats) {
    stats->topup_sweeps = out.topup;
    stats->graph_built = out.built;
    stats->classes = out.classes;
    int failed = 0;
    for (int st : out.state) failed += st == 3;
    stats->series_failed = failed;
  }
  return 0;
}

int syev_jacobi_batched(int batch, const int* n_host, const double* const* A, const int* lda, double* const* W,
                        double* const* V, const int* ldv, double tol, int* sweeps, int* info, void* stream) {
  return syev_jacobi_batched_ex(batch, n_host, A, lda, W, V, ldv, tol, sweeps, info, nullptr, nullptr, nullptr,
                                stream);
}

int jac_autotune_batched_ex(int batch, const int* n_host, const double* const* A, const int* lda, double tol,
                            const jac_batched_opts* opts, void* stream) {
  int e = check_batched(batch, n_host, A, lda, (double* const*)A, (double* const*)A, lda);
  if (e || batch == 0) return e;
  if (tol != tol) { set_error("tol is NaN"); return -5; }
  if (tol <= 0) tol = 20.0 * 1.1102230246251565e-16;
  int pre = 0, max_sweeps = 0;
  double tol32 = 0;
  if ((e = resolve_opts(opts, pre, tol32, max_sweeps))) return e;
  return autotune(batch, n_host, A, lda, tol, pre, tol32, reinterpret_cast<hipStream_t>(stream));
}

int jac_autotune_batched(int batch, const int* n_host, const double* const* A, const int* lda, double tol,
                         void* stream) {
  return jac_autotune_batched_ex(batch, n_host, A, lda, tol, nullptr, stream);
}

int jac_tune_entry_ex(int n, int precond, int* inner, int* sweeps, int* sweeps32) {
  if (n < 1 || n > kMaxBatchN) { set_error("n must be in [1, 512]"); return -1; }
  const TuneEntry t = tune_for(blk_np(n), precond == JAC_PRECOND_FP32 ? 1 : 0);
  if (inner) *inner = t.inner;
  if (sweeps) *sweeps = t.sweeps;
  if (sweeps32) *sweeps32 = t.sweeps32;
  return 0;
}

int jac_tune_entry(int n, int* inner, int* sweeps) { return jac_tune_entry_ex(n, JAC_PRECOND_NONE, inner, sweeps, nullptr); }

int jac_tune_clear(void) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune.clear();
  g_tune_loaded = true;   // the cache file is not read again in this process
  return 0;
}

}  // extern "C"
