// Batched path: thousands of independent symmetric eigenproblems of uneven
// order (n <= 512) in one graph launch.
//
// Matrices are grouped by padded order np (a multiple of 64).  Each size class
// advances through the block steps of the blocked Jacobi method in lockstep:
// every launch covers all matrices of the class (grid y = matrix).  A matrix
// that has converged costs little in later sweeps: its inner solves find
// nothing to rotate and its block updates are skipped.  The whole solve -- set
// up, every class's sweeps (one graph branch per class, so small classes run
// beside large ones), the per-sweep norms and the ordered output -- is
// captured once into a hipGraph that is cached and replayed while the inputs
// (sizes and pointers) stay the same.  No memset nodes are recorded (fill
// kernels instead).
//
// The number of sweeps and the inner-sweep cap of each size class come from an
// autotuner (jac_autotune_batched) that times the candidates on sample
// matrices and keeps the fastest configuration that converges; its table can
// be cached in the text file named by JACOBI_TUNE_CACHE.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <vector>

#include "../../include/jacobi.h"
#include "common.h"

namespace jac {

struct TuneEntry { int inner, sweeps; };
static std::map<int, TuneEntry> g_tune;
static bool g_tune_loaded = false;
static std::mutex g_tune_mu;
constexpr int kDefaultInner = 2, kDefaultSweeps = 16, kMaxBatchN = 512;

static void load_tune_locked() {
  g_tune_loaded = true;
  const char* p = std::getenv("JACOBI_TUNE_CACHE");
  if (!p) return;
  std::ifstream f(p);
  int np, inner, sweeps;
  while (f >> np >> inner >> sweeps)
    if (np > 0 && inner > 0 && sweeps > 0) g_tune[np] = {inner, sweeps};
}

static void save_tune_locked() {
  const char* p = std::getenv("JACOBI_TUNE_CACHE");
  if (!p) return;
  std::ofstream f(p);
  for (auto& kv : g_tune) f << kv.first << " " << kv.second.inner << " " << kv.second.sweeps << "\n";
}

static TuneEntry tune_for(int np) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  if (!g_tune_loaded) load_tune_locked();
  auto it = g_tune.find(np);
  if (it != g_tune.end()) return it->second;
  return {kDefaultInner, kDefaultSweeps};
}

static inline size_t al(size_t x) { return (x + 255) / 256 * 256; }

struct Plan {
  std::vector<uintptr_t> key;
  int batch = 0, sweeps = 0;
  void* mem = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> events;
  ~Plan() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    for (auto e : events) (void)hipEventDestroy(e);
    for (auto s : streams) (void)hipStreamDestroy(s);
    if (mem) (void)hipFree(mem);
  }
};
static Plan* g_plan = nullptr;
static std::mutex g_plan_mu;

// Build (capture) the graph of one batched solve.  overrides: if inner_force >
// 0 / sweeps_force > 0, they replace the tuned values (used by the autotuner).
static int build_plan(Plan& P, int batch, const int* n_host, const double* const* A_host, const int* lda_host,
                      double* const* W_host, double* const* V_host, const int* ldv_host, double tol,
                      int* sweeps_dev, int* info_dev, int inner_force, int sweeps_force) {
  // size classes
  std::vector<int> order(batch);
  for (int i = 0; i < batch; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return blk_np(n_host[a]) > blk_np(n_host[b]); });
  struct Cls { int np, off, cnt, maxn, inner, sweeps; };
  std::vector<Cls> cls;
  for (int k = 0; k < batch; ++k) {
    int np = blk_np(n_host[order[k]]);
    if (cls.empty() || cls.back().np != np) {
      TuneEntry t = tune_for(np);
      cls.push_back({np, k, 0, 0, inner_force > 0 ? inner_force : t.inner,
                     sweeps_force > 0 ? sweeps_force : t.sweeps});
    }
    cls.back().cnt++;
    cls.back().maxn = std::max(cls.back().maxn, n_host[order[k]]);
  }
  int S = 0;
  for (auto& c : cls) S = std::max(S, c.sweeps);
  P.sweeps = S;
  // memory
  size_t bytes = 0;
  bytes += al(sizeof(BDesc<double>) * batch) + al(sizeof(void*) * batch) * 3 + al(sizeof(int) * batch) * 3;
  bytes += al(sizeof(double) * 2 * (size_t)batch * (S + 1)) + al(sizeof(unsigned long long) * batch);
  for (int k = 0; k < batch; ++k) {
    int n = n_host[order[k]], np = blk_np(n), m = np / 64;
    bytes += al((size_t)np * np * 8) + al((size_t)n * np * 8) + al((size_t)m * 64 * 64 * 8) + al(m * 4);
  }
  if (hipMalloc(&P.mem, bytes) != hipSuccess) { set_error("batched: device allocation failed"); return 4; }
  Carve c(P.mem);
  BDesc<double>* d_desc = c.take<BDesc<double>>(batch);
  const double** d_A = c.take<const double*>(batch);
  double** d_W = c.take<double*>(batch);
  double** d_V = c.take<double*>(batch);
  int* d_lda = c.take<int>(batch);
  int* d_ldv = c.take<int>(batch);
  int* d_orig = c.take<int>(batch);
  const int stride = 2 * batch;
  double* d_norms = c.take<double>((size_t)stride * (S + 1));
  unsigned long long* d_rot = c.take<unsigned long long>(batch);
  std::vector<BDesc<double>> h_desc(batch);
  std::vector<const double*> hA(batch);
  std::vector<double*> hW(batch), hV(batch);
  std::vector<int> hlda(batch), hldv(batch);
  for (int k = 0; k < batch; ++k) {
    int i = order[k], n = n_host[i], np = blk_np(n), m = np / 64;
    BDesc<double>& d = h_desc[k];
    d.Tm = c.take<double>((size_t)np * np);
    d.V = c.take<double>((size_t)n * np);
    d.E = c.take<double>((size_t)m * 64 * 64);
    d.ident = c.take<int>(m);
    d.rot = d_rot + k;
    d.nrm2 = d_norms + 2 * (size_t)k + 1;
    d.n = n;
    d.ldt = np;
    d.ldv = n;
    d.pad = 0;
    d.tol_n = tol / n;
    hA[k] = A_host[i];
    hW[k] = W_host[i];
    hV[k] = V_host[i];
    hlda[k] = lda_host[i];
    hldv[k] = ldv_host[i];
  }
  JAC_HIP(hipMemcpy(d_desc, h_desc.data(), sizeof(BDesc<double>) * batch, hipMemcpyHostToDevice));
  JAC_HIP(hipMemcpy(d_A, hA.data(), sizeof(void*) * batch, hipMemcpyHostToDevice));
  JAC_HIP(hipMemcpy(d_W, hW.data(), sizeof(void*) * batch, hipMemcpyHostToDevice));
  JAC_HIP(hipMemcpy(d_V, hV.data(), sizeof(void*) * batch, hipMemcpyHostToDevice));
  JAC_HIP(hipMemcpy(d_lda, hlda.data(), sizeof(int) * batch, hipMemcpyHostToDevice));
  JAC_HIP(hipMemcpy(d_ldv, hldv.data(), sizeof(int) * batch, hipMemcpyHostToDevice));
  JAC_HIP(hipMemcpy(d_orig, order.data(), sizeof(int) * batch, hipMemcpyHostToDevice));
  // capture
  hipStream_t cs;
  JAC_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  P.streams.push_back(cs);
  for (size_t k = 0; k < cls.size(); ++k) {
    hipStream_t st;
    JAC_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    P.streams.push_back(st);
  }
  for (size_t k = 0; k < cls.size() + 1; ++k) {
    hipEvent_t e;
    JAC_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    P.events.push_back(e);
  }
  JAC_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed));
  int maxnp = cls.front().np;
  int e = batched_init<double>(d_desc, batch, maxnp, d_A, d_lda, cs);
  if (!e) e = batched_norms<double>(d_desc, batch, d_norms, cs);
  if (!e) {
    JAC_HIP(hipEventRecord(P.events[0], cs));
    for (size_t k = 0; k < cls.size() && !e; ++k) {
      hipStream_t st = P.streams[k + 1];
      const Cls& C = cls[k];
      JAC_HIP(hipStreamWaitEvent(st, P.events[0], 0));
      for (int sw = 1; sw <= S && !e; ++sw) {
        e = blk_sweep_batched<double>(d_desc + C.off, C.cnt, C.np, C.maxn, C.inner, st);
        if (!e) e = batched_norms<double>(d_desc + C.off, C.cnt, d_norms + (size_t)sw * stride + 2 * C.off, st);
      }
      JAC_HIP(hipEventRecord(P.events[k + 1], st));
      JAC_HIP(hipStreamWaitEvent(cs, P.events[k + 1], 0));
    }
  }
  if (!e)
    e = batched_finish<double>(d_desc, batch, d_W, d_V, d_ldv, d_norms, stride, S, tol, d_orig, sweeps_dev, info_dev,
                               cs);
  hipGraph_t g = nullptr;
  hipError_t ce = hipStreamEndCapture(cs, &g);
  if (e) { if (g) (void)hipGraphDestroy(g); return e; }
  if (ce != hipSuccess) { set_error(std::string("batched: capture failed: ") + hipGetErrorString(ce)); return 4; }
  P.graph = g;
  JAC_HIP(hipGraphInstantiate(&P.exec, g, nullptr, nullptr, 0));
  P.batch = batch;
  return 0;
}

static std::vector<uintptr_t> make_key(int batch, const int* n_host, const double* const* A, const int* lda,
                                       double* const* W, double* const* V, const int* ldv, double tol, int* sw,
                                       int* info, int inner_force, int sweeps_force) {
  std::vector<uintptr_t> k;
  k.reserve(6 * (size_t)batch + 8);
  k.push_back((uintptr_t)batch);
  for (int i = 0; i < batch; ++i) {
    k.push_back((uintptr_t)n_host[i]);
    k.push_back((uintptr_t)A[i]);
    k.push_back((uintptr_t)lda[i]);
    k.push_back((uintptr_t)W[i]);
    k.push_back((uintptr_t)V[i]);
    k.push_back((uintptr_t)ldv[i]);
  }
  uint64_t tb;
  static_assert(sizeof(tb) == sizeof(tol), "");
  std::memcpy(&tb, &tol, 8);
  k.push_back((uintptr_t)tb);
  k.push_back((uintptr_t)sw);
  k.push_back((uintptr_t)info);
  k.push_back((uintptr_t)inner_force);
  k.push_back((uintptr_t)sweeps_force);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (auto& kv : g_tune) { k.push_back(kv.first); k.push_back(kv.second.inner); k.push_back(kv.second.sweeps); }
  return k;
}

static int run_batched(int batch, const int* n_host, const double* const* A, const int* lda, double* const* W,
                       double* const* V, const int* ldv, double tol, int* sweeps_dev, int* info_dev,
                       hipStream_t s, int inner_force, int sweeps_force) {
  std::vector<uintptr_t> key =
      make_key(batch, n_host, A, lda, W, V, ldv, tol, sweeps_dev, info_dev, inner_force, sweeps_force);
  std::lock_guard<std::mutex> lk(g_plan_mu);
  if (!g_plan || g_plan->key != key) {
    if (g_plan) {
      (void)hipDeviceSynchronize();
      delete g_plan;
      g_plan = nullptr;
    }
    Plan* P = new Plan();
    int e = build_plan(*P, batch, n_host, A, lda, W, V, ldv, tol, sweeps_dev, info_dev, inner_force, sweeps_force);
    if (e) { delete P; return e; }
    P->key = std::move(key);
    g_plan = P;
  }
  JAC_HIP(hipGraphLaunch(g_plan->exec, s));
  return 0;
}

}  // namespace jac

using namespace jac;

static int check_batched(int batch, const int* n_host, const double* const* A, const int* lda, double* const* W,
                         double* const* V, const int* ldv) {
  if (batch < 0) { set_error("batch < 0"); return -1; }
  if (batch == 0) return 0;
  if (!n_host) { set_error("n is NULL"); return -2; }
  if (!A) { set_error("A is NULL"); return -3; }
  if (!lda) { set_error("lda is NULL"); return -4; }
  if (!W) { set_error("W is NULL"); return -5; }
  if (!V) { set_error("V is NULL"); return -6; }
  if (!ldv) { set_error("ldv is NULL"); return -7; }
  for (int i = 0; i < batch; ++i) {
    int n = n_host[i];
    if (n < 1 || n > kMaxBatchN) { set_error("batched: every n must be in [1, 512]"); return -2; }
    if (lda[i] < n) { set_error("batched: lda[i] < n[i]"); return -4; }
    if (ldv[i] < n) { set_error("batched: ldv[i] < n[i]"); return -7; }
    if (!A[i] || !W[i] || !V[i]) { set_error("batched: NULL matrix pointer"); return -3; }
  }
  return 0;
}

extern "C" {

int syev_jacobi_batched(int batch, const int* n_host, const double* const* A, const int* lda, double* const* W,
                        double* const* V, const int* ldv, double tol, int* sweeps, int* info, void* stream) {
  int e = check_batched(batch, n_host, A, lda, W, V, ldv);
  if (e || batch == 0) return e;
  if (tol != tol) { set_error("tol is NaN"); return -8; }
  if (tol <= 0) tol = 20.0 * 1.1102230246251565e-16;
  return run_batched(batch, n_host, A, lda, W, V, ldv, tol, sweeps, info, reinterpret_cast<hipStream_t>(stream), 0,
                     0);
}

int jac_autotune_batched(int batch, const int* n_host, const double* const* A, const int* lda, double tol,
                         void* stream) {
  int e = check_batched(batch, n_host, A, lda, (double* const*)A, (double* const*)A, lda);
  if (e || batch == 0) return e;
  if (tol <= 0) tol = 20.0 * 1.1102230246251565e-16;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  // sample up to 16 matrices of each size class
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
    int* dsw = nullptr;
    JAC_HIP(hipMalloc(&buf, tot * 8));
    JAC_HIP(hipMalloc(&dsw, 2 * cnt * sizeof(int)));
    size_t off = 0;
    for (int k = 0; k < cnt; ++k) {
      int n = n_host[idx[k]];
      ns[k] = n; ldas[k] = lda[idx[k]]; ldvs[k] = n; As[k] = A[idx[k]];
      Ws[k] = buf + off; off += n;
      Vs[k] = buf + off; off += (size_t)n * n;
    }
    TuneEntry best{kDefaultInner, kDefaultSweeps};
    float best_ms = 1e30f;
    hipEvent_t e0, e1;
    JAC_HIP(hipEventCreate(&e0));
    JAC_HIP(hipEventCreate(&e1));
    for (int inner = 1; inner <= 4; ++inner) {
      // sweeps needed with this cap
      int rc = run_batched(cnt, ns.data(), As.data(), ldas.data(), Ws.data(), Vs.data(), ldvs.data(), tol, dsw,
                           dsw + cnt, s, inner, 40);
      if (rc) { (void)hipFree(buf); (void)hipFree(dsw); return rc; }
      std::vector<int> h(2 * cnt);
      JAC_HIP(hipMemcpyAsync(h.data(), dsw, 2 * cnt * sizeof(int), hipMemcpyDeviceToHost, s));
      JAC_HIP(hipStreamSynchronize(s));
      int need = 0;
      bool ok = true;
      for (int k = 0; k < cnt; ++k) { need = std::max(need, h[k]); ok &= h[cnt + k] == 0; }
      if (!ok) continue;
      int sweeps = need + 1;
      // time the configuration with exactly that many sweeps (graph built outside the timing)
      rc = run_batched(cnt, ns.data(), As.data(), ldas.data(), Ws.data(), Vs.data(), ldvs.data(), tol, dsw,
                       dsw + cnt, s, inner, sweeps);
      if (rc) { (void)hipFree(buf); (void)hipFree(dsw); return rc; }
      JAC_HIP(hipEventRecord(e0, s));
      rc = run_batched(cnt, ns.data(), As.data(), ldas.data(), Ws.data(), Vs.data(), ldvs.data(), tol, dsw,
                       dsw + cnt, s, inner, sweeps);
      if (rc) { (void)hipFree(buf); (void)hipFree(dsw); return rc; }
      JAC_HIP(hipEventRecord(e1, s));
      JAC_HIP(hipEventSynchronize(e1));
      float ms = 0;
      JAC_HIP(hipEventElapsedTime(&ms, e0, e1));
      if (ms < best_ms) { best_ms = ms; best = {inner, sweeps}; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    JAC_HIP(hipStreamSynchronize(s));
    {
      std::lock_guard<std::mutex> lk(g_plan_mu);
      delete g_plan;     // its buffers were the temporary ones
      g_plan = nullptr;
    }
    (void)hipFree(buf);
    (void)hipFree(dsw);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (!g_tune_loaded) load_tune_locked();
    g_tune[kv.first] = best;
  }
  std::lock_guard<std::mutex> lk(g_tune_mu);
  save_tune_locked();
  return 0;
}

int jac_tune_entry(int n, int* inner, int* sweeps) {
  TuneEntry t = tune_for(blk_np(n));
  if (inner) *inner = t.inner;
  if (sweeps) *sweeps = t.sweeps;
  return 0;
}

}  // extern "C"
