// Low-precision step 1 of Algorithm 4.1 by a tridiagonalization-based FP32
// eigensolver -- the kind of solver the paper uses there (ssyevd / cuSOLVER
// syevd, Section 6 setup), whose backward stability (Lemma symeig) is all the
// analysis needs:
//
//   1. Householder tridiagonalization Q^T A Q = T in FP32 (sytrd_kernel): one
//      reflector H_k = I - tau u u^T per column, u(k+1) = 1, beta = -sign(alpha)
//      ||x||, the trailing block updated by the symmetric rank-2 update with
//      p = tau B u and w = p - (tau p^T u / 2) u.
//   2. Eigenvalues of T in FP64 by bisection on the Sturm count (the signs of
//      the pivots of T - x I), 64 points per wave and round (tri_bisect_kernel).
//   3. Eigenvectors of T in FP64 from the twisted factorization of T - lambda I
//      (forward and backward pivots; the twist index minimises the twisted
//      pivot; one outward solve), one thread per eigenvalue (tri_vectors_kernel).
//   4. Z = H_0 H_1 ... H_{n-3} Y in FP32, the reflectors grouped in blocks of
//      kBtNb as I - U T U^T (T from the reflectors' Gram matrix) and applied
//      by three GEMMs per block on the matrix cores.
//
// The tridiagonalization has one global reduction per column (p = B u); it
// runs as one cooperative launch of up to 256 workgroups.  Row i of the
// working matrix belongs to workgroup i mod G and stays in its LDS (or, for
// large n, in a private global slice).  Every workgroup computes each
// reflector itself from the published row (all with the same instructions, so
// the results agree bit for bit); per column the workgroups exchange only the
// entries of p and the next row.  The exchange words carry the column's tag in
// their upper half and the FP32 value in the lower half and are written and
// read as single 64-bit agent-scope atomics, so a reader that sees the tag has
// the value, without fences or counters.  Waits are bounded: a workgroup that
// waits about a second sets an abort flag, every workgroup then leaves, and
// the host reports a device error.
#include <cmath>
#include <type_traits>

#include "common.h"

namespace jac {

static inline int tcdiv(long long a, long long b) { return (int)((a + b - 1) / b); }

constexpr int kTdThreads = 256;
constexpr int kTdWaves = kTdThreads / 64;
constexpr int kTdMaxG = 256;          // workgroups of the tridiagonalization
constexpr int kTdRegMaxN = 4096;      // working rows held in registers up to this order
constexpr int kTdGlbRows = 32;        // global-slice rows per workgroup: n <= 32 G = 8192
constexpr int kTdMaxN = kTdGlbRows * kTdMaxG;
constexpr int kTdGather = 8;          // exchange words a thread loads per batch
constexpr int kBtNb = 128;            // reflectors per back-transformation block
constexpr int kVecChunk = 2048;       // eigenvectors per twisted-factorization launch

__device__ __forceinline__ unsigned long long td_pack(unsigned tag, float v) {
  return ((unsigned long long)tag << 32) | (unsigned long long)__float_as_uint(v);
}

__device__ __forceinline__ float wave_sum_f(float v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_sum_d(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

struct TdArgs {
  int n, G;
  float* rows;                    // global-slice mode: row i of the working matrix at rows + i * n
  unsigned long long* pbuf;       // [2][n] tagged entries of p, by column parity
  unsigned long long* rbuf;       // [2][n] tagged entries of the published row
  unsigned* hb;                   // [G] last column each workgroup has published (monotonic)
  double* d;                      // n diagonal entries of T
  double* e;                      // n - 1 subdiagonal entries
  float* tau;                     // n - 2 reflector scalars
  double* U;                      // n x ldu... column k = u_k (zero above row k + 1), FP32 values
  int ldu;
  double* Ut;                     // row k = u_k (Ut[k + j * ldut])
  int ldut;
  int* abort;                     // nonzero: some workgroup gave up waiting
};

// Column j of every LDS vector and of the own rows is always handled by thread j % kTdThreads, so a
// thread reads back only what it wrote itself except where a barrier separates the two.
__device__ __forceinline__ int td_first(int lo) {
  const int t = threadIdx.x;
  return lo <= t ? t : t + (lo - t + kTdThreads - 1) / kTdThreads * kTdThreads;
}

// Householder reflector of x = r(k+1 .. n-1) (row k of the working matrix, in LDS):
// v(j) for j >= k+1 into vL, tau and beta returned (identical in every workgroup).
__device__ void td_reflector(const float* rk, float* vL, int n, int k, double* red, int& slot, float& tau,
                             float& beta) {
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  double part = 0.0;
  for (int j = td_first(k + 2); j < n; j += kTdThreads) part += (double)rk[j] * (double)rk[j];
  part = wave_sum_d(part);
  double* r = red + slot * 8;
  slot ^= 1;
  if (lane == 0) r[wv] = part;
  __syncthreads();
  double tail = 0.0;
  for (int i = 0; i < kTdWaves; ++i) tail += r[i];
  const float alpha = rk[k + 1];
  float scal = 0.f;
  if (tail == 0.0) {
    tau = 0.f;
    beta = alpha;
  } else {
    const double a = (double)alpha;
    const double rr = sqrt(a * a + tail);
    const double b = a >= 0.0 ? -rr : rr;
    tau = (float)((b - a) / b);
    beta = (float)b;
    scal = (float)(1.0 / (a - b));
  }
  for (int j = td_first(k + 1); j < n; j += kTdThreads) vL[j] = (j == k + 1) ? 1.f : rk[j] * scal;
}

// Wait until entry j of buf carries tag; returns its value (0 and sets the abort flag on a timeout:
// abort[0] = 1, then the column tag, the workgroup, the entry and which buffer, for the error text).
__device__ __forceinline__ float td_wait(unsigned long long* buf, int j, unsigned tag, int* abort, bool& bad,
                                         int which) {
  unsigned long long x = __hip_atomic_load(buf + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if ((unsigned)(x >> 32) == tag) return __uint_as_float((unsigned)x);
  const unsigned long long t0 = wall_clock64();
  for (int spin = 1;; ++spin) {
    __builtin_amdgcn_s_sleep(1);
    x = __hip_atomic_load(buf + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if ((unsigned)(x >> 32) == tag) return __uint_as_float((unsigned)x);
    if ((spin & 255) == 0) {
      if (__hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) { bad = true; return 0.f; }
      if (wall_clock64() - t0 > 100000000ull) {   // ~1 s of the 100 MHz constant clock
        if (__hip_atomic_exchange(abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
          abort[1] = (int)tag;
          abort[2] = (int)blockIdx.x;
          abort[3] = j;
          abort[4] = which;
          abort[5] = (int)(x >> 32);
        }
        bad = true;
        return 0.f;
      }
    }
  }
}

// Wait until workgroup heartbeat *h has reached tag (same timeout rule as td_wait).
__device__ __forceinline__ void td_wait_hb(unsigned* h, unsigned tag, int* abort, bool& bad) {
  unsigned x = __hip_atomic_load(h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (x >= tag) return;
  const unsigned long long t0 = wall_clock64();
  for (int spin = 1;; ++spin) {
    __builtin_amdgcn_s_sleep(1);
    x = __hip_atomic_load(h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (x >= tag) return;
    if ((spin & 255) == 0) {
      if (__hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) { bad = true; return; }
      if (wall_clock64() - t0 > 100000000ull) {
        if (__hip_atomic_exchange(abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
          abort[1] = (int)tag;
          abort[2] = (int)blockIdx.x;
          abort[3] = (int)threadIdx.x;
          abort[4] = 2;
          abort[5] = (int)x;
        }
        bad = true;
        return;
      }
    }
  }
}

template <typename TA, bool kLds, int kMaxRows>
__global__ __launch_bounds__(kTdThreads) void sytrd_kernel(const TA* __restrict__ A, int lda, TdArgs a) {
  extern __shared__ __align__(16) unsigned char td_smem[];
  const int n = a.n, G = a.G, wg = blockIdx.x, t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int nr = (n - wg + G - 1) / G;   // own rows wg, wg + G, ...
  float* base = reinterpret_cast<float*>(td_smem);
  float* rowsL = base;
  float* vL = base + (kLds ? kMaxRows * n : 0);
  float* pL = vL + n;
  float* rk = pL + n;
  double* red = reinterpret_cast<double*>(rk + n + (n & 1));   // 2 slots x 8 doubles
  float* redf = reinterpret_cast<float*>(red + 16);           // 2 slots x (kTdWaves x kMaxRows)
  int slot = 0, fslot = 0;
  auto row = [&](int r) -> float* { return kLds ? rowsL + (size_t)r * n : a.rows + (size_t)(wg + r * G) * n; };

  // own rows (row i = column i of the symmetric input) and row 0 for the first reflector
  for (int r = 0; r < nr; ++r) {
    const int i = wg + r * G;
    float* R = row(r);
    for (int j = t; j < n; j += kTdThreads) R[j] = (float)A[j + (size_t)i * lda];
  }
  for (int j = t; j < n; j += kTdThreads) rk[j] = (float)A[j];
  __syncthreads();
  float tauk = 0.f, beta = 0.f;
  td_reflector(rk, vL, n, 0, red, slot, tauk, beta);
  if (wg == 0) {
    if (t == 0) { a.d[0] = rk[0]; a.e[0] = beta; a.tau[0] = tauk; }
    for (int j = t; j < n; j += kTdThreads) {
      const float u = j >= 1 ? vL[j] : 0.f;
      a.U[j] = u;
      a.Ut[(size_t)j * a.ldut] = u;
    }
  }
  bool bad = false;
  for (int k = 0; k + 2 < n; ++k) {
    const unsigned tag = (unsigned)k + 1u;
    const int par = k & 1;
    unsigned long long* pb = a.pbuf + (size_t)par * n;
    unsigned long long* rb = a.rbuf + (size_t)par * n;
    // (1) p(i) = tau B(i, k+1:) v for the own rows i > k
    float acc[kMaxRows];
#pragma unroll
    for (int r = 0; r < kMaxRows; ++r) acc[r] = 0.f;
    for (int j = td_first(k + 1); j < n; j += kTdThreads) {
      const float vj = vL[j];
#pragma unroll
      for (int r = 0; r < kMaxRows; ++r)
        if (r < nr) acc[r] = fmaf(row(r)[j], vj, acc[r]);
    }
    {
      float* rf = redf + fslot * (kTdWaves * kMaxRows);
      fslot ^= 1;
#pragma unroll
      for (int r = 0; r < kMaxRows; ++r) {
        const float sr = wave_sum_f(acc[r]);
        if (lane == 0 && r < nr) rf[wv * kMaxRows + r] = sr;
      }
      __syncthreads();
      // (2) publish the own entries of p and, from the owner of row k+1, that row
      if (t < nr) {
        const int i = wg + t * G;
        if (i > k) {
          float s = 0.f;
          for (int q = 0; q < kTdWaves; ++q) s += rf[q * kMaxRows + t];
          __hip_atomic_store(pb + i, td_pack(tag, tauk * s), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
    }
    if ((k + 1) % G == wg) {
      const float* R = row((k + 1 - wg) / G);
      for (int j = td_first(k + 1); j < n; j += kTdThreads)
        __hip_atomic_store(rb + j, td_pack(tag, R[j]), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    // heartbeat: this workgroup is done reading column k - 1 (it may own no entry of p(k+1:),
    // and the buffers of column k - 1 are reused at column k + 1)
    if (t == 0) __hip_atomic_store(a.hb + wg, tag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    // (3) gather p(k+1:) and the row: all loads of a batch are issued before any tag is tested
    for (int j0 = td_first(k + 1); j0 < n; j0 += kTdGather * kTdThreads) {
      unsigned long long xp[kTdGather], xr[kTdGather];
#pragma unroll
      for (int q = 0; q < kTdGather; ++q) {
        const int j = j0 + q * kTdThreads;
        if (j < n) {
          xp[q] = __hip_atomic_load(pb + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          xr[q] = __hip_atomic_load(rb + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
#pragma unroll
      for (int q = 0; q < kTdGather; ++q) {
        const int j = j0 + q * kTdThreads;
        if (j < n) {
          pL[j] = (unsigned)(xp[q] >> 32) == tag ? __uint_as_float((unsigned)xp[q]) : td_wait(pb, j, tag, a.abort, bad, 0);
          rk[j] = (unsigned)(xr[q] >> 32) == tag ? __uint_as_float((unsigned)xr[q]) : td_wait(rb, j, tag, a.abort, bad, 1);
        }
      }
    }
    if (t < G) td_wait_hb(a.hb + t, tag, a.abort, bad);
    // (4) s = p^T v, w = p - (tau s / 2) v
    float part = 0.f;
    for (int j = td_first(k + 1); j < n; j += kTdThreads) part = fmaf(pL[j], vL[j], part);
    part = wave_sum_f(part);
    {
      float* rf = redf + fslot * (kTdWaves * kMaxRows);
      fslot ^= 1;
      const bool wbad = __ballot(bad) != 0ull;   // a thread of this wave gave up waiting
      if (lane == 0) {
        rf[wv] = part;
        rf[kTdWaves + wv] = wbad ? 1.f : 0.f;
      }
      __syncthreads();
      float anybad = 0.f;
      part = 0.f;
      for (int q = 0; q < kTdWaves; ++q) {
        part += rf[q];
        anybad += rf[kTdWaves + q];
      }
      if (anybad != 0.f) break;
    }
    const float c = 0.5f * tauk * part;
    // (5) own rows i > k:  B(i, j) -= v(i) w(j) + w(i) v(j),  j > k
    for (int r = 0; r < nr; ++r) {
      const int i = wg + r * G;
      if (i <= k) continue;
      const float vi = vL[i], wi = pL[i] - c * vL[i];
      float* R = row(r);
      for (int j = td_first(k + 1); j < n; j += kTdThreads) {
        const float wj = pL[j] - c * vL[j];
        R[j] = R[j] - (vi * wj + wi * vL[j]);
      }
    }
    // (6) row k+1 of the updated matrix, then the next reflector
    const float wk1 = pL[k + 1] - c;   // v(k+1) = 1
    for (int j = td_first(k + 1); j < n; j += kTdThreads) {
      const float wj = pL[j] - c * vL[j];
      rk[j] = rk[j] - (wj + wk1 * vL[j]);
    }
    if (k + 3 < n) {
      td_reflector(rk, vL, n, k + 1, red, slot, tauk, beta);
      if (wg == 0) {
        if (t == 0) { a.d[k + 1] = rk[k + 1]; a.e[k + 1] = beta; a.tau[k + 1] = tauk; }
        double* Uc = a.U + (size_t)(k + 1) * a.ldu;
        for (int j = t; j < n; j += kTdThreads) {
          const float u = j >= k + 2 ? vL[j] : 0.f;
          Uc[j] = u;
          a.Ut[(k + 1) + (size_t)j * a.ldut] = u;
        }
      }
    } else {
      __syncthreads();
      if (wg == 0 && t == 0) { a.d[n - 2] = rk[n - 2]; a.e[n - 2] = rk[n - 1]; }
      if ((n - 1) % G == wg && t == 0) a.d[n - 1] = row((n - 1 - wg) / G)[n - 1];
    }
  }
}

// ---- wave and workgroup sums by lane exchanges ---------------------------------------------------
// A 32-bit value of another lane by a data-parallel-primitive move (CTRL = DPP control word).
template <int CTRL>
__device__ __forceinline__ float dppf(float x) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dppd(double x) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(x);
  const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
// Value of lane (lane ^ (1 << LVL)) inside a 16-lane row: quad permutations [1,0,3,2] and
// [2,3,0,1], a shift by 4 lanes up or down by bit 2, a rotation of the row by 8.
template <int LVL, typename T>
__device__ __forceinline__ T lane_xor(T x, int lane) {
  auto mv = [](T y, auto ctrl) -> T {
    if constexpr (sizeof(T) == 4) return dppf<decltype(ctrl)::value>(y);
    else return dppd<decltype(ctrl)::value>(y);
  };
  if constexpr (LVL == 0) return mv(x, std::integral_constant<int, 0xB1>{});
  else if constexpr (LVL == 1) return mv(x, std::integral_constant<int, 0x4E>{});
  else if constexpr (LVL == 2) {
    const T up = mv(x, std::integral_constant<int, 0x104>{}), dn = mv(x, std::integral_constant<int, 0x114>{});
    return (lane & 4) ? dn : up;
  } else return mv(x, std::integral_constant<int, 0x128>{});
}
// Value of lane (lane ^ 16) or (lane ^ 32) through the gfx950 row swaps.
template <int BIT>
__device__ __forceinline__ unsigned lane_swap32(unsigned x, int lane) {
  if constexpr (BIT == 16) {
    const auto r = __builtin_amdgcn_permlane16_swap(x, x, false, false);
    return (lane & 16) ? r[0] : r[1];
  } else {
    const auto r = __builtin_amdgcn_permlane32_swap(x, x, false, false);
    return (lane & 32) ? r[0] : r[1];
  }
}
template <int BIT>
__device__ __forceinline__ float lane_swap(float x, int lane) {
  return __uint_as_float(lane_swap32<BIT>(__float_as_uint(x), lane));
}
template <int BIT>
__device__ __forceinline__ double lane_swap(double x, int lane) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(x);
  const unsigned lo = lane_swap32<BIT>((unsigned)b, lane), hi = lane_swap32<BIT>((unsigned)(b >> 32), lane);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

constexpr int td_pow2(int x) { return x <= 1 ? 1 : 2 * td_pow2((x + 1) / 2); }
constexpr int td_log2(int x) { return x <= 1 ? 0 : 1 + td_log2(x / 2); }
// Largest divisor of x that is at most m (the gather's batch: whole batches only).
constexpr int td_batch(int x, int m) { return m <= 1 ? 1 : (x % m == 0 ? m : td_batch(x, m - 1)); }

template <int LVL, int NP, typename T>
__device__ __forceinline__ void td_halve(T (&w)[NP], int lane) {
  constexpr int half = NP >> (LVL + 1);
  const bool up = (lane & (1 << LVL)) != 0;
#pragma unroll
  for (int j = 0; j < half; ++j) {
    T lo = w[j], hi = w[j + half];
    asm volatile("" : "+v"(lo), "+v"(hi));   // keep both halves in registers (no runtime index into w)
    const T send = up ? lo : hi, keep = up ? hi : lo;
    w[j] = keep + lane_xor<LVL>(send, lane);
  }
}

// Sum NV <= 16 FP32 values over the workgroup (kThr threads) with one barrier; every thread gets
// the totals.  Inside a 16-lane row the NV values are summed by halving exchanges (lane l then
// holds value bitrev(l)), the row swaps add the wave's four rows, row 0 of each wave writes its
// sums to lds[par], and after the barrier every thread adds the waves' sums in wave order.
template <int NV, int kThr, typename T>
__device__ __forceinline__ void td_block_sum(T (&v)[NV], T* lds2, int& par, T (&tot)[NV]) {
  constexpr int NP = td_pow2(NV), K = td_log2(NP), kW = kThr / 64;
  static_assert(NP <= 16, "at most 16 values");
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  T* lds = lds2 + par * kW * 16;
  par ^= 1;
  T w[NP];
#pragma unroll
  for (int j = 0; j < NP; ++j) w[j] = j < NV ? v[j] : T(0);
  if constexpr (K > 0) td_halve<0, NP>(w, lane);
  if constexpr (K > 1) td_halve<1, NP>(w, lane);
  if constexpr (K > 2) td_halve<2, NP>(w, lane);
  if constexpr (K > 3) td_halve<3, NP>(w, lane);
  T x = w[0];
  if constexpr (K <= 0) x += lane_xor<0>(x, lane);
  if constexpr (K <= 1) x += lane_xor<1>(x, lane);
  if constexpr (K <= 2) x += lane_xor<2>(x, lane);
  if constexpr (K <= 3) x += lane_xor<3>(x, lane);
  x += lane_swap<16>(x, lane);
  x += lane_swap<32>(x, lane);
  if (lane < NP) {
    int idx = 0;
#pragma unroll
    for (int lvl = 0; lvl < K; ++lvl)
      if (lane & (1 << lvl)) idx += NP >> (lvl + 1);
    if (idx < NV) lds[wave * 16 + idx] = x;
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    T sacc = T(0);
#pragma unroll
    for (int q = 0; q < kW; ++q) sacc += lds[q * 16 + j];
    tot[j] = sacc;
  }
}

// Sum of one FP64 value over the workgroup (one barrier).
template <int kThr>
__device__ __forceinline__ double td_block_sum_d(double x, double* lds2, int& par) {
  constexpr int kW = kThr / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double* lds = lds2 + par * kW;
  par ^= 1;
  x += lane_xor<0>(x, lane);
  x += lane_xor<1>(x, lane);
  x += lane_xor<2>(x, lane);
  x += lane_xor<3>(x, lane);
  x += lane_swap<16>(x, lane);
  x += lane_swap<32>(x, lane);
  if (lane == 0) lds[wave] = x;
  __syncthreads();
  double sacc = 0.0;
#pragma unroll
  for (int q = 0; q < kW; ++q) sacc += lds[q];
  return sacc;
}

// ---- the reduction with the working rows in registers (n <= kCols * kThr, n <= kRows * G) -------
// Thread t holds column j = q kThr + t (q < kCols) of each own row and of v, p and the published
// row; LDS copies of v and p (two of each, by column parity) serve the few entries other threads
// need (v(i), w(i) of the own rows, p(k+1)).
// The rank-2 update of column k is applied one column late, off the dependency chain: the rows
// enter column k + 1 as B_k (updated through column k - 1) and its product is formed as
//   B_(k+1) u_(k+1) = B_k u_(k+1) - v_k (w_k^T u_(k+1)) - w_k (v_k^T u_(k+1)),
// the two scalars coming out of the workgroup sum that already yields the new reflector's norm.
// Per column: the owner of row k+1 publishes it (the pending update applied on the fly), one
// workgroup sum gives the own entries of p, which are published; the pending rank-2 update of the
// own rows then runs while the other workgroups publish; the gather brings p and the row, one sum
// gives p^T v, and one sum gives the norm of the next reflector's vector and the two scalars.
template <typename TA, int kThr, int kRows, int kCols, typename TS>
__global__ __launch_bounds__(kThr) void sytrd_reg_kernel(const TA* __restrict__ A, int lda, TdArgs a) {
  constexpr int kW = kThr / 64;
  __shared__ float vL[2][kCols * kThr];
  __shared__ float pL[2][kCols * kThr];
  __shared__ TS redf[2 * kW * 16];
  __shared__ double redd[2 * kW * 16];
  __shared__ float bc[2];
  __shared__ int bad_any[2];
  const int n = a.n, G = a.G, wg = blockIdx.x, t = threadIdx.x;
  const int nr = (n - wg + G - 1) / G;
  int fpar = 0, dpar = 0;
  TS R[kRows][kCols];
  float vq[kCols], pq[kCols], rq[kCols];
  float vp[kCols], wp[kCols];   // v and w of the pending update (column k - 1), own columns
#pragma unroll
  for (int r = 0; r < kRows; ++r) {
    const int i = wg + r * G;
#pragma unroll
    for (int q = 0; q < kCols; ++q) {
      const int j = q * kThr + t;
      R[r][q] = (r < nr && j < n) ? (TS)(float)A[j + (size_t)i * lda] : TS(0);
    }
  }
#pragma unroll
  for (int q = 0; q < kCols; ++q) {
    const int j = q * kThr + t;
    rq[q] = j < n ? (float)A[j] : 0.f;
    vp[q] = 0.f;
    wp[q] = 0.f;
  }
  if (t < 2) bad_any[t] = 0;
  // reflector of row k (entries of rq at j >= k+1): vq, vL[k & 1], tau, beta; with corr, also
  // al_w = w^T u_k and al_v = v^T u_k for the v = vq, w = pq - cw vq of column k - 1 (read before vq
  // is overwritten; their entries k+1 come from the LDS copies of column k - 1); uniform results
  float tauk = 0.f, beta = 0.f, cp = 0.f;
  double al_w = 0.0, al_v = 0.0;
  auto reflect = [&](int k, bool corr, float cw) {
    double part[3] = {0.0, 0.0, 0.0}, tot3[3];
#pragma unroll
    for (int q = 0; q < kCols; ++q) {
      const int j = q * kThr + t;
      if (j >= k + 2 && j < n) {
        const double x = (double)rq[q];
        part[0] += x * x;
        if (corr) {
          part[1] += (double)(pq[q] - cw * vq[q]) * x;
          part[2] += (double)vq[q] * x;
        }
      }
      if (j == k + 1) bc[dpar] = rq[q];
    }
    const int slot = dpar;
    td_block_sum<3, kThr, double>(part, redd, dpar, tot3);
    const double tail = tot3[0];
    const float alpha = bc[slot];
    float scal = 0.f;
    if (tail == 0.0) {
      tauk = 0.f;
      beta = alpha;
    } else {
      const double al = (double)alpha;
      const double rr = sqrt(al * al + tail);
      const double b = al >= 0.0 ? -rr : rr;
      tauk = (float)((b - al) / b);
      beta = (float)b;
      scal = (float)(1.0 / (al - b));
    }
    if (corr) {   // u_k = e_(k+1) + scal x(k+2:)
      const int pk = (k - 1) & 1;
      const float v1 = vL[pk][k + 1];
      al_v = (double)v1 + (double)scal * tot3[2];
      al_w = (double)(pL[pk][k + 1] - cw * v1) + (double)scal * tot3[1];
    } else {
      al_v = 0.0;
      al_w = 0.0;
    }
#pragma unroll
    for (int q = 0; q < kCols; ++q) {
      const int j = q * kThr + t;
      vq[q] = j == k + 1 ? 1.f : (j > k + 1 && j < n ? rq[q] * scal : 0.f);
      vL[k & 1][q * kThr + t] = vq[q];
    }
    if (wg == k % G) {   // the write-out rotates over the workgroups (none lags behind the others)
      if (t == 0) { a.e[k] = beta; a.tau[k] = tauk; }
      double* Uc = a.U + (size_t)k * a.ldu;
#pragma unroll
      for (int q = 0; q < kCols; ++q) {
        const int j = q * kThr + t;
        if (j < n) Uc[j] = vq[q];
        if (j == k) a.d[k] = rq[q];
      }
    }
  };
  reflect(0, false, 0.f);
  bool bad = false;
  for (int k = 0; k + 2 < n; ++k) {
    const unsigned tag = (unsigned)k + 1u;
    const int par = k & 1, pp = par ^ 1;   // LDS copies: column k, column k - 1
    unsigned long long* pb = a.pbuf + (size_t)par * n;
    unsigned long long* rb = a.rbuf + (size_t)par * n;
    // the owner of row k+1 publishes it, current through column k - 1 (the pending update of
    // column k - 1 applied on the fly; for k = 0 vp = wp = 0)
    if ((k + 1) % G == wg) {
      const int r1 = (k + 1 - wg) / G;
      const float vi = k > 0 ? vL[pp][k + 1] : 0.f;
      const float wi = k > 0 ? pL[pp][k + 1] - cp * vi : 0.f;
#pragma unroll
      for (int r = 0; r < kRows; ++r)
        if (r == r1) {
#pragma unroll
          for (int q = 0; q < kCols; ++q) {
            const int j = q * kThr + t;
            if (j > k && j < n) {
              const TS x = R[r][q] - ((TS)vi * (TS)wp[q] + (TS)wi * (TS)vp[q]);
              __hip_atomic_store(rb + j, td_pack(tag, (float)x), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
          }
        }
    }
    // (1) p(i) = tau B_k(i, :) u_k for the own rows i > k, from the rows B_(k-1) and the pending
    // update's scalars (u_k is zero at j <= k)
    TS acc[kRows], tot[kRows];
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
      acc[r] = TS(0);
#pragma unroll
      for (int q = 0; q < kCols; ++q) acc[r] = fma(R[r][q], (TS)vq[q], acc[r]);
    }
    td_block_sum<kRows, kThr, TS>(acc, redf, fpar, tot);
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
      const int i = wg + r * G;
      if (t == r && r < nr && i > k) {
        const float vi = k > 0 ? vL[pp][i] : 0.f;
        const float wi = k > 0 ? pL[pp][i] - cp * vi : 0.f;
        const TS pi = tot[r] - ((TS)vi * (TS)al_w + (TS)wi * (TS)al_v);
        __hip_atomic_store(pb + i, td_pack(tag, (float)((TS)tauk * pi)), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    if (t == 0) __hip_atomic_store(a.hb + wg, tag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    // (1b) the pending update of column k - 1 on the own rows i > k, while the others publish:
    // B(i, j) -= v(i) w(j) + w(i) v(j)
    if (k > 0) {
#pragma unroll
      for (int r = 0; r < kRows; ++r) {
        const int i = wg + r * G;
        if (r < nr && i > k) {
          const float vi = vL[pp][i], wi = pL[pp][i] - cp * vL[pp][i];
#pragma unroll
          for (int q = 0; q < kCols; ++q)   // FP32 operands: in FP64 storage the products are exact
            R[r][q] = R[r][q] - ((TS)vi * (TS)wp[q] + (TS)wi * (TS)vp[q]);
        }
      }
    }
    // (2) gather p(k+1:) and row k+1 in batches of up to 8 columns (a divisor of kCols): every
    // load of a batch is issued before any of its tags is tested
    float spart = 0.f;
    constexpr int kGB = td_batch(kCols, 8);
    static_assert(kCols % kGB == 0, "whole batches");
#pragma unroll
    for (int q0 = 0; q0 < kCols; q0 += kGB) {
      unsigned long long xp[kGB], xr[kGB];
#pragma unroll
      for (int u = 0; u < kGB; ++u) {
        const int j = (q0 + u) * kThr + t;
        if (j > k && j < n) {
          xp[u] = __hip_atomic_load(pb + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          xr[u] = __hip_atomic_load(rb + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
#pragma unroll
      for (int u = 0; u < kGB; ++u) {
        const int q = q0 + u, j = q * kThr + t;
        if (j > k && j < n) {
          pq[q] = (unsigned)(xp[u] >> 32) == tag ? __uint_as_float((unsigned)xp[u]) : td_wait(pb, j, tag, a.abort, bad, 0);
          rq[q] = (unsigned)(xr[u] >> 32) == tag ? __uint_as_float((unsigned)xr[u]) : td_wait(rb, j, tag, a.abort, bad, 1);
        } else {
          pq[q] = 0.f;
          rq[q] = 0.f;
        }
        pL[par][q * kThr + t] = pq[q];
        spart = fmaf(pq[q], vq[q], spart);
      }
    }
    // Column k + 1 reuses the buffers of column k - 1 (its parity): every workgroup must have read
    // them, i.e. published p for column k.  While k + G < n every workgroup owns a row > k, whose
    // entry of p this gather has just seen, so only the last G columns need the heartbeats.
    if (k + G >= n && t < G) td_wait_hb(a.hb + t, tag, a.abort, bad);
    if (bad) bad_any[par] = 1;
    // (3) s = p^T v (one workgroup sum), w = p - (tau s / 2) v
    TS sv[1] = {(TS)spart}, st[1];
    td_block_sum<1, kThr, TS>(sv, redf, fpar, st);
    if (bad_any[par]) break;
    if (t == 0) bad_any[par ^ 1] = 0;
    const float c = (float)(TS(0.5f * tauk) * st[0]);
    // (4) row k+1 of the updated matrix (v(k+1) = 1), then its reflector; column k's update
    // becomes the pending one
    const float wk1 = pL[par][k + 1] - c;
#pragma unroll
    for (int q = 0; q < kCols; ++q) rq[q] = rq[q] - ((pq[q] - c * vq[q]) + wk1 * vq[q]);
    if (k + 3 < n) {
      reflect(k + 1, true, c);
#pragma unroll
      for (int q = 0; q < kCols; ++q) {   // (vq was overwritten; its old values are in the LDS copy)
        const float v = vL[par][q * kThr + t];
        vp[q] = v;
        wp[q] = pq[q] - c * v;
      }
      cp = c;
    } else {
      if (wg == (n - 2) % G) {
#pragma unroll
        for (int q = 0; q < kCols; ++q) {
          const int j = q * kThr + t;
          if (j == n - 2) a.d[n - 2] = rq[q];
          if (j == n - 1) a.e[n - 2] = rq[q];
        }
      }
      if ((n - 1) % G == wg) {   // entry (n-1, n-1): rows through column n - 4, then column n - 3's update
        const int r1 = (n - 1 - wg) / G;
#pragma unroll
        for (int r = 0; r < kRows; ++r)
#pragma unroll
          for (int q = 0; q < kCols; ++q)
            if (r == r1 && q * kThr + t == n - 1) {
              const float w = pq[q] - c * vq[q];
              a.d[n - 1] = (float)(R[r][q] - ((TS)vq[q] * (TS)w + (TS)w * (TS)vq[q]));
            }
      }
    }
  }
}

// n <= 2: T is A itself.
template <typename TA>
__global__ void sytrd_small_kernel(const TA* A, int lda, int n, double* d, double* e) {
  if (threadIdx.x != 0) return;
  d[0] = (float)A[0];
  if (n == 2) { e[0] = (float)A[1]; d[1] = (float)A[1 + lda]; }
}

// ---------------------------------------------------------------- eigenvalues
// bnd: [0] lower Gershgorin bound, [1] upper, [2] pivmin (smallest pivot magnitude allowed).
__global__ __launch_bounds__(256) void tri_bounds_kernel(const double* d, const double* e, int n, double* bnd) {
  __shared__ double lo[256], hi[256], em[256];
  const int t = threadIdx.x;
  double l = HUGE_VAL, h = -HUGE_VAL, m = 1.0;
  for (int i = t; i < n; i += 256) {
    const double r = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < n ? fabs(e[i]) : 0.0);
    l = fmin(l, d[i] - r);
    h = fmax(h, d[i] + r);
    if (i + 1 < n) m = fmax(m, e[i] * e[i]);
  }
  lo[t] = l; hi[t] = h; em[t] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) {
      lo[t] = fmin(lo[t], lo[t + s]);
      hi[t] = fmax(hi[t], hi[t + s]);
      em[t] = fmax(em[t], em[t + s]);
    }
    __syncthreads();
  }
  if (t == 0) {
    const double span = hi[0] - lo[0];
    bnd[0] = lo[0] - 4.0 * 2.220446049250313e-16 * span - 1e-300;
    bnd[1] = hi[0] + 4.0 * 2.220446049250313e-16 * span + 1e-300;
    bnd[2] = 2.2250738585072014e-308 * em[0];
  }
}

// Number of eigenvalues below x: the sign changes of the Sturm sequence of T - x I, i.e. of the
// leading principal minors m_i = (d_i - x) m_(i-1) - e_(i-1)^2 m_(i-2) (m_0 = 1, m_(-1) = 0); the
// ratio m_i / m_(i-1) is the i-th pivot of the LDL^T factorization, so a sign change is a
// negative pivot.  No division: every 16 steps both kept minors are scaled by the same power of
// two (exact), and a zero minor is replaced by -pivmin times its predecessor (a pivot of -pivmin).
__device__ __forceinline__ int sturm_count(const double* __restrict__ d, const double* __restrict__ e2, int n16,
                                           double x, double pivmin) {
  // d, e2: n16 (a multiple of 16) entries, padded past n with d = (above every eigenvalue),
  // e^2 = 0, which add positive pivots and no sign change
  double m1 = 1.0, m0 = 0.0;   // m_(i-1), m_(i-2)
  double em = 0.0;             // e_(i-1)^2 (zero before the first row)
  int c = 0;
  for (int i0 = 0; i0 < n16; i0 += 16) {
    double dd[16], ee[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      dd[u] = d[i0 + u];
      ee[u] = e2[i0 + u];
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      double m = fma(dd[u] - x, m1, -em * m0);
      if (m == 0.0) m = -pivmin * m1;
      c += (m < 0.0) != (m1 < 0.0);
      m0 = m1;
      m1 = m;
      em = ee[u];
    }
    int ex;
    (void)frexp(fabs(m1) + fabs(m0), &ex);
    m1 = ldexp(m1, -ex);
    m0 = ldexp(m0, -ex);
  }
  return c;
}

constexpr int kBisThreads = 256;    // 8 eigenvalues per workgroup (one per 32 lanes), sharing one LDS copy of d, e^2
constexpr int kBisLanes = 32;       // points per eigenvalue and round

// kBisLanes lanes per eigenvalue index k: their Sturm counts narrow the interval holding the k-th
// smallest eigenvalue (kBisLanes + 1)-fold per round, until it spans no more than a few units of
// roundoff.
__global__ __launch_bounds__(kBisThreads) void tri_bisect_kernel(const double* __restrict__ d,
                                                                const double* __restrict__ e, int n,
                                                                const double* __restrict__ bnd,
                                                                double* __restrict__ w) {
  extern __shared__ double bis_smem[];
  const int n16 = (n + 15) / 16 * 16;
  double* sd = bis_smem;
  double* se2 = bis_smem + n16;
  const double dpad = bnd[1] + 1.0 + fabs(bnd[1]);
  for (int i = threadIdx.x; i < n16; i += kBisThreads) {
    sd[i] = i < n ? d[i] : dpad;
    se2[i] = i + 1 < n ? e[i] * e[i] : 0.0;
  }
  __syncthreads();
  const int k = blockIdx.x * (kBisThreads / kBisLanes) + (threadIdx.x / kBisLanes);
  const int lane = threadIdx.x & (kBisLanes - 1);
  const int half = (threadIdx.x & 63) & ~(kBisLanes - 1);   // first lane of this group in the wave
  const bool live = k < n;
  double lo = bnd[0], hi = bnd[1];
  const double pivmin = bnd[2];
  bool done = !live;
  for (int round = 0; round < 24; ++round) {
    const double width = hi - lo;
    if (width <= 4.0 * 1.1102230246251565e-16 * fmax(fabs(lo), fabs(hi)) + pivmin) done = true;
    // both groups of a wave run every round (ballot / shuffle span the wave); finished ones idle
    if (__all(done)) break;
    const double x = lo + width * (double)(lane + 1) / (double)(kBisLanes + 1);
    const bool below = !done && sturm_count(sd, se2, n16, x, pivmin) <= k;   // the k-th eigenvalue is >= x
    const unsigned long long m = (__ballot(below) >> half) & ((1ull << kBisLanes) - 1);
    const int hb = m ? 63 - __clzll(m) : -1;                       // last point with count <= k
    const double xl = __shfl(x, half + (hb < 0 ? 0 : hb), 64);
    const double xh = __shfl(x, half + (hb + 1 > kBisLanes - 1 ? kBisLanes - 1 : hb + 1), 64);
    if (!done) {
      const double nlo = hb < 0 ? lo : xl;
      const double nhi = hb >= kBisLanes - 1 ? hi : xh;
      if (!(nlo > lo || nhi < hi)) done = true;   // the points no longer split the interval
      else { lo = nlo; hi = nhi; }
    }
  }
  if (live && lane == 0) w[k] = 0.5 * (lo + hi);
}

// ---------------------------------------------------------------- eigenvectors
// Eigenvector of T for w[c0 + c], c < nc, from the twisted factorization of T - lambda I:
// forward pivots dp(i) of the LDL^T factorization, backward pivots dm(i) of the UDU^T one, twisted
// pivot g(i) = dp(i) + dm(i) - (d(i) - lambda); at the twist r = argmin |g|, z(r) = 1 and
// z(i) = -e(i) z(i+1) / dp(i) above, z(i) = -e(i-1) z(i-1) / dm(i) below; then z / ||z||.
// Scratch dp, dm: n x nc each (entry i of eigenvector c at i * nc + c), read back in prefetched
// chunks of kPre entries so that their loads do not sit in the recurrence's dependency chain;
// d and e come from an LDS copy.  Y column c0 + c receives z.
constexpr int kVecThreads = 64;
constexpr int kPre = 32;

template <typename TY>
__global__ __launch_bounds__(kVecThreads) void tri_vectors_kernel(const double* __restrict__ d,
                                                                 const double* __restrict__ e, int n,
                                                                 const double* __restrict__ w,
                                                                 const double* __restrict__ bnd, int c0, int nc,
                                                                 double* __restrict__ dp, double* __restrict__ dm,
                                                                 TY* __restrict__ Y, int ldy) {
  extern __shared__ double vec_smem[];
  double* sd = vec_smem;
  double* se = vec_smem + n;
  for (int i = threadIdx.x; i < n; i += kVecThreads) {
    sd[i] = d[i];
    se[i] = i + 1 < n ? e[i] : 0.0;
  }
  __syncthreads();
  const int c = blockIdx.x * kVecThreads + threadIdx.x;
  if (c >= nc) return;
  const double lam = w[c0 + c];
  const double pivmin = bnd[2];
  double q = sd[0] - lam;
  if (fabs(q) < pivmin) q = -pivmin;
  dp[c] = q;
  for (int i = 1; i < n; ++i) {
    q = (sd[i] - lam) - se[i - 1] * se[i - 1] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    dp[(size_t)i * nc + c] = q;
  }
  double qm = sd[n - 1] - lam;
  if (fabs(qm) < pivmin) qm = -pivmin;
  dm[(size_t)(n - 1) * nc + c] = qm;
  int r = n - 1;
  double best = fabs(q);   // g(n-1) = dp(n-1)
  for (int hi = n - 2; hi >= 0; hi -= kPre) {
    double pre[kPre];
#pragma unroll
    for (int u = 0; u < kPre; ++u) pre[u] = hi - u >= 0 ? dp[(size_t)(hi - u) * nc + c] : 0.0;
#pragma unroll
    for (int u = 0; u < kPre; ++u) {
      const int i = hi - u;
      if (i >= 0) {
        qm = (sd[i] - lam) - se[i] * se[i] / qm;
        if (fabs(qm) < pivmin) qm = -pivmin;
        dm[(size_t)i * nc + c] = qm;
        const double g = fabs(pre[u] + qm - (sd[i] - lam));
        if (g < best) { best = g; r = i; }
      }
    }
  }
  // outward solve; z(i) overwrites the pivot it consumed
  double nrm2 = 1.0, z = 1.0;
  for (int hi = r - 1; hi >= 0; hi -= kPre) {
    double pre[kPre];
#pragma unroll
    for (int u = 0; u < kPre; ++u) pre[u] = hi - u >= 0 ? dp[(size_t)(hi - u) * nc + c] : 1.0;
#pragma unroll
    for (int u = 0; u < kPre; ++u) {
      const int i = hi - u;
      if (i >= 0) {
        z = -se[i] * z / pre[u];
        dp[(size_t)i * nc + c] = z;
        nrm2 += z * z;
      }
    }
  }
  z = 1.0;
  for (int lo = r + 1; lo < n; lo += kPre) {
    double pre[kPre];
#pragma unroll
    for (int u = 0; u < kPre; ++u) pre[u] = lo + u < n ? dm[(size_t)(lo + u) * nc + c] : 1.0;
#pragma unroll
    for (int u = 0; u < kPre; ++u) {
      const int i = lo + u;
      if (i < n) {
        z = -se[i - 1] * z / pre[u];
        dm[(size_t)i * nc + c] = z;
        nrm2 += z * z;
      }
    }
  }
  const double inv = 1.0 / sqrt(nrm2);
  TY* y = Y + (size_t)(c0 + c) * ldy;
  for (int lo = 0; lo < n; lo += kPre) {
    double pre[kPre];
#pragma unroll
    for (int u = 0; u < kPre; ++u) {
      const int i = lo + u;
      pre[u] = i < r ? dp[(size_t)i * nc + c] : (i == r ? 1.0 : (i < n ? dm[(size_t)i * nc + c] : 0.0));
    }
#pragma unroll
    for (int u = 0; u < kPre; ++u)
      if (lo + u < n) y[lo + u] = (TY)(pre[u] * inv);
  }
}

// ---------------------------------------------------------------- back-transformation
// For reflector block b (reflectors k0 = b kBtNb ...), the triangular factor Tb with
// H_k0 ... H_(k0+NB-1) = I - Ub Tb Ub^T, from the block's Gram G = Ub^T Ub (computed beforehand on
// the matrix cores, column-major NB x NB per block).  The four diagonal 32 x 32 blocks of Tb follow
// column by column from Tb(i,i) = tau_i, Tb(0:i, i) = -tau_i Tb(0:i, 0:i) G(0:i, i) (all four at
// once); the off-diagonal blocks from joining two factors, [[Ta, -Ta Gab Tb], [0, Tb]], first
// pairwise (32 | 32) then (64 | 64), each product formed in the still-zero upper-right block.
__global__ __launch_bounds__(256) void bt_tfactor_kernel(const double* __restrict__ Gall, const float* __restrict__ tau,
                                                        int nref, double* __restrict__ Tall) {
  constexpr int NB = kBtNb, LD = NB + 1;
  static_assert(NB == 128, "block layout assumes 128 reflectors per block");
  extern __shared__ __align__(16) unsigned char bt_smem[];
  double* Ts = reinterpret_cast<double*>(bt_smem);   // NB x LD, Ts[a * LD + c]
  const int b = blockIdx.x, t = threadIdx.x, k0 = b * NB;
  const double* G = Gall + (size_t)b * NB * NB;     // G(a, c) = G[a + c * NB]
  for (int q = t; q < NB * LD; q += 256) Ts[q] = 0.0;
  __syncthreads();
  const int blk = t >> 5, l = t & 31;
  for (int i = 0; i < 32; ++i) {
    double yv = 0.0;
    if (t < 128) {
      const int base = blk * 32, col = base + i;
      const double ti = (k0 + col < nref) ? (double)tau[k0 + col] : 0.0;
      if (l < i) {
        double sacc = 0.0;
        for (int cc = l; cc < i; ++cc) sacc = fma(Ts[(base + l) * LD + base + cc], G[(base + cc) + (size_t)col * NB], sacc);
        yv = -ti * sacc;
      } else if (l == i) {
        yv = ti;
      }
    }
    __syncthreads();
    if (t < 128 && l <= i) Ts[(blk * 32 + l) * LD + blk * 32 + i] = yv;
    __syncthreads();
  }
  for (int lvl = 0; lvl < 2; ++lvl) {
    const int p = lvl == 0 ? 32 : 64;
    const int npairs = lvl == 0 ? 2 : 1;
    for (int pr = 0; pr < npairs; ++pr) {
      const int oa = pr * 2 * p, ob = oa + p;
      // M = Gab Tb into the (zero) upper-right block
      for (int q = t; q < p * p; q += 256) {
        const int x = q / p, y = q % p;
        double sacc = 0.0;
        for (int cc = 0; cc <= y; ++cc) sacc = fma(G[(oa + x) + (size_t)(ob + cc) * NB], Ts[(ob + cc) * LD + ob + y], sacc);
        Ts[(oa + x) * LD + ob + y] = sacc;
      }
      __syncthreads();
      // X = -Ta M, through registers (every entry of X reads a column of M)
      double xr[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int q = t + u * 256;
        xr[u] = 0.0;
        if (q < p * p) {
          const int x = q / p, y = q % p;
          double sacc = 0.0;
          for (int cc = x; cc < p; ++cc) sacc = fma(Ts[(oa + x) * LD + oa + cc], Ts[(oa + cc) * LD + ob + y], sacc);
          xr[u] = -sacc;
        }
      }
      __syncthreads();
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int q = t + u * 256;
        if (q < p * p) Ts[(oa + q / p) * LD + ob + q % p] = xr[u];
      }
      __syncthreads();
    }
  }
  double* Tb = Tall + (size_t)b * NB * NB;   // column-major NB x NB
  for (int q = t; q < NB * NB; q += 256) Tb[q] = Ts[(q % NB) * LD + q / NB];
}

// B (cols x rows block, ldb) = A^T for an m x n block of A (lda), 32 x 32 tiles through LDS.
template <typename T>
__global__ void td_transpose_kernel(const T* __restrict__ A, int lda, int m, int n, T* __restrict__ B, int ldb) {
  __shared__ T tl[32][33];
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int r = ty; r < 32; r += 8) {
    const int i = bx + tx, j = by + r;
    if (i < m && j < n) tl[r][tx] = A[i + (size_t)j * lda];
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int i = by + tx, j = bx + r;   // B(i, j) = A(j, i)
    if (i < n && j < m) B[i + (size_t)j * ldb] = tl[tx][r];
  }
}

__global__ void td_fill_u64_kernel(unsigned long long* p, long long count) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = 0ull;
}

__global__ void td_fill_f32_kernel(float* p, long long count) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = 0.f;
}

// ---------------------------------------------------------------- host side
// Above the register-resident range the working rows live in a private global slice.
static int td_rows_in_lds(int n) { return n <= kTdRegMaxN; }

static int td_nbp(int n) {
  const int nref = n > 2 ? n - 2 : 0;
  const int nb = nref > 0 ? tcdiv(nref, kBtNb) : 1;
  return nb * kBtNb;
}

// Workspace of the pieces (eig_tridiag_f32 takes all of them).
struct TdWork {
  unsigned long long *pbuf, *rbuf;
  unsigned* hb;
  int* abort;
  double *bnd, *d, *e, *w;
  float *tau, *rows;
  double *U, *Ut, *Y, *G, *Tf, *Wb, *W2;
  double *dp, *dm;
  int nbp, nc;
};

static TdWork td_carve(Carve& c, int n) {
  TdWork k;
  k.nbp = td_nbp(n);
  k.nc = n < kVecChunk ? n : kVecChunk;
  k.pbuf = c.take<unsigned long long>((size_t)2 * n);
  k.rbuf = c.take<unsigned long long>((size_t)2 * n);
  k.hb = c.take<unsigned>(kTdMaxG);
  k.abort = c.take<int>(8);
  k.bnd = c.take<double>(4);
  k.d = c.take<double>(n);
  k.e = c.take<double>(n);
  k.w = c.take<double>(n);
  k.tau = c.take<float>(k.nbp);
  k.U = c.take<double>((size_t)k.nbp * n);
  k.Ut = c.take<double>((size_t)k.nbp * n);
  k.Y = c.take<double>((size_t)n * n);
  k.dp = c.take<double>((size_t)n * k.nc);
  k.dm = c.take<double>((size_t)n * k.nc);
  k.G = c.take<double>((size_t)k.nbp * kBtNb);
  k.Tf = c.take<double>((size_t)k.nbp * kBtNb);
  k.Wb = c.take<double>((size_t)kBtNb * n);
  k.W2 = c.take<double>((size_t)kBtNb * n);
  k.rows = td_rows_in_lds(n) ? nullptr : c.take<float>((size_t)n * n);
  return k;
}

size_t tridiag_bytes(int n) {
  if (n <= 0) return 0;
  Carve c(nullptr);
  (void)td_carve(c, n);
  return c.off + 16 * 256;
}

bool tridiag_supported(int n) { return n >= 1 && n <= kTdMaxN; }

template <typename TA, int kThr, int kRows, int kCols, typename TS>
static int td_launch_reg(const TA* A, int lda, TdArgs& a, hipStream_t s) {
  void* args[] = {(void*)&A, (void*)&lda, (void*)&a};
  auto kern = sytrd_reg_kernel<TA, kThr, kRows, kCols, TS>;
  JAC_HIP(hipLaunchCooperativeKernel((const void*)kern, dim3(a.G), dim3(kThr), args, 0u, s));
  return 0;
}

template <typename TA, bool kLds, int kMaxRows>
static int td_launch(const TA* A, int lda, TdArgs& a, hipStream_t s) {
  const size_t sh = ((kLds ? (size_t)kMaxRows * a.n : 0) + 3 * (size_t)a.n + (a.n & 1)) * 4 + 16 * 8 +
                    2 * kTdWaves * kMaxRows * 4 + 64;
  void* args[] = {(void*)&A, (void*)&lda, (void*)&a};
  auto kern = sytrd_kernel<TA, kLds, kMaxRows>;
  JAC_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh));
  JAC_HIP(hipLaunchCooperativeKernel((const void*)kern, dim3(a.G), dim3(kTdThreads), args, (unsigned)sh, s));
  return 0;
}

// Step 1a: d, e, tau and the reflectors (U: column k = u_k, ld n; Ut: row k = u_k, ld nbp).
template <typename TA>
static int td_reduce(const TA* A, int n, int lda, TdWork& k, hipStream_t s) {
  hipLaunchKernelGGL(td_fill_u64_kernel, dim3(64), dim3(256), 0, s, k.pbuf, (long long)2 * n);
  JAC_CHECK_LAUNCH();
  hipLaunchKernelGGL(td_fill_u64_kernel, dim3(64), dim3(256), 0, s, k.rbuf, (long long)2 * n);
  JAC_CHECK_LAUNCH();
  hipLaunchKernelGGL(td_fill_u64_kernel, dim3(1), dim3(64), 0, s, reinterpret_cast<unsigned long long*>(k.abort), 4ll);
  JAC_CHECK_LAUNCH();
  hipLaunchKernelGGL(td_fill_u64_kernel, dim3(1), dim3(256), 0, s, reinterpret_cast<unsigned long long*>(k.hb),
                     (long long)kTdMaxG / 2);
  JAC_CHECK_LAUNCH();
  hipLaunchKernelGGL(td_fill_u64_kernel, dim3(1024), dim3(256), 0, s, reinterpret_cast<unsigned long long*>(k.U),
                     (long long)k.nbp * n);
  JAC_CHECK_LAUNCH();
  hipLaunchKernelGGL(td_fill_u64_kernel, dim3(1024), dim3(256), 0, s, reinterpret_cast<unsigned long long*>(k.Ut),
                     (long long)k.nbp * n);
  JAC_CHECK_LAUNCH();
  hipLaunchKernelGGL(td_fill_f32_kernel, dim3(1), dim3(256), 0, s, k.tau, (long long)k.nbp);
  JAC_CHECK_LAUNCH();
  if (n <= 2) {
    hipLaunchKernelGGL((sytrd_small_kernel<TA>), dim3(1), dim3(64), 0, s, A, lda, n, k.d, k.e);
    JAC_CHECK_LAUNCH();
    return 0;
  }
  TdArgs a;
  a.n = n;
  a.G = n < kTdMaxG ? n : kTdMaxG;
  a.rows = k.rows;
  a.pbuf = k.pbuf;
  a.rbuf = k.rbuf;
  a.hb = k.hb;
  a.d = k.d;
  a.e = k.e;
  a.tau = k.tau;
  a.U = k.U;
  a.ldu = n;
  a.Ut = k.Ut;
  a.ldut = k.nbp;
  a.abort = k.abort;
  // One 256-thread workgroup per CU (one wave per SIMD) leaves each wave the whole register file
  // (VGPRs and AGPRs): the rows stay in FP64 up to n = 2048 and in FP32 above, where a thread holds
  // up to 16 x 16 entries.  512-thread workgroups (two waves per SIMD, half the registers each)
  // spill at n = 4096 and are slower at n <= 2048.
  int rc;
  if (n <= 1024) rc = td_launch_reg<TA, 256, 4, 4, double>(A, lda, a, s);
  else if (n <= 2048) rc = td_launch_reg<TA, 256, 8, 8, double>(A, lda, a, s);
  else if (n <= 3072) rc = td_launch_reg<TA, 256, 12, 12, float>(A, lda, a, s);
  else if (n <= 4096) rc = td_launch_reg<TA, 256, 16, 16, float>(A, lda, a, s);
  else return td_launch<TA, false, kTdGlbRows>(A, lda, a, s);   // writes Ut itself
  if (rc) return rc;
  // Ut = U^T for the back-transformation's untransposed products
  hipLaunchKernelGGL(td_transpose_kernel<double>, dim3(tcdiv(n, 32), tcdiv(n - 2, 32)), dim3(256), 0, s, k.U, n, n,
                     n - 2, k.Ut, k.nbp);
  JAC_CHECK_LAUNCH();
  return 0;
}

static int td_abort_check(const TdWork& k, hipStream_t s) {
  int hab[6] = {0, 0, 0, 0, 0, 0};
  JAC_HIP(hipMemcpyAsync(hab, k.abort, sizeof(hab), hipMemcpyDeviceToHost, s));
  JAC_HIP(hipStreamSynchronize(s));
  if (hab[0]) {
    set_error("tridiagonal FP32 stage: a workgroup of the cooperative reduction timed out (column tag " +
              std::to_string(hab[1]) + ", workgroup " + std::to_string(hab[2]) + ", entry " +
              std::to_string(hab[3]) +
              (hab[4] == 2 ? " (heartbeat)" : hab[4] == 1 ? " of the published row" : " of p") + ", last tag seen " +
              std::to_string(hab[5]) + ")");
    return 4;
  }
  return 0;
}

// Step 1b: eigenvalues w (ascending) of (d, e) by bisection.
static int td_eigvals(const double* d, const double* e, int n, double* bnd, double* w, hipStream_t s) {
  hipLaunchKernelGGL(tri_bounds_kernel, dim3(1), dim3(256), 0, s, d, e, n, bnd);
  JAC_CHECK_LAUNCH();
  const size_t bsh = (size_t)2 * ((n + 15) / 16 * 16) * sizeof(double);
  JAC_HIP(hipFuncSetAttribute((const void*)tri_bisect_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bsh));
  hipLaunchKernelGGL(tri_bisect_kernel, dim3(tcdiv(n, kBisThreads / kBisLanes)), dim3(kBisThreads), bsh, s, d, e, n, bnd,
                     w);
  JAC_CHECK_LAUNCH();
  return 0;
}

// Step 1c: eigenvectors of (d, e) for w into Y (n x n, ldy).
template <typename TY>
static int td_vectors(const double* d, const double* e, int n, const double* w, const double* bnd, double* dp,
                      double* dm, int nc, TY* Y, int ldy, hipStream_t s) {
  for (int c0 = 0; c0 < n; c0 += nc) {
    const int cnt = n - c0 < nc ? n - c0 : nc;
    const size_t vsh = (size_t)2 * n * sizeof(double);
    JAC_HIP(hipFuncSetAttribute((const void*)tri_vectors_kernel<TY>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)vsh));
    hipLaunchKernelGGL((tri_vectors_kernel<TY>), dim3(tcdiv(cnt, kVecThreads)), dim3(kVecThreads), vsh, s, d, e, n, w,
                       bnd, c0, cnt, dp, dm, Y, ldy);
    JAC_CHECK_LAUNCH();
  }
  return 0;
}

// Step 1d: Y (n x n, ld n) <- H_0 ... H_{n-3} Y, in FP64 on the matrix cores: per block of kBtNb
// reflectors its Gram Ub^T Ub and triangular factor Tb, then Y -= Ub (Tb Ub^T) Y.
// Step 1d, first part (it depends on the reflectors only): the Gram matrix and triangular factor
// of every reflector block, then the rows of Ut (Ub^T) replaced by Tb Ub^T, so that the second
// part needs two products per block instead of three.  Wb (kBtNb x n) is scratch.
static int td_bt_factors(const double* U, double* Ut, int nbp, const float* tau, int n, double* Gb, double* Tf,
                         double* Wb, hipStream_t s, bool no_split) {
  const int nref = n > 2 ? n - 2 : 0;
  if (nref == 0) return 0;
  const int nblk = tcdiv(nref, kBtNb);
  const int msplit = no_split ? 1 : 0;
  for (int b = 0; b < nblk; ++b) {
    const int k0 = b * kBtNb, r0 = k0 + 1, m = n - r0;
    int e1 = gemm<double>(false, false, kBtNb, kBtNb, m, 1.0, Ut + k0 + (size_t)r0 * nbp, nbp, U + r0 + (size_t)k0 * n,
                          n, 0.0, Gb + (size_t)b * kBtNb * kBtNb, kBtNb, s, msplit);
    if (e1) return e1;
  }
  const size_t tsh = (size_t)kBtNb * (kBtNb + 1) * sizeof(double);
  JAC_HIP(hipFuncSetAttribute((const void*)bt_tfactor_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)tsh));
  hipLaunchKernelGGL(bt_tfactor_kernel, dim3(nblk), dim3(256), tsh, s, Gb, tau, nref, Tf);
  JAC_CHECK_LAUNCH();
  for (int b = 0; b < nblk; ++b) {
    const int k0 = b * kBtNb, r0 = k0 + 1, m = n - r0;
    double* Utb = Ut + k0 + (size_t)r0 * nbp;
    int e1 = gemm<double>(false, false, kBtNb, m, kBtNb, 1.0, Tf + (size_t)b * kBtNb * kBtNb, kBtNb, Utb, nbp, 0.0, Wb,
                          kBtNb, s, msplit);
    if (!e1) e1 = copy_convert<double, double>(Wb, kBtNb, m, kBtNb, Utb, nbp, s);
    if (e1) return e1;
  }
  return 0;
}

// Step 1d, second part: Y <- H_0 ... H_{n-3} Y, block by block from the last (Ut holds Tb Ub^T).
static int td_bt_apply(const double* U, const double* Ut, int nbp, int n, double* W2, double* Y, hipStream_t s,
                       bool no_split) {
  const int nref = n > 2 ? n - 2 : 0;
  if (nref == 0) return 0;
  const int nblk = tcdiv(nref, kBtNb);
  const int msplit = no_split ? 1 : 0;
  for (int b = nblk - 1; b >= 0; --b) {
    const int k0 = b * kBtNb, r0 = k0 + 1, m = n - r0;
    int e1 = gemm<double>(false, false, kBtNb, n, m, 1.0, Ut + k0 + (size_t)r0 * nbp, nbp, Y + r0, n, 0.0, W2, kBtNb,
                          s, msplit);
    if (e1) return e1;
    e1 = gemm<double>(false, false, m, n, kBtNb, -1.0, U + r0 + (size_t)k0 * n, n, W2, kBtNb, 1.0, Y + r0, n, s,
                      msplit);
    if (e1) return e1;
  }
  return 0;
}

static int td_backtransform(const double* U, double* Ut, int nbp, const float* tau, int n, double* Gb,
                            double* Tf, double* Wb, double* W2, double* Y, hipStream_t s, bool no_split) {
  int e = td_bt_factors(U, Ut, nbp, tau, n, Gb, Tf, Wb, s, no_split);
  if (e) return e;
  return td_bt_apply(U, Ut, nbp, n, W2, Y, s, no_split);
}

// FP32 eigenvectors of A (n x n, FP64 or FP32, lda) through the tridiagonal route.  Z (FP64,
// n x n, ldz) receives them in ascending order of the eigenvalues of T, which go to w_out (FP64,
// may be NULL).  no_split: GEMMs without split-K (nothing allocated).
template <typename TA>
int eig_tridiag_f32(const TA* A, int n, int lda, double* Z, int ldz, double* w_out, Carve& c, hipStream_t s,
                    bool no_split, Prof* prof) {
  if (n <= 0) return 0;
  if (!tridiag_supported(n)) { set_error("tridiagonal FP32 stage: order above 8192"); return -2; }
  TdWork k = td_carve(c, n);
  const int ev0 = prof ? prof->mark(s) : -1;
  int e = td_reduce<TA>(A, n, lda, k, s);
  if (e) return e;
  const int ev1 = prof ? prof->mark(s) : -1;
  // The blocks' Gram matrices and triangular factors need only the reflectors: they run on a
  // second stream while the eigenvalues and eigenvectors of T take the first (the eigenvector
  // kernel fills few CUs).  Not for the allocation-free form (no_split), which creates nothing.
  hipStream_t s2 = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  auto release = [&]() {
    if (fork) (void)hipEventDestroy(fork);
    if (join) (void)hipEventDestroy(join);
    if (s2) (void)hipStreamDestroy(s2);
    fork = join = nullptr;
    s2 = nullptr;
  };
  auto hip_ok = [](hipError_t r, const char* what) {
    if (r == hipSuccess) return 0;
    set_error(std::string(what) + ": " + hipGetErrorString(r));
    return 4;
  };
  if (!no_split && n >= 512) {   // (if the second stream cannot be set up, one stream does it all)
    if (hipStreamCreateWithFlags(&s2, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&join, hipEventDisableTiming) != hipSuccess)
      release();
  }
  if (s2) {
    e = hip_ok(hipEventRecord(fork, s), "hipEventRecord");
    if (!e) e = hip_ok(hipStreamWaitEvent(s2, fork, 0), "hipStreamWaitEvent");
    if (e) { release(); return e; }
  }
  e = td_bt_factors(k.U, k.Ut, k.nbp, k.tau, n, k.G, k.Tf, k.Wb, s2 ? s2 : s, no_split);
  if (!e && s2) e = hip_ok(hipEventRecord(join, s2), "hipEventRecord");
  if (!e) e = td_eigvals(k.d, k.e, n, k.bnd, k.w, s);
  if (!e) e = td_vectors<double>(k.d, k.e, n, k.w, k.bnd, k.dp, k.dm, k.nc, k.Y, n, s);
  if (!e && s2) e = hip_ok(hipStreamWaitEvent(s, join, 0), "hipStreamWaitEvent");
  if (e) {
    if (s2) (void)hipStreamSynchronize(s2);
    release();
    return e;
  }
  e = td_bt_apply(k.U, k.Ut, k.nbp, n, k.W2, k.Y, s, no_split);
  release();   // (destroying a stream whose work is queued or waited on is allowed; it completes)
  if (e) return e;
  e = copy_convert<double, double>(k.Y, n, n, n, Z, ldz, s);
  if (e) return e;
  if (prof) {
    const int ev2 = prof->mark(s);
    prof->interval(6, ev0, ev1, 1);
    prof->interval(7, ev1, ev2, 1);
  }
  if (w_out) {
    e = copy_convert<double, double>(k.w, n, 1, n, w_out, n, s);
    if (e) return e;
  }
  return td_abort_check(k, s);
}

template int eig_tridiag_f32<double>(const double*, int, int, double*, int, double*, Carve&, hipStream_t, bool,
                                     Prof*);
template int eig_tridiag_f32<float>(const float*, int, int, double*, int, double*, Carve&, hipStream_t, bool, Prof*);

// ---- stage entry points (parity tests) -----------------------------------------------------

// d, e (FP64 holding FP32 values), tau (n - 2) and U (n x (n - 2), ld ldu, column k = u_k).
int tridiag_reduce_entry(const double* A, int n, int lda, double* d, double* e, float* tau, float* U, int ldu,
                         hipStream_t s) {
  void* ws = workspace(tridiag_bytes(n));
  if (!ws) { set_error("workspace allocation failed"); return 4; }
  Carve c(ws);
  TdWork k = td_carve(c, n);
  int r = td_reduce<double>(A, n, lda, k, s);
  if (r) return r;
  r = copy_convert<double, double>(k.d, n, 1, n, d, n, s);
  if (r) return r;
  if (n > 1) {
    r = copy_convert<double, double>(k.e, n - 1, 1, n, e, n, s);
    if (r) return r;
  }
  if (n > 2) {
    r = copy_convert<float, float>(k.tau, n - 2, 1, n, tau, n, s);
    if (r) return r;
    r = copy_convert<double, float>(k.U, n, n - 2, n, U, ldu, s);
    if (r) return r;
  }
  return td_abort_check(k, s);
}

// w (ascending) and, if Z is not NULL, the eigenvectors (FP64, n x n, ldz) of the tridiagonal (d, e).
int tridiag_eig_entry(const double* d, const double* e, int n, double* w, double* Z, int ldz, hipStream_t s) {
  void* ws = workspace(tridiag_bytes(n));
  if (!ws) { set_error("workspace allocation failed"); return 4; }
  Carve c(ws);
  TdWork k = td_carve(c, n);
  int r = copy_convert<double, double>(d, n, 1, n, k.d, n, s);
  if (r) return r;
  if (n > 1) {
    r = copy_convert<double, double>(e, n - 1, 1, n, k.e, n, s);
    if (r) return r;
  }
  r = td_eigvals(k.d, k.e, n, k.bnd, w, s);
  if (r) return r;
  if (Z) {
    r = td_vectors<double>(k.d, k.e, n, w, k.bnd, k.dp, k.dm, k.nc, Z, ldz, s);
    if (r) return r;
  }
  JAC_HIP(hipStreamSynchronize(s));
  return 0;
}

// Y (n x ncol... here n x n FP64, ldy) <- H_0 ... H_{n-3} Y in FP32 arithmetic, for reflectors
// given as U (n x (n - 2), ld ldu) and tau.
int tridiag_backtransform_entry(const float* U, int ldu, const float* tau, int n, double* Y, int ldy, hipStream_t s) {
  void* ws = workspace(tridiag_bytes(n));
  if (!ws) { set_error("workspace allocation failed"); return 4; }
  Carve c(ws);
  TdWork k = td_carve(c, n);
  hipLaunchKernelGGL(td_fill_u64_kernel, dim3(1024), dim3(256), 0, s, reinterpret_cast<unsigned long long*>(k.U),
                     (long long)k.nbp * n);
  JAC_CHECK_LAUNCH();
  hipLaunchKernelGGL(td_fill_u64_kernel, dim3(1024), dim3(256), 0, s, reinterpret_cast<unsigned long long*>(k.Ut),
                     (long long)k.nbp * n);
  JAC_CHECK_LAUNCH();
  hipLaunchKernelGGL(td_fill_f32_kernel, dim3(1), dim3(256), 0, s, k.tau, (long long)k.nbp);
  JAC_CHECK_LAUNCH();
  int r = 0;
  if (n > 2) {
    r = copy_convert<float, double>(U, n, n - 2, ldu, k.U, n, s);
    if (r) return r;
    hipLaunchKernelGGL(td_transpose_kernel<double>, dim3(tcdiv(n, 32), tcdiv(n - 2, 32)), dim3(256), 0, s, k.U, n, n,
                       n - 2, k.Ut, k.nbp);
    JAC_CHECK_LAUNCH();
    r = copy_convert<float, float>(tau, n - 2, 1, n, k.tau, n, s);
    if (r) return r;
  }
  r = copy_convert<double, double>(Y, n, n, ldy, k.Y, n, s);
  if (r) return r;
  r = td_backtransform(k.U, k.Ut, k.nbp, k.tau, n, k.G, k.Tf, k.Wb, k.W2, k.Y, s, false);
  if (r) return r;
  r = copy_convert<double, double>(k.Y, n, n, n, Y, ldy, s);
  if (r) return r;
  JAC_HIP(hipStreamSynchronize(s));
  return 0;
}

}  // namespace jac
