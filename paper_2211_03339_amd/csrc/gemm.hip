// Dense GEMM on the matrix cores: C = alpha op(A) op(B) + beta C, column-major.
// FP64 uses v_mfma_f64_16x16x4f64, FP32 v_mfma_f32_16x16x4f32.  Both take one
// A value (row i = lane % 16, k = lane / 16) and one B value (k = lane / 16,
// column j = lane % 16) per lane and accumulate four C values per lane in
// column lane % 16: accumulator r holds row 4 r + lane / 16 for FP64 and row
// 4 (lane / 16) + r for FP32 (measured on gfx950).
//
// A workgroup of 4 waves (2 x 2) owns a BM x BN tile of C; each wave owns a
// (BM/2) x (BN/2) sub-tile made of 16 x 16 MFMA tiles.  K advances in steps of
// 16 through a double-buffered LDS stage (k-major, so the MFMA operand reads
// are 16 consecutive elements per k).  Split-K (grid z) writes partial tiles
// to a workspace that a second kernel sums in a fixed order.  The strided-batched form (BAT) runs
// grid z over independent products instead, each optionally switched off by a per-product state.
#include "common.h"

namespace jac {

constexpr int kBK = 16;
constexpr int kPad = 4;

template <typename T, int BM, int BN, bool TA, bool TB, bool BAT = false>
__global__ void __launch_bounds__(256)
gemm_kernel(int m, int n, int k, T alpha, const T* __restrict__ A, int lda, const T* __restrict__ B, int ldb,
            T beta, T* __restrict__ C, int ldc, int kchunk, T* __restrict__ part, int tri, long long sA = 0,
            long long sB = 0, long long sC = 0, const int* __restrict__ state = nullptr, int state_max = 0) {
  if (BAT) {   // product z of a strided batch; skipped when its state exceeds state_max
    const int z = blockIdx.z;
    if (state && state[z] > state_max) return;
    A += z * sA;
    B += z * sB;
    C += z * sC;
  }
  constexpr int WM = BM / 2, WN = BN / 2;        // wave tile
  constexpr int TM = WM / 16, TN = WN / 16;      // MFMA tiles per wave
  constexpr int LA = BM * kBK / 256;             // A elements loaded per thread
  constexpr int LB = BN * kBK / 256;
  __shared__ T As[2][kBK][BM + kPad];
  __shared__ T Bs[2][kBK][BN + kPad];
  typedef typename Mfma<T>::acc_t acc_t;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int i0 = blockIdx.x * BM, j0 = blockIdx.y * BN;
  const int kb = BAT ? 0 : blockIdx.z * kchunk;
  int ke = BAT ? k : min(k, kb + kchunk);
  // zero structure (tri): the K range that can contribute to this tile; a tile wholly below the
  // diagonal of an upper-only product gets none (and is written as zeros)
  if (tri & kGemmBUpper) ke = min(ke, j0 + BN);
  if (tri & kGemmALower) ke = min(ke, i0 + BM);
  if ((tri & kGemmCUpper) && i0 >= j0 + BN) ke = kb;

  acc_t acc[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) acc[a][b] = acc_t{0, 0, 0, 0};

  T ra[LA], rb[LB];
  // op(A)[i][kk]: TA ? A[kk + i*lda] : A[i + kk*lda]
  // A stage wholly inside the matrix and the K range (the same for every thread, so one scalar
  // branch) is loaded without the per-element checks.
  auto load_a = [&](int kt) {
    if (i0 + BM <= m && kt + kBK <= ke) {
#pragma unroll
      for (int e = 0; e < LA; ++e) {
        int idx = tid + e * 256;
        int ii, kk;
        if (!TA) { ii = idx % BM; kk = idx / BM; } else { kk = idx % kBK; ii = idx / kBK; }
        int gi = i0 + ii, gk = kt + kk;
        ra[e] = TA ? A[gk + (size_t)gi * lda] : A[gi + (size_t)gk * lda];
      }
      return;
    }
#pragma unroll
    for (int e = 0; e < LA; ++e) {
      int idx = tid + e * 256;
      int ii, kk;
      if (!TA) { ii = idx % BM; kk = idx / BM; } else { kk = idx % kBK; ii = idx / kBK; }
      int gi = i0 + ii, gk = kt + kk;
      ra[e] = (gi < m && gk < ke) ? (TA ? A[gk + (size_t)gi * lda] : A[gi + (size_t)gk * lda]) : T(0);
    }
  };
  auto load_b = [&](int kt) {
    if (j0 + BN <= n && kt + kBK <= ke) {
#pragma unroll
      for (int e = 0; e < LB; ++e) {
        int idx = tid + e * 256;
        int jj, kk;
        if (!TB) { kk = idx % kBK; jj = idx / kBK; } else { jj = idx % BN; kk = idx / BN; }
        int gj = j0 + jj, gk = kt + kk;
        rb[e] = TB ? B[gj + (size_t)gk * ldb] : B[gk + (size_t)gj * ldb];
      }
      return;
    }
#pragma unroll
    for (int e = 0; e < LB; ++e) {
      int idx = tid + e * 256;
      int jj, kk;
      if (!TB) { kk = idx % kBK; jj = idx / kBK; } else { jj = idx % BN; kk = idx / BN; }
      int gj = j0 + jj, gk = kt + kk;
      rb[e] = (gj < n && gk < ke) ? (TB ? B[gj + (size_t)gk * ldb] : B[gk + (size_t)gj * ldb]) : T(0);
    }
  };
  auto store_ab = [&](int buf) {
#pragma unroll
    for (int e = 0; e < LA; ++e) {
      int idx = tid + e * 256;
      int ii, kk;
      if (!TA) { ii = idx % BM; kk = idx / BM; } else { kk = idx % kBK; ii = idx / kBK; }
      As[buf][kk][ii] = ra[e];
    }
#pragma unroll
    for (int e = 0; e < LB; ++e) {
      int idx = tid + e * 256;
      int jj, kk;
      if (!TB) { kk = idx % kBK; jj = idx / kBK; } else { jj = idx % BN; kk = idx / BN; }
      Bs[buf][kk][jj] = rb[e];
    }
  };

  int buf = 0;
  if (kb < ke) {
    load_a(kb);
    load_b(kb);
    store_ab(0);
  }
  __syncthreads();
  for (int kt = kb; kt < ke; kt += kBK) {
    const bool more = kt + kBK < ke;
    if (more) { load_a(kt + kBK); load_b(kt + kBK); }
#pragma unroll
    for (int kk = 0; kk < kBK; kk += 4) {
      T av[TM], bv[TN];
      const int kr = kk + (lane >> 4), cc = lane & 15;
#pragma unroll
      for (int a = 0; a < TM; ++a) av[a] = As[buf][kr][wm * WM + a * 16 + cc];
#pragma unroll
      for (int b = 0; b < TN; ++b) bv[b] = Bs[buf][kr][wn * WN + b * 16 + cc];
#pragma unroll
      for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) acc[a][b] = Mfma<T>::op(av[a], bv[b], acc[a][b]);
    }
    if (more) {
      store_ab(buf ^ 1);
      __syncthreads();
      buf ^= 1;
    }
  }

  // Epilogue: accumulator r of a lane is row Mfma<T>::row(lane, r), column lane%16.
  const int col = lane & 15;
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) {
      int gj = j0 + wn * WN + b * 16 + col;
      if (gj >= n) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int gi = i0 + wm * WM + a * 16 + Mfma<T>::row(lane, r);
        if (gi >= m) continue;
        T v = alpha * acc[a][b][r];
        if (!BAT && part) {
          part[(size_t)blockIdx.z * m * n + gi + (size_t)gj * m] = v;
        } else {
          size_t o = gi + (size_t)gj * ldc;
          C[o] = beta == T(0) ? v : v + beta * C[o];
        }
      }
    }
}

template <typename T>
__global__ void splitk_reduce_kernel(const T* __restrict__ part, int S, int m, int n, T beta, T* __restrict__ C,
                                     int ldc) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  int j = blockIdx.y;
  if (i >= m) return;
  T acc = T(0);
  for (int z = 0; z < S; ++z) acc += part[(size_t)z * m * n + i + (size_t)j * m];
  size_t o = i + (size_t)j * ldc;
  C[o] = beta == T(0) ? acc : acc + beta * C[o];
}

static inline int cdiv(long long a, long long b) { return (int)((a + b - 1) / b); }

template <typename T, int BM, int BN>
static void launch_cfg(bool ta, bool tb, dim3 grid, hipStream_t s, int m, int n, int k, T alpha, const T* A,
                       int lda, const T* B, int ldb, T beta, T* C, int ldc, int kchunk, T* part, int tri) {
#define L(TA_, TB_)                                                                                       \
  hipLaunchKernelGGL((gemm_kernel<T, BM, BN, TA_, TB_>), grid, dim3(256), 0, s, m, n, k, alpha, A, lda, B, \
                     ldb, beta, C, ldc, kchunk, part, tri)
  if (!ta && !tb) L(false, false);
  else if (ta && !tb) L(true, false);
  else if (!ta && tb) L(false, true);
  else L(true, true);
#undef L
}

// Scratch for split-K partial sums (library-owned, grow-only).
static void* g_part = nullptr;
static size_t g_part_bytes = 0;

// max_split = 1: never split K (no partial-sum buffer, so nothing is allocated).
template <typename T>
int gemm(bool ta, bool tb, int m, int n, int k, T alpha, const T* A, int lda, const T* B, int ldb, T beta,
         T* C, int ldc, hipStream_t s, int max_split, int tri) {
  if (m <= 0 || n <= 0) return 0;
  if (k <= 0) {
    // C = beta C
    if (beta == T(1)) return 0;
    T* nul = nullptr;
    hipLaunchKernelGGL((splitk_reduce_kernel<T>), dim3(cdiv(m, 256), n), dim3(256), 0, s, nul, 0, m, n, beta, C,
                       ldc);
    JAC_CHECK_LAUNCH();
    return 0;
  }
  int cus = 256;
  // 64 x 64 tiles: at n = 2048 four workgroups per CU hide the loads better than one 128 x 128
  // (2048^3: 0.44 vs 0.51 ms; 4096^3: 2.9 vs 3.5 ms), 32-wide for skinny outputs.
  int BM = 64;
  int BN = 64;
  if (m <= 32) BM = 32;
  if (n <= 32) BN = 32;
  int tiles = cdiv(m, BM) * cdiv(n, BN);
  int S = 1;
  if (tiles < cus && k >= 512 && max_split != 1) {
    S = cdiv(2 * cus, tiles);
    int maxS = k / 256;
    if (S > maxS) S = maxS;
    if (S < 1) S = 1;
  }
  int kchunk = cdiv(cdiv(k, S), kBK) * kBK;
  S = cdiv(k, kchunk);
  T* part = nullptr;
  if (S > 1) {
    size_t need = (size_t)S * m * n * sizeof(T);
    if (need > g_part_bytes) {
      if (g_part) JAC_HIP(hipFree(g_part));
      g_part = nullptr;
      JAC_HIP(hipMalloc(&g_part, need));
      g_part_bytes = need;
    }
    part = static_cast<T*>(g_part);
  }
  dim3 grid(cdiv(m, BM), cdiv(n, BN), S);
  if (BM == 64 && BN == 64) launch_cfg<T, 64, 64>(ta, tb, grid, s, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, kchunk, part, tri);
  else if (BM == 32 && BN == 64) launch_cfg<T, 32, 64>(ta, tb, grid, s, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, kchunk, part, tri);
  else if (BM == 64 && BN == 32) launch_cfg<T, 64, 32>(ta, tb, grid, s, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, kchunk, part, tri);
  else launch_cfg<T, 32, 32>(ta, tb, grid, s, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, kchunk, part, tri);
  JAC_CHECK_LAUNCH();
  if (S > 1) {
    hipLaunchKernelGGL((splitk_reduce_kernel<T>), dim3(cdiv(m, 256), n), dim3(256), 0, s, part, S, m, n, beta, C,
                       ldc);
    JAC_CHECK_LAUNCH();
  }
  return 0;
}

// C_z = alpha op(A_z) op(B_z) + beta C_z for z < count (A_z = A + z sA, ...), no split-K.  state
// (device, may be NULL): product z runs only when state[z] <= state_max.
template <typename T>
int gemm_batched(bool ta, bool tb, int m, int n, int k, T alpha, const T* A, int lda, long long sA, const T* B,
                 int ldb, long long sB, T beta, T* C, int ldc, long long sC, int count, const int* state,
                 int state_max, hipStream_t s) {
  if (m <= 0 || n <= 0 || count <= 0) return 0;
  if (k <= 0) { set_error("gemm_batched: k must be positive"); return 4; }
  if (count > 65535) { set_error("gemm_batched: more than 65535 products"); return 4; }
  const int BM = m <= 32 ? 32 : 64, BN = n <= 32 ? 32 : 64;
  dim3 grid(cdiv(m, BM), cdiv(n, BN), count);
#define LB(BM_, BN_, TA_, TB_)                                                                                    \
  hipLaunchKernelGGL((gemm_kernel<T, BM_, BN_, TA_, TB_, true>), grid, dim3(256), 0, s, m, n, k, alpha, A, lda, B, \
                     ldb, beta, C, ldc, k, (T*)nullptr, 0, sA, sB, sC, state, state_max)
#define LT(BM_, BN_)                          \
  if (!ta && !tb) LB(BM_, BN_, false, false); \
  else if (ta && !tb) LB(BM_, BN_, true, false); \
  else if (!ta && tb) LB(BM_, BN_, false, true); \
  else LB(BM_, BN_, true, true)
  if (BM == 64 && BN == 64) { LT(64, 64); }
  else if (BM == 32 && BN == 64) { LT(32, 64); }
  else if (BM == 64 && BN == 32) { LT(64, 32); }
  else { LT(32, 32); }
#undef LT
#undef LB
  JAC_CHECK_LAUNCH();
  return 0;
}

template int gemm_batched<double>(bool, bool, int, int, int, double, const double*, int, long long, const double*,
                                  int, long long, double, double*, int, long long, int, const int*, int,
                                  hipStream_t);

template int gemm<double>(bool, bool, int, int, int, double, const double*, int, const double*, int, double,
                          double*, int, hipStream_t, int, int);
template int gemm<float>(bool, bool, int, int, int, float, const float*, int, const float*, int, float, float*,
                         int, hipStream_t, int, int);

}  // namespace jac
