// Block modified Gram-Schmidt in FP64 (step 2 of Algorithm 4.1).
//
// Columns are processed in panels of width P.  Inside a panel, one workgroup
// holds the panel in registers (R rows per thread) and runs MGS column by
// column: normalise column c, then remove its component from every later
// column of the panel (one workgroup reduction per column).
// After a panel is done, its projection is removed from all trailing columns
// with two GEMMs on the matrix cores: W = Q_P^T Z_R, Z_R -= Q_P W.  In exact
// arithmetic this is MGS; with kappa(Z) ~ 1 (Lemma main) the block form loses
// only O(u) orthogonality.  Q keeps Z's column order and signs (R has a
// positive diagonal).
#include "common.h"

namespace jac {

constexpr int kMT = 512;  // threads of the panel kernel (2 waves per SIMD: 256 VGPRs each)

constexpr int next_pow2(int x) { return x <= 1 ? 1 : 2 * next_pow2((x + 1) / 2); }
constexpr int ilog2(int x) { return x <= 1 ? 0 : 1 + ilog2(x / 2); }

// Sum NV values (compile-time count) across the workgroup; the totals are
// left in red[0..NV-1] for every thread.  Inside a wave the values are summed
// by halving exchanges: at offset 1 each lane keeps one half of its values and
// adds the partner's copy of that half, at offset 2 one half of the rest, and
// so on, so that NP = next_pow2(NV) values cost NP - 1 + 6 - log2(NP)
// shuffles instead of 6 NV (the many exchanges use the short offsets); lane l
// then holds the value whose index is the bit reversal of l's low log2(NP)
// bits.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* lds, double* red) {
  constexpr int NP = next_pow2(NV);
  constexpr int K = ilog2(NP);
  static_assert(NP <= 64, "at most 64 values");
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double w[NP];
#pragma unroll
  for (int j = 0; j < NP; ++j) w[j] = j < NV ? v[j] : 0.0;
#pragma unroll
  for (int lvl = 0; lvl < K; ++lvl) {
    const int o = 1 << lvl;
    const int half = NP >> (lvl + 1);
    const bool up = (lane & o) != 0;
#pragma unroll
    for (int j = 0; j < half; ++j) {
      // Both halves are pinned in registers before the select; otherwise the
      // compiler turns "up ? w[j] : w[j + half]" into a runtime index into w,
      // which it lowers to a compare-and-select chain over all of w.
      double lo = w[j], hi = w[j + half];
      asm volatile("" : "+v"(lo), "+v"(hi));
      const double send = up ? lo : hi;
      const double keep = up ? hi : lo;
      w[j] = keep + __shfl_xor(send, o, 64);
    }
  }
  double x = w[0];
#pragma unroll
  for (int o = 1 << K; o < 64; o <<= 1) x += __shfl_xor(x, o, 64);
  if (lane < NP) {
    int idx = 0;
#pragma unroll
    for (int lvl = 0; lvl < K; ++lvl)
      if (lane & (1 << lvl)) idx += NP >> (lvl + 1);
    if (idx < NV) lds[wave * NV + idx] = x;
  }
  __syncthreads();
  if (threadIdx.x < NV) {
    double s = 0;
#pragma unroll
    for (int w2 = 0; w2 < kMT / 64; ++w2) s += lds[w2 * NV + threadIdx.x];
    red[threadIdx.x] = s;
  }
  __syncthreads();
}

// Column c of the panel: one reduction gives ||v_c||^2 and v_c . v_j for the
// later columns j; then q_c = v_c / ||v_c|| and v_j -= (q_c . v_j) q_c with
// q_c . v_j = (v_c . v_j) / ||v_c||.  C is a compile-time column index so
// that the register panel is never indexed dynamically.
template <int R, int P, int C>
__device__ __forceinline__ void mgs_column(double (&v)[R][P], int ncols, const double* nrm0,
                                           double* lds, double* red, int* flag) {
  if constexpr (C < P) {
    if (C < ncols) {
      constexpr int NV = P - C;
      double part[NV];
#pragma unroll
      for (int j = 0; j < NV; ++j) {
        double acc = 0;
#pragma unroll
        for (int r = 0; r < R; ++r) acc = fma(v[r][C], v[r][C + j], acc);
        part[j] = acc;
      }
      block_sum<NV>(part, lds, red);
      double nrm = sqrt(red[0]);
      // Breakdown: what is left of the column after removing the earlier
      // directions is below sqrt(u) of its original length (numerically
      // rank deficient), or zero.
      if (!(nrm > 1.0536712127723509e-08 * nrm0[C])) {
        if (threadIdx.x == 0) atomicOr(flag, 1);
        if (!(nrm > 0)) nrm = 1;
      }
      // One division per column: q_c = v_c * (1 / ||v_c||) and q_c . v_j = (v_c . v_j) * (1 / ||v_c||)
      // (within an ulp of the quotients; FP64 division is a long instruction sequence).
      const double inv = 1.0 / nrm;
#pragma unroll
      for (int r = 0; r < R; ++r) v[r][C] = v[r][C] * inv;
#pragma unroll
      for (int j = 1; j < NV; ++j) {
        if (C + j < ncols) {
          double d = red[j] * inv;
#pragma unroll
          for (int r = 0; r < R; ++r) v[r][C + j] = fma(-d, v[r][C], v[r][C + j]);
        }
      }
      mgs_column<R, P, C + 1>(v, ncols, nrm0, lds, red, flag);
    }
  }
}

template <int R, int P>
__global__ void __launch_bounds__(kMT) mgs_panel_kernel(double* __restrict__ Q, int m, int ldq, int ncols,
                                                        const double* __restrict__ nrm0, int* __restrict__ flag) {
  __shared__ double lds[(kMT / 64) * P];
  __shared__ double red[P];
  __shared__ double n0[P];   // original column norms, staged once (a global read per column would
                             // sit behind every column's reduction)
  double v[R][P];
  if (threadIdx.x < P) n0[threadIdx.x] = (int)threadIdx.x < ncols ? nrm0[threadIdx.x] : 1.0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    int i = threadIdx.x + r * kMT;
#pragma unroll
    for (int c = 0; c < P; ++c) v[r][c] = (i < m && c < ncols) ? Q[i + (size_t)c * ldq] : 0.0;
  }
  mgs_column<R, P, 0>(v, ncols, n0, lds, red, flag);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    int i = threadIdx.x + r * kMT;
#pragma unroll
    for (int c = 0; c < P; ++c)
      if (i < m && c < ncols) Q[i + (size_t)c * ldq] = v[r][c];
  }
}

// Euclidean norms of the n columns of Z (one workgroup per column).
__global__ void colnorm_kernel(const double* __restrict__ Z, int m, int ldz, double* __restrict__ out) {
  __shared__ double red[4];
  const double* z = Z + (size_t)blockIdx.x * ldz;
  double acc = 0;
  for (int i = threadIdx.x; i < m; i += 256) acc = fma(z[i], z[i], acc);
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = sqrt(red[0] + red[1] + red[2] + red[3]);
}

// Rows per thread R and panel width P keep R*P <= 64 doubles in registers.
static int panel_width(int m) {
  int R = (m + kMT - 1) / kMT;
  if (R <= 1) return 32;
  if (R <= 4) return 16;
  if (R <= 8) return 8;
  return 4;
}

size_t mgs_scratch_elems(int m, int n) { return (size_t)33 * n + 64; }

int mgs_f64(double* Q, int m, int n, int ldq, double* W, int* flag, hipStream_t s) {
  if (m > 16 * kMT) {
    set_error("mgs: more than 8192 rows is not supported");
    return -2;
  }
  const int P = panel_width(m);
  const int R = (m + kMT - 1) / kMT;
  double* nrm0 = W + (size_t)32 * n;
  hipLaunchKernelGGL(colnorm_kernel, dim3(n), dim3(256), 0, s, Q, m, ldq, nrm0);
  JAC_CHECK_LAUNCH();
  for (int j0 = 0; j0 < n; j0 += P) {
    int w = n - j0 < P ? n - j0 : P;
    double* Qp = Q + (size_t)j0 * ldq;
    if (R <= 1) hipLaunchKernelGGL((mgs_panel_kernel<1, 32>), dim3(1), dim3(kMT), 0, s, Qp, m, ldq, w, nrm0 + j0, flag);
    else if (R <= 2) hipLaunchKernelGGL((mgs_panel_kernel<2, 16>), dim3(1), dim3(kMT), 0, s, Qp, m, ldq, w, nrm0 + j0, flag);
    else if (R <= 4) hipLaunchKernelGGL((mgs_panel_kernel<4, 16>), dim3(1), dim3(kMT), 0, s, Qp, m, ldq, w, nrm0 + j0, flag);
    else if (R <= 8) hipLaunchKernelGGL((mgs_panel_kernel<8, 8>), dim3(1), dim3(kMT), 0, s, Qp, m, ldq, w, nrm0 + j0, flag);
    else hipLaunchKernelGGL((mgs_panel_kernel<16, 4>), dim3(1), dim3(kMT), 0, s, Qp, m, ldq, w, nrm0 + j0, flag);
    JAC_CHECK_LAUNCH();
    int rest = n - j0 - w;
    if (rest > 0) {
      double* Zr = Q + (size_t)(j0 + w) * ldq;
      int e = gemm<double>(true, false, w, rest, m, 1.0, Qp, ldq, Zr, ldq, 0.0, W, w, s);
      if (e) return e;
      e = gemm<double>(false, false, m, rest, w, -1.0, Qp, ldq, W, w, 1.0, Zr, ldq, s);
      if (e) return e;
    }
  }
  return 0;
}

}  // namespace jac
