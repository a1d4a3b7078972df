// Block modified Gram-Schmidt in FP64 (step 2 of Algorithm 4.1).
//
// Columns are processed in panels of width P.  Inside a panel, one workgroup
// holds the panel in registers (R rows per thread) and runs MGS column by
// column: normalise column c, then remove its component from every later
// column of the panel (one workgroup reduction per column).
// After a panel is done, its projection is removed from all trailing columns:
// Z_R -= Q_P (Q_P^T Z_R), on the matrix cores in two launches per panel.  In
// exact arithmetic this is MGS; with kappa(Z) ~ 1 (Lemma main) the block form
// loses only O(u) orthogonality.  Q keeps Z's column order and signs (R has a
// positive diagonal).
#include "common.h"

namespace jac {

constexpr int kMT = 512;  // threads of the panel kernel (2 waves per SIMD: 256 VGPRs each)

constexpr int next_pow2(int x) { return x <= 1 ? 1 : 2 * next_pow2((x + 1) / 2); }
constexpr int ilog2(int x) { return x <= 1 ? 0 : 1 + ilog2(x / 2); }

// The 64-bit value of another lane by data-parallel-primitive moves (two 32-bit
// halves): CTRL is a DPP control word.
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double x) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(x);
  const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Value held by lane (lane ^ (1 << LVL)) of the same 16-lane row, LVL = 0..3:
// quad permutations [1,0,3,2] and [2,3,0,1]; a shift by 4 lanes up or down
// within the row (selected by bit 2); a rotation of the row by 8.
template <int LVL>
__device__ __forceinline__ double xor_lane(double x, int lane) {
  if constexpr (LVL == 0) return dpp_mov<0xB1>(x);
  else if constexpr (LVL == 1) return dpp_mov<0x4E>(x);
  else if constexpr (LVL == 2) {
    const double up = dpp_mov<0x104>(x), down = dpp_mov<0x114>(x);   // lanes + 4, lanes - 4
    return (lane & 4) ? down : up;
  } else return dpp_mov<0x128>(x);
}

// The 64-bit value of lane (lane ^ 16) (BIT = 16) or (lane ^ 32) (BIT = 32): the row swaps exchange
// the odd 16-lane rows (upper 32-lane half) of their first operand with the even rows (lower
// half) of their second; with the same value in both, the two results hold a lane's own value and
// its partner's, in an order set by the lane's bit.
template <int BIT>
__device__ __forceinline__ double swap_lane(double x, int lane) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(x);
  const unsigned lo = (unsigned)b, hi = (unsigned)(b >> 32);
  unsigned plo, phi;
  if constexpr (BIT == 16) {
    const auto rl = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    const auto rh = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    plo = (lane & 16) ? rl[0] : rl[1];
    phi = (lane & 16) ? rh[0] : rh[1];
  } else {
    const auto rl = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
    const auto rh = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
    plo = (lane & 32) ? rl[0] : rl[1];
    phi = (lane & 32) ? rh[0] : rh[1];
  }
  return __longlong_as_double((long long)(((unsigned long long)phi << 32) | plo));
}

// One halving level: each lane keeps one half of its NP values (by bit LVL of
// its lane) and adds the partner's copy of that half.
template <int LVL, int NP>
__device__ __forceinline__ void halve(double (&w)[NP], int lane) {
  constexpr int half = NP >> (LVL + 1);
  const bool up = (lane & (1 << LVL)) != 0;
#pragma unroll
  for (int j = 0; j < half; ++j) {
    // Both halves are pinned in registers before the select; otherwise the
    // compiler turns "up ? w[j] : w[j + half]" into a runtime index into w,
    // which it lowers to a compare-and-select chain over all of w.
    double lo = w[j], hi = w[j + half];
    asm volatile("" : "+v"(lo), "+v"(hi));
    const double send = up ? lo : hi;
    const double keep = up ? hi : lo;
    w[j] = keep + xor_lane<LVL>(send, lane);
  }
}

// Sum NV <= 16 values (compile-time count) across the workgroup with one
// barrier; every thread gets the totals in tot[] (uniform values).  Inside a
// 16-lane row the values are summed by halving exchanges (NP = next_pow2(NV)
// values cost NP - 1 + 4 - log2(NP) exchanges; lane l then holds the value
// whose index is the bit reversal of l's low log2(NP) bits); two row swaps add
// the wave's 4 row sums, row 0 of each of the kMT / 64 waves writes them to
// lds[par] (par alternates by column, so a wave one column ahead writes the
// other half), and after the barrier lane j < NV of every wave adds the
// kMT / 64 wave sums of value j and readlane broadcasts the totals.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* lds2, int par, double (&tot)[NV]) {
  constexpr int NP = next_pow2(NV);
  constexpr int K = ilog2(NP);
  static_assert(NP <= 16, "at most 16 values");
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double* lds = lds2 + par * (kMT / 16) * 16;
  double w[NP];
#pragma unroll
  for (int j = 0; j < NP; ++j) w[j] = j < NV ? v[j] : 0.0;
  if constexpr (K > 0) halve<0, NP>(w, lane);
  if constexpr (K > 1) halve<1, NP>(w, lane);
  if constexpr (K > 2) halve<2, NP>(w, lane);
  if constexpr (K > 3) halve<3, NP>(w, lane);
  double x = w[0];
  if constexpr (K <= 0) x += xor_lane<0>(x, lane);
  if constexpr (K <= 1) x += xor_lane<1>(x, lane);
  if constexpr (K <= 2) x += xor_lane<2>(x, lane);
  if constexpr (K <= 3) x += xor_lane<3>(x, lane);
  x += swap_lane<16>(x, lane);
  x += swap_lane<32>(x, lane);
  if (lane < NP) {
    int idx = 0;
#pragma unroll
    for (int lvl = 0; lvl < K; ++lvl)
      if (lane & (1 << lvl)) idx += NP >> (lvl + 1);
    if (idx < NV) lds[wave * 16 + idx] = x;
  }
  __syncthreads();
  double s[4] = {0, 0, 0, 0};
  if (lane < NV) {
#pragma unroll
    for (int q = 0; q < kMT / 64; ++q) s[q & 3] += lds[q * 16 + lane];
  }
  const double t = (s[0] + s[1]) + (s[2] + s[3]);
  const unsigned long long tb = (unsigned long long)__double_as_longlong(t);
  const int tlo = (int)(unsigned)tb, thi = (int)(unsigned)(tb >> 32);
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane(tlo, j);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane(thi, j);
    tot[j] = __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
  }
}

// Column c of the panel: one reduction gives ||v_c||^2 and v_c . v_j for the
// later columns j; then q_c = v_c / ||v_c|| and v_j -= (q_c . v_j) q_c with
// q_c . v_j = (v_c . v_j) / ||v_c||.  C is a compile-time column index so
// that the register panel is never indexed dynamically.  Columns at or past
// ncols (the short last panel) are zero and stay zero; FULL panels (ncols = P)
// are compiled without the column tests.  q_c is final once normalised and is
// stored right away, so its stores drain while the later columns are worked.
template <int R, int P, int C, bool FULL>
__device__ __forceinline__ void mgs_column(double (&v)[R][P], int ncols, const double* nrm0, double* lds2,
                                           int* flag, double* __restrict__ Q, int m, int ldq) {
  if constexpr (C < P) {
    if (FULL || C < ncols) {
      constexpr int NV = P - C;
      double part[NV];
#pragma unroll
      for (int j = 0; j < NV; ++j) {
        double acc = 0;
#pragma unroll
        for (int r = 0; r < R; ++r) acc = fma(v[r][C], v[r][C + j], acc);
        part[j] = acc;
      }
      double tot[NV];
      block_sum<NV>(part, lds2, C & 1, tot);
      double nrm = sqrt(tot[0]);
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
      for (int r = 0; r < R; ++r) {
        v[r][C] = v[r][C] * inv;
        const int i = threadIdx.x + r * kMT;
        if (i < m) Q[i + (size_t)C * ldq] = v[r][C];
      }
#pragma unroll
      for (int j = 1; j < NV; ++j) {
        const double d = tot[j] * inv;
#pragma unroll
        for (int r = 0; r < R; ++r) v[r][C + j] = fma(-d, v[r][C], v[r][C + j]);
      }
      mgs_column<R, P, C + 1, FULL>(v, ncols, nrm0, lds2, flag, Q, m, ldq);
    }
  }
}

template <int R, int P, bool FULL>
__global__ void __launch_bounds__(kMT) mgs_panel_kernel(double* __restrict__ Q, int m, int ldq, int ncols,
                                                        const double* __restrict__ nrm0, int* __restrict__ flag) {
  __shared__ double lds2[2 * (kMT / 16) * 16];
  __shared__ double n0[P];   // original column norms, staged once (a global read per column would
                             // sit behind every column's reduction)
  double v[R][P];
  if (threadIdx.x < P) n0[threadIdx.x] = (FULL || (int)threadIdx.x < ncols) ? nrm0[threadIdx.x] : 1.0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    int i = threadIdx.x + r * kMT;
#pragma unroll
    for (int c = 0; c < P; ++c) v[r][c] = (i < m && (FULL || c < ncols)) ? Q[i + (size_t)c * ldq] : 0.0;
  }
  __syncthreads();
  mgs_column<R, P, 0, FULL>(v, ncols, n0, lds2, flag, Q, m, ldq);
}

// Z_R -= Q_P (Q_P^T Z_R) in two launches over a grid of (16-column block,
// 256-row block) workgroups of four waves; Q_P is m x w (w <= kPW = 16), all
// column-major with leading dimension ld.
//  mgs_projw_kernel: each wave stages 64 rows of Q_P and of the column block
//    in LDS (rows along lanes, coalesced) and accumulates Q_P^T Z on the
//    16x16x4 FP64 matrix-core op (A(i = p, k = row) = Q(row, p),
//    B(k = row, j = col) = Z(row, col)); the four waves' sums give the row
//    block's partial W (16 x 16), stored to Wp[col block][row block].
//  mgs_projz_kernel: sums the partial W of all row blocks (same order in every
//    workgroup, so the result does not depend on scheduling) and applies
//    Z^T -= W^T Q_P^T on 16-row tiles (A(i = col, k = p) = W(p, col),
//    B(k = p, j = row) = Q(row, p)); in this orientation the accumulator holds
//    consecutive rows in consecutive lanes, so Z and Q move along columns.
constexpr int kPW = 16;
constexpr int kPT = 256;      // threads of the projection kernels
constexpr int kChunk = 64;    // rows per wave
constexpr int kRB = kChunk * (kPT / 64);   // rows per workgroup
constexpr int kSL = kPW + 1;

__global__ void __launch_bounds__(kPT) mgs_projw_kernel(const double* __restrict__ Qp, int w,
                                                        const double* __restrict__ Zr, int m, int ld, int rest,
                                                        double* __restrict__ Wp) {
  __shared__ double sq[kPT / 64][kChunk * kSL];
  __shared__ double sz[kPT / 64][kChunk * kSL];
  __shared__ double sw[kPT / 64][kPW * kPW];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int cb = blockIdx.x, rb = blockIdx.y;
  const int c0 = cb * kPW, nc = rest - c0 < kPW ? rest - c0 : kPW;
  const int li = lane & 15, lk = lane >> 4;
  const int row = rb * kRB + wave * kChunk + lane;
  double qv[kPW], zv[kPW];
#pragma unroll
  for (int c = 0; c < kPW; ++c) {
    qv[c] = (row < m && c < w) ? Qp[row + (size_t)c * ld] : 0.0;
    zv[c] = (row < m && c < nc) ? Zr[row + (size_t)(c0 + c) * ld] : 0.0;
  }
#pragma unroll
  for (int c = 0; c < kPW; ++c) {
    sq[wave][lane * kSL + c] = qv[c];
    sz[wave][lane * kSL + c] = zv[c];
  }
  __builtin_amdgcn_wave_barrier();
  f64x4 acc = {0, 0, 0, 0};
#pragma unroll
  for (int s = 0; s < kChunk / 4; ++s) {
    const double a = sq[wave][(4 * s + lk) * kSL + li];
    const double b = sz[wave][(4 * s + lk) * kSL + li];
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
  }
  // accumulator r: W(p = 4 r + lane / 16, col = lane % 16)
#pragma unroll
  for (int r = 0; r < 4; ++r) sw[wave][(4 * r + lk) * kPW + li] = acc[r];
  __syncthreads();
  const int e = threadIdx.x;
  if (e < kPW * kPW)
    Wp[((size_t)cb * gridDim.y + rb) * kPW * kPW + e] = (sw[0][e] + sw[1][e]) + (sw[2][e] + sw[3][e]);
}

__global__ void __launch_bounds__(kPT) mgs_projz_kernel(const double* __restrict__ Qp, int w, double* __restrict__ Zr,
                                                        int m, int ld, int rest, const double* __restrict__ Wp) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int cb = blockIdx.x, rb = blockIdx.y, nrb = gridDim.y;
  const int c0 = cb * kPW, nc = rest - c0 < kPW ? rest - c0 : kPW;
  const int li = lane & 15, lk = lane >> 4;
  constexpr int kTiles = kChunk / 16;
  const int row0 = rb * kRB + wave * kChunk;
  // loads first: Q_P and Z for the wave's four 16-row tiles, then the partial W
  double qb[kTiles][4], zb[kTiles][4];
#pragma unroll
  for (int t = 0; t < kTiles; ++t) {
    const int row = row0 + t * 16 + li;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int p = 4 * q + lk, col = 4 * q + lk;
      qb[t][q] = (row < m && p < w) ? Qp[row + (size_t)p * ld] : 0.0;
      zb[t][q] = (row < m && col < nc) ? Zr[row + (size_t)(c0 + col) * ld] : 0.0;
    }
  }
  double wv[4] = {0, 0, 0, 0};
  const double* wp = Wp + (size_t)cb * nrb * kPW * kPW;
  for (int k = 0; k < nrb; ++k) {
#pragma unroll
    for (int q = 0; q < 4; ++q) wv[q] += wp[(size_t)k * kPW * kPW + (4 * q + lk) * kPW + li];   // W(4q + lane/16, lane%16)
  }
#pragma unroll
  for (int t = 0; t < kTiles; ++t) {
    f64x4 upd = {0, 0, 0, 0};
#pragma unroll
    for (int q = 0; q < 4; ++q) upd = __builtin_amdgcn_mfma_f64_16x16x4f64(wv[q], qb[t][q], upd, 0, 0, 0);
    // accumulator r: (Q W)(row, col = 4 r + lane / 16)
    const int row = row0 + t * 16 + li;
    if (row < m) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int col = 4 * r + lk;
        if (col < nc) Zr[row + (size_t)(c0 + col) * ld] = zb[t][r] - upd[r];
      }
    }
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

// Rows per thread R and panel width P (<= kPW) keep R*P <= 64 doubles in registers.
static int panel_width(int m) {
  int R = (m + kMT - 1) / kMT;
  if (R <= 4) return 16;
  if (R <= 8) return 8;
  if (R <= 16) return 4;
  if (R <= 32) return 2;
  return 1;
}

// nrm0 (n) and the partial W of the projection kernels (per 16-column block and 256-row block).
template <bool FULL>
static void launch_panel(int R, hipStream_t s, double* Qp, int m, int ldq, int w, const double* nrm0, int* flag) {
  if (R <= 1) hipLaunchKernelGGL((mgs_panel_kernel<1, 16, FULL>), dim3(1), dim3(kMT), 0, s, Qp, m, ldq, w, nrm0, flag);
  else if (R <= 2) hipLaunchKernelGGL((mgs_panel_kernel<2, 16, FULL>), dim3(1), dim3(kMT), 0, s, Qp, m, ldq, w, nrm0, flag);
  else if (R <= 4) hipLaunchKernelGGL((mgs_panel_kernel<4, 16, FULL>), dim3(1), dim3(kMT), 0, s, Qp, m, ldq, w, nrm0, flag);
  else if (R <= 8) hipLaunchKernelGGL((mgs_panel_kernel<8, 8, FULL>), dim3(1), dim3(kMT), 0, s, Qp, m, ldq, w, nrm0, flag);
  else if (R <= 16) hipLaunchKernelGGL((mgs_panel_kernel<16, 4, FULL>), dim3(1), dim3(kMT), 0, s, Qp, m, ldq, w, nrm0, flag);
  else if (R <= 32) hipLaunchKernelGGL((mgs_panel_kernel<32, 2, FULL>), dim3(1), dim3(kMT), 0, s, Qp, m, ldq, w, nrm0, flag);
  else hipLaunchKernelGGL((mgs_panel_kernel<64, 1, FULL>), dim3(1), dim3(kMT), 0, s, Qp, m, ldq, w, nrm0, flag);
}

size_t mgs_scratch_elems(int m, int n) {
  return (size_t)n + 64 + (size_t)((n + kPW - 1) / kPW) * ((m + kRB - 1) / kRB) * kPW * kPW;
}

int mgs_f64(double* Q, int m, int n, int ldq, double* W, int* flag, hipStream_t s) {
  static_assert(kMgsMaxRows == 64 * kMT, "the panel kernel's largest register tile");
  if (m > kMgsMaxRows) {
    set_error("mgs: more than 32768 rows is not supported");
    return -2;
  }
  const int P = panel_width(m);
  const int R = (m + kMT - 1) / kMT;
  double* nrm0 = W;
  double* Wp = W + n + 64;
  hipLaunchKernelGGL(colnorm_kernel, dim3(n), dim3(256), 0, s, Q, m, ldq, nrm0);
  JAC_CHECK_LAUNCH();
  for (int j0 = 0; j0 < n; j0 += P) {
    int w = n - j0 < P ? n - j0 : P;
    double* Qp = Q + (size_t)j0 * ldq;
    if (w == P) launch_panel<true>(R, s, Qp, m, ldq, w, nrm0 + j0, flag);
    else launch_panel<false>(R, s, Qp, m, ldq, w, nrm0 + j0, flag);
    JAC_CHECK_LAUNCH();
    const int rest = n - j0 - w;
    if (rest > 0) {
      const dim3 g((rest + kPW - 1) / kPW, (m + kRB - 1) / kRB);
      double* Zr = Q + (size_t)(j0 + w) * ldq;
      hipLaunchKernelGGL(mgs_projw_kernel, g, dim3(kPT), 0, s, (const double*)Qp, w, (const double*)Zr, m, ldq, rest,
                         Wp);
      JAC_CHECK_LAUNCH();
      hipLaunchKernelGGL(mgs_projz_kernel, g, dim3(kPT), 0, s, (const double*)Qp, w, Zr, m, ldq, rest,
                         (const double*)Wp);
      JAC_CHECK_LAUNCH();
    }
  }
  return 0;
}

}  // namespace jac
