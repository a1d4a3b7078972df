// Step 2 of Algorithm 4.1 for a nearly orthonormal start: Q = Z R^{-1} with R upper triangular,
// positive diagonal and R^T R = Z^T Z -- the factor modified Gram-Schmidt returns in exact
// arithmetic (Lemma MGS: same column order and signs, ||Q - Z|| = O(||Z^T Z - I||)).
//
// With E = Z^T Z - I small, R = I + F where F is upper triangular and F + F^T + F^T F = E.  Writing
// U(X) for the strict upper triangle of X plus half its diagonal, F = U(E - F^T F); two fixed-point
// steps give F = U(E - F0^T F0), F0 = U(E), with an error O(||E||^3).  Then R^{-1} = I - F + F^2 - ...,
// and one pass
//     Q = Z - Z F + (Z F) F
// is exact to O(||E||^3) as well: four FP64 GEMMs on the matrix cores (Z^T Z, F0^T F0, Z F, (Z F) F)
// plus element-wise passes.  The constant of the O(||E||^3) term is about 1 for structured E (a
// random E gains a further 1/n), so a pass from ||E||_F <= kSeriesOnePass is final.  From a larger
// ||E||_F (up to kSeriesMax) the pass is followed by another: every pass multiplies Z on the right by
// an upper triangular matrix, so the QR factor stays the same and ||E|| falls to about ||E||^3.  The
// first Z^T Z of the next pass measures the result; a pass that left ||E||_F at rounding level
// (8 n 2^-53) is the last.
#include <cmath>

#include "common.h"

namespace jac {

static inline int ocdiv(long long a, long long b) { return (int)((a + b - 1) / b); }

static inline double orth_floor(int n) { return 8.0 * n * 1.1102230246251565e-16; }

// B = A^T (n x n, 32 x 32 tiles through LDS).
__global__ void orth_transpose_kernel(const double* __restrict__ A, int n, int lda, double* __restrict__ B, int ldb) {
  __shared__ double tl[32][33];
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int r = ty; r < 32; r += 8) {
    const int i = bx + tx, j = by + r;
    if (i < n && j < n) tl[r][tx] = A[i + (size_t)j * lda];
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int i = by + tx, j = bx + r;
    if (i < n && j < n) B[i + (size_t)j * ldb] = tl[tx][r];
  }
}

// F0 = U(G - I), and per workgroup the partial sum of (G - I)^2 (for ||E||_F).
__global__ __launch_bounds__(256) void orth_f0_kernel(const double* __restrict__ G, int n, double* __restrict__ F,
                                                     double* __restrict__ partial) {
  __shared__ double red[256];
  const int j = blockIdx.y;
  double acc = 0.0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    // only G's upper triangle is formed (G is symmetric): off-diagonal entries count twice
    const double e = i <= j ? G[i + (size_t)j * n] - (i == j ? 1.0 : 0.0) : 0.0;
    acc += (i < j ? 2.0 : 1.0) * (e * e);
    F[i + (size_t)j * n] = i < j ? e : (i == j ? 0.5 * e : 0.0);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.y * gridDim.x + blockIdx.x] = red[0];
}

// out = sum of the partials (one workgroup; fixed order).
__global__ __launch_bounds__(256) void orth_sum_kernel(const double* __restrict__ partial, int count, double* out) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < count; i += 256) acc += partial[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

// F = U(G - I - P), P = F0^T F0.
__global__ void orth_f1_kernel(const double* __restrict__ G, const double* __restrict__ P, int n, double* __restrict__ F) {
  const int j = blockIdx.y;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const size_t o = i + (size_t)j * n;
    const double e = G[o] - (i == j ? 1.0 : 0.0) - P[o];
    F[o] = i < j ? e : (i == j ? 0.5 * e : 0.0);
  }
}

// Z <- Z - Y + Y2 (Y = Z F, Y2 = Y F).
__global__ void orth_combine_kernel(double* __restrict__ Z, int n, int ldz, const double* __restrict__ Y,
                                    const double* __restrict__ Y2) {
  const int j = blockIdx.y;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const size_t o = i + (size_t)j * n;
    Z[i + (size_t)j * ldz] = (Z[i + (size_t)j * ldz] - Y[o]) + Y2[o];
  }
}

// Z (n x n, ldz) <- Q in place.  B1..B4: n x n scratch each (leading dimension n); part: 2 n
// doubles; scal: device double receiving ||E||_F^2.  *used = 1 when Q was formed, 0 when the series
// does not apply (Z then holds Z S, S upper triangular, and the caller orthogonalises it by block
// MGS).  no_split: GEMMs without split-K.
int orth_series_f64(double* Z, int n, int ldz, double* B1, double* B2, double* B3, double* B4, double* part,
                    double* scal, int* used, hipStream_t s, bool no_split) {
  // B1: Z^T, then F0^T, then Y = Z F.  B2: G = Z^T Z, then Y2 = Y F.  B3: F0, then F.  B4: F0^T F0.
  *used = 0;
  if (n <= 0) { *used = 1; return 0; }
  const int ms = no_split ? 1 : 0;
  const dim3 tg(ocdiv(n, 32), ocdiv(n, 32));
  const int gx = ocdiv(n, 256) < 2 ? ocdiv(n, 256) : 2;   // at most 2 n partial sums
  const dim3 eg(ocdiv(n, 256), n);
  // G = Z^T Z, F0 = U(G - I) and ||G - I||_F^2 (read back).
  auto measure = [&](double& e2) -> int {
    hipLaunchKernelGGL(orth_transpose_kernel, tg, dim3(256), 0, s, (const double*)Z, n, ldz, B1, n);
    JAC_CHECK_LAUNCH();
    int e = gemm<double>(false, false, n, n, n, 1.0, B1, n, Z, ldz, 0.0, B2, n, s, ms, kGemmCUpper);
    if (e) return e;
    hipLaunchKernelGGL(orth_f0_kernel, dim3(gx, n), dim3(256), 0, s, (const double*)B2, n, B3, part);
    JAC_CHECK_LAUNCH();
    hipLaunchKernelGGL(orth_sum_kernel, dim3(1), dim3(256), 0, s, (const double*)part, gx * n, scal);
    JAC_CHECK_LAUNCH();
    e2 = 0.0;
    JAC_HIP(hipMemcpyAsync(&e2, scal, sizeof(double), hipMemcpyDeviceToHost, s));
    JAC_HIP(hipStreamSynchronize(s));
    return 0;
  };
  // One pass from G (B2) and F0 (B3): Z <- Z - Z F + (Z F) F.
  auto apply = [&]() -> int {
    hipLaunchKernelGGL(orth_transpose_kernel, tg, dim3(256), 0, s, (const double*)B3, n, n, B1, n);
    JAC_CHECK_LAUNCH();
    // F0^T F0 (F0^T lower, F0 upper triangular; only its upper triangle is used), then Z F and
    // (Z F) F with F upper triangular: the GEMMs skip the zero blocks
    int e = gemm<double>(false, false, n, n, n, 1.0, B1, n, B3, n, 0.0, B4, n, s, ms,
                         kGemmALower | kGemmBUpper | kGemmCUpper);
    if (e) return e;
    hipLaunchKernelGGL(orth_f1_kernel, eg, dim3(256), 0, s, (const double*)B2, (const double*)B4, n, B3);
    JAC_CHECK_LAUNCH();
    e = gemm<double>(false, false, n, n, n, 1.0, Z, ldz, B3, n, 0.0, B1, n, s, ms, kGemmBUpper);
    if (e) return e;
    e = gemm<double>(false, false, n, n, n, 1.0, B1, n, B3, n, 0.0, B2, n, s, ms, kGemmBUpper);
    if (e) return e;
    hipLaunchKernelGGL(orth_combine_kernel, eg, dim3(256), 0, s, Z, n, ldz, (const double*)B1, (const double*)B2);
    JAC_CHECK_LAUNCH();
    return 0;
  };
  const double fl = orth_floor(n);
  double e2 = 0.0;
  int e = measure(e2);
  if (e) return e;
  for (int pass = 0; pass < kSeriesPasses; ++pass) {
    if (!(e2 <= kSeriesMax * kSeriesMax)) return 0;   // not nearly orthonormal (or NaN): block MGS
    if ((e = apply())) return e;
    if (e2 <= kSeriesOnePass * kSeriesOnePass) { *used = 1; return 0; }
    if ((e = measure(e2))) return e;
    if (e2 <= fl * fl) { *used = 1; return 0; }
  }
  return 0;
}

// ---------------------------------------------------------------- batched
// The same passes for `count` matrices of order np stored back to back (Z_z = Z + z np^2, leading
// dimension np; the part beyond a matrix's own order is the identity, which the passes leave
// alone).  Per matrix, state[z]:
//   0  measure (Z^T Z) at the next pass, then apply it
//   1  apply the current pass, which is final
//   2  done: Z_z is orthonormal to rounding level
//   3  failed (||E||_F > kSeriesMax, NaN, or not at rounding level after the last pass)
// e2_first[z] receives ||Z_z^T Z_z - I||_F^2 of the start.  Every kernel and GEMM skips the matrices
// it does not concern, so the whole sequence is a fixed list of launches (graph-capturable).

// B_z = A_z^T (np x np each, 32 x 32 tiles through LDS; grid z = matrix).
__global__ void orthb_transpose_kernel(const double* __restrict__ A, int np, double* __restrict__ B,
                                       const int* __restrict__ state, int state_max) {
  const int z = blockIdx.z;
  if (state[z] > state_max) return;
  __shared__ double tl[32][33];
  const size_t off = (size_t)z * np * np;
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

// For state 0: e2 = ||G - I||_F^2 (fixed order), F0 = U(G - I), and the pass decision.
__global__ __launch_bounds__(256) void orthb_f0_kernel(const double* __restrict__ G, int np, double* __restrict__ F,
                                                      int* __restrict__ state, double* __restrict__ e2_first,
                                                      int pass, int last_pass, double floor2) {
  const int z = blockIdx.x;
  if (state[z] != 0) return;
  __shared__ double red[256];
  const size_t off = (size_t)z * np * np;
  double acc = 0.0;
  for (long long t = threadIdx.x; t < (long long)np * np; t += 256) {
    const int i = (int)(t % np), j = (int)(t / np);
    const double e = G[off + t] - (i == j ? 1.0 : 0.0);
    acc += e * e;
    F[off + t] = i < j ? e : (i == j ? 0.5 * e : 0.0);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double e2 = red[0];
    if (pass == 0) e2_first[z] = e2;
    int st;
    if (pass > 0 && e2 <= floor2) st = 2;                                   // the last pass was enough
    else if (!(e2 <= kSeriesMax * kSeriesMax) || pass == last_pass) st = 3;  // too far, or out of passes
    else st = e2 <= kSeriesOnePass * kSeriesOnePass ? 1 : 0;
    state[z] = st;
  }
}

// F = U(G - I - P) for states 0 and 1.
__global__ void orthb_f1_kernel(const double* __restrict__ G, const double* __restrict__ P, int np,
                                double* __restrict__ F, const int* __restrict__ state) {
  const int z = blockIdx.y;
  if (state[z] > 1) return;
  const size_t off = (size_t)z * np * np;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < (long long)np * np;
       t += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(t % np), j = (int)(t / np);
    const double e = G[off + t] - (i == j ? 1.0 : 0.0) - P[off + t];
    F[off + t] = i < j ? e : (i == j ? 0.5 * e : 0.0);
  }
}

// Z <- Z - Y + Y2 for states 0 and 1 (orthb_settle_kernel then turns state 1 into 2).
__global__ void orthb_combine_kernel(double* __restrict__ Z, int np, const double* __restrict__ Y,
                                     const double* __restrict__ Y2, const int* __restrict__ state) {
  const int z = blockIdx.y;
  if (state[z] > 1) return;
  const size_t off = (size_t)z * np * np;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < (long long)np * np;
       t += (long long)gridDim.x * blockDim.x)
    Z[off + t] = (Z[off + t] - Y[off + t]) + Y2[off + t];
}

__global__ void orthb_settle_kernel(int* __restrict__ state, int count) {
  const int z = blockIdx.x * blockDim.x + threadIdx.x;
  if (z < count && state[z] == 1) state[z] = 2;
}

__global__ void orthb_reset_kernel(int* __restrict__ state, int count) {
  const int z = blockIdx.x * blockDim.x + threadIdx.x;
  if (z < count) state[z] = 0;
}

// S1..S4: count np^2 doubles each.  On return every state is 2 (Z_z orthonormal) or 3 (failed; Z_z
// then holds Z_z S, S upper triangular).
int orth_series_batched(double* Z, int np, int count, double* S1, double* S2, double* S3, double* S4, int* state,
                        double* e2_first, hipStream_t s) {
  if (count <= 0 || np <= 0) return 0;
  if (count > 65535) { set_error("orth_series_batched: more than 65535 matrices"); return 4; }
  const long long st = (long long)np * np;
  const dim3 tg(ocdiv(np, 32), ocdiv(np, 32), count);
  int ech = ocdiv(st, 256);
  if (ech > 64) ech = 64;
  const dim3 eg(ech, count);
  const double fl = orth_floor(np);
  hipLaunchKernelGGL(orthb_reset_kernel, dim3(ocdiv(count, 256)), dim3(256), 0, s, state, count);
  JAC_CHECK_LAUNCH();
  for (int pass = 0; pass <= kSeriesPasses; ++pass) {
    // measure (state 0): S1 = Z^T, S2 = G = Z^T Z, S3 = F0
    hipLaunchKernelGGL(orthb_transpose_kernel, tg, dim3(256), 0, s, (const double*)Z, np, S1, (const int*)state, 0);
    JAC_CHECK_LAUNCH();
    int e = gemm_batched<double>(false, false, np, np, np, 1.0, S1, np, st, Z, np, st, 0.0, S2, np, st, count,
                                 state, 0, s);
    if (e) return e;
    hipLaunchKernelGGL(orthb_f0_kernel, dim3(count), dim3(256), 0, s, (const double*)S2, np, S3, state, e2_first,
                       pass, kSeriesPasses, fl * fl);
    JAC_CHECK_LAUNCH();
    if (pass == kSeriesPasses) break;
    // apply (states 0 and 1): S1 = F0^T, S4 = F0^T F0, S3 = F, S1 = Y = Z F, S4 = Y F
    hipLaunchKernelGGL(orthb_transpose_kernel, tg, dim3(256), 0, s, (const double*)S3, np, S1, (const int*)state, 1);
    JAC_CHECK_LAUNCH();
    e = gemm_batched<double>(false, false, np, np, np, 1.0, S1, np, st, S3, np, st, 0.0, S4, np, st, count, state,
                             1, s);
    if (e) return e;
    hipLaunchKernelGGL(orthb_f1_kernel, eg, dim3(256), 0, s, (const double*)S2, (const double*)S4, np, S3,
                       (const int*)state);
    JAC_CHECK_LAUNCH();
    e = gemm_batched<double>(false, false, np, np, np, 1.0, Z, np, st, S3, np, st, 0.0, S1, np, st, count, state, 1,
                             s);
    if (e) return e;
    e = gemm_batched<double>(false, false, np, np, np, 1.0, S1, np, st, S3, np, st, 0.0, S4, np, st, count, state,
                             1, s);
    if (e) return e;
    hipLaunchKernelGGL(orthb_combine_kernel, eg, dim3(256), 0, s, Z, np, (const double*)S1, (const double*)S4,
                       (const int*)state);
    JAC_CHECK_LAUNCH();
    hipLaunchKernelGGL(orthb_settle_kernel, dim3(ocdiv(count, 256)), dim3(256), 0, s, state, count);
    JAC_CHECK_LAUNCH();
  }
  return 0;
}

}  // namespace jac
