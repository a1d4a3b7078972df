// Step 2 of Algorithm 4.1 for a nearly orthonormal start: Q = Z R^{-1} with R upper triangular,
// positive diagonal and R^T R = Z^T Z -- the factor modified Gram-Schmidt returns in exact
// arithmetic (Lemma MGS: same column order and signs, ||Q - Z|| = O(||Z^T Z - I||)).
//
// With E = Z^T Z - I small (every FP32 start: ||E||_2 is a few 1e-6), R = I + F where F is upper
// triangular and F + F^T + F^T F = E.  Writing U(X) for the strict upper triangle of X plus half its
// diagonal, F = U(E - F^T F); two fixed-point steps give F = U(E - F0^T F0), F0 = U(E), with an
// error O(||E||^3).  Then R^{-1} = I - F + F^2 - ..., and
//     Q = Z - Z F + (Z F) F
// is exact to O(||E||^3) as well.  Everything is four FP64 GEMMs on the matrix cores (Z^T Z,
// F0^T F0, Z F, (Z F) F) plus two transposes and two element-wise passes.  When ||E||_F exceeds
// kSeriesMax the caller uses block MGS instead.
#include <cmath>

#include "common.h"

namespace jac {

static inline int ocdiv(long long a, long long b) { return (int)((a + b - 1) / b); }

constexpr double kSeriesMax = 1e-3;   // ||E||_F bound for the series (error ~ ||E||^3 << 2^-53)

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
    const double e = G[i + (size_t)j * n] - (i == j ? 1.0 : 0.0);
    acc += e * e;
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
// doubles; scal: device double receiving ||E||_F^2.  *used = 1 when Q was formed, 0 when
// ||E||_F > kSeriesMax (Z is then unchanged and the caller orthogonalises it by block MGS).
// no_split: GEMMs without split-K.
int orth_series_f64(double* Z, int n, int ldz, double* B1, double* B2, double* B3, double* B4, double* part,
                    double* scal, int* used, hipStream_t s, bool no_split) {
  // B1: Z^T, then F0^T, then Y = Z F.  B2: G = Z^T Z, then Y2 = Y F.  B3: F0, then F.  B4: F0^T F0.
  *used = 0;
  if (n <= 0) { *used = 1; return 0; }
  const int ms = no_split ? 1 : 0;
  const dim3 tg(ocdiv(n, 32), ocdiv(n, 32));
  hipLaunchKernelGGL(orth_transpose_kernel, tg, dim3(256), 0, s, (const double*)Z, n, ldz, B1, n);
  JAC_CHECK_LAUNCH();
  int e = gemm<double>(false, false, n, n, n, 1.0, B1, n, Z, ldz, 0.0, B2, n, s, ms);
  if (e) return e;
  const int gx = ocdiv(n, 256) < 2 ? ocdiv(n, 256) : 2;   // at most 2 n partial sums
  hipLaunchKernelGGL(orth_f0_kernel, dim3(gx, n), dim3(256), 0, s, (const double*)B2, n, B3, part);
  JAC_CHECK_LAUNCH();
  hipLaunchKernelGGL(orth_sum_kernel, dim3(1), dim3(256), 0, s, (const double*)part, gx * n, scal);
  JAC_CHECK_LAUNCH();
  double e2 = 0.0;
  JAC_HIP(hipMemcpyAsync(&e2, scal, sizeof(double), hipMemcpyDeviceToHost, s));
  JAC_HIP(hipStreamSynchronize(s));
  if (!(e2 <= kSeriesMax * kSeriesMax)) return 0;   // not nearly orthonormal (or NaN): block MGS
  hipLaunchKernelGGL(orth_transpose_kernel, tg, dim3(256), 0, s, (const double*)B3, n, n, B1, n);
  JAC_CHECK_LAUNCH();
  e = gemm<double>(false, false, n, n, n, 1.0, B1, n, B3, n, 0.0, B4, n, s, ms);
  if (e) return e;
  const dim3 eg(ocdiv(n, 256), n);
  hipLaunchKernelGGL(orth_f1_kernel, eg, dim3(256), 0, s, (const double*)B2, (const double*)B4, n, B3);
  JAC_CHECK_LAUNCH();
  e = gemm<double>(false, false, n, n, n, 1.0, Z, ldz, B3, n, 0.0, B1, n, s, ms);
  if (e) return e;
  e = gemm<double>(false, false, n, n, n, 1.0, B1, n, B3, n, 0.0, B2, n, s, ms);
  if (e) return e;
  hipLaunchKernelGGL(orth_combine_kernel, eg, dim3(256), 0, s, Z, n, ldz, (const double*)B1, (const double*)B2);
  JAC_CHECK_LAUNCH();
  *used = 1;
  return 0;
}

}  // namespace jac
