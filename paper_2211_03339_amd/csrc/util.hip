// Small device utilities: norms, conversions, identity, output ordering.
#include <hip/hip_fp16.h>

#include "../../include/jacobi.h"

#include "common.h"

namespace jac {

static inline int cdiv(long long a, long long b) { return (int)((a + b - 1) / b); }

// ||A||_F^2 partial sums, one per workgroup (deterministic: fixed grid, fixed
// reduction tree), then a single-workgroup sum.
__global__ void fro2_partial_kernel(const double* __restrict__ A, int m, int n, int lda,
                                    double* __restrict__ partial) {
  __shared__ double red[4];
  double acc = 0;
  long long total = (long long)m * n;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    int j = (int)(e / m), i = (int)(e % m);
    double v = A[i + (size_t)j * lda];
    acc += v * v;
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ void sum_partials_kernel2(const double* __restrict__ partial, int count,
                                     double* __restrict__ out) {
  __shared__ double red[16];
  double acc = 0;
  for (int i = threadIdx.x; i < count; i += blockDim.x) acc += partial[i];
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0;
    for (int w = 0; w < (int)(blockDim.x / 64); ++w) s += red[w];
    *out = s;
  }
}

int fro2_f64(const double* A, int m, int n, int lda, double* partial, double* out, hipStream_t s) {
  int nwg = cdiv((long long)m * n, 256);
  if (nwg > 1024) nwg = 1024;
  if (nwg < 1) nwg = 1;
  hipLaunchKernelGGL(fro2_partial_kernel, dim3(nwg), dim3(256), 0, s, A, m, n, lda, partial);
  JAC_CHECK_LAUNCH();
  hipLaunchKernelGGL(sum_partials_kernel2, dim3(1), dim3(1024), 0, s, partial, nwg, out);
  JAC_CHECK_LAUNCH();
  return 0;
}

__global__ void off2_partial_kernel(const double* __restrict__ T, int n, int ldt, double* __restrict__ partial) {
  __shared__ double red[4];
  double acc = 0;
  long long total = (long long)n * n;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    int j = (int)(e / n), i = (int)(e % n);
    double v = i == j ? 0.0 : T[i + (size_t)j * ldt];
    acc += v * v;
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

int off2_f64(const double* T, int n, int ldt, double* partial, double* out, hipStream_t s) {
  int nwg = cdiv((long long)n * n, 256);
  if (nwg > 1024) nwg = 1024;
  if (nwg < 1) nwg = 1;
  hipLaunchKernelGGL(off2_partial_kernel, dim3(nwg), dim3(256), 0, s, T, n, ldt, partial);
  JAC_CHECK_LAUNCH();
  hipLaunchKernelGGL(sum_partials_kernel2, dim3(1), dim3(1024), 0, s, partial, nwg, out);
  JAC_CHECK_LAUNCH();
  return 0;
}

__global__ void finite_kernel(const double* __restrict__ A, int m, int n, int lda, int* flag) {
  long long total = (long long)m * n;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    int j = (int)(e / m), i = (int)(e % m);
    double v = A[i + (size_t)j * lda];
    if (!(v - v == 0.0)) atomicOr(flag, 1);
  }
}

int check_finite(const double* A, int m, int n, int lda, int* flag, hipStream_t s) {
  int nwg = cdiv((long long)m * n, 256);
  if (nwg > 1024) nwg = 1024;
  if (nwg < 1) nwg = 1;
  hipLaunchKernelGGL(finite_kernel, dim3(nwg), dim3(256), 0, s, A, m, n, lda, flag);
  JAC_CHECK_LAUNCH();
  return 0;
}

template <typename T>
__global__ void identity_kernel(T* __restrict__ V, int n, int ldv) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  int j = blockIdx.y;
  if (i < n) V[i + (size_t)j * ldv] = i == j ? T(1) : T(0);
}

template <typename T>
int set_identity(T* V, int n, int ldv, hipStream_t s) {
  if (n == 0) return 0;
  hipLaunchKernelGGL((identity_kernel<T>), dim3(cdiv(n, 256), n), dim3(256), 0, s, V, n, ldv);
  JAC_CHECK_LAUNCH();
  return 0;
}

template <typename Tin, typename Tout>
__global__ void convert_kernel(const Tin* __restrict__ A, int m, int lda, Tout* __restrict__ B, int ldb) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  int j = blockIdx.y;
  if (i < m) B[i + (size_t)j * ldb] = (Tout)A[i + (size_t)j * lda];
}

template <typename Tin, typename Tout>
int copy_convert(const Tin* A, int m, int n, int lda, Tout* B, int ldb, hipStream_t s) {
  if (m == 0 || n == 0) return 0;
  hipLaunchKernelGGL((convert_kernel<Tin, Tout>), dim3(cdiv(m, 256), n), dim3(256), 0, s, A, m, lda, B, ldb);
  JAC_CHECK_LAUNCH();
  return 0;
}

// Ascending order with ties kept in index order: rank(i) = #{j : d_j < d_i or
// (d_j == d_i and j < i)}.  A workgroup of 256 threads ranks 32 values: the d_j pass through LDS
// in chunks of 256, each of the 8 32-lane groups counts one eighth of every chunk, and the 8
// partial counts of a value are summed at the end (integer counts: the order does not matter).
template <typename T>
__global__ void __launch_bounds__(256) rank_kernel(const T* __restrict__ d, int n, int* __restrict__ rank,
                                                   double* __restrict__ W) {
  __shared__ T dc[256];
  __shared__ int part[8][32];
  const int tid = threadIdx.x, il = tid & 31, js = tid >> 5;
  const int i = blockIdx.x * 32 + il;
  const T di = i < n ? d[i] : T(0);
  int r = 0;
  for (int c = 0; c < n; c += 256) {
    __syncthreads();
    if (c + tid < n) dc[tid] = d[c + tid];
    __syncthreads();
    const int j0 = c + js * 32, cnt = min(32, n - j0);
    for (int q = 0; q < cnt; ++q) {
      const T dj = dc[js * 32 + q];
      r += (dj < di) || (dj == di && j0 + q < i);
    }
  }
  part[js][il] = r;
  __syncthreads();
  if (js == 0 && i < n) {
#pragma unroll
    for (int g = 1; g < 8; ++g) r += part[g][il];
    rank[i] = r;
    W[r] = (double)di;
  }
}

template <typename T>
__global__ void permute_cols_kernel(const T* __restrict__ Vw, int ldw, const int* __restrict__ rank, int n,
                                    double* __restrict__ Vout, int ldv) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  int j = blockIdx.y;
  if (i < n) Vout[i + (size_t)rank[j] * ldv] = (double)Vw[i + (size_t)j * ldw];
}

template <typename T>
int sort_eigs(const T* d, const T* Vw, int n, int ldw, double* W, double* Vout, int ldv, int* rank,
              hipStream_t s) {
  if (n == 0) return 0;
  hipLaunchKernelGGL((rank_kernel<T>), dim3(cdiv(n, 32)), dim3(256), 0, s, d, n, rank, W);
  JAC_CHECK_LAUNCH();
  if (Vout) {
    hipLaunchKernelGGL((permute_cols_kernel<T>), dim3(cdiv(n, 256), n), dim3(256), 0, s, Vw, ldw, rank, n,
                       Vout, ldv);
    JAC_CHECK_LAUNCH();
  }
  return 0;
}

// sigma_j = ||c_j|| (one workgroup per column, fixed reduction order).
__global__ void colnorm2_kernel(const double* __restrict__ C, int m, int ldc, double* __restrict__ sig) {
  __shared__ double red[4];
  const double* c = C + (size_t)blockIdx.x * ldc;
  double acc = 0;
  for (int i = threadIdx.x; i < m; i += 256) acc = fma(c[i], c[i], acc);
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) sig[blockIdx.x] = sqrt(red[0] + red[1] + red[2] + red[3]);
}

// Descending order, ties by index.
__global__ void rank_desc_kernel(const double* __restrict__ sig, int n, int* __restrict__ rank, double* __restrict__ S) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double v = sig[j];
  int r = 0;
  for (int i = 0; i < n; ++i) r += (sig[i] > v) || (sig[i] == v && i < j);
  rank[j] = r;
  S[r] = v;
}

// U(:, rank_j) = c_j / sigma_j (zero column if sigma_j = 0), V(:, rank_j) = v_j.
__global__ void svd_finish_kernel(const double* __restrict__ C, int m, int ldc, const double* __restrict__ Vw, int n,
                                  int ldvw, const double* __restrict__ sig, const int* __restrict__ rank,
                                  double* __restrict__ U, int ldu, double* __restrict__ V, int ldv) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  int j = blockIdx.y;
  int rj = rank[j];
  double sj = sig[j];
  if (i < m) U[i + (size_t)rj * ldu] = sj > 0 ? C[i + (size_t)j * ldc] / sj : 0.0;
  if (i < n) V[i + (size_t)rj * ldv] = Vw[i + (size_t)j * ldvw];
}

int svd_finish(const double* C, int m, int ldc, const double* Vw, int n, int ldvw, double* sig, int* rank,
               double* S, double* U, int ldu, double* V, int ldv, hipStream_t s) {
  if (n == 0) return 0;
  hipLaunchKernelGGL(colnorm2_kernel, dim3(n), dim3(256), 0, s, C, m, ldc, sig);
  JAC_CHECK_LAUNCH();
  hipLaunchKernelGGL(rank_desc_kernel, dim3(cdiv(n, 256)), dim3(256), 0, s, sig, n, rank, S);
  JAC_CHECK_LAUNCH();
  int rows = m > n ? m : n;
  hipLaunchKernelGGL(svd_finish_kernel, dim3(cdiv(rows, 256), n), dim3(256), 0, s, C, m, ldc, Vw, n, ldvw, sig, rank,
                     U, ldu, V, ldv);
  JAC_CHECK_LAUNCH();
  return 0;
}

template int set_identity<double>(double*, int, int, hipStream_t);
template int set_identity<float>(float*, int, int, hipStream_t);
template int copy_convert<double, float>(const double*, int, int, int, float*, int, hipStream_t);
template int copy_convert<float, double>(const float*, int, int, int, double*, int, hipStream_t);
template int copy_convert<double, double>(const double*, int, int, int, double*, int, hipStream_t);
template int copy_convert<float, float>(const float*, int, int, int, float*, int, hipStream_t);
template int sort_eigs<double>(const double*, const double*, int, int, double*, double*, int, int*, hipStream_t);
template int sort_eigs<float>(const float*, const float*, int, int, double*, double*, int, int*, hipStream_t);

// X <- fl_p(X scale) / scale in place (m x n, ldx): the value of precision p (FP16 or BF16, round to
// nearest even, reached through FP32) of each entry; scale is a power of two, so the scaling is exact.
__global__ void round_lowp_kernel(double* __restrict__ X, int m, int n, int ldx, int prec, double scale) {
  const int j = blockIdx.y;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) {
    double* x = X + i + (size_t)j * ldx;
    const float f = (float)(*x * scale);
    float r;
    if (prec == JAC_PREC_FP16) {
      r = __half2float(__float2half_rn(f));
    } else {   // BF16: keep the top 16 bits, rounded to nearest even
      unsigned int u = __float_as_uint(f);
      if ((u & 0x7F800000u) != 0x7F800000u) u += 0x7FFFu + ((u >> 16) & 1u);
      r = __uint_as_float(u & 0xFFFF0000u);
    }
    *x = (double)r / scale;
  }
}

int round_lowp(double* X, int m, int n, int ldx, int prec, double scale, hipStream_t s) {
  if (m <= 0 || n <= 0) return 0;
  int gx = (m + 255) / 256;
  if (gx > 16) gx = 16;
  hipLaunchKernelGGL(round_lowp_kernel, dim3(gx, n), dim3(256), 0, s, X, m, n, ldx, prec, scale);
  JAC_CHECK_LAUNCH();
  return 0;
}

}  // namespace jac
