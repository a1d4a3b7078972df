// Learned warm start (a project addition; the paper has no learned component): a three-layer
// perceptron theta (I values) -> H -> ReLU -> H -> ReLU -> O = n^2 values, read as the
// column-major entries of an approximate eigenvector matrix Z of A(theta), which then takes
// the place of the FP32 eigensolve (Algorithm 4.1, step 1) in front of MGS and Q^T A Q.
//
// Precision model: every matrix product takes bfloat16 operands, rounded to nearest even from
// FP32, and accumulates in FP32; the first layer (I <= 32 inputs) runs on the vector units with
// the same rounding, the other products on v_mfma_f32_16x16x32_bf16.  Biases, activations,
// gradients, the FP32 master weights and the AdamW moments are FP32.  W2 and W3 are also kept
// as bfloat16 copies, refreshed by the optimiser, so the large weight operand streams at two
// bytes per entry.
//
// Parameters are packed as [W1 (H x I), b1 (H), W2 (H x H), b2 (H), W3 (O x H), b3 (O)],
// row-major; activations are row-major (batch x features).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../include/jacobi.h"
#include "common.h"

struct jac_mlp {
  int I, H, n, O, maxB;
  long long P, oW1, ob1, oW2, ob2, oW3, ob3;
  long long t;  // optimiser steps taken
  float beta1, beta2, eps;
  float *p, *m, *v, *g;       // master weights, first and second moments, gradient
  uint16_t *w2b, *w3b;        // bfloat16 copies of W2 and W3
  float *H1, *H2, *dY, *dZ1, *dZ2;
  float* part;                // split-K partial products
  size_t part_elems;
  float* red;                 // per-workgroup loss partial sums
  int red_elems;
  void* mem;
};

namespace jac {

static inline int cdiv(long long a, long long b) { return (int)((a + b - 1) / b); }

// FP32 -> bfloat16 bits, round to nearest even (finite inputs).
__device__ __host__ inline uint16_t f2bf(float x) {
  uint32_t u = __builtin_bit_cast(uint32_t, x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __host__ inline float bf2f(uint16_t b) { return __builtin_bit_cast(float, (uint32_t)b << 16); }
__device__ inline float bfr(float x) { return bf2f(f2bf(x)); }

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------ BF16 GEMM
// C(m, n) = sum_k A(m, k) B(n, k) with
//   A(m, k) = A[m * lda + k]            (kind A_K: k contiguous, FP32)
//           = A[k * lda + m]            (kind A_M: m contiguous, FP32)
//   B(n, k) = B[n * ldb + k]            (kind B_K16: k contiguous, bfloat16)
//           = B[k * ldb + n]            (kind B_N32: n contiguous, FP32; B_N16: bfloat16)
// Operands are rounded to bfloat16 as they are staged into LDS ([row][k], k contiguous, rows
// padded to 40 entries so the 16-byte MFMA operand reads of 16 rows hit distinct banks).
// v_mfma_f32_16x16x32_bf16 takes 8 consecutive k of one row per lane (row lane % 16, k block
// lane / 16) from both operands and leaves row 4 (lane / 16) + r, column lane % 16 in
// accumulator r.  A workgroup of 4 waves (2 x 2) owns a 128 x 128 tile, each wave 64 x 64.
enum { A_K = 0, A_M = 1 };
enum { B_K16 = 0, B_N32 = 1, B_N16 = 2 };
enum { EPI_STORE = 0, EPI_BIAS = 1, EPI_BIAS_RELU = 2, EPI_MASK = 3, EPI_LOSS = 4, EPI_BIAS_F64 = 5 };

struct GemmArgs {
  int M, N, K, kchunk;
  const void* A;
  int lda;
  const void* B;
  int ldb;
  int epi;
  float* C;
  int ldc;
  const float* bias;
  const float* mask;  // EPI_MASK: keep C where mask(m, n) > 0 (same layout as C)
  const uint16_t* target;  // EPI_LOSS: bfloat16 targets, row stride ldt
  long long ldt;
  float scale;        // EPI_LOSS: C = scale * (acc + bias - target)
  float* red;         // EPI_LOSS: one sum of squared differences per workgroup
  double* Cd;         // EPI_BIAS_F64: column-major n x n matrix of the single sample
  int nsq, ldz;
  float* part;        // split-K: S x M x N partial products (row-major per slice)
};

constexpr int kGB = 128, kGK = 32, kGPad = 8, kGLd = kGK + kGPad;

__device__ inline float epilogue(const GemmArgs& a, int m, int n, float acc) {
  switch (a.epi) {
    case EPI_BIAS: return acc + a.bias[n];
    case EPI_BIAS_RELU: return fmaxf(acc + a.bias[n], 0.0f);
    case EPI_MASK: return a.mask[(size_t)m * a.ldc + n] > 0.0f ? acc : 0.0f;
    default: return acc;
  }
}

template <int AK, int BK>
__global__ void __launch_bounds__(256) bf16_gemm_kernel(GemmArgs a) {
  __shared__ __attribute__((aligned(16))) uint16_t As[2][kGB][kGLd];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[2][kGB][kGLd];
  __shared__ float wred[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int m0 = blockIdx.y * kGB, n0 = blockIdx.x * kGB;
  const int kb = blockIdx.z * a.kchunk;
  const int ke = min(a.K, kb + a.kchunk);

  f32x4_t acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f32x4_t{0, 0, 0, 0};

  float4 ra[4];
  uint4 rb16[2];
  float4 rb32[4];

  auto load_a = [&](int k0) {
    const float* A = static_cast<const float*>(a.A);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      int idx = tid + e * 256;
      if (AK == A_K) {
        int row = idx >> 3, kq = idx & 7;
        int gm = m0 + row;
        ra[e] = gm < a.M ? *reinterpret_cast<const float4*>(A + (size_t)gm * a.lda + k0 + 4 * kq)
                         : make_float4(0, 0, 0, 0);
      } else {
        int kk = idx >> 5, mq = idx & 31;
        int gm = m0 + 4 * mq, gk = k0 + kk;
        ra[e] = (gm < a.M && gk < ke) ? *reinterpret_cast<const float4*>(A + (size_t)gk * a.lda + gm)
                                      : make_float4(0, 0, 0, 0);
      }
    }
  };
  auto load_b = [&](int k0) {
    if (BK == B_K16) {
      const uint16_t* B = static_cast<const uint16_t*>(a.B);
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        int idx = tid + e * 256;
        int row = idx >> 2, kq = idx & 3;
        int gn = n0 + row;
        rb16[e] = gn < a.N ? *reinterpret_cast<const uint4*>(B + (size_t)gn * a.ldb + k0 + 8 * kq)
                           : make_uint4(0, 0, 0, 0);
      }
    } else if (BK == B_N16) {
      const uint16_t* B = static_cast<const uint16_t*>(a.B);
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        int idx = tid + e * 256;
        int kk = idx >> 4, nq = idx & 15;
        int gn = n0 + 8 * nq, gk = k0 + kk;
        rb16[e] = (gn < a.N && gk < ke) ? *reinterpret_cast<const uint4*>(B + (size_t)gk * a.ldb + gn)
                                        : make_uint4(0, 0, 0, 0);
      }
    } else {
      const float* B = static_cast<const float*>(a.B);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        int idx = tid + e * 256;
        int kk = idx >> 5, nq = idx & 31;
        int gn = n0 + 4 * nq, gk = k0 + kk;
        rb32[e] = (gn < a.N && gk < ke) ? *reinterpret_cast<const float4*>(B + (size_t)gk * a.ldb + gn)
                                        : make_float4(0, 0, 0, 0);
      }
    }
  };
  auto store_ab = [&](int buf) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      int idx = tid + e * 256;
      if (AK == A_K) {
        int row = idx >> 3, kq = idx & 7;
        uint2 w;
        w.x = (uint32_t)f2bf(ra[e].x) | ((uint32_t)f2bf(ra[e].y) << 16);
        w.y = (uint32_t)f2bf(ra[e].z) | ((uint32_t)f2bf(ra[e].w) << 16);
        *reinterpret_cast<uint2*>(&As[buf][row][4 * kq]) = w;
      } else {
        int kk = idx >> 5, mq = idx & 31;
        As[buf][4 * mq + 0][kk] = f2bf(ra[e].x);
        As[buf][4 * mq + 1][kk] = f2bf(ra[e].y);
        As[buf][4 * mq + 2][kk] = f2bf(ra[e].z);
        As[buf][4 * mq + 3][kk] = f2bf(ra[e].w);
      }
    }
    if (BK == B_K16) {
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        int idx = tid + e * 256;
        int row = idx >> 2, kq = idx & 3;
        *reinterpret_cast<uint4*>(&Bs[buf][row][8 * kq]) = rb16[e];
      }
    } else if (BK == B_N16) {
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        int idx = tid + e * 256;
        int kk = idx >> 4, nq = idx & 15;
        const uint32_t w[4] = {rb16[e].x, rb16[e].y, rb16[e].z, rb16[e].w};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          Bs[buf][8 * nq + 2 * q][kk] = (uint16_t)(w[q] & 0xFFFFu);
          Bs[buf][8 * nq + 2 * q + 1][kk] = (uint16_t)(w[q] >> 16);
        }
      }
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        int idx = tid + e * 256;
        int kk = idx >> 5, nq = idx & 31;
        Bs[buf][4 * nq + 0][kk] = f2bf(rb32[e].x);
        Bs[buf][4 * nq + 1][kk] = f2bf(rb32[e].y);
        Bs[buf][4 * nq + 2][kk] = f2bf(rb32[e].z);
        Bs[buf][4 * nq + 3][kk] = f2bf(rb32[e].w);
      }
    }
  };

  int buf = 0;
  if (kb < ke) {
    load_a(kb);
    load_b(kb);
    store_ab(0);
  }
  __syncthreads();
  const int r16 = lane & 15, kq = (lane >> 4) * 8;
  for (int k0 = kb; k0 < ke; k0 += kGK) {
    const bool more = k0 + kGK < ke;
    if (more) {
      load_a(k0 + kGK);
      load_b(k0 + kGK);
    }
    bf16x8_t af[4], bfv[4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
      af[i] = __builtin_bit_cast(bf16x8_t, *reinterpret_cast<const uint4*>(&As[buf][wm * 64 + i * 16 + r16][kq]));
#pragma unroll
    for (int j = 0; j < 4; ++j)
      bfv[j] = __builtin_bit_cast(bf16x8_t, *reinterpret_cast<const uint4*>(&Bs[buf][wn * 64 + j * 16 + r16][kq]));
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfv[j], acc[i][j], 0, 0, 0);
    if (more) {
      store_ab(buf ^ 1);
      __syncthreads();
      buf ^= 1;
    }
  }

  float sq = 0.0f;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int gn = n0 + wn * 64 + j * 16 + r16;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gm = m0 + wm * 64 + i * 16 + 4 * (lane >> 4) + r;
        if (gm >= a.M || gn >= a.N) continue;
        const float x = acc[i][j][r];
        if (a.part) {
          a.part[((size_t)blockIdx.z * a.M + gm) * a.N + gn] = x;
        } else if (a.epi == EPI_LOSS) {
          const float d = x + a.bias[gn] - bf2f(a.target[(size_t)gm * a.ldt + gn]);
          sq = fmaf(d, d, sq);
          a.C[(size_t)gm * a.ldc + gn] = a.scale * d;
        } else if (a.epi == EPI_BIAS_F64) {
          a.Cd[(gn % a.nsq) + (size_t)(gn / a.nsq) * a.ldz] = (double)(x + a.bias[gn]);
        } else {
          a.C[(size_t)gm * a.ldc + gn] = epilogue(a, gm, gn, x);
        }
      }
    }
  if (a.epi == EPI_LOSS && !a.part) {
    for (int o = 32; o > 0; o >>= 1) sq += __shfl_down(sq, o, 64);
    if (lane == 0) wred[wave] = sq;
    __syncthreads();
    if (tid == 0) a.red[blockIdx.y * gridDim.x + blockIdx.x] = (wred[0] + wred[1]) + (wred[2] + wred[3]);
  }
}

// Sum of the split-K slices in slice order, then the epilogue.
__global__ void splitk_sum_kernel(GemmArgs a, int S) {
  const size_t mn = (size_t)a.M * a.N;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < mn; e += (size_t)gridDim.x * blockDim.x) {
    float x = 0.0f;
    for (int z = 0; z < S; ++z) x += a.part[z * mn + e];
    const int gm = (int)(e / a.N), gn = (int)(e % a.N);
    a.C[(size_t)gm * a.ldc + gn] = epilogue(a, gm, gn, x);
  }
}

static int gemm_bf16(int akind, int bkind, GemmArgs a, float* part, size_t part_elems, hipStream_t s) {
  if (a.M <= 0 || a.N <= 0) return 0;
  const int tiles = cdiv(a.M, kGB) * cdiv(a.N, kGB);
  int S = 1;
  if (part && a.epi != EPI_LOSS && a.epi != EPI_BIAS_F64 && tiles < 256 && a.K >= 512) {
    S = cdiv(512, tiles);
    if (S > a.K / 256) S = a.K / 256;
    while (S > 1 && (size_t)S * a.M * a.N > part_elems) --S;
    if (S < 1) S = 1;
  }
  a.kchunk = cdiv(cdiv(a.K, S), kGK) * kGK;
  S = a.K > 0 ? cdiv(a.K, a.kchunk) : 1;
  if (S < 1) S = 1;
  a.part = S > 1 ? part : nullptr;
  dim3 grid(cdiv(a.N, kGB), cdiv(a.M, kGB), S);
  if (akind == A_K && bkind == B_K16)
    hipLaunchKernelGGL((bf16_gemm_kernel<A_K, B_K16>), grid, dim3(256), 0, s, a);
  else if (akind == A_M && bkind == B_N32)
    hipLaunchKernelGGL((bf16_gemm_kernel<A_M, B_N32>), grid, dim3(256), 0, s, a);
  else if (akind == A_K && bkind == B_N16)
    hipLaunchKernelGGL((bf16_gemm_kernel<A_K, B_N16>), grid, dim3(256), 0, s, a);
  else {
    set_error("gemm_bf16: unsupported operand layout");
    return -1;
  }
  JAC_CHECK_LAUNCH();
  if (S > 1) {
    int nb = cdiv((long long)a.M * a.N, 256);
    if (nb > 4096) nb = 4096;
    hipLaunchKernelGGL(splitk_sum_kernel, dim3(nb), dim3(256), 0, s, a, S);
    JAC_CHECK_LAUNCH();
  }
  return 0;
}

// ------------------------------------------------------------------ first layer (I <= 32)
constexpr int kMaxIn = 32;

__global__ void l1_forward_kernel(const float* __restrict__ X, int B, int I, const float* __restrict__ W1,
                                  const float* __restrict__ b1, int H, float* __restrict__ H1) {
  const int h = blockIdx.x * blockDim.x + threadIdx.x, b = blockIdx.y;
  if (h >= H || b >= B) return;
  float acc = 0.0f;
  for (int i = 0; i < I; ++i) acc = fmaf(bfr(X[(size_t)b * I + i]), bfr(W1[(size_t)h * I + i]), acc);
  H1[(size_t)b * H + h] = fmaxf(acc + b1[h], 0.0f);
}

// dW1(h, i) = sum_b bf(dZ1(b, h)) bf(X(b, i)), db1(h) = sum_b dZ1(b, h).
__global__ void l1_backward_kernel(const float* __restrict__ dZ1, const float* __restrict__ X, int B, int I, int H,
                                   float* __restrict__ gW1, float* __restrict__ gb1) {
  const int h = blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= H) return;
  float acc[kMaxIn];
#pragma unroll
  for (int i = 0; i < kMaxIn; ++i) acc[i] = 0.0f;
  float sb = 0.0f;
  for (int b = 0; b < B; ++b) {
    const float d = dZ1[(size_t)b * H + h];
    const float dr = bfr(d);
    sb += d;
#pragma unroll
    for (int i = 0; i < kMaxIn; ++i)
      if (i < I) acc[i] = fmaf(dr, bfr(X[(size_t)b * I + i]), acc[i]);
  }
#pragma unroll
  for (int i = 0; i < kMaxIn; ++i)
    if (i < I) gW1[(size_t)h * I + i] = acc[i];
  gb1[h] = sb;
}

// out(n) = sum_b D(b, n) in batch order.
__global__ void colsum_kernel(const float* __restrict__ D, int B, int N, int ld, float* __restrict__ out) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  float s = 0.0f;
  for (int b = 0; b < B; ++b) s += D[(size_t)b * ld + n];
  out[n] = s;
}

__global__ void loss_final_kernel(const float* __restrict__ red, int count, float inv, float* __restrict__ loss) {
  __shared__ float w[16];
  float s = 0.0f;
  for (int i = threadIdx.x; i < count; i += blockDim.x) s += red[i];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
  if ((threadIdx.x & 63) == 0) w[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    float t = 0.0f;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += w[i];
    *loss = t * inv;
  }
}

// ------------------------------------------------------------------ optimiser
// AdamW (decoupled weight decay): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
// p -= lr (c1 m / (sqrt(c2 v) + eps) + wd p) with c1 = 1/(1-b1^t), c2 = 1/(1-b2^t); the new
// W2 and W3 are also written as bfloat16.
__global__ void adamw_kernel(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                             const float* __restrict__ g, long long P, float lr, float wd, float b1, float b2,
                             float eps, float c1, float c2, uint16_t* __restrict__ w2b, long long oW2, long long nW2,
                             uint16_t* __restrict__ w3b, long long oW3, long long nW3) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < P;
       i += (long long)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    const float pi = p[i];
    const float pn = pi - lr * ((mi * c1) / (sqrtf(vi * c2) + eps) + wd * pi);
    m[i] = mi;
    v[i] = vi;
    p[i] = pn;
    if (i >= oW3 && i < oW3 + nW3) w3b[i - oW3] = f2bf(pn);
    else if (i >= oW2 && i < oW2 + nW2) w2b[i - oW2] = f2bf(pn);
  }
}

__global__ void to_bf16_kernel(const float* __restrict__ x, long long count, uint16_t* __restrict__ y) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (long long)gridDim.x * blockDim.x)
    y[i] = f2bf(x[i]);
}

// Initial weights: uniform in [-a, a] from SplitMix64 of (seed, index); biases zero.
__device__ inline uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

__global__ void init_uniform_kernel(float* __restrict__ p, long long off, long long count, float a,
                                    unsigned long long seed) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (long long)gridDim.x * blockDim.x) {
    const uint64_t r = splitmix64(seed ^ (uint64_t)(off + i) * 0xD1B54A32D192ED03ull);
    const float u = (float)((r >> 40) * (1.0 / 16777216.0));  // [0, 1), 24 bits
    p[off + i] = a * (2.0f * u - 1.0f);
  }
}

// Training targets: per column of each eigenvector matrix the entry of largest magnitude (the
// first one on ties) is made positive; the column-major entries are rounded to bfloat16 (from
// their FP32 value).  One workgroup per (column, matrix).
__global__ void pack_targets_kernel(const double* __restrict__ V, int n, int ldv, long long stride_v,
                                    uint16_t* __restrict__ T, long long ldt, int canonical) {
  __shared__ double bv[4];
  __shared__ int bi[4];
  const int j = blockIdx.x, c = blockIdx.y, tid = threadIdx.x;
  const double* col = V + c * stride_v + (size_t)j * ldv;
  double best = -1.0;
  int besti = 0x7fffffff;
  for (int i = tid; i < n; i += blockDim.x) {
    const double a = fabs(col[i]);
    if (a > best) { best = a; besti = i; }  // i increases: ties keep the first
  }
  for (int o = 32; o > 0; o >>= 1) {
    const double ob = __shfl_down(best, o, 64);
    const int oi = __shfl_down(besti, o, 64);
    if (ob > best || (ob == best && oi < besti)) { best = ob; besti = oi; }
  }
  if ((tid & 63) == 0) { bv[tid >> 6] = best; bi[tid >> 6] = besti; }
  __syncthreads();
  if (tid == 0) {
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w)
      if (bv[w] > bv[0] || (bv[w] == bv[0] && bi[w] < bi[0])) { bv[0] = bv[w]; bi[0] = bi[w]; }
  }
  __syncthreads();
  const double sgn = (canonical && col[bi[0]] < 0.0) ? -1.0 : 1.0;
  uint16_t* out = T + c * ldt + (size_t)j * n;
  for (int i = tid; i < n; i += blockDim.x) out[i] = f2bf((float)(sgn * col[i]));
}

// ------------------------------------------------------------------ network passes
static int forward_hidden(jac_mlp* net, const float* X, int B, hipStream_t s) {
  hipLaunchKernelGGL(l1_forward_kernel, dim3(cdiv(net->H, 256), B), dim3(256), 0, s, X, B, net->I,
                     net->p + net->oW1, net->p + net->ob1, net->H, net->H1);
  JAC_CHECK_LAUNCH();
  GemmArgs a{};
  a.M = B; a.N = net->H; a.K = net->H;
  a.A = net->H1; a.lda = net->H;
  a.B = net->w2b; a.ldb = net->H;
  a.epi = EPI_BIAS_RELU; a.C = net->H2; a.ldc = net->H; a.bias = net->p + net->ob2;
  return gemm_bf16(A_K, B_K16, a, net->part, net->part_elems, s);
}

static int backward(jac_mlp* net, const float* X, int B, hipStream_t s) {
  const int H = net->H, O = net->O;
  float* g = net->g;
  int e;
  hipLaunchKernelGGL(colsum_kernel, dim3(cdiv(O, 256)), dim3(256), 0, s, net->dY, B, O, O, g + net->ob3);
  JAC_CHECK_LAUNCH();
  {  // dW3 = bf(dY)^T bf(H2)
    GemmArgs a{};
    a.M = O; a.N = H; a.K = B;
    a.A = net->dY; a.lda = O;
    a.B = net->H2; a.ldb = H;
    a.epi = EPI_STORE; a.C = g + net->oW3; a.ldc = H;
    if ((e = gemm_bf16(A_M, B_N32, a, nullptr, 0, s))) return e;
  }
  {  // dZ2 = (bf(dY) bf(W3)) * [H2 > 0]
    GemmArgs a{};
    a.M = B; a.N = H; a.K = O;
    a.A = net->dY; a.lda = O;
    a.B = net->w3b; a.ldb = H;
    a.epi = EPI_MASK; a.mask = net->H2; a.C = net->dZ2; a.ldc = H;
    if ((e = gemm_bf16(A_K, B_N16, a, net->part, net->part_elems, s))) return e;
  }
  hipLaunchKernelGGL(colsum_kernel, dim3(cdiv(H, 256)), dim3(256), 0, s, net->dZ2, B, H, H, g + net->ob2);
  JAC_CHECK_LAUNCH();
  {  // dW2 = bf(dZ2)^T bf(H1)
    GemmArgs a{};
    a.M = H; a.N = H; a.K = B;
    a.A = net->dZ2; a.lda = H;
    a.B = net->H1; a.ldb = H;
    a.epi = EPI_STORE; a.C = g + net->oW2; a.ldc = H;
    if ((e = gemm_bf16(A_M, B_N32, a, nullptr, 0, s))) return e;
  }
  {  // dZ1 = (bf(dZ2) bf(W2)) * [H1 > 0]
    GemmArgs a{};
    a.M = B; a.N = H; a.K = H;
    a.A = net->dZ2; a.lda = H;
    a.B = net->w2b; a.ldb = H;
    a.epi = EPI_MASK; a.mask = net->H1; a.C = net->dZ1; a.ldc = H;
    if ((e = gemm_bf16(A_K, B_N16, a, net->part, net->part_elems, s))) return e;
  }
  hipLaunchKernelGGL(l1_backward_kernel, dim3(cdiv(H, 64)), dim3(64), 0, s, net->dZ1, X, B, net->I, H,
                     g + net->oW1, g + net->ob1);
  JAC_CHECK_LAUNCH();
  return 0;
}

static int loss_and_grads(jac_mlp* net, const float* X, const uint16_t* T, long long ldt, int B, float* loss,
                          hipStream_t s) {
  int e = forward_hidden(net, X, B, s);
  if (e) return e;
  GemmArgs a{};
  a.M = B; a.N = net->O; a.K = net->H;
  a.A = net->H2; a.lda = net->H;
  a.B = net->w3b; a.ldb = net->H;
  a.epi = EPI_LOSS; a.C = net->dY; a.ldc = net->O; a.bias = net->p + net->ob3;
  a.target = T; a.ldt = ldt;
  a.scale = (float)(2.0 / ((double)B * net->O));
  a.red = net->red;
  if ((e = gemm_bf16(A_K, B_K16, a, nullptr, 0, s))) return e;
  const int nred = cdiv(net->O, kGB) * cdiv(B, kGB);
  if (loss) {
    hipLaunchKernelGGL(loss_final_kernel, dim3(1), dim3(1024), 0, s, net->red, nred,
                       (float)(1.0 / ((double)B * net->O)), loss);
    JAC_CHECK_LAUNCH();
  }
  return backward(net, X, B, s);
}

static int refresh_bf16(jac_mlp* net, hipStream_t s) {
  long long n2 = (long long)net->H * net->H, n3 = (long long)net->O * net->H;
  hipLaunchKernelGGL(to_bf16_kernel, dim3(1024), dim3(256), 0, s, net->p + net->oW2, n2, net->w2b);
  JAC_CHECK_LAUNCH();
  hipLaunchKernelGGL(to_bf16_kernel, dim3(4096), dim3(256), 0, s, net->p + net->oW3, n3, net->w3b);
  JAC_CHECK_LAUNCH();
  return 0;
}

// Z (column-major n x n, leading dimension ldz) for one theta (device, I floats).
int mlp_predict_f64(const jac_mlp* cnet, const float* theta, double* Z, int ldz, hipStream_t s) {
  jac_mlp* net = const_cast<jac_mlp*>(cnet);
  int e = forward_hidden(net, theta, 1, s);
  if (e) return e;
  GemmArgs a{};
  a.M = 1; a.N = net->O; a.K = net->H;
  a.A = net->H2; a.lda = net->H;
  a.B = net->w3b; a.ldb = net->H;
  a.epi = EPI_BIAS_F64; a.bias = net->p + net->ob3;
  a.Cd = Z; a.nsq = net->n; a.ldz = ldz;
  return gemm_bf16(A_K, B_K16, a, nullptr, 0, s);
}

int mlp_order(const jac_mlp* net) { return net ? net->n : -1; }

}  // namespace jac

using namespace jac;

static hipStream_t as_stream(void* s) { return static_cast<hipStream_t>(s); }

extern "C" {

int jac_mlp_create(int n_in, int hidden, int n, int max_batch, unsigned long long seed, jac_mlp** out) {
  if (!out) { set_error("jac_mlp_create: out is NULL"); return -6; }
  *out = nullptr;
  if (n_in < 1 || n_in > kMaxIn) { set_error("jac_mlp_create: n_in must be in [1, 32]"); return -1; }
  if (hidden < 32 || hidden % 32) { set_error("jac_mlp_create: hidden must be a positive multiple of 32"); return -2; }
  if (n < 1 || ((long long)n * n) % 32) { set_error("jac_mlp_create: n^2 must be a positive multiple of 32"); return -3; }
  if (max_batch < 1) { set_error("jac_mlp_create: max_batch must be >= 1"); return -4; }
  jac_mlp* net = new jac_mlp{};
  net->I = n_in; net->H = hidden; net->n = n; net->O = n * n; net->maxB = max_batch;
  const long long I = n_in, H = hidden, O = (long long)n * n, B = max_batch;
  net->oW1 = 0; net->ob1 = H * I; net->oW2 = net->ob1 + H; net->ob2 = net->oW2 + H * H;
  net->oW3 = net->ob2 + H; net->ob3 = net->oW3 + O * H; net->P = net->ob3 + O;
  net->beta1 = 0.9f; net->beta2 = 0.999f; net->eps = 1e-8f;
  net->part_elems = (size_t)std::min<long long>(64, std::max<long long>(1, O / 256)) * B * H;
  net->red_elems = cdiv(O, kGB) * cdiv(B, kGB);
  size_t bytes = 0;
  auto add = [&](size_t b) { size_t o = bytes; bytes += align_up(b, 256); return o; };
  size_t op = add(net->P * 4), om = add(net->P * 4), ov = add(net->P * 4), og = add(net->P * 4);
  size_t ow2 = add(H * H * 2), ow3 = add(O * H * 2);
  size_t oh1 = add(B * H * 4), oh2 = add(B * H * 4), ody = add(B * O * 4), odz1 = add(B * H * 4),
         odz2 = add(B * H * 4);
  size_t opart = add(net->part_elems * 4), ored = add((size_t)net->red_elems * 4);
  if (hipMalloc(&net->mem, bytes) != hipSuccess) {
    delete net;
    set_error("jac_mlp_create: device allocation failed");
    return 4;
  }
  char* b = static_cast<char*>(net->mem);
  net->p = (float*)(b + op); net->m = (float*)(b + om); net->v = (float*)(b + ov); net->g = (float*)(b + og);
  net->w2b = (uint16_t*)(b + ow2); net->w3b = (uint16_t*)(b + ow3);
  net->H1 = (float*)(b + oh1); net->H2 = (float*)(b + oh2); net->dY = (float*)(b + ody);
  net->dZ1 = (float*)(b + odz1); net->dZ2 = (float*)(b + odz2);
  net->part = (float*)(b + opart); net->red = (float*)(b + ored);
  hipStream_t s = nullptr;
  auto fail = [&]() { (void)hipFree(net->mem); delete net; return 4; };
  if (hipMemsetAsync(net->mem, 0, bytes, s) != hipSuccess) return fail();
  const float a1 = std::sqrt(6.0f / I), a2 = std::sqrt(6.0f / H), a3 = std::sqrt(3.0f / H);
  hipLaunchKernelGGL(init_uniform_kernel, dim3(64), dim3(256), 0, s, net->p, net->oW1, H * I, a1, seed);
  hipLaunchKernelGGL(init_uniform_kernel, dim3(1024), dim3(256), 0, s, net->p, net->oW2, H * H, a2, seed);
  hipLaunchKernelGGL(init_uniform_kernel, dim3(4096), dim3(256), 0, s, net->p, net->oW3, O * H, a3, seed);
  if (hipGetLastError() != hipSuccess) return fail();
  if (refresh_bf16(net, s) != 0 || hipStreamSynchronize(s) != hipSuccess) return fail();
  *out = net;
  return 0;
}

void jac_mlp_free(jac_mlp* net) {
  if (!net) return;
  (void)hipDeviceSynchronize();
  (void)hipFree(net->mem);
  delete net;
}

long long jac_mlp_num_params(const jac_mlp* net) { return net ? net->P : -1; }

int jac_mlp_shape(const jac_mlp* net, int* n_in, int* hidden, int* n, int* max_batch, long long* steps) {
  if (!net) { set_error("jac_mlp_shape: net is NULL"); return -1; }
  if (n_in) *n_in = net->I;
  if (hidden) *hidden = net->H;
  if (n) *n = net->n;
  if (max_batch) *max_batch = net->maxB;
  if (steps) *steps = net->t;
  return 0;
}

static float* buffer_of(const jac_mlp* net, int which) {
  switch (which) {
    case JAC_MLP_PARAMS: return net->p;
    case JAC_MLP_GRADS: return net->g;
    case JAC_MLP_MOMENT1: return net->m;
    case JAC_MLP_MOMENT2: return net->v;
    default: return nullptr;
  }
}

int jac_mlp_get(const jac_mlp* net, int which, float* host) {
  if (!net || !host) { set_error("jac_mlp_get: NULL argument"); return -1; }
  float* src = buffer_of(net, which);
  if (!src) { set_error("jac_mlp_get: unknown buffer"); return -2; }
  JAC_HIP(hipDeviceSynchronize());
  JAC_HIP(hipMemcpy(host, src, net->P * sizeof(float), hipMemcpyDeviceToHost));
  return 0;
}

int jac_mlp_set(jac_mlp* net, int which, const float* host) {
  if (!net || !host) { set_error("jac_mlp_set: NULL argument"); return -1; }
  float* dst = buffer_of(net, which);
  if (!dst) { set_error("jac_mlp_set: unknown buffer"); return -2; }
  JAC_HIP(hipDeviceSynchronize());
  JAC_HIP(hipMemcpy(dst, host, net->P * sizeof(float), hipMemcpyHostToDevice));
  if (which == JAC_MLP_PARAMS) {
    int e = refresh_bf16(net, nullptr);
    if (e) return e;
    JAC_HIP(hipStreamSynchronize(nullptr));
  }
  return 0;
}

int jac_mlp_set_adam(jac_mlp* net, float beta1, float beta2, float eps, long long steps) {
  if (!net) { set_error("jac_mlp_set_adam: net is NULL"); return -1; }
  if (!(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0) || steps < 0) {
    set_error("jac_mlp_set_adam: need 0 <= beta < 1, eps > 0, steps >= 0");
    return -2;
  }
  net->beta1 = beta1; net->beta2 = beta2; net->eps = eps; net->t = steps;
  return 0;
}

int jac_mlp_forward(jac_mlp* net, const float* theta, int batch, float* Y, int ldy, void* stream) {
  if (!net || !theta || !Y) { set_error("jac_mlp_forward: NULL argument"); return -1; }
  if (batch < 0 || batch > net->maxB) { set_error("jac_mlp_forward: batch outside [0, max_batch]"); return -3; }
  if (ldy < net->O) { set_error("jac_mlp_forward: ldy < n^2"); return -5; }
  if (batch == 0) return 0;
  hipStream_t s = as_stream(stream);
  int e = forward_hidden(net, theta, batch, s);
  if (e) return e;
  GemmArgs a{};
  a.M = batch; a.N = net->O; a.K = net->H;
  a.A = net->H2; a.lda = net->H;
  a.B = net->w3b; a.ldb = net->H;
  a.epi = EPI_BIAS; a.C = Y; a.ldc = ldy; a.bias = net->p + net->ob3;
  return gemm_bf16(A_K, B_K16, a, nullptr, 0, s);
}

int jac_mlp_predict(const jac_mlp* net, const float* theta, double* Z, int ldz, void* stream) {
  if (!net || !theta || !Z) { set_error("jac_mlp_predict: NULL argument"); return -1; }
  if (ldz < net->n) { set_error("jac_mlp_predict: ldz < n"); return -4; }
  return mlp_predict_f64(net, theta, Z, ldz, as_stream(stream));
}

int jac_mlp_grads(jac_mlp* net, const float* theta, const unsigned short* target, long long ldt, int batch, float* loss,
                  void* stream) {
  if (!net || !theta || !target) { set_error("jac_mlp_grads: NULL argument"); return -1; }
  if (batch < 1 || batch > net->maxB) { set_error("jac_mlp_grads: batch outside [1, max_batch]"); return -5; }
  if (ldt < net->O) { set_error("jac_mlp_grads: ldt < n^2"); return -4; }
  return loss_and_grads(net, theta, target, ldt, batch, loss, as_stream(stream));
}

int jac_mlp_adamw(jac_mlp* net, float lr, float weight_decay, void* stream) {
  if (!net) { set_error("jac_mlp_adamw: net is NULL"); return -1; }
  if (!(lr >= 0) || !(weight_decay >= 0)) { set_error("jac_mlp_adamw: lr and weight_decay must be >= 0"); return -2; }
  net->t += 1;
  const double c1 = 1.0 / (1.0 - std::pow((double)net->beta1, (double)net->t));
  const double c2 = 1.0 / (1.0 - std::pow((double)net->beta2, (double)net->t));
  hipLaunchKernelGGL(adamw_kernel, dim3(8192), dim3(256), 0, as_stream(stream), net->p, net->m, net->v, net->g,
                     net->P, lr, weight_decay, net->beta1, net->beta2, net->eps, (float)c1, (float)c2, net->w2b,
                     net->oW2, (long long)net->H * net->H, net->w3b, net->oW3, (long long)net->O * net->H);
  JAC_CHECK_LAUNCH();
  return 0;
}

int jac_mlp_train_step(jac_mlp* net, const float* theta, const uint16_t* target, long long ldt, int batch, float lr,
                       float weight_decay, float* loss, void* stream) {
  int e = jac_mlp_grads(net, theta, target, ldt, batch, loss, stream);
  if (e) return e;
  return jac_mlp_adamw(net, lr, weight_decay, stream);
}

int jac_mlp_pack_targets_ex(const double* V, int n, int ldv, long long stride_v, int count, uint16_t* T,
                            long long ldt, int sign_mode, void* stream) {
  if (n < 0 || count < 0) { set_error("jac_mlp_pack_targets: negative size"); return -2; }
  if (sign_mode != 0 && sign_mode != 1) { set_error("jac_mlp_pack_targets_ex: sign_mode must be 0 or 1"); return -8; }
  if (n == 0 || count == 0) return 0;
  if (!V || !T) { set_error("jac_mlp_pack_targets: NULL argument"); return -1; }
  if (ldv < n) { set_error("jac_mlp_pack_targets: ldv < n"); return -3; }
  if (count > 1 && stride_v < (long long)ldv * n) { set_error("jac_mlp_pack_targets: stride_v < ldv * n"); return -4; }
  if (count > 1 && ldt < (long long)n * n) { set_error("jac_mlp_pack_targets: ldt < n^2"); return -7; }
  if (count > 65535) { set_error("jac_mlp_pack_targets: count > 65535"); return -5; }
  hipLaunchKernelGGL(pack_targets_kernel, dim3(n, count), dim3(256), 0, as_stream(stream), V, n, ldv, stride_v, T,
                     ldt, sign_mode == 0 ? 1 : 0);
  JAC_CHECK_LAUNCH();
  return 0;
}

int jac_mlp_pack_targets(const double* V, int n, int ldv, long long stride_v, int count, uint16_t* T, long long ldt,
                         void* stream) {
  return jac_mlp_pack_targets_ex(V, n, ldv, stride_v, count, T, ldt, 0, stream);
}

// File layout: "JACMLP01", int32 I, H, n, int64 steps, float beta1, beta2, eps, then P floats
// each of the weights, first moments and second moments (little-endian).
int jac_mlp_save(const jac_mlp* net, const char* path) {
  if (!net || !path) { set_error("jac_mlp_save: NULL argument"); return -1; }
  std::vector<float> buf((size_t)net->P);
  FILE* f = std::fopen(path, "wb");
  if (!f) { set_error(std::string("jac_mlp_save: cannot open ") + path); return 5; }
  bool ok = std::fwrite("JACMLP01", 1, 8, f) == 8;
  const int dims[3] = {net->I, net->H, net->n};
  const float hp[3] = {net->beta1, net->beta2, net->eps};
  ok = ok && std::fwrite(dims, 4, 3, f) == 3 && std::fwrite(&net->t, 8, 1, f) == 1 && std::fwrite(hp, 4, 3, f) == 3;
  for (int w = 0; ok && w < 3; ++w) {
    int e = jac_mlp_get(net, w == 0 ? JAC_MLP_PARAMS : w == 1 ? JAC_MLP_MOMENT1 : JAC_MLP_MOMENT2, buf.data());
    if (e) { std::fclose(f); return e; }
    ok = std::fwrite(buf.data(), 4, buf.size(), f) == buf.size();
  }
  if (std::fclose(f) != 0) ok = false;
  if (!ok) { set_error(std::string("jac_mlp_save: write failed on ") + path); return 5; }
  return 0;
}

int jac_mlp_load(jac_mlp* net, const char* path) {
  if (!net || !path) { set_error("jac_mlp_load: NULL argument"); return -1; }
  FILE* f = std::fopen(path, "rb");
  if (!f) { set_error(std::string("jac_mlp_load: cannot open ") + path); return 5; }
  char magic[8];
  int dims[3];
  long long t = 0;
  float hp[3];
  bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "JACMLP01", 8) == 0 &&
            std::fread(dims, 4, 3, f) == 3 && std::fread(&t, 8, 1, f) == 1 && std::fread(hp, 4, 3, f) == 3;
  if (!ok) { std::fclose(f); set_error("jac_mlp_load: not a network file"); return 5; }
  if (dims[0] != net->I || dims[1] != net->H || dims[2] != net->n) {
    std::fclose(f);
    set_error("jac_mlp_load: the file holds a network of another shape");
    return 6;
  }
  std::vector<float> buf((size_t)net->P);
  const int order[3] = {JAC_MLP_MOMENT1, JAC_MLP_MOMENT2, JAC_MLP_PARAMS};
  std::vector<float> w((size_t)net->P);
  ok = std::fread(w.data(), 4, w.size(), f) == w.size();
  for (int k = 0; ok && k < 2; ++k) {
    ok = std::fread(buf.data(), 4, buf.size(), f) == buf.size();
    if (ok) {
      int e = jac_mlp_set(net, order[k], buf.data());
      if (e) { std::fclose(f); return e; }
    }
  }
  std::fclose(f);
  if (!ok) { set_error("jac_mlp_load: file too short"); return 5; }
  int e = jac_mlp_set(net, JAC_MLP_PARAMS, w.data());
  if (e) return e;
  net->t = t; net->beta1 = hp[0]; net->beta2 = hp[1]; net->eps = hp[2];
  return 0;
}

}  // extern "C"
