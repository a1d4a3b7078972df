// Element-wise round-robin parallel Jacobi (Algorithm 3.2 / step 4 of
// Algorithm 4.1 with the non-overlapping parallel ordering of Section 6.2).
//
// Data layout.  The working matrix T (symmetric, order ne = n rounded up to
// even) is stored as the packed upper triangle of 2x2 "pair blocks" in
// Brent-Luk slot order (see RR in common.h): block (k, l), k <= l, holds rows
// (slot k, slot h+k) x columns (slot l, slot h+l), so every pair of the
// current step is the diagonal block (k, k).  A step applies R_k^T B R_l to
// the old blocks (row pass with pair k, column pass with pair l, tau form of
// the rotation; diagonal blocks use the t form of Lemma offa-jr and get
// b_pq = 0) and writes every block of the next step (the other ping-pong
// buffer) whole: each of its four entries is the rotated value of one old
// entry, whose old block neighbouring threads read as well (from L2).  HBM
// sees one pass over the stored triangle each way, and the V update (columns
// p, q of V in logical order, rotated in place) is one pass over the rotated
// columns: 8 n(n+1) + 32 n bytes per applied rotation per step.
//
// One launch per step.  Its grid has three roles: (1) pair-block updates of T,
// (2) "band" threads that recompute the few rotated entries feeding each new
// diagonal block and produce the angles of the next step, (3) column-pair
// updates of V with this step's angles.  No role reads what another writes in
// the same launch, so the step is race-free without atomics on data.
#include "common.h"

namespace jac {

template <typename T>
__device__ __forceinline__ void rotate_block(Blk<T>& b, const Ang<T>& ak, const Ang<T>& al) {
  rot2(b.tt, b.bt, ak.s, ak.tau);
  rot2(b.tb, b.bb, ak.s, ak.tau);
  rot2(b.tt, b.tb, al.s, al.tau);
  rot2(b.bt, b.bb, al.s, al.tau);
}

template <typename T>
__device__ __forceinline__ void rotate_diag(Blk<T>& b, const Ang<T>& a) {
  T x = b.tb;
  b.tt = fmaT(-a.t, x, b.tt);
  b.bb = fmaT(a.t, x, b.bb);
  b.tb = T(0);
  b.bt = T(0);
}

__device__ __forceinline__ void kl_from_g(long long g, int& k, int& l) {
  double x = sqrt(8.0 * (double)g + 1.0);
  long long L = (long long)((x - 1.0) * 0.5);
  while (L * (L + 1) / 2 > g) --L;
  while ((L + 1) * (L + 2) / 2 <= g) ++L;
  l = (int)L;
  k = (int)(g - L * (L + 1) / 2);
}

// Rotated value (this step) of the element at old slots (a, b).
template <typename T>
__device__ __forceinline__ T rotated_old(const Blk<T>* __restrict__ Told, const Ang<T>* __restrict__ ang, int h,
                         int a, int b) {
  int ka = a < h ? a : a - h, ra = a < h ? 0 : 1;
  int kb = b < h ? b : b - h, rb = b < h ? 0 : 1;
  if (ka == kb) {
    Blk<T> blk = Told[bidx(ka, ka)];
    rotate_diag(blk, ang[ka]);
    if (ra != rb) return T(0);
    return ra ? blk.bb : blk.tt;
  }
  int k1 = ka < kb ? ka : kb, l1 = ka < kb ? kb : ka;
  Blk<T> blk = Told[bidx(k1, l1)];
  rotate_block(blk, ang[k1], ang[l1]);
  int comp = ka < kb ? ra * 2 + rb : rb * 2 + ra;
  return comp == 0 ? blk.tt : comp == 1 ? blk.tb : comp == 2 ? blk.bt : blk.bb;
}

constexpr int kThreads = 256;
constexpr int kXcds = 8;   // accelerator complex dies of the MI355X (one L2 each)
// Work per thread of the step kernel: pair blocks of T (bpt) and rows of the
// two V columns (rpt, moved in 16-byte vectors of 2 FP64 / 4 FP32 rows).
// Measured at n = 2048: FP64 1 / 8 and FP32 2 / 8 (each block gathers four
// old blocks, so one or two per thread already keep enough loads in flight).
template <typename T> struct ElemCfg;
template <> struct ElemCfg<double> { static constexpr int bpt = 1, rpt = 8; };
template <> struct ElemCfg<float> { static constexpr int bpt = 2, rpt = 8; };

template <typename T> struct Vec16;
template <> struct Vec16<double> { typedef double type __attribute__((ext_vector_type(2))); };
template <> struct Vec16<float> { typedef float type __attribute__((ext_vector_type(4))); };

template <typename T>
__global__ void __launch_bounds__(kThreads)
elem_step_kernel(const Blk<T>* __restrict__ Told, Blk<T>* __restrict__ Tnew,
                 const Ang<T>* __restrict__ ang, Ang<T>* __restrict__ ang_next,
                 T* __restrict__ V, int ldv, int n, int ne, int r, long long gnext_sweep,
                 long long nblk, int nwgT, int nwgB, int vchunks, int vec_ok, T skip_abs,
                 unsigned long long* __restrict__ rot) {
  constexpr int kBPT = ElemCfg<T>::bpt, kRPT = ElemCfg<T>::rpt;
  const RR rr(ne);
  const int h = rr.h;
  const int wg = blockIdx.x;
  if (wg < nwgT) {
    // Gather: the thread owns stored blocks of the next step; each of a block's four entries is
    // the rotated value of one old entry (slots srcslot(.)), read from its old block (which
    // neighbouring threads read too, from L2) - so every block is written once, whole.
    // Workgroups are dispatched round-robin over the 8 XCDs, each with its own L2: workgroup
    // wg takes range (wg mod 8) * per + wg / 8, so that every XCD walks one contiguous part of
    // the triangle and the neighbouring blocks it reads stay in its L2 (nwgT is a multiple of 8).
    const int per = nwgT / kXcds;
    const long long g0 = (long long)((wg % kXcds) * per + wg / kXcds) * kThreads * kBPT + threadIdx.x;
#pragma unroll
    for (int it = 0; it < kBPT; ++it) {
      const long long g = g0 + it * kThreads;
      if (g >= nblk) break;
      int k, l;
      kl_from_g(g, k, l);
      const int sk = rr.srcslot(k), shk = rr.srcslot(h + k), sl = rr.srcslot(l), shl = rr.srcslot(h + l);
      Blk<T> b;
      b.tt = rotated_old(Told, ang, h, sk, sl);
      b.tb = rotated_old(Told, ang, h, sk, shl);
      b.bt = k == l ? b.tb : rotated_old(Told, ang, h, shk, sl);
      b.bb = rotated_old(Told, ang, h, shk, shl);
      Tnew[g] = b;
    }
  } else if (wg < nwgT + nwgB) {
    int kp = (wg - nwgT) * kThreads + threadIdx.x;
    bool applied = false;
    if (kp < h) {
      int a = rr.srcslot(kp), b = rr.srcslot(h + kp);
      T tt = rotated_old(Told, ang, h, a, a);
      T bb = rotated_old(Told, ang, h, b, b);
      T tb = rotated_old(Told, ang, h, a, b);
      int rn = (r + 1) % (ne - 1);
      Ang<T> an = make_angle(tt, bb, tb, rr.index(kp, rn), rr.index(h + kp, rn), n, skip_abs);
      ang_next[kp] = an;
      applied = an.applied != T(0);
    }
    unsigned long long mask = __ballot(applied);
    if ((threadIdx.x & 63) == 0 && mask) atomicAdd(&rot[gnext_sweep], (unsigned long long)__popcll(mask));
  } else {
    int w = wg - nwgT - nwgB;
    int k = w / vchunks, chunk = w % vchunks;
    Ang<T> a = ang[k];
    if (a.applied == T(0)) return;
    int ip = rr.index(k, r), iq = rr.index(h + k, r);
    T* vp = V + (size_t)ip * ldv;
    T* vq = V + (size_t)iq * ldv;
    if (vec_ok) {
      // 16-byte vectors (the columns start 16-byte aligned); rows past the last whole vector
      // are done one by one by the first threads of chunk 0
      typedef typename Vec16<T>::type VT;
      constexpr int kW = 16 / sizeof(T);
      constexpr int kVPT = kRPT / kW;
      const int nvec = n / kW;
      VT* xp = reinterpret_cast<VT*>(vp);
      VT* xq = reinterpret_cast<VT*>(vq);
      int j = chunk * kThreads * kVPT + threadIdx.x;
      VT xs[kVPT], ys[kVPT];
#pragma unroll
      for (int it = 0; it < kVPT; ++it)
        if (j + it * kThreads < nvec) { xs[it] = xp[j + it * kThreads]; ys[it] = xq[j + it * kThreads]; }
#pragma unroll
      for (int it = 0; it < kVPT; ++it) {
        if (j + it * kThreads < nvec) {
#pragma unroll
          for (int c = 0; c < kW; ++c) {
            T x = xs[it][c], y = ys[it][c];
            rot2(x, y, a.s, a.tau);
            xs[it][c] = x;
            ys[it][c] = y;
          }
          xp[j + it * kThreads] = xs[it];
          xq[j + it * kThreads] = ys[it];
        }
      }
      const int i = nvec * kW + (int)threadIdx.x;
      if (chunk == 0 && i < n) {
        T x = vp[i], y = vq[i];
        rot2(x, y, a.s, a.tau);
        vp[i] = x;
        vq[i] = y;
      }
    } else {
      int i = chunk * kThreads * kRPT + threadIdx.x;
#pragma unroll
      for (int it = 0; it < kRPT; ++it, i += kThreads) {
        if (i < n) {
          T x = vp[i], y = vq[i];
          rot2(x, y, a.s, a.tau);
          vp[i] = x;
          vq[i] = y;
        }
      }
    }
  }
}

// Angles of step r read straight from the packed T (no rotation pending).
template <typename T>
__global__ void elem_angles0_kernel(const Blk<T>* __restrict__ Tp, Ang<T>* __restrict__ ang, int n,
                                    int ne, int r, T skip_abs, unsigned long long* __restrict__ rot) {
  const RR rr(ne);
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  bool applied = false;
  if (k < rr.h) {
    Blk<T> b = Tp[bidx(k, k)];
    Ang<T> a = make_angle(b.tt, b.bb, b.tb, rr.index(k, r), rr.index(rr.h + k, r), n, skip_abs);
    ang[k] = a;
    applied = a.applied != T(0);
  }
  unsigned long long mask = __ballot(applied);
  if ((threadIdx.x & 63) == 0 && mask) atomicAdd(&rot[0], (unsigned long long)__popcll(mask));
}

// Pack a dense column-major matrix into the slot layout of step r.
template <typename Tin, typename T>
__global__ void elem_pack_kernel(const Tin* __restrict__ A, int lda, Blk<T>* __restrict__ Tp, int n,
                                 int ne, int r, long long nblk) {
  const RR rr(ne);
  long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nblk) return;
  int k, l;
  kl_from_g(g, k, l);
  int it = rr.index(k, r), ib = rr.index(rr.h + k, r);
  int jt = rr.index(l, r), jb = rr.index(rr.h + l, r);
  auto at = [&](int i, int j) -> T {
    return (i < n && j < n) ? (T)A[i + (size_t)j * lda] : T(0);
  };
  Blk<T> b;
  b.tt = at(it, jt);
  b.tb = at(it, jb);
  b.bt = at(ib, jt);
  b.bb = at(ib, jb);
  if (k == l) b.bt = b.tb;
  Tp[g] = b;
}

// Off-norm: stored off-diagonal entries each stand for two entries of T.
template <typename T>
__global__ void elem_off_partial_kernel(const Blk<T>* __restrict__ Tp, long long nblk,
                                        double* __restrict__ partial) {
  __shared__ double red[kThreads / 64];
  double acc = 0;
  for (long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x; g < nblk;
       g += (long long)gridDim.x * blockDim.x) {
    int k, l;
    kl_from_g(g, k, l);
    Blk<T> b = Tp[g];
    double tb = b.tb;
    if (k == l) {
      acc += 2.0 * tb * tb;
    } else {
      double tt = b.tt, bt = b.bt, bb = b.bb;
      acc += 2.0 * (tt * tt + tb * tb + bt * bt + bb * bb);
    }
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0;
    for (int w = 0; w < kThreads / 64; ++w) s += red[w];
    partial[blockIdx.x] = s;
  }
}

__global__ void sum_partials_kernel(const double* __restrict__ partial, int count,
                                    double* __restrict__ out) {
  __shared__ double red[1024 / 64];
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

template <typename T>
__global__ void elem_unpack_kernel(const Blk<T>* __restrict__ Tp, int n, int ne, int r, long long nblk,
                                   T* __restrict__ D, int ldd) {
  const RR rr(ne);
  long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nblk) return;
  int k, l;
  kl_from_g(g, k, l);
  Blk<T> b = Tp[g];
  int it = rr.index(k, r), ib = rr.index(rr.h + k, r);
  int jt = rr.index(l, r), jb = rr.index(rr.h + l, r);
  auto st = [&](int i, int j, T v) {
    if (i < n && j < n) { D[i + (size_t)j * ldd] = v; D[j + (size_t)i * ldd] = v; }
  };
  st(it, jt, b.tt);
  st(it, jb, b.tb);
  st(ib, jt, k == l ? b.tb : b.bt);
  st(ib, jb, b.bb);
}

template <typename T>
__global__ void elem_diag_kernel(const Blk<T>* __restrict__ Tp, int n, int ne, T* __restrict__ d) {
  const RR rr(ne);
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= ne) return;
  int k = s < rr.h ? s : s - rr.h;
  Blk<T> b = Tp[bidx(k, k)];
  int i = rr.index(s, 0);
  if (i < n) d[i] = s < rr.h ? b.tt : b.bb;
}

// ------------------------------------------------------------------ host side
static inline int cdiv(long long a, long long b) { return (int)((a + b - 1) / b); }

template <typename T>
int elem_pack(ElemState<T>& st, const double* A, int lda, int r, hipStream_t s) {
  hipLaunchKernelGGL((elem_pack_kernel<double, T>), dim3(cdiv(st.nblk, 256)), dim3(256), 0, s, A, lda,
                     st.Tp[st.cur], st.n, st.ne, r, st.nblk);
  JAC_CHECK_LAUNCH();
  return 0;
}

template <typename T>
int elem_pack_from(ElemState<T>& st, const T* A, int lda, int r, hipStream_t s) {
  hipLaunchKernelGGL((elem_pack_kernel<T, T>), dim3(cdiv(st.nblk, 256)), dim3(256), 0, s, A, lda,
                     st.Tp[st.cur], st.n, st.ne, r, st.nblk);
  JAC_CHECK_LAUNCH();
  return 0;
}

template <typename T>
int elem_init_angles(ElemState<T>& st, int r, hipStream_t s) {
  hipLaunchKernelGGL((elem_angles0_kernel<T>), dim3(cdiv(st.h, 256)), dim3(256), 0, s, st.Tp[st.cur],
                     st.A[st.cur], st.n, st.ne, r, st.skip_abs, st.rot);
  JAC_CHECK_LAUNCH();
  return 0;
}

// Run nsteps steps starting at global step gstep0 (step r = gstep0 mod (ne-1)
// of sweep gstep0 / (ne-1)).  st.cur flips every step.
template <typename T>
int elem_steps(ElemState<T>& st, long long gstep0, int nsteps, hipStream_t s) {
  const int per = st.ne - 1;
  const int nwgT = cdiv(cdiv(st.nblk, (long long)kThreads * ElemCfg<T>::bpt), kXcds) * kXcds;
  const int nwgB = cdiv(st.h, kThreads);
  const int vchunks = cdiv(st.n, kThreads * ElemCfg<T>::rpt);
  const int nwg = nwgT + nwgB + st.h * vchunks;
  // V columns as 16-byte vectors when every column starts 16-byte aligned
  const int vec_ok = (reinterpret_cast<uintptr_t>(st.V) % 16 == 0) && (st.ldv * sizeof(T)) % 16 == 0;
  Prof* pf = st.prof;
  const int e0 = pf ? pf->mark(s) : -1;
  for (int i = 0; i < nsteps; ++i) {
    long long g = gstep0 + i;
    int r = (int)(g % per);
    long long next_sweep = (g + 1) / per;
    int c = st.cur;
    hipLaunchKernelGGL((elem_step_kernel<T>), dim3(nwg), dim3(kThreads), 0, s, st.Tp[c], st.Tp[c ^ 1],
                       st.A[c], st.A[c ^ 1], st.V, st.ldv, st.n, st.ne, r, next_sweep, st.nblk, nwgT,
                       nwgB, vchunks, vec_ok, st.skip_abs, st.rot);
    JAC_CHECK_LAUNCH();
    st.cur = c ^ 1;
  }
  if (pf && nsteps > 0) pf->interval(st.cls, e0, pf->mark(s), nsteps);
  return 0;
}

template <typename T>
int elem_offnorm2(ElemState<T>& st, hipStream_t s) {
  int nwg = cdiv(st.nblk, kThreads);
  if (nwg > 1024) nwg = 1024;
  if (nwg < 1) nwg = 1;
  hipLaunchKernelGGL((elem_off_partial_kernel<T>), dim3(nwg), dim3(kThreads), 0, s, st.Tp[st.cur],
                     st.nblk, st.partial);
  JAC_CHECK_LAUNCH();
  hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(1024), 0, s, st.partial, nwg, st.scalars);
  JAC_CHECK_LAUNCH();
  return 0;
}

template <typename T>
int elem_unpack_dense(const ElemState<T>& st, int r, T* D, int ldd, hipStream_t s) {
  hipLaunchKernelGGL((elem_unpack_kernel<T>), dim3(cdiv(st.nblk, 256)), dim3(256), 0, s, st.Tp[st.cur],
                     st.n, st.ne, r, st.nblk, D, ldd);
  JAC_CHECK_LAUNCH();
  return 0;
}

template <typename T>
int elem_diag(const ElemState<T>& st, T* d, hipStream_t s) {
  hipLaunchKernelGGL((elem_diag_kernel<T>), dim3(cdiv(st.ne, 256)), dim3(256), 0, s, st.Tp[st.cur], st.n,
                     st.ne, d);
  JAC_CHECK_LAUNCH();
  return 0;
}

#define INST(T)                                                                          \
  template int elem_pack<T>(ElemState<T>&, const double*, int, int, hipStream_t);         \
  template int elem_pack_from<T>(ElemState<T>&, const T*, int, int, hipStream_t);         \
  template int elem_init_angles<T>(ElemState<T>&, int, hipStream_t);                      \
  template int elem_steps<T>(ElemState<T>&, long long, int, hipStream_t);                 \
  template int elem_offnorm2<T>(ElemState<T>&, hipStream_t);                              \
  template int elem_unpack_dense<T>(const ElemState<T>&, int, T*, int, hipStream_t);      \
  template int elem_diag<T>(const ElemState<T>&, T*, hipStream_t);
INST(double)
INST(float)
#undef INST

}  // namespace jac
