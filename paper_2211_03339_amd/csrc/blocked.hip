// Blocked round-robin Jacobi: 2b x 2b block rotations applied on the matrix
// cores.
//
// T (np x np, np = n rounded up to a multiple of 2b, zero padding) is split
// into 2m blocks of b consecutive indices.  One block step pairs the blocks of
// ring positions i and 2m-1-i (the same circle method as the element path, on
// blocks), giving m disjoint index sets P_k = I_k u J_k of size 2b.  Per step:
//
//  1. inner kernel, one workgroup per pair: S = T(P_k, P_k) is loaded into
//     LDS and diagonalised by cyclic Jacobi (round-robin over its 2b indices,
//     the rotations of Lemma offa-jr with the skip rule of Remark dc), while
//     the rotations are accumulated into W_k (2b x 2b, W_k = I at start).
//     The diagonalised S is written back to T(P_k, P_k); W_k and a flag
//     "W_k is exactly I" go to global memory.
//  2. update kernel: every tile T(P_k, P_l), k < l, becomes W_k^T T(P_k, P_l)
//     W_l (two 2b^3 GEMMs on v_mfma_*_16x16x4) and is mirrored into
//     T(P_l, P_k); every 64-row chunk of V(:, P_k) becomes V(:, P_k) W_k.
//     Pairs with W = I are skipped.  All updates are in place: each output
//     tile or chunk is read completely into LDS before it is written, and no
//     two workgroups touch the same entries.
//
// Since every block step is a product of Jacobi rotations on disjoint index
// sets, a block sweep (2m - 1 steps) is a cyclic Jacobi method whose order
// visits every pair of blocks once.
#include "common.h"

namespace jac {

constexpr int kB2 = 64;            // 2b
constexpr int kLD = kB2 + 1;       // LDS row stride (elements)
constexpr int kNT = 256;

__device__ __forceinline__ void tri_decode(int e, int& i, int& j) {
  // e -> (i, j), i <= j, e = j (j + 1) / 2 + i
  int jj = (int)((sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);
  while (jj * (jj + 1) / 2 > e) --jj;
  while ((jj + 1) * (jj + 2) / 2 <= e) ++jj;
  j = jj;
  i = e - jj * (jj + 1) / 2;
}

__device__ __forceinline__ void stri_decode(int e, int& k, int& l) {
  // e -> (k, l), k < l, e = l (l - 1) / 2 + k
  int ll = (int)((1.0f + sqrtf(1.0f + 8.0f * (float)e)) * 0.5f);
  while (ll * (ll - 1) / 2 > e) --ll;
  while ((ll + 1) * ll / 2 <= e) ++ll;
  l = ll;
  k = e - ll * (ll - 1) / 2;
}

// Slot movement of the round-robin on kB2 indices (same rule as RR, as
// compile-time functions so that register arrays are only indexed by
// constants).
constexpr int kH = kB2 / 2;
__host__ __device__ constexpr int ring_of(int s) { return s < kH ? s : kB2 - 1 - (s - kH); }
__host__ __device__ constexpr int src_of(int s) {
  return s == 0 ? 0 : s == kH ? 1 : s < kH - 1 ? s + 1 : s == kH - 1 ? kB2 - 1 : s - 1;
}
__host__ __device__ constexpr int new_of(int s) {
  return s == 0 ? 0 : s == 1 ? kH : s < kH ? s - 1 : s == kB2 - 1 ? kH - 1 : s + 1;
}
// The slots 1..kB2-1 form one cycle under src_of; cyc[i] = src_of^i(1).
struct Cycle {
  int v[kB2 - 1];
  constexpr Cycle() : v() {
    int t = 1;
    for (int i = 0; i < kB2 - 1; ++i) { v[i] = t; t = src_of(t); }
  }
};
constexpr Cycle kCyc{};

// new[t] = old[src_of(t)] for a register array, done in place along the cycle.
template <typename T>
__device__ __forceinline__ void permute_slots(T (&w)[kB2]) {
  T first = w[kCyc.v[0]];
#pragma unroll
  for (int i = 0; i < kB2 - 2; ++i) w[kCyc.v[i]] = w[kCyc.v[i + 1]];
  w[kCyc.v[kB2 - 2]] = first;
}

// Inner solver: one workgroup diagonalises S = T(P_k, P_k) (2b x 2b) by
// cyclic Jacobi and accumulates the product of its rotations as
// E_k = W_k - I (the deviation from the identity is kept so that its rounding
// errors scale with the size of the rotations).  S and E are kept in LDS in
// slot order (ping-pong): the pairs of every step are the slots (i, h+i) and
// entries move to the slots of the next step as they are written.
//   wave 0, lanes < h: "band" lanes recompute the three rotated entries that
//            form each pair of the NEXT step and derive its angle (Lemma
//            offa-jr), so that one barrier per step suffices;
//   waves 1-4: the pair blocks R_i^T B R_j of S (i <= j, mirrored) and the
//            column rotations of E (lane t: pair t mod h, 8 rows).
// Lane assignments and LDS offsets are fixed for all steps.
constexpr int kInnerThreads = 320;
constexpr int kWork = kInnerThreads - 64;
constexpr int kPairBlocks = kH * (kH + 1) / 2;
constexpr int kBlkPerLane = (kPairBlocks + kWork - 1) / kWork;
constexpr int kRowsPerLane = kB2 / (kWork / kH);

// Source of S: the diagonal tile T(P_k, P_k) (symmetric eigenproblem; the
// diagonalised S is written back), or, when Gpart is given, the sum of the
// gsplit partial Gram matrices of the one-sided SVD (rel > 0 selects its
// negligibility rule; nothing is written back to T).
template <typename T>
__global__ void __launch_bounds__(kInnerThreads)
blk_inner_kernel(T* __restrict__ Tm, int ldt, int n, int m2, int r, T* __restrict__ Eall, int* __restrict__ ident,
                 T skip_abs, int max_inner, unsigned long long* __restrict__ rot, const T* __restrict__ Gpart,
                 int gsplit, int npair, T rel, const BDesc<T>* __restrict__ desc) {
  if (desc) {   // batched: matrix blockIdx.y of a size class
    const BDesc<T> d = desc[blockIdx.y];
    Tm = d.Tm; ldt = d.ldt; n = d.n; Eall = d.E; ident = d.ident; rot = d.rot;
    skip_abs = (T)(d.tol_n * sqrt(*d.nrm2));
  }
  __shared__ T S[2][kB2 * kLD];
  __shared__ T E[2][kB2 * kLD];      // E[a * kLD + slot]: row a = local index
  __shared__ Ang<T> ang[2][kH];
  __shared__ int gsl[2][kB2];        // global index held by each slot
  __shared__ int lsl[2][kB2];        // local index held by each slot
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const RR rrb(m2);
  const int k = blockIdx.x;
  const int I = rrb.index(k, r), J = rrb.index(rrb.h + k, r);
  auto gidx = [&](int a) { return a < kH ? I * kH + a : J * kH + (a - kH); };
  if (tid < kB2) {
    gsl[0][tid] = gidx(ring_of(tid));
    lsl[0][tid] = ring_of(tid);
  }
  for (int e = tid; e < kB2 * kB2; e += kInnerThreads) {
    int s1 = e % kB2, s2 = e / kB2;
    T v;
    if (Gpart) {
      // partial Grams are indexed by local indices (a, c), column-major
      const int a = ring_of(s1), c = ring_of(s2);
      v = T(0);
      for (int z = 0; z < gsplit; ++z) v += Gpart[((size_t)z * npair + k) * kB2 * kB2 + a + c * kB2];
    } else {
      v = Tm[gidx(ring_of(s1)) + (size_t)gidx(ring_of(s2)) * ldt];
    }
    S[0][s1 * kLD + s2] = v;
    E[0][s1 * kLD + s2] = T(0);
  }
  unsigned long long cnt = 0;
  int pb_i[kBlkPerLane], pb_j[kBlkPerLane];
  const int w = tid - 64;          // work-lane index (waves 1-4)
  const int ek = w & (kH - 1), eg = w >> 5;
  if (wave >= 1) {
#pragma unroll
    for (int q = 0; q < kBlkPerLane; ++q) {
      int e = w + q * kWork;
      if (e < kPairBlocks) tri_decode(e, pb_i[q], pb_j[q]);
      else { pb_i[q] = -1; pb_j[q] = -1; }
    }
  }
  int ba = 0, bb_ = 0, bpa = 0, bra = 0, bpb = 0, brb = 0;
  if (wave == 0 && lane < kH) {
    ba = src_of(lane);
    bb_ = src_of(kH + lane);
    bpa = ba < kH ? ba : ba - kH; bra = ba < kH ? 0 : 1;
    bpb = bb_ < kH ? bb_ : bb_ - kH; brb = bb_ < kH ? 0 : 1;
  }
  __syncthreads();
  if (wave == 0 && lane < kH) {
    const T* Sc = S[0];
    ang[0][lane] = make_angle(Sc[lane * kLD + lane], Sc[(kH + lane) * kLD + kH + lane], Sc[lane * kLD + kH + lane],
                              gsl[0][lane], gsl[0][kH + lane], n, skip_abs, rel);
  }
  __syncthreads();
  int cur = 0;
  for (int sw = 0; sw < max_inner; ++sw) {
    bool big = false;
    for (int e = tid; e < kB2 * kB2; e += kInnerThreads) {
      int s1 = e % kB2, s2 = e / kB2;
      if (s1 < s2 && gsl[cur][s1] < n && gsl[cur][s2] < n)
        big |= !negligible2(S[cur][s1 * kLD + s1], S[cur][s2 * kLD + s2], S[cur][s1 * kLD + s2], skip_abs, rel);
    }
    if (!__syncthreads_or(big)) break;
    for (int ri = 0; ri < kB2 - 1; ++ri) {
      const T* Sc = S[cur];
      T* Sn = S[cur ^ 1];
      const Ang<T>* ac = ang[cur];
      if (wave == 0) {
        unsigned long long m = __ballot(lane < kH && ac[lane & (kH - 1)].applied != T(0));
        cnt += __popcll(m);
        if (lane < kH) {
          const Ang<T> apa = ac[bpa], apb = ac[bpb];
          T ta, tbv, tabv;
          {
            T x = Sc[bpa * kLD + kH + bpa];
            ta = bra ? fmaT(apa.t, x, Sc[(kH + bpa) * kLD + kH + bpa]) : fmaT(-apa.t, x, Sc[bpa * kLD + bpa]);
            T y = Sc[bpb * kLD + kH + bpb];
            tbv = brb ? fmaT(apb.t, y, Sc[(kH + bpb) * kLD + kH + bpb]) : fmaT(-apb.t, y, Sc[bpb * kLD + bpb]);
          }
          {
            const int k1 = bpa < bpb ? bpa : bpb, l1 = bpa < bpb ? bpb : bpa;
            const Ang<T> ak = bpa < bpb ? apa : apb, al = bpa < bpb ? apb : apa;
            T tt = Sc[k1 * kLD + l1], tb = Sc[k1 * kLD + kH + l1];
            T bt = Sc[(kH + k1) * kLD + l1], bb = Sc[(kH + k1) * kLD + kH + l1];
            rot2(tt, bt, ak.s, ak.tau);
            rot2(tb, bb, ak.s, ak.tau);
            rot2(tt, tb, al.s, al.tau);
            rot2(bt, bb, al.s, al.tau);
            const int comp = bpa < bpb ? bra * 2 + brb : brb * 2 + bra;
            tabv = comp == 0 ? tt : comp == 1 ? tb : comp == 2 ? bt : bb;
          }
          const int gi = gsl[cur][ba], gj = gsl[cur][bb_];
          ang[cur ^ 1][lane] = make_angle(ta, tbv, tabv, gi, gj, n, skip_abs, rel);
          gsl[cur ^ 1][lane] = gi;
          gsl[cur ^ 1][kH + lane] = gj;
          lsl[cur ^ 1][lane] = lsl[cur][ba];
          lsl[cur ^ 1][kH + lane] = lsl[cur][bb_];
        }
      } else {
#pragma unroll
        for (int q = 0; q < kBlkPerLane; ++q) {
          const int i = pb_i[q], j = pb_j[q];
          if (i < 0) continue;
          const Ang<T> ai = ac[i];
          const int ni = new_of(i), nhi = new_of(kH + i);
          if (i == j) {
            T tb = Sc[i * kLD + kH + i];
            Sn[ni * kLD + ni] = fmaT(-ai.t, tb, Sc[i * kLD + i]);
            Sn[nhi * kLD + nhi] = fmaT(ai.t, tb, Sc[(kH + i) * kLD + kH + i]);
            Sn[ni * kLD + nhi] = T(0);
            Sn[nhi * kLD + ni] = T(0);
          } else {
            const Ang<T> aj = ac[j];
            T tt = Sc[i * kLD + j], tb = Sc[i * kLD + kH + j];
            T bt = Sc[(kH + i) * kLD + j], bb = Sc[(kH + i) * kLD + kH + j];
            rot2(tt, bt, ai.s, ai.tau);
            rot2(tb, bb, ai.s, ai.tau);
            rot2(tt, tb, aj.s, aj.tau);
            rot2(bt, bb, aj.s, aj.tau);
            const int nj = new_of(j), nhj = new_of(kH + j);
            Sn[ni * kLD + nj] = tt; Sn[nj * kLD + ni] = tt;
            Sn[ni * kLD + nhj] = tb; Sn[nhj * kLD + ni] = tb;
            Sn[nhi * kLD + nj] = bt; Sn[nj * kLD + nhi] = bt;
            Sn[nhi * kLD + nhj] = bb; Sn[nhj * kLD + nhi] = bb;
          }
        }
        // E <- E R + (R - I) restricted to row a: with x = E(a, top), y =
        // E(a, bottom) and dt, db the entries of I in those columns,
        // x' = x - s (y + tau x + db + tau dt), y' = y + s (x - tau y + dt - tau db).
        {
          const Ang<T> a = ac[ek];
          const T* Ec = E[cur];
          T* En = E[cur ^ 1];
          const int lt = lsl[cur][ek], lb = lsl[cur][kH + ek];
          const int nt = new_of(ek), nb = new_of(kH + ek);
#pragma unroll
          for (int q = 0; q < kRowsPerLane; ++q) {
            const int row = eg + q * (kWork / kH);
            T x = Ec[row * kLD + ek], y = Ec[row * kLD + kH + ek];
            if (a.applied != T(0)) {
              const T dt = row == lt ? T(1) : T(0), db = row == lb ? T(1) : T(0);
              T px = fmaT(a.tau, x, y) + fmaT(a.tau, dt, db);
              T py = fmaT(-a.tau, y, x) + fmaT(-a.tau, db, dt);
              x = fmaT(-a.s, px, x);
              y = fmaT(a.s, py, y);
            }
            En[row * kLD + nt] = x;
            En[row * kLD + nb] = y;
          }
        }
      }
      __syncthreads();
      cur ^= 1;
    }
  }
  // After whole sweeps the slots hold their initial indices again.
  if (!Gpart) {
    for (int e = tid; e < kB2 * kB2; e += kInnerThreads) {
      int s1 = e % kB2, s2 = e / kB2;
      Tm[gidx(ring_of(s1)) + (size_t)gidx(ring_of(s2)) * ldt] = S[cur][s1 * kLD + s2];
    }
  }
  // E_k row-major: Eall[k][a * 2b + c] = E(a, c), c = local column index.
  T* Ek = Eall + (size_t)k * kB2 * kB2;
  for (int e = tid; e < kB2 * kB2; e += kInnerThreads) {
    int s1 = e % kB2, a = e / kB2;
    Ek[a * kB2 + ring_of(s1)] = E[cur][a * kLD + s1];
  }
  if (tid == 0) {
    ident[k] = cnt == 0;
    if (cnt) atomicAdd(rot, cnt);
  }
}

// Fragments of a 2b x 2b row-major E (global, L2-resident) for the MFMA
// operand of a wave's 32 x 32 quarter: as the A operand of E^T (A(i, kk) =
// E(kk, i)) or as the B operand of E (B(kk, j) = E(kk, j)) the lane reads
// E[(k0 + lane/16) * 2b + c0 + lane%16]: 16 consecutive elements per k.
template <typename T>
__device__ __forceinline__ void load_efrag(const T* __restrict__ Eg, int c0, T (&f)[2][kB2 / 4]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int q = 0; q < kB2 / 4; ++q) f[a][q] = Eg[(q * 4 + (lane >> 4)) * kB2 + c0 + a * 16 + (lane & 15)];
}

// acc += A * B for the wave's 32 x 32 quarter, A (i, kk) and B (kk, j) given
// either as register fragments (from load_efrag) or as k-major LDS arrays.
template <typename T>
__device__ __forceinline__ void mm_fragA_ldsB(const T (&fa)[2][kB2 / 4], const T* Bop, int wn,
                                              typename Mfma<T>::acc_t (&acc)[2][2]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int q = 0; q < kB2 / 4; ++q) {
    const int kr = q * 4 + (lane >> 4), cc = lane & 15;
    T bv[2];
#pragma unroll
    for (int c = 0; c < 2; ++c) bv[c] = Bop[kr * kLD + wn * 32 + c * 16 + cc];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int c = 0; c < 2; ++c) acc[a][c] = Mfma<T>::op(fa[a][q], bv[c], acc[a][c]);
  }
}

template <typename T>
__device__ __forceinline__ void mm_ldsA_fragB(const T* Aop, int wm, const T (&fb)[2][kB2 / 4],
                                              typename Mfma<T>::acc_t (&acc)[2][2]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int q = 0; q < kB2 / 4; ++q) {
    const int kr = q * 4 + (lane >> 4), cc = lane & 15;
    T av[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) av[a] = Aop[kr * kLD + wm * 32 + a * 16 + cc];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int c = 0; c < 2; ++c) acc[a][c] = Mfma<T>::op(av[a], fb[c][q], acc[a][c]);
  }
}

// acc <- M(i, j) for the wave's quarter, M held in LDS as M[j * kLD + i].
template <typename T>
__device__ __forceinline__ void acc_load(const T* M, int wm, int wn, typename Mfma<T>::acc_t (&acc)[2][2]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        int i = wm * 32 + a * 16 + Mfma<T>::row(lane, rr);
        int j = wn * 32 + c * 16 + (lane & 15);
        acc[a][c][rr] = M[j * kLD + i];
      }
}

// M[j * kLD + i] <- acc(i, j) for the wave's quarter.
template <typename T>
__device__ __forceinline__ void acc_store(T* M, int wm, int wn, const typename Mfma<T>::acc_t (&acc)[2][2]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        int i = wm * 32 + a * 16 + Mfma<T>::row(lane, rr);
        int j = wn * 32 + c * 16 + (lane & 15);
        M[j * kLD + i] = acc[a][c][rr];
      }
}

// Update kernel.  Tile (k, l), k < l:  X = T + E_k^T T,  Y = X + X E_l
// (= W_k^T T W_l), written to T(P_k, P_l) and mirrored into T(P_l, P_k).
// V chunk (k, 64 rows):  V(:, P_k) <- V + V E_k.  The accumulators start from
// T (or X, V) so that the matrix-core products only carry the E terms.
template <typename T>
__global__ void __launch_bounds__(kNT)
blk_update_kernel(T* __restrict__ Tm, int ldt, T* __restrict__ V, int ldv, int nvr, const T* __restrict__ Eall,
                  const int* __restrict__ ident, int m2, int r, int ntile, int nvchunk,
                  unsigned long long* __restrict__ work, const BDesc<T>* __restrict__ desc = nullptr) {
  if (desc) {   // batched: matrix blockIdx.y of a size class
    const BDesc<T> d = desc[blockIdx.y];
    Tm = d.Tm; ldt = d.ldt; V = d.V; ldv = d.ldv; nvr = d.n; Eall = d.E; ident = d.ident;
  }
  constexpr int b = kB2 / 2;
  __shared__ T Bs[kB2 * kLD];
  __shared__ int gk[kB2], gl[kB2];
  const int tid = threadIdx.x, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const RR rrb(m2);
  typename Mfma<T>::acc_t acc[2][2];
  T fa[2][kB2 / 4], fb[2][kB2 / 4];
  int w = blockIdx.x;
  if (w < ntile) {
    int k, l;
    stri_decode(w, k, l);
    if (ident[k] && ident[l]) return;
    if (work && tid == 0) atomicAdd(work, 1ull << 32);
    const T* Ek = Eall + (size_t)k * kB2 * kB2;
    const T* El = Eall + (size_t)l * kB2 * kB2;
    load_efrag<T>(Ek, wm * 32, fa);   // A(i, kk) = E_k(kk, i)
    load_efrag<T>(El, wn * 32, fb);   // B(kk, j) = E_l(kk, j)
    if (tid < kB2) {
      int Ik = rrb.index(k, r), Jk = rrb.index(rrb.h + k, r);
      int Il = rrb.index(l, r), Jl = rrb.index(rrb.h + l, r);
      gk[tid] = tid < b ? Ik * b + tid : Jk * b + (tid - b);
      gl[tid] = tid < b ? Il * b + tid : Jl * b + (tid - b);
    }
    __syncthreads();
    for (int e = tid; e < kB2 * kB2; e += kNT) {
      int kk = e % kB2, c = e / kB2;
      Bs[kk * kLD + c] = Tm[gk[kk] + (size_t)gl[c] * ldt];   // B(kk, j = c) = T(P_k[kk], P_l[c])
    }
    __syncthreads();
    // acc <- T(i, j): T tile is Bs[i * kLD + j], i.e. M[j' * kLD + i'] with (i', j') = (j, i)
    {
      const int lane = tid & 63;
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
          for (int rr = 0; rr < 4; ++rr) {
            int i = wm * 32 + a * 16 + Mfma<T>::row(lane, rr);
            int j = wn * 32 + c * 16 + (lane & 15);
            acc[a][c][rr] = Bs[i * kLD + j];
          }
    }
    mm_fragA_ldsB<T>(fa, Bs, wn, acc);      // X = T + E_k^T T
    __syncthreads();
    acc_store<T>(Bs, wm, wn, acc);          // Bs[j * kLD + i] = X(i, j): k-major A operand
    __syncthreads();
    mm_ldsA_fragB<T>(Bs, wm, fb, acc);      // Y = X + X E_l (acc still holds X)
    __syncthreads();
    acc_store<T>(Bs, wm, wn, acc);          // Bs[j * kLD + i] = Y(i, j)
    __syncthreads();
    for (int e = tid; e < kB2 * kB2; e += kNT) {
      int i = e % kB2, j = e / kB2;
      Tm[gk[i] + (size_t)gl[j] * ldt] = Bs[j * kLD + i];
    }
    for (int e = tid; e < kB2 * kB2; e += kNT) {
      int j = e % kB2, i = e / kB2;
      Tm[gl[j] + (size_t)gk[i] * ldt] = Bs[j * kLD + i];
    }
  } else {
    int wv = w - ntile;
    int k = wv / nvchunk, chunk = wv % nvchunk;
    if (ident[k]) return;
    if (work && tid == 0) atomicAdd(work, 1ull);
    const int row0 = chunk * kB2;
    const T* Ek = Eall + (size_t)k * kB2 * kB2;
    load_efrag<T>(Ek, wn * 32, fb);   // B(kk, j) = E_k(kk, j)
    if (tid < kB2) {
      int Ik = rrb.index(k, r), Jk = rrb.index(rrb.h + k, r);
      gk[tid] = tid < b ? Ik * b + tid : Jk * b + (tid - b);
    }
    __syncthreads();
    for (int e = tid; e < kB2 * kB2; e += kNT) {
      int i = e % kB2, kk = e / kB2;
      int row = row0 + i;
      Bs[kk * kLD + i] = row < nvr ? V[row + (size_t)gk[kk] * ldv] : T(0);   // A(i, kk) = V(row, P_k[kk])
    }
    __syncthreads();
    acc_load<T>(Bs, wm, wn, acc);           // acc <- V(i, j)
    mm_ldsA_fragB<T>(Bs, wm, fb, acc);      // V + V E_k
    __syncthreads();
    acc_store<T>(Bs, wm, wn, acc);
    __syncthreads();
    for (int e = tid; e < kB2 * kB2; e += kNT) {
      int i = e % kB2, j = e / kB2;
      int row = row0 + i;
      if (row < nvr) V[row + (size_t)gk[j] * ldv] = Bs[j * kLD + i];
    }
  }
}

// ---------------------------------------------------------------- one-sided
// Partial Gram of block pair k over the row range of split z:
// G_z(a, c) = sum_rows C(row, P_k[a]) C(row, P_k[c]) (2b x 2b, column-major,
// stored at Gpart[z][k]).  Rows are staged through LDS 16 at a time (k-major,
// so the same array serves as the A = C^T and B = C operands).
template <typename T>
__global__ void __launch_bounds__(kNT)
gram_partial_kernel(const T* __restrict__ C, int ldc, int mrows, int m2, int r, int krows, T* __restrict__ Gpart,
                    int npair) {
  constexpr int b = kB2 / 2;
  __shared__ T Cs[2][16 * kLD];
  __shared__ int gk[kB2];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int k = blockIdx.x, z = blockIdx.y;
  const RR rrb(m2);
  if (tid < kB2) {
    int Ik = rrb.index(k, r), Jk = rrb.index(rrb.h + k, r);
    gk[tid] = tid < b ? Ik * b + tid : Jk * b + (tid - b);
  }
  const int r0 = z * krows, r1 = min(mrows, r0 + krows);
  typename Mfma<T>::acc_t acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c) acc[a][c] = typename Mfma<T>::acc_t{0, 0, 0, 0};
  __syncthreads();
  T ld[4];
  auto load = [&](int rb) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      int e = tid + q * kNT;      // 16 x 64 piece: row kk = e % 16, column i = e / 16
      int kk = e & 15, i = e >> 4;
      int row = rb + kk;
      ld[q] = row < r1 ? C[row + (size_t)gk[i] * ldc] : T(0);
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      int e = tid + q * kNT;
      Cs[buf][(e & 15) * kLD + (e >> 4)] = ld[q];
    }
  };
  int buf = 0;
  if (r0 < r1) { load(r0); store(0); }
  __syncthreads();
  for (int rb = r0; rb < r1; rb += 16) {
    const bool more = rb + 16 < r1;
    if (more) load(rb + 16);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int kr = q * 4 + (lane >> 4), cc = lane & 15;
      T av[2], bv[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) av[a] = Cs[buf][kr * kLD + wm * 32 + a * 16 + cc];
#pragma unroll
      for (int c = 0; c < 2; ++c) bv[c] = Cs[buf][kr * kLD + wn * 32 + c * 16 + cc];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c) acc[a][c] = Mfma<T>::op(av[a], bv[c], acc[a][c]);
    }
    if (more) {
      store(buf ^ 1);
      __syncthreads();
      buf ^= 1;
    }
  }
  T* G = Gpart + ((size_t)z * npair + k) * kB2 * kB2;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        int i = wm * 32 + a * 16 + Mfma<T>::row(lane, rr);
        int j = wn * 32 + c * 16 + (lane & 15);
        G[i + j * kB2] = acc[a][c][rr];
      }
}

// One block sweep of the one-sided method (Algorithm 5.1 / step 4 of
// Algorithm 5.2): for every block step, the Gram of each block pair, its
// diagonalisation, and C(:, P_k) <- C(:, P_k)(I + E_k), V(:, P_k) likewise.
template <typename T>
int svd_sweep(T* C, int ldc, int mrows, T* V, int ldv, int n, int np, T* Ebuf, int* ident, T* Gpart, int gsplit,
              T rel, int max_inner, unsigned long long* rot, hipStream_t s) {
  const int m2 = np / (kB2 / 2), npair = m2 / 2;
  const int krows = ((mrows + gsplit - 1) / gsplit + 15) / 16 * 16;
  const int cch = (mrows + kB2 - 1) / kB2, vch = (n + kB2 - 1) / kB2;
  for (int r = 0; r < m2 - 1; ++r) {
    hipLaunchKernelGGL((gram_partial_kernel<T>), dim3(npair, gsplit), dim3(kNT), 0, s, C, ldc, mrows, m2, r, krows,
                       Gpart, npair);
    JAC_CHECK_LAUNCH();
    hipLaunchKernelGGL((blk_inner_kernel<T>), dim3(npair), dim3(kInnerThreads), 0, s, (T*)nullptr, 0, n, m2, r, Ebuf,
                       ident, T(0), max_inner, rot, (const T*)Gpart, gsplit, npair, rel, (const BDesc<T>*)nullptr);
    JAC_CHECK_LAUNCH();
    // column updates of C (mrows rows) and V (n rows): the chunk path of the update kernel
    hipLaunchKernelGGL((blk_update_kernel<T>), dim3(npair * cch), dim3(kNT), 0, s, (T*)nullptr, 0, C, ldc, mrows, Ebuf,
                       ident, m2, r, 0, cch, (unsigned long long*)nullptr);
    JAC_CHECK_LAUNCH();
    hipLaunchKernelGGL((blk_update_kernel<T>), dim3(npair * vch), dim3(kNT), 0, s, (T*)nullptr, 0, V, ldv, n, Ebuf,
                       ident, m2, r, 0, vch, (unsigned long long*)nullptr);
    JAC_CHECK_LAUNCH();
  }
  return 0;
}

template int svd_sweep<double>(double*, int, int, double*, int, int, int, double*, int*, double*, int, double, int,
                               unsigned long long*, hipStream_t);
template int svd_sweep<float>(float*, int, int, float*, int, int, int, float*, int*, float*, int, float, int,
                              unsigned long long*, hipStream_t);

// ||off(T)||^2 partial sums over the full np x np matrix.
template <typename T>
__global__ void offdiag2_partial_kernel(const T* __restrict__ Tm, int np, int ldt, double* __restrict__ partial) {
  __shared__ double red[4];
  double acc = 0;
  long long total = (long long)np * np;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    int j = (int)(e / np), i = (int)(e % np);
    if (i != j) {
      double v = Tm[i + (size_t)j * ldt];
      acc += v * v;
    }
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ void blk_sum_partials_kernel(const double* __restrict__ partial, int count, double* __restrict__ out) {
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

// Copy a dense n x n (lda) matrix into the padded np x np working array.
template <typename Tin, typename T>
__global__ void pad_copy_kernel(const Tin* __restrict__ A, int n, int lda, T* __restrict__ Tm, int np, int ldt) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  int j = blockIdx.y;
  if (i >= np) return;
  Tm[i + (size_t)j * ldt] = (i < n && j < n) ? (T)A[i + (size_t)j * lda] : T(0);
}

template <typename T>
__global__ void diag_kernel(const T* __restrict__ Tm, int n, int ldt, T* __restrict__ d) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = Tm[i + (size_t)i * ldt];
}

static inline int cdiv(long long a, long long b) { return (int)((a + b - 1) / b); }

int blk_np(int n) { return cdiv(n, kB2) * kB2; }
int blk_b2() { return kB2; }

template <typename T>
int blk_load(BlkState<T>& st, const void* A, bool a_is_double, int lda, hipStream_t s) {
  dim3 g(cdiv(st.np, 256), st.np);
  if (a_is_double)
    hipLaunchKernelGGL((pad_copy_kernel<double, T>), g, dim3(256), 0, s, (const double*)A, st.n, lda, st.Tm, st.np,
                       st.ldt);
  else
    hipLaunchKernelGGL((pad_copy_kernel<T, T>), g, dim3(256), 0, s, (const T*)A, st.n, lda, st.Tm, st.np, st.ldt);
  JAC_CHECK_LAUNCH();
  return 0;
}

template <typename T>
int blk_offnorm2(BlkState<T>& st, hipStream_t s) {
  int nwg = cdiv((long long)st.np * st.np, 256);
  if (nwg > 1024) nwg = 1024;
  hipLaunchKernelGGL((offdiag2_partial_kernel<T>), dim3(nwg), dim3(256), 0, s, st.Tm, st.np, st.ldt, st.partial);
  JAC_CHECK_LAUNCH();
  hipLaunchKernelGGL(blk_sum_partials_kernel, dim3(1), dim3(1024), 0, s, st.partial, nwg, st.scalars);
  JAC_CHECK_LAUNCH();
  return 0;
}

template <typename T>
int blk_sweep(BlkState<T>& st, int max_inner, hipStream_t s) {
  const int m2 = st.np / (kB2 / 2), m = m2 / 2;
  const int ntile = m * (m - 1) / 2;
  const int nvchunk = cdiv(st.nvr, kB2);
  Prof* pf = st.prof;
  unsigned long long* work = pf && pf->on ? pf->work + st.cls_update : nullptr;
  int e_prev = pf ? pf->mark(s) : -1;
  for (int r = 0; r < m2 - 1; ++r) {
    hipLaunchKernelGGL((blk_inner_kernel<T>), dim3(m), dim3(kInnerThreads), 0, s, st.Tm, st.ldt, st.n, m2, r, st.W,
                       st.ident, st.skip_abs, max_inner, st.rot, (const T*)nullptr, 0, m, T(0),
                       (const BDesc<T>*)nullptr);
    JAC_CHECK_LAUNCH();
    int e_mid = pf ? pf->mark(s) : -1;
    if (pf) pf->interval(st.cls_inner, e_prev, e_mid);
    int nwg = ntile + m * nvchunk;
    hipLaunchKernelGGL((blk_update_kernel<T>), dim3(nwg), dim3(kNT), 0, s, st.Tm, st.ldt, st.V, st.ldv, st.nvr, st.W,
                       st.ident, m2, r, ntile, nvchunk, work);
    JAC_CHECK_LAUNCH();
    int e_end = pf ? pf->mark(s) : -1;
    if (pf) pf->interval(st.cls_update, e_mid, e_end);
    e_prev = e_end;
  }
  return 0;
}

template <typename T>
int blk_diag(const BlkState<T>& st, T* d, hipStream_t s) {
  hipLaunchKernelGGL((diag_kernel<T>), dim3(cdiv(st.n, 256)), dim3(256), 0, s, st.Tm, st.n, st.ldt, d);
  JAC_CHECK_LAUNCH();
  return 0;
}

// ---------------------------------------------------------------- batched
// All matrices of one size class (same np) advance through the block steps
// together: grid.y runs over the class's matrices, each described by a BDesc.
template <typename T>
int blk_sweep_batched(const BDesc<T>* desc, int count, int np, int max_nvr, int max_inner, hipStream_t s) {
  const int m2 = np / (kB2 / 2), m = m2 / 2;
  const int ntile = m * (m - 1) / 2;
  const int nvchunk = cdiv(max_nvr, kB2);
  for (int r = 0; r < m2 - 1; ++r) {
    hipLaunchKernelGGL((blk_inner_kernel<T>), dim3(m, count), dim3(kInnerThreads), 0, s, (T*)nullptr, 0, 0, m2, r,
                       (T*)nullptr, (int*)nullptr, T(0), max_inner, (unsigned long long*)nullptr, (const T*)nullptr, 0,
                       m, T(0), desc);
    JAC_CHECK_LAUNCH();
    hipLaunchKernelGGL((blk_update_kernel<T>), dim3(ntile + m * nvchunk, count), dim3(kNT), 0, s, (T*)nullptr, 0,
                       (T*)nullptr, 0, 0, (const T*)nullptr, (const int*)nullptr, m2, r, ntile, nvchunk,
                       (unsigned long long*)nullptr, desc);
    JAC_CHECK_LAUNCH();
  }
  return 0;
}

// Per-matrix setup: T <- [A 0; 0 0] (np x np), V <- [I 0] (n x np), identity flags.
template <typename T>
__global__ void batched_init_kernel(const BDesc<T>* __restrict__ desc, const double* const* __restrict__ A,
                                    const int* __restrict__ lda) {
  const BDesc<T> d = desc[blockIdx.y];
  const double* a = A[blockIdx.y];
  const int la = lda[blockIdx.y];
  const int np = d.ldt;
  const long long total = (long long)np * np;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    int i = (int)(e % np), j = (int)(e / np);
    d.Tm[i + (size_t)j * np] = (i < d.n && j < d.n) ? (T)a[i + (size_t)j * la] : T(0);
    if (i < d.n) d.V[i + (size_t)j * d.ldv] = i == j ? T(1) : T(0);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) *d.rot = 0;
}

// Per matrix: ||off(T)||_F^2 and ||T||_F^2 (one workgroup per matrix, fixed order).
template <typename T>
__global__ void batched_norms_kernel(const BDesc<T>* __restrict__ desc, double* __restrict__ out) {
  __shared__ double red[2][4];
  const BDesc<T> d = desc[blockIdx.x];
  const int np = d.ldt;
  double off = 0, all = 0;
  for (long long e = threadIdx.x; e < (long long)np * np; e += blockDim.x) {
    int i = (int)(e % np), j = (int)(e / np);
    double v = d.Tm[i + (size_t)j * np];
    all += v * v;
    if (i != j) off += v * v;
  }
  for (int o = 32; o > 0; o >>= 1) { off += __shfl_down(off, o, 64); all += __shfl_down(all, o, 64); }
  if ((threadIdx.x & 63) == 0) { red[0][threadIdx.x >> 6] = off; red[1][threadIdx.x >> 6] = all; }
  __syncthreads();
  if (threadIdx.x == 0) {
    out[2 * blockIdx.x] = red[0][0] + red[0][1] + red[0][2] + red[0][3];
    out[2 * blockIdx.x + 1] = red[1][0] + red[1][1] + red[1][2] + red[1][3];
  }
}

// Per matrix: W ascending with V's columns permuted alike, info (0 if
// ||off(T)||_F <= tol ||A||_F after the last sweep, else 1) and the number of
// sweeps until that test first held (norms[s] = (off^2, ||T||^2) after s sweeps).
template <typename T>
__global__ void batched_finish_kernel(const BDesc<T>* __restrict__ desc, double* const* __restrict__ W,
                                      double* const* __restrict__ V, const int* __restrict__ ldv,
                                      const double* __restrict__ norms, int stride, int nsweeps, double tol,
                                      const int* __restrict__ orig, int* __restrict__ sweeps_out,
                                      int* __restrict__ info) {
  __shared__ int rank[512];
  const BDesc<T> d = desc[blockIdx.x];
  const int n = d.n;
  double* w = W[blockIdx.x];
  double* v = V[blockIdx.x];
  const int lv = ldv[blockIdx.x];
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    T di = d.Tm[i + (size_t)i * d.ldt];
    int rk = 0;
    for (int j = 0; j < n; ++j) {
      T dj = d.Tm[j + (size_t)j * d.ldt];
      rk += (dj < di) || (dj == di && j < i);
    }
    rank[i] = rk;
    w[rk] = (double)di;
  }
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    const int rk = rank[j];
    for (int row = threadIdx.x; row < n; row += blockDim.x)
      v[row + (size_t)rk * lv] = (double)d.V[row + (size_t)j * d.ldv];
  }
  if (threadIdx.x == 0) {
    const double nrm = sqrt(norms[2 * (size_t)blockIdx.x + 1]);
    int first = -1;
    for (int sw = 0; sw <= nsweeps; ++sw) {
      double off = sqrt(norms[(size_t)sw * stride + 2 * (size_t)blockIdx.x]);
      if (off <= tol * nrm) { first = sw; break; }
    }
    const int o = orig[blockIdx.x];
    if (info) info[o] = first < 0 ? 1 : 0;
    if (sweeps_out) sweeps_out[o] = first < 0 ? nsweeps : first;
  }
}

template <typename T>
int batched_init(const BDesc<T>* desc, int count, int maxnp, const double* const* A, const int* lda, hipStream_t s) {
  int gx = cdiv((long long)maxnp * maxnp, 256);
  if (gx > 64) gx = 64;
  hipLaunchKernelGGL((batched_init_kernel<T>), dim3(gx, count), dim3(256), 0, s, desc, A, lda);
  JAC_CHECK_LAUNCH();
  return 0;
}

template <typename T>
int batched_norms(const BDesc<T>* desc, int count, double* out, hipStream_t s) {
  hipLaunchKernelGGL((batched_norms_kernel<T>), dim3(count), dim3(256), 0, s, desc, out);
  JAC_CHECK_LAUNCH();
  return 0;
}

template <typename T>
int batched_finish(const BDesc<T>* desc, int count, double* const* W, double* const* V, const int* ldv,
                   const double* norms, int stride, int nsweeps, double tol, const int* orig, int* sweeps_out,
                   int* info, hipStream_t s) {
  hipLaunchKernelGGL((batched_finish_kernel<T>), dim3(count), dim3(256), 0, s, desc, W, V, ldv, norms, stride,
                     nsweeps, tol, orig, sweeps_out, info);
  JAC_CHECK_LAUNCH();
  return 0;
}

template int blk_sweep_batched<double>(const BDesc<double>*, int, int, int, int, hipStream_t);
template int batched_init<double>(const BDesc<double>*, int, int, const double* const*, const int*, hipStream_t);
template int batched_norms<double>(const BDesc<double>*, int, double*, hipStream_t);
template int batched_finish<double>(const BDesc<double>*, int, double* const*, double* const*, const int*,
                                    const double*, int, int, double, const int*, int*, int*, hipStream_t);

#define INST(T)                                                                    \
  template int blk_load<T>(BlkState<T>&, const void*, bool, int, hipStream_t);     \
  template int blk_offnorm2<T>(BlkState<T>&, hipStream_t);                         \
  template int blk_sweep<T>(BlkState<T>&, int, hipStream_t);                       \
  template int blk_diag<T>(const BlkState<T>&, T*, hipStream_t);
INST(double)
INST(float)
#undef INST

}  // namespace jac
