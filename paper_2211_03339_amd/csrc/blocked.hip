// Blocked round-robin Jacobi: 2b x 2b block rotations applied on the matrix
// cores.
//
// T (np x np, np = n rounded up to a multiple of 2b, zero padding) is split
// into 2m blocks of b consecutive indices.  One block step pairs the blocks of
// ring positions i and 2m-1-i (the same circle method as the element path, on
// blocks), giving m disjoint index sets P_k = I_k u J_k of size 2b.  Per step:
//
//  1. inner kernel, one workgroup per pair: S = T(P_k, P_k) is loaded into
//     LDS and swept by cyclic Jacobi (the rotations of Lemma offa-jr with the
//     skip rule of Remark dc; all pairs of the 2b indices at the first block
//     step of a sweep, only the pairs between I_k and J_k afterwards), while
//     the rotations are accumulated into W_k (2b x 2b, W_k = I at start).
//     S is written back to T(P_k, P_k); W_k and a flag "W_k is exactly I" go
//     to global memory.
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

__device__ __forceinline__ void stri_decode(int e, int& k, int& l) {
  // e -> (k, l), k < l, e = l (l - 1) / 2 + k
  int ll = (int)((1.0f + sqrtf(1.0f + 8.0f * (float)e)) * 0.5f);
  while (ll * (ll - 1) / 2 > e) --ll;
  while ((ll + 1) * ll / 2 <= e) ++ll;
  l = ll;
  k = e - ll * (ll - 1) / 2;
}

constexpr int kH = kB2 / 2;

// Two values read or written together in LDS.
template <typename T> struct alignas(2 * sizeof(T)) Rs { T x, y; };

// Inner solver: one workgroup diagonalises S = T(P_k, P_k) (2b x 2b) by
// cyclic Jacobi and accumulates the product of its rotations as
// E_k = W_k - I (the deviation from the identity is kept so that its rounding
// errors scale with the size of the rotations).  S (ping-pong) and E live in
// LDS in local index order (row-major, row stride 2b + 1).  Inner schedules:
//   block step 0 of a sweep (every block appears once): the full round-robin
//       on the 2b local indices; step ri pairs the indices held by ring
//       positions i and 2b-1-i of the circle method (position 0 fixed, the
//       others shifted by ri), 2b-1 steps;
//   later block steps: only the b x b pairs between the two blocks (the pairs
//       inside a block were rotated at step 0 of the sweep); step ri pairs
//       local index i < b with b + ((i + ri) mod b), b steps.
// So every index pair of the matrix is rotated exactly once per block sweep
// (a cyclic order) and a sweep takes about n sequential inner steps rather
// than 2n.  Per step, with one barrier:
//   wave 0, lanes 0..b-1: the angles of the NEXT step.  Each next pair (x, y)
//       takes x and y from two pairs of the current step, so its three entries
//       after this step follow from the current S and angles: the diagonal
//       ones by the t-form, the off-diagonal one by rotating the 2x2 block
//       with the same operations as the lane that owns that block.
//   waves 1..15: the 2x2 blocks S({p_k,q_k}, {p_l,q_l}) -> R_k^T S R_l, k <= l
//       (read from the current S, written with their mirror images to the
//       other copy; the (k, k) blocks by the t-form S_pp - t S_pq,
//       S_qq + t S_pq, 0) and the entry pairs (E_ap, E_aq) of
//       E <- E R + (R - I), in place.
// The blocks and their mirrors partition S and the (row, pair) items
// partition E, so no two lanes write the same entry within a step.
constexpr int kInnerThreads = 1024;
constexpr int kWorkLanes = kInnerThreads - 64;
constexpr int kBlocks = kH * (kH + 1) / 2;       // 2x2 blocks (k, l), k <= l, of S
constexpr int kBlockLanes = (kBlocks + 63) / 64 * 64;   // whole waves, so that work is wave-uniform
constexpr int kEItems = kB2 * kH;                // (row, pair) items of E
// Work split: lanes below kBlockLanes take one block and 2 E items, the others
// up to 3 E items; every E item of a lane has the lane's pair (offsets are
// multiples of kH), so one angle serves them all.
constexpr int kEPairLo = 2 * kBlockLanes;        // E items of the block lanes
static_assert(kEPairLo + 3 * (kWorkLanes - kBlockLanes) >= kEItems, "E items covered");
static_assert(kBlockLanes % kH == 0 && (kWorkLanes - kBlockLanes) % kH == 0, "pair-aligned offsets");

// Local index on ring position pos at step ri of the circle method on kB2
// indices: position 0 keeps index 0, position pos >= 1 holds
// 1 + ((pos - 1 + ri) mod (kB2 - 1)).
__device__ __forceinline__ int ring_index(int pos, int ri) {
  if (pos == 0) return 0;
  int x = pos - 1 + ri;
  if (x >= kB2 - 1) x -= kB2 - 1;
  return 1 + x;
}
__device__ __forceinline__ void ring_pair(int i, int ri, int& p, int& q) {
  const int a = ring_index(i, ri), b = ring_index(kB2 - 1 - i, ri);
  p = a < b ? a : b;
  q = a < b ? b : a;
}
// Pair (0 .. kH-1) that holds local index x at step ri.
__device__ __forceinline__ int ring_pair_of(int x, int ri) {
  if (x == 0) return 0;
  int pos = x - 1 - ri;
  if (pos < 0) pos += kB2 - 1;
  pos += 1;
  return pos < kH ? pos : kB2 - 1 - pos;
}

// R_k^T B R_l of the 2x2 block B = [tt tb; bt bb] = S({p_k,q_k}, {p_l,q_l}),
// k != l.  Rows are rotated by the pair with the smaller index first (the
// block owner works on k < l and writes the mirror image); for k > l the
// transpose is rotated, which reproduces the owner's values exactly.
template <typename T>
__device__ __forceinline__ void rotate_block(T& tt, T& tb, T& bt, T& bb, const Ang<T>& ak, const Ang<T>& al,
                                             bool tr) {
  const T s1 = tr ? al.s : ak.s, u1 = tr ? al.tau : ak.tau;
  const T s2 = tr ? ak.s : al.s, u2 = tr ? ak.tau : al.tau;
  T x01 = tr ? bt : tb, x10 = tr ? tb : bt;
  rot2(tt, x10, s1, u1);
  rot2(x01, bb, s1, u1);
  rot2(tt, x01, s2, u2);
  rot2(x10, bb, s2, u2);
  tb = tr ? x10 : x01;
  bt = tr ? x01 : x10;
}

// Source of S: the diagonal tile T(P_k, P_k) (symmetric eigenproblem; the
// diagonalised S is written back), or, when Gpart is given, the sum of the
// gsplit partial Gram matrices of the one-sided SVD (rel > 0 selects its
// negligibility rule; nothing is written back to T).
// LDS of one inner solve: S (ping-pong), E, angles (ping-pong).
// Block pair (0 .. m-1) holding block B at block step r of the circle method
// on m2 blocks (the slot rule of RR read backwards).
__device__ __forceinline__ int block_pair_of(const RR& rrb, int B, int r) {
  int p = 0;
  if (B != 0) {
    p = B - 1 - r;
    if (p < 0) p += rrb.ne - 1;
    p += 1;
  }
  return p < rrb.h ? p : rrb.ne - 1 - p;
}

// Y = W_k^T T(P_k, P_l) W_l (W = I + E) of one 64 x 64 tile by the 16 waves of
// a 1024-thread workgroup: wave w computes the 16 x 16 output block
// (w / 4, w % 4), so each wave runs 16 matrix-core steps per product and holds
// 16 E values per lane.  Global index of local index a: P_k(a) = a < b ? Ik + a
// : Jk + a (Jk already offset by -b), likewise P_l.  The products carry only
// the E terms; the base is added once.  Leaves Y in Bs (Bs[j * kLD + i] =
// Y(i, j), a 64 x (64+1) LDS tile) and ends with a barrier; every thread of
// the workgroup reaches the same barriers, inactive ones skip the work.
constexpr int kWT = 1024;   // threads of the 16-wave update paths

constexpr int kPer16 = kB2 * kB2 / kWT;   // tile values per thread (4)

// The thread's values of the tile T(P_k, P_l): tv[q] = T(P_k[e % 2b], P_l[e / 2b]), e = tid + q kWT.
template <typename T>
__device__ __forceinline__ void tile_vals16(const T* __restrict__ Tm, int ldt, int Ik, int Jk, int Il, int Jl,
                                            T (&tv)[kPer16]) {
  constexpr int b = kB2 / 2;
  auto gk = [&](int a) { return a < b ? Ik + a : Jk + a; };
  auto gl = [&](int a) { return a < b ? Il + a : Jl + a; };
#pragma unroll
  for (int q = 0; q < kPer16; ++q) {
    const int e = threadIdx.x + q * kWT, kk = e % kB2, c = e / kB2;
    tv[q] = Tm[gk(kk) + (size_t)gl(c) * ldt];
  }
}

struct NoHook { __device__ void operator()() const {} };

// The product of tile_product16 from the tile's values already in registers.  staged() runs
// once every thread's tile values are in LDS (the workgroup has read the tile).  With
// load_always the E operands are loaded even when the product is skipped, so that their loads
// need not wait for what decides active.
template <typename T, typename F = NoHook>
__device__ __forceinline__ void tile_product16_vals(const T (&tv)[kPer16], const T* __restrict__ Ek,
                                                    const T* __restrict__ El, T* __restrict__ Bs, bool active,
                                                    F staged = F(), bool load_always = false) {
  constexpr int kPer = kPer16;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int bi = wave >> 2, bj = wave & 3, cc = lane & 15, kq = lane >> 4;
  typename Mfma<T>::acc_t acc;
  T fa[kB2 / 4], fb[kB2 / 4];
  if (active || load_always) {
#pragma unroll
    for (int q = 0; q < kB2 / 4; ++q) fa[q] = Ek[(q * 4 + kq) * kB2 + bi * 16 + cc];   // A(i, kk) = E_k(kk, i)
#pragma unroll
    for (int q = 0; q < kB2 / 4; ++q) fb[q] = El[(q * 4 + kq) * kB2 + bj * 16 + cc];   // B(kk, j) = E_l(kk, j)
  }
  if (active) {
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int e = tid + q * kWT, kk = e % kB2, c = e / kB2;
      Bs[kk * kLD + c] = tv[q];   // B(kk, j = c) = T(P_k[kk], P_l[c])
    }
  }
  __syncthreads();
  staged();
  if (active) {
    acc = typename Mfma<T>::acc_t{0, 0, 0, 0};
#pragma unroll
    for (int q = 0; q < kB2 / 4; ++q) acc = Mfma<T>::op(fa[q], Bs[(q * 4 + kq) * kLD + bj * 16 + cc], acc);
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) acc[rr] += Bs[(bi * 16 + Mfma<T>::row(lane, rr)) * kLD + bj * 16 + cc];   // + T
  }
  __syncthreads();
  if (active) {
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) Bs[(bj * 16 + cc) * kLD + bi * 16 + Mfma<T>::row(lane, rr)] = acc[rr];   // X, k-major
  }
  __syncthreads();
  if (active) {
    acc = typename Mfma<T>::acc_t{0, 0, 0, 0};
#pragma unroll
    for (int q = 0; q < kB2 / 4; ++q) acc = Mfma<T>::op(Bs[(q * 4 + kq) * kLD + bi * 16 + cc], fb[q], acc);
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) acc[rr] += Bs[(bj * 16 + cc) * kLD + bi * 16 + Mfma<T>::row(lane, rr)];   // + X
  }
  __syncthreads();
  if (active) {
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) Bs[(bj * 16 + cc) * kLD + bi * 16 + Mfma<T>::row(lane, rr)] = acc[rr];   // Y
  }
  __syncthreads();
}

template <typename T, typename F = NoHook>
__device__ __forceinline__ void tile_product16(const T* __restrict__ Tm, int ldt, const T* __restrict__ Ek,
                                               const T* __restrict__ El, int Ik, int Jk, int Il, int Jl,
                                               T* __restrict__ Bs, bool active, F staged = F()) {
  T tv[kPer16];
  if (active) tile_vals16<T>(Tm, ldt, Ik, Jk, Il, Jl, tv);
  tile_product16_vals<T>(tv, Ek, El, Bs, active, staged);
}

template <typename T>
constexpr size_t inner_lds_bytes() { return 3 * kB2 * kLD * sizeof(T) + 2 * kH * sizeof(Ang<T>); }

template <typename T, bool BIP>
__device__ __forceinline__ void inner_solve(int k, T* __restrict__ Tm, int ldt, int n, int m2, int r,
                                            T* __restrict__ Eall, int* __restrict__ ident, T skip_abs,
                                            int max_inner, unsigned long long* __restrict__ rot,
                                            const T* __restrict__ Gpart, int gsplit, int npair, T rel,
                                            char* __restrict__ smem, const T* __restrict__ Ev = nullptr,
                                            const int* __restrict__ identv = nullptr,
                                            int* __restrict__ tcount = nullptr,
                                            unsigned long long* __restrict__ work = nullptr) {
  T (*S)[kB2 * kLD] = reinterpret_cast<T (*)[kB2 * kLD]>(smem);            // S[2][..]
  T* E = reinterpret_cast<T*>(smem) + 2 * kB2 * kLD;                         // E[a * kLD + c]
  // Angles (ping-pong), split so that the rotation lanes read only what they use:
  // rs[.][k] = (s, tau) of pair k, rt[.][k] = (t, applied).
  Rs<T> (*rs)[kH] = reinterpret_cast<Rs<T> (*)[kH]>(smem + 3 * kB2 * kLD * sizeof(T));
  Rs<T> (*rt)[kH] = rs + 2;
  auto put_angle = [&](int buf, int i, const Ang<T>& a) {
    rs[buf][i] = Rs<T>{a.s, a.tau};
    rt[buf][i] = Rs<T>{a.t, a.applied};
  };
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const RR rrb(m2);
  const int I = rrb.index(k, r), J = rrb.index(rrb.h + k, r);
  auto gidx = [&](int a) { return a < kH ? I * kH + a : J * kH + (a - kH); };
  constexpr bool bip = BIP;                // bipartite schedule (block steps after the first)
  constexpr int nsteps = bip ? kH : kB2 - 1;
  auto pair_at = [&](int i, int ri, int& p, int& q) {
    if (bip) { p = i; q = kH + ((i + ri) & (kH - 1)); }
    else ring_pair(i, ri, p, q);
  };
  auto pair_of = [&](int x, int ri) {
    return bip ? (x < kH ? x : ((x - kH - ri) & (kH - 1))) : ring_pair_of(x, ri);
  };
  auto first_angles = [&]() {
    if (tid < kH) {
      int p, q;
      pair_at(tid, 0, p, q);
      put_angle(0, tid, make_angle(S[0][p * kLD + p], S[0][q * kLD + q], S[0][p * kLD + q], gidx(p), gidx(q), n,
                                   skip_abs, rel));
    }
  };
  if (Ev) {
    // The update of block step r - 1 has not been applied to the tile that holds T(I, J):
    // compute that tile Y = W_ka^T T(P_ka, P_kb) W_kb here (ka < kb: the step r - 1 pairs of I
    // and J), take the quarter T(I, J) from it, and write back the quarters no inner solve of
    // this step reads.  A tile can hold the quarters of two pairs of this step; both compute it,
    // and the later of the two (per-tile counter, counted as soon as the workgroup has read the
    // tile) writes, after both have read the old tile.  The write-back runs while wave 0
    // computes the first angles.
    // T(I, I) and T(J, J) lie in diagonal blocks of step r - 1, final since its inner solves.
    constexpr int kPer = kB2 * kB2 / kInnerThreads;
    const int rv = r - 1;
    const int k1 = block_pair_of(rrb, I, rv), k2 = block_pair_of(rrb, J, rv);
    const bool swap = k1 > k2;   // I belongs to the second pair of the tile
    const int ka = swap ? k2 : k1, kb = swap ? k1 : k2;
    const int A0 = rrb.index(ka, rv), A1 = rrb.index(rrb.h + ka, rv);
    const int B0 = rrb.index(kb, rv), B1 = rrb.index(rrb.h + kb, rv);
    const int hI = I == (swap ? B0 : A0) ? 0 : 1, hJ = J == (swap ? A0 : B0) ? 0 : 1;
    // Every load is issued before the identity flags are known (all addresses are valid; when
    // both pairs are the identity the tile is already current and only the product is skipped).
    T sv[kPer], tv[kPer16];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int e = tid + q * kInnerThreads, a = e % kB2, c = e / kB2;
      sv[q] = Tm[gidx(a) + (size_t)gidx(c) * ldt];
    }
    tile_vals16<T>(Tm, ldt, A0 * kH, A1 * kH - kH, B0 * kH, B1 * kH - kH, tv);
    const bool id = identv[ka] && identv[kb];
    T* Y = S[1];
    int* flag = reinterpret_cast<int*>(rs);
    // quarters (x, y), x of pair ka, y of pair kb, that pairs of this step read
    auto read_now = [&](int x, int y) { return block_pair_of(rrb, x, r) == block_pair_of(rrb, y, r); };
    const int readers = (int)read_now(A0, B0) + (int)read_now(A0, B1) + (int)read_now(A1, B0) + (int)read_now(A1, B1);
    const int ti = kb * (kb - 1) / 2 + ka;
    int before = 0;   // thread 0: the tile's count before this workgroup's
    auto mark_read = [&]() {
      if (tid == 0 && !id && readers > 1) before = atomicAdd(tcount + ti, 1);
    };
    tile_product16_vals<T>(tv, Ev + (size_t)ka * kB2 * kB2, Ev + (size_t)kb * kB2 * kB2, Y, !id, mark_read, true);
    if (tid == 0 && !id) {
      const bool last = readers <= 1 || before == readers - 1;
      if (last && readers > 1) atomicExch(tcount + ti, 0);
      flag[0] = last;
      if (last && work) atomicAdd(work, 1ull << 32);
    }
    __syncthreads();
    const bool write_rest = !id && flag[0];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int e = tid + q * kInnerThreads, a = e % kB2, c = e / kB2;
      T v = sv[q];
      if (!id && (a < kH) != (c < kH)) {
        const int x = a < kH ? a : c, y = a < kH ? c - kH : a - kH;   // S(x, kH + y) = T(I_x, J_y)
        v = swap ? Y[(hI * kH + x) * kLD + hJ * kH + y] : Y[(hJ * kH + y) * kLD + hI * kH + x];
      }
      S[0][a * kLD + c] = v;
      if constexpr (!BIP) E[a * kLD + c] = T(0);   // (bipartite steps keep E in registers)
    }
    __syncthreads();
    first_angles();
    if (write_rest) {
      auto gA = [&](int u) { return u < kH ? A0 * kH + u : A1 * kH + u - kH; };
      auto gB = [&](int v) { return v < kH ? B0 * kH + v : B1 * kH + v - kH; };
      auto keep = [&](int u, int v) { return !read_now(u < kH ? A0 : A1, v < kH ? B0 : B1); };
#pragma unroll
      for (int q = 0; q < kPer; ++q) {
        const int e = tid + q * kInnerThreads, u = e % kB2, v = e / kB2;
        if (keep(u, v)) Tm[gA(u) + (size_t)gB(v) * ldt] = Y[v * kLD + u];
      }
#pragma unroll
      for (int q = 0; q < kPer; ++q) {
        const int e = tid + q * kInnerThreads, v = e % kB2, u = e / kB2;
        if (keep(u, v)) Tm[gB(v) + (size_t)gA(u) * ldt] = Y[v * kLD + u];
      }
    }
  } else {
    for (int e = tid; e < kB2 * kB2; e += kInnerThreads) {
      const int a = e % kB2, c = e / kB2;
      T v;
      if (Gpart) {
        // partial Grams are indexed by local indices (a, c), column-major
        v = T(0);
        for (int z = 0; z < gsplit; ++z) v += Gpart[((size_t)z * npair + k) * kB2 * kB2 + a + c * kB2];
      } else {
        v = Tm[gidx(a) + (size_t)gidx(c) * ldt];
      }
      S[0][a * kLD + c] = v;
      if constexpr (!BIP) E[a * kLD + c] = T(0);
    }
    __syncthreads();
    first_angles();
  }
  __syncthreads();
  // Block (bk, bl), bk <= bl, of work lane tid - 64 < kBlocks (fixed for all steps).
  int bk = -1, bl = -1;
  if (tid >= 64 && tid - 64 < kBlocks) {
    // e = l (l + 1) / 2 + k: l from the root of l^2 + l - 2e, then one correction each way
    // (e < 528, so the single-precision root is off by at most one)
    const int e = tid - 64;
    int l = (int)((sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);
    if ((l + 1) * (l + 2) / 2 <= e) ++l;
    if (l * (l + 1) / 2 > e) --l;
    bl = l;
    bk = e - l * (l + 1) / 2;
  }
  // E items of work lane t = tid - 64 (fixed for all steps): rows er[0..ne-1], pair pe; every
  // 32-lane group shares its rows and holds pairs 0..31.
  int er[3] = {0, 0, 0}, ne = 0;
  const int pe = (tid - 64) & (kH - 1);
  if (tid >= 64) {
    const int t = tid - 64;
    if (t < kBlockLanes) {
      er[0] = t >> 5;
      er[1] = (kBlockLanes + t) >> 5;
      ne = 2;
    } else {
      const int t2 = kEPairLo + (t - kBlockLanes);
      const int stride = kWorkLanes - kBlockLanes;
      er[0] = t2 >> 5;
      er[1] = (t2 + stride) >> 5;
      er[2] = (t2 + 2 * stride) >> 5;
      ne = t2 + 2 * stride < kEItems ? 3 : 2;
    }
  }
  // Bipartite schedule: the lane keeps its E entries in registers, ex = E(er, pe) and
  // ey = E(er, kH + ((pe + ri) mod kH)).  Step ri + 1 pairs pe with the column the lane of pair
  // pe + 1 holds, so after each step ey moves one lane down inside the 32-lane group.
  T ex[3] = {T(0), T(0), T(0)}, ey[3] = {T(0), T(0), T(0)};
  const int ey_src = (lane & 32) | ((lane + 1) & 31);
  unsigned long long cnt = 0;
  int cur = 0;
  for (int sw = 0; sw < max_inner; ++sw) {
    bool big = false;
    if constexpr (bip) {
      // only the b x b pairs between the two blocks rotate: one per thread
      static_assert(kInnerThreads == kH * kH, "one cross pair per thread");
      const int a = tid & (kH - 1), c = kH + (tid >> 5);
      if (gidx(a) < n && gidx(c) < n)
        big = !negligible2(S[cur][a * kLD + a], S[cur][c * kLD + c], S[cur][a * kLD + c], skip_abs, rel);
    } else {
      for (int e = tid; e < kB2 * kB2; e += kInnerThreads) {
        const int a = e % kB2, c = e / kB2;
        if (a < c && gidx(a) < n && gidx(c) < n)
          big |= !negligible2(S[cur][a * kLD + a], S[cur][c * kLD + c], S[cur][a * kLD + c], skip_abs, rel);
      }
    }
    if (!__syncthreads_or(big)) break;
    for (int ri = 0; ri < nsteps; ++ri) {
      const T* Sc = S[cur];
      T* Sn = S[cur ^ 1];
      const Rs<T>* acs = rs[cur];
      const Rs<T>* act = rt[cur];
      auto angle_at = [&](int i) {
        const Rs<T> a = acs[i], b = act[i];
        return Ang<T>{a.x, a.y, b.x, b.y};
      };
      if (wave == 0) {
        const unsigned long long m = __ballot(lane < kH && act[lane & (kH - 1)].y != T(0));
        cnt += __popcll(m);
        if (lane < kH) {
          const int r1 = ri == nsteps - 1 ? 0 : ri + 1;
          int x, y;
          pair_at(lane, r1, x, y);
          const int kx = pair_of(x, ri), ky = pair_of(y, ri);
          int pkx, qkx, pky, qky;
          pair_at(kx, ri, pkx, qkx);
          pair_at(ky, ri, pky, qky);
          const Ang<T> ax = angle_at(kx), ay = angle_at(ky);
          const T dx = Sc[pkx * kLD + qkx], dy = Sc[pky * kLD + qky];
          const T sxx = x == pkx ? fmaT(-ax.t, dx, Sc[pkx * kLD + pkx]) : fmaT(ax.t, dx, Sc[qkx * kLD + qkx]);
          const T syy = y == pky ? fmaT(-ay.t, dy, Sc[pky * kLD + pky]) : fmaT(ay.t, dy, Sc[qky * kLD + qky]);
          T tt, tb, bt, bb;
          if constexpr (BIP) {   // canonical positions (see the work lanes)
            tt = Sc[(pkx < pky ? pkx : pky) * kLD + (pkx < pky ? pky : pkx)];
            tb = Sc[pkx * kLD + qky];
            bt = Sc[pky * kLD + qkx];
            bb = Sc[(qkx < qky ? qkx : qky) * kLD + (qkx < qky ? qky : qkx)];
          } else {
            tt = Sc[pkx * kLD + pky];
            tb = Sc[pkx * kLD + qky];
            bt = Sc[qkx * kLD + pky];
            bb = Sc[qkx * kLD + qky];
          }
          rotate_block(tt, tb, bt, bb, ax, ay, kx > ky);
          const T sxy = x == pkx ? (y == pky ? tt : tb) : (y == pky ? bt : bb);
          put_angle(cur ^ 1, lane, make_angle(sxx, syy, sxy, gidx(x), gidx(y), n, skip_abs, rel));
        }
      } else {
        // Loads of all the lane's items first (S and E accesses share one array
        // each, so the compiler would otherwise keep every load behind the
        // previous item's stores), then the arithmetic, then the stores.
        const bool has_blk = bk >= 0;
        int pk = 0, qk = 0, pl = 0, ql = 0;
        T tt = T(0), tb = T(0), bt = T(0), bb = T(0);
        Ang<T> ak{}, al{};
        if (has_blk) {
          pair_at(bk, ri, pk, qk);
          pair_at(bl, ri, pl, ql);
          const Rs<T> sk = acs[bk], sl = acs[bl];
          ak.s = sk.x;
          ak.tau = sk.y;
          al.s = sl.x;
          al.tau = sl.y;
          if (bk == bl) ak.t = act[bk].x;   // the diagonal blocks use the t-form
          if constexpr (BIP) {
            // Bipartite steps keep S only at canonical positions: the upper triangles of the
            // two diagonal quadrants and the off-diagonal quadrant (rows < kH), each written
            // once per step (pk <= pl always; qk, ql >= kH in either order).
            tt = Sc[pk * kLD + pl];
            tb = Sc[pk * kLD + ql];
            bt = Sc[pl * kLD + qk];
            bb = Sc[(qk < ql ? qk : ql) * kLD + (qk < ql ? ql : qk)];
          } else {
            tt = Sc[pk * kLD + pl];
            tb = Sc[pk * kLD + ql];
            bt = Sc[qk * kLD + pl];
            bb = Sc[qk * kLD + ql];
          }
        }
        const Rs<T> se = acs[pe];
        Ang<T> ae{};
        ae.s = se.x;
        ae.tau = se.y;
        int pp, qp;
        pair_at(pe, ri, pp, qp);
        const bool rot_e = ae.s != T(0);   // (s = 0 leaves E exactly as it is)
        if constexpr (!BIP) {
          if (rot_e) {
#pragma unroll
            for (int q = 0; q < 3; ++q) {
              if (q < ne) {
                ex[q] = E[er[q] * kLD + pp];
                ey[q] = E[er[q] * kLD + qp];
              }
            }
          }
        }
        if (has_blk) {
          if (bk == bl) {
            tt = fmaT(-ak.t, tb, tt);
            bb = fmaT(ak.t, tb, bb);
            Sn[pk * kLD + pk] = tt;
            Sn[pk * kLD + qk] = T(0);
            if constexpr (!BIP) Sn[qk * kLD + pk] = T(0);
            Sn[qk * kLD + qk] = bb;
          } else {
            rotate_block(tt, tb, bt, bb, ak, al, false);
            if constexpr (BIP) {
              Sn[pk * kLD + pl] = tt;
              Sn[pk * kLD + ql] = tb;
              Sn[pl * kLD + qk] = bt;
              Sn[(qk < ql ? qk : ql) * kLD + (qk < ql ? ql : qk)] = bb;
            } else {
              Sn[pk * kLD + pl] = tt;
              Sn[pk * kLD + ql] = tb;
              Sn[qk * kLD + pl] = bt;
              Sn[qk * kLD + ql] = bb;
              Sn[pl * kLD + pk] = tt;
              Sn[ql * kLD + pk] = tb;
              Sn[pl * kLD + qk] = bt;
              Sn[ql * kLD + qk] = bb;
            }
          }
        }
        // E <- E R + (R - I) on columns (p, q): with x = E(a, p), y = E(a, q)
        // and dt, db the entries of I in those columns,
        // x' = x - s (y + tau x + db + tau dt), y' = y + s (x - tau y + dt - tau db).
        if (rot_e) {
#pragma unroll
          for (int q = 0; q < 3; ++q) {
            if (q < ne) {
              const int a = er[q];
              const T x = ex[q], y = ey[q];
              const T dt = a == pp ? T(1) : T(0), db = a == qp ? T(1) : T(0);
              const T px = fmaT(ae.tau, x, y) + fmaT(ae.tau, dt, db);
              const T py = fmaT(-ae.tau, y, x) + fmaT(-ae.tau, db, dt);
              ex[q] = fmaT(-ae.s, px, x);
              ey[q] = fmaT(ae.s, py, y);
              if constexpr (!BIP) {
                E[a * kLD + pp] = ex[q];
                E[a * kLD + qp] = ey[q];
              }
            }
          }
        }
        if constexpr (BIP) {
#pragma unroll
          for (int q = 0; q < 3; ++q) ey[q] = __shfl(ey[q], ey_src, 64);
        }
      }
      __syncthreads();
      cur ^= 1;
    }
  }
  if (!Gpart) {
    for (int e = tid; e < kB2 * kB2; e += kInnerThreads) {
      const int a = e % kB2, c = e / kB2;
      int ci = a * kLD + c;
      if constexpr (BIP) {   // canonical position of S(a, c)
        if ((a < kH) == (c < kH)) ci = (a < c ? a : c) * kLD + (a < c ? c : a);
        else if (a >= kH) ci = c * kLD + a;
      }
      Tm[gidx(a) + (size_t)gidx(c) * ldt] = S[cur][ci];
    }
  }
  // E_k row-major: Eall[k][a * 2b + c] = E(a, c).  (Bipartite: after whole inner sweeps ey is
  // back at column kH + pe.)
  T* Ek = Eall + (size_t)k * kB2 * kB2;
  if constexpr (BIP) {
    if (tid >= 64) {
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        if (q < ne) {
          Ek[er[q] * kB2 + pe] = ex[q];
          Ek[er[q] * kB2 + kH + pe] = ey[q];
        }
      }
    }
  } else {
    for (int e = tid; e < kB2 * kB2; e += kInnerThreads) {
      const int c = e % kB2, a = e / kB2;
      Ek[a * kB2 + c] = E[a * kLD + c];
    }
  }
  if (tid == 0) {
    ident[k] = cnt == 0;
    if (cnt) atomicAdd(rot, cnt);
  }
}

template <typename T, bool BIP>
__global__ void __launch_bounds__(kInnerThreads)
blk_inner_kernel(T* __restrict__ Tm, int ldt, int n, int m2, int r, T* __restrict__ Eall, int* __restrict__ ident,
                 T skip_abs, int max_inner, unsigned long long* __restrict__ rot, const T* __restrict__ Gpart,
                 int gsplit, int npair, T rel, const BDesc<T>* __restrict__ desc) {
  if (desc) {   // batched: matrix blockIdx.y of a size class
    const BDesc<T> d = desc[blockIdx.y];
    if (*d.conv >= 0) return;   // converged in an earlier sweep
    Tm = d.Tm; ldt = d.ldt; n = d.n; Eall = d.E; ident = d.ident; rot = d.rot;
    skip_abs = (T)(d.tol_n * sqrt(*d.nrm2));
  }
  __shared__ __attribute__((aligned(16))) char smem[inner_lds_bytes<T>()];
  inner_solve<T, BIP>(blockIdx.x, Tm, ldt, n, m2, r, Eall, ident, skip_abs, max_inner, rot, Gpart, gsplit, npair,
                      rel, smem);
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

// acc(i, j) += M[j * kLD + i] (jm = false) or M[i * kLD + j] (jm = true).
template <typename T>
__device__ __forceinline__ void acc_add(const T* M, int wm, int wn, bool jm, typename Mfma<T>::acc_t (&acc)[2][2]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        int i = wm * 32 + a * 16 + Mfma<T>::row(lane, rr);
        int j = wn * 32 + c * 16 + (lane & 15);
        acc[a][c][rr] += jm ? M[i * kLD + j] : M[j * kLD + i];
      }
}

template <typename T>
__device__ __forceinline__ void acc_zero(typename Mfma<T>::acc_t (&acc)[2][2]) {
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c) acc[a][c] = typename Mfma<T>::acc_t{0, 0, 0, 0};
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

// V(row0 .. row0+63, P_k) <- V + V E_k for one 64-row chunk by a 256-thread
// (four-wave) workgroup; Bs: a 64 x (64+1) LDS tile.  Ik and Jk are the global
// offsets of P_k's two blocks (local index a < b maps to Ik + a, a >= b to
// Jk + a).  The E operand is held in registers (64 values per lane in FP64).
template <typename T>
__device__ __forceinline__ void vchunk_update(T* __restrict__ V, int ldv, int nvr, const T* __restrict__ Ek, int Ik,
                                              int Jk, int row0, T* __restrict__ Bs) {
  constexpr int b = kB2 / 2;
  constexpr int kPer = kB2 * kB2 / kNT;
  const int tid = threadIdx.x, wave = tid >> 6, wm = wave >> 1, wn = wave & 1;
  auto gk = [&](int a) { return a < b ? Ik + a : Jk + a; };
  typename Mfma<T>::acc_t acc[2][2];
  T tv[kPer];
  T fb[2][kB2 / 4];
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int e = tid + q * kNT, i = e % kB2, kk = e / kB2;
    const int row = row0 + i;
    tv[q] = row < nvr ? V[row + (size_t)gk(kk) * ldv] : T(0);   // A(i, kk) = V(row, P_k[kk])
  }
  load_efrag<T>(Ek, wn * 32, fb);   // B(kk, j) = E_k(kk, j)
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int e = tid + q * kNT, i = e % kB2, kk = e / kB2;
    Bs[kk * kLD + i] = tv[q];
  }
  __syncthreads();
  acc_zero<T>(acc);
  mm_ldsA_fragB<T>(Bs, wm, fb, acc);    // V E_k
  acc_add<T>(Bs, wm, wn, false, acc);   // V + V E_k
  __syncthreads();
  acc_store<T>(Bs, wm, wn, acc);
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int e = tid + q * kNT, i = e % kB2, j = e / kB2;
    const int row = row0 + i;
    if (row < nvr) V[row + (size_t)gk(j) * ldv] = Bs[j * kLD + i];
  }
}

// T(P_k, P_l) <- W_k^T T(P_k, P_l) W_l (k < l, W = I + E) and its mirror
// T(P_l, P_k) by a 256-thread (four-wave) workgroup; Bs: a 64 x (64+1) LDS
// tile.  The matrix-core products carry only the E terms and the base tile is
// added once.  The E operands are held in registers.
template <typename T>
__device__ __forceinline__ void tile_update(T* __restrict__ Tm, int ldt, const T* __restrict__ Eall, const RR& rrb,
                                            int r, int k, int l, T* __restrict__ Bs) {
  constexpr int b = kB2 / 2;
  constexpr int kPer = kB2 * kB2 / kNT;
  const int tid = threadIdx.x, wave = tid >> 6, wm = wave >> 1, wn = wave & 1;
  typename Mfma<T>::acc_t acc[2][2];
  T tv[kPer];
  T fa[2][kB2 / 4], fb[2][kB2 / 4];
  const int Ik = rrb.index(k, r) * b, Jk = rrb.index(rrb.h + k, r) * b - b;
  const int Il = rrb.index(l, r) * b, Jl = rrb.index(rrb.h + l, r) * b - b;
  auto gk = [&](int a) { return a < b ? Ik + a : Jk + a; };   // global index of local index a of P_k
  auto gl = [&](int a) { return a < b ? Il + a : Jl + a; };
  const T* Ek = Eall + (size_t)k * kB2 * kB2;
  const T* El = Eall + (size_t)l * kB2 * kB2;
  // Issue the tile loads (HBM) first, then the E fragment loads (L2), then stage the tile.
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int e = tid + q * kNT, kk = e % kB2, c = e / kB2;
    tv[q] = Tm[gk(kk) + (size_t)gl(c) * ldt];
  }
  load_efrag<T>(Ek, wm * 32, fa);   // A(i, kk) = E_k(kk, i)
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int e = tid + q * kNT, kk = e % kB2, c = e / kB2;
    Bs[kk * kLD + c] = tv[q];   // B(kk, j = c) = T(P_k[kk], P_l[c])
  }
  __syncthreads();
  acc_zero<T>(acc);
  mm_fragA_ldsB<T>(fa, Bs, wn, acc);   // E_k^T T
  acc_add<T>(Bs, wm, wn, true, acc);   // X = T + E_k^T T (T tile is Bs[i * kLD + j])
  load_efrag<T>(El, wn * 32, fb);      // B(kk, j) = E_l(kk, j), once fa is dead
  __syncthreads();
  acc_store<T>(Bs, wm, wn, acc);       // Bs[j * kLD + i] = X(i, j): k-major A operand
  __syncthreads();
  acc_zero<T>(acc);
  mm_ldsA_fragB<T>(Bs, wm, fb, acc);   // X E_l
  acc_add<T>(Bs, wm, wn, false, acc);  // Y = X + X E_l
  __syncthreads();
  acc_store<T>(Bs, wm, wn, acc);       // Bs[j * kLD + i] = Y(i, j)
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int e = tid + q * kNT, i = e % kB2, j = e / kB2;
    Tm[gk(i) + (size_t)gl(j) * ldt] = Bs[j * kLD + i];
  }
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int e = tid + q * kNT, j = e % kB2, i = e / kB2;
    Tm[gl(j) + (size_t)gk(i) * ldt] = Bs[j * kLD + i];
  }
}

// Tiles of block step r that the inner solves of step r + 1 read: next pair
// k' = (B1, B2) reads T(B1, B2), which lies in the tile of the step-r pairs
// holding B1 and B2 (two next pairs can share a tile).  is_critical(a, b)
// tells those tiles.
__device__ __forceinline__ bool is_critical(const RR& rrb, int r, int a, int b) {
  const int r1 = r + 1;
  const int blocks[2] = {rrb.index(a, r), rrb.index(rrb.h + a, r)};
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int kn = block_pair_of(rrb, blocks[i], r1);
    const int P1 = rrb.index(kn, r1), P2 = rrb.index(rrb.h + kn, r1);
    const int partner = P1 == blocks[i] ? P2 : P1;
    if (block_pair_of(rrb, partner, r) == b) return true;
  }
  return false;
}

// Update kernel.  Tile (k, l), k < l:  X = T + E_k^T T,  Y = X + X E_l
// (= W_k^T T W_l), written to T(P_k, P_l) and mirrored into T(P_l, P_k).
// V chunk (k, 64 rows):  V(:, P_k) <- V + V E_k.  The matrix-core products
// accumulate only the E terms (from zero); the base T (X, V) is added once at
// the end, so each update rounds at the scale of the base once rather than
// at every k step.
template <typename T>
__global__ void __launch_bounds__(kNT)
blk_update_kernel(T* __restrict__ Tm, int ldt, T* __restrict__ V, int ldv, int nvr, const T* __restrict__ Eall,
                  const int* __restrict__ ident, int m2, int r, int ntile, int nvchunk,
                  unsigned long long* __restrict__ work, const BDesc<T>* __restrict__ desc = nullptr) {
  if (desc) {   // batched: matrix blockIdx.y of a size class
    const BDesc<T> d = desc[blockIdx.y];
    if (*d.conv >= 0) return;   // converged in an earlier sweep
    Tm = d.Tm; ldt = d.ldt; V = d.V; ldv = d.ldv; nvr = d.n; Eall = d.E; ident = d.ident;
  }
  constexpr int b = kB2 / 2;
  __shared__ T Bs[kB2 * kLD];
  const RR rrb(m2);
  const int w = blockIdx.x;
  if (w < ntile) {
    int k, l;
    stri_decode(w, k, l);
    if (ident[k] && ident[l]) return;
    if (work && threadIdx.x == 0) atomicAdd(work, 1ull << 32);
    tile_update<T>(Tm, ldt, Eall, rrb, r, k, l, Bs);
  } else {
    const int wv = w - ntile, k = wv / nvchunk, chunk = wv % nvchunk;
    if (ident[k]) return;
    if (work && threadIdx.x == 0) atomicAdd(work, 1ull);
    vchunk_update<T>(V, ldv, nvr, Eall + (size_t)k * kB2 * kB2, rrb.index(k, r) * b, rrb.index(rrb.h + k, r) * b - b,
                     chunk * kB2, Bs);
  }
}

// Y (in Bs after tile_product16) written to T(P_k, P_l) and mirrored into T(P_l, P_k).
template <typename T>
__device__ __forceinline__ void tile_store16(T* __restrict__ Tm, int ldt, int Ik, int Jk, int Il, int Jl,
                                             const T* __restrict__ Bs, bool active) {
  constexpr int b = kB2 / 2;
  const int tid = threadIdx.x;
  auto gk = [&](int a) { return a < b ? Ik + a : Jk + a; };
  auto gl = [&](int a) { return a < b ? Il + a : Jl + a; };
  if (active) {
#pragma unroll
    for (int q = 0; q < kPer16; ++q) {
      const int e = tid + q * kWT, i = e % kB2, j = e / kB2;
      Tm[gk(i) + (size_t)gl(j) * ldt] = Bs[j * kLD + i];
    }
#pragma unroll
    for (int q = 0; q < kPer16; ++q) {
      const int e = tid + q * kWT, j = e % kB2, i = e / kB2;
      Tm[gl(j) + (size_t)gk(i) * ldt] = Bs[j * kLD + i];
    }
  }
}

// Tile update by a 1024-thread workgroup: Y = W_k^T T(P_k, P_l) W_l written to
// T(P_k, P_l) and mirrored into T(P_l, P_k).
template <typename T>
__device__ __forceinline__ void tile_update16(T* __restrict__ Tm, int ldt, const T* __restrict__ Eall, const RR& rrb,
                                              int r, int k, int l, T* __restrict__ Bs, bool active) {
  constexpr int b = kB2 / 2;
  const int Ik = rrb.index(k, r) * b, Jk = rrb.index(rrb.h + k, r) * b - b;
  const int Il = rrb.index(l, r) * b, Jl = rrb.index(rrb.h + l, r) * b - b;
  tile_product16<T>(Tm, ldt, Eall + (size_t)k * kB2 * kB2, Eall + (size_t)l * kB2 * kB2, Ik, Jk, Il, Jl, Bs, active);
  tile_store16<T>(Tm, ldt, Ik, Jk, Il, Jl, Bs, active);
}

// The thread's values of the V chunk: tv[q] = V(row0 + e % 2b, P_k[e / 2b]), e = tid + q kWT.
template <typename T>
__device__ __forceinline__ void vchunk_vals16(const T* __restrict__ V, int ldv, int nvr, int Ik, int Jk, int row0,
                                              T (&tv)[kPer16]) {
  constexpr int b = kB2 / 2;
  auto gk = [&](int a) { return a < b ? Ik + a : Jk + a; };
#pragma unroll
  for (int q = 0; q < kPer16; ++q) {
    const int e = threadIdx.x + q * kWT, i = e % kB2, kk = e / kB2;
    const int row = row0 + i;
    tv[q] = row < nvr ? V[row + (size_t)gk(kk) * ldv] : T(0);   // A(i, kk) = V(row, P_k[kk])
  }
}

// The wave's fragment of E_k as the B operand: fb[q] = E_k(4 q + lane / 16, 16 (wave % 4) + lane % 16).
template <typename T>
__device__ __forceinline__ void efrag16(const T* __restrict__ Ek, T (&fb)[kB2 / 4]) {
  const int lane = threadIdx.x & 63, bj = (threadIdx.x >> 6) & 3;
#pragma unroll
  for (int q = 0; q < kB2 / 4; ++q) fb[q] = Ek[(q * 4 + (lane >> 4)) * kB2 + bj * 16 + (lane & 15)];
}

// V(row0 .. row0+63, P_k) <- V + V E_k by a 1024-thread workgroup (wave layout as in
// tile_product16) from the chunk's values and the E_k fragment already in registers.
template <typename T>
__device__ __forceinline__ void vchunk_update16_vals(const T (&tv)[kPer16], const T (&fb)[kB2 / 4],
                                                     T* __restrict__ V, int ldv, int nvr, int Ik, int Jk, int row0,
                                                     T* __restrict__ Bs, bool active) {
  constexpr int b = kB2 / 2;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int bi = wave >> 2, bj = wave & 3, cc = lane & 15, kq = lane >> 4;
  auto gk = [&](int a) { return a < b ? Ik + a : Jk + a; };
  typename Mfma<T>::acc_t acc;
  if (active) {
#pragma unroll
    for (int q = 0; q < kPer16; ++q) {
      const int e = tid + q * kWT, i = e % kB2, kk = e / kB2;
      Bs[kk * kLD + i] = tv[q];
    }
  }
  __syncthreads();
  if (active) {
    acc = typename Mfma<T>::acc_t{0, 0, 0, 0};
#pragma unroll
    for (int q = 0; q < kB2 / 4; ++q) acc = Mfma<T>::op(Bs[(q * 4 + kq) * kLD + bi * 16 + cc], fb[q], acc);
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) acc[rr] += Bs[(bj * 16 + cc) * kLD + bi * 16 + Mfma<T>::row(lane, rr)];   // + V
  }
  __syncthreads();
  if (active) {
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) Bs[(bj * 16 + cc) * kLD + bi * 16 + Mfma<T>::row(lane, rr)] = acc[rr];
  }
  __syncthreads();
  if (active) {
#pragma unroll
    for (int q = 0; q < kPer16; ++q) {
      const int e = tid + q * kWT, i = e % kB2, j = e / kB2;
      const int row = row0 + i;
      if (row < nvr) V[row + (size_t)gk(j) * ldv] = Bs[j * kLD + i];
    }
  }
}

template <typename T>
__device__ __forceinline__ void vchunk_update16(T* __restrict__ V, int ldv, int nvr, const T* __restrict__ Ek, int Ik,
                                                int Jk, int row0, T* __restrict__ Bs, bool active) {
  T tv[kPer16], fb[kB2 / 4];
  if (active) {
    vchunk_vals16<T>(V, ldv, nvr, Ik, Jk, row0, tv);
    efrag16<T>(Ek, fb);
  }
  vchunk_update16_vals<T>(tv, fb, V, ldv, nvr, Ik, Jk, row0, Bs, active);
}

// Update of one whole block step of the single-matrix path by 1024-thread
// workgroups: every tile, then the V chunks (workgroups ntile ..).
template <typename T>
__global__ void __launch_bounds__(kWT)
blk_update16_kernel(T* __restrict__ Tm, int ldt, T* __restrict__ V, int ldv, int nvr, const T* __restrict__ Eall,
                    const int* __restrict__ ident, int m2, int r, int ntile, int nvchunk,
                    unsigned long long* __restrict__ work) {
  constexpr int b = kB2 / 2;
  __shared__ T Bs[kB2 * kLD];
  const RR rrb(m2);
  const int w = blockIdx.x;
  if (w < ntile) {
    int k, l;
    stri_decode(w, k, l);
    if (ident[k] && ident[l]) return;
    if (work && threadIdx.x == 0) atomicAdd(work, 1ull << 32);
    tile_update16<T>(Tm, ldt, Eall, rrb, r, k, l, Bs, true);
  } else {
    const int wv = w - ntile, k = wv / nvchunk, chunk = wv % nvchunk;
    if (ident[k]) return;
    if (work && threadIdx.x == 0) atomicAdd(work, 1ull);
    vchunk_update16<T>(V, ldv, nvr, Eall + (size_t)k * kB2 * kB2, rrb.index(k, r) * b, rrb.index(rrb.h + k, r) * b - b,
                       chunk * kB2, Bs, true);
  }
}

// Helper-item forms with two LDS tiles (A and B), so that no barrier guards a
// tile against the previous phase's readers: a T tile is staged in A, X goes
// to B and Y back to A (3 barriers); consecutive tiles swap A and B, so the
// next tile's staging never meets the last one's readers.  A V chunk is staged
// in A and its result goes to B (2 barriers); the next chunk stages in A again,
// which only this chunk's first product read.
template <typename T>
__device__ __forceinline__ void tile_update16_ab(const T (&tv)[kPer16], const T* __restrict__ Ek,
                                                 const T* __restrict__ El, T* __restrict__ Tm, int ldt, int Ik,
                                                 int Jk, int Il, int Jl, T* __restrict__ A, T* __restrict__ B,
                                                 bool active) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int bi = wave >> 2, bj = wave & 3, cc = lane & 15, kq = lane >> 4;
  typename Mfma<T>::acc_t acc;
  T fa[kB2 / 4], fb[kB2 / 4];
  if (active) {
#pragma unroll
    for (int q = 0; q < kB2 / 4; ++q) fa[q] = Ek[(q * 4 + kq) * kB2 + bi * 16 + cc];   // A(i, kk) = E_k(kk, i)
#pragma unroll
    for (int q = 0; q < kB2 / 4; ++q) fb[q] = El[(q * 4 + kq) * kB2 + bj * 16 + cc];   // B(kk, j) = E_l(kk, j)
#pragma unroll
    for (int q = 0; q < kPer16; ++q) {
      const int e = tid + q * kWT, kk = e % kB2, c = e / kB2;
      A[kk * kLD + c] = tv[q];   // T tile
    }
  }
  __syncthreads();
  if (active) {
    acc = typename Mfma<T>::acc_t{0, 0, 0, 0};
#pragma unroll
    for (int q = 0; q < kB2 / 4; ++q) acc = Mfma<T>::op(fa[q], A[(q * 4 + kq) * kLD + bj * 16 + cc], acc);
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) acc[rr] += A[(bi * 16 + Mfma<T>::row(lane, rr)) * kLD + bj * 16 + cc];   // + T
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) B[(bj * 16 + cc) * kLD + bi * 16 + Mfma<T>::row(lane, rr)] = acc[rr];   // X, k-major
  }
  __syncthreads();
  if (active) {
    acc = typename Mfma<T>::acc_t{0, 0, 0, 0};
#pragma unroll
    for (int q = 0; q < kB2 / 4; ++q) acc = Mfma<T>::op(B[(q * 4 + kq) * kLD + bi * 16 + cc], fb[q], acc);
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) acc[rr] += B[(bj * 16 + cc) * kLD + bi * 16 + Mfma<T>::row(lane, rr)];   // + X
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) A[(bj * 16 + cc) * kLD + bi * 16 + Mfma<T>::row(lane, rr)] = acc[rr];   // Y
  }
  __syncthreads();
  tile_store16<T>(Tm, ldt, Ik, Jk, Il, Jl, A, active);
}

template <typename T>
__device__ __forceinline__ void vchunk_update16_ab(const T (&tv)[kPer16], const T (&fb)[kB2 / 4],
                                                   T* __restrict__ V, int ldv, int nvr, int Ik, int Jk, int row0,
                                                   T* __restrict__ A, T* __restrict__ B, bool active) {
  constexpr int b = kB2 / 2;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int bi = wave >> 2, bj = wave & 3, cc = lane & 15, kq = lane >> 4;
  auto gk = [&](int a) { return a < b ? Ik + a : Jk + a; };
  if (active) {
#pragma unroll
    for (int q = 0; q < kPer16; ++q) {
      const int e = tid + q * kWT, i = e % kB2, kk = e / kB2;
      A[kk * kLD + i] = tv[q];
    }
  }
  __syncthreads();
  if (active) {
    typename Mfma<T>::acc_t acc = {0, 0, 0, 0};
#pragma unroll
    for (int q = 0; q < kB2 / 4; ++q) acc = Mfma<T>::op(A[(q * 4 + kq) * kLD + bi * 16 + cc], fb[q], acc);
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) acc[rr] += A[(bj * 16 + cc) * kLD + bi * 16 + Mfma<T>::row(lane, rr)];   // + V
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) B[(bj * 16 + cc) * kLD + bi * 16 + Mfma<T>::row(lane, rr)] = acc[rr];
  }
  __syncthreads();
  if (active) {
#pragma unroll
    for (int q = 0; q < kPer16; ++q) {
      const int e = tid + q * kWT, i = e % kB2, j = e / kB2;
      const int row = row0 + i;
      if (row < nvr) V[row + (size_t)gk(j) * ldv] = B[j * kLD + i];
    }
  }
}

// Inner solves of block step r (workgroups 0 .. npair-1) together with the
// update of block step rv = r - 1 (the other workgroups, one tile or 64-row
// chunk at a time, by all 16 waves): the V chunks and, with merge_tiles, the
// T tiles the inner solves of step r do not read.  The tiles they do read are
// computed by the inner workgroups themselves (inner_solve with Ev), so the
// whole update of step rv runs inside this launch, the helpers on the CUs the
// inner solves leave idle.  Helper items touch no entry an inner solve
// touches.  E and the identity flags alternate between two buffers by step
// parity (Eall/ident for step r, Ev/identv for step rv).
template <typename T>
constexpr size_t inner_v_lds_bytes() {
  return inner_lds_bytes<T>() > 2 * kB2 * kLD * sizeof(T) ? inner_lds_bytes<T>() : 2 * kB2 * kLD * sizeof(T);
}

template <typename T, bool BIP>
__global__ void __launch_bounds__(kInnerThreads)
blk_inner_v_kernel(T* __restrict__ Tm, int ldt, int n, int m2, int r, T* __restrict__ Eall, int* __restrict__ ident,
                   T skip_abs, int max_inner, unsigned long long* __restrict__ rot, int npair, T* __restrict__ V,
                   int ldv, int nvr, const T* __restrict__ Ev, const int* __restrict__ identv, int nvchunk,
                   unsigned long long* __restrict__ work, int* __restrict__ tcount) {
  __shared__ __attribute__((aligned(16))) char smem[inner_v_lds_bytes<T>()];
  if ((int)blockIdx.x < npair) {
    inner_solve<T, BIP>(blockIdx.x, Tm, ldt, n, m2, r, Eall, ident, skip_abs, max_inner, rot, (const T*)nullptr, 0,
                        npair, T(0), smem, Ev, identv, tcount, work);
    return;
  }
  constexpr int b = kB2 / 2;
  const int vwg = (int)gridDim.x - npair;           // helper workgroups, one item at a time each
  const int wq = (int)blockIdx.x - npair;
  const int rv = r - 1;
  const RR rrb(m2);
  T* Bs = reinterpret_cast<T*>(smem);
  // The tiles of step rv that the inner solves of step r do not read (the inner workgroups
  // compute the others).  Every thread of a workgroup runs the same iterations (barriers).
  // The next item's values are loaded before the current item is computed (items are
  // disjoint, so the prefetch reads values no workgroup of this launch has written).
  const int ntile = npair * (npair - 1) / 2;
  const int per_t = (ntile + vwg - 1) / vwg;
  struct TileRef { int k, l, Ik, Jk, Il, Jl; bool act; };
  auto tile_at = [&](int it) {
    TileRef t{0, 1, 0, 0, 0, 0, false};
    const int ti = wq + it * vwg;
    if (it < per_t && ti < ntile) {
      stri_decode(ti, t.k, t.l);
      t.act = !is_critical(rrb, rv, t.k, t.l) && !(identv[t.k] && identv[t.l]);
      t.Ik = rrb.index(t.k, rv) * b;
      t.Jk = rrb.index(rrb.h + t.k, rv) * b - b;
      t.Il = rrb.index(t.l, rv) * b;
      t.Jl = rrb.index(rrb.h + t.l, rv) * b - b;
    }
    return t;
  };
  T* Bs2 = Bs + kB2 * kLD;
  T tv[kPer16], tn[kPer16];
  TileRef tc = tile_at(0);
  if (tc.act) tile_vals16<T>(Tm, ldt, tc.Ik, tc.Jk, tc.Il, tc.Jl, tv);
  for (int it = 0; it < per_t; ++it) {
    const TileRef tnx = tile_at(it + 1);
    if (tnx.act) tile_vals16<T>(Tm, ldt, tnx.Ik, tnx.Jk, tnx.Il, tnx.Jl, tn);
    if (tc.act && work && threadIdx.x == 0) atomicAdd(work, 1ull << 32);
    T* ta = (it & 1) ? Bs2 : Bs;
    T* tb = (it & 1) ? Bs : Bs2;
    tile_update16_ab<T>(tv, Ev + (size_t)tc.k * kB2 * kB2, Ev + (size_t)tc.l * kB2 * kB2, Tm, ldt, tc.Ik, tc.Jk,
                        tc.Il, tc.Jl, ta, tb, tc.act);
#pragma unroll
    for (int q = 0; q < kPer16; ++q) tv[q] = tn[q];
    tc = tnx;
  }
  __syncthreads();   // the last tile's stores still read its A tile
  // The V chunks of step rv, a contiguous range per workgroup: consecutive chunks of one pair
  // share E_k, whose fragment is loaded only when the pair changes.  A tile costs about two
  // chunks, so the ranges even out tiles + chunks: the trem workgroups that took one tile more
  // (tb + 1 instead of tb) take x - 2 chunks, the others x, with x the least count that covers
  // every chunk.
  const int total = npair * nvchunk;
  const int trem = ntile % vwg;
  int x = (total + 2 * trem + vwg - 1) / vwg;   // covers total when x >= 2: vwg x - 2 trem >= total
  if (x < 2) x = vwg - trem >= total ? (total > 0 ? 1 : 0) : 2;
  const int cA = x > 2 ? x - 2 : 0, cB = x;
  const bool more = wq < trem;
  const int per = more ? cA : cB;
  const int c0 = more ? wq * cA : trem * cA + (wq - trem) * cB;
  struct ChunkRef { int k, row0, Ik, Jk; bool act; };
  auto chunk_at = [&](int it) {
    ChunkRef c{0, 0, 0, 0, false};
    const int ci = c0 + it;
    if (it < per && ci < total) {
      c.k = ci / nvchunk;
      c.row0 = (ci % nvchunk) * kB2;
      c.act = identv[c.k] == 0;
      c.Ik = rrb.index(c.k, rv) * b;
      c.Jk = rrb.index(rrb.h + c.k, rv) * b - b;
    }
    return c;
  };
  T fb[kB2 / 4];
  int kfb = -1;
  ChunkRef cc = chunk_at(0);
  if (cc.act) vchunk_vals16<T>(V, ldv, nvr, cc.Ik, cc.Jk, cc.row0, tv);
  for (int it = 0; it < per; ++it) {
    const ChunkRef cnx = chunk_at(it + 1);
    if (cnx.act) vchunk_vals16<T>(V, ldv, nvr, cnx.Ik, cnx.Jk, cnx.row0, tn);
    if (cc.act && cc.k != kfb) {
      efrag16<T>(Ev + (size_t)cc.k * kB2 * kB2, fb);
      kfb = cc.k;
    }
    if (cc.act && work && threadIdx.x == 0) atomicAdd(work, 1ull);
    vchunk_update16_ab<T>(tv, fb, V, ldv, nvr, cc.Ik, cc.Jk, cc.row0, Bs, Bs2, cc.act);
#pragma unroll
    for (int q = 0; q < kPer16; ++q) tv[q] = tn[q];
    cc = cnx;
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
    if (r == 0)
      hipLaunchKernelGGL((blk_inner_kernel<T, false>), dim3(npair), dim3(kInnerThreads), 0, s, (T*)nullptr, 0, n, m2, r,
                         Ebuf, ident, T(0), max_inner, rot, (const T*)Gpart, gsplit, npair, rel,
                         (const BDesc<T>*)nullptr);
    else
      hipLaunchKernelGGL((blk_inner_kernel<T, true>), dim3(npair), dim3(kInnerThreads), 0, s, (T*)nullptr, 0, n, m2, r,
                         Ebuf, ident, T(0), max_inner, rot, (const T*)Gpart, gsplit, npair, rel,
                         (const BDesc<T>*)nullptr);
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
  // Merged launches: the helper workgroups (one 64 x 64 tile or V chunk at a time, all 16 waves)
  // are sized to the CUs the m inner solves leave free, each looping over its share of the items.
  static int cus = 0;
  if (!cus) {
    int dev = 0;
    hipDeviceProp_t prop;
    cus = (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
              ? prop.multiProcessorCount : 256;
  }
  // One helper per free CU: the kernel's registers (over 64 per lane for 16 waves) leave room
  // for one 1024-thread workgroup per CU, so a second helper per CU would only start once the
  // first has finished; the helpers loop over their share of the items instead.
  int vwg = m * nvchunk;
  const int free_wgs = cus - m > 16 ? cus - m : 16;
  if (vwg > free_wgs) vwg = free_wgs;
  // E and the identity flags alternate by step parity: step r's inner solve
  // writes buffer r & 1 while the V update of step r - 1 still reads the other.
  T* Eb[2] = {st.W, st.W + (size_t)m * kB2 * kB2};
  int* Ib[2] = {st.ident, st.ident + m};
  Prof* pf = st.prof;
  unsigned long long* work_u = pf && pf->on ? pf->work + st.cls_update : nullptr;
  unsigned long long* work_i = pf && pf->on ? pf->work + st.cls_inner : nullptr;
  // The whole update of block step r runs inside the launch of step r + 1: the tiles its inner
  // solves read by those inner workgroups, the other tiles and the V chunks by the helpers.  The
  // last step of a sweep is updated in full by a launch of its own.
  const int e0 = pf ? pf->mark(s) : -1;
  for (int r = 0; r < m2 - 1; ++r) {
    const int par = r & 1;
    if (r == 0)
      hipLaunchKernelGGL((blk_inner_kernel<T, false>), dim3(m), dim3(kInnerThreads), 0, s, st.Tm, st.ldt, st.n, m2, r,
                         Eb[par], Ib[par], st.skip_abs, max_inner, st.rot, (const T*)nullptr, 0, m, T(0),
                         (const BDesc<T>*)nullptr);
    else
      hipLaunchKernelGGL((blk_inner_v_kernel<T, true>), dim3(m + vwg), dim3(kInnerThreads), 0, s, st.Tm, st.ldt, st.n,
                         m2, r, Eb[par], Ib[par], st.skip_abs, max_inner, st.rot, m, st.V, st.ldv, st.nvr,
                         (const T*)Eb[par ^ 1], (const int*)Ib[par ^ 1], nvchunk, work_i, st.tcount);
    JAC_CHECK_LAUNCH();
  }
  const int e_mid = pf ? pf->mark(s) : -1;
  if (pf) pf->interval(st.cls_inner, e0, e_mid, m2 - 1);
  const int rl = m2 - 2;
  hipLaunchKernelGGL((blk_update16_kernel<T>), dim3(ntile + m * nvchunk), dim3(kWT), 0, s, st.Tm, st.ldt, st.V, st.ldv,
                     st.nvr, Eb[rl & 1], Ib[rl & 1], m2, rl, ntile, nvchunk, work_u);
  JAC_CHECK_LAUNCH();
  const int e_end = pf ? pf->mark(s) : -1;
  if (pf) pf->interval(st.cls_update, e_mid, e_end);
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
    if (r == 0)
      hipLaunchKernelGGL((blk_inner_kernel<T, false>), dim3(m, count), dim3(kInnerThreads), 0, s, (T*)nullptr, 0, 0, m2,
                         r, (T*)nullptr, (int*)nullptr, T(0), max_inner, (unsigned long long*)nullptr,
                         (const T*)nullptr, 0, m, T(0), desc);
    else
      hipLaunchKernelGGL((blk_inner_kernel<T, true>), dim3(m, count), dim3(kInnerThreads), 0, s, (T*)nullptr, 0, 0, m2,
                         r, (T*)nullptr, (int*)nullptr, T(0), max_inner, (unsigned long long*)nullptr,
                         (const T*)nullptr, 0, m, T(0), desc);
    JAC_CHECK_LAUNCH();
    hipLaunchKernelGGL((blk_update_kernel<T>), dim3(ntile + m * nvchunk, count), dim3(kNT), 0, s, (T*)nullptr, 0,
                       (T*)nullptr, 0, 0, (const T*)nullptr, (const int*)nullptr, m2, r, ntile, nvchunk,
                       (unsigned long long*)nullptr, desc);
    JAC_CHECK_LAUNCH();
  }
  return 0;
}

template int blk_sweep_batched<double>(const BDesc<double>*, int, int, int, int, hipStream_t);
template int blk_sweep_batched<float>(const BDesc<float>*, int, int, int, int, hipStream_t);

#define INST(T)                                                                    \
  template int blk_load<T>(BlkState<T>&, const void*, bool, int, hipStream_t);     \
  template int blk_offnorm2<T>(BlkState<T>&, hipStream_t);                         \
  template int blk_sweep<T>(BlkState<T>&, int, hipStream_t);                       \
  template int blk_diag<T>(const BlkState<T>&, T*, hipStream_t);
INST(double)
INST(float)
#undef INST

}  // namespace jac
