// Internal declarations shared by the HIP sources of libjacobi.
// (Library-internal: nothing here is part of the C-ABI in include/jacobi.h.)
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

namespace jac {

// ---------------------------------------------------------------- errors
void set_error(const std::string& msg);
const char* last_error();

#define JAC_HIP(call)                                                          \
  do {                                                                         \
    hipError_t e_ = (call);                                                    \
    if (e_ != hipSuccess) {                                                    \
      ::jac::set_error(std::string(#call) + ": " + hipGetErrorString(e_));     \
      return 4;                                                                \
    }                                                                          \
  } while (0)

#define JAC_CHECK_LAUNCH() JAC_HIP(hipGetLastError())

// ---------------------------------------------------------------- workspace
// Grow-only device scratch owned by the library (one pool per device).
void* workspace(size_t bytes);
void release_workspace();

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

struct Carve {
  char* base;
  size_t off = 0;
  explicit Carve(void* b) : base(static_cast<char*>(b)) {}
  template <typename T>
  T* take(size_t count) {
    off = align_up(off, 256);
    T* p = reinterpret_cast<T*>(base + off);
    off += count * sizeof(T);
    return p;
  }
};

// ---------------------------------------------------------------- types
template <typename T> struct Prec;
template <> struct Prec<double> {
  static constexpr double unit = 1.1102230246251565e-16;  // 2^-53
  static constexpr double bigmu = 1e150;
};
template <> struct Prec<float> {
  static constexpr float unit = 5.9604644775390625e-08f;  // 2^-24
  static constexpr float bigmu = 1e18f;
};

// A 2x2 pair block: rows (top_k, bottom_k) x cols (top_l, bottom_l).
template <typename T> struct alignas(4 * sizeof(T)) Blk { T tt, tb, bt, bb; };
// Rotation of one pair in slot roles: new_top = x_t - s (x_b + tau x_t),
// new_bottom = x_b + s (x_t - tau x_b); diagonal pair: tt -= t tb, bb += t tb.
template <typename T> struct alignas(4 * sizeof(T)) Ang { T s, tau, t, applied; };

// Round-robin (circle method) in Brent-Luk slots.  There are ne (even)
// indices; slot s < h = ne/2 is ring position s, slot h + j is ring position
// ne-1-j, so step r pairs slot k with slot h+k.  Ring position 0 holds index
// 0; position p >= 1 holds index 1 + ((p - 1 + r) mod (ne - 1)).  Between
// steps the occupants of positions 1..ne-1 shift one position down (position
// 1 wraps to ne-1), which in slots is: top slots move down by one, bottom
// slots up by one, slot 1 -> h and slot ne-1 -> h-1.
struct RR {
  int ne, h;
  __host__ __device__ RR(int ne_) : ne(ne_), h(ne_ / 2) {}
  __host__ __device__ int ringpos(int s) const { return s < h ? s : ne - 1 - (s - h); }
  __host__ __device__ int index(int s, int r) const {
    int p = ringpos(s);
    return p == 0 ? 0 : 1 + (p - 1 + r) % (ne - 1);
  }
  __host__ __device__ int newslot(int s) const {
    if (s == 0) return 0;
    if (s == 1) return h;
    if (s < h) return s - 1;
    if (s == ne - 1) return h - 1;
    return s + 1;
  }
  __host__ __device__ int srcslot(int s) const {
    if (s == 0) return 0;
    if (s == h) return 1;
    if (s < h - 1) return s + 1;
    if (s == h - 1) return ne - 1;
    return s - 1;
  }
};

// Packed upper triangle of pair blocks: block (k, l), k <= l.
__host__ __device__ inline long long bidx(int k, int l) { return (long long)l * (l + 1) / 2 + k; }

// ---------------------------------------------------------------- kernels
// Element-wise round-robin path (elem.hip).
template <typename T>
struct ElemState {
  int n, ne, h;
  long long nblk;
  Blk<T>* Tp[2];        // ping-pong packed T
  Ang<T>* A[2];         // ping-pong angles
  T* V;                 // n x n, leading dimension ldv, logical column order
  int ldv;
  T skip_abs;
  double* partial;      // off-norm partial sums (>= 1024)
  double* scalars;      // [0] off^2 result, [1] fro^2 result
  unsigned long long* rot;  // per-sweep applied-rotation counters
  int cur;              // which Tp / A holds the current step
};

// Pack / angles at the slot layout of step r (r = 0 at sweep boundaries).
template <typename T>
int elem_pack(ElemState<T>& st, const double* Adense, int lda, int r, hipStream_t s);
template <typename T>
int elem_pack_from(ElemState<T>& st, const T* Adense, int lda, int r, hipStream_t s);
template <typename T>
int elem_init_angles(ElemState<T>& st, int r, hipStream_t s);
template <typename T>
int elem_steps(ElemState<T>& st, long long gstep0, int nsteps, hipStream_t s);
template <typename T>
int elem_offnorm2(ElemState<T>& st, hipStream_t s);  // result -> st.scalars[0]
template <typename T>
int elem_unpack_dense(const ElemState<T>& st, int r, T* D, int ldd, hipStream_t s);
template <typename T>
int elem_diag(const ElemState<T>& st, T* d, hipStream_t s);  // logical-order diagonal

// Utilities (util.hip).
int fro2_f64(const double* A, int m, int n, int lda, double* partial, double* out, hipStream_t s);
template <typename T>
int set_identity(T* V, int n, int ldv, hipStream_t s);
template <typename Tin, typename Tout>
int copy_convert(const Tin* A, int m, int n, int lda, Tout* B, int ldb, hipStream_t s);
template <typename T>
int sort_eigs(const T* d, const T* Vw, int n, int ldw, double* W, double* Vout, int ldv,
              int* rank, hipStream_t s);
int check_finite(const double* A, int m, int n, int lda, int* flag, hipStream_t s);

// GEMM (gemm.hip): C = alpha * op(A) * op(B) + beta * C, column-major.
template <typename T>
int gemm(bool ta, bool tb, int m, int n, int k, T alpha, const T* A, int lda, const T* B, int ldb,
         T beta, T* C, int ldc, hipStream_t s);

// Block modified Gram-Schmidt in place (mgs.hip).  Returns 0 or 3 on breakdown.
int mgs_f64(double* Q, int m, int n, int ldq, double* scratch, int* flag, hipStream_t s);
size_t mgs_scratch_elems(int m, int n);

}  // namespace jac
