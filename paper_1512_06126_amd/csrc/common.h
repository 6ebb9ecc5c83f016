// Internal definitions shared by the HIP kernels and the host side of the
// library.  Not part of the public ABI (see include/giem.h).
#pragma once

#include <hip/hip_runtime.h>

#include <complex>
#include <cstdint>
#include <string>
#include <vector>

namespace giem {

// ---------------------------------------------------------------- complex
template <typename T>
struct alignas(2 * sizeof(T)) cplx {
  T x, y;
};

template <typename T>
__host__ __device__ __forceinline__ cplx<T> mk(T a, T b) {
  cplx<T> r;
  r.x = a;
  r.y = b;
  return r;
}
template <typename T>
__host__ __device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) {
  return mk<T>(a.x + b.x, a.y + b.y);
}
template <typename T>
__host__ __device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) {
  return mk<T>(a.x - b.x, a.y - b.y);
}
template <typename T>
__host__ __device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return mk<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
template <typename T>
__host__ __device__ __forceinline__ cplx<T> cmulc(cplx<T> a, cplx<T> b) {
  return mk<T>(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
template <typename T>
__host__ __device__ __forceinline__ cplx<T> cscale(cplx<T> a, T s) {
  return mk<T>(a.x * s, a.y * s);
}
// acc += a * b
template <typename T>
__host__ __device__ __forceinline__ void cfma(cplx<T> &acc, cplx<T> a, cplx<T> b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
}
template <typename T, typename U>
__host__ __device__ __forceinline__ cplx<T> ccast(cplx<U> a) {
  return mk<T>(static_cast<T>(a.x), static_cast<T>(a.y));
}

typedef cplx<double> c128;
typedef cplx<float> c64;

// ---------------------------------------------------------------- FFT plan
constexpr int kMaxFactors = 24;
struct FftDesc {
  int L;                  // transform length
  int nf;                 // number of radix stages
  int fac[kMaxFactors];   // radices in stage order (16, 8, 4, 2, 3, 5, 7, 11)
};

// Per-RHS vector pointers of one apply (the basis vectors of GMRES are not
// contiguous across right-hand sides); complex128 vectors, or complex64 ones
// for the inner solve of the precision form.  One apply takes up to kMaxRhs
// vectors per frequency and kMaxVec vectors over all its frequencies.
constexpr int kMaxRhs = 8;
constexpr int kMaxVec = 32;
template <typename VT>
struct VecPtrsT {
  const VT *in[kMaxVec];
  VT *out[kMaxVec];
};
using VecPtrs = VecPtrsT<c128>;
using VecPtrs32 = VecPtrsT<c64>;
// packed spectral tables of the frequencies of one batched apply
constexpr int kMaxFreqBatch = 16;
struct TabSet {
  const void *tab[kMaxFreqBatch];
};
// linear systems (frequencies x right-hand sides) of one batched solve
constexpr int kMaxSys = 96;

// Operator modes and precisions (mirror include/giem.h)
enum { MODE_A = 0, MODE_AT = 1, MODE_B = 2 };
enum { PREC_FP64 = 0, PREC_FP32 = 1 };

}  // namespace giem
