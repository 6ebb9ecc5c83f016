// Krylov vector kernels of GMRES (Sect. 3.3, flexible GMRES; Sect. 2.1, the
// L2 inner product (V, U) = int V . conj(U)).  On the cell grid the inner
// product is sum_n wt_n V_n conj(U_n) with wt_n = V_n (cell volume) when the
// weighted form is requested, else 1.  Vectors are stored as complex128, or
// as complex64 for the inner solve of the precision form; all arithmetic and
// accumulation is FP64.  Reductions are wavefront shuffles, LDS across the
// workgroup, then a second pass over the per-workgroup partials.
#include "kernels.h"

namespace giem {

constexpr int kRedBlocks = 480;  // workgroups of the first reduction stage

int dot_partials_per_rhs() { return kRedBlocks; }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Sum a per-thread value over the 256-thread workgroup; result in thread 0.
__device__ __forceinline__ double block_sum(double v, double *red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += red[i];
  }
  return s;
}

template <typename VT>
__device__ __forceinline__ c128 wide(VT v) {
  return ccast<double>(v);
}
template <typename VT>
__device__ __forceinline__ VT store_as(c128 v) {
  return ccast<decltype(VT::x)>(v);
}

__device__ __forceinline__ double weight_of(size_t k, int plane, int nz, const double *wlev) {
  return wlev ? wlev[(int)((k / plane) % nz)] : 1.0;
}

// part[r][slot][block]: slot s < nb: sum wt w conj(V_s); slot nb: sum wt |w|^2
// SLOTS inner products per workgroup pass (blockIdx.z selects the group).
// Eight: w is re-read once per group of eight basis vectors, but wider groups
// need more registers, and the lower occupancy cost more than the re-reads
// (measured on the 128 x 128 x 32 solve).
constexpr int kSlots = 8;
// P2 (complex64 vectors, n even, 16-byte aligned vectors): each thread takes
// two neighbouring elements per 16-byte load, which doubles the bytes in
// flight per load instruction.
template <typename VT, int SLOTS, bool P2>
__global__ void __launch_bounds__(256)
k_dots(DotArgsT<VT> a, int nb, size_t n, int nz, int plane, const double *__restrict__ wlev,
       c128 *__restrict__ part, const int *__restrict__ gate, int gate_off) {
  constexpr int kSlots = SLOTS;
  __shared__ double red[8];
  const int r = blockIdx.y;
  const int s0 = blockIdx.z * kSlots;
  if (gate && !gate[gate_off + r]) {
    // pass not wanted for this system: zero partials, nothing read
    if (threadIdx.x == 0)
      for (int q = 0; q < kSlots; ++q)
        if (s0 + q <= nb)
          part[((size_t)r * (nb + 1) + s0 + q) * gridDim.x + blockIdx.x] = mk<double>(0.0, 0.0);
    return;
  }
  const VT *w = a.w[r];
  const VT *V = a.basis[r];
  double accr[kSlots], acci[kSlots];
#pragma unroll
  for (int k = 0; k < kSlots; ++k) accr[k] = acci[k] = 0.0;
  if constexpr (P2) {
    const size_t n2 = n >> 1;
    const float4 *w2 = reinterpret_cast<const float4 *>(w);
    const float4 *V2 = reinterpret_cast<const float4 *>(V);
    for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n2;
         k += (size_t)gridDim.x * blockDim.x) {
      const float4 wq = w2[k];
      const c128 wa = mk<double>(wq.x, wq.y), wb = mk<double>(wq.z, wq.w);
      const double ta = weight_of(2 * k, plane, nz, wlev), tb = weight_of(2 * k + 1, plane, nz, wlev);
#pragma unroll
      for (int q = 0; q < kSlots; ++q) {
        const int s = s0 + q;
        if (s < nb) {
          const float4 vq = V2[(size_t)s * n2 + k];
          const c128 va = mk<double>(vq.x, vq.y), vb = mk<double>(vq.z, vq.w);
          accr[q] += ta * (wa.x * va.x + wa.y * va.y);
          acci[q] += ta * (wa.y * va.x - wa.x * va.y);
          accr[q] += tb * (wb.x * vb.x + wb.y * vb.y);
          acci[q] += tb * (wb.y * vb.x - wb.x * vb.y);
        } else if (s == nb) {
          accr[q] += ta * (wa.x * wa.x + wa.y * wa.y);
          accr[q] += tb * (wb.x * wb.x + wb.y * wb.y);
        }
      }
    }
  } else {
    for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n;
         k += (size_t)gridDim.x * blockDim.x) {
      const c128 wv = wide(w[k]);
      const double wt = weight_of(k, plane, nz, wlev);
#pragma unroll
      for (int q = 0; q < kSlots; ++q) {
        const int s = s0 + q;
        if (s < nb) {
          const c128 v = wide(V[(size_t)s * n + k]);
          accr[q] += wt * (wv.x * v.x + wv.y * v.y);
          acci[q] += wt * (wv.y * v.x - wv.x * v.y);
        } else if (s == nb) {
          accr[q] += wt * (wv.x * wv.x + wv.y * wv.y);
        }
      }
    }
  }
  const int nslots = nb + 1;
#pragma unroll
  for (int q = 0; q < kSlots; ++q) {
    const int s = s0 + q;
    const double sr = block_sum(accr[q], red);
    const double si = block_sum(acci[q], red);
    if (threadIdx.x == 0 && s < nslots)
      part[((size_t)r * nslots + s) * gridDim.x + blockIdx.x] = mk<double>(sr, si);
  }
}

// out[r][slot] = sum over blocks of part[r][slot][block]
__global__ void __launch_bounds__(256)
k_reduce(const c128 *__restrict__ part, int nblk, int nslots, c128 *__restrict__ out) {
  __shared__ double red[8];
  const int r = blockIdx.y, s = blockIdx.x;
  const c128 *p = part + ((size_t)r * nslots + s) * nblk;
  double ar = 0.0, ai = 0.0;
  for (int b = threadIdx.x; b < nblk; b += blockDim.x) {
    ar += p[b].x;
    ai += p[b].y;
  }
  ar = block_sum(ar, red);
  ai = block_sum(ai, red);
  if (threadIdx.x == 0) out[(size_t)r * nslots + s] = mk<double>(ar, ai);
}

// whether complex64 vectors can be read in 16-byte pairs: n even and every
// vector (w and basis bases, basis vectors at stride n) 16-byte aligned
template <typename VT>
static bool pairs_ok(const DotArgsT<VT> &a, int nrhs, size_t n) {
  if (sizeof(VT) != 8 || (n & 1)) return false;
  for (int r = 0; r < nrhs; ++r)
    if ((reinterpret_cast<uintptr_t>(a.w[r]) | reinterpret_cast<uintptr_t>(a.basis[r])) & 15)
      return false;
  return true;
}

template <typename VT>
static hipError_t launch_dots_t(const DotArgsT<VT> &a, int nrhs, int nb, size_t n, int nz,
                                int plane, const double *wlev, c128 *part, c128 *out,
                                hipStream_t s, const int *gate, int gate_off) {
  const int nslots = nb + 1;
  const dim3 grid(kRedBlocks, nrhs, (nslots + kSlots - 1) / kSlots);
  if (pairs_ok(a, nrhs, n))
    k_dots<VT, kSlots, true><<<grid, 256, 0, s>>>(a, nb, n, nz, plane, wlev, part, gate, gate_off);
  else
    k_dots<VT, kSlots, false><<<grid, 256, 0, s>>>(a, nb, n, nz, plane, wlev, part, gate, gate_off);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_reduce<<<dim3(nslots, nrhs), 256, 0, s>>>(part, kRedBlocks, nslots, out);
  return hipGetLastError();
}
hipError_t launch_dots(const DotArgs &a, int nrhs, int nb, size_t n, int nz, int plane,
                       const double *wlev, c128 *part, c128 *out, hipStream_t s, const int *gate,
                       int gate_off) {
  return launch_dots_t(a, nrhs, nb, n, nz, plane, wlev, part, out, s, gate, gate_off);
}
hipError_t launch_dots(const DotArgs32 &a, int nrhs, int nb, size_t n, int nz, int plane,
                       const double *wlev, c128 *part, c128 *out, hipStream_t s, const int *gate,
                       int gate_off) {
  return launch_dots_t(a, nrhs, nb, n, nz, plane, wlev, part, out, s, gate, gate_off);
}

// w -= sum_{i < nb} h[r][i] V_i ; partial ||w||^2 into part[r][0][block]
template <typename VT, bool P2>
__global__ void __launch_bounds__(256)
k_update(DotArgsT<VT> a, int nb, size_t n, int nz, int plane, const double *__restrict__ wlev,
         const c128 *__restrict__ h, int hstride, const double *__restrict__ hscale,
         int sstride, c128 *__restrict__ part, const int *__restrict__ gate, int gate_off) {
  __shared__ double red[8];
  __shared__ c128 hs[64];
  const int r = blockIdx.y;
  if (gate && !gate[gate_off + r]) {
    if (threadIdx.x == 0) part[(size_t)r * gridDim.x + blockIdx.x] = mk<double>(0.0, 0.0);
    return;
  }
  VT *w = const_cast<VT *>(a.w[r]);
  const VT *V = a.basis[r];
  for (int i = threadIdx.x; i < nb; i += blockDim.x) {
    const c128 hv = h[(size_t)r * hstride + i];
    const double f = hscale ? hscale[(size_t)r * sstride + i] : 1.0;
    hs[i] = mk<double>(hv.x * f, hv.y * f);
  }
  __syncthreads();
  double acc = 0.0;
  if constexpr (P2) {
    const size_t n2 = n >> 1;
    float4 *w2 = reinterpret_cast<float4 *>(w);
    const float4 *V2 = reinterpret_cast<const float4 *>(V);
    for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n2;
         k += (size_t)gridDim.x * blockDim.x) {
      const float4 wq = w2[k];
      c128 wa = mk<double>(wq.x, wq.y), wb = mk<double>(wq.z, wq.w);
      for (int i = 0; i < nb; ++i) {
        const float4 vq = V2[(size_t)i * n2 + k];
        const c128 hv = hs[i];
        wa.x -= hv.x * (double)vq.x - hv.y * (double)vq.y;
        wa.y -= hv.x * (double)vq.y + hv.y * (double)vq.x;
        wb.x -= hv.x * (double)vq.z - hv.y * (double)vq.w;
        wb.y -= hv.x * (double)vq.w + hv.y * (double)vq.z;
      }
      w2[k] = make_float4((float)wa.x, (float)wa.y, (float)wb.x, (float)wb.y);
      acc += weight_of(2 * k, plane, nz, wlev) * (wa.x * wa.x + wa.y * wa.y);
      acc += weight_of(2 * k + 1, plane, nz, wlev) * (wb.x * wb.x + wb.y * wb.y);
    }
  } else {
    for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n;
         k += (size_t)gridDim.x * blockDim.x) {
      c128 wv = wide(w[k]);
      for (int i = 0; i < nb; ++i) {
        const c128 v = wide(V[(size_t)i * n + k]);
        const c128 hv = hs[i];
        wv.x -= hv.x * v.x - hv.y * v.y;
        wv.y -= hv.x * v.y + hv.y * v.x;
      }
      w[k] = store_as<VT>(wv);
      acc += weight_of(k, plane, nz, wlev) * (wv.x * wv.x + wv.y * wv.y);
    }
  }
  const double sum = block_sum(acc, red);
  if (threadIdx.x == 0) part[(size_t)r * gridDim.x + blockIdx.x] = mk<double>(sum, 0.0);
}

template <typename VT>
static hipError_t launch_update_t(const DotArgsT<VT> &a, int nrhs, int nb, size_t n, int nz,
                                  int plane, const double *wlev, const c128 *h, int hstride,
                                  const double *hscale, int sstride, c128 *part, c128 *nrm,
                                  hipStream_t s, const int *gate, int gate_off) {
  if (nb > 64) return hipErrorInvalidValue;
  dim3 grid(kRedBlocks, nrhs);
  if (pairs_ok(a, nrhs, n))
    k_update<VT, true><<<grid, 256, 0, s>>>(a, nb, n, nz, plane, wlev, h, hstride, hscale,
                                             sstride, part, gate, gate_off);
  else
    k_update<VT, false><<<grid, 256, 0, s>>>(a, nb, n, nz, plane, wlev, h, hstride, hscale,
                                              sstride, part, gate, gate_off);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_reduce<<<dim3(1, nrhs), 256, 0, s>>>(part, kRedBlocks, 1, nrm);
  return hipGetLastError();
}
hipError_t launch_update(const DotArgs &a, int nrhs, int nb, size_t n, int nz, int plane,
                         const double *wlev, const c128 *h, int hstride, const double *hscale,
                         int sstride, c128 *part, c128 *nrm, hipStream_t s, const int *gate,
                         int gate_off) {
  return launch_update_t(a, nrhs, nb, n, nz, plane, wlev, h, hstride, hscale, sstride, part, nrm,
                         s, gate, gate_off);
}
hipError_t launch_update(const DotArgs32 &a, int nrhs, int nb, size_t n, int nz, int plane,
                         const double *wlev, const c128 *h, int hstride, const double *hscale,
                         int sstride, c128 *part, c128 *nrm, hipStream_t s, const int *gate,
                         int gate_off) {
  return launch_update_t(a, nrhs, nb, n, nz, plane, wlev, h, hstride, hscale, sstride, part, nrm,
                         s, gate, gate_off);
}

template <typename VT>
__global__ void __launch_bounds__(256)
k_norms(const VT *__restrict__ v, size_t n, int nz, int plane, const double *__restrict__ wlev,
        c128 *__restrict__ part) {
  __shared__ double red[8];
  const int r = blockIdx.y;
  const VT *x = v + (size_t)r * n;
  double acc = 0.0;
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n;
       k += (size_t)gridDim.x * blockDim.x) {
    const c128 a = wide(x[k]);
    acc += weight_of(k, plane, nz, wlev) * (a.x * a.x + a.y * a.y);
  }
  const double sum = block_sum(acc, red);
  if (threadIdx.x == 0) part[(size_t)r * gridDim.x + blockIdx.x] = mk<double>(sum, 0.0);
}

template <typename VT>
static hipError_t launch_norms_t(const VT *v, int nrhs, size_t n, int nz, int plane,
                                 const double *wlev, c128 *part, c128 *nrm, hipStream_t s) {
  dim3 grid(kRedBlocks, nrhs);
  k_norms<VT><<<grid, 256, 0, s>>>(v, n, nz, plane, wlev, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_reduce<<<dim3(1, nrhs), 256, 0, s>>>(part, kRedBlocks, 1, nrm);
  return hipGetLastError();
}
hipError_t launch_norms(const c128 *v, int nrhs, size_t n, int nz, int plane, const double *wlev,
                        c128 *part, c128 *nrm, hipStream_t s) {
  return launch_norms_t(v, nrhs, n, nz, plane, wlev, part, nrm, s);
}
hipError_t launch_norms(const c64 *v, int nrhs, size_t n, int nz, int plane, const double *wlev,
                        c128 *part, c128 *nrm, hipStream_t s) {
  return launch_norms_t(v, nrhs, n, nz, plane, wlev, part, nrm, s);
}

template <typename VD, typename VS>
struct ScaleArgs {
  VD *dst[kMaxRhs];
  const VS *src[kMaxRhs];
  c128 f[kMaxRhs];
};

template <typename VD, typename VS>
__global__ void k_scale(ScaleArgs<VD, VS> a, size_t n) {
  const int r = blockIdx.y;
  const c128 f = a.f[r];
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n;
       k += (size_t)gridDim.x * blockDim.x)
    a.dst[r][k] = store_as<VD>(cmul(wide(a.src[r][k]), f));
}

template <typename VD, typename VS>
static hipError_t launch_scale_t(VD *const *dst, const VS *const *src, const c128 *scal, int nrhs,
                                 size_t n, hipStream_t s) {
  ScaleArgs<VD, VS> a;
  for (int r = 0; r < nrhs; ++r) {
    a.dst[r] = dst[r];
    a.src[r] = src[r];
    a.f[r] = scal[r];
  }
  k_scale<VD, VS><<<dim3(1024, nrhs), 256, 0, s>>>(a, n);
  return hipGetLastError();
}
hipError_t launch_scale(c128 *const *dst, const c128 *const *src, const c128 *scal, int nrhs,
                        size_t n, hipStream_t s) {
  return launch_scale_t(dst, src, scal, nrhs, n, s);
}
hipError_t launch_scale(c64 *const *dst, const c64 *const *src, const c128 *scal, int nrhs,
                        size_t n, hipStream_t s) {
  return launch_scale_t(dst, src, scal, nrhs, n, s);
}
hipError_t launch_scale(c64 *const *dst, const c128 *const *src, const c128 *scal, int nrhs,
                        size_t n, hipStream_t s) {
  return launch_scale_t(dst, src, scal, nrhs, n, s);
}

template <typename VT>
__global__ void k_lincomb(LinArgsT<VT> a, int nb, size_t n, const c128 *__restrict__ y,
                          int ystride) {
  __shared__ c128 ys[64];
  const int r = blockIdx.y;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) ys[i] = y[(size_t)r * ystride + i];
  __syncthreads();
  VT *x = a.x[r];
  const VT *V = a.basis[r];
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n;
       k += (size_t)gridDim.x * blockDim.x) {
    c128 acc = wide(x[k]);
    for (int i = 0; i < nb; ++i) cfma(acc, ys[i], wide(V[(size_t)i * n + k]));
    x[k] = store_as<VT>(acc);
  }
}

hipError_t launch_lincomb(const LinArgs &a, int nrhs, int nb, size_t n, const c128 *y,
                          int ystride, hipStream_t s) {
  if (nb > 64) return hipErrorInvalidValue;
  k_lincomb<c128><<<dim3(1024, nrhs), 256, 0, s>>>(a, nb, n, y, ystride);
  return hipGetLastError();
}
hipError_t launch_lincomb(const LinArgs32 &a, int nrhs, int nb, size_t n, const c128 *y,
                          int ystride, hipStream_t s) {
  if (nb > 64) return hipErrorInvalidValue;
  k_lincomb<c64><<<dim3(1024, nrhs), 256, 0, s>>>(a, nb, n, y, ystride);
  return hipGetLastError();
}

// out = alpha a + beta b in FP64, stored as the type of out
template <typename VO, typename VA, typename VB>
__global__ void k_axpby(VO *__restrict__ out, const VA *__restrict__ a, const VB *__restrict__ b,
                        c128 alpha, c128 beta, size_t n) {
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n;
       k += (size_t)gridDim.x * blockDim.x) {
    c128 v = cmul(alpha, wide(a[k]));
    cfma(v, beta, wide(b[k]));
    out[k] = store_as<VO>(v);
  }
}

hipError_t launch_axpby(c128 *out, const c128 *a, const c128 *b, c128 alpha, c128 beta, size_t n,
                        hipStream_t s) {
  k_axpby<<<1024, 256, 0, s>>>(out, a, b, alpha, beta, n);
  return hipGetLastError();
}
hipError_t launch_axpby(c64 *out, const c64 *a, const c64 *b, c128 alpha, c128 beta, size_t n,
                        hipStream_t s) {
  k_axpby<<<1024, 256, 0, s>>>(out, a, b, alpha, beta, n);
  return hipGetLastError();
}
hipError_t launch_axpby(c128 *out, const c128 *a, const c64 *b, c128 alpha, c128 beta, size_t n,
                        hipStream_t s) {
  k_axpby<<<1024, 256, 0, s>>>(out, a, b, alpha, beta, n);
  return hipGetLastError();
}

// out[r][comp][cell] = u[r][comp][cell] (op) acell[cell]
__global__ void k_cellop(c128 *__restrict__ out, const c128 *__restrict__ u,
                         const c128 *__restrict__ acell, size_t ncell, size_t n, int divide) {
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n;
       k += (size_t)gridDim.x * blockDim.x) {
    const c128 a = acell[k % ncell];
    const c128 v = u[k];
    if (divide) {
      const double dd = a.x * a.x + a.y * a.y;
      out[k] = mk<double>((v.x * a.x + v.y * a.y) / dd, (v.y * a.x - v.x * a.y) / dd);
    } else {
      out[k] = cmul(v, a);
    }
  }
}

hipError_t launch_div_cells(c128 *out, const c128 *u, const c128 *acell, int nrhs, size_t ncell,
                            hipStream_t s) {
  k_cellop<<<1024, 256, 0, s>>>(out, u, acell, ncell, (size_t)nrhs * 3 * ncell, 1);
  return hipGetLastError();
}

hipError_t launch_mul_cells(c128 *out, const c128 *u, const c128 *acell, int nrhs, size_t ncell,
                            hipStream_t s) {
  k_cellop<<<1024, 256, 0, s>>>(out, u, acell, ncell, (size_t)nrhs * 3 * ncell, 0);
  return hipGetLastError();
}

// ------------------------------------------------------- device-side Arnoldi
// For GMRES cycles captured in a HIP graph (no host round trip per step):
// the decision for the second Gram-Schmidt pass, and the Hessenberg column,
// Givens rotation and residual estimate of step j, all on the device.

// gate[q] = 1 when the projection removed more than 1 - drop of the squared
// norm (||w'||^2 < drop ||w||^2), i.e. the pass is to be repeated
__global__ void k_gs_gate(int nq, const c128 *__restrict__ h1, int hstride,
                          const c128 *__restrict__ nrm1, int *__restrict__ gate, double drop) {
  const int q = threadIdx.x;
  if (q < nq) gate[q] = nrm1[q].x < drop * h1[(size_t)q * hstride + hstride - 1].x ? 1 : 0;
}

hipError_t launch_gs_gate(int nq, const c128 *h1, int hstride, const c128 *nrm1, int *gate,
                          double drop, hipStream_t s) {
  if (nq > 64) return hipErrorInvalidValue;
  k_gs_gate<<<1, 64, 0, s>>>(nq, h1, hstride, nrm1, gate, drop);
  return hipGetLastError();
}

__device__ __forceinline__ c128 cconj(c128 a) { return mk<double>(a.x, -a.y); }
__device__ __forceinline__ double cabs2(c128 a) { return hypot(a.x, a.y); }
__device__ __forceinline__ c128 cscal(c128 a, double f) { return mk<double>(a.x * f, a.y * f); }

// Step j of the Arnoldi process of systems q0 .. q0 + nq - 1 (one thread
// each).  The basis is kept unnormalised (vn2[i] = |V_i|^2); h1c (and h2c
// after a second pass, gate[q] set) hold <V_i, w> for i <= j of system q0 + t
// at offset t (j + 2); nrm1 and nrm2 the squared norm of the projected w after
// each pass.
__global__ void k_arnoldi_tail(ArnoldiState st, const c128 *__restrict__ h1c,
                               const c128 *__restrict__ h2c, int q0, int nq, int j, int m) {
  const int q = q0 + (int)threadIdx.x;
  if ((int)threadIdx.x >= nq) return;
  const int hs = j + 2;
  const c128 *h1 = h1c + (size_t)threadIdx.x * hs;
  const c128 *h2 = h2c + (size_t)threadIdx.x * hs;
  const bool two = st.gate[q] != 0;
  double *vn2 = st.vn2 + (size_t)q * kArnStride;
  double *scl = st.scale + (size_t)q * kArnStride;
  c128 *H = st.H + (size_t)q * (m + 1) * m;
  c128 *cs = st.cs + (size_t)q * m;
  c128 *sn = st.sn + (size_t)q * m;
  c128 *g = st.g + (size_t)q * (m + 1);
  const double nw = fmax(two ? st.nrm2[q].x : st.nrm1[q].x, 0.0);
  const double vj = sqrt(vn2[j]);
  for (int i = 0; i <= j; ++i) {
    c128 hv = h1[i];
    if (two) hv = cadd(hv, h2[i]);
    const double d = sqrt(vn2[i]) * vj;
    H[(size_t)i * m + j] = d > 0.0 ? cscal(hv, 1.0 / d) : mk<double>(0.0, 0.0);
  }
  const double wn = sqrt(nw);
  const double hn = vj > 0.0 ? wn / vj : 0.0;
  vn2[j + 1] = nw;
  scl[j + 1] = nw > 0.0 ? 1.0 / nw : 0.0;
  c128 hj1 = mk<double>(hn, 0.0);
  for (int i = 0; i < j; ++i) {  // earlier rotations
    const c128 a = H[(size_t)i * m + j], b = H[(size_t)(i + 1) * m + j];
    H[(size_t)i * m + j] = cadd(cmul(cs[i], a), cmul(sn[i], b));
    H[(size_t)(i + 1) * m + j] = csub(cmul(cs[i], b), cmul(cconj(sn[i]), a));
  }
  const c128 a = H[(size_t)j * m + j];
  const double an = cabs2(a), bn = cabs2(hj1);
  const double rr = hypot(an, bn);
  c128 c, sv;
  if (an == 0.0) {
    c = mk<double>(0.0, 0.0);
    sv = mk<double>(1.0, 0.0);
  } else {
    c = mk<double>(an / rr, 0.0);
    sv = cscal(cmul(cscal(a, 1.0 / an), cconj(hj1)), 1.0 / rr);
  }
  cs[j] = c;
  sn[j] = sv;
  H[(size_t)j * m + j] = cadd(cmul(c, a), cmul(sv, hj1));
  H[(size_t)(j + 1) * m + j] = mk<double>(0.0, 0.0);
  const c128 gj = g[j];
  g[j + 1] = cscal(cmul(cconj(sv), gj), -1.0);
  g[j] = cmul(c, gj);
  const double est = cabs2(g[j + 1]);
  if (!st.conv[q] && (est <= st.tolb[q] || hn == 0.0)) {
    st.conv[q] = 1;
    st.jlen[q] = j + 1;
  }
}

hipError_t launch_arnoldi_tail(const ArnoldiState &st, const c128 *h1c, const c128 *h2c, int q0,
                               int nq, int j, int m, hipStream_t s) {
  if (nq > 64) return hipErrorInvalidValue;
  k_arnoldi_tail<<<1, 64, 0, s>>>(st, h1c, h2c, q0, nq, j, m);
  return hipGetLastError();
}

}  // namespace giem
