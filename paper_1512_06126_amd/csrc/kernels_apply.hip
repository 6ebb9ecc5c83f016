// HIP kernels of the operator apply (Sect. 3.3 of the paper, three-step
// algorithm for the block-Toeplitz product B x):
//   step 1  forward 2-D FFT of the 3 Nz zero-padded planes  (x pass, y pass)
//   step 2  Nz-order block products with the stored spectra Q~(Kx, Ky)
//   step 3  inverse 2-D FFT                                   (y pass, x pass)
// The diagonal scalings of A = S + R1 B R2 (Sect. 3.1) are fused into the
// first and the last pass.
//
// Spectra live in one buffer laid out [Ky][Kx][r][p] (p = alpha Nz + iz is
// the plane, fastest), so that the block product reads the 3 Nz R values of a
// frequency point as one contiguous run and the FFT passes move G adjacent
// planes (128-byte runs) per frequency point.
//
// FFTs are mixed-radix (4, 2, 3, 5, 7) Stockham passes done in LDS, G
// sequences per workgroup, twiddles from a per-length table.
#include "kernels.h"

namespace giem {

constexpr int kFftThreads = 256;  // workgroup size of the FFT passes

// ------------------------------------------------------------------ small DFTs
template <typename T, int P>
__device__ __forceinline__ void small_dft(cplx<T> (&v)[P], bool inv,
                                          const cplx<T> *__restrict__ tw, int L) {
  if constexpr (P == 2) {
    cplx<T> a = cadd(v[0], v[1]);
    cplx<T> b = csub(v[0], v[1]);
    v[0] = a;
    v[1] = b;
  } else if constexpr (P == 4) {
    cplx<T> t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
    cplx<T> t2 = cadd(v[1], v[3]), t3 = csub(v[1], v[3]);
    // forward: y1 = t1 - i t3, y3 = t1 + i t3; inverse swaps them
    cplx<T> mit3 = mk<T>(t3.y, -t3.x);  // -i t3
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    if (!inv) {
      v[1] = cadd(t1, mit3);
      v[3] = csub(t1, mit3);
    } else {
      v[1] = csub(t1, mit3);
      v[3] = cadd(t1, mit3);
    }
  } else {
    // generic odd radix: y_t = sum_s x_s W^(s t mod P), W = exp(-+ 2 pi i / P)
    cplx<T> out[P];
    const int step = L / P;
#pragma unroll
    for (int t = 0; t < P; ++t) {
      cplx<T> acc = v[0];
#pragma unroll
      for (int s = 1; s < P; ++s) {
        cplx<T> w = tw[((s * t) % P) * step];
        if (inv) w.y = -w.y;
        cfma(acc, v[s], w);
      }
      out[t] = acc;
    }
#pragma unroll
    for (int t = 0; t < P; ++t) v[t] = out[t];
  }
}

// One Stockham pass of radix P over G sequences of length L held in LDS
// (row stride ld).  ns = product of the radices of the earlier passes.
// Butterfly j reads x[j + q L/P], applies the twiddle exp(-+2 pi i q k/(ns P))
// (k = j mod ns) and writes y[(j / ns) ns P + k + q ns]; after all passes the
// sequence is in natural order.  Inputs are staged in registers so the pass
// works in place.
template <typename T, int P, int EPT>
__device__ __forceinline__ void fft_pass(cplx<T> *buf, int G, int ld, int L, int ns,
                                         const cplx<T> *__restrict__ tw, bool inv) {
  constexpr int MB = (EPT + P - 1) / P;
  const int nthr = blockDim.x;
  const int lp = L / P;
  const int nb = G * lp;
  cplx<T> v[MB][P];
#pragma unroll
  for (int i = 0; i < MB; ++i) {
    const int b = threadIdx.x + i * nthr;
    if (b < nb) {
      const int g = b / lp, j = b - g * lp;
#pragma unroll
      for (int q = 0; q < P; ++q) v[i][q] = buf[g * ld + j + q * lp];
    }
  }
  __syncthreads();
  const int tstride = L / (ns * P);
#pragma unroll
  for (int i = 0; i < MB; ++i) {
    const int b = threadIdx.x + i * nthr;
    if (b < nb) {
      const int g = b / lp, j = b - g * lp;
      const int k = j % ns;
      if (k != 0) {
#pragma unroll
        for (int q = 1; q < P; ++q) {
          cplx<T> w = tw[q * k * tstride];
          if (inv) w.y = -w.y;
          v[i][q] = cmul(v[i][q], w);
        }
      }
      small_dft<T, P>(v[i], inv, tw, L);
      const int base = g * ld + (j / ns) * ns * P + k;
#pragma unroll
      for (int q = 0; q < P; ++q) buf[base + q * ns] = v[i][q];
    }
  }
  __syncthreads();
}

template <typename T, int EPT>
__device__ void fft_lds(cplx<T> *buf, int G, int ld, const FftDesc &fd,
                        const cplx<T> *__restrict__ tw, bool inv) {
  __syncthreads();
  int ns = 1;
  for (int s = 0; s < fd.nf; ++s) {
    const int p = fd.fac[s];
    switch (p) {
      case 4: fft_pass<T, 4, EPT>(buf, G, ld, fd.L, ns, tw, inv); break;
      case 2: fft_pass<T, 2, EPT>(buf, G, ld, fd.L, ns, tw, inv); break;
      case 3: fft_pass<T, 3, EPT>(buf, G, ld, fd.L, ns, tw, inv); break;
      case 5: fft_pass<T, 5, EPT>(buf, G, ld, fd.L, ns, tw, inv); break;
      default: fft_pass<T, 7, EPT>(buf, G, ld, fd.L, ns, tw, inv); break;
    }
    ns *= p;
  }
}

// ---------------------------------------------------------------- x passes
// Step 1, x pass: u -> R2 u (or u), zero-pad to 2 Nx, forward FFT along x.
// Grid: (y, plane group).  Output rows y < Ny of the spectra buffer.
template <typename T, int EPT>
__global__ void __launch_bounds__(kFftThreads)
k_fft_x_fwd(VecPtrs ptrs, const c128 *__restrict__ r2, cplx<T> *__restrict__ spec, int nx,
            int ny, int nz, int rp_total, int G, FftDesc fd, const cplx<T> *__restrict__ tw) {
  extern __shared__ unsigned char smem_raw[];
  cplx<T> *buf = reinterpret_cast<cplx<T> *>(smem_raw);
  const int L = fd.L, ld = L + 1;
  const int y = blockIdx.x;
  const int rp0 = blockIdx.y * G;
  const int p3 = 3 * nz;
  const size_t plane = (size_t)nx * ny;
  // all global loads of a thread are issued before its LDS stores
  c128 va[EPT], vs[EPT];
#pragma unroll
  for (int u = 0; u < EPT; ++u) {
    const int e = threadIdx.x + u * kFftThreads;
    const int g = e / L, xx = e - g * L;
    const int rp = rp0 + g;
    va[u] = mk<double>(0, 0);
    vs[u] = mk<double>(1, 0);
    if (e < G * L && xx < nx && rp < rp_total) {
      const int r = rp / p3, p = rp - r * p3;
      const int iz = p % nz;
      va[u] = ptrs.in[r][(size_t)p * plane + (size_t)y * nx + xx];
      if (r2) vs[u] = r2[(size_t)iz * plane + (size_t)y * nx + xx];
    }
  }
#pragma unroll
  for (int u = 0; u < EPT; ++u) {
    const int e = threadIdx.x + u * kFftThreads;
    if (e < G * L) {
      const int g = e / L, xx = e - g * L;
      buf[g * ld + xx] = ccast<T>(cmul(va[u], vs[u]));
    }
  }
  fft_lds<T, EPT>(buf, G, ld, fd, tw, false);
  for (int e = threadIdx.x; e < G * L; e += blockDim.x) {
    const int K = e / G, g = e - K * G;
    const int rp = rp0 + g;
    if (rp < rp_total) spec[((size_t)y * L + K) * rp_total + rp] = buf[g * ld + K];
  }
}

// Step 3, x pass: inverse FFT along x, keep x < Nx, scale by 1/(4 Nx Ny) and
// finish the operator: y = S u + R1 (B R2 u)  (mode A, with R1/R2 swapped for
// A^T), or y = B u (mode B: s == nullptr, r1 == nullptr).
template <typename T, int EPT>
__global__ void __launch_bounds__(kFftThreads)
k_fft_x_inv(VecPtrs ptrs, const c128 *__restrict__ sdiag, const c128 *__restrict__ r1,
            const cplx<T> *__restrict__ spec, int nx, int ny, int nz, int rp_total, int G,
            FftDesc fd, const cplx<T> *__restrict__ tw, double scale) {
  extern __shared__ unsigned char smem_raw[];
  cplx<T> *buf = reinterpret_cast<cplx<T> *>(smem_raw);
  const int L = fd.L, ld = L + 1;
  const int y = blockIdx.x;
  const int rp0 = blockIdx.y * G;
  const int p3 = 3 * nz;
  const size_t plane = (size_t)nx * ny;
  {
    cplx<T> v[EPT];
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
      const int e = threadIdx.x + u * kFftThreads;
      const int K = e / G, g = e - K * G;
      const int rp = rp0 + g;
      v[u] = mk<T>(0, 0);
      if (e < G * L && rp < rp_total) v[u] = spec[((size_t)y * L + K) * rp_total + rp];
    }
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
      const int e = threadIdx.x + u * kFftThreads;
      if (e < G * L) {
        const int K = e / G, g = e - K * G;
        buf[g * ld + K] = v[u];
      }
    }
  }
  // the diagonal terms of the epilogue are loaded while the FFT runs
  constexpr int EO = (EPT + 1) / 2;  // G * nx <= G * L / 2 outputs
  c128 xin[EO], dsd[EO], dr1[EO];
  if (r1) {
#pragma unroll
    for (int u = 0; u < EO; ++u) {
      const int e = threadIdx.x + u * kFftThreads;
      const int g = e / nx, xx = e - g * nx;
      const int rp = rp0 + g;
      if (e < G * nx && rp < rp_total) {
        const int r = rp / p3, p = rp - r * p3;
        const int iz = p % nz;
        const size_t cell = (size_t)iz * plane + (size_t)y * nx + xx;
        xin[u] = ptrs.in[r][(size_t)p * plane + (size_t)y * nx + xx];
        dsd[u] = sdiag[cell];
        dr1[u] = r1[cell];
      }
    }
  }
  fft_lds<T, EPT>(buf, G, ld, fd, tw, true);
#pragma unroll
  for (int u = 0; u < EO; ++u) {
    const int e = threadIdx.x + u * kFftThreads;
    const int g = e / nx, xx = e - g * nx;
    const int rp = rp0 + g;
    if (e < G * nx && rp < rp_total) {
      const int r = rp / p3, p = rp - r * p3;
      const size_t off = (size_t)p * plane + (size_t)y * nx + xx;
      c128 b = ccast<double>(buf[g * ld + xx]);
      b = cscale(b, scale);
      c128 out = b;
      if (r1) {
        out = cmul(dr1[u], b);
        cfma(out, dsd[u], xin[u]);
      }
      ptrs.out[r][off] = out;
    }
  }
}

// ---------------------------------------------------------------- y passes
// Forward (rows y >= Ny are zero, output all 2 Ny rows) or inverse (read all
// 2 Ny rows, write rows < Ny) FFT along y, in place.  Grid: (Kx, plane group).
template <typename T, int EPT>
__global__ void __launch_bounds__(kFftThreads)
k_fft_y(cplx<T> *__restrict__ spec, int nx2, int ny, int rp_total, int G, FftDesc fd,
        const cplx<T> *__restrict__ tw, int inverse) {
  extern __shared__ unsigned char smem_raw[];
  cplx<T> *buf = reinterpret_cast<cplx<T> *>(smem_raw);
  const int L = fd.L, ld = L + 1;
  const int kx = blockIdx.x;
  const int rp0 = blockIdx.y * G;
  const int nin = inverse ? L : ny;
  const int nout = inverse ? ny : L;
  {
    cplx<T> v[EPT];
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
      const int e = threadIdx.x + u * kFftThreads;
      const int yy = e / G, g = e - yy * G;
      const int rp = rp0 + g;
      v[u] = mk<T>(0, 0);
      if (e < G * L && yy < nin && rp < rp_total) v[u] = spec[((size_t)yy * nx2 + kx) * rp_total + rp];
    }
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
      const int e = threadIdx.x + u * kFftThreads;
      if (e < G * L) {
        const int yy = e / G, g = e - yy * G;
        buf[g * ld + yy] = v[u];
      }
    }
  }
  fft_lds<T, EPT>(buf, G, ld, fd, tw, inverse != 0);
  for (int e = threadIdx.x; e < G * nout; e += blockDim.x) {
    const int yy = e / G, g = e - yy * G;
    const int rp = rp0 + g;
    if (rp < rp_total) spec[((size_t)yy * nx2 + kx) * rp_total + rp] = buf[g * ld + yy];
  }
}

// ---------------------------------------------------------------- launchers
static int ept_for(int G, int L, int nthr) {
  const int need = (G * L + nthr - 1) / nthr;
  if (need <= 4) return 4;
  if (need <= 8) return 8;
  if (need <= 16) return 16;
  return 32;
}

template <typename T>
static hipError_t launch_fft_x_fwd_t(const VecPtrs &ptrs, const c128 *r2, void *spec, int nx,
                                     int ny, int nz, int rp_total, int G, const FftDesc &fd,
                                     const void *tw, hipStream_t s) {
  const int nthr = 256;
  dim3 grid(ny, (rp_total + G - 1) / G);
  size_t lds = (size_t)G * (fd.L + 1) * sizeof(cplx<T>);
  const cplx<T> *twp = static_cast<const cplx<T> *>(tw);
  cplx<T> *sp = static_cast<cplx<T> *>(spec);
  switch (ept_for(G, fd.L, nthr)) {
    case 4: k_fft_x_fwd<T, 4><<<grid, nthr, lds, s>>>(ptrs, r2, sp, nx, ny, nz, rp_total, G, fd, twp); break;
    case 8: k_fft_x_fwd<T, 8><<<grid, nthr, lds, s>>>(ptrs, r2, sp, nx, ny, nz, rp_total, G, fd, twp); break;
    case 16: k_fft_x_fwd<T, 16><<<grid, nthr, lds, s>>>(ptrs, r2, sp, nx, ny, nz, rp_total, G, fd, twp); break;
    default: k_fft_x_fwd<T, 32><<<grid, nthr, lds, s>>>(ptrs, r2, sp, nx, ny, nz, rp_total, G, fd, twp); break;
  }
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_fft_x_inv_t(const VecPtrs &ptrs, const c128 *sd, const c128 *r1,
                                     const void *spec, int nx, int ny, int nz, int rp_total,
                                     int G, const FftDesc &fd, const void *tw, double scale,
                                     hipStream_t s) {
  const int nthr = 256;
  dim3 grid(ny, (rp_total + G - 1) / G);
  size_t lds = (size_t)G * (fd.L + 1) * sizeof(cplx<T>);
  const cplx<T> *twp = static_cast<const cplx<T> *>(tw);
  const cplx<T> *sp = static_cast<const cplx<T> *>(spec);
  switch (ept_for(G, fd.L, nthr)) {
    case 4: k_fft_x_inv<T, 4><<<grid, nthr, lds, s>>>(ptrs, sd, r1, sp, nx, ny, nz, rp_total, G, fd, twp, scale); break;
    case 8: k_fft_x_inv<T, 8><<<grid, nthr, lds, s>>>(ptrs, sd, r1, sp, nx, ny, nz, rp_total, G, fd, twp, scale); break;
    case 16: k_fft_x_inv<T, 16><<<grid, nthr, lds, s>>>(ptrs, sd, r1, sp, nx, ny, nz, rp_total, G, fd, twp, scale); break;
    default: k_fft_x_inv<T, 32><<<grid, nthr, lds, s>>>(ptrs, sd, r1, sp, nx, ny, nz, rp_total, G, fd, twp, scale); break;
  }
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_fft_y_t(void *spec, int nx2, int ny, int rp_total, int G,
                                 const FftDesc &fd, const void *tw, int inverse, hipStream_t s) {
  const int nthr = 256;
  dim3 grid(nx2, (rp_total + G - 1) / G);
  size_t lds = (size_t)G * (fd.L + 1) * sizeof(cplx<T>);
  const cplx<T> *twp = static_cast<const cplx<T> *>(tw);
  cplx<T> *sp = static_cast<cplx<T> *>(spec);
  switch (ept_for(G, fd.L, nthr)) {
    case 4: k_fft_y<T, 4><<<grid, nthr, lds, s>>>(sp, nx2, ny, rp_total, G, fd, twp, inverse); break;
    case 8: k_fft_y<T, 8><<<grid, nthr, lds, s>>>(sp, nx2, ny, rp_total, G, fd, twp, inverse); break;
    case 16: k_fft_y<T, 16><<<grid, nthr, lds, s>>>(sp, nx2, ny, rp_total, G, fd, twp, inverse); break;
    default: k_fft_y<T, 32><<<grid, nthr, lds, s>>>(sp, nx2, ny, rp_total, G, fd, twp, inverse); break;
  }
  return hipGetLastError();
}

size_t fft_lds_bytes(int G, int L, int prec) {
  const size_t c = prec == PREC_FP32 ? sizeof(c64) : sizeof(c128);
  return (size_t)G * (L + 1) * c;
}

hipError_t set_lds_limits() {
  // gfx950 has 160 KB of LDS per CU; allow the large dynamic allocations.
  const int lim = 160 * 1024;
  hipError_t e = hipSuccess;
#define GIEM_SET(k) \
  if (e == hipSuccess) e = hipFuncSetAttribute(reinterpret_cast<const void *>(k), hipFuncAttributeMaxDynamicSharedMemorySize, lim)
  GIEM_SET((k_fft_x_fwd<double, 4>)); GIEM_SET((k_fft_x_fwd<double, 8>)); GIEM_SET((k_fft_x_fwd<double, 16>)); GIEM_SET((k_fft_x_fwd<double, 32>));
  GIEM_SET((k_fft_x_fwd<float, 4>)); GIEM_SET((k_fft_x_fwd<float, 8>)); GIEM_SET((k_fft_x_fwd<float, 16>)); GIEM_SET((k_fft_x_fwd<float, 32>));
  GIEM_SET((k_fft_x_inv<double, 4>)); GIEM_SET((k_fft_x_inv<double, 8>)); GIEM_SET((k_fft_x_inv<double, 16>)); GIEM_SET((k_fft_x_inv<double, 32>));
  GIEM_SET((k_fft_x_inv<float, 4>)); GIEM_SET((k_fft_x_inv<float, 8>)); GIEM_SET((k_fft_x_inv<float, 16>)); GIEM_SET((k_fft_x_inv<float, 32>));
  GIEM_SET((k_fft_y<double, 4>)); GIEM_SET((k_fft_y<double, 8>)); GIEM_SET((k_fft_y<double, 16>)); GIEM_SET((k_fft_y<double, 32>));
  GIEM_SET((k_fft_y<float, 4>)); GIEM_SET((k_fft_y<float, 8>)); GIEM_SET((k_fft_y<float, 16>)); GIEM_SET((k_fft_y<float, 32>));
#undef GIEM_SET
  if (e == hipSuccess) e = set_block_lds_limits();
  return e;
}

hipError_t launch_fft_x_fwd(int prec, const VecPtrs &ptrs, const c128 *r2, void *spec, int nx,
                            int ny, int nz, int rp_total, int G, const FftDesc &fd,
                            const void *tw, hipStream_t s) {
  return prec == PREC_FP32
             ? launch_fft_x_fwd_t<float>(ptrs, r2, spec, nx, ny, nz, rp_total, G, fd, tw, s)
             : launch_fft_x_fwd_t<double>(ptrs, r2, spec, nx, ny, nz, rp_total, G, fd, tw, s);
}
hipError_t launch_fft_x_inv(int prec, const VecPtrs &ptrs, const c128 *sd, const c128 *r1,
                            const void *spec, int nx, int ny, int nz, int rp_total, int G,
                            const FftDesc &fd, const void *tw, double scale, hipStream_t s) {
  return prec == PREC_FP32
             ? launch_fft_x_inv_t<float>(ptrs, sd, r1, spec, nx, ny, nz, rp_total, G, fd, tw, scale, s)
             : launch_fft_x_inv_t<double>(ptrs, sd, r1, spec, nx, ny, nz, rp_total, G, fd, tw, scale, s);
}
hipError_t launch_fft_y(int prec, void *spec, int nx2, int ny, int rp_total, int G,
                        const FftDesc &fd, const void *tw, int inverse, hipStream_t s) {
  return prec == PREC_FP32 ? launch_fft_y_t<float>(spec, nx2, ny, rp_total, G, fd, tw, inverse, s)
                           : launch_fft_y_t<double>(spec, nx2, ny, rp_total, G, fd, tw, inverse, s);
}
}  // namespace giem
