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
// FFTs are mixed-radix (16, 8, 4, 2, 3, 5, 7, 11) Stockham passes done in LDS,
// G sequences per workgroup; radix 16 and 8 are nested length-4 transforms in
// registers, so a 256-point transform takes two passes through LDS.  Twiddles
// between passes come from a per-length table.
#include "kernels.h"

namespace giem {

template <typename VT>
struct VTraits;
template <>
struct VTraits<c128> {
  using elem = double;
};
template <>
struct VTraits<c64> {
  using elem = float;
};

// ------------------------------------------------------------------ small DFTs
// The LDS copy of a sequence is padded by one element after every 16, so
// that the strided Stockham writes of radix 16, 8, 4 and 2 spread over all
// banks (element offsets 17, 8.5, 4.25, 2.125 per lane are distinct mod 16).
__host__ __device__ __forceinline__ int lds_pad(int i) { return i + (i >> 4); }
__host__ __device__ __forceinline__ int fft_ld(int L) { return L + (L >> 4) + 1; }

// cos and sin of 2 pi m / 16
__device__ constexpr double kC16[16] = {1.0, 0.92387953251128674, 0.70710678118654752, 0.38268343236508977,
                                        0.0, -0.38268343236508977, -0.70710678118654752, -0.92387953251128674,
                                        -1.0, -0.92387953251128674, -0.70710678118654752, -0.38268343236508977,
                                        0.0, 0.38268343236508977, 0.70710678118654752, 0.92387953251128674};
__device__ constexpr double kS16[16] = {0.0, 0.38268343236508977, 0.70710678118654752, 0.92387953251128674,
                                        1.0, 0.92387953251128674, 0.70710678118654752, 0.38268343236508977,
                                        0.0, -0.38268343236508977, -0.70710678118654752, -0.92387953251128674,
                                        -1.0, -0.92387953251128674, -0.70710678118654752, -0.38268343236508977};

// v * exp(-+ 2 pi i m / 16) (minus for the forward transform)
template <typename T>
__device__ __forceinline__ cplx<T> rot16(cplx<T> v, int m, bool inv) {
  const T c = (T)kC16[m & 15], sn = inv ? (T)kS16[m & 15] : -(T)kS16[m & 15];
  return mk<T>(v.x * c - v.y * sn, v.x * sn + v.y * c);
}

template <typename T>
__device__ __forceinline__ void dft4(cplx<T> &a0, cplx<T> &a1, cplx<T> &a2, cplx<T> &a3, bool inv) {
  const cplx<T> t0 = cadd(a0, a2), t1 = csub(a0, a2), t2 = cadd(a1, a3), t3 = csub(a1, a3);
  const cplx<T> mit3 = mk<T>(t3.y, -t3.x);  // -i t3
  a0 = cadd(t0, t2);
  a2 = csub(t0, t2);
  // forward: y1 = t1 - i t3, y3 = t1 + i t3; the inverse swaps them
  a1 = inv ? csub(t1, mit3) : cadd(t1, mit3);
  a3 = inv ? cadd(t1, mit3) : csub(t1, mit3);
}

template <typename T, int P>
__device__ __forceinline__ void small_dft(cplx<T> (&v)[P], bool inv,
                                          const cplx<T> *__restrict__ tw, int L) {
  if constexpr (P == 2) {
    cplx<T> a = cadd(v[0], v[1]);
    cplx<T> b = csub(v[0], v[1]);
    v[0] = a;
    v[1] = b;
  } else if constexpr (P == 4) {
    dft4(v[0], v[1], v[2], v[3], inv);
  } else if constexpr (P == 8) {
    // n = n1 + 2 n2, k = k2 + 4 k1: length-4 DFTs over n2, twiddles
    // W8^(n1 k2), length-2 DFTs over n1
    dft4(v[0], v[2], v[4], v[6], inv);
    dft4(v[1], v[3], v[5], v[7], inv);
    cplx<T> b[4];
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) b[k2] = rot16(v[2 * k2 + 1], 2 * k2, inv);
    cplx<T> out[8];
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) {
      out[k2] = cadd(v[2 * k2], b[k2]);
      out[k2 + 4] = csub(v[2 * k2], b[k2]);
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = out[k];
  } else if constexpr (P == 16) {
    // n = n1 + 4 n2, k = k2 + 4 k1: length-4 DFTs over n2, twiddles
    // W16^(n1 k2), length-4 DFTs over n1
#pragma unroll
    for (int n1 = 0; n1 < 4; ++n1) dft4(v[n1], v[n1 + 4], v[n1 + 8], v[n1 + 12], inv);
#pragma unroll
    for (int n1 = 1; n1 < 4; ++n1)
#pragma unroll
      for (int k2 = 1; k2 < 4; ++k2) v[n1 + 4 * k2] = rot16(v[n1 + 4 * k2], n1 * k2, inv);
    // now v[n1 + 4 k2] holds the twiddled inner results
    cplx<T> out[16];
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) {
      cplx<T> a0 = v[4 * k2], a1 = v[4 * k2 + 1], a2 = v[4 * k2 + 2], a3 = v[4 * k2 + 3];
      dft4(a0, a1, a2, a3, inv);
      out[k2] = a0;
      out[k2 + 4] = a1;
      out[k2 + 8] = a2;
      out[k2 + 12] = a3;
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = out[k];
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
// The thread index is made opaque to the compiler at every pass, so that the
// LDS addresses derived from it (the same in every pass of one radix) are
// recomputed per pass rather than held in registers across the whole
// transform: in FP64 the power-of-two passes drop from 128-140 to 88-98
// VGPRs and the mixed-radix ones from 184-235 to 103-144, none spilling.
template <typename T, int P, int EPT>
__device__ __forceinline__ void fft_pass(cplx<T> *buf, int G, int ld, int L, int ns,
                                         const cplx<T> *__restrict__ tw, bool inv) {
  constexpr int MB = (EPT + P - 1) / P;
  const int nthr = blockDim.x;
  int tid = threadIdx.x;
  asm volatile("" : "+v"(tid));
  const int lp = L / P;
  const int nb = G * lp;
  cplx<T> v[MB][P];
#pragma unroll
  for (int i = 0; i < MB; ++i) {
    const int b = tid + i * nthr;
    if (b < nb) {
      const int g = b / lp, j = b - g * lp;
#pragma unroll
      for (int q = 0; q < P; ++q) v[i][q] = buf[g * ld + lds_pad(j + q * lp)];
    }
  }
  __syncthreads();
  const int tstride = L / (ns * P);
#pragma unroll
  for (int i = 0; i < MB; ++i) {
    const int b = tid + i * nthr;
    if (b < nb) {
      const int g = b / lp, j = b - g * lp;
      const int k = j % ns;
      if (k != 0) {
        if constexpr (P >= 8) {
          // W^q by a running product from one table entry (at most P - 1
          // products deep: a few units of rounding), instead of P - 1 loads
          // held in registers
          cplx<T> w1 = tw[k * tstride];
          if (inv) w1.y = -w1.y;
          cplx<T> w = w1;
#pragma unroll
          for (int q = 1; q < P; ++q) {
            v[i][q] = cmul(v[i][q], w);
            if (q + 1 < P) w = cmul(w, w1);
          }
        } else {
#pragma unroll
          for (int q = 1; q < P; ++q) {
            cplx<T> w = tw[q * k * tstride];
            if (inv) w.y = -w.y;
            v[i][q] = cmul(v[i][q], w);
          }
        }
      }
      small_dft<T, P>(v[i], inv, tw, L);
      const int base = (j / ns) * ns * P + k;
#pragma unroll
      for (int q = 0; q < P; ++q) buf[g * ld + lds_pad(base + q * ns)] = v[i][q];
    }
  }
  __syncthreads();
}

// All passes of one transform.  POW2 instantiations (lengths 2^k) carry
// only the radix 16, 8, 4 and 2 passes: register allocation takes the
// largest path of the switch, and the odd-radix passes would cost occupancy.
template <typename T, int EPT, bool POW2>
__device__ void fft_lds(cplx<T> *buf, int G, int ld, const FftDesc &fd,
                        const cplx<T> *__restrict__ tw, bool inv) {
  __syncthreads();
  int ns = 1;
  for (int s = 0; s < fd.nf; ++s) {
    const int p = fd.fac[s];
    if constexpr (POW2) {
      switch (p) {
        case 16: fft_pass<T, 16, EPT>(buf, G, ld, fd.L, ns, tw, inv); break;
        case 8: fft_pass<T, 8, EPT>(buf, G, ld, fd.L, ns, tw, inv); break;
        case 4: fft_pass<T, 4, EPT>(buf, G, ld, fd.L, ns, tw, inv); break;
        default: fft_pass<T, 2, EPT>(buf, G, ld, fd.L, ns, tw, inv); break;
      }
    } else {
      switch (p) {
        case 16: fft_pass<T, 16, EPT>(buf, G, ld, fd.L, ns, tw, inv); break;
        case 8: fft_pass<T, 8, EPT>(buf, G, ld, fd.L, ns, tw, inv); break;
        case 4: fft_pass<T, 4, EPT>(buf, G, ld, fd.L, ns, tw, inv); break;
        case 2: fft_pass<T, 2, EPT>(buf, G, ld, fd.L, ns, tw, inv); break;
        case 3: fft_pass<T, 3, EPT>(buf, G, ld, fd.L, ns, tw, inv); break;
        case 5: fft_pass<T, 5, EPT>(buf, G, ld, fd.L, ns, tw, inv); break;
        case 7: fft_pass<T, 7, EPT>(buf, G, ld, fd.L, ns, tw, inv); break;
        default: fft_pass<T, 11, EPT>(buf, G, ld, fd.L, ns, tw, inv); break;
      }
    }
    ns *= p;
  }
}

// ---------------------------------------------------------------- x passes
// Step 1, x pass: u -> R2 u (or u), zero-pad to 2 Nx, forward FFT along x.
// Grid: (y, plane group).  Output rows y < Ny of the spectra buffer.
// With the transform's LDS addresses recomputed per pass (fft_pass) the
// FP64 kernel takes 98 VGPRs for power-of-two lengths (54 -> 48.5 us at
// 128 x 128 x 32 with 8 planes on 256 threads; the floor of four
// wavefronts per SIMD no longer binds).
template <typename T, int EPT, int NT, bool POW2, typename VT>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(POW2 ? 4 : 1)))
k_fft_x_fwd(VecPtrsT<VT> ptrs, const c128 *__restrict__ r2, cplx<T> *__restrict__ spec, int nx,
            int ny, int nz, int rp_total, int G, FftDesc fd, const cplx<T> *__restrict__ tw) {
  extern __shared__ unsigned char smem_raw[];
  cplx<T> *buf = reinterpret_cast<cplx<T> *>(smem_raw);
  const int L = fd.L, ld = fft_ld(L);
  const int y = blockIdx.x;
  const int rp0 = blockIdx.y * G;
  const int p3 = 3 * nz;
  const size_t plane = (size_t)nx * ny;
  // only the first nx of the L = 2 nx entries of a sequence are nonzero: the
  // G nx loads are spread over all threads, the padding is zero-filled
  constexpr int EH = (EPT + 1) / 2;
  c128 va[EH], vs[EH];
#pragma unroll
  for (int u = 0; u < EH; ++u) {
    const int e = threadIdx.x + u * NT;
    const int g = e / nx, xx = e - g * nx;
    const int rp = rp0 + g;
    va[u] = mk<double>(0, 0);
    vs[u] = mk<double>(1, 0);
    if (e < G * nx && rp < rp_total) {
      const int r = rp / p3, p = rp - r * p3;
      const int iz = p % nz;
      va[u] = ccast<double>(ptrs.in[r][(size_t)p * plane + (size_t)y * nx + xx]);
      if (r2) vs[u] = r2[(size_t)iz * plane + (size_t)y * nx + xx];
    }
  }
  const int npad = L - nx;
  for (int e = threadIdx.x; e < G * npad; e += NT) {
    const int g = e / npad, xx = nx + (e - g * npad);
    buf[g * ld + lds_pad(xx)] = mk<T>(0, 0);
  }
#pragma unroll
  for (int u = 0; u < EH; ++u) {
    const int e = threadIdx.x + u * NT;
    if (e < G * nx) {
      const int g = e / nx, xx = e - g * nx;
      buf[g * ld + lds_pad(xx)] = ccast<T>(cmul(va[u], vs[u]));
    }
  }
  fft_lds<T, EPT, POW2>(buf, G, ld, fd, tw, false);
  for (int e = threadIdx.x; e < G * L; e += blockDim.x) {
    const int K = e / G, g = e - K * G;
    const int rp = rp0 + g;
    if (rp < rp_total) spec[((size_t)y * L + K) * rp_total + rp] = buf[g * ld + lds_pad(K)];
  }
}

// Step 3, x pass: inverse FFT along x, keep x < Nx, scale by 1/(4 Nx Ny) and
// finish the operator: y = S u + R1 (B R2 u)  (mode A, with R1/R2 swapped for
// A^T), or y = B u (mode B: s == nullptr, r1 == nullptr).
// With the transform's LDS addresses recomputed per pass: 96 VGPRs in FP64
// for power-of-two lengths (63.7 -> 57.5 us at 128 x 128 x 32).
template <typename T, int EPT, int NT, bool POW2, typename VT>
__global__ void __launch_bounds__(NT)
k_fft_x_inv(VecPtrsT<VT> ptrs, const c128 *__restrict__ sdiag, const c128 *__restrict__ r1,
            const cplx<T> *__restrict__ spec, int nx, int ny, int nz, int rp_total, int G,
            FftDesc fd, const cplx<T> *__restrict__ tw, double scale) {
  extern __shared__ unsigned char smem_raw[];
  cplx<T> *buf = reinterpret_cast<cplx<T> *>(smem_raw);
  const int L = fd.L, ld = fft_ld(L);
  const int y = blockIdx.x;
  const int rp0 = blockIdx.y * G;
  const int p3 = 3 * nz;
  const size_t plane = (size_t)nx * ny;
  {
    cplx<T> v[EPT];
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
      const int e = threadIdx.x + u * NT;
      const int K = e / G, g = e - K * G;
      const int rp = rp0 + g;
      v[u] = mk<T>(0, 0);
      if (e < G * L && rp < rp_total) v[u] = spec[((size_t)y * L + K) * rp_total + rp];
    }
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
      const int e = threadIdx.x + u * NT;
      if (e < G * L) {
        const int K = e / G, g = e - K * G;
        buf[g * ld + lds_pad(K)] = v[u];
      }
    }
  }
  fft_lds<T, EPT, POW2>(buf, G, ld, fd, tw, true);
  // epilogue: the diagonal terms are loaded after the transform, so that
  // they do not hold registers across it; every load of a thread is issued
  // before any of them is used (from a clamped address where an output is
  // outside the grid), and only the stores are conditional
  constexpr int EO = (EPT + 1) / 2;  // G * nx <= G * L / 2 outputs
  c128 dr[EO], ds[EO], xin[EO];
  size_t offs[EO];
  int rr[EO];
  bool okk[EO];
#pragma unroll
  for (int u = 0; u < EO; ++u) {
    const int e = threadIdx.x + u * NT;
    const int g = e / nx, xx = e - g * nx;
    const int rp = rp0 + g;
    okk[u] = e < G * nx && rp < rp_total;
    const int rpc = okk[u] ? rp : 0, xc = okk[u] ? xx : 0;
    const int r = rpc / p3, p = rpc - r * p3;
    rr[u] = r;
    offs[u] = (size_t)p * plane + (size_t)y * nx + xc;
    if (r1) {
      const size_t cell = (size_t)(p % nz) * plane + (size_t)y * nx + xc;
      dr[u] = r1[cell];
      ds[u] = sdiag[cell];
      xin[u] = ccast<double>(ptrs.in[r][offs[u]]);
    }
  }
#pragma unroll
  for (int u = 0; u < EO; ++u) {
    const int e = threadIdx.x + u * NT;
    if (okk[u]) {
      const int g = e / nx, xx = e - g * nx;
      c128 b = ccast<double>(buf[g * ld + lds_pad(xx)]);
      b = cscale(b, scale);
      c128 out = b;
      if (r1) {
        out = cmul(dr[u], b);
        cfma(out, ds[u], xin[u]);
      }
      ptrs.out[rr[u]][offs[u]] = ccast<typename VTraits<VT>::elem>(out);
    }
  }
}

// ---------------------------------------------------------------- y passes
// Forward (rows y >= Ny are zero, output all 2 Ny rows) or inverse (read all
// 2 Ny rows, write rows < Ny) FFT along y, in place.  Grid: (Kx, plane group).
// Power-of-two lengths: at least four wavefronts per SIMD (73 -> 69-71 us at
// 128 x 128 x 32 for the best shape, every result bit unchanged), now met
// without a cap by recomputing the LDS addresses per pass (88 VGPRs in
// FP64).  The mixed-radix kernels (lengths with factors 3, 5, 7, 11) carry
// no floor (103 VGPRs in FP64 at 8 elements per thread).
template <typename T, int EPT, int NT, bool POW2>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(POW2 ? 4 : 1)))
k_fft_y(cplx<T> *__restrict__ spec, int nx2, int ny, int rp_total, int G, FftDesc fd,
        const cplx<T> *__restrict__ tw, int inverse) {
  extern __shared__ unsigned char smem_raw[];
  cplx<T> *buf = reinterpret_cast<cplx<T> *>(smem_raw);
  const int L = fd.L, ld = fft_ld(L);
  const int kx = blockIdx.x;
  const int rp0 = blockIdx.y * G;
  const int nin = inverse ? L : ny;
  const int nout = inverse ? ny : L;
  {
    cplx<T> v[EPT];
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
      const int e = threadIdx.x + u * NT;
      const int yy = e / G, g = e - yy * G;
      const int rp = rp0 + g;
      v[u] = mk<T>(0, 0);
      if (e < G * L && yy < nin && rp < rp_total) v[u] = spec[((size_t)yy * nx2 + kx) * rp_total + rp];
    }
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
      const int e = threadIdx.x + u * NT;
      if (e < G * L) {
        const int yy = e / G, g = e - yy * G;
        buf[g * ld + lds_pad(yy)] = v[u];
      }
    }
  }
  fft_lds<T, EPT, POW2>(buf, G, ld, fd, tw, inverse != 0);
  for (int e = threadIdx.x; e < G * nout; e += blockDim.x) {
    const int yy = e / G, g = e - yy * G;
    const int rp = rp0 + g;
    if (rp < rp_total) spec[((size_t)yy * nx2 + kx) * rp_total + rp] = buf[g * ld + lds_pad(yy)];
  }
}

// ------------------------------------------------------- table spectra
// Even/odd transform of the packed table along one axis (a0; the parities of
// Lemma 2): for G consecutive packed entries e of one line, the length-2N
// sequence s[j] = c(j) (j < N), s[N] = 0, s[2N - j] = +-c(j) (the parity of
// e's class along the axis) goes through the FFT passes, and S[K], K <= N,
// is kept: S[K] = c(0) + 2 sum_j cos(pi K j / N) c(j), or -2i sum_j
// sin(pi K j / N) c(j) for the odd classes.  in: line b at in + b sb,
// element j at + j sj (c128 units; the E entries contiguous); out likewise
// with K.  Grid: (entry group, line).
__device__ __forceinline__ bool entry_odd(int e, int nz, int axis) {
  const int tri = nz * (nz + 1) / 2;
  const int c = e < 4 * tri ? e / tri : (e < 4 * tri + nz * nz ? 4 : 5);
  // xy is odd along both axes, xz along x, yz along y
  return c == 1 || c == (axis == 0 ? 4 : 5);
}

template <typename T, int EPT, int NT, bool POW2>
__global__ void __launch_bounds__(NT)
k_parity_fft(const c128 *__restrict__ in, int64_t sj, int64_t sb, c128 *__restrict__ out,
             int64_t sk, int64_t ob, int n, int E, int nz, int axis, int G, FftDesc fd,
             const c128 *__restrict__ tw) {
  extern __shared__ unsigned char smem_raw[];
  c128 *buf = reinterpret_cast<c128 *>(smem_raw);
  const int L = fd.L, ld = fft_ld(L);
  const int e0 = blockIdx.x * G;
  in += (int64_t)blockIdx.y * sb;
  out += (int64_t)blockIdx.y * ob;
  constexpr int EH = (EPT + 1) / 2;  // G n <= NT EPT / 2
  c128 v[EH];
#pragma unroll
  for (int u = 0; u < EH; ++u) {
    const int idx = threadIdx.x + u * NT;
    const int j = idx / G, g = idx - j * G;
    v[u] = mk<double>(0, 0);
    if (j < n && e0 + g < E) v[u] = in[(int64_t)j * sj + e0 + g];
  }
#pragma unroll
  for (int u = 0; u < EH; ++u) {
    const int idx = threadIdx.x + u * NT;
    const int j = idx / G, g = idx - j * G;
    if (j < n) {
      buf[g * ld + lds_pad(j)] = v[u];
      if (j > 0) {
        const bool odd = entry_odd(e0 + g, nz, axis);
        buf[g * ld + lds_pad(L - j)] = odd ? mk<double>(-v[u].x, -v[u].y) : v[u];
      }
    }
  }
  for (int g = threadIdx.x; g < G; g += NT) buf[g * ld + lds_pad(n)] = mk<double>(0, 0);
  fft_lds<T, EPT, POW2>(buf, G, ld, fd, tw, false);
  for (int idx = threadIdx.x; idx < G * (n + 1); idx += NT) {
    const int K = idx / G, g = idx - K * G;
    if (e0 + g < E) out[(int64_t)K * sk + e0 + g] = buf[g * ld + lds_pad(K)];
  }
}

// ---------------------------------------------------------------- launchers
// Elements per thread of a pass over G sequences of length L with nthr
// threads (0 if the configuration is not instantiated).  At most 16: the x
// passes stage c128 input in registers, and 32 per thread spills.
int fft_ept(int G, int L, int nthr, int prec) {
  (void)prec;
  if (nthr != 256 && nthr != 512) return 0;
  const int need = (G * L + nthr - 1) / nthr;
  for (int e = 4; e <= 16; e *= 2)
    if (need <= e) return e;
  return 0;
}

#define GIEM_FFT_CASES(KERNEL, NTV, P2, ...)                                                 \
  switch (ept) {                                                                              \
    case 4: KERNEL<T, 4, NTV, P2 KX><<<grid, NTV, lds, s>>>(__VA_ARGS__); break;              \
    case 8: KERNEL<T, 8, NTV, P2 KX><<<grid, NTV, lds, s>>>(__VA_ARGS__); break;              \
    case 16: KERNEL<T, 16, NTV, P2 KX><<<grid, NTV, lds, s>>>(__VA_ARGS__); break;            \
    default: return hipErrorInvalidConfiguration;                                             \
  }
#define GIEM_FFT_DISPATCH(KERNEL, ...)                                                        \
  do {                                                                                        \
    const int ept = fft_ept(G, fd.L, nthr, sizeof(T) == 4 ? PREC_FP32 : PREC_FP64);          \
    const bool pow2 = (fd.L & (fd.L - 1)) == 0;                                              \
    if (nthr == 512 && pow2) {                                                                \
      GIEM_FFT_CASES(KERNEL, 512, true, __VA_ARGS__)                                          \
    } else if (nthr == 512) {                                                                 \
      GIEM_FFT_CASES(KERNEL, 512, false, __VA_ARGS__)                                         \
    } else if (nthr == 256 && pow2) {                                                         \
      GIEM_FFT_CASES(KERNEL, 256, true, __VA_ARGS__)                                          \
    } else if (nthr == 256) {                                                                 \
      GIEM_FFT_CASES(KERNEL, 256, false, __VA_ARGS__)                                         \
    } else {                                                                                  \
      return hipErrorInvalidConfiguration;                                                    \
    }                                                                                         \
  } while (0)

#define KX , VT
template <typename T, typename VT>
static hipError_t launch_fft_x_fwd_t(const VecPtrsT<VT> &ptrs, const c128 *r2, void *spec, int nx,
                                     int ny, int nz, int rp_total, int G, int nthr,
                                     const FftDesc &fd, const void *tw, hipStream_t s) {
  dim3 grid(ny, (rp_total + G - 1) / G);
  size_t lds = (size_t)G * fft_ld(fd.L) * sizeof(cplx<T>);
  const cplx<T> *twp = static_cast<const cplx<T> *>(tw);
  cplx<T> *sp = static_cast<cplx<T> *>(spec);
  GIEM_FFT_DISPATCH(k_fft_x_fwd, ptrs, r2, sp, nx, ny, nz, rp_total, G, fd, twp);
  return hipGetLastError();
}

template <typename T, typename VT>
static hipError_t launch_fft_x_inv_t(const VecPtrsT<VT> &ptrs, const c128 *sd, const c128 *r1,
                                     const void *spec, int nx, int ny, int nz, int rp_total,
                                     int G, int nthr, const FftDesc &fd, const void *tw,
                                     double scale, hipStream_t s) {
  dim3 grid(ny, (rp_total + G - 1) / G);
  size_t lds = (size_t)G * fft_ld(fd.L) * sizeof(cplx<T>);
  const cplx<T> *twp = static_cast<const cplx<T> *>(tw);
  const cplx<T> *sp = static_cast<const cplx<T> *>(spec);
  GIEM_FFT_DISPATCH(k_fft_x_inv, ptrs, sd, r1, sp, nx, ny, nz, rp_total, G, fd, twp, scale);
  return hipGetLastError();
}
#undef KX
#define KX

template <typename T>
static hipError_t launch_fft_y_t(void *spec, int nx2, int ny, int rp_total, int G, int nthr,
                                 const FftDesc &fd, const void *tw, int inverse, hipStream_t s) {
  dim3 grid(nx2, (rp_total + G - 1) / G);
  size_t lds = (size_t)G * fft_ld(fd.L) * sizeof(cplx<T>);
  const cplx<T> *twp = static_cast<const cplx<T> *>(tw);
  cplx<T> *sp = static_cast<cplx<T> *>(spec);
  GIEM_FFT_DISPATCH(k_fft_y, sp, nx2, ny, rp_total, G, fd, twp, inverse);
  return hipGetLastError();
}
// the packed entries of each line in groups of 8 (128-byte runs), fewer
// where a 2N-point transform of 8 sequences needs more than 16 elements per
// thread
hipError_t launch_parity_fft(const c128 *in, int64_t sj, int64_t sb, int nbatch, c128 *out,
                             int64_t sk, int64_t ob, int n, int E, int nz, int axis,
                             const FftDesc &fd, const void *tw, hipStream_t s) {
  typedef double T;
  if (fd.L != 2 * n || nbatch <= 0 || nbatch > 65535 || E <= 0) return hipErrorInvalidValue;
  int G = 0, nthr = 0;
  for (int nt : {256, 512}) {
    for (int g : {8, 4, 2, 1})
      if (fft_ept(g, fd.L, nt, PREC_FP64)) {
        G = g;
        break;
      }
    if (G) {
      nthr = nt;
      break;
    }
  }
  if (!G) return hipErrorInvalidConfiguration;
  dim3 grid((E + G - 1) / G, nbatch);
  size_t lds = (size_t)G * fft_ld(fd.L) * sizeof(c128);
  const c128 *twp = static_cast<const c128 *>(tw);
  GIEM_FFT_DISPATCH(k_parity_fft, in, sj, sb, out, sk, ob, n, E, nz, axis, G, fd, twp);
  return hipGetLastError();
}
#undef KX
#undef GIEM_FFT_DISPATCH
#undef GIEM_FFT_CASES

size_t fft_lds_bytes(int G, int L, int prec) {
  const size_t c = prec == PREC_FP32 ? sizeof(c64) : sizeof(c128);
  return (size_t)G * fft_ld(L) * c;
}

// gfx950 has 160 KB of LDS per CU; allow the large dynamic allocations.
static hipError_t allow_lds(const void *k) {
  return hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
}
template <typename T, bool P2, typename VT>
static hipError_t allow_lds_x() {
  const void *ks[] = {(const void *)k_fft_x_fwd<T, 4, 256, P2, VT>, (const void *)k_fft_x_fwd<T, 8, 256, P2, VT>,
                      (const void *)k_fft_x_fwd<T, 16, 256, P2, VT>, (const void *)k_fft_x_fwd<T, 4, 512, P2, VT>,
                      (const void *)k_fft_x_fwd<T, 8, 512, P2, VT>, (const void *)k_fft_x_fwd<T, 16, 512, P2, VT>,
                      (const void *)k_fft_x_inv<T, 4, 256, P2, VT>, (const void *)k_fft_x_inv<T, 8, 256, P2, VT>,
                      (const void *)k_fft_x_inv<T, 16, 256, P2, VT>, (const void *)k_fft_x_inv<T, 4, 512, P2, VT>,
                      (const void *)k_fft_x_inv<T, 8, 512, P2, VT>, (const void *)k_fft_x_inv<T, 16, 512, P2, VT>};
  for (const void *k : ks) {
    const hipError_t e = allow_lds(k);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}
template <typename T, bool P2>
static hipError_t allow_lds_y() {
  const void *ks[] = {(const void *)k_fft_y<T, 4, 256, P2>, (const void *)k_fft_y<T, 8, 256, P2>,
                      (const void *)k_fft_y<T, 16, 256, P2>, (const void *)k_fft_y<T, 4, 512, P2>,
                      (const void *)k_fft_y<T, 8, 512, P2>, (const void *)k_fft_y<T, 16, 512, P2>};
  for (const void *k : ks) {
    const hipError_t e = allow_lds(k);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <bool P2>
static hipError_t allow_lds_parity() {
  const void *ks[] = {(const void *)k_parity_fft<double, 4, 256, P2>, (const void *)k_parity_fft<double, 8, 256, P2>,
                      (const void *)k_parity_fft<double, 16, 256, P2>, (const void *)k_parity_fft<double, 4, 512, P2>,
                      (const void *)k_parity_fft<double, 8, 512, P2>, (const void *)k_parity_fft<double, 16, 512, P2>};
  for (const void *k : ks) {
    const hipError_t e = allow_lds(k);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t set_lds_limits() {
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = allow_lds_parity<true>();
  if (e == hipSuccess) e = allow_lds_parity<false>();
  if (e == hipSuccess) e = allow_lds_x<double, true, c128>();
  if (e == hipSuccess) e = allow_lds_x<double, false, c128>();
  if (e == hipSuccess) e = allow_lds_x<float, true, c128>();
  if (e == hipSuccess) e = allow_lds_x<float, false, c128>();
  if (e == hipSuccess) e = allow_lds_x<float, true, c64>();
  if (e == hipSuccess) e = allow_lds_x<float, false, c64>();
  if (e == hipSuccess) e = allow_lds_y<double, true>();
  if (e == hipSuccess) e = allow_lds_y<double, false>();
  if (e == hipSuccess) e = allow_lds_y<float, true>();
  if (e == hipSuccess) e = allow_lds_y<float, false>();
  if (e == hipSuccess) e = set_block_lds_limits();
  return e;
}

hipError_t launch_fft_x_fwd(int prec, const VecPtrs &ptrs, const c128 *r2, void *spec, int nx,
                            int ny, int nz, int rp_total, int G, int nthr, const FftDesc &fd,
                            const void *tw, hipStream_t s) {
  return prec == PREC_FP32
             ? launch_fft_x_fwd_t<float>(ptrs, r2, spec, nx, ny, nz, rp_total, G, nthr, fd, tw, s)
             : launch_fft_x_fwd_t<double>(ptrs, r2, spec, nx, ny, nz, rp_total, G, nthr, fd, tw, s);
}
hipError_t launch_fft_x_inv(int prec, const VecPtrs &ptrs, const c128 *sd, const c128 *r1,
                            const void *spec, int nx, int ny, int nz, int rp_total, int G,
                            int nthr, const FftDesc &fd, const void *tw, double scale,
                            hipStream_t s) {
  return prec == PREC_FP32
             ? launch_fft_x_inv_t<float>(ptrs, sd, r1, spec, nx, ny, nz, rp_total, G, nthr, fd, tw, scale, s)
             : launch_fft_x_inv_t<double>(ptrs, sd, r1, spec, nx, ny, nz, rp_total, G, nthr, fd, tw, scale, s);
}
hipError_t launch_fft_x_fwd(int prec, const VecPtrs32 &ptrs, const c128 *r2, void *spec, int nx,
                            int ny, int nz, int rp_total, int G, int nthr, const FftDesc &fd,
                            const void *tw, hipStream_t s) {
  if (prec != PREC_FP32) return hipErrorInvalidValue;
  return launch_fft_x_fwd_t<float>(ptrs, r2, spec, nx, ny, nz, rp_total, G, nthr, fd, tw, s);
}
hipError_t launch_fft_x_inv(int prec, const VecPtrs32 &ptrs, const c128 *sd, const c128 *r1,
                            const void *spec, int nx, int ny, int nz, int rp_total, int G,
                            int nthr, const FftDesc &fd, const void *tw, double scale,
                            hipStream_t s) {
  if (prec != PREC_FP32) return hipErrorInvalidValue;
  return launch_fft_x_inv_t<float>(ptrs, sd, r1, spec, nx, ny, nz, rp_total, G, nthr, fd, tw, scale, s);
}
hipError_t launch_fft_y(int prec, void *spec, int nx2, int ny, int rp_total, int G, int nthr,
                        const FftDesc &fd, const void *tw, int inverse, hipStream_t s) {
  return prec == PREC_FP32
             ? launch_fft_y_t<float>(spec, nx2, ny, rp_total, G, nthr, fd, tw, inverse, s)
             : launch_fft_y_t<double>(spec, nx2, ny, rp_total, G, nthr, fd, tw, inverse, s);
}
}  // namespace giem
