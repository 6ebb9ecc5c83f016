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
__global__ void __launch_bounds__(256)
k_fft_x_fwd(VecPtrs ptrs, const c128 *__restrict__ r2, cplx<T> *__restrict__ spec, int nx,
            int ny, int nz, int rp_total, int G, FftDesc fd, const cplx<T> *__restrict__ tw) {
  extern __shared__ unsigned char smem_raw[];
  cplx<T> *buf = reinterpret_cast<cplx<T> *>(smem_raw);
  const int L = fd.L, ld = L + 1;
  const int y = blockIdx.x;
  const int rp0 = blockIdx.y * G;
  const int p3 = 3 * nz;
  const size_t plane = (size_t)nx * ny;
  for (int e = threadIdx.x; e < G * L; e += blockDim.x) {
    const int g = e / L, xx = e - g * L;
    const int rp = rp0 + g;
    cplx<T> v = mk<T>(0, 0);
    if (xx < nx && rp < rp_total) {
      const int r = rp / p3, p = rp - r * p3;
      const int iz = p % nz;
      c128 a = ptrs.in[r][(size_t)p * plane + (size_t)y * nx + xx];
      if (r2) a = cmul(a, r2[(size_t)iz * plane + (size_t)y * nx + xx]);
      v = ccast<T>(a);
    }
    buf[g * ld + xx] = v;
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
__global__ void __launch_bounds__(256)
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
  for (int e = threadIdx.x; e < G * L; e += blockDim.x) {
    const int K = e / G, g = e - K * G;
    const int rp = rp0 + g;
    buf[g * ld + K] = (rp < rp_total) ? spec[((size_t)y * L + K) * rp_total + rp] : mk<T>(0, 0);
  }
  fft_lds<T, EPT>(buf, G, ld, fd, tw, true);
  for (int e = threadIdx.x; e < G * nx; e += blockDim.x) {
    const int g = e / nx, xx = e - g * nx;
    const int rp = rp0 + g;
    if (rp < rp_total) {
      const int r = rp / p3, p = rp - r * p3;
      const int iz = p % nz;
      const size_t off = (size_t)p * plane + (size_t)y * nx + xx;
      c128 b = ccast<double>(buf[g * ld + xx]);
      b = cscale(b, scale);
      c128 out;
      if (r1) {
        const size_t cell = (size_t)iz * plane + (size_t)y * nx + xx;
        out = cmul(r1[cell], b);
        cfma(out, sdiag[cell], ptrs.in[r][off]);
      } else {
        out = b;
      }
      ptrs.out[r][off] = out;
    }
  }
}

// ---------------------------------------------------------------- y passes
// Forward (rows y >= Ny are zero, output all 2 Ny rows) or inverse (read all
// 2 Ny rows, write rows < Ny) FFT along y, in place.  Grid: (Kx, plane group).
template <typename T, int EPT>
__global__ void __launch_bounds__(256)
k_fft_y(cplx<T> *__restrict__ spec, int nx2, int ny, int rp_total, int G, FftDesc fd,
        const cplx<T> *__restrict__ tw, int inverse) {
  extern __shared__ unsigned char smem_raw[];
  cplx<T> *buf = reinterpret_cast<cplx<T> *>(smem_raw);
  const int L = fd.L, ld = L + 1;
  const int kx = blockIdx.x;
  const int rp0 = blockIdx.y * G;
  const int nin = inverse ? L : ny;
  const int nout = inverse ? ny : L;
  for (int e = threadIdx.x; e < G * L; e += blockDim.x) {
    const int yy = e / G, g = e - yy * G;
    const int rp = rp0 + g;
    cplx<T> v = mk<T>(0, 0);
    if (yy < nin && rp < rp_total) v = spec[((size_t)yy * nx2 + kx) * rp_total + rp];
    buf[g * ld + yy] = v;
  }
  fft_lds<T, EPT>(buf, G, ld, fd, tw, inverse != 0);
  for (int e = threadIdx.x; e < G * nout; e += blockDim.x) {
    const int yy = e / G, g = e - yy * G;
    const int rp = rp0 + g;
    if (rp < rp_total) spec[((size_t)yy * nx2 + kx) * rp_total + rp] = buf[g * ld + yy];
  }
}

// ---------------------------------------------------------------- block product
// Step 2: for every frequency point K of the 2Nx x 2Ny grid,
//   Y^(K) = Q~(K) X^(K),   Q~(K) the 3Nz x 3Nz matrix of 3 x 3 Nz-blocks.
// Q~ is stored once per representative (Kx, Ky), 0 <= Kx <= Nx, 0 <= Ky <= Ny
// (Sect. 3.3: the transform keeps the parities of Lemma 2).  A mirrored point
// (2Nx - Kx or 2Ny - Ky) uses Q~_ab times t_a t_b, t = (-1, 1, 1) for an x
// mirror and (1, -1, 1) for a y mirror, i.e. Y = T Q~ T X: the sign flips are
// applied to the loaded vectors and to the results, and one read of the
// packed block serves the up to four mirror points and all R right-hand sides.
// Lemma 1 gives the blocks not stored: yx = xy, zx = -xz^T, zy = -yz^T, and
// xx, xy, yy, zz are read from their upper triangles.
//
// One workgroup per representative point.  LDS: the packed block (E complex)
// and the V = mirrors x R input vectors.  Thread (row, vector group) owns one
// output row of 3Nz for VPT vectors.
template <typename T, int VPT>
__global__ void __launch_bounds__(1024)
k_block(const cplx<T> *__restrict__ tab, cplx<T> *__restrict__ spec, int nx, int ny, int nz,
        int R) {
  extern __shared__ unsigned char smem_raw[];
  const int E = 2 * nz * (2 * nz + 1);
  const int p3 = 3 * nz;
  cplx<T> *qs = reinterpret_cast<cplx<T> *>(smem_raw);
  cplx<T> *xs = qs + E;  // [V][3nz]
  const int rep = blockIdx.x;
  const int kxr = rep % (nx + 1), kyr = rep / (nx + 1);
  const int nx2 = 2 * nx, ny2 = 2 * ny;
  // mirror points of this representative
  int mkx[4], mky[4], mtx[4], mty[4];
  int nm = 0;
  const bool mx = (kxr != 0 && kxr != nx), my = (kyr != 0 && kyr != ny);
  mkx[nm] = kxr; mky[nm] = kyr; mtx[nm] = 1; mty[nm] = 1; ++nm;
  if (mx) { mkx[nm] = nx2 - kxr; mky[nm] = kyr; mtx[nm] = -1; mty[nm] = 1; ++nm; }
  if (my) { mkx[nm] = kxr; mky[nm] = ny2 - kyr; mtx[nm] = 1; mty[nm] = -1; ++nm; }
  if (mx && my) { mkx[nm] = nx2 - kxr; mky[nm] = ny2 - kyr; mtx[nm] = -1; mty[nm] = -1; ++nm; }
  const int V = nm * R;

  // stage the packed block and the (sign-flipped) input vectors
  const cplx<T> *tsrc = tab + (size_t)rep * E;
  for (int e = threadIdx.x; e < E; e += blockDim.x) qs[e] = tsrc[e];
  for (int e = threadIdx.x; e < V * p3; e += blockDim.x) {
    const int v = e / p3, p = e - v * p3;
    const int m = v / R, r = v - m * R;
    cplx<T> val = spec[(((size_t)mky[m] * nx2 + mkx[m]) * R + r) * p3 + p];
    const int a = p / nz;
    if ((a == 0 && mtx[m] < 0) || (a == 1 && mty[m] < 0)) val = mk<T>(-val.x, -val.y);
    xs[e] = val;
  }
  __syncthreads();

  const int row = threadIdx.x % p3;
  const int vg = threadIdx.x / p3;
  const int v0 = vg * VPT;
  if (v0 < V) {
    const int a = row / nz, iz = row - a * nz;
    const int tri = nz * (nz + 1) / 2;
    const int o_xx = 0, o_xy = tri, o_yy = 2 * tri, o_zz = 3 * tri;
    const int o_xz = 4 * tri, o_yz = 4 * tri + nz * nz;
    cplx<T> acc[VPT];
#pragma unroll
    for (int k = 0; k < VPT; ++k) acc[k] = mk<T>(0, 0);
    const int nv = min(VPT, V - v0);
    // symmetric block (upper triangle) row iz times X_b
    auto sym_row = [&](int off, int b) {
      const cplx<T> *xb = xs + (size_t)v0 * p3 + b * nz;
      // jz < iz: element (jz, iz) at rowstart(jz) + iz - jz
      int idx = iz;  // rowstart(0) + iz
      for (int jz = 0; jz < iz; ++jz) {
        const cplx<T> q = qs[off + idx];
#pragma unroll
        for (int k = 0; k < VPT; ++k)
          if (k < nv) cfma(acc[k], q, xb[k * p3 + jz]);
        idx += nz - jz - 1;
      }
      // jz >= iz: element (iz, jz) at rowstart(iz) + jz - iz
      const int rs = iz * nz - (iz * (iz - 1)) / 2;
      for (int jz = iz; jz < nz; ++jz) {
        const cplx<T> q = qs[off + rs + jz - iz];
#pragma unroll
        for (int k = 0; k < VPT; ++k)
          if (k < nv) cfma(acc[k], q, xb[k * p3 + jz]);
      }
    };
    // full block row iz times X_b
    auto full_row = [&](int off, int b) {
      const cplx<T> *xb = xs + (size_t)v0 * p3 + b * nz;
      const cplx<T> *qr = qs + off + iz * nz;
      for (int jz = 0; jz < nz; ++jz) {
        const cplx<T> q = qr[jz];
#pragma unroll
        for (int k = 0; k < VPT; ++k)
          if (k < nv) cfma(acc[k], q, xb[k * p3 + jz]);
      }
    };
    // minus transposed full block: row iz of -F^T is -column iz of F
    auto negcol = [&](int off, int b) {
      const cplx<T> *xb = xs + (size_t)v0 * p3 + b * nz;
      for (int jz = 0; jz < nz; ++jz) {
        const cplx<T> q = qs[off + jz * nz + iz];
        const cplx<T> nq = mk<T>(-q.x, -q.y);
#pragma unroll
        for (int k = 0; k < VPT; ++k)
          if (k < nv) cfma(acc[k], nq, xb[k * p3 + jz]);
      }
    };
    if (a == 0) {
      sym_row(o_xx, 0);
      sym_row(o_xy, 1);
      full_row(o_xz, 2);
    } else if (a == 1) {
      sym_row(o_xy, 0);
      sym_row(o_yy, 1);
      full_row(o_yz, 2);
    } else {
      negcol(o_xz, 0);
      negcol(o_yz, 1);
      sym_row(o_zz, 2);
    }
#pragma unroll
    for (int k = 0; k < VPT; ++k) {
      if (k < nv) {
        const int v = v0 + k;
        const int m = v / R, r = v - m * R;
        cplx<T> o = acc[k];
        if ((a == 0 && mtx[m] < 0) || (a == 1 && mty[m] < 0)) o = mk<T>(-o.x, -o.y);
        spec[(((size_t)mky[m] * nx2 + mkx[m]) * R + r) * p3 + row] = o;
      }
    }
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

template <typename T>
static hipError_t launch_block_t(const void *tab, void *spec, int nx, int ny, int nz, int R,
                                 hipStream_t s) {
  constexpr int VPT = 4;
  const int E = 2 * nz * (2 * nz + 1);
  const int p3 = 3 * nz;
  const int vg = (4 * R + VPT - 1) / VPT;
  int nthr = p3 * vg;
  nthr = ((nthr + 63) / 64) * 64;
  size_t lds = ((size_t)E + (size_t)4 * R * p3) * sizeof(cplx<T>);
  dim3 grid((nx + 1) * (ny + 1));
  k_block<T, VPT><<<grid, nthr, lds, s>>>(static_cast<const cplx<T> *>(tab),
                                          static_cast<cplx<T> *>(spec), nx, ny, nz, R);
  return hipGetLastError();
}

int block_threads(int nz, int R) {
  const int vg = (4 * R + 3) / 4;
  int nthr = 3 * nz * vg;
  return ((nthr + 63) / 64) * 64;
}
size_t block_lds_bytes(int nz, int R, int prec) {
  const size_t c = prec == PREC_FP32 ? sizeof(c64) : sizeof(c128);
  return ((size_t)2 * nz * (2 * nz + 1) + (size_t)4 * R * 3 * nz) * c;
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
  GIEM_SET((k_block<double, 4>));
  GIEM_SET((k_block<float, 4>));
  GIEM_SET((k_fft_x_fwd<double, 4>)); GIEM_SET((k_fft_x_fwd<double, 8>)); GIEM_SET((k_fft_x_fwd<double, 16>)); GIEM_SET((k_fft_x_fwd<double, 32>));
  GIEM_SET((k_fft_x_fwd<float, 4>)); GIEM_SET((k_fft_x_fwd<float, 8>)); GIEM_SET((k_fft_x_fwd<float, 16>)); GIEM_SET((k_fft_x_fwd<float, 32>));
  GIEM_SET((k_fft_x_inv<double, 4>)); GIEM_SET((k_fft_x_inv<double, 8>)); GIEM_SET((k_fft_x_inv<double, 16>)); GIEM_SET((k_fft_x_inv<double, 32>));
  GIEM_SET((k_fft_x_inv<float, 4>)); GIEM_SET((k_fft_x_inv<float, 8>)); GIEM_SET((k_fft_x_inv<float, 16>)); GIEM_SET((k_fft_x_inv<float, 32>));
  GIEM_SET((k_fft_y<double, 4>)); GIEM_SET((k_fft_y<double, 8>)); GIEM_SET((k_fft_y<double, 16>)); GIEM_SET((k_fft_y<double, 32>));
  GIEM_SET((k_fft_y<float, 4>)); GIEM_SET((k_fft_y<float, 8>)); GIEM_SET((k_fft_y<float, 16>)); GIEM_SET((k_fft_y<float, 32>));
#undef GIEM_SET
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
hipError_t launch_block(int prec, const void *tab, void *spec, int nx, int ny, int nz, int R,
                        hipStream_t s) {
  return prec == PREC_FP32 ? launch_block_t<float>(tab, spec, nx, ny, nz, R, s)
                           : launch_block_t<double>(tab, spec, nx, ny, nz, R, s);
}

}  // namespace giem
