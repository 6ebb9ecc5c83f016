// Set-up kernels: spectra of the packed table (Sect. 3.3: the stored
// quantities are the discrete Fourier transforms Q~ of the blocks Q(i, j)),
// the diagonals of A = S + R1 B R2 (Sect. 3.1) and the plane-wave right-hand
// side U^0 = sqrt(Re sb) <E^N> (Sect. 2.2).
#include "kernels.h"

namespace giem {

// Class of a packed entry e (order xx, xy, yy, zz upper triangles, xz, yz
// full blocks) and its lateral parities from Lemma 2.
__device__ __forceinline__ void class_parity(int e, int nz, bool &odd_x, bool &odd_y) {
  const int tri = nz * (nz + 1) / 2;
  int c;
  if (e < 4 * tri) c = e / tri;
  else if (e < 4 * tri + nz * nz) c = 4;
  else c = 5;
  odd_x = (c == 1 || c == 4);  // xy, xz
  odd_y = (c == 1 || c == 5);  // xy, yz
}

// The zero-padded circulant of length 2N built from c(j), |j| < N, with
// c(-j) = +-c(j) has the transform
//   even:  c(0) + 2 sum_{j>=1} c(j) cos(pi K j / N)
//   odd:       -2i sum_{j>=1} c(j) sin(pi K j / N)
// for 0 <= K <= N; the other half follows from the same parity.
__device__ __forceinline__ c128 parity_term(c128 v, int j, int K, int n, bool odd,
                                            const c128 *__restrict__ cs) {
  const c128 t = cs[(int)(((long long)K * j) % (2 * n))];  // (cos, sin)(pi K j / n)
  if (!odd) {
    const double f = (j == 0) ? 1.0 : 2.0 * t.x;
    return mk<double>(v.x * f, v.y * f);
  }
  if (j == 0) return mk<double>(0.0, 0.0);
  const double s2 = 2.0 * t.y;
  return mk<double>(s2 * v.y, -s2 * v.x);  // (-2 i sin) v
}

// tmp[i][K][e] = sum_j term_x(K, j) spatial[i][j][e],  0 <= K <= Nx
__global__ void __launch_bounds__(256)
k_spectral_x(const c128 *__restrict__ spatial, c128 *__restrict__ tmp, const c128 *__restrict__ cs,
             int nx, int ny, int nz) {
  const int E = 2 * nz * (2 * nz + 1);
  const int K = blockIdx.x, i = blockIdx.y;
  for (int e = threadIdx.x + blockIdx.z * blockDim.x; e < E; e += blockDim.x * gridDim.z) {
    bool ox, oy;
    class_parity(e, nz, ox, oy);
    c128 acc = mk<double>(0, 0);
    for (int j = 0; j < nx; ++j) {
      const c128 v = spatial[((size_t)i * nx + j) * E + e];
      acc = cadd(acc, parity_term(v, j, K, nx, ox, cs));
    }
    tmp[((size_t)i * (nx + 1) + K) * E + e] = acc;
  }
}

// spectral[Ky][K][e] = sum_i term_y(Ky, i) tmp[i][K][e],  0 <= Ky <= Ny
__global__ void __launch_bounds__(256)
k_spectral_y(const c128 *__restrict__ tmp, c128 *__restrict__ spectral, const c128 *__restrict__ cs,
             int nx, int ny, int nz) {
  const int E = 2 * nz * (2 * nz + 1);
  const int K = blockIdx.x, ky = blockIdx.y;
  for (int e = threadIdx.x + blockIdx.z * blockDim.x; e < E; e += blockDim.x * gridDim.z) {
    bool ox, oy;
    class_parity(e, nz, ox, oy);
    c128 acc = mk<double>(0, 0);
    for (int i = 0; i < ny; ++i) {
      const c128 v = tmp[((size_t)i * (nx + 1) + K) * E + e];
      acc = cadd(acc, parity_term(v, i, ky, ny, oy, cs));
    }
    spectral[((size_t)ky * (nx + 1) + K) * E + e] = acc;
  }
}

hipError_t launch_spectral_x(const c128 *spatial, c128 *tmp, const c128 *cs_x, int nx, int ny,
                             int nz, hipStream_t s) {
  const int E = 2 * nz * (2 * nz + 1);
  dim3 grid(nx + 1, ny, (E + 255) / 256);
  k_spectral_x<<<grid, 256, 0, s>>>(spatial, tmp, cs_x, nx, ny, nz);
  return hipGetLastError();
}

hipError_t launch_spectral_y(const c128 *tmp, c128 *spectral, const c128 *cs_y, int nx, int ny,
                             int nz, hipStream_t s) {
  const int E = 2 * nz * (2 * nz + 1);
  dim3 grid(nx + 1, ny + 1, (E + 255) / 256);
  k_spectral_y<<<grid, 256, 0, s>>>(tmp, spectral, cs_y, nx, ny, nz);
  return hipGetLastError();
}

__global__ void k_to_c64(const c128 *__restrict__ src, c64 *__restrict__ dst, size_t n) {
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n;
       k += (size_t)gridDim.x * blockDim.x)
    dst[k] = ccast<float>(src[k]);
}

hipError_t launch_to_c64(const c128 *src, c64 *dst, size_t n, hipStream_t s) {
  k_to_c64<<<2048, 256, 0, s>>>(src, dst, n);
  return hipGetLastError();
}

// Per cell: gamma = (sa - sb)/(sa + conj sb), S = 1 - gamma,
// R1 = -2 sqrt(Re sb)/V, R2 = sqrt(Re sb) gamma, a = (sa + conj sb)/(2 sqrt(Re sb)).
__global__ void k_diagonals(const c128 *__restrict__ sigma_a, const c128 *__restrict__ sb_lev,
                            const double *__restrict__ vol_lev, int plane, int nz,
                            c128 *__restrict__ S, c128 *__restrict__ R1, c128 *__restrict__ R2,
                            c128 *__restrict__ a) {
  const size_t ncell = (size_t)plane * nz;
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < ncell;
       k += (size_t)gridDim.x * blockDim.x) {
    const int iz = (int)(k / plane);
    const c128 sb = sb_lev[iz];
    const c128 sa = sigma_a[k];
    const double sr = sqrt(sb.x);
    const c128 num = mk<double>(sa.x - sb.x, sa.y - sb.y);
    const c128 den = mk<double>(sa.x + sb.x, sa.y - sb.y);
    const double dd = den.x * den.x + den.y * den.y;
    const c128 g = mk<double>((num.x * den.x + num.y * den.y) / dd,
                              (num.y * den.x - num.x * den.y) / dd);
    S[k] = mk<double>(1.0 - g.x, -g.y);
    R1[k] = mk<double>(-2.0 * sr / vol_lev[iz], 0.0);
    R2[k] = mk<double>(sr * g.x, sr * g.y);
    a[k] = mk<double>(den.x / (2.0 * sr), den.y / (2.0 * sr));
  }
}

hipError_t launch_diagonals(const c128 *sigma_a, const c128 *sb_lev, const double *vol_lev,
                            int nx, int ny, int nz, c128 *S, c128 *R1, c128 *R2, c128 *a,
                            int * /*unused*/, hipStream_t s) {
  k_diagonals<<<1024, 256, 0, s>>>(sigma_a, sb_lev, vol_lev, nx * ny, nz, S, R1, R2, a);
  return hipGetLastError();
}

// U^0 for a plane wave polarised along x (pol 0) or y (pol 1).
__global__ void k_plane_wave(const c128 *__restrict__ en_lev, const double *__restrict__ sroot,
                             int plane, int nz, int pol, c128 *__restrict__ out) {
  const size_t n = (size_t)3 * nz * plane;
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n;
       k += (size_t)gridDim.x * blockDim.x) {
    const int comp = (int)(k / ((size_t)nz * plane));
    const int iz = (int)((k / plane) % nz);
    c128 v = mk<double>(0, 0);
    if (comp == pol) v = cscale(en_lev[iz], sroot[iz]);
    out[k] = v;
  }
}

hipError_t launch_plane_wave_rhs(const c128 *en_lev, const double *sroot_lev, int nx, int ny,
                                 int nz, int pol, c128 *out, hipStream_t s) {
  k_plane_wave<<<1024, 256, 0, s>>>(en_lev, sroot_lev, nx * ny, nz, pol, out);
  return hipGetLastError();
}

}  // namespace giem

namespace giem {

// Sensitivity of J = Re sum g . E to log sigma_a of each cell (real sigma).
// With U = a E, A U = U0, lambda = A^{-T} (g / a), w = B (R1 lambda):
//   dJ/dsigma = sum_alpha [(lambda - s w) U dgamma/dsigma - g U / (2 s a^2)],
//   dgamma/dsigma = 2 Re sb / (sigma + conj sb)^2,   da/dsigma = 1 / (2 s);
// grad += Re(sigma dJ/dsigma).
__global__ void k_adjoint_grad(const c128 *__restrict__ sigma_a, const c128 *__restrict__ sb_lev,
                               const c128 *__restrict__ acell, const c128 *__restrict__ g,
                               const c128 *__restrict__ E, const c128 *__restrict__ lam,
                               const c128 *__restrict__ w, int nrhs, int plane, int nz,
                               double *__restrict__ grad) {
  const size_t nc = (size_t)plane * nz;
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < nc;
       k += (size_t)gridDim.x * blockDim.x) {
    const int iz = (int)(k / plane);
    const c128 sb = sb_lev[iz];
    const double s = sqrt(sb.x);
    const c128 sa = sigma_a[k];
    const c128 den = mk<double>(sa.x + sb.x, sa.y - sb.y);  // sigma + conj sb
    const c128 den2 = cmul(den, den);
    const double dd = den2.x * den2.x + den2.y * den2.y;
    const c128 dg = mk<double>(2.0 * sb.x * den2.x / dd, -2.0 * sb.x * den2.y / dd);
    const c128 a = acell[k];
    const c128 a2 = cmul(a, a);
    const double ad = a2.x * a2.x + a2.y * a2.y;
    const c128 inva2 = mk<double>(a2.x / ad, -a2.y / ad);
    c128 acc = mk<double>(0, 0);
    for (int r = 0; r < nrhs; ++r) {
      for (int c = 0; c < 3; ++c) {
        const size_t idx = ((size_t)r * 3 + c) * nc + k;
        const c128 U = cmul(a, E[idx]);
        const c128 lw = mk<double>(lam[idx].x - s * w[idx].x, lam[idx].y - s * w[idx].y);
        cfma(acc, cmul(lw, U), dg);
        const c128 gu = cmul(g[idx], U);
        const c128 t2 = cscale(cmul(gu, inva2), -0.5 / s);
        acc = cadd(acc, t2);
      }
    }
    const c128 sd = cmul(sa, acc);
    grad[k] += sd.x;
  }
}

hipError_t launch_adjoint_grad(const c128 *sigma_a, const c128 *sb_lev, const c128 *acell,
                               const c128 *g, const c128 *E, const c128 *lam, const c128 *w,
                               int nrhs, int nx, int ny, int nz, double *grad, hipStream_t s) {
  k_adjoint_grad<<<1024, 256, 0, s>>>(sigma_a, sb_lev, acell, g, E, lam, w, nrhs, nx * ny, nz, grad);
  return hipGetLastError();
}

}  // namespace giem
