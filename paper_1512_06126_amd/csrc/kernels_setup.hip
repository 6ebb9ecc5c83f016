// Set-up kernels: the complex64 copy of the spectra of the packed table
// (the spectra themselves come from the FFT passes, kernels_apply.hip), the
// diagonals of A = S + R1 B R2 (Sect. 3.1), the plane-wave right-hand
// side U^0 = sqrt(Re sb) <E^N> (Sect. 2.2) and the per-cell gradient of a
// misfit from the forward and adjoint fields.
#include "kernels.h"

namespace giem {

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
