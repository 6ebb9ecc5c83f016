// Set-up kernels: spectra of the packed table (Sect. 3.3: the stored
// quantities are the discrete Fourier transforms Q~ of the blocks Q(i, j)),
// the diagonals of A = S + R1 B R2 (Sect. 3.1) and the plane-wave right-hand
// side U^0 = sqrt(Re sb) <E^N> (Sect. 2.2).
#include "kernels.h"

namespace giem {

// The zero-padded circulant of length 2N built from c(j), |j| < N, with
// c(-j) = +-c(j) has the transform
//   even:  c(0) + 2 sum_{j>=1} c(j) cos(pi K j / N)
//   odd:       -2i sum_{j>=1} c(j) sin(pi K j / N)
// for 0 <= K <= N (the other half follows from the same parity; Lemma 2
// gives each class of the packed entries its parity in x and y).  Along one
// axis this is a real (N + 1) x N matrix applied to every complex entry, so
// each pass is a batch of FP64 MFMA products over the entries of one parity.

typedef double d4 __attribute__((ext_vector_type(4)));

// T[j][K] = 1 or 0 (j = 0) and 2 cos or 2 sin (pi K j / N) (j >= 1): the even
// matrix at T, the odd one at T + N (N + 1)
__global__ void k_parity_matrices(const c128 *__restrict__ cs, int n, double *__restrict__ T) {
  const int np = n + 1;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < n * np;
       idx += gridDim.x * blockDim.x) {
    const int j = idx / np, K = idx % np;
    const c128 t = cs[(int)(((long long)K * j) % (2 * n))];  // (cos, sin)(pi K j / n)
    T[idx] = (j == 0) ? 1.0 : 2.0 * t.x;
    T[(size_t)n * np + idx] = (j == 0) ? 0.0 : 2.0 * t.y;
  }
}

// C[b][K][c] = sum_j T[j][K] B'[b][j][c] for K < m, j < k and the n doubles
// c of a run of complex entries, with B' = B (even) or, for the odd
// transform, B times -i: (x, y) -> (y, -x), i.e. column c reads column c ^ 1,
// negated for the imaginary parts.  Workgroup: 4 waves, 64 x 64 outputs of
// one batch entry b; wave w owns rows 32 (w >> 1), columns 32 (w & 1) as 2 x 2
// 16x16x4 MFMA tiles.  The row tiles of a column panel are consecutive
// workgroups, so the panel is read from HBM about once.
template <bool ROT>
__global__ __launch_bounds__(256) void k_parity_gemm(const double *__restrict__ T, int ldt,
                                                     const double *__restrict__ B, int64_t ldb,
                                                     int64_t sb, double *__restrict__ C,
                                                     int64_t ldc, int64_t sc, int m, int n, int k) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int m0 = blockIdx.x * 64 + (w >> 1) * 32;
  const int n0 = blockIdx.y * 64 + (w & 1) * 32;
  B += (int64_t)blockIdx.z * sb;
  C += (int64_t)blockIdx.z * sc;
  const int li = lane & 15, lk = lane >> 4;
  d4 acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
  const int ra0 = m0 + li, ra1 = m0 + 16 + li;
  const int cb0 = n0 + li, cb1 = n0 + 16 + li;
  const bool va0 = ra0 < m, va1 = ra1 < m, vb0 = cb0 < n, vb1 = cb1 < n;
  // n is even, so c ^ 1 < n whenever c < n
  const int sb0 = ROT ? (cb0 ^ 1) : cb0, sb1 = ROT ? (cb1 ^ 1) : cb1;
  const double g0 = (ROT && (cb0 & 1)) ? -1.0 : 1.0, g1 = (ROT && (cb1 & 1)) ? -1.0 : 1.0;
  for (int k0 = 0; k0 < k; k0 += 4) {
    const int kk = k0 + lk;
    const bool vk = kk < k;
    const double *ar = T + (int64_t)kk * ldt;
    const double *br = B + (int64_t)kk * ldb;
    const double a0 = (vk && va0) ? ar[ra0] : 0.0;
    const double a1 = (vk && va1) ? ar[ra1] : 0.0;
    const double b0 = (vk && vb0) ? g0 * br[sb0] : 0.0;
    const double b1 = (vk && vb1) ? g1 * br[sb1] : 0.0;
    acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
    acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
    acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
    acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
  }
  // D[(lane >> 4) + 4 q][lane & 15] in register q
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      const int col = n0 + 16 * b + li;
      if (col >= n) continue;
      for (int q = 0; q < 4; ++q) {
        const int row = m0 + 16 * a + lk + 4 * q;
        if (row < m) C[(int64_t)row * ldc + col] = acc[a][b][q];
      }
    }
}

// One pass along the x or y axis (length n) over the runs of packed entries
// with the same parity along it.  in/out: row
// j (K) of batch entry b at in + b sb + j ldb (out + b sc + K ldc), in c128
// units; E entries per row.
hipError_t parity_pass(const c128 *in, int64_t ldb, int64_t sb, c128 *out, int64_t ldc, int64_t sc,
                       int nbatch, const double *T, int n, int nz, bool x_axis, hipStream_t s) {
  const int tri = nz * (nz + 1) / 2, nz2 = nz * nz;
  // class runs: xx [0, tri), xy [tri, 2 tri), yy and zz [2 tri, 4 tri),
  // xz [4 tri, 4 tri + nz2), yz [4 tri + nz2, E); xy is odd along both axes,
  // xz only along x, yz only along y
  const int lo[4] = {0, tri, 2 * tri, 4 * tri};
  const int hi[4] = {tri, 2 * tri, 4 * tri, 4 * tri + 2 * nz2};
  if (nbatch <= 0 || nbatch > 65535) return hipErrorInvalidValue;
  const int np = n + 1;
  const double *Te = T, *To = T + (size_t)n * np;
  auto run = [&](int a, int b, bool odd) -> hipError_t {
    if (b <= a) return hipSuccess;
    const int nd = 2 * (b - a);
    const dim3 grid((np + 63) / 64, (nd + 63) / 64, nbatch);
    const double *Bp = reinterpret_cast<const double *>(in + a);
    double *Cp = reinterpret_cast<double *>(out + a);
    if (odd)
      hipLaunchKernelGGL(k_parity_gemm<true>, grid, dim3(256), 0, s, To, np, Bp, 2 * ldb, 2 * sb, Cp,
                         2 * ldc, 2 * sc, np, nd, n);
    else
      hipLaunchKernelGGL(k_parity_gemm<false>, grid, dim3(256), 0, s, Te, np, Bp, 2 * ldb, 2 * sb,
                         Cp, 2 * ldc, 2 * sc, np, nd, n);
    return hipGetLastError();
  };
  hipError_t e = hipSuccess;
  // xx, xy, yy + zz
  for (int r = 0; r < 3 && e == hipSuccess; ++r) e = run(lo[r], hi[r], r == 1);
  // xz (odd along x) and yz (odd along y)
  if (e == hipSuccess) e = run(lo[3], lo[3] + nz2, x_axis);
  if (e == hipSuccess) e = run(lo[3] + nz2, hi[3], !x_axis);
  return e;
}

hipError_t launch_parity_matrices(const c128 *cs, int n, double *T, hipStream_t s) {
  hipLaunchKernelGGL(k_parity_matrices, dim3((n * (n + 1) + 255) / 256), dim3(256), 0, s, cs, n, T);
  return hipGetLastError();
}

// tmp[i][K][e] = sum_j term_x(K, j) spatial[i][j][e],  0 <= K <= Nx
hipError_t launch_spectral_x(const c128 *spatial, c128 *tmp, const double *Tx, int nx, int ny,
                             int nz, hipStream_t s) {
  const int64_t E = 2 * nz * (2 * nz + 1);
  return parity_pass(spatial, E, (int64_t)nx * E, tmp, E, (int64_t)(nx + 1) * E, ny, Tx, nx, nz,
                     true, s);
}

// spectral[Ky][K][e] = sum_i term_y(Ky, i) tmp[i][K][e],  0 <= Ky <= Ny
hipError_t launch_spectral_y(const c128 *tmp, c128 *spectral, const double *Ty, int nx, int ny,
                             int nz, hipStream_t s) {
  const int64_t E = 2 * nz * (2 * nz + 1);
  const int64_t row = (int64_t)(nx + 1) * E;
  return parity_pass(tmp, row, E, spectral, row, E, nx + 1, Ty, ny, nz, false, s);
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
