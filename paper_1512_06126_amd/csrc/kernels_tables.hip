// Contractions of the coefficient-table build (Sect. 3.1 coefficients B_n^m;
// Appendix A horizontal integrals): a real FP64 GEMM used for
//   (1) the lambda -> rho Hankel contraction  H = W G   (W geometry only),
//   (2) the rho -> offset spatial contraction B_k = M_k H (M_k geometry only),
// and the kernel that forms the nine tensor components from the contracted
// blocks and writes the packed storage of Sect. 3.1.
#include "kernels.h"

namespace giem {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

// C[m][n] = sum_k At[k][m] B[k][n]  (row-major, FP64), 16x16x4 MFMA tiles.
// Workgroup: 4 waves, 64 x 64 outputs; wave w owns rows 32 (w >> 1), columns
// 32 (w & 1) as 2 x 2 tiles.  Operands come straight from global memory (the
// workgroup's 64-wide panels are re-read from L2 by its waves): both reads
// are coalesced, 16 consecutive doubles per quarter wave.
__global__ __launch_bounds__(256) void k_gemm_tn(const double *__restrict__ At, int64_t lda,
                                                 const double *__restrict__ B, int64_t ldb,
                                                 double *__restrict__ C, int64_t ldc, int m, int n,
                                                 int k) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int m0 = blockIdx.y * 64 + (w >> 1) * 32;
  const int n0 = blockIdx.x * 64 + (w & 1) * 32;
  const int li = lane & 15, lk = lane >> 4;
  d4 acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
  const int ra0 = m0 + li, ra1 = m0 + 16 + li;
  const int cb0 = n0 + li, cb1 = n0 + 16 + li;
  const bool va0 = ra0 < m, va1 = ra1 < m, vb0 = cb0 < n, vb1 = cb1 < n;
  for (int k0 = 0; k0 < k; k0 += 4) {
    const int kk = k0 + lk;
    const bool vk = kk < k;
    const double *ar = At + (int64_t)kk * lda;
    const double *br = B + (int64_t)kk * ldb;
    const double a0 = (vk && va0) ? ar[ra0] : 0.0;
    const double a1 = (vk && va1) ? ar[ra1] : 0.0;
    const double b0 = (vk && vb0) ? br[cb0] : 0.0;
    const double b1 = (vk && vb1) ? br[cb1] : 0.0;
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

// Packed entry e of offset o (layout of Sect. 3.1: upper triangles of xx, xy,
// yy, zz, then full xz and yz) from the contracted blocks:
//   c0[o][2T]     : (phi * h[A1]), (phi * h[A6/sigma])          (upper pairs)
//   c1[3][noff][T]: (-d_xx phi, -d_yy phi, -d_xy phi) * h[P/lambda^2]
//   c2[2][noff][nz^2]: (d_x phi, d_y phi) * h[A4/sigma]
//   xx = (i w mu0 c0_A1 + c1_xx) / 4pi,  yy likewise,  xy = c1_xy / 4pi,
//   zz = c0_A6 / 4pi,  xz = c2_x / 4pi,  yz = c2_y / 4pi.
// Entries odd in x at j = 0 or odd in y at i = 0 are set to zero (Lemma 2).
__global__ void k_assemble(const c128 *__restrict__ c0, const c128 *__restrict__ c1,
                           const c128 *__restrict__ c2, c128 *__restrict__ out, int nx, int ny,
                           int nz, double omega_mu0) {
  const int T = nz * (nz + 1) / 2, nz2 = nz * nz;
  const int E = 4 * T + 2 * nz2;
  const int64_t noff = (int64_t)nx * ny;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= noff * E) return;
  const int64_t o = idx / E;
  const int e = (int)(idx - o * E);
  const int i = (int)(o / nx), j = (int)(o - (int64_t)i * nx);
  const double c = 0.25 / 3.14159265358979323846;
  c128 v;
  if (e < T) {
    const c128 a1 = c0[o * 2 * T + e];
    v = mk<double>(c * (-omega_mu0 * a1.y + c1[o * T + e].x), c * (omega_mu0 * a1.x + c1[o * T + e].y));
  } else if (e < 2 * T) {
    const c128 q = c1[(2 * noff + o) * T + (e - T)];
    v = (i == 0 || j == 0) ? mk<double>(0.0, 0.0) : mk<double>(c * q.x, c * q.y);
  } else if (e < 3 * T) {
    const int u = e - 2 * T;
    const c128 a1 = c0[o * 2 * T + u];
    const c128 q = c1[(noff + o) * T + u];
    v = mk<double>(c * (-omega_mu0 * a1.y + q.x), c * (omega_mu0 * a1.x + q.y));
  } else if (e < 4 * T) {
    const c128 q = c0[o * 2 * T + T + (e - 3 * T)];
    v = mk<double>(c * q.x, c * q.y);
  } else if (e < 4 * T + nz2) {
    const c128 q = c2[o * nz2 + (e - 4 * T)];
    v = (j == 0) ? mk<double>(0.0, 0.0) : mk<double>(c * q.x, c * q.y);
  } else {
    const c128 q = c2[(noff + o) * nz2 + (e - 4 * T - nz2)];
    v = (i == 0) ? mk<double>(0.0, 0.0) : mk<double>(c * q.x, c * q.y);
  }
  out[idx] = v;
}

}  // namespace

hipError_t launch_gemm_tn(const double *At, int64_t lda, const double *B, int64_t ldb, double *C,
                          int64_t ldc, int m, int n, int k, hipStream_t s) {
  if (m <= 0 || n <= 0) return hipSuccess;
  dim3 grid((n + 63) / 64, (m + 63) / 64);
  if (grid.y > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_gemm_tn, grid, dim3(256), 0, s, At, lda, B, ldb, C, ldc, m, n, k);
  return hipGetLastError();
}

hipError_t launch_assemble(const c128 *c0, const c128 *c1, const c128 *c2, c128 *out, int nx,
                           int ny, int nz, double omega_mu0, hipStream_t s) {
  const int64_t total = (int64_t)nx * ny * (2 * nz * (2 * nz + 1));
  const int64_t blocks = (total + 255) / 256;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_assemble, dim3((unsigned)blocks), dim3(256), 0, s, c0, c1, c2, out, nx,
                     ny, nz, omega_mu0);
  return hipGetLastError();
}

}  // namespace giem
