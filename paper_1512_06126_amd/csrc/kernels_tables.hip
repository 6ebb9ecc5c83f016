// Contractions of the coefficient-table build (Sect. 3.1 coefficients B_n^m;
// Appendix A horizontal integrals): a real FP64 GEMM used for
//   (1) the lambda -> rho Hankel contraction  H = W G   (W geometry only),
//   (2) the rho -> offset spatial contraction B_k = M_k H (M_k geometry only),
// the kernel that forms the nine tensor components from the contracted
// blocks and writes the packed storage of Sect. 3.1, the lambda functions
// of the vertical integrals (Appendix B: one lambda node per thread for the
// layer recursions, one cell per thread for the cell factors, one depth
// level per thread for the rows of the products over the cells between, one
// lambda node per thread for a point observer's row), the two geometry-only
// rule matrices (Hankel weights; spatial fold, and its receiver form), and
// the receiver-side kernels (fields at receivers, impedance, dipole
// right-hand sides and the adjoint sums).
#include "kernels.h"
#include "vertical.h"

namespace giem {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

// C[m][n] = sum_k At[k][m] B[k][n]  (row-major, FP64), 16x16x4 MFMA tiles.
// Workgroup: 4 waves, 64 x 64 outputs; wave w owns rows 32 (w >> 1), columns
// 32 (w & 1) as 2 x 2 tiles.  Operands come straight from global memory (the
// workgroup's 64-wide panels are re-read from L2 by its waves): both reads
// are coalesced, 16 consecutive doubles per quarter wave.
// With krange, row tile t of C contracts only over [krange[2t], krange[2t+1])
// (the rows of At outside it are zero in that tile's columns).
__global__ __launch_bounds__(256) void k_gemm_tn(const double *__restrict__ At, int64_t lda,
                                                 const double *__restrict__ B, int64_t ldb,
                                                 double *__restrict__ C, int64_t ldc, int m, int n,
                                                 int k, const int *__restrict__ krange) {
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
  int kb = 0, ke = k;
  if (krange) {
    kb = krange[2 * blockIdx.y];
    ke = min(k, krange[2 * blockIdx.y + 1]);
  }
  for (int k0 = kb; k0 < ke; k0 += 4) {
    const int kk = k0 + lk;
    const bool vk = kk < ke;
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

// Receiver kernels: c[kind][off][f nz + jz] (kinds B0, BX, BY, BXX, BYY, BXY;
// functions A1, A2, dA1, A4/s, A5/s, A6/s, P, Q) -> out[off][jz][18], G^E then
// G^H row-major (row = field component at the receiver):
//   4pi E: xx = i w mu0 B0 A1 + BXX P, yy = i w mu0 B0 A1 + BYY P,
//          xy = yx = BXY P, xz = BX A4, yz = BY A4, zx = -BX A5,
//          zy = -BY A5, zz = B0 A6
//   4pi H: xx = BXY Q, yx = B0 dA1 - BXX Q, zx = -BY A1, xy = BYY Q - B0 dA1,
//          yy = -BXY Q, zy = BX A1, xz = BY A2, yz = -BX A2, zz = 0
__global__ void k_assemble_rec(const c128 *__restrict__ c, c128 *__restrict__ out, int noff,
                               int nz, double omega_mu0) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)noff * nz) return;
  const int o = (int)(idx / nz), jz = (int)(idx - (int64_t)o * nz);
  const int nf = 8 * nz;
  auto at = [&](int kind, int f) { return c[((int64_t)kind * noff + o) * nf + f * nz + jz]; };
  const double q = 0.25 / 3.14159265358979323846;
  auto sc = [&](c128 v, double f) { return mk<double>(q * f * v.x, q * f * v.y); };
  auto add = [&](c128 a, c128 b) { return mk<double>(a.x + b.x, a.y + b.y); };
  auto sub = [&](c128 a, c128 b) { return mk<double>(a.x - b.x, a.y - b.y); };
  auto iw = [&](c128 v) { return mk<double>(-omega_mu0 * v.y, omega_mu0 * v.x); };
  enum { B0 = 0, BX, BY, BXX, BYY, BXY };
  enum { A1 = 0, A2, DA1, A4, A5, A6, P, Q };
  c128 *r = out + idx * 18;
  const c128 zero = mk<double>(0.0, 0.0);
  r[0] = sc(add(iw(at(B0, A1)), at(BXX, P)), 1.0);
  r[1] = sc(at(BXY, P), 1.0);
  r[2] = sc(at(BX, A4), 1.0);
  r[3] = sc(at(BXY, P), 1.0);
  r[4] = sc(add(iw(at(B0, A1)), at(BYY, P)), 1.0);
  r[5] = sc(at(BY, A4), 1.0);
  r[6] = sc(at(BX, A5), -1.0);
  r[7] = sc(at(BY, A5), -1.0);
  r[8] = sc(at(B0, A6), 1.0);
  r[9] = sc(at(BXY, Q), 1.0);
  r[10] = sc(sub(at(BYY, Q), at(B0, DA1)), 1.0);
  r[11] = sc(at(BY, A2), 1.0);
  r[12] = sc(sub(at(B0, DA1), at(BXX, Q)), 1.0);
  r[13] = sc(at(BXY, Q), -1.0);
  r[14] = sc(at(BX, A2), -1.0);
  r[15] = sc(at(BY, A1), -1.0);
  r[16] = sc(at(BX, A1), 1.0);
  r[17] = zero;
}

// Fields at receivers above cell centres: one workgroup per (receiver, RHS);
// every thread sums the kernels against the currents (sa - sb) E of a
// stride of cells, then the workgroup reduces.
__global__ void __launch_bounds__(256)
k_fields(const c128 *__restrict__ K, const c128 *__restrict__ E, const c128 *__restrict__ sa,
         const c128 *__restrict__ sb_lev, const int *__restrict__ rec, int nrec, int nx, int ny,
         int nz, const c128 *__restrict__ en_hn, c128 *__restrict__ Erec, c128 *__restrict__ Hrec) {
  const int q = blockIdx.x, r = blockIdx.y;
  const int ir = rec[2 * q], jr = rec[2 * q + 1];
  const size_t plane = (size_t)nx * ny, N = plane * nz;
  const c128 *Er = E + (size_t)r * 3 * N;
  double acc[12];
  for (int i = 0; i < 12; ++i) acc[i] = 0.0;
  for (size_t n = threadIdx.x; n < N; n += blockDim.x) {
    const int iz = (int)(n / plane);
    const size_t rem = n - (size_t)iz * plane;
    const int iy = (int)(rem / nx), ix = (int)(rem - (size_t)iy * nx);
    const c128 ds = csub(sa[n], sb_lev[iz]);
    const c128 cu[3] = {cmul(ds, Er[n]), cmul(ds, Er[N + n]), cmul(ds, Er[2 * N + n])};
    const size_t off = (size_t)(jr - iy + ny - 1) * (2 * nx - 1) + (ir - ix + nx - 1);
    const c128 *k = K + (off * nz + iz) * 18;
#pragma unroll
    for (int a = 0; a < 6; ++a) {
      c128 s = mk<double>(0.0, 0.0);
#pragma unroll
      for (int b = 0; b < 3; ++b) cfma(s, k[3 * a + b], cu[b]);
      acc[2 * a] += s.x;
      acc[2 * a + 1] += s.y;
    }
  }
  __shared__ double red[256][13];
#pragma unroll
  for (int i = 0; i < 12; ++i) red[threadIdx.x][i] = acc[i];
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int i = 0; i < 12; ++i) red[threadIdx.x][i] += red[threadIdx.x + w][i];
    __syncthreads();
  }
  if (threadIdx.x < 6) {
    const int a = threadIdx.x;
    const c128 nf = en_hn[r * 6 + a];
    const c128 v = mk<double>(red[0][2 * a] + nf.x, red[0][2 * a + 1] + nf.y);
    if (a < 3)
      Erec[((size_t)r * nrec + q) * 3 + a] = v;
    else
      Hrec[((size_t)r * nrec + q) * 3 + (a - 3)] = v;
  }
}

// Impedance tensor at one receiver per thread: with Eh[c][p] = e_c of
// polarisation p and Hh likewise (c, p in {x, y}; RHS 0 / 1 = x / y
// polarisation), Z = Eh Hh^-1.  E, H: [2][nrec][3]; Z: [nrec][2][2].
__device__ inline void imp_load(const c128 *__restrict__ E, const c128 *__restrict__ H, int nrec,
                                int q, c128 (&Eh)[2][2], c128 (&Hi)[2][2]) {
  c128 Hh[2][2];
  for (int c = 0; c < 2; ++c)
    for (int p = 0; p < 2; ++p) {
      Eh[c][p] = E[((size_t)p * nrec + q) * 3 + c];
      Hh[c][p] = H[((size_t)p * nrec + q) * 3 + c];
    }
  const c128 det = csub(cmul(Hh[0][0], Hh[1][1]), cmul(Hh[0][1], Hh[1][0]));
  const double dn = det.x * det.x + det.y * det.y;
  const c128 id = mk<double>(det.x / dn, -det.y / dn);
  const c128 m1 = mk<double>(-1.0, 0.0);
  Hi[0][0] = cmul(Hh[1][1], id);
  Hi[0][1] = cmul(cmul(Hh[0][1], m1), id);
  Hi[1][0] = cmul(cmul(Hh[1][0], m1), id);
  Hi[1][1] = cmul(Hh[0][0], id);
}

__global__ void k_impedance(const c128 *__restrict__ E, const c128 *__restrict__ H, int nrec,
                            c128 *__restrict__ Z) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nrec) return;
  c128 Eh[2][2], Hi[2][2];
  imp_load(E, H, nrec, q, Eh, Hi);
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      c128 z = mk<double>(0.0, 0.0);
      for (int k = 0; k < 2; ++k) cfma(z, Eh[i][k], Hi[k][j]);
      Z[(size_t)q * 4 + i * 2 + j] = z;
    }
}

// Reverse mode of k_impedance.  G holds the gradient of a real L with respect
// to Z in the convention dL = Re sum conj(G_ij) dZ_ij.  Since
// dZ = (dEh - Z dHh) Hh^-1, with W = Hh^-1 G^H,
//   dL = Re sum_{p,c} ( W[p][c] dEh[c][p] - (W Z)[p][c] dHh[c][p] ),
// so the weights on the receiver fields are wE[p][q][c] = W[p][c] and
// wH[p][q][c] = -(W Z)[p][c] for c in {x, y}, and zero for c = z.
__global__ void k_impedance_adjoint(const c128 *__restrict__ E, const c128 *__restrict__ H, int nrec,
                                    const c128 *__restrict__ G, c128 *__restrict__ wE,
                                    c128 *__restrict__ wH) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nrec) return;
  c128 Eh[2][2], Hi[2][2], Z[2][2], W[2][2];
  imp_load(E, H, nrec, q, Eh, Hi);
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      c128 z = mk<double>(0.0, 0.0), w = mk<double>(0.0, 0.0);
      for (int k = 0; k < 2; ++k) {
        cfma(z, Eh[i][k], Hi[k][j]);
        const c128 g = G[(size_t)q * 4 + j * 2 + k];
        cfma(w, Hi[i][k], mk<double>(g.x, -g.y));
      }
      Z[i][j] = z;
      W[i][j] = w;
    }
  for (int p = 0; p < 2; ++p) {
    for (int c = 0; c < 2; ++c) {
      c128 wz = mk<double>(0.0, 0.0);
      for (int k = 0; k < 2; ++k) cfma(wz, W[p][k], Z[k][c]);
      wE[((size_t)p * nrec + q) * 3 + c] = W[p][c];
      wH[((size_t)p * nrec + q) * 3 + c] = mk<double>(-wz.x, -wz.y);
    }
    wE[((size_t)p * nrec + q) * 3 + 2] = mk<double>(0.0, 0.0);
    wH[((size_t)p * nrec + q) * 3 + 2] = mk<double>(0.0, 0.0);
  }
}

// Transpose of k_fields.  For dL = Re sum_{r,q,a} (wE[r][q][a] de_a + wH[r][q][a] dh_a)
// and the anomalous fields e = sum_n (sa_n - sb_n) KE(q, n) E_n (h likewise),
// per cell n and RHS r
//   v[b] = sum_q sum_a wE[r][q][a] KE(q, n)[a][b] + wH[r][q][a] KH(q, n)[a][b],
// the source of the adjoint solve is g[r][b][n] = (sa_n - sb_n) v[b] (the
// dependence through E) and, for real sa, the explicit dependence on log sa is
// grad[n] += Re sum_{r,b} sa_n v[b] E[r][b][n].  Threads run over depth first
// so that neighbouring threads read neighbouring entries of the kernel table
// [offset][Nz][18].
__global__ void __launch_bounds__(256)
k_fields_adjoint(const c128 *__restrict__ K, const c128 *__restrict__ E,
                 const c128 *__restrict__ sa, const c128 *__restrict__ sb_lev,
                 const int *__restrict__ rec, int nrec, int nrhs, int nx, int ny, int nz,
                 const c128 *__restrict__ wE, const c128 *__restrict__ wH, c128 *__restrict__ g,
                 double *__restrict__ grad) {
  const size_t plane = (size_t)nx * ny, N = plane * nz;
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  const int iz = (int)(t % nz);
  const size_t col = t / nz;
  const int ix = (int)(col % nx), iy = (int)(col / nx);
  const size_t n = (size_t)iz * plane + (size_t)iy * nx + ix;
  const c128 s = sa[n];
  const c128 ds = csub(s, sb_lev[iz]);
  double gsum = 0.0;
  for (int r = 0; r < nrhs; ++r) {
    c128 v[3] = {mk<double>(0.0, 0.0), mk<double>(0.0, 0.0), mk<double>(0.0, 0.0)};
    for (int q = 0; q < nrec; ++q) {
      const size_t off =
          (size_t)(rec[2 * q + 1] - iy + ny - 1) * (2 * nx - 1) + (rec[2 * q] - ix + nx - 1);
      const c128 *k = K + (off * nz + iz) * 18;
      const c128 *we = wE + ((size_t)r * nrec + q) * 3;
      const c128 *wh = wH + ((size_t)r * nrec + q) * 3;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const c128 ea = we[a], ha = wh[a];
#pragma unroll
        for (int b = 0; b < 3; ++b) {
          cfma(v[b], ea, k[3 * a + b]);
          cfma(v[b], ha, k[9 + 3 * a + b]);
        }
      }
    }
    for (int b = 0; b < 3; ++b) {
      g[((size_t)r * 3 + b) * N + n] = cmul(ds, v[b]);
      gsum += cmul(cmul(s, v[b]), E[((size_t)r * 3 + b) * N + n]).x;
    }
  }
  grad[n] += gsum;
}

// p/q recursions of every lambda node: eta, L, p, q of lambda l at l (nlay + 1)
// (p and q: both kinds, 2 (nlay + 1) per node)
__global__ __launch_bounds__(256) void k_vert_layers(vert::Model m, const double *__restrict__ lam,
                                                     int nl, vert::zc *eta, double *L,
                                                     vert::zc *p, vert::zc *q) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= nl) return;
  const int nlayers = m.nlay + 1;
  vert::layer_fns(lam[l], m, eta + (size_t)l * nlayers, L + (size_t)l * nlayers,
                  p + (size_t)2 * l * nlayers, q + (size_t)2 * l * nlayers);
}

// factors of cell c, kind k, lambda l at cells[(l 2 + k) nz + c]
__global__ __launch_bounds__(256) void k_vert_cells(vert::Model m, int nl,
                                                    const vert::zc *__restrict__ eta,
                                                    const double *__restrict__ L,
                                                    const vert::zc *__restrict__ p,
                                                    const vert::zc *__restrict__ q,
                                                    vert::Cell *cells) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)nl * 2 * m.nz) return;
  const int l = (int)(idx / (2 * m.nz)), k = (int)(idx / m.nz) % 2, c = (int)(idx % m.nz);
  const int nlayers = m.nlay + 1;
  vert::cell_factors(c, k, m, eta + (size_t)l * nlayers, L + (size_t)l * nlayers,
                     p + (size_t)2 * l * nlayers, q + (size_t)2 * l * nlayers, cells[idx]);
}

// the point observer's lambda functions of node l into G[l][8 nz]
__global__ __launch_bounds__(64) void k_vert_point(vert::Model m, vert::Observer ob,
                                                   const double *__restrict__ lam, int nl,
                                                   const vert::zc *__restrict__ eta,
                                                   const double *__restrict__ L,
                                                   const vert::zc *__restrict__ p,
                                                   const vert::zc *__restrict__ q,
                                                   const vert::Cell *__restrict__ cells,
                                                   vert::zc *G) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= nl) return;
  const int nlayers = m.nlay + 1;
  const vert::Cell *c0 = cells + (size_t)l * 2 * m.nz;
  vert::point_row(lam[l], m, ob, eta + (size_t)l * nlayers, L + (size_t)l * nlayers,
                  p + (size_t)2 * l * nlayers, q + (size_t)2 * l * nlayers, c0, c0 + m.nz,
                  G + (size_t)l * 8 * m.nz);
}

// row i of the lambda functions of node l into G[l][ncolc]
__global__ __launch_bounds__(256) void k_vert_rows(vert::Model m, const double *__restrict__ lam,
                                                   int nl, const vert::Cell *__restrict__ cells,
                                                   vert::zc *G, int ncolc) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)nl * m.nz) return;
  const int l = (int)(idx / m.nz), i = (int)(idx % m.nz);
  const vert::Cell *c0 = cells + (size_t)l * 2 * m.nz;
  vert::table_row(i, lam[l], m, c0, c0 + m.nz, G + (size_t)l * ncolc);
}

// Hankel weights (Sect. 3.1 horizontal integration, the lambda -> rho
// transform h(rho) = int J0(lambda rho) g(lambda) dlambda): row rho of the
// weight matrix sums, over the quadrature nodes of the lambda integral, the
// node weight times J0(lambda rho) times the barycentric interpolation
// weights of g at lambda on its panel of the logarithmic Chebyshev grid.
// The nodes: [lambda_lo, z1 / rho] in halving subpanels (lambda_a as a
// breakpoint), then the panels between consecutive zeros of J0 up to the
// K-th, then the tail panels weighted by the averaged limit of the last
// partial sums.  One wavefront per (rho, lambda panel) sums the nodes that
// fall into its panel and writes that panel's 16 columns (plain and
// regularised: J0 - 1 below lambda_a).
struct HankelArgs {
  const double *zeros, *edges, *node, *bw, *rho, *g1x, *g1w, *g2x, *g2w, *beta;
  int nzeros, npan, nr, ng1, ng2, nt;
  double lam_lo, lam_a, lam_asym;
};
constexpr int kHankelN = 16;  // nodes per lambda panel
constexpr double kPiD = 3.14159265358979323846;

__device__ __forceinline__ void hankel_node(const HankelArgs &a, int p, double rho, double lam,
                                            double w, double (&acc)[kHankelN],
                                            double (&accr)[kHankelN]) {
  const double u = log(lam);
  // panel of lambda: last edge <= u (upper bound - 1), clamped
  int lo = 0, hi = a.npan + 1;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (a.edges[mid] > u) hi = mid;
    else lo = mid + 1;
  }
  int pn = lo - 1;
  pn = pn < 0 ? 0 : (pn > a.npan - 1 ? a.npan - 1 : pn);
  if (pn != p) return;
  const double e0 = a.edges[p], e1 = a.edges[p + 1];
  const double sl = (2.0 * u - (e0 + e1)) / (e1 - e0);
  double wi[kHankelN];
  double tot = 0.0;
  int hit = -1;
#pragma unroll
  for (int j = 0; j < kHankelN; ++j) {
    const double d = sl - a.node[j];
    if (fabs(d) < 1e-14) hit = j;
    wi[j] = hit >= 0 ? 0.0 : a.bw[j] / d;
    tot += wi[j];
  }
#pragma unroll
  for (int j = 0; j < kHankelN; ++j) wi[j] = hit >= 0 ? (j == hit ? 1.0 : 0.0) : wi[j] / tot;
  const double jv = j0(lam * rho);
  const double jr = lam < a.lam_a ? jv - 1.0 : jv;
#pragma unroll
  for (int q = 0; q < kHankelN; ++q) {
    acc[q] += w * jv * wi[q];
    accr[q] += w * jr * wi[q];
  }
}

// One wavefront per (rho, lambda panel): its lanes take the subpanels and
// the zero panels in turn and the wavefront sums their partial columns with
// a fixed butterfly (the large rho nodes' high panels hold tens of
// thousands of quadrature nodes, the low ones a few).
__global__ __launch_bounds__(256) void k_hankel_weights(HankelArgs a, double *__restrict__ Wt,
                                                        double *__restrict__ Wt_reg) {
  const int lane = threadIdx.x & 63;
  const int64_t idx = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (idx >= (int64_t)a.nr * a.npan) return;  // whole wavefront
  const int p = (int)(idx % a.npan), ir = (int)(idx / a.npan);
  const double rho = a.rho[ir];
  // the panel's lambda range, widened (the node filter is exact)
  const double Llo = p == 0 ? 0.0 : exp(a.edges[p]) * (1.0 - 1e-9);
  const double Lhi = p == a.npan - 1 ? INFINITY : exp(a.edges[p + 1]) * (1.0 + 1e-9);
  double acc[kHankelN], accr[kHankelN];
#pragma unroll
  for (int q = 0; q < kHankelN; ++q) acc[q] = accr[q] = 0.0;
  const double l1 = a.zeros[0] / rho;
  if (Llo <= l1) {
    // subpanels [lam_lo, l1 / 2^M], ..., [l1 / 2, l1] (exact halvings), the
    // one holding lambda_a split there
    int M = 0;
    while (ldexp(l1, -M) / 2.0 > a.lam_lo) ++M;
    for (int m = M - lane; m >= 0; m -= 64) {
      const double a0 = m == M ? a.lam_lo : ldexp(l1, -(m + 1)), b0 = ldexp(l1, -m);
      if (b0 < Llo || a0 > Lhi) continue;
      const bool split = a.lam_a > a0 && a.lam_a < b0;
      for (int piece = 0; piece < (split ? 2 : 1); ++piece) {
        const double pa = split && piece == 1 ? a.lam_a : a0;
        const double pb = split && piece == 0 ? a.lam_a : b0;
        for (int q = 0; q < a.ng1; ++q) {
          const double lam = 0.5 * (pa + pb) + 0.5 * (pb - pa) * a.g1x[q];
          hankel_node(a, p, rho, lam, 0.5 * (pb - pa) * a.g1w[q], acc, accr);
        }
      }
    }
  }
  // panels k = 1 .. K - 1 + nt between zeros k - 1 and k (the last nt the
  // tail, weighted by beta)
  const int K = (int)ceil(a.lam_asym * rho / kPiD) + 1;
  const int klast = K - 1 + a.nt;
  // first k with zeros[k] / rho >= Llo, last k with zeros[k - 1] / rho <= Lhi
  int lo = 1, hi = klast + 1;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (a.zeros[mid] / rho >= Llo) hi = mid;
    else lo = mid + 1;
  }
  const int kmin = lo;
  lo = kmin;
  hi = klast + 1;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (a.zeros[mid - 1] / rho <= Lhi) lo = mid + 1;
    else hi = mid;
  }
  const int kmax = lo - 1;
  for (int k = kmin + lane; k <= kmax; k += 64) {
    const double za = a.zeros[k - 1] / rho, zb = a.zeros[k] / rho;
    const double scale = k < K ? 1.0 : a.beta[k - K];
    for (int q = 0; q < a.ng2; ++q) {
      const double lam = 0.5 * (za + zb) + 0.5 * (zb - za) * a.g2x[q];
      hankel_node(a, p, rho, lam, scale * 0.5 * (zb - za) * a.g2w[q], acc, accr);
    }
  }
#pragma unroll
  for (int q = 0; q < kHankelN; ++q) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      acc[q] += __shfl_xor(acc[q], off, 64);
      accr[q] += __shfl_xor(accr[q], off, 64);
    }
  }
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < kHankelN; ++q) {
      Wt[(size_t)(p * kHankelN + q) * a.nr + ir] = acc[q];
      Wt_reg[(size_t)(p * kHankelN + q) * a.nr + ir] = accr[q];
    }
  }
}

// Spatial fold matrix (Appendix A, the horizontal Galerkin integrals as
// convolutions of the radial functions with the footprint autocorrelation
// phi): column (kind, offset) holds, over the rho nodes, the quadrature
// weights of int w_kind(u, v) h(|D - (u, v)|) du dv (kinds phi, d_x phi,
// d_y phi, d_xy phi over the four quadrants of phi's support) or of the
// line integrals of -d_xx phi and -d_yy phi, each weight spread over the
// barycentric interpolation weights of h on its rho panel.  One thread per
// column (the columns are disjoint): quadrants with the singular vertex at D
// by two triangles with a graded radial variable (tanh-sinh), the others by
// tensor Gauss-Legendre rules (14 points within 2 h of D, split in 2 x 2
// within h / 2, 8 points beyond); lines by Gauss-Legendre pieces, the ends
// at D by the radial rule.  Weights of one rho panel are summed in
// registers and added to the column when the panel changes.
struct FoldArgs {
  const double *edges, *node, *bw;  // rho grid: npan + 1 edges, 12 nodes per panel
  const double *gs_x, *gs_w, *g14_x, *g14_w, *g8_x, *g8_w, *rad_x, *rad_w;
  int npan, nrad, nx, ny;
  double hx, hy, rho_min;
};
constexpr int kFoldN = 12;
enum { F_W0 = 0, F_XX, F_YY, F_XY, F_X, F_Y, F_COUNT };

struct FoldAcc {
  double acc[kFoldN];
  int cur, lo, hi;
};

__device__ __forceinline__ void fold_flush(FoldAcc &f, double *Mt, int64_t ncol, int64_t col) {
  if (f.cur < 0) return;
#pragma unroll
  for (int k = 0; k < kFoldN; ++k) {
    Mt[(int64_t)(f.cur * kFoldN + k) * ncol + col] += f.acc[k];
    f.acc[k] = 0.0;
  }
}

__device__ __forceinline__ void fold_emit(const FoldArgs &a, FoldAcc &f, double r, double w,
                                          double *Mt, int64_t ncol, int64_t col,
                                          bool deriv = false) {
  const double xq = r > a.rho_min ? r : a.rho_min;
  const double u = log(xq);
  int lo = 0, hi = a.npan + 1;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (a.edges[mid] > u) hi = mid;
    else lo = mid + 1;
  }
  int p = lo - 1;
  p = p < 0 ? 0 : (p > a.npan - 1 ? a.npan - 1 : p);
  if (p != f.cur) {
    fold_flush(f, Mt, ncol, col);
    f.cur = p;
    f.lo = min(f.lo, p * kFoldN);
    f.hi = max(f.hi, p * kFoldN + kFoldN);
  }
  const double e0 = a.edges[p], e1 = a.edges[p + 1];
  const double sl = (2.0 * u - (e0 + e1)) / (e1 - e0);
  if (deriv) {
    // d/d rho of the panel's interpolating polynomial in ln rho
    const double scale = 2.0 / (e1 - e0) / xq;
    int hit = -1;
#pragma unroll
    for (int j = 0; j < kFoldN; ++j)
      if (fabs(sl - a.node[j]) < 1e-14) hit = j;
    if (hit >= 0) {
      // row of the barycentric differentiation matrix
      double diag = 0.0;
#pragma unroll
      for (int j = 0; j < kFoldN; ++j) {
        if (j == hit) continue;
        const double dj = (a.bw[j] / a.bw[hit]) / (a.node[hit] - a.node[j]);
        diag -= dj;
        f.acc[j] += w * (dj * scale);
      }
      f.acc[hit] += w * (diag * scale);
    } else {
      double D = 0.0, Dd = 0.0;
#pragma unroll
      for (int j = 0; j < kFoldN; ++j) {
        const double d = sl - a.node[j];
        D += a.bw[j] / d;
        Dd += -a.bw[j] / (d * d);
      }
#pragma unroll
      for (int j = 0; j < kFoldN; ++j) {
        const double d = sl - a.node[j];
        const double aj = a.bw[j] / d, adj = -a.bw[j] / (d * d);
        f.acc[j] += w * ((adj / D - aj * Dd / (D * D)) * scale);
      }
    }
    return;
  }
  double wi[kFoldN];
  double tot = 0.0;
  int hit = -1;
#pragma unroll
  for (int j = 0; j < kFoldN; ++j) {
    const double d = sl - a.node[j];
    if (fabs(d) < 1e-14) hit = j;
    wi[j] = hit >= 0 ? 0.0 : a.bw[j] / d;
    tot += wi[j];
  }
#pragma unroll
  for (int j = 0; j < kFoldN; ++j)
    f.acc[j] += w * (hit >= 0 ? (j == hit ? 1.0 : 0.0) : wi[j] / tot);
}

__device__ __forceinline__ double fold_weight(int kind, double u, double v, double su, double sv,
                                              double hx, double hy) {
  switch (kind) {
    case F_W0: return (hx - fabs(u)) * (hy - fabs(v));
    case F_X: return -su * (hy - fabs(v));
    case F_Y: return -sv * (hx - fabs(u));
    default: return -su * sv;  // F_XY
  }
}

__global__ __launch_bounds__(128) void k_spatial_fold(FoldArgs a, double *__restrict__ Mt,
                                                      int *__restrict__ kcol) {
  const int64_t noff = (int64_t)a.nx * a.ny, ncol = F_COUNT * noff;
  const int64_t col = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= ncol) return;
  const int kind = (int)(col / noff), o = (int)(col - kind * noff);
  const double dx = (o % a.nx) * a.hx, dy = (o / a.nx) * a.hy;
  const double hx = a.hx, hy = a.hy;
  FoldAcc f;
  f.cur = -1;
  f.lo = 1 << 30;
  f.hi = 0;
#pragma unroll
  for (int k = 0; k < kFoldN; ++k) f.acc[k] = 0.0;
  if (kind == F_XX || kind == F_YY) {
    // -d_xx phi = -(delta(u + hx) - 2 delta(u) + delta(u - hx)) (hy - |v|)
    // (and with x, y exchanged): three lines along the other axis
    const double dfix = kind == F_XX ? dx : dy, drun = kind == F_XX ? dy : dx;
    const double hfix = kind == F_XX ? hx : hy, hrun = kind == F_XX ? hy : hx;
    for (int c = -1; c <= 1; ++c) {
      const double wc = c == 0 ? 2.0 : -1.0;
      const double off = dfix - c * hfix;
      double cuts[4] = {-hrun, 0.0, hrun, 0.0};
      int nc = 3;
      if (drun > -hrun && drun < hrun && drun != 0.0) {
        // insert drun in order
        cuts[3] = hrun;
        if (drun < 0.0) {
          cuts[2] = 0.0;
          cuts[1] = drun;
        } else {
          cuts[2] = drun;
        }
        nc = 4;
      }
      const bool on_line = fabs(off) < 1e-12 * hfix;
      for (int pc = 0; pc + 1 < nc; ++pc) {
        const double pa = cuts[pc], pb = cuts[pc + 1];
        const bool sa = on_line && fabs(pa - drun) < 1e-12 * hrun;
        const bool sb = on_line && fabs(pb - drun) < 1e-12 * hrun;
        if (sa || sb) {
          // logarithmic singularity at the end pa (sa) or pb (sb)
          for (int i = 0; i < a.nrad; ++i) {
            const double v = sa ? pa + (pb - pa) * a.rad_x[i] : pb - (pb - pa) * a.rad_x[i];
            fold_emit(a, f, hypot(off, drun - v), wc * (pb - pa) * a.rad_w[i] * (hrun - fabs(v)),
                      Mt, ncol, col);
          }
          continue;
        }
        for (int i = 0; i < 24; ++i) {
          const double v = 0.5 * (pa + pb) + 0.5 * (pb - pa) * a.gs_x[i];
          const double wv = 0.5 * (pb - pa) * a.gs_w[i];
          fold_emit(a, f, hypot(off, drun - v), wc * wv * (hrun - fabs(v)), Mt, ncol, col);
        }
      }
    }
  } else {
    for (int sx = -1; sx <= 1; sx += 2)
      for (int sy = -1; sy <= 1; sy += 2) {
        const double x0 = fmin(0.0, sx * hx), x1 = fmax(0.0, sx * hx);
        const double y0 = fmin(0.0, sy * hy), y1 = fmax(0.0, sy * hy);
        const double tx = 1e-9 * hx, ty = 1e-9 * hy;
        int sing = -1;
        const double vx[2] = {x0, x1}, vy[2] = {y0, y1};
        for (int ia = 0; ia < 2; ++ia)
          for (int ib = 0; ib < 2; ++ib)
            if (fabs(vx[ia] - dx) < tx && fabs(vy[ib] - dy) < ty) sing = 2 * ia + ib;
        if (sing >= 0) {
          // two triangles from the singular vertex P, graded radial variable
          const double px = vx[sing >> 1], py = vy[sing & 1];
          const double ox = vx[1 - (sing >> 1)], oy = vy[1 - (sing & 1)];
          for (int tri = 0; tri < 2; ++tri) {
            const double cx = tri == 0 ? ox : px, cy = tri == 0 ? py : oy;  // adjacent corner
            const double e1x = cx - px, e1y = cy - py;
            const double e2x = ox - cx, e2y = oy - cy;
            const double det = fabs(e1x * e2y - e1y * e2x);
            for (int i = 0; i < a.nrad; ++i) {
              const double r = a.rad_x[i], wr = a.rad_w[i];
              for (int j = 0; j < 24; ++j) {
                const double tt = 0.5 * (a.gs_x[j] + 1.0), wt = 0.5 * a.gs_w[j];
                const double uu = px + r * (e1x + tt * e2x), vv = py + r * (e1y + tt * e2y);
                fold_emit(a, f, hypot(dx - uu, dy - vv),
                          wr * wt * r * det * fold_weight(kind, uu, vv, sx, sy, hx, hy), Mt, ncol,
                          col);
              }
            }
          }
          continue;
        }
        const double ddx = fmax(fmax(x0 - dx, 0.0), dx - x1);
        const double ddy = fmax(fmax(y0 - dy, 0.0), dy - y1);
        const double dist = hypot(ddx, ddy), hm = fmin(hx, hy);
        const bool near = dist < 2.0 * hm;
        const double *rx = near ? a.g14_x : a.g8_x, *rw = near ? a.g14_w : a.g8_w;
        const int n = near ? 14 : 8;
        const int split = dist < 0.5 * hm ? 2 : 1;
        for (int ia = 0; ia < split; ++ia)
          for (int ib = 0; ib < split; ++ib) {
            const double xa = x0 + (x1 - x0) * ia / split, xb = x0 + (x1 - x0) * (ia + 1) / split;
            const double ya = y0 + (y1 - y0) * ib / split, yb = y0 + (y1 - y0) * (ib + 1) / split;
            for (int i = 0; i < n; ++i)
              for (int j = 0; j < n; ++j) {
                const double uu = 0.5 * (xa + xb) + 0.5 * (xb - xa) * rx[i];
                const double vv = 0.5 * (ya + yb) + 0.5 * (yb - ya) * rx[j];
                fold_emit(a, f, hypot(dx - uu, dy - vv),
                          0.25 * (xb - xa) * (yb - ya) * rw[i] * rw[j] *
                              fold_weight(kind, uu, vv, sx, sy, hx, hy),
                          Mt, ncol, col);
              }
          }
      }
  }
  fold_flush(f, Mt, ncol, col);
  kcol[2 * col] = f.lo < f.hi ? f.lo : 0;
  kcol[2 * col + 1] = f.lo < f.hi ? f.hi : 0;
}

// Receiver rule matrix: a receiver above the centre of a cell at lateral
// offset (dx, dy) from the centre of the source cell sees the footprint B =
// [-hx/2, hx/2] x [-hy/2, hy/2]; column (kind, offset) holds the weights of
// int_B h(|D - r'|) (kind 0; B split at the receiver's projection, the
// pieces with D at a vertex by two triangles with r = s^2 grading, the
// others by tensor Gauss-Legendre rules), of the face measures of d_x B and
// d_y B against h (kinds 1, 2), and of the same faces against -dh/dx or
// -dh/dy (kinds 3, 4, 5: derivative weights of h on its rho panel).  One
// thread per column; offsets (di, dj) with |di| < Nx, |dj| < Ny.
enum { RF_B0 = 0, RF_BX, RF_BY, RF_BXX, RF_BYY, RF_BXY, RF_COUNT };

__device__ void rec_box(const FoldArgs &a, FoldAcc &f, double dx, double dy, double x0, double x1,
                        double y0, double y1, double h, double *Mt, int64_t ncol, int64_t col) {
  const double tol = 1e-9 * h;
  int sing = -1;
  const double vx[2] = {x0, x1}, vy[2] = {y0, y1};
  for (int ia = 0; ia < 2; ++ia)
    for (int ib = 0; ib < 2; ++ib)
      if (fabs(vx[ia] - dx) < tol && fabs(vy[ib] - dy) < tol) sing = 2 * ia + ib;
  if (sing >= 0) {
    const double px = vx[sing >> 1], py = vy[sing & 1];
    const double ox = vx[1 - (sing >> 1)], oy = vy[1 - (sing & 1)];
    for (int tri = 0; tri < 2; ++tri) {
      const double cx = tri == 0 ? ox : px, cy = tri == 0 ? py : oy;
      const double e1x = cx - px, e1y = cy - py;
      const double e2x = ox - cx, e2y = oy - cy;
      const double det = fabs(e1x * e2y - e1y * e2x);
      for (int i = 0; i < 24; ++i) {
        const double sv = 0.5 * (a.gs_x[i] + 1.0), ws = 0.5 * a.gs_w[i];
        const double r = sv * sv, wr = ws * 2.0 * sv;
        for (int j = 0; j < 24; ++j) {
          const double tt = 0.5 * (a.gs_x[j] + 1.0), wt = 0.5 * a.gs_w[j];
          const double uu = px + r * (e1x + tt * e2x), vv = py + r * (e1y + tt * e2y);
          fold_emit(a, f, hypot(dx - uu, dy - vv), wr * wt * r * det, Mt, ncol, col);
        }
      }
    }
    return;
  }
  const double dist = hypot(fmax(fmax(x0 - dx, 0.0), dx - x1), fmax(fmax(y0 - dy, 0.0), dy - y1));
  const bool near = dist < 2.0 * h;
  const double *rx = near ? a.g14_x : a.g8_x, *rw = near ? a.g14_w : a.g8_w;
  const int n = near ? 14 : 8;
  const int split = dist < 0.5 * h ? 3 : 1;
  for (int ia = 0; ia < split; ++ia)
    for (int ib = 0; ib < split; ++ib) {
      const double xa = x0 + (x1 - x0) * ia / split, xb = x0 + (x1 - x0) * (ia + 1) / split;
      const double ya = y0 + (y1 - y0) * ib / split, yb = y0 + (y1 - y0) * (ib + 1) / split;
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
          const double uu = 0.5 * (xa + xb) + 0.5 * (xb - xa) * rx[i];
          const double vv = 0.5 * (ya + yb) + 0.5 * (yb - ya) * rx[j];
          fold_emit(a, f, hypot(dx - uu, dy - vv), 0.25 * (xb - xa) * (yb - ya) * rw[i] * rw[j],
                    Mt, ncol, col);
        }
    }
}

__global__ __launch_bounds__(128) void k_receiver_fold(FoldArgs a, double *__restrict__ Mt,
                                                       int *__restrict__ kcol) {
  const int nxo = 2 * a.nx - 1, nyo = 2 * a.ny - 1;
  const int64_t noff = (int64_t)nxo * nyo, ncol = RF_COUNT * noff;
  const int64_t col = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= ncol) return;
  const int kind = (int)(col / noff), o = (int)(col - kind * noff);
  const int dj = o / nxo - (a.ny - 1), di = o % nxo - (a.nx - 1);
  const double hx = a.hx, hy = a.hy, dx = di * hx, dy = dj * hy;
  FoldAcc f;
  f.cur = -1;
  f.lo = 1 << 30;
  f.hi = 0;
#pragma unroll
  for (int k = 0; k < kFoldN; ++k) f.acc[k] = 0.0;
  if (kind == RF_B0) {
    // the footprint split at the receiver's projection
    double xs[3] = {-hx / 2, hx / 2, hx / 2}, ys[3] = {-hy / 2, hy / 2, hy / 2};
    int nxs = 2, nys = 2;
    if (dx > -hx / 2 && dx < hx / 2) {
      xs[1] = dx;
      nxs = 3;
    }
    if (dy > -hy / 2 && dy < hy / 2) {
      ys[1] = dy;
      nys = 3;
    }
    for (int ia = 0; ia + 1 < nxs; ++ia)
      for (int ib = 0; ib + 1 < nys; ++ib)
        rec_box(a, f, dx, dy, xs[ia], xs[ia + 1], ys[ib], ys[ib + 1], fmin(hx, hy), Mt, ncol, col);
  } else {
    const bool xface = kind == RF_BX || kind == RF_BXX || kind == RF_BXY;
    for (int side = 0; side < 2; ++side) {
      const double sgn = side == 0 ? 1.0 : -1.0;
      const double fpos = (side == 0 ? -0.5 : 0.5) * (xface ? hx : hy);
      const double half = 0.5 * (xface ? hy : hx);
      const double dn = xface ? dx : dy;  // normal coordinate of the receiver
      const double dt = xface ? dy : dx;  // running coordinate
      double cuts[3] = {-half, half, half};
      int nc = 2;
      if (dt > -half && dt < half) {
        cuts[1] = dt;
        nc = 3;
      }
      for (int piece = 0; piece + 1 < nc; ++piece) {
        const double pa = cuts[piece], pb = cuts[piece + 1];
        for (int i = 0; i < 24; ++i) {
          const double tq = 0.5 * (pa + pb) + 0.5 * (pb - pa) * a.gs_x[i];
          const double w = sgn * 0.5 * (pb - pa) * a.gs_w[i];
          const double rho = hypot(dn - fpos, dt - tq);
          if (kind == RF_BX || kind == RF_BY)
            fold_emit(a, f, rho, w, Mt, ncol, col);
          else if (kind == RF_BXX || kind == RF_BYY)
            fold_emit(a, f, rho, -w * (dn - fpos) / rho, Mt, ncol, col, true);
          else
            fold_emit(a, f, rho, -w * (dt - tq) / rho, Mt, ncol, col, true);
        }
      }
    }
  }
  fold_flush(f, Mt, ncol, col);
  kcol[2 * col] = f.lo < f.hi ? f.lo : 0;
  kcol[2 * col + 1] = f.lo < f.hi ? f.hi : 0;
}

}  // namespace

hipError_t launch_receiver_fold(const double *args, int npan, int nrad, int nx, int ny, double hx,
                                 double hy, double rho_min, double *Mt, int *kcol, hipStream_t s) {
  // args as for launch_spatial_fold (the radial rule is not used)
  FoldArgs a;
  a.edges = args;
  a.node = a.edges + npan + 1;
  a.bw = a.node + kFoldN;
  a.gs_x = a.bw + kFoldN;
  a.gs_w = a.gs_x + 24;
  a.g14_x = a.gs_w + 24;
  a.g14_w = a.g14_x + 14;
  a.g8_x = a.g14_w + 14;
  a.g8_w = a.g8_x + 8;
  a.rad_x = a.g8_w + 8;
  a.rad_w = a.rad_x + nrad;
  a.npan = npan;
  a.nrad = nrad;
  a.nx = nx;
  a.ny = ny;
  a.hx = hx;
  a.hy = hy;
  a.rho_min = rho_min;
  const int64_t ncol = (int64_t)RF_COUNT * (2 * nx - 1) * (2 * ny - 1);
  if (ncol <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_receiver_fold, dim3((unsigned)((ncol + 127) / 128)), dim3(128), 0, s, a, Mt,
                     kcol);
  return hipGetLastError();
}

hipError_t launch_spatial_fold(const double *args, int npan, int nrad, int nx, int ny, double hx,
                               double hy, double rho_min, double *Mt, int *kcol, hipStream_t s) {
  // args: edges [npan + 1], node [12], bw [12], Gauss-Legendre 24, 14, 8 (x
  // then w), radial rule [nrad] (x then w); Mt zeroed by the caller
  FoldArgs a;
  a.edges = args;
  a.node = a.edges + npan + 1;
  a.bw = a.node + kFoldN;
  a.gs_x = a.bw + kFoldN;
  a.gs_w = a.gs_x + 24;
  a.g14_x = a.gs_w + 24;
  a.g14_w = a.g14_x + 14;
  a.g8_x = a.g14_w + 14;
  a.g8_w = a.g8_x + 8;
  a.rad_x = a.g8_w + 8;
  a.rad_w = a.rad_x + nrad;
  a.npan = npan;
  a.nrad = nrad;
  a.nx = nx;
  a.ny = ny;
  a.hx = hx;
  a.hy = hy;
  a.rho_min = rho_min;
  const int64_t ncol = (int64_t)F_COUNT * nx * ny;
  if (ncol <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_spatial_fold, dim3((unsigned)((ncol + 127) / 128)), dim3(128), 0, s, a, Mt,
                     kcol);
  return hipGetLastError();
}

hipError_t launch_hankel_weights(const double *args, int nzeros, int npan, int nr, int ng1, int ng2,
                                 int nt, double lam_lo, double lam_a, double lam_asym, double *Wt,
                                 double *Wt_reg, hipStream_t s) {
  // args: zeros [nzeros], edges [npan + 1], node [16], bw [16], rho [nr],
  // g1x, g1w [ng1], g2x, g2w [ng2], beta [nt]
  HankelArgs a;
  a.zeros = args;
  a.edges = a.zeros + nzeros;
  a.node = a.edges + npan + 1;
  a.bw = a.node + kHankelN;
  a.rho = a.bw + kHankelN;
  a.g1x = a.rho + nr;
  a.g1w = a.g1x + ng1;
  a.g2x = a.g1w + ng1;
  a.g2w = a.g2x + ng2;
  a.beta = a.g2w + ng2;
  a.nzeros = nzeros;
  a.npan = npan;
  a.nr = nr;
  a.ng1 = ng1;
  a.ng2 = ng2;
  a.nt = nt;
  a.lam_lo = lam_lo;
  a.lam_a = lam_a;
  a.lam_asym = lam_asym;
  const int64_t n = (int64_t)nr * npan;  // one wavefront each, four per workgroup
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_hankel_weights, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, a, Wt,
                     Wt_reg);
  return hipGetLastError();
}

hipError_t launch_vertical_point(const vert::Model &m, const vert::Observer &ob, const double *lam,
                                 int nl, vert::zc *eta, double *L, vert::zc *p, vert::zc *q,
                                 vert::Cell *cells, vert::zc *G, hipStream_t s) {
  if (nl <= 0 || m.nz <= 0) return hipSuccess;
  const int64_t ncell = (int64_t)nl * 2 * m.nz;
  if ((ncell + 255) / 256 > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_vert_layers, dim3((nl + 255) / 256), dim3(256), 0, s, m, lam, nl, eta, L, p,
                     q);
  hipLaunchKernelGGL(k_vert_cells, dim3((unsigned)((ncell + 255) / 256)), dim3(256), 0, s, m, nl,
                     eta, L, p, q, cells);
  hipLaunchKernelGGL(k_vert_point, dim3((nl + 63) / 64), dim3(64), 0, s, m, ob, lam, nl, eta, L, p,
                     q, cells, G);
  return hipGetLastError();
}

hipError_t launch_vertical_rows(const vert::Model &m, const double *lam, int nl, vert::zc *eta,
                                double *L, vert::zc *p, vert::zc *q, vert::Cell *cells,
                                vert::zc *G, int ncolc, hipStream_t s) {
  if (nl <= 0 || m.nz <= 0) return hipSuccess;
  const int64_t ncell = (int64_t)nl * 2 * m.nz, nrow = (int64_t)nl * m.nz;
  if ((ncell + 255) / 256 > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_vert_layers, dim3((nl + 255) / 256), dim3(256), 0, s, m, lam, nl, eta, L, p,
                     q);
  hipLaunchKernelGGL(k_vert_cells, dim3((unsigned)((ncell + 255) / 256)), dim3(256), 0, s, m, nl,
                     eta, L, p, q, cells);
  hipLaunchKernelGGL(k_vert_rows, dim3((unsigned)((nrow + 255) / 256)), dim3(256), 0, s, m, lam,
                     nl, cells, G, ncolc);
  return hipGetLastError();
}

hipError_t launch_impedance(const c128 *E, const c128 *H, int nrec, c128 *Z, hipStream_t s) {
  if (nrec <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_impedance, dim3((nrec + 127) / 128), dim3(128), 0, s, E, H, nrec, Z);
  return hipGetLastError();
}

hipError_t launch_impedance_adjoint(const c128 *E, const c128 *H, int nrec, const c128 *G, c128 *wE,
                                    c128 *wH, hipStream_t s) {
  if (nrec <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_impedance_adjoint, dim3((nrec + 127) / 128), dim3(128), 0, s, E, H, nrec, G,
                     wE, wH);
  return hipGetLastError();
}

hipError_t launch_fields_adjoint(const c128 *K, const c128 *E, const c128 *sa, const c128 *sb_lev,
                                 const int *rec, int nrec, int nrhs, int nx, int ny, int nz,
                                 const c128 *wE, const c128 *wH, c128 *g, double *grad,
                                 hipStream_t s) {
  const size_t N = (size_t)nx * ny * nz;
  hipLaunchKernelGGL(k_fields_adjoint, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, K, E,
                     sa, sb_lev, rec, nrec, nrhs, nx, ny, nz, wE, wH, g, grad);
  return hipGetLastError();
}

// Right-hand side of electric dipoles on the receiver lattice (Sect. 2.1,
// the external current of a point source; Sect. 2.2, the source enters
// through the cell averages of its normal field): by reciprocity of the
// layered medium, G^E(r, r_s) = G^E(r_s, r)^T, so
//   U0[s][c][n] = sqrt(Re sb_n) / V_n sum_a KE(r_s <- n)[a][c] p_s[a],
// with KE the receiver kernel of a receiver at the source point.  One
// thread per (cell, source); neighbouring threads take neighbouring cells.
__global__ void __launch_bounds__(256)
k_dipole_rhs(const c128 *__restrict__ K, const int *__restrict__ src, const c128 *__restrict__ p,
             int nsrc, int nx, int ny, int nz, const double *__restrict__ sroot_lev,
             const double *__restrict__ vol_lev, c128 *__restrict__ out) {
  const size_t plane = (size_t)nx * ny, N = plane * nz;
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int sidx = blockIdx.y;
  if (t >= N || sidx >= nsrc) return;
  const int iz = (int)(t / plane);
  const size_t rem = t - (size_t)iz * plane;
  const int iy = (int)(rem / nx), ix = (int)(rem - (size_t)iy * nx);
  const int is = src[2 * sidx], js = src[2 * sidx + 1];
  const size_t off = (size_t)(js - iy + ny - 1) * (2 * nx - 1) + (is - ix + nx - 1);
  const c128 *k = K + (off * nz + iz) * 18;
  const c128 *ps = p + (size_t)sidx * 3;
  const double f = sroot_lev[iz] / vol_lev[iz];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    c128 acc = mk<double>(0.0, 0.0);
#pragma unroll
    for (int a = 0; a < 3; ++a) cfma(acc, k[3 * a + c], ps[a]);
    out[((size_t)sidx * 3 + c) * N + t] = cscale(acc, f);
  }
}

hipError_t launch_dipole_rhs(const c128 *K, const int *src, const c128 *p, int nsrc, int nx,
                             int ny, int nz, const double *sroot_lev, const double *vol_lev,
                             c128 *out, hipStream_t s) {
  const size_t N = (size_t)nx * ny * nz;
  hipLaunchKernelGGL(k_dipole_rhs, dim3((unsigned)((N + 255) / 256), (unsigned)nsrc), dim3(256), 0,
                     s, K, src, p, nsrc, nx, ny, nz, sroot_lev, vol_lev, out);
  return hipGetLastError();
}

hipError_t launch_assemble_rec(const c128 *c, c128 *out, int noff, int nz, double omega_mu0,
                               hipStream_t s) {
  const int64_t total = (int64_t)noff * nz;
  hipLaunchKernelGGL(k_assemble_rec, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, c,
                     out, noff, nz, omega_mu0);
  return hipGetLastError();
}

hipError_t launch_fields(const c128 *K, const c128 *E, const c128 *sa, const c128 *sb_lev,
                         const int *rec, int nrec, int nrhs, int nx, int ny, int nz,
                         const c128 *en_hn, c128 *Erec, c128 *Hrec, hipStream_t s) {
  if (nrec <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fields, dim3(nrec, nrhs), dim3(256), 0, s, K, E, sa, sb_lev, rec, nrec, nx,
                     ny, nz, en_hn, Erec, Hrec);
  return hipGetLastError();
}

hipError_t launch_gemm_tn(const double *At, int64_t lda, const double *B, int64_t ldb, double *C,
                          int64_t ldc, int m, int n, int k, hipStream_t s, const int *krange) {
  if (m <= 0 || n <= 0) return hipSuccess;
  dim3 grid((n + 63) / 64, (m + 63) / 64);
  if (grid.y > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_gemm_tn, grid, dim3(256), 0, s, At, lda, B, ldb, C, ldc, m, n, k, krange);
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
