// Step 2 of the three-step apply (Sect. 3.3): the Nz-order block products
// with the stored spectra of the packed table.
//
// For every frequency point K of the 2Nx x 2Ny grid,
//   Y^(K) = Q~(K) X^(K),   Q~(K) the 3Nz x 3Nz matrix of 3 x 3 Nz-blocks.
// Q~ is stored once per representative (Kx, Ky), 0 <= Kx <= Nx, 0 <= Ky <= Ny
// (the transform keeps the parities of Lemma 2).  A mirrored point (2Nx - Kx
// or 2Ny - Ky) uses Q~_ab t_a t_b with t = (-1, 1, 1) for an x mirror and
// (1, -1, 1) for a y mirror, i.e. Y = T Q~ T X: the sign flips are applied to
// the loaded vectors and to the results, so one read of the packed block
// serves the up to four mirror points and all R right-hand sides.  Lemma 1
// gives the blocks that are not stored: yx = xy, zx = -xz^T, zy = -yz^T; xx,
// xy, yy, zz are read from their upper triangles.
//
// The product at one representative point is a dense contraction
//   [Yr | Yi] (3Nz x 16) = [Qr | Qi] (3Nz x 6Nz) [[Xr | Xi]; [-Xi | Xr]]
// over up to 8 complex vectors (mirrors x RHS) per pass, done with 16x16x4
// MFMA tiles (FP64 or FP32): one wavefront per 16 output rows, separate
// accumulators for the real and the imaginary part of Q.
//
// One workgroup per representative point.  The vectors are staged in LDS;
// the MFMA A fragments are gathered straight from the packed block in global
// memory (a symmetric entry serves two rows, its second read hits the L2), so
// that the small LDS footprint lets many workgroups share a CU.
#include <algorithm>
#include <vector>

#include "kernels.h"

namespace giem {

template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
  typedef double acc_t __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // row (within the 16-row tile) held by accumulator register q of a lane
  static __device__ __forceinline__ int row(int lane, int q) { return (lane >> 4) + 4 * q; }
};
template <>
struct Mfma<float> {
  typedef float acc_t __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int q) { return 4 * (lane >> 4) + q; }
};

// Mirror points of a representative (kxr, kyr): the point itself, then its
// x mirror, its y mirror and the xy mirror when they are distinct points.
// Coordinates are computed from the index (no local arrays, which would
// live in scratch memory).
struct MirrorSet {
  int kxr, kyr, n;
  bool mx, my;
};

__device__ __forceinline__ MirrorSet mirror_set(int rep, int nx, int ny) {
  MirrorSet m;
  m.kxr = rep % (nx + 1);
  m.kyr = rep / (nx + 1);
  m.mx = (m.kxr != 0 && m.kxr != nx);
  m.my = (m.kyr != 0 && m.kyr != ny);
  m.n = (m.mx ? 2 : 1) * (m.my ? 2 : 1);
  return m;
}

// point index (Ky * 2Nx + Kx) and component signs of mirror mi
__device__ __forceinline__ void mirror_of(const MirrorSet &m, int mi, int nx, int ny, int &pt,
                                          bool &fx, bool &fy) {
  fx = m.mx && (mi & 1);
  fy = m.my && (m.mx ? (mi >> 1) : (mi & 1));
  const int kx = fx ? 2 * nx - m.kxr : m.kxr;
  const int ky = fy ? 2 * ny - m.kyr : m.kyr;
  pt = ky * 2 * nx + kx;
}

// Gather plan: for tile t, k-step s and lane l (row r = 16 t + l % 16,
// column c = 4 s + l / 16) one word holds the packed offset of Q[r][c] (low
// 24 bits), its sign (bit 24, Lemma 1 transposes), validity (bit 25) and the
// component beta of column c (bits 26-27, for the mirror flips of X).  The
// plan depends on Nz only and is shared by every frequency point.
__host__ __device__ inline unsigned plan_word(int nz, int r, int c) {
  const int tri = nz * (nz + 1) / 2, p3 = 3 * nz;
  if (r >= p3 || c >= p3) return 0u;
  const int a = r / nz, iz = r - a * nz, b = c / nz, jz = c - b * nz;
  const int blk = a * 3 + b;
  const bool trans = (blk == 6) || (blk == 7);
  const bool full = (blk == 2) || (blk == 5) || trans;
  const bool second = (blk == 5) || (blk == 7);
  int idx;
  if (full) {
    const int row = trans ? jz : iz, col = trans ? iz : jz;
    idx = 4 * tri + (second ? nz * nz : 0) + row * nz + col;
  } else {
    const int lo = iz < jz ? iz : jz, hi = iz < jz ? jz : iz;
    const int base = (blk == 0) ? 0 : (blk == 4) ? 2 * tri : (blk == 8) ? 3 * tri : tri;
    idx = base + lo * nz - (lo * (lo - 1)) / 2 + (hi - lo);
  }
  return (unsigned)idx | (trans ? (1u << 24) : 0u) | (1u << 25) | ((unsigned)b << 26);
}

// One wavefront per (representative point, 16-row tile of the output); no
// LDS and no barriers: the wave gathers its A fragments from the packed block
// and its B fragments from the input spectra (with the mirror sign flips), and
// writes its rows of the output spectra, which live in a second buffer.
template <typename T>
__global__ void __launch_bounds__(256)
k_block(const cplx<T> *__restrict__ tab, const cplx<T> *__restrict__ sin,
        cplx<T> *__restrict__ sout, const unsigned *__restrict__ plan, int nx, int ny, int nz,
        int R) {
  typedef Mfma<T> M;
  const int E = 2 * nz * (2 * nz + 1);
  const int p3 = 3 * nz;
  const int nsteps = (p3 + 3) >> 2;
  const int ntiles = (p3 + 15) >> 4;
  const int npts = (nx + 1) * (ny + 1);
  const int gw = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);  // global wave
  const int rep = gw / ntiles, tile = gw - rep * ntiles;
  if (rep >= npts) return;  // whole wave exits together
  const int lane = threadIdx.x & 63;
  const MirrorSet m = mirror_set(rep, nx, ny);
  const int V = m.n * R;
  const cplx<T> *tq = tab + (size_t)rep * E;
  const unsigned *pl = plan + (size_t)tile * nsteps * 64 + lane;
  const int kk = lane >> 4;
  const int j = lane & 15;
  const int vloc = j & 7, part = j >> 3;
  for (int vg = 0; vg < V; vg += 8) {
    const int v = vg + vloc;
    const bool vvalid = v < V;
    int pt = 0;
    bool fx = false, fy = false;
    const int mi = vvalid ? v / R : 0, rr = vvalid ? v - mi * R : 0;
    mirror_of(m, mi, nx, ny, pt, fx, fy);
    const cplx<T> *xb = sin + ((size_t)pt * R + rr) * p3;
    typename M::acc_t accr = {0, 0, 0, 0}, acci = {0, 0, 0, 0};
    constexpr int U = 8;  // k-steps whose operands are requested ahead
    for (int s0 = 0; s0 < nsteps; s0 += U) {
      cplx<T> q[U], x[U];
      unsigned w[U];
#pragma unroll
      for (int u = 0; u < U; ++u) w[u] = (s0 + u < nsteps) ? pl[(s0 + u) * 64] : 0u;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int c = 4 * (s0 + u) + kk;
        const bool ok = (w[u] >> 25) & 1u;
        q[u] = tq[ok ? (w[u] & 0xffffffu) : 0];
        x[u] = xb[c < p3 ? c : 0];  // B[c][j] does not depend on the lane's A row
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const bool ok = (w[u] >> 25) & 1u;
        const T qs_ = ((w[u] >> 24) & 1u) ? (T)-1 : (T)1;
        const T qr = ok ? qs_ * q[u].x : (T)0;
        const T qim = ok ? qs_ * q[u].y : (T)0;
        const int cc = 4 * (s0 + u) + kk;
        const unsigned cb = (unsigned)(cc / nz);
        const bool xn = (cb == 0u && fx) || (cb == 1u && fy);
        const bool xok = vvalid && cc < p3;
        const T xs_ = xn ? (T)-1 : (T)1;
        const T xr = xok ? xs_ * x[u].x : (T)0;
        const T xi = xok ? xs_ * x[u].y : (T)0;
        const T b1 = part ? xi : xr;
        const T b2 = part ? xr : -xi;
        accr = M::mma(qr, b1, accr);
        acci = M::mma(qim, b2, acci);
      }
    }
    if (vvalid) {
      T *ob = reinterpret_cast<T *>(sout + ((size_t)pt * R + rr) * p3);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = tile * 16 + M::row(lane, q);
        if (row < p3) {
          const int a = row / nz;
          const T sg = ((a == 0 && fx) || (a == 1 && fy)) ? (T)-1 : (T)1;
          ob[2 * row + part] = sg * (accr[q] + acci[q]);
        }
      }
    }
  }
}

int block_threads(int nz, int R) {
  (void)nz;
  (void)R;
  return 256;
}

size_t block_lds_bytes(int nz, int R, int prec) {
  (void)nz;
  (void)R;
  (void)prec;
  return 0;
}

bool block_supported(int nz, int R) { return nz >= 1 && 2 * nz * (2 * nz + 1) < (1 << 24) && R >= 1 && R <= kMaxRhs; }

std::vector<unsigned> block_plan(int nz) {
  const int p3 = 3 * nz, nsteps = (p3 + 3) / 4, ntiles = (p3 + 15) / 16;
  std::vector<unsigned> w((size_t)ntiles * nsteps * 64);
  for (int t = 0; t < ntiles; ++t)
    for (int st = 0; st < nsteps; ++st)
      for (int l = 0; l < 64; ++l)
        w[((size_t)t * nsteps + st) * 64 + l] = plan_word(nz, 16 * t + (l & 15), 4 * st + (l >> 4));
  return w;
}

template <typename T>
static hipError_t launch_block_t(const void *tab, const void *sin, void *sout,
                                 const unsigned *plan, int nx, int ny, int nz, int R,
                                 hipStream_t s) {
  const int ntiles = (3 * nz + 15) / 16;
  const long long waves = (long long)(nx + 1) * (ny + 1) * ntiles;
  const int per_block = 4;
  const long long grid = (waves + per_block - 1) / per_block;
  k_block<T><<<(unsigned)grid, 64 * per_block, 0, s>>>(
      static_cast<const cplx<T> *>(tab), static_cast<const cplx<T> *>(sin),
      static_cast<cplx<T> *>(sout), plan, nx, ny, nz, R);
  return hipGetLastError();
}

hipError_t launch_block(int prec, const void *tab, const void *sin, void *sout,
                        const unsigned *plan, int nx, int ny, int nz, int R, hipStream_t s) {
  return prec == PREC_FP32 ? launch_block_t<float>(tab, sin, sout, plan, nx, ny, nz, R, s)
                           : launch_block_t<double>(tab, sin, sout, plan, nx, ny, nz, R, s);
}

}  // namespace giem
