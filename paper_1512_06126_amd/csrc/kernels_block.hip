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
// MFMA tiles (FP64 or FP32), two accumulators (real and imaginary part of Q).
//
// k_block_pipe (Nz <= 32): one persistent workgroup per CU stages a point's
// packed row (2Nz(2Nz+1) complex, 66.5 KB for Nz = 32 in FP64) in LDS with
// coalesced loads, so every table byte crosses HBM once, while the next
// point's row is in flight into registers; 12 wavefronts (two per 16-row
// tile, each half of the contraction) run the MFMAs from LDS.
//
// k_block_band (rows and input vectors that outgrow LDS: Nz > 32 at R = 2):
// one workgroup per point stages the packed row by pairs of 16-level bands,
// each entry once, and keeps the output tiles' accumulators in its
// wavefronts.
//
// Several frequencies can share one launch: the spectra of all their vectors
// are transformed together, a point's record holds nf R vectors (frequency
// f's at f R .. f R + R - 1) and each (frequency, point) pair reads its own
// table.
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

// Block product for rows too long for LDS (Nz > 32 at R = 2): one workgroup
// per (frequency, representative point), 8 wavefronts in FP32, 16 in FP64.  The 3Nz x 3Nz
// matrix is visited by pairs (I, J), I <= J, of 16-level bands: the
// workgroup stages every packed entry with one level in band I and the other
// in band J into LDS (the I-rows, J-columns tile of the four symmetric
// blocks xx, xy, yy, zz; the (I, J) and (J, I) tiles of xz and yz), each
// entry once per point, with 128-byte and longer runs, and applies it to the
// output bands I and J: yx = xy, and the symmetric blocks' (J, I) tiles are
// the transposes; zx = -xz^T, zy = -yz^T (Lemma 1).  Output tile (alpha,
// band) belongs to wavefront (3 band + alpha) mod NW, which keeps its
// accumulators over all pairs (the six tiles of a pair fall on different
// wavefronts where they can).  The next pair's entries are loaded into
// registers while the current pair's MFMAs run.  Slots of the staged tiles:
// 0 xx, 1 xy, 2 yy, 3 zz (I rows, J columns), 4 xz(I, J), 5 xz(J, I),
// 6 yz(I, J), 7 yz(J, I); rows padded to 17 entries.
constexpr int kBandLd = 17, kBandSlot = 16 * kBandLd;

template <typename T>
__device__ __forceinline__ cplx<T> band_entry(const cplx<T> *__restrict__ tq, int q, int I, int J,
                                              int nz, int tri) {
  const int slot = q >> 8, r = (q >> 4) & 15, c = q & 15;
  const bool swap = slot == 5 || slot == 7;  // the (J, I) tiles
  const int iz = (swap ? J : I) * 16 + r, jz = (swap ? I : J) * 16 + c;
  bool ok = iz < nz && jz < nz && !(swap && I == J);
  int idx;
  if (slot < 4) {
    ok = ok && jz >= iz;
    idx = slot * tri + iz * nz - (iz * (iz - 1)) / 2 + (jz - iz);
  } else {
    idx = 4 * tri + (slot >= 6 ? nz * nz : 0) + iz * nz + jz;
  }
  return ok ? tq[ok ? idx : 0] : mk<T>(0, 0);
}

// pairs (I, J), I <= J, in the order (0, 0), (0, 1), ..., (0, nb - 1), (1, 1), ...
__device__ __forceinline__ void band_next(int &I, int &J, int nb) {
  if (J + 1 < nb) {
    ++J;
  } else {
    ++I;
    J = I;
  }
}

template <typename T, int NT, int NPRE>
__device__ __forceinline__ void band_store(cplx<T> *buf, const cplx<T> (&pre)[NPRE], int tid) {
#pragma unroll
  for (int u = 0; u < NPRE; ++u) {
    const int q = tid + NT * u;
    if (NT * NPRE == 2048 || q < 2048)
      buf[(q >> 8) * kBandSlot + ((q >> 4) & 15) * kBandLd + (q & 15)] = pre[u];
  }
}

// NW wavefronts per workgroup, MAXT output tiles per wavefront
template <typename T, int MAXT, int KB, int WPE, int NW>
__global__ void __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(WPE)))
k_block_band(TabSet tabs, const cplx<T> *__restrict__ sin, cplx<T> *__restrict__ sout, int nx,
             int ny, int nz, int R, int nf) {
  typedef Mfma<T> M;
  extern __shared__ unsigned char smem_raw[];
  const int nb = (nz + 15) >> 4;
  cplx<T> *Xs = reinterpret_cast<cplx<T> *>(smem_raw);  // [3][16 nb][8]
  cplx<T> *Ts = Xs + 3 * nb * 16 * 8;                     // [8][16][17]
  const int E = 2 * nz * (2 * nz + 1), tri = nz * (nz + 1) / 2, p3 = 3 * nz;
  const int npairs = nb * (nb + 1) / 2;
  const int npts = (nx + 1) * (ny + 1);
  const int f = blockIdx.x / npts, rep = blockIdx.x - f * npts;
  const int rtot = nf * R;
  // threads, staged entries per thread (8 slots of 16 x 16)
  constexpr int NT = 64 * NW, NPRE = (2048 + NT - 1) / NT;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, kk = lane >> 4;
  const int vloc = li & 7, part = li >> 3;
  const MirrorSet m = mirror_set(rep, nx, ny);
  const int V = m.n * R;
  const cplx<T> *tq = static_cast<const cplx<T> *>(tabs.tab[f]) + (size_t)rep * E;
  for (int vg = 0; vg < V; vg += 8) {
    __syncthreads();  // the previous vector group's reads of Xs are done
    // Xs[(beta nb 16 + jz) 8 + v]: levels jz in [Nz, 16 nb) hold zeros
    for (int idx = tid; idx < 8 * 3 * nb * 16; idx += NT) {
      const int v = idx / (3 * nb * 16), cc = idx - v * (3 * nb * 16);
      const int b = cc / (nb * 16), jz = cc - b * (nb * 16), c = b * nz + jz;
      cplx<T> val = mk<T>(0, 0);
      if (vg + v < V && jz < nz) {
        const int mi = (vg + v) / R, rr = vg + v - mi * R;
        int pt;
        bool fx, fy;
        mirror_of(m, mi, nx, ny, pt, fx, fy);
        val = sin[((size_t)pt * rtot + f * R + rr) * p3 + c];
        if ((b == 0 && fx) || (b == 1 && fy)) val = mk<T>(-val.x, -val.y);
      }
      Xs[cc * 8 + v] = val;
    }
    typename M::acc_t accr[MAXT], acci[MAXT];
#pragma unroll
    for (int s = 0; s < MAXT; ++s) accr[s] = acci[s] = typename M::acc_t{0, 0, 0, 0};
    // the next pair's entries are loaded into registers during the current
    // pair's MFMAs
    cplx<T> pre[NPRE];
    int I = 0, J = 0, Ip = 0, Jp = 0;  // current pair, last pair requested
#pragma unroll
    for (int u = 0; u < NPRE; ++u)
      pre[u] = tid + NT * u < 2048 ? band_entry(tq, tid + NT * u, 0, 0, nz, tri) : mk<T>(0, 0);
    for (int p = 0; p < npairs; ++p) {
      __syncthreads();  // the previous pair's tiles are no longer read
      band_store<T, NT, NPRE>(Ts, pre, tid);
      if (p + 1 < npairs) {
        band_next(Ip, Jp, nb);
#pragma unroll
        for (int u = 0; u < NPRE; ++u)
          pre[u] = tid + NT * u < 2048 ? band_entry(tq, tid + NT * u, Ip, Jp, nz, tri) : mk<T>(0, 0);
      }
      __syncthreads();
      const cplx<T> *Tc = Ts;
#pragma unroll
      for (int s = 0; s < MAXT; ++s) {
        const int o = w + NW * s;
        if (o >= 3 * nb) continue;
        const int band = o / 3, a = o - 3 * band;
#pragma unroll 1
        for (int side = 0; side < 2; ++side) {
          // side 0: output band I from input band J; side 1: output band J
          // from input band I (I < J only)
          if (side == 0 ? band != I : (band != J || I == J)) continue;
          const bool obI = side == 0;
          const int ib = obI ? J : I;
#pragma unroll 1
          for (int b = 0; b < 3; ++b) {
            const bool sym = (a < 2 && b < 2) || (a == 2 && b == 2);
            int slot;
            bool tr;
            T sg = (T)1;
            if (sym) {
              slot = a == 2 ? 3 : a + b;
            } else if (b == 2) {
              slot = (a == 0 ? 4 : 6) + (obI ? 0 : 1);
            } else {
              slot = (b == 0 ? 4 : 6) + ((obI && I != J) ? 1 : 0);
              sg = (T)-1;
            }
            // KB k-steps' fragments are read before any MFMA uses them (no
            // conditional reads: Xs is zero past level Nz)
#pragma unroll
            for (int k0 = 0; k0 < 4; k0 += KB) {
              cplx<T> qv[KB], xv[KB];
#pragma unroll
              for (int u = 0; u < KB; ++u) {
                const int kl = 4 * (k0 + u) + kk;
                if (sym) tr = (I == J) ? (li > kl) : !obI;
                else tr = b != 2;
                qv[u] = Tc[slot * kBandSlot + (tr ? kl * kBandLd + li : li * kBandLd + kl)];
                xv[u] = Xs[((b * nb + ib) * 16 + kl) * 8 + vloc];
              }
              __builtin_amdgcn_sched_barrier(0);  // keep the reads ahead of the MFMAs
#pragma unroll
              for (int u = 0; u < KB; ++u) {
                const T b1 = part ? xv[u].y : xv[u].x;
                const T b2 = part ? xv[u].x : -xv[u].y;
                accr[s] = M::mma(sg * qv[u].x, b1, accr[s]);
                acci[s] = M::mma(sg * qv[u].y, b2, acci[s]);
              }
            }
          }
        }
      }
      band_next(I, J, nb);
    }
    const int v = vg + vloc;
    if (v < V) {
      const int mi = v / R, rr = v - mi * R;
      int pt;
      bool fx, fy;
      mirror_of(m, mi, nx, ny, pt, fx, fy);
      T *ob = reinterpret_cast<T *>(sout + ((size_t)pt * rtot + f * R + rr) * p3);
#pragma unroll
      for (int s = 0; s < MAXT; ++s) {
        const int o = w + NW * s;
        if (o >= 3 * nb) continue;
        const int band = o / 3, a = o - 3 * band;
        const T sgo = ((a == 0 && fx) || (a == 1 && fy)) ? (T)-1 : (T)1;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int iz = band * 16 + M::row(lane, q);
          if (iz < nz) ob[2 * (a * nz + iz) + part] = sgo * (accr[s][q] + acci[s][q]);
        }
      }
    }
  }
}

// The variants launched: (T, output tiles per wavefront, fragment batch,
// wavefronts per SIMD, wavefronts per workgroup).  FP32: 8 wavefronts of 3
// tiles up to 8 bands (two workgroups per CU), 16 of 3 beyond; FP64: 16 of 2
// up to 10 bands (four wavefronts per SIMD), 12 of 3 at 11 (170 VGPRs, three
// per SIMD)
template <typename T, int MAXT, int KB, int WPE, int NW>
static const void *band_kernel() {
  return reinterpret_cast<const void *>(k_block_band<T, MAXT, KB, WPE, NW>);
}

static size_t lds_bytes_band(int nz, size_t csize) {
  return ((size_t)3 * ((nz + 15) / 16) * 16 * 8 + 8 * (size_t)kBandSlot) * csize;
}

// LDS offset and sign of Q[row][col] (row = alpha Nz + iz, col = beta Nz +
// jz).  The staged row keeps the storage of Sect. 3.1 (upper triangles of
// xx, xy, yy, zz, then xz and yz), but the rows of the two full blocks are
// padded to Nz + 1 entries so that the 16 lanes of a fragment, which read 16
// consecutive rows of one column, fall into different LDS banks.  Lemma 1
// gives yx = xy, zx = -xz^T, zy = -yz^T.
__device__ __forceinline__ int staged_index(int a, int iz, int b, int jz, int nz, int tri,
                                            bool &neg) {
  const bool full = (a == 2) != (b == 2);
  const int lo = iz < jz ? iz : jz, hi = iz < jz ? jz : iz;
  const int sbase = (a == 2) ? 3 * tri : (a + b == 0) ? 0 : (a + b == 1) ? tri : 2 * tri;
  const int sidx = sbase + lo * nz - (lo * (lo - 1)) / 2 + (hi - lo);
  const int frow = (a == 2) ? jz : iz, fcol = (a == 2) ? iz : jz;
  const int fblk = (a == 1 || b == 1) ? nz : 0;
  const int fidx = 4 * tri + (fblk + frow) * (nz + 1) + fcol;
  neg = full && a == 2;
  return full ? fidx : sidx;
}

__device__ __forceinline__ int staged_of_packed(int e, int nz, int tri) {
  if (e < 4 * tri) return e;
  const int f = e - 4 * tri, r = f / nz;
  return 4 * tri + r * (nz + 1) + (f - r * nz);
}

// entries of the packed row and of the input vectors that a thread carries
// ahead in registers (the next point's data, loaded during the MFMAs)
constexpr int kStageRegs = 6;   // 12 wavefronts (KS = 2)
constexpr int kStageRegs1 = 11; // 6 wavefronts (KS = 1)
constexpr int kXRegs = 2;
// k-steps of 4 columns per wavefront (half of 3 Nz, rounded up)
constexpr int kMaxHalfSteps = 16;

// Workgroup barrier that waits only for this wave's LDS operations: the
// prefetch loads into registers stay in flight across it (__syncthreads()
// would also wait for them).  Global memory is not shared between the
// wavefronts here, so LDS ordering is all the barrier has to provide.
__device__ __forceinline__ void lds_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

__device__ __forceinline__ double flip_sign(double x, unsigned m) {
  return __hiloint2double(__double2hiint(x) ^ (int)m, __double2loint(x));
}
__device__ __forceinline__ float flip_sign(float x, unsigned m) {
  return __int_as_float(__float_as_int(x) ^ (int)m);
}

// Software-pipelined block product.  Each persistent workgroup takes the
// tasks g, g + grid, ... of the nf x (Nx + 1)(Ny + 1) (frequency,
// representative point) pairs; it holds one task's packed row and input
// vectors in LDS while the next task's are in flight into registers.
//   KS = 2: one workgroup per CU; two wavefronts per 16-row output tile split
//   the contraction into halves (split-k) and add them through LDS, so
//   2 x ceil(3Nz/16) wavefronts (12 for Nz = 32) keep the four SIMDs' matrix
//   cores busy.
//   KS = 1: two workgroups per CU, one wavefront per tile doing the whole
//   contraction (no reduction buffer, no barrier between column tiles), so
//   that one workgroup's MFMAs overlap the other's staging and stores.
// The LDS offsets of a lane's A fragments and the Lemma 1 signs (bit 15 of
// each 16-bit entry) do not depend on the point and are computed once.  The
// input vectors are staged as real B fragments: row c holds
// [Re X_0..7 | Im X_0..7]; the second operand [-Im | Re] is the same row read
// with its halves swapped and the sign of the first half flipped.
template <typename T, int NS, bool MF, int KS>
__global__ void __launch_bounds__(768) __attribute__((amdgpu_waves_per_eu(3, 3)))
k_block_pipe1(TabSet tabs, const cplx<T> *__restrict__ sin, cplx<T> *__restrict__ sout, int nx,
              int ny, int nz, int R, int nct, int nf) {
  typedef Mfma<T> M;
  typedef T v2 __attribute__((ext_vector_type(2)));
  constexpr int HS = NS / KS;  // k-steps per wavefront
  constexpr int SR = KS == 2 ? kStageRegs : kStageRegs1;  // packed entries per thread
  constexpr int kpad = 4 * NS;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const int E = 2 * nz * (2 * nz + 1);
  const int Es = E + 2 * nz;  // padded rows of the full blocks; entry Es is zero
  const int p3 = 3 * nz, tri = nz * (nz + 1) / 2;
  const int nrt = (p3 + 15) >> 4;
  v2 *Qv = reinterpret_cast<v2 *>(lds_raw);
  T *Bs = reinterpret_cast<T *>(Qv + Es + 2);          // [nct][kpad][16]
  T *Red = Bs + (size_t)nct * kpad * 16;  // [nrt][4][64] partial sums (KS = 2)
  const int npts = (nx + 1) * (ny + 1);
  // tasks: (frequency, representative point) pairs when the launch serves
  // several frequencies (MF), else the points of the one table, whose
  // pointer is then read once
  const int ntask = MF ? nf * npts : npts;
  const int rtot = MF ? nf * R : R;  // vectors per point record of the spectra
  const v2 *tab0 = reinterpret_cast<const v2 *>(tabs.tab[0]);
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int kk0 = lane >> 4, j = lane & 15, part = j >> 3;
  const int rt = wave % nrt, kh = KS == 2 ? wave / nrt : 0;  // output tile, contraction half
  const unsigned bmask = part ? 0u : 0x80000000u;
  unsigned aoff[(HS + 1) / 2];
  {
    const int row = rt * 16 + (lane & 15);
    const bool rowok = row < p3;
    const int a = rowok ? row / nz : 0, iz = rowok ? row - a * nz : 0;
#pragma unroll
    for (int u = 0; u < HS; ++u) {
      const int c = 4 * (kh * HS + u) + kk0;
      unsigned w = (unsigned)Es;
      if (rowok && c < p3) {
        const int b = c / nz, jz = c - b * nz;
        bool neg;
        w = (unsigned)staged_index(a, iz, b, jz, nz, tri, neg) | (neg ? 0x8000u : 0u);
      }
      if (u & 1)
        aoff[u >> 1] |= w << 16;
      else
        aoff[u >> 1] = w;
    }
  }
  if (tid == 0) Qv[Es] = v2{(T)0, (T)0};
  const int nxe = nct * 8 * kpad;  // input-vector elements (c, v)
  // point-independent staging maps of this thread: LDS slot of each packed
  // entry it carries; column v, row c (component b) and RHS of each input
  // element, and its place in the B rows
  int tdst[SR];
#pragma unroll
  for (int u = 0; u < SR; ++u) {
    const int e = tid + u * nthr;
    tdst[u] = e < E ? staged_of_packed(e, nz, tri) : -1;
  }
  int xv_[kXRegs], xc_[kXRegs], xmi_[kXRegs], xr_[kXRegs], xb_[kXRegs], xdst_[kXRegs];
#pragma unroll
  for (int u = 0; u < kXRegs; ++u) {
    const int idx = u * nthr + tid;
    const int v = idx < nxe ? idx / kpad : 1 << 20, c = idx < nxe ? idx - v * kpad : 0;
    xv_[u] = v;
    xc_[u] = c < p3 ? c : 0;
    xmi_[u] = idx < nxe ? v / R : 0;
    xr_[u] = idx < nxe ? v - (v / R) * R : 0;
    xb_[u] = c < p3 ? c / nz : 3;  // 3: padding row
    xdst_[u] = idx < nxe ? ((v >> 3) * kpad + c) * 16 + (v & 7) : -1;
  }
  v2 pre[SR];
  cplx<T> xpre[kXRegs];
  unsigned xneg = 0;  // mirror sign of each prefetched input element
  unsigned xval = 0;  // which prefetched input elements are real (else zero)
  // loads of one point's row and input vectors into the prefetch registers
  auto prefetch = [&](int task_) __attribute__((always_inline)) {
    const int f_ = MF ? task_ / npts : 0, rep_ = task_ - f_ * npts;
    const v2 *src = (MF ? reinterpret_cast<const v2 *>(tabs.tab[f_]) : tab0) + (size_t)rep_ * E;
#pragma unroll
    for (int u = 0; u < SR; ++u)
      if (tdst[u] >= 0) pre[u] = src[tid + u * nthr];
    const MirrorSet m = mirror_set(rep_, nx, ny);
    const int V = m.n * R;
    // the sign is applied when the element is written to LDS, so that no
    // instruction here waits for the loads
    // (every element is loaded, from a clamped address when it is padding,
    // so that no register is written between the loads and their use)
    xneg = 0;
    xval = 0;
#pragma unroll
    for (int u = 0; u < kXRegs; ++u) {
      const bool ok = xv_[u] < V && xb_[u] < 3;
      int pt;
      bool fx, fy;
      mirror_of(m, ok ? xmi_[u] : 0, nx, ny, pt, fx, fy);
      xpre[u] = sin[((size_t)pt * rtot + f_ * R + (ok ? xr_[u] : 0)) * p3 + xc_[u]];
      if (ok && ((xb_[u] == 0 && fx) || (xb_[u] == 1 && fy))) xneg |= 1u << u;
      if (ok) xval |= 1u << u;
    }
  };
  int task = blockIdx.x;
  if (task < ntask) prefetch(task);
  for (; task < ntask; task += gridDim.x) {
    const int f = MF ? task / npts : 0, rep = task - f * npts;
    lds_barrier();  // every wavefront is done with the previous point
#pragma unroll
    for (int u = 0; u < SR; ++u)
      if (tdst[u] >= 0) Qv[tdst[u]] = pre[u];
#pragma unroll
    for (int u = 0; u < kXRegs; ++u) {
      if (xdst_[u] >= 0) {
        T *brow = Bs + xdst_[u];
        const unsigned sm = ((xneg >> u) & 1u) ? 0x80000000u : 0u;
        const bool ok = (xval >> u) & 1u;
        brow[0] = ok ? flip_sign(xpre[u].x, sm) : (T)0;
        brow[8] = ok ? flip_sign(xpre[u].y, sm) : (T)0;
      }
    }
    const MirrorSet m = mirror_set(rep, nx, ny);
    const int V = m.n * R;
    // the next point's loads are issued one per k-step of the first column
    // tile below, so that waiting for queue space overlaps the MFMAs
    const int ntk = task + (int)gridDim.x;
    const bool more = ntk < ntask;
    const int fnx = MF ? (more ? ntk : task) / npts : 0;
    const int nrep = (more ? ntk : task) - fnx * npts;
    const v2 *nsrc = (MF ? reinterpret_cast<const v2 *>(tabs.tab[fnx]) : tab0) + (size_t)nrep * E;
    int xaddr[kXRegs];
    {
      const MirrorSet mn = mirror_set(nrep, nx, ny);
      const int Vn = mn.n * R;
      xneg = 0;
      xval = 0;
#pragma unroll
      for (int u = 0; u < kXRegs; ++u) {
        const bool ok = xv_[u] < Vn && xb_[u] < 3;
        int pt;
        bool fx, fy;
        mirror_of(mn, ok ? xmi_[u] : 0, nx, ny, pt, fx, fy);
        xaddr[u] = (pt * rtot + fnx * R + (ok ? xr_[u] : 0)) * p3 + xc_[u];
        if (ok && ((xb_[u] == 0 && fx) || (xb_[u] == 1 && fy))) xneg |= 1u << u;
        if (ok) xval |= 1u << u;
      }
    }
    lds_barrier();
    for (int ct = 0; ct * 8 < V; ++ct) {
      typename M::acc_t accr = {0, 0, 0, 0}, acci = {0, 0, 0, 0};
      const int kb = kh * HS * 4 + kk0;  // first B row of this half
      const T *b1p = Bs + ((size_t)ct * kpad + kb) * 16 + j;
      const T *b2p = Bs + ((size_t)ct * kpad + kb) * 16 + (j ^ 8);
#pragma unroll
      for (int u = 0; u < HS; ++u) {
        if (ct == 0 && more) {
          // prefetch slot u: packed entries first, then input elements
          if (u < SR) {
            if (tdst[u] >= 0) pre[u] = nsrc[tid + u * nthr];
          } else if (u - SR < kXRegs) {
            xpre[u - SR] = sin[xaddr[u - SR]];
          }
        }
        unsigned pw = aoff[u >> 1];
        // KS = 1: decode at the use (an opaque copy), so that the decoded
        // offsets and signs of all HS k-steps are not held in registers
        if constexpr (KS == 1) asm volatile("" : "+v"(pw));
        const unsigned w = (u & 1) ? (pw >> 16) : (pw & 0xffffu);
        const v2 q = Qv[w & 0x7fffu];
        const unsigned qm = (w & 0x8000u) << 16;
        const T b1 = b1p[u * 64];
        const T b2 = flip_sign(b2p[u * 64], bmask);
        accr = M::mma(flip_sign(q.x, qm), b1, accr);
        acci = M::mma(flip_sign(q.y, qm), b2, acci);
      }
      if (ct == 0 && more) {
#pragma unroll
        for (int u = HS; u < SR + kXRegs; ++u) {
          if (u < SR) {
            if (tdst[u] >= 0) pre[u] = nsrc[tid + u * nthr];
          } else {
            xpre[u - SR] = sin[xaddr[u - SR]];
          }
        }
      }
      if (KS == 2) {
        if (kh == 1) {
#pragma unroll
          for (int qq = 0; qq < 4; ++qq) Red[(rt * 4 + qq) * 64 + lane] = accr[qq] + acci[qq];
        }
        lds_barrier();
      }
      if (kh == 0) {
        const int v = ct * 8 + (j & 7);
        if (v < V) {
          const int mi = v / R, r = v - mi * R;
          int pt;
          bool fx, fy;
          mirror_of(m, mi, nx, ny, pt, fx, fy);
          T *ob = reinterpret_cast<T *>(sout + ((size_t)pt * rtot + f * R + r) * p3);
#pragma unroll
          for (int qq = 0; qq < 4; ++qq) {
            const int orow = rt * 16 + M::row(lane, qq);
            if (orow < p3) {
              const int oa = orow / nz;
              const T sg = ((oa == 0 && fx) || (oa == 1 && fy)) ? (T)-1 : (T)1;
              const T red = KS == 2 ? Red[(rt * 4 + qq) * 64 + lane] : (T)0;
              ob[2 * orow + part] = sg * (accr[qq] + acci[qq] + red);
            }
          }
        }
      }
      if (KS == 2) lds_barrier();  // Red is reused by the next column tile
    }
  }
}


// The same with NB register sets of prefetched points (used with NB = 2):
// the loads of point p + 2 grid are in flight while point p + grid is staged
// into LDS, so the memory pipe does not idle during staging.  It takes more
// registers, so the one-set kernel above is kept and the faster of the two
// is chosen per handle and precision (giem_tune).
template <typename T, int NS, int NB, bool MF>
__global__ void __launch_bounds__(768) __attribute__((amdgpu_waves_per_eu(3, 3)))
k_block_pipe(TabSet tabs, const cplx<T> *__restrict__ sin, cplx<T> *__restrict__ sout, int nx,
             int ny, int nz, int R, int nct, int nf) {
  typedef Mfma<T> M;
  typedef T v2 __attribute__((ext_vector_type(2)));
  constexpr int HS = NS / 2;  // k-steps per half
  constexpr int kpad = 4 * NS;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const int E = 2 * nz * (2 * nz + 1);
  const int Es = E + 2 * nz;  // padded rows of the full blocks; entry Es is zero
  const int p3 = 3 * nz, tri = nz * (nz + 1) / 2;
  const int nrt = (p3 + 15) >> 4;
  v2 *Qv = reinterpret_cast<v2 *>(lds_raw);
  T *Bs = reinterpret_cast<T *>(Qv + Es + 2);          // [nct][kpad][16]
  T *Red = Bs + (size_t)nct * kpad * 16;                 // [nrt][4][64] partial sums
  const int npts = (nx + 1) * (ny + 1);
  // tasks: (frequency, representative point) pairs when the launch serves
  // several frequencies (MF), else the points of the one table, whose
  // pointer is then read once
  const int ntask = MF ? nf * npts : npts;
  const int rtot = MF ? nf * R : R;  // vectors per point record of the spectra
  const v2 *tab0 = reinterpret_cast<const v2 *>(tabs.tab[0]);
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int kk0 = lane >> 4, j = lane & 15, part = j >> 3;
  const int rt = wave % nrt, kh = wave / nrt;  // output tile, contraction half
  const unsigned bmask = part ? 0u : 0x80000000u;
  unsigned aoff[(HS + 1) / 2];
  {
    const int row = rt * 16 + (lane & 15);
    const bool rowok = row < p3;
    const int a = rowok ? row / nz : 0, iz = rowok ? row - a * nz : 0;
#pragma unroll
    for (int u = 0; u < HS; ++u) {
      const int c = 4 * (kh * HS + u) + kk0;
      unsigned w = (unsigned)Es;
      if (rowok && c < p3) {
        const int b = c / nz, jz = c - b * nz;
        bool neg;
        w = (unsigned)staged_index(a, iz, b, jz, nz, tri, neg) | (neg ? 0x8000u : 0u);
      }
      if (u & 1)
        aoff[u >> 1] |= w << 16;
      else
        aoff[u >> 1] = w;
    }
  }
  if (tid == 0) Qv[Es] = v2{(T)0, (T)0};
  const int nxe = nct * 8 * kpad;  // input-vector elements (c, v)
  // point-independent staging maps of this thread: LDS slot of each packed
  // entry it carries; column v, row c (component b) and RHS of each input
  // element, and its place in the B rows
  int tdst[kStageRegs];
#pragma unroll
  for (int u = 0; u < kStageRegs; ++u) {
    const int e = tid + u * nthr;
    tdst[u] = e < E ? staged_of_packed(e, nz, tri) : -1;
  }
  int xv_[kXRegs], xc_[kXRegs], xmi_[kXRegs], xr_[kXRegs], xb_[kXRegs], xdst_[kXRegs];
#pragma unroll
  for (int u = 0; u < kXRegs; ++u) {
    const int idx = u * nthr + tid;
    const int v = idx < nxe ? idx / kpad : 1 << 20, c = idx < nxe ? idx - v * kpad : 0;
    xv_[u] = v;
    xc_[u] = c < p3 ? c : 0;
    xmi_[u] = idx < nxe ? v / R : 0;
    xr_[u] = idx < nxe ? v - (v / R) * R : 0;
    xb_[u] = c < p3 ? c / nz : 3;  // 3: padding row
    xdst_[u] = idx < nxe ? ((v >> 3) * kpad + c) * 16 + (v & 7) : -1;
  }
  v2 pre[NB][kStageRegs];
  cplx<T> xpre[NB][kXRegs];
  unsigned xneg[NB], xval[NB];  // mirror sign / presence of each prefetched input element
  // loads of one point's row and input vectors into prefetch set b
  auto prefetch = [&](int task_, int b) __attribute__((always_inline)) {
    const int f_ = MF ? task_ / npts : 0, rep_ = task_ - f_ * npts;
    const v2 *src = (MF ? reinterpret_cast<const v2 *>(tabs.tab[f_]) : tab0) + (size_t)rep_ * E;
#pragma unroll
    for (int u = 0; u < kStageRegs; ++u)
      if (tdst[u] >= 0) pre[b][u] = src[tid + u * nthr];
    const MirrorSet m = mirror_set(rep_, nx, ny);
    const int V = m.n * R;
    // the sign is applied when the element is written to LDS, so that no
    // instruction here waits for the loads
    // (every element is loaded, from a clamped address when it is padding,
    // so that no register is written between the loads and their use)
    xneg[b] = 0;
    xval[b] = 0;
#pragma unroll
    for (int u = 0; u < kXRegs; ++u) {
      const bool ok = xv_[u] < V && xb_[u] < 3;
      int pt;
      bool fx, fy;
      mirror_of(m, ok ? xmi_[u] : 0, nx, ny, pt, fx, fy);
      xpre[b][u] = sin[((size_t)pt * rtot + f_ * R + (ok ? xr_[u] : 0)) * p3 + xc_[u]];
      if (ok && ((xb_[u] == 0 && fx) || (xb_[u] == 1 && fy))) xneg[b] |= 1u << u;
      if (ok) xval[b] |= 1u << u;
    }
  };
  const int stride = NB * (int)gridDim.x;
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int t0 = (int)blockIdx.x + b * (int)gridDim.x;
    prefetch(t0 < ntask ? t0 : ntask - 1, b);
  }
  for (int task0 = blockIdx.x; task0 < ntask; task0 += stride) {
#pragma unroll
  for (int hb = 0; hb < NB; ++hb) {
    const int task = task0 + hb * (int)gridDim.x;
    if (task >= ntask) break;
    const int f = MF ? task / npts : 0, rep = task - f * npts;
    lds_barrier();  // every wavefront is done with the previous point
#pragma unroll
    for (int u = 0; u < kStageRegs; ++u)
      if (tdst[u] >= 0) Qv[tdst[u]] = pre[hb][u];
#pragma unroll
    for (int u = 0; u < kXRegs; ++u) {
      if (xdst_[u] >= 0) {
        T *brow = Bs + xdst_[u];
        const unsigned sm = ((xneg[hb] >> u) & 1u) ? 0x80000000u : 0u;
        const bool ok = (xval[hb] >> u) & 1u;
        brow[0] = ok ? flip_sign(xpre[hb][u].x, sm) : (T)0;
        brow[8] = ok ? flip_sign(xpre[hb][u].y, sm) : (T)0;
      }
    }
    const MirrorSet m = mirror_set(rep, nx, ny);
    const int V = m.n * R;
    // the loads of the point NB steps ahead go into the set just staged; they
    // are issued one per k-step of the first column tile below, so that
    // waiting for queue space overlaps the MFMAs (a clamped address past the
    // last point: the loads are always issued)
    const int ntk = task + stride;
    const bool more = ntk < ntask;
    const int fnx = MF ? (more ? ntk : task) / npts : 0;
    const int nrep = (more ? ntk : task) - fnx * npts;
    const v2 *nsrc = (MF ? reinterpret_cast<const v2 *>(tabs.tab[fnx]) : tab0) + (size_t)nrep * E;
    int xaddr[kXRegs];
    {
      const MirrorSet mn = mirror_set(nrep, nx, ny);
      const int Vn = mn.n * R;
      xneg[hb] = 0;
      xval[hb] = 0;
#pragma unroll
      for (int u = 0; u < kXRegs; ++u) {
        const bool ok = xv_[u] < Vn && xb_[u] < 3;
        int pt;
        bool fx, fy;
        mirror_of(mn, ok ? xmi_[u] : 0, nx, ny, pt, fx, fy);
        xaddr[u] = (pt * rtot + fnx * R + (ok ? xr_[u] : 0)) * p3 + xc_[u];
        if (ok && ((xb_[u] == 0 && fx) || (xb_[u] == 1 && fy))) xneg[hb] |= 1u << u;
        if (ok) xval[hb] |= 1u << u;
      }
    }
    lds_barrier();
    for (int ct = 0; ct * 8 < V; ++ct) {
      typename M::acc_t accr = {0, 0, 0, 0}, acci = {0, 0, 0, 0};
      const int kb = kh * HS * 4 + kk0;  // first B row of this half
      const T *b1p = Bs + ((size_t)ct * kpad + kb) * 16 + j;
      const T *b2p = Bs + ((size_t)ct * kpad + kb) * 16 + (j ^ 8);
#pragma unroll
      for (int u = 0; u < HS; ++u) {
        if (ct == 0 && (NB > 1 || more)) {
          // prefetch slot u: packed entries first, then input elements
          if (u < kStageRegs) {
            if (tdst[u] >= 0) pre[hb][u] = nsrc[tid + u * nthr];
          } else if (u - kStageRegs < kXRegs) {
            xpre[hb][u - kStageRegs] = sin[xaddr[u - kStageRegs]];
          }
        }
        const unsigned w = (u & 1) ? (aoff[u >> 1] >> 16) : (aoff[u >> 1] & 0xffffu);
        const v2 q = Qv[w & 0x7fffu];
        const unsigned qm = (w & 0x8000u) << 16;
        const T b1 = b1p[u * 64];
        const T b2 = flip_sign(b2p[u * 64], bmask);
        accr = M::mma(flip_sign(q.x, qm), b1, accr);
        acci = M::mma(flip_sign(q.y, qm), b2, acci);
      }
      if (ct == 0 && (NB > 1 || more)) {
#pragma unroll
        for (int u = HS; u < kStageRegs + kXRegs; ++u) {
          if (u < kStageRegs) {
            if (tdst[u] >= 0) pre[hb][u] = nsrc[tid + u * nthr];
          } else {
            xpre[hb][u - kStageRegs] = sin[xaddr[u - kStageRegs]];
          }
        }
      }
      if (kh == 1) {
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) Red[(rt * 4 + qq) * 64 + lane] = accr[qq] + acci[qq];
      }
      lds_barrier();
      if (kh == 0) {
        const int v = ct * 8 + (j & 7);
        if (v < V) {
          const int mi = v / R, r = v - mi * R;
          int pt;
          bool fx, fy;
          mirror_of(m, mi, nx, ny, pt, fx, fy);
          T *ob = reinterpret_cast<T *>(sout + ((size_t)pt * rtot + f * R + r) * p3);
#pragma unroll
          for (int qq = 0; qq < 4; ++qq) {
            const int orow = rt * 16 + M::row(lane, qq);
            if (orow < p3) {
              const int oa = orow / nz;
              const T sg = ((oa == 0 && fx) || (oa == 1 && fy)) ? (T)-1 : (T)1;
              ob[2 * orow + part] = sg * (accr[qq] + acci[qq] + Red[(rt * 4 + qq) * 64 + lane]);
            }
          }
        }
      }
      lds_barrier();  // Red is reused by the next column tile
    }
  }
  }
}

// Double-buffered variant: the packed rows of two points live in LDS.  While
// the wavefronts run the MFMAs of point p from one buffer, they write point
// p + 1's row (loaded into registers during point p - 1) into the other one
// and then issue the loads of point p + 2's row into the same registers, one
// slot per k-step; the input vectors of point p + 1 are loaded at the start
// of point p and staged after the barrier that starts point p + 1.  So the
// staging of the row is off the path between two points' MFMAs, and a row's
// loads have a whole point to arrive.  Needs two rows, the B rows and the
// reduction buffer in LDS (FP64: Nz <= 32 with R <= 2).
template <typename T, int NS, bool MF>
__global__ void __launch_bounds__(768) __attribute__((amdgpu_waves_per_eu(3, 3)))
k_block_dbl(TabSet tabs, const cplx<T> *__restrict__ sin, cplx<T> *__restrict__ sout, int nx,
            int ny, int nz, int R, int nct, int nf) {
  typedef Mfma<T> M;
  typedef T v2 __attribute__((ext_vector_type(2)));
  constexpr int HS = NS / 2;  // k-steps per half
  constexpr int kpad = 4 * NS;
  static_assert(HS >= kStageRegs, "one row slot per k-step of the first half");
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const int E = 2 * nz * (2 * nz + 1);
  const int Es = E + 2 * nz;  // padded rows of the full blocks; entry Es is zero
  const int QS = Es + 2;      // entries per row buffer
  const int p3 = 3 * nz, tri = nz * (nz + 1) / 2;
  const int nrt = (p3 + 15) >> 4;
  v2 *Qb = reinterpret_cast<v2 *>(lds_raw);            // [2][QS]
  T *Bs = reinterpret_cast<T *>(Qb + 2 * QS);           // [nct][kpad][16]
  T *Red = Bs + (size_t)nct * kpad * 16;                // [nrt][4][64] partial sums
  const int npts = (nx + 1) * (ny + 1);
  const int ntask = MF ? nf * npts : npts;
  const int rtot = MF ? nf * R : R;
  const v2 *tab0 = reinterpret_cast<const v2 *>(tabs.tab[0]);
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int kk0 = lane >> 4, j = lane & 15, part = j >> 3;
  const int rt = wave % nrt, kh = wave / nrt;  // output tile, contraction half
  const unsigned bmask = part ? 0u : 0x80000000u;
  unsigned aoff[(HS + 1) / 2];
  {
    const int row = rt * 16 + (lane & 15);
    const bool rowok = row < p3;
    const int a = rowok ? row / nz : 0, iz = rowok ? row - a * nz : 0;
#pragma unroll
    for (int u = 0; u < HS; ++u) {
      const int c = 4 * (kh * HS + u) + kk0;
      unsigned w = (unsigned)Es;
      if (rowok && c < p3) {
        const int b = c / nz, jz = c - b * nz;
        bool neg;
        w = (unsigned)staged_index(a, iz, b, jz, nz, tri, neg) | (neg ? 0x8000u : 0u);
      }
      if (u & 1)
        aoff[u >> 1] |= w << 16;
      else
        aoff[u >> 1] = w;
    }
  }
  if (tid == 0) {
    Qb[Es] = v2{(T)0, (T)0};
    Qb[QS + Es] = v2{(T)0, (T)0};
  }
  const int nxe = nct * 8 * kpad;  // input-vector elements (c, v)
  int tdst[kStageRegs];
#pragma unroll
  for (int u = 0; u < kStageRegs; ++u) {
    const int e = tid + u * nthr;
    tdst[u] = e < E ? staged_of_packed(e, nz, tri) : -1;
  }
  int xv_[kXRegs], xc_[kXRegs], xmi_[kXRegs], xr_[kXRegs], xb_[kXRegs], xdst_[kXRegs];
#pragma unroll
  for (int u = 0; u < kXRegs; ++u) {
    const int idx = u * nthr + tid;
    const int v = idx < nxe ? idx / kpad : 1 << 20, c = idx < nxe ? idx - v * kpad : 0;
    xv_[u] = v;
    xc_[u] = c < p3 ? c : 0;
    xmi_[u] = idx < nxe ? v / R : 0;
    xr_[u] = idx < nxe ? v - (v / R) * R : 0;
    xb_[u] = c < p3 ? c / nz : 3;  // 3: padding row
    xdst_[u] = idx < nxe ? ((v >> 3) * kpad + c) * 16 + (v & 7) : -1;
  }
  auto row_of = [&](int task_) __attribute__((always_inline)) {
    const int f_ = MF ? task_ / npts : 0, rep_ = task_ - f_ * npts;
    return (MF ? reinterpret_cast<const v2 *>(tabs.tab[f_]) : tab0) + (size_t)rep_ * E;
  };
  v2 pre[kStageRegs];
  cplx<T> xpre[kXRegs];
  unsigned xneg = 0, xval = 0;  // mirror sign / presence of each prefetched input element
  auto load_x = [&](int task_) __attribute__((always_inline)) {
    const int f_ = MF ? task_ / npts : 0, rep_ = task_ - f_ * npts;
    const MirrorSet mm = mirror_set(rep_, nx, ny);
    const int V = mm.n * R;
    xneg = 0;
    xval = 0;
#pragma unroll
    for (int u = 0; u < kXRegs; ++u) {
      const bool ok = xv_[u] < V && xb_[u] < 3;
      int pt;
      bool fx, fy;
      mirror_of(mm, ok ? xmi_[u] : 0, nx, ny, pt, fx, fy);
      xpre[u] = sin[((size_t)pt * rtot + f_ * R + (ok ? xr_[u] : 0)) * p3 + xc_[u]];
      if (ok && ((xb_[u] == 0 && fx) || (xb_[u] == 1 && fy))) xneg |= 1u << u;
      if (ok) xval |= 1u << u;
    }
  };
  int task = blockIdx.x;
  // prologue: the first point's row into buffer 0, its input vectors and the
  // second point's row into registers
  {
    const v2 *src = row_of(task);
#pragma unroll
    for (int u = 0; u < kStageRegs; ++u)
      if (tdst[u] >= 0) pre[u] = src[tid + u * nthr];
#pragma unroll
    for (int u = 0; u < kStageRegs; ++u)
      if (tdst[u] >= 0) Qb[tdst[u]] = pre[u];
    load_x(task);
    const int t1 = task + (int)gridDim.x;
    const v2 *src1 = row_of(t1 < ntask ? t1 : task);
#pragma unroll
    for (int u = 0; u < kStageRegs; ++u)
      if (tdst[u] >= 0) pre[u] = src1[tid + u * nthr];
  }
  int cur = 0;
  for (; task < ntask; task += gridDim.x) {
    const int f = MF ? task / npts : 0, rep = task - f * npts;
    // every wavefront is done with the previous point (its MFMAs, Bs, Red),
    // and this point's row, written during the previous point, is complete
    lds_barrier();
#pragma unroll
    for (int u = 0; u < kXRegs; ++u) {
      if (xdst_[u] >= 0) {
        T *brow = Bs + xdst_[u];
        const unsigned sm = ((xneg >> u) & 1u) ? 0x80000000u : 0u;
        const bool ok = (xval >> u) & 1u;
        brow[0] = ok ? flip_sign(xpre[u].x, sm) : (T)0;
        brow[8] = ok ? flip_sign(xpre[u].y, sm) : (T)0;
      }
    }
    const MirrorSet m = mirror_set(rep, nx, ny);
    const int V = m.n * R;
    const int ntk = task + (int)gridDim.x, ntk2 = ntk + (int)gridDim.x;
    const bool more = ntk < ntask;
    // the next point's input vectors (staged at its start) and the address of
    // the row two points ahead (clamped past the last point)
    load_x(more ? ntk : task);
    const v2 *src2 = row_of(ntk2 < ntask ? ntk2 : (more ? ntk : task));
    const v2 *Qv = Qb + cur * QS;
    v2 *Qn = Qb + (cur ^ 1) * QS;
    lds_barrier();
    for (int ct = 0; ct * 8 < V; ++ct) {
      typename M::acc_t accr = {0, 0, 0, 0}, acci = {0, 0, 0, 0};
      const int kb = kh * HS * 4 + kk0;  // first B row of this half
      const T *b1p = Bs + ((size_t)ct * kpad + kb) * 16 + j;
      const T *b2p = Bs + ((size_t)ct * kpad + kb) * 16 + (j ^ 8);
#pragma unroll
      for (int u = 0; u < HS; ++u) {
        const unsigned w = (u & 1) ? (aoff[u >> 1] >> 16) : (aoff[u >> 1] & 0xffffu);
        const v2 q = Qv[w & 0x7fffu];
        const unsigned qm = (w & 0x8000u) << 16;
        const T b1 = b1p[u * 64];
        const T b2 = flip_sign(b2p[u * 64], bmask);
        accr = M::mma(flip_sign(q.x, qm), b1, accr);
        acci = M::mma(flip_sign(q.y, qm), b2, acci);
        if (ct == 0 && more && u < kStageRegs && tdst[u] >= 0) {
          // slot u: the next point's entry into the other buffer (its reads
          // by the previous point's MFMAs ended before the barriers above),
          // then the load of the entry two points ahead into the freed
          // register; one slot per k-step, so that the writes drain behind
          // the MFMAs
          Qn[tdst[u]] = pre[u];
          pre[u] = src2[tid + u * nthr];
        }
        // keep each k-step's LDS traffic next to its MFMAs: hoisting it all
        // ahead, on top of the row loads in flight, would exceed the
        // registers of three wavefronts per SIMD
        __builtin_amdgcn_sched_barrier(0);
      }
      if (kh == 1) {
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) Red[(rt * 4 + qq) * 64 + lane] = accr[qq] + acci[qq];
      }
      lds_barrier();
      if (kh == 0) {
        const int v = ct * 8 + (j & 7);
        if (v < V) {
          const int mi = v / R, r = v - mi * R;
          int pt;
          bool fx, fy;
          mirror_of(m, mi, nx, ny, pt, fx, fy);
          T *ob = reinterpret_cast<T *>(sout + ((size_t)pt * rtot + f * R + r) * p3);
#pragma unroll
          for (int qq = 0; qq < 4; ++qq) {
            const int orow = rt * 16 + M::row(lane, qq);
            if (orow < p3) {
              const int oa = orow / nz;
              const T sg = ((oa == 0 && fx) || (oa == 1 && fy)) ? (T)-1 : (T)1;
              ob[2 * orow + part] = sg * (accr[qq] + acci[qq] + Red[(rt * 4 + qq) * 64 + lane]);
            }
          }
        }
      }
      lds_barrier();  // Red is reused by the next column tile
    }
    cur ^= 1;
  }
}

static int lds_nct(int R) { return (4 * R + 7) / 8; }

// k-steps rounded up to a multiple of 4 (the compiled variants)
static int lds_ns(int nz) { return 4 * (((3 * nz + 3) / 4 + 3) / 4); }

// LDS of one workgroup: staged row, B rows and (KS = 2) the reduction buffer
static size_t lds_bytes_t(int nz, int R, size_t csize, int ks) {
  const size_t Es = 2 * (size_t)nz * (2 * nz + 1) + 2 * nz;
  const size_t kpad = 4 * (size_t)lds_ns(nz);
  const size_t nrt = (3 * (size_t)nz + 15) / 16;
  return (Es + 2) * csize + (size_t)lds_nct(R) * kpad * 16 * (csize / 2) +
         (ks == 2 ? nrt * 256 * (csize / 2) : 0);
}

static const size_t kLdsLimit = 160 * 1024;

// the double-buffered kernel: a second staged row on top of the KS = 2 layout
static size_t lds_bytes_dbl(int nz, int R, size_t csize) {
  const size_t Es = 2 * (size_t)nz * (2 * nz + 1) + 2 * nz;
  return lds_bytes_t(nz, R, csize, 2) + (Es + 2) * csize;
}

// ks wavefronts (contraction parts) per 16-row tile
static int lds_waves(int nz, int ks) { return ks * ((3 * nz + 15) / 16); }

// whether the pipelined kernel with contraction split ks runs this shape (for
// ks = 1, with two workgroups per CU)
static bool lds_fits(int nz, int R, size_t csize, int ks) {
  const long long E = 2LL * nz * (2 * nz + 1);
  const int nthr = 64 * lds_waves(nz, ks);
  const long long nxe = (long long)lds_nct(R) * 8 * 4 * lds_ns(nz);
  const size_t lim = ks == 2 ? kLdsLimit : kLdsLimit / 2;
  const int sr = ks == 2 ? kStageRegs : kStageRegs1;
  return lds_bytes_t(nz, R, csize, ks) <= lim && lds_ns(nz) / ks <= kMaxHalfSteps * (3 - ks) &&
         nthr <= 768 && E <= (long long)sr * nthr && nxe <= (long long)kXRegs * nthr &&
         E + 2 * nz + 1 < 0x8000;
}

static bool dbl_fits(int nz, int R, size_t csize) {
  return lds_fits(nz, R, csize, 2) && lds_bytes_dbl(nz, R, csize) <= kLdsLimit &&
         lds_ns(nz) / 2 >= kStageRegs && lds_nct(R) == 1;
}

#define GIEM_BLOCK_VARIANTS(X, T) \
  X(T, 4) X(T, 8) X(T, 12) X(T, 16) X(T, 20) X(T, 24) X(T, 28) X(T, 32)

hipError_t set_block_lds_limits() {
  hipError_t e = hipSuccess;
#define GIEM_SET_ATTR(T, NS)                                                               \
  if (e == hipSuccess)                                                                     \
    e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_block_pipe1<T, NS, false, 2>), \
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsLimit);  \
  if (e == hipSuccess)                                                                     \
    e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_block_pipe1<T, NS, true, 2>),  \
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsLimit);  \
  if (e == hipSuccess)                                                                     \
    e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_block_pipe1<T, NS, false, 1>), \
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsLimit);  \
  if (e == hipSuccess)                                                                     \
    e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_block_pipe1<T, NS, true, 1>),  \
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsLimit);  \
  if (e == hipSuccess)                                                                     \
    e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_block_pipe<T, NS, 2, false>),  \
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsLimit);  \
  if (e == hipSuccess)                                                                     \
    e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_block_pipe<T, NS, 2, true>),   \
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsLimit);  \
  if (e == hipSuccess && NS / 2 >= kStageRegs)                                             \
    e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_block_dbl<T, (NS >= 12 ? NS : 12), false>), \
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsLimit);  \
  if (e == hipSuccess && NS / 2 >= kStageRegs)                                             \
    e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_block_dbl<T, (NS >= 12 ? NS : 12), true>), \
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsLimit);
  GIEM_BLOCK_VARIANTS(GIEM_SET_ATTR, double)
  GIEM_BLOCK_VARIANTS(GIEM_SET_ATTR, float)
#undef GIEM_SET_ATTR
  const void *band[] = {band_kernel<float, 3, 4, 4, 8>(), band_kernel<float, 3, 4, 4, 16>(),
                        band_kernel<double, 2, 4, 4, 16>(), band_kernel<double, 3, 4, 3, 12>()};
  for (const void *k : band)
    if (e == hipSuccess)
      e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsLimit);
  return e;
}

bool block_supported(int nz, int R) { return nz >= 1 && 2 * nz * (2 * nz + 1) < (1 << 24) && R >= 1 && R <= kMaxRhs; }

template <typename T>
static hipError_t launch_block_t(const TabSet &tabs, int nf, const void *sin, void *sout,
                                 int nx, int ny, int nz, int R, int nbuf, hipStream_t s) {
  const long long ntask = (long long)nf * (nx + 1) * (ny + 1);
  // the pipelined kernels form spectra element offsets in 32-bit integers
  const bool off32 = 4LL * nx * ny * nf * R * 3 * nz < (1LL << 31);
  const size_t cs = sizeof(cplx<T>);
  if (nbuf == 3 && !lds_fits(nz, R, cs, 1)) nbuf = 1;
  if (nbuf == 4 && !dbl_fits(nz, R, cs)) nbuf = 2;
  const int ks = nbuf == 3 ? 1 : 2;
  if (lds_fits(nz, R, cs, ks) && off32) {
    const size_t lds = nbuf == 4 ? lds_bytes_dbl(nz, R, cs) : lds_bytes_t(nz, R, cs, ks);
    const int nthr = 64 * lds_waves(nz, ks);
    // persistent grid: one workgroup per CU (two for ks = 1); more
    // workgroups per CU at small Nz measured slower (a larger tail round)
    const long long cap = ks == 1 ? 512 : 256;
    const long long grid = ntask < cap ? ntask : cap;
    const int ns = lds_ns(nz);
#define GIEM_LAUNCH_MF(TT, NS, MF)                                                        \
  if (nbuf == 4)                                                                          \
    k_block_dbl<TT, (NS >= 12 ? NS : 12), MF><<<(unsigned)grid, nthr, lds, s>>>(           \
        tabs, static_cast<const cplx<TT> *>(sin), static_cast<cplx<TT> *>(sout), nx, ny,   \
        nz, R, lds_nct(R), nf);                                                           \
  else if (nbuf == 2)                                                                     \
    k_block_pipe<TT, NS, 2, MF><<<(unsigned)grid, nthr, lds, s>>>(                         \
        tabs, static_cast<const cplx<TT> *>(sin), static_cast<cplx<TT> *>(sout), nx, ny,   \
        nz, R, lds_nct(R), nf);                                                           \
  else if (nbuf == 3)                                                                     \
    k_block_pipe1<TT, NS, MF, 1><<<(unsigned)grid, nthr, lds, s>>>(                        \
        tabs, static_cast<const cplx<TT> *>(sin), static_cast<cplx<TT> *>(sout), nx, ny,   \
        nz, R, lds_nct(R), nf);                                                           \
  else                                                                                    \
    k_block_pipe1<TT, NS, MF, 2><<<(unsigned)grid, nthr, lds, s>>>(                        \
        tabs, static_cast<const cplx<TT> *>(sin), static_cast<cplx<TT> *>(sout), nx, ny,   \
        nz, R, lds_nct(R), nf);
#define GIEM_LAUNCH(TT, NS)                                                               \
  if (ns == NS) {                                                                         \
    if (nf > 1) {                                                                         \
      GIEM_LAUNCH_MF(TT, NS, true)                                                        \
    } else {                                                                              \
      GIEM_LAUNCH_MF(TT, NS, false)                                                       \
    }                                                                                     \
    return hipGetLastError();                                                             \
  }
    GIEM_BLOCK_VARIANTS(GIEM_LAUNCH, T)
#undef GIEM_LAUNCH
#undef GIEM_LAUNCH_MF
  }
  // rows too long for LDS: the band-pair kernel (FP32: 8 wavefronts, 3 or 6
  // output tiles each; FP64: 16 wavefronts, 2 or 3 tiles each, its
  // accumulators being twice as wide): Nz <= 256, the handle refuses Nz > 170
  const int nb = (nz + 15) / 16;
  if (3 * nb > 48 || lds_bytes_band(nz, cs) > kLdsLimit || ntask > 0x7fffffffLL)
    return hipErrorInvalidValue;
  const size_t lds = lds_bytes_band(nz, cs);
  const cplx<T> *si = static_cast<const cplx<T> *>(sin);
  cplx<T> *so = static_cast<cplx<T> *>(sout);
  if constexpr (sizeof(T) == 4) {
    if (3 * nb <= 24)
      k_block_band<T, 3, 4, 4, 8><<<(unsigned)ntask, 512, lds, s>>>(tabs, si, so, nx, ny, nz, R, nf);
    else
      k_block_band<T, 3, 4, 4, 16><<<(unsigned)ntask, 1024, lds, s>>>(tabs, si, so, nx, ny, nz, R,
                                                                      nf);
  } else {
    if (3 * nb <= 32)
      k_block_band<T, 2, 4, 4, 16><<<(unsigned)ntask, 1024, lds, s>>>(tabs, si, so, nx, ny, nz, R,
                                                                      nf);
    else
      k_block_band<T, 3, 4, 3, 12><<<(unsigned)ntask, 768, lds, s>>>(tabs, si, so, nx, ny, nz, R,
                                                                    nf);
  }
  return hipGetLastError();
}

bool block_two_per_cu(int nz, int R, int prec) {
  return lds_fits(nz, R, prec == PREC_FP32 ? sizeof(c64) : sizeof(c128), 1);
}

bool block_dbl_supported(int nz, int R, int prec) {
  return dbl_fits(nz, R, prec == PREC_FP32 ? sizeof(c64) : sizeof(c128));
}

hipError_t launch_block(int prec, const TabSet &tabs, int nf, const void *sin, void *sout,
                        int nx, int ny, int nz, int R, int nbuf, hipStream_t s) {
  if (nf < 1 || nf > kMaxFreqBatch) return hipErrorInvalidValue;
  return prec == PREC_FP32 ? launch_block_t<float>(tabs, nf, sin, sout, nx, ny, nz, R, nbuf, s)
                           : launch_block_t<double>(tabs, nf, sin, sout, nx, ny, nz, R, nbuf, s);
}

}  // namespace giem
