// Launchers of the HIP kernels (internal).
#pragma once

#include <vector>

#include "common.h"

namespace giem {

// operator apply (kernels_apply.hip)
hipError_t set_lds_limits();
hipError_t set_block_lds_limits();
bool block_supported(int nz, int R);
size_t fft_lds_bytes(int G, int L, int prec);
// elements per thread for G sequences of length L on nthr threads; 0 when no
// kernel is instantiated for it (nthr in {256, 512})
int fft_ept(int G, int L, int nthr, int prec);
hipError_t launch_fft_x_fwd(int prec, const VecPtrs &ptrs, const c128 *r2, void *spec, int nx,
                            int ny, int nz, int rp_total, int G, int nthr, const FftDesc &fd,
                            const void *tw, hipStream_t s);
hipError_t launch_fft_x_inv(int prec, const VecPtrs &ptrs, const c128 *sd, const c128 *r1,
                            const void *spec, int nx, int ny, int nz, int rp_total, int G,
                            int nthr, const FftDesc &fd, const void *tw, double scale,
                            hipStream_t s);
hipError_t launch_fft_y(int prec, void *spec, int nx2, int ny, int rp_total, int G, int nthr,
                        const FftDesc &fd, const void *tw, int inverse, hipStream_t s);
// complex64 vectors (FP32 transforms only)
hipError_t launch_fft_x_fwd(int prec, const VecPtrs32 &ptrs, const c128 *r2, void *spec, int nx,
                            int ny, int nz, int rp_total, int G, int nthr, const FftDesc &fd,
                            const void *tw, hipStream_t s);
hipError_t launch_fft_x_inv(int prec, const VecPtrs32 &ptrs, const c128 *sd, const c128 *r1,
                            const void *spec, int nx, int ny, int nz, int rp_total, int G,
                            int nthr, const FftDesc &fd, const void *tw, double scale,
                            hipStream_t s);
// out-of-place: sin and sout are two spectra buffers.
// nf frequencies (tables tabs.tab[0..nf)) with R vectors each: a point's
// record of the spectra holds nf R vectors, frequency f's at f R .. f R + R - 1.
// nbuf: variant of the pipelined kernel: 1 or 2 register sets of prefetched
// points (one workgroup per CU), 3: two workgroups per CU with one set each
// (falls back to 1 where it does not fit, see block_two_per_cu), 4: the row of
// the next point staged into a second LDS buffer during the current point's
// MFMAs (falls back to 2, see block_dbl_supported)
// Where the row does not fit LDS (Nz > 32 at R = 2) every nbuf takes the
// band-pair kernel.
hipError_t launch_block(int prec, const TabSet &tabs, int nf, const void *sin, void *sout,
                        int nx, int ny, int nz, int R, int nbuf, hipStream_t s);
bool block_two_per_cu(int nz, int R, int prec);
bool block_dbl_supported(int nz, int R, int prec);

// even/odd transform of the packed table along axis 0 (x) or 1 (y): nbatch
// lines, element j of line b at in + b sb + j sj, K at out + b ob + K sk
// (c128 units), n elements per line, transforms of length fd.L = 2 n
// (kernels_apply.hip, on the FFT passes of the apply)
hipError_t launch_parity_fft(const c128 *in, int64_t sj, int64_t sb, int nbatch, c128 *out,
                             int64_t sk, int64_t ob, int n, int E, int nz, int axis,
                             const FftDesc &fd, const void *tw, hipStream_t s);

// table set-up (kernels_setup.hip)
hipError_t launch_to_c64(const c128 *src, c64 *dst, size_t n, hipStream_t s);
hipError_t launch_diagonals(const c128 *sigma_a, const c128 *sb_lev, const double *vol_lev,
                            int nx, int ny, int nz, c128 *S, c128 *R1, c128 *R2, c128 *a,
                            int *bad, hipStream_t s);
hipError_t launch_plane_wave_rhs(const c128 *en_lev, const double *sroot_lev, int nx, int ny,
                                 int nz, int pol, c128 *out, hipStream_t s);

// gradient of the adjoint misfit (kernels_setup.hip)
hipError_t launch_adjoint_grad(const c128 *sigma_a, const c128 *sb_lev, const c128 *acell,
                               const c128 *g, const c128 *E, const c128 *lam, const c128 *w,
                               int nrhs, int nx, int ny, int nz, double *grad, hipStream_t s);

// fields at receivers above cell centres (kernels_tables.hip)
hipError_t launch_fields(const c128 *K, const c128 *E, const c128 *sa, const c128 *sb_lev,
                         const int *rec, int nrec, int nrhs, int nx, int ny, int nz,
                         const c128 *en_hn, c128 *Erec, c128 *Hrec, hipStream_t s);

hipError_t launch_impedance(const c128 *E, const c128 *H, int nrec, c128 *Z, hipStream_t s);
hipError_t launch_impedance_adjoint(const c128 *E, const c128 *H, int nrec, const c128 *G, c128 *wE,
                                    c128 *wH, hipStream_t s);
hipError_t launch_fields_adjoint(const c128 *K, const c128 *E, const c128 *sa, const c128 *sb_lev,
                                 const int *rec, int nrec, int nrhs, int nx, int ny, int nz,
                                 const c128 *wE, const c128 *wH, c128 *g, double *grad,
                                 hipStream_t s);
// U0 of unit-free dipole moments p [nsrc][3] at lattice points src [nsrc][2]
// from the receiver kernels K of their depth: out [nsrc][3][N]
hipError_t launch_dipole_rhs(const c128 *K, const int *src, const c128 *p, int nsrc, int nx,
                             int ny, int nz, const double *sroot_lev, const double *vol_lev,
                             c128 *out, hipStream_t s);

// Krylov vector kernels (kernels_vec.hip); vectors of n = 3 Nz Ny Nx complex.
// Krylov vectors are complex128, or complex64 in the inner solve of the
// precision form (suffix 32); arithmetic and accumulation are FP64 for both.
template <typename VT>
struct DotArgsT {
  const VT *w[kMaxRhs];      // vector to project
  const VT *basis[kMaxRhs];  // basis base pointer, vectors at stride n
};
using DotArgs = DotArgsT<c128>;
using DotArgs32 = DotArgsT<c64>;
int dot_partials_per_rhs();
// partial sums of conj-weighted dots <w, V_i> (i < nb) and ||w||^2 into
// part[r][block][nb + 1]; then reduced into out[r][nb + 1].  With a gate,
// system r is skipped (zeros out) unless gate[gate_off + r] is set.
hipError_t launch_dots(const DotArgs &a, int nrhs, int nb, size_t n, int nz, int plane,
                       const double *wlev, c128 *part, c128 *out, hipStream_t s,
                       const int *gate = nullptr, int gate_off = 0);
hipError_t launch_dots(const DotArgs32 &a, int nrhs, int nb, size_t n, int nz, int plane,
                       const double *wlev, c128 *part, c128 *out, hipStream_t s,
                       const int *gate = nullptr, int gate_off = 0);
// w -= sum_i f[r][i] h[r][i] V_i (f = hscale[r * sstride + i], or 1 when
// hscale is null), and ||w||^2 reduced into nrm[r] (real in .x); gated as
// launch_dots (a skipped system keeps w and gets nrm 0)
hipError_t launch_update(const DotArgs &a, int nrhs, int nb, size_t n, int nz, int plane,
                         const double *wlev, const c128 *h, int hstride, const double *hscale,
                         int sstride, c128 *part, c128 *nrm, hipStream_t s,
                         const int *gate = nullptr, int gate_off = 0);
hipError_t launch_update(const DotArgs32 &a, int nrhs, int nb, size_t n, int nz, int plane,
                         const double *wlev, const c128 *h, int hstride, const double *hscale,
                         int sstride, c128 *part, c128 *nrm, hipStream_t s,
                         const int *gate = nullptr, int gate_off = 0);
// Device-side Arnoldi state of the systems of one graph-captured GMRES
// cycle (index q): raw projections of both Gram-Schmidt passes (each handle's
// systems in a region of their own, (m + 2) entries per system, laid out at
// stride j + 2 in step j), squared norms after each pass, the second-pass gates, the
// squared basis norms and their inverses at stride kArnStride, the rotated
// Hessenberg matrix [(m + 1) m], rotations [m], residual vector [m + 1], and
// per system the tolerance times |b|, convergence flag and Krylov length.
constexpr int kArnStride = 65;
struct ArnoldiState {
  c128 *h1, *h2, *nrm1, *nrm2;
  int *gate;
  double *vn2, *scale;
  c128 *H, *cs, *sn, *g;
  double *tolb;
  int *conv, *jlen;
};
hipError_t launch_gs_gate(int nq, const c128 *h1, int hstride, const c128 *nrm1, int *gate,
                          double drop, hipStream_t s);
// h1c, h2c: the raw projections of system q0 (the next at stride j + 2)
hipError_t launch_arnoldi_tail(const ArnoldiState &st, const c128 *h1c, const c128 *h2c, int q0,
                               int nq, int j, int m, hipStream_t s);
// dst[r] = src[r] * scal[r] (complex scalars from the host)
hipError_t launch_scale(c128 *const *dst, const c128 *const *src, const c128 *scal, int nrhs,
                        size_t n, hipStream_t s);
hipError_t launch_scale(c64 *const *dst, const c64 *const *src, const c128 *scal, int nrhs,
                        size_t n, hipStream_t s);
hipError_t launch_scale(c64 *const *dst, const c128 *const *src, const c128 *scal, int nrhs,
                        size_t n, hipStream_t s);
template <typename VT>
struct LinArgsT {
  VT *x[kMaxRhs];
  const VT *basis[kMaxRhs];
};
using LinArgs = LinArgsT<c128>;
using LinArgs32 = LinArgsT<c64>;
// x[r] += sum_i y[r][i] V_i
hipError_t launch_lincomb(const LinArgs &a, int nrhs, int nb, size_t n, const c128 *y,
                          int ystride, hipStream_t s);
hipError_t launch_lincomb(const LinArgs32 &a, int nrhs, int nb, size_t n, const c128 *y,
                          int ystride, hipStream_t s);
// out = alpha * a + beta * b  (element-wise, complex scalars from host)
hipError_t launch_axpby(c128 *out, const c128 *a, const c128 *b, c128 alpha, c128 beta,
                        size_t n, hipStream_t s);
hipError_t launch_axpby(c64 *out, const c64 *a, const c64 *b, c128 alpha, c128 beta, size_t n,
                        hipStream_t s);
hipError_t launch_axpby(c128 *out, const c128 *a, const c64 *b, c128 alpha, c128 beta,
                        size_t n, hipStream_t s);
// out[r] = u[r] / a_cell (E = U / a)
hipError_t launch_div_cells(c128 *out, const c128 *u, const c128 *acell, int nrhs, size_t ncell,
                            hipStream_t s);
hipError_t launch_mul_cells(c128 *out, const c128 *u, const c128 *acell, int nrhs, size_t ncell,
                            hipStream_t s);
// weighted squared norms of nrhs contiguous vectors into nrm[r].x
hipError_t launch_norms(const c128 *v, int nrhs, size_t n, int nz, int plane, const double *wlev,
                        c128 *part, c128 *nrm, hipStream_t s);
hipError_t launch_norms(const c64 *v, int nrhs, size_t n, int nz, int plane, const double *wlev,
                        c128 *part, c128 *nrm, hipStream_t s);

}  // namespace giem
