// The giem_handle and host-side helpers (internal).
#pragma once

#include <complex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/giem.h"
#include "kernels.h"

namespace giem {

typedef std::complex<double> cd;

void set_error(const std::string &msg);
const std::string &get_error();

struct FftPlan {
  FftDesc d{};
  void *tw64 = nullptr;  // c128 [L]
  void *tw32 = nullptr;  // c64  [L]
};

struct FreqTables {
  double freq = 0.0;
  void *spec64 = nullptr;      // c128 [(Ny+1)(Nx+1)][E] packed spectra
  void *spec32 = nullptr;      // c64 copy (GIEM_TABLES_C64)
  void *spatial = nullptr;     // c128 [Ny][Nx][E] packed spatial table (device)
  // receiver kernels (giem_fields, giem_dipole_source) per receiver depth,
  // built on first use
  std::vector<std::pair<double, void *>> rec_kernels;
};

struct SolveWork;

}  // namespace giem

struct giem_handle {
  int nx = 0, ny = 0, nz = 0, nlay = 0;
  double hx = 0, hy = 0, x0 = 0, y0 = 0;
  std::vector<double> d, z_edges;
  std::vector<giem::cd> sigma;     // [nlay + 1]
  std::vector<int> layer_of_cell;  // [nz]
  uint32_t flags = 0;
  int device = 0;
  std::vector<giem::FreqTables> f;
  giem::FftPlan px, py;            // lengths 2 Nx, 2 Ny
  // per-level device data
  void *sb_lev = nullptr;    // c128 [nz]
  void *vol_lev = nullptr;   // double [nz]
  void *sroot_lev = nullptr; // double [nz]
  // diagonals of the last sigma_a: S, R1, R2, a (c128 [N] each)
  void *diag = nullptr;
  // spectra workspace
  void *spec_ws = nullptr;
  size_t spec_ws_bytes = 0;
  // reduction scratch
  void *red_part = nullptr;  // c128 [kMaxRhs][65][nblk]
  void *red_out = nullptr;   // c128 [kMaxSys][65]
  void *red_host = nullptr;  // pinned host mirror of red_out
  void *coef_dev = nullptr;  // c128 [kMaxSys][65] coefficients for updates
  void *coef_host = nullptr; // pinned
  void *gs_scale_dev = nullptr;   // double [kMaxSys][65]: 1 / |V_i|^2 of the basis
  void *gs_scale_host = nullptr;  // pinned mirror
  // solver workspace (grown on demand)
  void *basis = nullptr;
  size_t basis_bytes = 0;
  void *vec_ws = nullptr;
  size_t vec_ws_bytes = 0;
  giem::SolveWork *sw = nullptr;
  // FFT launch shape per precision (0 = FP64, 1 = FP32) and pass (x forward,
  // y forward, y inverse, x inverse): sequences per workgroup and threads per
  // workgroup, set by giem_tune; 0 selects the built-in choice
  int fft_g[2][4] = {}, fft_nt[2][4] = {};
  // register sets of prefetched points in the block product per precision
  // (1 or 2), set by giem_tune; 0 selects the built-in choice
  int block_nbuf[2] = {};
  // stage profiling (giem_profile): 6 events per recorded apply, or 2 when
  // only one kernel (prof_stage >= 0) is bracketed
  bool prof = false;
  int prof_stage = -1;
  std::vector<hipEvent_t> prof_ev;
  std::vector<int> prof_meta;  // per recorded apply: precision, nrhs, stage (-1: all)
  size_t prof_used = 0;
  // right-hand sides of recorded applies whose results GMRES discarded (an
  // apply queued ahead for a system that then stopped, or before a second
  // Gram-Schmidt pass), per precision (FP64, FP32)
  int64_t prof_discarded[2] = {0, 0};

  size_t ncell() const { return (size_t)nx * ny * nz; }
  size_t nvec() const { return 3 * ncell(); }
  int E() const { return 2 * nz * (2 * nz + 1); }
};

namespace giem {

int check_hip(hipError_t e, const char *what);
int ensure_spec_ws(giem_handle *t, int nrhs, int prec);
int compute_diagonals(giem_handle *t, const c128 *sigma_a, hipStream_t s);
// y = op x on per-RHS pointers; diagonals must be current (compute_diagonals)
int apply_core(giem_handle *t, int ifreq, int nrhs, const VecPtrs &p, unsigned mode,
               unsigned prec, hipStream_t s, double *stage_ms);
// the same on complex64 vectors (FP32 operator only)
int apply_core(giem_handle *t, int ifreq, int nrhs, const VecPtrs32 &p, unsigned mode,
               unsigned prec, hipStream_t s, double *stage_ms);
// one apply over nf frequencies ifreqs[0..nf) with nrhs vectors each: p.in[f
// nrhs + r] is vector r of frequency ifreqs[f] (one launch per kernel for all)
int apply_multi(giem_handle *t, int nf, const int *ifreqs, int nrhs, const VecPtrs &p,
                unsigned mode, unsigned prec, hipStream_t s);
int apply_multi(giem_handle *t, int nf, const int *ifreqs, int nrhs, const VecPtrs32 &p,
                unsigned mode, unsigned prec, hipStream_t s);
int upload_spatial(giem_handle *t, hipStream_t s);
int plane_wave_levels(const giem_handle *t, double freq, std::vector<cd> &en_lev,
                      std::vector<cd> &hsurf);
// packed spatial tables of every frequency of the handle (t->f[q].spatial, device)
int compute_tables(giem_handle *t, hipStream_t s);
// receiver kernels of frequency ifreq (device, owned by the caller)
int compute_receiver_kernels(giem_handle *t, int ifreq, double z0, void **out, hipStream_t s);

}  // namespace giem
