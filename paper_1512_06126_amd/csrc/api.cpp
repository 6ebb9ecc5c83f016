// C-ABI entry points: handle construction, table upload and spectra, the
// operator apply, error reporting.  The GMRES driver is in solve.cpp.
#include <hip/hip_runtime.h>

#include <array>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <algorithm>

#include "handle.h"

namespace giem {

static thread_local std::string g_last_error;
void set_error(const std::string &msg) { g_last_error = msg; }
const std::string &get_error() { return g_last_error; }

int check_hip(hipError_t e, const char *what) {
  if (e == hipSuccess) return GIEM_OK;
  // the error is reported through the return code: take it out of the
  // runtime's last-error slot, or the next launch check (hipGetLastError
  // after a kernel launch) would report it again, e.g. after a failed
  // hipMalloc
  (void)hipGetLastError();
  set_error(std::string(what) + ": " + hipGetErrorString(e));
  return e == hipErrorOutOfMemory ? GIEM_ENOMEM : GIEM_EHIP;
}

#define GIEM_TRY(expr)          \
  do {                          \
    int rc__ = (expr);          \
    if (rc__ < 0) return rc__;  \
  } while (0)
#define GIEM_HIP(expr, what) GIEM_TRY(check_hip((expr), (what)))

static bool factor_ok(int L, FftDesc &d) {
  d.L = L;
  d.nf = 0;
  int m = L;
  const int radices[] = {16, 8, 4, 2, 3, 5, 7, 11};
  for (int r : radices) {
    while (m % r == 0) {
      if (d.nf >= kMaxFactors) return false;
      d.fac[d.nf++] = r;
      m /= r;
    }
  }
  return m == 1;
}

static int make_plan(int L, FftPlan &p) {
  if (!factor_ok(L, p.d)) {
    set_error("transform length " + std::to_string(L) +
              " must factor into 2, 3, 5, 7 and 11 (Nx and Ny must be 11-smooth)");
    return GIEM_EINVAL;
  }
  std::vector<c128> t64(L);
  std::vector<c64> t32(L);
  for (int k = 0; k < L; ++k) {
    long double a = -2.0L * 3.141592653589793238462643383279503L * (long double)k / (long double)L;
    t64[k] = mk<double>((double)cosl(a), (double)sinl(a));
    t32[k] = mk<float>((float)cosl(a), (float)sinl(a));
  }
  GIEM_HIP(hipMalloc(&p.tw64, L * sizeof(c128)), "hipMalloc twiddles");
  GIEM_HIP(hipMalloc(&p.tw32, L * sizeof(c64)), "hipMalloc twiddles");
  GIEM_HIP(hipMemcpy(p.tw64, t64.data(), L * sizeof(c128), hipMemcpyHostToDevice), "copy twiddles");
  GIEM_HIP(hipMemcpy(p.tw32, t32.data(), L * sizeof(c64), hipMemcpyHostToDevice), "copy twiddles");
  return GIEM_OK;
}

// Spectra workspace of giem_apply_noalloc: a fixed device array that every
// call on a device shares (the device holds it until the process ends).  In
// host code `scratch` is only a host-side stand-in for the symbol; its device
// address is looked up once per device (init_scratch, from the library's
// init call) and only that address is passed to kernels.
constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
static void *g_scratch_dev[kMaxDevices];
static std::mutex g_scratch_mu;

static int init_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) {
    set_error("device index out of range for the no-allocation workspace");
    return GIEM_EINVAL;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_dev[device]) return GIEM_OK;
  void *ptr = nullptr;
  GIEM_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
  g_scratch_dev[device] = ptr;
  return GIEM_OK;
}

static size_t spec_ws_need(const giem_handle *t, int nvec, unsigned prec) {
  const size_t c = prec == PREC_FP32 ? sizeof(c64) : sizeof(c128);
  return (size_t)2 * 4 * t->nx * t->ny * 3 * t->nz * nvec * c;
}

int ensure_spec_ws(giem_handle *t, int nrhs, int prec) {
  (void)prec;
  // two spectra buffers: the block product reads one and writes the other
  const size_t need = (size_t)2 * 4 * t->nx * t->ny * 3 * t->nz * nrhs * sizeof(c128);
  if (t->spec_ws_bytes >= need) return GIEM_OK;
  if (t->spec_ws) hipFree(t->spec_ws);
  t->spec_ws = nullptr;
  t->spec_ws_bytes = 0;
  GIEM_HIP(hipMalloc(&t->spec_ws, need), "hipMalloc spectra workspace");
  t->spec_ws_bytes = need;
  return GIEM_OK;
}

int compute_diagonals(giem_handle *t, const c128 *sigma_a, hipStream_t s) {
  c128 *dg = static_cast<c128 *>(t->diag);
  const size_t n = t->ncell();
  GIEM_HIP(launch_diagonals(sigma_a, static_cast<const c128 *>(t->sb_lev),
                            static_cast<const double *>(t->vol_lev), t->nx, t->ny, t->nz, dg,
                            dg + n, dg + 2 * n, dg + 3 * n, nullptr, s),
           "diagonals kernel");
  return GIEM_OK;
}

// Whether G sequences of length L on nthr threads can be launched.
static bool fft_shape_ok(int G, int nthr, int L, unsigned prec) {
  return G >= 1 && fft_ept(G, L, nthr, (int)prec) > 0 && fft_lds_bytes(G, L, (int)prec) <= 160 * 1024;
}

// Launch shape of the four FFT passes: the tuned one where set and valid,
// else 128-byte runs of planes (8 c128 or 16 c64) on 256 threads, halved
// until the sequences fit the per-thread register budget.
static void fft_shape(const giem_handle *t, unsigned prec, int G[4], int NT[4]) {
  const int pi = prec == PREC_FP32 ? 1 : 0;
  const int L[4] = {2 * t->nx, 2 * t->ny, 2 * t->ny, 2 * t->nx};
  for (int k = 0; k < 4; ++k) {
    if (t->fft_g[pi][k] > 0 && fft_shape_ok(t->fft_g[pi][k], t->fft_nt[pi][k], L[k], prec)) {
      G[k] = t->fft_g[pi][k];
      NT[k] = t->fft_nt[pi][k];
      continue;
    }
    int g = prec == PREC_FP32 ? 16 : 8;
    while (g > 1 && !fft_shape_ok(g, 256, L[k], prec)) g /= 2;
    G[k] = g;
    NT[k] = 256;
  }
}

// ws: spectra workspace of at least spec_ws_need() bytes supplied by the
// caller, or null for the handle's own (grown here when too small).
template <typename VT>
static int apply_core_t(giem_handle *t, int nf, const int *ifreqs, int nrhs,
                        const VecPtrsT<VT> &p, unsigned mode, unsigned prec, hipStream_t s,
                        double *stage_ms, void *ws = nullptr) {
  const int nx = t->nx, ny = t->ny, nz = t->nz;
  if (nf < 1 || nf > kMaxFreqBatch || nrhs < 1 || nrhs > kMaxRhs || nf * nrhs > kMaxVec) {
    set_error("apply: too many frequencies or vectors in one batched apply");
    return GIEM_EINVAL;
  }
  TabSet tabs{};
  for (int f = 0; f < nf; ++f) {
    if (ifreqs[f] < 0 || ifreqs[f] >= (int)t->f.size()) {
      set_error("apply: frequency index out of range");
      return GIEM_EINVAL;
    }
    const FreqTables &ft = t->f[ifreqs[f]];
    tabs.tab[f] = prec == PREC_FP32 ? ft.spec32 : ft.spec64;
    if (!tabs.tab[f]) {
      set_error("complex64 tables were not requested (GIEM_TABLES_C64)");
      return GIEM_EINVAL;
    }
  }
  const int nv = nf * nrhs;  // vectors of this apply, frequency-major
  if (!ws) GIEM_TRY(ensure_spec_ws(t, nv, prec));
  const c128 *dg = static_cast<const c128 *>(t->diag);
  const size_t n = t->ncell();
  const c128 *S = dg, *R1 = dg + n, *R2 = dg + 2 * n;
  const c128 *r2 = nullptr, *r1 = nullptr, *sd = nullptr;
  if (mode == MODE_A) {
    r2 = R2; r1 = R1; sd = S;
  } else if (mode == MODE_AT) {
    r2 = R1; r1 = R2; sd = S;
  }
  const int rp = nv * 3 * nz;
  int G[4], NT[4];
  fft_shape(t, prec, G, NT);
  if (!block_supported(nz, nrhs)) {
    set_error("block product: 3 Nz x nrhs too large for one workgroup");
    return GIEM_EINVAL;
  }
  const void *twx = prec == PREC_FP32 ? t->px.tw32 : t->px.tw64;
  const void *twy = prec == PREC_FP32 ? t->py.tw32 : t->py.tw64;
  const double scale = 1.0 / (4.0 * nx * ny);
  // Events around the five kernels: private ones for giem_apply_timed, pooled
  // ones (read back later by giem_profile_read) while profiling is on.
  hipEvent_t own[6];
  hipEvent_t *ev = nullptr;
  int only = -1;
  if (stage_ms) {
    for (int i = 0; i < 6; ++i) GIEM_HIP(hipEventCreate(&own[i]), "hipEventCreate");
    ev = own;
  } else if (t->prof && !ws) {
    const size_t need = t->prof_stage < 0 ? 6 : 2;
    while (t->prof_ev.size() < t->prof_used + need) {
      // timing only: no system-scope fence (a full L2 write-back) when the
      // event is recorded, which would stall the kernels around it
      hipEvent_t e;
      GIEM_HIP(hipEventCreateWithFlags(&e, hipEventDisableSystemFence), "hipEventCreate");
      t->prof_ev.push_back(e);
    }
    ev = t->prof_ev.data() + t->prof_used;
    t->prof_used += need;
    t->prof_meta.push_back((int)prec);
    t->prof_meta.push_back(nv);
    t->prof_meta.push_back(t->prof_stage);
    only = t->prof_stage;
  }
  // event i is recorded before kernel i (and i = 5 after the last); with one
  // kernel bracketed only its two events are recorded
  auto mark = [&](int i) -> int {
    if (!ev) return GIEM_OK;
    if (only < 0)
      GIEM_HIP(hipEventRecord(ev[i], s), "hipEventRecord");
    else if (i == only || i == only + 1)
      GIEM_HIP(hipEventRecord(ev[i - only], s), "hipEventRecord");
    return GIEM_OK;
  };
  const size_t cbytes = prec == PREC_FP32 ? sizeof(c64) : sizeof(c128);
  void *spa = ws ? ws : t->spec_ws;
  void *spb = static_cast<char *>(spa) + (size_t)4 * nx * ny * rp * cbytes;
  GIEM_TRY(mark(0));
  GIEM_HIP(launch_fft_x_fwd(prec, p, r2, spa, nx, ny, nz, rp, G[0], NT[0], t->px.d, twx, s),
           "x-FFT");
  GIEM_TRY(mark(1));
  GIEM_HIP(launch_fft_y(prec, spa, 2 * nx, ny, rp, G[1], NT[1], t->py.d, twy, 0, s), "y-FFT");
  GIEM_TRY(mark(2));
  const int bv = t->block_nbuf[prec == PREC_FP32 ? 1 : 0];
  const int nbuf = (bv >= 2 && bv <= 4) ? bv : 1;
  GIEM_HIP(launch_block(prec, tabs, nf, spa, spb, nx, ny, nz, nrhs, nbuf, s),
           "block product");
  GIEM_TRY(mark(3));
  GIEM_HIP(launch_fft_y(prec, spb, 2 * nx, ny, rp, G[2], NT[2], t->py.d, twy, 1, s),
           "inverse y-FFT");
  GIEM_TRY(mark(4));
  GIEM_HIP(launch_fft_x_inv(prec, p, sd, r1, spb, nx, ny, nz, rp, G[3], NT[3], t->px.d, twx, scale,
                            s),
           "inverse x-FFT");
  GIEM_TRY(mark(5));
  if (stage_ms) {
    GIEM_HIP(hipEventSynchronize(ev[5]), "hipEventSynchronize");
    for (int i = 0; i < 5; ++i) {
      float ms = 0.f;
      GIEM_HIP(hipEventElapsedTime(&ms, ev[i], ev[i + 1]), "hipEventElapsedTime");
      stage_ms[i] = ms;
    }
    for (int i = 0; i < 6; ++i) hipEventDestroy(own[i]);
  }
  return GIEM_OK;
}

int apply_core(giem_handle *t, int ifreq, int nrhs, const VecPtrs &p, unsigned mode,
               unsigned prec, hipStream_t s, double *stage_ms) {
  return apply_core_t(t, 1, &ifreq, nrhs, p, mode, prec, s, stage_ms);
}

int apply_core(giem_handle *t, int ifreq, int nrhs, const VecPtrs32 &p, unsigned mode,
               unsigned prec, hipStream_t s, double *stage_ms) {
  if (prec != PREC_FP32) {
    set_error("complex64 vectors need the FP32 operator");
    return GIEM_EINVAL;
  }
  return apply_core_t(t, 1, &ifreq, nrhs, p, mode, prec, s, stage_ms);
}

int apply_multi(giem_handle *t, int nf, const int *ifreqs, int nrhs, const VecPtrs &p,
                unsigned mode, unsigned prec, hipStream_t s) {
  return apply_core_t(t, nf, ifreqs, nrhs, p, mode, prec, s, nullptr);
}

int apply_multi(giem_handle *t, int nf, const int *ifreqs, int nrhs, const VecPtrs32 &p,
                unsigned mode, unsigned prec, hipStream_t s) {
  if (prec != PREC_FP32) {
    set_error("complex64 vectors need the FP32 operator");
    return GIEM_EINVAL;
  }
  return apply_core_t(t, nf, ifreqs, nrhs, p, mode, prec, s, nullptr);
}

// Packed spatial tables (device, kept for giem_tables_export) -> packed
// spectra (+ c64 copy).
int upload_spatial(giem_handle *t, hipStream_t s) {
  const int nx = t->nx, ny = t->ny, nz = t->nz, E = t->E();
  const size_t nsc = (size_t)(nx + 1) * (ny + 1) * E;
  void *tmp = nullptr;
  int rc = GIEM_OK;
  rc = check_hip(hipMalloc(&tmp, (size_t)ny * (nx + 1) * E * sizeof(c128)), "hipMalloc tmp");
  const int64_t row = (int64_t)(nx + 1) * E;
  for (size_t q = 0; rc == GIEM_OK && q < t->f.size(); ++q) {
    FreqTables &ft = t->f[q];
    if (rc == GIEM_OK) rc = check_hip(hipMalloc(&ft.spec64, nsc * sizeof(c128)), "hipMalloc spectra");
    // along x: tmp[i][K][e] from spatial[i][j][e]; along y: spectra[Ky][K][e]
    // from tmp[i][K][e] (the FFT passes of the apply at lengths 2 Nx, 2 Ny)
    if (rc == GIEM_OK)
      rc = check_hip(launch_parity_fft(static_cast<const c128 *>(ft.spatial), E, (int64_t)nx * E, ny,
                                       static_cast<c128 *>(tmp), E, row, nx, E, nz, 0, t->px.d,
                                       t->px.tw64, s),
                     "spectral x");
    if (rc == GIEM_OK)
      rc = check_hip(launch_parity_fft(static_cast<const c128 *>(tmp), row, E, nx + 1,
                                       static_cast<c128 *>(ft.spec64), row, E, ny, E, nz, 1, t->py.d,
                                       t->py.tw64, s),
                     "spectral y");
    if (rc == GIEM_OK && (t->flags & GIEM_TABLES_C64)) {
      rc = check_hip(hipMalloc(&ft.spec32, nsc * sizeof(c64)), "hipMalloc c64 spectra");
      if (rc == GIEM_OK)
        rc = check_hip(launch_to_c64(static_cast<c128 *>(ft.spec64), static_cast<c64 *>(ft.spec32), nsc, s),
                       "to c64");
    }
    if (rc == GIEM_OK) rc = check_hip(hipStreamSynchronize(s), "sync");
  }
  if (tmp) hipFree(tmp);
  return rc;
}

static int validate_model(const giem_model *m) {
  if (!m || m->nlay < 1 || !m->d || !m->sigma_b || !m->z_edges) {
    set_error("model: null pointer or nlay < 1");
    return GIEM_EINVAL;
  }
  if (m->nx < 1 || m->ny < 1 || m->nz < 1 || !(m->hx > 0) || !(m->hy > 0)) {
    set_error("model: grid sizes must be positive");
    return GIEM_EINVAL;
  }
  if (m->d[0] != 0.0) {
    set_error("model: the first interface must be the surface d_1 = 0");
    return GIEM_EINVAL;
  }
  for (int k = 1; k < m->nlay; ++k)
    if (!(m->d[k] > m->d[k - 1])) {
      set_error("model: interfaces must increase");
      return GIEM_EINVAL;
    }
  for (int k = 0; k < m->nz; ++k)
    if (!(m->z_edges[k + 1] > m->z_edges[k])) {
      set_error("model: z_edges must increase");
      return GIEM_EINVAL;
    }
  if (m->z_edges[0] < 0.0) {
    set_error("model: cells must lie in the earth (z >= 0)");
    return GIEM_EDOMAIN;
  }
  for (int k = 0; k <= m->nlay; ++k) {
    const double re = m->sigma_b[2 * k], im = m->sigma_b[2 * k + 1];
    if (!std::isfinite(re) || !std::isfinite(im) || re < 0.0) {
      set_error("model: sigma_b must be finite with Re >= 0");
      return GIEM_EDOMAIN;
    }
  }
  return GIEM_OK;
}

static int create_handle(const giem_model *m, int nfreq, const double *freq, uint32_t flags,
                         giem_handle **out) {
  GIEM_TRY(validate_model(m));
  if (nfreq < 1 || !freq || !out) {
    set_error("nfreq must be >= 1 with frequencies and an output pointer");
    return GIEM_EINVAL;
  }
  for (int q = 0; q < nfreq; ++q)
    if (!(freq[q] > 0.0) || !std::isfinite(freq[q])) {
      set_error("frequencies must be positive");
      return GIEM_EINVAL;
    }
  if (3 * m->nz * ((4 * kMaxRhs + 3) / 4) > 1024 * 4) {
    set_error("Nz too large");
    return GIEM_EINVAL;
  }
  if (m->nx > 2048 || m->ny > 2048) {
    set_error("Nx and Ny must not exceed 2048 (transform lengths up to 4096)");
    return GIEM_EINVAL;
  }
  giem_handle *t = new giem_handle();
  t->nx = m->nx; t->ny = m->ny; t->nz = m->nz; t->nlay = m->nlay;
  t->hx = m->hx; t->hy = m->hy; t->x0 = m->x0; t->y0 = m->y0;
  t->d.assign(m->d, m->d + m->nlay);
  t->z_edges.assign(m->z_edges, m->z_edges + m->nz + 1);
  for (int k = 0; k <= m->nlay; ++k) t->sigma.emplace_back(m->sigma_b[2 * k], m->sigma_b[2 * k + 1]);
  t->flags = flags;
  hipGetDevice(&t->device);
  {
    const int rc = init_scratch(t->device);
    if (rc != GIEM_OK) {
      delete t;
      return rc;
    }
  }
  // layer of every cell; no cell may straddle an interface
  for (int k = 0; k < t->nz; ++k) {
    const double a = t->z_edges[k], b = t->z_edges[k + 1];
    for (double di : t->d)
      if (a < di && di < b) {
        set_error("a cell straddles an interface (the vertical integrals need one layer per cell)");
        delete t;
        return GIEM_EDOMAIN;
      }
    const double mid = 0.5 * (a + b);
    int lay = 0;
    while (lay < t->nlay && t->d[lay] <= mid) ++lay;
    t->layer_of_cell.push_back(lay);
    if (lay == 0) {
      set_error("cells must lie below the surface d[0] (the anomaly domain is in the earth)");
      delete t;
      return GIEM_EDOMAIN;
    }
    if (!(t->sigma[lay].real() > 0.0)) {
      set_error("Re sigma_b must be positive in every layer that holds cells");
      delete t;
      return GIEM_EDOMAIN;
    }
  }
  t->f.resize(nfreq);
  for (int q = 0; q < nfreq; ++q) t->f[q].freq = freq[q];
  *out = t;
  return GIEM_OK;
}

// Launch shapes chosen by giem_tune, kept for the process and given to
// handles created later for the same grid on the same device.
struct TunedShapes {
  int fft_g[2][4], fft_nt[2][4], block_nbuf[2];
};
static std::mutex g_tuned_mu;
static std::map<std::array<int, 4>, TunedShapes> g_tuned;

static std::array<int, 4> tuned_key(const giem_handle *t) {
  return {t->device, t->nx, t->ny, t->nz};
}

static void remember_tuned(const giem_handle *t) {
  TunedShapes e;
  std::memcpy(e.fft_g, t->fft_g, sizeof(e.fft_g));
  std::memcpy(e.fft_nt, t->fft_nt, sizeof(e.fft_nt));
  std::memcpy(e.block_nbuf, t->block_nbuf, sizeof(e.block_nbuf));
  std::lock_guard<std::mutex> lk(g_tuned_mu);
  g_tuned[tuned_key(t)] = e;
}

static void recall_tuned(giem_handle *t) {
  std::lock_guard<std::mutex> lk(g_tuned_mu);
  auto it = g_tuned.find(tuned_key(t));
  if (it == g_tuned.end()) return;
  std::memcpy(t->fft_g, it->second.fft_g, sizeof(t->fft_g));
  std::memcpy(t->fft_nt, it->second.fft_nt, sizeof(t->fft_nt));
  std::memcpy(t->block_nbuf, it->second.block_nbuf, sizeof(t->block_nbuf));
}

static int finish_handle(giem_handle *t, hipStream_t s) {
  static bool lds_set = false;
  if (!lds_set) {
    GIEM_HIP(set_lds_limits(), "hipFuncSetAttribute");
    lds_set = true;
  }
  const int nz = t->nz;
  if (!block_supported(nz, 1)) {
    set_error("Nz too large for the packed block offsets");
    return GIEM_EINVAL;
  }
  recall_tuned(t);
  GIEM_TRY(make_plan(2 * t->nx, t->px));
  GIEM_TRY(make_plan(2 * t->ny, t->py));
  std::vector<c128> sb(nz);
  std::vector<double> vol(nz), sr(nz);
  for (int k = 0; k < nz; ++k) {
    cd s0 = t->sigma[t->layer_of_cell[k]];
    sb[k] = mk<double>(s0.real(), s0.imag());
    vol[k] = t->hx * t->hy * (t->z_edges[k + 1] - t->z_edges[k]);
    sr[k] = std::sqrt(s0.real());
  }
  GIEM_HIP(hipMalloc(&t->sb_lev, nz * sizeof(c128)), "hipMalloc");
  GIEM_HIP(hipMalloc(&t->vol_lev, nz * sizeof(double)), "hipMalloc");
  GIEM_HIP(hipMalloc(&t->sroot_lev, nz * sizeof(double)), "hipMalloc");
  GIEM_HIP(hipMemcpy(t->sb_lev, sb.data(), nz * sizeof(c128), hipMemcpyHostToDevice), "copy");
  GIEM_HIP(hipMemcpy(t->vol_lev, vol.data(), nz * sizeof(double), hipMemcpyHostToDevice), "copy");
  GIEM_HIP(hipMemcpy(t->sroot_lev, sr.data(), nz * sizeof(double), hipMemcpyHostToDevice), "copy");
  GIEM_HIP(hipMalloc(&t->diag, 4 * t->ncell() * sizeof(c128)), "hipMalloc diagonals");
  const size_t nred = (size_t)kMaxRhs * 65 * dot_partials_per_rhs();
  GIEM_HIP(hipMalloc(&t->red_part, nred * sizeof(c128)), "hipMalloc");
  GIEM_HIP(hipMalloc(&t->red_out, kMaxSys * 65 * sizeof(c128)), "hipMalloc");
  GIEM_HIP(hipHostMalloc(&t->red_host, kMaxSys * 65 * sizeof(c128), 0), "hipHostMalloc");
  GIEM_HIP(hipMalloc(&t->coef_dev, kMaxSys * 65 * sizeof(c128)), "hipMalloc");
  GIEM_HIP(hipHostMalloc(&t->coef_host, kMaxSys * 65 * sizeof(c128), 0), "hipHostMalloc");
  GIEM_HIP(hipMalloc(&t->gs_scale_dev, kMaxSys * 65 * sizeof(double)), "hipMalloc");
  GIEM_HIP(hipHostMalloc(&t->gs_scale_host, kMaxSys * 65 * sizeof(double), 0), "hipHostMalloc");
  GIEM_TRY(ensure_spec_ws(t, 2, PREC_FP64));
  return upload_spatial(t, s);
}

}  // namespace giem

using namespace giem;

extern "C" {

const char *giem_last_error(void) { return get_error().c_str(); }

void giem_free(giem_handle *t) {
  if (!t) return;
  for (auto &ft : t->f) {
    if (ft.spatial) hipFree(ft.spatial);
    if (ft.spec64) hipFree(ft.spec64);
    if (ft.spec32) hipFree(ft.spec32);
    for (auto &rk : ft.rec_kernels) hipFree(rk.second);
  }
  void *dev[] = {t->px.tw64, t->px.tw32, t->py.tw64, t->py.tw32,
                 t->sb_lev, t->vol_lev, t->sroot_lev, t->diag, t->spec_ws, t->red_part,
                 t->red_out, t->coef_dev, t->basis, t->vec_ws, t->gs_scale_dev};
  for (void *p : dev)
    if (p) hipFree(p);
  if (t->red_host) hipHostFree(t->red_host);
  if (t->coef_host) hipHostFree(t->coef_host);
  if (t->gs_scale_host) hipHostFree(t->gs_scale_host);
  for (hipEvent_t e : t->prof_ev) hipEventDestroy(e);
  delete t;
}

int giem_tables_import(const giem_model *model, int32_t nfreq, const double *freq_hz,
                       const void *host_packed_spatial, uint32_t flags, void *stream,
                       giem_handle **out) {
  if (!host_packed_spatial) {
    set_error("host_packed_spatial is null");
    return GIEM_EINVAL;
  }
  giem_handle *t = nullptr;
  GIEM_TRY(create_handle(model, nfreq, freq_hz, flags, &t));
  const size_t nsp = (size_t)t->nx * t->ny * t->E();
  const cd *src = static_cast<const cd *>(host_packed_spatial);
  int rc = GIEM_OK;
  for (int q = 0; q < nfreq && rc == GIEM_OK; ++q) {
    rc = check_hip(hipMalloc(&t->f[q].spatial, nsp * sizeof(c128)), "hipMalloc spatial table");
    if (rc == GIEM_OK)
      rc = check_hip(hipMemcpy(t->f[q].spatial, src + q * nsp, nsp * sizeof(c128), hipMemcpyHostToDevice),
                     "copy spatial table");
  }
  if (rc < 0) {
    giem_free(t);
    return rc;
  }
  rc = finish_handle(t, static_cast<hipStream_t>(stream));
  if (rc < 0) {
    giem_free(t);
    return rc;
  }
  *out = t;
  return GIEM_OK;
}

int giem_tables(const giem_model *model, int32_t nfreq, const double *freq_hz, uint32_t flags,
                void *stream, giem_handle **out) {
  giem_handle *t = nullptr;
  GIEM_TRY(create_handle(model, nfreq, freq_hz, flags, &t));
  int rc = compute_tables(t, static_cast<hipStream_t>(stream));
  if (rc < 0) {
    giem_free(t);
    return rc;
  }
  rc = finish_handle(t, static_cast<hipStream_t>(stream));
  if (rc < 0) {
    giem_free(t);
    return rc;
  }
  *out = t;
  return GIEM_OK;
}

int giem_tables_export(const giem_handle *t, int32_t ifreq, void *host_packed_spatial) {
  if (!t || !host_packed_spatial || ifreq < 0 || ifreq >= (int)t->f.size()) {
    set_error("giem_tables_export: bad handle, frequency index or pointer");
    return GIEM_EINVAL;
  }
  const size_t nsp = (size_t)t->nx * t->ny * t->E();
  if (check_hip(hipMemcpy(host_packed_spatial, t->f[ifreq].spatial, nsp * sizeof(c128),
                          hipMemcpyDeviceToHost),
                "copy spatial table"))
    return GIEM_EHIP;
  return GIEM_OK;
}

int giem_tables_bytes(const giem_handle *t, int64_t *b128, int64_t *b64) {
  if (!t) {
    set_error("null handle");
    return GIEM_EINVAL;
  }
  const int64_t n = (int64_t)(t->nx + 1) * (t->ny + 1) * t->E();
  if (b128) *b128 = n * (int64_t)sizeof(c128);
  if (b64) *b64 = (t->flags & GIEM_TABLES_C64) ? n * (int64_t)sizeof(c64) : 0;
  return GIEM_OK;
}

static int apply_entry(giem_handle *t, int32_t ifreq, const void *sigma_a, int32_t nrhs,
                       const void *x, void *y, uint32_t mode, uint32_t prec, void *stream,
                       double *stage_ms) {
  if (!t || ifreq < 0 || ifreq >= (int)t->f.size() || nrhs < 1 || nrhs > kMaxRhs || !x || !y ||
      mode > MODE_B || prec > PREC_FP32 || (mode != MODE_B && !sigma_a)) {
    set_error("giem_apply: bad argument");
    return GIEM_EINVAL;
  }
  const size_t nbytes = (size_t)nrhs * t->nvec() * sizeof(c128);
  const char *xa = static_cast<const char *>(x), *ya = static_cast<const char *>(y);
  if (xa < ya + nbytes && ya < xa + nbytes) {
    set_error("giem_apply: x and y overlap");
    return GIEM_EINVAL;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (mode != MODE_B) GIEM_TRY(compute_diagonals(t, static_cast<const c128 *>(sigma_a), s));
  VecPtrs p{};
  for (int r = 0; r < nrhs; ++r) {
    p.in[r] = static_cast<const c128 *>(x) + r * t->nvec();
    p.out[r] = static_cast<c128 *>(y) + r * t->nvec();
  }
  return apply_core(t, ifreq, nrhs, p, mode, prec, s, stage_ms);
}

int giem_apply(giem_handle *t, int32_t ifreq, const void *sigma_a, int32_t nrhs, const void *x,
               void *y, uint32_t mode, uint32_t prec, void *stream) {
  return apply_entry(t, ifreq, sigma_a, nrhs, x, y, mode, prec, stream, nullptr);
}

int giem_apply_noalloc(giem_handle *t, int32_t ifreq, const void *sigma_a, int32_t nrhs,
                       const void *x, void *y, uint32_t mode, uint32_t prec, void *stream) {
  if (!t || ifreq < 0 || ifreq >= (int)t->f.size() || nrhs < 1 || nrhs > kMaxRhs || !x || !y ||
      mode > MODE_B || prec > PREC_FP32 || (mode != MODE_B && !sigma_a)) {
    set_error("giem_apply_noalloc: bad argument");
    return GIEM_EINVAL;
  }
  const size_t need = spec_ws_need(t, nrhs, prec);
  if (need > kScratchBytes) {
    set_error("giem_apply_noalloc: spectra of " + std::to_string(need) +
              " bytes exceed the fixed workspace of " + std::to_string(kScratchBytes) + " bytes");
    return GIEM_EINVAL;
  }
  int dev = -1;
  GIEM_HIP(hipGetDevice(&dev), "hipGetDevice");
  if (dev != t->device || !g_scratch_dev[dev]) {
    set_error("giem_apply_noalloc: the handle's device must be current");
    return GIEM_EINVAL;
  }
  const size_t nbytes = (size_t)nrhs * t->nvec() * sizeof(c128);
  const char *xa = static_cast<const char *>(x), *ya = static_cast<const char *>(y);
  if (xa < ya + nbytes && ya < xa + nbytes) {
    set_error("giem_apply_noalloc: x and y overlap");
    return GIEM_EINVAL;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (mode != MODE_B) GIEM_TRY(compute_diagonals(t, static_cast<const c128 *>(sigma_a), s));
  VecPtrs p{};
  for (int r = 0; r < nrhs; ++r) {
    p.in[r] = static_cast<const c128 *>(x) + r * t->nvec();
    p.out[r] = static_cast<c128 *>(y) + r * t->nvec();
  }
  return apply_core_t(t, 1, &ifreq, nrhs, p, mode, prec, s, nullptr, g_scratch_dev[dev]);
}

int giem_apply_batch(giem_handle *t, int32_t nf, const int32_t *ifreqs, const void *sigma_a,
                     int32_t nrhs, const void *x, void *y, uint32_t mode, uint32_t prec,
                     void *stream) {
  if (!t || nf < 1 || nf > kMaxFreqBatch || !ifreqs || nrhs < 1 || nrhs > kMaxRhs ||
      nf * nrhs > kMaxVec || !x || !y || mode > MODE_B || prec > PREC_FP32 ||
      (mode != MODE_B && !sigma_a)) {
    set_error("giem_apply_batch: bad argument");
    return GIEM_EINVAL;
  }
  int ifr[kMaxFreqBatch];
  for (int f = 0; f < nf; ++f) {
    if (ifreqs[f] < 0 || ifreqs[f] >= (int)t->f.size()) {
      set_error("giem_apply_batch: frequency index out of range");
      return GIEM_EINVAL;
    }
    ifr[f] = ifreqs[f];
  }
  const int nv = nf * nrhs;
  const size_t nbytes = (size_t)nv * t->nvec() * sizeof(c128);
  const char *xa = static_cast<const char *>(x), *ya = static_cast<const char *>(y);
  if (xa < ya + nbytes && ya < xa + nbytes) {
    set_error("giem_apply_batch: x and y overlap");
    return GIEM_EINVAL;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (mode != MODE_B) GIEM_TRY(compute_diagonals(t, static_cast<const c128 *>(sigma_a), s));
  VecPtrs p{};
  for (int v = 0; v < nv; ++v) {
    p.in[v] = static_cast<const c128 *>(x) + (size_t)v * t->nvec();
    p.out[v] = static_cast<c128 *>(y) + (size_t)v * t->nvec();
  }
  return apply_multi(t, nf, ifr, nrhs, p, mode, prec, s);
}

int giem_apply_timed(giem_handle *t, int32_t ifreq, const void *sigma_a, int32_t nrhs,
                     const void *x, void *y, uint32_t mode, uint32_t prec, void *stream,
                     double *stage_ms) {
  if (!stage_ms) {
    set_error("stage_ms is null");
    return GIEM_EINVAL;
  }
  return apply_entry(t, ifreq, sigma_a, nrhs, x, y, mode, prec, stream, stage_ms);
}

int giem_tune(giem_handle *t, int32_t ifreq, const void *sigma_a, int32_t nrhs, void *stream,
              int32_t *chosen) {
  if (!t || ifreq < 0 || ifreq >= (int)t->f.size() || nrhs < 1 || nrhs > kMaxRhs || !sigma_a) {
    set_error("giem_tune: bad argument");
    return GIEM_EINVAL;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  GIEM_TRY(compute_diagonals(t, static_cast<const c128 *>(sigma_a), s));
  const size_t nbytes = (size_t)nrhs * t->nvec() * sizeof(c128);
  void *x = nullptr, *y = nullptr;
  struct Free {
    void **a, **b;
    ~Free() {
      if (*a) hipFree(*a);
      if (*b) hipFree(*b);
    }
  } fr{&x, &y};
  GIEM_HIP(hipMalloc(&x, nbytes), "hipMalloc tuning input");
  GIEM_HIP(hipMalloc(&y, nbytes), "hipMalloc tuning output");
  GIEM_HIP(hipMemsetAsync(x, 0x3f, nbytes, s), "fill tuning input");  // doubles of order 1e-4
  VecPtrs p{};
  for (int r = 0; r < nrhs; ++r) {
    p.in[r] = static_cast<const c128 *>(x) + r * t->nvec();
    p.out[r] = static_cast<c128 *>(y) + r * t->nvec();
  }
  const int L[4] = {2 * t->nx, 2 * t->ny, 2 * t->ny, 2 * t->nx};
  const int stage_of_pass[4] = {0, 1, 3, 4};
  for (int pi = 0; pi < 2; ++pi) {
    const unsigned prec = pi ? PREC_FP32 : PREC_FP64;
    const bool have = pi ? t->f[ifreq].spec32 != nullptr : t->f[ifreq].spec64 != nullptr;
    if (!have) {
      for (int k = 0; k < 4; ++k) t->fft_g[pi][k] = t->fft_nt[pi][k] = 0;
      continue;
    }
    // candidates: FFT shapes (applied to all four passes at once) and the
    // block-product prefetch depth; two interleaved rounds of seven timed
    // applies each, the best median per candidate counts
    struct Cand {
      int g, nt, nbuf;
    };
    std::vector<Cand> cands;
    for (int nt : {256, 512})
      for (int g = 1; g <= 64; g *= 2) {
        bool any = false;
        for (int k = 0; k < 4; ++k) any = any || fft_shape_ok(g, nt, L[k], prec);
        if (any) cands.push_back({g, nt, 0});
      }
    cands.push_back({0, 0, 1});
    cands.push_back({0, 0, 2});
    if (block_two_per_cu(t->nz, nrhs, (int)prec)) cands.push_back({0, 0, 3});
    if (block_dbl_supported(t->nz, nrhs, (int)prec)) cands.push_back({0, 0, 4});
    std::vector<std::array<double, 5>> med(cands.size());
    for (auto &m : med) m.fill(1e30);
    for (int round = 0; round < 2; ++round)
      for (size_t c = 0; c < cands.size(); ++c) {
        const Cand &cd = cands[c];
        for (int k = 0; k < 4; ++k) {
          t->fft_g[pi][k] = cd.g;
          t->fft_nt[pi][k] = cd.nt;
        }
        t->block_nbuf[pi] = cd.nbuf;
        double st[5];
        for (int w = 0; w < 2; ++w) GIEM_TRY(apply_core(t, ifreq, nrhs, p, MODE_A, prec, s, st));
        std::vector<double> ms[5];
        for (int rep = 0; rep < 7; ++rep) {
          GIEM_TRY(apply_core(t, ifreq, nrhs, p, MODE_A, prec, s, st));
          for (int k = 0; k < 5; ++k) ms[k].push_back(st[k]);
        }
        for (int k = 0; k < 5; ++k) {
          std::sort(ms[k].begin(), ms[k].end());
          med[c][k] = std::min(med[c][k], ms[k][3]);
        }
      }
    double best[4] = {1e30, 1e30, 1e30, 1e30};
    int bg[4] = {0, 0, 0, 0}, bt[4] = {0, 0, 0, 0};
    double bbest = 1e30;
    int bnb = 1;
    for (size_t c = 0; c < cands.size(); ++c) {
      const Cand &cd = cands[c];
      if (cd.g > 0) {
        for (int k = 0; k < 4; ++k) {
          if (!fft_shape_ok(cd.g, cd.nt, L[k], prec)) continue;
          const double v = med[c][stage_of_pass[k]];
          if (v < best[k]) {
            best[k] = v;
            bg[k] = cd.g;
            bt[k] = cd.nt;
          }
        }
      } else if (med[c][2] < bbest) {
        bbest = med[c][2];
        bnb = cd.nbuf;
      }
    }
    for (int k = 0; k < 4; ++k) {
      t->fft_g[pi][k] = bg[k];
      t->fft_nt[pi][k] = bt[k];
    }
    t->block_nbuf[pi] = bnb;
  }
  remember_tuned(t);
  if (chosen) {
    for (int pi = 0; pi < 2; ++pi) {
      int G[4], NT[4];
      fft_shape(t, pi ? PREC_FP32 : PREC_FP64, G, NT);
      for (int k = 0; k < 4; ++k) {
        chosen[(pi * 5 + k) * 2] = G[k];
        chosen[(pi * 5 + k) * 2 + 1] = NT[k];
      }
      const int bv = t->block_nbuf[pi];
      chosen[(pi * 5 + 4) * 2] = (bv >= 2 && bv <= 4) ? bv : 1;
      chosen[(pi * 5 + 4) * 2 + 1] = 0;
    }
  }
  return GIEM_OK;
}

int giem_set_fft_shape(giem_handle *t, uint32_t prec, const int32_t *shape) {
  if (!t || prec > PREC_FP32) {
    set_error("giem_set_fft_shape: bad argument");
    return GIEM_EINVAL;
  }
  const int pi = prec == PREC_FP32 ? 1 : 0;
  if (!shape) {
    for (int k = 0; k < 4; ++k) t->fft_g[pi][k] = t->fft_nt[pi][k] = 0;
    return GIEM_OK;
  }
  const int L[4] = {2 * t->nx, 2 * t->ny, 2 * t->ny, 2 * t->nx};
  for (int k = 0; k < 4; ++k)
    if (!fft_shape_ok(shape[2 * k], shape[2 * k + 1], L[k], prec)) {
      set_error("giem_set_fft_shape: pass " + std::to_string(k) + " cannot run " +
                std::to_string(shape[2 * k]) + " sequences on " + std::to_string(shape[2 * k + 1]) +
                " threads");
      return GIEM_EINVAL;
    }
  for (int k = 0; k < 4; ++k) {
    t->fft_g[pi][k] = shape[2 * k];
    t->fft_nt[pi][k] = shape[2 * k + 1];
  }
  return GIEM_OK;
}

int giem_set_block_buffers(giem_handle *t, uint32_t prec, int32_t nbuf) {
  if (!t || prec > PREC_FP32 || nbuf < 0 || nbuf > 4) {
    set_error("giem_set_block_buffers: bad argument (0 to 4)");
    return GIEM_EINVAL;
  }
  t->block_nbuf[prec == PREC_FP32 ? 1 : 0] = nbuf;
  return GIEM_OK;
}

int giem_profile(giem_handle *t, int32_t enable) {
  if (!t || enable < 0 || enable > 6) {
    set_error("giem_profile: null handle or enable outside 0 .. 6");
    return GIEM_EINVAL;
  }
  t->prof = enable != 0;
  t->prof_stage = enable >= 2 ? enable - 2 : -1;
  t->prof_used = 0;
  t->prof_meta.clear();
  t->prof_discarded[0] = t->prof_discarded[1] = 0;
  return GIEM_OK;
}

int giem_profile_read(giem_handle *t, double *stage_ms, int64_t *applies, int64_t *rhs) {
  if (!t || !stage_ms || !applies || !rhs) {
    set_error("giem_profile_read: null argument");
    return GIEM_EINVAL;
  }
  for (int i = 0; i < 10; ++i) stage_ms[i] = 0.0;
  for (int i = 0; i < 2; ++i) applies[i] = rhs[i] = 0;
  const size_t napp = t->prof_meta.size() / 3;
  if (napp) GIEM_HIP(hipEventSynchronize(t->prof_ev[t->prof_used - 1]), "hipEventSynchronize");
  size_t off = 0;
  for (size_t a = 0; a < napp; ++a) {
    const int pr = t->prof_meta[3 * a] == PREC_FP32 ? 1 : 0;
    const int only = t->prof_meta[3 * a + 2];
    const hipEvent_t *ev = t->prof_ev.data() + off;
    if (only < 0) {
      for (int i = 0; i < 5; ++i) {
        float ms = 0.f;
        GIEM_HIP(hipEventElapsedTime(&ms, ev[i], ev[i + 1]), "hipEventElapsedTime");
        stage_ms[5 * pr + i] += ms;
      }
      off += 6;
    } else {
      float ms = 0.f;
      GIEM_HIP(hipEventElapsedTime(&ms, ev[0], ev[1]), "hipEventElapsedTime");
      stage_ms[5 * pr + only] += ms;
      off += 2;
    }
    applies[pr] += 1;
    rhs[pr] += t->prof_meta[3 * a + 1];
  }
  for (int i = 0; i < 2; ++i) rhs[i] = std::max<int64_t>(0, rhs[i] - t->prof_discarded[i]);
  t->prof_used = 0;
  t->prof_meta.clear();
  t->prof_discarded[0] = t->prof_discarded[1] = 0;
  return GIEM_OK;
}

}  // extern "C"
