// GMRES driver (Sect. 3.3: the system is solved by flexible GMRES; without a
// preconditioner it reduces to GMRES(m)), the precision form (complex64
// convolution inside an inner GMRES, FP64 residual refinement outside), the
// adjoint solve, and the plane-wave normal field used for the right-hand side
// (Sect. 2.1).  The Arnoldi vectors are complex128 (complex64 in the inner
// solve of the precision form) and all inner products are accumulated in FP64
// on the device; the Hessenberg matrix, the Givens rotations and the small
// least-squares problem are FP64 on the host.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>

#include "handle.h"

namespace giem {

#define GIEM_TRY(expr)          \
  do {                          \
    int rc__ = (expr);          \
    if (rc__ < 0) return rc__;  \
  } while (0)
#define GIEM_HIP(expr, what) GIEM_TRY(check_hip((expr), (what)))

static const double kMu0 = 4e-7 * 3.14159265358979323846;

// ------------------------------------------------------------ normal field
// 1-D plane wave in the layered earth, exp(-i w t), E'' + k^2 E = 0 with
// k^2 = i w mu0 sigma, Im k >= 0, E(0) = 1.  In layer m (between d[m-1] and
// d[m]) E = a_m (e^{ik(z-d[m])} + r_m e^{-ik(z-d[m])}); r_m follows from the
// impedance of the medium below, evaluated from the lower half-space up.
struct PlaneWave {
  std::vector<cd> k, a, r;
  std::vector<double> d;
  int nl = 0;
  cd Zs;
  double omega = 0;

  PlaneWave(const std::vector<double> &dd, const std::vector<cd> &sigma, double freq) {
    d = dd;
    nl = (int)d.size();
    omega = 2.0 * M_PI * freq;
    k.resize(nl + 1);
    for (int m = 0; m <= nl; ++m) {
      cd kk = std::sqrt(cd(0.0, omega * kMu0) * sigma[m]);
      if (kk.imag() < 0) kk = -kk;
      k[m] = kk;
    }
    r.assign(nl + 1, 0.0);
    a.assign(nl + 1, 0.0);
    auto z0 = [&](int m) { return omega * kMu0 / k[m]; };
    cd zb = z0(nl);
    for (int m = nl - 1; m >= 1; --m) {
      const double l = d[m] - d[m - 1];
      const cd rr = (zb - z0(m)) / (zb + z0(m));
      r[m] = rr;
      const cd e = std::exp(cd(0, 2) * k[m] * l);
      zb = z0(m) * (1.0 + rr * e) / (1.0 - rr * e);
    }
    Zs = zb;
    cd etop = 1.0;
    for (int m = 1; m < nl; ++m) {
      const double l = d[m] - d[m - 1];
      const cd e = std::exp(cd(0, 1) * k[m] * l);
      a[m] = etop * e / (1.0 + r[m] * e * e);
      etop = a[m] * (1.0 + r[m]);
    }
    a[nl] = etop;
  }
  int layer(double z) const {
    int m = 0;
    while (m < nl && d[m] <= z) ++m;
    return m;
  }
  // E and dE/dz at depth z in the earth (z >= d[0])
  cd value(double z, cd *dz) const {
    const int m = layer(z);
    const cd ik = cd(0, 1) * k[m];
    if (m == nl) {
      const cd e = a[m] * std::exp(ik * (z - d[m - 1]));
      *dz = ik * e;
      return e;
    }
    const cd up = std::exp(ik * (z - d[m])), dn = std::exp(-ik * (z - d[m]));
    *dz = ik * a[m] * (up - r[m] * dn);
    return a[m] * (up + r[m] * dn);
  }
  // mean of E over [z1, z2] inside one earth layer
  cd average(double z1, double z2) const {
    const int m = layer(0.5 * (z1 + z2));
    const cd ik = cd(0, 1) * k[m];
    cd v;
    if (m == nl) {
      const double dd = d[m - 1];
      v = a[m] * (std::exp(ik * (z2 - dd)) - std::exp(ik * (z1 - dd))) / ik;
    } else {
      const double dm = d[m];
      const cd up = (std::exp(ik * (z2 - dm)) - std::exp(ik * (z1 - dm))) / ik;
      const cd dn = (std::exp(-ik * (z2 - dm)) - std::exp(-ik * (z1 - dm))) / (-ik);
      v = a[m] * (up + r[m] * dn);
    }
    return v / (z2 - z1);
  }
};

int plane_wave_levels(const giem_handle *t, double freq, std::vector<cd> &en_lev,
                      std::vector<cd> &hsurf) {
  PlaneWave pw(t->d, t->sigma, freq);
  en_lev.resize(t->nz);
  for (int k = 0; k < t->nz; ++k) en_lev[k] = pw.average(t->z_edges[k], t->z_edges[k + 1]);
  hsurf.assign(1, 1.0 / pw.Zs);
  return GIEM_OK;
}

// ------------------------------------------------------------ GMRES(m)
struct GmresParams {
  double tol = 1e-6;
  int m = 30;
  int max_iter = 1000;
  int weighted = 0;
  unsigned mode = MODE_A;
  unsigned prec = PREC_FP64;
  bool x_zero = true;
};

// Relative tolerance of one inner solve of the precision form: the inner
// tolerance itol, relaxed where less is enough, i.e. where a correction that
// reduces the residual of every unconverged system q by the factor
// 0.5 tol |b_q| / |r_q| already meets the outer tolerance (in practice the
// last refinement step, which would otherwise solve its correction far past
// the outer tolerance).  The outer loop still checks the true FP64 residual.
static double inner_tolerance(double itol, double tol, const std::vector<int> &act,
                              const std::vector<double> &normb, const std::vector<double> &rn) {
  double need = 0.5;
  for (int q : act)
    if (rn[q] > 0) need = std::min(need, 0.5 * tol * normb[q] / rn[q]);
  return std::max(itol, need);
}

// Residual history of one frequency's right-hand sides q0 .. q0 + nq - 1 into
// the stats: entry k is the largest k-th recorded residual among them, a
// system that stopped earlier counting with its final residual (so the last
// entry is the largest final residual); beyond GIEM_HISTORY entries the
// first GIEM_HISTORY - 1 and the last are kept.
static void fill_history(giem_solve_stats &st, const std::vector<std::vector<double>> &hist,
                         int q0, int nq) {
  size_t len = 0;
  for (int q = q0; q < q0 + nq; ++q) len = std::max(len, hist[q].size());
  auto at = [&](size_t k) {
    double v = 0.0;
    for (int q = q0; q < q0 + nq; ++q)
      if (!hist[q].empty()) v = std::max(v, hist[q][std::min(k, hist[q].size() - 1)]);
    return v;
  };
  st.n_history = (int32_t)std::min<size_t>(len, GIEM_HISTORY);
  for (int k = 0; k < st.n_history; ++k)
    st.history[k] = (len > GIEM_HISTORY && k == GIEM_HISTORY - 1) ? at(len - 1) : at(k);
}

struct GmresResult {
  int iters = 0;      // operator applies inside Arnoldi (max over RHS)
  int restarts = 0;
  std::vector<double> relres;  // final true residual / ||b||
  // per system: the true residual / ||b|| at the start of every restart
  // cycle, the last one being the final residual
  std::vector<std::vector<double>> hist;
  bool converged = false;
};

static int ensure_basis(giem_handle *t, int nrhs, int m) {
  const size_t need = (size_t)nrhs * (m + 1) * t->nvec() * sizeof(c128);
  if (t->basis_bytes >= need) return GIEM_OK;
  if (t->basis) hipFree(t->basis);
  t->basis = nullptr;
  t->basis_bytes = 0;
  GIEM_HIP(hipMalloc(&t->basis, need), "hipMalloc Krylov basis");
  t->basis_bytes = need;
  return GIEM_OK;
}

static int ensure_vec_ws(giem_handle *t, size_t nvecs) {
  const size_t need = nvecs * t->nvec() * sizeof(c128);
  if (t->vec_ws_bytes >= need) return GIEM_OK;
  if (t->vec_ws) hipFree(t->vec_ws);
  t->vec_ws = nullptr;
  t->vec_ws_bytes = 0;
  GIEM_HIP(hipMalloc(&t->vec_ws, need), "hipMalloc vector workspace");
  t->vec_ws_bytes = need;
  return GIEM_OK;
}

// weighted squared norms of nv vectors (each at its own pointer)
template <typename VT>
static int norms_of(giem_handle *t, const VT *const *v, int nv, const double *wlev,
                    hipStream_t s, std::vector<double> &out) {
  c128 *part = static_cast<c128 *>(t->red_part);
  c128 *res = static_cast<c128 *>(t->coef_dev);
  const int plane = t->nx * t->ny;
  for (int r = 0; r < nv; ++r)
    GIEM_HIP(launch_norms(v[r], 1, t->nvec(), t->nz, plane, wlev, part, res + r, s), "norm kernel");
  GIEM_HIP(hipMemcpyAsync(t->coef_host, res, nv * sizeof(c128), hipMemcpyDeviceToHost, s), "copy norms");
  GIEM_HIP(hipStreamSynchronize(s), "sync");
  out.resize(nv);
  const c128 *h = static_cast<const c128 *>(t->coef_host);
  for (int r = 0; r < nv; ++r) out[r] = std::sqrt(std::max(h[r].x, 0.0));
  return GIEM_OK;
}

// y_r = op(x_r) for a set of RHS given by pointers (batched in groups of 8)
template <typename VT>
static int apply_ptrs(giem_handle *t, int ifreq, const std::vector<const VT *> &in,
                      const std::vector<VT *> &out, unsigned mode, unsigned prec,
                      hipStream_t s) {
  for (size_t b0 = 0; b0 < in.size(); b0 += kMaxRhs) {
    const int nb = (int)std::min<size_t>(kMaxRhs, in.size() - b0);
    VecPtrsT<VT> p{};
    for (int r = 0; r < nb; ++r) {
      p.in[r] = in[b0 + r];
      p.out[r] = out[b0 + r];
    }
    GIEM_TRY(apply_core(t, ifreq, nb, p, mode, prec, s, nullptr));
  }
  return GIEM_OK;
}

// y = op x for systems of several frequencies: in[i], out[i] belong to system
// sys[i], whose operator is frequency fq[sys[i]].  The vectors of each
// frequency are cut into chunks of at most kMaxRhs; chunks of equal size are
// applied together, one launch per kernel for up to kMaxFreqBatch
// frequencies (kMaxVec vectors, and spectra workspace of at most 8 GiB unless
// one chunk alone needs more).
template <typename VT>
static int apply_sys(giem_handle *t, const std::vector<int> &fq, const std::vector<int> &sys,
                     const std::vector<const VT *> &in, const std::vector<VT *> &out,
                     unsigned mode, unsigned prec, hipStream_t s) {
  struct Chunk {
    int f;
    std::vector<size_t> idx;
  };
  std::vector<Chunk> chunks;
  std::vector<char> used(in.size(), 0);
  for (size_t i = 0; i < in.size(); ++i) {
    if (used[i]) continue;
    const int f = fq[sys[i]];
    std::vector<size_t> all;
    for (size_t k = i; k < in.size(); ++k)
      if (!used[k] && fq[sys[k]] == f) {
        all.push_back(k);
        used[k] = 1;
      }
    for (size_t c0 = 0; c0 < all.size(); c0 += kMaxRhs) {
      const size_t c1 = std::min(all.size(), c0 + (size_t)kMaxRhs);
      chunks.push_back(Chunk{f, std::vector<size_t>(all.begin() + c0, all.begin() + c1)});
    }
  }
  const size_t per_vec = (size_t)2 * 4 * t->nx * t->ny * 3 * t->nz * sizeof(c128);
  const size_t budget = (size_t)8 << 30;
  std::vector<char> done(chunks.size(), 0);
  for (size_t i = 0; i < chunks.size(); ++i) {
    if (done[i]) continue;
    const int R = (int)chunks[i].idx.size();
    const int cap_vec = std::max(R, (int)std::min<size_t>(kMaxVec, budget / per_vec));
    const int cap_f = std::max(1, std::min(kMaxFreqBatch, cap_vec / R));
    std::vector<size_t> group;
    for (size_t k = i; k < chunks.size() && (int)group.size() < cap_f; ++k)
      if (!done[k] && (int)chunks[k].idx.size() == R) {
        group.push_back(k);
        done[k] = 1;
      }
    VecPtrsT<VT> p{};
    int ifr[kMaxFreqBatch];
    for (size_t g = 0; g < group.size(); ++g) {
      const Chunk &c = chunks[group[g]];
      ifr[g] = c.f;
      for (int r = 0; r < R; ++r) {
        p.in[g * R + r] = in[c.idx[r]];
        p.out[g * R + r] = out[c.idx[r]];
      }
    }
    GIEM_TRY(apply_multi(t, (int)group.size(), ifr, R, p, mode, prec, s));
  }
  return GIEM_OK;
}

// Squared norm ratio below which a Gram-Schmidt pass is repeated: a second
// pass only when the projection removed more than 90% of the norm (severe
// cancellation).  On the layered-earth workloads this never changes the
// iteration count or the solution against the 0.7 criterion, and saves most
// second passes over the basis.
constexpr double kReorthDrop = 0.01;

// VT: storage of the Krylov vectors, x and b (complex128; complex64 for the
// inner solve of the precision form, which runs the FP32 operator).
// System r has right-hand side b[r], solution x[r] and operator fq[r] (the
// frequency index); systems of different frequencies advance in lockstep,
// with one host synchronisation per Arnoldi step for all of them.
template <typename VT>
static int gmres(giem_handle *t, const std::vector<int> &fq, int nrhs, const VT *const *b,
                 VT *const *x, const GmresParams &gp, hipStream_t s, GmresResult &res) {
  if (nrhs > kMaxSys || (int)fq.size() < nrhs) {
    set_error("too many linear systems in one solve");
    return GIEM_EINVAL;
  }
  const int m = gp.m;
  const size_t n = t->nvec();
  const int plane = t->nx * t->ny;
  const double *wlev = gp.weighted ? static_cast<const double *>(t->vol_lev) : nullptr;
  GIEM_TRY(ensure_basis(t, nrhs, m));
  VT *basis = static_cast<VT *>(t->basis);
  auto V = [&](int r, int i) { return basis + ((size_t)r * (m + 1) + i) * n; };
  std::vector<double> normb;
  GIEM_TRY(norms_of(t, b, nrhs, wlev, s, normb));
  res.relres.assign(nrhs, 0.0);
  res.hist.assign(nrhs, {});
  res.iters = 0;
  res.restarts = 0;
  std::vector<int> done(nrhs, 0);
  for (int r = 0; r < nrhs; ++r) {
    if (normb[r] == 0.0) {
      GIEM_HIP(hipMemsetAsync(x[r], 0, n * sizeof(VT), s), "zero x");
      done[r] = 1;
    }
  }
  bool x_zero = gp.x_zero;
  int iters = 0;
  std::vector<std::vector<cd>> H(nrhs), cs(nrhs), sn(nrhs), g(nrhs);
  // The basis vectors are stored unnormalised, V_i = |V_i| v_i, with the
  // norms kept here: h_ij = <V_i, A V_j> / (|V_i| |V_j|), the update
  // subtracts (<V_i, w> / |V_i|^2) V_i, and x += sum (y_i / |V_i|) V_i.  This
  // saves a scaling pass over every new basis vector.
  std::vector<std::vector<double>> vn(nrhs);
  double *sdev = static_cast<double *>(t->gs_scale_dev);
  double *shost = static_cast<double *>(t->gs_scale_host);
  constexpr int kSStride = 65;
  c128 *hdev = static_cast<c128 *>(t->red_out);
  c128 *ndev = static_cast<c128 *>(t->coef_dev);
  c128 *part = static_cast<c128 *>(t->red_part);
  c128 *hhost = static_cast<c128 *>(t->red_host);
  c128 *chost = static_cast<c128 *>(t->coef_host);
  hipEvent_t step_ev = nullptr;
  GIEM_HIP(hipEventCreateWithFlags(&step_ev, hipEventDisableTiming), "hipEventCreate");
  struct EvFree {
    hipEvent_t e;
    ~EvFree() { hipEventDestroy(e); }
  } ev_free{step_ev};
  while (true) {
    // residual r0 = b - A x into V(r, 0)
    std::vector<int> act;
    for (int r = 0; r < nrhs; ++r)
      if (!done[r]) act.push_back(r);
    if (act.empty()) break;
    if (x_zero) {
      for (int r : act) {
        GIEM_HIP(hipMemcpyAsync(V(r, 0), b[r], n * sizeof(VT), hipMemcpyDeviceToDevice, s), "copy b");
        GIEM_HIP(hipMemsetAsync(x[r], 0, n * sizeof(VT), s), "zero x");
      }
    } else {
      std::vector<const VT *> in;
      std::vector<VT *> out;
      for (int r : act) {
        in.push_back(x[r]);
        out.push_back(V(r, 0));
      }
      GIEM_TRY(apply_sys(t, fq, act, in, out, gp.mode, gp.prec, s));
      for (int r : act)
        GIEM_HIP(launch_axpby(V(r, 0), b[r], V(r, 0), mk<double>(1, 0), mk<double>(-1, 0), n, s), "axpby");
    }
    x_zero = false;
    std::vector<const VT *> r0p;
    for (int r : act) r0p.push_back(V(r, 0));
    std::vector<double> beta;
    GIEM_TRY(norms_of(t, r0p.data(), (int)act.size(), wlev, s, beta));
    std::vector<int> cyc;  // RHS iterating in this cycle
    for (size_t q = 0; q < act.size(); ++q) {
      const int r = act[q];
      res.relres[r] = beta[q] / normb[r];
      res.hist[r].push_back(res.relres[r]);
      if (beta[q] <= gp.tol * normb[r]) {
        done[r] = 1;
        continue;
      }
      if (iters >= gp.max_iter) continue;
      cyc.push_back(r);
      H[r].assign((size_t)(m + 1) * m, 0.0);
      cs[r].assign(m, 0.0);
      sn[r].assign(m, 0.0);
      g[r].assign(m + 1, 0.0);
      g[r][0] = beta[q];
      vn[r].assign(m + 1, 0.0);
      vn[r][0] = beta[q];
    }
    if (cyc.empty()) break;
    ++res.restarts;
    std::vector<int> jlen(nrhs, 0);
    std::vector<int> running = cyc;
    // w = A v_j into V(r, j+1) for the systems in `running`
    auto apply_step = [&](int j) -> int {
      std::vector<const VT *> in;
      std::vector<VT *> out;
      for (int r : running) {
        in.push_back(V(r, j));
        out.push_back(V(r, j + 1));
      }
      return apply_sys(t, fq, running, in, out, gp.mode, gp.prec, s);
    };
    bool ahead = false;  // the apply of step j is already on the stream
    for (int j = 0; j < m && !running.empty(); ++j) {
      if (iters >= gp.max_iter) break;
      const int na = (int)running.size();
      if (!ahead) GIEM_TRY(apply_step(j));
      ahead = false;
      ++iters;
      // classical Gram-Schmidt, repeated once when the norm drops sharply
      // (cancellation of more than a factor 10)
      std::vector<std::vector<cd>> hcol(na, std::vector<cd>(j + 1, 0.0));
      std::vector<double> nw0(na, 0.0), nw1(na, 0.0);
      for (int q = 0; q < na; ++q)
        for (int i = 0; i <= j; ++i)
          shost[(size_t)q * kSStride + i] = 1.0 / (vn[running[q]][i] * vn[running[q]][i]);
      GIEM_HIP(hipMemcpyAsync(sdev, shost, (size_t)na * kSStride * sizeof(double),
                              hipMemcpyHostToDevice, s),
               "copy basis scales");
      for (int pass = 0; pass < 2; ++pass) {
        const int nb = j + 1;
        for (int q0 = 0; q0 < na; q0 += kMaxRhs) {
          const int nq = std::min(kMaxRhs, na - q0);
          DotArgsT<VT> da{};
          for (int q = 0; q < nq; ++q) {
            da.w[q] = V(running[q0 + q], j + 1);
            da.basis[q] = V(running[q0 + q], 0);
          }
          c128 *hq = hdev + (size_t)q0 * (nb + 1);
          GIEM_HIP(launch_dots(da, nq, nb, n, t->nz, plane, wlev, part, hq, s), "dots");
          GIEM_HIP(launch_update(da, nq, nb, n, t->nz, plane, wlev, hq, nb + 1,
                                 sdev + (size_t)q0 * kSStride, kSStride, part, ndev + q0, s),
                   "update");
        }
        GIEM_HIP(hipMemcpyAsync(hhost, hdev, (size_t)na * (nb + 1) * sizeof(c128), hipMemcpyDeviceToHost, s), "copy h");
        GIEM_HIP(hipMemcpyAsync(chost, ndev, (size_t)na * sizeof(c128), hipMemcpyDeviceToHost, s), "copy norm");
        if (pass == 0 && j + 1 < m && iters < gp.max_iter) {
          // The next step's apply needs only the new (unnormalised) basis
          // vector, which is final unless a second pass follows: queue it
          // behind the copies and wait for the copies alone, so the GPU
          // works while the host updates the Hessenberg column.  It is
          // wasted for a system that stops here, and redone after a second
          // pass.
          GIEM_HIP(hipEventRecord(step_ev, s), "hipEventRecord");
          GIEM_TRY(apply_step(j + 1));
          ahead = true;
          GIEM_HIP(hipEventSynchronize(step_ev), "sync");
        } else {
          GIEM_HIP(hipStreamSynchronize(s), "sync");
        }
        bool again = false;
        for (int q = 0; q < na; ++q) {
          const std::vector<double> &nq_ = vn[running[q]];
          for (int i = 0; i < nb; ++i)
            hcol[q][i] += cd(hhost[(size_t)q * (nb + 1) + i].x, hhost[(size_t)q * (nb + 1) + i].y) /
                          (nq_[i] * nq_[j]);
          if (pass == 0) nw0[q] = hhost[(size_t)q * (nb + 1) + nb].x;
          nw1[q] = std::max(chost[q].x, 0.0);
          if (nw1[q] < kReorthDrop * nw0[q]) again = true;
        }
        if (!again) break;
        if (ahead && t->prof) t->prof_discarded[gp.prec == PREC_FP32 ? 1 : 0] += na;
        ahead = false;  // the second pass changes the vector the apply read
        for (int q = 0; q < na; ++q) nw0[q] = nw1[q];
      }
      std::vector<int> still;
      for (int q = 0; q < na; ++q) {
        const int r = running[q];
        const double wn = std::sqrt(nw1[q]);  // |V_{j+1}|
        const double hn = wn / vn[r][j];
        vn[r][j + 1] = wn;
        std::vector<cd> &Hr = H[r];
        auto Hc = [&](int i) -> cd & { return Hr[(size_t)i * m + j]; };
        for (int i = 0; i <= j; ++i) Hc(i) = hcol[q][i];
        Hc(j + 1) = hn;
        for (int i = 0; i < j; ++i) {  // earlier rotations
          const cd a = Hc(i), bb = Hc(i + 1);
          Hc(i) = cs[r][i] * a + sn[r][i] * bb;
          Hc(i + 1) = -std::conj(sn[r][i]) * a + cs[r][i] * bb;
        }
        const cd a = Hc(j);
        const double bn = std::abs(Hc(j + 1));
        const double rr = std::hypot(std::abs(a), bn);
        cd c, sv;
        if (std::abs(a) == 0.0) {
          c = 0.0;
          sv = 1.0;
        } else {
          c = std::abs(a) / rr;
          sv = (a / std::abs(a)) * std::conj(Hc(j + 1)) / rr;
        }
        cs[r][j] = c;
        sn[r][j] = sv;
        Hc(j) = c * a + sv * Hc(j + 1);
        Hc(j + 1) = 0.0;
        g[r][j + 1] = -std::conj(sv) * g[r][j];
        g[r][j] = c * g[r][j];
        jlen[r] = j + 1;
        const double est = std::abs(g[r][j + 1]);
        if (est > gp.tol * normb[r] && hn > 0.0) still.push_back(r);
      }
      // the applies queued ahead for the systems that stop here are wasted
      if (ahead && t->prof) t->prof_discarded[gp.prec == PREC_FP32 ? 1 : 0] += na - (int)still.size();
      running = still;
    }
    // x += V y, y = R^{-1} g (back substitution on the rotated Hessenberg)
    for (int r : cyc) {
      const int k = jlen[r];
      if (k == 0) continue;
      std::vector<cd> y(k);
      for (int i = k - 1; i >= 0; --i) {
        cd acc = g[r][i];
        for (int l = i + 1; l < k; ++l) acc -= H[r][(size_t)i * m + l] * y[l];
        y[i] = acc / H[r][(size_t)i * m + i];
      }
      c128 *yh = static_cast<c128 *>(t->coef_host);
      for (int i = 0; i < k; ++i) {
        const cd yi = y[i] / vn[r][i];
        yh[i] = mk<double>(yi.real(), yi.imag());
      }
      GIEM_HIP(hipMemcpyAsync(t->coef_dev, yh, k * sizeof(c128), hipMemcpyHostToDevice, s), "copy y");
      LinArgsT<VT> la{};
      la.x[0] = x[r];
      la.basis[0] = V(r, 0);
      GIEM_HIP(launch_lincomb(la, 1, k, n, static_cast<c128 *>(t->coef_dev), k, s), "lincomb");
      GIEM_HIP(hipStreamSynchronize(s), "sync");
    }
    if (iters >= gp.max_iter) {
      // final true residual for the report
      std::vector<int> left;
      for (int r = 0; r < nrhs; ++r)
        if (!done[r]) left.push_back(r);
      if (!left.empty()) {
        std::vector<const VT *> in;
        std::vector<VT *> out;
        for (int r : left) {
          in.push_back(x[r]);
          out.push_back(V(r, 0));
        }
        GIEM_TRY(apply_sys(t, fq, left, in, out, gp.mode, gp.prec, s));
        std::vector<const VT *> rp;
        for (int r : left) {
          GIEM_HIP(launch_axpby(V(r, 0), b[r], V(r, 0), mk<double>(1, 0), mk<double>(-1, 0), n, s), "axpby");
          rp.push_back(V(r, 0));
        }
        std::vector<double> rn;
        GIEM_TRY(norms_of(t, rp.data(), (int)left.size(), wlev, s, rn));
        for (size_t q = 0; q < left.size(); ++q) {
          res.relres[left[q]] = rn[q] / normb[left[q]];
          res.hist[left[q]].push_back(res.relres[left[q]]);
          if (rn[q] <= gp.tol * normb[left[q]]) done[left[q]] = 1;
        }
      }
      break;
    }
  }
  res.iters = iters;
  res.converged = true;
  for (int r = 0; r < nrhs; ++r)
    if (!done[r]) res.converged = false;
  return GIEM_OK;
}

// ------------------------------------------------------------ graph-captured GMRES
// The same GMRES(m) for systems of several handles (models of different grid
// size) and frequencies, with each restart cycle of L <= m Arnoldi steps
// recorded once as a HIP graph and replayed: the applies, both Gram-Schmidt
// passes (the second gated on the device), the Hessenberg column, the Givens
// rotation and the residual estimate all run on the device, so the host waits
// once per cycle instead of once per step.  Every system runs the whole
// cycle; one that converges (or breaks down) inside it records its Krylov
// length and its later steps are not used.  The systems of one handle form a
// contiguous range and get a branch (stream) of their own inside the graph,
// so the kernels of different models overlap.

template <typename VT>
struct GSys {
  giem_handle *t;
  int fq;        // frequency index of the handle
  const VT *b;
  VT *x;
};

struct GraphExecs {
  std::map<std::vector<int>, hipGraphExec_t> exec;
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> events;
  ~GraphExecs() {
    for (auto &e : exec) hipGraphExecDestroy(e.second);
    for (hipStream_t b : streams) hipStreamDestroy(b);
    for (hipEvent_t e : events) hipEventDestroy(e);
  }
};

// largest number of vectors apply_sys puts into one launch for these systems
static int apply_sys_max_vectors(const giem_handle *t, const std::vector<int> &fq,
                                 const std::vector<int> &sys) {
  std::map<int, int> per_f;
  for (int q : sys) per_f[fq[q]]++;
  const size_t per_vec = (size_t)2 * 4 * t->nx * t->ny * 3 * t->nz * sizeof(c128);
  const size_t budget = (size_t)8 << 30;
  int best = 0;
  std::map<int, int> chunks;  // chunk size -> count
  for (auto &kv : per_f)
    for (int left = kv.second; left > 0; left -= kMaxRhs) chunks[std::min(left, kMaxRhs)]++;
  for (auto &kv : chunks) {
    const int R = kv.first;
    const int cap_vec = std::max(R, (int)std::min<size_t>(kMaxVec, budget / per_vec));
    const int cap_f = std::max(1, std::min(kMaxFreqBatch, cap_vec / R));
    best = std::max(best, R * std::min(cap_f, kv.second));
  }
  return best;
}

template <typename VT>
static int gmres_graph(std::vector<GSys<VT>> &sys, const GmresParams &gp, hipStream_t s,
                       GmresResult &res) {
  const int ns = (int)sys.size();
  const int m = gp.m;
  if (ns < 1 || ns > kMaxSys || m < 1 || m > 64) {
    set_error("graph GMRES: 1 to 96 systems and 1 <= restart <= 64");
    return GIEM_EINVAL;
  }
  // handle blocks [hb[k], hb[k + 1])
  std::vector<int> hb{0};
  for (int q = 1; q < ns; ++q)
    if (sys[q].t != sys[q - 1].t) hb.push_back(q);
  hb.push_back(ns);
  const int nblk = (int)hb.size() - 1;
  std::vector<int> blk_of(ns);
  for (int k = 0; k < nblk; ++k)
    for (int q = hb[k]; q < hb[k + 1]; ++q) blk_of[q] = k;
  for (int k = 0; k < nblk; ++k) {
    giem_handle *t = sys[hb[k]].t;
    for (int q = hb[k + 1]; q < ns; ++q)
      if (sys[q].t == t) {
        set_error("graph GMRES: the systems of one handle must be contiguous");
        return GIEM_EINVAL;
      }
    GIEM_TRY(ensure_basis(t, hb[k + 1] - hb[k], m));
  }
  auto V = [&](int q, int i) -> VT * {
    const giem_handle *t = sys[q].t;
    return static_cast<VT *>(t->basis) + ((size_t)(q - hb[blk_of[q]]) * (m + 1) + i) * t->nvec();
  };
  auto wlev_of = [&](const giem_handle *t) {
    return gp.weighted ? static_cast<const double *>(t->vol_lev) : nullptr;
  };
  // per-system frequency list and per-block local views for apply_sys
  std::vector<std::vector<int>> bfq(nblk);
  for (int k = 0; k < nblk; ++k)
    for (int q = hb[k]; q < hb[k + 1]; ++q) bfq[k].push_back(sys[q].fq);
  // apply y_q = A x_q for the systems qs of block k (local indices q - hb[k])
  auto apply_block = [&](int k, const std::vector<int> &qs, const std::vector<const VT *> &in,
                         const std::vector<VT *> &out, hipStream_t st) -> int {
    std::vector<int> loc;
    for (int q : qs) loc.push_back(q - hb[k]);
    return apply_sys(sys[hb[k]].t, bfq[k], loc, in, out, gp.mode, gp.prec, st);
  };
  // spectra workspace sized before any capture (no allocation inside a graph)
  for (int k = 0; k < nblk; ++k) {
    std::vector<int> loc;
    for (int q = hb[k]; q < hb[k + 1]; ++q) loc.push_back(q - hb[k]);
    GIEM_TRY(ensure_spec_ws(sys[hb[k]].t, apply_sys_max_vectors(sys[hb[k]].t, bfq[k], loc),
                            (int)gp.prec));
  }
  // device Arnoldi state, indexed by the position c in the cycle's list
  const size_t nH = (size_t)(m + 1) * m;
  const size_t b_h = (size_t)ns * (m + 2) * sizeof(c128), b_n = (size_t)ns * sizeof(c128);
  const size_t b_v = (size_t)ns * kArnStride * sizeof(double);
  const size_t b_H = (size_t)ns * nH * sizeof(c128), b_r = (size_t)ns * m * sizeof(c128);
  const size_t b_g = (size_t)ns * (m + 1) * sizeof(c128), b_i = (size_t)ns * sizeof(int);
  const size_t b_d = (size_t)ns * sizeof(double);
  const size_t total = 2 * b_h + 2 * b_n + 2 * b_v + b_H + 2 * b_r + b_g + b_d + 3 * b_i + 256 * 16;
  struct Dev {
    void *p = nullptr;
    ~Dev() {
      if (p) hipFree(p);
    }
  } dev;
  GIEM_HIP(hipMalloc(&dev.p, total), "hipMalloc Arnoldi state");
  char *cur = static_cast<char *>(dev.p);
  auto take = [&](size_t bytes) {
    char *r = cur;
    cur += (bytes + 255) & ~(size_t)255;
    return r;
  };
  ArnoldiState st;
  st.h1 = reinterpret_cast<c128 *>(take(b_h));
  st.h2 = reinterpret_cast<c128 *>(take(b_h));
  st.nrm1 = reinterpret_cast<c128 *>(take(b_n));
  st.nrm2 = reinterpret_cast<c128 *>(take(b_n));
  st.vn2 = reinterpret_cast<double *>(take(b_v));
  st.scale = reinterpret_cast<double *>(take(b_v));
  st.H = reinterpret_cast<c128 *>(take(b_H));
  st.cs = reinterpret_cast<c128 *>(take(b_r));
  st.sn = reinterpret_cast<c128 *>(take(b_r));
  st.g = reinterpret_cast<c128 *>(take(b_g));
  st.tolb = reinterpret_cast<double *>(take(b_d));
  st.gate = reinterpret_cast<int *>(take(b_i));
  st.conv = reinterpret_cast<int *>(take(b_i));
  st.jlen = reinterpret_cast<int *>(take(b_i));
  // norms of b
  std::vector<double> normb(ns), beta(ns);
  for (int k = 0; k < nblk; ++k) {
    std::vector<const VT *> bp;
    for (int q = hb[k]; q < hb[k + 1]; ++q) bp.push_back(sys[q].b);
    std::vector<double> nb_;
    GIEM_TRY(norms_of(sys[hb[k]].t, bp.data(), (int)bp.size(), wlev_of(sys[hb[k]].t), s, nb_));
    for (int q = hb[k]; q < hb[k + 1]; ++q) normb[q] = nb_[q - hb[k]];
  }
  res.relres.assign(ns, 0.0);
  res.hist.assign(ns, {});
  res.iters = 0;
  res.restarts = 0;
  std::vector<int> done(ns, 0);
  for (int q = 0; q < ns; ++q)
    if (normb[q] == 0.0) {
      GIEM_HIP(hipMemsetAsync(sys[q].x, 0, sys[q].t->nvec() * sizeof(VT), s), "zero x");
      done[q] = 1;
    }
  GraphExecs gx;
  for (int k = 0; k < nblk; ++k) {
    hipStream_t b;
    GIEM_HIP(hipStreamCreateWithFlags(&b, hipStreamNonBlocking), "hipStreamCreate");
    gx.streams.push_back(b);
    hipEvent_t e;
    GIEM_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreate");
    gx.events.push_back(e);
  }
  hipEvent_t fork_ev;
  GIEM_HIP(hipEventCreateWithFlags(&fork_ev, hipEventDisableTiming), "hipEventCreate");
  gx.events.push_back(fork_ev);
  // graphs are recorded on a stream of their own (the caller's stream may be
  // the legacy default stream, which cannot be captured) and launched on s
  hipStream_t cap;
  GIEM_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking), "hipStreamCreate");
  gx.streams.push_back(cap);
  bool x_zero = gp.x_zero;
  int iters = 0;
  std::vector<c128> hostbuf;
  while (true) {
    std::vector<int> act;
    for (int q = 0; q < ns; ++q)
      if (!done[q]) act.push_back(q);
    if (act.empty()) break;
    // r0 = b - A x into V(q, 0) (eager)
    for (int k = 0; k < nblk; ++k) {
      std::vector<int> qs;
      for (int q : act)
        if (blk_of[q] == k) qs.push_back(q);
      if (qs.empty()) continue;
      if (x_zero) {
        for (int q : qs) {
          const size_t n = sys[q].t->nvec();
          GIEM_HIP(hipMemcpyAsync(V(q, 0), sys[q].b, n * sizeof(VT), hipMemcpyDeviceToDevice, s), "copy b");
          GIEM_HIP(hipMemsetAsync(sys[q].x, 0, n * sizeof(VT), s), "zero x");
        }
      } else {
        std::vector<const VT *> in;
        std::vector<VT *> out;
        for (int q : qs) {
          in.push_back(sys[q].x);
          out.push_back(V(q, 0));
        }
        GIEM_TRY(apply_block(k, qs, in, out, s));
        for (int q : qs)
          GIEM_HIP(launch_axpby(V(q, 0), sys[q].b, V(q, 0), mk<double>(1, 0), mk<double>(-1, 0),
                                sys[q].t->nvec(), s),
                   "axpby");
      }
      std::vector<const VT *> rp;
      for (int q : qs) rp.push_back(V(q, 0));
      std::vector<double> bt;
      GIEM_TRY(norms_of(sys[qs[0]].t, rp.data(), (int)qs.size(), wlev_of(sys[qs[0]].t), s, bt));
      for (size_t i = 0; i < qs.size(); ++i) beta[qs[i]] = bt[i];
    }
    x_zero = false;
    std::vector<int> cyc;
    for (int q : act) {
      res.relres[q] = beta[q] / normb[q];
      res.hist[q].push_back(res.relres[q]);
      if (beta[q] <= gp.tol * normb[q]) {
        done[q] = 1;
        continue;
      }
      if (iters < gp.max_iter) cyc.push_back(q);
    }
    if (cyc.empty()) break;
    const int L = std::min(m, gp.max_iter - iters);
    const int nc = (int)cyc.size();
    // per-cycle initial state (host image, one upload per array)
    {
      std::vector<double> vn2((size_t)ns * kArnStride, 0.0), scl((size_t)ns * kArnStride, 0.0);
      std::vector<c128> g((size_t)ns * (m + 1), mk<double>(0, 0));
      std::vector<double> tolb(ns, 0.0);
      std::vector<int> zi(ns, 0);
      for (int c = 0; c < nc; ++c) {
        const int q = cyc[c];
        vn2[(size_t)c * kArnStride] = beta[q] * beta[q];
        scl[(size_t)c * kArnStride] = 1.0 / (beta[q] * beta[q]);
        g[(size_t)c * (m + 1)] = mk<double>(beta[q], 0.0);
        tolb[c] = gp.tol * normb[q];
      }
      GIEM_HIP(hipMemcpyAsync(st.vn2, vn2.data(), vn2.size() * sizeof(double), hipMemcpyHostToDevice, s), "state");
      GIEM_HIP(hipMemcpyAsync(st.scale, scl.data(), scl.size() * sizeof(double), hipMemcpyHostToDevice, s), "state");
      GIEM_HIP(hipMemcpyAsync(st.g, g.data(), g.size() * sizeof(c128), hipMemcpyHostToDevice, s), "state");
      GIEM_HIP(hipMemcpyAsync(st.tolb, tolb.data(), tolb.size() * sizeof(double), hipMemcpyHostToDevice, s), "state");
      GIEM_HIP(hipMemcpyAsync(st.conv, zi.data(), zi.size() * sizeof(int), hipMemcpyHostToDevice, s), "state");
      GIEM_HIP(hipMemcpyAsync(st.jlen, zi.data(), zi.size() * sizeof(int), hipMemcpyHostToDevice, s), "state");
      // the host images must outlive the copies
      GIEM_HIP(hipStreamSynchronize(s), "sync");
    }
    std::vector<int> key = cyc;
    key.push_back(-L);
    auto it = gx.exec.find(key);
    if (it == gx.exec.end()) {
      // record one cycle: a branch per handle block, forked from s
      std::vector<bool> prof_was(nblk);
      for (int k = 0; k < nblk; ++k) {
        prof_was[k] = sys[hb[k]].t->prof;
        sys[hb[k]].t->prof = false;
      }
      int rc = check_hip(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal), "begin capture");
      if (rc == GIEM_OK) rc = check_hip(hipEventRecord(fork_ev, cap), "fork");
      for (int k = 0; k < nblk && rc == GIEM_OK; ++k) {
        std::vector<int> cs_;  // cycle positions of this block's systems
        for (int c = 0; c < nc; ++c)
          if (blk_of[cyc[c]] == k) cs_.push_back(c);
        if (cs_.empty()) continue;
        hipStream_t bs = gx.streams[k];
        giem_handle *t = sys[hb[k]].t;
        const size_t n = t->nvec();
        const int plane = t->nx * t->ny;
        c128 *part = static_cast<c128 *>(t->red_part);
        rc = check_hip(hipStreamWaitEvent(bs, fork_ev, 0), "fork wait");
        for (int j = 0; j < L && rc == GIEM_OK; ++j) {
          std::vector<int> qs;
          std::vector<const VT *> in;
          std::vector<VT *> out;
          for (int c : cs_) {
            qs.push_back(cyc[c]);
            in.push_back(V(cyc[c], j));
            out.push_back(V(cyc[c], j + 1));
          }
          rc = apply_block(k, qs, in, out, bs);
          const int nb = j + 1;
          for (size_t i0 = 0; i0 < cs_.size() && rc == GIEM_OK; i0 += kMaxRhs) {
            const int nq = (int)std::min<size_t>(kMaxRhs, cs_.size() - i0);
            const int c0 = cs_[i0];  // positions of one block are consecutive
            DotArgsT<VT> da{};
            for (int i = 0; i < nq; ++i) {
              da.w[i] = V(cyc[c0 + i], j + 1);
              da.basis[i] = V(cyc[c0 + i], 0);
            }
            // the projections of a block live in its own region (the
            // branches of different blocks run at different steps j)
            const size_t hoff = (size_t)cs_[0] * (m + 2) + i0 * (size_t)(nb + 1);
            c128 *h1 = st.h1 + hoff, *h2 = st.h2 + hoff;
            double *sc = st.scale + (size_t)c0 * kArnStride;
            const double *wl = wlev_of(t);
            rc = check_hip(launch_dots(da, nq, nb, n, t->nz, plane, wl, part, h1, bs), "dots");
            if (rc == GIEM_OK)
              rc = check_hip(launch_update(da, nq, nb, n, t->nz, plane, wl, h1, nb + 1, sc,
                                           kArnStride, part, st.nrm1 + c0, bs),
                             "update");
            if (rc == GIEM_OK)
              rc = check_hip(launch_gs_gate(nq, h1, nb + 1, st.nrm1 + c0, st.gate + c0,
                                            kReorthDrop, bs),
                             "gate");
            if (rc == GIEM_OK)
              rc = check_hip(launch_dots(da, nq, nb, n, t->nz, plane, wl, part, h2, bs, st.gate, c0),
                             "dots (second pass)");
            if (rc == GIEM_OK)
              rc = check_hip(launch_update(da, nq, nb, n, t->nz, plane, wl, h2, nb + 1, sc,
                                           kArnStride, part, st.nrm2 + c0, bs, st.gate, c0),
                             "update (second pass)");
            if (rc == GIEM_OK)
              rc = check_hip(launch_arnoldi_tail(st, h1, h2, c0, nq, j, m, bs), "Arnoldi tail");
          }
        }
        if (rc == GIEM_OK) rc = check_hip(hipEventRecord(gx.events[k], bs), "join");
        if (rc == GIEM_OK) rc = check_hip(hipStreamWaitEvent(cap, gx.events[k], 0), "join wait");
      }
      hipGraph_t graph = nullptr;
      const int rc_end = check_hip(hipStreamEndCapture(cap, &graph), "end capture");
      for (int k = 0; k < nblk; ++k) sys[hb[k]].t->prof = prof_was[k];
      if (rc == GIEM_OK) rc = rc_end;
      hipGraphExec_t exec = nullptr;
      if (rc == GIEM_OK)
        rc = check_hip(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0), "instantiate graph");
      if (graph) hipGraphDestroy(graph);
      if (rc != GIEM_OK) return rc;
      it = gx.exec.emplace(key, exec).first;
    }
    GIEM_HIP(hipGraphLaunch(it->second, s), "launch graph");
    iters += L;
    ++res.restarts;
    // read back the cycle's small state, solve R y = g on the host
    std::vector<c128> H((size_t)nc * nH), g((size_t)nc * (m + 1));
    std::vector<double> vn2((size_t)nc * kArnStride);
    std::vector<int> conv(nc), jlen(nc);
    GIEM_HIP(hipMemcpyAsync(H.data(), st.H, H.size() * sizeof(c128), hipMemcpyDeviceToHost, s), "read H");
    GIEM_HIP(hipMemcpyAsync(g.data(), st.g, g.size() * sizeof(c128), hipMemcpyDeviceToHost, s), "read g");
    GIEM_HIP(hipMemcpyAsync(vn2.data(), st.vn2, vn2.size() * sizeof(double), hipMemcpyDeviceToHost, s), "read norms");
    GIEM_HIP(hipMemcpyAsync(conv.data(), st.conv, nc * sizeof(int), hipMemcpyDeviceToHost, s), "read flags");
    GIEM_HIP(hipMemcpyAsync(jlen.data(), st.jlen, nc * sizeof(int), hipMemcpyDeviceToHost, s), "read lengths");
    GIEM_HIP(hipStreamSynchronize(s), "sync");
    std::vector<c128> yall((size_t)nc * 64, mk<double>(0, 0));
    std::vector<int> klen(nc, 0);
    for (int c = 0; c < nc; ++c) {
      int k = conv[c] ? jlen[c] : L;
      const c128 *Hc = H.data() + (size_t)c * nH;
      const c128 *gc = g.data() + (size_t)c * (m + 1);
      for (int i = 0; i < k; ++i)
        if (Hc[(size_t)i * m + i].x == 0.0 && Hc[(size_t)i * m + i].y == 0.0) {
          k = i;
          break;
        }
      std::vector<cd> y(k);
      for (int i = k - 1; i >= 0; --i) {
        cd acc(gc[i].x, gc[i].y);
        for (int l = i + 1; l < k; ++l)
          acc -= cd(Hc[(size_t)i * m + l].x, Hc[(size_t)i * m + l].y) * y[l];
        y[i] = acc / cd(Hc[(size_t)i * m + i].x, Hc[(size_t)i * m + i].y);
      }
      for (int i = 0; i < k; ++i) {
        const cd yi = y[i] / std::sqrt(vn2[(size_t)c * kArnStride + i]);
        yall[(size_t)c * 64 + i] = mk<double>(yi.real(), yi.imag());
      }
      klen[c] = k;
    }
    c128 *ydev = static_cast<c128 *>(sys[0].t->coef_dev);  // [kMaxSys][65]
    GIEM_HIP(hipMemcpyAsync(ydev, yall.data(), (size_t)nc * 64 * sizeof(c128), hipMemcpyHostToDevice, s),
             "copy y");
    for (int c = 0; c < nc; ++c) {
      if (klen[c] == 0) continue;
      const int q = cyc[c];
      LinArgsT<VT> la{};
      la.x[0] = sys[q].x;
      la.basis[0] = V(q, 0);
      GIEM_HIP(launch_lincomb(la, 1, klen[c], sys[q].t->nvec(), ydev + (size_t)c * 64, 64, s), "lincomb");
    }
    GIEM_HIP(hipStreamSynchronize(s), "sync");
    if (iters >= gp.max_iter) {
      // final true residual for the report
      for (int k = 0; k < nblk; ++k) {
        std::vector<int> qs;
        for (int q = hb[k]; q < hb[k + 1]; ++q)
          if (!done[q]) qs.push_back(q);
        if (qs.empty()) continue;
        std::vector<const VT *> in;
        std::vector<VT *> out;
        for (int q : qs) {
          in.push_back(sys[q].x);
          out.push_back(V(q, 0));
        }
        GIEM_TRY(apply_block(k, qs, in, out, s));
        std::vector<const VT *> rp;
        for (int q : qs) {
          GIEM_HIP(launch_axpby(V(q, 0), sys[q].b, V(q, 0), mk<double>(1, 0), mk<double>(-1, 0),
                                sys[q].t->nvec(), s),
                   "axpby");
          rp.push_back(V(q, 0));
        }
        std::vector<double> rn;
        GIEM_TRY(norms_of(sys[qs[0]].t, rp.data(), (int)qs.size(), wlev_of(sys[qs[0]].t), s, rn));
        for (size_t i = 0; i < qs.size(); ++i) {
          res.relres[qs[i]] = rn[i] / normb[qs[i]];
          res.hist[qs[i]].push_back(res.relres[qs[i]]);
          if (rn[i] <= gp.tol * normb[qs[i]]) done[qs[i]] = 1;
        }
      }
      break;
    }
  }
  res.iters = iters;
  res.converged = true;
  for (int q = 0; q < ns; ++q)
    if (!done[q]) res.converged = false;
  return GIEM_OK;
}

// ------------------------------------------------------------ solve entry
static int check_sigma_a(giem_handle *t, const void *sigma_a, hipStream_t s) {
  std::vector<c128> h(t->ncell());
  GIEM_HIP(hipMemcpyAsync(h.data(), sigma_a, h.size() * sizeof(c128), hipMemcpyDeviceToHost, s),
           "copy sigma_a");
  GIEM_HIP(hipStreamSynchronize(s), "sync");
  for (const c128 &v : h) {
    if (!std::isfinite(v.x) || !std::isfinite(v.y)) {
      set_error("sigma_a holds NaN or Inf");
      return GIEM_EINVAL;
    }
    if (v.x < 0.0) {
      set_error("Re sigma_a must be >= 0");
      return GIEM_EDOMAIN;
    }
  }
  return GIEM_OK;
}

// b of every system (f, r) into bv [nf][nrhs][n]: the caller's rhs[f], or the
// plane-wave source U^0 = sqrt(Re sigma_b) <E^N> (x then y polarisation)
static int prepare_rhs(giem_handle *t, int nf, const int *ifreqs, int nrhs,
                       const void *const *rhs, c128 *bv, hipStream_t s) {
  const size_t n = t->nvec();
  for (int f = 0; f < nf; ++f) {
    c128 *bf = bv + (size_t)f * nrhs * n;
    if (rhs && rhs[f]) {
      GIEM_HIP(hipMemcpyAsync(bf, rhs[f], (size_t)nrhs * n * sizeof(c128), hipMemcpyDeviceToDevice, s),
               "copy rhs");
    } else {
      std::vector<cd> en, hs;
      plane_wave_levels(t, t->f[ifreqs[f]].freq, en, hs);
      std::vector<c128> enc(t->nz);
      for (int k = 0; k < t->nz; ++k) enc[k] = mk<double>(en[k].real(), en[k].imag());
      // stage per-level E^N in the small coefficient buffer
      if ((size_t)t->nz > (size_t)kMaxSys * 65) {
        set_error("Nz too large");
        return GIEM_EINVAL;
      }
      GIEM_HIP(hipMemcpyAsync(t->coef_dev, enc.data(), t->nz * sizeof(c128), hipMemcpyHostToDevice, s),
               "copy EN");
      for (int r = 0; r < nrhs; ++r)
        GIEM_HIP(launch_plane_wave_rhs(static_cast<c128 *>(t->coef_dev),
                                       static_cast<double *>(t->sroot_lev), t->nx, t->ny, t->nz, r,
                                       bf + (size_t)r * n, s),
                 "plane wave");
      GIEM_HIP(hipStreamSynchronize(s), "sync");
    }
  }
  return GIEM_OK;
}

static int solve_groups_impl(int ng, const giem_solve_group *gr, int nrhs,
                             const giem_solve_opts *o, giem_solve_stats *st, hipStream_t s);

// Solve for nf frequencies of the handle at once (nf = 1 for giem_solve).
// System (f, r) = frequency ifreqs[f], right-hand side r; all systems share
// sigma_a and therefore the diagonals S, R1, R2, a.  rhs[f] (or NULL for the
// plane-wave source) and E_cells[f] are [nrhs][3][N] device arrays; st has nf
// entries (or is NULL).
static int solve_batch_impl(giem_handle *t, int nf, const int *ifreqs, const void *sigma_a,
                            int nrhs, const void *const *rhs, void *const *E_cells,
                            const giem_solve_opts *o, giem_solve_stats *st, hipStream_t s,
                            unsigned mode) {
  auto t0 = std::chrono::steady_clock::now();
  if (!t || nf < 1 || !ifreqs || nrhs < 1 || nrhs > kMaxRhs || !sigma_a || !E_cells || !o) {
    set_error("giem_solve: bad argument");
    return GIEM_EINVAL;
  }
  if (nf * nrhs > kMaxSys) {
    set_error("giem_solve_batch: more than " + std::to_string(kMaxSys) +
              " systems (frequencies x right-hand sides)");
    return GIEM_EINVAL;
  }
  for (int f = 0; f < nf; ++f) {
    if (ifreqs[f] < 0 || ifreqs[f] >= (int)t->f.size() || !E_cells[f]) {
      set_error("giem_solve: bad frequency index or output");
      return GIEM_EINVAL;
    }
    if (!(rhs && rhs[f]) && nrhs > 2) {
      set_error("giem_solve: the plane-wave source has two polarisations (nrhs <= 2)");
      return GIEM_EINVAL;
    }
    if (o->precision == PREC_FP32 && !t->f[ifreqs[f]].spec32) {
      set_error("giem_solve: the FP32 form needs tables built with GIEM_TABLES_C64");
      return GIEM_EINVAL;
    }
  }
  if (!(o->tol > 0) || o->restart < 1 || o->restart > 64 || o->max_iter < 1 ||
      (o->precision != PREC_FP64 && o->precision != PREC_FP32)) {
    set_error("giem_solve: bad options (tol > 0, 1 <= restart <= 64, max_iter >= 1)");
    return GIEM_EINVAL;
  }
  if (o->graph && mode == MODE_A) {
    const giem_solve_group G{t, nf, ifreqs, sigma_a, rhs, E_cells};
    return solve_groups_impl(1, &G, nrhs, o, st, s);
  }
  GIEM_TRY(check_sigma_a(t, sigma_a, s));
  GIEM_TRY(compute_diagonals(t, static_cast<const c128 *>(sigma_a), s));
  const size_t n = t->nvec(), nc = t->ncell();
  const int ns = nf * nrhs;  // systems, index f * nrhs + r
  // workspace: b, u, residual, correction (ns vectors each)
  GIEM_TRY(ensure_vec_ws(t, (size_t)4 * ns));
  c128 *ws = static_cast<c128 *>(t->vec_ws);
  c128 *bv = ws, *uv = ws + (size_t)ns * n, *dv = ws + (size_t)2 * ns * n;
  c128 *cv = ws + (size_t)3 * ns * n;
  const c128 *acell = static_cast<const c128 *>(t->diag) + 3 * nc;
  GIEM_TRY(prepare_rhs(t, nf, ifreqs, nrhs, rhs, bv, s));
  const bool warm = o->warm_start != 0;
  if (warm)
    for (int f = 0; f < nf; ++f)
      GIEM_HIP(launch_mul_cells(uv + (size_t)f * nrhs * n, static_cast<const c128 *>(E_cells[f]),
                                acell, nrhs, nc, s),
               "U = a E");
  std::vector<const c128 *> bp(ns);
  std::vector<c128 *> up(ns), dp(ns);
  std::vector<int> fq(ns);
  for (int q = 0; q < ns; ++q) {
    bp[q] = bv + (size_t)q * n;
    up[q] = uv + (size_t)q * n;
    dp[q] = dv + (size_t)q * n;
    fq[q] = ifreqs[q / nrhs];
  }
  GmresParams gp;
  gp.tol = o->tol;
  gp.m = o->restart;
  gp.max_iter = o->max_iter;
  gp.weighted = o->weighted_ip;
  gp.mode = mode;
  int rc = GIEM_OK;
  int iters_total = 0, outer_total = 0;
  std::vector<double> relres(ns, 0.0);
  std::vector<std::vector<double>> hist(ns);
  std::vector<char> sys_conv(ns, 0);
  if (o->precision == PREC_FP64) {
    gp.prec = PREC_FP64;
    gp.x_zero = !warm;
    GmresResult gr;
    GIEM_TRY(gmres(t, fq, ns, bp.data(), up.data(), gp, s, gr));
    iters_total = gr.iters;
    outer_total = gr.restarts;
    for (int q = 0; q < ns; ++q) {
      relres[q] = gr.relres[q];
      hist[q] = gr.hist[q];
      sys_conv[q] = gr.relres[q] <= o->tol;
    }
  } else {
    // refinement: r = b - A64 u (FP64), inner GMRES on A32 d = r, u += d
    const double *wlev = o->weighted_ip ? static_cast<const double *>(t->vol_lev) : nullptr;
    std::vector<double> normb, rn;
    GIEM_TRY(norms_of(t, bp.data(), ns, wlev, s, normb));
    if (!warm)
      for (int q = 0; q < ns; ++q) GIEM_HIP(hipMemsetAsync(up[q], 0, n * sizeof(c128), s), "zero");
    const int max_outer = o->max_outer > 0 ? o->max_outer : 20;
    const double itol = o->inner_tol > 0 ? o->inner_tol : 1e-3;
    std::vector<int> all(ns), act;
    for (int q = 0; q < ns; ++q) all[q] = q;
    int outer = 0, inner_total = 0;
    for (outer = 0; outer <= max_outer; ++outer) {
      // true FP64 residual of every system
      std::vector<const c128 *> in(up.begin(), up.end());
      GIEM_TRY(apply_sys(t, fq, all, in, dp, mode, PREC_FP64, s));
      for (int q = 0; q < ns; ++q)
        GIEM_HIP(launch_axpby(dp[q], bp[q], dp[q], mk<double>(1, 0), mk<double>(-1, 0), n, s), "axpby");
      std::vector<const c128 *> dcp(dp.begin(), dp.end());
      GIEM_TRY(norms_of(t, dcp.data(), ns, wlev, s, rn));
      act.clear();
      for (int q = 0; q < ns; ++q) {
        relres[q] = normb[q] > 0 ? rn[q] / normb[q] : 0.0;
        hist[q].push_back(relres[q]);
        sys_conv[q] = relres[q] <= o->tol;
        if (!sys_conv[q]) act.push_back(q);
      }
      if (act.empty()) break;
      if (outer == max_outer || inner_total >= o->max_iter) break;
      // inner solve of A d = r for the systems not yet converged, entirely in
      // complex64 (vectors, basis and operator; FP64 accumulation), in the
      // space of the correction buffer: r32 and d32 per system
      std::vector<const c64 *> rb;
      std::vector<c64 *> cx;
      std::vector<int> afq;
      for (int q : act) {
        c64 *r32 = reinterpret_cast<c64 *>(cv + (size_t)q * n);
        c64 *dst[1] = {r32};
        const c128 *src[1] = {dp[q]};
        const c128 one = mk<double>(1, 0);
        GIEM_HIP(launch_scale(dst, src, &one, 1, n, s), "r -> complex64");
        rb.push_back(r32);
        cx.push_back(r32 + n);
        afq.push_back(fq[q]);
      }
      GmresParams ip = gp;
      ip.prec = PREC_FP32;
      ip.tol = inner_tolerance(itol, o->tol, act, normb, rn);
      ip.x_zero = true;
      ip.max_iter = std::max(1, o->max_iter - inner_total);
      GmresResult gr;
      GIEM_TRY(gmres(t, afq, (int)act.size(), rb.data(), cx.data(), ip, s, gr));
      inner_total += gr.iters;
      for (size_t k = 0; k < act.size(); ++k)
        GIEM_HIP(launch_axpby(up[act[k]], up[act[k]], cx[k], mk<double>(1, 0), mk<double>(1, 0), n, s),
                 "u += d");
    }
    iters_total = inner_total;
    outer_total = outer;
  }
  // E = U / a
  bool all_conv = true;
  for (int f = 0; f < nf; ++f)
    GIEM_HIP(launch_div_cells(static_cast<c128 *>(E_cells[f]), uv + (size_t)f * nrhs * n, acell,
                              nrhs, nc, s),
             "E = U / a");
  GIEM_HIP(hipStreamSynchronize(s), "sync");
  const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  for (int f = 0; f < nf; ++f) {
    giem_solve_stats lst{};
    lst.iters = iters_total;
    lst.outer_iters = outer_total;
    lst.converged = 1;
    lst.rel_residual = 0.0;
    for (int r = 0; r < nrhs; ++r) {
      const int q = f * nrhs + r;
      lst.rel_residual = std::max(lst.rel_residual, relres[q]);
      if (!sys_conv[q]) lst.converged = 0;
    }
    fill_history(lst, hist, f * nrhs, nrhs);
    if (!lst.converged) all_conv = false;
    lst.ms = ms;
    if (st) st[f] = lst;
  }
  if (!all_conv) {
    rc = GIEM_ENOCONV;
    set_error("GMRES reached the iteration limit before the tolerance");
  }
  return rc;
}

// Solve the systems of several handles (models) and frequencies together
// with graph-captured GMRES cycles (gmres_graph).  Group g is handle t_g at
// frequencies ifreqs_g with its own sigma_a; system (g, f, r).  Outputs and
// stats as solve_batch_impl, stats ordered group by group.
static int solve_groups_impl(int ng, const giem_solve_group *gr, int nrhs,
                             const giem_solve_opts *o, giem_solve_stats *st, hipStream_t s) {
  auto t0 = std::chrono::steady_clock::now();
  if (ng < 1 || !gr || nrhs < 1 || nrhs > kMaxRhs || !o) {
    set_error("giem_solve_multi: bad argument");
    return GIEM_EINVAL;
  }
  if (!(o->tol > 0) || o->restart < 1 || o->restart > 64 || o->max_iter < 1 ||
      (o->precision != PREC_FP64 && o->precision != PREC_FP32)) {
    set_error("giem_solve_multi: bad options (tol > 0, 1 <= restart <= 64, max_iter >= 1)");
    return GIEM_EINVAL;
  }
  int total = 0;
  for (int g = 0; g < ng; ++g) {
    const giem_solve_group &G = gr[g];
    if (!G.t || G.nf < 1 || !G.ifreqs || !G.sigma_a || !G.E_cells) {
      set_error("giem_solve_multi: bad group");
      return GIEM_EINVAL;
    }
    for (int h = 0; h < g; ++h)
      if (gr[h].t == G.t) {
        set_error("giem_solve_multi: a handle may appear in one group only");
        return GIEM_EINVAL;
      }
    if (G.t->device != gr[0].t->device) {
      set_error("giem_solve_multi: every handle must live on the same device");
      return GIEM_EINVAL;
    }
    for (int f = 0; f < G.nf; ++f) {
      if (G.ifreqs[f] < 0 || G.ifreqs[f] >= (int)G.t->f.size() || !G.E_cells[f]) {
        set_error("giem_solve_multi: bad frequency index or output");
        return GIEM_EINVAL;
      }
      if (!(G.rhs && G.rhs[f]) && nrhs > 2) {
        set_error("giem_solve_multi: the plane-wave source has two polarisations (nrhs <= 2)");
        return GIEM_EINVAL;
      }
      if (o->precision == PREC_FP32 && !G.t->f[G.ifreqs[f]].spec32) {
        set_error("giem_solve_multi: the FP32 form needs tables built with GIEM_TABLES_C64");
        return GIEM_EINVAL;
      }
    }
    total += G.nf * nrhs;
  }
  if (total > kMaxSys) {
    set_error("giem_solve_multi: more than " + std::to_string(kMaxSys) + " systems");
    return GIEM_EINVAL;
  }
  const bool warm = o->warm_start != 0;
  // per group: diagonals, b, u; systems in group-major order
  std::vector<GSys<c128>> sys;
  std::vector<c128 *> dres, corr;  // FP64 residual and complex64 scratch per system
  for (int g = 0; g < ng; ++g) {
    const giem_solve_group &G = gr[g];
    giem_handle *t = G.t;
    GIEM_TRY(check_sigma_a(t, G.sigma_a, s));
    GIEM_TRY(compute_diagonals(t, static_cast<const c128 *>(G.sigma_a), s));
    const size_t n = t->nvec(), nc = t->ncell();
    const int nsg = G.nf * nrhs;
    GIEM_TRY(ensure_vec_ws(t, (size_t)4 * nsg));
    c128 *ws = static_cast<c128 *>(t->vec_ws);
    c128 *bv = ws, *uv = ws + (size_t)nsg * n;
    std::vector<int> fi(G.ifreqs, G.ifreqs + G.nf);
    GIEM_TRY(prepare_rhs(t, G.nf, fi.data(), nrhs, G.rhs, bv, s));
    const c128 *acell = static_cast<const c128 *>(t->diag) + 3 * nc;
    if (warm)
      for (int f = 0; f < G.nf; ++f)
        GIEM_HIP(launch_mul_cells(uv + (size_t)f * nrhs * n, static_cast<const c128 *>(G.E_cells[f]),
                                  acell, nrhs, nc, s),
                 "U = a E");
    for (int q = 0; q < nsg; ++q) {
      sys.push_back(GSys<c128>{t, G.ifreqs[q / nrhs], bv + (size_t)q * n, uv + (size_t)q * n});
      dres.push_back(ws + (size_t)(2 * nsg + q) * n);
      corr.push_back(ws + (size_t)(3 * nsg + q) * n);
    }
  }
  const int ns = (int)sys.size();
  GmresParams gp;
  gp.tol = o->tol;
  gp.m = o->restart;
  gp.max_iter = o->max_iter;
  gp.weighted = o->weighted_ip;
  gp.mode = MODE_A;
  int iters_total = 0, outer_total = 0;
  std::vector<double> relres(ns, 0.0);
  std::vector<std::vector<double>> hist(ns);
  std::vector<char> sys_conv(ns, 0);
  if (o->precision == PREC_FP64) {
    gp.prec = PREC_FP64;
    gp.x_zero = !warm;
    GmresResult res;
    GIEM_TRY(gmres_graph(sys, gp, s, res));
    iters_total = res.iters;
    outer_total = res.restarts;
    for (int q = 0; q < ns; ++q) {
      relres[q] = res.relres[q];
      hist[q] = res.hist[q];
      sys_conv[q] = res.relres[q] <= o->tol;
    }
  } else {
    // refinement: r = b - A64 u (FP64, eager), inner graph GMRES in complex64
    std::vector<double> normb(ns), rn(ns);
    auto norms_all = [&](const std::vector<const c128 *> &v, std::vector<double> &out) -> int {
      for (int q0 = 0; q0 < ns;) {
        int q1 = q0;
        while (q1 < ns && sys[q1].t == sys[q0].t) ++q1;
        std::vector<double> part;
        const double *wl = o->weighted_ip ? static_cast<const double *>(sys[q0].t->vol_lev) : nullptr;
        GIEM_TRY(norms_of(sys[q0].t, v.data() + q0, q1 - q0, wl, s, part));
        for (int q = q0; q < q1; ++q) out[q] = part[q - q0];
        q0 = q1;
      }
      return GIEM_OK;
    };
    {
      std::vector<const c128 *> bp;
      for (auto &x : sys) bp.push_back(x.b);
      GIEM_TRY(norms_all(bp, normb));
    }
    if (!warm)
      for (auto &x : sys) GIEM_HIP(hipMemsetAsync(x.x, 0, x.t->nvec() * sizeof(c128), s), "zero");
    const int max_outer = o->max_outer > 0 ? o->max_outer : 20;
    const double itol = o->inner_tol > 0 ? o->inner_tol : 1e-3;
    int outer = 0, inner_total = 0;
    for (outer = 0; outer <= max_outer; ++outer) {
      for (int q0 = 0; q0 < ns;) {
        int q1 = q0;
        while (q1 < ns && sys[q1].t == sys[q0].t) ++q1;
        std::vector<int> fq, loc;
        std::vector<const c128 *> in;
        std::vector<c128 *> out;
        for (int q = q0; q < q1; ++q) {
          fq.push_back(sys[q].fq);
          loc.push_back(q - q0);
          in.push_back(sys[q].x);
          out.push_back(dres[q]);
        }
        GIEM_TRY(apply_sys(sys[q0].t, fq, loc, in, out, MODE_A, PREC_FP64, s));
        for (int q = q0; q < q1; ++q)
          GIEM_HIP(launch_axpby(dres[q], sys[q].b, dres[q], mk<double>(1, 0), mk<double>(-1, 0),
                                sys[q].t->nvec(), s),
                   "axpby");
        q0 = q1;
      }
      {
        std::vector<const c128 *> dp(dres.begin(), dres.end());
        GIEM_TRY(norms_all(dp, rn));
      }
      std::vector<int> act;
      for (int q = 0; q < ns; ++q) {
        relres[q] = normb[q] > 0 ? rn[q] / normb[q] : 0.0;
        hist[q].push_back(relres[q]);
        sys_conv[q] = relres[q] <= o->tol;
        if (!sys_conv[q]) act.push_back(q);
      }
      if (act.empty() || outer == max_outer || inner_total >= o->max_iter) break;
      std::vector<GSys<c64>> isys;
      for (int q : act) {
        c64 *r32 = reinterpret_cast<c64 *>(corr[q]);
        c64 *dst[1] = {r32};
        const c128 *src[1] = {dres[q]};
        const c128 one = mk<double>(1, 0);
        GIEM_HIP(launch_scale(dst, src, &one, 1, sys[q].t->nvec(), s), "r -> complex64");
        isys.push_back(GSys<c64>{sys[q].t, sys[q].fq, r32, r32 + sys[q].t->nvec()});
      }
      GmresParams ip = gp;
      ip.prec = PREC_FP32;
      ip.tol = inner_tolerance(itol, o->tol, act, normb, rn);
      ip.x_zero = true;
      ip.max_iter = std::max(1, o->max_iter - inner_total);
      GmresResult res;
      GIEM_TRY(gmres_graph(isys, ip, s, res));
      inner_total += res.iters;
      for (size_t k = 0; k < act.size(); ++k)
        GIEM_HIP(launch_axpby(sys[act[k]].x, sys[act[k]].x, isys[k].x, mk<double>(1, 0),
                              mk<double>(1, 0), sys[act[k]].t->nvec(), s),
                 "u += d");
    }
    iters_total = inner_total;
    outer_total = outer;
  }
  // E = U / a, stats per (group, frequency)
  for (int g = 0, q = 0; g < ng; ++g) {
    const giem_solve_group &G = gr[g];
    const size_t nc = G.t->ncell();
    const c128 *acell = static_cast<const c128 *>(G.t->diag) + 3 * nc;
    for (int f = 0; f < G.nf; ++f, q += nrhs)
      GIEM_HIP(launch_div_cells(static_cast<c128 *>(G.E_cells[f]), sys[q].x, acell, nrhs, nc, s),
               "E = U / a");
  }
  GIEM_HIP(hipStreamSynchronize(s), "sync");
  const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  bool all_conv = true;
  for (int g = 0, q = 0, k = 0; g < ng; ++g)
    for (int f = 0; f < gr[g].nf; ++f, ++k) {
      giem_solve_stats lst{};
      lst.iters = iters_total;
      lst.outer_iters = outer_total;
      lst.converged = 1;
      lst.rel_residual = 0.0;
      lst.ms = ms;
      fill_history(lst, hist, q, nrhs);
      for (int r = 0; r < nrhs; ++r, ++q) {
        lst.rel_residual = std::max(lst.rel_residual, relres[q]);
        if (!sys_conv[q]) lst.converged = 0;
      }
      if (!lst.converged) all_conv = false;
      if (st) st[k] = lst;
    }
  if (!all_conv) {
    set_error("GMRES reached the iteration limit before the tolerance");
    return GIEM_ENOCONV;
  }
  return GIEM_OK;
}

static int solve_impl(giem_handle *t, int ifreq, const void *sigma_a, int nrhs, const void *rhs,
                      void *E_cells, const giem_solve_opts *o, giem_solve_stats *st,
                      hipStream_t s, unsigned mode) {
  const void *rp[1] = {rhs};
  void *ep[1] = {E_cells};
  return solve_batch_impl(t, 1, &ifreq, sigma_a, nrhs, rp, ep, o, st, s, mode);
}

// Adjoint: lambda = A^{-T} (g / a), then the per-cell sensitivity kernel.
static int adjoint_impl(giem_handle *t, int ifreq, const void *sigma_a, int nrhs,
                        const void *adj_src, const void *E_fwd, void *grad,
                        const giem_solve_opts *o, giem_solve_stats *st, hipStream_t s) {
  auto t0 = std::chrono::steady_clock::now();
  if (!t || ifreq < 0 || ifreq >= (int)t->f.size() || nrhs < 1 || nrhs > kMaxRhs || !sigma_a ||
      !adj_src || !E_fwd || !grad || !o || !(o->tol > 0) || o->restart < 1 || o->restart > 64 ||
      o->max_iter < 1) {
    set_error("giem_adjoint: bad argument");
    return GIEM_EINVAL;
  }
  GIEM_TRY(check_sigma_a(t, sigma_a, s));
  GIEM_TRY(compute_diagonals(t, static_cast<const c128 *>(sigma_a), s));
  const size_t n = t->nvec(), nc = t->ncell();
  GIEM_TRY(ensure_vec_ws(t, (size_t)4 * nrhs));
  c128 *ws = static_cast<c128 *>(t->vec_ws);
  c128 *rhs = ws, *lam = ws + (size_t)nrhs * n, *v = ws + (size_t)2 * nrhs * n,
       *w = ws + (size_t)3 * nrhs * n;
  const c128 *dg = static_cast<const c128 *>(t->diag);
  const c128 *R1 = dg + nc, *acell = dg + 3 * nc;
  GIEM_HIP(launch_div_cells(rhs, static_cast<const c128 *>(adj_src), acell, nrhs, nc, s), "g / a");
  std::vector<const c128 *> bp(nrhs);
  std::vector<c128 *> lp(nrhs);
  for (int r = 0; r < nrhs; ++r) {
    bp[r] = rhs + (size_t)r * n;
    lp[r] = lam + (size_t)r * n;
  }
  GmresParams gp;
  gp.tol = o->tol;
  gp.m = o->restart;
  gp.max_iter = o->max_iter;
  gp.weighted = o->weighted_ip;
  gp.mode = MODE_AT;
  gp.prec = PREC_FP64;
  gp.x_zero = true;
  GmresResult gr;
  GIEM_TRY(gmres(t, std::vector<int>(nrhs, ifreq), nrhs, bp.data(), lp.data(), gp, s, gr));
  GIEM_HIP(launch_mul_cells(v, lam, R1, nrhs, nc, s), "R1 lambda");
  std::vector<const c128 *> in(nrhs);
  std::vector<c128 *> out(nrhs);
  for (int r = 0; r < nrhs; ++r) {
    in[r] = v + (size_t)r * n;
    out[r] = w + (size_t)r * n;
  }
  GIEM_TRY(apply_ptrs(t, ifreq, in, out, MODE_B, PREC_FP64, s));
  GIEM_HIP(launch_adjoint_grad(static_cast<const c128 *>(sigma_a), static_cast<const c128 *>(t->sb_lev),
                               acell, static_cast<const c128 *>(adj_src),
                               static_cast<const c128 *>(E_fwd), lam, w, nrhs, t->nx, t->ny, t->nz,
                               static_cast<double *>(grad), s),
           "gradient kernel");
  GIEM_HIP(hipStreamSynchronize(s), "sync");
  if (st) {
    st->iters = gr.iters;
    st->outer_iters = gr.restarts;
    st->converged = gr.converged;
    st->rel_residual = *std::max_element(gr.relres.begin(), gr.relres.end());
    fill_history(*st, gr.hist, 0, nrhs);
    st->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  if (!gr.converged) {
    set_error("adjoint GMRES reached the iteration limit before the tolerance");
    return GIEM_ENOCONV;
  }
  return GIEM_OK;
}

}  // namespace giem

using namespace giem;

extern "C" {

int giem_solve(giem_handle *t, int32_t ifreq, const void *sigma_a, int32_t nrhs, const void *rhs,
               void *E_cells, const giem_solve_opts *opts, giem_solve_stats *stats, void *stream) {
  return solve_impl(t, ifreq, sigma_a, nrhs, rhs, E_cells, opts, stats,
                    static_cast<hipStream_t>(stream), MODE_A);
}

int giem_solve_batch(giem_handle *t, int32_t nf, const int32_t *ifreqs, const void *sigma_a,
                     int32_t nrhs, const void *const *rhs, void *const *E_cells,
                     const giem_solve_opts *opts, giem_solve_stats *stats, void *stream) {
  if (!t || nf < 1 || !ifreqs) {
    set_error("giem_solve_batch: bad argument");
    return GIEM_EINVAL;
  }
  std::vector<int> fi(ifreqs, ifreqs + nf);
  return solve_batch_impl(t, nf, fi.data(), sigma_a, nrhs, rhs, E_cells, opts, stats,
                          static_cast<hipStream_t>(stream), MODE_A);
}

int giem_solve_multi(int32_t ngroups, const giem_solve_group *groups, int32_t nrhs,
                     const giem_solve_opts *opts, giem_solve_stats *stats, void *stream) {
  return solve_groups_impl(ngroups, groups, nrhs, opts, stats, static_cast<hipStream_t>(stream));
}

int giem_adjoint(giem_handle *t, int32_t ifreq, const void *sigma_a, int32_t nrhs,
                 const void *adj_src, const void *E_fwd, void *grad_log_sigma,
                 const giem_solve_opts *opts, giem_solve_stats *stats, void *stream) {
  return adjoint_impl(t, ifreq, sigma_a, nrhs, adj_src, E_fwd, grad_log_sigma, opts, stats,
                      static_cast<hipStream_t>(stream));
}

}  // extern "C"

namespace giem {

// Lattice indices of receivers (or dipole sources) rec_xyz [nrec][3] above
// (or below) cell centres at one common depth z0 in the earth, d[0] <= z0 <=
// the top of the grid (on the first cells' top face, or above the grid), or
// z0 below the grid's bottom; EDOMAIN otherwise.
static int receiver_indices(const giem_handle *t, int nrec, const double *rec_xyz,
                            std::vector<int> &idx, double &z0, const char *who) {
  const double zscale = std::max(t->z_edges[t->nz] - t->d[0], t->z_edges[t->nz] - t->z_edges[0]);
  const double tol = 1e-9 * zscale;
  idx.assign(2 * (size_t)nrec, 0);
  z0 = nrec > 0 ? rec_xyz[2] : t->z_edges[0];
  const bool above = z0 >= t->d[0] - tol && z0 <= t->z_edges[0] + tol;
  const bool below = z0 > t->z_edges[t->nz] + tol;
  if (!above && !below) {
    set_error(std::string(who) + ": points must lie in the earth at or above the top of the "
              "anomaly grid (d[0] <= z <= top of the grid) or below its bottom");
    return GIEM_EDOMAIN;
  }
  if (std::fabs(z0 - t->z_edges[0]) <= tol) z0 = t->z_edges[0];
  if (std::fabs(z0 - t->d[0]) <= tol) z0 = t->d[0];
  for (int q = 0; q < nrec; ++q) {
    const double fx = (rec_xyz[3 * q] - t->x0) / t->hx - 0.5;
    const double fy = (rec_xyz[3 * q + 1] - t->y0) / t->hy - 0.5;
    const double ix = std::round(fx), iy = std::round(fy);
    if (!(std::fabs(rec_xyz[3 * q + 2] - z0) <= tol)) {
      set_error(std::string(who) + ": all points of one call must lie at one depth");
      return GIEM_EDOMAIN;
    }
    if (!(std::fabs(fx - ix) <= 1e-9) || !(std::fabs(fy - iy) <= 1e-9) || ix < 0 ||
        ix >= t->nx || iy < 0 || iy >= t->ny) {
      set_error(std::string(who) + ": points must lie above cell centres of the grid");
      return GIEM_EDOMAIN;
    }
    idx[2 * q] = (int)ix;
    idx[2 * q + 1] = (int)iy;
  }
  return GIEM_OK;
}

// Receiver kernels of frequency ifreq at depth z0, built on first use.
static int receiver_kernel(giem_handle *t, int ifreq, double z0, hipStream_t s, const c128 **K) {
  FreqTables &ft = t->f[ifreq];
  for (auto &rk : ft.rec_kernels)
    if (rk.first == z0) {
      *K = static_cast<const c128 *>(rk.second);
      return GIEM_OK;
    }
  void *k = nullptr;
  GIEM_TRY(compute_receiver_kernels(t, ifreq, z0, &k, s));
  ft.rec_kernels.emplace_back(z0, k);
  *K = static_cast<const c128 *>(k);
  return GIEM_OK;
}

// Device copy of a small host array, freed on scope exit.
struct DevCopy {
  void *p = nullptr;
  ~DevCopy() {
    if (p) hipFree(p);
  }
  int put(const void *h, size_t bytes, hipStream_t s, const char *what) {
    if (check_hip(hipMalloc(&p, bytes), what) ||
        check_hip(hipMemcpyAsync(p, h, bytes, hipMemcpyHostToDevice, s), what))
      return GIEM_EHIP;
    return GIEM_OK;
  }
};

static int fields_impl(giem_handle *t, int32_t ifreq, const void *sigma_a, int32_t nrhs,
                       const void *E_cells, int32_t nrec, const double *rec_xyz, void *E_rec,
                       void *H_rec, void *stream, bool normal, const char *who) {
  if (!t || ifreq < 0 || ifreq >= (int)t->f.size() || !sigma_a || nrhs < 1 || !E_cells ||
      nrec < 0 || (nrec > 0 && (!rec_xyz || !E_rec || !H_rec))) {
    set_error(std::string(who) + ": bad argument");
    return GIEM_EINVAL;
  }
  if (nrec == 0) return GIEM_OK;
  std::vector<int> idx;
  double z0 = 0.0;
  GIEM_TRY(receiver_indices(t, nrec, rec_xyz, idx, z0, who));
  hipStream_t s = static_cast<hipStream_t>(stream);
  const c128 *K = nullptr;
  GIEM_TRY(receiver_kernel(t, ifreq, z0, s, &K));
  // normal fields at the receivers' depth: RHS 0 x polarisation, RHS 1 y
  // polarisation of the unit-surface-field plane wave (H from Faraday's law)
  std::vector<c128> nf((size_t)nrhs * 6, mk<double>(0.0, 0.0));
  if (normal) {
    PlaneWave pw(t->d, t->sigma, t->f[ifreq].freq);
    cd e = 1.0, hy = 1.0 / pw.Zs, de;
    if (z0 != t->d[0]) {
      e = pw.value(z0, &de);
      hy = de / cd(0.0, pw.omega * kMu0);
    }
    if (nrhs >= 1) {
      nf[0] = mk<double>(e.real(), e.imag());
      nf[4] = mk<double>(hy.real(), hy.imag());
    }
    if (nrhs >= 2) {
      nf[6 + 1] = mk<double>(e.real(), e.imag());
      nf[6 + 3] = mk<double>(-hy.real(), -hy.imag());
    }
  }
  DevCopy drec, dnf;
  GIEM_TRY(drec.put(idx.data(), idx.size() * sizeof(int), s, "receivers"));
  GIEM_TRY(dnf.put(nf.data(), nf.size() * sizeof(c128), s, "normal fields"));
  GIEM_HIP(launch_fields(K, static_cast<const c128 *>(E_cells),
                         static_cast<const c128 *>(sigma_a), static_cast<const c128 *>(t->sb_lev),
                         static_cast<const int *>(drec.p), nrec, nrhs, t->nx, t->ny, t->nz,
                         static_cast<const c128 *>(dnf.p), static_cast<c128 *>(E_rec),
                         static_cast<c128 *>(H_rec), s),
           "fields kernel");
  GIEM_HIP(hipStreamSynchronize(s), "fields");
  return GIEM_OK;
}

}  // namespace giem

extern "C" int giem_fields(giem_handle *t, int32_t ifreq, const void *sigma_a, int32_t nrhs,
                           const void *E_cells, int32_t nrec, const double *rec_xyz, void *E_rec,
                           void *H_rec, void *stream) {
  return giem::fields_impl(t, ifreq, sigma_a, nrhs, E_cells, nrec, rec_xyz, E_rec, H_rec, stream,
                           true, "giem_fields");
}

extern "C" int giem_fields_anomalous(giem_handle *t, int32_t ifreq, const void *sigma_a,
                                     int32_t nrhs, const void *E_cells, int32_t nrec,
                                     const double *rec_xyz, void *E_rec, void *H_rec,
                                     void *stream) {
  return giem::fields_impl(t, ifreq, sigma_a, nrhs, E_cells, nrec, rec_xyz, E_rec, H_rec, stream,
                           false, "giem_fields_anomalous");
}

extern "C" int giem_dipole_source(giem_handle *t, int32_t ifreq, int32_t nsrc,
                                  const double *src_xyz, const double *moments, void *rhs,
                                  void *stream) {
  using namespace giem;
  if (!t || ifreq < 0 || ifreq >= (int)t->f.size() || nsrc < 1 || nsrc > kMaxRhs || !src_xyz ||
      !moments || !rhs) {
    set_error("giem_dipole_source: bad argument (1 .. 8 sources)");
    return GIEM_EINVAL;
  }
  for (int q = 0; q < 6 * nsrc; ++q)
    if (!std::isfinite(moments[q])) {
      set_error("giem_dipole_source: moments must be finite");
      return GIEM_EINVAL;
    }
  std::vector<int> idx;
  double z0 = 0.0;
  GIEM_TRY(receiver_indices(t, nsrc, src_xyz, idx, z0, "giem_dipole_source"));
  hipStream_t s = static_cast<hipStream_t>(stream);
  const c128 *K = nullptr;
  GIEM_TRY(receiver_kernel(t, ifreq, z0, s, &K));
  DevCopy dsrc, dmom;
  GIEM_TRY(dsrc.put(idx.data(), idx.size() * sizeof(int), s, "sources"));
  GIEM_TRY(dmom.put(moments, (size_t)nsrc * 3 * sizeof(c128), s, "moments"));
  GIEM_HIP(launch_dipole_rhs(K, static_cast<const int *>(dsrc.p), static_cast<const c128 *>(dmom.p),
                             nsrc, t->nx, t->ny, t->nz, static_cast<const double *>(t->sroot_lev),
                             static_cast<const double *>(t->vol_lev), static_cast<c128 *>(rhs), s),
           "dipole source kernel");
  GIEM_HIP(hipStreamSynchronize(s), "dipole source");
  return GIEM_OK;
}

extern "C" int giem_fields_adjoint(giem_handle *t, int32_t ifreq, const void *sigma_a,
                                   int32_t nrhs, const void *E_cells, int32_t nrec,
                                   const double *rec_xyz, const void *wE, const void *wH,
                                   void *adj_src, void *grad_log_sigma, void *stream) {
  using namespace giem;
  if (!t || ifreq < 0 || ifreq >= (int)t->f.size() || !sigma_a || nrhs < 1 || !E_cells ||
      nrec < 0 || (nrec > 0 && (!rec_xyz || !wE || !wH)) || !adj_src || !grad_log_sigma) {
    set_error("giem_fields_adjoint: bad argument");
    return GIEM_EINVAL;
  }
  std::vector<int> idx;
  double z0 = 0.0;
  if (nrec > 0) GIEM_TRY(receiver_indices(t, nrec, rec_xyz, idx, z0, "giem_fields_adjoint"));
  hipStream_t s = static_cast<hipStream_t>(stream);
  GIEM_TRY(check_sigma_a(t, sigma_a, s));
  const c128 *K = nullptr;
  if (nrec > 0) GIEM_TRY(receiver_kernel(t, ifreq, z0, s, &K));
  DevCopy drec;
  if (nrec > 0) GIEM_TRY(drec.put(idx.data(), idx.size() * sizeof(int), s, "receivers"));
  GIEM_HIP(launch_fields_adjoint(K,
                                 static_cast<const c128 *>(E_cells),
                                 static_cast<const c128 *>(sigma_a),
                                 static_cast<const c128 *>(t->sb_lev),
                                 static_cast<const int *>(drec.p), nrec, nrhs, t->nx, t->ny, t->nz,
                                 static_cast<const c128 *>(wE), static_cast<const c128 *>(wH),
                                 static_cast<c128 *>(adj_src), static_cast<double *>(grad_log_sigma),
                                 s),
           "fields adjoint kernel");
  GIEM_HIP(hipStreamSynchronize(s), "fields adjoint");
  return GIEM_OK;
}

extern "C" int giem_impedance(int32_t nrec, const void *E_rec, const void *H_rec, void *Z,
                              void *stream) {
  using namespace giem;
  if (nrec < 0 || (nrec > 0 && (!E_rec || !H_rec || !Z))) {
    set_error("giem_impedance: bad argument");
    return GIEM_EINVAL;
  }
  GIEM_HIP(launch_impedance(static_cast<const c128 *>(E_rec), static_cast<const c128 *>(H_rec), nrec,
                            static_cast<c128 *>(Z), static_cast<hipStream_t>(stream)),
           "impedance kernel");
  return GIEM_OK;
}

extern "C" int giem_impedance_adjoint(int32_t nrec, const void *E_rec, const void *H_rec,
                                      const void *gZ, void *wE, void *wH, void *stream) {
  using namespace giem;
  if (nrec < 0 || (nrec > 0 && (!E_rec || !H_rec || !gZ || !wE || !wH))) {
    set_error("giem_impedance_adjoint: bad argument");
    return GIEM_EINVAL;
  }
  GIEM_HIP(launch_impedance_adjoint(static_cast<const c128 *>(E_rec),
                                    static_cast<const c128 *>(H_rec), nrec,
                                    static_cast<const c128 *>(gZ), static_cast<c128 *>(wE),
                                    static_cast<c128 *>(wH), static_cast<hipStream_t>(stream)),
           "impedance adjoint kernel");
  return GIEM_OK;
}
