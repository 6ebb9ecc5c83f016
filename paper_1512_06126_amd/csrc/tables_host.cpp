// Coefficient tables B_n^m of eq. (bcyl) for a layered background
// (Sect. 3.1; Appendix A for the Green's tensor, Appendix B for the vertical
// integration, Appendix C for the horizontal integration).
//
// Structure of the computation (every step on the GPU; this file sets up
// the grids, rules and the layered model and drives the kernels of
// kernels_tables.hip), per frequency:
//  1. vertical integrals over every pair of depth cells, for lambda on a
//     logarithmic Chebyshev grid, from the p/q recursions of Appendix B and
//     the factorisation of the fundamental function U_gamma into a solution
//     F that satisfies the conditions above and G that satisfies those below
//     (U(z, z*) ~ F(z_<) G(z_>)); every exponential is evaluated with a
//     non-positive real part (vertical.h);
//  2. zero-order Hankel transforms h(rho) = int J0(lambda rho) g(lambda)
//     dlambda of the five lambda functions, on a logarithmic Chebyshev grid
//     in rho: a geometry-only weight matrix (Gauss-Legendre panels between
//     the zeros of J0, tail summed by repeated averaging), built once per
//     call and contracted with the lambda samples;
//  3. horizontal Galerkin integration: the product of the two cells'
//     footprints becomes their autocorrelation phi (a product of triangles),
//     and the tensor components are convolutions of h with phi, d phi or
//     d^2 phi, evaluated with quadrature rules whose nodes are graded towards
//     the singular vertex; folded onto the rho grid they form a second
//     geometry-only matrix, built once per call and contracted;
//  4. the nine components are formed and packed (upper triangles of xx, xy,
//     yy, zz; full xz, yz).
// The receiver kernels (compute_receiver_kernels) evaluate their lambda
// functions on the host (the same vertical.h); their rule matrix, Hankel
// weights and contractions run on the GPU.
// The lambda-functions, with sigma_n the conductivity of the observation
// cell and P = -i w mu0 A1 + A3 / sigma_n:
//   A1 = int int U_1;  A3 = int int (d_z d_z* U_sigma - 2 delta) (regular
//   part);  A4 = int int d_z U_sigma;  A6 = int int (lambda^2 U_sigma - 2
//   delta);  A2 = int int U_sigma.
//   xx = [i w mu0 phi*h(A1 lambda) + (-d_xx phi)*h(P / lambda)] / 4pi
//   yy likewise with d_yy;  xy = (-d_xy phi)*h(P / lambda) / 4pi
//   xz = (d_x phi)*h(lambda A4 / sigma_n) / 4pi;  yz with d_y
//   zz = phi*h(lambda A6 / sigma_n) / 4pi.
// h(P / lambda) diverges logarithmically at lambda -> 0; it is regularised by
// J0 -> J0 - 1 below a small lambda_a, which shifts it by a constant that the
// zero-mean weights d_xx phi, d_yy phi, d_xy phi annihilate.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <vector>

#include "handle.h"
#include "vertical.h"

namespace giem {

hipError_t launch_gemm_tn(const double *At, int64_t lda, const double *B, int64_t ldb, double *C,
                          int64_t ldc, int m, int n, int k, hipStream_t s,
                          const int *krange = nullptr);
hipError_t launch_assemble(const c128 *c0, const c128 *c1, const c128 *c2, c128 *out, int nx,
                           int ny, int nz, double omega_mu0, hipStream_t s);
hipError_t launch_assemble_rec(const c128 *c, c128 *out, int noff, int nz, double omega_mu0,
                               hipStream_t s);
hipError_t launch_vertical_rows(const vert::Model &m, const double *lam, int nl, vert::zc *eta,
                                double *L, vert::zc *p, vert::zc *q, vert::Cell *cells,
                                vert::zc *G, int ncolc, hipStream_t s);
hipError_t launch_vertical_point(const vert::Model &m, const vert::Observer &ob, const double *lam,
                                 int nl, vert::zc *eta, double *L, vert::zc *p, vert::zc *q,
                                 vert::Cell *cells, vert::zc *G, hipStream_t s);
hipError_t launch_hankel_weights(const double *args, int nzeros, int npan, int nr, int ng1, int ng2,
                                 int nt, double lam_lo, double lam_a, double lam_asym, double *Wt,
                                 double *Wt_reg, hipStream_t s);
hipError_t launch_spatial_fold(const double *args, int npan, int nrad, int nx, int ny, double hx,
                               double hy, double rho_min, double *Mt, int *kcol, hipStream_t s);
hipError_t launch_receiver_fold(const double *args, int npan, int nrad, int nx, int ny, double hx,
                                double hy, double rho_min, double *Mt, int *kcol, hipStream_t s);

namespace {

const double kPi = 3.14159265358979323846;
const double kMu0 = 4e-7 * kPi;

// ---------------------------------------------------------------- quadrature
struct Rule {
  std::vector<double> x, w;  // on [-1, 1]
};

Rule gauss_legendre(int n) {
  Rule r;
  r.x.resize(n);
  r.w.resize(n);
  for (int i = 0; i < n; ++i) {
    double x = std::cos(kPi * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (x * p1 - p0) / (x * x - 1.0);
      const double dx = p1 / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    double p0 = 1.0, p1 = x;
    for (int k = 2; k <= n; ++k) {
      const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    dp = n * (x * p1 - p0) / (x * x - 1.0);
    r.x[n - 1 - i] = x;
    r.w[n - 1 - i] = 2.0 / ((1.0 - x * x) * dp * dp);
  }
  return r;
}

// Double-exponential (tanh-sinh) rule on [0, 1] for integrands with an
// integrable singularity at 0 (here ln x, or x ln x): x = 1 / (1 + e^{-pi
// sinh t}) on the equispaced t = k h, |t| <= t_max, weight h dx/dt.  The
// nodes crowd towards both ends double-exponentially, which resolves the
// logarithm without any knowledge of its coefficient.
Rule tanh_sinh01(double h, double t_max) {
  Rule r;
  const int m = (int)std::floor(t_max / h);
  for (int k = -m; k <= m; ++k) {
    const double tk = k * h;
    const double e = std::exp(-kPi * std::sinh(tk));
    const double x = 1.0 / (1.0 + e);
    const double w = h * kPi * std::cosh(tk) * x * (e / (1.0 + e));
    if (x <= 0.0 || w <= 0.0) continue;
    r.x.push_back(x);
    r.w.push_back(w);
  }
  return r;
}

// Chebyshev-Lobatto panels of equal width in u = ln x (nodes, edges and
// the barycentric weights of a panel).
struct LogGrid {
  std::vector<double> edges, node, bw, x;
  int n = 0;
  // panels of equal width in ln x on [lo, hi]; with lead < lo one more,
  // wider panel [lead, lo] in front (for functions that are nearly linear in
  // ln x there)
  void init(double lo, double hi, double width, int npp, double lead = 0.0) {
    n = npp;
    const double u0 = std::log(lo), u1 = std::log(hi);
    const int np = std::max(1, (int)std::ceil((u1 - u0) / width));
    const int extra = (lead > 0.0 && lead < lo) ? 1 : 0;
    edges.resize(np + 1 + extra);
    if (extra) edges[0] = std::log(lead);
    for (int i = 0; i <= np; ++i) edges[i + extra] = u0 + (u1 - u0) * i / np;
    node.resize(n);
    bw.resize(n);
    for (int j = 0; j < n; ++j) {
      node[j] = -std::cos(kPi * j / (n - 1));
      bw[j] = (j & 1) ? -1.0 : 1.0;
      if (j == 0 || j == n - 1) bw[j] *= 0.5;
    }
    const int npan = np + extra;
    x.resize((size_t)npan * n);
    for (int p = 0; p < npan; ++p)
      for (int j = 0; j < n; ++j)
        x[(size_t)p * n + j] =
            std::exp(0.5 * (edges[p] + edges[p + 1]) + 0.5 * (edges[p + 1] - edges[p]) * node[j]);
  }
  size_t size() const { return x.size(); }
  // (the barycentric interpolation on a panel, and its derivative, run in
  // the rule-matrix kernels of kernels_tables.hip)
};


// ------------------------------------------------------------ Bessel zeros
std::vector<double> j0_zeros(int count) {
  std::vector<double> z(count);
  for (int s = 1; s <= count; ++s) {
    const double b = (s - 0.25) * kPi;
    double x = b + 1.0 / (8.0 * b) - 124.0 / (3.0 * std::pow(8.0 * b, 3));
    for (int it = 0; it < 20; ++it) {
      const double dx = std::cyl_bessel_j(0.0, x) / (-std::cyl_bessel_j(1.0, x));
      x -= dx;
      if (std::fabs(dx) < 1e-15 * x) break;
    }
    z[s - 1] = x;
  }
  return z;
}

// -------------------------------------------------------- grid parameters
struct Grids {
  LogGrid lam, rho;
  double lam_lo, lam_a, lam_asym, rho_min;
  int ntail = 30, levels = 14, ngl_main = 16, ngl_first = 12;
};

Grids make_grids(const giem_handle *t) {
  Grids g;
  double hmin = 1e300;
  for (int l = 0; l < t->nz; ++l) hmin = std::min(hmin, t->z_edges[l + 1] - t->z_edges[l]);
  const double href = std::min(t->hx, t->hy);
  // The radial functions grow like ln(1 / rho) at rho -> 0 and the line and
  // vertex rules evaluate them down to rho ~ 1e-12 h: below that the
  // clamped remainder is of relative size 1e-12.  Between rho_min and
  // 1e-9 h they contribute at most ~1e-9 of a coefficient, so one panel
  // (12 nodes over a factor 1000 in rho) resolves them well enough even where
  // they grow like 1 / rho (faces of touching cells).
  g.rho_min = 1e-12 * href;
  const double rho_max = 1.05 * std::hypot((t->nx + 1) * t->hx, (t->ny + 1) * t->hy);
  const double zmax = t->z_edges[t->nz];
  const double scale = std::max(rho_max, zmax);
  g.lam_asym = 40.0 / hmin;
  g.lam_lo = 1e-9 / scale;
  g.lam_a = 1e-3 / scale;
  const double lam_hi = 1.1 * (g.lam_asym + (g.ntail + 3) * kPi / g.rho_min);
  g.lam.init(0.5 * g.lam_lo, lam_hi, 0.5, 16);
  g.rho.init(1e-9 * href, rho_max, 0.5, 12, g.rho_min);
  return g;
}

struct DevBuf {
  void *p = nullptr;
  ~DevBuf() {
    if (p) hipFree(p);
  }
  hipError_t alloc(size_t bytes) { return hipMalloc(&p, bytes); }
  double *d() { return static_cast<double *>(p); }
  c128 *c() { return static_cast<c128 *>(p); }
};

// Hankel weights: rows Wt[lam][rho] (transposed for the GEMM) for the plain
// transform and for the regularised one, computed on the GPU
// (launch_hankel_weights) from what is set up here: the zeros of J0 that the
// panels need, the lambda grid, the rho nodes, the Gauss-Legendre rules of
// the first and the main panels, and the tail weights beta_i, the averaged
// limit of the last partial sums (binomial averaging over `levels` levels).
int hankel_weights(const Grids &g, double *dWt, double *dWt_reg, hipStream_t s) {
  const size_t nr = g.rho.size();
  const int npan = (int)g.lam.edges.size() - 1;
  if (g.lam.n != 16) {
    set_error("giem_tables: the lambda grid must have 16 nodes per panel");
    return GIEM_EINVAL;
  }
  const double rho_max = g.rho.x.back();
  const int kmax = (int)std::ceil(g.lam_asym * rho_max / kPi) + 1;
  const std::vector<double> zeros = j0_zeros(kmax + g.ntail + 2);
  const Rule r1 = gauss_legendre(g.ngl_first), r2 = gauss_legendre(g.ngl_main);
  const int nt = g.ntail, lv = std::min(g.levels, nt - 1);
  std::vector<double> c(nt, 0.0), beta(nt, 0.0);
  {
    std::vector<double> binom(lv + 1, 1.0);
    for (int i = 1; i <= lv; ++i) binom[i] = binom[i - 1] * (lv - i + 1) / i;
    for (int i = 0; i <= lv; ++i) c[nt - 1 - lv + i] = binom[i] / std::ldexp(1.0, lv);
    double acc = 0.0;
    for (int i = nt - 1; i >= 0; --i) {
      acc += c[i];
      beta[i] = acc;
    }
  }
  std::vector<double> args;
  auto put = [&](const std::vector<double> &v) { args.insert(args.end(), v.begin(), v.end()); };
  put(zeros);
  put(g.lam.edges);
  put(g.lam.node);
  put(g.lam.bw);
  put(g.rho.x);
  put(r1.x);
  put(r1.w);
  put(r2.x);
  put(r2.w);
  put(beta);
  DevBuf dargs;
  if (dargs.alloc(args.size() * 8) != hipSuccess) {
    (void)hipGetLastError();
    set_error("giem_tables: out of device memory");
    return GIEM_ENOMEM;
  }
  if (check_hip(hipMemcpyAsync(dargs.p, args.data(), args.size() * 8, hipMemcpyHostToDevice, s),
                "upload Hankel rules") ||
      check_hip(launch_hankel_weights(dargs.d(), (int)zeros.size(), npan, (int)nr, (int)r1.x.size(),
                                      (int)r2.x.size(), nt, g.lam_lo, g.lam_a, g.lam_asym, dWt,
                                      dWt_reg, s),
                "Hankel weights") ||
      check_hip(hipStreamSynchronize(s), "Hankel weights"))  // before dargs is freed
    return GIEM_EHIP;
  return GIEM_OK;
}

// ----------------------------------------------------- horizontal rules
enum { K_W0 = 0, K_XX, K_YY, K_XY, K_X, K_Y, K_COUNT };

// radial variable of the two triangles at a singular vertex (integrand
// r h(r ...), h ~ ln r) and the singular ends of the line rules
const Rule &radial_rule() {
  static const Rule r = tanh_sinh01(1.0 / 8.0, 3.75);
  return r;
}

// What the rule-matrix kernels read: the rho grid (edges, nodes and
// barycentric weights of a panel), Gauss-Legendre rules of 24, 14 and 8
// points and the radial (tanh-sinh) rule, nodes then weights.
std::vector<double> fold_args(const Grids &g, int &nrad) {
  const Rule gs = gauss_legendre(24), g14 = gauss_legendre(14), g8 = gauss_legendre(8);
  const Rule &rad = radial_rule();
  std::vector<double> args;
  auto put = [&](const std::vector<double> &v) { args.insert(args.end(), v.begin(), v.end()); };
  put(g.rho.edges);
  put(g.rho.node);
  put(g.rho.bw);
  put(gs.x);
  put(gs.w);
  put(g14.x);
  put(g14.w);
  put(g8.x);
  put(g8.w);
  put(rad.x);
  put(rad.w);
  nrad = (int)rad.x.size();
  return args;
}

// Spatial fold matrices Mt[rho][kind * noff + (i Nx + j)] for i, j >= 0,
// built on the GPU (launch_spatial_fold) into dMt from the rho grid and the
// quadrature rules set up here.  Rows of Mt with a non-zero entry in column c
// lie in [kcol[2c], kcol[2c+1]) (copied back into kcol).
int spatial_matrix(const giem_handle *t, const Grids &g, double *dMt, int *dkcol,
                   std::vector<int> &kcol, hipStream_t s) {
  const size_t noff = (size_t)t->nx * t->ny, nr = g.rho.size(), ncol = K_COUNT * noff;
  if (g.rho.n != 12) {
    set_error("giem_tables: the rho grid must have 12 nodes per panel");
    return GIEM_EINVAL;
  }
  int nrad = 0;
  const std::vector<double> args = fold_args(g, nrad);
  DevBuf dargs;
  if (dargs.alloc(args.size() * 8) != hipSuccess) {
    (void)hipGetLastError();
    set_error("giem_tables: out of device memory");
    return GIEM_ENOMEM;
  }
  kcol.resize(2 * ncol);
  if (check_hip(hipMemsetAsync(dMt, 0, nr * ncol * 8, s), "clear spatial weights") ||
      check_hip(hipMemcpyAsync(dargs.p, args.data(), args.size() * 8, hipMemcpyHostToDevice, s),
                "upload spatial rules") ||
      check_hip(launch_spatial_fold(dargs.d(), (int)g.rho.edges.size() - 1, nrad, t->nx, t->ny,
                                    t->hx, t->hy, g.rho_min, dMt, dkcol, s),
                "spatial weights") ||
      check_hip(hipMemcpyAsync(kcol.data(), dkcol, kcol.size() * sizeof(int),
                               hipMemcpyDeviceToHost, s),
                "spatial weight ranges") ||
      check_hip(hipStreamSynchronize(s), "spatial weights"))
    return GIEM_EHIP;
  return GIEM_OK;
}

// Contraction range of each 64-row tile of a GEMM over the columns col0 ..
// col0 + m of a rule matrix: the union of its columns' row ranges, widened to
// whole steps of 4 so that the tile's MFMAs visit the same 4-row groups as a
// dense loop (the groups skipped hold only zeros: the result is unchanged)
std::vector<int> tile_ranges(const std::vector<int> &kcol, size_t col0, int m) {
  const int nt = (m + 63) / 64;
  std::vector<int> r(2 * (size_t)nt);
  for (int tile = 0; tile < nt; ++tile) {
    int lo = 1 << 30, hi = 0;
    for (int c = tile * 64; c < std::min(m, tile * 64 + 64); ++c) {
      const int a = kcol[2 * (col0 + c)], b = kcol[2 * (col0 + c) + 1];
      if (a >= b) continue;
      lo = std::min(lo, a);
      hi = std::max(hi, b);
    }
    if (lo >= hi) lo = hi = 0;
    r[2 * tile] = lo / 4 * 4;
    r[2 * tile + 1] = (hi + 3) / 4 * 4;
  }
  return r;
}

// ------------------------------------------- receiver (point) rules
// A receiver above the centre of a cell at lateral offset (dx, dy) from the
// centre of the source cell sees the source footprint B = [-hx/2, hx/2] x
// [-hy/2, hy/2]: the plain terms need int_B h(|D - r'|) d^2 r', the i kx /
// i ky terms the line measures d_x B (faces x = -hx/2 with +1, x = +hx/2
// with -1) and d_y B, and the kx^2, ky^2, kx ky terms the same faces against
// -d h / d x or -d h / d y (derivative weights).
enum { R_B0 = 0, R_BX, R_BY, R_BXX, R_BYY, R_BXY, R_COUNT };

// ----------------------------------------------------- vertical functions
typedef std::complex<double> cx;

struct Layering {
  int nlay;                   // number of interfaces
  std::vector<double> d;      // [nlay]
  std::vector<cx> sigma;      // [nlay + 1]
};

// The layered model seen from the depth cells (and from a point observer for
// the receiver kernels): each cell's layer and local edge depths, the point
// observer's layer and gap pieces; the vertical functions themselves are
// computed on the GPU from these (vertical.h).
struct Vertical {
  const giem_handle *t;
  int nz;
  std::vector<int> lay;          // layer of each cell
  std::vector<double> ta, tb;    // local coordinates of the cell edges
  std::vector<vert::zc> sig;     // layer conductivities [nlay + 1]
  // point observer (receiver kernels) at depth z0 in the earth, at or above
  // the top of the grid: the gap [z0, top of the grid] split at interfaces
  // into pieces (layer, local top, local bottom); empty when z0 is the top
  // (or below the grid: the gap [bottom of the grid, z0])
  double z0 = 0.0;
  int lay_obs = 1;
  bool below = false;
  std::vector<int> gap_lay;
  std::vector<double> gap_ta, gap_tb;
  void set_observer(double z) {
    z0 = z;
    gap_lay.clear();
    gap_ta.clear();
    gap_tb.clear();
    const double top = t->z_edges[0], bot = t->z_edges[nz];
    auto layer_at = [&](double zz) {  // layer holding depth zz from below
      int n = 1;
      while (n < t->nlay && t->d[n] <= zz) ++n;
      return n;
    };
    below = z0 > bot;
    lay_obs = (z0 < top || below) ? layer_at(z0) : lay.empty() ? 1 : lay[0];
    double a = below ? bot : z0;
    const double end = below ? z0 : top;
    while (a < end) {
      const int n = layer_at(a);
      const double b = (n < t->nlay) ? std::min(end, t->d[n]) : end;
      gap_lay.push_back(n);
      gap_ta.push_back(a - t->d[n - 1]);
      gap_tb.push_back(b - t->d[n - 1]);
      a = b;
    }
  }
  void init(const giem_handle *h) {
    t = h;
    nz = h->nz;
    lay.resize(nz);
    ta.resize(nz);
    tb.resize(nz);
    sig.resize(h->sigma.size());
    for (size_t n = 0; n < sig.size(); ++n) sig[n] = vert::Z(h->sigma[n].real(), h->sigma[n].imag());
    for (int l = 0; l < nz; ++l) {
      const int n = h->layer_of_cell[l];
      lay[l] = n;
      const double top = h->d[n - 1];
      ta[l] = h->z_edges[l] - top;
      tb[l] = h->z_edges[l + 1] - top;
    }
    set_observer(h->z_edges[0]);
  }

  // large-lambda limit of lambda^2 A2 - 2 for the observer on the top face
  // of its own cell: every eta tends to lambda, so lambda^2 A2 -> 1 + p with
  // p -> (s0 - s1) / (s0 + s1) when an interface lies at that face (s0 the
  // layer above, e.g. the air at the surface) and p -> 0 when the cell's
  // layer continues above it (a grid below the top of its layer)
  cx a6_inf() const {
    const int n = lay[0];
    const cx s1 = t->sigma[n];
    const double top = t->z_edges[0], dn = t->d[n - 1];
    const bool interface = std::fabs(top - dn) <= 1e-9 * (t->z_edges[nz] - top);
    const cx s0 = interface ? t->sigma[n - 1] : s1;
    return (s0 - s1) / (s0 + s1) - 1.0;
  }
};


}  // namespace

namespace {

// The layered model, the lambda nodes and the workspace of the vertical
// functions on the device: sigma [nlay + 1] (complex), d [nlay], ta, tb [nz],
// lambda [nl], then the cells' layers [nz] and, for a point observer, its
// gap pieces (layer; local top and bottom); eta, p, q (complex) and L per
// node and layer, and the cell factors of both kinds per node and cell.
struct VertDev {
  DevBuf mod, ilay, ws, cell;
  std::vector<double> hmod;  // kept until the uploads have run
  std::vector<int> hlay;
  vert::Model m{};
  vert::Observer ob{};
  const double *lam = nullptr;
  vert::zc *eta = nullptr, *p = nullptr, *q = nullptr;
  double *L = nullptr;
  vert::Cell *cells = nullptr;

  int init(const giem_handle *t, const Vertical &v, const std::vector<double> &lamx,
           hipStream_t s) {
    const int nz = t->nz, nlayers = t->nlay + 1, ngap = (int)v.gap_lay.size();
    const size_t nl = lamx.size();
    hmod.clear();
    for (int n = 0; n < nlayers; ++n) {
      hmod.push_back(v.sig[n].x);
      hmod.push_back(v.sig[n].y);
    }
    hmod.insert(hmod.end(), t->d.begin(), t->d.end());
    hmod.insert(hmod.end(), v.ta.begin(), v.ta.end());
    hmod.insert(hmod.end(), v.tb.begin(), v.tb.end());
    hmod.insert(hmod.end(), lamx.begin(), lamx.end());
    hmod.insert(hmod.end(), v.gap_ta.begin(), v.gap_ta.end());
    hmod.insert(hmod.end(), v.gap_tb.begin(), v.gap_tb.end());
    hlay = v.lay;
    hlay.insert(hlay.end(), v.gap_lay.begin(), v.gap_lay.end());
    const size_t nws = nl * nlayers;  // (node, layer) pairs
    if (mod.alloc(hmod.size() * 8) != hipSuccess || ilay.alloc(hlay.size() * sizeof(int)) != hipSuccess ||
        ws.alloc(nws * (5 * sizeof(vert::zc) + sizeof(double))) != hipSuccess ||
        cell.alloc(nl * 2 * nz * sizeof(vert::Cell)) != hipSuccess) {
      (void)hipGetLastError();
      set_error("out of device memory for the vertical functions");
      return GIEM_ENOMEM;
    }
    if (check_hip(hipMemcpyAsync(mod.p, hmod.data(), hmod.size() * 8, hipMemcpyHostToDevice, s),
                  "upload layered model") ||
        check_hip(hipMemcpyAsync(ilay.p, hlay.data(), hlay.size() * sizeof(int),
                                 hipMemcpyHostToDevice, s),
                  "upload layered model"))
      return GIEM_EHIP;
    m.nz = nz;
    m.nlay = t->nlay;
    m.sigma = reinterpret_cast<const vert::zc *>(mod.d());
    m.d = mod.d() + 2 * nlayers;
    m.ta = m.d + t->nlay;
    m.tb = m.ta + nz;
    lam = m.tb + nz;
    m.lay = static_cast<const int *>(ilay.p);
    ob.z0 = v.z0;
    ob.lay_obs = v.lay_obs;
    ob.below = v.below;
    ob.ngap = ngap;
    ob.gap_ta = lam + nl;
    ob.gap_tb = ob.gap_ta + ngap;
    ob.gap_lay = m.lay + nz;
    const vert::zc a6 = vert::Z(v.a6_inf().real(), v.a6_inf().imag());
    ob.a6 = a6;
    eta = static_cast<vert::zc *>(ws.p);
    p = eta + nws;
    q = p + 2 * nws;
    L = reinterpret_cast<double *>(q + 2 * nws);
    cells = static_cast<vert::Cell *>(cell.p);
    return GIEM_OK;
  }
};

}  // namespace

int compute_tables(giem_handle *t, hipStream_t s) {
  const int nx = t->nx, ny = t->ny, nz = t->nz;
  const int T = nz * (nz + 1) / 2, nz2 = nz * nz;
  const int ncolc = 3 * T + nz2;  // complex columns of G and H
  const size_t noff = (size_t)nx * ny;
  if (noff * K_COUNT > (size_t)64 * 65535 * 1024) {
    set_error("giem_tables: grid too large for the table build");
    return GIEM_EINVAL;
  }
  const Grids g = make_grids(t);
  const size_t nl = g.lam.size(), nr = g.rho.size();
  // contraction ranges of the three spatial GEMMs' row tiles (filled below)
  const size_t kr1 = 2 * ((noff + 63) / 64), kr2 = kr1 + 2 * ((3 * noff + 63) / 64);
  const size_t nkr = kr2 + 2 * ((2 * noff + 63) / 64);
  const size_t ncolm = (size_t)K_COUNT * noff;
  Vertical v;
  v.init(t);
  DevBuf dW, dWr, dM, dG, dH, dc0, dc1, dc2, dkr, dkcol;
  if (dW.alloc(nl * nr * 8) != hipSuccess || dWr.alloc(nl * nr * 8) != hipSuccess ||
      dM.alloc(nr * ncolm * 8) != hipSuccess || dkcol.alloc(2 * ncolm * sizeof(int)) != hipSuccess ||
      dG.alloc(nl * ncolc * 16) != hipSuccess ||
      dH.alloc(nr * ncolc * 16) != hipSuccess || dc0.alloc(noff * 2 * T * 16) != hipSuccess ||
      dc1.alloc(3 * noff * T * 16) != hipSuccess || dc2.alloc(2 * noff * nz2 * 16) != hipSuccess ||
      dkr.alloc(nkr * sizeof(int)) != hipSuccess) {
    (void)hipGetLastError();  // reported here, not by the next launch check
    set_error("giem_tables: out of device memory");
    return GIEM_ENOMEM;
  }
  std::vector<int> kcol, kr;
  {
    int rc = hankel_weights(g, dW.d(), dWr.d(), s);
    if (rc == GIEM_OK) rc = spatial_matrix(t, g, dM.d(), static_cast<int *>(dkcol.p), kcol, s);
    if (rc != GIEM_OK) return rc;
    kr = tile_ranges(kcol, 0, (int)noff);
    const std::vector<int> a = tile_ranges(kcol, K_XX * noff, (int)(3 * noff));
    const std::vector<int> b = tile_ranges(kcol, K_X * noff, (int)(2 * noff));
    kr.insert(kr.end(), a.begin(), a.end());
    kr.insert(kr.end(), b.begin(), b.end());
  }
  VertDev vd;
  {
    const int rc = vd.init(t, v, g.lam.x, s);
    if (rc != GIEM_OK) return rc;
  }
  if (check_hip(hipMemcpyAsync(dkr.p, kr.data(), kr.size() * sizeof(int), hipMemcpyHostToDevice, s),
                "upload contraction ranges"))
    return GIEM_EHIP;
  const int *dkr0 = static_cast<const int *>(dkr.p);
  for (size_t q = 0; q < t->f.size(); ++q) {
    vd.m.omega_mu0 = 2 * kPi * t->f[q].freq * kMu0;
    if (check_hip(launch_vertical_rows(vd.m, vd.lam, (int)nl, vd.eta, vd.L, vd.p, vd.q, vd.cells,
                                       static_cast<vert::zc *>(dG.p), ncolc, s),
                  "vertical functions"))
      return GIEM_EHIP;
    const int64_t ldg = 2 * (int64_t)ncolc;  // doubles per row of G and H
    // H[:, P] = W_reg G[:, P];  H[:, rest] = W G[:, rest]
    if (check_hip(launch_gemm_tn(dWr.d(), nr, dG.d(), ldg, dH.d(), ldg, (int)nr, 2 * T, (int)nl, s),
                  "Hankel contraction") ||
        check_hip(launch_gemm_tn(dW.d(), nr, dG.d() + 2 * T, ldg, dH.d() + 2 * T, ldg, (int)nr,
                                 2 * (2 * T + nz2), (int)nl, s),
                  "Hankel contraction"))
      return GIEM_EHIP;
    const int64_t ldm = (int64_t)K_COUNT * noff;
    // c0 = M_W0 [A1 | A6];  c1 = M_{XX,YY,XY} P;  c2 = M_{X,Y} A4
    if (check_hip(launch_gemm_tn(dM.d(), ldm, dH.d() + 2 * T, ldg, dc0.d(), 4 * T, (int)noff, 4 * T,
                                 (int)nr, s, dkr0),
                  "spatial contraction") ||
        check_hip(launch_gemm_tn(dM.d() + K_XX * noff, ldm, dH.d(), ldg, dc1.d(), 2 * T,
                                 (int)(3 * noff), 2 * T, (int)nr, s, dkr0 + kr1),
                  "spatial contraction") ||
        check_hip(launch_gemm_tn(dM.d() + K_X * noff, ldm, dH.d() + 6 * T, ldg, dc2.d(), 2 * nz2,
                                 (int)(2 * noff), 2 * nz2, (int)nr, s, dkr0 + kr2),
                  "spatial contraction") ||
        check_hip(hipMalloc(&t->f[q].spatial, noff * t->E() * 16), "hipMalloc spatial table") ||
        check_hip(launch_assemble(dc0.c(), dc1.c(), dc2.c(), static_cast<c128 *>(t->f[q].spatial),
                                  nx, ny, nz, t->f[q].freq * 2 * kPi * kMu0, s),
                  "table assembly") ||
        check_hip(hipStreamSynchronize(s), "table build"))
      return GIEM_EHIP;
  }
  return GIEM_OK;
}

// Receiver kernels of one frequency: for receivers above cell centres at
// lateral offset (di hx, dj hy) from a source cell of level jz, the cell
// integrals of G^E and G^H, out[((dj + Ny - 1)(2 Nx - 1) + di + Nx - 1) nz +
// jz][18] (E row-major, then H).  Receivers are at depth z0 in the earth,
// d[0] <= z0 <= top of the grid (the top itself: on the first cell's face),
// or below the grid (z0 > its bottom).
int compute_receiver_kernels(giem_handle *t, int ifreq, double z0, void **out, hipStream_t s) {
  const int nx = t->nx, ny = t->ny, nz = t->nz;
  const int nxo = 2 * nx - 1, nyo = 2 * ny - 1;
  const size_t noff = (size_t)nxo * nyo;
  const int nf = 8 * nz;  // complex functions per lambda
  const Grids g = make_grids(t);
  const size_t nl = g.lam.size(), nr = g.rho.size();
  Vertical v;
  v.init(t);
  v.set_observer(z0);
  const bool touching = v.gap_lay.empty() && !v.below;
  const size_t ncolr = (size_t)R_COUNT * noff;
  DevBuf dW, dWr, dM, dG, dH, dC, dkr, dkcol;
  void *dK = nullptr;
  if (dW.alloc(nl * nr * 8) != hipSuccess || dWr.alloc(nl * nr * 8) != hipSuccess ||
      dM.alloc(nr * ncolr * 8) != hipSuccess || dkcol.alloc(2 * ncolr * sizeof(int)) != hipSuccess ||
      dG.alloc(nl * nf * 16) != hipSuccess ||
      dH.alloc(nr * nf * 16) != hipSuccess || dC.alloc((size_t)R_COUNT * noff * nf * 16) != hipSuccess ||
      dkr.alloc(2 * ((ncolr + 63) / 64) * sizeof(int)) != hipSuccess ||
      hipMalloc(&dK, noff * nz * 18 * sizeof(c128)) != hipSuccess) {
    if (dK) hipFree(dK);
    (void)hipGetLastError();  // reported here, not by the next launch check
    set_error("giem_fields: out of device memory for the receiver kernels");
    return GIEM_ENOMEM;
  }
  const int64_t ldg = 2 * (int64_t)nf;
  const int64_t ldm = (int64_t)R_COUNT * noff;
  int rc = GIEM_OK;
  std::vector<int> kr;
  {
    int hrc = hankel_weights(g, dW.d(), dWr.d(), s);
    if (hrc == GIEM_OK) {
      // the receiver rule matrix on the GPU, its row ranges back for the
      // contraction ranges
      int nrad = 0;
      const std::vector<double> args = fold_args(g, nrad);
      std::vector<int> kcol(2 * ncolr);
      DevBuf dargs;
      if (dargs.alloc(args.size() * 8) != hipSuccess) {
        (void)hipGetLastError();
        set_error("giem_fields: out of device memory for the receiver kernels");
        hrc = GIEM_ENOMEM;
      } else if (check_hip(hipMemsetAsync(dM.p, 0, nr * ncolr * 8, s), "clear receiver weights") ||
                 check_hip(hipMemcpyAsync(dargs.p, args.data(), args.size() * 8,
                                          hipMemcpyHostToDevice, s),
                           "upload receiver rules") ||
                 check_hip(launch_receiver_fold(dargs.d(), (int)g.rho.edges.size() - 1, nrad, nx, ny,
                                                t->hx, t->hy, g.rho_min, dM.d(),
                                                static_cast<int *>(dkcol.p), s),
                           "receiver weights") ||
                 check_hip(hipMemcpyAsync(kcol.data(), dkcol.p, kcol.size() * sizeof(int),
                                          hipMemcpyDeviceToHost, s),
                           "receiver weight ranges") ||
                 check_hip(hipStreamSynchronize(s), "receiver weights")) {
        hrc = GIEM_EHIP;
      } else {
        kr = tile_ranges(kcol, 0, (int)ncolr);
      }
    }
    if (hrc != GIEM_OK) {
      hipFree(dK);
      return hrc;
    }
  }
  // the observer's lambda functions on the GPU
  VertDev vd;
  {
    const int vrc = vd.init(t, v, g.lam.x, s);
    if (vrc != GIEM_OK) {
      hipFree(dK);
      return vrc;
    }
    vd.m.omega_mu0 = 2 * kPi * t->f[ifreq].freq * kMu0;
  }
  if (check_hip(launch_vertical_point(vd.m, vd.ob, vd.lam, (int)nl, vd.eta, vd.L, vd.p, vd.q,
                                      vd.cells, static_cast<vert::zc *>(dG.p), s),
                "receiver vertical functions") ||
      check_hip(hipMemcpyAsync(dkr.p, kr.data(), kr.size() * sizeof(int), hipMemcpyHostToDevice, s),
                "upload") ||
      // plain functions 0..5, regularised 6..7
      check_hip(launch_gemm_tn(dW.d(), nr, dG.d(), ldg, dH.d(), ldg, (int)nr, 2 * 6 * nz, (int)nl, s),
                "receiver Hankel contraction") ||
      check_hip(launch_gemm_tn(dWr.d(), nr, dG.d() + 2 * 6 * nz, ldg, dH.d() + 2 * 6 * nz, ldg,
                               (int)nr, 2 * 2 * nz, (int)nl, s),
                "receiver Hankel contraction") ||
      check_hip(launch_gemm_tn(dM.d(), ldm, dH.d(), ldg, dC.d(), ldg, (int)(R_COUNT * noff), 2 * nf,
                               (int)nr, s, static_cast<const int *>(dkr.p)),
                "receiver spatial contraction") ||
      check_hip(launch_assemble_rec(dC.c(), static_cast<c128 *>(dK), (int)noff, nz,
                                    2 * kPi * t->f[ifreq].freq * kMu0, s),
                "receiver kernel assembly") ||
      check_hip(hipStreamSynchronize(s), "receiver kernels"))
    rc = GIEM_EHIP;
  if (rc == GIEM_OK && touching) {
    // delta part of G_zz for the own cell (offset 0, level 0): the constant
    // a6_inf / s transforms to 2 pi a6_inf / s times the footprint's
    // indicator, i.e. a6_inf / (2 s) after the 1 / 4pi
    const cx add = v.a6_inf() / (2.0 * t->sigma[t->layer_of_cell[0]]);
    const size_t o0 = (size_t)(ny - 1) * nxo + (nx - 1);
    c128 *kzz = static_cast<c128 *>(dK) + (o0 * nz + 0) * 18 + 8;
    c128 val;
    if (check_hip(hipMemcpy(&val, kzz, sizeof(c128), hipMemcpyDeviceToHost), "read kernel") ||
        (val = mk<double>(val.x + add.real(), val.y + add.imag()),
         check_hip(hipMemcpy(kzz, &val, sizeof(c128), hipMemcpyHostToDevice), "write kernel")))
      rc = GIEM_EHIP;
  }
  if (rc != GIEM_OK) {
    hipFree(dK);
    return rc;
  }
  *out = dK;
  return GIEM_OK;
}

}  // namespace giem
