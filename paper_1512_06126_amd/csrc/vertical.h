// Vertical functions of the coefficient tables (Appendix B): the p/q
// recursions of the layered medium and the per-cell factors of the
// fundamental function U(z, z*) ~ F(z_<) G(z_>) / (eta D), written once for
// the host (receiver kernels) and the device (the lambda rows of the
// coefficient tables, computed for every lambda node in parallel).
//
// In layer n, with local depth t from the layer's top, thickness L (infinite
// for the lower half-space), eta = sqrt(lambda^2 - i w mu0 sigma) (Re >= 0):
//   F(t) = e^{eta t} + p e^{-eta t}        (conditions above: p from the top)
//   G(t) = e^{-eta t} (1 + q e^{-2 eta (L - t)})  (below: q from the bottom)
//   D = 1 - p q e^{-2 eta L}.
// Kind 0 uses gamma = 1, kind 1 gamma = sigma in the interface conditions
// (continuity of U and of U' / gamma).  Every exponential has a
// non-positive real part.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace giem {
namespace vert {

// layer thicknesses at or above this are the half-spaces (stored as infinity)
constexpr double kFinite = 1e300;

struct zc {
  double x, y;
};
__host__ __device__ inline zc Z(double a, double b = 0.0) { return zc{a, b}; }
__host__ __device__ inline zc operator+(zc a, zc b) { return Z(a.x + b.x, a.y + b.y); }
__host__ __device__ inline zc operator-(zc a, zc b) { return Z(a.x - b.x, a.y - b.y); }
__host__ __device__ inline zc operator-(zc a) { return Z(-a.x, -a.y); }
__host__ __device__ inline zc operator*(zc a, zc b) {
  return Z(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ inline zc operator*(double s, zc a) { return Z(s * a.x, s * a.y); }
__host__ __device__ inline zc operator*(zc a, double s) { return Z(s * a.x, s * a.y); }
__host__ __device__ inline zc operator+(double s, zc a) { return Z(s + a.x, a.y); }
__host__ __device__ inline zc operator-(double s, zc a) { return Z(s - a.x, -a.y); }
__host__ __device__ inline zc operator-(zc a, double s) { return Z(a.x - s, a.y); }
__host__ __device__ inline zc operator+(zc a, double s) { return Z(a.x + s, a.y); }
__host__ __device__ inline zc operator/(zc a, zc b) {
  // scaled by the larger part of b (Smith's method)
  if (::fabs(b.x) >= ::fabs(b.y)) {
    const double r = b.y / b.x, den = b.x + b.y * r;
    return Z((a.x + a.y * r) / den, (a.y - a.x * r) / den);
  }
  const double r = b.x / b.y, den = b.x * r + b.y;
  return Z((a.x * r + a.y) / den, (a.y * r - a.x) / den);
}
__host__ __device__ inline zc operator/(zc a, double s) { return Z(a.x / s, a.y / s); }
__host__ __device__ inline double zabs(zc a) { return ::hypot(a.x, a.y); }
__host__ __device__ inline zc zexp(zc a) {
  const double e = ::exp(a.x);
  return Z(e * ::cos(a.y), e * ::sin(a.y));
}
// principal square root (Re >= 0)
__host__ __device__ inline zc zsqrt(zc a) {
  const double r = zabs(a);
  if (r == 0.0) return Z(0.0, 0.0);
  const double t = ::sqrt(0.5 * (r + ::fabs(a.x)));
  if (a.x >= 0.0) return Z(t, a.y / (2.0 * t));
  return Z(::fabs(a.y) / (2.0 * t), ::copysign(t, a.y));
}

// Functions of x = eta h (Re x >= 0) that cancel for small |x|, by their
// power series there:
//   eps(x) = (1 - e^-x) / x       = sum_m (-x)^m / (m+1)!
//   phi(x) = (x - 1 + e^-x) / x^2 = sum_m (-x)^m / (m+2)!
//   psi(x) = (e^x - 1 - x) / x^2  = sum_m   x^m / (m+2)!
__host__ __device__ inline zc series(zc x, int shift, bool alternate) {
  zc s = Z(0.0), term = Z(1.0);
  double fact = 1.0;
  for (int q = 2; q <= shift; ++q) fact *= q;
  for (int m = 0; m < 24; ++m) {
    s = s + term / fact;
    term = term * (alternate ? -x : x);
    fact *= (m + 1 + shift);
  }
  return s;
}
__host__ __device__ inline zc f_eps(zc x) {
  return zabs(x) < 0.5 ? series(x, 1, true) : (1.0 - zexp(-x)) / x;
}
__host__ __device__ inline zc f_phi(zc x) {
  return zabs(x) < 0.5 ? series(x, 2, true) : (x - 1.0 + zexp(-x)) / (x * x);
}
// damp psi(x) and damp (e^x - 1) with damp = e^{-2 eta L}, L >= h (no
// overflow for large x: damp e^x = e^{x - 2 eta L})
__host__ __device__ inline zc f_psi_damped(zc x, zc damp, zc e_x_damped) {
  if (zabs(x) < 0.5) return damp * series(x, 2, false);
  return (e_x_damped - damp * (1.0 + x)) / (x * x);
}
__host__ __device__ inline zc f_expm1_damped(zc x, zc damp, zc e_x_damped) {
  if (zabs(x) < 0.5) return damp * x * series(x, 1, false);
  return e_x_damped - damp;
}

// The layered model as the vertical functions need it (host or device
// arrays): nlay interfaces d[0..nlay), conductivities sigma[0..nlay] (0 the
// air, nlay the lower half-space), and per cell its layer and the local
// depths of its edges from the layer's top.
struct Model {
  int nz, nlay;
  double omega_mu0;
  const zc *sigma;
  const double *d;
  const int *lay;
  const double *ta, *tb;
};

// per-cell factors of one kind (k = 0: gamma = 1, k = 1: gamma = sigma)
struct Cell {
  zc theta, FI, FD, GI, GD, diagA, diagA4, diagA3, diagA6;
  zc thetad;  // F'(top) / F(bottom): the top cell's ratio differentiated at its top
  zc GId;     // d/dz of int_cell U(z, z*) dz* at the cell's top edge
  zc GDd;     // d/dz of U(z, bottom) - U(z, top) at the top edge (regular part)
};

// eta, L and the p, q coefficients of both kinds for every layer n in
// 0..nlay (p[k * (nlay + 1) + n]); arrays of nlay + 1 entries
__host__ __device__ inline void layer_fns(double lam, const Model &m, zc *eta, double *L, zc *p,
                                          zc *q) {
  const int nl = m.nlay, nlayers = nl + 1;
  for (int n = 0; n < nlayers; ++n) {
    zc e = zsqrt(Z(lam * lam) - Z(0.0, m.omega_mu0) * m.sigma[n]);
    if (e.x < 0) e = -e;
    eta[n] = e;
    L[n] = (n >= 1 && n < nl) ? m.d[n] - m.d[n - 1] : INFINITY;  // 0 and nl: half-spaces
  }
  for (int k = 0; k < 2; ++k) {
    zc *pk = p + k * nlayers, *qk = q + k * nlayers;
    for (int n = 0; n < nlayers; ++n) pk[n] = qk[n] = Z(0.0);
    auto g = [&](int n) { return k == 0 ? Z(1.0) : m.sigma[n]; };
    // downward: p_n from the admittance of everything above layer n
    for (int n = 1; n < nlayers; ++n) {
      const zc Pm = (n - 1 >= 1) ? pk[n - 1] * zexp(-2.0 * eta[n - 1] * L[n - 1]) : Z(0.0);
      const zc a = g(n - 1) * (1.0 + Pm) * eta[n], b = g(n) * eta[n - 1] * (1.0 - Pm);
      pk[n] = (a - b) / (a + b);
    }
    // upward: q_n from the admittance of everything below layer n
    for (int n = nlayers - 2; n >= 1; --n) {
      const zc Qp = (n + 1 < nl) ? qk[n + 1] * zexp(-2.0 * eta[n + 1] * L[n + 1]) : Z(0.0);
      const zc a = g(n + 1) * eta[n] * (1.0 + Qp), b = g(n) * eta[n + 1] * (1.0 - Qp);
      qk[n] = (a - b) / (a + b);
    }
  }
}

// factors of cell l, kind k, from the layer functions of layer_fns
__host__ __device__ inline void cell_factors(int l, int k, const Model &m, const zc *eta,
                                             const double *L, const zc *p, const zc *q,
                                             Cell &c) {
  const int nlayers = m.nlay + 1;
  const int n = m.lay[l];
  const zc e = eta[n];
  const double ta = m.ta[l], tb = m.tb[l], h = tb - ta;
  const zc P = p[k * nlayers + n], Q = q[k * nlayers + n];
  const bool half = !(L[n] < kFinite);
  const zc eh = zexp(-e * h);
  const zc x = e * h;
  const zc E1 = h * f_eps(x);
  const zc ea = zexp(-2.0 * e * ta), eb = zexp(-2.0 * e * tb);
  const zc fa = 1.0 + P * ea, fb = 1.0 + P * eb;
  const zc fta = 1.0 - P * ea;  // F'(t_a) / (eta e^{eta t_a})
  const zc qa = half ? Z(0.0) : Q * zexp(-2.0 * e * (L[n] - ta));
  const zc qb = half ? Z(0.0) : Q * zexp(-2.0 * e * (L[n] - tb));
  const zc ga = 1.0 + qa, gb = 1.0 + qb;
  const zc damp = half ? Z(0.0) : zexp(-2.0 * e * L[n]);
  const zc pqd = P * Q * damp;
  const zc D = 1.0 - pqd;
  c.theta = eh * fa / fb;
  c.thetad = e * eh * fta / fb;
  c.FI = E1 * (1.0 + P * zexp(-e * (ta + tb))) / fb;
  c.FD = 1.0 - c.theta;
  const zc qm = half ? Z(0.0) : Q * zexp(-e * (2.0 * L[n] - ta - tb));
  c.GI = fa * E1 * (1.0 + qm) / (e * D);
  c.GD = fa * (eh * gb - ga) / (e * D);
  c.GId = fta * E1 * (1.0 + qm) / D;
  c.GDd = fta * (eh * gb - ga) / D;
  // same cell
  const zc Sp = ea * E1 * E1;
  const zc Sq = half ? Z(0.0) : zexp(-2.0 * e * (L[n] - tb)) * E1 * E1;
  const zc psi = half ? Z(0.0) : f_psi_damped(x, damp, zexp(x - 2.0 * e * L[n]));
  const zc phix = f_phi(x);
  c.diagA = (2.0 * h * h * phix + P * Sp + Q * Sq + P * Q * 2.0 * h * h * psi) / (e * D);
  c.diagA4 = E1 * E1 * (qb - P * ea) / D;
  {
    // U(b,b) + U(a,a) - 2 U(a,b) - 2h, with the free part written stably:
    // (2/(eta D))(1 - e^{-x}) - 2h = 2h (pqd - x phi(x)) / D
    const zc em = zexp(-e * ta) - zexp(-e * tb);
    const zc qq = half ? Z(0.0) : zexp(-e * (L[n] - tb)) - zexp(-e * (L[n] - ta));
    const zc pq_term =
        half ? Z(0.0) : -2.0 * P * Q * f_expm1_damped(x, damp, zexp(x - 2.0 * e * L[n]));
    c.diagA3 = 2.0 * h * (pqd - x * phix) / D + (P * em * em + Q * qq * qq + pq_term) / (e * D);
  }
  {
    // lambda^2 A2 - 2h = eta^2 A2 - 2h + k^2 A2 (stable for large lambda)
    const zc ep = f_eps(x);
    const zc kk2 = Z(0.0, m.omega_mu0) * m.sigma[n];
    const zc eta2A2m2h =
        (2.0 * h * (pqd - ep) + e * (P * Sp + Q * Sq + P * Q * 2.0 * h * h * psi)) / D;
    c.diagA6 = eta2A2m2h + kk2 * c.diagA;
  }
}

// Row i of the lambda functions of the coefficient tables: for every pair
// i <= j the upper-triangle entries P / lambda, lambda A1, lambda A6 / sigma_i
// (columns u, T + u, 2T + u of out, u the pair's row-major index), and
// lambda A4 / sigma_obs for (i, j) and (j, i) (column 3T + obs nz + src);
// c0, c1: the cells' factors of kind 0 and 1.
__host__ __device__ inline void table_row(int i, double lam, const Model &m, const Cell *c0,
                                          const Cell *c1, zc *out) {
  const int nz = m.nz, T = nz * (nz + 1) / 2;
  const zc iwm = Z(0.0, m.omega_mu0);
  const double lam2 = lam * lam;
  const zc si = m.sigma[m.lay[i]];
  zc R1 = Z(1.0), Rs = Z(1.0);  // products of theta over cells strictly between
  int u = i * nz - (i * (i - 1)) / 2;
  for (int j = i; j < nz; ++j, ++u) {
    zc A1, A2, A3;
    if (j == i) {
      A1 = c0[i].diagA;
      A2 = c1[i].diagA;
      A3 = c1[i].diagA3;
    } else {
      if (j > i + 1) {
        R1 = R1 * c0[j - 1].theta;
        Rs = Rs * c1[j - 1].theta;
      }
      A1 = c0[i].FI * R1 * c0[j].GI;
      A2 = c1[i].FI * Rs * c1[j].GI;
      A3 = c1[i].FD * Rs * c1[j].GD;
    }
    const zc Pv = (-iwm) * A1 + A3 / si;
    out[u] = Pv / lam;
    out[T + u] = lam * A1;
    const zc A6 = (j == i) ? c1[i].diagA6 : lam2 * A2;
    out[2 * T + u] = lam * A6 / si;
  }
  // A4 / sigma_obs, full [iz][jz]
  zc *A4 = out + 3 * T;
  A4[i * nz + i] = lam * c1[i].diagA4 / si;
  zc R = Z(1.0);
  for (int j = i + 1; j < nz; ++j) {
    if (j > i + 1) R = R * c1[j - 1].theta;
    // observation i above source j
    A4[i * nz + j] = lam * c1[i].FD * R * c1[j].GI / si;
    // observation j below source i: (sigma_j / sigma_i) FI_i R GD_j / sigma_j
    A4[j * nz + i] = lam * c1[i].FI * R * c1[j].GD / si;
  }
}

// A point observer at depth z0 in the earth (receiver kernels), at or above
// the top of the grid, or below its bottom: the layer holding it, and the
// gap between it and the grid split at interfaces into pieces (layer, local
// top, local bottom), empty when z0 is the top of the grid; a6 the
// large-lambda limit of lambda^2 A2 - 2 for the observer on its own cell's
// top face.
struct Observer {
  double z0;
  int lay_obs, ngap;
  bool below;
  const int *gap_lay;
  const double *gap_ta, *gap_tb;
  zc a6;
};

// The eight lambda functions of every source level jz for a point observer,
// out[f nz + jz]:
//   0 lambda A1, 1 lambda A2, 2 lambda dA1, 3 lambda A4 / s, 4 lambda A5 / s,
//   5 lambda A6 / s, 6 P / lambda, 7 Q / lambda   (s: the observer's layer)
// with A1 = int U_1, A2 = int U_s, dA1 = d/dz A1, A4 = d/dz A2,
// A5 = U_s(z, bottom) - U_s(z, top), A3 = d/dz A5 (regular part),
// A6 = lambda^2 A2 - 2 [observer in the cell], P = -i w mu0 A1 + A3 / s,
// Q = dA1 + A5.  Above the grid U(z0, z*) = F(z0) G(z*) / (eta D): each
// cell's functions at the top of the grid are carried up by F(z0) / F(top)
// (F'(z0) / F(top) for the derivatives), the product of the ratios
// F(a) / F(b) over the pieces of the gap and the cells above; the cell the
// observer touches uses the derivative at its own top edge.  Below the grid
// U(z0, z*) = F(z*) G(z0) / (eta D) in the observer's layer (times
// sigma_obs / sigma_source for the sigma kind: sigma_s U(z, z*) = sigma_r
// U(z*, z)), with the ratios F(bottom of the cell) / F(z0) over the cells
// below and the gap.  eta, L, p, q: from layer_fns; c0, c1: the cells'
// factors of both kinds.
__host__ __device__ inline void point_row(double lam, const Model &m, const Observer &ob,
                                          const zc *eta, const double *L, const zc *p,
                                          const zc *q, const Cell *c0, const Cell *c1, zc *out) {
  const int nz = m.nz, nlayers = m.nlay + 1;
  const Cell *cell[2] = {c0, c1};
  const zc iwm = Z(0.0, m.omega_mu0);
  const zc so = m.sigma[ob.lay_obs];
  if (ob.below) {
    const int n0 = ob.lay_obs;
    const double t0 = ob.z0 - m.d[n0 - 1];
    const bool half = !(L[n0] < kFinite);
    zc U0[2], U0d[2], Rb[2] = {Z(1.0), Z(1.0)};
    for (int k = 0; k < 2; ++k) {
      const zc e = eta[n0], P = p[k * nlayers + n0], Q = q[k * nlayers + n0];
      const zc fa0 = 1.0 + P * zexp(-2.0 * e * t0);
      const zc qq = half ? Z(0.0) : Q * zexp(-2.0 * e * (L[n0] - t0));
      const zc D = half ? Z(1.0) : 1.0 - P * Q * zexp(-2.0 * e * L[n0]);
      U0[k] = fa0 * (1.0 + qq) / (e * D);
      U0d[k] = -1.0 * (fa0 * (1.0 - qq) / D);
      for (int i = 0; i < ob.ngap; ++i) {
        const int n = ob.gap_lay[i];
        const zc en = eta[n], Pn = p[k * nlayers + n];
        const double a = ob.gap_ta[i], b = ob.gap_tb[i];
        Rb[k] = Rb[k] * (zexp(-en * (b - a)) * (1.0 + Pn * zexp(-2.0 * en * a)) /
                         (1.0 + Pn * zexp(-2.0 * en * b)));
      }
    }
    for (int jz = nz - 1; jz >= 0; --jz) {
      const zc ss = so / m.sigma[m.lay[jz]];  // sigma_obs / sigma_source
      const zc A1 = c0[jz].FI * Rb[0] * U0[0];
      const zc dA1 = c0[jz].FI * Rb[0] * U0d[0];
      const zc A2 = ss * c1[jz].FI * Rb[1] * U0[1];
      const zc A4 = ss * c1[jz].FI * Rb[1] * U0d[1];
      const zc A5 = ss * c1[jz].FD * Rb[1] * U0[1];
      const zc A3 = ss * c1[jz].FD * Rb[1] * U0d[1];
      const zc A6 = lam * lam * A2;
      out[0 * nz + jz] = lam * A1;
      out[1 * nz + jz] = lam * A2;
      out[2 * nz + jz] = lam * dA1;
      out[3 * nz + jz] = lam * A4 / so;
      out[4 * nz + jz] = lam * A5 / so;
      out[5 * nz + jz] = lam * A6 / so;
      out[6 * nz + jz] = ((-iwm) * A1 + A3 / so) / lam;
      out[7 * nz + jz] = (dA1 + A5) / lam;
      for (int k = 0; k < 2; ++k) Rb[k] = Rb[k] * cell[k][jz].theta;
    }
    return;
  }
  const bool gap = ob.ngap > 0;
  zc R[2] = {Z(1.0), Z(1.0)}, Rd[2] = {Z(0.0), Z(0.0)};
  if (gap) {
    for (int k = 0; k < 2; ++k) {
      for (int i = 0; i < ob.ngap; ++i) {
        const int n = ob.gap_lay[i];
        const zc e = eta[n], P = p[k * nlayers + n];
        const double a = ob.gap_ta[i], b = ob.gap_tb[i];
        const zc eh = zexp(-e * (b - a));
        const zc fa = 1.0 + P * zexp(-2.0 * e * a), fb = 1.0 + P * zexp(-2.0 * e * b);
        const zc th = eh * fa / fb;
        if (i == 0) Rd[k] = e * eh * (1.0 - P * zexp(-2.0 * e * a)) / fb;
        else Rd[k] = Rd[k] * th;
        R[k] = R[k] * th;
      }
    }
  }
  for (int jz = 0; jz < nz; ++jz) {
    zc A1, A2, dA1, A4, A5, A3;
    if (!gap && jz == 0) {
      A1 = c0[0].GI;
      A2 = c1[0].GI;
      dA1 = c0[0].GId;
      A4 = c1[0].GId;
      A5 = c1[0].GD;
      A3 = c1[0].GDd;
    } else {
      A1 = R[0] * c0[jz].GI;
      A2 = R[1] * c1[jz].GI;
      dA1 = Rd[0] * c0[jz].GI;
      A4 = Rd[1] * c1[jz].GI;
      A5 = R[1] * c1[jz].GD;
      A3 = Rd[1] * c1[jz].GD;
    }
    // the observer's own cell: A6 tends to the constant a6, whose transform
    // is a delta at the observer; it is taken out here and added exactly to
    // the own cell's G_zz
    const zc A6 = lam * lam * A2 - ((jz == 0 && !gap) ? 2.0 + ob.a6 : Z(0.0));
    out[0 * nz + jz] = lam * A1;
    out[1 * nz + jz] = lam * A2;
    out[2 * nz + jz] = lam * dA1;
    out[3 * nz + jz] = lam * A4 / so;
    out[4 * nz + jz] = lam * A5 / so;
    out[5 * nz + jz] = lam * A6 / so;
    out[6 * nz + jz] = ((-iwm) * A1 + A3 / so) / lam;
    out[7 * nz + jz] = (dA1 + A5) / lam;
    // ratios from the observer to the top of the next cell
    for (int k = 0; k < 2; ++k) {
      Rd[k] = (jz == 0 && !gap) ? cell[k][0].thetad : Rd[k] * cell[k][jz].theta;
      R[k] = R[k] * cell[k][jz].theta;
    }
  }
}

}  // namespace vert
}  // namespace giem
