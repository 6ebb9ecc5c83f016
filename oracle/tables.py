"""Galerkin coefficients B_n^m of a layered medium for every signed lateral
offset (Sect. 3.1, eq. for B_n^m as a double volume integral of G^E; Appendix
A for G^E, Appendix B for the fundamental functions).

Derivation used (from the tensor of Appendix A, written in the horizontal
wavenumber k = lambda (cos t, sin t), with A1..A6 of oracle.vertical and
sigma_n the background conductivity of the observation cell):
  F_xx = [i w mu0 A1 + (kx^2/lambda^2) P] / 4pi,     P = -i w mu0 A1 + A3/sigma_n
  F_yy = [i w mu0 A1 + (ky^2/lambda^2) P] / 4pi,     F_xy = F_yx = (kx ky/lambda^2) P / 4pi
  F_xz = (i kx) A4 / (4pi sigma_n),                  F_yz = (i ky) A4 / (4pi sigma_n)
  F_zx = -(i kx) A5 / (4pi sigma_n),                 F_zy = -(i ky) A5 / (4pi sigma_n)
  F_zz = A6 / (4pi sigma_n)
and B(Delta) = (1/2pi) int e^{i k.Delta} |box(k)|^2 F(k) d^2k.  With
phi = the autocorrelation of the cell's footprint (a product of triangles) and
h[f](rho) = int_0^inf J0(lambda rho) f(lambda) lambda dlambda, each term is a
convolution in the plane:
  |box|^2 G(lambda)          -> (phi * h[G])(Delta)
  (i kx)|box|^2 G            -> (d_x phi * h[G])
  kx^2/lambda^2 |box|^2 G    -> (-d_xx phi * h[G/lambda^2])       (and xy, yy)
The derivatives of phi are piecewise polynomials (d_xx phi is a line
measure), so every coefficient is a low-dimensional weighted integral of a
radial function with an integrable singularity at rho = 0; the quadratures
below put Duffy-type nodes on the singular vertices.

None of Lemma 1 or Lemma 2 is used: every component and every signed offset
is computed on its own, so the lemmas can be tested on the result.
"""
from __future__ import annotations

import functools

import numpy as np

from . import hankel, vertical
from .fundamental import MU0

# weight kinds
W0, WX, WY, WXY, WXX, WYY = range(6)


@functools.lru_cache(maxsize=None)
def _gl(n):
    return np.polynomial.legendre.leggauss(n)


def _weight(kind, u, v, hx, hy):
    au, av = np.abs(u), np.abs(v)
    su, sv = np.sign(u), np.sign(v)
    if kind == W0:
        return (hx - au) * (hy - av)
    if kind == WX:
        return -su * (hy - av)
    if kind == WY:
        return -sv * (hx - au)
    if kind == WXY:
        return -su * sv
    raise ValueError(kind)


def _duffy_rect(x0, x1, y0, y1, px, py, n):
    """Nodes/weights on [x0,x1]x[y0,y1] for an integrand singular at the
    vertex (px, py): two triangles from that vertex, radial variable graded
    quadratically."""
    xs, ws = _gl(n)
    s = 0.5 * (xs + 1.0)
    wsn = 0.5 * ws
    # graded radial coordinate r = s^2
    r = s ** 2
    wr = wsn * 2 * s
    t, wt = s, wsn
    P = np.array([px, py])
    corners = [np.array([x0, y0]), np.array([x1, y0]), np.array([x1, y1]), np.array([x0, y1])]
    others = [c for c in corners if not (c[0] == px and c[1] == py)]
    # the opposite corner is the one differing in both coordinates
    opp = [c for c in others if c[0] != px and c[1] != py][0]
    adj = [c for c in others if not (c[0] == opp[0] and c[1] == opp[1])]
    pts, wts = [], []
    for A in adj:
        e1 = A - P
        e2 = opp - A
        det = abs(e1[0] * e2[1] - e1[1] * e2[0])
        R, T = np.meshgrid(r, t, indexing="ij")
        WR, WT = np.meshgrid(wr, wt, indexing="ij")
        X = P[0] + R * (e1[0] + T * e2[0])
        Y = P[1] + R * (e1[1] + T * e2[1])
        pts.append(np.stack([X.ravel(), Y.ravel()], 1))
        wts.append((WR * WT * R * det).ravel())
    return np.concatenate(pts), np.concatenate(wts)


def _tensor_rect(x0, x1, y0, y1, n, split=1):
    xs, ws = _gl(n)
    out_p, out_w = [], []
    ex = np.linspace(x0, x1, split + 1)
    ey = np.linspace(y0, y1, split + 1)
    for a, b in zip(ex[:-1], ex[1:]):
        for c, d in zip(ey[:-1], ey[1:]):
            X = 0.5 * (a + b) + 0.5 * (b - a) * xs
            Y = 0.5 * (c + d) + 0.5 * (d - c) * xs
            WX_ = 0.5 * (b - a) * ws
            WY_ = 0.5 * (d - c) * ws
            XX, YY = np.meshgrid(X, Y, indexing="ij")
            WW = np.outer(WX_, WY_)
            out_p.append(np.stack([XX.ravel(), YY.ravel()], 1))
            out_w.append(WW.ravel())
    return np.concatenate(out_p), np.concatenate(out_w)


def area_rule(kind, dx, dy, hx, hy, n_sing=24, n_reg=14):
    """Points rho' and weights w so that sum w h(|Delta - rho'|) approximates
    int W_kind(rho') h(|Delta - rho'|) d^2 rho' for the offset Delta=(dx,dy)."""
    pts, wts = [], []
    for sx in (-1, 1):
        for sy in (-1, 1):
            x0, x1 = sorted((0.0, sx * hx))
            y0, y1 = sorted((0.0, sy * hy))
            vx = [x0, x1]
            vy = [y0, y1]
            sing = None
            for cx in vx:
                for cy in vy:
                    if np.isclose(cx, dx, atol=1e-9 * hx) and np.isclose(cy, dy, atol=1e-9 * hy):
                        sing = (cx, cy)
            if sing is not None:
                p, w = _duffy_rect(x0, x1, y0, y1, sing[0], sing[1], n_sing)
            else:
                dist = np.hypot(max(x0 - dx, 0, dx - x1), max(y0 - dy, 0, dy - y1))
                split = 2 if dist < 0.5 * min(hx, hy) else 1
                p, w = _tensor_rect(x0, x1, y0, y1, n_reg, split)
            # evaluate the weight strictly inside the quadrant (sign of 0)
            wk = _weight(kind, np.where(p[:, 0] == 0, sx * 1e-300, p[:, 0]),
                         np.where(p[:, 1] == 0, sy * 1e-300, p[:, 1]), hx, hy)
            pts.append(p)
            wts.append(w * wk)
    P = np.concatenate(pts)
    W = np.concatenate(wts)
    rho = np.hypot(dx - P[:, 0], dy - P[:, 1])
    return rho, W


def _graded_toward(a, b, n, ratio=0.15, depth=1e-13):
    """Gauss-Legendre nodes and weights on [a, b] (either order) for an
    integrand with a logarithmic singularity at a: pieces whose lengths shrink
    geometrically toward a (ratio per piece) down to depth * |b - a|, n
    points each, and a last piece with a quadratically graded rule."""
    xs, ws = _gl(n)
    L = b - a
    t_hi = 1.0
    nodes, wts = [], []
    while t_hi > depth:
        t_lo = t_hi * ratio
        nodes.append(a + L * (0.5 * (t_lo + t_hi) + 0.5 * (t_hi - t_lo) * xs))
        wts.append(0.5 * (t_hi - t_lo) * abs(L) * ws)
        t_hi = t_lo
    s = 0.5 * (xs + 1.0)
    nodes.append(a + L * t_hi * s ** 2)
    wts.append(abs(L) * t_hi * 0.5 * ws * 2 * s)
    return np.concatenate(nodes), np.concatenate(wts)


def line_rule(kind, dx, dy, hx, hy, n=16):
    """Rule for -d_xx phi (kind WXX) or -d_yy phi (kind WYY): the measure
    -(delta(u + h) - 2 delta(u) + delta(u - h)) times the triangle in the
    other direction.  On the line through the singular point (rho = 0, where
    the radial function has a logarithmic singularity) the pieces next to it
    are graded geometrically."""
    xs, ws = _gl(n)
    rhos, wts = [], []
    for c, wc in ((-1, -1.0), (0, 2.0), (1, -1.0)):
        if kind == WXX:
            a_fix, d_fix, d_run, h_fix, h_run = c * hx, dx, dy, hx, hy
        else:
            a_fix, d_fix, d_run, h_fix, h_run = c * hy, dy, dx, hy, hx
        off = d_fix - a_fix                       # fixed-coordinate separation
        cuts = sorted(set([-h_run, 0.0, h_run] + ([d_run] if -h_run < d_run < h_run else [])))
        for a, b in zip(cuts[:-1], cuts[1:]):
            singular_a = abs(off) < 1e-12 * h_fix and abs(a - d_run) < 1e-12 * h_run
            singular_b = abs(off) < 1e-12 * h_fix and abs(b - d_run) < 1e-12 * h_run
            if singular_a:
                v, wv = _graded_toward(a, b, n)
            elif singular_b:
                v, wv = _graded_toward(b, a, n)
            else:
                v = 0.5 * (a + b) + 0.5 * (b - a) * xs
                wv = 0.5 * (b - a) * ws
            tri = h_run - np.abs(v)
            rhos.append(np.hypot(off, d_run - v))
            wts.append(wc * wv * tri)
    return np.concatenate(rhos), np.concatenate(wts)


QUAD = dict(lam_width=0.5, lam_n=16, rho_width=0.5, rho_n=12, rho_min_rel=1e-13,
            lam_asym_rel=40.0, ntail=30, n_gl=16, n_gl0=12, levels=14,
            n_sing=32, n_reg=20, n_line=16)


def build_tables(model, freq=None, quad=None):
    """B for every signed offset: array [2Ny-1][2Nx-1][3][3][Nz][Nz] with
    index [i + Ny - 1, j + Nx - 1] for y-offset i and x-offset j.  quad
    overrides entries of QUAD (panel widths and orders of every quadrature,
    for convergence checks)."""
    q = dict(QUAD, **(quad or {}))
    f = model["freq"] if freq is None else freq
    nx, ny, nz = model["nx"], model["ny"], model["nz"]
    hx, hy = model["hx"], model["hy"]
    ze = np.asarray(model["z_edges"], float)
    d, sig = model["d"], model["sigma"]
    hmin = float(np.min(np.diff(ze)))
    href = min(hx, hy)
    rho_min = q["rho_min_rel"] * href
    rho_max = 1.05 * np.hypot((nx + 1) * hx, (ny + 1) * hy)
    lam_asym = q["lam_asym_rel"] / hmin
    lam_lo = 1e-9 / max(rho_max, ze[-1])
    lam_a = 1e-3 / max(rho_max, ze[-1])
    ntail = q["ntail"]
    lam_hi = 1.1 * (lam_asym + (ntail + 3) * np.pi / rho_min)
    lp = hankel.LogPanels(lam_lo * 0.5, lam_hi, q["lam_width"], q["lam_n"])
    K = vertical.kernel_functions(lp.x, d, sig, f, ze)          # [nl, 5, nz, nz]
    lam = lp.x[:, None, None, None]
    G = (K * lam).reshape(lp.size, -1)                          # g = f(lambda) lambda
    reg = np.zeros((5, nz, nz), bool)
    reg[1] = True
    reg = reg.reshape(-1)
    rp = hankel.LogPanels(rho_min, rho_max, q["rho_width"], q["rho_n"])
    H = hankel.hankel_on_grid(G, lp, rp.x, reg, lam_a, lam_lo, lam_asym, ntail,
                              n_gl=q["n_gl"], n_gl0=q["n_gl0"], levels=q["levels"])  # [nrho, F]
    # weighted quadratures, folded onto the radial grid
    offs = [(i, j) for i in range(-ny + 1, ny) for j in range(-nx + 1, nx)]
    rows = []
    for (i, j) in offs:
        dx, dy = j * hx, i * hy
        for kind in (W0, WX, WY, WXY):
            rho, w = area_rule(kind, dx, dy, hx, hy, q["n_sing"], q["n_reg"])
            rows.append((rho, w))
        for kind in (WXX, WYY):
            rho, w = line_rule(kind, dx, dy, hx, hy, q["n_line"])
            rows.append((rho, w))
    M = np.zeros((len(rows), rp.size))
    for r, (rho, w) in enumerate(rows):
        cols, iw = rp.interp_rows(np.maximum(rho, rho_min))
        np.add.at(M[r], cols.ravel(), (w[:, None] * iw).ravel())
    Vals = (M @ H).reshape(len(offs), 6, 5, nz, nz)            # [off, weight, func, iz, jz]
    iwm = 1j * 2 * np.pi * f * MU0
    c = 1.0 / (4 * np.pi)
    B = np.zeros((len(offs), 3, 3, nz, nz), dtype=np.complex128)
    B[:, 0, 0] = c * (iwm * Vals[:, W0, 0] + Vals[:, WXX, 1])
    B[:, 1, 1] = c * (iwm * Vals[:, W0, 0] + Vals[:, WYY, 1])
    B[:, 0, 1] = c * Vals[:, WXY, 1]
    B[:, 1, 0] = c * Vals[:, WXY, 1]
    B[:, 0, 2] = c * Vals[:, WX, 2]
    B[:, 1, 2] = c * Vals[:, WY, 2]
    B[:, 2, 0] = -c * Vals[:, WX, 3]
    B[:, 2, 1] = -c * Vals[:, WY, 3]
    B[:, 2, 2] = c * Vals[:, W0, 4]
    return B.reshape(2 * ny - 1, 2 * nx - 1, 3, 3, nz, nz)


def pack(Bfull, nx, ny, nz):
    """Packed spatial table [Ny][Nx][E] (storage of Sect. 3.1) taken from the
    non-negative offsets: upper triangles of xx, xy, yy, zz, full xz, yz."""
    from .packed import pack_classes
    q = Bfull[ny - 1:, nx - 1:]
    blocks = {"xx": q[:, :, 0, 0], "xy": q[:, :, 0, 1], "yy": q[:, :, 1, 1], "zz": q[:, :, 2, 2],
              "xz": q[:, :, 0, 2], "yz": q[:, :, 1, 2]}
    return pack_classes(blocks, nz)
