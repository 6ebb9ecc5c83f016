"""Electric and magnetic fields at receivers from the cell fields, and the
right-hand side of dipole sources
(Sect. 2.2, the representation of the anomalous fields through G^E and G^H
integrated over the cells; Appendix A for the tensors).  Test infrastructure.

  e(r) = E^N(r) + sum_n (sa_n - sb_n) [int_{cell n} G^E(r, M0) dM0] E_n
  h(r) = H^N(r) + sum_n (sa_n - sb_n) [int_{cell n} G^H(r, M0) dM0] E_n

The receiver sits at depth z0 (0 by default) on the earth side; horizontal E
and all of H are continuous across the surface, E_z is the earth-side value.
For a point observer the horizontal Galerkin weight becomes the source
footprint (a box) instead of the autocorrelation of two boxes.

Derivation (horizontal wavenumber k, lambda = |k|, vertical functions of the
observation depth z for a source cell [c, e] with sigma the conductivity at
z, P = -i w mu0 A1 + A3 / sigma, Q = dA1 + A5):
  A1 = int_c^e U_1(z, z*) dz*        dA1 = d/dz A1
  A2 = int_c^e U_s(z, z*) dz*        A4  = d/dz A2
  A5 = U_s(z, e) - U_s(z, c)         A3  = d/dz A5 - 2 [c <= z < e]
  A6 = lambda^2 A2 - 2 [c <= z < e]  (regular parts; see oracle.vertical)
  4pi G^E: xx = i w mu0 A1 + (kx^2/lambda^2) P,  xy = (kx ky/lambda^2) P,
           xz = i kx A4 / sigma,  zx = -i kx A5 / sigma,  zz = A6 / sigma
  G^H = curl_r G^E / (i w mu0) (derivatives on the observation point):
  4pi G^H: xx = (kx ky/lambda^2) Q,   yx = dA1 - (kx^2/lambda^2) Q,
           zx = -i ky A1,             xy = (ky^2/lambda^2) Q - dA1,
           yy = -(kx ky/lambda^2) Q,  zy = i kx A1,
           xz = i ky A2,              yz = -i kx A2,   zz = 0
(the P terms cancel in G^H, using d/dz A3 = eta^2 A5 and k^2 = i w mu0 s).
In the plane: box * h for the plain terms, (d_x box) * h for i kx, and
(d_x box) * (-d_x h) = (d_x box) * (h1 x/rho) for kx^2/lambda^2 (h1 the
order-one transform of f lambda^2, so that -dh/drho = h1), likewise for
ky^2 and kx ky; d_x box is a pair of line measures on the faces x = -+hx/2.
"""
from __future__ import annotations

import numpy as np

from . import hankel
from .fundamental import MU0, Profile, _layer_at
from .normal_field import LayeredPlaneWave
from .tables import _duffy_rect, _gl, _tensor_rect
from .vertical import cell_layers


def point_vertical(lam, d, sigma, freq, z_edges, z0=0.0):
    """Vertical functions of a point observer at z0 (right side) for every
    source level; arrays [nlam, nz] in a dict."""
    lam = np.asarray(lam, float)
    ze = np.asarray(z_edges, float)
    nz = ze.size - 1
    lays = cell_layers(d, ze)
    w = 2 * np.pi * freq
    s_obs = np.asarray(sigma, complex)[_layer_at(np.asarray(d, float), z0 + 1e-9)]
    out = {k: np.zeros((lam.size, nz), complex) for k in ("A1", "dA1", "A2", "A4", "A5", "A3", "A6")}
    for jz in range(nz):
        c, e = ze[jz], ze[jz + 1]
        p1 = Profile(lam, d, sigma, freq, "1", ("box", c, e))
        ps = Profile(lam, d, sigma, freq, "sigma", ("box", c, e))
        pc = Profile(lam, d, sigma, freq, "sigma", ("point", c, lays[jz]))
        pe = Profile(lam, d, sigma, freq, "sigma", ("point", e, lays[jz]))
        inside = 2.0 if (c <= z0 < e) else 0.0
        out["A1"][:, jz] = p1.value(z0)
        out["dA1"][:, jz] = p1.deriv(z0, +1)
        out["A2"][:, jz] = ps.value(z0)
        out["A4"][:, jz] = ps.deriv(z0, +1)
        out["A5"][:, jz] = pe.value(z0) - pc.value(z0)
        out["A3"][:, jz] = pe.deriv(z0, +1) - pc.deriv(z0, +1) - inside
        out["A6"][:, jz] = lam ** 2 * out["A2"][:, jz] - inside
        if inside:
            # for the observer's own cell A6 tends to a constant (a delta in
            # the plane); its value from the boundary-value problem at a very
            # large lambda is taken out and added exactly (receiver_kernels)
            big = np.array([1e9 / (e - c)])
            pb = Profile(big, d, sigma, freq, "sigma", ("box", c, e))
            a6_inf = complex(big[0] ** 2 * pb.value(z0)[0] - inside)
            out["A6"][:, jz] -= a6_inf
            out["a6_inf"] = (jz, a6_inf)
    out["P"] = -1j * w * MU0 * out["A1"] + out["A3"] / s_obs
    out["Q"] = out["dA1"] + out["A5"]
    out["sigma_obs"] = s_obs
    return out


# ------------------------------------------------------------ plane rules
def _split_rect(x0, x1, y0, y1, px, py):
    xs = [x0] + ([px] if x0 < px < x1 else []) + [x1]
    ys = [y0] + ([py] if y0 < py < y1 else []) + [y1]
    return [(a, b, c, d) for a, b in zip(xs[:-1], xs[1:]) for c, d in zip(ys[:-1], ys[1:])]


def box_rule(dx, dy, hx, hy, n_sing=24, n_reg=16):
    """Points (rho) and weights for int_{|x|<hx/2,|y|<hy/2} h(|D - r'|) d^2r'."""
    rhos, wts = [], []
    for (a, b, c, d) in _split_rect(-hx / 2, hx / 2, -hy / 2, hy / 2, dx, dy):
        vert = [(vx, vy) for vx in (a, b) for vy in (c, d)
                if abs(vx - dx) < 1e-12 * hx and abs(vy - dy) < 1e-12 * hy]
        if vert:
            p, w = _duffy_rect(a, b, c, d, vert[0][0], vert[0][1], n_sing)
        else:
            dist = np.hypot(max(a - dx, 0, dx - b), max(c - dy, 0, dy - d))
            split = 3 if dist < 0.5 * min(hx, hy) else 1
            p, w = _tensor_rect(a, b, c, d, n_reg, split)
        rhos.append(np.hypot(dx - p[:, 0], dy - p[:, 1]))
        wts.append(w)
    return np.concatenate(rhos), np.concatenate(wts)


def _line_nodes(a, b, t0, n=24):
    """Gauss-Legendre on [a, b], split at t0 when it lies inside."""
    cuts = [a] + ([t0] if a < t0 < b else []) + [b]
    x, w = _gl(n)
    ts, ws = [], []
    for p, q in zip(cuts[:-1], cuts[1:]):
        ts.append(0.5 * (p + q) + 0.5 * (q - p) * x)
        ws.append(0.5 * (q - p) * w)
    return np.concatenate(ts), np.concatenate(ws)


def face_rule(kind, dx, dy, hx, hy):
    """(rho, weight, geometric factor) for the line measures of d_x box
    (kind 'x': faces x = -hx/2 with +1 and x = +hx/2 with -1, running in y) or
    d_y box (kind 'y').  The factor is (D_n - t_face) / rho for the normal
    direction n (used with h1 for kx^2, ky^2) and (D_t - t) / rho for the
    running direction (kx ky)."""
    out = []
    for s, f in ((+1.0, -0.5), (-1.0, 0.5)):
        if kind == "x":
            xe = f * hx
            t, w = _line_nodes(-hy / 2, hy / 2, dy)
            rho = np.hypot(dx - xe, dy - t)
            out.append((rho, s * w, (dx - xe) / rho, (dy - t) / rho))
        else:
            ye = f * hy
            t, w = _line_nodes(-hx / 2, hx / 2, dx)
            rho = np.hypot(dy - ye, dx - t)
            out.append((rho, s * w, (dy - ye) / rho, (dx - t) / rho))
    rho = np.concatenate([o[0] for o in out])
    w = np.concatenate([o[1] for o in out])
    fn = np.concatenate([o[2] for o in out])
    ft = np.concatenate([o[3] for o in out])
    return rho, w, fn, ft


def receiver_kernels(model, offsets, freq=None, z0=0.0, n_lam_panel=16, lam_asym_rel=40.0):
    """Cell-integrated G^E and G^H for receivers at lateral offsets D (from
    the source cell centre, array [noff, 2]) and every source level:
    KE, KH arrays [noff, nz, 3, 3] (row = field component at the receiver)."""
    f = model["freq"] if freq is None else freq
    w = 2 * np.pi * f
    hx, hy = model["hx"], model["hy"]
    ze = np.asarray(model["z_edges"], float)
    d, sig = model["d"], model["sigma"]
    nz = ze.size - 1
    offsets = np.atleast_2d(np.asarray(offsets, float))
    hmin = float(np.min(np.diff(ze)))
    # the radial functions of the receiver's own cell grow like 1 / rho; the
    # clamp below rho_min costs a relative ~rho_min / h
    rho_min = 1e-13 * min(hx, hy)
    rho_max = 1.05 * (np.max(np.hypot(np.abs(offsets[:, 0]) + hx, np.abs(offsets[:, 1]) + hy)))
    lam_asym = lam_asym_rel / hmin
    lam_lo = 1e-9 / max(rho_max, ze[-1])
    lam_a = 1e-3 / max(rho_max, ze[-1])
    ntail = 30
    lam_hi = 1.1 * (lam_asym + (ntail + 3) * np.pi / rho_min)
    lp = hankel.LogPanels(lam_lo * 0.5, lam_hi, 0.5, n_lam_panel)
    V = point_vertical(lp.x, d, sig, f, ze, z0)
    so = V["sigma_obs"]
    lam = lp.x[:, None]
    # order 0: f * lambda;  order 1: (f / lambda^2) * lambda^2 = f
    g0 = np.concatenate([V["A1"] * lam, V["A2"] * lam, V["dA1"] * lam, V["A4"] / so * lam,
                         V["A5"] / so * lam, V["A6"] / so * lam], axis=1)
    g1 = np.concatenate([V["P"], V["Q"]], axis=1)
    rp = hankel.LogPanels(rho_min, rho_max, 0.5, 12)
    reg0 = np.zeros(g0.shape[1], bool)
    H0 = hankel.hankel_on_grid(g0, lp, rp.x, reg0, lam_a, lam_lo, lam_asym, ntail, order=0)
    H1 = hankel.hankel_on_grid(g1, lp, rp.x, None, lam_a, lam_lo, lam_asym, ntail, order=1)
    H0 = H0.reshape(rp.size, 6, nz)
    H1 = H1.reshape(rp.size, 2, nz)

    def interp(rho, wt, Hgrid):
        cols, iw = rp.interp_rows(np.maximum(rho, rho_min))
        row = np.zeros(rp.size)
        np.add.at(row, cols.ravel(), (wt[:, None] * iw).ravel())
        return np.tensordot(row, Hgrid, axes=(0, 0))   # [func, nz]

    A1, A2, dA1, A4, A5, A6 = range(6)
    P, Q = range(2)
    c = 1.0 / (4 * np.pi)
    iwm = 1j * w * MU0
    KE = np.zeros((len(offsets), nz, 3, 3), complex)
    KH = np.zeros((len(offsets), nz, 3, 3), complex)
    for k, (dx, dy) in enumerate(offsets):
        rb, wb = box_rule(dx, dy, hx, hy)
        b0 = interp(rb, wb, H0)                               # box * h
        rx, wx, fnx, ftx = face_rule("x", dx, dy, hx, hy)
        ry, wy, fny, fty = face_rule("y", dx, dy, hx, hy)
        bx = interp(rx, wx, H0)                               # (d_x box) * h
        by = interp(ry, wy, H0)
        bxx = interp(rx, wx * fnx, H1)                        # kx^2 / lambda^2
        byy = interp(ry, wy * fny, H1)
        bxy = interp(rx, wx * ftx, H1)                        # kx ky / lambda^2
        KE[k, :, 0, 0] = c * (iwm * b0[A1] + bxx[P])
        KE[k, :, 1, 1] = c * (iwm * b0[A1] + byy[P])
        KE[k, :, 0, 1] = c * bxy[P]
        KE[k, :, 1, 0] = c * bxy[P]
        KE[k, :, 0, 2] = c * bx[A4]
        KE[k, :, 1, 2] = c * by[A4]
        KE[k, :, 2, 0] = -c * bx[A5]
        KE[k, :, 2, 1] = -c * by[A5]
        KE[k, :, 2, 2] = c * b0[A6]
        if "a6_inf" in V and abs(dx) < 0.5 * hx and abs(dy) < 0.5 * hy:
            jz0, a6 = V["a6_inf"]
            # the constant's transform 2 pi a6 / s delta, integrated over the
            # footprint that holds the receiver
            KE[k, jz0, 2, 2] += c * 2 * np.pi * a6 / so
        KH[k, :, 0, 0] = c * bxy[Q]
        KH[k, :, 1, 0] = c * (b0[dA1] - bxx[Q])
        KH[k, :, 2, 0] = -c * by[A1]
        KH[k, :, 0, 1] = c * (byy[Q] - b0[dA1])
        KH[k, :, 1, 1] = -c * bxy[Q]
        KH[k, :, 2, 1] = c * bx[A1]
        KH[k, :, 0, 2] = c * by[A2]
        KH[k, :, 1, 2] = -c * bx[A2]
    return KE, KH


def surface_normal_fields(model, freq=None):
    """E^N and H^N at z = 0 for the x and the y polarisation: arrays [2][3]."""
    f = model["freq"] if freq is None else freq
    pw = LayeredPlaneWave(model["d"], model["sigma"], f)
    hy = pw.H_surface()
    EN = np.array([[1, 0, 0], [0, 1, 0]], complex)
    HN = np.array([[0, hy, 0], [-hy, 0, 0]], complex)
    return EN, HN


def normal_fields_at(model, z0=0.0, freq=None):
    """E^N and H^N at depth z0 in the earth for the x and the y polarisation
    of the unit-surface-field plane wave: arrays [2][3].  Faraday's law
    (curl E = i w mu0 H) for a field E_x(z): H_y = dE_x/dz / (i w mu0); for
    E_y(z): H_x = -dE_y/dz / (i w mu0)."""
    f = model["freq"] if freq is None else freq
    if z0 == model["d"][0]:
        return surface_normal_fields(model, f)      # E = 1 there by definition
    pw = LayeredPlaneWave(model["d"], model["sigma"], f)
    e = pw.E(z0)
    hy = pw.dE(z0) / (1j * pw.omega * MU0)
    EN = np.array([[e, 0, 0], [0, e, 0]], complex)
    HN = np.array([[0, hy, 0], [-hy, 0, 0]], complex)
    return EN, HN


def dipole_source(model, src_xy, moments, freq=None, z0=0.0):
    """Right-hand side U0 = sqrt(Re sigma_b) <E^0>_n of the scaled system for
    electric dipoles of moments p_s [nsrc, 3] (A m) at points (x, y, z0)
    (Sect. 2.1: the external current J_ext = p delta(r - r_s); Sect. 2.2: the
    source enters only through the normal field E^0 averaged over each cell).
    The normal field of a dipole is E^0(r) = G^E(r, r_s) p; by reciprocity of
    the layered medium (Appendix A: G^E(r, r') = G^E(r', r)^T),
      int_{cell n} E^0 = [int_{cell n} G^E(r_s, r) dr]^T p = KE(r_s <- n)^T p,
    the receiver kernel of a receiver at the source point, transposed.
    Array [nsrc, 3, nz, ny, nx]."""
    nx, ny, nz = model["nx"], model["ny"], model["nz"]
    hx, hy = model["hx"], model["hy"]
    x0, y0 = model.get("x0", 0.0), model.get("y0", 0.0)
    ze = np.asarray(model["z_edges"], float)
    cx = x0 + (np.arange(nx) + 0.5) * hx
    cy = y0 + (np.arange(ny) + 0.5) * hy
    src_xy = np.atleast_2d(np.asarray(src_xy, float))
    moments = np.atleast_2d(np.asarray(moments, complex))
    offs = np.array([(xs - cxx, ys - cyy) for (xs, ys) in src_xy for cyy in cy for cxx in cx])
    KE, _ = receiver_kernels(model, offs, freq, z0)
    KE = KE.reshape(len(src_xy), ny, nx, nz, 3, 3)
    vol = hx * hy * np.diff(ze)                                    # [nz]
    sb = np.asarray(model["sigma"], complex)[model["layer_of_cell"]]
    e0 = np.einsum("syxzrc,sr->sczyx", KE, moments) / vol[None, None, :, None, None]
    return np.sqrt(sb.real)[None, None, :, None, None] * e0


def fields_at(model, E_cells, rec_xy, sigma_a=None, freq=None, z0=0.0, normal=True):
    """e, h at receivers (x, y, z0) [nrec, 2] for E_cells [R][3][Nz][Ny][Nx]
    (RHS 0 / 1 = x / y polarisation of the plane-wave source, whose normal
    fields at z0 are added when normal is set; else, or for further RHS, the
    anomalous fields only): [R][nrec][3]."""
    sa = model["sigma_a"] if sigma_a is None else sigma_a
    nx, ny, nz = model["nx"], model["ny"], model["nz"]
    hx, hy = model["hx"], model["hy"]
    x0, y0 = model.get("x0", 0.0), model.get("y0", 0.0)
    sb = model["sigma"][model["layer_of_cell"]]
    dsig = sa - sb[:, None, None]
    cur = E_cells * dsig[None, None]                        # [R][3][nz][ny][nx]
    cx = x0 + (np.arange(nx) + 0.5) * hx
    cy = y0 + (np.arange(ny) + 0.5) * hy
    rec_xy = np.atleast_2d(np.asarray(rec_xy, float))
    R = E_cells.shape[0]
    EN, HN = normal_fields_at(model, z0, freq)
    offs = np.array([(xr - cxx, yr - cyy) for (xr, yr) in rec_xy for cyy in cy for cxx in cx])
    KE, KH = receiver_kernels(model, offs, freq, z0)
    KE = KE.reshape(len(rec_xy), ny, nx, nz, 3, 3)
    KH = KH.reshape(len(rec_xy), ny, nx, nz, 3, 3)
    e = np.einsum("qyxzab,rbzyx->rqa", KE, cur)
    h = np.einsum("qyxzab,rbzyx->rqa", KH, cur)
    n = min(R, 2) if normal else 0
    e[:n] += EN[:n, None, :]
    h[:n] += HN[:n, None, :]
    return e, h


def impedance(e, h):
    """Z = [Ex Ey] [Hx Hy]^-1 at every receiver from the two polarisations
    (columns: RHS 0 and 1): array [nrec, 2, 2]."""
    Eh = np.stack([e[0, :, :2], e[1, :, :2]], axis=-1)     # [nrec, comp, pol]
    Hh = np.stack([h[0, :, :2], h[1, :, :2]], axis=-1)
    return Eh @ np.linalg.inv(Hh)
