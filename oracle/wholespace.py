"""Galerkin coefficients in a homogeneous whole space (Appendix A with the
same conductivity in every layer, the air included): the layered part of the
Green's tensor vanishes and

  G^E(r) = i w mu0 (I + grad grad / k^2) g(R),   g = exp(i k R) / (4 pi R),
  k^2 = i w mu0 sigma, Im k > 0 (time factor exp(-i w t)).

With g' = g (ik - 1/R) and g'' = g ((ik - 1/R)^2 + 1/R^2):
  d_a d_b g = rhat_a rhat_b g'' + (delta_ab - rhat_a rhat_b) g' / R.

B_ab(n, m) = int_{cell n} int_{cell m} G^E_ab(r - r') dr' dr is computed
here by tensor Gauss-Legendre over both cells, which is exact up to the
quadrature error when the cells are separated (the integrand is smooth);
pairs that touch or overlap are rejected.
"""
from __future__ import annotations

import numpy as np

MU0 = 4e-7 * np.pi


def wavenumber(sigma, freq):
    k = np.sqrt(1j * 2 * np.pi * freq * MU0 * complex(sigma))
    return k if k.imag > 0 else -k


def greens_e(r, sigma, freq):
    """G^E at separation vectors r [..., 3]; returns [..., 3, 3]."""
    w = 2 * np.pi * freq
    k = wavenumber(sigma, freq)
    R = np.linalg.norm(r, axis=-1)
    rh = r / R[..., None]
    g = np.exp(1j * k * R) / (4 * np.pi * R)
    g1 = g * (1j * k - 1.0 / R)
    g2 = g * ((1j * k - 1.0 / R) ** 2 + 1.0 / R ** 2)
    rr = rh[..., :, None] * rh[..., None, :]
    eye = np.eye(3)
    dd = rr * g2[..., None, None] + (eye - rr) * (g1 / R)[..., None, None]
    return 1j * w * MU0 * (eye * g[..., None, None] + dd / k ** 2)


def _box_nodes(lo, hi, q):
    x, w = np.polynomial.legendre.leggauss(q)
    axes, wts = [], []
    for a, b in zip(lo, hi):
        axes.append(0.5 * (a + b) + 0.5 * (b - a) * x)
        wts.append(0.5 * (b - a) * w)
    X, Y, Z = np.meshgrid(*axes, indexing="ij")
    W = np.einsum("i,j,k->ijk", *wts)
    return np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1), W.ravel()


def cell_pair(lo_n, hi_n, lo_m, hi_m, sigma, freq, q=8):
    """B(n, m) [3, 3] for separated boxes n (observation) and m (source)."""
    lo_n, hi_n, lo_m, hi_m = map(np.asarray, (lo_n, hi_n, lo_m, hi_m))
    gap = np.maximum(0.0, np.maximum(lo_m - hi_n, lo_n - hi_m))
    if not np.any(gap > 0):
        raise ValueError("cells touch or overlap: the tensor rule does not apply")
    pn, wn = _box_nodes(lo_n, hi_n, q)
    pm, wm = _box_nodes(lo_m, hi_m, q)
    out = np.zeros((3, 3), dtype=np.complex128)
    for i in range(0, pn.shape[0], 64):
        r = pn[i:i + 64, None, :] - pm[None, :, :]
        G = greens_e(r, sigma, freq)
        out += np.einsum("i,j,ijab->ab", wn[i:i + 64], wm, G)
    return out


def greens_h(r, sigma, freq):
    """G^H = curl_r G^E / (i w mu0) at separation vectors r [..., 3]:
    G^H_ab = eps_acb d_c g (the field of a unit current element)."""
    k = wavenumber(sigma, freq)
    R = np.linalg.norm(r, axis=-1)
    g1 = np.exp(1j * k * R) / (4 * np.pi * R) * (1j * k - 1.0 / R)   # dg/dR
    grad = r / R[..., None] * g1[..., None]                          # d_c g
    out = np.zeros(r.shape[:-1] + (3, 3), complex)
    gx, gy, gz = grad[..., 0], grad[..., 1], grad[..., 2]
    out[..., 0, 1] = -gz
    out[..., 0, 2] = gy
    out[..., 1, 0] = gz
    out[..., 1, 2] = -gx
    out[..., 2, 0] = -gy
    out[..., 2, 1] = gx
    return out


def point_box(p, lo, hi, sigma, freq, q=12):
    """int over the box [lo, hi] of G^E(p - r') and G^H(p - r') for a point p
    outside the box: tensor Gauss-Legendre, ([3, 3], [3, 3])."""
    lo, hi, p = map(np.asarray, (lo, hi, p))
    pm, wm = _box_nodes(lo, hi, q)
    r = p[None, :] - pm
    return (np.einsum("i,iab->ab", wm, greens_e(r, sigma, freq)),
            np.einsum("i,iab->ab", wm, greens_h(r, sigma, freq)))


# ---------------------------------------------------------------------------
# Any pair of cells, touching or coincident ones included (Appendix A with
# one conductivity everywhere).  With u = r - r' and T_d(u_d) the length of
# [lo_n, hi_n] n [lo_m + u_d, hi_m + u_d] along axis d,
#
#   int_n int_m f(r - r') dr' dr = int f(u) T_x(u_x) T_y(u_y) T_z(u_z) du,
#
# and the second derivatives of g are moved onto the two cell boundaries by
# the divergence theorem, once in r' and once in r (a distributional identity,
# so the point term of grad grad g at coincident points is included):
#
#   int_n int_m d_a d_b g(r - r') = - oint_dn oint_dm g(r - r') n_a n'_b dS' dS.
#
# Every remaining integrand is g itself, singular like 1/R.  The integration
# boxes are cut at the break points of the T_d and at u = 0, so the singular
# point can only sit at a corner; boxes with that corner are mapped to
# pyramids with their apex there (the radial Jacobian t^(d-1) removes the
# 1/R), and boxes near it are bisected until their distance from it is at
# least twice their largest side.  This is a different route from the spectral
# (lambda) construction of oracle.tables: nothing is shared but g.
# ---------------------------------------------------------------------------


def _overlap_len(u, lo_n, hi_n, lo_m, hi_m):
    return np.clip(np.minimum(hi_n, hi_m + u) - np.maximum(lo_n, lo_m + u), 0.0, None)


def _pyramid_rule(lens, signs, q):
    """Nodes u [M, d] and weights for the box with sides lens whose corner
    at the origin is singular (the box extends along signs[d] * axis d):
    one pyramid per far face, apex at the origin."""
    x, w = np.polynomial.legendre.leggauss(q)
    s = 0.5 * (x + 1.0)
    ws = 0.5 * w
    d = len(lens)
    lens = np.asarray(lens, float)
    pts, wts = [], []
    for p in range(d):
        grids = np.meshgrid(*([s] * d), indexing="ij")
        wgrid = np.ones_like(grids[0])
        for g_ in np.meshgrid(*([ws] * d), indexing="ij"):
            wgrid = wgrid * g_
        t = grids[0]
        v = np.empty(t.shape + (d,))
        k = 1
        for a in range(d):
            if a == p:
                v[..., a] = t * lens[a]
            else:
                v[..., a] = t * grids[k] * lens[a]
                k += 1
        jac = t ** (d - 1) * np.prod(lens)
        pts.append((v * np.asarray(signs, float)).reshape(-1, d))
        wts.append((wgrid * jac).reshape(-1))
    return np.concatenate(pts), np.concatenate(wts)


def _tensor_rule(lo, hi, q):
    x, w = np.polynomial.legendre.leggauss(q)
    axes = [0.5 * (a + b) + 0.5 * (b - a) * x for a, b in zip(lo, hi)]
    wax = [0.5 * (b - a) * w for a, b in zip(lo, hi)]
    P = np.stack([g.ravel() for g in np.meshgrid(*axes, indexing="ij")], 1)
    W = np.ones(P.shape[0])
    for g in np.meshgrid(*wax, indexing="ij"):
        W = W * g.ravel()
    return P, W


def _box_cells(lo, hi, c, q, depth=0):
    """Quadrature (nodes, weights) for int over the box [lo, hi] of a function
    singular like 1/R at u = 0 (R^2 = c^2 + |u|^2), 0 never inside."""
    lo = np.asarray(lo, float)
    hi = np.asarray(hi, float)
    at0 = [(a == 0.0 or b == 0.0) for a, b in zip(lo, hi)]
    if c == 0.0 and all(at0):
        lens = hi - lo
        signs = [1.0 if a == 0.0 else -1.0 for a in lo]
        return _pyramid_rule(lens, signs, q)
    dist2 = c * c
    for a, b in zip(lo, hi):
        if not (a <= 0.0 <= b):
            dist2 += min(abs(a), abs(b)) ** 2
    side = np.max(hi - lo)
    if dist2 < 4.0 * side * side and depth < 24:
        ax = int(np.argmax(hi - lo))
        mid = 0.5 * (lo[ax] + hi[ax])
        h1 = hi.copy()
        h1[ax] = mid
        l2 = lo.copy()
        l2[ax] = mid
        p1, w1 = _box_cells(lo, h1, c, q, depth + 1)
        p2, w2 = _box_cells(l2, hi, c, q, depth + 1)
        return np.concatenate([p1, p2]), np.concatenate([w1, w2])
    return _tensor_rule(lo, hi, q)


def _singular_integral(kfun, axes, c, q):
    """int over the product of axes of kfun(R) * prod_d weight_d(u_d), with
    R^2 = c^2 + |u|^2.  axes: list of (break points, weight function)."""
    cuts = []
    for brk, _ in axes:
        b = np.unique(np.asarray(brk, float))
        if b[0] < 0.0 < b[-1]:
            b = np.unique(np.concatenate([b, [0.0]]))
        cuts.append(b)
    total = 0.0 + 0.0j
    import itertools
    for idx in itertools.product(*[range(len(b) - 1) for b in cuts]):
        lo = [cuts[d][i] for d, i in enumerate(idx)]
        hi = [cuts[d][i + 1] for d, i in enumerate(idx)]
        P, W = _box_cells(lo, hi, c, q)
        wt = W.copy()
        for d, (_, wf) in enumerate(axes):
            wt = wt * wf(P[:, d])
        R = np.sqrt(c * c + np.sum(P * P, axis=1))
        total += np.sum(wt * kfun(R))
    return total


def _trap_axis(lo_n, hi_n, lo_m, hi_m):
    brk = [lo_n - hi_m, lo_n - lo_m, hi_n - hi_m, hi_n - lo_m]
    return (brk, lambda u: _overlap_len(u, lo_n, hi_n, lo_m, hi_m))


def _flat_axis(a, b):
    return ([a, b], lambda u: np.ones_like(u))


def cell_pair_any(lo_n, hi_n, lo_m, hi_m, sigma, freq, q=12):
    """B(n, m) [3, 3] = int_n int_m G^E(r - r') for any two boxes, returned
    with its parts (I0 = int int g, F[a, b] = oint oint g n_a n'_b):
    B = i w mu0 (delta_ab I0 - F_ab / k^2)."""
    lo_n, hi_n, lo_m, hi_m = (np.asarray(v, float) for v in (lo_n, hi_n, lo_m, hi_m))
    w = 2 * np.pi * freq
    k = wavenumber(sigma, freq)

    def gfun(R):
        return np.exp(1j * k * R) / (4 * np.pi * R)

    I0 = _singular_integral(gfun, [_trap_axis(lo_n[d], hi_n[d], lo_m[d], hi_m[d])
                                   for d in range(3)], 0.0, q)
    F = np.zeros((3, 3), complex)
    for a in range(3):
        for b in range(3):
            acc = 0.0 + 0.0j
            for sn, Xn in ((1.0, hi_n[a]), (-1.0, lo_n[a])):
                for sm, Xm in ((1.0, hi_m[b]), (-1.0, lo_m[b])):
                    if a == b:
                        oth = [d for d in range(3) if d != a]
                        axes = [_trap_axis(lo_n[d], hi_n[d], lo_m[d], hi_m[d]) for d in oth]
                        val = _singular_integral(gfun, axes, abs(Xn - Xm), q)
                    else:
                        cax = 3 - a - b
                        # u_a = Xn - r'_a, u_b = r_b - Xm, u_c by overlap
                        axes = [_flat_axis(Xn - hi_m[a], Xn - lo_m[a]),
                                _flat_axis(lo_n[b] - Xm, hi_n[b] - Xm),
                                _trap_axis(lo_n[cax], hi_n[cax], lo_m[cax], hi_m[cax])]
                        val = _singular_integral(gfun, axes, 0.0, q)
                    acc += sn * sm * val
            F[a, b] = acc
    B = 1j * w * MU0 * (np.eye(3) * I0 - F / k ** 2)
    return B, I0, F
