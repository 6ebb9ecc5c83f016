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
