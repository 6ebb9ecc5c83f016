"""Vertical integrals of the fundamental functions for every cell pair
(Appendix A, the integrals V1..V5 of the coefficients B_n^m).

For an observation cell [a, b] (index iz, conductivity sigma_n) and a source
cell [c, e] (index jz), on an array of lambda values:
  A1 = int_a^b int_c^e U_1 dz* dz
  A2 = int_a^b int_c^e U_sigma dz* dz
  A3 = int int (d/dz d/dz* U_sigma - 2 delta(z - z*)) dz* dz     (regular part)
     = U(b,e) - U(a,e) - U(b,c) + U(a,c) - 2 |[a,b] n [c,e]|
  A4 = int int d/dz U_sigma       = Psi(b) - Psi(a), Psi = int_c^e U_sigma dz*
  A5 = int int d/dz* U_sigma      = int_a^b (U(z, e) - U(z, c)) dz
  A6 = int int (lambda^2 U_sigma - 2 delta(z - z*)) = lambda^2 A2 - 2 |overlap|
The paper writes the integral behind V3 with the z-derivative outside the
z*-integral, which keeps the 2 delta of d/dz d/dz* U; the tangential terms of
the tensor need the regular part A3 (the delta terms of the two contributions
cancel in G1 + dg/dz), which is what the whole-space closed form confirms.
Source points on a cell edge belong to the layer of that cell.

Everything comes from oracle.fundamental (boundary-value problems), never
from the recursions of Appendix B.
"""
from __future__ import annotations

import numpy as np

from .fundamental import Profile, _layer_at


def cell_layers(d, z_edges):
    return np.array([_layer_at(np.asarray(d, float), 0.5 * (z_edges[k] + z_edges[k + 1]))
                     for k in range(len(z_edges) - 1)])


def vertical_functions(lam, d, sigma, freq, z_edges):
    """Arrays A1..A6 with shape [nlam, nz, nz] (observation iz, source jz)."""
    lam = np.asarray(lam, dtype=np.float64)
    ze = np.asarray(z_edges, dtype=np.float64)
    nz = ze.size - 1
    lays = cell_layers(d, ze)
    nl = lam.size
    A = {k: np.zeros((nl, nz, nz), dtype=np.complex128) for k in ("A1", "A2", "A3", "A4", "A5")}
    for jz in range(nz):
        c, e = ze[jz], ze[jz + 1]
        p1 = Profile(lam, d, sigma, freq, "1", ("box", c, e))
        ps = Profile(lam, d, sigma, freq, "sigma", ("box", c, e))
        pc = Profile(lam, d, sigma, freq, "sigma", ("point", c, lays[jz]))
        pe = Profile(lam, d, sigma, freq, "sigma", ("point", e, lays[jz]))
        for iz in range(nz):
            a, b = ze[iz], ze[iz + 1]
            ov = (b - a) if iz == jz else 0.0
            A["A1"][:, iz, jz] = p1.integral(a, b)
            A["A2"][:, iz, jz] = ps.integral(a, b)
            A["A4"][:, iz, jz] = ps.value(b) - ps.value(a)
            A["A3"][:, iz, jz] = (pe.value(b) - pe.value(a) - pc.value(b) + pc.value(a)) - 2.0 * ov
            A["A5"][:, iz, jz] = pe.integral(a, b) - pc.integral(a, b)
    ov = np.diag(np.diff(ze))
    A["A6"] = lam[:, None, None] ** 2 * A["A2"] - 2.0 * ov[None]
    return A


def kernel_functions(lam, d, sigma, freq, z_edges):
    """The five lambda-functions whose Hankel transforms build the table,
    stacked as [nlam, 5, nz, nz]:
      0: A1                     (with lambda dlambda)
      1: P / lambda^2, P = -i w mu0 A1 + A3 / sigma_n   (regularised at 0)
      2: A4 / sigma_n,  3: A5 / sigma_n,  4: A6 / sigma_n   (with lambda dlambda)
    sigma_n is the background conductivity of the observation cell."""
    from .fundamental import MU0
    A = vertical_functions(lam, d, sigma, freq, z_edges)
    ze = np.asarray(z_edges, float)
    sn = np.asarray(sigma, np.complex128)[cell_layers(d, ze)][None, :, None]
    w = 2 * np.pi * freq
    lam = np.asarray(lam, float)[:, None, None]
    P = -1j * w * MU0 * A["A1"] + A["A3"] / sn
    return np.stack([A["A1"], P / lam ** 2, A["A4"] / sn, A["A5"] / sn, A["A6"] / sn], axis=1)
