"""Fundamental functions of the layered medium, Appendix B of the paper.

U_gamma(z, z*, lambda), gamma in {1, sigma}, is the decaying solution of
    U'' - eta_m^2 U = 0 in every layer (z != z*),  eta_m^2 = lambda^2 - k_m^2,
    [U] = 0 and [(1/gamma) U'] = 0 at every interface d_n,
    [U] = 0 and [U'] = -2 at the source z*.
The oracle does not use the paper's recursions for p, q and A: it writes the
solution as exponentials on each interval between breakpoints (interfaces
and source points) and solves the linear system of the jump conditions,
one small system per lambda.  A box source 1_[c,e](z*) integrated over z*
(Psi = int U dz*) solves Psi'' - eta^2 Psi = -2 on [c, e] and is solved the
same way with the particular solution 2/eta^2 inside the box.

The basis on a finite interval [zl, zr] is exp(-eta (z - zl)) and
exp(-eta (zr - z)), both bounded by one; the upper half-space uses
exp(-eta (B0 - z)) and the lower one exp(-eta (z - Blast)).
Conventions: d[0] = 0 is the surface, sigma[0] the air (0 allowed),
sigma[k] the layer below d[k-1]; Re eta > 0.
"""
from __future__ import annotations

import numpy as np

MU0 = 4e-7 * np.pi


def eta_of(lam, sigma, freq):
    """eta_m(lambda) = sqrt(lambda^2 - i omega mu0 sigma_m), Re eta > 0.
    Returns [nlam, nlayers]."""
    lam = np.asarray(lam, dtype=np.float64)[:, None]
    k2 = 1j * 2 * np.pi * freq * MU0 * np.asarray(sigma, dtype=np.complex128)[None, :]
    e = np.sqrt(lam ** 2 - k2)
    return np.where(e.real < 0, -e, e)


def _layer_at(d, z):
    return int(np.searchsorted(d, z, side="right"))


class Profile:
    """Solution of one boundary-value problem for an array of lambda values."""

    def __init__(self, lam, d, sigma, freq, kind, source):
        """kind: '1' or 'sigma'.  source: ('point', z0, layer) with the layer the
        source belongs to (matters only when z0 sits on an interface), or
        ('box', c, e) with c < e inside one layer."""
        self.lam = np.asarray(lam, dtype=np.float64)
        self.d = np.asarray(d, dtype=np.float64)
        self.sigma = np.asarray(sigma, dtype=np.complex128)
        self.kind = kind
        self.source = source
        eta_l = eta_of(self.lam, self.sigma, freq)          # [nl, nlay+1]
        pts = list(self.d)
        if source[0] == "point":
            pts.append(float(source[1]))
        else:
            pts += [float(source[1]), float(source[2])]
        self.B = np.array(sorted(set(pts)))
        nb = self.B.size
        # intervals 0..nb: (-inf,B0), (B0,B1), ..., (B_{nb-1}, inf)
        lay = []
        for k in range(nb + 1):
            if k == 0:
                mid = self.B[0] - 1.0
            elif k == nb:
                mid = self.B[-1] + 1.0
            else:
                mid = 0.5 * (self.B[k - 1] + self.B[k])
            lay.append(_layer_at(self.d, mid))
        self.layer = np.array(lay)
        self.eta = eta_l[:, self.layer]                      # [nl, nb+1]
        # particular solution 2/eta^2 on the box intervals
        self.part = np.zeros_like(self.eta)
        if source[0] == "box":
            c, e = source[1], source[2]
            for k in range(1, nb):
                if self.B[k - 1] >= c and self.B[k] <= e:
                    self.part[:, k] = 2.0 / self.eta[:, k] ** 2
        self._solve()

    # unknown indices
    def _nunk(self, k):
        return 1 if k == 0 or k == self.B.size else 2

    def _solve(self):
        nb = self.B.size
        offs = np.cumsum([0] + [self._nunk(k) for k in range(nb + 1)])
        nu = offs[-1]
        nl = self.lam.size
        M = np.zeros((nl, nu, nu), dtype=np.complex128)
        r = np.zeros((nl, nu), dtype=np.complex128)
        sig = self.sigma
        for k in range(nb):
            b = self.B[k]
            L, R = k, k + 1
            eL, eR = self.eta[:, L], self.eta[:, R]
            row_v, row_d = 2 * k, 2 * k + 1
            # left interval value / derivative at its right end
            oL = offs[L]
            if L == 0:
                M[:, row_v, oL] = 1.0
            else:
                w = self.B[L] - self.B[L - 1]
                ex = np.exp(-eL * w)
                M[:, row_v, oL] = ex
                M[:, row_v, oL + 1] = 1.0
            # interface factors
            is_iface = np.any(np.isclose(self.d, b, rtol=0, atol=0))
            layL, layR = self.layer[L], self.layer[R]
            if is_iface and self.kind == "sigma":
                aL, aR = sig[layR], sig[layL]
            else:
                aL, aR = 1.0, 1.0
            if L == 0:
                M[:, row_d, oL] = aL * eL
            else:
                M[:, row_d, oL] = aL * (-eL * ex)
                M[:, row_d, oL + 1] = aL * eL
            oR = offs[R]
            if R == nb:
                M[:, row_v, oR] = -1.0
                M[:, row_d, oR] = -aR * (-eR)
            else:
                w = self.B[R] - self.B[R - 1]
                exR = np.exp(-eR * w)
                M[:, row_v, oR] = -1.0
                M[:, row_v, oR + 1] = -exR
                M[:, row_d, oR] = -aR * (-eR)
                M[:, row_d, oR + 1] = -aR * (eR * exR)
            # value: hom_L + part_L = hom_R + part_R
            r[:, row_v] = self.part[:, R] - self.part[:, L]
            # derivative jump from a point source at b
            src = self.source
            if src[0] == "point" and b == float(src[1]):
                if is_iface and self.kind == "sigma":
                    side = src[2]
                    r[:, row_d] = 2.0 * (aL if side == layL else aR)
                else:
                    r[:, row_d] = 2.0
        self.coef = np.linalg.solve(M, r[..., None])[..., 0]
        self.offs = offs

    def _interval(self, z, side=0):
        """Interval index containing z (side=-1/+1 picks the interval to the
        left/right of a breakpoint)."""
        k = int(np.searchsorted(self.B, z, side="right"))
        if side < 0 and k > 0 and z == self.B[k - 1]:
            k -= 1
        return k

    def value(self, z, side=0):
        """Psi(z) (continuous, so the side only matters for tidiness)."""
        k = self._interval(z, side)
        o = self.offs[k]
        e = self.eta[:, k]
        nb = self.B.size
        if k == 0:
            v = self.coef[:, o] * np.exp(-e * (self.B[0] - z))
        elif k == nb:
            v = self.coef[:, o] * np.exp(-e * (z - self.B[-1]))
        else:
            zl, zr = self.B[k - 1], self.B[k]
            v = self.coef[:, o] * np.exp(-e * (z - zl)) + self.coef[:, o + 1] * np.exp(-e * (zr - z))
        return v + self.part[:, k]

    def deriv(self, z, side=0):
        """d/dz Psi(z) on the interval chosen by side (one-sided at a
        breakpoint: -1 left, +1 right)."""
        k = self._interval(z, side)
        o = self.offs[k]
        e = self.eta[:, k]
        nb = self.B.size
        if k == 0:
            return e * self.coef[:, o] * np.exp(-e * (self.B[0] - z))
        if k == nb:
            return -e * self.coef[:, o] * np.exp(-e * (z - self.B[-1]))
        zl, zr = self.B[k - 1], self.B[k]
        return (-e * self.coef[:, o] * np.exp(-e * (z - zl))
                + e * self.coef[:, o + 1] * np.exp(-e * (zr - z)))

    def integral(self, a, b):
        """int_a^b Psi(z) dz, a < b, splitting at breakpoints."""
        cuts = [a] + [x for x in self.B if a < x < b] + [b]
        tot = np.zeros(self.lam.size, dtype=np.complex128)
        nb = self.B.size
        for p, q in zip(cuts[:-1], cuts[1:]):
            k = self._interval(0.5 * (p + q))
            o = self.offs[k]
            e = self.eta[:, k]
            w = q - p
            # (exp(-e alpha) - exp(-e (alpha + w))) / e, stable for small e*w
            g = -np.expm1(-e * w) / e
            if k == 0:
                tot += self.coef[:, o] * np.exp(-e * (self.B[0] - q)) * g
            elif k == nb:
                tot += self.coef[:, o] * np.exp(-e * (p - self.B[-1])) * g
            else:
                zl, zr = self.B[k - 1], self.B[k]
                tot += self.coef[:, o] * np.exp(-e * (p - zl)) * g
                tot += self.coef[:, o + 1] * np.exp(-e * (zr - q)) * g
            tot += self.part[:, k] * w
        return tot


def U_point(lam, d, sigma, freq, kind, z, z0, layer0=None):
    """U_kind(z, z0; lambda) for scalar z, z0 (array over lambda)."""
    if layer0 is None:
        layer0 = _layer_at(np.asarray(d, float), z0)
    return Profile(lam, d, sigma, freq, kind, ("point", z0, layer0)).value(z)
