"""Normal (background) field of a plane wave in the layered earth.

Sect. 2.1 of the paper: E^N, H^N solve Maxwell's equations with the layered
conductivity sigma_b(z), time factor exp(-i omega t).  For a vertically
incident plane wave the field is horizontal and depends on z only:
    E'' + k^2 E = 0,  k^2 = i omega mu0 sigma,  Im k >= 0,
    H = (1 / (i omega mu0)) curl E.
The paper does not spell out the plane-wave source; the standard
magnetotelluric normalisation is used: E_x (x polarisation) or E_y
(y polarisation) equals 1 V/m at the surface z = 0.

Two independent evaluations are provided: the impedance recursion with
reflection coefficients (stable for any layer thickness) and a transfer
matrix of the first-order system [E, E'] (used as a cross-check).
"""
from __future__ import annotations

import numpy as np

MU0 = 4e-7 * np.pi


def wavenumbers(sigma, omega):
    """k_m = sqrt(i omega mu0 sigma_m) on the branch Im k >= 0."""
    k = np.sqrt(1j * omega * MU0 * np.asarray(sigma, dtype=np.complex128))
    return np.where(k.imag < 0, -k, k)


class LayeredPlaneWave:
    """E(z) of the unit-surface-field plane wave.  Interfaces d[0] = 0 < d[1]
    < ...; sigma[0] is the air, sigma[-1] the lower half-space."""

    def __init__(self, d, sigma, freq):
        self.d = np.asarray(d, dtype=np.float64)
        self.sigma = np.asarray(sigma, dtype=np.complex128)
        self.omega = 2.0 * np.pi * freq
        self.k = wavenumbers(self.sigma, self.omega)
        nl = self.d.size                # earth layers 1..nl, nl = half-space
        self.nl = nl
        z0 = self.omega * MU0 / np.where(self.k == 0, 1.0, self.k)
        self.z0 = z0
        # Impedance recursion from the lower half-space upwards.  In layer m
        # (1 <= m < nl, between d[m-1] and d[m]):
        #   E = a_m (exp(i k (z - d[m])) + r_m exp(-i k (z - d[m]))).
        zb = z0[nl]
        self.r = np.zeros(nl + 1, dtype=np.complex128)
        self.thick = np.zeros(nl + 1)
        for m in range(nl - 1, 0, -1):
            l = self.d[m] - self.d[m - 1]
            self.thick[m] = l
            r = (zb - z0[m]) / (zb + z0[m])
            self.r[m] = r
            e = np.exp(2j * self.k[m] * l)
            zb = z0[m] * (1 + r * e) / (1 - r * e)
        self.Zs = zb                    # surface impedance E_x / H_y
        # Amplitudes a_m from E(0) = 1 downwards.
        self.a = np.zeros(nl + 1, dtype=np.complex128)
        etop = 1.0 + 0j
        for m in range(1, nl):
            l = self.thick[m]
            e = np.exp(1j * self.k[m] * l)
            self.a[m] = etop * e / (1.0 + self.r[m] * e * e)
            etop = self.a[m] * (1.0 + self.r[m])
        self.a[nl] = etop                # E = a_nl exp(i k (z - d[nl-1]))

    def layer_of(self, z):
        return int(np.searchsorted(self.d, z, side="right"))

    def E(self, z):
        """E(z) (scalar field of the active polarisation)."""
        z = float(z)
        m = self.layer_of(z)
        if m == 0:
            return 1.0 + self.dE(0.0) * z       # air: k = 0, E linear in z
        if m == self.nl:
            return self.a[m] * np.exp(1j * self.k[m] * (z - self.d[m - 1]))
        k, dm = self.k[m], self.d[m]
        return self.a[m] * (np.exp(1j * k * (z - dm)) + self.r[m] * np.exp(-1j * k * (z - dm)))

    def dE(self, z):
        """dE/dz; in the air it equals its value at the surface."""
        z = float(z)
        m = self.layer_of(z)
        if m == 0:
            z, m = 0.0, 1 if self.nl > 1 else self.nl
        if m == self.nl:
            k = self.k[m]
            return 1j * k * self.a[m] * np.exp(1j * k * (z - self.d[m - 1]))
        k, dm = self.k[m], self.d[m]
        return 1j * k * self.a[m] * (np.exp(1j * k * (z - dm)) - self.r[m] * np.exp(-1j * k * (z - dm)))

    def H_surface(self):
        """H_y at z = 0 for the x polarisation (= 1 / Z)."""
        return self.dE(0.0) / (1j * self.omega * MU0)

    def cell_average(self, z1, z2):
        """(1 / (z2 - z1)) int_{z1}^{z2} E dz for an interval inside one layer."""
        m = self.layer_of(0.5 * (z1 + z2))
        if m == 0:
            raise ValueError("cell in the air")
        k = self.k[m]
        if m == self.nl:
            dd = self.d[m - 1]
            val = self.a[m] * (np.exp(1j * k * (z2 - dd)) - np.exp(1j * k * (z1 - dd))) / (1j * k)
        else:
            dm = self.d[m]
            up = (np.exp(1j * k * (z2 - dm)) - np.exp(1j * k * (z1 - dm))) / (1j * k)
            dn = (np.exp(-1j * k * (z2 - dm)) - np.exp(-1j * k * (z1 - dm))) / (-1j * k)
            val = self.a[m] * (up + self.r[m] * dn)
        return val / (z2 - z1)


def transfer_matrix_field(d, sigma, freq, z):
    """Independent evaluation: propagate [E, E'] with 2 x 2 layer matrices
    upward from the lower half-space (where E = exp(i k z)), then normalise
    E(0) = 1.  Suitable only where k*thickness is moderate."""
    d = np.asarray(d, float)
    omega = 2 * np.pi * freq
    k = wavenumbers(sigma, omega)
    nl = d.size
    # state at the top of the half-space (z = d[nl-1]): E = 1, E' = i k
    e, de = 1.0 + 0j, 1j * k[nl]
    states = {nl: (d[nl - 1], e, de)}
    for m in range(nl - 1, 0, -1):
        l = d[m] - d[m - 1]
        km = k[m]
        c, s = np.cos(km * l), np.sin(km * l)
        # going up by l: E(z - l) = E c - E' s / k, E'(z - l) = E k s + E' c
        e, de = e * c - de * s / km, e * km * s + de * c
        states[m] = (d[m - 1], e, de)
    scale = 1.0 / e
    zz = float(z)
    m = int(np.searchsorted(d, zz, side="right"))
    if m == 0:
        return 1.0 + de * scale * zz
    ztop, et, dt = states[m]
    km = k[m]
    t = zz - ztop
    return scale * (et * np.cos(km * t) + dt * np.sin(km * t) / km)


def cell_averages(model, freq=None):
    """<E^N>_n of each depth level for a unit surface field."""
    f = model["freq"] if freq is None else freq
    pw = LayeredPlaneWave(model["d"], model["sigma"], f)
    ze = model["z_edges"]
    return np.array([pw.cell_average(ze[k], ze[k + 1]) for k in range(ze.size - 1)])


def plane_wave_rhs(model, pols=("x", "y"), freq=None):
    """U^0 = sqrt(Re sb) <E^N> for each polarisation: [R][3][Nz][Ny][Nx]."""
    nz, ny, nx = model["nz"], model["ny"], model["nx"]
    avg = cell_averages(model, freq)
    sb = model["sigma"][model["layer_of_cell"]]
    s = np.sqrt(sb.real)
    out = np.zeros((len(pols), 3, nz, ny, nx), dtype=np.complex128)
    for r, p in enumerate(pols):
        c = {"x": 0, "y": 1}[p]
        out[r, c] = (s * avg)[:, None, None]
    return out


def normal_field_cells(model, pols=("x", "y"), freq=None):
    """<E^N>_n in the vector layout (unscaled)."""
    nz, ny, nx = model["nz"], model["ny"], model["nx"]
    avg = cell_averages(model, freq)
    out = np.zeros((len(pols), 3, nz, ny, nx), dtype=np.complex128)
    for r, p in enumerate(pols):
        out[r, {"x": 0, "y": 1}[p]] = avg[:, None, None]
    return out
