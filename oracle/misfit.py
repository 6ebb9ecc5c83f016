"""Impedance tensor, misfit and its gradient with respect to log sigma_a.
Test infrastructure.

The benchmark of Sect. 4 is compared through the impedance of the x and y
plane-wave polarisations (apparent resistivity is |Z|^2 / (w mu0)).  An
inversion built on the solver needs the misfit
    phi = sum_f sum_q sum_ij |Z_ij(f, q) - Zobs_ij(f, q)|^2
and d phi / d log sa for every anomaly cell with real conductivity (Sect. 4
uses real sigma).  Both are written out here in the plainest form:

Forward, per frequency (Sect. 2.1 integral equation averaged over cells,
Sect. 2.2 field representation):
    P E = <E^N>,  P = I - V^-1 B (sa - sb)         (dense LU)
    e = E^N + ME j,  h = H^N + MH j,  j = (sa - sb) E
    Z = Eh Hh^-1,  Eh[c][p] = e_c of polarisation p (c, p in {x, y}).
ME, MH are the receiver matrices: row (q, a) holds the cell integrals of
G^E_a. and G^H_a. for receiver q over every cell and current component.

Gradient by forward sensitivities, one dense solve per cell (a different
route from the adjoint solve the library uses):
    dE/dsa_k = P^-1 V^-1 B[:, k] E_k      (the three columns of cell k)
    de/dsa_k = ME[:, k] E_k + ME (sa - sb) dE/dsa_k,   dh likewise
    dZ = (dEh - Z dHh) Hh^-1
    d phi / d log sa_k = sa_k 2 Re sum conj(Z - Zobs) dZ.
Pinned by central finite differences of phi (tests/test_oracle_misfit.py).
"""
from __future__ import annotations

import numpy as np

from . import dense, fields, normal_field


def receiver_matrices(model, rec_xy, freq=None, z0=0.0):
    """ME, MH [nrec][3][3N]: anomalous surface fields per unit current in the
    vector layout [3][Nz][Ny][Nx]."""
    nx, ny, nz = model["nx"], model["ny"], model["nz"]
    hx, hy = model["hx"], model["hy"]
    x0, y0 = model.get("x0", 0.0), model.get("y0", 0.0)
    rec_xy = np.atleast_2d(np.asarray(rec_xy, float))
    cx = x0 + (np.arange(nx) + 0.5) * hx
    cy = y0 + (np.arange(ny) + 0.5) * hy
    offs = np.array([(xr - cxx, yr - cyy) for (xr, yr) in rec_xy for cyy in cy for cxx in cx])
    KE, KH = fields.receiver_kernels(model, offs, freq, z0)
    nq = len(rec_xy)
    # K[q, y, x, z, a, b] -> M[q, a, (b, z, y, x)]
    ME = KE.reshape(nq, ny, nx, nz, 3, 3).transpose(0, 4, 5, 3, 1, 2).reshape(nq, 3, -1)
    MH = KH.reshape(nq, ny, nx, nz, 3, 3).transpose(0, 4, 5, 3, 1, 2).reshape(nq, 3, -1)
    return ME, MH


def operator(model, packed, rec_xy, freq):
    """Everything the forward map needs at one frequency: the dense B of a
    packed table, the receiver matrices, the normal fields."""
    ME, MH = receiver_matrices(model, rec_xy, freq)
    EN, HN = fields.surface_normal_fields(model, freq)
    return dict(freq=freq, B=dense.dense_from_packed(packed, model), ME=ME, MH=MH, EN=EN, HN=HN,
                en=normal_field.normal_field_cells(model, freq=freq))


def _dsig(model, sigma_a):
    sb = model["sigma"][model["layer_of_cell"]]
    return np.tile((sigma_a - sb[:, None, None]).reshape(-1), 3)


def forward(model, op, sigma_a):
    """E [2][3N], e, h [2][nrec][3] and the matrix P at one frequency."""
    P = dense.physical_matrix(op["B"], model, sigma_a)
    E = np.linalg.solve(P, op["en"].reshape(2, -1).T).T
    j = E * _dsig(model, sigma_a)[None]
    e = np.einsum("qak,rk->rqa", op["ME"], j) + op["EN"][:, None, :]
    h = np.einsum("qak,rk->rqa", op["MH"], j) + op["HN"][:, None, :]
    return E, e, h, P


def impedance(e, h):
    """Z [nrec][2][2] from the two polarisations."""
    return fields.impedance(e, h)


def misfit(model, ops, sigma_a, Zobs):
    """phi and Z [nf][nrec][2][2]."""
    Zs = np.array([impedance(*forward(model, op, sigma_a)[1:3]) for op in ops])
    return float(np.sum(np.abs(Zs - Zobs) ** 2)), Zs


def misfit_gradient(model, ops, sigma_a, Zobs):
    """d phi / d log sa [Nz][Ny][Nx] by forward sensitivities (real sa)."""
    N = sigma_a.size
    vol = np.tile(np.repeat(dense.cell_volumes(model), sigma_a[0].size), 3)
    dsig = _dsig(model, sigma_a)
    grad = np.zeros(N)
    for f, op in enumerate(ops):
        B = op["B"]
        E, e, h, P = forward(model, op, sigma_a)
        Z = impedance(e, h)
        Eh = np.stack([e[0, :, :2], e[1, :, :2]], axis=-1)
        Hh = np.stack([h[0, :, :2], h[1, :, :2]], axis=-1)
        Hi = np.linalg.inv(Hh)
        dZres = np.conj(Z - Zobs[f])
        de = np.zeros((2, e.shape[1], 3, N), complex)
        dh = np.zeros_like(de)
        for r in range(2):
            # column k of M: sum_b B[:, (b, k)] E[(b, k)] / V
            M = (B * E[r][None, :]).reshape(3 * N, 3, N).sum(axis=1) / vol[:, None]
            dE = np.linalg.solve(P, M)                               # [3N][N]
            Ek = E[r].reshape(3, N)
            de[r] = (np.einsum("qabk,bk->qak", op["ME"].reshape(-1, 3, 3, N), Ek)
                     + np.einsum("qaj,jk->qak", op["ME"], dsig[:, None] * dE))
            dh[r] = (np.einsum("qabk,bk->qak", op["MH"].reshape(-1, 3, 3, N), Ek)
                     + np.einsum("qaj,jk->qak", op["MH"], dsig[:, None] * dE))
        for k in range(N):
            dEh = np.stack([de[0, :, :2, k], de[1, :, :2, k]], axis=-1)
            dHh = np.stack([dh[0, :, :2, k], dh[1, :, :2, k]], axis=-1)
            dZ = (dEh - Z @ dHh) @ Hi
            grad[k] += 2.0 * np.real(sigma_a.reshape(-1)[k] * np.sum(dZres * dZ))
    return grad.reshape(sigma_a.shape)
