"""Dense assembly, direct apply and LU solve of the discrete contracting
integral equation (Sect. 2.2 and Sect. 3.1 of the paper).

System (Sect. 2.2, linear system for U_n with matrices K, B, gamma, U^0):
    U_n - sum_m gamma^m K_n^m U_m = U_n^0,
    K_n^m = delta_nm I + (2 / V_n) sqrt(Re sb^m Re sb^n) B_n^m,
    gamma^m = (sa^m - sb^m) / (sa^m + conj(sb^m)),
    U_n^0 = sqrt(Re sb^n) <E^N>_n   (cell average of the normal field).
The identity term is read as delta_nm I; with that reading the system is the
cell average of the integral equation for E (checked by physical_matrix).

Factorised form (Sect. 3.1): A = S + R1 B R2 with the diagonals
    S = 1 - gamma,  R1 = -2 sqrt(Re sb) / V,  R2 = sqrt(Re sb) gamma,
and, because B is symmetric (Lemma 1 with Lemma 2), A^T = S + R2 B R1.
The field is recovered as E_n = U_n / a_n, a = (sa + conj sb) / (2 sqrt(Re sb))
(Sect. 2.1, definition of the scaled field).
"""
from __future__ import annotations

import numpy as np

from . import packed as _packed


def cell_layer_sigma(model):
    """sigma_b of every depth level (the layer holding the cell)."""
    return model["sigma"][model["layer_of_cell"]]


def cell_volumes(model):
    dz = np.diff(model["z_edges"])
    return model["hx"] * model["hy"] * dz


def cie_diagonals(model, sigma_a=None):
    """Per-cell diagonals of the factorised system; arrays [Nz][Ny][Nx]."""
    if sigma_a is None:
        sigma_a = model["sigma_a"]
    sb = cell_layer_sigma(model)[:, None, None] * np.ones_like(sigma_a)
    if np.any(sb.real <= 0.0):
        raise ValueError("Re sigma_b must be positive inside the anomaly domain")
    if np.any(sigma_a.real < 0.0):
        raise ValueError("Re sigma_a must be non-negative")
    s = np.sqrt(sb.real)
    gamma = (sigma_a - sb) / (sigma_a + np.conj(sb))
    a = (sigma_a + np.conj(sb)) / (2.0 * s)
    vol = cell_volumes(model)[:, None, None] * np.ones(sigma_a.shape)
    return dict(S=1.0 - gamma, R1=-2.0 * s / vol, R2=s * gamma, gamma=gamma,
                a=a, s=s, vol=vol, sb=sb)


def _rep3(d):
    """Repeat a per-cell diagonal for the three field components."""
    return np.tile(d.reshape(-1), 3)


def system_matrix(B, diags):
    """A = S + R1 B R2 (dense)."""
    return np.diag(_rep3(diags["S"])) + (_rep3(diags["R1"])[:, None] * B
                                          * _rep3(diags["R2"])[None, :])


def system_matrix_from_K(B, diags):
    """A = I - K Gamma written exactly as the paper's system (Sect. 2.2), as an
    independent assembly of the same matrix."""
    n3 = B.shape[0]
    s = _rep3(diags["s"])
    vol = _rep3(diags["vol"])
    K = np.eye(n3, dtype=np.complex128) + (2.0 / vol)[:, None] * np.outer(s, s) * B
    return np.eye(n3, dtype=np.complex128) - K * _rep3(diags["gamma"])[None, :]


def physical_matrix(B, model, sigma_a=None):
    """P = I - V^{-1} B (sigma_a - sigma_b): the cell average of the integral
    equation E = E^N + int G^E (sa - sb) E (Sect. 2.1)."""
    if sigma_a is None:
        sigma_a = model["sigma_a"]
    d = cie_diagonals(model, sigma_a)
    dsig = _rep3(sigma_a - d["sb"])
    vol = _rep3(d["vol"])
    return np.eye(B.shape[0], dtype=np.complex128) - (B / vol[:, None]) * dsig[None, :]


def apply_direct(B, diags, x, mode="A"):
    """y = A x, A^T x or B x by O(N^2) summation; x has layout [R][3][Nz][Ny][Nx]."""
    xr = x.reshape(x.shape[0], -1)
    if mode == "B":
        return (xr @ B.T).reshape(x.shape)
    S, R1, R2 = _rep3(diags["S"]), _rep3(diags["R1"]), _rep3(diags["R2"])
    if mode == "AT":
        R1, R2 = R2, R1
    y = S[None, :] * xr + R1[None, :] * ((R2[None, :] * xr) @ B.T)
    return y.reshape(x.shape)


def solve_lu(A, rhs):
    """u = A^{-1} b by LU; rhs [R][...]."""
    r = rhs.reshape(rhs.shape[0], -1).T
    return np.linalg.solve(A, r).T.reshape(rhs.shape)


def dense_from_packed(packed, model):
    return _packed.dense_B(packed, model["nx"], model["ny"], model["nz"])


def gradient_log_sigma(B, model, g, en_cells, sigma_a=None):
    """d/d(log sigma_a) of J = Re sum_r g_r . E_r for real conductivities.

    Uses the physical form P(sigma) E = <E^N>, P = I - V^{-1} B Dsigma
    (Sect. 2.1 integral equation averaged over cells):
      dE = P^{-1} V^{-1} B dDsigma E,  mu = P^{-T} g,
      dJ/dsigma_k = sum_alpha (mu^T V^{-1} B)_(alpha,k) E_(alpha,k),
      grad_k = Re(sigma_k dJ/dsigma_k)."""
    if sigma_a is None:
        sigma_a = model["sigma_a"]
    P = physical_matrix(B, model, sigma_a)
    d = cie_diagonals(model, sigma_a)
    vol = _rep3(d["vol"])
    E = solve_lu(P, en_cells)
    nr = g.shape[0]
    grad = np.zeros(sigma_a.size, dtype=np.complex128)
    for r in range(nr):
        mu = np.linalg.solve(P.T, g[r].reshape(-1))
        row = (mu / vol) @ B
        grad += (row * E[r].reshape(-1)).reshape(3, -1).sum(axis=0)
    return np.real(sigma_a.reshape(-1) * grad).reshape(sigma_a.shape)


def objective(B, model, g, en_cells, sigma_a):
    """J = Re sum_r g_r . E_r with E from the physical form (for finite differences)."""
    P = physical_matrix(B, model, sigma_a)
    E = solve_lu(P, en_cells)
    return float(np.real(np.sum(g * E)))


def offset_blocks(qnn, dy, dx):
    """Q(dy, dx) for arrays of signed offsets from a non-negative tensor
    qnn[Ny][Nx][3][3][...] (packed.full_tensor_nonneg, or a slice of it over
    the trailing depth indices): Lemma 2 mirror signs, with the odd
    components zero on the axis they are odd in."""
    dy = np.asarray(dy)
    dx = np.asarray(dx)
    q = qnn[np.abs(dy), np.abs(dx)]                       # [..., 3, 3, *rest]
    sx = np.where((dx < 0)[..., None, None], _packed.SIGN_X, 1.0)
    sy = np.where((dy < 0)[..., None, None], _packed.SIGN_Y, 1.0)
    zx = np.where((dx == 0)[..., None, None] & (_packed.SIGN_X < 0), 0.0, 1.0)
    zy = np.where((dy == 0)[..., None, None] & (_packed.SIGN_Y < 0), 0.0, 1.0)
    sgn = sx * sy * zx * zy
    return q * sgn.reshape(sgn.shape + (1,) * (q.ndim - sgn.ndim))


def apply_cells(qnn, model, x, cells, mode="A", sigma_a=None):
    """Selected rows of y = A x (mode "A"), A^T x ("AT") or B x ("B"), each
    by direct summation over every source cell of eq. (bcyl), with no FFT:
      (B x)_(a, n) = sum_m sum_b Q_ab(y_n - y_m, x_n - x_m)[iz_n, iz_m] x_(b, m).
    qnn from packed.full_tensor_nonneg, or a function iz -> its row
    (packed.tensor_row) for grids where the whole tensor is too large;
    x [R][3][Nz][Ny][Nx]; cells is a list of (iz, iy, ix).  Returns
    [R][len(cells)][3].  A^T uses B = B^T (reciprocity), so A^T = S + R2 B R1."""
    nz, ny, nx = model["nz"], model["ny"], model["nx"]
    d = cie_diagonals(model, sigma_a) if mode != "B" else None
    xs = x
    if mode == "A":
        xs = x * d["R2"][None, None]
    elif mode == "AT":
        xs = x * d["R1"][None, None]
    ym = np.arange(ny)
    xm = np.arange(nx)
    out = np.zeros((x.shape[0], len(cells), 3), dtype=np.complex128)
    for k, (iz, iy, ix) in enumerate(cells):
        qrow = qnn(iz) if callable(qnn) else qnn[:, :, :, :, iz, :]
        row = offset_blocks(qrow, (iy - ym)[:, None], (ix - xm)[None, :])  # [ny,nx,a,b,jz]
        bx = np.einsum("yxabj,rbjyx->ra", row, xs, optimize=True)
        if mode == "B":
            out[:, k] = bx
        else:
            left = d["R1"] if mode == "A" else d["R2"]
            out[:, k] = d["S"][iz, iy, ix] * x[:, :, iz, iy, ix] + left[iz, iy, ix] * bx
    return out
