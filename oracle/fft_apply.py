"""The operator apply by the three steps of Sect. 3.3 on the CPU (scipy.fft and
batched matrix products): a timing baseline and a check of the
block-Toeplitz structure.  Test infrastructure.

B x is a 2-D convolution over lateral offsets with 3Nz x 3Nz blocks:
  (B x)(n) = sum_m Q(y_n - y_m, x_n - x_m) x(m)      (eq. bcyl, Sect. 3.1).
Placing Q(i, j) at ((i mod 2Ny), (j mod 2Nx)) of a 2Ny x 2Nx grid (row Ny and
column Nx stay zero) makes it a cyclic convolution of the zero-padded input,
which the 2-D DFT turns into one 3Nz x 3Nz matrix product per frequency:
  1. X^ = DFT2(x padded to 2Ny x 2Nx), per component and depth;
  2. Y^(k) = Q^(k) X^(k), Q^ = DFT2 of the embedded blocks;
  3. B x = inverse DFT2(Y^) restricted to [0, Ny) x [0, Nx).
The whole spectral table is kept unpacked (no use of the symmetries of
Lemmas 1 and 2 beyond building Q for negative offsets), so it holds
4 NxNy (3Nz)^2 complex numbers.  A x = S x + R1 B (R2 x) as in oracle.dense.
"""
from __future__ import annotations

import os

import numpy as np
import scipy.fft

from . import packed as _packed


def _workers():
    return os.cpu_count() or 1


def spectral_blocks(packed, nz):
    """Q^ as [2Ny * 2Nx][3Nz][3Nz] (frequency-major, row (alpha, iz), column
    (beta, jz)) from a packed table [Ny][Nx][E]."""
    ny, nx = packed.shape[:2]
    qf = _packed.full_tensor_signed(packed, nz)              # [2Ny-1][2Nx-1][3][3][nz][nz]
    c = np.zeros((2 * ny, 2 * nx, 3, 3, nz, nz), dtype=np.complex128)
    iy = np.arange(-(ny - 1), ny) % (2 * ny)
    ix = np.arange(-(nx - 1), nx) % (2 * nx)
    c[iy[:, None], ix[None, :]] = qf
    del qf
    c = scipy.fft.fft2(c, axes=(0, 1), workers=_workers(), overwrite_x=True)
    p3 = 3 * nz
    return np.ascontiguousarray(c.transpose(0, 1, 2, 4, 3, 5)).reshape(4 * ny * nx, p3, p3)


def apply_B(qhat, x):
    """B x for x [R][3][Nz][Ny][Nx]."""
    R, _, nz, ny, nx = x.shape
    p3, K = 3 * nz, 4 * ny * nx
    pad = np.zeros((R, 3, nz, 2 * ny, 2 * nx), dtype=np.complex128)
    pad[..., :ny, :nx] = x
    X = scipy.fft.fft2(pad, axes=(-2, -1), workers=_workers(), overwrite_x=True)
    Xm = X.reshape(R, p3, K).transpose(2, 1, 0)               # [K][3Nz][R]
    Ym = np.matmul(qhat, Xm)                                  # [K][3Nz][R]
    Y = np.ascontiguousarray(Ym.transpose(2, 1, 0)).reshape(R, 3, nz, 2 * ny, 2 * nx)
    y = scipy.fft.ifft2(Y, axes=(-2, -1), workers=_workers(), overwrite_x=True)
    return np.ascontiguousarray(y[..., :ny, :nx])


def apply(qhat, diags, x, mode="A"):
    """y = A x, A^T x or B x with the diagonals of oracle.dense.cie_diagonals."""
    if mode == "B":
        return apply_B(qhat, x)
    S, R1, R2 = diags["S"], diags["R1"], diags["R2"]
    if mode == "AT":
        R1, R2 = R2, R1
    return S[None, None] * x + R1[None, None] * apply_B(qhat, R2[None, None] * x)
