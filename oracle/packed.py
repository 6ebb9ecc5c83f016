"""Unpacking of the symmetry-packed coefficient table.

Sect. 3.1 of the paper: B_n^m depends on the lateral offset (i, j) of the two
cells and on their depths, and its 3 x 3 block structure Q(i, j) obeys
  Q_zx = -Q_xz^T, Q_zy = -Q_yz^T, Q_xx, Q_yy, Q_zz, Q_xy symmetric, Q_yx = Q_xy
(Lemma 1), and Lemma 2 fixes the sign of each component under i -> -i and
j -> -j.  Only Q_xz, Q_yz and the upper triangles of Q_xx, Q_xy, Q_yy, Q_zz
for i in [0, Ny), j in [0, Nx) are stored: 2 Nz (2 Nz + 1) complex numbers per
offset.

The storage order inside one offset block (an interface shared with the
library, stated in include/giem.h) is
  [xx upper][xy upper][yy upper][zz upper][xz full][yz full],
upper triangles row-major over iz <= jz, full blocks row-major [iz][jz]; iz is
the depth index of the observation cell n, jz that of the source cell m.

The oracle rebuilds the full tensor for every signed offset directly from
the two lemmas, without reference to any transform.
"""
from __future__ import annotations

import numpy as np

COMP = {"x": 0, "y": 1, "z": 2}


def _upper_to_full(vals, nz):
    m = np.zeros(vals.shape[:-1] + (nz, nz), dtype=np.complex128)
    iu = np.triu_indices(nz)
    m[..., iu[0], iu[1]] = vals
    m[..., iu[1], iu[0]] = vals
    return m


def split_classes(packed, nz):
    """Return the six stored classes of a packed table [..., E] as full
    Nz x Nz blocks: xx, xy, yy, zz (symmetric) and xz, yz (general)."""
    t = nz * (nz + 1) // 2
    out = {}
    for k, name in enumerate(("xx", "xy", "yy", "zz")):
        out[name] = _upper_to_full(packed[..., k * t:(k + 1) * t], nz)
    base = 4 * t
    out["xz"] = packed[..., base:base + nz * nz].reshape(packed.shape[:-1] + (nz, nz))
    out["yz"] = packed[..., base + nz * nz:base + 2 * nz * nz].reshape(
        packed.shape[:-1] + (nz, nz))
    return out


def tensor_row(packed, nz, iz):
    """Q(i, j)[..., iz, :] for i, j >= 0, the row of observation depth iz:
    shape [Ny][Nx][3][3][Nz].  The same numbers as full_tensor_nonneg
    restricted to one row, read straight from the stored classes (Lemma 1)
    so that large grids need not form the whole tensor."""
    t = nz * (nz + 1) // 2
    iu = np.triu_indices(nz)
    pos = np.zeros((nz, nz), dtype=int)
    pos[iu[0], iu[1]] = np.arange(t)
    pos[iu[1], iu[0]] = np.arange(t)
    up = pos[iz]                                  # upper-triangle slot of (iz, jz)
    base = 4 * t
    jz = np.arange(nz)
    q = np.zeros(packed.shape[:2] + (3, 3, nz), dtype=np.complex128)
    q[:, :, 0, 0] = packed[..., up]
    q[:, :, 0, 1] = packed[..., t + up]
    q[:, :, 1, 0] = packed[..., t + up]
    q[:, :, 1, 1] = packed[..., 2 * t + up]
    q[:, :, 2, 2] = packed[..., 3 * t + up]
    q[:, :, 0, 2] = packed[..., base + iz * nz + jz]                 # xz[iz][jz]
    q[:, :, 1, 2] = packed[..., base + nz * nz + iz * nz + jz]       # yz[iz][jz]
    q[:, :, 2, 0] = -packed[..., base + jz * nz + iz]                # zx = -xz^T
    q[:, :, 2, 1] = -packed[..., base + nz * nz + jz * nz + iz]      # zy = -yz^T
    return q


def pack_classes(blocks, nz):
    """Inverse of split_classes for tables built from full blocks."""
    iu = np.triu_indices(nz)
    parts = [blocks[n][..., iu[0], iu[1]] for n in ("xx", "xy", "yy", "zz")]
    lead = blocks["xz"].shape[:-2]
    parts.append(blocks["xz"].reshape(lead + (nz * nz,)))
    parts.append(blocks["yz"].reshape(lead + (nz * nz,)))
    return np.concatenate(parts, axis=-1)


def full_tensor_nonneg(packed, nz):
    """3 x 3 block tensor Q(i, j) for i, j >= 0: shape [Ny][Nx][3][3][Nz][Nz].
    Lemma 1: yx = xy, zx = -xz^T, zy = -yz^T."""
    c = split_classes(packed, nz)
    ny, nx = packed.shape[:2]
    q = np.zeros((ny, nx, 3, 3, nz, nz), dtype=np.complex128)
    q[:, :, 0, 0] = c["xx"]
    q[:, :, 0, 1] = c["xy"]
    q[:, :, 1, 0] = c["xy"]
    q[:, :, 1, 1] = c["yy"]
    q[:, :, 2, 2] = c["zz"]
    q[:, :, 0, 2] = c["xz"]
    q[:, :, 1, 2] = c["yz"]
    q[:, :, 2, 0] = -np.swapaxes(c["xz"], -1, -2)
    q[:, :, 2, 1] = -np.swapaxes(c["yz"], -1, -2)
    return q


# Sign of component (alpha, beta) under x -> -x: the x component of a vector
# changes sign, so the sign is t_alpha t_beta with t = (-1, 1, 1); likewise
# t = (1, -1, 1) under y -> -y.  This reproduces Lemma 2 component by
# component (xx, yy, zz even; xy odd/odd; zx odd in x; zy odd in y).
_TX = np.array([-1.0, 1.0, 1.0])
_TY = np.array([1.0, -1.0, 1.0])
SIGN_X = np.outer(_TX, _TX)
SIGN_Y = np.outer(_TY, _TY)


def full_tensor_signed(packed, nz):
    """Q(i, j) for every signed offset i in (-Ny, Ny), j in (-Nx, Nx).

    Returned array qf has shape [2Ny-1][2Nx-1][3][3][Nz][Nz] and
    qf[i + Ny - 1, j + Nx - 1] = Q(i, j).  Components that are odd in x
    vanish at j = 0 and those odd in y at i = 0 (an odd function is zero at the
    origin); stored values there are ignored."""
    ny, nx = packed.shape[:2]
    q = full_tensor_nonneg(packed, nz)
    q = q.copy()
    odd_x = SIGN_X < 0
    odd_y = SIGN_Y < 0
    q[:, 0][:, odd_x] = 0.0
    q[0, :][:, odd_y] = 0.0
    qf = np.zeros((2 * ny - 1, 2 * nx - 1, 3, 3, nz, nz), dtype=np.complex128)
    sx = SIGN_X[:, :, None, None]
    sy = SIGN_Y[:, :, None, None]
    for i in range(ny):
        for j in range(nx):
            blk = q[i, j]
            qf[ny - 1 + i, nx - 1 + j] = blk
            qf[ny - 1 + i, nx - 1 - j] = sx * blk
            qf[ny - 1 - i, nx - 1 + j] = sy * blk
            qf[ny - 1 - i, nx - 1 - j] = sx * sy * blk
    return qf


def dense_B(packed, nx, ny, nz):
    """The 3N x 3N block-Toeplitz matrix B of eq. (bcyl) in the vector order
    (alpha, iz, iy, ix), ix fastest:
      B[(a, iz, yn, xn), (b, jz, ym, xm)] = Q_ab(yn - ym, xn - xm)[iz, jz]."""
    qf = full_tensor_signed(packed, nz)
    yn = np.arange(ny)[:, None, None, None]
    xn = np.arange(nx)[None, :, None, None]
    ym = np.arange(ny)[None, None, :, None]
    xm = np.arange(nx)[None, None, None, :]
    blocks = qf[yn - ym + ny - 1, xn - xm + nx - 1]      # [yn,xn,ym,xm,3,3,nz,nz]
    blocks = blocks.transpose(4, 6, 0, 1, 5, 7, 2, 3)    # [a,iz,yn,xn,b,jz,ym,xm]
    n3 = 3 * nz * ny * nx
    return np.ascontiguousarray(blocks).reshape(n3, n3)


def packed_table_bytes(nx, ny, nz, bytes_per_complex=16):
    """Storage of the packed table: 2 Nx Ny Nz (2 Nz + 1) complex (Sect. 3.1)."""
    return 2 * nx * ny * nz * (2 * nz + 1) * bytes_per_complex


def full_table_bytes(nx, ny, nz, bytes_per_complex=16):
    """Storage of the unpacked table used by earlier solvers: 36 Nx Ny Nz^2
    complex (Sect. 3.1)."""
    return 36 * nx * ny * nz * nz * bytes_per_complex
