"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only draws numbers and lays out geometry: layered backgrounds,
anomaly boxes, random vectors and random tables that carry the storage
symmetries of the packed format.  It contains none of the method's arithmetic
(no Green's tensor, no operator, no transform), so that the oracle and the
HIP library can both consume its output without sharing any computation.

Conventions (Sect. 2.1 and Appendix B of the paper):
  * z points down, the earth surface is the first interface d_1 = 0,
  * sigma[0] is the air (upper half-space), sigma[nlay] the lower half-space,
  * cells are indexed [iz][iy][ix], x fastest; lateral cell size is uniform.
"""
from __future__ import annotations

import numpy as np

# Storage classes of the packed table: four symmetric Nz x Nz blocks kept as
# upper triangles and two full blocks (Sect. 3.1, consequences of Lemmas 1-2).
PACKED_CLASSES = ("xx", "xy", "yy", "zz", "xz", "yz")
# Lateral parity of each class under x -> -x and y -> -y (Lemma 2).
CLASS_PARITY = {"xx": (1, 1), "yy": (1, 1), "zz": (1, 1), "xy": (-1, -1),
                "xz": (-1, 1), "yz": (1, -1)}


def packed_len(nz: int) -> int:
    """Complex entries stored per lateral offset: 2 Nz (2 Nz + 1)."""
    return 2 * nz * (2 * nz + 1)


def packed_offsets(nz: int) -> dict:
    """Start of each class inside one offset block of the packed table."""
    t = nz * (nz + 1) // 2
    return {"xx": 0, "xy": t, "yy": 2 * t, "zz": 3 * t, "xz": 4 * t,
            "yz": 4 * t + nz * nz}


def make_model(nx, ny, nz, hx, hy, z_edges, d, sigma, freq, sigma_a=None,
               x0=0.0, y0=0.0):
    """Bundle a model description (plain data, no derived quantities)."""
    z_edges = np.asarray(z_edges, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    sigma = np.asarray(sigma, dtype=np.complex128)
    assert z_edges.shape == (nz + 1,)
    assert sigma.shape == (d.size + 1,)
    m = dict(nx=int(nx), ny=int(ny), nz=int(nz), hx=float(hx), hy=float(hy),
             x0=float(x0), y0=float(y0), z_edges=z_edges, d=d, sigma=sigma,
             freq=float(freq))
    m["layer_of_cell"] = layer_index_of_cells(z_edges, d)
    if sigma_a is None:
        sigma_a = np.broadcast_to(sigma[m["layer_of_cell"]][:, None, None],
                                  (nz, ny, nx)).copy()
    m["sigma_a"] = np.asarray(sigma_a, dtype=np.complex128).reshape(nz, ny, nx)
    return m


def layer_index_of_cells(z_edges, d):
    """Index of the layer holding each cell (0 = air).  A cell that straddles
    an interface is rejected: the vertical integrals assume one layer per cell
    (Appendix A)."""
    z_edges = np.asarray(z_edges, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    out = []
    for k in range(z_edges.size - 1):
        a, b = z_edges[k], z_edges[k + 1]
        if not b > a:
            raise ValueError("z_edges must increase")
        mid = 0.5 * (a + b)
        lay = int(np.searchsorted(d, mid, side="right"))
        for di in d:
            if a < di < b:
                raise ValueError(f"cell [{a},{b}] straddles interface {di}")
        out.append(lay)
    return np.asarray(out, dtype=np.int64)


def background_of_cells(model):
    """sigma_b of each z level (pure lookup)."""
    return model["sigma"][model["layer_of_cell"]]


# ----------------------------------------------------------------------------
# Workloads.  Structure follows the paper's test model (Sect. 4): rectangular
# blocks of high contrast in a layered earth under air; real conductivities.
# ----------------------------------------------------------------------------

def config_small(seed=1, freq=0.1):
    """16 x 16 x 4 cells of 500 x 500 x 250 m in air | 0.01 | 0.001 | 0.1 S/m
    (interfaces at 0, 1 km, 10 km); one random box whose cells are the
    background times 10**U(0,3)."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = 16, 16, 4
    z_edges = np.arange(nz + 1) * 250.0
    d = np.array([0.0, 1000.0, 10000.0])
    sigma = np.array([0.0, 0.01, 0.001, 0.1], dtype=np.complex128)
    m = make_model(nx, ny, nz, 500.0, 500.0, z_edges, d, sigma, freq)
    box = _random_box(rng, nx, ny, nz)
    sa = m["sigma_a"].copy()
    sl = (slice(box[4], box[5]), slice(box[2], box[3]), slice(box[0], box[1]))
    fac = 10.0 ** rng.uniform(0.0, 3.0, size=sa[sl].shape)
    sa[sl] = sa[sl] * fac
    m["sigma_a"] = sa
    m["boxes"] = [box]
    return m


def _random_box(rng, nx, ny, nz):
    ix = np.sort(rng.choice(nx + 1, size=2, replace=False))
    iy = np.sort(rng.choice(ny + 1, size=2, replace=False))
    iz = np.sort(rng.choice(nz + 1, size=2, replace=False))
    return (int(ix[0]), int(ix[1]), int(iy[0]), int(iy[1]), int(iz[0]), int(iz[1]))


def config_layered(nx, ny, nz, hx, hy, hz, seed, freq, n_earth_layers=5,
                   n_boxes=3, side_xy=(8, 48), side_z=(4, 16),
                   max_log_contrast=4.0, interface_step=100.0):
    """Seeded layered earth with rectangular anomalies.

    n_earth_layers earth layers: interfaces at interface_step times sorted
    distinct draws from {1..99} below the surface; layer conductivity
    10**U(-4, 0) S/m; n_boxes boxes of U{side_xy} x U{side_xy} x U{side_z}
    cells placed uniformly, conductivity factor 10**U(0, max_log_contrast),
    the last box fixed at the maximum contrast; later boxes override earlier
    ones.  Interfaces are snapped to cell boundaries because interface_step is
    a multiple of hz."""
    rng = np.random.default_rng(seed)
    k = np.sort(rng.choice(np.arange(1, 100), size=n_earth_layers - 1, replace=False))
    d = np.concatenate([[0.0], interface_step * k.astype(np.float64)])
    sig_e = 10.0 ** rng.uniform(-4.0, 0.0, size=n_earth_layers)
    sigma = np.concatenate([[0.0], sig_e]).astype(np.complex128)
    z_edges = np.arange(nz + 1) * float(hz)
    m = make_model(nx, ny, nz, hx, hy, z_edges, d, sigma, freq)
    sa = m["sigma_a"].copy()
    boxes = []
    for b in range(n_boxes):
        sx = int(rng.integers(side_xy[0], side_xy[1] + 1))
        sy = int(rng.integers(side_xy[0], side_xy[1] + 1))
        sz = int(rng.integers(side_z[0], side_z[1] + 1))
        sx, sy, sz = min(sx, nx), min(sy, ny), min(sz, nz)
        x0 = int(rng.integers(0, nx - sx + 1))
        y0 = int(rng.integers(0, ny - sy + 1))
        z0 = int(rng.integers(0, nz - sz + 1))
        if b == n_boxes - 1:
            fac = 10.0 ** max_log_contrast
        else:
            fac = 10.0 ** rng.uniform(0.0, max_log_contrast)
        bg = sigma[m["layer_of_cell"]][z0:z0 + sz]
        sa[z0:z0 + sz, y0:y0 + sy, x0:x0 + sx] = (bg * fac)[:, None, None]
        boxes.append((x0, x0 + sx, y0, y0 + sy, z0, z0 + sz, fac))
    m["sigma_a"] = sa
    m["boxes"] = boxes
    return m


def config_128x128x32(seed=2):
    """128 x 128 x 32 cells of 200 x 200 x 100 m, f = 0.01 Hz."""
    return config_layered(128, 128, 32, 200.0, 200.0, 100.0, seed, 0.01)


def config_precision(seed=3):
    """256 x 256 x 32 cells of 100 x 100 x 50 m, f = 0.01 Hz."""
    return config_layered(256, 256, 32, 100.0, 100.0, 50.0, seed, 0.01)


def config_batched():
    """Three models of uneven size and twelve frequencies 1e-3 .. 10 Hz."""
    freqs = 10.0 ** (-3.0 + 4.0 * np.arange(12) / 11.0)
    models = [config_layered(64, 64, 16, 200.0, 200.0, 100.0, 41, freqs[0]),
              config_layered(96, 96, 24, 200.0, 200.0, 100.0, 42, freqs[0]),
              config_layered(128, 128, 32, 200.0, 200.0, 100.0, 43, freqs[0])]
    return models, freqs


# Blocks of the paper's benchmark model (Sect. 4, Table commemi_table): opposite
# corners (x1, y1, z1), (x2, y2, z2) in km and conductivity in S/m.
COMMEMI3D3_BLOCKS = [
    (0.0, 2.4, 0.05, 3.0, 2.8, 0.30, 0.0033),
    (0.0, 1.8, 0.05, 3.0, 2.4, 0.45, 0.033),
    (0.0, 1.4, 0.05, 3.0, 1.8, 0.30, 0.1),
    (0.0, 0.8, 0.05, 3.0, 1.4, 0.45, 0.033),
    (0.0, 0.4, 0.05, 3.0, 0.8, 0.30, 0.0033),
    (3.4, 2.8, 0.20, 4.4, 4.8, 1.00, 10.0),
    (1.4, 0.0, 1.00, 2.4, 5.6, 3.00, 3.3333),
]


def config_commemi3d3(freq=1.0, h=25.0):
    """The paper's benchmark model (Sect. 4): air | 0-1 km 1e-3 S/m | 1-7.5 km
    1e-4 S/m | half-space 0.1 S/m, the seven blocks of COMMEMI3D3_BLOCKS, on
    cubes of h metres covering x in [0, 4.4] km, y in [0, 5.6] km and
    z in [0.05, 3] km (176 x 224 x 118 cells for h = 25 m, as in the paper's
    scalability runs).  Cells outside the blocks carry the background."""
    nx, ny = int(round(4400.0 / h)), int(round(5600.0 / h))
    nz = int(round(2950.0 / h))
    z_edges = 50.0 + h * np.arange(nz + 1)
    d = np.array([0.0, 1000.0, 7500.0])
    sigma = np.array([0.0, 1e-3, 1e-4, 0.1], dtype=np.complex128)
    m = make_model(nx, ny, nz, h, h, z_edges, d, sigma, freq)
    sa = m["sigma_a"].copy()
    boxes = []
    for (x1, y1, z1, x2, y2, z2, sg) in COMMEMI3D3_BLOCKS:
        ix = (int(round(1000.0 * x1 / h)), int(round(1000.0 * x2 / h)))
        iy = (int(round(1000.0 * y1 / h)), int(round(1000.0 * y2 / h)))
        iz = (int(round((1000.0 * z1 - 50.0) / h)), int(round((1000.0 * z2 - 50.0) / h)))
        sa[iz[0]:iz[1], iy[0]:iy[1], ix[0]:ix[1]] = sg
        boxes.append((ix[0], ix[1], iy[0], iy[1], iz[0], iz[1], sg))
    m["sigma_a"] = sa
    m["boxes"] = boxes
    return m


def config_gradient(seed=5):
    """64 x 64 x 16 cells of 200 x 200 x 100 m, four frequencies, a 32 x 32
    receiver lattice at the surface over every second cell centre."""
    m = config_layered(64, 64, 16, 200.0, 200.0, 100.0, seed, 0.01)
    freqs = np.array([0.01, 0.0464, 0.215, 1.0])
    i = np.arange(32)
    rx = (2 * i + 0.5) * m["hx"]
    ry = (2 * i + 0.5) * m["hy"]
    return m, freqs, (rx, ry)


# ----------------------------------------------------------------------------
# Random data
# ----------------------------------------------------------------------------

def random_complex(rng, shape, scale=1.0):
    return scale * (rng.standard_normal(shape) + 1j * rng.standard_normal(shape))


def random_packed_table(rng, nx, ny, nz, scale=1.0, decay=0.0):
    """Random complex packed spatial table [Ny][Nx][2Nz(2Nz+1)].

    Entries of the classes that are odd in x (xy, xz) at x-offset 0 and of the
    classes that are odd in y (xy, yz) at y-offset 0 are set to zero, as the
    lateral parity of Lemma 2 requires.  decay > 0 damps far offsets."""
    e = packed_len(nz)
    t = random_complex(rng, (ny, nx, e), scale)
    if decay > 0.0:
        ii, jj = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
        t *= np.exp(-decay * np.sqrt(ii ** 2 + jj ** 2))[:, :, None]
    off = packed_offsets(nz)
    sz = {"xx": nz * (nz + 1) // 2, "xy": nz * (nz + 1) // 2,
          "yy": nz * (nz + 1) // 2, "zz": nz * (nz + 1) // 2,
          "xz": nz * nz, "yz": nz * nz}
    for c in PACKED_CLASSES:
        px, py = CLASS_PARITY[c]
        s = slice(off[c], off[c] + sz[c])
        if px < 0:
            t[:, 0, s] = 0.0
        if py < 0:
            t[0, :, s] = 0.0
    return t


def random_vector(rng, nrhs, nz, ny, nx, scale=1.0):
    """Random field coefficients in the vector layout [R][3][Nz][Ny][Nx]."""
    return random_complex(rng, (nrhs, 3, nz, ny, nx), scale)
