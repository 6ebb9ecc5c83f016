"""Pins of the oracle's hot-path parts against what the paper and the
mathematics fix: storage symmetry (Sect. 3.1), table size (8x claim), the
relation between the scaled and the physical system (Sect. 2.2), the
sigma_a = sigma_b special case, and the 1-D normal field."""
import os

import numpy as np
import pytest

import giem_synth as gs
from oracle import dense, normal_field, packed


def _small_model(seed=7, nx=5, ny=4, nz=3):
    rng = np.random.default_rng(seed)
    z = np.array([0.0, 100.0, 250.0, 300.0])[: nz + 1]
    m = gs.make_model(nx, ny, nz, 50.0, 60.0, z, [0.0, 250.0, 2000.0],
                      [0.0, 0.01, 0.1, 0.003], 1.0)
    sa = m["sigma_a"] * 10 ** rng.uniform(0, 2, size=m["sigma_a"].shape)
    m["sigma_a"] = sa
    return m


def test_pack_roundtrip_exact():
    rng = np.random.default_rng(0)
    t = gs.random_packed_table(rng, 4, 3, 5)
    c = packed.split_classes(t, 5)
    assert np.array_equal(packed.pack_classes(c, 5), t)
    for k in ("xx", "xy", "yy", "zz"):
        assert np.array_equal(c[k], np.swapaxes(c[k], -1, -2))


def test_table_sizes_eight_fold():
    # 2 Nx Ny Nz (2Nz+1) complex vs 36 Nx Ny Nz^2 (Sect. 3.1); ratio -> 9 for
    # the 36-form and -> 8 for the 32-form as Nz grows.
    nx, ny, nz = 128, 128, 32
    assert gs.packed_len(nz) * nx * ny * 16 == packed.packed_table_bytes(nx, ny, nz)
    assert packed.packed_table_bytes(nx, ny, nz) == 2 * 128 * 128 * 32 * 65 * 16
    r32 = 32 * nx * ny * nz * nz * 16 / packed.packed_table_bytes(nx, ny, nz)
    assert abs(r32 - 8 * 2 * nz / (2 * nz + 1)) < 1e-12 and 7.8 < r32 < 8.0


def _storage_golden():
    path = os.path.join(os.path.dirname(__file__), "golden", "storage_bytes.txt")
    forms = {}
    with open(path) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                tok = line.split()
                forms[tok[0]] = tuple(int(v) for v in tok[1:3]) if tok[0] != "factor" else int(tok[1])
    return forms


def _golden_bytes(form, nx, ny, nz):
    a, b = form
    return 16 * nx * ny * (a * nz * nz + b * nz)


@pytest.mark.parametrize("nx,ny,nz", [(3, 2, 1), (5, 4, 3), (6, 3, 4)])
def test_storage_matches_paper_figures(nx, ny, nz):
    # the counts printed in Sect. 3.1 against what the oracle actually holds:
    # its unpacked spectral blocks (4 Nx Ny offsets of the cyclic embedding,
    # 9 Nz x Nz blocks), the same with the yx block dropped (it equals xy,
    # Lemma 1) and the packed table (Lemmas 1 and 2), which unpacks and packs
    # back unchanged
    from oracle import fft_apply, tables
    g = _storage_golden()
    t = gs.random_packed_table(np.random.default_rng(nx + ny + nz), nx, ny, nz)
    qhat = fft_apply.spectral_blocks(t, nz).reshape(2 * ny, 2 * nx, 3, nz, 3, nz)
    assert qhat.size * 16 == _golden_bytes(g["unpacked"], nx, ny, nz)
    assert np.allclose(qhat[:, :, 1, :, 0], qhat[:, :, 0, :, 1], rtol=0, atol=1e-12 * np.abs(qhat).max())
    assert 8 * (qhat.size // 9) * 16 == _golden_bytes(g["symmetric"], nx, ny, nz)
    assert np.array_equal(tables.pack(packed.full_tensor_signed(t, nz), nx, ny, nz), t)
    assert t.size * 16 == _golden_bytes(g["packed"], nx, ny, nz)
    # the reduction approaches the printed factor from below as Nz grows
    ratios = [_golden_bytes(g["symmetric"], 1, 1, k) / _golden_bytes(g["packed"], 1, 1, k)
              for k in (1, 4, 32, 10 ** 4)]
    assert all(r < g["factor"] for r in ratios) and ratios == sorted(ratios)
    assert abs(ratios[-1] - g["factor"]) < 1e-3


def test_unpacked_tensor_satisfies_lemmas():
    rng = np.random.default_rng(1)
    nx, ny, nz = 4, 3, 3
    t = gs.random_packed_table(rng, nx, ny, nz)
    qf = packed.full_tensor_signed(t, nz)
    c = lambda i, j: qf[i + ny - 1, j + nx - 1]
    for i in range(-ny + 1, ny):
        for j in range(-nx + 1, nx):
            q = c(i, j)
            # Lemma 1 / block relations
            assert np.array_equal(q[2, 0], -q[0, 2].T)
            assert np.array_equal(q[2, 1], -q[1, 2].T)
            assert np.array_equal(q[1, 0], q[0, 1])
            for a in range(3):
                assert np.array_equal(q[a, a], q[a, a].T)
            # Lemma 2 parities
            qx, qy = c(i, -j), c(-i, j)
            assert np.array_equal(qx[0, 0], q[0, 0]) and np.array_equal(qy[2, 2], q[2, 2])
            assert np.array_equal(qx[0, 1], -q[0, 1]) and np.array_equal(qy[0, 1], -q[0, 1])
            assert np.array_equal(qx[2, 0], -q[2, 0]) and np.array_equal(qy[2, 0], q[2, 0])
            assert np.array_equal(qx[2, 1], q[2, 1]) and np.array_equal(qy[2, 1], -q[2, 1])


def test_dense_B_symmetric_and_toeplitz():
    rng = np.random.default_rng(2)
    nx, ny, nz = 4, 3, 2
    t = gs.random_packed_table(rng, nx, ny, nz)
    B = packed.dense_B(t, nx, ny, nz)
    # reciprocity: B = B^T (not B^H)
    assert np.array_equal(B, B.T)
    # block-Toeplitz: entry depends on the lateral offset only
    Bv = B.reshape(3, nz, ny, nx, 3, nz, ny, nx)
    assert np.array_equal(Bv[:, :, 1, 2, :, :, 0, 1], Bv[:, :, 2, 3, :, :, 1, 2])


def test_scaled_system_equals_physical_system():
    """With U = a E the scaled system of Sect. 2.2 is the cell average of the
    integral equation: A u = s <E^N> and P E = <E^N> give the same E."""
    m = _small_model()
    rng = np.random.default_rng(3)
    t = gs.random_packed_table(rng, m["nx"], m["ny"], m["nz"], scale=1e3)
    B = dense.dense_from_packed(t, m)
    d = dense.cie_diagonals(m)
    A = dense.system_matrix(B, d)
    assert np.allclose(A, dense.system_matrix_from_K(B, d), rtol=0, atol=1e-12 * np.abs(A).max())
    en = normal_field.normal_field_cells(m)
    b = normal_field.plane_wave_rhs(m)
    u = dense.solve_lu(A, b)
    E1 = u / np.tile(d["a"].reshape(-1), 3).reshape(1, 3, *d["a"].shape)
    P = dense.physical_matrix(B, m)
    E2 = dense.solve_lu(P, en)
    assert np.linalg.norm(E1 - E2) <= 1e-11 * np.linalg.norm(E2)


def test_no_anomaly_gives_normal_field():
    m = _small_model()
    m["sigma_a"] = np.broadcast_to(dense.cell_layer_sigma(m)[:, None, None],
                                   m["sigma_a"].shape).copy()
    rng = np.random.default_rng(4)
    t = gs.random_packed_table(rng, m["nx"], m["ny"], m["nz"], scale=1e3)
    B = dense.dense_from_packed(t, m)
    d = dense.cie_diagonals(m)
    assert np.all(d["gamma"] == 0)
    A = dense.system_matrix(B, d)
    assert np.array_equal(A, np.eye(A.shape[0]))


def test_transpose_mode_is_bilinear_adjoint():
    m = _small_model()
    rng = np.random.default_rng(5)
    t = gs.random_packed_table(rng, m["nx"], m["ny"], m["nz"])
    B = dense.dense_from_packed(t, m)
    d = dense.cie_diagonals(m)
    x = gs.random_vector(rng, 1, m["nz"], m["ny"], m["nx"])
    y = gs.random_vector(rng, 1, m["nz"], m["ny"], m["nx"])
    Ax = dense.apply_direct(B, d, x, "A")
    ATy = dense.apply_direct(B, d, y, "AT")
    lhs, rhs = np.sum(Ax * y), np.sum(x * ATy)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


@pytest.mark.parametrize("mode", ["A", "AT", "B"])
def test_direct_apply_equals_paper_system_matrix(mode):
    """The O(N^2) apply in the factorised form S + R1 B R2 against the dense
    matrix written as the paper's system, I - K Gamma (Sect. 2.2), its
    transpose, and B itself: a swapped R1/R2 or a dropped term fails."""
    m = _small_model()
    rng = np.random.default_rng(11)
    t = gs.random_packed_table(rng, m["nx"], m["ny"], m["nz"], scale=1e3)
    B = dense.dense_from_packed(t, m)
    d = dense.cie_diagonals(m)
    x = gs.random_vector(rng, 2, m["nz"], m["ny"], m["nx"])
    M = {"A": dense.system_matrix_from_K(B, d), "B": B}.get(mode)
    if mode == "AT":
        M = dense.system_matrix_from_K(B, d).T
    ref = (x.reshape(2, -1) @ M.T).reshape(x.shape)
    got = dense.apply_direct(B, d, x, mode)
    assert np.linalg.norm(got - ref) <= 1e-13 * np.linalg.norm(ref)


# ---------------------------------------------------------------- normal field

def test_half_space_impedance_closed_form():
    for sig, f in ((0.01, 1.0), (1.0, 1e-3), (1e-4, 10.0)):
        pw = normal_field.LayeredPlaneWave([0.0], [0.0, sig], f)
        w = 2 * np.pi * f
        k = np.sqrt(1j * w * normal_field.MU0 * sig)
        assert abs(pw.Zs - w * normal_field.MU0 / k) <= 1e-14 * abs(pw.Zs)
        rho = abs(pw.Zs) ** 2 / (w * normal_field.MU0)
        assert abs(rho * sig - 1) < 1e-12
        # e^{-i w t}: the impedance phase is -45 degrees
        assert abs(np.degrees(np.angle(pw.Zs)) + 45.0) < 1e-10
        assert abs(pw.H_surface() - 1.0 / pw.Zs) <= 1e-13 * abs(pw.H_surface())


def test_layered_field_recursion_vs_transfer_matrix():
    d = [0.0, 1000.0, 10000.0]
    s = [0.0, 0.01, 0.001, 0.1]
    pw = normal_field.LayeredPlaneWave(d, s, 0.1)
    for z in (-50.0, 0.0, 10.0, 999.0, 1001.0, 5000.0, 10500.0, 20000.0):
        a, b = pw.E(z), normal_field.transfer_matrix_field(d, s, 0.1, z)
        assert abs(a - b) <= 1e-12 * max(abs(a), 1e-3)


def test_layered_field_satisfies_interface_conditions():
    d = [0.0, 300.0, 1200.0, 4000.0]
    s = [0.0, 0.05, 0.002, 1.0, 0.01]
    pw = normal_field.LayeredPlaneWave(d, s, 3.0)
    eps = 1e-7
    for di in d[1:]:
        assert abs(pw.E(di - eps) - pw.E(di + eps)) < 1e-8
        assert abs(pw.dE(di - eps) - pw.dE(di + eps)) < 1e-8 * abs(pw.dE(di))
    # ODE E'' + k^2 E = 0 inside a layer, by central differences
    z, h = 700.0, 0.5
    k2 = 1j * 2 * np.pi * 3.0 * normal_field.MU0 * s[2]
    e2 = (pw.E(z + h) - 2 * pw.E(z) + pw.E(z - h)) / h ** 2
    assert abs(e2 + k2 * pw.E(z)) < 1e-6 * abs(k2 * pw.E(z))


def test_cell_average_vs_quadrature():
    d = [0.0, 1000.0, 10000.0]
    s = [0.0, 0.01, 0.001, 0.1]
    pw = normal_field.LayeredPlaneWave(d, s, 0.1)
    x, w = np.polynomial.legendre.leggauss(20)
    for z1, z2 in ((0.0, 250.0), (750.0, 1000.0), (1000.0, 1100.0), (10000.0, 10100.0)):
        zz = 0.5 * (z2 - z1) * x + 0.5 * (z1 + z2)
        q = 0.5 * np.sum(w * np.array([pw.E(v) for v in zz]))
        assert abs(pw.cell_average(z1, z2) - q) < 1e-13


def test_oracle_adjoint_gradient_vs_finite_differences():
    m = _small_model(seed=21, nx=3, ny=2, nz=3)
    rng = np.random.default_rng(22)
    t = gs.random_packed_table(rng, m["nx"], m["ny"], m["nz"], scale=3e4)
    B = dense.dense_from_packed(t, m)
    g = gs.random_vector(rng, 2, m["nz"], m["ny"], m["nx"])
    en = normal_field.normal_field_cells(m)
    grad = dense.gradient_log_sigma(B, m, g, en)
    h = 1e-6
    sa = m["sigma_a"]
    for idx in [(0, 0, 0), (1, 1, 2), (2, 0, 1)]:
        sp, sm = sa.copy(), sa.copy()
        sp[idx] *= np.exp(h)
        sm[idx] *= np.exp(-h)
        fd = (dense.objective(B, m, g, en, sp) - dense.objective(B, m, g, en, sm)) / (2 * h)
        assert abs(fd - grad[idx]) <= 1e-6 * np.abs(grad).max() + 1e-5 * abs(fd), (idx, fd, grad[idx])


@pytest.mark.parametrize("mode", ["A", "AT", "B"])
def test_row_evaluator_matches_dense_apply(mode):
    # The per-cell direct sum (used at sizes where no dense matrix fits)
    # against the dense matrix-vector product; the table is scaled so that
    # R1 B R2 is of order one and the B part decides the result.
    m = _small_model(seed=9)
    rng = np.random.default_rng(4)
    t = gs.random_packed_table(rng, m["nx"], m["ny"], m["nz"])
    d = dense.cie_diagonals(m)
    t = t / (np.abs(d["R1"]).max() * np.abs(d["R2"]).max())
    B = dense.dense_from_packed(t, m)
    x = gs.random_vector(rng, 2, m["nz"], m["ny"], m["nx"])
    y = dense.apply_direct(B, d, x, mode)
    cells = [(iz, iy, ix) for iz in range(m["nz"]) for iy in range(m["ny"])
             for ix in range(m["nx"])]
    yc = dense.apply_cells(packed.full_tensor_nonneg(t, m["nz"]), m, x, cells, mode)
    ref = np.stack([y[:, :, iz, iy, ix] for (iz, iy, ix) in cells], 1)
    assert np.abs(yc - ref).max() <= 1e-13 * np.abs(ref).max()


def test_tensor_row_is_a_row_of_the_full_tensor():
    from oracle import packed
    rng = np.random.default_rng(41)
    nz = 5
    t = gs.random_packed_table(rng, 4, 3, nz)
    full = packed.full_tensor_nonneg(t, nz)
    for iz in range(nz):
        assert np.array_equal(packed.tensor_row(t, nz, iz), full[:, :, :, :, iz, :])


@pytest.mark.parametrize("nx,ny,nz,R", [(1, 1, 1, 1), (5, 4, 3, 2), (7, 3, 2, 1), (6, 9, 2, 2)])
@pytest.mark.parametrize("mode", ["A", "AT", "B"])
def test_fft_apply_equals_dense_product(nx, ny, nz, R, mode):
    # the three-step FFT apply (Sect. 3.3) is the dense block-Toeplitz
    # product (eq. bcyl) up to rounding
    from oracle import fft_apply
    m = _small_model(seed=50 + nx + ny, nx=nx, ny=ny, nz=nz)
    rng = np.random.default_rng(51)
    t = gs.random_packed_table(rng, nx, ny, nz, decay=0.1)
    B = dense.dense_from_packed(t, m)
    d = dense.cie_diagonals(m)
    x = gs.random_vector(rng, R, nz, ny, nx)
    ref = dense.apply_direct(B, d, x, mode)
    got = fft_apply.apply(fft_apply.spectral_blocks(t, nz), d, x, mode)
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)
