"""Pins of the oracle's receiver kernels and surface fields (Sect. 2.2 field
representation through G^E and G^H): the whole-space closed form, Faraday's
law between the two kernels, the insulating-air boundary condition, the
normal-field limit and the half-space impedance."""
import numpy as np
import pytest

import giem_synth as gs
from oracle import dense, fields, wholespace
from oracle.fundamental import MU0


def test_receiver_kernels_whole_space_closed_form():
    sig, f = 0.01, 1.0
    m = dict(nx=3, ny=3, nz=2, hx=100.0, hy=120.0, z_edges=np.array([50.0, 90.0, 140.0]),
             d=np.array([0.0]), sigma=np.array([sig, sig], complex), freq=f)
    offs = np.array([[0.0, 0.0], [100.0, 0.0], [0.0, 120.0], [230.0, -70.0], [-45.0, 30.0]])
    KE, KH = fields.receiver_kernels(m, offs)
    for k, (dx, dy) in enumerate(offs):
        for jz in range(2):
            lo = [-50.0, -60.0, m["z_edges"][jz]]
            hi = [50.0, 60.0, m["z_edges"][jz + 1]]
            E, H = wholespace.point_box([dx, dy, 0.0], lo, hi, sig, f, q=16)
            assert np.abs(KE[k, jz] - E).max() <= 1e-8 * np.abs(E).max()
            assert np.abs(KH[k, jz] - H).max() <= 1e-8 * np.abs(H).max()


def test_faraday_vertical_field_at_the_surface():
    # H_z = (d_x E_y - d_y E_x) / (i w mu0) at a receiver on the top face of a
    # surface cell; 100 Hz so that the inductive part is not swamped by the
    # galvanic one, fourth-order differences
    rng = np.random.default_rng(3)
    m = gs.make_model(2, 2, 2, 100.0, 100.0, np.array([0.0, 50.0, 120.0]), [0.0, 50.0, 800.0],
                      [0.0, 0.2, 1.0, 0.05], 100.0)
    m["sigma_a"] = m["sigma_a"] * 10 ** rng.uniform(0, 1, m["sigma_a"].shape)
    E = gs.random_vector(rng, 1, 2, 2, 2)
    r0, dl = np.array([137.0, 63.0]), 1.0
    st = [r0 + [dl, 0], r0 - [dl, 0], r0 + [2 * dl, 0], r0 - [2 * dl, 0],
          r0 + [0, dl], r0 - [0, dl], r0 + [0, 2 * dl], r0 - [0, 2 * dl], r0]
    e, h = fields.fields_at(m, E, np.array(st))

    def d4(fp, fm, f2p, f2m):
        return (8 * (fp - fm) - (f2p - f2m)) / (12 * dl)

    curl = (d4(e[0, 0, 1], e[0, 1, 1], e[0, 2, 1], e[0, 3, 1])
            - d4(e[0, 4, 0], e[0, 5, 0], e[0, 6, 0], e[0, 7, 0])) / (1j * 2 * np.pi * m["freq"] * MU0)
    assert abs(curl - h[0, 8, 2]) <= 1e-5 * abs(h[0, 8, 2])


def test_insulating_air_boundary_condition():
    # sigma_0 = 0: no current crosses the surface, sigma_1 E_z + j_z = 0 just
    # below it, so the anomalous E_z above a cell is -j_z / sigma_1 of the top cell
    rng = np.random.default_rng(5)
    m = gs.make_model(3, 2, 2, 100.0, 100.0, np.array([0.0, 40.0, 100.0]), [0.0, 40.0],
                      [0.0, 0.03, 0.2], 1.0)
    m["sigma_a"] = m["sigma_a"] * 10 ** rng.uniform(0, 1, m["sigma_a"].shape)
    E = gs.random_vector(rng, 1, 2, 2, 3)
    rec = np.array([[150.0, 50.0], [50.0, 150.0]])
    e, h = fields.fields_at(m, E, rec)
    s1 = m["sigma"][1]
    for q, (ix, iy) in enumerate([(1, 0), (0, 1)]):
        jz = (m["sigma_a"][0, iy, ix] - s1) * E[0, 2, 0, iy, ix]
        assert abs(e[0, q, 2] + jz / s1) <= 1e-10 * abs(jz / s1)


def test_no_anomaly_gives_normal_fields():
    m = gs.make_model(2, 2, 2, 100.0, 100.0, np.array([0.0, 40.0, 100.0]), [0.0, 40.0],
                      [0.0, 0.03, 0.2], 1.0)
    E = gs.random_vector(np.random.default_rng(1), 2, 2, 2, 2)
    e, h = fields.fields_at(m, E, np.array([[50.0, 50.0]]))
    EN, HN = fields.surface_normal_fields(m)
    assert np.array_equal(e[:, 0], EN) and np.array_equal(h[:, 0], HN)


def test_half_space_impedance():
    # uniform earth: Z = [[0, Z], [-Z, 0]], Z = w mu0 / k (time factor exp(-i w t))
    sig, f = 0.05, 0.3
    m = gs.make_model(1, 1, 1, 100.0, 100.0, np.array([0.0, 100.0]), [0.0], [0.0, sig], f)
    EN, HN = fields.surface_normal_fields(m)
    Z = fields.impedance(EN[:, None, :], HN[:, None, :])[0]
    w = 2 * np.pi * f
    k = np.sqrt(1j * w * MU0 * sig)
    zc = w * MU0 / k
    assert abs(Z[0, 0]) < 1e-14 and abs(Z[1, 1]) < 1e-14
    assert abs(Z[0, 1] - zc) <= 1e-12 * abs(zc) and abs(Z[1, 0] + zc) <= 1e-12 * abs(zc)


@pytest.mark.parametrize("z0", [25.0, 170.0])
def test_receiver_kernels_whole_space_at_depth(z0):
    # receivers inside the earth above the anomaly grid (z0 = 25 m, grid from
    # 50 m to 140 m) and below it (170 m): the cell integrals of G^E and G^H
    # against the closed form
    sig, f = 0.02, 3.0
    m = dict(nx=3, ny=3, nz=2, hx=100.0, hy=120.0, z_edges=np.array([50.0, 90.0, 140.0]),
             d=np.array([0.0]), sigma=np.array([sig, sig], complex), freq=f)
    offs = np.array([[0.0, 0.0], [100.0, 0.0], [0.0, 120.0], [230.0, -70.0]])
    KE, KH = fields.receiver_kernels(m, offs, z0=z0)
    for k, (dx, dy) in enumerate(offs):
        for jz in range(2):
            lo = [-50.0, -60.0, m["z_edges"][jz]]
            hi = [50.0, 60.0, m["z_edges"][jz + 1]]
            # 25-30 m from a 100 m face the closed form's Gauss rule needs 48
            # points per axis to reach 1e-12
            E, H = wholespace.point_box([dx, dy, z0], lo, hi, sig, f, q=48)
            assert np.abs(KE[k, jz] - E).max() <= 1e-8 * np.abs(E).max()
            assert np.abs(KH[k, jz] - H).max() <= 1e-8 * np.abs(H).max()


def test_normal_fields_at_depth_half_space():
    # uniform earth: E = exp(i k z), H_y = (k / (w mu0)) exp(i k z)
    sig, f = 0.05, 0.3
    m = gs.make_model(1, 1, 1, 100.0, 100.0, np.array([0.0, 100.0]), [0.0], [0.0, sig], f)
    w = 2 * np.pi * f
    k = np.sqrt(1j * w * MU0 * sig)
    for z0 in (0.0, 37.0, 400.0):
        EN, HN = fields.normal_fields_at(m, z0)
        e, hy = np.exp(1j * k * z0), k / (w * MU0) * np.exp(1j * k * z0)
        assert abs(EN[0, 0] - e) <= 1e-13 and abs(EN[1, 1] - e) <= 1e-13
        assert abs(HN[0, 1] - hy) <= 1e-13 * abs(hy) and abs(HN[1, 0] + hy) <= 1e-13 * abs(hy)
    EN, HN = fields.normal_fields_at(m, 0.0)
    ES, HS = fields.surface_normal_fields(m)
    assert np.allclose(EN, ES, rtol=0, atol=1e-15) and np.allclose(HN, HS, rtol=1e-14, atol=0)


def _dipole_response(m, B, src, comps, rec, z0, transpose=True):
    """Anomalous E at rec from unit dipoles of components comps at src, one
    right-hand side each (the oracle's dense solve of the scaled system):
    array [len(comps)][3]."""
    p = np.zeros((len(comps), 3), complex)
    p[np.arange(len(comps)), list(comps)] = 1.0
    if transpose:
        u0 = fields.dipole_source(m, [src] * len(comps), p, z0=z0)
    else:
        # a plausible mistake: the receiver kernel used without transposing
        nx, ny, nz = m["nx"], m["ny"], m["nz"]
        cx = m["x0"] + (np.arange(nx) + 0.5) * m["hx"]
        cy = m["y0"] + (np.arange(ny) + 0.5) * m["hy"]
        offs = np.array([(src[0] - a, src[1] - b) for b in cy for a in cx])
        KE, _ = fields.receiver_kernels(m, offs, z0=z0)
        KE = KE.reshape(ny, nx, nz, 3, 3)
        vol = m["hx"] * m["hy"] * np.diff(m["z_edges"])
        sb = m["sigma"][m["layer_of_cell"]]
        u0 = (np.sqrt(sb.real)[None, None, :, None, None]
              * np.einsum("yxzcr,sr->sczyx", KE, p) / vol[None, None, :, None, None])
    d = dense.cie_diagonals(m)
    u = dense.solve_lu(dense.system_matrix(B, d), u0)
    E = u / d["a"][None, None]
    e, _ = fields.fields_at(m, E, np.array([rec]), z0=z0, normal=False)
    return e[:, 0]


@pytest.mark.parametrize("z0,comps", [(25.0, (0, 1, 2)), (0.0, (0, 1)), (170.0, (0, 1, 2))])
def test_dipole_source_reciprocity(z0, comps):
    # the anomalous response of the discretised problem is reciprocal:
    # E^a_i(A; unit dipole j at B) = E^a_j(B; unit dipole i at A), for sources
    # and receivers on the lattice above the grid (z0 = 25 m over a grid from
    # 50 m: every component; at the surface of an insulating air the vertical
    # ones are earth-side values and only the horizontal ones are compared;
    # z0 = 170 m below the grid, in the second layer: every component); the
    # untransposed kernel breaks it
    from oracle import tables
    rng = np.random.default_rng(77)
    nx, ny, nz = 3, 3, 2
    m = gs.make_model(nx, ny, nz, 100.0, 120.0, np.array([50.0, 90.0, 140.0]), [0.0, 90.0],
                      [0.0, 0.02, 0.004], 1.0)
    m["sigma_a"] = m["sigma_a"] * 10 ** rng.uniform(0.5, 2.0, m["sigma_a"].shape)
    B = dense.dense_from_packed(tables.pack(tables.build_tables(m), nx, ny, nz), m)
    A, Bp = (50.0, 60.0), (250.0, 180.0)
    resp_ab = _dipole_response(m, B, Bp, comps, A, z0)     # [j][i]
    resp_ba = _dipole_response(m, B, A, comps, Bp, z0)     # [i][j]
    M1 = resp_ab[:, list(comps)]          # [j, i] = E_i(A; j at B)
    M2 = resp_ba[:, list(comps)].T        # [j, i] = E_j(B; i at A)
    scale = np.abs(M1).max()
    assert scale > 0 and np.abs(M1 - M2).max() <= 1e-9 * scale, (M1, M2)
    if z0 > 0:
        bad_ab = _dipole_response(m, B, Bp, comps, A, z0, transpose=False)
        bad_ba = _dipole_response(m, B, A, comps, Bp, z0, transpose=False)
        W1, W2 = bad_ab[:, list(comps)], bad_ba[:, list(comps)].T
        assert np.abs(W1 - W2).max() > 1e-3 * np.abs(W1).max()
