"""Receivers in the earth above or below the anomaly grid and electric dipole sources
(Sect. 2.1, an external current as the source; Sect. 2.2, the field
representation through the cell integrals of G^E and G^H; Appendix A, the
reciprocity G^E(r, r') = G^E(r', r)^T), through the C ABI: against the
oracle's receiver kernels, normal fields and dipole right-hand sides, and
against the reciprocity of the anomalous response of the solved problem."""
import numpy as np
import pytest

import giem_synth as gs
from oracle import fields
from tests.gpu_util import component_errors, rel_err, to_dev

pytestmark = pytest.mark.gpu


def _buried(seed, nx=4, ny=3, freq=1.0):
    """A grid from 50 m to 140 m under the surface, cells in two layers."""
    rng = np.random.default_rng(seed)
    m = gs.make_model(nx, ny, 2, 100.0, 120.0, np.array([50.0, 90.0, 140.0]),
                      [0.0, 90.0, 600.0], [0.0, 0.02, 0.004, 0.1], freq)
    m["sigma_a"] = m["sigma_a"] * 10 ** rng.uniform(0.3, 1.5, m["sigma_a"].shape)
    return m, rng


def _lattice(m):
    return np.array([[(ix + 0.5) * m["hx"], (iy + 0.5) * m["hy"]]
                     for iy in range(m["ny"]) for ix in range(m["nx"])])


@pytest.mark.parametrize("z0", [0.0, 25.0, 50.0, 170.0])
def test_fields_at_depth_match_oracle(lib, z0):
    # the surface above a buried grid, a depth between them, the grid's top
    # face, and 30 m below the grid; normal fields of the plane wave at z0
    # included
    import torch
    m, rng = _buried(31)
    nx, ny, nz = m["nx"], m["ny"], m["nz"]
    E = gs.random_vector(rng, 2, nz, ny, nx)
    rec = _lattice(m)
    rxyz = np.concatenate([rec, np.full((len(rec), 1), z0)], 1)
    h = lib.tables(m, [m["freq"]])
    Er = torch.empty((2, len(rec), 3), dtype=torch.complex128, device="cuda")
    Hr = torch.empty_like(Er)
    h.fields(to_dev(m["sigma_a"]), to_dev(E), rxyz, Er, Hr)
    Ea, Ha = torch.empty_like(Er), torch.empty_like(Er)
    h.fields(to_dev(m["sigma_a"]), to_dev(E), rxyz, Ea, Ha, anomalous=True)
    torch.cuda.synchronize()
    h.close()
    e_ref, h_ref = fields.fields_at(m, E, rec, z0=z0)
    ea_ref, ha_ref = fields.fields_at(m, E, rec, z0=z0, normal=False)
    ee, eh = rel_err(Er.cpu().numpy(), e_ref), rel_err(Hr.cpu().numpy(), h_ref)
    ce = component_errors(Er.cpu().numpy(), e_ref, (0, 2))
    ch = component_errors(Hr.cpu().numpy(), h_ref, (0, 2))
    ca = component_errors(Ea.cpu().numpy(), ea_ref, (0, 2))
    print(f"z0 = {z0}: fields vs oracle E {ee:.2e} H {eh:.2e}, per component E {ce:.2e} "
          f"H {ch:.2e}, anomalous part {ca:.2e}", flush=True)
    assert ee <= 1e-9 and eh <= 1e-9
    assert ce <= 1e-8 and ch <= 1e-8 and ca <= 1e-8


@pytest.mark.parametrize("z0", [0.0, 25.0, 170.0])
def test_dipole_source_matches_oracle(lib, z0):
    import torch
    m, rng = _buried(32)
    nx, ny, nz = m["nx"], m["ny"], m["nz"]
    src = _lattice(m)[[0, 5, 11]]
    mom = rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3))
    h = lib.tables(m, [m["freq"]])
    rhs = torch.empty((3, 3, nz, ny, nx), dtype=torch.complex128, device="cuda")
    h.dipole_source(np.concatenate([src, np.full((3, 1), z0)], 1), mom, rhs)
    torch.cuda.synchronize()
    h.close()
    ref = fields.dipole_source(m, src, mom, z0=z0)
    err = rel_err(rhs.cpu().numpy(), ref)
    ce = component_errors(rhs.cpu().numpy(), ref, (0, 1))
    print(f"z0 = {z0}: dipole right-hand side vs oracle {err:.2e}, per source and "
          f"component {ce:.2e}", flush=True)
    assert err <= 1e-9 and ce <= 1e-8


@pytest.mark.parametrize("z0", [25.0, 170.0])
def test_dipole_source_reciprocity(lib, z0):
    # solve with dipole sources at A and at B (unit moments along x, y, z),
    # anomalous fields at the other point: E^a_i(A; j at B) = E^a_j(B; i at A)
    # (above the grid and below it)
    import torch
    m, rng = _buried(33, nx=8, ny=6, freq=2.0)
    nx, ny, nz = m["nx"], m["ny"], m["nz"]
    A = np.array([[150.0, 180.0, z0]])
    B = np.array([[650.0, 540.0, z0]])
    h = lib.tables(m, [m["freq"]])
    sa = to_dev(m["sigma_a"])

    def response(src, rec):
        rhs = torch.empty((3, 3, nz, ny, nx), dtype=torch.complex128, device="cuda")
        h.dipole_source(np.repeat(src, 3, 0), np.eye(3, dtype=complex), rhs)
        E = torch.zeros_like(rhs)
        st = h.solve(sa, E, rhs=rhs, tol=1e-13, restart=30, max_iter=4000)
        assert st["converged"] == 1, st
        Er = torch.empty((3, 1, 3), dtype=torch.complex128, device="cuda")
        h.fields(sa, E, rec, Er, torch.empty_like(Er), anomalous=True)
        torch.cuda.synchronize()
        return Er[:, 0].cpu().numpy()           # [source component][field component]

    M1 = response(B, A)          # [j][i] = E^a_i(A; j at B)
    M2 = response(A, B).T        # [j][i] = E^a_j(B; i at A)
    h.close()
    diff = np.abs(M1 - M2).max() / np.abs(M1).max()
    print(f"reciprocity of the anomalous response: {diff:.2e} (max |E^a| {np.abs(M1).max():.3e})",
          flush=True)
    assert diff <= 1e-8


def test_receivers_and_sources_rejected_outside_the_supported_set(lib):
    import torch
    m, rng = _buried(34)
    nx, ny, nz = m["nx"], m["ny"], m["nz"]
    h = lib.tables(m, [m["freq"]])
    sa = to_dev(m["sigma_a"])
    E = torch.zeros((1, 3, nz, ny, nx), dtype=torch.complex128, device="cuda")
    Er = torch.empty((1, 2, 3), dtype=torch.complex128, device="cuda")
    for bad in ([[50.0, 60.0, 0.0], [150.0, 60.0, 10.0]],     # two depths
                [[50.0, 60.0, 70.0], [150.0, 60.0, 70.0]],     # inside the grid
                [[50.0, 60.0, 140.0], [150.0, 60.0, 140.0]],   # on its bottom face
                [[50.0, 60.0, -5.0], [150.0, 60.0, -5.0]]):    # in the air
        with pytest.raises(lib.GiemError) as ex:
            h.fields(sa, E, np.array(bad), Er, Er.clone())
        assert ex.value.code == lib.GIEM_EDOMAIN
    rhs = torch.empty((9, 3, nz, ny, nx), dtype=torch.complex128, device="cuda")
    with pytest.raises(lib.GiemError) as ex:
        h.dipole_source(np.array([[50.0, 60.0, 0.0]] * 9), np.ones((9, 3)), rhs)
    assert ex.value.code == lib.GIEM_EINVAL
    with pytest.raises(lib.GiemError) as ex:
        h.dipole_source(np.array([[50.0, 60.0, 100.0]]), np.ones((1, 3)), rhs)
    assert ex.value.code == lib.GIEM_EDOMAIN
    h.close()
