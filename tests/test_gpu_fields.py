"""giem_fields (surface fields through the cell integrals of G^E and G^H)
against the oracle's independent receiver kernels, alone and after a solve."""
import numpy as np
import pytest

import giem_synth as gs
from oracle import dense, fields, normal_field
from tests.gpu_util import component_errors, rel_err, to_dev

pytestmark = pytest.mark.gpu


def _model(seed, nx=4, ny=3, nz=3, freq=1.0):
    rng = np.random.default_rng(seed)
    m = gs.make_model(nx, ny, nz, 100.0, 120.0, np.arange(nz + 1) * 40.0, [0.0, 80.0, 600.0],
                      [0.0, 0.02, 0.1, 0.005], freq)
    m["sigma_a"] = m["sigma_a"] * 10 ** rng.uniform(0, 1.5, m["sigma_a"].shape)
    return m, rng


def _centres(m, cells):
    return np.array([[(ix + 0.5) * m["hx"], (iy + 0.5) * m["hy"]] for (ix, iy) in cells])


def test_fields_match_oracle(lib):
    import torch
    m, rng = _model(21)
    nx, ny, nz = m["nx"], m["ny"], m["nz"]
    E = gs.random_vector(rng, 2, nz, ny, nx)
    rec = _centres(m, [(ix, iy) for iy in range(ny) for ix in range(nx)])
    h = lib.tables(m, [m["freq"]])
    Er = torch.empty((2, len(rec), 3), dtype=torch.complex128, device="cuda")
    Hr = torch.empty_like(Er)
    h.fields(to_dev(m["sigma_a"]), to_dev(E), rec, Er, Hr)
    torch.cuda.synchronize()
    h.close()
    e_ref, h_ref = fields.fields_at(m, E, rec)
    ee = rel_err(Er.cpu().numpy(), e_ref)
    eh = rel_err(Hr.cpu().numpy(), h_ref)
    # per RHS and field component ([nrhs][nrec][3])
    ce = component_errors(Er.cpu().numpy(), e_ref, (0, 2))
    ch = component_errors(Hr.cpu().numpy(), h_ref, (0, 2))
    print(f"fields vs oracle: E {ee:.2e}  H {eh:.2e}  per component E {ce:.2e}  H {ch:.2e}",
          flush=True)
    assert ee <= 1e-9 and eh <= 1e-9
    assert ce <= 1e-8 and ch <= 1e-8


def test_fields_after_solve_match_oracle(lib):
    # tables -> plane-wave solve -> surface fields, against the oracle's LU
    # solve on the exported table and its own receiver kernels
    import torch
    m, rng = _model(22, nx=5, ny=4, nz=3, freq=0.5)
    nx, ny, nz = m["nx"], m["ny"], m["nz"]
    h = lib.tables(m, [m["freq"]])
    E = torch.zeros((2, 3, nz, ny, nx), dtype=torch.complex128, device="cuda")
    st = h.solve(to_dev(m["sigma_a"]), E, tol=1e-13, restart=30, max_iter=3000)
    assert st["converged"] == 1
    rec = _centres(m, [(0, 0), (2, 1), (4, 3), (1, 2)])
    Er = torch.empty((2, len(rec), 3), dtype=torch.complex128, device="cuda")
    Hr = torch.empty_like(Er)
    h.fields(to_dev(m["sigma_a"]), E, rec, Er, Hr)
    torch.cuda.synchronize()
    t = h.export(0)
    h.close()
    d = dense.cie_diagonals(m)
    A = dense.system_matrix(dense.dense_from_packed(t, m), d)
    Eref = dense.solve_lu(A, normal_field.plane_wave_rhs(m)) / d["a"][None, None]
    e_ref, h_ref = fields.fields_at(m, Eref, rec)
    ee = rel_err(Er.cpu().numpy(), e_ref)
    eh = rel_err(Hr.cpu().numpy(), h_ref)
    ce = component_errors(Er.cpu().numpy(), e_ref, (0, 2))
    ch = component_errors(Hr.cpu().numpy(), h_ref, (0, 2))
    print(f"fields after solve: E {ee:.2e}  H {eh:.2e}  per component E {ce:.2e}  H {ch:.2e}",
          flush=True)
    assert ee <= 1e-9 and eh <= 1e-9
    assert ce <= 1e-8 and ch <= 1e-8
    # impedance from both polarisations
    Z = fields.impedance(Er.cpu().numpy(), Hr.cpu().numpy())
    Zr = fields.impedance(e_ref, h_ref)
    assert rel_err(Z, Zr) <= 1e-9


def test_fields_reject_receivers_off_centres(lib):
    import torch
    m, rng = _model(23)
    h = lib.tables(m, [m["freq"]])
    E = torch.zeros((1, 3, m["nz"], m["ny"], m["nx"]), dtype=torch.complex128, device="cuda")
    Er = torch.empty((1, 1, 3), dtype=torch.complex128, device="cuda")
    with pytest.raises(lib.GiemError) as ex:
        h.fields(to_dev(m["sigma_a"]), E, np.array([[10.0, 60.0]]), Er, Er.clone())
    assert ex.value.code == lib.GIEM_EDOMAIN
    # above a cell centre but inside the grid (which starts at the surface)
    with pytest.raises(lib.GiemError) as ex:
        h.fields(to_dev(m["sigma_a"]), E, np.array([[50.0, 60.0, 20.0]]), Er, Er.clone())
    assert ex.value.code == lib.GIEM_EDOMAIN
    # the same receiver on the surface, given as (x, y, z)
    h.fields(to_dev(m["sigma_a"]), E, np.array([[50.0, 60.0, 0.0]]), Er, Er.clone())
    h.close()
