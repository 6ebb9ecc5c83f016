"""The library's coefficient tables (giem_tables: Appendix B recursions,
Hankel transforms and horizontal quadratures, contracted on the GPU) against
the oracle's independent construction, and the whole physical chain (tables,
plane-wave source, GMRES) against a dense LU solve."""
import numpy as np
import pytest

import giem_synth as gs
from oracle import dense, normal_field, tables
from tests.gpu_util import component_errors, rel_err, to_dev

pytestmark = pytest.mark.gpu

# table accuracy bound, relative to the largest entry of each stored class
TAU_TAB = 1e-9

MODELS = {
    "whole_space": dict(nx=4, ny=3, nz=2, hx=100.0, hy=120.0, z_edges=np.array([0.0, 60.0, 100.0]),
                        d=np.array([0.0]), sigma=np.array([0.01, 0.01], complex), freq=1.0),
    "layered_air": dict(nx=3, ny=3, nz=3, hx=80.0, hy=110.0,
                        z_edges=np.array([0.0, 40.0, 100.0, 130.0]), d=np.array([0.0, 100.0]),
                        sigma=np.array([0.0, 0.02, 0.1], complex), freq=2.0),
    "contrast_1e4": dict(nx=3, ny=2, nz=3, hx=100.0, hy=100.0,
                         z_edges=np.array([0.0, 50.0, 100.0, 150.0]), d=np.array([0.0, 50.0]),
                         sigma=np.array([0.0, 1e-4, 1.0], complex), freq=0.01),
    # 240 offsets (several 64-column tiles of every spatial contraction and
    # of the spatial fold), uneven cells, three earth layers under the air
    # with interfaces between cells of the grid
    "several_tiles": dict(nx=20, ny=12, nz=5, hx=90.0, hy=70.0,
                          z_edges=np.array([0.0, 30.0, 70.0, 120.0, 180.0, 260.0]),
                          d=np.array([0.0, 70.0, 180.0]),
                          sigma=np.array([0.0, 0.05, 0.002, 0.3], complex), freq=3.0),
}


def _lib_model(m):
    return gs.make_model(m["nx"], m["ny"], m["nz"], m["hx"], m["hy"], m["z_edges"], m["d"],
                         m["sigma"], m["freq"])


def _class_errors(lib_t, ref_t, nz):
    T = nz * (nz + 1) // 2
    cuts = {"xx": (0, T), "xy": (T, 2 * T), "yy": (2 * T, 3 * T), "zz": (3 * T, 4 * T),
            "xz": (4 * T, 4 * T + nz * nz), "yz": (4 * T + nz * nz, 4 * T + 2 * nz * nz)}
    return {k: float(np.abs(lib_t[..., a:b] - ref_t[..., a:b]).max() / np.abs(ref_t[..., a:b]).max())
            for k, (a, b) in cuts.items()}


@pytest.mark.parametrize("name", list(MODELS))
def test_tables_match_oracle(lib, name):
    m = MODELS[name]
    print(f"tables {name}", flush=True)
    h = lib.tables(_lib_model(m), [m["freq"]])
    got = h.export(0)
    h.close()
    ref = tables.pack(tables.build_tables(m), m["nx"], m["ny"], m["nz"])
    errs = _class_errors(got, ref, m["nz"])
    print("  per-class errors", errs, flush=True)
    assert max(errs.values()) <= TAU_TAB, errs


def test_tables_whole_space_every_touching_pair(lib):
    # the library's tables alone against the whole-space reference built by
    # another route (difference-variable integrals with the second
    # derivatives moved onto the cell faces, Appendix A with one sigma):
    # all nine components of every self and touching pair, and separated
    # pairs at the first two offsets
    from oracle import packed, wholespace
    m = MODELS["whole_space"]
    h = lib.tables(_lib_model(m), [m["freq"]])
    q = packed.full_tensor_signed(h.export(0), m["nz"])
    h.close()
    ze, ny, nx = m["z_edges"], m["ny"], m["nx"]
    worst = 0.0
    for i in (-1, 0, 1, 2):
        for j in (-2, -1, 0, 1, 2):
            for iz in range(m["nz"]):
                for jz in range(m["nz"]):
                    lo_n = [j * m["hx"], i * m["hy"], ze[iz]]
                    hi_n = [(j + 1) * m["hx"], (i + 1) * m["hy"], ze[iz + 1]]
                    ref, _, _ = wholespace.cell_pair_any(lo_n, hi_n, [0.0, 0.0, ze[jz]],
                                                         [m["hx"], m["hy"], ze[jz + 1]],
                                                         m["sigma"][0].real, m["freq"], q=12)
                    got = q[i + ny - 1, j + nx - 1, :, :, iz, jz]
                    worst = max(worst, float(np.abs(got - ref).max() / np.abs(ref).max()))
    print(f"  worst pair error {worst:.3e}", flush=True)
    assert worst <= 1e-9, worst


def test_tables_whole_space_sum_rule(lib):
    # the library's tables alone, no oracle table: in a whole space whose
    # cells are five skin depths across, the coefficients of one observation
    # cell summed over all source cells give -V_n I / sigma (the Green's
    # tensor integrates to -I / sigma); the +-4-cell window leaves out terms
    # of order exp(-22).  Self and touching pairs carry most of the sum.
    from oracle import packed
    K = 4
    hz = np.array([90.0, 110.0, 95.0, 120.0, 100.0, 85.0, 115.0, 105.0, 92.0])
    hx, hy, sig = 100.0, 130.0, 0.5
    delta = min(hx, hy, hz.min()) / 5.0
    freq = 2.0 / (delta ** 2 * 4e-7 * np.pi * sig) / (2 * np.pi)
    m = dict(nx=K + 1, ny=K + 1, nz=hz.size, hx=hx, hy=hy,
             z_edges=np.concatenate([[0.0], np.cumsum(hz)]), d=np.array([0.0]),
             sigma=np.array([sig, sig], complex), freq=freq)
    h = lib.tables(_lib_model(m), [freq])
    t = h.export(0)
    h.close()
    B = packed.full_tensor_signed(t, m["nz"])           # [2Ny-1][2Nx-1][3][3][Nz][Nz]
    S = B[:, :, :, :, K, :].sum(axis=(0, 1, 4))
    dev = float(np.abs(S / (-hx * hy * hz[K] / sig) - np.eye(3)).max())
    print(f"  sum-rule deviation {dev:.3e}", flush=True)
    assert dev <= 1e-7, dev


def test_tables_air_limit(lib):
    # sigma_0 = 0 (the limit p = -1) against a tiny air conductivity
    m = dict(MODELS["layered_air"])
    h0 = lib.tables(_lib_model(m), [m["freq"]])
    t0 = h0.export(0)
    h0.close()
    m["sigma"] = np.array([1e-12, 0.02, 0.1], complex)
    h1 = lib.tables(_lib_model(m), [m["freq"]])
    t1 = h1.export(0)
    h1.close()
    errs = _class_errors(t1, t0, m["nz"])
    assert max(errs.values()) <= 1e-8, errs


def test_physical_solve_matches_lu(lib):
    # 16 x 16 x 4 model of contrast up to 1e3, plane-wave source: the library's
    # tables, exported and solved densely by LU, against giem_solve
    import torch
    m = gs.config_small()
    nx, ny, nz = m["nx"], m["ny"], m["nz"]
    print("physical solve 16x16x4", flush=True)
    h = lib.tables(m, [m["freq"]])
    t = h.export(0)
    B = dense.dense_from_packed(t, m)
    d = dense.cie_diagonals(m)
    A = dense.system_matrix(B, d)
    rhs = normal_field.plane_wave_rhs(m)
    ref = dense.solve_lu(A, rhs) / d["a"][None, None]
    E = torch.zeros((2, 3, nz, ny, nx), dtype=torch.complex128, device="cuda")
    st = h.solve(to_dev(m["sigma_a"]), E, tol=1e-13, restart=30, max_iter=4000)
    print("  stats", st, flush=True)
    assert st["converged"] == 1
    err = rel_err(E.cpu().numpy(), ref)
    # per polarisation and field component ([R][3][Nz][Ny][Nx])
    cerr = component_errors(E.cpu().numpy(), ref, (0, 1))
    print(f"  field rel err {err:.3e}, worst component {cerr:.3e}", flush=True)
    assert err <= 1e-10 and cerr <= 1e-9
    # the workload's own tolerance, 1e-8: the error it actually reaches
    E8 = torch.zeros_like(E)
    st8 = h.solve(to_dev(m["sigma_a"]), E8, tol=1e-8, restart=30, max_iter=4000)
    h.close()
    err8 = rel_err(E8.cpu().numpy(), ref)
    cerr8 = component_errors(E8.cpu().numpy(), ref, (0, 1))
    print(f"  at tol 1e-8: {st8['iters']} steps, residual {st8['rel_residual']:.2e}, "
          f"field error {err8:.3e}, worst component {cerr8:.3e}", flush=True)
    assert st8["converged"] == 1 and err8 <= 1e-6


@pytest.mark.parametrize("precision", ["fp64", "fp32_refined"])
def test_contrast_1e4_solve_matches_lu(lib, precision):
    # the generator of the 128 x 128 x 32 workload on an 8 x 8 x 6 grid, the
    # last block at contrast 1e4 (|gamma| close to 1, where GMRES works
    # hardest): library tables, plane-wave source, against dense LU
    import torch
    m = gs.config_layered(8, 8, 6, 200.0, 200.0, 100.0, 12, 0.01, side_xy=(3, 6),
                          side_z=(2, 4))
    nx, ny, nz = m["nx"], m["ny"], m["nz"]
    print(f"contrast 1e4 solve 8x8x6 {precision}, blocks {m['boxes']}", flush=True)
    h = lib.tables(m, [m["freq"]], flags=lib.TABLES_C64 if precision != "fp64" else 0)
    t = h.export(0)
    d = dense.cie_diagonals(m)
    A = dense.system_matrix(dense.dense_from_packed(t, m), d)
    print(f"  max |gamma| {np.abs(d['gamma']).max():.6f}", flush=True)
    ref = dense.solve_lu(A, normal_field.plane_wave_rhs(m)) / d["a"][None, None]
    E = torch.zeros((2, 3, nz, ny, nx), dtype=torch.complex128, device="cuda")
    kw = dict(tol=1e-13, restart=30, max_iter=20000)
    if precision != "fp64":
        kw.update(tol=1e-11, precision=lib.FP32)
    st = h.solve(to_dev(m["sigma_a"]), E, **kw)
    h.close()
    err = rel_err(E.cpu().numpy(), ref)
    cerr = component_errors(E.cpu().numpy(), ref, (0, 1))
    print(f"  stats {st}; field error {err:.3e}, worst component {cerr:.3e}", flush=True)
    assert st["converged"] == 1
    bar = 1e-10 if precision == "fp64" else 1e-8
    assert err <= bar and cerr <= 10 * bar
