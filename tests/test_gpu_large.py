"""The paper's benchmark model on one GPU (Sect. 4, Table commemi_table):
176 x 224 x 118 cubes of 25 m from z = 50 m (4.65 M cells, 14 M unknowns per
right-hand side, two plane-wave sources at 1 Hz), seven blocks of contrast up
to 3.3e4, tables from giem_tables (35 GB of FP64 spectra plus a complex64
copy).  Only internal checks are possible at this size:
  - the FP64 apply at sampled cells against the oracle's direct sum on the
    exported table (band-pair block-product kernel, 352-point transforms with a
    radix-11 pass, 448-point transforms);
  - the precision form against the FP64 solve (both GMRES(60) to 1e-7);
  - sigma_a = sigma_b (A = I) returns the normal field in one Arnoldi step,
    and the impedance at the surface (over the grid, which starts at 50 m)
    is then the 1-D surface impedance of the background;
  - apparent resistivity and phase along a surface profile across the blocks
    (the quantity of the paper's maps), finite and positive."""
import time

import numpy as np
import pytest

import giem_synth as gs
from oracle import dense, normal_field, packed
from oracle.fundamental import MU0
from tests.gpu_util import rel_err, to_dev

pytestmark = pytest.mark.gpu


def test_large_grid(lib):
    import torch
    m = gs.config_commemi3d3()
    nx, ny, nz = m["nx"], m["ny"], m["nz"]
    t0 = time.perf_counter()
    h = lib.tables(m, [m["freq"]], flags=lib.TABLES_C64)
    sa = to_dev(m["sigma_a"])
    print(f"{nx}x{ny}x{nz}: tables {time.perf_counter() - t0:.1f} s", flush=True)

    # sampled FP64 apply against the oracle on the exported table
    rng = np.random.default_rng(707)
    x = gs.random_vector(rng, 2, nz, ny, nx)
    xd = to_dev(x)
    yd = torch.empty_like(xd)
    h.apply(xd, yd, sa, mode=lib.MODE_A)
    torch.cuda.synchronize()
    cells = [(0, 0, 0), (nz - 1, ny - 1, nx - 1), (60, 101, 33)]
    got = np.stack([yd[:, :, iz, iy, ix].cpu().numpy() for (iz, iy, ix) in cells], 1)
    del yd, xd
    tab = h.export(0)
    ref = dense.apply_cells(lambda iz: packed.tensor_row(tab, nz, iz), m, x, cells, "A")
    del tab
    ea = rel_err(got, ref)
    print(f"  sampled FP64 apply vs oracle: {ea:.2e}", flush=True)
    assert ea <= 1e-10

    # precision form against FP64, GMRES(60) to 1e-7 (contrast 3.3e4: about
    # 1,800 steps); solved in chunks of warm-started calls so that every
    # chunk reports its residual
    shape = (2, 3, nz, ny, nx)

    def chunked(prec, E):
        done, t = 0, time.perf_counter()
        while True:
            st = h.solve(sa, E, tol=1e-7, restart=60, max_iter=600, precision=prec,
                         warm_start=1 if done else 0, max_outer=40)
            done += st["iters"]
            print(f"    prec {prec}: {done} steps, residual {st['rel_residual']:.2e}, "
                  f"{time.perf_counter() - t:.1f} s", flush=True)
            if st["converged"] or done >= 6000:
                return st, done, time.perf_counter() - t

    E64 = torch.zeros(shape, dtype=torch.complex128, device="cuda")
    s64, n64, t64 = chunked(lib.FP64, E64)
    E32 = torch.zeros_like(E64)
    s32, n32, t32 = chunked(lib.FP32, E32)
    assert s64["converged"] == 1 and s32["converged"] == 1, (s64, s32)
    errs = [float(torch.linalg.vector_norm(E32[p] - E64[p]) / torch.linalg.vector_norm(E64[p]))
            for p in range(2)]
    print(f"  FP64 to 1e-7: {n64} steps {t64:.1f} s; FP32-refined: {n32} inner steps "
          f"{t32:.1f} s; difference {errs[0]:.1e} {errs[1]:.1e}", flush=True)
    assert max(errs) <= 1e-5
    del E32

    # surface profile across the blocks at y = 2.8 km: Z and rho_a, phase
    w = 2 * np.pi * m["freq"]
    sites = np.array([[(ix + 0.5) * m["hx"], (ny // 2 + 0.5) * m["hy"], 0.0]
                      for ix in range(10, nx, 20)])
    t1 = time.perf_counter()
    Er = torch.empty((2, len(sites), 3), dtype=torch.complex128, device="cuda")
    Hr = torch.empty_like(Er)
    h.fields(sa, E64, sites, Er, Hr)
    Z = torch.empty((len(sites), 2, 2), dtype=torch.complex128, device="cuda")
    lib.impedance(Er, Hr, Z)
    torch.cuda.synchronize()
    z = Z.cpu().numpy()
    rho = np.abs(z[:, 0, 1]) ** 2 / (w * MU0)
    phase = np.degrees(np.angle(z[:, 0, 1]))
    print(f"  surface profile (receiver kernels + fields {time.perf_counter() - t1:.1f} s): "
          + ", ".join(f"{x / 1e3:.2f} km {r:.0f} ohm m {p:.0f} deg"
                      for x, r, p in zip(sites[:, 0], rho, phase)), flush=True)
    assert np.isfinite(z).all() and (rho > 0).all()

    # no anomaly: the normal field
    sb = m["sigma"][m["layer_of_cell"]][:, None, None] * np.ones(m["sigma_a"].shape)
    E64.zero_()
    st = h.solve(to_dev(sb), E64, tol=1e-12)
    en = normal_field.normal_field_cells(m)
    assert st["iters"] <= 1   # A = I: one Arnoldi step from x = 0
    assert rel_err(E64.cpu().numpy(), en) <= 1e-12
    sb_d = to_dev(sb)
    h.fields(sb_d, E64, sites, Er, Hr)
    lib.impedance(Er, Hr, Z)
    torch.cuda.synchronize()
    zs = normal_field.LayeredPlaneWave(m["d"], m["sigma"], m["freq"]).Zs
    z = Z.cpu().numpy()
    assert np.abs(z[:, 0, 1] - zs).max() <= 1e-10 * abs(zs)
    assert np.abs(z[:, 1, 0] + zs).max() <= 1e-10 * abs(zs)
    h.close()
