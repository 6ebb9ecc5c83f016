"""A grid of the size of the paper's scalability workload on one GPU: 175 x
224 x 118 cubes of 25 m (4.6 M cells, 13.9 M unknowns per right-hand side,
two plane-wave sources), seven blocks of contrast up to 3.3e4, tables from
giem_tables (35 GB of FP64 spectra plus a complex64 copy).  Only internal
checks are possible at this size:
  - the FP64 apply at sampled cells against the oracle's direct sum on the
    exported table (gather block-product kernel, 350- and 448-point FFTs);
  - the precision form against the FP64 solve (both to 1e-8);
  - sigma_a = sigma_b (A = I) returns the normal field in one Arnoldi step."""
import time

import numpy as np
import pytest

import giem_synth as gs
from oracle import dense, normal_field, packed
from tests.gpu_util import rel_err, to_dev

pytestmark = pytest.mark.gpu


def test_large_grid(lib):
    import torch
    m = gs.config_large()
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

    # precision form against FP64
    shape = (2, 3, nz, ny, nx)
    E64 = torch.zeros(shape, dtype=torch.complex128, device="cuda")
    t1 = time.perf_counter()
    s64 = h.solve(sa, E64, tol=1e-8, max_iter=8000)
    t2 = time.perf_counter()
    E32 = torch.zeros_like(E64)
    s32 = h.solve(sa, E32, tol=1e-8, max_iter=8000, precision=lib.FP32, max_outer=60)
    t3 = time.perf_counter()
    assert s64["converged"] == 1 and s32["converged"] == 1, (s64, s32)
    errs = [float(torch.linalg.vector_norm(E32[p] - E64[p]) / torch.linalg.vector_norm(E64[p]))
            for p in range(2)]
    print(f"  FP64 to 1e-8: {s64['iters']} it {t2 - t1:.1f} s; FP32-refined: {s32['iters']} it "
          f"{s32['outer_iters']} outer {t3 - t2:.1f} s; difference {errs[0]:.1e} {errs[1]:.1e}",
          flush=True)
    assert max(errs) <= 1e-6
    del E32

    # no anomaly: the normal field
    sb = m["sigma"][m["layer_of_cell"]][:, None, None] * np.ones(m["sigma_a"].shape)
    E64.zero_()
    st = h.solve(to_dev(sb), E64, tol=1e-12)
    en = normal_field.normal_field_cells(m)
    assert st["iters"] <= 1   # A = I: one Arnoldi step from x = 0
    assert rel_err(E64.cpu().numpy(), en) <= 1e-12
    h.close()
