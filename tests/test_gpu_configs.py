"""The larger workloads on tables from giem_tables:
  - 256 x 256 x 32 cells of 100 x 100 x 50 m (padded transforms of 512
    points): the FP64 apply at sampled cells against the oracle's direct sum
    on the exported table, and the precision form (complex64 operator and
    Krylov basis, FP64 refinement) against an FP64 solve at 1e-12;
  - three models of uneven size, 64 x 64 x 16, 96 x 96 x 24 (padded length
    192 needs a radix-3 pass) and 128 x 128 x 32, each at twelve frequencies
    1e-3 .. 10 Hz: the precision form against the FP64 solve at every
    frequency.
The precision form runs to 1e-9 so that its error, not the tolerance of the
comparison, is measured; the bar is 1e-6 relative per polarisation."""
import time

import numpy as np
import pytest

import giem_synth as gs
from oracle import dense, packed
from tests.gpu_util import rel_err, to_dev

pytestmark = pytest.mark.gpu


def _pair(lib, h, sa, shape, ifreq):
    import torch
    E64 = torch.zeros((2,) + shape, dtype=torch.complex128, device="cuda")
    s64 = h.solve(sa, E64, tol=1e-12, restart=30, max_iter=40000, ifreq=ifreq)
    E32 = torch.zeros_like(E64)
    s32 = h.solve(sa, E32, tol=1e-9, restart=30, max_iter=40000, precision=lib.FP32,
                  inner_tol=1e-3, max_outer=60, ifreq=ifreq)
    assert s64["converged"] == 1 and s32["converged"] == 1, (s64, s32)
    errs = [float(torch.linalg.vector_norm(E32[p] - E64[p]) / torch.linalg.vector_norm(E64[p]))
            for p in range(2)]
    return errs, s64, s32


def test_precision_256(lib):
    import torch
    m = gs.config_precision()
    nx, ny, nz = m["nx"], m["ny"], m["nz"]
    t0 = time.perf_counter()
    h = lib.tables(m, [m["freq"]], flags=lib.TABLES_C64)
    sa = to_dev(m["sigma_a"])
    shape = h.tune(sa)
    print(f"256x256x32: tables + tuning {time.perf_counter() - t0:.1f} s, shapes {shape}", flush=True)
    # FP64 apply at sampled cells against the oracle on the exported table
    rng = np.random.default_rng(303)
    x = gs.random_vector(rng, 2, nz, ny, nx)
    xd = to_dev(x)
    yd = torch.empty_like(xd)
    h.apply(xd, yd, sa, mode=lib.MODE_A)
    torch.cuda.synchronize()
    y = yd.cpu().numpy()
    tab = h.export(0)
    cells = [(0, 0, 0), (nz - 1, ny - 1, nx - 1), (nz // 2, 17, 200), (3, ny - 1, 0)]
    ref = dense.apply_cells(lambda iz: packed.tensor_row(tab, nz, iz), m, x, cells, "A")
    got = np.stack([y[:, :, iz, iy, ix] for (iz, iy, ix) in cells], 1)
    ea = rel_err(got, ref)
    del tab
    print(f"  sampled FP64 apply vs oracle: {ea:.2e}", flush=True)
    assert ea <= 1e-10
    errs, s64, s32 = _pair(lib, h, sa, (3, nz, ny, nx), 0)
    h.close()
    print(f"  precision form vs FP64: {errs[0]:.2e} {errs[1]:.2e}; FP64 {s64['iters']} it "
          f"{s64['ms']:.0f} ms, FP32-refined {s32['iters']} inner / {s32['outer_iters']} outer "
          f"{s32['ms']:.0f} ms", flush=True)
    assert max(errs) <= 1e-6


@pytest.mark.parametrize("which", [0, 1, 2])
def test_batched_models_and_frequencies(lib, which):
    models, freqs = gs.config_batched()
    m = models[which]
    nx, ny, nz = m["nx"], m["ny"], m["nz"]
    t0 = time.perf_counter()
    h = lib.tables(m, freqs, flags=lib.TABLES_C64)
    sa = to_dev(m["sigma_a"])
    h.tune(sa)
    print(f"{nx}x{ny}x{nz}: tables for {len(freqs)} frequencies + tuning "
          f"{time.perf_counter() - t0:.1f} s", flush=True)
    worst = 0.0
    for q in range(len(freqs)):
        errs, s64, s32 = _pair(lib, h, sa, (3, nz, ny, nx), q)
        worst = max(worst, max(errs))
        print(f"  f = {freqs[q]:.4g} Hz: err {max(errs):.2e}, FP64 {s64['iters']} it "
              f"{s64['ms']:.0f} ms, FP32-refined {s32['iters']} it {s32['ms']:.0f} ms", flush=True)
        assert max(errs) <= 1e-6, (freqs[q], errs)
    h.close()
    print(f"  worst {worst:.2e}", flush=True)
