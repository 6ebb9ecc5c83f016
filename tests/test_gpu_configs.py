"""The larger workloads on tables from giem_tables:
  - 256 x 256 x 32 cells of 100 x 100 x 50 m (padded transforms of 512
    points): the FP64 apply at sampled cells against the oracle's direct sum
    on the exported table, and the precision form (complex64 operator and
    Krylov basis, FP64 refinement) against an FP64 solve at 1e-12;
  - the lockstep solver of several frequencies of one model against the
    oracle and against separate solves (the three-model, twelve-frequency
    set is in test_gpu_graph.py).
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


def test_batched_solve_matches_oracle(lib):
    # three frequencies of a small model solved together, each against the
    # oracle's LU on its exported table
    import torch
    from oracle import normal_field
    rng = np.random.default_rng(404)
    m = gs.make_model(6, 5, 3, 100.0, 120.0, np.arange(4) * 50.0, [0.0, 100.0, 900.0],
                      [0.0, 0.02, 0.2, 0.004], 1.0)
    m["sigma_a"] = m["sigma_a"] * 10 ** rng.uniform(0, 2, m["sigma_a"].shape)
    freqs = [0.1, 1.0, 10.0]
    h = lib.tables(m, freqs, flags=lib.TABLES_C64)
    sa = to_dev(m["sigma_a"])
    Es = [torch.zeros((2, 3, 3, 5, 6), dtype=torch.complex128, device="cuda") for _ in freqs]
    st = h.solve_batch(sa, Es, tol=1e-13, max_iter=4000)
    E32 = [torch.zeros_like(e) for e in Es]
    st32 = h.solve_batch(sa, E32, ifreqs=[2, 0, 1], tol=1e-12, precision=lib.FP32,
                         max_iter=8000, max_outer=60)
    torch.cuda.synchronize()
    for q, f in enumerate(freqs):
        assert st[q]["converged"] == 1 and st32[q]["converged"] == 1
        mf = dict(m, freq=f)
        d = dense.cie_diagonals(mf)
        A = dense.system_matrix(dense.dense_from_packed(h.export(q), mf), d)
        ref = dense.solve_lu(A, normal_field.plane_wave_rhs(mf)) / d["a"][None, None]
        e64 = rel_err(Es[q].cpu().numpy(), ref)
        e32 = rel_err(E32[[1, 2, 0][q]].cpu().numpy(), ref)
        print(f"  f = {f} Hz: batched FP64 {e64:.2e}, batched FP32-refined {e32:.2e}", flush=True)
        assert e64 <= 1e-10 and e32 <= 1e-9
    h.close()


def test_batched_solve_equals_separate_solves(lib):
    # the 64 x 64 x 16 model at its twelve frequencies: one lockstep solve
    # against twelve separate ones, and the wall time of both
    import torch
    models, freqs = gs.config_batched()
    m = models[0]
    shape = (2, 3, m["nz"], m["ny"], m["nx"])
    h = lib.tables(m, freqs, flags=lib.TABLES_C64)
    sa = to_dev(m["sigma_a"])
    h.tune(sa)
    for prec, name in ((lib.FP64, "FP64"), (lib.FP32, "FP32-refined")):
        sep = [torch.zeros(shape, dtype=torch.complex128, device="cuda") for _ in freqs]
        bat = [torch.zeros_like(e) for e in sep]
        kw = dict(tol=1e-8, max_iter=20000, precision=prec, max_outer=40)
        h.solve(sa, sep[0], ifreq=0, **kw)                 # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for q in range(len(freqs)):
            h.solve(sa, sep[q], ifreq=q, **kw)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st = h.solve_batch(sa, bat, **kw)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        assert all(s["converged"] == 1 for s in st)
        err = max(float(torch.linalg.vector_norm(b - a) / torch.linalg.vector_norm(a))
                  for a, b in zip(sep, bat))
        print(f"  {name}: 12 separate solves {1e3 * (t1 - t0):.0f} ms, one batched solve "
              f"{1e3 * (t2 - t1):.0f} ms ({(t1 - t0) / (t2 - t1):.2f}x); max difference {err:.1e}",
              flush=True)
        assert err <= 1e-7
    h.close()


def test_batched_solve_more_frequencies_than_one_launch(lib):
    # 18 frequencies: the applies of a step need two launches per kernel (at
    # most 16 frequencies share one); the batch must equal separate solves
    import torch
    rng = np.random.default_rng(405)
    m = gs.make_model(6, 5, 3, 100.0, 120.0, np.arange(4) * 50.0, [0.0, 100.0, 900.0],
                      [0.0, 0.02, 0.2, 0.004], 1.0)
    m["sigma_a"] = m["sigma_a"] * 10 ** rng.uniform(0, 2, m["sigma_a"].shape)
    freqs = list(np.logspace(-2, 1, 18))
    h = lib.tables(m, freqs)
    sa = to_dev(m["sigma_a"])
    shape = (2, 3, 3, 5, 6)
    bat = [torch.zeros(shape, dtype=torch.complex128, device="cuda") for _ in freqs]
    st = h.solve_batch(sa, bat, tol=1e-12, max_iter=4000)
    assert all(s["converged"] == 1 for s in st)
    worst = 0.0
    for q in range(len(freqs)):
        sep = torch.zeros(shape, dtype=torch.complex128, device="cuda")
        s1 = h.solve(sa, sep, tol=1e-12, max_iter=4000, ifreq=q)
        assert s1["converged"] == 1
        worst = max(worst, float(torch.linalg.vector_norm(bat[q] - sep) / torch.linalg.vector_norm(sep)))
    h.close()
    print(f"  18 frequencies: batched vs separate, worst {worst:.1e}", flush=True)
    assert worst <= 1e-12
