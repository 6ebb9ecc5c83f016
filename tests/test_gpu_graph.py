"""Graph-captured GMRES cycles (the Arnoldi step on the device, one host wait
per restart cycle) and the solve of several models together
(giem_solve_multi): against the oracle's LU, against the host-driven
lockstep solver, and on the batched workload of three models of uneven size
at twelve frequencies and both polarisations (72 systems)."""
import time

import numpy as np
import pytest

import giem_synth as gs
from oracle import dense, normal_field
from tests.gpu_util import component_errors, rel_err, to_dev

pytestmark = pytest.mark.gpu


def _small(seed, nx=6, ny=5, nz=3):
    rng = np.random.default_rng(seed)
    m = gs.make_model(nx, ny, nz, 100.0, 120.0, np.arange(nz + 1) * 50.0, [0.0, 100.0, 900.0],
                      [0.0, 0.02, 0.2, 0.004], 1.0)
    m["sigma_a"] = m["sigma_a"] * 10 ** rng.uniform(0, 2, m["sigma_a"].shape)
    return m


def _lu(h, m, q, f):
    mf = dict(m, freq=f)
    d = dense.cie_diagonals(mf)
    A = dense.system_matrix(dense.dense_from_packed(h.export(q), mf), d)
    return dense.solve_lu(A, normal_field.plane_wave_rhs(mf)) / d["a"][None, None]


def test_graph_solve_matches_lu(lib):
    import torch
    m = _small(501)
    freqs = [0.1, 1.0, 10.0]
    h = lib.tables(m, freqs, flags=lib.TABLES_C64)
    sa = to_dev(m["sigma_a"])
    shape = (2, 3, m["nz"], m["ny"], m["nx"])
    print("graph-captured GMRES, 6x5x3 at 3 frequencies", flush=True)
    for prec, tol, bar in ((lib.FP64, 1e-13, 1e-10), (lib.FP32, 1e-12, 1e-9)):
        Es = [torch.zeros(shape, dtype=torch.complex128, device="cuda") for _ in freqs]
        st = h.solve_batch(sa, Es, tol=tol, max_iter=8000, precision=prec, max_outer=60,
                           restart=20, graph=1)
        torch.cuda.synchronize()
        for q, f in enumerate(freqs):
            ref = _lu(h, m, q, f)
            err = rel_err(Es[q].cpu().numpy(), ref)
            cerr = component_errors(Es[q].cpu().numpy(), ref, (0, 1))
            print(f"  prec {prec} f = {f} Hz: {st[q]['iters']} steps, error {err:.2e}, "
                  f"worst component {cerr:.2e}", flush=True)
            assert st[q]["converged"] == 1 and err <= bar and cerr <= 10 * bar
    h.close()


def test_graph_equals_host_driven_and_second_pass(lib):
    # same iterates as the host-driven lockstep solver up to rounding, also
    # on a system whose every step repeats the Gram-Schmidt pass (sigma_a =
    # 3 sigma_b with a small table: S = I / 2 dominates)
    import torch
    for case in ("random", "second_pass"):
        m = _small(502, nx=8, ny=7, nz=3)
        rng = np.random.default_rng(503)
        t = gs.random_packed_table(rng, 8, 7, 3, decay=0.2)
        if case == "second_pass":
            m["sigma_a"] = 3.0 * gs.background_of_cells(m)[:, None, None] * np.ones_like(m["sigma_a"])
            t = t * 1e-3
        else:
            d = dense.cie_diagonals(m)
            t *= 0.3 / (np.abs(d["R1"]).max() * np.abs(d["R2"]).max() * 2 * np.sqrt(3 * 8 * 7 * 3))
        h = lib.tables_import(m, [m["freq"], 2 * m["freq"]], np.stack([t, 0.7 * t]))
        sa = to_dev(m["sigma_a"])
        rhs = [to_dev(gs.random_vector(rng, 2, 3, 7, 8)) for _ in range(2)]
        a = [torch.zeros_like(r) for r in rhs]
        b = [torch.zeros_like(r) for r in rhs]
        sa_ = h.solve_batch(sa, a, rhs=rhs, tol=1e-13, max_iter=4000, restart=12)
        sb_ = h.solve_batch(sa, b, rhs=rhs, tol=1e-13, max_iter=4000, restart=12, graph=1)
        torch.cuda.synchronize()
        diff = max(rel_err(x.cpu().numpy(), y.cpu().numpy()) for x, y in zip(a, b))
        print(f"  {case}: host-driven {sa_[0]['iters']} steps, graph {sb_[0]['iters']} steps, "
              f"difference {diff:.1e}", flush=True)
        assert all(s["converged"] == 1 for s in sa_ + sb_)
        assert diff <= 1e-10
        h.close()


def test_graph_many_systems_and_two_models(lib):
    # more systems of one handle than one Gram-Schmidt launch takes (12 > 8),
    # and two handles of different grids in one giem_solve_multi call, each
    # against the host-driven lockstep solver, FP64 and the precision form
    import torch
    ma = _small(504, nx=5, ny=4, nz=3)
    mb = _small(505, nx=7, ny=6, nz=2)
    fa = list(np.logspace(-1, 1, 6))
    fb = [0.3, 3.0]
    ha = lib.tables(ma, fa, flags=lib.TABLES_C64)
    hb = lib.tables(mb, fb, flags=lib.TABLES_C64)
    saa, sab = to_dev(ma["sigma_a"]), to_dev(mb["sigma_a"])
    za = (2, 3, ma["nz"], ma["ny"], ma["nx"])
    zb = (2, 3, mb["nz"], mb["ny"], mb["nx"])
    for prec, tol, bar in ((lib.FP64, 1e-12, 1e-10), (lib.FP32, 1e-11, 1e-9)):
        kw = dict(tol=tol, max_iter=20000, precision=prec, max_outer=60, restart=16)
        ra = [torch.zeros(za, dtype=torch.complex128, device="cuda") for _ in fa]
        rb = [torch.zeros(zb, dtype=torch.complex128, device="cuda") for _ in fb]
        ha.solve_batch(saa, ra, **kw)
        hb.solve_batch(sab, rb, **kw)
        ga = [torch.zeros_like(e) for e in ra]
        st1 = ha.solve_batch(saa, ga, graph=1, **kw)
        ea = max(rel_err(x.cpu().numpy(), y.cpu().numpy()) for x, y in zip(ga, ra))
        ma_ = [torch.zeros_like(e) for e in ra]
        mb_ = [torch.zeros_like(e) for e in rb]
        st2 = lib.solve_multi([(ha, saa, ma_, None, None), (hb, sab, mb_, None, None)], **kw)
        torch.cuda.synchronize()
        em = max(rel_err(x.cpu().numpy(), y.cpu().numpy()) for x, y in zip(ma_ + mb_, ra + rb))
        print(f"  prec {prec}: 12 systems of one handle (graph) vs host-driven {ea:.1e} "
              f"({st1[0]['iters']} steps); two handles {em:.1e} ({st2[0]['iters']} steps)",
              flush=True)
        assert all(s["converged"] == 1 for s in st1 + st2)
        assert ea <= bar and em <= bar
    ha.close()
    hb.close()


@pytest.fixture(scope="module")
def batched_set(lib):
    """The three models of uneven size at twelve frequencies (tables with
    their complex64 copies) and the FP64 reference of every system (tol
    1e-12, one host-driven batched solve per model)."""
    import torch
    models, freqs = gs.config_batched()
    out = []
    for m in models:
        t0 = time.perf_counter()
        h = lib.tables(m, freqs, flags=lib.TABLES_C64)
        sa = to_dev(m["sigma_a"])
        h.tune(sa)
        shape = (2, 3, m["nz"], m["ny"], m["nx"])
        ref = [torch.zeros(shape, dtype=torch.complex128, device="cuda") for _ in freqs]
        st = h.solve_batch(sa, ref, tol=1e-12, max_iter=60000)
        assert all(s["converged"] == 1 for s in st)
        print(f"{m['nx']}x{m['ny']}x{m['nz']}: tables, tuning and FP64 references "
              f"{time.perf_counter() - t0:.1f} s", flush=True)
        out.append((m, h, sa, ref))
    yield out, freqs
    for (_, h, _, _) in out:
        h.close()


def _pol_errors(Es, refs):
    return [rel_err(E[p].cpu().numpy(), R[p].cpu().numpy()) for E, R in zip(Es, refs)
            for p in range(2)]


@pytest.mark.parametrize("which", [0, 1, 2])
def test_batched_solve_each_model(lib, batched_set, which):
    # one lockstep solve per model at its twelve frequencies, FP64 and the
    # precision form, per polarisation against the FP64 references
    import torch
    sets, freqs = batched_set
    m, h, sa, ref = sets[which]
    shape = ref[0].shape
    for prec, name in ((lib.FP64, "FP64"), (lib.FP32, "FP32-refined")):
        Es = [torch.zeros(shape, dtype=torch.complex128, device="cuda") for _ in freqs]
        t0 = time.perf_counter()
        st = h.solve_batch(sa, Es, tol=1e-9, max_iter=60000, precision=prec, max_outer=60)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        errs = _pol_errors(Es, ref)
        print(f"  {m['nx']}x{m['ny']}x{m['nz']} {name} batched (tol 1e-9): {dt:.2f} s, "
              f"worst polarisation error {max(errs):.2e}", flush=True)
        assert all(s["converged"] == 1 for s in st)
        assert max(errs) <= 1e-6


def test_three_models_one_graph_sequence(lib, batched_set):
    # all 72 systems (3 models x 12 frequencies x 2 polarisations) in one
    # giem_solve_multi call, precision form, against the FP64 references;
    # wall time against the three per-model batched solves and 36 single
    # solves
    import torch
    sets, freqs = batched_set
    groups, outs = [], []
    for (m, h, sa, ref) in sets:
        Es = [torch.zeros(ref[0].shape, dtype=torch.complex128, device="cuda") for _ in freqs]
        outs.append(Es)
        groups.append((h, sa, Es, None, None))
    kw = dict(tol=1e-9, max_iter=60000, precision=lib.FP32, max_outer=60)
    lib.solve_multi(groups, **kw)            # warm-up (graph capture included)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = lib.solve_multi(groups, **kw)
    torch.cuda.synchronize()
    t_multi = time.perf_counter() - t0
    assert len(st) == 36 and all(s["converged"] == 1 for s in st)
    worst = 0.0
    for Es, (m, h, sa, ref) in zip(outs, sets):
        worst = max(worst, max(_pol_errors(Es, ref)))
    # the same systems per model (host-driven lockstep) and one by one
    t1 = time.perf_counter()
    for Es, (m, h, sa, ref) in zip(outs, sets):
        h.solve_batch(sa, Es, **kw)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t1
    t2 = time.perf_counter()
    for Es, (m, h, sa, ref) in zip(outs, sets):
        for q in range(len(freqs)):
            h.solve(sa, Es[q], ifreq=q, **kw)
    torch.cuda.synchronize()
    t_single = time.perf_counter() - t2
    worst_single = 0.0
    for Es, (m, h, sa, ref) in zip(outs, sets):
        worst_single = max(worst_single, max(_pol_errors(Es, ref)))
    print(f"  72 systems, precision form to 1e-9: one graph-captured sequence {t_multi:.2f} s, "
          f"three lockstep batches {t_batch:.2f} s, 36 separate solves {t_single:.2f} s; "
          f"worst polarisation error vs FP64 {worst:.2e} (separate solves {worst_single:.2e})",
          flush=True)
    assert worst <= 1e-6 and worst_single <= 1e-6
