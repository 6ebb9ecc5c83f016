"""GPU parity of the GMRES solve (Sect. 2.2 system, Sect. 3.3 solver) with the
oracle's dense LU on the same packed table, the precision form, the adjoint
gradient, and the failure paths."""
import numpy as np
import pytest

import giem_synth as gs
from oracle import dense, normal_field
from tests.gpu_util import random_model, rel_err, to_dev

pytestmark = pytest.mark.gpu


def _conditioned_case(nx, ny, nz, seed, contrast=1.0):
    """Random packed table scaled so that ||R1 B R2|| is about 0.2 (condition
    number about 6; the random table is not a contracting operator, so the
    contrast is kept moderate)."""
    rng = np.random.default_rng(seed)
    m = random_model(nx, ny, nz, seed, contrast=contrast)
    t = gs.random_packed_table(rng, nx, ny, nz, decay=0.2)
    d = dense.cie_diagonals(m)
    n3 = 3 * nx * ny * nz
    scale = 0.2 / (np.abs(d["R1"]).max() * np.abs(d["R2"]).max() * 2 * np.sqrt(n3))
    return m, t * scale, rng


def _oracle_E(m, t, rhs_u):
    B = dense.dense_from_packed(t, m)
    d = dense.cie_diagonals(m)
    A = dense.system_matrix(B, d)
    u = dense.solve_lu(A, rhs_u)
    a = d["a"][None, None]
    return u / a


@pytest.mark.parametrize("nx,ny,nz", [(4, 3, 2), (15, 7, 3), (16, 16, 4)])
def test_solve_fp64_matches_lu(lib, nx, ny, nz):
    import torch
    m, t, rng = _conditioned_case(nx, ny, nz, 11 + nx)
    rhs = gs.random_vector(rng, 2, nz, ny, nx)
    ref = _oracle_E(m, t, rhs)
    h = lib.tables_import(m, [m["freq"]], t[None])
    E = torch.empty((2, 3, nz, ny, nx), dtype=torch.complex128, device="cuda")
    st = h.solve(to_dev(m["sigma_a"]), E, rhs=to_dev(rhs), tol=1e-13, restart=30, max_iter=3000)
    assert st["converged"] == 1, st
    err = rel_err(E.cpu().numpy(), ref)
    assert err <= 1e-10, (err, st)
    h.close()


def _second_pass_case():
    """sigma_a = 3 sigma_b in every cell (S = I/2) and a table scaled to a few
    percent of S: every Arnoldi step repeats the Gram-Schmidt pass."""
    nx, ny, nz = 6, 5, 3
    rng = np.random.default_rng(321)
    m = random_model(nx, ny, nz, 321, contrast=0.0)
    m["sigma_a"] = 3.0 * m["sigma_a"]
    t = gs.random_packed_table(rng, nx, ny, nz, decay=0.2)
    d = dense.cie_diagonals(m)
    n3 = 3 * nx * ny * nz
    t = t * (0.04 / (np.abs(d["R1"]).max() * np.abs(d["R2"]).max() * 2 * np.sqrt(n3)))
    return m, t, rng


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_second_gram_schmidt_pass(lib, prec):
    # sigma_a = 3 sigma_b in every cell makes S = I/2, and the table is
    # scaled so that R1 B R2 is a few percent of it: each new Krylov vector
    # is nearly parallel to the last, the projection removes more than 99.9%
    # of its squared norm (checked below on the oracle's matrix), and every
    # Arnoldi step takes the second Gram-Schmidt pass, which discards the
    # apply already queued for the next step and redoes it.
    import torch
    m, t, rng = _second_pass_case()
    nz, ny, nx = m["sigma_a"].shape
    d = dense.cie_diagonals(m)
    assert np.allclose(d["S"], 0.5)
    rhs = gs.random_vector(rng, 2, nz, ny, nx)
    A = dense.system_matrix(dense.dense_from_packed(t, m), d)
    for r in range(2):
        V = [rhs[r].reshape(-1) / np.linalg.norm(rhs[r])]
        for _ in range(4):
            w = A @ V[-1]
            Q = np.stack(V, 1)
            res = w - Q @ (Q.conj().T @ w)
            assert np.vdot(res, res).real < 1e-3 * np.vdot(w, w).real
            V.append(res / np.linalg.norm(res))
    ref = _oracle_E(m, t, rhs)
    h = lib.tables_import(m, [m["freq"]], t[None], flags=lib.TABLES_C64)
    E = torch.empty((2, 3, nz, ny, nx), dtype=torch.complex128, device="cuda")
    if prec == "fp64":
        st = h.solve(to_dev(m["sigma_a"]), E, rhs=to_dev(rhs), tol=1e-13, restart=30,
                     max_iter=100)
        assert st["iters"] >= 5, st
        bar = 1e-10
    else:
        # the complex64 inner solves of the precision form take the same
        # second passes
        st = h.solve(to_dev(m["sigma_a"]), E, rhs=to_dev(rhs), tol=1e-10, precision=lib.FP32,
                     inner_tol=1e-4, max_iter=200)
        bar = 1e-8
    assert st["converged"] == 1, st
    err = rel_err(E.cpu().numpy(), ref)
    assert err <= bar, (err, st)
    h.close()


@pytest.mark.parametrize("case", ["plain", "second_pass"])
def test_profile_counts_only_used_applies(lib, case):
    # GMRES queues each step's apply before the host has finished the step
    # before; the profile counts every launch in "applies" but in "rhs" only
    # the right-hand sides whose results were used: one per Arnoldi step and
    # one residual per cycle (the first cycle starts from x = 0)
    import torch
    if case == "plain":
        m, t, rng = _conditioned_case(8, 6, 3, 17)
    else:
        m, t, rng = _second_pass_case()
    nz, ny, nx = m["sigma_a"].shape
    rhs = gs.random_vector(rng, 1, nz, ny, nx)
    h = lib.tables_import(m, [m["freq"]], t[None])
    E = torch.empty((1, 3, nz, ny, nx), dtype=torch.complex128, device="cuda")
    h.profile(True)
    st = h.solve(to_dev(m["sigma_a"]), E, rhs=to_dev(rhs), tol=1e-12, restart=30, max_iter=500)
    p = h.profile_read()["fp64"]
    h.profile(False)
    assert st["converged"] == 1, st
    assert p["rhs"] == st["iters"] + st["outer_iters"], (p, st)
    assert p["applies"] > p["rhs"], (p, st)     # at least the apply queued at convergence
    assert rel_err(E.cpu().numpy(), _oracle_E(m, t, rhs)) <= 1e-10
    h.close()


def test_plane_wave_rhs_matches_oracle(lib):
    import torch
    nx, ny, nz = 8, 6, 3
    m, t, _ = _conditioned_case(nx, ny, nz, 5)
    ref = _oracle_E(m, t, normal_field.plane_wave_rhs(m))
    h = lib.tables_import(m, [m["freq"]], t[None])
    E = torch.empty((2, 3, nz, ny, nx), dtype=torch.complex128, device="cuda")
    st = h.solve(to_dev(m["sigma_a"]), E, tol=1e-13)
    assert st["converged"] == 1
    assert rel_err(E.cpu().numpy(), ref) <= 1e-10
    h.close()


def test_no_anomaly_returns_normal_field(lib):
    import torch
    nx, ny, nz = 6, 5, 3
    m, t, _ = _conditioned_case(nx, ny, nz, 6)
    sb = dense.cell_layer_sigma(m)[:, None, None] * np.ones((nz, ny, nx))
    h = lib.tables_import(m, [m["freq"]], t[None])
    E = torch.empty((2, 3, nz, ny, nx), dtype=torch.complex128, device="cuda")
    st = h.solve(to_dev(sb.astype(np.complex128)), E, tol=1e-12)
    en = normal_field.normal_field_cells(m)
    assert st["converged"] == 1 and st["iters"] <= 1
    assert rel_err(E.cpu().numpy(), en) <= 1e-14
    h.close()


def test_precision_form_refines_to_fp64(lib):
    import torch
    nx, ny, nz = 15, 7, 3
    m, t, rng = _conditioned_case(nx, ny, nz, 9)
    rhs = gs.random_vector(rng, 2, nz, ny, nx)
    ref = _oracle_E(m, t, rhs)
    h = lib.tables_import(m, [m["freq"]], t[None], flags=lib.TABLES_C64)
    E = torch.empty((2, 3, nz, ny, nx), dtype=torch.complex128, device="cuda")
    st = h.solve(to_dev(m["sigma_a"]), E, rhs=to_dev(rhs), tol=1e-10, precision=lib.FP32,
                 inner_tol=1e-4, max_iter=5000)
    assert st["converged"] == 1, st
    assert rel_err(E.cpu().numpy(), ref) <= 1e-8, st
    h.close()


def test_warm_start_and_weighted_product(lib):
    import torch
    nx, ny, nz = 8, 6, 3
    m, t, rng = _conditioned_case(nx, ny, nz, 12)
    rhs = gs.random_vector(rng, 1, nz, ny, nx)
    ref = _oracle_E(m, t, rhs)
    h = lib.tables_import(m, [m["freq"]], t[None])
    E = to_dev(ref * (1 + 1e-3))
    st = h.solve(to_dev(m["sigma_a"]), E, rhs=to_dev(rhs), tol=1e-13, warm_start=1, weighted_ip=1)
    assert st["converged"] == 1
    assert rel_err(E.cpu().numpy(), ref) <= 1e-10
    h.close()


def test_iteration_limit_reports_noconv(lib):
    import torch
    nx, ny, nz = 8, 6, 3
    m, t, rng = _conditioned_case(nx, ny, nz, 13)
    h = lib.tables_import(m, [m["freq"]], t[None])
    E = torch.empty((1, 3, nz, ny, nx), dtype=torch.complex128, device="cuda")
    rhs = to_dev(gs.random_vector(rng, 1, nz, ny, nx))
    st = h.solve(to_dev(m["sigma_a"]), E, rhs=rhs, tol=1e-15, max_iter=2, restart=2)
    assert st["rc"] == lib.GIEM_ENOCONV and st["converged"] == 0
    assert np.isfinite(E.cpu().numpy()).all()
    h.close()


def test_residual_history(lib):
    # giem_solve_stats.history: the true residual at the start of every
    # restart cycle (FP64; from x = 0 the first is 1) or after every
    # refinement step (precision form), the last equal to rel_residual; with
    # restarts the true residual of GMRES does not grow
    import torch
    nx, ny, nz = 8, 6, 3
    m, t, rng = _conditioned_case(nx, ny, nz, 15)
    h = lib.tables_import(m, [m["freq"]], t[None], flags=lib.TABLES_C64)
    sa = to_dev(m["sigma_a"])
    rhs = to_dev(gs.random_vector(rng, 2, nz, ny, nx))
    E = torch.empty((2, 3, nz, ny, nx), dtype=torch.complex128, device="cuda")
    st = h.solve(sa, E, rhs=rhs, tol=1e-12, restart=4, max_iter=3000)
    hist = st["history"]
    print(f"FP64 GMRES(4): {st['outer_iters']} cycles, history {len(hist)} entries "
          f"{hist[0]:.2e} .. {hist[-1]:.2e}", flush=True)
    assert st["converged"] == 1
    assert len(hist) == min(st["outer_iters"] + 1, 64)
    assert abs(hist[0] - 1.0) <= 1e-12
    assert hist[-1] == st["rel_residual"] and hist[-1] <= 1e-12
    assert all(b <= a * (1 + 1e-9) for a, b in zip(hist, hist[1:]))
    st = h.solve(sa, E, rhs=rhs, tol=1e-12, precision=lib.FP32, inner_tol=1e-3)
    hist = st["history"]
    print(f"precision form: {st['outer_iters']} refinement steps, history {hist}", flush=True)
    assert st["converged"] == 1 and len(hist) == st["outer_iters"] + 1
    assert hist[-1] == st["rel_residual"] and hist[-1] <= 1e-12
    assert all(b < a for a, b in zip(hist, hist[1:]))
    h.close()


def test_invalid_sigma_rejected(lib):
    import torch
    nx, ny, nz = 4, 3, 2
    m, t, _ = _conditioned_case(nx, ny, nz, 14)
    h = lib.tables_import(m, [m["freq"]], t[None])
    E = torch.empty((1, 3, nz, ny, nx), dtype=torch.complex128, device="cuda")
    sa = m["sigma_a"].copy()
    sa[0, 0, 0] = np.nan
    with pytest.raises(lib.GiemError) as e:
        h.solve(to_dev(sa), E)
    assert e.value.code == lib.GIEM_EINVAL
    sa = m["sigma_a"].copy()
    sa[1, 1, 1] = -1.0
    with pytest.raises(lib.GiemError) as e:
        h.solve(to_dev(sa), E)
    assert e.value.code == lib.GIEM_EDOMAIN
    h.close()


def test_adjoint_gradient_matches_oracle(lib):
    import torch
    nx, ny, nz = 6, 5, 3
    m, t, rng = _conditioned_case(nx, ny, nz, 15)
    g = gs.random_vector(rng, 2, nz, ny, nx)
    ref = dense.gradient_log_sigma(dense.dense_from_packed(t, m), m, g,
                                   normal_field.normal_field_cells(m))
    h = lib.tables_import(m, [m["freq"]], t[None])
    sa = to_dev(m["sigma_a"])
    E = torch.empty((2, 3, nz, ny, nx), dtype=torch.complex128, device="cuda")
    h.solve(sa, E, tol=1e-13)
    grad = torch.zeros((nz, ny, nx), dtype=torch.float64, device="cuda")
    st = h.adjoint(sa, to_dev(g), E, grad, tol=1e-13)
    assert st["converged"] == 1
    assert rel_err(grad.cpu().numpy(), ref) <= 1e-9
    h.close()
