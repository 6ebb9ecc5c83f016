"""Impedance, its reverse mode and the misfit gradient through the C-ABI
(giem_impedance, giem_impedance_adjoint, giem_fields_adjoint, giem_adjoint,
driven by the torch.autograd wrapper) against the oracle's impedance and its
forward-sensitivity gradient, and at the full 64 x 64 x 16 size with four
frequencies and 1024 receivers against central differences of the misfit."""
import time

import numpy as np
import pytest

import giem_synth as gs
from oracle import fields, misfit
from tests.gpu_util import rel_err, to_dev

pytestmark = pytest.mark.gpu


def test_impedance_and_reverse_mode(lib):
    import torch
    rng = np.random.default_rng(61)
    nrec = 300
    E = gs.random_complex(rng, (2, nrec, 3))
    H = gs.random_complex(rng, (2, nrec, 3), 0.2)
    H[0, :, 1] += 2.0 + 1.0j        # keep Hh = [[Hx0 Hx1] [Hy0 Hy1]] well conditioned
    H[1, :, 0] -= 2.0 + 1.0j
    G = gs.random_complex(rng, (nrec, 2, 2))
    dE, dH = gs.random_complex(rng, E.shape), gs.random_complex(rng, H.shape)
    Ed, Hd, Gd = to_dev(E), to_dev(H), to_dev(G)
    Z = torch.empty((nrec, 2, 2), dtype=torch.complex128, device="cuda")
    lib.impedance(Ed, Hd, Z)
    wE, wH = torch.empty_like(Ed), torch.empty_like(Ed)
    lib.impedance_adjoint(Ed, Hd, Gd, wE, wH)
    torch.cuda.synchronize()
    Zr = fields.impedance(E, H)
    assert rel_err(Z.cpu().numpy(), Zr) <= 1e-13
    # Z is holomorphic in (E, H): central differences along a real step give
    # the directional derivative to O(t^2)
    t = 1e-5
    dZ = (fields.impedance(E + t * dE, H + t * dH) - fields.impedance(E - t * dE, H - t * dH)) / (2 * t)
    lhs = np.real(np.sum(np.conj(G) * dZ, axis=(1, 2)))
    w_e, w_h = wE.cpu().numpy(), wH.cpu().numpy()
    rhs = np.real(np.sum(w_e * dE + w_h * dH, axis=(0, 2)))
    assert np.abs(lhs - rhs).max() <= 1e-8 * np.abs(lhs).max()
    assert np.all(w_e[:, :, 2] == 0) and np.all(w_h[:, :, 2] == 0)


def _small(seed):
    rng = np.random.default_rng(seed)
    m = gs.make_model(4, 3, 3, 100.0, 120.0, np.arange(4) * 40.0, [0.0, 80.0, 600.0],
                      [0.0, 0.02, 0.1, 0.005], 1.0)
    m["sigma_a"] = (m["sigma_a"] * 10 ** rng.uniform(0, 1.5, m["sigma_a"].shape)).real + 0j
    return m, rng


def test_gradient_matches_oracle(lib):
    import torch
    from paper_1512_06126_amd.autograd import impedance_tensor
    m, rng = _small(62)
    freqs = [1.0, 0.1]
    rec = np.array([[50.0, 60.0], [250.0, 60.0], [150.0, 180.0], [350.0, 300.0], [50.0, 300.0]])
    h = lib.tables(m, freqs)
    ops = [misfit.operator(m, h.export(i), rec, f) for i, f in enumerate(freqs)]
    sobs = m["sigma_a"] * np.exp(0.2 * rng.standard_normal(m["sigma_a"].shape))
    _, Zobs = misfit.misfit(m, ops, sobs, 0.0)
    phi_ref, Zref = misfit.misfit(m, ops, m["sigma_a"], Zobs)
    g_ref = misfit.misfit_gradient(m, ops, m["sigma_a"], Zobs)
    ls = torch.tensor(np.log(m["sigma_a"].real), dtype=torch.float64, device="cuda",
                      requires_grad=True)
    Z = impedance_tensor(h, ls, rec, tol=1e-13)
    phi = (Z - to_dev(Zobs)).abs().pow(2).sum()
    phi.backward()
    torch.cuda.synchronize()
    h.close()
    ez = rel_err(Z.detach().cpu().numpy(), Zref)
    g = ls.grad.cpu().numpy()
    eg = np.abs(g - g_ref).max() / np.abs(g_ref).max()
    print(f"impedance {ez:.2e}, misfit {phi.item():.6e} vs {phi_ref:.6e}, gradient {eg:.2e}",
          flush=True)
    assert ez <= 1e-9
    assert abs(phi.item() - phi_ref) <= 1e-8 * phi_ref
    assert eg <= 1e-7


def test_gradient_full_size_finite_differences(lib):
    # 64 x 64 x 16 cells, four frequencies, 32 x 32 receivers: the gradient of
    # every cell from one forward and one adjoint solve per frequency, against
    # central differences (h = 1e-6 in log sigma, solves at 1e-13) on 50 cells
    import torch
    from paper_1512_06126_amd.autograd import impedance_tensor
    m, freqs, (rx, ry) = gs.config_gradient(seed=5)
    rec = np.array([(x, y) for y in ry for x in rx])
    nz, ny, nx = m["sigma_a"].shape
    t0 = time.perf_counter()
    h = lib.tables(m, freqs)
    ls0 = np.log(m["sigma_a"].real)
    lobs = ls0 + 0.1 * np.random.default_rng(55).standard_normal(ls0.shape)
    tol = 1e-13
    with torch.no_grad():
        Zobs = impedance_tensor(h, torch.tensor(lobs, device="cuda"), rec, tol=tol)
    ls = torch.tensor(ls0, device="cuda", requires_grad=True)
    Z = impedance_tensor(h, ls, rec, tol=tol)
    phi = (Z - Zobs).abs().pow(2).sum()
    phi.backward()
    g = ls.grad.cpu().numpy()
    t1 = time.perf_counter()
    print(f"tables + forward + gradient: {t1 - t0:.1f} s, phi {phi.item():.4e}", flush=True)

    # warm-started forward solves for the differences
    sa0 = torch.exp(ls.detach()).to(torch.complex128)
    E0 = []
    for f in range(len(freqs)):
        E = torch.zeros((2, 3, nz, ny, nx), dtype=torch.complex128, device="cuda")
        h.solve(sa0, E, tol=tol, max_iter=6000, ifreq=f)
        E0.append(E)
    Er = torch.empty((2, len(rec), 3), dtype=torch.complex128, device="cuda")
    Hr = torch.empty_like(Er)
    Zf = torch.empty((len(rec), 2, 2), dtype=torch.complex128, device="cuda")

    def phi_at(lsig):
        sa = torch.exp(lsig).to(torch.complex128)
        tot = 0.0
        for f in range(len(freqs)):
            E = E0[f].clone()
            st = h.solve(sa, E, tol=tol, max_iter=6000, warm_start=1, ifreq=f)
            assert st["converged"] == 1
            h.fields(sa, E, rec, Er, Hr, ifreq=f)
            lib.impedance(Er, Hr, Zf)
            tot += (Zf - Zobs[f]).abs().pow(2).sum().item()
        return tot

    cells = np.random.default_rng(56).choice(nx * ny * nz, 50, replace=False)
    step = 1e-6
    worst = 0.0
    for c in cells:
        idx = np.unravel_index(c, (nz, ny, nx))
        lp, lm = ls.detach().clone(), ls.detach().clone()
        lp[idx] += step
        lm[idx] -= step
        fd = (phi_at(lp) - phi_at(lm)) / (2 * step)
        bound = 1e-6 * np.abs(g).max() + 1e-4 * abs(fd)
        worst = max(worst, abs(fd - g[idx]) / bound)
        assert abs(fd - g[idx]) <= bound, (idx, fd, g[idx])
    h.close()
    print(f"50 cells: worst |g - fd| / bound = {worst:.3f}; max |g| {np.abs(g).max():.3e}; "
          f"differences {time.perf_counter() - t1:.1f} s", flush=True)
