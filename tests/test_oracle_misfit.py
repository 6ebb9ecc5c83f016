"""Pins of the oracle's impedance misfit and its gradient: the forward
sensitivities against central finite differences of the misfit with dense
re-solves, the zero-residual case, and the impedance of a laterally uniform
earth through the full forward map."""
import numpy as np

import giem_synth as gs
from oracle import dense, misfit
from oracle.fundamental import MU0
from oracle.normal_field import LayeredPlaneWave


def _setup(seed, nfreq=2):
    rng = np.random.default_rng(seed)
    m = gs.make_model(3, 2, 2, 100.0, 120.0, np.array([0.0, 40.0, 100.0]), [0.0, 40.0, 500.0],
                      [0.0, 0.02, 0.1, 0.005], 1.0)
    m["sigma_a"] = m["sigma_a"] * 10 ** rng.uniform(0, 1.5, m["sigma_a"].shape)
    rec = np.array([[50.0, 60.0], [250.0, 60.0], [150.0, 180.0], [50.0, 180.0]])
    freqs = [1.0, 0.1][:nfreq]
    ops = []
    for f in freqs:
        t = gs.random_packed_table(rng, m["nx"], m["ny"], m["nz"], scale=1.0)
        d = dense.cie_diagonals(m)
        # keep V^-1 B (sa - sb) of order 0.3 so that P is well conditioned
        t *= 0.3 / (np.abs(t).max() * np.abs(m["sigma_a"]).max() / d["vol"].min() * 6)
        ops.append(misfit.operator(m, t, rec, f))
    return m, ops, rng


def test_gradient_matches_central_differences():
    m, ops, rng = _setup(31)
    sa = m["sigma_a"]
    sobs = sa * np.exp(0.3 * rng.standard_normal(sa.shape))
    _, Zobs = misfit.misfit(m, ops, sobs, 0.0)
    g = misfit.misfit_gradient(m, ops, sa, Zobs)
    h = 1e-6
    for idx in np.ndindex(sa.shape):
        sp, sm = sa.copy(), sa.copy()
        sp[idx] *= np.exp(h)
        sm[idx] *= np.exp(-h)
        fd = (misfit.misfit(m, ops, sp, Zobs)[0] - misfit.misfit(m, ops, sm, Zobs)[0]) / (2 * h)
        assert abs(fd - g[idx]) <= 1e-7 * np.abs(g).max() + 1e-6 * abs(fd), (idx, fd, g[idx])


def test_zero_residual_gives_zero_misfit_and_gradient():
    m, ops, _ = _setup(32, nfreq=1)
    phi0, Z = misfit.misfit(m, ops, m["sigma_a"], 0.0)
    phi, _ = misfit.misfit(m, ops, m["sigma_a"], Z)
    assert phi0 > 0 and phi == 0.0
    assert np.abs(misfit.misfit_gradient(m, ops, m["sigma_a"], Z)).max() == 0.0


def test_uniform_layered_earth_impedance():
    # sa = sb: no anomalous field, Z = [[0, Z1], [-Z1, 0]] with Z1 = E/H of
    # the 1-D layered plane wave at the surface, the same at every receiver
    m, ops, _ = _setup(33, nfreq=2)
    sb = m["sigma"][m["layer_of_cell"]][:, None, None] * np.ones(m["sigma_a"].shape)
    _, Z = misfit.misfit(m, ops, sb, 0.0)
    for f, op in enumerate(ops):
        pw = LayeredPlaneWave(m["d"], m["sigma"], op["freq"])
        z1 = 1.0 / pw.H_surface()
        assert np.abs(Z[f][:, 0, 0]).max() < 1e-14 * abs(z1)
        assert np.abs(Z[f][:, 0, 1] - z1).max() <= 1e-13 * abs(z1)
        assert np.abs(Z[f][:, 1, 0] + z1).max() <= 1e-13 * abs(z1)
        # apparent resistivity lies between the layer resistivities
        rho_a = abs(z1) ** 2 / (2 * np.pi * op["freq"] * MU0)
        s = m["sigma"][1:].real
        assert 1 / s.max() <= rho_a <= 1 / s.min()
