"""Helpers shared by the GPU tests (test infrastructure only)."""
import numpy as np

import giem_synth as gs


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def rel_err(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def component_errors(a, b, axes, floor=1e-3):
    """Relative 2-norm error of every slice of a against b that fixes the
    indices along axes (for example the RHS and the field component), each
    relative to the larger of that slice's norm and floor times the norm of
    all of b: small components (E_z, cross-polarised parts) are checked on
    their own scale instead of hiding under the large ones."""
    a = np.asarray(a)
    b = np.asarray(b)
    axes = tuple(ax % b.ndim for ax in axes)
    rest = tuple(ax for ax in range(b.ndim) if ax not in axes)
    num = np.sqrt(np.sum(np.abs(a - b) ** 2, axis=rest))
    den = np.sqrt(np.sum(np.abs(b) ** 2, axis=rest))
    den = np.maximum(den, floor * np.linalg.norm(b.ravel()))
    return float(np.max(num / np.maximum(den, 1e-300)))


def random_model(nx, ny, nz, seed, contrast=2.0, freq=1.0):
    """A layered model whose cells sit in two earth layers, random sigma_a."""
    rng = np.random.default_rng(seed)
    hz = 100.0
    z = np.arange(nz + 1) * hz
    # an interface at a cell boundary inside the grid when nz > 1
    dint = z[max(1, nz // 2)] if nz > 1 else 5 * hz
    d = [0.0, dint, 10 * nz * hz + 1000.0]
    sig = [0.0, 0.02, 0.005, 0.1]
    m = gs.make_model(nx, ny, nz, 50.0, 70.0, z, d, sig, freq)
    fac = 10.0 ** rng.uniform(0.0, contrast, size=m["sigma_a"].shape)
    m["sigma_a"] = m["sigma_a"] * fac
    return m
