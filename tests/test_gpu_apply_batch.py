"""GPU parity of giem_apply_batch, the operator apply for several frequencies
in one launch per kernel (the three steps of Sect. 3.3 over all frequencies'
spectra, the block product over (frequency, point) pairs):
  - against the oracle's dense product on each frequency's table;
  - bit for bit against separate giem_apply calls (every plane's transforms
    and every point's products do the same arithmetic in both);
  - the block-product kernels for Nz > 32, the largest batch (32
    vectors), repeated and permuted frequency indices, modes A, A^T and B,
    FP64 and FP32;
  - argument errors."""
import ctypes

import numpy as np
import pytest

import giem_synth as gs
from oracle import dense
from tests.gpu_util import random_model, rel_err, to_dev

pytestmark = pytest.mark.gpu


def _tables(rng, nx, ny, nz, nf):
    return np.stack([gs.random_packed_table(rng, nx, ny, nz, decay=0.1) for _ in range(nf)])


@pytest.mark.parametrize("nx,ny,nz,nrhs,ifreqs", [
    (15, 7, 3, 2, [0, 1, 2]),
    (6, 9, 2, 1, [2, 0, 2, 1]),
    (16, 16, 4, 3, [1, 0]),
])
@pytest.mark.parametrize("mode", ["A", "AT", "B"])
def test_apply_batch_matches_dense(lib, nx, ny, nz, nrhs, ifreqs, mode):
    import torch
    seed = 500 + nx * 11 + ny * 5 + nz + len(ifreqs)
    rng = np.random.default_rng(seed)
    m = random_model(nx, ny, nz, seed)
    freqs = [0.1, 1.0, 10.0]
    tabs = _tables(rng, nx, ny, nz, len(freqs))
    h = lib.tables_import(m, freqs, tabs)
    d = dense.cie_diagonals(m)
    nf = len(ifreqs)
    x = np.stack([gs.random_vector(rng, nrhs, nz, ny, nx) for _ in range(nf)])
    xd = to_dev(x)
    yd = torch.empty_like(xd)
    sa = to_dev(m["sigma_a"])
    code = {"A": lib.MODE_A, "AT": lib.MODE_AT, "B": lib.MODE_B}[mode]
    h.apply_batch(xd, yd, sa, ifreqs=ifreqs, mode=code)
    torch.cuda.synchronize()
    y = yd.cpu().numpy()
    for f, q in enumerate(ifreqs):
        ref = dense.apply_direct(dense.dense_from_packed(tabs[q], m), d, x[f], mode)
        err = rel_err(y[f], ref)
        assert err <= 1e-10, (f, q, err)
    h.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_apply_batch_equals_separate(lib, prec):
    import torch
    nx, ny, nz, nrhs = 20, 12, 5, 2
    rng = np.random.default_rng(77)
    m = random_model(nx, ny, nz, 77)
    freqs = [0.01, 0.1, 1.0, 10.0]
    tabs = _tables(rng, nx, ny, nz, len(freqs))
    h = lib.tables_import(m, freqs, tabs, flags=lib.TABLES_C64)
    p = lib.FP64 if prec == "fp64" else lib.FP32
    ifreqs = [3, 1, 0, 2, 1]
    x = np.stack([gs.random_vector(rng, nrhs, nz, ny, nx) for _ in ifreqs])
    xd = to_dev(x)
    sa = to_dev(m["sigma_a"])
    for nbuf in (1, 2, 3, 4):
        h.set_block_buffers(p, nbuf)
        for mode in (lib.MODE_A, lib.MODE_AT, lib.MODE_B):
            yb = torch.empty_like(xd)
            h.apply_batch(xd, yb, sa, ifreqs=ifreqs, mode=mode, prec=p)
            ys = torch.empty_like(xd)
            for f, q in enumerate(ifreqs):
                h.apply(xd[f], ys[f], sa, mode=mode, prec=p, ifreq=q)
            torch.cuda.synchronize()
            assert torch.equal(yb, ys), (nbuf, mode, float((yb - ys).abs().max()))
    h.close()


def test_apply_batch_deep_kernel(lib):
    # Nz = 33: the packed row no longer fits one workgroup's LDS, the block
    # product stages it by pairs of level bands
    import torch
    nx, ny, nz, nrhs = 4, 3, 33, 2
    rng = np.random.default_rng(91)
    m = random_model(nx, ny, nz, 91)
    freqs = [0.1, 1.0]
    tabs = _tables(rng, nx, ny, nz, len(freqs))
    h = lib.tables_import(m, freqs, tabs, flags=lib.TABLES_C64)
    d = dense.cie_diagonals(m)
    ifreqs = [1, 0]
    x = np.stack([gs.random_vector(rng, nrhs, nz, ny, nx) for _ in ifreqs])
    xd = to_dev(x)
    yd = torch.empty_like(xd)
    sa = to_dev(m["sigma_a"])
    h.apply_batch(xd, yd, sa, ifreqs=ifreqs, mode=lib.MODE_A)
    torch.cuda.synchronize()
    y = yd.cpu().numpy()
    for f, q in enumerate(ifreqs):
        ref = dense.apply_direct(dense.dense_from_packed(tabs[q], m), d, x[f], "A")
        assert rel_err(y[f], ref) <= 1e-10
    ys = torch.empty_like(xd)
    for f, q in enumerate(ifreqs):
        h.apply(xd[f], ys[f], sa, mode=lib.MODE_A, ifreq=q)
    torch.cuda.synchronize()
    assert torch.equal(yd, ys)
    # FP32 as well
    h.apply_batch(xd, yd, sa, ifreqs=ifreqs, mode=lib.MODE_A, prec=lib.FP32)
    for f, q in enumerate(ifreqs):
        h.apply(xd[f], ys[f], sa, mode=lib.MODE_A, ifreq=q, prec=lib.FP32)
    torch.cuda.synchronize()
    assert torch.equal(yd, ys)
    y = yd.cpu().numpy()
    for f, q in enumerate(ifreqs):
        ref = dense.apply_direct(dense.dense_from_packed(tabs[q], m), d, x[f], "A")
        assert rel_err(y[f], ref) <= 2e-5
    h.close()


def test_apply_batch_largest(lib):
    # 4 frequencies x 8 RHS = 32 vectors, the most one batched apply takes
    import torch
    nx, ny, nz, nrhs = 9, 8, 2, 8
    rng = np.random.default_rng(92)
    m = random_model(nx, ny, nz, 92)
    freqs = [0.1, 1.0, 3.0, 10.0]
    tabs = _tables(rng, nx, ny, nz, len(freqs))
    h = lib.tables_import(m, freqs, tabs)
    d = dense.cie_diagonals(m)
    ifreqs = [0, 1, 2, 3]
    x = np.stack([gs.random_vector(rng, nrhs, nz, ny, nx) for _ in ifreqs])
    xd = to_dev(x)
    yd = torch.empty_like(xd)
    sa = to_dev(m["sigma_a"])
    h.apply_batch(xd, yd, sa, ifreqs=ifreqs, mode=lib.MODE_A)
    torch.cuda.synchronize()
    y = yd.cpu().numpy()
    for f, q in enumerate(ifreqs):
        ref = dense.apply_direct(dense.dense_from_packed(tabs[q], m), d, x[f], "A")
        assert rel_err(y[f], ref) <= 1e-10
    h.close()


def test_apply_batch_errors(lib):
    import torch
    nx, ny, nz = 5, 4, 2
    rng = np.random.default_rng(93)
    m = random_model(nx, ny, nz, 93)
    tabs = _tables(rng, nx, ny, nz, 2)
    h = lib.tables_import(m, [0.1, 1.0], tabs)
    sa = to_dev(m["sigma_a"])
    raw = lib.load()

    def call(nf, ifr, nrhs, x, y):
        arr = (ctypes.c_int32 * max(len(ifr), 1))(*ifr)
        return raw.giem_apply_batch(h._p, nf, arr, ctypes.c_void_p(sa.data_ptr()), nrhs,
                                    ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                    lib.MODE_A, lib.FP64, None)

    x = torch.zeros((17, 2, 3, nz, ny, nx), dtype=torch.complex128, device="cuda")
    y = torch.zeros_like(x)
    assert call(17, [0] * 17, 1, x, y) == lib.GIEM_EINVAL        # more than 16 frequencies
    assert call(5, [0] * 5, 7, x, y) == lib.GIEM_EINVAL          # 35 vectors
    assert call(2, [0, 2], 1, x, y) == lib.GIEM_EINVAL           # no frequency 2
    assert call(2, [0, -1], 1, x, y) == lib.GIEM_EINVAL
    assert call(2, [0, 1], 9, x, y) == lib.GIEM_EINVAL           # more than 8 RHS
    assert call(2, [0, 1], 1, x, x) == lib.GIEM_EINVAL           # x and y overlap
    assert call(0, [], 1, x, y) == lib.GIEM_EINVAL               # no frequency
    assert call(2, [0, 1], 0, x, y) == lib.GIEM_EINVAL           # no right-hand side
    assert call(2, [0, 1], 1, x, y) == lib.GIEM_OK
    torch.cuda.synchronize()
    h.close()
