"""GPU parity of the operator apply (Sect. 3.3 three-step FFT algorithm) with
the oracle's O(N^2) dense product on the same packed table."""
import numpy as np
import pytest

import giem_synth as gs
from oracle import dense
from tests.gpu_util import random_model, rel_err, to_dev

pytestmark = pytest.mark.gpu

# (nx, ny, nz, nrhs): single-cell and single-row edge cases, ragged 11-smooth
# sizes whose padded lengths need radices 3, 5, 7 and 11, the 16 x 16 x 4 grid.
SHAPES = [(1, 1, 1, 1), (1, 5, 2, 1), (6, 1, 3, 2), (4, 3, 2, 3), (15, 7, 3, 2),
          (10, 14, 2, 1), (16, 16, 4, 2), (9, 12, 5, 1), (11, 22, 2, 2), (33, 4, 3, 1)]


def _case(nx, ny, nz, seed):
    rng = np.random.default_rng(seed)
    m = random_model(nx, ny, nz, seed)
    t = gs.random_packed_table(rng, nx, ny, nz, decay=0.1)
    return m, t, rng


@pytest.mark.parametrize("nx,ny,nz,nrhs", SHAPES)
@pytest.mark.parametrize("mode", ["B", "A", "AT"])
def test_apply_fp64_matches_dense(lib, nx, ny, nz, nrhs, mode):
    import torch
    m, t, rng = _case(nx, ny, nz, 100 + nx * 7 + ny * 3 + nz)
    h = lib.tables_import(m, [m["freq"]], t[None])
    B = dense.dense_from_packed(t, m)
    d = dense.cie_diagonals(m)
    x = gs.random_vector(rng, nrhs, nz, ny, nx)
    ref = dense.apply_direct(B, d, x, mode)
    xd = to_dev(x)
    yd = torch.empty_like(xd)
    sa = to_dev(m["sigma_a"])
    code = {"A": lib.MODE_A, "AT": lib.MODE_AT, "B": lib.MODE_B}[mode]
    h.apply(xd, yd, sa, mode=code)
    torch.cuda.synchronize()
    err = rel_err(yd.cpu().numpy(), ref)
    assert err <= 1e-10, err
    h.close()


@pytest.mark.parametrize("nx,ny,nz,nrhs", [(15, 7, 3, 2), (16, 16, 4, 2)])
def test_apply_fp32_error(lib, nx, ny, nz, nrhs):
    import torch
    m, t, rng = _case(nx, ny, nz, 7)
    h = lib.tables_import(m, [m["freq"]], t[None], flags=lib.TABLES_C64)
    B = dense.dense_from_packed(t, m)
    d = dense.cie_diagonals(m)
    x = gs.random_vector(rng, nrhs, nz, ny, nx)
    ref = dense.apply_direct(B, d, x, "B")
    xd = to_dev(x)
    yd = torch.empty_like(xd)
    h.apply(xd, yd, None, mode=lib.MODE_B, prec=lib.FP32)
    torch.cuda.synchronize()
    err = rel_err(yd.cpu().numpy(), ref)
    # complex64 FFTs and FP32 accumulation: a few units of 1e-7 per term
    assert err <= 2e-5, err
    h.close()


def test_table_bytes_is_packed_size(lib):
    m, t, _ = _case(6, 5, 3, 3)
    h = lib.tables_import(m, [m["freq"]], t[None], flags=lib.TABLES_C64)
    b128, b64 = h.table_bytes()
    assert b128 == 7 * 6 * 2 * 3 * 7 * 16 and b64 == b128 // 2
    h.close()


def test_export_roundtrip(lib):
    m, t, _ = _case(5, 4, 2, 4)
    h = lib.tables_import(m, [m["freq"]], t[None])
    assert np.array_equal(h.export(0), t)
    h.close()


def test_apply_argument_errors_leave_output_untouched(lib):
    # empty and out-of-range arguments are refused on the host before any
    # kernel writes y; a valid call afterwards still matches the oracle
    import ctypes
    import torch
    nx, ny, nz = 5, 4, 2
    m, t, rng = _case(nx, ny, nz, 8)
    h = lib.tables_import(m, [m["freq"]], t[None])       # no complex64 tables
    raw = lib.load()
    x = to_dev(gs.random_vector(rng, 2, nz, ny, nx))
    sentinel = torch.full((2, 3, nz, ny, nx), 7.0 + 1.0j, dtype=torch.complex128, device="cuda")
    y = sentinel.clone()
    sa = to_dev(m["sigma_a"])

    def call(ifreq=0, nrhs=2, xp=x, yp=y, sap=sa, mode=lib.MODE_A, prec=lib.FP64):
        ptr = lambda v: None if v is None else ctypes.c_void_p(v.data_ptr())
        return raw.giem_apply(h._p, ifreq, ptr(sap), nrhs, ptr(xp), ptr(yp), mode, prec, None)

    assert call(nrhs=0) == lib.GIEM_EINVAL                 # no right-hand side
    assert call(nrhs=-1) == lib.GIEM_EINVAL
    assert call(nrhs=9) == lib.GIEM_EINVAL                 # more than 8
    assert call(ifreq=1) == lib.GIEM_EINVAL                # one frequency only
    assert call(ifreq=-1) == lib.GIEM_EINVAL
    assert call(mode=3) == lib.GIEM_EINVAL
    assert call(prec=2) == lib.GIEM_EINVAL
    assert call(xp=None) == lib.GIEM_EINVAL
    assert call(yp=None) == lib.GIEM_EINVAL
    assert call(sap=None) == lib.GIEM_EINVAL               # mode A needs sigma_a
    assert call(yp=x) == lib.GIEM_EINVAL                   # x and y overlap
    assert call(prec=lib.FP32) == lib.GIEM_EINVAL          # complex64 tables absent
    torch.cuda.synchronize()
    assert torch.equal(y, sentinel)
    assert call(sap=None, mode=lib.MODE_B) == lib.GIEM_OK  # mode B ignores sigma_a
    assert call() == lib.GIEM_OK
    torch.cuda.synchronize()
    ref = dense.apply_direct(dense.dense_from_packed(t, m), dense.cie_diagonals(m),
                             x.cpu().numpy(), "A")
    assert rel_err(y.cpu().numpy(), ref) <= 1e-10
    h.close()


def test_rejects_non_smooth_sizes_and_bad_models(lib):
    m, t, _ = _case(13, 4, 2, 5)
    with pytest.raises(lib.GiemError):
        lib.tables_import(m, [m["freq"]], t[None])
    m2, t2, _ = _case(4, 4, 2, 6)
    m2 = dict(m2)
    m2["z_edges"] = np.array([0.0, 150.0, 300.0])  # second interface at 100: straddles
    m2["d"] = np.array([0.0, 100.0, 5000.0])
    with pytest.raises(lib.GiemError) as e:
        lib.tables_import(m2, [1.0], t2[None])
    assert e.value.code == lib.GIEM_EDOMAIN


@pytest.fixture(scope="module")
def full_case():
    """The 128 x 128 x 32 layered workload (2 RHS) with a random table."""
    from oracle import packed
    m = gs.config_128x128x32()
    rng = np.random.default_rng(77)
    t = gs.random_packed_table(rng, m["nx"], m["ny"], m["nz"], decay=0.2)
    d = dense.cie_diagonals(m)
    t = t / (np.abs(d["R1"]).max() * np.abs(d["R2"]).max() * 1e3)
    x = gs.random_vector(rng, 2, m["nz"], m["ny"], m["nx"])
    qnn = packed.full_tensor_nonneg(t, m["nz"])
    nz, ny, nx = m["nz"], m["ny"], m["nx"]
    cells = [(0, 0, 0), (nz - 1, ny - 1, nx - 1), (0, ny - 1, 0), (nz - 1, 0, nx - 1),
             (nz // 2, ny // 2, nx // 2)]
    cells += [(int(rng.integers(nz)), int(rng.integers(ny)), int(rng.integers(nx)))
              for _ in range(5)]
    return m, t, x, qnn, cells


@pytest.mark.parametrize("nbuf", [1, 2, 3, 4])
@pytest.mark.parametrize("mode,prec,tol", [("A", 0, 1e-10), ("B", 0, 1e-10), ("AT", 0, 1e-10),
                                           ("B", 1, 1e-4)])
def test_apply_full_size_sampled(lib, full_case, mode, prec, tol, nbuf):
    # The launch configuration the benchmark times (128 x 128 x 32, 2 RHS),
    # checked at sampled output cells against the oracle's direct sum, with
    # each block-product variant: one or two prefetch sets in one workgroup
    # per CU, or two workgroups per CU.
    import torch
    m, t, x, qnn, cells = full_case
    print(f"full-size apply mode={mode} prec={prec} block buffers={nbuf}", flush=True)
    h = lib.tables_import(m, [m["freq"]], t[None], flags=lib.TABLES_C64)
    h.set_block_buffers(prec, nbuf)
    xd = to_dev(x)
    yd = torch.empty_like(xd)
    code = {"A": lib.MODE_A, "AT": lib.MODE_AT, "B": lib.MODE_B}[mode]
    h.apply(xd, yd, to_dev(m["sigma_a"]), mode=code, prec=prec)
    torch.cuda.synchronize()
    y = yd.cpu().numpy()
    h.close()
    got = np.stack([y[:, :, iz, iy, ix] for (iz, iy, ix) in cells], 1)
    ref = dense.apply_cells(qnn, m, x, cells, mode)
    err = rel_err(got, ref)
    print(f"  sampled rel err {err:.3e}", flush=True)
    assert err <= tol, err


@pytest.mark.parametrize("nx,ny,nz,nrhs", [(15, 7, 3, 2), (16, 16, 4, 2), (48, 40, 2, 1), (11, 22, 2, 2)])
def test_every_fft_shape_matches_dense(lib, nx, ny, nz, nrhs):
    # every (sequences, threads) launch shape of the four FFT passes gives the
    # dense product; giem_tune then keeps one of them per pass
    import torch
    m, t, rng = _case(nx, ny, nz, 300 + nx + ny + nz)
    h = lib.tables_import(m, [m["freq"]], t[None], flags=lib.TABLES_C64)
    B = dense.dense_from_packed(t, m)
    d = dense.cie_diagonals(m)
    x = gs.random_vector(rng, nrhs, nz, ny, nx)
    ref = dense.apply_direct(B, d, x, "A")
    xd, sa = to_dev(x), to_dev(m["sigma_a"])
    yd = torch.empty_like(xd)
    tried = 0
    for prec, tol in ((lib.FP64, 1e-10), (lib.FP32, 2e-5)):
        first = {}
        for nt in (256, 512):
            for g in (1, 2, 4, 8, 16, 32, 64):
                try:
                    h.set_fft_shape(prec, [(g, nt)] * 4)
                except lib.GiemError:
                    continue
                h.apply(xd, yd, sa, mode=lib.MODE_A, prec=prec)
                torch.cuda.synchronize()
                err = rel_err(yd.cpu().numpy(), ref)
                assert err <= tol, (prec, g, nt, err)
                # every shape gives the same bits
                if first:
                    assert torch.equal(yd, next(iter(first.values()))), (prec, g, nt)
                first[(g, nt)] = yd.clone()
                tried += 1
        h.set_fft_shape(prec, None)
        for nbuf in (4, 3, 2, 1):
            h.set_block_buffers(prec, nbuf)
            h.apply(xd, yd, sa, mode=lib.MODE_A, prec=prec)
            torch.cuda.synchronize()
            assert rel_err(yd.cpu().numpy(), ref) <= tol, (prec, nbuf)
    with pytest.raises(lib.GiemError):
        h.set_fft_shape(lib.FP64, [(8, 384)] * 4)
    chosen = h.tune(sa, nrhs=nrhs)
    h.apply(xd, yd, sa, mode=lib.MODE_A)
    torch.cuda.synchronize()
    assert rel_err(yd.cpu().numpy(), ref) <= 1e-10
    assert all(nt in (256, 512) and g >= 1 for g, nt in chosen["fp64"] + chosen["fp32"])
    print(f"{nx}x{ny}x{nz}: {tried} shapes; tuned {chosen}", flush=True)
    h.close()


@pytest.mark.parametrize("nz", [31, 32])
def test_block_product_every_rhs_count_at_deepest_grids(lib, nz):
    # the deepest grids the pipelined block product stages, with every
    # right-hand-side count up to the maximum of 8: the row and the input
    # fragments outgrow the LDS somewhere in between and the launcher falls
    # back (two workgroups per CU -> one, pipelined -> gather); every variant
    # on both sides of that boundary matches the dense product
    import torch
    nx, ny = 2, 3
    m, t, rng = _case(nx, ny, nz, 600 + nz)
    h = lib.tables_import(m, [m["freq"]], t[None], flags=lib.TABLES_C64)
    B = dense.dense_from_packed(t, m)
    d = dense.cie_diagonals(m)
    sa = to_dev(m["sigma_a"])
    x = gs.random_vector(rng, 8, nz, ny, nx)
    ref = dense.apply_direct(B, d, x, "A")
    for nrhs in range(1, 9):
        xd = to_dev(x[:nrhs])
        yd = torch.empty_like(xd)
        for prec, tol in ((lib.FP64, 1e-10), (lib.FP32, 2e-5)):
            for nbuf in (1, 2, 3, 4):
                h.set_block_buffers(prec, nbuf)
                h.apply(xd, yd, sa, mode=lib.MODE_A, prec=prec)
                torch.cuda.synchronize()
                err = rel_err(yd.cpu().numpy(), ref[:nrhs])
                assert err <= tol, (nrhs, prec, nbuf, err)
    h.close()


@pytest.mark.parametrize("nx,ny,nz,nrhs", [(4, 3, 40, 2), (3, 2, 32, 8), (2, 3, 33, 1),
                                            (2, 3, 47, 2), (3, 2, 64, 1), (2, 2, 40, 8),
                                            (2, 2, 118, 2), (2, 3, 130, 2), (2, 2, 170, 8)])
@pytest.mark.parametrize("prec,tol", [(0, 1e-10), (1, 2e-5)])
def test_apply_deep_block_product(lib, nx, ny, nz, nrhs, prec, tol):
    # shapes whose packed row and input fragments do not fit the pipelined
    # kernel (more than 32 layers, or 8 right-hand sides at 32 layers) take
    # the band-pair kernel: partial last bands (33, 47, 118, 130 levels),
    # whole bands (64), the two tile counts per wavefront of each precision
    # (FP32: three up to 8 bands, six from 9; FP64: two up to 10 bands,
    # three at 11; 170 levels is the deepest grid a handle accepts), several
    # vector groups (8 right-hand sides at up to four mirror points); same
    # bar against the dense product
    import torch
    m, t, rng = _case(nx, ny, nz, 500 + nz + nrhs)
    h = lib.tables_import(m, [m["freq"]], t[None], flags=lib.TABLES_C64)
    B = dense.dense_from_packed(t, m)
    d = dense.cie_diagonals(m)
    x = gs.random_vector(rng, nrhs, nz, ny, nx)
    ref = dense.apply_direct(B, d, x, "A")
    xd = to_dev(x)
    yd = torch.empty_like(xd)
    h.apply(xd, yd, to_dev(m["sigma_a"]), mode=lib.MODE_A, prec=prec)
    torch.cuda.synchronize()
    err = rel_err(yd.cpu().numpy(), ref)
    h.close()
    assert err <= tol, err


def test_deepest_grid_limit(lib):
    # 170 levels is the deepest grid: 171 is refused when the handle is made
    import torch  # noqa: F401
    for nz, ok in ((170, True), (171, False)):
        m, t, _ = _case(1, 1, nz, 950 + nz)
        if ok:
            lib.tables_import(m, [m["freq"]], t[None]).close()
        else:
            with pytest.raises(lib.GiemError):
                lib.tables_import(m, [m["freq"]], t[None])


def test_profile_modes(lib):
    # all five kernels bracketed, then only the block product: the same number
    # of applies and RHS, only stage 2 filled in the second mode
    import torch
    m, t, rng = _case(16, 16, 4, 8)
    h = lib.tables_import(m, [m["freq"]], t[None])
    x = to_dev(gs.random_vector(rng, 2, 4, 16, 16))
    y = torch.empty_like(x)
    sa = to_dev(m["sigma_a"])
    h.profile(True)
    for _ in range(3):
        h.apply(x, y, sa)
    p_all = h.profile_read()["fp64"]
    h.profile(True, stage=2)
    for _ in range(3):
        h.apply(x, y, sa)
    p_one = h.profile_read()["fp64"]
    h.profile(False)
    assert p_all["applies"] == p_one["applies"] == 3 and p_all["rhs"] == p_one["rhs"] == 6
    assert all(v > 0 for v in p_all["stage_ms"])
    assert p_one["stage_ms"][2] > 0 and all(p_one["stage_ms"][k] == 0 for k in (0, 1, 3, 4))
    with pytest.raises(lib.GiemError):
        h.profile(True, stage=5)
    h.close()
