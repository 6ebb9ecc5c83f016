"""giem_apply_noalloc (the apply whose spectra live in the library's fixed
device array instead of the handle's workspace) against giem_apply, through
the C ABI: two calls in a row, the second with a smaller input, in both
precisions, and the refusal of a call whose spectra exceed the array."""
import numpy as np
import pytest

import giem_synth as gs
from tests.gpu_util import random_model, rel_err, to_dev

pytestmark = pytest.mark.gpu


def _handle(lib, nx, ny, nz, seed):
    rng = np.random.default_rng(seed)
    m = random_model(nx, ny, nz, seed)
    t = gs.random_packed_table(rng, nx, ny, nz, decay=0.3)
    h = lib.tables_import(m, [m["freq"]], t[None], flags=lib.TABLES_C64)
    return h, m, rng


def test_apply_noalloc_matches_apply(lib):
    import torch
    h, m, rng = _handle(lib, 24, 20, 6, 71)
    nx, ny, nz = m["nx"], m["ny"], m["nz"]
    sa = to_dev(m["sigma_a"])
    print("noalloc 24x20x6: 2 RHS then 1 RHS, FP64 and FP32", flush=True)
    for prec, bar in ((lib.FP64, 1e-10), (lib.FP32, 1e-5)):
        for nrhs in (2, 1):
            x = to_dev(gs.random_vector(rng, nrhs, nz, ny, nx))
            y_ref = torch.empty_like(x)
            y = torch.full_like(x, float("nan"))
            h.apply(x, y_ref, sa, prec=prec)
            h.apply_noalloc(x, y, sa, prec=prec)
            torch.cuda.synchronize()
            err = rel_err(y.cpu().numpy(), y_ref.cpu().numpy())
            print(f"  prec {prec} nrhs {nrhs}: rel err {err:.2e}", flush=True)
            assert err <= bar
    h.close()


def test_apply_noalloc_smaller_grid_after_larger(lib):
    # the shared array keeps the previous call's contents: a smaller grid on
    # a second handle right after a larger one must not see them
    import torch
    out = []
    for (nx, ny, nz, seed) in ((40, 36, 8, 72), (9, 7, 3, 73)):
        h, m, rng = _handle(lib, nx, ny, nz, seed)
        sa = to_dev(m["sigma_a"])
        x = to_dev(gs.random_vector(rng, 2, nz, ny, nx))
        y_ref = torch.empty_like(x)
        y = torch.empty_like(x)
        h.apply(x, y_ref, sa, mode=lib.MODE_AT)
        h.apply_noalloc(x, y, sa, mode=lib.MODE_AT)
        torch.cuda.synchronize()
        out.append(rel_err(y.cpu().numpy(), y_ref.cpu().numpy()))
        h.close()
    print(f"  larger then smaller grid: {out}", flush=True)
    assert max(out) <= 1e-10


def test_apply_noalloc_refuses_oversized_spectra(lib):
    # 64 x 64 x 16: 2 RHS fit the 64 MiB array in FP64, 3 do not
    import torch
    h, m, rng = _handle(lib, 64, 64, 16, 74)
    sa = to_dev(m["sigma_a"])
    x = to_dev(gs.random_vector(rng, 3, 16, 64, 64))
    y = torch.zeros_like(x)
    with pytest.raises(lib.GiemError) as ex:
        h.apply_noalloc(x, y, sa)
    assert ex.value.code == lib.GIEM_EINVAL
    assert float(torch.abs(y).max()) == 0.0
    y2 = torch.empty_like(x[:2])
    y2_ref = torch.empty_like(x[:2])
    h.apply_noalloc(x[:2].contiguous(), y2, sa)
    h.apply(x[:2].contiguous(), y2_ref, sa)
    torch.cuda.synchronize()
    assert rel_err(y2.cpu().numpy(), y2_ref.cpu().numpy()) <= 1e-10
    h.close()
