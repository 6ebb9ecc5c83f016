"""Device memory exhaustion (the failure path of every allocation in the
library): with nearly all free device memory held by the test, giem_tables
and a giem_apply that must grow its spectra workspace return GIEM_ENOMEM,
leave nothing allocated behind, and work once the memory is free again.
The condition is forced from the host (a large torch allocation), so every
kernel still runs normally."""
import numpy as np
import pytest

import giem_synth as gs
from tests.gpu_util import random_model, rel_err, to_dev

pytestmark = pytest.mark.gpu

MiB = 1 << 20


def _hold_all_but(torch, keep_bytes):
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    return torch.empty(max(free - keep_bytes, 0), dtype=torch.uint8, device="cuda")


def _release(torch):
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def _small_model():
    return random_model(8, 6, 3, 90)


def test_tables_and_apply_report_enomem(lib):
    import torch
    m = gs.config_128x128x32()      # 1.1 GB of FP64 spectra per frequency
    # load the library's code objects (and their fixed device arrays) first,
    # so that the free memory before and after compares handles only
    lib.tables(_small_model(), [1.0]).close()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    free0, _ = torch.cuda.mem_get_info()
    print(f"free device memory {free0 / 2**30:.1f} GiB; holding all but 256 MiB", flush=True)
    hog = _hold_all_but(torch, 256 * MiB)
    with pytest.raises(lib.GiemError) as e:
        lib.tables(m, [m["freq"]], flags=lib.TABLES_C64)
    del hog
    _release(torch)
    assert e.value.code == lib.GIEM_ENOMEM, e.value
    free1, _ = torch.cuda.mem_get_info()
    print(f"  giem_tables: ENOMEM; free afterwards {free1 / 2**30:.1f} GiB", flush=True)
    assert free1 >= free0 - 64 * MiB          # nothing of the failed handle is left

    # the same handle built with the memory free, then an apply whose
    # spectra workspace must grow from 2 to 8 right-hand sides (1.6 GB)
    rng = np.random.default_rng(91)
    nx, ny, nz = m["nx"], m["ny"], m["nz"]
    h = lib.tables(m, [m["freq"]])
    sa = to_dev(m["sigma_a"])
    x = to_dev(gs.random_vector(rng, 8, nz, ny, nx))
    y = torch.zeros_like(x)
    ref = torch.empty_like(x)
    hog = _hold_all_but(torch, 64 * MiB)
    with pytest.raises(lib.GiemError) as e:
        h.apply(x, y, sa)
    del hog
    _release(torch)
    assert e.value.code == lib.GIEM_ENOMEM, e.value
    assert not y.any()                          # no kernel wrote y
    h.apply(x, ref, sa)
    h.apply(x, y, sa)
    torch.cuda.synchronize()
    assert torch.equal(y, ref) and bool(torch.isfinite(torch.view_as_real(ref)).all())
    print("  giem_apply: ENOMEM while the workspace cannot grow, then the same results", flush=True)
    h.close()

    # and a normal handle afterwards
    h = lib.tables(m, [m["freq"]])
    h.close()
