#!/usr/bin/env python3
"""Throughput of the contracting-IE hot path on one GPU.

One step = one GMRES(30) solve to a relative residual of 1e-6 of the
128 x 128 x 32 layered-earth workload (200 x 200 x 100 m cells, 5 earth
layers, 3 blocks of contrast up to 1e4, f = 0.01 Hz) for both plane-wave
polarisations at once (2 right-hand sides), with the tables and all vectors
resident in HBM.  Every operator apply inside the solve runs the five HIP
kernels (x-FFT, y-FFT, packed block product, inverse y-FFT, inverse x-FFT).

value = RHS operator applies per second of solve wall time (whole solve,
orthogonalisation included).  Also reported: the apply alone, the solve time
of the FP32-refined form and its field error against a tight FP64 solve,
both forms at matched accuracy (each at the loosest residual tolerance whose
field error against an FP64 solve to 1e-12 is at most 1e-6, and the
speed-up there), the same for the 256 x 256 x 32 workload of the precision
form, the roofline of the dominant kernel (HIP events around each of its
launches in the timed region, only that kernel bracketed; it is found by one
fully bracketed solve before) and the oracle's CPU FFT apply timed on the
host cores.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--table physical|synthetic]
                  [--no-cpu] [--no-extra]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

HBM_PEAK_GBS = 8000.0
COUNTERS_FILE = os.path.join(HERE, "profiles", "block_product_128x128x32_r2_fp64_counters.md")
BLOCK_SOURCE = os.path.join(HERE, "paper_1512_06126_amd", "csrc", "kernels_block.hip")
STAGES = ("fft_x", "fft_y", "block_product", "ifft_y", "ifft_x")


def stage_bytes(nx, ny, nz, R, c):
    """Algorithmic HBM bytes of one launch of each kernel (R right-hand sides,
    c bytes per complex of the spectra; vectors are always complex128)."""
    n = nx * ny * nz
    P = 3 * nz
    half = R * P * 2 * nx * ny * c          # x-transformed planes, Ny rows
    full = R * P * 4 * nx * ny * c          # padded 2-D spectra
    T = (nx + 1) * (ny + 1) * 2 * nz * (2 * nz + 1) * c
    return {
        "fft_x": R * 3 * n * 16 + n * 16 + half,
        "fft_y": half + full,
        "block_product": T + 2 * full,
        "ifft_y": full + half,
        "ifft_x": half + 2 * R * 3 * n * 16 + 2 * n * 16,
    }


def m3_bytes(nx, ny, nz, R, c):
    """Three-step model: table once + 78 N c per right-hand side."""
    T = (nx + 1) * (ny + 1) * 2 * nz * (2 * nz + 1) * c
    return T + R * 78 * nx * ny * nz * c


def read_traffic(block_buffers):
    """HBM bytes per launch of the block product from the committed counter
    summary, or None when absent, taken on another version of the kernel, or
    on the other prefetch depth than the one in use."""
    if not os.path.exists(COUNTERS_FILE):
        return None
    kv = {}
    for line in open(COUNTERS_FILE):
        if ":" in line and line.strip().startswith("- "):
            k, v = line.strip()[2:].split(":", 1)
            kv[k.strip()] = v.strip().strip("`")
    with open(BLOCK_SOURCE, "rb") as fh:
        sha = hashlib.sha256(fh.read()).hexdigest()
    if kv.get("kernel_source_sha256") != sha or kv.get("block_buffers") != str(block_buffers):
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def counter_summary(dirs):
    """Markdown summary of rocprofv3 --pmc runs of `bench.py --counter-run`
    (their output directories): per kernel of the apply and of the
    Gram-Schmidt step, the mean counter value per dispatch; FETCH_SIZE and
    WRITE_SIZE (KiB) scaled by what they read for the 1 GiB calibration
    copy, against the algorithmic bytes of the 128 x 128 x 32, R = 2
    workload; SQ_VALU_MFMA_BUSY_CYCLES as a share of the 1024 SIMDs over
    the kernel's duration (GRBM_GUI_ACTIVE, summed over the 8 XCDs), and
    SQ_LDS_IDX_ACTIVE, SQ_LDS_BANK_CONFLICT and SQ_WAVE_CYCLES per CU and
    cycle (means over the dispatches of each run).  The
    Gram-Schmidt kernels are summed over the GMRES(30) cycle (step j reads
    V_0 .. V_j and w; the update also writes w)."""
    import collections
    import csv
    rows = []
    for d in dirs:
        for root, _, files in os.walk(d):
            for f in files:
                if f.endswith("counter_collection.csv"):
                    rows += list(csv.DictReader(open(os.path.join(root, f))))

    def short(k):
        k = k.split("(")[0].replace("giem::", "").replace("void ", "")
        return k.replace("cplx<double>", "c128").replace("cplx<float>", "c64").strip()

    vals = collections.defaultdict(lambda: collections.defaultdict(list))
    for r in sorted(rows, key=lambda r: int(r["Dispatch_Id"])):
        vals[r["Counter_Name"]][short(r["Kernel_Name"])].append(float(r["Counter_Value"]))
    cal = {}
    for c in ("FETCH_SIZE", "WRITE_SIZE"):
        cp = [v for v in vals.get(c, {}).get("__amd_rocclr_copyBuffer", []) if v > 4e5]
        if cp:
            cal[c] = 1048576.0 / cp[0]
    nx = ny = 128
    nz, R = 32, 2
    vec = R * 3 * nx * ny * nz * 16
    alg = {}
    for c, b in ((16, stage_bytes(nx, ny, nz, R, 16)), (8, stage_bytes(nx, ny, nz, R, 8))):
        T = "double" if c == 16 else "float"
        alg[f"k_fft_x_fwd<{T}"] = b["fft_x"]
        alg[f"k_fft_y<{T}"] = (b["fft_y"] + b["ifft_y"]) / 2   # forward and inverse alike
        alg[f"k_block_pipe<{T}"] = alg[f"k_block_pipe1<{T}"] = b["block_product"]
        alg[f"k_block_dbl<{T}"] = b["block_product"]
        alg[f"k_fft_x_inv<{T}"] = b["ifft_x"]
    gs_alg = {"k_dots": (sum(j + 2 for j in range(30)) * vec, 0),
              "k_update": (sum(j + 2 for j in range(30)) * vec, 30 * vec)}
    names = [k for k in vals.get("FETCH_SIZE", vals[next(iter(vals))])
             if k.startswith(("k_fft", "k_block", "k_dots", "k_update"))]
    out = [f"Calibration: FETCH_SIZE x {cal.get('FETCH_SIZE', float('nan')):.5f}, "
           f"WRITE_SIZE x {cal.get('WRITE_SIZE', float('nan')):.5f} (1 GiB copy).", "",
           "| Kernel | dispatches | read (MB) | write (MB) | algorithmic (MB) | traffic / algorithmic | MFMA busy | MFMA flop | LDS busy | LDS bank conflict | waves / CU |",
           "|---|---|---|---|---|---|---|---|---|---|---|"]
    for k in names:
        f = vals["FETCH_SIZE"].get(k, []) if "FETCH_SIZE" in vals else []
        w = vals["WRITE_SIZE"].get(k, []) if "WRITE_SIZE" in vals else []
        gsk = next((g for g in gs_alg if k.startswith(g + "<")), None)
        if gsk:   # whole cycle
            rd = sum(f) * 1024 * cal.get("FETCH_SIZE", 0) if len(f) == 30 else float("nan")
            wr = sum(w) * 1024 * cal.get("WRITE_SIZE", 0) if len(w) == 30 else float("nan")
            a = sum(gs_alg[gsk])
            label = f"`{k}` (30 steps, summed)"
        else:
            rd = sum(f) / len(f) * 1024 * cal.get("FETCH_SIZE", 0) if f else float("nan")
            wr = sum(w) / len(w) * 1024 * cal.get("WRITE_SIZE", 0) if w else float("nan")
            a = next((v for p, v in alg.items() if k.startswith(p + ",") or k.startswith(p + "<")), float("nan"))
            label = f"`{k}`"
        busy = vals.get("SQ_VALU_MFMA_BUSY_CYCLES", {}).get(k)
        gui = vals.get("GRBM_GUI_ACTIVE", {}).get(k)
        mops = (vals.get("SQ_INSTS_VALU_MFMA_MOPS_F64", {}).get(k, []) +
                vals.get("SQ_INSTS_VALU_MFMA_MOPS_F32", {}).get(k, []))
        nmops = len(vals.get("SQ_INSTS_VALU_MFMA_MOPS_F64", {}).get(k, [])) or 1
        mean = lambda x: sum(x) / len(x)
        util = (f"{100 * mean(busy) / (mean(gui) / 8 * 1024):.1f}%"
                if busy and gui and sum(busy) > 0 else "")
        flop = f"{sum(mops) / nmops * 512 / 1e9:.2f} G" if mops and sum(mops) > 0 else ""
        # LDS and occupancy: per CU and cycle of the kernel's duration
        # (SQ_WAVE_CYCLES counts every fourth cycle)
        lds = []
        for c, scale, fmt in (("SQ_LDS_IDX_ACTIVE", 100, "{:.1f}%"),
                              ("SQ_LDS_BANK_CONFLICT", 100, "{:.1f}%"),
                              ("SQ_WAVE_CYCLES", 4, "{:.1f}")):
            x = vals.get(c, {}).get(k)
            g2 = vals.get("GRBM_GUI_ACTIVE", {}).get(k)
            lds.append(fmt.format(scale * mean(x) / (mean(g2) / 8 * 256)) if x and g2 else "")
        n = max(len(f), len(w))
        out.append(f"| {label} | {n} | {rd / 1e6:.1f} | {wr / 1e6:.1f} | {a / 1e6:.1f} | "
                   f"{(rd + wr) / a:.3f} | {util} | {flop} | " + " | ".join(lds) + " |")
    return "\n".join(out)


def synthetic_table(model, seed=20):
    """Random packed table with the storage symmetries, scaled so that the
    system stays well conditioned (stand-in until tables are computed)."""
    import giem_synth as gs
    rng = np.random.default_rng(seed)
    nx, ny, nz = model["nx"], model["ny"], model["nz"]
    t = gs.random_packed_table(rng, nx, ny, nz, decay=0.2)
    # |R1| <= 2 sqrt(Re sb) / V and |R2| <= sqrt(Re sb) since |gamma| < 1
    sb = np.asarray(model["sigma"])[model["layer_of_cell"]].real
    vol = model["hx"] * model["hy"] * np.diff(model["z_edges"])
    bound = (2 * np.sqrt(sb) / vol).max() * np.sqrt(sb).max() * 2 * np.sqrt(3 * nx * ny * nz)
    return t * (0.2 / bound)


def cpu_baseline(model, table, budget_s=15.0, seed=30):
    """The oracle's three-step FFT apply (Sect. 3.3 on the CPU: scipy.fft
    with every host core, one batched matrix product per frequency) timed on
    whole applies of the same workload, 2 RHS, for about budget_s seconds; the
    set-up of its unpacked spectral table is not counted (as the GPU table
    build is not)."""
    from oracle import dense, fft_apply
    import giem_synth as gs
    try:
        from threadpoolctl import threadpool_info
        blas = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    except Exception:
        blas = 1
    cores = max(blas, os.cpu_count() or 1)
    rng = np.random.default_rng(seed)
    nx, ny, nz = model["nx"], model["ny"], model["nz"]
    x = gs.random_vector(rng, 2, nz, ny, nx)
    t_set = time.perf_counter()
    qhat = fft_apply.spectral_blocks(table, nz)
    d = dense.cie_diagonals(model)
    setup_s = time.perf_counter() - t_set
    done = 0
    t0 = time.perf_counter()
    while done == 0 or time.perf_counter() - t0 < budget_s:
        fft_apply.apply(qhat, d, x, "A")
        done += 1
    dt = time.perf_counter() - t0
    del qhat
    return {"value": 2 * done / dt, "unit": "RHS-applies/s", "cores": cores, "kind": "oracle",
            "sample": f"{done} whole applies of the {nx}x{ny}x{nz} operator to 2 RHS by the "
                      f"oracle's three-step FFT path (scipy.fft and batched products, "
                      f"{os.cpu_count()} host threads) in {dt:.1f} s; its spectral table "
                      f"set-up ({setup_s:.1f} s) not counted"}


TOL_LADDER = (1e-6, 3e-7, 1e-7, 3e-8, 1e-8, 3e-9, 1e-9, 3e-10, 1e-10)
FIELD_ERR_TARGET = 1e-6


def relerr(a, b):
    import torch
    return float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))


def matched_accuracy(g, solve, E, Eref, reps):
    """For the plain FP64 and the FP32-refined forms, the loosest residual
    tolerance of TOL_LADDER whose field error against Eref is at most
    FIELD_ERR_TARGET, the mean solve time there over reps solves, and the
    speed-up of the refined form at that accuracy."""
    import torch
    out = {"target_field_err": FIELD_ERR_TARGET}
    for prec, key in ((g.FP64, "fp64"), (g.FP32, "fp32_refined")):
        pick = None
        for tol in TOL_LADDER:
            Et = torch.zeros_like(E)
            st = solve(prec, tol, Et)
            err = relerr(Et, Eref)
            if err <= FIELD_ERR_TARGET:
                pick = (tol, err, st)
                break
        if pick is None:
            out[key] = None
            continue
        tol, err, st = pick
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            st = solve(prec, tol, Et)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / reps
        out[key] = {"tol": tol, "field_err": err, "ms": round(ms, 3), "iters": st["iters"],
                    "outer_iters": st["outer_iters"]}
    if out.get("fp64") and out.get("fp32_refined"):
        out["speedup_fp32_refined"] = round(out["fp64"]["ms"] / out["fp32_refined"]["ms"], 3)
    return out


def precision_workload(g, torch, dev):
    """The 256 x 256 x 32 workload (100 x 100 x 50 m cells, same generator,
    f = 0.01 Hz, 2 plane-wave RHS): FP64 tables and their complex64 copy,
    reference FP64 solve to 1e-12, then both forms at matched accuracy."""
    import giem_synth as gs
    m = gs.config_precision()
    nx, ny, nz = m["nx"], m["ny"], m["nz"]
    t0 = time.perf_counter()
    h = g.tables(m, [m["freq"]], flags=g.TABLES_C64)
    torch.cuda.synchronize()
    tab_s = time.perf_counter() - t0
    sa = torch.from_numpy(np.ascontiguousarray(m["sigma_a"])).to(dev)
    h.tune(sa, nrhs=2)
    E = torch.zeros((2, 3, nz, ny, nx), dtype=torch.complex128, device=dev)

    def solve(prec, tol, out=E):
        return h.solve(sa, out, tol=tol, restart=30, max_iter=6000, precision=prec,
                       inner_tol=1e-3, max_outer=30)

    Eref = torch.zeros_like(E)
    sref = solve(g.FP64, 1e-12, Eref)
    res = matched_accuracy(g, solve, E, Eref, 1)
    res.update({"workload": "256x256x32 cells of 100x100x50 m, same generator (seed 3), "
                            "f = 0.01 Hz, 2 plane-wave RHS",
                "table_build_s": round(tab_s, 3), "reference_iters": sref["iters"]})
    h.close()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--table", choices=("physical", "synthetic"), default="physical")
    ap.add_argument("--apply-reps", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the 256x256x32 precision-form workload")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--counter-run", action="store_true",
                    help="only a 1 GiB device copy (counter calibration), 3 FP64 and 3 FP32 "
                         "applies at fixed launch shapes and one GMRES(30) cycle, for "
                         "hardware-counter passes")
    ap.add_argument("--counter-summary", nargs="+", metavar="DIR",
                    help="print the markdown summary of rocprofv3 --pmc runs of --counter-run "
                         "(their output directories) and exit")
    ap.add_argument("--block-buffers", type=int, default=4,
                    help="FP64 block-product variant in --counter-run (1 or 2 prefetch sets, 3 = "
                         "two workgroups per CU, 4 = the next row staged into a second LDS "
                         "buffer; giem_tune chooses 4 for FP64 on this workload)")
    ap.add_argument("--table-build", action="store_true",
                    help="only time giem_tables for the benchmark model of Sect. 4 on "
                         "176x224x118 cells of 25 m, for one and for two frequencies, and exit")
    args = ap.parse_args()
    if args.counter_summary:
        print(counter_summary(args.counter_summary))
        return
    if args.gpus != 1:
        print(f"bench.py: this solver runs on one GPU; --gpus {args.gpus} is not supported "
              "(independent frequencies and models shard across GPUs without communication, "
              "which is not part of this benchmark)", file=sys.stderr)
        sys.exit(2)

    import torch
    import giem_synth as gs
    import paper_1512_06126_amd as g
    g.load()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    if args.table_build:
        m = gs.config_commemi3d3()
        for nf in (1, 2):
            freqs = m["freq"] * 2.0 ** np.arange(nf)
            t0 = time.perf_counter()
            h = g.tables(m, freqs)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            h.close()
            print(f"giem_tables, {m['nx']}x{m['ny']}x{m['nz']} cells, {nf} frequencies: "
                  f"{dt:.2f} s", flush=True)
        return

    model = gs.config_128x128x32()
    nx, ny, nz = model["nx"], model["ny"], model["nz"]
    R = 2
    f = model["freq"]
    t_tab = time.perf_counter()
    if args.table == "physical":
        h = g.tables(model, [f], flags=g.TABLES_C64)
        table = None
    else:
        table = synthetic_table(model)
        h = g.tables_import(model, [f], table[None], flags=g.TABLES_C64)
    torch.cuda.synchronize()
    table_s = time.perf_counter() - t_tab
    sa = torch.from_numpy(np.ascontiguousarray(model["sigma_a"])).to(dev)
    E = torch.zeros((R, 3, nz, ny, nx), dtype=torch.complex128, device=dev)

    if args.counter_run:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)   # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        x = torch.randn((R, 3, nz, ny, nx), dtype=torch.complex128, device=dev)
        y = torch.empty_like(x)
        # the launch shapes giem_tune chose in the timed runs of this workload
        # (tuning under the profiler would time perturbed candidates)
        fft_shape = {"fp64": [(8, 256), (16, 256), (16, 256), (8, 256)],
                     "fp32": [(16, 256), (16, 256), (16, 256), (8, 256)]}
        h.set_fft_shape(g.FP64, fft_shape["fp64"])
        h.set_fft_shape(g.FP32, fft_shape["fp32"])
        h.set_block_buffers(g.FP32, 1)
        h.set_block_buffers(g.FP64, args.block_buffers)
        for _ in range(3):
            h.apply(x, y, sa, prec=g.FP64)
        for _ in range(3):
            h.apply(x, y, sa, prec=g.FP32)
        # one GMRES(30) cycle: the Gram-Schmidt kernels at j = 0 .. 29
        st = h.solve(sa, E, tol=1e-30, restart=30, max_iter=30, precision=g.FP64)
        torch.cuda.synchronize()
        print(f"counter run done: copy 1073741824 B, 3 FP64 and 3 FP32 applies, one GMRES(30) "
              f"cycle of {st['iters']} steps (block-product variant {args.block_buffers}; "
              f"tuned {fft_shape})", flush=True)
        h.close()
        return

    # launch shapes of the FFT passes, tuned once per handle (not timed)
    t_tune = time.perf_counter()
    fft_shape = h.tune(sa, nrhs=R)
    torch.cuda.synchronize()
    tune_s = time.perf_counter() - t_tune

    def solve(prec, tol, out=E):
        return h.solve(sa, out, tol=tol, restart=30, max_iter=3000, precision=prec,
                       inner_tol=1e-3, max_outer=30)

    for _ in range(args.warmup):
        solve(g.FP64, 1e-6)
    torch.cuda.synchronize()
    # the dominant kernel, from one solve with all five kernels bracketed
    # (outside the timed region); the timed solves bracket only that kernel,
    # two events per apply instead of six
    h.profile(True)
    solve(g.FP64, 1e-6)
    dom = int(np.argmax(h.profile_read()["fp64"]["stage_ms"]))
    h.profile(True, stage=dom)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = [solve(g.FP64, 1e-6) for _ in range(args.steps)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = h.profile_read()
    h.profile(False)
    p64 = prof["fp64"]
    rhs_applies = p64["rhs"]
    ms_per_step = 1e3 * wall / args.steps
    value = rhs_applies / wall

    # roofline of the dominant kernel, from the events of the timed region
    name = STAGES[dom]
    avg_ms = p64["stage_ms"][dom] / max(p64["applies"], 1)
    # right-hand sides used per launch: the few vectors GMRES queued ahead
    # and discarded are not counted, so the byte figure errs low
    avg_rhs = p64["rhs"] / max(p64["applies"], 1)
    bytes_launch = stage_bytes(nx, ny, nz, avg_rhs, 16)[name]
    achieved = bytes_launch / (avg_ms * 1e-3) / 1e9
    traffic = read_traffic(fft_shape["block_buffers"]["fp64"]) if name == "block_product" else None
    roofline = {"bound": "hbm", "kernel": name, "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic, "bytes_per_launch": bytes_launch,
                "avg_launch_ms": round(avg_ms, 5), "launches": p64["applies"]}

    # the apply alone, both precisions
    x = torch.randn((R, 3, nz, ny, nx), dtype=torch.complex128, device=dev)
    y = torch.empty_like(x)
    apply = {}
    for prec, key, c in ((g.FP64, "fp64", 16), (g.FP32, "fp32", 8)):
        for _ in range(3):
            h.apply(x, y, sa, prec=prec)
        torch.cuda.synchronize()
        st = np.array([h.apply_timed(x, y, sa, prec=prec) for _ in range(args.apply_reps)])
        med = np.median(st, axis=0)
        tot = float(med.sum())
        m3 = m3_bytes(nx, ny, nz, R, c)
        apply[key] = {"ms_per_apply": round(tot, 4), "rhs_applies_per_s": round(R / tot * 1e3, 1),
                      "stage_ms": [round(v, 4) for v in med], "m3_bytes": m3,
                      "hbm_frac_m3": round(m3 / (tot * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                      "min_ms": round(float(st.sum(1).min()), 4),
                      "max_ms": round(float(st.sum(1).max()), 4)}

    if table is None and not args.no_cpu:
        table = h.export(0)

    # FP32-refined solve vs FP64, both against a tight FP64 reference: at
    # the benchmark's tolerance, and at matched accuracy (for each form the
    # loosest tolerance whose field error is <= 1e-6)
    Eref = torch.zeros_like(E)
    sref = solve(g.FP64, 1e-12, Eref)
    E32 = torch.zeros_like(E)
    solve(g.FP32, 1e-6, E32)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    s32 = [solve(g.FP32, 1e-6, E32) for _ in range(max(1, args.steps // 2))]
    torch.cuda.synchronize()
    ms32 = 1e3 * (time.perf_counter() - t1) / len(s32)

    solve_info = {
        "fp64_ms": round(ms_per_step, 3), "fp64_iters": stats[-1]["iters"],
        "fp64_rel_residual": stats[-1]["rel_residual"],
        "fp64_field_err": relerr(E, Eref),
        "fp32_refined_ms": round(ms32, 3), "fp32_refined_inner_iters": s32[-1]["iters"],
        "fp32_refined_outer": s32[-1]["outer_iters"],
        "fp32_refined_field_err": relerr(E32, Eref),
        "speedup_fp32_refined_at_tol_1e-6": round(ms_per_step / ms32, 3),
        "matched_accuracy": matched_accuracy(g, solve, E, Eref, max(2, args.steps // 2)),
        "reference_iters": sref["iters"], "table_build_s": round(table_s, 3),
        "fft_tune_s": round(tune_s, 3), "fft_shape": fft_shape,
    }
    h.close()
    del Eref, E32
    extra = None if args.no_extra else precision_workload(g, torch, dev)

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(model, table, args.cpu_seconds)

    line = {
        "metric": "IE operator applies/s + GMRES solve time to 1e-6, FP32-refined vs FP64, HBM %",
        "value": round(value, 2), "unit": "RHS-applies/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "c128",
        "data": "synthetic (seeded layered-earth model; tables computed by giem_tables)" if args.table == "physical" else "synthetic (random stand-in table)",
        "config": {"workload": "128x128x32 cells of 200x200x100 m, 5-layer earth, 3 blocks "
                               "contrast <= 1e4, f = 0.01 Hz, 2 plane-wave RHS, GMRES(30) "
                               "to 1e-6, FP64",
                   "table": args.table, "rhs": R},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "apply": apply,
        "solve": solve_info,
        "precision_256x256x32": extra,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
