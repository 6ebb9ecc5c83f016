"""Python binding of libgiem (include/giem.h): argument marshalling only.

Every step of the solver runs in the HIP library; this module converts model
descriptions to the C structs, passes torch tensors' device pointers and the
current HIP stream, and turns error codes into exceptions.  It never computes
anything itself and it fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "lib", "libgiem.so")

GIEM_OK, GIEM_EINVAL, GIEM_EDOMAIN, GIEM_ENOMEM, GIEM_EHIP, GIEM_ENOCONV = 0, -1, -2, -3, -4, 1
MODE_A, MODE_AT, MODE_B = 0, 1, 2
FP64, FP32 = 0, 1
TABLES_C64 = 1

_lib = None


class GiemError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"giem error {code}: {msg}")
        self.code = code


class NotConverged(RuntimeWarning):
    pass


class _Model(ctypes.Structure):
    _fields_ = [("nlay", ctypes.c_int32), ("d", ctypes.c_void_p), ("sigma_b", ctypes.c_void_p),
                ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("hx", ctypes.c_double), ("hy", ctypes.c_double), ("x0", ctypes.c_double),
                ("y0", ctypes.c_double), ("z_edges", ctypes.c_void_p)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("restart", ctypes.c_int32),
                ("max_iter", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("inner_tol", ctypes.c_double), ("max_outer", ctypes.c_int32),
                ("weighted_ip", ctypes.c_int32), ("warm_start", ctypes.c_int32),
                ("graph", ctypes.c_int32)]


class SolveGroup(ctypes.Structure):
    _fields_ = [("t", ctypes.c_void_p), ("nf", ctypes.c_int32), ("ifreqs", ctypes.c_void_p),
                ("sigma_a", ctypes.c_void_p), ("rhs", ctypes.c_void_p),
                ("E_cells", ctypes.c_void_p)]


HISTORY = 64


class SolveStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("outer_iters", ctypes.c_int32),
                ("converged", ctypes.c_int32), ("rel_residual", ctypes.c_double),
                ("ms", ctypes.c_double), ("n_history", ctypes.c_int32),
                ("history", ctypes.c_double * HISTORY)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k not in ("n_history", "history")}
        d["history"] = [self.history[i] for i in range(self.n_history)]
        return d


def load():
    """Load libgiem.so (built by __graft_entry__.build()); raise if missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIBPATH):
        raise ImportError(f"HIP library not built: {LIBPATH} is missing "
                          "(run __graft_entry__.build())")
    # torch ships its own HIP runtime; load it first so that libgiem binds to
    # the same libamdhip64 instance (one runtime, one device context).
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIBPATH)
    P, I32, U32, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32, ctypes.c_double
    sig = {
        "giem_tables": [P, I32, P, U32, P, P],
        "giem_tables_import": [P, I32, P, P, U32, P, P],
        "giem_tables_export": [P, I32, P],
        "giem_tables_bytes": [P, P, P],
        "giem_apply": [P, I32, P, I32, P, P, U32, U32, P],
        "giem_apply_noalloc": [P, I32, P, I32, P, P, U32, U32, P],
        "giem_apply_timed": [P, I32, P, I32, P, P, U32, U32, P, P],
        "giem_apply_batch": [P, I32, P, P, I32, P, P, U32, U32, P],
        "giem_solve": [P, I32, P, I32, P, P, P, P, P],
        "giem_solve_multi": [I32, P, I32, P, P, P],
        "giem_solve_batch": [P, I32, P, P, I32, P, P, P, P, P],
        "giem_adjoint": [P, I32, P, I32, P, P, P, P, P, P],
        "giem_fields": [P, I32, P, I32, P, I32, P, P, P, P],
        "giem_fields_adjoint": [P, I32, P, I32, P, I32, P, P, P, P, P, P],
        "giem_fields_anomalous": [P, I32, P, I32, P, I32, P, P, P, P],
        "giem_dipole_source": [P, I32, I32, P, P, P, P],
        "giem_impedance": [I32, P, P, P, P],
        "giem_impedance_adjoint": [I32, P, P, P, P, P, P],
        "giem_profile": [P, I32],
        "giem_tune": [P, I32, P, I32, P, P],
        "giem_set_fft_shape": [P, U32, P],
        "giem_set_block_buffers": [P, U32, I32],
        "giem_profile_read": [P, P, P, P],
        "giem_free": [P],
        "giem_last_error": [],
    }
    for name, argt in sig.items():
        f = getattr(lib, name)
        f.argtypes = argt
        f.restype = ctypes.c_int
    lib.giem_free.restype = None
    lib.giem_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def exported_symbols():
    return ["giem_tables", "giem_tables_import", "giem_tables_export", "giem_tables_bytes",
            "giem_apply", "giem_apply_noalloc", "giem_apply_timed", "giem_apply_batch", "giem_tune", "giem_set_fft_shape", "giem_set_block_buffers", "giem_profile", "giem_profile_read", "giem_solve", "giem_solve_batch", "giem_solve_multi",
            "giem_adjoint", "giem_fields", "giem_fields_anomalous", "giem_fields_adjoint",
            "giem_dipole_source", "giem_impedance",
            "giem_impedance_adjoint", "giem_free", "giem_last_error"]


def _check(rc, allow_noconv=False):
    if rc == GIEM_OK:
        return rc
    msg = _lib.giem_last_error().decode()
    if rc == GIEM_ENOCONV and allow_noconv:
        return rc
    raise GiemError(rc, msg)


def _stream(stream):
    if stream is not None:
        return ctypes.c_void_p(stream)
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _model_struct(m):
    keep = {
        "d": np.ascontiguousarray(m["d"], dtype=np.float64),
        "sigma": np.ascontiguousarray(m["sigma"], dtype=np.complex128),
        "z": np.ascontiguousarray(m["z_edges"], dtype=np.float64),
    }
    s = _Model(nlay=keep["d"].size, d=keep["d"].ctypes.data, sigma_b=keep["sigma"].ctypes.data,
               nx=m["nx"], ny=m["ny"], nz=m["nz"], hx=m["hx"], hy=m["hy"],
               x0=m.get("x0", 0.0), y0=m.get("y0", 0.0), z_edges=keep["z"].ctypes.data)
    return s, keep


class Handle:
    """Owns a giem_handle (device tables + workspace)."""

    def __init__(self, ptr, model, freqs):
        self._p = ctypes.c_void_p(ptr)
        self.model = model
        self.freqs = np.asarray(freqs, dtype=np.float64)

    def close(self):
        if self._p and self._p.value:
            _lib.giem_free(self._p)
            self._p = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def export(self, ifreq=0):
        nz = self.model["nz"]
        e = 2 * nz * (2 * nz + 1)
        out = np.empty((self.model["ny"], self.model["nx"], e), dtype=np.complex128)
        _check(_lib.giem_tables_export(self._p, ifreq, out.ctypes.data))
        return out

    def table_bytes(self):
        a, b = ctypes.c_int64(), ctypes.c_int64()
        _check(_lib.giem_tables_bytes(self._p, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def apply(self, x, y, sigma_a=None, mode=MODE_A, prec=FP64, ifreq=0, stream=None):
        nrhs = x.shape[0]
        sa = _ptr(sigma_a) if sigma_a is not None else ctypes.c_void_p(0)
        _check(_lib.giem_apply(self._p, ifreq, sa, nrhs, _ptr(x), _ptr(y), mode, prec,
                               _stream(stream)))
        return y

    def apply_noalloc(self, x, y, sigma_a=None, mode=MODE_A, prec=FP64, ifreq=0, stream=None):
        """giem_apply_noalloc: the same apply with its spectra in the library's
        fixed device array (no allocation during the call)."""
        nrhs = x.shape[0]
        sa = _ptr(sigma_a) if sigma_a is not None else ctypes.c_void_p(0)
        _check(_lib.giem_apply_noalloc(self._p, ifreq, sa, nrhs, _ptr(x), _ptr(y), mode, prec,
                                       _stream(stream)))
        return y

    def apply_batch(self, x, y, sigma_a=None, ifreqs=None, mode=MODE_A, prec=FP64, stream=None):
        """y[f] = op_{ifreqs[f]} x[f] for x, y of shape [nf][nrhs][3][Nz][Ny][Nx]
        (complex128, on the device), one launch per kernel for all nf
        frequencies; ifreqs defaults to 0 .. nf - 1."""
        nf, nrhs = x.shape[0], x.shape[1]
        ifr = list(range(nf)) if ifreqs is None else [int(q) for q in ifreqs]
        if len(ifr) != nf:
            raise ValueError("one frequency index per leading slice of x")
        arr = (ctypes.c_int32 * nf)(*ifr)
        sa = _ptr(sigma_a) if sigma_a is not None else ctypes.c_void_p(0)
        _check(_lib.giem_apply_batch(self._p, nf, arr, sa, nrhs, _ptr(x), _ptr(y), mode, prec,
                                     _stream(stream)))
        return y

    def apply_timed(self, x, y, sigma_a=None, mode=MODE_A, prec=FP64, ifreq=0, stream=None):
        nrhs = x.shape[0]
        sa = _ptr(sigma_a) if sigma_a is not None else ctypes.c_void_p(0)
        ms = (ctypes.c_double * 5)()
        _check(_lib.giem_apply_timed(self._p, ifreq, sa, nrhs, _ptr(x), _ptr(y), mode, prec,
                                     _stream(stream), ms))
        return list(ms)

    def tune(self, sigma_a, nrhs=2, ifreq=0, stream=None):
        """Time the FFT launch shapes and the block-product variants on this
        handle and keep the fastest; returns {"fp64"|"fp32": [(sequences,
        threads) per pass], "block_buffers": {"fp64"|"fp32": 1, 2 or 3}}
        (see set_block_buffers)."""
        ch = (ctypes.c_int32 * 20)()
        _check(_lib.giem_tune(self._p, ifreq, _ptr(sigma_a), nrhs, _stream(stream), ch))
        out = {k: [(ch[(i * 5 + j) * 2], ch[(i * 5 + j) * 2 + 1]) for j in range(4)]
               for i, k in enumerate(("fp64", "fp32"))}
        out["block_buffers"] = {k: ch[(i * 5 + 4) * 2] for i, k in enumerate(("fp64", "fp32"))}
        return out

    def set_fft_shape(self, prec, shape=None):
        """shape: four (sequences, threads) pairs, or None for the built-in choice."""
        if shape is None:
            _check(_lib.giem_set_fft_shape(self._p, prec, None))
            return
        arr = (ctypes.c_int32 * 8)(*[int(v) for pair in shape for v in pair])
        _check(_lib.giem_set_fft_shape(self._p, prec, arr))

    def set_block_buffers(self, prec, nbuf):
        """Variant of the block product: 1 or 2 prefetch sets in one
        workgroup per CU, 3 = two workgroups per CU, 4 = the next point's row
        staged into a second LDS buffer during the current point (0 = built-in, 1)."""
        _check(_lib.giem_set_block_buffers(self._p, prec, nbuf))

    def profile(self, enable=True, stage=None):
        """Record HIP events around the kernels of every later apply: all
        five (stage None) or only kernel `stage` (0 .. 4, the order of
        apply_timed), which adds two events per apply instead of six."""
        code = 0 if not enable else (1 if stage is None else 2 + int(stage))
        _check(_lib.giem_profile(self._p, code))

    def profile_read(self):
        """Summed kernel times per precision since the last read:
        {"fp64"|"fp32": {"stage_ms": [5], "applies": n, "rhs": n}}."""
        ms = (ctypes.c_double * 10)()
        ap = (ctypes.c_int64 * 2)()
        rh = (ctypes.c_int64 * 2)()
        _check(_lib.giem_profile_read(self._p, ms, ap, rh))
        return {k: {"stage_ms": list(ms[5 * i:5 * i + 5]), "applies": ap[i], "rhs": rh[i]}
                for i, k in enumerate(("fp64", "fp32"))}

    def solve(self, sigma_a, E_out, rhs=None, tol=1e-6, restart=30, max_iter=2000,
              precision=FP64, inner_tol=1e-3, max_outer=20, weighted_ip=0, warm_start=0,
              ifreq=0, stream=None, graph=0):
        o = SolveOpts(tol=tol, restart=restart, max_iter=max_iter, precision=precision,
                      inner_tol=inner_tol, max_outer=max_outer, weighted_ip=weighted_ip,
                      warm_start=warm_start, graph=graph)
        st = SolveStats()
        nrhs = E_out.shape[0]
        rp = _ptr(rhs) if rhs is not None else ctypes.c_void_p(0)
        rc = _lib.giem_solve(self._p, ifreq, _ptr(sigma_a), nrhs, rp, _ptr(E_out),
                             ctypes.byref(o), ctypes.byref(st), _stream(stream))
        _check(rc, allow_noconv=True)
        d = st.as_dict()
        d["rc"] = rc
        return d

    def solve_batch(self, sigma_a, E_outs, ifreqs=None, rhs=None, tol=1e-6, restart=30,
                    max_iter=2000, precision=FP64, inner_tol=1e-3, max_outer=20, weighted_ip=0,
                    warm_start=0, stream=None, graph=0):
        """Solve at several frequencies at once: E_outs[f] receives the
        solution at frequency ifreqs[f] (all frequencies by default); rhs is
        None (plane waves) or a list of tensors.  Returns one stats dict per
        frequency."""
        nf = len(E_outs)
        if ifreqs is None:
            ifreqs = list(range(nf))
        fi = (ctypes.c_int32 * nf)(*ifreqs)
        ep = (ctypes.c_void_p * nf)(*[e.data_ptr() for e in E_outs])
        rp = None
        if rhs is not None:
            rp = (ctypes.c_void_p * nf)(*[(r.data_ptr() if r is not None else None) for r in rhs])
        o = SolveOpts(tol=tol, restart=restart, max_iter=max_iter, precision=precision,
                      inner_tol=inner_tol, max_outer=max_outer, weighted_ip=weighted_ip,
                      warm_start=warm_start, graph=graph)
        st = (SolveStats * nf)()
        rc = _lib.giem_solve_batch(self._p, nf, fi, _ptr(sigma_a), E_outs[0].shape[0], rp, ep,
                                   ctypes.byref(o), st, _stream(stream))
        _check(rc, allow_noconv=True)
        out = []
        for k in range(nf):
            d = st[k].as_dict()
            d["rc"] = rc
            out.append(d)
        return out

    def adjoint(self, sigma_a, adj_src, E_fwd, grad, tol=1e-10, restart=30, max_iter=4000,
                weighted_ip=0, ifreq=0, stream=None):
        o = SolveOpts(tol=tol, restart=restart, max_iter=max_iter, precision=FP64,
                      inner_tol=0.0, max_outer=0, weighted_ip=weighted_ip, warm_start=0)
        st = SolveStats()
        rc = _lib.giem_adjoint(self._p, ifreq, _ptr(sigma_a), adj_src.shape[0], _ptr(adj_src),
                               _ptr(E_fwd), _ptr(grad), ctypes.byref(o), ctypes.byref(st),
                               _stream(stream))
        _check(rc, allow_noconv=True)
        d = st.as_dict()
        d["rc"] = rc
        return d

    def receivers(self, rec):
        """Receiver (or source) positions as host float64 [nrec][3]; (x, y)
        pairs are placed on the earth's surface z = d[0] of the handle's model."""
        rec = np.asarray(rec, dtype=np.float64)
        if rec.ndim == 2 and rec.shape[1] == 2:
            rec = np.concatenate([rec, np.full((rec.shape[0], 1), float(self.model["d"][0]))], 1)
        return np.ascontiguousarray(rec.reshape(-1, 3))

    def fields(self, sigma_a, E_cells, rec_xyz, E_rec, H_rec, ifreq=0, stream=None,
               anomalous=False):
        """giem_fields (plane-wave normal fields added for RHS 0 and 1), or
        giem_fields_anomalous (the anomalous fields only, for any source)."""
        rec = self.receivers(rec_xyz)
        fn = _lib.giem_fields_anomalous if anomalous else _lib.giem_fields
        _check(fn(self._p, ifreq, _ptr(sigma_a), E_cells.shape[0], _ptr(E_cells), rec.shape[0],
                  rec.ctypes.data, _ptr(E_rec), _ptr(H_rec), _stream(stream)))
        return E_rec, H_rec

    def dipole_source(self, src_xyz, moments, rhs, ifreq=0, stream=None):
        """giem_dipole_source: rhs [nsrc][3][Nz][Ny][Nx] (complex128, on the
        device) receives the right-hand side of electric dipoles of moments
        [nsrc][3] (A m) at src_xyz [nsrc][3] (or (x, y) on the surface), to be
        passed to solve(rhs=...)."""
        src = self.receivers(src_xyz)
        mom = np.ascontiguousarray(np.asarray(moments, dtype=np.complex128).reshape(-1, 3))
        _check(_lib.giem_dipole_source(self._p, ifreq, src.shape[0], src.ctypes.data,
                                       mom.ctypes.data, _ptr(rhs), _stream(stream)))
        return rhs

    def fields_adjoint(self, sigma_a, E_cells, rec_xyz, wE, wH, adj_src, grad, ifreq=0,
                       stream=None):
        rec = self.receivers(rec_xyz)
        _check(_lib.giem_fields_adjoint(self._p, ifreq, _ptr(sigma_a), E_cells.shape[0],
                                        _ptr(E_cells), rec.shape[0], rec.ctypes.data, _ptr(wE),
                                        _ptr(wH), _ptr(adj_src), _ptr(grad), _stream(stream)))
        return adj_src, grad


def solve_multi(groups, tol=1e-6, restart=30, max_iter=2000, precision=FP64, inner_tol=1e-3,
                max_outer=20, weighted_ip=0, warm_start=0, stream=None):
    """giem_solve_multi: groups is a list of (handle, sigma_a, E_outs, ifreqs,
    rhs) tuples (ifreqs None: all of the handle's frequencies; rhs None: plane
    waves, else a list of tensors); every E_outs[f] has the same number of
    right-hand sides.  Returns one stats dict per (group, frequency)."""
    load()
    keep = []
    arr = (SolveGroup * len(groups))()
    nrhs = None
    total = 0
    for g, (h, sa, E_outs, ifreqs, rhs) in enumerate(groups):
        nf = len(E_outs)
        if ifreqs is None:
            ifreqs = list(range(nf))
        fi = (ctypes.c_int32 * nf)(*ifreqs)
        ep = (ctypes.c_void_p * nf)(*[e.data_ptr() for e in E_outs])
        rp = None
        if rhs is not None:
            rp = (ctypes.c_void_p * nf)(*[(r.data_ptr() if r is not None else None) for r in rhs])
        keep += [fi, ep, rp]
        arr[g] = SolveGroup(t=h._p, nf=nf, ifreqs=ctypes.cast(fi, ctypes.c_void_p),
                            sigma_a=sa.data_ptr(), rhs=ctypes.cast(rp, ctypes.c_void_p) if rp else None,
                            E_cells=ctypes.cast(ep, ctypes.c_void_p))
        nrhs = E_outs[0].shape[0]
        total += nf
    o = SolveOpts(tol=tol, restart=restart, max_iter=max_iter, precision=precision,
                  inner_tol=inner_tol, max_outer=max_outer, weighted_ip=weighted_ip,
                  warm_start=warm_start, graph=1)
    st = (SolveStats * total)()
    rc = _lib.giem_solve_multi(len(groups), arr, nrhs, ctypes.byref(o), st, _stream(stream))
    _check(rc, allow_noconv=True)
    out = []
    for k in range(total):
        d = st[k].as_dict()
        d["rc"] = rc
        out.append(d)
    return out


def impedance(E_rec, H_rec, Z, stream=None):
    """Z [nrec][2][2] = Eh Hh^-1 from the fields of the two polarisations."""
    load()
    _check(_lib.giem_impedance(E_rec.shape[1], _ptr(E_rec), _ptr(H_rec), _ptr(Z),
                               _stream(stream)))
    return Z


def impedance_adjoint(E_rec, H_rec, gZ, wE, wH, stream=None):
    """Weights on the receiver fields from the gradient with respect to Z."""
    load()
    _check(_lib.giem_impedance_adjoint(E_rec.shape[1], _ptr(E_rec), _ptr(H_rec), _ptr(gZ),
                                       _ptr(wE), _ptr(wH), _stream(stream)))
    return wE, wH


def tables(model, freqs, flags=0, stream=None):
    load()
    s, keep = _model_struct(model)
    f = np.ascontiguousarray(np.atleast_1d(freqs), dtype=np.float64)
    out = ctypes.c_void_p()
    _check(_lib.giem_tables(ctypes.byref(s), f.size, f.ctypes.data, flags, _stream(stream),
                            ctypes.byref(out)))
    return Handle(out.value, model, f)


def tables_import(model, freqs, packed, flags=0, stream=None):
    load()
    s, keep = _model_struct(model)
    f = np.ascontiguousarray(np.atleast_1d(freqs), dtype=np.float64)
    pk = np.ascontiguousarray(packed, dtype=np.complex128)
    out = ctypes.c_void_p()
    _check(_lib.giem_tables_import(ctypes.byref(s), f.size, f.ctypes.data, pk.ctypes.data, flags,
                                   _stream(stream), ctypes.byref(out)))
    return Handle(out.value, model, f)
