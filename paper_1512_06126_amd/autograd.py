"""torch.autograd wrapper: impedance tensors as a differentiable function of
log sigma_a (argument marshalling only; every step runs in libgiem).

Forward, per frequency: giem_solve with the plane-wave source (x and y
polarisation), giem_fields at the receivers, giem_impedance.
Backward, per frequency: giem_impedance_adjoint turns the incoming gradient
with respect to Z into weights on the receiver fields, giem_fields_adjoint
turns those into the adjoint source and the explicit part of the gradient,
and giem_adjoint adds the part that flows through the cell field by one
solve with A^T.  The gradient is exact for real conductivities (Sect. 4
uses real sigma); the imaginary part of log sigma is not a parameter.
"""
from __future__ import annotations

import warnings

import numpy as np
import torch

from . import NotConverged, impedance, impedance_adjoint


class _ImpedanceFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, log_sigma, handle, rec, ifreqs, opts):
        sa = torch.exp(log_sigma.detach()).to(torch.complex128).contiguous()
        nz, ny, nx = sa.shape
        nrec = rec.shape[0]
        Z = torch.empty((len(ifreqs), nrec, 2, 2), dtype=torch.complex128, device=sa.device)
        saved = []
        for i, f in enumerate(ifreqs):
            E = torch.zeros((2, 3, nz, ny, nx), dtype=torch.complex128, device=sa.device)
            st = handle.solve(sa, E, tol=opts["tol"], restart=opts["restart"],
                              max_iter=opts["max_iter"], ifreq=f)
            if st["converged"] != 1:
                warnings.warn(f"forward solve at frequency {f} stopped at relative residual "
                              f"{st['rel_residual']:.2e}", NotConverged)
            Er = torch.empty((2, nrec, 3), dtype=torch.complex128, device=sa.device)
            Hr = torch.empty_like(Er)
            handle.fields(sa, E, rec, Er, Hr, ifreq=f)
            impedance(Er, Hr, Z[i])
            saved.append((E, Er, Hr))
        ctx.handle, ctx.rec, ctx.ifreqs, ctx.opts = handle, rec, ifreqs, opts
        ctx.sa, ctx.saved = sa, saved
        return Z

    @staticmethod
    def backward(ctx, gZ):
        sa, opts = ctx.sa, ctx.opts
        gZ = gZ.to(torch.complex128).contiguous()
        grad = torch.zeros(sa.shape, dtype=torch.float64, device=sa.device)
        for i, f in enumerate(ctx.ifreqs):
            E, Er, Hr = ctx.saved[i]
            wE, wH = torch.empty_like(Er), torch.empty_like(Er)
            impedance_adjoint(Er, Hr, gZ[i], wE, wH)
            g = torch.empty_like(E)
            ctx.handle.fields_adjoint(sa, E, ctx.rec, wE, wH, g, grad, ifreq=f)
            st = ctx.handle.adjoint(sa, g, E, grad, tol=opts["adj_tol"], restart=opts["restart"],
                                    max_iter=opts["max_iter"], ifreq=f)
            if st["converged"] != 1:
                warnings.warn(f"adjoint solve at frequency {f} stopped at relative residual "
                              f"{st['rel_residual']:.2e}", NotConverged)
        return grad, None, None, None, None


def impedance_tensor(handle, log_sigma, rec_xyz, ifreqs=None, tol=1e-10, adj_tol=None,
                     restart=30, max_iter=4000):
    """Z [nfreq][nrec][2][2] (complex128, on log_sigma's device) for the
    anomaly conductivity exp(log_sigma) ([Nz][Ny][Nx], float64), receivers
    rec_xyz [nrec][3] (or (x, y) pairs [nrec][2], placed on the surface) above
    cell centres and the handle's frequencies ifreqs
    (all by default).  Differentiable with respect to log_sigma."""
    if ifreqs is None:
        ifreqs = list(range(len(handle.freqs)))
    rec = handle.receivers(rec_xyz)
    opts = dict(tol=tol, adj_tol=tol if adj_tol is None else adj_tol, restart=restart,
                max_iter=max_iter)
    return _ImpedanceFn.apply(log_sigma, handle, rec, list(ifreqs), opts)
