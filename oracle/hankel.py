"""Hankel transforms used by the coefficient tables and the receiver kernels
(Appendix A: the horizontal integrals of J0(lambda rho) against functions of
lambda; J1 gives their radial derivatives for the fields at receivers).

  h(rho) = int_0^inf J0(lambda rho) g(lambda) dlambda   (order 0)
  h1(rho) = int_0^inf J1(lambda rho) g(lambda) dlambda  (order 1)

computed the plain way: Gauss-Legendre panels between consecutive zeros of
J0 (or J1) (a geometric subdivision of the first panel resolves the
structure of g at small lambda), and the oscillating algebraic tail beyond
the last panels summed by repeated pairwise averaging of the partial sums
(Euler's transform of an alternating series).
A log-divergent integrand at lambda -> 0 is regularised by subtracting 1 from
J0 below a fixed lambda_a; that only adds a rho-independent constant, which
the weights of the tables annihilate.

The lambda-functions come from boundary-value problems, so they are sampled
once on Chebyshev panels in t = ln(lambda) and interpolated (barycentric
formula); the transform at each rho is then a fixed linear combination of the
samples.  Radial results are likewise sampled on Chebyshev panels in ln(rho).
"""
from __future__ import annotations

import functools

import numpy as np
from scipy import special


def _lobatto(n):
    j = np.arange(n)
    x = np.cos(np.pi * j / (n - 1))[::-1]            # increasing
    w = (-1.0) ** j
    w[0] *= 0.5
    w[-1] *= 0.5
    return x, w[::-1] * ((-1.0) ** (n - 1))


class LogPanels:
    """Chebyshev-Lobatto panels of equal width in u = ln(x) on [x_lo, x_hi]."""

    def __init__(self, x_lo, x_hi, width=0.5, n=16):
        u0, u1 = np.log(x_lo), np.log(x_hi)
        npan = max(1, int(np.ceil((u1 - u0) / width)))
        self.edges = np.linspace(u0, u1, npan + 1)
        self.n = n
        xr, self.bw = _lobatto(n)
        self.xr = xr
        a, b = self.edges[:-1, None], self.edges[1:, None]
        self.u = 0.5 * (a + b) + 0.5 * (b - a) * xr[None, :]      # [npan, n]
        self.x = np.exp(self.u).reshape(-1)

    @property
    def size(self):
        return self.x.size

    def interp_rows(self, xq):
        """(column index [m, n], weight [m, n]) so that f(xq) ~ sum w f(nodes)."""
        uq = np.log(np.asarray(xq, dtype=np.float64))
        p = np.clip(np.searchsorted(self.edges, uq, side="right") - 1, 0, len(self.edges) - 2)
        a, b = self.edges[p], self.edges[p + 1]
        s = (2 * uq - (a + b)) / (b - a)                          # in [-1, 1]
        d = s[:, None] - self.xr[None, :]
        hit = np.abs(d) < 1e-14
        with np.errstate(divide="ignore", invalid="ignore"):
            t = self.bw[None, :] / d
            w = t / t.sum(axis=1, keepdims=True)
        rows_hit = hit.any(axis=1)
        if rows_hit.any():
            w[rows_hit] = hit[rows_hit].astype(float)
        cols = p[:, None] * self.n + np.arange(self.n)[None, :]
        return cols, w


@functools.lru_cache(maxsize=None)
def _gl(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return x, w


_ZEROS = {}


def _jn_zeros(order, count):
    """First count positive zeros of J_order (computed once, grown on demand)."""
    z = _ZEROS.get(order)
    if z is None or z.size < count:
        z = special.jn_zeros(order, max(count, 2 * (0 if z is None else z.size), 64))
        _ZEROS[order] = z
    return z[:count]


def _averaged_limit(S, levels=14):
    """Limit of partial sums S[k, f] over consecutive half-periods of an
    oscillating tail by repeated pairwise averaging (Euler's transform of an
    alternating series): linear, and stable against rounding in S."""
    T = np.asarray(S)
    for _ in range(min(levels, T.shape[0] - 1)):
        T = 0.5 * (T[1:] + T[:-1])
    return T[-1]


def transform_weights(lp, rho, lam_a, lam_lo, lam_asym, ntail=30, n_gl=16, order=0, n_gl0=12):
    """Weights over the samples of lp (LogPanels in lambda) such that
      main @ g  = int over [lam_lo, lambda_K] of J_order(lambda rho) g
      tail[k] @ g = integral over the k-th panel after lambda_K,
      corr @ g  = int over [lam_lo, lam_a] of g (for the regularised kind).
    lambda_K is the first zero of J_order beyond lam_asym."""
    ncols = lp.size
    jn = special.j0 if order == 0 else special.j1
    K = int(np.ceil(lam_asym * rho / np.pi)) + 1
    zeros = _jn_zeros(order, K + ntail + 1) / rho
    l1 = zeros[0]
    # geometric subpanels of [lam_lo, l1], with lam_a as a breakpoint
    brk = [l1]
    while brk[-1] / 2.0 > lam_lo:
        brk.append(brk[-1] / 2.0)
    brk.append(lam_lo)
    brk = sorted(set(brk + ([lam_a] if lam_lo < lam_a < l1 else [])))
    xg, wg = _gl(n_gl0)
    pa = np.array(brk[:-1])[:, None]
    pb = np.array(brk[1:])[:, None]
    nod0 = (0.5 * (pa + pb) + 0.5 * (pb - pa) * xg[None, :]).ravel()
    w0 = (0.5 * (pb - pa) * wg[None, :]).ravel()
    # zero panels up to lambda_K
    xg2, wg2 = _gl(n_gl)
    za = np.concatenate([[l1], zeros[1:K]])[:-1][:, None]
    zb = zeros[1:K][:, None]
    if zb.size:
        nod1 = (0.5 * (za + zb) + 0.5 * (zb - za) * xg2[None, :]).ravel()
        w1 = (0.5 * (zb - za) * wg2[None, :]).ravel()
    else:
        nod1 = np.zeros(0)
        w1 = np.zeros(0)
    nodes = np.concatenate([nod0, nod1])
    wts = np.concatenate([w0, w1]) * jn(nodes * rho)
    main = np.zeros(ncols)
    cols, iw = lp.interp_rows(nodes)
    np.add.at(main, cols.ravel(), (wts[:, None] * iw).ravel())
    # regularisation row (rho-independent): int_{lam_lo}^{lam_a} g
    corr = np.zeros(ncols)
    sel = nod0 < lam_a
    if sel.any():
        c2, i2 = lp.interp_rows(nod0[sel])
        np.add.at(corr, c2.ravel(), (w0[sel][:, None] * i2).ravel())
    # tail panels
    tail = np.zeros((ntail, ncols))
    a = zeros[K - 1:K - 1 + ntail][:, None]
    b = zeros[K:K + ntail][:, None]
    nd = 0.5 * (a + b) + 0.5 * (b - a) * xg2[None, :]          # [ntail, n_gl]
    ww = 0.5 * (b - a) * wg2[None, :] * jn(nd * rho)
    c3, i3 = lp.interp_rows(nd.ravel())
    rows = np.repeat(np.arange(ntail), xg2.size)
    np.add.at(tail, (np.repeat(rows, i3.shape[1]), c3.ravel()), (ww.ravel()[:, None] * i3).ravel())
    return main, tail, corr


def hankel_on_grid(G, lp, rhos, reg, lam_a, lam_lo, lam_asym, ntail=30, order=0,
                   n_gl=16, n_gl0=12, levels=14):
    """h[rho, f] = int J_order(lambda rho) G[lambda, f] dlambda, with the
    regularisation (order 0 only) applied to the functions where reg[f] is
    True.  G holds the samples of g on lp's nodes, shape [lp.size, F]."""
    G = np.asarray(G)
    out = np.zeros((len(rhos), G.shape[1]), dtype=np.complex128)
    corr_val = None
    if order != 0:
        reg = np.zeros(G.shape[1], bool)
    for ir, rho in enumerate(rhos):
        main, tail, corr = transform_weights(lp, rho, lam_a, lam_lo, lam_asym, ntail, n_gl=n_gl,
                                             order=order, n_gl0=n_gl0)
        if corr_val is None:
            corr_val = corr @ G
        s0 = main @ G
        s0 = s0 - np.where(reg, corr_val, 0.0)
        parts = tail @ G
        S = s0[None, :] + np.cumsum(parts, axis=0)
        out[ir] = _averaged_limit(S, levels)
    return out
