"""Entropic optimal transport on a tree metric by Sinkhorn scaling, with
every kernel-vector product K x computed by the tree field integrator.

Follows the paper's Sinkhorn implementation appendix: FP64 scaling vectors
started at u = v = 1, the alternating updates
    u <- a / (K v + delta),   v <- b / (K u + delta),   delta = 1e-30
(K is symmetric), and the absolute marginal residual
    R_t = max(|u * (K v) - a|_inf, |v * (K u) - b|_inf)
checked after the first iteration and every 20 iterations thereafter. The
products run on the GPU in the kernel table's precision; the vectors are
rounded to it before each product.
"""
from __future__ import annotations

import torch


def sinkhorn(integrator, f, a, b, iters=200, delta=1e-30, tol=None, check_every=20,
             on_product=None):
    """Run ``iters`` Sinkhorn iterations (or stop at the first residual
    check below ``tol``).

    integrator  TreeIntegrator of the tree; f its kernel table (device), or
                a pair (c, lam) of device tensors for f(k) = sum_l c_l lam_l^k,
                whose products then run through the backbone sweeps
                (``integrate_expsum``)
    a, b        marginals, device tensors [N] (any float dtype; kept FP64)
    on_product  optional callback(x_in, Kx) after every product (for checks)
    Returns (u, v, residuals) with residuals a list of (t, R_t).
    """
    a = a.to(torch.float64)
    b = b.to(torch.float64)
    u = torch.ones_like(a)
    v = torch.ones_like(b)

    sweeps = isinstance(f, tuple)
    dtype = f[0].dtype if sweeps else f.dtype

    def K(x):
        xin = x.to(dtype).contiguous()
        y = integrator.integrate_expsum(f[0], f[1], xin) if sweeps else integrator.integrate(f, xin)
        if on_product is not None:
            on_product(xin, y)
        return y.to(torch.float64)

    residuals = []
    for t in range(1, iters + 1):
        u = a / (K(v) + delta)
        v = b / (K(u) + delta)
        if t == 1 or (t - 1) % check_every == 0:
            r = max((u * K(v) - a).abs().max().item(), (v * K(u) - b).abs().max().item())
            residuals.append((t, r))
            if tol is not None and r < tol:
                break
    return u, v, residuals
