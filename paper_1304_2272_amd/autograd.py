"""torch.autograd.Function over the library's forward and reverse passes.

``GwasGLS.apply(y, h2, Phi, XL, XR, sigma2, options)`` returns (b, var) for
every SNP row of XR under M = sigma2 (h2 Phi + (1 - h2) I), and its backward
gives dl/dy, dl/dh2 and (when sigma2 is a tensor) dl/dsigma2 for any scalar
loss l built from b and var with torch.  The covariance is assembled with
torch (input marshalling); every step of the GLS solves and of their reverse
pass runs in the HIP library.  With dM/dh2 = sigma2 (Phi - I) =
(M - sigma2 I) / h2 (h2 > 0) and dM/dsigma2 = M / sigma2 the library only
needs the contractions <Mbar, M> and tr Mbar.  As h2 -> 0 the two terms of
dl/dh2 = (<Mbar, M> - sigma2 tr Mbar) / h2 approach each other, and its
relative error grows like 1/h2 (about 5e-11 at h2 = 0.001 on the tests'
workloads).  One trait (y is an n-vector).
"""

from __future__ import annotations

import torch

from . import binding


class GwasGLS(torch.autograd.Function):
    @staticmethod
    def forward(ctx, y, h2, Phi, XL, XR, sigma2=1.0, options=None):
        opts = dict(options or {})
        n = Phi.shape[0]
        h = float(h2)
        if not h > 0.0:
            raise ValueError("the reverse pass needs h2 > 0")
        ctx.sigma2_is_tensor = torch.is_tensor(sigma2)
        sigma2 = float(sigma2)
        M = Phi * (sigma2 * h)
        M.diagonal().add_(sigma2 * (1.0 - h))
        g = binding.GwasContext(M, XL, y.detach().reshape(n, 1), **opts)
        del M
        b, var, info = g.stream_block(XR)
        ctx.g = g
        ctx.h2 = h
        ctx.sigma2 = float(sigma2)
        ctx.XR = XR
        ctx.save_for_backward(b, var, info)
        ctx.mark_non_differentiable(info)
        return b[:, 0, :], var

    @staticmethod
    def backward(ctx, gb, gvar):
        b, var, info = ctx.saved_tensors
        g = ctx.g
        if gb is None:
            gb = torch.zeros_like(b[:, 0, :])
        g.backward_begin()
        g.backward_block(ctx.XR, b[:, 0, :].contiguous(), var, info, gb.contiguous(),
                         None if gvar is None else gvar.contiguous())
        gy = torch.empty(g.n, dtype=torch.float64, device=b.device)
        gy, tr, ip = g.backward_end(gy)
        dh2 = (ip - ctx.sigma2 * tr) / ctx.h2
        dsigma2 = ip / ctx.sigma2
        g.close()
        ctx.g = None
        f64 = dict(dtype=torch.float64, device=b.device)
        return (gy, torch.tensor(dh2, **f64), None, None, None,
                torch.tensor(dsigma2, **f64) if ctx.sigma2_is_tensor else None, None)
