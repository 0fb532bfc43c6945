"""torch.autograd.Function around the engine's residual and its VJP.

``stokes_residual(engine, u, p, logA, beta, n=3, eps=1e-10, B0=0.5, body=(0,0,0))``
returns the residual (r_u [3, n_nodes], r_p [n_el, n_p]) of eq. (weak) at (u, p)
computed by the HIP engine in FP64.  Its backward is the engine's hand-written
adjoint kernel: for a cotangent w = (w_u, w_p) it returns J_c^T w for u and p
(J_c is the Newton Jacobian, symmetric, eq. (newton) with the tensor of
eq. (rank4)), and d<w, r>/dlogA and d<w, r>/dbeta for the per-element log rate
factor and the per-face basal friction.
"""
from __future__ import annotations

import torch


class StokesResidualFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u, p, logA, beta, engine, params):
        engine.set_params(params["n"], params["eps"], params["B0"], params["body"], logA.detach().contiguous(),
                          beta.detach().contiguous())
        engine.set_state(u.detach().contiguous(), p.detach().contiguous())
        ctx.engine, ctx.params = engine, params
        ctx.version = engine.state_version
        ctx.save_for_backward(u, p, logA, beta)
        r_u, r_p = engine.residual()
        return r_u, r_p

    @staticmethod
    def backward(ctx, g_ru, g_rp):
        eng, prm = ctx.engine, ctx.params
        u, p, logA, beta = ctx.saved_tensors
        if eng.state_version != ctx.version:
            # another forward re-linearised the engine meanwhile: restore this one's point
            eng.set_params(prm["n"], prm["eps"], prm["B0"], prm["body"], logA.detach().contiguous(),
                           beta.detach().contiguous())
            eng.set_state(u.detach().contiguous(), p.detach().contiguous())
        if g_ru is None:
            g_ru = torch.zeros_like(u)
        if g_rp is None:
            g_rp = torch.zeros_like(p)
        g_u, g_p, g_A, g_b = eng.residual_vjp(g_ru.contiguous(), g_rp.contiguous(), "fp64")
        return g_u, g_p, g_A, g_b, None, None


def stokes_residual(engine, u, p, logA, beta, n=3.0, eps=1e-10, B0=0.5, body=(0.0, 0.0, 0.0)):
    params = dict(n=n, eps=eps, B0=B0, body=tuple(body))
    return StokesResidualFn.apply(u, p, logA, beta, engine, params)
