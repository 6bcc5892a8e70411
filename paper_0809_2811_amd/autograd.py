"""torch.autograd.Function over an NVE trajectory of the HIP engine.

    loss, xS, vS = trajectory_loss(ctx, x0, v0, theta, nsteps=200, ckpt_every=20)

theta is a float64 tensor (lambda, epsilon, sigma); x0, v0 are the engine's
float32 [N, 4] tensors.  loss[r] = 1/(S+1) sum_s [aU U_r(x_s) + a3 U3_r(x_s)] / N_r.
The forward pass runs sw_adjoint (forward with checkpoints + discrete
adjoint) for unit loss weights; backward scales that result by the incoming
gradient, or reruns sw_adjoint with the incoming seeds on (xS, vS).
"""
from __future__ import annotations

import torch

from . import sw


def _params(theta: torch.Tensor) -> sw.sw_params:
    lam, eps, sig = (float(t) for t in theta.detach().cpu())
    return sw.params_mw(lambda_=lam, epsilon=eps, sigma=sig)


class TrajectoryLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x0, v0, theta, engine, nsteps, dt, mass, ckpt_every, aU, a3):
        p = _params(theta)
        res = engine.adjoint(x0.detach(), v0.detach(), nsteps, dt=dt, mass=mass, ckpt_every=ckpt_every,
                             aU=aU, a3=a3, params=p)
        ctx.engine, ctx.args = engine, (nsteps, dt, mass, ckpt_every, aU, a3)
        ctx.save_for_backward(x0, v0, theta, res["xbar0"], res["vbar0"], res["thbar"])
        return res["loss"], res["xS"], res["vS"]

    @staticmethod
    def backward(ctx, g_loss, g_xS, g_vS):
        x0, v0, theta, xbar0, vbar0, thbar = ctx.saved_tensors
        nsteps, dt, mass, ckpt_every, aU, a3 = ctx.args
        seeds = [g for g in (g_xS, g_vS) if g is not None and bool(torch.any(g != 0))]
        if g_loss is None:
            g_loss = torch.zeros(thbar.shape[0], dtype=torch.float64, device=thbar.device)
        if not seeds:
            if thbar.shape[0] == 1:
                gl = g_loss.reshape(1)
                gx = (xbar0 * gl.to(xbar0.dtype)) if ctx.needs_input_grad[0] else None
                gv = (vbar0 * gl.to(vbar0.dtype)) if ctx.needs_input_grad[1] else None
                gth = (thbar[0] * gl[0]).to(theta.dtype).to(theta.device) if ctx.needs_input_grad[2] else None
                return gx, gv, gth, None, None, None, None, None, None, None
        if not torch.all(g_loss == g_loss.reshape(-1)[0]):
            raise NotImplementedError("different loss weights per replica")
        gl = float(g_loss.reshape(-1)[0])
        xs = None if g_xS is None else g_xS.contiguous()
        vs = None if g_vS is None else g_vS.contiguous()
        res = ctx.engine.adjoint(x0.detach(), v0.detach(), nsteps, dt=dt, mass=mass, ckpt_every=ckpt_every,
                                 aU=aU * gl, a3=a3 * gl, params=_params(theta), xbar_S=xs, vbar_S=vs)
        gth = res["thbar"].sum(0).to(theta.dtype).to(theta.device)
        return res["xbar0"], res["vbar0"], gth, None, None, None, None, None, None, None


def trajectory_loss(engine: "sw.Context", x0, v0, theta, nsteps: int = 200, dt: float = 10.0, mass: float = 18.015,
                    ckpt_every: int = 20, aU: float = 1.0, a3: float = 1.0):
    return TrajectoryLoss.apply(x0, v0, theta, engine, nsteps, dt, mass, ckpt_every, aU, a3)
