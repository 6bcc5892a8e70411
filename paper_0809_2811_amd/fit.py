"""Fitting the potential's parameters through the differentiable form.

Sec. II.D of the paper fixes lambda and epsilon (sigma from the density) by
scanning them against target properties.  Here the same kind of fit is a
gradient problem: trajectory observables of the batched engine, each an
average over R replicas of short NVE trajectories from fixed starts,

    O_U(theta)  = mean_r 1/(S+1) sum_s U_r(x_s) / N_r
    O_3(theta)  = mean_r 1/(S+1) sum_s U3_r(x_s) / N_r

are differentiated exactly by the discrete adjoint (sw_adjoint, one call per
observable gives dO/d(lambda, epsilon, sigma)), and Gauss-Newton steps move
theta = (lambda, epsilon) until the observables meet their targets.  The
trajectories are short (tens of steps) so that the observables are smooth
functions of theta (the liquid is chaotic over longer horizons).
"""
from __future__ import annotations

import numpy as np

NAMES = ("lambda_", "epsilon", "sigma")


def observables(ctx, x0, v0, theta: dict, nsteps: int = 20, ckpt_every: int = 20):
    """(O_U, O_3) and their gradients [2][3] in (lambda, epsilon, sigma)."""
    from paper_0809_2811_amd import sw
    p = sw.params_mw(**theta)
    out, grad = [], []
    for aU, a3 in ((1.0, 0.0), (0.0, 1.0)):
        r = ctx.adjoint(x0, v0, nsteps, ckpt_every=ckpt_every, aU=aU, a3=a3, params=p)
        out.append(float(r["loss"].mean()))
        grad.append(r["thbar"].mean(dim=0).cpu().numpy())
    return np.array(out), np.array(grad)


def gauss_newton(ctx, x0, v0, target, theta0: dict, fit=("lambda_", "epsilon"), iters: int = 8,
                 nsteps: int = 20, tol: float = 1e-10, log=None):
    """Solve O(theta) = target for the parameters in `fit` (the others fixed
    at theta0); returns the path of (theta, residual)."""
    theta = dict(theta0)
    idx = [NAMES.index(k) for k in fit]
    path = []
    for it in range(iters):
        o, g = observables(ctx, x0, v0, theta, nsteps)
        res = o - np.asarray(target)
        path.append((dict(theta), res.copy()))
        if log:
            log(it, theta, res)
        if np.max(np.abs(res)) < tol:
            break
        J = g[:, idx]
        step = np.linalg.lstsq(J, -res, rcond=None)[0]
        for k, d in zip(fit, step):
            theta[k] = theta[k] + float(d)
    return path
