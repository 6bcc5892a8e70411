"""Fitting the potential's parameters through the differentiable form.

Sec. II.D of the paper fixes epsilon (from the melting point), lambda (from
the enthalpy of vaporisation) and sigma (from the 298 K density) by scanning
them against target properties.  Here the same kind of fit is a gradient
problem: trajectory observables of the batched engine, each an average over
R replicas of short NVE trajectories from fixed starts,

    O_U(theta)  = mean_r 1/(S+1) sum_s U_r(x_s) / N_r       (potential energy per atom)
    O_3(theta)  = mean_r 1/(S+1) sum_s U3_r(x_s) / N_r      (three-body energy per atom)
    O_W(theta)  = mean_r 1/(S+1) sum_s W_r(x_s) / N_r       (virial trace per atom)

are differentiated exactly by the discrete adjoint (sw_adjoint, one call per
observable gives dO/d(lambda, epsilon, sigma)), and Gauss-Newton steps move
the fitted parameters until the observables meet their targets.  The
trajectories are short (tens of steps) so that the observables are smooth
functions of theta (the liquid is chaotic over longer horizons).

Table 1 targets (`table1_fit`): the potential energy per atom of the 298 K
liquid, U/N = RT - dH_vap (the vapour is ideal and monatomic, H_gas = 2.5 RT,
Sec. II.C; the liquid's kinetic energy is 1.5 RT and p V ~ 0), and zero
pressure at the 298 K density 0.997 g/cm^3 (p = 0 in every isobaric run,
Sec. II.B), i.e. P V = (2 KE + W)/3 = 0, W/N = -2 KE/N with KE measured on
the same trajectories.
"""
from __future__ import annotations

import numpy as np

NAMES = ("lambda_", "epsilon", "sigma")
KCAL_R = 8.314462618 / 4184.0          # gas constant, kcal/(mol K)
DH_VAP_298 = 10.65                     # Table 1, kcal/mol
RHO_298 = 0.997                        # Table 1, g/cm^3


def observables(ctx, x0, v0, theta: dict, nsteps: int = 20, ckpt_every: int = 20,
                weights=((1.0, 0.0, 0.0), (0.0, 1.0, 0.0))):
    """Observables with loss weights (aU, a3, aW) each, averaged over the
    context's replicas, and their gradients [len(weights)][3] in (lambda,
    epsilon, sigma)."""
    from paper_0809_2811_amd import sw
    p = sw.params_mw(**theta)
    out, grad = [], []
    for aU, a3, aW in weights:
        r = ctx.adjoint(x0, v0, nsteps, ckpt_every=ckpt_every, aU=aU, a3=a3, aW=aW, params=p)
        out.append(float(r["loss"].mean()))
        grad.append(r["thbar"].mean(dim=0).cpu().numpy())
    return np.array(out), np.array(grad)


def gauss_newton(ctx, x0, v0, target, theta0: dict, fit=("lambda_", "epsilon"), iters: int = 8,
                 nsteps: int = 20, tol: float = 1e-10, log=None, weights=((1.0, 0.0, 0.0), (0.0, 1.0, 0.0)),
                 target_fn=None):
    """Solve O(theta) = target for the parameters in `fit` (the others fixed
    at theta0); returns the path of (theta, residual).  target_fn(theta), if
    given, recomputes the target at each iterate (a target measured on the
    same trajectories, held fixed within a step)."""
    theta = dict(theta0)
    idx = [NAMES.index(k) for k in fit]
    path = []
    for it in range(iters):
        tgt = np.asarray(target_fn(theta) if target_fn else target, dtype=np.float64)
        o, g = observables(ctx, x0, v0, theta, nsteps, weights=weights)
        res = o - tgt
        path.append((dict(theta), res.copy()))
        if log:
            log(it, theta, res)
        J = g[:, idx]
        if not (np.all(np.isfinite(res)) and np.all(np.isfinite(J))):
            raise FloatingPointError(f"non-finite observables or gradients at iterate {it}, theta={theta}: "
                                     f"residual {res}, Jacobian {J.tolist()}")
        if np.max(np.abs(res)) < tol:
            break
        step = np.linalg.lstsq(J, -res, rcond=None)[0]
        for k, d in zip(fit, step):
            theta[k] = theta[k] + float(d)
    return path


def mean_kinetic_per_atom(ctx, x0, v0, theta: dict, nsteps: int, mass: float = 18.015):
    """Mean over the frames 0..S (and the replicas) of the kinetic energy per
    atom of the same NVE trajectories the adjoint differentiates (kcal/mol)."""
    import torch
    from paper_0809_2811_amd import sw
    p = sw.params_mw(**theta)
    x, v = x0.clone(), v0.clone()
    k0 = 0.5 * mass / 4.184e-4 * (v[:, :3].double() ** 2).sum().item()
    _, th = ctx.step(x, v, nsteps, params=p, thermo_every=1)
    ke = th[:, :, 2].sum(dim=1).cpu().numpy()       # per step, summed over replicas
    n = int(ctx.n)
    return float((k0 + ke.sum()) / ((nsteps + 1) * n))


def table1_fit(ctx, x0, v0, theta0: dict, temperature: float = 298.0, nsteps: int = 20, iters: int = 8,
               fit=("epsilon", "sigma"), log=None):
    """Fit (epsilon, sigma) (lambda fixed at theta0) to the Table 1 targets:
    U/N = R T - dH_vap and zero pressure (W/N = -2 KE/N) at the starts'
    density.  Returns the Gauss-Newton path."""
    u_target = KCAL_R * temperature - DH_VAP_298

    def target(theta):
        return [u_target, -2.0 * mean_kinetic_per_atom(ctx, x0, v0, theta, nsteps)]

    return gauss_newton(ctx, x0, v0, None, theta0, fit=fit, iters=iters, nsteps=nsteps, log=log,
                        weights=((1.0, 0.0, 0.0), (0.0, 0.0, 1.0)), target_fn=target)
