"""Host logic of the Gauss-Newton parameter fit (no GPU): the trajectory
observables are replaced by a known smooth function of theta, so the solver's
steps, its use of a per-iterate target and its refusal of non-finite values
are checked on their own."""
import numpy as np
import pytest

from paper_0809_2811_amd import fit


def _model(theta):
    """Two observables of (lambda, epsilon, sigma): mildly nonlinear, with
    the Jacobian rows the solver needs."""
    lam, eps, sig = theta["lambda_"], theta["epsilon"], theta["sigma"]
    o = np.array([-eps * (1.0 + 0.01 * (sig - 2.4) ** 2), 50.0 * (sig - 2.39) + 0.1 * eps])
    g = np.array([[0.0, -(1.0 + 0.01 * (sig - 2.4) ** 2), -0.02 * eps * (sig - 2.4)],
                  [0.0, 0.1, 50.0]])
    return o, g


def test_gauss_newton_converges_on_a_known_function(monkeypatch):
    monkeypatch.setattr(fit, "observables", lambda ctx, x0, v0, theta, nsteps, **kw: _model(theta))
    truth = dict(lambda_=23.15, epsilon=6.189, sigma=2.3925)
    target, _ = _model(truth)
    path = fit.gauss_newton(None, None, None, target, dict(lambda_=23.15, epsilon=6.0, sigma=2.35),
                            fit=("epsilon", "sigma"), iters=10, tol=1e-12)
    th, res = path[-1]
    assert abs(th["epsilon"] - 6.189) < 1e-9 and abs(th["sigma"] - 2.3925) < 1e-9
    assert np.abs(res).max() < 1e-10
    assert th["lambda_"] == 23.15                      # parameters outside `fit` stay fixed


def test_target_function_is_evaluated_at_every_iterate(monkeypatch):
    monkeypatch.setattr(fit, "observables", lambda ctx, x0, v0, theta, nsteps, **kw: _model(theta))
    seen = []

    def target_fn(theta):
        seen.append(dict(theta))
        return _model(dict(lambda_=23.15, epsilon=6.189, sigma=2.3925))[0]

    path = fit.gauss_newton(None, None, None, None, dict(lambda_=23.15, epsilon=6.0, sigma=2.35),
                            fit=("epsilon", "sigma"), iters=4, target_fn=target_fn)
    assert len(seen) == len(path)
    assert [p[0] for p in path] == seen


def test_non_finite_observables_raise_with_the_iterate(monkeypatch):
    def bad(ctx, x0, v0, theta, nsteps, **kw):
        o, g = _model(theta)
        if theta["sigma"] > 2.38:
            o[1] = np.nan
        return o, g

    monkeypatch.setattr(fit, "observables", bad)
    target, _ = _model(dict(lambda_=23.15, epsilon=6.189, sigma=2.3925))
    with pytest.raises(FloatingPointError, match="iterate 1"):
        fit.gauss_newton(None, None, None, target, dict(lambda_=23.15, epsilon=6.0, sigma=2.35),
                         fit=("epsilon", "sigma"), iters=5)
