"""Pins of the oracle's discrete adjoint of velocity Verlet.

The loss is the frame average of (aU U + a3 U3) / N over an NVE trajectory.
Checks: the zero-step case reduces to the closed parameter derivatives of the
reduced form (dU/deps = U/eps, dU/dlambda = U3/lambda, dU/dsigma = W/sigma),
and every gradient matches central finite differences of the forward loss
(relative step 1e-4 in the parameters, 1e-4 sigma along directions in x0, v0).
"""
import numpy as np
import pytest

import oracle
from paper_0809_2811_amd import synth


def small_liquid_like(cells=3, seed=5, temperature=298.0):
    d = synth.lattice_at_density(cells, 1.0, sigma=0.3, temperature=temperature, seed=seed)
    return d["x"], d["v"], d["box"]


def test_zero_steps_reduces_to_closed_forms():
    x, v, L = small_liquid_like()
    n = len(x)
    aU, a3 = 1.0, 1.0
    res = oracle.adjoint(x, v, L, 0, aU=aU, a3=a3)
    o = oracle.forces(x, L)
    U, U3 = o["E2"] + o["E3"], o["E3"]
    W, W3 = np.trace(o["W2"] + o["W3"]), np.trace(o["W3"])
    lam, eps, sig = oracle.MW["lam"], oracle.MW["eps"], oracle.MW["sig"]
    assert abs(res["loss"] - (aU * U + a3 * U3) / n) < 1e-12 * abs(res["loss"])
    expect = np.array([(aU + a3) * U3 / lam, (aU * U + a3 * U3) / eps, (aU * W + a3 * W3) / sig]) / n
    assert np.allclose(res["thbar"], expect, rtol=1e-9, atol=0)
    assert np.allclose(res["xbar0"], -(aU * o["F"] + a3 * o["F3"]) / n, rtol=1e-12, atol=1e-15)
    assert np.all(res["vbar0"] == 0.0)


@pytest.mark.parametrize("nsteps", [1, 12])
def test_parameter_gradient_matches_central_differences(nsteps):
    x, v, L = small_liquid_like(seed=8)
    res = oracle.adjoint(x, v, L, nsteps)
    P0 = oracle.params()
    for k in range(3):
        h = 1e-4 * P0[k]
        Pp = P0.copy(); Pp[k] += h
        Pm = P0.copy(); Pm[k] -= h
        fd = (oracle.traj_loss(x, v, L, nsteps, P=Pp)[0] - oracle.traj_loss(x, v, L, nsteps, P=Pm)[0]) / (2 * h)
        assert abs(fd - res["thbar"][k]) <= 1e-4 * abs(fd) + 1e-9, (k, fd, res["thbar"][k])


@pytest.mark.parametrize("nsteps", [1, 12])
def test_state_gradient_matches_central_differences(nsteps):
    x, v, L = small_liquid_like(seed=9)
    res = oracle.adjoint(x, v, L, nsteps, aU=1.0, a3=0.5)
    rng = np.random.default_rng(nsteps)
    sig = oracle.MW["sig"]
    for _ in range(3):
        u = rng.normal(size=x.shape); u /= np.linalg.norm(u)
        h = 1e-4 * sig
        fd = (oracle.traj_loss(x + h * u, v, L, nsteps, aU=1.0, a3=0.5)[0]
              - oracle.traj_loss(x - h * u, v, L, nsteps, aU=1.0, a3=0.5)[0]) / (2 * h)
        ad = float((res["xbar0"] * u).sum())
        assert abs(fd - ad) <= 1e-4 * abs(fd) + 1e-10
        hv = 1e-4 * float(np.abs(v).max())
        fd = (oracle.traj_loss(x, v + hv * u, L, nsteps, aU=1.0, a3=0.5)[0]
              - oracle.traj_loss(x, v - hv * u, L, nsteps, aU=1.0, a3=0.5)[0]) / (2 * hv)
        ad = float((res["vbar0"] * u).sum())
        assert abs(fd - ad) <= 1e-4 * abs(fd) + 1e-10


def test_terminal_seeds():
    """Seeds on (x_S, v_S) give d(g.x_S + k.v_S)/d(x0) by the same recursion."""
    x, v, L = small_liquid_like(seed=12)
    nsteps = 6
    rng = np.random.default_rng(1)
    g = rng.normal(size=x.shape)
    kk = rng.normal(size=x.shape)
    res = oracle.adjoint(x, v, L, nsteps, aU=0.0, a3=0.0, xbar_S=g, vbar_S=kk)

    def obj(x0, v0):
        _, xs, vs = oracle.traj_loss(x0, v0, L, nsteps, aU=0.0, a3=0.0)
        dx = xs - x0  # unwrapped displacement is what the seed differentiates; wrap-safe
        dx -= L * np.round(dx / L)
        return float((g * (x0 + dx)).sum() + (kk * vs).sum())

    u = rng.normal(size=x.shape); u /= np.linalg.norm(u)
    h = 1e-4
    fd = (obj(x + h * u, v) - obj(x - h * u, v)) / (2 * h)
    assert abs(fd - float((res["xbar0"] * u).sum())) <= 1e-5 * abs(fd)
    fd = (obj(x, v + h * 1e-2 * u) - obj(x, v - h * 1e-2 * u)) / (2 * h * 1e-2)
    assert abs(fd - float((res["vbar0"] * u).sum())) <= 1e-5 * abs(fd)


# --------------------------------------------------------------- virial term
def virial(x, L, P=None):
    o = oracle.forces(x, L, P)
    return float(np.trace(o["W2"] + o["W3"]))


def test_virial_term_zero_steps_against_differences_of_the_virial():
    """aW W / N alone at S = 0: the loss is the virial trace per atom, and its
    gradients in x0 and in (lambda, epsilon, sigma) equal central differences
    of the virial trace itself (forces() in FP64), not of the loss routine."""
    x, v, L = small_liquid_like(seed=14)
    n = len(x)
    res = oracle.adjoint(x, v, L, 0, aU=0.0, a3=0.0, aW=1.0)
    assert abs(res["loss"] - virial(x, L) / n) <= 1e-12 * abs(res["loss"])
    P0 = oracle.params()
    for k in range(3):
        h = 1e-5 * P0[k]
        Pp = P0.copy(); Pp[k] += h
        Pm = P0.copy(); Pm[k] -= h
        fd = (virial(x, L, Pp) - virial(x, L, Pm)) / (2 * h) / n
        assert abs(fd - res["thbar"][k]) <= 1e-6 * abs(fd), (k, fd, res["thbar"][k])
    rng = np.random.default_rng(3)
    for a in rng.choice(n, 5, replace=False):
        for c in range(3):
            h = 1e-5
            xp = x.copy(); xp[a, c] += h
            xm = x.copy(); xm[a, c] -= h
            fd = (virial(xp, L) - virial(xm, L)) / (2 * h) / n
            assert abs(fd - res["xbar0"][a, c]) <= 1e-6 * np.abs(res["xbar0"]).max(), (a, c)
    assert np.all(res["vbar0"] == 0.0)


@pytest.mark.parametrize("nsteps", [1, 10])
def test_virial_term_gradients_match_central_differences(nsteps):
    """The full loss with the virial term (aU U + aW W): parameter and
    initial-state gradients against central differences of the forward loss."""
    x, v, L = small_liquid_like(seed=15)
    kw = dict(aU=0.5, a3=0.0, aW=1.0)
    res = oracle.adjoint(x, v, L, nsteps, **kw)
    P0 = oracle.params()
    for k in range(3):
        h = 1e-4 * P0[k]
        Pp = P0.copy(); Pp[k] += h
        Pm = P0.copy(); Pm[k] -= h
        fd = (oracle.traj_loss(x, v, L, nsteps, P=Pp, **kw)[0] - oracle.traj_loss(x, v, L, nsteps, P=Pm, **kw)[0]) / (2 * h)
        assert abs(fd - res["thbar"][k]) <= 1e-4 * abs(fd) + 1e-9, (k, fd, res["thbar"][k])
    rng = np.random.default_rng(nsteps + 40)
    h = 1e-4 * oracle.MW["sig"]
    for _ in range(3):
        u = rng.normal(size=x.shape); u /= np.linalg.norm(u)
        fd = (oracle.traj_loss(x + h * u, v, L, nsteps, **kw)[0] - oracle.traj_loss(x - h * u, v, L, nsteps, **kw)[0]) / (2 * h)
        assert abs(fd - float((res["xbar0"] * u).sum())) <= 1e-4 * abs(fd) + 1e-10
        hv = h / 10.0
        fd = (oracle.traj_loss(x, v + hv * u, L, nsteps, **kw)[0] - oracle.traj_loss(x, v - hv * u, L, nsteps, **kw)[0]) / (2 * hv)
        assert abs(fd - float((res["vbar0"] * u).sum())) <= 1e-4 * abs(fd) + 1e-10
