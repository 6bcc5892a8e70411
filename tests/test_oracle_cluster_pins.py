"""Absolute pins of the oracle's three-body term (Sec. II.A, Eq. phi3).

The ratio pins in test_oracle_pins.py cancel the radial factors; these do
not.  Each cluster is small enough to have a closed form:

* equilateral and linear three-atom clusters at r = 3.0 A against the values
  stored in tests/golden/sw_cluster_values.txt (evaluated in FP64 apart from
  the oracle, from the printed constants);
* clusters with one vertex (the third side beyond a*sigma) and two unequal
  legs: log E3 is a straight line in 1/(r1 - a*sigma) with slope gamma*sigma
  (pins gamma and the shift a*sigma of the leg factor), E3 is symmetric in
  the two legs, scales with the angle as (cos theta + 1/3)^2 (anchored to the
  stored linear-chain value), and the two-body energy is the sum over the two
  legs only.
"""
import math
import pathlib

import numpy as np
import pytest

import oracle

GOLDEN = pathlib.Path(__file__).resolve().parent / "golden" / "sw_cluster_values.txt"
LAM, EPS, SIG = 23.15, 6.189, 2.3925
GAM, A_RED = 1.2, 1.8
RC = A_RED * SIG
L = np.array([30.0, 30.0, 30.0])
O = np.array([7.0, 9.0, 11.0])


def golden():
    out = {}
    for line in GOLDEN.read_text().splitlines():
        if line.strip() and not line.startswith("#"):
            key, r, val = line.split()[:3]
            out[key] = (float(r), float(val))
    return out


def equilateral(r):
    return np.array([O, O + [r, 0, 0], O + [r / 2, r * math.sqrt(3) / 2, 0]])


def linear(r):
    return np.array([O, O + [r, 0, 0], O + [2 * r, 0, 0]])


def vee(r1, r2, theta_deg):
    """Vertex atom at O, legs of length r1 (along x) and r2 at angle theta."""
    t = math.radians(theta_deg)
    return np.array([O, O + [r1, 0, 0], O + [r2 * math.cos(t), r2 * math.sin(t), 0]])


def third_side(r1, r2, theta_deg):
    return math.sqrt(r1 * r1 + r2 * r2 - 2 * r1 * r2 * math.cos(math.radians(theta_deg)))


@pytest.mark.parametrize("kind", ["equilateral", "linear"])
def test_cluster_energies_against_closed_forms(kind):
    g = golden()
    r, e2 = g[f"{kind}_E2"]
    _, e3 = g[f"{kind}_E3"]
    x = equilateral(r) if kind == "equilateral" else linear(r)
    for E2, E3 in (oracle.energy_brute(x, L), (lambda o: (o["E2"], o["E3"]))(oracle.forces(x, L))):
        assert abs(E2 - e2) <= 1e-11 * abs(e2), (E2, e2)
        assert abs(E3 - e3) <= 1e-11 * abs(e3), (E3, e3)


def test_leg_factor_is_exp_gamma_sigma_over_r_minus_a_sigma():
    """One vertex, legs (r1, 3.0 A) at 150 deg: log E3 against 1/(r1 - a sigma)
    is a straight line of slope gamma*sigma."""
    r1s = np.array([2.5, 2.8, 3.1, 3.4, 3.7, 4.0, 4.2])
    assert all(third_side(r, 3.0, 150.0) > RC + 0.5 for r in r1s)
    e3 = np.array([oracle.energy_brute(vee(r, 3.0, 150.0), L)[1] for r in r1s])
    assert np.all(e3 > 0)
    xs = 1.0 / (r1s - RC)
    slope, icpt = np.polyfit(xs, np.log(e3), 1)
    assert abs(slope - GAM * SIG) < 1e-9 * GAM * SIG, slope
    assert np.abs(np.log(e3) - (slope * xs + icpt)).max() < 1e-11


def test_unequal_legs_symmetric_and_angular_factor():
    """E3(r1, r2) = E3(r2, r1); at fixed legs E3 follows (cos theta + 1/3)^2,
    anchored to the stored linear-chain value (legs 3.0 A, cos = -1)."""
    g = golden()
    r, e_lin = g["linear_E3"]
    a = oracle.energy_brute(vee(2.7, 3.6, 140.0), L)[1]
    b = oracle.energy_brute(vee(3.6, 2.7, 140.0), L)[1]
    assert abs(a - b) <= 1e-13 * abs(a)
    for th in (100.0, 120.0, 135.0, 150.0, 165.0, 180.0):
        assert third_side(r, r, th) > RC
        e3 = oracle.energy_brute(vee(r, r, th), L)[1]
        want = e_lin * (math.cos(math.radians(th)) + 1.0 / 3.0) ** 2 / (4.0 / 9.0)
        assert abs(e3 - want) <= 1e-11 * e_lin, (th, e3, want)


def test_unequal_leg_cluster_absolute():
    """Legs 2.7 and 3.6 A at 140 deg (third side 5.9 A): both radial factors
    kept.  The expected value scales the stored linear-chain energy by the
    angular factor and by the two leg factors relative to the 3.0 A legs."""
    g = golden()
    r, e_lin = g["linear_E3"]
    r1, r2, th = 2.7, 3.6, 140.0
    want = (e_lin * (math.cos(math.radians(th)) + 1.0 / 3.0) ** 2 / (4.0 / 9.0)
            * math.exp(GAM * SIG * (1.0 / (r1 - RC) + 1.0 / (r2 - RC) - 2.0 / (r - RC))))
    x = vee(r1, r2, th)
    e2, e3 = oracle.energy_brute(x, L)
    assert abs(e3 - want) <= 1e-11 * want, (e3, want)
    o = oracle.forces(x, L)
    assert abs(o["E3"] - want) <= 1e-11 * want
    # two-body energy: only the two legs interact (third side beyond a sigma)
    assert abs(e2 - (oracle.phi2(r1) + oracle.phi2(r2))) <= 1e-13 * abs(e2)
    assert oracle.phi2(third_side(r1, r2, th)) == 0.0
    # the cluster's net force is zero and the vertex atom balances the legs
    assert np.abs(o["F"].sum(0)).max() < 1e-12 * np.abs(o["F"]).max()
