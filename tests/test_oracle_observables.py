"""Pins of the observables oracle (Sec. II.C: g(r), n_c, P(theta), D) against
closed forms of the cubic-diamond lattice (the oxygen sites of ice Ic), an
independent brute-force pair count, and the closed forms of the coordinate
convention and of a uniform drift across periodic boundaries."""
import math

import numpy as np

import oracle
from paper_0809_2811_amd import synth

A = 6.36   # ice Ic lattice constant used by the ice workload (A)

# Shells of the diamond lattice around any site: (distance / a, count).
DIAMOND_SHELLS = [(math.sqrt(3) / 4, 4), (math.sqrt(2) / 2, 12), (math.sqrt(11) / 4, 12), (1.0, 6)]


def lattice():
    return synth.diamond_lattice(4, 4, 4, A)


def test_quantize_convention():
    L = np.array([25.0, 30.0, 40.0])
    x = np.array([[0.0, 15.0, -10.0], [25.0, 7.5, 50.0]])
    u = oracle.quantize(x, L)
    assert u[0].tolist() == [0, 2 ** 31, 3 * 2 ** 30]
    assert u[1].tolist() == [0, 2 ** 30, 2 ** 30]


def test_rdf_diamond_shells():
    x, L = lattice()
    n = len(x)
    # bins 0.02 A wide, offset so that no shell sits on an edge
    r = np.arange(0.011, 6.5, 0.02)
    counts = oracle.rdf_counts(x, L, r ** 2)
    for frac, mult in DIAMOND_SHELLS:
        k = int(np.searchsorted(r, frac * A, side="right")) - 1
        assert counts[k] == n * mult, (frac * A, counts[k], n * mult)
    assert counts.sum() == n * sum(m for _, m in DIAMOND_SHELLS)
    # n_c as the integral of g(r): the running count over the first shell
    assert counts[: int(np.searchsorted(r, 3.3))].sum() / n == 4


def test_rdf_total_matches_brute_force():
    rng = np.random.default_rng(11)
    L = np.array([14.0, 15.0, 16.0])
    x = rng.uniform(0, 1, size=(300, 3)) * L
    rmax = 4.0
    d = x[None, :, :] - x[:, None, :]
    d -= L * np.rint(d / L)
    r = np.sqrt((d ** 2).sum(-1))
    np.fill_diagonal(r, np.inf)
    assert np.min(np.abs(r - rmax)) > 1e-6          # no pair on the edge
    counts = oracle.rdf_counts(x, L, np.array([0.0, 2.0, 3.0, rmax]) ** 2)
    assert counts.sum() == int((r < rmax).sum())
    assert counts[0] == int((r < 2.0).sum())


def theta_edges():
    th = np.concatenate([[0.0], np.arange(0.5, 180.0, 1.0), [180.0]])
    return th, np.cos(np.radians(th))


def bin_of(th_edges, angle):
    return int(np.searchsorted(th_edges, angle, side="right")) - 1


def test_adf_first_shell_is_tetrahedral():
    x, L = lattice()
    th, c = theta_edges()
    counts, short = oracle.adf_counts(x, L, 4, 3.3, c)
    assert short == 0
    k = bin_of(th, math.degrees(math.acos(-1.0 / 3.0)))
    assert counts[k] == 6 * len(x) and counts.sum() == 6 * len(x)


def test_adf_two_shells_closed_form():
    """16 closest = 4 first + 12 second neighbours: the 12 second neighbours
    form a cuboctahedron (60: 24, 90: 12, 120: 24, 180: 6 pairs), first with
    second neighbours give 35.26 (12), 90 (24), 144.74 (12), first with first
    the tetrahedral angle (6)."""
    x, L = lattice()
    n = len(x)
    th, c = theta_edges()
    counts, short = oracle.adf_counts(x, L, 16, 5.0, c)
    assert short == 0
    want = {60.0: 24, 90.0: 36, 120.0: 24, 180.0: 6, math.degrees(math.acos(-1 / 3)): 6,
            math.degrees(math.acos(math.sqrt(2 / 3))): 12, math.degrees(math.acos(-math.sqrt(2 / 3))): 12}
    for ang, m in want.items():
        assert counts[bin_of(th, ang) if ang < 180 else len(counts) - 1] == n * m, ang
    assert counts.sum() == n * 120


def test_adf_skips_centres_without_enough_neighbours():
    x, L = lattice()
    th, c = theta_edges()
    counts, short = oracle.adf_counts(x, L, 8, 3.3, c)   # only 4 inside 3.3 A
    assert short == len(x) and counts.sum() == 0


def test_displacement_uniform_drift_across_boundaries():
    x, L = lattice()
    step = np.array([0.3, -0.7, 1.1])
    tr = oracle.Displacement(x, L)
    for t in range(1, 101):
        msd = tr.update(synth.wrap(x + t * step, L))
    assert abs(msd - 100 ** 2 * float(step @ step)) < 1e-8


def test_displacement_random_walk():
    rng = np.random.default_rng(5)
    L = np.array([10.0, 11.0, 12.0])
    x0 = rng.uniform(0, 1, size=(50, 3)) * L
    steps = rng.normal(scale=0.8, size=(40, 50, 3))
    tr = oracle.Displacement(x0, L)
    pos = x0.copy()
    for s in steps:
        pos = pos + s
        tr.update(synth.wrap(pos, L))
    total = steps.sum(axis=0)
    assert np.allclose(tr.acc, total, atol=1e-9)
