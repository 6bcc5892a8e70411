"""GPU observables (sw_rdf, sw_adf, sw_msd) against the FP64 oracle: the
histograms are integer counts and must be identical; the mean square
displacement agrees to FP64 rounding.  The last tests check the 298 K liquid
against the paper's loose physics (coordination, diffusion; Sec. III, Table 1)."""
import math

import numpy as np
import pytest

import oracle
from paper_0809_2811_amd import observables, synth
from tests.gpu_util import RC, f32, from_dev, liquid, to_dev

pytestmark = pytest.mark.gpu

THETA = np.concatenate([[0.0], np.arange(0.5, 180.0, 1.0), [180.0]])


def ctx_for(offsets, boxes, skin=0.5):
    from paper_0809_2811_amd import sw
    return sw.Context(offsets, boxes, cutoff=RC, skin=skin, nbr_capacity=64)


def r_edges(ctx, step=0.02, start=0.011):
    rmax = ctx.max_search_radius()
    e = np.arange(start, rmax, step)
    return e


def test_rdf_exact_ice_lattice_and_liquids():
    cases = [synth.diamond_lattice(4, 4, 4, 6.36)]
    x, _, L = liquid(1, sigma=0.0)
    cases.append((x, L))
    x, _, L = liquid(2)
    cases.append((x, L))
    for x, L in cases:
        x = f32(x)
        ctx = ctx_for([0, len(x)], [L])
        e = r_edges(ctx)
        g = ctx.rdf(to_dev(x), e).cpu().numpy()[0].astype(np.uint64)
        o = oracle.rdf_counts(x, L, e ** 2)
        assert np.array_equal(g, o), (len(x), np.nonzero(g != o))


def test_rdf_exact_replicas():
    tab = synth.replica_table(n_replicas=4)
    off, boxes = tab["offsets"], tab["boxes"]
    x = f32(tab["x"])
    ctx = ctx_for(off, boxes)
    e = r_edges(ctx, step=0.05)
    g = ctx.rdf(to_dev(x), e).cpu().numpy().astype(np.uint64)
    for r in range(len(boxes)):
        o = oracle.rdf_counts(x[off[r]:off[r + 1]], boxes[r], e ** 2)
        assert np.array_equal(g[r], o), r


def test_adf_exact_with_ties_on_the_lattice():
    """Ice Ic: the 8 closest are the 4 first neighbours and 4 of 12 equidistant
    second neighbours, chosen by caller index on both sides."""
    x, L = synth.diamond_lattice(4, 4, 4, 6.36)
    x = f32(x)
    ctx = ctx_for([0, len(x)], [L])
    for n_near in (4, 8):
        g, short = ctx.adf(to_dev(x), THETA, n_near=n_near)
        o, oshort = oracle.adf_counts(x, L, n_near, ctx.max_search_radius(), np.cos(np.radians(THETA)))
        assert short == oshort == 0
        assert np.array_equal(g.cpu().numpy()[0].astype(np.uint64), o), n_near
    k = int(np.searchsorted(THETA, math.degrees(math.acos(-1 / 3)), side="right")) - 1
    g4, _ = ctx.adf(to_dev(x), THETA, n_near=4)
    assert int(g4[0, k]) == 6 * len(x)


@pytest.mark.parametrize("reps", [1, 2])
def test_adf_exact_liquid(reps):
    x, _, L = liquid(reps, sigma=0.0 if reps == 1 else 0.02)
    x = f32(x)
    ctx = ctx_for([0, len(x)], [L])
    rs = ctx.max_search_radius()
    g, short = ctx.adf(to_dev(x), THETA, n_near=8)
    o, oshort = oracle.adf_counts(x, L, 8, rs, np.cos(np.radians(THETA)))
    assert short == oshort
    assert np.array_equal(g.cpu().numpy()[0].astype(np.uint64), o)
    # a search radius too small for 8 neighbours skips centres, identically
    g, short = ctx.adf(to_dev(x), THETA, n_near=8, r_search=3.4)
    o, oshort = oracle.adf_counts(x, L, 8, 3.4, np.cos(np.radians(THETA)))
    assert short == oshort > 0
    assert np.array_equal(g.cpu().numpy()[0].astype(np.uint64), o)


def test_observables_reject_radius_beyond_the_cells():
    from paper_0809_2811_amd import sw
    x, _, L = liquid(1, sigma=0.0)
    ctx = ctx_for([0, len(x)], [L])
    rmax = ctx.max_search_radius()
    with pytest.raises(sw.SWError):
        ctx.rdf(to_dev(f32(x)), [0.0, rmax + 0.01])
    with pytest.raises(sw.SWError):
        ctx.adf(to_dev(f32(x)), THETA, n_near=8, r_search=rmax + 0.01)


def test_msd_matches_oracle_over_a_trajectory():
    x, v, L = liquid(1, sigma=0.0)
    x, v = f32(x), f32(v)
    ctx = ctx_for([0, len(x)], [L])
    xd, vd = to_dev(x), to_dev(v)
    ref = oracle.Displacement(x, L)
    ctx.msd(xd, reset=True)
    for _ in range(30):
        ctx.step(xd, vd, 20)
        xs = from_dev(xd)
        want = ref.update(xs)
        got = float(ctx.msd(xd)[0])
        assert abs(got - want) <= 1e-12 * max(want, 1.0), (got, want)
    assert want > 1.0


def test_msd_uniform_drift_closed_form():
    from paper_0809_2811_amd import sw
    x, L = synth.diamond_lattice(4, 4, 4, 6.36)
    ctx = ctx_for([0, len(x)], [L])
    step = np.array([0.3, -0.7, 1.1])
    with pytest.raises(sw.SWError):
        ctx_for([0, len(x)], [L]).msd(to_dev(f32(x)))     # no reference yet
    ctx.msd(to_dev(f32(x)), reset=True)
    for t in range(1, 41):
        m = float(ctx.msd(to_dev(f32(synth.wrap(x + t * step, L))))[0])
    assert abs(m - 40 ** 2 * float(step @ step)) < 1e-3


def test_liquid_298K_structure_and_diffusion():
    """298 K liquid at 1.00 g/cm^3 (4096 atoms): first-shell coordination and
    the self-diffusion coefficient against the paper's values (Sec. III:
    4.25 neighbours within 3.3 A, 5.1 within 3.5 A; Table 1: D = 6.5e-5 cm^2/s),
    with loose bounds (ensemble and density differ slightly from the paper's
    NPT runs)."""
    from paper_0809_2811_amd import sw
    x, v, L = liquid(2)
    x, v = f32(x), f32(v)
    ctx = ctx_for([0, len(x)], [L], skin=1.0)
    xd, vd = to_dev(x), to_dev(v)
    ctx.step(xd, vd, 3000, thermostat=sw.SW_RESCALE, T0=298.0)
    edges = np.round(np.arange(0.0, 4.61, 0.1), 10)
    tot = np.zeros(len(edges) - 1)
    ctx.msd(xd, reset=True)
    t, m = [], []
    for k in range(1, 41):
        ctx.step(xd, vd, 250)
        tot += ctx.rdf(xd, edges).cpu().numpy()[0]
        t.append(k * 250 * 10.0)
        m.append(float(ctx.msd(xd)[0]))
    n = len(x)
    n33 = observables.coordination(tot, edges, n, 3.3, frames=40)
    n35 = observables.coordination(tot, edges, n, 3.5, frames=40)
    D = observables.diffusion_coefficient(t, m, t_min_fs=20000.0)
    assert 3.9 < n33 < 4.6, n33
    assert 4.7 < n35 < 5.5, n35
    assert 4.5e-5 < D < 9.0e-5, D
    r, g = observables.g_of_r(tot, edges, n, float(np.prod(L)), frames=40)
    assert 2.6 < r[int(np.argmax(g))] < 3.0
