"""CPU pins of the Sec. II.C estimators in paper_0809_2811_amd/observables.py.

The device calls give exact counts and displacements; these functions turn
them into g(r), n_c, P(theta), D and gamma_lv.  Each estimator is checked on
input whose answer is fixed by geometry or by the definition of the quantity,
not by a retyped estimator:

* n_c on the perfect diamond lattice (4 first, 16 second, 28 third, 34 fourth
  neighbours), and g(r) integrated back to the same counts;
* g(r) of uniform random points tends to 1;
* P(theta) of the lattice puts all weight in the bin of the tetrahedral angle
  and integrates to one;
* D from synthetic Brownian walks with a known diffusion constant (variance
  2 D dt per component per step), in cm^2/s;
* gamma_lv of a synthetic slab whose tangential pressure deficit is confined
  to two interfaces of known width: gamma is the integral of p_N - p_T across
  one interface.
"""
import math

import numpy as np

from paper_0809_2811_amd import observables as ob
from paper_0809_2811_amd import synth


def pair_distances(x, L):
    d = x[None, :, :] - x[:, None, :]
    d -= L * np.rint(d / L)
    r = np.sqrt((d ** 2).sum(-1))
    np.fill_diagonal(r, np.inf)
    return r[np.isfinite(r)].ravel()


def test_coordination_counts_diamond_shells():
    a = 6.36
    x, L = synth.diamond_lattice(4, 4, 4, a)
    n = len(x)
    edges = np.arange(0.0, 7.0001, 0.01)
    counts, _ = np.histogram(pair_distances(x, L), bins=edges)
    for rc, want in ((3.3, 4), (4.6, 16), (5.5, 28), (6.5, 34)):
        assert ob.coordination(counts, edges, n, rc) == want
    # g(r) integrated with the shell volumes gives back the pair counts
    V = float(np.prod(L))
    rmid, g = ob.g_of_r(counts, edges, n, V)
    shell = 4.0 / 3.0 * np.pi * (edges[1:] ** 3 - edges[:-1] ** 3)
    k = int(np.searchsorted(edges, 4.6))
    assert abs((g[:k] * shell[:k]).sum() * n / V - 16.0) < 1e-9


def test_g_of_r_of_uniform_points_is_one():
    rng = np.random.default_rng(3)
    L = np.array([30.0, 30.0, 30.0])
    frames, n = 4, 1500
    edges = np.linspace(2.0, 8.0, 7)
    counts = np.zeros(len(edges) - 1)
    for _ in range(frames):
        x = rng.uniform(0, 1, size=(n, 3)) * L
        counts += np.histogram(pair_distances(x, L), bins=edges)[0]
    _, g = ob.g_of_r(counts, edges, n, float(np.prod(L)), frames=frames)
    # (n - 1) / n of the pairs are distinct atoms; statistical error ~1 %
    assert np.all(np.abs(g - 1.0) < 0.03), g


def test_angle_distribution_of_the_lattice():
    th = np.arange(0.0, 180.0001, 1.0)
    counts = np.zeros(len(th) - 1)
    tet = math.degrees(math.acos(-1.0 / 3.0))
    counts[int(tet)] = 6 * 512            # six angles per site among its four neighbours
    c, p = ob.angle_distribution(counts, th)
    assert abs((p * np.diff(th)).sum() - 1.0) < 1e-12
    assert c[np.argmax(p)] == int(tet) + 0.5 and abs(c[np.argmax(p)] - tet) < 1.0


def test_diffusion_coefficient_of_brownian_walks():
    """Walks with D = 6.5e-5 cm^2/s = 6.5e-4 A^2/fs: increments of variance
    2 D dt per component (the Einstein relation's 6 D t in three
    dimensions)."""
    D_cm2s = 6.5e-5
    D = D_cm2s * 10.0                    # 1 cm^2/s = 10 A^2/fs
    rng = np.random.default_rng(17)
    dt, steps, n = 100.0, 400, 4000
    x = np.zeros((n, 3))
    t, msd = [0.0], [0.0]
    for s in range(1, steps + 1):
        x += rng.normal(0.0, math.sqrt(2 * D * dt), size=x.shape)
        t.append(s * dt)
        msd.append(float((x ** 2).sum(1).mean()))
    est = ob.diffusion_coefficient(t, msd)
    assert abs(est / D_cm2s - 1.0) < 0.03, est
    # an exactly linear MSD with a ballistic offset: the slope alone matters
    tt = np.linspace(0.0, 1e5, 50)
    assert abs(ob.diffusion_coefficient(tt, 6 * D * tt + 0.7, t_min_fs=1e3) / D_cm2s - 1.0) < 1e-12


def test_surface_tension_of_a_synthetic_slab():
    """Two flat interfaces normal to z, each with a tangential pressure
    deficit delta (bar) over a width w (A); p_N = 0 everywhere (mechanical
    equilibrium).  gamma = integral over one interface of (p_N - p_T) dz =
    delta * w bar A = delta * w * 1e-5 N/m.  The box averages are what the
    engine's pressure tensor gives."""
    lz, w, delta = 100.0, 3.0, 250.0
    z = (np.arange(100000) + 0.5) * lz / 100000
    in_iface = (np.abs(z - 35.0) < w / 2) | (np.abs(z - 65.0) < w / 2)
    p_t = np.where(in_iface, -delta, 0.0)
    p_n = np.zeros_like(z)
    rng = np.random.default_rng(5)
    noise = rng.normal(0.0, 1.0, size=(3, 200))
    pxx = p_t.mean() + noise[0] - noise[0].mean()
    pyy = p_t.mean() + noise[1] - noise[1].mean()
    pzz = p_n.mean() + noise[2] - noise[2].mean()
    want_mN_m = delta * w * 1e-5 * 1e3
    assert abs(ob.surface_tension(pxx, pyy, pzz, lz) - want_mN_m) < 1e-9 * want_mN_m
