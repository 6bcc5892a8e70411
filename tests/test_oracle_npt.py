"""Pins of the Nose-Hoover NPT oracle (Sec. II.B: thermostat and barostat,
relaxation times 1 and 2.5 ps, p = 0): the NVE limit reproduces velocity
Verlet, the map is time reversible, and the extended energy H' is conserved
with an error that scales as dt^2."""
import numpy as np

import oracle
from tests.gpu_util import liquid


def test_frozen_thermostat_and_barostat_is_velocity_verlet():
    x, v, L = liquid(1, sigma=0.0)
    r = oracle.npt(x, v, L, 20, T0=298.0, tau_T=1e12, tau_P=1e12)
    xo, vo, _, _ = oracle.vv(x, v, L, 20, dt=10.0)
    d = r["x"] - xo
    d -= L * np.rint(d / L)
    assert np.abs(d).max() < 1e-9
    assert np.abs(r["v"] - vo).max() < 1e-12
    assert np.allclose(r["box"], L, rtol=1e-12, atol=0)


def test_time_reversible():
    x, v, L = liquid(1, sigma=0.0)
    a = oracle.npt(x, v, L, 40, T0=298.0, p_bar=0.0, tau_T=200.0, tau_P=500.0)
    st = a["state"].copy()
    st[0] = -st[0]; st[5:9] = -st[5:9]; st[13:17] = -st[13:17]
    b = oracle.npt(a["x"], -a["v"], a["box"], 40, T0=298.0, p_bar=0.0, tau_T=200.0, tau_P=500.0, state=st)
    d = b["x"] - x
    d -= L * np.rint(d / L)
    assert np.abs(d).max() < 1e-8
    assert np.abs(-b["v"] - v).max() < 1e-10
    assert np.allclose(b["box"], L, rtol=1e-12, atol=0)
    assert np.abs(b["state"][1:5]).max() < 1e-10 and np.abs(b["state"][9:13]).max() < 1e-10


def test_extended_energy_conserved_and_second_order():
    """Over 2 ps of a 298 K liquid with strong coupling (tau_T 0.2 ps, tau_P
    0.5 ps) the excursion of H' stays within twice that of the total energy
    under plain velocity Verlet at the same step, and falls as dt^2."""
    x, v, L = liquid(1, sigma=0.0)
    exc = {}
    for dt in (10.0, 5.0):
        n = int(round(2000.0 / dt))
        r = oracle.npt(x, v, L, n, T0=298.0, p_bar=0.0, tau_T=200.0, tau_P=500.0, dt=dt)
        H = r["rows"][:, 7]
        exc[dt] = np.abs(H - H[0]).max()
        _, _, _, th = oracle.vv(x, v, L, n, dt=dt)
        E = th[:, 0] + th[:, 1] + th[:, 2]
        assert exc[dt] < 2.0 * np.abs(E - E[0]).max()
        # the barostat and the thermostat do act
        assert np.ptp(r["rows"][:, 0]) > 1e-2 * r["rows"][0, 0]
    assert 2.5 < exc[10.0] / exc[5.0] < 6.0


def test_extended_energy_conserved_under_load():
    """p = 1000 bar: the p V term enters H' and the barostat force."""
    x, v, L = liquid(1, sigma=0.0)
    r = oracle.npt(x, v, L, 200, T0=298.0, p_bar=1000.0, tau_T=200.0, tau_P=500.0)
    H = r["rows"][:, 7]
    _, _, _, th = oracle.vv(x, v, L, 200, dt=10.0)
    E = th[:, 0] + th[:, 1] + th[:, 2]
    assert np.abs(H - H[0]).max() < 2.0 * np.abs(E - E[0]).max()
    assert r["rows"][0, 5] > 100.0          # p V is a sizeable term


def test_fixed_box_thermostat_and_tensor_trace():
    """tau_P <= 0: Nose-Hoover NVT.  The box stays put, H' (now without
    barostat terms) is conserved like the NVE energy, and the scalar
    pressure is the mean of the tensor diagonal."""
    x, v, L = liquid(1, sigma=0.0)
    r = oracle.npt(x, v, L, 200, T0=280.0, tau_T=200.0, tau_P=0.0)
    assert np.array_equal(r["box"], L)
    assert r["state"][0] == 0.0 and np.all(r["state"][9:17] == 0.0)
    H = r["rows"][:, 7]
    _, _, _, th = oracle.vv(x, v, L, 200, dt=10.0)
    E = th[:, 0] + th[:, 1] + th[:, 2]
    assert np.abs(H - H[0]).max() < 2.0 * np.abs(E - E[0]).max()
    assert np.allclose(r["rows"][:, 1], r["rows"][:, 8:11].mean(axis=1), rtol=1e-9, atol=1e-6)
    assert abs(r["rows"][-50:, 2].mean() - 280.0) < 25.0       # pulled from 298 K toward 280 K
