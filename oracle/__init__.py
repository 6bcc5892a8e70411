"""FP64 CPU oracle for the mW Stillinger-Weber hot path (ctypes wrapper).

TEST INFRASTRUCTURE ONLY: this package may be imported by the tests, by the
smoke check and by the benchmark's CPU-baseline leg, and by nothing else.  It
shares no code with the HIP engine in ``paper_0809_2811_amd``; the product path
never calls it.

The arithmetic lives in ``sw_oracle.cpp`` (plain C++ doubles, dual numbers for
tangents) and ``obs_oracle.cpp`` (the observables of Sec. II.C); this module
only marshals numpy arrays, except for the mean square displacement, which is
a few numpy lines here.  See the sources' headers for the equations they
follow (Sec. II.A of the mW paper, Eq. E, phi2, phi3; Sec. II.C).
"""
from __future__ import annotations

import ctypes
import pathlib
import subprocess

import numpy as np

_HERE = pathlib.Path(__file__).resolve().parent
_SRC = _HERE / "sw_oracle.cpp"
_SRCS = (_SRC, _HERE / "obs_oracle.cpp")
_LIB_PATH = _HERE / "liboracle_sw.so"
_lib = None

# mW parameters (Sec. II.A constants; lambda, epsilon, sigma from Sec. II.D).
# cos(theta0) is -1/3 exactly, the tetrahedral angle the paper quotes as 109.47 deg.
MW = dict(lam=23.15, eps=6.189, sig=2.3925, A=7.049556277, B=0.6022245584,
          p=4.0, q=0.0, gam=1.2, a=1.8, cos0=-1.0 / 3.0)
M_WATER = 18.015
ACC = 4.184e-4
KB = 8.314462618 / 4184.0
THERMO_WIDTH = 12


def build(force: bool = True) -> pathlib.Path:
    """Compile the oracle with g++ (FP64, no fast-math)."""
    if force or not _LIB_PATH.exists():
        cmd = ["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fPIC", "-shared", "-o", str(_LIB_PATH),
               *[str(s) for s in _SRCS]]
        subprocess.run(cmd, check=True)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not _LIB_PATH.exists() or any(_LIB_PATH.stat().st_mtime < s.stat().st_mtime for s in _SRCS):
            build()
        L = ctypes.CDLL(str(_LIB_PATH))
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        llp = ctypes.POINTER(ctypes.c_longlong)
        c_int, c_double = ctypes.c_int, ctypes.c_double
        L.ora_phi2.argtypes = [c_double, dp]; L.ora_phi2.restype = c_double
        L.ora_phi3.argtypes = [c_double, c_double, c_double, dp]; L.ora_phi3.restype = c_double
        L.ora_energy_brute.argtypes = [c_int, dp, dp, dp, dp, dp]
        L.ora_forces.argtypes = [c_int, dp, dp, dp, dp, dp, dp, dp, dp]
        L.ora_tangent.argtypes = [c_int, dp, dp, dp, dp, dp, dp, dp, dp, dp, dp, dp, dp]
        L.ora_vv.argtypes = [c_int, dp, dp, dp, dp, dp, c_double, c_double, c_int, c_int,
                             c_double, c_double, dp]
        L.ora_traj_loss.argtypes = [c_int, dp, dp, dp, dp, c_double, c_double, c_int, c_double,
                                    c_double, c_double, dp, dp]
        L.ora_traj_loss.restype = c_double
        L.ora_adjoint.argtypes = [c_int, dp, dp, dp, dp, c_double, c_double, c_int, c_double,
                                  c_double, c_double, dp, dp, dp, dp, dp, dp]
        L.ora_neighbour_counts.argtypes = [c_int, dp, dp, c_double, ip]
        L.ora_neighbour_lists.argtypes = [c_int, dp, dp, c_double, llp, ip]
        L.ora_npt.argtypes = [c_int, dp, dp, dp, dp, c_double, c_double, c_int, c_double, c_double, c_double,
                              c_double, c_int, dp, dp]
        u64p = ctypes.POINTER(ctypes.c_uint64)
        L.ora_quantize.argtypes = [c_int, dp, dp, ctypes.POINTER(ctypes.c_uint32)]
        L.ora_rdf.argtypes = [c_int, dp, dp, c_int, dp, u64p]
        L.ora_adf.argtypes = [c_int, dp, dp, c_int, c_double, c_int, dp, u64p, llp]
        _lib = L
    return _lib


def params(**over) -> np.ndarray:
    """Parameter block (lambda, epsilon, sigma, A, B, p, q, gamma, a, cos_theta0)."""
    p = dict(MW)
    p.update(over)
    return np.array([p["lam"], p["eps"], p["sig"], p["A"], p["B"], p["p"], p["q"],
                     p["gam"], p["a"], p["cos0"]], dtype=np.float64)


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check(rc):
    if rc != 0:
        raise ValueError("oracle: box edge shorter than twice the cut-off")


def phi2(r, P=None):
    P = params() if P is None else _d(P)
    return lib().ora_phi2(float(r), _ptr(P))


def phi3(r, s, costh, P=None):
    P = params() if P is None else _d(P)
    return lib().ora_phi3(float(r), float(s), float(costh), _ptr(P))


def energy_brute(x, box, P=None):
    """O(N^3) energy straight from Eq. E: returns (E2, E3)."""
    x = _d(x); box = _d(box); P = params() if P is None else _d(P)
    e2 = ctypes.c_double(); e3 = ctypes.c_double()
    _check(lib().ora_energy_brute(len(x), _ptr(x), _ptr(box), _ptr(P), ctypes.byref(e2), ctypes.byref(e3)))
    return e2.value, e3.value


def forces(x, box, P=None):
    """Cell-list energy, forces and virial: dict(F, F3, E2, E3, W2, W3) (W are 3x3)."""
    x = _d(x); box = _d(box); P = params() if P is None else _d(P)
    n = len(x)
    F = np.zeros((n, 3)); F3 = np.zeros((n, 3)); e = np.zeros(2); w2 = np.zeros(9); w3 = np.zeros(9)
    _check(lib().ora_forces(n, _ptr(x), _ptr(box), _ptr(P), _ptr(F), _ptr(F3), _ptr(e), _ptr(w2), _ptr(w3)))
    return dict(F=F, F3=F3, E2=e[0], E3=e[1], W2=w2.reshape(3, 3), W3=w3.reshape(3, 3))


def tangent(x, box, xdot=None, P=None, Pdot=None):
    """Forward-mode tangent: dict(F, Fdot, F3, F3dot, E, Edot, Wdot_trace)."""
    x = _d(x); box = _d(box); P = params() if P is None else _d(P)
    xdot = None if xdot is None else _d(xdot)
    Pdot = None if Pdot is None else _d(Pdot)
    n = len(x)
    out = {k: np.zeros((n, 3)) for k in ("F", "Fdot", "F3", "F3dot")}
    e = np.zeros(2); ed = np.zeros(2); wt = np.zeros(2)
    _check(lib().ora_tangent(n, _ptr(x), _ptr(xdot), _ptr(box), _ptr(P), _ptr(Pdot), _ptr(out["F"]),
                             _ptr(out["Fdot"]), _ptr(out["F3"]), _ptr(out["F3dot"]), _ptr(e), _ptr(ed),
                             _ptr(wt)))
    out.update(E=e, Edot=ed, Wdot_trace=wt)
    return out


def vv(x, v, box, nsteps, dt=10.0, mass=M_WATER, P=None, thermostat=0, T0=0.0, tau=1000.0):
    """FP64 velocity Verlet; returns (x, v, F, thermo[nsteps, 12])."""
    x = _d(x).copy(); v = _d(v).copy(); box = _d(box); P = params() if P is None else _d(P)
    n = len(x)
    F = np.zeros((n, 3)); thermo = np.zeros((max(nsteps, 1), THERMO_WIDTH))
    _check(lib().ora_vv(n, _ptr(x), _ptr(v), _ptr(F), _ptr(box), _ptr(P), float(mass), float(dt),
                        int(nsteps), int(thermostat), float(T0), float(tau), _ptr(thermo)))
    return x, v, F, thermo[:nsteps]


def traj_loss(x0, v0, box, nsteps, dt=10.0, mass=M_WATER, P=None, aU=1.0, a3=1.0, aW=0.0):
    """1/(S+1) sum_s [aU U + a3 U3 + aW W](x_s) / N over an NVE trajectory; (loss, xS, vS)."""
    x0 = _d(x0); v0 = _d(v0); box = _d(box); P = params() if P is None else _d(P)
    n = len(x0)
    xS = np.zeros((n, 3)); vS = np.zeros((n, 3))
    loss = lib().ora_traj_loss(n, _ptr(x0), _ptr(v0), _ptr(box), _ptr(P), float(mass), float(dt),
                               int(nsteps), float(aU), float(a3), float(aW), _ptr(xS), _ptr(vS))
    return loss, xS, vS


def adjoint(x0, v0, box, nsteps, dt=10.0, mass=M_WATER, P=None, aU=1.0, a3=1.0,
            xbar_S=None, vbar_S=None, aW=0.0):
    """Discrete adjoint of NVE velocity Verlet: dict(loss, xbar0, vbar0, thbar[3])."""
    x0 = _d(x0); v0 = _d(v0); box = _d(box); P = params() if P is None else _d(P)
    n = len(x0)
    xs = None if xbar_S is None else _d(xbar_S)
    vs = None if vbar_S is None else _d(vbar_S)
    loss = ctypes.c_double()
    xb = np.zeros((n, 3)); vb = np.zeros((n, 3)); th = np.zeros(3)
    _check(lib().ora_adjoint(n, _ptr(x0), _ptr(v0), _ptr(box), _ptr(P), float(mass), float(dt),
                             int(nsteps), float(aU), float(a3), float(aW), _ptr(xs), _ptr(vs),
                             ctypes.byref(loss), _ptr(xb), _ptr(vb), _ptr(th)))
    return dict(loss=loss.value, xbar0=xb, vbar0=vb, thbar=th)


def neighbour_counts(x, box, rc):
    x = _d(x); box = _d(box)
    c = np.zeros(len(x), dtype=np.int32)
    _check(lib().ora_neighbour_counts(len(x), _ptr(x), _ptr(box), float(rc),
                                      c.ctypes.data_as(ctypes.POINTER(ctypes.c_int))))
    return c


def neighbour_lists(x, box, rc):
    """Sorted neighbour rows within rc as a list of numpy int arrays."""
    x = _d(x); box = _d(box)
    n = len(x)
    off = np.zeros(n + 1, dtype=np.int64)
    llp = ctypes.POINTER(ctypes.c_longlong)
    _check(lib().ora_neighbour_lists(n, _ptr(x), _ptr(box), float(rc), off.ctypes.data_as(llp), None))
    idx = np.zeros(max(int(off[-1]), 1), dtype=np.int32)
    _check(lib().ora_neighbour_lists(n, _ptr(x), _ptr(box), float(rc), off.ctypes.data_as(llp),
                                     idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int))))
    return [idx[off[i]:off[i + 1]] for i in range(n)]


def temperature(v, mass=M_WATER):
    """T = 2 KE / ((3N - 3) k_B)."""
    v = _d(v)
    ke = 0.5 * mass * float(np.sum(v * v)) / ACC
    return 2.0 * ke / ((3 * len(v) - 3) * KB)


# ---------------------------------------------------------------- observables
# Sec. II.C: pair distribution, angular distribution of the n_c closest
# neighbours, mean square displacement.

def quantize(x, box):
    """The engine's coordinate convention: u = floor(frac(x / L) 2^32)."""
    x = _d(x); box = _d(box)
    u = np.zeros((len(x), 3), dtype=np.uint32)
    lib().ora_quantize(len(x), _ptr(x), _ptr(box), u.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)))
    return u


def rdf_counts(x, box, r2_edges):
    """Ordered-pair counts per bin of squared distance (edges ascending)."""
    x = _d(x); box = _d(box); e = _d(r2_edges)
    c = np.zeros(len(e) - 1, dtype=np.uint64)
    lib().ora_rdf(len(x), _ptr(x), _ptr(box), len(e) - 1, _ptr(e), c.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
    return c


def adf_counts(x, box, n_near, r_search, cos_edges):
    """Angle counts over the n_near closest neighbours within r_search of each
    centre (cosine edges descending); returns (counts, centres skipped)."""
    x = _d(x); box = _d(box); e = _d(cos_edges)
    c = np.zeros(len(e) - 1, dtype=np.uint64)
    short = ctypes.c_longlong(0)
    lib().ora_adf(len(x), _ptr(x), _ptr(box), int(n_near), float(r_search) ** 2, len(e) - 1, _ptr(e),
                  c.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), ctypes.byref(short))
    return c, short.value


class Displacement:
    """Unwrapped displacement of every atom since the reference frame
    (Einstein relation of Sec. II.C): between two frames each atom moves by
    the minimum image of its position difference, accumulated in FP64."""

    def __init__(self, x, box):
        self.last = _d(x).copy()
        self.box = _d(box)
        self.acc = np.zeros_like(self.last)

    def update(self, x):
        x = _d(x)
        d = x - self.last
        d = d - self.box * np.rint(d / self.box)
        self.acc += d
        self.last = x.copy()
        return float(np.mean(np.sum(self.acc * self.acc, axis=1)))


# ---------------------------------------------------------------- NPT
BAR = 1e5 * 1e-30 * 6.02214076e23 / 4184.0      # kcal/mol/A^3 per bar
NPT_STATE = 17
NPT_ROW = 11


def npt(x, v, box, nsteps, T0, p_bar=0.0, tau_T=1000.0, tau_P=2500.0, chain=3, state=None, dt=10.0,
        mass=M_WATER, P=None):
    """Nose-Hoover NPT (see ora_npt; tau_P <= 0: fixed box, NVT); returns the
    final x, v, box, extended state and one row per step (V, P_int in bar, T,
    U, KE, pV, E_ext, H', P_xx, P_yy, P_zz in bar)."""
    x = _d(x).copy(); v = _d(v).copy(); L = _d(box).copy()
    st = np.zeros(NPT_STATE) if state is None else _d(state).copy()
    rows = np.zeros((max(nsteps, 1), NPT_ROW))
    P = params() if P is None else _d(P)
    rc = lib().ora_npt(len(x), _ptr(x), _ptr(v), _ptr(L), _ptr(P), float(mass), float(dt), int(nsteps),
                       float(T0), float(p_bar) * BAR, float(tau_T), float(tau_P), int(chain), _ptr(st), _ptr(rows))
    if rc != 0:
        raise ValueError(f"oracle npt: error {rc}")
    rows = rows[:nsteps].copy()
    rows[:, 1] /= BAR
    rows[:, 8:11] /= BAR
    return dict(x=x, v=v, box=L, state=st, rows=rows)
