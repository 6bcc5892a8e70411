"""ctypes binding of libsw (include/sw.h).

Argument marshalling only: every function here checks tensor shapes, dtypes
and devices, then calls the C entry point of the same name with raw device
pointers and the current HIP stream.  All computation happens in the HIP
kernels.  There is no CPU fallback: if libsw.so is missing or no GPU is
present, the calls raise.
"""
from __future__ import annotations

import atexit
import ctypes
import pathlib
import sys
import weakref
from typing import Optional, Sequence

import numpy as np

_LIB_PATH = pathlib.Path(__file__).resolve().parent / "libsw.so"
_lib = None

SW_OK = 0
SW_EINVAL = -1
SW_EBOX_TOO_SMALL = -2
SW_ENBR_OVERFLOW = -3
SW_ECELL_OVERFLOW = -4
SW_EOVERLAP = -5
SW_EHIP = -6
SW_ENOMEM = -7
SW_EUNSUPPORTED = -8
SW_ESTATE = -9
SW_ETIMEOUT = -10
SW_ESCRATCH = -11
SW_NOALLOC_MAX_ATOMS = 16384

SW_NVE, SW_RESCALE, SW_BERENDSEN = 0, 1, 2
SW_TERM_TWO_BODY, SW_TERM_THREE_BODY = 1, 2
SW_THERMO_WIDTH = 12
SW_Q_NATOMS, SW_Q_NREPLICAS, SW_Q_NBR_CAPACITY, SW_Q_REBUILDS = 0, 1, 2, 3
SW_Q_CELL_CAPACITY, SW_Q_DEVICE_BYTES, SW_Q_STEPS = 5, 6, 7
SW_Q_TIME_MOMENTS_NS, SW_Q_TIME_FORCES_NS, SW_Q_TIMED_STEPS = 8, 9, 10
SW_Q_AUDIT_PAIRS, SW_Q_MISSED_PAIRS, SW_Q_PERSISTENT_GROUPS = 12, 13, 14

# symbols declared in include/sw.h
EXPORTS = ("sw_params_mw", "sw_create", "sw_destroy", "sw_build_neighbors", "sw_get_neighbors",
           "sw_forces", "sw_step", "sw_grad", "sw_adjoint", "sw_set_tuning", "sw_get_tuning",
           "sw_query", "sw_status_string", "sw_last_hip_error", "sw_rdf", "sw_adf", "sw_msd",
           "sw_npt", "sw_get_box", "sw_npt_state", "sw_forces_noalloc")
SW_NPT_WIDTH = 11
SW_Q_MIN_CELL_EDGE = 11
SW_NPT_STATE = 17


class sw_params(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in
                ("lambda_", "epsilon", "sigma", "A", "B", "p", "q", "gamma", "a", "cos_theta0")]


class sw_tuning(ctypes.Structure):
    _fields_ = [("lanes_per_atom", ctypes.c_int), ("graph_steps", ctypes.c_int),
                ("persistent", ctypes.c_int), ("rebuild_every", ctypes.c_int), ("timing", ctypes.c_int),
                ("sync_rebuild", ctypes.c_int), ("audit_every", ctypes.c_int)]


class SWError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {status_string(code)} ({code})")


def library_path() -> pathlib.Path:
    return _LIB_PATH


def lib():
    """Load libsw.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        # torch ships its own libamdhip64.so.7; load it first so that libsw
        # binds to the same HIP runtime instead of a second copy.
        import torch  # noqa: F401
        if not _LIB_PATH.exists():
            raise RuntimeError(f"{_LIB_PATH} is missing: build it with paper_0809_2811_amd.build.build()")
        L = ctypes.CDLL(str(_LIB_PATH))
        vp, ip, dp, fp = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_void_p
        P = ctypes.POINTER
        L.sw_params_mw.argtypes = [P(sw_params)]; L.sw_params_mw.restype = None
        L.sw_create.argtypes = [P(vp), ip, P(ctypes.c_longlong), P(ctypes.c_double), dp, dp, ip]
        L.sw_destroy.argtypes = [vp]; L.sw_destroy.restype = None
        L.sw_build_neighbors.argtypes = [vp, fp, vp]
        L.sw_get_neighbors.argtypes = [vp, P(ctypes.c_int), P(ctypes.c_int), ip]
        L.sw_forces.argtypes = [vp, fp, P(sw_params), fp, vp, vp, vp]
        L.sw_step.argtypes = [vp, fp, fp, fp, P(sw_params), dp, dp, ip, ip, P(ctypes.c_double), dp, vp, ip, vp]
        L.sw_grad.argtypes = [vp, fp, fp, P(sw_params), ip, fp, vp, vp, vp]
        L.sw_adjoint.argtypes = [vp, fp, fp, P(sw_params), dp, dp, ip, ip, dp, dp, dp, fp, fp, vp, fp, fp, vp,
                                 fp, fp, vp]
        L.sw_set_tuning.argtypes = [vp, P(sw_tuning)]
        L.sw_get_tuning.argtypes = [vp, P(sw_tuning)]
        L.sw_query.argtypes = [vp, ip, P(ctypes.c_longlong)]
        L.sw_status_string.argtypes = [ip]; L.sw_status_string.restype = ctypes.c_char_p
        L.sw_last_hip_error.argtypes = [vp]
        L.sw_rdf.argtypes = [vp, fp, ip, P(ctypes.c_double), vp, vp]
        L.sw_adf.argtypes = [vp, fp, ip, dp, ip, P(ctypes.c_double), vp, P(ctypes.c_longlong), vp]
        L.sw_msd.argtypes = [vp, fp, ip, vp, vp]
        L.sw_npt.argtypes = [vp, fp, fp, fp, P(sw_params), dp, dp, ip, P(ctypes.c_double), P(ctypes.c_double),
                             dp, dp, ip, ip, vp, ip, vp]
        L.sw_get_box.argtypes = [vp, P(ctypes.c_double)]
        L.sw_npt_state.argtypes = [vp, P(ctypes.c_double), ip]
        L.sw_forces_noalloc.argtypes = [fp, ctypes.c_longlong, P(ctypes.c_double), P(sw_params), fp, vp, vp, vp]
        _lib = L
    return _lib


def status_string(code: int) -> str:
    return lib().sw_status_string(int(code)).decode()


def _check(code: int, where: str):
    if code != SW_OK:
        raise SWError(code, where)


def params_mw(**over) -> sw_params:
    """mW parameter block (Sec. II.A / II.D) from the library, with overrides
    given as lambda_, epsilon, sigma, A, B, p, q, gamma, a, cos_theta0."""
    p = sw_params()
    lib().sw_params_mw(ctypes.byref(p))
    for k, val in over.items():
        setattr(p, k, float(val))
    return p


def params_from_array(arr) -> sw_params:
    """From the 10-vector (lambda, epsilon, sigma, A, B, p, q, gamma, a, cos_theta0)."""
    a = [float(x) for x in arr]
    return sw_params(*a)


# ------------------------------------------------------------------ tensors
def _torch():
    import torch
    return torch


def _stream():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _atoms(t, n, name, writable=False):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float32 or not t.is_cuda:
        raise TypeError(f"{name}: expected a float32 CUDA tensor")
    if tuple(t.shape) != (n, 4) or not t.is_contiguous():
        raise ValueError(f"{name}: expected a contiguous [{n}, 4] tensor, got {tuple(t.shape)}")
    return ctypes.c_void_p(t.data_ptr())


def _doubles(t, shape, name):
    torch = _torch()
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda:
        raise TypeError(f"{name}: expected a float64 CUDA tensor")
    if tuple(t.shape) != tuple(shape) or not t.is_contiguous():
        raise ValueError(f"{name}: expected a contiguous {tuple(shape)} tensor, got {tuple(t.shape)}")
    return ctypes.c_void_p(t.data_ptr())


# ------------------------------------------------------------------ entry points
def sw_create(offsets: Sequence[int], boxes, cutoff: float, skin: float, nbr_capacity: int = 48) -> int:
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    box = np.ascontiguousarray(boxes, dtype=np.float64).reshape(-1)
    R = len(off) - 1
    if R < 1 or box.size != 3 * R:
        raise ValueError("offsets must have R+1 entries and boxes R*3")
    h = ctypes.c_void_p()
    _check(lib().sw_create(ctypes.byref(h), R, off.ctypes.data_as(ctypes.POINTER(ctypes.c_longlong)),
                           box.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), float(cutoff), float(skin),
                           int(nbr_capacity)), "sw_create")
    return h.value


def sw_destroy(ctx: int):
    lib().sw_destroy(ctypes.c_void_p(ctx))


def sw_build_neighbors(ctx: int, x, n: int):
    _check(lib().sw_build_neighbors(ctypes.c_void_p(ctx), _atoms(x, n, "x"), _stream()), "sw_build_neighbors")


def sw_get_neighbors(ctx: int, n: int, max_per_row: int):
    counts = np.zeros(n, dtype=np.int32)
    rows = np.zeros((n, max_per_row), dtype=np.int32)
    ip = ctypes.POINTER(ctypes.c_int)
    _check(lib().sw_get_neighbors(ctypes.c_void_p(ctx), counts.ctypes.data_as(ip), rows.ctypes.data_as(ip),
                                  int(max_per_row)), "sw_get_neighbors")
    return counts, rows


def sw_forces(ctx: int, x, params: sw_params, f, energy=None, virial=None, n: Optional[int] = None,
              R: Optional[int] = None):
    n = x.shape[0] if n is None else n
    R = (energy.shape[0] if energy is not None else virial.shape[0] if virial is not None else 1) if R is None else R
    _check(lib().sw_forces(ctypes.c_void_p(ctx), _atoms(x, n, "x"), ctypes.byref(params), _atoms(f, n, "f"),
                           _doubles(energy, (R, 2), "energy"), _doubles(virial, (R, 6), "virial"), _stream()),
           "sw_forces")


def sw_forces_noalloc(x, box, params: sw_params, f, energy=None, virial=None):
    """Context-free, allocation-free sw_forces for one box (see include/sw.h)."""
    n = x.shape[0]
    b = np.ascontiguousarray(box, dtype=np.float64).reshape(3)
    _check(lib().sw_forces_noalloc(_atoms(x, n, "x"), int(n), b.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                   ctypes.byref(params), _atoms(f, n, "f"), _doubles(energy, (1, 2), "energy"),
                                   _doubles(virial, (1, 6), "virial"), _stream()), "sw_forces_noalloc")


def sw_step(ctx: int, x, v, f, params: sw_params, mass: float, dt: float, nsteps: int, thermostat: int = SW_NVE,
            T0=None, tau_fs: float = 1000.0, thermo=None, thermo_every: int = 1, R: int = 1):
    n = x.shape[0]
    t0 = None
    if T0 is not None:
        t0 = np.ascontiguousarray(np.broadcast_to(np.asarray(T0, dtype=np.float64), (R,)))
    rows = (nsteps // thermo_every) if thermo is not None else 0
    _check(lib().sw_step(ctypes.c_void_p(ctx), _atoms(x, n, "x"), _atoms(v, n, "v"), _atoms(f, n, "f"),
                         ctypes.byref(params), float(mass), float(dt), int(nsteps), int(thermostat),
                         None if t0 is None else t0.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                         float(tau_fs), _doubles(thermo, (rows, R, SW_THERMO_WIDTH), "thermo"), int(thermo_every),
                         _stream()), "sw_step")


def sw_grad(ctx: int, x, w, params: sw_params, hvp, wdF=None, dU=None, R: int = 1,
            term_mask: int = SW_TERM_TWO_BODY | SW_TERM_THREE_BODY):
    n = x.shape[0]
    _check(lib().sw_grad(ctypes.c_void_p(ctx), _atoms(x, n, "x"), _atoms(w, n, "w"), ctypes.byref(params),
                         int(term_mask), _atoms(hvp, n, "hvp"), _doubles(wdF, (R, 3), "wdF"),
                         _doubles(dU, (R, 3), "dU"), _stream()), "sw_grad")


def sw_adjoint(ctx: int, x0, v0, params: sw_params, mass: float, dt: float, nsteps: int, ckpt_every: int,
               aU: float, a3: float, xbar_S, vbar_S, loss, xbar0, vbar0, thbar, xS=None, vS=None, R: int = 1,
               aW: float = 0.0):
    n = x0.shape[0]
    opt = lambda t, name: None if t is None else _atoms(t, n, name)  # noqa: E731
    _check(lib().sw_adjoint(ctypes.c_void_p(ctx), _atoms(x0, n, "x0"), _atoms(v0, n, "v0"), ctypes.byref(params),
                            float(mass), float(dt), int(nsteps), int(ckpt_every), float(aU), float(a3), float(aW),
                            opt(xbar_S, "xbar_S"), opt(vbar_S, "vbar_S"), _doubles(loss, (R,), "loss"),
                            _atoms(xbar0, n, "xbar0"), _atoms(vbar0, n, "vbar0"), _doubles(thbar, (R, 3), "thbar"),
                            opt(xS, "xS"), opt(vS, "vS"), _stream()), "sw_adjoint")


def _counts(t, shape, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or t.dtype != torch.int64 or not t.is_cuda:
        raise TypeError(f"{name}: expected an int64 CUDA tensor (holds unsigned counts)")
    if tuple(t.shape) != tuple(shape) or not t.is_contiguous():
        raise ValueError(f"{name}: expected a contiguous {tuple(shape)} tensor, got {tuple(t.shape)}")
    return ctypes.c_void_p(t.data_ptr())


def _host_doubles(a, name):
    import numpy as np
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.ndim != 1 or len(a) < 2:
        raise ValueError(f"{name}: expected at least two edges")
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def sw_rdf(ctx: int, x, r2_edges, counts, R: int = 1):
    n = x.shape[0]
    e, ep = _host_doubles(r2_edges, "r2_edges")
    nb = len(e) - 1
    _check(lib().sw_rdf(ctypes.c_void_p(ctx), _atoms(x, n, "x"), nb, ep, _counts(counts, (R, nb), "counts"),
                        _stream()), "sw_rdf")


def sw_adf(ctx: int, x, n_near: int, r_search: float, cos_edges, counts, R: int = 1) -> int:
    n = x.shape[0]
    e, ep = _host_doubles(cos_edges, "cos_edges")
    nb = len(e) - 1
    short = ctypes.c_longlong(0)
    _check(lib().sw_adf(ctypes.c_void_p(ctx), _atoms(x, n, "x"), int(n_near), float(r_search), nb, ep,
                        _counts(counts, (R, nb), "counts"), ctypes.byref(short), _stream()), "sw_adf")
    return short.value


def sw_msd(ctx: int, x, reset: bool, msd, R: int = 1):
    n = x.shape[0]
    _check(lib().sw_msd(ctypes.c_void_p(ctx), _atoms(x, n, "x"), 1 if reset else 0, _doubles(msd, (R,), "msd"),
                        _stream()), "sw_msd")


def sw_npt(ctx: int, x, v, f, params: sw_params, mass: float, dt: float, nsteps: int, T0, p_bar,
           tau_T: float, tau_P: float, chain: int, reset: bool, rows, every: int, R: int = 1):
    import numpy as np
    n = x.shape[0]
    t0 = np.ascontiguousarray(np.broadcast_to(np.asarray(T0, dtype=np.float64), (R,)))
    pb = np.ascontiguousarray(np.broadcast_to(np.asarray(p_bar, dtype=np.float64), (R,)))
    dptr = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))  # noqa: E731
    nrec = nsteps // every if every > 0 else 0
    _check(lib().sw_npt(ctypes.c_void_p(ctx), _atoms(x, n, "x"), _atoms(v, n, "v"),
                        None if f is None else _atoms(f, n, "f"), ctypes.byref(params), float(mass), float(dt),
                        int(nsteps), dptr(t0), dptr(pb), float(tau_T), float(tau_P), int(chain), 1 if reset else 0,
                        None if rows is None else _doubles(rows, (nrec, R, SW_NPT_WIDTH), "rows"), int(every),
                        _stream()), "sw_npt")


def sw_get_box(ctx: int, R: int = 1):
    import numpy as np
    b = np.zeros((R, 3), dtype=np.float64)
    _check(lib().sw_get_box(ctypes.c_void_p(ctx), b.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), "sw_get_box")
    return b


def sw_npt_state(ctx: int, R: int = 1, state=None):
    """Read (state None) or replace the extended variables, [R][SW_NPT_STATE]."""
    import numpy as np
    if state is None:
        out = np.zeros((R, SW_NPT_STATE), dtype=np.float64)
        _check(lib().sw_npt_state(ctypes.c_void_p(ctx), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 0),
               "sw_npt_state")
        return out
    st = np.ascontiguousarray(np.asarray(state, dtype=np.float64).reshape(R, SW_NPT_STATE))
    _check(lib().sw_npt_state(ctypes.c_void_p(ctx), st.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 1),
           "sw_npt_state")
    return st


def sw_set_tuning(ctx: int, lanes_per_atom=8, graph_steps=0, persistent=0, rebuild_every=0, timing=0,
                  sync_rebuild=0, audit_every=0):
    t = sw_tuning(int(lanes_per_atom), int(graph_steps), int(persistent), int(rebuild_every), int(timing),
                  int(sync_rebuild), int(audit_every))
    _check(lib().sw_set_tuning(ctypes.c_void_p(ctx), ctypes.byref(t)), "sw_set_tuning")


def sw_get_tuning(ctx: int) -> dict:
    t = sw_tuning()
    _check(lib().sw_get_tuning(ctypes.c_void_p(ctx), ctypes.byref(t)), "sw_get_tuning")
    return dict(lanes_per_atom=t.lanes_per_atom, graph_steps=t.graph_steps, persistent=t.persistent,
                rebuild_every=t.rebuild_every, timing=t.timing, sync_rebuild=t.sync_rebuild,
                audit_every=t.audit_every)


def sw_query(ctx: int, what: int) -> int:
    out = ctypes.c_longlong()
    _check(lib().sw_query(ctypes.c_void_p(ctx), int(what), ctypes.byref(out)), "sw_query")
    return out.value


# ------------------------------------------------------------------ convenience
# Contexts still open, destroyed by close_all() when the interpreter exits.
_live: "weakref.WeakSet[Context]" = weakref.WeakSet()


def close_all():
    """Destroy every open context now, newest first.  Registered with atexit,
    so that sw_destroy (graph, stream and device-memory release) runs while
    the HIP runtime is still up, before interpreter shutdown collects the
    remaining objects in no fixed order."""
    for c in sorted(list(_live), key=lambda c: -c._serial):
        c.close()


atexit.register(close_all)
_serial = [0]


class Context:
    """Owns one sw_ctx.  offsets: int[R+1]; boxes: [R,3] (A).

    Use it as a context manager (`with Context(...) as c:`) or call close();
    contexts left open are destroyed at interpreter exit by close_all(), and
    never from a finaliser during interpreter shutdown."""

    def __init__(self, offsets, boxes, cutoff: Optional[float] = None, skin: float = 1.0,
                 nbr_capacity: int = 48, tuning: Optional[dict] = None):
        if cutoff is None:
            p = params_mw()
            cutoff = p.a * p.sigma
        self.offsets = np.asarray(offsets, dtype=np.int64)
        self.boxes = np.asarray(boxes, dtype=np.float64).reshape(-1, 3)
        self.R = len(self.offsets) - 1
        self.n = int(self.offsets[-1])
        self.cutoff, self.skin = float(cutoff), float(skin)
        self.handle = sw_create(self.offsets, self.boxes, cutoff, skin, nbr_capacity)
        _serial[0] += 1
        self._serial = _serial[0]
        _live.add(self)
        if tuning:
            self.set_tuning(**tuning)

    def close(self):
        """Release the device context (idempotent)."""
        if getattr(self, "handle", None):
            h, self.handle = self.handle, None
            _live.discard(self)
            sw_destroy(h)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False

    def __del__(self):
        # A context dropped during interpreter shutdown is left to the
        # process exit: the HIP runtime may already be finalising.
        if sys is None or sys.is_finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def set_tuning(self, **kw):
        cur = sw_get_tuning(self.handle)
        cur.update(kw)
        sw_set_tuning(self.handle, **cur)

    def tuning(self) -> dict:
        return sw_get_tuning(self.handle)

    def build_neighbors(self, x):
        sw_build_neighbors(self.handle, x, self.n)

    def neighbors(self, max_per_row: int = 256):
        return sw_get_neighbors(self.handle, self.n, max_per_row)

    def forces(self, x, params: Optional[sw_params] = None):
        torch = _torch()
        params = params_mw() if params is None else params
        f = torch.empty_like(x)
        e = torch.empty((self.R, 2), dtype=torch.float64, device=x.device)
        w = torch.empty((self.R, 6), dtype=torch.float64, device=x.device)
        sw_forces(self.handle, x, params, f, e, w, n=self.n, R=self.R)
        return f, e, w

    def step(self, x, v, nsteps: int, dt: float = 10.0, mass: float = 18.015, params: Optional[sw_params] = None,
             thermostat: int = SW_NVE, T0=None, tau_fs: float = 1000.0, thermo_every: int = 0, f=None):
        """Advance (x, v) in place; returns (f, thermo or None)."""
        torch = _torch()
        params = params_mw() if params is None else params
        f = torch.empty_like(x) if f is None else f
        thermo = None
        if thermo_every > 0 and nsteps >= thermo_every:
            thermo = torch.empty((nsteps // thermo_every, self.R, SW_THERMO_WIDTH), dtype=torch.float64,
                                 device=x.device)
        sw_step(self.handle, x, v, f, params, mass, dt, nsteps, thermostat, T0, tau_fs, thermo,
                max(thermo_every, 1), R=self.R)
        return f, thermo

    def grad(self, x, w, params: Optional[sw_params] = None, term_mask: int = SW_TERM_TWO_BODY | SW_TERM_THREE_BODY):
        """(dF/dx) w, w . dF/d(lambda, eps, sigma) and dU/d(lambda, eps, sigma)
        of the terms selected by term_mask (see sw_grad in include/sw.h)."""
        torch = _torch()
        params = params_mw() if params is None else params
        hvp = torch.empty_like(x)
        wdF = torch.empty((self.R, 3), dtype=torch.float64, device=x.device)
        dU = torch.empty((self.R, 3), dtype=torch.float64, device=x.device)
        sw_grad(self.handle, x, w, params, hvp, wdF, dU, R=self.R, term_mask=term_mask)
        return hvp, wdF, dU

    def adjoint(self, x0, v0, nsteps: int, dt: float = 10.0, mass: float = 18.015, ckpt_every: int = 20,
                aU: float = 1.0, a3: float = 1.0, params: Optional[sw_params] = None, xbar_S=None, vbar_S=None,
                aW: float = 0.0):
        """Loss, dL/dx0, dL/dv0, dL/d(lambda, eps, sigma) and the final state of
        an NVE trajectory (see sw_adjoint in include/sw.h; aW weights the
        virial trace)."""
        torch = _torch()
        params = params_mw() if params is None else params
        loss = torch.empty(self.R, dtype=torch.float64, device=x0.device)
        thbar = torch.empty((self.R, 3), dtype=torch.float64, device=x0.device)
        xbar0, vbar0 = torch.empty_like(x0), torch.empty_like(x0)
        xS, vS = torch.empty_like(x0), torch.empty_like(x0)
        sw_adjoint(self.handle, x0, v0, params, mass, dt, nsteps, ckpt_every, aU, a3, xbar_S, vbar_S, loss,
                   xbar0, vbar0, thbar, xS, vS, R=self.R, aW=aW)
        return dict(loss=loss, xbar0=xbar0, vbar0=vbar0, thbar=thbar, xS=xS, vS=vS)

    def npt(self, x, v, nsteps: int, T0, p_bar=0.0, tau_T: float = 1000.0, tau_P: float = 2500.0, chain: int = 3,
            reset: bool = False, every: int = 0, dt: float = 10.0, mass: float = 18.015,
            params: Optional[sw_params] = None, f=None):
        """Isothermal-isobaric steps (see sw_npt in include/sw.h); returns the
        forces and, if every > 0, the records [nsteps // every][R][11]
        (V, P_int bar, T, U, KE, pV, extended energy, H', P_xx, P_yy, P_zz
        bar).  tau_P <= 0: fixed box (Nose-Hoover NVT).  The box follows
        (`box`)."""
        torch = _torch()
        params = params_mw() if params is None else params
        f = torch.empty_like(x) if f is None else f
        rows = None
        if every > 0:
            rows = torch.zeros((nsteps // every, self.R, SW_NPT_WIDTH), dtype=torch.float64, device=x.device)
        sw_npt(self.handle, x, v, f, params, mass, dt, nsteps, T0, p_bar, tau_T, tau_P, chain, reset, rows, every,
               R=self.R)
        return f, rows

    @property
    def box(self):
        """Current box edges [R][3] (A); isobaric runs change them."""
        return sw_get_box(self.handle, R=self.R)

    def npt_state(self, state=None):
        return sw_npt_state(self.handle, R=self.R, state=state)

    def rdf(self, x, r_edges):
        """Ordered-pair counts per distance bin (edges in A, ascending), per
        replica: int64 tensor [R][len(r_edges) - 1] (see sw_rdf)."""
        import numpy as np
        torch = _torch()
        e = np.asarray(r_edges, dtype=np.float64) ** 2
        counts = torch.empty((self.R, len(e) - 1), dtype=torch.int64, device=x.device)
        sw_rdf(self.handle, x, e, counts, R=self.R)
        return counts

    def adf(self, x, theta_edges_deg, n_near: int = 8, r_search: Optional[float] = None):
        """Angle counts over the n_near closest neighbours (edges in degrees,
        ascending), per replica, and the number of centres skipped for lack of
        neighbours within r_search (default: the largest allowed)."""
        import numpy as np
        torch = _torch()
        c = np.cos(np.radians(np.asarray(theta_edges_deg, dtype=np.float64)))
        if r_search is None:
            r_search = self.max_search_radius()
        counts = torch.empty((self.R, len(c) - 1), dtype=torch.int64, device=x.device)
        short = sw_adf(self.handle, x, n_near, r_search, c, counts, R=self.R)
        return counts, short

    def msd(self, x, reset: bool = False):
        """Per-replica mean square displacement since the last reset (A^2)."""
        torch = _torch()
        out = torch.empty(self.R, dtype=torch.float64, device=x.device)
        sw_msd(self.handle, x, reset, out, R=self.R)
        return out

    def max_search_radius(self) -> float:
        """Smallest binning-cell edge: the largest r_max / r_search the
        observables accept."""
        return sw_query(self.handle, SW_Q_MIN_CELL_EDGE) * 1e-6

    def query(self, what: int) -> int:
        return sw_query(self.handle, what)
