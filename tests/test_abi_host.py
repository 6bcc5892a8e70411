"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every entry point include/sw.h declares, and rejects bad arguments before it
touches the device."""
import ctypes
import pathlib
import re

import numpy as np
import pytest

from paper_0809_2811_amd import sw

ROOT = pathlib.Path(__file__).resolve().parents[1]


def declared_functions():
    text = (ROOT / "include" / "sw.h").read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sw_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = sw.lib()
    names = declared_functions()
    assert len(names) >= 12
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(sw.EXPORTS)


def test_status_strings():
    for code in range(0, -12, -1):
        s = sw.status_string(code)
        assert s and s != "unknown status"
    assert sw.status_string(-99) == "unknown status"


def test_default_parameters_are_the_papers():
    from tests.test_oracle_pins import paper_values
    pv = paper_values()
    p = sw.params_mw()
    assert p.lambda_ == pv["lambda"] and p.epsilon == pv["epsilon_kcal_mol"] and p.sigma == pv["sigma_A"]
    assert p.A == pv["A"] and p.B == pv["B"] and p.p == pv["p"] and p.q == pv["q"]
    assert p.gamma == pv["gamma"] and p.a == pv["a"] and p.cos_theta0 == -1.0 / 3.0


def _create(offsets, boxes, cutoff=4.3065, skin=0.5, cap=32):
    L = sw.lib()
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    box = np.ascontiguousarray(boxes, dtype=np.float64).reshape(-1)
    h = ctypes.c_void_p()
    return L.sw_create(ctypes.byref(h), len(off) - 1, off.ctypes.data_as(ctypes.POINTER(ctypes.c_longlong)),
                       box.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), cutoff, skin, cap)


@pytest.mark.parametrize("offsets,boxes,cutoff,skin,cap,code", [
    ([0, 512], [[25.0, 25.0, 25.0]], 4.3065, -0.1, 32, sw.SW_EINVAL),        # negative skin
    ([0, 512], [[25.0, 25.0, 25.0]], 0.0, 0.5, 32, sw.SW_EINVAL),            # zero cut-off
    ([0, 512], [[25.0, 25.0, 25.0]], 4.3065, 0.5, 0, sw.SW_EINVAL),          # zero capacity
    ([0, 512], [[25.0, 25.0, 25.0]], 4.3065, 0.5, 4096, sw.SW_EINVAL),       # capacity too large
    ([1, 512], [[25.0, 25.0, 25.0]], 4.3065, 0.5, 32, sw.SW_EINVAL),         # offsets[0] != 0
    ([0, 512, 513], [[25.0] * 3, [25.0] * 3], 4.3065, 0.5, 32, sw.SW_EINVAL),  # 1-atom replica
    ([0, 512], [[25.0, -1.0, 25.0]], 4.3065, 0.5, 32, sw.SW_EINVAL),         # negative edge
    ([0, 512], [[25.0, 14.0, 25.0]], 4.3065, 0.5, 32, sw.SW_EBOX_TOO_SMALL),  # 14 A < 3 * 4.8065
    ([0, 64], [[12.4, 12.4, 12.4]], 4.3065, 0.0, 32, sw.SW_EBOX_TOO_SMALL),   # 2 cells only
])
def test_create_rejects_before_touching_the_device(offsets, boxes, cutoff, skin, cap, code):
    assert _create(offsets, boxes, cutoff, skin, cap) == code


def test_null_arguments_rejected():
    L = sw.lib()
    assert L.sw_create(None, 1, None, None, 4.3, 0.5, 32) == sw.SW_EINVAL
    assert L.sw_forces(None, None, None, None, None, None, None) == sw.SW_EINVAL
    assert L.sw_step(None, None, None, None, None, 18.0, 10.0, 1, 0, None, 1.0, None, 1, None) == sw.SW_EINVAL
    assert L.sw_query(None, 0, None) == sw.SW_EINVAL
    L.sw_destroy(None)


def _struct_fields(name):
    """(type, field) pairs of `typedef struct name { ... } name;` in include/sw.h."""
    text = (ROOT / "include" / "sw.h").read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    body = re.search(r"typedef struct %s\s*\{(.*?)\}\s*%s;" % (name, name), text, flags=re.S).group(1)
    out = []
    for ct, names in re.findall(r"\b(int|double|float|long long)\s+([\w\s,]+);", body):
        out += [(ct, n.strip()) for n in names.split(",")]
    return out


@pytest.mark.parametrize("name", ["sw_params", "sw_tuning"])
def test_binding_structs_match_the_header(name):
    """The ctypes mirrors of the ABI's structs have the header's fields, in
    order, with the same C types and size."""
    ctype = {"int": ctypes.c_int, "double": ctypes.c_double, "float": ctypes.c_float,
             "long long": ctypes.c_longlong}
    header = _struct_fields(name)
    py = getattr(sw, name)._fields_
    assert len(header) == len(py) and len(header) > 0
    for (ct, fname), (pname, ptype) in zip(header, py):
        assert ptype is ctype[ct], (fname, ct, ptype)
        assert pname.rstrip("_") == fname, (fname, pname)
    assert ctypes.sizeof(getattr(sw, name)) == sum(ctypes.sizeof(ctype[t]) for t, _ in header)
