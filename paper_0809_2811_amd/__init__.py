"""mW (Stillinger-Weber) molecular dynamics on AMD MI355X.

The compute path is libsw.so (hand-written HIP for gfx950, C ABI in
include/sw.h); ``paper_0809_2811_amd.sw`` is its ctypes binding and
``paper_0809_2811_amd.synth`` generates seeded inputs.
"""
from . import synth  # noqa: F401

__all__ = ["synth", "sw", "build"]
