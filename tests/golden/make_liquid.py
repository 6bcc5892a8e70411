"""Write tests/golden/liquid512_298K.npz using only the FP64 oracle.

Recipe: 4x4x4 diamond cells scaled to 1.00 g/cm^3 (512 atoms, seed 1001,
0.05 A Gaussian perturbation, Maxwell-Boltzmann at 400 K), 2000 velocity-Verlet
steps of 10 fs with velocity rescaling to 400 K (melt), then 500 steps with
rescaling to 298 K.  The stored x, v (float64) are a 298 K mW liquid used as a
seeded input by the parity tests and, tiled, for larger liquid boxes.

Run:  python tests/golden/make_liquid.py
"""
import pathlib
import sys

import numpy as np

ROOT = pathlib.Path(__file__).resolve().parents[2]
sys.path.insert(0, str(ROOT))

import oracle  # noqa: E402
from paper_0809_2811_amd import synth  # noqa: E402


def main():
    d = synth.lattice_at_density(4, 1.0, sigma=0.05, temperature=400.0, seed=1001)
    x, v, L = d["x"], d["v"], d["box"]
    x, v, _, _ = oracle.vv(x, v, L, 2000, dt=10.0, thermostat=1, T0=400.0)
    x, v, _, th = oracle.vv(x, v, L, 500, dt=10.0, thermostat=1, T0=298.0)
    out = pathlib.Path(__file__).resolve().parent / "liquid512_298K.npz"
    np.savez(out, x=x, v=v, box=L)
    print(out, "PE/N", (th[-1, 0] + th[-1, 1]) / len(x))


if __name__ == "__main__":
    main()
