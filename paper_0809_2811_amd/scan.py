"""Density of the liquid against temperature at fixed pressure, on the batched
isobaric engine: one replica per temperature, Nose-Hoover thermostat and
barostat (tau_T = 1 ps, tau_P = 2.5 ps, p = 0 as in Sec. II.B), density
rho = N M / (N_A <V>) as in Sec. II.C.  The paper locates mW's density maximum
at 250 K and 1.003 g/cm^3 (Sec. III, Table 1).

    python -m paper_0809_2811_amd.scan --temps 220 230 240 250 260 270 280 300 320
"""
from __future__ import annotations

import argparse
import json
import os

import numpy as np

RC = 1.8 * 2.3925
N_A = 6.02214076e23
M_WATER = 18.015


def start_liquid(reps: int = 2):
    """The stored 298 K liquid (512 atoms, made by the oracle) tiled reps^3 times."""
    from paper_0809_2811_amd import synth
    here = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(os.path.dirname(here), "tests", "golden", "liquid512_298K.npz")
    x, v, L = synth.load_state(path)
    return synth.tile(x, v, L, reps, sigma=0.02, seed=5)


def density_scan(temperatures, reps: int = 2, p_bar: float = 0.0, equil_steps: int = 100000,
                 sample_steps: int = 400000, every: int = 100, chunk: int = 50000, dt: float = 10.0,
                 skin: float = 1.0, tau_T: float = 1000.0, tau_P: float = 2500.0, log=None):
    import torch
    from paper_0809_2811_amd import sw, synth, tune
    x0, _, L0 = start_liquid(reps)
    n = len(x0)
    R = len(temperatures)
    xs, vs = [], []
    for r, T in enumerate(temperatures):
        rng = np.random.default_rng(7000 + r)
        xs.append(x0)
        vs.append(synth.maxwell_boltzmann(n, float(T), M_WATER, rng))
    x = torch.from_numpy(synth.to_float4(np.concatenate(xs))).cuda()
    v = torch.from_numpy(synth.to_float4(np.concatenate(vs))).cuda()
    ctx = sw.Context(np.arange(R + 1) * n, [L0] * R, cutoff=RC, skin=skin, nbr_capacity=48,
                     tuning=dict(lanes_per_atom=tune.best(R * n, 1.0, skin)["lanes_per_atom"], graph_steps=50,
                                 sync_rebuild=1))   # all replicas rebuild their rows together
    T0 = [float(t) for t in temperatures]
    kw = dict(T0=T0, p_bar=p_bar, tau_T=tau_T, tau_P=tau_P, dt=dt)
    done = 0
    while done < equil_steps:
        k = min(chunk, equil_steps - done)
        ctx.npt(x, v, k, reset=done == 0, **kw)
        done += k
        if log:
            log(f"equilibrated {done} steps")
    vols = []
    done = 0
    while done < sample_steps:
        k = min(chunk, sample_steps - done)
        _, rows = ctx.npt(x, v, k, every=every, **kw)
        vols.append(rows[:, :, 0].cpu().numpy())
        done += k
        if log:
            log(f"sampled {done} steps")
    V = np.concatenate(vols)                       # [records][R]
    rho = n * M_WATER / N_A / (V * 1e-24)
    mean = rho.mean(axis=0)
    # standard error from 10 blocks
    blocks = np.array_split(rho, 10)
    err = np.std([b.mean(axis=0) for b in blocks], axis=0, ddof=1) / np.sqrt(len(blocks))
    out = dict(T=list(map(float, temperatures)), rho=mean.tolist(), err=err.tolist(), n_atoms=n,
               p_bar=p_bar, sample_ps=sample_steps * dt / 1000.0, equil_ps=equil_steps * dt / 1000.0)
    out.update(maximum(temperatures, mean))
    return out


def maximum(T, rho):
    """Temperature and density of the maximum of a cubic fit of rho(T)."""
    T = np.asarray(T, dtype=np.float64)
    rho = np.asarray(rho, dtype=np.float64)
    c = np.polyfit(T, rho, 3)
    grid = np.linspace(T.min(), T.max(), 2001)
    fit = np.polyval(c, grid)
    k = int(np.argmax(fit))
    return dict(tmd=float(grid[k]), rho_max=float(fit[k]), interior=bool(0 < k < len(grid) - 1))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--temps", type=float, nargs="+", default=[220, 230, 240, 250, 260, 270, 280, 300, 320])
    ap.add_argument("--reps", type=int, default=2, help="tiles of the 512-atom liquid per edge (2: 4096 atoms)")
    ap.add_argument("--equil", type=int, default=100000)
    ap.add_argument("--sample", type=int, default=400000)
    ap.add_argument("--p-bar", type=float, default=0.0)
    a = ap.parse_args()
    res = density_scan(a.temps, reps=a.reps, p_bar=a.p_bar, equil_steps=a.equil, sample_steps=a.sample,
                       log=lambda s: print(s, flush=True))
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
