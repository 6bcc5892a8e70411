"""Autotuner for the engine's launch parameters.

The search space is the sw_tuning block (include/sw.h): lanes of a wavefront
per atom (4, 8, 16), steps per captured hipGraph, persistent launch on/off,
plus the Verlet skin.  `search()` times short NVE runs of a synthetic liquid
for every candidate on the current GPU and writes the winner for the
(arch, atom-count bucket, density bucket) key to tuning_cache.json next to
this file; `best()` reads that cache (falling back to defaults).

    python -m paper_0809_2811_amd.tune --atoms 4096 262144 --replicas
"""
from __future__ import annotations

import argparse
import json
import math
import pathlib
import time

CACHE = pathlib.Path(__file__).resolve().parent / "tuning_cache.json"
DEFAULT = dict(lanes_per_atom=8, graph_steps=0, persistent=0, rebuild_every=0, timing=0)


def _arch() -> str:
    try:
        import torch
        if torch.cuda.is_available():
            return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        pass
    return "gfx950"


def bucket(n_atoms: int, rho: float) -> str:
    return f"n{int(round(math.log2(max(n_atoms, 1))))}_rho{rho:.2f}"


def load_cache() -> dict:
    if CACHE.exists():
        return json.loads(CACHE.read_text())
    return {}


def best(n_atoms: int, rho: float = 1.0, skin: float = 1.0, arch: str | None = None) -> dict:
    key = f"{arch or 'gfx950'}/{bucket(n_atoms, rho)}/skin{skin:.2f}"
    out = dict(DEFAULT)
    out.update(load_cache().get(key, {}).get("tuning", {}))
    return out


def _time_candidate(x0, v0, box, tuning, skin, steps):
    import torch
    from paper_0809_2811_amd import sw
    ctx = sw.Context([0, x0.shape[0]], [box], skin=skin, nbr_capacity=64, tuning=tuning)
    x, v = x0.clone(), v0.clone()
    ctx.step(x, v, 20)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.step(x, v, steps)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def search(n_cells: int, rho: float = 1.0, skins=(0.5, 1.0), steps: int = 400, write: bool = True):
    """Time every candidate on a 298 K liquid of 8 n_cells^3 atoms."""
    import torch
    from paper_0809_2811_amd import sw, synth
    cfg = synth.lattice_at_density(n_cells, rho, sigma=0.05, temperature=400.0, seed=7)
    box = cfg["box"]
    x = torch.from_numpy(synth.to_float4(cfg["x"])).cuda()
    v = torch.from_numpy(synth.to_float4(cfg["v"])).cuda()
    prep = sw.Context([0, x.shape[0]], [box], skin=1.0, nbr_capacity=64)
    prep.step(x, v, 1000, thermostat=sw.SW_RESCALE, T0=400.0)
    prep.step(x, v, 300, thermostat=sw.SW_RESCALE, T0=298.0)
    results = []
    for skin in skins:
        for lpa in (4, 8, 16):
            tun = dict(DEFAULT, lanes_per_atom=lpa)
            dt = _time_candidate(x, v, box, tun, skin, steps)
            results.append(dict(skin=skin, tuning=tun, s_per_step=dt))
    cache = load_cache()
    n = x.shape[0]
    for skin in skins:
        cands = [r for r in results if r["skin"] == skin]
        win = min(cands, key=lambda r: r["s_per_step"])
        cache[f"{_arch()}/{bucket(n, rho)}/skin{skin:.2f}"] = dict(
            tuning=win["tuning"], s_per_step=win["s_per_step"],
            candidates=[(r["tuning"]["lanes_per_atom"], r["s_per_step"]) for r in cands])
    if write:
        CACHE.write_text(json.dumps(cache, indent=1, sort_keys=True))
    return results


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--cells", type=int, nargs="+", default=[8, 32])
    ap.add_argument("--steps", type=int, default=400)
    a = ap.parse_args()
    for c in a.cells:
        for r in search(c, steps=a.steps):
            print(json.dumps(r), flush=True)


if __name__ == "__main__":
    main()
