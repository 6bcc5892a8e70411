"""Helpers shared by the GPU tests: seeded inputs, FP32 rounding, metrics."""
import pathlib

import numpy as np

from paper_0809_2811_amd import synth

GOLDEN = pathlib.Path(__file__).resolve().parent / "golden"
RC = 1.8 * 2.3925


def f32(x):
    """FP32-rounded copy of positions, returned as float64 for the oracle."""
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def to_dev(x3):
    import torch
    return torch.from_numpy(synth.to_float4(x3)).cuda()


def from_dev(t):
    return t.detach().cpu().numpy()[:, :3].astype(np.float64)


def liquid512():
    return synth.load_state(GOLDEN / "liquid512_298K.npz")


def liquid(reps=1, sigma=0.02, seed=5):
    """Oracle-made 298 K liquid (512 atoms) tiled reps^3 times and perturbed."""
    x, v, L = liquid512()
    if reps == 1 and sigma == 0:
        return x, v, L
    return synth.tile(x, v, L, reps, sigma=sigma, seed=seed)


def force_error(F_gpu, F_ora):
    """max_i |F_gpu - F_ora| / RMS_i |F_ora|."""
    rms = np.sqrt((F_ora ** 2).sum(axis=1).mean())
    return np.abs(F_gpu - F_ora).max() / rms


def oracle_virial6(o):
    W = o["W2"] + o["W3"]
    return np.array([W[0, 0], W[1, 1], W[2, 2], W[0, 1], W[0, 2], W[1, 2]])
