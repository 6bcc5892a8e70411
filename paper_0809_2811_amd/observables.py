"""Estimators of Sec. II.C of the mW paper from the engine's histograms.

The device calls (`Context.rdf`, `Context.adf`, `Context.msd`) return exact
counts and per-replica mean square displacements; these functions turn them
into the quantities the paper reports:

  g(r)      = V / N^2 < sum_i sum_{j != i} delta(r - r_ij) >   (histogram form)
  n_c(R_c)  = 4 pi N/V int_0^{R_c} r^2 g(r) dr  = ordered pairs within R_c / N
  P(theta)  = 1/(N n_theta) < sum_k sum_{i<j in the n_c closest} delta(theta - theta_ikj) >
  D         = lim_{t -> inf} <|r(t) - r(0)|^2> / (6 t)   (Einstein relation)
  gamma_lv  = L_z / 2 [<p_N> - <p_T>]   (slab with interfaces normal to z)
"""
from __future__ import annotations

import numpy as np


def g_of_r(counts, r_edges, n_atoms: int, volume: float, frames: int = 1):
    """Pair distribution at the bin centres from ordered-pair counts summed
    over `frames` frames."""
    r = np.asarray(r_edges, dtype=np.float64)
    shell = 4.0 / 3.0 * np.pi * (r[1:] ** 3 - r[:-1] ** 3)
    g = np.asarray(counts, dtype=np.float64) * volume / (float(n_atoms) ** 2 * shell * frames)
    return 0.5 * (r[1:] + r[:-1]), g


def coordination(counts, r_edges, n_atoms: int, r_c: float, frames: int = 1) -> float:
    """Mean number of neighbours within r_c (r_c must be one of the edges)."""
    r = np.asarray(r_edges, dtype=np.float64)
    k = int(np.argmin(np.abs(r - r_c)))
    if abs(r[k] - r_c) > 1e-9 * max(1.0, r_c):
        raise ValueError("r_c must be a bin edge")
    return float(np.asarray(counts, dtype=np.float64)[:k].sum()) / (n_atoms * frames)


def angle_distribution(counts, theta_edges_deg):
    """P(theta) at the bin centres, normalised to unit integral over degrees."""
    th = np.asarray(theta_edges_deg, dtype=np.float64)
    c = np.asarray(counts, dtype=np.float64)
    total = c.sum()
    p = c / (total * np.diff(th)) if total > 0 else np.zeros_like(c)
    return 0.5 * (th[1:] + th[:-1]), p


def diffusion_coefficient(t_fs, msd_A2, t_min_fs: float = 0.0) -> float:
    """D in cm^2/s from a least-squares line through MSD(t) for t >= t_min
    (A^2/fs -> cm^2/s: 1e-16 / 1e-15 = 0.1)."""
    t = np.asarray(t_fs, dtype=np.float64)
    m = np.asarray(msd_A2, dtype=np.float64)
    sel = t >= t_min_fs
    slope = np.polyfit(t[sel], m[sel], 1)[0]
    return slope / 6.0 * 0.1


def surface_tension(p_xx, p_yy, p_zz, lz: float) -> float:
    """Liquid-vapour surface tension in mN/m (= mJ/m^2) of a slab with its two
    interfaces normal to z, from pressure-tensor samples in bar and the box
    length L_z in A: gamma = L_z/2 [<p_zz> - (<p_xx> + <p_yy>)/2]
    (1 bar A = 1e-5 N/m)."""
    pn = float(np.mean(p_zz))
    pt = 0.5 * (float(np.mean(p_xx)) + float(np.mean(p_yy)))
    return 0.5 * lz * (pn - pt) * 1e-2
