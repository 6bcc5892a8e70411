"""Seeded synthetic inputs for mW boxes.

This module only *generates inputs*: lattices, density scaling, Gaussian
perturbations, Maxwell-Boltzmann velocities and the uneven replica table.  It
contains none of the Stillinger-Weber arithmetic (no energies, forces or
integration), so that both the FP64 oracle and the HIP engine can be fed the
same arrays without sharing any of the method's code.

Units throughout: Angstrom, femtosecond, kcal/mol, g/mol, Kelvin.

* Ice Ic without hydrogens is the cubic-diamond lattice (Sec. II.C,
  "Melting temperature"): an FCC lattice with a two-atom basis, 8 atoms per
  cubic cell.
* Density is rho = N M / (N_A V) with M = 18.015 g/mol (Sec. II.C, "Density,
  enthalpy ..."); a lattice is brought to a target density by isotropic
  scaling of its cubic cell.
* Velocities are drawn per Cartesian component from N(0, k_B T / m), the
  centre-of-mass velocity is removed and the set is rescaled so that
  2 KE / (N_dof k_B) equals T exactly with N_dof = 3N - 3.
"""
from __future__ import annotations

import numpy as np

# --- unit constants (input generation only) -------------------------------
M_WATER = 18.015                 # g/mol, Sec. II.C
N_AVOGADRO = 6.02214076e23       # 1/mol (SI 2019 exact)
KB = 8.314462618 / 4184.0        # kcal/(mol K): gas constant / thermochemical calorie
ACC = 4.184e-4                   # (A/fs^2) per (kcal/mol/A)/(g/mol)

SEED_CONFIG_BASE = 1000          # config k uses seed 1000 + k
SEED_REPLICA_BASE = 4000         # replica b uses seed 4000 + b


def lattice_constant_for_density(rho_gcc: float, mass: float = M_WATER) -> float:
    """Cubic-diamond lattice constant (A) giving number density for rho (g/cm^3).

    8 atoms occupy a^3, so rho = 8 M / (N_A a^3)."""
    a_cm = (8.0 * mass / (N_AVOGADRO * rho_gcc)) ** (1.0 / 3.0)
    return a_cm * 1e8


def density_gcc(n_atoms: int, box, mass: float = M_WATER) -> float:
    """rho = N M / (N_A V) in g/cm^3 for a box given in Angstrom."""
    vol_cm3 = float(np.prod(np.asarray(box, dtype=np.float64))) * 1e-24
    return n_atoms * mass / (N_AVOGADRO * vol_cm3)


def diamond_lattice(nx: int, ny: int, nz: int, a: float):
    """Cubic-diamond lattice of nx*ny*nz cubic cells with lattice constant a.

    Returns (x[N,3] float64 in [0, L), box[3] float64)."""
    fcc = np.array([[0.0, 0.0, 0.0], [0.0, 0.5, 0.5], [0.5, 0.0, 0.5], [0.5, 0.5, 0.0]])
    basis = np.concatenate([fcc, fcc + 0.25], axis=0)               # 8 sites per cell
    ii, jj, kk = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    cells = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], axis=1).astype(np.float64)
    frac = (cells[:, None, :] + basis[None, :, :]).reshape(-1, 3)
    x = frac * a
    box = np.array([nx * a, ny * a, nz * a], dtype=np.float64)
    return x, box


def wrap(x: np.ndarray, box) -> np.ndarray:
    box = np.asarray(box, dtype=np.float64)
    return x - np.floor(x / box) * box


def perturb(x: np.ndarray, box, sigma: float, rng: np.random.Generator) -> np.ndarray:
    """Gaussian displacement of every coordinate by N(0, sigma^2), then wrap."""
    return wrap(x + rng.normal(0.0, sigma, size=x.shape), box)


def maxwell_boltzmann(n: int, temperature: float, mass: float, rng: np.random.Generator) -> np.ndarray:
    """Velocities (A/fs) at exactly `temperature` with N_dof = 3N - 3."""
    kT = KB * temperature
    v = rng.normal(0.0, np.sqrt(kT * ACC / mass), size=(n, 3))
    v -= v.mean(axis=0, keepdims=True)
    ke = 0.5 * mass * float(np.sum(v * v)) / ACC
    t_now = 2.0 * ke / ((3 * n - 3) * KB)
    return v * np.sqrt(temperature / t_now)


# --- the five workloads ------------------------------------------------------

def ice_box(cells: int = 4, a: float = 6.36, sigma: float = 0.05, temperature: float = 250.0,
            seed: int = SEED_CONFIG_BASE + 0):
    """Perturbed cubic ice (cells^3 diamond cells, lattice constant a) with MB velocities."""
    rng = np.random.default_rng(seed)
    x, box = diamond_lattice(cells, cells, cells, a)
    x = perturb(x, box, sigma, rng)
    v = maxwell_boltzmann(len(x), temperature, M_WATER, rng)
    return dict(x=x, v=v, box=box, mass=M_WATER, temperature=temperature, seed=seed)


def lattice_at_density(cells, rho_gcc: float = 1.0, sigma: float = 0.0, temperature: float = 0.0,
                       seed: int = SEED_CONFIG_BASE + 1):
    """Diamond lattice of cells=(nx,ny,nz) scaled isotropically to rho (g/cm^3)."""
    if np.isscalar(cells):
        cells = (int(cells),) * 3
    rng = np.random.default_rng(seed)
    a = lattice_constant_for_density(rho_gcc)
    x, box = diamond_lattice(*cells, a)
    if sigma > 0.0:
        x = perturb(x, box, sigma, rng)
    v = maxwell_boltzmann(len(x), temperature, M_WATER, rng) if temperature > 0 else np.zeros_like(x)
    return dict(x=x, v=v, box=box, mass=M_WATER, temperature=temperature, seed=seed, rho=rho_gcc,
                lattice_constant=a)


def config(k: int):
    """Starting state of workload k (0..4).

    0: 512-atom perturbed ice at 6.36 A, 250 K, 100 NVE steps at 10 fs.
    1: 4096 atoms (8^3 cells) at 1.00 g/cm^3; melt at 400 K for 2000 steps,
       then 298 K NVE (10000 steps).
    2: 262144 atoms (32^3 cells) at 1.00 g/cm^3, same melt protocol, 1000 NVE
       steps with a 0.5 A skin.
    3: replica table (see replica_table).
    4: as 1, 200-step trajectory for the adjoint.
    The melt itself is dynamics and is done by whichever engine runs the
    workload; this function returns the lattice it starts from."""
    if k == 0:
        d = ice_box(4, 6.36, 0.05, 250.0, seed=SEED_CONFIG_BASE + 0)
        d.update(dt=10.0, nsteps=100, skin=0.5)
        return d
    if k in (1, 4):
        d = lattice_at_density(8, 1.0, sigma=0.05, temperature=400.0, seed=SEED_CONFIG_BASE + k)
        d.update(dt=10.0, melt_T=400.0, melt_steps=2000, T=298.0,
                 nsteps=10000 if k == 1 else 200, skin=1.0, ckpt_every=20)
        return d
    if k == 2:
        d = lattice_at_density(32, 1.0, sigma=0.05, temperature=400.0, seed=SEED_CONFIG_BASE + 2)
        d.update(dt=10.0, melt_T=400.0, melt_steps=2000, T=298.0, nsteps=1000, skin=0.5,
                 rebuild_every=10)
        return d
    if k == 3:
        return replica_table()
    raise ValueError(f"unknown workload {k}")


def _best_cells(n_target: float, min_cells: int = 4, max_cells: int = 16):
    """(nx <= ny <= nz), each >= min_cells, minimising |8 nx ny nz - n_target|."""
    best = None
    for nx in range(min_cells, max_cells + 1):
        for ny in range(nx, max_cells + 1):
            for nz in range(ny, max_cells + 1):
                err = abs(8 * nx * ny * nz - n_target)
                key = (err, nz - nx, nx, ny, nz)
                if best is None or key < best[0]:
                    best = (key, (nx, ny, nz))
    return best[1]


def replica_table(n_replicas: int = 64, n_min: int = 512, n_max: int = 8192,
                  rho_min: float = 0.92, rho_max: float = 1.05,
                  t_min: float = 200.0, t_max: float = 320.0, sigma: float = 0.05):
    """Uneven replicas of a density-maximum scan.

    Replica b: N* ~ U[n_min, n_max] and rho_b ~ U[rho_min, rho_max] from seed
    4000 + b; lattice cells (nx<=ny<=nz, each >= 4) closest to N*; temperature
    spaced linearly from t_min to t_max.  Returns a dict with concatenated x, v,
    CSR offsets[R+1], boxes[R,3], temperatures[R], densities[R]."""
    xs, vs, boxes, temps, rhos, offs = [], [], [], [], [], [0]
    for b in range(n_replicas):
        rng = np.random.default_rng(SEED_REPLICA_BASE + b)
        n_star = rng.uniform(n_min, n_max)
        rho = rng.uniform(rho_min, rho_max)
        cells = _best_cells(n_star)
        t_b = t_min + (t_max - t_min) * b / max(n_replicas - 1, 1)
        a = lattice_constant_for_density(rho)
        x, box = diamond_lattice(*cells, a)
        x = perturb(x, box, sigma, rng)
        v = maxwell_boltzmann(len(x), t_b, M_WATER, rng)
        xs.append(x); vs.append(v); boxes.append(box); temps.append(t_b); rhos.append(rho)
        offs.append(offs[-1] + len(x))
    return dict(x=np.concatenate(xs), v=np.concatenate(vs), offsets=np.array(offs, dtype=np.int64),
                boxes=np.array(boxes), temperatures=np.array(temps), densities=np.array(rhos),
                mass=M_WATER, dt=10.0, nsteps=5000, skin=1.0, tau=1000.0)


def slab_lattice(cells=(4, 4, 8), lxy: float = 30.0, rho_gcc: float = 1.0, lz: float = 100.0,
                 temperature: float = 400.0, seed: int = SEED_CONFIG_BASE + 5):
    """Start of the liquid-vapour slab workload (Sec. II.C: 1024 particles,
    Lx = Ly = 30 A, Lz = 100 A): a diamond lattice of `cells`, stretched to
    lxy x lxy x lz_liq at rho (to be melted in that box), and the slab box
    with the liquid centred along z.  Returns x (in the liquid box), v, the
    liquid box and the slab box."""
    nx, ny, nz = cells
    n = 8 * nx * ny * nz
    lz_liq = n * M_WATER / (N_AVOGADRO * rho_gcc * 1e-24) / (lxy * lxy)
    x, _ = diamond_lattice(nx, ny, nz, 1.0)
    liq = np.array([lxy, lxy, lz_liq])
    x = x / np.array([nx, ny, nz], dtype=np.float64) * liq
    rng = np.random.default_rng(seed)
    v = maxwell_boltzmann(n, temperature, M_WATER, rng)
    return dict(x=x, v=v, liquid_box=liq, slab_box=np.array([lxy, lxy, lz]), z_shift=0.5 * (lz - lz_liq))


def to_float4(x: np.ndarray) -> np.ndarray:
    """Pack [N,3] into the engine's [N,4] float32 layout (4th lane zero)."""
    out = np.zeros((len(x), 4), dtype=np.float32)
    out[:, :3] = x
    return out


def tile(x: np.ndarray, v: np.ndarray, box, reps, sigma: float = 0.0, seed: int = 0):
    """Periodic replication of a box reps=(rx,ry,rz) times, optionally followed
    by an N(0, sigma^2) displacement that breaks the copies' symmetry."""
    if np.isscalar(reps):
        reps = (int(reps),) * 3
    box = np.asarray(box, dtype=np.float64)
    shifts = np.array([[i, j, k] for i in range(reps[0]) for j in range(reps[1]) for k in range(reps[2])],
                      dtype=np.float64) * box
    xt = (x[None, :, :] + shifts[:, None, :]).reshape(-1, 3)
    vt = np.tile(v, (len(shifts), 1))
    big = box * np.asarray(reps, dtype=np.float64)
    if sigma > 0.0:
        xt = perturb(xt, big, sigma, np.random.default_rng(seed))
    return xt, vt, big


def load_state(path):
    """Read an (x, v, box) state written with numpy.savez (no pickles)."""
    with np.load(path, allow_pickle=False) as z:
        return np.array(z["x"]), np.array(z["v"]), np.array(z["box"])
