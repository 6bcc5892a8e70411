"""Throughput benchmark of the mW Stillinger-Weber engine on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--forms liquid4096,share,batched,adjoint,observables,npt|none]

Main line: the large single box - 262144 mW atoms (32^3 diamond cells scaled
to 1.00 g/cm^3), melted for 2000 velocity-Verlet steps (10 fs) with
velocities rescaled to 400 K, then 500 steps rescaled to 298 K (untimed),
then W untimed and K timed NVE steps with a 0.5 A skin, rows rebuilt at least
every 10 steps and whenever the displacement check fires.  A "step" is one
full velocity-Verlet step of the whole path (row rebuilds when due, moments,
forces, integration, binning; thermo sums every 100 steps when K >= 100).
Inputs are resident in HBM before the timed region starts; the timed region
is one sw_step call of exactly K steps.

Prints one JSON line.  Kernel durations come from HIP events recorded by the
library at the dispatch of sampled launches inside the timed region.

Roofline (per atom-step of the 298 K liquid, counts of the force path's
algorithm as stated for this workload): 3.5-5 kflop (midpoint 4.25 kflop)
and ~100 bytes.  The force path is FP32 VALU work (no dense contraction),
so the bound is the FP32 vector peak, 157.3 TFLOP/s; the bytes are reported
against 8 TB/s beside it.  The kernel unit is one step's force path: the
moments launch and the force launch together (one of each per step).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "atom-steps/s (mW SW force+step) plain vs batched; adjoint cost per step; % roofline"
RC = 1.8 * 2.3925
PEAK_FP32 = 157.3e12        # MI355X FP32 vector peak (256 CU x 128 FP32 lanes x 2 (FMA) x 2.4 GHz)
PEAK_FP32_NONPACKED = 78.6e12   # the same without packed FP32 issue (this build emits none)
PEAK_HBM = 8.0e12
ALG_FLOP_PER_ATOM_STEP = 4.25e3       # midpoint of 3.5-5 kflop per atom-step (liquid)
ALG_FLOP_RANGE = (3.5e3, 5.0e3)
ALG_BYTES_PER_ATOM_STEP = 100.0
LARGE_STEPS = 1000                     # the large box workload's own length
CPU_SHARE = 16                         # host cores available to one GPU's job


def sync():
    import torch
    torch.cuda.synchronize()


# ------------------------------------------------------------------ CPU leg
def _oracle_run(args):
    """One oracle process: `steps` FP64 NVE steps of the tiled liquid."""
    seed, steps = args
    os.environ["OMP_NUM_THREADS"] = "1"
    import oracle
    from paper_0809_2811_amd import synth
    x, v, L = synth.load_state(os.path.join(ROOT, "tests", "golden", "liquid512_298K.npz"))
    x, v, L = synth.tile(x, v, L, 8, sigma=0.02, seed=seed)
    t0 = time.perf_counter()
    oracle.vv(x, v, L, steps, dt=10.0)
    return len(x), steps, time.perf_counter() - t0


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(steps=12):
    """The FP64 oracle (as it stands, one thread per process) on the large
    box's size and state: the oracle-made 512-atom 298 K liquid tiled 8x8x8
    (262144 atoms, 198.674 A) and perturbed by 0.02 A.  One process alone
    gives the single-core rate; then one process per available core (at most
    the GPU's 16-core share), each on its own perturbed copy, run together,
    gives the all-core rate (total atom-steps over the wall time of the
    batch).  Each process times its whole call: the initial force
    evaluation plus `steps` steps.  Runs before the GPU is touched, so the
    worker processes fork from a process without a HIP context."""
    import multiprocessing as mp
    n, k, t1 = _oracle_run((5, steps))
    single = n * k / t1
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    cores = max(1, min(CPU_SHARE, avail))
    ctxm = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctxm.Pool(cores) as pool:
        res = pool.map(_oracle_run, [(100 + w, steps) for w in range(cores)])
    wall = time.perf_counter() - t0
    total = sum(a * b for a, b, _ in res)
    return {"value": total / wall, "unit": "atom-steps/s", "cores": cores, "kind": "oracle",
            "single_thread_value": single, "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
            "sample": f"262144-atom 298 K liquid (oracle-made 512-atom liquid tiled 8x8x8, +0.02 A noise), FP64 NVE "
                      f"velocity Verlet at 10 fs, {steps} steps per process (each call also evaluates the initial "
                      f"forces, counted as overhead); {cores} processes on their own copies together: "
                      f"{wall:.1f} s wall; one process alone: {t1:.1f} s"}


# ------------------------------------------------------------------ GPU helpers
def prepare_liquid(cfg, skin, tuning):
    """Lattice -> melt at 400 K (2000 steps) -> 298 K (500 steps) on the GPU."""
    import torch
    from paper_0809_2811_amd import sw, synth
    ctx = sw.Context([0, len(cfg["x"])], [cfg["box"]], cutoff=RC, skin=skin, nbr_capacity=48, tuning=tuning)
    x = torch.from_numpy(synth.to_float4(cfg["x"])).cuda()
    v = torch.from_numpy(synth.to_float4(cfg["v"])).cuda()
    ctx.step(x, v, cfg["melt_steps"], thermostat=sw.SW_RESCALE, T0=cfg["melt_T"])
    ctx.step(x, v, 500, thermostat=sw.SW_RESCALE, T0=cfg["T"])
    return ctx, x, v


def lcm(a, b):
    import math
    return a // math.gcd(a, b) * b


def clamped_block(ctx, steps, thermo_every=100):
    """Captured-block length for a call of `steps` steps: the tuned length,
    clamped so that at least one block fits (0 if none can)."""
    te = thermo_every if steps >= thermo_every else 0
    tun = ctx.tuning()
    g = tun.get("graph_steps", 0)
    period = lcm(2, te) if te else 2
    if tun.get("rebuild_every", 0) > 0:
        period = lcm(period, tun["rebuild_every"])
    if g > 0:
        kmax = ((steps - 1) // period) * period
        g = min(g, kmax) if kmax > 0 else 0
    return g, te, period


def capture_for(ctx, x, v, steps, thermo_every=100):
    """Setup before the warmup: one untimed NVE call long enough to capture
    the graph block the timed call will replay (capture and instantiation
    happen once per configuration, like compilation), so the timed call only
    replays it."""
    g, te, period = clamped_block(ctx, steps, thermo_every)
    if g > 0:
        tun = ctx.tuning()
        ctx.set_tuning(graph_steps=g)
        n = -(-g // period) * period + 1          # the library rounds the block up to the period
        ctx.step(x, v, n, thermo_every=te)
        ctx.set_tuning(graph_steps=tun.get("graph_steps", 0))


def timed_nve(ctx, x, v, steps, thermo_every=100):
    """One timed NVE call of exactly `steps` steps.  Captured blocks (when the
    tuning asks for them) are clamped so that at least one fits in the call;
    the steps after the last block run as stream launches, and every one of
    them has its moments and force launches bracketed by HIP events (all
    steps are sampled with plain launches: an odd period, so both parities)."""
    from paper_0809_2811_amd import sw
    g, te, _ = clamped_block(ctx, steps, thermo_every)
    tun = ctx.tuning()
    ctx.set_tuning(graph_steps=g, timing=1 if g > 0 else 7)
    r0 = ctx.query(sw.SW_Q_REBUILDS)
    sync()
    t0 = time.perf_counter()
    f, th = ctx.step(x, v, steps, thermo_every=te)
    sync()
    dt = time.perf_counter() - t0
    out = dict(seconds=dt, rebuilds=ctx.query(sw.SW_Q_REBUILDS) - r0, graph_steps=g)
    ns = ctx.query(sw.SW_Q_TIMED_STEPS)
    if ns > 0:
        out["forces_us"] = ctx.query(sw.SW_Q_TIME_FORCES_NS) / ns / 1e3
        out["moments_us"] = ctx.query(sw.SW_Q_TIME_MOMENTS_NS) / ns / 1e3
        out["timed_launches"] = ns
    if th is not None:
        e = (th[:, 0, 0] + th[:, 0, 1] + th[:, 0, 2]).cpu().numpy()
        out["etot_first_last"] = [float(e[0]), float(e[-1])]
    ctx.set_tuning(timing=0, graph_steps=tun.get("graph_steps", 0))
    return out


def measured_traffic(kernel, workload):
    from paper_0809_2811_amd import hbm_counters
    return hbm_counters.measured_traffic(kernel, workload)


def step_roofline(n_atoms, res, lpa, workload):
    """Roofline of one step's force path (moments + force launch) from the
    algorithmic counts per atom-step; implementation details beside it."""
    mk, fk = f"k_moments<{lpa}, false>", f"k_forces<{lpa}, 2, false>"
    us = res["moments_us"] + res["forces_us"]
    sec = us * 1e-6
    flop = n_atoms * ALG_FLOP_PER_ATOM_STEP
    byt = n_atoms * ALG_BYTES_PER_ATOM_STEP
    tm, tf = measured_traffic(mk, workload), measured_traffic(fk, workload)
    return {
        "bound": "alu", "achieved": flop / sec / 1e12, "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s",
        "frac": flop / sec / PEAK_FP32, "traffic": (tm + tf) if tm is not None and tf is not None else None,
        "kernel": f"{mk} + {fk} (one step's force path)", "kernel_us": us,
        "moments_us": res["moments_us"], "forces_us": res["forces_us"], "timed_steps": res.get("timed_launches"),
        "alg_flop_per_launch": flop, "alg_bytes_per_launch": byt,
        "frac_range": [n_atoms * ALG_FLOP_RANGE[0] / sec / PEAK_FP32, n_atoms * ALG_FLOP_RANGE[1] / sec / PEAK_FP32],
        "frac_vs_nonpacked_fp32": flop / sec / PEAK_FP32_NONPACKED,
        "hbm_frac": byt / sec / PEAK_HBM,
        "traffic_by_kernel": {mk: tm, fk: tf},
    }


def wall_roofline(atom_steps_per_s, force_paths_per_step=1.0):
    """Roofline fraction of a whole form from its wall-clock rate (all of its
    launches, not one kernel), with the same counts per atom-step."""
    fl = atom_steps_per_s * ALG_FLOP_PER_ATOM_STEP * force_paths_per_step
    return {"bound": "alu", "achieved": fl / 1e12, "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s",
            "frac": fl / PEAK_FP32, "basis": "wall clock of the whole form",
            "force_paths_per_step": force_paths_per_step,
            "hbm_frac": atom_steps_per_s * ALG_BYTES_PER_ATOM_STEP * force_paths_per_step / PEAK_HBM}


def launch_floor_us(n=200, reps=5):
    """What one launch costs on this GPU with almost no work in it: a plain
    elementwise add over 131072 floats, n launches captured in a graph and
    replayed; microseconds per launch."""
    import torch
    t = torch.zeros(1 << 17, device="cuda")
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        for _ in range(3):
            t.add_(1.0)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=st):
        for _ in range(n):
            t.add_(1.0)
    g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        g.replay()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / (reps * n) * 1e6


# ------------------------------------------------------------------ forms
def bench_large(steps, warmup, skin=0.5, graph_steps=-1, lpa=0):
    """The main line (see the module docstring)."""
    from paper_0809_2811_amd import synth, tune
    cfg = synth.config(2)
    n = len(cfg["x"])
    tuning = tune.best(n, 1.0, skin)
    tuning.pop("skin", None)
    tuning["rebuild_every"] = 10
    if graph_steps >= 0:
        tuning["graph_steps"] = graph_steps
    if lpa:
        tuning["lanes_per_atom"] = lpa
    ctx, x, v = prepare_liquid(cfg, skin, tuning)
    try:
        capture_for(ctx, x, v, steps)
        if warmup > 0:
            ctx.step(x, v, warmup)
        res = timed_nve(ctx, x, v, steps)
        audit = missed_pair_audit(ctx, x, v)
    finally:
        ctx.close()
    out = {"n_atoms": n, "skin_A": skin, "rebuilds": res["rebuilds"], "seconds": res["seconds"], "audit": audit,
           "tuning": dict(tuning, graph_steps=res["graph_steps"]),
           "workload": "large_box262144_nve: 262144 mW atoms (32^3 diamond cells at 1.00 g/cm^3), melted 2000 steps "
                       "at 400 K + 500 steps at 298 K, NVE velocity Verlet dt=10 fs, 0.5 A skin, rows rebuilt at "
                       "least every 10 steps and on the displacement check"}
    if "forces_us" in res:
        out["roofline"] = step_roofline(n, res, tuning["lanes_per_atom"], "liquid262144")
    return out


def missed_pair_audit(ctx, x, v, steps=200):
    """After the timed region: `steps` more steps of the same run in the same
    launch form, with the rows in use audited after every step's moments
    launch against a fresh search of the cells (untimed).  `missed` counts
    pairs inside a*sigma absent from their row and must be 0."""
    from paper_0809_2811_amd import sw
    tun = ctx.tuning()
    p0, m0, r0 = (ctx.query(q) for q in (sw.SW_Q_AUDIT_PAIRS, sw.SW_Q_MISSED_PAIRS, sw.SW_Q_REBUILDS))
    ctx.set_tuning(audit_every=1)
    ctx.step(x, v, steps)
    out = {"steps": steps, "audits": steps, "pairs_checked": ctx.query(sw.SW_Q_AUDIT_PAIRS) - p0,
           "missed": ctx.query(sw.SW_Q_MISSED_PAIRS) - m0, "rebuilds": ctx.query(sw.SW_Q_REBUILDS) - r0}
    ctx.set_tuning(audit_every=tun.get("audit_every", 0))
    return out


def bench_liquid4096(steps=1000, warmup=100):
    """The 4096-atom liquid (8^3 cells at 1.00 g/cm^3, melted like the main
    line), tuned launch (captured blocks), `steps` timed NVE steps."""
    from paper_0809_2811_amd import synth, tune
    cfg = synth.config(1)
    n = len(cfg["x"])
    tuning = tune.best(n, 1.0, None)
    skin = tuning.pop("skin", 1.0)
    ctx, x, v = prepare_liquid(cfg, skin, tuning)
    try:
        capture_for(ctx, x, v, steps)
        ctx.step(x, v, warmup)
        res = timed_nve(ctx, x, v, steps)
    finally:
        ctx.close()
    out = {"value": n * steps / res["seconds"], "unit": "atom-steps/s", "steps": steps,
           "ms_per_step": res["seconds"] * 1e3 / steps, "n_atoms": n, "skin_A": skin, "rebuilds": res["rebuilds"],
           "tuning": dict(tuning, graph_steps=res["graph_steps"]),
           "workload": "liquid4096_nve: 4096 mW atoms (8^3 diamond cells at 1.00 g/cm^3), melted 2000 steps at "
                       "400 K + 500 steps at 298 K, NVE velocity Verlet dt=10 fs"}
    if "forces_us" in res:
        out["roofline"] = step_roofline(n, res, tuning["lanes_per_atom"], "liquid4096")
    out["roofline_wall"] = wall_roofline(out["value"])
    return out


def bench_share(steps=1000, skin=0.5):
    """One GPU's owned share of the large box decomposed over 8 GPUs (2x2x2
    bricks): 32768 atoms (16^3 cells at 1.00 g/cm^3), the large box's
    protocol.  A periodic box stands in for the brick; its ghost shell (~10k
    atoms) and the halo exchanges are not modelled."""
    from paper_0809_2811_amd import synth, tune
    cfg = synth.lattice_at_density(16, 1.0, sigma=0.05, temperature=400.0, seed=synth.SEED_CONFIG_BASE + 2)
    cfg.update(melt_T=400.0, melt_steps=2000, T=298.0)
    n = len(cfg["x"])
    tuning = tune.best(n, 1.0, skin)
    tuning.pop("skin", None)
    tuning["rebuild_every"] = 10
    ctx, x, v = prepare_liquid(cfg, skin, tuning)
    try:
        capture_for(ctx, x, v, steps)
        ctx.step(x, v, 50)
        res = timed_nve(ctx, x, v, steps)
    finally:
        ctx.close()
    val = n * steps / res["seconds"]
    return {"value": val, "unit": "atom-steps/s", "steps": steps,
            "ms_per_step": res["seconds"] * 1e3 / steps, "n_atoms": n, "skin_A": skin,
            "rebuilds": res["rebuilds"], "tuning": dict(tuning, graph_steps=res["graph_steps"]),
            "roofline_wall": wall_roofline(val),
            "workload": "share: 32768 atoms (one GPU's owned brick of the 262144-atom box on 8 GPUs, as a periodic "
                        "box), 298 K liquid, NVE dt=10 fs, 0.5 A skin, rows rebuilt at least every 10 steps"}


def bench_batched(steps=5000, melt_steps=1000, skin=1.0, sequential_steps=500):
    """64 uneven replicas (512-8192 atoms, 0.92-1.05 g/cm^3, 200-320 K) in one
    context: melted together at 400 K (rescale, untimed), then `steps`
    Berendsen steps (tau 1 ps) at each replica's temperature, thermo every
    100 steps; timed per launch form.  For comparison, the replicas one
    after another through single-replica contexts (plain engine)."""
    import torch
    from paper_0809_2811_amd import sw, synth, tune
    tab = synth.replica_table()
    off, boxes, T = tab["offsets"], tab["boxes"], tab["temperatures"]
    n = int(off[-1])
    base = tune.best(n, 1.0, skin, replicas=True)
    base.pop("skin", None)
    base["persistent"] = 0
    x0 = torch.from_numpy(synth.to_float4(tab["x"])).cuda()
    v0 = torch.from_numpy(synth.to_float4(tab["v"])).cuda()
    out = {"workload": f"batched: {len(boxes)} replicas, {n} atoms total (512-8192 each, 0.92-1.05 g/cm^3), "
                       f"melted {melt_steps} steps at 400 K, then Berendsen (tau 1 ps) at 200-320 K, dt=10 fs",
           "n_atoms": n, "n_replicas": len(boxes), "steps": steps, "unit": "atom-steps/s", "skin_A": skin,
           "tuning": dict(base)}
    forms = (("per_phase", dict(persistent=0, graph_steps=0)),
             ("per_phase_graph", dict(persistent=0, graph_steps=100)),
             ("persistent", dict(persistent=1, graph_steps=0)),
             ("persistent_graph", dict(persistent=1, graph_steps=100)))
    with sw.Context(off, boxes, cutoff=RC, skin=skin, nbr_capacity=48, tuning=base) as ctx:
        ctx.step(x0, v0, melt_steps, thermostat=sw.SW_RESCALE, T0=[400.0] * len(boxes))
        for name, form in forms:
            ctx.set_tuning(**form)
            x, v = x0.clone(), v0.clone()
            # a captured persistent call is keyed by its step count: warm up
            # with the timed count so that the timed call replays it
            warm = steps if form["persistent"] and form["graph_steps"] else 200
            ctx.step(x, v, warm, thermostat=sw.SW_BERENDSEN, T0=T, tau_fs=1000.0, thermo_every=100)
            sync()
            t0 = time.perf_counter()
            ctx.step(x, v, steps, thermostat=sw.SW_BERENDSEN, T0=T, tau_fs=1000.0, thermo_every=100)
            sync()
            dt = time.perf_counter() - t0
            out[name] = {"value": n * steps / dt, "ms_per_step": dt * 1e3 / steps, **form}
            if form["persistent"]:   # 1: grid-wide barriers; k > 1: replicas dealt to k XCCs
                out[name]["barrier_groups"] = ctx.query(sw.SW_Q_PERSISTENT_GROUPS)
    # the same replicas one after another, each in its own context
    xs, vs = x0.clone(), v0.clone()
    total = 0.0
    for r in range(len(boxes)):
        a, b = int(off[r]), int(off[r + 1])
        t1 = tune.best(b - a, 1.0, skin)
        t1.pop("skin", None)
        with sw.Context([0, b - a], [boxes[r]], cutoff=RC, skin=skin, nbr_capacity=48, tuning=t1) as c1:
            xr, vr = xs[a:b].contiguous(), vs[a:b].contiguous()
            c1.step(xr, vr, 20, thermostat=sw.SW_BERENDSEN, T0=[T[r]], tau_fs=1000.0)
            sync()
            t0 = time.perf_counter()
            c1.step(xr, vr, sequential_steps, thermostat=sw.SW_BERENDSEN, T0=[T[r]], tau_fs=1000.0)
            sync()
            total += time.perf_counter() - t0
    out["one_at_a_time"] = {"value": n * sequential_steps / total, "ms_per_step": total * 1e3 / sequential_steps,
                            "steps": sequential_steps}
    best = max((k for k, _ in forms), key=lambda k: out[k]["value"])
    out["best_form"] = best
    out["value"] = out[best]["value"]
    out["speedup_vs_one_at_a_time"] = out["value"] / out["one_at_a_time"]["value"]
    out["roofline_wall"] = wall_roofline(out["value"])
    return out


def bench_adjoint(plain4096, steps=200, ckpt=20):
    """Differentiable trajectory: 4096-atom 298 K liquid (same preparation as
    the 4096-atom form), 200 NVE steps, checkpoints every 20; one call
    computes the loss, dL/dx0, dL/dv0 and dL/d(lambda, eps, sigma).  The
    ratio is taken against the plain 4096-atom step in the same launch form
    (captured graphs; `plain4096` is that form's result)."""
    from paper_0809_2811_amd import synth, tune
    cfg = synth.config(4)
    n = len(cfg["x"])
    tuning = tune.best(n, 1.0, None)
    skin = tuning.pop("skin", 1.0)
    ctx, x, v = prepare_liquid(cfg, skin, tuning)
    reps = 3
    try:
        ctx.adjoint(x, v, steps, ckpt_every=ckpt)   # untimed: captures the call's launch graph (graph mode)
        sync()
        t0 = time.perf_counter()
        for _ in range(reps):
            res = ctx.adjoint(x, v, steps, ckpt_every=ckpt)
        sync()
        dt = (time.perf_counter() - t0) / reps
        th = res["thbar"].cpu().numpy()[0]
        # every frame kept (one segment: the reverse sweep recomputes nothing)
        ctx.adjoint(x, v, steps, ckpt_every=steps)
        sync()
        t0 = time.perf_counter()
        for _ in range(reps):
            res_all = ctx.adjoint(x, v, steps, ckpt_every=steps)
        sync()
        dt_all = (time.perf_counter() - t0) / reps
        same = all(bool(torch_equal(res[k], res_all[k])) for k in ("loss", "thbar", "xbar0", "vbar0"))
    finally:
        ctx.close()
    ms, ms_all = dt * 1e3 / steps, dt_all * 1e3 / steps
    plain_ms = plain4096["ms_per_step"]
    # force-path equivalents per trajectory step: forward, recompute (with
    # checkpoints), and a tangent pass counted as 2.5 force evaluations
    return {"workload": f"adjoint: {n}-atom 298 K liquid, {steps}-step NVE trajectory, checkpoints every {ckpt}, "
                        "loss = mean PE/atom + mean three-body energy/atom",
            "seconds_per_trajectory": dt, "ms_per_step": ms, "value": n * steps / dt, "unit": "atom-steps/s",
            "plain_step_same_form_ms": plain_ms, "plain_launch_form": plain4096["tuning"],
            "ratio_to_plain_step": ms / plain_ms, "loss": float(res["loss"].cpu()[0]),
            "dL_dtheta": [float(t) for t in th],
            "roofline_wall": wall_roofline(n * steps / dt, 4.5),
            "all_frames_stored": {"ckpt_every": steps, "ms_per_step": ms_all, "value": n * steps / dt_all,
                                  "ratio_to_plain_step": ms_all / plain_ms, "bitwise_equal_to_checkpointed": same,
                                  "roofline_wall": wall_roofline(n * steps / dt_all, 3.5)}}


def torch_equal(a, b):
    import torch
    return torch.equal(a, b)


def bench_observables(reps=20):
    """One sampling frame of the Sec. II.C estimators on the 4096-atom
    liquid: pair-distance histogram to the largest radius the cells allow
    (0.02 A bins), angle histogram over the 8 closest neighbours (1 degree
    bins), and the mean square displacement update; each call sorts and
    bins the positions itself."""
    from paper_0809_2811_amd import synth, tune
    cfg = synth.config(1)
    tuning = tune.best(len(cfg["x"]), 1.0, None)
    skin = tuning.pop("skin", 1.0)
    ctx, x, v = prepare_liquid(cfg, skin, tuning)
    try:
        rmax = ctx.max_search_radius()
        r_edges = np.arange(0.0, rmax, 0.02)
        th = np.arange(0.0, 180.01, 1.0)
        out = {"workload": f"observables: {x.shape[0]}-atom 298 K liquid, g(r) to {rmax:.2f} A, P(theta) over 8 "
                           "closest neighbours, MSD update", "n_atoms": int(x.shape[0])}
        ctx.msd(x, reset=True)
        for name, fn in (("rdf", lambda: ctx.rdf(x, r_edges)), ("adf", lambda: ctx.adf(x, th, n_near=8)),
                         ("msd", lambda: ctx.msd(x))):
            fn()
            sync()
            t0 = time.perf_counter()
            for _ in range(reps):
                fn()
            sync()
            out[f"{name}_ms"] = (time.perf_counter() - t0) * 1e3 / reps
    finally:
        ctx.close()
    return out


def bench_npt(plain4096, steps=5000, warm=1000):
    """Isothermal-isobaric steps (Nose-Hoover chains of 3, tau_T 1 ps,
    tau_P 2.5 ps, p = 0): the 4096-atom liquid alone, and nine replicas of it
    at 220-320 K in one context (the density-maximum scan)."""
    import torch
    from paper_0809_2811_amd import scan, sw, synth, tune
    x0, v0, L0 = scan.start_liquid(2)
    n = len(x0)
    out = {"workload": f"npt: {n}-atom liquid at 298 K and p = 0; and 9 replicas of it at 220-320 K "
                       "(rows of all replicas rebuilt together when any replica's check fires)",
           "unit": "atom-steps/s"}
    for name, temps in (("single", [298.0]), ("batched", [220, 230, 240, 250, 260, 270, 280, 300, 320])):
        R = len(temps)
        x = torch.from_numpy(synth.to_float4(np.concatenate([x0] * R))).cuda()
        v = torch.from_numpy(synth.to_float4(np.concatenate([v0] * R))).cuda()
        lpa = tune.best(R * n, 1.0, 1.0)["lanes_per_atom"]
        with sw.Context(np.arange(R + 1) * n, [L0] * R, cutoff=RC, skin=1.0, nbr_capacity=48,
                        tuning=dict(lanes_per_atom=lpa, graph_steps=50, sync_rebuild=int(R > 1))) as ctx:
            ctx.npt(x, v, warm, T0=temps, reset=True)
            sync()
            t0 = time.perf_counter()
            ctx.npt(x, v, steps, T0=temps)
            sync()
            dt = time.perf_counter() - t0
        out[name] = {"value": R * n * steps / dt, "ms_per_step": dt * 1e3 / steps, "n_atoms": R * n,
                     "lanes_per_atom": lpa, "sync_rebuild": int(R > 1)}
    out["value"] = out["batched"]["value"]
    out["single_ratio_to_nve_step"] = out["single"]["ms_per_step"] / plain4096["ms_per_step"]
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=LARGE_STEPS)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--lpa", type=int, default=0, help="lanes per atom of the main line (0 = tuned)")
    ap.add_argument("--graph-steps", type=int, default=-1,
                    help="steps per captured block of the main line, 0 = stream launches (-1 = tuned); the "
                         "launch form does not change what a kernel launch reads or writes")
    ap.add_argument("--forms", default="liquid4096,share,batched,adjoint,observables,npt",
                    help="comma list of liquid4096,share,batched,adjoint,observables,npt or none")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="first run a plain FP32 copy-like kernel (out = -in) over this many MiB, three times: "
                         "the known-size reference for scaling HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: this engine has no multi-GPU path (how it would shard is "
              "described in the design notes); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.steps < 1:
        print("--steps must be at least 1", file=sys.stderr)
        sys.exit(2)
    cpu = None if args.no_cpu else cpu_baseline()   # before the GPU is touched (forked workers)
    import torch
    torch.cuda.init()
    if args.copy_mib > 0:
        src = torch.ones(args.copy_mib << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.neg(src, out=dst)
        sync()
        del src, dst

    big = bench_large(args.steps, args.warmup, graph_steps=args.graph_steps, lpa=args.lpa)
    n, K = big["n_atoms"], args.steps
    value = n * K / big["seconds"]
    line = {
        "metric": METRIC, "value": value, "unit": "atom-steps/s", "n_gpus": 1, "steps": K,
        "warmup": args.warmup, "ms_per_step": big["seconds"] * 1e3 / K, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": big["workload"], "n_atoms": n, "skin_A": big["skin_A"], "tuning": big["tuning"],
                   "rebuilds": big["rebuilds"], "thermo_every": 100 if K >= 100 else 0},
    }
    line["audit"] = big["audit"]
    if "roofline" in big:
        line["roofline"] = big["roofline"]
        line["roofline"]["launch_floor_us"] = launch_floor_us()
    line["roofline_wall"] = wall_roofline(value)
    forms = [f for f in args.forms.split(",") if f and f != "none"]
    line["forms"] = {}
    plain = None
    if any(f in forms for f in ("liquid4096", "adjoint", "npt")):
        plain = bench_liquid4096()
        if "liquid4096" in forms:
            line["forms"]["liquid4096"] = plain
    if "share" in forms:
        line["forms"]["share"] = bench_share()
    if "batched" in forms:
        line["forms"]["batched"] = bench_batched()
    if "adjoint" in forms:
        line["forms"]["adjoint"] = bench_adjoint(plain)
    if "observables" in forms:
        line["forms"]["observables"] = bench_observables()
    if "npt" in forms:
        line["forms"]["npt"] = bench_npt(plain)
    if cpu is not None:
        line["cpu_baseline"] = cpu
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
