"""Throughput benchmark of the mW Stillinger-Weber engine on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--forms large,batched,adjoint|none]

Main line: the 4096-atom liquid workload - 8x8x8 diamond cells scaled to
1.00 g/cm^3, melted for 2000 velocity-Verlet steps (10 fs) with velocities
rescaled to 400 K, then 500 steps rescaled to 298 K, then W untimed and K
timed NVE steps.  A "step" is one full velocity-Verlet step of the whole path
(neighbour rows rebuilt on the device when the displacement check fires,
moments, forces, integration, thermo sums every 100 steps).  Inputs are
resident in HBM before the timed region starts.

Prints one JSON line.  The dominant kernel's duration comes from HIP events
recorded by the library around sampled launches inside the timed region.
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
PEAK_FP32_VALU = 78.6e12   # 256 CU x 64 lanes x 2 flop (FMA) x 2.4 GHz, non-packed FP32
PEAK_HBM = 8.0e12

# Algorithmic work per launch, counted from the kernel sources.
# k_forces (NVE mode): per active directed pair (r < a sigma) 120 flop
# including 4 transcendentals; per row entry beyond a sigma 14 flop (distance
# test); per atom 30 flop (group reduction, two half-kicks, drift).  Bytes per
# atom: own position, own moments, row length and row, force, velocity in and
# out, new position, binning slot: 16+48+4+4*row+16+32+16+8.  With 8 or fewer
# lanes per atom the kernel reads the moments launch's list of the entries
# within the cutoff instead of the row (4 + 4*active bytes, no inactive
# entries), and the moments launch writes that list (4 + 4*active more).
FLOP_PER_ACTIVE = 120.0
FLOP_PER_INACTIVE = 14.0
FLOP_PER_ATOM = 30.0
# k_moments: 44 flop incl. 3 transcendentals per active pair, 14 per inactive
# entry, 20 per atom; bytes per atom: position, row length and row, moments
# out (16+4+4*row+48).  On a rebuild step add 12 flop per candidate of the 27
# cells and, per atom, the cell slot read, the row written and the reference
# position (16+4*row+4+16).
MOM_FLOP_PER_ACTIVE = 44.0
MOM_FLOP_PER_ATOM = 20.0
REBUILD_FLOP_PER_CAND = 12.0


def number_density(rho_gcc=1.0, mass=18.015):
    return rho_gcc / mass * 6.02214076e23 * 1e-24


def expected_counts(rho_gcc, skin):
    n = number_density(rho_gcc)
    act = 4.0 / 3.0 * np.pi * RC ** 3 * n
    row = 4.0 / 3.0 * np.pi * (RC + skin) ** 3 * n
    return act, row


def force_kernel_work(n_atoms, rho_gcc, skin, lpa=32):
    act, row = expected_counts(rho_gcc, skin)
    listed = act if lpa <= 8 else row
    flop = n_atoms * (act * FLOP_PER_ACTIVE + (listed - act) * FLOP_PER_INACTIVE + FLOP_PER_ATOM)
    bytes_ = n_atoms * (16 + 48 + 4 + 4 * listed + 16 + 32 + 16 + 8)
    return flop, bytes_


def moments_kernel_work(n_atoms, rho_gcc, skin, box, rebuild_frac, lpa=32):
    """Average over launches; rebuild_frac of them rebuild the rows."""
    act, row = expected_counts(rho_gcc, skin)
    ncell = [max(3, int(np.floor(b / (RC + skin)))) for b in np.atleast_1d(box) * np.ones(3)]
    cand = 27.0 * number_density(rho_gcc) * np.prod([b / c for b, c in zip(np.atleast_1d(box) * np.ones(3), ncell)])
    flop = n_atoms * (act * MOM_FLOP_PER_ACTIVE + (row - act) * FLOP_PER_INACTIVE + MOM_FLOP_PER_ATOM
                      + rebuild_frac * cand * REBUILD_FLOP_PER_CAND)
    bytes_ = n_atoms * (16 + 4 + 4 * row + 48 + rebuild_frac * (16 + 4 * row + 4 + 16)
                        + (4 + 4 * act if lpa <= 8 else 0))
    return flop, bytes_


def kernel_sources_digest():
    from paper_0809_2811_amd import hbm_counters
    return hbm_counters.kernel_sources_digest()


def measured_traffic(kernel, workload):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, each scaled by the same
    counter's reading for a plain copy of known size) recorded for this
    kernel and workload, or None when no record exists or the kernel sources
    changed since the counters were taken."""
    from paper_0809_2811_amd import hbm_counters
    return hbm_counters.measured_traffic(kernel, workload)


def sync():
    import torch
    torch.cuda.synchronize()


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


def timed_nve(ctx, x, v, steps, thermo_every=100, timing=49):
    """One timed NVE call.  Kernel durations come from HIP events around the
    two launches of every `timing`-th step (odd: both buffer parities).  When
    the call replays captured step blocks, only the steps after the last
    block run as stream launches, so every one of them is sampled."""
    from paper_0809_2811_amd import sw
    if ctx.tuning().get("graph_steps", 0) > 0:
        timing = 1
    ctx.set_tuning(timing=timing)
    r0 = ctx.query(sw.SW_Q_REBUILDS)
    sync()
    t0 = time.perf_counter()
    f, th = ctx.step(x, v, steps, thermo_every=thermo_every if steps >= thermo_every else 0)
    sync()
    dt = time.perf_counter() - t0
    out = dict(seconds=dt, rebuilds=ctx.query(sw.SW_Q_REBUILDS) - r0)
    ns = ctx.query(sw.SW_Q_TIMED_STEPS)
    if ns > 0:
        out["forces_us"] = ctx.query(sw.SW_Q_TIME_FORCES_NS) / ns / 1e3
        out["moments_us"] = ctx.query(sw.SW_Q_TIME_MOMENTS_NS) / ns / 1e3
        out["timed_launches"] = ns
    if th is not None:
        e = th[:, 0, 0] + th[:, 0, 1] + th[:, 0, 2]
        e = e.cpu().numpy()
        out["etot_first_last"] = [float(e[0]), float(e[-1])]
    ctx.set_tuning(timing=0)
    return out


def kernel_roofline(kernel, flop, bytes_, kernel_us, workload):
    """Roofline entry of one kernel: the bound is the roof the algorithmic
    counts reach first (bytes at 8 TB/s against flop at the non-packed FP32
    vector peak)."""
    sec = kernel_us * 1e-6
    t_alu, t_hbm = flop / PEAK_FP32_VALU, bytes_ / PEAK_HBM
    traffic = measured_traffic(kernel, workload)
    out = {"kernel": kernel, "kernel_us": kernel_us, "flop_per_launch": flop, "alg_bytes_per_launch": bytes_,
           "alu_frac": flop / sec / PEAK_FP32_VALU, "hbm_frac": bytes_ / sec / PEAK_HBM}
    if t_hbm >= t_alu:
        out.update(bound="hbm", achieved=bytes_ / sec / 1e9, peak=PEAK_HBM / 1e9, unit="GB/s",
                   frac=bytes_ / sec / PEAK_HBM)
    else:
        out.update(bound="alu", achieved=flop / sec / 1e12, peak=PEAK_FP32_VALU / 1e12, unit="TFLOP/s",
                   frac=flop / sec / PEAK_FP32_VALU)
    out["traffic"] = traffic
    return out


def step_rooflines(n_atoms, rho, skin, box, res, steps, lpa, workload):
    """Both kernels of the step; the dominant one (longest average launch)
    becomes the line's roofline, the other is kept under "other"."""
    ff, fb = force_kernel_work(n_atoms, rho, skin, lpa)
    mf, mb = moments_kernel_work(n_atoms, rho, skin, box, min(1.0, res["rebuilds"] / max(steps, 1)), lpa)
    kf = kernel_roofline(f"k_forces<{lpa}, 2, false>", ff, fb, res["forces_us"], workload)
    km = kernel_roofline(f"k_moments<{lpa}, false>", mf, mb, res["moments_us"], workload)
    dom, other = (kf, km) if res["forces_us"] >= res["moments_us"] else (km, kf)
    order = ("bound", "achieved", "peak", "unit", "frac", "traffic")
    line = {k: dom[k] for k in order}
    line.update({k: v for k, v in dom.items() if k not in order})
    line["other"] = other
    return line


def launch_floor_us(n=200, reps=5):
    """What one launch costs on this GPU with almost no work in it: a plain
    elementwise add over 131072 floats, n launches captured in a graph and
    replayed (the step kernels are replayed the same way); microseconds per
    launch.  Context for the step kernels' durations, which sit close to a
    few of these."""
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


def cpu_baseline(target_s=15.0):
    """The FP64 oracle (single thread) on a 4096-atom 298 K liquid: the
    oracle-made 512-atom liquid tiled 2x2x2 and perturbed by 0.02 A."""
    import oracle
    from paper_0809_2811_amd import synth
    x, v, L = synth.load_state(os.path.join(ROOT, "tests", "golden", "liquid512_298K.npz"))
    x, v, L = synth.tile(x, v, L, 2, sigma=0.02, seed=5)
    n = len(x)
    t0 = time.perf_counter()
    x1, v1, _, _ = oracle.vv(x, v, L, 10, dt=10.0)
    per_step = (time.perf_counter() - t0) / 10
    steps = max(10, int(target_s / per_step))
    t0 = time.perf_counter()
    oracle.vv(x1, v1, L, steps, dt=10.0)
    dt = time.perf_counter() - t0
    return {"value": n * steps / dt, "unit": "atom-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{n}-atom 298 K liquid (oracle-made 512-atom liquid tiled 2x2x2), {steps} FP64 NVE "
                      f"velocity-Verlet steps at 10 fs, single thread, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=500)
    ap.add_argument("--skin", type=float, default=0.0, help="Verlet skin in A (0 = tuned)")
    ap.add_argument("--lpa", type=int, default=0, help="lanes per atom (0 = tuned default)")
    ap.add_argument("--graph-steps", type=int, default=-1,
                    help="steps per captured block, 0 = stream launches (-1 = tuned); the launch form does not "
                         "change what a kernel launch reads or writes")
    ap.add_argument("--forms", default="large,share,batched,adjoint,observables,npt",
                    help="comma list of large,share,batched,adjoint,observables,npt or none")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="first run a plain FP32 copy-like kernel (out = -in) over this many MiB, three times: "
                         "the known-size reference for scaling HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: this engine has no multi-GPU path; run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_0809_2811_amd import synth, tune
    torch.cuda.init()
    if args.copy_mib > 0:
        src = torch.ones(args.copy_mib << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.neg(src, out=dst)
        sync()
        del src, dst

    cfg = synth.config(1)
    n = len(cfg["x"])
    tuning = tune.best(n, 1.0, args.skin if args.skin > 0 else None)
    skin = args.skin if args.skin > 0 else tuning.get("skin", 1.0)
    tuning.pop("skin", None)
    if args.lpa:
        tuning["lanes_per_atom"] = args.lpa
    if args.graph_steps >= 0:
        tuning["graph_steps"] = args.graph_steps
    args.skin = skin
    ctx, x, v = prepare_liquid(cfg, args.skin, tuning)
    if args.warmup > 0:
        ctx.step(x, v, args.warmup)
    res = timed_nve(ctx, x, v, args.steps)
    value = n * args.steps / res["seconds"]
    line = {
        "metric": METRIC, "value": value, "unit": "atom-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": res["seconds"] * 1e3 / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "liquid4096_nve: 4096 mW atoms (8^3 diamond cells at 1.00 g/cm^3), melted "
                               "2000 steps at 400 K + 500 steps at 298 K, NVE velocity Verlet dt=10 fs",
                   "n_atoms": n, "skin_A": args.skin, "tuning": tuning, "rebuilds": res["rebuilds"],
                   "thermo_every": 100},
    }
    if "forces_us" in res:
        line["roofline"] = step_rooflines(n, 1.0, args.skin, cfg["box"], res, args.steps,
                                          tuning["lanes_per_atom"], "liquid4096")
        line["roofline"]["launch_floor_us"] = launch_floor_us()
    forms = [f for f in args.forms.split(",") if f and f != "none"]
    line["forms"] = {}
    if "large" in forms:
        line["forms"]["large_box"] = bench_large(graph_steps=args.graph_steps)
    if "share" in forms:
        line["forms"]["share"] = bench_share()
    if "batched" in forms:
        line["forms"]["batched"] = bench_batched()
    if "adjoint" in forms:
        line["forms"]["adjoint"] = bench_adjoint(line["ms_per_step"])
    if "observables" in forms:
        line["forms"]["observables"] = bench_observables(ctx, x)
    if "npt" in forms:
        line["forms"]["npt"] = bench_npt(line["ms_per_step"])
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)


def bench_share(steps=1000, skin=0.5):
    """One GPU's owned share of the large box decomposed over 8 GPUs (2x2x2
    bricks): 32768 atoms (16^3 cells at 1.00 g/cm^3), the large box's
    protocol (melt, 0.5 A skin, rows rebuilt at least every 10 steps).  A
    periodic box stands in for the brick; its ghost shell (~10k atoms) and
    the halo exchanges are not modelled."""
    from paper_0809_2811_amd import synth, tune
    cfg = synth.lattice_at_density(16, 1.0, sigma=0.05, temperature=400.0, seed=synth.SEED_CONFIG_BASE + 2)
    cfg.update(melt_T=400.0, melt_steps=2000, T=298.0)
    n = len(cfg["x"])
    tuning = tune.best(n, 1.0, skin)
    tuning.pop("skin", None)
    tuning["rebuild_every"] = 10
    ctx, x, v = prepare_liquid(cfg, skin, tuning)
    ctx.step(x, v, 50)
    res = timed_nve(ctx, x, v, steps)
    return {"value": n * steps / res["seconds"], "unit": "atom-steps/s", "steps": steps,
            "ms_per_step": res["seconds"] * 1e3 / steps, "n_atoms": n, "skin_A": skin,
            "rebuilds": res["rebuilds"], "tuning": tuning,
            "workload": "share: 32768 atoms (one GPU's owned brick of the 262144-atom box on 8 GPUs, as a periodic "
                        "box), 298 K liquid, NVE dt=10 fs, 0.5 A skin, rows rebuilt at least every 10 steps"}


def bench_large(steps=1000, skin=0.5, graph_steps=-1):
    """262144 atoms (32^3 cells, 1.00 g/cm^3), 298 K liquid, 1000 NVE steps,
    rows rebuilt at least every 10 steps and whenever the skin check fires."""
    from paper_0809_2811_amd import synth, tune
    cfg = synth.config(2)
    n = len(cfg["x"])
    tuning = tune.best(n, 1.0, skin)
    tuning.pop("skin", None)
    tuning["rebuild_every"] = 10
    if graph_steps >= 0:
        tuning["graph_steps"] = graph_steps
    ctx, x, v = prepare_liquid(cfg, skin, tuning)
    ctx.step(x, v, 50)
    res = timed_nve(ctx, x, v, steps)
    out = {"value": n * steps / res["seconds"], "unit": "atom-steps/s", "steps": steps,
           "ms_per_step": res["seconds"] * 1e3 / steps, "n_atoms": n, "skin_A": skin,
           "rebuilds": res["rebuilds"], "tuning": tuning,
           "workload": "large_box: 262144 atoms, 298 K liquid, NVE dt=10 fs, 0.5 A skin, rows rebuilt at "
                       "least every 10 steps"}
    if "forces_us" in res:
        out["roofline"] = step_rooflines(n, 1.0, skin, cfg["box"], res, steps, tuning["lanes_per_atom"],
                                         "liquid262144")
    return out


def bench_batched(steps=5000, melt_steps=1000, skin=1.0, sequential_steps=500):
    """64 uneven replicas (512-8192 atoms, 0.92-1.05 g/cm^3, 200-320 K) in one
    context: melted together at 400 K (rescale, untimed), then `steps`
    Berendsen steps (tau 1 ps) at each replica's temperature, thermo every
    100 steps.  Timed with one launch per phase and with the persistent
    cooperative kernel; and, for comparison, the replicas one after another
    through single-replica contexts (plain engine)."""
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
    ctx = sw.Context(off, boxes, cutoff=RC, skin=skin, nbr_capacity=48, tuning=base)
    ctx.step(x0, v0, melt_steps, thermostat=sw.SW_RESCALE, T0=[400.0] * len(boxes))
    out = {"workload": f"batched: {len(boxes)} replicas, {n} atoms total (512-8192 each, 0.92-1.05 g/cm^3), "
                       f"melted {melt_steps} steps at 400 K, then Berendsen (tau 1 ps) at 200-320 K, dt=10 fs",
           "n_atoms": n, "n_replicas": len(boxes), "steps": steps, "unit": "atom-steps/s", "skin_A": skin,
           "tuning": dict(base)}
    for name, persistent in (("per_phase", 0), ("persistent", 1)):
        ctx.set_tuning(persistent=persistent)
        x, v = x0.clone(), v0.clone()
        ctx.step(x, v, 50, thermostat=sw.SW_BERENDSEN, T0=T, tau_fs=1000.0)
        sync()
        t0 = time.perf_counter()
        ctx.step(x, v, steps, thermostat=sw.SW_BERENDSEN, T0=T, tau_fs=1000.0, thermo_every=100)
        sync()
        dt = time.perf_counter() - t0
        out[name] = {"value": n * steps / dt, "ms_per_step": dt * 1e3 / steps}
    ctx.set_tuning(persistent=0)
    # the same replicas one after another, each in its own context
    xs, vs = x0.clone(), v0.clone()
    total = 0.0
    for r in range(len(boxes)):
        a, b = int(off[r]), int(off[r + 1])
        t1 = tune.best(b - a, 1.0, skin)
        t1.pop("skin", None)
        c1 = sw.Context([0, b - a], [boxes[r]], cutoff=RC, skin=skin, nbr_capacity=48, tuning=t1)
        xr, vr = xs[a:b].contiguous(), vs[a:b].contiguous()
        c1.step(xr, vr, 20, thermostat=sw.SW_BERENDSEN, T0=[T[r]], tau_fs=1000.0)
        sync()
        t0 = time.perf_counter()
        c1.step(xr, vr, sequential_steps, thermostat=sw.SW_BERENDSEN, T0=[T[r]], tau_fs=1000.0)
        sync()
        total += time.perf_counter() - t0
    out["one_at_a_time"] = {"value": n * sequential_steps / total, "ms_per_step": total * 1e3 / sequential_steps,
                            "steps": sequential_steps}
    best = max(out["per_phase"]["value"], out["persistent"]["value"])
    out["value"] = best
    out["speedup_vs_one_at_a_time"] = best / out["one_at_a_time"]["value"]
    return out


def bench_adjoint(plain_ms_per_step, steps=200, ckpt=20, skin=None):
    """Differentiable trajectory: 4096-atom 298 K liquid (same preparation as
    the main line), 200 NVE steps, checkpoints every 20; one call computes
    the loss, dL/dx0, dL/dv0 and dL/d(lambda, eps, sigma)."""
    from paper_0809_2811_amd import synth, tune
    cfg = synth.config(4)
    n = len(cfg["x"])
    tuning = tune.best(n, 1.0, skin)
    skin = tuning.pop("skin", 1.0) if skin is None else skin
    ctx, x, v = prepare_liquid(cfg, skin, tuning)
    ctx.adjoint(x, v, steps, ckpt_every=ckpt)   # untimed: captures the call's launch graph (graph mode)
    sync()
    t0 = time.perf_counter()
    reps = 3
    for _ in range(reps):
        res = ctx.adjoint(x, v, steps, ckpt_every=ckpt)
    sync()
    dt = (time.perf_counter() - t0) / reps
    ms = dt * 1e3 / steps
    th = res["thbar"].cpu().numpy()[0]
    # The same call with every frame kept (one segment: the frame store holds
    # all steps + 1 frames, ~90 MB here, so the reverse sweep recomputes
    # nothing); its results are bitwise those of the checkpointed call.
    ctx.adjoint(x, v, steps, ckpt_every=steps)
    sync()
    t0 = time.perf_counter()
    for _ in range(reps):
        res_all = ctx.adjoint(x, v, steps, ckpt_every=steps)
    sync()
    dt_all = (time.perf_counter() - t0) / reps
    same = all(bool(torch_equal(res[k], res_all[k])) for k in ("loss", "thbar", "xbar0", "vbar0"))
    return {"workload": f"adjoint: {n}-atom 298 K liquid, {steps}-step NVE trajectory, checkpoints every {ckpt}, "
                        "loss = mean PE/atom + mean three-body energy/atom",
            "seconds_per_trajectory": dt, "ms_per_step": ms, "value": n * steps / dt, "unit": "atom-steps/s",
            "ratio_to_plain_step": ms / plain_ms_per_step, "loss": float(res["loss"].cpu()[0]),
            "dL_dtheta": [float(t) for t in th],
            "all_frames_stored": {"ckpt_every": steps, "ms_per_step": dt_all * 1e3 / steps,
                                  "value": n * steps / dt_all, "ratio_to_plain_step": dt_all * 1e3 / steps / plain_ms_per_step,
                                  "bitwise_equal_to_checkpointed": same}}


def torch_equal(a, b):
    import torch
    return torch.equal(a, b)


def bench_observables(ctx, x, reps=20):
    """One sampling frame of the Sec. II.C estimators on the main-line liquid
    (4096 atoms): pair-distance histogram to the largest radius the cells allow
    (0.02 A bins), angle histogram over the 8 closest neighbours (1 degree
    bins), and the mean square displacement update; each call sorts and bins
    the positions itself."""
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
    return out


def bench_npt(plain_ms_per_step, steps=5000, warm=1000):
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
        # captured 50-step blocks: faster for isobaric steps at both sizes (16.9 vs 17.8 us, 37.4 vs 37.9 us);
        # replicas rebuilding together: 36.3 -> 27.7 us per step for the nine
        ctx = sw.Context(np.arange(R + 1) * n, [L0] * R, cutoff=RC, skin=1.0, nbr_capacity=48,
                         tuning=dict(lanes_per_atom=lpa, graph_steps=50, sync_rebuild=int(R > 1)))
        ctx.npt(x, v, warm, T0=temps, reset=True)
        sync()
        t0 = time.perf_counter()
        ctx.npt(x, v, steps, T0=temps)
        sync()
        dt = time.perf_counter() - t0
        out[name] = {"value": R * n * steps / dt, "ms_per_step": dt * 1e3 / steps, "n_atoms": R * n,
                     "lanes_per_atom": lpa, "sync_rebuild": int(R > 1)}
    out["value"] = out["batched"]["value"]
    out["single_ratio_to_nve_step"] = out["single"]["ms_per_step"] / plain_ms_per_step
    return out


if __name__ == "__main__":
    main()
