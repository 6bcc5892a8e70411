"""GPU parity of sw_step (velocity Verlet, thermostats) against the oracle.

Trajectories are chaotic, so trajectory parity is short-horizon (10 steps)
from identical FP32-rounded states; longer runs are checked through NVE
drift (the paper's 1/10000 criterion, read as a windowed drift) and through
exact properties (determinism, replica independence, thermostat targets).
"""
import numpy as np
import pytest

import oracle
from paper_0809_2811_amd import synth
from tests.gpu_util import RC, f32, force_error, from_dev, liquid, to_dev

pytestmark = pytest.mark.gpu


def make_ctx(x, L, skin=0.5, lpa=8, offsets=None, boxes=None, **tune):
    from paper_0809_2811_amd import sw
    offsets = [0, len(x)] if offsets is None else offsets
    boxes = [L] if boxes is None else boxes
    t = dict(lanes_per_atom=lpa)
    t.update(tune)
    return sw.Context(offsets, boxes, cutoff=RC, skin=skin, nbr_capacity=48, tuning=t)


def run_gpu(x, v, L, nsteps, thermo_every=1, **kw):
    from paper_0809_2811_amd import sw
    skin = kw.pop("skin", 0.5)
    lpa = kw.pop("lpa", 8)
    ctx = make_ctx(x, L, skin=skin, lpa=lpa)
    xd, vd = to_dev(x), to_dev(v)
    f, th = ctx.step(xd, vd, nsteps, thermo_every=thermo_every, **kw)
    return from_dev(xd), from_dev(vd), from_dev(f), (None if th is None else th.cpu().numpy()[:, 0, :]), ctx


def min_image(d, L):
    return d - L * np.round(d / L)


@pytest.mark.parametrize("which,lpa", [("ice", 8), ("liquid", 8), ("liquid", 32), ("liquid4096", 32), ("liquid4096", 64)])
def test_ten_steps_match_oracle(which, lpa):
    """liquid4096 at 32 lanes per atom is also the regression case for the
    per-block partial sums, which must hold 8-atom blocks."""
    if which == "ice":
        d = synth.config(0)
        x, v, L = d["x"], d["v"], d["box"]
    elif which == "liquid4096":
        x, v, L = liquid(2)
    else:
        x, v, L = liquid(1, sigma=0.0)
    x, v = f32(x), f32(v)
    xg, vg, fg, thg, _ = run_gpu(x, v, L, 10, lpa=lpa)
    xo, vo, fo, tho = oracle.vv(x, v, L, 10, dt=10.0)
    assert np.abs(min_image(xg - xo, L)).max() < 1e-4
    assert np.abs(vg - vo).max() < 1e-5 * np.abs(vo).max() * 10
    assert force_error(fg, fo) < 1e-4
    etot = np.abs(tho[:, 0] + tho[:, 1]).max()
    for k in range(12):
        assert np.abs(thg[:, k] - tho[:, k]).max() <= 2e-5 * max(etot, np.abs(tho[:, k]).max()), k


def test_benchmark_launch_configuration_matches_oracle():
    """The 4096-atom liquid in the launch form the benchmark times: 32 lanes
    per atom, 1.0 A skin, 48-slot rows, captured blocks of 50 steps.
    (1) 51 steps with a record every step: steps 1-50 replay one captured
    block, step 51 is launched from the stream; positions and every record
    against the FP64 oracle.  (2) 101 steps with the benchmark's thermo
    interval (100, so one 100-step block): the same bits as plain launches,
    and the step-100 energies against the oracle.  The FP32 trajectory leaves
    the FP64 one exponentially (largest position difference 4e-5 A after 50
    steps, 4e-3 A after 101 in this liquid) while the energies stay within
    1e-6 of |E|, so the long run is checked through its energies."""
    from paper_0809_2811_amd import sw
    x, v, L = liquid(2)
    x, v = f32(x), f32(v)

    def run(n, every, gs):
        ctx = sw.Context([0, len(x)], [L], cutoff=RC, skin=1.0, nbr_capacity=48,
                         tuning=dict(lanes_per_atom=32, graph_steps=gs))
        xd, vd = to_dev(x), to_dev(v)
        f, th = ctx.step(xd, vd, n, thermo_every=every)
        return from_dev(xd), from_dev(vd), from_dev(f), th.cpu().numpy()[:, 0]

    xg, vg, fg, thg = run(51, 1, 50)
    xo, vo, fo, tho = oracle.vv(x, v, L, 51, dt=10.0)
    assert np.abs(min_image(xg - xo, L)).max() < 5e-4
    assert np.abs(vg - vo).max() < 5e-4 * np.abs(vo).max()
    assert force_error(fg, fo) < 5e-4
    etot = np.abs(tho[:, 0] + tho[:, 1]).max()
    for k in range(12):
        assert np.abs(thg[:, k] - tho[:, k]).max() <= 2e-5 * max(etot, np.abs(tho[:, k]).max()), k

    a = run(101, 100, 50)
    b = run(101, 100, 0)
    for p, q in zip(a, b):
        assert np.array_equal(p, q)
    _, _, _, tho = oracle.vv(x, v, L, 101, dt=10.0)
    etot = abs(tho[99, 0] + tho[99, 1] + tho[99, 2])
    for k in (0, 1, 2):   # E2, E3, KE at step 100
        assert abs(a[3][0, k] - tho[99, k]) <= 1e-5 * etot, (k, a[3][0, k], tho[99, k])


def test_large_box_launch_configuration_matches_oracle():
    """262144 atoms (198.7 A box) in the benchmark's large-box launch form:
    8 lanes per atom, 0.5 A skin, rows rebuilt at least every 10 steps,
    captured blocks of 10 steps.  11 steps (one replayed block, then one
    stream-launched step): every atom against the FP64 oracle, and the same
    bits as plain launches."""
    from paper_0809_2811_amd import sw
    x, v, L = liquid(8)
    x, v = f32(x), f32(v)
    assert len(x) == 262144

    def run(gs):
        ctx = sw.Context([0, len(x)], [L], cutoff=RC, skin=0.5, nbr_capacity=48,
                         tuning=dict(lanes_per_atom=8, graph_steps=gs, rebuild_every=10))
        xd, vd = to_dev(x), to_dev(v)
        f, _ = ctx.step(xd, vd, 11)
        return from_dev(xd), from_dev(vd), from_dev(f)

    xg, vg, fg = run(10)
    for p, q in zip((xg, vg, fg), run(0)):
        assert np.array_equal(p, q)
    xo, vo, fo, _ = oracle.vv(x, v, L, 11, dt=10.0)
    assert np.abs(min_image(xg - xo, L)).max() < 1e-4
    assert np.abs(vg - vo).max() < 1e-4 * np.abs(vo).max()
    assert force_error(fg, fo) < 1e-4


def test_zero_steps_returns_forces():
    x, v, L = liquid(1, sigma=0.0)
    x, v = f32(x), f32(v)
    xg, vg, fg, _, _ = run_gpu(x, v, L, 0, thermo_every=0)
    assert force_error(fg, oracle.forces(x, L)["F"]) <= 1e-5
    assert np.array_equal(vg, v)
    assert np.abs(min_image(xg - x, L)).max() < 1e-5


def windowed_drift(e, frac=0.2):
    w = max(1, int(len(e) * frac))
    return abs(e[-w:].mean() - e[:w].mean()) / abs(e[0])


def test_nve_drift_ice_workload():
    d = synth.config(0)
    _, _, _, th, _ = run_gpu(f32(d["x"]), f32(d["v"]), d["box"], 100)
    e = th[:, 0] + th[:, 1] + th[:, 2]
    assert windowed_drift(e) < 1e-4


def test_nve_drift_liquid_4096():
    x, v, L = liquid(2)
    _, _, _, th, ctx = run_gpu(f32(x), f32(v), L, 2000, thermo_every=10, skin=1.0)
    e = th[:, 0] + th[:, 1] + th[:, 2]
    assert windowed_drift(e) < 1e-4
    from paper_0809_2811_amd import sw
    assert ctx.query(sw.SW_Q_REBUILDS) > 1


def test_rescale_thermostat_hits_target():
    from paper_0809_2811_amd import sw
    x, v, L = liquid(1, sigma=0.0)
    xg, vg, _, th, _ = run_gpu(f32(x), f32(v), L, 3, thermostat=sw.SW_RESCALE, T0=400.0)
    assert abs(oracle.temperature(vg) - 400.0) < 1e-3


def test_berendsen_matches_oracle():
    from paper_0809_2811_amd import sw
    x, v, L = liquid(1, sigma=0.0)
    x, v = f32(x), f32(v)
    xg, vg, _, thg, _ = run_gpu(x, v, L, 5, thermostat=sw.SW_BERENDSEN, T0=320.0, tau_fs=200.0)
    xo, vo, _, tho = oracle.vv(x, v, L, 5, dt=10.0, thermostat=2, T0=320.0, tau=200.0)
    assert np.abs(vg - vo).max() < 1e-4 * np.abs(vo).max()
    assert np.abs(thg[:, 2] - tho[:, 2]).max() < 1e-5 * tho[:, 2].max()


@pytest.mark.parametrize("reps,lpa,every", [(1, 8, 4), (2, 64, 1), (2, 64, 4)])
def test_berendsen_kinetic_sums_match_oracle(reps, lpa, every):
    """The thermostat's kinetic energy comes from the kernel's own sums (a
    512-atom replica: 16 force blocks) or, for a 4096-atom replica at 64 lanes
    per atom (1024 blocks), from the reduction launch; steps between thermo
    records run without that launch."""
    from paper_0809_2811_amd import sw
    x, v, L = liquid(reps)
    x, v = f32(x), f32(v)
    xg, vg, _, thg, _ = run_gpu(x, v, L, 8, lpa=lpa, thermo_every=every, thermostat=sw.SW_BERENDSEN, T0=350.0,
                                tau_fs=150.0)
    xo, vo, _, tho = oracle.vv(x, v, L, 8, dt=10.0, thermostat=2, T0=350.0, tau=150.0)
    assert np.abs(vg - vo).max() < 1e-4 * np.abs(vo).max()
    assert np.abs(min_image(xg - xo, L)).max() < 1e-4
    assert np.abs(thg[:, 2] - tho[every - 1::every, 2]).max() < 1e-5 * tho[:, 2].max()


def test_step_is_deterministic():
    x, v, L = liquid(2)
    a = run_gpu(f32(x), f32(v), L, 50, thermo_every=10)
    b = run_gpu(f32(x), f32(v), L, 50, thermo_every=10)
    for k in range(4):
        assert np.array_equal(a[k], b[k])


def test_large_context_thermostat_binning_keeps_replicas_exact():
    """16 replicas of the 4096-atom liquid in one context (65536 atoms: the
    thermostat kernel appends a wavefront's cell entries with one counter
    atomic per distinct cell) through Berendsen steps with row rebuilds:
    replica 0 follows the oracle over the first 8 steps, and after 40 every
    replica checked equals the same replica run alone (4096 atoms: one atomic
    per atom) bit for bit."""
    from paper_0809_2811_amd import sw
    x, v, L = liquid(2)
    x, v = f32(x), f32(v)
    n, R = len(x), 16
    T0 = [230.0 + 10.0 * r for r in range(R)]
    ctx = make_ctx(np.tile(x, (R, 1)), None, offsets=np.arange(R + 1) * n, boxes=[L] * R)
    xd, vd = to_dev(np.tile(x, (R, 1))), to_dev(np.tile(v, (R, 1)))
    r0 = ctx.query(sw.SW_Q_REBUILDS)
    ctx.step(xd, vd, 8, thermostat=sw.SW_BERENDSEN, T0=T0, tau_fs=100.0)
    xo, vo, _, _ = oracle.vv(x, v, L, 8, dt=10.0, thermostat=2, T0=T0[0], tau=100.0)
    xb, vb = from_dev(xd), from_dev(vd)
    assert np.abs(min_image(xb[:n] - xo, L)).max() < 1e-4
    assert np.abs(vb[:n] - vo).max() < 1e-4 * np.abs(vo).max()
    ctx.step(xd, vd, 32, thermostat=sw.SW_BERENDSEN, T0=T0, tau_fs=100.0)
    assert ctx.query(sw.SW_Q_REBUILDS) - r0 >= 5 * R
    xb, vb = from_dev(xd), from_dev(vd)
    for r in (0, 9, 15):
        c1 = make_ctx(x, L)
        x1, v1 = to_dev(x), to_dev(v)
        c1.step(x1, v1, 8, thermostat=sw.SW_BERENDSEN, T0=[T0[r]], tau_fs=100.0)
        c1.step(x1, v1, 32, thermostat=sw.SW_BERENDSEN, T0=[T0[r]], tau_fs=100.0)
        assert np.array_equal(from_dev(x1), xb[r * n:(r + 1) * n]), r
        assert np.array_equal(from_dev(v1), vb[r * n:(r + 1) * n]), r


def test_synchronised_rebuilds_keep_every_replica_on_the_oracle():
    """sync_rebuild: every replica rebuilds its rows whenever any replica's
    check fires (rows are still supersets of the cutoff sphere, so only the
    summation order can change): each replica follows the oracle over 8
    Berendsen steps, and every row rebuild counted is a rebuild of all
    replicas."""
    from paper_0809_2811_amd import sw
    specs = [((4, 4, 4), 1.0, 300.0), ((3, 4, 5), 0.93, 250.0), ((4, 5, 5), 1.05, 220.0)]
    xs, vs, boxes = [], [], []
    for k, (cells, rho, T) in enumerate(specs):
        d = synth.lattice_at_density(cells, rho, sigma=0.2, temperature=T, seed=40 + k)
        xs.append(f32(d["x"])); vs.append(f32(d["v"])); boxes.append(d["box"])
    offsets = np.cumsum([0] + [len(x) for x in xs])
    ctx = make_ctx(np.concatenate(xs), None, offsets=offsets, boxes=boxes, sync_rebuild=1)
    assert ctx.tuning()["sync_rebuild"] == 1
    xd, vd = to_dev(np.concatenate(xs)), to_dev(np.concatenate(vs))
    T0 = [s[2] for s in specs]
    ctx.step(xd, vd, 8, thermostat=sw.SW_BERENDSEN, T0=T0, tau_fs=100.0)
    xb, vb = from_dev(xd), from_dev(vd)
    for r in range(len(specs)):
        a, b = offsets[r], offsets[r + 1]
        xo, vo, _, _ = oracle.vv(xs[r], vs[r], boxes[r], 8, dt=10.0, thermostat=2, T0=T0[r], tau=100.0)
        assert np.abs(min_image(xb[a:b] - xo, boxes[r])).max() < 1e-4, r
        assert np.abs(vb[a:b] - vo).max() < 1e-4 * np.abs(vo).max(), r
    # 30 more steps: the call's opening build plus at least one fired check,
    # each a rebuild of every replica
    r0 = ctx.query(sw.SW_Q_REBUILDS)
    ctx.step(xd, vd, 30, thermostat=sw.SW_BERENDSEN, T0=T0, tau_fs=100.0)
    nrb = ctx.query(sw.SW_Q_REBUILDS) - r0
    assert nrb >= 2 * len(specs) and nrb % len(specs) == 0, nrb


def test_replicas_evolve_independently():
    """Each replica of a batched context equals the same replica run alone."""
    from paper_0809_2811_amd import sw
    specs = [((4, 4, 4), 1.0, 300.0), ((3, 4, 5), 0.93, 250.0), ((4, 5, 5), 1.05, 220.0)]
    xs, vs, boxes = [], [], []
    for k, (cells, rho, T) in enumerate(specs):
        d = synth.lattice_at_density(cells, rho, sigma=0.2, temperature=T, seed=40 + k)
        xs.append(f32(d["x"])); vs.append(f32(d["v"])); boxes.append(d["box"])
    offsets = np.cumsum([0] + [len(x) for x in xs])
    ctx = make_ctx(np.concatenate(xs), None, offsets=offsets, boxes=boxes)
    xd, vd = to_dev(np.concatenate(xs)), to_dev(np.concatenate(vs))
    T0 = [s[2] for s in specs]
    f, th = ctx.step(xd, vd, 30, thermostat=sw.SW_BERENDSEN, T0=T0, tau_fs=100.0, thermo_every=5)
    xb, vb = from_dev(xd), from_dev(vd)
    for r in range(3):
        c1 = make_ctx(xs[r], boxes[r])
        x1, v1 = to_dev(xs[r]), to_dev(vs[r])
        f1, th1 = c1.step(x1, v1, 30, thermostat=sw.SW_BERENDSEN, T0=[T0[r]], tau_fs=100.0, thermo_every=5)
        sl = slice(offsets[r], offsets[r + 1])
        assert np.array_equal(from_dev(x1), xb[sl])
        assert np.array_equal(from_dev(v1), vb[sl])
        assert np.array_equal(th1.cpu().numpy()[:, 0], th.cpu().numpy()[:, r])


def test_thermo_recording_does_not_change_the_trajectory():
    """Steps that also sum energies and the virial use other kernel variants;
    the trajectory must not depend on how often thermo rows are recorded."""
    x, v, L = liquid(1, sigma=0.0)
    x, v = f32(x), f32(v)
    a = run_gpu(x, v, L, 30, thermo_every=1)
    b = run_gpu(x, v, L, 30, thermo_every=0)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


@pytest.mark.parametrize("thermostat", ["nve", "berendsen"])
def test_persistent_launch_equals_launch_per_phase(thermostat):
    """The cooperative persistent kernel runs the same tile functions between
    grid barriers: results are bitwise those of one launch per phase."""
    from paper_0809_2811_amd import sw
    specs = [((4, 4, 4), 1.0, 300.0), ((3, 4, 5), 0.93, 250.0), ((4, 5, 6), 1.05, 220.0)]
    xs, vs, boxes = [], [], []
    for k, (cells, rho, T) in enumerate(specs):
        d = synth.lattice_at_density(cells, rho, sigma=0.2, temperature=T, seed=60 + k)
        xs.append(f32(d["x"])); vs.append(f32(d["v"])); boxes.append(d["box"])
    offsets = np.cumsum([0] + [len(x) for x in xs])
    kw = dict(thermo_every=5)
    if thermostat == "berendsen":
        kw.update(thermostat=sw.SW_BERENDSEN, T0=[s[2] for s in specs], tau_fs=100.0)
    out = []
    for persistent in (0, 1):
        ctx = make_ctx(np.concatenate(xs), None, offsets=offsets, boxes=boxes, persistent=persistent,
                       rebuild_every=10)
        xd, vd = to_dev(np.concatenate(xs)), to_dev(np.concatenate(vs))
        f, th = ctx.step(xd, vd, 40, **kw)
        out.append((from_dev(xd), from_dev(vd), from_dev(f), th.cpu().numpy(), ctx.query(sw.SW_Q_REBUILDS)))
        if persistent:
            assert ctx.query(sw.SW_Q_PERSISTENT_GROUPS) == 1      # three replicas: grid-wide barriers
    for k in range(5):
        assert np.array_equal(out[0][k], out[1][k]), k


@pytest.mark.parametrize("thermostat,sync", [("nve", 0), ("nve", 1), ("berendsen", 0), ("berendsen", 1)])
def test_persistent_groups_per_xcc_equal_launch_per_phase(thermostat, sync):
    """Sixteen replicas of one size: the persistent launch deals them to the
    device's XCCs and keeps each group's barriers on its XCC (with
    synchronised rebuilds the groups also meet once per step).  Results are
    bitwise those of one launch per phase, over two calls of more steps than
    one persistent launch holds (two launches each), also when the second
    call replays the first one's captured launches."""
    from paper_0809_2811_amd import sw
    xs, vs, boxes, T0 = [], [], [], []
    for k in range(16):
        rho, T = 0.92 + 0.01 * k, 220.0 + 6.0 * k
        d = synth.lattice_at_density(4, rho, sigma=0.2, temperature=T, seed=300 + k)
        xs.append(f32(d["x"])); vs.append(f32(d["v"])); boxes.append(d["box"]); T0.append(T)
    offsets = np.cumsum([0] + [len(x) for x in xs])
    kw = dict(thermo_every=7)
    if thermostat == "berendsen":
        kw.update(thermostat=sw.SW_BERENDSEN, T0=T0, tau_fs=100.0)
    nsteps = 4096 + 45
    out = []
    # per-phase launches, persistent launches, and persistent launches
    # captured on the first call and replayed on the second
    for persistent, graph_steps in ((0, 0), (1, 0), (1, 10)):
        ctx = make_ctx(np.concatenate(xs), None, offsets=offsets, boxes=boxes, persistent=persistent,
                       sync_rebuild=sync, graph_steps=graph_steps)
        xd, vd = to_dev(np.concatenate(xs)), to_dev(np.concatenate(vs))
        res = []
        for call in range(2):
            print(f"persistent={persistent} graph={graph_steps} thermostat={thermostat} sync={sync} call={call}",
                  flush=True)
            f, th = ctx.step(xd, vd, nsteps, **kw)
            res += [from_dev(xd), from_dev(vd), from_dev(f), th.cpu().numpy()]
            if persistent:
                assert ctx.query(sw.SW_Q_PERSISTENT_GROUPS) > 1
        out.append(res + [ctx.query(sw.SW_Q_REBUILDS)])
    assert out[0][-1] > 16 * 100                                   # rows were rebuilt many times
    for run in (1, 2):
        for k in range(len(out[0])):
            assert np.array_equal(out[0][k], out[run][k]), (run, k)


@pytest.mark.parametrize("thermostat", ["nve", "berendsen"])
def test_persistent_groups_with_padded_replicas(thermostat):
    """Replicas of 480 and 800 atoms (padded to 512 and 832 in the internal
    order) dealt to the XCCs: padding atoms inside a group's tiles and
    64-atom units, bitwise equal to one launch per phase."""
    from paper_0809_2811_amd import sw
    xs, vs, boxes, T0 = [], [], [], []
    for k in range(16):
        cells = (3, 4, 5) if k % 2 == 0 else (4, 5, 5)
        d = synth.lattice_at_density(cells, 0.94 + 0.007 * k, sigma=0.2, temperature=230.0 + 5.0 * k, seed=700 + k)
        xs.append(f32(d["x"])); vs.append(f32(d["v"])); boxes.append(d["box"]); T0.append(230.0 + 5.0 * k)
    offsets = np.cumsum([0] + [len(x) for x in xs])
    assert {len(x) for x in xs} == {480, 800}
    kw = dict(thermo_every=11)
    if thermostat == "berendsen":
        kw.update(thermostat=sw.SW_BERENDSEN, T0=T0, tau_fs=100.0)
    out = []
    for persistent in (0, 1):
        ctx = make_ctx(np.concatenate(xs), None, offsets=offsets, boxes=boxes, persistent=persistent,
                       sync_rebuild=1)
        xd, vd = to_dev(np.concatenate(xs)), to_dev(np.concatenate(vs))
        print(f"persistent={persistent} thermostat={thermostat}", flush=True)
        f, th = ctx.step(xd, vd, 330, **kw)
        out.append((from_dev(xd), from_dev(vd), from_dev(f), th.cpu().numpy(), ctx.query(sw.SW_Q_REBUILDS)))
        if persistent:
            assert ctx.query(sw.SW_Q_PERSISTENT_GROUPS) > 1
    for k in range(5):
        assert np.array_equal(out[0][k], out[1][k]), k


@pytest.mark.parametrize("nsteps", [1, 4096, 4097])
def test_persistent_groups_at_launch_boundaries(nsteps):
    """Calls whose last step falls at the end of the first persistent launch,
    one step after it (a second launch of one step), or in a one-step call,
    with forced rebuilds: bitwise equal to one launch per phase."""
    from paper_0809_2811_amd import sw
    xs, vs, boxes = [], [], []
    for k in range(16):
        d = synth.lattice_at_density(4, 0.95 + 0.005 * k, sigma=0.2, temperature=260.0, seed=500 + k)
        xs.append(f32(d["x"])); vs.append(f32(d["v"])); boxes.append(d["box"])
    offsets = np.cumsum([0] + [len(x) for x in xs])
    out = []
    for persistent in (0, 1):
        ctx = make_ctx(np.concatenate(xs), None, offsets=offsets, boxes=boxes, persistent=persistent,
                       rebuild_every=7, sync_rebuild=1)
        xd, vd = to_dev(np.concatenate(xs)), to_dev(np.concatenate(vs))
        print(f"persistent={persistent} nsteps={nsteps}", flush=True)
        f, _ = ctx.step(xd, vd, nsteps)
        out.append((from_dev(xd), from_dev(vd), from_dev(f), ctx.query(sw.SW_Q_REBUILDS)))
        if persistent:
            assert ctx.query(sw.SW_Q_PERSISTENT_GROUPS) > 1
    for k in range(4):
        assert np.array_equal(out[0][k], out[1][k]), k


@pytest.mark.parametrize("thermostat", ["nve", "berendsen"])
def test_graph_replays_equal_plain_launches(thermostat):
    """Blocks of steps replayed from a captured hipGraph give bitwise the
    results of plain launches, on every replay: the same context runs three
    calls in a row with eager work and synchronisations in between."""
    import torch
    from paper_0809_2811_amd import sw
    x, v, L = liquid(2)
    x, v = f32(x), f32(v)
    kw = dict(thermo_every=5)
    if thermostat == "berendsen":
        kw.update(thermostat=sw.SW_BERENDSEN, T0=[320.0], tau_fs=100.0)
    runs = {}
    for graph_steps in (0, 10):
        ctx = make_ctx(x, L, skin=0.6, graph_steps=graph_steps, rebuild_every=5)
        xd, vd = to_dev(x), to_dev(v)
        out = []
        for call in range(3):
            f, th = ctx.step(xd, vd, 37, **kw)
            out.append((from_dev(xd), from_dev(vd), from_dev(f), th.cpu().numpy()))
            junk = torch.randn(1000, device="cuda").sum()      # eager work between replays
            torch.cuda.synchronize()
            assert torch.isfinite(junk)
        runs[graph_steps] = out
    for call in range(3):
        for k in range(4):
            assert np.array_equal(runs[0][call][k], runs[10][call][k]), (call, k)


@pytest.mark.parametrize("lpa,graph", [(8, 0), (32, 0), (8, 20)])
def test_missed_pair_audit(lpa, graph):
    """The rows in use are audited against a fresh search of the cells after
    every step's moments launch: 120 NVE steps of the 4096-atom liquid with a
    0.5 A skin (rows rebuilt on the displacement check only) miss no pair
    inside a*sigma, and the audited pair count of a single step equals the
    oracle's count of ordered pairs within a*sigma at the returned
    positions (up to pairs within float rounding of the cut-off)."""
    from paper_0809_2811_amd import sw
    x, v, L = liquid(2)
    x, v = f32(x), f32(v)
    ctx = sw.Context([0, len(x)], [L], cutoff=RC, skin=0.5, nbr_capacity=48,
                     tuning=dict(lanes_per_atom=lpa, graph_steps=graph, audit_every=1))
    xd, vd = to_dev(x), to_dev(v)
    ctx.step(xd, vd, 1)
    pairs1 = ctx.query(sw.SW_Q_AUDIT_PAIRS)
    ref = int(oracle.neighbour_counts(from_dev(xd), L, RC).sum())
    assert abs(pairs1 - ref) <= 2, (pairs1, ref)
    r0 = ctx.query(sw.SW_Q_REBUILDS)
    ctx.step(xd, vd, 120)
    assert ctx.query(sw.SW_Q_REBUILDS) - r0 >= 10          # the check fired many times
    pairs = ctx.query(sw.SW_Q_AUDIT_PAIRS) - pairs1
    assert 0.9 * 120 * pairs1 < pairs < 1.1 * 120 * pairs1
    assert ctx.query(sw.SW_Q_MISSED_PAIRS) == 0
    ctx.close()
