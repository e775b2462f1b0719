"""Two steps per pass (temporal blocking) against single steps, through the
C-ABI: the states must be bitwise identical, for both models, widths from one
to sixteen waves, ragged strips, step counts that are not multiples of four,
a fresh start inside the fused run, graphs and direct launches; and the fused
trajectory against the FP64 oracle to the FP32 bar."""
import sys

import numpy as np
import pytest

import oracle
from paper_2409_06412_amd import workloads

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def run(xyl, spec, fusion, nsteps_list, graph_steps=32, state=None, shape=None):
    lat = xyl.Lattice(spec.Lx, spec.Ly, dtype="f32", schedule=spec.schedule, seed=spec.seed, replica=spec.replica,
                      **spec.params())
    lat.set_fusion(fusion)
    lat.set_graph_steps(graph_steps)
    if shape is not None:
        lat.set_step2_shape(*shape)
    if state is None:
        lat.init_random()
    else:
        lat.set_state(*state)
    for n in nsteps_list:
        lat.step(n)
    out = lat.get_state()
    lat.close()
    return out


@pytest.mark.parametrize("Lx,Ly,model,graphs,steps", [
    (256, 37, "xy", 32, [41]),             # one wave per row, ragged strips, remainder steps
    (512, 64, "xy", 0, [8, 3, 12]),        # direct launches, mixed counts
    (1024, 20, "si", 32, [64, 7]),         # Si model
    (4096, 48, "xy", 32, [100]),           # sixteen waves per row (full workgroup)
    (768, 9, "xy", 8, [40]),               # three waves, 9 rows (strips of 2 rows)
    (4096, 4, "xy", 0, [24]),              # the smallest height: two strips whose halos wrap onto each other
    (256, 5, "si", 32, [20]),              # one wave, an odd height (a one-row last strip)
    (2048, 2048, "si", 32, [36]),          # the size rule's 8-row strips, Si model
    (192, 20, "xy", 32, [44]),             # a partial wave: 48 of 64 lanes
    (384, 33, "si", 0, [24]),              # a full and a half wave, Si model
    (448, 64, "xy", 32, [40]),             # 2 waves, the last 48 lanes
    (640, 17, "xy", 8, [16, 8]),           # 3 waves, the last half full
    (4000, 10, "xy", 32, [20]),            # 16 waves, the last 40 lanes
    (776, 7, "xy", 32, [24]),              # 4 waves, the last with two lanes (the fewest taken)
    (1020, 19, "si", 0, [16]),             # 4 waves, the last 63 lanes
    (4092, 6, "xy", 32, [12]),             # 16 waves, the last 63 lanes
    (196, 33, "xy", 8, [20]),              # one wave of 49 lanes
    (4100, 9, "xy", 32, [24]),             # wider than 16 waves: two column tiles with one-quad halos
    (5000, 7, "si", 0, [16]),              # two tiles, Si model
    (8192, 12, "xy", 32, [20]),            # three tiles
    (12288, 6, "xy", 8, [12, 8]),          # four tiles
])
def test_two_steps_per_pass_equal_single_steps(xyl, Lx, Ly, model, graphs, steps):
    say("fusion", Lx, Ly, model, graphs, steps)
    if model == "si":
        spec = workloads.si_lattice(Lx, Ly, seed=3, replica=2)
    else:
        spec = workloads.LatticeSpec(Lx, Ly, schedule=((0, 0.9), (60, 0.2)), seed=3, replica=2)
    a = run(xyl, spec, 1, steps, graphs)
    b = run(xyl, spec, 2, steps, graphs)
    assert a[2] == b[2] == sum(steps)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])


@pytest.mark.parametrize("Lx,Ly,model,tile_waves,rows,tiles", [
    (8192, 12, "xy", 16, 4, 3),            # the fewest tiles: 3 of 11 waves
    (8192, 12, "xy", 8, 4, 5),             # 5 tiles of 7 waves (the last wave 8 lanes)
    (8192, 12, "xy", 6, 2, 6),             # 6 tiles of 6 waves
    (8192, 12, "xy", 4, 8, 9),             # 9 tiles of 4 waves
    (8200, 9, "si", 4, 4, 9),              # Si model, the last tile narrower
    (6144, 7, "xy", 11, 2, 3),             # 3 tiles of 9 waves, the ninth two lanes
    (4100, 10, "si", 8, 4, 3),             # 3 tiles of 6 waves, Si model
    (8192, 40, "xy", 3, 32, 11),           # 11 tiles of 3 waves, a ragged second strip
    (8192, 12, "xy", 2, 4, 17),            # 17 tiles of 2 waves
    (4096, 12, "xy", 16, 4, 1),            # whole rows (one workgroup per strip)
    (4096, 10, "xy", 4, 4, 5),             # a row that fits one workgroup, split: 5 tiles of 4 waves
    (4096, 9, "si", 2, 2, 9),              # 9 tiles of 2 waves, Si model
    (2048, 8, "xy", 3, 8, 3),              # 3 tiles of 3 waves
    (1024, 6, "xy", 2, 2, 3),              # 3 tiles of 2 waves, the smallest height
])
def test_column_tile_widths_equal_single_steps(xyl, Lx, Ly, model, tile_waves, rows, tiles):
    """Every tile width the shape setting (and the autotuner) may pick: the
    two-step pass over narrower tiles, in the instances bounded to 4 and 8
    waves, equals single steps bit for bit."""
    say("tile widths", Lx, Ly, model, tile_waves, rows)
    if model == "si":
        spec = workloads.si_lattice(Lx, Ly, seed=5, replica=1)
    else:
        spec = workloads.LatticeSpec(Lx, Ly, schedule=((0, 0.8), (40, 0.3)), seed=5, replica=1)
    lat = xyl.Lattice(Lx, Ly, dtype="f32", schedule=spec.schedule, seed=spec.seed, replica=spec.replica,
                      **spec.params())
    lat.set_fusion(2)
    lat.set_step2_shape(rows, tile_waves)
    assert lat.step2_shape() == (rows, tile_waves, tiles)
    lat.close()
    a = run(xyl, spec, 1, [22], 32)
    b = run(xyl, spec, 2, [22], 32, shape=(rows, tile_waves))
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])


def test_fused_run_from_a_fresh_state_matches_oracle(xyl):
    """set_state makes the first step fresh; the fused path takes it inside a
    pass.  Against the FP64 oracle from the same FP32-representable start."""
    Lx, Ly = 512, 40
    spec = workloads.LatticeSpec(Lx, Ly, schedule=((0, 0.5),), seed=6, replica=1)
    th, om = workloads.random_state(Lx, Ly, seed=8, omega_scale=0.5)
    th = th.astype(np.float32).astype(np.float64)
    om = om.astype(np.float32).astype(np.float64)
    a = run(xyl, spec, 2, [100], 32, state=(th, om))
    b = run(xyl, spec, 1, [100], 32, state=(th, om))
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])
    o = oracle.Oracle(**spec.oracle_kwargs())
    tr, wr = o.run(th, om, 0, 100)
    d = np.abs(np.remainder(a[0] - tr + np.pi, 2 * np.pi) - np.pi).max()
    say("fused vs oracle max|dtheta|", d)
    assert d <= 1e-4


@pytest.mark.parametrize("Lx,Ly,model", [(8200, 6, "xy"), (4100, 9, "xy"), (448, 33, "xy"),
                                         (8200, 6, "si"), (4100, 9, "si"), (448, 33, "si")])
def test_fused_tiles_and_partial_waves_match_oracle(xyl, Lx, Ly, model):
    """Column tiles (8200 and 4100 wide) and a partial last wave (448) in the
    two-step pass against the FP64 oracle from the same FP32-representable
    start, to the FP32 bar.  XY: 100 steps from random angles and velocities,
    1e-4 at every site.  Si: 20 steps from the random start at T_c (zero
    velocities), with the bar of the small Si lattices (at most 1% of the
    sites beyond 1e-4, median within 1e-5): its field has a cusp at the
    half-circle wrap, across which one ulp of rounding per step can move a
    site within 20 steps (tests/test_oracle_sensitivity.py)."""
    if model == "si":
        spec = workloads.si_lattice(Lx, Ly, seed=9, replica=4)
        th, om = oracle.Oracle(**spec.oracle_kwargs()).init_random()
        period, nsteps = np.pi, 20
    else:
        spec = workloads.LatticeSpec(Lx, Ly, schedule=((0, 0.7), (50, 0.3)), seed=9, replica=4)
        th, om = workloads.random_state(Lx, Ly, seed=21, omega_scale=0.5)
        period, nsteps = 2 * np.pi, 100
    th = th.astype(np.float32).astype(np.float64)
    om = om.astype(np.float32).astype(np.float64)
    say("fused vs oracle", Lx, Ly, model)
    got = run(xyl, spec, 2, [nsteps], 32, state=(th, om))
    o = oracle.Oracle(**spec.oracle_kwargs())
    tr, _ = o.run(th, om, 0, nsteps)
    d = np.abs(np.remainder(got[0] - tr + period / 2, period) - period / 2)
    say("max|dtheta|", d.max(), "sites beyond 1e-4", int(np.count_nonzero(d > 1e-4)))
    if model == "xy":
        assert d.max() <= 1e-4
    else:
        assert np.count_nonzero(d > 1e-4) <= 0.01 * Lx * Ly
        assert np.median(d) <= 1e-5


def test_fusion_keeps_measurement_and_state_buffers(xyl):
    """Sampled runs (measurement steps are single steps) and the lattice's own
    buffers: after fused stepping the velocity lives in the lattice's buffer."""
    spec = workloads.LatticeSpec(1024, 64, schedule=((0, 0.6),), seed=2)
    res = []
    for fusion in (1, 2):
        lat = xyl.Lattice(1024, 64, dtype="f32", schedule=spec.schedule, seed=2, **spec.params())
        lat.set_fusion(fusion)
        lat.init_random()
        s = lat.step_measured(250, 50)
        th_buf, u_buf, fresh = lat.state_buffers()
        assert u_buf == lat._bufs[2].data_ptr()          # the lattice's own velocity buffer
        res.append((s, lat.get_state()))
        lat.close()
    np.testing.assert_array_equal(res[0][0], res[1][0])
    np.testing.assert_array_equal(res[0][1][0], res[1][1][0])
    np.testing.assert_array_equal(res[0][1][1], res[1][1][1])


def test_fusion_query_reports_the_mode_in_effect(xyl):
    """xyl_get_fusion: rows per strip where the two-step pass applies (taller
    strips on wider lattices, 2..16 rows, up to 32 for column tiles), 0 where
    it does not (FP64, a width up
    to 4096 using less than 3/4 of its waves' lanes or a single lane of the last
    wave, steps_per_pass 1); widths above 4096 run as column tiles."""
    import torch
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    cases = [((4096, 4096, "f32"), True), ((2048, 2048, "f32"), True), ((1024, 1024, "f32"), True),
             ((256, 64, "f32"), True), ((4096, 4096, "f64"), False), ((8192, 64, "f64"), False),
             ((300, 64, "f32"), False), ((192, 64, "f32"), True), ((320, 64, "f32"), False),
             ((772, 64, "f32"), False), ((2052, 64, "f32"), False), ((776, 64, "f32"), True),
             ((8200, 64, "f32"), True)]
    for (Lx, Ly, dt), fused in cases:
        lat = xyl.Lattice(Lx, Ly, dtype=dt, schedule=((0, 0.5),), seed=1)
        lat.set_fusion(2)      # a shape tuned earlier in the process may have chosen 1
        sp, rows = lat.fusion()
        say(Lx, Ly, dt, "->", sp, rows)
        assert sp == 2
        if fused:
            assert 1 <= rows <= 32
        else:
            assert rows == 0
        lat.set_fusion(1)
        assert lat.fusion() == (1, 0)
        lat.close()


def _ensemble_run(xyl, specs, fusion, nsteps, every, states=None):
    ens = xyl.Ensemble(specs, dtype="f32")
    ens.set_fusion(fusion)
    if states:
        for r, (th, om) in states.items():
            ens.set_state(r, th, om)
    samples = ens.step(nsteps, every=every)
    out = [ens.get_state(r) for r in range(len(specs))]
    ens.close()
    return samples, out


@pytest.mark.parametrize("fusion", [2, 1])
def test_ensemble_graph_captured_chunks_equal_direct_launches(xyl, fusion):
    """Repeated chunks of batched stepping replayed as graphs (step index from
    a device counter; two-step classes on their streams as parallel branches)
    against the same launches issued directly: samples and states bit for
    bit, across a replica that ends (the tables, hence the graphs, rebuilt),
    sampled and unsampled calls."""
    specs = [workloads.LatticeSpec(1024, 256, schedule=((0, 0.6), (120, 0.2)), seed=8, replica=0, nsteps=10 ** 6),
             workloads.LatticeSpec(512, 384, schedule=((0, 0.5),), seed=8, replica=1, nsteps=10 ** 6),
             workloads.LatticeSpec(192, 192, schedule=((0, 0.8),), seed=8, replica=2, nsteps=130),
             workloads.LatticeSpec(320, 40, schedule=((0, 0.6),), seed=8, replica=3, nsteps=10 ** 6),
             workloads.LatticeSpec(64, 64, schedule=((0, 0.6),), seed=8, replica=4, nsteps=10 ** 6)]
    res = []
    # 2: every repeated chunk as a graph, so the classes' parallel branches are
    # captured too; 1 (the default): only chunks with at most one class (all of
    # them with fusion 1); 0: every launch direct
    for graphs in (2, 1, 0):
        ens = xyl.Ensemble(specs, dtype="f32")
        ens.set_fusion(fusion)
        ens.set_graphs(graphs)
        s1 = ens.step(203, every=25)
        ens.step(40)
        ens.step(40)
        ens.step(40)
        s2 = ens.step(60, every=20)
        res.append((s1, s2, [ens.get_state(r) for r in range(len(specs))]))
        if graphs == 0:
            with pytest.raises(xyl.XylError):
                ens.set_graphs(3)
        ens.close()
    say("graph modes 2 and 1 vs direct, fusion", fusion)
    for other in res[:2]:
        for a, b in zip(other[0], res[2][0]):
            np.testing.assert_array_equal(a, b)
        for a, b in zip(other[1], res[2][1]):
            np.testing.assert_array_equal(a, b)
        for (ta, wa, ka), (tb, wb, kb) in zip(other[2], res[2][2]):
            assert ka == kb
            np.testing.assert_array_equal(ta, tb)
            np.testing.assert_array_equal(wa, wb)


def test_ensemble_autotune_picks_steps_per_pass_without_changing_results(xyl):
    """xyl_ensemble_autotune times the tile launch shapes on scratch copies,
    then the two-step classes against tile steps, and keeps the faster; the
    ensemble's own state is untouched and its results do not change."""
    specs = [workloads.LatticeSpec(1024, 512, schedule=((0, 0.6),), seed=9, replica=0, nsteps=10 ** 6),
             workloads.LatticeSpec(256, 256, schedule=((0, 0.4),), seed=9, replica=1, nsteps=10 ** 6),
             workloads.LatticeSpec(320, 40, schedule=((0, 0.6),), seed=9, replica=2, nsteps=10 ** 6),
             workloads.LatticeSpec(64, 64, schedule=((0, 0.6),), seed=9, replica=3, nsteps=10 ** 6)]
    res = []
    for tune in (True, False):
        ens = xyl.Ensemble(specs, dtype="f32")
        ens.step(5)
        if tune:
            rows, wpb = ens.autotune()
            say("ensemble autotune", rows, wpb, "steps per pass", ens.fusion())
            assert ens.fusion() in (1, 2)
        smp = ens.step(120, every=40)
        res.append((smp, [ens.get_state(r) for r in range(len(specs))]))
        ens.close()
    for a, b in zip(res[0][0], res[1][0]):
        np.testing.assert_array_equal(a, b)
    for (ta, wa, ka), (tb, wb, kb) in zip(res[0][1], res[1][1]):
        assert ka == kb
        np.testing.assert_array_equal(ta, tb)
        np.testing.assert_array_equal(wa, wb)


@pytest.mark.parametrize("mixed", [False, True])
def test_ensemble_two_steps_per_pass_equal_batched_single_steps(xyl, mixed):
    """FP32 replicas on the tile path whose width the two-step pass takes, of
    different shapes, parameters, schedules and step budgets, take batched
    two-step passes between samples (one launch per class of waves per row);
    the others keep one tile launch per step, small ones stay whole-in-LDS.
    The same samples and states as one batched launch per step, bit for bit."""
    specs = [
        workloads.LatticeSpec(1024, 1024, schedule=((0, 0.6), (40, 0.2)), seed=3, replica=0, nsteps=10 ** 6),
        workloads.LatticeSpec(2048, 512, Jx=0.8, h=0.3, schedule=((0, 0.4),), seed=3, replica=1, nsteps=57),
        workloads.LatticeSpec(256, 4096, schedule=((0, 0.9), (30, 0.5, 2), (90, 0.1)), seed=4, replica=2,
                              nsteps=10 ** 6),
    ]
    if mixed:
        # both two-step classes (one and two waves, partial ones included), a
        # width the two-step pass does not take (tile launches alone) and a
        # whole-in-LDS replica
        specs += [workloads.LatticeSpec(512, 384, schedule=((0, 0.5),), seed=5, replica=3, nsteps=10 ** 6),
                  workloads.LatticeSpec(192, 192, schedule=((0, 0.8),), seed=5, replica=4, nsteps=10 ** 6),
                  workloads.LatticeSpec(384, 96, h=0.25, schedule=((0, 0.3),), seed=5, replica=5, nsteps=70),
                  workloads.LatticeSpec(320, 40, schedule=((0, 0.6),), seed=5, replica=6, nsteps=10 ** 6),
                  workloads.LatticeSpec(64, 64, schedule=((0, 0.6),), seed=5, replica=7, nsteps=10 ** 6)]
    rng = np.random.default_rng(11)
    states = {2: (rng.uniform(-np.pi, np.pi, (4096, 256)).astype(np.float32).astype(np.float64),
                  rng.normal(0, 0.5, (4096, 256)).astype(np.float32).astype(np.float64))}
    say("ensemble", [(s.Lx, s.Ly) for s in specs], "mixed", mixed)
    a = _ensemble_run(xyl, specs, 2, 83, 20, states)
    b = _ensemble_run(xyl, specs, 1, 83, 20, states)
    for r in range(len(specs)):
        np.testing.assert_array_equal(a[0][r], b[0][r])
        np.testing.assert_array_equal(a[1][r][0], b[1][r][0])
        np.testing.assert_array_equal(a[1][r][1], b[1][r][1])
        assert a[1][r][2] == b[1][r][2]
    assert a[1][1][2] == 57 and a[1][0][2] == 83


def test_autotune_picks_steps_per_pass_and_leaves_results_alone(xyl):
    """xyl_autotune times single-step shapes and two-step passes on scratch
    copies: the lattice's state is untouched, the choice is reported by
    fusion(), applied to lattices of the same shape created afterwards, and the
    trajectory equals single steps bit for bit whatever it chose."""
    Lx, Ly = 1024, 768          # a shape no other test tunes (the choice is cached per process)
    spec = workloads.LatticeSpec(Lx, Ly, schedule=((0, 0.7), (60, 0.3)), seed=5, replica=2)

    def make():
        lat = xyl.Lattice(Lx, Ly, dtype="f32", schedule=spec.schedule, seed=5, replica=2, **spec.params())
        lat.init_random()
        lat.step(10)
        return lat

    a = make()
    before = a.get_state()
    launch = a.autotune()
    after = a.get_state()
    np.testing.assert_array_equal(before[0], after[0])
    np.testing.assert_array_equal(before[1], after[1])
    assert before[2] == after[2]
    sp, rows = a.fusion()
    say("autotune: launch", launch, "steps per pass", sp, "rows", rows)
    assert sp in (1, 2) and ((sp == 2 and 1 <= rows <= 16) or (sp == 1 and rows == 0))
    c = xyl.Lattice(Lx, Ly, dtype="f32", schedule=spec.schedule, seed=5)
    assert c.fusion() == (sp, rows) and c.launch() == a.launch()
    c.close()
    a.step(64)
    b = make()
    b.set_fusion(1)
    b.step(64)
    ta, tb = a.get_state(), b.get_state()
    np.testing.assert_array_equal(ta[0], tb[0])
    np.testing.assert_array_equal(ta[1], tb[1])
    a.close()
    b.close()


@pytest.mark.parametrize("Lx,Ly,model", [(448, 33, "xy"), (768, 20, "si"), (256, 8, "xy"), (4096, 12, "xy")])
def test_sampled_runs_on_two_step_passes_equal_single_steps(xyl, Lx, Ly, model):
    """Sampled runs whose spans between samples go through two-step passes (a
    measurement without a step, then the span's steps) equal, bit for bit,
    those of measured single steps and the same steps one at a time; sample
    spans of 4 (one pair of passes), 5 and 10 steps, a partial last wave, the
    Si model, and the trailing sample at the run's last step."""
    if model == "si":
        spec = workloads.si_lattice(Lx, Ly, seed=6, replica=2)
    else:
        spec = workloads.LatticeSpec(Lx, Ly, schedule=((0, 0.9), (30, 0.4)), seed=6, replica=2)
    res = []
    for fusion in (1, 2):
        lat = xyl.Lattice(Lx, Ly, dtype="f32", schedule=spec.schedule, seed=spec.seed, replica=spec.replica,
                          **spec.params())
        lat.set_fusion(fusion)
        if fusion == 2:
            assert lat.fusion()[1] > 0, "the two-step pass applies to this shape"
        lat.init_random()
        s = [lat.step_measured(8, 4), lat.step_measured(23, 5), lat.step_measured(40, 10)]
        res.append((s, lat.get_state()))
        lat.close()
    for a, b in zip(res[0][0], res[1][0]):
        np.testing.assert_array_equal(a, b)
    for a, b in zip(res[0][1], res[1][1]):
        np.testing.assert_array_equal(a, b)
