"""GPU parity of the batched path (ragged lattices, per-lattice constants,
hipGraph replay, autotuner) against the oracle, lattice by lattice."""
import json
import os
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
from parity_util import TOL, gpu_params, max_err, oracle_params, random_state

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def lbm():
    from paper_1802_02369_amd import lbm as m
    return m


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def pack(states):
    """Batch layout (6, n_total) from per-lattice (6, L_i) states."""
    return np.ascontiguousarray(np.concatenate(states, axis=1))


def unpack(f, offsets):
    return [f[:, offsets[i]:offsets[i + 1]] for i in range(len(offsets) - 1)]


def oracle_runs(states, params, steps, workers=16):
    with ThreadPoolExecutor(workers) as ex:
        return list(ex.map(lambda a: oracle.run(a[0], steps, a[1]),
                           zip(states, params)))


RAGGED = [3, 5, 64, 100, 513, 1000, 2049, 7]
PNAMES = ["paper", "odd", "nosource", "linear", "odd", "paper", "odd", "nosource"]
SHAPES = [(2, 8, 4), (4, 5, 2), (2, 16, 8), (2, 1, 1), (8, 12, 2), (8, 32, 4), (1, 12, 1)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("steps", [1, 16, 37])
def test_ragged_batch(shape, steps):
    rng = np.random.default_rng(1000 + steps)
    params = [oracle_params(p, s_e=1.2 + 0.1 * i) for i, p in enumerate(PNAMES)]
    states = [random_state(rng, L, p) for L, p in zip(RAGGED, params)]
    offsets = np.concatenate([[0], np.cumsum(RAGGED)])
    say(f"ragged batch shape={shape} steps={steps}")
    b = lbm().Batch(offsets, [gpu_params(p) for p in params])
    P, K, W = shape
    b.set_tuning(P, K, W)
    f = torch.from_numpy(pack(states)).to(dev())
    b.run(f, steps, use_graph=False)
    got = unpack(f.cpu().numpy(), offsets)
    want = oracle_runs(states, params, steps)
    for i, (g, w) in enumerate(zip(got, want)):
        assert max_err(g, w) < TOL, (i, RAGGED[i], PNAMES[i])


@pytest.mark.parametrize("mixed", [False, True])
def test_batch_bitwise_equals_single_lattice(mixed):
    """A lattice advanced inside a batch (any neighbours, any tile shape)
    ends bitwise equal to the same lattice advanced alone: the kernels share
    one rounding sequence per node-update.  mixed: the batch also holds
    lattices with linear equilibria (the per-lattice equilibrium switch)."""
    rng = np.random.default_rng(5)
    lens = [6007, 100, 4099, 3]
    names = ["paper", "linear" if mixed else "odd", "odd", "paper"]
    params = [oracle_params(p) for p in names]
    states = [random_state(rng, L, p, amp=0.1, u=0.05, ds=0.1)
              for L, p in zip(lens, params)]
    offsets = np.concatenate([[0], np.cumsum(lens)])
    say(f"batch vs single bitwise mixed={mixed}")
    singles = []
    for s, p in zip(states, params):
        lat = lbm().Lattice(s.shape[1], gpu_params(p))
        f = torch.from_numpy(s.copy()).to(dev())
        lat.step(f, 29)
        singles.append(f.cpu().numpy())
        assert np.isfinite(singles[-1]).all()
    for shape in [(2, 8, 4), (8, 32, 4), (4, 5, 2)]:
        b = lbm().Batch(offsets, [gpu_params(p) for p in params])
        b.set_tuning(*shape)
        f = torch.from_numpy(pack(states)).to(dev())
        b.run(f, 29, use_graph=False)
        for i, g in enumerate(unpack(f.cpu().numpy(), offsets)):
            assert np.array_equal(g, singles[i]), (shape, i)


def _groups_by_length(lens, shapes):
    """Assignment by length: the widest shape whose tile is at most a
    quarter of the lattice, else the narrowest."""
    import numpy as np
    widths = [P * (62 * W + 2) for P, K, W in shapes]
    order = sorted(range(len(shapes)), key=lambda g: -widths[g])
    out = []
    for L in lens:
        g = next((g for g in order if 4 * widths[g] <= L), order[-1])
        out.append(g)
    return np.asarray(out, dtype=np.int32)


@pytest.mark.parametrize("steps", [1, 2, 37])
def test_shape_groups_bitwise_equal_single_shape(steps):
    """Lattices split over three tile shapes, each group a launch sequence
    on its own stream: the state equals the single-shape run bit for bit
    (every shape rounds the same), for direct launches and graph replays;
    steps = 1 takes the odd-launch path (each group's tiles copied back from
    the workspace state)."""
    rng = np.random.default_rng(17)
    lens = [9000, 60, 3001, 700, 20000, 5, 2048, 130, 4096, 11111, 640, 333]
    names = ["paper", "odd", "linear", "paper", "odd", "nosource",
             "paper", "odd", "paper", "fluid", "odd", "paper"]
    params = [oracle_params(p) for p in names]
    states = [random_state(rng, L, p, amp=0.1, u=0.05, ds=0.1)
              for L, p in zip(lens, params)]
    offsets = np.concatenate([[0], np.cumsum(lens)])
    say(f"shape groups steps={steps}")
    b = lbm().Batch(offsets, [gpu_params(p) for p in params])
    b.set_tuning(4, 16, 4)
    f0 = torch.from_numpy(pack(states)).to(dev())
    ref = f0.clone()
    b.run(ref, steps, use_graph=False)
    shapes = [(8, 40, 4), (4, 16, 4), (2, 8, 1)]
    b.set_groups(shapes, _groups_by_length(lens, shapes))
    got_shapes, go = b.get_groups()
    assert got_shapes == shapes and go is not None
    f = f0.clone()
    b.run(f, steps, use_graph=False)
    assert torch.equal(f, ref)
    for rep in range(3):
        f = f0.clone()
        _ = (f * 2).sum().item()
        b.run(f, steps, use_graph=True)
        torch.cuda.synchronize()
        assert torch.equal(f, ref), rep
    # back to one shape
    b.set_groups([])
    f = f0.clone()
    b.run(f, steps, use_graph=False)
    assert torch.equal(f, ref)
    want = oracle_runs(states, params, steps)
    for i, (g, w) in enumerate(zip(unpack(ref.cpu().numpy(), offsets), want)):
        assert max_err(g, w) < TOL, i


def test_graph_replays_match_direct_launches():
    """The captured graph, replayed several times with eager work and
    synchronisations in between, gives bitwise the direct launches' result."""
    rng = np.random.default_rng(7)
    params = [oracle_params(p, s_e=1.3 + 0.05 * i) for i, p in enumerate(PNAMES)]
    states = [random_state(rng, L, p) for L, p in zip(RAGGED, params)]
    offsets = np.concatenate([[0], np.cumsum(RAGGED)])
    b = lbm().Batch(offsets, [gpu_params(p) for p in params])
    b.set_tuning(2, 8, 4)
    f0 = torch.from_numpy(pack(states)).to(dev())
    ref = f0.clone()
    b.run(ref, 33, use_graph=False)
    for rep in range(4):
        f = f0.clone()
        _ = (f * 2).sum().item()  # eager work between replays
        b.run(f, 33, use_graph=True)
        torch.cuda.synchronize()
        assert torch.equal(f, ref), rep
    # a different step count re-captures
    f = f0.clone()
    b.run(f, 34, use_graph=True)
    ref2 = f0.clone()
    b.run(ref2, 34, use_graph=False)
    assert torch.equal(f, ref2)


def test_batch_diagnostics_and_equilibrium():
    rng = np.random.default_rng(11)
    params = [oracle_params(p) for p in PNAMES]
    fields = []
    for L, p in zip(RAGGED, params):
        rho = p.rho0 * (1 + 0.1 * rng.uniform(-1, 1, L))
        fields.append((rho, rho * 0.05 * rng.uniform(-1, 1, L),
                       rho * (p.s0 + 0.1 * rng.uniform(-1, 1, L))))
    offsets = np.concatenate([[0], np.cumsum(RAGGED)])
    b = lbm().Batch(offsets, [gpu_params(p) for p in params])
    cat = [torch.from_numpy(np.concatenate([x[k] for x in fields])).to(dev())
           for k in range(3)]
    f = b.equilibrium(*cat)
    got = unpack(f.cpu().numpy(), offsets)
    for i, (fl, p) in enumerate(zip(fields, params)):
        want = oracle.init(*fl, p)
        assert max_err(got[i], want) < TOL, i
    d = b.diagnostics(f)
    for i, p in enumerate(params):
        np.testing.assert_allclose(d[i], oracle.diagnostics(got[i], p),
                                   rtol=1e-12, atol=1e-14)


def test_batched_config_subset():
    """4096 lattices, lengths log-uniform in [512, 16384], amplitudes up to
    0.3, s_e inside the stable range, 5000 steps in one graph launch: a
    seeded 64-lattice subset is run by the oracle.  Checked: the final state
    relative to the state norm (1e-11), and one GPU step from the oracle's
    state at step 4999 against the oracle's step 5000 (1e-12 per field)."""
    from paper_1802_02369_amd import workloads
    cfg = workloads.config_batched()
    bt, steps = cfg["batch"], cfg["steps"]
    say(f"batched config: {bt.n_inst} lattices, {bt.offsets[-1]} nodes, {steps} steps")
    ps = []
    for s_e in bt.s_e:
        p = oracle_params("paper", s_e=float(s_e))
        ps.append(p)
    b = lbm().Batch(bt.offsets, [gpu_params(p) for p in ps])
    fl = bt.fields
    f = b.equilibrium(*[torch.from_numpy(x).to(dev()) for x in (fl.rho, fl.J, fl.zeta)])
    b.run(f, steps, use_graph=True)
    d = b.diagnostics(f)
    assert np.all(d[:, 6] == 0) and np.all(d[:, 7] == 0)
    fin = f.cpu().numpy()
    rng = np.random.default_rng(64)
    sub = np.sort(rng.choice(bt.n_inst, 64, replace=False))
    # the subset's 64 lattices: oracle run to step 4999, then one more step
    init = [oracle.init(*[x[bt.offsets[i]:bt.offsets[i + 1]] for x in (fl.rho, fl.J, fl.zeta)], ps[i])
            for i in sub]
    say("  oracle: 64 lattices x 4999 steps")
    prev = oracle_runs(init, [ps[i] for i in sub], steps - 1)
    last = oracle_runs(prev, [ps[i] for i in sub], 1)
    worst_traj = 0.0
    for k, i in enumerate(sub):
        g = fin[:, bt.offsets[i]:bt.offsets[i + 1]]
        worst_traj = max(worst_traj, np.abs(g - last[k]).max() / np.abs(last[k]).max())
    say(f"  final-state error / state norm over the subset: {worst_traj:.3e}")
    # two correct FP64 trajectories drift apart through the shocks by their
    # rounding (measured 9.8e-13 after 5000 steps)
    assert worst_traj < 1e-11
    # one batched GPU step from the oracle's states at step 4999
    lens = bt.lengths[sub]
    offs = np.concatenate([[0], np.cumsum(lens)])
    bs = lbm().Batch(offs, [gpu_params(ps[i]) for i in sub])
    bs.set_tuning(**{k: v for k, v in b.get_tuning().items() if k != "kernel"})
    g = torch.from_numpy(pack(prev)).to(dev())
    bs.run(g, 1, use_graph=False)
    got = unpack(g.cpu().numpy(), offs)
    worst = max(max_err(got[k], last[k]) for k in range(len(sub)))
    say(f"  one-step error from oracle states (floored metric): {worst:.3e}")
    assert worst < TOL


def test_autotune_restores_state_and_caches(tmp_path):
    rng = np.random.default_rng(3)
    lens = rng.integers(300, 3000, 40)
    offsets = np.concatenate([[0], np.cumsum(lens)])
    params = [oracle_params("paper", s_e=float(s)) for s in rng.uniform(1.2, 1.8, 40)]
    states = [random_state(rng, L, p, amp=0.05, u=0.02, ds=0.05) for L, p in zip(lens, params)]
    b = lbm().Batch(offsets, [gpu_params(p) for p in params])
    f = torch.from_numpy(pack(states)).to(dev())
    f0 = f.clone()
    cache = str(tmp_path / "tune.json")
    t1 = b.autotune(f, probe_steps=16, cache_path=cache)
    assert torch.equal(f, f0)
    entries = json.load(open(cache))
    assert len(entries) == 1
    (key, val), = entries.items()
    assert key.split("/")[1] == "batch"
    # lattices of 300 .. 3000 nodes may run resident: the search timed both
    # modes and stored the one it kept
    assert key.split("/")[-2] == "res" and val["resident"] in (0, 1)
    assert (val["P"], val["K"], val["W"]) == (t1["nodes_per_lane"], t1["steps_per_launch"],
                                             t1["waves_per_group"])
    b2 = lbm().Batch(offsets, [gpu_params(p) for p in params])
    t2 = b2.autotune(f, probe_steps=16, cache_path=cache)
    assert t2 == t1
    assert b2.resident_lattices() == b.resident_lattices() == (40 if val["resident"] else 0)
    g1, g2 = b.get_groups(), b2.get_groups()
    assert g1[0] == g2[0] and (g1[1] is None) == (g2[1] is None)
    if g1[1] is not None:
        assert np.array_equal(g1[1], g2[1]) and "groups" in val
    # the tuned batch still matches the oracle
    b2.run(f, 10)
    got = unpack(f.cpu().numpy(), offsets)
    want = oracle_runs(states, params, 10)
    assert max(max_err(g, w) for g, w in zip(got, want)) < TOL
    # single-lattice autotuner
    n = 5000
    po = oracle_params("paper")
    s0 = random_state(rng, n, po)
    lat = lbm().Lattice(n, gpu_params(po))
    g = torch.from_numpy(s0).to(dev())
    t = lat.autotune(g, probe_steps=16, cache_path=cache)
    assert torch.equal(g, torch.from_numpy(s0).to(dev()))
    assert len(json.load(open(cache))) == 2
    lat.step(g, 9)
    assert max_err(g.cpu().numpy(), oracle.run(s0, 9, po)) < TOL, t


def test_autotune_shape_groups_wide_lengths(tmp_path):
    """Lengths spread over 300 .. 30000 nodes (log-uniform): the autotuner
    times single shapes and the best modelled grouping; whatever it keeps,
    the state is restored, the cache round-trips, and the tuned run equals
    the run of its single shape bit for bit."""
    rng = np.random.default_rng(8)
    lens = np.round(np.exp(rng.uniform(np.log(300), np.log(30000), 160))).astype(int)
    offsets = np.concatenate([[0], np.cumsum(lens)])
    params = [oracle_params("paper", s_e=float(s)) for s in rng.uniform(1.2, 1.8, len(lens))]
    states = [random_state(rng, L, p, amp=0.05, u=0.02, ds=0.05) for L, p in zip(lens, params)]
    say(f"autotune groups, {len(lens)} lattices, {offsets[-1]} nodes")
    b = lbm().Batch(offsets, [gpu_params(p) for p in params])
    f0 = torch.from_numpy(pack(states)).to(dev())
    f = f0.clone()
    cache = str(tmp_path / "tune.json")
    t = b.autotune(f, probe_steps=24, cache_path=cache)
    assert torch.equal(f, f0)
    shapes, go = b.get_groups()
    say(f"  tuning {t}, groups {shapes}")
    entry = next(iter(json.load(open(cache)).values()))
    assert ("groups" in entry) == bool(shapes)
    b.run(f, 13, use_graph=True)
    single = lbm().Batch(offsets, [gpu_params(p) for p in params])
    single.set_tuning(t["nodes_per_lane"], t["steps_per_launch"], t["waves_per_group"])
    g = f0.clone()
    single.run(g, 13, use_graph=False)
    assert torch.equal(f, g)
    b2 = lbm().Batch(offsets, [gpu_params(p) for p in params])
    b2.autotune(f0.clone(), probe_steps=24, cache_path=cache)
    s2, go2 = b2.get_groups()
    assert s2 == shapes and ((go is None and go2 is None) or np.array_equal(go, go2))


# Lengths around every boundary of the resident layout (496 nodes per
# wavefront at P = 8, lattices of 16 .. 5952 nodes in workgroups of twelve
# wavefronts): the limits, one node past a wavefront (the last holds fewer
# than P nodes, so the periodic copy reaches back into the wavefront before
# it), full wavefronts, and lattices that stay on tiles (3, 15, 5953, 9000).
RES_LENS = [16, 5952, 497, 15, 17, 496, 499, 992, 995, 1000, 3969, 30, 1488,
            2500, 3, 503, 9000, 24, 1991, 3001, 5953, 4961, 5457]
# (section-8 equilibria only: a batch that selects the equilibria per
# lattice runs every lattice on tiles)
RES_NAMES = ["paper", "odd", "nosource", "paper", "nosource", "odd", "paper",
             "odd", "odd", "nosource", "paper", "odd", "paper", "nosource",
             "odd", "paper", "odd", "paper", "odd", "nosource", "paper", "odd",
             "nosource"]


@pytest.mark.parametrize("steps", [1, 2, 3, 4, 5, 37, 100])
def test_resident_bitwise_equals_tiles(steps):
    """Resident lattices (all the steps of a run in one launch, state in
    registers) end bitwise equal to the tiled run of the same batch, for
    direct launches and graph replays, with and without shape groups, and
    match the oracle.  The groups put one shape at K = 1, whose odd step
    counts end in the workspace state and are copied back tile by tile
    while the other group ends in place."""
    rng = np.random.default_rng(300 + steps)
    params = [oracle_params(p) for p in RES_NAMES]
    states = [random_state(rng, L, p, amp=0.1, u=0.05, ds=0.1)
              for L, p in zip(RES_LENS, params)]
    offsets = np.concatenate([[0], np.cumsum(RES_LENS)])
    say(f"resident vs tiles steps={steps}")
    b = lbm().Batch(offsets, [gpu_params(p) for p in params])
    b.set_tuning(4, 16, 4)
    b.set_resident(0)
    assert b.resident_lattices() == 0
    f0 = torch.from_numpy(pack(states)).to(dev())
    ref = f0.clone()
    b.run(ref, steps, use_graph=False)
    b.set_resident(1)
    want_res = sum(lbm().RESIDENT_MIN <= L <= lbm().RESIDENT_MAX for L in RES_LENS)
    assert b.resident_lattices() == want_res == len(RES_LENS) - 4
    f = f0.clone()
    b.run(f, steps, use_graph=False)
    bad = [i for i, (g, r) in enumerate(zip(unpack(f.cpu().numpy(), offsets),
                                             unpack(ref.cpu().numpy(), offsets)))
           if not np.array_equal(g, r)]
    assert not bad, [(i, RES_LENS[i]) for i in bad]
    for rep in range(3):
        f = f0.clone()
        _ = (f * 2).sum().item()  # eager work between replays
        b.run(f, steps, use_graph=True)
        torch.cuda.synchronize()
        assert torch.equal(f, ref), rep
    shapes = [(8, 40, 4), (2, 1, 1)]
    go = _groups_by_length(RES_LENS, shapes)
    assert set(go) == {0, 1}
    b.set_groups(shapes, go)
    f = f0.clone()
    b.run(f, steps, use_graph=True)
    assert torch.equal(f, ref)
    want = oracle_runs(states, params, steps)
    for i, (g, w) in enumerate(zip(unpack(ref.cpu().numpy(), offsets), want)):
        assert max_err(g, w) < TOL, (i, RES_LENS[i], RES_NAMES[i])


def test_resident_only_batch_and_mode_switch():
    """A batch whose lattices are all resident (no tiles at all) equals its
    tiled run bitwise for even and odd step counts and through a graph; the
    autotuner leaves it untouched; switching the mode re-captures."""
    rng = np.random.default_rng(41)
    lens = rng.integers(16, lbm().RESIDENT_MAX + 1, 64)
    params = [oracle_params("paper", s_e=float(s)) for s in rng.uniform(1.2, 1.8, 64)]
    states = [random_state(rng, L, p, amp=0.1, u=0.05, ds=0.1)
              for L, p in zip(lens, params)]
    offsets = np.concatenate([[0], np.cumsum(lens)])
    say(f"resident-only batch, {offsets[-1]} nodes")
    b = lbm().Batch(offsets, [gpu_params(p) for p in params])
    assert b.resident_lattices() == 64
    f0 = torch.from_numpy(pack(states)).to(dev())
    g = f0.clone()
    b.autotune(g, probe_steps=8)
    assert torch.equal(g, f0)
    for steps in (1, 6, 7):
        b.set_resident(0)
        ref = f0.clone()
        b.run(ref, steps, use_graph=True)
        b.set_resident(1)
        for use_graph in (False, True):
            f = f0.clone()
            b.run(f, steps, use_graph=use_graph)
            assert torch.equal(f, ref), (steps, use_graph)
    with pytest.raises(lbm().LBMError):
        b.set_resident(2)
    # one lattice with linear equilibria puts the whole batch on tiles
    mixed = [gpu_params(p) for p in params]
    mixed[5] = gpu_params(oracle_params("linear"))
    assert lbm().Batch(offsets, mixed).resident_lattices() == 0


def test_resident_run_longer_than_one_launch():
    """A run of more steps than one resident launch holds (65536) chains
    launches and equals the tiled run bitwise."""
    rng = np.random.default_rng(77)
    lens = [16, 100, 997]
    params = [oracle_params(p) for p in ("paper", "odd", "nosource")]
    states = [random_state(rng, L, p, amp=0.02, u=0.01, ds=0.02)
              for L, p in zip(lens, params)]
    offsets = np.concatenate([[0], np.cumsum(lens)])
    steps = (1 << 16) + 3
    say(f"resident run of {steps} steps")
    b = lbm().Batch(offsets, [gpu_params(p) for p in params])
    b.set_tuning(2, 16, 1)
    f0 = torch.from_numpy(pack(states)).to(dev())
    b.set_resident(0)
    ref = f0.clone()
    b.run(ref, steps, use_graph=False)
    b.set_resident(1)
    assert b.resident_lattices() == 3
    f = f0.clone()
    b.run(f, steps, use_graph=False)
    assert torch.isfinite(ref).all()
    assert torch.equal(f, ref)


def test_resident_check_finite_per_launch():
    """LBM_CHECK_FINITE on a resident lattice of a run longer than one
    resident launch: a NaN in its state is reported after the first launch's
    65536 steps, naming that lattice; without the NaN the run is bitwise the
    unchecked one."""
    import re
    rng = np.random.default_rng(78)
    lens = [40, 300]
    params = [oracle_params(p) for p in ("paper", "odd")]
    states = [random_state(rng, L, p, amp=0.02, u=0.01, ds=0.02)
              for L, p in zip(lens, params)]
    offsets = np.concatenate([[0], np.cumsum(lens)])
    steps = (1 << 16) + 5
    gp = [gpu_params(p) for p in params]
    gp[1].flags = lbm().LBM_CHECK_FINITE
    b = lbm().Batch(offsets, gp)
    assert b.resident_lattices() == 2
    f0 = torch.from_numpy(pack(states)).to(dev())
    ref = f0.clone()
    lbm().Batch(offsets, [gpu_params(p) for p in params]).run(ref, steps, use_graph=False)
    f = f0.clone()
    b.run(f, steps, use_graph=False)
    assert torch.equal(f, ref)
    f = f0.clone()
    f[2, int(offsets[1]) + 11] = float("nan")
    say("resident check after one launch")
    with pytest.raises(lbm().LBMError) as e:
        b.run(f, steps, use_graph=False)
    assert e.value.code == lbm().LBM_ENONFINITE
    m = re.search(r"after (\d+) time steps: first failing lattice (\d+)", str(e.value))
    assert m and int(m.group(1)) == 1 << 16 and int(m.group(2)) == 1, str(e.value)


@pytest.mark.parametrize("seed", range(6))
def test_resident_random_batches(seed):
    """Seeded random batches (lengths 3 .. 7000, some of them resident,
    random step counts, the section-8 parameter sets): resident and tiled
    runs bitwise equal."""
    rng = np.random.default_rng(9000 + seed)
    n = int(rng.integers(1, 40))
    lens = [int(x) for x in np.exp(rng.uniform(np.log(3), np.log(7000), n)).round()]
    names = [("paper", "odd", "nosource")[int(i)] for i in rng.integers(0, 3, n)]
    params = [oracle_params(p, s_e=float(s)) for p, s in zip(names, rng.uniform(1.1, 1.8, n))]
    states = [random_state(rng, L, p, amp=0.05, u=0.02, ds=0.05)
              for L, p in zip(lens, params)]
    offsets = np.concatenate([[0], np.cumsum(lens)])
    steps = int(rng.integers(1, 120))
    shape = [(8, 40, 4), (4, 24, 4), (2, 16, 4), (8, 8, 2)][seed % 4]
    say(f"random batch seed={seed}: {n} lattices, {steps} steps, shape {shape}")
    b = lbm().Batch(offsets, [gpu_params(p) for p in params])
    b.set_tuning(*shape)
    f0 = torch.from_numpy(pack(states)).to(dev())
    b.set_resident(0)
    ref = f0.clone()
    b.run(ref, steps, use_graph=False)
    b.set_resident(1)
    f = f0.clone()
    b.run(f, steps, use_graph=bool(seed & 1))
    assert torch.isfinite(ref).all()
    assert torch.equal(f, ref), (b.resident_lattices(), lens)
