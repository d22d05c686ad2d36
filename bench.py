"""Benchmark of the coupled D1Q3Q3 lattice Boltzmann hot path on one MI355X.

One bench step = one full run of the single-lattice workload: N = 2^24 nodes,
FP64, progressive wave of amplitude 0.2 steepening into shocks, 2000 time
steps from its equilibrium initial state (synthetic, seeded).  The timed
region holds exactly the --steps runs (each bracketed by device
synchronisation; the reset of the state to the initial field between runs is
outside the timed region).  Prints one JSON line on stdout; progress goes to
stderr.

Extra keys: "plain" (the one-step-per-launch kernel on the same lattice),
"batched" and "adjoint" (the batched and gradient paths, when built), each
with its own throughput, so that batched and fwd+adjoint throughput can be
compared against the plain single-lattice kernel on the same GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
FP64_PEAK_TFLOPS = 78.6        # MI355X vector FP64, published (FMA = 2 flops)
# Vector ALU issue: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3 T lane
# instructions/s, one wave64 instruction per SIMD every 4 clocks; every FP64
# add, mul, FMA or transcendental takes one such slot (78.6 TFLOP/s / 2).
LANE_INSTR_PEAK_T = 256 * 4 * 16 * 2.4e9 / 1e12
BYTES_PER_NODE_LAUNCH = 96.0   # read 6 + write 6 FP64 per node per launch
METRIC = ("node-updates/s (GLUPS) FP64: plain vs batched vs fwd+adjoint; "
          "% HBM roofline")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--lbm-steps", type=int, default=2000,
                    help="time steps per bench step (the workload has 2000)")
    ap.add_argument("--n", type=int, default=1 << 24)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--only", type=str, default=None,
                    help="comma list of extra legs to run: plain,batched,"
                         "adjoint,batched_adjoint")
    ap.add_argument("--instr-per-node", type=float, default=None,
                    help="override the FP64 instructions per node-update")
    ap.add_argument("--tuning", type=str, default=None,
                    help="P,K,W of the blocked kernel (default: library's)")
    ap.add_argument("--batched-tuning", type=str, default=None,
                    help="P,K,W of the batched leg (default: its autotuner)")
    ap.add_argument("--counter-run", type=str, default=None,
                    choices=["single", "batched", "adjoint", "batched_adjoint"],
                    help="run one unit of work of this leg only (for "
                         "rocprofv3 --pmc) and print its useful units")
    ap.add_argument("--counter-steps", type=int, default=None,
                    help="time steps of a single or batched counter run "
                         "(default: two launches of the tile shape's K)")
    ap.add_argument("--summarize-counters", nargs="+", default=None,
                    metavar=("LEG", "RUN_JSON"),
                    help="LEG RUN_JSON DIR...: add the totals of the --pmc "
                         "passes in DIR... to profiles/counters_legs.json")
    return ap.parse_args()


LEG_COUNTERS = os.path.join(ROOT, "profiles", "counters_legs.json")
# Host threads for the oracle's multi-core baselines: the host share of one
# GPU on the boxes this runs on (16), or fewer where the machine has fewer.
CPU_THREADS = min(16, os.cpu_count() or 1)
# Algorithmic HBM bytes of one forward node-step of a gradient without
# register blocking: forward 96 + recompute 96 + reverse 144 (read f(t) and
# fbar(t+1), write fbar(t)).  The blocked kernels keep the state and fbar in
# registers for K steps and move a fraction of it, so their rate can exceed
# 8 TB/s on this basis.
GRAD_BYTES_PER_NODE_STEP = 336.0
GRAD_BYTES_BASIS = ("bytes per forward node-step of the one-step gradient "
                    "(no register blocking); the blocked kernels move fewer, "
                    "see measured_gbs")


def source_code(text: str) -> str:
    """A source file's code: comments removed, whitespace runs collapsed
    (the kernels' sources hold no comment markers inside string literals)."""
    import re
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return re.sub(r"\s+", " ", text).strip()


def source_hash(files) -> str:
    """Hash of the kernel sources' code; counter figures taken on other code
    are not reported (comments do not count)."""
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_1802_02369_amd", "csrc", f)) as fh:
            h.update(source_code(fh.read()).encode())
    return h.hexdigest()[:16]


def leg_key(leg: str, tuning=None) -> str:
    """Key of a leg's counter totals: tiled legs per tile shape (+res: with
    resident lattices)."""
    if not tuning:
        return leg
    return f"{leg}@{tuning['nodes_per_lane']},{tuning['steps_per_launch']}," \
           f"{tuning['waves_per_group']}" + ("+res" if tuning.get("resident") else "")


def leg_counters(leg: str, tuning=None):
    """Counter totals of one counter run of a leg (rocprofv3 --pmc,
    summarised by --summarize-counters), or None if absent or taken on
    other sources."""
    if not os.path.exists(LEG_COUNTERS):
        return None
    with open(LEG_COUNTERS) as fh:
        rec = json.load(fh)
    e = rec.get("legs", {}).get(leg_key(leg, tuning))
    if e is None or e.get("source_hash") != source_hash(e.get("source_files", [])):
        return None
    return e


def leg_roofline(leg: str, units_per_s: float, alg_bytes_per_unit: float,
                 unit: str, tuning=None, bytes_basis: str | None = None):
    """Roofline object of an extra leg: the vector-ALU issue fraction from
    the counted FP64 instructions per useful unit (every kernel of the leg,
    halo and recomputation included), and the HBM fraction of the
    algorithmic bytes per unit against 8 TB/s (bytes_basis: what those bytes
    count, when not the leg's own kernels); the counted HBM bytes per unit
    and their fraction of 8 TB/s beside them."""
    c = leg_counters(leg, tuning)
    hbm = alg_bytes_per_unit * units_per_s / 1e9
    roof = {"bound": "alu", "unit": "T FP64 instr/s", "peak": LANE_INSTR_PEAK_T,
            "achieved": None, "frac": None, "traffic": None,
            "per": unit,
            "hbm": {"algorithmic_bytes_per_unit": alg_bytes_per_unit,
                    "achieved": hbm, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": hbm / HBM_PEAK_GBS},
            "counters_current": c is not None}
    if bytes_basis:
        roof["hbm"]["basis"] = bytes_basis
    if c is not None:
        # algorithmic: per computed node-update where the tiles' work is
        # known (the arithmetic of one node-update), else per useful unit
        # (halo and recomputation included)
        fi = c["fp64_instr"] / (c.get("computed_units") or c["units"])
        roof["fp64_instr_per_unit"] = fi
        roof["fp64_instr_per_unit_basis"] = ("computed node-update"
                                             if c.get("computed_units") else unit)
        roof["achieved"] = fi * units_per_s / 1e12
        roof["frac"] = roof["achieved"] / LANE_INSTR_PEAK_T
        ff = c["flops"] / (c.get("computed_units") or c["units"])
        roof["flops"] = {"per_unit": ff, "achieved": ff * units_per_s / 1e12,
                         "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": ff * units_per_s / 1e12 / FP64_PEAK_TFLOPS}
        # every VALU instruction the leg issues (halo, recomputation, moves)
        # over the issue peak: how busy the SIMDs are
        roof["valu_issue_frac"] = (c["valu_instr"] / c["units"] * units_per_s
                                   / (LANE_INSTR_PEAK_T * 1e12))
        if c.get("fetch_bytes") is not None and c.get("write_bytes") is not None:
            roof["traffic"] = (c["fetch_bytes"] + c["write_bytes"]) / c["units"]
            roof["traffic_unit"] = f"measured HBM bytes per {unit}"
            roof["hbm"]["measured_gbs"] = roof["traffic"] * units_per_s / 1e9
            roof["hbm"]["measured_frac"] = roof["hbm"]["measured_gbs"] / HBM_PEAK_GBS
        roof["wave_cycle_fractions"] = c.get("wave_cycle_fractions")
    return roof


def _no_nan(x):
    """The object with every non-finite float replaced by null (the line
    stays strict JSON)."""
    if isinstance(x, float) and not math.isfinite(x):
        return None
    if isinstance(x, dict):
        return {k: _no_nan(v) for k, v in x.items()}
    if isinstance(x, (list, tuple)):
        return [_no_nan(v) for v in x]
    return x


def split_steps(nsteps: int, K: int) -> list:
    """Steps per launch as the library splits a run (an even number of
    launches of K or fewer steps)."""
    L = -(-nsteps // K)
    if L % 2 and nsteps > L:
        L += 1
    return [nsteps // L + (1 if i < nsteps % L else 0) for i in range(L)]


def time_runs(fn, reset, runs: int, torch, stream):
    """Total milliseconds of `runs` calls of fn, each bracketed by a device
    synchronisation; HIP events on the stream the kernels run on."""
    total = 0.0
    for _ in range(runs):
        reset()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        torch.cuda.synchronize()
        total += e0.elapsed_time(e1)
    return total


def cpu_baseline(n: int, min_s: float = 12.0, max_steps: int = 20):
    """The oracle (single thread, as it stands) on a bounded sample of the
    same workload: whole time steps of the full N = 2^24 lattice, about
    min_s seconds of them (one step timed first to size the rest, at most
    max_steps in all)."""
    import numpy as np  # noqa: F401

    import oracle
    from paper_1802_02369_amd import workloads
    cfg = workloads.config_large(n=n)
    fl = cfg["fields"]
    s_psi, s_eps = oracle.coupled_rates(cfg["s_e"])
    p = oracle.Params(s_e=cfg["s_e"], s_psi=s_psi, s_eps=s_eps)
    f = oracle.init(fl.rho, fl.J, fl.zeta, p)
    t0 = time.perf_counter()
    f = oracle.run(f, 1, p)
    t1 = time.perf_counter() - t0
    more = max(0, min(max_steps - 1, int(math.ceil(min_s / t1)) - 1))
    if more:
        oracle.run(f, more, p)
    dt = time.perf_counter() - t0
    steps = 1 + more
    return {"value": n * steps / dt / 1e9, "unit": "GLUPS", "cores": 1,
            "kind": "oracle",
            "sample": f"{steps} time steps of the N={n} lattice "
                      f"({n * steps:.3g} node-updates, {dt:.1f} s, 1 thread)"}


def _dev_fields(torch, fl, dev):
    return [torch.from_numpy(x).to(dev) for x in (fl.rho, fl.J, fl.zeta)]


def _oracle_params(s_e: float):
    import oracle
    s_psi, s_eps = oracle.coupled_rates(s_e)
    return oracle.Params(s_e=s_e, s_psi=s_psi, s_eps=s_eps)


def _on_threads(fn, items, threads):
    """fn over items on `threads` host threads (the oracle's ctypes calls
    release the interpreter lock, so they run in parallel)."""
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(threads) as ex:
        return list(ex.map(fn, items))


def cpu_baseline_batched(min_s: float = 10.0, n_sample: int = 64):
    """The oracle on the host's cores, one lattice per thread: a seeded
    sample of n_sample lattices of the 4096-lattice workload, each advanced
    the same number of steps (sized from one step of each to about min_s of
    wall time)."""
    import numpy as np

    import oracle
    from paper_1802_02369_amd import workloads
    bt = workloads.config_batched()["batch"]
    sub = np.sort(np.random.default_rng(2024).choice(bt.n_inst, n_sample,
                                                     replace=False))
    lat = []
    for i in sub:
        x = bt.instance(int(i))
        p = _oracle_params(float(bt.s_e[i]))
        lat.append((oracle.init(x.rho, x.J, x.zeta, p), p))
    nodes = int(sum(f.shape[1] for f, _ in lat))
    t0 = time.perf_counter()
    _on_threads(lambda a: oracle.run(a[0], 1, a[1]), lat, CPU_THREADS)
    probe = time.perf_counter() - t0
    steps = max(1, int(min_s / max(probe, 1e-6)))
    t0 = time.perf_counter()
    _on_threads(lambda a: oracle.run(a[0], steps, a[1]), lat, CPU_THREADS)
    dt = time.perf_counter() - t0
    return {"value": nodes * steps / dt / 1e9, "unit": "GLUPS",
            "cores": CPU_THREADS, "kind": "oracle",
            "sample": f"{n_sample} seeded lattices of the batch ({nodes} nodes), "
                      f"{steps} steps each, {dt:.1f} s on {CPU_THREADS} threads "
                      "(one lattice per thread at a time)"}


def cpu_baseline_adjoint(min_s: float = 8.0):
    """The oracle's gradient (checkpointed forward, recompute, adjoint of
    each step, initialisation adjoint) and its tangent-linear directional
    derivative, one thread each, on the N = 8192 gradient workload over a
    shortened run (steps sized from a 10-step probe to about min_s each;
    checkpoints every ~sqrt(steps))."""
    import numpy as np

    import oracle
    from paper_1802_02369_amd import workloads
    cfg = workloads.config_adjoint()
    n, fl = cfg["n"], cfg["fields"]
    p = _oracle_params(cfg["s_e"])
    tgt = np.ones(n)
    out = {}
    for kind in ("gradient", "tlm"):
        def run(steps):
            if kind == "gradient":
                oracle.gradient(fl.rho, fl.J, fl.zeta, steps, tgt, p,
                                ckpt=max(1, int(round(math.sqrt(steps)))))
            else:
                oracle.directional(fl.rho, fl.J, fl.zeta, np.ones(n), np.zeros(n),
                                   np.zeros(n), np.zeros(3), steps, tgt, p)
        t0 = time.perf_counter()
        run(10)
        probe = (time.perf_counter() - t0) / 10
        steps = max(10, int(min_s / probe))
        t0 = time.perf_counter()
        run(steps)
        dt = time.perf_counter() - t0
        out[kind] = (n * steps / dt / 1e9, steps, dt)
    g, steps, dt = out["gradient"]
    t, tsteps, tdt = out["tlm"]
    return {"value": g, "unit": "G forward node-steps/s (whole gradient)",
            "cores": 1, "kind": "oracle",
            "sample": f"gradient of the N={n} workload over {steps} steps "
                      f"(checkpoints every {max(1, int(round(math.sqrt(steps))))}), "
                      f"{dt:.1f} s, 1 thread",
            "tangent_linear": {"value": t, "unit": "G node-steps/s",
                               "sample": f"directional derivative over {tsteps} "
                                         f"steps, {tdt:.1f} s, 1 thread"}}


def cpu_baseline_batched_adjoint(min_s: float = 10.0, n_sample: int = 32):
    """The oracle's gradient lattice by lattice on the host's cores: a seeded
    sample of n_sample lattices of the 1024-lattice gradient workload over a
    shortened run (steps sized from a 4-step probe to about min_s of wall
    time, checkpoints every 63 as in the workload)."""
    import numpy as np

    import oracle
    from paper_1802_02369_amd import workloads
    cfg = workloads.config_batched_adjoint()
    bt, ck = cfg["batch"], cfg["ckpt"]
    sub = np.sort(np.random.default_rng(2025).choice(bt.n_inst, n_sample,
                                                     replace=False))
    items = [(bt.instance(int(i)), _oracle_params(float(bt.s_e[i]))) for i in sub]
    nodes = int(sum(len(x.rho) for x, _ in items))

    def run(steps):
        _on_threads(lambda a: oracle.gradient(a[0].rho, a[0].J, a[0].zeta, steps,
                                              np.ones(len(a[0].rho)), a[1],
                                              ckpt=ck),
                    items, CPU_THREADS)
    t0 = time.perf_counter()
    run(4)
    probe = (time.perf_counter() - t0) / 4
    steps = max(4, int(min_s / probe))
    t0 = time.perf_counter()
    run(steps)
    dt = time.perf_counter() - t0
    return {"value": nodes * steps / dt / 1e9,
            "unit": "G forward node-steps/s (whole gradient)",
            "cores": CPU_THREADS, "kind": "oracle",
            "sample": f"{n_sample} seeded lattices ({nodes} nodes) over {steps} "
                      f"steps, checkpoints every {ck}, {dt:.1f} s on "
                      f"{CPU_THREADS} threads (one lattice per thread at a time)"}


def _batch_params(lbm, bt):
    params = []
    for s_e in bt.s_e:
        s_psi, s_eps, _ = lbm.coupled_rates(float(s_e))
        params.append(lbm.Params(s_e=float(s_e), s_psi=s_psi, s_eps=s_eps))
    return params


# device copy of known size in every counter run, larger than any other
# copy those runs make (the summary takes the largest copy dispatch)
CALIB_BYTES = 2 << 30


def calibration_copy(torch):
    """One device-to-device copy of CALIB_BYTES (the runtime's copy kernel):
    its FETCH_SIZE and WRITE_SIZE calibrate the HBM byte counters."""
    a = torch.ones(CALIB_BYTES // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b


def lattice_lane_nodes(L: int, P: int, K: int, W: int) -> int:
    """Lane-nodes a lattice of L nodes computes per step with tile shape
    (P, K, W): its tiles, each with the wavefronts its nodes and halos need
    (as the library's tiles run them)."""
    H = 2 * K
    out = P * (62 * W + 2) - 2 * H
    s, first = 0, 0
    while first < L:
        need = (L - first) + 2 * H - 2 * P
        nw = max(1, min(W, -(-need // (62 * P))))
        s += 64 * P * nw
        first += out
    return s


RES_P, RES_WAVE_NODES = 8, 62 * 8   # resident layout: 8 nodes per lane


def batch_split(lbm, lens, resident_on: bool):
    """Lattices of a section-8 batch that run resident (all the steps of a
    run in one launch) and those on tiles, as the library splits them."""
    import numpy as np
    lens = np.asarray(lens)
    res = (lens >= lbm.RESIDENT_MIN) & (lens <= lbm.RESIDENT_MAX) & bool(resident_on)
    return res


def batch_computed(lens, res, P, K, W) -> int:
    """Lane-nodes per step of a batch: the tiled lattices' tiles (shape P, K,
    W) and the resident lattices' wavefronts (64 x 8 lane-nodes each)."""
    s = 0
    for L, r in zip(lens, res):
        L = int(L)
        s += (64 * RES_P * -(-L // RES_WAVE_NODES) if r
              else lattice_lane_nodes(L, P, K, W))
    return s


def counter_run_single(torch, lbm, workloads, steps: int):
    """One run of `steps` steps of the single-lattice workload (default
    tiles), for the counter passes; useful and computed node-updates."""
    dev = torch.device("cuda:0")
    cfg = workloads.config_large()
    n, fl = cfg["n"], cfg["fields"]
    s_psi, s_eps, _ = lbm.coupled_rates(cfg["s_e"])
    lat = lbm.Lattice(n, lbm.Params(s_e=cfg["s_e"], s_psi=s_psi, s_eps=s_eps))
    t = lat.get_tuning()
    f = lat.equilibrium(*_dev_fields(torch, fl, dev))
    ws = lat.workspace(dev)
    calibration_copy(torch)
    lat.step(f, steps, ws)
    torch.cuda.synchronize()
    P, K, W = t["nodes_per_lane"], t["steps_per_launch"], t["waves_per_group"]
    ks = split_steps(steps, K)
    span = P * (62 * W + 2)
    computed = sum(-(-n // (span - 4 * k)) * 64 * P * W * k for k in ks)
    return {"leg": "single", "units": n * steps, "computed_units": computed,
            "launches": len(ks), "tuning": t}


def bench_batched(torch, lbm, workloads, stream, single_glups, tuning=None,
                  counter_run=False, counter_steps=None):
    """4096 lattices, lengths log-uniform in [512, 16384], 5000 steps in one
    hipGraph launch, tile shape from the autotuner (or `tuning`)."""
    import tempfile

    import numpy as np
    dev = torch.device("cuda:0")
    cfg = workloads.config_batched()
    bt, steps = cfg["batch"], cfg["steps"]
    log(f"bench: batched, {bt.n_inst} lattices, {bt.offsets[-1]} nodes, "
        f"{steps} steps")
    b = lbm.Batch(bt.offsets, _batch_params(lbm, bt))
    f0 = b.equilibrium(*_dev_fields(torch, bt.fields, dev))
    f = f0.clone()
    if tuning:
        b.set_tuning(*tuning)
        tune = b.get_tuning()
    else:
        cache = os.path.join(tempfile.gettempdir(), "lbm_tune_cache.json")
        # a longer probe ranks shapes whose times differ by a few per cent
        tune = b.autotune(f, probe_steps=160, cache_path=cache)
    lens = np.diff(np.asarray(bt.offsets))
    res = batch_split(lbm, lens, b.resident_lattices() > 0)
    assert int(res.sum()) == b.resident_lattices()
    if counter_run:
        steps = counter_steps or 2 * tune["steps_per_launch"]
        calibration_copy(torch)
        b.run(f, steps, use_graph=False)
        torch.cuda.synchronize()
        P, K, W = (tune[k] for k in ("nodes_per_lane", "steps_per_launch",
                                     "waves_per_group"))
        work = batch_computed(lens, res, P, K, W)
        return {"leg": "batched", "units": b.n_total * steps,
                "computed_units": work * steps, "resident": int(res.sum()),
                "launches": len(split_steps(steps, K)),
                "tuning": dict(tune, resident=True) if res.any() else tune}
    b.run(f, steps)  # warm-up, captures the graph
    torch.cuda.synchronize()
    ms = time_runs(lambda: b.run(f, steps), lambda: f.copy_(f0), 1, torch,
                   stream)
    d = b.diagnostics(f)
    ok = bool((d[:, 6] == 0).all() and (d[:, 7] == 0).all())
    g = b.n_total * steps / (ms * 1e-3) / 1e9
    shapes, group_of = b.get_groups()
    groups = []
    if shapes:
        for k, (P, K, W) in enumerate(shapes):
            sel = (group_of == k) & ~res
            groups.append({"nodes_per_lane": P, "steps_per_launch": K,
                           "waves_per_group": W, "lattices": int(sel.sum()),
                           "nodes": int(lens[sel].sum())})
    resident = {"lattices": int(res.sum()), "nodes": int(lens[res].sum()),
                "max_length": lbm.RESIDENT_MAX}
    launches = (len(split_steps(steps, tune["steps_per_launch"])) if not shapes
                else None)
    log(f"bench: batched {g:.2f} GLUPS, tuning {tune}, groups {groups}, "
        f"resident {resident}, finite: {ok}")
    key = tune if not resident["lattices"] else dict(tune, resident=True)
    roof = leg_roofline("batched", g * 1e9, 0.0, "node-update",
                        None if shapes else key)
    if not shapes and not roof["counters_current"]:
        roof.update(batched_roofline_from_arithmetic(bt, tune, steps, ms, g, res))
    # algorithmic HBM bytes: 96 per node per launch for the tiled lattices
    # (each launch reads and writes their state once), 96 per node per run
    # for the resident ones
    if launches:
        tiled = int(lens[~res].sum())
        per_run = BYTES_PER_NODE_LAUNCH * (tiled * launches + resident["nodes"])
        hbm = per_run / (ms * 1e-3) / 1e9
        roof["hbm"].update({"algorithmic_bytes_per_unit":
                            per_run / (b.n_total * steps),
                            "achieved": hbm, "frac": hbm / HBM_PEAK_GBS,
                            "launches": launches})
    return {"value": g, "unit": "GLUPS", "n_inst": bt.n_inst,
            "n_nodes": b.n_total, "time_steps": steps, "ms": ms,
            "tuning": tune, "groups": groups, "resident": resident,
            "graph": True, "valid": ok,
            "vs_single_lattice": g / single_glups, "roofline": roof}


def batched_roofline_from_arithmetic(bt, tune, steps, ms, glups, res):
    """ALU roofline of a batched run whose tile shape has no counter run of
    its own: the FP64 (and VALU) instructions per computed node-update of a
    counted batched run (the same node arithmetic, whatever the tile shape)
    times the node-updates this shape computes (its tiles, halos included)."""
    import glob  # noqa: F401
    import numpy as np
    if not os.path.exists(LEG_COUNTERS):
        return {}
    with open(LEG_COUNTERS) as fh:
        legs = json.load(fh).get("legs", {})
    ref = None
    for key, e in sorted(legs.items()):
        if key.startswith("batched@") and e.get("computed_units") and \
                e.get("source_hash") == source_hash(e.get("source_files", [])):
            ref = (key, e)
            break
    if ref is None:
        return {}
    key, e = ref
    P, K, W = (tune[k] for k in ("nodes_per_lane", "steps_per_launch",
                                 "waves_per_group"))
    lens = np.diff(np.asarray(bt.offsets))
    computed = batch_computed(lens, res, P, K, W) * steps
    fi = e["fp64_instr"] / e["computed_units"]
    fv = e["valu_instr"] / e["computed_units"]
    ff = e["flops"] / e["computed_units"]
    t = ms * 1e-3
    ach = fi * glups * 1e9 / 1e12
    return {"achieved": ach, "frac": ach / LANE_INSTR_PEAK_T,
            "fp64_instr_per_unit": fi,
            "fp64_instr_per_unit_basis": "computed node-update",
            "arithmetic_from": key,
            "flops": {"per_unit": ff, "achieved": ff * glups * 1e9 / 1e12,
                      "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                      "frac": ff * glups * 1e9 / 1e12 / FP64_PEAK_TFLOPS},
            "valu_issue_frac": fv * computed / t / (LANE_INSTR_PEAK_T * 1e12),
            "computed_per_useful": computed / (bt.offsets[-1] * steps)}


def bench_adjoint(torch, lbm, workloads, stream, counter_run=False):
    """Gradient of L = 1/2 |rho(T) - target|^2 on one lattice of 8192 nodes
    through 10000 steps (checkpoints every 100): forward with checkpoints,
    loss seed, recompute + reverse sweep (one hipGraph), equilibrium adjoint.
    Throughput in forward node-steps per second of the whole gradient; beside
    it the forward alone on the same lattice with the default tiles and with
    the one-step kernel."""
    dev = torch.device("cuda:0")
    cfg = workloads.config_adjoint()
    n, steps, ck = cfg["n"], cfg["steps"], cfg["ckpt"]
    s_psi, s_eps, _ = lbm.coupled_rates(cfg["s_e"])
    params = lbm.Params(s_e=cfg["s_e"], s_psi=s_psi, s_eps=s_eps)
    lat = lbm.Lattice(n, params)
    tgt_f = lat.equilibrium(*_dev_fields(torch, cfg["target_fields"], dev))
    lat.step(tgt_f, steps)
    target = lat.moments(tgt_f)[0].clone()
    fields = _dev_fields(torch, cfg["fields"], dev)
    aws = lat.adjoint_workspace(steps, ck, dev)
    log(f"bench: adjoint, n={n}, {steps} steps, checkpoints every {ck}")

    def grad():
        f = lat.equilibrium(*fields)
        lat.forward_ckpt(f, steps, ck, aws)
        _, fbar = lat.loss(f, target, aws)
        r = lat.adjoint(aws, steps, ck, fbar)
        lat.equilibrium_adjoint(*fields, fbar, aws)
        return r

    if counter_run:
        calibration_copy(torch)
        grad()
        torch.cuda.synchronize()
        return {"leg": "adjoint", "units": n * steps}
    grad()  # warm-up, captures the reverse graph
    torch.cuda.synchronize()
    ms = time_runs(grad, lambda: None, 2, torch, stream) / 2
    g = n * steps / (ms * 1e-3) / 1e9
    log(f"bench: adjoint {g:.3f} G node-steps/s ({ms:.1f} ms per gradient)")
    # the forward alone on the same lattice: default tiles, one-step kernel
    fwd = {}
    for name in ("default", "plain"):
        fl_ = lbm.Lattice(n, params)
        if name == "plain":
            fl_.set_tuning(lbm.KERNEL_PLAIN)
        f = fl_.equilibrium(*fields)
        fl_.step(f, 100)
        fms = time_runs(lambda: fl_.step(f, steps), lambda: None, 1, torch, stream)
        fwd[name] = n * steps / (fms * 1e-3) / 1e9
    log(f"bench: N={n} forward alone: default tiles {fwd['default']:.2f}, "
        f"one-step kernel {fwd['plain']:.2f} GLUPS")
    # A lattice this small leaves the chip mostly idle: each step is a chain
    # of dependent arithmetic per lane, so the time per step, not the issue
    # rate, bounds it.
    t = lat.get_tuning()
    span = t["nodes_per_lane"] * (62 * t["waves_per_group"] + 2) \
        if t["nodes_per_lane"] > 1 else 64
    tiles = -(-n // (span - 4 * t["steps_per_launch"]))
    roof = leg_roofline("adjoint", g * 1e9, GRAD_BYTES_PER_NODE_STEP,
                        "forward node-step", bytes_basis=GRAD_BYTES_BASIS)
    roof["latency"] = {
        "us_per_time_step": ms * 1e3 / steps,
        "forward_alone_us_per_time_step": n / (fwd["default"] * 1e9) * 1e6,
        "forward_wavefronts_per_launch": tiles * t["waves_per_group"],
        "chip_wavefronts_at_two_per_simd": 2048}
    return {"value": g, "unit": "G forward node-steps/s (whole gradient)",
            "n_nodes": n, "time_steps": steps, "ckpt_every": ck,
            "ms_per_gradient": ms, "workspace_gb": aws.numel() * 8 / 1e9,
            "forward_same_n": {"default_tiles_glups": fwd["default"],
                               "one_step_kernel_glups": fwd["plain"],
                               "gradient_vs_one_step_forward": g / fwd["plain"],
                               "gradient_vs_default_forward": g / fwd["default"]},
            "roofline": roof}


def bench_batched_adjoint(torch, lbm, workloads, stream, counter_run=False):
    """Per-lattice rate gradients of 1024 lattices (lengths uniform in
    [1024, 8192]) through 4000 steps, checkpoints every 63, one reverse
    hipGraph."""
    dev = torch.device("cuda:0")
    cfg = workloads.config_batched_adjoint()
    bt, steps, ck = cfg["batch"], cfg["steps"], cfg["ckpt"]
    b = lbm.Batch(bt.offsets, _batch_params(lbm, bt))
    fields = _dev_fields(torch, bt.fields, dev)
    aws = b.adjoint_workspace(steps, ck, dev)
    log(f"bench: batched adjoint, {bt.n_inst} lattices, {b.n_total} nodes, "
        f"{steps} steps, checkpoints every {ck} ({aws.numel() * 8 / 1e9:.1f} GB)")

    def grad():
        f = b.equilibrium(*fields)
        b.forward_ckpt(f, steps, ck, aws)
        _, fbar = b.loss(f, None, aws)
        return b.adjoint(aws, steps, ck, fbar)

    if counter_run:
        calibration_copy(torch)
        grad()
        torch.cuda.synchronize()
        del aws
        return {"leg": "batched_adjoint", "units": b.n_total * steps}
    grad()
    torch.cuda.synchronize()
    ms = time_runs(grad, lambda: None, 1, torch, stream)
    g = b.n_total * steps / (ms * 1e-3) / 1e9
    log(f"bench: batched adjoint {g:.3f} G node-steps/s ({ms:.1f} ms)")
    ws_gb = aws.numel() * 8 / 1e9
    del aws
    return {"value": g, "unit": "G forward node-steps/s (whole gradient)",
            "n_inst": bt.n_inst, "n_nodes": b.n_total, "time_steps": steps,
            "ckpt_every": ck, "ms_per_gradient": ms, "workspace_gb": ws_gb,
            "roofline": leg_roofline("batched_adjoint", g * 1e9,
                                     GRAD_BYTES_PER_NODE_STEP,
                                     "forward node-step",
                                     bytes_basis=GRAD_BYTES_BASIS)}


def copy_peak(torch, stream, nbytes: int, reps: int = 20):
    """HBM bandwidth of the runtime's device-to-device copy of nbytes (read
    plus written bytes over the time), for comparison with 8 TB/s."""
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    b.copy_(a)
    torch.cuda.synchronize()
    ms = time_runs(lambda: [b.copy_(a) for _ in range(reps)], lambda: None, 1,
                   torch, stream) / reps
    return 2 * nbytes / (ms * 1e-3) / 1e9


def summarize_counters(leg: str, run_json: str, dirs: list, out: str):
    """Totals of the rocprofv3 --pmc passes of one counter run of a leg (the
    dispatches of the leg's own kernels), written into the leg-counter file.
    run_json: the line the counter run printed (its useful units); dirs: the
    output directories of the passes (CSV).  FETCH_SIZE and WRITE_SIZE are
    scaled by what they read for the run's device copy of CALIB_BYTES."""
    import csv
    import glob
    with open(run_json) as fh:
        run = json.loads(fh.read().strip().splitlines()[-1])
    tot = {}
    n_disp = {}
    per_kernel = {}
    for d in dirs:
        for path in glob.glob(os.path.join(d, "**", "*counter_collection.csv"),
                              recursive=True):
            with open(path) as fh:
                for row in csv.DictReader(fh):
                    name = row["Kernel_Name"]
                    if not leg_kernel(leg, name):
                        continue
                    c = row["Counter_Name"]
                    v = float(row["Counter_Value"])
                    tot[c] = tot.get(c, 0.0) + v
                    n_disp.setdefault(c, set()).add(row.get("Dispatch_Id"))
                    short = name.replace("void ", "").replace(
                        "(anonymous namespace)::", "").split("(")[0]
                    k = per_kernel.setdefault(short, {"dispatches": {}})
                    k[c] = k.get(c, 0.0) + v
                    k["dispatches"].setdefault(c, set()).add(row.get("Dispatch_Id"))
    for k in per_kernel.values():
        k["dispatches"] = max(len(x) for x in k["dispatches"].values())
    # calibration: the run's copy of CALIB_BYTES (the largest copy dispatch)
    calib = {}
    for d in dirs:
        for path in glob.glob(os.path.join(d, "**", "*counter_collection.csv"),
                              recursive=True):
            with open(path) as fh:
                for row in csv.DictReader(fh):
                    if "copyBuffer" not in row["Kernel_Name"]:
                        continue
                    c = row["Counter_Name"]
                    if c in ("FETCH_SIZE", "WRITE_SIZE"):
                        calib[c] = max(calib.get(c, 0.0), float(row["Counter_Value"]))
    fs = CALIB_BYTES / (1024 * calib["FETCH_SIZE"]) if calib.get("FETCH_SIZE") else None
    ws_ = CALIB_BYTES / (1024 * calib["WRITE_SIZE"]) if calib.get("WRITE_SIZE") else None
    f64 = sum(tot.get(f"SQ_INSTS_VALU_{k}_F64", 0.0) for k in ("ADD", "MUL", "FMA", "TRANS"))
    wc = tot.get("SQ_WAVE_CYCLES")
    entry = {"units": run["units"], "tuning": run.get("tuning"),
             "computed_units": run.get("computed_units"),
             "launches": run.get("launches"),
             "fetch_scale": fs, "write_scale": ws_,
             "wave_cycle_fractions": ({c: tot[c] / wc for c in (
                 "SQ_ACTIVE_INST_VALU", "SQ_WAIT_INST_ANY", "SQ_WAIT_ANY",
                 "SQ_ACTIVE_INST_LDS", "SQ_LDS_BANK_CONFLICT") if c in tot}
                 if wc else None),
             "fp64_instr": 64 * f64,
             "flops": 64 * (f64 + tot.get("SQ_INSTS_VALU_FMA_F64", 0.0)),
             "valu_instr": 64 * tot.get("SQ_INSTS_VALU", 0.0),
             "fetch_bytes": (1024 * fs * tot["FETCH_SIZE"]
                             if fs and "FETCH_SIZE" in tot else None),
             "write_bytes": (1024 * ws_ * tot["WRITE_SIZE"]
                             if ws_ and "WRITE_SIZE" in tot else None),
             "dispatches": max((len(v) for v in n_disp.values()), default=0),
             "counters": {k: v for k, v in sorted(tot.items())},
             "kernels": per_kernel}
    rec = {}
    if os.path.exists(out):
        with open(out) as fh:
            rec = json.load(fh)
    # the sources of the leg's kernels
    files = ["lbm.hip", "lbm_device.hpp", "lbm_tile.hpp"]
    if leg in ("adjoint", "batched_adjoint"):
        files.append("lbm_adjoint.hip")
    entry["source_files"] = files
    entry["source_hash"] = source_hash(files)
    rec.setdefault("legs", {})[leg_key(leg, run.get("tuning"))] = entry
    with open(out, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps({leg: {k: v for k, v in entry.items() if k != "counters"}}))


def leg_kernel(leg: str, name: str) -> bool:
    """Whether a dispatch belongs to the counted work of a leg's counter run
    (the setup kernels of the run are left out: the target run and field
    initialisation of the single-lattice path)."""
    if leg == "batched":
        return "k_batch_tile" in name or "k_batch_resident" in name
    if leg == "single":
        return "k_step_tile" in name
    return not any(k in name for k in ("k_step_tile", "k_step_plain",
                                       "k_equilibrium(", "k_moments(", "k_diag",
                                       "__amd_rocclr", "k_batch_equilibrium",
                                       "at::"))


def main():
    args = parse()
    if args.summarize_counters:
        leg, run_json, *dirs = args.summarize_counters
        summarize_counters(leg, run_json, dirs, LEG_COUNTERS)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_1802_02369_amd import lbm, workloads

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    if args.counter_run:
        leg = args.counter_run
        if leg == "single":
            res = counter_run_single(torch, lbm, workloads, args.counter_steps or 80)
        elif leg == "batched":
            res = bench_batched(torch, lbm, workloads, stream, None,
                                tuning=tuple(int(x) for x in
                                             (args.batched_tuning or "4,24,4").split(",")),
                                counter_run=True, counter_steps=args.counter_steps)
        else:
            fn = bench_adjoint if leg == "adjoint" else bench_batched_adjoint
            res = fn(torch, lbm, workloads, stream, counter_run=True)
        print(json.dumps(res), flush=True)
        return
    n = args.n
    log(f"bench: building the N={n} workload")
    cfg = workloads.config_large(n=n)
    fl = cfg["fields"]
    s_psi, s_eps, _ = lbm.coupled_rates(cfg["s_e"])
    params = lbm.Params(s_e=cfg["s_e"], s_psi=s_psi, s_eps=s_eps)
    lat = lbm.Lattice(n, params)
    if args.tuning:
        P, K, W = (int(x) for x in args.tuning.split(","))
        lat.set_tuning(lbm.KERNEL_BLOCKED, P, K, W)
    tune = lat.get_tuning()
    rho, J, zeta = (torch.from_numpy(x).to(dev) for x in (fl.rho, fl.J, fl.zeta))
    f0 = lat.equilibrium(rho, J, zeta)
    f = f0.clone()
    ws = lat.workspace(dev)
    T = args.lbm_steps

    def reset():
        f.copy_(f0)

    def run():
        lat.step(f, T, ws)

    log(f"bench: warmup {args.warmup} x {T} steps, tuning {tune}")
    for _ in range(args.warmup):
        reset()
        run()
    torch.cuda.synchronize()
    log(f"bench: timing {args.steps} x {T} steps")
    ms = time_runs(run, reset, args.steps, torch, stream)
    node_updates = n * T * args.steps
    value = node_updates / (ms * 1e-3) / 1e9
    d = lat.diagnostics(f, ws)
    d0 = lat.diagnostics(f0, ws)
    ok = d[6] == 0 and d[7] == 0 and abs(d[0] - d0[0]) < 1e-10 * abs(d0[0])
    log(f"bench: {value:.2f} GLUPS, {ms / args.steps:.1f} ms per run, "
        f"state finite and mass conserved: {ok}")

    # launches of the blocked kernel per run, and node-updates they compute
    # (tiles of W = P (62 Wg + 2) nodes, W - 4k of them stored, for a launch
    # of k steps; every tile computes 64 P Wg node-updates per step, the
    # two-lane overlaps of its wavefronts included)
    P, K, Wg = (tune["nodes_per_lane"], tune["steps_per_launch"],
                tune["waves_per_group"])
    ks = split_steps(T, K)
    L = len(ks)
    W = P * (62 * Wg + 2)
    computed = sum(-(-n // (W - 4 * k)) * 64 * P * Wg * k for k in ks)
    launch_ms = ms / (args.steps * L)
    run_s = ms / args.steps * 1e-3
    # counted FP64 instructions (flops, VALU instructions) per computed
    # node-update of this kernel and tile shape, from the counter record
    # (null figures when no counter run was taken on the current sources)
    c = leg_counters("single", tune)
    Fi = args.instr_per_node or (c["fp64_instr"] / c["computed_units"] if c else None)
    Ff = c["flops"] / c["computed_units"] if c else None
    Fv = c["valu_instr"] / c["computed_units"] if c else None
    traffic = ((c["fetch_bytes"] + c["write_bytes"]) / c["launches"]
               if c and c.get("fetch_bytes") and c.get("write_bytes") else None)
    kname = f"k_step_tile<{P}, {Wg}, 0>"
    # algorithmic FP64 instructions per launch: per node-update figure times
    # the node-updates one launch delivers (halo recomputation is overhead)
    per_launch_s = n * T / L / (launch_ms * 1e-3) / 1e12
    achieved = Fi * per_launch_s if Fi is not None else None
    flops = Ff * per_launch_s if Ff is not None else None
    roof = {"bound": "alu", "achieved": achieved, "peak": LANE_INSTR_PEAK_T,
            "unit": "T FP64 instr/s",
            "frac": achieved / LANE_INSTR_PEAK_T if achieved is not None else None,
            "traffic": traffic,
            "kernel": kname,
            "launch_ms": launch_ms, "launches_per_run": L,
            "fp64_instr_per_node_update": Fi,
            "counters_current": c is not None,
            "flops": {"per_node_update": Ff, "achieved": flops,
                      "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                      "frac": flops / FP64_PEAK_TFLOPS if flops is not None else None},
            # every VALU instruction (FP64, moves, DPP, compares) over the
            # issue peak, halo node-updates included: how busy the SIMDs are
            "valu_issue_frac": (Fv * computed / run_s / (LANE_INSTR_PEAK_T * 1e12)
                                if Fv is not None else None),
            "algorithmic_bytes_per_launch": BYTES_PER_NODE_LAUNCH * n,
            "hbm_gbs_algorithmic": BYTES_PER_NODE_LAUNCH * n / (launch_ms * 1e-3) / 1e9}
    out = {
        "metric": METRIC, "value": value, "unit": "GLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "single periodic lattice, progressive shock "
                   "wave a=0.2", "n_nodes": n, "time_steps_per_step": T,
                   "s_e": cfg["s_e"], "kernel": "blocked", "tuning": tune},
        "roofline": roof,
        "valid": bool(ok),
    }

    if not args.no_extras and "plain" in (args.only or "plain").split(","):
        # one launch per time step on the same lattice: HBM-bound reference
        plat = lbm.Lattice(n, params)
        plat.set_tuning(lbm.KERNEL_PLAIN)
        Tp = 200
        log(f"bench: plain kernel, {Tp} steps")
        plat.step(f, 2, ws)
        torch.cuda.synchronize()
        pms = time_runs(lambda: plat.step(f, Tp, ws), reset, 1, torch, stream)
        plaunch = pms / Tp
        copy_gbs = copy_peak(torch, stream, 48 * n)
        pgbs = BYTES_PER_NODE_LAUNCH * n / (plaunch * 1e-3) / 1e9
        out["plain"] = {
            "value": n * Tp / (pms * 1e-3) / 1e9, "unit": "GLUPS",
            "kernel": "k_step_plain", "launch_ms": plaunch,
            "roofline": {"bound": "hbm", "achieved": pgbs,
                         "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": pgbs / HBM_PEAK_GBS,
                         # the runtime's device copy of one state (48 B per
                         # node read and written) on the same GPU
                         "measured_copy_gbs": copy_gbs,
                         "frac_of_measured_copy": pgbs / copy_gbs}}
        log(f"bench: plain {out['plain']['value']:.2f} GLUPS, {pgbs:.0f} GB/s "
            f"(device copy {copy_gbs:.0f} GB/s)")

    legs = set((args.only or "plain,batched,adjoint,batched_adjoint").split(","))
    bt_tune = (tuple(int(x) for x in args.batched_tuning.split(","))
               if args.batched_tuning else None)
    if not args.no_extras and "batched" in legs:
        out["batched"] = bench_batched(torch, lbm, workloads, stream, out["value"],
                                       tuning=bt_tune)
    if not args.no_extras and "adjoint" in legs:
        out["adjoint"] = bench_adjoint(torch, lbm, workloads, stream)
    if not args.no_extras and "batched_adjoint" in legs:
        out["batched_adjoint"] = bench_batched_adjoint(torch, lbm, workloads,
                                                       stream)

    if not args.no_cpu_baseline:
        log("bench: oracle CPU baseline (10 to 30 s)")
        out["cpu_baseline"] = cpu_baseline(n)
        # the oracle beside each extra leg, on its own workload's sample
        for leg, fn in (("batched", cpu_baseline_batched),
                        ("adjoint", cpu_baseline_adjoint),
                        ("batched_adjoint", cpu_baseline_batched_adjoint)):
            if leg in out:
                log(f"bench: oracle CPU baseline of the {leg} leg")
                out[leg]["cpu_baseline"] = fn()
    print(json.dumps(_no_nan(out)), flush=True)


if __name__ == "__main__":
    main()
