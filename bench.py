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
    return ap.parse_args()


COUNTERS = os.path.join(ROOT, "profiles", "counters_n16M.json")


def source_hash() -> str:
    """Hash of the sources of the blocked forward kernel; counter figures
    taken from other sources are not reported as this kernel's traffic."""
    import hashlib
    h = hashlib.sha256()
    for f in counter_record().get("source_files", []):
        with open(os.path.join(ROOT, "paper_1802_02369_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def counter_record():
    if os.path.exists(COUNTERS):
        with open(COUNTERS) as fh:
            return json.load(fh)
    return {}


def per_node_update(key: str) -> float:
    """Instructions (or flops) of one node-update of the blocked kernel, from
    the rocprofv3 counter run summarised under profiles/: FP64 instructions
    (device log/exp/reciprocals included), flops, all VALU instructions."""
    return float(counter_record().get(key, float("nan")))


def split_steps(nsteps: int, K: int) -> list:
    """Steps per launch as the library splits a run (an even number of
    launches of K or fewer steps)."""
    L = -(-nsteps // K)
    if L % 2 and nsteps > L:
        L += 1
    return [nsteps // L + (1 if i < nsteps % L else 0) for i in range(L)]


def measured_traffic(kernel: str, tune: dict):
    """HBM bytes per launch (calibrated FETCH_SIZE + WRITE_SIZE) of the kernel
    with this tuning, or None if the counters are missing or stale."""
    rec = counter_record()
    k = rec.get("kernels", {}).get(kernel)
    if not k or rec.get("source_hash") != source_hash():
        return None
    t = k.get("tuning", {})
    if any(t.get(x) != tune.get(x) for x in t):
        return None
    return k["fetch_bytes_per_dispatch"] + k["write_bytes_per_dispatch"]


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


def bench_batched(torch, lbm, workloads, stream, single_glups):
    """4096 lattices, lengths log-uniform in [512, 16384], 5000 steps in one
    hipGraph launch, tile shape from the autotuner."""
    import tempfile
    dev = torch.device("cuda:0")
    cfg = workloads.config_batched()
    bt, steps = cfg["batch"], cfg["steps"]
    log(f"bench: batched, {bt.n_inst} lattices, {bt.offsets[-1]} nodes, "
        f"{steps} steps")
    params = []
    for s_e in bt.s_e:
        s_psi, s_eps, _ = lbm.coupled_rates(float(s_e))
        params.append(lbm.Params(s_e=float(s_e), s_psi=s_psi, s_eps=s_eps))
    b = lbm.Batch(bt.offsets, params)
    f0 = b.equilibrium(*_dev_fields(torch, bt.fields, dev))
    f = f0.clone()
    cache = os.path.join(tempfile.gettempdir(), "lbm_tune_cache.json")
    # a longer probe ranks shapes whose times differ by a few per cent
    tune = b.autotune(f, probe_steps=160, cache_path=cache)
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
        import numpy as np
        lens = np.diff(np.asarray(bt.offsets))
        for k, (P, K, W) in enumerate(shapes):
            sel = group_of == k
            groups.append({"nodes_per_lane": P, "steps_per_launch": K,
                           "waves_per_group": W, "lattices": int(sel.sum()),
                           "nodes": int(lens[sel].sum())})
    log(f"bench: batched {g:.2f} GLUPS, tuning {tune}, groups {groups}, "
        f"finite: {ok}")
    return {"value": g, "unit": "GLUPS", "n_inst": bt.n_inst,
            "n_nodes": b.n_total, "time_steps": steps, "ms": ms,
            "tuning": tune, "groups": groups, "graph": True, "valid": ok,
            "vs_single_lattice": g / single_glups}


def bench_adjoint(torch, lbm, workloads, stream):
    """Gradient of L = 1/2 |rho(T) - target|^2 on one lattice of 8192 nodes
    through 10000 steps (checkpoints every 100): forward with checkpoints,
    loss seed, recompute + reverse sweep (one hipGraph), equilibrium adjoint.
    Throughput in forward node-steps per second of the whole gradient."""
    dev = torch.device("cuda:0")
    cfg = workloads.config_adjoint()
    n, steps, ck = cfg["n"], cfg["steps"], cfg["ckpt"]
    s_psi, s_eps, _ = lbm.coupled_rates(cfg["s_e"])
    lat = lbm.Lattice(n, lbm.Params(s_e=cfg["s_e"], s_psi=s_psi, s_eps=s_eps))
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

    grad()  # warm-up, captures the reverse graph
    torch.cuda.synchronize()
    ms = time_runs(grad, lambda: None, 2, torch, stream) / 2
    g = n * steps / (ms * 1e-3) / 1e9
    log(f"bench: adjoint {g:.3f} G node-steps/s ({ms:.1f} ms per gradient)")
    return {"value": g, "unit": "G forward node-steps/s (whole gradient)",
            "n_nodes": n, "time_steps": steps, "ckpt_every": ck,
            "ms_per_gradient": ms, "workspace_gb": aws.numel() * 8 / 1e9}


def bench_batched_adjoint(torch, lbm, workloads, stream):
    """Per-lattice rate gradients of 1024 lattices (lengths uniform in
    [1024, 8192]) through 4000 steps, checkpoints every 63, one reverse
    hipGraph."""
    dev = torch.device("cuda:0")
    cfg = workloads.config_batched_adjoint()
    bt, steps, ck = cfg["batch"], cfg["steps"], cfg["ckpt"]
    params = []
    for s_e in bt.s_e:
        s_psi, s_eps, _ = lbm.coupled_rates(float(s_e))
        params.append(lbm.Params(s_e=float(s_e), s_psi=s_psi, s_eps=s_eps))
    b = lbm.Batch(bt.offsets, params)
    fields = _dev_fields(torch, bt.fields, dev)
    aws = b.adjoint_workspace(steps, ck, dev)
    log(f"bench: batched adjoint, {bt.n_inst} lattices, {b.n_total} nodes, "
        f"{steps} steps, checkpoints every {ck} ({aws.numel() * 8 / 1e9:.1f} GB)")

    def grad():
        f = b.equilibrium(*fields)
        b.forward_ckpt(f, steps, ck, aws)
        _, fbar = b.loss(f, None, aws)
        return b.adjoint(aws, steps, ck, fbar)

    grad()
    torch.cuda.synchronize()
    ms = time_runs(grad, lambda: None, 1, torch, stream)
    g = b.n_total * steps / (ms * 1e-3) / 1e9
    log(f"bench: batched adjoint {g:.3f} G node-steps/s ({ms:.1f} ms)")
    ws_gb = aws.numel() * 8 / 1e9
    del aws
    return {"value": g, "unit": "G forward node-steps/s (whole gradient)",
            "n_inst": bt.n_inst, "n_nodes": b.n_total, "time_steps": steps,
            "ckpt_every": ck, "ms_per_gradient": ms, "workspace_gb": ws_gb}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_1802_02369_amd import lbm, workloads

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
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
    Fi = args.instr_per_node or per_node_update("fp64_instr_per_node_update")
    Ff = per_node_update("flops_per_node_update")
    Fv = per_node_update("valu_instr_per_node_update")
    kname = f"k_step_tile<{P}>"
    # algorithmic FP64 instructions per launch: per node-update figure times
    # the node-updates one launch delivers (halo recomputation is overhead)
    achieved = Fi * n * T / L / (launch_ms * 1e-3) / 1e12
    flops = Ff * n * T / L / (launch_ms * 1e-3) / 1e12
    roof = {"bound": "alu", "achieved": achieved, "peak": LANE_INSTR_PEAK_T,
            "unit": "T FP64 instr/s", "frac": achieved / LANE_INSTR_PEAK_T,
            "traffic": measured_traffic(kname, tune),
            "kernel": kname,
            "launch_ms": launch_ms, "launches_per_run": L,
            "fp64_instr_per_node_update": Fi,
            "counters_current": counter_record().get("source_hash") == source_hash(),
            "flops": {"per_node_update": Ff, "achieved": flops,
                      "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                      "frac": flops / FP64_PEAK_TFLOPS},
            # every VALU instruction (FP64, moves, DPP, compares) over the
            # issue peak, halo node-updates included: how busy the SIMDs are
            "valu_issue_frac": Fv * computed / run_s / (LANE_INSTR_PEAK_T * 1e12),
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
        out["plain"] = {
            "value": n * Tp / (pms * 1e-3) / 1e9, "unit": "GLUPS",
            "kernel": "k_step_plain", "launch_ms": plaunch,
            "roofline": {"bound": "hbm",
                         "achieved": BYTES_PER_NODE_LAUNCH * n / (plaunch * 1e-3) / 1e9,
                         "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": BYTES_PER_NODE_LAUNCH * n / (plaunch * 1e-3) / 1e9
                         / HBM_PEAK_GBS}}
        log(f"bench: plain {out['plain']['value']:.2f} GLUPS")

    legs = set((args.only or "plain,batched,adjoint,batched_adjoint").split(","))
    if not args.no_extras and "batched" in legs:
        out["batched"] = bench_batched(torch, lbm, workloads, stream, out["value"])
    if not args.no_extras and "adjoint" in legs:
        out["adjoint"] = bench_adjoint(torch, lbm, workloads, stream)
    if not args.no_extras and "batched_adjoint" in legs:
        out["batched_adjoint"] = bench_batched_adjoint(torch, lbm, workloads,
                                                       stream)

    if not args.no_cpu_baseline:
        log("bench: oracle CPU baseline (10 to 30 s)")
        out["cpu_baseline"] = cpu_baseline(n)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
