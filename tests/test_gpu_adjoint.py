"""GPU parity of the reverse mode (adjoint step, checkpointed gradients, loss
seed, equilibrium adjoint, batch form, autograd wrapper) against the oracle's
adjoint, its tangent-linear model and central differences."""
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


def T(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dev())


def rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


@pytest.mark.parametrize("adj", ["plain", "blocked"])
@pytest.mark.parametrize("pname", ["paper", "odd", "nosource", "linear", "fluid",
                                   "thermal", "fluid_odd", "thermal_odd"])
@pytest.mark.parametrize("n", [3, 5, 64, 251, 252, 253, 256, 1000, 3001])
def test_one_adjoint_step(pname, n, adj):
    """fbar(t) and the rate partials of one step against the oracle's
    adjoint (exact per-node Jacobian blocks, transposed)."""
    rng = np.random.default_rng(n)
    po = oracle_params(pname)
    f0 = random_state(rng, n, po)
    fbn = rng.standard_normal((6, n))
    want_fb, want_r = oracle.step_adjoint(f0, fbn, po)
    lat = lbm().Lattice(n, gpu_params(po))
    if adj == "blocked":
        lat.set_adjoint_kernel(lbm().KERNEL_BLOCKED)
    aws = lat.adjoint_workspace(1, 1, dev())
    f = T(f0)
    lat.forward_ckpt(f, 1, 1, aws)
    assert max_err(f.cpu().numpy(), oracle.step(f0, po)) < TOL
    fb = T(fbn)
    r = lat.adjoint(aws, 1, 1, fb, use_graph=False)
    assert max_err(fb.cpu().numpy(), want_fb) < TOL
    # Each rate partial is a sum over the nodes of (deviation of a moment
    # from its equilibrium) x (an adjoint): the deviation is a difference of
    # O(1) populations, so each term carries a few ulp of the populations
    # times |fbar| of absolute rounding, whatever the partial's size; the
    # absolute bar is 8 ulp of that per node.
    atol = 8 * n * np.finfo(float).eps * np.abs(f0).max() * np.abs(fbn).max()
    np.testing.assert_allclose(r, want_r, rtol=1e-11, atol=atol)


@pytest.mark.parametrize("kernel", ["plain", "blocked", "blocked_p4w2k5",
                                    "blocked_p8w2k6", "blocked_p8w8k9",
                                    "plainfwd", "blocked_s2", "blocked_p4w2k5_s2",
                                    "blocked_p8w8k9_s2", "blocked_p2w1k16",
                                    "blocked_p1w1k7"])
@pytest.mark.parametrize("pname,n,steps,ckpt", [
    ("paper", 64, 40, 7), ("odd", 300, 33, 33), ("nosource", 97, 25, 1),
    ("linear", 260, 18, 5), ("odd", 1200, 50, 8), ("fluid", 700, 37, 20),
    ("thermal", 500, 30, 30), ("odd", 5000, 70, 35), ("fluid_odd", 400, 25, 6),
    ("thermal_odd", 600, 28, 9)])
def test_checkpointed_gradient(pname, n, steps, ckpt, kernel):
    rng = np.random.default_rng(steps)
    po = oracle_params(pname)
    j = np.arange(n)
    rho = po.rho0 * (1 + 0.05 * np.sin(2 * np.pi * j / n) + 0.01 * rng.standard_normal(n))
    J = po.rho0 * po.lam * 0.02 * np.cos(2 * np.pi * j / n)
    zeta = rho * (po.s0 + 0.02 * po.cp * rng.standard_normal(n))
    tgt = po.rho0 * (1 + 0.03 * np.sin(2 * np.pi * j / n + 1))
    L, rb, Jb, zb, sb = oracle.gradient(rho, J, zeta, steps, tgt, po)
    lat = lbm().Lattice(n, gpu_params(po))
    if kernel.endswith("_s2"):
        # keep only the even recomputed states (the reverse kernel
        # recomputes the odd ones)
        lat.set_recompute_stride(2)
        kernel = kernel[:-3]
    if kernel == "plainfwd":
        lat.set_tuning(kernel=lbm().KERNEL_PLAIN)
    elif kernel == "blocked":
        lat.set_adjoint_kernel(lbm().KERNEL_BLOCKED)
    elif kernel == "blocked_p4w2k5":
        lat.set_adjoint_kernel(lbm().KERNEL_BLOCKED)
        lat.set_tuning(nodes_per_lane=4, steps_per_launch=5, waves_per_group=2)
    elif kernel == "blocked_p8w2k6":
        lat.set_adjoint_kernel(lbm().KERNEL_BLOCKED)
        lat.set_tuning(nodes_per_lane=8, steps_per_launch=6, waves_per_group=2)
    elif kernel == "blocked_p8w8k9":
        lat.set_adjoint_kernel(lbm().KERNEL_BLOCKED)
        lat.set_tuning(nodes_per_lane=8, steps_per_launch=9, waves_per_group=8)
    elif kernel == "blocked_p2w1k16":
        lat.set_adjoint_kernel(lbm().KERNEL_BLOCKED)
        lat.set_tuning(nodes_per_lane=2, steps_per_launch=16, waves_per_group=1)
    elif kernel == "blocked_p1w1k7":
        lat.set_adjoint_kernel(lbm().KERNEL_BLOCKED)
        lat.set_tuning(nodes_per_lane=1, steps_per_launch=7, waves_per_group=1)
    aws = lat.adjoint_workspace(steps, ckpt, dev())
    r_, J_, z_ = T(rho), T(J), T(zeta)
    f = lat.equilibrium(r_, J_, z_)
    lat.forward_ckpt(f, steps, ckpt, aws)
    Lg, fbar = lat.loss(f, T(tgt), aws)
    assert rel(Lg, L) < 1e-11
    r = lat.adjoint(aws, steps, ckpt, fbar)
    g = lat.equilibrium_adjoint(r_, J_, z_, fbar, aws)
    for got, want in zip(g, (rb, Jb, zb)):
        w = np.abs(want).max()
        assert np.abs(got.cpu().numpy() - want).max() <= 1e-10 * w + 1e-300
    np.testing.assert_allclose(r, sb, rtol=1e-10, atol=1e-12 * np.abs(sb).max())


def test_blocked_adjoint_rejects_halo_beyond_reverse_tile():
    """P = 8 with 8 wavefronts runs its reverse on tiles of 2048 nodes (P = 4,
    8 wavefronts): a forward K of 512 is a valid forward shape (tiles of 3984
    nodes) but leaves the reverse tiles no interior, so the checkpointed
    forward refuses it before any launch; the one-step adjoint kernel accepts
    the same tile shape."""
    po = oracle_params("paper")
    n = 3000
    lat = lbm().Lattice(n, gpu_params(po))
    lat.set_tuning(nodes_per_lane=8, steps_per_launch=512, waves_per_group=8)
    lat.set_adjoint_kernel(lbm().KERNEL_BLOCKED)
    aws = lat.adjoint_workspace(10, 5, dev())
    f = T(random_state(np.random.default_rng(3), n, po))
    with pytest.raises(lbm().LBMError) as e:
        lat.forward_ckpt(f, 10, 5, aws)
    assert e.value.code == lbm().LBM_ENOTSUP
    lat.set_adjoint_kernel(lbm().KERNEL_PLAIN)
    lat.forward_ckpt(f, 10, 5, aws)
    # the default (AUTO) falls back to the one-step kernel for this shape
    lat.set_adjoint_kernel(lbm().KERNEL_AUTO)
    lat.forward_ckpt(f, 10, 5, aws)


def test_graph_adjoint_matches_direct():
    rng = np.random.default_rng(5)
    po = oracle_params("odd")
    n, steps, ckpt = 700, 40, 9
    f0 = random_state(rng, n, po)
    lat = lbm().Lattice(n, gpu_params(po))
    aws = lat.adjoint_workspace(steps, ckpt, dev())
    f = T(f0)
    lat.forward_ckpt(f, steps, ckpt, aws)
    seed = T(rng.standard_normal((6, n)))
    ref = seed.clone()
    rr = lat.adjoint(aws, steps, ckpt, ref, use_graph=False)
    for rep in range(3):
        fb = seed.clone()
        _ = (fb * 3).sum().item()
        r = lat.adjoint(aws, steps, ckpt, fb, use_graph=True)
        torch.cuda.synchronize()
        assert torch.equal(fb, ref) and r == rr, rep


def test_adjoint_config_gradient():
    """N = 8192, eight-mode initial field, 10000 steps, checkpoints every
    100: the gradient of L = 1/2 |rho(T) - target|^2 (target: the oracle's
    run of the seed-4 field) against the oracle's tangent-linear directional
    derivatives (random directions in rho(0), J(0) and each rate) and
    against central differences of the GPU forward run in the rates."""
    from paper_1802_02369_amd import workloads
    cfg = workloads.config_adjoint()
    n, steps, ckpt = cfg["n"], cfg["steps"], cfg["ckpt"]
    fl, tf = cfg["fields"], cfg["target_fields"]
    po = oracle_params("paper", s_e=cfg["s_e"])
    say(f"adjoint config n={n} steps={steps} ckpt={ckpt}")
    tgt = oracle.moments(oracle.run(oracle.init(tf.rho, tf.J, tf.zeta, po), steps, po), po)[0]
    lat = lbm().Lattice(n, gpu_params(po))
    aws = lat.adjoint_workspace(steps, ckpt, dev())
    r_, J_, z_ = T(fl.rho), T(fl.J), T(fl.zeta)
    f = lat.equilibrium(r_, J_, z_)
    lat.forward_ckpt(f, steps, ckpt, aws)
    Lg, fbar = lat.loss(f, T(tgt), aws)
    rbar = lat.adjoint(aws, steps, ckpt, fbar)
    g_rho, g_J, g_z = (x.cpu().numpy() for x in lat.equilibrium_adjoint(r_, J_, z_, fbar, aws))
    rng = np.random.default_rng(9)
    dirs = []
    for k in range(4):
        dirs.append((rng.standard_normal(n), rng.standard_normal(n), np.zeros(n), np.zeros(3)))
    for q in range(3):
        e = np.zeros(3)
        e[q] = 1.0
        dirs.append((np.zeros(n), np.zeros(n), np.zeros(n), e))
    say("  oracle tangent-linear runs: 7 directions")
    with ThreadPoolExecutor(7) as ex:
        res = list(ex.map(lambda d: oracle.directional(fl.rho, fl.J, fl.zeta, *d, steps, tgt, po), dirs))
    for (Lo, dL), d in zip(res, dirs):
        adj = g_rho @ d[0] + g_J @ d[1] + np.dot(rbar, d[3])
        say(f"  <grad, v> = {adj:.12e}   tangent-linear {dL:.12e}")
        assert rel(Lg, Lo) < 1e-9
        assert rel(adj, dL) < 1e-6
    # central differences of the GPU forward run in each rate, measured
    # against the size of the whole rate gradient.  This arm pins dL/ds_e and
    # dL/ds_psi; it does not pin dL/ds_eps (~4e-8 here, below the rounding
    # floor of a difference quotient of L ~ 1: the bound admits ~25 % error
    # in it).  dL/ds_eps is held by the tangent-linear direction e_3 above,
    # to 1e-6 relative.
    h = 1e-5
    scale = np.abs(rbar).max()
    for q in range(3):
        vals = []
        for sgn in (1, -1):
            rates = [po.s_e, po.s_psi, po.s_eps]
            rates[q] += sgn * h
            p2 = oracle_params("paper", s_e=rates[0], s_psi=rates[1], s_eps=rates[2])
            l2 = lbm().Lattice(n, gpu_params(p2))
            g = l2.equilibrium(r_, J_, z_)
            l2.step(g, steps)
            vals.append(0.5 * float(((g[:3].sum(0) * po.rho0 - T(tgt)) ** 2).sum()))
        fd = (vals[0] - vals[1]) / (2 * h)
        say(f"  dL/drate[{q}]: adjoint {rbar[q]:.10e}  central difference {fd:.10e}")
        assert abs(rbar[q] - fd) < 1e-6 * scale


@pytest.mark.parametrize("adj", ["plain", "blocked", "blocked_s2"])
def test_batched_adjoint(adj):
    """Per-lattice gradients of a ragged batch against the oracle, lattice by
    lattice (loss 1/2 sum (rho(T) - rho0)^2 per lattice)."""
    from paper_1802_02369_amd import workloads
    cfg = workloads.config_batched_adjoint(n_inst=24, steps=150, ckpt=13,
                                           lmin=100, lmax=1500)
    bt, steps, ckpt = cfg["batch"], cfg["steps"], cfg["ckpt"]
    ps = [oracle_params("paper", s_e=float(s)) for s in bt.s_e]
    b = lbm().Batch(bt.offsets, [gpu_params(p) for p in ps])
    if adj.startswith("blocked"):
        b.set_adjoint_kernel(lbm().KERNEL_BLOCKED)
    if adj == "blocked_s2":
        b.set_recompute_stride(2)
    fl = bt.fields
    r_, J_, z_ = T(fl.rho), T(fl.J), T(fl.zeta)
    f = b.equilibrium(r_, J_, z_)
    aws = b.adjoint_workspace(steps, ckpt, dev())
    b.forward_ckpt(f, steps, ckpt, aws)
    loss, fbar = b.loss(f, None, aws)
    rbar = b.adjoint(aws, steps, ckpt, fbar).cpu().numpy()
    g_rho = b.equilibrium_adjoint(r_, J_, z_, fbar, aws)[0].cpu().numpy()
    loss = loss.cpu().numpy()

    def one(i):
        a, c = bt.offsets[i], bt.offsets[i + 1]
        x = bt.instance(i)
        return oracle.gradient(x.rho, x.J, x.zeta, steps, np.full(c - a, ps[i].rho0), ps[i])

    with ThreadPoolExecutor(16) as ex:
        res = list(ex.map(one, range(bt.n_inst)))
    for i, (L, rb, Jb, zb, sb) in enumerate(res):
        a, c = bt.offsets[i], bt.offsets[i + 1]
        assert rel(loss[i], L) < 1e-10, i
        assert np.abs(g_rho[a:c] - rb).max() <= 1e-10 * np.abs(rb).max(), i
        np.testing.assert_allclose(rbar[i], sb, rtol=1e-9, atol=1e-12 * np.abs(sb).max())


def oracle_gradient_by_segments(rho, J, zeta, steps, ckpt, target, p):
    """oracle.gradient for a long run, driven from here segment by segment
    with the oracle's own step, step adjoint, loss and initialisation
    adjoint (the same checkpointed sweep, one line of progress per tenth of
    the segments).  Returns (loss, rho_bar, J_bar, zeta_bar, rbar)."""
    f = oracle.init(rho, J, zeta, p)
    cks = []
    for t0 in range(0, steps, ckpt):
        cks.append(f)
        f = oracle.run(f, min(ckpt, steps - t0), p)
    L, fbar = oracle.loss(f, target, p)
    rbar = np.zeros(3)
    nseg = len(cks)
    for k in range(nseg - 1, -1, -1):
        t0 = k * ckpt
        states = [cks[k]]
        for _ in range(min(ckpt, steps - t0) - 1):
            states.append(oracle.step(states[-1], p))
        for st in reversed(states):
            fbar, r = oracle.step_adjoint(st, fbar, p)
            rbar += r
        if k % max(1, nseg // 10) == 0:
            say(f"    oracle sweep of the {len(rho)}-node lattice: segment {k} of {nseg}")
    rb, Jb, zb = oracle.init_adjoint(rho, J, zeta, fbar, p)
    return L, rb, Jb, zb, rbar


@pytest.mark.timeout(900)
def test_batched_adjoint_config_sampled():
    """The batched-gradient workload in the configuration the benchmark
    times (1024 lattices, lengths in [1024, 8192], 4000 steps, checkpoints
    every 63, default tile shape, automatic reverse kernel and recompute
    stride, captured graph): loss, rate gradients and dL/drho(0) of four
    seeded lattices (among the shorter ones, for the oracle's time) against
    the oracle's adjoint of each lattice alone, and of the shortest lattice
    of at least 6000 nodes (its reverse sweep spans 12 reverse tiles)."""
    from paper_1802_02369_amd import workloads
    cfg = workloads.config_batched_adjoint()
    bt, steps, ckpt = cfg["batch"], cfg["steps"], cfg["ckpt"]
    say(f"batched adjoint config: {bt.n_inst} lattices, {bt.offsets[-1]} nodes, "
        f"{steps} steps, checkpoints every {ckpt}")
    ps = []
    for s_e in bt.s_e:
        s_psi, s_eps, _ = lbm().coupled_rates(float(s_e))
        ps.append(oracle_params("paper", s_e=float(s_e), s_psi=s_psi, s_eps=s_eps))
    b = lbm().Batch(bt.offsets, [gpu_params(p) for p in ps])
    fl = bt.fields
    r_, J_, z_ = T(fl.rho), T(fl.J), T(fl.zeta)
    f = b.equilibrium(r_, J_, z_)
    aws = b.adjoint_workspace(steps, ckpt, dev())
    b.forward_ckpt(f, steps, ckpt, aws)
    loss, fbar = b.loss(f, None, aws)
    rbar = b.adjoint(aws, steps, ckpt, fbar).cpu().numpy()
    g_rho = b.equilibrium_adjoint(r_, J_, z_, fbar, aws)[0].cpu().numpy()
    loss = loss.cpu().numpy()
    del aws
    rng = np.random.default_rng(1024)
    lengths = np.asarray(bt.lengths)
    short = np.flatnonzero(lengths <= 1300)
    sub = np.sort(rng.choice(short, 4, replace=False))
    # and the shortest lattice of at least 6000 nodes (12 reverse tiles)
    big = np.flatnonzero(lengths >= 6000)
    long_i = int(big[np.argmin(lengths[big])])
    say(f"  oracle adjoint of lattices {[int(i) for i in sub]} "
        f"(lengths {[int(n) for n in lengths[sub]]}) and {long_i} "
        f"(length {int(lengths[long_i])})")

    def one(i):
        a, c = bt.offsets[i], bt.offsets[i + 1]
        x = bt.instance(i)
        return oracle.gradient(x.rho, x.J, x.zeta, steps, np.full(c - a, ps[i].rho0),
                               ps[i])

    def one_long(i):
        a, c = bt.offsets[i], bt.offsets[i + 1]
        x = bt.instance(i)
        return oracle_gradient_by_segments(x.rho, x.J, x.zeta, steps, ckpt,
                                           np.full(c - a, ps[i].rho0), ps[i])

    with ThreadPoolExecutor(5) as ex:
        fut_long = ex.submit(one_long, long_i)
        res = list(ex.map(one, sub))
        res_long = fut_long.result()
    for i, (L, rb, Jb, zb, sb) in zip(list(sub) + [long_i], res + [res_long]):
        a, c = bt.offsets[i], bt.offsets[i + 1]
        err = np.abs(g_rho[a:c] - rb).max() / np.abs(rb).max()
        say(f"  lattice {i}: loss rel {rel(loss[i], L):.1e}, dL/drho(0) {err:.1e}, "
            f"rates {np.abs(rbar[i] - sb).max() / np.abs(sb).max():.1e}")
        assert rel(loss[i], L) < 1e-10, i
        assert err <= 1e-10, i
        np.testing.assert_allclose(rbar[i], sb, rtol=1e-9, atol=1e-12 * np.abs(sb).max())


def test_blocked_reverse_large_batch_matches_one_step_reverse():
    """A batch large enough for the blocked reverse sweep to run on one
    stream (its launches fill the chip: 256 lattices, 2.06M nodes): the
    gradients equal those of the one-step reverse kernel, which the oracle
    tests pin on smaller batches, and the rate gradients of two of its
    lattices match the oracle.  These small-amplitude lattices have rate
    gradients of 1e-10 .. 1e-7 (s_eps: 1e-17 .. 1e-14) that are sums over
    nodes and steps with cancellation: both kernels sit up to a few 1e-10
    (s_eps: a few 1e-9) from the oracle, which bounds their agreement; the
    same holds for dL/dzeta(0) (measured 4e-11 and 5e-10 of its largest
    value from the oracle on lattices 0 and 1, for either kernel; dL/drho(0)
    2e-14, dL/dJ(0) 5e-13)."""
    from paper_1802_02369_amd import workloads
    cfg = workloads.config_batched_adjoint(n_inst=256, steps=40, ckpt=7,
                                           lmin=7000, lmax=9000)
    bt, steps, ckpt = cfg["batch"], cfg["steps"], cfg["ckpt"]
    ps = [gpu_params(oracle_params("paper", s_e=float(s))) for s in bt.s_e]
    fl = bt.fields
    out = {}
    for adj in ("blocked", "plain"):
        b = lbm().Batch(bt.offsets, ps)
        b.set_tuning(4, 16, 4)
        b.set_adjoint_kernel(lbm().KERNEL_BLOCKED if adj == "blocked"
                             else lbm().KERNEL_PLAIN)
        r_, J_, z_ = T(fl.rho), T(fl.J), T(fl.zeta)
        f = b.equilibrium(r_, J_, z_)
        aws = b.adjoint_workspace(steps, ckpt, dev())
        b.forward_ckpt(f, steps, ckpt, aws)
        _, fbar = b.loss(f, None, aws)
        rbar = b.adjoint(aws, steps, ckpt, fbar).cpu().numpy()
        g = b.equilibrium_adjoint(r_, J_, z_, fbar, aws)
        out[adj] = (rbar, [x.cpu().numpy() for x in g])
        del aws, b
    rb, gb = out["blocked"]
    rp, gp = out["plain"]
    assert np.isfinite(rb).all()
    np.testing.assert_allclose(rb[:, :2], rp[:, :2], rtol=2e-9,
                               atol=1e-13 * np.abs(rp).max())
    np.testing.assert_allclose(rb[:, 2], rp[:, 2], rtol=1e-8,
                               atol=1e-13 * np.abs(rp[:, 2]).max())
    for k, (x, y) in enumerate(zip(gb, gp)):
        say(f"  initial-field adjoint {k}: max |tile - one-step| / max |one-step| "
            f"{np.abs(x - y).max() / np.abs(y).max():.2e}")
    for i in (0, 1):
        o0, o1 = bt.offsets[i], bt.offsets[i + 1]
        po = oracle_params("paper", s_e=float(bt.s_e[i]))
        want = oracle.gradient(fl.rho[o0:o1], fl.J[o0:o1], fl.zeta[o0:o1], steps,
                               np.full(o1 - o0, po.rho0), po, ckpt=ckpt)
        err_b = np.abs(rb[i] - want[4]) / np.abs(want[4])
        err_p = np.abs(rp[i] - want[4]) / np.abs(want[4])
        say(f"  lattice {i}: rate gradients vs oracle, reverse tile {err_b}, one-step {err_p}")
        for k in range(3):
            w = want[1 + k]
            eb = np.abs(gb[k][o0:o1] - w).max() / np.abs(w).max()
            ep = np.abs(gp[k][o0:o1] - w).max() / np.abs(w).max()
            say(f"  lattice {i}: initial-field adjoint {k} vs oracle: tile {eb:.2e}, one-step {ep:.2e}")
            assert eb < FIELD_BARS[k] and ep < FIELD_BARS[k], (i, k)
        assert (err_b < [2e-9, 2e-9, 1e-8]).all() and (err_p < [2e-9, 2e-9, 1e-8]).all()
    for k, (x, y) in enumerate(zip(gb, gp)):
        assert np.abs(x - y).max() <= FIELD_BARS[k] * np.abs(y).max(), k


# dL/drho(0), dL/dJ(0), dL/dzeta(0) of the small-amplitude batched-gradient
# lattices, relative to the largest value: see the test above
FIELD_BARS = (1e-12, 1e-11, 2e-9)


def _stride_run(make, stride, steps, ckpt, fields):
    m = make()
    m.set_adjoint_kernel(lbm().KERNEL_BLOCKED)
    m.set_recompute_stride(stride)
    r_, J_, z_ = fields
    f = m.equilibrium(r_, J_, z_)
    aws = m.adjoint_workspace(steps, ckpt, dev())
    m.forward_ckpt(f, steps, ckpt, aws)
    _, fbar = m.loss(f, None, aws)
    rbar = m.adjoint(aws, steps, ckpt, fbar, use_graph=False)
    rbar = rbar.cpu().numpy() if hasattr(rbar, "cpu") else np.asarray(rbar)
    g = [x.cpu().numpy() for x in m.equilibrium_adjoint(r_, J_, z_, fbar, aws)]
    return fbar.cpu().numpy(), rbar, g, aws.numel()


@pytest.mark.parametrize("pname", ["paper", "linear", "fluid", "nosource"])
@pytest.mark.parametrize("shape,n,steps,ckpt", [
    ((2, 16, 1), 3000, 70, 33),     # K even, segments of odd and even length
    ((4, 5, 2), 2500, 41, 12),      # K odd: recompute launches of 4 steps
    ((8, 9, 8), 9000, 60, 19),      # odd tops of the reverse launches
    ((8, 40, 4), 4000, 95, 95),     # one segment, two reverse launches
    ((4, 7, 4), 100, 30, 30),       # a lattice shorter than one tile
    ((2, 2, 1), 1000, 9, 4),        # the smallest K with stride 2
    ((2, 6, 2), 2000, 30, 11),      # two-wavefront reverse tiles
    ((2, 16, 1), 500, 1, 1),        # one step: no segment states at all
    ((4, 5, 2), 700, 2, 5),         # one segment of two steps
    ((8, 9, 8), 3000, 3, 2)])       # segments of two steps and one
def test_recompute_stride_is_bitwise(shape, n, steps, ckpt, pname):
    """Keeping only the even recomputed states (the reverse kernel recomputes
    each odd one from the state before) gives bitwise the same dL/df(0) and
    initial-field adjoints as keeping every state; the rate gradients, summed
    over a different tiling (halo 2K + 2), agree to rounding.  The workspace
    holds half the segment states."""
    rng = np.random.default_rng(n + steps)
    po = oracle_params(pname)
    j = np.arange(n)
    fields = (T(po.rho0 * (1 + 0.05 * np.sin(2 * np.pi * j / n)
                          + 0.01 * rng.standard_normal(n))),
              T(po.rho0 * po.lam * 0.02 * np.cos(2 * np.pi * j / n)),
              T(po.rho0 * (po.s0 + 0.02 * po.cp * rng.standard_normal(n))))
    P, K, W = shape

    def make():
        lat = lbm().Lattice(n, gpu_params(po))
        lat.set_tuning(nodes_per_lane=P, steps_per_launch=K, waves_per_group=W)
        return lat

    say(f"  stride 1 vs 2: {pname} shape {shape} n={n} steps={steps} ckpt={ckpt}")
    fb1, r1, g1, ws1 = _stride_run(make, 1, steps, ckpt, fields)
    fb2, r2, g2, ws2 = _stride_run(make, 2, steps, ckpt, fields)
    assert np.isfinite(fb1).all()
    assert np.array_equal(fb1, fb2)
    for a, b in zip(g1, g2):
        assert np.array_equal(a, b)
    np.testing.assert_allclose(r2, r1, rtol=1e-12, atol=1e-14 * np.abs(r1).max())
    if min(ckpt, steps) > 2:
        assert ws2 < ws1


def test_recompute_stride_batch_is_bitwise():
    """The same for a ragged batch with mixed equilibria, both strides under
    a captured graph."""
    from paper_1802_02369_amd import workloads
    cfg = workloads.config_batched_adjoint(n_inst=40, steps=50, ckpt=11,
                                           lmin=60, lmax=3000)
    bt, steps, ckpt = cfg["batch"], cfg["steps"], cfg["ckpt"]
    names = ["paper", "linear", "fluid", "thermal", "odd"]
    ps = [gpu_params(oracle_params(names[i % len(names)])) for i in range(bt.n_inst)]
    fl = bt.fields
    fields = (T(fl.rho), T(fl.J), T(fl.zeta))
    out = []
    for stride in (1, 2):
        b = lbm().Batch(bt.offsets, ps)
        b.set_tuning(4, 6, 4)
        b.set_adjoint_kernel(lbm().KERNEL_BLOCKED)
        b.set_recompute_stride(stride)
        f = b.equilibrium(*fields)
        aws = b.adjoint_workspace(steps, ckpt, dev())
        b.forward_ckpt(f, steps, ckpt, aws)
        _, fbar = b.loss(f, None, aws)
        rbar = b.adjoint(aws, steps, ckpt, fbar).cpu().numpy()
        out.append((fbar.cpu().numpy(), rbar))
        del aws, b
    assert np.isfinite(out[0][0]).all()
    assert np.array_equal(out[0][0], out[1][0])
    np.testing.assert_allclose(out[1][1], out[0][1], rtol=1e-12,
                               atol=1e-14 * np.abs(out[0][1]).max())


def test_autograd_function():
    from paper_1802_02369_amd.autograd import LBMFunction
    po = oracle_params("paper", s_e=1.7)
    n, steps, ckpt = 128, 60, 8
    rng = np.random.default_rng(4)
    j = np.arange(n)
    rho = 1 + 0.05 * np.sin(2 * np.pi * j / n) + 0.01 * rng.standard_normal(n)
    J = 0.02 * np.cos(2 * np.pi * j / n)
    zeta = 0.01 * rng.standard_normal(n)
    tgt = 1 + 0.02 * np.sin(2 * np.pi * j / n + 2)
    r_ = T(rho).requires_grad_()
    J_ = T(J).requires_grad_()
    z_ = T(zeta).requires_grad_()
    se = torch.tensor(1.7, dtype=torch.float64, device=dev(), requires_grad=True)
    seps = torch.tensor(1.5, dtype=torch.float64, device=dev(), requires_grad=True)
    rho_T = LBMFunction.apply(r_, J_, z_, se, seps, steps, ckpt, None)
    loss = 0.5 * ((rho_T - T(tgt)) ** 2).sum()
    loss.backward()
    L, rb, Jb, zb, sb = oracle.gradient(rho, J, zeta, steps, tgt, po)
    assert rel(loss.item(), L) < 1e-11
    for got, want in ((r_.grad, rb), (J_.grad, Jb), (z_.grad, zb)):
        assert np.abs(got.cpu().numpy() - want).max() <= 1e-10 * np.abs(want).max()
    _, _, dpsi = lbm().coupled_rates(1.7)
    assert rel(se.grad.item(), sb[0] + sb[1] * dpsi) < 1e-9
    assert rel(seps.grad.item(), sb[2]) < 1e-9


@pytest.mark.parametrize("rate_device", ["cpu", "cuda"])
def test_batch_autograd_function(rate_device):
    """BatchLBMFunction on a small ragged batch: gradients of
    1/2 sum (rho(T) - target)^2 with respect to the initial fields and each
    lattice's s_e (total, through the coupling s_psi(s_e)) and s_eps, against
    the oracle's adjoint lattice by lattice, with the rates given on the CPU
    or on the GPU (their gradients come back on the same device)."""
    from paper_1802_02369_amd import workloads
    from paper_1802_02369_amd.autograd import BatchLBMFunction
    cfg = workloads.config_batched_adjoint(n_inst=5, steps=40, ckpt=9,
                                           lmin=90, lmax=700)
    bt, steps, ckpt = cfg["batch"], cfg["steps"], cfg["ckpt"]
    fl = bt.fields
    rng = np.random.default_rng(17)
    tgt = 1 + 0.01 * rng.standard_normal(bt.offsets[-1])
    rdev = torch.device("cpu") if rate_device == "cpu" else dev()
    se = torch.tensor(np.asarray(bt.s_e, dtype=np.float64), device=rdev,
                      requires_grad=True)
    seps = torch.full((bt.n_inst,), 1.5, dtype=torch.float64, device=rdev,
                      requires_grad=True)
    r_ = T(fl.rho).requires_grad_()
    J_ = T(fl.J).requires_grad_()
    z_ = T(fl.zeta).requires_grad_()
    rho_T = BatchLBMFunction.apply(r_, J_, z_, se, seps, list(bt.offsets), steps,
                                   ckpt, None)
    loss = 0.5 * ((rho_T - T(tgt)) ** 2).sum()
    loss.backward()
    assert se.grad.device == rdev and seps.grad.device == rdev
    for i in range(bt.n_inst):
        a, c = bt.offsets[i], bt.offsets[i + 1]
        x = bt.instance(i)
        po = oracle_params("paper", s_e=float(bt.s_e[i]))
        L, rb, Jb, zb, sb = oracle.gradient(x.rho, x.J, x.zeta, steps, tgt[a:c], po)
        for got, want in ((r_.grad[a:c], rb), (J_.grad[a:c], Jb), (z_.grad[a:c], zb)):
            assert np.abs(got.cpu().numpy() - want).max() <= 1e-10 * np.abs(want).max(), i
        _, _, dpsi = lbm().coupled_rates(float(bt.s_e[i]))
        want = np.array([sb[0] + sb[1] * dpsi, sb[2]])
        got = np.array([se.grad[i].item(), seps.grad[i].item()])
        # dL/ds_eps is ~1e-5 of dL/ds_e here: a sum of much larger terms
        # whose rounding depends on the summation order, hence the bound
        # relative to the whole rate gradient
        np.testing.assert_allclose(got, want, rtol=1e-9,
                                   atol=1e-10 * np.abs(sb).max(), err_msg=str(i))
    with pytest.raises(ValueError):
        BatchLBMFunction.apply(r_, J_, z_, 1.7, seps, list(bt.offsets), steps, ckpt, None)


def test_autograd_function_python_rates():
    """LBMFunction with the rates given as Python numbers: no rate
    gradients, field gradients as with tensor rates."""
    from paper_1802_02369_amd.autograd import LBMFunction
    po = oracle_params("paper", s_e=1.7)
    n, steps, ckpt = 96, 30, 7
    j = np.arange(n)
    rho = 1 + 0.05 * np.sin(2 * np.pi * j / n)
    J = 0.02 * np.cos(2 * np.pi * j / n)
    zeta = np.zeros(n)
    r_ = T(rho).requires_grad_()
    rho_T = LBMFunction.apply(r_, T(J), T(zeta), 1.7, 1.5, steps, ckpt, None)
    (0.5 * ((rho_T - 1.0) ** 2).sum()).backward()
    L, rb, Jb, zb, sb = oracle.gradient(rho, J, zeta, steps, np.ones(n), po)
    assert np.abs(r_.grad.cpu().numpy() - rb).max() <= 1e-10 * np.abs(rb).max()
