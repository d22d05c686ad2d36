"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/lbm.h declares, and rejects bad arguments before any
HIP call."""
import ctypes
import os
import re

import pytest

from paper_1802_02369_amd import lbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_\w+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = lbm.lib()
    names = declared_functions()
    assert len(names) >= 12
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_coupled_rates_host():
    s_psi, s_eps, d = lbm.coupled_rates(1.9, 1.4, 1.0)
    # sigma_psi = 1.5 gamma / Pr sigma_e (section 7)
    assert 1 / s_psi - 0.5 == pytest.approx(1.5 * 1.4 * (1 / 1.9 - 0.5), rel=1e-14)
    assert s_eps == 1.5
    h = 1e-6
    fd = (lbm.coupled_rates(1.9 + h)[0] - lbm.coupled_rates(1.9 - h)[0]) / (2 * h)
    assert d == pytest.approx(fd, rel=1e-8)
    with pytest.raises(lbm.LBMError):
        lbm.coupled_rates(2.0)
    with pytest.raises(lbm.LBMError):
        lbm.coupled_rates(1.0, gamma=1.0)


def _init(n, **kw):
    p = lbm.Params(**kw).c() if "s_psi" in kw else lbm.Params(s_psi=1.0, **kw).c()
    h = ctypes.c_void_p()
    rc = lbm.lib().lbm_init(ctypes.byref(h), n, ctypes.byref(p), None)
    return rc, h


@pytest.mark.parametrize("n,kw", [
    (2, {}),
    (0, {}),
    ((1 << 36) + 1, {}),
    (16, dict(s_e=2.0)),
    (16, dict(s_e=0.0)),
    (16, dict(s_eps=-1.0)),
    (16, dict(gamma=1.0)),
    (16, dict(cp=0.0)),
    (16, dict(c0=-0.5)),
    (16, dict(prandtl=float("nan"))),
    (16, dict(source_on=2)),
    (16, dict(eq_kind=3)),
    (16, dict(eq_kind=1, lam=2.0)),
    (16, dict(flags=2)),
    (16, dict(flags=-1)),
])
def test_init_rejects_bad_arguments(n, kw):
    rc, h = _init(n, **kw)
    assert rc == lbm.LBM_EINVAL
    assert not h.value
    assert lbm.lib().lbm_last_error()


def test_params_struct_matches_header():
    """The binding's lbm_params record has the header's fields, in order,
    with the header's types."""
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    body = re.search(r"typedef struct lbm_params \{(.*?)\} lbm_params;", text,
                     flags=re.S).group(1)
    fields = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        ctype, names = decl.split(None, 1)
        fields += [(n.strip(), ctype) for n in names.split(",")]
    want = {"double": ctypes.c_double, "int32_t": ctypes.c_int32}
    got = lbm.CParams._fields_
    assert len(got) == len(fields)
    for (gn, gt), (hn, ht) in zip(got, fields):
        assert gt is want[ht], (gn, hn)
        assert gn == hn or (gn, hn) == ("lam", "lambda")


def test_flags_validation_host():
    p = lbm.Params(s_psi=1.0, flags=lbm.LBM_CHECK_FINITE).c()
    h = ctypes.c_void_p()
    assert lbm.lib().lbm_init(ctypes.byref(h), 16, ctypes.byref(p), None) == lbm.LBM_OK
    lbm.lib().lbm_destroy(h)
    p.reserved = 1
    h = ctypes.c_void_p()
    assert lbm.lib().lbm_init(ctypes.byref(h), 16, ctypes.byref(p), None) == lbm.LBM_EINVAL
    assert not h.value


def test_init_and_workspace_and_tuning_host():
    rc, h = _init(1000)
    assert rc == lbm.LBM_OK and h.value
    L = lbm.lib()
    nb = L.lbm_workspace_bytes(h, lbm.WS_STEP)
    assert nb >= 6 * 1000 * 8
    assert L.lbm_workspace_bytes(None, lbm.WS_STEP) == 0
    for bad in [(lbm.KERNEL_BLOCKED, 3, 4, 4), (lbm.KERNEL_BLOCKED, 4, 256, 4),
                (lbm.KERNEL_BLOCKED, 4, 0, 4), (lbm.KERNEL_BLOCKED, 2, 4, 3),
                (lbm.KERNEL_BLOCKED, 6, 4, 4), (lbm.KERNEL_BLOCKED, 16, 4, 4),
                (lbm.KERNEL_BLOCKED, 8, 512, 4), (7, 2, 4, 4)]:
        t = lbm.CTuning(*bad)
        assert L.lbm_set_tuning(h, ctypes.byref(t)) == lbm.LBM_EINVAL
    t = lbm.CTuning(lbm.KERNEL_BLOCKED, 4, 15, 2)
    assert L.lbm_set_tuning(h, ctypes.byref(t)) == lbm.LBM_OK
    t2 = lbm.CTuning()
    assert L.lbm_get_tuning(h, ctypes.byref(t2)) == lbm.LBM_OK
    assert (t2.nodes_per_lane, t2.steps_per_launch, t2.waves_per_group) == (4, 15, 2)
    # step argument validation fails before touching the device
    assert L.lbm_step(h, None, None, 0, 1) == lbm.LBM_EINVAL
    assert L.lbm_step(h, ctypes.c_void_p(4096), ctypes.c_void_p(1 << 20), 8,
                      1) == lbm.LBM_EWORKSPACE
    assert L.lbm_step(h, ctypes.c_void_p(4096), ctypes.c_void_p(4096 + 8),
                      nb, 1) == lbm.LBM_EINVAL  # overlap
    assert L.lbm_step(h, ctypes.c_void_p(4096), ctypes.c_void_p(1 << 30), nb,
                      -1) == lbm.LBM_EINVAL
    # nsteps = 0 is a no-op that never touches memory
    assert L.lbm_step(h, ctypes.c_void_p(4096), ctypes.c_void_p(1 << 30), nb,
                      0) == lbm.LBM_OK
    L.lbm_destroy(h)


@pytest.mark.parametrize("n,shape", [
    (1 << 24, (8, 40, 4)),   # wide tiles: 9119 tiles of 1840 output nodes
    (1 << 21, (8, 40, 4)),
    (1 << 20, (4, 24, 4)),   # too few P = 8 tiles for 4 workgroups per CU
    (1 << 19, (2, 16, 4)),
    (40000, (2, 16, 1)),     # small lattices: the narrowest tile, K = 16
    (8192, (1, 13, 1)),      # up to 16384 nodes: one node per lane
    (3, (1, 13, 1))])
def test_default_tuning_follows_lattice_length(n, shape):
    rc, h = _init(n)
    assert rc == lbm.LBM_OK
    t = lbm.CTuning()
    assert lbm.lib().lbm_get_tuning(h, ctypes.byref(t)) == lbm.LBM_OK
    assert (t.kernel, t.nodes_per_lane, t.steps_per_launch,
            t.waves_per_group) == (lbm.KERNEL_BLOCKED,) + shape
    lbm.lib().lbm_destroy(h)


def test_batch_default_tuning_uses_mean_length():
    """4096 lattices of ~4.6k nodes: P = 8 tiles (2000 wide) would waste a
    third of each lattice's work, so the default is the 1000-wide P = 4 tile."""
    n_inst, L = 4096, 4615
    offs = (ctypes.c_int64 * (n_inst + 1))(*[i * L for i in range(n_inst + 1)])
    p = lbm.Params(s_psi=1.0).c()
    ps = (type(p) * n_inst)(*([p] * n_inst))
    b = ctypes.c_void_p()
    assert lbm.lib().lbm_batch_init(ctypes.byref(b), n_inst, offs, ps, None) == lbm.LBM_OK
    t = lbm.CTuning()
    assert lbm.lib().lbm_batch_get_tuning(b, ctypes.byref(t)) == lbm.LBM_OK
    assert (t.nodes_per_lane, t.steps_per_launch, t.waves_per_group) == (4, 24, 4)
    lbm.lib().lbm_batch_destroy(b)


def test_batch_groups_validation_host():
    """Shape-group arguments are checked before any HIP call."""
    n_inst, L = 6, 100
    offs = (ctypes.c_int64 * (n_inst + 1))(*[i * L for i in range(n_inst + 1)])
    p = lbm.Params(s_psi=1.0).c()
    ps = (type(p) * n_inst)(*([p] * n_inst))
    b = ctypes.c_void_p()
    Lb = lbm.lib()
    assert Lb.lbm_batch_init(ctypes.byref(b), n_inst, offs, ps, None) == lbm.LBM_OK
    shapes = (lbm.CTuning * 2)(lbm.CTuning(lbm.KERNEL_BLOCKED, 2, 8, 1),
                               lbm.CTuning(lbm.KERNEL_BLOCKED, 4, 8, 2))
    good = (ctypes.c_int32 * n_inst)(0, 1, 0, 1, 0, 1)
    bad = (ctypes.c_int32 * n_inst)(0, 1, 2, 1, 0, 1)
    i32 = ctypes.POINTER(ctypes.c_int32)
    assert Lb.lbm_batch_set_groups(None, 2, shapes, good) == lbm.LBM_EINVAL
    assert Lb.lbm_batch_set_groups(b, lbm.MAX_GROUPS + 1, shapes, good) == lbm.LBM_EINVAL
    assert Lb.lbm_batch_set_groups(b, -1, shapes, good) == lbm.LBM_EINVAL
    assert Lb.lbm_batch_set_groups(b, 2, None, good) == lbm.LBM_EINVAL
    assert Lb.lbm_batch_set_groups(b, 2, shapes, None) == lbm.LBM_EINVAL
    assert Lb.lbm_batch_set_groups(b, 2, shapes, bad) == lbm.LBM_EINVAL
    badshape = (lbm.CTuning * 2)(lbm.CTuning(lbm.KERNEL_BLOCKED, 3, 8, 1),
                                 lbm.CTuning(lbm.KERNEL_BLOCKED, 4, 8, 2))
    assert Lb.lbm_batch_set_groups(b, 2, badshape, good) == lbm.LBM_EINVAL
    assert Lb.lbm_batch_set_groups(b, 0, None, None) == lbm.LBM_OK
    n = ctypes.c_int32(-1)
    assert Lb.lbm_batch_get_groups(b, ctypes.byref(n), None, None) == lbm.LBM_OK
    assert n.value == 0
    assert Lb.lbm_batch_get_groups(b, None, None, None) == lbm.LBM_EINVAL
    Lb.lbm_batch_destroy(b)


@pytest.mark.parametrize("shape,ok", [
    ((8, 40, 4), True), ((8, 9, 8), True), ((8, 511, 8), True),
    ((8, 512, 8), False), ((4, 63, 1), True), ((2, 60, 8), True)])
def test_blocked_adjoint_shape_check_host(shape, ok):
    """Workspace sizes exist for every valid forward shape; the checkpointed
    forward with the blocked reverse kernel refuses, before any HIP call, a
    shape whose halo leaves the reverse tiles (64 P W nodes: P = 2, else
    P = 4 with 8 wavefronts for halos of 4K >= 128 W) no interior:
    4K >= 2048, possible only for P = 8 with 8 wavefronts."""
    rc, h = _init(5000)
    assert rc == lbm.LBM_OK
    L = lbm.lib()
    P, K, W = shape
    t = lbm.CTuning(lbm.KERNEL_BLOCKED, P, K, W)
    assert L.lbm_set_tuning(h, ctypes.byref(t)) == lbm.LBM_OK
    assert L.lbm_set_adjoint_kernel(h, lbm.KERNEL_BLOCKED) == lbm.LBM_OK
    nb = L.lbm_adjoint_workspace_bytes(h, 10, 5)
    assert nb >= 6 * 5000 * 8
    if not ok:
        rc = L.lbm_forward_ckpt(h, ctypes.c_void_p(4096),
                                ctypes.c_void_p(1 << 40), nb, 10, 5)
        assert rc == lbm.LBM_ENOTSUP
        assert b"halo" in L.lbm_last_error()
    L.lbm_destroy(h)


def test_one_node_per_lane_needs_one_wavefront_host():
    rc, h = _init(1000)
    assert rc == lbm.LBM_OK
    L = lbm.lib()
    for P, K, W, ok in [(1, 12, 1, True), (1, 15, 1, True), (1, 16, 1, False),
                        (1, 4, 2, False), (3, 4, 1, False)]:
        t = lbm.CTuning(lbm.KERNEL_BLOCKED, P, K, W)
        rc = L.lbm_set_tuning(h, ctypes.byref(t))
        assert (rc == lbm.LBM_OK) == ok, (P, K, W)
    L.lbm_destroy(h)


def test_recompute_stride_host():
    """Stride 2 keeps floor((C-1)/2) of the C-1 recomputed states of a
    segment (twice, on this small pipelined problem); it needs K >= 2 and
    the blocked reverse kernel, and strides outside 0..2 are refused."""
    n, steps, C = 5000, 100, 20
    rc, h = _init(n)
    assert rc == lbm.LBM_OK
    L = lbm.lib()
    state = 6 * n * 8
    t = lbm.CTuning(lbm.KERNEL_BLOCKED, 2, 16, 1)
    assert L.lbm_set_tuning(h, ctypes.byref(t)) == lbm.LBM_OK
    auto = L.lbm_adjoint_workspace_bytes(h, steps, C)
    assert L.lbm_set_recompute_stride(h, 1) == lbm.LBM_OK
    assert L.lbm_adjoint_workspace_bytes(h, steps, C) == auto
    assert L.lbm_set_recompute_stride(h, 2) == lbm.LBM_OK
    two = L.lbm_adjoint_workspace_bytes(h, steps, C)
    assert abs((auto - two) - 2 * (19 - 9) * state) < 256
    assert L.lbm_set_adjoint_kernel(h, lbm.KERNEL_PLAIN) == lbm.LBM_OK
    assert L.lbm_adjoint_workspace_bytes(h, steps, C) > two
    assert L.lbm_set_adjoint_kernel(h, lbm.KERNEL_AUTO) == lbm.LBM_OK
    t = lbm.CTuning(lbm.KERNEL_BLOCKED, 2, 1, 1)
    assert L.lbm_set_tuning(h, ctypes.byref(t)) == lbm.LBM_OK
    k1 = L.lbm_adjoint_workspace_bytes(h, steps, C)
    assert L.lbm_set_recompute_stride(h, 1) == lbm.LBM_OK
    assert L.lbm_adjoint_workspace_bytes(h, steps, C) == k1
    for bad in (-1, 3):
        assert L.lbm_set_recompute_stride(h, bad) == lbm.LBM_EINVAL
        assert b"stride" in L.lbm_last_error()
    assert L.lbm_batch_set_recompute_stride(None, 1) == lbm.LBM_EINVAL
    L.lbm_destroy(h)


@pytest.mark.parametrize("n_inst,Ln,auto", [(256, 8000, 2), (4, 1000, 1)])
def test_recompute_stride_automatic_host(n_inst, Ln, auto):
    """The automatic recompute stride is 2 where the blocked reverse
    launches fill the chip (256 lattices of 8000 nodes at P2/W8: about
    17000 wavefronts) and 1 on a small batch (launch-bound, pipelined)."""
    L = lbm.lib()
    offs = (ctypes.c_int64 * (n_inst + 1))(*[i * Ln for i in range(n_inst + 1)])
    p = lbm.Params(s_psi=1.0).c()
    ps = (type(p) * n_inst)(*([p] * n_inst))
    b = ctypes.c_void_p()
    assert L.lbm_batch_init(ctypes.byref(b), n_inst, offs, ps, None) == lbm.LBM_OK
    t = lbm.CTuning(lbm.KERNEL_BLOCKED, 4, 16, 4)
    assert L.lbm_batch_set_tuning(b, ctypes.byref(t)) == lbm.LBM_OK
    ws = {}
    for stride in (1, 2, 0):
        assert L.lbm_batch_set_recompute_stride(b, stride) == lbm.LBM_OK
        ws[stride] = L.lbm_batch_adjoint_workspace_bytes(b, 200, 50)
    assert ws[2] < ws[1]
    assert ws[0] == ws[auto]
    L.lbm_batch_destroy(b)


@pytest.mark.parametrize("kw,shape", [
    (dict(), (8, 40, 4)),
    (dict(eq_kind=1), (4, 24, 4)),
    (dict(eq_kind=2, source_on=0), (4, 24, 4))])
def test_default_tuning_follows_equilibria(kw, shape):
    """Lattices whose kernels select the equilibria per lattice (eq_kind 1,
    2) default to P = 4: at P = 8 those kernels need more than 256 VGPRs."""
    rc, h = _init(1 << 24, **kw)
    assert rc == lbm.LBM_OK
    t = lbm.CTuning()
    assert lbm.lib().lbm_get_tuning(h, ctypes.byref(t)) == lbm.LBM_OK
    assert (t.nodes_per_lane, t.steps_per_launch, t.waves_per_group) == shape
    lbm.lib().lbm_destroy(h)


def test_set_params_rederives_only_the_default_tuning():
    L = lbm.lib()
    rc, h = _init(1 << 24)
    assert rc == lbm.LBM_OK
    t = lbm.CTuning()
    p1 = lbm.Params(s_psi=1.0, eq_kind=1).c()
    assert L.lbm_set_params(h, ctypes.byref(p1)) == lbm.LBM_OK
    L.lbm_get_tuning(h, ctypes.byref(t))
    assert (t.nodes_per_lane, t.steps_per_launch, t.waves_per_group) == (4, 24, 4)
    p0 = lbm.Params(s_psi=1.0).c()
    assert L.lbm_set_params(h, ctypes.byref(p0)) == lbm.LBM_OK
    L.lbm_get_tuning(h, ctypes.byref(t))
    assert (t.nodes_per_lane, t.steps_per_launch, t.waves_per_group) == (8, 40, 4)
    mine = lbm.CTuning(lbm.KERNEL_BLOCKED, 2, 8, 2)
    assert L.lbm_set_tuning(h, ctypes.byref(mine)) == lbm.LBM_OK
    assert L.lbm_set_params(h, ctypes.byref(p1)) == lbm.LBM_OK
    L.lbm_get_tuning(h, ctypes.byref(t))
    assert (t.nodes_per_lane, t.steps_per_launch, t.waves_per_group) == (2, 8, 2)
    L.lbm_destroy(h)


def test_batch_default_tuning_follows_equilibria():
    """One lattice with linear equilibria puts the whole batch on the
    per-lattice equilibrium kernels, hence the P = 4 defaults."""
    n_inst, Ln = 4096, 4615
    offs = (ctypes.c_int64 * (n_inst + 1))(*[i * Ln for i in range(n_inst + 1)])
    p = lbm.Params(s_psi=1.0).c()
    q = lbm.Params(s_psi=1.0, eq_kind=1).c()
    ps = (type(p) * n_inst)(*([q] + [p] * (n_inst - 1)))
    b = ctypes.c_void_p()
    assert lbm.lib().lbm_batch_init(ctypes.byref(b), n_inst, offs, ps, None) == lbm.LBM_OK
    t = lbm.CTuning()
    assert lbm.lib().lbm_batch_get_tuning(b, ctypes.byref(t)) == lbm.LBM_OK
    assert (t.nodes_per_lane, t.steps_per_launch, t.waves_per_group) == (4, 24, 4)
    lbm.lib().lbm_batch_destroy(b)
