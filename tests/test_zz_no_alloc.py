"""lbm_step_noalloc (the entry point for callers that cannot allocate):
through the C ABI, two calls in a row, the second on a smaller lattice, each
bitwise equal to lbm_step with a caller workspace on the same input, and the
size limit."""
import ctypes

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


def test_step_noalloc_matches_step():
    from paper_1802_02369_amd import lbm
    L = lbm.lib()
    rng = np.random.default_rng(77)
    po = oracle_params("odd")
    # a lattice near the limit, then a smaller one; odd and even step counts
    # (an odd number of launches ends with a copy out of the scratch)
    for n, steps, tuning in ((lbm.NOALLOC_MAX_NODES - 5, 24, None),
                             (3001, 7, (2, 8, 4)),
                             (257, 1, None)):
        print(f"step_noalloc n={n} steps={steps} tuning={tuning}", flush=True)
        f0 = random_state(rng, n, po, amp=0.1, u=0.05, ds=0.1)
        lat = lbm.Lattice(n, gpu_params(po))
        if tuning:
            lat.set_tuning(nodes_per_lane=tuning[0], steps_per_launch=tuning[1],
                           waves_per_group=tuning[2])
        want = torch.from_numpy(f0).to(dev())
        lat.step(want, steps)
        got = torch.from_numpy(f0).to(dev())
        rc = L.lbm_step_noalloc(lat._h, ctypes.c_void_p(got.data_ptr()), steps)
        assert rc == lbm.LBM_OK, L.lbm_last_error().decode()
        torch.cuda.synchronize()
        assert torch.equal(got, want)
        if n <= 5000:
            assert max_err(got.cpu().numpy(), oracle.run(f0, steps, po)) < TOL


def test_step_noalloc_rejects_lattices_beyond_its_scratch():
    from paper_1802_02369_amd import lbm
    po = oracle_params("paper")
    n = lbm.NOALLOC_MAX_NODES + 1
    lat = lbm.Lattice(n, gpu_params(po))
    f = torch.empty((6, n), dtype=torch.float64, device=dev())
    rc = lbm.lib().lbm_step_noalloc(lat._h, ctypes.c_void_p(f.data_ptr()), 3)
    assert rc == lbm.LBM_EINVAL
    assert b"LBM_NOALLOC_MAX_NODES" in lbm.lib().lbm_last_error()


def test_step_noalloc_check_finite():
    """The failure record of LBM_CHECK_FINITE also lives in the scratch: a
    NaN is reported, and the next call starts from a clean record."""
    from paper_1802_02369_amd import lbm
    rng = np.random.default_rng(78)
    po = oracle_params("paper")
    n = 4000
    f0 = random_state(rng, n, po, amp=0.1, u=0.05, ds=0.1)
    p = gpu_params(po)
    p.flags = lbm.LBM_CHECK_FINITE
    lat = lbm.Lattice(n, p)
    f = torch.from_numpy(f0).to(dev())
    f[4, 1234] = float("nan")
    with pytest.raises(lbm.LBMError) as e:
        lat.step_noalloc(f, 20)
    assert e.value.code == lbm.LBM_ENONFINITE
    f = torch.from_numpy(f0).to(dev())
    lat.step_noalloc(f, 20)
    ref = torch.from_numpy(f0).to(dev())
    lat.step(ref, 20)
    assert torch.equal(f, ref)
