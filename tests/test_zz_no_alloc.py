"""mibh_forces_static (the force step on the library's static workspace, for
callers that cannot allocate) against mibh_forces on a caller's workspace:
the same kernels on the same inputs, so acc and pot must be equal bit for bit.
Two calls in a row, the second with a smaller input (the static workspace
keeps the first call's contents), then the limit: n above the maximum is
rejected with EINVAL before anything is enqueued."""
import numpy as np
import pytest

from gpu_helpers import gpu_context
from paper_1204_2280_amd import workloads as W

pytestmark = pytest.mark.gpu


def _run_static(pos, mass, theta):
    import torch
    from paper_1204_2280_amd import mibh
    p = torch.from_numpy(pos).cuda()
    m = torch.from_numpy(mass).cuda()
    acc = torch.full((len(mass), 3), float("nan"), device="cuda")
    pot = torch.full((len(mass),), float("nan"), device="cuda")
    mibh.forces_static(p, m, theta, acc, pot)
    torch.cuda.synchronize()
    return acc.cpu().numpy(), pot.cpu().numpy()


def _run_context(pos, mass, theta):
    import torch
    ctx = gpu_context(len(mass), anchor_up=0)  # the static workspace walks from the root
    acc, pot = ctx.forces(torch.from_numpy(pos).cuda(), torch.from_numpy(mass).cuda(), theta)
    ctx.sync()
    return acc.cpu().numpy(), pot.cpu().numpy()


def test_static_forces_equal_context_forces_on_two_calls():
    gpu_context(16)  # torch's HIP runtime starts before the library's, as in every GPU test
    from paper_1204_2280_amd import mibh
    assert mibh.static_n_max() == 32768
    cases = [(W.plummer(32768, 1, with_velocities=False), 0.75), (W.plummer(5003, 21, with_velocities=False), 0.5)]
    for (pos, _, mass), theta in cases:
        n = len(mass)
        print(f"[gpu] static workspace: n={n} theta={theta}", flush=True)
        a_s, p_s = _run_static(pos, mass, theta)
        a_c, p_c = _run_context(pos, mass, theta)
        assert np.isfinite(a_s).all() and np.isfinite(p_s).all()
        np.testing.assert_array_equal(a_s, a_c)
        np.testing.assert_array_equal(p_s, p_c)


def test_static_forces_reject_sizes_beyond_the_limit():
    import torch
    gpu_context(16)
    from paper_1204_2280_amd import mibh
    n = mibh.static_n_max() + 1
    p = torch.zeros((n, 3), device="cuda")
    m = torch.ones(n, device="cuda")
    acc = torch.empty((n, 3), device="cuda")
    pot = torch.empty(n, device="cuda")
    with pytest.raises(mibh.MibhError) as ei:
        mibh.forces_static(p, m, 0.75, acc, pot)
    assert ei.value.status == -1 and "static workspace" in str(ei.value)
    with pytest.raises(mibh.MibhError):
        mibh.forces_static(p[:10], m[:10], 0.0, acc[:10], pot[:10])
