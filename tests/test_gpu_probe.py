"""The float32 fused multiply-add probe that sets the walk's measured ceiling:
every accumulator gains a * b per iteration.  With a * b a power of two and
all values on its grid the sums are exact (v_n = v_0 + n a b); otherwise each
step rounds once and the sum stays within n half-ulps of the exact one."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _start(blocks):
    lane = np.arange(blocks * 64)[:, None]
    j = np.arange(32)[None, :]
    return ((lane % 256) / 256.0 + j / 32.0).astype(np.float32)


def _run(blocks, iters, a, b):
    import torch
    from paper_1204_2280_amd import mibh
    out = torch.full((blocks * 2048,), -1.0, dtype=torch.float32, device="cuda")
    mibh.fma_probe(out, blocks, iters, a, b)
    torch.cuda.synchronize()
    return out.cpu().numpy().reshape(blocks * 64, 32)


@pytest.mark.parametrize("iters,a,b", [(1000, 0.5, 2.0 ** -12), (0, 0.3, 0.7), (37, 0.0, 5.0), (513, -2.0, 2.0 ** -10)])
def test_exact_sums(iters, a, b):
    got = _run(3, iters, a, b).astype(np.float64)
    ref = _start(3).astype(np.float64) + iters * (a * b)
    np.testing.assert_array_equal(got, ref)


def test_rounded_sums():
    iters, a, b = 2000, np.float32(0.1), np.float32(0.3)
    got = _run(2, iters, float(a), float(b)).astype(np.float64)
    ref = _start(2).astype(np.float64) + iters * (float(a) * float(b))
    # one rounding per step, |v| < 64: at most iters * 2^-19 apart
    assert np.max(np.abs(got - ref)) <= iters * 2.0 ** -19


def test_rejects_bad_arguments():
    import torch
    from paper_1204_2280_amd import mibh
    out = torch.empty(2048, dtype=torch.float32, device="cuda")
    with pytest.raises(ValueError):
        mibh.fma_probe(out, 2, 10)
    with pytest.raises(mibh.MibhError):
        mibh.fma_probe(out, 1, -1)
