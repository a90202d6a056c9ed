"""The allocation-free entry point adscl_constraints_noalloc against
adscl_constraints, through the C ABI: same kernels, so the outputs must agree
bit for bit (NaN where the other has NaN), on two calls in a row (the second on
a smaller batch, so the fixed scratch holds the first call's data), with host
and device outputs; a batch beyond the fixed scratch is rejected."""
import numpy as np
import pytest

from paper_1706_07413_amd import adscl

pytestmark = pytest.mark.gpu


def same(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return a.shape == b.shape and np.array_equal(np.isnan(a), np.isnan(b)) and \
        np.array_equal(a[~np.isnan(a)], b[~np.isnan(b)])


def run_case(Ns, eps, sig, steps, gauge):
    import torch
    b = adscl.Batch(Ns, gauge=gauge, a_collapse=0.0)
    b.init_gaussian(np.asarray(eps, float), np.asarray(sig, float))
    b.step(steps, 1e9)
    ref = b.constraints()
    got = b.constraints_noalloc()
    dev = torch.full((len(Ns), 5), -1.0, dtype=torch.float64, device="cuda")
    b.constraints_noalloc(dev)
    b.close()
    assert same(got, ref), (got, ref)
    assert same(dev.cpu().numpy(), ref)
    assert np.all(np.isfinite(ref))
    return ref


def test_noalloc_constraints_match_twice_second_smaller():
    big = run_case([1025, 4097, 777, 16385, 257] * 4, [3.0, 5.0, 2.0, 4.0, 6.0] * 4,
                   [0.2, 0.15, 0.25, 0.2, 0.3] * 4, 120, adscl.GAUGE_BOUNDARY)
    small = run_case([129, 65], [4.0, 2.0], [0.2, 0.25], 60, adscl.GAUGE_ORIGIN)
    assert big.shape == (20, 5) and small.shape == (2, 5)


def test_noalloc_frozen_gives_nan_residual_like_the_allocating_call():
    b = adscl.Batch([129, 513], flags=adscl.FROZEN_METRIC, n_modes=2)
    b.init_modes(np.array([0.5, 0.2]), np.array([[1.0, 0.3], [0.2, 1.0]]))
    b.step(10, 1e9)
    ref, got = b.constraints(), b.constraints_noalloc()
    b.close()
    assert same(got, ref) and np.all(np.isnan(got[:, 2]))


def test_noalloc_rejects_a_batch_beyond_the_fixed_scratch():
    Ns = [65537] * 17  # 2 * 1114129 + 85 doubles > 2^21
    b = adscl.Batch(Ns)
    b.init_gaussian(np.full(17, 1.0), np.full(17, 0.2))
    with pytest.raises(adscl.AdsclError) as e:
        b.constraints_noalloc()
    assert e.value.code == adscl.EINVAL and "fixed scratch" in str(e.value)
    b.close()
