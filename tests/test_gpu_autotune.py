"""The autotuner (adscl_autotune): it picks, per grid size, one of the compiled
configurations at the tightest lane capacity, reports a positive rate, and a
Batch created after an applied tuning uses that configuration and still
matches the oracle."""
import numpy as np
import pytest

import oracle as O
from paper_1706_07413_amd import adscl

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _clear_table():
    adscl.autotune_clear()
    yield
    adscl.autotune_clear()


def test_autotune_picks_a_configuration_at_the_tightest_capacity():
    res = adscl.autotune([257, 1025, 1537], steps=16, apply=False)
    for N, (P, W, rate) in res.items():
        cap = 64 * P * W
        assert cap >= N - 1 and cap < 2 * (N - 1), (N, P, W)
        assert rate > 0.0
    # not applied: the default rule still decides
    b = adscl.Batch([1025])
    classes, cls = b.kernel_stats()
    assert (classes[cls[0]]["P"], classes[cls[0]]["W"]) == (4, 4)


def test_applied_choice_is_used_and_matches_the_oracle():
    res = adscl.autotune([1025], steps=16, apply=True)
    P, W, _ = res[1025]
    b = adscl.Batch([1025, 1025], a_collapse=0.02)
    b.init_gaussian(np.array([6.0, 3.0]), np.array([0.15, 0.2]))
    b.step(100, 1e9)
    classes, cls = b.kernel_stats()
    assert (classes[cls[0]]["P"], classes[cls[0]]["W"]) == (P, W)
    s = b.get_state()
    for i, (eps, sig) in enumerate(((6.0, 0.15), (3.0, 0.2))):
        Phi, Pi = O.init_gaussian(1025, eps, sig)
        ref = O.evolve(Phi, Pi, 100)
        for f in ("Phi", "Pi", "A", "delta", "m"):
            g = b.split(s[f].cpu().numpy())[i]
            e = np.max(np.abs(g - ref[f])) / max(np.max(np.abs(ref[f])), 1e-300)
            assert e <= 1e-11, (i, f, e)
