"""GPU parity of the scheme options of Sec. II against the oracle: second- and
third-order (Shu-Osher SSP) Runge-Kutta, and A evolved by Eq. (4) with its
periodic re-integration from Eq. (5), alone or with any of the three orders.

Same bar as the classical path: every field (Phi, Pi, A, delta, m) at <= 1e-11
relative max-norm (absolute 1e-13 below a norm of 1e-12), steps and states
exact.  The evolved A is part of the state, so the runs cross segment and call
boundaries (snapshots, then a second call) where it must persist."""
import numpy as np
import pytest

import oracle as O
from paper_1706_07413_amd import adscl

pytestmark = pytest.mark.gpu

TOL = 1e-11
FIELDS = ("Phi", "Pi", "A", "delta", "m")
# one grid per one-workgroup configuration of the scheme kernels, full and ragged
NS = [65, 257, 513, 777, 1025, 2049, 4097]


def rel(g, o):
    n = np.max(np.abs(o))
    d = np.max(np.abs(np.asarray(g) - np.asarray(o)))
    return d / 1e-13 * TOL if n < 1e-12 else d / n


def check(g, o, what):
    e = rel(g, o)
    assert e <= TOL, "%s: relative max-norm error %.3e" % (what, e)


@pytest.mark.parametrize("rk,K,gauge", [(2, 0, 0), (3, 0, 0), (3, 0, 1), (2, 3, 0), (3, 1, 0), (3, 7, 1),
                                        (4, 5, 0)])
def test_scheme_matches_oracle_across_segments_and_calls(rk, K, gauge):
    import torch
    rng = np.random.default_rng(100 + 10 * rk + K)
    eps = rng.uniform(2.0, 6.0, len(NS))
    sig = rng.uniform(0.15, 0.3, len(NS))
    b = adscl.Batch(NS, gauge=gauge, a_collapse=0.0, rk_order=rk, a_reint=K)
    b.init_gaussian(eps, sig)
    n1, n2, every, slots = 200, 237, 50, 5
    snaps = torch.zeros((slots, 5, b.total), dtype=torch.float64, device="cuda")
    b.step(n1, 1e9, snap_every=every, snaps=snaps)
    sn = snaps.cpu().numpy()
    b.step(n2 - n1, 1e9)
    st = {k: v.cpu().numpy() for k, v in b.get_state().items()}
    s = b.status()
    for i, N in enumerate(NS):
        Phi, Pi = O.init_gaussian(N, eps[i], sig[i])
        r1 = O.evolve_scheme(Phi, Pi, n1, rk=rk, a_reint=K, gauge=gauge, snap_every=every, n_slots=slots)
        for sl in range(slots):
            for f in range(5):
                check(b.split(sn[sl, f])[i], r1["snaps"][sl, f], "rk%d K%d N=%d slot %d %s" % (rk, K, N, sl, FIELDS[f]))
        r2 = O.evolve_scheme(r1["Phi"], r1["Pi"], n2, n0=n1, A=r1["A"], rk=rk, a_reint=K, gauge=gauge)
        assert s["steps"][i] == r2["steps"] == n2
        assert s["state"][i] == adscl.RUNNING
        for f in FIELDS:
            check(b.split(st[f])[i], r2[f], "rk%d K%d N=%d %s" % (rk, K, N, f))
    b.close()


@pytest.mark.parametrize("rk,K", [(3, 0), (3, 16), (2, 4)])
def test_scheme_collapse_step_matches_oracle(rk, K):
    """Strong pulses that fall below min A = 0.2 within a few hundred steps; with
    A evolved the test is on the evolved A."""
    Ns = [257, 513, 1025]
    eps = np.array([20.0, 30.0, 20.0])
    sig = np.array([0.2, 0.15, 0.25])
    b = adscl.Batch(Ns, a_collapse=0.2, rk_order=rk, a_reint=K)
    b.init_gaussian(eps, sig)
    b.step(3000, 1e9)
    s = b.status()
    st = {k: v.cpu().numpy() for k, v in b.get_state().items()}
    for i, N in enumerate(Ns):
        Phi, Pi = O.init_gaussian(N, eps[i], sig[i])
        r = O.evolve_scheme(Phi, Pi, 3000, rk=rk, a_reint=K, a_collapse=0.2)
        assert r["state"] == O.COLLAPSED, (N, r["steps"])
        assert s["state"][i] == adscl.COLLAPSED and s["steps"][i] == r["steps"], (N, s["steps"][i], r["steps"])
        assert abs(s["t_c"][i] - r["t_c"]) <= 1e-12 * r["t_c"]
        for f in FIELDS:
            check(b.split(st[f])[i], r[f], "collapse rk%d K%d N=%d %s" % (rk, K, N, f))
    b.close()


def test_rk3_frozen_metric_matches_oracle():
    Ns = [129, 1025, 4097]
    c = np.array([[1.0, -0.5, 0.25, 0.1]] * 3)
    b = adscl.Batch(Ns, n_modes=4, flags=adscl.FROZEN_METRIC, rk_order=3)
    b.init_modes(np.ones(3), c)
    b.step(300, 1e9)
    st = {k: v.cpu().numpy() for k, v in b.get_state().items()}
    for i, N in enumerate(Ns):
        Phi, Pi = O.init_modes(N, 1.0, c[i])
        r = O.evolve_scheme(Phi, Pi, 300, rk=3, frozen=True)
        for f in ("Phi", "Pi"):
            check(b.split(st[f])[i], r[f], "frozen rk3 N=%d %s" % (N, f))
    b.close()


def test_scheme_options_refuse_the_adjoint():
    b = adscl.Batch([65], n_modes=4, rk_order=3)
    with pytest.raises(adscl.AdsclError) as e:
        b.adjoint(np.array([0.5]), np.array([[1.0, 0.2, 0.0, 0.0]]), 4, 0.01, 8)
    assert e.value.code == adscl.EUNSUPPORTED
    b.close()


@pytest.mark.parametrize("rk,K", [(3, 0), (3, 5), (2, 3), (4, 7)])
def test_scheme_on_multi_workgroup_grids(rk, K):
    """The scheme options on grids above 4097 points (chunks of 2048 points over
    several workgroups; 10001 leaves a short last chunk) next to a small grid,
    across a snapshot segment and a second call."""
    import torch
    Ns = [6145, 257, 10001]
    eps = np.array([5.0, 3.0, 6.0])
    sig = np.array([0.2, 0.25, 0.18])
    b = adscl.Batch(Ns, a_collapse=0.0, rk_order=rk, a_reint=K)
    b.init_gaussian(eps, sig)
    n1, n2, every, slots = 120, 157, 40, 4
    snaps = torch.zeros((slots, 5, b.total), dtype=torch.float64, device="cuda")
    b.step(n1, 1e9, snap_every=every, snaps=snaps)
    sn = snaps.cpu().numpy()
    b.step(n2 - n1, 1e9)
    st = {k: v.cpu().numpy() for k, v in b.get_state().items()}
    s = b.status()
    b.close()
    for i, N in enumerate(Ns):
        Phi, Pi = O.init_gaussian(N, eps[i], sig[i])
        r1 = O.evolve_scheme(Phi, Pi, n1, rk=rk, a_reint=K, snap_every=every, n_slots=slots)
        for sl in range(slots):
            for f in range(5):
                check(b.split(sn[sl, f])[i], r1["snaps"][sl, f], "rk%d K%d N=%d slot %d %s" % (rk, K, N, sl, FIELDS[f]))
        r2 = O.evolve_scheme(r1["Phi"], r1["Pi"], n2, n0=n1, A=r1["A"], rk=rk, a_reint=K)
        assert s["steps"][i] == r2["steps"] == n2
        for f in FIELDS:
            check(b.split(st[f])[i], r2[f], "rk%d K%d N=%d %s" % (rk, K, N, f))
