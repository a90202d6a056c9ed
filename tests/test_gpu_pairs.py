"""Pair launches (opt-in, ADSCL_PAIR=1): a batch that holds both full (8, 8)
instances (N = 4097) and full (8, 4) instances (N = 2049) runs the latter two
per workgroup inside the (8, 8) launch, the two halves of a workgroup in
lock-step.  Checked against the
oracle, and against the same batch with every class in a launch of its own
(ADSCL_PAIR=0): the steps and states exactly, the fields to 1e-12 (the same
arithmetic, compiled into another kernel, where the compiler may fuse other
multiply-adds; a scheduling fault -- a half that missed a barrier, a stale flag,
a wrong slot -- shows as an O(1) difference).

Cases: a half whose instance collapses mid-run while its partner goes on, a
half whose instance had already stopped before the call, a workgroup with one
half empty (an odd number of N = 2049 instances), the frozen metric (one
barrier per stage instead of three), and snapshot segments.
"""
import numpy as np
import pytest

import oracle as O
from paper_1706_07413_amd import adscl

pytestmark = pytest.mark.gpu

TOL = 1e-11
FIELDS = ("Phi", "Pi", "A", "delta", "m")

# N, eps, sigma.  With a collapse threshold of 0.19 the second instance
# (N = 2049, eps = 38.26, sigma = 0.1313) collapses at step 1190 (oracle), its
# partner in the first pair runs on; the third N = 2049 instance has a
# workgroup to itself.
CASE = [(4097, 4.0, 0.15), (2049, 38.26, 0.1313), (2049, 6.0, 0.2), (2049, 3.0, 0.12), (4097, 8.0, 0.25)]
THR = 0.19


def rel(g, o):
    n = np.max(np.abs(o))
    d = np.max(np.abs(g - o))
    return d / 1e-13 * TOL if n < 1e-12 else d / n


def state(b):
    return {k: v.cpu().numpy() for k, v in b.get_state().items()}


def batch(monkeypatch, Ns, pair, **kw):
    monkeypatch.setenv("ADSCL_PAIR", "1" if pair else "0")
    monkeypatch.delenv("ADSCL_TUNE", raising=False)
    b = adscl.Batch(Ns, **kw)
    classes, cls = b.kernel_stats()
    by_n = {n: {(classes[cls[i]]["P"], classes[cls[i]]["W"]) for i in range(len(Ns)) if Ns[i] == n}
            for n in set(Ns)}
    if pair:
        # the N = 2049 instances run in the (8, 8) launch
        assert by_n[2049] == {(8, 8)} and by_n[4097] == {(8, 8)}
    else:
        assert by_n[2049] == {(8, 4)} and by_n[4097] == {(8, 8)}
    return b


SAME = 1e-12


def assert_same(b1, b2, what):
    s1, s2 = state(b1), state(b2)
    for f in FIELDS:
        e = rel(s1[f], s2[f])
        assert e <= SAME, "%s: %s differs between pair and separate launches by %.3e" % (what, f, e)
    t1, t2 = b1.status(), b2.status()
    for k in ("steps", "state"):
        assert np.array_equal(t1[k], t2[k]), (what, k, t1[k], t2[k])


def test_pair_launch_collapse_mid_run_and_stopped_partner(monkeypatch):
    Ns = [n for n, _, _ in CASE]
    eps = np.array([e for _, e, _ in CASE])
    sig = np.array([s for _, _, s in CASE])
    runs = {}
    for pair in (True, False):
        b = batch(monkeypatch, Ns, pair, a_collapse=THR)
        b.init_gaussian(eps, sig)
        b.step(1400, 1e9)
        runs[pair] = b
    b = runs[True]
    st, s = state(b), b.status()
    for i, (N, e, sg) in enumerate(CASE):
        Phi, Pi = O.init_gaussian(N, e, sg)
        ref = O.evolve(Phi, Pi, 1400, a_collapse=THR)
        assert s["steps"][i] == ref["steps"], (i, s["steps"][i], ref["steps"])
        want = ref["state"] if ref["state"] != O.DONE else adscl.RUNNING
        assert s["state"][i] == want, (i, s["state"][i], want)
        for f in FIELDS:
            e_ = rel(b.split(st[f])[i], ref[f])
            assert e_ <= TOL, "N=%d inst %d %s: %.3e" % (N, i, f, e_)
    assert s["steps"][1] == 1190 and s["state"][1] == adscl.COLLAPSED
    assert_same(runs[True], runs[False], "first call")
    # second call: the collapsed half takes no step, its partner goes on
    for pair in (True, False):
        runs[pair].step(300, 1e9)
    assert_same(runs[True], runs[False], "second call")
    assert runs[True].status()["steps"][2] == 1700
    for b in runs.values():
        b.close()


def test_pair_launch_frozen_metric(monkeypatch):
    Ns = [4097, 2049, 2049, 2049]
    c = np.array([[0.8, -0.5, 0.25, 0.1], [0.3, 0.2, -0.7, 0.05], [1.0, 0.0, 0.4, -0.2], [0.1, 0.9, 0.0, 0.3]])
    runs = {}
    for pair in (True, False):
        b = batch(monkeypatch, Ns, pair, n_modes=4, flags=adscl.FROZEN_METRIC)
        b.init_modes(np.ones(4), c)
        b.step(300, 1e9)
        runs[pair] = b
    b = runs[True]
    st = state(b)
    for i, N in enumerate(Ns):
        Phi, Pi = O.init_modes(N, 1.0, c[i])
        ref = O.evolve(Phi, Pi, 300, frozen=True)
        for f in ("Phi", "Pi"):
            e_ = rel(b.split(st[f])[i], ref[f])
            assert e_ <= TOL, "frozen N=%d %s: %.3e" % (N, f, e_)
    assert_same(runs[True], runs[False], "frozen")
    for b in runs.values():
        b.close()


def test_pair_launch_snapshot_segments(monkeypatch):
    import torch
    Ns = [2049, 4097, 2049]
    eps = np.array([5.0, 3.0, 7.0])
    sig = np.array([0.2, 0.15, 0.1])
    out = {}
    for pair in (True, False):
        b = batch(monkeypatch, Ns, pair, a_collapse=0.02)
        b.init_gaussian(eps, sig)
        snaps = torch.zeros((5, 5, b.total), dtype=torch.float64, device="cuda")
        b.step(256, 1e9, snap_every=64, snaps=snaps)
        out[pair] = (b, snaps.cpu().numpy())
    for k in range(5):
        for f in range(5):
            assert rel(out[True][1][k, f], out[False][1][k, f]) <= SAME, (k, f)
    assert_same(out[True][0], out[False][0], "snapshots")
    for b, _ in out.values():
        b.close()


def test_pair_launch_timing_is_reported_on_the_host_class(monkeypatch):
    Ns = [4097, 2049, 2049]
    b = batch(monkeypatch, Ns, True, a_collapse=0.02, flags=adscl.TIME_KERNELS)
    b.init_gaussian(np.array([3.0, 4.0, 5.0]), np.array([0.2, 0.2, 0.2]))
    b.step(64, 1e9)
    classes, cls = b.kernel_stats()
    host = classes[cls[0]]
    assert (host["P"], host["W"]) == (8, 8) and host["last_ms"] > 0.0
    guest = [k for k, c in enumerate(classes) if (c["P"], c["W"]) == (8, 4)]
    assert len(guest) == 1 and classes[guest[0]]["members"] == 2 and classes[guest[0]]["last_ms"] == -1.0
    assert list(cls) == [cls[0]] * 3
    b.close()
