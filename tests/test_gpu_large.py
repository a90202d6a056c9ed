"""Parity of the multi-workgroup path (grids above 4097 points) with the oracle.

A large instance is cut into chunks of 2048 points, one workgroup each, that
exchange stage-input halos, scan carries and flux halos through global memory
every stage.  The computation is the same scheme with the prefix sums
re-associated (a chunk's carry enters as one factor), so the fields must match
the oracle to the same 1e-11 relative max-norm as the single-workgroup path.
"""
import concurrent.futures

import numpy as np
import pytest

import oracle as O
from paper_1706_07413_amd import adscl
from paper_1706_07413_amd import inputs as I
from test_gpu_parity import FIELDS, assert_close, gpu_state

pytestmark = pytest.mark.gpu


def test_two_mode_data_on_16385_points():
    """The 16385-point two-mode workload 0.05 (e_0 + 0.6 e_1): 8 chunks, 200
    steps, with snapshots every 50 steps."""
    import torch
    c = I.config1()
    N = int(c["N"][0])
    print("large N", N, flush=True)
    b = adscl.Batch(c["N"], gauge=c["gauge"], a_collapse=c["a_collapse"], n_modes=8)
    b.init_modes(c["eps"], np.ascontiguousarray(c["c"]))
    snaps = torch.zeros((5, 5, b.total), dtype=torch.float64, device="cuda")
    b.step(200, 1e9, snap_every=50, snaps=snaps)
    st = b.status()
    assert st["steps"][0] == 200 and st["state"][0] == adscl.RUNNING
    Phi, Pi = O.init_modes(N, float(c["eps"][0]), c["c"][0])
    ref = O.evolve(Phi, Pi, 200, gauge=c["gauge"], snap_every=50, n_slots=5)
    g = gpu_state(b)
    for f in FIELDS:
        assert_close(g[f], ref[f], "N=%d %s" % (N, f))
    sn = snaps.cpu().numpy()
    for s in range(5):
        for f in range(5):
            assert_close(sn[s, f], ref["snaps"][s, f], "snapshot %d %s" % (s, FIELDS[f]))


@pytest.mark.parametrize("gauge", [O.GAUGE_BOUNDARY, O.GAUGE_ORIGIN])
def test_ragged_chunks_with_small_instances_in_one_batch(gauge):
    """N = 10001 (chunks of 2048, 1808 and the end in the last) and N = 6145
    next to small instances; strong Gaussian data, 300 steps."""
    Ns = np.array([10001, 129, 6145, 4097], np.int32)
    eps = np.array([6.0, 3.0, 5.0, 4.0])
    sig = np.array([0.2, 0.25, 0.15, 0.2])
    print("large ragged gauge", gauge, flush=True)
    b = adscl.Batch(Ns, gauge=gauge, a_collapse=0.0)
    b.init_gaussian(eps, sig)
    b.step(300, 1e9)
    st = b.status()
    g = gpu_state(b)
    for i, N in enumerate(Ns):
        Phi, Pi = O.init_gaussian(int(N), float(eps[i]), float(sig[i]))
        ref = O.evolve(Phi, Pi, 300, gauge=gauge)
        assert st["steps"][i] == ref["steps"]
        for f in FIELDS:
            assert_close(b.split(g[f])[i], ref[f], "N=%d %s" % (N, f))


def test_collapse_of_a_large_instance_at_the_oracle_step():
    """A pulse whose min A falls through 0.2 after about 1500 steps on 4609
    points (chunks of 2048, 2048, 512): every chunk stops at the same step, the
    oracle's."""
    N, eps, sig, thr = 4609, 60.0, 0.08, 0.2
    print("large collapse", flush=True)
    b = adscl.Batch([N], a_collapse=thr)
    b.init_gaussian(np.array([eps]), np.array([sig]))
    b.step(2000, 1e9)
    st = b.status()
    Phi, Pi = O.init_gaussian(N, eps, sig)
    ref = O.evolve(Phi, Pi, 2000, a_collapse=thr)
    assert ref["state"] == O.COLLAPSED, ref["state"]
    assert st["state"][0] == adscl.COLLAPSED and st["steps"][0] == ref["steps"]
    g = gpu_state(b)
    for f in FIELDS:
        assert_close(g[f], ref[f], "collapsed N=%d %s" % (N, f))


def test_large_instance_equals_itself_alone_and_chunked_calls():
    """Bitwise: a large instance in a batch equals it alone, and 3 calls of 40
    steps equal one call of 120."""
    Ns = np.array([8193, 257], np.int32)
    b = adscl.Batch(Ns)
    b.init_gaussian(np.array([5.0, 2.0]), np.array([0.2, 0.2]))
    b.step(120, 1e9)
    g = gpu_state(b)
    b1 = adscl.Batch(Ns[:1])
    b1.init_gaussian(np.array([5.0]), np.array([0.2]))
    for _ in range(3):
        b1.step(40, 1e9)
    g1 = gpu_state(b1)
    for f in FIELDS:
        assert np.array_equal(b.split(g[f])[0], g1[f]), f


@pytest.mark.parametrize("Ns,n", [([16385, 129], 120), ([65537], 24)])
def test_frozen_metric_on_chunked_grids(Ns, n):
    """The frozen-metric mode (A = 1, delta = 0: the linear wave of the paper's
    fixed-metric benchmark) on grids split over several workgroups, up to the
    largest supported N, beside a one-workgroup instance."""
    c = np.array([[1.0, -0.5, 0.25, 0.1]] * len(Ns))
    print("frozen chunked", Ns, n, flush=True)
    b = adscl.Batch(Ns, n_modes=4, flags=adscl.FROZEN_METRIC)
    b.init_modes(np.full(len(Ns), 0.3), c)
    b.step(n, 1e9)
    st = gpu_state(b)
    for i, N in enumerate(Ns):
        Phi, Pi = O.init_modes(N, 0.3, c[i])
        ref = O.evolve(Phi, Pi, n, frozen=True)
        for f in ("Phi", "Pi"):
            assert_close(b.split(st[f])[i], ref[f], "frozen N=%d %s" % (N, f))
        assert np.all(b.split(st["A"])[i] == 1.0)
        assert np.all(b.split(st["delta"])[i] == 0.0)


@pytest.mark.parametrize("N,frozen,n", [(10001, False, 200), (16385, False, 120), (65537, True, 24),
                                        (65537, False, 24)])
def test_chunks_of_1024_points(monkeypatch, N, frozen, n):
    """The other chunk shape of the multi-workgroup kernel, (4, 4): 1024 points
    per workgroup (10001: nine full chunks and 784 points in the last; 65537:
    64 chunks, the most a launch takes, so that the chunk carries fill every
    lane of the wavefront that scans them), selected with ADSCL_TUNE at context
    creation."""
    monkeypatch.setenv("ADSCL_TUNE", "%d:4x4" % N)
    c = np.array([[1.0, 0.6, -0.2]])
    eps = 0.3 if frozen else 0.05
    print("chunks of 1024", N, frozen, n, flush=True)
    b = adscl.Batch([N], n_modes=3, flags=adscl.FROZEN_METRIC if frozen else 0)
    b.init_modes(np.array([eps]), c)
    b.step(n, 1e9)
    st = b.status()
    assert st["steps"][0] == n
    g = gpu_state(b)
    Phi, Pi = O.init_modes(N, eps, c[0])
    ref = O.evolve(Phi, Pi, n, frozen=frozen)
    for f in (("Phi", "Pi") if frozen else FIELDS):
        assert_close(g[f], ref[f], "4x4 chunks N=%d %s" % (N, f))


@pytest.mark.parametrize("N,n", [(32769, 40), (65537, 24)])
def test_dynamic_metric_on_the_speed_table_grids(N, n):
    """The dynamic metric on the paper's speed-table grids: N = 32769 (16
    chunks of 2048 points) and the largest supported N = 65537 (32 chunks),
    two-mode data 0.05 (e_0 + 0.6 e_1)."""
    c = np.array([[1.0, 0.6]])
    print("speed-table grid", N, n, flush=True)
    b = adscl.Batch([N], a_collapse=0.01, n_modes=2)
    b.init_modes(np.array([0.05]), c)
    b.step(n, 1e9)
    st = b.status()
    assert st["steps"][0] == n and st["state"][0] == adscl.RUNNING
    g = gpu_state(b)
    Phi, Pi = O.init_modes(N, 0.05, c[0])
    ref = O.evolve(Phi, Pi, n)
    for f in FIELDS:
        assert_close(g[f], ref[f], "N=%d %s" % (N, f))


def test_several_large_instances_side_by_side():
    """Five large instances (three grid sizes, one collapsing early at the
    oracle's step) share one cooperative launch next to a small one: each
    matches the oracle, and each is bitwise equal to itself run alone."""
    Ns = np.array([8193, 4609, 6145, 257, 8193, 10001], np.int32)
    eps = np.array([5.0, 60.0, 4.0, 2.0, 3.0, 6.0])
    sig = np.array([0.2, 0.08, 0.25, 0.2, 0.3, 0.2])
    thr = 0.2
    n = 1500
    print("several large", flush=True)
    O.grid(17)  # load the oracle before its worker threads call it

    def oracle_run(i):
        Phi, Pi = O.init_gaussian(int(Ns[i]), float(eps[i]), float(sig[i]))
        return O.evolve(Phi, Pi, n, a_collapse=thr)

    with concurrent.futures.ThreadPoolExecutor(max_workers=len(Ns)) as ex:
        futs = [ex.submit(oracle_run, i) for i in range(len(Ns))]
        b = adscl.Batch(Ns, a_collapse=thr)
        b.init_gaussian(eps, sig)
        b.step(n, 1e9)
        st = b.status()
        g = gpu_state(b)
        b.close()
        refs = [f.result() for f in futs]
    for i, N in enumerate(Ns):
        ref = refs[i]
        assert st["steps"][i] == ref["steps"], (i, st["steps"][i], ref["steps"])
        want = adscl.RUNNING if ref["state"] == O.DONE else ref["state"]
        assert st["state"][i] == want, i
        for f in FIELDS:
            assert_close(b.split(g[f])[i], ref[f], "N=%d #%d %s" % (N, i, f))
    assert st["state"][1] == adscl.COLLAPSED and st["steps"][1] < n
    for i in (0, 5):
        one = adscl.Batch(Ns[i:i + 1], a_collapse=thr)
        one.init_gaussian(eps[i:i + 1], sig[i:i + 1])
        one.step(n, 1e9)
        g1 = gpu_state(one)
        one.close()
        for f in FIELDS:
            assert np.array_equal(b.split(g[f])[i], g1[f]), (i, f)
