"""The oracle's batch drivers (one instance per OpenMP thread, used to time the
CPU baseline) compute exactly what the sequential oracle computes per instance."""
import numpy as np

import oracle as O


def test_evolve_gaussian_batch_equals_per_instance_runs():
    Ns = np.array([65, 129, 97, 257, 65], np.int32)
    eps = np.array([2.0, 30.0, 1.0, 5.0, 80.0])
    sig = np.array([0.2, 0.1, 0.25, 0.15, 0.08])
    n_stop = np.array([100, 3000, 50, 200, 100])
    steps, state = O.evolve_gaussian_batch(Ns, eps, sig, n_stop, a_collapse=0.02)
    for b in range(len(Ns)):
        Phi, Pi = O.init_gaussian(int(Ns[b]), eps[b], sig[b])
        r = O.evolve(Phi, Pi, int(n_stop[b]), a_collapse=0.02)
        assert steps[b] == r["steps"]
        assert state[b] == (r["state"] if r["state"] != O.DONE else O.RUNNING)
    assert state[1] == O.COLLAPSED and state[4] == O.COLLAPSED  # strong data stop early
    assert O.threads() >= 1


def test_objective_batch_equals_per_instance_objective():
    rng = np.random.default_rng(3)
    Ns = np.array([33, 65, 33], np.int32)
    c = rng.standard_normal((3, 4))
    eps = np.array([0.3, 0.5, 0.2])
    n_steps = np.array([20, 30, 25])
    L, g, v = O.objective_batch(Ns, eps, c, 3, n_steps, 8)
    for b in range(3):
        r = O.objective(int(Ns[b]), eps[b], c[b], n_steps=int(n_steps[b]), J=3, K=8)
        assert v[b] == 1 and r["valid"]
        assert L[b] == r["L"]
        assert np.array_equal(g[b], r["grad"])
