"""Pins of the oracle's discrete adjoint.

The reverse pass (oracle/adscl_oracle_adj.c) is written separately from the
forward scheme; each of its pieces must be the transpose of the derivative of
the corresponding forward piece.  Checked with the dot-product identity
<J v, w> = <v, J^T w>, where J v comes from central differences of the
oracle's forward code (step 1e-6 relative), and the whole gradient dL/dc of the
mode-energy drift objective against central differences of L itself.
"""
import math

import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def state(N, seed, eps=3.0):
    rng = np.random.default_rng(seed)
    Phi, Pi = O.init_gaussian(N, eps, 0.25)
    x, _ = O.grid(N)
    Phi = Phi + 0.3 * np.sin(2 * x) ** 3 * np.cos(x) ** 2 * rng.standard_normal()
    Phi[0] = Phi[-1] = 0.0
    Pi[-1] = 0.0
    return Phi, Pi


def pinned_dir(N, rng):
    v0, v1 = rng.standard_normal(N), rng.standard_normal(N)
    v0[0] = v0[-1] = 0.0
    v1[-1] = 0.0
    return v0, v1


def fd(f, x, v, h):
    return (f(x + h * v) - f(x - h * v)) / (2 * h)


@pytest.mark.parametrize("gauge", [O.GAUGE_BOUNDARY, O.GAUGE_ORIGIN])
def test_constraint_solve_transpose(gauge):
    N = 65
    rng = np.random.default_rng(3)
    Phi, Pi = state(N, 1)
    v0, v1 = pinned_dir(N, rng)
    Ab, db = rng.standard_normal(N), rng.standard_normal(N)

    def fwd(u):
        c = O.constraints(u[:N], u[N:], gauge=gauge)
        return np.concatenate([c["A"], c["delta"]])

    u = np.concatenate([Phi, Pi])
    Jv = fd(fwd, u, np.concatenate([v0, v1]), 1e-6)
    lhs = Jv @ np.concatenate([Ab, db])
    Pb, Qb = O.constraints_vjp(Phi, Pi, Ab, db, gauge=gauge)
    rhs = v0 @ Pb + v1 @ Qb
    assert abs(lhs - rhs) <= 1e-7 * max(abs(lhs), 1e-3), (lhs, rhs)


def test_rhs_transpose():
    N = 65
    rng = np.random.default_rng(4)
    Phi, Pi = state(N, 2)
    c = O.constraints(Phi, Pi)
    A, d = c["A"], c["delta"]
    dirs = [rng.standard_normal(N) for _ in range(4)]
    dirs[0][[0, -1]] = 0.0
    dirs[1][-1] = 0.0
    k0b, k1b = rng.standard_normal(N), rng.standard_normal(N)

    def fwd(u):
        a, b = O.rhs(u[:N], u[N:2 * N], u[2 * N:3 * N], u[3 * N:])
        return np.concatenate([a, b])

    u = np.concatenate([Phi, Pi, A, d])
    Jv = fd(fwd, u, np.concatenate(dirs), 1e-6)
    lhs = Jv @ np.concatenate([k0b, k1b])
    outs = O.rhs_vjp(Phi, Pi, A, d, k0b, k1b)
    rhs = sum(v @ o for v, o in zip(dirs, outs))
    assert abs(lhs - rhs) <= 1e-7 * max(abs(lhs), 1e-3), (lhs, rhs)


def test_rk4_step_transpose():
    N = 65
    rng = np.random.default_rng(5)
    Phi, Pi = state(N, 3)
    v0, v1 = pinned_dir(N, rng)
    w0, w1 = rng.standard_normal(N), rng.standard_normal(N)

    def fwd(u):
        a, b = O.step(u[:N], u[N:])
        return np.concatenate([a, b])

    u = np.concatenate([Phi, Pi])
    Jv = fd(fwd, u, np.concatenate([v0, v1]), 1e-6)
    lhs = Jv @ np.concatenate([w0, w1])
    Pb, Qb = O.step_vjp(Phi, Pi, w0, w1)
    rhs = v0 @ Pb + v1 @ Qb
    assert abs(lhs - rhs) <= 1e-7 * max(abs(lhs), 1e-3), (lhs, rhs)


def test_spectrum_transpose():
    N = 129
    J = 8
    rng = np.random.default_rng(6)
    Phi, Pi = state(N, 4)
    A = O.constraints(Phi, Pi)["A"]
    dirs = [rng.standard_normal(N) for _ in range(3)]
    for d in dirs:
        d[[0, -1]] = 0.0
    Eb = rng.standard_normal(J)

    def fwd(u):
        return O.spectrum(u[:N], u[N:2 * N], u[2 * N:], J)[0]

    u = np.concatenate([Phi, Pi, A])
    Jv = fd(fwd, u, np.concatenate(dirs), 1e-6)
    lhs = Jv @ Eb
    outs = O.spectrum_vjp(Phi, Pi, A, Eb)
    rhs = sum(v @ o for v, o in zip(dirs, outs))
    assert abs(lhs - rhs) <= 1e-7 * max(abs(lhs), 1e-6), (lhs, rhs)


def test_objective_gradient_against_central_differences():
    """Mode-sum data with 8 modes, eps = 0.5 (well inside the nonlinear regime),
    N = 65, 120 steps, drift of the first 4 mode energies."""
    N, Jc, J, n = 65, 8, 4, 120
    rng = np.random.default_rng(7)
    c = rng.standard_normal(Jc) * np.exp(-np.arange(Jc) / 4)
    eps = 0.5
    r = O.objective(N, eps, c, n_steps=n, J=J, K=50)
    assert r["valid"] and r["L"] > 0
    g = r["grad"]
    h = 1e-6
    fdg = np.array([(O.objective(N, eps, c + h * e, n_steps=n, J=J, grad=False)["L"]
                     - O.objective(N, eps, c - h * e, n_steps=n, J=J, grad=False)["L"]) / (2 * h)
                    for e in np.eye(Jc)])
    assert np.max(np.abs(g - fdg)) <= 1e-6 * np.max(np.abs(fdg)), (g, fdg)


def test_checkpoint_interval_does_not_change_the_gradient():
    N, Jc, J, n = 33, 6, 3, 97
    c = np.linspace(1.0, 0.2, Jc)
    ref = O.objective(N, 0.4, c, n_steps=n, J=J, K=n)["grad"]
    for K in (1, 7, 32):
        assert np.array_equal(O.objective(N, 0.4, c, n_steps=n, J=J, K=K)["grad"], ref)


def test_linear_limit_objective_vanishes():
    """For eps -> 0 the evolution is linear and every E_j is conserved, so the
    drift objective is O(eps^8) and tiny; its gradient is O(eps^6)."""
    N = 65
    c = np.array([1.0, 0.5, -0.3])
    r1 = O.objective(N, 1e-2, c, n_steps=200, J=3)
    r2 = O.objective(N, 2e-2, c, n_steps=200, J=3)
    # L scales as eps^8 (the drift of E_j ~ eps^4 itself scales as eps^4)
    assert 200 < r2["L"] / r1["L"] < 320
    assert np.max(np.abs(r1["grad"])) < 1e-3 * np.max(np.abs(r1["E0"]))


def test_descend_decreases_the_objective_with_steps_of_the_stated_length():
    """With a small step the gradient is a descent direction: every iteration
    lowers L (first-order decrease s |c| |g| > second-order terms), and each
    update moves c by exactly s |c| in Euclidean norm."""
    Ns = [33, 65]
    eps = [0.5, 0.4]
    r = np.random.default_rng(21)
    c0 = r.standard_normal((2, 6)) * np.exp(-np.arange(6) / 4)
    iters, step0 = 4, 0.01
    c, hist, active = O.descend(Ns, eps, c0, J=3, T=0.1, K=8, iters=iters, step0=step0)
    assert list(active) == [1, 1]
    assert np.all(np.diff(hist, axis=0) < 0), hist
    c1, _, _ = O.descend(Ns, eps, c0, J=3, T=0.1, K=8, iters=1, step0=step0)
    for b in range(2):
        step = np.linalg.norm(c1[b] - c0[b])
        assert abs(step - step0 * np.linalg.norm(c0[b])) <= 1e-13 * np.linalg.norm(c0[b])


def test_descend_masks_a_collapsing_instance():
    c0 = np.array([[1.0, 0.8, 0.6, 0.4, 0.2, 0.1], [0.3, -0.2, 0.1, 0.0, 0.05, 0.02]])
    c, hist, active = O.descend([129, 65], [0.8, 0.2], c0, J=3, T=1.0, K=64, iters=2, step0=0.01,
                                a_collapse=0.15)
    assert list(active) == [0, 1]
    assert np.array_equal(c[0], c0[0])
    assert np.isfinite(hist[0, 0]) and np.isnan(hist[1, 0])
    assert np.all(np.isfinite(hist[:, 1]))
