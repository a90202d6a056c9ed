"""Pins of the oracle's scheme options (Sec. II: Runge-Kutta of order 2, 3 or
4; A evolved with Eq. (4) and re-integrated periodically from Eq. (5), delta
integrated from Eq. (6) at every stage)."""
import math

import numpy as np
import pytest

import oracle as O

BIG = 10 ** 9  # re-integration interval longer than any run: A from Eq. (5) at t = 0 only


def rate(e1, e2):
    return math.log2(e1 / e2)


@pytest.mark.parametrize("rk", [2, 3, 4])
def test_one_linear_step_is_the_taylor_polynomial_of_the_method_order(rk):
    """With the metric frozen the right-hand side is a linear operator L; one
    step of an order-p Runge-Kutta method of p stages is the degree-p Taylor
    polynomial of exp(dt L): U' = sum_{k<=p} (dt L)^k U / k!  (exact, so any
    wrong stage coefficient fails)."""
    N = 65
    rng = np.random.default_rng(rk)
    Phi = rng.standard_normal(N)
    Pi = rng.standard_normal(N)
    Phi[0] = Phi[-1] = Pi[-1] = 0.0
    one, zero = np.ones(N), np.zeros(N)
    dt = O.dt_of(N)

    def L(u):
        return O.rhs(u[0], u[1], one, zero, frozen=True)

    term = [Phi.copy(), Pi.copy()]
    want = [Phi.copy(), Pi.copy()]
    for k in range(1, rk + 1):
        r = L(term)
        term = [dt * r[0] / k, dt * r[1] / k]
        want = [want[0] + term[0], want[1] + term[1]]
    got = O.evolve_scheme(Phi, Pi, 1, rk=rk, frozen=True)
    for f, w in zip(("Phi", "Pi"), want):
        assert np.max(np.abs(got[f] - w)) <= 1e-13 * np.max(np.abs(w)), (rk, f)


def test_plain_rk4_option_is_the_oracle_evolution_bit_for_bit():
    for gauge in (O.GAUGE_BOUNDARY, O.GAUGE_ORIGIN):
        Phi, Pi = O.init_gaussian(129, 6.0, 0.15)
        a = O.evolve(Phi, Pi, 200, gauge=gauge, a_collapse=0.01)
        b = O.evolve_scheme(Phi, Pi, 200, rk=4, gauge=gauge, a_collapse=0.01)
        for f in ("Phi", "Pi", "A", "delta", "m"):
            assert np.array_equal(a[f], b[f]), (gauge, f)
        assert a["steps"] == b["steps"] and a["state"] == b["state"]


@pytest.mark.parametrize("rk,a_reint", [(2, 0), (3, 0), (2, BIG), (3, BIG), (4, BIG)])
def test_time_order_on_a_fixed_grid(rk, a_reint):
    """The order of the time integration alone: one grid (N = 129), dt halved
    twice, against a run with dt 16 times smaller; the errors fall as dt^p."""
    N, T = 129, 0.4
    Phi, Pi = O.init_gaussian(N, 3.0, 0.25)
    h = (math.pi / 2) / (N - 1)

    def run(cfl):
        n = int(round(T / (cfl * h)))
        return O.evolve_scheme(Phi, Pi, n, rk=rk, a_reint=a_reint, cfl=cfl)["Pi"]

    base = 0.2
    ref = run(base / 16)
    e = [np.max(np.abs(run(base / s) - ref)) for s in (1, 2, 4)]
    assert abs(rate(e[0], e[1]) - rk) < 0.3 and abs(rate(e[1], e[2]) - rk) < 0.3, (rk, e)


def test_rk3_with_evolved_A_converges_at_third_order_and_keeps_eq5():
    """The paper's configuration (third-order Runge-Kutta, A evolved by Eq. (4);
    Sec. II and its convergence figure): Pi self-converges at least at order 3
    when the grid is refined with dt = h/4 (at these grids the 4th-order spatial
    error still dominates the small third-order time error, whose order the
    fixed-grid test isolates); the evolved A stays the solution of Eq. (5) up to
    truncation error, which falls with the grid (so Eq. (4) is consistent with
    Eqs. (2), (3), (5)); the mass loss falls too."""
    T = 1.0
    res = {}
    for N in (129, 257, 513):
        Phi, Pi = O.init_gaussian(N, 3.0, 0.25)
        r = O.evolve_scheme(Phi, Pi, O.n_steps_for(T, N), rk=3, a_reint=BIG)
        c = O.constraints(r["Phi"], r["Pi"])
        M0 = O.constraints(Phi, Pi)["m"][-1]
        res[N] = (r, np.max(np.abs(r["A"] - c["A"])), abs(r["m"][-1] - M0) / M0)
    a, b, c = (res[N][0]["Pi"] for N in (129, 257, 513))
    d1, d2 = np.max(np.abs(a - b[::2])), np.max(np.abs(b[::2] - c[::4]))
    assert 2.7 < rate(d1, d2) < 5.0, (d1, d2)
    drift = [res[N][1] for N in (129, 257, 513)]
    assert drift[0] < 1e-6 and rate(drift[0], drift[1]) > 2.5 and rate(drift[1], drift[2]) > 2.5, drift
    loss = [res[N][2] for N in (129, 257, 513)]
    assert rate(loss[0], loss[1]) > 2.5 and rate(loss[1], loss[2]) > 2.5, loss


def test_reintegration_replaces_A_at_multiples_of_K():
    """A equals Eq. (5)'s solution exactly at steps that are multiples of K, and
    differs from it (by truncation error) in between; with K = 1 the state's A is
    the constraint solution at every step start."""
    N, K = 129, 8
    Phi, Pi = O.init_gaussian(N, 4.0, 0.2)
    r = O.evolve_scheme(Phi, Pi, 3 * K, rk=3, a_reint=K, snap_every=1, n_slots=3 * K + 1)
    for n, S in enumerate(r["snaps"]):
        Ac = O.constraints(S[0], S[1])["A"]
        if n % K == 0:
            assert np.array_equal(S[2], Ac), n
        else:
            assert 0 < np.max(np.abs(S[2] - Ac)) < 1e-6, n
        assert S[2][0] == 1.0 and S[2][-1] == 1.0


def test_evolved_A_drives_the_collapse_test():
    """Strong data collapse with either metric option, at nearby times; the
    evolved-A run stops on its own A."""
    N = 257
    Phi, Pi = O.init_gaussian(N, 20.0, 0.1)
    a = O.evolve_scheme(Phi, Pi, 20000, rk=3, a_reint=0, a_collapse=0.02)
    b = O.evolve_scheme(Phi, Pi, 20000, rk=3, a_reint=BIG, a_collapse=0.02)
    assert a["state"] == O.COLLAPSED and b["state"] == O.COLLAPSED
    assert b["minA"] < 0.02 and abs(a["steps"] - b["steps"]) < 0.05 * a["steps"]


def test_invalid_options_are_refused():
    Phi, Pi = O.init_gaussian(65, 1.0, 0.2)
    for kw in (dict(rk=1), dict(rk=5), dict(a_reint=-1), dict(a_reint=4, frozen=True)):
        with pytest.raises(ValueError):
            O.evolve_scheme(Phi, Pi, 1, **kw)
