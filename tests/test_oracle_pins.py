"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle (``oracle/``) against something other than itself:
polynomial exactness of the stencils, closed-form and library solutions of the
constraint equations (Liebling & Khanna, Sec. II, Eqs. (5)-(6)), the exact linear
solution in a frozen metric, the linear frequencies omega_j = 3 + 2j, mass
conservation, 4th-order convergence of the solution and of the residuals of
Eqs. (4)-(6), the boundary/regularity conditions Eqs. (7)-(12), and the
collapse/non-finite criteria.  None of these needs a GPU.
"""
import math
import os

import numpy as np
import pytest
from scipy import integrate, special

import oracle as O

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def rate(e1, e2):
    return math.log2(e1 / e2)


# --------------------------------------------------------------------------
# Stencils, quadrature and parity ghosts
# --------------------------------------------------------------------------

def test_D_exact_on_quartics_and_KO_annihilates_quintics():
    N = 33
    x, h = O.grid(N)
    rng = np.random.default_rng(1)
    for deg in range(6):
        c = rng.standard_normal(deg + 1)
        u = np.polyval(c, x)
        du = np.polyval(np.polyder(c), x)
        D = O.op_D(u, h, 1, 1)
        KO = O.op_KO(u, h, 0.5, 1, 1)
        inner = slice(3, N - 3)  # no ghost involved
        if deg <= 4:
            assert np.max(np.abs(D[inner] - du[inner])) < 1e-10 * max(1, np.max(np.abs(du)))
        assert np.max(np.abs(KO[inner])) < 1e-9 * max(1, np.max(np.abs(u))) / h
    # degree 6 is NOT annihilated: the 6th difference of x^6 is 720 h^6
    u = x ** 6
    KO = O.op_KO(u, h, 0.5, 1, 1)
    assert abs(KO[10] - 0.5 / (64 * h) * 720 * h ** 6) < 1e-12


def test_cell_rule_exact_on_cubics():
    N = 21
    x, h = O.grid(N)
    c = np.array([0.7, -1.3, 2.1, 0.4])
    u = np.polyval(c, x)
    P = np.polyint(c)
    exact = np.polyval(P, x[1:]) - np.polyval(P, x[:-1])
    cells = O.op_cell4(u, h, 1, 1)
    # interior cells have all 4 nodes on the grid
    assert np.max(np.abs(cells[1:-1] - exact[1:-1])) < 1e-14


@pytest.mark.parametrize("p", [1, -1])
def test_parity_ghosts_exact_for_matching_polynomials(p):
    """Ghost u_{-k} = p u_k is exact for a function of parity p about x=0, and
    u_{N-1+k} = p u_{N-1-k} for parity p about pi/2; then D and KO at the first
    points equal the values computed with the true polynomial continued past the
    end."""
    N = 33
    x, h = O.grid(N)
    # about x = 0
    u0 = (x ** 2 + 0.3 * x ** 4) if p == 1 else (x ** 3 - 0.2 * x)
    du0 = (2 * x + 1.2 * x ** 3) if p == 1 else (3 * x ** 2 - 0.2)
    D = O.op_D(u0, h, p, 1)
    assert np.max(np.abs(D[:3] - du0[:3])) < 1e-12
    # about x = pi/2
    y = math.pi / 2 - x
    u1 = (y ** 2 + 0.3 * y ** 4) if p == 1 else (y ** 3 - 0.2 * y)
    du1 = -((2 * y + 1.2 * y ** 3) if p == 1 else (3 * y ** 2 - 0.2))
    D = O.op_D(u1, h, 1, p)
    assert np.max(np.abs(D[-3:] - du1[-3:])) < 1e-12
    KO = O.op_KO(u1, h, 0.5, 1, p)
    assert np.max(np.abs(KO[-3:])) < 1e-11


def test_tables_match_libm():
    N = 65
    t = O.tables(N)
    x = t["x"]
    i = np.arange(1, N - 1)
    assert np.allclose(t["sc"][i], np.sin(x[i]) * np.cos(x[i]), rtol=1e-15, atol=0)
    assert np.allclose(t["t2"][i], np.tan(x[i]) ** 2, rtol=1e-14, atol=0)
    assert np.allclose(t["c3s"][i], np.cos(x[i]) ** 3 / np.sin(x[i]), rtol=1e-14, atol=0)
    assert t["sc"][0] == 0 and t["sc"][-1] == 0 and t["t2"][0] == 0


# --------------------------------------------------------------------------
# Constraint solve, Eqs. (5)-(6)
# --------------------------------------------------------------------------

def _mode0(N, eps):
    x, h = O.grid(N)
    d0 = math.sqrt(32 / math.pi)
    Pi = eps * d0 * np.cos(x) ** 3
    Pi[-1] = 0.0
    return x, np.zeros(N), Pi


def test_delta_closed_form_order4():
    """Phi=0, Pi=eps e_0: Eq. (6) integrates to delta~ = eps^2 (32/pi)(cos^8 x - 1)/8."""
    eps = 0.3
    errs = []
    for N in (65, 129, 257, 513):
        x, Phi, Pi = _mode0(N, eps)
        c = O.constraints(Phi, Pi)
        exact = eps ** 2 * (32 / math.pi) * (np.cos(x) ** 8 - 1) / 8
        errs.append(np.max(np.abs(c["dtil"] - exact)))
    rates = [rate(errs[k], errs[k + 1]) for k in range(3)]
    assert errs[-1] < 1e-10
    assert all(3.8 < r < 4.3 for r in rates), rates


def _A_by_ode(x_eval, qfun):
    """A from Eq. (5) itself, integrated outward by scipy at tight tolerance,
    started from the regular series A = 1 - q(0) x^2/3 near the origin."""
    x0 = 1e-5
    q0 = qfun(0.0)

    def f(x, A):
        s, c = math.sin(x), math.cos(x)
        return [(1 + 2 * s * s) / (s * c) * (1 - A[0]) - s * c * A[0] * qfun(x)]

    xe = x_eval[(x_eval > x0) & (x_eval < math.pi / 2 - 1e-3)]
    sol = integrate.solve_ivp(f, (x0, xe[-1]), [1 - q0 * x0 * x0 / 3], t_eval=xe, method="DOP853",
                              rtol=1e-13, atol=1e-15)
    return xe, sol.y[0]


def test_A_against_direct_ode_of_eq5():
    """The m-form used by the oracle reproduces Eq. (5) integrated as written."""
    eps, sigma = 2.0, 0.3
    qfun = lambda x: ((2 * eps / math.pi) * math.exp(-4 * math.tan(x) ** 2 / (math.pi ** 2 * sigma ** 2))) ** 2
    errs = []
    for N in (129, 257, 513):
        Phi, Pi = O.init_gaussian(N, eps, sigma)
        c = O.constraints(Phi, Pi)
        x, _ = O.grid(N)
        xe, A = _A_by_ode(x, qfun)
        mask = np.isin(x, xe)
        errs.append(np.max(np.abs(c["A"][mask] - A)))
    assert errs[-1] < 1e-8
    assert rate(errs[0], errs[1]) > 3.5 and rate(errs[1], errs[2]) > 3.5, errs


def test_delta_of_gaussian_against_quad_and_gauges():
    eps, sigma, N = 10.0, 1 / 16, 513
    Phi, Pi = O.init_gaussian(N, eps, sigma)
    x, _ = O.grid(N)
    qfun = lambda y: ((2 * eps / math.pi) * math.exp(-4 * math.tan(y) ** 2 / (math.pi ** 2 * sigma ** 2))) ** 2
    ref = np.array([-integrate.quad(lambda y: math.sin(y) * math.cos(y) * qfun(y), 0, xi,
                                    epsabs=1e-14, epsrel=1e-13, limit=200)[0] for xi in x[::32]])
    cb = O.constraints(Phi, Pi, gauge=O.GAUGE_BOUNDARY)
    co = O.constraints(Phi, Pi, gauge=O.GAUGE_ORIGIN)
    e1 = np.max(np.abs(cb["dtil"][::32] - ref))
    Phi2, Pi2 = O.init_gaussian(2 * N - 1, eps, sigma)
    e2 = np.max(np.abs(O.constraints(Phi2, Pi2)["dtil"][::64] - ref))
    assert e2 < 1e-7 * np.max(np.abs(ref)) and 3.7 < rate(e1, e2) < 4.3, (e1, e2)
    # gauges, Eq. (12) and delta(0)=0
    assert cb["delta"][-1] == 0.0 and co["delta"][0] == 0.0
    assert np.allclose(cb["delta"] - co["delta"], -co["delta"][-1], rtol=0, atol=1e-15)
    # Eq. (6): delta~ non-increasing outward
    assert np.all(np.diff(cb["dtil"]) <= 1e-18)


def test_mass_function_end_value_equals_paper_mass_integral():
    """m(pi/2) is the mass integral of Sec. II; both discretisations converge to it."""
    vals = []
    for N in (129, 257, 513, 1025):
        Phi, Pi = O.init_gaussian(N, 10.0, 1 / 16)
        c = O.constraints(Phi, Pi)
        vals.append((c["m"][-1], O.mass_paper(Phi, Pi, c["A"])))
    d = [abs(a - b) for a, b in vals]
    assert d[-1] < 1e-9 * vals[-1][0]
    assert d[1] < d[0] and d[2] < d[1]


def test_constraint_residuals_order4():
    """Residuals of Eqs. (5)-(6) vanish at 4th order: pointwise away from the
    origin, and weighted by sin x cos x everywhere (the 1/(sin x cos x) factor of
    Eq. (5) amplifies the O(h^5) quadrature error of m at the first points)."""
    errs = []
    for N in (129, 257, 513):
        Phi, Pi = O.init_gaussian(N, 4.0, 0.25)
        c = O.constraints(Phi, Pi)
        RA, Rd = O.residuals(Phi, Pi, c["A"], c["delta"])
        x, _ = O.grid(N)
        mid = (x > math.pi / 16) & (x < 7 * math.pi / 16)
        errs.append((np.max(np.abs(RA[mid])), np.max(np.abs(np.sin(x) * np.cos(x) * RA)),
                     np.max(np.abs(Rd))))
    for k in range(3):
        r = [rate(errs[0][k], errs[1][k]), rate(errs[1][k], errs[2][k])]
        assert min(r) > 3.7, (k, r, errs)


def test_regularity_and_boundary_values():
    Phi, Pi = O.init_gaussian(1025, 6.0, 0.2)
    c = O.constraints(Phi, Pi)
    A = c["A"]
    assert A[0] == 1.0 and A[-1] == 1.0
    # regularity at the origin: 1 - A ~ x^2, so (1-A_1)/(1-A_2) -> 1/4
    assert abs((1 - A[1]) / (1 - A[2]) - 0.25) < 1e-3
    # near pi/2: 1 - A ~ (pi/2 - x)^3
    r = (1 - A[-2]) / (1 - A[-3])
    assert abs(r - 1 / 8) < 1e-2


# --------------------------------------------------------------------------
# Linear AdS modes
# --------------------------------------------------------------------------

def test_jacobi_against_scipy():
    for n in range(0, 40, 3):
        for a, b in ((0.5, 1.5), (1.5, 2.5)):
            for z in (-0.99, -0.3, 0.0, 0.42, 0.97):
                ref = special.eval_jacobi(n, a, b, z)
                assert abs(O.jacobi(n, a, b, z) - ref) <= 1e-12 * max(1.0, abs(ref))


def test_modes_orthonormal_and_derivative():
    N, J = 513, 16
    e, de = O.modes(N, J)
    x, h = O.grid(N)
    w = h * np.tan(x) ** 2
    w[0] = w[-1] = 0.0
    G = (e * w) @ e.T
    om = 3 + 2 * np.arange(J)
    Gd = ((de / om[:, None]) * w) @ (de / om[:, None]).T
    assert np.max(np.abs(G - np.eye(J))) < 1e-12
    assert np.max(np.abs(Gd - np.eye(J))) < 1e-12
    # derivative formula vs numerical differentiation of e_j
    xs = np.linspace(0.1, 1.4, 7)
    hh = 1e-5
    for j in (0, 3, 9):
        def ej(t):
            return math.sqrt(1) * 0 + (2 * math.exp(0.5 * (math.lgamma(j + 1) + math.lgamma(j + 3)) - math.lgamma(j + 1.5))
                                       * math.cos(t) ** 3 * special.eval_jacobi(j, 0.5, 1.5, math.cos(2 * t)))
        num = np.array([(ej(t + hh) - ej(t - hh)) / (2 * hh) for t in xs])
        Nf = 2 ** 14 + 1
        xf, hf = O.grid(Nf)
        ef, def_ = O.modes(Nf, j + 1)
        ana = np.interp(xs, xf, def_[j])
        assert np.max(np.abs(num - ana)) < 1e-5 * max(1, np.max(np.abs(num)))


def test_modes_eigen_equation():
    """-(tan^-2)(tan^2 e')' = omega^2 e with omega_j = 3 + 2j (checked with the
    oracle's own D on e' and the analytic e)."""
    N, J = 2049, 5
    e, de = O.modes(N, J)
    x, h = O.grid(N)
    t2 = np.tan(x) ** 2
    i = np.arange(100, N - 100)
    for j in range(J):
        flux = t2 * de[j]
        flux[-1] = 0.0
        d = O.op_D(flux, h, -1, 1)
        lhs = -d[i] / t2[i]
        assert np.max(np.abs(lhs - (3 + 2 * j) ** 2 * e[j][i])) < 1e-6 * (3 + 2 * j) ** 2 * np.max(np.abs(e[j]))


# --------------------------------------------------------------------------
# Evolution: linear limit
# --------------------------------------------------------------------------

def test_frozen_metric_matches_exact_linear_solution_order4():
    """A=1, delta=0 (Table II's fixed metric): Pi = sum c_j cos(w_j t) e_j and
    Phi = sum (c_j/w_j) sin(w_j t) e_j' exactly; the scheme converges at 4th order."""
    c = np.array([1.0, -0.5, 0.25])
    om = 3 + 2 * np.arange(3)
    T = 1.3
    errs = []
    for N in (65, 129, 257):
        Phi, Pi = O.init_modes(N, 1.0, c)
        n = O.n_steps_for(T, N)
        r = O.evolve(Phi, Pi, n, frozen=True)
        t = r["t"]
        e, de = O.modes(N, 3)
        Pi_ex = (c * np.cos(om * t)) @ e
        Phi_ex = (c / om * np.sin(om * t)) @ de
        x, h = O.grid(N)
        l2 = math.sqrt(h * np.sum((r["Pi"] - Pi_ex) ** 2 + (r["Phi"] - Phi_ex) ** 2))
        mx = max(np.max(np.abs(r["Pi"] - Pi_ex)), np.max(np.abs(r["Phi"] - Phi_ex)))
        errs.append((l2, mx))
    assert errs[-1][1] < 1e-5
    # L2 error at 4th order; the max-norm, set by the cot^2 x factor of Eq. (3)
    # at the first points off the origin, at about 3.66
    for k, lo in ((0, 3.8), (1, 3.55)):
        assert rate(errs[0][k], errs[1][k]) > lo and rate(errs[1][k], errs[2][k]) > lo, errs


def test_tiny_amplitude_oscillates_at_3_plus_2j():
    """Linearised about AdS (eps -> 0), mode j of Pi oscillates at omega_j = 3 + 2j
    in boundary time; after half a period it flips sign, and its energy stays put."""
    N = 257
    for j in (0, 1):
        c = np.zeros(j + 1)
        c[j] = 1.0
        eps = 1e-6
        Phi, Pi = O.init_modes(N, eps, c)
        dt = O.dt_of(N)
        om = 3 + 2 * j
        # a step count close to half a period, and the phase at that time
        n = int(round(math.pi / om / dt))
        r = O.evolve(Phi, Pi, n)
        t = r["t"]
        e, de = O.modes(N, j + 1)
        pred = eps * math.cos(om * t) * e[j]
        assert np.max(np.abs(r["Pi"] - pred)) < 2e-4 * eps
        E0, _, _ = O.spectrum(Phi, Pi, np.ones(N), j + 1)
        E1, _, _ = O.spectrum(r["Phi"], r["Pi"], r["A"], j + 1)
        assert abs(E1[j] - E0[j]) < 1e-4 * E0[j]


# --------------------------------------------------------------------------
# Evolution: nonlinear invariants and convergence
# --------------------------------------------------------------------------

def _run(N, T, eps=3.0, sigma=0.25, **kw):
    Phi, Pi = O.init_gaussian(N, eps, sigma)
    return O.evolve(Phi, Pi, O.n_steps_for(T, N), **kw)


def test_self_convergence_order4_and_mass_conservation():
    T = 1.0
    res = {N: _run(N, T, snap_every=1, n_slots=0) for N in (129, 257, 513)}
    # time levels coincide: dt scales with h and T/dt is the same integer ratio
    steps = [res[N]["steps"] for N in (129, 257, 513)]
    assert steps[1] == 2 * steps[0] and steps[2] == 2 * steps[1]
    a, b, c = (res[N]["Pi"] for N in (129, 257, 513))
    d1 = np.max(np.abs(a - b[::2]))
    d2 = np.max(np.abs(b[::2] - c[::4]))
    assert 3.6 < rate(d1, d2) < 4.5, (d1, d2)
    # mass loss converges to zero at 4th order (Sec. II, Fig. 1)
    loss = []
    for N in (129, 257, 513):
        Phi, Pi = O.init_gaussian(N, 3.0, 0.25)
        M0 = O.constraints(Phi, Pi)["m"][-1]
        loss.append(abs(res[N]["m"][-1] - M0) / M0)
    assert loss[-1] < 1e-8
    assert rate(loss[0], loss[1]) > 3.0 and rate(loss[1], loss[2]) > 3.0, loss


def test_adot_residual_order4():
    """Eq. (4), which the scheme never imposes, holds to truncation error:
    the 4th-order time difference of A plus 2 sin x cos x A^2 e^-delta Phi Pi -> 0."""
    out = []
    for N in (129, 257, 513):
        Phi, Pi = O.init_gaussian(N, 3.0, 0.25)
        n_mid = O.n_steps_for(0.5, N)
        r = O.evolve(Phi, Pi, n_mid + 2, snap_every=1, n_slots=n_mid + 3)
        S = r["snaps"]
        dt = O.dt_of(N)
        Ad = (S[n_mid - 2, 2] - 8 * S[n_mid - 1, 2] + 8 * S[n_mid + 1, 2] - S[n_mid + 2, 2]) / (12 * dt)
        x, h = O.grid(N)
        Ph, P, A, d = S[n_mid, 0], S[n_mid, 1], S[n_mid, 2], S[n_mid, 3]
        R = Ad + 2 * np.sin(x) * np.cos(x) * A ** 2 * np.exp(-d) * Ph * P
        out.append(np.max(np.abs(R[1:-1])))
    assert rate(out[0], out[1]) > 3.3 and rate(out[1], out[2]) > 3.5, out


def _gauss_at(N, T=0.5, eps=3.0, sigma=0.25, gauge=O.GAUGE_BOUNDARY):
    Phi, Pi = O.init_gaussian(N, eps, sigma)
    return O.evolve(Phi, Pi, O.n_steps_for(T, N), gauge=gauge)


def test_adot_residual_function_order4():
    """The library's Eq. (4) diagnostic as the oracle defines it (A_t the
    derivative of the constraint solve along the right-hand sides): its
    residual converges to zero at order 4 on a nonlinear Gaussian."""
    out = []
    for N in (129, 257, 513, 1025):
        r = _gauss_at(N)
        _, R = O.adot_residual(r["Phi"], r["Pi"])
        assert R[0] == 0.0 and R[-1] == 0.0
        out.append(np.max(np.abs(R)))
    for e1, e2 in zip(out, out[1:]):
        assert 3.7 < rate(e1, e2) < 4.3, out


def test_adot_is_the_derivative_of_the_constraint_solve():
    """A_t against central differences of the oracle's constraint solve along
    the direction (Phi_t, Pi_t): A(U + tau F) - A(U - tau F) over 2 tau, in both
    gauges (A does not depend on the gauge, the right-hand sides do)."""
    N = 257
    for gauge in (O.GAUGE_BOUNDARY, O.GAUGE_ORIGIN):
        r = _gauss_at(N, gauge=gauge)
        Phi, Pi = r["Phi"], r["Pi"]
        c = O.constraints(Phi, Pi, gauge)
        dPhi, dPi = O.rhs(Phi, Pi, c["A"], c["delta"])
        Ad, _ = O.adot_residual(Phi, Pi, gauge=gauge)
        tau = 1e-5
        Ap = O.constraints(Phi + tau * dPhi, Pi + tau * dPi, gauge)["A"]
        Am = O.constraints(Phi - tau * dPhi, Pi - tau * dPi, gauge)["A"]
        fd = (Ap - Am) / (2 * tau)
        assert np.max(np.abs(Ad - fd)) <= 1e-8 * np.max(np.abs(Ad)), gauge


def test_adot_matches_time_difference_of_the_evolution():
    """A_t of the diagnostic against the 5-level 4th-order time difference of A
    over RK4 steps around the same state: they differ by the O(dt^4) error of
    the difference and of the time integrator only."""
    diffs = []
    for N in (257, 513):
        Phi, Pi = O.init_gaussian(N, 3.0, 0.25)
        n_mid = O.n_steps_for(0.5, N)
        r = O.evolve(Phi, Pi, n_mid + 2, snap_every=1, n_slots=n_mid + 3)
        S = r["snaps"]
        dt = O.dt_of(N)
        Atd = (S[n_mid - 2, 2] - 8 * S[n_mid - 1, 2] + 8 * S[n_mid + 1, 2] - S[n_mid + 2, 2]) / (12 * dt)
        Ad, _ = O.adot_residual(S[n_mid, 0], S[n_mid, 1])
        diffs.append(np.max(np.abs(Ad - Atd)[1:-1]) / np.max(np.abs(Ad)))
    assert diffs[0] < 1e-6 and rate(diffs[0], diffs[1]) > 3.5, diffs


def test_adot_vanishes_for_time_symmetric_data_without_dissipation():
    """Phi = 0 and no Kreiss-Oliger term: Pi_t = cot^2 x D(tan^2 x A e^-delta Phi) = 0
    and the origin row 3 D(A e^-delta Phi) = 0, so q_t = 0 and A_t = 0 exactly;
    Eq. (4) gives 0 as well (Phi Pi = 0)."""
    for N in (65, 257):
        Phi, Pi = O.init_gaussian(N, 5.0, 0.2)
        Ad, R = O.adot_residual(Phi, Pi, ko=0.0)
        assert np.all(Ad == 0.0) and np.all(R == 0.0)
        Ad, R = O.adot_residual(Phi, Pi, ko=0.5)  # the dissipation alone: O(h^5) rounding-free
        assert 0.0 < np.max(np.abs(Ad)) < 1e-4


def test_boundary_conditions_hold_at_every_snapshot():
    N = 257
    for gauge in (O.GAUGE_BOUNDARY, O.GAUGE_ORIGIN):
        Phi, Pi = O.init_gaussian(N, 5.0, 0.2)
        r = O.evolve(Phi, Pi, 400, gauge=gauge, snap_every=50, n_slots=9)
        for s in r["snaps"]:
            Ph, P, A, d, m = s
            assert Ph[0] == 0 and Ph[-1] == 0 and P[-1] == 0
            assert A[0] == 1 and A[-1] == 1
            assert (d[-1] if gauge == O.GAUGE_BOUNDARY else d[0]) == 0
            assert np.all(np.diff(d) <= 1e-15)


# --------------------------------------------------------------------------
# Collapse, non-finite data, degenerate calls (Sec. II: stop when min A small)
# --------------------------------------------------------------------------

def test_collapse_detected_and_state_frozen():
    N = 257
    Phi, Pi = O.init_gaussian(N, 20.0, 0.1)
    r = O.evolve(Phi, Pi, 20000, a_collapse=0.02, snap_every=0)
    assert r["state"] == O.COLLAPSED
    assert r["minA"] < 0.02
    n = r["steps"]
    # the step before collapse still had min A >= threshold
    r2 = O.evolve(Phi, Pi, n - 1, a_collapse=0.02)
    assert r2["state"] == O.DONE and r2["minA"] >= 0.02
    assert r["t_c"] == pytest.approx(n * O.dt_of(N))


def test_born_collapsed_nonfinite_and_zero_steps():
    N = 129
    Phi, Pi = O.init_gaussian(N, 100.0, 0.15)  # min A = 0.038 at t = 0
    r = O.evolve(Phi, Pi, 100, a_collapse=0.05)
    assert r["state"] == O.COLLAPSED and r["steps"] == 0 and r["t_c"] == 0.0
    Phi, Pi = O.init_gaussian(N, 1.0, 0.25)
    Pi[40] = np.nan
    r = O.evolve(Phi, Pi, 100, a_collapse=0.02)
    assert r["state"] == O.NONFINITE and r["steps"] == 0
    Phi, Pi = O.init_gaussian(N, 1.0, 0.25)
    r = O.evolve(Phi, Pi, 0)
    assert r["state"] == O.DONE and r["steps"] == 0
    assert np.array_equal(r["Pi"], Pi)


# --------------------------------------------------------------------------
# Spectrum (Sec. II: decomposition into normal modes)
# --------------------------------------------------------------------------

def test_spectrum_parseval_and_linear_limit():
    N = 1025
    Phi, Pi = O.init_gaussian(N, 6.0, 0.3)
    r = O.evolve(Phi, Pi, 300)
    Mp = O.mass_paper(r["Phi"], r["Pi"], r["A"])
    E, _, _ = O.spectrum(r["Phi"], r["Pi"], r["A"], 96)
    tot = np.cumsum(E)
    assert abs(tot[-1] - Mp) < 1e-6 * Mp
    assert abs(tot[15] - Mp) > abs(tot[-1] - Mp)
    # mode-sum data: E_j(0) = eps^2 c_j^2 (1 + O(eps^2))
    c = np.array([0.8, -0.3, 0.5, 0.1])
    for eps in (1e-2, 1e-3):
        Phi, Pi = O.init_modes(N, eps, c)
        A = O.constraints(Phi, Pi)["A"]
        E, Ph, _ = O.spectrum(Phi, Pi, A, 4)
        assert np.max(np.abs(E / (eps ** 2 * c ** 2) - 1)) < 5 * eps ** 2


def qp_family_rows():
    rows = []
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "qp_family_temperatures.txt")
    for line in open(path):
        if line.strip() and not line.startswith("#"):
            kd, mu, T, dec = line.split()
            rows.append((int(kd), float(mu), float(T), int(dec)))
    return rows


def family_coefficients(kd, mu, J):
    """Pi(x,0) = sum_k omega_k A_k e_k(x) with A_k = exp(-mu |k - k_d|) (eps applied separately)."""
    k = np.arange(J)
    return (3.0 + 2.0 * k) * np.exp(-mu * np.abs(k - kd))


def temperature(E):
    w = 3.0 + 2.0 * np.arange(len(E))
    return float(np.sum(E) / np.sum(E / w))


@pytest.mark.parametrize("kd,mu,T,dec", qp_family_rows())
def test_qp_family_temperature_matches_the_paper(kd, mu, T, dec):
    """The paper's printed temperatures of its approximate QP families (tests/golden),
    through the oracle's mode sum, constraint solve at t = 0 and projection, in the
    linear regime (eps = 1e-6, A = 1 to 1e-12)."""
    N, J = 1025, 40
    Phi, Pi = O.init_modes(N, 1e-6, family_coefficients(kd, mu, J))
    r = O.evolve(Phi, Pi, 0)
    E, _, _ = O.spectrum(Phi, Pi, r["A"], J)
    assert abs(temperature(E) - T) <= 0.5 * 10.0 ** (-dec), (kd, mu, temperature(E), T)
