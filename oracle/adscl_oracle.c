/*
 * adscl oracle: forward scheme.  TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, sequential CPU FP64 implementation of the method-of-lines
 * evolution of the spherically symmetric Einstein-Klein-Gordon system in
 * asymptotically AdS4 of Liebling & Khanna, "Scalar collapse in AdS with an
 * OpenCL open source code" (arXiv:1706.07413), Sec. II.  It is the yardstick the
 * HIP library is checked against.  Only the test-suite, the package smoke check
 * and the CPU-baseline leg of the benchmark may load it; the product library
 * never calls it and shares no code, header, table or constant with it.
 *
 * Built with gcc -O2 -ffp-contract=off -fno-fast-math (oracle/build.py), so every
 * expression is evaluated exactly in the order written, with libm exp/sin/cos/tan.
 *
 * Notation (one instance):
 *   N odd, h = (pi/2)/(N-1), x_i = i h, i = 0..N-1.
 *   Phi = phi', Pi = e^delta phi_dot / A        (Sec. II, text above Eq. (2)).
 *   State of an instance = (Phi, Pi) on the grid; A and delta are re-derived from
 *   it by the two radial constraints, Eqs. (5)-(6), at every Runge-Kutta stage.
 *
 * Readings where the paper is silent (each one is listed in the design notes):
 *   - classical RK4 (the paper offers RK2/3/4, Sec. II), dt = cfl*h;
 *   - 5-point 4th-order centred D, 7-point Kreiss-Oliger term of 6th-difference
 *     type with coefficient sigma_KO (the paper only says "fourth order accurate
 *     finite differences", Sec. II);
 *   - parity ghost points, three on each side of the grid;
 *   - Eq. (3) in conservative form cot^2 x * D[tan^2 x * A e^-delta Phi], with the
 *     value of tan^2 x A e^-delta Phi at x = pi/2 extrapolated (it is a finite limit);
 *   - the constraints solved through the mass function m = (1-A) sin x / cos^3 x,
 *     which turns Eq. (5) into two additive prefix integrals plus one exp, with
 *     4th-order 4-point cell quadrature;
 *   - collapse tested on the A of the state at the start of each step (Sec. II
 *     says the code stops when min A is small; the threshold is a parameter).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "oracle_internal.h"

/* ------------------------------------------------------------------------ */
/* Grid and coefficient tables                                               */
/* ------------------------------------------------------------------------ */

void grid_free(ora_grid* g)
{
    free(g->x); free(g->sn); free(g->cs); free(g->sc);
    free(g->t2); free(g->ct2); free(g->c3s);
}

void grid_make(ora_grid* g, int N)
{
    int i;
    g->N = N;
    g->h = (ORA_PI / 2.0) / (double)(N - 1);
    g->x = malloc(sizeof(double) * N);
    g->sn = malloc(sizeof(double) * N);
    g->cs = malloc(sizeof(double) * N);
    g->sc = malloc(sizeof(double) * N);
    g->t2 = malloc(sizeof(double) * N);
    g->ct2 = malloc(sizeof(double) * N);
    g->c3s = malloc(sizeof(double) * N);
    for (i = 0; i < N; ++i) {
        double x = (double)i * g->h;
        double s = sin(x), c = cos(x), t = tan(x);
        if (i == 0) { s = 0.0; c = 1.0; t = 0.0; }
        if (i == N - 1) { x = ORA_PI / 2.0; s = 1.0; c = 0.0; t = 0.0; }
        g->x[i] = x;
        g->sn[i] = s;
        g->cs[i] = c;
        g->sc[i] = s * c;
        g->t2[i] = t * t;
        g->ct2[i] = (i > 0 && i < N - 1) ? 1.0 / (t * t) : 0.0;
        g->c3s[i] = (i > 0 && i < N - 1) ? c * c * c / s : 0.0;
    }
}

void ora_tables(int N, double* x, double* sc, double* t2, double* ct2, double* c3s)
{
    ora_grid g;
    grid_make(&g, N);
    memcpy(x, g.x, sizeof(double) * N);
    memcpy(sc, g.sc, sizeof(double) * N);
    memcpy(t2, g.t2, sizeof(double) * N);
    memcpy(ct2, g.ct2, sizeof(double) * N);
    memcpy(c3s, g.c3s, sizeof(double) * N);
    grid_free(&g);
}

/* ------------------------------------------------------------------------ */
/* Parity ghosts and the three stencils                                      */
/* ------------------------------------------------------------------------ */

/* Value of u at index i in [-3, N+2]: u_{-k} = p0 u_k, u_{N-1+k} = p1 u_{N-1-k}.
 * p0/p1 are +1 (even) or -1 (odd) about x=0 / x=pi/2.  Smooth solutions of the
 * regular problem are even/odd functions about both ends (regularity at the
 * origin, Eqs. (7)-(8); reflecting boundary, Eqs. (9)-(11)). */
double gv(const double* u, int N, int i, double p0, double p1)
{
    if (i < 0) return p0 * u[-i];
    if (i > N - 1) return p1 * u[2 * (N - 1) - i];
    return u[i];
}

/* 4th-order centred first derivative at i. */
double stencil_D(const double* u, int N, int i, double h, double p0, double p1)
{
    return (gv(u, N, i - 2, p0, p1) - 8.0 * gv(u, N, i - 1, p0, p1)
            + 8.0 * gv(u, N, i + 1, p0, p1) - gv(u, N, i + 2, p0, p1)) / (12.0 * h);
}

/* Kreiss-Oliger dissipation built on the 6th undivided difference. */
double stencil_KO(const double* u, int N, int i, double h, double sig, double p0, double p1)
{
    double d6 = gv(u, N, i - 3, p0, p1) - 6.0 * gv(u, N, i - 2, p0, p1)
              + 15.0 * gv(u, N, i - 1, p0, p1) - 20.0 * u[i]
              + 15.0 * gv(u, N, i + 1, p0, p1) - 6.0 * gv(u, N, i + 2, p0, p1)
              + gv(u, N, i + 3, p0, p1);
    return sig / (64.0 * h) * d6;
}

/* Integral of u over the cell [x_i, x_{i+1}] by the 4-point rule that is exact
 * for cubics through x_{i-1}..x_{i+2}. */
double cell4(const double* u, int N, int i, double h, double p0, double p1)
{
    return h * (-gv(u, N, i - 1, p0, p1) + 13.0 * u[i] + 13.0 * gv(u, N, i + 1, p0, p1)
                - gv(u, N, i + 2, p0, p1)) / 24.0;
}

void ora_op_D(int N, double h, const double* u, int p0, int p1, double* out)
{
    int i;
    for (i = 0; i < N; ++i) out[i] = stencil_D(u, N, i, h, (double)p0, (double)p1);
}

void ora_op_KO(int N, double h, double sig, const double* u, int p0, int p1, double* out)
{
    int i;
    for (i = 0; i < N; ++i) out[i] = stencil_KO(u, N, i, h, sig, (double)p0, (double)p1);
}

void ora_op_cell4(int N, double h, const double* u, int p0, int p1, double* out)
{
    int i;
    for (i = 0; i < N - 1; ++i) out[i] = cell4(u, N, i, h, (double)p0, (double)p1);
}

/* ------------------------------------------------------------------------ */
/* Constraint solve, Sec. II Eqs. (5)-(6) with the gauge choice Eq. (12)     */
/* ------------------------------------------------------------------------ */

void cwork_alloc(ora_cwork* w, int N)
{
    w->q = malloc(sizeof(double) * N);
    w->p = malloc(sizeof(double) * N);
    w->dtil = malloc(sizeof(double) * N);
    w->E = malloc(sizeof(double) * N);
    w->sig = malloc(sizeof(double) * N);
    w->S = malloc(sizeof(double) * N);
}

void cwork_free(ora_cwork* w)
{
    free(w->q); free(w->p); free(w->dtil); free(w->E); free(w->sig); free(w->S);
}

/*
 * Given (Phi, Pi) solve Eq. (6) and Eq. (5) radially outward from x=0.
 *
 * Eq. (6): delta' = -sin x cos x (Phi^2+Pi^2).  Integrated from delta~(0)=0:
 *   delta~_{i+1} = delta~_i - int_{x_i}^{x_{i+1}} sin x cos x q dx.
 * Eq. (5) rewritten through m = (1-A) sin x / cos^3 x (so that m(pi/2) is the
 * mass of Sec. II):  m' = tan^2 x q - m sin x cos x q, a linear equation whose
 * integrating factor is e^{-delta~}.  With E = e^{-delta~}:
 *   S(x) = int_0^x tan^2 y q E dy,   m = S / E,   A = 1 - m cos^3 x / sin x.
 * Boundary values A(0) = A(pi/2) = 1 (Eqs. (8), (11)).
 * Gauge: boundary time delta(pi/2)=0 (Eq. (12)) shifts delta~ by its last value;
 * the origin gauge keeps delta = delta~ (delta(0)=0).
 */
void constraint_solve(const ora_grid* g, int gauge, const double* Phi, const double* Pi,
                             ora_cwork* w, double* A, double* delta, double* m)
{
    int N = g->N, i;
    double h = g->h;
    for (i = 0; i < N; ++i) w->q[i] = Phi[i] * Phi[i] + Pi[i] * Pi[i];
    for (i = 0; i < N; ++i) w->p[i] = g->sc[i] * w->q[i];
    w->p[0] = 0.0;
    w->p[N - 1] = 0.0;
    /* sin x cos x q is odd about both ends */
    w->dtil[0] = 0.0;
    for (i = 0; i < N - 1; ++i) w->dtil[i + 1] = w->dtil[i] - cell4(w->p, N, i, h, -1.0, -1.0);
    for (i = 0; i < N; ++i) w->E[i] = exp(-w->dtil[i]);
    for (i = 0; i < N; ++i) w->sig[i] = g->t2[i] * w->q[i] * w->E[i];
    w->sig[0] = 0.0;      /* tan^2 0 = 0 */
    w->sig[N - 1] = 0.0;  /* limit: q ~ (pi/2-x)^4 beats tan^2 x ~ (pi/2-x)^-2 */
    /* tan^2 x q E is even about both ends */
    w->S[0] = 0.0;
    for (i = 0; i < N - 1; ++i) w->S[i + 1] = w->S[i] + cell4(w->sig, N, i, h, 1.0, 1.0);
    for (i = 0; i < N; ++i) m[i] = w->S[i] / w->E[i];
    A[0] = 1.0;
    A[N - 1] = 1.0;
    for (i = 1; i < N - 1; ++i) A[i] = 1.0 - g->c3s[i] * m[i];
    for (i = 0; i < N; ++i)
        delta[i] = (gauge == ORA_GAUGE_BOUNDARY) ? w->dtil[i] - w->dtil[N - 1] : w->dtil[i];
}

/* Exported single solve (t = 0 data, tests). Returns nothing; outputs A, delta, m,
 * and delta~ (the origin-anchored integral of Eq. (6)). */
void ora_constraints(int N, int gauge, const double* Phi, const double* Pi,
                     double* A, double* delta, double* m, double* dtil)
{
    ora_grid g;
    ora_cwork w;
    grid_make(&g, N);
    cwork_alloc(&w, N);
    constraint_solve(&g, gauge, Phi, Pi, &w, A, delta, m);
    if (dtil) memcpy(dtil, w.dtil, sizeof(double) * N);
    cwork_free(&w);
    grid_free(&g);
}

/* ------------------------------------------------------------------------ */
/* Right-hand sides, Sec. II Eqs. (2)-(3)                                    */
/* ------------------------------------------------------------------------ */

void rwork_alloc(ora_rwork* r, int N)
{
    r->w = malloc(sizeof(double) * N);
    r->f1 = malloc(sizeof(double) * N);
    r->f2 = malloc(sizeof(double) * N);
    r->g = malloc(sizeof(double) * N);
}

void rwork_free(ora_rwork* r)
{
    free(r->w); free(r->f1); free(r->f2); free(r->g);
}

/*
 * Eq. (2): Phi_t = (A e^-delta Pi)'.
 * Eq. (3): Pi_t  = tan^-2 x (tan^2 x A e^-delta Phi)'.
 * With w = A e^-delta, f1 = w Pi, f2 = w Phi, g = tan^2 x f2:
 *   interior:  Phi_t = D f1 + KO Phi,   Pi_t = cot^2 x D g + KO Pi;
 *   x = 0:     Phi_t = 0 (Phi(0)=0, Eq. (7)),
 *              Pi_t  = 3 D f2 + KO Pi  (limit of tan^-2 (tan^2 f2)' for odd f2);
 *   x = pi/2:  Phi_t = Pi_t = 0 (Phi = Pi = 0 there, Eqs. (9)-(10)).
 * g tends to a finite constant at pi/2 and is even there; its end value is the
 * even 6th-order extrapolation (15 g_{N-2} - 6 g_{N-3} + g_{N-4}) / 10.
 * Ghost parities: Phi odd/even, Pi even/odd, f1 even/odd, g and f2 odd/even
 * (first entry about x=0, second about x=pi/2).
 */
void rhs_eval(const ora_grid* gr, double ko, int frozen, const double* Phi, const double* Pi,
                     const double* A, const double* delta, ora_rwork* r, double* dPhi, double* dPi)
{
    int N = gr->N, i;
    double h = gr->h;
    for (i = 0; i < N; ++i) r->w[i] = frozen ? 1.0 : A[i] * exp(-delta[i]);
    for (i = 0; i < N; ++i) {
        r->f1[i] = r->w[i] * Pi[i];
        r->f2[i] = r->w[i] * Phi[i];
    }
    for (i = 0; i < N - 1; ++i) r->g[i] = gr->t2[i] * r->f2[i];
    r->g[N - 1] = (15.0 * r->g[N - 2] - 6.0 * r->g[N - 3] + r->g[N - 4]) / 10.0;

    for (i = 1; i < N - 1; ++i) {
        dPhi[i] = stencil_D(r->f1, N, i, h, 1.0, -1.0) + stencil_KO(Phi, N, i, h, ko, -1.0, 1.0);
        dPi[i] = gr->ct2[i] * stencil_D(r->g, N, i, h, -1.0, 1.0) + stencil_KO(Pi, N, i, h, ko, 1.0, -1.0);
    }
    dPhi[0] = 0.0;
    dPi[0] = 3.0 * stencil_D(r->f2, N, 0, h, -1.0, 1.0) + stencil_KO(Pi, N, 0, h, ko, 1.0, -1.0);
    dPhi[N - 1] = 0.0;
    dPi[N - 1] = 0.0;
}

void ora_rhs(int N, double ko, int frozen, const double* Phi, const double* Pi,
             const double* A, const double* delta, double* dPhi, double* dPi)
{
    ora_grid g;
    ora_rwork r;
    grid_make(&g, N);
    rwork_alloc(&r, N);
    rhs_eval(&g, ko, frozen, Phi, Pi, A, delta, &r, dPhi, dPi);
    rwork_free(&r);
    grid_free(&g);
}

/* ------------------------------------------------------------------------ */
/* Time stepping (Sec. II: Runge-Kutta method of lines; classical RK4 here)  */
/* ------------------------------------------------------------------------ */

/* A and delta of a stage input: the constraint solve, or A=1, delta=0 when the
 * metric is frozen (the fixed-metric case of Table II). */
void stage_metric(const ora_grid* g, int gauge, int frozen, const double* Phi, const double* Pi,
                         ora_cwork* w, double* A, double* delta, double* m)
{
    int i;
    if (frozen) {
        for (i = 0; i < g->N; ++i) { A[i] = 1.0; delta[i] = 0.0; m[i] = 0.0; }
        return;
    }
    constraint_solve(g, gauge, Phi, Pi, w, A, delta, m);
}

/*
 * Evolve one instance from step n0 to step n_stop (t_n = n dt, dt = cfl h).
 * At the start of every step n (and at n = n_stop) the constraints of U^n are
 * solved; the instance is then
 *   - NONFINITE if any Phi, Pi, A or delta is not finite,
 *   - COLLAPSED (t_c = t_n) if min_i A_i < a_collapse  (Sec. II: stop when min A
 *     is small; the paper records t_c at min A = 0.01),
 * and stops without taking step n.  A snapshot (Phi, Pi, A, delta, m), each N
 * values, goes to slot n / snap_every whenever n is a multiple of snap_every and
 * the slot is < n_slots.  On return Phi, Pi hold U^n and A, delta, m its metric;
 * the return value is the state code and *n_out, *minA_out, *tc_out are set.
 */
int ora_evolve(int N, int gauge, int frozen, double cfl, double ko, double a_collapse,
               double* Phi, double* Pi, int64_t n0, int64_t n_stop,
               int32_t snap_every, int64_t n_slots, double* snaps,
               double* A, double* delta, double* m,
               int64_t* n_out, double* minA_out, double* tc_out)
{
    ora_grid g;
    ora_cwork cw;
    ora_rwork rw;
    double *k1p, *k1q, *k2p, *k2q, *k3p, *k3q, *k4p, *k4q, *up, *uq, *As, *ds, *ms;
    double dt, minA = 1.0;
    int64_t n;
    int i, state = ORA_RUNNING;

    grid_make(&g, N);
    cwork_alloc(&cw, N);
    rwork_alloc(&rw, N);
    k1p = malloc(sizeof(double) * N); k1q = malloc(sizeof(double) * N);
    k2p = malloc(sizeof(double) * N); k2q = malloc(sizeof(double) * N);
    k3p = malloc(sizeof(double) * N); k3q = malloc(sizeof(double) * N);
    k4p = malloc(sizeof(double) * N); k4q = malloc(sizeof(double) * N);
    up = malloc(sizeof(double) * N); uq = malloc(sizeof(double) * N);
    As = malloc(sizeof(double) * N); ds = malloc(sizeof(double) * N); ms = malloc(sizeof(double) * N);
    dt = cfl * g.h;
    *tc_out = -1.0;

    for (n = n0;; ++n) {
        int bad = 0;
        stage_metric(&g, gauge, frozen, Phi, Pi, &cw, A, delta, m);
        minA = A[0];
        for (i = 0; i < N; ++i) {
            if (!isfinite(Phi[i]) || !isfinite(Pi[i]) || !isfinite(A[i]) || !isfinite(delta[i])) bad = 1;
            if (A[i] < minA) minA = A[i];
        }
        if (snap_every > 0 && n % snap_every == 0 && n / snap_every < n_slots) {
            double* s = snaps + (size_t)(n / snap_every) * 5 * (size_t)N;
            memcpy(s, Phi, sizeof(double) * N);
            memcpy(s + N, Pi, sizeof(double) * N);
            memcpy(s + 2 * N, A, sizeof(double) * N);
            memcpy(s + 3 * N, delta, sizeof(double) * N);
            memcpy(s + 4 * N, m, sizeof(double) * N);
        }
        if (bad) { state = ORA_NONFINITE; *tc_out = (double)n * dt; break; }
        if (minA < a_collapse) { state = ORA_COLLAPSED; *tc_out = (double)n * dt; break; }
        if (n >= n_stop) break;

        /* k1 = F(U^n) */
        rhs_eval(&g, ko, frozen, Phi, Pi, A, delta, &rw, k1p, k1q);
        /* k2 = F(U^n + dt/2 k1) */
        for (i = 0; i < N; ++i) { up[i] = Phi[i] + (dt / 2.0) * k1p[i]; uq[i] = Pi[i] + (dt / 2.0) * k1q[i]; }
        stage_metric(&g, gauge, frozen, up, uq, &cw, As, ds, ms);
        rhs_eval(&g, ko, frozen, up, uq, As, ds, &rw, k2p, k2q);
        /* k3 = F(U^n + dt/2 k2) */
        for (i = 0; i < N; ++i) { up[i] = Phi[i] + (dt / 2.0) * k2p[i]; uq[i] = Pi[i] + (dt / 2.0) * k2q[i]; }
        stage_metric(&g, gauge, frozen, up, uq, &cw, As, ds, ms);
        rhs_eval(&g, ko, frozen, up, uq, As, ds, &rw, k3p, k3q);
        /* k4 = F(U^n + dt k3) */
        for (i = 0; i < N; ++i) { up[i] = Phi[i] + dt * k3p[i]; uq[i] = Pi[i] + dt * k3q[i]; }
        stage_metric(&g, gauge, frozen, up, uq, &cw, As, ds, ms);
        rhs_eval(&g, ko, frozen, up, uq, As, ds, &rw, k4p, k4q);
        /* U^{n+1} = U^n + dt/6 (k1 + 2 k2 + 2 k3 + k4) */
        for (i = 0; i < N; ++i) {
            Phi[i] = Phi[i] + (dt / 6.0) * (k1p[i] + 2.0 * k2p[i] + 2.0 * k3p[i] + k4p[i]);
            Pi[i] = Pi[i] + (dt / 6.0) * (k1q[i] + 2.0 * k2q[i] + 2.0 * k3q[i] + k4q[i]);
        }
    }
    *n_out = n;
    *minA_out = minA;

    free(k1p); free(k1q); free(k2p); free(k2q); free(k3p); free(k3q); free(k4p); free(k4q);
    free(up); free(uq); free(As); free(ds); free(ms);
    rwork_free(&rw);
    cwork_free(&cw);
    grid_free(&g);
    return state;
}

/* ------------------------------------------------------------------------ */
/* Diagnostics (Sec. II: mass and constraint residuals)                      */
/* ------------------------------------------------------------------------ */

/* M = int_0^{pi/2} tan^2 x A (Phi^2 + Pi^2) dx (Sec. II), by the 4-point cell
 * rule; the integrand is even about both ends and vanishes at both. */
double ora_mass_paper(int N, const double* Phi, const double* Pi, const double* A)
{
    ora_grid g;
    double *u, M = 0.0;
    int i;
    grid_make(&g, N);
    u = malloc(sizeof(double) * N);
    for (i = 0; i < N; ++i) u[i] = g.t2[i] * A[i] * (Phi[i] * Phi[i] + Pi[i] * Pi[i]);
    u[0] = 0.0;
    u[N - 1] = 0.0;
    for (i = 0; i < N - 1; ++i) M += cell4(u, N, i, g.h, 1.0, 1.0);
    free(u);
    grid_free(&g);
    return M;
}

/* Pointwise residuals of the two constraints at interior points 1..N-2 (end
 * entries are set to 0):
 *   RA[i] = D A - [ (1 + 2 sin^2 x)/(sin x cos x) (1 - A) - sin x cos x A q ]   (Eq. (5))
 *   Rd[i] = D delta + sin x cos x q                                          (Eq. (6))
 * Ghosts: A even about 0 and A-1 odd about pi/2; delta even about both ends. */
void ora_residuals(int N, const double* Phi, const double* Pi, const double* A, const double* delta,
                   double* RA, double* Rd)
{
    ora_grid g;
    double* Am1;
    int i;
    grid_make(&g, N);
    Am1 = malloc(sizeof(double) * N);
    for (i = 0; i < N; ++i) Am1[i] = A[i] - 1.0;
    for (i = 0; i < N; ++i) { RA[i] = 0.0; Rd[i] = 0.0; }
    for (i = 1; i < N - 1; ++i) {
        double q = Phi[i] * Phi[i] + Pi[i] * Pi[i];
        double s = g.sn[i];
        double dA = stencil_D(Am1, N, i, g.h, 1.0, -1.0);
        RA[i] = dA - ((1.0 + 2.0 * s * s) / g.sc[i] * (1.0 - A[i]) - g.sc[i] * A[i] * q);
        Rd[i] = stencil_D(delta, N, i, g.h, 1.0, 1.0) + g.sc[i] * q;
    }
    free(Am1);
    grid_free(&g);
}

/*
 * Residual of Eq. (4), A_t = -2 sin x cos x A^2 e^-delta Phi Pi, which the scheme
 * never imposes (Sec. II monitors the residuals of the equations).  A_t is the
 * time derivative of the discrete A of constraint_solve along the semi-discrete
 * flow, i.e. the derivative of A(Phi, Pi) in the direction of the right-hand
 * sides (Phi_t, Pi_t) of rhs_eval, taken through every step of the solve:
 *   q_t = 2 (Phi Phi_t + Pi Pi_t),   p_t = sin x cos x q_t (0 at both ends),
 *   delta~_t: 0 at x = 0, delta~_t,{i+1} = delta~_t,i - cell4(p_t)_i,
 *   E = e^{-delta~}:  E_t = -E delta~_t,
 *   sigma_t = tan^2 x (q_t E + q E_t) (0 at both ends),
 *   S_t: 0 at x = 0, S_t,{i+1} = S_t,i + cell4(sigma_t)_i,
 *   m = S / E:  m_t = (S_t - m E_t) / E,
 *   A = 1 - cos^3 x / sin x m:  A_t = -cos^3 x / sin x m_t  (0 at both ends).
 * Outputs, N values each: Adot = A_t and R = A_t + 2 sin x cos x A^2 e^-delta Phi Pi
 * (both 0 at the end points, where A is pinned).  The metric is the solve's of
 * (Phi, Pi) in the given gauge; ko is the Kreiss-Oliger coefficient of the
 * right-hand sides.
 */
void ora_adot_residual(int N, int gauge, double ko, const double* Phi, const double* Pi,
                       double* Adot, double* R)
{
    ora_grid g;
    ora_cwork w;
    ora_rwork r;
    double *A, *delta, *m, *dPhi, *dPi, *qt, *pt, *dt, *Et, *st, *St;
    double h;
    int i;
    grid_make(&g, N);
    cwork_alloc(&w, N);
    rwork_alloc(&r, N);
    h = g.h;
    A = malloc(sizeof(double) * N); delta = malloc(sizeof(double) * N); m = malloc(sizeof(double) * N);
    dPhi = malloc(sizeof(double) * N); dPi = malloc(sizeof(double) * N);
    qt = malloc(sizeof(double) * N); pt = malloc(sizeof(double) * N); dt = malloc(sizeof(double) * N);
    Et = malloc(sizeof(double) * N); st = malloc(sizeof(double) * N); St = malloc(sizeof(double) * N);

    constraint_solve(&g, gauge, Phi, Pi, &w, A, delta, m);
    rhs_eval(&g, ko, 0, Phi, Pi, A, delta, &r, dPhi, dPi);

    for (i = 0; i < N; ++i) qt[i] = 2.0 * (Phi[i] * dPhi[i] + Pi[i] * dPi[i]);
    for (i = 0; i < N; ++i) pt[i] = g.sc[i] * qt[i];
    pt[0] = 0.0;
    pt[N - 1] = 0.0;
    dt[0] = 0.0;
    for (i = 0; i < N - 1; ++i) dt[i + 1] = dt[i] - cell4(pt, N, i, h, -1.0, -1.0);
    for (i = 0; i < N; ++i) Et[i] = -w.E[i] * dt[i];
    for (i = 0; i < N; ++i) st[i] = g.t2[i] * (qt[i] * w.E[i] + w.q[i] * Et[i]);
    st[0] = 0.0;
    st[N - 1] = 0.0;
    St[0] = 0.0;
    for (i = 0; i < N - 1; ++i) St[i + 1] = St[i] + cell4(st, N, i, h, 1.0, 1.0);
    for (i = 0; i < N; ++i) {
        if (i == 0 || i == N - 1) {
            Adot[i] = 0.0;
            R[i] = 0.0;
            continue;
        }
        Adot[i] = -g.c3s[i] * ((St[i] - m[i] * Et[i]) / w.E[i]);
        R[i] = Adot[i] + 2.0 * g.sc[i] * A[i] * A[i] * exp(-delta[i]) * Phi[i] * Pi[i];
    }

    free(A); free(delta); free(m); free(dPhi); free(dPi);
    free(qt); free(pt); free(dt); free(Et); free(st); free(St);
    rwork_free(&r);
    cwork_free(&w);
    grid_free(&g);
}

/* ------------------------------------------------------------------------ */
/* Linear AdS4 eigenmodes (Sec. II: normal-mode spectrum)                    */
/* ------------------------------------------------------------------------ */

/* Jacobi polynomial P_n^(a,b)(z) by the three-term recurrence of DLMF 18.9.1-2. */
double ora_jacobi(int n, double a, double b, double z)
{
    double p0 = 1.0, p1, p2;
    int k;
    if (n == 0) return 1.0;
    p1 = (a + b + 2.0) * z / 2.0 + (a - b) / 2.0;
    for (k = 1; k < n; ++k) {
        double s = 2.0 * k + a + b;
        double An = (s + 1.0) * (s + 2.0) / (2.0 * (k + 1.0) * (k + a + b + 1.0));
        double Bn = (a * a - b * b) * (s + 1.0) / (2.0 * (k + 1.0) * (k + a + b + 1.0) * s);
        double Cn = (k + a) * (k + b) * (s + 2.0) / ((k + 1.0) * (k + a + b + 1.0) * s);
        p2 = (An * z + Bn) * p1 - Cn * p0;
        p0 = p1;
        p1 = p2;
    }
    return p1;
}

/* Normalisation d_j = 2 sqrt(j! (j+2)!) / Gamma(j + 3/2) of
 * e_j(x) = d_j cos^3 x P_j^(1/2,3/2)(cos 2x), unit norm in int f g tan^2 x dx. */
static double mode_norm(int j)
{
    return 2.0 * exp(0.5 * (lgamma(j + 1.0) + lgamma(j + 3.0)) - lgamma(j + 1.5));
}

/* e_j(x_i) and e_j'(x_i) for j < J, row-major [J][N]; omega_j = 3 + 2j.
 * e_j' uses dP_n^(a,b)/dz = (n+a+b+1)/2 P_{n-1}^(a+1,b+1) (DLMF 18.9.15). */
void ora_modes(int N, int J, double* e, double* de)
{
    ora_grid g;
    int i, j;
    grid_make(&g, N);
    for (j = 0; j < J; ++j) {
        double d = mode_norm(j);
        for (i = 0; i < N; ++i) {
            double s = g.sn[i], c = g.cs[i];
            double z = c * c - s * s; /* cos 2x */
            double P = ora_jacobi(j, 0.5, 1.5, z);
            double dP = (j > 0) ? 0.5 * (j + 3.0) * ora_jacobi(j - 1, 1.5, 2.5, z) : 0.0;
            e[(size_t)j * N + i] = d * c * c * c * P;
            de[(size_t)j * N + i] = d * (-3.0 * c * c * s * P - 2.0 * (2.0 * s * c) * c * c * c * dP);
        }
    }
    grid_free(&g);
}

/* Mode energies: Pihat_j = sum_i h tan^2 x_i e_j(x_i) sqrt(A_i) Pi_i,
 * Phihat_j = sum_i h tan^2 x_i e_j'(x_i)/omega_j sqrt(A_i) Phi_i over interior
 * points, E_j = Pihat_j^2 + Phihat_j^2. */
void ora_spectrum(int N, int J, const double* Phi, const double* Pi, const double* A,
                  double* E, double* Pihat, double* Phihat)
{
    ora_grid g;
    double *e, *de;
    int i, j;
    grid_make(&g, N);
    e = malloc(sizeof(double) * (size_t)J * N);
    de = malloc(sizeof(double) * (size_t)J * N);
    ora_modes(N, J, e, de);
    for (j = 0; j < J; ++j) {
        double a = 0.0, b = 0.0, om = 3.0 + 2.0 * j;
        for (i = 1; i < N - 1; ++i) {
            double sA = sqrt(A[i]);
            a += g.h * g.t2[i] * e[(size_t)j * N + i] * sA * Pi[i];
            b += g.h * g.t2[i] * (de[(size_t)j * N + i] / om) * sA * Phi[i];
        }
        Pihat[j] = a;
        Phihat[j] = b;
        E[j] = a * a + b * b;
    }
    free(e);
    free(de);
    grid_free(&g);
}

/* ------------------------------------------------------------------------ */
/* Initial data (Sec. II: choose Phi(x,0), Pi(x,0), then solve Eqs. (5)-(6)) */
/* ------------------------------------------------------------------------ */

/* Pi(x,0) = (2 eps/pi) exp(-4 tan^2 x / (pi^2 sigma^2)), Phi(x,0) = 0; the
 * pinned values Phi_0 = Phi_{N-1} = Pi_{N-1} = 0 (Eqs. (7), (9)-(10)). */
void ora_init_gaussian(int N, double eps, double sigma, double* Phi, double* Pi)
{
    ora_grid g;
    int i;
    grid_make(&g, N);
    for (i = 0; i < N; ++i) {
        Phi[i] = 0.0;
        Pi[i] = (2.0 * eps / ORA_PI) * exp(-4.0 * g.t2[i] / (ORA_PI * ORA_PI * sigma * sigma));
    }
    Pi[N - 1] = 0.0;
    grid_free(&g);
}

/* Pi(x,0) = eps sum_{j<Jc} c_j e_j(x), Phi(x,0) = 0, pinned values as above. */
void ora_init_modes(int N, double eps, int Jc, const double* c, double* Phi, double* Pi)
{
    double *e, *de;
    int i, j;
    e = malloc(sizeof(double) * (size_t)Jc * N);
    de = malloc(sizeof(double) * (size_t)Jc * N);
    ora_modes(N, Jc, e, de);
    for (i = 0; i < N; ++i) {
        double s = 0.0;
        for (j = 0; j < Jc; ++j) s += c[j] * e[(size_t)j * N + i];
        Phi[i] = 0.0;
        Pi[i] = eps * s;
    }
    Pi[N - 1] = 0.0;
    free(e);
    free(de);
}
