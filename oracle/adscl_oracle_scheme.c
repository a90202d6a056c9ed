/*
 * adscl oracle: the scheme options of Sec. II.  TEST INFRASTRUCTURE ONLY.
 *
 * Sec. II says the code offers second, third and fourth order Runge-Kutta
 * (its results use the third-order one), and that it evolves the metric
 * function A with Eq. (4) at every step instead of integrating Eq. (5), with a
 * periodic re-integration of A over space for stability and accuracy, while
 * delta is always integrated from Eq. (6).  This file evolves one instance with
 * any of those options, built from the oracle's own pieces (constraint_solve,
 * rhs_eval; adscl_oracle.c), in plain sequential loops.
 *
 * Readings where the paper is silent (listed in the design notes):
 *   - the second and third order methods are the strong-stability-preserving
 *     Runge-Kutta methods of Shu and Osher (J. Comput. Phys. 77 (1988) 439),
 *       RK2:  U1 = U + dt F(U),  U' = 1/2 U + 1/2 (U1 + dt F(U1)),
 *       RK3:  U1 = U + dt F(U),  U2 = 3/4 U + 1/4 (U1 + dt F(U1)),
 *             U' = 1/3 U + 2/3 (U2 + dt F(U2));
 *     the fourth order one is the classical method of ora_evolve;
 *   - evolved A ("a_reint" = K >= 1): the state is (Phi, Pi, A); every stage
 *     integrates Eq. (6) for delta from the stage's Phi, Pi (in the gauge), takes
 *     the right-hand sides of Eqs. (2)-(3) with the stage's A, and A_t from
 *     Eq. (4), A_t = -2 sin x cos x A^2 e^-delta Phi Pi, pointwise (no
 *     dissipation on A; it vanishes at both ends, where sin x cos x = 0, so A
 *     keeps its boundary values 1); at the start of every step n with n a
 *     multiple of K, A is replaced by the solution of Eq. (5) for U^n (n = 0
 *     included: the initial data's A solves Eq. (5));
 *   - the collapse and finiteness tests use the state's A; the mass function m
 *     returned is Eq. (5)'s for the state's Phi, Pi (so m(pi/2) is the mass
 *     integral of Sec. II whatever A is).
 * K = 0 is the plain method: A from Eq. (5) at every stage, as ora_evolve.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "oracle_internal.h"

typedef struct {
    const ora_grid* g;
    int gauge, frozen, evolve_A;
    double ko;
    ora_cwork* cw;
    ora_rwork* rw;
    double *Ac, *dl, *ml;  /* the stage's Eq. (5) A, delta, m */
} scheme_ctx;

/* F(V) for the stage input V = (V0, V1, V2 = A when A is evolved): k0, k1 (and
 * k2 = A_t). */
static void stage_rhs(scheme_ctx* s, const double* V0, const double* V1, const double* V2, double* k0,
                      double* k1, double* k2)
{
    int i, N = s->g->N;
    stage_metric(s->g, s->gauge, s->frozen, V0, V1, s->cw, s->Ac, s->dl, s->ml);
    if (!s->evolve_A) {
        rhs_eval(s->g, s->ko, s->frozen, V0, V1, s->Ac, s->dl, s->rw, k0, k1);
        return;
    }
    rhs_eval(s->g, s->ko, 0, V0, V1, V2, s->dl, s->rw, k0, k1);
    for (i = 0; i < N; ++i) k2[i] = -2.0 * s->g->sc[i] * V2[i] * V2[i] * exp(-s->dl[i]) * V0[i] * V1[i];
    k2[0] = 0.0;
    k2[N - 1] = 0.0;
}

/*
 * Evolve one instance from step n0 to n_stop with Runge-Kutta order rk (2, 3 or
 * 4) and metric option a_reint (0: A from Eq. (5) at every stage; K >= 1: A
 * evolved, re-integrated every K steps).  A is in/out: with A evolved it holds
 * the state's A on entry (replaced at n0 when n0 is a multiple of K) and on
 * return; otherwise it receives the metric of U^n.  Step starts, collapse and
 * finiteness tests, snapshots and outputs as ora_evolve, with the state's A.
 * Returns the state code, or -1 for an invalid option.
 */
int ora_evolve_scheme(int N, int gauge, int frozen, double cfl, double ko, double a_collapse, int rk, int a_reint,
                      double* Phi, double* Pi, double* A, int64_t n0, int64_t n_stop, int32_t snap_every,
                      int64_t n_slots, double* snaps, double* delta, double* m, int64_t* n_out, double* minA_out,
                      double* tc_out)
{
    ora_grid g;
    ora_cwork cw;
    ora_rwork rw;
    scheme_ctx s;
    double* buf;
    double *k[4][3], *V[3], *Ac, *dl, *ml;
    double dt, minA = 1.0;
    int64_t n;
    int i, j, f, nf, state = ORA_RUNNING;

    if (rk < 2 || rk > 4 || a_reint < 0 || (a_reint > 0 && frozen)) return -1;
    grid_make(&g, N);
    cwork_alloc(&cw, N);
    rwork_alloc(&rw, N);
    buf = calloc((size_t)N * 18, sizeof(double));
    for (j = 0; j < 4; ++j)
        for (f = 0; f < 3; ++f) k[j][f] = buf + (size_t)N * (3 * j + f);
    for (f = 0; f < 3; ++f) V[f] = buf + (size_t)N * (12 + f);
    Ac = buf + (size_t)N * 15;
    dl = buf + (size_t)N * 16;
    ml = buf + (size_t)N * 17;
    s.g = &g;
    s.gauge = gauge;
    s.frozen = frozen;
    s.evolve_A = a_reint > 0;
    s.ko = ko;
    s.cw = &cw;
    s.rw = &rw;
    s.Ac = Ac;
    s.dl = dl;
    s.ml = ml;
    nf = s.evolve_A ? 3 : 2;
    dt = cfl * g.h;
    *tc_out = -1.0;

    for (n = n0;; ++n) {
        int bad = 0;
        double* U[3] = {Phi, Pi, A};
        /* metric of U^n: Eq. (5)-(6); an evolved A is kept unless re-integrated */
        stage_metric(&g, gauge, frozen, Phi, Pi, &cw, Ac, delta, m);
        if (!s.evolve_A || n % a_reint == 0) memcpy(A, Ac, sizeof(double) * N);
        minA = A[0];
        for (i = 0; i < N; ++i) {
            if (!isfinite(Phi[i]) || !isfinite(Pi[i]) || !isfinite(A[i]) || !isfinite(delta[i])) bad = 1;
            if (A[i] < minA) minA = A[i];
        }
        if (snap_every > 0 && n % snap_every == 0 && n / snap_every < n_slots) {
            double* sn = snaps + (size_t)(n / snap_every) * 5 * (size_t)N;
            memcpy(sn, Phi, sizeof(double) * N);
            memcpy(sn + N, Pi, sizeof(double) * N);
            memcpy(sn + 2 * N, A, sizeof(double) * N);
            memcpy(sn + 3 * N, delta, sizeof(double) * N);
            memcpy(sn + 4 * N, m, sizeof(double) * N);
        }
        if (bad) { state = ORA_NONFINITE; *tc_out = (double)n * dt; break; }
        if (minA < a_collapse) { state = ORA_COLLAPSED; *tc_out = (double)n * dt; break; }
        if (n >= n_stop) break;

        if (rk == 4) {
            /* classical: k1 = F(U), k2 = F(U + dt/2 k1), k3 = F(U + dt/2 k2),
             * k4 = F(U + dt k3), U' = U + dt/6 (k1 + 2 k2 + 2 k3 + k4) */
            stage_rhs(&s, Phi, Pi, A, k[0][0], k[0][1], k[0][2]);
            for (f = 0; f < nf; ++f)
                for (i = 0; i < N; ++i) V[f][i] = U[f][i] + (dt / 2.0) * k[0][f][i];
            stage_rhs(&s, V[0], V[1], V[2], k[1][0], k[1][1], k[1][2]);
            for (f = 0; f < nf; ++f)
                for (i = 0; i < N; ++i) V[f][i] = U[f][i] + (dt / 2.0) * k[1][f][i];
            stage_rhs(&s, V[0], V[1], V[2], k[2][0], k[2][1], k[2][2]);
            for (f = 0; f < nf; ++f)
                for (i = 0; i < N; ++i) V[f][i] = U[f][i] + dt * k[2][f][i];
            stage_rhs(&s, V[0], V[1], V[2], k[3][0], k[3][1], k[3][2]);
            for (f = 0; f < nf; ++f)
                for (i = 0; i < N; ++i)
                    U[f][i] = U[f][i] + (dt / 6.0) * (k[0][f][i] + 2.0 * k[1][f][i] + 2.0 * k[2][f][i] + k[3][f][i]);
        } else if (rk == 3) {
            /* U1 = U + dt F(U) */
            stage_rhs(&s, Phi, Pi, A, k[0][0], k[0][1], k[0][2]);
            for (f = 0; f < nf; ++f)
                for (i = 0; i < N; ++i) V[f][i] = U[f][i] + dt * k[0][f][i];
            /* U2 = 3/4 U + 1/4 (U1 + dt F(U1)) */
            stage_rhs(&s, V[0], V[1], V[2], k[1][0], k[1][1], k[1][2]);
            for (f = 0; f < nf; ++f)
                for (i = 0; i < N; ++i) V[f][i] = 0.75 * U[f][i] + 0.25 * (V[f][i] + dt * k[1][f][i]);
            /* U' = 1/3 U + 2/3 (U2 + dt F(U2)) */
            stage_rhs(&s, V[0], V[1], V[2], k[2][0], k[2][1], k[2][2]);
            for (f = 0; f < nf; ++f)
                for (i = 0; i < N; ++i) U[f][i] = U[f][i] / 3.0 + (2.0 / 3.0) * (V[f][i] + dt * k[2][f][i]);
        } else {
            /* U1 = U + dt F(U), U' = 1/2 U + 1/2 (U1 + dt F(U1)) */
            stage_rhs(&s, Phi, Pi, A, k[0][0], k[0][1], k[0][2]);
            for (f = 0; f < nf; ++f)
                for (i = 0; i < N; ++i) V[f][i] = U[f][i] + dt * k[0][f][i];
            stage_rhs(&s, V[0], V[1], V[2], k[1][0], k[1][1], k[1][2]);
            for (f = 0; f < nf; ++f)
                for (i = 0; i < N; ++i) U[f][i] = 0.5 * U[f][i] + 0.5 * (V[f][i] + dt * k[1][f][i]);
        }
    }
    *n_out = n;
    *minA_out = minA;
    free(buf);
    rwork_free(&rw);
    cwork_free(&cw);
    grid_free(&g);
    return state;
}
