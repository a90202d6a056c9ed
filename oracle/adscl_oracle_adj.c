/*
 * adscl oracle: reverse-mode derivative of the forward scheme.  TEST
 * INFRASTRUCTURE ONLY (same rules as adscl_oracle.c).
 *
 * The objective is the drift of the low-mode energy spectrum of one instance
 * between t = 0 and t_n = n dt,
 *     L(c) = sum_{j < J} (E_j(t_n) - E_j(0))^2,
 * for mode-sum initial data Pi(x,0) = eps sum_{k<Jc} c_k e_k(x), Phi(x,0) = 0
 * (Sec. II: initial data from a mode spectrum; spectrum of normal modes).  Its
 * gradient dL/dc is the exact derivative of the discrete computation: every
 * forward piece below has its transposed Jacobian applied in reverse order,
 *   - the spectrum E_j = (sum_i W_ij sqrt(A_i) Pi_i)^2 + (sum_i W'_ij sqrt(A_i) Phi_i)^2,
 *   - the constraint solve (prefix sums become suffix sums; the cell-rule and
 *     derivative stencils are transposed, their ghost entries folded back onto
 *     the mirror points with the parity signs),
 *   - the right-hand sides of Eqs. (2)-(3), including the end extrapolation of
 *     tan^2 x A e^-delta Phi, and
 *   - the four stages of every classical RK4 step,
 * with the state stored every K steps and each segment recomputed forward
 * before it is reversed.  Derivatives are accumulated (+=) into the outputs.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "oracle_internal.h"

static double* zalloc(int n) { return calloc((size_t)n, sizeof(double)); }

/* ubar[j] += val for a stencil reference to index j in [-3, N+2], folding a
 * ghost reference back onto its mirror point with the parity sign. */
static void gacc(double* ubar, int N, int j, double p0, double p1, double val)
{
    if (j < 0) ubar[-j] += p0 * val;
    else if (j > N - 1) ubar[2 * (N - 1) - j] += p1 * val;
    else ubar[j] += val;
}

/* Transpose of the cell integrals C_k = h(-u_{k-1}+13u_k+13u_{k+1}-u_{k+2})/24,
 * k = 0..N-2, given Cbar_k. */
static void cell4_T(int N, double h, double p0, double p1, const double* Cbar, double* ubar)
{
    int k;
    for (k = 0; k < N - 1; ++k) {
        double v = h * Cbar[k] / 24.0;
        gacc(ubar, N, k - 1, p0, p1, -v);
        gacc(ubar, N, k, p0, p1, 13.0 * v);
        gacc(ubar, N, k + 1, p0, p1, 13.0 * v);
        gacc(ubar, N, k + 2, p0, p1, -v);
    }
}

/* Transpose of D at row i (weight v = ybar_i). */
static void D_T(double* ubar, int N, int i, double h, double p0, double p1, double v)
{
    double s = v / (12.0 * h);
    gacc(ubar, N, i - 2, p0, p1, s);
    gacc(ubar, N, i - 1, p0, p1, -8.0 * s);
    gacc(ubar, N, i + 1, p0, p1, 8.0 * s);
    gacc(ubar, N, i + 2, p0, p1, -s);
}

/* Transpose of KO at row i. */
static void KO_T(double* ubar, int N, int i, double h, double sig, double p0, double p1, double v)
{
    static const double c[7] = {1.0, -6.0, 15.0, -20.0, 15.0, -6.0, 1.0};
    double s = sig / (64.0 * h) * v;
    int t;
    for (t = 0; t < 7; ++t) gacc(ubar, N, i - 3 + t, p0, p1, c[t] * s);
}

/* (Abar, dbar) -> (Phibar, Pibar) through the constraint solve of (Phi, Pi). */
static void constraints_vjp(const ora_grid* g, int gauge, const double* Phi, const double* Pi,
                            const double* Abar, const double* dbar, double* Phibar, double* Pibar)
{
    int N = g->N, i, k;
    double h = g->h, acc, tot;
    ora_cwork w;
    double *A = zalloc(N), *dl = zalloc(N), *m = zalloc(N);
    double *mbar = zalloc(N), *Sbar = zalloc(N), *Ebar = zalloc(N), *dtbar = zalloc(N);
    double *sigbar = zalloc(N), *pbar = zalloc(N), *qbar = zalloc(N), *Cbar = zalloc(N);
    cwork_alloc(&w, N);
    constraint_solve(g, gauge, Phi, Pi, &w, A, dl, m);

    /* A_i = 1 - c3s_i m_i (interior), m = S / E */
    for (i = 1; i < N - 1; ++i) mbar[i] = -g->c3s[i] * Abar[i];
    for (i = 0; i < N; ++i) {
        Sbar[i] = mbar[i] / w.E[i];
        Ebar[i] = -mbar[i] * w.S[i] / (w.E[i] * w.E[i]);
    }
    /* delta = delta~ - delta~_{N-1} (boundary gauge) or delta~ */
    tot = 0.0;
    for (i = 0; i < N; ++i) {
        dtbar[i] = dbar[i];
        tot += dbar[i];
    }
    if (gauge == ORA_GAUGE_BOUNDARY) dtbar[N - 1] -= tot;
    /* S_i = sum_{k<i} C_k(sigma): C_k gets the suffix sum of Sbar beyond k */
    acc = 0.0;
    for (k = N - 2; k >= 0; --k) {
        acc += Sbar[k + 1];
        Cbar[k] = acc;
    }
    cell4_T(N, h, 1.0, 1.0, Cbar, sigbar);
    sigbar[0] = 0.0;       /* sigma_0 and sigma_{N-1} are fixed to 0 */
    sigbar[N - 1] = 0.0;
    /* sigma = tan^2 x q E */
    for (i = 1; i < N - 1; ++i) {
        qbar[i] += g->t2[i] * w.E[i] * sigbar[i];
        Ebar[i] += g->t2[i] * w.q[i] * sigbar[i];
    }
    /* E = exp(-delta~) */
    for (i = 0; i < N; ++i) dtbar[i] += -w.E[i] * Ebar[i];
    /* delta~_i = -sum_{k<i} C_k(p) */
    acc = 0.0;
    for (k = N - 2; k >= 0; --k) {
        acc += dtbar[k + 1];
        Cbar[k] = -acc;
    }
    cell4_T(N, h, -1.0, -1.0, Cbar, pbar);
    pbar[0] = 0.0;         /* p_0 and p_{N-1} are fixed to 0 */
    pbar[N - 1] = 0.0;
    for (i = 0; i < N; ++i) qbar[i] += g->sc[i] * pbar[i];
    for (i = 0; i < N; ++i) {
        Phibar[i] += 2.0 * Phi[i] * qbar[i];
        Pibar[i] += 2.0 * Pi[i] * qbar[i];
    }
    cwork_free(&w);
    free(A); free(dl); free(m); free(mbar); free(Sbar); free(Ebar); free(dtbar);
    free(sigbar); free(pbar); free(qbar); free(Cbar);
}

/* (kbar0, kbar1) = adjoint of (Phi_t, Pi_t) -> (Phibar, Pibar, Abar, dbar)
 * through the right-hand sides at (Phi, Pi, A, delta). */
static void rhs_vjp(const ora_grid* gr, double ko, int frozen, const double* Phi, const double* Pi,
                    const double* A, const double* delta, const double* kbar0, const double* kbar1,
                    double* Phibar, double* Pibar, double* Abar, double* dbar)
{
    int N = gr->N, i;
    double h = gr->h;
    double *w = zalloc(N), *f1bar = zalloc(N), *f2bar = zalloc(N), *gbar = zalloc(N);
    for (i = 0; i < N; ++i) w[i] = frozen ? 1.0 : A[i] * exp(-delta[i]);
    for (i = 1; i < N - 1; ++i) {
        D_T(f1bar, N, i, h, 1.0, -1.0, kbar0[i]);
        KO_T(Phibar, N, i, h, ko, -1.0, 1.0, kbar0[i]);
        D_T(gbar, N, i, h, -1.0, 1.0, gr->ct2[i] * kbar1[i]);
        KO_T(Pibar, N, i, h, ko, 1.0, -1.0, kbar1[i]);
    }
    /* origin row: Pi_t(0) = 3 D f2 + KO Pi; Phi_t(0) = 0 */
    D_T(f2bar, N, 0, h, -1.0, 1.0, 3.0 * kbar1[0]);
    KO_T(Pibar, N, 0, h, ko, 1.0, -1.0, kbar1[0]);
    /* g_{N-1} = (15 g_{N-2} - 6 g_{N-3} + g_{N-4}) / 10 */
    gbar[N - 2] += 1.5 * gbar[N - 1];
    gbar[N - 3] += -0.6 * gbar[N - 1];
    gbar[N - 4] += 0.1 * gbar[N - 1];
    for (i = 0; i < N - 1; ++i) f2bar[i] += gr->t2[i] * gbar[i];
    for (i = 0; i < N; ++i) {
        double wbar = Pi[i] * f1bar[i] + Phi[i] * f2bar[i];
        Pibar[i] += w[i] * f1bar[i];
        Phibar[i] += w[i] * f2bar[i];
        if (!frozen) {
            double e = exp(-delta[i]);
            Abar[i] += e * wbar;
            dbar[i] += -w[i] * wbar;
        }
    }
    free(w); free(f1bar); free(f2bar); free(gbar);
}

/* Adjoint of one stage map V -> k = F(V) = RHS(V, constraints(V)):
 * Vbar += J_F(V)^T kbar. */
static void stage_vjp(const ora_grid* g, int gauge, int frozen, double ko, const double* V0, const double* V1,
                      const double* kbar0, const double* kbar1, double* Vbar0, double* Vbar1)
{
    int N = g->N;
    ora_cwork cw;
    double *A = zalloc(N), *dl = zalloc(N), *m = zalloc(N), *Abar = zalloc(N), *dbar = zalloc(N);
    cwork_alloc(&cw, N);
    stage_metric(g, gauge, frozen, V0, V1, &cw, A, dl, m);
    rhs_vjp(g, ko, frozen, V0, V1, A, dl, kbar0, kbar1, Vbar0, Vbar1, Abar, dbar);
    if (!frozen) constraints_vjp(g, gauge, V0, V1, Abar, dbar, Vbar0, Vbar1);
    cwork_free(&cw);
    free(A); free(dl); free(m); free(Abar); free(dbar);
}

static void stage_eval(const ora_grid* g, int gauge, int frozen, double ko, const double* V0, const double* V1,
                       double* k0, double* k1)
{
    int N = g->N;
    ora_cwork cw;
    ora_rwork rw;
    double *A = zalloc(N), *dl = zalloc(N), *m = zalloc(N);
    cwork_alloc(&cw, N);
    rwork_alloc(&rw, N);
    stage_metric(g, gauge, frozen, V0, V1, &cw, A, dl, m);
    rhs_eval(g, ko, frozen, V0, V1, A, dl, &rw, k0, k1);
    cwork_free(&cw);
    rwork_free(&rw);
    free(A); free(dl); free(m);
}

/* One classical RK4 step U -> U' and its adjoint Ubar' -> Ubar (in place). */
static void rk4_step(const ora_grid* g, int gauge, int frozen, double ko, double dt, double* U0, double* U1)
{
    int N = g->N, i, s;
    double *k0[4], *k1[4], *V0 = zalloc(N), *V1 = zalloc(N);
    static const double c[4] = {0.0, 0.5, 0.5, 1.0};
    for (s = 0; s < 4; ++s) {
        k0[s] = zalloc(N);
        k1[s] = zalloc(N);
        for (i = 0; i < N; ++i) {
            V0[i] = (s == 0) ? U0[i] : U0[i] + (c[s] * dt) * k0[s - 1][i];
            V1[i] = (s == 0) ? U1[i] : U1[i] + (c[s] * dt) * k1[s - 1][i];
        }
        stage_eval(g, gauge, frozen, ko, V0, V1, k0[s], k1[s]);
    }
    for (i = 0; i < N; ++i) {
        U0[i] = U0[i] + (dt / 6.0) * (k0[0][i] + 2.0 * k0[1][i] + 2.0 * k0[2][i] + k0[3][i]);
        U1[i] = U1[i] + (dt / 6.0) * (k1[0][i] + 2.0 * k1[1][i] + 2.0 * k1[2][i] + k1[3][i]);
    }
    for (s = 0; s < 4; ++s) { free(k0[s]); free(k1[s]); }
    free(V0); free(V1);
}

static void rk4_step_vjp(const ora_grid* g, int gauge, int frozen, double ko, double dt, const double* U0,
                         const double* U1, double* Ub0, double* Ub1)
{
    int N = g->N, i, s;
    double *V0[4], *V1[4], *k0[4], *k1[4], *kb0[4], *kb1[4], *Vb0 = zalloc(N), *Vb1 = zalloc(N);
    static const double c[4] = {0.0, 0.5, 0.5, 1.0};
    static const double b[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
    /* recompute the four stage inputs */
    for (s = 0; s < 4; ++s) {
        V0[s] = zalloc(N); V1[s] = zalloc(N); k0[s] = zalloc(N); k1[s] = zalloc(N);
        kb0[s] = zalloc(N); kb1[s] = zalloc(N);
        for (i = 0; i < N; ++i) {
            V0[s][i] = (s == 0) ? U0[i] : U0[i] + (c[s] * dt) * k0[s - 1][i];
            V1[s][i] = (s == 0) ? U1[i] : U1[i] + (c[s] * dt) * k1[s - 1][i];
        }
        stage_eval(g, gauge, frozen, ko, V0[s], V1[s], k0[s], k1[s]);
    }
    /* U' = U + dt sum_s b_s k_s  ->  kbar_s = dt b_s Ubar' (Ubar' stays in Ub) */
    for (s = 0; s < 4; ++s)
        for (i = 0; i < N; ++i) {
            kb0[s][i] = dt * b[s] * Ub0[i];
            kb1[s][i] = dt * b[s] * Ub1[i];
        }
    /* stage s input V_s = U + c_s dt k_{s-1}: reverse s = 3..0 */
    for (s = 3; s >= 0; --s) {
        memset(Vb0, 0, sizeof(double) * N);
        memset(Vb1, 0, sizeof(double) * N);
        stage_vjp(g, gauge, frozen, ko, V0[s], V1[s], kb0[s], kb1[s], Vb0, Vb1);
        for (i = 0; i < N; ++i) {
            Ub0[i] += Vb0[i];
            Ub1[i] += Vb1[i];
            if (s > 0) {
                kb0[s - 1][i] += c[s] * dt * Vb0[i];
                kb1[s - 1][i] += c[s] * dt * Vb1[i];
            }
        }
    }
    for (s = 0; s < 4; ++s) {
        free(V0[s]); free(V1[s]); free(k0[s]); free(k1[s]); free(kb0[s]); free(kb1[s]);
    }
    free(Vb0); free(Vb1);
}

/* Spectrum of (Phi, Pi) with metric A: a_j, b_j and E_j for j < J. */
static void spectrum_ab(const ora_grid* g, int J, const double* e, const double* de, const double* Phi,
                        const double* Pi, const double* A, double* a, double* bb, double* E)
{
    int N = g->N, i, j;
    for (j = 0; j < J; ++j) {
        double sa = 0.0, sb = 0.0, om = 3.0 + 2.0 * j;
        for (i = 1; i < N - 1; ++i) {
            double sA = sqrt(A[i]);
            sa += g->h * g->t2[i] * e[(size_t)j * N + i] * sA * Pi[i];
            sb += g->h * g->t2[i] * (de[(size_t)j * N + i] / om) * sA * Phi[i];
        }
        a[j] = sa;
        bb[j] = sb;
        E[j] = sa * sa + sb * sb;
    }
}

/* Ebar -> (Phibar, Pibar, Abar). */
static void spectrum_vjp(const ora_grid* g, int J, const double* e, const double* de, const double* Phi,
                         const double* Pi, const double* A, const double* a, const double* bb,
                         const double* Ebar, double* Phibar, double* Pibar, double* Abar)
{
    int N = g->N, i, j;
    for (j = 0; j < J; ++j) {
        double abar = 2.0 * a[j] * Ebar[j], bbar = 2.0 * bb[j] * Ebar[j], om = 3.0 + 2.0 * j;
        for (i = 1; i < N - 1; ++i) {
            double sA = sqrt(A[i]);
            double wa = g->h * g->t2[i] * e[(size_t)j * N + i];
            double wb = g->h * g->t2[i] * (de[(size_t)j * N + i] / om);
            Pibar[i] += abar * wa * sA;
            Phibar[i] += bbar * wb * sA;
            Abar[i] += (abar * wa * Pi[i] + bbar * wb * Phi[i]) / (2.0 * sA);
        }
    }
}

/*
 * L(c) and, when grad != NULL, dL/dc for one instance (the objective above).
 * K = ckpt_every (>= 1): the state is stored every K steps and each segment is
 * recomputed forward before it is reversed.  Returns 1 when the gradient is
 * valid, 0 when min A fell below a_collapse at some step start in [0, t_n]
 * (the forward then stops there and L is evaluated at that step).
 */
int ora_objective(int N, int gauge, double cfl, double ko, double a_collapse, double eps, int Jc, const double* c,
                  int J, int64_t n_steps, int64_t K, double* L, double* grad, double* E0_out, double* ET_out)
{
    ora_grid g;
    ora_cwork cw;
    double *e, *de, *Phi, *Pi, *A, *dl, *m, *a0, *b0, *E0, *aT, *bT, *ET, *Ebar, *Phib, *Pib, *Ab, *db;
    double dt, Lv = 0.0, minA;
    double *ck;
    int64_t n, nseg, seg;
    int i, j, valid = 1, ej = (Jc > J) ? Jc : J;

    grid_make(&g, N);
    cwork_alloc(&cw, N);
    dt = cfl * g.h;
    e = malloc(sizeof(double) * (size_t)ej * N);
    de = malloc(sizeof(double) * (size_t)ej * N);
    ora_modes(N, ej, e, de);
    Phi = zalloc(N); Pi = zalloc(N); A = zalloc(N); dl = zalloc(N); m = zalloc(N);
    a0 = zalloc(J); b0 = zalloc(J); E0 = zalloc(J); aT = zalloc(J); bT = zalloc(J); ET = zalloc(J);
    Ebar = zalloc(J);
    Phib = zalloc(N); Pib = zalloc(N); Ab = zalloc(N); db = zalloc(N);

    /* initial data, Pi(x,0) = eps sum_k c_k e_k(x), pinned Pi_{N-1} = 0 */
    for (i = 0; i < N; ++i) {
        double s = 0.0;
        int k;
        for (k = 0; k < Jc; ++k) s += c[k] * e[(size_t)k * N + i];
        Phi[i] = 0.0;
        Pi[i] = eps * s;
    }
    Pi[N - 1] = 0.0;
    constraint_solve(&g, gauge, Phi, Pi, &cw, A, dl, m);
    spectrum_ab(&g, J, e, de, Phi, Pi, A, a0, b0, E0);

    /* forward with checkpoints every K steps */
    nseg = (n_steps + K - 1) / K;
    ck = malloc(sizeof(double) * 2 * (size_t)N * (size_t)(nseg + 1));
    memcpy(ck, Phi, sizeof(double) * N);
    memcpy(ck + N, Pi, sizeof(double) * N);
    for (n = 0; n < n_steps; ++n) {
        constraint_solve(&g, gauge, Phi, Pi, &cw, A, dl, m);
        minA = A[0];
        for (i = 0; i < N; ++i) if (A[i] < minA) minA = A[i];
        if (minA < a_collapse) { valid = 0; break; }
        rk4_step(&g, gauge, 0, ko, dt, Phi, Pi);
        if ((n + 1) % K == 0) {
            memcpy(ck + 2 * (size_t)N * (size_t)((n + 1) / K), Phi, sizeof(double) * N);
            memcpy(ck + 2 * (size_t)N * (size_t)((n + 1) / K) + N, Pi, sizeof(double) * N);
        }
    }
    constraint_solve(&g, gauge, Phi, Pi, &cw, A, dl, m);
    minA = A[0];
    for (i = 0; i < N; ++i) if (A[i] < minA) minA = A[i];
    if (minA < a_collapse) valid = 0;
    spectrum_ab(&g, J, e, de, Phi, Pi, A, aT, bT, ET);
    for (j = 0; j < J; ++j) Lv += (ET[j] - E0[j]) * (ET[j] - E0[j]);
    *L = Lv;
    if (E0_out) memcpy(E0_out, E0, sizeof(double) * J);
    if (ET_out) memcpy(ET_out, ET, sizeof(double) * J);

    if (grad && valid) {
        double *S0 = zalloc(N), *S1 = zalloc(N), *seg0 = malloc(sizeof(double) * 2 * (size_t)N * (size_t)K);
        /* final spectrum */
        for (j = 0; j < J; ++j) Ebar[j] = 2.0 * (ET[j] - E0[j]);
        spectrum_vjp(&g, J, e, de, Phi, Pi, A, aT, bT, Ebar, Phib, Pib, Ab);
        constraints_vjp(&g, gauge, Phi, Pi, Ab, db, Phib, Pib);
        /* reverse the steps segment by segment */
        for (seg = nseg - 1; seg >= 0; --seg) {
            int64_t n0 = seg * K, n1 = (seg + 1) * K < n_steps ? (seg + 1) * K : n_steps, t;
            memcpy(S0, ck + 2 * (size_t)N * (size_t)seg, sizeof(double) * N);
            memcpy(S1, ck + 2 * (size_t)N * (size_t)seg + N, sizeof(double) * N);
            for (t = n0; t < n1; ++t) {
                memcpy(seg0 + 2 * (size_t)N * (size_t)(t - n0), S0, sizeof(double) * N);
                memcpy(seg0 + 2 * (size_t)N * (size_t)(t - n0) + N, S1, sizeof(double) * N);
                rk4_step(&g, gauge, 0, ko, dt, S0, S1);
            }
            for (t = n1 - 1; t >= n0; --t) {
                const double* u0 = seg0 + 2 * (size_t)N * (size_t)(t - n0);
                rk4_step_vjp(&g, gauge, 0, ko, dt, u0, u0 + N, Phib, Pib);
            }
        }
        /* initial spectrum: E_j(0) enters L with the opposite sign */
        for (j = 0; j < J; ++j) Ebar[j] = -2.0 * (ET[j] - E0[j]);
        for (i = 0; i < N; ++i) {
            Phi[i] = 0.0;
            Pi[i] = ck[N + i];
            Ab[i] = 0.0;
            db[i] = 0.0;
        }
        constraint_solve(&g, gauge, Phi, Pi, &cw, A, dl, m);
        spectrum_vjp(&g, J, e, de, Phi, Pi, A, a0, b0, Ebar, Phib, Pib, Ab);
        constraints_vjp(&g, gauge, Phi, Pi, Ab, db, Phib, Pib);
        /* initial data map */
        for (j = 0; j < Jc; ++j) {
            double s = 0.0;
            for (i = 0; i < N - 1; ++i) s += Pib[i] * e[(size_t)j * N + i];
            grad[j] = eps * s;
        }
        free(S0); free(S1); free(seg0);
    }
    free(ck);
    free(e); free(de); free(Phi); free(Pi); free(A); free(dl); free(m);
    free(a0); free(b0); free(E0); free(aT); free(bT); free(ET); free(Ebar);
    free(Phib); free(Pib); free(Ab); free(db);
    cwork_free(&cw);
    grid_free(&g);
    return valid;
}

/* Exported pieces for the transpose tests. */
void ora_constraints_vjp(int N, int gauge, const double* Phi, const double* Pi, const double* Abar,
                         const double* dbar, double* Phibar, double* Pibar)
{
    ora_grid g;
    grid_make(&g, N);
    constraints_vjp(&g, gauge, Phi, Pi, Abar, dbar, Phibar, Pibar);
    grid_free(&g);
}

void ora_rhs_vjp(int N, double ko, int frozen, const double* Phi, const double* Pi, const double* A,
                 const double* delta, const double* kbar0, const double* kbar1, double* Phibar, double* Pibar,
                 double* Abar, double* dbar)
{
    ora_grid g;
    grid_make(&g, N);
    rhs_vjp(&g, ko, frozen, Phi, Pi, A, delta, kbar0, kbar1, Phibar, Pibar, Abar, dbar);
    grid_free(&g);
}

void ora_step(int N, int gauge, double cfl, double ko, double* Phi, double* Pi)
{
    ora_grid g;
    grid_make(&g, N);
    rk4_step(&g, gauge, 0, ko, cfl * g.h, Phi, Pi);
    grid_free(&g);
}

void ora_step_vjp(int N, int gauge, double cfl, double ko, const double* Phi, const double* Pi, double* Phibar,
                  double* Pibar)
{
    ora_grid g;
    grid_make(&g, N);
    rk4_step_vjp(&g, gauge, 0, ko, cfl * g.h, Phi, Pi, Phibar, Pibar);
    grid_free(&g);
}

void ora_spectrum_vjp(int N, int J, const double* Phi, const double* Pi, const double* A, const double* Ebar,
                      double* Phibar, double* Pibar, double* Abar)
{
    ora_grid g;
    double *e = malloc(sizeof(double) * (size_t)J * N), *de = malloc(sizeof(double) * (size_t)J * N);
    double *a = zalloc(J), *bb = zalloc(J), *E = zalloc(J);
    grid_make(&g, N);
    ora_modes(N, J, e, de);
    spectrum_ab(&g, J, e, de, Phi, Pi, A, a, bb, E);
    spectrum_vjp(&g, J, e, de, Phi, Pi, A, a, bb, Ebar, Phibar, Pibar, Abar);
    free(e); free(de); free(a); free(bb); free(E);
    grid_free(&g);
}
