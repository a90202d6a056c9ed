/*
 * adscl oracle: batch drivers.  TEST INFRASTRUCTURE ONLY.
 *
 * Independent instances of the oracle's evolution (adscl_oracle.c) and of its
 * objective and discrete adjoint (adscl_oracle_adj.c), one instance per OpenMP
 * thread at a time (the instances share nothing; each call allocates its own
 * work arrays).  The arithmetic of an instance is the sequential oracle's,
 * unchanged; this file only distributes instances over the host's cores, which
 * is how the CPU baseline of a batched workload is timed.  Built without
 * -fopenmp the loops run on one thread.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#include "oracle_internal.h"

int ora_evolve(int N, int gauge, int frozen, double cfl, double ko, double a_collapse,
               double* Phi, double* Pi, int64_t n0, int64_t n_stop,
               int32_t snap_every, int64_t n_slots, double* snaps,
               double* A, double* delta, double* m,
               int64_t* n_out, double* minA_out, double* tc_out);
void ora_init_gaussian(int N, double eps, double sigma, double* Phi, double* Pi);
int ora_objective(int N, int gauge, double cfl, double ko, double a_collapse, double eps, int Jc, const double* c,
                  int J, int64_t n_steps, int64_t K, double* L, double* grad, double* E0, double* ET);

/* Threads an OpenMP parallel region of this library uses (1 without OpenMP). */
int ora_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Gaussian data (ora_init_gaussian) for instance b, evolved from step 0 to
 * n_stop[b] (or collapse / non-finite): steps[b] and state[b] out. */
void ora_evolve_gaussian_batch(int n, const int32_t* Ns, const double* eps, const double* sigma, int gauge,
                               double cfl, double ko, double a_collapse, const int64_t* n_stop, int64_t* steps,
                               int32_t* state)
{
    int b;
#pragma omp parallel for schedule(dynamic, 1)
    for (b = 0; b < n; ++b) {
        int N = Ns[b];
        double* w = malloc(sizeof(double) * 5 * (size_t)N);
        double *Phi = w, *Pi = w + N, *A = w + 2 * N, *delta = w + 3 * N, *m = w + 4 * N;
        int64_t nout = 0;
        double minA = 0.0, tc = 0.0;
        ora_init_gaussian(N, eps[b], sigma[b], Phi, Pi);
        state[b] = ora_evolve(N, gauge, 0, cfl, ko, a_collapse, Phi, Pi, 0, n_stop[b], 0, 0, NULL, A, delta, m,
                              &nout, &minA, &tc);
        steps[b] = nout;
        free(w);
    }
}

/* ora_objective for every instance b (c row-major [n][Jc]): L[b], grad [n][Jc],
 * valid[b]. */
void ora_objective_batch(int n, const int32_t* Ns, int gauge, double cfl, double ko, double a_collapse,
                         const double* eps, int Jc, const double* c, int J, const int64_t* n_steps, int64_t K,
                         double* L, double* grad, int32_t* valid)
{
    int b;
#pragma omp parallel for schedule(dynamic, 1)
    for (b = 0; b < n; ++b) {
        double* e = malloc(sizeof(double) * 2 * (size_t)J);
        valid[b] = ora_objective(Ns[b], gauge, cfl, ko, a_collapse, eps[b], Jc, c + (size_t)b * Jc, J, n_steps[b],
                                 K, L + b, grad + (size_t)b * Jc, e, e + J);
        free(e);
    }
}
