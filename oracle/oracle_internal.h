/* Internals shared by the two oracle translation units (forward scheme and its
 * reverse-mode derivative).  TEST INFRASTRUCTURE ONLY. */
#ifndef ORACLE_INTERNAL_H
#define ORACLE_INTERNAL_H

#include <stdint.h>

#define ORA_PI 3.14159265358979323846

enum { ORA_GAUGE_BOUNDARY = 0, ORA_GAUGE_ORIGIN = 1 };
enum { ORA_RUNNING = 0, ORA_COLLAPSED = 1, ORA_NONFINITE = 2, ORA_DONE = 3 };

typedef struct {
    int N;
    double h;
    double *x, *sn, *cs;   /* sin x_i, cos x_i (exact 0/1 at the two ends)      */
    double *sc;            /* sin x cos x                                        */
    double *t2;            /* tan^2 x (0 at x=0; unused at x=pi/2)               */
    double *ct2;           /* 1/tan^2 x (interior only)                          */
    double *c3s;           /* cos^3 x / sin x (interior only)                    */
} ora_grid;

typedef struct {
    double *q, *p, *dtil, *E, *sig, *S;
} ora_cwork;

typedef struct {
    double *w, *f1, *f2, *g;
} ora_rwork;

void grid_make(ora_grid* g, int N);
void grid_free(ora_grid* g);
double gv(const double* u, int N, int i, double p0, double p1);
double stencil_D(const double* u, int N, int i, double h, double p0, double p1);
double stencil_KO(const double* u, int N, int i, double h, double sig, double p0, double p1);
double cell4(const double* u, int N, int i, double h, double p0, double p1);
void cwork_alloc(ora_cwork* w, int N);
void cwork_free(ora_cwork* w);
void constraint_solve(const ora_grid* g, int gauge, const double* Phi, const double* Pi, ora_cwork* w,
                      double* A, double* delta, double* m);
void rwork_alloc(ora_rwork* r, int N);
void rwork_free(ora_rwork* r);
void rhs_eval(const ora_grid* gr, double ko, int frozen, const double* Phi, const double* Pi, const double* A,
              const double* delta, ora_rwork* r, double* dPhi, double* dPi);
void stage_metric(const ora_grid* g, int gauge, int frozen, const double* Phi, const double* Pi, ora_cwork* w,
                  double* A, double* delta, double* m);
void ora_modes(int N, int J, double* e, double* de);

#endif
