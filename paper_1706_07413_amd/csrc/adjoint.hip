// Discrete adjoint (reverse-mode derivative) of the batched AdS4 evolution
// (Liebling & Khanna, arXiv:1706.07413, Sec. II), gfx950.
//
// The derivative is that of the computation the forward kernels perform: the
// constraint solve of Eqs. (5)-(6) by two prefix sums, the right-hand sides of
// Eqs. (2)-(3) with their parity ghosts and end extrapolation, the
// Kreiss-Oliger terms and the four stages of classical RK4.  Transposed, the
// prefix sums become suffix sums (total minus exclusive prefix), each stencil
// becomes its mirror image, and a ghost entry's weight goes back to the point
// it mirrors with the parity sign.
//
// Layout and launch shape are those of the forward kernel (stage.h): one
// workgroup per instance, lane l owns points l*P .. l*P+P-1, lane-interleaved
// LDS rows.  For each step t (in reverse) the kernel takes the four stage
// inputs V_s with their e^-delta and S from the stage record that the forward
// recompute of the segment kept (the forward kernel's own arithmetic, its
// tables in LDS), or, where the records would not fit, recomputes them from
// the stored U^t into a per-instance scratch; both are lane-interleaved, so
// each lane reads back only what it (or its forward counterpart) wrote.  Then
// it runs the four stage adjoints in reverse.
#include <math.h>

#include "stage.h"

namespace adscl {
namespace {

// The per-instance stage scratch, in fields of [P][64 W] doubles: the first 16
// hold a step's stage record (StageRec: Phi_s, Pi_s, e^-delta_s, S_s of the
// four stages) when the reverse kernel recomputes the stages itself; then, as
// LaneArr fields, the adjoint state at the start of the step's reverse
// (Phibar', Pibar': 16, 17) and the running adjoint state (18, 19).
constexpr int kFields = 20;

template <int P, int W, bool FULL>
struct Rev {
    static constexpr int NL = 64 * W;
    static constexpr int RS = NL + 2;
    using S_t = Stage<P, W, FULL>;

    // Adds to (vb0, vb1) the adjoint, through the constraint solve of the state
    // (v0, v1), of the cotangents Eb (of e^-delta, gauge applied) and Sb (of S).
    //   S_k = h/24 (24 R_k - 12 s_k + s_{k-1} - s_{k+1}), R_k = sum_{i<=k} s_i,
    //   s = tan^2 x q e^-delta  ->  sbar_j = h/24 (24 sum_{k>=j} Sb_k - 12 Sb_j + Sb_{j+1} - Sb_{j-1});
    //   e^-delta = exp(-(dt_k - shift)), shift = dt_{N-1} (boundary gauge) or 0;
    //   dt_k = -h/24 (24 R_k - 12 p_k + p_{k-1} - p_{k+1} + 2 p_1), p = sin x cos x q.
    // Non-own points must carry Eb = Sb = 0.  The LDS edge and reduction slots
    // must be free on entry; contains two barriers.
    // `val(f, k)` gives Phi (f = 0), Pi (1) and e^-delta (2) of the state at the
    // lane's point k (re-read where needed rather than held across the scans).
    template <class V>
    static __device__ __forceinline__ void constraint_reverse(S_t& sg, V&& val, double* Eb, const double* Sb,
                                                              double* vb0, double* vb1)
    {
        const auto tb = sg.tables();
        const int tid = sg.tid, lane = sg.lane, wv = sg.wv, N = sg.N, i0 = sg.i0;
        const double h24 = sg.h24;
        double* red = sg.red;

        // suffix sums of Sb, accumulated from the outer end: the lane's points
        // from P-1 down, the lanes to its right by doubling steps, the
        // wavefronts to its right from the last one in (never a total minus a
        // prefix, which would lose the small suffixes away from the origin)
        double lt = 0.0;
#pragma unroll
        for (int k = P - 1; k >= 0; --k) lt += Sb[k];
        const double sinc = wave_incl_suffix(lt);
        if (lane == 0) red[W + wv] = sinc;
        if constexpr (S_t::EDGE) {
            if (lane == 0) sg.RSb[2 * wv] = Sb[0];
            if (lane == 63) sg.RSb[2 * wv + 1] = Sb[P - 1];
        } else {
            sg.SE[tid] = Sb[0];
            sg.SE[NL + tid] = Sb[P - 1];
        }
        __syncthreads();
        double sufS[P];
        {
            double run = S_t::from_right(sinc);  // the lanes right of this one in its wavefront
#pragma unroll
            for (int v = W - 1; v > 0; --v)
                if (v > wv) run += red[W + v];
#pragma unroll
            for (int k = P - 1; k >= 0; --k) {
                run += Sb[k];
                sufS[k] = run;
            }
        }
        double sl, sr;
        if constexpr (S_t::EDGE) {
            sl = S_t::from_left(Sb[P - 1]);
            sr = S_t::from_right(Sb[0]);
            if (lane == 0) sl = (wv > 0) ? sg.RSb[2 * (wv > 0 ? wv : 1) - 1] : 0.0;
            if (lane == 63) sr = (wv < W - 1) ? sg.RSb[2 * (wv < W - 1 ? wv : 0) + 2] : 0.0;
        } else {
            sl = (tid > 0) ? sg.SE[NL + tid - 1] : 0.0;
            sr = (tid < NL - 1) ? sg.SE[tid + 1] : 0.0;
        }
        double qb[P], d[P];
        double d0 = 0.0;
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const double suf = sufS[k];
            const double sm = (k == 0) ? sl : Sb[k - 1];
            const double sp = (k == P - 1) ? sr : Sb[k + 1];
            const double sb = h24 * (24.0 * suf - 12.0 * Sb[k] + sp - sm);
            const double t2 = sg.tab(tb, 1, k);
            const double v0 = val(0, k), v1 = val(1, k), Ek = val(2, k);
            const double q = v0 * v0 + v1 * v1;
            qb[k] = sg.own(k) ? t2 * Ek * sb : 0.0;
            const double eb = Eb[k] + (sg.own(k) ? t2 * q * sb : 0.0);
            // cotangent of dt_k; dt_0 is identically 0, its share goes to the shift only
            const double dk = sg.own(k) ? -Ek * eb : 0.0;
            if (k == 0 && tid == 0) {
                d0 = dk;
                d[k] = 0.0;
            } else {
                d[k] = dk;
            }
        }
        // suffix sums of d, the same way
        double lt2 = 0.0;
#pragma unroll
        for (int k = P - 1; k >= 0; --k) lt2 += d[k];
        const double sinc2 = wave_incl_suffix(lt2);
        if (lane == 0) red[wv] = sinc2;
        if constexpr (S_t::EDGE) {
            if (lane == 0) sg.RDt[2 * wv] = d[0];
            if (lane == 63) sg.RDt[2 * wv + 1] = d[P - 1];
        } else {
            sg.PE[tid] = d[0];
            sg.PE[NL + tid] = d[P - 1];
        }
        if (tid == 0) red[4 * W] = d0;
        __syncthreads();
        double sufD[P], tot2 = 0.0;
        {
            double run = S_t::from_right(sinc2);
#pragma unroll
            for (int v = W - 1; v >= 0; --v) {
                if (v > wv) run += red[v];
                tot2 += red[v];
            }
#pragma unroll
            for (int k = P - 1; k >= 0; --k) {
                run += d[k];
                sufD[k] = run;
            }
        }
        // boundary gauge: shift = dt_{N-1} = -h/24 (24 sum p + 2 p_{N-2} + 2 p_1)
        const double shb = sg.bgauge ? -(tot2 + red[4 * W]) : 0.0;
        double dl, dr;
        if constexpr (S_t::EDGE) {
            dl = S_t::from_left(d[P - 1]);
            dr = S_t::from_right(d[0]);
            if (lane == 0) dl = (wv > 0) ? sg.RDt[2 * (wv > 0 ? wv : 1) - 1] : 0.0;
            if (lane == 63) dr = (wv < W - 1) ? sg.RDt[2 * (wv < W - 1 ? wv : 0) + 2] : 0.0;
        } else {
            dl = (tid > 0) ? sg.PE[NL + tid - 1] : 0.0;
            dr = (tid < NL - 1) ? sg.PE[tid + 1] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const int j = i0 + k;
            const double suf = sufD[k];
            const double dm = (k == 0) ? dl : d[k - 1];
            const double dp = (k == P - 1) ? dr : d[k + 1];
            double pb = -h24 * (24.0 * suf - 12.0 * d[k] + dp - dm);
            double ws = 24.0;
            if (j == 1) {
                pb += -h24 * (2.0 * tot2);
                ws += 2.0;
            }
            if (j == N - 2) ws += 2.0;
            pb += shb * (-h24 * ws);
            const double q2 = qb[k] + sg.tab(tb, 0, k) * pb;  // table is 0 off 1..N-2
            if (sg.own(k)) {
                vb0[k] += 2.0 * val(0, k) * q2;
                vb1[k] += 2.0 * val(1, k) * q2;
            }
        }
    }

    // Adjoint of one stage map V -> k = (Phi_t, Pi_t)(V): given the cotangents
    // (kb0, kb1) of k at the own points, returns (vb0, vb1) = J^T kb.  V, e^-delta
    // and S of the stage are stage si of the step's record `stg` (StageRec).
    static __device__ __forceinline__ void stage_reverse(S_t& sg, ADSCL_GLOBAL double* stg, int si,
                                                         const double* kb0,
                                                         const double* kb1, double* vb0, double* vb1)
    {
        // e^-delta of the stage, held through the reverse scans; loaded first,
        // so that the record's lines (which hold the stage's other fields as
        // well) arrive while the cotangents are exchanged
        double VE[P];
        {
            const auto sv = stage_rec<P, NL>(stg, sg.tid);
#pragma unroll
            for (int k = 0; k < P; ++k) VE[k] = sv.ld(si, 2, k);
        }
        const auto tb = sg.tables();
        const int tid = sg.tid, col = sg.col, N = sg.N, i0 = sg.i0;
        const double i12h = sg.i12h, kof = sg.kof;
        double2* U = sg.U;
        double2* F = sg.F;

        double koa[P], kob[P], f1b[P], gb[P];
        if constexpr (S_t::EDGE) {
            // row cotangents in registers: ya (Phi_t rows 1..N-2), yb = kb1 (Pi_t
            // rows 0..N-2), yg = cot^2 x yb (rows of D g); the neighbours' by DPP,
            // the adjacent wavefronts' through RU / RF; ghosts carry zero
            const int lane = sg.lane, wv = sg.wv;
            double ya[P], yg[P];
#pragma unroll
            for (int k = 0; k < P; ++k) {
                ya[k] = (k == 0 && tid == 0) ? 0.0 : kb0[k];
                yg[k] = sg.tab(tb, 2, k) * kb1[k];
            }
            if (lane == 0) {
#pragma unroll
                for (int r = 0; r < 3; ++r) sg.RU[wv * 6 + r] = make_double2(ya[r], kb1[r]);
                sg.RF[wv * 4] = yg[0];
                sg.RF[wv * 4 + 1] = yg[1];
            }
            if (lane == 63) {
#pragma unroll
                for (int r = 0; r < 3; ++r) sg.RU[wv * 6 + 3 + r] = make_double2(ya[P - 1 - r], kb1[P - 1 - r]);
                sg.RF[wv * 4 + 2] = yg[P - 1];
                sg.RF[wv * 4 + 3] = yg[P - 2];
            }
            __syncthreads();
            {
                double2 w[P + 6];  // points i0-3 .. i0+P+2
#pragma unroll
                for (int r = 0; r < 3; ++r) {
                    w[r] = make_double2(S_t::from_left(ya[P - 3 + r]), S_t::from_left(kb1[P - 3 + r]));
                    w[P + 3 + r] = make_double2(S_t::from_right(ya[r]), S_t::from_right(kb1[r]));
                }
#pragma unroll
                for (int k = 0; k < P; ++k) w[3 + k] = make_double2(ya[k], kb1[k]);
                const double2 z = make_double2(0.0, 0.0);
                if (lane == 0) {
                    const bool in = wv > 0;
                    const double2* x = sg.RU + (in ? wv - 1 : 0) * 6;
                    w[2] = in ? x[3] : z;
                    w[1] = in ? x[4] : z;
                    w[0] = in ? x[5] : z;
                }
                if (lane == 63) {
                    const bool in = wv < W - 1;
                    const double2* x = sg.RU + (in ? wv + 1 : 0) * 6;
#pragma unroll
                    for (int r = 0; r < 3; ++r) w[P + 3 + r] = in ? x[r] : z;
                }
#pragma unroll
                for (int k = 0; k < P; ++k) {
                    // the Kreiss-Oliger stencil is symmetric: its transpose is itself
                    koa[k] = kof * (w[k].x - 6.0 * w[k + 1].x + 15.0 * w[k + 2].x - 20.0 * w[k + 3].x
                                    + 15.0 * w[k + 4].x - 6.0 * w[k + 5].x + w[k + 6].x);
                    kob[k] = kof * (w[k].y - 6.0 * w[k + 1].y + 15.0 * w[k + 2].y - 20.0 * w[k + 3].y
                                    + 15.0 * w[k + 4].y - 6.0 * w[k + 5].y + w[k + 6].y);
                    // D is antisymmetric: its transpose is -D
                    f1b[k] = (w[k + 5].x - 8.0 * w[k + 4].x + 8.0 * w[k + 2].x - w[k + 1].x) * i12h;
                }
            }
            {
                double fw[P + 4];  // points i0-2 .. i0+P+1
#pragma unroll
                for (int r = 0; r < 2; ++r) {
                    fw[r] = S_t::from_left(yg[P - 2 + r]);
                    fw[P + 2 + r] = S_t::from_right(yg[r]);
                }
#pragma unroll
                for (int k = 0; k < P; ++k) fw[2 + k] = yg[k];
                if (lane == 0) {
                    const bool in = wv > 0;
                    const double* x = sg.RF + (in ? wv - 1 : 0) * 4;
                    fw[1] = in ? x[2] : 0.0;
                    fw[0] = in ? x[3] : 0.0;
                }
                if (lane == 63) {
                    const bool in = wv < W - 1;
                    const double* x = sg.RF + (in ? wv + 1 : 0) * 4;
                    fw[P + 2] = in ? x[0] : 0.0;
                    fw[P + 3] = in ? x[1] : 0.0;
                }
#pragma unroll
                for (int k = 0; k < P; ++k) gb[k] = (fw[k + 4] - 8.0 * fw[k + 3] + 8.0 * fw[k + 1] - fw[k]) * i12h;
            }
        } else {
            __syncthreads();  // last readers of the LDS rows and edges are done
            // cotangents of the rows: ya (Phi_t rows 1..N-2), yb (Pi_t rows 0..N-2),
            // yg = cot^2 x yb (rows of D g); every other entry of the rows is 0
#pragma unroll
            for (int k = 0; k < P; ++k) {
                if (sg.own(k)) {
                    const double ya = (k == 0 && tid == 0) ? 0.0 : kb0[k];
                    U[k * RS + col] = make_double2(ya, kb1[k]);
                    F[k * RS + col] = make_double2(sg.tab(tb, 2, k) * kb1[k], 0.0);
                }
            }
            const double2 z = make_double2(0.0, 0.0);
            if (tid == 0) {
                U[(P - 1) * RS] = z;
                U[(P - 2) * RS] = z;
                U[(P - 3) * RS] = z;
                F[(P - 1) * RS] = z;
                F[(P - 2) * RS] = z;
            }
            if (FULL) {
                if (tid == NL - 1) {
                    U[0 * RS + NL + 1] = z;
                    U[1 * RS + NL + 1] = z;
                    U[2 * RS + NL + 1] = z;
                    F[0 * RS + NL + 1] = z;
                    F[1 * RS + NL + 1] = z;
                }
            } else if (sg.has_nm2) {
                U[sg.slot(N - 1)] = z;
                U[sg.slot(N)] = z;
                U[sg.slot(N + 1)] = z;
                F[sg.slot(N - 1)] = z;
                F[sg.slot(N)] = z;
            }
            __syncthreads();

            {
                double2 w[P + 6];  // points i0-3 .. i0+P+2
#pragma unroll
                for (int t = 0; t < P + 6; ++t) {
                    const int tt = t - 3;
                    if (tt < 0) w[t] = U[(P + tt) * RS + col - 1];
                    else if (tt < P) w[t] = U[tt * RS + col];
                    else w[t] = U[(tt - P) * RS + col + 1];
                }
#pragma unroll
                for (int k = 0; k < P; ++k) {
                    // the Kreiss-Oliger stencil is symmetric: its transpose is itself
                    koa[k] = kof * (w[k].x - 6.0 * w[k + 1].x + 15.0 * w[k + 2].x - 20.0 * w[k + 3].x
                                    + 15.0 * w[k + 4].x - 6.0 * w[k + 5].x + w[k + 6].x);
                    kob[k] = kof * (w[k].y - 6.0 * w[k + 1].y + 15.0 * w[k + 2].y - 20.0 * w[k + 3].y
                                    + 15.0 * w[k + 4].y - 6.0 * w[k + 5].y + w[k + 6].y);
                    // D is antisymmetric: its transpose is -D
                    f1b[k] = (w[k + 5].x - 8.0 * w[k + 4].x + 8.0 * w[k + 2].x - w[k + 1].x) * i12h;
                }
            }
            {
                double fw[P + 4];  // points i0-2 .. i0+P+1
#pragma unroll
                for (int t = 0; t < P + 4; ++t) {
                    const int tt = t - 2;
                    if (tt < 0) fw[t] = F[(P + tt) * RS + col - 1].x;
                    else if (tt < P) fw[t] = F[tt * RS + col].x;
                    else fw[t] = F[(tt - P) * RS + col + 1].x;
                }
#pragma unroll
                for (int k = 0; k < P; ++k) gb[k] = (fw[k + 4] - 8.0 * fw[k + 3] + 8.0 * fw[k + 1] - fw[k]) * i12h;
            }

        }
        // rows whose stencils reach the ghosts left of x = 0 (Phi odd, Pi even,
        // f1 even, g odd) and the origin row Pi_t(0) = 3 D f2(0) + KO Pi
        double ob = 0.0;
        if (tid == 0) {
            const double ya1 = kb0[1], ya2 = kb0[2];
            const double yb0 = kb1[0], yb1 = kb1[1], yb2 = kb1[2];
            const double yg1 = sg.tab(tb, 2, 1) * kb1[1];
            koa[1] -= kof * (-6.0 * ya1 + ya2);
            koa[2] -= kof * ya1;
            kob[1] += kof * (15.0 * yb0 - 6.0 * yb1 + yb2);
            kob[2] += kof * (-6.0 * yb0 + yb1);
            kob[3] += kof * yb0;
            f1b[1] += ya1 * i12h;
            gb[1] -= yg1 * i12h;
            ob = 3.0 * yb0 * i12h;
        }
        // rows whose stencils reach past pi/2 (Phi even, Pi odd, f1 odd, g even)
        // and g_{N-1} = (15 g_{N-2} - 6 g_{N-3} + g_{N-4}) / 10
        if (sg.near_end) {
            double2 u2, u3;
            double yg2, yg3;
            if constexpr (S_t::EDGE) {  // the last lane owns N-2 (k = P-1) and N-3
                u2 = make_double2(kb0[P - 1], kb1[P - 1]);
                u3 = make_double2(kb0[P - 2], kb1[P - 2]);
                yg2 = sg.tab(tb, 2, P - 1) * kb1[P - 1];
                yg3 = sg.tab(tb, 2, P - 2) * kb1[P - 2];
            } else {
                u2 = U[sg.slot(N - 2)];
                u3 = U[sg.slot(N - 3)];
                yg2 = F[sg.slot(N - 2)].x;
                yg3 = F[sg.slot(N - 3)].x;
            }
            const double gN1 = (8.0 * yg2 - yg3) * i12h;
#pragma unroll
            for (int k = 0; k < P; ++k) {
                const int j = i0 + k;
                if (j == N - 2) {
                    koa[k] += kof * (-6.0 * u2.x + u3.x);
                    kob[k] -= kof * (-6.0 * u2.y + u3.y);
                    f1b[k] += u2.x * i12h;
                    gb[k] += -yg2 * i12h + 1.5 * gN1;
                }
                if (j == N - 3) {
                    koa[k] += kof * u2.x;
                    kob[k] -= kof * u2.y;
                    gb[k] += -0.6 * gN1;
                }
                if (j == N - 4) gb[k] += 0.1 * gN1;
            }
        }

        // stage values: e^-delta held through the reverse scans, Phi_s, Pi_s re-read
        double Eb[P], Sb[P];
        {
            const auto sv = stage_rec<P, NL>(stg, tid);
#pragma unroll
            for (int k = 0; k < P; ++k) {
                const double v0 = sv.ld(si, 0, k), v1 = sv.ld(si, 1, k), E = VE[k], S = sv.ld(si, 3, k);
            double f2b = sg.tab(tb, 1, k) * gb[k];
            if (tid == 0 && k == 1) f2b += 16.0 * ob;
            if (tid == 0 && k == 2) f2b -= 2.0 * ob;
            const double c3s = sg.tab(tb, 2, k) * sg.tab(tb, 0, k);
            const double wk = E - c3s * S;
            const double wb = v1 * f1b[k] + v0 * f2b;
            const bool o = sg.own(k);
            vb0[k] = o ? koa[k] + wk * f2b : 0.0;
            vb1[k] = o ? kob[k] + wk * f1b[k] : 0.0;
            Eb[k] = o ? wb : 0.0;
            Sb[k] = o ? -c3s * wb : 0.0;
            }
        }
        constraint_reverse(
            sg, [&](int f, int k) -> double { return f == 2 ? VE[k] : stage_rec<P, NL>(stg, tid).ld(si, f, k); }, Eb,
            Sb, vb0, vb1);
        if (tid == 0) vb0[0] = 0.0;  // Phi_0 is pinned
    }
};

template <int P, int W, bool FULL>
__global__ void __launch_bounds__(64 * W) adjoint_kernel(AdjointArgs a)
{
    constexpr int NL = 64 * W;
    using R = Rev<P, W, FULL>;
    extern __shared__ double lds[];
    const int b = a.order[blockIdx.x];
    const AdjSeg sq = a.sg[b];
    if (!sq.active) return;
    const InstConst ic = a.ic[b];
    using S_t = Stage<P, W, FULL>;
    S_t sg;
    sg.setup(lds, ic, a.tab[b], a.gauge, 0.0);
    const int N = sg.N, i0 = sg.i0, tid = sg.tid;
    const double dt = sg.dt;
    ADSCL_GLOBAL double* const stg = gmem(a.stg[b]);
    // the step's incoming adjoint state U-bar' (fields 0, 1) and the running one
    // (2, 3): on the edge path in the LDS past the stage's (each lane its own
    // entries), otherwise in the scratch fields 16..19
    double* const au = lds + S_t::lds_doubles;
    auto ub_ld = [&](int f, int k) -> double {
        if constexpr (S_t::EDGE) return au[(f * P + k) * NL + tid];
        return lane_arr<P, NL>(stg, tid).ld(16 + f, k);
    };
    auto ub_st = [&](int f, int k, double v) {
        if constexpr (S_t::EDGE) au[(f * P + k) * NL + tid] = v;
        else lane_arr<P, NL>(stg, tid).st(16 + f, k, v);
    };

#pragma unroll
    for (int k = 0; k < P; ++k) {
        const bool o = sg.own(k);
        ub_st(2, k, o ? a.Ubar[ic.off + i0 + k] : 0.0);
        ub_st(3, k, o ? a.Ubar[a.total + ic.off + i0 + k] : 0.0);
    }

    // the segment's stage record, when the forward recompute kept one
    constexpr size_t kRec = (size_t)16 * P * NL;
    ADSCL_GLOBAL double* const rec = a.keep ? gmem(a.keep[b]) : nullptr;
    for (int64_t t = sq.n1 - 1; t >= sq.n0; --t) {
        // the adjoint state at the start of this step's reverse, U-bar'
#pragma unroll
        for (int k = 0; k < P; ++k) {
            ub_st(0, k, ub_ld(2, k));
            ub_st(1, k, ub_ld(3, k));
        }
        // the stage inputs V_s of step t and their e^-delta and S: read from the
        // record, or recomputed from U^t into the scratch
        ADSCL_GLOBAL double* const st = rec ? rec + (size_t)(t - sq.n0) * kRec : stg;
        if (!rec) {
            const ADSCL_GLOBAL double* u = gmem(a.seg[b]) + (size_t)(t - sq.n0) * 2 * (size_t)N;
            double un0[P], un1[P];
#pragma unroll
            for (int k = 0; k < P; ++k) {
                const bool o = sg.own(k);
                un0[k] = o ? u[i0 + k] : 0.0;
                un1[k] = o ? u[N + i0 + k] : 0.0;
            }
            // the reverse sweep's last readers of the LDS edges are done
            __syncthreads();
            sg.publish(un0, un1);
            double cv0[P], cv1[P];
#pragma unroll
            for (int k = 0; k < P; ++k) {
                cv0[k] = un0[k];
                cv1[k] = un1[k];
            }
#pragma unroll 1
            for (int s = 0; s < 4; ++s) {
                double r0[P], r1[P];
                // stores V_s, e^-delta and S as stage s of the scratch's record
                sg.template rhs<true>(false, false, cv0, cv1, r0, r1, stg, s);
                if (s < 3) {
                    const double c_next = (s == 2) ? dt : 0.5 * dt;
#pragma unroll
                    for (int k = 0; k < P; ++k) {
                        cv0[k] = un0[k] + c_next * r0[k];
                        cv1[k] = un1[k] + c_next * r1[k];
                    }
                    sg.publish(cv0, cv1);
                }
            }
        }
        // reverse of U' = U + dt sum_s b_s k_s with stage inputs V_s = U + c_s dt k_{s-1}:
        // kbar_s = dt b_s U-bar' + c_{s+1} dt Vbar_{s+1}, U-bar = U-bar' + sum_s Vbar_s
        double kb0[P], kb1[P];
#pragma unroll
        for (int k = 0; k < P; ++k) {
            kb0[k] = (dt / 6.0) * ub_ld(0, k);
            kb1[k] = (dt / 6.0) * ub_ld(1, k);
        }
#pragma unroll 1
        for (int s = 3; s >= 0; --s) {
            double vb0[P], vb1[P];
            R::stage_reverse(sg, st, s, kb0, kb1, vb0, vb1);
            const double cs = (s == 3) ? dt : 0.5 * dt;
            const double bp = (s == 1) ? dt / 6.0 : dt / 3.0;
#pragma unroll
            for (int k = 0; k < P; ++k) {
                ub_st(2, k, ub_ld(2, k) + vb0[k]);
                ub_st(3, k, ub_ld(3, k) + vb1[k]);
                kb0[k] = bp * ub_ld(0, k) + cs * vb0[k];
                kb1[k] = bp * ub_ld(1, k) + cs * vb1[k];
            }
        }
    }
#pragma unroll
    for (int k = 0; k < P; ++k) {
        if (sg.own(k)) {
            a.Ubar[ic.off + i0 + k] = ub_ld(2, k);
            a.Ubar[a.total + ic.off + i0 + k] = ub_ld(3, k);
        }
    }
}

// Adjoint at an end point: E_j = Pihat_j^2 + Phihat_j^2 with Pihat_j =
// sum_i wPi_ji sqrt(A_i) Pi_i, Phihat_j = sum_i wPhi_ji sqrt(A_i) Phi_i, then
// A = 1 - cos^3 x / sin x S / e^-delta through the constraint solve.
template <int P, int W, bool FULL>
__global__ void __launch_bounds__(64 * W) endpoint_kernel(EndArgs a)
{
    using R = Rev<P, W, FULL>;
    extern __shared__ double lds[];
    const int b = a.order[blockIdx.x];
    if (a.status[b].state != ST_DONE) return;
    const InstConst ic = a.ic[b];
    Stage<P, W, FULL> sg;
    sg.setup(lds, ic, a.tab[b], a.gauge, 0.0);
    const int N = sg.N, i0 = sg.i0, tid = sg.tid;
    const auto tb = sg.tables();

    double v0[P], v1[P], q[P];
#pragma unroll
    for (int k = 0; k < P; ++k) {
        const bool o = sg.own(k);
        v0[k] = o ? a.Phi[ic.off + i0 + k] : 0.0;
        v1[k] = o ? a.Pi[ic.off + i0 + k] : 0.0;
        q[k] = o ? v0[k] * v0[k] + v1[k] * v1[k] : 0.0;
    }
    double dl[P], E[P], S[P], dN, tot2;
    sg.constraints(q, dl, E, S, dN, tot2);

    double sp[P], sf[P];
#pragma unroll
    for (int k = 0; k < P; ++k) {
        sp[k] = 0.0;
        sf[k] = 0.0;
    }
    const ADSCL_GLOBAL double* wp = gmem(a.wPi[b]);
    const ADSCL_GLOBAL double* wf = gmem(a.wPhi[b]);
    for (int m = 0; m < a.J; ++m) {
        const size_t bj = (size_t)b * a.J + m;
        const double eb = 2.0 * a.sgn * (a.ET[bj] - a.E0[bj]);
        const double ab = 2.0 * a.Pihat[bj] * eb;
        const double bb = 2.0 * a.Phihat[bj] * eb;
#pragma unroll
        for (int k = 0; k < P; ++k) {
            if (sg.own(k)) {
                sp[k] += ab * wp[(size_t)m * N + i0 + k];
                sf[k] += bb * wf[(size_t)m * N + i0 + k];
            }
        }
    }
    double vb0[P], vb1[P], Eb[P], Sb[P];
#pragma unroll
    for (int k = 0; k < P; ++k) {
        const double c3s = sg.tab(tb, 2, k) * sg.tab(tb, 0, k);
        const double Ak = 1.0 - c3s * (S[k] / E[k]);
        const double sA = sqrt(Ak);
        const bool o = sg.own(k);
        vb0[k] = o ? sA * sf[k] : 0.0;
        vb1[k] = o ? sA * sp[k] : 0.0;
        const double Ab = o ? (sp[k] * v1[k] + sf[k] * v0[k]) / (2.0 * sA) : 0.0;
        // A = 1 - c3s S / E
        Eb[k] = o ? c3s * S[k] * Ab / (E[k] * E[k]) : 0.0;
        Sb[k] = o ? -c3s * Ab / E[k] : 0.0;
    }
    __syncthreads();  // the solve's readers of the edge and reduction slots are done
    R::constraint_reverse(
        sg, [&](int f, int k) -> double { return f == 0 ? v0[k] : (f == 1 ? v1[k] : E[k]); }, Eb, Sb, vb0, vb1);
    if (tid == 0) vb0[0] = 0.0;
#pragma unroll
    for (int k = 0; k < P; ++k) {
        if (sg.own(k)) {
            a.Ubar[ic.off + i0 + k] += vb0[k];
            a.Ubar[a.total + ic.off + i0 + k] += vb1[k];
        }
    }
}

__global__ void adj_prepare_kernel(int n_inst, const InstConst* ic, const InstStatus* st, int64_t K, int64_t r,
                                   InstStatus* rst, AdjSeg* sg)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n_inst) return;
    const int64_t nf = ic[b].n_final;
    const int64_t nseg = (nf + K - 1) / K;
    const int64_t s = nseg - 1 - r;
    const bool act = st[b].state == ST_DONE && s >= 0;
    AdjSeg g;
    g.n0 = act ? s * K : 0;
    g.n1 = act ? ((s + 1) * K < nf ? (s + 1) * K : nf) : 0;
    g.active = act ? 1 : 0;
    g.pad = 0;
    sg[b] = g;
    InstStatus o;
    o.steps = g.n0;
    o.target = g.n1;
    o.t_c = -1.0;
    o.minA = 1.0;
    o.mass = 0.0;
    o.state = act ? ST_RUNNING : ST_COLLAPSED;
    o.pad = 0;
    rst[b] = o;
}

// One 256-thread block per instance.
__global__ void __launch_bounds__(256) adj_finish_kernel(int n_inst, const InstConst* ic, const InstStatus* st,
                                                         const double* Ubar, int64_t total,
                                                         const double* const* emode, const double* eps, int Jc,
                                                         const double* E0, const double* ET, int J, double* L,
                                                         double* dLdc, int32_t* valid)
{
    __shared__ double sh[4];
    const int b = blockIdx.x, tid = threadIdx.x;
    const InstConst c = ic[b];
    const bool ok = st[b].state == ST_DONE;
    const double* pib = Ubar + total + c.off;
    for (int k = 0; k < Jc; ++k) {
        const double* e = emode[b] + (size_t)k * c.N;
        double s = 0.0;
        for (int i = tid; i <= c.N - 2; i += 256) s += pib[i] * e[i];
        for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d, 64);
        if ((tid & 63) == 0) sh[tid >> 6] = s;
        __syncthreads();
        if (tid == 0) dLdc[(size_t)b * Jc + k] = ok ? eps[b] * ((sh[0] + sh[1]) + (sh[2] + sh[3])) : 0.0;
        __syncthreads();
    }
    if (tid == 0) {
        double l = 0.0;
        for (int j = 0; j < J; ++j) {
            const double d = ET[(size_t)b * J + j] - E0[(size_t)b * J + j];
            l += d * d;
        }
        L[b] = l;
        valid[b] = ok ? 1 : 0;
    }
}

// Device fill (used instead of a memset so that the enqueue sequence can be
// captured into a graph).
__global__ void fill_kernel(double* p, int64_t n, double v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void mask_kernel(int n_inst, InstStatus* st, const int32_t* active)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n_inst || active[b]) return;
    InstStatus o = st[b];
    o.state = ST_COLLAPSED;
    st[b] = o;
}

__global__ void gd_init_kernel(int n_inst, double step0, GdState g)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b == 0) g.iter[0] = 0;
    if (b >= n_inst) return;
    g.s[b] = step0;
    g.Lprev[b] = INFINITY;
    g.active[b] = 1;
}

// One thread per instance: the descent step of iteration g.iter[0].
__global__ void gd_update_kernel(int n_inst, int Jc, double* c, const double* grad, const double* L,
                                 const int32_t* valid, GdState g, double* L_hist)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n_inst) return;
    const int it = g.iter[0];
    double* lh = L_hist + (size_t)it * n_inst + b;
    if (!g.active[b]) {
        *lh = NAN;
        return;
    }
    const double l = L[b];
    *lh = l;
    if (!valid[b]) {
        g.active[b] = 0;
        return;
    }
    double s = g.s[b];
    if (l > g.Lprev[b]) s *= 0.5;
    g.s[b] = s;
    g.Lprev[b] = l;
    double* cb = c + (size_t)b * Jc;
    const double* gb = grad + (size_t)b * Jc;
    double cn = 0.0, gn = 0.0;
    for (int k = 0; k < Jc; ++k) {
        cn += cb[k] * cb[k];
        gn += gb[k] * gb[k];
    }
    if (gn > 0.0) {
        const double f = s * sqrt(cn) / sqrt(gn);
        for (int k = 0; k < Jc; ++k) cb[k] -= f * gb[k];
    }
}

__global__ void gd_tick_kernel(GdState g)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) g.iter[0] += 1;
}

// LDS of the reverse kernel (the stage's, plus the adjoint state on the edge
// path) and of the end-point kernel
template <int P, int W, bool FULL>
constexpr size_t adj_lds_bytes()
{
    using S_t = Stage<P, W, FULL>;
    return (S_t::lds_doubles + (S_t::EDGE ? (size_t)4 * P * 64 * W : 0)) * sizeof(double);
}

template <int P, int W, bool FULL>
constexpr size_t end_lds_bytes()
{
    return Stage<P, W, FULL>::lds_doubles * sizeof(double);
}

template <int P, int W>
hipError_t launch_adj_t(bool full, int n_blocks, const AdjointArgs& a, hipStream_t s)
{
    if (full)
        adjoint_kernel<P, W, true><<<dim3(n_blocks), dim3(64 * W), adj_lds_bytes<P, W, true>(), s>>>(a);
    else
        adjoint_kernel<P, W, false><<<dim3(n_blocks), dim3(64 * W), adj_lds_bytes<P, W, false>(), s>>>(a);
    return hipGetLastError();
}

template <int P, int W>
hipError_t launch_end_t(bool full, int n_blocks, const EndArgs& a, hipStream_t s)
{
    if (full)
        endpoint_kernel<P, W, true><<<dim3(n_blocks), dim3(64 * W), end_lds_bytes<P, W, true>(), s>>>(a);
    else
        endpoint_kernel<P, W, false><<<dim3(n_blocks), dim3(64 * W), end_lds_bytes<P, W, false>(), s>>>(a);
    return hipGetLastError();
}

template <int P, int W>
hipError_t prepare_adj_t(size_t max_lds)
{
    const void* fns[4] = {(const void*)adjoint_kernel<P, W, true>, (const void*)adjoint_kernel<P, W, false>,
                          (const void*)endpoint_kernel<P, W, true>, (const void*)endpoint_kernel<P, W, false>};
    const size_t need[4] = {adj_lds_bytes<P, W, true>(), adj_lds_bytes<P, W, false>(), end_lds_bytes<P, W, true>(),
                            end_lds_bytes<P, W, false>()};
    for (int i = 0; i < 4; ++i) {
        if (need[i] > max_lds) return hipErrorInvalidValue;
        hipError_t e = hipFuncSetAttribute(fns[i], hipFuncAttributeMaxDynamicSharedMemorySize, (int)need[i]);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

#define ADSCL_ADJ_CLASSES(X) \
    X(4, 1)                  \
    X(4, 2)                  \
    X(4, 4)                  \
    X(4, 8)                  \
    X(4, 16)                 \
    X(8, 1)                  \
    X(8, 2)                  \
    X(8, 4)                  \
    X(8, 8)                  \
    X(16, 1)                 \
    X(16, 2)                 \
    X(16, 4)

size_t adjoint_scratch_len(ClassCfg c) { return (size_t)kFields * c.P * 64 * c.W; }
size_t stage_record_len(ClassCfg c) { return (size_t)16 * c.P * 64 * c.W; }

hipError_t prepare_adjoint(ClassCfg c, size_t max_lds)
{
#define X(p, w) \
    if (c.P == p && c.W == w) return prepare_adj_t<p, w>(max_lds);
    ADSCL_ADJ_CLASSES(X)
#undef X
    return hipErrorInvalidValue;
}

hipError_t launch_adjoint(ClassCfg c, bool full, int n_blocks, const AdjointArgs& a, hipStream_t s)
{
#define X(p, w) \
    if (c.P == p && c.W == w) return launch_adj_t<p, w>(full, n_blocks, a, s);
    ADSCL_ADJ_CLASSES(X)
#undef X
    return hipErrorInvalidValue;
}

hipError_t launch_endpoint(ClassCfg c, bool full, int n_blocks, const EndArgs& a, hipStream_t s)
{
#define X(p, w) \
    if (c.P == p && c.W == w) return launch_end_t<p, w>(full, n_blocks, a, s);
    ADSCL_ADJ_CLASSES(X)
#undef X
    return hipErrorInvalidValue;
}

hipError_t launch_adj_prepare(int n_inst, const InstConst* ic, const InstStatus* st, int64_t K, int64_t r,
                              InstStatus* rst, AdjSeg* sg, hipStream_t s)
{
    adj_prepare_kernel<<<dim3((n_inst + 255) / 256), dim3(256), 0, s>>>(n_inst, ic, st, K, r, rst, sg);
    return hipGetLastError();
}

hipError_t launch_fill(double* p, int64_t n, double v, hipStream_t s)
{
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    fill_kernel<<<dim3((unsigned)blocks), dim3(256), 0, s>>>(p, n, v);
    return hipGetLastError();
}

hipError_t launch_mask(int n_inst, InstStatus* st, const int32_t* active, hipStream_t s)
{
    mask_kernel<<<dim3((n_inst + 255) / 256), dim3(256), 0, s>>>(n_inst, st, active);
    return hipGetLastError();
}

hipError_t launch_gd_init(int n_inst, double step0, const GdState& g, hipStream_t s)
{
    gd_init_kernel<<<dim3((n_inst + 255) / 256), dim3(256), 0, s>>>(n_inst, step0, g);
    return hipGetLastError();
}

hipError_t launch_gd_update(int n_inst, int Jc, double* c, const double* grad, const double* L, const int32_t* valid,
                            const GdState& g, double* L_hist, hipStream_t s)
{
    gd_update_kernel<<<dim3((n_inst + 255) / 256), dim3(256), 0, s>>>(n_inst, Jc, c, grad, L, valid, g, L_hist);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    gd_tick_kernel<<<dim3(1), dim3(64), 0, s>>>(g);
    return hipGetLastError();
}

hipError_t launch_adj_finish(int n_inst, const InstConst* ic, const InstStatus* st, const double* Ubar,
                             int64_t total, const double* const* emode, const double* eps, int Jc,
                             const double* E0, const double* ET, int J, double* L, double* dLdc,
                             int32_t* valid, hipStream_t s)
{
    adj_finish_kernel<<<dim3(n_inst), dim3(256), 0, s>>>(n_inst, ic, st, Ubar, total, emode, eps, Jc, E0, ET, J, L,
                                                        dLdc, valid);
    return hipGetLastError();
}

}  // namespace adscl
