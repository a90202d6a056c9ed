// Fused RK4 evolution of the AdS4 Einstein-Klein-Gordon system for a batch of
// instances (Liebling & Khanna, arXiv:1706.07413, Sec. II), gfx950.
//
// One workgroup owns one instance for the whole call and keeps its state on
// chip: lane l owns the P consecutive grid points l*P .. l*P+P-1 and holds U^n,
// the RK4 accumulator and the Kreiss-Oliger terms of its points in registers;
// the stage input lives in LDS.  A stage is
//   B0  stage input (Phi_s, Pi_s) with parity ghosts in LDS; every lane reads
//       its +-3 window (Kreiss-Oliger terms, q = Phi^2 + Pi^2).
//   B1  delta~ = -int sin x cos x q  (Eq. (6)) as one prefix sum of
//       p = sin x cos x q: lane-serial sums, a wavefront shuffle scan, and the
//       wavefront totals through LDS; then the end correction of the 4-point
//       cell rule.
//   B2  S = int tan^2 x q e^{-delta} as a second prefix sum (Eq. (5) through
//       m = (1 - A) sin x / cos^3 x), and A e^{-delta} = e^{-delta} - cos^3 x/sin x S.
//   B3  fluxes f1 = A e^-delta Pi and g = tan^2 x A e^-delta Phi with parity
//       ghosts in LDS; each lane applies the centred D and KO stencils to its
//       points (Eqs. (2)-(3)), does the RK4 combination and publishes the next
//       stage input.
// Between the first and the last step of a call nothing goes to HBM; the
// metric (A, delta, m) is written only at snapshot steps and at the end.
//
// Prefix-sum form of the cell rule: with C_i = h(-u_{i-1}+13u_i+13u_{i+1}-u_{i+2})/24
// and R_k = sum_{j<=k} u_j,
//   sum_{i<k} C_i = h/24 (24 R_k - 12 u_k + u_{k-1} - u_{k+1} - u_{-1} - 12 u_0 + u_1),
// the same sum of cells regrouped; for p (odd about 0, p_0 = 0) the last three
// terms are 2 p_1, for sigma (even, sigma_0 = 0) they vanish.
// The gauge shift is applied before the exponential: e^{-delta} with delta =
// delta~ - delta~_{N-1} (boundary time, Eq. (12)) or delta = delta~ (origin
// time); S, e^{-delta} and so A e^{-delta} scale consistently, and m = S/e^{-delta}
// does not depend on the shift, so one exponential per point suffices.
#include <math.h>

#include "internal.h"

namespace adscl {
namespace {

__device__ __forceinline__ double wave_incl_scan(double v, int lane)
{
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const double t = __shfl_up(v, d, 64);
        if (lane >= d) v += t;
    }
    return v;
}

__device__ __forceinline__ double wave_min(double v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v = fmin(v, __shfl_xor(v, d, 64));
    return v;
}

// Keeps the compiler from hoisting loop-invariant table loads into registers
// (the tables are re-read from L2 each stage instead): an offset of zero that
// the compiler cannot see through.
__device__ __forceinline__ int opaque_zero()
{
    int z = 0;
    asm volatile("" : "+s"(z));
    return z;
}

template <int P, int W, bool FULL>
__global__ void __launch_bounds__(64 * W) evolve_kernel(EvolveArgs a)
{
    constexpr int NL = 64 * W;      // lanes per instance
    constexpr int CAP = NL * P;     // grid points 0..CAP-1 owned by lanes
    constexpr int LEN = CAP + 8;    // LDS slot of point j is j + 3, j in [-3, CAP+4]
    static_assert(P >= 4, "lane 0 must own grid points 0..3");

    extern __shared__ double lds[];
    double* U0 = lds;               // Phi_s
    double* U1 = lds + LEN;         // Pi_s
    double* F0 = lds + 2 * LEN;     // f1;  p first-values between B0 and B2
    double* F1 = lds + 3 * LEN;     // g;   p last-values between B0 and B2
    double* SE = lds + 4 * LEN;     // sigma first / last values, [2 NL]
    double* red = SE + 2 * NL;      // [0,W) delta~ totals, [W,2W) S totals, [2W,3W) flags,
                                    // [3W,4W) min A, 4W: p_1, 4W+1: p_{N-2}

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wv = tid >> 6;
    const int b = a.order[blockIdx.x];
    const InstStatus st0 = a.status[b];
    if (st0.state == ST_COLLAPSED || st0.state == ST_NONFINITE) return;

    const InstConst ic = a.ic[b];
    const int N = ic.N;
    const int64_t off = ic.off;
    const double h = ic.h, dt = ic.dt, h24 = ic.h24, i12h = ic.i12h, kof = ic.kof;
    const bool frozen = a.frozen != 0;
    const bool bgauge = a.gauge == 0;
    const double thr = a.a_collapse;
    const int64_t n_final = ic.n_final;
    int64_t n_stop = st0.steps + a.max_steps;
    if (n_stop > n_final) n_stop = n_final;
    if (n_stop < st0.steps) n_stop = st0.steps;

    const int i0 = tid * P;
    // FULL: N - 1 == CAP, so every lane owns P evolved points and the last
    // lane owns N-4..N-2; otherwise lanes past N-2 idle and the ends move.
    const bool has_nm2 = FULL ? (tid == NL - 1) : ((i0 <= N - 2) && (N - 2 < i0 + P));
    const bool near_end = FULL ? (tid == NL - 1) : ((i0 + P - 1 >= N - 4) && (i0 <= N - 2));
    auto own = [&](int k) -> bool { return FULL || (i0 + k <= N - 2); };
    const double* const tab0 = a.tab[b];

    // Publish (v0, v1) = (Phi, Pi) at own points with parity ghosts:
    // Phi odd / Pi even about x = 0, Phi even / Pi odd about pi/2, Phi = Pi = 0 at pi/2.
    auto publish = [&](const double* v0, const double* v1) {
#pragma unroll
        for (int k = 0; k < P; ++k) {
            if (own(k)) {
                U0[i0 + k + 3] = v0[k];
                U1[i0 + k + 3] = v1[k];
            }
        }
        if (tid == 0) {
            U0[2] = -v0[1]; U1[2] = v1[1];
            U0[1] = -v0[2]; U1[1] = v1[2];
            U0[0] = -v0[3]; U1[0] = v1[3];
        }
        if (FULL) {
            if (tid == NL - 1) {
                // slots of N-1, N, N+1, N+2 are i0+P+3 .. i0+P+6
                U0[i0 + P + 3] = 0.0;            U1[i0 + P + 3] = 0.0;
                U0[i0 + P + 4] = v0[P - 1];      U1[i0 + P + 4] = -v1[P - 1];
                U0[i0 + P + 5] = v0[P - 2];      U1[i0 + P + 5] = -v1[P - 2];
                U0[i0 + P + 6] = v0[P - 3];      U1[i0 + P + 6] = -v1[P - 3];
            }
        } else if (near_end) {
            // ghost slot of point j >= N-4 is 2(N-1) - j + 3 = base + (P-1-k)
            double* r0 = U0 + (2 * N + 1 - i0 - (P - 1));
            double* r1 = U1 + (2 * N + 1 - i0 - (P - 1));
#pragma unroll
            for (int k = 0; k < P; ++k) {
                const int j = i0 + k;
                if (j >= N - 4 && j <= N - 2) {
                    r0[P - 1 - k] = v0[k];
                    r1[P - 1 - k] = -v1[k];
                }
            }
            if (has_nm2) {
                U0[N + 2] = 0.0;
                U1[N + 2] = 0.0;
            }
        }
    };

    // Constraint solve of the published state: delta (gauge applied),
    // e^{-delta} and S at own points.  Needs the state in U (B0 done by caller).
    // Also returns q, the delta~ end value dN and the S total tot2.
    auto constraints = [&](const double* q, double* dl, double* E, double* S, double& dN, double& tot2) {
        const double* tb = tab0 + opaque_zero();
        double p[P];
        double ptot = 0.0;
#pragma unroll
        for (int k = 0; k < P; ++k) {
            p[k] = tb[(0 * P + k) * NL + tid] * q[k];  // table is 0 off 1..N-2
            ptot += p[k];
        }
        const double incl = wave_incl_scan(ptot, lane);
        if (lane == 63) red[wv] = incl;
        F0[tid] = p[0];
        F1[tid] = p[P - 1];
        if (tid == 0) red[4 * W] = p[1];
        if (FULL) {
            if (tid == NL - 1) red[4 * W + 1] = p[P - 1];
        } else if (has_nm2) {
#pragma unroll
            for (int k = 0; k < P; ++k)
                if (i0 + k == N - 2) red[4 * W + 1] = p[k];
        }
        __syncthreads();  // B1
        double carry = incl - ptot, tot = 0.0;
#pragma unroll
        for (int v = 0; v < W; ++v) {
            const double t = red[v];
            if (v < wv) carry += t;
            tot += t;
        }
        const double p1 = red[4 * W], pN2 = red[4 * W + 1];
        const double pl = (tid > 0) ? F1[tid - 1] : -p1;      // p_{-1} = -p_1
        const double pr = (tid < NL - 1) ? F0[tid + 1] : 0.0; // p_{N-1} = 0
        dN = -h24 * (24.0 * tot + 2.0 * pN2 + 2.0 * p1);       // delta~_{N-1}
        const double shift = bgauge ? dN : 0.0;

        double sg[P];
        double R = carry, stot = 0.0;
#pragma unroll
        for (int k = 0; k < P; ++k) {
            R += p[k];
            const double pm = (k == 0) ? pl : p[k - 1];
            const double pp = (k == P - 1) ? pr : p[k + 1];
            const double dtil = -h24 * (24.0 * R - 12.0 * p[k] + pm - pp + 2.0 * p1);
            dl[k] = dtil - shift;
            E[k] = exp(-dl[k]);
            sg[k] = tb[(1 * P + k) * NL + tid] * q[k] * E[k];  // table is 0 off 1..N-2
            stot += sg[k];
        }
        const double incl2 = wave_incl_scan(stot, lane);
        if (lane == 63) red[W + wv] = incl2;
        SE[tid] = sg[0];
        SE[NL + tid] = sg[P - 1];
        __syncthreads();  // B2
        double carry2 = incl2 - stot;
        tot2 = 0.0;
#pragma unroll
        for (int v = 0; v < W; ++v) {
            const double t = red[W + v];
            if (v < wv) carry2 += t;
            tot2 += t;
        }
        const double sl = (tid > 0) ? SE[NL + tid - 1] : sg[1];  // sigma_{-1} = sigma_1
        const double sr = (tid < NL - 1) ? SE[tid + 1] : 0.0;    // sigma_{N-1} = 0
        double R2 = carry2;
#pragma unroll
        for (int k = 0; k < P; ++k) {
            R2 += sg[k];
            const double sm = (k == 0) ? sl : sg[k - 1];
            const double sp = (k == P - 1) ? sr : sg[k + 1];
            S[k] = h24 * (24.0 * R2 - 12.0 * sg[k] + sm - sp);
        }
    };

    // Solve the constraints of U^n = (v0, v1), write (Phi, Pi, A, delta, m) of
    // the own points to the five arrays o (stride `total`), and reduce min A and
    // the stop flags over the workgroup.  Ends with a barrier.
    auto solve_write = [&](const double* v0, const double* v1, double* o, double& mA, bool& collapsed,
                           bool& nonfinite, double& mass) {
        publish(v0, v1);
        __syncthreads();  // B0
        double q[P], dl[P], E[P], S[P];
        double dN = 0.0, tot2 = 0.0;
#pragma unroll
        for (int k = 0; k < P; ++k) q[k] = v0[k] * v0[k] + v1[k] * v1[k];
        if (!frozen) {
            constraints(q, dl, E, S, dN, tot2);
        } else {
#pragma unroll
            for (int k = 0; k < P; ++k) { dl[k] = 0.0; E[k] = 1.0; S[k] = 0.0; }
        }
        const double* tb = tab0 + opaque_zero();
        double mn = 1.0, chk = 0.0;
        int col = 0;
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const int j = i0 + k;
            if (own(k)) {
                // c3s = cos^3 x / sin x is 0 at x = 0 in the table, so A_0 = 1, w_0 = E_0
                const double c3s = tb[(2 * P + k) * NL + tid] * tb[(0 * P + k) * NL + tid];
                const double mk = S[k] / E[k];
                const double Ak = 1.0 - c3s * mk;
                const double wk = E[k] - c3s * S[k];
                if (wk < thr * E[k]) col = 1;
                mn = fmin(mn, Ak);
                chk = fma(q[k], 0.0, chk);
                chk = fma(wk, 0.0, chk);
                chk = fma(dl[k], 0.0, chk);
                chk = fma(Ak, 0.0, chk);
                o[off + j] = v0[k];
                o[a.total + off + j] = v1[k];
                o[2 * a.total + off + j] = Ak;
                o[3 * a.total + off + j] = dl[k];
                o[4 * a.total + off + j] = frozen ? 0.0 : mk;
            }
        }
        const double Eend = frozen ? 1.0 : (bgauge ? 1.0 : exp(-dN));
        mass = frozen ? 0.0 : h * tot2 / Eend;
        if (has_nm2) {
            o[off + N - 1] = 0.0;
            o[a.total + off + N - 1] = 0.0;
            o[2 * a.total + off + N - 1] = 1.0;
            o[3 * a.total + off + N - 1] = (frozen || bgauge) ? 0.0 : dN;
            o[4 * a.total + off + N - 1] = mass;
        }
        if (!isfinite(dN) || !isfinite(chk)) col |= 2;
        if (1.0 < thr) col |= 1;
        mn = wave_min(mn);
        const int wcol = __any(col & 1) ? 1 : 0;
        const int wnf = __any(col & 2) ? 2 : 0;
        if (lane == 0) {
            red[2 * W + wv] = (double)(wcol | wnf);
            red[3 * W + wv] = mn;
        }
        __syncthreads();
        int fl = 0;
        mA = 1.0;
#pragma unroll
        for (int v = 0; v < W; ++v) {
            fl |= (int)red[2 * W + v];
            mA = fmin(mA, red[3 * W + v]);
        }
        collapsed = (fl & 1) != 0;
        nonfinite = (fl & 2) != 0;
        __syncthreads();  // red and U are reused by the caller
    };

    double un0[P], un1[P], acc0[P], acc1[P];
#pragma unroll
    for (int k = 0; k < P; ++k) {
        const int j = i0 + k;
        const bool own = j <= N - 2;
        un0[k] = own ? a.Phi[off + j] : 0.0;
        un1[k] = own ? a.Pi[off + j] : 0.0;
        acc0[k] = 0.0;
        acc1[k] = 0.0;
    }

    // One RK4 stage on the published stage input; returns true when stage 0
    // finds the instance collapsed or non-finite (nothing is updated then).
    auto stage = [&](const int s) -> bool {
        __syncthreads();  // B0
        const double* tb = tab0 + opaque_zero();
        double q[P];
#pragma unroll
        for (int k = 0; k < P; ++k) {
            // points past N-2 (general N only) read slots nobody wrote: keep them out
            const double v0 = U0[i0 + k + 3], v1 = U1[i0 + k + 3];
            q[k] = own(k) ? v0 * v0 + v1 * v1 : 0.0;
        }
        double dl[P], E[P], S[P];
        double dN = 0.0, tot2 = 0.0;
        if (!frozen) {
            constraints(q, dl, E, S, dN, tot2);
        } else {
#pragma unroll
            for (int k = 0; k < P; ++k) { dl[k] = 0.0; E[k] = 1.0; S[k] = 0.0; }
        }

        // fluxes; c3s and tan^2 x are 0 at x = 0 in the tables, so w_0 = E_0, g_0 = 0
        double f2_1 = 0.0, f2_2 = 0.0, chk = 0.0;
        double gl[3] = {0.0, 0.0, 0.0};  // g at N-2, N-3, N-4 (last lane, FULL)
        int col = 0;
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const int j = i0 + k;
            if (own(k)) {
                const double v0 = U0[i0 + k + 3], v1 = U1[i0 + k + 3];
                const double c3s = tb[(2 * P + k) * NL + tid] * tb[(0 * P + k) * NL + tid];
                const double wk = E[k] - c3s * S[k];
                const double f1 = wk * v1;
                const double f2 = wk * v0;
                const double g = tb[(1 * P + k) * NL + tid] * f2;
                if (k == 1) f2_1 = f2;
                if (k == 2) f2_2 = f2;
                if (k >= P - 3) gl[P - 1 - k] = g;
                if (s == 0) {
                    if (wk < thr * E[k]) col = 1;
                    chk = fma(q[k], 0.0, chk);
                    chk = fma(wk, 0.0, chk);
                    chk = fma(E[k], 0.0, chk);
                }
                F0[j + 3] = f1;
                F1[j + 3] = g;
                if (!FULL) {
                    if (j >= N - 3) {                // f1 odd, g even about pi/2
                        F0[2 * N + 1 - j] = -f1;
                        F1[2 * N + 1 - j] = g;
                    }
                }
            }
        }
        if (tid == 0) {                              // f1 even, g odd about x = 0
            // own values of points 1, 2 are in this lane's registers via F (LDS)
            F0[2] = F0[4]; F1[2] = -F1[4];
            F0[1] = F0[5]; F1[1] = -F1[5];
        }
        if (FULL) {
            if (tid == NL - 1) {                     // slots of N-1, N, N+1
                F0[i0 + P + 3] = 0.0;
                F0[i0 + P + 4] = -F0[i0 + P + 2];
                F1[i0 + P + 4] = F1[i0 + P + 2];
                F0[i0 + P + 5] = -F0[i0 + P + 1];
                F1[i0 + P + 5] = F1[i0 + P + 1];
            }
        } else if (has_nm2) {
            F0[N + 2] = 0.0;                         // f1_{N-1} = 0; g_{N-1} set by readers
        }
        if (s == 0) {
            if (!isfinite(dN) || !isfinite(chk) || 1.0 < thr) col = 1;
            const int wcol = __any(col);
            if (lane == 0) red[2 * W + wv] = wcol ? 1.0 : 0.0;
        }
        __syncthreads();  // B3
        if (s == 0) {
            bool stop = false;
#pragma unroll
            for (int v = 0; v < W; ++v) stop = stop || (red[2 * W + v] != 0.0);
            if (stop) return true;
        }

        // RHS in chunks of C points, so that only the windows of one chunk are
        // live in registers at a time
        constexpr int C = (P >= 8) ? 4 : P;
        const double c_next = (s == 2) ? dt : 0.5 * dt;
        const double wacc = (s == 0 || s == 3) ? 1.0 : 2.0;
        double us0[P], us1[P];
#pragma unroll
        for (int k0 = 0; k0 < P; k0 += C) {
            double fw[C + 4], gw[C + 4];             // points i0+k0-2 .. i0+k0+C+1
            double w0[C + 6], w1[C + 6];             // points i0+k0-3 .. i0+k0+C+2
#pragma unroll
            for (int t = 0; t < C + 4; ++t) {
                fw[t] = F0[i0 + k0 + 1 + t];
                gw[t] = F1[i0 + k0 + 1 + t];
            }
#pragma unroll
            for (int t = 0; t < C + 6; ++t) {
                w0[t] = U0[i0 + k0 + t];
                w1[t] = U1[i0 + k0 + t];
            }
            // g_{N-1}: even 6th-order extrapolation of the finite limit at pi/2
            if (FULL) {
                if (k0 + C == P && tid == NL - 1) gw[C + 2] = (15.0 * gl[0] - 6.0 * gl[1] + gl[2]) / 10.0;
            } else if (near_end) {
                const int tN = (N - 1) - (i0 + k0 - 2);
                if (tN >= 0 && tN < C + 4) {
                    const double gext = (15.0 * F1[N + 1] - 6.0 * F1[N] + F1[N - 1]) / 10.0;
#pragma unroll
                    for (int t = 0; t < C + 4; ++t)
                        if (t == tN) gw[t] = gext;
                }
            }
#pragma unroll
            for (int kk = 0; kk < C; ++kk) {
                const int k = k0 + kk;
                // interior formula everywhere (cot^2 x is 0 at x = 0 in the table);
                // the origin row and points past N-2 are fixed up below
                const double ko0 = kof * (w0[kk] - 6.0 * w0[kk + 1] + 15.0 * w0[kk + 2] - 20.0 * w0[kk + 3]
                                          + 15.0 * w0[kk + 4] - 6.0 * w0[kk + 5] + w0[kk + 6]);
                const double ko1 = kof * (w1[kk] - 6.0 * w1[kk + 1] + 15.0 * w1[kk + 2] - 20.0 * w1[kk + 3]
                                          + 15.0 * w1[kk + 4] - 6.0 * w1[kk + 5] + w1[kk + 6]);
                const double Df1 = (fw[kk] - 8.0 * fw[kk + 1] + 8.0 * fw[kk + 3] - fw[kk + 4]) * i12h;
                const double Dg = (gw[kk] - 8.0 * gw[kk + 1] + 8.0 * gw[kk + 3] - gw[kk + 4]) * i12h;
                double r0 = Df1 + ko0;
                double r1 = tb[(2 * P + k) * NL + tid] * Dg + ko1;
                if (k == 0 && tid == 0) {
                    // Phi_0 = 0; lim tan^-2 (tan^2 f2)' = 3 f2'(0) with f2 odd about x = 0
                    r0 = 0.0;
                    r1 = 3.0 * ((16.0 * f2_1 - 2.0 * f2_2) * i12h) + ko1;
                }
                if (!own(k)) {
                    r0 = 0.0;
                    r1 = 0.0;
                }
                if (s == 0) {
                    acc0[k] = r0;
                    acc1[k] = r1;
                } else {
                    acc0[k] = acc0[k] + wacc * r0;
                    acc1[k] = acc1[k] + wacc * r1;
                }
                if (s < 3) {
                    us0[k] = un0[k] + c_next * r0;
                    us1[k] = un1[k] + c_next * r1;
                } else {
                    un0[k] = un0[k] + (dt / 6.0) * acc0[k];
                    un1[k] = un1[k] + (dt / 6.0) * acc1[k];
                    us0[k] = un0[k];
                    us1[k] = un1[k];
                }
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        __syncthreads();  // B4: every lane has read U_s before U_{s+1} replaces it
        publish(us0, us1);
        return false;
    };

    const bool snaps_on = a.snap_every > 0 && a.snaps != nullptr;
    int64_t n = st0.steps;
    double mA = 1.0, mass = 0.0;
    bool col = false, nf = false;
    publish(un0, un1);
    for (;;) {
        if (n >= n_stop) break;
        if (snaps_on && (n % a.snap_every) == 0 && n / a.snap_every < a.n_slots) {
            double* o = a.snaps + (size_t)(n / a.snap_every) * 5 * (size_t)a.total;
            solve_write(un0, un1, o, mA, col, nf, mass);
            publish(un0, un1);
        }
        int64_t seg_end = n_stop;
        if (snaps_on) {
            const int64_t nb = (n / a.snap_every + 1) * a.snap_every;
            if (nb < seg_end) seg_end = nb;
        }
        bool flagged = false;
        while (n < seg_end) {
            if (stage(0)) { flagged = true; break; }
            stage(1);
            stage(2);
            stage(3);
            ++n;
        }
        if (flagged) break;
    }

    // final solve of U^n: outputs and status, and the snapshot of step n if due
    solve_write(un0, un1, a.Phi, mA, col, nf, mass);
    if (snaps_on && (n % a.snap_every) == 0 && n / a.snap_every < a.n_slots) {
        double* o = a.snaps + (size_t)(n / a.snap_every) * 5 * (size_t)a.total;
        solve_write(un0, un1, o, mA, col, nf, mass);
    }
    if (tid == 0) {
        InstStatus o;
        o.steps = n;
        o.minA = mA;
        o.mass = mass;
        o.t_c = st0.t_c;
        o.pad = 0;
        if (nf) {
            o.state = ST_NONFINITE;
            o.t_c = (double)n * dt;
        } else if (col) {
            o.state = ST_COLLAPSED;
            o.t_c = (double)n * dt;
        } else {
            o.state = (n >= n_final) ? ST_DONE : ST_RUNNING;
        }
        a.status[b] = o;
    }
}

template <int P, int W>
constexpr size_t lds_bytes_for()
{
    return (size_t)(4 * (64 * W * P + 8) + 2 * 64 * W + 4 * W + 8) * sizeof(double);
}

template <int P, int W>
hipError_t launch_t(bool full, int n_blocks, const EvolveArgs& a, hipStream_t s)
{
    const size_t lds = lds_bytes_for<P, W>();
    if (full)
        evolve_kernel<P, W, true><<<dim3(n_blocks), dim3(64 * W), lds, s>>>(a);
    else
        evolve_kernel<P, W, false><<<dim3(n_blocks), dim3(64 * W), lds, s>>>(a);
    return hipGetLastError();
}

template <int P, int W>
hipError_t prepare_t(size_t max_lds)
{
    const size_t need = lds_bytes_for<P, W>();
    if (need > max_lds) return hipErrorInvalidValue;
    hipError_t e = hipFuncSetAttribute((const void*)evolve_kernel<P, W, true>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)need);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void*)evolve_kernel<P, W, false>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)need);
}

}  // namespace

#define ADSCL_CLASSES(X) \
    X(4, 1)              \
    X(4, 2)              \
    X(4, 4)              \
    X(4, 8)              \
    X(4, 16)             \
    X(8, 1)              \
    X(8, 2)              \
    X(8, 4)              \
    X(8, 8)              \
    X(16, 1)             \
    X(16, 2)             \
    X(16, 4)

size_t table_len(ClassCfg c) { return (size_t)3 * c.P * 64 * c.W; }

bool class_supported(ClassCfg c)
{
#define X(p, w) \
    if (c.P == p && c.W == w) return true;
    ADSCL_CLASSES(X)
#undef X
    return false;
}

size_t evolve_lds_bytes(ClassCfg c)
{
    return (size_t)(4 * (64 * c.W * c.P + 8) + 2 * 64 * c.W + 4 * c.W + 8) * sizeof(double);
}

hipError_t prepare_evolve(ClassCfg c, size_t max_lds)
{
#define X(p, w) \
    if (c.P == p && c.W == w) return prepare_t<p, w>(max_lds);
    ADSCL_CLASSES(X)
#undef X
    return hipErrorInvalidValue;
}

hipError_t launch_evolve(ClassCfg c, bool full, int n_blocks, const EvolveArgs& a, hipStream_t s)
{
#define X(p, w) \
    if (c.P == p && c.W == w) return launch_t<p, w>(full, n_blocks, a, s);
    ADSCL_CLASSES(X)
#undef X
    return hipErrorInvalidValue;
}

}  // namespace adscl
