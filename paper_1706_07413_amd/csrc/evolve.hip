// Fused RK4 evolution of the AdS4 Einstein-Klein-Gordon system for a batch of
// instances (Liebling & Khanna, arXiv:1706.07413, Sec. II), gfx950.
//
// One workgroup owns one instance for the whole call and keeps its state on
// chip: lane l owns the P consecutive grid points l*P .. l*P+P-1 and holds U^n,
// the RK4 accumulator and the Kreiss-Oliger terms of its points in registers;
// the stage input and the fluxes are exchanged through lane-interleaved LDS
// rows.  A stage is
//   B0  stage input (Phi_s, Pi_s) with parity ghosts in LDS; every lane reads
//       its +-3 window: Kreiss-Oliger terms and q = Phi^2 + Pi^2.
//   B1  delta~ = -int sin x cos x q  (Eq. (6)) as one prefix sum of
//       p = sin x cos x q: lane-serial sums, a DPP wavefront scan, and the
//       wavefront totals through LDS; then the end correction of the 4-point
//       cell rule.
//   B2  S = int tan^2 x q e^{-delta} as a second prefix sum (Eq. (5) through
//       m = (1 - A) sin x / cos^3 x), and A e^{-delta} = e^{-delta} - cos^3 x/sin x S.
//   B3  fluxes f1 = A e^-delta Pi and g = tan^2 x A e^-delta Phi with parity
//       ghosts in LDS; each lane applies the centred D stencil to its points
//       (Eqs. (2)-(3)), does the RK4 combination and publishes the next stage
//       input.
// Between the first and the last step of a segment nothing goes to HBM but
// the coefficient-table reads (L2-resident); the segment ends at the call's
// last step or at the next snapshot step, where the finalize kernel solves the
// constraints of the state for the outputs (A, delta, m).
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

// DPP move of a double: both 32-bit halves through the same data-parallel
// primitive (lanes without a source read 0).
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_d(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, ROW_MASK, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROW_MASK, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Inclusive prefix sum over the 64 lanes of a wavefront: shifts by 1, 2, 4, 8
// within rows of 16 lanes, then the row totals through the row broadcasts of
// lanes 15 and 31 (gfx9 DPP row_shr / row_bcast).
__device__ __forceinline__ double wave_incl_scan(double v, int)
{
    v += dpp_d<0x111, 0xf>(v);  // row_shr:1
    v += dpp_d<0x112, 0xf>(v);  // row_shr:2
    v += dpp_d<0x114, 0xf>(v);  // row_shr:4
    v += dpp_d<0x118, 0xf>(v);  // row_shr:8
    v += dpp_d<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
    v += dpp_d<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
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
    constexpr int RS = NL + 2;      // LDS row: column 0 = lane -1, 1..NL = lanes, NL+1 = lane NL
    constexpr int SLOTS = P * RS;
    static_assert(P >= 4, "lane 0 must own grid points 0..3");

    // LDS rows are lane-interleaved: point j = l*P + k sits in row k, column
    // l + 1, so the P reads of a lane's own points and the reads of its
    // neighbours' edge points are consecutive across lanes (no bank conflicts).
    // Column 0 holds the ghosts left of x = 0, column NL + 1 the points past
    // the last lane (the end point and ghosts when N - 1 = 64 W P).
    extern __shared__ double lds[];
    double2* U = reinterpret_cast<double2*>(lds);  // (Phi_s, Pi_s)
    double2* F = U + SLOTS;                        // (f1, g)
    // p first / last per lane: F is free from B0 (its last readers finished
    // the previous stage) until the flux writes after B2
    double* PE = reinterpret_cast<double*>(F);
    double* SE = reinterpret_cast<double*>(F + SLOTS);  // sigma first / last per lane
    double* red = SE + 2 * NL;                     // [0,W) delta~ totals, [W,2W) S totals,
                                                   // [2W,3W) flags, [3W,4W) min A, 4W: p_1, 4W+1: p_{N-2}

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

    const int i0 = tid * P;
    const int col = tid + 1;
    // FULL: N - 1 == 64 W P, so every lane owns P evolved points and the last
    // lane owns N-4..N-2; otherwise lanes past N-2 idle and the end moves.
    const bool has_nm2 = FULL ? (tid == NL - 1) : ((i0 <= N - 2) && (N - 2 < i0 + P));
    const bool near_end = FULL ? (tid == NL - 1) : ((i0 + P + 2 >= N - 4) && (i0 <= N - 2));
    auto own = [&](int k) -> bool { return FULL || (i0 + k <= N - 2); };
    auto slot = [&](int j) -> int {  // LDS index of point j, -P <= j < 64 W P + P
        const int l = (j >= 0) ? (j / P) : -1 - ((-1 - j) / P);
        return (j - l * P) * RS + l + 1;
    };
    const double* const tab0 = a.tab[b];

    // Publish (v0, v1) = (Phi, Pi) of the own points with parity ghosts:
    // Phi odd / Pi even about x = 0, Phi even / Pi odd about pi/2, Phi = Pi = 0 at pi/2.
    auto publish = [&](const double* v0, const double* v1) {
#pragma unroll
        for (int k = 0; k < P; ++k)
            if (own(k)) U[k * RS + col] = make_double2(v0[k], v1[k]);
        if (tid == 0) {
            U[(P - 1) * RS] = make_double2(-v0[1], v1[1]);
            U[(P - 2) * RS] = make_double2(-v0[2], v1[2]);
            U[(P - 3) * RS] = make_double2(-v0[3], v1[3]);
        }
        if (FULL) {
            if (tid == NL - 1) {
                U[0 * RS + NL + 1] = make_double2(0.0, 0.0);
                U[1 * RS + NL + 1] = make_double2(v0[P - 1], -v1[P - 1]);
                U[2 * RS + NL + 1] = make_double2(v0[P - 2], -v1[P - 2]);
                U[3 * RS + NL + 1] = make_double2(v0[P - 3], -v1[P - 3]);
            }
        } else if (near_end) {
#pragma unroll
            for (int k = 0; k < P; ++k) {
                const int j = i0 + k;
                if (j >= N - 4 && j <= N - 2) U[slot(2 * (N - 1) - j)] = make_double2(v0[k], -v1[k]);
            }
            if (has_nm2) U[slot(N - 1)] = make_double2(0.0, 0.0);
        }
    };

    // Constraint solve of the published state given q = Phi^2 + Pi^2 of the
    // own points: delta (gauge applied), e^{-delta} and S at own points, the
    // delta~ end value dN and the S total tot2.  Contains barriers B1 and B2.
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
        PE[tid] = p[0];
        PE[NL + tid] = p[P - 1];
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
        const double pl = (tid > 0) ? PE[NL + tid - 1] : -p1;  // p_{-1} = -p_1
        const double pr = (tid < NL - 1) ? PE[tid + 1] : 0.0;  // p_{N-1} = 0
        dN = -h24 * (24.0 * tot + 2.0 * pN2 + 2.0 * p1);        // delta~_{N-1}
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

    double un0[P], un1[P], acc0[P], acc1[P];
#pragma unroll
    for (int k = 0; k < P; ++k) {
        const int j = i0 + k;
        const bool o = own(k);
        un0[k] = o ? a.Phi[off + j] : 0.0;
        un1[k] = o ? a.Pi[off + j] : 0.0;
        acc0[k] = 0.0;
        acc1[k] = 0.0;
    }

    // One RK4 stage on the published stage input; returns true when stage 0
    // finds the instance collapsed or non-finite (nothing is updated then).
    int stop_bits = 0;
    auto stage = [&](const int s) -> bool {
        __syncthreads();  // B0
        const double* tb = tab0 + opaque_zero();
        // Kreiss-Oliger terms and q of the own points from the +-3 window
        double ko0[P], ko1[P], q[P];
        {
            double2 w[P + 6];                        // points i0-3 .. i0+P+2
#pragma unroll
            for (int t = 0; t < P + 6; ++t) {
                const int tt = t - 3;
                if (tt < 0) w[t] = U[(P + tt) * RS + col - 1];
                else if (tt < P) w[t] = U[tt * RS + col];
                else w[t] = U[(tt - P) * RS + col + 1];
            }
#pragma unroll
            for (int k = 0; k < P; ++k) {
                ko0[k] = kof * (w[k].x - 6.0 * w[k + 1].x + 15.0 * w[k + 2].x - 20.0 * w[k + 3].x
                                + 15.0 * w[k + 4].x - 6.0 * w[k + 5].x + w[k + 6].x);
                ko1[k] = kof * (w[k].y - 6.0 * w[k + 1].y + 15.0 * w[k + 2].y - 20.0 * w[k + 3].y
                                + 15.0 * w[k + 4].y - 6.0 * w[k + 5].y + w[k + 6].y);
                // points past N-2 (general N only) may hold stale slots: keep them out
                q[k] = own(k) ? w[k + 3].x * w[k + 3].x + w[k + 3].y * w[k + 3].y : 0.0;
            }
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
        double fl[3] = {0.0, 0.0, 0.0}, gl[3] = {0.0, 0.0, 0.0};  // f1, g at N-2, N-3, N-4 (FULL)
        double f1a[3] = {0.0, 0.0, 0.0}, ga[3] = {0.0, 0.0, 0.0}; // f1, g at points 1, 2 (lane 0)
        int cl = 0;
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const int j = i0 + k;
            if (own(k)) {
                const double2 v = U[k * RS + col];
                const double c3s = tb[(2 * P + k) * NL + tid] * tb[(0 * P + k) * NL + tid];
                const double wk = E[k] - c3s * S[k];
                const double f1 = wk * v.y;
                const double f2 = wk * v.x;
                const double g = tb[(1 * P + k) * NL + tid] * f2;
                if (k == 1) { f2_1 = f2; f1a[1] = f1; ga[1] = g; }
                if (k == 2) { f2_2 = f2; f1a[2] = f1; ga[2] = g; }
                if (k >= P - 3) { fl[P - 1 - k] = f1; gl[P - 1 - k] = g; }
                if (s == 0) {
                    if (wk < thr * E[k]) cl = 1;
                    chk = fma(q[k], 0.0, chk);
                    chk = fma(wk, 0.0, chk);
                    chk = fma(E[k], 0.0, chk);
                }
                F[k * RS + col] = make_double2(f1, g);
                if (!FULL) {
                    if (j >= N - 3 && j <= N - 2)    // f1 odd, g even about pi/2
                        F[slot(2 * (N - 1) - j)] = make_double2(-f1, g);
                }
            }
        }
        if (tid == 0) {                              // f1 even, g odd about x = 0
            F[(P - 1) * RS] = make_double2(f1a[1], -ga[1]);
            F[(P - 2) * RS] = make_double2(f1a[2], -ga[2]);
        }
        if (FULL) {
            if (tid == NL - 1) {
                // f1_{N-1} = 0; g_{N-1} is the even 6th-order extrapolation of
                // the finite limit at pi/2; then the ghosts N, N+1
                F[0 * RS + NL + 1] = make_double2(0.0, (15.0 * gl[0] - 6.0 * gl[1] + gl[2]) / 10.0);
                F[1 * RS + NL + 1] = make_double2(-fl[0], gl[0]);
                F[2 * RS + NL + 1] = make_double2(-fl[1], gl[1]);
            }
        } else if (has_nm2) {
            F[slot(N - 1)] = make_double2(0.0, 0.0);  // g_{N-1} set by the readers
        }
        if (s == 0) {
            if (1.0 < thr) cl = 1;
            if (!isfinite(dN) || !isfinite(chk)) cl |= 2;
            const int wcol = __any(cl & 1) ? 1 : 0;
            const int wnf = __any(cl & 2) ? 2 : 0;
            if (lane == 0) red[2 * W + wv] = (double)(wcol | wnf);
        }
        __syncthreads();  // B3
        if (s == 0) {
            int fl = 0;
#pragma unroll
            for (int v = 0; v < W; ++v) fl |= (int)red[2 * W + v];
            if (fl) {
                stop_bits = fl;
                return true;
            }
        }

        double2 fw[P + 4];                           // points i0-2 .. i0+P+1
#pragma unroll
        for (int t = 0; t < P + 4; ++t) {
            const int tt = t - 2;
            if (tt < 0) fw[t] = F[(P + tt) * RS + col - 1];
            else if (tt < P) fw[t] = F[tt * RS + col];
            else fw[t] = F[(tt - P) * RS + col + 1];
        }
        if (!FULL && near_end) {
            const int tN = (N - 1) - (i0 - 2);
            if (tN >= 0 && tN < P + 4) {
                const double gext = (15.0 * F[slot(N - 2)].y - 6.0 * F[slot(N - 3)].y + F[slot(N - 4)].y) / 10.0;
#pragma unroll
                for (int t = 0; t < P + 4; ++t)
                    if (t == tN) fw[t].y = gext;
            }
        }
        const double c_next = (s == 2) ? dt : 0.5 * dt;
        const double wacc = (s == 0 || s == 3) ? 1.0 : 2.0;
        double us0[P], us1[P];
#pragma unroll
        for (int k = 0; k < P; ++k) {
            // interior formula everywhere (cot^2 x is 0 at x = 0 in the table);
            // the origin row and points past N-2 are fixed up below
            const double Df1 = (fw[k].x - 8.0 * fw[k + 1].x + 8.0 * fw[k + 3].x - fw[k + 4].x) * i12h;
            const double Dg = (fw[k].y - 8.0 * fw[k + 1].y + 8.0 * fw[k + 3].y - fw[k + 4].y) * i12h;
            double r0 = Df1 + ko0[k];
            double r1 = tb[(2 * P + k) * NL + tid] * Dg + ko1[k];
            if (k == 0 && tid == 0) {
                // Phi_0 = 0; lim tan^-2 (tan^2 f2)' = 3 f2'(0) with f2 odd about x = 0
                r0 = 0.0;
                r1 = 3.0 * ((16.0 * f2_1 - 2.0 * f2_2) * i12h) + ko1[k];
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
        // every lane read U_s before B3, so U_{s+1} may replace it now
        publish(us0, us1);
        return false;
    };

    // Advance to the end of this segment: the call's target step, or the next
    // snapshot step when snapshots are on.
    int64_t n = st0.steps;
    int64_t seg_end = st0.target;
    if (a.snap_every > 0) {
        const int64_t nb = (n / a.snap_every + 1) * a.snap_every;
        if (nb < seg_end) seg_end = nb;
    }
    publish(un0, un1);
    while (n < seg_end) {
        if (stage(0)) break;
#pragma unroll 1
        for (int s = 1; s < 4; ++s) stage(s);
        ++n;
    }
#pragma unroll
    for (int k = 0; k < P; ++k) {
        if (own(k)) {
            a.Phi[off + i0 + k] = un0[k];
            a.Pi[off + i0 + k] = un1[k];
        }
    }
    if (tid == 0) {
        InstStatus o = st0;
        o.steps = n;
        if (stop_bits) {
            o.state = (stop_bits & 2) ? ST_NONFINITE : ST_COLLAPSED;
            o.t_c = (double)n * dt;
        }
        a.status[b] = o;
    }
}

template <int P, int W>
constexpr size_t lds_bytes_for()
{
    // U and F: 2 x P x (64 W + 2) pairs; sigma edges: 2 x 64 W; reductions
    return (size_t)(4 * P * (64 * W + 2) + 2 * 64 * W + 4 * W + 8) * sizeof(double);
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
    return (size_t)(4 * c.P * (64 * c.W + 2) + 2 * 64 * c.W + 4 * c.W + 8) * sizeof(double);
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
