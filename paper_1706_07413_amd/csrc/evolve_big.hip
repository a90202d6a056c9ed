// RK4 evolution of one large instance (N above what one workgroup holds) over
// several workgroups, gfx950 (Liebling & Khanna, arXiv:1706.07413, Sec. II).
//
// The instance's evolved points are cut into G chunks of C = 64 W P points; the
// workgroup of chunk g keeps its points on chip exactly as the single-workgroup
// kernel does (lane-interleaved LDS rows, state in registers) and exchanges
// with the other workgroups through a small global record per chunk, behind
// three grid-wide synchronisations per stage:
//   A  stage input: each chunk's first and last three points (the +-3 stencil
//      halo of its neighbours);
//   B  the constraint scans.  Within a chunk both prefix sums are taken
//      locally, the first without its carry: with R'_k the local prefix of
//      p = sin x cos x q, delta~'_k = -h/24 (24 R'_k - 12 p_k + p_{k-1} - p_{k+1})
//      and E'_k = exp(-delta~'_k), the true weight is e^{-(delta~_k - shift)} =
//      E'_k F_g with one factor per chunk, F_g = exp(24 h/24 C_g + 2 h/24 p_1 +
//      shift), C_g the p total of the chunks before g.  So the local prefix
//      sums of p and of sigma' = tan^2 x q E'_k are all a chunk publishes
//      (with its edge values), and every chunk then finishes its own points:
//      S_k = h/24 (24 (D_g + F_g R2'_k) - 12 s_k + s_{k-1} - s_{k+1}), s = F sigma',
//      D_g = sum_{h<g} F_h (sigma' total of h);
//   C  fluxes: each chunk's first and last two (f1, g) values, and the
//      collapse / non-finite bits of the step's first stage.
// Several large instances share one cooperative launch (as many as the device
// holds at once): each workgroup finds its instance in the launch's table of
// instances and its chunk within it, and every instance keeps its own records
// and counter, so the instances run side by side and only wait for their own
// chunks.
//
// The synchronisation is a monotonic 64-bit arrival counter per instance:
// every workgroup adds one and waits, with a bounded spin, until all G have
// arrived; a spin that runs out sets an error flag and every workgroup leaves
// (the host reports it).  The launch is cooperative, so all G workgroups are
// resident together.
#include <math.h>

#include "stage.h"

namespace adscl {
namespace {

// Per-chunk exchange record (doubles).
enum : int {
    XU_L = 0,    // (Phi, Pi) of points a, a+1, a+2
    XU_R = 6,    // (Phi, Pi) of points a+C-1, a+C-2, a+C-3
    XS_P = 12,   // p total of the chunk
    XS_S = 13,   // sigma' total of the chunk
    XS_SF = 14,  // sigma' at the first point
    XS_SL = 15,  // sigma' at the last point
    XS_P1 = 16,  // p_1 (chunk 0)
    XS_PN = 17,  // p_{N-2} (last chunk)
    XF_L = 18,   // (f1, g) of points a, a+1
    XF_R = 22,   // (f1, g) of points a+C-1, a+C-2
    XF_B = 26,   // collapse / non-finite bits of the chunk
    XREC = 32
};

constexpr unsigned long long kSpinLimit = 1ull << 22;  // about seconds: legitimate waits are microseconds

template <int P, int W>
struct Chunk {
    static constexpr int NL = 64 * W;
    static constexpr int RS = NL + 2;
    static constexpr int SLOTS = P * RS;
    static constexpr int C = P * NL;
    static_assert(P >= 4, "a lane must own at least 4 points");

    double2* U;
    double2* F;
    double* PE;
    double* SE;
    double* red;   // [0,W) p totals, [W,2W) sigma totals, [2W,3W) check bits, 3W gathered bits, 4W.. p_1, p_{N-2}, 4W+7 error
    double* T;     // this chunk's coefficient tables, [3][P][NL], copied into LDS at launch
    double* X64;   // 2^(j/64), j = 0..63, the table of exp_tab
    int tid, lane, wv, g, G, a, i0, col, N;
    bool first, last, has_nm2, near_end, bgauge, frozen;
    double h24, i12h, kof, thr;
    const ADSCL_GLOBAL double* tabI;  // tables of the whole instance, [g][3][P][NL]
    const ADSCL_GLOBAL double* tab0;  // this chunk's
    double tabL, tabR;                 // table 0 at points a - 1 (thread 0) and a + C (the last thread)
    double* xg;                        // exchange records [G][XREC]
    unsigned long long* ctr;
    int* err;
    unsigned long long target;

    __device__ __forceinline__ bool own(int k) const { return i0 + k <= N - 2; }
    __device__ __forceinline__ int slot(int j) const
    {
        const int jl = j - a;
        const int l = (jl >= 0) ? (jl / P) : -1 - ((-1 - jl) / P);
        return (jl - l * P) * RS + l + 1;
    }
    struct TabView {
        const ADSCL_GLOBAL char* base;
        unsigned o;
    };
    __device__ __forceinline__ TabView tables() const
    {
        unsigned o = (unsigned)tid * 8u;
        asm volatile("" : "+v"(o));
        return TabView{(const ADSCL_GLOBAL char*)tab0, o};
    }
    __device__ __forceinline__ double tab(const TabView&, int t, int k) const
    {
        return T[(t * P + k) * NL + tid];
    }
    // table t at global point j of any chunk
    __device__ __forceinline__ double tab_at(int t, int j) const
    {
        const int gg = j / C, jl = j - gg * C, l = jl / P, k = jl - l * P;
        return tabI[(size_t)gg * 3 * C + (size_t)(t * P + k) * NL + l];
    }

    // Grid-wide barrier over the instance's G workgroups.  Returns false when
    // the wait ran out (or another workgroup's did): the caller leaves.
    // Every wavefront first waits for its own stores (the exchange records) to
    // complete, so that after the workgroup barrier one thread's device-scope
    // release (an L2 write-back) covers the whole workgroup; that thread counts
    // in, polls the counter with relaxed loads (an acquiring poll would
    // invalidate L2 on every iteration), acquires once, and the closing barrier
    // passes the acquisition on.
    __device__ __forceinline__ bool grid_sync()
    {
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        target += (unsigned long long)G;
        if (tid == 0) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __hip_atomic_fetch_add(ctr, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            unsigned long long n = 0;
            while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
                __builtin_amdgcn_s_sleep(1);
                if (++n > kSpinLimit || __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                    __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
            }
            red[4 * W + 7] = __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ? 1.0 : 0.0;
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        __syncthreads();
        return red[4 * W + 7] == 0.0;
    }

    __device__ __forceinline__ double* rec(int c) const { return xg + (size_t)c * XREC; }

    // Own points and the parity ghosts at x = 0 / pi/2 into LDS; the chunk's
    // edge points into its exchange record.
    __device__ __forceinline__ void publish(const double* v0, const double* v1)
    {
#pragma unroll
        for (int k = 0; k < P; ++k)
            if (own(k)) U[k * RS + col] = make_double2(v0[k], v1[k]);
        if (tid == 0) {
            if (first) {
                U[(P - 1) * RS] = make_double2(-v0[1], v1[1]);
                U[(P - 2) * RS] = make_double2(-v0[2], v1[2]);
                U[(P - 3) * RS] = make_double2(-v0[3], v1[3]);
            } else {
                double* r = rec(g) + XU_L;
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    r[2 * k] = v0[k];
                    r[2 * k + 1] = v1[k];
                }
            }
        }
        if (!last && tid == NL - 1) {
            double* r = rec(g) + XU_R;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                r[2 * k] = v0[P - 1 - k];
                r[2 * k + 1] = v1[P - 1 - k];
            }
        }
        if (last && near_end) {
#pragma unroll
            for (int k = 0; k < P; ++k) {
                const int j = i0 + k;
                if (j >= N - 4 && j <= N - 2) U[slot(2 * (N - 1) - j)] = make_double2(v0[k], -v1[k]);
            }
            if (has_nm2) U[slot(N - 1)] = make_double2(0.0, 0.0);
        }
    }

    // Sync A and the neighbours' edge points into the ghost columns.
    __device__ __forceinline__ bool exchange_u()
    {
        if (!grid_sync()) return false;
        if (tid == 0 && !first) {
            const double* r = rec(g - 1) + XU_R;
#pragma unroll
            for (int k = 0; k < 3; ++k) U[(P - 1 - k) * RS] = make_double2(r[2 * k], r[2 * k + 1]);
        }
        if (tid == NL - 1 && !last) {
            const double* r = rec(g + 1) + XU_L;
#pragma unroll
            for (int k = 0; k < 3; ++k) U[k * RS + NL + 1] = make_double2(r[2 * k], r[2 * k + 1]);
        }
        return true;
    }

    // Right-hand sides at the published stage input (after exchange_u).  With
    // `check`, the collapse / non-finite bits of the whole instance are
    // returned (nothing else is computed when any is set).  Returns -1 when a
    // grid synchronisation failed.  EVA (A evolved by Eq. (4)): the stage's A
    // of the own points is `av`; only delta's prefix sum runs, the fluxes take
    // w = av e^-delta and the collapse test is av < thr; with `reint` the full
    // solve runs and its A, 1 - cos^3 x/sin x S/e^-delta, replaces `av`.
    // `wout` receives w = A e^-delta of the own points (EVA).
    template <bool EVA = false>
    __device__ __forceinline__ int rhs(bool check, double* r0, double* r1, double* av = nullptr,
                                       double* wout = nullptr, bool reint = false)
    {
        const bool solveS = !EVA || reint;
        __syncthreads();  // B0
        const auto tb = tables();
        double ko0[P], ko1[P], q[P];
        {
            double2 w[P + 6];
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
                q[k] = own(k) ? w[k + 3].x * w[k + 3].x + w[k + 3].y * w[k + 3].y : 0.0;
            }
        }
        // the constraint solve: two scans over the grid (skipped, uniformly for
        // every chunk, with the metric frozen: A = 1, delta = 0)
        double E[P], S[P];
        double dN = 0.0;
        if (frozen) {
#pragma unroll
            for (int k = 0; k < P; ++k) {
                E[k] = 1.0;
                S[k] = 0.0;
            }
        } else {
            // local prefix sums of p and sigma'
            double p[P];
            double ptot = 0.0;
#pragma unroll
            for (int k = 0; k < P; ++k) {
                p[k] = tab(tb, 0, k) * q[k];
                ptot += p[k];
            }
            const double incl = wave_incl_scan(ptot);
            if (lane == 63) red[wv] = incl;
            PE[tid] = p[0];
            PE[NL + tid] = p[P - 1];
            if (first && tid == 0) red[4 * W] = p[1];
            if (has_nm2) {
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
            double pl, pr;
            if (tid > 0) {
                pl = PE[NL + tid - 1];
            } else if (first) {
                pl = -red[4 * W];
            } else {
                const double2 u = U[(P - 1) * RS];  // point a - 1
                pl = tabL * (u.x * u.x + u.y * u.y);
            }
            if (tid < NL - 1) {
                pr = PE[tid + 1];
            } else if (last) {
                pr = 0.0;
            } else {
                const double2 u = U[NL + 1];  // point a + C
                pr = tabR * (u.x * u.x + u.y * u.y);
            }
            double sg[P];
            double R = carry, stot = 0.0;
            const double a24 = 24.0 * h24, a12 = -12.0 * h24;
#pragma unroll
            for (int k = 0; k < P; ++k) {
                R += p[k];
                const double pm = (k == 0) ? pl : p[k - 1];
                const double pp = (k == P - 1) ? pr : p[k + 1];
                // minus the chunk-local delta~': h24 (24 R - 12 p + p_m - p_p), h24 distributed
                E[k] = exp_tab(fma(a24, R, fma(a12, p[k], h24 * (pm - pp))), X64);
                sg[k] = solveS ? tab(tb, 1, k) * q[k] * E[k] : 0.0;
                stot += sg[k];
            }
            double carry2 = 0.0, tot2 = 0.0;
            if (solveS) {  // uniform: the sigma' prefix sums only where S is needed
                const double incl2 = wave_incl_scan(stot);
                if (lane == 63) red[W + wv] = incl2;
                SE[tid] = sg[0];
                SE[NL + tid] = sg[P - 1];
                __syncthreads();  // B2
                carry2 = incl2 - stot;
#pragma unroll
                for (int v = 0; v < W; ++v) {
                    const double t = red[W + v];
                    if (v < wv) carry2 += t;
                    tot2 += t;
                }
            }
            // sync B: chunk totals and edge values
            if (tid == 0) {
                double* r = rec(g);
                r[XS_P] = tot;
                r[XS_S] = tot2;
                r[XS_SF] = sg[0];
                if (first) r[XS_P1] = red[4 * W];
                if (last) r[XS_PN] = red[4 * W + 1];
            }
            if (tid == NL - 1 && !last) rec(g)[XS_SL] = sg[P - 1];
            if (!grid_sync()) return -1;
            // per-chunk factors F_h and the sigma carry D_h: every wavefront
            // forms them itself, lane h (< G <= 64) reading chunk h's record
            // (so the reads after the barrier cost one memory latency) and
            // scanning the chunk totals; its own chunk's values and the
            // neighbours' edge values come by lane shuffles, with no LDS round
            // trip and no workgroup barrier.  Every lane loads from its own
            // record only (vector loads; a lane reads fields no one wrote only
            // where its value is not used).
            double vP = 0.0, vS = 0.0, vSF = 0.0, vSL = 0.0, vP1 = 0.0, vPN = 0.0;
            if (lane < G) {
                const double* r = rec(lane);
                vP = r[XS_P];
                vS = r[XS_S];
                vSF = r[XS_SF];
                vSL = r[XS_SL];
                vP1 = r[XS_P1];
                vPN = r[XS_PN];
            }
            const double p1 = __shfl(vP1, 0);
            const double pN2 = __shfl(vPN, G - 1);
            const double inc = wave_incl_scan(vP);
            const double tp = __shfl(inc, 63);
            const double dNg = -h24 * (24.0 * tp + 2.0 * pN2 + 2.0 * p1);
            const double shift = bgauge ? dNg : 0.0;
            const double Fh = exp_tab(fma(24.0 * h24, inc - vP, fma(2.0 * h24, p1, shift)), X64);
            const double fs = (lane < G) ? Fh * vS : 0.0;
            const double Dh = wave_incl_scan(fs) - fs;
            const double Fg = __shfl(Fh, g);
            const double Dg = __shfl(Dh, g);
            const double Fl = __shfl(Fh, first ? g : g - 1);
            const double Fr = __shfl(Fh, last ? g : g + 1);
            const double eL = __shfl(vSL, first ? g : g - 1);  // sigma' at the last point of chunk g - 1
            const double eR = __shfl(vSF, last ? g : g + 1);   // sigma' at the first point of chunk g + 1
            const double sl = !solveS ? 0.0 : (tid > 0) ? SE[NL + tid - 1]
                                        : (first ? sg[1] : eL * Fl / Fg);
            const double sr = !solveS ? 0.0 : (tid < NL - 1) ? SE[tid + 1]
                                        : (last ? 0.0 : eR * Fr / Fg);
            {
                const double aF = 24.0 * h24 * Fg, hF = h24 * Fg, aD = 24.0 * h24 * Dg;
                double R2 = carry2;
#pragma unroll
                for (int k = 0; k < P; ++k) {
                    R2 += sg[k];
                    const double sm = (k == 0) ? sl : sg[k - 1];
                    const double sp = (k == P - 1) ? sr : sg[k + 1];
                    // h24 (24 (Dg + Fg R2) + Fg (-12 sigma + sigma_m - sigma_p)), h24 and Fg distributed
                    S[k] = fma(aF, R2, fma(hF, fma(-12.0, sg[k], sm - sp), aD));
                    E[k] *= Fg;
                }
            }
            dN = dNg;
        }

        // fluxes
        double f2_1 = 0.0, f2_2 = 0.0, chk = 0.0;
        double f1a[3] = {0.0, 0.0, 0.0}, ga[3] = {0.0, 0.0, 0.0};
        double fb[2][2] = {{0.0, 0.0}, {0.0, 0.0}};  // (f1, g) of the chunk's last two points
        int cl = 0;
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const int j = i0 + k;
            if (own(k)) {
                const double2 v = U[k * RS + col];
                const double c3s = tab(tb, 2, k) * tab(tb, 0, k);
                double wk;
                if constexpr (EVA) {
                    if (reint) av[k] = 1.0 - c3s * (S[k] / E[k]);
                    wk = av[k] * E[k];
                    wout[k] = wk;
                } else {
                    wk = E[k] - c3s * S[k];
                }
                const double f1 = wk * v.y;
                const double f2 = wk * v.x;
                const double gk = tab(tb, 1, k) * f2;
                if (k == 0) { f1a[0] = f1; ga[0] = gk; }
                if (k == 1) { f2_1 = f2; f1a[1] = f1; ga[1] = gk; }
                if (k == 2) { f2_2 = f2; f1a[2] = f1; ga[2] = gk; }
                if (k == P - 1) { fb[0][0] = f1; fb[0][1] = gk; }
                if (k == P - 2) { fb[1][0] = f1; fb[1][1] = gk; }
                if (check) {
                    if (wk < thr * E[k]) cl = 1;
                    chk = fma(q[k], 0.0, chk);
                    chk = fma(wk, 0.0, chk);
                    chk = fma(E[k], 0.0, chk);
                }
                F[k * RS + col] = make_double2(f1, gk);
                if (last && j >= N - 3 && j <= N - 2) F[slot(2 * (N - 1) - j)] = make_double2(-f1, gk);
            }
        }
        if (tid == 0) {
            if (first) {
                F[(P - 1) * RS] = make_double2(f1a[1], -ga[1]);
                F[(P - 2) * RS] = make_double2(f1a[2], -ga[2]);
            } else {
                double* r = rec(g) + XF_L;
                r[0] = f1a[0];
                r[1] = ga[0];
                r[2] = f1a[1];
                r[3] = ga[1];
            }
        }
        if (tid == NL - 1 && !last) {
            double* r = rec(g) + XF_R;
            r[0] = fb[0][0];
            r[1] = fb[0][1];
            r[2] = fb[1][0];
            r[3] = fb[1][1];
        }
        if (has_nm2) F[slot(N - 1)] = make_double2(0.0, 0.0);
        if (check) {
            if (1.0 < thr) cl = 1;
            if (!isfinite(dN) || !isfinite(chk)) cl |= 2;
            const int wcol = __any(cl & 1) ? 1 : 0;
            const int wnf = __any(cl & 2) ? 2 : 0;
            if (lane == 0) red[2 * W + wv] = (double)(wcol | wnf);
        }
        __syncthreads();  // B3
        if (check && tid == 0) {
            int b = 0;
            for (int v = 0; v < W; ++v) b |= (int)red[2 * W + v];
            rec(g)[XF_B] = (double)b;
        }
        if (!grid_sync()) return -1;  // sync C
        if (check) {
            // the first wavefront gathers the chunks' bits, lane h reading chunk h's (G <= 64)
            if (wv == 0) {
                const int bl = (lane < G) ? (int)rec(lane)[XF_B] : 0;
                const int bb = (__any(bl & 1) ? 1 : 0) | (__any(bl & 2) ? 2 : 0);
                if (lane == 0) red[3 * W] = (double)bb;
            }
            __syncthreads();
            const int b = (int)red[3 * W];
            if (b) return b;
        }
        if (tid == 0 && !first) {
            const double* r = rec(g - 1) + XF_R;
            F[(P - 1) * RS] = make_double2(r[0], r[1]);
            F[(P - 2) * RS] = make_double2(r[2], r[3]);
        }
        if (tid == NL - 1 && !last) {
            const double* r = rec(g + 1) + XF_L;
            F[NL + 1] = make_double2(r[0], r[1]);
            F[RS + NL + 1] = make_double2(r[2], r[3]);
        }
        __syncthreads();

        double2 fw[P + 4];
#pragma unroll
        for (int t = 0; t < P + 4; ++t) {
            const int tt = t - 2;
            if (tt < 0) fw[t] = F[(P + tt) * RS + col - 1];
            else if (tt < P) fw[t] = F[tt * RS + col];
            else fw[t] = F[(tt - P) * RS + col + 1];
        }
        if (last && near_end) {
            const int tN = (N - 1) - (i0 - 2);
            if (tN >= 0 && tN < P + 4) {
                const double gext = (15.0 * F[slot(N - 2)].y - 6.0 * F[slot(N - 3)].y + F[slot(N - 4)].y) / 10.0;
#pragma unroll
                for (int t = 0; t < P + 4; ++t)
                    if (t == tN) fw[t].y = gext;
            }
        }
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const double Df1 = (fw[k].x - 8.0 * fw[k + 1].x + 8.0 * fw[k + 3].x - fw[k + 4].x) * i12h;
            const double Dg = (fw[k].y - 8.0 * fw[k + 1].y + 8.0 * fw[k + 3].y - fw[k + 4].y) * i12h;
            r0[k] = Df1 + ko0[k];
            r1[k] = tab(tb, 2, k) * Dg + ko1[k];
            if (first && k == 0 && tid == 0) {
                r0[k] = 0.0;
                r1[k] = 3.0 * ((16.0 * f2_1 - 2.0 * f2_2) * i12h) + ko1[k];
            }
            if (!own(k)) {
                r0[k] = 0.0;
                r1[k] = 0.0;
            }
        }
        return 0;
    }
};

// LDS of a chunk: rows, sigma edges, reductions, tables
template <int P, int W>
constexpr size_t big_lds_bytes_for()
{
    return (StageLayout<P, W>::lds_doubles + (size_t)3 * P * 64 * W + 64) * sizeof(double);
}

// RK: Runge-Kutta order (4 classical; 3 and 2 the Shu-Osher methods, as the
// one-workgroup scheme kernel); EVA: A evolved by Eq. (4) and re-integrated
// from Eq. (5) at steps that are multiples of a.a_reint (its A row of the
// packed state holds the evolved A between calls).
template <int P, int W, int RK, bool EVA>
__global__ void __launch_bounds__(64 * W) evolve_big_kernel(EvolveArgs a, BigArgs x)
{
    extern __shared__ double lds[];
    // this workgroup's instance in the launch (workgroup-uniform)
    int d = 0;
    while (d + 1 < x.n_desc && (int)blockIdx.x >= x.desc[d + 1].first) ++d;
    const BigDesc bd = x.desc[d];
    const int b = bd.inst;
    const InstStatus st0 = a.status[b];
    if (st0.state == ST_COLLAPSED || st0.state == ST_NONFINITE) return;
    const InstConst ic = a.ic[b];
    using Ch = Chunk<P, W>;
    Ch cs;
    cs.U = reinterpret_cast<double2*>(lds);
    cs.F = cs.U + Ch::SLOTS;
    cs.PE = reinterpret_cast<double*>(cs.F);
    cs.SE = reinterpret_cast<double*>(cs.F + Ch::SLOTS);
    cs.red = cs.SE + 2 * Ch::NL;
    cs.tid = threadIdx.x;
    cs.lane = cs.tid & 63;
    cs.wv = cs.tid >> 6;
    cs.g = (int)blockIdx.x - bd.first;
    cs.G = bd.chunks;
    cs.a = cs.g * Ch::C;
    cs.i0 = cs.a + cs.tid * P;
    cs.col = cs.tid + 1;
    cs.N = ic.N;
    cs.first = cs.g == 0;
    cs.last = cs.g == cs.G - 1;
    const int N = ic.N;
    cs.has_nm2 = cs.last && (cs.i0 <= N - 2) && (N - 2 < cs.i0 + P);
    cs.near_end = cs.last && (cs.i0 + P + 2 >= N - 4) && (cs.i0 <= N - 2);
    cs.bgauge = a.gauge == 0;
    cs.frozen = a.frozen != 0;
    cs.h24 = ic.h24;
    cs.i12h = ic.i12h;
    cs.kof = ic.kof;
    cs.thr = a.a_collapse;
    cs.tabI = gmem(a.tab[b]);
    cs.tab0 = cs.tabI + (size_t)cs.g * 3 * Ch::C;
    cs.tabL = (!cs.first && cs.tid == 0) ? cs.tab_at(0, cs.a - 1) : 0.0;
    cs.tabR = (!cs.last && cs.tid == Ch::NL - 1) ? cs.tab_at(0, cs.a + Ch::C) : 0.0;
    // each lane copies exactly the table entries it reads later: no barrier
    cs.T = cs.red + 4 * W + 8;
    cs.X64 = cs.T + 3 * P * Ch::NL;
    // read only after the first stage's barrier B0
    if (cs.tid < 64) cs.X64[cs.tid] = exp2((double)cs.tid * (1.0 / 64.0));
#pragma unroll
    for (int t = 0; t < 3 * P; ++t) cs.T[t * Ch::NL + cs.tid] = cs.tab0[t * Ch::NL + cs.tid];
    cs.xg = x.xch + (size_t)bd.first * XREC;
    cs.ctr = x.ctr + (size_t)d * kBigCtrStride;
    cs.err = reinterpret_cast<int*>(x.ctr + (size_t)d * kBigCtrStride + 1);
    cs.target = 0;
    const double dt = ic.dt;
    const int i0 = cs.i0;

    const int64_t K = a.a_reint;
    // u: U^n; cv: the current stage input; acc: the RK4 accumulator
    double un0[P], un1[P], unA[P], cv0[P], cv1[P], cvA[P], acc0[P], acc1[P], accA[P];
#pragma unroll
    for (int k = 0; k < P; ++k) {
        const bool o = cs.own(k);
        un0[k] = o ? a.Phi[ic.off + i0 + k] : 0.0;
        un1[k] = o ? a.Pi[ic.off + i0 + k] : 0.0;
        unA[k] = (EVA && o) ? a.A[ic.off + i0 + k] : 1.0;
        cv0[k] = un0[k];
        cv1[k] = un1[k];
        cvA[k] = unA[k];
        acc0[k] = acc1[k] = accA[k] = 0.0;
    }
    int stop_bits = 0;
    bool failed = false;
    int64_t n = st0.steps;
    int64_t seg_end = st0.target;
    if (a.snap_every > 0) {
        const int64_t nb = (n / a.snap_every + 1) * a.snap_every;
        if (nb < seg_end) seg_end = nb;
    }
    cs.publish(un0, un1);
    while (n < seg_end && !failed) {
        for (int s = 0; s < RK; ++s) {
            if (!cs.exchange_u()) {
                failed = true;
                break;
            }
            double r0[P], r1[P], w[P], rA[P];
            const bool reint = EVA && s == 0 && (n % K) == 0;
            const int bits = cs.template rhs<EVA>(s == 0, r0, r1, cvA, w, reint);
            if (bits < 0) {
                failed = true;
                break;
            }
            if (bits) {
                stop_bits = bits;
                break;
            }
            if (reint) {
#pragma unroll
                for (int k = 0; k < P; ++k) unA[k] = cvA[k];
            }
            if constexpr (EVA) {
                const auto tb = cs.tables();
#pragma unroll
                for (int k = 0; k < P; ++k) rA[k] = -2.0 * cs.tab(tb, 0, k) * cvA[k] * w[k] * cv0[k] * cv1[k];
            }
            if constexpr (RK == 4 && !EVA) {
                // classical RK4 with the stage value as a per-stage temporary
                const double c_next = (s == 2) ? dt : 0.5 * dt;
                const double wacc = (s == 0 || s == 3) ? 1.0 : 2.0;
                double us0[P], us1[P];
#pragma unroll
                for (int k = 0; k < P; ++k) {
                    if (s == 0) {
                        acc0[k] = r0[k];
                        acc1[k] = r1[k];
                    } else {
                        acc0[k] = acc0[k] + wacc * r0[k];
                        acc1[k] = acc1[k] + wacc * r1[k];
                    }
                    if (s < 3) {
                        us0[k] = un0[k] + c_next * r0[k];
                        us1[k] = un1[k] + c_next * r1[k];
                    } else {
                        un0[k] = un0[k] + (dt / 6.0) * acc0[k];
                        un1[k] = un1[k] + (dt / 6.0) * acc1[k];
                        us0[k] = un0[k];
                        us1[k] = un1[k];
                    }
                }
                cs.publish(us0, us1);
                continue;
            }
#pragma unroll
            for (int k = 0; k < P; ++k) {
                if constexpr (RK == 4) {
                    const double c_next = (s == 2) ? dt : 0.5 * dt;
                    const double wacc = (s == 0 || s == 3) ? 1.0 : 2.0;
                    if (s == 0) {
                        acc0[k] = r0[k];
                        acc1[k] = r1[k];
                        if (EVA) accA[k] = rA[k];
                    } else {
                        acc0[k] = acc0[k] + wacc * r0[k];
                        acc1[k] = acc1[k] + wacc * r1[k];
                        if (EVA) accA[k] = accA[k] + wacc * rA[k];
                    }
                    if (s < 3) {
                        cv0[k] = un0[k] + c_next * r0[k];
                        cv1[k] = un1[k] + c_next * r1[k];
                        if (EVA) cvA[k] = unA[k] + c_next * rA[k];
                    } else {
                        un0[k] = un0[k] + (dt / 6.0) * acc0[k];
                        un1[k] = un1[k] + (dt / 6.0) * acc1[k];
                        if (EVA) unA[k] = unA[k] + (dt / 6.0) * accA[k];
                    }
                } else if constexpr (RK == 3) {
                    if (s == 0) {
                        cv0[k] = un0[k] + dt * r0[k];
                        cv1[k] = un1[k] + dt * r1[k];
                        if (EVA) cvA[k] = unA[k] + dt * rA[k];
                    } else if (s == 1) {
                        cv0[k] = 0.75 * un0[k] + 0.25 * (cv0[k] + dt * r0[k]);
                        cv1[k] = 0.75 * un1[k] + 0.25 * (cv1[k] + dt * r1[k]);
                        if (EVA) cvA[k] = 0.75 * unA[k] + 0.25 * (cvA[k] + dt * rA[k]);
                    } else {
                        un0[k] = un0[k] / 3.0 + (2.0 / 3.0) * (cv0[k] + dt * r0[k]);
                        un1[k] = un1[k] / 3.0 + (2.0 / 3.0) * (cv1[k] + dt * r1[k]);
                        if (EVA) unA[k] = unA[k] / 3.0 + (2.0 / 3.0) * (cvA[k] + dt * rA[k]);
                    }
                } else {
                    if (s == 0) {
                        cv0[k] = un0[k] + dt * r0[k];
                        cv1[k] = un1[k] + dt * r1[k];
                        if (EVA) cvA[k] = unA[k] + dt * rA[k];
                    } else {
                        un0[k] = 0.5 * un0[k] + 0.5 * (cv0[k] + dt * r0[k]);
                        un1[k] = 0.5 * un1[k] + 0.5 * (cv1[k] + dt * r1[k]);
                        if (EVA) unA[k] = 0.5 * unA[k] + 0.5 * (cvA[k] + dt * rA[k]);
                    }
                }
            }
            if (s == RK - 1) {
#pragma unroll
                for (int k = 0; k < P; ++k) {
                    cv0[k] = un0[k];
                    cv1[k] = un1[k];
                    cvA[k] = unA[k];
                }
            }
            cs.publish(cv0, cv1);
        }
        if (stop_bits || failed) break;
        ++n;
    }
#pragma unroll
    for (int k = 0; k < P; ++k) {
        if (cs.own(k)) {
            a.Phi[ic.off + i0 + k] = un0[k];
            a.Pi[ic.off + i0 + k] = un1[k];
            if (EVA) a.A[ic.off + i0 + k] = unA[k];
        }
    }
    if (cs.g == 0 && cs.tid == 0) {
        InstStatus o = st0;
        o.steps = n;
        if (failed) {
            o.state = ST_NONFINITE;
            o.t_c = -2.0;
        } else if (stop_bits) {
            o.state = (stop_bits & 2) ? ST_NONFINITE : ST_COLLAPSED;
            o.t_c = (double)n * dt;
        }
        a.status[b] = o;
    }
}

// Counters and error flags of the launch's instances to zero.
__global__ void big_reset_kernel(BigArgs x)
{
    const int d = threadIdx.x;
    if (d < x.n_desc) {
        x.ctr[(size_t)d * kBigCtrStride] = 0ull;
        x.ctr[(size_t)d * kBigCtrStride + 1] = 0ull;
    }
}

template <int P, int W, int RK, bool EVA>
hipError_t launch_big_t(int blocks, const EvolveArgs& a, const BigArgs& x, hipStream_t s)
{
    if (x.n_desc < 1 || x.n_desc > 1024) return hipErrorInvalidValue;
    big_reset_kernel<<<dim3(1), dim3(1024), 0, s>>>(x);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t lds = big_lds_bytes_for<P, W>();
    EvolveArgs ea = a;
    BigArgs xa = x;
    void* args[] = {(void*)&ea, (void*)&xa};
    return hipLaunchCooperativeKernel((const void*)evolve_big_kernel<P, W, RK, EVA>, dim3(blocks), dim3(64 * W), args,
                                      lds, s);
}

template <int P, int W, int RK, bool EVA>
hipError_t capacity_t(int device, int* blocks)
{
    int cus = 0, per_cu = 0;
    hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
    if (e != hipSuccess) return e;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)evolve_big_kernel<P, W, RK, EVA>, 64 * W,
                                                     big_lds_bytes_for<P, W>());
    if (e != hipSuccess) return e;
    *blocks = per_cu * cus;
    return hipSuccess;
}

template <int P, int W, int RK, bool EVA>
hipError_t prepare_big_t(size_t max_lds)
{
    const size_t need = big_lds_bytes_for<P, W>();
    if (need > max_lds) return hipErrorInvalidValue;
    return hipFuncSetAttribute((const void*)evolve_big_kernel<P, W, RK, EVA>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)need);
}

// The kernel variant of a scheme: RK order 2, 3 or 4, A solved or evolved.
#define ADSCL_BIG_SCHEME(FN, p, w, ...)                                               \
    do {                                                                              \
        if (rk == 4 && !eva) return FN<p, w, 4, false>(__VA_ARGS__);                 \
        if (rk == 4 && eva) return FN<p, w, 4, true>(__VA_ARGS__);                   \
        if (rk == 3 && !eva) return FN<p, w, 3, false>(__VA_ARGS__);                 \
        if (rk == 3 && eva) return FN<p, w, 3, true>(__VA_ARGS__);                   \
        if (rk == 2 && !eva) return FN<p, w, 2, false>(__VA_ARGS__);                 \
        if (rk == 2 && eva) return FN<p, w, 2, true>(__VA_ARGS__);                   \
        return hipErrorInvalidValue;                                                  \
    } while (0)

}  // namespace

#define ADSCL_BIG_CLASSES(X) \
    X(4, 4)                  \
    X(4, 8)

bool big_class_supported(ClassCfg c)
{
#define X(p, w) \
    if (c.P == p && c.W == w) return true;
    ADSCL_BIG_CLASSES(X)
#undef X
    return false;
}

size_t big_lds_bytes(ClassCfg c)
{
    return ((size_t)4 * c.P * (64 * c.W + 2) + 2 * 64 * c.W + 4 * c.W + 8 + 3 * c.P * 64 * c.W) *
           sizeof(double);
}

hipError_t prepare_evolve_big(ClassCfg c, int rk, bool eva, size_t max_lds)
{
#define X(p, w) \
    if (c.P == p && c.W == w) ADSCL_BIG_SCHEME(prepare_big_t, p, w, max_lds);
    ADSCL_BIG_CLASSES(X)
#undef X
    return hipErrorInvalidValue;
}

hipError_t launch_evolve_big(ClassCfg c, int rk, bool eva, int blocks, const EvolveArgs& a, const BigArgs& x,
                             hipStream_t s)
{
#define X(p, w) \
    if (c.P == p && c.W == w) ADSCL_BIG_SCHEME(launch_big_t, p, w, blocks, a, x, s);
    ADSCL_BIG_CLASSES(X)
#undef X
    return hipErrorInvalidValue;
}

hipError_t big_capacity(ClassCfg c, int rk, bool eva, int device, int* blocks)
{
#define X(p, w) \
    if (c.P == p && c.W == w) ADSCL_BIG_SCHEME(capacity_t, p, w, device, blocks);
    ADSCL_BIG_CLASSES(X)
#undef X
    return hipErrorInvalidValue;
}

}  // namespace adscl
