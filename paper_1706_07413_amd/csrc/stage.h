// One workgroup's view of one instance during an RK4 stage of the AdS4
// Einstein-Klein-Gordon evolution (Liebling & Khanna, arXiv:1706.07413,
// Sec. II), shared by the forward evolution kernel and the reverse (adjoint)
// kernel, which recomputes forward stages.
//
// Lane l of the workgroup owns the P consecutive grid points l*P .. l*P+P-1.
// LDS rows are lane-interleaved: point j = l*P + k sits in row k, column l + 1,
// so the P reads of a lane's own points and the reads of its neighbours' edge
// points are consecutive across lanes (no bank conflicts).  Column 0 holds the
// ghosts left of x = 0, column NL + 1 the points past the last lane (the end
// point and its ghosts when N - 1 = 64 W P, "FULL").
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
#pragma once

#include <math.h>

#include "internal.h"

namespace adscl {

// Global-memory (address space 1) view of a device pointer.  A pointer read
// from a per-instance pointer array is generic to the compiler, which then
// emits flat memory instructions (64-bit VGPR addresses per access, counted
// against the LDS wait counter as well); through this cast it emits global ones.
#define ADSCL_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ ADSCL_GLOBAL T* gmem(T* p)
{
    return (ADSCL_GLOBAL T*)p;
}

// DPP move of a double: both 32-bit halves through the same data-parallel
// primitive (lanes without a source read 0).  With every row enabled the
// zero comes from the bound control, so no destination has to be cleared
// first; a partial row mask keeps the old value (0) in the masked rows.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_d(double v)
{
    constexpr bool bc = ROW_MASK == 0xf;
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, ROW_MASK, 0xf, bc);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROW_MASK, 0xf, bc);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// DPP move of a double where lanes without a source lane keep `old`.
template <int CTRL>
__device__ __forceinline__ double dpp_old(double old, double v)
{
    const long long o = __double_as_longlong(old), b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp((int)(o & 0xffffffffll), (int)(b & 0xffffffffll), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(o >> 32), (int)(b >> 32), CTRL, 0xf, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// e^x by Tang's table-driven method (P. T. P. Tang, ACM Trans. Math. Softw. 15
// (1989) 144-157): x = (64 m + j) ln 2/64 + r with |r| <= ln 2/128, so that
// e^x = 2^m 2^(j/64) e^r.  r is formed against a two-part ln 2/64 (the second
// part holds the bits the first drops), e^r - 1 is its degree-5 Taylor
// polynomial (truncation below r^6/720 < 4e-17), and the 64 values 2^(j/64)
// come from a table (t64, in LDS).  Arguments below -746 are raised to -746
// (e^x is 0 in double there), and so is a NaN (the constraint solve tests q,
// e^-delta and delta~_{N-1} for finiteness itself); up to x = 2.3e7 it is
// e^x within about 2 ulp (1.3 ulp over [-700, 700] with correctly rounded table
// entries; the table's own exp2 adds at most its error), overflowing to +inf
// through the exponent m, and past that it is not finite.
__device__ __forceinline__ double exp_tab(double x, const double* t64)
{
    x = __builtin_fmax(x, -746.0);
    const double n = __builtin_rint(x * 0x1.71547652b82fep+6);  // 64/ln 2
    double r = __builtin_fma(-n, 0x1.62e42fefa39efp-7, x);       // ln 2/64, leading part
    r = __builtin_fma(-n, 0x1.abc9e3b39803fp-62, r);             // and the rest
    const int ni = (int)n;
    double e = __builtin_fma(r, 1.0 / 120.0, 1.0 / 24.0);
    e = __builtin_fma(r, e, 1.0 / 6.0);
    e = __builtin_fma(r, e, 0.5);
    e = __builtin_fma(r, e, 1.0);
    e *= r;  // e^r - 1
    const double t = t64[ni & 63];
    return __builtin_ldexp(__builtin_fma(t, e, t), ni >> 6);
}

// Double of lane `l` (wavefront-uniform) broadcast to every lane.
__device__ __forceinline__ double readlane_d(double v, int l)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Inclusive prefix sum over the 64 lanes of a wavefront: shifts by 1, 2, 4, 8
// within rows of 16 lanes, then the row totals through the row broadcasts of
// lanes 15 and 31 (gfx9 DPP row_shr / row_bcast).
__device__ __forceinline__ double wave_incl_scan(double v)
{
    v += dpp_d<0x111, 0xf>(v);  // row_shr:1
    v += dpp_d<0x112, 0xf>(v);  // row_shr:2
    v += dpp_d<0x114, 0xf>(v);  // row_shr:4
    v += dpp_d<0x118, 0xf>(v);  // row_shr:8
    v += dpp_d<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
    v += dpp_d<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
    return v;
}

// Inclusive suffix sum over the 64 lanes of a wavefront (lane l: the sum over
// lanes l..63): shifts from higher lanes by 1, 2, 4, 8 within rows of 16 lanes
// (DPP row_shl; lanes past a row's end read 0), then the totals of the rows to
// the right, the outermost first, read from each row's first lane.  Every
// partial result is a sum over a run of lanes to the right, so no total is ever
// subtracted: a suffix keeps its own precision even when the terms left of it
// are far larger (the adjoint of the constraint solve meets cotangents of order
// 1/e^-delta at the origin of strong fields).
__device__ __forceinline__ double wave_incl_suffix(double v)
{
    v += dpp_d<0x101, 0xf>(v);  // row_shl:1
    v += dpp_d<0x102, 0xf>(v);  // row_shl:2
    v += dpp_d<0x104, 0xf>(v);  // row_shl:4
    v += dpp_d<0x108, 0xf>(v);  // row_shl:8
    const int row = (threadIdx.x & 63) >> 4;
    const double t3 = readlane_d(v, 48), t2 = readlane_d(v, 32), t1 = readlane_d(v, 16);
    double right = (row < 3) ? t3 : 0.0;
    if (row < 2) right += t2;
    if (row < 1) right += t1;
    return v + right;
}

// A lane-interleaved global array of doubles, [field][P][64 W]: entry (f, k) of
// lane l at ((f P + k) 64 W + l).  Held as a uniform base and the lane's byte
// offset, the latter opaque to the compiler, so that each access is a scalar
// base plus a 32-bit vector offset formed where it is used (rather than a
// 64-bit address per entry computed once and kept, or spilled, for the whole
// kernel).  Make a fresh view per phase with lane_arr().
template <int P, int NL>
struct LaneArr {
    ADSCL_GLOBAL char* base;
    unsigned o;
    __device__ __forceinline__ ADSCL_GLOBAL double* at(int f, int k) const
    {
        return (ADSCL_GLOBAL double*)(base + (o + (unsigned)((f * P + k) * NL * 8)));
    }
    __device__ __forceinline__ double ld(int f, int k) const { return *at(f, k); }
    __device__ __forceinline__ void st(int f, int k, double v) const { *at(f, k) = v; }
};

template <int P, int NL>
__device__ __forceinline__ LaneArr<P, NL> lane_arr(ADSCL_GLOBAL double* base, int lane_id)
{
    unsigned o = (unsigned)lane_id * 8u;
    asm volatile("" : "+v"(o));
    return LaneArr<P, NL>{(ADSCL_GLOBAL char*)base, o};
}

// One step's stage record for the adjoint: for RK stage s (0..3) and point k of
// lane l, the stage input (Phi, Pi), e^-delta and S side by side, 32 bytes at
// ((s P + k) 64 W + l) 32, so that a 128-byte line holds four lanes' whole
// entries (one load brings a stage's other fields of those lanes along).  The
// same scalar base and opaque lane offset as LaneArr.
template <int P, int NL>
struct StageRec {
    ADSCL_GLOBAL char* base;
    unsigned o;
    __device__ __forceinline__ ADSCL_GLOBAL double* at(int s, int k) const
    {
        return (ADSCL_GLOBAL double*)(base + (o + (unsigned)((s * P + k) * NL * 32)));
    }
    __device__ __forceinline__ double ld(int s, int f, int k) const { return at(s, k)[f]; }
    typedef double pair_t __attribute__((ext_vector_type(2)));
    __device__ __forceinline__ void st(int s, int k, double v0, double v1, double e, double sv) const
    {
        ADSCL_GLOBAL pair_t* p = reinterpret_cast<ADSCL_GLOBAL pair_t*>(at(s, k));
        p[0] = pair_t{v0, v1};
        p[1] = pair_t{e, sv};
    }
};

template <int P, int NL>
__device__ __forceinline__ StageRec<P, NL> stage_rec(ADSCL_GLOBAL double* base, int lane_id)
{
    unsigned o = (unsigned)lane_id * 32u;
    asm volatile("" : "+v"(o));
    return StageRec<P, NL>{(ADSCL_GLOBAL char*)base, o};
}

// LDS of the row layout used by the chunked large-grid kernel.
template <int P, int W>
struct StageLayout {
    static constexpr int NL = 64 * W;      // lanes per instance
    static constexpr int RS = NL + 2;      // LDS row: column 0 = lane -1, NL+1 = lane NL
    static constexpr int SLOTS = P * RS;
    // U and F: 2 x SLOTS pairs; sigma edges: 2 NL; reductions: 4 W + 8; with
    // P >= 8, a separate region for the p edges (2 NL)
    static constexpr size_t lds_doubles = (size_t)4 * SLOTS + 2 * NL + 4 * W + 8 + (P >= 8 ? 2 * NL : 0);
};

template <int P, int W, bool FULL, bool FWD = false>
struct Stage {
    static constexpr int NL = 64 * W;
    static constexpr int RS = NL + 2;
    static constexpr int SLOTS = P * RS;
    static_assert(P >= 4, "lane 0 must own grid points 0..3");

    // Full lanes (EDGE: N - 1 = 64 W P) keep their own points in registers and take
    // their neighbours' edge values (the last / first three stage-input points,
    // p and sigma, the last / first two fluxes) across lanes with DPP wavefront
    // shifts; only lanes 0 and 63 go through small LDS slots (X*, and R* for the
    // adjoint's transposed stencils and reverse scans) to reach the adjacent
    // wavefront.  Every other case exchanges whole lane-interleaved rows.  The
    // forward edge kernel (FWD) keeps the coefficient tables in LDS (LT); the
    // adjoint reads them from global memory and keeps its own state in the LDS
    // the rows would take.
    static constexpr bool EDGE = FULL;
    static constexpr bool LT = FWD && EDGE;
    static constexpr bool ROWS = !EDGE;
    static constexpr size_t lds_doubles = (ROWS ? (size_t)4 * SLOTS + 2 * NL : 0)
                                          + (EDGE ? (size_t)44 * (W + 2) + 20 * W : 0) + (LT ? (size_t)3 * P * NL : 0)
                                          + 4 * W + 8 + 64;

    double2* U;     // (Phi_s, Pi_s) rows
    double2* F;     // (f1, g) rows; p first / last per lane between B0 and B2
    double* PE;
    double* SE;     // sigma first / last per lane
    // EDGE slots, one per wavefront (slot wv + 1) plus two ghost slots: slot 0
    // holds the parity images left of x = 0 as if a wavefront -1 had written
    // them, slot W + 1 the end point and its images past pi/2, so that every
    // wavefront reads its two neighbours' slots the same way
    double2* XU;    // [2 buffers][W+2][6] points 0..2 of lane 0, then P-1..P-3 of lane 63
    double* XP;     // [W+2][2] p of the first point of lane 0, of the last point of lane 63
    double* XS;     // [W+2][2] the same for sigma
    double2* XF;    // [2 buffers][W+2][4] fluxes of points 0, 1 of lane 0 and P-1, P-2 of lane 63;
                    // the buffer follows XU's, since with the metric frozen B3 is the only
                    // barrier of a stage and a wavefront may write its next stage's fluxes
                    // while its neighbour still reads this stage's
    double2* RU;    // EDGE, adjoint: [W][6] row cotangents (Phi_t, Pi_t) of points 0..2 of lane 0, P-1..P-3 of lane 63
    double* RF;     // EDGE, adjoint: [W][4] cotangents of the D g rows, points 0, 1 of lane 0, P-1, P-2 of lane 63
    double* RSb;    // EDGE, adjoint: [W][2] S-bar of the first point of lane 0, of the last point of lane 63
    double* RDt;    // EDGE, adjoint: [W][2] the same for the delta~ cotangents
    double* T;      // LT: the coefficient tables, [3][P][64 W] as in global memory
    double* red;    // [0,W) delta~ totals, [W,2W) S totals, [2W,3W) flags,
                    // [3W,4W) spare, 4W: p_1, 4W+1: p_{N-2}
    double* X64;    // 2^(j/64), j = 0..63, the table of exp_tab
    int tid, lane, wv, i0, col, N;
    int buf;        // XU buffer of the last publish (EDGE)
    bool has_nm2, near_end, bgauge;
    double h, dt, h24, i12h, kof, thr;
    const ADSCL_GLOBAL double* tab0;

    __device__ __forceinline__ void setup(double* lds, const InstConst& ic, const double* tab, int gauge,
                                          double a_collapse)
    {
        setup(lds, ic, tab, gauge, a_collapse, (int)threadIdx.x);
    }

    // t: the thread's index within the 64 W threads that run the instance (the
    // workgroup's own index unless the workgroup runs several instances).
    __device__ __forceinline__ void setup(double* lds, const InstConst& ic, const double* tab, int gauge,
                                          double a_collapse, int t)
    {
        double* p = lds;
        U = F = XU = XF = RU = nullptr;
        PE = SE = XP = XS = T = RF = RSb = RDt = nullptr;
        if (ROWS) {
            U = reinterpret_cast<double2*>(p);
            F = U + SLOTS;
            // F is free from B0 (its last readers finished the previous stage)
            // until the flux writes after B2 (the edge path keeps its p edges in
            // XP; the adjoint's reverse writes PE only after a barrier that
            // follows its last reads of F)
            PE = reinterpret_cast<double*>(F);
            SE = reinterpret_cast<double*>(F + SLOTS);
            p = SE + 2 * NL;
        }
        if (EDGE) {
            XU = reinterpret_cast<double2*>(p);
            p += 24 * (W + 2);
            XP = p;
            p += 2 * (W + 2);
            XS = p;
            p += 2 * (W + 2);
            XF = reinterpret_cast<double2*>(p);
            p += 16 * (W + 2);
            RU = reinterpret_cast<double2*>(p);
            p += 12 * W;
            RF = p;
            p += 4 * W;
            RSb = p;
            p += 2 * W;
            RDt = p;
            p += 2 * W;
        }
        if (LT) {
            T = p;
            p += 3 * P * NL;
        }
        red = p;
        X64 = red + 4 * W + 8;
        buf = 0;
        tid = t;
        // read only after the barrier of the first constraint solve
        if (tid < 64) X64[tid] = exp2((double)tid * (1.0 / 64.0));
        lane = tid & 63;
        wv = tid >> 6;
        N = ic.N;
        h = ic.h;
        dt = ic.dt;
        h24 = ic.h24;
        i12h = ic.i12h;
        kof = ic.kof;
        thr = a_collapse;
        bgauge = gauge == 0;
        i0 = tid * P;
        col = tid + 1;
        // FULL: N - 1 == 64 W P, so every lane owns P evolved points and the
        // last lane owns N-4..N-2; otherwise lanes past N-2 idle and the end moves.
        has_nm2 = FULL ? (tid == NL - 1) : ((i0 <= N - 2) && (N - 2 < i0 + P));
        near_end = FULL ? (tid == NL - 1) : ((i0 + P + 2 >= N - 4) && (i0 <= N - 2));
        tab0 = gmem(tab);
        if constexpr (LT) {
            // each lane copies exactly the entries it reads later, so no barrier
#pragma unroll
            for (int t = 0; t < 3 * P; ++t) T[t * NL + tid] = tab0[t * NL + tid];
        }
    }

    // Value of v at the lane to the left (tid - 1) / right (tid + 1) within the
    // wavefront (DPP wave_shr:1 / wave_shl:1); lanes 0 / 63 get 0.  All lanes
    // must be active.
    static __device__ __forceinline__ double from_left(double v) { return dpp_d<0x138, 0xf>(v); }
    static __device__ __forceinline__ double from_right(double v) { return dpp_d<0x130, 0xf>(v); }

    __device__ __forceinline__ bool own(int k) const { return FULL || (i0 + k <= N - 2); }

    // LDS index of point j, -P <= j < 64 W P + P
    __device__ __forceinline__ int slot(int j) const
    {
        const int l = (j >= 0) ? (j / P) : -1 - ((-1 - j) / P);
        return (j - l * P) * RS + l + 1;
    }

    // Per-stage view of the coefficient tables: a uniform base and the lane's
    // byte offset, opaque to the compiler so that table loads are issued again
    // in each stage (L2 hits) instead of being held in registers across the
    // time loop, and take the scalar-base plus 32-bit vector-offset form.
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

    // Table t (0 sin x cos x, 1 tan^2 x, 2 cot^2 x) at the lane's point k.
    __device__ __forceinline__ double tab(const TabView& v, int t, int k) const
    {
        if constexpr (LT) return T[(t * P + k) * NL + tid];
        return *(const ADSCL_GLOBAL double*)(v.base + (v.o + (unsigned)((t * P + k) * NL * 8)));
    }

    // Publish (v0, v1) = (Phi, Pi) of the own points with parity ghosts:
    // Phi odd / Pi even about x = 0, Phi even / Pi odd about pi/2, Phi = Pi = 0 at pi/2.
    __device__ __forceinline__ void publish(const double* v0, const double* v1)
    {
        if constexpr (EDGE) {
            // neighbours within the wavefront read the registers; lanes 0 and 63
            // leave their edge points for the adjacent wavefronts
            buf ^= 1;
            double2* xu = XU + (buf * (W + 2) + wv + 1) * 6;
            if (lane == 0) {
#pragma unroll
                for (int r = 0; r < 3; ++r) xu[r] = make_double2(v0[r], v1[r]);
            }
            if (lane == 63) {
#pragma unroll
                for (int r = 0; r < 3; ++r) xu[3 + r] = make_double2(v0[P - 1 - r], v1[P - 1 - r]);
            }
            if (tid == 0) {  // Phi odd, Pi even about x = 0: points -1, -2, -3
                double2* g = XU + buf * (W + 2) * 6;
#pragma unroll
                for (int r = 0; r < 3; ++r) g[3 + r] = make_double2(-v0[1 + r], v1[1 + r]);
            }
            if (tid == NL - 1) {  // Phi = Pi = 0 at pi/2; Phi even, Pi odd about it: points N-1, N, N+1
                double2* g = XU + (buf * (W + 2) + W + 1) * 6;
                g[0] = make_double2(0.0, 0.0);
                g[1] = make_double2(v0[P - 1], -v1[P - 1]);
                g[2] = make_double2(v0[P - 2], -v1[P - 2]);
            }
            return;
        }
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
    }

    // Sums of the wavefront totals r[0..W): over the wavefronts before this one
    // (`before`) and over all (`all`).  Lanes v < W hold r[v], a DPP prefix
    // runs over them (W <= 16: within the first row of 16 lanes), and two
    // wavefront-uniform lane reads broadcast the results, instead of every lane
    // adding all W totals under a mask.
    __device__ __forceinline__ void wave_totals(const double* r, double& before, double& all) const
    {
        double x = (lane < W) ? r[lane < W ? lane : 0] : 0.0;
        if constexpr (W > 1) x += dpp_d<0x111, 0xf>(x);  // row_shr:1
        if constexpr (W > 2) x += dpp_d<0x112, 0xf>(x);  // row_shr:2
        if constexpr (W > 4) x += dpp_d<0x114, 0xf>(x);  // row_shr:4
        if constexpr (W > 8) x += dpp_d<0x118, 0xf>(x);  // row_shr:8
        all = readlane_d(x, W - 1);
        const int w = __builtin_amdgcn_readfirstlane(wv);
        before = (w > 0) ? readlane_d(x, w > 0 ? w - 1 : 0) : 0.0;
    }

    // Constraint solve of the published state given q = Phi^2 + Pi^2 of the own
    // points (Eqs. (5)-(6)): delta (gauge applied), e^{-delta} and S at own
    // points, the delta~ end value dN and the S total tot2.  Contains barriers
    // B1 and B2.
    __device__ __forceinline__ void constraints(const double* q, double* dl, double* E, double* S, double& dN,
                                                double& tot2)
    {
        const auto tb = tables();
        double p[P];
        double ptot = 0.0;
#pragma unroll
        for (int k = 0; k < P; ++k) {
            p[k] = tab(tb, 0, k) * q[k];  // table is 0 off 1..N-2
            ptot += p[k];
        }
        const double incl = wave_incl_scan(ptot);
        if (lane == 63) red[wv] = incl;
        if constexpr (EDGE) {
            if (lane == 0) XP[2 * (wv + 1)] = p[0];
            if (lane == 63) XP[2 * (wv + 1) + 1] = p[P - 1];
            if (tid == 0) XP[1] = -p[1];                // p_{-1} = -p_1
            if (tid == NL - 1) XP[2 * (W + 1)] = 0.0;  // p_{N-1} = 0
        } else {
            PE[tid] = p[0];
            PE[NL + tid] = p[P - 1];
        }
        if (tid == 0) red[4 * W] = p[1];
        if (FULL) {
            if (tid == NL - 1) red[4 * W + 1] = p[P - 1];
        } else if (has_nm2) {
#pragma unroll
            for (int k = 0; k < P; ++k)
                if (i0 + k == N - 2) red[4 * W + 1] = p[k];
        }
        __syncthreads();  // B1
        double carry, tot;
        wave_totals(red, carry, tot);
        carry += incl - ptot;
        const double p1 = red[4 * W], pN2 = red[4 * W + 1];
        double pl, pr;
        if constexpr (EDGE) {
            // lanes 0 / 63 take the neighbouring wavefront's (or the ghost) slot
            pl = dpp_old<0x138>(XP[2 * wv + 1], p[P - 1]);
            pr = dpp_old<0x130>(XP[2 * (wv + 2)], p[0]);
        } else {
            pl = (tid > 0) ? PE[NL + tid - 1] : -p1;  // p_{-1} = -p_1
            pr = (tid < NL - 1) ? PE[tid + 1] : 0.0;  // p_{N-1} = 0
        }
        dN = -h24 * (24.0 * tot + 2.0 * pN2 + 2.0 * p1);        // delta~_{N-1}
        const double shift = bgauge ? dN : 0.0;
        // -delta = h24 (24 R - 12 p + p_m - p_p + 2 p_1) + shift, with h24
        // distributed over the terms: one add and three FMAs per point
        const double a24 = 24.0 * h24, a12 = -12.0 * h24, c0 = fma(2.0 * h24, p1, shift);

        double sg[P];
        double R = carry, stot = 0.0;
#pragma unroll
        for (int k = 0; k < P; ++k) {
            R += p[k];
            const double pm = (k == 0) ? pl : p[k - 1];
            const double pp = (k == P - 1) ? pr : p[k + 1];
            const double nd = fma(a24, R, fma(a12, p[k], fma(h24, pm - pp, c0)));
            dl[k] = -nd;
            E[k] = exp_tab(nd, X64);
            sg[k] = tab(tb, 1, k) * q[k] * E[k];  // table is 0 off 1..N-2
            stot += sg[k];
        }
        const double incl2 = wave_incl_scan(stot);
        if (lane == 63) red[W + wv] = incl2;
        if constexpr (EDGE) {
            if (lane == 0) XS[2 * (wv + 1)] = sg[0];
            if (lane == 63) XS[2 * (wv + 1) + 1] = sg[P - 1];
            if (tid == 0) XS[1] = sg[1];                // sigma_{-1} = sigma_1
            if (tid == NL - 1) XS[2 * (W + 1)] = 0.0;  // sigma_{N-1} = 0
        } else {
            SE[tid] = sg[0];
            SE[NL + tid] = sg[P - 1];
        }
        __syncthreads();  // B2
        double carry2;
        wave_totals(red + W, carry2, tot2);
        carry2 += incl2 - stot;
        double sl, sr;
        if constexpr (EDGE) {
            sl = dpp_old<0x138>(XS[2 * wv + 1], sg[P - 1]);
            sr = dpp_old<0x130>(XS[2 * (wv + 2)], sg[0]);
        } else {
            sl = (tid > 0) ? SE[NL + tid - 1] : sg[1];  // sigma_{-1} = sigma_1
            sr = (tid < NL - 1) ? SE[tid + 1] : 0.0;    // sigma_{N-1} = 0
        }
        double R2 = carry2;
#pragma unroll
        for (int k = 0; k < P; ++k) {
            R2 += sg[k];
            const double sm = (k == 0) ? sl : sg[k - 1];
            const double sp = (k == P - 1) ? sr : sg[k + 1];
            // h24 (24 R2 - 12 sigma + sigma_m - sigma_p), h24 distributed
            S[k] = fma(a24, R2, fma(a12, sg[k], h24 * (sm - sp)));
        }
    }

    // The first prefix sum of the constraint solve alone (Eq. (6)): delta (gauge
    // applied) and e^{-delta} at own points and the delta~ end value dN, for
    // stages whose A is evolved with Eq. (4) instead of solved from Eq. (5).
    // Contains barrier B1.
    __device__ __forceinline__ void delta_scan(const double* q, double* dl, double* E, double& dN)
    {
        const auto tb = tables();
        double p[P];
        double ptot = 0.0;
#pragma unroll
        for (int k = 0; k < P; ++k) {
            p[k] = tab(tb, 0, k) * q[k];  // table is 0 off 1..N-2
            ptot += p[k];
        }
        const double incl = wave_incl_scan(ptot);
        if (lane == 63) red[wv] = incl;
        if constexpr (EDGE) {
            if (lane == 0) XP[2 * (wv + 1)] = p[0];
            if (lane == 63) XP[2 * (wv + 1) + 1] = p[P - 1];
            if (tid == 0) XP[1] = -p[1];                // p_{-1} = -p_1
            if (tid == NL - 1) XP[2 * (W + 1)] = 0.0;  // p_{N-1} = 0
        } else {
            PE[tid] = p[0];
            PE[NL + tid] = p[P - 1];
        }
        if (tid == 0) red[4 * W] = p[1];
        if (FULL) {
            if (tid == NL - 1) red[4 * W + 1] = p[P - 1];
        } else if (has_nm2) {
#pragma unroll
            for (int k = 0; k < P; ++k)
                if (i0 + k == N - 2) red[4 * W + 1] = p[k];
        }
        __syncthreads();  // B1
        double carry, tot;
        wave_totals(red, carry, tot);
        carry += incl - ptot;
        const double p1 = red[4 * W], pN2 = red[4 * W + 1];
        double pl, pr;
        if constexpr (EDGE) {
            pl = dpp_old<0x138>(XP[2 * wv + 1], p[P - 1]);
            pr = dpp_old<0x130>(XP[2 * (wv + 2)], p[0]);
        } else {
            pl = (tid > 0) ? PE[NL + tid - 1] : -p1;
            pr = (tid < NL - 1) ? PE[tid + 1] : 0.0;
        }
        dN = -h24 * (24.0 * tot + 2.0 * pN2 + 2.0 * p1);
        const double shift = bgauge ? dN : 0.0;
        const double a24 = 24.0 * h24, a12 = -12.0 * h24, c0 = fma(2.0 * h24, p1, shift);
        double R = carry;
#pragma unroll
        for (int k = 0; k < P; ++k) {
            R += p[k];
            const double pm = (k == 0) ? pl : p[k - 1];
            const double pp = (k == P - 1) ? pr : p[k + 1];
            const double nd = fma(a24, R, fma(a12, p[k], fma(h24, pm - pp, c0)));  // -delta, as in constraints
            dl[k] = -nd;
            E[k] = exp_tab(nd, X64);
        }
    }

    // Right-hand sides of Eqs. (2)-(3) at the published stage input: barrier B0,
    // Kreiss-Oliger terms and q from the +-3 window, the constraint solve (B1,
    // B2), the fluxes f1 = A e^-delta Pi, g = tan^2 x A e^-delta Phi with parity
    // ghosts (B3), the centred D stencil.  With `check`, the division-free test
    // e^-delta - cos^3 x/sin x S < thr e^-delta (A < thr) and a finiteness test
    // run before B3 and the function returns their workgroup-wide bits
    // (1 collapsed, 2 non-finite) without computing r when any is set.
    // r0, r1: Phi_t, Pi_t of the own points (0 at pinned points).  KEEP: also
    // stores the stage input (v0, v1), e^-delta and S of the lane's points as
    // stage ks of the stage record ES (StageRec).
    // v0, v1: the published stage input of the own points (read on the edge
    // path, where it is not in LDS).
    // EVA (A evolved by Eq. (4), the paper's alternative to solving Eq. (5) at
    // every stage): the stage's A of the own points is `av`; only the first
    // prefix sum runs (delta from Eq. (6)), the fluxes take w = av e^-delta, the
    // collapse test is av < thr; with `reint` the full solve runs instead and
    // its A, 1 - cos^3 x/sin x S/e^-delta, replaces `av` (re-integration from
    // Eq. (5)).  `wout` receives w = A e^-delta of the own points.
    template <bool KEEP = false, bool EVA = false>
    __device__ __forceinline__ int rhs(bool check, bool frozen, const double* v0, const double* v1, double* r0,
                                       double* r1, ADSCL_GLOBAL double* ES = nullptr, int ks = 0,
                                       double* av = nullptr, double* wout = nullptr, bool reint = false)
    {
        if constexpr (EDGE) return rhs_edge<KEEP, EVA>(check, frozen, v0, v1, r0, r1, ES, ks, av, wout, reint);
        __syncthreads();  // B0
        const auto tb = tables();
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
            if (EVA && !reint) {
                delta_scan(q, dl, E, dN);
#pragma unroll
                for (int k = 0; k < P; ++k) S[k] = 0.0;
            } else {
                constraints(q, dl, E, S, dN, tot2);
            }
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
                const double g = tab(tb, 1, k) * f2;
                if (k == 1) { f2_1 = f2; f1a[1] = f1; ga[1] = g; }
                if (k == 2) { f2_2 = f2; f1a[2] = f1; ga[2] = g; }
                if (k >= P - 3) { fl[P - 1 - k] = f1; gl[P - 1 - k] = g; }
                if (check) {
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
        if (check) {
            if (1.0 < thr) cl = 1;
            if (!isfinite(dN) || !isfinite(chk)) cl |= 2;
            const int wcol = __any(cl & 1) ? 1 : 0;
            const int wnf = __any(cl & 2) ? 2 : 0;
            if (lane == 0) red[2 * W + wv] = (double)(wcol | wnf);
        }
        if constexpr (KEEP) {
            // after the flux loop, so that its table loads do not wait for
            // these stores (vector loads and stores retire in issue order)
            const auto es = stage_rec<P, NL>(ES, tid);
#pragma unroll
            for (int k = 0; k < P; ++k) es.st(ks, k, v0[k], v1[k], E[k], S[k]);
        }
        __syncthreads();  // B3
        if (check) {
            int fl_ = 0;
#pragma unroll
            for (int v = 0; v < W; ++v) fl_ |= (int)red[2 * W + v];
            if (fl_) return fl_;
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
#pragma unroll
        for (int k = 0; k < P; ++k) {
            // interior formula everywhere (cot^2 x is 0 at x = 0 in the table);
            // the origin row and points past N-2 are fixed up below
            const double Df1 = (fw[k].x - 8.0 * fw[k + 1].x + 8.0 * fw[k + 3].x - fw[k + 4].x) * i12h;
            const double Dg = (fw[k].y - 8.0 * fw[k + 1].y + 8.0 * fw[k + 3].y - fw[k + 4].y) * i12h;
            r0[k] = Df1 + ko0[k];
            r1[k] = tab(tb, 2, k) * Dg + ko1[k];
            if (k == 0 && tid == 0) {
                // Phi_0 = 0; lim tan^-2 (tan^2 f2)' = 3 f2'(0) with f2 odd about x = 0
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

    // rhs on the edge path.  No barrier before the scans: the stage input is in
    // registers and its edges were published before the first scan barrier.
    // The stage-input and flux slots (XU, XF) are double-buffered by stage, so
    // their last readers (after B3) never meet the next stage's writers even
    // with the metric frozen, when B3 is a stage's only barrier; the scan slots
    // (XP, XS) are written before B1 / B2 and read after them, with B3 between
    // a stage's reads and the next stage's writes.
    // Barriers one call of rhs_edge passes (EVA off): B1, B2 and B3, or B3
    // alone with the metric frozen.
    static __device__ __forceinline__ int edge_barriers(bool frozen) { return frozen ? 1 : 3; }

    template <bool KEEP, bool EVA>
    __device__ __forceinline__ int rhs_edge(bool check, bool frozen, const double* v0, const double* v1, double* r0,
                                            double* r1, ADSCL_GLOBAL double* ES, int ks, double* av, double* wout,
                                            bool reint)
    {
        const auto tb = tables();
        double q[P];
#pragma unroll
        for (int k = 0; k < P; ++k) q[k] = v0[k] * v0[k] + v1[k] * v1[k];
        double dl[P], E[P], S[P];
        double dN = 0.0, tot2 = 0.0;
        if (!frozen) {
            if (EVA && !reint) {
                delta_scan(q, dl, E, dN);
#pragma unroll
                for (int k = 0; k < P; ++k) S[k] = 0.0;
            } else {
                constraints(q, dl, E, S, dN, tot2);
            }
        } else {
#pragma unroll
            for (int k = 0; k < P; ++k) { dl[k] = 0.0; E[k] = 1.0; S[k] = 0.0; }
        }
        double ff[P], fg[P], chk = 0.0, f2_1 = 0.0, f2_2 = 0.0;
        int cl = 0;
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const double c3s = tab(tb, 2, k) * tab(tb, 0, k);
            double wk;
            if constexpr (EVA) {
                if (reint) av[k] = 1.0 - c3s * (S[k] / E[k]);
                wk = av[k] * E[k];
                wout[k] = wk;
            } else {
                wk = E[k] - c3s * S[k];
            }
            const double f2 = wk * v0[k];
            ff[k] = wk * v1[k];
            fg[k] = tab(tb, 1, k) * f2;
            if (k == 1) f2_1 = f2;
            if (k == 2) f2_2 = f2;
            if (check) {
                if (wk < thr * E[k]) cl = 1;
                chk = fma(q[k], 0.0, chk);
                chk = fma(wk, 0.0, chk);
                chk = fma(E[k], 0.0, chk);
            }
        }
        double2* const XFb = XF + buf * (W + 2) * 4;  // this stage's flux slots
        {
            double2* xf = XFb + (wv + 1) * 4;
            if (lane == 0) {
                xf[0] = make_double2(ff[0], fg[0]);
                xf[1] = make_double2(ff[1], fg[1]);
            }
            if (lane == 63) {
                xf[2] = make_double2(ff[P - 1], fg[P - 1]);
                xf[3] = make_double2(ff[P - 2], fg[P - 2]);
            }
            if (tid == 0) {  // f1 even, g odd about x = 0: points -1, -2
                XFb[2] = make_double2(ff[1], -fg[1]);
                XFb[3] = make_double2(ff[2], -fg[2]);
            }
            if (tid == NL - 1) {
                // f1_{N-1} = 0, g_{N-1} the even 6th-order extrapolation; ghost N
                XFb[(W + 1) * 4] = make_double2(0.0, (15.0 * fg[P - 1] - 6.0 * fg[P - 2] + fg[P - 3]) / 10.0);
                XFb[(W + 1) * 4 + 1] = make_double2(-ff[P - 1], fg[P - 1]);
            }
        }
        if (check) {
            if (1.0 < thr) cl = 1;
            if (!isfinite(dN) || !isfinite(chk)) cl |= 2;
            const int wcol = __any(cl & 1) ? 1 : 0;
            const int wnf = __any(cl & 2) ? 2 : 0;
            if (lane == 0) red[2 * W + wv] = (double)(wcol | wnf);
        }
        if constexpr (KEEP) {
            // after the flux loop, so that its table loads do not wait for
            // these stores (vector loads and stores retire in issue order)
            const auto es = stage_rec<P, NL>(ES, tid);
#pragma unroll
            for (int k = 0; k < P; ++k) es.st(ks, k, v0[k], v1[k], E[k], S[k]);
        }
        __syncthreads();  // B3
        if (check) {
            int fl_ = 0;
#pragma unroll
            for (int v = 0; v < W; ++v) fl_ |= (int)red[2 * W + v];
            if (fl_) return fl_;
        }
        double ko0[P], ko1[P];
        {
            double2 w[P + 6];  // points i0-3 .. i0+P+2
            {
                // lanes 0 / 63 take the neighbouring wavefront's (or the ghost) slot
                const double2* xl = XU + (buf * (W + 2) + wv) * 6;
                const double2* xr = XU + (buf * (W + 2) + wv + 2) * 6;
#pragma unroll
                for (int r = 0; r < 3; ++r) {
                    const double2 gl = xl[5 - r], gr = xr[r];
                    w[r] = make_double2(dpp_old<0x138>(gl.x, v0[P - 3 + r]), dpp_old<0x138>(gl.y, v1[P - 3 + r]));
                    w[P + 3 + r] = make_double2(dpp_old<0x130>(gr.x, v0[r]), dpp_old<0x130>(gr.y, v1[r]));
                }
            }
#pragma unroll
            for (int k = 0; k < P; ++k) w[3 + k] = make_double2(v0[k], v1[k]);
#pragma unroll
            for (int k = 0; k < P; ++k) {
                ko0[k] = kof * (w[k].x - 6.0 * w[k + 1].x + 15.0 * w[k + 2].x - 20.0 * w[k + 3].x
                                + 15.0 * w[k + 4].x - 6.0 * w[k + 5].x + w[k + 6].x);
                ko1[k] = kof * (w[k].y - 6.0 * w[k + 1].y + 15.0 * w[k + 2].y - 20.0 * w[k + 3].y
                                + 15.0 * w[k + 4].y - 6.0 * w[k + 5].y + w[k + 6].y);
            }
        }
        double2 fw[P + 4];  // points i0-2 .. i0+P+1
        {
            const double2* xl = XFb + wv * 4;
            const double2* xr = XFb + (wv + 2) * 4;
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                const double2 gl = xl[3 - r], gr = xr[r];
                fw[r] = make_double2(dpp_old<0x138>(gl.x, ff[P - 2 + r]), dpp_old<0x138>(gl.y, fg[P - 2 + r]));
                fw[P + 2 + r] = make_double2(dpp_old<0x130>(gr.x, ff[r]), dpp_old<0x130>(gr.y, fg[r]));
            }
        }
#pragma unroll
        for (int k = 0; k < P; ++k) fw[2 + k] = make_double2(ff[k], fg[k]);
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const double Df1 = (fw[k].x - 8.0 * fw[k + 1].x + 8.0 * fw[k + 3].x - fw[k + 4].x) * i12h;
            const double Dg = (fw[k].y - 8.0 * fw[k + 1].y + 8.0 * fw[k + 3].y - fw[k + 4].y) * i12h;
            r0[k] = Df1 + ko0[k];
            r1[k] = tab(tb, 2, k) * Dg + ko1[k];
        }
        if (tid == 0) {
            // Phi_0 = 0; lim tan^-2 (tan^2 f2)' = 3 f2'(0) with f2 odd about x = 0
            r0[0] = 0.0;
            r1[0] = 3.0 * ((16.0 * f2_1 - 2.0 * f2_2) * i12h) + ko1[0];
        }
        return 0;
    }
};

}  // namespace adscl
