// Fused RK4 evolution of the AdS4 Einstein-Klein-Gordon system for a batch of
// instances (Liebling & Khanna, arXiv:1706.07413, Sec. II), gfx950.
//
// One workgroup owns one instance for the whole call and keeps its state on
// chip: lane l owns the P consecutive grid points l*P .. l*P+P-1 and holds U^n,
// the RK4 accumulator and the Kreiss-Oliger terms of its points in registers.
// On grids that fill every lane (N - 1 = 64 W P) the stage input stays in
// registers too and neighbours' values cross lanes by DPP, with small LDS
// slots between wavefronts (no B0 below); otherwise the stage input and the
// fluxes are exchanged through lane-interleaved LDS rows.  A stage is
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
// The stage machinery (LDS layout, parity ghosts, the two scans, fluxes)
// lives in stage.h, shared with the adjoint kernel's forward recomputation.
#include <algorithm>

#include "stage.h"

namespace adscl {
namespace {

// KEEP: also writes the stage record of every step (EvolveArgs::keep).
template <int P, int W, bool FULL, bool KEEP>
__global__ void __launch_bounds__(64 * W) evolve_kernel(EvolveArgs a)
{
    extern __shared__ double lds[];
    const int b = a.order[blockIdx.x];
    const InstStatus st0 = a.status[b];
    if (st0.state == ST_COLLAPSED || st0.state == ST_NONFINITE) return;

    const InstConst ic = a.ic[b];
    const int64_t off = ic.off;
    const bool frozen = a.frozen != 0;
    Stage<P, W, FULL, true> sg;
    sg.setup(lds, ic, a.tab[b], a.gauge, a.a_collapse);
    const int N = sg.N, i0 = sg.i0;
    const double dt = sg.dt;

    double un0[P], un1[P], acc0[P], acc1[P], cv0[P], cv1[P];  // cv: the current stage input
    const ADSCL_GLOBAL double* s0 = gmem(a.Phi + off);
    const ADSCL_GLOBAL double* s1 = gmem(a.Pi + off);
    if (a.src) {
        s0 = gmem(a.src[b]) + (size_t)(st0.steps / a.src_every) * 2 * (size_t)N;
        s1 = s0 + N;
    }
#pragma unroll
    for (int k = 0; k < P; ++k) {
        const int j = i0 + k;
        const bool o = sg.own(k);
        un0[k] = o ? s0[j] : 0.0;
        un1[k] = o ? s1[j] : 0.0;
        acc0[k] = 0.0;
        acc1[k] = 0.0;
        cv0[k] = un0[k];
        cv1[k] = un1[k];
    }

    // One RK4 stage on the published stage input; returns true when stage 0
    // finds the instance collapsed or non-finite (nothing is updated then).
    int stop_bits = 0;
    constexpr size_t kRec = (size_t)16 * P * 64 * W;  // doubles of one step's stage record
    ADSCL_GLOBAL double* const kp = KEEP ? gmem(a.keep[b]) : nullptr;
    ADSCL_GLOBAL double* krec = nullptr;  // the current step's record
    auto stage = [&](const int s) -> bool {
        double r0[P], r1[P];
        const int bits = sg.template rhs<KEEP>(s == 0, frozen, cv0, cv1, r0, r1, krec, s);
        if (bits) {
            stop_bits = bits;
            return true;
        }
        const double c_next = (s == 2) ? dt : 0.5 * dt;
        const double wacc = (s == 0 || s == 3) ? 1.0 : 2.0;
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
                cv0[k] = un0[k] + c_next * r0[k];
                cv1[k] = un1[k] + c_next * r1[k];
            } else {
                un0[k] = un0[k] + (dt / 6.0) * acc0[k];
                un1[k] = un1[k] + (dt / 6.0) * acc1[k];
                cv0[k] = un0[k];
                cv1[k] = un1[k];
            }
        }
        // every lane read U_s before B3, so U_{s+1} may replace it now
        sg.publish(cv0, cv1);
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
    // checkpoints of the segment: U^n for n - n_start a multiple of ckpt_every
    ADSCL_GLOBAL double* const ck = (a.ckpt && a.ckpt_every > 0) ? gmem(a.ckpt[b]) : nullptr;
    auto store_ckpt = [&]() {
        const int64_t r = n - st0.steps;
        if (ck && r % a.ckpt_every == 0) {
            ADSCL_GLOBAL double* d = ck + (size_t)(r / a.ckpt_every) * 2 * (size_t)N;
#pragma unroll
            for (int k = 0; k < P; ++k) {
                if (sg.own(k)) {
                    d[i0 + k] = un0[k];
                    d[N + i0 + k] = un1[k];
                }
            }
            if (sg.has_nm2) {
                d[N - 1] = 0.0;
                d[2 * N - 1] = 0.0;
            }
        }
    };
    sg.publish(un0, un1);
    while (n < seg_end) {
        store_ckpt();
        if (KEEP) krec = kp + (size_t)(n - st0.steps) * kRec;
        if (stage(0)) break;
#pragma unroll 1
        for (int s = 1; s < 4; ++s) stage(s);
        ++n;
    }
    if (n == seg_end) store_ckpt();
#pragma unroll
    for (int k = 0; k < P; ++k) {
        if (sg.own(k)) {
            a.Phi[off + i0 + k] = un0[k];
            a.Pi[off + i0 + k] = un1[k];
        }
    }
    if (threadIdx.x == 0) {
        InstStatus o = st0;
        o.steps = n;
        if (stop_bits) {
            o.state = (stop_bits & 2) ? ST_NONFINITE : ST_COLLAPSED;
            o.t_c = (double)n * dt;
        }
        a.status[b] = o;
    }
}

template <int P, int W, bool FULL>
constexpr size_t lds_bytes_for()
{
    return Stage<P, W, FULL, true>::lds_doubles * sizeof(double);
}

template <int P, int W>
hipError_t launch_t(bool full, int n_blocks, const EvolveArgs& a, hipStream_t s)
{
    const dim3 g(n_blocks), t(64 * W);
    if (a.keep) {
        if (full) evolve_kernel<P, W, true, true><<<g, t, lds_bytes_for<P, W, true>(), s>>>(a);
        else evolve_kernel<P, W, false, true><<<g, t, lds_bytes_for<P, W, false>(), s>>>(a);
    } else {
        if (full) evolve_kernel<P, W, true, false><<<g, t, lds_bytes_for<P, W, true>(), s>>>(a);
        else evolve_kernel<P, W, false, false><<<g, t, lds_bytes_for<P, W, false>(), s>>>(a);
    }
    return hipGetLastError();
}

template <int P, int W>
hipError_t prepare_t(size_t max_lds)
{
    const size_t nf = lds_bytes_for<P, W, true>(), np = lds_bytes_for<P, W, false>();
    if (nf > max_lds || np > max_lds) return hipErrorInvalidValue;
    const void* kf[] = {(const void*)evolve_kernel<P, W, true, false>, (const void*)evolve_kernel<P, W, true, true>};
    const void* kn[] = {(const void*)evolve_kernel<P, W, false, false>, (const void*)evolve_kernel<P, W, false, true>};
    for (int i = 0; i < 2; ++i) {
        hipError_t e = hipFuncSetAttribute(kf[i], hipFuncAttributeMaxDynamicSharedMemorySize, (int)nf);
        if (e != hipSuccess) return e;
        e = hipFuncSetAttribute(kn[i], hipFuncAttributeMaxDynamicSharedMemorySize, (int)np);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
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
#define X(p, w) \
    if (c.P == p && c.W == w) return std::max(lds_bytes_for<p, w, true>(), lds_bytes_for<p, w, false>());
    ADSCL_CLASSES(X)
#undef X
    return 0;
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
