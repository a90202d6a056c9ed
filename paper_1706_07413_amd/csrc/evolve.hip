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
// evolve_pair_kernel (opt-in) runs the instances of a (P, W/2) class two per
// workgroup inside a (P, W) class's launch.
#include <algorithm>

#include "stage.h"

namespace adscl {
namespace {

// The evolution of one instance by W wavefronts: its state in registers, its
// Stage over the LDS at `lds`, t the thread's index within the instance.
// KEEP: also writes the stage record of every step (EvolveArgs::keep).
template <int P, int W, bool FULL, bool KEEP>
struct Run {
    static constexpr size_t kRec = (size_t)16 * P * 64 * W;  // doubles of one step's stage record
    Stage<P, W, FULL, true> sg;
    double un0[P], un1[P], acc0[P], acc1[P], cv0[P], cv1[P];  // cv: the current stage input
    InstStatus st0;
    int64_t off, n, seg_end;
    double dt;
    int stop_bits;
    bool frozen;
    ADSCL_GLOBAL double* ck;    // checkpoints of the segment, or null
    ADSCL_GLOBAL double* kp;    // KEEP: the segment's stage records
    ADSCL_GLOBAL double* krec;  // KEEP: the current step's record

    // Loads instance b; false when it has already stopped (nothing to run).
    __device__ __forceinline__ bool init(const EvolveArgs& a, int b, double* lds, int t)
    {
        st0 = a.status[b];
        if (st0.state == ST_COLLAPSED || st0.state == ST_NONFINITE) return false;
        const InstConst ic = a.ic[b];
        off = ic.off;
        frozen = a.frozen != 0;
        sg.setup(lds, ic, a.tab[b], a.gauge, a.a_collapse, t);
        const int N = sg.N, i0 = sg.i0;
        dt = sg.dt;
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
        stop_bits = 0;
        kp = KEEP ? gmem(a.keep[b]) : nullptr;
        krec = nullptr;
        // Advance to the end of this segment: the call's target step, or the
        // next snapshot step when snapshots are on.
        n = st0.steps;
        seg_end = st0.target;
        if (a.snap_every > 0) {
            const int64_t nb = (n / a.snap_every + 1) * a.snap_every;
            if (nb < seg_end) seg_end = nb;
        }
        // checkpoints of the segment: U^n for n - n_start a multiple of ckpt_every
        ck = (a.ckpt && a.ckpt_every > 0) ? gmem(a.ckpt[b]) : nullptr;
        return true;
    }

    // One RK4 stage on the published stage input; returns true when stage 0
    // finds the instance collapsed or non-finite (nothing is updated then).
    __device__ __forceinline__ bool stage(const int s)
    {
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
    }

    // Start of step n: the checkpoint due at n, the step's stage record.
    __device__ __forceinline__ void begin_step(const EvolveArgs& a)
    {
        const int64_t r = n - st0.steps;
        if (ck && r % a.ckpt_every == 0) {
            const int N = sg.N, i0 = sg.i0;
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
        if (KEEP) krec = kp + (size_t)(n - st0.steps) * kRec;
    }

    // End of the segment: the last checkpoint, the state and the status (thread
    // t == 0 writes the status).
    __device__ __forceinline__ void finish(const EvolveArgs& a, int b, int t)
    {
        if (n == seg_end && ck) begin_step(a);
        const int i0 = sg.i0;
#pragma unroll
        for (int k = 0; k < P; ++k) {
            if (sg.own(k)) {
                a.Phi[off + i0 + k] = un0[k];
                a.Pi[off + i0 + k] = un1[k];
            }
        }
        if (t == 0) {
            InstStatus o = st0;
            o.steps = n;
            if (stop_bits) {
                o.state = (stop_bits & 2) ? ST_NONFINITE : ST_COLLAPSED;
                o.t_c = (double)n * dt;
            }
            a.status[b] = o;
        }
    }
};

template <int P, int W, bool FULL, bool KEEP>
__device__ __forceinline__ void evolve_one(const EvolveArgs& a, int b, double* lds)
{
    Run<P, W, FULL, KEEP> r;
    if (!r.init(a, b, lds, threadIdx.x)) return;
    r.sg.publish(r.un0, r.un1);
    while (r.n < r.seg_end) {
        r.begin_step(a);
        if (r.stage(0)) break;
#pragma unroll 1
        for (int s = 1; s < 4; ++s) r.stage(s);
        ++r.n;
    }
    r.finish(a, b, threadIdx.x);
}

template <int P, int W, bool FULL, bool KEEP>
__global__ void __launch_bounds__(64 * W) evolve_kernel(EvolveArgs a)
{
    extern __shared__ double lds[];
    evolve_one<P, W, FULL, KEEP>(a, a.order[blockIdx.x], lds);
}

// LDS doubles of one half of a pair workgroup (even, so that the second half's
// double2 slots stay 16-byte aligned).
template <int P, int WH>
constexpr size_t pair_half_doubles()
{
    return (Stage<P, WH, true, true>::lds_doubles + 1) & ~(size_t)1;
}

// One launch of a full (P, W) class whose workgroups past the first n_single
// each run two instances of a full (P, W/2) class side by side: order[0,
// n_single) are the (P, W) instances, order[n_single, n_inst) the (P, W/2)
// ones, taken two per workgroup.  Each half keeps its own Stage over its own
// LDS; the halves share only the workgroup barriers, so they step in
// lock-step, and a half whose instance has stopped (or that has none) passes
// the same barriers without computing until both have stopped.  Placed in the
// dispatch order after the (P, W) instances, the pairs take the compute units
// those free as they end, instead of waiting for the whole (P, W) launch.
template <int P, int W>
__global__ void __launch_bounds__(64 * W) evolve_pair_kernel(EvolveArgs a, int n_single, int n_inst)
{
    extern __shared__ double lds[];
    if ((int)blockIdx.x < n_single) {
        evolve_one<P, W, true, false>(a, a.order[blockIdx.x], lds);
        return;
    }
    constexpr int WH = W / 2;
    constexpr size_t HL = pair_half_doubles<P, WH>();
    const int half = __builtin_amdgcn_readfirstlane((int)threadIdx.x / (64 * WH));  // uniform per wavefront
    const int t = (int)threadIdx.x - half * 64 * WH;
    volatile int* const act = reinterpret_cast<volatile int*>(lds + 2 * HL);  // [2]: half running this step
    const int slot = n_single + 2 * ((int)blockIdx.x - n_single) + half;
    const int b = slot < n_inst ? a.order[slot] : -1;
    Run<P, WH, true, false> r;
    // `loaded`, `run` and the exit test are uniform over each half (readfirstlane
    // makes that visible to the compiler), so the branches below are jumps of
    // whole wavefronts and no wavefront passes a barrier of the branch it skips
    const bool loaded = __builtin_amdgcn_readfirstlane((b >= 0) && r.init(a, b, lds + half * HL, t)) != 0;
    bool run = loaded;
    // a stage of Stage::rhs on the edge path passes this many barriers
    const int nbar = Stage<P, WH, true, true>::edge_barriers(a.frozen != 0);
    auto idle = [&]() {
#pragma unroll 1
        for (int i = 0; i < nbar; ++i) __syncthreads();
    };
    if (run) r.sg.publish(r.un0, r.un1);
    for (;;) {
        if (run && r.n >= r.seg_end) run = false;
        run = __builtin_amdgcn_readfirstlane(run) != 0;
        // written before this step's first barrier, read after it; the next
        // write follows the barriers of stages 1-3
        if (t == 0) act[half] = run ? 1 : 0;
        if (run) {
            r.begin_step(a);
            if (r.stage(0)) run = false;
        } else {
            idle();
        }
        run = __builtin_amdgcn_readfirstlane(run) != 0;
        // both halves leave after the same stage, on the same two flags
        if (__builtin_amdgcn_readfirstlane(act[0] | act[1]) == 0) break;
#pragma unroll 1
        for (int s = 1; s < 4; ++s) {
            if (run) r.stage(s);
            else idle();
        }
        if (run) ++r.n;
    }
    if (loaded) r.finish(a, b, t);
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

template <int P, int W>
constexpr size_t pair_lds_bytes()
{
    return std::max(lds_bytes_for<P, W, true>(), (2 * pair_half_doubles<P, W / 2>() + 2) * sizeof(double));
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

// Pair launches (evolve_pair_kernel): the (P, W) configurations whose launch
// can also run (P, W/2) instances two per workgroup.
#define ADSCL_PAIR_CLASSES(X) X(8, 8)

bool pair_supported(ClassCfg c)
{
#define X(p, w) \
    if (c.P == p && c.W == w) return true;
    ADSCL_PAIR_CLASSES(X)
#undef X
    return false;
}

hipError_t prepare_evolve_pair(ClassCfg c, size_t max_lds)
{
#define X(p, w)                                                                                            \
    if (c.P == p && c.W == w) {                                                                           \
        if (pair_lds_bytes<p, w>() > max_lds) return hipErrorInvalidValue;                                 \
        return hipFuncSetAttribute((const void*)evolve_pair_kernel<p, w>,                                 \
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)pair_lds_bytes<p, w>()); \
    }
    ADSCL_PAIR_CLASSES(X)
#undef X
    return hipErrorInvalidValue;
}

hipError_t launch_evolve_pair(ClassCfg c, int n_single, int n_inst, const EvolveArgs& a, hipStream_t s)
{
    if (n_single < 0 || n_inst < n_single) return hipErrorInvalidValue;
    const int blocks = n_single + (n_inst - n_single + 1) / 2;
    if (blocks == 0) return hipSuccess;
#define X(p, w)                                                                                                   \
    if (c.P == p && c.W == w) {                                                                                  \
        evolve_pair_kernel<p, w><<<dim3(blocks), dim3(64 * w), pair_lds_bytes<p, w>(), s>>>(a, n_single, n_inst); \
        return hipGetLastError();                                                                                \
    }
    ADSCL_PAIR_CLASSES(X)
#undef X
    return hipErrorInvalidValue;
}

}  // namespace adscl
