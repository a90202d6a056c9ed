// Internal declarations shared by the adscl kernels and the C-ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace adscl {

constexpr double kPi = 3.14159265358979323846;

enum : int32_t { ST_RUNNING = 0, ST_COLLAPSED = 1, ST_NONFINITE = 2, ST_DONE = 3 };

// Per-instance status kept on the device.
struct InstStatus {
    int64_t steps;   // current step n (state is U^n)
    int64_t target;  // last step of the current call
    double t_c;      // time of collapse / non-finite detection, -1 if none
    double minA;     // min A of U^n
    double mass;     // m(pi/2) of U^n
    int32_t state;   // ST_*
    int32_t pad;
};

// Per-instance constants of one call, built on the host so that the kernel
// reads them with uniform (scalar) loads.
struct InstConst {
    int64_t off;      // packed offset of the instance
    int64_t n_final;  // ceil(t_end / dt - 1e-9)
    int32_t N;
    int32_t pad;
    double h;         // (pi/2)/(N-1)
    double dt;        // cfl h
    double h24;       // h/24
    double i12h;      // 1/(12 h)
    double kof;       // sigma_KO/(64 h)
};

// Arguments of the fused evolution kernel (one launch per (P, W) class).
struct EvolveArgs {
    double* Phi;            // packed state, [total]
    double* Pi;
    double* A;              // packed metric of the current state, [total]
    double* delta;
    double* m;
    const InstConst* ic;    // [n_inst]
    const int32_t* order;   // instance index per workgroup of this launch
    const double* const* tab;  // per instance: lane-interleaved tables of its class
    InstStatus* status;     // [n_inst]
    // optional: per instance, stored states ([slot][2][N]: Phi then Pi, one
    // every src_every steps) to start from, slot = n_start / src_every,
    // instead of (Phi, Pi); and where to store the state every ckpt_every steps
    // of the segment ([slot][2][N], slot = (n - n_start) / ckpt_every)
    const double* const* src;
    double* const* ckpt;
    // optional (the adjoint's segment recompute): per instance, the stage record
    // of every step of the segment, [n - n_start][4 stages][P][64 W][4]: each RK
    // stage's input (Phi, Pi), e^-delta and S (StageRec in stage.h)
    double* const* keep;
    int64_t total;
    double a_collapse;
    int32_t snap_every;     // > 0: stop each instance at the next multiple
    int32_t gauge;          // 0 boundary, 1 origin
    int32_t frozen;
    int32_t ckpt_every;
    int32_t src_every;
    int32_t a_reint;        // A evolved by Eq. (4), re-integrated every a_reint steps (0: solved)
};

// A kernel configuration: P grid points per lane, W wavefronts per instance.
struct ClassCfg {
    int P;
    int W;
};

// Tables for one (N, P, W): three arrays sc, t2, ct2, each [P][64 W] with entry
// (k, lane) = value at grid point lane*P + k (zero outside 1..N-2).
size_t table_len(ClassCfg c);

bool class_supported(ClassCfg c);
size_t evolve_lds_bytes(ClassCfg c);
hipError_t prepare_evolve(ClassCfg c, size_t max_lds);
// full: every instance of the launch has N - 1 == 64 W P.
hipError_t launch_evolve(ClassCfg c, bool full, int n_blocks, const EvolveArgs& a, hipStream_t s);
// Pair launch of a full (P, W) class: a.order[0, n_single) are its instances
// (one workgroup each), a.order[n_single, n_inst) instances of a full
// (P, W/2) class, two per workgroup, in the same launch.
bool pair_supported(ClassCfg c);
hipError_t prepare_evolve_pair(ClassCfg c, size_t max_lds);
hipError_t launch_evolve_pair(ClassCfg c, int n_single, int n_inst, const EvolveArgs& a, hipStream_t s);
// The scheme variants (scheme.hip): RK order 2 or 3 (A solved or evolved), or
// 4 with A evolved (eva), on the configurations scheme_class_supported accepts.
bool scheme_class_supported(ClassCfg c);
hipError_t prepare_evolve_scheme(ClassCfg c, int rk, bool eva, size_t max_lds);
hipError_t launch_evolve_scheme(ClassCfg c, int rk, bool eva, bool full, int n_blocks, const EvolveArgs& a,
                                hipStream_t s);

// One large instance of a (merged) launch of the multi-workgroup kernel: its
// workgroups are [first, first + chunks) of the launch.
struct BigDesc {
    int32_t inst;             // instance index
    int32_t chunks;           // G
    int32_t first;            // its first workgroup in the launch, and its first exchange record
    int32_t pad;
};
// The pointers sit in the kernel arguments (not in the table) so that the
// compiler knows they address global memory and emits global, not flat,
// loads and atomics for the exchange records and counters.
struct BigArgs {
    const BigDesc* desc;      // device [n_desc]
    double* xch;              // exchange records [blocks][32], in launch order
    unsigned long long* ctr;  // per instance: arrival counter, then the error flag (int) [n_desc][kBigCtrStride]
    int32_t n_desc;
    int32_t pad;
};
bool big_class_supported(ClassCfg c);
size_t big_lds_bytes(ClassCfg c);
// The multi-workgroup kernel of a scheme (rk: Runge-Kutta order 2, 3 or 4;
// eva: A evolved by Eq. (4)) in chunk configuration c.
hipError_t prepare_evolve_big(ClassCfg c, int rk, bool eva, size_t max_lds);
// Workgroups of that kernel the device holds at once.
hipError_t big_capacity(ClassCfg c, int rk, bool eva, int device, int* blocks);
// One cooperative launch of `blocks` workgroups over the instances of x (all in
// configuration c, sum of their chunks = blocks <= big_capacity).
hipError_t launch_evolve_big(ClassCfg c, int rk, bool eva, int blocks, const EvolveArgs& a, const BigArgs& x,
                             hipStream_t s);
// At most 64 chunks: the kernel scans the chunks' totals and gathers their
// collapse bits with one wavefront lane per chunk.
constexpr int kBigMaxChunks = 64;
// 64-bit words between two instances' barrier counters: one 256-byte block
// each, so that the instances of a launch do not poll and count on one line.
constexpr int kBigCtrStride = 32;

// Initial data: Pi = (2 eps/pi) exp(-4 tan^2 x/(pi^2 sigma^2)), Phi = 0 (pins applied).
hipError_t launch_init_gaussian(int n_inst, const InstConst* ic, const double* eps, const double* sigma,
                                double* Phi, double* Pi, int64_t max_N, hipStream_t s);
// Pi = eps sum_j c_j e_j(x_i) with the mode table emode[b] = e_j(x_i), [Jtab][N].
hipError_t launch_init_modes(int n_inst, const InstConst* ic, const double* eps, const double* c, int Jc,
                             const double* const* emode, double* Phi, double* Pi, int64_t max_N,
                             hipStream_t s);
// Pins Phi_0 = Phi_{N-1} = Pi_{N-1} = 0.
hipError_t launch_pins(int n_inst, const InstConst* ic, double* Phi, double* Pi, hipStream_t s);
hipError_t launch_reset_status(int n_inst, InstStatus* st, hipStream_t s);
// target = clamp(steps + max_steps, steps, n_final) for instances still evolving.
hipError_t launch_set_targets(int n_inst, const InstConst* ic, InstStatus* st, int64_t max_steps, hipStream_t s);
// Constraint solve of the packed state (Phi, Pi) -> A, delta, m, min A, mass.
// Writes (Phi, Pi, A, delta, m) to `out` (5 rows of `total`) when `final` and
// to snapshot slot steps / snap_every when snapshots are on and due; when
// `final`, an instance at its target is tested for collapse / non-finite data
// and marked DONE at n_final.
hipError_t launch_finalize(int n_inst, const InstConst* ic, InstStatus* st, double* state5, int64_t total,
                           int gauge, int frozen, double a_collapse, bool final, int32_t snap_every,
                           int32_t n_slots, double* snaps, hipStream_t s, int32_t a_reint = 0);
// Diagnostics: out[b*4 + {0..3}] = max|R_A'|, max|R_delta'|, m(pi/2), M (cell rule).
hipError_t launch_diagnostics(int n_inst, const InstConst* ic, const double* Phi, const double* Pi,
                              const double* A, const double* delta, const double* m, double* out,
                              hipStream_t s);
// Residual of Eq. (4) into column 2 of out [n_inst][5]; scr: 2 * total doubles.
hipError_t launch_adot_residual(int n_inst, const InstConst* ic, const double* state5, int64_t total, int frozen,
                                double ko, double* scr, double* out, hipStream_t s);

// Fixed device scratch of the allocation-free entry point: 2^21 doubles
// (16 MiB) per GPU, held until the process ends.  static_scratch_init looks up
// its address on `device`, which must be the current device (once per device;
// later calls return at once); static_scratch returns it, or NULL before that.
constexpr size_t kStaticScratchDoubles = (size_t)1 << 21;
hipError_t static_scratch_init(int device);
double* static_scratch(int device);
// Spectrum rows: one state of one instance, as element offsets of its Phi, Pi
// and A rows from a common base, and its output row.
struct SpecRow {
    int64_t phi;
    int64_t pi;
    int64_t a;
    int64_t out;
};
// Projection of sqrt(A) Pi, sqrt(A) Phi of `n_rows` rows of grid size N on the
// weight tables wPi = h t2 e_j, wPhi = h t2 e_j'/omega_j ([Jtab][N]); outputs
// [out][J] (any may be NULL).  FP64 MFMA.
hipError_t launch_spectrum_rows(const double* base, const SpecRow* rows, int n_rows, int N, const double* wPi,
                                const double* wPhi, int J, double* E, double* Pihat, double* Phihat, hipStream_t s);

// ---- discrete adjoint -------------------------------------------------------

// The steps [n0, n1) one reverse launch takes an instance through.
struct AdjSeg {
    int64_t n0;
    int64_t n1;
    int32_t active;
    int32_t pad;
};

// Arguments of the reverse (adjoint) kernel: for every active instance, the
// steps n1-1 down to n0 in reverse, each from its stored state U^t.
struct AdjointArgs {
    const InstConst* ic;
    const int32_t* order;
    const double* const* tab;
    const double* const* seg;  // per instance: U^t for t = n0..n1, [t - n0][2][N]
    double* const* stg;        // per instance: stage scratch, adjoint_scratch_len(cfg)
    // optional: per instance, the segment's stage record written by the forward
    // recompute (EvolveArgs::keep); the reverse then reads each step's stages
    // from it instead of recomputing them from seg
    double* const* keep;
    const AdjSeg* sg;          // [n_inst]
    double* Ubar;              // packed adjoint state, [2][total], updated in place
    int64_t total;
    int32_t gauge;
    int32_t pad;
};

// Arguments of the end-point kernel: adjoint of E_j = Pihat_j^2 + Phihat_j^2 and
// of the constraint solve at a state, Ebar_j = 2 sgn (ET_j - E0_j), added to Ubar.
struct EndArgs {
    const InstConst* ic;
    const int32_t* order;
    const double* const* tab;
    const double* Phi;         // packed state, [total]
    const double* Pi;
    const double* const* wPi;  // [Jtab][N] per instance
    const double* const* wPhi;
    const double* Pihat;       // [n_inst][J] at this state
    const double* Phihat;
    const double* E0;          // [n_inst][J]
    const double* ET;
    const InstStatus* status;  // instances in state DONE only
    double* Ubar;
    int64_t total;
    double sgn;
    int32_t J;
    int32_t gauge;
};

size_t adjoint_scratch_len(ClassCfg c);
// Doubles of one step's stage record (EvolveArgs::keep) in configuration c.
size_t stage_record_len(ClassCfg c);
hipError_t prepare_adjoint(ClassCfg c, size_t max_lds);
hipError_t launch_adjoint(ClassCfg c, bool full, int n_blocks, const AdjointArgs& a, hipStream_t s);
hipError_t launch_endpoint(ClassCfg c, bool full, int n_blocks, const EndArgs& a, hipStream_t s);
// Segment r (counted from the end) of every instance that is DONE: recompute
// status rst (steps n0, target n1; others COLLAPSED so the kernels skip them)
// and the reverse range sg.
hipError_t launch_adj_prepare(int n_inst, const InstConst* ic, const InstStatus* st, int64_t K, int64_t r,
                              InstStatus* rst, AdjSeg* sg, hipStream_t s);
// L_b = sum_j (ET - E0)^2; dL/dc_bk = eps_b sum_{i <= N-2} Pibar_i e_k(x_i) for
// DONE instances (0 otherwise); valid_b = (state == DONE).
hipError_t launch_adj_finish(int n_inst, const InstConst* ic, const InstStatus* st, const double* Ubar,
                             int64_t total, const double* const* emode, const double* eps, int Jc,
                             const double* E0, const double* ET, int J, double* L, double* dLdc,
                             int32_t* valid, hipStream_t s);

// Fill n doubles with v (a kernel, so that it can sit in a captured graph).
hipError_t launch_fill(double* p, int64_t n, double v, hipStream_t s);
// Mark instances with active[b] == 0 as COLLAPSED (the kernels skip them).
hipError_t launch_mask(int n_inst, InstStatus* st, const int32_t* active, hipStream_t s);

// State of the batched gradient descent, on the device.
struct GdState {
    double* s;        // [n_inst] step fraction
    double* Lprev;    // [n_inst] objective of the previous iteration
    int32_t* active;  // [n_inst] 0 once the instance collapsed
    int32_t* iter;    // [1] iteration counter
};
hipError_t launch_gd_init(int n_inst, double step0, const GdState& g, hipStream_t s);
// Iteration iter: L_hist[iter][b] = L_b (NaN for masked instances); an invalid
// instance is masked; s_b halves when L_b grew; c_b -= s_b |c_b| / |g_b| g_b;
// then iter += 1.
hipError_t launch_gd_update(int n_inst, int Jc, double* c, const double* grad, const double* L, const int32_t* valid,
                            const GdState& g, double* L_hist, hipStream_t s);

}  // namespace adscl
