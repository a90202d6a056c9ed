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
    int64_t total;
    double a_collapse;
    int32_t snap_every;     // > 0: stop each instance at the next multiple
    int32_t gauge;          // 0 boundary, 1 origin
    int32_t frozen;
    int32_t pad;
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
                           int32_t n_slots, double* snaps, hipStream_t s);
// Diagnostics: out[b*4 + {0..3}] = max|R_A'|, max|R_delta'|, m(pi/2), M (cell rule).
hipError_t launch_diagnostics(int n_inst, const InstConst* ic, const double* Phi, const double* Pi,
                              const double* A, const double* delta, const double* m, double* out,
                              hipStream_t s);
// Spectrum: per instance projection of sqrt(A) Pi, sqrt(A) Phi on weight tables
// wPi[b] = h t2 e_j, wPhi[b] = h t2 e_j'/omega_j, each [Jtab][N].
hipError_t launch_spectrum(int n_inst, const InstConst* ic, const double* Phi, const double* Pi,
                           const double* A, const double* const* wPi, const double* const* wPhi, int J,
                           double* E, double* Pihat, double* Phihat, hipStream_t s);

}  // namespace adscl
