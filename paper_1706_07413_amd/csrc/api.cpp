// C-ABI layer and host runtime of the adscl library: context, packed ragged
// batch layout, per-N coefficient and mode tables, per-class launch plan.
// Declarations and the meaning of every call are in include/adscl.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/adscl.h"
#include "internal.h"

using namespace adscl;

namespace {

thread_local std::string g_create_error;
constexpr int kMaxN = 65537;       // largest grid
constexpr int kMaxOneGroup = 4097;  // largest grid one workgroup holds

// One launch of the fused kernel: a (P, W) configuration, whether all its
// instances fill it exactly, and its instances in launch order.
struct LaunchClass {
    ClassCfg cfg;
    bool full;
    std::vector<int32_t> inst;
    int32_t* d_order = nullptr;
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    hipEvent_t t0 = nullptr, t1 = nullptr;  // timing (ADSCL_TIME_KERNELS)
    bool timed = false;
    // one large instance over `chunks` workgroups (0: one workgroup per instance)
    int chunks = 0;
    // forward pass only: the class whose instances this class's launch also
    // runs, two per workgroup (-1: none), and its launch order (this class's
    // instances, then that class's); or, for that class, the class whose launch
    // runs its instances (-1: its own launch)
    int pair = -1;
    int32_t* d_order_pair = nullptr;
    int host = -1;
};

// One cooperative launch of the multi-workgroup kernel over several large
// instances (classes `cls` of the context, all in configuration cfg).
struct BigGroup {
    ClassCfg cfg;
    int blocks = 0;
    std::vector<int> cls;
    BigDesc* d_desc = nullptr;
    double* xch = nullptr;              // exchange records [blocks][32]
    unsigned long long* ctr = nullptr;  // [cls.size()][kBigCtrStride]: arrival counter, error flag
};

// Host-side tables of one grid size N.
struct NTables {
    ClassCfg cfg;
    double* d_tab = nullptr;     // lane-interleaved sc, t2, ct2 for cfg
    double* d_emode = nullptr;   // e_j(x_i), [J][N]
    double* d_wPi = nullptr;     // h tan^2 x e_j, [J][N]
    double* d_wPhi = nullptr;    // h tan^2 x e_j'/omega_j, [J][N]
};

}  // namespace

struct adscl_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int n_inst = 0;
    std::vector<int32_t> N;
    std::vector<int64_t> off;
    int64_t total = 0;
    int64_t max_N = 0;
    double cfl = 0.25, ko = 0.5, thr = 0.01;
    int gauge = 0, n_modes = 0, flags = 0;
    int rk = 4, a_reint = 0;    // scheme options (adscl_config.rk_order, a_reint)
    size_t max_lds = 0;

    double* state5 = nullptr;   // [5][total]: Phi, Pi, A, delta, m
    InstStatus* d_status = nullptr;
    InstConst* d_ic = nullptr;
    std::vector<InstConst> h_ic;
    const double** d_tab = nullptr;
    const double** d_emode = nullptr;
    const double** d_wPi = nullptr;
    const double** d_wPhi = nullptr;
    std::map<int, NTables> tables;
    std::vector<LaunchClass> classes;
    double* d_tmp = nullptr;    // staging for host inputs / outputs
    size_t tmp_bytes = 0;
    // adjoint working memory, kept for reuse by later calls
    std::map<std::string, std::pair<void*, size_t>> bufs;
    hipEvent_t fork = nullptr;  // start of a multi-class launch, recorded on `stream`
    int n_big = 0;              // classes holding one large (multi-workgroup) instance
    std::vector<BigGroup> big_groups;  // their launches
    // spectrum rows for states laid out as [slot][5][total], grouped by N:
    // (N, first row, rows) per group, for spec_slots slots
    int spec_slots = -1;
    std::vector<std::array<int, 3>> spec_groups;
    SpecRow* d_spec_rows = nullptr;
    bool initialized = false;
    std::string err;
};

namespace {

int fail(adscl_ctx* c, int code, const std::string& msg)
{
    if (c) c->err = msg;
    else g_create_error = msg;
    return code;
}

#define HIP_TRY(ctx, call)                                                                        \
    do {                                                                                          \
        hipError_t e_ = (call);                                                                   \
        if (e_ != hipSuccess)                                                                     \
            return fail(ctx, e_ == hipErrorOutOfMemory ? ADSCL_ENOMEM : ADSCL_EHIP,               \
                        std::string(#call) + ": " + hipGetErrorString(e_));                       \
    } while (0)

// Configurations chosen by adscl_autotune (grid size -> configuration), and the
// one a tuning trial forces on the calling thread.
std::mutex g_tune_mu;
std::map<int, ClassCfg> g_tuned;
thread_local int g_force_N = 0;
thread_local ClassCfg g_force{0, 0};

// Every configuration the kernels are compiled for.
const ClassCfg kAllClasses[] = {{4, 1}, {4, 2}, {4, 4},  {4, 8},  {4, 16}, {8, 1},
                                {8, 2}, {8, 4}, {8, 8}, {16, 1}, {16, 2}, {16, 4}};

// The smallest lane capacity 64 W P of the default configurations that holds
// the N-1 evolved points, taking P = 8 over W = 8 at 2048 points (four
// wavefronts, one per SIMD, so that two instances can share a compute unit).
ClassCfg default_class(int N)
{
    static const ClassCfg pref[] = {{4, 1}, {4, 2}, {4, 4}, {8, 4}, {8, 8}};
    for (const ClassCfg& c : pref)
        if (64 * c.W * c.P >= N - 1) return c;
    return ClassCfg{0, 0};
}

// Kernel configuration for grid size N: ADSCL_TUNE="N:PxW,..." if it names one
// for N, else the configuration a tuning trial forces, else the autotuner's
// choice for N, else default_class(N).
ClassCfg choose_class(int N)
{
    if (const char* t = std::getenv("ADSCL_TUNE")) {
        std::string s(t);
        size_t pos = 0;
        while (pos < s.size()) {
            size_t end = s.find(',', pos);
            if (end == std::string::npos) end = s.size();
            int n = 0, p = 0, w = 0;
            if (std::sscanf(s.substr(pos, end - pos).c_str(), "%d:%dx%d", &n, &p, &w) == 3 && n == N) {
                ClassCfg c{p, w};
                if (class_supported(c) && 64 * w * p >= N - 1) return c;
            }
            pos = end + 1;
        }
    }
    if (g_force_N == N) return g_force;
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        auto it = g_tuned.find(N);
        if (it != g_tuned.end()) return it->second;
    }
    return default_class(N);
}

// Chunk configuration for a grid too large for one workgroup: (4, 8), i.e.
// 2048 points per workgroup, unless ADSCL_TUNE names another supported one.
ClassCfg choose_big_class(int N)
{
    if (const char* t = std::getenv("ADSCL_TUNE")) {
        std::string s(t);
        size_t pos = 0;
        while (pos < s.size()) {
            size_t end = s.find(',', pos);
            if (end == std::string::npos) end = s.size();
            int n = 0, p = 0, w = 0;
            if (std::sscanf(s.substr(pos, end - pos).c_str(), "%d:%dx%d", &n, &p, &w) == 3 && n == N) {
                ClassCfg c{p, w};
                if (big_class_supported(c)) return c;
            }
            pos = end + 1;
        }
    }
    return ClassCfg{4, 8};
}

// sin, cos in long double for the tables (the kernel reads FP64 values).
// `chunks` > 1: one [3][P][64 W] block per chunk of 64 W P points.
void host_tables(int N, ClassCfg cfg, std::vector<double>& tab, int chunks = 1)
{
    const int NL = 64 * cfg.W, P = cfg.P;
    tab.assign(table_len(cfg) * chunks, 0.0);
    const long double h = (3.14159265358979323846264338327950288L / 2.0L) / (long double)(N - 1);
    for (int ch = 0; ch < chunks; ++ch)
    for (int lane = 0; lane < NL; ++lane) {
        for (int k = 0; k < P; ++k) {
            const int i = ch * NL * P + lane * P + k;
            double sc = 0.0, t2 = 0.0, ct2 = 0.0;
            if (i >= 1 && i <= N - 2) {
                const long double x = h * (long double)i;
                const long double s = sinl(x), c = cosl(x);
                sc = (double)(s * c);
                t2 = (double)((s * s) / (c * c));
                ct2 = (double)((c * c) / (s * s));
            }
            const size_t base = (size_t)ch * table_len(cfg);
            tab[base + (size_t)(0 * P + k) * NL + lane] = sc;
            tab[base + (size_t)(1 * P + k) * NL + lane] = t2;
            tab[base + (size_t)(2 * P + k) * NL + lane] = ct2;
        }
    }
}

// Linear AdS4 eigenmodes e_j(x) = d_j cos^3 x P_j^(1/2,3/2)(cos 2x), unit norm in
// int f g tan^2 x dx, and their x-derivatives, evaluated in long double with the
// three-term recurrence for P_n^(a,b) (DLMF 18.9.1).
void host_modes(int N, int J, std::vector<double>& e, std::vector<double>& wpi, std::vector<double>& wphi)
{
    e.assign((size_t)J * N, 0.0);
    wpi.assign((size_t)J * N, 0.0);
    wphi.assign((size_t)J * N, 0.0);
    const long double PI = 3.14159265358979323846264338327950288L;
    const long double h = (PI / 2.0L) / (long double)(N - 1);
    auto jacobi = [](int n, long double a, long double b, long double z) -> long double {
        long double pm = 1.0L;
        if (n == 0) return pm;
        long double p = 0.5L * ((a + b + 2.0L) * z + (a - b));
        for (int m = 2; m <= n; ++m) {
            const long double c = 2.0L * m + a + b;
            const long double num1 = (c - 1.0L) * (c * (c - 2.0L) * z + a * a - b * b);
            const long double num2 = 2.0L * (m + a - 1.0L) * (m + b - 1.0L) * c;
            const long double den = 2.0L * m * (m + a + b) * (c - 2.0L);
            const long double pn = (num1 * p - num2 * pm) / den;
            pm = p;
            p = pn;
        }
        return p;
    };
    for (int j = 0; j < J; ++j) {
        const long double d = 2.0L * expl(0.5L * (lgammal(j + 1.0L) + lgammal(j + 3.0L)) - lgammal(j + 1.5L));
        const long double om = 3.0L + 2.0L * j;
        for (int i = 0; i < N; ++i) {
            const long double x = h * (long double)i;
            long double s = sinl(x), c = cosl(x);
            if (i == N - 1) { s = 1.0L; c = 0.0L; }
            const long double z = c * c - s * s;
            const long double Pj = jacobi(j, 0.5L, 1.5L, z);
            const long double dPj = (j > 0) ? 0.5L * (j + 3.0L) * jacobi(j - 1, 1.5L, 2.5L, z) : 0.0L;
            const long double ej = d * c * c * c * Pj;
            const long double dej = d * (-3.0L * c * c * s * Pj - 4.0L * s * c * c * c * c * dPj);
            e[(size_t)j * N + i] = (double)ej;
            if (i >= 1 && i <= N - 2) {
                const long double t2 = (s * s) / (c * c);
                wpi[(size_t)j * N + i] = (double)(h * t2 * ej);
                wphi[(size_t)j * N + i] = (double)(h * t2 * dej / om);
            }
        }
    }
}

int ensure_tmp(adscl_ctx* c, size_t bytes)
{
    if (bytes <= c->tmp_bytes) return ADSCL_OK;
    if (c->d_tmp) (void)hipFree(c->d_tmp);
    c->d_tmp = nullptr;
    c->tmp_bytes = 0;
    HIP_TRY(c, hipMalloc((void**)&c->d_tmp, bytes));
    c->tmp_bytes = bytes;
    return ADSCL_OK;
}

// Device pointer to `n` doubles of `src`: the pointer itself for device memory,
// else a copy in the staging buffer at double offset `slot`.
int stage_in(adscl_ctx* c, const double* src, size_t n, int mem, size_t slot, const double** out)
{
    if (mem == ADSCL_MEM_DEVICE) {
        *out = src;
        return ADSCL_OK;
    }
    HIP_TRY(c, hipMemcpyAsync(c->d_tmp + slot, src, n * sizeof(double), hipMemcpyHostToDevice, c->stream));
    *out = c->d_tmp + slot;
    return ADSCL_OK;
}

int check_mem(adscl_ctx* c, int mem)
{
    if (mem != ADSCL_MEM_HOST && mem != ADSCL_MEM_DEVICE) return fail(c, ADSCL_EINVAL, "mem must be HOST or DEVICE");
    return ADSCL_OK;
}

int upload_ic(adscl_ctx* c, double t_end)
{
    for (int b = 0; b < c->n_inst; ++b) {
        InstConst& k = c->h_ic[b];
        const double r = t_end / k.dt - 1e-9;
        int64_t nf;
        if (!(r < 4.0e18)) nf = (int64_t)4e18;
        else if (r <= 0.0) nf = 0;
        else nf = (int64_t)std::ceil(r);
        k.n_final = nf;
    }
    // the previous call may still read d_ic
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    HIP_TRY(c, hipMemcpy(c->d_ic, c->h_ic.data(), sizeof(InstConst) * c->n_inst, hipMemcpyHostToDevice));
    return ADSCL_OK;
}

// Device buffer `name` of the context with at least `bytes` bytes (grown, not
// preserved, when too small).
int buffer(adscl_ctx* c, const char* name, size_t bytes, void** out)
{
    auto& e = c->bufs[name];
    if (e.second < bytes) {
        if (e.first) {
            HIP_TRY(c, hipStreamSynchronize(c->stream));
            HIP_TRY(c, hipFree(e.first));
        }
        e.first = nullptr;
        e.second = 0;
        HIP_TRY(c, hipMalloc(&e.first, std::max<size_t>(bytes, 256)));
        e.second = std::max<size_t>(bytes, 256);
    }
    *out = e.first;
    return ADSCL_OK;
}

// One launch per class, the classes concurrently (one stream per class, forked
// from and joined back into the context stream).  `launch(lc, stream)` enqueues
// the class's work.
template <class F>
int run_classes(adscl_ctx* c, F&& launch)
{
    hipEvent_t fork = c->fork;
    const bool multi = c->classes.size() - c->n_big > 1;
    if (multi) HIP_TRY(c, hipEventRecord(fork, c->stream));
    for (LaunchClass& lc : c->classes) {
        if (lc.chunks > 0) continue;
        hipStream_t s = multi ? lc.stream : c->stream;
        if (s != c->stream) HIP_TRY(c, hipStreamWaitEvent(s, fork, 0));
        HIP_TRY(c, launch(lc, s));
        if (s != c->stream) {
            HIP_TRY(c, hipEventRecord(lc.done, s));
            HIP_TRY(c, hipStreamWaitEvent(c->stream, lc.done, 0));
        }
    }
    return ADSCL_OK;
}

// Whether the context uses a scheme option other than classical RK4 with A
// solved at every stage.
bool scheme(const adscl_ctx* c) { return c->rk != 4 || c->a_reint > 0; }

EvolveArgs evolve_args(adscl_ctx* c, int32_t snap_every)
{
    EvolveArgs a;
    a.Phi = c->state5;
    a.Pi = c->state5 + c->total;
    a.A = c->state5 + 2 * c->total;
    a.delta = c->state5 + 3 * c->total;
    a.m = c->state5 + 4 * c->total;
    a.ic = c->d_ic;
    a.order = nullptr;
    a.tab = c->d_tab;
    a.status = c->d_status;
    a.src = nullptr;
    a.ckpt = nullptr;
    a.keep = nullptr;
    a.total = c->total;
    a.a_collapse = c->thr;
    a.snap_every = snap_every;
    a.gauge = c->gauge;
    a.frozen = (c->flags & ADSCL_FROZEN_METRIC) ? 1 : 0;
    a.ckpt_every = 0;
    a.src_every = 1;
    a.a_reint = c->a_reint;
    return a;
}

// One segment of the fused kernel over all classes: every instance advances to
// its target step, or to its next multiple of snap_every when that is > 0.
int run_evolve(adscl_ctx* c, const EvolveArgs& base, bool timing = true)
{
    for (BigGroup& g : c->big_groups) {
        BigArgs x;
        x.desc = g.d_desc;
        x.xch = g.xch;
        x.ctr = g.ctr;
        x.n_desc = (int32_t)g.cls.size();
        x.pad = 0;
        EvolveArgs a = base;
        a.order = nullptr;
        for (int k : g.cls)
            if (timing && c->classes[k].t0) HIP_TRY(c, hipEventRecord(c->classes[k].t0, c->stream));
        HIP_TRY(c, launch_evolve_big(g.cfg, c->rk, c->a_reint > 0, g.blocks, a, x, c->stream));
        for (int k : g.cls) {
            LaunchClass& lc = c->classes[k];
            if (timing && lc.t1) {
                HIP_TRY(c, hipEventRecord(lc.t1, c->stream));
                lc.timed = true;
            }
        }
    }
    const bool pairs = base.keep == nullptr;  // the pair kernel writes no stage records
    return run_classes(c, [&](LaunchClass& lc, hipStream_t s) -> hipError_t {
        if (pairs && lc.host >= 0) {  // runs in its host class's launch
            lc.timed = false;
            return hipSuccess;
        }
        EvolveArgs a = base;
        a.order = lc.d_order;
        hipError_t e = hipSuccess;
        if (timing && lc.t0 && (e = hipEventRecord(lc.t0, s)) != hipSuccess) return e;
        if (pairs && lc.pair >= 0) {
            a.order = lc.d_order_pair;
            const int ns = (int)lc.inst.size();
            e = launch_evolve_pair(lc.cfg, ns, ns + (int)c->classes[lc.pair].inst.size(), a, s);
        } else {
            e = scheme(c) ? launch_evolve_scheme(lc.cfg, c->rk, c->a_reint > 0, lc.full, (int)lc.inst.size(), a, s)
                          : launch_evolve(lc.cfg, lc.full, (int)lc.inst.size(), a, s);
        }
        if (e != hipSuccess) return e;
        if (timing && lc.t1) {
            if ((e = hipEventRecord(lc.t1, s)) != hipSuccess) return e;
            lc.timed = true;
        }
        return hipSuccess;
    });
}

int run_evolve(adscl_ctx* c, int32_t snap_every) { return run_evolve(c, evolve_args(c, snap_every)); }

int run_finalize(adscl_ctx* c, bool final, int32_t snap_every, int32_t n_slots, double* snaps)
{
    HIP_TRY(c, launch_finalize(c->n_inst, c->d_ic, c->d_status, c->state5, c->total, c->gauge,
                               (c->flags & ADSCL_FROZEN_METRIC) ? 1 : 0, c->thr, final, snap_every, n_slots,
                               snaps, c->stream, c->a_reint));
    return ADSCL_OK;
}

// Spectrum rows of `n_slots` states laid out as [slot][5][total] (Phi, Pi, A,
// ... rows), grouped by grid size; rebuilt when n_slots changes.  Synchronises.
int spec_rows(adscl_ctx* c, int n_slots)
{
    if (c->spec_slots == n_slots) return ADSCL_OK;
    std::vector<SpecRow> rows;
    c->spec_groups.clear();
    for (const auto& kv : c->tables) {
        const int N = kv.first;
        const int first = (int)rows.size();
        for (int sl = 0; sl < n_slots; ++sl) {
            const int64_t base = (int64_t)sl * 5 * c->total;
            for (int b = 0; b < c->n_inst; ++b) {
                if (c->N[b] != N) continue;
                rows.push_back(SpecRow{base + c->off[b], base + c->total + c->off[b], base + 2 * c->total + c->off[b],
                                       (int64_t)sl * c->n_inst + b});
            }
        }
        c->spec_groups.push_back({N, first, (int)rows.size() - first});
    }
    void* d;
    int rc = buffer(c, "spec_rows", sizeof(SpecRow) * rows.size(), &d);
    if (rc) return rc;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    HIP_TRY(c, hipMemcpy(d, rows.data(), sizeof(SpecRow) * rows.size(), hipMemcpyHostToDevice));
    c->d_spec_rows = (SpecRow*)d;
    c->spec_slots = n_slots;
    return ADSCL_OK;
}

// Spectra of the states at `base` (the layout spec_rows was built for).
int run_spectrum(adscl_ctx* c, const double* base, int J, double* E, double* Pihat, double* Phihat)
{
    for (const auto& g : c->spec_groups) {
        const NTables& t = c->tables[g[0]];
        HIP_TRY(c, launch_spectrum_rows(base, c->d_spec_rows + g[1], g[2], g[0], t.d_wPi, t.d_wPhi, J, E, Pihat,
                                        Phihat, c->stream));
    }
    return ADSCL_OK;
}

// Whole call: targets, then either one segment, or segments between snapshot
// steps with a snapshot after each; then the final solve and status.
int run_call(adscl_ctx* c, int64_t max_steps, double t_end, int32_t snap_every, int32_t n_slots, double* snaps)
{
    int rc = upload_ic(c, t_end);
    if (rc) return rc;
    HIP_TRY(c, launch_set_targets(c->n_inst, c->d_ic, c->d_status, max_steps, c->stream));
    if (snap_every > 0 && n_slots > 0) {
        if ((rc = run_finalize(c, false, snap_every, n_slots, snaps))) return rc;
        std::vector<InstStatus> st(c->n_inst);
        for (;;) {
            HIP_TRY(c, hipMemcpyAsync(st.data(), c->d_status, sizeof(InstStatus) * c->n_inst,
                                      hipMemcpyDeviceToHost, c->stream));
            HIP_TRY(c, hipStreamSynchronize(c->stream));
            bool more = false;
            for (const InstStatus& s : st)
                if ((s.state == ST_RUNNING || s.state == ST_DONE) && s.steps < s.target) more = true;
            if (!more) break;
            if ((rc = run_evolve(c, snap_every))) return rc;
            if ((rc = run_finalize(c, false, snap_every, n_slots, snaps))) return rc;
        }
    } else {
        if ((rc = run_evolve(c, 0))) return rc;
    }
    return run_finalize(c, true, 0, 0, nullptr);
}

// A large instance whose grid synchronisation ran out of time (reported as
// an error; its state is then NONFINITE).  Synchronises.
int check_big(adscl_ctx* c)
{
    for (const BigGroup& g : c->big_groups) {
        std::vector<unsigned long long> ctr(kBigCtrStride * g.cls.size());
        HIP_TRY(c, hipMemcpyAsync(ctr.data(), g.ctr, sizeof(unsigned long long) * ctr.size(), hipMemcpyDeviceToHost,
                                  c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        for (size_t d = 0; d < g.cls.size(); ++d) {
            int e = 0;
            std::memcpy(&e, &ctr[d * kBigCtrStride + 1], sizeof(int));
            if (e)
                return fail(c, ADSCL_EHIP, "instance " + std::to_string(c->classes[g.cls[d]].inst[0]) +
                                               ": a grid synchronisation of its workgroups timed out");
        }
    }
    return ADSCL_OK;
}

int after_init(adscl_ctx* c)
{
    double* Phi = c->state5;
    double* Pi = c->state5 + c->total;
    HIP_TRY(c, launch_pins(c->n_inst, c->d_ic, Phi, Pi, c->stream));
    HIP_TRY(c, launch_reset_status(c->n_inst, c->d_status, c->stream));
    int rc = upload_ic(c, 1.0e300);
    if (rc) return rc;
    // solve the constraints at t = 0 (no step), flag collapsed / non-finite data
    if ((rc = run_finalize(c, true, 0, 0, nullptr))) return rc;
    // Launch order within a class: longest expected run first.  Instances of
    // one class share N, so their cost is set by how long they live; a smaller
    // initial mass collapses later (or not at all), so it goes first.
    std::vector<InstStatus> st(c->n_inst);
    HIP_TRY(c, hipMemcpyAsync(st.data(), c->d_status, sizeof(InstStatus) * c->n_inst, hipMemcpyDeviceToHost,
                              c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (LaunchClass& lc : c->classes) {
        std::stable_sort(lc.inst.begin(), lc.inst.end(), [&](int x, int y) {
            if (c->N[x] != c->N[y]) return c->N[x] > c->N[y];
            return st[x].mass < st[y].mass;
        });
        HIP_TRY(c, hipMemcpy(lc.d_order, lc.inst.data(), lc.inst.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    }
    c->initialized = true;
    return ADSCL_OK;
}

// ---- adjoint -------------------------------------------------------------

// Device buffers and step counts of one adjoint configuration (T, K, J).
struct AdjPlan {
    int J = 0;
    int64_t K = 0;
    int64_t max_seg = 0;
    double *ub = nullptr, *u0 = nullptr, *dummy = nullptr;
    double *E0 = nullptr, *a0 = nullptr, *b0 = nullptr, *ET = nullptr, *aT = nullptr, *bT = nullptr;
    double** d_ckp = nullptr;
    double** d_segp = nullptr;
    double** d_stgp = nullptr;
    double** d_keepp = nullptr;  // the segments' stage records, when kept (`stored`)
    bool stored = false;
    InstStatus* rst = nullptr;
    AdjSeg* sgs = nullptr;
};

// Host part: step counts n_final for T, buffer sizes, per-instance pointer
// tables, the constants upload.  Synchronises the stream.
int adj_plan(adscl_ctx* c, double T, int64_t K, int J, AdjPlan& pl)
{
    const int n = c->n_inst;
    int rc;
    std::vector<int64_t> nf(n), ck_off(n + 1), seg_off(n + 1), stg_off(n + 1), keep_off(n + 1);
    pl.J = J;
    pl.K = K;
    pl.max_seg = 0;
    for (int b = 0; b < n; ++b) {
        const double r = T / c->h_ic[b].dt - 1e-9;
        nf[b] = (r <= 0.0) ? 0 : (int64_t)std::ceil(r);
        const NTables& t = c->tables[c->N[b]];
        ck_off[b + 1] = ck_off[b] + (nf[b] / K + 1) * 2 * (int64_t)c->N[b];
        seg_off[b + 1] = seg_off[b] + (std::min<int64_t>(K, nf[b]) + 1) * 2 * (int64_t)c->N[b];
        stg_off[b + 1] = stg_off[b] + (int64_t)adjoint_scratch_len(t.cfg);
        keep_off[b + 1] = keep_off[b] + std::min<int64_t>(K, nf[b]) * (int64_t)stage_record_len(t.cfg);
        pl.max_seg = std::max<int64_t>(pl.max_seg, (nf[b] + K - 1) / K);
    }
    // Keep each segment's stage record from the forward recompute (the reverse
    // kernel then reads the stages instead of recomputing them) when the
    // records take at most a quarter of the device memory; ADSCL_ADJOINT_RECOMPUTE
    // set to a value other than 0 always recomputes.
    {
        size_t free_b = 0, total_b = 0;
        HIP_TRY(c, hipMemGetInfo(&free_b, &total_b));
        const char* env = std::getenv("ADSCL_ADJOINT_RECOMPUTE");
        const bool force = env && env[0] && std::strcmp(env, "0") != 0;
        pl.stored = !force && sizeof(double) * (size_t)keep_off[n] <= total_b / 4;
    }
    void *ck, *seg, *stg, *keep = nullptr, *ub, *u0, *dummy, *spec, *ptrs, *rst, *sgs;
    const size_t nJ = (size_t)n * J;
    if ((rc = buffer(c, "ckpt", sizeof(double) * ck_off[n], &ck))) return rc;
    if (pl.stored) {
        if ((rc = buffer(c, "keep", sizeof(double) * keep_off[n], &keep))) return rc;
        seg_off.assign(n + 1, 0);  // no per-step states needed
    }
    if ((rc = buffer(c, "seg", sizeof(double) * seg_off[n], &seg))) return rc;
    if ((rc = buffer(c, "stage", sizeof(double) * stg_off[n], &stg))) return rc;
    if ((rc = buffer(c, "ubar", sizeof(double) * 2 * c->total, &ub))) return rc;
    if ((rc = buffer(c, "u0", sizeof(double) * 2 * c->total, &u0))) return rc;
    if ((rc = buffer(c, "dummy", sizeof(double) * 2 * c->total, &dummy))) return rc;
    if ((rc = buffer(c, "spec", sizeof(double) * 6 * nJ, &spec))) return rc;
    if ((rc = buffer(c, "ptrs", sizeof(double*) * 4 * n, &ptrs))) return rc;
    if ((rc = buffer(c, "rstatus", sizeof(InstStatus) * n, &rst))) return rc;
    if ((rc = buffer(c, "segs", sizeof(AdjSeg) * n, &sgs))) return rc;
    pl.ub = (double*)ub;
    pl.u0 = (double*)u0;
    pl.dummy = (double*)dummy;
    pl.E0 = (double*)spec;
    pl.a0 = pl.E0 + nJ;
    pl.b0 = pl.a0 + nJ;
    pl.ET = pl.b0 + nJ;
    pl.aT = pl.ET + nJ;
    pl.bT = pl.aT + nJ;
    pl.d_ckp = (double**)ptrs;
    pl.d_segp = pl.d_ckp + n;
    pl.d_stgp = pl.d_segp + n;
    pl.d_keepp = pl.d_stgp + n;
    pl.rst = (InstStatus*)rst;
    pl.sgs = (AdjSeg*)sgs;
    std::vector<double*> hp(4 * n);
    for (int b = 0; b < n; ++b) {
        hp[b] = (double*)ck + ck_off[b];
        hp[n + b] = (double*)seg + seg_off[b];
        hp[2 * n + b] = (double*)stg + stg_off[b];
        hp[3 * n + b] = pl.stored ? (double*)keep + keep_off[b] : nullptr;
    }
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    HIP_TRY(c, hipMemcpy(ptrs, hp.data(), sizeof(double*) * 4 * n, hipMemcpyHostToDevice));
    if ((rc = spec_rows(c, 1))) return rc;
    return upload_ic(c, T);
}

// Device part: the whole gradient computation for data eps, c (device arrays)
// -- initial data and its spectrum, the evolution with checkpoints, the final
// spectrum, then the reverse sweep segment by segment and the initial map.
// Only kernel launches, event waits and device copies: no host
// synchronisation and no memset, so that it can be captured into a graph.
// Instances with active[b] == 0 (when active is given) are skipped.
int adj_enqueue(adscl_ctx* c, const AdjPlan& pl, const double* d_eps, const double* d_c, int Jc,
                const int32_t* d_active, bool timing, double* oL, double* oG, int32_t* oV)
{
    const int n = c->n_inst;
    const int J = pl.J;
    double* s5 = c->state5;
    int rc;
    HIP_TRY(c, launch_init_modes(n, c->d_ic, d_eps, d_c, Jc, c->d_emode, s5, s5 + c->total, c->max_N, c->stream));
    HIP_TRY(c, launch_pins(n, c->d_ic, s5, s5 + c->total, c->stream));
    HIP_TRY(c, launch_reset_status(n, c->d_status, c->stream));
    if ((rc = run_finalize(c, true, 0, 0, nullptr))) return rc;
    if (d_active) HIP_TRY(c, launch_mask(n, c->d_status, d_active, c->stream));
    HIP_TRY(c, hipMemcpyAsync(pl.u0, s5, sizeof(double) * 2 * c->total, hipMemcpyDeviceToDevice, c->stream));
    if ((rc = run_spectrum(c, s5, J, pl.E0, pl.a0, pl.b0))) return rc;
    HIP_TRY(c, launch_set_targets(n, c->d_ic, c->d_status, INT64_MAX / 4, c->stream));
    {
        EvolveArgs a = evolve_args(c, 0);
        a.ckpt = pl.d_ckp;
        a.ckpt_every = (int32_t)pl.K;
        if ((rc = run_evolve(c, a, timing))) return rc;
    }
    if ((rc = run_finalize(c, true, 0, 0, nullptr))) return rc;
    if ((rc = run_spectrum(c, s5, J, pl.ET, pl.aT, pl.bT))) return rc;

    HIP_TRY(c, launch_fill(pl.ub, 2 * c->total, 0.0, c->stream));
    EndArgs ea;
    ea.ic = c->d_ic;
    ea.order = nullptr;
    ea.tab = c->d_tab;
    ea.Phi = s5;
    ea.Pi = s5 + c->total;
    ea.wPi = c->d_wPi;
    ea.wPhi = c->d_wPhi;
    ea.Pihat = pl.aT;
    ea.Phihat = pl.bT;
    ea.E0 = pl.E0;
    ea.ET = pl.ET;
    ea.status = c->d_status;
    ea.Ubar = pl.ub;
    ea.total = c->total;
    ea.sgn = 1.0;
    ea.J = J;
    ea.gauge = c->gauge;
    auto run_end = [&]() {
        return run_classes(c, [&](LaunchClass& lc, hipStream_t s) -> hipError_t {
            EndArgs e = ea;
            e.order = lc.d_order;
            return launch_endpoint(lc.cfg, lc.full, (int)lc.inst.size(), e, s);
        });
    };
    if ((rc = run_end())) return rc;

    EvolveArgs ra = evolve_args(c, 0);
    ra.Phi = pl.dummy;
    ra.Pi = pl.dummy + c->total;
    ra.status = pl.rst;
    ra.src = pl.d_ckp;
    ra.src_every = (int32_t)pl.K;
    ra.ckpt = pl.stored ? nullptr : pl.d_segp;
    ra.ckpt_every = pl.stored ? 0 : 1;
    ra.keep = pl.stored ? pl.d_keepp : nullptr;
    AdjointArgs aa;
    aa.ic = c->d_ic;
    aa.order = nullptr;
    aa.tab = c->d_tab;
    aa.seg = pl.d_segp;
    aa.stg = pl.d_stgp;
    aa.keep = pl.stored ? pl.d_keepp : nullptr;
    aa.sg = pl.sgs;
    aa.Ubar = pl.ub;
    aa.total = c->total;
    aa.gauge = c->gauge;
    aa.pad = 0;
    for (int64_t r = 0; r < pl.max_seg; ++r) {
        HIP_TRY(c, launch_adj_prepare(n, c->d_ic, c->d_status, pl.K, r, pl.rst, pl.sgs, c->stream));
        rc = run_classes(c, [&](LaunchClass& lc, hipStream_t s) -> hipError_t {
            EvolveArgs e = ra;
            e.order = lc.d_order;
            hipError_t err = launch_evolve(lc.cfg, lc.full, (int)lc.inst.size(), e, s);
            if (err != hipSuccess) return err;
            AdjointArgs g = aa;
            g.order = lc.d_order;
            return launch_adjoint(lc.cfg, lc.full, (int)lc.inst.size(), g, s);
        });
        if (rc) return rc;
    }
    ea.Phi = pl.u0;
    ea.Pi = pl.u0 + c->total;
    ea.Pihat = pl.a0;
    ea.Phihat = pl.b0;
    ea.sgn = -1.0;
    if ((rc = run_end())) return rc;
    HIP_TRY(c, launch_adj_finish(n, c->d_ic, c->d_status, pl.ub, c->total, c->d_emode, d_eps, Jc, pl.E0, pl.ET, J,
                                 oL, oG, oV, c->stream));
    return ADSCL_OK;
}

int check_adjoint_args(adscl_ctx* c, const double* eps, const double* coef, int32_t Jc, int32_t J, double T,
                       int32_t ckpt_every, int mem)
{
    if (!eps || !coef) return fail(c, ADSCL_EINVAL, "NULL argument");
    if (c->flags & ADSCL_FROZEN_METRIC) return fail(c, ADSCL_EUNSUPPORTED, "adjoint needs the dynamic metric");
    if (scheme(c)) return fail(c, ADSCL_EUNSUPPORTED, "adjoint of classical RK4 with A solved at every stage only");
    if (c->n_big > 0) return fail(c, ADSCL_EUNSUPPORTED, "adjoint supports N <= 4097");
    if (Jc < 1 || Jc > c->n_modes || J < 1 || J > c->n_modes)
        return fail(c, ADSCL_EINVAL, "need 1 <= Jc, J <= n_modes");
    if (!(T >= 0.0) || std::isinf(T)) return fail(c, ADSCL_EINVAL, "T must be finite and >= 0");
    if (ckpt_every < 1) return fail(c, ADSCL_EINVAL, "ckpt_every must be >= 1");
    return check_mem(c, mem);
}

// Device copies of eps [n] and c [n x Jc] in context buffers.
int stage_inputs(adscl_ctx* c, const double* eps, const double* coef, int32_t Jc, int mem, double** d_eps,
                 double** d_c)
{
    void *e, *k;
    int rc;
    const int n = c->n_inst;
    if ((rc = buffer(c, "in_eps", sizeof(double) * n, &e))) return rc;
    if ((rc = buffer(c, "in_c", sizeof(double) * (size_t)n * Jc, &k))) return rc;
    const hipMemcpyKind kind = mem == ADSCL_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    HIP_TRY(c, hipMemcpyAsync(e, eps, sizeof(double) * n, kind, c->stream));
    HIP_TRY(c, hipMemcpyAsync(k, coef, sizeof(double) * (size_t)n * Jc, kind, c->stream));
    *d_eps = (double*)e;
    *d_c = (double*)k;
    return ADSCL_OK;
}

// One tuning trial: a batch of `n_inst` instances of grid size N in
// configuration cfg, weak Gaussian data, `steps` RK4 steps after 8 warm-up
// steps; the rate in pt-steps/s, or a negative adscl error code.
double tune_trial(int N, ClassCfg cfg, int n_inst, int steps, std::string& err)
{
    g_force_N = N;
    g_force = cfg;
    std::vector<int32_t> grid(n_inst, N);
    adscl_config c;
    c.n_inst = n_inst;
    c.n_grid = grid.data();
    c.cfl = 0.25;
    c.ko_sigma = 0.5;
    c.a_collapse = 0.0;
    c.gauge = ADSCL_GAUGE_BOUNDARY;
    c.n_modes = 1;
    c.flags = 0;
    c.rk_order = 4;
    c.a_reint = 0;
    adscl_ctx* ctx = nullptr;
    int rc = adscl_create(&c, nullptr, &ctx);
    g_force_N = 0;
    if (rc) {
        err = adscl_last_error(nullptr);
        return rc;
    }
    std::vector<double> eps(n_inst, 1e-3), sig(n_inst, 0.2);
    hipEvent_t t0 = nullptr, t1 = nullptr;
    float ms = 0.0f;
    double rate = 0.0;
    if ((rc = adscl_init_gaussian(ctx, eps.data(), sig.data(), ADSCL_MEM_HOST)) == 0 &&
        (rc = adscl_step(ctx, 8, 1e300, 0, 0, nullptr, ADSCL_MEM_DEVICE)) == 0 && (rc = adscl_sync(ctx)) == 0) {
        if (hipEventCreate(&t0) != hipSuccess || hipEventCreate(&t1) != hipSuccess ||
            hipEventRecord(t0, ctx->stream) != hipSuccess)
            rc = ADSCL_EHIP;
        if (!rc) rc = adscl_step(ctx, steps, 1e300, 0, 0, nullptr, ADSCL_MEM_DEVICE);
        if (!rc && (hipEventRecord(t1, ctx->stream) != hipSuccess || hipEventSynchronize(t1) != hipSuccess ||
                    hipEventElapsedTime(&ms, t0, t1) != hipSuccess))
            rc = ADSCL_EHIP;
        if (!rc) rate = (double)n_inst * N * steps / (ms * 1e-3);
    }
    if (rc) err = adscl_last_error(ctx) ? adscl_last_error(ctx) : "tuning trial failed";
    if (t0) (void)hipEventDestroy(t0);
    if (t1) (void)hipEventDestroy(t1);
    adscl_destroy(ctx);
    return rc ? (double)rc : rate;
}

}  // namespace

extern "C" {

int adscl_create(const adscl_config* cfg, void* hip_stream, adscl_ctx** out)
{
    if (!out) return fail(nullptr, ADSCL_EINVAL, "out is NULL");
    *out = nullptr;
    if (!cfg || !cfg->n_grid) return fail(nullptr, ADSCL_EINVAL, "config or n_grid is NULL");
    if (cfg->n_inst < 1) return fail(nullptr, ADSCL_EINVAL, "n_inst must be >= 1");
    for (int b = 0; b < cfg->n_inst; ++b) {
        const int N = cfg->n_grid[b];
        if (N < 17 || N > kMaxN || (N % 2) == 0)
            return fail(nullptr, ADSCL_EINVAL,
                        "instance " + std::to_string(b) + ": N=" + std::to_string(N) +
                            " (need odd N, 17 <= N <= 65537)");
    }
    if (!(cfg->cfl > 0.0 && cfg->cfl <= 1.0)) return fail(nullptr, ADSCL_EINVAL, "cfl must be in (0, 1]");
    if (!(cfg->ko_sigma >= 0.0 && cfg->ko_sigma <= 2.0)) return fail(nullptr, ADSCL_EINVAL, "ko_sigma must be in [0, 2]");
    if (!(cfg->a_collapse >= 0.0 && cfg->a_collapse <= 1.0)) return fail(nullptr, ADSCL_EINVAL, "a_collapse must be in [0, 1]");
    if (cfg->gauge != ADSCL_GAUGE_BOUNDARY && cfg->gauge != ADSCL_GAUGE_ORIGIN) return fail(nullptr, ADSCL_EINVAL, "bad gauge");
    if (cfg->n_modes < 0 || cfg->n_modes > 128) return fail(nullptr, ADSCL_EINVAL, "n_modes must be in [0, 128]");
    if (cfg->flags & ~(ADSCL_FROZEN_METRIC | ADSCL_TIME_KERNELS)) return fail(nullptr, ADSCL_EINVAL, "unknown flags");
    if (cfg->rk_order != 0 && cfg->rk_order != 2 && cfg->rk_order != 3 && cfg->rk_order != 4)
        return fail(nullptr, ADSCL_EINVAL, "rk_order must be 0, 2, 3 or 4");
    if (cfg->a_reint < 0) return fail(nullptr, ADSCL_EINVAL, "a_reint must be >= 0");
    if (cfg->a_reint > 0 && (cfg->flags & ADSCL_FROZEN_METRIC))
        return fail(nullptr, ADSCL_EINVAL, "an evolved A (a_reint > 0) needs the dynamic metric");
    const int rk_order = cfg->rk_order == 0 ? 4 : cfg->rk_order;

    adscl_ctx* c = new adscl_ctx();
    c->n_inst = cfg->n_inst;
    c->N.assign(cfg->n_grid, cfg->n_grid + cfg->n_inst);
    c->off.resize(c->n_inst);
    int64_t acc = 0;
    for (int b = 0; b < c->n_inst; ++b) {
        c->off[b] = acc;
        acc += c->N[b];
        c->max_N = std::max<int64_t>(c->max_N, c->N[b]);
    }
    c->total = acc;
    c->cfl = cfg->cfl;
    c->ko = cfg->ko_sigma;
    c->thr = cfg->a_collapse;
    c->gauge = cfg->gauge;
    c->n_modes = cfg->n_modes;
    c->flags = cfg->flags;
    c->rk = rk_order;
    c->a_reint = cfg->a_reint;

    auto bail = [&](int code) {
        g_create_error = c->err;
        adscl_destroy(c);
        return code;
    };
#define TRY_C(call)                                                                               \
    do {                                                                                          \
        hipError_t e_ = (call);                                                                   \
        if (e_ != hipSuccess) {                                                                   \
            c->err = std::string(#call) + ": " + hipGetErrorString(e_);                           \
            return bail(e_ == hipErrorOutOfMemory ? ADSCL_ENOMEM : ADSCL_EHIP);                   \
        }                                                                                         \
    } while (0)

    TRY_C(hipGetDevice(&c->device));
    // address of this device's fixed scratch (adscl_constraints_noalloc), looked
    // up once per device while it is current
    TRY_C(static_scratch_init(c->device));
    int lds = 0;
    TRY_C(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device));
    c->max_lds = (size_t)lds;
    if (hip_stream) {
        c->stream = (hipStream_t)hip_stream;
    } else {
        TRY_C(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
        c->own_stream = true;
    }

    // per-instance constants
    c->h_ic.resize(c->n_inst);
    for (int b = 0; b < c->n_inst; ++b) {
        InstConst& k = c->h_ic[b];
        k.off = c->off[b];
        k.N = c->N[b];
        k.pad = 0;
        k.h = (kPi / 2.0) / (double)(k.N - 1);
        k.dt = c->cfl * k.h;
        k.h24 = k.h / 24.0;
        k.i12h = 1.0 / (12.0 * k.h);
        k.kof = c->ko / (64.0 * k.h);
        k.n_final = 0;
    }

    // classes and tables per distinct N
    std::map<std::pair<int, int>, std::map<bool, int>> class_index;
    for (int b = 0; b < c->n_inst; ++b) {
        const int N = c->N[b];
        if (N > kMaxOneGroup) {
            // a large instance: chunks of one class over several workgroups
            int coop = 0;
            TRY_C(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, c->device));
            if (!coop) {
                c->err = "N=" + std::to_string(N) + " needs cooperative launches";
                return bail(ADSCL_EUNSUPPORTED);
            }
            const ClassCfg cfg = choose_big_class(N);
            const int C = 64 * cfg.W * cfg.P;
            const int G = (N - 1 + C - 1) / C;
            const int rem = (N - 1) - (G - 1) * C;
            if (G > kBigMaxChunks || rem < 8 || big_lds_bytes(cfg) > c->max_lds) {
                c->err = "N=" + std::to_string(N) + ": no chunk configuration (chunks of " + std::to_string(C) +
                         " points leave " + std::to_string(rem) + " in the last)";
                return bail(ADSCL_EUNSUPPORTED);
            }
            if (!c->tables.count(N)) {
                NTables t;
                t.cfg = cfg;
                TRY_C(prepare_evolve_big(cfg, c->rk, c->a_reint > 0, c->max_lds));
                std::vector<double> tab, e, wpi, wphi;
                host_tables(N, cfg, tab, G);
                TRY_C(hipMalloc((void**)&t.d_tab, tab.size() * sizeof(double)));
                TRY_C(hipMemcpy(t.d_tab, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice));
                if (c->n_modes > 0) {
                    host_modes(N, c->n_modes, e, wpi, wphi);
                    const size_t bytes = e.size() * sizeof(double);
                    TRY_C(hipMalloc((void**)&t.d_emode, bytes));
                    TRY_C(hipMalloc((void**)&t.d_wPi, bytes));
                    TRY_C(hipMalloc((void**)&t.d_wPhi, bytes));
                    TRY_C(hipMemcpy(t.d_emode, e.data(), bytes, hipMemcpyHostToDevice));
                    TRY_C(hipMemcpy(t.d_wPi, wpi.data(), bytes, hipMemcpyHostToDevice));
                    TRY_C(hipMemcpy(t.d_wPhi, wphi.data(), bytes, hipMemcpyHostToDevice));
                }
                c->tables[N] = t;
            }
            LaunchClass lc;
            lc.cfg = cfg;
            lc.full = false;
            lc.chunks = G;
            lc.inst.push_back(b);
            c->classes.push_back(lc);
            continue;
        }
        if (!c->tables.count(N)) {
            NTables t;
            t.cfg = scheme(c) ? default_class(N) : choose_class(N);
            if (t.cfg.P == 0) {
                c->err = "no kernel configuration for N=" + std::to_string(N);
                return bail(ADSCL_EUNSUPPORTED);
            }
            if (evolve_lds_bytes(t.cfg) > c->max_lds) {
                c->err = "N=" + std::to_string(N) + " needs " + std::to_string(evolve_lds_bytes(t.cfg)) +
                         " B of LDS, device allows " + std::to_string(c->max_lds);
                return bail(ADSCL_EUNSUPPORTED);
            }
            if (scheme(c)) TRY_C(prepare_evolve_scheme(t.cfg, c->rk, c->a_reint > 0, c->max_lds));
            else TRY_C(prepare_evolve(t.cfg, c->max_lds));
            TRY_C(prepare_adjoint(t.cfg, c->max_lds));
            std::vector<double> tab, e, wpi, wphi;
            host_tables(N, t.cfg, tab);
            TRY_C(hipMalloc((void**)&t.d_tab, tab.size() * sizeof(double)));
            TRY_C(hipMemcpy(t.d_tab, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice));
            if (c->n_modes > 0) {
                host_modes(N, c->n_modes, e, wpi, wphi);
                const size_t bytes = e.size() * sizeof(double);
                TRY_C(hipMalloc((void**)&t.d_emode, bytes));
                TRY_C(hipMalloc((void**)&t.d_wPi, bytes));
                TRY_C(hipMalloc((void**)&t.d_wPhi, bytes));
                TRY_C(hipMemcpy(t.d_emode, e.data(), bytes, hipMemcpyHostToDevice));
                TRY_C(hipMemcpy(t.d_wPi, wpi.data(), bytes, hipMemcpyHostToDevice));
                TRY_C(hipMemcpy(t.d_wPhi, wphi.data(), bytes, hipMemcpyHostToDevice));
            }
            c->tables[N] = t;
        }
        const NTables& t = c->tables[N];
        const bool full = (64 * t.cfg.W * t.cfg.P == N - 1);
        auto key = std::make_pair(t.cfg.P, t.cfg.W);
        if (!class_index[key].count(full)) {
            LaunchClass lc;
            lc.cfg = t.cfg;
            lc.full = full;
            class_index[key][full] = (int)c->classes.size();
            c->classes.push_back(lc);
        }
        c->classes[class_index[key][full]].inst.push_back(b);
    }
    // within a class, larger N first (longest-processing-time order)
    for (LaunchClass& lc : c->classes) {
        std::stable_sort(lc.inst.begin(), lc.inst.end(), [&](int x, int y) { return c->N[x] > c->N[y]; });
        TRY_C(hipMalloc((void**)&lc.d_order, lc.inst.size() * sizeof(int32_t)));
        TRY_C(hipMemcpy(lc.d_order, lc.inst.data(), lc.inst.size() * sizeof(int32_t), hipMemcpyHostToDevice));
        if (c->classes.size() > 1 && lc.chunks == 0) {
            TRY_C(hipStreamCreateWithFlags(&lc.stream, hipStreamNonBlocking));
            TRY_C(hipEventCreateWithFlags(&lc.done, hipEventDisableTiming));
        }
        if (c->flags & ADSCL_TIME_KERNELS) {
            TRY_C(hipEventCreate(&lc.t0));
            TRY_C(hipEventCreate(&lc.t1));
        }
    }
    if (c->classes.size() > 1) TRY_C(hipEventCreateWithFlags(&c->fork, hipEventDisableTiming));
    // one-workgroup classes by lane capacity, largest first (their launch
    // order); large instances are listed last, but run_evolve launches them
    // first, all in one cooperative launch per chunk configuration on the
    // context stream (several when the device cannot hold their workgroups
    // at once), before it forks the one-workgroup classes onto their streams:
    // the two never overlap
    std::stable_sort(c->classes.begin(), c->classes.end(), [](const LaunchClass& x, const LaunchClass& y) {
        if ((x.chunks > 0) != (y.chunks > 0)) return y.chunks > 0;
        return 64 * x.cfg.W * x.cfg.P > 64 * y.cfg.W * y.cfg.P;
    });
    c->n_big = 0;
    for (const LaunchClass& lc : c->classes) c->n_big += lc.chunks > 0;
    // Pair launches (plain RK4 only; after the sort, which fixes the class
    // indices that `pair` and `host` hold): a full (P, W) class also runs a full
    // (P, W/2) class's instances two per workgroup in its own launch, after its
    // own instances in dispatch order, so that they start on the compute units
    // its instances free instead of after its whole launch.  Opt-in
    // (ADSCL_PAIR=1): on the 1024-instance Gaussian workload the pass took
    // longer this way than with every class in a launch of its own.
    const char* pair_env = std::getenv("ADSCL_PAIR");
    if (!scheme(c) && pair_env && std::strcmp(pair_env, "1") == 0) {
        for (int x = 0; x < (int)c->classes.size(); ++x) {
            LaunchClass& X = c->classes[x];
            if (X.chunks || !X.full || X.host >= 0 || !pair_supported(X.cfg)) continue;
            for (int y = 0; y < (int)c->classes.size(); ++y) {
                LaunchClass& Y = c->classes[y];
                if (y == x || Y.chunks || !Y.full || Y.pair >= 0 || Y.host >= 0) continue;
                if (Y.cfg.P != X.cfg.P || 2 * Y.cfg.W != X.cfg.W) continue;
                TRY_C(prepare_evolve_pair(X.cfg, c->max_lds));
                std::vector<int32_t> ord = X.inst;
                ord.insert(ord.end(), Y.inst.begin(), Y.inst.end());
                TRY_C(hipMalloc((void**)&X.d_order_pair, ord.size() * sizeof(int32_t)));
                TRY_C(hipMemcpy(X.d_order_pair, ord.data(), ord.size() * sizeof(int32_t), hipMemcpyHostToDevice));
                X.pair = y;
                Y.host = x;
                break;
            }
        }
    }
    // large instances: one cooperative launch per configuration, split where
    // the device cannot hold all their workgroups at once
    for (int k = 0; k < (int)c->classes.size(); ++k) {
        const LaunchClass& lc = c->classes[k];
        if (lc.chunks == 0) continue;
        int cap = 0;
        TRY_C(big_capacity(lc.cfg, c->rk, c->a_reint > 0, c->device, &cap));
        if (lc.chunks > cap) {
            c->err = "N=" + std::to_string(c->N[lc.inst[0]]) + " needs " + std::to_string(lc.chunks) +
                     " workgroups at once, the device holds " + std::to_string(cap);
            return bail(ADSCL_EUNSUPPORTED);
        }
        BigGroup* g = nullptr;
        for (BigGroup& x : c->big_groups)
            if (x.cfg.P == lc.cfg.P && x.cfg.W == lc.cfg.W && x.blocks + lc.chunks <= cap && x.cls.size() < 1024)
                g = &x;
        if (!g) {
            c->big_groups.emplace_back();
            g = &c->big_groups.back();
            g->cfg = lc.cfg;
        }
        g->cls.push_back(k);
        g->blocks += lc.chunks;
    }
    for (BigGroup& g : c->big_groups) {
        std::vector<BigDesc> desc;
        int first = 0;
        for (int k : g.cls) {
            const LaunchClass& lc = c->classes[k];
            BigDesc d;
            d.inst = lc.inst[0];
            d.chunks = lc.chunks;
            d.first = first;
            d.pad = 0;
            desc.push_back(d);
            first += lc.chunks;
        }
        TRY_C(hipMalloc((void**)&g.d_desc, sizeof(BigDesc) * desc.size()));
        TRY_C(hipMemcpy(g.d_desc, desc.data(), sizeof(BigDesc) * desc.size(), hipMemcpyHostToDevice));
        TRY_C(hipMalloc((void**)&g.xch, sizeof(double) * 32 * (size_t)g.blocks));
        TRY_C(hipMalloc((void**)&g.ctr, sizeof(unsigned long long) * kBigCtrStride * desc.size()));
        TRY_C(hipMemset(g.ctr, 0, sizeof(unsigned long long) * kBigCtrStride * desc.size()));
    }

    std::vector<const double*> tabp(c->n_inst), ep(c->n_inst), wpp(c->n_inst), wfp(c->n_inst);
    for (int b = 0; b < c->n_inst; ++b) {
        const NTables& t = c->tables[c->N[b]];
        tabp[b] = t.d_tab;
        ep[b] = t.d_emode;
        wpp[b] = t.d_wPi;
        wfp[b] = t.d_wPhi;
    }
    const size_t pb = sizeof(double*) * c->n_inst;
    TRY_C(hipMalloc((void**)&c->d_tab, pb));
    TRY_C(hipMalloc((void**)&c->d_emode, pb));
    TRY_C(hipMalloc((void**)&c->d_wPi, pb));
    TRY_C(hipMalloc((void**)&c->d_wPhi, pb));
    TRY_C(hipMemcpy(c->d_tab, tabp.data(), pb, hipMemcpyHostToDevice));
    TRY_C(hipMemcpy(c->d_emode, ep.data(), pb, hipMemcpyHostToDevice));
    TRY_C(hipMemcpy(c->d_wPi, wpp.data(), pb, hipMemcpyHostToDevice));
    TRY_C(hipMemcpy(c->d_wPhi, wfp.data(), pb, hipMemcpyHostToDevice));

    TRY_C(hipMalloc((void**)&c->state5, sizeof(double) * 5 * (size_t)c->total));
    TRY_C(hipMemset(c->state5, 0, sizeof(double) * 5 * (size_t)c->total));
    TRY_C(hipMalloc((void**)&c->d_status, sizeof(InstStatus) * c->n_inst));
    TRY_C(hipMalloc((void**)&c->d_ic, sizeof(InstConst) * c->n_inst));
    TRY_C(hipMemcpy(c->d_ic, c->h_ic.data(), sizeof(InstConst) * c->n_inst, hipMemcpyHostToDevice));
    if (ensure_tmp(c, sizeof(double) * (size_t)std::max<int64_t>(2 * c->total, 130 * (int64_t)c->n_inst))) {
        return bail(ADSCL_ENOMEM);
    }
#undef TRY_C
    *out = c;
    return ADSCL_OK;
}

void adscl_destroy(adscl_ctx* c)
{
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    for (BigGroup& g : c->big_groups) {
        if (g.d_desc) (void)hipFree(g.d_desc);
        if (g.xch) (void)hipFree(g.xch);
        if (g.ctr) (void)hipFree(g.ctr);
    }
    for (LaunchClass& lc : c->classes) {
        if (lc.d_order) (void)hipFree(lc.d_order);
        if (lc.d_order_pair) (void)hipFree(lc.d_order_pair);
        if (lc.stream) (void)hipStreamDestroy(lc.stream);
        if (lc.done) (void)hipEventDestroy(lc.done);
        if (lc.t0) (void)hipEventDestroy(lc.t0);
        if (lc.t1) (void)hipEventDestroy(lc.t1);
    }
    for (auto& kv : c->tables) {
        if (kv.second.d_tab) (void)hipFree(kv.second.d_tab);
        if (kv.second.d_emode) (void)hipFree(kv.second.d_emode);
        if (kv.second.d_wPi) (void)hipFree(kv.second.d_wPi);
        if (kv.second.d_wPhi) (void)hipFree(kv.second.d_wPhi);
    }
    if (c->d_tab) (void)hipFree((void*)c->d_tab);
    if (c->d_emode) (void)hipFree((void*)c->d_emode);
    if (c->d_wPi) (void)hipFree((void*)c->d_wPi);
    if (c->d_wPhi) (void)hipFree((void*)c->d_wPhi);
    if (c->state5) (void)hipFree(c->state5);
    if (c->d_status) (void)hipFree(c->d_status);
    if (c->d_ic) (void)hipFree(c->d_ic);
    if (c->d_tmp) (void)hipFree(c->d_tmp);
    if (c->fork) (void)hipEventDestroy(c->fork);
    for (auto& kv : c->bufs)
        if (kv.second.first) (void)hipFree(kv.second.first);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

int adscl_init(adscl_ctx* c, const double* Phi0, const double* Pi0, int mem)
{
    if (!c) return fail(nullptr, ADSCL_EINVAL, "ctx is NULL");
    if (!Phi0 || !Pi0) return fail(c, ADSCL_EINVAL, "Phi0 / Pi0 is NULL");
    if (int rc = check_mem(c, mem)) return rc;
    const hipMemcpyKind kind = mem == ADSCL_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    const size_t bytes = sizeof(double) * (size_t)c->total;
    HIP_TRY(c, hipMemcpyAsync(c->state5, Phi0, bytes, kind, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->state5 + c->total, Pi0, bytes, kind, c->stream));
    return after_init(c);
}

int adscl_init_gaussian(adscl_ctx* c, const double* eps, const double* sigma, int mem)
{
    if (!c) return fail(nullptr, ADSCL_EINVAL, "ctx is NULL");
    if (!eps || !sigma) return fail(c, ADSCL_EINVAL, "eps / sigma is NULL");
    if (int rc = check_mem(c, mem)) return rc;
    const double *de, *ds;
    if (int rc = stage_in(c, eps, c->n_inst, mem, 0, &de)) return rc;
    if (int rc = stage_in(c, sigma, c->n_inst, mem, c->n_inst, &ds)) return rc;
    HIP_TRY(c, launch_init_gaussian(c->n_inst, c->d_ic, de, ds, c->state5, c->state5 + c->total, c->max_N,
                                    c->stream));
    return after_init(c);
}

int adscl_init_modes(adscl_ctx* c, const double* eps, const double* coef, int32_t Jc, int mem)
{
    if (!c) return fail(nullptr, ADSCL_EINVAL, "ctx is NULL");
    if (!eps || !coef) return fail(c, ADSCL_EINVAL, "eps / c is NULL");
    if (Jc < 1 || Jc > c->n_modes) return fail(c, ADSCL_EINVAL, "need 1 <= Jc <= n_modes");
    if (int rc = check_mem(c, mem)) return rc;
    const double *de, *dc;
    if (int rc = stage_in(c, eps, c->n_inst, mem, 0, &de)) return rc;
    if (int rc = stage_in(c, coef, (size_t)c->n_inst * Jc, mem, c->n_inst, &dc)) return rc;
    HIP_TRY(c, launch_init_modes(c->n_inst, c->d_ic, de, dc, Jc, c->d_emode, c->state5, c->state5 + c->total,
                                 c->max_N, c->stream));
    return after_init(c);
}

int adscl_step(adscl_ctx* c, int64_t max_steps, double t_end, int32_t snap_every, int32_t n_snap_slots,
               double* snaps, int mem)
{
    if (!c) return fail(nullptr, ADSCL_EINVAL, "ctx is NULL");
    if (!c->initialized) return fail(c, ADSCL_ESTATE, "adscl_step before any adscl_init*");
    if (max_steps < 0) return fail(c, ADSCL_EINVAL, "max_steps must be >= 0");
    if (!(t_end >= 0.0) || std::isinf(t_end)) return fail(c, ADSCL_EINVAL, "t_end must be finite and >= 0");
    if (snap_every < 0 || n_snap_slots < 0) return fail(c, ADSCL_EINVAL, "snap_every / n_snap_slots < 0");
    if (snap_every > 0 && n_snap_slots > 0 && !snaps) return fail(c, ADSCL_EINVAL, "snaps is NULL");
    if (int rc = check_mem(c, mem)) return rc;
    const bool want = snap_every > 0 && n_snap_slots > 0;
    double* dsn = nullptr;
    const size_t snap_bytes = want ? sizeof(double) * 5 * (size_t)c->total * n_snap_slots : 0;
    if (want) {
        if (mem == ADSCL_MEM_DEVICE) {
            dsn = snaps;
        } else {
            HIP_TRY(c, hipStreamSynchronize(c->stream));
            HIP_TRY(c, hipMalloc((void**)&dsn, snap_bytes));
            HIP_TRY(c, hipMemcpy(dsn, snaps, snap_bytes, hipMemcpyHostToDevice));
        }
    }
    int rc = run_call(c, max_steps, t_end, want ? snap_every : 0, want ? n_snap_slots : 0, dsn);
    if (rc == ADSCL_OK && c->n_big > 0) rc = check_big(c);
    if (want && mem == ADSCL_MEM_HOST) {
        if (rc == ADSCL_OK) {
            hipError_t e = hipMemcpyAsync(snaps, dsn, snap_bytes, hipMemcpyDeviceToHost, c->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
            if (e != hipSuccess) rc = fail(c, ADSCL_EHIP, std::string("snapshot copy: ") + hipGetErrorString(e));
        }
        (void)hipFree(dsn);
    }
    return rc;
}

int adscl_get_state(adscl_ctx* c, double* Phi, double* Pi, double* A, double* delta, double* m, int mem)
{
    if (!c) return fail(nullptr, ADSCL_EINVAL, "ctx is NULL");
    if (!c->initialized) return fail(c, ADSCL_ESTATE, "adscl_get_state before any adscl_init*");
    if (int rc = check_mem(c, mem)) return rc;
    const hipMemcpyKind kind = mem == ADSCL_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    double* outs[5] = {Phi, Pi, A, delta, m};
    const size_t bytes = sizeof(double) * (size_t)c->total;
    for (int f = 0; f < 5; ++f)
        if (outs[f]) HIP_TRY(c, hipMemcpyAsync(outs[f], c->state5 + f * c->total, bytes, kind, c->stream));
    if (mem == ADSCL_MEM_HOST) HIP_TRY(c, hipStreamSynchronize(c->stream));
    return ADSCL_OK;
}

int adscl_status(adscl_ctx* c, double* t, int64_t* steps, int32_t* state, double* t_collapse, double* minA)
{
    if (!c) return fail(nullptr, ADSCL_EINVAL, "ctx is NULL");
    if (!c->initialized) return fail(c, ADSCL_ESTATE, "adscl_status before any adscl_init*");
    std::vector<InstStatus> st(c->n_inst);
    HIP_TRY(c, hipMemcpyAsync(st.data(), c->d_status, sizeof(InstStatus) * c->n_inst, hipMemcpyDeviceToHost,
                              c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (int b = 0; b < c->n_inst; ++b) {
        if (t) t[b] = (double)st[b].steps * c->h_ic[b].dt;
        if (steps) steps[b] = st[b].steps;
        if (state) state[b] = st[b].state;
        if (t_collapse) t_collapse[b] = st[b].t_c;
        if (minA) minA[b] = st[b].minA;
    }
    return ADSCL_OK;
}

// The diagnostics of adscl_constraints with `scr` (2 * total + 5 * n_inst
// doubles of device memory) as the residual kernel's scratch and the staging of
// host outputs.
static int constraints_call(adscl_ctx* c, double* scr, double* out, int mem)
{
    double* dst = mem == ADSCL_MEM_DEVICE ? out : scr + 2 * c->total;
    const double* s = c->state5;
    HIP_TRY(c, launch_diagnostics(c->n_inst, c->d_ic, s, s + c->total, s + 2 * c->total, s + 3 * c->total,
                                  s + 4 * c->total, dst, c->stream));
    const int frozen = (c->flags & ADSCL_FROZEN_METRIC) ? 1 : 0;
    HIP_TRY(c, launch_adot_residual(c->n_inst, c->d_ic, s, c->total, frozen, c->ko, scr, dst, c->stream));
    if (mem == ADSCL_MEM_HOST) {
        HIP_TRY(c, hipMemcpyAsync(out, dst, sizeof(double) * 5 * c->n_inst, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
    }
    return ADSCL_OK;
}

static int constraints_check(adscl_ctx* c, const double* out, int mem)
{
    if (!c) return fail(nullptr, ADSCL_EINVAL, "ctx is NULL");
    if (!c->initialized) return fail(c, ADSCL_ESTATE, "adscl_constraints before any adscl_init*");
    if (!out) return fail(c, ADSCL_EINVAL, "out is NULL");
    return check_mem(c, mem);
}

int adscl_constraints(adscl_ctx* c, double* out, int mem)
{
    if (int rc = constraints_check(c, out, mem)) return rc;
    void* scr;
    if (int rc = buffer(c, "constraints", sizeof(double) * (2 * (size_t)c->total + 5 * (size_t)c->n_inst), &scr))
        return rc;
    return constraints_call(c, (double*)scr, out, mem);
}

int adscl_constraints_noalloc(adscl_ctx* c, double* out, int mem)
{
    if (int rc = constraints_check(c, out, mem)) return rc;
    const size_t need = 2 * (size_t)c->total + 5 * (size_t)c->n_inst;
    if (need > kStaticScratchDoubles)
        return fail(c, ADSCL_EINVAL,
                    "adscl_constraints_noalloc: 2 * sum N_b + 5 * n_inst = " + std::to_string(need) +
                        " exceeds the fixed scratch of " + std::to_string(kStaticScratchDoubles) + " doubles");
    double* scr = static_scratch(c->device);
    if (!scr) return fail(c, ADSCL_ESTATE, "adscl_constraints_noalloc: no fixed scratch on this device");
    return constraints_call(c, scr, out, mem);
}

// Spectra of n_slots states at `base` ([slot][5][total] on the device) into
// E, Pihat, Phihat ([n_slots][n_inst][J], host or device per mem).
static int spectrum_call(adscl_ctx* c, const double* base, int n_slots, int32_t J, double* E, double* Pihat, double* Phihat,
                  int mem)
{
    int rc;
    if ((rc = spec_rows(c, n_slots))) return rc;
    const size_t n = (size_t)n_slots * c->n_inst * J;
    double *dE = E, *dP = Pihat, *dF = Phihat;
    if (mem == ADSCL_MEM_HOST) {
        void* t;
        if ((rc = buffer(c, "spec_out", 3 * n * sizeof(double), &t))) return rc;
        dE = E ? (double*)t : nullptr;
        dP = Pihat ? (double*)t + n : nullptr;
        dF = Phihat ? (double*)t + 2 * n : nullptr;
    }
    if ((rc = run_spectrum(c, base, J, dE, dP, dF))) return rc;
    if (mem == ADSCL_MEM_HOST) {
        if (E) HIP_TRY(c, hipMemcpyAsync(E, dE, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        if (Pihat) HIP_TRY(c, hipMemcpyAsync(Pihat, dP, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        if (Phihat) HIP_TRY(c, hipMemcpyAsync(Phihat, dF, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
    }
    return ADSCL_OK;
}

int adscl_spectrum(adscl_ctx* c, int32_t J, double* E, double* Pihat, double* Phihat, int mem)
{
    if (!c) return fail(nullptr, ADSCL_EINVAL, "ctx is NULL");
    if (!c->initialized) return fail(c, ADSCL_ESTATE, "adscl_spectrum before any adscl_init*");
    if (J < 1 || J > c->n_modes) return fail(c, ADSCL_EINVAL, "need 1 <= J <= n_modes");
    if (int rc = check_mem(c, mem)) return rc;
    return spectrum_call(c, c->state5, 1, J, E, Pihat, Phihat, mem);
}

int adscl_spectrum_snaps(adscl_ctx* c, int32_t J, int32_t n_slots, const double* snaps, double* E, double* Pihat,
                         double* Phihat, int mem)
{
    if (!c) return fail(nullptr, ADSCL_EINVAL, "ctx is NULL");
    if (J < 1 || J > c->n_modes) return fail(c, ADSCL_EINVAL, "need 1 <= J <= n_modes");
    if (n_slots < 1 || !snaps) return fail(c, ADSCL_EINVAL, "need n_slots >= 1 and snaps");
    if (int rc = check_mem(c, mem)) return rc;
    const double* base = snaps;
    if (mem == ADSCL_MEM_HOST) {
        void* t;
        const size_t bytes = sizeof(double) * 5 * (size_t)c->total * n_slots;
        if (int rc = buffer(c, "snaps_in", bytes, &t)) return rc;
        HIP_TRY(c, hipMemcpyAsync(t, snaps, bytes, hipMemcpyHostToDevice, c->stream));
        base = (const double*)t;
    }
    return spectrum_call(c, base, n_slots, J, E, Pihat, Phihat, mem);
}

int adscl_adjoint(adscl_ctx* c, const double* eps, const double* coef, int32_t Jc, int32_t J, double T,
                  int32_t ckpt_every, double* L, double* dLdc, int32_t* valid, int mem)
{
    if (!c) return fail(nullptr, ADSCL_EINVAL, "ctx is NULL");
    if (!L || !dLdc || !valid) return fail(c, ADSCL_EINVAL, "NULL output");
    int rc = check_adjoint_args(c, eps, coef, Jc, J, T, ckpt_every, mem);
    if (rc) return rc;
    const int n = c->n_inst;
    double *d_eps, *d_c;
    if ((rc = stage_inputs(c, eps, coef, Jc, mem, &d_eps, &d_c))) return rc;
    AdjPlan pl;
    if ((rc = adj_plan(c, T, ckpt_every, J, pl))) return rc;
    void* outs;
    if ((rc = buffer(c, "outs", sizeof(double) * ((size_t)n * Jc + 2 * n), &outs))) return rc;
    double* oL = (double*)outs;
    double* oG = oL + n;
    int32_t* oV = (int32_t*)(oG + (size_t)n * Jc);
    if (mem == ADSCL_MEM_DEVICE) {
        oL = L;
        oG = dLdc;
        oV = valid;
    }
    if ((rc = adj_enqueue(c, pl, d_eps, d_c, Jc, nullptr, true, oL, oG, oV))) return rc;
    c->initialized = true;
    if (mem == ADSCL_MEM_HOST) {
        HIP_TRY(c, hipMemcpyAsync(L, oL, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipMemcpyAsync(dLdc, oG, sizeof(double) * n * Jc, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipMemcpyAsync(valid, oV, sizeof(int32_t) * n, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
    }
    return ADSCL_OK;
}

int adscl_descend(adscl_ctx* c, const double* eps, double* coef, int32_t Jc, int32_t J, double T,
                  int32_t ckpt_every, int32_t iters, double step0, int32_t flags, double* L_hist, int32_t* active,
                  int mem)
{
    if (!c) return fail(nullptr, ADSCL_EINVAL, "ctx is NULL");
    if (!L_hist || !active) return fail(c, ADSCL_EINVAL, "NULL output");
    int rc = check_adjoint_args(c, eps, coef, Jc, J, T, ckpt_every, mem);
    if (rc) return rc;
    if (iters < 1) return fail(c, ADSCL_EINVAL, "iters must be >= 1");
    if (!(step0 > 0.0) || std::isinf(step0)) return fail(c, ADSCL_EINVAL, "step0 must be finite and > 0");
    if (flags & ~ADSCL_DESCEND_EAGER) return fail(c, ADSCL_EINVAL, "unknown flags");
    const int n = c->n_inst;
    double *d_eps, *d_c;
    if ((rc = stage_inputs(c, eps, coef, Jc, mem, &d_eps, &d_c))) return rc;
    AdjPlan pl;
    if ((rc = adj_plan(c, T, ckpt_every, J, pl))) return rc;
    void *g, *lv, *vv, *st, *act, *it, *hist;
    if ((rc = buffer(c, "gd_grad", sizeof(double) * (size_t)n * Jc, &g))) return rc;
    if ((rc = buffer(c, "gd_L", sizeof(double) * n, &lv))) return rc;
    if ((rc = buffer(c, "gd_valid", sizeof(int32_t) * n, &vv))) return rc;
    if ((rc = buffer(c, "gd_state", sizeof(double) * 2 * n, &st))) return rc;
    if ((rc = buffer(c, "gd_active", sizeof(int32_t) * n, &act))) return rc;
    if ((rc = buffer(c, "gd_iter", sizeof(int32_t), &it))) return rc;
    if ((rc = buffer(c, "gd_hist", sizeof(double) * (size_t)iters * n, &hist))) return rc;
    GdState gs;
    gs.s = (double*)st;
    gs.Lprev = (double*)st + n;
    gs.active = (int32_t*)act;
    gs.iter = (int32_t*)it;
    HIP_TRY(c, launch_gd_init(n, step0, gs, c->stream));
    auto one_iteration = [&](bool timing) -> int {
        int r = adj_enqueue(c, pl, d_eps, d_c, Jc, gs.active, timing, (double*)lv, (double*)g, (int32_t*)vv);
        if (r) return r;
        HIP_TRY(c, launch_gd_update(n, Jc, d_c, (const double*)g, (const double*)lv, (const int32_t*)vv, gs,
                                    (double*)hist, c->stream));
        return ADSCL_OK;
    };
    if (flags & ADSCL_DESCEND_EAGER) {
        for (int i = 0; i < iters; ++i)
            if ((rc = one_iteration(true))) return rc;
    } else {
        // one iteration captured once, replayed `iters` times
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        HIP_TRY(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed));
        rc = one_iteration(false);
        hipError_t e = hipStreamEndCapture(c->stream, &graph);
        if (rc) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc;
        }
        if (e != hipSuccess) return fail(c, ADSCL_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(graph);
            return fail(c, ADSCL_EHIP, std::string("graph instantiate: ") + hipGetErrorString(e));
        }
        for (int i = 0; i < iters && e == hipSuccess; ++i) e = hipGraphLaunch(exec, c->stream);
        hipError_t e2 = hipStreamSynchronize(c->stream);
        (void)hipGraphExecDestroy(exec);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess || e2 != hipSuccess)
            return fail(c, ADSCL_EHIP, std::string("graph launch: ") + hipGetErrorString(e != hipSuccess ? e : e2));
    }
    c->initialized = true;
    const hipMemcpyKind kind = mem == ADSCL_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    HIP_TRY(c, hipMemcpyAsync(coef, d_c, sizeof(double) * (size_t)n * Jc, kind, c->stream));
    HIP_TRY(c, hipMemcpyAsync(L_hist, hist, sizeof(double) * (size_t)iters * n, kind, c->stream));
    HIP_TRY(c, hipMemcpyAsync(active, act, sizeof(int32_t) * n, kind, c->stream));
    if (mem == ADSCL_MEM_HOST) HIP_TRY(c, hipStreamSynchronize(c->stream));
    return ADSCL_OK;
}

int adscl_sync(adscl_ctx* c)
{
    if (!c) return fail(nullptr, ADSCL_EINVAL, "ctx is NULL");
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return ADSCL_OK;
}

int adscl_kernel_stats(adscl_ctx* c, int32_t max_classes, int32_t* n_classes, int32_t* P, int32_t* W,
                       int32_t* members, double* last_ms, int32_t* cls)
{
    if (!c) return fail(nullptr, ADSCL_EINVAL, "ctx is NULL");
    if (max_classes < 0) return fail(c, ADSCL_EINVAL, "max_classes < 0");
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    const int nc = (int)c->classes.size();
    if (n_classes) *n_classes = nc;
    for (int k = 0; k < nc && k < max_classes; ++k) {
        LaunchClass& lc = c->classes[k];
        if (P) P[k] = lc.cfg.P;
        if (W) W[k] = lc.cfg.W;
        if (members) members[k] = (int32_t)lc.inst.size();
        if (last_ms) {
            float ms = -1.0f;
            if (lc.t0 && lc.timed) HIP_TRY(c, hipEventElapsedTime(&ms, lc.t0, lc.t1));
            last_ms[k] = ms;
        }
        if (cls)
            for (int32_t b : lc.inst) cls[b] = lc.host >= 0 ? lc.host : k;
    }
    return ADSCL_OK;
}

int adscl_layout(const adscl_ctx* c, int64_t* off, int64_t* total)
{
    if (!c) return fail(nullptr, ADSCL_EINVAL, "ctx is NULL");
    if (off) std::memcpy(off, c->off.data(), sizeof(int64_t) * c->n_inst);
    if (total) *total = c->total;
    return ADSCL_OK;
}

int adscl_autotune(const int32_t* n_grid, int32_t n, int32_t steps, int32_t apply, int32_t* P, int32_t* W,
                   double* rate)
{
    if (!n_grid || n < 1) return fail(nullptr, ADSCL_EINVAL, "autotune: n_grid is NULL or n < 1");
    if (steps < 1) return fail(nullptr, ADSCL_EINVAL, "autotune: steps < 1");
    for (int i = 0; i < n; ++i) {
        const int N = n_grid[i];
        if (N < 17 || N > kMaxOneGroup || (N % 2) == 0)
            return fail(nullptr, ADSCL_EINVAL,
                        "autotune: N=" + std::to_string(N) + " (need odd N, 17 <= N <= 4097)");
    }
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return fail(nullptr, ADSCL_EHIP, std::string("autotune: ") + hipGetErrorString(e));
    const int n_inst = 4 * std::max(cus, 1);
    for (int i = 0; i < n; ++i) {
        const int N = n_grid[i];
        // the tightest capacity level that holds the grid
        int cap = 0;
        for (const ClassCfg& c : kAllClasses) {
            const int k = 64 * c.W * c.P;
            if (k >= N - 1 && (cap == 0 || k < cap)) cap = k;
        }
        ClassCfg best{0, 0};
        double best_rate = -1.0;
        std::string err;
        for (const ClassCfg& c : kAllClasses) {
            if (64 * c.W * c.P != cap) continue;
            const double r = tune_trial(N, c, n_inst, steps, err);
            if (r > best_rate) {
                best_rate = r;
                best = c;
            }
        }
        if (best_rate <= 0.0)
            return fail(nullptr, (int)best_rate < 0 ? (int)best_rate : ADSCL_EHIP, "autotune N=" +
                        std::to_string(N) + ": no configuration ran (" + err + ")");
        if (P) P[i] = best.P;
        if (W) W[i] = best.W;
        if (rate) rate[i] = best_rate;
        if (apply) {
            std::lock_guard<std::mutex> lock(g_tune_mu);
            g_tuned[N] = best;
        }
    }
    return ADSCL_OK;
}

void adscl_autotune_clear(void)
{
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tuned.clear();
}

const char* adscl_last_error(const adscl_ctx* c)
{
    return c ? c->err.c_str() : g_create_error.c_str();
}

}  // extern "C"
