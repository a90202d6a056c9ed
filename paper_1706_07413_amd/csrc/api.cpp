// C-ABI layer and host runtime of the adscl library: context, packed ragged
// batch layout, per-N coefficient and mode tables, per-class launch plan.
// Declarations and the meaning of every call are in include/adscl.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../include/adscl.h"
#include "internal.h"

using namespace adscl;

namespace {

thread_local std::string g_create_error;

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

// Kernel configuration for grid size N: the smallest lane capacity 64 W P that
// holds the N-1 evolved points.  ADSCL_TUNE="N:PxW,..." overrides per N.
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
    static const ClassCfg pref[] = {{4, 1}, {4, 2}, {4, 4}, {4, 8}, {8, 8}};
    for (const ClassCfg& c : pref)
        if (64 * c.W * c.P >= N - 1) return c;
    return ClassCfg{0, 0};
}

// sin, cos in long double for the tables (the kernel reads FP64 values).
void host_tables(int N, ClassCfg cfg, std::vector<double>& tab)
{
    const int NL = 64 * cfg.W, P = cfg.P;
    tab.assign(table_len(cfg), 0.0);
    const long double h = (3.14159265358979323846264338327950288L / 2.0L) / (long double)(N - 1);
    for (int lane = 0; lane < NL; ++lane) {
        for (int k = 0; k < P; ++k) {
            const int i = lane * P + k;
            double sc = 0.0, t2 = 0.0, ct2 = 0.0;
            if (i >= 1 && i <= N - 2) {
                const long double x = h * (long double)i;
                const long double s = sinl(x), c = cosl(x);
                sc = (double)(s * c);
                t2 = (double)((s * s) / (c * c));
                ct2 = (double)((c * c) / (s * s));
            }
            tab[(size_t)(0 * P + k) * NL + lane] = sc;
            tab[(size_t)(1 * P + k) * NL + lane] = t2;
            tab[(size_t)(2 * P + k) * NL + lane] = ct2;
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
    if (c->d_tmp) hipFree(c->d_tmp);
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
    hipEvent_t fork;
    HIP_TRY(c, hipEventCreateWithFlags(&fork, hipEventDisableTiming));
    HIP_TRY(c, hipEventRecord(fork, c->stream));
    for (LaunchClass& lc : c->classes) {
        hipStream_t s = c->classes.size() == 1 ? c->stream : lc.stream;
        if (s != c->stream) HIP_TRY(c, hipStreamWaitEvent(s, fork, 0));
        HIP_TRY(c, launch(lc, s));
        if (s != c->stream) {
            HIP_TRY(c, hipEventRecord(lc.done, s));
            HIP_TRY(c, hipStreamWaitEvent(c->stream, lc.done, 0));
        }
    }
    HIP_TRY(c, hipEventDestroy(fork));
    return ADSCL_OK;
}

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
    a.total = c->total;
    a.a_collapse = c->thr;
    a.snap_every = snap_every;
    a.gauge = c->gauge;
    a.frozen = (c->flags & ADSCL_FROZEN_METRIC) ? 1 : 0;
    a.ckpt_every = 0;
    a.src_every = 1;
    a.pad = 0;
    return a;
}

// One segment of the fused kernel over all classes: every instance advances to
// its target step, or to its next multiple of snap_every when that is > 0.
int run_evolve(adscl_ctx* c, const EvolveArgs& base)
{
    return run_classes(c, [&](LaunchClass& lc, hipStream_t s) -> hipError_t {
        EvolveArgs a = base;
        a.order = lc.d_order;
        hipError_t e = hipSuccess;
        if (lc.t0 && (e = hipEventRecord(lc.t0, s)) != hipSuccess) return e;
        if ((e = launch_evolve(lc.cfg, lc.full, (int)lc.inst.size(), a, s)) != hipSuccess) return e;
        if (lc.t1) {
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
                               snaps, c->stream));
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
        if (N < 17 || N > 4097 || (N % 2) == 0)
            return fail(nullptr, ADSCL_EINVAL,
                        "instance " + std::to_string(b) + ": N=" + std::to_string(N) +
                            " (need odd N, 17 <= N <= 4097)");
    }
    if (!(cfg->cfl > 0.0 && cfg->cfl <= 1.0)) return fail(nullptr, ADSCL_EINVAL, "cfl must be in (0, 1]");
    if (!(cfg->ko_sigma >= 0.0 && cfg->ko_sigma <= 2.0)) return fail(nullptr, ADSCL_EINVAL, "ko_sigma must be in [0, 2]");
    if (!(cfg->a_collapse >= 0.0 && cfg->a_collapse <= 1.0)) return fail(nullptr, ADSCL_EINVAL, "a_collapse must be in [0, 1]");
    if (cfg->gauge != ADSCL_GAUGE_BOUNDARY && cfg->gauge != ADSCL_GAUGE_ORIGIN) return fail(nullptr, ADSCL_EINVAL, "bad gauge");
    if (cfg->n_modes < 0 || cfg->n_modes > 128) return fail(nullptr, ADSCL_EINVAL, "n_modes must be in [0, 128]");
    if (cfg->flags & ~(ADSCL_FROZEN_METRIC | ADSCL_TIME_KERNELS)) return fail(nullptr, ADSCL_EINVAL, "unknown flags");

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
        if (!c->tables.count(N)) {
            NTables t;
            t.cfg = choose_class(N);
            if (t.cfg.P == 0) {
                c->err = "no kernel configuration for N=" + std::to_string(N);
                return bail(ADSCL_EUNSUPPORTED);
            }
            if (evolve_lds_bytes(t.cfg) > c->max_lds) {
                c->err = "N=" + std::to_string(N) + " needs " + std::to_string(evolve_lds_bytes(t.cfg)) +
                         " B of LDS, device allows " + std::to_string(c->max_lds);
                return bail(ADSCL_EUNSUPPORTED);
            }
            TRY_C(prepare_evolve(t.cfg, c->max_lds));
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
        if (c->classes.size() > 1) {
            TRY_C(hipStreamCreateWithFlags(&lc.stream, hipStreamNonBlocking));
            TRY_C(hipEventCreateWithFlags(&lc.done, hipEventDisableTiming));
        }
        if (c->flags & ADSCL_TIME_KERNELS) {
            TRY_C(hipEventCreate(&lc.t0));
            TRY_C(hipEventCreate(&lc.t1));
        }
    }
    // launch the biggest classes first
    std::stable_sort(c->classes.begin(), c->classes.end(), [](const LaunchClass& x, const LaunchClass& y) {
        return 64 * x.cfg.W * x.cfg.P > 64 * y.cfg.W * y.cfg.P;
    });

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
    if (c->stream) hipStreamSynchronize(c->stream);
    for (LaunchClass& lc : c->classes) {
        if (lc.d_order) hipFree(lc.d_order);
        if (lc.stream) hipStreamDestroy(lc.stream);
        if (lc.done) hipEventDestroy(lc.done);
        if (lc.t0) hipEventDestroy(lc.t0);
        if (lc.t1) hipEventDestroy(lc.t1);
    }
    for (auto& kv : c->tables) {
        if (kv.second.d_tab) hipFree(kv.second.d_tab);
        if (kv.second.d_emode) hipFree(kv.second.d_emode);
        if (kv.second.d_wPi) hipFree(kv.second.d_wPi);
        if (kv.second.d_wPhi) hipFree(kv.second.d_wPhi);
    }
    if (c->d_tab) hipFree((void*)c->d_tab);
    if (c->d_emode) hipFree((void*)c->d_emode);
    if (c->d_wPi) hipFree((void*)c->d_wPi);
    if (c->d_wPhi) hipFree((void*)c->d_wPhi);
    if (c->state5) hipFree(c->state5);
    if (c->d_status) hipFree(c->d_status);
    if (c->d_ic) hipFree(c->d_ic);
    if (c->d_tmp) hipFree(c->d_tmp);
    for (auto& kv : c->bufs)
        if (kv.second.first) hipFree(kv.second.first);
    if (c->own_stream && c->stream) hipStreamDestroy(c->stream);
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
    if (want && mem == ADSCL_MEM_HOST) {
        if (rc == ADSCL_OK) {
            hipError_t e = hipMemcpyAsync(snaps, dsn, snap_bytes, hipMemcpyDeviceToHost, c->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
            if (e != hipSuccess) rc = fail(c, ADSCL_EHIP, std::string("snapshot copy: ") + hipGetErrorString(e));
        }
        hipFree(dsn);
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

int adscl_constraints(adscl_ctx* c, double* out, int mem)
{
    if (!c) return fail(nullptr, ADSCL_EINVAL, "ctx is NULL");
    if (!c->initialized) return fail(c, ADSCL_ESTATE, "adscl_constraints before any adscl_init*");
    if (!out) return fail(c, ADSCL_EINVAL, "out is NULL");
    if (int rc = check_mem(c, mem)) return rc;
    double* dst = mem == ADSCL_MEM_DEVICE ? out : c->d_tmp;
    const double* s = c->state5;
    HIP_TRY(c, launch_diagnostics(c->n_inst, c->d_ic, s, s + c->total, s + 2 * c->total, s + 3 * c->total,
                                  s + 4 * c->total, dst, c->stream));
    if (mem == ADSCL_MEM_HOST) {
        HIP_TRY(c, hipMemcpyAsync(out, dst, sizeof(double) * 4 * c->n_inst, hipMemcpyDeviceToHost, c->stream));
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
    const size_t n = (size_t)c->n_inst * J;
    double *dE = E, *dP = Pihat, *dF = Phihat;
    if (mem == ADSCL_MEM_HOST) {
        dE = E ? c->d_tmp : nullptr;
        dP = Pihat ? c->d_tmp + n : nullptr;
        dF = Phihat ? c->d_tmp + 2 * n : nullptr;
        if (int rc = ensure_tmp(c, 3 * n * sizeof(double))) return rc;
        dE = E ? c->d_tmp : nullptr;
        dP = Pihat ? c->d_tmp + n : nullptr;
        dF = Phihat ? c->d_tmp + 2 * n : nullptr;
    }
    const double* s = c->state5;
    HIP_TRY(c, launch_spectrum(c->n_inst, c->d_ic, s, s + c->total, s + 2 * c->total, c->d_wPi, c->d_wPhi, J, dE,
                               dP, dF, c->stream));
    if (mem == ADSCL_MEM_HOST) {
        if (E) HIP_TRY(c, hipMemcpyAsync(E, dE, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        if (Pihat) HIP_TRY(c, hipMemcpyAsync(Pihat, dP, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        if (Phihat) HIP_TRY(c, hipMemcpyAsync(Phihat, dF, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
    }
    return ADSCL_OK;
}

int adscl_adjoint(adscl_ctx* c, const double* eps, const double* coef, int32_t Jc, int32_t J, double T,
                  int32_t ckpt_every, double* L, double* dLdc, int32_t* valid, int mem)
{
    if (!c) return fail(nullptr, ADSCL_EINVAL, "ctx is NULL");
    if (!eps || !coef || !L || !dLdc || !valid) return fail(c, ADSCL_EINVAL, "NULL argument");
    if (c->flags & ADSCL_FROZEN_METRIC) return fail(c, ADSCL_EUNSUPPORTED, "adjoint needs the dynamic metric");
    if (Jc < 1 || Jc > c->n_modes || J < 1 || J > c->n_modes)
        return fail(c, ADSCL_EINVAL, "need 1 <= Jc, J <= n_modes");
    if (!(T >= 0.0) || std::isinf(T)) return fail(c, ADSCL_EINVAL, "T must be finite and >= 0");
    if (ckpt_every < 1) return fail(c, ADSCL_EINVAL, "ckpt_every must be >= 1");
    if (int rc = check_mem(c, mem)) return rc;
    const int n = c->n_inst;
    const int64_t K = ckpt_every;
    int rc;

    // per-instance step counts and buffer sizes (doubles)
    std::vector<int64_t> nf(n), ck_off(n + 1), seg_off(n + 1), stg_off(n + 1);
    for (int b = 0; b < n; ++b) {
        const double r = T / c->h_ic[b].dt - 1e-9;
        nf[b] = (r <= 0.0) ? 0 : (int64_t)std::ceil(r);
        const NTables& t = c->tables[c->N[b]];
        ck_off[b + 1] = ck_off[b] + (nf[b] / K + 1) * 2 * (int64_t)c->N[b];
        seg_off[b + 1] = seg_off[b] + (std::min<int64_t>(K, nf[b]) + 1) * 2 * (int64_t)c->N[b];
        stg_off[b + 1] = stg_off[b] + (int64_t)adjoint_scratch_len(t.cfg);
    }
    void *ck, *seg, *stg, *ub, *u0, *dummy, *spec, *deps, *ptrs, *rst, *sgs, *outs;
    const size_t nJ = (size_t)n * J;
    if ((rc = buffer(c, "ckpt", sizeof(double) * ck_off[n], &ck))) return rc;
    if ((rc = buffer(c, "seg", sizeof(double) * seg_off[n], &seg))) return rc;
    if ((rc = buffer(c, "stage", sizeof(double) * stg_off[n], &stg))) return rc;
    if ((rc = buffer(c, "ubar", sizeof(double) * 2 * c->total, &ub))) return rc;
    if ((rc = buffer(c, "u0", sizeof(double) * 2 * c->total, &u0))) return rc;
    if ((rc = buffer(c, "dummy", sizeof(double) * 2 * c->total, &dummy))) return rc;
    if ((rc = buffer(c, "spec", sizeof(double) * 6 * nJ, &spec))) return rc;
    if ((rc = buffer(c, "eps", sizeof(double) * n, &deps))) return rc;
    if ((rc = buffer(c, "ptrs", sizeof(double*) * 3 * n, &ptrs))) return rc;
    if ((rc = buffer(c, "rstatus", sizeof(InstStatus) * n, &rst))) return rc;
    if ((rc = buffer(c, "segs", sizeof(AdjSeg) * n, &sgs))) return rc;
    if ((rc = buffer(c, "outs", sizeof(double) * ((size_t)n * Jc + 2 * n), &outs))) return rc;
    double* E0 = (double*)spec;
    double* a0 = E0 + nJ;
    double* b0 = a0 + nJ;
    double* ET = b0 + nJ;
    double* aT = ET + nJ;
    double* bT = aT + nJ;
    double** d_ckp = (double**)ptrs;
    double** d_segp = d_ckp + n;
    double** d_stgp = d_segp + n;
    {
        std::vector<double*> hp(3 * n);
        for (int b = 0; b < n; ++b) {
            hp[b] = (double*)ck + ck_off[b];
            hp[n + b] = (double*)seg + seg_off[b];
            hp[2 * n + b] = (double*)stg + stg_off[b];
        }
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        HIP_TRY(c, hipMemcpy(ptrs, hp.data(), sizeof(double*) * 3 * n, hipMemcpyHostToDevice));
    }
    HIP_TRY(c, hipMemcpyAsync(deps, eps, sizeof(double) * n,
                              mem == ADSCL_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->stream));

    // forward: initial data, its spectrum, the evolution with checkpoints, the
    // final spectrum
    if ((rc = adscl_init_modes(c, eps, coef, Jc, mem))) return rc;
    const double* s5 = c->state5;
    HIP_TRY(c, hipMemcpyAsync(u0, s5, sizeof(double) * 2 * c->total, hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(c, launch_spectrum(n, c->d_ic, s5, s5 + c->total, s5 + 2 * c->total, c->d_wPi, c->d_wPhi, J, E0, a0, b0,
                               c->stream));
    if ((rc = upload_ic(c, T))) return rc;
    HIP_TRY(c, launch_set_targets(n, c->d_ic, c->d_status, INT64_MAX / 4, c->stream));
    {
        EvolveArgs a = evolve_args(c, 0);
        a.ckpt = d_ckp;
        a.ckpt_every = (int32_t)K;
        if ((rc = run_evolve(c, a))) return rc;
    }
    if ((rc = run_finalize(c, true, 0, 0, nullptr))) return rc;
    HIP_TRY(c, launch_spectrum(n, c->d_ic, s5, s5 + c->total, s5 + 2 * c->total, c->d_wPi, c->d_wPhi, J, ET, aT, bT,
                               c->stream));

    // reverse: final spectrum, segments from the last to the first, initial
    // spectrum, initial map
    HIP_TRY(c, hipMemsetAsync(ub, 0, sizeof(double) * 2 * c->total, c->stream));
    EndArgs ea;
    ea.ic = c->d_ic;
    ea.order = nullptr;
    ea.tab = c->d_tab;
    ea.Phi = s5;
    ea.Pi = s5 + c->total;
    ea.wPi = c->d_wPi;
    ea.wPhi = c->d_wPhi;
    ea.Pihat = aT;
    ea.Phihat = bT;
    ea.E0 = E0;
    ea.ET = ET;
    ea.status = c->d_status;
    ea.Ubar = (double*)ub;
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

    int64_t max_seg = 0;
    for (int b = 0; b < n; ++b) max_seg = std::max<int64_t>(max_seg, (nf[b] + K - 1) / K);
    EvolveArgs ra = evolve_args(c, 0);
    ra.Phi = (double*)dummy;
    ra.Pi = (double*)dummy + c->total;
    ra.status = (InstStatus*)rst;
    ra.src = d_ckp;
    ra.src_every = (int32_t)K;
    ra.ckpt = d_segp;
    ra.ckpt_every = 1;
    AdjointArgs aa;
    aa.ic = c->d_ic;
    aa.order = nullptr;
    aa.tab = c->d_tab;
    aa.seg = d_segp;
    aa.stg = d_stgp;
    aa.sg = (AdjSeg*)sgs;
    aa.Ubar = (double*)ub;
    aa.total = c->total;
    aa.gauge = c->gauge;
    aa.pad = 0;
    for (int64_t r = 0; r < max_seg; ++r) {
        HIP_TRY(c, launch_adj_prepare(n, c->d_ic, c->d_status, K, r, (InstStatus*)rst, (AdjSeg*)sgs, c->stream));
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
    ea.Phi = (const double*)u0;
    ea.Pi = (const double*)u0 + c->total;
    ea.Pihat = a0;
    ea.Phihat = b0;
    ea.sgn = -1.0;
    if ((rc = run_end())) return rc;

    double* oL = (double*)outs;
    double* oG = oL + n;
    int32_t* oV = (int32_t*)(oG + (size_t)n * Jc);
    if (mem == ADSCL_MEM_DEVICE) {
        oL = L;
        oG = dLdc;
        oV = valid;
    }
    HIP_TRY(c, launch_adj_finish(n, c->d_ic, c->d_status, (const double*)ub, c->total, c->d_emode,
                                 (const double*)deps, Jc, E0, ET, J, oL, oG, oV, c->stream));
    if (mem == ADSCL_MEM_HOST) {
        HIP_TRY(c, hipMemcpyAsync(L, oL, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipMemcpyAsync(dLdc, oG, sizeof(double) * n * Jc, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipMemcpyAsync(valid, oV, sizeof(int32_t) * n, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
    }
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
            for (int32_t b : lc.inst) cls[b] = k;
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

const char* adscl_last_error(const adscl_ctx* c)
{
    return c ? c->err.c_str() : g_create_error.c_str();
}

}  // extern "C"
