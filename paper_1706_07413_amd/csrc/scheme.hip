// The scheme options of Sec. II on the one-workgroup path, gfx950: second- and
// third-order Runge-Kutta (the paper's results use the third-order one), and A
// evolved by Eq. (4) between periodic re-integrations from Eq. (5) (delta from
// Eq. (6) at every stage), with any of the three orders.  The classical RK4
// with A solved at every stage is evolve.hip's kernel.
//
// The second- and third-order methods are the strong-stability-preserving
// Runge-Kutta methods of Shu and Osher (J. Comput. Phys. 77 (1988) 439):
//   RK2: U1 = U + dt F(U),  U' = U/2 + (U1 + dt F(U1))/2,
//   RK3: U1 = U + dt F(U),  U2 = 3U/4 + (U1 + dt F(U1))/4,
//        U' = U/3 + 2 (U2 + dt F(U2))/3.
// With A evolved the state is (Phi, Pi, A) and F's third component is
// A_t = -2 sin x cos x A^2 e^-delta Phi Pi, pointwise (zero at both ends, where
// sin x cos x is); at the first stage of every step n with n a multiple of the
// re-integration interval K, A is replaced by the solution of Eq. (5) for U^n.
// The collapse test then uses the state's A.  The state's A persists between
// calls in the A row of the packed state.
//
// Layout, exchange and scans as the classical kernel (stage.h): lane l owns P
// consecutive points and keeps U^n, the stage input and (RK4) the accumulator
// in registers; nothing leaves the chip within a segment.
#include "stage.h"

namespace adscl {
namespace {

template <int P, int W, bool FULL, int RK, bool EVA>
__global__ void __launch_bounds__(64 * W) evolve_scheme_kernel(EvolveArgs a)
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
    const int i0 = sg.i0;
    const double dt = sg.dt;
    const int64_t K = a.a_reint;

    // u: U^n; cv: the current stage input; acc: the RK4 accumulator
    double un0[P], un1[P], unA[P], cv0[P], cv1[P], cvA[P], acc0[P], acc1[P], accA[P];
#pragma unroll
    for (int k = 0; k < P; ++k) {
        const int j = i0 + k;
        const bool o = sg.own(k);
        un0[k] = o ? a.Phi[off + j] : 0.0;
        un1[k] = o ? a.Pi[off + j] : 0.0;
        unA[k] = (EVA && o) ? a.A[off + j] : 1.0;
        cv0[k] = un0[k];
        cv1[k] = un1[k];
        cvA[k] = unA[k];
        acc0[k] = acc1[k] = accA[k] = 0.0;
    }

    int stop_bits = 0;
    int64_t n = st0.steps;
    // One stage s of the method on the published stage input cv; returns true
    // when the first stage finds the instance collapsed or non-finite.
    auto stage = [&](const int s) -> bool {
        double r0[P], r1[P], w[P], rA[P];
        const bool reint = EVA && s == 0 && (n % K) == 0;
        const int bits = sg.template rhs<false, EVA>(s == 0, frozen, cv0, cv1, r0, r1, nullptr, 0, cvA, w, reint);
        if (bits) {
            stop_bits = bits;
            return true;
        }
        if (reint) {
#pragma unroll
            for (int k = 0; k < P; ++k) unA[k] = cvA[k];
        }
        if constexpr (EVA) {
            const auto tb = sg.tables();
#pragma unroll
            for (int k = 0; k < P; ++k) rA[k] = -2.0 * sg.tab(tb, 0, k) * cvA[k] * w[k] * cv0[k] * cv1[k];
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
        // every lane read the stage input before B3, so the next may replace it
        sg.publish(cv0, cv1);
        return false;
    };

    int64_t seg_end = st0.target;
    if (a.snap_every > 0) {
        const int64_t nb = (n / a.snap_every + 1) * a.snap_every;
        if (nb < seg_end) seg_end = nb;
    }
    sg.publish(un0, un1);
    while (n < seg_end) {
        if (stage(0)) break;
#pragma unroll 1
        for (int s = 1; s < RK; ++s) stage(s);
        ++n;
    }
#pragma unroll
    for (int k = 0; k < P; ++k) {
        if (sg.own(k)) {
            a.Phi[off + i0 + k] = un0[k];
            a.Pi[off + i0 + k] = un1[k];
            if (EVA) a.A[off + i0 + k] = unA[k];
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

template <int P, int W, int RK, bool EVA>
hipError_t launch_t(bool full, int n_blocks, const EvolveArgs& a, hipStream_t s)
{
    if (full)
        evolve_scheme_kernel<P, W, true, RK, EVA>
            <<<dim3(n_blocks), dim3(64 * W), lds_bytes_for<P, W, true>(), s>>>(a);
    else
        evolve_scheme_kernel<P, W, false, RK, EVA>
            <<<dim3(n_blocks), dim3(64 * W), lds_bytes_for<P, W, false>(), s>>>(a);
    return hipGetLastError();
}

template <int P, int W, int RK, bool EVA>
hipError_t prepare_t(size_t max_lds)
{
    const size_t nf = lds_bytes_for<P, W, true>(), np = lds_bytes_for<P, W, false>();
    if (nf > max_lds || np > max_lds) return hipErrorInvalidValue;
    hipError_t e = hipFuncSetAttribute((const void*)evolve_scheme_kernel<P, W, true, RK, EVA>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)nf);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void*)evolve_scheme_kernel<P, W, false, RK, EVA>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)np);
}

}  // namespace

// Configurations of the scheme kernels: the default lane capacities per grid
// size (the autotuner's table applies to the classical kernel only).
#define ADSCL_SCHEME_CLASSES(X) \
    X(4, 1)                     \
    X(4, 2)                     \
    X(4, 4)                     \
    X(8, 4)                     \
    X(8, 8)

bool scheme_class_supported(ClassCfg c)
{
#define X(p, w) \
    if (c.P == p && c.W == w) return true;
    ADSCL_SCHEME_CLASSES(X)
#undef X
    return false;
}

template <int RK, bool EVA>
hipError_t prepare_scheme_rk(ClassCfg c, size_t max_lds)
{
#define X(p, w) \
    if (c.P == p && c.W == w) return prepare_t<p, w, RK, EVA>(max_lds);
    ADSCL_SCHEME_CLASSES(X)
#undef X
    return hipErrorInvalidValue;
}

template <int RK, bool EVA>
hipError_t launch_scheme_rk(ClassCfg c, bool full, int n_blocks, const EvolveArgs& a, hipStream_t s)
{
#define X(p, w) \
    if (c.P == p && c.W == w) return launch_t<p, w, RK, EVA>(full, n_blocks, a, s);
    ADSCL_SCHEME_CLASSES(X)
#undef X
    return hipErrorInvalidValue;
}

hipError_t prepare_evolve_scheme(ClassCfg c, int rk, bool eva, size_t max_lds)
{
    if (rk == 2) return eva ? prepare_scheme_rk<2, true>(c, max_lds) : prepare_scheme_rk<2, false>(c, max_lds);
    if (rk == 3) return eva ? prepare_scheme_rk<3, true>(c, max_lds) : prepare_scheme_rk<3, false>(c, max_lds);
    if (rk == 4 && eva) return prepare_scheme_rk<4, true>(c, max_lds);
    return hipErrorInvalidValue;
}

hipError_t launch_evolve_scheme(ClassCfg c, int rk, bool eva, bool full, int n_blocks, const EvolveArgs& a,
                                hipStream_t s)
{
    if (rk == 2) return eva ? launch_scheme_rk<2, true>(c, full, n_blocks, a, s)
                            : launch_scheme_rk<2, false>(c, full, n_blocks, a, s);
    if (rk == 3) return eva ? launch_scheme_rk<3, true>(c, full, n_blocks, a, s)
                            : launch_scheme_rk<3, false>(c, full, n_blocks, a, s);
    if (rk == 4 && eva) return launch_scheme_rk<4, true>(c, full, n_blocks, a, s);
    return hipErrorInvalidValue;
}

}  // namespace adscl
