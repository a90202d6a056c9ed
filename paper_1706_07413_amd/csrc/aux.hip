// Initial data, status reset, diagnostics and mode projection kernels for the
// AdS4 scalar-collapse library (Liebling & Khanna, arXiv:1706.07413, Sec. II).
#include <math.h>

#include "internal.h"

namespace adscl {
namespace {

// Pi(x,0) = (2 eps/pi) exp(-4 tan^2 x/(pi^2 sigma^2)), Phi(x,0) = 0 (Sec. II:
// data Phi, Pi given at t = 0); Pi = 0 at x = pi/2 (Eq. (10)).
__global__ void init_gaussian_kernel(int n_inst, const InstConst* ic, const double* eps, const double* sigma,
                                     double* Phi, double* Pi)
{
    const int b = blockIdx.y;
    if (b >= n_inst) return;
    const InstConst c = ic[b];
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < c.N; i += gridDim.x * blockDim.x) {
        const double x = (double)i * c.h;
        const double t = tan(x);
        const double s = sigma[b];
        double v = (2.0 * eps[b] / kPi) * exp(-4.0 * t * t / (kPi * kPi * s * s));
        if (i == c.N - 1) v = 0.0;
        Phi[c.off + i] = 0.0;
        Pi[c.off + i] = v;
    }
}

// Pi(x,0) = eps sum_{j<Jc} c_j e_j(x), Phi(x,0) = 0.
__global__ void init_modes_kernel(int n_inst, const InstConst* ic, const double* eps, const double* c, int Jc,
                                  const double* const* emode, double* Phi, double* Pi)
{
    const int b = blockIdx.y;
    if (b >= n_inst) return;
    const InstConst k = ic[b];
    const double* e = emode[b];
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < k.N; i += gridDim.x * blockDim.x) {
        double sum = 0.0;
        for (int j = 0; j < Jc; ++j) sum += c[(size_t)b * Jc + j] * e[(size_t)j * k.N + i];
        Phi[k.off + i] = 0.0;
        Pi[k.off + i] = (i == k.N - 1) ? 0.0 : eps[b] * sum;
    }
}

// Phi(0) = 0, Phi(pi/2) = Pi(pi/2) = 0 (Eqs. (7), (9), (10)).
__global__ void pins_kernel(int n_inst, const InstConst* ic, double* Phi, double* Pi)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n_inst) return;
    const InstConst c = ic[b];
    Phi[c.off] = 0.0;
    Phi[c.off + c.N - 1] = 0.0;
    Pi[c.off + c.N - 1] = 0.0;
}

__global__ void reset_status_kernel(int n_inst, InstStatus* st)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n_inst) return;
    InstStatus o;
    o.steps = 0;
    o.target = 0;
    o.t_c = -1.0;
    o.minA = 1.0;
    o.mass = 0.0;
    o.state = ST_RUNNING;
    o.pad = 0;
    st[b] = o;
}

__global__ void set_targets_kernel(int n_inst, const InstConst* ic, InstStatus* st, int64_t max_steps)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n_inst) return;
    InstStatus o = st[b];
    int64_t t = o.steps + max_steps;
    if (t > ic[b].n_final) t = ic[b].n_final;
    if (t < o.steps) t = o.steps;
    o.target = t;
    st[b] = o;
}

// Block-wide exclusive prefix sum of one value per thread (256 threads).
__device__ double block_excl_scan(double v, double* sh, double& total)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    double x = v;
    for (int d = 1; d < 64; d <<= 1) {
        const double t = __shfl_up(x, d, 64);
        if (lane >= d) x += t;
    }
    __syncthreads();
    if (lane == 63) sh[wv] = x;
    __syncthreads();
    double carry = 0.0;
    total = 0.0;
    for (int w = 0; w < 4; ++w) {
        if (w < wv) carry += sh[w];
        total += sh[w];
    }
    return carry + x - v;
}

struct FinArgs {
    const InstConst* ic;
    InstStatus* st;
    double* state5;
    int64_t total;
    double a_collapse;
    double* snaps;
    int32_t snap_every;
    int32_t n_slots;
    int32_t gauge;
    int32_t frozen;
    int32_t final_;
    int32_t a_reint;  // > 0: A is evolved; the state's A is kept unless steps % a_reint == 0
};

// Constraint solve of the packed state of one instance per 256-thread block
// (Sec. II, Eqs. (5)-(6), the same discretisation as the evolution kernel:
// 4-point cell rule in prefix-sum form, m = (1 - A) sin x / cos^3 x), written
// out as (Phi, Pi, A, delta, m); then min A, the mass m(pi/2) and, at the end
// of a call, the collapse / non-finite test of the final state.  With A evolved
// (a_reint > 0) the state's A is kept (and tested) except at steps that are a
// multiple of a_reint, where the solve's A replaces it as the evolution would.
__global__ void __launch_bounds__(256) finalize_kernel(FinArgs f)
{
    __shared__ double sh[16];
    __shared__ int ish[4];
    const int b = blockIdx.x;
    const InstStatus st = f.st[b];
    const InstConst c = f.ic[b];
    const bool snap = f.snaps && f.snap_every > 0 && (st.steps % f.snap_every) == 0 &&
                      (st.steps / f.snap_every) < f.n_slots;
    if (!snap && !f.final_) return;
    const int N = c.N;
    const double h = c.h;
    const double* Phi = f.state5 + c.off;
    const double* Pi = f.state5 + f.total + c.off;
    double* dst[2] = {f.final_ ? f.state5 : nullptr,
                      snap ? f.snaps + (size_t)(st.steps / f.snap_every) * 5 * (size_t)f.total : nullptr};
    // scratch for delta~ before the gauge shift: the delta row of the first target
    double* dscr = (dst[0] ? dst[0] : dst[1]) + 3 * f.total + c.off;

    const int tid = threadIdx.x;
    const int C = (N + 255) / 256;
    const int i0 = tid * C;
    const int i1 = min(N, i0 + C);
    auto q_at = [&](int i) -> double { return Phi[i] * Phi[i] + Pi[i] * Pi[i]; };
    auto sc_at = [&](int i) -> double {
        const double x = (double)i * h;
        return sin(x) * cos(x);
    };
    auto t2_at = [&](int i) -> double {
        const double t = tan((double)i * h);
        return t * t;
    };
    // p = sin x cos x q: 0 at both ends, odd ghosts about both ends
    auto p_at = [&](int i) -> double {
        double sgn = 1.0;
        if (i < 0) { i = -i; sgn = -1.0; }
        if (i > N - 1) { i = 2 * (N - 1) - i; sgn = -sgn; }
        if (i == 0 || i == N - 1) return 0.0;
        return sgn * sc_at(i) * q_at(i);
    };

    double dN = 0.0, tot2 = 0.0, shift = 0.0;
    if (!f.frozen) {
        double ps = 0.0;
        for (int i = i0; i < i1; ++i) ps += p_at(i);
        double tot;
        const double carry = block_excl_scan(ps, sh, tot);
        const double p1 = p_at(1);
        double R = carry;
        for (int i = i0; i < i1; ++i) {
            const double pi_ = p_at(i);
            R += pi_;
            dscr[i] = -(h / 24.0) * (24.0 * R - 12.0 * pi_ + p_at(i - 1) - p_at(i + 1) + 2.0 * p1);
        }
        dN = -(h / 24.0) * (24.0 * tot + 2.0 * p_at(N - 2) + 2.0 * p1);
        shift = (f.gauge == 0) ? dN : 0.0;
        __syncthreads();
    }
    // sigma = tan^2 x q e^{-delta}: 0 at both ends, even ghosts
    auto sig_at = [&](int i) -> double {
        if (i < 0) i = -i;
        if (i > N - 1) i = 2 * (N - 1) - i;
        if (i == 0 || i == N - 1) return 0.0;
        return t2_at(i) * q_at(i) * exp(-(dscr[i] - shift));
    };
    double mn = 1.0, chk = 0.0;
    int col = 0;
    const bool keepA = f.a_reint > 0 && (st.steps % f.a_reint) != 0;
    const double* Arow = f.state5 + 2 * f.total + c.off;
    if (!f.frozen) {
        double ss = 0.0;
        for (int i = i0; i < i1; ++i) ss += sig_at(i);
        double carry2 = block_excl_scan(ss, sh + 4, tot2);
        double R2 = carry2;
        for (int i = i0; i < i1; ++i) {
            const double si = sig_at(i);
            R2 += si;
            const double S = (h / 24.0) * (24.0 * R2 - 12.0 * si + sig_at(i - 1) - sig_at(i + 1));
            const double dl = dscr[i] - shift;
            const double E = exp(-dl);
            const double m = S / E;
            double A = 1.0;
            if (keepA) {
                A = Arow[i];
                if (A < f.a_collapse) col = 1;
            } else if (i >= 1 && i <= N - 2) {
                const double x = (double)i * h;
                const double s = sin(x), co = cos(x);
                const double c3s = co * co * co / s;
                A = 1.0 - c3s * m;
                if (E - c3s * S < f.a_collapse * E) col = 1;
            }
            mn = fmin(mn, A);
            chk = fma(q_at(i), 0.0, chk);
            chk = fma(A, 0.0, chk);
            chk = fma(dl, 0.0, chk);
            for (int d = 0; d < 2; ++d) {
                if (!dst[d]) continue;
                dst[d][2 * f.total + c.off + i] = A;
                dst[d][4 * f.total + c.off + i] = m;
            }
        }
        __syncthreads();  // all reads of the delta~ scratch are done
        for (int i = i0; i < i1; ++i) {
            const double dl = (i == N - 1) ? ((f.gauge == 0) ? 0.0 : dN) : dscr[i] - shift;
            for (int d = 0; d < 2; ++d)
                if (dst[d]) dst[d][3 * f.total + c.off + i] = dl;
        }
    } else {
        for (int i = i0; i < i1; ++i) {
            chk = fma(q_at(i), 0.0, chk);
            for (int d = 0; d < 2; ++d) {
                if (!dst[d]) continue;
                double* o = dst[d];
                o[2 * f.total + c.off + i] = 1.0;
                o[3 * f.total + c.off + i] = 0.0;
                o[4 * f.total + c.off + i] = 0.0;
            }
        }
    }
    if (dst[1]) {
        double* o = dst[1];
        for (int i = i0; i < i1; ++i) {
            o[c.off + i] = Phi[i];
            o[f.total + c.off + i] = Pi[i];
        }
    }
    if (!isfinite(chk) || !isfinite(dN)) col |= 2;
    if (1.0 < f.a_collapse) col |= 1;
    // block reductions of min A and the flags
    for (int d = 32; d >= 1; d >>= 1) mn = fmin(mn, __shfl_xor(mn, d, 64));
    const int wcol = __any(col & 1) ? 1 : 0;
    const int wnf = __any(col & 2) ? 2 : 0;
    __syncthreads();
    if ((tid & 63) == 0) {
        sh[8 + (tid >> 6)] = mn;
        ish[tid >> 6] = wcol | wnf;
    }
    __syncthreads();
    if (tid == 0) {
        double mA = 1.0;
        int fl = 0;
        for (int w = 0; w < 4; ++w) {
            mA = fmin(mA, sh[8 + w]);
            fl |= ish[w];
        }
        if (f.final_) {
            InstStatus o = st;
            o.minA = mA;
            o.mass = f.frozen ? 0.0 : h * tot2 / ((f.gauge == 0) ? 1.0 : exp(-dN));
            if (o.state == ST_RUNNING || o.state == ST_DONE) {
                if (fl & 2) {
                    o.state = ST_NONFINITE;
                    o.t_c = (double)o.steps * c.dt;
                } else if (fl & 1) {
                    o.state = ST_COLLAPSED;
                    o.t_c = (double)o.steps * c.dt;
                } else {
                    o.state = (o.steps >= c.n_final) ? ST_DONE : ST_RUNNING;
                }
            }
            f.st[b] = o;
        }
    }
}

__device__ double block_reduce(double v, bool take_max, double* sh)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int d = 32; d >= 1; d >>= 1) {
        const double o = __shfl_xor(v, d, 64);
        v = take_max ? fmax(v, o) : v + o;
    }
    __syncthreads();
    if (lane == 0) sh[wv] = v;
    __syncthreads();
    double r = take_max ? 0.0 : 0.0;
    for (int w = 0; w < nw; ++w) r = take_max ? fmax(r, sh[w]) : r + sh[w];
    return r;
}

// Residuals of Eqs. (5)-(6) at interior points and the mass integral of Sec. II,
// into columns 0, 1, 3, 4 of out [n_inst][5].  One 256-thread block per instance.
__global__ void __launch_bounds__(256) diagnostics_kernel(int n_inst, const InstConst* ic, const double* Phi,
                                                          const double* Pi, const double* A,
                                                          const double* delta, const double* m, double* out)
{
    __shared__ double sh[8];
    const int b = blockIdx.x;
    const InstConst c = ic[b];
    const int N = c.N;
    const double h = c.h;
    const double* Ph = Phi + c.off;
    const double* Pq = Pi + c.off;
    const double* Aa = A + c.off;
    const double* dd = delta + c.off;
    // ghosts: A even about 0, A - 1 odd about pi/2; delta even about both ends
    auto Ag = [&](int i) -> double {
        if (i < 0) return Aa[-i];
        if (i > N - 1) return 2.0 - Aa[2 * (N - 1) - i];
        return Aa[i];
    };
    auto dg = [&](int i) -> double {
        if (i < 0) return dd[-i];
        if (i > N - 1) return dd[2 * (N - 1) - i];
        return dd[i];
    };
    // integrand tan^2 x A q, even about both ends, zero at both ends
    auto mg = [&](int i) -> double {
        if (i < 0) i = -i;
        if (i > N - 1) i = 2 * (N - 1) - i;
        if (i == 0 || i == N - 1) return 0.0;
        const double t = tan((double)i * h);
        return t * t * Aa[i] * (Ph[i] * Ph[i] + Pq[i] * Pq[i]);
    };
    double rA = 0.0, rd = 0.0, M = 0.0;
    for (int i = threadIdx.x; i < N - 1; i += blockDim.x) {
        M += h * (-mg(i - 1) + 13.0 * mg(i) + 13.0 * mg(i + 1) - mg(i + 2)) / 24.0;
        if (i >= 1) {
            const double x = (double)i * h;
            const double s = sin(x), co = cos(x);
            const double sc = s * co;
            const double q = Ph[i] * Ph[i] + Pq[i] * Pq[i];
            const double DA = (Ag(i - 2) - 8.0 * Ag(i - 1) + 8.0 * Ag(i + 1) - Ag(i + 2)) / (12.0 * h);
            const double Dd = (dg(i - 2) - 8.0 * dg(i - 1) + 8.0 * dg(i + 1) - dg(i + 2)) / (12.0 * h);
            const double ra = DA - ((1.0 + 2.0 * s * s) / sc * (1.0 - Aa[i]) - sc * Aa[i] * q);
            const double rdl = Dd + sc * q;
            rA = fmax(rA, fabs(ra));
            rd = fmax(rd, fabs(rdl));
        }
    }
    rA = block_reduce(rA, true, sh);
    rd = block_reduce(rd, true, sh);
    M = block_reduce(M, false, sh);
    if (threadIdx.x == 0) {
        out[b * 5 + 0] = rA;
        out[b * 5 + 1] = rd;
        out[b * 5 + 3] = m[c.off + N - 1];
        out[b * 5 + 4] = M;
    }
}

// Residual of Eq. (4), A_t = -2 sin x cos x A^2 e^-delta Phi Pi, which the
// evolution never imposes (Sec. II monitors the residuals of its equations).
// A_t is the time derivative of the discrete A of the constraint solve along
// the semi-discrete flow: the derivative of A(Phi, Pi) in the direction of the
// right-hand sides (Phi_t, Pi_t) of Eqs. (2)-(3), taken through each step of
// the solve (q = Phi^2 + Pi^2, p = sin x cos x q, delta~ = -prefix cell rule of
// p, E = e^-delta, sigma = tan^2 x q E, S = prefix cell rule of sigma,
// m = S / E, A = 1 - cos^3 x / sin x m):
//   q_t = 2 (Phi Phi_t + Pi Pi_t),  p_t = sin x cos x q_t,
//   delta~_t = -prefix cell rule of p_t,  E_t = -E delta~_t,
//   sigma_t = tan^2 x (q_t E + q E_t),  S_t = prefix cell rule of sigma_t,
//   m_t = (S_t - m E_t) / E,  A_t = -cos^3 x / sin x m_t.
// E is e^-delta of the gauge-shifted delta: m_t is homogeneous of degree 0 in
// a constant factor of E, S and their derivatives, so the shift drops out.
// Input: the packed state (Phi, Pi, A, delta, m) of the current step, whose
// metric is the constraint solve of (Phi, Pi).  One 256-thread block per
// instance, thread t owning a run of consecutive points; `scr` holds two
// doubles per packed point: X = p_t for the whole kernel, Y = q_t of the own
// points, then sigma_t (each thread overwrites only its own entries, and the
// neighbours read Y only after the barrier that follows).  delta~_t is formed
// twice from X with the same carry, so it needs no storage.
// out[b*5 + 2] = max over interior points of |A_t + 2 sin x cos x A^2
// e^-delta Phi Pi|; NaN with the metric frozen (A is then held, not solved).
__global__ void __launch_bounds__(256) adot_residual_kernel(int n_inst, const InstConst* ic,
                                                            const double* state5, int64_t total, int frozen,
                                                            double ko, double* scr, double* out)
{
    __shared__ double sh[16];
    const int b = blockIdx.x;
    if (b >= n_inst) return;
    const InstConst c = ic[b];
    const int N = c.N;
    const double h = c.h;
    if (frozen) {
        if (threadIdx.x == 0) out[b * 5 + 2] = __builtin_nan("");
        return;
    }
    const double* Ph = state5 + c.off;
    const double* Pq = state5 + total + c.off;
    const double* Aa = state5 + 2 * total + c.off;
    const double* dd = state5 + 3 * total + c.off;
    const double* mm = state5 + 4 * total + c.off;
    double* X = scr + c.off;
    double* Y = scr + total + c.off;
    const double kof = ko / (64.0 * h), i12h = 1.0 / (12.0 * h);
    auto t2_at = [&](int i) -> double {
        const double t = tan((double)i * h);
        return t * t;
    };
    // Phi odd about 0, even about pi/2; Pi even about 0, odd about pi/2
    auto phg = [&](int i) -> double {
        if (i < 0) return -Ph[-i];
        if (i > N - 1) return Ph[2 * (N - 1) - i];
        return Ph[i];
    };
    auto pig = [&](int i) -> double {
        if (i < 0) return Pq[-i];
        if (i > N - 1) return -Pq[2 * (N - 1) - i];
        return Pq[i];
    };
    auto w_at = [&](int i) -> double { return Aa[i] * exp(-dd[i]); };
    // f1 = w Pi: even about 0, odd about pi/2
    auto f1g = [&](int i) -> double {
        if (i < 0) return w_at(-i) * Pq[-i];
        if (i > N - 1) {
            const int j = 2 * (N - 1) - i;
            return -(w_at(j) * Pq[j]);
        }
        return w_at(i) * Pq[i];
    };
    // g = tan^2 x w Phi up to N - 2, the even 6th-order extrapolation at N - 1;
    // odd about 0, even about pi/2
    auto g_in = [&](int i) -> double {
        if (i == N - 1) {
            const double g2 = t2_at(N - 2) * (w_at(N - 2) * Ph[N - 2]);
            const double g3 = t2_at(N - 3) * (w_at(N - 3) * Ph[N - 3]);
            const double g4 = t2_at(N - 4) * (w_at(N - 4) * Ph[N - 4]);
            return (15.0 * g2 - 6.0 * g3 + g4) / 10.0;
        }
        return t2_at(i) * (w_at(i) * Ph[i]);
    };
    auto gg = [&](int i) -> double {
        if (i < 0) return -g_in(-i);
        if (i > N - 1) return g_in(2 * (N - 1) - i);
        return g_in(i);
    };
    auto ko7 = [&](auto&& u, int i) -> double {
        return kof * (u(i - 3) - 6.0 * u(i - 2) + 15.0 * u(i - 1) - 20.0 * u(i) + 15.0 * u(i + 1) - 6.0 * u(i + 2)
                      + u(i + 3));
    };
    auto d5 = [&](auto&& u, int i) -> double { return (u(i - 2) - 8.0 * u(i - 1) + 8.0 * u(i + 1) - u(i + 2)) * i12h; };

    const int tid = threadIdx.x;
    const int C = (N + 255) / 256;
    const int i0 = tid * C;
    const int i1 = min(N, i0 + C);
    // right-hand sides of Eqs. (2)-(3) (pinned points 0 except Pi at the origin),
    // q_t and p_t at the own points
    for (int i = i0; i < i1; ++i) {
        double rPh = 0.0, rPi = 0.0;
        if (i >= 1 && i <= N - 2) {
            const double t = tan((double)i * h);
            rPh = d5(f1g, i) + ko7(phg, i);
            rPi = (1.0 / (t * t)) * d5(gg, i) + ko7(pig, i);
        } else if (i == 0) {
            // lim tan^-2 x (tan^2 x f2)' = 3 f2'(0), f2 = w Phi odd about 0
            const double f21 = w_at(1) * Ph[1], f22 = w_at(2) * Ph[2];
            rPi = 3.0 * ((16.0 * f21 - 2.0 * f22) * i12h) + ko7(pig, 0);
        }
        const double qt = 2.0 * (Ph[i] * rPh + Pq[i] * rPi);
        const double x = (double)i * h;
        X[i] = (i == 0 || i == N - 1) ? 0.0 : sin(x) * cos(x) * qt;
        Y[i] = qt;
    }
    __syncthreads();
    // delta~_t: 0 at x = 0, minus the prefix cell rule of p_t (odd about both
    // ends), in the prefix form of the sum of cells (for an odd u with u_0 = 0
    // the terms -u_{-1} - 12 u_0 + u_1 are 2 u_1)
    auto ptg = [&](int i) -> double {
        double sg = 1.0;
        if (i < 0) { i = -i; sg = -1.0; }
        if (i > N - 1) { i = 2 * (N - 1) - i; sg = -sg; }
        return sg * X[i];
    };
    double ps = 0.0;
    for (int i = i0; i < i1; ++i) ps += X[i];
    double tot;
    const double carry = block_excl_scan(ps, sh, tot);
    const double p1 = X[1];
    auto dtil_t = [&](double Rk, int i) -> double {
        return -(h / 24.0) * (24.0 * Rk - 12.0 * X[i] + ptg(i - 1) - ptg(i + 1) + 2.0 * p1);
    };
    double R = carry, ss = 0.0;
    for (int i = i0; i < i1; ++i) {
        R += X[i];
        const double E = exp(-dd[i]);
        const double Et = -E * dtil_t(R, i);
        const double q = Ph[i] * Ph[i] + Pq[i] * Pq[i];
        const double sg = (i == 0 || i == N - 1) ? 0.0 : t2_at(i) * (Y[i] * E + q * Et);
        Y[i] = sg;
        ss += sg;
    }
    __syncthreads();
    // S_t: 0 at x = 0, the prefix cell rule of sigma_t (even about both ends,
    // 0 there); then m_t, A_t and the residual at interior points
    auto sgg = [&](int i) -> double {
        if (i < 0) i = -i;
        if (i > N - 1) i = 2 * (N - 1) - i;
        return Y[i];
    };
    double tot2;
    const double carry2 = block_excl_scan(ss, sh + 4, tot2);
    double R1 = carry, R2 = carry2, rmax = 0.0;
    for (int i = i0; i < i1; ++i) {
        R1 += X[i];
        R2 += Y[i];
        if (i == 0 || i == N - 1) continue;
        const double St = (h / 24.0) * (24.0 * R2 - 12.0 * Y[i] + sgg(i - 1) - sgg(i + 1));
        const double E = exp(-dd[i]);
        const double Et = -E * dtil_t(R1, i);
        const double mt = (St - mm[i] * Et) / E;
        const double x = (double)i * h;
        const double sn = sin(x), co = cos(x);
        const double At = -(co * co * co / sn) * mt;
        const double r = At + 2.0 * (sn * co) * Aa[i] * Aa[i] * E * Ph[i] * Pq[i];
        rmax = fmax(rmax, fabs(r));
        if (!(r == r)) rmax = r;  // keep a NaN
    }
    for (int d = 32; d >= 1; d >>= 1) {
        const double o = __shfl_xor(rmax, d, 64);
        rmax = (o == o) ? fmax(rmax, o) : o;
    }
    __syncthreads();
    if ((tid & 63) == 0) sh[8 + (tid >> 6)] = rmax;
    __syncthreads();
    if (tid == 0) {
        double r = 0.0;
        for (int w = 0; w < 4; ++w) r = (sh[8 + w] == sh[8 + w]) ? fmax(r, sh[8 + w]) : sh[8 + w];
        out[b * 5 + 2] = r;
    }
}

}  // namespace

hipError_t launch_init_gaussian(int n_inst, const InstConst* ic, const double* eps, const double* sigma,
                                double* Phi, double* Pi, int64_t max_N, hipStream_t s)
{
    const int gx = (int)((max_N + 255) / 256);
    init_gaussian_kernel<<<dim3(gx, n_inst), dim3(256), 0, s>>>(n_inst, ic, eps, sigma, Phi, Pi);
    return hipGetLastError();
}

hipError_t launch_init_modes(int n_inst, const InstConst* ic, const double* eps, const double* c, int Jc,
                             const double* const* emode, double* Phi, double* Pi, int64_t max_N, hipStream_t s)
{
    const int gx = (int)((max_N + 255) / 256);
    init_modes_kernel<<<dim3(gx, n_inst), dim3(256), 0, s>>>(n_inst, ic, eps, c, Jc, emode, Phi, Pi);
    return hipGetLastError();
}

hipError_t launch_pins(int n_inst, const InstConst* ic, double* Phi, double* Pi, hipStream_t s)
{
    pins_kernel<<<dim3((n_inst + 255) / 256), dim3(256), 0, s>>>(n_inst, ic, Phi, Pi);
    return hipGetLastError();
}

hipError_t launch_reset_status(int n_inst, InstStatus* st, hipStream_t s)
{
    reset_status_kernel<<<dim3((n_inst + 255) / 256), dim3(256), 0, s>>>(n_inst, st);
    return hipGetLastError();
}

hipError_t launch_set_targets(int n_inst, const InstConst* ic, InstStatus* st, int64_t max_steps, hipStream_t s)
{
    set_targets_kernel<<<dim3((n_inst + 255) / 256), dim3(256), 0, s>>>(n_inst, ic, st, max_steps);
    return hipGetLastError();
}

hipError_t launch_finalize(int n_inst, const InstConst* ic, InstStatus* st, double* state5, int64_t total,
                           int gauge, int frozen, double a_collapse, bool final, int32_t snap_every,
                           int32_t n_slots, double* snaps, hipStream_t s, int32_t a_reint)
{
    FinArgs f;
    f.ic = ic;
    f.st = st;
    f.state5 = state5;
    f.total = total;
    f.a_collapse = a_collapse;
    f.snaps = snaps;
    f.snap_every = snap_every;
    f.n_slots = n_slots;
    f.gauge = gauge;
    f.frozen = frozen;
    f.final_ = final ? 1 : 0;
    f.a_reint = a_reint;
    finalize_kernel<<<dim3(n_inst), dim3(256), 0, s>>>(f);
    return hipGetLastError();
}

hipError_t launch_diagnostics(int n_inst, const InstConst* ic, const double* Phi, const double* Pi,
                              const double* A, const double* delta, const double* m, double* out, hipStream_t s)
{
    diagnostics_kernel<<<dim3(n_inst), dim3(256), 0, s>>>(n_inst, ic, Phi, Pi, A, delta, m, out);
    return hipGetLastError();
}

hipError_t launch_adot_residual(int n_inst, const InstConst* ic, const double* state5, int64_t total, int frozen,
                                double ko, double* scr, double* out, hipStream_t s)
{
    adot_residual_kernel<<<dim3(n_inst), dim3(256), 0, s>>>(n_inst, ic, state5, total, frozen, ko, scr, out);
    return hipGetLastError();
}

}  // namespace adscl
