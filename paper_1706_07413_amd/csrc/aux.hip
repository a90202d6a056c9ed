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
    o.t_c = -1.0;
    o.minA = 1.0;
    o.mass = 0.0;
    o.state = ST_RUNNING;
    o.pad = 0;
    st[b] = o;
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

// Residuals of Eqs. (5)-(6) at interior points and the mass integral of Sec. II.
// One 256-thread block per instance.
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
        out[b * 4 + 0] = rA;
        out[b * 4 + 1] = rd;
        out[b * 4 + 2] = m[c.off + N - 1];
        out[b * 4 + 3] = M;
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

hipError_t launch_diagnostics(int n_inst, const InstConst* ic, const double* Phi, const double* Pi,
                              const double* A, const double* delta, const double* m, double* out, hipStream_t s)
{
    diagnostics_kernel<<<dim3(n_inst), dim3(256), 0, s>>>(n_inst, ic, Phi, Pi, A, delta, m, out);
    return hipGetLastError();
}

}  // namespace adscl
