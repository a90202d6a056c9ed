// Projection of the state on the linear AdS4 eigenmodes (Liebling & Khanna,
// arXiv:1706.07413, Sec. II: decomposition into normal modes).
//
//   Pihat_j = sum_i wPi[j][i] sqrt(A_i) Pi_i,   Phihat_j = sum_i wPhi[j][i] sqrt(A_i) Phi_i,
//   E_j = Pihat_j^2 + Phihat_j^2,
// with wPi = h tan^2 x e_j(x), wPhi = h tan^2 x e_j'(x)/omega_j (zero at both ends).
#include <math.h>

#include "internal.h"

namespace adscl {
namespace {

// One 256-thread block per (instance, mode).
__global__ void __launch_bounds__(256) spectrum_kernel(int n_inst, const InstConst* ic, const double* Phi,
                                                       const double* Pi, const double* A,
                                                       const double* const* wPi, const double* const* wPhi,
                                                       int J, double* E, double* Pihat, double* Phihat)
{
    __shared__ double sh[2][4];
    const int b = blockIdx.y, j = blockIdx.x;
    const InstConst c = ic[b];
    const double* wp = wPi[b] + (size_t)j * c.N;
    const double* wf = wPhi[b] + (size_t)j * c.N;
    double a = 0.0, f = 0.0;
    for (int i = threadIdx.x; i < c.N; i += blockDim.x) {
        const double sA = sqrt(A[c.off + i]);
        a += wp[i] * (sA * Pi[c.off + i]);
        f += wf[i] * (sA * Phi[c.off + i]);
    }
    for (int d = 32; d >= 1; d >>= 1) {
        a += __shfl_xor(a, d, 64);
        f += __shfl_xor(f, d, 64);
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) {
        sh[0][wv] = a;
        sh[1][wv] = f;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const double pa = sh[0][0] + sh[0][1] + sh[0][2] + sh[0][3];
        const double pf = sh[1][0] + sh[1][1] + sh[1][2] + sh[1][3];
        if (Pihat) Pihat[(size_t)b * J + j] = pa;
        if (Phihat) Phihat[(size_t)b * J + j] = pf;
        if (E) E[(size_t)b * J + j] = pa * pa + pf * pf;
    }
}

}  // namespace

hipError_t launch_spectrum(int n_inst, const InstConst* ic, const double* Phi, const double* Pi, const double* A,
                           const double* const* wPi, const double* const* wPhi, int J, double* E,
                           double* Pihat, double* Phihat, hipStream_t s)
{
    spectrum_kernel<<<dim3(J, n_inst), dim3(256), 0, s>>>(n_inst, ic, Phi, Pi, A, wPi, wPhi, J, E, Pihat, Phihat);
    return hipGetLastError();
}

}  // namespace adscl
