// Projection of states on the linear AdS4 eigenmodes (Liebling & Khanna,
// arXiv:1706.07413, Sec. II: decomposition into normal modes), as FP64 matrix
// products on the MFMA units.
//
//   Pihat_rj = sum_i sqrt(A_ri) Pi_ri wPi[j][i],   Phihat_rj = sum_i sqrt(A_ri) Phi_ri wPhi[j][i],
//   E_rj = Pihat_rj^2 + Phihat_rj^2,
// with wPi = h tan^2 x e_j(x), wPhi = h tan^2 x e_j'(x)/omega_j (zero at both
// ends).  A row r is one state of one instance (an instance of the current
// batch, or an instance in one snapshot slot); rows of one grid size N form one
// (rows x N) . (N x J) product, evaluated in 16 x 16 output tiles with
// v_mfma_f64_16x16x4_f64: lane l supplies A[l % 16][l / 16] of the 16 x 4 block
// and B[l / 16][l % 16] of the 4 x 16 block, and holds accumulators
// D[l / 16 + 4 q][l % 16], q = 0..3.
#include <math.h>

#include "internal.h"

namespace adscl {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

// One workgroup of four wavefronts per (16-row tile, 16-mode tile); the
// wavefronts take interleaved 4-point slices of the contraction and their
// partial tiles are summed through LDS in a fixed order.
__global__ void __launch_bounds__(256) spectrum_mfma_kernel(const double* base, const SpecRow* rows, int n_rows,
                                                            int N, const double* wPi, const double* wPhi, int J,
                                                            double* E, double* Pihat, double* Phihat)
{
    __shared__ double part[3][8][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int i = lane & 15, kk = lane >> 4;
    const int r = blockIdx.x * 16 + i;  // row of the A operand this lane supplies
    const int j = blockIdx.y * 16 + i;  // mode of the B operand this lane supplies
    const bool vr = r < n_rows, vj = j < J;
    SpecRow R{0, 0, 0, 0};
    if (vr) R = rows[r];
    v4d cp = {0.0, 0.0, 0.0, 0.0}, cf = {0.0, 0.0, 0.0, 0.0};
    for (int k0 = 4 * wv; k0 < N; k0 += 16) {
        const int k = k0 + kk;
        double ap = 0.0, af = 0.0, bp = 0.0, bf = 0.0;
        if (k < N) {
            if (vr) {
                const double sA = sqrt(base[R.a + k]);
                ap = sA * base[R.pi + k];
                af = sA * base[R.phi + k];
            }
            if (vj) {
                bp = wPi[(size_t)j * N + k];
                bf = wPhi[(size_t)j * N + k];
            }
        }
        cp = __builtin_amdgcn_mfma_f64_16x16x4f64(ap, bp, cp, 0, 0, 0);
        cf = __builtin_amdgcn_mfma_f64_16x16x4f64(af, bf, cf, 0, 0, 0);
    }
    if (wv > 0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            part[wv - 1][q][lane] = cp[q];
            part[wv - 1][4 + q][lane] = cf[q];
        }
    }
    __syncthreads();
    if (wv != 0) return;
#pragma unroll
    for (int w = 0; w < 3; ++w) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            cp[q] += part[w][q][lane];
            cf[q] += part[w][4 + q][lane];
        }
    }
    // accumulator q of lane l is output row l / 16 + 4 q, column l % 16
    const int col = blockIdx.y * 16 + (lane & 15);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int row = blockIdx.x * 16 + (lane >> 4) + 4 * q;
        if (row < n_rows && col < J) {
            const size_t o = (size_t)rows[row].out * J + col;
            if (Pihat) Pihat[o] = cp[q];
            if (Phihat) Phihat[o] = cf[q];
            if (E) E[o] = cp[q] * cp[q] + cf[q] * cf[q];
        }
    }
}

}  // namespace

hipError_t launch_spectrum_rows(const double* base, const SpecRow* rows, int n_rows, int N, const double* wPi,
                                const double* wPhi, int J, double* E, double* Pihat, double* Phihat, hipStream_t s)
{
    if (n_rows <= 0) return hipSuccess;
    spectrum_mfma_kernel<<<dim3((n_rows + 15) / 16, (J + 15) / 16), dim3(256), 0, s>>>(base, rows, n_rows, N, wPi,
                                                                                        wPhi, J, E, Pihat, Phihat);
    return hipGetLastError();
}

}  // namespace adscl
