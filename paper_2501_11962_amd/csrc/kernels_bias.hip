// Metadynamics of paths (section 1.2): the end-to-end variable of eq. (8),
// S = s(R^N) - s(R^1), with s the distance between the centres of mass of atom groups A
// and B (section 3: ligand and binding pocket), and a Gaussian bias V(S) on it.
//
// One block per call (the groups are small):
//   1. centres of mass of A and B in beads 1 and N, each from the minimum-image offsets to
//      the group's first atom, FP64 block sums;
//   2. V(S) and dV/dS over the deposited Gaussians, FP64 block sums;
//   3. gradient of V added to G:  dV/dR^N = V'(S) ds/dR^N,  dV/dR^1 = -V'(S) ds/dR^1,
//      ds/dr_i = +m_i/M_B e (i in B), -m_i/M_A e (i in A), e the unit vector from A to B;
//   4. optionally a new Gaussian at S, height w0 or, well-tempered,
//      w0 exp(-V(S) / (kT (gamma - 1))); a full history sets the capacity status bit.
#include "device_common.h"
#include "launch.h"

namespace mop {

namespace {

constexpr int BIAS_THREADS = 256;

// Sums m_i mi(x_i - x_ref) over a group (3 components) and the group mass.
__device__ void group_moment(const double* X, const int* idx, int n, const double* minv,
                             const double L[3], double* sh, double out[4]) {
    const double* xr = X + 3 * (size_t)idx[0];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k = threadIdx.x; k < n; k += BIAS_THREADS) {
        const int i = idx[k];
        const double m = 1.0 / minv[i];
        for (int a = 0; a < 3; ++a) acc[a] += m * min_img(X[3 * (size_t)i + a] - xr[a], L[a]);
        acc[3] += m;
    }
    for (int a = 0; a < 4; ++a) {
        const double t = block_sum(acc[a], sh);
        if (threadIdx.x == 0) out[a] = t;
    }
}

}  // namespace

__global__ void __launch_bounds__(BIAS_THREADS) k_bias(BiasDev bd, const double* __restrict__ R,
                                                       int N, int Q, double* __restrict__ G,
                                                       double* __restrict__ out, int deposit,
                                                       int* __restrict__ status) {
    __shared__ double sh[BIAS_THREADS / 64];
    __shared__ double mom[4][4];    // [bead 1 A, bead 1 B, bead N A, bead N B][x, y, z, M]
    __shared__ double res[8];       // e1 (3), eN (3), dV/dS, V
    const double* R1 = R;
    const double* RN = R + (size_t)(N - 1) * Q * 3;
    group_moment(R1, bd.A, bd.nA, bd.minv, bd.L, sh, mom[0]);
    group_moment(R1, bd.B, bd.nB, bd.minv, bd.L, sh, mom[1]);
    group_moment(RN, bd.A, bd.nA, bd.minv, bd.L, sh, mom[2]);
    group_moment(RN, bd.B, bd.nB, bd.minv, bd.L, sh, mom[3]);
    __syncthreads();
    // s and e for bead 1 (k = 0) and bead N (k = 1), computed redundantly by every thread
    double s[2], e[2][3];
    for (int k = 0; k < 2; ++k) {
        const double* X = k == 0 ? R1 : RN;
        const double* ma = mom[2 * k];
        const double* mb = mom[2 * k + 1];
        double d2 = 0.0, d[3];
        for (int a = 0; a < 3; ++a) {
            const double ca = X[3 * (size_t)bd.A[0] + a] + ma[a] / ma[3];
            const double cb = X[3 * (size_t)bd.B[0] + a] + mb[a] / mb[3];
            d[a] = min_img(cb - ca, bd.L[a]);
            d2 += d[a] * d[a];
        }
        s[k] = sqrt(d2);
        for (int a = 0; a < 3; ++a) e[k][a] = d[a] / s[k];
    }
    const double S = s[1] - s[0];
    // V(S) and V'(S)
    const int ng = *bd.count;
    double v = 0.0, dv = 0.0;
    const double is2 = 1.0 / (bd.sigma * bd.sigma);
    for (int k = threadIdx.x; k < ng; k += BIAS_THREADS) {
        const double x = S - bd.centers[k];
        const double g = bd.heights[k] * exp(-0.5 * x * x * is2);
        v += g;
        dv -= x * is2 * g;
    }
    const double V = block_sum(v, sh);
    const double dV = block_sum(dv, sh);
    if (threadIdx.x == 0) {
        res[6] = dV;
        res[7] = V;
    }
    __syncthreads();
    const double dVs = res[6];
    // gradient: bead N gets +dV ds/dR^N, bead 1 gets -dV ds/dR^1
    if (G) {
        double* G1 = G;
        double* GN = G + (size_t)(N - 1) * Q * 3;
        const double MA0 = mom[0][3], MB0 = mom[1][3];
        for (int k = threadIdx.x; k < bd.nA; k += BIAS_THREADS) {
            const int i = bd.A[k];
            const double w = dVs / (bd.minv[i] * MA0);
            for (int a = 0; a < 3; ++a) {
                GN[3 * (size_t)i + a] -= w * e[1][a];
                G1[3 * (size_t)i + a] += w * e[0][a];
            }
        }
        for (int k = threadIdx.x; k < bd.nB; k += BIAS_THREADS) {
            const int i = bd.B[k];
            const double w = dVs / (bd.minv[i] * MB0);
            for (int a = 0; a < 3; ++a) {
                GN[3 * (size_t)i + a] += w * e[1][a];
                G1[3 * (size_t)i + a] -= w * e[0][a];
            }
        }
    }
    if (threadIdx.x == 0) {
        const double Vb = res[7];
        if (out) {
            out[0] = Vb;
            out[1] = S;
        }
        if (deposit) {
            if (ng < bd.capacity) {
                double w = bd.height;
                if (bd.bias_factor > 1.0) w *= exp(-Vb / (bd.kT * (bd.bias_factor - 1.0)));
                bd.centers[ng] = S;
                bd.heights[ng] = w;
                *bd.count = ng + 1;
            } else {
                atomicOr(status, ST_CAPACITY);
            }
        }
        if (!isfinite(S) || !isfinite(Vb)) atomicOr(status, ST_NONFINITE);
    }
}

// Clears the Gaussian history (a kernel, so that it can sit in a captured graph).
__global__ void k_bias_reset(int* count) { *count = 0; }

void run_bias(const BiasDev& bd, const double* R, int N, int Q, double* G, double* out,
              int deposit, int* status, hipStream_t st) {
    hipLaunchKernelGGL(k_bias, dim3(1), dim3(BIAS_THREADS), 0, st, bd, R, N, Q, G, out, deposit,
                       status);
}

void run_bias_reset(const BiasDev& bd, hipStream_t st) {
    hipLaunchKernelGGL(k_bias_reset, dim3(1), dim3(1), 0, st, bd.count);
}

}  // namespace mop
