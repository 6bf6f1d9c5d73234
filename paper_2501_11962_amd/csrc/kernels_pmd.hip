// Path molecular dynamics (eq. 4): the polymer of beads R^1..R^N moves under
// F_eff = -grad V_eff with fictitious masses M (read as the physical masses), by the
// splitting B A O A B with step tau:
//   k_pmd_pre   B (half kick with the gradient G of the current R), A (half drift),
//               O (Langevin: V <- c1 V + c2 xi / sqrt(M)), A (half drift)
//   [veff_grad on the new R: G and V_eff]
//   k_pmd_post  B (half kick with the new G) and per-block kinetic-energy partials
//   k_reduce_ke deterministic FP64 sum of the partials, per path
// With a metadynamics bias the gradient of each step includes the bias (kernels_bias.hip),
// added after the V_eff gradient and before the second half kick.
// With gamma = 0 (c1 = 1, c2 = 0) the O part is skipped and the step is velocity
// Verlet, the constant-energy integrator of appendix A.2; gamma > 0 is the Langevin
// thermostat of the constant-temperature runs.  All FP64, elementwise, HBM-bound:
// 72 bytes read and 48 written per atom and bead in k_pmd_pre, 48 + 24 in k_pmd_post.
//
// Normal deviates xi: Philox4x64-10 (Salmon, Moraes, Dror and Shaw, SC 2011) keyed by
// (seed, 0) on the counter (bead * Q + atom, step, 0, 0); outputs become uniforms
// (floor(x / 2^12) + 1/2) 2^-52 and pairs of uniforms go through Box-Muller
// (outputs 0, 1 -> x and y deviates, outputs 2, 3 -> z).
#include "device_common.h"
#include "launch.h"

namespace mop {

namespace {

constexpr uint64_t PHILOX_M0 = 0xD2E7470EE14C6C93ull;
constexpr uint64_t PHILOX_M1 = 0xCA5A826395121157ull;
constexpr uint64_t PHILOX_W0 = 0x9E3779B97F4A7C15ull;
constexpr uint64_t PHILOX_W1 = 0xBB67AE8584CAA73Bull;

__device__ __forceinline__ void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t hi0 = __umul64hi(PHILOX_M0, c[0]), lo0 = PHILOX_M0 * c[0];
        const uint64_t hi1 = __umul64hi(PHILOX_M1, c[2]), lo1 = PHILOX_M1 * c[2];
        const uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
        k0 += PHILOX_W0;
        k1 += PHILOX_W1;
    }
}

__device__ __forceinline__ double uniform52(uint64_t x) {
    return ((double)(x >> 12) + 0.5) * 0x1.0p-52;
}

// Three standard normal deviates for counter (idx, step) and key (seed, 0).
__device__ __forceinline__ void normals3(uint64_t idx, uint64_t step, uint64_t seed, double z[3]) {
    uint64_t c[4] = {idx, step, 0ull, 0ull};
    philox4x64_10(c, seed, 0ull);
    const double two_pi = 6.283185307179586476925286766559;
    const double r0 = sqrt(-2.0 * log(uniform52(c[0])));
    const double a0 = two_pi * uniform52(c[1]);
    const double r1 = sqrt(-2.0 * log(uniform52(c[2])));
    const double a1 = two_pi * uniform52(c[3]);
    z[0] = r0 * cos(a0);
    z[1] = r0 * sin(a0);
    z[2] = r1 * cos(a1);
}

}  // namespace

template <bool THERMO>
__global__ void __launch_bounds__(EWB) k_pmd_pre(const SegDev* __restrict__ segs, Launch L,
                                                 double* __restrict__ R, double* __restrict__ V,
                                                 const double* __restrict__ G, PmdCoef pc,
                                                 uint64_t step) {
    const int blk = blockIdx.x;
    const int p = find_seg(L, blk);
    const SegDev& sg = segs[p];
    const int local = blk - L.pf[p];
    const int n = local / sg.bpb;
    const int i = (local - n * sg.bpb) * EWB + threadIdx.x;
    const int Q = sg.s.Q;
    if (i >= Q) return;
    const size_t o = sg.roff + ((size_t)n * Q + i) * 3;
    const double minv = sg.s.minv[i];
    const double ht = 0.5 * pc.tau;
    double z[3] = {0.0, 0.0, 0.0};
    if (THERMO) normals3((uint64_t)n * (uint64_t)Q + (uint64_t)i, step, pc.seed, z);
    const double sn = pc.c2 * sqrt(minv);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double v = V[o + a] - ht * G[o + a] * minv;
        double r = R[o + a] + ht * v;
        if (THERMO) v = pc.c1 * v + sn * z[a];
        r += ht * v;
        R[o + a] = r;
        V[o + a] = v;
    }
}

__global__ void __launch_bounds__(EWB) k_pmd_post(const SegDev* __restrict__ segs, Launch L,
                                                  double* __restrict__ V,
                                                  const double* __restrict__ G, PmdCoef pc,
                                                  char* __restrict__ ws) {
    __shared__ double sh[EWB / 64];
    const int blk = blockIdx.x;
    const int p = find_seg(L, blk);
    const SegDev& sg = segs[p];
    const int local = blk - L.pf[p];
    const int n = local / sg.bpb;
    const int bi = local - n * sg.bpb;
    const int i = bi * EWB + threadIdx.x;
    const int Q = sg.s.Q;
    double ke = 0.0;
    if (i < Q) {
        const size_t o = sg.roff + ((size_t)n * Q + i) * 3;
        const double minv = sg.s.minv[i];
        const double ht = 0.5 * pc.tau;
        double v2 = 0.0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double v = V[o + a] - ht * G[o + a] * minv;
            V[o + a] = v;
            v2 += v * v;
        }
        ke = 0.5 * v2 / minv;
    }
    const double s = block_sum(ke, sh);
    if (threadIdx.x == 0) wsp<double>(ws, sg.o_rpart)[2 * ((size_t)n * sg.bpb + bi)] = s;
}

// One block per path: kinetic energy, and V_eff of the step from the reduction slot.
__global__ void __launch_bounds__(EWB) k_reduce_ke(const SegDev* __restrict__ segs, Launch L,
                                                   char* __restrict__ ws, double* __restrict__ out,
                                                   int stride, int has_bias) {
    __shared__ double sh[EWB / 64];
    const int p = blockIdx.x;
    const SegDev& sg = segs[p];
    const int N = L.N[p];
    const double* rp = wsp<const double>(ws, sg.o_rpart);
    double ke = 0.0;
    for (int k = threadIdx.x; k < N * sg.bpb; k += EWB) ke += rp[2 * k];
    const double s = block_sum(ke, sh);
    if (threadIdx.x == 0) {
        double* o = out + (size_t)sg.vidx * stride;
        o[0] = wsp<const double>(ws, sg.o_eres)[0];
        o[1] = s;
        if (!has_bias) {
            o[2] = 0.0;
            o[3] = 0.0;
        }
    }
}

void run_pmd_pre(const SegDev* dsegs, const SegDev* hsegs, const Launch& base, double* R, double* V,
                 const double* G, const PmdCoef& pc, uint64_t step, hipStream_t st) {
    Launch L = base;
    L.pf[0] = 0;
    for (int p = 0; p < base.nseg; ++p) L.pf[p + 1] = L.pf[p] + base.N[p] * hsegs[p].bpb;
    if (L.pf[L.nseg] == 0) return;
    if (pc.c2 > 0.0)
        hipLaunchKernelGGL(k_pmd_pre<true>, dim3(L.pf[L.nseg]), dim3(EWB), 0, st, dsegs, L, R, V,
                           G, pc, step);
    else
        hipLaunchKernelGGL(k_pmd_pre<false>, dim3(L.pf[L.nseg]), dim3(EWB), 0, st, dsegs, L, R, V,
                           G, pc, step);
}

void run_pmd_post(const SegDev* dsegs, const SegDev* hsegs, const Launch& base, double* V,
                  const double* G, const PmdCoef& pc, char* ws, double* energies, int stride,
                  int has_bias, hipStream_t st) {
    Launch L = base;
    L.pf[0] = 0;
    for (int p = 0; p < base.nseg; ++p) L.pf[p + 1] = L.pf[p] + base.N[p] * hsegs[p].bpb;
    if (L.pf[L.nseg] == 0) return;
    hipLaunchKernelGGL(k_pmd_post, dim3(L.pf[L.nseg]), dim3(EWB), 0, st, dsegs, L, V, G, pc, ws);
    if (energies)
        hipLaunchKernelGGL(k_reduce_ke, dim3(base.nseg), dim3(EWB), 0, st, dsegs, base, ws,
                           energies, stride, has_bias);
}

}  // namespace mop
