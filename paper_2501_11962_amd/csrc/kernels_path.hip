// FP64 path kernels (the seven kernels of section 2.1, fused differently):
//   k_resid     d^n = mi(R^{n+1} - R^n) - c F^n (kernel 1), spring energy (kernel 7),
//               bond forces/energy in FP64, FP32 slot-order copy of d^n for the HVP
//               pass, per-bead max |d^n|^2 for the finite-difference step.
//   k_assemble  G^n = -[n=1] F^1 + [n>=2] K d^{n-1} + [n<=N-1](-K d^n + 1/2 H d^n)
//               (kernels 4-6 as one gradient; F_eff = -G is eqs. 5-7), or with the
//               finite-difference term [F(R+eps d) - F(R-eps d)]/(4 eps) of eq. (5)
//               (kernels 2-3) in place of -1/2 H d.
//   k_reduce_*  deterministic FP64 sums of the per-block partials.
// All elementwise, HBM-bound; blocks never straddle beads (per-bead block counts).
#include "device_common.h"
#include "launch.h"

namespace mop {

__device__ __forceinline__ void flag(int* status, int bits) {
    if (bits) atomicOr(status, bits);
}

__device__ __forceinline__ bool finite3(double a, double b, double c) {
    return isfinite(a) && isfinite(b) && isfinite(c);
}

// PME systems: add the reciprocal-space force (or H v) of atom i of bead b, kept in FP64.
__device__ __forceinline__ void add_mesh(const SegDev& sg, char* ws, size_t off, int b, int i,
                                         double v[3]) {
    if (sg.s.elec != 1) return;
    const double* m = wsp<const double>(ws, off) + ((size_t)b * sg.s.Q + i) * 3;
    v[0] += m[0];
    v[1] += m[1];
    v[2] += m[2];
}

// want_dmax: also the per-bead max |d|^2 (finite-difference step, PME dipole-grid scale).
__global__ void __launch_bounds__(EWB) k_resid(const SegDev* __restrict__ segs, Launch L,
                                               CallPtrs cp, int want_dmax) {
    __shared__ double sh[3][EWB / 64];
    const int blk = blockIdx.x;
    const int p = find_seg(L, blk);
    const SegDev& sg = segs[p];
    const SysDev& s = sg.s;
    const int local = blk - L.pf[p];
    const int n = local / sg.bpb;
    const int bi = local - n * sg.bpb;
    const int i = bi * EWB + threadIdx.x;
    const int Q = s.Q, N = L.N[p];
    char* ws = cp.ws;
    double es = 0.0, eb = 0.0, d2max = 0.0;
    if (i < Q) {
        const double* Rn = cp.R + sg.roff + (size_t)n * Q * 3;
        const float4 fp = wsp<const float4>(ws, sg.o_f32)[(size_t)n * Q + i];
        double f[3] = {fp.x, fp.y, fp.z};
        add_mesh(sg, ws, sg.o_frec, n, i, f);
        bond_force(s, Rn, nullptr, 0.0, i, f, n == 0 ? &eb : nullptr);
        if (n < N - 1) {
            const double* Rn1 = Rn + (size_t)Q * 3;
            const double ci = s.c[i], Ki = s.K[i];
            double d[3];
            for (int a = 0; a < 3; ++a)
                d[a] = min_img(Rn1[3 * (size_t)i + a] - Rn[3 * (size_t)i + a], s.L[a]) - ci * f[a];
            double* d64 = wsp<double>(ws, sg.o_d64) + ((size_t)n * Q + i) * 3;
            d64[0] = d[0];
            d64[1] = d[1];
            d64[2] = d[2];
            const int slot = wsp<const int>(ws, sg.o_slotof)[(size_t)n * Q + i];
            wsp<float4>(ws, sg.o_vs)[(size_t)n * s.S + slot] =
                make_float4((float)d[0], (float)d[1], (float)d[2], 0.0f);
            const double d2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            es = 0.5 * Ki * d2;
            if (!finite3(d[0], d[1], d[2])) flag(cp.status, ST_NONFINITE);
            else d2max = d2;
        } else if (!finite3(f[0], f[1], f[2])) {
            flag(cp.status, ST_NONFINITE);
        }
    }
    // the three block reductions share one barrier (same summation order as block_sum)
    es = wave_sum(es);
    eb = wave_sum(eb);
    d2max = wave_max(d2max);
    if ((threadIdx.x & 63) == 0) {
        sh[0][threadIdx.x >> 6] = es;
        sh[1][threadIdx.x >> 6] = eb;
        sh[2][threadIdx.x >> 6] = d2max;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double ses = 0.0, seb = 0.0, smax = 0.0;
        for (int k = 0; k < EWB / 64; ++k) {
            ses += sh[0][k];
            seb += sh[1][k];
            smax = fmax(smax, sh[2][k]);
        }
        double* rp = wsp<double>(ws, sg.o_rpart) + 2 * ((size_t)n * sg.bpb + bi);
        rp[0] = ses;
        rp[1] = seb;
        // non-negative doubles order like their bit patterns
        if (want_dmax && n < N - 1)
            atomicMax(wsp<unsigned long long>(ws, sg.o_dmax) + n,
                      (unsigned long long)__double_as_longlong(smax));
    }
}

__global__ void __launch_bounds__(EWB) k_assemble(const SegDev* __restrict__ segs, Launch L,
                                                  CallPtrs cp, int fd) {
    const int blk = blockIdx.x;
    const int p = find_seg(L, blk);
    const SegDev& sg = segs[p];
    const SysDev& s = sg.s;
    const int local = blk - L.pf[p];
    const int n = local / sg.bpb;
    const int i = (local - n * sg.bpb) * EWB + threadIdx.x;
    const int Q = s.Q, N = L.N[p];
    if (i >= Q) return;
    char* ws = cp.ws;
    const double Ki = s.K[i];
    const double* d64 = wsp<const double>(ws, sg.o_d64);
    double g[3] = {0.0, 0.0, 0.0};
    if (n == 0) {
        const float4 fp = wsp<const float4>(ws, sg.o_f32)[i];
        double f[3] = {fp.x, fp.y, fp.z};
        add_mesh(sg, ws, sg.o_frec, 0, i, f);
        bond_force(s, cp.R + sg.roff, nullptr, 0.0, i, f, nullptr);
        for (int a = 0; a < 3; ++a) g[a] -= f[a];
    }
    if (n >= 1) {
        const double* dm = d64 + ((size_t)(n - 1) * Q + i) * 3;
        for (int a = 0; a < 3; ++a) g[a] += Ki * dm[a];
    }
    if (n <= N - 2) {
        const double* Rn = cp.R + sg.roff + (size_t)n * Q * 3;
        const double* Dn = d64 + (size_t)n * Q * 3;
        const double* dn = Dn + (size_t)i * 3;
        for (int a = 0; a < 3; ++a) g[a] -= Ki * dn[a];
        if (!fd) {
            const float4 hp = wsp<const float4>(ws, sg.o_hv32)[(size_t)n * Q + i];
            double hv[3] = {hp.x, hp.y, hp.z};
            add_mesh(sg, ws, sg.o_hrec, n, i, hv);
            bond_hvp(s, Rn, Dn, i, hv);
            for (int a = 0; a < 3; ++a) g[a] += 0.5 * hv[a];
        } else {
            const double m2 = __longlong_as_double(
                (long long)wsp<const unsigned long long>(ws, sg.o_dmax)[n]);
            if (m2 > 0.0) {
                const double eps = cp.fd_h / sqrt(m2);
                const float4 fpp = wsp<const float4>(ws, sg.o_hv32)[(size_t)n * Q + i];
                const float4 fmm = wsp<const float4>(ws, sg.o_f32m)[(size_t)n * Q + i];
                double fpl[3] = {fpp.x, fpp.y, fpp.z}, fmi[3] = {fmm.x, fmm.y, fmm.z};
                bond_force(s, Rn, Dn, eps, i, fpl, nullptr);
                bond_force(s, Rn, Dn, -eps, i, fmi, nullptr);
                for (int a = 0; a < 3; ++a) g[a] -= (fpl[a] - fmi[a]) / (4.0 * eps);
            }
        }
    }
    double* G = cp.G + sg.roff + ((size_t)n * Q + i) * 3;
    G[0] = g[0];
    G[1] = g[1];
    G[2] = g[2];
    if (!finite3(g[0], g[1], g[2])) flag(cp.status, ST_NONFINITE);
}

// Sum of the per-cluster pair-energy partials of bead b (weights applied in the kernel).
__device__ double pair_energy_of_bead(const SegDev& sg, char* ws, int b, int t0, int stride) {
    const int ncol = sg.s.ncol;
    const int nslots = wsp<const int>(ws, sg.o_colstart)[(size_t)b * (ncol + 1) + ncol];
    const int ncl = nslots / CLUSTER;
    const double* ep = wsp<const double>(ws, sg.o_epart) + (size_t)b * sg.s.cpb;
    double e0 = 0.0, e1 = 0.0;
    int c = t0;
    for (; c + stride < ncl; c += 2 * stride) {  // two independent chains in flight
        e0 += ep[c];
        e1 += ep[c + stride];
    }
    if (c < ncl) e0 += ep[c];
    return e0 + e1;
}

// This thread's share of the PME reciprocal energy of bead b (partials of the solve
// kernel, already halved); 0 without PME.
__device__ double pme_energy_of_bead(const SegDev& sg, char* ws, int b, int t0, int stride) {
    if (sg.s.elec != 1) return 0.0;
    const double* ep = wsp<const double>(ws, sg.o_pep) + (size_t)b * sg.s.nsb;
    double e = 0.0;
    for (int k = t0; k < sg.s.nsb; k += stride) e += ep[k];
    return e;
}

// Block-wide sum over RVB threads (result valid in thread 0).
constexpr int RVB = 1024;
__device__ __forceinline__ double block_sum_rvb(double v, double* sh) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < RVB / 64; ++k) s += sh[k];
    return s;
}

// One block per path: V_eff = U(R^1) + E_spring.
__global__ void __launch_bounds__(RVB) k_reduce_veff(const SegDev* __restrict__ segs, Launch L,
                                                     CallPtrs cp) {
    __shared__ double sh[RVB / 64];
    const int p = blockIdx.x;
    const SegDev& sg = segs[p];
    char* ws = cp.ws;
    const int N = L.N[p];
    const int nbr = N > 1 ? N - 1 : 1;
    const double* rp = wsp<const double>(ws, sg.o_rpart);
    double es = 0.0, eb = 0.0;
    for (int k = threadIdx.x; k < nbr * sg.bpb; k += RVB) es += rp[2 * k];
    for (int k = threadIdx.x; k < sg.bpb; k += RVB) eb += rp[2 * k + 1];
    const double ep = pair_energy_of_bead(sg, ws, 0, threadIdx.x, RVB) +
                      pme_energy_of_bead(sg, ws, 0, threadIdx.x, RVB);
    const double S_es = block_sum_rvb(es, sh);
    const double S_u = block_sum_rvb(eb + ep, sh) + (sg.s.elec == 1 ? sg.s.e_const : 0.0);
    if (threadIdx.x == 0) {
        double* er = wsp<double>(ws, sg.o_eres);
        er[0] = S_u + S_es;
        er[1] = S_u;
        er[2] = S_es;
        if (cp.veff) cp.veff[sg.vidx] = S_u + S_es;
        if (cp.u1) cp.u1[sg.vidx] = S_u;
        if (cp.espring) cp.espring[sg.vidx] = S_es;
        if (!isfinite(S_u + S_es)) flag(cp.status, ST_NONFINITE);
    }
}

// bead_forces: F = F_pair + F_bond (FP64 sum, FP32 out); bond energies per block.
__global__ void __launch_bounds__(EWB) k_finalize_forces(const SegDev* __restrict__ segs, Launch L,
                                                         CallPtrs cp) {
    __shared__ double sh[EWB / 64];
    const int blk = blockIdx.x;
    const int p = find_seg(L, blk);
    const SegDev& sg = segs[p];
    const int local = blk - L.pf[p];
    const int b = local / sg.bpb;
    const int bi = local - b * sg.bpb;
    const int i = bi * EWB + threadIdx.x;
    const int Q = sg.s.Q;
    double eb = 0.0;
    if (i < Q) {
        const float4 fp = wsp<const float4>(cp.ws, sg.o_f32)[(size_t)b * Q + i];
        double f[3] = {fp.x, fp.y, fp.z};
        add_mesh(sg, cp.ws, sg.o_frec, b, i, f);
        bond_force(sg.s, cp.R + sg.roff + (size_t)b * Q * 3, nullptr, 0.0, i, f, &eb);
        float* o = cp.Fout + sg.roff + ((size_t)b * Q + i) * 3;
        o[0] = (float)f[0];
        o[1] = (float)f[1];
        o[2] = (float)f[2];
        if (!finite3(f[0], f[1], f[2])) flag(cp.status, ST_NONFINITE);
    }
    const double s = block_sum(eb, sh);
    if (threadIdx.x == 0) wsp<double>(cp.ws, sg.o_rpart)[2 * ((size_t)b * sg.bpb + bi) + 1] = s;
}

// bead_forces energies: one block per (path, bead).
__global__ void __launch_bounds__(EWB) k_reduce_beads(const SegDev* __restrict__ segs, Launch L,
                                                      CallPtrs cp) {
    __shared__ double sh[EWB / 64];
    const int blk = blockIdx.x;
    const int p = find_seg(L, blk);
    const SegDev& sg = segs[p];
    const int b = blk - L.pf[p];
    const double* rp = wsp<const double>(cp.ws, sg.o_rpart);
    double eb = 0.0;
    for (int k = threadIdx.x; k < sg.bpb; k += EWB) eb += rp[2 * ((size_t)b * sg.bpb + k) + 1];
    const double ep = pair_energy_of_bead(sg, cp.ws, b, threadIdx.x, EWB) +
                      pme_energy_of_bead(sg, cp.ws, b, threadIdx.x, EWB);
    const double s = block_sum(eb + ep, sh);
    if (threadIdx.x == 0) cp.Uout[sg.vidx + b] = s + (sg.s.elec == 1 ? sg.s.e_const : 0.0);
}

// bead_hvp: vector in slot order, FP32.
__global__ void __launch_bounds__(EWB) k_prep_v(const SegDev* __restrict__ segs, Launch L, CallPtrs cp) {
    const int blk = blockIdx.x;
    const int p = find_seg(L, blk);
    const SegDev& sg = segs[p];
    const int local = blk - L.pf[p];
    const int b = local / sg.bpb;
    const int i = (local - b * sg.bpb) * EWB + threadIdx.x;
    const int Q = sg.s.Q;
    if (i >= Q) return;
    const double* v = cp.V + sg.roff + ((size_t)b * Q + i) * 3;
    const int slot = wsp<const int>(cp.ws, sg.o_slotof)[(size_t)b * Q + i];
    wsp<float4>(cp.ws, sg.o_vs)[(size_t)b * sg.s.S + slot] =
        make_float4((float)v[0], (float)v[1], (float)v[2], 0.0f);
}

// bead_hvp: H v = (H v)_pair + (H v)_bond (FP64 sum, FP32 out).
__global__ void __launch_bounds__(EWB) k_finalize_hvp(const SegDev* __restrict__ segs, Launch L,
                                                      CallPtrs cp) {
    const int blk = blockIdx.x;
    const int p = find_seg(L, blk);
    const SegDev& sg = segs[p];
    const int local = blk - L.pf[p];
    const int b = local / sg.bpb;
    const int i = (local - b * sg.bpb) * EWB + threadIdx.x;
    const int Q = sg.s.Q;
    if (i >= Q) return;
    const float4 hp = wsp<const float4>(cp.ws, sg.o_hv32)[(size_t)b * Q + i];
    double hv[3] = {hp.x, hp.y, hp.z};
    add_mesh(sg, cp.ws, sg.o_hrec, b, i, hv);
    bond_hvp(sg.s, cp.R + sg.roff + (size_t)b * Q * 3, cp.V + sg.roff + (size_t)b * Q * 3, i, hv);
    float* o = cp.Fout + sg.roff + ((size_t)b * Q + i) * 3;
    o[0] = (float)hv[0];
    o[1] = (float)hv[1];
    o[2] = (float)hv[2];
    if (!finite3(hv[0], hv[1], hv[2])) flag(cp.status, ST_NONFINITE);
}

__global__ void k_status_clear(int* status) { *status = 0; }
__global__ void k_status_copy(const int* status, int* out) { *out = *status; }

// ---- launchers ----------------------------------------------------------------------

static Launch per_bead_blocks(const Launch& base, const SegDev* hsegs, bool resid_beads,
                              bool all_beads) {
    Launch L = base;
    L.pf[0] = 0;
    for (int p = 0; p < base.nseg; ++p) {
        int nbeads = base.nb[p];
        if (resid_beads) nbeads = base.N[p] > 1 ? base.N[p] - 1 : 1;
        if (all_beads) nbeads = base.N[p];
        L.pf[p + 1] = L.pf[p] + nbeads * hsegs[p].bpb;
    }
    return L;
}

void run_resid(const SegDev* dsegs, const SegDev* hsegs, const Launch& base, const CallPtrs& cp,
               int want_dmax, hipStream_t st) {
    const Launch L = per_bead_blocks(base, hsegs, true, false);
    hipLaunchKernelGGL(k_resid, dim3(L.pf[L.nseg]), dim3(EWB), 0, st, dsegs, L, cp, want_dmax);
}

void run_assemble(const SegDev* dsegs, const SegDev* hsegs, const Launch& base, const CallPtrs& cp,
                  int fd, hipStream_t st) {
    const Launch L = per_bead_blocks(base, hsegs, false, true);
    hipLaunchKernelGGL(k_assemble, dim3(L.pf[L.nseg]), dim3(EWB), 0, st, dsegs, L, cp, fd);
}

void run_reduce_veff(const SegDev* dsegs, const SegDev* hsegs, const Launch& base,
                     const CallPtrs& cp, hipStream_t st) {
    (void)hsegs;
    hipLaunchKernelGGL(k_reduce_veff, dim3(base.nseg), dim3(RVB), 0, st, dsegs, base, cp);
}

void run_finalize_forces(const SegDev* dsegs, const SegDev* hsegs, const Launch& base,
                         const CallPtrs& cp, hipStream_t st) {
    const Launch L = per_bead_blocks(base, hsegs, false, false);
    hipLaunchKernelGGL(k_finalize_forces, dim3(L.pf[L.nseg]), dim3(EWB), 0, st, dsegs, L, cp);
    if (cp.Uout) {
        Launch Lb = base;
        Lb.pf[0] = 0;
        for (int p = 0; p < base.nseg; ++p) Lb.pf[p + 1] = Lb.pf[p] + base.nb[p];
        hipLaunchKernelGGL(k_reduce_beads, dim3(Lb.pf[Lb.nseg]), dim3(EWB), 0, st, dsegs, Lb, cp);
    }
}

void run_prep_v(const SegDev* dsegs, const SegDev* hsegs, const Launch& base, const CallPtrs& cp,
                hipStream_t st) {
    const Launch L = per_bead_blocks(base, hsegs, false, false);
    hipLaunchKernelGGL(k_prep_v, dim3(L.pf[L.nseg]), dim3(EWB), 0, st, dsegs, L, cp);
}

void run_finalize_hvp(const SegDev* dsegs, const SegDev* hsegs, const Launch& base,
                      const CallPtrs& cp, hipStream_t st) {
    const Launch L = per_bead_blocks(base, hsegs, false, false);
    hipLaunchKernelGGL(k_finalize_hvp, dim3(L.pf[L.nseg]), dim3(EWB), 0, st, dsegs, L, cp);
}

void run_status_copy(const int* status, int* out, hipStream_t st) {
    hipLaunchKernelGGL(k_status_copy, dim3(1), dim3(1), 0, st, status, out);
}

void run_status_clear(int* status, hipStream_t st) {
    hipLaunchKernelGGL(k_status_clear, dim3(1), dim3(1), 0, st, status);
}

}  // namespace mop
