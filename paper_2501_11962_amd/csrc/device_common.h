// Device helpers shared by the kernel files.
#pragma once

#include "mop_internal.h"

namespace mop {

// Segment (path) that owns logical block `blk`; block prefixes are uniform, so this
// is a short scalar loop.
__device__ __forceinline__ int find_seg(const Launch& L, int blk) {
    int p = 0;
    while (p + 1 < L.nseg && L.pf[p + 1] <= blk) ++p;
    return p;
}

template <class T>
__device__ __forceinline__ T* wsp(char* ws, size_t off) {
    return reinterpret_cast<T*>(ws + off);
}

// Minimum image of a coordinate difference in a periodic box of length L.
__device__ __forceinline__ double min_img(double d, double L) { return d - L * rint(d / L); }

// Fixed-point coordinate: the box [0, L) maps onto [0, 2^32); wrap-around of unsigned
// differences is then exactly the minimum image.
__device__ __forceinline__ uint32_t to_fixed(double x, double L) {
    double t = x / L;
    t -= floor(t);
    const double v = t * 4294967296.0;
    return v >= 4294967295.0 ? 0xFFFFFFFFu : static_cast<uint32_t>(v);
}

// Column / z-bin index of a fixed-point coordinate among n equal bins.
__device__ __forceinline__ int fixed_bin(uint32_t u, int n) {
    return static_cast<int>((static_cast<uint64_t>(u) * static_cast<uint64_t>(n)) >> 32);
}

// Orders LDS traffic between the lanes of one wave: the compiler moves no memory
// access across it.  A wave's LDS instructions execute in issue order, so wavefront
// scope needs no wait for earlier LDS accesses to complete.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Value of lane (l ^ M) for lane l of a wave.  M < 32: a swizzle in bit mode (and-mask
// 0x1F, xor-mask M, within each half of the wave); M == 32: a permute across the halves.
// Unlike __shfl_xor these need no per-lane bound, which the compiler would otherwise keep
// in a register for the whole kernel.
template <int M>
__device__ __forceinline__ int lane_xor(int v) {
    static_assert(M > 0 && M <= 32 && (M & (M - 1)) == 0, "lane mask");
    if constexpr (M < 32) {
        return __builtin_amdgcn_ds_swizzle(v, 0x1F | (M << 10));
    } else {
        const int l = (int)__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
        return __builtin_amdgcn_ds_bpermute((l ^ 32) << 2, v);
    }
}
template <int M>
__device__ __forceinline__ float lane_xor(float v) {
    return __int_as_float(lane_xor<M>(__float_as_int(v)));
}
template <int M>
__device__ __forceinline__ double lane_xor(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = lane_xor<M>((int)(b & 0xFFFFFFFFll)), hi = lane_xor<M>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

__device__ __forceinline__ int wave_incl_scan(int v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int t = __shfl_up(v, d, 64);
        if (lane >= d) v += t;
    }
    return v;
}

// Sum over the 64 lanes of a wave (pairwise: lanes 32 apart first, then 16, ..., 1).
__device__ __forceinline__ double wave_sum(double v) {
    v += lane_xor<32>(v);
    v += lane_xor<16>(v);
    v += lane_xor<8>(v);
    v += lane_xor<4>(v);
    v += lane_xor<2>(v);
    v += lane_xor<1>(v);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
    v = fmax(v, lane_xor<32>(v));
    v = fmax(v, lane_xor<16>(v));
    v = fmax(v, lane_xor<8>(v));
    v = fmax(v, lane_xor<4>(v));
    v = fmax(v, lane_xor<2>(v));
    v = fmax(v, lane_xor<1>(v));
    return v;
}

// Block-wide sum of a double (blockDim.x == EWB), result valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* sh) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) s += sh[k];
    return s;
}

// Block-wide max of a double (blockDim.x == EWB), result valid in thread 0.
__device__ __forceinline__ double block_max(double v, double* sh) {
    v = wave_max(v);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) s = fmax(s, sh[k]);
    return s;
}

// Harmonic bonds of atom i in FP64 (each bond is listed for both of its atoms).
// Adds the force on i to f; adds k/2 (r - r0)^2 of bonds with partner j > i to *e.
__device__ __forceinline__ void bond_force(const SysDev& s, const double* Rb, const double* Db,
                                           double eps, int i, double f[3], double* e) {
    const int k0 = s.bstart[i], k1 = s.bstart[i + 1];
    if (k0 == k1) return;
    double xi[3];
    for (int a = 0; a < 3; ++a) {
        xi[a] = Rb[3 * (size_t)i + a];
        if (Db) xi[a] += eps * Db[3 * (size_t)i + a];
    }
    for (int k = k0; k < k1; ++k) {
        const int j = s.bpart[k];
        double d[3], r2 = 0.0;
        for (int a = 0; a < 3; ++a) {
            double xj = Rb[3 * (size_t)j + a];
            if (Db) xj += eps * Db[3 * (size_t)j + a];
            d[a] = min_img(xj - xi[a], s.L[a]);
            r2 += d[a] * d[a];
        }
        const double r = sqrt(r2), kb = s.bk[k], r0 = s.br0[k];
        const double g = kb * (1.0 - r0 / r);
        for (int a = 0; a < 3; ++a) f[a] += g * d[a];
        if (e && j > i) *e += 0.5 * kb * (r - r0) * (r - r0);
    }
}

// Bond part of (H v)_i in FP64: sum_k g (v_i - v_j) + h (d . (v_i - v_j)) d,
// g = k (1 - r0/r), h = k r0 / r^3.
__device__ __forceinline__ void bond_hvp(const SysDev& s, const double* Rb, const double* Vb,
                                         int i, double hv[3]) {
    const int k0 = s.bstart[i], k1 = s.bstart[i + 1];
    for (int k = k0; k < k1; ++k) {
        const int j = s.bpart[k];
        double d[3], dv[3], r2 = 0.0, sd = 0.0;
        for (int a = 0; a < 3; ++a) {
            d[a] = min_img(Rb[3 * (size_t)j + a] - Rb[3 * (size_t)i + a], s.L[a]);
            dv[a] = Vb[3 * (size_t)i + a] - Vb[3 * (size_t)j + a];
            r2 += d[a] * d[a];
            sd += d[a] * dv[a];
        }
        const double r = sqrt(r2), kb = s.bk[k], r0 = s.br0[k];
        const double g = kb * (1.0 - r0 / r);
        const double h = kb * r0 / (r2 * r);
        for (int a = 0; a < 3; ++a) hv[a] += g * dv[a] + h * sd * d[a];
    }
}

}  // namespace mop
