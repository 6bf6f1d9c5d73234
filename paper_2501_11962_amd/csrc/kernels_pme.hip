// Reciprocal part of particle-mesh Ewald electrostatics (smooth PME, Essmann et al.
// 1995), the long-range method of the paper's standard MD runs (Appendix A.1), with
// the exact Hessian-vector product the path gradient needs.
//
// Per pair bead b (one thread per atom for the particle kernels, grid-stride for the
// grid kernels):
//   spread   Q(k) = sum_i q_i theta_i(k)                      (charges, force pass)
//            dQ(k) = sum_i q_i grad theta_i(k) . v_i           (dipoles, Hessian pass)
//            theta_i(k) = M_p(u_ix - k_x) M_p(u_iy - k_y) M_p(u_iz - k_z), u = K frac(x/L).
//            Contributions are rounded to 64-bit fixed point and added with integer
//            atomics, so the grid (and everything after it) is the same on every call:
//            the scale is a power of two chosen so that no grid value can overflow
//            (sum |q| bounds every charge-grid value; sum |q| * 3 max(K/L) max|v_i|
//            every dipole-grid value).
//   convert  fixed point -> FP64 real grid (FFT input).
//   FFT      real-to-complex, multiply by f B(m) C(m) (solve, which also forms the
//            energy 1/2 sum_m f B C |Q^(m)|^2 over the half spectrum), complex-to-real:
//            phi = the grid potential.
//   gather   F_i = -q_i sum_k grad theta_i(k) phi(k)
//            (H v)_i = q_i sum_k [grad theta_i(k) . dphi(k) + (grad grad theta_i(k) v_i) phi(k)]
//            added to the pair kernels' FP32 results.
// Spline weights come from the recursion M_n(x) = [x M_{n-1}(x) + (n - x) M_{n-1}(x-1)]
// / (n - 1) started at M_2, in FP64 registers; M_n' = M_{n-1}(x) - M_{n-1}(x - 1) and
// M_n'' = M_{n-2}(x) - 2 M_{n-2}(x - 1) + M_{n-2}(x - 2) reuse the lower orders.
// All PME arithmetic is FP64.  The FFTs run in rocFFT (host side, mop_api.hip).
#include <algorithm>

#include "device_common.h"
#include "launch.h"

namespace mop {

namespace {

// Weights th[j] = M_P(w + j), j = 0..P-1, of fractional offset w in [0, 1), and (DER >= 1)
// first / (DER >= 2) second derivatives with respect to u.
template <int P, int DER>
__device__ __forceinline__ void bspline(double w, double* th, double* d1, double* d2) {
    double a[P], o1[P], o2[P];
#pragma unroll
    for (int j = 0; j < P; ++j) a[j] = o1[j] = o2[j] = 0.0;
    a[0] = w;          // M_2(w)
    a[1] = 1.0 - w;    // M_2(w + 1)
    if (P - 2 == 2) {
#pragma unroll
        for (int j = 0; j < P; ++j) o2[j] = a[j];
    }
#pragma unroll
    for (int n = 3; n <= P; ++n) {
        const double inv = 1.0 / (n - 1);
#pragma unroll
        for (int j = n - 1; j >= 0; --j) {
            const double left = j < n - 1 ? (w + j) * a[j] : 0.0;
            const double right = j > 0 ? (n - w - j) * a[j - 1] : 0.0;
            a[j] = (left + right) * inv;
        }
        if (n == P - 2) {
#pragma unroll
            for (int j = 0; j < P; ++j) o2[j] = a[j];
        }
        if (n == P - 1) {
#pragma unroll
            for (int j = 0; j < P; ++j) o1[j] = a[j];
        }
    }
#pragma unroll
    for (int j = 0; j < P; ++j) {
        th[j] = a[j];
        if (DER >= 1) d1[j] = o1[j] - (j > 0 ? o1[j - 1] : 0.0);
        if (DER >= 2)
            d2[j] = o2[j] - 2.0 * (j > 0 ? o2[j - 1] : 0.0) + (j > 1 ? o2[j - 2] : 0.0);
    }
}

// Grid indices (base - j mod K) and fractional offset of one coordinate.
template <int P>
__device__ __forceinline__ double grid_point(double x, double L, int K, int* idx) {
    double s = x / L;
    s -= floor(s);
    const double u = K * s;
    const double fb = floor(u);
    const double w = u - fb;
    // u = K (s rounded up to 1) wraps to 0; a non-finite coordinate keeps every index in
    // range (its NaN weights reach the forces, which the status word reports)
    const int base = (fb >= 0.0 && fb < (double)K) ? (int)fb : 0;
#pragma unroll
    for (int j = 0; j < P; ++j) {
        int k = base - j;
        if (k < 0) k += K;
        idx[j] = k;
    }
    return w;
}

// Fixed-point scale of the dipole grid of a bead whose largest |v_i|^2 is m2.
__device__ __forceinline__ double dipole_scale(const SysDev& s, double m2) {
    if (!(m2 > 0.0) || !isfinite(m2)) return 1.0;
    const double bound = s.vbound * sqrt(m2);
    if (!(bound > 0.0) || !isfinite(bound)) return 1.0;
    return ldexp(1.0, 61 - (ilogb(bound) + 1));
}

__device__ __forceinline__ double bead_m2(const SegDev& sg, char* ws, int b) {
    return __longlong_as_double((long long)wsp<const unsigned long long>(ws, sg.o_dmax)[b]);
}

// Position of atom i of bead b, displaced by fdsign * eps_b d^b_i for the
// finite-difference term.
__device__ __forceinline__ void atom_pos(const SegDev& sg, char* ws, const double* R, int b, int i,
                                         int fdsign, double fdh, double x[3]) {
    const int Q = sg.s.Q;
    const double* r = R + sg.roff + ((size_t)b * Q + i) * 3;
    x[0] = r[0];
    x[1] = r[1];
    x[2] = r[2];
    if (fdsign != 0) {
        const double m2 = bead_m2(sg, ws, b);
        const double eps = m2 > 0.0 ? fdsign * fdh / sqrt(m2) : 0.0;
        const double* d = wsp<const double>(ws, sg.o_d64) + ((size_t)b * Q + i) * 3;
        for (int a = 0; a < 3; ++a) x[a] += eps * d[a];
    }
}

}  // namespace

__global__ void __launch_bounds__(PME_BLOCK) k_pme_clear(const SegDev* __restrict__ segs,
                                                         size_t n, char* ws) {
    long long* g = wsp<long long>(ws, segs[0].o_pgi);
    for (size_t k = (size_t)blockIdx.x * PME_BLOCK + threadIdx.x; k < n;
         k += (size_t)gridDim.x * PME_BLOCK)
        g[k] = 0;
}

// KIND 0: charges of R (displaced with fdsign); KIND 1: dipoles q_i v_i (V: [nb][Q][3]).
template <int P, int KIND>
__global__ void __launch_bounds__(EWB) k_pme_spread(const SegDev* __restrict__ segs, int nb,
                                                    char* ws, const double* __restrict__ R,
                                                    const double* __restrict__ V, int fdsign,
                                                    double fdh) {
    const SegDev& sg = segs[0];
    const SysDev& s = sg.s;
    const int b = blockIdx.x / sg.bpb;
    const int i = (blockIdx.x - b * sg.bpb) * EWB + threadIdx.x;
    if (b >= nb || i >= s.Q) return;
    double x[3];
    atom_pos(sg, ws, R, b, i, fdsign, fdh, x);
    int ix[P], iy[P], iz[P];
    double tx[P], ty[P], tz[P], dx[P], dy[P], dz[P];
    bspline<P, KIND>(grid_point<P>(x[0], s.L[0], s.Kg[0], ix), tx, dx, nullptr);
    bspline<P, KIND>(grid_point<P>(x[1], s.L[1], s.Kg[1], iy), ty, dy, nullptr);
    bspline<P, KIND>(grid_point<P>(x[2], s.L[2], s.Kg[2], iz), tz, dz, nullptr);
    const size_t Kt = (size_t)s.Kg[0] * s.Kg[1] * s.Kg[2];
    unsigned long long* g = wsp<unsigned long long>(ws, sg.o_pgi) + (size_t)b * Kt;
    double c, vx = 0.0, vy = 0.0, vz = 0.0;
    if (KIND == 0) {
        c = s.qd[i] * s.qscale;
    } else {
        c = s.qd[i] * dipole_scale(s, bead_m2(sg, ws, b));
        const double* v = V + ((size_t)b * s.Q + i) * 3;
        vx = v[0] * s.kl[0];
        vy = v[1] * s.kl[1];
        vz = v[2] * s.kl[2];
    }
#pragma unroll
    for (int a = 0; a < P; ++a) {
#pragma unroll
        for (int e = 0; e < P; ++e) {
            const size_t row = ((size_t)ix[a] * s.Kg[1] + iy[e]) * s.Kg[2];
            double pxy, qx = 0.0, qy = 0.0;
            if (KIND == 0) {
                pxy = c * tx[a] * ty[e];
            } else {
                pxy = c * tx[a] * ty[e] * vz;          // times dz
                qx = c * dx[a] * ty[e] * vx;           // times tz
                qy = c * tx[a] * dy[e] * vy;           // times tz
            }
#pragma unroll
            for (int f = 0; f < P; ++f) {
                const double val = KIND == 0 ? pxy * tz[f] : fma(qx + qy, tz[f], pxy * dz[f]);
                atomicAdd(g + row + iz[f], (unsigned long long)__double2ll_rn(val));
            }
        }
    }
}

// Fixed point -> FP64 real grid for beads < nb; zeros for the rest of the FFT batch.
__global__ void __launch_bounds__(PME_BLOCK) k_pme_convert(const SegDev* __restrict__ segs,
                                                           int nb, int nbatch, char* ws, int kind) {
    const SegDev& sg = segs[0];
    const SysDev& s = sg.s;
    const size_t Kt = (size_t)s.Kg[0] * s.Kg[1] * s.Kg[2];
    const size_t n = (size_t)nbatch * Kt;
    const long long* gi = wsp<const long long>(ws, sg.o_pgi);
    double* gr = wsp<double>(ws, sg.o_pgr);
    for (size_t k = (size_t)blockIdx.x * PME_BLOCK + threadIdx.x; k < n;
         k += (size_t)gridDim.x * PME_BLOCK) {
        const int b = (int)(k / Kt);
        double v = 0.0;
        if (b < nb) {
            const double sc = kind == 0 ? s.qscale : dipole_scale(s, bead_m2(sg, ws, b));
            v = (double)gi[k] / sc;
        }
        gr[k] = v;
    }
}

// Spectrum times f B C; with want_e, per-block partials of 1/2 sum_m f B C |Q^(m)|^2
// (half spectrum: interior z frequencies count twice).
__global__ void __launch_bounds__(PME_BLOCK) k_pme_solve(const SegDev* __restrict__ segs, int nb,
                                                         char* ws, int want_e) {
    __shared__ double sh[PME_BLOCK / 64];
    const SegDev& sg = segs[0];
    const SysDev& s = sg.s;
    const int b = blockIdx.x / s.nsb;
    const int blk = blockIdx.x - b * s.nsb;
    if (b >= nb) return;
    const size_t Kc = (size_t)s.Kg[0] * s.Kg[1] * s.Kzh;
    const size_t m = (size_t)blk * PME_BLOCK + threadIdx.x;
    double e = 0.0;
    if (m < Kc) {
        double2* c = wsp<double2>(ws, sg.o_pgc) + (size_t)b * Kc + m;
        const double ph = s.phihat[m];
        double2 v = *c;
        if (want_e) {
            const int mz = (int)(m % (size_t)s.Kzh);
            const double w = (mz == 0 || 2 * mz == s.Kg[2]) ? 0.5 : 1.0;
            e = w * ph * (v.x * v.x + v.y * v.y);
        }
        v.x *= ph;
        v.y *= ph;
        *c = v;
    }
    if (want_e) {
        const double t = block_sum(e, sh);
        if (threadIdx.x == 0) wsp<double>(ws, sg.o_pep)[(size_t)b * s.nsb + blk] = t;
    }
}

// KIND 0: forces from phi (pphi, or pgr for displaced configurations) added to the
// float4 output (outsel 0: f32, 1: hv32, 2: f32m).  KIND 1: H v from pphi and the
// dipole potential in pgr, added to hv32.
template <int P, int KIND>
__global__ void __launch_bounds__(EWB) k_pme_gather(const SegDev* __restrict__ segs, int nb,
                                                    char* ws, const double* __restrict__ R,
                                                    const double* __restrict__ V, int fdsign,
                                                    double fdh, int outsel, int use_pgr) {
    const SegDev& sg = segs[0];
    const SysDev& s = sg.s;
    const int b = blockIdx.x / sg.bpb;
    const int i = (blockIdx.x - b * sg.bpb) * EWB + threadIdx.x;
    if (b >= nb || i >= s.Q) return;
    double x[3];
    atom_pos(sg, ws, R, b, i, fdsign, fdh, x);
    int ix[P], iy[P], iz[P];
    double tx[P], ty[P], tz[P], dx[P], dy[P], dz[P], hx[P], hy[P], hz[P];
    constexpr int DER = KIND == 0 ? 1 : 2;
    bspline<P, DER>(grid_point<P>(x[0], s.L[0], s.Kg[0], ix), tx, dx, hx);
    bspline<P, DER>(grid_point<P>(x[1], s.L[1], s.Kg[1], iy), ty, dy, hy);
    bspline<P, DER>(grid_point<P>(x[2], s.L[2], s.Kg[2], iz), tz, dz, hz);
    const size_t Kt = (size_t)s.Kg[0] * s.Kg[1] * s.Kg[2];
    const double* phi = wsp<const double>(ws, (KIND == 0 && use_pgr) ? sg.o_pgr : sg.o_pphi) +
                        (size_t)b * Kt;
    const double* dphi = wsp<const double>(ws, sg.o_pgr) + (size_t)b * Kt;
    double vx = 0.0, vy = 0.0, vz = 0.0;
    if (KIND == 1) {
        const double* v = V + ((size_t)b * s.Q + i) * 3;
        vx = v[0] * s.kl[0];
        vy = v[1] * s.kl[1];
        vz = v[2] * s.kl[2];
    }
    // accumulators: a* = sum grad theta * (phi or dphi); h* = curvature term
    double ax = 0.0, ay = 0.0, az = 0.0;
#pragma unroll
    for (int a = 0; a < P; ++a) {
#pragma unroll
        for (int e = 0; e < P; ++e) {
            const size_t row = ((size_t)ix[a] * s.Kg[1] + iy[e]) * s.Kg[2];
            const double txy = tx[a] * ty[e], dxy = dx[a] * ty[e], xdy = tx[a] * dy[e];
            double hxx = 0.0, hyy = 0.0, hxy = 0.0;
            if (KIND == 1) {
                hxx = hx[a] * ty[e];
                hyy = tx[a] * hy[e];
                hxy = dx[a] * dy[e];
            }
#pragma unroll
            for (int f = 0; f < P; ++f) {
                const size_t k = row + iz[f];
                if (KIND == 0) {
                    const double p = phi[k];
                    ax = fma(dxy * tz[f], p, ax);
                    ay = fma(xdy * tz[f], p, ay);
                    az = fma(txy * dz[f], p, az);
                } else {
                    const double p = phi[k], q = dphi[k];
                    // grad theta . dphi (per unit u; K/L applied below)
                    const double gx = dxy * tz[f], gy = xdy * tz[f], gz = txy * dz[f];
                    // (grad grad theta) v per unit u (v already scaled by K/L)
                    const double cx = hxx * tz[f] * vx + hxy * tz[f] * vy + dx[a] * ty[e] * dz[f] * vz;
                    const double cy = hxy * tz[f] * vx + hyy * tz[f] * vy + tx[a] * dy[e] * dz[f] * vz;
                    const double cz = dxy * dz[f] * vx + xdy * dz[f] * vy + txy * hz[f] * vz;
                    ax = fma(gx, q, fma(cx, p, ax));
                    ay = fma(gy, q, fma(cy, p, ay));
                    az = fma(gz, q, fma(cz, p, az));
                }
            }
        }
    }
    (void)hx;
    (void)hy;
    (void)hz;
    const double qi = s.qd[i];
    double o[3];
    if (KIND == 0) {
        o[0] = -qi * s.kl[0] * ax;
        o[1] = -qi * s.kl[1] * ay;
        o[2] = -qi * s.kl[2] * az;
    } else {
        o[0] = qi * s.kl[0] * ax;
        o[1] = qi * s.kl[1] * ay;
        o[2] = qi * s.kl[2] * az;
    }
    size_t off = sg.o_f32;
    if (outsel == 1) off = sg.o_hv32;
    else if (outsel == 2) off = sg.o_f32m;
    float4* out = wsp<float4>(ws, off) + (size_t)b * s.Q + i;
    float4 t = *out;
    t.x = (float)((double)t.x + o[0]);
    t.y = (float)((double)t.y + o[1]);
    t.z = (float)((double)t.z + o[2]);
    *out = t;
}

// Largest |v_i|^2 per bead into the per-bead max (zeroed by the binning), for the
// dipole scale of bead_hvp.
__global__ void __launch_bounds__(EWB) k_pme_vmax(const SegDev* __restrict__ segs, int nb, char* ws,
                                                  const double* __restrict__ V) {
    __shared__ double sh[EWB / 64];
    const SegDev& sg = segs[0];
    const int b = blockIdx.x / sg.bpb;
    const int i = (blockIdx.x - b * sg.bpb) * EWB + threadIdx.x;
    if (b >= nb) return;
    double m2 = 0.0;
    if (i < sg.s.Q) {
        const double* v = V + ((size_t)b * sg.s.Q + i) * 3;
        const double t = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
        if (isfinite(t)) m2 = t;
    }
    const double bm = block_max(m2, sh);
    if (threadIdx.x == 0)
        atomicMax(wsp<unsigned long long>(ws, sg.o_dmax) + b,
                  (unsigned long long)__double_as_longlong(bm));
}

// ---- launchers ----------------------------------------------------------------------

namespace {

int grid_blocks(size_t n) {
    const size_t b = (n + PME_BLOCK - 1) / PME_BLOCK;
    return (int)std::min<size_t>(b, 8192);
}

template <int P>
void spread_p(const SegDev* dsegs, const SegDev& h, int nb, char* ws, const double* R,
              const double* V, int kind, int fdsign, double fdh, hipStream_t st) {
    const dim3 grid(nb * h.bpb);
    if (kind == 0)
        hipLaunchKernelGGL((k_pme_spread<P, 0>), grid, dim3(EWB), 0, st, dsegs, nb, ws, R, V, fdsign, fdh);
    else
        hipLaunchKernelGGL((k_pme_spread<P, 1>), grid, dim3(EWB), 0, st, dsegs, nb, ws, R, V, fdsign, fdh);
}

template <int P>
void gather_p(const SegDev* dsegs, const SegDev& h, int nb, char* ws, const double* R,
              const double* V, int kind, int fdsign, double fdh, int outsel, int use_pgr,
              hipStream_t st) {
    const dim3 grid(nb * h.bpb);
    if (kind == 0)
        hipLaunchKernelGGL((k_pme_gather<P, 0>), grid, dim3(EWB), 0, st, dsegs, nb, ws, R, V, fdsign,
                           fdh, outsel, use_pgr);
    else
        hipLaunchKernelGGL((k_pme_gather<P, 1>), grid, dim3(EWB), 0, st, dsegs, nb, ws, R, V, fdsign,
                           fdh, outsel, use_pgr);
}

}  // namespace

void run_pme_spread(const SegDev* dsegs, const SegDev& h, int nb, char* ws, const double* R,
                    const double* V, int kind, int fdsign, double fdh, hipStream_t st) {
    const size_t Kt = (size_t)h.s.Kg[0] * h.s.Kg[1] * h.s.Kg[2];
    hipLaunchKernelGGL(k_pme_clear, dim3(grid_blocks((size_t)nb * Kt)), dim3(PME_BLOCK), 0, st,
                       dsegs, (size_t)nb * Kt, ws);
    switch (h.s.pme_p) {
        case 6: spread_p<6>(dsegs, h, nb, ws, R, V, kind, fdsign, fdh, st); break;
        case 8: spread_p<8>(dsegs, h, nb, ws, R, V, kind, fdsign, fdh, st); break;
        default: spread_p<4>(dsegs, h, nb, ws, R, V, kind, fdsign, fdh, st); break;
    }
}

void run_pme_convert(const SegDev* dsegs, const SegDev& h, int nb, int nbatch, char* ws, int kind,
                     hipStream_t st) {
    const size_t Kt = (size_t)h.s.Kg[0] * h.s.Kg[1] * h.s.Kg[2];
    hipLaunchKernelGGL(k_pme_convert, dim3(grid_blocks((size_t)nbatch * Kt)), dim3(PME_BLOCK), 0, st,
                       dsegs, nb, nbatch, ws, kind);
}

void run_pme_solve(const SegDev* dsegs, const SegDev& h, int nb, char* ws, int want_e,
                   hipStream_t st) {
    hipLaunchKernelGGL(k_pme_solve, dim3(nb * h.s.nsb), dim3(PME_BLOCK), 0, st, dsegs, nb, ws, want_e);
}

void run_pme_gather(const SegDev* dsegs, const SegDev& h, int nb, char* ws, const double* R,
                    const double* V, int kind, int fdsign, double fdh, int outsel, int use_pgr,
                    hipStream_t st) {
    switch (h.s.pme_p) {
        case 6: gather_p<6>(dsegs, h, nb, ws, R, V, kind, fdsign, fdh, outsel, use_pgr, st); break;
        case 8: gather_p<8>(dsegs, h, nb, ws, R, V, kind, fdsign, fdh, outsel, use_pgr, st); break;
        default: gather_p<4>(dsegs, h, nb, ws, R, V, kind, fdsign, fdh, outsel, use_pgr, st); break;
    }
}

void run_pme_vmax(const SegDev* dsegs, const SegDev& h, int nb, char* ws, const double* V,
                  hipStream_t st) {
    hipLaunchKernelGGL(k_pme_vmax, dim3(nb * h.bpb), dim3(EWB), 0, st, dsegs, nb, ws, V);
}

}  // namespace mop
