// Reciprocal part of particle-mesh Ewald electrostatics (smooth PME, Essmann et al.
// 1995), the long-range method of the paper's standard MD runs (Appendix A.1), with
// the exact Hessian-vector product the path gradient needs.
//
// Per pair bead b:
//   sort     atoms by the grid tile of their base point (counting sort; tiles of about
//            8^3 points), storing per atom, in tile order, its base point and atom index
//            (int4) and its fractional offsets and charge (double4): the spreading and
//            gathering kernels read these contiguously and never divide again.
//   spread   Q(k) = sum_i q_i theta_i(k)                      (charges, force pass)
//            dQ(k) = sum_i q_i grad theta_i(k) . v_i           (dipoles, Hessian pass)
//            theta_i(k) = M_p(u_ix - k_x) M_p(u_iy - k_y) M_p(u_iz - k_z), u = K frac(x/L).
//            One workgroup owns one tile: an atom with base point b touches points
//            b - p + 1 .. b along each axis, so the tile's points receive only from atoms
//            of the tile and of its upper neighbours (8 tiles).  Contributions are
//            rounded to 64-bit fixed point and summed with LDS integer atomics, so the
//            grid is the same on every call whatever the order; the owner then writes
//            its points to the real grid: FP64 for the charge grid, FP32 (the value
//            divided by the power-of-two dipole scale) for the dipole grid (no global
//            atomics, no clearing pass).  The
//            scale is a power of two chosen so that no value can overflow (sum |q|
//            bounds every charge-grid value; sum |q| * 3 max(K/L) max|v_i| every
//            dipole-grid value).
//   FFT      real-to-complex, multiply by f B(m) C(m) (solve, which also forms the
//            energy 1/2 sum_m f B C |Q^(m)|^2 over the half spectrum), complex-to-real:
//            phi = the grid potential.
//   gather   F_i = -q_i sum_k grad theta_i(k) phi(k)
//            (H v)_i = q_i sum_k [grad theta_i(k) . dphi(k) + (grad grad theta_i(k) v_i) phi(k)]
//            added to the pair kernels' FP32 results.
// Spline weights come from the recursion M_n(x) = [x M_{n-1}(x) + (n - x) M_{n-1}(x-1)]
// / (n - 1) started at M_2, in FP64 registers; M_n' = M_{n-1}(x) - M_{n-1}(x - 1) and
// M_n'' = M_{n-2}(x) - 2 M_{n-2}(x - 1) + M_{n-2}(x - 2) reuse the lower orders.
// Precision: spline weights, fixed-point spreading and the gathers' sums are FP64.  The
// charge grids of the force passes are transformed, solved and gathered in FP64 (forces
// and the energy).  The dipole grid of the Hessian pass is stored, transformed
// (single-precision rocFFT), solved and read back in FP32: that adds about 1e-6
// relative error to the mesh part of the Hessian-vector product, against the 1e-4
// tolerance of Hessian-vector products (measured against the FP64 oracle: Hessian-vector
// products of PME systems stay within 9e-7 relative L2 in total).  The FFTs run in
// rocFFT (host side, mop_api.hip).
#include <algorithm>

#include <type_traits>

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

// Base points and fractional offsets of a position (all three axes).
__device__ __forceinline__ void grid_base(const SysDev& s, const double x[3], int bse[3],
                                          double w[3]) {
    for (int a = 0; a < 3; ++a) {
        int idx[1];
        w[a] = grid_point<1>(x[a], s.L[a], s.Kg[a], idx);
        bse[a] = idx[0];
    }
}

// Grid indices base - j (mod K), j = 0..P-1.
template <int P>
__device__ __forceinline__ void support(int base, int K, int* idx) {
#pragma unroll
    for (int j = 0; j < P; ++j) {
        int k = base - j;
        if (k < 0) k += K;
        idx[j] = k;
    }
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

// Tile of each atom's base point and its rank in the tile (counts zeroed first).
__global__ void __launch_bounds__(EWB) k_pme_tile_count(const SegDev* __restrict__ segs, int nb,
                                                        char* ws, const double* __restrict__ R,
                                                        int fdsign, double fdh) {
    const SegDev& sg = segs[0];
    const SysDev& s = sg.s;
    const int b = blockIdx.x / sg.bpb;
    const int i = (blockIdx.x - b * sg.bpb) * EWB + threadIdx.x;
    if (b >= nb) return;
    const bool valid = i < s.Q;
    int tile = -1;
    if (valid) {
        double x[3], w[3];
        atom_pos(sg, ws, R, b, i, fdsign, fdh, x);
        int bse[3];
        grid_base(s, x, bse, w);
        tile = (s.tile_of[s.tof_off[0] + bse[0]] * s.ntl[1] + s.tile_of[s.tof_off[1] + bse[1]]) *
                   s.ntl[2] +
               s.tile_of[s.tof_off[2] + bse[2]];
    }
    // Neighbouring atoms mostly share a tile: one atomic per distinct tile of the wave,
    // ranks in lane order inside it.
    int* cnt = wsp<int>(ws, sg.o_ptc) + (size_t)b * s.ntile;
    const int lane = threadIdx.x & 63;
    unsigned long long todo = __ballot(valid);
    int rank = 0;
    while (todo) {
        const int leader = __ffsll((long long)todo) - 1;
        const int lt = __shfl(tile, leader, 64);
        const unsigned long long same = __ballot(tile == lt) & todo;
        int base = 0;
        if (lane == leader) base = atomicAdd(cnt + lt, (int)__popcll(same));
        base = __shfl(base, leader, 64);
        if (tile == lt)
            rank = base + (int)__builtin_amdgcn_mbcnt_hi((unsigned)(same >> 32),
                                                         __builtin_amdgcn_mbcnt_lo((unsigned)same, 0u));
        todo &= ~same;
    }
    if (valid) {
        wsp<int>(ws, sg.o_ptid)[(size_t)b * s.Q + i] = tile;
        wsp<int>(ws, sg.o_ptrk)[(size_t)b * s.Q + i] = rank;
    }
}

__global__ void __launch_bounds__(PME_BLOCK) k_pme_tile_zero(const SegDev* __restrict__ segs,
                                                             int n, char* ws) {
    const int k = blockIdx.x * PME_BLOCK + threadIdx.x;
    if (k < n) wsp<int>(ws, segs[0].o_ptc)[k] = 0;
}

// Exclusive scan of the tile counts of one bead per block.
constexpr int SCAN_BLOCK = 1024;
__global__ void __launch_bounds__(SCAN_BLOCK) k_pme_tile_scan(const SegDev* __restrict__ segs,
                                                              char* ws) {
    __shared__ int wsum[SCAN_BLOCK / 64];
    __shared__ int carry;
    const SegDev& sg = segs[0];
    const int nt = sg.s.ntile;
    const int b = blockIdx.x;
    const int* cnt = wsp<const int>(ws, sg.o_ptc) + (size_t)b * nt;
    int* start = wsp<int>(ws, sg.o_pts) + (size_t)b * (nt + 1);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < nt; base += SCAN_BLOCK) {
        const int k = base + threadIdx.x;
        const int v = k < nt ? cnt[k] : 0;
        const int incl = wave_incl_scan(v);
        if (lane == 63) wsum[w] = incl;
        __syncthreads();
        int off = carry;
        for (int u = 0; u < w; ++u) off += wsum[u];
        if (k < nt) start[k] = off + incl - v;
        __syncthreads();
        if (threadIdx.x == SCAN_BLOCK - 1) carry = off + incl;
        __syncthreads();
    }
    if (threadIdx.x == 0) start[nt] = carry;
}

__global__ void __launch_bounds__(EWB) k_pme_tile_scatter(const SegDev* __restrict__ segs, int nb,
                                                          char* ws, const double* __restrict__ R,
                                                          int fdsign, double fdh) {
    const SegDev& sg = segs[0];
    const SysDev& s = sg.s;
    const int b = blockIdx.x / sg.bpb;
    const int i = (blockIdx.x - b * sg.bpb) * EWB + threadIdx.x;
    if (b >= nb || i >= s.Q) return;
    const size_t o = (size_t)b * s.Q + i;
    const int tile = wsp<const int>(ws, sg.o_ptid)[o];
    const int st = wsp<const int>(ws, sg.o_pts)[(size_t)b * (s.ntile + 1) + tile];
    const size_t slot = (size_t)b * s.Q + st + wsp<const int>(ws, sg.o_ptrk)[o];
    double x[3], w[3];
    atom_pos(sg, ws, R, b, i, fdsign, fdh, x);
    int bse[3];
    grid_base(s, x, bse, w);
    wsp<int4>(ws, sg.o_ptb)[slot] = make_int4(bse[0], bse[1], bse[2], i);
    wsp<double4>(ws, sg.o_ptw)[slot] = make_double4(w[0], w[1], w[2], s.qd[i]);
}

// One workgroup per (bead, tile): KIND 0 charges of R (displaced with fdsign), KIND 1
// dipoles q_i v_i (V: [nb][Q][3]).  Beads nb .. nbatch-1 of the FFT batch get zeros.
constexpr int SPREAD_CAP = 1024;  // candidate list of the spreading kernel (LDS)

template <int P, int KIND>
__global__ void __launch_bounds__(PME_BLOCK) k_pme_spread(const SegDev* __restrict__ segs, int nb,
                                                          char* ws, const double* __restrict__ R,
                                                          const double* __restrict__ V, int fdsign,
                                                          double fdh) {
    extern __shared__ unsigned long long acc[];
    __shared__ int cand_k[SPREAD_CAP], cand_m[SPREAD_CAP];
    __shared__ int ncand;
    const SegDev& sg = segs[0];
    const SysDev& s = sg.s;
    const int b = blockIdx.x / s.ntile;
    const int t = blockIdx.x - b * s.ntile;
    const int tz = t % s.ntl[2], ty = (t / s.ntl[2]) % s.ntl[1], tx = t / (s.ntl[2] * s.ntl[1]);
    const int lo[3] = {s.tile_lo[s.tlo_off[0] + tx], s.tile_lo[s.tlo_off[1] + ty],
                       s.tile_lo[s.tlo_off[2] + tz]};
    const int ex = s.tile_lo[s.tlo_off[0] + tx + 1] - lo[0];
    const int ey = s.tile_lo[s.tlo_off[1] + ty + 1] - lo[1];
    const int ez = s.tile_lo[s.tlo_off[2] + tz + 1] - lo[2];
    const int npts = ex * ey * ez;
    for (int k = threadIdx.x; k < npts; k += PME_BLOCK) acc[k] = 0ull;
    __syncthreads();
    double scale = 1.0;
    if (b < nb) {
        scale = KIND == 0 ? s.qscale : dipole_scale(s, bead_m2(sg, ws, b));
        const int* start = wsp<const int>(ws, sg.o_pts) + (size_t)b * (s.ntile + 1);
        const int4* pb = wsp<const int4>(ws, sg.o_ptb) + (size_t)b * s.Q;
        const double4* pw = wsp<const double4>(ws, sg.o_ptw) + (size_t)b * s.Q;
        // Adds the listed atoms' contributions; lanes hold different atoms.
        auto flush = [&](int n) {
            for (int c = threadIdx.x; c < n; c += PME_BLOCK) {
                const int k = cand_k[c];
                const unsigned m = (unsigned)cand_m[c];
                const unsigned mx = m & 0xffu, my = (m >> 8) & 0xffu, mz = (m >> 16) & 0xffu;
                const int4 ab = pb[k];
                const int i = ab.w;
                int ix[P], iy[P], iz[P];
                support<P>(ab.x, s.Kg[0], ix);
                support<P>(ab.y, s.Kg[1], iy);
                support<P>(ab.z, s.Kg[2], iz);
                const double4 aw = pw[k];
                double tx_[P], ty_[P], tz_[P], dx_[P], dy_[P], dz_[P];
                bspline<P, KIND>(aw.x, tx_, dx_, nullptr);
                bspline<P, KIND>(aw.y, ty_, dy_, nullptr);
                bspline<P, KIND>(aw.z, tz_, dz_, nullptr);
                const double c0 = aw.w * scale;
                double vx = 0.0, vy = 0.0, vz = 0.0;
                if (KIND == 1) {
                    const double* v = V + ((size_t)b * s.Q + i) * 3;
                    vx = v[0] * s.kl[0];
                    vy = v[1] * s.kl[1];
                    vz = v[2] * s.kl[2];
                }
#pragma unroll
                for (int a = 0; a < P; ++a) {
                    if (!((mx >> a) & 1u)) continue;
#pragma unroll
                    for (int e = 0; e < P; ++e) {
                        if (!((my >> e) & 1u)) continue;
                        const int row = ((ix[a] - lo[0]) * ey + (iy[e] - lo[1])) * ez - lo[2];
                        double pxy, qx = 0.0, qy = 0.0;
                        if (KIND == 0) {
                            pxy = c0 * tx_[a] * ty_[e];
                        } else {
                            pxy = c0 * tx_[a] * ty_[e] * vz;     // times dz
                            qx = c0 * dx_[a] * ty_[e] * vx;      // times tz
                            qy = c0 * tx_[a] * dy_[e] * vy;      // times tz
                        }
#pragma unroll
                        for (int f = 0; f < P; ++f) {
                            if (!((mz >> f) & 1u)) continue;
                            const double val =
                                KIND == 0 ? pxy * tz_[f] : fma(qx + qy, tz_[f], pxy * dz_[f]);
                            atomicAdd(acc + row + iz[f], (unsigned long long)__double2ll_rn(val));
                        }
                    }
                }
            }
        };
        if (threadIdx.x == 0) ncand = 0;
        __syncthreads();
        const int lane = threadIdx.x & 63;
        const int nx = s.ntl[0] > 1 ? 2 : 1, ny = s.ntl[1] > 1 ? 2 : 1, nz = s.ntl[2] > 1 ? 2 : 1;
        for (int n = 0; n < nx * ny * nz; ++n) {
            const int ux = (tx + n / (ny * nz)) % s.ntl[0];
            const int uy = (ty + (n / nz) % ny) % s.ntl[1];
            const int uz = (tz + n % nz) % s.ntl[2];
            const int u = (ux * s.ntl[1] + uy) * s.ntl[2] + uz;
            for (int k0 = start[u]; k0 < start[u + 1]; k0 += PME_BLOCK) {
                // keep the atoms whose spline support meets this tile (list them in LDS)
                const int k = k0 + threadIdx.x;
                unsigned m = 0;
                if (k < start[u + 1]) {
                    const int4 ab = pb[k];
                    int ix[P], iy[P], iz[P];
                    support<P>(ab.x, s.Kg[0], ix);
                    support<P>(ab.y, s.Kg[1], iy);
                    support<P>(ab.z, s.Kg[2], iz);
                    unsigned mx = 0, my = 0, mz = 0;
#pragma unroll
                    for (int j = 0; j < P; ++j) {
                        mx |= (unsigned)(ix[j] >= lo[0] && ix[j] < lo[0] + ex) << j;
                        my |= (unsigned)(iy[j] >= lo[1] && iy[j] < lo[1] + ey) << j;
                        mz |= (unsigned)(iz[j] >= lo[2] && iz[j] < lo[2] + ez) << j;
                    }
                    if (mx && my && mz) m = mx | (my << 8) | (mz << 16);
                }
                const unsigned long long bal = __ballot(m != 0);
                int base = 0;
                if (lane == 0 && bal) base = atomicAdd(&ncand, (int)__popcll(bal));
                base = __shfl(base, 0, 64);
                if (m) {
                    const int pos = base + (int)__builtin_amdgcn_mbcnt_hi(
                                               (unsigned)(bal >> 32),
                                               __builtin_amdgcn_mbcnt_lo((unsigned)bal, 0u));
                    cand_k[pos] = k;
                    cand_m[pos] = (int)m;
                }
                __syncthreads();
                const int nc = ncand;
                __syncthreads();  // every thread has read the count before it changes again
                if (nc > SPREAD_CAP - PME_BLOCK) {  // room for one more round of appends
                    flush(nc);
                    __syncthreads();
                    if (threadIdx.x == 0) ncand = 0;
                    __syncthreads();
                }
            }
        }
        flush(ncand);
    }
    __syncthreads();
    // charges: FP64 grid; dipoles (Hessian pass, FP32 transforms): FP32 grid
    const size_t Kt = (size_t)s.Kg[0] * s.Kg[1] * s.Kg[2];
    using G = typename std::conditional<KIND == 0, double, float>::type;
    G* gr = wsp<G>(ws, sg.o_pgr) + (size_t)b * Kt;
    const double inv = 1.0 / scale;
    for (int k = threadIdx.x; k < npts; k += PME_BLOCK) {
        const int kz = k % ez, ky = (k / ez) % ey, kx = k / (ez * ey);
        const size_t g = ((size_t)(lo[0] + kx) * s.Kg[1] + (lo[1] + ky)) * s.Kg[2] + lo[2] + kz;
        gr[g] = b < nb ? (G)((double)(long long)acc[k] * inv) : (G)0;
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

// The same for the dipole grid of the Hessian pass, in FP32 (no energy).
__global__ void __launch_bounds__(PME_BLOCK) k_pme_solve32(const SegDev* __restrict__ segs, int nb,
                                                           char* ws) {
    const SegDev& sg = segs[0];
    const SysDev& s = sg.s;
    const int b = blockIdx.x / s.nsb;
    const int blk = blockIdx.x - b * s.nsb;
    if (b >= nb) return;
    const size_t Kc = (size_t)s.Kg[0] * s.Kg[1] * s.Kzh;
    const size_t m = (size_t)blk * PME_BLOCK + threadIdx.x;
    if (m < Kc) {
        float2* c = wsp<float2>(ws, sg.o_pgc) + (size_t)b * Kc + m;
        const float ph = (float)s.phihat[m];
        float2 v = *c;
        v.x *= ph;
        v.y *= ph;
        *c = v;
    }
}

// KIND 0: forces from phi (pphi, or pgr for displaced configurations); KIND 1: H v
// from pphi and the dipole potential in pgr (FP32).  outsel 0, 1, 2: added to the float4 pair
// output f32, hv32, f32m; outsel 3, 4: written to the FP64 buffer frec, hrec.
template <int P, int KIND>
__global__ void __launch_bounds__(EWB) k_pme_gather(const SegDev* __restrict__ segs, int nb,
                                                    char* ws, const double* __restrict__ R,
                                                    const double* __restrict__ V, int fdsign,
                                                    double fdh, int outsel, int use_pgr) {
    const SegDev& sg = segs[0];
    const SysDev& s = sg.s;
    const int b = blockIdx.x / sg.bpb;
    const int slot = (blockIdx.x - b * sg.bpb) * EWB + threadIdx.x;
    if (b >= nb || slot >= s.Q) return;
    // atoms in tile order: the lanes of a wave read neighbouring grid points
    const int4 ab = wsp<const int4>(ws, sg.o_ptb)[(size_t)b * s.Q + slot];
    const double4 aw = wsp<const double4>(ws, sg.o_ptw)[(size_t)b * s.Q + slot];
    const int i = ab.w;
    int ix[P], iy[P], iz[P];
    support<P>(ab.x, s.Kg[0], ix);
    support<P>(ab.y, s.Kg[1], iy);
    support<P>(ab.z, s.Kg[2], iz);
    double tx[P], ty[P], tz[P], dx[P], dy[P], dz[P], hx[P], hy[P], hz[P];
    constexpr int DER = KIND == 0 ? 1 : 2;
    bspline<P, DER>(aw.x, tx, dx, hx);
    bspline<P, DER>(aw.y, ty, dy, hy);
    bspline<P, DER>(aw.z, tz, dz, hz);
    const size_t Kt = (size_t)s.Kg[0] * s.Kg[1] * s.Kg[2];
    const double* phi = wsp<const double>(ws, (KIND == 0 && use_pgr) ? sg.o_pgr : sg.o_pphi) +
                        (size_t)b * Kt;
    const float* dphi = wsp<const float>(ws, sg.o_pgr) + (size_t)b * Kt;
    double vx = 0.0, vy = 0.0, vz = 0.0;
    if (KIND == 1) {
        const double* v = V + ((size_t)b * s.Q + i) * 3;
        vx = v[0] * s.kl[0];
        vy = v[1] * s.kl[1];
        vz = v[2] * s.kl[2];
    }
    // Sums over z first (per x-y pair of spline points), 32-bit grid indices:
    //   St = sum_f phi tz, Sd = sum_f phi dz, Sh = sum_f phi hz, Tt / Td the same of dphi.
    // Force:  a = sum_{a,e} (dx ty St, tx dy St, tx ty Sd)
    // H v:    a = sum_{a,e} grad(theta) . dphi + (grad grad theta) v phi, expanded by axis.
    double ax = 0.0, ay = 0.0, az = 0.0;
    const int K1 = s.Kg[1], K2 = s.Kg[2];
#pragma unroll
    for (int a = 0; a < P; ++a) {
#pragma unroll
        for (int e = 0; e < P; ++e) {
            const int row = (ix[a] * K1 + iy[e]) * K2;
            const double txy = tx[a] * ty[e], dxy = dx[a] * ty[e], xdy = tx[a] * dy[e];
            double St = 0.0, Sd = 0.0, Sh = 0.0, Tt = 0.0, Td = 0.0;
#pragma unroll
            for (int f = 0; f < P; ++f) {
                const double p = phi[row + iz[f]];
                St = fma(p, tz[f], St);
                Sd = fma(p, dz[f], Sd);
                if (KIND == 1) {
                    const double q = (double)dphi[row + iz[f]];
                    Sh = fma(p, hz[f], Sh);
                    Tt = fma(q, tz[f], Tt);
                    Td = fma(q, dz[f], Td);
                }
            }
            if (KIND == 0) {
                ax = fma(dxy, St, ax);
                ay = fma(xdy, St, ay);
                az = fma(txy, Sd, az);
            } else {
                const double hxx = hx[a] * ty[e], hyy = tx[a] * hy[e], hxy = dx[a] * dy[e];
                ax = fma(dxy, Tt, fma(fma(hxx, vx, hxy * vy), St, fma(dxy * vz, Sd, ax)));
                ay = fma(xdy, Tt, fma(fma(hxy, vx, hyy * vy), St, fma(xdy * vz, Sd, ay)));
                az = fma(txy, Td, fma(fma(dxy, vx, xdy * vy), Sd, fma(txy * vz, Sh, az)));
            }
        }
    }
    (void)hx;
    (void)hy;
    (void)hz;
    const double qi = aw.w;
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
    if (outsel >= 3) {
        double* d = wsp<double>(ws, outsel == 3 ? sg.o_frec : sg.o_hrec) + ((size_t)b * s.Q + i) * 3;
        d[0] = o[0];
        d[1] = o[1];
        d[2] = o[2];
        return;
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

template <int P>
void spread_p(const SegDev* dsegs, const SegDev& h, int nb, int nbatch, char* ws, const double* R,
              const double* V, int kind, int fdsign, double fdh, hipStream_t st) {
    const dim3 grid(nbatch * h.s.ntile);
    const size_t lds = (size_t)h.s.tile_pts * sizeof(unsigned long long);
    if (kind == 0)
        hipLaunchKernelGGL((k_pme_spread<P, 0>), grid, dim3(PME_BLOCK), lds, st, dsegs, nb, ws, R, V,
                           fdsign, fdh);
    else
        hipLaunchKernelGGL((k_pme_spread<P, 1>), grid, dim3(PME_BLOCK), lds, st, dsegs, nb, ws, R, V,
                           fdsign, fdh);
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

void run_pme_sort(const SegDev* dsegs, const SegDev& h, int nb, char* ws, const double* R,
                  int fdsign, double fdh, hipStream_t st) {
    const int n = nb * h.s.ntile;
    hipLaunchKernelGGL(k_pme_tile_zero, dim3((n + PME_BLOCK - 1) / PME_BLOCK), dim3(PME_BLOCK), 0, st,
                       dsegs, n, ws);
    hipLaunchKernelGGL(k_pme_tile_count, dim3(nb * h.bpb), dim3(EWB), 0, st, dsegs, nb, ws, R, fdsign,
                       fdh);
    hipLaunchKernelGGL(k_pme_tile_scan, dim3(nb), dim3(SCAN_BLOCK), 0, st, dsegs, ws);
    hipLaunchKernelGGL(k_pme_tile_scatter, dim3(nb * h.bpb), dim3(EWB), 0, st, dsegs, nb, ws, R,
                       fdsign, fdh);
}

void run_pme_spread(const SegDev* dsegs, const SegDev& h, int nb, int nbatch, char* ws,
                    const double* R, const double* V, int kind, int fdsign, double fdh,
                    hipStream_t st) {
    switch (h.s.pme_p) {
        case 6: spread_p<6>(dsegs, h, nb, nbatch, ws, R, V, kind, fdsign, fdh, st); break;
        case 8: spread_p<8>(dsegs, h, nb, nbatch, ws, R, V, kind, fdsign, fdh, st); break;
        default: spread_p<4>(dsegs, h, nb, nbatch, ws, R, V, kind, fdsign, fdh, st); break;
    }
}

void run_pme_solve(const SegDev* dsegs, const SegDev& h, int nb, char* ws, int want_e,
                   hipStream_t st) {
    hipLaunchKernelGGL(k_pme_solve, dim3(nb * h.s.nsb), dim3(PME_BLOCK), 0, st, dsegs, nb, ws, want_e);
}

void run_pme_solve32(const SegDev* dsegs, const SegDev& h, int nb, char* ws, hipStream_t st) {
    hipLaunchKernelGGL(k_pme_solve32, dim3(nb * h.s.nsb), dim3(PME_BLOCK), 0, st, dsegs, nb, ws);
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
