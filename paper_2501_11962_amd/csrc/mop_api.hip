// Host runtime behind include/mop.h: validation, device tables, plan geometry,
// workspace layout and the call sequences of every entry point.
#include <hip/hip_runtime.h>
#include <rocfft/rocfft.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <map>
#include <vector>

#include "../../include/mop.h"
#include "launch.h"
#include "mop_internal.h"

using namespace mop;

namespace {

constexpr double F_ELEC = 138.935458;  // kJ mol^-1 nm e^-2
// nm added to the cutoff for neighbour pruning; displacements of up to half of it keep a
// recorded neighbour list exact (the shared-bin finite differences replay the lists of R
// for R +/- eps d with max |eps d_i| = fd_h)
constexpr double SEARCH_MARGIN = 2.0e-4;
constexpr double PI = 3.14159265358979323846;
constexpr double PME_SPACING = 0.12;      // nm per grid point of the automatic PME grid

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

template <class T>
T* wsp_host(char* ws, size_t off) {
    return reinterpret_cast<T*>(ws + off);
}

// Batched double-precision 3-D real FFTs of one PME grid shape (rocFFT).
struct PmeFft {
    rocfft_plan fwd = nullptr, bwd = nullptr;      // FP64: charges (force passes)
    rocfft_plan fwd32 = nullptr, bwd32 = nullptr;  // FP32: dipoles (Hessian pass)
    rocfft_execution_info info = nullptr;
    size_t work = 0;
};

}  // namespace

// Workspace of bead_forces_static, for callers that cannot allocate device memory: one
// copy per device, held until the process ends, shared by every such call on that device.
constexpr size_t SCRATCH_BYTES = MOP_STATIC_WORKSPACE_BYTES;
static __device__ __align__(256) char scratch[SCRATCH_BYTES];

struct mop_ctx_s {
    int device;
    hipStream_t stream;
    char* scratch;        // device address of this device's copy of `scratch` (or null)
};

struct mop_system_s {
    mop_ctx ctx;
    SysDev dev;           // device pointers; geometry fields filled per plan
    double box[3];
    double rc;
    double beta;          // PME systems
    std::vector<void*> allocs;
};

struct mop_plan_s {
    mop_system sys;
    int max_beads;
    int waves;
    int newton3;
    SegDev hseg;          // single-path layout (capacity max_beads)
    SegDev* dseg;
    size_t ws_bytes;
    PmeFft fft;           // PME systems
    mutable bool fft_failed = false;  // a transform could not be enqueued (reported by the call)
    // PME systems: the mesh work runs on a second stream, forked from and joined to the
    // context stream with events, concurrently with the pair kernels (unless one_stream)
    int one_stream = 0;
    hipStream_t side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
};

struct mop_bias_s {
    mop_plan plan;
    BiasDev dev;
    int stride;
    std::vector<void*> allocs;
};

struct mop_batch_s {
    mop_ctx ctx;
    int P;
    int waves;
    int newton3;
    std::vector<int> N;
    std::vector<SegDev> hsegs;
    SegDev* dsegs;
    size_t ws_bytes;
};

// ---------------------------------------------------------------------------------
// validation and exclusion keys
// ---------------------------------------------------------------------------------

static int check_desc(const mop_system_desc* d) {
    if (!d || d->Q < 1 || !d->mass || !d->charge || !d->type || !d->sigma || !d->epsilon)
        return MOP_EINVAL;
    if (d->ntypes < 1) return MOP_ETYPE;
    if (d->ntypes > MAXTYPES) return MOP_ETYPE;
    if (d->nbonds < 0 || (d->nbonds > 0 && (!d->bond_ij || !d->bond_r0 || !d->bond_k)))
        return MOP_EINVAL;
    if ((d->excl_mol == nullptr) != (d->excl_pos == nullptr)) return MOP_EINVAL;
    for (int a = 0; a < 3; ++a)
        if (!(d->box[a] > 0.0) || !std::isfinite(d->box[a])) return MOP_EINVAL;
    if (!(d->dt > 0.0) || !(d->nu > 0.0) || !(d->eps_r > 0.0) || !std::isfinite(d->eps_rf))
        return MOP_EINVAL;
    const double bmin = std::min(d->box[0], std::min(d->box[1], d->box[2]));
    if (!(d->r_cut > 0.0) || !(d->r_cut + SEARCH_MARGIN < 0.5 * bmin)) return MOP_ECUTOFF;
    for (int i = 0; i < d->Q; ++i) {
        if (!(d->mass[i] > 0.0) || !std::isfinite(d->charge[i])) return MOP_EINVAL;
        if (d->type[i] < 0 || d->type[i] >= d->ntypes) return MOP_ETYPE;
    }
    for (int t = 0; t < d->ntypes; ++t)
        if (!(d->sigma[t] >= 0.0) || !(d->epsilon[t] >= 0.0)) return MOP_EINVAL;
    for (int b = 0; b < d->nbonds; ++b) {
        const int i = d->bond_ij[2 * b], j = d->bond_ij[2 * b + 1];
        if (i < 0 || j < 0 || i >= d->Q || j >= d->Q || i == j) return MOP_EINVAL;
        if (!(d->bond_r0[b] > 0.0) || !(d->bond_k[b] >= 0.0)) return MOP_EINVAL;
    }
    if (d->excl_mol)
        for (int i = 0; i < d->Q; ++i)
            if (d->excl_mol[i] < 0 || d->excl_pos[i] < 0) return MOP_EINVAL;
    if (d->elec != MOP_ELEC_RF && d->elec != MOP_ELEC_PME) return MOP_EINVAL;
    if (d->elec == MOP_ELEC_PME) {
        const int p = d->pme_order ? d->pme_order : 4;
        if (p != 4 && p != 6 && p != 8) return MOP_EINVAL;
        // beta r_c <= 6 (the range of the pair kernels' erfc): rtol >= erfc(6) = 2.2e-17
        if (!(d->ewald_rtol == 0.0 || (d->ewald_rtol >= 1e-16 && d->ewald_rtol < 1.0)))
            return MOP_EINVAL;
        const int* g = d->pme_grid;
        const bool autog = g[0] == 0 && g[1] == 0 && g[2] == 0;
        if (!autog) {
            double n = 1.0;
            for (int a = 0; a < 3; ++a) {
                if (g[a] < p) return MOP_EINVAL;
                n *= g[a];
            }
            if (n > 134217728.0) return MOP_EINVAL;
        }
    }
    return MOP_OK;
}

// ---------------------------------------------------------------------------------
// particle-mesh Ewald constants
// ---------------------------------------------------------------------------------

// Cardinal B-spline M_n(x) by its recursion from M_2 (host, for the spline moduli).
static double bspline_host(int n, double x) {
    if (n == 2) return (x >= 0.0 && x <= 2.0) ? 1.0 - std::fabs(x - 1.0) : 0.0;
    return (x * bspline_host(n - 1, x) + (n - x) * bspline_host(n - 1, x - 1.0)) / (n - 1);
}

// |b(m)|^2 = 1 / |sum_{k=0}^{p-2} M_p(k+1) exp(2 pi i m k / K)|^2, m = 0..K-1.
static std::vector<double> bspline_moduli_host(int p, int K) {
    std::vector<double> out(K);
    for (int m = 0; m < K; ++m) {
        double re = 0.0, im = 0.0;
        for (int k = 0; k <= p - 2; ++k) {
            const double w = bspline_host(p, k + 1.0), a = 2.0 * PI * m * k / K;
            re += w * std::cos(a);
            im += w * std::sin(a);
        }
        out[m] = 1.0 / (re * re + im * im);
    }
    return out;
}

static int smooth_at_least(int n) {
    for (int k = std::max(n, 1);; ++k) {
        int m = k;
        for (int f : {2, 3, 5, 7})
            while (m % f == 0) m /= f;
        if (m == 1) return k;
    }
}

// beta with erfc(beta r_c) = rtol (bisection).
static double ewald_beta(double rc, double rtol) {
    double lo = 0.0, hi = 1.0;
    while (std::erfc(hi * rc) > rtol) hi *= 2.0;
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        (std::erfc(mid * rc) > rtol ? lo : hi) = mid;
    }
    return 0.5 * (lo + hi);
}

// Exclusion key per atom: the molecule's offset plus the position along its chain.
// Molecules get offsets in the order of their ids, each one its largest position + 3
// after the previous one, so |key_i - key_j| <= 2 only within a molecule and every key is
// below Q + 3 * (number of molecules) <= 4 Q.  Keys must stay below 2^27: the pair kernels
// keep key * 16 + LJ type in one 32-bit word.
// Without explicit molecules the bonds must form linear chains (degree <= 2, no cycles),
// which are walked from one end.
static int make_keys(const mop_system_desc* d, std::vector<int>& key) {
    const int Q = d->Q;
    std::vector<int> mol(Q), pos(Q);
    if (d->excl_mol) {
        for (int i = 0; i < Q; ++i) {
            mol[i] = d->excl_mol[i];
            pos[i] = d->excl_pos[i];
        }
    } else {
        std::vector<int> deg(Q, 0), nb0(Q, -1), nb1(Q, -1);
        for (int b = 0; b < d->nbonds; ++b) {
            const int i = d->bond_ij[2 * b], j = d->bond_ij[2 * b + 1];
            for (int k = 0; k < 2; ++k) {
                const int a = k ? j : i, o = k ? i : j;
                if (deg[a] >= 2) return MOP_ETOPOLOGY;
                if (deg[a] == 1 && nb0[a] == o) return MOP_ETOPOLOGY;  // duplicate bond
                (deg[a] == 0 ? nb0[a] : nb1[a]) = o;
                ++deg[a];
            }
        }
        std::vector<char> seen(Q, 0);
        int m = 0;
        for (int s = 0; s < Q; ++s) {
            if (seen[s] || deg[s] == 2) continue;  // start at chain ends and lone atoms
            int prev = -1, cur = s, p = 0;
            while (cur >= 0) {
                seen[cur] = 1;
                mol[cur] = m;
                pos[cur] = p++;
                const int nxt = nb0[cur] != prev ? nb0[cur] : nb1[cur];
                prev = cur;
                cur = (nxt >= 0 && !seen[nxt]) ? nxt : -1;
            }
            ++m;
        }
        for (int i = 0; i < Q; ++i)
            if (!seen[i]) return MOP_ETOPOLOGY;  // an atom on a ring
    }
    std::map<int, long long> off;  // molecule id -> largest position, then offset
    for (int i = 0; i < Q; ++i) {
        auto it = off.find(mol[i]);
        if (it == off.end()) off.emplace(mol[i], pos[i]);
        else it->second = std::max<long long>(it->second, pos[i]);
    }
    long long next = 0;
    for (auto& m : off) {
        const long long len = m.second + 1;
        m.second = next;
        next += len + 2;
    }
    if (next >= (1LL << 27)) return MOP_ETOPOLOGY;
    key.resize(Q);
    for (int i = 0; i < Q; ++i) key[i] = (int)(off[mol[i]] + pos[i]);
    return MOP_OK;
}

template <class T>
static int upload(mop_system sys, const T* h, size_t n, const T** out) {
    void* p = nullptr;
    const size_t bytes = std::max<size_t>(n, 1) * sizeof(T);
    if (hipMalloc(&p, bytes) != hipSuccess) return MOP_ENOMEM;
    sys->allocs.push_back(p);
    if (n && hipMemcpy(p, h, n * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) return MOP_EHIP;
    *out = static_cast<const T*>(p);
    return MOP_OK;
}

// ---------------------------------------------------------------------------------
// workspace layout
// ---------------------------------------------------------------------------------

// Offsets of one path's arrays starting at byte `base`; returns the end offset.
static size_t layout(SegDev& sg, int maxb, int maxN, size_t base) {
    const SysDev& s = sg.s;
    const size_t Q = s.Q, S = s.S, nc = s.ncol, nz = s.nzb, B = maxb;
    size_t o = align256(base);
    auto take = [&](size_t& off, size_t bytes) {
        off = o;
        o = align256(o + bytes);
    };
    take(sg.o_upos, B * S * 16);
    take(sg.o_umeta, B * S * 8);
    take(sg.o_orig, B * S * 4);
    take(sg.o_slotof, B * Q * 4);
    take(sg.o_atomu, B * Q * 16);
    take(sg.o_rank, B * Q * 4);
    take(sg.o_tmpo, B * S * 4);
    take(sg.o_bincnt, B * nc * nz * 4);
    take(sg.o_binoff, B * nc * (nz + 1) * 4);
    take(sg.o_colcnt, B * nc * 4);
    take(sg.o_colstart, B * (nc + 1) * 4);
    take(sg.o_vs, B * S * 16);
    take(sg.o_fs, B * S * 12);
    take(sg.o_f32, B * Q * 16);
    take(sg.o_f32m, B * Q * 16);
    take(sg.o_hv32, B * Q * 16);
    take(sg.o_epart, B * (size_t)s.cpb * 8);
    take(sg.o_d64, (size_t)std::max(maxN - 1, 1) * Q * 24);
    take(sg.o_rpart, (size_t)std::max(maxN, maxb) * sg.bpb * 16);
    take(sg.o_dmax, (size_t)std::max(maxN, 1) * 8);
    take(sg.o_eres, 4 * 8);
    sg.o_nl = sg.o_nlc = 0;
    if (s.lcap > 0) {
        take(sg.o_nl, B * s.cpb * (size_t)s.lcap * 4);
        take(sg.o_nlc, B * s.cpb * 4);
    }
    sg.o_ptc = sg.o_pts = sg.o_ptid = sg.o_ptrk = sg.o_ptb = sg.o_ptw = 0;
    sg.o_pgr = sg.o_pgc = sg.o_pphi = sg.o_pep = sg.o_pfw = sg.o_frec = sg.o_hrec = 0;
    if (s.elec == 1) {
        const size_t Kt = (size_t)s.Kg[0] * s.Kg[1] * s.Kg[2];
        const size_t Kc = (size_t)s.Kg[0] * s.Kg[1] * s.Kzh;
        take(sg.o_ptc, B * (size_t)s.ntile * 4);
        take(sg.o_pts, B * (size_t)(s.ntile + 1) * 4);
        take(sg.o_ptid, B * Q * 4);
        take(sg.o_ptrk, B * Q * 4);
        take(sg.o_ptb, B * Q * 16);
        take(sg.o_ptw, B * Q * 32);
        take(sg.o_pgr, B * Kt * 8);
        take(sg.o_pgc, B * Kc * 16);
        take(sg.o_pphi, B * Kt * 8);
        take(sg.o_pep, B * (size_t)s.nsb * 8);
        take(sg.o_frec, B * Q * 24);
        take(sg.o_hrec, B * Q * 24);
    }
    sg.maxb = maxb;
    sg.maxN = maxN;
    return o;
}

static SysDev plan_geometry(const mop_system_s* sys, const mop_plan_opts* opts) {
    SysDev s = sys->dev;
    const double cwt = (opts && opts->col_width > 0.0) ? opts->col_width : 0.4;
    const double zbt = (opts && opts->zbin > 0.0) ? opts->zbin : 0.1;
    const double* L = sys->box;
    s.ncx = std::max(1, (int)std::floor(L[0] / cwt));
    s.ncy = std::max(1, (int)std::floor(L[1] / cwt));
    s.nzb = std::max(1, (int)std::floor(L[2] / zbt));
    s.ncol = s.ncx * s.ncy;
    const double cwx = L[0] / s.ncx, cwy = L[1] / s.ncy;
    const double rcs = sys->rc + SEARCH_MARGIN;
    s.rx = (int)std::ceil(rcs / cwx);
    s.ry = (int)std::ceil(rcs / cwy);
    s.wx = 2 * s.rx + 1;
    s.wy = 2 * s.ry + 1;
    s.allx = s.wx >= s.ncx;
    s.ally = s.wy >= s.ncy;
    if (s.allx) s.wx = s.ncx;
    if (s.ally) s.wy = s.ncy;
    s.S = ((s.Q + 7 * s.ncol) + 7) & ~7;
    s.cpb = s.S / CLUSTER;
    for (int a = 0; a < 3; ++a) {
        s.L[a] = L[a];
        s.Lf[a] = (float)L[a];
        s.sc[a] = (float)(L[a] / 4294967296.0);
        s.ovr[a] = (uint32_t)std::min(std::ceil(OVERLAP_R / L[a] * 4294967296.0) + 1.0, 4294967295.0);
    }
    s.cw[0] = (float)cwx;
    s.cw[1] = (float)cwy;
    s.rcs = (float)rcs;
    s.rcs2 = (float)(rcs * rcs);
    // neighbour-list capacity in records (one per neighbouring cluster with an atom in
    // range): 1.5 x the expected number of 8-atom clusters whose box lies within the search
    // radius of a cluster's box (boxes cw x cw x the height 8 atoms fill at the mean
    // density: the volume swept by one box around the other, grown by the radius, times
    // the cluster density), rounded up to a multiple of 64.  A record keeps the cluster
    // index in 24 bits, so slot counts from 2^26 on take no lists.
    const int lc = opts ? opts->list_cap : 0;
    if (lc > 0) {
        s.lcap = lc;
    } else if (lc < 0) {
        s.lcap = 0;
    } else {
        const double rho = s.Q / (L[0] * L[1] * L[2]);
        const double c0 = std::min(L[2], CLUSTER / (rho * cwx * cwy));
        const double a = 2.0 * cwx, b = 2.0 * cwy, c = 2.0 * c0, r = rcs;
        const double pi = 3.14159265358979323846;
        const double vol = a * b * c + 2.0 * (a * b + b * c + c * a) * r +
                           pi * r * r * (a + b + c) + 4.0 / 3.0 * pi * r * r * r;
        const double est = std::min(1.5 * rho * vol / CLUSTER, (double)s.cpb);
        s.lcap = std::max(64, ((int)std::ceil(est) + 63) & ~63);
    }
    if (s.S >= (1 << 26)) s.lcap = 0;
    return s;
}

static void base_seg(SegDev& sg, const SysDev& s) {
    std::memset(&sg, 0, sizeof(sg));
    sg.s = s;
    sg.bpb = (s.Q + EWB - 1) / EWB;
}

// ---------------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------------

extern "C" {

const char* mop_strerror(int code) {
    switch (code) {
        case MOP_OK: return "ok";
        case MOP_EINVAL: return "invalid argument";
        case MOP_ECUTOFF: return "cutoff must be positive and below half the smallest box length";
        case MOP_ETYPE: return "atom type out of range or too many types (max 16)";
        case MOP_EHIP: return "HIP runtime error (no usable device?)";
        case MOP_ENOMEM: return "device allocation failed";
        case MOP_ETOPOLOGY: return "bonds do not form linear chains; give excl_mol/excl_pos";
        case MOP_ESIZE: return "more beads or paths than the plan or batch was created for";
        default: return "unknown error";
    }
}

int mop_system_check(const mop_system_desc* desc) {
    int rc = check_desc(desc);
    if (rc) return rc;
    std::vector<int> key;
    return make_keys(desc, key);
}

int mop_ctx_create(int device, void* hip_stream, mop_ctx* out) {
    if (!out) return MOP_EINVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return MOP_EHIP;
    if (hipSetDevice(device) != hipSuccess) return MOP_EHIP;
    mop_ctx c = new (std::nothrow) mop_ctx_s;
    if (!c) return MOP_ENOMEM;
    c->device = device;
    c->stream = static_cast<hipStream_t>(hip_stream);
    // this device's copy of the static scratch workspace of bead_forces_static: the
    // array's name is only a host-side stand-in, so its device address is looked up once
    // here, with the device current, and used wherever host code needs the array
    c->scratch = nullptr;
    void* sp = nullptr;
    if (hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch)) == hipSuccess) c->scratch = static_cast<char*>(sp);
    else (void)hipGetLastError();
    *out = c;
    return MOP_OK;
}

int mop_ctx_set_stream(mop_ctx ctx, void* hip_stream) {
    if (!ctx) return MOP_EINVAL;
    ctx->stream = static_cast<hipStream_t>(hip_stream);
    return MOP_OK;
}

void mop_ctx_destroy(mop_ctx ctx) { delete ctx; }

int mop_system_create(mop_ctx ctx, const mop_system_desc* d, mop_system* out) {
    if (!ctx || !out) return MOP_EINVAL;
    *out = nullptr;
    int err = check_desc(d);
    if (err) return err;
    std::vector<int> key;
    err = make_keys(d, key);
    if (err) return err;
    if (hipSetDevice(ctx->device) != hipSuccess) return MOP_EHIP;
    mop_system sys = new (std::nothrow) mop_system_s;
    if (!sys) return MOP_ENOMEM;
    sys->ctx = ctx;
    std::memset(&sys->dev, 0, sizeof(SysDev));
    const int Q = d->Q, nt = d->ntypes;
    for (int a = 0; a < 3; ++a) sys->box[a] = d->box[a];
    sys->rc = d->r_cut;
    SysDev& s = sys->dev;
    s.Q = Q;
    s.nt = nt;
    const double rc = d->r_cut;
    const double fq = F_ELEC / d->eps_r;
    const double krf = (d->eps_rf - d->eps_r) / ((2.0 * d->eps_rf + d->eps_r) * rc * rc * rc);
    const double crf = 1.0 / rc + krf * rc * rc;
    const double crf1 = 1.0 / (rc * rc) - 2.0 * krf * rc;
    s.rc2 = (float)(rc * rc);
    s.krf = (float)krf;
    s.krf2 = (float)(2.0 * krf);
    s.crf = (float)crf;
    s.crf1 = (float)crf1;
    s.e0rf = (float)(-rc * crf1);
    s.elec = d->elec;
    std::vector<double> phihat;
    std::vector<int> tile_lo, tile_of;
    if (d->elec == MOP_ELEC_PME) {
        // Ewald real space: psi = erfc(beta r)/r, shifted-force at r_c
        const double rtol = d->ewald_rtol > 0.0 ? d->ewald_rtol : 1e-5;
        const double beta = ewald_beta(rc, rtol);
        sys->beta = beta;
        const double c2b = 2.0 * beta / std::sqrt(PI);
        const double psic = std::erfc(beta * rc) / rc;
        const double dpsic = -std::erfc(beta * rc) / (rc * rc) - c2b * std::exp(-beta * beta * rc * rc) / rc;
        s.krf = s.krf2 = s.crf = 0.0f;
        s.crf1 = (float)(-dpsic);
        s.e0rf = (float)(-psic + rc * dpsic);
        s.ew_beta = (float)beta;
        s.ew_c2b = (float)c2b;
        s.ew_b2x2 = (float)(2.0 * beta * beta);
        // reciprocal part
        const int p = d->pme_order ? d->pme_order : 4;
        s.pme_p = p;
        const bool autog = d->pme_grid[0] == 0 && d->pme_grid[1] == 0 && d->pme_grid[2] == 0;
        for (int a = 0; a < 3; ++a)
            s.Kg[a] = autog ? std::max(smooth_at_least((int)std::ceil(d->box[a] / PME_SPACING)), 2 * p)
                            : d->pme_grid[a];
        s.Kzh = s.Kg[2] / 2 + 1;
        const size_t Kc = (size_t)s.Kg[0] * s.Kg[1] * s.Kzh;
        s.nsb = (int)((Kc + PME_BLOCK - 1) / PME_BLOCK);
        double klmax = 0.0;
        for (int a = 0; a < 3; ++a) {
            s.kl[a] = s.Kg[a] / d->box[a];
            klmax = std::max(klmax, s.kl[a]);
        }
        double sabs = 0.0, sq = 0.0, sq2 = 0.0;
        for (int i = 0; i < Q; ++i) {
            sabs += std::fabs(d->charge[i]);
            sq += d->charge[i];
            sq2 += d->charge[i] * d->charge[i];
        }
        s.qscale = sabs > 0.0 ? std::ldexp(1.0, 61 - (std::ilogb(sabs) + 1)) : 1.0;
        s.vbound = sabs * 3.0 * klmax;
        const double V = d->box[0] * d->box[1] * d->box[2];
        s.e_const = -fq * beta / std::sqrt(PI) * sq2 - fq * PI * sq * sq / (2.0 * V * beta * beta);
        // f B(m) C(m) on the half spectrum (z frequencies 0 .. Kz/2)
        std::vector<double> bm[3];
        for (int a = 0; a < 3; ++a) bm[a] = bspline_moduli_host(p, s.Kg[a]);
        phihat.resize(Kc);
        for (int mx = 0; mx < s.Kg[0]; ++mx)
            for (int my = 0; my < s.Kg[1]; ++my)
                for (int mz = 0; mz < s.Kzh; ++mz) {
                    const int fx = 2 * mx < s.Kg[0] ? mx : mx - s.Kg[0];
                    const int fy = 2 * my < s.Kg[1] ? my : my - s.Kg[1];
                    const double ax = fx / d->box[0], ay = fy / d->box[1], az = mz / d->box[2];
                    const double m2 = ax * ax + ay * ay + az * az;
                    double v = 0.0;
                    if (m2 > 0.0)
                        v = fq * bm[0][mx] * bm[1][my] * bm[2][mz] *
                            std::exp(-PI * PI * m2 / (beta * beta)) / (PI * V * m2);
                    phihat[((size_t)mx * s.Kg[1] + my) * s.Kzh + mz] = v;
                }
        // spreading tiles: about PME_TILE points per edge, balanced
        int maxe[3];
        for (int a = 0; a < 3; ++a) {
            const int K = s.Kg[a];
            const int nt = std::max(1, K / PME_TILE);
            s.ntl[a] = nt;
            s.tlo_off[a] = (int)tile_lo.size();
            s.tof_off[a] = (int)tile_of.size();
            maxe[a] = 0;
            for (int t = 0; t <= nt; ++t) tile_lo.push_back((int)((long long)t * K / nt));
            for (int t = 0; t < nt; ++t) {
                const int a0 = tile_lo[s.tlo_off[a] + t], a1 = tile_lo[s.tlo_off[a] + t + 1];
                maxe[a] = std::max(maxe[a], a1 - a0);
                for (int k = a0; k < a1; ++k) tile_of.push_back(t);
            }
        }
        s.ntile = s.ntl[0] * s.ntl[1] * s.ntl[2];
        s.tile_pts = maxe[0] * maxe[1] * maxe[2];
    }
    // per atom
    std::vector<float> qs(Q);
    std::vector<int> typ(Q);
    std::vector<double> c(Q), K(Q), minv(Q);
    const double sq = std::sqrt(fq);
    for (int i = 0; i < Q; ++i) {
        qs[i] = (float)(d->charge[i] * sq);
        typ[i] = d->type[i];
        c[i] = d->dt / (d->mass[i] * d->nu);
        K[i] = d->mass[i] * d->nu / (2.0 * d->dt);
        minv[i] = 1.0 / d->mass[i];
    }
    // type-pair tables (Lorentz-Berthelot), shifted-force constants at r_cut
    std::vector<float4> tab(nt * nt), tab2(nt * nt), tabh(nt * nt);
    for (int a = 0; a < nt; ++a)
        for (int b = 0; b < nt; ++b) {
            const double sg = 0.5 * (d->sigma[a] + d->sigma[b]);
            const double ep = std::sqrt(d->epsilon[a] * d->epsilon[b]);
            const double s6 = std::pow(sg, 6.0);
            const double c6 = 4.0 * ep * s6, c12 = 4.0 * ep * s6 * s6;
            const double ir = 1.0 / rc, ir6 = std::pow(ir, 6.0);
            const double phic = c12 * ir6 * ir6 - c6 * ir6;
            const double dphic = (-12.0 * c12 * ir6 * ir6 + 6.0 * c6 * ir6) * ir;
            const double csf = -dphic;
            const double e0 = -phic - rc * csf;
            tab[a * nt + b] = make_float4((float)(-12.0 * c12), (float)(6.0 * c6), (float)csf, (float)e0);
            tab2[a * nt + b] = make_float4((float)(168.0 * c12), (float)(-48.0 * c6), (float)c12, (float)c6);
            tabh[a * nt + b] = make_float4((float)(-12.0 * c12), (float)(6.0 * c6), (float)csf,
                                           (float)(-9.0 * c12));
        }
    // bond CSR (each bond listed for both atoms)
    std::vector<int> bstart(Q + 1, 0), bpart(2 * (size_t)d->nbonds);
    std::vector<double> br0(2 * (size_t)d->nbonds), bk(2 * (size_t)d->nbonds);
    for (int b = 0; b < d->nbonds; ++b) {
        ++bstart[d->bond_ij[2 * b] + 1];
        ++bstart[d->bond_ij[2 * b + 1] + 1];
    }
    for (int i = 0; i < Q; ++i) bstart[i + 1] += bstart[i];
    {
        std::vector<int> fill(bstart.begin(), bstart.end() - 1);
        for (int b = 0; b < d->nbonds; ++b) {
            const int i = d->bond_ij[2 * b], j = d->bond_ij[2 * b + 1];
            int k = fill[i]++;
            bpart[k] = j;
            br0[k] = d->bond_r0[b];
            bk[k] = d->bond_k[b];
            k = fill[j]++;
            bpart[k] = i;
            br0[k] = d->bond_r0[b];
            bk[k] = d->bond_k[b];
        }
    }
    s.nbond_entries = 2 * d->nbonds;
    int e = 0;
    if (!e) e = upload(sys, qs.data(), Q, &s.qs);
    for (int i = 0; i < Q; ++i) key[i] = key[i] * 16 + typ[i];  // type < MAXTYPES = 16
    if (!e) e = upload(sys, key.data(), Q, &s.key);
    if (!e) e = upload(sys, typ.data(), Q, &s.type);
    if (!e) e = upload(sys, c.data(), Q, &s.c);
    if (!e) e = upload(sys, K.data(), Q, &s.K);
    if (!e) e = upload(sys, minv.data(), Q, &s.minv);
    if (!e) e = upload(sys, bstart.data(), Q + 1, &s.bstart);
    if (!e) e = upload(sys, bpart.data(), bpart.size(), &s.bpart);
    if (!e) e = upload(sys, br0.data(), br0.size(), &s.br0);
    if (!e) e = upload(sys, bk.data(), bk.size(), &s.bk);
    if (!e) e = upload(sys, tab.data(), tab.size(), &s.tab);
    if (!e) e = upload(sys, tab2.data(), tab2.size(), &s.tab2);
    if (!e) e = upload(sys, tabh.data(), tabh.size(), &s.tabh);
    if (!e && s.elec == 1) e = upload(sys, d->charge, Q, &s.qd);
    if (!e && s.elec == 1) e = upload(sys, phihat.data(), phihat.size(), &s.phihat);
    if (!e && s.elec == 1) e = upload(sys, tile_lo.data(), tile_lo.size(), &s.tile_lo);
    if (!e && s.elec == 1) e = upload(sys, tile_of.data(), tile_of.size(), &s.tile_of);
    if (e) {
        mop_system_destroy(sys);
        return e;
    }
    *out = sys;
    return MOP_OK;
}

void mop_system_destroy(mop_system sys) {
    if (!sys) return;
    for (void* p : sys->allocs) (void)hipFree(p);
    delete sys;
}

static void destroy_fft(PmeFft& f) {
    if (f.fwd) (void)rocfft_plan_destroy(f.fwd);
    if (f.bwd) (void)rocfft_plan_destroy(f.bwd);
    if (f.fwd32) (void)rocfft_plan_destroy(f.fwd32);
    if (f.bwd32) (void)rocfft_plan_destroy(f.bwd32);
    if (f.info) (void)rocfft_execution_info_destroy(f.info);
    f = PmeFft();
}

// Out-of-place real <-> half-complex 3-D transforms of `batch` grids K0 x K1 x K2 (K2
// fastest), real grids packed K apart, spectra Kc apart: in double precision for the
// charge grids, in single precision for the dipole grids of the Hessian pass.
static int make_fft(PmeFft& f, const int K[3], int batch) {
    static bool ready = false;
    if (!ready) {
        if (rocfft_setup() != rocfft_status_success) return MOP_EHIP;
        ready = true;
    }
    const size_t Kzh = K[2] / 2 + 1;
    size_t len[3] = {(size_t)K[2], (size_t)K[1], (size_t)K[0]};
    size_t rs[3] = {1, (size_t)K[2], (size_t)K[2] * K[1]};
    size_t cs[3] = {1, Kzh, Kzh * K[1]};
    const size_t rdist = (size_t)K[0] * K[1] * K[2], cdist = (size_t)K[0] * K[1] * Kzh;
    rocfft_plan_description df = nullptr, db = nullptr;
    bool ok = rocfft_plan_description_create(&df) == rocfft_status_success &&
              rocfft_plan_description_create(&db) == rocfft_status_success;
    ok = ok && rocfft_plan_description_set_data_layout(
                   df, rocfft_array_type_real, rocfft_array_type_hermitian_interleaved, nullptr,
                   nullptr, 3, rs, rdist, 3, cs, cdist) == rocfft_status_success;
    ok = ok && rocfft_plan_description_set_data_layout(
                   db, rocfft_array_type_hermitian_interleaved, rocfft_array_type_real, nullptr,
                   nullptr, 3, cs, cdist, 3, rs, rdist) == rocfft_status_success;
    ok = ok && rocfft_plan_create(&f.fwd, rocfft_placement_notinplace,
                                  rocfft_transform_type_real_forward, rocfft_precision_double, 3,
                                  len, batch, df) == rocfft_status_success;
    ok = ok && rocfft_plan_create(&f.bwd, rocfft_placement_notinplace,
                                  rocfft_transform_type_real_inverse, rocfft_precision_double, 3,
                                  len, batch, db) == rocfft_status_success;
    ok = ok && rocfft_plan_create(&f.fwd32, rocfft_placement_notinplace,
                                  rocfft_transform_type_real_forward, rocfft_precision_single, 3,
                                  len, batch, df) == rocfft_status_success;
    ok = ok && rocfft_plan_create(&f.bwd32, rocfft_placement_notinplace,
                                  rocfft_transform_type_real_inverse, rocfft_precision_single, 3,
                                  len, batch, db) == rocfft_status_success;
    size_t w1 = 0, w2 = 0, w3 = 0, w4 = 0;
    ok = ok && rocfft_plan_get_work_buffer_size(f.fwd, &w1) == rocfft_status_success &&
         rocfft_plan_get_work_buffer_size(f.bwd, &w2) == rocfft_status_success &&
         rocfft_plan_get_work_buffer_size(f.fwd32, &w3) == rocfft_status_success &&
         rocfft_plan_get_work_buffer_size(f.bwd32, &w4) == rocfft_status_success;
    ok = ok && rocfft_execution_info_create(&f.info) == rocfft_status_success;
    if (df) (void)rocfft_plan_description_destroy(df);
    if (db) (void)rocfft_plan_description_destroy(db);
    if (!ok) {
        destroy_fft(f);
        return MOP_EHIP;
    }
    f.work = std::max(std::max(w1, w2), std::max(w3, w4));
    return MOP_OK;
}

// One batched transform on `st` (the work buffer lives in the caller's workspace).
static void run_fft(const mop_plan_s* pl, bool forward, void* in, void* out, void* work,
                    hipStream_t st, bool single = false) {
    const PmeFft& f = pl->fft;
    bool ok = rocfft_execution_info_set_stream(f.info, st) == rocfft_status_success;
    if (f.work)
        ok = ok && rocfft_execution_info_set_work_buffer(f.info, work, f.work) == rocfft_status_success;
    void* ib[1] = {in};
    void* ob[1] = {out};
    const rocfft_plan plan = single ? (forward ? f.fwd32 : f.bwd32) : (forward ? f.fwd : f.bwd);
    ok = ok && rocfft_execute(plan, ib, ob, f.info) == rocfft_status_success;
    if (!ok) pl->fft_failed = true;
}

int mop_plan_create(mop_system sys, int32_t max_beads, const mop_plan_opts* opts, mop_plan* out) {
    if (!sys || !out || max_beads < 1) return MOP_EINVAL;
    *out = nullptr;
    if (opts && (opts->flags & ~(MOP_PLAN_NEWTON3 | MOP_PLAN_ONE_STREAM | MOP_PLAN_PERSISTENT)))
        return MOP_EINVAL;
    if (sys->dev.elec == 1 && opts && (opts->flags & MOP_PLAN_NEWTON3)) return MOP_EINVAL;
    int waves = opts && opts->waves ? opts->waves : 4;
    if (waves != 1 && waves != 2 && waves != 4 && waves != 8) return MOP_EINVAL;
    if (opts && (opts->col_width < 0.0 || opts->zbin < 0.0)) return MOP_EINVAL;
    if (hipSetDevice(sys->ctx->device) != hipSuccess) return MOP_EHIP;
    mop_plan pl = new (std::nothrow) mop_plan_s;
    if (!pl) return MOP_ENOMEM;
    pl->sys = sys;
    pl->max_beads = max_beads;
    pl->waves = waves | ((opts && (opts->flags & MOP_PLAN_PERSISTENT)) ? WAVES_PERSISTENT : 0);
    pl->newton3 = (opts && (opts->flags & MOP_PLAN_NEWTON3)) ? 1 : 0;
    pl->one_stream = (opts && (opts->flags & MOP_PLAN_ONE_STREAM)) ? 1 : 0;
    base_seg(pl->hseg, plan_geometry(sys, opts));
    pl->hseg.roff = 0;
    pl->hseg.vidx = 0;
    pl->ws_bytes = layout(pl->hseg, max_beads, max_beads, 256);
    pl->dseg = nullptr;
    if (pl->hseg.s.elec == 1) {
        int e = make_fft(pl->fft, pl->hseg.s.Kg, pl->hseg.maxb);
        if (!e && !pl->one_stream &&
            (hipStreamCreateWithFlags(&pl->side, hipStreamNonBlocking) != hipSuccess ||
             hipEventCreateWithFlags(&pl->fork, hipEventDisableTiming) != hipSuccess ||
             hipEventCreateWithFlags(&pl->join, hipEventDisableTiming) != hipSuccess))
            e = MOP_EHIP;
        if (e) {
            destroy_fft(pl->fft);
            if (pl->side) (void)hipStreamDestroy(pl->side);
            if (pl->fork) (void)hipEventDestroy(pl->fork);
            if (pl->join) (void)hipEventDestroy(pl->join);
            delete pl;
            return e;
        }
        pl->hseg.o_pfw = align256(pl->ws_bytes);
        pl->ws_bytes = pl->hseg.o_pfw + std::max<size_t>(pl->fft.work, 256);
    }
    if (hipMalloc(&pl->dseg, sizeof(SegDev)) != hipSuccess) {
        pl->dseg = nullptr;
        mop_plan_destroy(pl);
        return MOP_ENOMEM;
    }
    if (hipMemcpy(pl->dseg, &pl->hseg, sizeof(SegDev), hipMemcpyHostToDevice) != hipSuccess) {
        mop_plan_destroy(pl);
        return MOP_EHIP;
    }
    *out = pl;
    return MOP_OK;
}

void mop_plan_destroy(mop_plan plan) {
    if (!plan) return;
    if (plan->dseg) (void)hipFree(plan->dseg);
    destroy_fft(plan->fft);
    if (plan->side) (void)hipStreamDestroy(plan->side);
    if (plan->fork) (void)hipEventDestroy(plan->fork);
    if (plan->join) (void)hipEventDestroy(plan->join);
    delete plan;
}

int mop_system_pme_info(mop_system sys, int32_t grid[3], double* beta) {
    if (!sys || sys->dev.elec != 1) return MOP_EINVAL;
    if (grid)
        for (int a = 0; a < 3; ++a) grid[a] = sys->dev.Kg[a];
    if (beta) *beta = sys->beta;
    return MOP_OK;
}

int mop_workspace_size(mop_plan plan, size_t* bytes) {
    if (!plan || !bytes) return MOP_EINVAL;
    *bytes = plan->ws_bytes;
    return MOP_OK;
}

int mop_plan_info(mop_plan plan, int32_t* ncx, int32_t* ncy, int32_t* nzb, int32_t* slots) {
    if (!plan) return MOP_EINVAL;
    if (ncx) *ncx = plan->hseg.s.ncx;
    if (ncy) *ncy = plan->hseg.s.ncy;
    if (nzb) *nzb = plan->hseg.s.nzb;
    if (slots) *slots = plan->hseg.s.S;
    return MOP_OK;
}

static Launch one_path(int N, int nb) {
    Launch L;
    std::memset(&L, 0, sizeof(L));
    L.nseg = 1;
    L.N[0] = N;
    L.nb[0] = nb;
    return L;
}

static CallPtrs call_ptrs(void* ws) {
    CallPtrs cp;
    std::memset(&cp, 0, sizeof(cp));
    cp.ws = static_cast<char*>(ws);
    cp.status = static_cast<int*>(ws);
    return cp;
}

static int finish(mop_ctx ctx) {
    (void)ctx;
    return hipGetLastError() == hipSuccess ? MOP_OK : MOP_EHIP;
}

// finish() plus the plan's transform errors (PME), which are cleared once reported.
static int finish_plan(mop_plan plan) {
    int rc = finish(plan->sys->ctx);
    if (plan->fft_failed) {
        plan->fft_failed = false;
        rc = MOP_EHIP;
    }
    return rc;
}

// PME reciprocal forces of nb pair beads at R (displaced by fdsign eps d) into output
// outsel of the gather (when gather): 3 = the FP64 buffer frec, 1 / 2 = added to the
// float4 buffers of the displaced force passes.  The potential goes to pphi for the
// undisplaced configuration (kept for the Hessian pass), else to pgr.  Energy partials
// are formed for the undisplaced configuration.
static void pme_forces(const mop_plan_s* pl, int nb, const CallPtrs& cp, int fdsign, int outsel,
                       bool gather, hipStream_t st) {
    const SegDev& h = pl->hseg;
    char* ws = cp.ws;
    run_pme_sort(pl->dseg, h, nb, ws, cp.R, fdsign, cp.fd_h, st);
    run_pme_spread(pl->dseg, h, nb, h.maxb, ws, cp.R, nullptr, 0, fdsign, cp.fd_h, st);
    run_fft(pl, true, ws + h.o_pgr, ws + h.o_pgc, ws + h.o_pfw, st);
    run_pme_solve(pl->dseg, h, nb, ws, fdsign == 0 ? 1 : 0, st);
    run_fft(pl, false, ws + h.o_pgc, ws + (fdsign == 0 ? h.o_pphi : h.o_pgr), ws + h.o_pfw, st);
    if (gather)
        run_pme_gather(pl->dseg, h, nb, ws, cp.R, nullptr, 0, fdsign, cp.fd_h, outsel,
                       fdsign != 0 ? 1 : 0, st);
}

// PME reciprocal H v of nb pair beads (V: [nb][Q][3]; needs pphi and the tile order of
// the same beads from pme_forces, and the per-bead max |v|^2), written to hrec.
static void pme_hvp(const mop_plan_s* pl, int nb, const CallPtrs& cp, const double* V,
                    hipStream_t st) {
    const SegDev& h = pl->hseg;
    char* ws = cp.ws;
    run_pme_spread(pl->dseg, h, nb, h.maxb, ws, cp.R, V, 1, 0, 0.0, st);
    run_fft(pl, true, ws + h.o_pgr, ws + h.o_pgc, ws + h.o_pfw, st, true);
    run_pme_solve32(pl->dseg, h, nb, ws, st);
    run_fft(pl, false, ws + h.o_pgc, ws + h.o_pgr, ws + h.o_pfw, st, true);
    run_pme_gather(pl->dseg, h, nb, ws, cp.R, V, 1, 0, 0.0, 4, 0, st);
}

// Fork: work enqueued on the plan's side stream after this waits for everything enqueued
// on st so far.  Join: work enqueued on st after this waits for the side stream.  With
// MOP_PLAN_ONE_STREAM the mesh work goes to st itself and both are no-ops.
static hipStream_t mesh_stream(const mop_plan_s* pl, hipStream_t st) {
    return pl->one_stream ? st : pl->side;
}

static void fork_side(const mop_plan_s* pl, hipStream_t st) {
    if (pl->one_stream) return;
    (void)hipEventRecord(pl->fork, st);
    (void)hipStreamWaitEvent(pl->side, pl->fork, 0);
}

static void join_side(const mop_plan_s* pl, hipStream_t st) {
    if (pl->one_stream) return;
    (void)hipEventRecord(pl->join, pl->side);
    (void)hipStreamWaitEvent(st, pl->join, 0);
}

int bead_forces(mop_plan plan, const double* R, int32_t B, float* F, double* U, void* ws) {
    if (!plan || !R || !F || !ws) return MOP_EINVAL;
    if (B < 1) return MOP_EINVAL;
    if (B > plan->max_beads) return MOP_ESIZE;
    hipStream_t st = plan->sys->ctx->stream;
    CallPtrs cp = call_ptrs(ws);
    cp.R = R;
    cp.Fout = F;
    cp.Uout = U;
    const Launch L = one_path(B, B);
    const bool pme = plan->hseg.s.elec == 1;
    if (pme) {
        fork_side(plan, st);
        pme_forces(plan, B, cp, 0, 3, true, mesh_stream(plan, st));
    }
    run_binning(plan->dseg, &plan->hseg, L, cp.ws, R, 0, 0.0, st);
    run_pair(plan->dseg, &plan->hseg, L, cp.ws, 0, 0, U ? -2 : -1, plan->waves, plan->newton3, st);
    if (pme) join_side(plan, st);
    run_finalize_forces(plan->dseg, &plan->hseg, L, cp, st);
    return finish_plan(plan);
}

int bead_forces_static(mop_plan plan, const double* R, int32_t B, float* F, double* U,
                       int32_t* status) {
    if (!plan || !R || !F) return MOP_EINVAL;
    if (B < 1) return MOP_EINVAL;
    if (B > plan->max_beads) return MOP_ESIZE;
    // reaction-field full-shell plans only: Newton-3 kernels need a zeroed slot-order
    // buffer, PME plans hand part of the workspace to rocFFT
    if (plan->hseg.s.elec == 1 || plan->newton3) return MOP_EINVAL;
    if (plan->ws_bytes > SCRATCH_BYTES) return MOP_ESIZE;
    mop_ctx ctx = plan->sys->ctx;
    if (!ctx->scratch) return MOP_EHIP;
    hipStream_t st = ctx->stream;
    CallPtrs cp = call_ptrs(ctx->scratch);
    cp.R = R;
    cp.Fout = F;
    cp.Uout = U;
    const Launch L = one_path(B, B);
    // the array keeps the previous call's contents: start from a clear status word (a
    // kernel, not a memset, so that the call can be captured in a graph)
    run_status_clear(cp.status, st);
    run_binning(plan->dseg, &plan->hseg, L, cp.ws, R, 0, 0.0, st);
    run_pair(plan->dseg, &plan->hseg, L, cp.ws, 0, 0, U ? -2 : -1, plan->waves, 0, st);
    run_finalize_forces(plan->dseg, &plan->hseg, L, cp, st);
    if (status) run_status_copy(cp.status, status, st);
    return finish(ctx);
}

int bead_hvp(mop_plan plan, const double* R, const double* V, int32_t B, float* HV, void* ws) {
    if (!plan || !R || !V || !HV || !ws) return MOP_EINVAL;
    if (B < 1) return MOP_EINVAL;
    if (B > plan->max_beads) return MOP_ESIZE;
    hipStream_t st = plan->sys->ctx->stream;
    CallPtrs cp = call_ptrs(ws);
    cp.R = R;
    cp.V = V;
    cp.Fout = HV;
    const Launch L = one_path(B, B);
    const bool pme = plan->hseg.s.elec == 1;
    run_binning(plan->dseg, &plan->hseg, L, cp.ws, R, 0, 0.0, st);
    if (pme) {
        // after the binning, which clears the per-bead max |v|^2
        fork_side(plan, st);
        pme_forces(plan, B, cp, 0, 3, false, mesh_stream(plan, st));
        run_pme_vmax(plan->dseg, plan->hseg, B, cp.ws, V, mesh_stream(plan, st));
        pme_hvp(plan, B, cp, V, mesh_stream(plan, st));
    }
    run_prep_v(plan->dseg, &plan->hseg, L, cp, st);
    run_pair(plan->dseg, &plan->hseg, L, cp.ws, 1, 0, -1, plan->waves, plan->newton3, st);
    if (pme) join_side(plan, st);
    run_finalize_hvp(plan->dseg, &plan->hseg, L, cp, st);
    return finish_plan(plan);
}

// The phases of V_eff and its gradient over every path of `base`.  ev, when given,
// receives an event after each phase (MOP_NPHASES + 1 events, ev[0] at the start).
// pl: the plan of a single-path call (PME steps run for PME systems), null for batches.
static void path_sequence(const SegDev* dsegs, const SegDev* hsegs, const Launch& base,
                          const CallPtrs& cp, bool grad, int mode, int waves, int n3,
                          hipStream_t st, hipEvent_t* ev = nullptr, const mop_plan_s* pl = nullptr) {
    const bool pme = pl && pl->hseg.s.elec == 1;
    const bool side = pme && !pl->one_stream;
    auto mark = [&](int k) {
        if (ev) (void)hipEventRecord(ev[k], st);
    };
    mark(0);
    // PME: the mesh forces run beside the binning and the pair forces (on one stream:
    // after them, as a phase of their own)
    if (side) {
        fork_side(pl, st);
        pme_forces(pl, base.nb[0], cp, 0, 3, true, pl->side);
    }
    // forces of beads 1..N-1 (bead 1 alone for N = 1), energy of bead 1
    run_binning(dsegs, hsegs, base, cp.ws, cp.R, 0, 0.0, st);
    mark(1);
    // exact gradients: the force pass records neighbour lists for the Hessian pass; with
    // shared-bin finite differences, for the two displaced force passes
    const int lists = (grad && (mode == 0 || mode == 2)) ? 1 : 0;
    run_pair(dsegs, hsegs, base, cp.ws, 0, 0, 0, waves, n3, st, lists);
    mark(2);
    if (side) join_side(pl, st);
    else if (pme) pme_forces(pl, base.nb[0], cp, 0, 3, true, st);
    mark(3);
    // max |d|^2 per bead: the finite-difference steps and the PME dipole-grid scale
    run_resid(dsegs, hsegs, base, cp, grad && (mode != 0 || pme), st);
    mark(4);
    if (grad) {
        Launch Lh = base;
        bool any = false;
        for (int p = 0; p < base.nseg; ++p) {
            Lh.nb[p] = base.N[p] - 1;
            any = any || Lh.nb[p] > 0;
        }
        // PME: the mesh Hessian-vector products run beside the pair Hessian kernel
        const bool mesh = any && mode == 0 && pme;
        const double* d64 = mesh ? wsp_host<double>(cp.ws, hsegs[0].o_d64) : nullptr;
        if (mesh && side) {
            fork_side(pl, st);
            pme_hvp(pl, Lh.nb[0], cp, d64, pl->side);
        }
        if (any && mode == 0) run_pair(dsegs, hsegs, Lh, cp.ws, 1, 0, -1, waves, n3, st, 2 * lists);
        mark(5);
        if (mesh && side) join_side(pl, st);
        else if (mesh) pme_hvp(pl, Lh.nb[0], cp, d64, st);
        mark(6);
        if (any && mode != 0) {
            // mode 1 re-bins each displaced configuration; mode 2 keeps R's binning
            for (int sgn : {+1, -1}) {
                if (mode == 1) run_binning(dsegs, hsegs, Lh, cp.ws, cp.R, sgn, cp.fd_h, st);
                else run_displace(dsegs, hsegs, Lh, cp.ws, cp.R, sgn, cp.fd_h, st);
                run_pair(dsegs, hsegs, Lh, cp.ws, 0, sgn > 0 ? 1 : 2, -1, waves, n3, st,
                         mode == 2 ? 2 * lists : 0);
                if (pme) pme_forces(pl, Lh.nb[0], cp, sgn, sgn > 0 ? 1 : 2, true, st);
            }
        }
        mark(7);
        run_assemble(dsegs, hsegs, base, cp, mode != 0 ? 1 : 0, st);
    } else {
        mark(5);
        mark(6);
        mark(7);
    }
    run_reduce_veff(dsegs, hsegs, base, cp, st);
    mark(8);
}

int veff_energy(mop_plan plan, const double* R, int32_t N, double* veff, double* u1,
                double* espring, void* ws) {
    if (!plan || !R || !ws) return MOP_EINVAL;
    if (N < 1) return MOP_EINVAL;
    if (N > plan->max_beads) return MOP_ESIZE;
    CallPtrs cp = call_ptrs(ws);
    cp.R = R;
    cp.veff = veff;
    cp.u1 = u1;
    cp.espring = espring;
    const Launch L = one_path(N, N > 1 ? N - 1 : 1);
    path_sequence(plan->dseg, &plan->hseg, L, cp, false, 0, plan->waves, plan->newton3,
                  plan->sys->ctx->stream, nullptr, plan);
    return finish_plan(plan);
}

int veff_grad(mop_plan plan, const double* R, int32_t N, double* G, double* veff, int32_t mode,
              double fd_h, void* ws) {
    if (!plan || !R || !G || !ws) return MOP_EINVAL;
    if (N < 1 || mode < 0 || mode > 2) return MOP_EINVAL;
    if (mode != 0 && !(fd_h > 0.0)) return MOP_EINVAL;
    if (N > plan->max_beads) return MOP_ESIZE;
    CallPtrs cp = call_ptrs(ws);
    cp.R = R;
    cp.G = G;
    cp.veff = veff;
    cp.fd_h = fd_h;
    const Launch L = one_path(N, N > 1 ? N - 1 : 1);
    path_sequence(plan->dseg, &plan->hseg, L, cp, true, mode, plan->waves, plan->newton3,
                  plan->sys->ctx->stream, nullptr, plan);
    return finish_plan(plan);
}

int veff_grad_timed(mop_plan plan, const double* R, int32_t N, double* G, double* veff,
                    int32_t mode, double fd_h, void* ws, float* phase_ms) {
    if (!plan || !R || !G || !ws || !phase_ms) return MOP_EINVAL;
    if (N < 1 || mode < 0 || mode > 2) return MOP_EINVAL;
    if (mode != 0 && !(fd_h > 0.0)) return MOP_EINVAL;
    if (N > plan->max_beads) return MOP_ESIZE;
    hipStream_t st = plan->sys->ctx->stream;
    hipEvent_t ev[MOP_NPHASES + 1];
    for (int k = 0; k <= MOP_NPHASES; ++k)
        if (hipEventCreate(&ev[k]) != hipSuccess) return MOP_EHIP;
    CallPtrs cp = call_ptrs(ws);
    cp.R = R;
    cp.G = G;
    cp.veff = veff;
    cp.fd_h = fd_h;
    const Launch L = one_path(N, N > 1 ? N - 1 : 1);
    path_sequence(plan->dseg, &plan->hseg, L, cp, true, mode, plan->waves, plan->newton3, st, ev,
                  plan);
    int rc = finish_plan(plan);
    if (hipEventSynchronize(ev[MOP_NPHASES]) != hipSuccess) rc = MOP_EHIP;
    for (int k = 0; k < MOP_NPHASES; ++k) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, ev[k], ev[k + 1]) != hipSuccess) rc = MOP_EHIP;
        phase_ms[k] = ms;
    }
    for (int k = 0; k <= MOP_NPHASES; ++k) (void)hipEventDestroy(ev[k]);
    return rc;
}

int mop_bias_create(mop_plan plan, const mop_bias_desc* d, mop_bias* out) {
    if (!plan || !d || !out) return MOP_EINVAL;
    *out = nullptr;
    const int Q = plan->hseg.s.Q;
    if (d->nA < 1 || d->nB < 1 || !d->groupA || !d->groupB) return MOP_EINVAL;
    if (!(d->sigma > 0.0) || !(d->height >= 0.0) || d->stride < 1 || d->max_gaussians < 1)
        return MOP_EINVAL;
    if (!(d->bias_factor == 0.0 || d->bias_factor > 1.0)) return MOP_EINVAL;
    if (d->bias_factor > 1.0 && !(d->kT > 0.0)) return MOP_EINVAL;
    std::vector<char> seen(Q, 0);
    for (int k = 0; k < d->nA + d->nB; ++k) {
        const int i = k < d->nA ? d->groupA[k] : d->groupB[k - d->nA];
        if (i < 0 || i >= Q || seen[i]) return MOP_EINVAL;  // in range, groups disjoint
        seen[i] = 1;
    }
    if (hipSetDevice(plan->sys->ctx->device) != hipSuccess) return MOP_EHIP;
    mop_bias b = new (std::nothrow) mop_bias_s;
    if (!b) return MOP_ENOMEM;
    b->plan = plan;
    b->stride = d->stride;
    BiasDev& bd = b->dev;
    std::memset(&bd, 0, sizeof(bd));
    bd.nA = d->nA;
    bd.nB = d->nB;
    bd.minv = plan->sys->dev.minv;
    for (int a = 0; a < 3; ++a) bd.L[a] = plan->sys->box[a];
    bd.sigma = d->sigma;
    bd.height = d->height;
    bd.bias_factor = d->bias_factor;
    bd.kT = d->kT;
    bd.capacity = d->max_gaussians;
    auto dalloc = [&](void** p, size_t bytes) {
        if (hipMalloc(p, bytes) != hipSuccess) return MOP_ENOMEM;
        b->allocs.push_back(*p);
        return MOP_OK;
    };
    int e = 0;
    void *pa = nullptr, *pb = nullptr, *pc = nullptr, *ph = nullptr, *pn = nullptr;
    if (!e) e = dalloc(&pa, sizeof(int) * d->nA);
    if (!e) e = dalloc(&pb, sizeof(int) * d->nB);
    if (!e) e = dalloc(&pc, sizeof(double) * d->max_gaussians);
    if (!e) e = dalloc(&ph, sizeof(double) * d->max_gaussians);
    if (!e) e = dalloc(&pn, sizeof(int));
    if (!e && (hipMemcpy(pa, d->groupA, sizeof(int) * d->nA, hipMemcpyHostToDevice) != hipSuccess ||
               hipMemcpy(pb, d->groupB, sizeof(int) * d->nB, hipMemcpyHostToDevice) != hipSuccess ||
               hipMemset(pn, 0, sizeof(int)) != hipSuccess))
        e = MOP_EHIP;
    if (e) {
        mop_bias_destroy(b);
        return e;
    }
    bd.A = static_cast<const int*>(pa);
    bd.B = static_cast<const int*>(pb);
    bd.centers = static_cast<double*>(pc);
    bd.heights = static_cast<double*>(ph);
    bd.count = static_cast<int*>(pn);
    *out = b;
    return MOP_OK;
}

void mop_bias_destroy(mop_bias b) {
    if (!b) return;
    for (void* p : b->allocs) (void)hipFree(p);
    delete b;
}

int mop_bias_reset(mop_bias b) {
    if (!b) return MOP_EINVAL;
    run_bias_reset(b->dev, b->plan->sys->ctx->stream);
    return finish(b->plan->sys->ctx);
}

int mop_bias_apply(mop_bias b, const double* R, int32_t N, double* G, double* out,
                   int32_t deposit, void* ws) {
    if (!b || !R || !ws) return MOP_EINVAL;
    if (N < 1) return MOP_EINVAL;
    if (N > b->plan->max_beads) return MOP_ESIZE;
    run_bias(b->dev, R, N, b->plan->hseg.s.Q, G, out, deposit ? 1 : 0, static_cast<int*>(ws),
             b->plan->sys->ctx->stream);
    return finish(b->plan->sys->ctx);
}

int mop_bias_history(mop_bias b, int32_t* count, double* centers, double* heights,
                     int32_t capacity) {
    if (!b || !count) return MOP_EINVAL;
    hipStream_t st = b->plan->sys->ctx->stream;
    if (hipStreamSynchronize(st) != hipSuccess) return MOP_EHIP;
    int n = 0;
    if (hipMemcpy(&n, b->dev.count, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
        return MOP_EHIP;
    *count = n;
    const int m = std::min(n, std::max(capacity, 0));
    if (m > 0 && centers &&
        hipMemcpy(centers, b->dev.centers, sizeof(double) * m, hipMemcpyDeviceToHost) != hipSuccess)
        return MOP_EHIP;
    if (m > 0 && heights &&
        hipMemcpy(heights, b->dev.heights, sizeof(double) * m, hipMemcpyDeviceToHost) != hipSuccess)
        return MOP_EHIP;
    return MOP_OK;
}

int pmd_step(mop_plan plan, mop_bias bias, double* R, double* V, double* G, int32_t N,
             const mop_pmd_params* prm, uint64_t step0, int32_t nsteps, double* energies,
             void* ws) {
    if (!plan || !R || !V || !G || !prm || !ws) return MOP_EINVAL;
    if (bias && bias->plan != plan) return MOP_EINVAL;
    if (N < 1 || nsteps < 1) return MOP_EINVAL;
    if (N > plan->max_beads) return MOP_ESIZE;
    if (!(prm->tau > 0.0) || !(prm->gamma >= 0.0) || !(prm->kT >= 0.0)) return MOP_EINVAL;
    if (!std::isfinite(prm->tau) || !std::isfinite(prm->gamma) || !std::isfinite(prm->kT))
        return MOP_EINVAL;
    hipStream_t st = plan->sys->ctx->stream;
    PmdCoef pc;
    pc.tau = prm->tau;
    pc.c1 = std::exp(-prm->gamma * prm->tau);
    pc.c2 = prm->gamma > 0.0 ? std::sqrt((1.0 - pc.c1 * pc.c1) * prm->kT) : 0.0;
    pc.seed = prm->seed;
    CallPtrs cp = call_ptrs(ws);
    cp.R = R;
    cp.G = G;
    const Launch L = one_path(N, N > 1 ? N - 1 : 1);
    for (int32_t k = 0; k < nsteps; ++k) {
        const uint64_t step = step0 + (uint64_t)k;
        double* ek = energies ? energies + 4 * (size_t)k : nullptr;
        run_pmd_pre(plan->dseg, &plan->hseg, L, R, V, G, pc, step, st);
        cp.veff = nullptr;
        path_sequence(plan->dseg, &plan->hseg, L, cp, true, 0, plan->waves, plan->newton3, st,
                      nullptr, plan);
        if (bias)
            run_bias(bias->dev, R, N, plan->hseg.s.Q, G, ek ? ek + 2 : nullptr,
                     step % (uint64_t)bias->stride == 0 ? 1 : 0, cp.status, st);
        run_pmd_post(plan->dseg, &plan->hseg, L, V, G, pc, cp.ws, ek, 4, bias ? 1 : 0, st);
    }
    return finish_plan(plan);
}

int mop_batch_create(int32_t P, const mop_plan* plans, const int32_t* N, mop_batch* out) {
    if (!out || !plans || !N || P < 1) return MOP_EINVAL;
    *out = nullptr;
    if (P > MAXSEG) return MOP_ESIZE;
    mop_ctx ctx = plans[0] ? plans[0]->sys->ctx : nullptr;
    if (!ctx) return MOP_EINVAL;
    for (int p = 0; p < P; ++p) {
        if (!plans[p] || plans[p]->sys->ctx != ctx || N[p] < 1) return MOP_EINVAL;
        if (plans[p]->hseg.s.elec != 0) return MOP_EINVAL;
        if (N[p] > plans[p]->max_beads) return MOP_ESIZE;
    }
    if (hipSetDevice(ctx->device) != hipSuccess) return MOP_EHIP;
    mop_batch bt = new (std::nothrow) mop_batch_s;
    if (!bt) return MOP_ENOMEM;
    bt->ctx = ctx;
    bt->P = P;
    bt->waves = plans[0]->waves;
    bt->newton3 = plans[0]->newton3;
    bt->N.assign(N, N + P);
    bt->hsegs.resize(P);
    size_t off = 256;
    long long roff = 0;
    for (int p = 0; p < P; ++p) {
        SegDev& sg = bt->hsegs[p];
        base_seg(sg, plans[p]->hseg.s);
        sg.roff = roff;
        sg.vidx = p;
        off = layout(sg, std::max(N[p] - 1, 1), N[p], off);
        roff += (long long)N[p] * sg.s.Q * 3;
    }
    bt->ws_bytes = off;
    bt->dsegs = nullptr;
    if (hipMalloc(&bt->dsegs, sizeof(SegDev) * P) != hipSuccess) {
        delete bt;
        return MOP_ENOMEM;
    }
    if (hipMemcpy(bt->dsegs, bt->hsegs.data(), sizeof(SegDev) * P, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(bt->dsegs);
        delete bt;
        return MOP_EHIP;
    }
    *out = bt;
    return MOP_OK;
}

void mop_batch_destroy(mop_batch batch) {
    if (!batch) return;
    if (batch->dsegs) (void)hipFree(batch->dsegs);
    delete batch;
}

int mop_batch_workspace_size(mop_batch batch, size_t* bytes) {
    if (!batch || !bytes) return MOP_EINVAL;
    *bytes = batch->ws_bytes;
    return MOP_OK;
}

int mop_batch_veff_grad(mop_batch batch, const double* R, double* G, double* veff, int32_t mode,
                        double fd_h, void* ws) {
    if (!batch || !R || !G || !ws) return MOP_EINVAL;
    if (mode < 0 || mode > 2 || (mode != 0 && !(fd_h > 0.0))) return MOP_EINVAL;
    CallPtrs cp = call_ptrs(ws);
    cp.R = R;
    cp.G = G;
    cp.veff = veff;
    cp.fd_h = fd_h;
    Launch L;
    std::memset(&L, 0, sizeof(L));
    L.nseg = batch->P;
    for (int p = 0; p < batch->P; ++p) {
        L.N[p] = batch->N[p];
        L.nb[p] = batch->N[p] > 1 ? batch->N[p] - 1 : 1;
    }
    path_sequence(batch->dsegs, batch->hsegs.data(), L, cp, true, mode, batch->waves,
                  batch->newton3, batch->ctx->stream);
    return finish(batch->ctx);
}

int mop_status(mop_plan plan, const void* ws, int32_t* device_status) {
    if (!plan || !ws || !device_status) return MOP_EINVAL;
    if (hipStreamSynchronize(plan->sys->ctx->stream) != hipSuccess) return MOP_EHIP;
    int v = 0;
    if (hipMemcpy(&v, ws, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return MOP_EHIP;
    *device_status = v;
    return MOP_OK;
}

int mop_status_clear(mop_plan plan, void* ws) {
    if (!plan || !ws) return MOP_EINVAL;
    run_status_clear(static_cast<int*>(ws), plan->sys->ctx->stream);
    return finish(plan->sys->ctx);
}

}  // extern "C"
