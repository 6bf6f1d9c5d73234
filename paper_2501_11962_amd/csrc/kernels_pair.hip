// Pair kernels: the physical force F(R^n) (the do_force work of section 2.1) and the
// exact Hessian-vector product H(R^n) v that replaces the finite-difference term of
// eq. (5), for every pair bead of every path of a call in one launch (in two when only
// bead 1 needs energies: see launch_pair_e).
//
// Work unit: one wave per 8-atom i-cluster (8 consecutive slots of one column).
//   1. Lane-parallel over the x-y column stencil: keep columns whose rectangle lies
//      within the search radius of the cluster's bounding box, and per column the
//      cluster range covering the z window [zlo - r, zhi + r] (two ranges when the
//      window wraps around the box).
//   2. Candidate clusters are listed in LDS; 8 of them (64 atoms) are loaded per step,
//      one atom per lane, converted to FP32 coordinates relative to the i-cluster's box
//      centre (exact integer minimum image, then one rounding) and kept when within the
//      cutoff of the i-cluster's bounding box.  Survivors are compacted (ballot + mbcnt)
//      into a per-wave LDS ring.
//   3. Every EB (64) ring entries, EB/8 steps of 8 j-atoms x 8 i-atoms (lane = 8*i + j)
//      evaluate the pair terms; each lane accumulates a partial sum for its i atom.
//   4. Partial sums are reduced over the 8 j lanes.
//   The force pass records each cluster's neighbour list (one record per candidate
//   cluster with survivors); the Hessian pass of the same bead replays it instead of
//   steps 1-2.
// Launch: a flat grid (one workgroup per W clusters, k_pair) or, as a plan option, a
// persistent grid over per-XCD work queues (k_pair_q); both run the same per-wave body.
// Energies are a template parameter, so that kernels that need none take fewer
// registers and hold more waves per SIMD (PAIR_WAVES).
//
// Two variants:
//   N3 = 1 (opt-in): Newton's third law.  A wave takes only clusters with a larger
//      index than its own, so every pair of distinct clusters is evaluated once.  The
//      j-side contribution of a step is summed over the 8 i lanes (lane exchanges) and
//      added to its ring entry by one lane, and, once per EB entries, flushed to a
//      slot-order FP32 buffer with one global atomic per entry and component; i-sums are
//      added the same way.  The own cluster is one 8 x 8 block evaluated from both
//      sides.  Summation order depends on scheduling.
//   N3 = 0 (default): every pair evaluated from both sides; no atomics; run-to-run
//      reproducible for a given binning.  Results go straight to original atom order.
//      Measured on MI355X (150,000 atoms, 15 beads), this is the faster variant: the
//      global flush of the j-side sums (three float atomics per ring entry) costs more
//      than the pair work it saves.
//
// Pair terms, d = x_j - x_i, r = |d|, shifted-force LJ + reaction field:
//   g = phi_sf'(r)/r = G6 r^-8 + qq (2 k_rf - r^-3) + C1 r^-1,   G6 = a12 r^-6 + a6,
//       C1 = -phi'(r_c) = csf + qq crf1
//   h = (phi'' - phi_sf'/r)/r^2 = (b12 r^-6 + b6) r^-10 + 3 qq r^-5 - C1 r^-3,
//       where b12 r^-6 + b6 = -8 (0.75 a12 r^-6 + G6) (b12 = -14 a12, b6 = -8 a6), so
//       the Hessian kernel reads one table entry {a12, a6, csf, 0.75 a12} per pair
//   F_i += g d,   (H v)_i += g (v_i - v_j) + h (d . (v_i - v_j)) d   (j: the opposite)
//
// Ewald variant (EL = 1, systems with particle-mesh Ewald): the reaction-field terms
// become the Ewald real-space term qq psi(r), psi = erfc(beta r)/r, shifted-force at r_c
// (C1 = csf + qq crf1 with crf1 = -psi'(r_c)), and excluded partners within r_c carry
// the correction qq (erfc(beta r) - 1)/r = -qq erf(beta r)/r instead of nothing.  With
// E = erfc(beta r) (minus 1 for excluded pairs) and D = 2 beta/sqrt(pi) exp(-beta^2 r^2):
//   g_el = -(D r^-2 + E r^-3),   h_el = (2 beta^2 D + 3 D r^-2 + 3 E r^-3) r^-2.
// erfc(x) = exp(-x^2) erfcx(x) with erfcx a polynomial in t = 1/(1 + x/2) fitted on
// 0 <= x <= 6 (coefficients from erfc_fit.py next to this package; relative error below
// 4e-7 in FP32), so E and D share one exponential.
#include <algorithm>
#include <atomic>
#include <type_traits>

#include "device_common.h"
#include "launch.h"

namespace mop {

// Ring entries evaluated per batch (EB / 8 steps of 8 j-atoms), as soon as that many wait.
// Each lane sums its entries in ring order, so the batch size changes no result; measured
// on the membrane workload, batches of 32 and 16 were 2% and 8% slower than 64 (the fixed
// cost of a batch outweighs the better spread of pair work between candidate loads).
#ifndef MOP_EVAL_BATCH
#define MOP_EVAL_BATCH 64
#endif
constexpr int EB = MOP_EVAL_BATCH;
static_assert(EB % 8 == 0 && EB <= 64 && RING % EB == 0, "evaluation batch");

// Ring of j-atoms, one per wave in LDS (ints stored as float bits; the key word is the
// packed 16 * exclusion key + LJ type of the system's key table).  Full-shell kernels keep
// entries as float4 {x, y, z, q} followed by float4 {key, v_x, v_y, v_z} (Hessian) or a
// float {key} (force), so a step reads a j-atom with one or two 16-byte loads.  The
// Newton-3 kernels keep one array per field [field][entry], F_* below.
constexpr int F_X = 0, F_Y = 1, F_Z = 2, F_Q = 3, F_K = 4, F_S = 5, F_J = 6;

// Table entries per type pair in LDS, 16 bytes apart: the force kernels keep
// {a12, a6, csf, e0lj} for the nt^2 pairs followed by {b12, b6, c12, c6} (energies);
// the Hessian kernel keeps {a12, a6, csf, 0.75 a12}.
template <int MODE>
constexpr int TAB_COPIES = MODE == 1 ? 1 : 2;

// erfc(x) for 0 <= x <= 6 given ex2 = exp(-x^2).
__device__ __forceinline__ float erfc_ex2(float x, float ex2) {
    const float t = __builtin_amdgcn_rcpf(fmaf(0.5f, x, 1.0f));
    float p = -3.256256573e-02f;
    p = fmaf(p, t, 2.505454269e-01f);
    p = fmaf(p, t, -6.964120320e-01f);
    p = fmaf(p, t, 7.776858691e-01f);
    p = fmaf(p, t, -2.269658047e-01f);
    p = fmaf(p, t, 3.915052002e-01f);
    p = fmaf(p, t, 2.504345553e-01f);
    p = fmaf(p, t, 2.859732478e-01f);
    p = fmaf(p, t, -2.038257043e-04f);
    return ex2 * p;
}

template <int MODE, int N3>
struct Fields {
    static constexpr int V = N3 ? F_J + 3 : F_K + 1;  // v_j (HVP only)
    static constexpr int NF = MODE == 1 ? V + 3 : V;
};

struct IAtom {
    float x, y, z, q, vx, vy, vz;
    uint32_t ux, uy, uz;
    uint32_t kp;  // 16 * (key + 2) + 15, from the packed word 16 * key + type
    int tiN;
    bool v;
};

struct PairK {
    float sx, sy, sz, rc2, krf2, crf1, krf, crf, e0rf, beta, c2b, b2x2;
    float krf2_3, crf1_3;  // krf2 / 3, crf1 / 3 (Hessian kernel: charges carried as 3 q_j)
};

// The reaction-field Hessian kernel keeps 3 q_j in its ring, so that the 3 qq of h needs no
// multiply; g and C1 then use constants divided by 3.
template <int MODE, int N3, int EL>
constexpr bool THREE_Q = MODE == 1 && N3 == 0 && EL == 0;

// One pair term for lane atom I and j-atom (jx, jy, jz): coordinates relative to the
// box centre, or (EX) raw fixed-point bits.  The contribution to atom i (force: g d;
// HVP: g (v_i - v_j) + h (d . (v_i - v_j)) d) is added to (ax, ay, az) with fused
// multiply-adds; with T_OUT it is also returned in t (for the j side).  tabrow points
// at the type-table row of atom i.
template <int MODE, bool EX, bool WANTE, bool T_OUT, int EL, bool Q3 = false>
__device__ __forceinline__ void pair_term(const IAtom& I, const PairK& P, const float4* tabrow,
                                          int ntab,
                                          float jx, float jy, float jz,
                                          float qj, uint32_t kj, float vjx, float vjy,
                                          float vjz, bool valid, float& ax, float& ay,
                                          float& az, float& tx, float& ty, float& tz,
                                          float& en) {
    float dx, dy, dz;
    if (EX) {
        dx = (float)(int)(__float_as_uint(jx) - I.ux) * P.sx;
        dy = (float)(int)(__float_as_uint(jy) - I.uy) * P.sy;
        dz = (float)(int)(__float_as_uint(jz) - I.uz) * P.sz;
    } else {
        dx = jx - I.x;
        dy = jy - I.y;
        dz = jz - I.z;
    }
    const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
    // kj = 16 key_j + type_j, so I.kp - kj = 16 (key_i - key_j + 2) + 15 - type_j (keys
    // below 2^27, no wrap-around): it lies in [0, 79] exactly when |key_i - key_j| <= 2
    // (same molecule within two chain positions), and in [32, 47] for the atom itself
    const uint32_t kd = I.kp - kj;
    const int tj = (int)(kj & 15u);
    const bool exc = kd <= 79u;
    const bool near = valid & I.v & (r2 < P.rc2);
    const bool in = near & !exc;
    const bool cor = EL == 1 && near && exc && (kd - 32u > 15u);  // Ewald correction
    // masked lanes (self pair at r = 0, stale ring entries) may form inf/NaN here; every
    // result they feed is replaced by 0 through a select below, never multiplied
    const float r2s = r2;
    const float rinv = __builtin_amdgcn_rsqf(r2s);
    const float rinv2 = rinv * rinv;
    const float rinv3 = rinv2 * rinv;
    const float rinv6 = rinv3 * rinv3;
    const float4 T = tabrow[tj];
    const float qq = I.q * qj;  // 3 q_i q_j when Q3
    const float C1 = fmaf(qq, Q3 ? P.crf1_3 : P.crf1, T.z);
    const float G6 = fmaf(T.x, rinv6, T.y);
    const float rinv8 = rinv6 * rinv2;
    float g, E = 0.0f, D = 0.0f, r = 0.0f;
    if (EL == 0) {
        g = G6 * rinv8;
        g = fmaf(qq, Q3 ? fmaf(rinv3, -1.0f / 3.0f, P.krf2_3) : P.krf2 - rinv3, g);
        g = fmaf(C1, rinv, g);
        g = in ? g : 0.0f;
    } else {
        r = r2s * rinv;
        const float bx = P.beta * r;
        const float ex2 = __expf(-bx * bx);
        const float ec = erfc_ex2(bx, ex2);
        D = P.c2b * ex2;
        E = exc ? ec - 1.0f : ec;
        const float ge = -fmaf(D, rinv2, E * rinv3);
        const float gs = fmaf(G6, rinv8, C1 * rinv);
        g = in ? fmaf(qq, ge, gs) : (cor ? qq * ge : 0.0f);
    }
    if (MODE == 0) {
        if (T_OUT) {
            tx = g * dx;
            ty = g * dy;
            tz = g * dz;
            ax += tx;
            ay += ty;
            az += tz;
        } else {
            ax = fmaf(g, dx, ax);
            ay = fmaf(g, dy, ay);
            az = fmaf(g, dz, az);
        }
        if (WANTE) {
            const float4 T2 = tabrow[ntab + tj];
            if (EL == 0) r = r2s * rinv;
            float e = fmaf(T2.z, rinv6, -T2.w) * rinv6;
            const float eel = EL == 0 ? rinv + P.krf * r2s - P.crf + P.e0rf + P.crf1 * r
                                      : fmaf(E, rinv, fmaf(P.crf1, r, P.e0rf));
            e = fmaf(qq, eel, e);
            e += fmaf(T.z, r, T.w);
            en = in ? e : (cor ? qq * E * rinv : 0.0f);
        }
    } else {
        const float h6 = fmaf(T.w, rinv6, G6);
        float h;
        if (EL == 0) {
            // h = r^-5 (3 qq - 8 h6 r^-5) - C1 r^-3
            const float rinv5 = rinv3 * rinv2;
            h = fmaf(h6 * rinv5, -8.0f, Q3 ? qq : 3.0f * qq);
            h = fmaf(rinv5, h, -(C1 * rinv3));
            h = in ? h : 0.0f;
        } else {
            h = h6 * (rinv8 * (-8.0f * rinv2));
            const float he = fmaf(P.b2x2, D, 3.0f * fmaf(D, rinv2, E * rinv3)) * rinv2;
            h = fmaf(-C1, rinv3, h);
            h = in ? fmaf(qq, he, h) : (cor ? qq * he : 0.0f);
        }
        const float dvx = I.vx - vjx, dvy = I.vy - vjy, dvz = I.vz - vjz;
        const float sd = fmaf(dx, dvx, fmaf(dy, dvy, dz * dvz));
        const float hs = h * sd;
        if (T_OUT) {
            tx = fmaf(g, dvx, hs * dx);
            ty = fmaf(g, dvy, hs * dy);
            tz = fmaf(g, dvz, hs * dz);
            ax += tx;
            ay += ty;
            az += tz;
        } else {
            ax = fmaf(g, dvx, fmaf(hs, dx, ax));
            ay = fmaf(g, dvy, fmaf(hs, dy, ay));
            az = fmaf(g, dvz, fmaf(hs, dz, az));
        }
    }
}

// Copy segment p's pair table(s) to LDS: threads t0, t0 + stride, ... of the caller's group.
template <int MODE>
__device__ __forceinline__ void load_table(const SegDev* __restrict__ sg, float4* s_tab, int t0, int stride) {
    const int nt = sg->s.nt;
    for (int t = t0; t < nt * nt; t += stride) {
        if (MODE == 1) {
            s_tab[t] = sg->s.tabh[t];
        } else {
            s_tab[t] = sg->s.tab[t];
            s_tab[nt * nt + t] = sg->s.tab2[t];
        }
    }
}

// The work of one wave: i-cluster gw of path p (bead bead0 + gw / cpb, cluster gw % cpb),
// with the path's table at s_tab and the wave's own ring and candidate list in LDS.
// ENERGY: the kernel can sum pair energies (of bead energy_bead, or of every bead for -2);
// kernels without it need fewer registers.
template <int MODE, int N3, int EL, int ENERGY>
__device__ __forceinline__ void pair_wave(const SegDev* __restrict__ segs, const Launch& L,
                                          char* __restrict__ ws, int outsel, int energy_bead,
                                          int lists, int bead0, int p, int gw, const float4* s_tab,
                                          float* ring, int* clist) {
    using FL = Fields<MODE, N3>;
    constexpr int NF = FL::NF, FV = FL::V;
    const SegDev* __restrict__ sg = segs + p;
    const int nt = sg->s.nt;
    const int lane = threadIdx.x & 63;
    const int cpb = sg->s.cpb;
    const int bl = gw / cpb, c = gw - bl * cpb;
    if (bl >= L.nb[p]) return;
    const int b = bead0 + bl;
    const int S = sg->s.S, Q = sg->s.Q, ncol = sg->s.ncol, nzb = sg->s.nzb;
    const int ncx = sg->s.ncx, ncy = sg->s.ncy;
    const uint4* __restrict__ upos = wsp<const uint4>(ws, sg->o_upos) + (size_t)b * S;
    const int2* __restrict__ umeta = wsp<const int2>(ws, sg->o_umeta) + (size_t)b * S;
    const int* __restrict__ colstart = wsp<const int>(ws, sg->o_colstart) + (size_t)b * (ncol + 1);
    const int* __restrict__ binoff = wsp<const int>(ws, sg->o_binoff) + (size_t)b * ncol * (nzb + 1);
    const float4* __restrict__ vs = wsp<const float4>(ws, sg->o_vs) + (size_t)b * S;
    float* __restrict__ fsx = wsp<float>(ws, sg->o_fs) + (size_t)b * 3 * S;
    float* __restrict__ fsy = fsx + S;
    float* __restrict__ fsz = fsy + S;
    const int nslots = colstart[ncol];
    if (c * CLUSTER >= nslots) return;

    const bool wantE = MODE == 0 && ENERGY && (energy_bead == -2 || energy_bead == b);
    PairK P;
    P.sx = sg->s.sc[0];
    P.sy = sg->s.sc[1];
    P.sz = sg->s.sc[2];
    P.rc2 = sg->s.rc2;
    P.krf2 = sg->s.krf2;
    P.crf1 = sg->s.crf1;
    P.krf = sg->s.krf;
    P.crf = sg->s.crf;
    P.e0rf = sg->s.e0rf;
    P.beta = sg->s.ew_beta;
    P.c2b = sg->s.ew_c2b;
    P.b2x2 = sg->s.ew_b2x2;
    P.krf2_3 = sg->s.krf2 * (1.0f / 3.0f);
    P.crf1_3 = sg->s.crf1 * (1.0f / 3.0f);
    constexpr float QSC = THREE_Q<MODE, N3, EL> ? 3.0f : 1.0f;
    const float sx = P.sx, sy = P.sy, sz = P.sz;
    const float rcs = sg->s.rcs, rcs2 = sg->s.rcs2;

    // ---- the i-cluster ------------------------------------------------------------
    const int isub = lane >> 3, jslot = lane & 7;
    const int si = c * CLUSTER + isub;
    const uint4 ui = upos[si];
    const int2 mi = umeta[si];
    // first reference point: the cluster's middle atom (atoms of a cluster are z-sorted
    // inside one column)
    const uint4 ref = upos[c * CLUSTER + 3];
    IAtom I;
    I.v = mi.x != DUMMY_KEY;
    I.q = __uint_as_float(ui.w);
    I.kp = (uint32_t)(mi.x - mi.y) + 47u;
    I.tiN = mi.y * nt;
    const float4* tabrow = s_tab + I.tiN;
    const int ntab = nt * nt;
    I.ux = ui.x;
    I.uy = ui.y;
    I.uz = ui.z;
    I.vx = I.vy = I.vz = 0.0f;
    if (MODE == 1) {
        const float4 v4 = vs[si];
        I.vx = v4.x;
        I.vy = v4.y;
        I.vz = v4.z;
    }
    // bounding box relative to the reference atom, then to its own centre
    float lox, hix, loy, hiy, loz, hiz;
    auto bbox = [&](float x, float y, float z) __attribute__((always_inline)) {
        lox = I.v ? x : 3.0e38f;
        hix = I.v ? x : -3.0e38f;
        loy = I.v ? y : 3.0e38f;
        hiy = I.v ? y : -3.0e38f;
        loz = I.v ? z : 3.0e38f;
        hiz = I.v ? z : -3.0e38f;
        auto step = [&](auto mc) __attribute__((always_inline)) {
            constexpr int M = decltype(mc)::value;
            lox = fminf(lox, lane_xor<M>(lox));
            hix = fmaxf(hix, lane_xor<M>(hix));
            loy = fminf(loy, lane_xor<M>(loy));
            hiy = fmaxf(hiy, lane_xor<M>(hiy));
            loz = fminf(loz, lane_xor<M>(loz));
            hiz = fmaxf(hiz, lane_xor<M>(hiz));
        };
        step(std::integral_constant<int, 8>{});
        step(std::integral_constant<int, 16>{});
        step(std::integral_constant<int, 32>{});
    };
    bbox((float)(int)(ui.x - ref.x) * sx, (float)(int)(ui.y - ref.y) * sy,
         (float)(int)(ui.z - ref.z) * sz);
    // re-reference to the box centre uc: the image of an atom nearest the centre is the
    // one nearest the box, which keeps the candidate test conservative in small boxes.
    // The shifted bounds may differ from the atoms' new coordinates by an ulp, which the
    // search-radius margin absorbs.
    const int ocx = (int)rintf(0.5f * (lox + hix) / sx);
    const int ocy = (int)rintf(0.5f * (loy + hiy) / sy);
    const int ocz = (int)rintf(0.5f * (loz + hiz) / sz);
    const uint32_t ucx = ref.x + (uint32_t)ocx, ucy = ref.y + (uint32_t)ocy, ucz = ref.z + (uint32_t)ocz;
    {
        const float fx = (float)ocx * sx, fy = (float)ocy * sy, fz = (float)ocz * sz;
        lox -= fx;
        hix -= fx;
        loy -= fy;
        hiy -= fy;
        loz -= fz;
        hiz -= fz;
    }
    I.x = (float)(int)(ui.x - ucx) * sx;
    I.y = (float)(int)(ui.y - ucy) * sy;
    I.z = (float)(int)(ui.z - ucz) * sz;
    // Coordinates relative to the reference give exact pair differences when
    // max(|lo|, |hi|) + search radius < L/2 along every axis: for a pair within the
    // cutoff, (image of i) + d then lies within L/2 of the reference, so it is the image
    // of j that the relative coordinate picks.  Otherwise each pair difference is taken
    // from the fixed-point coordinates (small boxes, sparse columns).
    const bool exact = (fmaxf(-lox, hix) + rcs >= 0.5f * sg->s.Lf[0]) ||
                       (fmaxf(-loy, hiy) + rcs >= 0.5f * sg->s.Lf[1]) ||
                       (fmaxf(-loz, hiz) + rcs >= 0.5f * sg->s.Lf[2]);
    const int cx = fixed_bin(ref.x, ncx), cy = fixed_bin(ref.y, ncy);

    // z window of candidate atoms of a column whose rectangle is (gx, gy) away from the
    // bounding box: |z - box| < sqrt(rcs^2 - gx^2 - gy^2), in z bins (per lane)
    const float Lz = sg->s.Lf[2];
    // reciprocals instead of divisions: a z bound off by one fixed-point unit, or a
    // column image chosen either way at an exact half-box tie (both images then lie at
    // the same distance), changes no test
    const float isz = 1.0f / sz;
    auto zwindow = [&](float g2, bool& fullz, bool& zwrap, int& zb0, int& zb1)
                       __attribute__((always_inline)) {
        const float hz = sqrtf(fmaxf(rcs2 - g2, 0.0f));
        fullz = (hiz - loz + 2.0f * hz) >= Lz;
        zb0 = 0;
        zb1 = nzb - 1;
        zwrap = false;
        if (!fullz) {
            const long long dlo = (long long)floorf((loz - hz) * isz);
            const long long dhi = (long long)ceilf((hiz + hz) * isz);
            const uint32_t zlo = ucz + (uint32_t)dlo;
            const uint32_t zhi = ucz + (uint32_t)dhi;
            zb0 = fixed_bin(zlo, nzb);
            zb1 = fixed_bin(zhi, nzb);
            zwrap = zlo > zhi;
            if (zwrap && zb1 + 1 >= zb0) fullz = true;
        }
    };
    const float bcx = 0.5f * (lox + hix), bhx = 0.5f * (hix - lox);
    const float bcy = 0.5f * (loy + hiy), bhy = 0.5f * (hiy - loy);
    const float xref = (float)ucx * sx, yref = (float)ucy * sy;
    const float Lx = sg->s.Lf[0], Ly = sg->s.Lf[1];
    const float iLx = 1.0f / Lx, iLy = 1.0f / Ly;
    const float cwx = sg->s.cw[0], cwy = sg->s.cw[1];

    float ax = 0.f, ay = 0.f, az = 0.f;
    float eacc = 0.0f;
    double eacc64 = 0.0;
    int wp = 0, rp = 0;  // ring write / read counters (uniform); rp stays a multiple of EB
    int wr = 0;          // neighbour-list records written (force pass)

    float4* ring4 = reinterpret_cast<float4*>(ring);

    // neighbour lists (full-shell kernels): the force pass records the slots that pass
    // the search, the Hessian pass of the same bead replays them
    const int lcap = sg->s.lcap;
    const bool rec = !N3 && MODE == 0 && lists == 1 && lcap > 0;
    const bool rpl = !N3 && lists == 2 && lcap > 0;
    int* __restrict__ nl = nullptr;
    int* __restrict__ nlc = nullptr;
    if (rec || rpl) {
        nl = wsp<int>(ws, sg->o_nl) + ((size_t)b * cpb + c) * lcap;
        nlc = wsp<int>(ws, sg->o_nlc) + (size_t)b * cpb + c;
    }

    // ---- own cluster (N3): one 8 x 8 block, both sides, weight 1/2 for energies ----
    if (N3) {
        const int sj = c * CLUSTER + jslot;
        const uint4 uj = upos[sj];
        const int2 mj = umeta[sj];
        float jx, jy, jz, vjx = 0.f, vjy = 0.f, vjz = 0.f;
        if (exact) {
            jx = __uint_as_float(uj.x);
            jy = __uint_as_float(uj.y);
            jz = __uint_as_float(uj.z);
        } else {
            jx = (float)(int)(uj.x - ucx) * sx;
            jy = (float)(int)(uj.y - ucy) * sy;
            jz = (float)(int)(uj.z - ucz) * sz;
        }
        if (MODE == 1) {
            const float4 v4 = vs[sj];
            vjx = v4.x;
            vjy = v4.y;
            vjz = v4.z;
        }
        float tx, ty, tz, en = 0.f;
        const bool vj = mj.x != DUMMY_KEY;
        const float qj = __uint_as_float(uj.w);
        if (exact) {
            if (wantE)
                pair_term<MODE, true, true, false, EL>(I, P, tabrow, ntab, jx, jy, jz, qj, (uint32_t)mj.x, vjx,
                                            vjy, vjz, vj, ax, ay, az, tx, ty, tz, en);
            else
                pair_term<MODE, true, false, false, EL>(I, P, tabrow, ntab, jx, jy, jz, qj, (uint32_t)mj.x, vjx,
                                             vjy, vjz, vj, ax, ay, az, tx, ty, tz, en);
        } else {
            if (wantE)
                pair_term<MODE, false, true, false, EL>(I, P, tabrow, ntab, jx, jy, jz, qj, (uint32_t)mj.x, vjx,
                                             vjy, vjz, vj, ax, ay, az, tx, ty, tz, en);
            else
                pair_term<MODE, false, false, false, EL>(I, P, tabrow, ntab, jx, jy, jz, qj, (uint32_t)mj.x, vjx,
                                              vjy, vjz, vj, ax, ay, az, tx, ty, tz, en);
        }
        eacc += 0.5f * en;
    }

    // ---- 8 j-atoms x 8 i-atoms per step from ring entries [base, base + count) ------
    // base is a multiple of EB, so reads of a chunk never wrap and every field of every
    // step is one immediate offset from the same address.
    auto eval_t = [&]<bool EX, bool WE, bool FULL>(int base, int count)
                      __attribute__((always_inline)) {
        float* rb = ring + (base & (RING - 1)) + jslot;
        const int e0 = (base & (RING - 1)) + jslot;
        const int nsteps = FULL ? EB / 8 : (count + 7) >> 3;
#pragma unroll
        for (int s = 0; s < nsteps; ++s) {
            const int o = s * 8;
            float jx, jy, jz, qj, vjx = 0.f, vjy = 0.f, vjz = 0.f;
            uint32_t kj;
            if (N3) {
                jx = rb[F_X * RING + o];
                jy = rb[F_Y * RING + o];
                jz = rb[F_Z * RING + o];
                qj = rb[F_Q * RING + o];
                kj = __float_as_uint(rb[F_K * RING + o]);
                if (MODE == 1) {
                    vjx = rb[FV * RING + o];
                    vjy = rb[(FV + 1) * RING + o];
                    vjz = rb[(FV + 2) * RING + o];
                }
            } else {
                const float4 a = ring4[e0 + o];
                jx = a.x;
                jy = a.y;
                jz = a.z;
                qj = a.w;
                if (MODE == 1) {
                    const float4 w = ring4[RING + e0 + o];
                    kj = __float_as_uint(w.x);
                    vjx = w.y;
                    vjy = w.z;
                    vjz = w.w;
                } else {
                    kj = __float_as_uint(ring[4 * RING + e0 + o]);
                }
            }
            const bool valid = FULL || o + jslot < count;
            // Entries past the count of a partial chunk may hold anything (never written
            // in this wave's lifetime): masked products are still formed (0 * dx, 0 * dv),
            // so give them finite operands and a valid table index.
            float jxv = jx, jyv = jy, jzv = jz, qjv = qj;
            uint32_t kjv = kj;
            if (!FULL) {
                jxv = valid ? jx : 0.0f;
                jyv = valid ? jy : 0.0f;
                jzv = valid ? jz : 0.0f;
                qjv = valid ? qj : 0.0f;
                kjv = valid ? kj : 0u;
                if (MODE == 1) {
                    vjx = valid ? vjx : 0.0f;
                    vjy = valid ? vjy : 0.0f;
                    vjz = valid ? vjz : 0.0f;
                }
            }
            float tx, ty, tz, en = 0.f;
            pair_term<MODE, EX, WE, N3 == 1, EL, THREE_Q<MODE, N3, EL>>(I, P, tabrow, ntab, jxv, jyv, jzv, qjv, kjv, vjx, vjy,
                                             vjz, valid, ax, ay, az, tx, ty, tz, en);
            if (WE) eacc += N3 ? en : 0.5f * en;
            if (N3) {
                // sum the j side over the 8 i lanes (lanes 8 apart), then the 8 lanes of
                // i-atom 0 add it to their ring entries: one plain LDS update per entry
                tx += lane_xor<8>(tx);
                ty += lane_xor<8>(ty);
                tz += lane_xor<8>(tz);
                tx += lane_xor<16>(tx);
                ty += lane_xor<16>(ty);
                tz += lane_xor<16>(tz);
                tx += lane_xor<32>(tx);
                ty += lane_xor<32>(ty);
                tz += lane_xor<32>(tz);
                if (lane < 8) {
                    rb[(F_J + 0) * RING + o] += tx;
                    rb[(F_J + 1) * RING + o] += ty;
                    rb[(F_J + 2) * RING + o] += tz;
                }
            }
        }
        if (WE) {  // FP32 partial of at most 64 pair terms per lane, summed in FP64
            eacc64 += (double)eacc;
            eacc = 0.0f;
        }
        if (N3) {
            // j-side sums of this chunk (stored with the sign of the i side) go to the
            // slot-order buffer, one entry per lane
            wave_sync();
            if (FULL ? lane < EB : lane < count) {
                const int e = (base & (RING - 1)) + lane;
                const int slot = __float_as_int(ring[F_S * RING + e]);
                unsafeAtomicAdd(fsx + slot, -ring[(F_J + 0) * RING + e]);
                unsafeAtomicAdd(fsy + slot, -ring[(F_J + 1) * RING + e]);
                unsafeAtomicAdd(fsz + slot, -ring[(F_J + 2) * RING + e]);
            }
        }
    };
    auto eval = [&]<bool FULL>(int base, int count) __attribute__((always_inline)) {
        if (exact) {
            if (wantE) eval_t.template operator()<true, true, FULL>(base, count);
            else eval_t.template operator()<true, false, FULL>(base, count);
        } else {
            if (wantE) eval_t.template operator()<false, true, FULL>(base, count);
            else eval_t.template operator()<false, false, FULL>(base, count);
        }
    };

    // ---- candidate clusters [0, T) of clist --------------------------------------
    // Candidate atoms are loaded one chunk (8 clusters) ahead of their use, so the
    // global-load latency of chunk q+1 overlaps the tests, ring writes and pair
    // evaluations of chunk q.
    auto process = [&](int T) __attribute__((always_inline)) {
        // lanes without a candidate load slot 0 (always present) and are rejected by
        // the slot test below; no select between pointers, so the loads stay global
        int nslot = (lane >> 3) < T ? clist[lane >> 3] * CLUSTER + (lane & 7) : -1;
        uint4 nuj = upos[max(nslot, 0)];
        int2 nmj = umeta[max(nslot, 0)];
        float4 njv = make_float4(0.f, 0.f, 0.f, 0.f);
        if (MODE == 1) njv = vs[max(nslot, 0)];
        for (int q = 0; q < T; q += 8) {
            const int slot = nslot;
            const uint4 uj = nuj;
            const int2 mj = nmj;
            const float4 jv = njv;
            {
                const int cn = q + 8 + (lane >> 3);
                nslot = cn < T ? clist[cn] * CLUSTER + (lane & 7) : -1;
                if (nslot >= 0) {
                    nuj = upos[nslot];
                    nmj = umeta[nslot];
                    if (MODE == 1) njv = vs[nslot];
                }
            }
            float jx = (float)(int)(uj.x - ucx) * sx;
            float jy = (float)(int)(uj.y - ucy) * sy;
            float jz = (float)(int)(uj.z - ucz) * sz;
            const float ex = fmaxf(fmaxf(lox - jx, jx - hix), 0.0f);
            const float ey = fmaxf(fmaxf(loy - jy, jy - hiy), 0.0f);
            const float ez = fmaxf(fmaxf(loz - jz, jz - hiz), 0.0f);
            const bool pass = (slot >= 0) & (mj.x != DUMMY_KEY) &
                              (fmaf(ex, ex, fmaf(ey, ey, ez * ez)) < rcs2);
            if (exact) {
                jx = __uint_as_float(uj.x);
                jy = __uint_as_float(uj.y);
                jz = __uint_as_float(uj.z);
            }
            const float jq = __uint_as_float(uj.w);
            const int jk = mj.x;
            const unsigned long long m = __ballot(pass);
            const int off = __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                                      __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
            wave_sync();  // previous reads of the ring are done before it is overwritten
            if (rec) {
                // one record per candidate cluster of this chunk with a survivor, in
                // candidate order: (cluster index << 8) | mask of its surviving atoms.
                // Lanes 8k .. 8k+7 hold the atoms of the chunk's k-th cluster; lane 8k
                // writes its record (its slot is the cluster's first).
                const uint32_t mk = (lane & 7) == 0 ? (uint32_t)(m >> lane) & 0xFFu : 0u;
                const unsigned long long nzm = __ballot(mk != 0u);
                if (mk != 0u) {
                    const int pos = wr + __builtin_amdgcn_mbcnt_hi(
                        (unsigned)(nzm >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)nzm, 0u));
                    if (pos < lcap) nl[pos] = (int)(((uint32_t)slot << 5) | mk);
                }
                wr += (int)__popcll(nzm);
            }
            if (pass) {
                const int e = (wp + off) & (RING - 1);
                if (N3) {
                    float* re = ring + e;
                    re[F_X * RING] = jx;
                    re[F_Y * RING] = jy;
                    re[F_Z * RING] = jz;
                    re[F_Q * RING] = QSC * jq;
                    re[F_K * RING] = __int_as_float(jk);
                    re[F_S * RING] = __int_as_float(slot);
                    re[(F_J + 0) * RING] = 0.0f;
                    re[(F_J + 1) * RING] = 0.0f;
                    re[(F_J + 2) * RING] = 0.0f;
                    if (MODE == 1) {
                        re[FV * RING] = jv.x;
                        re[(FV + 1) * RING] = jv.y;
                        re[(FV + 2) * RING] = jv.z;
                    }
                } else {
                    ring4[e] = make_float4(jx, jy, jz, QSC * jq);
                    if (MODE == 1) ring4[RING + e] = make_float4(__int_as_float(jk), jv.x, jv.y, jv.z);
                    else ring[4 * RING + e] = __int_as_float(jk);
                }
            }
            wp += __popcll(m);
            wave_sync();
            while (wp - rp >= EB) {
                eval.template operator()<true>(rp, EB);
                rp += EB;
                wave_sync();
            }
        }
    };

    // ---- replay of a recorded list: 8 records (up to 64 atoms) per chunk -----------
    // Lane l takes atom l & 7 of record l >> 3 and keeps it when the record's mask has its
    // bit; survivors are compacted into the ring exactly as the search compacted them, so
    // the ring order, and every sum, is the search's.  Records are read two chunks ahead,
    // atom data one chunk ahead.
    auto replay = [&](int cnt) __attribute__((always_inline)) {
        const int rsub = lane >> 3, atom = lane & 7;
        uint32_t r1 = rsub < cnt ? (uint32_t)nl[rsub] : 0u;
        uint32_t r2 = 8 + rsub < cnt ? (uint32_t)nl[8 + rsub] : 0u;
        bool p1 = (r1 >> atom) & 1u;
        int s1 = (int)(r1 >> 8) * CLUSTER + atom;  // a lane without a record reads slot atom
        uint4 nuj = make_uint4(0u, 0u, 0u, 0u);
        int2 nmj = make_int2(0, 0);
        float4 njv = make_float4(0.f, 0.f, 0.f, 0.f);
        if (p1) {
            nuj = upos[s1];
            nmj = umeta[s1];
            if (MODE == 1) njv = vs[s1];
        }
        for (int k0 = 0; k0 < cnt; k0 += 8) {
            const uint4 uj = nuj;
            const int2 mj = nmj;
            const float4 jv = njv;
            const bool pass = p1;
            r1 = r2;
            p1 = (r1 >> atom) & 1u;
            s1 = (int)(r1 >> 8) * CLUSTER + atom;
            if (p1) {
                nuj = upos[s1];
                nmj = umeta[s1];
                if (MODE == 1) njv = vs[s1];
            }
            r2 = k0 + 16 + rsub < cnt ? (uint32_t)nl[k0 + 16 + rsub] : 0u;
            float jx, jy, jz;
            if (exact) {
                jx = __uint_as_float(uj.x);
                jy = __uint_as_float(uj.y);
                jz = __uint_as_float(uj.z);
            } else {
                jx = (float)(int)(uj.x - ucx) * sx;
                jy = (float)(int)(uj.y - ucy) * sy;
                jz = (float)(int)(uj.z - ucz) * sz;
            }
            const unsigned long long m = __ballot(pass);
            const int off = __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                                      __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
            wave_sync();  // the previous reads of the ring are done before it is overwritten
            if (!N3 && pass) {  // full-shell kernels only
                const int e = (wp + off) & (RING - 1);
                ring4[e] = make_float4(jx, jy, jz, QSC * __uint_as_float(uj.w));
                if (MODE == 1) ring4[RING + e] = make_float4(__int_as_float(mj.x), jv.x, jv.y, jv.z);
                else ring[4 * RING + e] = __int_as_float(mj.x);
            }
            wp += __popcll(m);
            wave_sync();
            while (wp - rp >= EB) {
                eval.template operator()<true>(rp, EB);
                rp += EB;
                wave_sync();
            }
        }
    };
    bool searched = true;
    if (rpl) {
        const int cnt = *nlc;
        if (cnt <= lcap) {
            replay(cnt);
            searched = false;
        }
    }

    // ---- column stencil, 64 columns per pass ---------------------------------------
    const int wx = sg->s.wx, wy = sg->s.wy, nst = searched ? wx * wy : 0;
    for (int k0 = 0; k0 < nst; k0 += 64) {
        const int k = k0 + lane;
        int a0 = 0, a1 = 0, b0 = 0, b1 = 0;
        if (k < nst) {
            const int ox = k / wy, oy = k - ox * wy;
            // stencil half widths are below the column counts (else the stencil spans
            // every column), so one wrap suffices
            int jxc = sg->s.allx ? ox : cx + ox - sg->s.rx;
            int jyc = sg->s.ally ? oy : cy + oy - sg->s.ry;
            jxc += jxc < 0 ? ncx : (jxc >= ncx ? -ncx : 0);
            jyc += jyc < 0 ? ncy : (jyc >= ncy ? -ncy : 0);
            float dxc = ((float)jxc + 0.5f) * cwx - xref;
            dxc -= Lx * rintf(dxc * iLx);
            dxc -= bcx;
            dxc -= Lx * rintf(dxc * iLx);
            float dyc = ((float)jyc + 0.5f) * cwy - yref;
            dyc -= Ly * rintf(dyc * iLy);
            dyc -= bcy;
            dyc -= Ly * rintf(dyc * iLy);
            const float gx = fmaxf(0.0f, fabsf(dxc) - 0.5f * cwx - bhx);
            const float gy = fmaxf(0.0f, fabsf(dyc) - 0.5f * cwy - bhy);
            const int col = jxc * ncy + jyc;
            if (gx * gx + gy * gy < rcs2) {
                bool fullz, zwrap;
                int zb0, zb1;
                zwindow(gx * gx + gy * gy, fullz, zwrap, zb0, zb1);
                const int base = colstart[col];
                const int* bo = binoff + (size_t)col * (nzb + 1);
                const int cnt = bo[nzb];
                if (cnt > 0) {
                    if (fullz) {
                        a0 = base >> 3;
                        a1 = (base + cnt + 7) >> 3;
                    } else if (!zwrap) {
                        a0 = (base + bo[zb0]) >> 3;
                        a1 = (base + bo[zb1 + 1] + 7) >> 3;
                    } else {
                        a0 = (base + bo[zb0]) >> 3;
                        a1 = (base + cnt + 7) >> 3;
                        b0 = base >> 3;
                        b1 = (base + bo[zb1 + 1] + 7) >> 3;
                        if (b1 > a0) b1 = a0;  // never list a cluster twice
                    }
                    if (N3) {  // only clusters after the own one
                        a0 = max(a0, c + 1);
                        b0 = max(b0, c + 1);
                    }
                    if (a1 < a0) a1 = a0;
                    if (b1 < b0) b1 = b0;
                }
            }
        }
        // flatten the per-column cluster ranges into clist, CLIST at a time
        for (;;) {
            const int len = (a1 - a0) + (b1 - b0);
            const int incl = wave_incl_scan(len);
            const int total = __builtin_amdgcn_readlane(incl, 63);
            if (total == 0) break;
            const int excl = incl - len;
            const int take = min(len, max(0, CLIST - excl));
            wave_sync();  // the previous list has been consumed
            for (int t = 0; t < take; ++t) {
                int cl;
                if (a0 < a1) {
                    cl = a0++;
                } else {
                    cl = b0++;
                }
                clist[excl + t] = cl;
            }
            wave_sync();
            process(min(total, CLIST));
        }
    }
    // ---- remaining ring entries ---------------------------------------------------
    if (wp - rp > 0) eval.template operator()<false>(rp, wp - rp);
    if (rec && lane == 0) *nlc = wr;

    // ---- reduce over the 8 j lanes of each i atom and store ------------------------
    ax += lane_xor<1>(ax);
    ay += lane_xor<1>(ay);
    az += lane_xor<1>(az);
    ax += lane_xor<2>(ax);
    ay += lane_xor<2>(ay);
    az += lane_xor<2>(az);
    ax += lane_xor<4>(ax);
    ay += lane_xor<4>(ay);
    az += lane_xor<4>(az);
    if (jslot == 0 && I.v) {
        if (N3) {
            unsafeAtomicAdd(fsx + si, ax);
            unsafeAtomicAdd(fsy + si, ay);
            unsafeAtomicAdd(fsz + si, az);
        } else {
            const int oi = wsp<const int>(ws, sg->o_orig)[(size_t)b * S + si];
            size_t o = sg->o_f32;
            if (MODE == 1 || outsel == 1) o = sg->o_hv32;
            else if (outsel == 2) o = sg->o_f32m;
            wsp<float4>(ws, o)[(size_t)b * Q + oi] = make_float4(ax, ay, az, 0.0f);
        }
    }
    if (wantE) {
        eacc64 += (double)eacc;
        eacc64 += lane_xor<1>(eacc64);
        eacc64 += lane_xor<2>(eacc64);
        eacc64 += lane_xor<4>(eacc64);
        eacc64 += lane_xor<8>(eacc64);
        eacc64 += lane_xor<16>(eacc64);
        eacc64 += lane_xor<32>(eacc64);
        if (lane == 0) wsp<double>(ws, sg->o_epart)[(size_t)b * cpb + c] = eacc64;
    }
}

// Waves per SIMD the pair kernels are compiled for (register budget 512 / waves, in
// steps of 8): 6 (80 registers) for the reaction-field force kernel without energies and
// the full-shell reaction-field Hessian kernel, 5 (96) for the rest; every flat-grid
// kernel fits without spills.  Measured per veff_grad call on the 150,000-atom workload
// against 4 waves (128 registers): -7.5% with reaction field, -1.5% with particle-mesh
// Ewald (whose mesh kernels on the second stream need room beside the pair kernels).  The
// wave index is made scalar (readfirstlane) and the lane exchanges use swizzles
// (lane_xor), so that per-wave pointers and shuffle bounds take no vector registers.
template <int MODE, int N3, int EL, int WE>
constexpr int PAIR_WAVES = EL == 0 && N3 == 0 && (MODE == 1 || WE == 0) ? 6 : 5;

// One workgroup per PW i-clusters; consecutive workgroups of the logical order
// (neighbouring clusters) go to one XCD (workgroups are dealt to the 8 XCDs in turn).
// The launch covers beads bead0 .. bead0 + L.nb[p] - 1 of every path p.
template <int MODE, int PW, int N3, int EL, int WE>
__global__ void __launch_bounds__(64 * PW, (PAIR_WAVES<MODE, N3, EL, WE>))
    k_pair(const SegDev* __restrict__ segs, Launch L, char* __restrict__ ws, int outsel,
           int energy_bead, int lists, int bead0) {
    constexpr int NF = Fields<MODE, N3>::NF;
    extern __shared__ float4 s_dyn[];
    const int nblk = L.pf[L.nseg];
    const int per = (nblk + 7) >> 3;
    const int lblk = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
    if (lblk >= nblk) return;
    const int p = find_seg(L, lblk);
    float4* s_tab = s_dyn;
    float* s_ring = reinterpret_cast<float*>(s_dyn + TAB_COPIES<MODE> * L.ntmax * L.ntmax);
    int* s_cl = reinterpret_cast<int*>(s_ring + PW * NF * RING);
    load_table<MODE>(segs + p, s_tab, threadIdx.x, 64 * PW);
    __syncthreads();  // the only block barrier: waves are independent from here on
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform: scalar indices
    pair_wave<MODE, N3, EL, WE>(segs, L, ws, outsel, energy_bead, lists, bead0, p,
                                (lblk - L.pf[p]) * PW + wave, s_tab, s_ring + wave * NF * RING,
                                s_cl + wave * CLIST);
}

// Persistent form: as many workgroups as the GPU holds at once, each taking logical blocks
// of PW i-clusters (the flat form's workgroups) from its XCD's queue until the queue is
// empty; XCD x owns logical blocks x*per .. (x+1)*per - 1, taken in order.  One block
// barrier per logical block: the taken index goes through two alternating LDS words, so a
// word is rewritten only after every wave has passed the barrier that follows its next
// read.  The path's table is reloaded only when the path changes.  queue: 8 counters, zero
// before the launch.  A block's results do not depend on which workgroup computes it:
// results equal k_pair's.
template <int MODE, int PW, int N3, int EL, int WE>
__global__ void __launch_bounds__(64 * PW, (PAIR_WAVES<MODE, N3, EL, WE>))
    k_pair_q(const SegDev* __restrict__ segs, Launch L, char* __restrict__ ws, int outsel,
             int energy_bead, int lists, int bead0, int* __restrict__ queue) {
    constexpr int NF = Fields<MODE, N3>::NF;
    extern __shared__ float4 s_dyn[];
    __shared__ int s_next[2];
    const int nblk = L.pf[L.nseg];
    const int per = (nblk + 7) >> 3;
    const int x = (int)(blockIdx.x & 7);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform: scalar indices
    float4* s_tab = s_dyn;
    float* s_ring = reinterpret_cast<float*>(s_dyn + TAB_COPIES<MODE> * L.ntmax * L.ntmax);
    int* s_cl = reinterpret_cast<int*>(s_ring + PW * NF * RING);
    int cur = -1;
    for (int it = 0;; it ^= 1) {
        if (threadIdx.x == 0) s_next[it] = atomicAdd(queue + x, 1);
        __syncthreads();  // also: every wave is done with the previous block (and table)
        const int k = s_next[it];
        const int lblk = x * per + k;
        if (k >= per || lblk >= nblk) break;
        const int p = find_seg(L, lblk);
        if (p != cur) {
            load_table<MODE>(segs + p, s_tab, threadIdx.x, 64 * PW);
            __syncthreads();
            cur = p;
        }
        pair_wave<MODE, N3, EL, WE>(segs, L, ws, outsel, energy_bead, lists, bead0, p,
                                    (lblk - L.pf[p]) * PW + wave, s_tab, s_ring + wave * NF * RING,
                                    s_cl + wave * CLIST);
    }
}

__global__ void k_queue_reset(int* queue) { queue[threadIdx.x] = 0; }

// Slot-order sums of the Newton-3 kernel to original atom order (float4), clearing the
// slot-order buffer for the next pass.
__global__ void __launch_bounds__(EWB) k_unsort(const SegDev* __restrict__ segs, Launch L, char* ws,
                                                int outsel) {
    const int blk = blockIdx.x;
    const int p = find_seg(L, blk);
    const SegDev& sg = segs[p];
    const int local = blk - L.pf[p];
    const int b = local / sg.bpb;
    const int i = (local - b * sg.bpb) * EWB + threadIdx.x;
    const int Q = sg.s.Q, S = sg.s.S;
    if (i >= Q) return;
    const int slot = wsp<const int>(ws, sg.o_slotof)[(size_t)b * Q + i];
    float* f = wsp<float>(ws, sg.o_fs) + (size_t)b * 3 * S + slot;
    const float4 v = make_float4(f[0], f[S], f[2 * S], 0.0f);
    f[0] = 0.0f;
    f[S] = 0.0f;
    f[2 * S] = 0.0f;
    size_t o = sg.o_f32;
    if (outsel == 1) o = sg.o_hv32;
    else if (outsel == 2) o = sg.o_f32m;
    wsp<float4>(ws, o)[(size_t)b * Q + i] = v;
}

// Beads bead0 .. bead0 + base.nb[p] - 1 of every path p.
template <int MODE, int PW, int N3, int EL, int WE>
static void launch_pair_t(const SegDev* dsegs, const SegDev* hsegs, const Launch& base, char* ws,
                          int outsel, int energy_bead, int lists, int bead0, bool persistent,
                          hipStream_t st) {
    Launch L = base;
    L.pf[0] = 0;
    L.ntmax = 1;
    for (int p = 0; p < base.nseg; ++p) {
        L.pf[p + 1] = L.pf[p] + (base.nb[p] * hsegs[p].s.cpb + PW - 1) / PW;
        L.ntmax = std::max(L.ntmax, hsegs[p].s.nt);
    }
    const int nblk = L.pf[base.nseg];
    if (nblk == 0) return;
    const size_t tab = TAB_COPIES<MODE> * (size_t)L.ntmax * L.ntmax * sizeof(float4);
    const size_t wlds = (size_t)Fields<MODE, N3>::NF * RING * sizeof(float) + CLIST * sizeof(int);
    if (persistent) {
        // a grid of what the GPU holds at once: a multiple of 8 workgroups (one set per XCD
        // queue), no more workgroups than logical blocks
        const size_t lds = tab + PW * wlds;
        // CU count and resident workgroups per CU, cached per kernel as (lds << 32 | occ)
        static std::atomic<int> ncu_c{0};
        static std::atomic<unsigned long long> occ_c{0};
        int ncu = ncu_c.load(std::memory_order_relaxed);
        if (ncu <= 0) {
            int dev = 0;
            if (hipGetDevice(&dev) != hipSuccess ||
                hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
                ncu <= 0)
                ncu = 256;
            ncu_c.store(ncu, std::memory_order_relaxed);
        }
        unsigned long long oc = occ_c.load(std::memory_order_relaxed);
        int occ = (int)(oc & 0xFFFFFFFFull);
        if (occ <= 0 || (oc >> 32) != lds) {
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_pair_q<MODE, PW, N3, EL, WE>, 64 * PW,
                                                            lds) != hipSuccess ||
                occ <= 0)
                occ = 1;
            occ_c.store(((unsigned long long)lds << 32) | (unsigned)occ, std::memory_order_relaxed);
        }
        const int per = (nblk + 7) / 8;
        const int wg = std::max(1, std::min(per, occ * ncu / 8));
        int* queue = reinterpret_cast<int*>(ws + WS_QUEUE);
        hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(8), 0, st, queue);
        hipLaunchKernelGGL((k_pair_q<MODE, PW, N3, EL, WE>), dim3(8 * wg), dim3(64 * PW), lds, st, dsegs,
                           L, ws, outsel, energy_bead, lists, bead0, queue);
        return;
    }
    hipLaunchKernelGGL((k_pair<MODE, PW, N3, EL, WE>), dim3(8 * ((nblk + 7) / 8)), dim3(64 * PW),
                       tab + PW * wlds, st, dsegs, L, ws, outsel, energy_bead, lists, bead0);
}

// Waves (i-clusters) of a pair launch over every bead of base.
static long long pair_waves(const SegDev* hsegs, const Launch& base) {
    long long n = 0;
    for (int p = 0; p < base.nseg; ++p) n += (long long)base.nb[p] * hsegs[p].s.cpb;
    return n;
}
constexpr long long SPLIT_MIN_WAVES = 16384;  // about 2 rounds of the GPU's resident waves

template <int MODE, int PW, int N3, int EL>
static void launch_pair_e(const SegDev* dsegs, const SegDev* hsegs, const Launch& base, char* ws,
                          int outsel, int energy_bead, int lists, bool pq, hipStream_t st) {
    if constexpr (MODE == 1) {
        launch_pair_t<MODE, PW, N3, EL, 0>(dsegs, hsegs, base, ws, outsel, energy_bead, lists, 0, pq, st);
    } else if (energy_bead == -1) {
        launch_pair_t<MODE, PW, N3, EL, 0>(dsegs, hsegs, base, ws, outsel, energy_bead, lists, 0, pq, st);
    } else if (energy_bead == 0 && EL == 0 && pair_waves(hsegs, base) >= SPLIT_MIN_WAVES) {
        // bead 0 of every path with energies, the other beads without (6 waves per SIMD
        // instead of 5; the Ewald kernels run at 5 either way, so they keep one launch;
        // launches too small to fill the GPU gain nothing from a second launch)
        Launch L0 = base, L1 = base;
        for (int p = 0; p < base.nseg; ++p) {
            L0.nb[p] = std::min(base.nb[p], 1);
            L1.nb[p] = base.nb[p] - L0.nb[p];
        }
        launch_pair_t<MODE, PW, N3, EL, 1>(dsegs, hsegs, L0, ws, outsel, energy_bead, lists, 0, pq, st);
        launch_pair_t<MODE, PW, N3, EL, 0>(dsegs, hsegs, L1, ws, outsel, energy_bead, lists, 1, pq, st);
    } else {
        launch_pair_t<MODE, PW, N3, EL, 1>(dsegs, hsegs, base, ws, outsel, energy_bead, lists, 0, pq, st);
    }
}

template <int MODE, int N3, int EL>
static void launch_pair_w(const SegDev* dsegs, const SegDev* hsegs, const Launch& base, char* ws,
                          int outsel, int energy_bead, int waves, int lists, hipStream_t st) {
    const bool pq = (waves & WAVES_PERSISTENT) != 0;
    switch (waves & ~WAVES_PERSISTENT) {
        case 1: launch_pair_e<MODE, 1, N3, EL>(dsegs, hsegs, base, ws, outsel, energy_bead, lists, pq, st); break;
        case 2: launch_pair_e<MODE, 2, N3, EL>(dsegs, hsegs, base, ws, outsel, energy_bead, lists, pq, st); break;
        case 8: launch_pair_e<MODE, 8, N3, EL>(dsegs, hsegs, base, ws, outsel, energy_bead, lists, pq, st); break;
        default: launch_pair_e<MODE, 4, N3, EL>(dsegs, hsegs, base, ws, outsel, energy_bead, lists, pq, st); break;
    }
}

void run_pair(const SegDev* dsegs, const SegDev* hsegs, const Launch& base, char* ws, int mode,
              int outsel, int energy_bead, int waves, int newton3, hipStream_t st, int lists) {
    if (mode == 1) outsel = 1;
    // Ewald systems: full-shell kernels only (the host rejects Newton-3 plans for them;
    // a launch holds one path then)
    if (hsegs[0].s.elec == 1) {
        if (mode == 0) launch_pair_w<0, 0, 1>(dsegs, hsegs, base, ws, outsel, energy_bead, waves, lists, st);
        else launch_pair_w<1, 0, 1>(dsegs, hsegs, base, ws, outsel, energy_bead, waves, lists, st);
        return;
    }
    if (newton3) {
        if (mode == 0) launch_pair_w<0, 1, 0>(dsegs, hsegs, base, ws, outsel, energy_bead, waves, 0, st);
        else launch_pair_w<1, 1, 0>(dsegs, hsegs, base, ws, outsel, energy_bead, waves, 0, st);
        Launch L = base;
        L.pf[0] = 0;
        for (int p = 0; p < base.nseg; ++p) L.pf[p + 1] = L.pf[p] + base.nb[p] * hsegs[p].bpb;
        if (L.pf[base.nseg] > 0)
            hipLaunchKernelGGL(k_unsort, dim3(L.pf[base.nseg]), dim3(EWB), 0, st, dsegs, L, ws, outsel);
    } else {
        if (mode == 0) launch_pair_w<0, 0, 0>(dsegs, hsegs, base, ws, outsel, energy_bead, waves, lists, st);
        else launch_pair_w<1, 0, 0>(dsegs, hsegs, base, ws, outsel, energy_bead, waves, lists, st);
    }
}

}  // namespace mop
