// Pair kernels: the physical force F(R^n) (the do_force work of section 2.1) and the
// exact Hessian-vector product H(R^n) v that replaces the finite-difference term of
// eq. (5), for every pair bead of every path of a call in one launch.
//
// Work unit: one wave per 8-atom i-cluster (8 consecutive slots of one column).
//   1. Lane-parallel over the x-y column stencil: keep columns whose rectangle lies
//      within the search radius of the cluster's bounding box, and per column the
//      cluster range covering the z window [zlo - r, zhi + r] (two ranges when the
//      window wraps around the box).
//   2. Candidate clusters are listed in LDS; 8 of them (64 atoms) are loaded per step,
//      one atom per lane.  Each atom is converted to FP32 coordinates relative to the
//      i-cluster's first atom (exact integer minimum image, then one rounding) and kept
//      when it lies within the cutoff of the i-cluster's bounding box.  Survivors are
//      compacted (ballot + mbcnt) into a per-wave LDS ring.
//   3. Every 64 ring entries, 8 steps of 8 j-atoms x 8 i-atoms (lane = 8*i + j) evaluate
//      the pair terms; each lane accumulates a partial sum for its i atom.
//   4. Partial sums are reduced over the 8 j lanes and written in original atom order.
// Every pair is evaluated from both sides (no Newton-3 scatter): no atomics, and
// results do not depend on scheduling.
//
// Pair terms, d = x_j - x_i, r = |d|, shifted-force LJ + reaction field:
//   g = phi_sf'(r)/r = (a12 r^-6 + a6) r^-8 + qq (2 k_rf - r^-3) + C1 r^-1,
//       C1 = -phi'(r_c) = csf + qq crf1
//   h = (phi'' - phi_sf'/r)/r^2 = (b12 r^-6 + b6) r^-10 + 3 qq r^-5 - C1 r^-3
//   F_i += g d,   (H v)_i += g (v_i - v_j) + h (d . (v_i - v_j)) d
#include "device_common.h"
#include "launch.h"

namespace mop {

template <int MODE, int PW>
__global__ void __launch_bounds__(64 * PW) k_pair(const SegDev* __restrict__ segs, Launch L,
                                                 char* __restrict__ ws, int outsel, int energy_bead) {
    constexpr int TT = MAXTYPES * MAXTYPES;
    constexpr int VR = MODE == 1 ? RING : 1;
    __shared__ float4 s_tab[TT];
    __shared__ float4 s_tab2[TT];
    __shared__ float s_rx[PW][RING], s_ry[PW][RING], s_rz[PW][RING], s_rq[PW][RING];
    __shared__ int s_rk[PW][RING], s_rt[PW][RING];
    __shared__ float s_vx[PW][VR], s_vy[PW][VR], s_vz[PW][VR];
    __shared__ int s_cl[PW][CLIST];

    const int nblk = L.pf[L.nseg];
    const int per = (nblk + 7) >> 3;
    // consecutive logical blocks (neighbouring clusters) stay on one XCD
    const int lblk = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
    if (lblk >= nblk) return;
    const int p = find_seg(L, lblk);
    const SegDev* __restrict__ sg = segs + p;
    const int nt = sg->s.nt;
    for (int t = threadIdx.x; t < nt * nt; t += 64 * PW) {
        s_tab[t] = sg->s.tab[t];
        s_tab2[t] = sg->s.tab2[t];
    }
    __syncthreads();  // the only block barrier: waves are independent from here on

    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int cpb = sg->s.cpb;
    const int gw = (lblk - L.pf[p]) * PW + wave;
    const int b = gw / cpb, c = gw - b * cpb;
    if (b >= L.nb[p]) return;
    const int S = sg->s.S, Q = sg->s.Q, ncol = sg->s.ncol, nzb = sg->s.nzb;
    const int ncx = sg->s.ncx, ncy = sg->s.ncy;
    const uint4* __restrict__ upos = wsp<const uint4>(ws, sg->o_upos) + (size_t)b * S;
    const int2* __restrict__ umeta = wsp<const int2>(ws, sg->o_umeta) + (size_t)b * S;
    const int* __restrict__ colstart = wsp<const int>(ws, sg->o_colstart) + (size_t)b * (ncol + 1);
    const int* __restrict__ binoff = wsp<const int>(ws, sg->o_binoff) + (size_t)b * ncol * (nzb + 1);
    const float4* __restrict__ vs = wsp<const float4>(ws, sg->o_vs) + (size_t)b * S;
    const int nslots = colstart[ncol];
    if (c * CLUSTER >= nslots) return;

    const bool wantE = MODE == 0 && (energy_bead == -2 || energy_bead == b);
    const float sx = sg->s.sc[0], sy = sg->s.sc[1], sz = sg->s.sc[2];
    const float rc2 = sg->s.rc2, rcs = sg->s.rcs, rcs2 = sg->s.rcs2;
    const float krf2 = sg->s.krf2, crf1 = sg->s.crf1;

    // ---- the i-cluster ------------------------------------------------------------
    const int isub = lane >> 3, jslot = lane & 7;
    const int si = c * CLUSTER + isub;
    const uint4 ui = upos[si];
    const int2 mi = umeta[si];
    const uint4 ref = upos[c * CLUSTER];
    const bool vi = mi.x != DUMMY_KEY;
    const float qi = __uint_as_float(ui.w);
    const int keyi2 = mi.x + 2;
    const int tiN = mi.y * nt;
    float vxi = 0.f, vyi = 0.f, vzi = 0.f;
    if (MODE == 1) {
        const float4 v4 = vs[si];
        vxi = v4.x;
        vyi = v4.y;
        vzi = v4.z;
    }
    // bounding box of the cluster in coordinates relative to its first atom, then
    // re-referenced to the box centre uc (fixed point)
    float lox, hix, loy, hiy, loz, hiz;
    auto bbox = [&](float x, float y, float z) {
        lox = vi ? x : 3.0e38f;
        hix = vi ? x : -3.0e38f;
        loy = vi ? y : 3.0e38f;
        hiy = vi ? y : -3.0e38f;
        loz = vi ? z : 3.0e38f;
        hiz = vi ? z : -3.0e38f;
#pragma unroll
        for (int m = 8; m < 64; m <<= 1) {
            lox = fminf(lox, __shfl_xor(lox, m, 64));
            hix = fmaxf(hix, __shfl_xor(hix, m, 64));
            loy = fminf(loy, __shfl_xor(loy, m, 64));
            hiy = fmaxf(hiy, __shfl_xor(hiy, m, 64));
            loz = fminf(loz, __shfl_xor(loz, m, 64));
            hiz = fmaxf(hiz, __shfl_xor(hiz, m, 64));
        }
    };
    bbox((float)(int)(ui.x - ref.x) * sx, (float)(int)(ui.y - ref.y) * sy,
         (float)(int)(ui.z - ref.z) * sz);
    const uint32_t ucx = ref.x + (uint32_t)(long long)rintf(0.5f * (lox + hix) / sx);
    const uint32_t ucy = ref.y + (uint32_t)(long long)rintf(0.5f * (loy + hiy) / sy);
    const uint32_t ucz = ref.z + (uint32_t)(long long)rintf(0.5f * (loz + hiz) / sz);
    const float xi = (float)(int)(ui.x - ucx) * sx;
    const float yi = (float)(int)(ui.y - ucy) * sy;
    const float zi = (float)(int)(ui.z - ucz) * sz;
    bbox(xi, yi, zi);
    // Coordinates relative to the centre give exact pair differences when
    // extent + search radius < L/2 along every axis; otherwise each pair difference is
    // taken from the fixed-point coordinates (small boxes, sparse columns).
    const bool exact = (hix - lox + rcs >= 0.5f * sg->s.Lf[0]) ||
                       (hiy - loy + rcs >= 0.5f * sg->s.Lf[1]) ||
                       (hiz - loz + rcs >= 0.5f * sg->s.Lf[2]);
    const int cx = fixed_bin(ref.x, ncx), cy = fixed_bin(ref.y, ncy);

    // z window of candidate atoms, in z bins
    bool fullz = (hiz - loz + 2.0f * rcs) >= sg->s.Lf[2];
    int zb0 = 0, zb1 = nzb - 1;
    bool zwrap = false;
    if (!fullz) {
        const long long dlo = (long long)floorf((loz - rcs) / sz);
        const long long dhi = (long long)ceilf((hiz + rcs) / sz);
        const uint32_t zlo = ucz + (uint32_t)dlo;
        const uint32_t zhi = ucz + (uint32_t)dhi;
        zb0 = fixed_bin(zlo, nzb);
        zb1 = fixed_bin(zhi, nzb);
        zwrap = zlo > zhi;
        if (zwrap && zb1 + 1 >= zb0) fullz = true;
    }
    // bounding-box centre / half widths for the column test
    const float bcx = 0.5f * (lox + hix), bhx = 0.5f * (hix - lox);
    const float bcy = 0.5f * (loy + hiy), bhy = 0.5f * (hiy - loy);
    const float xref = (float)ucx * sx, yref = (float)ucy * sy;
    const float Lx = sg->s.Lf[0], Ly = sg->s.Lf[1];
    const float cwx = sg->s.cw[0], cwy = sg->s.cw[1];

    float ax = 0.f, ay = 0.f, az = 0.f;
    double eacc = 0.0;
    int wp = 0, rp = 0;  // ring write / read counters (uniform)

    float* rx = s_rx[wave];
    float* ry = s_ry[wave];
    float* rz = s_rz[wave];
    float* rq = s_rq[wave];
    int* rk = s_rk[wave];
    int* rt = s_rt[wave];
    float* rvx = s_vx[wave];
    float* rvy = s_vy[wave];
    float* rvz = s_vz[wave];
    int* clist = s_cl[wave];
    // Ring entries past the valid count are read by the last step of an evaluation and
    // masked by a select on g and h; masked products are still formed (0 * dx, 0 * dv),
    // so every field such an entry can feed must hold a finite value, and the type
    // field a valid table index: clear the ring once.
    for (int e = lane; e < RING; e += 64) {
        rx[e] = 0.0f;
        ry[e] = 0.0f;
        rz[e] = 0.0f;
        rq[e] = 0.0f;
        rk[e] = 0;
        rt[e] = 0;
        if (MODE == 1) {
            rvx[e] = 0.0f;
            rvy[e] = 0.0f;
            rvz[e] = 0.0f;
        }
    }
    wave_sync();
    const float krf = sg->s.krf, crf = sg->s.crf, e0rf = sg->s.e0rf;

    // ---- 8 j-atoms x 8 i-atoms per step from ring entries [base, base + count) ------
    auto eval_t = [&]<bool EX>(int base, int nsteps, int count) {
        for (int s = 0; s < nsteps; ++s) {
            const int idx = s * 8 + jslot;
            const int e = (base + idx) & (RING - 1);
            float dx, dy, dz;
            if (EX) {
                dx = (float)(int)(__float_as_uint(rx[e]) - ui.x) * sx;
                dy = (float)(int)(__float_as_uint(ry[e]) - ui.y) * sy;
                dz = (float)(int)(__float_as_uint(rz[e]) - ui.z) * sz;
            } else {
                dx = rx[e] - xi;
                dy = ry[e] - yi;
                dz = rz[e] - zi;
            }
            const float qj = rq[e];
            const int kj = rk[e], tj = rt[e];
            const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
            const bool in = (idx < count) & vi & (r2 < rc2) & ((unsigned)(keyi2 - kj) > 4u);
            const float r2s = in ? r2 : 1.0f;
            const float rinv = __builtin_amdgcn_rsqf(r2s);
            const float rinv2 = rinv * rinv;
            const float rinv6 = rinv2 * rinv2 * rinv2;
            const float rinv3 = rinv2 * rinv;
            const float4 T = s_tab[tiN + tj];
            const float qq = qi * qj;
            const float C1 = fmaf(qq, crf1, T.z);
            float g = fmaf(T.x, rinv6, T.y) * rinv6 * rinv2;
            g = fmaf(qq, krf2 - rinv3, g);
            g = fmaf(C1, rinv, g);
            g = in ? g : 0.0f;
            if (MODE == 0) {
                ax = fmaf(g, dx, ax);
                ay = fmaf(g, dy, ay);
                az = fmaf(g, dz, az);
                if (wantE) {
                    const float4 T2 = s_tab2[tiN + tj];
                    const float r = r2s * rinv;
                    float en = fmaf(T2.z, rinv6, -T2.w) * rinv6;
                    const float erf = rinv + krf * r2s - crf + e0rf + crf1 * r;
                    en = fmaf(qq, erf, en);
                    en += fmaf(T.z, r, T.w);
                    eacc += in ? (double)en : 0.0;
                }
            } else {
                const float4 T2 = s_tab2[tiN + tj];
                const float rinv4 = rinv2 * rinv2;
                float h = fmaf(T2.x, rinv6, T2.y) * rinv6 * rinv4;
                h = fmaf(3.0f * qq, rinv3 * rinv2, h);
                h = fmaf(-C1, rinv3, h);
                h = in ? h : 0.0f;
                const float dvx = vxi - rvx[e], dvy = vyi - rvy[e], dvz = vzi - rvz[e];
                const float sd = fmaf(dx, dvx, fmaf(dy, dvy, dz * dvz));
                const float hs = h * sd;
                ax = fmaf(g, dvx, fmaf(hs, dx, ax));
                ay = fmaf(g, dvy, fmaf(hs, dy, ay));
                az = fmaf(g, dvz, fmaf(hs, dz, az));
            }
        }
    };

    auto eval = [&](int base, int nsteps, int count) {
        if (exact) eval_t.template operator()<true>(base, nsteps, count);
        else eval_t.template operator()<false>(base, nsteps, count);
    };

    // ---- candidate clusters [0, T) of clist --------------------------------------
    auto process = [&](int T) {
        for (int q = 0; q < T; q += 8) {
            const int ci = q + (lane >> 3);
            bool pass = false;
            float jx = 0.f, jy = 0.f, jz = 0.f, jq = 0.f;
            int jk = 0, jt = 0;
            float4 jv = make_float4(0.f, 0.f, 0.f, 0.f);
            if (ci < T) {
                const int slot = clist[ci] * CLUSTER + (lane & 7);
                const uint4 uj = upos[slot];
                const int2 mj = umeta[slot];
                if (MODE == 1) jv = vs[slot];
                jx = (float)(int)(uj.x - ucx) * sx;
                jy = (float)(int)(uj.y - ucy) * sy;
                jz = (float)(int)(uj.z - ucz) * sz;
                const float ex = fmaxf(fmaxf(lox - jx, jx - hix), 0.0f);
                const float ey = fmaxf(fmaxf(loy - jy, jy - hiy), 0.0f);
                const float ez = fmaxf(fmaxf(loz - jz, jz - hiz), 0.0f);
                pass = (mj.x != DUMMY_KEY) & (fmaf(ex, ex, fmaf(ey, ey, ez * ez)) < rcs2);
                if (exact) {
                    jx = __uint_as_float(uj.x);
                    jy = __uint_as_float(uj.y);
                    jz = __uint_as_float(uj.z);
                }
                jq = __uint_as_float(uj.w);
                jk = mj.x;
                jt = mj.y;
            }
            const unsigned long long m = __ballot(pass);
            const int off = __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                                      __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
            wave_sync();  // previous reads of the ring are done before it is overwritten
            if (pass) {
                const int e = (wp + off) & (RING - 1);
                rx[e] = jx;
                ry[e] = jy;
                rz[e] = jz;
                rq[e] = jq;
                rk[e] = jk;
                rt[e] = jt;
                if (MODE == 1) {
                    rvx[e] = jv.x;
                    rvy[e] = jv.y;
                    rvz[e] = jv.z;
                }
            }
            wp += __popcll(m);
            wave_sync();
            while (wp - rp >= 64) {
                eval(rp, 8, 64);
                rp += 64;
            }
        }
    };

    // ---- column stencil, 64 columns per pass ---------------------------------------
    const int wx = sg->s.wx, wy = sg->s.wy, nst = wx * wy;
    for (int k0 = 0; k0 < nst; k0 += 64) {
        const int k = k0 + lane;
        int a0 = 0, a1 = 0, b0 = 0, b1 = 0;
        if (k < nst) {
            const int ox = k / wy, oy = k - ox * wy;
            int jxc = sg->s.allx ? ox : cx + ox - sg->s.rx;
            int jyc = sg->s.ally ? oy : cy + oy - sg->s.ry;
            jxc = ((jxc % ncx) + ncx) % ncx;
            jyc = ((jyc % ncy) + ncy) % ncy;
            float dxc = ((float)jxc + 0.5f) * cwx - xref;
            dxc -= Lx * rintf(dxc / Lx);
            dxc -= bcx;
            dxc -= Lx * rintf(dxc / Lx);
            float dyc = ((float)jyc + 0.5f) * cwy - yref;
            dyc -= Ly * rintf(dyc / Ly);
            dyc -= bcy;
            dyc -= Ly * rintf(dyc / Ly);
            const float gx = fmaxf(0.0f, fabsf(dxc) - 0.5f * cwx - bhx);
            const float gy = fmaxf(0.0f, fabsf(dyc) - 0.5f * cwy - bhy);
            if (gx * gx + gy * gy < rcs2) {
                const int col = jxc * ncy + jyc;
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
                    if (a1 < a0) a1 = a0;
                    if (b1 < b0) b1 = b0;
                }
            }
        }
        // flatten the per-column cluster ranges into clist, CLIST at a time
        for (;;) {
            const int len = (a1 - a0) + (b1 - b0);
            const int incl = wave_incl_scan(len);
            const int total = __shfl(incl, 63, 64);
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
    {
        const int n = wp - rp;
        if (n > 0) eval(rp, (n + 7) >> 3, n);
    }

    // ---- reduce over the 8 j lanes of each i atom and store ------------------------
#pragma unroll
    for (int m = 1; m < 8; m <<= 1) {
        ax += __shfl_xor(ax, m, 64);
        ay += __shfl_xor(ay, m, 64);
        az += __shfl_xor(az, m, 64);
    }
    if (jslot == 0 && vi) {
        const int oi = wsp<const int>(ws, sg->o_orig)[(size_t)b * S + si];
        size_t o = sg->o_f32;
        if (MODE == 1 || outsel == 1) o = sg->o_hv32;
        else if (outsel == 2) o = sg->o_f32m;
        wsp<float4>(ws, o)[(size_t)b * Q + oi] = make_float4(ax, ay, az, 0.0f);
    }
    if (wantE) {
#pragma unroll
        for (int m = 1; m < 64; m <<= 1) eacc += __shfl_xor(eacc, m, 64);
        if (lane == 0) wsp<double>(ws, sg->o_epart)[(size_t)b * cpb + c] = eacc;
    }
}

template <int MODE, int PW>
static void launch_pair_t(const SegDev* dsegs, const SegDev* hsegs, const Launch& base, char* ws,
                          int outsel, int energy_bead, hipStream_t st) {
    Launch L = base;
    L.pf[0] = 0;
    for (int p = 0; p < base.nseg; ++p)
        L.pf[p + 1] = L.pf[p] + (base.nb[p] * hsegs[p].s.cpb + PW - 1) / PW;
    const int nblk = L.pf[base.nseg];
    if (nblk == 0) return;
    const int grid = ((nblk + 7) / 8) * 8;
    hipLaunchKernelGGL((k_pair<MODE, PW>), dim3(grid), dim3(64 * PW), 0, st, dsegs, L, ws, outsel,
                       energy_bead);
}

void run_pair(const SegDev* dsegs, const SegDev* hsegs, const Launch& base, char* ws, int mode,
              int outsel, int energy_bead, int waves, hipStream_t st) {
    if (mode == 0) {
        switch (waves) {
            case 1: launch_pair_t<0, 1>(dsegs, hsegs, base, ws, outsel, energy_bead, st); break;
            case 2: launch_pair_t<0, 2>(dsegs, hsegs, base, ws, outsel, energy_bead, st); break;
            case 8: launch_pair_t<0, 8>(dsegs, hsegs, base, ws, outsel, energy_bead, st); break;
            default: launch_pair_t<0, 4>(dsegs, hsegs, base, ws, outsel, energy_bead, st); break;
        }
    } else {
        switch (waves) {
            case 1: launch_pair_t<1, 1>(dsegs, hsegs, base, ws, outsel, energy_bead, st); break;
            case 2: launch_pair_t<1, 2>(dsegs, hsegs, base, ws, outsel, energy_bead, st); break;
            case 8: launch_pair_t<1, 8>(dsegs, hsegs, base, ws, outsel, energy_bead, st); break;
            default: launch_pair_t<1, 4>(dsegs, hsegs, base, ws, outsel, energy_bead, st); break;
        }
    }
}

}  // namespace mop
