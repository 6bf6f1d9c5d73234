// Binning of every pair bead of every path of a call into the column/cluster layout.
//
// Per bead: wrap coordinates into 32-bit fixed point, histogram atoms over
// (column, z bin), scan bins inside each column, scan padded column counts, scatter
// atoms into slot order, and fill each column's padding slots.  The counting sort
// replaces the pair search of the physical force routine (do_force, section 2.1).
// Inside a bin atoms are ordered by index (the histogram's atomic ranks only reserve
// places), so the slot order, and with it every pair sum, is the same on every call.
// HBM-bound, O(Q) per bead.
#include "device_common.h"
#include "launch.h"

namespace mop {

// Zero the bin histograms, the slot-order pair sums and (zero_dmax) the per-bead
// max |d|^2 of every segment.
__global__ void __launch_bounds__(EWB) k_zero(const SegDev* __restrict__ segs, Launch L, char* ws,
                                              int zero_dmax) {
    const int blk = blockIdx.x;
    const int p = find_seg(L, blk);
    const SegDev& sg = segs[p];
    const size_t idx = (size_t)(blk - L.pf[p]) * EWB + threadIdx.x;
    const size_t n1 = (size_t)L.nb[p] * sg.s.ncol * sg.s.nzb;
    const size_t n2 = (size_t)L.nb[p] * 3 * sg.s.S;
    if (idx < n1) {
        wsp<int>(ws, sg.o_bincnt)[idx] = 0;
    } else if (idx - n1 < n2) {
        wsp<float>(ws, sg.o_fs)[idx - n1] = 0.0f;
    } else if (zero_dmax && idx - n1 - n2 < (size_t)sg.maxN) {
        wsp<unsigned long long>(ws, sg.o_dmax)[idx - n1 - n2] = 0ull;
    }
}

// Fixed-point coordinates, bin key and rank inside the bin.  fdsign != 0 bins the
// displaced configuration R^b + fdsign * eps_b d^b of the finite-difference term.
__global__ void __launch_bounds__(EWB) k_bin_count(const SegDev* __restrict__ segs, Launch L,
                                                   char* ws, const double* __restrict__ R,
                                                   int fdsign, double fdh) {
    const int blk = blockIdx.x;
    const int p = find_seg(L, blk);
    const SegDev& sg = segs[p];
    const int local = blk - L.pf[p];
    const int b = local / sg.bpb;
    const int i = (local - b * sg.bpb) * EWB + threadIdx.x;
    const int Q = sg.s.Q;
    if (i >= Q) return;
    const double* r = R + sg.roff + ((size_t)b * Q + i) * 3;
    double x = r[0], y = r[1], z = r[2];
    if (fdsign != 0) {
        const double m2 = __longlong_as_double(
            (long long)wsp<unsigned long long>(ws, sg.o_dmax)[b]);
        const double eps = m2 > 0.0 ? fdsign * fdh / sqrt(m2) : 0.0;
        const double* d = wsp<const double>(ws, sg.o_d64) + ((size_t)b * Q + i) * 3;
        x += eps * d[0];
        y += eps * d[1];
        z += eps * d[2];
    }
    const uint32_t ux = to_fixed(x, sg.s.L[0]), uy = to_fixed(y, sg.s.L[1]), uz = to_fixed(z, sg.s.L[2]);
    const int col = fixed_bin(ux, sg.s.ncx) * sg.s.ncy + fixed_bin(uy, sg.s.ncy);
    const int key = col * sg.s.nzb + fixed_bin(uz, sg.s.nzb);
    int* cnt = wsp<int>(ws, sg.o_bincnt) + (size_t)b * sg.s.ncol * sg.s.nzb;
    const int rank = atomicAdd(cnt + key, 1);
    wsp<uint4>(ws, sg.o_atomu)[(size_t)b * Q + i] = make_uint4(ux, uy, uz, (uint32_t)key);
    wsp<int>(ws, sg.o_rank)[(size_t)b * Q + i] = rank;
}

// Exclusive scan of the z bins of each column; column totals.  One wave per column:
// each lane sums a run of consecutive bins, a wave scan places the runs.
__global__ void __launch_bounds__(EWB) k_bin_colscan(const SegDev* __restrict__ segs, Launch L, char* ws) {
    const int blk = blockIdx.x;
    const int p = find_seg(L, blk);
    const SegDev& sg = segs[p];
    const int t = (blk - L.pf[p]) * (EWB / 64) + (threadIdx.x >> 6);  // column of this wave
    const int lane = threadIdx.x & 63;
    const int ncol = sg.s.ncol, nzb = sg.s.nzb;
    if (t >= L.nb[p] * ncol) return;
    const int b = t / ncol, col = t - b * ncol;
    const int* cnt = wsp<const int>(ws, sg.o_bincnt) + ((size_t)b * ncol + col) * nzb;
    int* off = wsp<int>(ws, sg.o_binoff) + ((size_t)b * ncol + col) * (nzb + 1);
    const int per = (nzb + 63) >> 6;
    const int z0 = min(lane * per, nzb), z1 = min(z0 + per, nzb);
    int sum = 0;
    for (int z = z0; z < z1; ++z) sum += cnt[z];
    const int incl = wave_incl_scan(sum);
    int run = incl - sum;
    for (int z = z0; z < z1; ++z) {
        off[z] = run;
        run += cnt[z];
    }
    if (lane == 63) {
        off[nzb] = incl;
        wsp<int>(ws, sg.o_colcnt)[(size_t)b * ncol + col] = incl;
    }
}

// Exclusive scan of the padded (multiple of 8) column counts of one bead per block.
constexpr int CSB = 1024;
__global__ void __launch_bounds__(CSB) k_bin_colstart(const SegDev* __restrict__ segs, Launch L, char* ws) {
    __shared__ int sh[CSB];
    const int blk = blockIdx.x;
    const int p = find_seg(L, blk);
    const SegDev& sg = segs[p];
    const int b = blk - L.pf[p];
    const int ncol = sg.s.ncol;
    const int* cc = wsp<const int>(ws, sg.o_colcnt) + (size_t)b * ncol;
    int* cs = wsp<int>(ws, sg.o_colstart) + (size_t)b * (ncol + 1);
    const int per = (ncol + CSB - 1) / CSB;
    const int c0 = threadIdx.x * per, c1 = min(ncol, c0 + per);
    int sum = 0;
    for (int c = c0; c < c1; ++c) sum += (cc[c] + 7) & ~7;
    sh[threadIdx.x] = sum;
    __syncthreads();
    for (int d = 1; d < CSB; d <<= 1) {
        const int v = threadIdx.x >= d ? sh[threadIdx.x - d] : 0;
        __syncthreads();
        sh[threadIdx.x] += v;
        __syncthreads();
    }
    int run = sh[threadIdx.x] - sum;
    for (int c = c0; c < c1; ++c) {
        cs[c] = run;
        run += (cc[c] + 7) & ~7;
    }
    if (threadIdx.x == CSB - 1) cs[ncol] = sh[CSB - 1];
}

// Atom i's bin: first slot and atom count.
__device__ __forceinline__ void bin_range(const SegDev& sg, char* ws, int b, int key, int& first,
                                          int& count) {
    const int ncol = sg.s.ncol, nzb = sg.s.nzb;
    const int col = key / nzb, zb = key - col * nzb;
    const int* bo = wsp<const int>(ws, sg.o_binoff) + ((size_t)b * ncol + col) * (nzb + 1);
    first = wsp<const int>(ws, sg.o_colstart)[(size_t)b * (ncol + 1) + col] + bo[zb];
    count = bo[zb + 1] - bo[zb];
}

// Reserve places: the atoms of each bin in the order of their atomic ranks.
__global__ void __launch_bounds__(EWB) k_bin_scatter(const SegDev* __restrict__ segs, Launch L, char* ws) {
    const int blk = blockIdx.x;
    const int p = find_seg(L, blk);
    const SegDev& sg = segs[p];
    const int local = blk - L.pf[p];
    const int b = local / sg.bpb;
    const int i = (local - b * sg.bpb) * EWB + threadIdx.x;
    const int Q = sg.s.Q;
    if (i >= Q) return;
    const int key = (int)wsp<const uint4>(ws, sg.o_atomu)[(size_t)b * Q + i].w;
    int first, count;
    bin_range(sg, ws, b, key, first, count);
    wsp<int>(ws, sg.o_tmpo)[(size_t)b * sg.s.S + first + wsp<const int>(ws, sg.o_rank)[(size_t)b * Q + i]] = i;
}

// Place each atom at its bin's first slot plus the number of atoms of the bin with a
// smaller index.
__global__ void __launch_bounds__(EWB) k_bin_place(const SegDev* __restrict__ segs, Launch L, char* ws) {
    const int blk = blockIdx.x;
    const int p = find_seg(L, blk);
    const SegDev& sg = segs[p];
    const int local = blk - L.pf[p];
    const int b = local / sg.bpb;
    const int i = (local - b * sg.bpb) * EWB + threadIdx.x;
    const int Q = sg.s.Q, S = sg.s.S;
    if (i >= Q) return;
    const uint4 u = wsp<const uint4>(ws, sg.o_atomu)[(size_t)b * Q + i];
    int first, count;
    bin_range(sg, ws, b, (int)u.w, first, count);
    const int* tmpo = wsp<const int>(ws, sg.o_tmpo) + (size_t)b * S + first;
    int r = 0;
    for (int k = 0; k < count; ++k) r += tmpo[k] < i;
    const int slot = first + r;
    wsp<uint4>(ws, sg.o_upos)[(size_t)b * S + slot] =
        make_uint4(u.x, u.y, u.z, __float_as_uint(sg.s.qs[i]));
    wsp<int2>(ws, sg.o_umeta)[(size_t)b * S + slot] = make_int2(sg.s.key[i], sg.s.type[i]);
    wsp<int>(ws, sg.o_orig)[(size_t)b * S + slot] = i;
    wsp<int>(ws, sg.o_slotof)[(size_t)b * Q + i] = slot;
}

// Padding slots of each column: position of the column's last atom, DUMMY_KEY.
__global__ void __launch_bounds__(EWB) k_bin_pad(const SegDev* __restrict__ segs, Launch L, char* ws) {
    const int blk = blockIdx.x;
    const int p = find_seg(L, blk);
    const SegDev& sg = segs[p];
    const int t = (blk - L.pf[p]) * EWB + threadIdx.x;
    const int ncol = sg.s.ncol, S = sg.s.S;
    if (t >= L.nb[p] * ncol) return;
    const int b = t / ncol, col = t - b * ncol;
    const int n = wsp<const int>(ws, sg.o_colcnt)[(size_t)b * ncol + col];
    const int pad = (n + 7) & ~7;
    if (pad == n) return;
    const int base = wsp<const int>(ws, sg.o_colstart)[(size_t)b * (ncol + 1) + col];
    uint4* up = wsp<uint4>(ws, sg.o_upos) + (size_t)b * S;
    int2* um = wsp<int2>(ws, sg.o_umeta) + (size_t)b * S;
    int* og = wsp<int>(ws, sg.o_orig) + (size_t)b * S;
    const uint4 last = up[base + n - 1];
    for (int k = n; k < pad; ++k) {
        up[base + k] = last;
        um[base + k] = make_int2(DUMMY_KEY, 0);
        og[base + k] = -1;
    }
}

// Shared-bin finite differences: the displaced coordinates R^b + fdsign eps_b d^b written
// into the slots the binning of R gave each atom (no new sort).
__global__ void __launch_bounds__(EWB) k_bin_displace(const SegDev* __restrict__ segs, Launch L,
                                                      char* ws, const double* __restrict__ R,
                                                      int fdsign, double fdh) {
    const int blk = blockIdx.x;
    const int p = find_seg(L, blk);
    const SegDev& sg = segs[p];
    const int local = blk - L.pf[p];
    const int b = local / sg.bpb;
    const int i = (local - b * sg.bpb) * EWB + threadIdx.x;
    const int Q = sg.s.Q;
    if (i >= Q) return;
    const double* r = R + sg.roff + ((size_t)b * Q + i) * 3;
    const double m2 = __longlong_as_double((long long)wsp<unsigned long long>(ws, sg.o_dmax)[b]);
    const double eps = m2 > 0.0 ? fdsign * fdh / sqrt(m2) : 0.0;
    const double* d = wsp<const double>(ws, sg.o_d64) + ((size_t)b * Q + i) * 3;
    const int slot = wsp<const int>(ws, sg.o_slotof)[(size_t)b * Q + i];
    wsp<uint4>(ws, sg.o_upos)[(size_t)b * sg.s.S + slot] =
        make_uint4(to_fixed(r[0] + eps * d[0], sg.s.L[0]), to_fixed(r[1] + eps * d[1], sg.s.L[1]),
                   to_fixed(r[2] + eps * d[2], sg.s.L[2]), __float_as_uint(sg.s.qs[i]));
}

// Overlap check of a binned configuration: the atom of each slot against every atom whose
// fixed-point coordinates lie within OVERLAP_R of its own along each axis.  Columns and
// z bins are contiguous ranges of fixed-point values, so those atoms sit in the columns
// of u_x -/+ d and u_y -/+ d (at most two each, d being far below a column width) and in
// the z bins from that of u_z - d to that of u_z + d.  A non-excluded pair closer than
// OVERLAP_R (the same FP32 difference of fixed-point coordinates the pair kernels form)
// sets ST_OVERLAP in the status word, which leads the workspace.
__global__ void __launch_bounds__(EWB) k_overlap(const SegDev* __restrict__ segs, Launch L, char* ws) {
    const int blk = blockIdx.x;
    const int p = find_seg(L, blk);
    const SegDev& sg = segs[p];
    const int local = blk - L.pf[p];
    const int S = sg.s.S, ncx = sg.s.ncx, ncy = sg.s.ncy, nzb = sg.s.nzb;
    const int bps = (S + EWB - 1) / EWB;  // blocks per bead (slot order)
    const int b = local / bps;
    const int si = (local - b * bps) * EWB + threadIdx.x;
    if (si >= S) return;
    const uint4* up = wsp<const uint4>(ws, sg.o_upos) + (size_t)b * S;
    const int2* um = wsp<const int2>(ws, sg.o_umeta) + (size_t)b * S;
    const int* cs = wsp<const int>(ws, sg.o_colstart) + (size_t)b * (sg.s.ncol + 1);
    const int* bo = wsp<const int>(ws, sg.o_binoff) + (size_t)b * sg.s.ncol * (nzb + 1);
    const int2 mi = um[si];
    // slots past the last column and padding slots hold no atom
    if (si >= cs[sg.s.ncol] || mi.x == DUMMY_KEY) return;
    const uint4 ui = up[si];
    const int ki = mi.x >> 4;
    const uint32_t* dr = sg.s.ovr;  // OVERLAP_R in fixed-point units per axis, with margin
    const int x0 = fixed_bin(ui.x - dr[0], ncx), x1 = fixed_bin(ui.x + dr[0], ncx);
    const int y0 = fixed_bin(ui.y - dr[1], ncy), y1 = fixed_bin(ui.y + dr[1], ncy);
    const int z0 = fixed_bin(ui.z - dr[2], nzb), z1 = fixed_bin(ui.z + dr[2], nzb);
    const float sx = sg.s.sc[0], sy = sg.s.sc[1], sz = sg.s.sc[2];
    bool hit = false;
    for (int a = 0; a < 2; ++a) {
        const int cx = a ? x1 : x0;
        if (a && x1 == x0) break;
        for (int c = 0; c < 2; ++c) {
            const int cy = c ? y1 : y0;
            if (c && y1 == y0) break;
            const int col = cx * ncy + cy;
            const int base = cs[col];
            const int* o = bo + (size_t)col * (nzb + 1);
            for (int zb = z0;; zb = zb + 1 == nzb ? 0 : zb + 1) {
                for (int sj = base + o[zb]; sj < base + o[zb + 1]; ++sj) {
                    if (sj == si) continue;
                    const uint4 uj = up[sj];
                    const int kj = um[sj].x >> 4;
                    const float dx = (float)(int)(uj.x - ui.x) * sx;
                    const float dy = (float)(int)(uj.y - ui.y) * sy;
                    const float dz = (float)(int)(uj.z - ui.z) * sz;
                    const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                    hit |= (r2 < OVERLAP_R2) & (abs(ki - kj) > 2);
                }
                if (zb == z1) break;
            }
        }
    }
    if (hit) atomicOr(reinterpret_cast<int*>(ws), ST_OVERLAP);
}

void run_displace(const SegDev* dsegs, const SegDev* hsegs, const Launch& base, char* ws,
                  const double* R, int fdsign, double fdh, hipStream_t st) {
    Launch La = base;
    La.pf[0] = 0;
    for (int p = 0; p < base.nseg; ++p) La.pf[p + 1] = La.pf[p] + base.nb[p] * hsegs[p].bpb;
    hipLaunchKernelGGL(k_bin_displace, dim3(La.pf[base.nseg]), dim3(EWB), 0, st, dsegs, La, ws, R,
                       fdsign, fdh);
    Launch Lc = base;
    Lc.pf[0] = 0;
    for (int p = 0; p < base.nseg; ++p)
        Lc.pf[p + 1] = Lc.pf[p] + (base.nb[p] * hsegs[p].s.ncol + EWB - 1) / EWB;
    hipLaunchKernelGGL(k_bin_pad, dim3(Lc.pf[base.nseg]), dim3(EWB), 0, st, dsegs, Lc, ws);
}

void run_binning(const SegDev* dsegs, const SegDev* hsegs, const Launch& base, char* ws,
                 const double* R, int fdsign, double fdh, hipStream_t st) {
    Launch L = base;
    // zero histograms (+ max |d|^2 when not binning a displaced configuration)
    L.pf[0] = 0;
    for (int p = 0; p < base.nseg; ++p) {
        const size_t n = (size_t)base.nb[p] * hsegs[p].s.ncol * hsegs[p].s.nzb +
                         (size_t)base.nb[p] * 3 * hsegs[p].s.S +
                         (fdsign == 0 ? hsegs[p].maxN : 0);
        L.pf[p + 1] = L.pf[p] + (int)((n + EWB - 1) / EWB);
    }
    if (L.pf[base.nseg] > 0) hipLaunchKernelGGL(k_zero, dim3(L.pf[base.nseg]), dim3(EWB), 0, st, dsegs, L, ws,
                                                 fdsign == 0 ? 1 : 0);
    // atoms
    Launch La = base;
    La.pf[0] = 0;
    for (int p = 0; p < base.nseg; ++p) La.pf[p + 1] = La.pf[p] + base.nb[p] * hsegs[p].bpb;
    hipLaunchKernelGGL(k_bin_count, dim3(La.pf[base.nseg]), dim3(EWB), 0, st, dsegs, La, ws, R, fdsign, fdh);
    // columns
    Launch Lc = base;
    Lc.pf[0] = 0;
    for (int p = 0; p < base.nseg; ++p)
        Lc.pf[p + 1] = Lc.pf[p] + (base.nb[p] * hsegs[p].s.ncol + EWB - 1) / EWB;
    Launch Lw = base;  // one wave per column
    Lw.pf[0] = 0;
    for (int p = 0; p < base.nseg; ++p)
        Lw.pf[p + 1] = Lw.pf[p] + (base.nb[p] * hsegs[p].s.ncol + EWB / 64 - 1) / (EWB / 64);
    hipLaunchKernelGGL(k_bin_colscan, dim3(Lw.pf[base.nseg]), dim3(EWB), 0, st, dsegs, Lw, ws);
    Launch Lb = base;
    Lb.pf[0] = 0;
    for (int p = 0; p < base.nseg; ++p) Lb.pf[p + 1] = Lb.pf[p] + base.nb[p];
    hipLaunchKernelGGL(k_bin_colstart, dim3(Lb.pf[base.nseg]), dim3(CSB), 0, st, dsegs, Lb, ws);
    hipLaunchKernelGGL(k_bin_scatter, dim3(La.pf[base.nseg]), dim3(EWB), 0, st, dsegs, La, ws);
    hipLaunchKernelGGL(k_bin_place, dim3(La.pf[base.nseg]), dim3(EWB), 0, st, dsegs, La, ws);
    hipLaunchKernelGGL(k_bin_pad, dim3(Lc.pf[base.nseg]), dim3(EWB), 0, st, dsegs, Lc, ws);
    Launch Ls = base;  // overlap check: one thread per slot
    Ls.pf[0] = 0;
    for (int p = 0; p < base.nseg; ++p)
        Ls.pf[p + 1] = Ls.pf[p] + base.nb[p] * ((hsegs[p].s.S + EWB - 1) / EWB);
    hipLaunchKernelGGL(k_overlap, dim3(Ls.pf[base.nseg]), dim3(EWB), 0, st, dsegs, Ls, ws);
}

}  // namespace mop
