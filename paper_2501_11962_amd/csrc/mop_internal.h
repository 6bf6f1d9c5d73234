// Internal layout shared by the host runtime (mop_api.cpp) and the HIP kernels.
//
// Data layout in HBM, per bead with pair work (a "pair bead"):
//   atoms are binned into nc_x * nc_y columns of the x-y plane (column width about
//   0.5 nm) and, inside each column, counting-sorted by z bin.  Each column's slot
//   range is padded to a multiple of 8 so that it splits into 8-atom clusters; padding
//   slots carry DUMMY_KEY.  Sorted arrays (structure of arrays, one entry per slot):
//     upos  uint4  {x, y, z fixed point (box = 2^32 units), charge bits (float)}
//     umeta int2   {16 * exclusion key + LJ type, LJ type}
//     orig  int    atom index of the slot (-1 for padding)
//     vs    float4 the vector of a Hessian-vector product, slot order
//     fs    float  x3 pair sums in slot order (structure of arrays), Newton-3 kernels
//   Per atom (original order): slotof, pair force / pair HVP outputs (float4).
//   Per cluster: the neighbour list a force pass records for the Hessian pass of the
//     same bead (nl: int [lcap] records, one per candidate cluster with atoms that passed
//     the search, in search order: cluster index << 8 | 8-bit mask of those atoms; nlc:
//     their count, which may exceed lcap, then the list is incomplete).
// Per path: FP64 residuals d^n [(N-1)][Q][3], reduction partials, per-bead max |d|^2.
// Particle-mesh Ewald (systems with Ewald electrostatics), per pair bead:
//     ptc   int [ntile]    atoms per grid tile; pts int [ntile + 1] their starts
//     ptid, ptrk int [Q]   tile and rank of each atom
//     ptb   int4 [Q]       in tile order: base grid point (x, y, z) and atom index
//     ptw   double4 [Q]    in tile order: fractional offsets (x, y, z) and charge
//     pgr   double [K]     real grid (FFT input; also the output of displaced and
//                          Hessian passes)
//     pgc   double2 [Kc]   half spectrum (Kc = Kx Ky (Kz/2 + 1))
//     pphi  double [K]     grid potential of the force pass, kept for the Hessian pass
//     pep   double [nsb]   energy partials of the solve kernel
//     frec, hrec double [Q][3]  reciprocal forces / Hessian-vector products (original
//                          order), added by the FP64 path kernels
//   plus one FFT work buffer.
#pragma once

#include <hip/hip_runtime.h>

#include <climits>
#include <cstddef>
#include <cstdint>

namespace mop {

constexpr int MAXSEG = 32;        // paths per launch
constexpr int CLUSTER = 8;        // atoms per cluster
constexpr int RING = 128;         // j-atom ring per wave (power of two, >= 2*64)
constexpr int CLIST = 256;        // candidate-cluster list per wave
constexpr int MAXTYPES = 16;      // LJ types (the type fills the low 4 bits of a packed key)
constexpr int EWB = 256;          // block size of the elementwise kernels
constexpr int WAVES_PERSISTENT = 0x100;  // or-ed into a plan's waves: persistent pair launches
constexpr size_t WS_QUEUE = 64;   // workspace byte offset of the 8 work-queue counters
constexpr int32_t DUMMY_KEY = INT32_MIN;

// Status bits (mirrors MOP_DEV_* of the public header).
constexpr int ST_NONFINITE = 1;
constexpr int ST_CAPACITY = 2;
constexpr int ST_OVERLAP = 4;    // a binned configuration has a non-excluded pair closer than OVERLAP_R
constexpr double OVERLAP_R = 0.01;     // nm
constexpr float OVERLAP_R2 = 1.0e-4f;  // (0.01 nm)^2

constexpr int PME_BLOCK = 256;    // block size of the grid kernels
constexpr int PME_TILE = 8;       // nominal grid tile edge of the spreading kernel

struct SysDev {
    int Q, ncx, ncy, ncol, nzb, nt;
    int S;            // slots per bead (multiple of 8)
    int cpb;          // clusters per bead (S / 8)
    int lcap;         // neighbour-list records per cluster (0: no lists)
    int allx, ally;   // 1: the column stencil spans every column along that axis
    int rx, ry;       // stencil half widths (columns) when not spanning
    int wx, wy;       // stencil widths (columns)
    int nbond_entries;
    double L[3];
    float sc[3];      // nm per fixed-point unit: L / 2^32
    float Lf[3];
    float cw[2];      // column widths (nm)
    uint32_t ovr[3];  // OVERLAP_R in fixed-point units per axis, rounded up, plus one
    float rc2;        // cutoff^2
    float rcs;        // neighbour-search radius (cutoff + margin)
    float rcs2;
    float krf2;       // 2 k_rf
    float krf, crf;   // reaction-field constants (energy)
    float crf1;       // 1/rc^2 - 2 k_rf rc: -phi_RF'(rc) / (q_i q_j)
    float e0rf;       // -rc * crf1
    const float* qs;      // [Q] charge * sqrt(f / eps_r)
    const int* key;       // [Q] 16 * exclusion key + LJ type; excluded pairs: |key_i - key_j| <= 2
    const int* type;      // [Q]
    const double* c;      // [Q] dt / (m nu)
    const double* K;      // [Q] m nu / (2 dt)
    const double* minv;   // [Q] 1 / m (path dynamics)
    const int* bstart;    // [Q + 1] bond CSR (each bond listed for both atoms)
    const int* bpart;     // partner atom
    const double* br0;
    const double* bk;
    const float4* tab;    // [nt*nt] {a12 = -12 c12, a6 = 6 c6, csf = -phi_LJ'(rc), e0lj}
    const float4* tab2;   // [nt*nt] {b12 = 168 c12, b6 = -48 c6, c12, c6}
    const float4* tabh;   // [nt*nt] {a12, a6, csf, 0.75 a12}: the Hessian kernel's table
                          // (b12 = -14 a12 and b6 = -8 a6 follow from a12, a6)
    // electrostatics: 0 reaction field; 1 Ewald real space + particle-mesh reciprocal
    // part.  With Ewald, crf1 = -psi'(r_c) and e0rf = -psi(r_c) - r_c crf1 for
    // psi = erfc(beta r)/r, and krf = krf2 = crf = 0.
    int elec;
    float ew_beta;        // beta
    float ew_c2b;         // 2 beta / sqrt(pi)
    float ew_b2x2;        // 2 beta^2
    int pme_p;            // B-spline order
    int Kg[3];            // grid points per axis
    int Kzh;              // Kz/2 + 1
    int nsb;              // solve-kernel blocks per bead
    double kl[3];         // K_a / L_a
    double qscale;        // fixed-point scale of the charge grid (power of two)
    double vbound;        // sum |q| * 3 * max K_a/L_a (bound of the dipole grid per unit |v|)
    double e_const;       // self + neutralising-background energy
    const double* qd;     // [Q] charges (e)
    const double* phihat; // [Kx Ky Kzh] f B(m) C(m), half spectrum
    // grid tiles of the spreading kernel: ntl[a] tiles per axis with edges
    // tile_lo[tlo_off[a] + t] (balanced, each at least PME_TILE points unless the axis is
    // shorter), tile_of[tof_off[a] + k] the tile of grid index k; tile_pts = largest tile
    int ntl[3], ntile, tile_pts;
    int tlo_off[3], tof_off[3];
    const int* tile_lo;
    const int* tile_of;
};

// One path (segment) of a launch.  Byte offsets are relative to the workspace base.
struct SegDev {
    SysDev s;
    int maxb;             // pair-bead capacity of the layout
    int maxN;             // bead capacity of the path arrays
    long long roff;       // element offset of this path's bead 0 in R / G / V / F
    int vidx;             // index of this path's scalar outputs
    int bpb;              // elementwise blocks per bead: ceil(Q / EWB)
    size_t o_upos, o_umeta, o_orig, o_slotof, o_atomu, o_rank, o_bincnt, o_binoff,
        o_colcnt, o_colstart, o_vs, o_fs, o_f32, o_f32m, o_hv32, o_epart, o_d64, o_rpart,
        o_dmax, o_eres, o_nl, o_nlc, o_tmpo, o_ptc, o_pts, o_ptid, o_ptrk, o_ptb, o_ptw, o_pgr, o_pgc,
        o_pphi, o_pep, o_pfw, o_frec, o_hrec;
};

// Per-launch description, passed by value.
struct Launch {
    int nseg;
    int ntmax;            // largest LJ type count of the launch (pair kernels)
    int pf[MAXSEG + 1];   // block prefix per segment
    int N[MAXSEG];        // beads of each path in this call
    int nb[MAXSEG];       // pair beads of each path in this call
};

// Coefficients of one step of the path integrator.
struct PmdCoef {
    double tau;           // time step (ps)
    double c1;            // exp(-gamma tau)
    double c2;            // sqrt((1 - c1^2) kT); 0 without thermostat
    uint64_t seed;        // key of the normal deviates
};

// Metadynamics bias on the end-to-end variable (device state of one mop_bias).
struct BiasDev {
    const int* A;         // [nA] atoms of group A
    const int* B;         // [nB] atoms of group B
    int nA, nB;
    const double* minv;   // [Q] 1 / m of the system
    double L[3];
    double sigma;         // Gaussian width in S (nm)
    double height;        // initial height (kJ/mol)
    double bias_factor;   // > 1: well-tempered; 0: standard
    double kT;
    double* centers;      // [capacity]
    double* heights;      // [capacity]
    int* count;           // deposited Gaussians
    int capacity;
};

// Pointers of one call (device).
struct CallPtrs {
    const double* R;      // bead coordinates, packed paths
    const double* V;      // HVP input (bead_hvp) or null
    double* G;            // gradient out
    float* Fout;          // bead_forces / bead_hvp out (float)
    double* Uout;         // bead_forces energies / scalar outputs
    double* veff;         // [P] or null
    double* u1;
    double* espring;
    char* ws;
    int* status;
    double fd_h;
};

}  // namespace mop
