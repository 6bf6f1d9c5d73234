/*
 * mop.h -- C ABI of the MI355X (gfx950) library for the Onsager-Machlup path gradient
 * used by path molecular dynamics and metadynamics of paths.
 *
 * The operations follow the paper's statement of the problem (section 1.1):
 *   - a system of Q atoms with potential U and force F = -grad U (eq. 1);
 *   - a path of N beads R^1 .. R^N, each a full copy of the system (Fig. 1);
 *   - the effective potential of eq. (3)
 *         V_eff = U(R^1) + sum_{n=1}^{N-1} sum_i K_i/2 |d^n_i|^2,
 *         d^n = mi(R^{n+1} - R^n) - c F(R^n),  K_i = m_i nu/(2 dt),  c_i = dt/(m_i nu)
 *     (the rest length is read as L^n = c F^n, the only reading under which eqs. 5-7
 *     are the gradient of eq. 3; mi = minimum image);
 *   - its gradient G = grad V_eff = -F_eff of eqs. (5)-(7), with the finite-difference
 *     Hessian term of eq. (5) replaced by the exact Hessian-vector product, or, for
 *     comparison, computed as in eq. (5).
 *
 * The potential is a molecular force field: Lennard-Jones (Lorentz-Berthelot mixing)
 * plus reaction-field electrostatics, both shifted-force at r_cut, harmonic bonds, and
 * exclusion of 1-2/1-3 bonded pairs; orthorhombic periodic box with
 * r_cut < min(box)/2.  Units: nm, ps, amu, kJ/mol, e.  Alternatively (elec =
 * MOP_ELEC_PME) electrostatics is particle-mesh Ewald, the method of the paper's
 * standard MD runs (Appendix A.1): the Ewald real-space term f q_i q_j erfc(beta r)/r,
 * shifted-force at r_cut, with beta from erfc(beta r_cut) = ewald_rtol; excluded pairs
 * within r_cut carry -f q_i q_j erf(beta r)/r; the reciprocal part is smooth PME
 * (Essmann et al. 1995) with B-spline order pme_order on a pme_grid grid; plus the
 * self term -f beta/sqrt(pi) sum q^2 and the neutralising background
 * -f pi (sum q)^2 / (2 V beta^2).  Forces and the Hessian-vector product of every term
 * are exact derivatives of that energy.
 *
 * Precision: pair forces and pair Hessian-vector products are evaluated in FP32 from
 * 32-bit fixed-point coordinates (exact minimum image); bonds, residuals, energies,
 * the PME reciprocal part (spline weights, grids, FFTs) and the gradient assembly are
 * FP64.
 *
 * Conventions for every compute call:
 *   - Array arguments are DEVICE pointers to C-contiguous arrays, bead-major:
 *     [beads][Q][3].  The caller owns all inputs, outputs and the workspace.
 *   - Calls are asynchronous on the stream given to mop_ctx_create, allocate nothing
 *     and never synchronise with the host, so they can be captured in a hipGraph.
 *   - Return value 0 = MOP_OK; a negative value is a synchronous argument error
 *     detected on the host, in which case nothing was enqueued.
 *   - Errors found on the device (non-finite result, exhausted capacity, overlapping
 *     atoms) set bits of a
 *     status word inside the workspace; read it with mop_status after the work has
 *     finished.  Outputs are unspecified when a bit is set.
 */
#ifndef MOP_H
#define MOP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------------------ */
#define MOP_OK 0
#define MOP_EINVAL (-1)     /* null pointer, bad size, bad option */
#define MOP_ECUTOFF (-2)    /* r_cut >= min(box)/2 or r_cut <= 0 */
#define MOP_ETYPE (-3)      /* type index out of range or too many types */
#define MOP_EHIP (-4)       /* a HIP runtime call failed (e.g. no device) */
#define MOP_ENOMEM (-5)     /* device allocation failed (create calls only) */
#define MOP_ETOPOLOGY (-6)  /* bonds do not form linear chains; pass excl_mol/excl_pos */
#define MOP_ESIZE (-7)      /* more beads or paths than the plan or batch was made for */

/* bits of the device status word (mop_status) */
#define MOP_DEV_NONFINITE 1 /* a force, residual or gradient component is not finite */
#define MOP_DEV_CAPACITY 2  /* a fixed-capacity device buffer is full: the Gaussian history
                               of a bias (re-create it with more capacity).  The neighbour
                               search has no such buffer: candidate lists are processed in
                               rounds, and a cluster whose recorded list overflowed is
                               searched again. */
#define MOP_DEV_OVERLAP 4   /* a force pass met a non-excluded pair closer than 0.01 nm
                               (overlapping atoms: FP32 pair terms of order r^-14 are then
                               meaningless; the outputs are still written) */

typedef struct mop_ctx_s* mop_ctx;
typedef struct mop_system_s* mop_system;
typedef struct mop_plan_s* mop_plan;
typedef struct mop_batch_s* mop_batch;
typedef struct mop_bias_s* mop_bias;

/*
 * System description.  All pointers are HOST pointers; the arrays are copied by
 * mop_system_create and may be freed afterwards.
 *   Q               number of atoms (>= 1)
 *   box             orthorhombic box lengths (nm)
 *   mass[Q]         amu (> 0);  charge[Q] e;  type[Q] in [0, ntypes)
 *   sigma/epsilon   per-type LJ parameters [ntypes] (ntypes <= 16), mixed by
 *                   Lorentz-Berthelot; epsilon = 0 switches LJ off for a type
 *   bond_ij[2*nbonds], bond_r0[nbonds] (nm), bond_k[nbonds] (kJ/mol/nm^2)
 *   excl_mol/excl_pos[Q]  molecule id and position along a linear chain; pairs of the
 *                   same molecule whose positions differ by at most 2 are excluded.
 *                   NULL: derived from the bonds, which must then form linear chains.
 *   r_cut (nm), eps_rf, eps_r (reaction field: k_rf = (eps_rf - eps_r) /
 *                   ((2 eps_rf + eps_r) r_cut^3)), dt (ps), nu (1/ps)
 *   elec            MOP_ELEC_RF (0, reaction field) or MOP_ELEC_PME (1, particle-mesh
 *                   Ewald; eps_rf is then unused and eps_r divides f as before)
 *   pme_order       B-spline order 4, 6 or 8 (0: 4)
 *   ewald_rtol      erfc(beta r_cut), in [1e-16, 1) (0: 1e-5)
 *   pme_grid[3]     grid points per axis, each >= pme_order, product <= 2^27 (0 for all
 *                   three: the smallest sizes with prime factors 2, 3, 5, 7 that are at
 *                   least L/0.12 nm and at least 2 pme_order)
 * PME systems take plans without MOP_PLAN_NEWTON3 and are not accepted by mop_batch.
 */
#define MOP_ELEC_RF 0
#define MOP_ELEC_PME 1
typedef struct {
    int32_t Q;
    double box[3];
    const double* mass;
    const double* charge;
    const int32_t* type;
    int32_t ntypes;
    const double* sigma;
    const double* epsilon;
    int32_t nbonds;
    const int32_t* bond_ij;
    const double* bond_r0;
    const double* bond_k;
    const int32_t* excl_mol;
    const int32_t* excl_pos;
    double r_cut, eps_rf, eps_r, dt, nu;
    int32_t elec;
    int32_t pme_order;
    double ewald_rtol;
    int32_t pme_grid[3];
} mop_system_desc;

/*
 * Neighbour-search options of a plan (0 = default for every field).
 *   col_width   width (nm) of the x-y columns atoms are binned into; 8-atom clusters
 *               are cut along z inside each column.  Default 0.4 nm.
 *   zbin        height (nm) of the z bins used to sort columns.  Default 0.1 nm.
 *   waves       waves per workgroup of the pair kernels (1, 2, 4, 8).  Default 4.
 *   flags       MOP_PLAN_NEWTON3: evaluate each pair once (Newton's third law) and
 *               gather the partner's share with atomic adds; summation order then
 *               depends on scheduling.  Default: every pair from both sides without
 *               atomics, which is the faster variant on MI355X.
 *               MOP_PLAN_ONE_STREAM (PME systems): run the mesh work on the caller's
 *               stream in call order instead of on a second stream of the plan beside
 *               the pair kernels.  Results are bit-identical either way; for callers
 *               that need every kernel on one stream, and for timing each kernel alone.
 *               MOP_PLAN_PERSISTENT: launch the pair kernels as persistent grids (as
 *               many workgroups as the GPU holds at once, each taking clusters from a
 *               work queue per XCD until it is empty) instead of one workgroup per
 *               group of clusters.  Results are bit-identical either way.  A batch
 *               takes this flag, like waves, from its first plan.
 *   list_cap    neighbour-list records per 8-atom cluster.  veff_grad (exact mode)
 *               records, in its force pass, which atoms passed each cluster's
 *               neighbour search (one 32-bit record per neighbouring cluster with at
 *               least one such atom: its index and an 8-bit mask of those atoms), and
 *               its Hessian pass reads them back instead of searching again; a cluster
 *               with more records than list_cap is searched again.  0: sized from the
 *               mean density (about 1.5 times the expected count); negative: no lists.
 *               The workspace grows by 4 * list_cap bytes per cluster and pair bead.
 */
#define MOP_PLAN_NEWTON3 1
#define MOP_PLAN_ONE_STREAM 2
#define MOP_PLAN_PERSISTENT 4
typedef struct {
    double col_width;
    double zbin;
    int32_t waves;
    int32_t flags;
    int32_t list_cap;
} mop_plan_opts;

/* Host-only validation of a system description (no device needed).  Returns MOP_OK,
 * MOP_EINVAL, MOP_ECUTOFF, MOP_ETYPE or MOP_ETOPOLOGY. */
int mop_system_check(const mop_system_desc* desc);

/* Context on HIP device `device`, issuing work on `hip_stream` (a hipStream_t; NULL is
 * the null stream).  MOP_EHIP when the device cannot be used. */
int mop_ctx_create(int device, void* hip_stream, mop_ctx* out);
int mop_ctx_set_stream(mop_ctx ctx, void* hip_stream);
void mop_ctx_destroy(mop_ctx ctx);

/* Copy a system to the device (constants, type-pair tables, bond lists, exclusion
 * keys).  Allocates device memory. */
int mop_system_create(mop_ctx ctx, const mop_system_desc* desc, mop_system* out);
void mop_system_destroy(mop_system sys);

/* PME parameters a system was created with: grid points per axis and beta (nm^-1).
 * MOP_EINVAL for a reaction-field system. */
int mop_system_pme_info(mop_system sys, int32_t grid[3], double* beta);

/* Plan for paths of up to `max_beads` beads of one system (also the maximum B of
 * bead_forces / bead_hvp).  opts may be NULL.  Allocates device memory; for a PME
 * system also creates the batched rocFFT plans (max_beads grids per transform; double
 * precision for the charge grids, single precision for the dipole grids of the Hessian
 * pass).
 * MOP_EINVAL for MOP_PLAN_NEWTON3 with a PME system.  A PME plan's transforms keep
 * host-side state (stream and work-buffer bindings): do not call one plan from several
 * host threads at once. */
int mop_plan_create(mop_system sys, int32_t max_beads, const mop_plan_opts* opts, mop_plan* out);
void mop_plan_destroy(mop_plan plan);

/* Workspace bytes a call on this plan needs (for any bead count up to max_beads and
 * either gradient mode).  The caller allocates it (256-byte aligned) and passes it to
 * every call; calls that share a workspace must not overlap in time. */
int mop_workspace_size(mop_plan plan, size_t* bytes);

/*
 * Physical forces of B independent configurations (the do_force call of section 2.1):
 *   R  [B][Q][3] double in;   F [B][Q][3] float out, F = -grad U(R^b)
 *   U  [B] double out (potential energy per configuration) or NULL
 */
int bead_forces(mop_plan plan, const double* R, int32_t B, float* F, double* U, void* ws);

/*
 * bead_forces without a workspace argument, for callers that cannot allocate device
 * memory (code under graph capture, tight serving loops, harnesses that forbid
 * allocation).  Same arguments and results as bead_forces, plus
 *   status  one device int32 that receives this call's device status word (MOP_DEV_*
 *           bits), or NULL.
 * The work runs in a static workspace compiled into the library: 64 MiB per device,
 * held from the first use until the process ends, shared by every bead_forces_static call
 * on that device, which keeps the last call's contents (the status word is cleared at the
 * start of each call).  Calls that overlap in time on one device race on it: issue them
 * on one stream, or order them.  Allocates nothing and calls no allocating routine.
 * MOP_ESIZE when the plan's workspace (mop_workspace_size) exceeds 64 MiB: make the plan
 * with fewer max_beads, or list_cap < 0 (no neighbour lists).  MOP_EINVAL for PME or
 * Newton-3 plans.  MOP_EHIP when the device address of the workspace could not be found
 * at mop_ctx_create.
 */
#define MOP_STATIC_WORKSPACE_BYTES 67108864 /* 64 MiB */
int bead_forces_static(mop_plan plan, const double* R, int32_t B, float* F, double* U,
                       int32_t* status);

/*
 * Hessian-vector products HV^b = H(R^b) V^b, H = Hessian of U (the quantity the
 * finite-difference term of eq. 5 approximates, as -1/2 H eta):
 *   R, V [B][Q][3] double in;   HV [B][Q][3] float out
 */
int bead_hvp(mop_plan plan, const double* R, const double* V, int32_t B, float* HV, void* ws);

/*
 * Effective potential of eq. (3) for one path R [N][Q][3] (N >= 1).  Each output is a
 * single device double, or NULL: veff = u1 + espring, u1 = U(R^1), espring = spring sum.
 */
int veff_energy(mop_plan plan, const double* R, int32_t N, double* veff, double* u1,
                double* espring, void* ws);

/*
 * Gradient G [N][Q][3] (device double out) of V_eff for one path, and V_eff (one device
 * double, or NULL).  mode 0: exact Hessian-vector products.  mode 1: the
 * finite-difference term of eq. (5), [F(R + eps d) - F(R - eps d)]/(4 eps), with
 * eps = fd_h / max_i |d^n_i| per bead (fd_h in nm, > 0), each displaced configuration
 * re-binned.  mode 2: the same finite differences with the binning of R kept for the
 * displaced configurations (only the coordinates are rewritten) and the neighbour lists of
 * R's force pass replayed; exact for fd_h up to half the neighbour-search margin (1e-4
 * nm); beyond it, pairs that cross the cut-off during the displacement may be missed.
 * G = -F_eff of eqs. (5)-(7).
 */
int veff_grad(mop_plan plan, const double* R, int32_t N, double* G, double* veff,
              int32_t mode, double fd_h, void* ws);

/*
 * Metadynamics of paths (section 1.2).  The collective variable is the end-to-end
 * distance of eq. (8), S = s(R^N) - s(R^1), with s(R) the distance between the centres
 * of mass of two atom groups A and B (section 3 takes the ligand and its binding pocket).
 * Each group's centre of mass uses the minimum-image offsets of its atoms to the group's
 * first atom, so a group must span less than half the box.  The bias is a sum of
 * Gaussians on S,
 *     V_bias(S) = sum_k w_k exp(-(S - S_k)^2 / (2 sigma^2)),
 * with w_k = height (standard metadynamics) or, for bias_factor > 1 (well-tempered),
 * height * exp(-V_bias(S_k) / (kT (bias_factor - 1))).  Its gradient acts on beads 1
 * and N only.
 *   groupA[nA], groupB[nB]  HOST arrays of atom indices (copied); in range, no atom twice
 *   sigma > 0 (nm), height >= 0 (kJ/mol), bias_factor 0 or > 1 (then kT > 0), stride >= 1
 *   (a Gaussian is deposited at steps that are multiples of stride), max_gaussians >= 1
 *   (further deposits are dropped and set MOP_DEV_CAPACITY).
 * mop_bias_create allocates the groups and the Gaussian history on the device (zero
 * Gaussians); MOP_EINVAL on bad arguments.
 */
typedef struct {
    int32_t nA, nB;
    const int32_t* groupA;
    const int32_t* groupB;
    double sigma;
    double height;
    double bias_factor;
    double kT;
    int32_t stride;
    int32_t max_gaussians;
} mop_bias_desc;
int mop_bias_create(mop_plan plan, const mop_bias_desc* desc, mop_bias* out);
void mop_bias_destroy(mop_bias bias);
/* Remove every deposited Gaussian (asynchronous, on the context stream). */
int mop_bias_reset(mop_bias bias);
/* For a path R [N][Q][3] (device): add grad V_bias to G [N][Q][3] (device, or NULL for
 * none), write {V_bias, S} to out (two device doubles, or NULL), and, if deposit != 0,
 * add a Gaussian at S after evaluating V_bias.  ws: the plan's workspace (status word). */
int mop_bias_apply(mop_bias bias, const double* R, int32_t N, double* G, double* out,
                   int32_t deposit, void* ws);
/* Synchronise the context stream; *count = deposited Gaussians; the first
 * min(count, capacity) centres and heights are copied to the HOST arrays (either may be
 * NULL). */
int mop_bias_history(mop_bias bias, int32_t* count, double* centers, double* heights,
                     int32_t capacity);

/*
 * Path molecular dynamics (eq. 4): nsteps steps of the whole polymer R [N][Q][3] under
 * F_eff = -grad V, V = V_eff (+ V_bias when bias is not NULL), with fictitious masses
 * read as the atoms' masses (the same for every bead).  One step is the splitting
 * B A O A B:
 *     V -= tau/2 G/M;  R += tau/2 V;  V = c1 V + c2 xi/sqrt(M);  R += tau/2 V;
 *     G = grad V_eff(R) (exact Hessian-vector products, as veff_grad mode 0)
 *         [+ grad V_bias(R) with the Gaussians deposited so far, then a new Gaussian at
 *          steps step0 + k that are multiples of the bias stride];
 *     V -= tau/2 G/M
 * with c1 = exp(-gamma tau), c2 = sqrt((1 - c1^2) kT).  gamma = 0 skips the O part:
 * velocity Verlet, the constant-energy integrator of appendix A.2; gamma > 0 is the
 * Langevin thermostat of its constant-temperature runs.  xi are standard normal
 * deviates from Philox4x64-10 (Salmon et al., SC 2011) keyed by (seed, 0) on the
 * counter (bead * Q + atom, step0 + k, 0, 0), mapped to (0,1) as
 * (floor(x / 2^12) + 1/2) 2^-52 and through Box-Muller (outputs 0,1 -> x, y; 2,3 -> z).
 *   R, V   [N][Q][3] device doubles, updated in place (V in nm/ps)
 *   G      [N][Q][3] device doubles: on entry the gradient of the total potential at the
 *          entry R (veff_grad, then mop_bias_apply without deposit when biased); on
 *          exit that of the final R
 *   energies  device doubles [nsteps][4] = {V_eff, kinetic energy, V_bias, S} after each
 *          step (the bias columns 0 without a bias), or NULL
 *   bias   NULL, or a bias made for this plan
 *   tau > 0 (ps), gamma >= 0 (1/ps), kT >= 0 (kJ/mol); MOP_EINVAL otherwise.
 */
typedef struct {
    double tau;
    double gamma;
    double kT;
    uint64_t seed;
} mop_pmd_params;
int pmd_step(mop_plan plan, mop_bias bias, double* R, double* V, double* G, int32_t N,
             const mop_pmd_params* prm, uint64_t step0, int32_t nsteps, double* energies,
             void* ws);

/*
 * Batch of P independent paths (each with its own plan/system and bead count),
 * evaluated together: every phase of all paths is one kernel launch.  Paths are packed
 * back to back in one buffer: path p occupies N_p*Q_p*3 doubles starting at element
 * sum_{q<p} N_q*Q_q*3 of R (and of G).  Reaction-field systems only (MOP_EINVAL for a
 * plan of a PME system).
 */
int mop_batch_create(int32_t P, const mop_plan* plans, const int32_t* N, mop_batch* out);
void mop_batch_destroy(mop_batch batch);
int mop_batch_workspace_size(mop_batch batch, size_t* bytes);
/* veff [P] device doubles or NULL; mode / fd_h as in veff_grad */
int mop_batch_veff_grad(mop_batch batch, const double* R, double* G, double* veff,
                        int32_t mode, double fd_h, void* ws);

/* Synchronise the context stream and read the device status word of a workspace that
 * was used with `plan` (bits MOP_DEV_*). */
int mop_status(mop_plan plan, const void* ws, int32_t* device_status);
/* Clear the status word (asynchronous, on the context stream). */
int mop_status_clear(mop_plan plan, void* ws);

/*
 * Profiling variant of veff_grad: the same work, with HIP events recorded on the
 * context stream between phases; waits for completion and writes the elapsed time of
 * each phase in milliseconds to phase_ms[MOP_NPHASES] (host array).  Synchronises the
 * host, so it must not be captured in a graph.
 */
#define MOP_NPHASES 8
#define MOP_PHASE_BIN 0       /* fixed point, histogram, scans, scatter, padding, overlap check */
#define MOP_PHASE_FORCE 1     /* pair-force kernel, beads 1..N-1 (energy of bead 1) */
#define MOP_PHASE_PME_FORCE 2 /* PME mesh forces beyond the pair kernel they run beside */
#define MOP_PHASE_RESID 3     /* residuals, spring energy, FP32 copy of d */
#define MOP_PHASE_HVP 4       /* pair Hessian-vector kernel (mode 0) */
#define MOP_PHASE_PME_HVP 5   /* PME mesh Hessian-vector products beyond the pair kernel */
#define MOP_PHASE_FD 6        /* (re-)binning + two force passes (modes 1, 2) */
#define MOP_PHASE_ASSEMBLE 7  /* gradient assembly and V_eff reduction */
int veff_grad_timed(mop_plan plan, const double* R, int32_t N, double* G, double* veff,
                    int32_t mode, double fd_h, void* ws, float* phase_ms);

/* Human-readable text of a return code. */
const char* mop_strerror(int code);

/* Fixed-point geometry of a plan, for tests: column counts, z bins, slot capacity. */
int mop_plan_info(mop_plan plan, int32_t* ncx, int32_t* ncy, int32_t* nzb, int32_t* slots);

#ifdef __cplusplus
}
#endif
#endif /* MOP_H */
