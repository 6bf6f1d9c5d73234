// Host-side launchers of the kernel files (all asynchronous on `st`).
#pragma once

#include "mop_internal.h"

namespace mop {

// Bin every pair bead (fdsign: 0 = R, +1 / -1 = R -/+ eps d for the FD term).
void run_binning(const SegDev* dsegs, const SegDev* hsegs, const Launch& base, char* ws,
                 const double* R, int fdsign, double fdh, hipStream_t st);

// Shared-bin finite differences: rewrite the coordinates of the current slots with
// R + fdsign * eps d (binning of R kept).
void run_displace(const SegDev* dsegs, const SegDev* hsegs, const Launch& base, char* ws,
                  const double* R, int fdsign, double fdh, hipStream_t st);

// Pair kernels.  mode 0: forces into f32 (outsel 0), hv32 (outsel 1) or f32m (outsel 2);
// energy_bead: -1 none, -2 every bead, b >= 0 that bead only.  mode 1: H v from vs into hv32.
// newton3: each pair once with atomics (1) or from both sides without atomics (0).
// lists: 1 = the force pass records neighbour lists, 2 = a later pass over the same
// binning reads them (the Hessian pass, or the displaced force passes of shared-bin finite
// differences; full-shell kernels of segments with lcap > 0), 0 = neither.
void run_pair(const SegDev* dsegs, const SegDev* hsegs, const Launch& base, char* ws, int mode,
              int outsel, int energy_bead, int waves, int newton3, hipStream_t st,
              int lists = 0);

// FP64 path kernels.
void run_resid(const SegDev* dsegs, const SegDev* hsegs, const Launch& base, const CallPtrs& cp,
               int want_dmax, hipStream_t st);
void run_assemble(const SegDev* dsegs, const SegDev* hsegs, const Launch& base, const CallPtrs& cp,
                  int fd, hipStream_t st);
void run_reduce_veff(const SegDev* dsegs, const SegDev* hsegs, const Launch& base,
                     const CallPtrs& cp, hipStream_t st);
// bead_forces / bead_hvp finishing kernels.
void run_finalize_forces(const SegDev* dsegs, const SegDev* hsegs, const Launch& base,
                         const CallPtrs& cp, hipStream_t st);
void run_prep_v(const SegDev* dsegs, const SegDev* hsegs, const Launch& base, const CallPtrs& cp,
                hipStream_t st);
void run_finalize_hvp(const SegDev* dsegs, const SegDev* hsegs, const Launch& base,
                      const CallPtrs& cp, hipStream_t st);
void run_status_clear(int* status, hipStream_t st);
void run_status_copy(const int* status, int* out, hipStream_t st);

// Metadynamics bias: adds its gradient to G (if non-null), writes {V_bias, S} to out (if
// non-null) and, with deposit, appends a Gaussian at S.
void run_bias(const BiasDev& bd, const double* R, int N, int Q, double* G, double* out,
              int deposit, int* status, hipStream_t st);
void run_bias_reset(const BiasDev& bd, hipStream_t st);

// Path integrator: the parts of one B A O A B step around the gradient evaluation.
void run_pmd_pre(const SegDev* dsegs, const SegDev* hsegs, const Launch& base, double* R, double* V,
                 const double* G, const PmdCoef& pc, uint64_t step, hipStream_t st);
// energies (device, or null): {V_eff, kinetic} of path p at energies + p * stride, and,
// unless has_bias, zeros for the bias columns {V_bias, S} that follow.
void run_pmd_post(const SegDev* dsegs, const SegDev* hsegs, const Launch& base, double* V,
                  const double* G, const PmdCoef& pc, char* ws, double* energies, int stride,
                  int has_bias, hipStream_t st);

// Particle-mesh Ewald (single-path launches; nb pair beads).  kind 0: charges / forces,
// kind 1: dipoles q v / Hessian-vector product.  fdsign != 0 displaces R by fdsign * eps d
// (finite-difference term).  run_pme_sort orders the atoms by grid tile (needed by the
// spread and gather of the same configuration); run_pme_spread writes the real grid of
// beads < nb and zeros for beads nb .. nbatch-1 of the FFT batch: FP64 for kind 0, FP32
// for kind 1 (the Hessian pass transforms in single precision; run_pme_solve32 is its
// solve, and the kind-1 gather reads that FP32 potential).
void run_pme_sort(const SegDev* dsegs, const SegDev& h, int nb, char* ws, const double* R,
                  int fdsign, double fdh, hipStream_t st);
void run_pme_spread(const SegDev* dsegs, const SegDev& h, int nb, int nbatch, char* ws,
                    const double* R, const double* V, int kind, int fdsign, double fdh,
                    hipStream_t st);
void run_pme_solve(const SegDev* dsegs, const SegDev& h, int nb, char* ws, int want_e,
                   hipStream_t st);
void run_pme_solve32(const SegDev* dsegs, const SegDev& h, int nb, char* ws, hipStream_t st);
// outsel: added to 0 f32, 1 hv32, 2 f32m (float4); written to 3 frec, 4 hrec (FP64);
// use_pgr: kind-0 potential read from pgr instead of pphi.
void run_pme_gather(const SegDev* dsegs, const SegDev& h, int nb, char* ws, const double* R,
                    const double* V, int kind, int fdsign, double fdh, int outsel, int use_pgr,
                    hipStream_t st);
void run_pme_vmax(const SegDev* dsegs, const SegDev& h, int nb, char* ws, const double* V,
                  hipStream_t st);

}  // namespace mop
