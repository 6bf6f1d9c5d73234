/*
 * FP64 CPU oracle: short-range potential U, force F = -grad U and Hessian-vector
 * product H v, with a cell list for neighbour search.  TEST INFRASTRUCTURE ONLY:
 * linked by the test suite and the benchmark's CPU-baseline leg, never by the HIP
 * library (which shares no code with this file).
 *
 * Same definitions as oracle/potential.py (shifted-force Lennard-Jones + reaction
 * field, harmonic bonds, 1-2/1-3 exclusions; the system of section 1.1, eq. 1).  With
 * ewald set, the reaction field is replaced by the Ewald real-space term
 * qq erfc(beta r)/r (shifted-force) and excluded pairs within r_c carry
 * -qq erf(beta r)/r; the reciprocal part is added by the Python wrapper (pme.py).
 *   pair separation d = x_j - x_i (minimum image), r = |d|
 *   g = phi_sf'(r)/r, h = (phi''(r) - phi_sf'(r)/r)/r^2
 *   F_i += g d;  (H v)_i += g (v_i - v_j) + h (d . (v_i - v_j)) d
 * Every atom i loops over all its neighbours j (each pair is visited from both sides,
 * each visit only updates atom i), so there are no write races between threads.
 * The cell list only finds neighbours: cells are at least r_c wide and the 27-cell
 * stencil collapses to one cell along any axis with fewer than 3 cells, so each
 * neighbour within r_c is visited exactly once per atom.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int Q;
    double box[3];
    double rc;
    const int* type;      /* [Q] */
    int ntypes;
    const double* c6;     /* [ntypes*ntypes] */
    const double* c12;    /* [ntypes*ntypes] */
    const double* q;      /* [Q] charges (e) */
    double fq;            /* electric conversion factor / eps_r */
    double krf, crf;      /* reaction-field constants */
    const int* excl_start;/* [Q+1] CSR of excluded partners (sorted per atom) */
    const int* excl;      /* [excl_start[Q]] */
    int nbonds;
    const int* bonds;     /* [nbonds*2] */
    const double* r0;     /* [nbonds] */
    const double* kb;     /* [nbonds] */
    int ewald;            /* 1: Ewald real space instead of the reaction field */
    double beta;          /* Ewald splitting parameter (nm^-1) */
} oracle_sys;

static const double PI_D = 3.14159265358979323846;

static double mi(double d, double L) { return d - L * nearbyint(d / L); }

static int is_excluded(const oracle_sys* s, int i, int j) {
    for (int k = s->excl_start[i]; k < s->excl_start[i + 1]; ++k)
        if (s->excl[k] == j) return 1;
    return 0;
}

/* Electrostatic pair energy (reaction field, or Ewald real space qq erfc(beta r)/r) and
 * its first and second derivatives. */
static double elec_terms(const oracle_sys* s, double qq, double r, double* d1, double* d2) {
    double ir = 1.0 / r;
    if (!s->ewald) {
        *d1 = qq * (-ir * ir + 2.0 * s->krf * r);
        *d2 = qq * (2.0 * ir * ir * ir + 2.0 * s->krf);
        return qq * (ir + s->krf * r * r - s->crf);
    }
    double br = s->beta * r, E = erfc(br);
    double D = 2.0 * s->beta / sqrt(PI_D) * exp(-br * br);
    *d1 = qq * (-E * ir * ir - D * ir);
    *d2 = qq * (2.0 * E * ir * ir * ir + D * (2.0 * ir * ir + 2.0 * s->beta * s->beta));
    return qq * E * ir;
}

/* Ewald correction of an excluded pair: -qq erf(beta r)/r and its derivatives. */
static double excl_terms(const oracle_sys* s, double qq, double r, double* d1, double* d2) {
    double ir = 1.0 / r, br = s->beta * r, A = erf(br);
    double D = 2.0 * s->beta / sqrt(PI_D) * exp(-br * br);
    *d1 = -qq * (D * ir - A * ir * ir);
    *d2 = -qq * (-2.0 * s->beta * s->beta * D - 2.0 * D * ir * ir + 2.0 * A * ir * ir * ir);
    return -qq * A * ir;
}

/* Shifted-force LJ + electrostatics: returns phi_sf(r); writes phi_sf'(r) and phi''(r). */
static double pair_terms(const oracle_sys* s, int ti, int tj, double qq, double r,
                         double* d1_out, double* d2_out) {
    const double c6 = s->c6[ti * s->ntypes + tj], c12 = s->c12[ti * s->ntypes + tj];
    const double rc = s->rc;
    /* Lennard-Jones */
    double ir = 1.0 / r, ir6 = pow(ir, 6.0), ir12 = ir6 * ir6;
    double lj = c12 * ir12 - c6 * ir6;
    double lj1 = (-12.0 * c12 * ir12 + 6.0 * c6 * ir6) * ir;
    double lj2 = (156.0 * c12 * ir12 - 42.0 * c6 * ir6) * ir * ir;
    double el1, el2, el = elec_terms(s, qq, r, &el1, &el2);
    /* values at the cutoff */
    double irc = 1.0 / rc, irc6 = pow(irc, 6.0), irc12 = irc6 * irc6;
    double ljc = c12 * irc12 - c6 * irc6;
    double ljc1 = (-12.0 * c12 * irc12 + 6.0 * c6 * irc6) * irc;
    double elc1, elc2, elc = elec_terms(s, qq, rc, &elc1, &elc2);
    double phic = ljc + elc, d1c = ljc1 + elc1;
    *d1_out = lj1 + el1 - d1c;
    *d2_out = lj2 + el2;
    return lj + el - phic - (r - rc) * d1c;
}

typedef struct {
    int n[3];
    int* start;   /* [ncell+1] */
    int* atoms;   /* [Q] */
    int* cell;    /* [Q] */
} cells_t;

static void build_cells(const oracle_sys* s, const double* X, cells_t* c) {
    for (int d = 0; d < 3; ++d) {
        int n = (int)floor(s->box[d] / s->rc);
        c->n[d] = n >= 3 ? n : 1;
    }
    int nc = c->n[0] * c->n[1] * c->n[2];
    c->start = (int*)calloc((size_t)nc + 1, sizeof(int));
    c->atoms = (int*)malloc(sizeof(int) * (size_t)s->Q);
    c->cell = (int*)malloc(sizeof(int) * (size_t)s->Q);
    for (int i = 0; i < s->Q; ++i) {
        int idx[3];
        for (int d = 0; d < 3; ++d) {
            double L = s->box[d];
            double x = X[3 * i + d] - L * floor(X[3 * i + d] / L);
            int k = (int)floor(x / L * c->n[d]);
            if (k >= c->n[d]) k = c->n[d] - 1;
            if (k < 0) k = 0;
            idx[d] = k;
        }
        c->cell[i] = (idx[0] * c->n[1] + idx[1]) * c->n[2] + idx[2];
        c->start[c->cell[i] + 1]++;
    }
    for (int k = 0; k < nc; ++k) c->start[k + 1] += c->start[k];
    int* fill = (int*)calloc((size_t)nc, sizeof(int));
    for (int i = 0; i < s->Q; ++i) {
        int k = c->cell[i];
        c->atoms[c->start[k] + fill[k]++] = i;
    }
    free(fill);
}

static void free_cells(cells_t* c) { free(c->start); free(c->atoms); free(c->cell); }

/*
 * Evaluate U (if U != NULL), F (if F != NULL) and H V (if V and HV are non-NULL) at
 * coordinates X [Q*3].  nthreads <= 0 uses the OpenMP default.  Returns 0.
 */
int oracle_eval(const oracle_sys* s, const double* X, const double* V, double* F,
                double* HV, double* U, int nthreads) {
    cells_t c;
    build_cells(s, X, &c);
    const int Q = s->Q;
    const double rc2 = s->rc * s->rc;
    double esum = 0.0;
    int nt = 1;
#ifdef _OPENMP
    /* a per-call thread count (the OpenMP default is left unchanged) */
    nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#endif
    (void)nt;
    int lo[3], hi[3];
    for (int d = 0; d < 3; ++d) { lo[d] = c.n[d] >= 3 ? -1 : 0; hi[d] = c.n[d] >= 3 ? 1 : 0; }

#pragma omp parallel for num_threads(nt) schedule(dynamic, 64) reduction(+ : esum)
    for (int i = 0; i < Q; ++i) {
        double fi[3] = {0, 0, 0}, hi_[3] = {0, 0, 0}, ei = 0.0;
        const int ci = c.cell[i];
        const int cx = ci / (c.n[1] * c.n[2]), cy = (ci / c.n[2]) % c.n[1], cz = ci % c.n[2];
        for (int ox = lo[0]; ox <= hi[0]; ++ox)
            for (int oy = lo[1]; oy <= hi[1]; ++oy)
                for (int oz = lo[2]; oz <= hi[2]; ++oz) {
                    int nx = (cx + ox + c.n[0]) % c.n[0];
                    int ny = (cy + oy + c.n[1]) % c.n[1];
                    int nz = (cz + oz + c.n[2]) % c.n[2];
                    int k = (nx * c.n[1] + ny) * c.n[2] + nz;
                    for (int a = c.start[k]; a < c.start[k + 1]; ++a) {
                        int j = c.atoms[a];
                        if (j == i) continue;
                        double d[3];
                        for (int e = 0; e < 3; ++e) d[e] = mi(X[3 * j + e] - X[3 * i + e], s->box[e]);
                        double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                        if (r2 >= rc2) continue;
                        const int ex = is_excluded(s, i, j);
                        if (ex && !s->ewald) continue;
                        double r = sqrt(r2), d1, d2;
                        double qq = s->fq * s->q[i] * s->q[j];
                        double phi = ex ? excl_terms(s, qq, r, &d1, &d2)
                                        : pair_terms(s, s->type[i], s->type[j], qq, r, &d1, &d2);
                        double g = d1 / r;
                        ei += 0.5 * phi;
                        for (int e = 0; e < 3; ++e) fi[e] += g * d[e];
                        if (V) {
                            double h = (d2 - g) / r2;
                            double dv[3], sdot = 0.0;
                            for (int e = 0; e < 3; ++e) {
                                dv[e] = V[3 * i + e] - V[3 * j + e];
                                sdot += d[e] * dv[e];
                            }
                            for (int e = 0; e < 3; ++e) hi_[e] += g * dv[e] + h * sdot * d[e];
                        }
                    }
                }
        if (F) for (int e = 0; e < 3; ++e) F[3 * i + e] = fi[e];
        if (V && HV) for (int e = 0; e < 3; ++e) HV[3 * i + e] = hi_[e];
        esum += ei;
    }
    /* harmonic bonds, serial */
    for (int b = 0; b < s->nbonds; ++b) {
        int i = s->bonds[2 * b], j = s->bonds[2 * b + 1];
        double d[3];
        for (int e = 0; e < 3; ++e) d[e] = mi(X[3 * j + e] - X[3 * i + e], s->box[e]);
        double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2], r = sqrt(r2);
        double k = s->kb[b], r0 = s->r0[b];
        esum += 0.5 * k * (r - r0) * (r - r0);
        double g = k * (r - r0) / r;
        if (F) for (int e = 0; e < 3; ++e) { F[3 * i + e] += g * d[e]; F[3 * j + e] -= g * d[e]; }
        if (V && HV) {
            double h = (k - g) / r2;
            double dv[3], sdot = 0.0;
            for (int e = 0; e < 3; ++e) { dv[e] = V[3 * i + e] - V[3 * j + e]; sdot += d[e] * dv[e]; }
            for (int e = 0; e < 3; ++e) {
                double t = g * dv[e] + h * sdot * d[e];
                HV[3 * i + e] += t;
                HV[3 * j + e] -= t;
            }
        }
    }
    if (U) *U = esum;
    free_cells(&c);
    return 0;
}

int oracle_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
