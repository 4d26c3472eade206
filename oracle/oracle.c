/*
 * oracle.c -- plain FP64 CPU reference of one explicit time step of the
 * 1D2V electron kinetic model of "An alternative simulation approach for
 * surface flashover in vacuum using a 1D2V continuum and kinetic model"
 * (Sun et al., arXiv 2303.14119), Section 2.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker the HIP library is
 * compared against.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it.  It shares no code, header,
 * table or constant with the HIP library.
 *
 * What it computes, in the paper's order:
 *   - the kinetic equation reduced to x, v_x, v_y (Eq 2) advanced by an
 *     explicit first-order upwind scheme (Section 2, the paragraph after
 *     Eq 2), here as three literal, separate sweeps x -> v_x -> v_y
 *     followed by the field-emission band source (Eq 7);
 *   - E_x from the 1D Poisson problem with E_x(0) = sigma/2eps0 at the
 *     dielectric (Section 2, paragraph on the two velocity advections);
 *   - the SEE yield matrix (Eq 8-11), the primary and secondary wall fluxes
 *     (Eq 12-14), the half-Maxwellian emission boundary (Eq 15-16), the
 *     absorbing vacuum boundary (Eq 17) and the surface-charge update (Eq 18);
 *   - optionally a wall reflection coefficient R_f (Section 2, after Eq 14),
 *     split into an elastic share (reflected specularly, v_x -> -v_x, into
 *     the emission row) and an inelastic share (re-emitted with the Eq 15
 *     shape at T_se); the rest of the arrivals induces SEE;
 *   - optionally (ORC_NOSC) the field of the surface charge alone, without
 *     the electrons' space charge: the setting of the single-particle
 *     theory of Eq 19-20, used to separate the two in the tests;
 *   - optionally (scheme 1) a second-order variant, not in the paper: each
 *     sweep in flux form with minmod-limited slopes, and the split order
 *     reversed on odd steps;
 *   - optionally (ORC_BGK) the electron-electron collision term: relaxation
 *     towards the Maxwellian of Eq 5 at T_e, at the frequency of Eq 4
 *     (Eq 3), evaluated on f^n and n^n and added after the source.
 *
 * Readings taken where the paper is silent (all listed in the design notes):
 *   cell-centred grids; Lie splitting x, v_x, v_y, source; E_x^n from
 *   (n^n, sigma^n); fluxes from f^n; ghost row from Gamma_see^n; zero inflow
 *   and tallied outflow at the velocity-box edges; discrete normalisation of
 *   the emitted, source and collisional-equilibrium VDFs; source rate J_src
 *   as a parameter; the collision term taken explicitly at f^n (so it
 *   conserves each plane's density exactly) rather than after the sweeps.
 *
 * Parity is pinned by the CPU tests (binomial closed forms of upwind
 * transport, uniform-acceleration shift, linear field for uniform charge,
 * particle conservation, SEY identities, emission normalisation, the
 * table's energy/angle mapping and the VDF temperatures; for the collision
 * term the textbook electron collision time, the geometric relaxation of
 * BGK alone and the temperature of its fixed point; for the second-order
 * variant Lax-Wendroff's exact transport of a quadratic, second-order
 * convergence and the split-order centroid).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* CODATA 2018 values (the paper states none). */
#define ORC_E    1.602176634e-19   /* elementary charge, C */
#define ORC_ME   9.1093837015e-31  /* electron mass, kg */
#define ORC_EPS0 8.8541878128e-12  /* vacuum permittivity, F/m */
#define ORC_PI   3.14159265358979323846

/* physics switches (closed-form tests turn parts of the step off) */
#define ORC_X     1u   /* x advection by v_x, with both wall boundaries */
#define ORC_VX    2u   /* v_x advection by a_x = -e E_x / m */
#define ORC_VY    4u   /* v_y advection by a_y = -e E_y / m */
#define ORC_SRC   8u   /* field-emission band source, Eq 7 */
#define ORC_SEE  16u   /* secondary emission, Eq 12-16 */
#define ORC_SELF 32u   /* E_x from sigma and the electron charge */
#define ORC_BGK  64u   /* electron-electron collisions, Eq 3-5 */
#define ORC_NOSC 128u  /* with ORC_SELF: E_x from sigma only, the electrons' space
                          charge left out (the field of the Eq 19-20 theory) */

typedef struct {
    int nx, nvx, nvy;
    double length;          /* domain extent normal to the surface, m */
    double vmax_x, vmax_y;  /* velocity box half-widths, m/s */
    double dt;              /* time step, s; 0 -> default CFL rule below */
    double cfl;
    double ey;              /* applied tangential field, V/m (negative) */
    double delta_max, a_max_ev, ks, t_se_ev;
    double j_src, x_src_lo, x_src_hi, t_src_ev;
    int emission_norm;      /* 0: discrete (emitted flux equals Gamma_see on the grid), 1: Eq 15 prefactor */
    unsigned physics_mask;
    double ex_external;     /* uniform E_x added to the self field, V/m */
    double t_e_ev;          /* temperature of the collisional equilibrium (Eq 4-5), eV */
    double ln_lambda;       /* Coulomb logarithm of Eq 4 */
    double r_refl;          /* elastic (specular) share of the wall reflection R_f (Section 2, after Eq 14) */
    double r_inel;          /* inelastic share of R_f: re-emitted with the Eq 15 shape at T_se */
    int scheme;             /* 0: first-order upwind, Lie split x, v_x, v_y, source (Section 2);
                               1: minmod-limited second order, split order reversed on odd steps */
} orc_params;

/* The observables of the state (f^n, sigma^n) after n steps. */
typedef struct {
    int64_t step;
    double t;
    double sigma;     /* sigma^n, C/m^2 */
    double g_pe;      /* primary flux into the wall from f^n, Eq 13-14, 1/(m^2 s) */
    double g_see;     /* secondary flux, Eq 12-14 (times 1 - R_f) */
    double g_top;     /* flux leaving through the vacuum boundary from f^n */
    double emitted;   /* flux carried by the emission ghost row, sum v_x g dv^2 */
    double loss_v;    /* electrons/m^2 lost through the velocity-box edges in step n-1 */
    double n_total;   /* electrons/m^2 in the domain, sum f dx dv^2 */
    double resid;     /* particle-balance residual of step n-1, electrons/m^2 */
} orc_record;

typedef struct {
    orc_params p;
    double dx, dvx, dvy, dt;
    double *vx, *vy;          /* cell-centre velocities */
    double *delta;            /* nvx*nvy, SEY on v_x<0 cells (Eq 8-11), 0 elsewhere */
    double *ghat;             /* nvx*nvy, unnormalised emission shape on v_x>0 cells */
    double zsum;              /* sum_{v_x>0} v_x ghat dvx dvy */
    double *fsrc;             /* nvx*nvy, source VDF, sum fsrc dvx dvy = 1 */
    double *feq;              /* nvx*nvy, Eq 5 equilibrium at T_e, sum feq dvx dvy = 1 */
    double *coll;             /* nx*nvx*nvy, collision increment of the step (ORC_BGK only) */
    double *wband;            /* nx, overlap of each cell with the band, fraction of dx */
    double *f, *g;            /* state and scratch, nx*nvx*nvy each */
    double *ne, *ex;          /* prologue: density and E_x of the current state */
    double *ghost;            /* nvx*nvy emission row used by the x sweep */
    double sigma;
    int64_t step;
    double last_loss_v, last_resid;
    double cfl_max_vx;        /* largest |a_x| dt / dvx seen so far */
    double nu_dt_max;         /* largest nu_ee dt seen so far (ORC_BGK) */
} orc_sim;

static size_t idx(const orc_sim* s, int k, int i, int j)
{
    return ((size_t)k * s->p.nvx + (size_t)i) * s->p.nvy + (size_t)j;
}

/* ---- SEY, Eq 8-11 ---------------------------------------------------- */
double orc_sey(double delta_max, double a_max_ev, double ks, double a_in_ev, double alpha)
{
    double z = 1.284 * a_in_ev / (a_max_ev * (1.0 + ks * alpha * alpha / ORC_PI));
    if (z <= 0.0) return 0.0;
    return 1.526 * delta_max * (1.0 + ks * alpha * alpha / (2.0 * ORC_PI))
         * -expm1(-pow(z, 1.725)) / pow(z, 0.725);   /* 1 - exp(-z^1.725) */
}

/* ---- field-emission current density, Eq 6 ----------------------------
   e_field in V/m (its magnitude times beta is the junction field), phi_ev
   the work function in eV; the result is in A/m^2. */
#define ORC_PLANCK 6.62607015e-34   /* J s */
double orc_fn_current(double e_field, double phi_ev, double beta)
{
    double E = beta * fabs(e_field);
    double phi = phi_ev * ORC_E;
    if (E == 0.0) return 0.0;
    double a = pow(ORC_E, 3) * E * E / (8.0 * ORC_PI * ORC_PLANCK * phi);
    double expo = 8.0 * ORC_PI * sqrt(2.0 * ORC_ME * pow(phi, 3)) / (3.0 * ORC_E * ORC_PLANCK * E);
    return a * exp(-expo);
}

/* ---- electron-electron collision frequency, Eq 4 ----------------------
   n_e in 1/m^3, T_e in eV (converted to joules); the result is in 1/s. */
double orc_nu_ee(double n_e, double t_e_ev, double ln_lambda)
{
    double te = t_e_ev * ORC_E;
    return n_e * pow(ORC_E, 4) * ln_lambda
         / (12.0 * pow(ORC_PI, 1.5) * ORC_EPS0 * ORC_EPS0 * sqrt(ORC_ME) * pow(te, 1.5));
}

static void build_tables(orc_sim* s)
{
    const orc_params* p = &s->p;
    /* cell centres of [-vmax, vmax]: (i + 1/2 - N/2) dv, which is the same
       number as -vmax + (i + 1/2) dv but exact in sign, so the middle cell of
       an odd grid is exactly v = 0 and opposite cells are exact negatives */
    for (int i = 0; i < p->nvx; ++i) s->vx[i] = (i + 0.5 - 0.5 * p->nvx) * s->dvx;
    for (int j = 0; j < p->nvy; ++j) s->vy[j] = (j + 0.5 - 0.5 * p->nvy) * s->dvy;

    double zsum = 0.0, srcsum = 0.0;
    for (int i = 0; i < p->nvx; ++i) {
        for (int j = 0; j < p->nvy; ++j) {
            double vx = s->vx[i], vy = s->vy[j];
            size_t m = (size_t)i * p->nvy + j;
            s->delta[m] = 0.0;
            s->ghat[m] = 0.0;
            s->fsrc[m] = 0.0;
            if (vx < 0.0) {
                /* Eq 10: incident energy in eV; Eq 11: angle to the normal */
                double a_in = 0.5 * ORC_ME * (vx * vx + vy * vy) / ORC_E;
                double alpha = atan(fabs(vy / vx));
                s->delta[m] = orc_sey(p->delta_max, p->a_max_ev, p->ks, a_in, alpha);
            }
            if (vx > 0.0) {
                /* Eq 15 shape: half Maxwellian in v_x, full in v_y, at T_se */
                s->ghat[m] = exp(-ORC_ME * (vx * vx + vy * vy) / (2.0 * p->t_se_ev * ORC_E));
                zsum += vx * s->ghat[m] * s->dvx * s->dvy;
            }
            if (vy > 0.0) {
                /* Eq 7 source VDF: full Maxwellian in v_x, half in v_y, at T_src */
                s->fsrc[m] = exp(-ORC_ME * (vx * vx + vy * vy) / (2.0 * p->t_src_ev * ORC_E));
                srcsum += s->fsrc[m] * s->dvx * s->dvy;
            }
        }
    }
    s->zsum = zsum;
    for (int m = 0; m < p->nvx * p->nvy; ++m)
        s->fsrc[m] = srcsum > 0.0 ? s->fsrc[m] / srcsum : 0.0;

    /* Eq 5: full Maxwellian in both velocity components at T_e, normalised
       on the grid so that its discrete integral is one (then the collision
       term moves no electrons between planes) */
    double eqsum = 0.0;
    for (int i = 0; i < p->nvx; ++i)
        for (int j = 0; j < p->nvy; ++j) {
            double vx = s->vx[i], vy = s->vy[j];
            size_t m = (size_t)i * p->nvy + j;
            s->feq[m] = p->t_e_ev > 0.0
                ? exp(-ORC_ME * (vx * vx + vy * vy) / (2.0 * p->t_e_ev * ORC_E)) : 0.0;
            eqsum += s->feq[m] * s->dvx * s->dvy;
        }
    for (int m = 0; m < p->nvx * p->nvy; ++m)
        s->feq[m] = eqsum > 0.0 ? s->feq[m] / eqsum : 0.0;

    for (int k = 0; k < p->nx; ++k) {
        double lo = k * s->dx, hi = (k + 1) * s->dx;
        double a = lo > p->x_src_lo ? lo : p->x_src_lo;
        double b = hi < p->x_src_hi ? hi : p->x_src_hi;
        s->wband[k] = b > a ? (b - a) / s->dx : 0.0;
    }
}

/* ---- prologue: moments, field, wall fluxes of the current state ------ */
typedef struct { double g_pe, g_see, g_top, emitted, n_total; } orc_moments;

static orc_moments prologue(orc_sim* s)
{
    const orc_params* p = &s->p;
    orc_moments mo = {0, 0, 0, 0, 0};
    const double dv2 = s->dvx * s->dvy;

    /* electron density of each x cell */
#pragma omp parallel for schedule(static)
    for (int k = 0; k < p->nx; ++k) {
        double acc = 0.0;
        for (int i = 0; i < p->nvx; ++i)
            for (int j = 0; j < p->nvy; ++j)
                acc += s->f[idx(s, k, i, j)];
        s->ne[k] = acc * dv2;
    }
    for (int k = 0; k < p->nx; ++k) mo.n_total += s->ne[k] * s->dx;

    /* Gauss's law in 1D: dE/dx = -e n / eps0 with E(0) = sigma / 2 eps0.
       At the centre of cell k the enclosed charge is the cells below k plus
       half of cell k. */
    double below = 0.0;
    for (int k = 0; k < p->nx; ++k) {
        double enclosed = below + 0.5 * s->ne[k];
        double self = 0.0;
        if (p->physics_mask & ORC_SELF) {
            self = s->sigma / (2.0 * ORC_EPS0);
            if (!(p->physics_mask & ORC_NOSC)) self -= ORC_E / ORC_EPS0 * s->dx * enclosed;
        }
        s->ex[k] = self + p->ex_external;
        below += s->ne[k];
    }

    if (p->physics_mask & ORC_X) {
        /* Eq 13-14: primary flux element and its SEE share at the wall cell */
        for (int i = 0; i < p->nvx; ++i) {
            if (!(s->vx[i] < 0.0)) continue;
            for (int j = 0; j < p->nvy; ++j) {
                double dgpe = -s->vx[i] * s->f[idx(s, 0, i, j)] * dv2;
                mo.g_pe += dgpe;
                if (p->physics_mask & ORC_SEE)
                    mo.g_see += s->delta[(size_t)i * p->nvy + j] * dgpe;   /* Eq 12 */
            }
        }
        for (int i = 0; i < p->nvx; ++i) {
            if (!(s->vx[i] > 0.0)) continue;
            for (int j = 0; j < p->nvy; ++j)
                mo.g_top += s->vx[i] * s->f[idx(s, p->nx - 1, i, j)] * dv2;
        }
    }

    /* only the fraction 1 - R_f of the arriving electrons induces SEE; R_f
       is split into an elastic (specular) and an inelastic share */
    mo.g_see *= 1.0 - p->r_refl - p->r_inel;

    /* Eq 15: emission boundary row at x = 0 for v_x > 0.  The inelastically
       reflected electrons leave with the secondaries' shape (they have lost
       their energy to the wall) */
    double g_shape = mo.g_see + p->r_inel * mo.g_pe;
    double coef;
    if (p->emission_norm == 0)
        coef = s->zsum > 0.0 ? g_shape / s->zsum : 0.0;
    else {
        double mt = ORC_ME / (p->t_se_ev * ORC_E);
        coef = g_shape / sqrt(2.0 * ORC_PI) * pow(mt, 1.5);
    }
    for (int i = 0; i < p->nvx; ++i)
        for (int j = 0; j < p->nvy; ++j) {
            size_t m = (size_t)i * p->nvy + j;
            s->ghost[m] = coef * s->ghat[m];
            /* specular reflection: the wall cell's electrons at -v_x come
               back at +v_x (cell nvx-1-i holds -v_x of cell i) */
            if (s->vx[i] > 0.0 && p->r_refl > 0.0)
                s->ghost[m] += p->r_refl * s->f[idx(s, 0, p->nvx - 1 - i, j)];
            if (s->vx[i] > 0.0) mo.emitted += s->vx[i] * s->ghost[m] * dv2;
        }
    if (!(p->physics_mask & ORC_X)) mo.emitted = 0.0;
    return mo;
}

/* ---- the three sweeps ------------------------------------------------ */

/* x advection by v_x, upwind (Eq 2 first term); the emission row is the
   inflow at the dielectric and nothing enters through the vacuum face
   (Eq 17). */
static void sweep_x(orc_sim* s, const double* in, double* out)
{
    const orc_params* p = &s->p;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < p->nx; ++k)
        for (int i = 0; i < p->nvx; ++i) {
            double c = s->vx[i] * s->dt / s->dx;
            for (int j = 0; j < p->nvy; ++j) {
                double fk = in[idx(s, k, i, j)];
                double r;
                if (c > 0.0) {
                    double fup = k > 0 ? in[idx(s, k - 1, i, j)] : s->ghost[(size_t)i * p->nvy + j];
                    r = fk - c * (fk - fup);
                } else if (c < 0.0) {
                    double fup = k < p->nx - 1 ? in[idx(s, k + 1, i, j)] : 0.0;
                    r = fk - c * (fup - fk);
                } else {
                    r = fk;
                }
                out[idx(s, k, i, j)] = r;
            }
        }
}

/* v_x advection by a_x(x_k) = -e E_x(x_k) / m, upwind on the sign of a_x.
   Nothing enters through the velocity-box edges; what leaves is tallied. */
static double sweep_vx(orc_sim* s, const double* in, double* out)
{
    const orc_params* p = &s->p;
    double lost = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : lost)
    for (int k = 0; k < p->nx; ++k) {
        double ax = -ORC_E * s->ex[k] / ORC_ME;
        double d = ax * s->dt / s->dvx;
        for (int i = 0; i < p->nvx; ++i)
            for (int j = 0; j < p->nvy; ++j) {
                double fi = in[idx(s, k, i, j)];
                double r;
                if (d > 0.0) {
                    double fup = i > 0 ? in[idx(s, k, i - 1, j)] : 0.0;
                    r = fi - d * (fi - fup);
                    if (i == p->nvx - 1) lost += d * fi;
                } else if (d < 0.0) {
                    double fup = i < p->nvx - 1 ? in[idx(s, k, i + 1, j)] : 0.0;
                    r = fi - d * (fup - fi);
                    if (i == 0) lost += -d * fi;
                } else {
                    r = fi;
                }
                out[idx(s, k, i, j)] = r;
            }
    }
    return lost * s->dx * s->dvx * s->dvy;
}

/* v_y advection by a_y = -e E_y / m (constant), upwind. */
static double sweep_vy(orc_sim* s, const double* in, double* out)
{
    const orc_params* p = &s->p;
    double ay = -ORC_E * p->ey / ORC_ME;
    double d = ay * s->dt / s->dvy;
    double lost = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : lost)
    for (int k = 0; k < p->nx; ++k)
        for (int i = 0; i < p->nvx; ++i)
            for (int j = 0; j < p->nvy; ++j) {
                double fj = in[idx(s, k, i, j)];
                double r;
                if (d > 0.0) {
                    double fup = j > 0 ? in[idx(s, k, i, j - 1)] : 0.0;
                    r = fj - d * (fj - fup);
                    if (j == p->nvy - 1) lost += d * fj;
                } else if (d < 0.0) {
                    double fup = j < p->nvy - 1 ? in[idx(s, k, i, j + 1)] : 0.0;
                    r = fj - d * (fup - fj);
                    if (j == 0) lost += -d * fj;
                } else {
                    r = fj;
                }
                out[idx(s, k, i, j)] = r;
            }
    return lost * s->dx * s->dvx * s->dvy;
}

/* ---- second-order sweeps (scheme 1) ------------------------------------
   Each 1D advection at constant Courant number c (|c| <= 1) is taken in
   flux form.  The value carried through a face is the upwind cell's value
   moved towards the face by its limited slope: for c > 0 the face right of
   cell m carries f_m + (1 - c)/2 s_m, for c < 0 the face left of cell m
   carries f_m - (1 + c)/2 s_m, and f'_m = f_m - c (right face - left face).
   s_m is the minmod of the two one-sided differences of cell m; it is zero
   in the first and last cell of every line, so every boundary face (the
   dielectric, the vacuum face, the velocity-box edges) carries the plain
   upwind value and the wall, emission, escape and loss bookkeeping is the
   same as in the first-order scheme.  With s = 0 everywhere the update is
   the first-order upwind one. */
static double minmod(double a, double b)
{
    if (a > 0.0 && b > 0.0) return a < b ? a : b;
    if (a < 0.0 && b < 0.0) return a > b ? a : b;
    return 0.0;
}

/* slope of cell m of a line of n cells, values v(m) = line[m * stride] */
static double line_slope(const double* line, size_t stride, int m, int n)
{
    if (m <= 0 || m >= n - 1) return 0.0;
    return minmod(line[m * stride] - line[(m - 1) * stride], line[(m + 1) * stride] - line[m * stride]);
}

/* the limited update of cell m; lo / hi are the values upwind of the first
   and last face from outside the line (what flows in there) */
static double line_update(const double* line, size_t stride, int m, int n, double c, double lo, double hi)
{
    double fm = line[m * stride];
    double right, left;
    if (c > 0.0) {
        right = fm + 0.5 * (1.0 - c) * line_slope(line, stride, m, n);
        left = m > 0 ? line[(m - 1) * stride] + 0.5 * (1.0 - c) * line_slope(line, stride, m - 1, n) : lo;
    } else if (c < 0.0) {
        left = fm - 0.5 * (1.0 + c) * line_slope(line, stride, m, n);
        right = m < n - 1 ? line[(m + 1) * stride] - 0.5 * (1.0 + c) * line_slope(line, stride, m + 1, n) : hi;
    } else {
        return fm;
    }
    return fm - c * (right - left);
}

static void sweep_x2(orc_sim* s, const double* in, double* out)
{
    const orc_params* p = &s->p;
    const size_t plane = (size_t)p->nvx * p->nvy;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < p->nx; ++k)
        for (int i = 0; i < p->nvx; ++i) {
            double c = s->vx[i] * s->dt / s->dx;
            for (int j = 0; j < p->nvy; ++j) {
                const double* line = in + idx(s, 0, i, j);
                double ghost = s->ghost[(size_t)i * p->nvy + j];
                out[idx(s, k, i, j)] = line_update(line, plane, k, p->nx, c, ghost, 0.0);
            }
        }
}

static double sweep_vx2(orc_sim* s, const double* in, double* out)
{
    const orc_params* p = &s->p;
    double lost = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : lost)
    for (int k = 0; k < p->nx; ++k) {
        double d = -ORC_E * s->ex[k] / ORC_ME * s->dt / s->dvx;
        for (int i = 0; i < p->nvx; ++i)
            for (int j = 0; j < p->nvy; ++j) {
                const double* line = in + idx(s, k, 0, j);
                out[idx(s, k, i, j)] = line_update(line, (size_t)p->nvy, i, p->nvx, d, 0.0, 0.0);
                if (d > 0.0 && i == p->nvx - 1) lost += d * line[(size_t)i * p->nvy];
                if (d < 0.0 && i == 0) lost += -d * line[0];
            }
    }
    return lost * s->dx * s->dvx * s->dvy;
}

static double sweep_vy2(orc_sim* s, const double* in, double* out)
{
    const orc_params* p = &s->p;
    double d = -ORC_E * p->ey / ORC_ME * s->dt / s->dvy;
    double lost = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : lost)
    for (int k = 0; k < p->nx; ++k)
        for (int i = 0; i < p->nvx; ++i) {
            const double* line = in + idx(s, k, i, 0);
            for (int j = 0; j < p->nvy; ++j) {
                out[idx(s, k, i, j)] = line_update(line, 1, j, p->nvy, d, 0.0, 0.0);
                if (d > 0.0 && j == p->nvy - 1) lost += d * line[j];
                if (d < 0.0 && j == 0) lost += -d * line[0];
            }
        }
    return lost * s->dx * s->dvx * s->dvy;
}

/* Flux of the array entering an x sweep through the dielectric (v_x < 0,
   absorbed) and through x = L (v_x > 0): the first and last cell's values,
   as their slopes are zero. */
static void boundary_outflow(const orc_sim* s, const double* f, double* wall, double* top)
{
    const orc_params* p = &s->p;
    const double dv2 = s->dvx * s->dvy;
    double w = 0.0, t = 0.0;
    for (int i = 0; i < p->nvx; ++i)
        for (int j = 0; j < p->nvy; ++j) {
            if (s->vx[i] < 0.0) w += -s->vx[i] * f[idx(s, 0, i, j)] * dv2;
            if (s->vx[i] > 0.0) t += s->vx[i] * f[idx(s, p->nx - 1, i, j)] * dv2;
        }
    *wall = w;
    *top = t;
}

/* Eq 7 band source, added after the advections. */
static double add_source(orc_sim* s, double* f)
{
    const orc_params* p = &s->p;
    double band = p->x_src_hi - p->x_src_lo;
    double injected = 0.0;
    if (!(band > 0.0)) return 0.0;
    for (int k = 0; k < p->nx; ++k) {
        double rate = s->dt * (p->j_src / ORC_E) * s->wband[k] / band;
        if (rate == 0.0) continue;
        for (int i = 0; i < p->nvx; ++i)
            for (int j = 0; j < p->nvy; ++j)
                f[idx(s, k, i, j)] += rate * s->fsrc[(size_t)i * p->nvy + j];
        injected += rate * s->dx;
    }
    double srcnorm = 0.0;
    for (int m = 0; m < p->nvx * p->nvy; ++m) srcnorm += s->fsrc[m] * s->dvx * s->dvy;
    return injected * srcnorm;
}

/* Eq 3: the BGK collision increment dt nu_ee (n_e feq - f) of every cell,
   from the state at the start of the step (f^n, and n^n from the prologue);
   it is added to f after the sweeps and the source. */
static void collision_increment(orc_sim* s)
{
    const orc_params* p = &s->p;
    for (int k = 0; k < p->nx; ++k) {
        double nk = s->ne[k];
        double nudt = orc_nu_ee(nk, p->t_e_ev, p->ln_lambda) * s->dt;
        if (nudt > s->nu_dt_max) s->nu_dt_max = nudt;
        for (int i = 0; i < p->nvx; ++i)
            for (int j = 0; j < p->nvy; ++j) {
                size_t c = idx(s, k, i, j);
                s->coll[c] = nudt * (nk * s->feq[(size_t)i * p->nvy + j] - s->f[c]);
            }
    }
}

/* ---- public API --------------------------------------------------------- */

orc_sim* orc_create(const orc_params* p)
{
    if (p->nx < 1 || p->nvx < 1 || p->nvy < 1) return NULL;
    orc_sim* s = (orc_sim*)calloc(1, sizeof(orc_sim));
    if (!s) return NULL;
    s->p = *p;
    s->dx = p->length / p->nx;
    s->dvx = 2.0 * p->vmax_x / p->nvx;
    s->dvy = 2.0 * p->vmax_y / p->nvy;
    /* default step: the CFL fraction of the tightest of the x transit time
       of the fastest cell and the time the applied field needs to move one
       velocity cell (in v_x too, since the surface-charge field stays below
       the applied one in SEEA) */
    if (p->dt > 0.0) {
        s->dt = p->dt;
    } else {
        double tmin = s->dx / p->vmax_x;
        double ay = fabs(ORC_E * p->ey / ORC_ME);
        if (ay > 0.0) {
            if (s->dvx / ay < tmin) tmin = s->dvx / ay;
            if (s->dvy / ay < tmin) tmin = s->dvy / ay;
        }
        s->dt = p->cfl * tmin;
    }
    size_t cells = (size_t)p->nx * p->nvx * p->nvy;
    size_t vcells = (size_t)p->nvx * p->nvy;
    s->vx = (double*)calloc(p->nvx, sizeof(double));
    s->vy = (double*)calloc(p->nvy, sizeof(double));
    s->delta = (double*)calloc(vcells, sizeof(double));
    s->ghat = (double*)calloc(vcells, sizeof(double));
    s->fsrc = (double*)calloc(vcells, sizeof(double));
    s->feq = (double*)calloc(vcells, sizeof(double));
    s->coll = (p->physics_mask & ORC_BGK) ? (double*)calloc(cells, sizeof(double)) : NULL;
    s->ghost = (double*)calloc(vcells, sizeof(double));
    s->wband = (double*)calloc(p->nx, sizeof(double));
    s->ne = (double*)calloc(p->nx, sizeof(double));
    s->ex = (double*)calloc(p->nx, sizeof(double));
    s->f = (double*)calloc(cells, sizeof(double));
    s->g = (double*)calloc(cells, sizeof(double));
    if (!s->vx || !s->vy || !s->delta || !s->ghat || !s->fsrc || !s->feq || !s->ghost || !s->wband ||
        !s->ne || !s->ex || !s->f || !s->g || ((p->physics_mask & ORC_BGK) && !s->coll)) {
        free(s->vx); free(s->vy); free(s->delta); free(s->ghat); free(s->fsrc); free(s->feq);
        free(s->coll); free(s->ghost);
        free(s->wband); free(s->ne); free(s->ex); free(s->f); free(s->g); free(s);
        return NULL;
    }
    build_tables(s);
    return s;
}

void orc_destroy(orc_sim* s)
{
    if (!s) return;
    free(s->vx); free(s->vy); free(s->delta); free(s->ghat); free(s->fsrc); free(s->feq);
    free(s->coll); free(s->ghost);
    free(s->wband); free(s->ne); free(s->ex); free(s->f); free(s->g); free(s);
}

void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

double orc_dt(const orc_sim* s) { return s->dt; }

/* Replace the state: f (NULL keeps it), sigma and the step counter. */
void orc_set_state(orc_sim* s, const double* f, double sigma, int64_t step)
{
    size_t cells = (size_t)s->p.nx * s->p.nvx * s->p.nvy;
    if (f) memcpy(s->f, f, cells * sizeof(double));
    s->sigma = sigma;
    s->step = step;
    s->last_loss_v = 0.0;
    s->last_resid = 0.0;
}

static void fill_record(orc_sim* s, const orc_moments* mo, orc_record* r)
{
    r->step = s->step;
    r->t = (double)s->step * s->dt;
    r->sigma = s->sigma;
    r->g_pe = mo->g_pe;
    r->g_see = mo->g_see;
    r->g_top = mo->g_top;
    r->emitted = mo->emitted;
    r->loss_v = s->last_loss_v;
    r->n_total = mo->n_total;
    r->resid = s->last_resid;
}

/* Advance n steps.  If trace is not NULL, trace[m] receives the observables
   of the state after step m+1.

   Scheme 0 (the paper's): x, v_x, v_y, source in every step.  Scheme 1:
   the limited sweeps in that order on even steps (step counter n even) and
   in the reverse order (source, v_y, v_x, x) on odd steps, so that two
   consecutive steps form a symmetric composition.  The wall fluxes, the
   yield and the emission row come from f^n in both orders (the prologue);
   on a reversed step the electrons absorbed at the wall and at x = L are
   those of the array the x sweep transports (the wall cell after the
   velocity sweeps), and Eq 18 charges the wall with that absorbed flux. */
void orc_step(orc_sim* s, int64_t n, orc_record* trace)
{
    const orc_params* p = &s->p;
    for (int64_t it = 0; it < n; ++it) {
        orc_moments mo = prologue(s);

        for (int k = 0; k < p->nx; ++k) {
            double d = fabs(-ORC_E * s->ex[k] / ORC_ME * s->dt / s->dvx);
            if ((p->physics_mask & ORC_VX) && d > s->cfl_max_vx) s->cfl_max_vx = d;
        }

        if (p->physics_mask & ORC_BGK) collision_increment(s);

        double* a = s->f;
        double* b = s->g;
        double lost = 0.0, injected = 0.0;
        /* absorbed at the wall and escaped at x = L during the x sweep */
        double g_abs = mo.g_pe, top_abs = mo.g_top;
        const int second = p->scheme == 1;
        const int reversed = second && (s->step & 1);
        if (!reversed) {
            if (p->physics_mask & ORC_X) {
                if (second) sweep_x2(s, a, b); else sweep_x(s, a, b);
                double* t = a; a = b; b = t;
            }
            if (p->physics_mask & ORC_VX) {
                lost += second ? sweep_vx2(s, a, b) : sweep_vx(s, a, b);
                double* t = a; a = b; b = t;
            }
            if (p->physics_mask & ORC_VY) {
                lost += second ? sweep_vy2(s, a, b) : sweep_vy(s, a, b);
                double* t = a; a = b; b = t;
            }
            if (p->physics_mask & ORC_SRC) injected = add_source(s, a);
        } else {
            if (p->physics_mask & ORC_SRC) injected = add_source(s, a);
            if (p->physics_mask & ORC_VY) { lost += sweep_vy2(s, a, b); double* t = a; a = b; b = t; }
            if (p->physics_mask & ORC_VX) { lost += sweep_vx2(s, a, b); double* t = a; a = b; b = t; }
            if (p->physics_mask & ORC_X) {
                boundary_outflow(s, a, &g_abs, &top_abs);
                sweep_x2(s, a, b);
                double* t = a; a = b; b = t;
            }
        }
        if (!(p->physics_mask & ORC_X)) g_abs = top_abs = 0.0;
        if (p->physics_mask & ORC_BGK) {
            size_t cells = (size_t)p->nx * p->nvx * p->nvy;
            for (size_t c = 0; c < cells; ++c) a[c] += s->coll[c];
        }
        s->f = a;
        s->g = b;

        /* Eq 18: the surface charge of the next step.  Secondaries and the
           reflected electrons (elastic R_f and inelastic shares, taken from
           f^n like the yield) leave the wall; the absorbed electrons charge it */
        double g_back = (p->physics_mask & ORC_X) ? (p->r_refl + p->r_inel) * mo.g_pe : 0.0;
        s->sigma = s->sigma + ORC_E * s->dt * (mo.g_see + g_back - g_abs);
        s->step += 1;

        orc_moments nx = prologue(s);
        double expected = s->dt * (mo.emitted - g_abs - top_abs) + injected - lost;
        s->last_loss_v = lost;
        s->last_resid = (nx.n_total - mo.n_total) - expected;
        if (trace) fill_record(s, &nx, &trace[it]);
    }
}

void orc_get_record(orc_sim* s, orc_record* r)
{
    orc_moments mo = prologue(s);
    fill_record(s, &mo, r);
}

void orc_get_f(const orc_sim* s, double* out)
{
    memcpy(out, s->f, (size_t)s->p.nx * s->p.nvx * s->p.nvy * sizeof(double));
}

/* E_x and n_e of the current state (from the prologue). */
void orc_get_field(orc_sim* s, double* ex, double* ne)
{
    prologue(s);
    if (ex) memcpy(ex, s->ex, (size_t)s->p.nx * sizeof(double));
    if (ne) memcpy(ne, s->ne, (size_t)s->p.nx * sizeof(double));
}

/* Tables, for the pins: any pointer may be NULL. */
void orc_get_tables(const orc_sim* s, double* vx, double* vy, double* delta, double* ghat,
                    double* fsrc, double* wband, double* zsum)
{
    size_t vcells = (size_t)s->p.nvx * s->p.nvy;
    if (vx) memcpy(vx, s->vx, (size_t)s->p.nvx * sizeof(double));
    if (vy) memcpy(vy, s->vy, (size_t)s->p.nvy * sizeof(double));
    if (delta) memcpy(delta, s->delta, vcells * sizeof(double));
    if (ghat) memcpy(ghat, s->ghat, vcells * sizeof(double));
    if (fsrc) memcpy(fsrc, s->fsrc, vcells * sizeof(double));
    if (wband) memcpy(wband, s->wband, (size_t)s->p.nx * sizeof(double));
    if (zsum) *zsum = s->zsum;
}

/* Emission row of the current state (what the next x sweep injects). */
void orc_get_ghost(orc_sim* s, double* ghost)
{
    prologue(s);
    memcpy(ghost, s->ghost, (size_t)s->p.nvx * s->p.nvy * sizeof(double));
}

double orc_cfl_max_vx(const orc_sim* s) { return s->cfl_max_vx; }

double orc_nu_dt_max(const orc_sim* s) { return s->nu_dt_max; }

/* The collisional equilibrium of Eq 5 on the grid (nvx*nvy). */
void orc_get_feq(const orc_sim* s, double* out)
{
    memcpy(out, s->feq, (size_t)s->p.nvx * s->p.nvy * sizeof(double));
}
