/*
 * THIIM reference oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously-correct FP64 CPU implementation of the iterated
 * split-field Yee update of the Time Harmonic Inverse Iteration Method
 * (Malas et al., "Optimization of an electromagnetics code with multicore
 * wavefront diamond blocking and multi-dimensional intra-tile
 * parallelization", arXiv:1510.05218).
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this library.  It shares no source with the GPU library.
 *
 * What it follows:
 *   - Sec. I-A, Eq. (3) and (4): leapfrog pseudo-time update with the phase
 *     factors exp(i w tau) and exp(i w tau / 2); H^{n+1/2} uses E^n, E^{n+1}
 *     uses H^{n+1/2}.
 *   - Sec. I-A, Eq. (5): "back iteration" for cells with negative
 *     permittivity (only the E coefficients change).
 *   - Sec. I-A, Eq. (6) and (7): Berenger split field, 12 split components.
 *   - Sec. III, Listings 1 and 2: one loop nest over k, j, i per split
 *     component, the interleaved (re, im) layout with x fastest, the index
 *     shift of each difference and the flop count of one update (22 with a
 *     source array, 20 without).
 *   - Sec. II-B / Fig. 3: H depends on E at an offset of -1, E depends on H
 *     in the opposite (+1) direction.
 *
 * Readings taken where the paper is silent (each is listed in the design
 * notes of the repository):
 *   - Normalised units eps0 = mu0 = c0 = 1, mu_r = 1, grid step h.
 *   - Complex relative permittivity eps_r = eps' - i eps'' (paper's
 *     exp(+i w tau) convention); the loss enters as sigma_mat = w eps''.
 *   - The PML conductivity profiles (electric, per E plane; magnetic, per H
 *     plane) are inputs; they act only on the four z-difference components.
 *   - Ghost values beyond the z walls are zero (homogeneous Dirichlet);
 *     x and y are periodic or Dirichlet.
 *   - Source arrays exist only for the four z-difference components, as in
 *     the paper's array inventory.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -shared -fPIC (no fast-math).
 */
#include <complex.h>
#include <math.h>
#include <stddef.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NCOMP 12
#define NCOEF 28

/* Split components, listing naming: F_ab is the part of field F, component a,
 * driven by the other field's component b.  Index order (also the order of
 * field arrays across the API):
 *   0 H_xy  1 H_xz  2 H_yx  3 H_yz  4 H_zx  5 H_zy
 *   6 E_xy  7 E_xz  8 E_yx  9 E_yz 10 E_zx 11 E_zy
 *
 * For each: the two split arrays forming the driving component G_b, the axis
 * of the difference (0 = x, 1 = y, 2 = z) and the sign of that derivative in
 * the curl of Eq. (1)/(2):
 *   dH/dt = -curl E :  H_x <- +d_z E_y - d_y E_z,  H_y <- -d_z E_x + d_x E_z,
 *                      H_z <- -d_x E_y + d_y E_x
 *   dE/dt = +curl H :  E_x <- +d_y H_z - d_z H_y,  E_y <- +d_z H_x - d_x H_z,
 *                      E_z <- +d_x H_y - d_y H_x
 */
typedef struct {
    int g1, g2;  /* indices of the two split parts of the driving component */
    int axis;    /* 0 x, 1 y, 2 z */
    int sign;    /* +1 / -1 */
    int src;     /* index of the source array (0..3) or -1 */
} comp_t;

static const comp_t COMP[NCOMP] = {
    /* H_xy */ { 8,  9, 2, +1,  0},   /* E_y = E_yx + E_yz */
    /* H_xz */ {10, 11, 1, -1, -1},   /* E_z = E_zx + E_zy */
    /* H_yx */ { 6,  7, 2, -1,  1},   /* E_x = E_xy + E_xz (Listing 1) */
    /* H_yz */ {10, 11, 0, +1, -1},
    /* H_zx */ { 6,  7, 1, +1, -1},   /* Listing 2 */
    /* H_zy */ { 8,  9, 0, -1, -1},
    /* E_xy */ { 2,  3, 2, -1,  2},   /* H_y = H_yx + H_yz */
    /* E_xz */ { 4,  5, 1, +1, -1},   /* H_z = H_zx + H_zy */
    /* E_yx */ { 0,  1, 2, +1,  3},   /* H_x = H_xy + H_xz */
    /* E_yz */ { 4,  5, 0, -1, -1},
    /* E_zx */ { 0,  1, 1, -1, -1},
    /* E_zy */ { 2,  3, 0, +1, -1},
};

/* Coefficient array order: t_q = q, c_q = 12 + q (q = 0..11),
 * Src for H_xy, H_yx, E_xy, E_yx = 24..27.  Source input order:
 * S_Hx, S_Hy, S_Ex, S_Ey (the field component each source drives). */

typedef struct {
    int nx, ny, nz;
    int bcx, bcy; /* 0 periodic, 1 Dirichlet */
} grid_t;

/* Index of the neighbour of (k, j, i) one step along `axis` in direction
 * `dir` (+1 / -1), or -1 when it lies outside the domain (ghost value 0). */
static long nbr(const grid_t *g, int k, int j, int i, int axis, int dir)
{
    if (axis == 0) {
        i += dir;
        if (i < 0 || i >= g->nx) {
            if (g->bcx) return -1;
            i = (i + g->nx) % g->nx;
        }
    } else if (axis == 1) {
        j += dir;
        if (j < 0 || j >= g->ny) {
            if (g->bcy) return -1;
            j = (j + g->ny) % g->ny;
        }
    } else {
        k += dir;
        if (k < 0 || k >= g->nz) return -1;
    }
    return ((long)k * g->ny + j) * g->nx + i;
}

/* ---------------------------------------------------------------------- */
/* Coefficients (Eq. 3, 4, 5 solved for the new value).                    */
/* ---------------------------------------------------------------------- */

/* H update, Eq. (4) with mu = 1:
 *   (e^{iwt/2} H^{n+1/2} - e^{-iwt/2} H^{n-1/2}) / tau
 *       = -(curl E^n) - sigma* H^{n+1/2} + S_H
 *   => H^{n+1/2} = t H^{n-1/2} + s c dE + Src, d = e^{iwt/2} + tau sigma*,
 *      t = e^{-iwt/2} / d,  c = (tau / h) / d,  Src = tau S_H / d. */
static void coef_h_ph(double complex ph2, double tau, double h, double sig_star,
                      double complex *t, double complex *c, double complex *sscale)
{
    double complex d = ph2 + tau * sig_star;
    *t = conj(ph2) / d;
    *c = (tau / h) / d;
    *sscale = tau / d;
}

static void coef_h(double omega, double tau, double h, double sig_star,
                   double complex *t, double complex *c, double complex *sscale)
{
    coef_h_ph(cexp(I * (omega * tau / 2.0)), tau, h, sig_star, t, c, sscale);
}

/* E update.  Forward iteration, Eq. (3), for eps' > 0:
 *   (e^{iwt} E^{n+1} - E^n) / tau
 *       = (1/eps) curl H e^{iwt/2} - (sigma/eps) E^{n+1} e^{iwt} + S_E
 *   => d = 1 + tau sigma / eps,  t = e^{-iwt} / d,
 *      c = (tau / (eps h)) e^{-iwt/2} / d,  Src = tau e^{-iwt} S_E / d.
 * Back iteration, Eq. (5), for eps' < 0:
 *   (e^{iwt} E^n - E^{n+1}) / tau
 *       = (1/eps) curl H e^{iwt/2} - (sigma/eps) E^{n+1} + S_E
 *   => d = 1 - tau sigma / eps,  t = e^{iwt} / d,
 *      c = -(tau / (eps h)) e^{iwt/2} / d,  Src = -tau S_E / d. */
static void coef_e_ph(double complex ph, double complex ph2, double tau, double h,
                      double eps, double sigma, double complex *t, double complex *c,
                      double complex *sscale)
{
    if (eps > 0.0) {
        double d = 1.0 + tau * sigma / eps;
        *t = conj(ph) / d;
        *c = (tau / (eps * h)) * conj(ph2) / d;
        *sscale = tau * conj(ph) / d;
    } else {
        double d = 1.0 - tau * sigma / eps;
        *t = ph / d;
        *c = -(tau / (eps * h)) * ph2 / d;
        *sscale = -tau / d;
    }
}

static void coef_e(double omega, double tau, double h, double eps, double sigma,
                   double complex *t, double complex *c, double complex *sscale)
{
    coef_e_ph(cexp(I * (omega * tau)), cexp(I * (omega * tau / 2.0)), tau, h, eps, sigma,
              t, c, sscale);
}

static void put(double *a, long p, double complex v)
{
    a[2 * p] = creal(v);
    a[2 * p + 1] = cimag(v);
}

/* Builds the 28 coefficient arrays (interleaved complex, [nz][ny][nx]).
 *   eps   : 2*N doubles, (eps', eps'') per cell, eps_r = eps' - i eps''
 *   sig_e : nz, electric PML conductivity at the E planes
 *   sig_h : nz, magnetic PML conductivity at the H planes
 *   src   : 4 pointers (S_Hx, S_Hy, S_Ex, S_Ey), 2*N doubles each, or NULL
 * Returns 0, or -1 on eps' == 0 / non-finite input. */
int oracle_coeffs(int nx, int ny, int nz, const double *eps,
                  const double *sig_e, const double *sig_h,
                  const double *const *src, double omega, double tau, double h,
                  double *const *coef)
{
    long N = (long)nx * ny * nz;
    for (long p = 0; p < N; p++) {
        double ep = eps[2 * p], epp = eps[2 * p + 1];
        if (!(ep != 0.0) || !isfinite(ep) || !isfinite(epp)) return -1;
    }
    for (int k = 0; k < nz; k++) {
        for (int j = 0; j < ny; j++) {
            for (int i = 0; i < nx; i++) {
                long p = ((long)k * ny + j) * nx + i;
                double ep = eps[2 * p], epp = eps[2 * p + 1];
                double sig_mat = omega * epp;
                for (int q = 0; q < NCOMP; q++) {
                    const comp_t *cq = &COMP[q];
                    double complex t, c, s;
                    if (q < 6) {
                        double sst = (cq->axis == 2) ? sig_h[k] : 0.0;
                        coef_h(omega, tau, h, sst, &t, &c, &s);
                    } else {
                        double sg = sig_mat + ((cq->axis == 2) ? sig_e[k] : 0.0);
                        coef_e(omega, tau, h, ep, sg, &t, &c, &s);
                    }
                    put(coef[q], p, t);
                    put(coef[12 + q], p, c);
                    if (cq->src >= 0) {
                        double complex S = 0.0;
                        const double *sa = src ? src[cq->src] : NULL;
                        if (sa) S = sa[2 * p] + I * sa[2 * p + 1];
                        put(coef[24 + cq->src], p, s * S);
                    }
                }
            }
        }
    }
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Where an update finds t, c and Src of a part at a cell: the 28 stored   */
/* arrays, or (memory-light mode) the same formulas evaluated on the fly   */
/* from eps, the PML profiles and the raw sources.  Both modes call the    */
/* same coefficient functions with the same phase factors, so they agree   */
/* bit for bit.                                                            */
/* ---------------------------------------------------------------------- */
typedef struct {
    const double *tq, *cq, *srcq; /* stored mode (srcq NULL: no source) */
    int light;
    const double *eps, *sig_e, *sig_h, *S; /* light mode (S NULL: zero) */
    double complex ph, ph2;
    double omega, tau, h;
} csrc_t;

/* t, c and Src of part q at cell p of plane k; returns whether the part has
 * a source term. */
static int coef_at(const csrc_t *cs, int q, int k, long p, double *tr, double *ti,
                   double *cr, double *ci, double *sr, double *si)
{
    const comp_t *cm = &COMP[q];
    if (!cs->light) {
        *tr = cs->tq[2 * p]; *ti = cs->tq[2 * p + 1];
        *cr = cs->cq[2 * p]; *ci = cs->cq[2 * p + 1];
        if (!cs->srcq) return 0;
        *sr = cs->srcq[2 * p]; *si = cs->srcq[2 * p + 1];
        return 1;
    }
    double complex t, c, s;
    if (q < 6) {
        double sst = (cm->axis == 2) ? cs->sig_h[k] : 0.0;
        coef_h_ph(cs->ph2, cs->tau, cs->h, sst, &t, &c, &s);
    } else {
        double sg = cs->omega * cs->eps[2 * p + 1] + ((cm->axis == 2) ? cs->sig_e[k] : 0.0);
        coef_e_ph(cs->ph, cs->ph2, cs->tau, cs->h, cs->eps[2 * p], sg, &t, &c, &s);
    }
    *tr = creal(t); *ti = cimag(t);
    *cr = creal(c); *ci = cimag(c);
    if (cm->src < 0) return 0;
    double complex S = 0.0;
    if (cs->S) S = cs->S[2 * p] + I * cs->S[2 * p + 1];
    double complex v = s * S;
    *sr = creal(v); *si = cimag(v);
    return 1;
}

/* ---------------------------------------------------------------------- */
/* The 12 loop nests (Listings 1 and 2).                                   */
/* ---------------------------------------------------------------------- */

/* One component update over the whole domain: Eq. (3) (E) or Eq. (4) (H)
 * solved for the new value,
 *     F(p) <- t(p) F(p) + Src(p) + s c(p) D(p),
 * with D the difference of the driving component G = G1 + G2 (the sum of its
 * two split parts) along the part's axis: the backward difference
 * G(p) - G(p - e) for H, the forward difference G(p + e) - G(p) for E
 * (Fig. 3: the two fields depend on each other in opposite directions); a
 * neighbour outside the domain contributes 0, and s is the sign of that
 * derivative in the curl.  Real arithmetic with one complex product per
 * coefficient: D costs 6 flops (the two sums and their difference, real and
 * imaginary parts), t F and c D 6 each, combining them 2 and adding Src 2
 * more -- the 20 and 22 flops per update of the paper's count (Sec. III-A).
 * Real and imaginary parts are formed in locals and stored together. */
static void update_component(const grid_t *g, int q, double *F, const csrc_t *cs,
                             const double *G1, const double *G2)
{
    const comp_t *cm = &COMP[q];
    const int is_h = q < 6;
    const int dir = is_h ? -1 : +1;
    int k;
#pragma omp parallel for schedule(static)
    for (k = 0; k < g->nz; k++) {
        for (int j = 0; j < g->ny; j++) {
            for (int ii = 0; ii < g->nx; ii++) {
                long p = ((long)k * g->ny + j) * g->nx + ii;
                long ps = nbr(g, k, j, ii, cm->axis, dir);
                /* G at the cell and at its neighbour along the axis */
                double gr = G1[2 * p] + G2[2 * p];
                double gi = G1[2 * p + 1] + G2[2 * p + 1];
                double nr = 0.0, ni = 0.0;
                if (ps >= 0) {
                    nr = G1[2 * ps] + G2[2 * ps];
                    ni = G1[2 * ps + 1] + G2[2 * ps + 1];
                }
                double dr = is_h ? gr - nr : nr - gr;
                double di = is_h ? gi - ni : ni - gi;
                double fr = F[2 * p], fi = F[2 * p + 1];
                double tr, ti, cr, ci, sr = 0.0, si = 0.0;
                int has_src = coef_at(cs, q, k, p, &tr, &ti, &cr, &ci, &sr, &si);
                double tf_r = tr * fr - ti * fi, tf_i = tr * fi + ti * fr;
                double cd_r = cr * dr - ci * di, cd_i = cr * di + ci * dr;
                double new_r = cm->sign > 0 ? tf_r + cd_r : tf_r - cd_r;
                double new_i = cm->sign > 0 ? tf_i + cd_i : tf_i - cd_i;
                if (has_src) {
                    new_r = new_r + sr;
                    new_i = new_i + si;
                }
                F[2 * p] = new_r;
                F[2 * p + 1] = new_i;
            }
        }
    }
}

/* n THIIM iterations in place: each is the H half-step (6 loop nests, Eq. 4)
 * followed by the E half-step (6 loop nests, Eq. 3/5). */
int oracle_iterate(int nx, int ny, int nz, int bcx, int bcy,
                   const double *const *coef, double *const *F, int n)
{
    grid_t g = {nx, ny, nz, bcx, bcy};
    for (int it = 0; it < n; it++) {
        for (int half = 0; half < 2; half++) {
            for (int q = 6 * half; q < 6 * half + 6; q++) {
                const comp_t *cm = &COMP[q];
                const double *srcq = cm->src >= 0 ? coef[24 + cm->src] : NULL;
                csrc_t cs = {0};
                cs.tq = coef[q];
                cs.cq = coef[12 + q];
                cs.srcq = srcq;
                update_component(&g, q, F[q], &cs, F[cm->g1], F[cm->g2]);
            }
        }
    }
    return 0;
}

/* n THIIM iterations in memory-light mode: no coefficient arrays, t, c and
 * Src evaluated per cell from eps (2*N), the PML profiles (nz each) and the
 * raw sources (4 pointers S_Hx, S_Hy, S_Ex, S_Ey, 2*N each, or NULL).
 * Bit-identical to oracle_coeffs + oracle_iterate; about 40 B of inputs per
 * cell instead of 448. */
int oracle_iterate_light(int nx, int ny, int nz, int bcx, int bcy, const double *eps,
                         const double *sig_e, const double *sig_h,
                         const double *const *src, double omega, double tau, double h,
                         double *const *F, int n)
{
    grid_t g = {nx, ny, nz, bcx, bcy};
    long N = (long)nx * ny * nz;
    for (long p = 0; p < N; p++) {
        double ep = eps[2 * p], epp = eps[2 * p + 1];
        if (!(ep != 0.0) || !isfinite(ep) || !isfinite(epp)) return -1;
    }
    for (int it = 0; it < n; it++) {
        for (int half = 0; half < 2; half++) {
            for (int q = 6 * half; q < 6 * half + 6; q++) {
                const comp_t *cm = &COMP[q];
                csrc_t cs = {0};
                cs.light = 1;
                cs.eps = eps;
                cs.sig_e = sig_e;
                cs.sig_h = sig_h;
                cs.S = (cm->src >= 0 && src) ? src[cm->src] : NULL;
                cs.ph = cexp(I * (omega * tau));
                cs.ph2 = cexp(I * (omega * tau / 2.0));
                cs.omega = omega;
                cs.tau = tau;
                cs.h = h;
                update_component(&g, q, F[q], &cs, F[cm->g1], F[cm->g2]);
            }
        }
    }
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Transposed iteration (gradient support).                                */
/* ---------------------------------------------------------------------- */

/* Eq. (3)/(4) make one iteration an affine map x <- M x + c, and M is the
 * product M_E M_H of the H half-step (H parts rewritten from E) and the E
 * half-step (E parts rewritten from the new H), so M^T = M_H^T M_E^T.
 *
 * A half-step rewrites each of its six parts q as
 *     F_q(p) <- t_q(p) F_q(p) + s_q c_q(p) (G(p_hi) - G(p_lo)),
 * with G the sum of the two split parts of the driving component,
 * (p_hi, p_lo) = (p, p - e) for H (backward difference) and (p + e, p) for
 * E (forward difference); a neighbour outside the domain is a ghost that
 * contributes nothing.  Its transpose, written as a scatter: for every q and
 * p, with u = s_q c_q(p) L_q(p) taken from the value of L_q before it is
 * rescaled, add u to both split parts of the driving component at p_hi and
 * subtract it at p_lo; then L_q(p) <- t_q(p) L_q(p).  The scatter writes
 * only the other field's parts, so its order does not matter. */
static void transpose_half(const grid_t *g, int half, const double *const *coef,
                           double *const *L)
{
    for (int q = 6 * half; q < 6 * half + 6; q++) {
        const comp_t *cm = &COMP[q];
        const double *cq = coef[12 + q];
        for (int k = 0; k < g->nz; k++) {
            for (int j = 0; j < g->ny; j++) {
                for (int i = 0; i < g->nx; i++) {
                    long p = ((long)k * g->ny + j) * g->nx + i;
                    double complex c = cq[2 * p] + I * cq[2 * p + 1];
                    double complex l = L[q][2 * p] + I * L[q][2 * p + 1];
                    double complex u = (double)cm->sign * (c * l);
                    long hi, lo;
                    if (half == 0) {
                        hi = p;
                        lo = nbr(g, k, j, i, cm->axis, -1);
                    } else {
                        hi = nbr(g, k, j, i, cm->axis, +1);
                        lo = p;
                    }
                    const int parts[2] = {cm->g1, cm->g2};
                    for (int m = 0; m < 2; m++) {
                        double *G = L[parts[m]];
                        if (hi >= 0) {
                            G[2 * hi] += creal(u);
                            G[2 * hi + 1] += cimag(u);
                        }
                        if (lo >= 0) {
                            G[2 * lo] -= creal(u);
                            G[2 * lo + 1] -= cimag(u);
                        }
                    }
                }
            }
        }
    }
    for (int q = 6 * half; q < 6 * half + 6; q++) {
        const double *tq = coef[q];
        long N = (long)g->nx * g->ny * g->nz;
        for (long p = 0; p < N; p++) {
            double complex t = tq[2 * p] + I * tq[2 * p + 1];
            double complex l = L[q][2 * p] + I * L[q][2 * p + 1];
            put(L[q], p, t * l);
        }
    }
}

/* n transposed iterations in place: L <- M^T L + Gs (the E half-step's
 * transpose first, then the H half-step's), Gs = 12 arrays or NULL
 * entries for zero. */
int oracle_adjoint_iterate(int nx, int ny, int nz, int bcx, int bcy,
                           const double *const *coef, double *const *L,
                           const double *const *Gs, int n)
{
    grid_t g = {nx, ny, nz, bcx, bcy};
    long N = (long)nx * ny * nz;
    for (int it = 0; it < n; it++) {
        transpose_half(&g, 1, coef, L);
        transpose_half(&g, 0, coef, L);
        for (int q = 0; q < NCOMP; q++) {
            if (!Gs || !Gs[q]) continue;
            for (long p = 0; p < 2 * N; p++) L[q][p] += Gs[q][p];
        }
    }
    return 0;
}

/* Flop count of one component update as written in update_component. */
int oracle_flops_per_update(int has_src) { return has_src ? 22 : 20; }

void oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
