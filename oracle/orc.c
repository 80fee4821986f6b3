/*
 * Oracle: a plain, slow FP64 CPU implementation of one electromagnetic
 * particle-in-cell step on a patch-decomposed Yee grid.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no code, header or table with the HIP path.
 *
 * What the paper fixes and what it leaves open.  The paper (Beck, Frederiksen
 * and Derouillat, sections 3 and 3.1) describes the load-balancing problem and
 * the patch data structure (fields and super-particles of a sub-domain held in
 * small independent patches), but never writes down the PIC step itself.  The
 * step implemented here is therefore the standard explicit scheme, each piece
 * following its published method:
 *   - quadratic B-spline shape factors for gather and charge (Birdsall and
 *     Langdon, "Plasma Physics via Computer Simulation", ch. 8);
 *   - the relativistic Boris rotation (Boris 1970);
 *   - charge-conserving current deposition (Esirkepov 2001, Comput. Phys.
 *     Commun. 135, 144), written as the time integral of linearly
 *     interpolated shape products;
 *   - the Yee staggered-grid FDTD update (Yee 1966, IEEE TAP 14, 302), as a
 *     half B step, a full E step and a half B step;
 *   - first-order Silver-Mueller characteristic boundaries on the x faces,
 *     with an incident-field table driving the x = 0 face (the laser of the
 *     paper's LWFA runs, section 2.2);
 *   - a canonical per-patch re-binning rule (see orc_rebin) that fixes the
 *     patch occupancy and the slot of every particle bit for bit.
 *
 * Units: c = eps0 = e = m_e = 1; lengths in c/omega_r, time in 1/omega_r
 * (section 2.2 quotes resolutions in c/omega_0 and 1/omega_0).  Positions are
 * kept in cell units xi = x / dx, global, in FP64.
 *
 * Functions follow the step order: gather, Boris, move, deposit, boundary,
 * Maxwell, re-bin; then the options of the step's end: particle merging
 * (section 3.2) and the moving window (sections 2.1, 2.3), and the
 * sixth-order field solver (section 2.1).  Everything is plain loops in FP64.
 */
#define _DEFAULT_SOURCE
#include <math.h>
#include <stdint.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdlib.h>
#include <string.h>

#define ORC_NCOMP 9 /* Ex Ey Ez Bx By Bz Jx Jy Jz */

typedef struct {
    int ndim;         /* 2 or 3 */
    int n[3];         /* cells per axis (n[2] = 1 in 2-D) */
    double d[3];      /* cell size per axis */
    double dt;
    int patch[3];     /* patch size in cells per axis */
    int periodic[3];  /* 1 periodic; 0 open (x only): Silver-Mueller fields, absorbing particles */
    double q, m;      /* species charge and mass (electrons: -1, 1) */
} orc_desc;

typedef struct {
    orc_desc g;
    int fn[3];        /* nodes stored per axis: n (periodic) or n + 1 (open) */
    int np[3];        /* patches per axis */
    int npatch;
    int64_t fsize;
    double *F[ORC_NCOMP];
    int64_t npart;
    double *x[3], *u[3], *w;
    int64_t *id;
    int32_t *count;
    int64_t laser_steps;
    int laser_n1;     /* transverse nodes per table row (n[1] * n[2]) */
    double *laser_ey, *laser_ez;
    /* Gaussian lasers through x = 0 (see orc_add_laser): a0, omega0, w0, tau,
     * t0, x_focus, y_center, phase; polarisation 1 (Ey) or 2 (Ez) */
    int nlaser;
    double las[4][8];
    int las_pol[4];
    int64_t step;
    double U_last, K_last;
    int64_t removed;
    int morder;       /* spatial order of the field solver: 2 (Yee) or 6 */
    /* moving window along x (see orc_set_window) */
    int win;          /* 1: the window moves */
    int64_t win_start;/* completed steps before the window starts to move */
    double win_v;     /* window speed in units of c */
    int win_ppc[2];   /* injected particles per cell along x and y */
    double *win_dens; /* plasma density of global cell column c (the last entry beyond) */
    int64_t win_ncols;
    int64_t win_shift;/* shifts done so far (the window has moved win_shift * patch[0] cells) */
    int64_t next_id;  /* id of the next injected particle */
    /* particle merging (see orc_merge) */
    double **jbuf;    /* OpenMP build only: per-thread current arrays (3 per thread) */
    double **jpriv;   /* jbuf while the particle loop runs, else NULL */
    int jthreads;
    int merge_every;  /* merge after every merge_every-th step (0: never) */
    int merge_cmax, merge_iters;
    int64_t merged;   /* particles taken out by merging so far */
} orc_sim;

/* Staggering of Ex Ey Ez Bx By Bz (J shares E's): 1 = half a cell up. */
static const int STAG[6][3] = {
    {1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {0, 1, 1}, {1, 0, 1}, {1, 1, 0}};

static int stag_of(const orc_sim *s, int comp, int a)
{
    if (a >= s->g.ndim) return 0;
    return STAG[comp < 6 ? comp : comp - 6][a];
}

/* Map a node index on axis a to storage, or -1 when it lies outside an open
 * axis (values there read as zero, deposits there are dropped). */
static int64_t node_index(const orc_sim *s, int a, int64_t i, int stag)
{
    int n = s->g.n[a];
    if (a >= s->g.ndim) return 0;
    if (s->g.periodic[a]) {
        i %= n;
        if (i < 0) i += n;
        return i;
    }
    if (i < 0) return -1;
    if (stag ? i > n - 1 : i > n) return -1;
    return i;
}

static int64_t flat3(const orc_sim *s, int comp, int64_t i, int64_t j, int64_t k)
{
    int64_t a = node_index(s, 0, i, stag_of(s, comp, 0));
    int64_t b = node_index(s, 1, j, stag_of(s, comp, 1));
    int64_t c = node_index(s, 2, k, stag_of(s, comp, 2));
    if (a < 0 || b < 0 || c < 0) return -1;
    return a + (int64_t)s->fn[0] * (b + (int64_t)s->fn[1] * c);
}

static double fget(const orc_sim *s, int comp, int64_t i, int64_t j, int64_t k)
{
    int64_t f = flat3(s, comp, i, j, k);
    return f < 0 ? 0.0 : s->F[comp][f];
}

/* ---------------------------------------------------------------------- */
/* Quadratic B-spline shape (Birdsall-Langdon).                            */

/* S2(delta): 3/4 - d^2 for |d| <= 1/2; (3/2 - |d|)^2 / 2 for 1/2 <= |d| <= 3/2. */
double orc_s2(double dl)
{
    double a = fabs(dl);
    if (a <= 0.5) return 0.75 - a * a;
    if (a <= 1.5) return 0.5 * (1.5 - a) * (1.5 - a);
    return 0.0;
}

/* Nearest node and the three weights for a sample staggered by stag/2. */
void orc_shape(double xi, int stag, int64_t *i0, double w[3])
{
    double p = xi - 0.5 * stag;
    int64_t c = (int64_t)floor(p + 0.5);
    double dl = p - (double)c;
    *i0 = c;
    w[0] = 0.5 * (0.5 - dl) * (0.5 - dl);
    w[1] = 0.75 - dl * dl;
    w[2] = 0.5 * (0.5 + dl) * (0.5 + dl);
}

/* Field gather: F_c(x_p) = sum over the 3^ndim nearest nodes of the
 * component's own staggered grid of F * product of shape weights. */
void orc_gather(const orc_sim *s, const double xi[3], double EB[6])
{
    for (int c = 0; c < 6; ++c) {
        int64_t i0[3] = {0, 0, 0};
        double w[3][3];
        for (int a = 0; a < 3; ++a) {
            if (a < s->g.ndim) {
                orc_shape(xi[a], stag_of(s, c, a), &i0[a], w[a]);
            } else {
                w[a][0] = 0.0; w[a][1] = 1.0; w[a][2] = 0.0;
            }
        }
        double acc = 0.0;
        int kz0 = s->g.ndim == 3 ? -1 : 0, kz1 = s->g.ndim == 3 ? 1 : 0;
        for (int kz = kz0; kz <= kz1; ++kz)
            for (int ky = -1; ky <= 1; ++ky)
                for (int kx = -1; kx <= 1; ++kx)
                    acc += fget(s, c, i0[0] + kx, i0[1] + ky, i0[2] + kz)
                         * w[0][kx + 1] * w[1][ky + 1] * w[2][kz + 1];
        EB[c] = acc;
    }
}

/* ---------------------------------------------------------------------- */
/* Relativistic Boris push (Boris 1970): half electric kick, magnetic
 * rotation, half electric kick.  u = p / (m c). */
void orc_boris(double u[3], const double E[3], const double B[3],
               double q, double m, double dt)
{
    double eps = q * dt / (2.0 * m);
    double um[3], t[3], sv[3], up[3], uq[3];
    for (int a = 0; a < 3; ++a) um[a] = u[a] + eps * E[a];
    double g = sqrt(1.0 + um[0] * um[0] + um[1] * um[1] + um[2] * um[2]);
    for (int a = 0; a < 3; ++a) t[a] = eps * B[a] / g;
    double t2 = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
    for (int a = 0; a < 3; ++a) sv[a] = 2.0 * t[a] / (1.0 + t2);
    /* u' = u- + u- x t */
    up[0] = um[0] + (um[1] * t[2] - um[2] * t[1]);
    up[1] = um[1] + (um[2] * t[0] - um[0] * t[2]);
    up[2] = um[2] + (um[0] * t[1] - um[1] * t[0]);
    /* u+ = u- + u' x s */
    uq[0] = um[0] + (up[1] * sv[2] - up[2] * sv[1]);
    uq[1] = um[1] + (up[2] * sv[0] - up[0] * sv[2]);
    uq[2] = um[2] + (up[0] * sv[1] - up[1] * sv[0]);
    for (int a = 0; a < 3; ++a) u[a] = uq[a] + eps * E[a];
}

/* ---------------------------------------------------------------------- */
/* Esirkepov charge-conserving deposition.
 *
 * Per axis, i0 is the nearest primal node of the old position; on the
 * five-node window i0-2..i0+2, S0 holds the old weights and S1 the new ones
 * (shifted by the change of nearest node), DS = S1 - S0.  The W factors are
 * the time integrals over the step of the products of linearly interpolated
 * shape factors; the current along an axis is the running sum of -q w
 * (dx/dt) W along that axis.  In 2-D the out-of-plane current is
 * q w v_z W_z with W_z the time-averaged shape product. */
static void window_weights(double x0, double x1, int64_t *i0, double S0[5], double DS[5])
{
    int64_t c0, c1;
    double w0[3], w1[3], S1[5];
    orc_shape(x0, 0, &c0, w0);
    orc_shape(x1, 0, &c1, w1);
    int64_t sh = c1 - c0; /* -1, 0 or +1 when the move is under one cell */
    for (int k = 0; k < 5; ++k) { S0[k] = 0.0; S1[k] = 0.0; }
    for (int k = -1; k <= 1; ++k) S0[k + 2] = w0[k + 1];
    for (int k = -1; k <= 1; ++k) {
        int64_t slot = k + sh + 2;
        if (slot >= 0 && slot < 5) S1[slot] = w1[k + 1];
    }
    for (int k = 0; k < 5; ++k) DS[k] = S1[k] - S0[k];
    *i0 = c0;
}

static void jadd(orc_sim *s, int comp, int64_t i, int64_t j, int64_t k, double v)
{
    int64_t f = flat3(s, comp, i, j, k);
    if (f < 0) return;
#ifdef _OPENMP
    if (s->jpriv) {
        s->jpriv[3 * omp_get_thread_num() + comp - 6][f] += v;
        return;
    }
#endif
    s->F[comp][f] += v;
}

/* Host threads of the particle loop (OpenMP build; 1 otherwise). */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_deposit(orc_sim *s, const double xa[3], const double xb[3], double w, double vz)
{
    const int nd = s->g.ndim;
    const double q = s->g.q, dt = s->g.dt;
    int64_t i0[3] = {0, 0, 0};
    double S0[3][5], DS[3][5];
    for (int a = 0; a < nd; ++a) window_weights(xa[a], xb[a], &i0[a], S0[a], DS[a]);
    if (nd == 2) {
        double Wx[5][5], Wy[5][5], Wz[5][5];
        for (int i = 0; i < 5; ++i)
            for (int j = 0; j < 5; ++j) {
                Wx[i][j] = DS[0][i] * (S0[1][j] + 0.5 * DS[1][j]);
                Wy[i][j] = DS[1][j] * (S0[0][i] + 0.5 * DS[0][i]);
                Wz[i][j] = S0[0][i] * S0[1][j] + 0.5 * DS[0][i] * S0[1][j]
                         + 0.5 * S0[0][i] * DS[1][j] + DS[0][i] * DS[1][j] / 3.0;
            }
        double cx = -q * w * s->g.d[0] / dt, cy = -q * w * s->g.d[1] / dt;
        for (int j = 0; j < 5; ++j) {
            double acc = 0.0;
            for (int i = 0; i < 4; ++i) { /* dual node i0 + (i - 2) + 1/2 */
                acc += cx * Wx[i][j];
                jadd(s, 6, i0[0] + i - 2, i0[1] + j - 2, 0, acc);
            }
        }
        for (int i = 0; i < 5; ++i) {
            double acc = 0.0;
            for (int j = 0; j < 4; ++j) {
                acc += cy * Wy[i][j];
                jadd(s, 7, i0[0] + i - 2, i0[1] + j - 2, 0, acc);
            }
        }
        for (int i = 0; i < 5; ++i)
            for (int j = 0; j < 5; ++j)
                jadd(s, 8, i0[0] + i - 2, i0[1] + j - 2, 0, q * w * vz * Wz[i][j]);
        return;
    }
    /* 3-D: W_a = DS_a (S0_b S0_c + DS_b S0_c / 2 + S0_b DS_c / 2 + DS_b DS_c / 3) */
    for (int a = 0; a < 3; ++a) {
        int b = (a + 1) % 3, c = (a + 2) % 3;
        double coef = -q * w * s->g.d[a] / dt;
        for (int kb = 0; kb < 5; ++kb)
            for (int kc = 0; kc < 5; ++kc) {
                double tr = S0[b][kb] * S0[c][kc] + 0.5 * DS[b][kb] * S0[c][kc]
                          + 0.5 * S0[b][kb] * DS[c][kc] + DS[b][kb] * DS[c][kc] / 3.0;
                double acc = 0.0;
                for (int ka = 0; ka < 4; ++ka) {
                    acc += coef * DS[a][ka] * tr;
                    int64_t idx[3];
                    idx[a] = i0[a] + ka - 2;
                    idx[b] = i0[b] + kb - 2;
                    idx[c] = i0[c] + kc - 2;
                    jadd(s, 6 + a, idx[0], idx[1], idx[2], acc);
                }
            }
    }
}

/* ---------------------------------------------------------------------- */
/* Yee update.  E updates use backward differences of B, B updates forward
 * differences of E.  On an open x axis the E update at x = 0 and x = L
 * needs By and Bz half a cell outside the domain; they come from the
 * first-order characteristic (Silver-Mueller) condition written at the face
 * and at time n + 1/2, combined with the 1-D part of the E update:
 *   x = 0 (incoming E_inc):  Ey + Bz = 2 Ey_inc,  Ez - By = 2 Ez_inc
 *   x = L (outflow):         Ey - Bz = 0,         Ez + By = 0
 * With r = dt/dx, B_1 the first interior dual B and E^n the face E:
 *   Bz_ghost(0) = (4 Ey_inc - 2 Ey^n - (1 - r) Bz_1) / (1 + r)
 *   By_ghost(0) = (2 Ez^n - (1 - r) By_1 - 4 Ez_inc) / (1 + r)
 *   Bz_ghost(L) = (2 Ey^n - (1 - r) Bz_1) / (1 + r)
 *   By_ghost(L) = (-2 Ez^n - (1 - r) By_1) / (1 + r)
 * (transverse derivative terms are left out of the condition). */

/* Sixth-order staggered first difference (the high-order field solver the
 * paper mentions for one of its comparison codes, section 2; it gives no
 * coefficients).  The derivative at the midpoint of nodes i and i + 1 is
 * sum_m c_m (f(i + m) - f(i + 1 - m)) / h, m = 1..3; matching the Taylor
 * series of f at the midpoint, c1 + 3 c2 + 5 c3 = 1 and c1 + 3^3 c2 + 5^3 c3 =
 * c1 + 3^5 c2 + 5^5 c3 = 0, whose solution is below. */
static const double C6[3] = {75.0 / 64.0, -25.0 / 384.0, 3.0 / 640.0};

/* Difference of component c along axis a at the half point after node
 * (i, j, k) (fwd = 1: between the node and the next one) or before it
 * (fwd = 0: between the previous node and this one), not yet divided by the
 * cell size.  Order 2: the two neighbours; order 6: the three pairs above. */
static double dstag(const orc_sim *s, int c, int a, int64_t i, int64_t j, int64_t k, int fwd)
{
    int64_t p[3] = {i, j, k};
    if (!fwd) p[a] -= 1;            /* midpoint between p and p + 1 along a */
    if (s->morder == 2) {
        int64_t q[3] = {p[0], p[1], p[2]};
        q[a] += 1;
        return fget(s, c, q[0], q[1], q[2]) - fget(s, c, p[0], p[1], p[2]);
    }
    double acc = 0.0;
    for (int m = 1; m <= 3; ++m) {
        int64_t hi[3] = {p[0], p[1], p[2]}, lo[3] = {p[0], p[1], p[2]};
        hi[a] += m;
        lo[a] += 1 - m;
        acc += C6[m - 1] * (fget(s, c, hi[0], hi[1], hi[2]) - fget(s, c, lo[0], lo[1], lo[2]));
    }
    return acc;
}

/* Field solver of order 6 (periodic axes only; the Yee update below covers
 * order 2 with its open faces): the same three sweeps with dstag. */
static void b_half_hi(orc_sim *s)
{
    const double h = 0.5 * s->g.dt;
    const double ix = 1.0 / s->g.d[0], iy = 1.0 / s->g.d[1];
    const double iz = s->g.ndim == 3 ? 1.0 / s->g.d[2] : 0.0;
    for (int64_t k = 0; k < s->fn[2]; ++k)
        for (int64_t j = 0; j < s->fn[1]; ++j)
            for (int64_t i = 0; i < s->fn[0]; ++i) {
                const int64_t f = flat3(s, 3, i, j, k);
                double bx = dstag(s, 2, 1, i, j, k, 1) * iy, by = -dstag(s, 2, 0, i, j, k, 1) * ix;
                double bz = dstag(s, 1, 0, i, j, k, 1) * ix - dstag(s, 0, 1, i, j, k, 1) * iy;
                if (s->g.ndim == 3) {
                    bx -= dstag(s, 1, 2, i, j, k, 1) * iz;
                    by += dstag(s, 0, 2, i, j, k, 1) * iz;
                }
                s->F[3][f] -= h * bx;
                s->F[4][f] -= h * by;
                s->F[5][f] -= h * bz;
            }
}

static void maxwell_hi(orc_sim *s)
{
    const double dt = s->g.dt;
    const double ix = 1.0 / s->g.d[0], iy = 1.0 / s->g.d[1];
    const double iz = s->g.ndim == 3 ? 1.0 / s->g.d[2] : 0.0;
    b_half_hi(s);
    for (int64_t k = 0; k < s->fn[2]; ++k)
        for (int64_t j = 0; j < s->fn[1]; ++j)
            for (int64_t i = 0; i < s->fn[0]; ++i) {
                const int64_t f = flat3(s, 0, i, j, k);
                /* Ex += dt (dBz/dy - dBy/dz - Jx), Ey += dt (dBx/dz - dBz/dx - Jy),
                   Ez += dt (dBy/dx - dBx/dy - Jz); backward differences */
                double ex = dstag(s, 5, 1, i, j, k, 0) * iy, ey = -dstag(s, 5, 0, i, j, k, 0) * ix;
                double ez = dstag(s, 4, 0, i, j, k, 0) * ix - dstag(s, 3, 1, i, j, k, 0) * iy;
                if (s->g.ndim == 3) {
                    ex -= dstag(s, 4, 2, i, j, k, 0) * iz;
                    ey += dstag(s, 3, 2, i, j, k, 0) * iz;
                }
                s->F[0][f] += dt * (ex - s->F[6][f]);
                s->F[1][f] += dt * (ey - s->F[7][f]);
                s->F[2][f] += dt * (ez - s->F[8][f]);
            }
    b_half_hi(s);
}

/* Choose the field solver order: 2 (Yee, default) or 6 (all axes periodic).
 * Returns 0, or -1 for an unsupported request. */
int orc_set_maxwell_order(orc_sim *s, int order)
{
    if (order == 2) { s->morder = 2; return 0; }
    if (order != 6) return -1;
    for (int a = 0; a < s->g.ndim; ++a)
        if (!s->g.periodic[a]) return -1;
    s->morder = 6;
    return 0;
}

static void b_half(orc_sim *s)
{
    const double h = 0.5 * s->g.dt;
    const double ix = 1.0 / s->g.d[0], iy = 1.0 / s->g.d[1];
    const double iz = s->g.ndim == 3 ? 1.0 / s->g.d[2] : 0.0;
    const int nz = s->fn[2];
    for (int64_t k = 0; k < nz; ++k)
        for (int64_t j = 0; j < s->fn[1]; ++j)
            for (int64_t i = 0; i < s->fn[0]; ++i) {
                int64_t f;
                /* Bx -= h (dEz/dy - dEy/dz) */
                if ((f = flat3(s, 3, i, j, k)) >= 0)
                    s->F[3][f] -= h * ((fget(s, 2, i, j + 1, k) - fget(s, 2, i, j, k)) * iy
                                     - (fget(s, 1, i, j, k + 1) - fget(s, 1, i, j, k)) * iz);
                /* By -= h (dEx/dz - dEz/dx) */
                if ((f = flat3(s, 4, i, j, k)) >= 0)
                    s->F[4][f] -= h * ((fget(s, 0, i, j, k + 1) - fget(s, 0, i, j, k)) * iz
                                     - (fget(s, 2, i + 1, j, k) - fget(s, 2, i, j, k)) * ix);
                /* Bz -= h (dEy/dx - dEx/dy) */
                if ((f = flat3(s, 5, i, j, k)) >= 0)
                    s->F[5][f] -= h * ((fget(s, 1, i + 1, j, k) - fget(s, 1, i, j, k)) * ix
                                     - (fget(s, 0, i, j + 1, k) - fget(s, 0, i, j, k)) * iy);
            }
}

static double laser_row(const orc_sim *s, const double *tab, int64_t j, int64_t k)
{
    if (!tab || s->step >= s->laser_steps) return 0.0;
    return tab[s->step * s->laser_n1 + j + (int64_t)s->g.n[1] * k];
}

/* Incident field of a y- or z-polarised 2-D paraxial Gaussian beam at the
 * x = 0 face, time t, transverse position y (the laser of the LWFA runs,
 * section 2.2: a focused Gaussian pulse of amplitude a0).  Waist w0 (1/e
 * radius of the field) in the plane x = x_focus, Rayleigh length
 * x_R = omega0 w0^2 / 2 (c = 1).  At distance xi = 0 - x_focus from the
 * focus the beam has radius w = w0 sqrt(1 + (xi / x_R)^2), wavefront
 * curvature 1/R = xi / (xi^2 + x_R^2) and Gouy phase atan(xi / x_R) / 2 (half
 * the 3-D value: one transverse dimension), and its amplitude falls as
 * sqrt(w0 / w) (power per unit length kept).  Temporal envelope
 * exp(-2 ln 2 (t - t0)^2 / tau^2): tau is the FWHM of the intensity.  Peak
 * field a0 omega0 (units m_e c omega_r / e). */
static double gauss_beam(const double *L, double t, double y)
{
    const double a0 = L[0], om = L[1], w0 = L[2], tau = L[3], t0 = L[4], xf = L[5], yc = L[6], ph = L[7];
    const double xr = 0.5 * om * w0 * w0;
    const double xi = 0.0 - xf;
    const double w = w0 * sqrt(1.0 + (xi / xr) * (xi / xr));
    const double inv_r = xi / (xi * xi + xr * xr);
    const double gouy = 0.5 * atan2(xi, xr);
    const double dy = y - yc;
    const double amp = a0 * om * sqrt(w0 / w);
    const double env = exp(-2.0 * log(2.0) * ((t - t0) / tau) * ((t - t0) / tau));
    const double tr = exp(-(dy / w) * (dy / w));
    return amp * env * tr * sin(om * (t - t0) - 0.5 * om * dy * dy * inv_r + gouy + ph);
}

/* Incident Ey (comp 1, on dual y positions (j + 1/2) dy) or Ez (comp 2, on
 * primal y positions j dy) at the x = 0 face during the step in flight
 * (time (step + 1/2) dt): the table row plus every Gaussian laser. */
static double incident(const orc_sim *s, int comp, int64_t j, int64_t k)
{
    double v = laser_row(s, comp == 1 ? s->laser_ey : s->laser_ez, j, k);
    const double t = ((double)s->step + 0.5) * s->g.dt;
    const double y = ((double)j + (comp == 1 ? 0.5 : 0.0)) * s->g.d[1];
    for (int l = 0; l < s->nlaser; ++l)
        if (s->las_pol[l] == comp) v += gauss_beam(s->las[l], t, y);
    return v;
}

/* Add a Gaussian laser driving the open x = 0 face (2-D): parameters as in
 * gauss_beam, pol 1 (Ey) or 2 (Ez).  Returns 0, or -1 for an unsupported
 * request (3-D, periodic x, more than four lasers, bad values). */
int orc_add_laser(orc_sim *s, double a0, double omega0, double w0, double tau, double t0,
                  double x_focus, double y_center, double phase, int pol)
{
    if (s->g.ndim != 2 || s->g.periodic[0] || s->nlaser >= 4) return -1;
    if (!(omega0 > 0.0 && w0 > 0.0 && tau > 0.0 && a0 >= 0.0) || (pol != 1 && pol != 2)) return -1;
    double *L = s->las[s->nlaser];
    L[0] = a0; L[1] = omega0; L[2] = w0; L[3] = tau; L[4] = t0; L[5] = x_focus; L[6] = y_center; L[7] = phase;
    s->las_pol[s->nlaser++] = pol;
    return 0;
}

double orc_gauss_beam(double a0, double omega0, double w0, double tau, double t0, double x_focus,
                      double y_center, double phase, double t, double y)
{
    const double L[8] = {a0, omega0, w0, tau, t0, x_focus, y_center, phase};
    return gauss_beam(L, t, y);
}

void orc_maxwell(orc_sim *s)
{
    if (s->morder == 6) {
        maxwell_hi(s);
        return;
    }
    const double dt = s->g.dt;
    const double ix = 1.0 / s->g.d[0], iy = 1.0 / s->g.d[1];
    const double iz = s->g.ndim == 3 ? 1.0 / s->g.d[2] : 0.0;
    const int nx = s->g.n[0], nz = s->fn[2];
    const int64_t ntr = (int64_t)s->fn[1] * nz;

    b_half(s);

    /* ghost By, Bz half a cell outside each open x face, at time n + 1/2 */
    double *gby0 = NULL, *gbz0 = NULL, *gby1 = NULL, *gbz1 = NULL;
    if (!s->g.periodic[0]) {
        const double r = dt * ix;
        gby0 = calloc(ntr, sizeof(double)); gbz0 = calloc(ntr, sizeof(double));
        gby1 = calloc(ntr, sizeof(double)); gbz1 = calloc(ntr, sizeof(double));
        for (int64_t k = 0; k < nz; ++k)
            for (int64_t j = 0; j < s->fn[1]; ++j) {
                int64_t t = j + s->fn[1] * k;
                double eyi = incident(s, 1, j, k);
                double ezi = incident(s, 2, j, k);
                gbz0[t] = (4.0 * eyi - 2.0 * fget(s, 1, 0, j, k) - (1.0 - r) * fget(s, 5, 0, j, k)) / (1.0 + r);
                gby0[t] = (2.0 * fget(s, 2, 0, j, k) - (1.0 - r) * fget(s, 4, 0, j, k) - 4.0 * ezi) / (1.0 + r);
                gbz1[t] = (2.0 * fget(s, 1, nx, j, k) - (1.0 - r) * fget(s, 5, nx - 1, j, k)) / (1.0 + r);
                gby1[t] = (-2.0 * fget(s, 2, nx, j, k) - (1.0 - r) * fget(s, 4, nx - 1, j, k)) / (1.0 + r);
            }
    }
    /* B accessor that supplies the ghosts for the dual-x components */
#define BGET(c, i, j, k) ( (!s->g.periodic[0] && ((c) == 4 || (c) == 5) && ((i) < 0 || (i) > nx - 1)) \
        ? ((i) < 0 ? ((c) == 4 ? gby0 : gbz0)[(j) + s->fn[1] * (k)]                                  \
                   : ((c) == 4 ? gby1 : gbz1)[(j) + s->fn[1] * (k)])                                 \
        : fget(s, (c), (i), (j), (k)) )

    for (int64_t k = 0; k < nz; ++k)
        for (int64_t j = 0; j < s->fn[1]; ++j)
            for (int64_t i = 0; i < s->fn[0]; ++i) {
                int64_t f;
                int64_t km = k - 1;
                /* Ex += dt (dBz/dy - dBy/dz - Jx) */
                if ((f = flat3(s, 0, i, j, k)) >= 0)
                    s->F[0][f] += dt * ((BGET(5, i, j, k) - BGET(5, i, j - 1, k)) * iy
                                      - (s->g.ndim == 3 ? (BGET(4, i, j, k) - BGET(4, i, j, km)) * iz : 0.0)
                                      - s->F[6][f]);
                /* Ey += dt (dBx/dz - dBz/dx - Jy) */
                if ((f = flat3(s, 1, i, j, k)) >= 0)
                    s->F[1][f] += dt * ((s->g.ndim == 3 ? (BGET(3, i, j, k) - BGET(3, i, j, km)) * iz : 0.0)
                                      - (BGET(5, i, j, k) - BGET(5, i - 1, j, k)) * ix
                                      - s->F[7][f]);
                /* Ez += dt (dBy/dx - dBx/dy - Jz) */
                if ((f = flat3(s, 2, i, j, k)) >= 0)
                    s->F[2][f] += dt * ((BGET(4, i, j, k) - BGET(4, i - 1, j, k)) * ix
                                      - (BGET(3, i, j, k) - BGET(3, i, j - 1, k)) * iy
                                      - s->F[8][f]);
            }
#undef BGET
    free(gby0); free(gbz0); free(gby1); free(gbz1);

    b_half(s);
}

/* ---------------------------------------------------------------------- */
/* Canonical re-binning.
 *
 * Patch P holds slots 0..n-1.  Lv are the slots whose particle leaves P
 * (or is removed), L = |Lv|; Ar are the particles arriving at P ordered by
 * (source patch id, source slot); n' = n - L + A.  H are the leaver slots
 * below n' (ascending), T the stayer slots in [n', n) (ascending).  The
 * fill sequence F = Ar followed by T goes into H in order, and what is left
 * of F goes to slots n, n+1, ...  Stayers below n' that are not holes keep
 * their slots.
 *
 * count[p] old occupancy; dest[k] for every old particle k (flat,
 * patch-major order) is its new patch id, or -1 when removed.  On return
 * newcount[q] is the new occupancy and src[k'] gives, for every new flat
 * index k', the old flat index of the particle placed there. */
void orc_rebin(int npatch, const int32_t *count, const int32_t *dest,
               int32_t *newcount, int64_t *src)
{
    int64_t *off = malloc(sizeof(int64_t) * (npatch + 1));
    int64_t *arr_n = calloc(npatch, sizeof(int64_t));
    off[0] = 0;
    for (int p = 0; p < npatch; ++p) off[p + 1] = off[p] + count[p];
    int64_t N = off[npatch];
    /* arrivals per destination, in (source patch, source slot) order */
    for (int p = 0; p < npatch; ++p)
        for (int64_t k = off[p]; k < off[p + 1]; ++k)
            if (dest[k] >= 0 && dest[k] != p) arr_n[dest[k]]++;
    int64_t *arr_off = malloc(sizeof(int64_t) * (npatch + 1));
    arr_off[0] = 0;
    for (int p = 0; p < npatch; ++p) arr_off[p + 1] = arr_off[p] + arr_n[p];
    int64_t *arr = malloc(sizeof(int64_t) * (arr_off[npatch] + 1));
    int64_t *fillpos = calloc(npatch, sizeof(int64_t));
    for (int p = 0; p < npatch; ++p)
        for (int64_t k = off[p]; k < off[p + 1]; ++k)
            if (dest[k] >= 0 && dest[k] != p) {
                int q = dest[k];
                arr[arr_off[q] + fillpos[q]++] = k;
            }
    (void)N;
    int64_t *newoff = malloc(sizeof(int64_t) * (npatch + 1));
    newoff[0] = 0;
    for (int q = 0; q < npatch; ++q) {
        int64_t n = count[q], L = 0;
        for (int64_t sl = 0; sl < n; ++sl)
            if (dest[off[q] + sl] != q) ++L;
        int64_t A = arr_n[q];
        newcount[q] = (int32_t)(n - L + A);
        newoff[q + 1] = newoff[q] + newcount[q];
    }
    for (int q = 0; q < npatch; ++q) {
        int64_t n = count[q], np = newcount[q], A = arr_n[q];
        int64_t *slot_src = src + newoff[q];
        /* H: leaver slots below n'; T: stayer slots in [n', n) */
        int64_t *H = malloc(sizeof(int64_t) * (n + 1));
        int64_t *T = malloc(sizeof(int64_t) * (n + 1));
        int64_t nh = 0, nt = 0;
        for (int64_t sl = 0; sl < n; ++sl) {
            int stays = dest[off[q] + sl] == q;
            if (!stays && sl < np) H[nh++] = sl;
            if (stays && sl >= np) T[nt++] = sl;
            if (stays && sl < np) slot_src[sl] = off[q] + sl;
        }
        /* F = Ar ++ T */
        int64_t nf = A + nt;
        for (int64_t f = 0; f < nf; ++f) {
            int64_t from = f < A ? arr[arr_off[q] + f] : off[q] + T[f - A];
            int64_t to = f < nh ? H[f] : n + (f - nh);
            slot_src[to] = from;
        }
        free(H);
        free(T);
    }
    free(off); free(arr_n); free(arr_off); free(arr); free(fillpos); free(newoff);
}

/* ---------------------------------------------------------------------- */
/* Simulation object.                                                      */

orc_sim *orc_create(const orc_desc *d)
{
    if (d->ndim != 2 && d->ndim != 3) return NULL;
    orc_sim *s = calloc(1, sizeof(orc_sim));
    s->g = *d;
    s->morder = 2;
    if (s->g.ndim == 2) { s->g.n[2] = 1; s->g.patch[2] = 1; s->g.periodic[2] = 1; s->g.d[2] = 1.0; }
    for (int a = 0; a < 3; ++a) {
        if (s->g.n[a] <= 0 || s->g.patch[a] <= 0 || s->g.n[a] % s->g.patch[a]) { free(s); return NULL; }
        if (a > 0 && !s->g.periodic[a]) { free(s); return NULL; } /* open faces only on x */
        s->fn[a] = s->g.periodic[a] ? s->g.n[a] : s->g.n[a] + 1;
        if (a >= s->g.ndim) s->fn[a] = 1;
        s->np[a] = s->g.n[a] / s->g.patch[a];
    }
    s->npatch = s->np[0] * s->np[1] * s->np[2];
    s->fsize = (int64_t)s->fn[0] * s->fn[1] * s->fn[2];
    for (int c = 0; c < ORC_NCOMP; ++c) s->F[c] = calloc(s->fsize, sizeof(double));
    s->count = calloc(s->npatch, sizeof(int32_t));
    s->laser_n1 = s->g.n[1] * (s->g.ndim == 3 ? s->g.n[2] : 1);
    return s;
}

static void free_particles(orc_sim *s)
{
    for (int a = 0; a < 3; ++a) { free(s->x[a]); free(s->u[a]); s->x[a] = s->u[a] = NULL; }
    free(s->w); free(s->id); s->w = NULL; s->id = NULL;
}

void orc_destroy(orc_sim *s)
{
    if (!s) return;
    for (int c = 0; c < ORC_NCOMP; ++c) free(s->F[c]);
    free_particles(s);
    free(s->count);
    free(s->laser_ey); free(s->laser_ez);
    free(s->win_dens);
    if (s->jbuf)
        for (int t = 0; t < 3 * s->jthreads; ++t) free(s->jbuf[t]);
    free(s->jbuf);
    free(s);
}

int64_t orc_fsize(const orc_sim *s) { return s->fsize; }
int orc_npatch(const orc_sim *s) { return s->npatch; }
int64_t orc_npart(const orc_sim *s) { return s->npart; }
int64_t orc_step_index(const orc_sim *s) { return s->step; }
int64_t orc_removed(const orc_sim *s) { return s->removed; }
void orc_set_step(orc_sim *s, int64_t n) { s->step = n; }

/* Patch of a position: floor of the cell coordinate divided by the patch
 * size, row-major with x fastest. */
static int patch_of(const orc_sim *s, const double xi[3])
{
    int pc[3] = {0, 0, 0};
    for (int a = 0; a < s->g.ndim; ++a) {
        int64_t c = (int64_t)floor(xi[a]);
        if (c < 0) c = 0;
        if (c > s->g.n[a] - 1) c = s->g.n[a] - 1;
        pc[a] = (int)(c / s->g.patch[a]);
    }
    return pc[0] + s->np[0] * (pc[1] + s->np[1] * pc[2]);
}

int orc_patch_of(const orc_sim *s, const double xi[3]) { return patch_of(s, xi); }

/* Load particles given in id order; the initial binning is the re-binning
 * rule applied from empty patches, which keeps id order inside a patch. */
int orc_set_particles(orc_sim *s, int64_t n, const double *const xs[3],
                      const double *const us[3], const double *w)
{
    for (int64_t k = 0; k < n; ++k)
        for (int a = 0; a < s->g.ndim; ++a)
            if (!(xs[a][k] >= 0.0 && xs[a][k] < (double)s->g.n[a])) return -1;
    free_particles(s);
    s->npart = n;
    for (int a = 0; a < 3; ++a) {
        s->x[a] = malloc(sizeof(double) * (n + 1));
        s->u[a] = malloc(sizeof(double) * (n + 1));
    }
    s->w = malloc(sizeof(double) * (n + 1));
    s->id = malloc(sizeof(int64_t) * (n + 1));
    memset(s->count, 0, sizeof(int32_t) * s->npatch);
    int32_t *pid = malloc(sizeof(int32_t) * (n + 1));
    for (int64_t k = 0; k < n; ++k) {
        double xi[3] = {xs[0][k], xs[1][k], s->g.ndim == 3 ? xs[2][k] : 0.0};
        pid[k] = patch_of(s, xi);
        s->count[pid[k]]++;
    }
    int64_t *pos = malloc(sizeof(int64_t) * (s->npatch + 1));
    pos[0] = 0;
    for (int p = 0; p < s->npatch; ++p) pos[p + 1] = pos[p] + s->count[p];
    for (int64_t k = 0; k < n; ++k) {
        int64_t t = pos[pid[k]]++;
        for (int a = 0; a < 3; ++a) {
            s->x[a][t] = (a < s->g.ndim) ? xs[a][k] : 0.0;
            s->u[a][t] = us[a][k];
        }
        s->w[t] = w[k];
        s->id[t] = k;
    }
    free(pos);
    free(pid);
    s->next_id = n;
    return 0;
}

/* ---- particle loading from a species description ---------------------
 *
 * Random numbers: SplitMix64 (Steele, Lea and Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014).  The generator adds the
 * odd constant gamma = 0x9E3779B97F4A7C15 to its state and returns the state
 * through two xor-shift-multiply rounds and a final xor-shift, so output n of
 * the generator seeded with s depends only on s + (n + 1) gamma: any draw is
 * reached directly from its counter.  Draw d (< 8) of particle g (the
 * particle's index in generation order, < 2^41) in stream r uses counter
 * r 2^44 + 8 g + d; a uniform double is the top 53 bits times 2^-53.
 * Stream 0: positions, stream 1: momenta. */
uint64_t orc_splitmix64(uint64_t seed, uint64_t n)
{
    uint64_t z = seed + (n + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static double draw01(uint64_t seed, uint64_t stream, int64_t g, int d)
{
    const uint64_t c = (stream << 44) + ((uint64_t)g << 3) + (uint64_t)d;
    return (double)(orc_splitmix64(seed, c) >> 11) * 0x1.0p-53;
}

/* Species description: profile 0 uniform n0; 1 vacuum below x0 = p[0], a
 * linear ramp from 0 at x0 to n0 at x1 = p[1], then n0 (x0 on a cell face);
 * 2 n0 (1 + p[0] cos(2 pi x / L_x)) with a sphere of centre (p[1], p[2],
 * p[3]) and radius p[4] at p[5] n0 (evaluated at cell centres).  loading 0:
 * ppc particles in every cell where the density is positive (profile 1:
 * cells at or beyond x0), weight n(x) / ppc at the particle's position
 * (profile 1) or the cell centre; loading 1: round(ppc n / n0) particles in a
 * cell, weight n0 / ppc.  Lengths in c/omega_r.  temperature = kT / (m c^2):
 * every momentum component Gaussian with sigma = sqrt(temperature) (Box-
 * Muller on draws 0, 1 and 2, 3 of stream 1); 0 gives a cold species.
 * Particles are made cell by cell in row-major order (x fastest), k = 0 ..
 * count - 1 in a cell; that order is the id order.  A position is the cell
 * index plus a uniform draw (draw a of stream 0 on axis a), kept below the
 * cell's upper face. */
typedef struct {
    int profile, loading, ppc;
    double n0, p[6], temperature;
    uint64_t seed;
} orc_species;

static double density_at(const orc_sim *s, const orc_species *sp, const double xc[3])
{
    if (sp->profile == 1) {
        const double X0 = sp->p[0] / s->g.d[0], X1 = sp->p[1] / s->g.d[0];
        if (xc[0] < X0) return 0.0;
        if (X1 <= X0 || xc[0] >= X1) return sp->n0;
        return sp->n0 * ((xc[0] - X0) / (X1 - X0));
    }
    if (sp->profile == 2) {
        double r2 = 0.0;
        for (int a = 0; a < s->g.ndim; ++a) {
            const double dd = xc[a] * s->g.d[a] - sp->p[1 + a];
            r2 += dd * dd;
        }
        if (r2 <= sp->p[4] * sp->p[4]) return sp->p[5] * sp->n0;
        return sp->n0 * (1.0 + sp->p[0] * cos(2.0 * M_PI * xc[0] / (double)s->g.n[0]));
    }
    return sp->n0;
}

static int cell_count(const orc_sim *s, const orc_species *sp, const int64_t c[3])
{
    double xc[3] = {(double)c[0] + 0.5, (double)c[1] + 0.5, (double)c[2] + 0.5};
    if (sp->profile == 1) {
        /* every cell at or beyond the ramp start holds plasma */
        return (double)c[0] >= sp->p[0] / s->g.d[0] ? sp->ppc : 0;
    }
    const double n = density_at(s, sp, xc);
    if (sp->loading == 1) return (int)rint((double)sp->ppc * n / sp->n0);
    return n > 0.0 ? sp->ppc : 0;
}

int orc_particles_init(orc_sim *s, int profile, int loading, int ppc, double n0, const double *p,
                       double temperature, uint64_t seed)
{
    orc_species sp;
    memset(&sp, 0, sizeof(sp));
    sp.profile = profile; sp.loading = loading; sp.ppc = ppc; sp.n0 = n0;
    for (int i = 0; i < 6; ++i) sp.p[i] = p ? p[i] : 0.0;
    sp.temperature = temperature; sp.seed = seed;
    if (profile < 0 || profile > 2 || loading < 0 || loading > 1 || ppc < 1 || !(n0 > 0.0)) return -1;
    const int nd = s->g.ndim;
    const int64_t nc[3] = {s->g.n[0], s->g.n[1], nd == 3 ? s->g.n[2] : 1};
    int64_t total = 0;
    for (int64_t k = 0; k < nc[2]; ++k)
        for (int64_t j = 0; j < nc[1]; ++j)
            for (int64_t i = 0; i < nc[0]; ++i) {
                const int64_t c[3] = {i, j, k};
                total += cell_count(s, &sp, c);
            }
    double *xs[3], *us[3], *w = malloc(sizeof(double) * (total + 1));
    for (int a = 0; a < 3; ++a) {
        xs[a] = calloc(total + 1, sizeof(double));
        us[a] = calloc(total + 1, sizeof(double));
    }
    const double sig = sqrt(temperature);
    int64_t g = 0;
    for (int64_t k = 0; k < nc[2]; ++k)
        for (int64_t j = 0; j < nc[1]; ++j)
            for (int64_t i = 0; i < nc[0]; ++i) {
                const int64_t c[3] = {i, j, k};
                const int cnt = cell_count(s, &sp, c);
                for (int q = 0; q < cnt; ++q, ++g) {
                    double x[3] = {0.0, 0.0, 0.0};
                    for (int a = 0; a < nd; ++a) {
                        x[a] = (double)c[a] + draw01(seed, 0, g, a);
                        if (x[a] >= (double)(c[a] + 1)) x[a] = nextafter((double)(c[a] + 1), 0.0);
                        xs[a][g] = x[a];
                    }
                    if (profile == 1) {
                        w[g] = density_at(s, &sp, x) / ppc;
                    } else {
                        const double xc[3] = {(double)i + 0.5, (double)j + 0.5, (double)k + 0.5};
                        w[g] = loading == 1 ? n0 / ppc : density_at(s, &sp, xc) / ppc;
                    }
                    if (temperature > 0.0) {
                        const double r1 = sqrt(-2.0 * log(1.0 - draw01(seed, 1, g, 0)));
                        const double r2 = sqrt(-2.0 * log(1.0 - draw01(seed, 1, g, 2)));
                        const double f1 = 2.0 * M_PI * draw01(seed, 1, g, 1);
                        const double f2 = 2.0 * M_PI * draw01(seed, 1, g, 3);
                        us[0][g] = sig * r1 * cos(f1);
                        us[1][g] = sig * r1 * sin(f1);
                        us[2][g] = sig * r2 * cos(f2);
                    }
                }
            }
    const int rc = orc_set_particles(s, total, (const double *const *)xs, (const double *const *)us, w);
    for (int a = 0; a < 3; ++a) { free(xs[a]); free(us[a]); }
    free(w);
    return rc;
}

/* Round the particle state to FP32 storage and back: positions become
 * patch origin + (float)(x - origin), kept below the patch's upper face (the
 * offset a patch-local FP32 position holds); momenta and weights become their
 * nearest floats. */
void orc_round_storage(orc_sim *s)
{
    for (int64_t q = 0; q < s->npart; ++q) {
        double xi[3] = {s->x[0][q], s->x[1][q], s->x[2][q]};
        const int p = patch_of(s, xi);
        const int pc[3] = {p % s->np[0], (p / s->np[0]) % s->np[1], p / (s->np[0] * s->np[1])};
        for (int a = 0; a < s->g.ndim; ++a) {
            const double o = (double)(pc[a] * s->g.patch[a]);
            float loc = (float)(s->x[a][q] - o);
            const float top = nextafterf((float)s->g.patch[a], 0.0f);
            if (loc > top) loc = top;
            if (loc < 0.0f) loc = 0.0f;
            s->x[a][q] = o + (double)loc;
        }
        for (int a = 0; a < 3; ++a) s->u[a][q] = (double)(float)s->u[a][q];
        s->w[q] = (double)(float)s->w[q];
    }
}

void orc_get_particles(const orc_sim *s, double *xo[3], double *uo[3], double *wo, int64_t *ido)
{
    for (int64_t k = 0; k < s->npart; ++k) {
        for (int a = 0; a < 3; ++a) {
            if (xo[a]) xo[a][k] = s->x[a][k];
            if (uo[a]) uo[a][k] = s->u[a][k];
        }
        if (wo) wo[k] = s->w[k];
        if (ido) ido[k] = s->id[k];
    }
}

void orc_get_counts(const orc_sim *s, int32_t *out)
{
    memcpy(out, s->count, sizeof(int32_t) * s->npatch);
}

void orc_get_field(const orc_sim *s, int comp, double *out)
{
    memcpy(out, s->F[comp], sizeof(double) * s->fsize);
}

void orc_set_field(orc_sim *s, int comp, const double *in)
{
    memcpy(s->F[comp], in, sizeof(double) * s->fsize);
}

/* Incident-field table for the x = 0 face: row t holds the incident Ey and
 * Ez on the transverse nodes at time (t + 1/2) dt (Ey sampled on its dual y
 * positions, Ez on primal ones). */
void orc_set_laser(orc_sim *s, int64_t nsteps, const double *ey, const double *ez)
{
    free(s->laser_ey); free(s->laser_ez);
    s->laser_ey = s->laser_ez = NULL;
    s->laser_steps = nsteps;
    size_t sz = sizeof(double) * (size_t)(nsteps * s->laser_n1);
    if (ey) { s->laser_ey = malloc(sz); memcpy(s->laser_ey, ey, sz); }
    if (ez) { s->laser_ez = malloc(sz); memcpy(s->laser_ez, ez, sz); }
}

double orc_cell_volume(const orc_sim *s)
{
    double v = 1.0;
    for (int a = 0; a < s->g.ndim; ++a) v *= s->g.d[a];
    return v;
}

/* Field energy 1/2 sum (E^2 + B^2) V_cell over the stored (valid) nodes. */
double orc_field_energy(const orc_sim *s)
{
    double acc = 0.0;
    for (int c = 0; c < 6; ++c)
        for (int64_t k = 0; k < s->fn[2]; ++k)
            for (int64_t j = 0; j < s->fn[1]; ++j)
                for (int64_t i = 0; i < s->fn[0]; ++i) {
                    int64_t f = flat3(s, c, i, j, k);
                    if (f >= 0) acc += s->F[c][f] * s->F[c][f];
                }
    return 0.5 * acc * orc_cell_volume(s);
}

/* Charge density q sum_p w_p prod_a S2 on primal nodes. */
static int64_t primal_flat(const orc_sim *s, int64_t i, int64_t j, int64_t k)
{
    int64_t a = node_index(s, 0, i, 0), b = node_index(s, 1, j, 0), c = node_index(s, 2, k, 0);
    if (a < 0 || b < 0 || c < 0) return -1;
    return a + (int64_t)s->fn[0] * (b + (int64_t)s->fn[1] * c);
}

void orc_rho(const orc_sim *s, double *out)
{
    memset(out, 0, sizeof(double) * s->fsize);
    for (int64_t p = 0; p < s->npart; ++p) {
        int64_t i0[3] = {0, 0, 0};
        double w[3][3];
        for (int a = 0; a < 3; ++a) {
            if (a < s->g.ndim) orc_shape(s->x[a][p], 0, &i0[a], w[a]);
            else { w[a][0] = 0.0; w[a][1] = 1.0; w[a][2] = 0.0; }
        }
        int kz0 = s->g.ndim == 3 ? -1 : 0, kz1 = s->g.ndim == 3 ? 1 : 0;
        for (int kz = kz0; kz <= kz1; ++kz)
            for (int ky = -1; ky <= 1; ++ky)
                for (int kx = -1; kx <= 1; ++kx) {
                    int64_t f = primal_flat(s, i0[0] + kx, i0[1] + ky, i0[2] + kz);
                    if (f >= 0) out[f] += s->g.q * s->w[p] * w[0][kx + 1] * w[1][ky + 1] * w[2][kz + 1];
                }
    }
}

/* ---- moving window -----------------------------------------------------
 *
 * The LWFA runs of the paper follow the pulse over more than a millimetre of
 * plasma (sections 2.1 and 2.3), which a box of fixed size covers only if it
 * moves with the pulse.  The patch structure makes the move a relabelling: the window
 * jumps by one patch column (patch[0] cells) whenever the distance it should
 * have travelled, v c (n - start) dt after n completed steps, reaches the next
 * multiple of the patch width.  At a jump the fields and currents move left by
 * patch[0] cells with zeros entering at the right, the particles of the first
 * patch column leave the box (counted as removed), every other patch becomes
 * its left neighbour with its particles in the same slots (positions lose
 * patch[0] cells), and the new last column is filled with a cold plasma:
 * ppc_x x ppc_y particles per cell on a regular lattice at offsets
 * ((a + 1/2) / ppc_x, (b + 1/2) / ppc_y), weight density / (ppc_x ppc_y),
 * zero momentum, in the order (patch row, cell row, cell column, b, a), ids
 * continuing from the largest one handed out. */

/* Shifts due after `done` completed steps. */
static int64_t win_due(const orc_sim *s, int64_t done)
{
    const int64_t N = done - s->win_start;
    if (N <= 0) return 0;
    return (int64_t)floor(s->win_v * (double)N * s->g.dt / ((double)s->g.patch[0] * s->g.d[0]));
}

static double win_density(const orc_sim *s, int64_t col)
{
    return s->win_dens[col < s->win_ncols ? col : s->win_ncols - 1];
}

static void window_shift(orc_sim *s)
{
    const int S = s->g.patch[0], P1 = s->g.patch[1];
    const int npx = s->np[0], npy = s->np[1];
    const int64_t fn0 = s->fn[0], fn1 = s->fn[1];
    /* fields and currents */
    for (int c = 0; c < ORC_NCOMP; ++c)
        for (int64_t j = 0; j < fn1; ++j) {
            double *row = s->F[c] + j * fn0;
            for (int64_t i = 0; i < fn0; ++i) row[i] = i + S < fn0 ? row[i + S] : 0.0;
        }
    /* injected particles per new patch (density depends on the column only) */
    const int ppc = s->win_ppc[0] * s->win_ppc[1];
    const int64_t col0 = (s->win_shift + 1) * S + (int64_t)(npx - 1) * S;  /* global column of the new column's first cell */
    int64_t per_patch = 0;
    for (int il = 0; il < S; ++il)
        if (win_density(s, col0 + il) > 0.0) per_patch += (int64_t)P1 * ppc;
    /* particles: old patch starts */
    int64_t *start = malloc(sizeof(int64_t) * (s->npatch + 1));
    start[0] = 0;
    for (int p = 0; p < s->npatch; ++p) start[p + 1] = start[p] + s->count[p];
    int64_t gone = 0;
    for (int py = 0; py < npy; ++py) gone += s->count[npx * py];
    const int64_t nnew = s->npart - gone + per_patch * npy;
    double *nx[3], *nu[3], *nw = malloc(sizeof(double) * (nnew + 1));
    int64_t *nid = malloc(sizeof(int64_t) * (nnew + 1));
    for (int a = 0; a < 3; ++a) {
        nx[a] = malloc(sizeof(double) * (nnew + 1));
        nu[a] = malloc(sizeof(double) * (nnew + 1));
    }
    int32_t *ncount = malloc(sizeof(int32_t) * s->npatch);
    int64_t t = 0;
    for (int py = 0; py < npy; ++py)
        for (int px = 0; px < npx; ++px) {
            const int p = px + npx * py;
            if (px + 1 < npx) {
                const int q = p + 1;  /* the patch that becomes p */
                for (int64_t k = start[q]; k < start[q + 1]; ++k, ++t) {
                    for (int a = 0; a < 3; ++a) { nx[a][t] = s->x[a][k]; nu[a][t] = s->u[a][k]; }
                    nx[0][t] -= (double)S;
                    nw[t] = s->w[k];
                    nid[t] = s->id[k];
                }
                ncount[p] = s->count[q];
            } else {
                const double X0 = (double)(px * S), Y0 = (double)(py * P1);
                for (int jl = 0; jl < P1; ++jl)
                    for (int il = 0; il < S; ++il) {
                        const double dens = win_density(s, col0 + il);
                        if (!(dens > 0.0)) continue;
                        for (int b = 0; b < s->win_ppc[1]; ++b)
                            for (int a = 0; a < s->win_ppc[0]; ++a, ++t) {
                                nx[0][t] = X0 + il + (a + 0.5) / s->win_ppc[0];
                                nx[1][t] = Y0 + jl + (b + 0.5) / s->win_ppc[1];
                                nx[2][t] = 0.0;
                                nu[0][t] = nu[1][t] = nu[2][t] = 0.0;
                                nw[t] = dens / ppc;
                                nid[t] = s->next_id++;
                            }
                    }
                ncount[p] = (int32_t)per_patch;
            }
        }
    s->removed += gone;
    free_particles(s);
    for (int a = 0; a < 3; ++a) { s->x[a] = nx[a]; s->u[a] = nu[a]; }
    s->w = nw;
    s->id = nid;
    s->npart = nnew;
    memcpy(s->count, ncount, sizeof(int32_t) * s->npatch);
    free(ncount);
    free(start);
    s->win_shift += 1;
}

/* Start a moving window: 2-D boxes with open x faces; 0 < v <= 1; density
 * per global cell column (ncols >= 1 entries, non-negative).  Returns 0, or -1
 * for an unsupported request. */
int orc_set_window(orc_sim *s, int64_t start, double v, int ppc_x, int ppc_y,
                   const double *dens, int64_t ncols)
{
    if (s->g.ndim != 2 || s->g.periodic[0]) return -1;
    if (!(v > 0.0 && v <= 1.0) || start < 0 || ppc_x < 1 || ppc_y < 1 || ncols < 1 || !dens) return -1;
    for (int64_t c = 0; c < ncols; ++c)
        if (!(dens[c] >= 0.0) || !isfinite(dens[c])) return -1;
    free(s->win_dens);
    s->win_dens = malloc(sizeof(double) * ncols);
    memcpy(s->win_dens, dens, sizeof(double) * ncols);
    s->win_ncols = ncols;
    s->win = 1;
    s->win_start = start;
    s->win_v = v;
    s->win_ppc[0] = ppc_x;
    s->win_ppc[1] = ppc_y;
    return 0;
}

int64_t orc_window_shift(const orc_sim *s) { return s->win_shift; }
int64_t orc_next_id(const orc_sim *s) { return s->next_id; }

/* ---- particle merging ----------------------------------------------------
 *
 * Dynamic load limiting (section 3.2): where a cell holds too many
 * super-particles they are merged, by a k-means clustering, in a way that
 * keeps the conserved quantities.  The paper leaves the scheme to its
 * reference; this is the reading built here.  In a 2-D cell holding more than
 * cmax particles (taken in slot order), the momenta u = p / (m c) are grouped
 * into k = cmax / 2 clusters by weighted Lloyd iterations: the centroids
 * start at the momenta of members floor(j n / k), then `iters` rounds assign
 * every member to its nearest centroid (squared distance, lowest index on
 * ties) and move every non-empty centroid to its cluster's weighted mean.  A
 * final cluster of three or more members becomes two particles of half its
 * weight W each, at its weighted mean position, with momenta
 * |u_t| (cos t e1 +- sin t e2): gamma_t = E / W is the cluster's mean Lorentz
 * factor, |u_t| = sqrt(gamma_t^2 - 1), e1 the direction of its momentum P
 * (x if P = 0), cos t = |P| / (W |u_t|) (at most 1 by the convexity of gamma),
 * e2 the unit vector along the axis least aligned with e1 made orthogonal to
 * it.  Weight, momentum and kinetic energy of the cell stay as they were
 * (each cell's charge too); the pair carries the two smallest ids of the
 * cluster.  Clusters of one or two members stay as they are.  The patch then
 * holds its untouched particles in their slot order, followed by the pairs in
 * (cell, cluster) order. */

#define ORC_MERGE_KMAX 16

/* k-means and pair for one cell: mem[0..n) particle indices (slot order).
 * Writes kept[] flags for the members and appends pairs to the out arrays;
 * returns the number of pairs. */
static int merge_cell(const orc_sim *s, const int64_t *mem, int n, int cmax, int iters, char *kept,
                      double *ox[3], double *ou[3], double *ow, int64_t *oid, int64_t base)
{
    const int k = cmax / 2;
    double c[ORC_MERGE_KMAX][3];
    int *asg = malloc(sizeof(int) * n);
    for (int j = 0; j < k; ++j)
        for (int a = 0; a < 3; ++a) c[j][a] = s->u[a][mem[(int64_t)j * n / k]];
    for (int it = 0; it < iters; ++it) {
        for (int i = 0; i < n; ++i) {
            const int64_t q = mem[i];
            int best = 0;
            double bd = 0.0;
            for (int j = 0; j < k; ++j) {
                const double dx = s->u[0][q] - c[j][0], dy = s->u[1][q] - c[j][1], dz = s->u[2][q] - c[j][2];
                const double d2 = dx * dx + dy * dy + dz * dz;
                if (j == 0 || d2 < bd) { bd = d2; best = j; }
            }
            asg[i] = best;
        }
        for (int j = 0; j < k; ++j) {
            double sw = 0.0, su[3] = {0.0, 0.0, 0.0};
            for (int i = 0; i < n; ++i)
                if (asg[i] == j) {
                    const int64_t q = mem[i];
                    sw += s->w[q];
                    for (int a = 0; a < 3; ++a) su[a] += s->w[q] * s->u[a][q];
                }
            if (sw > 0.0)
                for (int a = 0; a < 3; ++a) c[j][a] = su[a] / sw;
        }
    }
    int pairs = 0;
    for (int j = 0; j < k; ++j) {
        int cnt = 0;
        for (int i = 0; i < n; ++i) cnt += asg[i] == j;
        if (cnt < 3) {
            for (int i = 0; i < n; ++i)
                if (asg[i] == j) kept[i] = 1;
            continue;
        }
        double W = 0.0, E = 0.0, P[3] = {0.0, 0.0, 0.0}, X[2] = {0.0, 0.0};
        int64_t id0 = INT64_MAX, id1 = INT64_MAX;
        for (int i = 0; i < n; ++i) {
            if (asg[i] != j) continue;
            const int64_t q = mem[i];
            const double w = s->w[q];
            const double g = sqrt(1.0 + s->u[0][q] * s->u[0][q] + s->u[1][q] * s->u[1][q] + s->u[2][q] * s->u[2][q]);
            W += w;
            E += w * g;
            for (int a = 0; a < 3; ++a) P[a] += w * s->u[a][q];
            X[0] += w * s->x[0][q];
            X[1] += w * s->x[1][q];
            const int64_t id = s->id[q];
            if (id < id0) { id1 = id0; id0 = id; }
            else if (id < id1) id1 = id;
        }
        const double gt = E / W;
        const double ut = gt > 1.0 ? sqrt(gt * gt - 1.0) : 0.0;
        const double pn = sqrt(P[0] * P[0] + P[1] * P[1] + P[2] * P[2]);
        double e1[3] = {1.0, 0.0, 0.0};
        if (pn > 0.0)
            for (int a = 0; a < 3; ++a) e1[a] = P[a] / pn;
        int ax = 0;
        for (int a = 1; a < 3; ++a)
            if (fabs(e1[a]) < fabs(e1[ax])) ax = a;
        double e2[3] = {0.0, 0.0, 0.0};
        e2[ax] = 1.0;
        const double dp = e1[ax];
        for (int a = 0; a < 3; ++a) e2[a] -= dp * e1[a];
        const double en = sqrt(e2[0] * e2[0] + e2[1] * e2[1] + e2[2] * e2[2]);
        for (int a = 0; a < 3; ++a) e2[a] /= en;
        double ct = ut > 0.0 ? pn / (W * ut) : 0.0;
        if (ct > 1.0) ct = 1.0;
        const double st = sqrt(1.0 - ct * ct);
        for (int h = 0; h < 2; ++h) {
            const int64_t t = base + 2 * pairs + h;
            const double sg = h == 0 ? 1.0 : -1.0;
            for (int a = 0; a < 3; ++a) ou[a][t] = ut * (ct * e1[a] + sg * st * e2[a]);
            ox[0][t] = X[0] / W;
            ox[1][t] = X[1] / W;
            ox[2][t] = 0.0;
            ow[t] = 0.5 * W;
            oid[t] = h == 0 ? id0 : id1;
        }
        ++pairs;
    }
    free(asg);
    return pairs;
}

/* One merge pass over every patch (2-D).  Returns the particles taken out. */
int64_t orc_merge(orc_sim *s, int cmax, int iters)
{
    const int P0 = s->g.patch[0], P1 = s->g.patch[1], ncell = P0 * P1;
    int64_t *start = malloc(sizeof(int64_t) * (s->npatch + 1));
    start[0] = 0;
    for (int p = 0; p < s->npatch; ++p) start[p + 1] = start[p] + s->count[p];
    /* at most as many particles as before */
    const int64_t cap = s->npart + 1;
    double *nx[3], *nu[3], *nw = malloc(sizeof(double) * cap);
    int64_t *nid = malloc(sizeof(int64_t) * cap);
    for (int a = 0; a < 3; ++a) {
        nx[a] = malloc(sizeof(double) * cap);
        nu[a] = malloc(sizeof(double) * cap);
    }
    /* pairs of a patch before they are appended */
    double *px_[3], *pu_[3], *pw_ = malloc(sizeof(double) * cap);
    int64_t *pid_ = malloc(sizeof(int64_t) * cap);
    for (int a = 0; a < 3; ++a) {
        px_[a] = malloc(sizeof(double) * cap);
        pu_[a] = malloc(sizeof(double) * cap);
    }
    int *cellof = malloc(sizeof(int) * cap);
    char *keep = malloc(cap);
    int64_t *mem = malloc(sizeof(int64_t) * cap);
    char *mkept = malloc(cap);
    int *ccount = malloc(sizeof(int) * ncell);
    int64_t t = 0, taken = 0;
    for (int p = 0; p < s->npatch; ++p) {
        const int px = p % s->np[0], py = p / s->np[0];
        const int64_t a0 = start[p], a1 = start[p + 1];
        memset(ccount, 0, sizeof(int) * ncell);
        for (int64_t q = a0; q < a1; ++q) {
            int cx = (int)floor(s->x[0][q]) - px * P0, cy = (int)floor(s->x[1][q]) - py * P1;
            if (cx < 0) cx = 0;
            if (cx > P0 - 1) cx = P0 - 1;
            if (cy < 0) cy = 0;
            if (cy > P1 - 1) cy = P1 - 1;
            cellof[q - a0] = cx + P0 * cy;
            ccount[cx + P0 * cy]++;
            keep[q - a0] = 1;
        }
        int64_t npair = 0;
        for (int cidx = 0; cidx < ncell; ++cidx) {
            if (ccount[cidx] <= cmax) continue;
            int n = 0;
            for (int64_t q = a0; q < a1; ++q)
                if (cellof[q - a0] == cidx) mem[n++] = q;
            memset(mkept, 0, n);
            npair += merge_cell(s, mem, n, cmax, iters, mkept, px_, pu_, pw_, pid_, 2 * npair);
            for (int i = 0; i < n; ++i) keep[mem[i] - a0] = mkept[i];
        }
        int32_t c = 0;
        for (int64_t q = a0; q < a1; ++q) {
            if (!keep[q - a0]) continue;
            for (int a = 0; a < 3; ++a) { nx[a][t] = s->x[a][q]; nu[a][t] = s->u[a][q]; }
            nw[t] = s->w[q];
            nid[t] = s->id[q];
            ++t;
            ++c;
        }
        for (int64_t i = 0; i < 2 * npair; ++i, ++t, ++c) {
            for (int a = 0; a < 3; ++a) { nx[a][t] = px_[a][i]; nu[a][t] = pu_[a][i]; }
            nw[t] = pw_[i];
            nid[t] = pid_[i];
        }
        taken += s->count[p] - c;
        s->count[p] = c;
    }
    free_particles(s);
    for (int a = 0; a < 3; ++a) { s->x[a] = nx[a]; s->u[a] = nu[a]; free(px_[a]); free(pu_[a]); }
    s->w = nw;
    s->id = nid;
    s->npart = t;
    s->merged += taken;
    free(pw_); free(pid_); free(cellof); free(keep); free(mem); free(mkept); free(ccount); free(start);
    return taken;
}

/* Merge after every `every`-th step (0: never); 2-D only, 4 <= cmax <= 32,
 * 1 <= iters <= 64.  Returns 0, or -1 for an unsupported request. */
int orc_set_merge(orc_sim *s, int every, int cmax, int iters)
{
    if (every < 0) return -1;
    if (every > 0 && (s->g.ndim != 2 || cmax < 4 || cmax > 2 * ORC_MERGE_KMAX || iters < 1 || iters > 64)) return -1;
    s->merge_every = every;
    s->merge_cmax = cmax;
    s->merge_iters = iters;
    return 0;
}

int64_t orc_merged(const orc_sim *s) { return s->merged; }

/* One full step n -> n+1 (state x^n, u^{n-1/2}, E^n, B^n on entry). */
static void one_step(orc_sim *s)
{
    const int nd = s->g.ndim;
    const double dt = s->g.dt, q = s->g.q, m = s->g.m, vol = orc_cell_volume(s);
    s->U_last = orc_field_energy(s);
    for (int c = 6; c < 9; ++c) memset(s->F[c], 0, sizeof(double) * s->fsize);
    int32_t *dest = malloc(sizeof(int32_t) * (s->npart + 1));
    double K = 0.0;
#ifdef _OPENMP
    /* timing build: threads push disjoint particle ranges and deposit into
     * private current arrays, summed below in thread order */
    const int nth = omp_get_max_threads();
    if (nth > 1 && s->jthreads != nth) {
        if (s->jbuf)
            for (int t = 0; t < 3 * s->jthreads; ++t) free(s->jbuf[t]);
        free(s->jbuf);
        s->jbuf = malloc(sizeof(double *) * 3 * nth);
        for (int t = 0; t < 3 * nth; ++t) s->jbuf[t] = malloc(sizeof(double) * s->fsize);
        s->jthreads = nth;
    }
    if (nth > 1)
        for (int t = 0; t < 3 * nth; ++t) memset(s->jbuf[t], 0, sizeof(double) * s->fsize);
    double **jp = nth > 1 ? s->jbuf : NULL;
    s->jpriv = jp;
#pragma omp parallel for reduction(+ : K) schedule(static)
#endif
    for (int64_t k = 0; k < s->npart; ++k) {
        {
            double x0[3] = {s->x[0][k], s->x[1][k], s->x[2][k]};
            double u[3] = {s->u[0][k], s->u[1][k], s->u[2][k]};
            double EB[6];
            orc_gather(s, x0, EB);
            double g0 = sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
            orc_boris(u, EB, EB + 3, q, m, dt);
            double g1 = sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
            K += s->w[k] * m * (0.5 * (g0 + g1) - 1.0) * vol;
            double x1[3] = {x0[0], x0[1], x0[2]};
            for (int a = 0; a < nd; ++a) x1[a] = x0[a] + dt * u[a] / (g1 * s->g.d[a]);
            orc_deposit(s, x0, x1, s->w[k], u[2] / g1);
            int removed = 0;
            for (int a = 0; a < nd; ++a) {
                double n = (double)s->g.n[a];
                if (s->g.periodic[a]) {
                    if (x1[a] >= n) x1[a] -= n;
                    else if (x1[a] < 0.0) x1[a] += n;
                    if (x1[a] == n) x1[a] = 0.0;
                } else if (x1[a] < 0.0 || x1[a] >= n) {
                    removed = 1;
                }
            }
            for (int a = 0; a < 3; ++a) { s->x[a][k] = x1[a]; s->u[a][k] = u[a]; }
            dest[k] = removed ? -1 : patch_of(s, x1);
        }
    }
#ifdef _OPENMP
    if (jp)
        for (int t = 0; t < nth; ++t)
            for (int c = 0; c < 3; ++c)
                for (int64_t f = 0; f < s->fsize; ++f) s->F[6 + c][f] += jp[3 * t + c][f];
    s->jpriv = NULL;
#endif
    s->K_last = K;

    orc_maxwell(s);

    /* re-bin */
    int32_t *newcount = malloc(sizeof(int32_t) * s->npatch);
    int64_t *src = malloc(sizeof(int64_t) * (s->npart + 1));
    orc_rebin(s->npatch, s->count, dest, newcount, src);
    int64_t nnew = 0;
    for (int p = 0; p < s->npatch; ++p) nnew += newcount[p];
    double *nx[3], *nu[3], *nw = malloc(sizeof(double) * (nnew + 1));
    int64_t *nid = malloc(sizeof(int64_t) * (nnew + 1));
    for (int a = 0; a < 3; ++a) {
        nx[a] = malloc(sizeof(double) * (nnew + 1));
        nu[a] = malloc(sizeof(double) * (nnew + 1));
    }
    for (int64_t t = 0; t < nnew; ++t) {
        int64_t f = src[t];
        for (int a = 0; a < 3; ++a) { nx[a][t] = s->x[a][f]; nu[a][t] = s->u[a][f]; }
        nw[t] = s->w[f];
        nid[t] = s->id[f];
    }
    s->removed += s->npart - nnew;
    free_particles(s);
    for (int a = 0; a < 3; ++a) { s->x[a] = nx[a]; s->u[a] = nu[a]; }
    s->w = nw;
    s->id = nid;
    s->npart = nnew;
    memcpy(s->count, newcount, sizeof(int32_t) * s->npatch);
    free(newcount);
    free(src);
    free(dest);
    if (s->merge_every > 0 && (s->step + 1) % s->merge_every == 0)
        orc_merge(s, s->merge_cmax, s->merge_iters);
    if (s->win && win_due(s, s->step + 1) > s->win_shift) window_shift(s);
    s->step += 1;
}

void orc_step(orc_sim *s, int64_t nsteps)
{
    for (int64_t t = 0; t < nsteps; ++t) one_step(s);
}

/* Energies of the last completed step: U(E^n, B^n) and K^n. */
void orc_energy(const orc_sim *s, double *U, double *K)
{
    *U = s->U_last;
    *K = s->K_last;
}
