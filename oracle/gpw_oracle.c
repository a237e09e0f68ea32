/*
 * Plain CPU oracle for multigrid Gaussian-plane-wave collocation (rho),
 * integration (mat) and the nuclear gradient of the collocation (grad).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library or its Python binding may
 * call, link or load this file.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark use it.  It shares no code with the HIP
 * path: its own pair enumeration, truncation, level rule, mesh rule, grid
 * evaluation and AO ordering are written here from the paper's definitions.
 *
 * What it computes (all FP64, Gamma point; orthorhombic cells with a 1-D table
 * per axis, general cells point by point, see eval_pair_general):
 *
 *   rho_l[j mod N] = sum over ordered primitive-shell pairs (a,k),(b,l) and
 *                    lattice vectors T of the second one, with level(p) = l,
 *                    and over unwrapped grid points x_j inside the truncation
 *                    sphere of the pair image p, of
 *                    sum_{mu in a, nu in b} D_{mu nu} c_ak c_bl G_{ak,mu}(x_j) G_{bl,nu}(x_j - T)
 *
 *   This is the single-lattice-sum-plus-fold form of the density
 *   (Sec. III.A, Eq. (rho_wrap)), equal term by term to the double lattice
 *   sum of Eq. (rho) (Sec. II).  G is the un-normalised Cartesian primitive
 *   (x-Ax)^i (y-Ay)^j (z-Az)^k exp(-a |r-A|^2) (Sec. III.A, Eq. (gx)).
 *
 *   M_{mu nu} = sum_l w_l sum over the same terms with D replaced by v_l[j mod N],
 *   with the quadrature weight w_l = Omega / N_l (Sec. III.A, Eq. (J_wrap) and
 *   the weight stated with the V tensor).
 *
 *   grad_X = d/dR_X of E = sum_l w_l <v_l, rho_l(D; R)> at fixed D and v: both
 *   factors of every ordered pair are differentiated and credited to their
 *   atoms (Sec. III.B, Alg. 3).
 *
 * Meta-GGA terms (Sec. II, the kinetic energy density and Eq. (J_metaGGA);
 * Sec. III.B, the substitution of the pair function by grad g_a . grad g_b
 * stated with Algs. 1-3):
 *
 *   tau_l[j mod N] = 1/2 sum over the same ordered pair images and points of
 *                    sum_{mu nu} D_{mu nu} c_ak c_bl grad G_{ak,mu}(x_j) . grad G_{bl,nu}(x_j - T)
 *   Mtau_{mu nu}   = sum_l w_l sum over the same terms with D replaced by
 *                    vtau_l[j mod N]: the variational derivative of
 *                    E_tau = sum_l w_l <vtau_l, tau_l(D)> with respect to D
 *   gradtau_X      = d/dR_X of E_tau at fixed D and vtau (second derivatives of
 *                    the primitives)
 *
 *   The factor 1/2 of the kinetic energy density is kept in all three (the
 *   paper's integration note keeps it, Eq. (J_metaGGA) and its gradient note
 *   drop it; only with it are the three mutually consistent derivatives of
 *   E_tau).
 *
 * Truncation (reading of Sec. III.A, Eq. (cut), applied to the pair product):
 *   K = c_ak c_bl exp(-a_k a_l / (a_k + a_l) |A - B - T|^2), alpha_p = a_k + a_l,
 *   P = (a_k A + a_l (B + T)) / alpha_p, L = l_a + l_b,
 *   f(r) = |K| r^(L+2) exp(-alpha_p r^2).  The pair image is dropped when the
 *   maximum of f (at r* = sqrt((L+2) / (2 alpha_p))) is below tau; otherwise its
 *   radius R is the root of f(R) = tau beyond r*, found by bisection, and the
 *   pair image contributes at the grid points with |x_j - P| <= R (Sec. III.A:
 *   the grid points inside a sphere about P whose radius comes from Eq. (cut)).
 *
 * Levels (Sec. II, multigrid; the Quickstep convention it cites): a pair image
 * goes to the coarsest level i with cutoff E_i >= alpha_p * E_rel (Ry), and to
 * the finest level when none qualifies.  Mesh of a level: per axis the smallest
 * 2,3,5-smooth N with N >= sqrt(E) L / pi.
 *
 * The evaluation is deliberately plain: each primitive is tabulated about its
 * own centre with one exp per 1-D grid point, and every point is visited
 * directly.  No product-Gaussian recursion, no binomial expansion, no blocking.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_MAXL 4                  /* up to g shells */
#define OR_NCART 15                /* Cartesian components of a g shell */
#define OR_NCNT 25                 /* per-(l_a, l_b) counters, index 5 l_a + l_b */

typedef struct {
    double cell[3];
    int natm;
    const double *coords;      /* natm*3 */
    int nshell;
    const int *shell_atom, *shell_l, *shell_nprim, *shell_prim0;
    const double *exps, *coefs;
    int nlevels;
    const int *mesh;           /* nlevels*3 */
    const double *level_cut;   /* nlevels, Ry (NULL allowed when nlevels == 1) */
    double rel_cut;
    double tau;
    const unsigned char *atom_mask;  /* optional: only pairs whose first atom is set */
    int mask_either;                 /* with atom_mask: pairs with either atom set */
    const double *lat;               /* optional general cell: lattice vectors a_d as rows (9
                                        doubles); NULL: the orthorhombic cell[] */
} osys;

/* Inverse of the lattice matrix (rows a_d): r = u . A, u = r . inv; returns det. */
static double lat_inverse(const double *a, double *inv)
{
    double det = a[0] * (a[4] * a[8] - a[5] * a[7]) - a[1] * (a[3] * a[8] - a[5] * a[6]) +
                 a[2] * (a[3] * a[7] - a[4] * a[6]);
    inv[0] = (a[4] * a[8] - a[5] * a[7]) / det;
    inv[1] = (a[2] * a[7] - a[1] * a[8]) / det;
    inv[2] = (a[1] * a[5] - a[2] * a[4]) / det;
    inv[3] = (a[5] * a[6] - a[3] * a[8]) / det;
    inv[4] = (a[0] * a[8] - a[2] * a[6]) / det;
    inv[5] = (a[2] * a[3] - a[0] * a[5]) / det;
    inv[6] = (a[3] * a[7] - a[4] * a[6]) / det;
    inv[7] = (a[1] * a[6] - a[0] * a[7]) / det;
    inv[8] = (a[0] * a[4] - a[1] * a[3]) / det;
    return det;
}

/* Length of column d of inv: the change of fractional coordinate u_d per unit
 * distance along its steepest direction. */
static double inv_col_norm(const double *inv, int d)
{
    return sqrt(inv[d] * inv[d] + inv[3 + d] * inv[3 + d] + inv[6 + d] * inv[6 + d]);
}

/* ---------------------------------------------------------------- basics */

static int ncart(int l) { return (l + 1) * (l + 2) / 2; }

/* Cartesian exponents of component c of shell l, lexicographic order with
 * lx descending, then ly descending. */
static void cart_exps(int l, int c, int *ix, int *iy, int *iz)
{
    int n = 0;
    for (int x = l; x >= 0; --x)
        for (int y = l - x; y >= 0; --y) {
            if (n == c) { *ix = x; *iy = y; *iz = l - x - y; return; }
            ++n;
        }
    *ix = *iy = *iz = 0;
}

static int is_smooth235(long n)
{
    if (n < 1) return 0;
    while (n % 2 == 0) n /= 2;
    while (n % 3 == 0) n /= 3;
    while (n % 5 == 0) n /= 5;
    return n == 1;
}

/* Mesh rule: smallest 2,3,5-smooth N >= sqrt(E) * L / pi per axis. */
int oracle_meshes(const double *cell, int nlevels, const double *cut_ry, int *mesh_out)
{
    for (int i = 0; i < nlevels; ++i)
        for (int d = 0; d < 3; ++d) {
            double need = sqrt(cut_ry[i]) * cell[d] / M_PI;
            long n = (long)ceil(need);
            if (n < 1) n = 1;
            while (!is_smooth235(n)) ++n;
            mesh_out[3 * i + d] = (int)n;
        }
    return 0;
}

static int level_of(const osys *s, double alpha_p)
{
    if (s->nlevels <= 1 || !s->level_cut) return 0;
    for (int i = s->nlevels - 1; i >= 0; --i)
        if (s->level_cut[i] >= alpha_p * s->rel_cut) return i;
    return 0;
}

/* log f(r) - log tau for f(r) = |K| r^(L+2) exp(-alpha r^2). */
static double logf_minus(double logK, int L, double alpha, double r, double logtau)
{
    return logK + (L + 2) * log(r) - alpha * r * r - logtau;
}

/* Truncation radius; returns 0 when the pair image is dropped. */
static int trunc_radius(double K, int L, double alpha, double tau, double *R)
{
    if (K == 0.0) return 0;
    double logK = log(fabs(K)), logtau = log(tau);
    double rs = sqrt((L + 2) / (2.0 * alpha));
    if (logf_minus(logK, L, alpha, rs, logtau) < 0.0) return 0;
    double lo = rs, hi = 2.0 * rs + 1.0;
    while (logf_minus(logK, L, alpha, hi, logtau) >= 0.0) hi *= 2.0;
    for (int it = 0; it < 400; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (logf_minus(logK, L, alpha, mid, logtau) >= 0.0) lo = mid; else hi = mid;
    }
    *R = lo;
    return 1;
}

static long lmod(long a, long n) { long r = a % n; return r < 0 ? r + n : r; }

/* ------------------------------------------------------------ pair images */

typedef struct {
    int sa, ka, sb, kb;        /* shells and primitive indices */
    int la, lb, atom_a, atom_b;
    double A[3], B[3];         /* B includes the image translation */
    double aa, ab, ca, cb;     /* exponents and raw coefficients */
    double alpha, P[3], R;
    int level;
} opair;

/* Visit every ordered pair image that survives truncation. */
typedef void (*pair_fn)(const osys *s, const opair *p, void *ctx, int tid);

static void for_each_pair(const osys *s, pair_fn fn, void *ctx)
{
    int nps = 0;
    for (int sh = 0; sh < s->nshell; ++sh) nps += s->shell_nprim[sh];
    int *ps_shell = (int *)malloc(sizeof(int) * nps);
    int *ps_prim = (int *)malloc(sizeof(int) * nps);
    int q = 0;
    for (int sh = 0; sh < s->nshell; ++sh)
        for (int k = 0; k < s->shell_nprim[sh]; ++k) { ps_shell[q] = sh; ps_prim[q] = k; ++q; }

    long ntot = (long)nps * nps;
#pragma omp parallel for schedule(dynamic, 16)
    for (long idx = 0; idx < ntot; ++idx) {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        int i = (int)(idx / nps), j = (int)(idx % nps);
        int sa = ps_shell[i], ka = ps_prim[i], sb = ps_shell[j], kb = ps_prim[j];
        int atom_a = s->shell_atom[sa], atom_b = s->shell_atom[sb];
        if (s->atom_mask && !s->atom_mask[atom_a] && !(s->mask_either && s->atom_mask[atom_b])) continue;
        opair p;
        p.sa = sa; p.ka = ka; p.sb = sb; p.kb = kb;
        p.la = s->shell_l[sa]; p.lb = s->shell_l[sb];
        p.atom_a = atom_a; p.atom_b = atom_b;
        p.aa = s->exps[s->shell_prim0[sa] + ka];
        p.ab = s->exps[s->shell_prim0[sb] + kb];
        p.ca = s->coefs[s->shell_prim0[sa] + ka];
        p.cb = s->coefs[s->shell_prim0[sb] + kb];
        if (p.ca == 0.0 || p.cb == 0.0) continue;
        int L = p.la + p.lb;
        double alpha = p.aa + p.ab, mu = p.aa * p.ab / alpha;
        double rs = sqrt((L + 2) / (2.0 * alpha));
        /* largest |A - B - T| that can survive: mu d^2 <= Q */
        double Q = log(fabs(p.ca * p.cb)) + (L + 2) * log(rs) - 0.5 * (L + 2) - log(s->tau);
        if (Q < 0.0) continue;
        double dmax = sqrt(Q / mu);
        const double *A = s->coords + 3 * atom_a, *B = s->coords + 3 * atom_b;
        long nlo[3], nhi[3];
        double inv[9];
        if (s->lat) lat_inverse(s->lat, inv);
        for (int d = 0; d < 3; ++d) {
            if (s->lat) {
                /* |A - B - T| <= dmax bounds the fractional coordinate of A - B - T */
                double u = (A[0] - B[0]) * inv[d] + (A[1] - B[1]) * inv[3 + d] + (A[2] - B[2]) * inv[6 + d];
                double du = dmax * inv_col_norm(inv, d);
                nlo[d] = (long)ceil(u - du) - 1;
                nhi[d] = (long)floor(u + du) + 1;
            } else {
                double ab = A[d] - B[d];
                nlo[d] = (long)ceil((ab - dmax) / s->cell[d]) - 1;
                nhi[d] = (long)floor((ab + dmax) / s->cell[d]) + 1;
            }
        }
        for (long n0 = nlo[0]; n0 <= nhi[0]; ++n0)
            for (long n1 = nlo[1]; n1 <= nhi[1]; ++n1)
                for (long n2 = nlo[2]; n2 <= nhi[2]; ++n2) {
                    long nn[3] = {n0, n1, n2};
                    double d2 = 0.0;
                    for (int d = 0; d < 3; ++d) {
                        p.A[d] = A[d];
                        if (s->lat)   /* T = n_0 a_0 + n_1 a_1 + n_2 a_2 */
                            p.B[d] = B[d] + nn[0] * s->lat[d] + nn[1] * s->lat[3 + d] + nn[2] * s->lat[6 + d];
                        else
                            p.B[d] = B[d] + nn[d] * s->cell[d];
                        double t = p.A[d] - p.B[d];
                        d2 += t * t;
                    }
                    double K = p.ca * p.cb * exp(-mu * d2);
                    double R;
                    if (!trunc_radius(K, L, alpha, s->tau, &R)) continue;
                    p.alpha = alpha;
                    for (int d = 0; d < 3; ++d) p.P[d] = (p.aa * p.A[d] + p.ab * p.B[d]) / alpha;
                    p.R = R;
                    p.level = level_of(s, alpha);
                    fn(s, &p, ctx, tid);
                }
    }
    free(ps_shell);
    free(ps_prim);
}

/* 1-D tables of one primitive about its own centre over [lo, hi]:
 * g[i][t] = (x_t - C)^i exp(-a (x_t - C)^2), i = 0..lmax, x_t = (lo + t) h. */
static void tab1d(double C, double a, double h, long lo, long n, int lmax, double *g)
{
    for (long t = 0; t < n; ++t) {
        double x = (double)(lo + t) * h;
        double dx = x - C;
        double e = exp(-a * dx * dx);
        double pw = 1.0;
        for (int i = 0; i <= lmax; ++i) { g[i * n + t] = pw * e; pw *= dx; }
    }
}

enum { MODE_RHO = 0, MODE_MAT = 1, MODE_GRAD = 2, MODE_TAU = 3, MODE_MAT_TAU = 4, MODE_GRAD_TAU = 5 };

/* First and second derivative along one axis of (x-C)^i exp(-a (x-C)^2) at
 * point t, from the table g of (x-C)^k exp(-a (x-C)^2), k = 0..lmax:
 *   d/dx   = i (x-C)^(i-1) e - 2a (x-C)^(i+1) e
 *   d2/dx2 = i(i-1) (x-C)^(i-2) e - 2a(2i+1) (x-C)^i e + 4a^2 (x-C)^(i+2) e */
static double tab_d1(const double *g, long n, long t, int i, double a)
{
    double v = -2.0 * a * g[(i + 1) * n + t];
    if (i >= 1) v += i * g[(i - 1) * n + t];
    return v;
}

static double tab_d2(const double *g, long n, long t, int i, double a)
{
    double v = -2.0 * a * (2 * i + 1) * g[i * n + t] + 4.0 * a * a * g[(i + 2) * n + t];
    if (i >= 2) v += i * (i - 1) * g[(i - 2) * n + t];
    return v;
}

/* grad G_mu(x) along axis d (the derivative with respect to r), a primitive
 * with Cartesian exponents e[3] tabulated in g[3] at point tt[3]. */
static double cart_d1(double *const *g, const long *n, const long *tt, const int *e, double a, int d)
{
    double v = 1.0;
    for (int k = 0; k < 3; ++k)
        v *= (k == d) ? tab_d1(g[k], n[k], tt[k], e[k], a) : g[k][e[k] * n[k] + tt[k]];
    return v;
}

/* d2 G_mu / dr_d dr_f */
static double cart_d2(double *const *g, const long *n, const long *tt, const int *e, double a, int d, int f)
{
    double v = 1.0;
    for (int k = 0; k < 3; ++k) {
        if (d == f && k == d) v *= tab_d2(g[k], n[k], tt[k], e[k], a);
        else if (k == d || k == f) v *= tab_d1(g[k], n[k], tt[k], e[k], a);
        else v *= g[k][e[k] * n[k] + tt[k]];
    }
    return v;
}

typedef struct {
    int mode;
    const double *D;           /* n_ao x n_ao */
    const double *V;           /* concatenated levels */
    long *lvl_off;             /* nlevels+1 */
    int n_ao;
    int *ao_off;               /* nshell+1 */
    int nthreads;
    double **tbuf;             /* per-thread output buffers */
    long tlen;
    /* sampled points (rho only): level, wrapped flat indices */
    int samp_level;
    long nsamp;
    const long *samp_idx;
    /* requested matrix blocks (mat only): shell-pair -> offset or -1 */
    const long *sp_slot;
    /* evaluation counters per (la, lb) and thread */
    long *counts;              /* nthreads * OR_NCNT */
} octx;

/* The contributions of one pair image at one grid point (wrapped flat index
 * wflat of its level; sample slot sidx in the sampled modes), from the 1-D
 * tables ga, gb (n[d] entries per power along axis d) at table position tt. */
static void point_terms(const osys *s, octx *c, const opair *p, double *const *ga, double *const *gb,
                        const long *n, const long *tt, const int (*ax)[3], const int (*bx)[3], long wflat,
                        long sidx, double w, double *out)
{
    const int lv = p->level, la = p->la, lb = p->lb, na = ncart(la), nb = ncart(lb);
    const int mu0 = c->ao_off[p->sa], nu0 = c->ao_off[p->sb];
    const double cc = p->ca * p->cb;
    double Ga[OR_NCART], Gb[OR_NCART];
    for (int m = 0; m < na; ++m)
        Ga[m] = ga[0][ax[m][0] * n[0] + tt[0]] * ga[1][ax[m][1] * n[1] + tt[1]] *
                ga[2][ax[m][2] * n[2] + tt[2]];
    for (int m = 0; m < nb; ++m)
        Gb[m] = gb[0][bx[m][0] * n[0] + tt[0]] * gb[1][bx[m][1] * n[1] + tt[1]] *
                gb[2][bx[m][2] * n[2] + tt[2]];
    if (c->mode >= MODE_TAU) {
        double Da[OR_NCART][3], Db[OR_NCART][3];   /* grad G along each axis */
        for (int m = 0; m < na; ++m)
            for (int d = 0; d < 3; ++d) Da[m][d] = cart_d1(ga, n, tt, ax[m], p->aa, d);
        for (int m = 0; m < nb; ++m)
            for (int d = 0; d < 3; ++d) Db[m][d] = cart_d1(gb, n, tt, bx[m], p->ab, d);
        if (c->mode == MODE_TAU) {
            double acc = 0.0;
            for (int i = 0; i < na; ++i)
                for (int j = 0; j < nb; ++j) {
                    double dot = Da[i][0] * Db[j][0] + Da[i][1] * Db[j][1] + Da[i][2] * Db[j][2];
                    acc += c->D[(long)(mu0 + i) * c->n_ao + nu0 + j] * dot;
                }
            if (c->nsamp > 0) out[sidx] += 0.5 * cc * acc;
            else out[c->lvl_off[lv] + wflat] += 0.5 * cc * acc;
        } else if (c->mode == MODE_MAT_TAU) {
            double f = 0.5 * w * c->V[c->lvl_off[lv] + wflat] * cc;
            for (int i = 0; i < na; ++i)
                for (int j = 0; j < nb; ++j) {
                    double dot = Da[i][0] * Db[j][0] + Da[i][1] * Db[j][1] + Da[i][2] * Db[j][2];
                    long o;
                    if (c->sp_slot) o = c->sp_slot[(long)p->sa * s->nshell + p->sb] + i * nb + j;
                    else o = (long)(mu0 + i) * c->n_ao + nu0 + j;
                    out[o] += f * dot;
                }
        } else {
            /* d/dA_e grad G_a = -d/dr_e grad G_a (G_a depends on r - A) */
            double f = 0.5 * w * c->V[c->lvl_off[lv] + wflat] * cc;
            double gA[3] = {0, 0, 0}, gB[3] = {0, 0, 0};
            for (int i = 0; i < na; ++i)
                for (int j = 0; j < nb; ++j) {
                    double Dij = c->D[(long)(mu0 + i) * c->n_ao + nu0 + j];
                    if (Dij == 0.0) return;
                    for (int e = 0; e < 3; ++e)
                        for (int d = 0; d < 3; ++d) {
                            gA[e] -= Dij * cart_d2(ga, n, tt, ax[i], p->aa, e, d) * Db[j][d];
                            gB[e] -= Dij * Da[i][d] * cart_d2(gb, n, tt, bx[j], p->ab, e, d);
                        }
                }
            for (int e = 0; e < 3; ++e) {
                out[3 * p->atom_a + e] += f * gA[e];
                out[3 * p->atom_b + e] += f * gB[e];
            }
        }
        return;
    }
    if (c->mode == MODE_RHO) {
        double acc = 0.0;
        for (int i = 0; i < na; ++i) {
            double t = 0.0;
            for (int j = 0; j < nb; ++j)
                t += c->D[(long)(mu0 + i) * c->n_ao + nu0 + j] * Gb[j];
            acc += Ga[i] * t;
        }
        if (c->nsamp > 0) out[sidx] += cc * acc;
        else out[c->lvl_off[lv] + wflat] += cc * acc;
    } else if (c->mode == MODE_MAT) {
        double f = w * c->V[c->lvl_off[lv] + wflat] * cc;
        long base;
        long stride;
        if (c->sp_slot) {
            base = c->sp_slot[(long)p->sa * s->nshell + p->sb];
            if (base < 0) return;
            stride = nb;
            for (int i = 0; i < na; ++i)
                for (int j = 0; j < nb; ++j)
                    out[base + i * stride + j] += f * Ga[i] * Gb[j];
        } else {
            for (int i = 0; i < na; ++i)
                for (int j = 0; j < nb; ++j)
                    out[(long)(mu0 + i) * c->n_ao + nu0 + j] += f * Ga[i] * Gb[j];
        }
    } else {
        /* d/dA_d of the first factor and d/dB_d of the second:
         * d/dC [(x-C)^i e^{-a (x-C)^2}] = -i (x-C)^(i-1) e + 2a (x-C)^(i+1) e */
        double f = w * c->V[c->lvl_off[lv] + wflat] * cc;
        double gA[3] = {0, 0, 0}, gB[3] = {0, 0, 0};
        for (int i = 0; i < na; ++i) {
            for (int j = 0; j < nb; ++j) {
                double Dij = c->D[(long)(mu0 + i) * c->n_ao + nu0 + j];
                if (Dij == 0.0) return;
                for (int d = 0; d < 3; ++d) {
                    /* derivative of the first primitive along d */
                    double da = 1.0, db = 1.0;
                    for (int e = 0; e < 3; ++e) {
                        int pa = ax[i][e], pb = bx[j][e];
                        double va = ga[e][pa * n[e] + tt[e]];
                        double vb = gb[e][pb * n[e] + tt[e]];
                        if (e == d) {
                            double dva = 2.0 * p->aa * ga[e][(pa + 1) * n[e] + tt[e]];
                            if (pa > 0) dva -= pa * ga[e][(pa - 1) * n[e] + tt[e]];
                            double dvb = 2.0 * p->ab * gb[e][(pb + 1) * n[e] + tt[e]];
                            if (pb > 0) dvb -= pb * gb[e][(pb - 1) * n[e] + tt[e]];
                            da *= dva * vb;
                            db *= va * dvb;
                        } else {
                            da *= va * vb;
                            db *= va * vb;
                        }
                    }
                    gA[d] += Dij * da;
                    gB[d] += Dij * db;
                }
            }
        }
        for (int d = 0; d < 3; ++d) {
            out[3 * p->atom_a + d] += f * gA[d];
            out[3 * p->atom_b + d] += f * gB[d];
        }
    }
}

/* General cell: grid point i of a level at r = sum_d (i_d / N_d) a_d.  The
 * truncation sphere is an ellipsoid in index space; the box of indices whose
 * fractional coordinate can lie within R of P is visited point by point, and
 * each primitive is tabulated at the point itself (its Cartesian factors
 * x, y, z still separate), then the same per-point terms apply. */
static void eval_pair_general(const osys *s, const opair *p, octx *c, int tid)
{
    const int lv = p->level;
    const int *N = s->mesh + 3 * lv;
    double inv[9];
    const double det = fabs(lat_inverse(s->lat, inv));
    const double w = det / ((double)N[0] * N[1] * N[2]);
    long lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
        double u = p->P[0] * inv[d] + p->P[1] * inv[3 + d] + p->P[2] * inv[6 + d];
        double du = p->R * inv_col_norm(inv, d);
        lo[d] = (long)ceil((u - du) * N[d]);
        hi[d] = (long)floor((u + du) * N[d]);
        if (hi[d] < lo[d]) return;
    }
    if (c->nsamp > 0 && lv != c->samp_level) return;
    if ((c->mode == MODE_MAT || c->mode == MODE_MAT_TAU) && c->sp_slot &&
        c->sp_slot[(long)p->sa * s->nshell + p->sb] < 0)
        return;
    const int la = p->la, lb = p->lb, na = ncart(la), nb = ncart(lb);
    const int extra = c->mode == MODE_GRAD ? 1 : c->mode == MODE_TAU || c->mode == MODE_MAT_TAU ? 1
                      : c->mode == MODE_GRAD_TAU ? 2 : 0;
    const int ea = la + extra, eb = lb + extra;
    int ax[OR_NCART][3], bx[OR_NCART][3];
    for (int m = 0; m < na; ++m) cart_exps(la, m, &ax[m][0], &ax[m][1], &ax[m][2]);
    for (int m = 0; m < nb; ++m) cart_exps(lb, m, &bx[m][0], &bx[m][1], &bx[m][2]);
    double tga[3][OR_MAXL + 3], tgb[3][OR_MAXL + 3];
    double *ga[3] = {tga[0], tga[1], tga[2]}, *gb[3] = {tgb[0], tgb[1], tgb[2]};
    const long one[3] = {1, 1, 1}, zero[3] = {0, 0, 0};
    const double R2 = p->R * p->R;
    double *out = c->tbuf[tid];
    long nvis = 0;
    const long nlist = (c->nsamp > 0) ? c->nsamp : 1;
    for (long sidx = 0; sidx < nlist; ++sidx) {
        long ulo[3], ustep[3];
        if (c->nsamp > 0) {
            long f = c->samp_idx[sidx];
            long wv[3] = {f / ((long)N[1] * N[2]), (f / N[2]) % N[1], f % N[2]};
            for (int d = 0; d < 3; ++d) {
                long u = wv[d] + N[d] * (long)ceil((double)(lo[d] - wv[d]) / N[d]);
                while (u < lo[d]) u += N[d];
                while (u - N[d] >= lo[d]) u -= N[d];
                ulo[d] = u;
                ustep[d] = N[d];
            }
        } else {
            for (int d = 0; d < 3; ++d) { ulo[d] = lo[d]; ustep[d] = 1; }
        }
        for (long i0 = ulo[0]; i0 <= hi[0]; i0 += ustep[0])
            for (long i1 = ulo[1]; i1 <= hi[1]; i1 += ustep[1])
                for (long i2 = ulo[2]; i2 <= hi[2]; i2 += ustep[2]) {
                    const double f0 = (double)i0 / N[0], f1 = (double)i1 / N[1], f2 = (double)i2 / N[2];
                    double r[3], d2 = 0.0;
                    for (int k = 0; k < 3; ++k) {
                        r[k] = f0 * s->lat[k] + f1 * s->lat[3 + k] + f2 * s->lat[6 + k];
                        const double t = r[k] - p->P[k];
                        d2 += t * t;
                    }
                    if (d2 > R2) continue;
                    ++nvis;
                    /* (x - C)^q exp(-a (x - C)^2) of each primitive at this point, per axis */
                    for (int k = 0; k < 3; ++k) {
                        double dx = r[k] - p->A[k], e = exp(-p->aa * dx * dx), pw = 1.0;
                        for (int q = 0; q <= ea; ++q) { ga[k][q] = pw * e; pw *= dx; }
                        dx = r[k] - p->B[k];
                        e = exp(-p->ab * dx * dx);
                        pw = 1.0;
                        for (int q = 0; q <= eb; ++q) { gb[k][q] = pw * e; pw *= dx; }
                    }
                    const long wflat = (lmod(i0, N[0]) * N[1] + lmod(i1, N[1])) * N[2] + lmod(i2, N[2]);
                    point_terms(s, c, p, ga, gb, one, zero, ax, bx, wflat, sidx, w, out);
                }
    }
    c->counts[tid * OR_NCNT + 5 * la + lb] += nvis;
}

static void eval_pair(const osys *s, const opair *p, void *vctx, int tid)
{
    octx *c = (octx *)vctx;
    if (s->lat) {
        eval_pair_general(s, p, c, tid);
        return;
    }
    const int lv = p->level;
    const int *N = s->mesh + 3 * lv;
    double h[3];
    for (int d = 0; d < 3; ++d) h[d] = s->cell[d] / N[d];
    double w = s->cell[0] * s->cell[1] * s->cell[2] / ((double)N[0] * N[1] * N[2]);

    long lo[3], hi[3], n[3];
    for (int d = 0; d < 3; ++d) {
        lo[d] = (long)ceil((p->P[d] - p->R) / h[d]);
        hi[d] = (long)floor((p->P[d] + p->R) / h[d]);
        n[d] = hi[d] - lo[d] + 1;
        if (n[d] <= 0) return;
    }
    /* sampled outputs: a pair image that cannot contribute is skipped before
     * anything is tabulated */
    if (c->nsamp > 0 && lv != c->samp_level) return;
    if ((c->mode == MODE_MAT || c->mode == MODE_MAT_TAU) && c->sp_slot &&
        c->sp_slot[(long)p->sa * s->nshell + p->sb] < 0)
        return;
    const int la = p->la, lb = p->lb, na = ncart(la), nb = ncart(lb);
    /* table depth: the powers the mode's derivatives reach */
    const int extra = c->mode == MODE_GRAD ? 1 : c->mode == MODE_TAU || c->mode == MODE_MAT_TAU ? 1
                      : c->mode == MODE_GRAD_TAU ? 2 : 0;
    const int ea = la + extra;
    const int eb = lb + extra;
    double *ga[3], *gb[3];
    for (int d = 0; d < 3; ++d) {
        ga[d] = (double *)malloc(sizeof(double) * (ea + 1) * n[d]);
        gb[d] = (double *)malloc(sizeof(double) * (eb + 1) * n[d]);
        tab1d(p->A[d], p->aa, h[d], lo[d], n[d], ea, ga[d]);
        tab1d(p->B[d], p->ab, h[d], lo[d], n[d], eb, gb[d]);
    }
    int ax[OR_NCART][3], bx[OR_NCART][3];
    for (int m = 0; m < na; ++m) cart_exps(la, m, &ax[m][0], &ax[m][1], &ax[m][2]);
    for (int m = 0; m < nb; ++m) cart_exps(lb, m, &bx[m][0], &bx[m][1], &bx[m][2]);
    const double R2 = p->R * p->R;
    double *out = c->tbuf[tid];
    long nvis = 0;

    /* The point set: either every unwrapped point of the bounding box, or the
     * unwrapped images of the sampled wrapped points that fall in the box. */
    long nlist = (c->nsamp > 0) ? c->nsamp : 1;
    if (c->nsamp > 0 && lv != c->samp_level) goto done;
    for (long sidx = 0; sidx < nlist; ++sidx) {
        long ulo[3], uhi[3], ustep[3];
        if (c->nsamp > 0) {
            long f = c->samp_idx[sidx];
            long wz = f % N[2], wy = (f / N[2]) % N[1], wx = f / ((long)N[1] * N[2]);
            long wv[3] = {wx, wy, wz};
            for (int d = 0; d < 3; ++d) {
                /* first unwrapped image of wv[d] at or above lo[d] */
                long u = wv[d] + N[d] * (long)ceil((double)(lo[d] - wv[d]) / N[d]);
                while (u < lo[d]) u += N[d];
                while (u - N[d] >= lo[d]) u -= N[d];
                ulo[d] = u; uhi[d] = hi[d]; ustep[d] = N[d];
            }
        } else {
            for (int d = 0; d < 3; ++d) { ulo[d] = lo[d]; uhi[d] = hi[d]; ustep[d] = 1; }
        }
        for (long ux = ulo[0]; ux <= uhi[0]; ux += ustep[0]) {
            long tx = ux - lo[0];
            double dx = (double)ux * h[0] - p->P[0];
            for (long uy = ulo[1]; uy <= uhi[1]; uy += ustep[1]) {
                long ty = uy - lo[1];
                double dy = (double)uy * h[1] - p->P[1];
                for (long uz = ulo[2]; uz <= uhi[2]; uz += ustep[2]) {
                    long tz = uz - lo[2];
                    double dz = (double)uz * h[2] - p->P[2];
                    if (dx * dx + dy * dy + dz * dz > R2) continue;
                    ++nvis;
                    long wflat = (lmod(ux, N[0]) * N[1] + lmod(uy, N[1])) * N[2] + lmod(uz, N[2]);
                    point_terms(s, c, p, ga, gb, n, (const long[3]){tx, ty, tz}, ax, bx, wflat, sidx, w, out);
                }
            }
        }
    }
done:
    c->counts[tid * OR_NCNT + 5 * la + lb] += nvis;
    for (int d = 0; d < 3; ++d) { free(ga[d]); free(gb[d]); }
}

static int n_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

static void setup_ctx(const osys *s, octx *c, int mode)
{
    memset(c, 0, sizeof(*c));
    c->mode = mode;
    c->ao_off = (int *)malloc(sizeof(int) * (s->nshell + 1));
    c->ao_off[0] = 0;
    for (int i = 0; i < s->nshell; ++i) c->ao_off[i + 1] = c->ao_off[i] + ncart(s->shell_l[i]);
    c->n_ao = c->ao_off[s->nshell];
    c->lvl_off = (long *)malloc(sizeof(long) * (s->nlevels + 1));
    c->lvl_off[0] = 0;
    for (int i = 0; i < s->nlevels; ++i)
        c->lvl_off[i + 1] = c->lvl_off[i] + (long)s->mesh[3 * i] * s->mesh[3 * i + 1] * s->mesh[3 * i + 2];
    c->nthreads = n_threads();
    c->counts = (long *)calloc((size_t)c->nthreads * OR_NCNT, sizeof(long));
}

static int alloc_bufs(octx *c, long len)
{
    c->tlen = len;
    c->tbuf = (double **)calloc(c->nthreads, sizeof(double *));
    for (int t = 0; t < c->nthreads; ++t) {
        c->tbuf[t] = (double *)calloc((size_t)len, sizeof(double));
        if (!c->tbuf[t]) return -1;
    }
    return 0;
}

static void finish(octx *c, double *out, long *counts_out)
{
    if (out) {
        memset(out, 0, sizeof(double) * c->tlen);
        for (int t = 0; t < c->nthreads; ++t)
            for (long i = 0; i < c->tlen; ++i) out[i] += c->tbuf[t][i];
    }
    if (counts_out)
        for (int k = 0; k < OR_NCNT; ++k) {
            long acc = 0;
            for (int t = 0; t < c->nthreads; ++t) acc += c->counts[t * OR_NCNT + k];
            counts_out[k] = acc;
        }
    if (c->tbuf)
        for (int t = 0; t < c->nthreads; ++t) free(c->tbuf[t]);
    free(c->tbuf);
    free(c->ao_off);
    free(c->lvl_off);
    free(c->counts);
}

/* ------------------------------------------------------------- entry points */

/* rho on every level, concatenated in level order (C-order grids). */
int oracle_rho(const osys *s, const double *D, double *rho, long *counts)
{
    octx c;
    setup_ctx(s, &c, MODE_RHO);
    c.D = D;
    if (alloc_bufs(&c, c.lvl_off[s->nlevels])) { finish(&c, NULL, NULL); return -1; }
    for_each_pair(s, eval_pair, &c);
    finish(&c, rho, counts);
    return 0;
}

/* rho at sampled wrapped points (flat C-order indices) of one level. */
int oracle_rho_points(const osys *s, const double *D, int level, long npts,
                      const long *idx, double *out, long *counts)
{
    octx c;
    setup_ctx(s, &c, MODE_RHO);
    c.D = D;
    c.samp_level = level;
    c.nsamp = npts;
    c.samp_idx = idx;
    if (alloc_bufs(&c, npts)) { finish(&c, NULL, NULL); return -1; }
    if (npts > 0) for_each_pair(s, eval_pair, &c);
    finish(&c, out, counts);
    return 0;
}

/* Full matrix M (n_ao x n_ao) from concatenated level potentials. */
int oracle_mat(const osys *s, const double *V, double *M, long *counts)
{
    octx c;
    setup_ctx(s, &c, MODE_MAT);
    c.V = V;
    if (alloc_bufs(&c, (long)c.n_ao * c.n_ao)) { finish(&c, NULL, NULL); return -1; }
    for_each_pair(s, eval_pair, &c);
    finish(&c, M, counts);
    return 0;
}

/* Shell-pair blocks of M.  sp_slot[a*nshell+b] gives the offset of block (a,b)
 * in out (row-major na x nb), or -1 for blocks that are not wanted. */
int oracle_mat_blocks(const osys *s, const double *V, const long *sp_slot, long out_len,
                      double *out, long *counts)
{
    octx c;
    setup_ctx(s, &c, MODE_MAT);
    c.V = V;
    c.sp_slot = sp_slot;
    if (alloc_bufs(&c, out_len)) { finish(&c, NULL, NULL); return -1; }
    for_each_pair(s, eval_pair, &c);
    finish(&c, out, counts);
    return 0;
}

/* dE/dR (natm x 3) of E = sum_l w_l <v_l, rho_l(D)> at fixed D and v. */
int oracle_grad(const osys *s, const double *D, const double *V, double *grad, long *counts)
{
    octx c;
    setup_ctx(s, &c, MODE_GRAD);
    c.D = D;
    c.V = V;
    if (alloc_bufs(&c, 3L * s->natm)) { finish(&c, NULL, NULL); return -1; }
    for_each_pair(s, eval_pair, &c);
    finish(&c, grad, counts);
    return 0;
}

/* Kinetic energy density tau on every level, concatenated in level order. */
int oracle_tau(const osys *s, const double *D, double *tau, long *counts)
{
    octx c;
    setup_ctx(s, &c, MODE_TAU);
    c.D = D;
    if (alloc_bufs(&c, c.lvl_off[s->nlevels])) { finish(&c, NULL, NULL); return -1; }
    for_each_pair(s, eval_pair, &c);
    finish(&c, tau, counts);
    return 0;
}

/* tau at sampled wrapped points (flat C-order indices) of one level. */
int oracle_tau_points(const osys *s, const double *D, int level, long npts,
                      const long *idx, double *out, long *counts)
{
    octx c;
    setup_ctx(s, &c, MODE_TAU);
    c.D = D;
    c.samp_level = level;
    c.nsamp = npts;
    c.samp_idx = idx;
    if (alloc_bufs(&c, npts)) { finish(&c, NULL, NULL); return -1; }
    if (npts > 0) for_each_pair(s, eval_pair, &c);
    finish(&c, out, counts);
    return 0;
}

/* The tau term of the matrix, from concatenated level potentials vtau. */
int oracle_mat_tau(const osys *s, const double *V, double *M, long *counts)
{
    octx c;
    setup_ctx(s, &c, MODE_MAT_TAU);
    c.V = V;
    if (alloc_bufs(&c, (long)c.n_ao * c.n_ao)) { finish(&c, NULL, NULL); return -1; }
    for_each_pair(s, eval_pair, &c);
    finish(&c, M, counts);
    return 0;
}

/* Shell-pair blocks of the tau term of the matrix (as oracle_mat_blocks). */
int oracle_mat_tau_blocks(const osys *s, const double *V, const long *sp_slot, long out_len,
                          double *out, long *counts)
{
    octx c;
    setup_ctx(s, &c, MODE_MAT_TAU);
    c.V = V;
    c.sp_slot = sp_slot;
    if (alloc_bufs(&c, out_len)) { finish(&c, NULL, NULL); return -1; }
    for_each_pair(s, eval_pair, &c);
    finish(&c, out, counts);
    return 0;
}

/* dE_tau/dR (natm x 3) of E_tau = sum_l w_l <vtau_l, tau_l(D)> at fixed D, vtau. */
int oracle_grad_tau(const osys *s, const double *D, const double *V, double *grad, long *counts)
{
    octx c;
    setup_ctx(s, &c, MODE_GRAD_TAU);
    c.D = D;
    c.V = V;
    if (alloc_bufs(&c, 3L * s->natm)) { finish(&c, NULL, NULL); return -1; }
    for_each_pair(s, eval_pair, &c);
    finish(&c, grad, counts);
    return 0;
}

/* Number of pair images per level (ordered pairs), for cross-checks. */
typedef struct { long *cnt; int nthreads; int nlevels; } cctx;
static void count_pair(const osys *s, const opair *p, void *vctx, int tid)
{
    cctx *c = (cctx *)vctx;
    (void)s;
    c->cnt[(long)tid * c->nlevels + p->level] += 1;
}

int oracle_count_pairs(const osys *s, long *per_level)
{
    cctx c;
    c.nthreads = n_threads();
    c.nlevels = s->nlevels;
    c.cnt = (long *)calloc((size_t)c.nthreads * s->nlevels, sizeof(long));
    for_each_pair(s, count_pair, &c);
    for (int l = 0; l < s->nlevels; ++l) {
        long a = 0;
        for (int t = 0; t < c.nthreads; ++t) a += c.cnt[(long)t * s->nlevels + l];
        per_level[l] = a;
    }
    free(c.cnt);
    return 0;
}

int oracle_num_threads(void) { return n_threads(); }

/* Threads of the following calls (n >= 1); for timing runs at a set width. */
int oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
    return n_threads();
}
