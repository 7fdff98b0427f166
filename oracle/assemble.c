/*
 * Reference oracle (TEST INFRASTRUCTURE ONLY): FP64 row-wise weighted-quadrature
 * assembly written out as direct sums, for checking the product library.
 *
 * Paper: Barton, Puzyrev, Deng, Calo, "Efficient mass and stiffness matrix assembly
 * via weighted Gaussian quadrature rules for B-splines" (arXiv 1710.01048).
 *
 * Row i = (i_1..i_d) of the mass matrix uses the weight function B_i and its own
 * rule (nodes x, weights w) in every direction (Sec. 3, eq:Decompo, eq:GaussQuadSys):
 *
 *   M[i][s] = sum over all q in [0,Q)^d of
 *             c(x_q) * prod_k  w_k[i_k][q_k] B_{i_k}(x_k[i_k][q_k]) B_{j_k}(x_k[i_k][q_k]),
 *
 * with column j_k = i_k - p + s_k.  The stiffness matrix with a diagonal coefficient
 * A = diag(a_1..a_d) (eq:Stiffness after folding the geometry into a_k) is the sum
 * over directions k' of the same expression with the stiffness rule and B' in
 * direction k', the mass rule and B elsewhere, and a_{k'} sampled on that mixed grid.
 * Slots whose column falls outside [0, n_k) are written as 0.
 *
 * The adjoint of both maps (the gradient of <G_M, M> + <G_K, K> with respect to every
 * coefficient sample) is the same product of factors summed over slots instead of
 * points.
 *
 * Nothing here is sum-factorized: each output is one flat loop over the Q^d points
 * (or the S^d slots) of its row.  Basis values come from this file's own Cox-de Boor
 * recursion.  OpenMP splits the work over rows only.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define MAXD 3
#define MAXP 3
#define MAXQ (MAXP + 1)
#define MAXS (2 * MAXP + 1)

/* Open knot vector on [0,1] (eq:Gmap3): p+1 zeros, the interior breakpoints, p+1 ones.
 * breaks == NULL: uniform, k/N_el; else breaks[0..N_el] (0 = b_0 < ... < b_N = 1). */
static void make_knots(int p, int64_t n_el, const double *breaks, double *t)
{
    int64_t m = 0;
    for (int k = 0; k < p; ++k) t[m++] = 0.0;
    for (int64_t k = 0; k <= n_el; ++k) t[m++] = breaks ? breaks[k] : (double)k / (double)n_el;
    for (int k = 0; k < p; ++k) t[m++] = 1.0;
}

/* Cox-de Boor: value of B_{i,deg} at x on knots t (length n_knots).  Degree-0 pieces
 * are right-continuous; the last non-empty interval is closed at the right end. */
static double bspline(const double *t, int64_t n_knots, int64_t i, int deg, double x)
{
    double v[MAXP + 2];
    const double last = t[n_knots - 1];
    for (int k = 0; k <= deg; ++k) {
        double a = t[i + k], b = t[i + k + 1];
        int inside = (a <= x && x < b) || (x == last && b == last && a < b);
        v[k] = inside ? 1.0 : 0.0;
    }
    for (int r = 1; r <= deg; ++r) {
        for (int k = 0; k <= deg - r; ++k) {
            int64_t ii = i + k;
            double term = 0.0;
            double d1 = t[ii + r] - t[ii];
            if (d1 != 0.0) term += (x - t[ii]) / d1 * v[k];
            double d2 = t[ii + r + 1] - t[ii + 1];
            if (d2 != 0.0) term += (t[ii + r + 1] - x) / d2 * v[k + 1];
            v[k] = term;
        }
    }
    return v[0];
}

/* d/dx B_{i,p}(x) = p/(t_{i+p}-t_i) B_{i,p-1} - p/(t_{i+p+1}-t_{i+1}) B_{i+1,p-1} */
static double bspline_deriv(const double *t, int64_t n_knots, int64_t i, int p, double x)
{
    double out = 0.0;
    double d1 = t[i + p] - t[i];
    if (d1 != 0.0) out += p / d1 * bspline(t, n_knots, i, p - 1, x);
    double d2 = t[i + p + 1] - t[i + 1];
    if (d2 != 0.0) out -= p / d2 * bspline(t, n_knots, i + 1, p - 1, x);
    return out;
}

typedef struct {
    int d, p, Q, S;
    int64_t n[MAXD];        /* basis functions per direction = N_el + p */
    int64_t N[MAXD];        /* grid points per direction = n * Q */
    double *knots[MAXD];
    int64_t n_knots[MAXD];
} space_t;

static void space_free(space_t *sp)
{
    for (int k = 0; k < MAXD; ++k) { free(sp->knots[k]); sp->knots[k] = NULL; }
}

static int space_init(space_t *sp, int d, int p, const int64_t *n_el, const double *const *brk)
{
    memset(sp, 0, sizeof(*sp));
    if (d < 1 || d > MAXD || p < 1 || p > MAXP) return -1;
    sp->d = d; sp->p = p; sp->Q = p + 1; sp->S = 2 * p + 1;
    for (int k = 0; k < d; ++k) {
        if (n_el[k] < 1) { space_free(sp); return -1; }
        sp->n[k] = n_el[k] + p;
        sp->N[k] = sp->n[k] * sp->Q;
        sp->n_knots[k] = n_el[k] + 1 + 2 * p;
        sp->knots[k] = (double *)malloc(sizeof(double) * (size_t)sp->n_knots[k]);
        if (!sp->knots[k]) { space_free(sp); return -2; }
        make_knots(p, n_el[k], brk ? brk[k] : NULL, sp->knots[k]);
    }
    return 0;
}


/* Per-direction factor of the integrand of row index ik at its q-th node, for slot s:
 *   w[ik][q] * phi_{ik}(x) * phi_{ik-p+s}(x),  phi = B (mass rule) or B' (stiffness rule).
 * Out-of-range columns give 0. */
static void direction_factors(const space_t *sp, int k, int64_t ik, const double *x, const double *w,
                              int deriv, double f[MAXQ][MAXS])
{
    const int p = sp->p;
    for (int q = 0; q < sp->Q; ++q) {
        double xq = x[ik * sp->Q + q];
        double wq = w[ik * sp->Q + q];
        double own = deriv ? bspline_deriv(sp->knots[k], sp->n_knots[k], ik, p, xq)
                           : bspline(sp->knots[k], sp->n_knots[k], ik, p, xq);
        for (int s = 0; s < sp->S; ++s) {
            int64_t j = ik - p + s;
            if (j < 0 || j >= sp->n[k]) { f[q][s] = 0.0; continue; }
            double other = deriv ? bspline_deriv(sp->knots[k], sp->n_knots[k], j, p, xq)
                                 : bspline(sp->knots[k], sp->n_knots[k], j, p, xq);
            f[q][s] = wq * own * other;
        }
    }
}

static void unflatten(const space_t *sp, int64_t row, int64_t *idx)
{
    for (int k = sp->d - 1; k >= 0; --k) { idx[k] = row % sp->n[k]; row /= sp->n[k]; }
}

static int slot_valid(const space_t *sp, const int64_t *idx, const int *s)
{
    for (int k = 0; k < sp->d; ++k) {
        int64_t j = idx[k] - sp->p + s[k];
        if (j < 0 || j >= sp->n[k]) return 0;
    }
    return 1;
}

/* Grid offset of point (i_k*Q + q_k)_k in a C-ordered [N_1..N_d] array. */
static int64_t grid_offset(const space_t *sp, const int64_t *idx, const int *q)
{
    int64_t off = 0;
    for (int k = 0; k < sp->d; ++k) off = off * sp->N[k] + idx[k] * sp->Q + q[k];
    return off;
}

static void decode(int code, int base, int d, int *digits)
{
    for (int k = d - 1; k >= 0; --k) { digits[k] = code % base; code /= base; }
}

static int ipow(int b, int e) { int r = 1; while (e-- > 0) r *= b; return r; }

/*
 * Forward assembly of the listed rows (the exported entry points follow).
 *   xM[k], wM[k]: mass-rule nodes and weights of direction k, [n_k * Q] each.
 *   xK[k], wK[k]: stiffness-rule nodes and weights (only read when K_out != NULL).
 *   c: mass coefficient on the all-mass grid (read when M_out != NULL).
 *   a[k]: stiffness coefficient k on the grid with the stiffness rule in direction k.
 *   rows: flat C-order row indices, n_list of them; NULL means every row in order.
 *   M_out, K_out: [n_list][S^d] (either may be NULL).
 * Returns 0, or -1 for bad arguments, -2 when out of memory.
 */
static int assemble_impl(int d, int p, const int64_t *n_el, const double *const *brk,
                         const double *const *xM, const double *const *wM,
                         const double *const *xK, const double *const *wK,
                         const double *c, const double *const *a, int per_row,
                         const int64_t *rows, int64_t n_list,
                         double *M_out, double *K_out)
{
    space_t sp;
    int rc = space_init(&sp, d, p, n_el, brk);
    if (rc) return rc;
    int64_t n_rows = 1;
    for (int k = 0; k < d; ++k) n_rows *= sp.n[k];
    if (!rows) n_list = n_rows;
    const int QD = ipow(sp.Q, d), SD = ipow(sp.S, d);
    int bad = 0;

    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < n_list; ++r) {
        int64_t row = rows ? rows[r] : r;
        if (row < 0 || row >= n_rows) { bad = 1; continue; }
        int64_t idx[MAXD];
        unflatten(&sp, row, idx);
        double fM[MAXD][MAXQ][MAXS], fK[MAXD][MAXQ][MAXS];
        for (int k = 0; k < d; ++k) {
            direction_factors(&sp, k, idx[k], xM[k], wM[k], 0, fM[k]);
            if (K_out) direction_factors(&sp, k, idx[k], xK[k], wK[k], 1, fK[k]);
        }
        for (int sc = 0; sc < SD; ++sc) {
            int s[MAXD];
            decode(sc, sp.S, d, s);
            int valid = slot_valid(&sp, idx, s);
            if (M_out) {
                double acc = 0.0;
                if (valid) {
                    for (int qc = 0; qc < QD; ++qc) {
                        int q[MAXD];
                        decode(qc, sp.Q, d, q);
                        double prod = c[per_row ? r * QD + qc : grid_offset(&sp, idx, q)];
                        for (int k = 0; k < d; ++k) prod *= fM[k][q[k]][s[k]];
                        acc += prod;
                    }
                }
                M_out[r * SD + sc] = acc;
            }
            if (K_out) {
                double acc = 0.0;
                if (valid) {
                    for (int kk = 0; kk < d; ++kk) {
                        for (int qc = 0; qc < QD; ++qc) {
                            int q[MAXD];
                            decode(qc, sp.Q, d, q);
                            double prod = a[kk][per_row ? r * QD + qc : grid_offset(&sp, idx, q)];
                            for (int k = 0; k < d; ++k)
                                prod *= (k == kk) ? fK[k][q[k]][s[k]] : fM[k][q[k]][s[k]];
                            acc += prod;
                        }
                    }
                }
                K_out[r * SD + sc] = acc;
            }
        }
    }
    space_free(&sp);
    return bad ? -1 : 0;
}

/* brk: NULL (uniform knots in every direction) or per-direction breakpoints, each
 * NULL (uniform) or breaks[0..N_el] of that direction. */
int oracle_assemble(int d, int p, const int64_t *n_el, const double *const *brk,
                    const double *const *xM, const double *const *wM,
                    const double *const *xK, const double *const *wK,
                    const double *c, const double *const *a,
                    const int64_t *rows, int64_t n_list,
                    double *M_out, double *K_out)
{
    return assemble_impl(d, p, n_el, brk, xM, wM, xK, wK, c, a, 0, rows, n_list, M_out, K_out);
}

/* Same as oracle_assemble, but the coefficients come per listed row: c[r][q] and
 * a[k][r][q] hold the samples at the Q^d points of row rows[r] (q in C order), so
 * a few rows of a very large space need no full grid on the host. */
int oracle_assemble_rows(int d, int p, const int64_t *n_el, const double *const *brk,
                         const double *const *xM, const double *const *wM,
                         const double *const *xK, const double *const *wK,
                         const double *c, const double *const *a,
                         const int64_t *rows, int64_t n_list,
                         double *M_out, double *K_out)
{
    if (!rows) return -1;
    return assemble_impl(d, p, n_el, brk, xM, wM, xK, wK, c, a, 1, rows, n_list, M_out, K_out);
}

/*
 * Adjoint of the listed rows: with L = <G_M, M> + <G_K, K>,
 *   dc[r][q]    = dL/dc at the q-th point of row rows[r]    (q in C order over [0,Q)^d),
 *   da[k][r][q] = dL/da_k at the q-th point of that row on a_k's grid.
 * gM, gK are [n_list][S^d] rows of the upstream gradient; slots whose column falls
 * outside the space are ignored.  Either side may be NULL (its outputs are then not
 * written).  absolute != 0 sums the magnitudes of the same terms instead,
 * sum_s |G[s]| prod_k |factor_k|: the scale against which a rounding error of one
 * gradient entry is measured.  Returns 0, -1 for bad arguments, -2 when out of memory.
 */
static int adjoint_impl(int d, int p, const int64_t *n_el, const double *const *brk,
                        const double *const *xM, const double *const *wM,
                        const double *const *xK, const double *const *wK,
                        const int64_t *rows, int64_t n_list,
                        const double *gM, const double *gK,
                        double *dc, double *const *da, int absolute)
{
    space_t sp;
    int rc = space_init(&sp, d, p, n_el, brk);
    if (rc) return rc;
    int64_t n_rows = 1;
    for (int k = 0; k < d; ++k) n_rows *= sp.n[k];
    if (!rows) n_list = n_rows;
    const int QD = ipow(sp.Q, d), SD = ipow(sp.S, d);
    int bad = 0;

    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < n_list; ++r) {
        int64_t row = rows ? rows[r] : r;
        if (row < 0 || row >= n_rows) { bad = 1; continue; }
        int64_t idx[MAXD];
        unflatten(&sp, row, idx);
        double fM[MAXD][MAXQ][MAXS], fK[MAXD][MAXQ][MAXS];
        for (int k = 0; k < d; ++k) {
            direction_factors(&sp, k, idx[k], xM[k], wM[k], 0, fM[k]);
            if (gK) direction_factors(&sp, k, idx[k], xK[k], wK[k], 1, fK[k]);
        }
        for (int qc = 0; qc < QD; ++qc) {
            int q[MAXD];
            decode(qc, sp.Q, d, q);
            if (gM) {
                double acc = 0.0;
                for (int sc = 0; sc < SD; ++sc) {
                    int s[MAXD];
                    decode(sc, sp.S, d, s);
                    if (!slot_valid(&sp, idx, s)) continue;
                    double prod = absolute ? fabs(gM[r * SD + sc]) : gM[r * SD + sc];
                    for (int k = 0; k < d; ++k) prod *= absolute ? fabs(fM[k][q[k]][s[k]]) : fM[k][q[k]][s[k]];
                    acc += prod;
                }
                dc[r * QD + qc] = acc;
            }
            if (gK) {
                for (int kk = 0; kk < d; ++kk) {
                    double acc = 0.0;
                    for (int sc = 0; sc < SD; ++sc) {
                        int s[MAXD];
                        decode(sc, sp.S, d, s);
                        if (!slot_valid(&sp, idx, s)) continue;
                        double prod = absolute ? fabs(gK[r * SD + sc]) : gK[r * SD + sc];
                        for (int k = 0; k < d; ++k) {
                            const double f = (k == kk) ? fK[k][q[k]][s[k]] : fM[k][q[k]][s[k]];
                            prod *= absolute ? fabs(f) : f;
                        }
                        acc += prod;
                    }
                    da[kk][r * QD + qc] = acc;
                }
            }
        }
    }
    space_free(&sp);
    return bad ? -1 : 0;
}

int oracle_adjoint(int d, int p, const int64_t *n_el, const double *const *brk,
                   const double *const *xM, const double *const *wM,
                   const double *const *xK, const double *const *wK,
                   const int64_t *rows, int64_t n_list,
                   const double *gM, const double *gK,
                   double *dc, double *const *da)
{
    return adjoint_impl(d, p, n_el, brk, xM, wM, xK, wK, rows, n_list, gM, gK, dc, da, 0);
}

/* Same arguments as oracle_adjoint; writes sum_s |G[s]| prod_k |factor_k| per point. */
int oracle_adjoint_abs(int d, int p, const int64_t *n_el, const double *const *brk,
                       const double *const *xM, const double *const *wM,
                       const double *const *xK, const double *const *wK,
                       const int64_t *rows, int64_t n_list,
                       const double *gM, const double *gK,
                       double *dc, double *const *da)
{
    return adjoint_impl(d, p, n_el, brk, xM, wM, xK, wK, rows, n_list, gM, gK, dc, da, 1);
}
