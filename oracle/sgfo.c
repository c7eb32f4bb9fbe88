/*
 * sgfo.c -- plain FP64 CPU oracle for the shifted-COCG Green's-function path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no source
 * with the GPU library: every step below is written out plainly, in the order
 * the method defines it, with no blocking, fusion or reordering.
 *
 * What it computes (paper, Introduction): instead of the generalized
 * eigenproblem H y = lambda S y, solve the generalized shifted linear
 * equations (z S - H) x = b for many complex energies z, at a cost
 * proportional to the number of atoms.  Here b = e_j is one basis column, the
 * system is restricted to the local subspace L(j) (atoms within a radius of
 * the atom that carries orbital j), and all shifts share one Krylov subspace
 * (shifted COCG: collinear residuals across shifts, unconjugated bilinear
 * form).  Outputs are the Green's-function elements G_ij(z_k) = x^k_i on the
 * projection rows P(j) and the density-matrix entries
 *     rho_ij = -(1/pi) sum_k Im(w_k G_ij(z_k)).
 *
 * Layout conventions (shared by definition with the GPU library's header, not
 * by code): block-sparse row (BSR) matrices with 4x4 real blocks, one block
 * row per atom, row_ptr int32[n+1], col int32[nnzb] sorted within each row,
 * values double[nnzb][4][4] row-major.  Global orbital = 4*atom + o with
 * o = (s, px, py, pz).  Complex arrays are interleaved (re, im) doubles.
 */
#define _GNU_SOURCE
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

enum { SGFO_OK = 0, SGFO_EINVAL = -1, SGFO_ENOMEM = -2 };
enum { SGFO_CONVERGED = 0, SGFO_MAXITER = 1, SGFO_BREAKDOWN = 2, SGFO_NONFINITE = 3 };

typedef struct {
    double e_s, e_p, v_sss, v_sps, v_pps, v_ppp;
    double r0, power, r_cut;
    int32_t overlap;
    double s_amp, s_decay;
} sgfo_tb_params;

/* ------------------------------------------------------------------------ */
/* Distances.  Squared distances are always formed as (dx*dx + dy*dy) + dz*dz */
/* with no fused multiply-add (the library is built with -ffp-contract=off),  */
/* so a cutoff test decides the same way wherever it is evaluated.            */
/* ------------------------------------------------------------------------ */
static double dist2(const double *a, const double *b)
{
    double dx = b[0] - a[0], dy = b[1] - a[1], dz = b[2] - a[2];
    return (dx * dx + dy * dy) + dz * dz;
}

/* ------------------------------------------------------------------------ */
/* Neighbour search: cell list with cell edge r_cut.  Pair (a, b), a != b, is  */
/* bonded when |R_b - R_a|^2 <= r_cut^2.  Each row's neighbours end up sorted. */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t nx, ny, nz;
    double lo[3], h;
    int64_t *start; /* n_cells + 1 */
    int64_t *atoms; /* atoms sorted by cell */
} cells_t;

static int64_t cell_coord(double x, double lo, double h, int64_t n)
{
    int64_t c = (int64_t)floor((x - lo) / h);
    if (c < 0) c = 0;
    if (c >= n) c = n - 1;
    return c;
}

static int cells_build(cells_t *cl, int64_t n, const double *xyz, double h)
{
    double hi[3];
    for (int d = 0; d < 3; ++d) { cl->lo[d] = xyz[d]; hi[d] = xyz[d]; }
    for (int64_t a = 1; a < n; ++a)
        for (int d = 0; d < 3; ++d) {
            if (xyz[3 * a + d] < cl->lo[d]) cl->lo[d] = xyz[3 * a + d];
            if (xyz[3 * a + d] > hi[d]) hi[d] = xyz[3 * a + d];
        }
    cl->h = h;
    cl->nx = (int64_t)floor((hi[0] - cl->lo[0]) / h) + 1;
    cl->ny = (int64_t)floor((hi[1] - cl->lo[1]) / h) + 1;
    cl->nz = (int64_t)floor((hi[2] - cl->lo[2]) / h) + 1;
    int64_t nc = cl->nx * cl->ny * cl->nz;
    cl->start = calloc((size_t)nc + 1, sizeof(int64_t));
    cl->atoms = malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    int64_t *cid = malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    int64_t *fill = calloc((size_t)nc, sizeof(int64_t));
    if (!cl->start || !cl->atoms || !cid || !fill) { free(cid); free(fill); return SGFO_ENOMEM; }
    for (int64_t a = 0; a < n; ++a) {
        int64_t cx = cell_coord(xyz[3 * a + 0], cl->lo[0], h, cl->nx);
        int64_t cy = cell_coord(xyz[3 * a + 1], cl->lo[1], h, cl->ny);
        int64_t cz = cell_coord(xyz[3 * a + 2], cl->lo[2], h, cl->nz);
        cid[a] = (cx * cl->ny + cy) * cl->nz + cz;
        cl->start[cid[a] + 1]++;
    }
    for (int64_t c = 0; c < nc; ++c) cl->start[c + 1] += cl->start[c];
    for (int64_t a = 0; a < n; ++a) cl->atoms[cl->start[cid[a]] + fill[cid[a]]++] = a;
    free(cid);
    free(fill);
    return SGFO_OK;
}

static void cells_free(cells_t *cl) { free(cl->start); free(cl->atoms); }

static int cmp_i32(const void *x, const void *y)
{
    int32_t a = *(const int32_t *)x, b = *(const int32_t *)y;
    return (a > b) - (a < b);
}

/* Neighbours of atom a (a excluded) within r_cut; returns count, fills out if non-NULL. */
static int64_t neighbours(const cells_t *cl, const double *xyz, int64_t a, double r_cut, int32_t *out)
{
    int64_t cx = cell_coord(xyz[3 * a + 0], cl->lo[0], cl->h, cl->nx);
    int64_t cy = cell_coord(xyz[3 * a + 1], cl->lo[1], cl->h, cl->ny);
    int64_t cz = cell_coord(xyz[3 * a + 2], cl->lo[2], cl->h, cl->nz);
    double rc2 = r_cut * r_cut;
    int64_t k = 0;
    for (int64_t ix = cx - 1; ix <= cx + 1; ++ix) {
        if (ix < 0 || ix >= cl->nx) continue;
        for (int64_t iy = cy - 1; iy <= cy + 1; ++iy) {
            if (iy < 0 || iy >= cl->ny) continue;
            for (int64_t iz = cz - 1; iz <= cz + 1; ++iz) {
                if (iz < 0 || iz >= cl->nz) continue;
                int64_t c = (ix * cl->ny + iy) * cl->nz + iz;
                for (int64_t t = cl->start[c]; t < cl->start[c + 1]; ++t) {
                    int64_t b = cl->atoms[t];
                    if (b == a) continue;
                    if (dist2(&xyz[3 * a], &xyz[3 * b]) <= rc2) {
                        if (out) out[k] = (int32_t)b;
                        ++k;
                    }
                }
            }
        }
    }
    if (out) qsort(out, (size_t)k, sizeof(int32_t), cmp_i32);
    return k;
}

/* Number of stored blocks (diagonal included) of the bond pattern. */
int64_t sgfo_tb_nnzb(int64_t n_atoms, const double *xyz, double r_cut)
{
    if (n_atoms <= 0 || !xyz || !(r_cut > 0)) return SGFO_EINVAL;
    cells_t cl;
    if (cells_build(&cl, n_atoms, xyz, r_cut) != SGFO_OK) { cells_free(&cl); return SGFO_ENOMEM; }
    int64_t total = 0;
    for (int64_t a = 0; a < n_atoms; ++a) total += 1 + neighbours(&cl, xyz, a, r_cut, NULL);
    cells_free(&cl);
    return total;
}

/*
 * Slater-Koster two-centre block for the bond a -> b (orthogonal sp basis).
 * With direction cosines c = (R_b - R_a)/r and scale f = (r0/r)^power:
 *   H[s][s]   = Vss_sigma f
 *   H[s][pA]  =  c_A Vsp_sigma f
 *   H[pA][s]  = -c_A Vsp_sigma f
 *   H[pA][pB] = (c_A c_B (Vpp_sigma - Vpp_pi) + delta_AB Vpp_pi) f
 * (Slater and Koster, Phys. Rev. 94, 1498 (1954), Table I; distance scaling
 * after Harrison.)  The block for b -> a is the transpose.
 */
static void sk_block(const sgfo_tb_params *p, const double *ra, const double *rb, double *blk)
{
    double d[3] = {rb[0] - ra[0], rb[1] - ra[1], rb[2] - ra[2]};
    double r = sqrt(dist2(ra, rb));
    double c[3] = {d[0] / r, d[1] / r, d[2] / r};
    double f = pow(p->r0 / r, p->power);
    blk[0] = p->v_sss * f;
    for (int A = 0; A < 3; ++A) {
        blk[0 * 4 + (1 + A)] = c[A] * p->v_sps * f;
        blk[(1 + A) * 4 + 0] = -c[A] * p->v_sps * f;
        for (int B = 0; B < 3; ++B)
            blk[(1 + A) * 4 + (1 + B)] = (c[A] * c[B] * (p->v_pps - p->v_ppp) + (A == B ? p->v_ppp : 0.0)) * f;
    }
}

/* Off-diagonal overlap block: s_amp * exp(-(r - r0)/s_decay) * I4. */
static void overlap_block(const sgfo_tb_params *p, const double *ra, const double *rb, double *blk)
{
    double r = sqrt(dist2(ra, rb));
    double v = p->s_amp * exp(-(r - p->r0) / p->s_decay);
    memset(blk, 0, 16 * sizeof(double));
    for (int o = 0; o < 4; ++o) blk[o * 5] = v;
}

/*
 * Build H (and S when p->overlap) in BSR form.  onsite: optional 4*n_atoms
 * on-site energies; when NULL the diagonal block is diag(e_s, e_p, e_p, e_p).
 * s may be NULL when p->overlap == 0.  Returns nnzb or a negative error.
 */
int64_t sgfo_tb_build(int64_t n_atoms, const double *xyz, const double *onsite, const sgfo_tb_params *p,
                      int64_t nnzb_cap, int32_t *row_ptr, int32_t *col, double *h, double *s)
{
    if (n_atoms <= 0 || !xyz || !p || !row_ptr || !col || !h) return SGFO_EINVAL;
    if (p->overlap && !s) return SGFO_EINVAL;
    cells_t cl;
    if (cells_build(&cl, n_atoms, xyz, p->r_cut) != SGFO_OK) { cells_free(&cl); return SGFO_ENOMEM; }
    int32_t *nb = malloc(4096 * sizeof(int32_t));
    int64_t pos = 0;
    row_ptr[0] = 0;
    for (int64_t a = 0; a < n_atoms; ++a) {
        int64_t k = neighbours(&cl, xyz, a, p->r_cut, NULL);
        if (k + 1 > 4096 || pos + k + 1 > nnzb_cap) { free(nb); cells_free(&cl); return SGFO_EINVAL; }
        neighbours(&cl, xyz, a, p->r_cut, nb);
        nb[k] = (int32_t)a; /* the diagonal block joins the row, then the row is sorted */
        qsort(nb, (size_t)(k + 1), sizeof(int32_t), cmp_i32);
        for (int64_t t = 0; t <= k; ++t) {
            int32_t b = nb[t];
            col[pos] = b;
            double *hb = &h[16 * pos];
            if (b == a) {
                memset(hb, 0, 16 * sizeof(double));
                for (int o = 0; o < 4; ++o)
                    hb[o * 5] = onsite ? onsite[4 * a + o] : (o == 0 ? p->e_s : p->e_p);
                if (p->overlap) {
                    memset(&s[16 * pos], 0, 16 * sizeof(double));
                    for (int o = 0; o < 4; ++o) s[16 * pos + o * 5] = 1.0;
                }
            } else {
                sk_block(p, &xyz[3 * a], &xyz[3 * b], hb);
                if (p->overlap) overlap_block(p, &xyz[3 * a], &xyz[3 * b], &s[16 * pos]);
            }
            ++pos;
        }
        row_ptr[a + 1] = (int32_t)pos;
    }
    free(nb);
    cells_free(&cl);
    return pos;
}

/*
 * One-orbital chain, grouped four sites to a 4x4 block: H_ii = eps_i,
 * H_{i,i+1} = H_{i+1,i} = t, open ends.  n_sites must be a multiple of 4.
 * Returns nnzb (= 3 * n_sites/4 - 2 for more than one block row).
 */
int64_t sgfo_chain_build(int64_t n_sites, const double *eps, double t, int64_t nnzb_cap,
                         int32_t *row_ptr, int32_t *col, double *h)
{
    if (n_sites <= 0 || n_sites % 4 || !eps || !row_ptr || !col || !h) return SGFO_EINVAL;
    int64_t nb = n_sites / 4, pos = 0;
    row_ptr[0] = 0;
    for (int64_t A = 0; A < nb; ++A) {
        for (int64_t B = A - 1; B <= A + 1; ++B) {
            if (B < 0 || B >= nb) continue;
            if (pos >= nnzb_cap) return SGFO_EINVAL;
            col[pos] = (int32_t)B;
            double *blk = &h[16 * pos];
            memset(blk, 0, 16 * sizeof(double));
            for (int o = 0; o < 4; ++o)
                for (int q = 0; q < 4; ++q) {
                    int64_t i = 4 * A + o, j = 4 * B + q;
                    if (i == j) blk[o * 4 + q] = eps[i];
                    else if (i - j == 1 || j - i == 1) blk[o * 4 + q] = t;
                }
            ++pos;
        }
        row_ptr[A + 1] = (int32_t)pos;
    }
    return pos;
}

/* ------------------------------------------------------------------------ */
/* Local subspace of a column.                                                */
/* ------------------------------------------------------------------------ */

/* Atoms with |R_a - R_c| <= radius (all atoms when radius <= 0 or xyz is NULL),
 * in increasing global order.  When prune != 0 the set is further reduced to
 * the atoms connected to c through stored blocks whose two ends both lie in
 * the ball.  Returns the count; *out is malloc'ed. */
static int64_t local_atoms(int64_t n_atoms, const int32_t *row_ptr, const int32_t *col, const double *xyz,
                           int64_t c, double radius, int prune, int32_t **out)
{
    char *in_ball = calloc((size_t)n_atoms, 1);
    int64_t n_in = 0;
    double r2 = radius * radius;
    for (int64_t a = 0; a < n_atoms; ++a) {
        int keep = (radius <= 0.0 || !xyz) ? 1 : (dist2(&xyz[3 * c], &xyz[3 * a]) <= r2);
        in_ball[a] = (char)keep;
        n_in += keep;
    }
    if (prune) {
        /* breadth-first search from c over stored blocks inside the ball */
        char *seen = calloc((size_t)n_atoms, 1);
        int64_t *queue = malloc((size_t)n_in * sizeof(int64_t));
        int64_t head = 0, tail = 0;
        queue[tail++] = c;
        seen[c] = 1;
        while (head < tail) {
            int64_t a = queue[head++];
            for (int32_t t = row_ptr[a]; t < row_ptr[a + 1]; ++t) {
                int32_t b = col[t];
                if (in_ball[b] && !seen[b]) { seen[b] = 1; queue[tail++] = b; }
            }
        }
        free(queue);
        free(in_ball);
        in_ball = seen;
        n_in = tail;
    }
    int32_t *list = malloc((size_t)(n_in > 0 ? n_in : 1) * sizeof(int32_t));
    int64_t k = 0;
    for (int64_t a = 0; a < n_atoms; ++a)
        if (in_ball[a]) list[k++] = (int32_t)a;
    free(in_ball);
    *out = list;
    return k;
}

/* Index of global atom a in the sorted local list, or -1. */
static int64_t local_index(const int32_t *list, int64_t n, int32_t a)
{
    int64_t lo = 0, hi = n - 1;
    while (lo <= hi) {
        int64_t mid = (lo + hi) / 2;
        if (list[mid] == a) return mid;
        if (list[mid] < a) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

/* Projection atoms of column j (atom c): c and every atom sharing a stored
 * block with c, intersected with the local set; increasing global order. */
static int64_t projection_atoms(const int32_t *row_ptr, const int32_t *col, int64_t c,
                                const int32_t *loc, int64_t n_loc, int32_t *out)
{
    int64_t k = 0;
    for (int32_t t = row_ptr[c]; t < row_ptr[c + 1]; ++t)
        if (local_index(loc, n_loc, col[t]) >= 0) out[k++] = col[t];
    return k; /* row c's columns are sorted and include c itself */
}

/* ------------------------------------------------------------------------ */
/* Local operator: the principal sub-blocks of H (and S) on the local atoms.  */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t n_loc;          /* local atoms */
    int64_t nl;             /* local orbitals = 4 n_loc */
    int64_t *lrow;          /* n_loc + 1 */
    int64_t *lcol;          /* local column atom */
    const double **hblk;    /* pointers into global H */
    const double **sblk;    /* pointers into global S, or NULL */
} local_op;

static int local_op_build(local_op *op, const int32_t *row_ptr, const int32_t *col, const double *h,
                          const double *s, const int32_t *loc, int64_t n_loc)
{
    op->n_loc = n_loc;
    op->nl = 4 * n_loc;
    op->lrow = malloc((size_t)(n_loc + 1) * sizeof(int64_t));
    int64_t cnt = 0;
    for (int64_t A = 0; A < n_loc; ++A)
        for (int32_t t = row_ptr[loc[A]]; t < row_ptr[loc[A] + 1]; ++t)
            if (local_index(loc, n_loc, col[t]) >= 0) ++cnt;
    op->lcol = malloc((size_t)(cnt > 0 ? cnt : 1) * sizeof(int64_t));
    op->hblk = malloc((size_t)(cnt > 0 ? cnt : 1) * sizeof(double *));
    op->sblk = s ? malloc((size_t)(cnt > 0 ? cnt : 1) * sizeof(double *)) : NULL;
    int64_t k = 0;
    op->lrow[0] = 0;
    for (int64_t A = 0; A < n_loc; ++A) {
        for (int32_t t = row_ptr[loc[A]]; t < row_ptr[loc[A] + 1]; ++t) {
            int64_t B = local_index(loc, n_loc, col[t]);
            if (B < 0) continue;
            op->lcol[k] = B;
            op->hblk[k] = &h[16 * (int64_t)t];
            if (s) op->sblk[k] = &s[16 * (int64_t)t];
            ++k;
        }
        op->lrow[A + 1] = k;
    }
    return SGFO_OK;
}

static void local_op_free(local_op *op) { free(op->lrow); free(op->lcol); free(op->hblk); free(op->sblk); }

/* y = M v for the local real block matrix M (H when use_s == 0, S otherwise). */
static void local_matvec(const local_op *op, int use_s, const cplx *v, cplx *y)
{
    for (int64_t A = 0; A < op->n_loc; ++A)
        for (int o = 0; o < 4; ++o) {
            cplx acc = 0.0;
            for (int64_t t = op->lrow[A]; t < op->lrow[A + 1]; ++t) {
                const double *blk = use_s ? op->sblk[t] : op->hblk[t];
                for (int q = 0; q < 4; ++q) acc += blk[o * 4 + q] * v[4 * op->lcol[t] + q];
            }
            y[4 * A + o] = acc;
        }
}

/* Dense Cholesky S_L = C C^T of the local overlap (lower C, row-major nl x nl).
 * Returns 0, or -1 when S_L is not positive definite. */
static int local_cholesky(const local_op *op, double *C)
{
    int64_t n = op->nl;
    memset(C, 0, (size_t)(n * n) * sizeof(double));
    for (int64_t A = 0; A < op->n_loc; ++A)
        for (int64_t t = op->lrow[A]; t < op->lrow[A + 1]; ++t)
            for (int o = 0; o < 4; ++o)
                for (int q = 0; q < 4; ++q)
                    C[(4 * A + o) * n + 4 * op->lcol[t] + q] = op->sblk[t][o * 4 + q];
    for (int64_t j = 0; j < n; ++j) {
        double d = C[j * n + j];
        for (int64_t k = 0; k < j; ++k) d -= C[j * n + k] * C[j * n + k];
        if (!(d > 0.0)) return -1;
        d = sqrt(d);
        C[j * n + j] = d;
        for (int64_t i = j + 1; i < n; ++i) {
            double v = C[i * n + j];
            for (int64_t k = 0; k < j; ++k) v -= C[i * n + k] * C[j * n + k];
            C[i * n + j] = v / d;
        }
        for (int64_t i = 0; i < j; ++i) C[i * n + j] = 0.0;
    }
    return 0;
}

/* r = S_L^{-1} s by forward and back substitution with the Cholesky factor. */
static void local_solve_s(const double *C, int64_t n, const cplx *s, cplx *r)
{
    for (int64_t i = 0; i < n; ++i) {
        cplx v = s[i];
        for (int64_t k = 0; k < i; ++k) v -= C[i * n + k] * r[k];
        r[i] = v / C[i * n + i];
    }
    for (int64_t i = n - 1; i >= 0; --i) {
        cplx v = r[i];
        for (int64_t k = i + 1; k < n; ++k) v -= C[k * n + i] * r[k];
        r[i] = v / C[i * n + i];
    }
}

/* Unconjugated bilinear form u^T v. */
static cplx bilinear(const cplx *u, const cplx *v, int64_t n)
{
    cplx acc = 0.0;
    for (int64_t i = 0; i < n; ++i) acc += u[i] * v[i];
    return acc;
}

static double norm2(const cplx *u, int64_t n)
{
    double acc = 0.0;
    for (int64_t i = 0; i < n; ++i) acc += creal(u[i]) * creal(u[i]) + cimag(u[i]) * cimag(u[i]);
    return sqrt(acc);
}

static int finite_c(cplx v) { return isfinite(creal(v)) && isfinite(cimag(v)); }

/*
 * Shifted COCG for one column (b = e_jl in the local basis).
 *
 * Seed system A = S^{-1}(z_s S - H) with the S-bilinear form [u, v] = u^T S v
 * (A is symmetric in it because H and S are real symmetric).  Seed vectors:
 * s = true-space residual b - (z_s S - H) x, r = S^{-1} s, p search direction,
 * q = S p.  Shift k solves A + sigma_k I with sigma_k = z_k - z_s; its residual
 * is collinear with the seed's, r^k_n = r_n / pi^k_n, where
 *   pi^k_{n+1} = (1 + alpha_n sigma_k) pi^k_n
 *              + (alpha_n beta_{n-1} / alpha_{n-1}) (pi^k_n - pi^k_{n-1}),
 *   alpha^k_n = alpha_n pi^k_n / pi^k_{n+1},
 *   beta^k_n  = (pi^k_n / pi^k_{n+1})^2 beta_n,
 *   x^k += alpha^k_n p^k,  p^k = r_{n+1} / pi^k_{n+1} + beta^k_n p^k
 * (COCG: van der Vorst and Melissen 1990; shifted form: Frommer 2003,
 * Takayama et al. 2006).  A shift is frozen once its true-space relative
 * residual ||s_{n+1}|| / |pi^k_{n+1}| drops to tol ||b||.
 *
 * Only the rows in prow[0..np) of x^k and p^k are kept when full == 0; with
 * full != 0 every local row is kept and written to xfull (nl x ns).
 */
typedef struct {
    int32_t iters, status;
} col_result;

static col_result cocg_column(const local_op *op, const double *chol, int64_t jl, int ns, const cplx *z,
                              int seed, double tol, int max_iter, int64_t np, const int64_t *prow,
                              cplx *G /* np x ns */, double *resid /* ns */, int full, cplx *xfull,
                              cplx *s_out, cplx *pi_out)
{
    int64_t n = op->nl;
    int gen = op->sblk != NULL;
    cplx *s = calloc((size_t)n, sizeof(cplx)), *r = calloc((size_t)n, sizeof(cplx));
    cplx *p = calloc((size_t)n, sizeof(cplx)), *q = calloc((size_t)n, sizeof(cplx));
    cplx *w = calloc((size_t)n, sizeof(cplx)), *hp = calloc((size_t)n, sizeof(cplx));
    int64_t nrow = full ? n : np;
    cplx *X = calloc((size_t)(nrow * ns), sizeof(cplx)), *P = calloc((size_t)(nrow * ns), sizeof(cplx));
    cplx *pi_cur = malloc((size_t)ns * sizeof(cplx)), *pi_old = malloc((size_t)ns * sizeof(cplx));
    char *active = malloc((size_t)ns);
    col_result res = {0, SGFO_MAXITER};
    cplx zs = z[seed];

    /* start: x = 0, s_0 = b, r_0 = S^{-1} s_0, p_0 = r_0, q_0 = s_0 */
    s[jl] = 1.0;
    if (gen) local_solve_s(chol, n, s, r); else memcpy(r, s, (size_t)n * sizeof(cplx));
    memcpy(p, r, (size_t)n * sizeof(cplx));
    memcpy(q, s, (size_t)n * sizeof(cplx));
    cplx rho = bilinear(r, s, n);
    double bnorm = 1.0;
    cplx alpha_old = 1.0, beta_old = 0.0;
    for (int k = 0; k < ns; ++k) {
        pi_cur[k] = 1.0;
        pi_old[k] = 1.0;
        active[k] = 1;
        resid[k] = 1.0;
        for (int64_t i = 0; i < nrow; ++i) P[i * ns + k] = r[full ? i : prow[i]];
    }
    int n_active = ns;
    for (int it = 0; it < max_iter; ++it) {
        /* w = (z_s S - H) p = z_s q - H p */
        local_matvec(op, 0, p, hp);
        for (int64_t i = 0; i < n; ++i) w[i] = zs * q[i] - hp[i];
        cplx mu = bilinear(p, w, n);
        res.iters = it + 1;
        if (!finite_c(mu) || !finite_c(rho)) { res.status = SGFO_NONFINITE; break; }
        if (mu == 0.0) { res.status = SGFO_BREAKDOWN; break; }
        cplx alpha = rho / mu;
        for (int64_t i = 0; i < n; ++i) s[i] -= alpha * w[i];
        if (gen) local_solve_s(chol, n, s, r); else memcpy(r, s, (size_t)n * sizeof(cplx));
        cplx rho_new = bilinear(r, s, n);
        double snorm = norm2(s, n);
        cplx beta = rho_new / rho;
        for (int64_t i = 0; i < n; ++i) p[i] = r[i] + beta * p[i];
        for (int64_t i = 0; i < n; ++i) q[i] = s[i] + beta * q[i];

        for (int k = 0; k < ns; ++k) {
            if (!active[k]) continue;
            cplx sigma = z[k] - zs;
            cplx pi_new = (1.0 + alpha * sigma) * pi_cur[k] + (alpha * beta_old / alpha_old) * (pi_cur[k] - pi_old[k]);
            cplx alpha_k = alpha * pi_cur[k] / pi_new;
            cplx ratio = pi_cur[k] / pi_new;
            cplx beta_k = ratio * ratio * beta;
            for (int64_t i = 0; i < nrow; ++i) {
                X[i * ns + k] += alpha_k * P[i * ns + k];
                P[i * ns + k] = r[full ? i : prow[i]] / pi_new + beta_k * P[i * ns + k];
            }
            pi_old[k] = pi_cur[k];
            pi_cur[k] = pi_new;
            resid[k] = snorm / cabs(pi_new);
            if (resid[k] <= tol * bnorm) { active[k] = 0; --n_active; }
        }
        alpha_old = alpha;
        beta_old = beta;
        rho = rho_new;
        if (n_active == 0) { res.status = SGFO_CONVERGED; break; }
        if (snorm == 0.0) { res.status = SGFO_CONVERGED; break; } /* Krylov space exhausted */
        if (rho_new == 0.0) { res.status = SGFO_BREAKDOWN; break; }
        if (!finite_c(rho_new) || !isfinite(snorm)) { res.status = SGFO_NONFINITE; break; }
    }
    if (full) memcpy(xfull, X, (size_t)(n * ns) * sizeof(cplx));
    else memcpy(G, X, (size_t)(np * ns) * sizeof(cplx));
    if (s_out) memcpy(s_out, s, (size_t)n * sizeof(cplx));
    if (pi_out) memcpy(pi_out, pi_cur, (size_t)ns * sizeof(cplx));
    free(s); free(r); free(p); free(q); free(w); free(hp);
    free(X); free(P); free(pi_cur); free(pi_old); free(active);
    return res;
}

/* ------------------------------------------------------------------------ */
/* Public entry points.                                                       */
/* ------------------------------------------------------------------------ */

/* Subspace and projection sizes per column: n_loc[c] local atoms and
 * n_proj[c] projection rows (4 per projection atom). */
int sgfo_plan_sizes(int64_t n_atoms, const int32_t *row_ptr, const int32_t *col, const double *xyz,
                    int64_t n_cols, const int64_t *cols, double radius, const double *radius_per_col,
                    int prune, int64_t *n_loc, int64_t *n_proj, int threads)
{
    if (n_atoms <= 0 || !row_ptr || !col || n_cols < 0 || (n_cols && !cols) || !n_loc || !n_proj) return SGFO_EINVAL;
    for (int64_t c = 0; c < n_cols; ++c)
        if (cols[c] < 0 || cols[c] >= 4 * n_atoms) return SGFO_EINVAL;
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t c = 0; c < n_cols; ++c) {
        int64_t atom = cols[c] / 4;
        int32_t *loc = NULL;
        double R = radius_per_col ? radius_per_col[c] : radius;
        int64_t nloc = local_atoms(n_atoms, row_ptr, col, xyz, atom, R, prune, &loc);
        int32_t pa[4096];
        int64_t npa = projection_atoms(row_ptr, col, atom, loc, nloc, pa);
        n_loc[c] = nloc;
        n_proj[c] = 4 * npa;
        free(loc);
    }
    return SGFO_OK;
}

/*
 * Shifted solve for many columns.
 *   proj_ptr: int64[n_cols+1] (output) offsets of each column's projection rows
 *   proj_row: int32[proj_cap]  (output) global orbital index of each row
 *   G:        complex [proj_cap][n_shifts] (interleaved doubles) Green's function
 *   rho:      double  [proj_cap] density-matrix entries rho_ij = -(1/pi) sum_k Im(w_k G_ij(z_k))
 *   iters, status: int32[n_cols]; resid: double[n_cols][n_shifts]
 * z and w are interleaved complex arrays of n_shifts entries (w may be NULL).
 * s may be NULL (S = I).  max_iter <= 0 means 10 * (local orbitals);
 * seed_index < 0 means n_shifts / 2.
 */
int sgfo_shifted_solve(int64_t n_atoms, const int32_t *row_ptr, const int32_t *col, const double *h,
                       const double *s, const double *xyz, int64_t n_cols, const int64_t *cols,
                       double radius, const double *radius_per_col, int prune, int n_shifts, const double *z,
                       const double *w, double tol, int max_iter, int seed_index, int64_t proj_cap,
                       int64_t *proj_ptr, int32_t *proj_row, double *G, double *rho, int32_t *iters,
                       int32_t *status, double *resid, int threads)
{
    if (n_atoms <= 0 || !row_ptr || !col || !h || n_cols < 0 || (n_cols && !cols) || n_shifts < 1 || !z)
        return SGFO_EINVAL;
    if (!(tol > 0) || !proj_ptr || !proj_row || !G || !rho || !iters || !status || !resid) return SGFO_EINVAL;
    int seed = seed_index < 0 ? n_shifts / 2 : seed_index;
    if (seed >= n_shifts) return SGFO_EINVAL;
    for (int k = 0; k < n_shifts; ++k)
        if (!(z[2 * k + 1] > 0)) return SGFO_EINVAL;
    int64_t *n_loc = malloc((size_t)(n_cols > 0 ? n_cols : 1) * sizeof(int64_t));
    int64_t *n_proj = malloc((size_t)(n_cols > 0 ? n_cols : 1) * sizeof(int64_t));
    int rc = sgfo_plan_sizes(n_atoms, row_ptr, col, xyz, n_cols, cols, radius, radius_per_col, prune, n_loc, n_proj,
                             threads);
    if (rc) { free(n_loc); free(n_proj); return rc; }
    proj_ptr[0] = 0;
    for (int64_t c = 0; c < n_cols; ++c) proj_ptr[c + 1] = proj_ptr[c] + n_proj[c];
    if (proj_ptr[n_cols] > proj_cap) { free(n_loc); free(n_proj); return SGFO_EINVAL; }
    cplx *zc = malloc((size_t)n_shifts * sizeof(cplx)), *wc = malloc((size_t)n_shifts * sizeof(cplx));
    for (int k = 0; k < n_shifts; ++k) {
        zc[k] = z[2 * k] + I * z[2 * k + 1];
        wc[k] = w ? w[2 * k] + I * w[2 * k + 1] : 0.0;
    }
    int fail = 0;
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t c = 0; c < n_cols; ++c) {
        int64_t j = cols[c], atom = j / 4;
        int32_t *loc = NULL;
        double R = radius_per_col ? radius_per_col[c] : radius;
        int64_t nloc = local_atoms(n_atoms, row_ptr, col, xyz, atom, R, prune, &loc);
        local_op op;
        local_op_build(&op, row_ptr, col, h, s, loc, nloc);
        double *chol = NULL;
        if (s) {
            chol = malloc((size_t)(op.nl * op.nl) * sizeof(double));
            if (local_cholesky(&op, chol)) {
#ifdef _OPENMP
#pragma omp atomic write
#endif
                fail = 1;
            }
        }
        int32_t pa[4096];
        int64_t npa = projection_atoms(row_ptr, col, atom, loc, nloc, pa);
        int64_t np = 4 * npa;
        int64_t *prow = malloc((size_t)(np > 0 ? np : 1) * sizeof(int64_t));
        for (int64_t a = 0; a < npa; ++a)
            for (int o = 0; o < 4; ++o) {
                prow[4 * a + o] = 4 * local_index(loc, nloc, pa[a]) + o;
                proj_row[proj_ptr[c] + 4 * a + o] = 4 * pa[a] + o;
            }
        int64_t jl = 4 * local_index(loc, nloc, (int32_t)atom) + j % 4;
        int mi = max_iter > 0 ? max_iter : (int)(10 * op.nl);
        cplx *Gc = (cplx *)&G[2 * proj_ptr[c] * n_shifts];
        col_result cr = cocg_column(&op, chol, jl, n_shifts, zc, seed, tol, mi, np, prow, Gc,
                                    &resid[c * n_shifts], 0, NULL, NULL, NULL);
        iters[c] = cr.iters;
        status[c] = cr.status;
        for (int64_t i = 0; i < np; ++i) {
            double acc = 0.0;
            for (int k = 0; k < n_shifts; ++k) acc += cimag(wc[k] * Gc[i * n_shifts + k]);
            rho[proj_ptr[c] + i] = -acc / 3.14159265358979323846;
        }
        free(prow);
        free(chol);
        local_op_free(&op);
        free(loc);
    }
    free(zc);
    free(wc);
    free(n_loc);
    free(n_proj);
    return fail ? SGFO_EINVAL : SGFO_OK;
}

/*
 * Full-vector shifted COCG for one column: keeps x^k over every local row.
 * Outputs: loc_atoms int32[n_loc] (caller sizes it from sgfo_plan_sizes),
 * x complex [nl][n_shifts], s_final complex [nl], pi_final complex [n_shifts],
 * resid double[n_shifts]; *iters and *status.  Used for the collinearity
 * check b - (z_k S - H) x^k = s / pi^k and for variational estimates.
 */
int sgfo_solve_full(int64_t n_atoms, const int32_t *row_ptr, const int32_t *col, const double *h, const double *s,
                    const double *xyz, int64_t j, double radius, int prune, int n_shifts, const double *z, double tol,
                    int max_iter, int seed_index, int64_t loc_cap, int32_t *loc_atoms, double *x, double *s_final,
                    double *pi_final, double *resid, int32_t *iters, int32_t *status)
{
    if (n_atoms <= 0 || !row_ptr || !col || !h || j < 0 || j >= 4 * n_atoms || n_shifts < 1 || !z) return SGFO_EINVAL;
    int seed = seed_index < 0 ? n_shifts / 2 : seed_index;
    if (seed >= n_shifts) return SGFO_EINVAL;
    int32_t *loc = NULL;
    int64_t nloc = local_atoms(n_atoms, row_ptr, col, xyz, j / 4, radius, prune, &loc);
    if (nloc > loc_cap) { free(loc); return SGFO_EINVAL; }
    memcpy(loc_atoms, loc, (size_t)nloc * sizeof(int32_t));
    local_op op;
    local_op_build(&op, row_ptr, col, h, s, loc, nloc);
    double *chol = NULL;
    int rc = SGFO_OK;
    if (s) {
        chol = malloc((size_t)(op.nl * op.nl) * sizeof(double));
        if (local_cholesky(&op, chol)) rc = SGFO_EINVAL;
    }
    if (rc == SGFO_OK) {
        cplx *zc = malloc((size_t)n_shifts * sizeof(cplx));
        for (int k = 0; k < n_shifts; ++k) zc[k] = z[2 * k] + I * z[2 * k + 1];
        int64_t jl = 4 * local_index(loc, nloc, (int32_t)(j / 4)) + j % 4;
        int mi = max_iter > 0 ? max_iter : (int)(10 * op.nl);
        col_result cr = cocg_column(&op, chol, jl, n_shifts, zc, seed, tol, mi, 0, NULL, NULL, resid, 1,
                                    (cplx *)x, (cplx *)s_final, (cplx *)pi_final);
        *iters = cr.iters;
        *status = cr.status;
        free(zc);
    }
    free(chol);
    local_op_free(&op);
    free(loc);
    return rc;
}
