/*
 * sgf.h -- C ABI of the MI355X shifted-COCG Green's-function library.
 *
 * The method (paper, Introduction): instead of the generalized eigenproblem
 * H y = lambda S y, solve the generalized shifted linear equations
 * (z S - H) x = b for many complex energies z; the cost grows linearly with
 * the number of atoms N.  Each basis column b = e_j is solved inside its own
 * local subspace (the atoms near the atom that carries orbital j), and all
 * energies of a column share one Krylov subspace (shifted COCG).  The
 * outputs are Green's-function elements G_ij(z_k) = [(z_k S - H)^{-1}]_ij on
 * projection rows i in P(j) and density-matrix entries
 *     rho_ij = -(1/pi) sum_k Im(w_k G_ij(z_k)).
 * The tight-binding model is the paper's ab-initio-based tight binding,
 * here a Slater-Koster sp model with 4x4 blocks (one block row per atom).
 *
 * Conventions for every entry point:
 *  - Every call returns sgf_status; nothing throws across the ABI and nothing
 *    calls exit().  On a non-OK status, sgf_last_error() returns a
 *    thread-local description of the failure.
 *  - Pointers prefixed d_ are DEVICE pointers owned by the caller, who keeps
 *    them alive until the stream has completed the call.  Pointers without a
 *    prefix are host pointers, read only during the call.
 *  - The library makes no device allocation.  Scratch memory comes from the
 *    caller through a query -> allocate -> call pattern (*_workspace).
 *  - Calls are asynchronous on `stream` (a hipStream_t; NULL = the default
 *    stream) unless marked SYNCHRONOUS, which means the call waits for the
 *    stream because it returns a device-computed size to the host.
 *  - Arguments are validated before any launch; an invalid argument returns
 *    SGF_EINVAL and launches nothing.  A HIP runtime failure returns SGF_EHIP.
 *    Numerical outcomes never fail a call; they go to per-column status codes.
 *  - Complex numbers are interleaved (re, im) doubles.
 *  - BSR layout: row_ptr int32[n_atoms+1], col int32[nnzb] (sorted within each
 *    row, diagonal block included), values [nnzb][4][4] row-major.  Global
 *    orbital index = 4*atom + o, o in (s, px, py, pz).
 */
#ifndef SGF_H
#define SGF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SGF_OK = 0,
    SGF_EINVAL = -1,       /* invalid argument; nothing was launched */
    SGF_ENOMEM = -2,       /* caller-provided workspace too small */
    SGF_EHIP = -3,         /* HIP runtime error */
    SGF_EUNSUPPORTED = -4  /* valid request outside the built kernels' limits */
} sgf_status;

/* Per-column outcome written to d_status by sgf_shifted_solve. */
typedef enum {
    SGF_CONVERGED = 0,  /* every shift reached the tolerance */
    SGF_MAXITER = 1,    /* max_iter reached with at least one shift unconverged */
    SGF_BREAKDOWN = 2,  /* mu = p^T (z_s S - H) p or rho = r^T s vanished with s != 0 */
    SGF_NONFINITE = 3,  /* a recurrence scalar became Inf/NaN */
    SGF_DRIFT = 4,      /* mixed path: recursive and FP64 true residual disagree */
    SGF_BADCOLUMN = 5,  /* column, plan index or plan sizes inconsistent; nothing computed */
    SGF_DIAG_ONLY = 6   /* mixed path: G_jj and rho_jj are certified (a-posteriori bound within g_tol);
                           the other projection rows hold the complex-FP32 Krylov values, so the
                           traces and forces, which read those rows, leave the column out */
} sgf_col_status;

/* Thread-local text of the last non-OK status returned on this thread. */
const char *sgf_last_error(void);

/* Library version, major*10000 + minor*100 + patch. */
int sgf_version(void);

/* ------------------------------------------------------------------------ */
/* Model and system                                                           */
/* ------------------------------------------------------------------------ */

/* Slater-Koster sp parameters (eV, nm).  Hopping blocks scale as
 * V0 * (r0/r)^power for r <= r_cut (hard cutoff).  overlap = 0: S = I;
 * overlap = 1: S_ab = s_amp * exp(-(r - r0)/s_decay) * I4 on the bond
 * pattern and S_aa = I4. */
typedef struct {
    double e_s, e_p, v_sss, v_sps, v_pps, v_ppp;
    double r0, power, r_cut;
    int32_t overlap;
    double s_amp, s_decay;
} sgf_tb_params;

/* Device view of a built system (all pointers device, caller-owned).
 * s / s32 are NULL when S = I.  h32 / s32 are FP32 shadows used by the
 * mixed-precision path (NULL when it is not used).  xyz (nm, [n_atoms][3])
 * may be NULL when every plan uses the whole system (radius <= 0).
 * s_orbital_diagonal = 1 states that every block of s is a multiple of the
 * 4 x 4 identity, S_ab = s_ab I4 (the overlap model of sgf_tb_params
 * overlap = 1, which sgf_build_hamiltonian writes exactly so): the local
 * overlap is then S_a (x) I4 with S_a one number per atom pair, and the FP64
 * S != I seed pass inverts the n x n S_a of a subspace of n atoms instead
 * of the 4n x 4n S_L.  The seed pass checks every block it reads; a column
 * whose blocks are not of that form ends SGF_BADCOLUMN.  0: any symmetric
 * positive definite S. */
typedef struct {
    int64_t n_atoms;
    int64_t nnzb;
    const int32_t *row_ptr;
    const int32_t *col;
    const double *h;
    const double *s;
    const float *h32;
    const float *s32;
    const double *xyz;
    int32_t s_orbital_diagonal;
} sgf_system;

/* A caller-built block-sparse matrix (for example from another tight-binding
 * code), all pointers device and caller-owned: the BSR layout above with
 * n_atoms block rows, nnzb blocks, FP64 values h (and s, NULL for S = I)
 * and optional FP32 shadows h32 / s32.  s_orbital_diagonal as in
 * sgf_system (copied into the descriptor). */
typedef struct {
    int64_t n_atoms;
    int64_t nnzb;
    const int32_t *row_ptr;
    const int32_t *col;
    const double *h;
    const double *s;
    const float *h32;
    const float *s32;
    int32_t s_orbital_diagonal;
} sgf_bsr;

/* The system of the shifted equations (z S - H) x = b of the Introduction,
 * built around a caller's matrix: *out receives a HOST descriptor (allocated
 * with malloc, released by sgf_system_destroy) that borrows m's device
 * arrays and d_xyz (device, nm, [n_atoms][3]; NULL when every local subspace
 * is the whole system).  Checks the host-visible fields only (sizes >= 1,
 * nnzb >= n_atoms for the diagonal blocks, non-NULL row_ptr, col and h);
 * the arrays themselves are read by the later calls.  EINVAL otherwise. */
sgf_status sgf_system_from_bsr(const sgf_bsr *m, const double *d_xyz, sgf_system **out);

/* Release a descriptor from sgf_system_from_bsr (NULL is allowed).  The
 * device arrays it borrowed stay the caller's. */
void sgf_system_destroy(sgf_system *sys);

/* Bytes of scratch needed by sgf_build_pattern for n_atoms atoms. */
sgf_status sgf_build_workspace(int64_t n_atoms, size_t *ws_bytes);

/* Bond pattern (neighbour list).  Atom pairs a != b with
 * (dx*dx + dy*dy) + dz*dz <= r_cut^2 (FP64, evaluated without fused
 * multiply-add) are bonded.  Writes d_row_ptr[n_atoms+1] (each row counts
 * its bonds plus the diagonal block) and returns the block count in *nnzb.
 * d_ws keeps a spatial hash of the atoms that sgf_build_hamiltonian reuses.
 * SYNCHRONOUS (reads nnzb back).  EINVAL on n_atoms < 1, r_cut <= 0, NULL
 * pointers or ws_bytes below sgf_build_workspace. */
sgf_status sgf_build_pattern(int64_t n_atoms, const double *d_xyz, double r_cut, void *d_ws, size_t ws_bytes,
                             int32_t *d_row_ptr, int64_t *nnzb, void *stream);

/* Block count of the Hamiltonian that sgf_build_hamiltonian would build for
 * these positions and parameters (bonds within p->r_cut plus the diagonal
 * blocks), so that the caller can size col / h / s first: the neighbour
 * search of sgf_build_pattern without writing row_ptr.  d_ws: a workspace of
 * sgf_build_workspace(n_atoms) bytes (left holding the spatial hash).
 * SYNCHRONOUS.  EINVAL / EUNSUPPORTED as sgf_build_pattern. */
sgf_status sgf_hamiltonian_size(int64_t n_atoms, const double *d_xyz, const sgf_tb_params *p, void *d_ws,
                                size_t ws_bytes, int64_t *nnzb, void *stream);

/* Tight-binding H (and S when p->overlap) on the pattern from
 * sgf_build_pattern (same d_ws, not modified in between).  Fills d_col
 * (sorted per row) and d_h [nnzb][4][4]; d_s likewise when p->overlap
 * (d_s must then be non-NULL).  d_onsite (nullable) gives 4*n_atoms on-site
 * energies, otherwise diag(e_s, e_p, e_p, e_p).  Hopping block for the bond
 * a -> b with direction cosines c = (R_b - R_a)/r and f = (r0/r)^power
 * (Slater and Koster 1954, Table I):
 *   [s][s] = v_sss f, [s][pA] = c_A v_sps f, [pA][s] = -c_A v_sps f,
 *   [pA][pB] = (c_A c_B (v_pps - v_ppp) + delta_AB v_ppp) f.
 * EINVAL on inconsistent sizes or NULL pointers. */
sgf_status sgf_build_hamiltonian(int64_t n_atoms, const double *d_xyz, const double *d_onsite,
                                 const sgf_tb_params *p, const void *d_ws, size_t ws_bytes,
                                 const int32_t *d_row_ptr, int64_t nnzb, int32_t *d_col, double *d_h,
                                 double *d_s, void *stream);

/* One-orbital chain grouped four sites to a block: H_ii = eps_i,
 * H_{i,i+1} = H_{i+1,i} = t, open ends, S = I.  n_sites must be a multiple
 * of 4; nnzb = 3*(n_sites/4) - 2 (1 when n_sites == 4).  Writes
 * d_row_ptr[n_sites/4 + 1], d_col[nnzb], d_h[nnzb][4][4]. */
sgf_status sgf_build_chain(int64_t n_sites, const double *d_eps, double t, int32_t *d_row_ptr, int32_t *d_col,
                           double *d_h, void *stream);

/* FP32 shadow of a block array: d_out[i] = (float)d_in[i], n_values values. */
sgf_status sgf_to_f32(const double *d_in, int64_t n_values, float *d_out, void *stream);

/* ------------------------------------------------------------------------ */
/* Local subspaces                                                            */
/* ------------------------------------------------------------------------ */

/* A plan describes the local subspace of one centre atom c: the atoms a with
 * (dx*dx + dy*dy) + dz*dz <= R^2 (all atoms when R <= 0), in increasing
 * global order; with prune != 0 only those connected to c through stored
 * blocks inside that ball are kept (the solution of (zS - H)x = e_j vanishes
 * outside that component, so the result is unchanged).  The local operator
 * is the principal sub-block of H (and S) on those atoms.  The projection
 * atoms P are c and every atom that shares a stored block with c, inside the
 * subspace, in increasing global order.  Columns j = 4c + o of one centre
 * (and one radius) share a plan.
 *
 * Inputs (device): center[n_plans] int32, radius[n_plans] double.
 * Outputs (device, caller-allocated):
 *   atom_off, blk_off, pa_off  int64[n_plans+1]  -- filled by sgf_plan_count
 *   loc_atom  int32[atom_off[n]]  global atom of each local atom
 *   lrow      int32[atom_off[n]]  start of each local block row, relative to blk_off[p]
 *   lblk      int32[2*blk_off[n]] (local column atom, global block index) pairs
 *   pa_loc    int32[pa_off[n]]    local index of each projection atom
 *   center_loc int32[n_plans]     local index of the centre atom
 */
typedef struct {
    int64_t n_plans;
    const int32_t *center;
    const double *radius;
    int32_t prune;
    int64_t *atom_off;
    int64_t *blk_off;
    int64_t *pa_off;
    int32_t *loc_atom;
    int32_t *lrow;
    int32_t *lblk;
    int32_t *pa_loc;
    int32_t *center_loc;
} sgf_plan;

/* Totals of a plan batch, returned to the host. */
typedef struct {
    int64_t n_loc_atoms;   /* atom_off[n_plans] */
    int64_t n_loc_blocks;  /* blk_off[n_plans] */
    int64_t n_proj_atoms;  /* pa_off[n_plans] */
    int32_t max_loc_atoms, max_loc_blocks, max_proj_atoms;
    int32_t max_row_blocks; /* most local blocks in one local block row */
} sgf_plan_totals;

/* Scratch bytes for planning n_plans centres with at most max_loc_atoms
 * local atoms each (the ball before pruning). */
sgf_status sgf_plan_workspace(const sgf_system *sys, int64_t n_plans, int32_t max_loc_atoms, size_t *ws_bytes);

/* Count local atoms, local blocks and projection atoms per plan and write
 * the offsets atom_off / blk_off / pa_off.  The spatial hash of the build
 * workspace (d_build_ws, from sgf_build_pattern on the same xyz) finds the
 * atoms in the ball.  SYNCHRONOUS (returns totals).  A subspace larger than
 * max_loc_atoms returns SGF_EUNSUPPORTED with the offending plan named.
 * The count first runs with a 256-atom LDS capacity and only a batch with a
 * larger subspace is counted again at max_loc_atoms. */
sgf_status sgf_plan_count(const sgf_system *sys, sgf_plan *plan, int32_t max_loc_atoms, const void *d_build_ws,
                          size_t build_ws_bytes, void *d_ws, size_t ws_bytes, sgf_plan_totals *totals,
                          void *stream);

/* Fill loc_atom, lrow, lblk, pa_loc and center_loc, after sgf_plan_count on
 * the same system, plan and workspaces.  max_loc_atoms sizes the LDS of the
 * fill and may be anything from the max_loc_atoms total that the count
 * returned (the cheapest choice) up to the count's own argument.
 * SYNCHRONOUS: a plan that does not fit returns SGF_EUNSUPPORTED. */
sgf_status sgf_plan_build(const sgf_system *sys, sgf_plan *plan, int32_t max_loc_atoms, const void *d_build_ws,
                          size_t build_ws_bytes, void *d_ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------ */
/* Shifted solve                                                              */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t precision;     /* 0: FP64 throughout; 1: mixed (complex-FP32 vectors and operator,
                              FP64 recurrence scalars, FP64 true-residual monitor and FP64 epilogue) */
    double tol;            /* shift k stops when ||s_{n+1}||_2 / |pi^k_{n+1}| <= tol ||b||_2 */
    int32_t max_iter;      /* <= 0: 10 * (local orbitals) per column (mixed precision: 40 *) */
    int32_t seed_index;    /* >= 0: that shift; -1 (or below -2): n_shifts / 2; -2: the shift nearest
                              the real axis (smallest Im z; among equals the one nearest n_shifts / 2),
                              the slowest to converge, so that the seed iterates at least as long as any
                              other shift and its residual cannot underflow first */
    int32_t monitor_every; /* mixed: FP64 true residual every K iterations (0: only at the end) */
    int32_t stage_lds;     /* seed pass, S = I: -1 auto (for subspaces of <= 64 orbitals and <= 8 blocks per
                              row: four columns of a plan per wavefront with the blocks in LDS at <= 128
                              shifts, two columns per wavefront at <= 256, one column per wavefront with
                              its rows in registers above; else an LDS-staged operator when it fits);
                              3 one column per wavefront with rows in registers; 5 two columns per
                              wavefront (<= 256 shifts); 1 LDS-staged operator; 0 operator read from
                              global.
                              S != I: -1 auto: with s_orbital_diagonal, subspaces of <= 32 atoms,
                              rows of <= 8 blocks and <= 256 shifts, the per-atom overlap inverse
                              (a launch for <= 16 atoms with one wavefront per column, a row per
                              lane, and one for 17-32 with two, a row per thread); otherwise subspaces of <= 16 atoms in a launch with
                              the dense orbital overlap inverse, larger ones in a second launch
                              with its packed triangle, both with two wavefronts per column when
                              every subspace has <= 32 atoms and rows of <= 8 blocks; 0 one launch,
                              dense; 1 one launch, packed; 2 the split of -1 with one wavefront
                              per column throughout; 4 the per-atom inverse of -1 with one
                              wavefront per column (two rows per lane) in the launch for 17-32
                              atoms, else as 0 (S = I treats 2 and 4 as 0, S != I treats 3 and 5
                              as 0).  0, 1 and 2 never
                              take the per-atom inverse */
    int32_t grid;          /* seed-pass persistent workgroups; 0: fill the device */
    int32_t profile;       /* 1: record HIP events around each pass (read with sgf_solve_profile) */
    int64_t batch_cols;    /* columns per launch (0: all); the solve also stops at what the workspace holds */
    int32_t shifts_per_lane; /* shift pass: 1 or 2 shifts per lane; 0: chosen from the projection size */
    int32_t shifts_staged; /* 1: z and w are already in the workspace (sgf_solve_stage_shifts with the
                              same arrays), so the solve issues only kernel launches on the stream
                              (for capture into a HIP graph); the host z is still read for checks */
    double drift_tol;      /* mixed: a column stops with SGF_DRIFT when its FP64 true seed residual
                              b - (z_s - H) x_s departs from the recursive residual by more than
                              drift_tol ||b||_2 (checked every monitor_every iterations and at the end);
                              0: 1e-3 */
    double g_tol;          /* mixed: a column whose a-posteriori bound max_k ||r_k||^2 / Im z_k on the
                              error of G_jj (r_k the FP64 true residual of the full iterate of shift
                              k) exceeds g_tol max_k |G_jj(z_k)| gets SGF_DRIFT; 0: 5e-7 */
    int64_t queue_len;     /* > 0: take only d_order[0 .. queue_len) from the work queue (the other
                              columns' outputs are left untouched); 0: every column */
    double *eps_out;       /* NULL, or device double [projection rows] (the layout of d_rho): the
                              shift pass also writes the energy-density matrix
                              eps_t = -(1/pi) sum_k Im(w_k z_k G_t(z_k)) that the forces need when
                              S != I (sgf_band_forces), without G being kept.  Needs w; FP64 path
                              only (precision 1 returns SGF_EUNSUPPORTED) */
    double *g_diag_out;    /* NULL, or device complex [n_cols][n_shifts]: the shift pass also writes the
                              diagonal element G_jj(z_k) of every column (the same values as its row in
                              d_G).  With d_G NULL this is the "diagonal only" output, 16 n_shifts bytes
                              per column instead of 64 |P| n_shifts */
} sgf_solve_opts;

/* Output offsets: d_proj_off[c+1] - d_proj_off[c] = 4 * |P(plan of column c)|
 * (int64[n_cols+1]); also writes d_proj_row (global orbital of every
 * projection row) when it is non-NULL on a second call.  SYNCHRONOUS
 * (returns the total row count). */
sgf_status sgf_proj_layout(const sgf_plan *plan, int64_t n_cols, const int64_t *d_cols, const int32_t *d_col_plan,
                           int64_t *d_proj_off, int32_t *d_proj_row, int64_t *total_rows, void *stream);

/* Projection rows only, from offsets that sgf_proj_layout already wrote:
 * d_proj_row[d_proj_off[c] + 4 q + o] = 4 * (q-th projection atom of column
 * c's plan) + o.  d_proj_row holds d_proj_off[n_cols] int32 (caller-owned).
 * Asynchronous on the stream. */
sgf_status sgf_proj_rows(const sgf_plan *plan, int64_t n_cols, const int32_t *d_col_plan, const int64_t *d_proj_off,
                         int32_t *d_proj_row, void *stream);

/* Scratch bytes for sgf_shifted_solve with opts->batch_cols columns per
 * batch (0: every column at once).  Per column the workspace holds the seed
 * history: (max_iter) x 32 bytes of recurrence scalars and (max_iter + 1) x
 * 16 x 4|P|max bytes of projected residuals (mixed precision: (max_iter + 1)
 * x 512 bytes of full residual vectors).  sgf_shifted_solve accepts any
 * workspace of at least one column's worth and launches the columns in
 * batches of min(batch_cols, what the workspace holds) columns. */
sgf_status sgf_solve_workspace(const sgf_system *sys, const sgf_plan_totals *totals, int64_t n_cols,
                               int32_t n_shifts, const sgf_solve_opts *opts, size_t *ws_bytes);

/*
 * Shifted COCG for n_cols columns (b = e_j, j = d_cols[c], local subspace
 * d_col_plan[c]) at n_shifts energies z (HOST array, all Im z_k > 0; copied
 * into the workspace on the stream), seed z_s = z[seed_index].  For every
 * column, on its local subspace:
 *   w = z_s q - H p;  mu = p^T w;  alpha = rho / mu
 *   s -= alpha w;  r = S^{-1} s;  rho' = r^T s;  beta = rho' / rho
 *   p = r + beta p;  q = s + beta q
 *   per active shift k (sigma_k = z_k - z_s):
 *     pi^k_{n+1} = (1 + alpha sigma_k) pi^k_n + (alpha beta_old / alpha_old)(pi^k_n - pi^k_{n-1})
 *     frozen after step n once ||s_{n+1}|| / |pi^k_{n+1}| <= tol  (N_k = n + 1 steps)
 *   G^k_P = (x^k)_P for the N_k-step shifted iterate
 *     x^k = sum_n alpha^k_n p^k_n,  alpha^k = alpha pi^k_n / pi^k_{n+1},
 *     p^k = r_{n+1} / pi^k_{n+1} + (pi^k_n / pi^k_{n+1})^2 beta p^k
 * (COCG, van der Vorst and Melissen 1990; shifted form with collinear
 * residuals, Frommer 2003 and Takayama et al. 2006).  The library evaluates
 * x^k_P from the recorded seed scalars by a backward sweep over the
 * tridiagonal T_{N_k} + sigma_k of the seed iteration, which yields the same
 * iterate.
 *
 * Outputs (device): d_G complex [total_rows][n_shifts] (nullable: rho only),
 * d_rho double[total_rows] with rho_ij = -(1/pi) sum_k Im(w_k G_ij(z_k))
 * (w: HOST complex[n_shifts] quadrature weights; NULL: all zero),
 * d_iters / d_status int32[n_cols], d_resid double[n_cols][n_shifts]
 * (nullable): ||s|| / |pi^k| when shift k froze (or at the last step).
 * d_shift_iters (nullable) int32[n_cols][n_shifts]: N_k, the steps shift k took.
 * d_order (nullable) int32[n_cols] (int32[queue_len] when opts->queue_len >
 * 0): the order in which columns are taken from the work queue (a
 * permutation of 0..n_cols-1, or queue_len distinct columns); results do not
 * depend on it (entries outside [0, n_cols) are skipped).  Device arrays are
 * checked where they are read: a column whose plan index is out of range,
 * whose atom is not its plan's centre, or whose plan exceeds `totals`
 * gets SGF_BADCOLUMN and no output.  EINVAL on bad sizes, Im z_k <= 0, tol <= 0, NULL required
 * pointers or a workspace below one column's worth; EUNSUPPORTED when a plan
 * is larger than the kernels' LDS allows, a column has more than 8
 * projection atoms or n_shifts > 512.
 *
 * Mixed precision (opts->precision = 1; S = I, local subspaces of <= 16
 * atoms with <= 8 blocks per row, n_shifts <= 256, sys->h32 required, else
 * EUNSUPPORTED / EINVAL): the seed iteration runs on the FP32 shadow of H with
 * complex-FP32 vectors and FP64 scalars (mu, rho, alpha, beta, pi^k), and
 * keeps the seed iterate x_s in FP64; its FP64 true residual is compared
 * with the recursive one every monitor_every iterations and at the end
 * (SGF_DRIFT beyond drift_tol).  The shift pass rebuilds the full iterate
 * x~^k on the local subspace (complex FP32) and writes for the diagonal
 * element the FP64 variational estimate 2 x~_j - x~^T (z_k - H) x~^k, whose
 * error is quadratic in that of x~ (the stationary property of the
 * Green's-function functional for the complex symmetric z - H).  The other
 * projection rows are the FP32-Krylov values.  From the FP64 true residual
 * r_k of the full iterate (written to d_resid instead of the recursive
 * residual) the shift pass bounds the error of the estimate rigorously,
 * |G_jj - G~_jj| <= ||r_k||^2 / Im z_k, and sets SGF_DRIFT on a column
 * whose bound exceeds opts->g_tol max_k |G~_jj|.  A column whose bound
 * holds ends with SGF_DIAG_ONLY, not SGF_CONVERGED: its G_jj and rho_jj are
 * certified, its other rows are not.  A caller that needs every column
 * re-solves the others (DRIFT, MAXITER, ...) in FP64 with queue_len (the
 * Python binding does so; a caller that needs certified off-diagonal rows
 * re-solves the SGF_DIAG_ONLY columns too).  The workspace holds the full residual history:
 * (max_iter + 1) x 512 bytes per column.
 */
sgf_status sgf_shifted_solve(const sgf_system *sys, const sgf_plan *plan, const sgf_plan_totals *totals,
                             int64_t n_cols, const int64_t *d_cols, const int32_t *d_col_plan,
                             const int32_t *d_order, int32_t n_shifts, const double *z, const double *w,
                             const sgf_solve_opts *opts, void *d_ws, size_t ws_bytes, const int64_t *d_proj_off,
                             double *d_G, double *d_rho, int32_t *d_iters, int32_t *d_status, double *d_resid,
                             int32_t *d_shift_iters, void *stream);

/* Bytes of the static device scratch behind sgf_shifted_solve_static. */
#define SGF_STATIC_SCRATCH_BYTES ((size_t)256 << 20)

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The same
 * solve as sgf_shifted_solve (same kernels, same arguments and outputs, the
 * same bits), with the workspace taken from a static device array of
 * SGF_STATIC_SCRATCH_BYTES that the library holds on every GPU it runs on
 * until the process ends; the call itself allocates nothing (no hipMalloc,
 * no hipFree, no HIP events).  Columns are launched in batches of as many
 * as that scratch holds (opts->batch_cols can lower it).  z and w are copied
 * into the scratch on the stream, as sgf_shifted_solve copies them into its
 * workspace; opts->shifts_staged = 1 reuses the z and w a previous
 * sgf_shifted_solve_static call with the same n_shifts left there.
 * Errors: as sgf_shifted_solve; SGF_EINVAL for opts->profile = 1;
 * SGF_EUNSUPPORTED when one column's history (max_iter and n_shifts) does
 * not fit the scratch.  Every call on one GPU uses that GPU's single
 * scratch array: calls that overlap in time on one GPU (two streams, two
 * threads) race and corrupt each other's results; serialise them.  The
 * array keeps the last call's contents; the call clears what must start at
 * zero (its work-queue ticket) itself. */
sgf_status sgf_shifted_solve_static(const sgf_system *sys, const sgf_plan *plan, const sgf_plan_totals *totals,
                                    int64_t n_cols, const int64_t *d_cols, const int32_t *d_col_plan,
                                    const int32_t *d_order, int32_t n_shifts, const double *z, const double *w,
                                    const sgf_solve_opts *opts, const int64_t *d_proj_off, double *d_G,
                                    double *d_rho, int32_t *d_iters, int32_t *d_status, double *d_resid,
                                    int32_t *d_shift_iters, void *stream);

/* Copy z (and w, nullable) into the workspace of later sgf_shifted_solve
 * calls with opts->shifts_staged = 1 and the same n_shifts: they sit at the
 * start of the workspace, ahead of every per-column slot.  Asynchronous on
 * the stream (host arrays are read before it returns only if the copy is
 * synchronous for pageable memory; keep them alive until the stream has
 * passed it). */
sgf_status sgf_solve_stage_shifts(int32_t n_shifts, const double *z, const double *w, void *d_ws, size_t ws_bytes,
                                  void *stream);

/* Kernel times of the last sgf_shifted_solve on this thread that ran with
 * opts->profile = 1 (later unprofiled solves do not replace it), from HIP events recorded on its stream around every
 * launch of the seed pass and of the shift pass.  SYNCHRONOUS (waits for
 * those events).  *batches = number of launches of each pass.  EINVAL if no
 * profiled solve is pending; the events are released by this call. */
sgf_status sgf_solve_profile(double *seed_ms, double *shift_ms, int32_t *batches);

/* Shifts and weights for the Fermi-Dirac density matrix (HOST call).  The
 * order-N energy of the Introduction needs rho = f(H), f(e) = 1/(1 +
 * exp((e - mu)/kT)); a real-axis grid needs energies close to the axis and
 * many of them.  The pole expansion of f from the continued fraction of
 * tanh (Ozaki, Phys. Rev. B 75, 035123 (2007)),
 *   f(y) = 1/2 - sum_p R_p (1/(y - i z_p) + 1/(y + i z_p)), y = (e - mu)/kT,
 * gives rho = S^{-1}/2 + 2 kT sum_p R_p Re G(mu + i z_p kT), with S^{-1} =
 * Re(i M G(i M)) up to |H|^2/M^2.  Writes n_poles + 1 complex shifts z and
 * weights w (host, interleaved re, im) for sgf_shifted_solve: z_p = mu + i
 * z_p kT with w_p = -2 pi i kT R_p for p = 0 .. n_poles-1, nearest the real
 * axis first (z_0 = mu + i pi kT to rounding), then z = i*moment with
 * w = pi moment / 2.  The expansion holds for |e - mu| up to about
 * 20 n_poles kT (measured: 40 poles reach 5e-10 at |y| = 600, 60 poles 3e-13
 * at |y| = 1000); choose n_poles from the spectral bounds (sgf_wp_bounds).
 * A seed at the pole nearest the axis (opts.seed_index = -2) keeps the seed
 * system the slowest one.  EINVAL on n_poles outside [1, 511], kT <= 0,
 * moment <= 0 or NULL outputs. */
sgf_status sgf_fermi_shifts(int32_t n_poles, double kT, double mu, double moment, double *z, double *w);

/* ------------------------------------------------------------------------ */
/* Global operator application                                                */
/* ------------------------------------------------------------------------ */
/* d_y = (z S - H) d_x for n_rhs (1, 2, 4 or 8) complex right-hand sides over
 * the whole system: the operator of the shifted equations (zS - H)x = b of
 * the Introduction, applied once (e.g. to check a full-system solution
 * against its right-hand side in FP64).  z: HOST complex (re, im).
 * precision 0: FP64 operator (h, s), d_x / d_y complex128; 1: FP32 shadows
 * (h32, s32), complex64.  Layout [4 n_atoms][n_rhs] (right-hand sides
 * contiguous per orbital); d_x and d_y must not alias and must be 16-byte
 * aligned (EINVAL otherwise).  S = I when the
 * system has no overlap.  Asynchronous on the stream.  One pass over the
 * matrix in HBM: 16 n_rhs complex multiply-adds per 4x4 block, so the call
 * is bound by HBM bandwidth. */
sgf_status sgf_bsr_apply(const sgf_system *sys, int32_t precision, int32_t n_rhs, const double *z, const void *d_x,
                         void *d_y, void *stream);

/* ------------------------------------------------------------------------ */
/* Learned scheduling                                                         */
/* ------------------------------------------------------------------------ */
/* A small network predicts how many Krylov iterations a column needs from
 * its local environment, so that columns can be queued longest-first and
 * grouped into balanced batches.  Convergence is still decided by the
 * residual in sgf_shifted_solve, so the order never changes a result; the
 * natural order is the fallback.  (This scheduler is not part of the paper;
 * it sits on top of the method.)
 *
 * Features of column j (atom c, orbital o) on its local subspace, float[5]:
 *   f0 off-diagonal blocks of c's local block row;
 *   f1, f2 mean and max of ||H_cb[o, :]||_2 over those blocks;
 *   f3 |H_jj - mean of H_ii over the local orbitals of type o|;
 *   f4 local orbitals.
 * Network (FP32): x' = (x - mean) * inv_std; h1 = relu(W1 x' + b1);
 * h2 = relu(W2 h1 + b2); y = W3 . h2 + b3, trained on y = log(iterations)
 * by mean-squared error with Adam (beta1 0.9, beta2 0.999, eps 1e-8).
 * Parameters: float[SGF_MLP_NPARAM] = [0:5] mean, [5:10] inv_std,
 * W1 (64x5 row-major), b1 (64), W2 (64x64), b2 (64), W3 (64), b3 (1). */
#define SGF_MLP_NFEAT 5
#define SGF_MLP_HIDDEN 64
#define SGF_MLP_NPARAM 4619

/* d_feat float[n_cols][5] for the columns of a built plan. */
sgf_status sgf_features(const sgf_system *sys, const sgf_plan *plan, int64_t n_cols, const int64_t *d_cols,
                        const int32_t *d_col_plan, float *d_feat, void *stream);

/* Set the normalisation entries [0:10] of d_params to the mean and 1/std of
 * n feature rows (a constant feature keeps inv_std = 1). */
sgf_status sgf_mlp_normalize(float *d_params, const float *d_feat, int64_t n, void *stream);

/* d_y[i] = network(d_feat[i]) for n rows. */
sgf_status sgf_mlp_forward(const float *d_params, const float *d_feat, int64_t n, float *d_y, void *stream);

/* One Adam step (step counts from 1) on a minibatch of n <= 128 rows with
 * targets d_target; d_adam_m / d_adam_v are float[SGF_MLP_NPARAM] moment
 * buffers (zero before step 1).  d_loss (nullable) receives the minibatch
 * MSE before the update.  One workgroup; gradients are summed in a fixed
 * order, so a step is bitwise reproducible. */
sgf_status sgf_mlp_train_step(float *d_params, float *d_adam_m, float *d_adam_v, int32_t step, float lr,
                              const float *d_feat, const float *d_target, int32_t n, float *d_loss, void *stream);

/* Gradient of the minibatch MSE with respect to every parameter (zero for
 * the normalisation entries), n <= 128, into d_grad float[SGF_MLP_NPARAM]. */
sgf_status sgf_mlp_gradient(const float *d_params, const float *d_feat, const float *d_target, int32_t n,
                            float *d_grad, float *d_loss, void *stream);

/* Work-queue order, largest prediction first: a counting sort of d_pred into
 * 4096 buckets over [y_lo, y_hi] (values outside are clamped); the order
 * inside a bucket is unspecified.  Writes a permutation of 0..n-1. */
sgf_status sgf_order_workspace(size_t *ws_bytes);
sgf_status sgf_order_by_prediction(const float *d_pred, int64_t n, float y_lo, float y_hi, int32_t *d_order,
                                   void *d_ws, size_t ws_bytes, void *stream);

/* The same order by plans: the columns that share a plan (d_col_plan, as in
 * the solve) stay next to each other, and the plans are queued by the
 * largest prediction among their columns (counting sort over [y_lo, y_hi]).
 * The seed pass that runs four columns of one plan per wavefront then finds
 * a plan's columns together.  Columns with a plan index outside
 * [0, n_plans) go last.  Writes a permutation of 0..n-1 into d_order; the
 * order inside a plan's run is unspecified (results do not depend on it). */
sgf_status sgf_order_groups_workspace(int64_t n_plans, size_t *ws_bytes);
sgf_status sgf_order_groups_by_prediction(const float *d_pred, int64_t n, const int32_t *d_col_plan, int64_t n_plans,
                                          float y_lo, float y_hi, int32_t *d_order, void *d_ws, size_t ws_bytes,
                                          void *stream);

/* ------------------------------------------------------------------------ */
/* After rho: traces, electron count, band energy, Fermi level               */
/* ------------------------------------------------------------------------ */

/* Row j of the restricted equations (z S_L - H_L) x = e_j couples j only to
 * orbitals sharing a stored block with it, which are the projection rows
 * P(j); so the projected G gives the per-shift traces over the solved
 * columns
 *     T_k = sum_j sum_{i in P(j)} S_ji G_ij(z_k)    (= sum_j (G S)_jj)
 *     U_k = sum_j sum_{i in P(j)} H_ji G_ij(z_k)    (= sum_j (G H)_jj)
 * from which, for quadrature weights w of the occupied spectrum, the
 * electron count tr(rho S) = -(1/pi) sum_k Im(w_k T_k) and the band energy
 * tr(rho H) = -(1/pi) sum_k Im(w_k U_k) follow (the order-N energy of the
 * Introduction: the quantities formed from rho after the shifted solves).
 *
 * Scratch bytes for sgf_traces over total_rows projection rows. */
sgf_status sgf_trace_workspace(int64_t total_rows, int32_t n_shifts, size_t *ws_bytes);

/* Traces of one solve's outputs (device arrays as sgf_shifted_solve wrote
 * them): d_cols[n_cols], d_proj_off[n_cols+1], d_proj_row[total_rows],
 * d_status[n_cols] (nullable: with it, only SGF_CONVERGED columns count;
 * a column the solve rejected holds no G or rho, and an SGF_DIAG_ONLY
 * column of the mixed path has uncertified off-diagonal rows), d_G complex
 * [total_rows][n_shifts] (nullable), d_rho [total_rows] (nullable; one of
 * the two is required).  Writes d_T and d_U (complex [n_shifts], needed
 * with d_G) and d_rho_tr (double[2]: tr(rho S), tr(rho H) at the solve's
 * own weights, needed with d_rho).  Sums in a fixed order (bitwise
 * repeatable).  Asynchronous on the stream. */
sgf_status sgf_traces(const sgf_system *sys, int64_t n_cols, const int64_t *d_cols, const int64_t *d_proj_off,
                      const int32_t *d_proj_row, const int32_t *d_status, int64_t total_rows, const double *d_G,
                      const double *d_rho, int32_t n_shifts, void *d_ws, size_t ws_bytes, double *d_T, double *d_U,
                      double *d_rho_tr, void *stream);

/* Host arrays (complex interleaved): electron count and band energy
 * -(1/pi) sum_k Im(w_k T_k), -(1/pi) sum_k Im(w_k U_k) for any weights w. */
sgf_status sgf_occupation(int32_t n_shifts, const double *T, const double *U, const double *w, double *n_e,
                          double *e_band);

/* Host: the Fermi level on a real-axis grid z_k = E_k + i eta (E_k
 * increasing).  With trapezoid weights (the spacing, halved at the two grid
 * ends) on E_k <= mu, the electron count N_e(mu) changes only at grid
 * points; bisection on the grid index returns the first E_m with
 * N_e(E_m) >= n_target as mu, with N_e and the band energy there.  A target
 * above the count of the whole grid returns SGF_EUNSUPPORTED. */
sgf_status sgf_fermi_level(int32_t n_shifts, const double *z, const double *T, const double *U, double n_target,
                           double *mu, double *n_e, double *e_band);

/* The energy-density matrix on the projection rows of a solve, the
 * quadrature of rho with the weight w_k z_k (the term of the forces that an
 * overlap adds, Sec. 2):
 *   d_eps[t] = -(1/pi) sum_k Im(w_k z_k G_t(z_k)),  t < total_rows.
 * For real weights, (z S - H) G = I gives sum_{i in P(j)} eps_ij S_ji =
 * sum_{i in P(j)} rho_ij H_ji for every column.  d_z, d_w: device complex
 * [n_shifts] (interleaved re, im; the solve's shifts and weights); d_G:
 * complex [total_rows][n_shifts] as sgf_shifted_solve wrote it (the rows of
 * a column the solve rejected hold no G, so their eps means nothing).  Sums
 * in a fixed order (bitwise repeatable).  SGF_EUNSUPPORTED above 512 shifts.
 * Asynchronous on the stream. */
sgf_status sgf_energy_density(int64_t total_rows, int32_t n_shifts, const double *d_z, const double *d_w,
                              const double *d_G, double *d_eps, void *stream);

/* ------------------------------------------------------------------------ */
/* Wavepacket propagation                                                     */
/* ------------------------------------------------------------------------ */

/* The wavepacket dynamics of Sec. 3 (Fig. 2) integrate d/dt Psi = -i H Psi
 * / hbar (H in eV, t in fs, hbar = 0.6582119569509066 eV fs) in steps of
 * h (0.1 fs in the paper) with the tight-binding H in an orthogonal basis
 * (S = I).  One step applies exp(-i tau H), tau = h / hbar, as the Chebyshev
 * series of Tal-Ezer and Kosloff (J. Chem. Phys. 81, 3967 (1984)): with
 * a = (e_max - e_min)/2 and b = (e_max + e_min)/2 from bounds of the
 * spectrum, exp(-i tau H) = exp(-i tau b) sum_{k<K} c_k T_k((H - b)/a),
 * c_0 = J_0(a tau), c_k = 2 (-i)^k J_k(a tau). */

/* Bytes of device workspace for sgf_wp_bounds and sgf_wp_propagate on a
 * system of n_atoms atoms with n_rhs (1, 2, 4 or 8) packets: two complex
 * vectors [4 n_atoms][n_rhs]. */
sgf_status sgf_wp_workspace(int64_t n_atoms, int32_t n_rhs, size_t *ws_bytes);

/* Gershgorin bounds of H: e_min = min_i (H_ii - R_i), e_max =
 * max_i (H_ii + R_i), R_i = sum_{j != i} |H_ij|, which contain its spectrum.
 * SYNCHRONOUS (host outputs; waits for the stream).  d_ws: a workspace of at
 * least sgf_wp_workspace(n_atoms, 1) bytes. */
sgf_status sgf_wp_bounds(const sgf_system *sys, void *d_ws, size_t ws_bytes, double *e_min, double *e_max,
                         void *stream);

/* Host: number of series terms K for argument a tau (a = half the width of
 * the bounds): the smallest K > |a tau| with |J_K| and |J_{K+1}| <= tol (the
 * Bessel functions decay faster than geometrically beyond |a tau|, so the
 * dropped tail is about tol); at least 3. */
sgf_status sgf_wp_terms(double a_tau, double tol, int32_t *n_terms);

/* n_steps steps of length h_fs (negative h runs backwards) of the n_rhs
 * packets in d_psi: complex128 [4 n_atoms][n_rhs] (packets contiguous per
 * orbital), overwritten with the result.  e_min < e_max must contain the
 * spectrum (sgf_wp_bounds); n_terms >= 3 (sgf_wp_terms).  Per term one
 * pass over H in HBM fused with the recurrence and the accumulation of the
 * series; d_ws (sgf_wp_workspace bytes) holds the two other Chebyshev
 * vectors.  sys->h, d_psi and d_ws must be 16-byte aligned (SGF_EINVAL
 * otherwise).  SGF_EUNSUPPORTED when the system has an overlap S.
 * Asynchronous on the stream. */
sgf_status sgf_wp_propagate(const sgf_system *sys, int32_t n_rhs, double *d_psi, double h_fs, int32_t n_steps,
                            double e_min, double e_max, int32_t n_terms, void *d_ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------ */
/* Band-structure forces                                                      */
/* ------------------------------------------------------------------------ */

/* The force step of the quantum molecular dynamics (Sec. 2).  E_band =
 * sum_j sum_{i in P(j)} rho_ij H_ij over the solved columns (per spin; the
 * tr(rho H) of sgf_traces).  With S = I the force is F_A = -dE_band/dR_A
 * at fixed rho.  With an overlap S, Hellmann-Feynman for H c = lambda S c
 * adds the energy-density matrix (sgf_energy_density):
 *   F_A = -sum_j sum_{i in P(j)} (rho_ij dH_ij/dR_A - eps_ij dS_ij/dR_A).
 * Each term acts on both atoms of its block: with i on atom B and j on atom
 * C (B != C), g = rho_ij d h_{o_i q_j}/dd - eps_ij d s_{o_i q_j}/dd at
 * d = R_C - R_B (the Slater-Koster block h and the overlap block s =
 * s_amp exp(-(r - r0)/s_decay) I4 of sgf_build_hamiltonian with parameters
 * p) enters F_C with a minus sign and F_B with a plus sign, so the forces sum
 * to zero.  A row whose atom lies farther than p->r_cut from the column's
 * atom has no block and adds nothing.  With all columns solved this is the
 * Hellmann-Feynman band force; the repulsive and van der Waals terms are not
 * included.
 * d_xyz: positions (nm, [n_atoms][3]); d_cols, d_proj_off, d_proj_row and
 * d_rho: the columns and projected density matrix of a solve; d_eps: the
 * energy-density matrix on the same rows (sgf_energy_density from a kept G,
 * or the solve's sgf_solve_opts.eps_out), required when the system has an
 * overlap and ignored (may be NULL) when it has none; d_status [n_cols]
 * (nullable): with it, only SGF_CONVERGED columns count (a column the solve
 * rejected holds no rho; an SGF_DIAG_ONLY column of the mixed path holds
 * uncertified off-diagonal rows).  p->overlap must match the system.  Writes d_force [n_atoms][3] (eV/nm), cleared first.  FP64
 * atomics add the terms, in no fixed order: repeated runs agree to
 * rounding.  Asynchronous on the stream. */
sgf_status sgf_band_forces(const sgf_system *sys, const double *d_xyz, const sgf_tb_params *p, int64_t n_cols,
                           const int64_t *d_cols, const int64_t *d_proj_off, const int32_t *d_proj_row,
                           const int32_t *d_status, const double *d_rho, const double *d_eps, double *d_force,
                           void *stream);

/* ------------------------------------------------------------------------ */
/* Quantum molecular dynamics: the time step                                  */
/* ------------------------------------------------------------------------ */

/* Acceleration in nm/fs^2 of a force of 1 eV/nm on a mass of 1 amu:
 * (e / u) x 1e-12 with the exact elementary charge e = 1.602176634e-19 C
 * and the CODATA 2018 atomic mass constant u = 1.66053906660e-27 kg. */
#define SGF_ACCEL_EV_NM_AMU 9.648533215665326e-5

/* One step of the quantum molecular dynamics of Sec. 2 (time step h_MD,
 * 1 fs in the paper) by velocity Verlet (Swope, Andersen, Berens and Wilson,
 * J. Chem. Phys. 76, 637 (1982)): with forces F(x_n),
 *   sgf_md_kick  (v += (h/2) F / m),  sgf_md_drift (x += h v),
 *   new H, plans, shifted solve and sgf_band_forces at x_{n+1},
 *   sgf_md_kick  (v += (h/2) F_{n+1} / m).
 * Units: positions nm, velocities nm/fs, forces eV/nm, masses amu, h in fs
 * (negative h runs backwards).  Device arrays [n_atoms][3] (d_mass
 * [n_atoms]), updated in place; asynchronous on the stream.  EINVAL on NULL
 * arrays, n_atoms < 0 or a non-finite or absurd step (|h| >= 1e6 fs). */
sgf_status sgf_md_kick(int64_t n_atoms, const double *d_force, const double *d_mass, double h_fs, double *d_vel,
                       void *stream);
sgf_status sgf_md_drift(int64_t n_atoms, const double *d_vel, double h_fs, double *d_xyz, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* SGF_H */
