// scocg.hpp -- argument blocks, workspace layout and launch configuration of
// the two-pass shifted-COCG solver.
#pragma once

#include "common.hpp"

namespace sgf {

constexpr int SEED_T = 64;    // seed pass: one wavefront per workgroup
constexpr int SHIFT_CH = 16;  // shift pass: backward steps staged in LDS at a time
// the 2 SHIFT_CH + 2 recurrence scalars of a chunk are staged one per thread
static_assert(2 * SHIFT_CH + 2 <= 64, "a 64-thread shift workgroup stages a chunk's scalars in one pass");
constexpr double INV_PI = 0.318309886183790671537767526745;

// Column metadata written by the seed pass for the shift pass.
struct ColMeta {
    int32_t col;     // column index (-1: slot unused or rejected)
    int32_t iters;   // seed iterations performed
    int32_t npa;     // projection atoms (mixed path: | local atoms << 8)
    int32_t status;  // sgf_col_status
};

struct SolveArgs {
    // system (device)
    const int32_t *row_ptr, *col;
    const double *h, *s;
    const float *h32;   // FP32 shadow of h (mixed path)
    // plan (device)
    const int64_t *atom_off, *blk_off, *pa_off;
    const int32_t *loc_atom, *lrow, *lblk, *pa_loc, *center_loc;
    int64_t n_plans;
    int max_loc_atoms, max_loc_blocks, npa_max;
    // S != I seed pass: with loc_hi > 0 this launch takes only the columns of
    // loc_lo .. loc_hi local atoms, and only a launch with loc_lo <= 1
    // reports columns that cannot be solved
    int loc_lo, loc_hi;
    // columns
    int64_t n_cols;
    const int64_t *cols;
    const int32_t *col_plan;
    const int32_t *order;
    int64_t batch_begin, batch_end;  // ticket range of this batch
    // shifts
    int ns, ns_pad, seed;
    const double2 *z, *w;
    double tol;
    int max_iter;       // per column; <= 0: 10 * (local orbitals)
    int monitor_every;  // mixed: FP64 true-residual check every K iterations (0: at the end only)
    double drift_tol;   // mixed: DRIFT when ||b - A x_s - s|| > drift_tol ||b||
    double g_tol;       // mixed: DRIFT when max_k ||r_k||^2 / Im z_k > g_tol max_k |G~_jj(z_k)|
    // outputs
    const int64_t *proj_off;
    double *G, *rho, *resid;
    double *eps;        // energy-density matrix on the projection rows (nullable)
    double *gdiag;      // G_jj(z_k) per column, complex [n_cols][ns] (nullable)
    int32_t *iters, *status, *shift_iters;
    // history (per batch slot)
    int cap;            // recorded iterations per slot (max_iter of the batch)
    int rmax;           // projection rows per slot (4 * npa_max)
    ColMeta *meta;      // [slots]
    int32_t *nk;        // [slots][ns_pad] freeze iteration of every shift
    double *fz;         // [slots][ns_pad] ||s||^2 when each shift froze (four-column seed pass:
                        // the residual estimates are formed after the column)
    double2 *hab;       // [slots][cap][2]: 1/alpha_n, beta_n/alpha_n
    double2 *hr;        // [slots][cap+1][rmax]: projected residuals r_n on P
                        // (mixed: the same bytes hold r_n on all 64 rows as float2)
    int64_t *ticket;
    // seed-pass LDS carve (bytes)
    size_t off_p, off_s, off_w, off_hs, off_cs, off_rs, off_q, off_r, off_sinv;
};

struct SolveLayout {
    int64_t *ticket;
    double2 *z, *w;
    ColMeta *meta;
    int32_t *nk;
    double *fz;
    double2 *hab, *hr;
    int64_t slots;
    size_t bytes;
};

// History capacity and per-column bytes for a solve.
struct HistoryShape {
    int cap, rmax, ns_pad;
    size_t per_col, fixed;
};

HistoryShape history_shape(const sgf_plan_totals &tot, int ns, const sgf_solve_opts &o);
SolveLayout solve_layout(const HistoryShape &hs, int ns, int64_t slots, void *base, size_t cap);

using KernelFn = void (*)(SolveArgs);

// Mixed-precision passes (mixed.hip).
KernelFn pick_seed_mx(int M, int bmax);
KernelFn shift_mx_kernel();

// S != I seed pass with the per-atom overlap inverse (seed_kron.hip):
// rows_per_lane 1 for subspaces of <= 16 atoms, 2 for 17 to 32.
KernelFn pick_seed_kron(int rows_per_lane, int M, int bmax);
// the same for 17 to 32 atoms with two wavefronts per column (a row per
// thread), M2 = ns_pad / 128 rounded up
KernelFn pick_seed_kron2(int M2, int bmax);

}  // namespace sgf
