// trace.hip -- traces of the projected Green's function over the solved
// columns, and what follows from them after rho in an order-N energy step:
// electron count, band energy, the Fermi level and the energy-density matrix.
//
// Row j of the restricted equations (z S_L - H_L) x = e_j couples j only to
// orbitals that share a stored block with it, and those are the projection
// rows P(j) of the column.  So the projected G is enough for the per-shift
// traces
//   T_k = sum_j sum_{i in P(j)} S_ji G_ij(z_k)   ( = sum_j (G S)_jj )
//   U_k = sum_j sum_{i in P(j)} H_ji G_ij(z_k)   ( = sum_j (G H)_jj )
// and, for quadrature weights w of the occupied spectrum,
//   N_e    = -(1/pi) sum_k Im(w_k T_k) = tr(rho S)
//   E_band = -(1/pi) sum_k Im(w_k U_k) = tr(rho H)
// over the solved columns.  The same row gives z_k T_k - U_k = (number of
// columns) up to the solve's residuals, which the tests use as a pin.
//
// The energy-density matrix, which the forces need when S != I, is the same
// quadrature as rho with the weight w_k z_k:
//   eps_ij = -(1/pi) sum_k Im(w_k z_k G_ij(z_k)),
// one value per projection row.  Because (z S - H) G = I, it satisfies
// sum_{i in P(j)} eps_ij S_ji = sum_{i in P(j)} rho_ij H_ji per column for
// real weights.
#include "common.hpp"

namespace sgf {

constexpr int TR_NB = 1024;   // workgroups of the partial-sum passes
constexpr int TR_UNROLL = 8;  // projection rows in flight per thread
constexpr int TR_RHO_T = 256;
constexpr int TR_RED_T = 256;  // threads of the final reductions
constexpr int TR_COEF_L = 16; // lanes per column in the coefficient pass
constexpr double INV_PI_D = 0.318309886183790671537767526745;

// S_ji and H_ji of every projection row (TR_COEF_L lanes per column, each
// taking every TR_COEF_L-th row of it).  A row whose atom shares no stored
// block with the column's atom gets zeros (it cannot occur for rows built by
// sgf_proj_layout), and so do all rows of a column that is left out.
__global__ void k_trace_coef(int64_t n_cols, int64_t n_orb, const int64_t *cols, const int64_t *proj_off,
                             const int32_t *proj_row, const int32_t *status, const int32_t *row_ptr,
                             const int32_t *col, const double *h, const double *s, double2 *coef) {
    const int lane = (int)(threadIdx.x % TR_COEF_L);
    const int64_t step = (int64_t)gridDim.x * (blockDim.x / TR_COEF_L);
    for (int64_t c = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / TR_COEF_L; c < n_cols; c += step) {
        const int64_t j = cols[c];
        // a column left out (status given and not converged) contributes zeros
        const bool ok = j >= 0 && j < n_orb && (!status || status[c] == SGF_CONVERGED);
        const int32_t a = ok ? (int32_t)(j >> 2) : 0;
        const int o = (int)(j & 3);
        const int32_t t0 = ok ? row_ptr[a] : 0, t1 = ok ? row_ptr[a + 1] : 0;
        for (int64_t r = proj_off[c] + lane; r < proj_off[c + 1]; r += TR_COEF_L) {
            const int32_t i = proj_row[r];
            const int32_t b = i >> 2;
            const int q = i & 3;
            int32_t t = -1;
            for (int32_t u = t0; u < t1; ++u)  // a block row holds a handful of blocks
                if (col[u] == b) { t = u; break; }
            double sv = 0.0, hv = 0.0;
            if (t >= 0) {
                hv = h[16 * (int64_t)t + 4 * o + q];
                sv = s ? s[16 * (int64_t)t + 4 * o + q] : (i == j ? 1.0 : 0.0);
            }
            coef[r] = make_double2(sv, hv);
        }
    }
}

constexpr int ED_T = 256;   // threads per workgroup of the energy-density pass
constexpr int ED_MAXK = 8;  // shifts per lane (512 / 64)
constexpr int ED_NB = 8192; // workgroups (grid-stride over rows)

// eps_t = -(1/pi) sum_k Im(w_k z_k G_t(z_k)): one wavefront per projection
// row (grid-stride), lane l reading shifts l, l + 64, ... of the row, so each
// load of a wavefront is 1 KiB of contiguous G.  The weights w_k z_k of a
// lane's shifts stay in registers.  Fixed summation order.
__global__ __launch_bounds__(ED_T) void k_energy_density(int64_t n_rows, int32_t ns, const double2 *z,
                                                         const double2 *w, const double2 *G, double *eps) {
    const int lane = threadIdx.x & 63;
    double2 c[ED_MAXK];
#pragma unroll
    for (int u = 0; u < ED_MAXK; ++u) {
        const int k = lane + 64 * u;
        c[u] = k < ns ? cmul(w[k], z[k]) : make_double2(0.0, 0.0);
    }
    const int64_t nw = ((int64_t)gridDim.x * ED_T) >> 6;
    for (int64_t r = ((int64_t)blockIdx.x * ED_T + threadIdx.x) >> 6; r < n_rows; r += nw) {
        const double2 *g = G + r * ns;
        double2 v[ED_MAXK];
#pragma unroll
        for (int u = 0; u < ED_MAXK; ++u) {
            const int k = lane + 64 * u;
            v[u] = (64 * u < ns && k < ns) ? g[k] : make_double2(0.0, 0.0);
        }
        double t = 0.0;
#pragma unroll
        for (int u = 0; u < ED_MAXK; ++u) t = fma(c[u].x, v[u].y, fma(c[u].y, v[u].x, t));
        t = wave_reduce(t);
        if (lane == 0) eps[r] = -t * INV_PI_D;
    }
}

// Partial traces over a contiguous chunk of projection rows per workgroup;
// thread k owns shift k (and k + blockDim.x, ...).  Rows are summed in order.
__global__ void k_trace_partial(int64_t n_rows, int32_t ns, const double2 *G, const double2 *coef, double2 *part) {
    const int64_t per = (n_rows + gridDim.x - 1) / gridDim.x;
    const int64_t r0 = (int64_t)blockIdx.x * per;
    const int64_t r1 = r0 + per < n_rows ? r0 + per : n_rows;
    for (int k = threadIdx.x; k < ns; k += blockDim.x) {
        double tx = 0.0, ty = 0.0, ux = 0.0, uy = 0.0;
        int64_t r = r0;
        for (; r + TR_UNROLL <= r1; r += TR_UNROLL) {
            double2 g[TR_UNROLL], cf[TR_UNROLL];
#pragma unroll
            for (int u = 0; u < TR_UNROLL; ++u) {
                g[u] = G[(r + u) * ns + k];
                cf[u] = coef[r + u];
            }
#pragma unroll
            for (int u = 0; u < TR_UNROLL; ++u) {
                tx = fma(cf[u].x, g[u].x, tx);
                ty = fma(cf[u].x, g[u].y, ty);
                ux = fma(cf[u].y, g[u].x, ux);
                uy = fma(cf[u].y, g[u].y, uy);
            }
        }
        for (; r < r1; ++r) {
            const double2 g = G[r * ns + k], cf = coef[r];
            tx = fma(cf.x, g.x, tx);
            ty = fma(cf.x, g.y, ty);
            ux = fma(cf.y, g.x, ux);
            uy = fma(cf.y, g.y, uy);
        }
        part[((size_t)blockIdx.x * ns + k) * 2] = make_double2(tx, ty);
        part[((size_t)blockIdx.x * ns + k) * 2 + 1] = make_double2(ux, uy);
    }
}

// Fixed-shape sum of the block's (t, u) pairs: strided per thread, then an
// LDS tree, so the result does not depend on timing.
__device__ inline void tree_sum2(double2 &t, double2 &u, double2 (*red)[2]) {
    red[threadIdx.x][0] = t;
    red[threadIdx.x][1] = u;
    __syncthreads();
    for (int off = TR_RED_T / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            red[threadIdx.x][0] = cadd(red[threadIdx.x][0], red[threadIdx.x + off][0]);
            red[threadIdx.x][1] = cadd(red[threadIdx.x][1], red[threadIdx.x + off][1]);
        }
        __syncthreads();
    }
    t = red[0][0];
    u = red[0][1];
}

// T_k and U_k: one workgroup per shift adds the partials of all workgroups
// of the partial pass.
__global__ __launch_bounds__(TR_RED_T) void k_trace_final(int32_t ns, int nb, const double2 *part, double2 *T,
                                                          double2 *U) {
    __shared__ double2 red[TR_RED_T][2];
    const int k = blockIdx.x;
    double2 t = make_double2(0.0, 0.0), u = make_double2(0.0, 0.0);
    for (int b = threadIdx.x; b < nb; b += TR_RED_T) {
        t = cadd(t, part[((size_t)b * ns + k) * 2]);
        u = cadd(u, part[((size_t)b * ns + k) * 2 + 1]);
    }
    tree_sum2(t, u, red);
    if (threadIdx.x == 0) {
        T[k] = t;
        U[k] = u;
    }
}

// tr(rho S) and tr(rho H) over the projection rows: per-workgroup sums
// (thread-strided, then a fixed LDS tree), added in workgroup order.
__global__ __launch_bounds__(TR_RHO_T) void k_trace_rho_partial(int64_t n_rows, const double *rho, const double2 *coef,
                                                                 double2 *part) {
    __shared__ double2 red[TR_RHO_T];
    const int64_t per = (n_rows + gridDim.x - 1) / gridDim.x;
    const int64_t r0 = (int64_t)blockIdx.x * per;
    const int64_t r1 = r0 + per < n_rows ? r0 + per : n_rows;
    double ts = 0.0, th = 0.0;
    for (int64_t r = r0 + threadIdx.x; r < r1; r += TR_RHO_T) {
        const double2 cf = coef[r];
        ts = fma(cf.x, rho[r], ts);
        th = fma(cf.y, rho[r], th);
    }
    red[threadIdx.x] = make_double2(ts, th);
    __syncthreads();
    for (int off = TR_RHO_T / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] = cadd(red[threadIdx.x], red[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(TR_RED_T) void k_trace_rho_final(int nb, const double2 *part, double *out) {
    __shared__ double2 red[TR_RED_T][2];
    double2 t = make_double2(0.0, 0.0), u = make_double2(0.0, 0.0);
    for (int b = threadIdx.x; b < nb; b += TR_RED_T) t = cadd(t, part[b]);
    tree_sum2(t, u, red);
    if (threadIdx.x == 0) {
        out[0] = t.x;
        out[1] = t.y;
    }
}

struct TraceLayout {
    double2 *coef, *part, *rpart;
    size_t bytes;
};

static TraceLayout trace_layout(int64_t total_rows, int32_t ns, void *base, size_t cap) {
    TraceLayout L;
    Carve c(base, cap);
    L.coef = c.take<double2>((size_t)(total_rows > 0 ? total_rows : 1));
    L.part = c.take<double2>((size_t)TR_NB * (ns > 0 ? ns : 1) * 2);
    L.rpart = c.take<double2>(TR_NB);
    L.bytes = c.used;
    return L;
}

// Trapezoid weight of grid point k for an occupation up to grid point m
// (inclusive): the grid spacing, halved at the two ends of the grid.
static double trap_weight(int32_t n, const double *z, int32_t k) {
    if (n == 1) return 1.0;
    const double de = (z[2 * (n - 1)] - z[0]) / (double)(n - 1);
    return (k == 0 || k == n - 1) ? 0.5 * de : de;
}

}  // namespace sgf

using namespace sgf;

extern "C" sgf_status sgf_trace_workspace(int64_t total_rows, int32_t n_shifts, size_t *ws_bytes) {
    SGF_REQUIRE(ws_bytes && total_rows >= 0 && n_shifts >= 1, "sgf_trace_workspace: bad arguments");
    *ws_bytes = trace_layout(total_rows, n_shifts, nullptr, 0).bytes;
    return SGF_OK;
}

extern "C" sgf_status sgf_traces(const sgf_system *sys, int64_t n_cols, const int64_t *d_cols, const int64_t *d_proj_off,
                                 const int32_t *d_proj_row, const int32_t *d_status, int64_t total_rows,
                                 const double *d_G, const double *d_rho, int32_t n_shifts, void *d_ws,
                                 size_t ws_bytes, double *d_T, double *d_U, double *d_rho_tr, void *stream) {
    SGF_REQUIRE(sys && sys->row_ptr && sys->col && sys->h, "sgf_traces: system has no operator");
    SGF_REQUIRE(n_cols >= 0 && total_rows >= 0, "sgf_traces: negative size");
    SGF_REQUIRE(n_cols == 0 || (d_cols && d_proj_off && d_proj_row), "sgf_traces: column layout is NULL");
    SGF_REQUIRE(d_G || d_rho, "sgf_traces: neither G nor rho given");
    SGF_REQUIRE(!d_G || (d_T && d_U && n_shifts >= 1), "sgf_traces: G needs T, U and n_shifts >= 1");
    SGF_REQUIRE(!d_rho || d_rho_tr, "sgf_traces: rho needs rho_tr");
    SGF_REQUIRE(d_ws, "sgf_traces: workspace is NULL");
    const TraceLayout L = trace_layout(total_rows, n_shifts > 0 ? n_shifts : 1, d_ws, ws_bytes);
    SGF_REQUIRE(L.bytes <= ws_bytes, "sgf_traces: workspace %zu bytes < %zu", ws_bytes, L.bytes);
    hipStream_t st = as_stream(stream);
    if (n_cols > 0) {
        const int64_t per_wg = 256 / TR_COEF_L;
        const unsigned g = (unsigned)((n_cols + per_wg - 1) / per_wg < 65536 ? (n_cols + per_wg - 1) / per_wg : 65536);
        k_trace_coef<<<g, 256, 0, st>>>(n_cols, 4 * sys->n_atoms, d_cols, d_proj_off, d_proj_row, d_status,
                                        sys->row_ptr, sys->col, sys->h, sys->s, L.coef);
        SGF_LAUNCHED();
    }
    const int nb = total_rows > 0 ? (int)(total_rows < TR_NB ? total_rows : TR_NB) : 1;
    if (d_G) {
        const int threads = ((n_shifts + 63) / 64) * 64 > 512 ? 512 : ((n_shifts + 63) / 64) * 64;
        k_trace_partial<<<nb, threads, 0, st>>>(total_rows, n_shifts, reinterpret_cast<const double2 *>(d_G), L.coef,
                                                L.part);
        SGF_LAUNCHED();
        k_trace_final<<<n_shifts, TR_RED_T, 0, st>>>(n_shifts, nb, L.part, reinterpret_cast<double2 *>(d_T),
                                                     reinterpret_cast<double2 *>(d_U));
        SGF_LAUNCHED();
    }
    if (d_rho) {
        k_trace_rho_partial<<<nb, TR_RHO_T, 0, st>>>(total_rows, d_rho, L.coef, L.rpart);
        SGF_LAUNCHED();
        k_trace_rho_final<<<1, TR_RED_T, 0, st>>>(nb, L.rpart, d_rho_tr);
        SGF_LAUNCHED();
    }
    return SGF_OK;
}

extern "C" sgf_status sgf_occupation(int32_t n_shifts, const double *T, const double *U, const double *w, double *n_e,
                                     double *e_band) {
    SGF_REQUIRE(n_shifts >= 1 && T && U && w && n_e && e_band, "sgf_occupation: bad arguments");
    double ne = 0.0, eb = 0.0;
    for (int32_t k = 0; k < n_shifts; ++k) {
        // -(1/pi) Im(w_k T_k)
        ne += -INV_PI_D * (w[2 * k] * T[2 * k + 1] + w[2 * k + 1] * T[2 * k]);
        eb += -INV_PI_D * (w[2 * k] * U[2 * k + 1] + w[2 * k + 1] * U[2 * k]);
    }
    *n_e = ne;
    *e_band = eb;
    return SGF_OK;
}

extern "C" sgf_status sgf_fermi_level(int32_t n_shifts, const double *z, const double *T, const double *U,
                                      double n_target, double *mu, double *n_e, double *e_band) {
    SGF_REQUIRE(n_shifts >= 1 && z && T && U && mu && n_e && e_band, "sgf_fermi_level: bad arguments");
    for (int32_t k = 1; k < n_shifts; ++k)
        SGF_REQUIRE(z[2 * k] > z[2 * (k - 1)], "sgf_fermi_level: Re z must increase along the grid");
    // cumulative occupation N_e(E_m) with the trapezoid weights up to grid point m
    auto count = [&](int32_t m, double *eb) {
        double ne = 0.0, e = 0.0;
        for (int32_t k = 0; k <= m; ++k) {
            const double wk = trap_weight(n_shifts, z, k);
            ne += -INV_PI_D * wk * T[2 * k + 1];
            e += -INV_PI_D * wk * U[2 * k + 1];
        }
        *eb = e;
        return ne;
    };
    double eb_top = 0.0;
    if (count(n_shifts - 1, &eb_top) < n_target) {
        set_error("sgf_fermi_level: %g electrons exceed the occupation of the whole grid", n_target);
        return SGF_EUNSUPPORTED;
    }
    // bisection on the grid index: the smallest m with N_e(E_m) >= n_target
    // (N_e is non-decreasing while every -Im T_k >= 0, which Im (G S)_jj < 0 gives)
    int32_t lo = 0, hi = n_shifts - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi) / 2;
        double eb = 0.0;
        if (count(mid, &eb) >= n_target) hi = mid;
        else lo = mid + 1;
    }
    *mu = z[2 * lo];
    *n_e = count(lo, e_band);
    return SGF_OK;
}

extern "C" sgf_status sgf_energy_density(int64_t total_rows, int32_t n_shifts, const double *d_z, const double *d_w,
                                         const double *d_G, double *d_eps, void *stream) {
    SGF_REQUIRE(total_rows >= 0 && n_shifts >= 1, "sgf_energy_density: bad sizes");
    if (n_shifts > 64 * ED_MAXK) {
        set_error("sgf_energy_density: %d shifts (limit %d)", n_shifts, 64 * ED_MAXK);
        return SGF_EUNSUPPORTED;
    }
    if (total_rows == 0) return SGF_OK;
    SGF_REQUIRE(d_z && d_w && d_G && d_eps, "sgf_energy_density: NULL argument");
    const int64_t wgs = (total_rows + ED_T / 64 - 1) / (ED_T / 64);
    k_energy_density<<<(unsigned)(wgs < ED_NB ? wgs : ED_NB), ED_T, 0, as_stream(stream)>>>(
        total_rows, n_shifts, reinterpret_cast<const double2 *>(d_z), reinterpret_cast<const double2 *>(d_w),
        reinterpret_cast<const double2 *>(d_G), d_eps);
    SGF_LAUNCHED();
    return SGF_OK;
}
