// wp.hip -- time propagation of wavepackets with the tight-binding H
// (Sec. 3 of the paper, Fig. 2: d/dt Psi = -i H Psi / hbar, steps of 0.1 fs), by the
// Chebyshev expansion of the step operator (Tal-Ezer and Kosloff 1984):
// with H = a X + b (spectrum of X in [-1, 1], a and b from Gershgorin
// bounds) and tau = h / hbar,
//     exp(-i tau H) = exp(-i tau b) sum_{k < K} c_k T_k(X),
//     c_0 = J_0(a tau), c_k = 2 (-i)^k J_k(a tau),
// and T_k(X) Psi from T_{k+1} = 2 X T_k - T_{k-1}.
//
// Each term is one pass over H in HBM fused with the recurrence and the
// accumulation of the series.  One packet: thread per orbital row i forms
// entry i of H T_k.  Several packets: thread per (atom A, packet r), packets
// fastest, forms the four entries of A's rows for packet r from whole 4 x 4
// blocks, so a block of H and a neighbour's four entries of T_k are each
// read once per thread (the n_rhs threads of an atom share the block's loads
// through the cache; a thread per orbital row read every entry of T_k four
// times over).  Then
// T_{k+1} = (2/a)(H T_k - b T_k) - T_{k-1} and acc += c_{k+1} T_{k+1}.
// T_{k+1} overwrites T_{k-1} in place (only this thread reads that entry),
// and the last term writes the finished step, acc + c_{K-1} T_{K-1}, there
// too.  Per term and packet: 64 flops per block against 128 bytes of H, so
// the pass is bound by HBM bandwidth.
#include <cmath>
#include <vector>

#include "common.hpp"

namespace sgf {

namespace {

constexpr double HBAR_EV_FS = 0.6582119569509066;  // eV fs (CODATA 2018)
constexpr int WP_T = 256;

enum { TERM_FIRST = 0, TERM_MID = 1, TERM_LAST = 2 };

// One term of the series.  x = T_k (read by neighbours), z = T_{k-1} (read
// and overwritten by this thread), acc = sum so far.  FIRST: x = T_0, writes
// T_1 to z and c_0 T_0 + c_1 T_1 to acc.  MID: writes T_{k+1} to z and adds
// c_{k+1} T_{k+1} to acc.  LAST: writes acc + c_{k+1} T_{k+1} to z.
template <int NRHS, int MODE>
__global__ __launch_bounds__(WP_T) void k_cheb_term(int64_t n_atoms, const int32_t *__restrict__ row_ptr,
                                                    const int32_t *__restrict__ col,
                                                    const double *__restrict__ h, double scale, double shift,
                                                    double2 c_new, double2 c_0, const double2 *__restrict__ x,
                                                    double2 *__restrict__ z, double2 *__restrict__ acc) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t i = gid / NRHS;  // orbital row
    const int r = (int)(gid % NRHS);
    const int64_t A = i >> 2;
    const int o = (int)(i & 3);
    if (A >= n_atoms) return;
    double hx = 0.0, hy = 0.0;
    const int t0 = row_ptr[A], t1 = row_ptr[A + 1];
    for (int t = t0; t < t1; ++t) {
        const int64_t B = col[t];
        double hr[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) hr[q] = h[16 * (int64_t)t + 4 * o + q];
        const double2 *xb = x + 4 * B * NRHS + r;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double2 v = xb[q * NRHS];
            hx = fma(hr[q], v.x, hx);
            hy = fma(hr[q], v.y, hy);
        }
    }
    const int64_t e = i * NRHS + r;
    const double2 xi = x[e];
    // X T_k = (H T_k - b T_k) / a, scaled by 1 (first term) or 2
    double2 tn = make_double2(scale * fma(-shift, xi.x, hx), scale * fma(-shift, xi.y, hy));
    if (MODE != TERM_FIRST) tn = csub(tn, z[e]);
    double2 s;
    if (MODE == TERM_FIRST)
        s = cfma(c_0, xi, cmul(c_new, tn));
    else
        s = cfma(c_new, tn, acc[e]);
    if (MODE == TERM_LAST) {
        z[e] = s;
    } else {
        z[e] = tn;
        acc[e] = s;
    }
}

// The same term with a thread per (atom, packet): the four rows of atom A
// for packet r.  Each row sums its products in the order of the row
// variant, so both give the same bits.
template <int NRHS, int MODE>
__global__ __launch_bounds__(WP_T) void k_cheb_term_atom(int64_t n_atoms, const int32_t *__restrict__ row_ptr,
                                                         const int32_t *__restrict__ col,
                                                         const double *__restrict__ h, double scale, double shift,
                                                         double2 c_new, double2 c_0, const double2 *__restrict__ x,
                                                         double2 *__restrict__ z, double2 *__restrict__ acc) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t A = gid / NRHS;
    const int r = (int)(gid % NRHS);
    if (A >= n_atoms) return;
    double hx[4] = {0.0, 0.0, 0.0, 0.0}, hy[4] = {0.0, 0.0, 0.0, 0.0};
    const int t0 = row_ptr[A], t1 = row_ptr[A + 1];
    for (int t = t0; t < t1; ++t) {
        const int64_t B = col[t];
        const double2 *hb = reinterpret_cast<const double2 *>(h + 16 * (int64_t)t);
        double2 hv[8];  // row o of the block: hv[2 o] = (h_o0, h_o1), hv[2 o + 1] = (h_o2, h_o3)
#pragma unroll
        for (int k = 0; k < 8; ++k) hv[k] = hb[k];
        const double2 *xb = x + 4 * B * NRHS + r;
        double2 v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = xb[q * NRHS];
#pragma unroll
        for (int o = 0; o < 4; ++o) {
            const double hr[4] = {hv[2 * o].x, hv[2 * o].y, hv[2 * o + 1].x, hv[2 * o + 1].y};
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                hx[o] = fma(hr[q], v[q].x, hx[o]);
                hy[o] = fma(hr[q], v[q].y, hy[o]);
            }
        }
    }
#pragma unroll
    for (int o = 0; o < 4; ++o) {
        const int64_t e = (4 * A + o) * NRHS + r;
        const double2 xi = x[e];
        double2 tn = make_double2(scale * fma(-shift, xi.x, hx[o]), scale * fma(-shift, xi.y, hy[o]));
        if (MODE != TERM_FIRST) tn = csub(tn, z[e]);
        double2 s;
        if (MODE == TERM_FIRST)
            s = cfma(c_0, xi, cmul(c_new, tn));
        else
            s = cfma(c_new, tn, acc[e]);
        if (MODE == TERM_LAST) {
            z[e] = s;
        } else {
            z[e] = tn;
            acc[e] = s;
        }
    }
}

// Gershgorin discs per orbital row: per-workgroup min of H_ii - R_i and max
// of H_ii + R_i, R_i = sum_{j != i} |H_ij|.
__global__ __launch_bounds__(WP_T) void k_gershgorin(int64_t n_atoms, const int32_t *__restrict__ row_ptr,
                                                     const int32_t *__restrict__ col, const double *__restrict__ h,
                                                     double2 *__restrict__ part) {
    __shared__ double lo[WP_T], hi[WP_T];
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t A = gid >> 2;
    const int o = (int)(gid & 3);
    double l = INFINITY, u = -INFINITY;
    if (A < n_atoms) {
        double d = 0.0, rad = 0.0;
        for (int t = row_ptr[A]; t < row_ptr[A + 1]; ++t) {
            const bool diag_blk = col[t] == A;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const double v = h[16 * (int64_t)t + 4 * o + q];
                if (diag_blk && q == o) d += v;
                else rad += fabs(v);
            }
        }
        l = d - rad;
        u = d + rad;
    }
    lo[threadIdx.x] = l;
    hi[threadIdx.x] = u;
    __syncthreads();
    for (int off = WP_T / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            lo[threadIdx.x] = fmin(lo[threadIdx.x], lo[threadIdx.x + off]);
            hi[threadIdx.x] = fmax(hi[threadIdx.x], hi[threadIdx.x + off]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = make_double2(lo[0], hi[0]);
}

template <int MODE>
void launch_term(int n_rhs, hipStream_t st, const sgf_system *sys, double scale, double shift, double2 c_new,
                 double2 c_0, const double2 *x, double2 *z, double2 *acc) {
    const int64_t n = sys->n_atoms;
    const dim3 rows((unsigned)((4 * n + WP_T - 1) / WP_T));
    const dim3 atoms((unsigned)((n * n_rhs + WP_T - 1) / WP_T));
    switch (n_rhs) {
        case 1: k_cheb_term<1, MODE><<<rows, WP_T, 0, st>>>(n, sys->row_ptr, sys->col, sys->h, scale, shift, c_new, c_0, x, z, acc); break;
        case 2: k_cheb_term_atom<2, MODE><<<atoms, WP_T, 0, st>>>(n, sys->row_ptr, sys->col, sys->h, scale, shift, c_new, c_0, x, z, acc); break;
        case 4: k_cheb_term_atom<4, MODE><<<atoms, WP_T, 0, st>>>(n, sys->row_ptr, sys->col, sys->h, scale, shift, c_new, c_0, x, z, acc); break;
        default: k_cheb_term_atom<8, MODE><<<atoms, WP_T, 0, st>>>(n, sys->row_ptr, sys->col, sys->h, scale, shift, c_new, c_0, x, z, acc); break;
    }
}

int64_t gersh_blocks(int64_t n_atoms) { return (4 * n_atoms + WP_T - 1) / WP_T; }

// J_k(x) for k = 0 .. n-1 (the C library's Bessel functions of the first kind)
std::vector<double> bessel_j(int n, double x) {
    std::vector<double> j(n);
    for (int k = 0; k < n; ++k) j[k] = ::jn(k, x);
    return j;
}

}  // namespace

}  // namespace sgf

using namespace sgf;

extern "C" sgf_status sgf_wp_workspace(int64_t n_atoms, int32_t n_rhs, size_t *ws_bytes) {
    SGF_REQUIRE(ws_bytes && n_atoms > 0 && (n_rhs == 1 || n_rhs == 2 || n_rhs == 4 || n_rhs == 8),
                "sgf_wp_workspace: bad arguments");
    const size_t vec = align_up((size_t)4 * n_atoms * n_rhs * 16);
    const size_t part = align_up((size_t)gersh_blocks(n_atoms) * 16);
    *ws_bytes = 2 * vec > part ? 2 * vec : part;
    return SGF_OK;
}

extern "C" sgf_status sgf_wp_bounds(const sgf_system *sys, void *d_ws, size_t ws_bytes, double *e_min, double *e_max,
                                    void *stream) {
    SGF_REQUIRE(sys && d_ws && e_min && e_max, "sgf_wp_bounds: NULL argument");
    SGF_REQUIRE(sys->row_ptr && sys->col && sys->h && sys->n_atoms > 0, "sgf_wp_bounds: system incomplete");
    const int64_t nb = gersh_blocks(sys->n_atoms);
    SGF_REQUIRE((size_t)nb * 16 <= ws_bytes, "sgf_wp_bounds: workspace %zu bytes < %zu", ws_bytes,
                (size_t)nb * 16);
    hipStream_t st = as_stream(stream);
    double2 *part = static_cast<double2 *>(d_ws);
    k_gershgorin<<<(unsigned)nb, WP_T, 0, st>>>(sys->n_atoms, sys->row_ptr, sys->col, sys->h, part);
    SGF_LAUNCHED();
    std::vector<double2> hp((size_t)nb);
    SGF_HIP(hipMemcpyAsync(hp.data(), part, (size_t)nb * 16, hipMemcpyDeviceToHost, st));
    SGF_HIP(hipStreamSynchronize(st));
    double lo = INFINITY, hi = -INFINITY;
    for (const double2 &p : hp) {
        lo = p.x < lo ? p.x : lo;
        hi = p.y > hi ? p.y : hi;
    }
    *e_min = lo;
    *e_max = hi;
    return SGF_OK;
}

extern "C" sgf_status sgf_wp_terms(double a_tau, double tol, int32_t *n_terms) {
    SGF_REQUIRE(n_terms && std::isfinite(a_tau) && tol > 0.0 && tol < 1.0, "sgf_wp_terms: bad arguments");
    const double x = std::fabs(a_tau);
    // the smallest K > |a tau| whose J_K and J_{K+1} are both <= tol
    int k = (int)std::floor(x) + 1;
    while (!(std::fabs(::jn(k, x)) <= tol && std::fabs(::jn(k + 1, x)) <= tol)) {
        ++k;
        SGF_REQUIRE(k < 100000, "sgf_wp_terms: no cut found");
    }
    *n_terms = k < 3 ? 3 : k;
    return SGF_OK;
}

extern "C" sgf_status sgf_wp_propagate(const sgf_system *sys, int32_t n_rhs, double *d_psi, double h_fs,
                                       int32_t n_steps, double e_min, double e_max, int32_t n_terms, void *d_ws,
                                       size_t ws_bytes, void *stream) {
    SGF_REQUIRE(sys && d_psi && d_ws, "sgf_wp_propagate: NULL argument");
    SGF_REQUIRE(sys->row_ptr && sys->col && sys->h && sys->n_atoms > 0, "sgf_wp_propagate: system incomplete");
    if (sys->s) {
        set_error("sgf_wp_propagate: the propagation is defined for an orthogonal basis (S = I)");
        return SGF_EUNSUPPORTED;
    }
    SGF_REQUIRE(n_rhs == 1 || n_rhs == 2 || n_rhs == 4 || n_rhs == 8, "sgf_wp_propagate: n_rhs must be 1, 2, 4 or 8");
    SGF_REQUIRE(((uintptr_t)sys->h & 15) == 0 && ((uintptr_t)d_psi & 15) == 0 && ((uintptr_t)d_ws & 15) == 0,
                "sgf_wp_propagate: h, psi and the workspace must be 16-byte aligned");
    SGF_REQUIRE(n_steps >= 0 && n_terms >= 3 && n_terms <= 100000, "sgf_wp_propagate: need n_steps >= 0, n_terms >= 3");
    SGF_REQUIRE(std::isfinite(h_fs) && std::isfinite(e_min) && std::isfinite(e_max) && e_max > e_min,
                "sgf_wp_propagate: need finite h and e_max > e_min");
    size_t need = 0;
    SGF_REQUIRE(sgf_wp_workspace(sys->n_atoms, n_rhs, &need) == SGF_OK && need <= ws_bytes,
                "sgf_wp_propagate: workspace %zu bytes < %zu", ws_bytes, need);
    if (n_steps == 0) return SGF_OK;
    const double a = 0.5 * (e_max - e_min), b = 0.5 * (e_max + e_min);
    const double tau = h_fs / HBAR_EV_FS;
    // c_k exp(-i tau b): c_0 = J_0(a tau), c_k = 2 (-i)^k J_k(a tau)
    const std::vector<double> J = bessel_j(n_terms, a * tau);
    const double pr = std::cos(tau * b), pi = -std::sin(tau * b);
    std::vector<double2> c((size_t)n_terms);
    for (int k = 0; k < n_terms; ++k) {
        const double m = (k == 0 ? 1.0 : 2.0) * J[k];
        double re = 0.0, im = 0.0;  // m (-i)^k
        switch (k & 3) {
            case 0: re = m; break;
            case 1: im = -m; break;
            case 2: re = -m; break;
            default: im = m; break;
        }
        c[k] = make_double2(re * pr - im * pi, re * pi + im * pr);
    }
    const size_t vec = align_up((size_t)4 * sys->n_atoms * n_rhs * 16);
    double2 *bufs[3] = {reinterpret_cast<double2 *>(d_psi), static_cast<double2 *>(d_ws),
                        reinterpret_cast<double2 *>(static_cast<char *>(d_ws) + vec)};
    hipStream_t st = as_stream(stream);
    int cur = 0;  // buffer holding Psi at the start of the step
    for (int step = 0; step < n_steps; ++step) {
        const int acc = (cur + 2) % 3;
        int x = cur, z = (cur + 1) % 3;
        // T_1 into z, c_0 T_0 + c_1 T_1 into acc
        launch_term<TERM_FIRST>(n_rhs, st, sys, 1.0 / a, b, c[1], c[0], bufs[x], bufs[z], bufs[acc]);
        SGF_LAUNCHED();
        // x = T_1, z = T_0: T_{k+1} replaces T_{k-1}
        int xx = z, zz = x;
        for (int k = 2; k < n_terms; ++k) {
            if (k + 1 < n_terms)
                launch_term<TERM_MID>(n_rhs, st, sys, 2.0 / a, b, c[k], c[0], bufs[xx], bufs[zz], bufs[acc]);
            else
                launch_term<TERM_LAST>(n_rhs, st, sys, 2.0 / a, b, c[k], c[0], bufs[xx], bufs[zz], bufs[acc]);
            SGF_LAUNCHED();
            const int t = xx;
            xx = zz;
            zz = t;
        }
        // the last term wrote the finished step where T_{K-1} would go (now xx)
        cur = xx;
    }
    if (cur != 0)
        SGF_HIP(hipMemcpyAsync(d_psi, bufs[cur], (size_t)4 * sys->n_atoms * n_rhs * 16, hipMemcpyDeviceToDevice, st));
    return SGF_OK;
}
