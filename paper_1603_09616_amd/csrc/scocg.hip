// scocg.hip -- shifted COCG for many columns in two passes.
//
// Seed pass (k_seed): one wavefront per column, pulling columns from a work
// queue.  It runs COCG on the seed system z_s - H inside the column's local
// subspace (vectors in LDS, wavefront DPP reductions, no workgroup barrier),
// steps the collinearity factors pi^k of every shift only to decide when each
// shift k has converged, and records per iteration 1/alpha_n and
// beta_n/alpha_n together with the residual r_n restricted to the projection
// rows P.
//
// Shift pass (k_shift): one workgroup per column, one lane per shift.  The
// seed recurrences say (z_s - H) R = R T - r_N e^T / alpha_{N-1} with the
// tridiagonal T (diagonal 1/alpha_n + beta_{n-1}/alpha_{n-1}, superdiagonal
// -beta_n/alpha_n, subdiagonal -1/alpha_n), so the shifted Galerkin solution
// after N_k steps is x^k = R y^k with (T_{N_k} + sigma_k) y^k = e_0.  Each lane
// factors that tridiagonal from the bottom up (UL, no pivoting: T + sigma_k is
// similar to z_k - T_L with T_L the real Lanczos matrix of H, whose trailing
// minors cannot vanish for Im z_k > 0) and accumulates the rows of P by
// Horner's rule on the way:  G^k_P = y_0 S_0,  S_m = r_{m,P} + g_{m+1} S_{m+1}.
// Mathematically this is the x^k of the shifted recurrences of Frommer (2003)
// / Takayama et al. (2006); it costs 8 flops per row and step instead of 22
// and has no barriers, so the shift work streams at FP64 ALU rate.
#include "scocg.hpp"

#include <mutex>
#include <vector>

namespace sgf {


// ---------------------------------------------------------------------------
// Seed pass
// ---------------------------------------------------------------------------
template <bool STAGE, int M>
__global__ __launch_bounds__(SEED_T) void k_seed(SolveArgs a) {
    extern __shared__ double4 lds4[];
    char *lds = reinterpret_cast<char *>(lds4);
    double2 *vp = reinterpret_cast<double2 *>(lds + a.off_p);
    double2 *vs = reinterpret_cast<double2 *>(lds + a.off_s);
    double2 *vw = reinterpret_cast<double2 *>(lds + a.off_w);
    double *hs = reinterpret_cast<double *>(lds + a.off_hs);
    int32_t *cs = reinterpret_cast<int32_t *>(lds + a.off_cs);
    int32_t *rs = reinterpret_cast<int32_t *>(lds + a.off_rs);
    const int lane = threadIdx.x;
    const double2 zs = a.z[a.seed];
    double2 sigma[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int k = lane + 64 * m;
        sigma[m] = k < a.ns ? csub(a.z[k], zs) : make_double2(0.0, 0.0);
    }
    const double tol2 = a.tol * a.tol;

    for (;;) {
        int64_t ticket = 0;
        if (lane == 0) ticket = (int64_t)atomicAdd(reinterpret_cast<unsigned long long *>(a.ticket), 1ull);
        ticket = __shfl(ticket, 0, 64);
        if (ticket >= a.batch_end - a.batch_begin) break;
        const int64_t slot = ticket;
        ticket += a.batch_begin;
        const int64_t c = a.order ? (int64_t)a.order[ticket] : ticket;
        ColMeta *meta = &a.meta[slot];
        if (c < 0 || c >= a.n_cols) {
            if (lane == 0) *meta = ColMeta{-1, 0, 0, SGF_BADCOLUMN};
            continue;
        }
        const int64_t j = a.cols[c];
        const int32_t pl = a.col_plan[c];
        bool bad = pl < 0 || pl >= a.n_plans || j < 0;
        int64_t a0 = 0, b0 = 0, p0 = 0;
        int n_loc = 0, nblk = 0, npa = 0, cl = 0;
        if (!bad) {
            a0 = a.atom_off[pl];
            n_loc = (int)(a.atom_off[pl + 1] - a0);
            b0 = a.blk_off[pl];
            nblk = (int)(a.blk_off[pl + 1] - b0);
            p0 = a.pa_off[pl];
            npa = (int)(a.pa_off[pl + 1] - p0);
            cl = a.center_loc[pl];
            bad = n_loc < 1 || n_loc > a.max_loc_atoms || npa < 1 || 4 * npa > a.rmax ||
                  (STAGE && nblk > a.max_loc_blocks) || cl < 0 || cl >= n_loc ||
                  a.loc_atom[a0 + cl] != (int32_t)(j >> 2);
        }
        if (bad) {
            if (lane == 0) {
                *meta = ColMeta{-1, 0, 0, SGF_BADCOLUMN};
                a.iters[c] = 0;
                a.status[c] = SGF_BADCOLUMN;
            }
            continue;
        }
        const int nl = 4 * n_loc;
        const int jl = 4 * cl + (int)(j & 3);
        const int nprow = 4 * npa;  // <= 32 (checked on the host)
        const int prow = lane < nprow ? 4 * a.pa_loc[p0 + (lane >> 2)] + (lane & 3) : 0;
        double2 *hab = a.hab + (size_t)slot * a.cap * 2;
        double2 *hr = a.hr + (size_t)slot * (a.cap + 1) * a.rmax;

        // start: x = 0, s_0 = p_0 = e_jl (S = I: r = s, q = p)
        for (int i = lane; i < nl; i += SEED_T) {
            const double2 v = make_double2(i == jl ? 1.0 : 0.0, 0.0);
            vp[i] = v;
            vs[i] = v;
        }
        if (STAGE) {
            for (int e = lane; e < nblk * 16; e += SEED_T)
                hs[e] = a.h[16 * (int64_t)a.lblk[2 * (b0 + (e >> 4)) + 1] + (e & 15)];
            for (int t = lane; t < nblk; t += SEED_T) cs[t] = a.lblk[2 * (b0 + t)];
            for (int A = lane; A <= n_loc; A += SEED_T) rs[A] = A < n_loc ? a.lrow[a0 + A] : nblk;
        }
        if (lane < nprow) hr[lane] = make_double2(prow == jl ? 1.0 : 0.0, 0.0);
        wave_lds_fence();

        double2 pc[M], po[M];
        bool act[M];
        int nkm[M];
        double res[M];
#pragma unroll
        for (int m = 0; m < M; ++m) {
            pc[m] = po[m] = make_double2(1.0, 0.0);
            act[m] = lane + 64 * m < a.ns;
            nkm[m] = 0;
            res[m] = 1.0;
        }
        double2 rho = make_double2(1.0, 0.0);
        double2 alpha_old = make_double2(1.0, 0.0), beta_old = make_double2(0.0, 0.0);
        int status = SGF_MAXITER, iters = 0, applied = 0;
        double snorm2 = 1.0;
        const int max_iter = a.max_iter > 0 ? a.max_iter : 10 * nl;  // <= cap by construction

        for (int it = 0; it < max_iter; ++it) {
            // w = z_s p - H p ; mu = p^T w
            double m0 = 0.0, m1 = 0.0;
            for (int i = lane; i < nl; i += SEED_T) {
                const int A = i >> 2, o = i & 3;
                double ax = 0.0, ay = 0.0;
                int t0, t1;
                if (STAGE) { t0 = rs[A]; t1 = rs[A + 1]; }
                else { t0 = a.lrow[a0 + A]; t1 = A + 1 < n_loc ? a.lrow[a0 + A + 1] : nblk; }
                for (int t = t0; t < t1; ++t) {
                    const double *hrow;
                    int B;
                    if (STAGE) { hrow = &hs[16 * t + 4 * o]; B = cs[t]; }
                    else {
                        B = a.lblk[2 * (b0 + t)];
                        hrow = &a.h[16 * (int64_t)a.lblk[2 * (b0 + t) + 1] + 4 * o];
                    }
                    const double2 *pb = &vp[4 * B];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const double hv = hrow[q];
                        const double2 pv = pb[q];
                        ax = fma(hv, pv.x, ax);
                        ay = fma(hv, pv.y, ay);
                    }
                }
                const double2 pi_ = vp[i];
                const double2 wi = make_double2(zs.x * pi_.x - zs.y * pi_.y - ax, zs.x * pi_.y + zs.y * pi_.x - ay);
                vw[i] = wi;
                m0 = fma(pi_.x, wi.x, fma(-pi_.y, wi.y, m0));
                m1 = fma(pi_.x, wi.y, fma(pi_.y, wi.x, m1));
            }
            const double2 mu = make_double2(wave_reduce(m0), wave_reduce(m1));
            iters = it + 1;
            if (!cfinite(mu) || !cfinite(rho)) { status = SGF_NONFINITE; break; }
            if (mu.x == 0.0 && mu.y == 0.0) { status = SGF_BREAKDOWN; break; }
            const double2 alpha = cdiv(rho, mu);

            // s -= alpha w ; rho' = s^T s ; ||s||^2
            double r0 = 0.0, r1 = 0.0, r2 = 0.0;
            for (int i = lane; i < nl; i += SEED_T) {
                const double2 si = csub(vs[i], cmul(alpha, vw[i]));
                vs[i] = si;
                r0 = fma(si.x, si.x, fma(-si.y, si.y, r0));
                r1 = fma(2.0 * si.x, si.y, r1);
                r2 = fma(si.x, si.x, fma(si.y, si.y, r2));
            }
            const double2 rho_new = make_double2(wave_reduce(r0), wave_reduce(r1));
            snorm2 = wave_reduce(r2);
            const double2 ia = crcp(alpha);
            const double2 beta = cmul(rho_new, crcp(rho));
            for (int i = lane; i < nl; i += SEED_T) vp[i] = cfma(beta, vp[i], vs[i]);

            // history of this step: 1/alpha_n, beta_n/alpha_n and r_{n+1} on P
            if (lane == 0) {
                hab[2 * it] = ia;
                hab[2 * it + 1] = cmul(beta, ia);
            }
            wave_lds_fence();  // s and p of this step are in LDS for every lane
            if (lane < nprow) hr[(size_t)(it + 1) * a.rmax + lane] = vs[prow];

            // collinearity factors of the shifts; freeze test ||s|| <= tol |pi^k|
            const double2 coup = cmul(cmul(alpha, beta_old), crcp(alpha_old));
            int alive = 0;
#pragma unroll
            for (int m = 0; m < M; ++m) {
                if (!act[m]) continue;
                const double2 pn = cadd(cmul(cfma(alpha, sigma[m], make_double2(1.0, 0.0)), pc[m]),
                                        cmul(coup, csub(pc[m], po[m])));
                po[m] = pc[m];
                pc[m] = pn;
                const double pn2 = fma(pn.x, pn.x, pn.y * pn.y);
                if (snorm2 <= tol2 * pn2) {
                    act[m] = false;
                    nkm[m] = it + 1;
                    res[m] = sqrt(snorm2 / pn2);
                } else {
                    alive = 1;
                }
            }
            applied = it + 1;
            alpha_old = alpha;
            beta_old = beta;
            rho = rho_new;
            const bool any_alive = __any(alive);
            if (!any_alive || snorm2 == 0.0) { status = SGF_CONVERGED; break; }
            if (rho_new.x == 0.0 && rho_new.y == 0.0) { status = SGF_BREAKDOWN; break; }
            if (!cfinite(rho_new) || !isfinite(snorm2)) { status = SGF_NONFINITE; break; }
        }

        // shifts still running took every applied update
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int k = lane + 64 * m;
            if (k >= a.ns) continue;
            if (act[m]) {
                nkm[m] = applied;
                const double pn2 = fma(pc[m].x, pc[m].x, pc[m].y * pc[m].y);
                res[m] = applied > 0 ? sqrt(snorm2 / pn2) : 1.0;
            }
            a.nk[(size_t)slot * a.ns_pad + k] = nkm[m];
            if (a.resid) a.resid[c * a.ns + k] = res[m];
            if (a.shift_iters) a.shift_iters[c * a.ns + k] = nkm[m];
        }
        if (lane == 0) {
            *meta = ColMeta{(int32_t)c, iters, npa, status};
            a.iters[c] = iters;
            a.status[c] = status;
        }
        wave_lds_fence();  // LDS reuse by the next column
    }
}

// ---------------------------------------------------------------------------
// Seed pass, register variant for local subspaces of at most 64 orbitals:
// lane i owns row i; s, w, p and the row's blocks of H (with their local
// columns) stay in registers for the whole column, p is mirrored in LDS for
// the neighbour reads of the block product, and each iteration needs two
// complex reciprocals (1/mu and 1/rho') instead of four divisions.
// ---------------------------------------------------------------------------
template <int M, int BMAX>
__global__ __launch_bounds__(SEED_T) void k_seed_r1(SolveArgs a) {
    // p in LDS, orbital-major: vp[16 o + A] is orbital o of local atom A, so
    // the rows of different atoms read by one block-product instruction fall
    // on different LDS banks (atom-major storage put them on two)
    __shared__ double2 vp[64];
    __shared__ __align__(16) double red_mu[2 * 64], red_s[3 * 64];  // wavefront sums through LDS (read as double2)
    const int lane = threadIdx.x;
    const double2 zs = a.z[a.seed];
    double2 sigma[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int k = lane + 64 * m;
        sigma[m] = k < a.ns ? csub(a.z[k], zs) : make_double2(0.0, 0.0);
    }
    const double tol2 = a.tol * a.tol;
    const double2 zero = make_double2(0.0, 0.0), one = make_double2(1.0, 0.0);

    for (;;) {
        int64_t ticket = 0;
        if (lane == 0) ticket = (int64_t)atomicAdd(reinterpret_cast<unsigned long long *>(a.ticket), 1ull);
        ticket = __shfl(ticket, 0, 64);
        if (ticket >= a.batch_end - a.batch_begin) break;
        const int64_t slot = ticket;
        ticket += a.batch_begin;
        const int64_t c = a.order ? (int64_t)a.order[ticket] : ticket;
        ColMeta *meta = &a.meta[slot];
        if (c < 0 || c >= a.n_cols) {
            if (lane == 0) *meta = ColMeta{-1, 0, 0, SGF_BADCOLUMN};
            continue;
        }
        const int64_t j = a.cols[c];
        const int32_t pl = a.col_plan[c];
        bool bad = pl < 0 || pl >= a.n_plans || j < 0;
        int64_t a0 = 0, b0 = 0, p0 = 0;
        int n_loc = 0, nblk = 0, npa = 0, cl = 0;
        if (!bad) {
            a0 = a.atom_off[pl];
            n_loc = (int)(a.atom_off[pl + 1] - a0);
            b0 = a.blk_off[pl];
            nblk = (int)(a.blk_off[pl + 1] - b0);
            p0 = a.pa_off[pl];
            npa = (int)(a.pa_off[pl + 1] - p0);
            cl = a.center_loc[pl];
            bad = n_loc < 1 || n_loc > 16 || npa < 1 || 4 * npa > a.rmax || cl < 0 || cl >= n_loc ||
                  a.loc_atom[a0 + cl] != (int32_t)(j >> 2);
        }
        // this lane's row: its blocks and local columns
        const int nl = 4 * n_loc;
        const int A = lane >> 2, o = lane & 3;
        const bool row = !bad && lane < nl;
        int nb = 0, t0 = 0;
        if (row) {
            t0 = a.lrow[a0 + A];
            nb = (A + 1 < n_loc ? a.lrow[a0 + A + 1] : nblk) - t0;
        }
        bad = bad || __any(nb > BMAX);
        if (bad) {
            if (lane == 0) {
                *meta = ColMeta{-1, 0, 0, SGF_BADCOLUMN};
                a.iters[c] = 0;
                a.status[c] = SGF_BADCOLUMN;
            }
            continue;
        }
        int bcol[BMAX];
        double hrow[BMAX][4];
#pragma unroll
        for (int b = 0; b < BMAX; ++b) {
            bcol[b] = 0;
            hrow[b][0] = hrow[b][1] = hrow[b][2] = hrow[b][3] = 0.0;
            if (b < nb) {
                const int32_t *lb = &a.lblk[2 * (b0 + t0 + b)];
                bcol[b] = lb[0];
                const double *hb = &a.h[16 * (int64_t)lb[1] + 4 * o];
#pragma unroll
                for (int q = 0; q < 4; ++q) hrow[b][q] = hb[q];
            }
        }
        const int jl = 4 * cl + (int)(j & 3);
        int pidx = -1;  // position of this lane's row among the projection rows
        for (int q = 0; q < npa; ++q)
            if (row && a.pa_loc[p0 + q] == A) pidx = 4 * q + o;
        double2 *hab = a.hab + (size_t)slot * a.cap * 2;
        double2 *hr = a.hr + (size_t)slot * (a.cap + 1) * a.rmax;

        // start: x = 0, s_0 = p_0 = e_jl
        double2 s = (row && lane == jl) ? one : zero, p = s;
        vp[16 * o + A] = p;
        if (pidx >= 0) hr[pidx] = s;
        wave_lds_fence();

        double2 pc[M], po[M];
        bool act[M];
        int nkm[M];
        double res[M], fzs[M];  // a frozen shift's |pi^k|^2 and ||s||^2 at its freeze
#pragma unroll
        for (int m = 0; m < M; ++m) {
            pc[m] = po[m] = one;
            act[m] = lane + 64 * m < a.ns;
            nkm[m] = 0;
            res[m] = 1.0;
            fzs[m] = 1.0;
        }
        double2 rho = one, inv_rho = one;
        double2 ba_old = zero;  // beta_{n-1} / alpha_{n-1}
        int status = SGF_MAXITER, iters = 0, applied = 0;
        double snorm2 = 1.0;
        const int max_iter = a.max_iter > 0 ? a.max_iter : 10 * nl;

        for (int it = 0; it < max_iter; ++it) {
            // w = z_s p - H p ; mu = p^T w.  Every lane runs all BMAX blocks:
            // the absent ones hold zeros and point at column 0, which keeps
            // the wavefront free of divergent branches.
            double ax = 0.0, ay = 0.0;
#pragma unroll
            for (int b = 0; b < BMAX; ++b) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const double2 pv = vp[16 * q + bcol[b]];
                    ax = fma(hrow[b][q], pv.x, ax);
                    ay = fma(hrow[b][q], pv.y, ay);
                }
            }
            const double2 w = make_double2(zs.x * p.x - zs.y * p.y - ax, zs.x * p.y + zs.y * p.x - ay);
            double2 mu;
            {
                const double part[2] = {fma(p.x, w.x, -p.y * w.y), fma(p.x, w.y, p.y * w.x)};
                double sum[2];
                wave_sum_lds<2>(part, red_mu, sum);
                mu = make_double2(sum[0], sum[1]);
            }
            iters = it + 1;
            if (!cfinite(mu)) { status = SGF_NONFINITE; break; }  // rho was checked when it was formed
            if (mu.x == 0.0 && mu.y == 0.0) { status = SGF_BREAKDOWN; break; }
            const double2 alpha = cmul(rho, crcp(mu));
            const double2 ia = cmul(mu, inv_rho);  // 1/alpha

            // s -= alpha w ; rho' = s^T s ; ||s||^2
            s = csub(s, cmul(alpha, w));
            double2 rho_new;
            {
                const double part[3] = {fma(s.x, s.x, -s.y * s.y), 2.0 * s.x * s.y, fma(s.x, s.x, s.y * s.y)};
                double sum[3];
                wave_sum_lds<3>(part, red_s, sum);
                rho_new = make_double2(sum[0], sum[1]);
                snorm2 = sum[2];
            }
            const double2 beta = cmul(rho_new, inv_rho);
            const double2 ba = cmul(beta, ia);  // beta_n / alpha_n
            p = cfma(beta, p, s);
            vp[16 * o + A] = p;

            // history: 1/alpha_n, beta_n/alpha_n, r_{n+1} on P
            if (lane == 0) {
                hab[2 * it] = ia;
                hab[2 * it + 1] = ba;
            }
            if (pidx >= 0) hr[(size_t)(it + 1) * a.rmax + pidx] = s;

            // collinearity factors; freeze test ||s|| <= tol |pi^k|.
            // pi^k_{n+1} = (1 + alpha sigma_k) pi^k_n + c (pi^k_n - pi^k_{n-1})
            //            = (1 + c + alpha sigma_k) pi^k_n - c pi^k_{n-1},
            // c = alpha_n beta_{n-1} / alpha_{n-1}
            const double2 coup = cmul(alpha, ba_old);
            const double2 c1 = cadd(one, coup), ncoup = make_double2(-coup.x, -coup.y);
            int alive = 0;
#pragma unroll
            for (int m = 0; m < M; ++m) {
                // Stepped for every shift of a slot that still has a running
                // one, frozen or not: a frozen shift's pi^k is never read again
                // (its step count and the squares of its residual estimate
                // were kept when it froze), so no selects are spent keeping it.
                if (!__any(act[m])) continue;
                const double2 pn = cfma(cfma(alpha, sigma[m], c1), pc[m], cmul(ncoup, po[m]));
                const double pn2 = fma(pn.x, pn.x, pn.y * pn.y);
                const bool on = act[m];
                const bool done = on && snorm2 <= tol2 * pn2;
                po[m] = pc[m];
                pc[m] = pn;
                if (done) {
                    nkm[m] = it + 1;
                    res[m] = pn2;
                    fzs[m] = snorm2;
                }
                act[m] = on && !done;
                alive |= act[m] ? 1 : 0;
            }
            applied = it + 1;
            ba_old = ba;
            rho = rho_new;
            wave_lds_fence();  // p is in LDS for the next block product
            const bool any_alive = __any(alive);
            if (!any_alive || snorm2 == 0.0) { status = SGF_CONVERGED; break; }
            if (rho_new.x == 0.0 && rho_new.y == 0.0) { status = SGF_BREAKDOWN; break; }
            // a NaN or an infinity anywhere makes the sum non-finite
            if (!isfinite(rho_new.x + rho_new.y + snorm2)) { status = SGF_NONFINITE; break; }
            inv_rho = crcp(rho_new);
        }

#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int k = lane + 64 * m;
            if (k >= a.ns) continue;
            if (act[m]) {
                nkm[m] = applied;
                const double pn2 = fma(pc[m].x, pc[m].x, pc[m].y * pc[m].y);
                res[m] = applied > 0 ? sqrt(snorm2 / pn2) : 1.0;
            } else {
                res[m] = sqrt(fzs[m] / res[m]);  // ||s|| / |pi^k| at the freeze
            }
            a.nk[(size_t)slot * a.ns_pad + k] = nkm[m];
            if (a.resid) a.resid[c * a.ns + k] = res[m];
            if (a.shift_iters) a.shift_iters[c * a.ns + k] = nkm[m];
        }
        if (lane == 0) {
            *meta = ColMeta{(int32_t)c, iters, npa, status};
            a.iters[c] = iters;
            a.status[c] = status;
        }
        wave_lds_fence();  // vp reuse by the next column
    }
}

// ---------------------------------------------------------------------------
// Seed pass, S = I, four (or two) columns per wavefront.  Lane l serves
// column slot cs = l / 16 of a group of four consecutive work-queue entries
// and local atom a = l % 16 of that column's subspace (at most 16 atoms, 64
// orbitals): its four orbital rows of s, p and w stay in registers, and the
// subspace's blocks of H sit in LDS, shared by the columns of the group that
// have the same plan (the four orbitals of one atom).  The recurrence
// scalars of a column are formed by its 16 lanes only: per iteration a
// wavefront pays the complex divisions and the branch logic of the COCG
// recurrence once for four columns, and its sums are 16-lane row reductions
// (DPP row shifts, the row total handed to the row's lanes through LDS, so
// all of them hold the same bits).  Each lane steps the collinearity factors
// of ns/16 shifts of its own column, which bounds the four-column form at
// 128 shifts; up to 256, two columns per wavefront take 32 lanes each (two
// lanes per atom, two rows each) and ns/32 shifts per lane.  The columns of
// a group whose plans differ run one after another, each with its own plan's
// blocks in LDS.
// ---------------------------------------------------------------------------
constexpr int Q4_HS = 18;   // doubles per staged block: 16 values and 2 of padding (bank spread)
constexpr int Q4_VP = 17;   // double2 per (column slot, orbital) row of p: 16 atoms and 1 of padding

// Sum over the 16 lanes of each row, delivered to every lane of the row
// (fixed order, so the lanes of a row agree bit for bit).  rb: 4 rows x NV
// doubles of LDS scratch.
template <int NV>
__device__ __forceinline__ void row_sums16(double (&v)[NV], double *rb) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        double t = v[i];
        t += dpp_shr<0x111>(t);  // row_shr:1
        t += dpp_shr<0x112>(t);  // row_shr:2
        t += dpp_shr<0x114>(t);  // row_shr:4
        t += dpp_shr<0x118>(t);  // row_shr:8
        v[i] = t;
    }
    if ((lane & 15) == 15) {
#pragma unroll
        for (int i = 0; i < NV; ++i) rb[(lane >> 4) * 8 + i] = v[i];
    }
    wave_lds_fence();
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] = rb[(lane >> 4) * 8 + i];
    wave_lds_fence();  // rb may be written again by the next call
}

template <int M4, int BMAX>
__global__ __launch_bounds__(SEED_T) void k_seed_q4(SolveArgs a) {
    __shared__ __align__(16) double hs[16 * BMAX * Q4_HS];  // block b of local atom A's row in slot 16 b + A
    __shared__ int hcol[16 * BMAX];                         // local column atom of each slot's block
    __shared__ __align__(16) double2 vp[16 * Q4_VP];               // p: [slot][orbital] rows of 16 atoms
    __shared__ __align__(16) double rb[4 * 8];                     // row sums
    __shared__ __align__(16) double2 sg[16 * M4];                  // sigma_k = z_k - z_s
    const int lane = threadIdx.x;
    const int cs = lane >> 4, al = lane & 15;
    const double2 zs = a.z[a.seed];
    for (int k = lane; k < 16 * M4; k += 64) sg[k] = k < a.ns ? csub(a.z[k], zs) : make_double2(0.0, 0.0);
    const double tol2 = a.tol * a.tol;
    const double2 zero = make_double2(0.0, 0.0), one = make_double2(1.0, 0.0);
    const int64_t nbatch = a.batch_end - a.batch_begin;

    for (;;) {
        int64_t ticket = 0;
        if (lane == 0) ticket = (int64_t)atomicAdd(reinterpret_cast<unsigned long long *>(a.ticket), 1ull);
        ticket = __shfl(ticket, 0, 64);
        if (4 * ticket >= nbatch) break;
        // this lane's column: queue entry 4 ticket + cs of the batch
        const int64_t slot = 4 * ticket + cs;
        const bool have = slot < nbatch;
        int64_t c = -1, j = -1;
        int32_t pl = -1;
        int64_t a0 = 0, b0 = 0, p0 = 0;
        int n_loc = 0, nblk = 0, npa = 0, cl = 0;
        bool bad = !have;
        if (have) {
            c = a.order ? (int64_t)a.order[a.batch_begin + slot] : a.batch_begin + slot;
            bad = c < 0 || c >= a.n_cols;
        }
        if (!bad) {
            j = a.cols[c];
            pl = a.col_plan[c];
            bad = pl < 0 || pl >= a.n_plans || j < 0;
        }
        if (!bad) {
            a0 = a.atom_off[pl];
            n_loc = (int)(a.atom_off[pl + 1] - a0);
            b0 = a.blk_off[pl];
            nblk = (int)(a.blk_off[pl + 1] - b0);
            p0 = a.pa_off[pl];
            npa = (int)(a.pa_off[pl + 1] - p0);
            cl = a.center_loc[pl];
            bad = n_loc < 1 || n_loc > 16 || nblk > 16 * BMAX || npa < 1 || 4 * npa > a.rmax || cl < 0 ||
                  cl >= n_loc || a.loc_atom[a0 + cl] != (int32_t)(j >> 2);
        }
        if (!bad) {  // rows of more than BMAX blocks: this kernel cannot take the column
            int nb = 0;
            if (al < n_loc) nb = (al + 1 < n_loc ? a.lrow[a0 + al + 1] : nblk) - a.lrow[a0 + al];
            const uint64_t over = __ballot(nb > BMAX);
            bad = ((over >> (16 * cs)) & 0xffffull) != 0;
        }
        if (have && bad && al == 0) {
            a.meta[slot] = ColMeta{-1, 0, 0, SGF_BADCOLUMN};
            if (c >= 0 && c < a.n_cols) {
                a.iters[c] = 0;
                a.status[c] = SGF_BADCOLUMN;
            }
        }
        // column slots still to run (bit cs), one plan at a time
        uint32_t todo = 0;
        {
            const uint64_t ok = __ballot(!bad && al == 0);
#pragma unroll
            for (int g = 0; g < 4; ++g) todo |= ((ok >> (16 * g)) & 1ull) ? (1u << g) : 0u;
        }
        while (todo) {
            const int lead = __builtin_ctz(todo);
            const int32_t plead = __shfl(pl, 16 * lead, 64);
            const uint64_t same = __ballot(al == 0 && ((todo >> cs) & 1u) && pl == plead);
            uint32_t pass = 0;
#pragma unroll
            for (int g = 0; g < 4; ++g) pass |= ((same >> (16 * g)) & 1ull) ? (1u << g) : 0u;
            todo &= ~pass;
            const bool mine = (pass >> cs) & 1u;   // this lane's column runs in this pass
            // the plan's sizes, from the lead column's lanes (all equal within the pass)
            const int64_t pa0 = __shfl(a0, 16 * lead, 64), pb0 = __shfl(b0, 16 * lead, 64);
            const int64_t pp0 = __shfl(p0, 16 * lead, 64);
            const int pn_loc = __shfl(n_loc, 16 * lead, 64), pnblk = __shfl(nblk, 16 * lead, 64);
            const int pnpa = __shfl(npa, 16 * lead, 64), pcl = __shfl(cl, 16 * lead, 64);
            // stage the plan's blocks of H: block b of local atom A's row in
            // slot 16 b + A, a zero block (times atom 0's p) where the row has
            // b or fewer blocks or there is no atom A.  At step b the 16 lanes
            // of a column read 16 consecutive slots, whose stride of 9 x 16 B
            // starts them on 8 different 16-byte bank groups (the row-major
            // order put the rows' first blocks about 4 slots apart, on 2)
            wave_lds_fence();
            for (int i = lane; i < 16 * BMAX * 8; i += 64) {
                const int sl = i >> 3, h2 = i & 7, A = sl & 15, b = sl >> 4;
                double2 v = zero;
                int cb = 0;
                if (A < pn_loc) {
                    const int u0 = a.lrow[pa0 + A];
                    const int u1 = A + 1 < pn_loc ? a.lrow[pa0 + A + 1] : pnblk;
                    if (b < u1 - u0) {
                        const int32_t *lb = &a.lblk[2 * (pb0 + u0 + b)];
                        v = reinterpret_cast<const double2 *>(a.h + 16 * (int64_t)lb[1])[h2];
                        cb = lb[0];
                    }
                }
                reinterpret_cast<double2 *>(hs + sl * Q4_HS)[h2] = v;
                if (h2 == 0) hcol[sl] = cb;
            }
            // this lane's row
            const bool row = mine && al < pn_loc;
            int pq = -1;  // projection index of this lane's atom
            for (int q = 0; q < pnpa; ++q)
                if (row && a.pa_loc[pp0 + q] == al) pq = q;
            const int jo = (int)(j & 3);
            double2 *hab = a.hab + (size_t)slot * a.cap * 2;
            double2 *hr = a.hr + (size_t)slot * (a.cap + 1) * a.rmax;
            // start: x = 0, s_0 = p_0 = e_j
            double2 sv[4], pv[4];
#pragma unroll
            for (int o = 0; o < 4; ++o) {
                sv[o] = (row && al == pcl && o == jo) ? one : zero;
                pv[o] = sv[o];
                vp[(4 * cs + o) * Q4_VP + al] = pv[o];
                if (mine && pq >= 0) hr[4 * pq + o] = sv[o];
            }
            wave_lds_fence();

            double2 pc[M4], po[M4];
            uint32_t act = 0;
#pragma unroll
            for (int m = 0; m < M4; ++m) {
                pc[m] = po[m] = one;
                if (mine && al + 16 * m < a.ns) act |= 1u << m;
            }
            double2 rho = one, inv_rho = one, ba_old = zero;
            int status = SGF_MAXITER, iters = 0, applied = 0;
            bool running = mine;
            double snorm2 = 1.0;
            const int max_iter = a.max_iter > 0 ? a.max_iter : 40 * pn_loc;  // 10 per local orbital

            const double *hsl = hs + al * Q4_HS;       // this lane's slots: hsl + 16 b Q4_HS
            const double2 *vpc = vp + 4 * cs * Q4_VP;  // this lane's column of p

            for (int it = 0; it < max_iter; ++it) {
                // w = z_s p - H p on this lane's four rows
                double ax[4] = {0.0, 0.0, 0.0, 0.0}, ay[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int b = 0; b < BMAX; ++b) {
                    const double2 *hb = reinterpret_cast<const double2 *>(hsl + 16 * Q4_HS * b);
                    const int bcol = hcol[16 * b + al];
                    double2 pb[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) pb[q] = vpc[q * Q4_VP + bcol];
#pragma unroll
                    for (int o = 0; o < 4; ++o) {
                        const double2 h01 = hb[2 * o], h23 = hb[2 * o + 1];
                        ax[o] = fma(h01.x, pb[0].x, ax[o]);
                        ay[o] = fma(h01.x, pb[0].y, ay[o]);
                        ax[o] = fma(h01.y, pb[1].x, ax[o]);
                        ay[o] = fma(h01.y, pb[1].y, ay[o]);
                        ax[o] = fma(h23.x, pb[2].x, ax[o]);
                        ay[o] = fma(h23.x, pb[2].y, ay[o]);
                        ax[o] = fma(h23.y, pb[3].x, ax[o]);
                        ay[o] = fma(h23.y, pb[3].y, ay[o]);
                    }
                }
                double2 wv[4];
                double sm[2] = {0.0, 0.0};
#pragma unroll
                for (int o = 0; o < 4; ++o) {
                    wv[o] = make_double2(zs.x * pv[o].x - zs.y * pv[o].y - ax[o],
                                         zs.x * pv[o].y + zs.y * pv[o].x - ay[o]);
                    sm[0] = fma(pv[o].x, wv[o].x, fma(-pv[o].y, wv[o].y, sm[0]));
                    sm[1] = fma(pv[o].x, wv[o].y, fma(pv[o].y, wv[o].x, sm[1]));
                }
                row_sums16<2>(sm, rb);
                const double2 mu = make_double2(sm[0], sm[1]);
                if (running) {
                    iters = it + 1;
                    if (!cfinite(mu)) { status = SGF_NONFINITE; running = false; }
                    else if (mu.x == 0.0 && mu.y == 0.0) { status = SGF_BREAKDOWN; running = false; }
                }
                const double2 alpha = cmul(rho, crcp(mu));
                const double2 ia = cmul(mu, inv_rho);  // 1/alpha
                double sr[3] = {0.0, 0.0, 0.0};
#pragma unroll
                for (int o = 0; o < 4; ++o) {
                    sv[o] = csub(sv[o], cmul(alpha, wv[o]));
                    sr[0] = fma(sv[o].x, sv[o].x, fma(-sv[o].y, sv[o].y, sr[0]));
                    sr[1] = fma(2.0 * sv[o].x, sv[o].y, sr[1]);
                    sr[2] = fma(sv[o].x, sv[o].x, fma(sv[o].y, sv[o].y, sr[2]));
                }
                row_sums16<3>(sr, rb);
                const double2 rho_new = make_double2(sr[0], sr[1]);
                const double2 beta = cmul(rho_new, inv_rho);
                const double2 ba = cmul(beta, ia);  // beta_n / alpha_n
#pragma unroll
                for (int o = 0; o < 4; ++o) {
                    pv[o] = cfma(beta, pv[o], sv[o]);
                    vp[(4 * cs + o) * Q4_VP + al] = pv[o];
                }
                if (running) {
                    snorm2 = sr[2];
                    // history: 1/alpha_n, beta_n/alpha_n, r_{n+1} on P
                    if (al == 0) {
                        hab[2 * it] = ia;
                        hab[2 * it + 1] = ba;
                    }
                    if (pq >= 0) {
#pragma unroll
                        for (int o = 0; o < 4; ++o) hr[(size_t)(it + 1) * a.rmax + 4 * pq + o] = sv[o];
                    }
                    // collinearity factors and the freeze test ||s|| <= tol |pi^k|;
                    // a slot whose shifts have all frozen, in every running
                    // column of the wavefront, is not stepped (its factors
                    // are never read again)
                    const double2 coup = cmul(alpha, ba_old);
                    const double2 c1 = cadd(one, coup), ncoup = make_double2(-coup.x, -coup.y);
#pragma unroll
                    for (int m = 0; m < M4; ++m) {
                        if (!__any((act >> m) & 1u)) continue;
                        const double2 pn = cfma(cfma(alpha, sg[al + 16 * m], c1), pc[m], cmul(ncoup, po[m]));
                        const double pn2 = fma(pn.x, pn.x, pn.y * pn.y);
                        po[m] = pc[m];
                        pc[m] = pn;
                        if (((act >> m) & 1u) && snorm2 <= tol2 * pn2) {
                            // the estimate ||s|| / |pi^k| is formed after the
                            // column from the two squares kept here
                            act &= ~(1u << m);
                            const int k = al + 16 * m;
                            a.nk[(size_t)slot * a.ns_pad + k] = it + 1;
                            if (a.resid) {
                                a.resid[c * a.ns + k] = pn2;
                                a.fz[(size_t)slot * a.ns_pad + k] = snorm2;
                            }
                            if (a.shift_iters) a.shift_iters[c * a.ns + k] = it + 1;
                        }
                    }
                    applied = it + 1;
                    ba_old = ba;
                    rho = rho_new;
                    // the column stops when none of its 16 lanes holds an active shift
                    const uint64_t alive = __ballot(act != 0);
                    const bool any_alive = ((alive >> (16 * cs)) & 0xffffull) != 0;
                    if (!any_alive || snorm2 == 0.0) { status = SGF_CONVERGED; running = false; }
                    else if (rho_new.x == 0.0 && rho_new.y == 0.0) { status = SGF_BREAKDOWN; running = false; }
                    else if (!isfinite(rho_new.x + rho_new.y + snorm2)) { status = SGF_NONFINITE; running = false; }
                    else inv_rho = crcp(rho_new);
                }
                wave_lds_fence();  // p is in LDS for the next block product
                if (!__any(running)) break;
            }
            if (mine) {
#pragma unroll
                for (int m = 0; m < M4; ++m) {
                    const int k = al + 16 * m;
                    if (k >= a.ns) continue;
                    if (!((act >> m) & 1u)) {  // frozen: ||s|| / |pi^k| at its freeze
                        if (a.resid)
                            a.resid[c * a.ns + k] = sqrt(a.fz[(size_t)slot * a.ns_pad + k] / a.resid[c * a.ns + k]);
                        continue;
                    }
                    const double pn2 = fma(pc[m].x, pc[m].x, pc[m].y * pc[m].y);
                    const double res = applied > 0 ? sqrt(snorm2 / pn2) : 1.0;
                    a.nk[(size_t)slot * a.ns_pad + k] = applied;
                    if (a.resid) a.resid[c * a.ns + k] = res;
                    if (a.shift_iters) a.shift_iters[c * a.ns + k] = applied;
                }
                if (al == 0) {
                    a.meta[slot] = ColMeta{(int32_t)c, iters, pnpa, status};
                    a.iters[c] = iters;
                    a.status[c] = status;
                }
            }
        }
        wave_lds_fence();  // hs and vp are reused by the next group
    }
}

// Sums over the lanes of each column (16 or 32 consecutive lanes), delivered
// to every lane of the column in a fixed order, so that they all hold the
// same bits: DPP row shifts sum each 16-lane row, the row totals go through
// LDS, and a 32-lane column adds its two row totals, lower row first.
// rb: 4 rows x 8 doubles of LDS scratch.
template <int NV, int LPC>
__device__ __forceinline__ void column_sums(double (&v)[NV], double *rb) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        double t = v[i];
        t += dpp_shr<0x111>(t);  // row_shr:1
        t += dpp_shr<0x112>(t);  // row_shr:2
        t += dpp_shr<0x114>(t);  // row_shr:4
        t += dpp_shr<0x118>(t);  // row_shr:8
        v[i] = t;
    }
    if ((lane & 15) == 15) {
#pragma unroll
        for (int i = 0; i < NV; ++i) rb[(lane >> 4) * 8 + i] = v[i];
    }
    wave_lds_fence();
    if (LPC == 16) {
#pragma unroll
        for (int i = 0; i < NV; ++i) v[i] = rb[(lane >> 4) * 8 + i];
    } else {
        const int r0 = (lane >> 5) * 2;
#pragma unroll
        for (int i = 0; i < NV; ++i) v[i] = rb[r0 * 8 + i] + rb[(r0 + 1) * 8 + i];
    }
    wave_lds_fence();  // rb may be written again by the next call
}

// The seed pass with CPW columns of one plan per wavefront (CPW = 4: sixteen
// lanes per column, a lane per local atom and its four orbital rows; CPW = 2:
// thirty-two lanes per column, two lanes per local atom, each with two of
// its rows).  A lane steps the collinearity factors of M4 shifts of its own
// column: shift k = l + LPC m for its lane l of the column.  Only the
// two-column kernel is built from this body: k_seed_q4 keeps its own, since
// compiling the four-column case from it reorders the compiler's floating
// point and changes the rounding (and the iteration count) of columns that
// pass close to a breakdown.
template <int CPW, int M4, int BMAX>
__device__ __forceinline__ void seed_columns(const SolveArgs &a) {
    constexpr int LPC = 64 / CPW;   // lanes per column
    constexpr int RPL = 64 / LPC;   // orbital rows per lane (4 or 2)
    static_assert(CPW == 4 || CPW == 2, "two or four columns per wavefront");
    __shared__ __align__(16) double hs[16 * BMAX * Q4_HS];  // block b of local atom A's row in slot 16 b + A
    __shared__ int hcol[16 * BMAX];                         // local column atom of each slot's block
    __shared__ __align__(16) double2 vp[4 * CPW * Q4_VP];   // p: [column slot][orbital] rows of 16 atoms
    __shared__ __align__(16) double rb[4 * 8];              // row sums
    __shared__ __align__(16) double2 sg[LPC * M4];          // sigma_k = z_k - z_s
    const int lane = threadIdx.x;
    const int cs = lane / LPC, l = lane % LPC;  // column slot, lane within the column
    const int al = l & 15, o0 = (l >> 4) * RPL;  // local atom, first of this lane's rows
    constexpr uint64_t CMASK = LPC == 64 ? ~0ull : ((1ull << LPC) - 1);
    const double2 zs = a.z[a.seed];
    for (int k = lane; k < LPC * M4; k += 64) sg[k] = k < a.ns ? csub(a.z[k], zs) : make_double2(0.0, 0.0);
    const double tol2 = a.tol * a.tol;
    const double2 zero = make_double2(0.0, 0.0), one = make_double2(1.0, 0.0);
    const int64_t nbatch = a.batch_end - a.batch_begin;

    for (;;) {
        int64_t ticket = 0;
        if (lane == 0) ticket = (int64_t)atomicAdd(reinterpret_cast<unsigned long long *>(a.ticket), 1ull);
        ticket = __shfl(ticket, 0, 64);
        if (CPW * ticket >= nbatch) break;
        // this lane's column: queue entry CPW ticket + cs of the batch
        const int64_t slot = CPW * ticket + cs;
        const bool have = slot < nbatch;
        int64_t c = -1, j = -1;
        int32_t pl = -1;
        int64_t a0 = 0, b0 = 0, p0 = 0;
        int n_loc = 0, nblk = 0, npa = 0, cl = 0;
        bool bad = !have;
        if (have) {
            c = a.order ? (int64_t)a.order[a.batch_begin + slot] : a.batch_begin + slot;
            bad = c < 0 || c >= a.n_cols;
        }
        if (!bad) {
            j = a.cols[c];
            pl = a.col_plan[c];
            bad = pl < 0 || pl >= a.n_plans || j < 0;
        }
        if (!bad) {
            a0 = a.atom_off[pl];
            n_loc = (int)(a.atom_off[pl + 1] - a0);
            b0 = a.blk_off[pl];
            nblk = (int)(a.blk_off[pl + 1] - b0);
            p0 = a.pa_off[pl];
            npa = (int)(a.pa_off[pl + 1] - p0);
            cl = a.center_loc[pl];
            bad = n_loc < 1 || n_loc > 16 || nblk > 16 * BMAX || npa < 1 || 4 * npa > a.rmax || cl < 0 ||
                  cl >= n_loc || a.loc_atom[a0 + cl] != (int32_t)(j >> 2);
        }
        if (!bad) {  // rows of more than BMAX blocks: this kernel cannot take the column
            int nb = 0;
            if (al < n_loc) nb = (al + 1 < n_loc ? a.lrow[a0 + al + 1] : nblk) - a.lrow[a0 + al];
            const uint64_t over = __ballot(nb > BMAX);
            bad = ((over >> (LPC * cs)) & CMASK) != 0;
        }
        if (have && bad && l == 0) {
            a.meta[slot] = ColMeta{-1, 0, 0, SGF_BADCOLUMN};
            if (c >= 0 && c < a.n_cols) {
                a.iters[c] = 0;
                a.status[c] = SGF_BADCOLUMN;
            }
        }
        // column slots still to run (bit cs), one plan at a time
        uint32_t todo = 0;
        {
            const uint64_t ok = __ballot(!bad && l == 0);
#pragma unroll
            for (int g = 0; g < CPW; ++g) todo |= ((ok >> (LPC * g)) & 1ull) ? (1u << g) : 0u;
        }
        while (todo) {
            const int lead = __builtin_ctz(todo);
            const int32_t plead = __shfl(pl, LPC * lead, 64);
            const uint64_t same = __ballot(l == 0 && ((todo >> cs) & 1u) && pl == plead);
            uint32_t pass = 0;
#pragma unroll
            for (int g = 0; g < CPW; ++g) pass |= ((same >> (LPC * g)) & 1ull) ? (1u << g) : 0u;
            todo &= ~pass;
            const bool mine = (pass >> cs) & 1u;   // this lane's column runs in this pass
            // the plan's sizes, from the lead column's lanes (all equal within the pass)
            const int64_t pa0 = __shfl(a0, LPC * lead, 64), pb0 = __shfl(b0, LPC * lead, 64);
            const int64_t pp0 = __shfl(p0, LPC * lead, 64);
            const int pn_loc = __shfl(n_loc, LPC * lead, 64), pnblk = __shfl(nblk, LPC * lead, 64);
            const int pnpa = __shfl(npa, LPC * lead, 64), pcl = __shfl(cl, LPC * lead, 64);
            // stage the plan's blocks of H: block b of local atom A's row in
            // slot 16 b + A, a zero block (times atom 0's p) where the row has
            // b or fewer blocks or there is no atom A.  At step b the 16 lanes
            // of a column read 16 consecutive slots, whose stride of 9 x 16 B
            // starts them on 8 different 16-byte bank groups (the row-major
            // order put the rows' first blocks about 4 slots apart, on 2)
            wave_lds_fence();
            for (int i = lane; i < 16 * BMAX * 8; i += 64) {
                const int sl = i >> 3, h2 = i & 7, A = sl & 15, b = sl >> 4;
                double2 v = zero;
                int cb = 0;
                if (A < pn_loc) {
                    const int u0 = a.lrow[pa0 + A];
                    const int u1 = A + 1 < pn_loc ? a.lrow[pa0 + A + 1] : pnblk;
                    if (b < u1 - u0) {
                        const int32_t *lb = &a.lblk[2 * (pb0 + u0 + b)];
                        v = reinterpret_cast<const double2 *>(a.h + 16 * (int64_t)lb[1])[h2];
                        cb = lb[0];
                    }
                }
                reinterpret_cast<double2 *>(hs + sl * Q4_HS)[h2] = v;
                if (h2 == 0) hcol[sl] = cb;
            }
            // this lane's rows
            const bool row = mine && al < pn_loc;
            int pq = -1;  // projection index of this lane's atom
            for (int q = 0; q < pnpa; ++q)
                if (row && a.pa_loc[pp0 + q] == al) pq = q;
            const int jo = (int)(j & 3);
            double2 *hab = a.hab + (size_t)slot * a.cap * 2;
            double2 *hr = a.hr + (size_t)slot * (a.cap + 1) * a.rmax;
            // start: x = 0, s_0 = p_0 = e_j
            double2 sv[RPL], pv[RPL];
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
                const int o = o0 + r;
                sv[r] = (row && al == pcl && o == jo) ? one : zero;
                pv[r] = sv[r];
                vp[(4 * cs + o) * Q4_VP + al] = pv[r];
                if (mine && pq >= 0) hr[4 * pq + o] = sv[r];
            }
            wave_lds_fence();

            double2 pc[M4], po[M4];
            uint32_t act = 0;
#pragma unroll
            for (int m = 0; m < M4; ++m) {
                pc[m] = po[m] = one;
                if (mine && l + LPC * m < a.ns) act |= 1u << m;
            }
            double2 rho = one, inv_rho = one, ba_old = zero;
            int status = SGF_MAXITER, iters = 0, applied = 0;
            bool running = mine;
            double snorm2 = 1.0;
            const int max_iter = a.max_iter > 0 ? a.max_iter : 40 * pn_loc;  // 10 per local orbital

            const double *hsl = hs + al * Q4_HS + 4 * o0;  // this lane's rows of its slots (slot stride 16 Q4_HS)
            const double2 *vpc = vp + 4 * cs * Q4_VP;      // this lane's column of p

            for (int it = 0; it < max_iter; ++it) {
                // w = z_s p - H p on this lane's rows
                double ax[RPL], ay[RPL];
#pragma unroll
                for (int r = 0; r < RPL; ++r) ax[r] = ay[r] = 0.0;
#pragma unroll
                for (int b = 0; b < BMAX; ++b) {
                    const double2 *hb = reinterpret_cast<const double2 *>(hsl + 16 * Q4_HS * b);
                    const int bcol = hcol[16 * b + al];
                    double2 pb[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) pb[q] = vpc[q * Q4_VP + bcol];
#pragma unroll
                    for (int r = 0; r < RPL; ++r) {
                        const double2 h01 = hb[2 * r], h23 = hb[2 * r + 1];
                        ax[r] = fma(h01.x, pb[0].x, ax[r]);
                        ay[r] = fma(h01.x, pb[0].y, ay[r]);
                        ax[r] = fma(h01.y, pb[1].x, ax[r]);
                        ay[r] = fma(h01.y, pb[1].y, ay[r]);
                        ax[r] = fma(h23.x, pb[2].x, ax[r]);
                        ay[r] = fma(h23.x, pb[2].y, ay[r]);
                        ax[r] = fma(h23.y, pb[3].x, ax[r]);
                        ay[r] = fma(h23.y, pb[3].y, ay[r]);
                    }
                }
                double2 wv[RPL];
                double sm[2] = {0.0, 0.0};
#pragma unroll
                for (int r = 0; r < RPL; ++r) {
                    wv[r] = make_double2(zs.x * pv[r].x - zs.y * pv[r].y - ax[r],
                                         zs.x * pv[r].y + zs.y * pv[r].x - ay[r]);
                    sm[0] = fma(pv[r].x, wv[r].x, fma(-pv[r].y, wv[r].y, sm[0]));
                    sm[1] = fma(pv[r].x, wv[r].y, fma(pv[r].y, wv[r].x, sm[1]));
                }
                column_sums<2, LPC>(sm, rb);
                const double2 mu = make_double2(sm[0], sm[1]);
                if (running) {
                    iters = it + 1;
                    if (!cfinite(mu)) { status = SGF_NONFINITE; running = false; }
                    else if (mu.x == 0.0 && mu.y == 0.0) { status = SGF_BREAKDOWN; running = false; }
                }
                const double2 alpha = cmul(rho, crcp(mu));
                const double2 ia = cmul(mu, inv_rho);  // 1/alpha
                double sr[3] = {0.0, 0.0, 0.0};
#pragma unroll
                for (int r = 0; r < RPL; ++r) {
                    sv[r] = csub(sv[r], cmul(alpha, wv[r]));
                    sr[0] = fma(sv[r].x, sv[r].x, fma(-sv[r].y, sv[r].y, sr[0]));
                    sr[1] = fma(2.0 * sv[r].x, sv[r].y, sr[1]);
                    sr[2] = fma(sv[r].x, sv[r].x, fma(sv[r].y, sv[r].y, sr[2]));
                }
                column_sums<3, LPC>(sr, rb);
                const double2 rho_new = make_double2(sr[0], sr[1]);
                const double2 beta = cmul(rho_new, inv_rho);
                const double2 ba = cmul(beta, ia);  // beta_n / alpha_n
#pragma unroll
                for (int r = 0; r < RPL; ++r) {
                    pv[r] = cfma(beta, pv[r], sv[r]);
                    vp[(4 * cs + o0 + r) * Q4_VP + al] = pv[r];
                }
                if (running) {
                    snorm2 = sr[2];
                    // history: 1/alpha_n, beta_n/alpha_n, r_{n+1} on P
                    if (l == 0) {
                        hab[2 * it] = ia;
                        hab[2 * it + 1] = ba;
                    }
                    if (pq >= 0) {
#pragma unroll
                        for (int r = 0; r < RPL; ++r) hr[(size_t)(it + 1) * a.rmax + 4 * pq + o0 + r] = sv[r];
                    }
                    // collinearity factors and the freeze test ||s|| <= tol |pi^k|;
                    // a slot whose shifts have all frozen, in every running
                    // column of the wavefront, is not stepped (its factors
                    // are never read again)
                    const double2 coup = cmul(alpha, ba_old);
                    const double2 c1 = cadd(one, coup), ncoup = make_double2(-coup.x, -coup.y);
#pragma unroll
                    for (int m = 0; m < M4; ++m) {
                        if (!__any((act >> m) & 1u)) continue;
                        const double2 pn = cfma(cfma(alpha, sg[l + LPC * m], c1), pc[m], cmul(ncoup, po[m]));
                        const double pn2 = fma(pn.x, pn.x, pn.y * pn.y);
                        po[m] = pc[m];
                        pc[m] = pn;
                        if (((act >> m) & 1u) && snorm2 <= tol2 * pn2) {
                            // the estimate ||s|| / |pi^k| is formed after the
                            // column from the two squares kept here
                            act &= ~(1u << m);
                            const int k = l + LPC * m;
                            a.nk[(size_t)slot * a.ns_pad + k] = it + 1;
                            if (a.resid) {
                                a.resid[c * a.ns + k] = pn2;
                                a.fz[(size_t)slot * a.ns_pad + k] = snorm2;
                            }
                            if (a.shift_iters) a.shift_iters[c * a.ns + k] = it + 1;
                        }
                    }
                    applied = it + 1;
                    ba_old = ba;
                    rho = rho_new;
                    // the column stops when none of its lanes holds an active shift
                    const uint64_t alive = __ballot(act != 0);
                    const bool any_alive = ((alive >> (LPC * cs)) & CMASK) != 0;
                    if (!any_alive || snorm2 == 0.0) { status = SGF_CONVERGED; running = false; }
                    else if (rho_new.x == 0.0 && rho_new.y == 0.0) { status = SGF_BREAKDOWN; running = false; }
                    else if (!isfinite(rho_new.x + rho_new.y + snorm2)) { status = SGF_NONFINITE; running = false; }
                    else inv_rho = crcp(rho_new);
                }
                wave_lds_fence();  // p is in LDS for the next block product
                if (!__any(running)) break;
            }
            if (mine) {
#pragma unroll
                for (int m = 0; m < M4; ++m) {
                    const int k = l + LPC * m;
                    if (k >= a.ns) continue;
                    if (!((act >> m) & 1u)) {  // frozen: ||s|| / |pi^k| at its freeze
                        if (a.resid)
                            a.resid[c * a.ns + k] = sqrt(a.fz[(size_t)slot * a.ns_pad + k] / a.resid[c * a.ns + k]);
                        continue;
                    }
                    const double pn2 = fma(pc[m].x, pc[m].x, pc[m].y * pc[m].y);
                    const double res = applied > 0 ? sqrt(snorm2 / pn2) : 1.0;
                    a.nk[(size_t)slot * a.ns_pad + k] = applied;
                    if (a.resid) a.resid[c * a.ns + k] = res;
                    if (a.shift_iters) a.shift_iters[c * a.ns + k] = applied;
                }
                if (l == 0) {
                    a.meta[slot] = ColMeta{(int32_t)c, iters, pnpa, status};
                    a.iters[c] = iters;
                    a.status[c] = status;
                }
            }
        }
        wave_lds_fence();  // hs and vp are reused by the next group
    }
}

// Two columns of a plan per wavefront: up to 256 shifts (M2 = ns_pad / 32).
template <int M2, int BMAX>
__global__ __launch_bounds__(SEED_T) void k_seed_q2(SolveArgs a) {
    seed_columns<2, M2, BMAX>(a);
}

// ---------------------------------------------------------------------------
// Seed pass for S != I.  COCG on A = S^{-1}(z_s S - H) with the S-bilinear
// form [u, v] = u^T S v (A is symmetric in it since H and S are real
// symmetric): s is the true-space residual, r = S^{-1} s, q = S p and
// w = (z_s S - H) p = z_s q - H p, so mu = p^T w and rho = r^T s.  The inverse
// of the local overlap S_L is formed once per column in LDS, in the packed
// lower triangle of a symmetric matrix, by the sweep operator (Gauss-Jordan
// elimination that keeps the matrix symmetric; S_L is positive definite, so
// no pivoting), and applied as a dense product each iteration, four
// independent partial sums per row so that the LDS reads overlap.  Lane l owns rows l
// and l + 64; with BMAX > 0 their blocks of H (at most BMAX per row) and
// local columns stay in registers for the whole column, with BMAX = 0 (any
// number of blocks per row) they are read from the local operator in global
// memory every iteration.  The recorded history holds r on P: the
// shifted iterates are combinations of the r_n.
// ---------------------------------------------------------------------------
// Row stride (doubles) of the dense local overlap inverse: the smallest
// 32k + 1 >= nl.  Lane i reading row i then starts on bank pair 2i (mod 64).
__host__ __device__ inline int sinv_ld(int nl) { return 32 * ((nl + 30) / 32) + 1; }
// Packed lower triangle of a symmetric nl x nl matrix: entry (i, j), j <= i,
// at tri(i) + j, tri(i) = i (i + 1) / 2; (j, i) shares it.
__host__ __device__ inline int tri(int i) { return i * (i + 1) / 2; }

template <int M, int BMAX, bool PACKED>
__global__ __launch_bounds__(SEED_T) void k_seed_gen(SolveArgs a) {
    extern __shared__ double4 lds4[];
    char *lds = reinterpret_cast<char *>(lds4);
    double2 *vp = reinterpret_cast<double2 *>(lds + a.off_p);
    double2 *vs = reinterpret_cast<double2 *>(lds + a.off_s);
    double2 *vw = reinterpret_cast<double2 *>(lds + a.off_w);
    double2 *vq = reinterpret_cast<double2 *>(lds + a.off_q);
    double2 *vr = reinterpret_cast<double2 *>(lds + a.off_r);
    double *Si = reinterpret_cast<double *>(lds + a.off_sinv);  // packed lower triangle, tri(nl) doubles
    const int lane = threadIdx.x;
    const double2 zs = a.z[a.seed];
    double2 sigma[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int k = lane + 64 * m;
        sigma[m] = k < a.ns ? csub(a.z[k], zs) : make_double2(0.0, 0.0);
    }
    const double tol2 = a.tol * a.tol;
    const double2 zero = make_double2(0.0, 0.0);

    for (;;) {
        int64_t ticket = 0;
        if (lane == 0) ticket = (int64_t)atomicAdd(reinterpret_cast<unsigned long long *>(a.ticket), 1ull);
        ticket = __shfl(ticket, 0, 64);
        if (ticket >= a.batch_end - a.batch_begin) break;
        const int64_t slot = ticket;
        ticket += a.batch_begin;
        const int64_t c = a.order ? (int64_t)a.order[ticket] : ticket;
        ColMeta *meta = &a.meta[slot];
        if (c < 0 || c >= a.n_cols) {
            if (lane == 0) *meta = ColMeta{-1, 0, 0, SGF_BADCOLUMN};
            continue;
        }
        const int64_t j = a.cols[c];
        const int32_t pl = a.col_plan[c];
        bool bad = pl < 0 || pl >= a.n_plans || j < 0;
        int64_t a0 = 0, b0 = 0, p0 = 0;
        int n_loc = 0, nblk = 0, npa = 0, cl = 0;
        if (!bad) {
            a0 = a.atom_off[pl];
            n_loc = (int)(a.atom_off[pl + 1] - a0);
            b0 = a.blk_off[pl];
            nblk = (int)(a.blk_off[pl + 1] - b0);
            p0 = a.pa_off[pl];
            npa = (int)(a.pa_off[pl + 1] - p0);
            cl = a.center_loc[pl];
            bad = n_loc < 1 || n_loc > 32 || n_loc > a.max_loc_atoms || npa < 1 || 4 * npa > a.rmax || cl < 0 ||
                  cl >= n_loc || a.loc_atom[a0 + cl] != (int32_t)(j >> 2);
        }
        // a launch for one size class leaves the other columns to the other
        // launch; unsolvable columns are reported by the first
        if (a.loc_hi > 0 && (bad ? a.loc_lo > 1 : (n_loc < a.loc_lo || n_loc > a.loc_hi))) continue;
        if (bad) {
            if (lane == 0) {
                *meta = ColMeta{-1, 0, 0, SGF_BADCOLUMN};
                a.iters[c] = 0;
                a.status[c] = SGF_BADCOLUMN;
            }
            continue;
        }
        const int nl = 4 * n_loc;
        // rows lane and lane + 64 of H: their blocks and local columns;
        // absent blocks hold zeros and point at atom 0
        constexpr int NBR = BMAX > 0 ? BMAX : 1;
        int bcol[2][NBR];
        double hrow[2][NBR][4];
        bool wide = false;
#pragma unroll
        for (int r = 0; r < (BMAX > 0 ? 2 : 0); ++r) {
            const int i = lane + 64 * r;
            const int A = i >> 2, o = i & 3;
            int t0 = 0, nb = 0;
            if (i < nl) {
                t0 = a.lrow[a0 + A];
                nb = (A + 1 < n_loc ? a.lrow[a0 + A + 1] : nblk) - t0;
            }
            wide = wide || nb > BMAX;
#pragma unroll
            for (int b = 0; b < NBR; ++b) {
                bcol[r][b] = 0;
                hrow[r][b][0] = hrow[r][b][1] = hrow[r][b][2] = hrow[r][b][3] = 0.0;
                if (b < nb) {
                    const int32_t *lb = &a.lblk[2 * (b0 + t0 + b)];
                    bcol[r][b] = lb[0];
                    const double *hb = &a.h[16 * (int64_t)lb[1] + 4 * o];
#pragma unroll
                    for (int q = 0; q < 4; ++q) hrow[r][b][q] = hb[q];
                }
            }
        }
        if (__any(wide)) {
            if (lane == 0) {
                *meta = ColMeta{-1, 0, 0, SGF_BADCOLUMN};
                a.iters[c] = 0;
                a.status[c] = SGF_BADCOLUMN;
            }
            continue;
        }
        const int jl = 4 * cl + (int)(j & 3);
        const int nprow = 4 * npa;
        const int prow = lane < nprow ? 4 * a.pa_loc[p0 + (lane >> 2)] + (lane & 3) : 0;
        double2 *hab = a.hab + (size_t)slot * a.cap * 2;
        double2 *hr = a.hr + (size_t)slot * (a.cap + 1) * a.rmax;

        if constexpr (!PACKED) {
            // row stride of the dense inverse: 32k + 1 doubles, so that the lanes
            // of a wavefront, each on its own row, read consecutive LDS banks
            const int ld = sinv_ld(nl);
            // dense S_L, then its inverse in place
            for (int e = lane; e < nl * ld; e += SEED_T) Si[e] = 0.0;
            wave_lds_fence();
            for (int A = lane; A < n_loc; A += SEED_T) {
                const int t0 = a.lrow[a0 + A], t1 = A + 1 < n_loc ? a.lrow[a0 + A + 1] : nblk;
                for (int t = t0; t < t1; ++t) {
                    const int B = a.lblk[2 * (b0 + t)];
                    const double *sb = &a.s[16 * (int64_t)a.lblk[2 * (b0 + t) + 1]];
                    for (int o = 0; o < 4; ++o)
                        for (int q = 0; q < 4; ++q) Si[(4 * A + o) * ld + 4 * B + q] = sb[4 * o + q];
                }
            }
            wave_lds_fence();
            for (int kk = 0; kk < nl; ++kk) {
                const double piv = 1.0 / Si[kk * ld + kk];
                wave_lds_fence();
                for (int jj = lane; jj < nl; jj += SEED_T) Si[kk * ld + jj] = (jj == kk) ? piv : Si[kk * ld + jj] * piv;
                wave_lds_fence();
                // rows lane and lane + 64 (not the pivot row): a_ij -= a_ik a_kj for
                // every j, then a_ik = -a_ik piv; the two rows share each read of
                // the pivot row (nl is a multiple of 4)
                {
                    const double *pr = &Si[kk * ld];
                    const int i0 = lane, i1 = lane + 64;
                    const bool e0 = i0 < nl && i0 != kk, e1 = i1 < nl && i1 != kk;
                    double *w0 = &Si[(e0 ? i0 : kk) * ld], *w1 = &Si[(e1 ? i1 : kk) * ld];
                    const double f0 = e0 ? w0[kk] : 0.0, f1 = e1 ? w1[kk] : 0.0;
                    if (nl > 64) {
                        if (e0 || e1) {
                            for (int jj = 0; jj < nl; jj += 4) {
#pragma unroll
                                for (int u = 0; u < 4; ++u) {
                                    const double pv = pr[jj + u];
                                    if (e0) w0[jj + u] = fma(-f0, pv, w0[jj + u]);
                                    if (e1) w1[jj + u] = fma(-f1, pv, w1[jj + u]);
                                }
                            }
                        }
                    } else if (e0) {
                        for (int jj = 0; jj < nl; jj += 4) {
#pragma unroll
                            for (int u = 0; u < 4; ++u) w0[jj + u] = fma(-f0, pr[jj + u], w0[jj + u]);
                        }
                    }
                    if (e0) w0[kk] = -f0 * piv;
                    if (e1) w1[kk] = -f1 * piv;
                }
                wave_lds_fence();
            }
        } else {
            // S_L packed, then the sweep in place
            for (int e = lane; e < tri(nl); e += SEED_T) Si[e] = 0.0;
            wave_lds_fence();
            for (int A = lane; A < n_loc; A += SEED_T) {
                const int t0 = a.lrow[a0 + A], t1 = A + 1 < n_loc ? a.lrow[a0 + A + 1] : nblk;
                for (int t = t0; t < t1; ++t) {
                    const int B = a.lblk[2 * (b0 + t)];
                    if (B > A) continue;  // the upper blocks mirror the lower ones
                    const double *sb = &a.s[16 * (int64_t)a.lblk[2 * (b0 + t) + 1]];
                    for (int o = 0; o < 4; ++o)
                        for (int q = 0; q < 4; ++q)
                            if (4 * B + q <= 4 * A + o) Si[tri(4 * A + o) + 4 * B + q] = sb[4 * o + q];
                }
            }
            wave_lds_fence();
            // Sweep on pivot k, v = column k, d = v_k: a_ij -= v_i v_j / d for
            // i, j != k, a_ik = v_i / d for i != k, a_kk = -1 / d.  After the last
            // pivot the triangle holds -S_L^{-1}.  v lives in vw, which is free
            // until the iteration starts.
            {
                double *v = reinterpret_cast<double *>(vw);
                const int i0 = lane, i1 = lane + 64;
                double *row0 = &Si[tri(i0 < nl ? i0 : 0)], *row1 = &Si[tri(i1 < nl ? i1 : 0)];
                for (int kk = 0; kk < nl; ++kk) {
                    for (int i = lane; i < nl; i += SEED_T) v[i] = i >= kk ? Si[tri(i) + kk] : Si[tri(kk) + i];
                    wave_lds_fence();
                    const double id = 1.0 / v[kk];
                    const bool g0 = i0 < nl && i0 != kk, g1 = i1 < nl && i1 != kk;
                    const double c0 = g0 ? v[i0] * id : 0.0, c1 = g1 ? v[i1] * id : 0.0;
                    // both rows of the lane in one pass over the columns of the longer
                    const int len = g1 ? i1 + 1 : (g0 ? i0 + 1 : 0);
                    for (int jj = 0; jj < len; ++jj) {
                        const double vj = v[jj];
                        if (g0 && jj <= i0) row0[jj] = fma(-c0, vj, row0[jj]);
                        if (g1) row1[jj] = fma(-c1, vj, row1[jj]);
                    }
                    if (g0 && kk <= i0) row0[kk] = c0;
                    if (g1 && kk <= i1) row1[kk] = c1;
                    // the pivot row
                    if (i0 == kk || i1 == kk) {
                        double *rk = i0 == kk ? row0 : row1;
                        for (int jj = 0; jj < kk; ++jj) rk[jj] = v[jj] * id;
                        rk[kk] = -id;
                    }
                    wave_lds_fence();
                }
            }

        }

        // start: s_0 = q_0 = e_jl, r_0 = p_0 = S^{-1} e_jl, rho_0 = r_0^T s_0
        for (int i = lane; i < nl; i += SEED_T) {
            const double2 sv = make_double2(i == jl ? 1.0 : 0.0, 0.0);
            double rvx;
            if constexpr (PACKED)
                rvx = -(i >= jl ? Si[tri(i) + jl] : Si[tri(jl) + i]);
            else
                rvx = Si[i * sinv_ld(nl) + jl];
            const double2 rv = make_double2(rvx, 0.0);
            vs[i] = sv;
            vq[i] = sv;
            vr[i] = rv;
            vp[i] = rv;
        }
        wave_lds_fence();
        if (lane < nprow) hr[lane] = vr[prow];

        double2 pc[M], po[M];
        bool act[M];
        int nkm[M];
        double res[M];
#pragma unroll
        for (int m = 0; m < M; ++m) {
            pc[m] = po[m] = make_double2(1.0, 0.0);
            act[m] = lane + 64 * m < a.ns;
            nkm[m] = 0;
            res[m] = 1.0;
        }
        double2 rho = make_double2(PACKED ? -Si[tri(jl) + jl] : Si[jl * sinv_ld(nl) + jl], 0.0);
        double2 alpha_old = make_double2(1.0, 0.0), beta_old = zero;
        int status = SGF_MAXITER, iters = 0, applied = 0;
        double snorm2 = 1.0;
        const int max_iter = a.max_iter > 0 ? a.max_iter : 10 * nl;

        for (int it = 0; it < max_iter; ++it) {
            // w = z_s q - H p ; mu = p^T w
            double m0 = 0.0, m1 = 0.0;
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                const int i = lane + 64 * r;
                if (i >= nl) continue;
                double ax = 0.0, ay = 0.0;
                if constexpr (BMAX > 0) {
#pragma unroll
                    for (int b = 0; b < BMAX; ++b) {
                        const double2 *pb = &vp[4 * bcol[r][b]];
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            ax = fma(hrow[r][b][q], pb[q].x, ax);
                            ay = fma(hrow[r][b][q], pb[q].y, ay);
                        }
                    }
                } else {
                    const int A = i >> 2, o = i & 3;
                    const int t0 = a.lrow[a0 + A], t1 = A + 1 < n_loc ? a.lrow[a0 + A + 1] : nblk;
                    for (int t = t0; t < t1; ++t) {
                        const int B = a.lblk[2 * (b0 + t)];
                        const double *hb = &a.h[16 * (int64_t)a.lblk[2 * (b0 + t) + 1] + 4 * o];
                        const double2 *pb = &vp[4 * B];
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            ax = fma(hb[q], pb[q].x, ax);
                            ay = fma(hb[q], pb[q].y, ay);
                        }
                    }
                }
                const double2 pi_ = vp[i], qi = vq[i];
                const double2 wi = make_double2(zs.x * qi.x - zs.y * qi.y - ax, zs.x * qi.y + zs.y * qi.x - ay);
                vw[i] = wi;
                m0 = fma(pi_.x, wi.x, fma(-pi_.y, wi.y, m0));
                m1 = fma(pi_.x, wi.y, fma(pi_.y, wi.x, m1));
            }
            const double2 mu = make_double2(wave_reduce(m0), wave_reduce(m1));
            iters = it + 1;
            if (!cfinite(mu) || !cfinite(rho)) { status = SGF_NONFINITE; break; }
            if (mu.x == 0.0 && mu.y == 0.0) { status = SGF_BREAKDOWN; break; }
            const double2 alpha = cdiv(rho, mu);

            // s -= alpha w ; ||s||^2
            double r2 = 0.0;
            for (int i = lane; i < nl; i += SEED_T) {
                const double2 si = csub(vs[i], cmul(alpha, vw[i]));
                vs[i] = si;
                r2 = fma(si.x, si.x, fma(si.y, si.y, r2));
            }
            snorm2 = wave_reduce(r2);
            wave_lds_fence();
            // r = S^{-1} s ; rho' = r^T s.  Rows lane and lane + 64 share each
            // read of s (nl is a multiple of 4).  Dense inverse: row i is
            // contiguous.  Packed triangle A = -S^{-1}: row i reads its own
            // entries (j <= i), then column i of the rows below it, and the
            // sums are negated.
            double r0 = 0.0, r1 = 0.0;
            {
                const int i0 = lane, i1 = lane + 64;
                double ax[4] = {0.0, 0.0, 0.0, 0.0}, ay[4] = {0.0, 0.0, 0.0, 0.0};
                double bx[4] = {0.0, 0.0, 0.0, 0.0}, by[4] = {0.0, 0.0, 0.0, 0.0};
                if constexpr (!PACKED) {
                    const int ld = sinv_ld(nl);
                    const double *s0 = &Si[(i0 < nl ? i0 : 0) * ld], *s1 = &Si[(i1 < nl ? i1 : 0) * ld];
                    if (nl > 64) {
                        for (int jj = 0; jj < nl; jj += 4) {
#pragma unroll
                            for (int u = 0; u < 4; ++u) {
                                const double2 sj = vs[jj + u];
                                const double a = s0[jj + u], b = s1[jj + u];
                                ax[u] = fma(a, sj.x, ax[u]);
                                ay[u] = fma(a, sj.y, ay[u]);
                                bx[u] = fma(b, sj.x, bx[u]);
                                by[u] = fma(b, sj.y, by[u]);
                            }
                        }
                    } else {
                        for (int jj = 0; jj < nl; jj += 4) {
#pragma unroll
                            for (int u = 0; u < 4; ++u) {
                                const double2 sj = vs[jj + u];
                                const double a = s0[jj + u];
                                ax[u] = fma(a, sj.x, ax[u]);
                                ay[u] = fma(a, sj.y, ay[u]);
                            }
                        }
                    }
                } else {
                    const int c0 = i0 < nl ? i0 : nl - 1, c1 = i1 < nl ? i1 : nl - 1;  // rows read (clamped)
                    const int b0t = tri(c0), b1t = tri(c1);
                    int tj = 0;  // tri(jj)
                    if (nl > 64) {
                        for (int jj = 0; jj < nl; jj += 4) {
#pragma unroll
                            for (int u = 0; u < 4; ++u) {
                                const int jn = jj + u;
                                const double2 sj = vs[jn];
                                const double av = Si[jn <= c0 ? b0t + jn : tj + c0];
                                const double bv = Si[jn <= c1 ? b1t + jn : tj + c1];
                                tj += jn + 1;
                                ax[u] = fma(av, sj.x, ax[u]);
                                ay[u] = fma(av, sj.y, ay[u]);
                                bx[u] = fma(bv, sj.x, bx[u]);
                                by[u] = fma(bv, sj.y, by[u]);
                            }
                        }
                    } else {
                        for (int jj = 0; jj < nl; jj += 4) {
#pragma unroll
                            for (int u = 0; u < 4; ++u) {
                                const int jn = jj + u;
                                const double2 sj = vs[jn];
                                const double av = Si[jn <= c0 ? b0t + jn : tj + c0];
                                tj += jn + 1;
                                ax[u] = fma(av, sj.x, ax[u]);
                                ay[u] = fma(av, sj.y, ay[u]);
                            }
                        }
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        ax[u] = -ax[u];
                        ay[u] = -ay[u];
                        bx[u] = -bx[u];
                        by[u] = -by[u];
                    }
                }
                if (i0 < nl) {
                    const double rxs = (ax[0] + ax[1]) + (ax[2] + ax[3]), rys = (ay[0] + ay[1]) + (ay[2] + ay[3]);
                    vr[i0] = make_double2(rxs, rys);
                    const double2 si = vs[i0];
                    r0 = fma(rxs, si.x, fma(-rys, si.y, r0));
                    r1 = fma(rxs, si.y, fma(rys, si.x, r1));
                }
                if (i1 < nl) {
                    const double rxs = (bx[0] + bx[1]) + (bx[2] + bx[3]), rys = (by[0] + by[1]) + (by[2] + by[3]);
                    vr[i1] = make_double2(rxs, rys);
                    const double2 si = vs[i1];
                    r0 = fma(rxs, si.x, fma(-rys, si.y, r0));
                    r1 = fma(rxs, si.y, fma(rys, si.x, r1));
                }
            }
            const double2 rho_new = make_double2(wave_reduce(r0), wave_reduce(r1));
            const double2 ia = crcp(alpha);
            const double2 beta = cmul(rho_new, crcp(rho));
            for (int i = lane; i < nl; i += SEED_T) {
                vp[i] = cfma(beta, vp[i], vr[i]);
                vq[i] = cfma(beta, vq[i], vs[i]);
            }
            if (lane == 0) {
                hab[2 * it] = ia;
                hab[2 * it + 1] = cmul(beta, ia);
            }
            wave_lds_fence();
            if (lane < nprow) hr[(size_t)(it + 1) * a.rmax + lane] = vr[prow];

            const double2 coup = cmul(cmul(alpha, beta_old), crcp(alpha_old));
            int alive = 0;
#pragma unroll
            for (int m = 0; m < M; ++m) {
                if (!act[m]) continue;
                const double2 pn = cadd(cmul(cfma(alpha, sigma[m], make_double2(1.0, 0.0)), pc[m]),
                                        cmul(coup, csub(pc[m], po[m])));
                po[m] = pc[m];
                pc[m] = pn;
                const double pn2 = fma(pn.x, pn.x, pn.y * pn.y);
                if (snorm2 <= tol2 * pn2) {
                    act[m] = false;
                    nkm[m] = it + 1;
                    res[m] = sqrt(snorm2 / pn2);
                } else {
                    alive = 1;
                }
            }
            applied = it + 1;
            alpha_old = alpha;
            beta_old = beta;
            rho = rho_new;
            const bool any_alive = __any(alive);
            if (!any_alive || snorm2 == 0.0) { status = SGF_CONVERGED; break; }
            if (rho_new.x == 0.0 && rho_new.y == 0.0) { status = SGF_BREAKDOWN; break; }
            if (!cfinite(rho_new) || !isfinite(snorm2)) { status = SGF_NONFINITE; break; }
        }

#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int k = lane + 64 * m;
            if (k >= a.ns) continue;
            if (act[m]) {
                nkm[m] = applied;
                const double pn2 = fma(pc[m].x, pc[m].x, pc[m].y * pc[m].y);
                res[m] = applied > 0 ? sqrt(snorm2 / pn2) : 1.0;
            }
            a.nk[(size_t)slot * a.ns_pad + k] = nkm[m];
            if (a.resid) a.resid[c * a.ns + k] = res[m];
            if (a.shift_iters) a.shift_iters[c * a.ns + k] = nkm[m];
        }
        if (lane == 0) {
            *meta = ColMeta{(int32_t)c, iters, npa, status};
            a.iters[c] = iters;
            a.status[c] = status;
        }
        wave_lds_fence();
    }
}

// ---------------------------------------------------------------------------
// S != I seed pass with two wavefronts per column, for subspaces of 17 to 32
// atoms: thread t owns row t, so the product with the packed inverse and the
// block product are split over 128 threads, and the LDS that holds one
// column's inverse feeds two wavefronts instead of one.  The iteration is
// that of k_seed_gen with the packed triangle; the sums of an iteration go
// through a wavefront reduction and then the two wavefronts' totals, added in
// wavefront order, so every thread holds the same scalars and every branch on
// them is uniform over the workgroup.  Four barriers per iteration: after
// mu, after the update of s, after rho' and ||s||^2, and the vote on the
// running shifts.
// ---------------------------------------------------------------------------
constexpr int GEN2_T = 128;

// sum over the workgroup of NV values per thread, the same in every thread
template <int NV>
__device__ __forceinline__ void gen2_sum(const double (&v)[NV], double (*red)[NV], double (&out)[NV]) {
    const int wv = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        const double t = wave_reduce(v[i]);
        if ((threadIdx.x & 63) == 0) red[wv][i] = t;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NV; ++i) out[i] = red[0][i] + red[1][i];
}

template <int M, int BMAX>
__global__ __launch_bounds__(GEN2_T) void k_seed_gen2(SolveArgs a) {
    extern __shared__ double4 lds4[];
    char *lds = reinterpret_cast<char *>(lds4);
    double2 *vp = reinterpret_cast<double2 *>(lds + a.off_p);
    double2 *vs = reinterpret_cast<double2 *>(lds + a.off_s);
    double2 *vw = reinterpret_cast<double2 *>(lds + a.off_w);
    double2 *vq = reinterpret_cast<double2 *>(lds + a.off_q);
    double2 *vr = reinterpret_cast<double2 *>(lds + a.off_r);
    double *Si = reinterpret_cast<double *>(lds + a.off_sinv);  // packed lower triangle, tri(nl) doubles
    __shared__ double red_mu[2][2], red_rs[2][3];
    __shared__ int64_t sh_ticket;
    const int tid = threadIdx.x;
    const double2 zs = a.z[a.seed];
    double2 sigma[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int k = tid + GEN2_T * m;
        sigma[m] = k < a.ns ? csub(a.z[k], zs) : make_double2(0.0, 0.0);
    }
    const double tol2 = a.tol * a.tol;
    const double2 zero = make_double2(0.0, 0.0);
    constexpr int NBR = BMAX > 0 ? BMAX : 1;

    for (;;) {
        if (tid == 0) sh_ticket = (int64_t)atomicAdd(reinterpret_cast<unsigned long long *>(a.ticket), 1ull);
        __syncthreads();
        int64_t ticket = sh_ticket;
        __syncthreads();  // sh_ticket is read by all before the next column writes it
        if (ticket >= a.batch_end - a.batch_begin) break;
        const int64_t slot = ticket;
        ticket += a.batch_begin;
        const int64_t c = a.order ? (int64_t)a.order[ticket] : ticket;
        if (c < 0 || c >= a.n_cols) continue;  // reported by the launch of the other class
        const int64_t j = a.cols[c];
        const int32_t pl = a.col_plan[c];
        bool bad = pl < 0 || pl >= a.n_plans || j < 0;
        int64_t a0 = 0, b0 = 0, p0 = 0;
        int n_loc = 0, nblk = 0, npa = 0, cl = 0;
        if (!bad) {
            a0 = a.atom_off[pl];
            n_loc = (int)(a.atom_off[pl + 1] - a0);
            b0 = a.blk_off[pl];
            nblk = (int)(a.blk_off[pl + 1] - b0);
            p0 = a.pa_off[pl];
            npa = (int)(a.pa_off[pl + 1] - p0);
            cl = a.center_loc[pl];
            bad = n_loc < 1 || n_loc > 32 || n_loc > a.max_loc_atoms || npa < 1 || 4 * npa > a.rmax || cl < 0 ||
                  cl >= n_loc || a.loc_atom[a0 + cl] != (int32_t)(j >> 2);
        }
        // this launch takes the good columns of its size class only
        if (bad || n_loc < a.loc_lo || n_loc > a.loc_hi) continue;
        const int nl = 4 * n_loc;
        const int i = tid;  // this thread's row
        const bool row = i < nl;
        int bcol[NBR];
        double hrow[NBR][4];
        int wide = 0;
        {
            const int A = i >> 2, o = i & 3;
            int t0 = 0, nb = 0;
            if (row) {
                t0 = a.lrow[a0 + A];
                nb = (A + 1 < n_loc ? a.lrow[a0 + A + 1] : nblk) - t0;
            }
            wide = nb > BMAX ? 1 : 0;
#pragma unroll
            for (int b = 0; b < NBR; ++b) {
                bcol[b] = 0;
                hrow[b][0] = hrow[b][1] = hrow[b][2] = hrow[b][3] = 0.0;
                if (b < nb) {
                    const int32_t *lb = &a.lblk[2 * (b0 + t0 + b)];
                    bcol[b] = lb[0];
                    const double *hb = &a.h[16 * (int64_t)lb[1] + 4 * o];
#pragma unroll
                    for (int q = 0; q < 4; ++q) hrow[b][q] = hb[q];
                }
            }
        }
        if (__syncthreads_or(wide)) {
            if (tid == 0) {
                a.meta[slot] = ColMeta{-1, 0, 0, SGF_BADCOLUMN};
                a.iters[c] = 0;
                a.status[c] = SGF_BADCOLUMN;
            }
            continue;
        }
        const int jl = 4 * cl + (int)(j & 3);
        const int nprow = 4 * npa;
        const int prow = tid < nprow ? 4 * a.pa_loc[p0 + (tid >> 2)] + (tid & 3) : 0;
        double2 *hab = a.hab + (size_t)slot * a.cap * 2;
        double2 *hr = a.hr + (size_t)slot * (a.cap + 1) * a.rmax;

        // S_L packed, then the sweep in place (after the last pivot the
        // triangle holds -S_L^{-1}); v = column k of the pivot lives in vw
        for (int e = tid; e < tri(nl); e += GEN2_T) Si[e] = 0.0;
        __syncthreads();
        for (int A = tid; A < n_loc; A += GEN2_T) {
            const int t0 = a.lrow[a0 + A], t1 = A + 1 < n_loc ? a.lrow[a0 + A + 1] : nblk;
            for (int t = t0; t < t1; ++t) {
                const int B = a.lblk[2 * (b0 + t)];
                if (B > A) continue;  // the upper blocks mirror the lower ones
                const double *sb = &a.s[16 * (int64_t)a.lblk[2 * (b0 + t) + 1]];
                for (int o = 0; o < 4; ++o)
                    for (int q = 0; q < 4; ++q)
                        if (4 * B + q <= 4 * A + o) Si[tri(4 * A + o) + 4 * B + q] = sb[4 * o + q];
            }
        }
        __syncthreads();
        {
            double *v = reinterpret_cast<double *>(vw);
            double *rw = &Si[tri(row ? i : 0)];
            for (int kk = 0; kk < nl; ++kk) {
                if (row) v[i] = i >= kk ? Si[tri(i) + kk] : Si[tri(kk) + i];
                __syncthreads();
                const double id = 1.0 / v[kk];
                if (row && i != kk) {
                    const double ci = v[i] * id;
                    for (int jj = 0; jj <= i; ++jj) rw[jj] = fma(-ci, v[jj], rw[jj]);
                    if (kk <= i) rw[kk] = ci;
                } else if (row) {
                    for (int jj = 0; jj < kk; ++jj) rw[jj] = v[jj] * id;
                    rw[kk] = -id;
                }
                __syncthreads();
            }
        }

        // start: s_0 = q_0 = e_jl, r_0 = p_0 = S^{-1} e_jl, rho_0 = r_0^T s_0
        if (row) {
            const double2 sv = make_double2(i == jl ? 1.0 : 0.0, 0.0);
            const double2 rv = make_double2(-(i >= jl ? Si[tri(i) + jl] : Si[tri(jl) + i]), 0.0);
            vs[i] = sv;
            vq[i] = sv;
            vr[i] = rv;
            vp[i] = rv;
        }
        __syncthreads();
        if (tid < nprow) hr[tid] = vr[prow];

        double2 pc[M], po[M];
        bool act[M];
        int nkm[M];
        double res[M];
#pragma unroll
        for (int m = 0; m < M; ++m) {
            pc[m] = po[m] = make_double2(1.0, 0.0);
            act[m] = tid + GEN2_T * m < a.ns;
            nkm[m] = 0;
            res[m] = 1.0;
        }
        double2 rho = make_double2(-Si[tri(jl) + jl], 0.0);
        double2 alpha_old = make_double2(1.0, 0.0), beta_old = zero;
        int status = SGF_MAXITER, iters = 0, applied = 0;
        double snorm2 = 1.0;
        const int max_iter = a.max_iter > 0 ? a.max_iter : 10 * nl;
        const int c0 = row ? i : nl - 1;  // row read by the product (clamped)
        const int b0t = tri(c0);

        for (int it = 0; it < max_iter; ++it) {
            // w = z_s q - H p ; mu = p^T w
            double2 mu;
            {
                double m0 = 0.0, m1 = 0.0;
                if (row) {
                    double ax = 0.0, ay = 0.0;
#pragma unroll
                    for (int b = 0; b < BMAX; ++b) {
                        const double2 *pb = &vp[4 * bcol[b]];
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            ax = fma(hrow[b][q], pb[q].x, ax);
                            ay = fma(hrow[b][q], pb[q].y, ay);
                        }
                    }
                    const double2 pi_ = vp[i], qi = vq[i];
                    const double2 wi = make_double2(zs.x * qi.x - zs.y * qi.y - ax, zs.x * qi.y + zs.y * qi.x - ay);
                    vw[i] = wi;
                    m0 = fma(pi_.x, wi.x, -pi_.y * wi.y);
                    m1 = fma(pi_.x, wi.y, pi_.y * wi.x);
                }
                const double v[2] = {m0, m1};
                double sum[2];
                gen2_sum<2>(v, red_mu, sum);
                mu = make_double2(sum[0], sum[1]);
            }
            iters = it + 1;
            if (!cfinite(mu) || !cfinite(rho)) { status = SGF_NONFINITE; break; }
            if (mu.x == 0.0 && mu.y == 0.0) { status = SGF_BREAKDOWN; break; }
            const double2 alpha = cdiv(rho, mu);

            // s -= alpha w
            double2 si = zero;
            if (row) {
                si = csub(vs[i], cmul(alpha, vw[i]));
                vs[i] = si;
            }
            __syncthreads();
            // r = S^{-1} s (the triangle holds -S^{-1}: row i's own entries,
            // then column i of the rows below it, negated) ; rho' = r^T s ; ||s||^2
            double2 rho_new;
            {
                double rr[3] = {0.0, 0.0, 0.0};
                if (row) {
                    double ax[4] = {0.0, 0.0, 0.0, 0.0}, ay[4] = {0.0, 0.0, 0.0, 0.0};
                    int tj = 0;  // tri(jj)
                    for (int jj = 0; jj < nl; jj += 4) {
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            const int jn = jj + u;
                            const double2 sj = vs[jn];
                            const double av = Si[jn <= c0 ? b0t + jn : tj + c0];
                            tj += jn + 1;
                            ax[u] = fma(av, sj.x, ax[u]);
                            ay[u] = fma(av, sj.y, ay[u]);
                        }
                    }
                    const double rxs = -((ax[0] + ax[1]) + (ax[2] + ax[3]));
                    const double rys = -((ay[0] + ay[1]) + (ay[2] + ay[3]));
                    vr[i] = make_double2(rxs, rys);
                    rr[0] = fma(rxs, si.x, -rys * si.y);
                    rr[1] = fma(rxs, si.y, rys * si.x);
                    rr[2] = fma(si.x, si.x, si.y * si.y);
                }
                double sum[3];
                gen2_sum<3>(rr, red_rs, sum);
                rho_new = make_double2(sum[0], sum[1]);
                snorm2 = sum[2];
            }
            const double2 ia = crcp(alpha);
            const double2 beta = cmul(rho_new, crcp(rho));
            if (row) {
                vp[i] = cfma(beta, vp[i], vr[i]);
                vq[i] = cfma(beta, vq[i], si);
            }
            if (tid == 0) {
                hab[2 * it] = ia;
                hab[2 * it + 1] = cmul(beta, ia);
            }
            if (tid < nprow) hr[(size_t)(it + 1) * a.rmax + tid] = vr[prow];

            const double2 coup = cmul(cmul(alpha, beta_old), crcp(alpha_old));
            int alive = 0;
#pragma unroll
            for (int m = 0; m < M; ++m) {
                if (!act[m]) continue;
                const double2 pn = cadd(cmul(cfma(alpha, sigma[m], make_double2(1.0, 0.0)), pc[m]),
                                        cmul(coup, csub(pc[m], po[m])));
                po[m] = pc[m];
                pc[m] = pn;
                const double pn2 = fma(pn.x, pn.x, pn.y * pn.y);
                if (snorm2 <= tol2 * pn2) {
                    act[m] = false;
                    nkm[m] = it + 1;
                    res[m] = sqrt(snorm2 / pn2);
                } else {
                    alive = 1;
                }
            }
            applied = it + 1;
            alpha_old = alpha;
            beta_old = beta;
            rho = rho_new;
            // the vote is also the barrier that ends the iteration (p is in vp)
            const bool any_alive = __syncthreads_or(alive) != 0;
            if (!any_alive || snorm2 == 0.0) { status = SGF_CONVERGED; break; }
            if (rho_new.x == 0.0 && rho_new.y == 0.0) { status = SGF_BREAKDOWN; break; }
            if (!cfinite(rho_new) || !isfinite(snorm2)) { status = SGF_NONFINITE; break; }
        }

#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int k = tid + GEN2_T * m;
            if (k >= a.ns) continue;
            if (act[m]) {
                nkm[m] = applied;
                const double pn2 = fma(pc[m].x, pc[m].x, pc[m].y * pc[m].y);
                res[m] = applied > 0 ? sqrt(snorm2 / pn2) : 1.0;
            }
            a.nk[(size_t)slot * a.ns_pad + k] = nkm[m];
            if (a.resid) a.resid[c * a.ns + k] = res[m];
            if (a.shift_iters) a.shift_iters[c * a.ns + k] = nkm[m];
        }
        if (tid == 0) {
            a.meta[slot] = ColMeta{(int32_t)c, iters, npa, status};
            a.iters[c] = iters;
            a.status[c] = status;
        }
        __syncthreads();  // LDS reuse by the next column
    }
}

// ---------------------------------------------------------------------------
// S != I seed pass with two wavefronts per column for subspaces of at most 16
// atoms (nl <= 64) and the dense inverse: lane l of wavefront h works on row
// l and on the columns of the inverse that belong to the first ceil(n_loc/2)
// atoms (h = 0) or to the others (h = 1), so each row's product and each
// row's elimination step are split between the two wavefronts; the two
// halves of a row's product are added in wavefront order.  Wavefront 0 forms
// the block product of H and the vector updates.
// The Gauss-Jordan elimination is that of k_seed_gen (the same bits); the
// iteration sums run over the workgroup as in k_seed_gen2.
// ---------------------------------------------------------------------------
template <int M, int BMAX>
__global__ __launch_bounds__(GEN2_T) void k_seed_gen2s(SolveArgs a) {
    extern __shared__ double4 lds4[];
    char *lds = reinterpret_cast<char *>(lds4);
    double2 *vp = reinterpret_cast<double2 *>(lds + a.off_p);
    double2 *vs = reinterpret_cast<double2 *>(lds + a.off_s);
    double2 *vw = reinterpret_cast<double2 *>(lds + a.off_w);
    double2 *vq = reinterpret_cast<double2 *>(lds + a.off_q);
    double2 *vr = reinterpret_cast<double2 *>(lds + a.off_r);
    double *Si = reinterpret_cast<double *>(lds + a.off_sinv);  // dense, row stride sinv_ld(nl)
    __shared__ double red_mu[2][2], red_rs[2][3];
    __shared__ double2 half1[64];  // wavefront 1's half of each row's product
    __shared__ int64_t sh_ticket;
    const int tid = threadIdx.x;
    const int lane = tid & 63, h = tid >> 6;
    const double2 zs = a.z[a.seed];
    double2 sigma[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int k = tid + GEN2_T * m;
        sigma[m] = k < a.ns ? csub(a.z[k], zs) : make_double2(0.0, 0.0);
    }
    const double tol2 = a.tol * a.tol;
    const double2 zero = make_double2(0.0, 0.0);
    constexpr int NBR = BMAX > 0 ? BMAX : 1;

    for (;;) {
        if (tid == 0) sh_ticket = (int64_t)atomicAdd(reinterpret_cast<unsigned long long *>(a.ticket), 1ull);
        __syncthreads();
        int64_t ticket = sh_ticket;
        __syncthreads();
        if (ticket >= a.batch_end - a.batch_begin) break;
        const int64_t slot = ticket;
        ticket += a.batch_begin;
        const int64_t c = a.order ? (int64_t)a.order[ticket] : ticket;
        if (c < 0 || c >= a.n_cols) {
            if (tid == 0) a.meta[slot] = ColMeta{-1, 0, 0, SGF_BADCOLUMN};
            continue;
        }
        const int64_t j = a.cols[c];
        const int32_t pl = a.col_plan[c];
        bool bad = pl < 0 || pl >= a.n_plans || j < 0;
        int64_t a0 = 0, b0 = 0, p0 = 0;
        int n_loc = 0, nblk = 0, npa = 0, cl = 0;
        if (!bad) {
            a0 = a.atom_off[pl];
            n_loc = (int)(a.atom_off[pl + 1] - a0);
            b0 = a.blk_off[pl];
            nblk = (int)(a.blk_off[pl + 1] - b0);
            p0 = a.pa_off[pl];
            npa = (int)(a.pa_off[pl + 1] - p0);
            cl = a.center_loc[pl];
            bad = n_loc < 1 || n_loc > 32 || n_loc > a.max_loc_atoms || npa < 1 || 4 * npa > a.rmax || cl < 0 ||
                  cl >= n_loc || a.loc_atom[a0 + cl] != (int32_t)(j >> 2);
        }
        // this launch takes the columns of up to loc_hi (<= 16) atoms and
        // reports the unsolvable ones
        if (!bad && n_loc > a.loc_hi) continue;
        const int nl = 4 * n_loc;
        const int i = lane;  // this thread's row
        const bool row = !bad && i < nl;
        int bcol[NBR];
        double hrow[NBR][4];
        int wide = 0;
        {
            const int A = i >> 2, o = i & 3;
            int t0 = 0, nb = 0;
            if (row) {
                t0 = a.lrow[a0 + A];
                nb = (A + 1 < n_loc ? a.lrow[a0 + A + 1] : nblk) - t0;
            }
            wide = nb > BMAX ? 1 : 0;
#pragma unroll
            for (int b = 0; b < NBR; ++b) {
                bcol[b] = 0;
                hrow[b][0] = hrow[b][1] = hrow[b][2] = hrow[b][3] = 0.0;
                if (b < nb) {
                    const int32_t *lb = &a.lblk[2 * (b0 + t0 + b)];
                    bcol[b] = lb[0];
                    const double *hb = &a.h[16 * (int64_t)lb[1] + 4 * o];
#pragma unroll
                    for (int q = 0; q < 4; ++q) hrow[b][q] = hb[q];
                }
            }
        }
        if (__syncthreads_or(bad || wide)) {
            if (tid == 0) {
                a.meta[slot] = ColMeta{-1, 0, 0, SGF_BADCOLUMN};
                a.iters[c] = 0;
                a.status[c] = SGF_BADCOLUMN;
            }
            continue;
        }
        const int jl = 4 * cl + (int)(j & 3);
        const int nprow = 4 * npa;
        const int prow = tid < nprow ? 4 * a.pa_loc[p0 + (tid >> 2)] + (tid & 3) : 0;
        double2 *hab = a.hab + (size_t)slot * a.cap * 2;
        double2 *hr = a.hr + (size_t)slot * (a.cap + 1) * a.rmax;
        const int ld = sinv_ld(nl);
        // this thread's columns: the first ceil(n_loc / 2) atoms for wavefront
        // 0, the rest for wavefront 1, so both ranges are whole multiples of 4
        const int hw = 4 * ((n_loc + 1) >> 1);
        const int j0 = h == 0 ? 0 : hw, j1 = h == 0 ? hw : nl;

        // dense S_L, then its inverse in place (Gauss-Jordan without pivoting)
        for (int e = tid; e < nl * ld; e += GEN2_T) Si[e] = 0.0;
        __syncthreads();
        for (int A = tid; A < n_loc; A += GEN2_T) {
            const int t0 = a.lrow[a0 + A], t1 = A + 1 < n_loc ? a.lrow[a0 + A + 1] : nblk;
            for (int t = t0; t < t1; ++t) {
                const int B = a.lblk[2 * (b0 + t)];
                const double *sb = &a.s[16 * (int64_t)a.lblk[2 * (b0 + t) + 1]];
                for (int o = 0; o < 4; ++o)
                    for (int q = 0; q < 4; ++q) Si[(4 * A + o) * ld + 4 * B + q] = sb[4 * o + q];
            }
        }
        __syncthreads();
        {
            double *w0 = &Si[(row ? i : 0) * ld];
            for (int kk = 0; kk < nl; ++kk) {
                const double piv = 1.0 / Si[kk * ld + kk];
                // multiplier of this row, read before any thread changes column kk
                const double f0 = (row && i != kk) ? w0[kk] : 0.0;
                __syncthreads();
                for (int jj = tid; jj < nl; jj += GEN2_T) Si[kk * ld + jj] = (jj == kk) ? piv : Si[kk * ld + jj] * piv;
                __syncthreads();
                if (row && i != kk) {
                    const double *pr = &Si[kk * ld];
                    for (int jj = j0; jj < j1; jj += 4) {
#pragma unroll
                        for (int u = 0; u < 4; ++u) w0[jj + u] = fma(-f0, pr[jj + u], w0[jj + u]);
                    }
                    if (kk >= j0 && kk < j1) w0[kk] = -f0 * piv;
                }
                __syncthreads();
            }
        }

        // start: s_0 = q_0 = e_jl, r_0 = p_0 = S^{-1} e_jl, rho_0 = r_0^T s_0
        if (h == 0 && row) {
            const double2 sv = make_double2(i == jl ? 1.0 : 0.0, 0.0);
            const double2 rv = make_double2(Si[i * ld + jl], 0.0);
            vs[i] = sv;
            vq[i] = sv;
            vr[i] = rv;
            vp[i] = rv;
        }
        __syncthreads();
        if (tid < nprow) hr[tid] = vr[prow];

        double2 pc[M], po[M];
        bool act[M];
        int nkm[M];
        double res[M];
#pragma unroll
        for (int m = 0; m < M; ++m) {
            pc[m] = po[m] = make_double2(1.0, 0.0);
            act[m] = tid + GEN2_T * m < a.ns;
            nkm[m] = 0;
            res[m] = 1.0;
        }
        double2 rho = make_double2(Si[jl * ld + jl], 0.0);
        double2 alpha_old = make_double2(1.0, 0.0), beta_old = zero;
        int status = SGF_MAXITER, iters = 0, applied = 0;
        double snorm2 = 1.0;
        const int max_iter = a.max_iter > 0 ? a.max_iter : 10 * nl;
        const double *srow = &Si[(row ? i : 0) * ld];

        for (int it = 0; it < max_iter; ++it) {
            // w = z_s q - H p ; mu = p^T w (wavefront 0)
            double2 mu;
            {
                double m0 = 0.0, m1 = 0.0;
                if (h == 0 && row) {
                    double ax = 0.0, ay = 0.0;
#pragma unroll
                    for (int b = 0; b < BMAX; ++b) {
                        const double2 *pb = &vp[4 * bcol[b]];
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            ax = fma(hrow[b][q], pb[q].x, ax);
                            ay = fma(hrow[b][q], pb[q].y, ay);
                        }
                    }
                    const double2 pi_ = vp[i], qi = vq[i];
                    const double2 wi = make_double2(zs.x * qi.x - zs.y * qi.y - ax, zs.x * qi.y + zs.y * qi.x - ay);
                    vw[i] = wi;
                    m0 = fma(pi_.x, wi.x, -pi_.y * wi.y);
                    m1 = fma(pi_.x, wi.y, pi_.y * wi.x);
                }
                const double v[2] = {m0, m1};
                double sum[2];
                gen2_sum<2>(v, red_mu, sum);
                mu = make_double2(sum[0], sum[1]);
            }
            iters = it + 1;
            if (!cfinite(mu) || !cfinite(rho)) { status = SGF_NONFINITE; break; }
            if (mu.x == 0.0 && mu.y == 0.0) { status = SGF_BREAKDOWN; break; }
            const double2 alpha = cdiv(rho, mu);

            // s -= alpha w (wavefront 0)
            double2 si = zero;
            if (h == 0 && row) {
                si = csub(vs[i], cmul(alpha, vw[i]));
                vs[i] = si;
            }
            __syncthreads();
            // r = S^{-1} s: each wavefront one half of the row, four partial sums
            double2 part = zero;
            if (row) {
                double ax[4] = {0.0, 0.0, 0.0, 0.0}, ay[4] = {0.0, 0.0, 0.0, 0.0};
                for (int jj = j0; jj < j1; jj += 4) {
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const double2 sj = vs[jj + u];
                        const double av = srow[jj + u];
                        ax[u] = fma(av, sj.x, ax[u]);
                        ay[u] = fma(av, sj.y, ay[u]);
                    }
                }
                part = make_double2((ax[0] + ax[1]) + (ax[2] + ax[3]), (ay[0] + ay[1]) + (ay[2] + ay[3]));
                if (h == 1) half1[i] = part;
            }
            __syncthreads();
            // rho' = r^T s ; ||s||^2 (wavefront 0)
            double2 rho_new;
            {
                double rr[3] = {0.0, 0.0, 0.0};
                if (h == 0 && row) {
                    const double2 o1 = half1[i];
                    const double rxs = part.x + o1.x, rys = part.y + o1.y;
                    vr[i] = make_double2(rxs, rys);
                    rr[0] = fma(rxs, si.x, -rys * si.y);
                    rr[1] = fma(rxs, si.y, rys * si.x);
                    rr[2] = fma(si.x, si.x, si.y * si.y);
                }
                double sum[3];
                gen2_sum<3>(rr, red_rs, sum);
                rho_new = make_double2(sum[0], sum[1]);
                snorm2 = sum[2];
            }
            const double2 ia = crcp(alpha);
            const double2 beta = cmul(rho_new, crcp(rho));
            if (h == 0 && row) {
                vp[i] = cfma(beta, vp[i], vr[i]);
                vq[i] = cfma(beta, vq[i], si);
            }
            if (tid == 0) {
                hab[2 * it] = ia;
                hab[2 * it + 1] = cmul(beta, ia);
            }
            if (tid < nprow) hr[(size_t)(it + 1) * a.rmax + tid] = vr[prow];

            const double2 coup = cmul(cmul(alpha, beta_old), crcp(alpha_old));
            int alive = 0;
#pragma unroll
            for (int m = 0; m < M; ++m) {
                if (!act[m]) continue;
                const double2 pn = cadd(cmul(cfma(alpha, sigma[m], make_double2(1.0, 0.0)), pc[m]),
                                        cmul(coup, csub(pc[m], po[m])));
                po[m] = pc[m];
                pc[m] = pn;
                const double pn2 = fma(pn.x, pn.x, pn.y * pn.y);
                if (snorm2 <= tol2 * pn2) {
                    act[m] = false;
                    nkm[m] = it + 1;
                    res[m] = sqrt(snorm2 / pn2);
                } else {
                    alive = 1;
                }
            }
            applied = it + 1;
            alpha_old = alpha;
            beta_old = beta;
            rho = rho_new;
            const bool any_alive = __syncthreads_or(alive) != 0;
            if (!any_alive || snorm2 == 0.0) { status = SGF_CONVERGED; break; }
            if (rho_new.x == 0.0 && rho_new.y == 0.0) { status = SGF_BREAKDOWN; break; }
            if (!cfinite(rho_new) || !isfinite(snorm2)) { status = SGF_NONFINITE; break; }
        }

#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int k = tid + GEN2_T * m;
            if (k >= a.ns) continue;
            if (act[m]) {
                nkm[m] = applied;
                const double pn2 = fma(pc[m].x, pc[m].x, pc[m].y * pc[m].y);
                res[m] = applied > 0 ? sqrt(snorm2 / pn2) : 1.0;
            }
            a.nk[(size_t)slot * a.ns_pad + k] = nkm[m];
            if (a.resid) a.resid[c * a.ns + k] = res[m];
            if (a.shift_iters) a.shift_iters[c * a.ns + k] = nkm[m];
        }
        if (tid == 0) {
            a.meta[slot] = ColMeta{(int32_t)c, iters, npa, status};
            a.iters[c] = iters;
            a.status[c] = status;
        }
        __syncthreads();  // LDS reuse by the next column
    }
}

// ---------------------------------------------------------------------------
// Shift pass
// ---------------------------------------------------------------------------

// S <- g S + r for two projection rows, in place; the same four fused
// multiply-adds per row as cfma(g, S, r), so the same bits.  Written as VALU
// FMAs with S tied to its own registers: compiled from cfma, the new value
// lands in the register of the loaded row and is copied back afterwards, two
// 64-bit moves per row and step.  Both temporaries of a row are formed before
// that row's S is overwritten.
__device__ __forceinline__ void cfma_rows2(double2 &S0, double2 &S1, double2 r0, double2 r1, double2 g) {
    double t0x, t0y, t1x, t1y;
    asm("v_fma_f64 %[t0x], -%[gy], %[s0y], %[r0x]\n\t"
        "v_fma_f64 %[t0y], %[gy], %[s0x], %[r0y]\n\t"
        "v_fma_f64 %[t1x], -%[gy], %[s1y], %[r1x]\n\t"
        "v_fma_f64 %[t1y], %[gy], %[s1x], %[r1y]\n\t"
        "v_fma_f64 %[s0x], %[gx], %[s0x], %[t0x]\n\t"
        "v_fma_f64 %[s0y], %[gx], %[s0y], %[t0y]\n\t"
        "v_fma_f64 %[s1x], %[gx], %[s1x], %[t1x]\n\t"
        "v_fma_f64 %[s1y], %[gx], %[s1y], %[t1y]"
        : [s0x] "+v"(S0.x), [s0y] "+v"(S0.y), [s1x] "+v"(S1.x), [s1y] "+v"(S1.y), [t0x] "=&v"(t0x),
          [t0y] "=&v"(t0y), [t1x] "=&v"(t1x), [t1y] "=&v"(t1y)
        : [gx] "v"(g.x), [gy] "v"(g.y), [r0x] "v"(r0.x), [r0y] "v"(r0.y), [r1x] "v"(r1.x), [r1y] "v"(r1.y));
}

// Orders this wavefront's LDS accesses (release, wave barrier, acquire)
// and waits for them: lanes read what other lanes of the wavefront wrote.
__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    __builtin_amdgcn_s_waitcnt(0xC07F);
}

// One workgroup per column; each lane carries MS shifts.  The shifts are
// first sorted by their step count N_k so that the lanes of a wavefront (and
// the MS shifts of a lane) end their sweeps together.
template <int NPA, int MS>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(MS == 1 && NPA <= 4 ? 4 : (MS == 1 && NPA <= 6 ? 3 : 1)))) void k_shift(SolveArgs a) {
    // The history is staged in LDS a chunk of backward steps at a time.
    // PWV: each wavefront stages its own chunks (dynamic LDS, a region per
    // wavefront) and sweeps only its own steps, so a wavefront of short
    // shifts does not wait at the chunk barriers of a longer one (bundle
    // 28.9 -> 28.1 ms, overlap bundle 57.3 -> 53.3 ms).  With four or six
    // and more projection atoms the extra staging registers spill, and the
    // workgroup stages each chunk once (static LDS, 24 steps where that
    // still fits the register budget, else 16).
    constexpr bool PWV = NPA <= 5 && NPA != 4;
    constexpr int CH = PWV ? SHIFT_CH : (NPA <= 3 || (NPA == 5 && MS == 1)) ? 24 : SHIFT_CH;
    static_assert(2 * CH + 2 <= 64, "a 64-thread shift workgroup stages a chunk's scalars in one pass");
    __shared__ int skey[512];                      // (N_k << 10) | k, sorted ascending
    __shared__ double rpart[32 * 8];               // [row][wave] partial rho sums
    const int64_t slot = blockIdx.x;
    const ColMeta meta = a.meta[slot];
    if (meta.col < 0) return;  // uniform over the workgroup
    const int64_t c = meta.col;
    const int npa = meta.npa;
    const int nrow = 4 * npa;
    const int tid = threadIdx.x, T = blockDim.x;
    const int wv = tid >> 6, lane = tid & 63, nwv = T >> 6;
    const double2 *hab = a.hab + (size_t)slot * a.cap * 2;
    const double2 *hr = a.hr + (size_t)slot * (a.cap + 1) * a.rmax;
    const double2 zero = make_double2(0.0, 0.0);

    // sort the shifts of this column by step count (bitonic, power-of-two length)
    int nsort = 64;
    while (nsort < a.ns_pad) nsort <<= 1;
    constexpr int SENT = 0x7fffffff;
    for (int i = tid; i < 512; i += T)
        skey[i] = i < a.ns ? (a.nk[(size_t)slot * a.ns_pad + i] << 10) | i : (i < a.ns_pad ? i : SENT);
    __syncthreads();
    for (int kk = 2; kk <= nsort; kk <<= 1)
        for (int jj = kk >> 1; jj > 0; jj >>= 1) {
            for (int i = tid; i < nsort; i += T) {
                const int l = i ^ jj;
                if (l > i) {
                    const int x = skey[i], y = skey[l];
                    if ((x > y) == ((i & kk) == 0)) { skey[i] = y; skey[l] = x; }
                }
            }
            __syncthreads();
        }
    int kof[MS], nk[MS];
    double2 sigma[MS];
#pragma unroll
    for (int u = 0; u < MS; ++u) {
        const int key = skey[tid * MS + u];
        const bool live = key != SENT && (key & 1023) < a.ns;
        kof[u] = live ? (key & 1023) : -1;
        nk[u] = live ? (key >> 10) : 0;
        sigma[u] = live ? csub(a.z[kof[u]], a.z[a.seed]) : zero;
    }
    const int top = skey[a.ns_pad - 1] >> 10;  // largest N_k (ns_pad - ns padding keys sort first)
    int wtop = 0;  // largest N_k in this wavefront
#pragma unroll
    for (int u = 0; u < MS; ++u) wtop = max(wtop, nk[u]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) wtop = max(wtop, __shfl_xor(wtop, off, 64));

    double2 S[MS][4 * NPA];
    double2 g[MS], y0[MS];
#pragma unroll
    for (int u = 0; u < MS; ++u) {
        g[u] = y0[u] = zero;
#pragma unroll
        for (int r = 0; r < 4 * NPA; ++r) S[u][r] = zero;
    }
    if constexpr (PWV) {
        constexpr int PW = (CH + 1) * 2 + CH * 4 * NPA;  // double2 per wavefront
        extern __shared__ __align__(16) double2 shift_dyn[];
        double2 (*sab)[2] = reinterpret_cast<double2 (*)[2]>(shift_dyn + (size_t)wv * PW);
        double2 (*srow)[4 * NPA] = reinterpret_cast<double2 (*)[4 * NPA]>(shift_dyn + (size_t)wv * PW + (CH + 1) * 2);
        for (int hi = wtop - 1; hi >= 0; hi -= CH) {
            const int lo = hi - CH + 1 > 0 ? hi - CH + 1 : 0;
            const int nstep = hi - lo + 1;
            // every load of the chunk issued before this wavefront's reads of
            // the previous one are ordered, written to its LDS region after
            constexpr int UR = (CH * 4 * NPA + 63) / 64;
            const int nab = (nstep + 1) * 2, nrv = nstep * nrow;
            double2 vab = zero;
            if (lane < nab && lo - 1 + (lane >> 1) >= 0) vab = hab[2 * (lo - 1 + (lane >> 1)) + (lane & 1)];
            double2 vr[UR];
#pragma unroll
            for (int u = 0; u < UR; ++u) {
                const int idx = lane + u * 64;
                vr[u] = zero;
                if (idx < nrv) {
                    const int sm = idx / nrow, r = idx - sm * nrow;
                    vr[u] = hr[(size_t)(lo + sm) * a.rmax + r];
                }
            }
            wave_sync_lds();  // this wavefront's reads of the previous chunk are done
            if (lane < nab) sab[lane >> 1][lane & 1] = vab;
#pragma unroll
            for (int u = 0; u < UR; ++u) {
                const int idx = lane + u * 64;
                if (idx < nrv) {
                    const int sm = idx / nrow, r = idx - sm * nrow;
                    srow[sm][r] = vr[u];
                }
            }
            wave_sync_lds();
            for (int m = hi; m >= lo; --m) {
                // 1/alpha and beta/alpha of steps m and m - 1, read from LDS at every
                // step (carrying the step-m pair over would cost register moves)
                const double2 ia_m = sab[m - lo + 1][0], ba_m = sab[m - lo + 1][1];
                const double2 ia_p = sab[m - lo][0], ba_p = sab[m - lo][1];
                const double2 *rm = srow[m - lo];
#pragma unroll
                for (int u = 0; u < MS; ++u) {
                    if (m >= nk[u]) continue;
                    // g is exactly zero up to the shift's first step (m = N_k - 1),
                    // where this is the bare diagonal
                    const double2 d = csub(cadd(cadd(ia_m, ba_p), sigma[u]), cmul(ba_m, g[u]));
#pragma unroll
                    for (int q = 0; q < NPA; ++q) {
                        if (q < npa) {
                            cfma_rows2(S[u][4 * q], S[u][4 * q + 1], rm[4 * q], rm[4 * q + 1], g[u]);
                            cfma_rows2(S[u][4 * q + 2], S[u][4 * q + 3], rm[4 * q + 2], rm[4 * q + 3], g[u]);
                        }
                    }
                    y0[u] = crcp_fast(d);  // the last step of every shift is m = 0: y_0 = 1 / d_0
                    g[u] = cmul(ia_p, y0[u]);  // (at m = 0, ia_p is the zero staged for step -1)
                }
            }
        }
    } else {
        __shared__ double2 sab[CH + 1][2];             // 1/alpha, beta/alpha of steps lo-1 .. hi
        __shared__ double2 srow[CH][4 * NPA];          // r_m on P for steps lo .. hi
        for (int hi = top - 1; hi >= 0; hi -= CH) {
            const int lo = hi - CH + 1 > 0 ? hi - CH + 1 : 0;
            const int nstep = hi - lo + 1;
            // The chunk's loads are all issued before the barrier that ends the
            // previous chunk's reads, and written to LDS after it: one memory
            // latency per chunk instead of one per staged element a thread holds.
            // UR covers the rows at 128 threads and more; a 64-thread workgroup
            // stages the rest in a plain loop.
            constexpr int UR = (CH * 4 * NPA + 127) / 128;
            const int nab = (nstep + 1) * 2, nrv = nstep * nrow;
            double2 vab = zero;  // (assigned, not selected: a select of two lvalues goes through scratch)
            if (tid < nab && lo - 1 + (tid >> 1) >= 0) vab = hab[2 * (lo - 1 + (tid >> 1)) + (tid & 1)];
            double2 vr[UR];
#pragma unroll
            for (int u = 0; u < UR; ++u) {
                const int idx = tid + u * T;
                vr[u] = zero;
                if (idx < nrv) {
                    const int sm = idx / nrow, r = idx - sm * nrow;
                    vr[u] = hr[(size_t)(lo + sm) * a.rmax + r];
                }
            }
            __syncthreads();  // the previous chunk has been consumed
            if (tid < nab) sab[tid >> 1][tid & 1] = vab;
#pragma unroll
            for (int u = 0; u < UR; ++u) {
                const int idx = tid + u * T;
                if (idx < nrv) {
                    const int sm = idx / nrow, r = idx - sm * nrow;
                    srow[sm][r] = vr[u];
                }
            }
            for (int idx = tid + UR * T; idx < nrv; idx += T) {
                const int sm = idx / nrow, r = idx - sm * nrow;
                srow[sm][r] = hr[(size_t)(lo + sm) * a.rmax + r];
            }
            __syncthreads();
            if (lo >= wtop) continue;  // nothing for this wavefront in this chunk
            for (int m = hi; m >= lo; --m) {
                // 1/alpha and beta/alpha of steps m and m - 1, read from LDS at every
                // step (carrying the step-m pair over would cost register moves)
                const double2 ia_m = sab[m - lo + 1][0], ba_m = sab[m - lo + 1][1];
                const double2 ia_p = sab[m - lo][0], ba_p = sab[m - lo][1];
                const double2 *rm = srow[m - lo];
#pragma unroll
                for (int u = 0; u < MS; ++u) {
                    if (m >= nk[u]) continue;
                    // g is exactly zero up to the shift's first step (m = N_k - 1),
                    // where this is the bare diagonal
                    const double2 d = csub(cadd(cadd(ia_m, ba_p), sigma[u]), cmul(ba_m, g[u]));
#pragma unroll
                    for (int q = 0; q < NPA; ++q) {
                        if (q < npa) {
                            cfma_rows2(S[u][4 * q], S[u][4 * q + 1], rm[4 * q], rm[4 * q + 1], g[u]);
                            cfma_rows2(S[u][4 * q + 2], S[u][4 * q + 3], rm[4 * q + 2], rm[4 * q + 3], g[u]);
                        }
                    }
                    y0[u] = crcp_fast(d);  // the last step of every shift is m = 0: y_0 = 1 / d_0
                    g[u] = cmul(ia_p, y0[u]);  // (at m = 0, ia_p is the zero staged for step -1)
                }
            }
        }
    }

    // G rows and the density matrix rho_i = -(1/pi) sum_k Im(w_k G_i(z_k))
    double2 wk[MS];
#pragma unroll
    for (int u = 0; u < MS; ++u) {
        wk[u] = zero;
        if (kof[u] >= 0 && a.w) wk[u] = a.w[kof[u]];
    }
    const int64_t out0 = a.proj_off[c];
    // the projection row of the column's own orbital (for the diagonal output)
    int rdiag = -1;
    if (a.gdiag) {  // uniform
        const int32_t pl = a.col_plan[c];
        const int64_t p0 = a.pa_off[pl];
        const int32_t cl = a.center_loc[pl];
        for (int q = 0; q < npa; ++q)
            if (a.pa_loc[p0 + q] == cl) rdiag = 4 * q + (int)(a.cols[c] & 3);
    }
#pragma unroll
    for (int r = 0; r < 4 * NPA; ++r) {
        if (r >= nrow) continue;  // uniform
        double t = 0.0;
#pragma unroll
        for (int u = 0; u < MS; ++u) {
            if (kof[u] < 0) continue;
            const double2 Gr = nk[u] > 0 ? cmul(y0[u], S[u][r]) : zero;
            if (a.G) {
                a.G[2 * ((out0 + r) * a.ns + kof[u])] = Gr.x;
                a.G[2 * ((out0 + r) * a.ns + kof[u]) + 1] = Gr.y;
            }
            if (r == rdiag) {  // uniform
                a.gdiag[2 * (c * a.ns + kof[u])] = Gr.x;
                a.gdiag[2 * (c * a.ns + kof[u]) + 1] = Gr.y;
            }
            t = fma(wk[u].x, Gr.y, fma(wk[u].y, Gr.x, t));
        }
        t = wave_reduce(t);
        if (lane == 0) rpart[r * 8 + wv] = t;
    }
    __syncthreads();
    for (int r = tid; r < nrow; r += T) {
        double acc = 0.0;
        for (int v = 0; v < nwv; ++v) acc += rpart[r * 8 + v];
        a.rho[out0 + r] = -acc * INV_PI;
    }
    if (a.eps) {  // uniform: the energy-density matrix, eps_i = -(1/pi) sum_k Im(w_k z_k G_i(z_k))
#pragma unroll
        for (int u = 0; u < MS; ++u)
            if (kof[u] >= 0) wk[u] = cmul(wk[u], a.z[kof[u]]);
        __syncthreads();  // rpart is reused
#pragma unroll
        for (int r = 0; r < 4 * NPA; ++r) {
            if (r >= nrow) continue;  // uniform
            double t = 0.0;
#pragma unroll
            for (int u = 0; u < MS; ++u) {
                if (kof[u] < 0) continue;
                const double2 Gr = nk[u] > 0 ? cmul(y0[u], S[u][r]) : zero;
                t = fma(wk[u].x, Gr.y, fma(wk[u].y, Gr.x, t));
            }
            t = wave_reduce(t);
            if (lane == 0) rpart[r * 8 + wv] = t;
        }
        __syncthreads();
        for (int r = tid; r < nrow; r += T) {
            double acc = 0.0;
            for (int v = 0; v < nwv; ++v) acc += rpart[r * 8 + v];
            a.eps[out0 + r] = -acc * INV_PI;
        }
    }
}

__global__ void k_zero_ticket(int64_t *t) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *t = 0;
}

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------
HistoryShape history_shape(const sgf_plan_totals &tot, int ns, const sgf_solve_opts &o) {
    HistoryShape h;
    h.ns_pad = (ns + 63) / 64 * 64;
    const int nl_max = 4 * (tot.max_loc_atoms > 0 ? tot.max_loc_atoms : 1);
    h.cap = o.max_iter > 0 ? o.max_iter : (o.precision == 1 ? 40 : 10) * nl_max;
    h.rmax = o.precision == 1 ? 32 : 4 * (tot.max_proj_atoms > 0 ? tot.max_proj_atoms : 1);
    h.per_col = align_up(sizeof(ColMeta), 16) + align_up((size_t)h.ns_pad * 4, 16) + (size_t)h.ns_pad * 8 +
                (size_t)h.cap * 32 + (size_t)(h.cap + 1) * h.rmax * 16;
    h.fixed = 4096 + 2 * align_up((size_t)ns * 16);
    return h;
}

SolveLayout solve_layout(const HistoryShape &hs, int ns, int64_t slots, void *base, size_t cap) {
    SolveLayout L;
    Carve c(base, cap);
    L.ticket = c.take<int64_t>(1);
    L.z = c.take<double2>(ns);
    L.w = c.take<double2>(ns);
    L.meta = c.take<ColMeta>(slots);
    L.nk = c.take<int32_t>((size_t)slots * hs.ns_pad);
    L.fz = c.take<double>((size_t)slots * hs.ns_pad);
    L.hab = c.take<double2>((size_t)slots * hs.cap * 2);
    L.hr = c.take<double2>((size_t)slots * (hs.cap + 1) * hs.rmax);
    L.slots = slots;
    L.bytes = c.used;
    return L;
}


// Events of the last profiled solve on this thread (seed start, seed end =
// shift start, shift end per batch).
struct Profile {
    std::vector<hipEvent_t> events;
    hipError_t add(hipEvent_t &e) {
        hipError_t r = hipEventCreate(&e);
        if (r == hipSuccess) events.push_back(e);
        return r;
    }
    void release() {
        for (hipEvent_t e : events) (void)hipEventDestroy(e);
        events.clear();
    }
    ~Profile() { release(); }
};
static thread_local Profile g_profile;

template <bool STAGE>
static KernelFn pick_seed_m(int M) {
    switch (M) {
        case 1: return k_seed<STAGE, 1>;
        case 2: return k_seed<STAGE, 2>;
        case 3:
        case 4: return k_seed<STAGE, 4>;
        default: return k_seed<STAGE, 8>;
    }
}

static KernelFn pick_seed(bool stage, int M) { return stage ? pick_seed_m<true>(M) : pick_seed_m<false>(M); }

template <int BMAX>
static KernelFn pick_seed_r1_m(int M) {
    switch (M) {
        case 1: return k_seed_r1<1, BMAX>;
        case 2: return k_seed_r1<2, BMAX>;
        case 3:
        case 4: return k_seed_r1<4, BMAX>;
        default: return k_seed_r1<8, BMAX>;
    }
}

static KernelFn pick_seed_r1(int M, int bmax) {
    return bmax <= 5 ? pick_seed_r1_m<5>(M) : bmax <= 6 ? pick_seed_r1_m<6>(M) : pick_seed_r1_m<8>(M);
}

// four columns per wavefront; M4 = shifts per lane (ns_pad / 16: 4 or 8)
template <int BMAX>
static KernelFn pick_seed_q4_m(int M4) { return M4 <= 4 ? k_seed_q4<4, BMAX> : k_seed_q4<8, BMAX>; }
static KernelFn pick_seed_q4(int M4, int bmax) {
    return bmax <= 5 ? pick_seed_q4_m<5>(M4) : bmax <= 6 ? pick_seed_q4_m<6>(M4) : pick_seed_q4_m<8>(M4);
}
// two columns per wavefront; M2 = shifts per lane (ns_pad / 32 rounded up to 4 or 8)
template <int BMAX>
static KernelFn pick_seed_q2_m(int M2) { return M2 <= 4 ? k_seed_q2<4, BMAX> : k_seed_q2<8, BMAX>; }
static KernelFn pick_seed_q2(int M2, int bmax) {
    return bmax <= 5 ? pick_seed_q2_m<5>(M2) : bmax <= 6 ? pick_seed_q2_m<6>(M2) : pick_seed_q2_m<8>(M2);
}

template <int BMAX, bool PACKED>
static KernelFn pick_seed_gen_m(int M) {
    switch (M) {
        case 1: return k_seed_gen<1, BMAX, PACKED>;
        case 2: return k_seed_gen<2, BMAX, PACKED>;
        case 3:
        case 4: return k_seed_gen<4, BMAX, PACKED>;
        default: return k_seed_gen<8, BMAX, PACKED>;
    }
}

template <bool PACKED>
static KernelFn pick_seed_gen_p(int M, int bmax) {
    return bmax <= 5   ? pick_seed_gen_m<5, PACKED>(M)
           : bmax <= 6 ? pick_seed_gen_m<6, PACKED>(M)
           : bmax <= 8 ? pick_seed_gen_m<8, PACKED>(M) : pick_seed_gen_m<0, PACKED>(M);
}

// BMAX = 0: rows of more than 8 blocks, read from global memory
static KernelFn pick_seed_gen(int M, int bmax, bool packed) {
    return packed ? pick_seed_gen_p<true>(M, bmax) : pick_seed_gen_p<false>(M, bmax);
}

// two wavefronts per column; M2 shifts per thread (128 threads), rows of at
// most bmax <= 8 blocks
template <int BMAX>
static KernelFn pick_seed_gen2_m(int M2) {
    switch (M2) {
        case 1: return k_seed_gen2<1, BMAX>;
        case 2: return k_seed_gen2<2, BMAX>;
        default: return k_seed_gen2<4, BMAX>;
    }
}
static KernelFn pick_seed_gen2(int M2, int bmax) {
    return bmax <= 5 ? pick_seed_gen2_m<5>(M2) : bmax <= 6 ? pick_seed_gen2_m<6>(M2) : pick_seed_gen2_m<8>(M2);
}
template <int BMAX>
static KernelFn pick_seed_gen2s_m(int M2) {
    switch (M2) {
        case 1: return k_seed_gen2s<1, BMAX>;
        case 2: return k_seed_gen2s<2, BMAX>;
        default: return k_seed_gen2s<4, BMAX>;
    }
}
static KernelFn pick_seed_gen2s(int M2, int bmax) {
    return bmax <= 5 ? pick_seed_gen2s_m<5>(M2) : bmax <= 6 ? pick_seed_gen2s_m<6>(M2) : pick_seed_gen2s_m<8>(M2);
}

template <int MS>
static KernelFn pick_shift_ms(int npa) {
    switch (npa) {
        case 1: return k_shift<1, MS>;
        case 2: return k_shift<2, MS>;
        case 3: return k_shift<3, MS>;
        case 4: return k_shift<4, MS>;
        case 5: return k_shift<5, MS>;
        case 6: return k_shift<6, MS>;
        case 7: return k_shift<7, MS>;
        default: return k_shift<8, MS>;
    }
}

// Shifts per lane: one by default (measured faster on the bundle: the extra
// registers of a second shift halve the occupancy); two on request when the
// projection rows leave room in registers.
static int shift_ms(int npa, int requested) { return requested == 2 && npa <= 5 ? 2 : 1; }

static KernelFn pick_shift(int npa, int ms) { return ms == 2 ? pick_shift_ms<2>(npa) : pick_shift_ms<1>(npa); }

}  // namespace sgf

using namespace sgf;

extern "C" sgf_status sgf_solve_workspace(const sgf_system *sys, const sgf_plan_totals *totals, int64_t n_cols,
                                          int32_t n_shifts, const sgf_solve_opts *opts, size_t *ws_bytes) {
    SGF_REQUIRE(sys && totals && opts && ws_bytes, "sgf_solve_workspace: NULL argument");
    SGF_REQUIRE(n_cols >= 0 && n_shifts >= 1, "sgf_solve_workspace: bad sizes");
    const HistoryShape hs = history_shape(*totals, n_shifts, *opts);
    int64_t slots = opts->batch_cols > 0 ? opts->batch_cols : n_cols;
    if (slots > n_cols) slots = n_cols;
    if (slots < 1) slots = 1;
    *ws_bytes = solve_layout(hs, n_shifts, slots, nullptr, 0).bytes;
    return SGF_OK;
}

// The body of sgf_shifted_solve and of its allocation-free variant: the
// workspace is the caller's (from_scratch false) or the library's static
// scratch array (from_scratch true; then profiling, which creates HIP events,
// is refused, and a workspace that cannot hold one column is an unsupported
// size rather than an invalid argument).
static sgf_status shifted_solve_in(const sgf_system *sys, const sgf_plan *plan, const sgf_plan_totals *totals,
                                   int64_t n_cols, const int64_t *d_cols, const int32_t *d_col_plan,
                                   const int32_t *d_order, int32_t n_shifts, const double *z, const double *w,
                                   const sgf_solve_opts *opts, void *d_ws, size_t ws_bytes,
                                   const int64_t *d_proj_off, double *d_G, double *d_rho, int32_t *d_iters,
                                   int32_t *d_status, double *d_resid, int32_t *d_shift_iters, void *stream,
                                   bool from_scratch) {
    SGF_REQUIRE(sys && plan && totals && opts, "sgf_shifted_solve: NULL system, plan, totals or options");
    SGF_REQUIRE(sys->row_ptr && sys->col && sys->h && sys->n_atoms > 0, "sgf_shifted_solve: system incomplete");
    SGF_REQUIRE(plan->atom_off && plan->blk_off && plan->pa_off && plan->loc_atom && plan->lrow && plan->lblk &&
                    plan->pa_loc && plan->center_loc,
                "sgf_shifted_solve: plan has not been built");
    SGF_REQUIRE(n_cols >= 0, "sgf_shifted_solve: n_cols < 0");
    SGF_REQUIRE(opts->queue_len >= 0 && opts->queue_len <= n_cols && (opts->queue_len == 0 || d_order),
                "sgf_shifted_solve: queue_len must be in [0, n_cols] and needs d_order");
    // columns taken from the work queue: d_order[0 .. n_tickets)
    const int64_t n_tickets = opts->queue_len > 0 ? opts->queue_len : n_cols;
    SGF_REQUIRE(n_cols == 0 || (d_cols && d_col_plan && d_proj_off && d_rho && d_iters && d_status),
                "sgf_shifted_solve: NULL column or output array");
    SGF_REQUIRE(n_shifts >= 1, "sgf_shifted_solve: n_shifts must be >= 1");
    SGF_REQUIRE(z, "sgf_shifted_solve: z is NULL");
    SGF_REQUIRE(opts->tol > 0, "sgf_shifted_solve: tol must be positive");
    SGF_REQUIRE(opts->precision == 0 || opts->precision == 1, "sgf_shifted_solve: precision must be 0 or 1");
    if (opts->eps_out && opts->precision != 0) {
        set_error("sgf_shifted_solve: the energy-density output is formed by the FP64 shift pass only");
        return SGF_EUNSUPPORTED;
    }
    SGF_REQUIRE(!opts->eps_out || w, "sgf_shifted_solve: the energy-density output needs the weights w");
    SGF_REQUIRE(opts->max_iter >= 0, "sgf_shifted_solve: max_iter must be >= 0");
    int seed = opts->seed_index < 0 ? n_shifts / 2 : opts->seed_index;
    if (opts->seed_index == -2) {  // the shift nearest the real axis
        for (int kk = 0; kk < n_shifts; ++kk) {
            const double a = z[2 * kk + 1], b = z[2 * seed + 1];
            if (a < b || (a == b && std::abs(kk - n_shifts / 2) < std::abs(seed - n_shifts / 2))) seed = kk;
        }
    }
    SGF_REQUIRE(seed < n_shifts, "sgf_shifted_solve: seed_index %d >= n_shifts %d", seed, n_shifts);
    for (int kk = 0; kk < n_shifts; ++kk)
        SGF_REQUIRE(z[2 * kk + 1] > 0, "sgf_shifted_solve: Im z[%d] = %g is not positive", kk, z[2 * kk + 1]);
    if (n_shifts > 512) {
        set_error("sgf_shifted_solve: %d shifts (limit 512)", n_shifts);
        return SGF_EUNSUPPORTED;
    }
    if (totals->max_proj_atoms > 8) {
        set_error("sgf_shifted_solve: a column has %d projection atoms (limit 8)", totals->max_proj_atoms);
        return SGF_EUNSUPPORTED;
    }
    const bool mixed = opts->precision == 1;
    if (mixed) {
        if (sys->s) {
            set_error("sgf_shifted_solve: the mixed-precision path supports S = I only");
            return SGF_EUNSUPPORTED;
        }
        if (totals->max_loc_atoms > 16 || totals->max_row_blocks > 8) {
            set_error("sgf_shifted_solve: the mixed-precision path needs local subspaces of <= 16 atoms with "
                      "<= 8 blocks per row (got %d atoms, %d blocks)", totals->max_loc_atoms,
                      totals->max_row_blocks);
            return SGF_EUNSUPPORTED;
        }
        if (n_shifts > 256) {
            set_error("sgf_shifted_solve: the mixed-precision path takes at most 256 shifts (got %d)", n_shifts);
            return SGF_EUNSUPPORTED;
        }
        SGF_REQUIRE(sys->h32, "sgf_shifted_solve: the mixed-precision path needs the FP32 shadow h32 (sgf_to_f32)");
        SGF_REQUIRE(opts->drift_tol >= 0 && opts->g_tol >= 0, "sgf_shifted_solve: drift_tol and g_tol must be >= 0");
        SGF_REQUIRE(opts->monitor_every >= 0, "sgf_shifted_solve: monitor_every must be >= 0");
    }
    SGF_REQUIRE(d_ws, "sgf_shifted_solve: workspace is NULL");
    const HistoryShape hs = history_shape(*totals, n_shifts, *opts);
    const SolveLayout L1 = solve_layout(hs, n_shifts, 1, nullptr, 0);
    if (from_scratch) {
        SGF_REQUIRE(!opts->profile, "sgf_shifted_solve_static: profile = 1 records HIP events, which this entry "
                                    "point does not create");
        if (L1.bytes > ws_bytes) {
            set_error("sgf_shifted_solve_static: one column of this solve needs %zu bytes of history (max_iter "
                      "%d, %d shifts), more than the %zu-byte static scratch; use sgf_shifted_solve with a "
                      "workspace", L1.bytes, hs.cap, n_shifts, ws_bytes);
            return SGF_EUNSUPPORTED;
        }
    }
    SGF_REQUIRE(L1.bytes <= ws_bytes, "sgf_shifted_solve: workspace %zu bytes < %zu (one column)", ws_bytes, L1.bytes);
    if (n_cols == 0) return SGF_OK;
    // columns per launch: batch_cols (0: all), at most as many history slots
    // as the workspace holds (the largest count whose layout fits)
    int64_t slots = opts->batch_cols > 0 && opts->batch_cols < n_tickets ? opts->batch_cols : n_tickets;
    if (solve_layout(hs, n_shifts, slots, nullptr, 0).bytes > ws_bytes) {
        int64_t lo = 1, hi = slots;  // layout(lo) fits, layout(hi) does not
        while (hi - lo > 1) {
            const int64_t mid = lo + (hi - lo) / 2;
            (solve_layout(hs, n_shifts, mid, nullptr, 0).bytes <= ws_bytes ? lo : hi) = mid;
        }
        slots = lo;
    }
    SolveLayout L = solve_layout(hs, n_shifts, slots, d_ws, ws_bytes);
    hipStream_t st = as_stream(stream);
    if (!opts->shifts_staged) {
        SGF_HIP(hipMemcpyAsync(L.z, z, 16 * (size_t)n_shifts, hipMemcpyHostToDevice, st));
        if (w) SGF_HIP(hipMemcpyAsync(L.w, w, 16 * (size_t)n_shifts, hipMemcpyHostToDevice, st));
    }

    SolveArgs a{};
    a.row_ptr = sys->row_ptr;
    a.col = sys->col;
    a.h = sys->h;
    a.s = sys->s;
    a.h32 = sys->h32;
    a.atom_off = plan->atom_off;
    a.blk_off = plan->blk_off;
    a.pa_off = plan->pa_off;
    a.loc_atom = plan->loc_atom;
    a.lrow = plan->lrow;
    a.lblk = plan->lblk;
    a.pa_loc = plan->pa_loc;
    a.center_loc = plan->center_loc;
    a.n_plans = plan->n_plans;
    a.max_loc_atoms = totals->max_loc_atoms;
    a.max_loc_blocks = totals->max_loc_blocks;
    a.npa_max = totals->max_proj_atoms;
    a.n_cols = n_cols;
    a.cols = d_cols;
    a.col_plan = d_col_plan;
    a.order = d_order;
    a.ns = n_shifts;
    a.ns_pad = hs.ns_pad;
    a.seed = seed;
    a.z = L.z;
    a.w = w ? L.w : nullptr;
    a.tol = opts->tol;
    a.max_iter = opts->max_iter;
    a.monitor_every = opts->monitor_every;
    a.drift_tol = opts->drift_tol > 0 ? opts->drift_tol : 1e-3;
    a.g_tol = opts->g_tol > 0 ? opts->g_tol : 5e-7;
    a.proj_off = d_proj_off;
    a.G = d_G;
    a.rho = d_rho;
    a.eps = opts->eps_out;
    a.gdiag = opts->g_diag_out;
    a.resid = d_resid;
    a.iters = d_iters;
    a.status = d_status;
    a.shift_iters = d_shift_iters;
    a.cap = hs.cap;
    a.rmax = hs.rmax;
    a.meta = L.meta;
    a.nk = L.nk;
    a.fz = L.fz;
    a.hab = L.hab;
    a.hr = L.hr;
    a.ticket = L.ticket;

    // seed-pass LDS: p, s, w vectors and (optionally) the staged local operator
    const int nl = 4 * (totals->max_loc_atoms > 0 ? totals->max_loc_atoms : 1);
    const int blk = totals->max_loc_blocks > 0 ? totals->max_loc_blocks : 1;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t r = off; off = align_up(off + bytes, 16); return r; };
    a.off_p = take((size_t)nl * 16);
    a.off_s = take((size_t)nl * 16);
    a.off_w = take((size_t)nl * 16);
    const size_t lds_plain = off;
    a.off_hs = take((size_t)blk * 128);
    a.off_cs = take((size_t)blk * 4);
    a.off_rs = take((size_t)(totals->max_loc_atoms + 1) * 4);
    const size_t lds_staged = off;
    const bool stage = opts->stage_lds == 1 || (opts->stage_lds < 0 && lds_staged <= 16 * 1024);
    const size_t lds = stage ? lds_staged : lds_plain;
    if (lds > 160 * 1024 && !sys->s) {
        set_error("sgf_shifted_solve: a local subspace of %d atoms needs %zu bytes of LDS (limit 163840)",
                  totals->max_loc_atoms, lds);
        return SGF_EUNSUPPORTED;
    }
    const int M = hs.ns_pad / 64;
    // register variant when every subspace has <= 64 orbitals and <= 8 blocks per row
    const bool gen = sys->s != nullptr;
    const bool r1 = !gen && (opts->stage_lds < 0 || opts->stage_lds == 3 || opts->stage_lds == 5) &&
                    totals->max_loc_atoms <= 16 && totals->max_row_blocks <= 8;
    // columns of a plan per wavefront: four at up to 128 shifts, two at up to
    // 256 (eight shifts per lane either way); stage_lds 5 takes two at any
    // shift count up to 256
    const int cpw = (!r1 || mixed || (opts->stage_lds >= 0 && opts->stage_lds != 5) || hs.ns_pad > 256)
                        ? 0
                        : (opts->stage_lds == 5 || hs.ns_pad > 128) ? 2 : 4;
    const bool q4 = cpw == 4, q2 = cpw == 2;
    // S != I, dense-LDS variant.  stage_lds < 0: subspaces of up to 16 atoms
    // in a launch of their own with the dense inverse, the larger ones in a
    // second launch with the packed triangle (half the LDS, so twice the
    // wavefronts per compute unit).  stage_lds = 0: one launch, dense;
    // stage_lds = 1: one launch, packed.
    // stage_lds = 2: the same split, with one wavefront per column in the
    // second launch too.  Otherwise the second launch (17 to 32 atoms, rows of
    // at most 8 blocks) runs two wavefronts per column (k_seed_gen2).
    // S != I with every block of S a multiple of I4: the per-atom overlap
    // inverse, one wavefront per column (a second launch for 17 to 32 atoms,
    // two rows per lane; stage_lds 4: two wavefronts per column there)
    const bool kron = gen && sys->s_orbital_diagonal == 1 && !mixed &&
                      (opts->stage_lds < 0 || opts->stage_lds == 4) && hs.ns_pad <= 256 &&
                      totals->max_loc_atoms <= 32 && totals->max_row_blocks <= 8;
    const bool kron_split = kron && totals->max_loc_atoms > 16;
    const bool kron_two_waves = kron_split && opts->stage_lds < 0;
    const bool gen_split = gen && !kron && !mixed && (opts->stage_lds < 0 || opts->stage_lds == 2) &&
                           totals->max_loc_atoms > 16;
    const bool gen2 = gen_split && opts->stage_lds < 0 && totals->max_loc_atoms <= 32 && totals->max_row_blocks <= 8;
    // every subspace of at most 16 atoms: one launch of the two-wavefront
    // dense kernel of the small class
    const bool gen2_one = gen && !kron && !mixed && opts->stage_lds < 0 && !gen_split &&
                          totals->max_loc_atoms <= 16 && totals->max_row_blocks <= 8;
    const bool gen_packed = gen_split || (gen && opts->stage_lds == 1);
    KernelFn seed_fn = mixed ? pick_seed_mx(M, totals->max_row_blocks)
                       : kron ? (kron_two_waves ? pick_seed_kron2((hs.ns_pad + 127) / 128, totals->max_row_blocks)
                                                : pick_seed_kron(kron_split ? 2 : 1, M, totals->max_row_blocks))
                       : gen2 ? pick_seed_gen2((hs.ns_pad + GEN2_T - 1) / GEN2_T, totals->max_row_blocks)
                       : gen2_one ? pick_seed_gen2s((hs.ns_pad + GEN2_T - 1) / GEN2_T, totals->max_row_blocks)
                       : gen ? pick_seed_gen(M, totals->max_row_blocks, gen_packed)
                             : q4 ? pick_seed_q4(hs.ns_pad / 16, totals->max_row_blocks)
                             : q2 ? pick_seed_q2((hs.ns_pad + 31) / 32, totals->max_row_blocks)
                             : (r1 ? pick_seed_r1(M, totals->max_row_blocks) : pick_seed(stage, M));
    const int seed_threads = (gen2 || gen2_one || kron_two_waves) ? GEN2_T : SEED_T;
    size_t seed_lds = (r1 || mixed || kron) ? 0 : lds;
    // S != I: p, s, w, q, r and the dense inverse of the local overlap, laid
    // out for subspaces of up to nlx orbitals
    auto gen_layout = [](SolveArgs &g, int nlx, bool packed) {
        size_t goff = 0;
        auto gtake = [&](size_t bytes) { size_t r = goff; goff = align_up(goff + bytes, 16); return r; };
        g.off_p = gtake((size_t)nlx * 16);
        g.off_s = gtake((size_t)nlx * 16);
        g.off_w = gtake((size_t)nlx * 16);
        g.off_q = gtake((size_t)nlx * 16);
        g.off_r = gtake((size_t)nlx * 16);
        g.off_sinv = gtake(packed ? (size_t)tri(nlx) * 8 : (size_t)nlx * sinv_ld(nlx) * 8);
        return goff;
    };
    // the launch for subspaces of up to 16 atoms (gen_split)
    SolveArgs a_small{};
    // with gen2, the small class also runs two wavefronts per column (each
    // row's product split between them by column halves)
    KernelFn seed_fn_small = kron_split ? pick_seed_kron(1, M, totals->max_row_blocks)
                             : !gen_split ? nullptr
                             : gen2    ? pick_seed_gen2s((hs.ns_pad + GEN2_T - 1) / GEN2_T, totals->max_row_blocks)
                                       : pick_seed_gen(M, totals->max_row_blocks, false);
    const int small_threads = gen2 ? GEN2_T : SEED_T;
    size_t lds_small = 0;
    if (gen && !kron && !mixed) {
        seed_lds = gen_layout(a, nl, gen_packed);
        if (seed_lds > 160 * 1024) {
            set_error("sgf_shifted_solve: S != I with a local subspace of %d orbitals needs %zu bytes of LDS "
                      "for the dense local overlap inverse (limit 163840); prune the subspaces or reduce the radius",
                      nl, seed_lds);
            return SGF_EUNSUPPORTED;
        }
    }
    if (gen_split) {
        a.loc_lo = 17;
        a.loc_hi = totals->max_loc_atoms;
    }
    if (gen2_one) {
        a.loc_lo = 0;
        a.loc_hi = 16;
    }
    if (kron) {  // loc_hi: the largest subspace that this solve's launches take
        a.loc_lo = 0;
        a.loc_hi = kron_split ? 32 : 16;
    }
    const int ms = mixed ? 1 : shift_ms(totals->max_proj_atoms, opts->shifts_per_lane);
    KernelFn shift_fn = mixed ? shift_mx_kernel() : pick_shift(totals->max_proj_atoms, ms);
    // shift-pass workgroup: ns_pad / ms lanes rounded up to whole wavefronts (<= 512)
    const int shift_threads = ((hs.ns_pad / ms + 63) / 64) * 64;
    // mixed: the full iterates of every shift, complex FP32 [64][ns_pad]
    // per-wavefront history staging of the FP64 shift pass (up to five
    // projection atoms, not four): a chunk of SHIFT_CH steps per wavefront
    const int npa_t = totals->max_proj_atoms < 1 ? 1 : (totals->max_proj_atoms > 8 ? 8 : totals->max_proj_atoms);
    const bool shift_pwv = npa_t <= 5 && npa_t != 4;
    const size_t shift_lds = mixed       ? (size_t)64 * hs.ns_pad * 8
                             : shift_pwv ? (size_t)(shift_threads / 64) * ((SHIFT_CH + 1) * 2 + SHIFT_CH * 4 * npa_t) * 16
                                         : 0;
    SGF_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(shift_fn),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)shift_lds));
    SGF_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(seed_fn), hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)seed_lds));
    int per_cu = 0;
    SGF_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(seed_fn),
                                                         seed_threads, seed_lds));
    if (per_cu < 1) {
        set_error("sgf_shifted_solve: seed kernel does not fit a compute unit (LDS %zu)", lds);
        return SGF_EUNSUPPORTED;
    }
    int dev = 0, n_cu = 0;
    SGF_HIP(hipGetDevice(&dev));
    SGF_HIP(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
    const int64_t seed_grid_max = opts->grid > 0 ? opts->grid : (int64_t)per_cu * n_cu;
    int64_t seed_grid_small = 0;
    if (gen_split || kron_split) {
        a_small = a;
        lds_small = kron_split ? 0 : gen_layout(a_small, 64, false);
        a_small.loc_lo = 0;
        a_small.loc_hi = kron_split ? 32 : 16;
        int per_cu_s = 0;
        SGF_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(seed_fn_small),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_small));
        SGF_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu_s, reinterpret_cast<const void *>(seed_fn_small),
                                                             small_threads, lds_small));
        if (per_cu_s < 1) {
            set_error("sgf_shifted_solve: seed kernel does not fit a compute unit (LDS %zu)", lds_small);
            return SGF_EUNSUPPORTED;
        }
        seed_grid_small = opts->grid > 0 ? opts->grid : (int64_t)per_cu_s * n_cu;
    }

    Profile &prof = g_profile;
    const bool timed = opts->profile != 0;
    if (timed) prof.release();  // an unprofiled solve leaves the last profiled one readable
    for (int64_t b0 = 0; b0 < n_tickets; b0 += slots) {
        const int64_t b1 = b0 + slots < n_tickets ? b0 + slots : n_tickets;
        a.batch_begin = b0;
        a.batch_end = b1;
        const int64_t n_tk = cpw ? (b1 - b0 + cpw - 1) / cpw : b1 - b0;  // work-queue tickets of this batch
        const int64_t grid = seed_grid_max < n_tk ? seed_grid_max : n_tk;
        k_zero_ticket<<<1, 64, 0, st>>>(L.ticket);
        SGF_LAUNCHED();
        hipEvent_t e0 = nullptr, e1 = nullptr, e2 = nullptr;
        if (timed) {
            SGF_HIP(prof.add(e0));
            SGF_HIP(prof.add(e1));
            SGF_HIP(prof.add(e2));
            SGF_HIP(hipEventRecord(e0, st));
        }
        if (gen_split || kron_split) {
            // subspaces of up to 16 atoms first, then the same tickets again
            // for the larger ones
            a_small.batch_begin = b0;
            a_small.batch_end = b1;
            const int64_t gs = seed_grid_small < b1 - b0 ? seed_grid_small : b1 - b0;
            hipLaunchKernelGGL(seed_fn_small, dim3((unsigned)gs), dim3(small_threads), lds_small, st, a_small);
            SGF_LAUNCHED();
            k_zero_ticket<<<1, 64, 0, st>>>(L.ticket);
            SGF_LAUNCHED();
        }
        hipLaunchKernelGGL(seed_fn, dim3((unsigned)grid), dim3(seed_threads), seed_lds, st, a);
        SGF_LAUNCHED();
        if (timed) SGF_HIP(hipEventRecord(e1, st));
        hipLaunchKernelGGL(shift_fn, dim3((unsigned)(b1 - b0)), dim3(shift_threads), shift_lds, st, a);
        SGF_LAUNCHED();
        if (timed) SGF_HIP(hipEventRecord(e2, st));
    }
    return SGF_OK;
}

extern "C" sgf_status sgf_shifted_solve(const sgf_system *sys, const sgf_plan *plan, const sgf_plan_totals *totals,
                                        int64_t n_cols, const int64_t *d_cols, const int32_t *d_col_plan,
                                        const int32_t *d_order, int32_t n_shifts, const double *z, const double *w,
                                        const sgf_solve_opts *opts, void *d_ws, size_t ws_bytes,
                                        const int64_t *d_proj_off, double *d_G, double *d_rho, int32_t *d_iters,
                                        int32_t *d_status, double *d_resid, int32_t *d_shift_iters,
                                        void *stream) {
    return shifted_solve_in(sys, plan, totals, n_cols, d_cols, d_col_plan, d_order, n_shifts, z, w, opts, d_ws,
                            ws_bytes, d_proj_off, d_G, d_rho, d_iters, d_status, d_resid, d_shift_iters, stream,
                            false);
}

// ---------------------------------------------------------------------------
// Allocation-free solve: the workspace is a static device array of the
// library.  Each GPU the library runs on holds its own copy from the moment
// the code object is loaded there until the process ends.  In host code the
// array's name stands for a host-side shadow, not for device memory, so its
// device address is looked up once per device (with that device current) and
// only that address is ever handed to kernels or copies.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[SGF_STATIC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

static sgf_status scratch_address(void **out) {
    int dev = 0;
    SGF_HIP(hipGetDevice(&dev));
    SGF_REQUIRE(dev >= 0 && dev < kMaxDevices, "sgf_shifted_solve_static: device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        SGF_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        SGF_REQUIRE(p, "sgf_shifted_solve_static: no device address for the static scratch on device %d", dev);
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return SGF_OK;
}

extern "C" sgf_status sgf_shifted_solve_static(const sgf_system *sys, const sgf_plan *plan,
                                               const sgf_plan_totals *totals, int64_t n_cols, const int64_t *d_cols,
                                               const int32_t *d_col_plan, const int32_t *d_order, int32_t n_shifts,
                                               const double *z, const double *w, const sgf_solve_opts *opts,
                                               const int64_t *d_proj_off, double *d_G, double *d_rho,
                                               int32_t *d_iters, int32_t *d_status, double *d_resid,
                                               int32_t *d_shift_iters, void *stream) {
    void *ws = nullptr;
    const sgf_status r = scratch_address(&ws);
    if (r != SGF_OK) return r;
    return shifted_solve_in(sys, plan, totals, n_cols, d_cols, d_col_plan, d_order, n_shifts, z, w, opts, ws,
                            SGF_STATIC_SCRATCH_BYTES, d_proj_off, d_G, d_rho, d_iters, d_status, d_resid,
                            d_shift_iters, stream, true);
}

extern "C" sgf_status sgf_solve_stage_shifts(int32_t n_shifts, const double *z, const double *w, void *d_ws,
                                              size_t ws_bytes, void *stream) {
    SGF_REQUIRE(n_shifts >= 1 && n_shifts <= 512 && z && d_ws, "sgf_solve_stage_shifts: bad arguments");
    // z and w sit at the start of the workspace, before any per-column slot,
    // so their place depends on n_shifts only
    HistoryShape hs{};
    hs.cap = 1;
    hs.rmax = 1;
    hs.ns_pad = (n_shifts + 63) / 64 * 64;
    const SolveLayout L0 = solve_layout(hs, n_shifts, 0, nullptr, 0);
    SGF_REQUIRE(L0.bytes <= ws_bytes, "sgf_solve_stage_shifts: workspace too small");
    const SolveLayout L = solve_layout(hs, n_shifts, 0, d_ws, ws_bytes);
    hipStream_t st = as_stream(stream);
    SGF_HIP(hipMemcpyAsync(L.z, z, 16 * (size_t)n_shifts, hipMemcpyHostToDevice, st));
    if (w) SGF_HIP(hipMemcpyAsync(L.w, w, 16 * (size_t)n_shifts, hipMemcpyHostToDevice, st));
    return SGF_OK;
}

extern "C" sgf_status sgf_solve_profile(double *seed_ms, double *shift_ms, int32_t *batches) {
    SGF_REQUIRE(seed_ms && shift_ms && batches, "sgf_solve_profile: NULL argument");
    Profile &prof = g_profile;
    SGF_REQUIRE(!prof.events.empty(), "sgf_solve_profile: no profiled solve is pending on this thread");
    double t_seed = 0.0, t_shift = 0.0;
    for (size_t i = 0; i + 2 < prof.events.size(); i += 3) {
        float a = 0.f, b = 0.f;
        SGF_HIP(hipEventSynchronize(prof.events[i + 2]));
        SGF_HIP(hipEventElapsedTime(&a, prof.events[i], prof.events[i + 1]));
        SGF_HIP(hipEventElapsedTime(&b, prof.events[i + 1], prof.events[i + 2]));
        t_seed += a;
        t_shift += b;
    }
    *seed_ms = t_seed;
    *shift_ms = t_shift;
    *batches = (int32_t)(prof.events.size() / 3);
    prof.release();
    return SGF_OK;
}
