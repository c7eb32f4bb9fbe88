// seed_kron.hip -- seed pass of the generalized shifted equations
// (z S - H) x = e_j (Introduction) for an overlap whose blocks are multiples
// of the 4 x 4 identity: S_ab = s_ab I4, as in the orbital-diagonal overlap
// model of the builder.  The local overlap is then S_L = S_a (x) I4 with
// S_a the n x n matrix of the numbers s_ab over the subspace's n atoms, and
// S_L^{-1} = S_a^{-1} (x) I4: the inverse is formed per atom pair (n^3
// instead of (4n)^3 flops, n^2 doubles of LDS instead of 16 n^2) and the
// product r = S_L^{-1} s costs n multiply-adds per orbital row instead of 4n.
//
// COCG in the S-bilinear form, as in the general S != I seed passes: s is the
// residual, r = S^{-1} s, q = S p (kept by its recurrence q <- s + beta q,
// since S r = s), w = z_s q - H p, mu = p^T w, rho = r^T s; the history holds
// 1/alpha, beta/alpha and r on the projection rows.
//
// k_seed_kr: one wavefront per column, persistent over an atomic ticket
// queue.  Lane l owns orbital rows l + 64 i, i < R: R = 1 takes the
// subspaces of at most 16 atoms, R = 2 is the one-wavefront choice for those
// of 17 to 32 (by default k_seed_kr2 below runs them on two wavefronts, a
// row per thread).
// Each row's blocks of H stay in registers; p and s sit in LDS orbital-major
// (row o of atom A at [KP o + A]), S_a^{-1} row-major with an odd stride, so
// that the lanes of different atoms read different banks and the four lanes
// of one atom read one address.
#include "scocg.hpp"

namespace sgf {
namespace {

template <int R, int M, int BMAX>
__global__ __launch_bounds__(SEED_T) void k_seed_kr(SolveArgs a) {
    constexpr int NA = 16 * R;  // atoms a subspace of this class may have
    constexpr int KP = NA + 1;  // LDS row stride
    __shared__ double2 vp[4 * KP];
    __shared__ double2 vs[4 * KP];
    __shared__ double si[NA * KP];
    __shared__ __align__(16) double red_mu[2 * 64], red_s[3 * 64];
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
            if (R == 1 && lane == 0) *meta = ColMeta{-1, 0, 0, SGF_BADCOLUMN};
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
            bad = n_loc < 1 || npa < 1 || 4 * npa > a.rmax || cl < 0 || cl >= n_loc ||
                  a.loc_atom[a0 + cl] != (int32_t)(j >> 2);
        }
        // R = 1 takes (and reports) the columns that cannot be solved and the
        // subspaces of up to 16 atoms, R = 2 the larger ones; with no R = 2
        // launch to follow (loc_hi <= 16) R = 1 takes every column.  A
        // subspace beyond a launch's NA atoms is reported as unsolvable.
        const bool take = R == 1 ? (bad || n_loc <= 16 || a.loc_hi <= 16) : (!bad && n_loc > 16);
        if (!take) continue;
        bad = bad || n_loc > NA;
        const int nl = 4 * n_loc;

        // this lane's rows: blocks per row and the first block
        int t0[R], nb[R];
        bool rowv[R];
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const int row = lane + 64 * i, A = row >> 2;
            rowv[i] = !bad && row < nl;
            t0[i] = 0;
            nb[i] = 0;
            if (rowv[i]) {
                t0[i] = a.lrow[a0 + A];
                nb[i] = (A + 1 < n_loc ? a.lrow[a0 + A + 1] : nblk) - t0[i];
            }
            bad = bad || nb[i] > BMAX;
        }
        // S_a from the blocks of S: lane A < n_loc reads its atom's row and
        // checks that each block is s_ab I4
        wave_lds_fence();  // the previous column's LDS reads are done
        for (int e = lane; e < NA * KP; e += 64) si[e] = 0.0;
        for (int e = lane; e < 4 * KP; e += 64) {
            vp[e] = zero;
            vs[e] = zero;
        }
        wave_lds_fence();
        bool notk = false;
        if (!bad && lane < n_loc) {
            const int u0 = a.lrow[a0 + lane], u1 = lane + 1 < n_loc ? a.lrow[a0 + lane + 1] : nblk;
            for (int t = u0; t < u1; ++t) {
                const int B = a.lblk[2 * (b0 + t)];
                if (B < 0 || B >= n_loc) {
                    notk = true;
                    break;
                }
                const double *sb = &a.s[16 * (int64_t)a.lblk[2 * (b0 + t) + 1]];
                const double d = sb[0];
                bool ok = sb[5] == d && sb[10] == d && sb[15] == d;
#pragma unroll
                for (int e = 1; e < 15; ++e)
                    if (e % 5 != 0) ok = ok && sb[e] == 0.0;
                notk = notk || !ok;
                si[KP * lane + B] = d;
            }
        }
        bad = __any(bad || notk);
        if (bad) {
            if (lane == 0) {
                *meta = ColMeta{-1, 0, 0, SGF_BADCOLUMN};
                a.iters[c] = 0;
                a.status[c] = SGF_BADCOLUMN;
            }
            continue;
        }
        int bcol[R][BMAX];
        double hrow[R][BMAX][4];
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const int o = (lane + 64 * i) & 3;
#pragma unroll
            for (int b = 0; b < BMAX; ++b) {
                bcol[i][b] = 0;
                hrow[i][b][0] = hrow[i][b][1] = hrow[i][b][2] = hrow[i][b][3] = 0.0;
                if (b < nb[i]) {
                    const int32_t *lb = &a.lblk[2 * (b0 + t0[i] + b)];
                    bcol[i][b] = lb[0];
                    const double *hb = &a.h[16 * (int64_t)lb[1] + 4 * o];
#pragma unroll
                    for (int q = 0; q < 4; ++q) hrow[i][b][q] = hb[q];
                }
            }
        }
        wave_lds_fence();  // S_a is complete

        // S_a^{-1} in place: Gauss-Jordan elimination without pivoting (S_a
        // is positive definite); lane l updates row l
        for (int kk = 0; kk < n_loc; ++kk) {
            const double piv = 1.0 / si[KP * kk + kk];
            const double f = (lane < n_loc && lane != kk) ? si[KP * lane + kk] : 0.0;
            wave_lds_fence();
            if (lane < n_loc) si[KP * kk + lane] = lane == kk ? piv : si[KP * kk + lane] * piv;
            wave_lds_fence();
            if (lane < n_loc && lane != kk) {
                for (int jj = 0; jj < n_loc; ++jj) si[KP * lane + jj] = fma(-f, si[KP * kk + jj], si[KP * lane + jj]);
                si[KP * lane + kk] = -f * piv;
            }
            wave_lds_fence();
        }

        const int jA = cl, jo = (int)(j & 3);
        const int n4 = (n_loc + 3) & ~3;  // product length, zero-padded
        int pidx[R];
#pragma unroll
        for (int i = 0; i < R; ++i) {
            pidx[i] = -1;
            const int row = lane + 64 * i;
            for (int q = 0; q < npa; ++q)
                if (rowv[i] && a.pa_loc[p0 + q] == (row >> 2)) pidx[i] = 4 * q + (row & 3);
        }
        double2 *hab = a.hab + (size_t)slot * a.cap * 2;
        double2 *hr = a.hr + (size_t)slot * (a.cap + 1) * a.rmax;

        // start: x = 0, s_0 = q_0 = e_j, r_0 = p_0 = S^{-1} e_j,
        // rho_0 = r_0^T s_0 = (S_a^{-1})_{jA jA}
        double2 s[R], p[R], q[R];
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const int row = lane + 64 * i, A = row >> 2, o = row & 3;
            s[i] = (rowv[i] && A == jA && o == jo) ? one : zero;
            q[i] = s[i];
            p[i] = (rowv[i] && o == jo) ? make_double2(si[KP * A + jA], 0.0) : zero;
            vp[KP * o + A] = p[i];
            if (pidx[i] >= 0) hr[pidx[i]] = p[i];
        }
        double2 rho = make_double2(si[KP * jA + jA], 0.0);
        double2 inv_rho = crcp(rho);
        wave_lds_fence();

        double2 pc[M], po[M];
        uint32_t act = 0;
#pragma unroll
        for (int m = 0; m < M; ++m) {
            pc[m] = po[m] = one;
            if (lane + 64 * m < a.ns) act |= 1u << m;
        }
        double2 ba_old = zero;  // beta_{n-1} / alpha_{n-1}
        int status = SGF_MAXITER, iters = 0, applied = 0;
        double snorm2 = 1.0;
        const int max_iter = a.max_iter > 0 ? a.max_iter : 10 * nl;

        for (int it = 0; it < max_iter; ++it) {
            // w = z_s q - H p ; mu = p^T w (absent blocks hold zeros and point
            // at atom 0, so every lane runs the same instructions)
            double2 w[R];
            double mp[2] = {0.0, 0.0};
#pragma unroll
            for (int i = 0; i < R; ++i) {
                double ax = 0.0, ay = 0.0;
#pragma unroll
                for (int b = 0; b < BMAX; ++b) {
#pragma unroll
                    for (int qq = 0; qq < 4; ++qq) {
                        const double2 pv = vp[KP * qq + bcol[i][b]];
                        ax = fma(hrow[i][b][qq], pv.x, ax);
                        ay = fma(hrow[i][b][qq], pv.y, ay);
                    }
                }
                w[i] = make_double2(zs.x * q[i].x - zs.y * q[i].y - ax, zs.x * q[i].y + zs.y * q[i].x - ay);
                mp[0] = fma(p[i].x, w[i].x, fma(-p[i].y, w[i].y, mp[0]));
                mp[1] = fma(p[i].x, w[i].y, fma(p[i].y, w[i].x, mp[1]));
            }
            double2 mu;
            {
                double sum[2];
                wave_sum_lds<2>(mp, red_mu, sum);
                mu = make_double2(sum[0], sum[1]);
            }
            iters = it + 1;
            if (!cfinite(mu)) { status = SGF_NONFINITE; break; }
            if (mu.x == 0.0 && mu.y == 0.0) { status = SGF_BREAKDOWN; break; }
            const double2 alpha = cmul(rho, crcp(mu));
            const double2 ia = cmul(mu, inv_rho);  // 1/alpha

            // s -= alpha w, then r = S^{-1} s row by row
#pragma unroll
            for (int i = 0; i < R; ++i) {
                const int row = lane + 64 * i;
                s[i] = csub(s[i], cmul(alpha, w[i]));
                vs[KP * (row & 3) + (row >> 2)] = s[i];
            }
            wave_lds_fence();
            double2 r[R];
            double rs[3] = {0.0, 0.0, 0.0};
#pragma unroll
            for (int i = 0; i < R; ++i) {
                const int row = lane + 64 * i;
                const double *srow = &si[KP * (row >> 2)];
                const double2 *scol = &vs[KP * (row & 3)];
                double ax[4] = {0.0, 0.0, 0.0, 0.0}, ay[4] = {0.0, 0.0, 0.0, 0.0};
                for (int B = 0; B < n4; B += 4) {
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const double av = srow[B + u];
                        const double2 sv = scol[B + u];
                        ax[u] = fma(av, sv.x, ax[u]);
                        ay[u] = fma(av, sv.y, ay[u]);
                    }
                }
                r[i] = make_double2((ax[0] + ax[1]) + (ax[2] + ax[3]), (ay[0] + ay[1]) + (ay[2] + ay[3]));
                rs[0] = fma(r[i].x, s[i].x, fma(-r[i].y, s[i].y, rs[0]));
                rs[1] = fma(r[i].x, s[i].y, fma(r[i].y, s[i].x, rs[1]));
                rs[2] = fma(s[i].x, s[i].x, fma(s[i].y, s[i].y, rs[2]));
            }
            double2 rho_new;
            {
                double sum[3];
                wave_sum_lds<3>(rs, red_s, sum);
                rho_new = make_double2(sum[0], sum[1]);
                snorm2 = sum[2];
            }
            const double2 beta = cmul(rho_new, inv_rho);
            const double2 ba = cmul(beta, ia);  // beta_n / alpha_n
#pragma unroll
            for (int i = 0; i < R; ++i) {
                const int row = lane + 64 * i;
                p[i] = cfma(beta, p[i], r[i]);
                q[i] = cfma(beta, q[i], s[i]);
                vp[KP * (row & 3) + (row >> 2)] = p[i];
                if (pidx[i] >= 0) hr[(size_t)(it + 1) * a.rmax + pidx[i]] = r[i];
            }
            if (lane == 0) {
                hab[2 * it] = ia;
                hab[2 * it + 1] = ba;
            }

            // collinearity factors and the freeze test ||s|| <= tol |pi^k|
            // (pi^k stepped for every shift of a slot with a running one: a
            // frozen one is never read again)
            const double2 coup = cmul(alpha, ba_old);
            const double2 c1 = cadd(one, coup), ncoup = make_double2(-coup.x, -coup.y);
#pragma unroll
            for (int m = 0; m < M; ++m) {
                if (!__any((act >> m) & 1u)) continue;  // every shift of the slot has frozen
                const double2 pn = cfma(cfma(alpha, sigma[m], c1), pc[m], cmul(ncoup, po[m]));
                const double pn2 = fma(pn.x, pn.x, pn.y * pn.y);
                po[m] = pc[m];
                pc[m] = pn;
                if (((act >> m) & 1u) && snorm2 <= tol2 * pn2) {
                    // the estimate ||s|| / |pi^k| is formed after the column
                    act &= ~(1u << m);
                    const int k = lane + 64 * m;
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
            wave_lds_fence();  // p is in LDS for the next block product
            if (!__any(act != 0) || snorm2 == 0.0) { status = SGF_CONVERGED; break; }
            if (rho_new.x == 0.0 && rho_new.y == 0.0) { status = SGF_BREAKDOWN; break; }
            if (!isfinite(rho_new.x + rho_new.y + snorm2)) { status = SGF_NONFINITE; break; }
            inv_rho = crcp(rho_new);
        }

#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int k = lane + 64 * m;
            if (k >= a.ns) continue;
            if (!((act >> m) & 1u)) {  // frozen: ||s|| / |pi^k| at its freeze
                if (a.resid)
                    a.resid[c * a.ns + k] = sqrt(a.fz[(size_t)slot * a.ns_pad + k] / a.resid[c * a.ns + k]);
                continue;
            }
            const double pn2 = fma(pc[m].x, pc[m].x, pc[m].y * pc[m].y);
            a.nk[(size_t)slot * a.ns_pad + k] = applied;
            if (a.resid) a.resid[c * a.ns + k] = applied > 0 ? sqrt(snorm2 / pn2) : 1.0;
            if (a.shift_iters) a.shift_iters[c * a.ns + k] = applied;
        }
        if (lane == 0) {
            *meta = ColMeta{(int32_t)c, iters, npa, status};
            a.iters[c] = iters;
            a.status[c] = status;
        }
    }
}

// Subspaces of 17 to 32 atoms: two wavefronts per column.  Thread t owns
// orbital row t, so a thread keeps one row of H in registers (as the
// one-row kernel does) and ns/128 shifts.  Each sum of an iteration is a
// wavefront sum, then the two wavefront totals added in wavefront order, so
// every thread holds the same scalars and every branch on them is uniform
// over the workgroup.  An iteration has four barriers: after mu, after the
// update of s (the product needs all of it), after rho' and ||s||^2, and the
// vote on the running shifts, which also orders p for the next iteration.
template <int M, int BMAX>
__global__ __launch_bounds__(2 * SEED_T) void k_seed_kr2(SolveArgs a) {
    constexpr int T = 2 * SEED_T, NA = 32, KP = NA + 1, PA = 5;
    __shared__ double2 vp[PA * NA];
    __shared__ double2 vs[4 * KP];
    __shared__ double si[NA * KP];
    __shared__ __align__(16) double red_mu[2][2 * 64], red_s[2][3 * 64];
    __shared__ double tot_mu[2][2], tot_s[2][3];
    __shared__ int64_t sh_ticket;
    const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
    const double2 zs = a.z[a.seed];
    double2 sigma[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int k = tid + T * m;
        sigma[m] = k < a.ns ? csub(a.z[k], zs) : make_double2(0.0, 0.0);
    }
    const double tol2 = a.tol * a.tol;
    const double2 zero = make_double2(0.0, 0.0), one = make_double2(1.0, 0.0);

    for (;;) {
        if (tid == 0) sh_ticket = (int64_t)atomicAdd(reinterpret_cast<unsigned long long *>(a.ticket), 1ull);
        __syncthreads();
        int64_t ticket = sh_ticket;
        __syncthreads();  // sh_ticket is read by all before the next column writes it
        if (ticket >= a.batch_end - a.batch_begin) break;
        const int64_t slot = ticket;
        ticket += a.batch_begin;
        const int64_t c = a.order ? (int64_t)a.order[ticket] : ticket;
        if (c < 0 || c >= a.n_cols) continue;  // reported by the one-row launch
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
            bad = n_loc < 1 || npa < 1 || 4 * npa > a.rmax || cl < 0 || cl >= n_loc ||
                  a.loc_atom[a0 + cl] != (int32_t)(j >> 2);
        }
        // the subspaces of 17 atoms or more (beyond 32: reported here); the
        // others, and the columns that cannot be solved, go to the one-row launch
        if (bad || n_loc <= 16) continue;
        bad = n_loc > NA;
        const int nl = 4 * n_loc;
        const int row = tid, A = row >> 2, o = row & 3;
        const bool rowv = !bad && row < nl;
        int t0 = 0, nb = 0;
        if (rowv) {
            t0 = a.lrow[a0 + A];
            nb = (A + 1 < n_loc ? a.lrow[a0 + A + 1] : nblk) - t0;
        }
        for (int e = tid; e < NA * KP; e += T) si[e] = 0.0;
        for (int e = tid; e < 4 * KP; e += T) vs[e] = zero;
        for (int e = tid; e < PA * NA; e += T) vp[e] = zero;
        __syncthreads();
        // S_a from the blocks of S (thread A < n_loc reads its atom's row)
        bool notk = false;
        if (!bad && tid < n_loc) {
            const int u0 = a.lrow[a0 + tid], u1 = tid + 1 < n_loc ? a.lrow[a0 + tid + 1] : nblk;
            for (int t = u0; t < u1; ++t) {
                const int B = a.lblk[2 * (b0 + t)];
                if (B < 0 || B >= n_loc) {
                    notk = true;
                    break;
                }
                const double *sb = &a.s[16 * (int64_t)a.lblk[2 * (b0 + t) + 1]];
                const double d = sb[0];
                bool ok = sb[5] == d && sb[10] == d && sb[15] == d;
#pragma unroll
                for (int e = 1; e < 15; ++e)
                    if (e % 5 != 0) ok = ok && sb[e] == 0.0;
                notk = notk || !ok;
                si[KP * tid + B] = d;
            }
        }
        if (__syncthreads_or(bad || nb > BMAX || notk)) {
            if (tid == 0) {
                a.meta[slot] = ColMeta{-1, 0, 0, SGF_BADCOLUMN};
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
        // S_a^{-1} in place by the first wavefront (n_loc <= 32 rows):
        // Gauss-Jordan elimination without pivoting, lane l updates row l
        if (wv == 0) {
            for (int kk = 0; kk < n_loc; ++kk) {
                const double piv = 1.0 / si[KP * kk + kk];
                const double f = (lane < n_loc && lane != kk) ? si[KP * lane + kk] : 0.0;
                wave_lds_fence();
                if (lane < n_loc) si[KP * kk + lane] = lane == kk ? piv : si[KP * kk + lane] * piv;
                wave_lds_fence();
                if (lane < n_loc && lane != kk) {
                    for (int jj = 0; jj < n_loc; ++jj)
                        si[KP * lane + jj] = fma(-f, si[KP * kk + jj], si[KP * lane + jj]);
                    si[KP * lane + kk] = -f * piv;
                }
                wave_lds_fence();
            }
        }
        __syncthreads();

        const int jA = cl, jo = (int)(j & 3);
        const int n4 = (n_loc + 3) & ~3;
        int pidx = -1;
        for (int q = 0; q < npa; ++q)
            if (rowv && a.pa_loc[p0 + q] == A) pidx = 4 * q + o;
        double2 *hab = a.hab + (size_t)slot * a.cap * 2;
        double2 *hr = a.hr + (size_t)slot * (a.cap + 1) * a.rmax;

        // start: x = 0, s_0 = q_0 = e_j, r_0 = p_0 = S^{-1} e_j
        double2 s = (rowv && A == jA && o == jo) ? one : zero, q = s;
        double2 p = (rowv && o == jo) ? make_double2(si[KP * A + jA], 0.0) : zero;
        vp[PA * A + o] = p;
        if (pidx >= 0) hr[pidx] = p;
        double2 rho = make_double2(si[KP * jA + jA], 0.0);
        double2 inv_rho = crcp(rho);
        const double *srow = &si[KP * A];
        const double2 *scol = &vs[KP * o];
        __syncthreads();

        double2 pc[M], po[M];
        uint32_t act = 0;
#pragma unroll
        for (int m = 0; m < M; ++m) {
            pc[m] = po[m] = one;
            if (tid + T * m < a.ns) act |= 1u << m;
        }
        double2 ba_old = zero;
        int status = SGF_MAXITER, iters = 0, applied = 0;
        double snorm2 = 1.0;
        const int max_iter = a.max_iter > 0 ? a.max_iter : 10 * nl;

        for (int it = 0; it < max_iter; ++it) {
            // w = z_s q - H p ; mu = p^T w
            double ax = 0.0, ay = 0.0;
#pragma unroll
            for (int b = 0; b < BMAX; ++b) {
#pragma unroll
                for (int qq = 0; qq < 4; ++qq) {
                    const double2 pv = vp[PA * bcol[b] + qq];
                    ax = fma(hrow[b][qq], pv.x, ax);
                    ay = fma(hrow[b][qq], pv.y, ay);
                }
            }
            const double2 w = make_double2(zs.x * q.x - zs.y * q.y - ax, zs.x * q.y + zs.y * q.x - ay);
            double2 mu;
            {
                const double part[2] = {fma(p.x, w.x, -p.y * w.y), fma(p.x, w.y, p.y * w.x)};
                double sum[2];
                wave_sum_lds<2>(part, red_mu[wv], sum);
                if (lane == 0) {
                    tot_mu[wv][0] = sum[0];
                    tot_mu[wv][1] = sum[1];
                }
                __syncthreads();
                mu = make_double2(tot_mu[0][0] + tot_mu[1][0], tot_mu[0][1] + tot_mu[1][1]);
            }
            iters = it + 1;
            if (!cfinite(mu)) { status = SGF_NONFINITE; break; }
            if (mu.x == 0.0 && mu.y == 0.0) { status = SGF_BREAKDOWN; break; }
            const double2 alpha = cmul(rho, crcp(mu));
            const double2 ia = cmul(mu, inv_rho);

            // s -= alpha w ; r = S^{-1} s ; rho' = r^T s ; ||s||^2
            s = csub(s, cmul(alpha, w));
            vs[KP * o + A] = s;
            __syncthreads();
            double2 r;
            {
                double bx[4] = {0.0, 0.0, 0.0, 0.0}, by[4] = {0.0, 0.0, 0.0, 0.0};
                for (int B = 0; B < n4; B += 4) {
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const double av = srow[B + u];
                        const double2 sv = scol[B + u];
                        bx[u] = fma(av, sv.x, bx[u]);
                        by[u] = fma(av, sv.y, by[u]);
                    }
                }
                r = make_double2((bx[0] + bx[1]) + (bx[2] + bx[3]), (by[0] + by[1]) + (by[2] + by[3]));
            }
            double2 rho_new;
            {
                const double part[3] = {fma(r.x, s.x, -r.y * s.y), fma(r.x, s.y, r.y * s.x),
                                        fma(s.x, s.x, s.y * s.y)};
                double sum[3];
                wave_sum_lds<3>(part, red_s[wv], sum);
                if (lane == 0) {
                    tot_s[wv][0] = sum[0];
                    tot_s[wv][1] = sum[1];
                    tot_s[wv][2] = sum[2];
                }
                __syncthreads();
                rho_new = make_double2(tot_s[0][0] + tot_s[1][0], tot_s[0][1] + tot_s[1][1]);
                snorm2 = tot_s[0][2] + tot_s[1][2];
            }
            const double2 beta = cmul(rho_new, inv_rho);
            const double2 ba = cmul(beta, ia);
            p = cfma(beta, p, r);
            q = cfma(beta, q, s);
            vp[PA * A + o] = p;
            if (pidx >= 0) hr[(size_t)(it + 1) * a.rmax + pidx] = r;
            if (tid == 0) {
                hab[2 * it] = ia;
                hab[2 * it + 1] = ba;
            }

            const double2 coup = cmul(alpha, ba_old);
            const double2 c1 = cadd(one, coup), ncoup = make_double2(-coup.x, -coup.y);
#pragma unroll
            for (int m = 0; m < M; ++m) {
                if (!__any((act >> m) & 1u)) continue;  // every shift of the slot has frozen
                const double2 pn = cfma(cfma(alpha, sigma[m], c1), pc[m], cmul(ncoup, po[m]));
                const double pn2 = fma(pn.x, pn.x, pn.y * pn.y);
                po[m] = pc[m];
                pc[m] = pn;
                if (((act >> m) & 1u) && snorm2 <= tol2 * pn2) {
                    // the estimate ||s|| / |pi^k| is formed after the column
                    act &= ~(1u << m);
                    const int k = tid + T * m;
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
            const bool any_alive = __syncthreads_or(act != 0) != 0;
            if (!any_alive || snorm2 == 0.0) { status = SGF_CONVERGED; break; }
            if (rho_new.x == 0.0 && rho_new.y == 0.0) { status = SGF_BREAKDOWN; break; }
            if (!isfinite(rho_new.x + rho_new.y + snorm2)) { status = SGF_NONFINITE; break; }
            inv_rho = crcp(rho_new);
        }

#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int k = tid + T * m;
            if (k >= a.ns) continue;
            if (!((act >> m) & 1u)) {  // frozen: ||s|| / |pi^k| at its freeze
                if (a.resid)
                    a.resid[c * a.ns + k] = sqrt(a.fz[(size_t)slot * a.ns_pad + k] / a.resid[c * a.ns + k]);
                continue;
            }
            const double pn2 = fma(pc[m].x, pc[m].x, pc[m].y * pc[m].y);
            a.nk[(size_t)slot * a.ns_pad + k] = applied;
            if (a.resid) a.resid[c * a.ns + k] = applied > 0 ? sqrt(snorm2 / pn2) : 1.0;
            if (a.shift_iters) a.shift_iters[c * a.ns + k] = applied;
        }
        if (tid == 0) {
            a.meta[slot] = ColMeta{(int32_t)c, iters, npa, status};
            a.iters[c] = iters;
            a.status[c] = status;
        }
    }
}

template <int BMAX>
KernelFn pick_kr2_m(int M2) {
    return M2 <= 1 ? k_seed_kr2<1, BMAX> : k_seed_kr2<2, BMAX>;
}

template <int R, int BMAX>
KernelFn pick_kr_m(int M) {
    switch (M) {
        case 1: return k_seed_kr<R, 1, BMAX>;
        case 2: return k_seed_kr<R, 2, BMAX>;
        default: return k_seed_kr<R, 4, BMAX>;
    }
}

template <int R>
KernelFn pick_kr_b(int M, int bmax) {
    return bmax <= 5 ? pick_kr_m<R, 5>(M) : bmax <= 6 ? pick_kr_m<R, 6>(M) : pick_kr_m<R, 8>(M);
}

}  // namespace

KernelFn pick_seed_kron(int rows_per_lane, int M, int bmax) {
    return rows_per_lane == 1 ? pick_kr_b<1>(M, bmax) : pick_kr_b<2>(M, bmax);
}

KernelFn pick_seed_kron2(int M2, int bmax) {
    return bmax <= 5 ? pick_kr2_m<5>(M2) : bmax <= 6 ? pick_kr2_m<6>(M2) : pick_kr2_m<8>(M2);
}

}  // namespace sgf
