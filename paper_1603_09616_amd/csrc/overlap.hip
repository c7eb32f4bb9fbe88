// overlap.hip -- seed pass of the shifted COCG for S != I with the inverse of
// the local overlap held in registers.
//
// The iteration is the one of the generic S != I seed pass: COCG on
// A = S_L^{-1}(z_s S_L - H_L) in the S-bilinear form [u, v] = u^T S_L v, with
// s the true-space residual, r = S_L^{-1} s, q = S_L p (kept by the recurrence
// q <- s + beta q) and w = z_s q - H_L p, so mu = p^T w and rho = r^T s.  What
// differs is where S_L^{-1} lives and how it is formed:
//
// * The nl x nl inverse is cut into 8 x 8 tiles on an NB x NB grid and thread
//   t < NB^2 keeps tile (t / NB, t % NB) in 64 registers for the whole
//   column.  The product r = S_L^{-1} s then reads only the 8 entries of s of
//   the tile's column block and writes 8 partial row sums; the owner of row i
//   (thread i) adds the partials of its row in tile order.  Nothing of the
//   inverse passes through LDS after it is formed.
// * The inverse is formed in those registers by the symmetric sweep operator
//   (Gauss-Jordan elimination without pivoting on a symmetric positive
//   definite matrix; after all pivots the matrix holds -S_L^{-1}).  The sweep
//   keeps the matrix symmetric, so the pivot row, passed through LDS, is also
//   the pivot column, and every register index is a compile-time constant.
//
// One wavefront takes a column of at most 16 local atoms (nl <= 64, NB = 8);
// a workgroup of two wavefronts takes 17 to 22 atoms (nl <= 88, NB = 11).
// Both variants run over the whole batch and take the columns of their own
// size class; the one-wavefront variant also reports columns that cannot be
// solved.
#include "scocg.hpp"

namespace sgf {

namespace {

template <int W>
__device__ __forceinline__ void blk_sync() {
    if constexpr (W == 1)
        wave_lds_fence();
    else
        __syncthreads();
}

// Sums over the workgroup of NV values per thread: each wavefront's sum (the
// LDS wave sum), then the wavefronts' totals added in wavefront order.
template <int W, int NV>
__device__ __forceinline__ void blk_sum(const double (&v)[NV], double *red_wave, double (*tot)[4],
                                        double (&out)[NV]) {
    wave_sum_lds<NV>(v, red_wave, out);
    if constexpr (W > 1) {
        if ((threadIdx.x & 63) == 0) {
#pragma unroll
            for (int i = 0; i < NV; ++i) tot[threadIdx.x >> 6][i] = out[i];
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            double s = tot[0][i];
#pragma unroll
            for (int w = 1; w < W; ++w) s += tot[w][i];
            out[i] = s;
        }
    }
}

template <int W>
__device__ __forceinline__ bool blk_any(bool v) {
    if constexpr (W == 1)
        return __any(v);
    else
        return __syncthreads_or(v ? 1 : 0) != 0;
}

template <int W, int M, int BMAX>
__global__ __launch_bounds__(64 * W) void k_seed_ovl(SolveArgs a) {
    constexpr int NT = 64 * W;
    constexpr int NB = W == 1 ? 8 : 11;  // tile grid
    constexpr int NLMAX = 8 * NB;        // orbitals
    constexpr int NA = NLMAX / 4;        // local atoms
    constexpr int A_LO = W == 1 ? 1 : 17, A_HI = W == 1 ? 16 : 22;

    __shared__ double2 vs[NLMAX];         // s for the tile products (zero beyond nl)
    __shared__ double2 vp[NLMAX];         // p, orbital-major (vp[NA o + A]), for the block product
    __shared__ double hl[BMAX * 4 * NLMAX];  // H_L by rows: entry q of block b of row i at hl[NLMAX (4 b + q) + i]
    __shared__ double2 sig[64 * M * W];      // z_k - z_s
    __shared__ double2 part[NB * NLMAX];  // partial row sums part[NLMAX cb + i]; the sweep's pivot rows
    __shared__ __align__(16) double red[W][5 * 64];  // wave sums: 2 values for mu, 3 for rho and ||s||^2
    __shared__ double tot[2][W][4];
    __shared__ int64_t sh_ticket;

    const int tid = threadIdx.x;
    double *red_mu = red[tid >> 6], *red_s = red[tid >> 6] + 2 * 64;
    const double2 zs = a.z[a.seed];
    for (int k = tid; k < NT * M; k += NT) sig[k] = k < a.ns ? csub(a.z[k], zs) : make_double2(0.0, 0.0);
    const double tol2 = a.tol * a.tol;
    const double2 zero = make_double2(0.0, 0.0), one = make_double2(1.0, 0.0);
    const bool tile = tid < NB * NB;
    const int rb = tile ? tid / NB : 0, cb = tile ? tid % NB : 0;

    for (;;) {
        int64_t ticket = 0;
        if constexpr (W == 1) {
            if (tid == 0) ticket = (int64_t)atomicAdd(reinterpret_cast<unsigned long long *>(a.ticket), 1ull);
            ticket = __shfl(ticket, 0, 64);
        } else {
            if (tid == 0) sh_ticket = (int64_t)atomicAdd(reinterpret_cast<unsigned long long *>(a.ticket), 1ull);
            __syncthreads();
            ticket = sh_ticket;
            __syncthreads();
        }
        if (ticket >= a.batch_end - a.batch_begin) break;
        const int64_t slot = ticket;
        ticket += a.batch_begin;
        const int64_t c = a.order ? (int64_t)a.order[ticket] : ticket;
        ColMeta *meta = &a.meta[slot];
        if (c < 0 || c >= a.n_cols) {
            if (W == 1 && tid == 0) *meta = ColMeta{-1, 0, 0, SGF_BADCOLUMN};
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
            bad = n_loc < 1 || n_loc > 22 || n_loc > a.max_loc_atoms || npa < 1 || 4 * npa > a.rmax || cl < 0 ||
                  cl >= n_loc || a.loc_atom[a0 + cl] != (int32_t)(j >> 2);
        }
        // the one-wavefront variant reports unsolvable columns; each variant
        // solves the columns of its own size
        if (bad ? W != 1 : (n_loc < A_LO || n_loc > A_HI)) continue;
        const int nl = 4 * n_loc;
        const bool row = !bad && tid < nl;
        const int A = tid >> 2, o = tid & 3;
        int nb = 0, t0 = 0;
        if (row) {
            t0 = a.lrow[a0 + A];
            nb = (A + 1 < n_loc ? a.lrow[a0 + A + 1] : nblk) - t0;
        }
        bad = blk_any<W>(bad || nb > BMAX);
        if (bad) {
            if (tid == 0) {
                *meta = ColMeta{-1, 0, 0, SGF_BADCOLUMN};
                a.iters[c] = 0;
                a.status[c] = SGF_BADCOLUMN;
            }
            blk_sync<W>();
            continue;
        }
        const int jl = 4 * cl + (int)(j & 3);
        int pidx = -1;  // position of this thread's row among the projection rows
        for (int q = 0; q < npa; ++q)
            if (row && a.pa_loc[p0 + q] == A) pidx = 4 * q + o;
        double2 *hab = a.hab + (size_t)slot * a.cap * 2;
        double2 *hr = a.hr + (size_t)slot * (a.cap + 1) * a.rmax;

        // the tile of S_L: rows 8 rb .. 8 rb + 7 are local atoms 2 rb and
        // 2 rb + 1, columns those of atoms 2 cb and 2 cb + 1; zero beyond nl
        double T[8][8];
#pragma unroll
        for (int m = 0; m < 8; ++m)
#pragma unroll
            for (int n = 0; n < 8; ++n) T[m][n] = 0.0;
        if (tile) {
#pragma unroll
            for (int ra = 0; ra < 2; ++ra) {
                const int Ar = 2 * rb + ra;
                if (Ar >= n_loc) continue;
                const int u0 = a.lrow[a0 + Ar], u1 = Ar + 1 < n_loc ? a.lrow[a0 + Ar + 1] : nblk;
                for (int u = u0; u < u1; ++u) {
                    const int B = a.lblk[2 * (b0 + u)];
                    const double *sb = &a.s[16 * (int64_t)a.lblk[2 * (b0 + u) + 1]];
                    if (B == 2 * cb) {
#pragma unroll
                        for (int oo = 0; oo < 4; ++oo)
#pragma unroll
                            for (int q = 0; q < 4; ++q) T[4 * ra + oo][q] = sb[4 * oo + q];
                    } else if (B == 2 * cb + 1) {
#pragma unroll
                        for (int oo = 0; oo < 4; ++oo)
#pragma unroll
                            for (int q = 0; q < 4; ++q) T[4 * ra + oo][4 + q] = sb[4 * oo + q];
                    }
                }
            }
        }
        for (int i = tid; i < NLMAX; i += NT) vs[i] = make_double2(i == jl ? 1.0 : 0.0, 0.0);

        // Sweep on pivot k (d = a_kk): a_ij -= a_ik a_kj / d for i, j != k,
        // a_ik /= d, a_kj /= d, a_kk = -1/d.  All four cases are one update
        // a_ij = c_i a_ij + g_i b_j with b_j = a_kj (j != k), b_k = d - 1,
        // g_i = -a_ik / d, c_i = 1 (i != k) and g_k = 1 + 1/d, c_k = -1.
        // The pivots of the unit-diagonal overlap stay in (0, 1], where these
        // forms lose no accuracy.
        const int nbk = (nl + 7) >> 3;
        double *prow = reinterpret_cast<double *>(part);  // two pivot-row buffers of NLMAX doubles
        for (int kb = 0; kb < nbk; ++kb) {
#pragma unroll
            for (int ko = 0; ko < 8; ++ko) {
                const int k = 8 * kb + ko;
                if (k >= nl) break;
                double *buf = prow + (ko & 1) * NLMAX;
                if (tile && rb == kb) {
#pragma unroll
                    for (int n = 0; n < 8; ++n) buf[8 * cb + n] = T[ko][n];
                }
                blk_sync<W>();
                const double d = buf[k];
                const double id = 1.0 / d;
                if (tile) {
                    double g[8], bv[8];
#pragma unroll
                    for (int m = 0; m < 8; ++m) g[m] = -buf[8 * rb + m] * id;
#pragma unroll
                    for (int n = 0; n < 8; ++n) bv[n] = buf[8 * cb + n];
                    if (rb == kb) {
                        g[ko] = 1.0 + id;
#pragma unroll
                        for (int n = 0; n < 8; ++n) T[ko][n] = -T[ko][n];
                    }
                    if (cb == kb) bv[ko] = d - 1.0;
#pragma unroll
                    for (int m = 0; m < 8; ++m)
#pragma unroll
                        for (int n = 0; n < 8; ++n) T[m][n] = fma(g[m], bv[n], T[m][n]);
                }
            }
        }

        // this thread's row of H (in LDS) and the local atoms of its blocks;
        // absent blocks hold zeros and point at atom 0
        int bcol[BMAX];
#pragma unroll
        for (int b = 0; b < BMAX; ++b) {
            bcol[b] = 0;
            double hv[4] = {0.0, 0.0, 0.0, 0.0};
            if (b < nb) {
                const int32_t *lb = &a.lblk[2 * (b0 + t0 + b)];
                bcol[b] = lb[0];
                const double *hb = &a.h[16 * (int64_t)lb[1] + 4 * o];
#pragma unroll
                for (int q = 0; q < 4; ++q) hv[q] = hb[q];
            }
            if (tid < NLMAX) {
#pragma unroll
                for (int q = 0; q < 4; ++q) hl[NLMAX * (4 * b + q) + tid] = hv[q];
            }
        }

        // r = S_L^{-1} s for the s in vs (T holds -S_L^{-1}); the caller has
        // written vs.  Two passes of four rows keep the accumulators short.
        auto apply_inverse = [&]() -> double2 {
            blk_sync<W>();
            if (tile) {
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    double2 acc[4];
#pragma unroll
                    for (int m = 0; m < 4; ++m) acc[m] = zero;
#pragma unroll
                    for (int n = 0; n < 8; ++n) {
                        const double2 x = vs[8 * cb + n];
#pragma unroll
                        for (int m = 0; m < 4; ++m) {
                            acc[m].x = fma(T[4 * h + m][n], x.x, acc[m].x);
                            acc[m].y = fma(T[4 * h + m][n], x.y, acc[m].y);
                        }
                    }
#pragma unroll
                    for (int m = 0; m < 4; ++m) part[NLMAX * cb + 8 * rb + 4 * h + m] = acc[m];
                }
            }
            blk_sync<W>();
            double2 r = zero;
            if (row)
                for (int u = 0; u < nbk; ++u) r = cadd(r, part[NLMAX * u + tid]);
            return make_double2(-r.x, -r.y);
        };

        // start: s_0 = q_0 = e_jl, r_0 = p_0 = S^{-1} e_jl, rho_0 = r_0^T s_0
        double2 s = make_double2(row && tid == jl ? 1.0 : 0.0, 0.0), q = s;
        double2 r = apply_inverse();
        double2 p = r;
        if (row) vp[NA * o + A] = p;
        if (pidx >= 0) hr[pidx] = r;
        double2 rho;
        {
            const double v[2] = {fma(r.x, s.x, -r.y * s.y), fma(r.x, s.y, r.y * s.x)};
            double sum[2];
            blk_sum<W, 2>(v, red_mu, tot[0], sum);
            rho = make_double2(sum[0], sum[1]);
        }

        // pi^k of this thread's shifts; bit m of act: shift tid + NT m is running
        double2 pc[M], po[M];
        unsigned act = 0;
#pragma unroll
        for (int m = 0; m < M; ++m) {
            pc[m] = po[m] = one;
            if (tid + NT * m < a.ns) act |= 1u << m;
        }
        double2 inv_rho = crcp(rho), ba_old = zero;
        int status = SGF_MAXITER, iters = 0, applied = 0;
        double snorm2 = 1.0;
        const int max_iter = a.max_iter > 0 ? a.max_iter : 10 * nl;
        if (!cfinite(rho) || (rho.x == 0.0 && rho.y == 0.0)) {
            status = cfinite(rho) ? SGF_BREAKDOWN : SGF_NONFINITE;
        } else {
            for (int it = 0; it < max_iter; ++it) {
                blk_sync<W>();  // p is in vp
                // H_L and z - z_s are read from LDS where they are used: an
                // offset the compiler cannot see through keeps those loads
                // from being hoisted out of the loop into registers
                int lo = 0;
                asm volatile("" : "+v"(lo));
                // w = z_s q - H p ; mu = p^T w
                double ax = 0.0, ay = 0.0;
#pragma unroll
                for (int b = 0; b < BMAX; ++b) {
#pragma unroll
                    for (int qq = 0; qq < 4; ++qq) {
                        const double2 pv = vp[NA * qq + bcol[b]];
                        const double hv = tid < NLMAX ? hl[lo + NLMAX * (4 * b + qq) + tid] : 0.0;
                        ax = fma(hv, pv.x, ax);
                        ay = fma(hv, pv.y, ay);
                    }
                }
                const double2 w = make_double2(zs.x * q.x - zs.y * q.y - ax, zs.x * q.y + zs.y * q.x - ay);
                double2 mu;
                {
                    const double v[2] = {fma(p.x, w.x, -p.y * w.y), fma(p.x, w.y, p.y * w.x)};
                    double sum[2];
                    blk_sum<W, 2>(v, red_mu, tot[0], sum);
                    mu = make_double2(sum[0], sum[1]);
                }
                iters = it + 1;
                if (!cfinite(mu)) { status = SGF_NONFINITE; break; }
                if (mu.x == 0.0 && mu.y == 0.0) { status = SGF_BREAKDOWN; break; }
                const double2 alpha = cmul(rho, crcp(mu));
                const double2 ia = cmul(mu, inv_rho);  // 1/alpha

                // s -= alpha w ; r = S^{-1} s ; rho' = r^T s ; ||s||^2
                if (row) {
                    s = csub(s, cmul(alpha, w));
                    vs[tid] = s;
                }
                r = apply_inverse();
                double2 rho_new;
                {
                    const double v[3] = {fma(r.x, s.x, -r.y * s.y), fma(r.x, s.y, r.y * s.x),
                                         fma(s.x, s.x, s.y * s.y)};
                    double sum[3];
                    blk_sum<W, 3>(v, red_s, tot[1], sum);
                    rho_new = make_double2(sum[0], sum[1]);
                    snorm2 = sum[2];
                }
                const double2 beta = cmul(rho_new, inv_rho);
                const double2 ba = cmul(beta, ia);  // beta_n / alpha_n
                if (row) {
                    p = cfma(beta, p, r);
                    q = cfma(beta, q, s);
                    vp[NA * o + A] = p;
                }
                if (tid == 0) {
                    hab[2 * it] = ia;
                    hab[2 * it + 1] = ba;
                }
                if (pidx >= 0) hr[(size_t)(it + 1) * a.rmax + pidx] = r;

                // pi^k_{n+1} = (1 + c + alpha sigma_k) pi^k_n - c pi^k_{n-1},
                // c = alpha_n beta_{n-1} / alpha_{n-1}; freeze at ||s|| <= tol |pi^k|
                const double2 coup = cmul(alpha, ba_old);
                const double2 c1 = cadd(one, coup), ncoup = make_double2(-coup.x, -coup.y);
#pragma unroll
                for (int m = 0; m < M; ++m) {
                    const double2 pn = cfma(cfma(alpha, sig[lo + tid + NT * m], c1), pc[m], cmul(ncoup, po[m]));
                    const double pn2 = fma(pn.x, pn.x, pn.y * pn.y);
                    po[m] = pc[m];
                    pc[m] = pn;
                    if ((act >> m & 1u) && snorm2 <= tol2 * pn2) {
                        // frozen: its step count and residual are final
                        act &= ~(1u << m);
                        const int k = tid + NT * m;
                        a.nk[(size_t)slot * a.ns_pad + k] = it + 1;
                        if (a.resid) a.resid[c * a.ns + k] = sqrt(snorm2 / pn2);
                        if (a.shift_iters) a.shift_iters[c * a.ns + k] = it + 1;
                    }
                }
                const bool alive = act != 0;
                applied = it + 1;
                ba_old = ba;
                rho = rho_new;
                const bool any_alive = blk_any<W>(alive);
                if (!any_alive || snorm2 == 0.0) { status = SGF_CONVERGED; break; }
                if (rho_new.x == 0.0 && rho_new.y == 0.0) { status = SGF_BREAKDOWN; break; }
                if (!isfinite(rho_new.x + rho_new.y + snorm2)) { status = SGF_NONFINITE; break; }
                inv_rho = crcp(rho_new);
            }
        }

        // shifts still running took every applied update
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int k = tid + NT * m;
            if (!(act >> m & 1u)) continue;
            const double pn2 = fma(pc[m].x, pc[m].x, pc[m].y * pc[m].y);
            a.nk[(size_t)slot * a.ns_pad + k] = applied;
            if (a.resid) a.resid[c * a.ns + k] = applied > 0 ? sqrt(snorm2 / pn2) : 1.0;
            if (a.shift_iters) a.shift_iters[c * a.ns + k] = applied;
        }
        if (tid == 0) {
            *meta = ColMeta{(int32_t)c, iters, npa, status};
            a.iters[c] = iters;
            a.status[c] = status;
        }
        blk_sync<W>();  // LDS reuse by the next column
    }
}

template <int W, int BMAX>
KernelFn pick_m(int M) {
    switch (M) {
        case 1: return k_seed_ovl<W, 1, BMAX>;
        case 2: return k_seed_ovl<W, 2, BMAX>;
        default: return k_seed_ovl<W, 4, BMAX>;
    }
}

}  // namespace

KernelFn pick_seed_ovl(int W, int M, int bmax) {
    if (W == 1) return bmax <= 5 ? pick_m<1, 5>(M) : bmax <= 6 ? pick_m<1, 6>(M) : pick_m<1, 8>(M);
    return bmax <= 5 ? pick_m<2, 5>(M) : bmax <= 6 ? pick_m<2, 6>(M) : pick_m<2, 8>(M);
}

}  // namespace sgf
