// mixed.hip -- mixed-precision shifted COCG (S = I, local subspaces of at
// most 64 orbitals).
//
// Seed pass: the operator (FP32 shadow of H) and the Krylov vectors s, p, w
// are complex FP32; every scalar of the recurrence (mu, rho, alpha, beta and
// the per-shift collinear factors pi^k) is FP64, and the reductions that
// produce them sum exact FP64 products of the FP32 entries.  The seed
// iterate x_s = sum alpha_n p_n is kept in FP64, and every monitor_every
// iterations (and at the end) the FP64 true residual b - (z_s - H) x_s is
// formed with the FP64 operator: if it departs from the recursive residual s
// by more than drift_tol ||b||, the column stops with status DRIFT.  The
// pass records the full residual vectors r_n (complex FP32) instead of their
// projection rows.
//
// Shift pass: the same backward UL factorization of the shifted tridiagonal
// as the FP64 pass, accumulated over every local row, gives the full iterate
// x~^k of each shift (complex FP32, staged in LDS).  The diagonal element is
// then replaced by the FP64 variational estimate
//     G_jj(z_k) ~ 2 x~_j - x~^T (z_k - H) x~,
// whose error is -e^T (z_k - H) e for e = x - x~, i.e. quadratic in the error
// of x~ (this holds for any approximation x~ because z_k - H is complex
// symmetric).  The other projection rows are the FP32-Krylov iterate itself.
// The residual of the full iterate gives a rigorous bound on the error of
// the estimate, which accepts or rejects (DRIFT) each column.
#include "scocg.hpp"

namespace sgf {

namespace {

__device__ __forceinline__ double2 to_d(float2 v) { return make_double2((double)v.x, (double)v.y); }
__device__ __forceinline__ float2 to_f(double2 v) { return make_float2((float)v.x, (float)v.y); }

template <int M, int BMAX>
__global__ __launch_bounds__(SEED_T) void k_seed_mx(SolveArgs a) {
    __shared__ float2 vp[64];   // p, for the neighbour reads of the block product
    __shared__ double2 vx[64];  // x_s, for the FP64 monitor
    const int lane = threadIdx.x;
    const double2 zs = a.z[a.seed];
    const float2 zsf = to_f(zs);
    double2 sigma[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int k = lane + 64 * m;
        sigma[m] = k < a.ns ? csub(a.z[k], zs) : make_double2(0.0, 0.0);
    }
    const double tol2 = a.tol * a.tol;
    const double drift2 = a.drift_tol * a.drift_tol;
    const double2 zero = make_double2(0.0, 0.0), one = make_double2(1.0, 0.0);
    const float2 fzero = make_float2(0.f, 0.f);

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
            bad = n_loc < 1 || n_loc > 16 || npa < 1 || npa > 8 || cl < 0 || cl >= n_loc ||
                  a.loc_atom[a0 + cl] != (int32_t)(j >> 2);
        }
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
        float hrow[BMAX][4];
#pragma unroll
        for (int b = 0; b < BMAX; ++b) {
            bcol[b] = 0;
            hrow[b][0] = hrow[b][1] = hrow[b][2] = hrow[b][3] = 0.f;
            if (b < nb) {
                const int32_t *lb = &a.lblk[2 * (b0 + t0 + b)];
                bcol[b] = 4 * lb[0];
                const float *hb = &a.h32[16 * (int64_t)lb[1] + 4 * o];
#pragma unroll
                for (int q = 0; q < 4; ++q) hrow[b][q] = hb[q];
            }
        }
        const int jl = 4 * cl + (int)(j & 3);
        double2 *hab = a.hab + (size_t)slot * a.cap * 2;
        float2 *hist = reinterpret_cast<float2 *>(a.hr + (size_t)slot * (a.cap + 1) * a.rmax);  // [cap+1][64]

        // FP64 true residual of the seed system against the recursive one:
        // returns ||b - (z_s - H) x_s - s||^2 (all lanes)
        auto gap2 = [&](double2 x, float2 s) -> double {
            vx[lane] = x;
            wave_lds_fence();
            double hx = 0.0, hy = 0.0;
#pragma unroll
            for (int b = 0; b < BMAX; ++b) {
                if (b < nb) {
                    const double *hb = &a.h[16 * (int64_t)a.lblk[2 * (b0 + t0 + b) + 1] + 4 * o];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const double2 xv = vx[bcol[b] + q];
                        hx = fma(hb[q], xv.x, hx);
                        hy = fma(hb[q], xv.y, hy);
                    }
                }
            }
            double d = 0.0;
            if (row) {
                const double tx = (lane == jl ? 1.0 : 0.0) - (zs.x * x.x - zs.y * x.y - hx);
                const double ty = -(zs.x * x.y + zs.y * x.x - hy);
                const double ex = tx - (double)s.x, ey = ty - (double)s.y;
                d = fma(ex, ex, ey * ey);
            }
            const double g = wave_reduce(d);
            wave_lds_fence();  // vx reads done before it is written again
            return g;
        };

        float2 s = (row && lane == jl) ? make_float2(1.f, 0.f) : fzero, p = s;
        double2 x = zero;
        vp[lane] = p;
        hist[lane] = s;
        wave_lds_fence();

        double2 pc[M], po[M];
        bool act[M];
        int nkm[M];
        double res[M];
#pragma unroll
        for (int m = 0; m < M; ++m) {
            pc[m] = po[m] = one;
            act[m] = lane + 64 * m < a.ns;
            nkm[m] = 0;
            res[m] = 1.0;
        }
        double2 rho = one, inv_rho = one;
        double2 beta_old = zero, ia_old = one;
        int status = SGF_MAXITER, iters = 0, applied = 0;
        double snorm2 = 1.0;
        // FP32 Krylov vectors lose their bi-orthogonality sooner than FP64
        // ones, which delays convergence (3-4x the FP64 iteration count on
        // the bundle, with a long tail): the default cap is 40 n_L
        const int max_iter = a.max_iter > 0 ? a.max_iter : 40 * nl;
        const int K = a.monitor_every;

        for (int it = 0; it < max_iter; ++it) {
            // w = z_s p - H p (FP32) ; mu = p^T w (FP64 sum of exact products)
            float ax = 0.f, ay = 0.f;
#pragma unroll
            for (int b = 0; b < BMAX; ++b) {
                if (b < nb) {
                    const float2 *pb = &vp[bcol[b]];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const float2 pv = pb[q];
                        ax = fmaf(hrow[b][q], pv.x, ax);
                        ay = fmaf(hrow[b][q], pv.y, ay);
                    }
                }
            }
            const float2 w = make_float2(zsf.x * p.x - zsf.y * p.y - ax, zsf.x * p.y + zsf.y * p.x - ay);
            const double2 mu =
                make_double2(wave_reduce((double)p.x * (double)w.x - (double)p.y * (double)w.y),
                             wave_reduce((double)p.x * (double)w.y + (double)p.y * (double)w.x));
            iters = it + 1;
            if (!cfinite(mu) || !cfinite(rho)) { status = SGF_NONFINITE; break; }
            if (mu.x == 0.0 && mu.y == 0.0) { status = SGF_BREAKDOWN; break; }
            const double2 alpha = cmul(rho, crcp(mu));
            const double2 ia = cmul(mu, inv_rho);  // 1/alpha

            // x_s += alpha p (FP64) ; s -= alpha w (FP32) ; rho', ||s||^2 (FP64)
            x = cfma(alpha, to_d(p), x);
            const float2 af = to_f(alpha);
            s = make_float2(s.x - (af.x * w.x - af.y * w.y), s.y - (af.x * w.y + af.y * w.x));
            const double sx = (double)s.x, sy = (double)s.y;
            const double2 rho_new = make_double2(wave_reduce(sx * sx - sy * sy), wave_reduce(2.0 * sx * sy));
            snorm2 = wave_reduce(fma(sx, sx, sy * sy));
            const double2 beta = cmul(rho_new, inv_rho);
            const float2 bf = to_f(beta);
            p = make_float2(s.x + (bf.x * p.x - bf.y * p.y), s.y + (bf.x * p.y + bf.y * p.x));
            vp[lane] = p;

            if (lane == 0) {
                hab[2 * it] = ia;
                hab[2 * it + 1] = cmul(beta, ia);
            }
            hist[(size_t)(it + 1) * 64 + lane] = s;

            const double2 coup = cmul(cmul(alpha, beta_old), ia_old);
            int alive = 0;
#pragma unroll
            for (int m = 0; m < M; ++m) {
                if (!act[m]) continue;
                const double2 pn = cadd(cmul(cfma(alpha, sigma[m], one), pc[m]), cmul(coup, csub(pc[m], po[m])));
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
            beta_old = beta;
            ia_old = ia;
            rho = rho_new;
            wave_lds_fence();  // p is in LDS for the next block product
            const bool any_alive = __any(alive);
            if (!any_alive || snorm2 == 0.0) {
                status = gap2(x, s) > drift2 ? SGF_DRIFT : SGF_CONVERGED;
                break;
            }
            if (K > 0 && (it + 1) % K == 0 && gap2(x, s) > drift2) { status = SGF_DRIFT; break; }
            if (rho_new.x == 0.0 && rho_new.y == 0.0) { status = SGF_BREAKDOWN; break; }
            if (!cfinite(rho_new) || !isfinite(snorm2)) { status = SGF_NONFINITE; break; }
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
            }
            a.nk[(size_t)slot * a.ns_pad + k] = nkm[m];
            if (a.resid) a.resid[c * a.ns + k] = res[m];
            if (a.shift_iters) a.shift_iters[c * a.ns + k] = nkm[m];
        }
        if (lane == 0) {
            // the shift pass needs the local size: npa in the low byte, n_loc above
            *meta = ColMeta{(int32_t)c, iters, npa | (n_loc << 8), status};
            a.iters[c] = iters;
            a.status[c] = status;
        }
        wave_lds_fence();  // vp reuse by the next column
    }
}

// ---------------------------------------------------------------------------
// Mixed shift pass: one workgroup per column, one lane per shift (ns_pad <=
// 256 lanes).  Dynamic LDS: x~ as float2 [64][ns_pad].
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_shift_mx(SolveArgs a) {
    extern __shared__ float2 xt[];                 // [64][ns_pad]
    __shared__ double2 sab[SHIFT_CH + 1][2];       // 1/alpha, beta/alpha of steps lo-1 .. hi
    __shared__ float2 srow[SHIFT_CH][64];          // r_m on every local row for steps lo .. hi
    __shared__ int skey[256];                      // (N_k << 10) | k, sorted ascending
    __shared__ double rpart[32 * 4];               // [projection row][wave] partial rho sums
    const int64_t slot = blockIdx.x;
    const ColMeta meta = a.meta[slot];
    if (meta.col < 0) return;  // uniform over the workgroup
    const int64_t c = meta.col;
    const int npa = meta.npa & 255, n_loc = meta.npa >> 8;
    const int nl = 4 * n_loc, nrow = 4 * npa;
    const int tid = threadIdx.x, T = blockDim.x;
    const int wv = tid >> 6, lane = tid & 63, nwv = T >> 6;
    const double2 *hab = a.hab + (size_t)slot * a.cap * 2;
    const float2 *hist = reinterpret_cast<const float2 *>(a.hr + (size_t)slot * (a.cap + 1) * a.rmax);
    const double2 zero = make_double2(0.0, 0.0);
    const int32_t pl = a.col_plan[c];
    const int64_t a0 = a.atom_off[pl], b0 = a.blk_off[pl], p0 = a.pa_off[pl];
    const int nblk = (int)(a.blk_off[pl + 1] - b0);
    const int jl = 4 * a.center_loc[pl] + (int)(a.cols[c] & 3);

    // sort the shifts by step count (bitonic over the next power of two >=
    // ns_pad, at most 256 keys; sentinels sort last)
    int nsort = 64;
    while (nsort < a.ns_pad) nsort <<= 1;
    constexpr int SENT = 0x7fffffff;
    for (int i = tid; i < 256; i += T)
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
    const int key = skey[tid];
    const bool live = key != SENT && (key & 1023) < a.ns;
    const int kof = live ? (key & 1023) : -1;
    const int nk = live ? (key >> 10) : 0;
    const double2 zk = live ? a.z[kof] : zero;
    const double2 sigma = live ? csub(zk, a.z[a.seed]) : zero;
    const int top = skey[a.ns_pad - 1] >> 10;
    int wtop = nk;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) wtop = max(wtop, __shfl_xor(wtop, off, 64));

    float2 S[64];
#pragma unroll
    for (int r = 0; r < 64; ++r) S[r] = make_float2(0.f, 0.f);
    double2 g = zero, y0 = zero;
    for (int hi = top - 1; hi >= 0; hi -= SHIFT_CH) {
        const int lo = hi - SHIFT_CH + 1 > 0 ? hi - SHIFT_CH + 1 : 0;
        const int nstep = hi - lo + 1;
        __syncthreads();  // the previous chunk has been consumed
        for (int idx = tid; idx < (nstep + 1) * 2; idx += T) {
            const int m = lo - 1 + (idx >> 1);
            sab[idx >> 1][idx & 1] = m >= 0 ? hab[2 * m + (idx & 1)] : zero;
        }
        for (int idx = tid; idx < nstep * 64; idx += T) srow[idx >> 6][idx & 63] = hist[(size_t)lo * 64 + idx];
        __syncthreads();
        if (lo >= wtop) continue;  // nothing for this wavefront in this chunk
        double2 ia_m = sab[hi - lo + 1][0], ba_m = sab[hi - lo + 1][1];
        for (int m = hi; m >= lo; --m) {
            const double2 ia_p = sab[m - lo][0], ba_p = sab[m - lo][1];
            if (m < nk) {
                const double2 diag = cadd(cadd(ia_m, ba_p), sigma);
                const double2 d = (m == nk - 1) ? diag : csub(diag, cmul(ba_m, g));
                const float2 gf = to_f(g);
                const float2 *rm = srow[m - lo];
#pragma unroll
                for (int r = 0; r < 64; ++r) {
                    if (r < nl) {
                        const float2 rv = rm[r];
                        S[r] = make_float2(fmaf(gf.x, S[r].x, fmaf(-gf.y, S[r].y, rv.x)),
                                           fmaf(gf.x, S[r].y, fmaf(gf.y, S[r].x, rv.y)));
                    }
                }
                const double2 inv = crcp_fast(d);
                if (m > 0) g = cmul(ia_p, inv);
                else y0 = inv;
            }
            ia_m = ia_p;
            ba_m = ba_p;
        }
    }
    // x~ = y0 S, staged in LDS (complex FP32) for the epilogue
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 64; ++r)
        if (r < nl) xt[r * a.ns_pad + tid] = nk > 0 ? to_f(cmul(y0, to_d(S[r]))) : make_float2(0.f, 0.f);
    __syncthreads();

    // FP64 variational estimate of G_jj: 2 x~_j - x~^T (z_k - H) x~, and the
    // true residual r = e_j - (z_k - H) x~ of the full iterate
    double2 quad = zero;
    double rr = 0.0;
    for (int Aa = 0; Aa < n_loc; ++Aa) {
        const int t0 = a.lrow[a0 + Aa];
        const int t1 = Aa + 1 < n_loc ? a.lrow[a0 + Aa + 1] : nblk;
        double2 hx[4] = {zero, zero, zero, zero};
        for (int t = t0; t < t1; ++t) {
            const int Bb = a.lblk[2 * (b0 + t)];
            const double *hb = &a.h[16 * (int64_t)a.lblk[2 * (b0 + t) + 1]];
            double2 xb[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) xb[q] = to_d(xt[(4 * Bb + q) * a.ns_pad + tid]);
#pragma unroll
            for (int oo = 0; oo < 4; ++oo)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    hx[oo].x = fma(hb[4 * oo + q], xb[q].x, hx[oo].x);
                    hx[oo].y = fma(hb[4 * oo + q], xb[q].y, hx[oo].y);
                }
        }
#pragma unroll
        for (int oo = 0; oo < 4; ++oo) {
            const double2 xi = to_d(xt[(4 * Aa + oo) * a.ns_pad + tid]);
            const double2 ax = csub(cmul(zk, xi), hx[oo]);
            quad = cfma(xi, ax, quad);
            const double tx = (4 * Aa + oo == jl ? 1.0 : 0.0) - ax.x, ty = -ax.y;
            rr = fma(tx, tx, fma(ty, ty, rr));
        }
    }
    const double2 xj = to_d(xt[jl * a.ns_pad + tid]);
    const double2 gjj = csub(make_double2(2.0 * xj.x, 2.0 * xj.y), quad);

    // A-posteriori bound: G_jj - G~_jj = r^T (z_k - H)^{-1} r, and z_k - H is
    // normal with ||(z_k - H)^{-1}||_2 <= 1 / Im z_k, so
    // |G_jj - G~_jj| <= ||r||^2 / Im z_k.  The column is accepted when the
    // largest bound over its shifts is within g_tol of max_k |G~_jj|;
    // otherwise its status becomes DRIFT.  resid receives ||r||.
    // a non-finite estimate or residual has no bound (fmax below would drop a NaN)
    const bool fin = isfinite(rr) && isfinite(gjj.x) && isfinite(gjj.y);
    const double bound = (live && nk > 0) ? (fin ? rr / zk.y : INFINITY) : 0.0;
    const double gmag = (live && nk > 0) ? sqrt(fma(gjj.x, gjj.x, gjj.y * gjj.y)) : 0.0;
    if (live && a.resid) a.resid[c * a.ns + kof] = sqrt(rr);
    double wb = bound, wg = gmag;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        wb = fmax(wb, __shfl_xor(wb, off, 64));
        wg = fmax(wg, __shfl_xor(wg, off, 64));
    }
    if (lane == 0) {
        rpart[wv] = wb;
        rpart[4 + wv] = wg;
    }
    __syncthreads();
    if (tid == 0) {
        double mb = 0.0, mg = 0.0;
        for (int v = 0; v < nwv; ++v) {
            mb = fmax(mb, rpart[v]);
            mg = fmax(mg, rpart[4 + v]);
        }
        // certified diagonal: SGF_DIAG_ONLY (the other rows are FP32-Krylov values)
        if (meta.status == SGF_CONVERGED) a.status[c] = mb <= a.g_tol * mg ? SGF_DIAG_ONLY : SGF_DRIFT;
    }
    __syncthreads();  // rpart is reused below

    // G rows on P and the density matrix
    const double2 wk = (kof >= 0 && a.w) ? a.w[kof] : zero;
    const int64_t out0 = a.proj_off[c];
    for (int r = 0; r < nrow; ++r) {  // uniform
        const int lrow_ = 4 * a.pa_loc[p0 + (r >> 2)] + (r & 3);
        double2 Gr = zero;
        if (nk > 0) Gr = lrow_ == jl ? gjj : to_d(xt[lrow_ * a.ns_pad + tid]);
        if (kof >= 0 && a.G) {
            a.G[2 * ((out0 + r) * a.ns + kof)] = Gr.x;
            a.G[2 * ((out0 + r) * a.ns + kof) + 1] = Gr.y;
        }
        if (kof >= 0 && a.gdiag && lrow_ == jl) {
            a.gdiag[2 * (c * a.ns + kof)] = Gr.x;
            a.gdiag[2 * (c * a.ns + kof) + 1] = Gr.y;
        }
        double t = kof >= 0 ? fma(wk.x, Gr.y, wk.y * Gr.x) : 0.0;
        t = wave_reduce(t);
        if (lane == 0) rpart[r * 4 + wv] = t;
    }
    __syncthreads();
    for (int r = tid; r < nrow; r += T) {
        double acc = 0.0;
        for (int v = 0; v < nwv; ++v) acc += rpart[r * 4 + v];
        a.rho[out0 + r] = -acc * INV_PI;
    }
}

}  // namespace

KernelFn pick_seed_mx(int M, int bmax) {
    if (bmax <= 6) {
        switch (M) {
            case 1: return k_seed_mx<1, 6>;
            case 2: return k_seed_mx<2, 6>;
            default: return k_seed_mx<4, 6>;
        }
    }
    switch (M) {
        case 1: return k_seed_mx<1, 8>;
        case 2: return k_seed_mx<2, 8>;
        default: return k_seed_mx<4, 8>;
    }
}

KernelFn shift_mx_kernel() { return k_shift_mx; }

}  // namespace sgf
