// apply.hip -- global block-sparse operator application Y = (z S - H) X
// for n_rhs complex right-hand sides (stream mode: the matrix is read from
// HBM once per call).
//
// Layout (one right-hand side): one thread per orbital row (atom A, orbital
// o); the four threads of a block row read the four 32-byte (FP64) or
// 16-byte (FP32) rows of each 128/64-byte block, so a wavefront's 16 block
// rows stream 16 contiguous blocks per step.  X and Y are [n_orb][n_rhs] complex (right-hand sides
// contiguous per orbital), so a thread's neighbour reads are n_rhs
// consecutive complex values per column orbital, shared by the four threads
// of its block row through the cache.  Each block is 16 real values against
// 4 complex inputs per right-hand side: 64 flops per block and RHS over 128
// bytes of FP64 matrix (4 flop/B at 8 RHS), far below the FP64 ridge of
// ~10 flop/B, so the kernel is HBM-bound and plain FMA is the right engine.
#include "common.hpp"

namespace sgf {

namespace {

template <typename T> struct cplx;
template <> struct cplx<double> { using type = double2; };
template <> struct cplx<float> { using type = float2; };

template <typename T, int NRHS, bool HAS_S>
__global__ __launch_bounds__(256) void k_bsr_apply(int64_t n_atoms, const int32_t *__restrict__ row_ptr,
                                                   const int32_t *__restrict__ col, const T *__restrict__ h,
                                                   const T *__restrict__ s, double zr, double zi,
                                                   const typename cplx<T>::type *__restrict__ x,
                                                   typename cplx<T>::type *__restrict__ y) {
    using C = typename cplx<T>::type;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t A = gid >> 2;
    const int o = (int)(gid & 3);
    if (A >= n_atoms) return;
    T hx[NRHS], hy[NRHS], sx[NRHS], sy[NRHS];
#pragma unroll
    for (int r = 0; r < NRHS; ++r) hx[r] = hy[r] = sx[r] = sy[r] = T(0);
    const int t0 = row_ptr[A], t1 = row_ptr[A + 1];
    // Two blocks per trip: both blocks' rows and both neighbours' x are
    // loaded before either product, two loads in flight per thread instead
    // of one (same products in the same order).
    auto block = [&](const T (&hr)[4], const T (&sr)[4], const C (&v)[4][NRHS]) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int r = 0; r < NRHS; ++r) {
                hx[r] = fma(hr[q], v[q][r].x, hx[r]);
                hy[r] = fma(hr[q], v[q][r].y, hy[r]);
                if (HAS_S) {
                    sx[r] = fma(sr[q], v[q][r].x, sx[r]);
                    sy[r] = fma(sr[q], v[q][r].y, sy[r]);
                }
            }
    };
    auto load = [&](int t, T (&hr)[4], T (&sr)[4], C (&v)[4][NRHS]) {
        const int64_t B = col[t];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            hr[q] = h[16 * (int64_t)t + 4 * o + q];
            sr[q] = HAS_S ? s[16 * (int64_t)t + 4 * o + q] : T(0);
        }
        const C *xb = x + 4 * B * NRHS;
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int r = 0; r < NRHS; ++r) v[q][r] = xb[q * NRHS + r];
    };
    int t = t0;
    for (; t + 1 < t1; t += 2) {
        T h0[4], s0[4], h1[4], s1[4];
        C v0[4][NRHS], v1[4][NRHS];
        load(t, h0, s0, v0);
        load(t + 1, h1, s1, v1);
        block(h0, s0, v0);
        block(h1, s1, v1);
    }
    if (t < t1) {
        T h0[4], s0[4];
        C v0[4][NRHS];
        load(t, h0, s0, v0);
        block(h0, s0, v0);
    }
    const int64_t row = 4 * A + o;
    const T zx = (T)zr, zy = (T)zi;
#pragma unroll
    for (int r = 0; r < NRHS; ++r) {
        T ux, uy;  // S x (S = I: x itself)
        if (HAS_S) { ux = sx[r]; uy = sy[r]; }
        else { const C v = x[row * NRHS + r]; ux = v.x; uy = v.y; }
        C out;
        out.x = zx * ux - zy * uy - hx[r];
        out.y = zx * uy + zy * ux - hy[r];
        y[row * NRHS + r] = out;
    }
}

// Mapping with X staged in LDS: one thread per (block row A, group of RPT
// right-hand sides).  A workgroup first copies the rows of X that its block
// rows can reach -- its own atoms and APPLY_HALO atoms on either side, which
// covers bonded neighbours along a chain in chain order -- into LDS with
// coalesced 16-byte loads, and the block products read their neighbours from
// there (a neighbour outside that window, which an atom ordering without
// locality can produce, is read from global memory).  Every element of X
// then leaves HBM about once per call instead of once per referencing block:
// with the matrix streaming through L2 ahead of it, the neighbour reads of
// the unstaged mapping missed L2 and came back from HBM 1.5-1.7 times over.
// Measured on the 1,000,300-atom share: with one RHS the thread per orbital
// row without staging stays faster in both precisions (FP64 140 us; FP32 82
// us against 85 us staged, also with the next block loaded ahead); with 4
// and 8 RHS staging takes
// FP64 from 277 and 429 us to 211 and 308 us, and RPT 2 at 8 RHS (and at 4
// in FP32) halves the redundant block reads of the threads of a block row
// (FP32 x8: 260 -> 160 us).  Two blocks per loop trip then take FP32 x1
// from 81 to 71 us, x4 from 125 to 116 us and x8 from 160 to 156 us.
constexpr int APPLY_T = 256;
constexpr int APPLY_HALO = 2;

template <typename T, int NRHS, int RPT, bool HAS_S>
__global__ __launch_bounds__(APPLY_T) void k_bsr_apply_lx(int64_t n_atoms, const int32_t *__restrict__ row_ptr,
                                                         const int32_t *__restrict__ col, const T *__restrict__ h,
                                                         const T *__restrict__ s, double zr, double zi,
                                                         const typename cplx<T>::type *__restrict__ x,
                                                         typename cplx<T>::type *__restrict__ y) {
    using C = typename cplx<T>::type;
    constexpr int TPA = NRHS / RPT;                     // threads per block row
    constexpr int NA = APPLY_T / TPA;                   // block rows per workgroup
    constexpr int WIN = NA + 2 * APPLY_HALO;            // atoms of X staged
    constexpr int NV = HAS_S ? 32 : 16;                 // block values read per block
    __shared__ __align__(16) C xs[WIN * 4 * NRHS];
    const int64_t A0 = (int64_t)blockIdx.x * NA;
    const int64_t lo = A0 - APPLY_HALO > 0 ? A0 - APPLY_HALO : 0;
    const int64_t hi = A0 + NA + APPLY_HALO < n_atoms ? A0 + NA + APPLY_HALO : n_atoms;
    const int64_t A = A0 + threadIdx.x / TPA;
    const int r0 = (threadIdx.x % TPA) * RPT;
    const bool live = A < n_atoms;
    {
        // (hi - lo) * 4 * NRHS complex values, copied as 16-byte words
        constexpr int PER = 16 / (int)sizeof(C);        // complex values per 16 bytes (1 or 2)
        const int64_t nw = (hi - lo) * 4 * NRHS / PER;
        const float4 *src = reinterpret_cast<const float4 *>(x + lo * 4 * NRHS);
        float4 *dst = reinterpret_cast<float4 *>(xs);
        for (int64_t i = threadIdx.x; i < nw; i += APPLY_T) dst[i] = src[i];
    }
    __syncthreads();
    if (!live) return;
    const int t0 = row_ptr[A], t1 = row_ptr[A + 1];
    T hx[4][RPT], hy[4][RPT], sx[4][RPT], sy[4][RPT];
#pragma unroll
    for (int o = 0; o < 4; ++o)
#pragma unroll
        for (int u = 0; u < RPT; ++u) hx[o][u] = hy[o][u] = sx[o][u] = sy[o][u] = T(0);
    auto load = [&](int t, T (&hb)[NV], C (&v)[4][RPT]) {
        const int64_t B = col[t];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            hb[i] = h[16 * (int64_t)t + i];
            if (HAS_S) hb[16 + i] = s[16 * (int64_t)t + i];
        }
        if (B >= lo && B < hi) {
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int u = 0; u < RPT; ++u) v[q][u] = xs[((B - lo) * 4 + q) * NRHS + r0 + u];
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int u = 0; u < RPT; ++u) v[q][u] = x[(4 * B + q) * NRHS + r0 + u];
        }
    };
    auto block = [&](const T (&hb)[NV], const C (&v)[4][RPT]) {
#pragma unroll
        for (int o = 0; o < 4; ++o)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const T hv = hb[4 * o + q];
#pragma unroll
                for (int u = 0; u < RPT; ++u) {
                    hx[o][u] = fma(hv, v[q][u].x, hx[o][u]);
                    hy[o][u] = fma(hv, v[q][u].y, hy[o][u]);
                    if (HAS_S) {
                        const T sv = hb[16 + 4 * o + q];
                        sx[o][u] = fma(sv, v[q][u].x, sx[o][u]);
                        sy[o][u] = fma(sv, v[q][u].y, sy[o][u]);
                    }
                }
            }
    };
    // FP32: two blocks per trip, both loaded before either product (FP64
    // keeps one: at 8 right-hand sides the second block's registers cost
    // more than the extra load in flight gains)
    constexpr bool PAIR = sizeof(T) == 4;
    int t = t0;
    for (; PAIR && t + 1 < t1; t += 2) {
        // both blocks' values first, then both neighbours' x, then the products
        const int64_t Bp[2] = {col[t], col[t + 1]};
        T hp[2][NV];
#pragma unroll
        for (int e = 0; e < 2; ++e)
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                hp[e][i] = h[16 * (int64_t)(t + e) + i];
                if (HAS_S) hp[e][16 + i] = s[16 * (int64_t)(t + e) + i];
            }
        C vv[2][4][RPT];
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int64_t B = Bp[e];
            if (B >= lo && B < hi) {
#pragma unroll
                for (int q = 0; q < 4; ++q)
#pragma unroll
                    for (int u = 0; u < RPT; ++u) vv[e][q][u] = xs[((B - lo) * 4 + q) * NRHS + r0 + u];
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q)
#pragma unroll
                    for (int u = 0; u < RPT; ++u) vv[e][q][u] = x[(4 * B + q) * NRHS + r0 + u];
            }
        }
        block(hp[0], vv[0]);
        block(hp[1], vv[1]);
    }
    for (; t < t1; ++t) {
        T hb[NV];   // the block of H (and of S)
        C v[4][RPT];
        load(t, hb, v);
        block(hb, v);
    }
    const T zx = (T)zr, zy = (T)zi;
#pragma unroll
    for (int o = 0; o < 4; ++o)
#pragma unroll
        for (int u = 0; u < RPT; ++u) {
            T ux, uy;  // S x (S = I: x itself)
            if (HAS_S) { ux = sx[o][u]; uy = sy[o][u]; }
            else { const C v = xs[((A - lo) * 4 + o) * NRHS + r0 + u]; ux = v.x; uy = v.y; }
            C out;
            out.x = zx * ux - zy * uy - hx[o][u];
            out.y = zx * uy + zy * ux - hy[o][u];
            y[(4 * A + o) * NRHS + r0 + u] = out;
        }
}

template <typename T, bool HAS_S>
void launch_apply(int n_rhs, dim3 grid, hipStream_t st, int64_t n_atoms, const int32_t *row_ptr, const int32_t *col,
                  const T *h, const T *s, double zr, double zi, const typename cplx<T>::type *x,
                  typename cplx<T>::type *y) {
    // one right-hand side: one thread per orbital row; otherwise a thread per
    // (block row, RPT right-hand sides) with X staged in LDS
    constexpr bool F32 = sizeof(T) == 4;
    auto blocks = [&](int tpa) { return dim3((unsigned)((n_atoms * tpa + APPLY_T - 1) / APPLY_T)); };
    switch (n_rhs) {
        case 1:
            k_bsr_apply<T, 1, HAS_S><<<grid, 256, 0, st>>>(n_atoms, row_ptr, col, h, s, zr, zi, x, y);
            break;
        case 2: k_bsr_apply_lx<T, 2, 1, HAS_S><<<blocks(2), APPLY_T, 0, st>>>(n_atoms, row_ptr, col, h, s, zr, zi, x, y); break;
        case 4:
            if (F32) k_bsr_apply_lx<T, 4, 2, HAS_S><<<blocks(2), APPLY_T, 0, st>>>(n_atoms, row_ptr, col, h, s, zr, zi, x, y);
            else k_bsr_apply_lx<T, 4, 1, HAS_S><<<blocks(4), APPLY_T, 0, st>>>(n_atoms, row_ptr, col, h, s, zr, zi, x, y);
            break;
        default: k_bsr_apply_lx<T, 8, 2, HAS_S><<<blocks(4), APPLY_T, 0, st>>>(n_atoms, row_ptr, col, h, s, zr, zi, x, y); break;
    }
}

}  // namespace

}  // namespace sgf

using namespace sgf;

extern "C" sgf_status sgf_bsr_apply(const sgf_system *sys, int32_t precision, int32_t n_rhs, const double *z,
                                    const void *d_x, void *d_y, void *stream) {
    SGF_REQUIRE(sys && z && d_x && d_y, "sgf_bsr_apply: NULL argument");
    SGF_REQUIRE(sys->row_ptr && sys->col && sys->n_atoms > 0, "sgf_bsr_apply: system incomplete");
    SGF_REQUIRE(precision == 0 || precision == 1, "sgf_bsr_apply: precision must be 0 (FP64) or 1 (FP32)");
    SGF_REQUIRE(n_rhs == 1 || n_rhs == 2 || n_rhs == 4 || n_rhs == 8, "sgf_bsr_apply: n_rhs must be 1, 2, 4 or 8");
    SGF_REQUIRE(d_x != d_y, "sgf_bsr_apply: d_x and d_y must not alias");
    SGF_REQUIRE(reinterpret_cast<uintptr_t>(d_x) % 16 == 0 && reinterpret_cast<uintptr_t>(d_y) % 16 == 0,
                "sgf_bsr_apply: d_x and d_y must be 16-byte aligned");
    const bool has_s = precision == 0 ? sys->s != nullptr : sys->s32 != nullptr;
    if (precision == 0) SGF_REQUIRE(sys->h, "sgf_bsr_apply: h is NULL");
    else SGF_REQUIRE(sys->h32 && (!sys->s || sys->s32), "sgf_bsr_apply: FP32 needs h32 (and s32 when S != I)");
    const int64_t threads = 4 * sys->n_atoms;
    const dim3 grid((unsigned)((threads + 255) / 256));
    hipStream_t st = as_stream(stream);
    const double zr = z[0], zi = z[1];
    if (precision == 0) {
        const double2 *x = static_cast<const double2 *>(d_x);
        double2 *y = static_cast<double2 *>(d_y);
        if (has_s) launch_apply<double, true>(n_rhs, grid, st, sys->n_atoms, sys->row_ptr, sys->col, sys->h, sys->s, zr, zi, x, y);
        else launch_apply<double, false>(n_rhs, grid, st, sys->n_atoms, sys->row_ptr, sys->col, sys->h, nullptr, zr, zi, x, y);
    } else {
        const float2 *x = static_cast<const float2 *>(d_x);
        float2 *y = static_cast<float2 *>(d_y);
        if (has_s) launch_apply<float, true>(n_rhs, grid, st, sys->n_atoms, sys->row_ptr, sys->col, sys->h32, sys->s32, zr, zi, x, y);
        else launch_apply<float, false>(n_rhs, grid, st, sys->n_atoms, sys->row_ptr, sys->col, sys->h32, nullptr, zr, zi, x, y);
    }
    SGF_LAUNCHED();
    return SGF_OK;
}
