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
    for (int t = t0; t < t1; ++t) {
        const int64_t B = col[t];
        T hr[4], sr[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            hr[q] = h[16 * (int64_t)t + 4 * o + q];
            if (HAS_S) sr[q] = s[16 * (int64_t)t + 4 * o + q];
        }
        const C *xb = x + 4 * B * NRHS;
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int r = 0; r < NRHS; ++r) {
                const C v = xb[q * NRHS + r];
                hx[r] = fma(hr[q], v.x, hx[r]);
                hy[r] = fma(hr[q], v.y, hy[r]);
                if (HAS_S) {
                    sx[r] = fma(sr[q], v.x, sx[r]);
                    sy[r] = fma(sr[q], v.y, sy[r]);
                }
            }
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

// Multi-RHS mapping: one thread per (block row A, right-hand side r).  The
// thread reads whole blocks (the n_rhs threads of a block row read the same
// block, merged by the coalescer) and only its own column of X, once per
// block, and writes the four outputs of its block row; consecutive threads
// write consecutive right-hand sides.
template <typename T, int NRHS, bool HAS_S>
__global__ __launch_bounds__(256) void k_bsr_apply_br(int64_t n_atoms, const int32_t *__restrict__ row_ptr,
                                                      const int32_t *__restrict__ col, const T *__restrict__ h,
                                                      const T *__restrict__ s, double zr, double zi,
                                                      const typename cplx<T>::type *__restrict__ x,
                                                      typename cplx<T>::type *__restrict__ y) {
    using C = typename cplx<T>::type;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t A = gid / NRHS;
    const int r = (int)(gid - A * NRHS);
    if (A >= n_atoms) return;
    T hx[4], hy[4], sx[4], sy[4];
#pragma unroll
    for (int o = 0; o < 4; ++o) hx[o] = hy[o] = sx[o] = sy[o] = T(0);
    const int t0 = row_ptr[A], t1 = row_ptr[A + 1];
    for (int t = t0; t < t1; ++t) {
        const int64_t B = col[t];
        C v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = x[(4 * B + q) * NRHS + r];
        const T *hb = h + 16 * (int64_t)t;
        const T *sb = HAS_S ? s + 16 * (int64_t)t : nullptr;
#pragma unroll
        for (int o = 0; o < 4; ++o)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const T hv = hb[4 * o + q];
                hx[o] = fma(hv, v[q].x, hx[o]);
                hy[o] = fma(hv, v[q].y, hy[o]);
                if (HAS_S) {
                    const T sv = sb[4 * o + q];
                    sx[o] = fma(sv, v[q].x, sx[o]);
                    sy[o] = fma(sv, v[q].y, sy[o]);
                }
            }
    }
    const T zx = (T)zr, zy = (T)zi;
#pragma unroll
    for (int o = 0; o < 4; ++o) {
        const int64_t idx = (4 * A + o) * NRHS + r;
        T ux, uy;
        if (HAS_S) { ux = sx[o]; uy = sy[o]; }
        else { const C v = x[idx]; ux = v.x; uy = v.y; }
        C out;
        out.x = zx * ux - zy * uy - hx[o];
        out.y = zx * uy + zy * ux - hy[o];
        y[idx] = out;
    }
}

template <typename T, bool HAS_S>
void launch_apply(int n_rhs, dim3 grid, hipStream_t st, int64_t n_atoms, const int32_t *row_ptr, const int32_t *col,
                  const T *h, const T *s, double zr, double zi, const typename cplx<T>::type *x,
                  typename cplx<T>::type *y) {
    // one thread per orbital row for a single right-hand side; one thread per
    // (block row, right-hand side) otherwise (n_atoms * n_rhs threads)
    const dim3 gbr((unsigned)((n_atoms * n_rhs + 255) / 256));
    switch (n_rhs) {
        case 1: k_bsr_apply<T, 1, HAS_S><<<grid, 256, 0, st>>>(n_atoms, row_ptr, col, h, s, zr, zi, x, y); break;
        case 2: k_bsr_apply_br<T, 2, HAS_S><<<gbr, 256, 0, st>>>(n_atoms, row_ptr, col, h, s, zr, zi, x, y); break;
        case 4: k_bsr_apply_br<T, 4, HAS_S><<<gbr, 256, 0, st>>>(n_atoms, row_ptr, col, h, s, zr, zi, x, y); break;
        default: k_bsr_apply_br<T, 8, HAS_S><<<gbr, 256, 0, st>>>(n_atoms, row_ptr, col, h, s, zr, zi, x, y); break;
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
