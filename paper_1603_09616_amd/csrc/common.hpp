// common.hpp -- shared helpers of the gfx950 library: error state, complex
// arithmetic, wavefront reductions and a device-wide prefix sum.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/sgf.h"

namespace sgf {

// ---------------------------------------------------------------------------
// Errors: a thread-local message behind sgf_last_error().
// ---------------------------------------------------------------------------
void set_error(const char *fmt, ...);

#define SGF_REQUIRE(cond, ...)                 \
    do {                                       \
        if (!(cond)) {                         \
            ::sgf::set_error(__VA_ARGS__);     \
            return SGF_EINVAL;                 \
        }                                      \
    } while (0)

#define SGF_HIP(call)                                                                       \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess) {                                                             \
            ::sgf::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, \
                             __LINE__);                                                     \
            return SGF_EHIP;                                                                \
        }                                                                                   \
    } while (0)

#define SGF_LAUNCHED()                                                                        \
    do {                                                                                      \
        hipError_t e_ = hipGetLastError();                                                    \
        if (e_ != hipSuccess) {                                                               \
            ::sgf::set_error("kernel launch failed: %s (%s:%d)", hipGetErrorString(e_), __FILE__, \
                             __LINE__);                                                       \
            return SGF_EHIP;                                                                  \
        }                                                                                     \
    } while (0)

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

inline size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

// Bump allocator over a caller-provided workspace.
struct Carve {
    char *base;
    size_t used = 0, cap;
    Carve(void *b, size_t c) : base(static_cast<char *>(b)), cap(c) {}
    template <class T>
    T *take(size_t n) {
        size_t off = align_up(used);
        used = off + n * sizeof(T);
        return base ? reinterpret_cast<T *>(base + off) : nullptr;
    }
    bool fits() const { return used <= cap; }
};

// ---------------------------------------------------------------------------
// Complex double helpers (double2 = re, im).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a*b + c
__device__ __forceinline__ double2 cfma(double2 a, double2 b, double2 c) {
    return make_double2(fma(a.x, b.x, fma(-a.y, b.y, c.x)), fma(a.x, b.y, fma(a.y, b.x, c.y)));
}
// real * complex
__device__ __forceinline__ double2 rmul(double r, double2 b) { return make_double2(r * b.x, r * b.y); }
// 1 / a: both parts are first scaled by a power of two (exact) so that |a|^2
// neither overflows nor underflows; one correctly rounded division.  The
// seed recurrences use this one: COCG has no look-ahead, so near a
// breakdown its trajectory is sensitive to the rounding of its scalars.
__device__ __forceinline__ double2 crcp(double2 a) {
    const int e = ilogb(fmax(fabs(a.x), fabs(a.y)));
    const double x = ldexp(a.x, -e), y = ldexp(a.y, -e);
    const double inv = 1.0 / fma(x, x, y * y);
    return make_double2(ldexp(x * inv, -e), ldexp(-y * inv, -e));
}
// 1 / a = conj(a) / |a|^2 with a shorter dependency chain, for the pivots of
// the shift pass (which feed nothing back into the Krylov process): when
// |a|^2 is comfortably inside the normal range its reciprocal comes from the
// hardware estimate refined by two Newton steps r <- r + r (1 - n r) (each
// squares the relative error; the result is within about an ulp), otherwise
// the scaled division above.
__device__ __forceinline__ double2 crcp_fast(double2 a) {
    const double n = fma(a.x, a.x, a.y * a.y);
    if (n >= 0x1p-1000 && n <= 0x1p+1000) {
        double r = __builtin_amdgcn_rcp(n);
        r = fma(r, fma(-n, r, 1.0), r);
        r = fma(r, fma(-n, r, 1.0), r);
        return make_double2(a.x * r, -a.y * r);
    }
    return crcp(a);
}
__device__ __forceinline__ double2 cdiv(double2 a, double2 b) { return cmul(a, crcp(b)); }
__device__ __forceinline__ bool cfinite(double2 a) { return isfinite(a.x) && isfinite(a.y); }

// ---------------------------------------------------------------------------
// Wavefront (64-lane) sums via cross-lane shuffles; fixed order, so every
// lane gets the same bits and repeated runs agree bit for bit.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// ---------------------------------------------------------------------------
// LDS ordering inside one wavefront: every LDS access issued before this point
// has completed (lgkmcnt(0)) and the compiler keeps memory accesses on their
// side of it.  Unlike __syncthreads() it does not wait for outstanding global
// loads or stores (vmcnt) and it involves no other wavefront.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void wave_lds_fence() {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0xC07F);  // gfx9 encoding: vmcnt=63, expcnt=7, lgkmcnt=0
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// ---------------------------------------------------------------------------
// DPP wavefront reduction (CDNA row operations).  The partial sums climb to
// the last lane of each 16-lane row (row_shr 1, 2, 4, 8), rows 1 and 3 add
// row 0 / row 2 (row_bcast15), rows 2 and 3 add lane 31 (row_bcast31); lane 63
// then holds the total, which readlane broadcasts.  Fixed order, so the
// result is the same bit pattern on every run.
// ---------------------------------------------------------------------------
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_take(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROW_MASK, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROW_MASK, 0xf, false);
    return __hiloint2double(hi, lo);
}
// Shift within rows; lanes without a source read zero (bound control), so
// no destination needs clearing first.
template <int CTRL>
__device__ __forceinline__ double dpp_shr(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wave_reduce(double v) {
    v += dpp_shr<0x111>(v);  // row_shr:1
    v += dpp_shr<0x112>(v);  // row_shr:2
    v += dpp_shr<0x114>(v);  // row_shr:4
    v += dpp_shr<0x118>(v);  // row_shr:8
    v += dpp_take<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
    v += dpp_take<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
    return __hiloint2double(hi, lo);
}

// Wavefront sums of NV doubles per lane (NV <= 4), with the cross-lane moves
// done by the LDS instead of VALU DPP moves.  Each lane stores its values in
// buf (NV * 64 doubles, value v of lane l at buf[64 v + l]); lane 16 v + c of
// row v adds the four values of lanes 4c .. 4c + 3 in order, and a row
// reduction (row_shr 1, 2, 4, 8) leaves the sum of value v in lane 16 v + 15.
// About 5 + NV VALU operations per value instead of 20 for wave_reduce.  The
// caller must not touch buf again before the returned sums are used.
template <int NV>
__device__ __forceinline__ void wave_sum_lds(const double (&v)[NV], double *buf, double (&out)[NV]) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int i = 0; i < NV; ++i) buf[64 * i + lane] = v[i];
    wave_lds_fence();
    const int row = lane >> 4;
    const double *src = buf + 64 * (row < NV ? row : NV - 1) + 4 * (lane & 15);
    const double2 a = reinterpret_cast<const double2 *>(src)[0], b = reinterpret_cast<const double2 *>(src)[1];
    double t = ((a.x + a.y) + b.x) + b.y;
    t += dpp_shr<0x111>(t);  // row_shr:1
    t += dpp_shr<0x112>(t);  // row_shr:2
    t += dpp_shr<0x114>(t);  // row_shr:4
    t += dpp_shr<0x118>(t);  // row_shr:8
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        const int lo = __builtin_amdgcn_readlane(__double2loint(t), 16 * i + 15);
        const int hi = __builtin_amdgcn_readlane(__double2hiint(t), 16 * i + 15);
        out[i] = __hiloint2double(hi, lo);
    }
}

// ---------------------------------------------------------------------------
// Device-wide inclusive prefix sum of int64 values in place (three kernels:
// per-block scan, scan of block totals, add-back).  Scratch: prefix_scratch().
// ---------------------------------------------------------------------------
size_t prefix_scratch_bytes(int64_t n);
sgf_status inclusive_scan_i64(int64_t *d_data, int64_t n, void *d_scratch, hipStream_t st);
// Same result with no scratch (three launches; the tile totals are read
// from the tiles themselves).
sgf_status inclusive_scan_noscratch(int64_t *d_data, int64_t n, hipStream_t st);

}  // namespace sgf
