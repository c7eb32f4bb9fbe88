// common.hip -- error state, version, prefix sum, FP32 shadow conversion.
#include "common.hpp"

namespace sgf {

static thread_local std::string g_last_error;

void set_error(const char *fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
}

// --- prefix sum ------------------------------------------------------------
constexpr int SCAN_T = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_T * SCAN_ITEMS;

// Block-level inclusive scan of one tile; writes the tile total to sums[bid].
__global__ __launch_bounds__(SCAN_T) void k_scan_tiles(int64_t *data, int64_t n, int64_t *sums) {
    __shared__ int64_t part[SCAN_T];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
    int64_t v[SCAN_ITEMS];
    int64_t run = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        int64_t x = (base + i < n) ? data[base + i] : 0;
        run += x;
        v[i] = run;
    }
    part[threadIdx.x] = run;
    __syncthreads();
    // Hillis-Steele over the thread totals (256 entries).
    for (int off = 1; off < SCAN_T; off <<= 1) {
        int64_t add = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
        __syncthreads();
        part[threadIdx.x] += add;
        __syncthreads();
    }
    const int64_t prefix = threadIdx.x > 0 ? part[threadIdx.x - 1] : 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i)
        if (base + i < n) data[base + i] = v[i] + prefix;
    if (sums && threadIdx.x == SCAN_T - 1) sums[blockIdx.x] = part[SCAN_T - 1];
}

// One workgroup scans the tile totals (exclusive result in place).
__global__ __launch_bounds__(SCAN_T) void k_scan_sums(int64_t *sums, int64_t nb) {
    __shared__ int64_t part[SCAN_T];
    __shared__ int64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t start = 0; start < nb; start += SCAN_T) {
        const int64_t i = start + threadIdx.x;
        const int64_t x = i < nb ? sums[i] : 0;
        part[threadIdx.x] = x;
        __syncthreads();
        for (int off = 1; off < SCAN_T; off <<= 1) {
            int64_t add = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
            __syncthreads();
            part[threadIdx.x] += add;
            __syncthreads();
        }
        if (i < nb) sums[i] = carry + part[threadIdx.x] - x;
        __syncthreads();
        if (threadIdx.x == SCAN_T - 1) carry += part[SCAN_T - 1];
        __syncthreads();
    }
}

__global__ __launch_bounds__(SCAN_T) void k_scan_add(int64_t *data, int64_t n, const int64_t *sums) {
    const int64_t add = sums[blockIdx.x];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    for (int i = threadIdx.x; i < SCAN_TILE; i += SCAN_T)
        if (base + i < n) data[base + i] += add;
}

size_t prefix_scratch_bytes(int64_t n) {
    const int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    return align_up((size_t)(nb > 0 ? nb : 1) * sizeof(int64_t));
}

sgf_status inclusive_scan_i64(int64_t *d_data, int64_t n, void *d_scratch, hipStream_t st) {
    if (n <= 0) return SGF_OK;
    const int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    int64_t *sums = static_cast<int64_t *>(d_scratch);
    k_scan_tiles<<<dim3((unsigned)nb), dim3(SCAN_T), 0, st>>>(d_data, n, sums);
    SGF_LAUNCHED();
    if (nb > 1) {
        k_scan_sums<<<1, SCAN_T, 0, st>>>(sums, nb);
        SGF_LAUNCHED();
        k_scan_add<<<dim3((unsigned)nb), dim3(SCAN_T), 0, st>>>(d_data, n, sums);
        SGF_LAUNCHED();
    }
    return SGF_OK;
}

// The same inclusive scan with no scratch, in three launches over tiles of
// SCAN_TILE items: (1) each tile scanned in place, so a full tile's last
// item holds the tile's total; (2) tile b adds the totals of tiles 0 .. b-1,
// read from those last items, to its other items (a full tile's last item
// is left alone, since later tiles still read it); (3) one workgroup turns
// the last items of the full tiles into their running sums.  Integer sums,
// so the result is that of the sequential scan.
__global__ __launch_bounds__(SCAN_T) void k_scan_carry_in(int64_t *data, int64_t n) {
    __shared__ int64_t wsum[SCAN_T / 64];
    const int64_t b = blockIdx.x + 1;  // tile 0 has nothing to add
    int64_t s = 0;
    for (int64_t j = threadIdx.x; j < b; j += SCAN_T) s += data[(j + 1) * SCAN_TILE - 1];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = s;
    __syncthreads();
    int64_t off = 0;
#pragma unroll
    for (int w = 0; w < SCAN_T / 64; ++w) off += wsum[w];
    const int64_t t0 = b * SCAN_TILE;
    const int64_t t1 = t0 + SCAN_TILE < n ? t0 + SCAN_TILE - 1 : n;  // a full tile keeps its last item
    for (int64_t i = t0 + threadIdx.x; i < t1; i += SCAN_T) data[i] += off;
}

__global__ __launch_bounds__(SCAN_T) void k_scan_tile_ends(int64_t *data, int64_t n_full) {
    __shared__ int64_t part[SCAN_T];
    int64_t carry = 0;  // uniform
    for (int64_t start = 0; start < n_full; start += SCAN_T) {
        const int64_t j = start + threadIdx.x;
        const int64_t x = j < n_full ? data[(j + 1) * SCAN_TILE - 1] : 0;
        part[threadIdx.x] = x;
        __syncthreads();
        for (int off = 1; off < SCAN_T; off <<= 1) {
            const int64_t add = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
            __syncthreads();
            part[threadIdx.x] += add;
            __syncthreads();
        }
        if (j < n_full) data[(j + 1) * SCAN_TILE - 1] = carry + part[threadIdx.x];
        carry += part[SCAN_T - 1];
        __syncthreads();  // part is rewritten by the next round
    }
}

sgf_status inclusive_scan_noscratch(int64_t *d_data, int64_t n, hipStream_t st) {
    if (n <= 0) return SGF_OK;
    const int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    k_scan_tiles<<<dim3((unsigned)nb), dim3(SCAN_T), 0, st>>>(d_data, n, nullptr);
    SGF_LAUNCHED();
    if (nb > 1) {
        k_scan_carry_in<<<dim3((unsigned)(nb - 1)), dim3(SCAN_T), 0, st>>>(d_data, n);
        SGF_LAUNCHED();
        // the full tiles: all but the last, which may be partial
        k_scan_tile_ends<<<1, SCAN_T, 0, st>>>(d_data, nb - 1);
        SGF_LAUNCHED();
    }
    return SGF_OK;
}

__global__ void k_to_f32(const double *in, int64_t n, float *out) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (float)in[i];
}

}  // namespace sgf

extern "C" const char *sgf_last_error(void) { return sgf::g_last_error.c_str(); }

extern "C" int sgf_version(void) { return 10000; }

extern "C" sgf_status sgf_to_f32(const double *d_in, int64_t n_values, float *d_out, void *stream) {
    SGF_REQUIRE(n_values >= 0, "sgf_to_f32: n_values < 0");
    SGF_REQUIRE(n_values == 0 || (d_in && d_out), "sgf_to_f32: NULL pointer");
    if (n_values == 0) return SGF_OK;
    int64_t blocks = (n_values + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    sgf::k_to_f32<<<dim3((unsigned)blocks), dim3(256), 0, sgf::as_stream(stream)>>>(d_in, n_values, d_out);
    SGF_LAUNCHED();
    return SGF_OK;
}
