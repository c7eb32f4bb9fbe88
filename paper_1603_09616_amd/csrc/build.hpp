// build.hpp -- spatial hash shared by the builder and the subspace planner.
#pragma once

#include "common.hpp"

namespace sgf {

struct BuildHeader {
    double cell;        // cell edge (nm) = r_cut of the pattern
    int64_t nbuck;      // hash buckets (power of two)
    int64_t n_atoms;
    int64_t max_row;    // largest block-row length (bonds + diagonal)
};

// Views into the build workspace (same carve order on every call).
struct BuildLayout {
    BuildHeader *hdr;
    int64_t nbuck;
    int64_t *bucket;      // [nbuck+1] start of each bucket in sorted order
    int32_t *fill;        // [nbuck]
    int32_t *sorted_atom; // [n_atoms] atoms grouped by bucket
    int4 *sorted_cell;    // [n_atoms] integer cell of each sorted atom
    int64_t *row_cnt;     // [n_atoms+1] row lengths, then their prefix sum
    char *scan;           // prefix-sum scratch
    size_t bytes;
};

int64_t hash_buckets(int64_t n_atoms);
BuildLayout build_layout(int64_t n_atoms, void *base, size_t cap);

// Squared distance formed as (dx*dx + dy*dy) + dz*dz with every operation
// rounded separately (no fused multiply-add), so cutoff decisions are
// reproducible by any IEEE FP64 implementation that evaluates it that way.
__device__ __forceinline__ double dist2_exact(const double *a, const double *b) {
    const double dx = b[0] - a[0], dy = b[1] - a[1], dz = b[2] - a[2];
    return __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
}

__device__ __forceinline__ int4 cell_of(const double *r, double cell) {
    return make_int4((int)floor(r[0] / cell), (int)floor(r[1] / cell), (int)floor(r[2] / cell), 0);
}

__device__ __forceinline__ uint32_t hash_cell(int4 c, uint32_t mask) {
    return (((uint32_t)c.x * 73856093u) ^ ((uint32_t)c.y * 19349663u) ^ ((uint32_t)c.z * 83492791u)) & mask;
}

}  // namespace sgf
