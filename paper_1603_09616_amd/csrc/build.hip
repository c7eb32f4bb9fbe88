// build.hip -- neighbour search and tight-binding assembly on the GPU.
//
// Atoms are binned into cubic cells of edge r_cut; cells are addressed through
// a power-of-two spatial hash so that the workspace depends only on the atom
// count (no bounding box, no host pass).  A bond is a pair within r_cut; each
// block row lists its bonds plus the diagonal, sorted by column.
#include "build.hpp"

#include <cstdlib>

namespace sgf {

constexpr int BUILD_T = 256;
constexpr int NB_MAX = 64;  // bonds per atom supported by the fill kernel

int64_t hash_buckets(int64_t n_atoms) {
    int64_t nb = 1024;
    while (nb < 2 * n_atoms) nb <<= 1;
    return nb;
}

BuildLayout build_layout(int64_t n_atoms, void *base, size_t cap) {
    BuildLayout L;
    Carve c(base, cap);
    L.nbuck = hash_buckets(n_atoms);
    L.hdr = c.take<BuildHeader>(1);
    L.bucket = c.take<int64_t>(L.nbuck + 1);
    L.fill = c.take<int32_t>(L.nbuck);
    L.sorted_atom = c.take<int32_t>(n_atoms);
    L.sorted_cell = c.take<int4>(n_atoms);
    L.row_cnt = c.take<int64_t>(n_atoms + 1);
    const int64_t big = L.nbuck > n_atoms ? L.nbuck : n_atoms;
    L.scan = c.take<char>(prefix_scratch_bytes(big + 1));
    L.bytes = c.used;
    return L;
}

// ---------------------------------------------------------------------------
__global__ void k_zero_i64(int64_t *p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}
__global__ void k_zero_i32(int32_t *p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

__global__ void k_init_header(BuildHeader *h, double cell, int64_t nbuck, int64_t n_atoms) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        h->cell = cell;
        h->nbuck = nbuck;
        h->n_atoms = n_atoms;
        h->max_row = 0;
    }
}

__global__ __launch_bounds__(BUILD_T) void k_hash_count(const double *xyz, int64_t n, BuildLayout L, double cell) {
    const int64_t a = (int64_t)blockIdx.x * BUILD_T + threadIdx.x;
    if (a >= n) return;
    const int4 c = cell_of(&xyz[3 * a], cell);
    const uint32_t b = hash_cell(c, (uint32_t)(L.nbuck - 1));
    atomicAdd(reinterpret_cast<unsigned long long *>(&L.bucket[b + 1]), 1ull);
}

__global__ __launch_bounds__(BUILD_T) void k_hash_scatter(const double *xyz, int64_t n, BuildLayout L, double cell) {
    const int64_t a = (int64_t)blockIdx.x * BUILD_T + threadIdx.x;
    if (a >= n) return;
    const int4 c = cell_of(&xyz[3 * a], cell);
    const uint32_t b = hash_cell(c, (uint32_t)(L.nbuck - 1));
    const int64_t pos = L.bucket[b] + atomicAdd(&L.fill[b], 1);
    L.sorted_atom[pos] = (int32_t)a;
    L.sorted_cell[pos] = c;
}

// Visit every atom q != a within r_cut of atom a (any order).
template <class F>
__device__ __forceinline__ void for_bonds(const double *xyz, int64_t a, const BuildLayout &L, double cell,
                                          double rc2, F &&f) {
    const double *ra = &xyz[3 * a];
    const int4 c = cell_of(ra, cell);
    const uint32_t mask = (uint32_t)(L.nbuck - 1);
    for (int dx = -1; dx <= 1; ++dx)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dz = -1; dz <= 1; ++dz) {
                const int4 t = make_int4(c.x + dx, c.y + dy, c.z + dz, 0);
                const uint32_t b = hash_cell(t, mask);
                for (int64_t i = L.bucket[b]; i < L.bucket[b + 1]; ++i) {
                    const int4 qc = L.sorted_cell[i];
                    if (qc.x != t.x || qc.y != t.y || qc.z != t.z) continue;  // another cell in this bucket
                    const int32_t q = L.sorted_atom[i];
                    if (q == a) continue;
                    if (dist2_exact(ra, &xyz[3 * (int64_t)q]) <= rc2) f(q);
                }
            }
}

__global__ __launch_bounds__(BUILD_T) void k_bond_count(const double *xyz, int64_t n, BuildLayout L, double cell,
                                                        double rc2) {
    const int64_t a = (int64_t)blockIdx.x * BUILD_T + threadIdx.x;
    if (a >= n) return;
    int64_t k = 0;
    for_bonds(xyz, a, L, cell, rc2, [&](int32_t) { ++k; });
    L.row_cnt[a + 1] = k + 1;
    atomicMax(reinterpret_cast<unsigned long long *>(&L.hdr->max_row), (unsigned long long)(k + 1));
}

__global__ void k_row_ptr(const int64_t *cnt, int64_t n, int32_t *row_ptr) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= n; i += (int64_t)gridDim.x * blockDim.x)
        row_ptr[i] = i == 0 ? 0 : (int32_t)cnt[i];
}

// Slater-Koster block for the bond a -> b, written row-major into blk[16].
__device__ void sk_block(const sgf_tb_params &p, const double *ra, const double *rb, double *blk) {
    const double d0 = rb[0] - ra[0], d1 = rb[1] - ra[1], d2 = rb[2] - ra[2];
    const double r = sqrt(dist2_exact(ra, rb));
    const double cs[3] = {d0 / r, d1 / r, d2 / r};
    const double f = pow(p.r0 / r, p.power);
    blk[0] = p.v_sss * f;
#pragma unroll
    for (int A = 0; A < 3; ++A) {
        blk[1 + A] = cs[A] * p.v_sps * f;
        blk[4 * (1 + A)] = -cs[A] * p.v_sps * f;
#pragma unroll
        for (int B = 0; B < 3; ++B)
            blk[4 * (1 + A) + 1 + B] = (cs[A] * cs[B] * (p.v_pps - p.v_ppp) + (A == B ? p.v_ppp : 0.0)) * f;
    }
}

__global__ __launch_bounds__(BUILD_T) void k_bond_fill(const double *xyz, const double *onsite, int64_t n,
                                                       BuildLayout L, sgf_tb_params p, const int32_t *row_ptr,
                                                       int32_t *col, double *h, double *s) {
    const int64_t a = (int64_t)blockIdx.x * BUILD_T + threadIdx.x;
    if (a >= n) return;
    int32_t nb[NB_MAX];
    int k = 0;
    for_bonds(xyz, a, L, L.hdr->cell, p.r_cut * p.r_cut, [&](int32_t q) {
        if (k < NB_MAX - 1) nb[k] = q;
        ++k;
    });
    if (k > NB_MAX - 1) return;  // host rejected this before launching
    nb[k++] = (int32_t)a;
    for (int i = 1; i < k; ++i) {  // insertion sort: rows hold a handful of bonds
        const int32_t v = nb[i];
        int j = i - 1;
        while (j >= 0 && nb[j] > v) {
            nb[j + 1] = nb[j];
            --j;
        }
        nb[j + 1] = v;
    }
    const int64_t base = row_ptr[a];
    for (int i = 0; i < k; ++i) {
        const int32_t b = nb[i];
        col[base + i] = b;
        double blk[16];
        if (b == a) {
#pragma unroll
            for (int e = 0; e < 16; ++e) blk[e] = 0.0;
#pragma unroll
            for (int o = 0; o < 4; ++o) blk[5 * o] = onsite ? onsite[4 * a + o] : (o == 0 ? p.e_s : p.e_p);
        } else {
            sk_block(p, &xyz[3 * a], &xyz[3 * (int64_t)b], blk);
        }
        double *dst = &h[16 * (base + i)];
#pragma unroll
        for (int e = 0; e < 16; ++e) dst[e] = blk[e];
        if (s) {
            double *ds = &s[16 * (base + i)];
            double v = 1.0;
            if (b != a) {
                const double r = sqrt(dist2_exact(&xyz[3 * a], &xyz[3 * (int64_t)b]));
                v = p.s_amp * exp(-(r - p.r0) / p.s_decay);
            }
#pragma unroll
            for (int e = 0; e < 16; ++e) ds[e] = (e % 5 == 0) ? v : 0.0;
        }
    }
}

__global__ void k_chain(int64_t nb, const double *eps, double t, int32_t *row_ptr, int32_t *col, double *h) {
    const int64_t A = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (A > nb) return;
    row_ptr[A] = A == 0 ? 0 : (int32_t)(nb == 1 ? 1 : (A == nb ? 3 * nb - 2 : 3 * A - 1));
    if (A == nb) return;
    int64_t pos = A == 0 ? 0 : 3 * A - 1;
    for (int64_t B = A - 1; B <= A + 1; ++B) {
        if (B < 0 || B >= nb) continue;
        col[pos] = (int32_t)B;
        double *blk = &h[16 * pos];
        for (int o = 0; o < 4; ++o)
            for (int q = 0; q < 4; ++q) {
                const int64_t i = 4 * A + o, j = 4 * B + q;
                blk[4 * o + q] = (i == j) ? eps[i] : ((i - j == 1 || j - i == 1) ? t : 0.0);
            }
        ++pos;
    }
}

static unsigned grid_for(int64_t n, int t = BUILD_T) { return (unsigned)((n + t - 1) / t > 0 ? (n + t - 1) / t : 1); }

}  // namespace sgf

using namespace sgf;

extern "C" sgf_status sgf_build_workspace(int64_t n_atoms, size_t *ws_bytes) {
    SGF_REQUIRE(n_atoms > 0 && n_atoms < (int64_t)1 << 30, "sgf_build_workspace: n_atoms out of range");
    SGF_REQUIRE(ws_bytes, "sgf_build_workspace: ws_bytes is NULL");
    *ws_bytes = build_layout(n_atoms, nullptr, 0).bytes;
    return SGF_OK;
}

// The neighbour search behind sgf_build_pattern and sgf_hamiltonian_size;
// d_row_ptr NULL counts the blocks without writing the row pointers.
static sgf_status bond_pattern(int64_t n_atoms, const double *d_xyz, double r_cut, void *d_ws, size_t ws_bytes,
                               int32_t *d_row_ptr, int64_t *nnzb, void *stream) {
    SGF_REQUIRE(n_atoms > 0 && n_atoms < (int64_t)1 << 30, "sgf_build_pattern: n_atoms out of range");
    SGF_REQUIRE(d_xyz && d_ws && nnzb, "sgf_build_pattern: NULL pointer");
    SGF_REQUIRE(r_cut > 0 && r_cut < 1e6, "sgf_build_pattern: r_cut must be positive");
    BuildLayout L = build_layout(n_atoms, d_ws, ws_bytes);
    SGF_REQUIRE(L.bytes <= ws_bytes, "sgf_build_pattern: workspace %zu bytes < %zu", ws_bytes, L.bytes);
    hipStream_t st = as_stream(stream);
    k_init_header<<<1, 64, 0, st>>>(L.hdr, r_cut, L.nbuck, n_atoms);
    k_zero_i64<<<grid_for(L.nbuck + 1), BUILD_T, 0, st>>>(L.bucket, L.nbuck + 1);
    k_zero_i32<<<grid_for(L.nbuck), BUILD_T, 0, st>>>(L.fill, L.nbuck);
    k_zero_i64<<<1, 64, 0, st>>>(L.row_cnt, 1);
    SGF_LAUNCHED();
    k_hash_count<<<grid_for(n_atoms), BUILD_T, 0, st>>>(d_xyz, n_atoms, L, r_cut);
    SGF_LAUNCHED();
    sgf_status rc = inclusive_scan_i64(L.bucket + 1, L.nbuck, L.scan, st);
    if (rc) return rc;
    k_hash_scatter<<<grid_for(n_atoms), BUILD_T, 0, st>>>(d_xyz, n_atoms, L, r_cut);
    k_bond_count<<<grid_for(n_atoms), BUILD_T, 0, st>>>(d_xyz, n_atoms, L, r_cut, r_cut * r_cut);
    SGF_LAUNCHED();
    rc = inclusive_scan_i64(L.row_cnt + 1, n_atoms, L.scan, st);
    if (rc) return rc;
    if (d_row_ptr) {
        k_row_ptr<<<grid_for(n_atoms + 1), BUILD_T, 0, st>>>(L.row_cnt, n_atoms, d_row_ptr);
        SGF_LAUNCHED();
    }
    int64_t total = 0;
    BuildHeader hdr;
    SGF_HIP(hipMemcpyAsync(&total, L.row_cnt + n_atoms, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    SGF_HIP(hipMemcpyAsync(&hdr, L.hdr, sizeof(BuildHeader), hipMemcpyDeviceToHost, st));
    SGF_HIP(hipStreamSynchronize(st));
    if (hdr.max_row > NB_MAX) {
        set_error("sgf_build_pattern: an atom has %lld bonds (limit %d)", (long long)hdr.max_row - 1, NB_MAX - 1);
        return SGF_EUNSUPPORTED;
    }
    if (total >= ((int64_t)1 << 31)) {
        set_error("sgf_build_pattern: %lld blocks exceed int32 indexing", (long long)total);
        return SGF_EUNSUPPORTED;
    }
    *nnzb = total;
    return SGF_OK;
}

extern "C" sgf_status sgf_build_pattern(int64_t n_atoms, const double *d_xyz, double r_cut, void *d_ws, size_t ws_bytes,
                                        int32_t *d_row_ptr, int64_t *nnzb, void *stream) {
    SGF_REQUIRE(d_row_ptr, "sgf_build_pattern: NULL pointer");
    return bond_pattern(n_atoms, d_xyz, r_cut, d_ws, ws_bytes, d_row_ptr, nnzb, stream);
}

extern "C" sgf_status sgf_hamiltonian_size(int64_t n_atoms, const double *d_xyz, const sgf_tb_params *p, void *d_ws,
                                           size_t ws_bytes, int64_t *nnzb, void *stream) {
    SGF_REQUIRE(p, "sgf_hamiltonian_size: NULL parameters");
    return bond_pattern(n_atoms, d_xyz, p->r_cut, d_ws, ws_bytes, nullptr, nnzb, stream);
}

extern "C" sgf_status sgf_system_from_bsr(const sgf_bsr *m, const double *d_xyz, sgf_system **out) {
    SGF_REQUIRE(m && out, "sgf_system_from_bsr: NULL argument");
    SGF_REQUIRE(m->n_atoms >= 1 && m->n_atoms < (int64_t)1 << 30, "sgf_system_from_bsr: n_atoms %lld out of range",
                (long long)m->n_atoms);
    SGF_REQUIRE(m->nnzb >= m->n_atoms && m->nnzb < (int64_t)1 << 31,
                "sgf_system_from_bsr: nnzb %lld (need at least one diagonal block per row, below 2^31)",
                (long long)m->nnzb);
    SGF_REQUIRE(m->row_ptr && m->col && m->h, "sgf_system_from_bsr: row_ptr, col and h are required");
    SGF_REQUIRE(!m->s32 || m->s, "sgf_system_from_bsr: an FP32 overlap shadow without the overlap");
    SGF_REQUIRE(m->s_orbital_diagonal == 0 || m->s_orbital_diagonal == 1,
                "sgf_system_from_bsr: s_orbital_diagonal must be 0 or 1");
    sgf_system *sys = static_cast<sgf_system *>(std::malloc(sizeof(sgf_system)));
    if (!sys) {
        set_error("sgf_system_from_bsr: out of host memory");
        return SGF_ENOMEM;
    }
    *sys = sgf_system{m->n_atoms, m->nnzb, m->row_ptr, m->col, m->h, m->s, m->h32, m->s32, d_xyz,
                      m->s ? m->s_orbital_diagonal : 0};
    *out = sys;
    return SGF_OK;
}

extern "C" void sgf_system_destroy(sgf_system *sys) { std::free(sys); }

extern "C" sgf_status sgf_build_hamiltonian(int64_t n_atoms, const double *d_xyz, const double *d_onsite,
                                            const sgf_tb_params *p, const void *d_ws, size_t ws_bytes,
                                            const int32_t *d_row_ptr, int64_t nnzb, int32_t *d_col, double *d_h,
                                            double *d_s, void *stream) {
    SGF_REQUIRE(n_atoms > 0 && n_atoms < (int64_t)1 << 30, "sgf_build_hamiltonian: n_atoms out of range");
    SGF_REQUIRE(p && d_xyz && d_ws && d_row_ptr && d_col && d_h, "sgf_build_hamiltonian: NULL pointer");
    SGF_REQUIRE(!p->overlap || d_s, "sgf_build_hamiltonian: overlap requested but d_s is NULL");
    SGF_REQUIRE(p->r_cut > 0 && p->r0 > 0 && (!p->overlap || p->s_decay > 0),
                "sgf_build_hamiltonian: r_cut, r0 and s_decay must be positive");
    SGF_REQUIRE(nnzb >= n_atoms, "sgf_build_hamiltonian: nnzb smaller than n_atoms");
    BuildLayout L = build_layout(n_atoms, const_cast<void *>(d_ws), ws_bytes);
    SGF_REQUIRE(L.bytes <= ws_bytes, "sgf_build_hamiltonian: workspace %zu bytes < %zu", ws_bytes, L.bytes);
    k_bond_fill<<<grid_for(n_atoms), BUILD_T, 0, as_stream(stream)>>>(d_xyz, d_onsite, n_atoms, L, *p, d_row_ptr,
                                                                      d_col, d_h, p->overlap ? d_s : nullptr);
    SGF_LAUNCHED();
    return SGF_OK;
}

extern "C" sgf_status sgf_build_chain(int64_t n_sites, const double *d_eps, double t, int32_t *d_row_ptr,
                                      int32_t *d_col, double *d_h, void *stream) {
    SGF_REQUIRE(n_sites > 0 && n_sites % 4 == 0, "sgf_build_chain: n_sites must be a positive multiple of 4");
    SGF_REQUIRE(n_sites < (int64_t)1 << 31, "sgf_build_chain: n_sites too large");
    SGF_REQUIRE(d_eps && d_row_ptr && d_col && d_h, "sgf_build_chain: NULL pointer");
    const int64_t nb = n_sites / 4;
    k_chain<<<grid_for(nb + 1), BUILD_T, 0, as_stream(stream)>>>(nb, d_eps, t, d_row_ptr, d_col, d_h);
    SGF_LAUNCHED();
    return SGF_OK;
}
