// plan.hip -- local subspaces of the order-N solve.
//
// Each plan is the subspace of one centre atom c: the atoms within radius R
// of c (Euclidean, FP64, no fused multiply-add in the distance), optionally
// pruned to those connected to c through stored blocks inside that ball.  One
// wavefront builds one plan in LDS: ball search through the spatial hash,
// bitonic sort, frontier BFS for the pruning, then the local block-row
// structure (local column atom + global block index) and the projection atoms.
#include <algorithm>

#include "build.hpp"

namespace sgf {

constexpr int PLAN_T = 64;

enum : int64_t { PLAN_ERR_NONE = 0, PLAN_ERR_OVERFLOW = 1, PLAN_ERR_NOGEOM = 2, PLAN_ERR_CENTER = 3 };

struct PlanMeta {
    int64_t err;        // PLAN_ERR_*
    int64_t err_plan;   // first failing plan (smallest index)
    int64_t max_loc_atoms, max_loc_blocks, max_proj_atoms, max_row_blocks;
};

struct PlanLayout {
    PlanMeta *meta;
    char *scan;
    size_t bytes;
};

static PlanLayout plan_layout(int64_t n_plans, void *base, size_t cap) {
    PlanLayout L;
    Carve c(base, cap);
    L.meta = c.take<PlanMeta>(1);
    L.scan = c.take<char>(prefix_scratch_bytes(n_plans + 1));
    L.bytes = c.used;
    return L;
}

__device__ __forceinline__ int bsearch_lds(const int32_t *v, int n, int32_t key) {
    int lo = 0, hi = n - 1;
    while (lo <= hi) {
        const int mid = (lo + hi) >> 1;
        const int32_t x = v[mid];
        if (x == key) return mid;
        if (x < key) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

__device__ __forceinline__ void plan_fail(PlanMeta *m, int64_t code, int64_t p) {
    atomicMax(reinterpret_cast<unsigned long long *>(&m->err), (unsigned long long)code);
    atomicMin(reinterpret_cast<long long *>(&m->err_plan), (long long)p);
}

// Inclusive wavefront scan of an int (64 lanes).
__device__ __forceinline__ int wave_scan_incl(int v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int u = __shfl_up(v, off, 64);
        if (lane >= off) v += u;
    }
    return v;
}

__device__ __forceinline__ int wave_max_int(int v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
    return v;
}

// Running maximum shared by all plans: most plans do not raise it, so read it
// first and take the atomic only when v is larger.  A stale read can only be
// lower than the true value, which costs an extra atomic and nothing else.
__device__ __forceinline__ void raise_max(int64_t *m, int64_t v) {
    if (v > __hip_atomic_load(m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
        atomicMax(reinterpret_cast<unsigned long long *>(m), (unsigned long long)v);
}

// Stage the stored-block ranges of atoms rows[e0 .. min(e0 + 64, e1)) for a
// pair loop: s_r0[k] is the first block of the k-th atom's row, s_ex[k] the
// number of pairs before it.  Returns the pair count (uniform).  Ends with a
// barrier, so the staged ranges are visible to every lane.
__device__ __forceinline__ int stage_rows(const int32_t *row_ptr, const int32_t *rows, int e0, int e1, int32_t *s_r0,
                                         int32_t *s_ex) {
    const int lane = threadIdx.x;
    const int e = e0 + lane;
    int32_t r0 = 0;
    int n = 0;
    if (e < e1) {
        const int32_t at = rows[e];
        r0 = row_ptr[at];
        n = row_ptr[at + 1] - r0;
    }
    const int incl = wave_scan_incl(n);
    s_r0[lane] = r0;
    s_ex[lane] = incl - n;
    __syncthreads();
    return __shfl(incl, 63, 64);
}

// Row that owns pair q (0 <= q < pair count): the largest k with s_ex[k] <= q.
// Rows with no pairs share s_ex with the next row, so the largest such k has
// at least one pair.
__device__ __forceinline__ int pair_owner(const int32_t *s_ex, int q) {
    int k = 0;
#pragma unroll
    for (int step = 32; step > 0; step >>= 1)
        if (s_ex[k + step] <= q) k += step;
    return k;
}

struct PlanArgs {
    int64_t n_plans, n_atoms;
    const int32_t *center;
    const double *radius;
    int32_t prune;
    const int32_t *row_ptr, *col;
    const double *xyz;
    BuildLayout B;  // spatial hash (valid when has_hash)
    int has_hash;
    int maxl;       // LDS capacity in atoms (power of two)
    int limit;      // most local atoms a plan may hold (<= maxl); more is PLAN_ERR_OVERFLOW
    int64_t *atom_off, *blk_off, *pa_off;
    int32_t *loc_atom, *lrow, *lblk, *pa_loc, *center_loc;
    PlanMeta *meta;
};

template <bool FILL>
__global__ __launch_bounds__(PLAN_T) void k_plan(PlanArgs a) {
    extern __shared__ int32_t lds[];
    int32_t *cand = lds;                 // [maxl]; with the next maxl ints, the BFS hash set
    int32_t *queue = lds + 2 * a.maxl;   // [maxl]
    int32_t *list = lds + 3 * a.maxl;    // [maxl]
    __shared__ int s_n, s_tail;
    __shared__ int32_t s_r0[PLAN_T], s_ex[PLAN_T], s_cnt[PLAN_T];
    const int lane = threadIdx.x;
    const int64_t p = blockIdx.x;
    if (p >= a.n_plans) return;
    const int32_t c = a.center[p];
    const double R = a.radius[p];
    if (c < 0 || c >= a.n_atoms) {
        if (lane == 0) plan_fail(a.meta, PLAN_ERR_CENTER, p);
        return;
    }
    if (lane == 0) s_n = 0;
    __syncthreads();

    int nloc;
    if (a.prune) {
        // Connected component of c inside the ball (R <= 0: in the whole block
        // pattern), found by a breadth-first search along stored blocks that
        // admits only atoms within R of c; the ball itself is never enumerated.
        // Visited atoms go to an open-addressing hash set in LDS (2 * maxl
        // slots, i.e. cand and visit together).
        if (R > 0.0 && !a.xyz) {
            if (lane == 0) plan_fail(a.meta, PLAN_ERR_NOGEOM, p);
            return;
        }
        int32_t *hset = cand;  // 2 * maxl slots
        const uint32_t hmask = (uint32_t)(2 * a.maxl - 1);
        for (int i = lane; i < 2 * a.maxl; i += PLAN_T) hset[i] = -1;
        __syncthreads();
        const double *rc = R > 0.0 ? &a.xyz[3 * (int64_t)c] : nullptr;
        const double R2 = R * R;
        if (lane == 0) {
            hset[((uint32_t)c * 2654435761u) & hmask] = c;
            queue[0] = c;
            s_tail = 1;
        }
        __syncthreads();
        int head = 0;
        while (true) {
            const int tail = s_tail;
            __syncthreads();
            if (head == tail || tail > a.maxl) break;
            // One level: the (frontier atom, stored block) pairs are spread over
            // the lanes, so the row, column and coordinate loads of a level are
            // issued together rather than one neighbour at a time per lane.
            for (int e0 = head; e0 < tail; e0 += PLAN_T) {
                const int total = stage_rows(a.row_ptr, queue, e0, tail, s_r0, s_ex);
                for (int q = lane; q < total; q += PLAN_T) {
                    const int k = pair_owner(s_ex, q);
                    const int32_t b = a.col[s_r0[k] + q - s_ex[k]];
                    if (rc && dist2_exact(rc, &a.xyz[3 * (int64_t)b]) > R2) continue;
                    // Once maxl atoms are in, only look b up: a new b means the
                    // component has more than maxl atoms.  Before that point at most
                    // 64 inserts race past the check, so the set holds fewer than
                    // maxl + 64 <= 2 * maxl atoms and every probe meets an empty slot.
                    const bool full = *reinterpret_cast<volatile int *>(&s_tail) >= a.maxl;
                    uint32_t h = ((uint32_t)b * 2654435761u) & hmask;
                    while (true) {
                        const int32_t prev = full ? *reinterpret_cast<volatile int32_t *>(&hset[h])
                                                  : atomicCAS(&hset[h], -1, b);
                        if (prev == b) break;
                        if (prev == -1) {
                            const int pos = atomicAdd(&s_tail, 1);
                            if (pos < a.maxl) queue[pos] = b;
                            break;
                        }
                        h = (h + 1) & hmask;
                    }
                }
                __syncthreads();
            }
            head = tail;
            __syncthreads();
        }
        if (s_tail > a.limit) {
            if (lane == 0) plan_fail(a.meta, PLAN_ERR_OVERFLOW, p);
            return;
        }
        nloc = s_tail;
        // sort the component (bitonic, INT_MAX padding) into list
        int np = 1;
        while (np < nloc) np <<= 1;
        for (int i = lane; i < np; i += PLAN_T) list[i] = i < nloc ? queue[i] : 0x7fffffff;
        __syncthreads();
        for (int k = 2; k <= np; k <<= 1)
            for (int j = k >> 1; j > 0; j >>= 1) {
                for (int i = lane; i < np; i += PLAN_T) {
                    const int l = i ^ j;
                    if (l > i) {
                        const int32_t x = list[i], y = list[l];
                        if ((x > y) == ((i & k) == 0)) { list[i] = y; list[l] = x; }
                    }
                }
                __syncthreads();
            }
    } else {
        // 1. Candidates: the ball around c, or every atom.
        if (R <= 0.0) {
            if (a.n_atoms > a.limit) {
                if (lane == 0) plan_fail(a.meta, PLAN_ERR_OVERFLOW, p);
                return;
            }
            for (int i = lane; i < a.n_atoms; i += PLAN_T) cand[i] = i;
            if (lane == 0) s_n = (int)a.n_atoms;
            __syncthreads();
        } else {
            if (!a.has_hash || !a.xyz) {
                if (lane == 0) plan_fail(a.meta, PLAN_ERR_NOGEOM, p);
                return;
            }
            const double cell = a.B.hdr->cell;
            const double *rc = &a.xyz[3 * (int64_t)c];
            const int4 cc = cell_of(rc, cell);
            const int m = (int)ceil(R / cell);
            const int w = 2 * m + 1;
            const int ncell = w * w * w;
            const double R2 = R * R;
            const uint32_t mask = (uint32_t)(a.B.nbuck - 1);
            for (int ci = lane; ci < ncell; ci += PLAN_T) {
                const int4 t = make_int4(cc.x + ci / (w * w) - m, cc.y + (ci / w) % w - m, cc.z + ci % w - m, 0);
                const uint32_t b = hash_cell(t, mask);
                for (int64_t i = a.B.bucket[b]; i < a.B.bucket[b + 1]; ++i) {
                    const int4 qc = a.B.sorted_cell[i];
                    if (qc.x != t.x || qc.y != t.y || qc.z != t.z) continue;
                    const int32_t q = a.B.sorted_atom[i];
                    if (dist2_exact(rc, &a.xyz[3 * (int64_t)q]) <= R2) {
                        const int pos = atomicAdd(&s_n, 1);
                        if (pos < a.maxl) cand[pos] = q;
                    }
                }
            }
            __syncthreads();
            if (s_n > a.limit) {
                if (lane == 0) plan_fail(a.meta, PLAN_ERR_OVERFLOW, p);
                return;
            }
            // bitonic sort of cand[0..np) with INT_MAX padding
            int np = 1;
            while (np < s_n) np <<= 1;
            for (int i = s_n + lane; i < np; i += PLAN_T) cand[i] = 0x7fffffff;
            __syncthreads();
            for (int k = 2; k <= np; k <<= 1)
                for (int j = k >> 1; j > 0; j >>= 1) {
                    for (int i = lane; i < np; i += PLAN_T) {
                        const int l = i ^ j;
                        if (l > i) {
                            const int32_t x = cand[i], y = cand[l];
                            const bool up = (i & k) == 0;
                            if ((x > y) == up) { cand[i] = y; cand[l] = x; }
                        }
                    }
                    __syncthreads();
                }
        }
        const int ncand = s_n;

        // every candidate is local (no pruning)
        for (int i = lane; i < ncand; i += PLAN_T) list[i] = cand[i];
        nloc = ncand;
    }
    __syncthreads();

    // 3. Local block rows and projection atoms.  The stored blocks of 64 local
    // rows at a time are spread over the lanes as (row, block) pairs; a pair
    // whose column atom is local is a local block, and its place in lblk is the
    // count of local blocks before it in (row, column position) order.
    const int64_t abase = FILL ? a.atom_off[p] : 0;
    const int64_t bbase = FILL ? a.blk_off[p] : 0;
    int carry = 0, rmax = 0;
    for (int start = 0; start < nloc; start += PLAN_T) {
        const int A = start + lane;
        const int total = stage_rows(a.row_ptr, list, start, nloc, s_r0, s_ex);
        s_cnt[lane] = 0;
        __syncthreads();
        int run = carry;
        for (int q0 = 0; q0 < total; q0 += PLAN_T) {
            const int q = q0 + lane;
            int k = 0, B = -1;
            int32_t t = 0;
            if (q < total) {
                k = pair_owner(s_ex, q);
                t = s_r0[k] + q - s_ex[k];
                B = bsearch_lds(list, nloc, a.col[t]);
            }
            const int hit = B >= 0;
            const int hincl = wave_scan_incl(hit);
            if (hit) {
                atomicAdd(&s_cnt[k], 1);
                if (FILL) {
                    const int64_t pos = bbase + run + hincl - 1;
                    a.lblk[2 * pos] = B;
                    a.lblk[2 * pos + 1] = t;
                }
            }
            run += __shfl(hincl, 63, 64);
        }
        __syncthreads();
        const int cnt = s_cnt[lane];
        const int cincl = wave_scan_incl(cnt);
        if (FILL && A < nloc) {
            a.loc_atom[abase + A] = list[A];
            a.lrow[abase + A] = carry + cincl - cnt;
        }
        rmax = max(rmax, cnt);
        carry = run;
        __syncthreads();
    }
    const int nblk = carry;
    // projection atoms: local column atoms of the centre's stored blocks, in order
    int npa = 0;
    {
        const int32_t c0 = a.row_ptr[c], c1 = a.row_ptr[c + 1];
        const int64_t pbase = FILL ? a.pa_off[p] : 0;
        for (int32_t t0 = c0; t0 < c1; t0 += PLAN_T) {
            const int32_t t = t0 + lane;
            const int B = t < c1 ? bsearch_lds(list, nloc, a.col[t]) : -1;
            const int hit = B >= 0;
            const int hincl = wave_scan_incl(hit);
            if (FILL && hit) a.pa_loc[pbase + npa + hincl - 1] = B;
            npa += __shfl(hincl, 63, 64);
        }
    }
    if (!FILL) rmax = wave_max_int(rmax);
    if (lane == 0) {
        if (FILL) {
            a.center_loc[p] = bsearch_lds(list, nloc, c);
        } else {
            a.atom_off[p + 1] = nloc;
            a.blk_off[p + 1] = nblk;
            a.pa_off[p + 1] = npa;
            raise_max(&a.meta->max_loc_atoms, nloc);
            raise_max(&a.meta->max_loc_blocks, nblk);
            raise_max(&a.meta->max_proj_atoms, npa);
            raise_max(&a.meta->max_row_blocks, rmax);
        }
    }
}

__global__ void k_plan_init(PlanMeta *m, int64_t *atom_off, int64_t *blk_off, int64_t *pa_off) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        m->err = PLAN_ERR_NONE;
        m->err_plan = INT64_MAX;
        m->max_loc_atoms = m->max_loc_blocks = m->max_proj_atoms = m->max_row_blocks = 0;
        atom_off[0] = blk_off[0] = pa_off[0] = 0;
    }
}

static int maxl_pow2(int32_t max_loc_atoms) {
    int m = 64;
    while (m < max_loc_atoms) m <<= 1;
    return m;
}

static sgf_status plan_args(const char *who, const sgf_system *sys, sgf_plan *plan, int32_t max_loc_atoms,
                            const void *d_build_ws, size_t build_ws_bytes, void *d_ws, size_t ws_bytes, PlanArgs &a,
                            PlanLayout &L) {
    SGF_REQUIRE(sys && plan, "%s: NULL system or plan", who);
    SGF_REQUIRE(sys->n_atoms > 0 && sys->row_ptr && sys->col, "%s: system has no block pattern", who);
    SGF_REQUIRE(plan->n_plans >= 0 && (plan->n_plans == 0 || (plan->center && plan->radius)),
                "%s: plan centres/radii missing", who);
    SGF_REQUIRE(plan->atom_off && plan->blk_off && plan->pa_off, "%s: plan offsets are NULL", who);
    SGF_REQUIRE(max_loc_atoms >= 1 && max_loc_atoms <= 8192, "%s: max_loc_atoms must be in [1, 8192]", who);
    SGF_REQUIRE(d_ws, "%s: workspace is NULL", who);
    L = plan_layout(plan->n_plans, d_ws, ws_bytes);
    SGF_REQUIRE(L.bytes <= ws_bytes, "%s: workspace %zu bytes < %zu", who, ws_bytes, L.bytes);
    a = PlanArgs{};
    a.n_plans = plan->n_plans;
    a.n_atoms = sys->n_atoms;
    a.center = plan->center;
    a.radius = plan->radius;
    a.prune = plan->prune;
    a.row_ptr = sys->row_ptr;
    a.col = sys->col;
    a.xyz = sys->xyz;
    a.has_hash = d_build_ws != nullptr;
    if (d_build_ws) {
        a.B = build_layout(sys->n_atoms, const_cast<void *>(d_build_ws), build_ws_bytes);
        SGF_REQUIRE(a.B.bytes <= build_ws_bytes, "%s: build workspace too small", who);
    }
    a.maxl = maxl_pow2(max_loc_atoms);
    a.limit = max_loc_atoms;
    a.atom_off = plan->atom_off;
    a.blk_off = plan->blk_off;
    a.pa_off = plan->pa_off;
    a.loc_atom = plan->loc_atom;
    a.lrow = plan->lrow;
    a.lblk = plan->lblk;
    a.pa_loc = plan->pa_loc;
    a.center_loc = plan->center_loc;
    a.meta = L.meta;
    return SGF_OK;
}

__global__ void k_proj_count(int64_t n_cols, int64_t n_plans, const int32_t *col_plan, const int64_t *pa_off,
                             int64_t *proj_off) {
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c <= n_cols; c += (int64_t)gridDim.x * blockDim.x) {
        if (c == 0) proj_off[0] = 0;
        else {
            const int32_t pl = col_plan[c - 1];
            proj_off[c] = (pl >= 0 && pl < n_plans) ? 4 * (pa_off[pl + 1] - pa_off[pl]) : 0;
        }
    }
}

__global__ void k_proj_rows(int64_t n_cols, int64_t n_plans, const int32_t *col_plan, const int64_t *atom_off, const int64_t *pa_off,
                            const int32_t *loc_atom, const int32_t *pa_loc, const int64_t *proj_off, int32_t *proj_row) {
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n_cols; c += (int64_t)gridDim.x * blockDim.x) {
        const int32_t pl = col_plan[c];
        if (pl < 0 || pl >= n_plans) continue;
        const int64_t npa = pa_off[pl + 1] - pa_off[pl];
        for (int64_t q = 0; q < npa; ++q) {
            const int32_t atom = loc_atom[atom_off[pl] + pa_loc[pa_off[pl] + q]];
            for (int o = 0; o < 4; ++o) proj_row[proj_off[c] + 4 * q + o] = 4 * atom + o;
        }
    }
}

}  // namespace sgf

using namespace sgf;

extern "C" sgf_status sgf_plan_workspace(const sgf_system *sys, int64_t n_plans, int32_t max_loc_atoms,
                                         size_t *ws_bytes) {
    SGF_REQUIRE(sys && ws_bytes && n_plans >= 0, "sgf_plan_workspace: bad arguments");
    SGF_REQUIRE(max_loc_atoms >= 1 && max_loc_atoms <= 8192, "sgf_plan_workspace: max_loc_atoms out of range");
    *ws_bytes = plan_layout(n_plans, nullptr, 0).bytes;
    return SGF_OK;
}

// First LDS capacity of the count pass, in atoms.  Residency of the one-wave
// plan workgroups is bounded by LDS (four arrays of maxl ints each), and the
// pass is bound by the latency of its dependent loads, so a small capacity
// (4 KiB, the full 32 waves per CU) is tried first; a batch with a larger
// subspace is counted again at the caller's capacity.
constexpr int PLAN_FIRST_MAXL = 256;

static sgf_status launch_plan(bool fill, const PlanArgs &a, hipStream_t st) {
    const size_t lds = 4 * (size_t)a.maxl * sizeof(int32_t);
    const void *fn = fill ? reinterpret_cast<const void *>(k_plan<true>) : reinterpret_cast<const void *>(k_plan<false>);
    SGF_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    if (fill) k_plan<true><<<dim3((unsigned)a.n_plans), dim3(PLAN_T), lds, st>>>(a);
    else k_plan<false><<<dim3((unsigned)a.n_plans), dim3(PLAN_T), lds, st>>>(a);
    SGF_LAUNCHED();
    return SGF_OK;
}

extern "C" sgf_status sgf_plan_count(const sgf_system *sys, sgf_plan *plan, int32_t max_loc_atoms,
                                     const void *d_build_ws, size_t build_ws_bytes, void *d_ws, size_t ws_bytes,
                                     sgf_plan_totals *totals, void *stream) {
    PlanArgs a;
    PlanLayout L;
    sgf_status rc = plan_args("sgf_plan_count", sys, plan, max_loc_atoms, d_build_ws, build_ws_bytes, d_ws, ws_bytes,
                              a, L);
    if (rc) return rc;
    SGF_REQUIRE(totals, "sgf_plan_count: totals is NULL");
    hipStream_t st = as_stream(stream);
    const int full_maxl = a.maxl;
    PlanMeta m;
    int64_t t3[3] = {0, 0, 0};
    const int full_limit = a.limit;
    for (a.maxl = std::min(full_maxl, PLAN_FIRST_MAXL);; a.maxl = full_maxl) {
        a.limit = std::min(full_limit, a.maxl);
        k_plan_init<<<1, 64, 0, st>>>(L.meta, plan->atom_off, plan->blk_off, plan->pa_off);
        SGF_LAUNCHED();
        if (plan->n_plans > 0) {
            rc = launch_plan(false, a, st);
            if (rc) return rc;
            for (int64_t *off : {plan->atom_off, plan->blk_off, plan->pa_off}) {
                rc = inclusive_scan_i64(off + 1, plan->n_plans, L.scan, st);
                if (rc) return rc;
            }
        }
        SGF_HIP(hipMemcpyAsync(&m, L.meta, sizeof(m), hipMemcpyDeviceToHost, st));
        SGF_HIP(hipMemcpyAsync(&t3[0], plan->atom_off + plan->n_plans, 8, hipMemcpyDeviceToHost, st));
        SGF_HIP(hipMemcpyAsync(&t3[1], plan->blk_off + plan->n_plans, 8, hipMemcpyDeviceToHost, st));
        SGF_HIP(hipMemcpyAsync(&t3[2], plan->pa_off + plan->n_plans, 8, hipMemcpyDeviceToHost, st));
        SGF_HIP(hipStreamSynchronize(st));
        if (m.err != PLAN_ERR_OVERFLOW || a.maxl == full_maxl) break;
    }
    if (m.err == PLAN_ERR_OVERFLOW) {
        set_error("sgf_plan_count: plan %lld holds more than max_loc_atoms=%d atoms", (long long)m.err_plan,
                  max_loc_atoms);
        return SGF_EUNSUPPORTED;
    }
    if (m.err == PLAN_ERR_CENTER) {
        set_error("sgf_plan_count: plan %lld has a centre atom outside [0, n_atoms)", (long long)m.err_plan);
        return SGF_EINVAL;
    }
    if (m.err == PLAN_ERR_NOGEOM) {
        set_error("sgf_plan_count: plan %lld has a positive radius but no xyz / build workspace was given",
                  (long long)m.err_plan);
        return SGF_EINVAL;
    }
    if (t3[1] >= ((int64_t)1 << 31)) {
        set_error("sgf_plan_count: %lld local blocks exceed int32 indexing; plan fewer centres per batch",
                  (long long)t3[1]);
        return SGF_EUNSUPPORTED;
    }
    totals->n_loc_atoms = t3[0];
    totals->n_loc_blocks = t3[1];
    totals->n_proj_atoms = t3[2];
    totals->max_loc_atoms = (int32_t)m.max_loc_atoms;
    totals->max_loc_blocks = (int32_t)m.max_loc_blocks;
    totals->max_proj_atoms = (int32_t)m.max_proj_atoms;
    totals->max_row_blocks = (int32_t)m.max_row_blocks;
    return SGF_OK;
}

extern "C" sgf_status sgf_plan_build(const sgf_system *sys, sgf_plan *plan, int32_t max_loc_atoms,
                                     const void *d_build_ws, size_t build_ws_bytes, void *d_ws, size_t ws_bytes,
                                     void *stream) {
    PlanArgs a;
    PlanLayout L;
    sgf_status rc = plan_args("sgf_plan_build", sys, plan, max_loc_atoms, d_build_ws, build_ws_bytes, d_ws, ws_bytes,
                              a, L);
    if (rc) return rc;
    SGF_REQUIRE(plan->n_plans == 0 || (plan->loc_atom && plan->lrow && plan->lblk && plan->pa_loc && plan->center_loc),
                "sgf_plan_build: plan output arrays are NULL");
    if (plan->n_plans == 0) return SGF_OK;
    hipStream_t st = as_stream(stream);
    k_plan_init<<<1, 64, 0, st>>>(L.meta, plan->atom_off, plan->blk_off, plan->pa_off);
    SGF_LAUNCHED();
    rc = launch_plan(true, a, st);
    if (rc) return rc;
    PlanMeta m;
    SGF_HIP(hipMemcpyAsync(&m, L.meta, sizeof(m), hipMemcpyDeviceToHost, st));
    SGF_HIP(hipStreamSynchronize(st));
    if (m.err == PLAN_ERR_OVERFLOW) {
        set_error("sgf_plan_build: plan %lld holds more than max_loc_atoms=%d atoms (pass at least the "
                  "max_loc_atoms total of sgf_plan_count)", (long long)m.err_plan, max_loc_atoms);
        return SGF_EUNSUPPORTED;
    }
    SGF_REQUIRE(m.err == PLAN_ERR_NONE, "sgf_plan_build: plan %lld failed (code %lld) although it was counted",
                (long long)m.err_plan, (long long)m.err);
    return SGF_OK;
}

extern "C" sgf_status sgf_proj_layout(const sgf_plan *plan, int64_t n_cols, const int64_t *d_cols,
                                      const int32_t *d_col_plan, int64_t *d_proj_off, int32_t *d_proj_row,
                                      int64_t *total_rows, void *stream) {
    SGF_REQUIRE(plan && plan->pa_off && plan->atom_off, "sgf_proj_layout: plan offsets are NULL");
    SGF_REQUIRE(n_cols >= 0 && (n_cols == 0 || (d_cols && d_col_plan)), "sgf_proj_layout: columns missing");
    SGF_REQUIRE(d_proj_off && total_rows, "sgf_proj_layout: NULL output");
    hipStream_t st = as_stream(stream);
    const unsigned g = (unsigned)((n_cols + 256) / 256);
    k_proj_count<<<g, 256, 0, st>>>(n_cols, plan->n_plans, d_col_plan, plan->pa_off, d_proj_off);
    SGF_LAUNCHED();
    if (n_cols > 0) {
        sgf_status rc = inclusive_scan_noscratch(d_proj_off + 1, n_cols, st);
        if (rc) return rc;
    }
    if (d_proj_row && n_cols > 0) {
        SGF_REQUIRE(plan->loc_atom && plan->pa_loc, "sgf_proj_layout: plan has not been built");
        k_proj_rows<<<g, 256, 0, st>>>(n_cols, plan->n_plans, d_col_plan, plan->atom_off, plan->pa_off, plan->loc_atom, plan->pa_loc,
                                       d_proj_off, d_proj_row);
        SGF_LAUNCHED();
    }
    SGF_HIP(hipMemcpyAsync(total_rows, d_proj_off + n_cols, 8, hipMemcpyDeviceToHost, st));
    SGF_HIP(hipStreamSynchronize(st));
    return SGF_OK;
}

extern "C" sgf_status sgf_proj_rows(const sgf_plan *plan, int64_t n_cols, const int32_t *d_col_plan,
                                    const int64_t *d_proj_off, int32_t *d_proj_row, void *stream) {
    SGF_REQUIRE(plan && plan->pa_off && plan->atom_off && plan->loc_atom && plan->pa_loc,
                "sgf_proj_rows: plan has not been built");
    SGF_REQUIRE(n_cols >= 0 && (n_cols == 0 || (d_col_plan && d_proj_off && d_proj_row)), "sgf_proj_rows: NULL array");
    if (n_cols == 0) return SGF_OK;
    const unsigned g = (unsigned)((n_cols + 255) / 256);
    k_proj_rows<<<g, 256, 0, as_stream(stream)>>>(n_cols, plan->n_plans, d_col_plan, plan->atom_off, plan->pa_off,
                                                  plan->loc_atom, plan->pa_loc, d_proj_off, d_proj_row);
    SGF_LAUNCHED();
    return SGF_OK;
}
