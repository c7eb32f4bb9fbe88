// mlp.hip -- learned scheduling: per-column features, the iteration-count
// network (forward, backward, Adam) and a longest-predicted-first ordering of
// the columns for the solver's work queue.
//
// Network: x' = (x - mean) * inv_std; h1 = relu(W1 x' + b1);
// h2 = relu(W2 h1 + b2); y = W3 . h2 + b3, predicting log(iterations).
// Parameters are one float vector:
//   [0:5] mean, [5:10] inv_std, W1 (64x5 row-major), b1 (64), W2 (64x64),
//   b2 (64), W3 (64), b3 (1)  -> 4619 floats; Adam updates the last 4609.
#include "common.hpp"

namespace sgf {

constexpr int NF = 5, NH = 64;
constexpr int OFF_W1 = 2 * NF, OFF_B1 = OFF_W1 + NH * NF, OFF_W2 = OFF_B1 + NH, OFF_B2 = OFF_W2 + NH * NH,
              OFF_W3 = OFF_B2 + NH, OFF_B3 = OFF_W3 + NH, NPARAM = OFF_B3 + 1;
constexpr int TRAIN_T = 128;  // samples per training step (one per thread)
constexpr int ORDER_BUCKETS = 4096;

static_assert(NPARAM == 4619, "parameter layout");

// ---------------------------------------------------------------------------
// Features of column j (atom c, orbital o) on its local subspace:
//   f0 off-diagonal blocks of c's local row, f1 / f2 mean / max of
//   ||H_cb[o, :]||_2 over them, f3 |H_jj - mean of H_ii over local orbitals of
//   type o|, f4 local orbitals.
// ---------------------------------------------------------------------------
struct FeatArgs {
    int64_t n_cols, n_plans;
    const int64_t *cols;
    const int32_t *col_plan;
    const double *h;
    const int64_t *atom_off, *blk_off;
    const int32_t *lrow, *lblk, *center_loc;
    float *feat;
};

__global__ void k_features(FeatArgs a) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.n_cols) return;
    float *f = &a.feat[c * NF];
    const int64_t j = a.cols[c];
    const int32_t pl = a.col_plan[c];
    if (pl < 0 || pl >= a.n_plans || j < 0) {
        for (int e = 0; e < NF; ++e) f[e] = 0.0f;
        return;
    }
    const int o = (int)(j & 3);
    const int64_t a0 = a.atom_off[pl], b0 = a.blk_off[pl];
    const int n_loc = (int)(a.atom_off[pl + 1] - a0);
    const int nblk = (int)(a.blk_off[pl + 1] - b0);
    const int cl = a.center_loc[pl];
    int nb = 0;
    double sum = 0.0, mx = 0.0, hjj = 0.0, dsum = 0.0;
    for (int A = 0; A < n_loc; ++A) {
        const int t0 = a.lrow[a0 + A], t1 = A + 1 < n_loc ? a.lrow[a0 + A + 1] : nblk;
        for (int t = t0; t < t1; ++t) {
            const int B = a.lblk[2 * (b0 + t)];
            const double *blk = &a.h[16 * (int64_t)a.lblk[2 * (b0 + t) + 1]];
            if (B == A) {
                dsum += blk[5 * o];
                if (A == cl) hjj = blk[5 * o];
            } else if (A == cl) {
                const double *r = &blk[4 * o];
                const double nrm = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2] + r[3] * r[3]);
                ++nb;
                sum += nrm;
                mx = fmax(mx, nrm);
            }
        }
    }
    f[0] = (float)nb;
    f[1] = (float)(nb ? sum / nb : 0.0);
    f[2] = (float)mx;
    f[3] = (float)fabs(hjj - dsum / n_loc);
    f[4] = (float)(4 * n_loc);
}

// ---------------------------------------------------------------------------
// Forward pass (inference): one sample per thread.  Every parameter index is
// the same for all lanes, so the parameters are read with scalar loads into
// SGPRs and feed the multiply-adds directly (staged in LDS, each multiply-add
// waited for an LDS read of its weight).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_mlp_forward(const float *__restrict__ P, const float *X, int64_t n,
                                                     float *Y) {
    const float *sp = P;
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n; s += (int64_t)gridDim.x * blockDim.x) {
        float x[NF];
#pragma unroll
        for (int e = 0; e < NF; ++e) x[e] = (X[s * NF + e] - sp[e]) * sp[NF + e];
        float h1[NH];
#pragma unroll
        for (int i = 0; i < NH; ++i) {
            float acc = sp[OFF_B1 + i];
#pragma unroll
            for (int e = 0; e < NF; ++e) acc = fmaf(sp[OFF_W1 + i * NF + e], x[e], acc);
            h1[i] = fmaxf(acc, 0.0f);
        }
        float y = sp[OFF_B3];
#pragma unroll 1
        for (int jj = 0; jj < NH; ++jj) {
            float acc = sp[OFF_B2 + jj];
#pragma unroll
            for (int i = 0; i < NH; ++i) acc = fmaf(sp[OFF_W2 + jj * NH + i], h1[i], acc);
            y = fmaf(sp[OFF_W3 + jj], fmaxf(acc, 0.0f), y);
        }
        Y[s] = y;
    }
}

// ---------------------------------------------------------------------------
// Training step: one workgroup, one sample per thread (n <= 128).  The
// activations and the backpropagated errors go to LDS (H1, H2, D2, D1 of
// [128][64] floats); the parameter gradients are then sums over samples in
// a fixed order (dW2 = D2^T H1, dW1 = D1^T X', dW3 = dy^T H2) and each
// parameter is owned by one thread, which applies Adam to it in global
// memory (or writes the gradient out).
// ---------------------------------------------------------------------------
struct TrainArgs {
    float *P, *m, *v, *grad, *loss;
    const float *X, *T;
    int n, step;
    float lr;
};

__device__ __forceinline__ void adam_or_store(const TrainArgs &a, bool update, int e, float g, float c1, float c2) {
    if (!update) {
        a.grad[e] = g;
        return;
    }
    const float m = 0.9f * a.m[e] + 0.1f * g;
    const float v = 0.999f * a.v[e] + 0.001f * g * g;
    a.m[e] = m;
    a.v[e] = v;
    a.P[e] -= a.lr * (m * c1) / (sqrtf(v * c2) + 1e-8f);
}

template <bool UPDATE>
__global__ __launch_bounds__(TRAIN_T) void k_mlp_train(TrainArgs a) {
    extern __shared__ float lds[];
    float *sp = lds;                        // [NPARAM]
    float *H1 = sp + NPARAM;                // [TRAIN_T][NH]
    float *H2 = H1 + TRAIN_T * NH;          // [TRAIN_T][NH]
    float *D2 = H2 + TRAIN_T * NH;          // [TRAIN_T][NH]
    float *D1 = D2 + TRAIN_T * NH;          // [TRAIN_T][NH]
    float *dyv = D1 + TRAIN_T * NH;         // [TRAIN_T]
    float *xs = dyv + TRAIN_T;              // [TRAIN_T][NF]
    float *red = xs + TRAIN_T * NF;         // [TRAIN_T]
    const int s = threadIdx.x;
    for (int i = s; i < NPARAM; i += TRAIN_T) sp[i] = a.P[i];
    __syncthreads();
    const bool live = s < a.n;
    float x[NF];
#pragma unroll
    for (int e = 0; e < NF; ++e) {
        x[e] = live ? (a.X[(int64_t)s * NF + e] - sp[e]) * sp[NF + e] : 0.0f;
        xs[s * NF + e] = x[e];
    }
    // forward
    float h1[NH];
#pragma unroll
    for (int i = 0; i < NH; ++i) {
        float acc = sp[OFF_B1 + i];
#pragma unroll
        for (int e = 0; e < NF; ++e) acc = fmaf(sp[OFF_W1 + i * NF + e], x[e], acc);
        h1[i] = fmaxf(acc, 0.0f);
        H1[s * NH + i] = h1[i];
    }
    float y = sp[OFF_B3];
#pragma unroll 1
    for (int jj = 0; jj < NH; ++jj) {
        float acc = sp[OFF_B2 + jj];
#pragma unroll
        for (int i = 0; i < NH; ++i) acc = fmaf(sp[OFF_W2 + jj * NH + i], h1[i], acc);
        const float h2 = fmaxf(acc, 0.0f);
        H2[s * NH + jj] = h2;
        y = fmaf(sp[OFF_W3 + jj], h2, y);
    }
    const float err = live ? y - a.T[s] : 0.0f;
    const float dy = 2.0f * err / (float)a.n;
    dyv[s] = dy;
    red[s] = err * err;
    // backward: d2 = dy W3 on active units; d1 = W2^T d2 on active units
    float d2[NH];
#pragma unroll
    for (int jj = 0; jj < NH; ++jj) {
        d2[jj] = H2[s * NH + jj] > 0.0f ? dy * sp[OFF_W3 + jj] : 0.0f;
        D2[s * NH + jj] = d2[jj];
    }
#pragma unroll 1
    for (int i = 0; i < NH; ++i) {
        float acc = 0.0f;
#pragma unroll
        for (int jj = 0; jj < NH; ++jj) acc = fmaf(sp[OFF_W2 + jj * NH + i], d2[jj], acc);
        D1[s * NH + i] = H1[s * NH + i] > 0.0f ? acc : 0.0f;
    }
    __syncthreads();
    for (int off = TRAIN_T / 2; off > 0; off >>= 1) {
        if (s < off) red[s] += red[s + off];
        __syncthreads();
    }
    if (s == 0 && a.loss) a.loss[0] = red[0] / (float)a.n;
    const float c1 = 1.0f / (1.0f - powf(0.9f, (float)a.step));
    const float c2 = 1.0f / (1.0f - powf(0.999f, (float)a.step));
    // dW2[j][i] = sum_s d2[s][j] h1[s][i]
    for (int e = s; e < NH * NH; e += TRAIN_T) {
        const int jj = e / NH, i = e % NH;
        float g = 0.0f;
        for (int q = 0; q < TRAIN_T; ++q) g = fmaf(D2[q * NH + jj], H1[q * NH + i], g);
        adam_or_store(a, UPDATE, OFF_W2 + e, g, c1, c2);
    }
    // dW1[i][f] = sum_s d1[s][i] x'[s][f]
    for (int e = s; e < NH * NF; e += TRAIN_T) {
        const int i = e / NF, ff = e % NF;
        float g = 0.0f;
        for (int q = 0; q < TRAIN_T; ++q) g = fmaf(D1[q * NH + i], xs[q * NF + ff], g);
        adam_or_store(a, UPDATE, OFF_W1 + e, g, c1, c2);
    }
    if (s < NH) {
        float gb1 = 0.0f, gb2 = 0.0f, gw3 = 0.0f;
        for (int q = 0; q < TRAIN_T; ++q) {
            gb1 += D1[q * NH + s];
            gb2 += D2[q * NH + s];
            gw3 = fmaf(dyv[q], H2[q * NH + s], gw3);
        }
        adam_or_store(a, UPDATE, OFF_B1 + s, gb1, c1, c2);
        adam_or_store(a, UPDATE, OFF_B2 + s, gb2, c1, c2);
        adam_or_store(a, UPDATE, OFF_W3 + s, gw3, c1, c2);
    }
    if (s == NH) {
        float g = 0.0f;
        for (int q = 0; q < TRAIN_T; ++q) g += dyv[q];
        adam_or_store(a, UPDATE, OFF_B3, g, c1, c2);
    }
    // the normalisation entries are not trained: their gradient is zero
    if (!UPDATE && s >= NH + 1 && s < NH + 1 + 2 * NF) a.grad[s - NH - 1] = 0.0f;
}

constexpr size_t TRAIN_LDS = sizeof(float) * (NPARAM + 4 * TRAIN_T * NH + TRAIN_T + TRAIN_T * NF + TRAIN_T);

// Feature mean and 1/std over n samples into P[0:10] (one workgroup).
__global__ __launch_bounds__(256) void k_mlp_normalize(float *P, const float *X, int64_t n) {
    __shared__ double part[256][2 * NF];
    double acc[2 * NF];
#pragma unroll
    for (int e = 0; e < 2 * NF; ++e) acc[e] = 0.0;
    for (int64_t q = threadIdx.x; q < n; q += blockDim.x)
#pragma unroll
        for (int e = 0; e < NF; ++e) {
            const double v = X[q * NF + e];
            acc[e] += v;
            acc[NF + e] += v * v;
        }
#pragma unroll
    for (int e = 0; e < 2 * NF; ++e) part[threadIdx.x][e] = acc[e];
    __syncthreads();
    if (threadIdx.x < NF) {
        double s1 = 0.0, s2 = 0.0;
        for (int t = 0; t < (int)blockDim.x; ++t) {
            s1 += part[t][threadIdx.x];
            s2 += part[t][NF + threadIdx.x];
        }
        const double mean = s1 / (double)n;
        const double var = s2 / (double)n - mean * mean;
        P[threadIdx.x] = (float)mean;
        P[NF + threadIdx.x] = var > 1e-12 ? (float)(1.0 / sqrt(var)) : 1.0f;
    }
}

// ---------------------------------------------------------------------------
// Longest-predicted-first order: counting sort of the predictions into
// ORDER_BUCKETS buckets over [y_lo, y_hi], largest prediction first.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int order_bucket(float y, float y_lo, float y_hi) {
    const float t = (y_hi - y) / (y_hi - y_lo);
    int b = (int)(t * ORDER_BUCKETS);
    return b < 0 ? 0 : (b >= ORDER_BUCKETS ? ORDER_BUCKETS - 1 : b);
}

__global__ void k_order_zero(int64_t *cnt, int32_t *fill) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i <= ORDER_BUCKETS; i += gridDim.x * blockDim.x) {
        cnt[i] = 0;
        if (i < ORDER_BUCKETS) fill[i] = 0;
    }
}

// Counting sort in chunks of ORDER_CHUNK predictions per workgroup.  The
// predictions crowd into few buckets, so each workgroup counts its chunk in
// LDS and touches a global counter once per non-empty bucket, not once per
// column.
constexpr int ORDER_T = 256;
constexpr int ORDER_CHUNK = 8192;

__global__ __launch_bounds__(ORDER_T) void k_order_hist(const float *y, int64_t n, float y_lo, float y_hi,
                                                        int64_t *cnt) {
    __shared__ uint32_t h[ORDER_BUCKETS];
    for (int i = threadIdx.x; i < ORDER_BUCKETS; i += ORDER_T) h[i] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * ORDER_CHUNK;
    const int64_t end = base + ORDER_CHUNK < n ? base + ORDER_CHUNK : n;
    for (int64_t i = base + threadIdx.x; i < end; i += ORDER_T) atomicAdd(&h[order_bucket(y[i], y_lo, y_hi)], 1u);
    __syncthreads();
    for (int i = threadIdx.x; i < ORDER_BUCKETS; i += ORDER_T)
        if (h[i]) atomicAdd(reinterpret_cast<unsigned long long *>(&cnt[i + 1]), (unsigned long long)h[i]);
}

// Same chunks: each workgroup reserves a run of every non-empty bucket with
// one global atomic, then places its columns inside its runs.
__global__ __launch_bounds__(ORDER_T) void k_order_scatter(const float *y, int64_t n, float y_lo, float y_hi,
                                                           const int64_t *start, int32_t *fill, int32_t *order) {
    __shared__ uint32_t h[ORDER_BUCKETS];
    __shared__ int32_t run0[ORDER_BUCKETS];
    for (int i = threadIdx.x; i < ORDER_BUCKETS; i += ORDER_T) h[i] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * ORDER_CHUNK;
    const int64_t end = base + ORDER_CHUNK < n ? base + ORDER_CHUNK : n;
    for (int64_t i = base + threadIdx.x; i < end; i += ORDER_T) atomicAdd(&h[order_bucket(y[i], y_lo, y_hi)], 1u);
    __syncthreads();
    for (int i = threadIdx.x; i < ORDER_BUCKETS; i += ORDER_T) {
        if (h[i]) run0[i] = atomicAdd(&fill[i], (int32_t)h[i]);
        h[i] = 0;
    }
    __syncthreads();
    for (int64_t i = base + threadIdx.x; i < end; i += ORDER_T) {
        const int b = order_bucket(y[i], y_lo, y_hi);
        order[start[b] + run0[b] + (int64_t)atomicAdd(&h[b], 1u)] = (int32_t)i;
    }
}

// ---------------------------------------------------------------------------
// The same order at the granularity of plans: the columns that share a plan
// (the orbitals of one atom) are kept next to each other, so that the seed
// pass that runs a plan's columns in one wavefront finds them together; plans
// are queued by the largest prediction among their columns.
// ---------------------------------------------------------------------------
__global__ void k_zero_i64_one(int64_t *p) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *p = 0;
}

__global__ void k_group_init(int32_t n_plans, float y_lo, float *key, int32_t *cnt, int32_t *fill) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_plans; i += gridDim.x * blockDim.x) {
        key[i] = y_lo;
        cnt[i] = 0;
        fill[i] = 0;
    }
}

// per plan: the largest (clamped) prediction of its columns, and its column count
__global__ void k_group_key(const float *pred, int64_t n, const int32_t *col_plan, int32_t n_plans, float y_lo,
                            float y_hi, float *key, int32_t *cnt) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t p = col_plan[i];
        if (p < 0 || p >= n_plans) continue;
        const float y = fminf(fmaxf(pred[i], y_lo), y_hi) - y_lo;   // >= 0: its bits order like the values
        atomicMax(reinterpret_cast<int32_t *>(&key[p]), __float_as_int(y));
        atomicAdd(&cnt[p], 1);
    }
}

// after the plans are ordered: rank of each plan, and its column count by rank
__global__ void k_group_rank(const int32_t *plan_order, int32_t n_plans, const int32_t *cnt, int32_t *rank,
                             int64_t *size_by_rank) {
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n_plans; r += gridDim.x * blockDim.x) {
        const int32_t p = plan_order[r];
        rank[p] = r;
        size_by_rank[r + 1] = cnt[p];
        if (r == 0) size_by_rank[0] = 0;
    }
}

// every column into its plan's run (offsets are inclusive sums shifted by one)
__global__ void k_group_scatter(int64_t n, const int32_t *col_plan, int32_t n_plans, const int32_t *rank,
                                const int64_t *start, int32_t *fill, int32_t *order, int64_t *n_out) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t p = col_plan[i];
        if (p < 0 || p >= n_plans) {
            // a column without a valid plan goes last; the solve reports it
            order[n - 1 - atomicAdd(reinterpret_cast<unsigned long long *>(n_out), 1ull)] = (int32_t)i;
            continue;
        }
        order[start[rank[p]] + atomicAdd(&fill[p], 1)] = (int32_t)i;
    }
}

}  // namespace sgf

using namespace sgf;

extern "C" sgf_status sgf_features(const sgf_system *sys, const sgf_plan *plan, int64_t n_cols, const int64_t *d_cols,
                                   const int32_t *d_col_plan, float *d_feat, void *stream) {
    SGF_REQUIRE(sys && plan && sys->h, "sgf_features: NULL system or plan");
    SGF_REQUIRE(plan->atom_off && plan->blk_off && plan->lrow && plan->lblk && plan->center_loc,
                "sgf_features: plan has not been built");
    SGF_REQUIRE(n_cols >= 0 && (n_cols == 0 || (d_cols && d_col_plan && d_feat)), "sgf_features: NULL array");
    if (n_cols == 0) return SGF_OK;
    FeatArgs a{n_cols, plan->n_plans, d_cols, d_col_plan, sys->h, plan->atom_off, plan->blk_off, plan->lrow,
               plan->lblk, plan->center_loc, d_feat};
    k_features<<<dim3((unsigned)((n_cols + 255) / 256)), 256, 0, as_stream(stream)>>>(a);
    SGF_LAUNCHED();
    return SGF_OK;
}

extern "C" sgf_status sgf_mlp_normalize(float *d_params, const float *d_feat, int64_t n, void *stream) {
    SGF_REQUIRE(d_params && d_feat && n > 0, "sgf_mlp_normalize: bad arguments");
    k_mlp_normalize<<<1, 256, 0, as_stream(stream)>>>(d_params, d_feat, n);
    SGF_LAUNCHED();
    return SGF_OK;
}

extern "C" sgf_status sgf_mlp_forward(const float *d_params, const float *d_feat, int64_t n, float *d_y, void *stream) {
    SGF_REQUIRE(d_params && n >= 0 && (n == 0 || (d_feat && d_y)), "sgf_mlp_forward: bad arguments");
    if (n == 0) return SGF_OK;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    k_mlp_forward<<<dim3((unsigned)blocks), 256, 0, as_stream(stream)>>>(d_params, d_feat, n, d_y);
    SGF_LAUNCHED();
    return SGF_OK;
}

static sgf_status train_launch(bool update, TrainArgs a, void *stream) {
    auto fn = update ? k_mlp_train<true> : k_mlp_train<false>;
    SGF_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(fn), hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)TRAIN_LDS));
    hipLaunchKernelGGL(fn, dim3(1), dim3(TRAIN_T), TRAIN_LDS, as_stream(stream), a);
    SGF_LAUNCHED();
    return SGF_OK;
}

extern "C" sgf_status sgf_mlp_train_step(float *d_params, float *d_adam_m, float *d_adam_v, int32_t step, float lr,
                                         const float *d_feat, const float *d_target, int32_t n, float *d_loss,
                                         void *stream) {
    SGF_REQUIRE(d_params && d_adam_m && d_adam_v && d_feat && d_target, "sgf_mlp_train_step: NULL pointer");
    SGF_REQUIRE(n >= 1 && n <= TRAIN_T, "sgf_mlp_train_step: n must be in [1, %d]", TRAIN_T);
    SGF_REQUIRE(step >= 1 && lr > 0.0f, "sgf_mlp_train_step: step >= 1 and lr > 0 required");
    TrainArgs a{d_params, d_adam_m, d_adam_v, nullptr, d_loss, d_feat, d_target, n, step, lr};
    return train_launch(true, a, stream);
}

extern "C" sgf_status sgf_mlp_gradient(const float *d_params, const float *d_feat, const float *d_target, int32_t n,
                                       float *d_grad, float *d_loss, void *stream) {
    SGF_REQUIRE(d_params && d_feat && d_target && d_grad, "sgf_mlp_gradient: NULL pointer");
    SGF_REQUIRE(n >= 1 && n <= TRAIN_T, "sgf_mlp_gradient: n must be in [1, %d]", TRAIN_T);
    TrainArgs a{const_cast<float *>(d_params), nullptr, nullptr, d_grad, d_loss, d_feat, d_target, n, 1, 1.0f};
    return train_launch(false, a, stream);
}

extern "C" sgf_status sgf_order_workspace(size_t *ws_bytes) {
    SGF_REQUIRE(ws_bytes, "sgf_order_workspace: NULL");
    *ws_bytes = align_up(sizeof(int64_t) * (ORDER_BUCKETS + 1)) + align_up(sizeof(int32_t) * ORDER_BUCKETS) +
                prefix_scratch_bytes(ORDER_BUCKETS);
    return SGF_OK;
}

extern "C" sgf_status sgf_order_by_prediction(const float *d_pred, int64_t n, float y_lo, float y_hi,
                                              int32_t *d_order, void *d_ws, size_t ws_bytes, void *stream) {
    SGF_REQUIRE(n >= 0 && (n == 0 || (d_pred && d_order)), "sgf_order_by_prediction: NULL array");
    SGF_REQUIRE(y_hi > y_lo, "sgf_order_by_prediction: y_hi must exceed y_lo");
    SGF_REQUIRE(n < ((int64_t)1 << 31), "sgf_order_by_prediction: n too large");
    size_t need = 0;
    sgf_order_workspace(&need);
    SGF_REQUIRE(d_ws && ws_bytes >= need, "sgf_order_by_prediction: workspace %zu < %zu", ws_bytes, need);
    if (n == 0) return SGF_OK;
    Carve cv(d_ws, ws_bytes);
    int64_t *cnt = cv.take<int64_t>(ORDER_BUCKETS + 1);
    int32_t *fill = cv.take<int32_t>(ORDER_BUCKETS);
    char *scan = cv.take<char>(prefix_scratch_bytes(ORDER_BUCKETS));
    hipStream_t st = as_stream(stream);
    const int64_t blocks = (n + ORDER_CHUNK - 1) / ORDER_CHUNK;
    k_order_zero<<<(ORDER_BUCKETS + 256) / 256, 256, 0, st>>>(cnt, fill);
    k_order_hist<<<dim3((unsigned)blocks), ORDER_T, 0, st>>>(d_pred, n, y_lo, y_hi, cnt);
    SGF_LAUNCHED();
    sgf_status rc = inclusive_scan_i64(cnt + 1, ORDER_BUCKETS, scan, st);
    if (rc) return rc;
    k_order_scatter<<<dim3((unsigned)blocks), ORDER_T, 0, st>>>(d_pred, n, y_lo, y_hi, cnt, fill, d_order);
    SGF_LAUNCHED();
    return SGF_OK;
}

extern "C" sgf_status sgf_order_groups_workspace(int64_t n_plans, size_t *ws_bytes) {
    SGF_REQUIRE(ws_bytes && n_plans >= 0 && n_plans < ((int64_t)1 << 31), "sgf_order_groups_workspace: bad arguments");
    size_t order_ws = 0;
    sgf_order_workspace(&order_ws);
    const int64_t np = n_plans > 0 ? n_plans : 1;
    *ws_bytes = align_up(4 * np) * 5 + align_up(8 * (np + 1)) + align_up(8) + prefix_scratch_bytes(np) + align_up(order_ws);
    return SGF_OK;
}

extern "C" sgf_status sgf_order_groups_by_prediction(const float *d_pred, int64_t n, const int32_t *d_col_plan,
                                                     int64_t n_plans, float y_lo, float y_hi, int32_t *d_order,
                                                     void *d_ws, size_t ws_bytes, void *stream) {
    SGF_REQUIRE(n >= 0 && (n == 0 || (d_pred && d_col_plan && d_order)), "sgf_order_groups_by_prediction: NULL array");
    SGF_REQUIRE(y_hi > y_lo, "sgf_order_groups_by_prediction: y_hi must exceed y_lo");
    SGF_REQUIRE(n < ((int64_t)1 << 31) && n_plans >= 1 && n_plans < ((int64_t)1 << 31),
                "sgf_order_groups_by_prediction: bad sizes");
    size_t need = 0;
    sgf_order_groups_workspace(n_plans, &need);
    SGF_REQUIRE(d_ws && ws_bytes >= need, "sgf_order_groups_by_prediction: workspace %zu < %zu", ws_bytes, need);
    if (n == 0) return SGF_OK;
    size_t order_ws = 0;
    sgf_order_workspace(&order_ws);
    Carve cv(d_ws, ws_bytes);
    float *key = cv.take<float>(n_plans);
    int32_t *cnt = cv.take<int32_t>(n_plans);
    int32_t *fill = cv.take<int32_t>(n_plans);
    int32_t *rank = cv.take<int32_t>(n_plans);
    int32_t *plan_order = cv.take<int32_t>(n_plans);
    int64_t *start = cv.take<int64_t>(n_plans + 1);
    int64_t *n_out = cv.take<int64_t>(1);
    char *scan = cv.take<char>(prefix_scratch_bytes(n_plans));
    void *ows = cv.take<char>(order_ws);
    hipStream_t st = as_stream(stream);
    const unsigned gp = (unsigned)((n_plans + 255) / 256 < 4096 ? (n_plans + 255) / 256 : 4096);
    const unsigned gc = (unsigned)((n + 255) / 256 < 8192 ? (n + 255) / 256 : 8192);
    k_group_init<<<gp, 256, 0, st>>>((int32_t)n_plans, 0.0f, key, cnt, fill);
    k_zero_i64_one<<<1, 64, 0, st>>>(n_out);
    k_group_key<<<gc, 256, 0, st>>>(d_pred, n, d_col_plan, (int32_t)n_plans, y_lo, y_hi, key, cnt);
    SGF_LAUNCHED();
    // plans, largest key first (keys are predictions shifted by y_lo)
    sgf_status rc = sgf_order_by_prediction(key, n_plans, 0.0f, y_hi - y_lo, plan_order, ows, order_ws, stream);
    if (rc) return rc;
    k_group_rank<<<gp, 256, 0, st>>>(plan_order, (int32_t)n_plans, cnt, rank, start);
    SGF_LAUNCHED();
    rc = inclusive_scan_i64(start + 1, n_plans, scan, st);
    if (rc) return rc;
    k_group_scatter<<<gc, 256, 0, st>>>(n, d_col_plan, (int32_t)n_plans, rank, start, fill, d_order, n_out);
    SGF_LAUNCHED();
    return SGF_OK;
}
