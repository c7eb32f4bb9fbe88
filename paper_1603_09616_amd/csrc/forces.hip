// forces.hip -- band-structure forces from the density matrix (the force
// step of the quantum molecular dynamics, Sec. 2 of the paper), and the
// velocity-Verlet update that advances the atoms with them.
//
// The band energy of the solved columns is E_band = sum_j sum_{i in P(j)}
// rho_ij H_ij (per spin).  With an orthogonal basis (S = I) the force is
// F_A = -dE_band/dR_A at fixed rho.  With an overlap S, Hellmann-Feynman
// for H c = lambda S c adds the energy-density matrix eps (the quadrature of
// rho with the weight w_k z_k):
//   F_A = -sum_j sum_{i in P(j)} (rho_ij dH_ij/dR_A - eps_ij dS_ij/dR_A).
// Each column's rho and eps come from its own local subspace, so they are
// not symmetric and both atoms of a block take part: H_ij and S_ij for
// orbital i on atom B and j on atom C (B != C) are element (o_i, q_j) of the
// Slater-Koster block h(d) and of the overlap block s(d) = s_amp
// exp(-(r - r0)/s_decay) I4, d = R_C - R_B, and the term
// g = rho_ij grad h_{o_i q_j}(d) - eps_ij grad s_{o_i q_j}(d) enters F_C with
// a minus sign and F_B with a plus sign.  On-site blocks do not depend on
// positions, and a pair farther apart than r_cut has no block.
//
// One thread per column walks its projection rows, sums the terms of each
// neighbour atom (its rows are consecutive) and adds them, and the total of
// the column, into the force array with FP64 atomics.  The summation order of
// those atomics is not fixed: repeated runs agree to rounding, not bit for
// bit.
#include "common.hpp"

namespace sgf {

namespace {

constexpr int FORCE_T = 256;

// Gradient with respect to d of element (o, q) of the Slater-Koster block
// (orbitals s, px, py, pz): with c = d / r and f = (r0 / r)^power,
// dc_a/dd_k = (delta_ak - c_a c_k) / r and df/dd_k = -power f c_k / r.
__device__ void sk_elem_grad(const sgf_tb_params &p, double d0, double d1, double d2, int o, int q, double g[3]) {
    const double r = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
    const double ir = 1.0 / r;
    const double c[3] = {d0 * ir, d1 * ir, d2 * ir};
    const double f = pow(p.r0 * ir, p.power);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double df = -p.power * f * c[k] * ir;
        double v;
        if (o == 0 && q == 0) {
            v = p.v_sss * df;
        } else if (o == 0 || q == 0) {
            const int a = (o == 0 ? q : o) - 1;
            const double dca = ((a == k ? 1.0 : 0.0) - c[a] * c[k]) * ir;
            v = p.v_sps * (dca * f + c[a] * df);
            if (q == 0) v = -v;
        } else {
            const int a = o - 1, b = q - 1;
            const double dca = ((a == k ? 1.0 : 0.0) - c[a] * c[k]) * ir;
            const double dcb = ((b == k ? 1.0 : 0.0) - c[b] * c[k]) * ir;
            v = (dca * c[b] + c[a] * dcb) * (p.v_pps - p.v_ppp) * f +
                (c[a] * c[b] * (p.v_pps - p.v_ppp) + (a == b ? p.v_ppp : 0.0)) * df;
        }
        g[k] = v;
    }
}

__device__ __forceinline__ void add3(double *F, int64_t atom, const double g[3], double sign) {
    atomicAdd(&F[3 * atom + 0], sign * g[0]);
    atomicAdd(&F[3 * atom + 1], sign * g[1]);
    atomicAdd(&F[3 * atom + 2], sign * g[2]);
}

__global__ __launch_bounds__(FORCE_T) void k_zero_f64(int64_t n, double *x) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        x[i] = 0.0;
}

__global__ __launch_bounds__(FORCE_T) void k_band_force(int64_t n_cols, int64_t n_atoms, const double *xyz,
                                                        sgf_tb_params p, const int64_t *cols, const int64_t *proj_off,
                                                        const int32_t *proj_row, const int32_t *status, const double *rho,
                                                        const double *eps, double *F) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_cols) return;
    if (status && status[c] != SGF_CONVERGED) return;  // a rejected column holds no rho
    const int64_t j = cols[c];
    const int64_t C = j >> 2;
    if (j < 0 || C >= n_atoms) return;
    const int q = (int)(j & 3);
    const double rc0 = xyz[3 * C], rc1 = xyz[3 * C + 1], rc2 = xyz[3 * C + 2];
    double own[3] = {0.0, 0.0, 0.0}, nb[3] = {0.0, 0.0, 0.0};
    int64_t cur = -1;
    for (int64_t t = proj_off[c]; t < proj_off[c + 1]; ++t) {
        const int32_t i = proj_row[t];
        const int64_t B = i >> 2;
        if (B == C || B < 0 || B >= n_atoms) continue;
        const double d0 = rc0 - xyz[3 * B], d1 = rc1 - xyz[3 * B + 1], d2 = rc2 - xyz[3 * B + 2];
        const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
        if (r2 > p.r_cut * p.r_cut) continue;  // no block beyond the cut
        if (B != cur) {
            if (cur >= 0) add3(F, cur, nb, 1.0);
            cur = B;
            nb[0] = nb[1] = nb[2] = 0.0;
        }
        double g[3];
        sk_elem_grad(p, d0, d1, d2, i & 3, q, g);
        const double w = rho[t];
#pragma unroll
        for (int k = 0; k < 3; ++k) g[k] *= w;
        if (eps && (i & 3) == q) {
            // -eps grad s: grad s = -s(r) d / (s_decay r) on the diagonal of the block
            const double r = sqrt(r2);
            const double e = eps[t] * p.s_amp * exp(-(r - p.r0) / p.s_decay) / (p.s_decay * r);
            g[0] = fma(e, d0, g[0]);
            g[1] = fma(e, d1, g[1]);
            g[2] = fma(e, d2, g[2]);
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            nb[k] += g[k];
            own[k] += g[k];
        }
    }
    if (cur >= 0) add3(F, cur, nb, 1.0);
    add3(F, C, own, -1.0);
}

// Velocity Verlet (Swope et al. 1982), one thread per coordinate: the half
// kick v += (h / 2) F / m and the drift x += h v, in nm, fs, eV/nm and amu.
__global__ void k_md_kick(int64_t n3, const double *__restrict__ F, const double *__restrict__ mass, double c,
                          double *__restrict__ v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n3; i += (int64_t)gridDim.x * blockDim.x)
        v[i] = fma(c / mass[i / 3], F[i], v[i]);
}

__global__ void k_md_drift(int64_t n3, const double *__restrict__ v, double h, double *__restrict__ x) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n3; i += (int64_t)gridDim.x * blockDim.x)
        x[i] = fma(h, v[i], x[i]);
}

}  // namespace

}  // namespace sgf

using namespace sgf;

extern "C" sgf_status sgf_md_kick(int64_t n_atoms, const double *d_force, const double *d_mass, double h_fs,
                                  double *d_vel, void *stream) {
    SGF_REQUIRE(n_atoms >= 0 && d_force && d_mass && d_vel, "sgf_md_kick: NULL argument or n_atoms < 0");
    SGF_REQUIRE(h_fs == h_fs && h_fs > -1e6 && h_fs < 1e6, "sgf_md_kick: bad time step");
    if (n_atoms == 0) return SGF_OK;
    const int64_t n3 = 3 * n_atoms;
    const unsigned g = (unsigned)((n3 + FORCE_T - 1) / FORCE_T < 65536 ? (n3 + FORCE_T - 1) / FORCE_T : 65536);
    k_md_kick<<<g, FORCE_T, 0, as_stream(stream)>>>(n3, d_force, d_mass, 0.5 * h_fs * SGF_ACCEL_EV_NM_AMU, d_vel);
    SGF_LAUNCHED();
    return SGF_OK;
}

extern "C" sgf_status sgf_md_drift(int64_t n_atoms, const double *d_vel, double h_fs, double *d_xyz, void *stream) {
    SGF_REQUIRE(n_atoms >= 0 && d_vel && d_xyz, "sgf_md_drift: NULL argument or n_atoms < 0");
    SGF_REQUIRE(h_fs == h_fs && h_fs > -1e6 && h_fs < 1e6, "sgf_md_drift: bad time step");
    if (n_atoms == 0) return SGF_OK;
    const int64_t n3 = 3 * n_atoms;
    const unsigned g = (unsigned)((n3 + FORCE_T - 1) / FORCE_T < 65536 ? (n3 + FORCE_T - 1) / FORCE_T : 65536);
    k_md_drift<<<g, FORCE_T, 0, as_stream(stream)>>>(n3, d_vel, h_fs, d_xyz);
    SGF_LAUNCHED();
    return SGF_OK;
}

extern "C" sgf_status sgf_band_forces(const sgf_system *sys, const double *d_xyz, const sgf_tb_params *p,
                                      int64_t n_cols, const int64_t *d_cols, const int64_t *d_proj_off,
                                      const int32_t *d_proj_row, const int32_t *d_status, const double *d_rho,
                                      const double *d_eps, double *d_force, void *stream) {
    SGF_REQUIRE(sys && d_xyz && p && d_force, "sgf_band_forces: NULL argument");
    SGF_REQUIRE(sys->n_atoms > 0 && n_cols >= 0, "sgf_band_forces: bad sizes");
    SGF_REQUIRE(n_cols == 0 || (d_cols && d_proj_off && d_proj_row && d_rho), "sgf_band_forces: column layout is NULL");
    SGF_REQUIRE(p->r0 > 0.0 && p->r_cut > 0.0, "sgf_band_forces: r0 and r_cut must be positive");
    SGF_REQUIRE(!sys->s == !p->overlap, "sgf_band_forces: the parameters' overlap flag does not match the system");
    SGF_REQUIRE(!sys->s || p->s_decay > 0.0, "sgf_band_forces: s_decay must be positive");
    SGF_REQUIRE(!sys->s || n_cols == 0 || d_eps, "sgf_band_forces: an overlap needs the energy-density matrix");
    hipStream_t st = as_stream(stream);
    const int64_t nf = 3 * sys->n_atoms;
    const unsigned gz = (unsigned)((nf + FORCE_T - 1) / FORCE_T < 65536 ? (nf + FORCE_T - 1) / FORCE_T : 65536);
    k_zero_f64<<<gz, FORCE_T, 0, st>>>(nf, d_force);
    SGF_LAUNCHED();
    if (n_cols > 0) {
        k_band_force<<<(unsigned)((n_cols + FORCE_T - 1) / FORCE_T), FORCE_T, 0, st>>>(
            n_cols, sys->n_atoms, d_xyz, *p, d_cols, d_proj_off, d_proj_row, d_status, d_rho,
            sys->s ? d_eps : nullptr, d_force);
        SGF_LAUNCHED();
    }
    return SGF_OK;
}
