// contour.hip -- shifts and weights that give the Fermi-Dirac density matrix
// from a few complex energies (host code; the shifted solve does the rest).
//
// The order-N energy of the Introduction needs rho = f(H) for the Fermi
// occupation f(e) = 1 / (1 + exp((e - mu)/kT)).  With y = (e - mu)/kT,
// f = 1/2 - tanh(y/2)/2, and Lambert's continued fraction for tanh, cut
// after 2N partial denominators, is a rational function whose poles lie on
// the imaginary axis (the representation of Ozaki, Phys. Rev. B 75, 035123
// (2007)):
//     f(y) = 1/2 - sum_{p=1..N} R_p (1/(y - i z_p) + 1/(y + i z_p)).
// The z_p and R_p follow from the symmetric tridiagonal matrix B of order 2N
// with zero diagonal and off-diagonal b_m = 1/sqrt((2m-1)(2m+1)): for each
// positive eigenvalue l, z = 2/l and R = q1^2/l^2, q1 the first entry of the
// unit eigenvector.  With G(z) = (zS - H)^{-1} and sum over eigenpairs
// v v^T = S^{-1}:
//     rho = S^{-1}/2 + 2 kT sum_p R_p Re G(mu + i z_p kT),
// and S^{-1} = Re(i M G(i M)) up to |H|^2/M^2.  In the solve's quadrature
// form rho = -(1/pi) sum_k Im(w_k G(z_k)) that is N + 1 shifts.
//
// Eigenvalues: bisection on the Sturm count of B - x (each to a last bit).
// q1^2: with T_k(x) = det(x - B[k:, k:]) (trailing minors, T_0 the
// characteristic polynomial), e1^T (x - B)^{-1} e1 = T_1(x) / T_0(x), whose
// residue at an eigenvalue l is q1^2 = T_1(l) / T_0'(l); T and T' follow one
// three-term recurrence from the bottom, rescaled jointly (the ratio does not
// change) to stay within the exponent range.
#include "common.hpp"

#include <cmath>
#include <vector>

namespace sgf {
namespace {

// eigenvalues of B below x
int sturm_below(const std::vector<double> &b2, double x) {
    const int n = (int)b2.size() + 1;
    int cnt = 0;
    double q = -x;
    if (q < 0) ++cnt;
    for (int m = 1; m < n; ++m) {
        if (q == 0.0) q = 1e-300;
        q = -x - b2[m - 1] / q;
        if (q < 0) ++cnt;
    }
    return cnt;
}

}  // namespace
}  // namespace sgf

using namespace sgf;

extern "C" sgf_status sgf_fermi_shifts(int32_t n_poles, double kT, double mu, double moment, double *z, double *w) {
    SGF_REQUIRE(n_poles >= 1 && n_poles <= 511, "sgf_fermi_shifts: n_poles must be in [1, 511]");
    SGF_REQUIRE(kT > 0 && std::isfinite(kT) && std::isfinite(mu), "sgf_fermi_shifts: kT must be positive, mu finite");
    SGF_REQUIRE(moment > 0 && std::isfinite(moment), "sgf_fermi_shifts: the moment shift must be positive");
    SGF_REQUIRE(z && w, "sgf_fermi_shifts: NULL output");
    const int n = 2 * n_poles;
    std::vector<double> b2(n - 1);
    for (int m = 1; m < n; ++m) b2[m - 1] = 1.0 / ((2.0 * m - 1.0) * (2.0 * m + 1.0));
    // |eigenvalues| <= 2 max b < 1.2 (Gershgorin); the positive ones are the
    // (n_poles + 1)-th to n-th smallest, and pole p = 1 (nearest the real
    // axis) belongs to the largest eigenvalue
    for (int p = 0; p < n_poles; ++p) {
        const int k = n - p;  // 1-based rank of the eigenvalue
        double lo = 0.0, hi = 1.2;
        for (int it = 0; it < 2000; ++it) {
            const double mid = 0.5 * (lo + hi);
            if (mid <= lo || mid >= hi) break;
            (sturm_below(b2, mid) >= k ? hi : lo) = mid;
        }
        const double l = 0.5 * (lo + hi);
        double T2 = 1.0, T1 = l, d2 = 0.0, d1 = 1.0;
        for (int kk = n - 2; kk >= 0; --kk) {
            const double T0 = l * T1 - b2[kk] * T2;
            const double d0 = T1 + l * d1 - b2[kk] * d2;
            T2 = T1;
            T1 = T0;
            d2 = d1;
            d1 = d0;
            const double s = std::fmax(std::fmax(std::fabs(T1), std::fabs(T2)), std::fmax(std::fabs(d1), std::fabs(d2)));
            if (s > 1e100 || (s < 1e-100 && s > 0.0)) {
                T1 /= s;
                T2 /= s;
                d1 /= s;
                d2 /= s;
            }
        }
        const double zp = 2.0 / l, Rp = T2 / d1 / (l * l);
        z[2 * p] = mu;
        z[2 * p + 1] = zp * kT;
        w[2 * p] = 0.0;
        w[2 * p + 1] = -2.0 * M_PI * kT * Rp;
    }
    z[2 * n_poles] = 0.0;
    z[2 * n_poles + 1] = moment;
    w[2 * n_poles] = 0.5 * M_PI * moment;
    w[2 * n_poles + 1] = 0.0;
    return SGF_OK;
}
