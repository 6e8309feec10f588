// Finite-size-scaling analysis (host only).  t*(N) follows the definition before Eq. (4):
// the time at which the disorder-averaged OTOC falls to F0.  The inverse slope of Eq. (5)
// uses the difference t*(N + dN) - t*(N) of the supplement (Sec. II.A, dN = 8), read as a
// central difference in log N; Eq. (6) is linear in (gamma_0, 1/lambda, gamma_1/lambda,
// gamma_2/lambda) and is solved in that form.
#include "analysis.hpp"

#include <algorithm>
#include <cmath>
#include <limits>

#include "internal.hpp"

namespace syk {

bool crossing_time(const double *t, const double *F, const double *F_err, int nt, double F0, double &tstar,
                   double *err) {
    const double nan = std::numeric_limits<double>::quiet_NaN();
    for (int n = 1; n < nt; ++n) {
        if (!(F[n] <= F0 && F0 < F[n - 1])) continue;
        const double dt = t[n] - t[n - 1];
        if (dt == 0.0) {
            tstar = t[n];
            if (err) *err = 0.0;
            return true;
        }
        const double w = (F[n - 1] - F0) / (F[n - 1] - F[n]);
        tstar = t[n - 1] + w * dt;
        if (err) {
            if (F_err) {
                const double sF = (1.0 - w) * F_err[n - 1] + w * F_err[n];
                *err = sF * dt / (F[n - 1] - F[n]);
            } else {
                *err = nan;
            }
        }
        return true;
    }
    tstar = nan;
    if (err) *err = nan;
    return false;
}

std::vector<SlopePoint> slope_points(const double *N, const double *tstar, const double *tstar_err, int n,
                                     int dN) {
    std::vector<SlopePoint> out;
    for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) {
            if (N[b] != N[a] + dN) continue;
            const double delta = tstar[b] - tstar[a];
            if (!(delta != 0.0) || !std::isfinite(delta))
                fail(SYK_EINVAL, "t* must differ between N and N + dN");
            const double y = std::log(N[b] / N[a]) / delta;
            double e = std::numeric_limits<double>::quiet_NaN();
            if (tstar_err) e = std::fabs(y) * std::hypot(tstar_err[a], tstar_err[b]) / std::fabs(delta);
            out.push_back(SlopePoint{std::sqrt(N[a] * N[b]), y, e});
        }
    return out;
}

LsqSolution least_squares(const std::vector<double> &A, const std::vector<double> &y,
                          const std::vector<double> &w, int n, int k) {
    if (n < k) fail(SYK_EINVAL, "fewer data points than fit parameters");
    // B = diag(sqrt w) A diag(1/colnorm), b = diag(sqrt w) y
    std::vector<double> B(static_cast<size_t>(n) * k), b(n), scale(k, 0.0);
    for (int i = 0; i < n; ++i) {
        const double sw = std::sqrt(w[i]);
        b[i] = sw * y[i];
        for (int j = 0; j < k; ++j) B[i * k + j] = sw * A[i * k + j];
    }
    for (int j = 0; j < k; ++j) {
        double s = 0.0;
        for (int i = 0; i < n; ++i) s += B[i * k + j] * B[i * k + j];
        scale[j] = std::sqrt(s);
        if (!(scale[j] > 0.0)) fail(SYK_EINVAL, "fit column is zero");
        for (int i = 0; i < n; ++i) B[i * k + j] /= scale[j];
    }
    // Householder QR: B = Q R, Q^T applied to b as we go
    for (int j = 0; j < k; ++j) {
        double nrm = 0.0;
        for (int i = j; i < n; ++i) nrm += B[i * k + j] * B[i * k + j];
        nrm = std::sqrt(nrm);
        const double alpha = B[j * k + j] > 0.0 ? -nrm : nrm;
        std::vector<double> v(n - j);
        for (int i = j; i < n; ++i) v[i - j] = B[i * k + j];
        v[0] -= alpha;
        double vv = 0.0;
        for (double e : v) vv += e * e;
        if (vv > 0.0) {
            for (int c = j; c < k; ++c) {
                double d = 0.0;
                for (int i = j; i < n; ++i) d += v[i - j] * B[i * k + c];
                const double f = 2.0 * d / vv;
                for (int i = j; i < n; ++i) B[i * k + c] -= f * v[i - j];
            }
            double d = 0.0;
            for (int i = j; i < n; ++i) d += v[i - j] * b[i];
            const double f = 2.0 * d / vv;
            for (int i = j; i < n; ++i) b[i] -= f * v[i - j];
        }
    }
    double rmax = 0.0;
    for (int j = 0; j < k; ++j) rmax = std::max(rmax, std::fabs(B[j * k + j]));
    for (int j = 0; j < k; ++j)
        if (!(std::fabs(B[j * k + j]) > 1e-12 * rmax)) fail(SYK_EINVAL, "fit is degenerate (dependent columns)");
    // R p' = (Q^T b)[0:k]; Rinv by back substitution; cov' = Rinv Rinv^T
    std::vector<double> p(k), Rinv(static_cast<size_t>(k) * k, 0.0);
    for (int j = k - 1; j >= 0; --j) {
        double s = b[j];
        for (int c = j + 1; c < k; ++c) s -= B[j * k + c] * p[c];
        p[j] = s / B[j * k + j];
    }
    for (int col = 0; col < k; ++col)
        for (int j = col; j >= 0; --j) {
            double s = j == col ? 1.0 : 0.0;
            for (int c = j + 1; c <= col; ++c) s -= B[j * k + c] * Rinv[c * k + col];
            Rinv[j * k + col] = s / B[j * k + j];
        }
    LsqSolution sol;
    sol.p.resize(k);
    sol.cov.assign(static_cast<size_t>(k) * k, 0.0);
    for (int j = 0; j < k; ++j) sol.p[j] = p[j] / scale[j];
    for (int r = 0; r < k; ++r)
        for (int c = 0; c < k; ++c) {
            double s = 0.0;
            for (int m = std::max(r, c); m < k; ++m) s += Rinv[r * k + m] * Rinv[c * k + m];
            sol.cov[r * k + c] = s / (scale[r] * scale[c]);
        }
    sol.rss = 0.0;
    for (int i = k; i < n; ++i) sol.rss += b[i] * b[i];
    return sol;
}

}  // namespace syk
