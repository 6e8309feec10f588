// Finite-size-scaling analysis of OTOC curves (host only): crossing times t*(N), inverse
// slopes and the fits of Eq. (5) and Eq. (6).
#pragma once

#include <vector>

namespace syk {

// First n >= 1 with F[n] <= F0 < F[n-1]; linear interpolation inside [t[n-1], t[n]].
// Returns false (t* undefined) when the curve never falls to F0.  err (may be null) gets
// sigma_F(t*) / |slope| with sigma_F interpolated linearly (NaN when F_err is null).
bool crossing_time(const double *t, const double *F, const double *F_err, int nt, double F0, double &tstar,
                   double *err);

struct SlopePoint {
    double N_mid, y, err;
};

// Inverse slopes y = log(N_b / N_a) / (t*_b - t*_a) for every pair N_b = N_a + dN, placed at
// sqrt(N_a N_b); err = |y| sqrt(s_a^2 + s_b^2) / |t*_b - t*_a| (NaN without errors).
std::vector<SlopePoint> slope_points(const double *N, const double *tstar, const double *tstar_err, int n,
                                     int dN);

// Linear least squares min sum_i w_i (y_i - sum_j A_ij p_j)^2 by Householder QR of the
// column-scaled, row-weighted matrix.  cov = (A^T W A)^{-1}.  Throws SYK_EINVAL when the
// columns are (numerically) dependent.
struct LsqSolution {
    std::vector<double> p, cov;   // cov: k x k row-major
    double rss;                   // weighted residual sum of squares
};
LsqSolution least_squares(const std::vector<double> &A, const std::vector<double> &y,
                          const std::vector<double> &w, int n, int k);

}  // namespace syk
