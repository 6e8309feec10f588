"""Finite-size-scaling analysis of the OTOC: crossing times t*(N) and the Lyapunov exponent.

Test infrastructure only (a plain float64 reference for the tests and the CPU baseline);
the library computes the same quantities in its own code.

* t*(N) is the time at which the disorder-averaged OTOC first falls to F0 (main text, the
  definition before Eq. (4)); here by linear interpolation between the two samples of the
  curve that bracket the crossing.
* Eq. (5) (and Eq. (S2) of the supplement): the inverse slope 1/(N dt*/dN) is fitted by
  lambda + alpha_1/N + alpha_2/N^2.  The slope comes from t*(N + dN) - t*(N), dN = 8
  (supplement Sec. II.A).  Reading: the inverse slope is dlog N / dt*, taken as the
  difference quotient log((N + dN)/N) / (t*(N + dN) - t*(N)) and placed at the geometric
  mid-point sqrt(N (N + dN)) (a central difference in log N).
* Eq. (6): t*(N) = gamma_0 + (log N / lambda)(1 + gamma_1/N + gamma_2/N^2), a model that is
  linear in (gamma_0, 1/lambda, gamma_1/lambda, gamma_2/lambda); it is solved as that linear
  least-squares problem and mapped back, with first-order error propagation.

Errors: with per-point standard errors the fit is weighted by 1/sigma^2 and the
parameter covariance is (A^T W A)^{-1}; without them the fit is unweighted and the
covariance is scaled by the residual variance chi^2 / (n - p).  The slope points of
neighbouring pairs share a t* value; their covariance is ignored (each inverse slope
carries its own propagated error).
"""
import numpy as np


def crossing_time(t, F, F0, F_err=None):
    """First downward crossing of F0 by the sampled curve F(t): the first n >= 1 with
    F[n] <= F0 < F[n-1], then linear interpolation between samples n-1 and n.
    Returns (t*, sigma_t*) with sigma_t* = sigma_F(t*) / |dF/dt| (sigma_F interpolated
    linearly, the slope that of the bracketing segment); (nan, nan) without a crossing."""
    t = np.asarray(t, dtype=np.float64)
    F = np.asarray(F, dtype=np.float64)
    for n in range(1, len(t)):
        if F[n] <= F0 < F[n - 1]:
            dt = t[n] - t[n - 1]
            if dt == 0.0:
                return float(t[n]), 0.0
            w = (F[n - 1] - F0) / (F[n - 1] - F[n])       # fraction of the segment
            ts = t[n - 1] + w * dt
            if F_err is None:
                return float(ts), float("nan")
            sF = (1.0 - w) * F_err[n - 1] + w * F_err[n]
            slope = (F[n] - F[n - 1]) / dt
            return float(ts), float(sF / abs(slope))
    return float("nan"), float("nan")


def slope_points(N, tstar, tstar_err=None, dN=8):
    """Inverse slopes 1/(N dt*/dN) from every pair (N, N + dN) present in the data.
    Returns arrays (N_mid, y, sigma_y); sigma_y is nan without tstar errors."""
    N = np.asarray(N, dtype=np.float64)
    ts = np.asarray(tstar, dtype=np.float64)
    out_n, out_y, out_e = [], [], []
    for a in range(len(N)):
        for b in range(len(N)):
            if N[b] == N[a] + dN:
                delta = ts[b] - ts[a]
                y = np.log(N[b] / N[a]) / delta
                out_n.append(np.sqrt(N[a] * N[b]))
                out_y.append(y)
                if tstar_err is None:
                    out_e.append(np.nan)
                else:
                    s = np.hypot(tstar_err[a], tstar_err[b])
                    out_e.append(abs(y) * s / abs(delta))
    return np.array(out_n), np.array(out_y), np.array(out_e)


def _lsq(A, y, sigma):
    """Weighted (sigma given) or unweighted linear least squares; returns (p, cov, chi2)."""
    n, k = A.shape
    if sigma is None:
        p, *_ = np.linalg.lstsq(A, y, rcond=None)
        r = y - A @ p
        chi2 = float(r @ r)
        cov = np.linalg.inv(A.T @ A)
        cov = cov * (chi2 / (n - k)) if n > k else np.full((k, k), np.nan)
        return p, cov, chi2
    w = 1.0 / np.asarray(sigma, dtype=np.float64)
    Aw = A * w[:, None]
    p, *_ = np.linalg.lstsq(Aw, y * w, rcond=None)
    r = (y - A @ p) * w
    return p, np.linalg.inv(Aw.T @ Aw), float(r @ r)


def fit_slope(N_mid, y, sigma=None, a1=True, a2=False):
    """Eq. (5): y = lambda + alpha_1/N + alpha_2/N^2 over the slope points.
    Returns dict(lambda, alpha1, alpha2, errors, chi2, dof); absent terms are 0."""
    N_mid = np.asarray(N_mid, dtype=np.float64)
    cols = [np.ones_like(N_mid)]
    if a1:
        cols.append(1.0 / N_mid)
    if a2:
        cols.append(1.0 / N_mid ** 2)
    A = np.stack(cols, axis=1)
    p, cov, chi2 = _lsq(A, np.asarray(y, dtype=np.float64), sigma)
    err = np.sqrt(np.diag(cov))
    out = {"lambda": p[0], "lambda_err": err[0], "alpha1": 0.0, "alpha1_err": 0.0, "alpha2": 0.0,
           "alpha2_err": 0.0, "chi2": chi2, "dof": len(y) - A.shape[1]}
    c = 1
    if a1:
        out["alpha1"], out["alpha1_err"] = p[c], err[c]
        c += 1
    if a2:
        out["alpha2"], out["alpha2_err"] = p[c], err[c]
    return out


def fit_global(N, tstar, sigma=None, g1=True, g2=False):
    """Eq. (6): t* = gamma_0 + (log N / lambda)(1 + gamma_1/N + gamma_2/N^2).
    Returns dict(lambda, gamma0, gamma1, gamma2, errors, chi2, dof); absent terms are 0."""
    N = np.asarray(N, dtype=np.float64)
    lg = np.log(N)
    cols = [np.ones_like(N), lg]
    if g1:
        cols.append(lg / N)
    if g2:
        cols.append(lg / N ** 2)
    A = np.stack(cols, axis=1)
    q, cov, chi2 = _lsq(A, np.asarray(tstar, dtype=np.float64), sigma)
    # q = (gamma_0, a, b, c) with a = 1/lambda, b = gamma_1/lambda, c = gamma_2/lambda
    a = q[1]
    J = np.zeros((A.shape[1], A.shape[1]))
    J[0, 0] = 1.0
    J[1, 1] = -1.0 / a ** 2
    for c in range(2, A.shape[1]):
        J[c, 1] = -q[c] / a ** 2
        J[c, c] = 1.0 / a
    cv = J @ cov @ J.T
    err = np.sqrt(np.diag(cv))
    out = {"lambda": 1.0 / a, "lambda_err": err[1], "gamma0": q[0], "gamma0_err": err[0], "gamma1": 0.0,
           "gamma1_err": 0.0, "gamma2": 0.0, "gamma2_err": 0.0, "chi2": chi2, "dof": len(N) - A.shape[1]}
    c = 2
    if g1:
        out["gamma1"], out["gamma1_err"] = q[c] / a, err[c]
        c += 1
    if g2:
        out["gamma2"], out["gamma2_err"] = q[c] / a, err[c]
    return out


def ensemble_mean(F_norm_rows):
    """Disorder average of per-realisation normalised curves (each F(0) = 1, Eq. (2)) and
    its standard error (sample standard deviation / sqrt(R); 0 for R = 1)."""
    F = np.atleast_2d(np.asarray(F_norm_rows, dtype=np.float64))
    R = F.shape[0]
    mean = F.mean(axis=0)
    sem = F.std(axis=0, ddof=1) / np.sqrt(R) if R > 1 else np.zeros_like(mean)
    return mean, sem
