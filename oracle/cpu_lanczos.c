/* Plain CPU comparator for the matrix-free Krylov path: complex128, OpenMP over amplitudes,
 * no tiling.  Test and benchmark infrastructure only (compared against, never called by, the
 * GPU library).
 *
 * A block Hamiltonian is a sum of Pauli strings c_t X^{x_t} Z^{z_t} (Z applied first), so
 *   (H v)[m] = sum_t c_t (-1)^{popcount((m ^ x_t) & z_t)} v[m ^ x_t]
 * (the matrix-free application of the supplement, Sec. I.A).  Lanczos is the plain three-term
 * recurrence of the supplement's Krylov propagator: w = H v_j - beta_{j-1} v_{j-1},
 * alpha_j = <v_j, w>, w -= alpha_j v_j, beta_j = ||w||, v_{j+1} = w / beta_j. */
#include <complex.h>
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

void cpu_apply(int L, int K, const uint64_t *xm, const uint64_t *zm, const double *cre, const double *cim,
               const double complex *v, double complex *y) {
    const int64_t n = (int64_t)1 << L;
#pragma omp parallel for schedule(static)
    for (int64_t m = 0; m < n; ++m) {
        double complex acc = 0.0;
        for (int t = 0; t < K; ++t) {
            const uint64_t s = (uint64_t)m ^ xm[t];
            const double complex c = cre[t] + I * cim[t];
            acc += (__builtin_popcountll(s & zm[t]) & 1) ? -c * v[s] : c * v[s];
        }
        y[m] = acc;
    }
}

/* steps Lanczos iterations from v0 (normalised first).  alpha, beta: steps values each.
 * seconds[0] = total time in cpu_apply, seconds[1] = total time of the whole iterations.
 * Returns the number of OpenMP threads used, or -1 when memory runs out. */
int cpu_lanczos(int L, int K, const uint64_t *xm, const uint64_t *zm, const double *cre, const double *cim,
                const double complex *v0, int steps, double *alpha, double *beta, double *seconds) {
    const int64_t n = (int64_t)1 << L;
    double complex *vp = calloc((size_t)n, sizeof(double complex));
    double complex *v = malloc((size_t)n * sizeof(double complex));
    double complex *w = malloc((size_t)n * sizeof(double complex));
    if (!vp || !v || !w) {
        free(vp);
        free(v);
        free(w);
        return -1;
    }
    double nrm = 0.0;
#pragma omp parallel for reduction(+ : nrm)
    for (int64_t m = 0; m < n; ++m) nrm += creal(v0[m] * conj(v0[m]));
    nrm = sqrt(nrm);
#pragma omp parallel for
    for (int64_t m = 0; m < n; ++m) v[m] = v0[m] / nrm;
    double t_apply = 0.0, t0 = omp_get_wtime(), b_prev = 0.0;
    for (int j = 0; j < steps; ++j) {
        const double ta = omp_get_wtime();
        cpu_apply(L, K, xm, zm, cre, cim, v, w);
        t_apply += omp_get_wtime() - ta;
        double ar = 0.0;
#pragma omp parallel for reduction(+ : ar)
        for (int64_t m = 0; m < n; ++m) {
            w[m] -= b_prev * vp[m];
            ar += creal(conj(v[m]) * w[m]);
        }
        double bb = 0.0;
#pragma omp parallel for reduction(+ : bb)
        for (int64_t m = 0; m < n; ++m) {
            w[m] -= ar * v[m];
            bb += creal(w[m] * conj(w[m]));
        }
        alpha[j] = ar;
        beta[j] = sqrt(bb);
        const double s = beta[j] > 0.0 ? 1.0 / beta[j] : 0.0;
#pragma omp parallel for
        for (int64_t m = 0; m < n; ++m) {
            vp[m] = v[m];
            v[m] = w[m] * s;
        }
        b_prev = beta[j];
    }
    seconds[0] = t_apply;
    seconds[1] = omp_get_wtime() - t0;
    free(vp);
    free(v);
    free(w);
    return omp_get_max_threads();
}
