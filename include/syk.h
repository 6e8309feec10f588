/*
 * syk.h -- C ABI of libsyk: the sparse q=4 SYK Hamiltonian applied matrix-free to
 * parity-block state vectors on an AMD Instinct MI355X (gfx950), and the Lanczos
 * propagators and regularised OTOC built on it.
 *
 * Paper: A. M. Garcia-Garcia, C. Liu, J. J. M. Verbaarschot, "Sparsity independent
 * Lyapunov exponent in the Sachdev-Ye-Kitaev model" (arXiv:2311.00639).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - N Majoranas, N even, 6 <= N <= 64.  L = N/2 - 1 block qubits; a parity block holds
 *    2^L amplitudes; the full space 2^(L+1), the parity qubit being the most significant
 *    index bit, U = parity 0 (first half), D = parity 1 (second half).
 *  - Majoranas chi_n = gamma_n / sqrt(2) with gamma_n the Jordan-Wigner Pauli strings of
 *    supplement Eq. (S1) (compact form): block strings A_0 = prod_q X_q and, for
 *    1 <= n <= N-2, A_n = (Y if n odd else Z)_{floor((n-1)/2)} prod_{q >= floor((n+1)/2)} X_q;
 *    gamma_n = X_parity (x) A_n (n <= N-2), gamma_{N-1} = Y_parity (x) 1, with
 *    sigma_y = [[0,-i],[i,0]].  Qubit q is bit q of the amplitude index.
 *  - H = sum_a J_a chi_i chi_j chi_k chi_l (Eq. (1)); each term restricted to a block is
 *    (J_a/4) i^p X^x Z^z, Z applied first (the <bits, coeff> encoding of supplement Sec. I.A).
 *  - State vectors are interleaved complex: (re, im) pairs of float (SYK_C64) or double
 *    (SYK_C128).  Vector pointers are DEVICE pointers on the current HIP device unless a
 *    parameter says "host"; the caller owns them.  Reductions (norms, dots, Lanczos
 *    alpha/beta, the tridiagonal exponential) are done in double for both dtypes.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Device work is enqueued on
 *    it; functions returning host results synchronise it.
 *  - Errors: every function returns a syk_status; no C++ exception crosses the ABI.  On
 *    failure, syk_last_error() returns a thread-local message.  Output buffers are left
 *    unspecified on failure.
 */
#ifndef SYK_H
#define SYK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct syk_ham syk_ham;      /* opaque, owned by the library, immutable after create */

typedef enum {
    SYK_OK = 0,
    SYK_EINVAL = 1,        /* invalid argument (range, null pointer, size mismatch) */
    SYK_EUNSUPPORTED = 2,  /* valid but not supported (q != 4) */
    SYK_ENOMEM = 3,        /* device or host allocation failed */
    SYK_EDEVICE = 4,       /* a HIP runtime call failed, or no GPU */
    SYK_ENOTCONV = 5,      /* Krylov step control could not meet the tolerance */
    SYK_ENUMERIC = 6,      /* NaN/Inf met in a reduction */
    SYK_ECANCELLED = 7,    /* request cancelled (engine) */
    SYK_EAGAIN = 8         /* engine: no finished request within the wait */
} syk_status;

typedef enum { SYK_C64 = 0, SYK_C128 = 1 } syk_dtype;
typedef enum {
    SYK_ENSEMBLE_EXACT_K = 0,   /* exactly K = round(k N) distinct 4-subsets, uniform */
    SYK_ENSEMBLE_BERNOULLI = 1  /* every 4-subset kept with probability p = k N / C(N,4) */
} syk_ensemble;
/* Parity sector of a state vector: the U block (even parity of the most significant qubit,
 * 2^L amplitudes), the D block, or the full 2^(L+1)-amplitude space (U block first, then D;
 * H is block diagonal in parity, so it acts on the two halves separately). */
typedef enum { SYK_BLOCK_U = 0, SYK_BLOCK_D = 1, SYK_FULL = 2 } syk_block;

typedef struct {
    int N, L, K;           /* Majoranas, block qubits, number of terms */
    double k;              /* requested sparsity k (K = round(k N)) */
    double p;              /* K / C(N,4) */
    double sigma;          /* coupling standard deviation sqrt(3! / (p N^3)) */
    double sum_J2;         /* sum_a J_a^2 (Tr H^2 / dim = sum_J2 / 16) */
    uint64_t seed;
    uint64_t block_dim;    /* 2^L */
} syk_ham_info;

/* ---------------------------------------------------------------- Hamiltonian
 * Draw one disorder realisation of Eq. (1) (main text, "Sparse SYK Model"): exactly
 * K = round(k N) distinct 4-subsets chosen uniformly and J ~ N(0, sigma^2),
 * sigma^2 = 3!/(p N^3), p = K / C(N,4).  Draws come from one SplitMix64 stream seeded
 * with `seed`: subset ranks by rejection (r >= 2^64 - 2^64 mod C(N,4) rejected), r mod
 * C(N,4) unranked in the colex combinatorial number system, duplicates skipped, subsets
 * sorted lexicographically, then per subset J = sigma sqrt(-2 ln u1) cos(2 pi u2) with
 * u1 = ((r1>>11)+1) 2^-53, u2 = (r2>>11) 2^-53.  Host-only: needs no GPU; device term
 * tables are uploaded lazily on first use on each device.
 * Errors: EINVAL (N odd or outside [6,64], K < 1 or K > C(N,4), out == NULL),
 * EUNSUPPORTED (q != 4), ENOMEM. */
syk_status syk_create_hamiltonian(int N, int q, double k, uint64_t seed, syk_ham **out);

/* As syk_create_hamiltonian for ensemble SYK_ENSEMBLE_EXACT_K.  SYK_ENSEMBLE_BERNOULLI is the
 * paper's own ensemble of Eq. (1): p_ijkl ~ B(p) with p = k N / C(N,4) (0 < p <= 1; p = 1
 * gives the dense SYK model, k = C(N,4) / N), J ~ N(0, 3!/(p N^3)).  Draws from one
 * SplitMix64 stream seeded with `seed`: one uniform (r>>11) 2^-53 per 4-subset in
 * lexicographic order, the subset kept iff it is below p; then per kept subset, in order,
 * J = sigma sqrt(-2 ln u1) cos(2 pi u2) as above.  The number of kept terms K is random
 * (reported by syk_ham_get_info).  Errors: EINVAL (as above, p outside (0, 1], no term
 * kept, unknown ensemble), EUNSUPPORTED (q != 4), ENOMEM. */
syk_status syk_create_hamiltonian_ensemble(int N, int q, double k, uint64_t seed, syk_ensemble ensemble,
                                           syk_ham **out);

/* Free a handle and its device tables on every device.  NULL is a no-op. */
syk_status syk_destroy_hamiltonian(syk_ham *h);

syk_status syk_ham_get_info(const syk_ham *h, syk_ham_info *out);

/* Copy the term table to host arrays of capacity `cap` (>= K; any pointer may be NULL):
 * ijkl[4a..4a+3] the sorted subset, J[a], and the block forms (J/4) i^phase X^x Z^z of
 * gamma_i gamma_j gamma_k gamma_l on U (phase_U) and D (phase_D), phase in {0,1,2,3}.
 * The product of the four strings is formed in canonical form by
 * (X^a Z^b)(X^c Z^d) = (-1)^{popcount(b & c)} X^{a^c} Z^{b^d} (supplement Sec. I.A: product
 * of spin operators = XOR of bits and a sign).  Host-only.  Errors: EINVAL (cap < K). */
syk_status syk_get_terms(const syk_ham *h, size_t cap, int32_t *ijkl, double *J,
                         uint64_t *xmask, uint64_t *zmask, int8_t *phase_U, int8_t *phase_D);

/* ---------------------------------------------------------------- apply_H
 * y = H_blk x, matrix-free (supplement Sec. I.A, Algorithm 1): for every m < 2^L,
 * y[m] = sum_a (J_a/4) i^{p_a} (-1)^{popcount((m ^ x_a) & z_a)} x[m ^ x_a].
 * x, y: device, `nvec` vectors, vector v at element offset v*ld, n_amps = 2^L complex
 * elements each (2^(L+1) for SYK_FULL: H_UU on the first half, H_DD on the second), ld >=
 * n_amps.  x and y must not overlap.  y is overwritten.
 * Errors: EINVAL (n_amps not the sector size, nvec < 1, ld < n_amps, null), EUNSUPPORTED
 * (SYK_FULL on an operator handle of syk_op_to_hamiltonian), EDEVICE. */
syk_status syk_apply_H(const syk_ham *h, syk_block blk, syk_dtype dt, const void *x, void *y,
                       uint64_t n_amps, int nvec, uint64_t ld, void *stream);

/* ---------------------------------------------------------------- Haar states
 * Random state of the typicality estimator (supplement Sec. I: a Haar-random state is
 * drawn and its parity components used).  Full-space amplitude n (n < 2^L: U block,
 * else D block, index n - 2^L) is a standard complex Gaussian from two SplitMix64
 * finaliser outputs of counters: base = mix(state_seed + (v+1) G),
 * w1 = mix(base + (2n+1) G), w2 = mix(base + (2n+2) G), G = 0x9E3779B97F4A7C15,
 * psi_n = sqrt(-2 ln u1) e^{2 pi i u2}; the vector is normalised in double over both
 * blocks.  psi_U, psi_D: device, 2^L elements each.  Errors: EINVAL, EDEVICE. */
syk_status syk_haar_state(int N, uint64_t state_seed, int v, syk_dtype dt,
                          void *psi_U, void *psi_D, void *stream);

/* The same state as syk_haar_state, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * this entry point calls no hipMalloc, hipFree or allocating library routine.  Its norm
 * partial sums (at most 2049 doubles for N <= 64) live in a fixed device array of 4096
 * doubles (32 KiB) that each device holds from library load until the process ends.
 * The call is asynchronous on `stream` (no synchronisation); the array keeps the last
 * call's partial sums, and calls that overlap on one device (other streams or threads)
 * race on it, so the caller orders them.  Same arguments and errors as syk_haar_state;
 * EINVAL also if a size needed more scratch than the array holds. */
syk_status syk_haar_state_noalloc(int N, uint64_t state_seed, int v, syk_dtype dt,
                                  void *psi_U, void *psi_D, void *stream);

/* ---------------------------------------------------------------- Majorana insertion
 * y = scale * (gamma_n)_{dst,src} x, the block of gamma_n mapping block `src` to the other
 * block (supplement Sec. I: Majoranas are block off-diagonal).  n <= N-2: the block is A_n
 * in both directions; n = N-1: gamma_{N-1}^{UD} = -i (src = D), gamma_{N-1}^{DU} = +i
 * (src = U).  scale = scale_re + i scale_im.  x, y device, 2^L elements; x == y allowed
 * only for n = N-1 or when A_n flips no qubit.  Errors: EINVAL, EDEVICE. */
syk_status syk_apply_majorana(int N, int n, syk_block src, syk_dtype dt, const void *x, void *y,
                              uint64_t n_amps, double scale_re, double scale_im, void *stream);

/* ---------------------------------------------------------------- Krylov propagator */
typedef struct {
    int m;             /* maximum Krylov dimension per sub-step, 2 <= m <= 128 */
    double tol;        /* accepted a-posteriori error per propagation, relative to ||v|| */
    int reorth;        /* 0: three-term recurrence only; 1: local (second pass against
                          v_j, v_{j-1}); 2: full, classical Gram-Schmidt twice (CGS2)
                          against every basis vector; 3: partial (Simon 1984): the loss
                          of orthogonality is estimated from the alpha/beta recurrence and
                          a full CGS2 pass runs only on the steps where the estimate
                          exceeds sqrt(eps) of the vector precision (and the step after) */
    int max_substeps;  /* 0 = unlimited */
} syk_krylov_opts;

typedef struct {
    int substeps;      /* restarts taken */
    int matvecs;       /* apply_H calls */
    int breakdown;     /* 1 if an invariant subspace ended a Lanczos run (exact) */
    double err_est;    /* sum over sub-steps of the accepted error estimates, relative */
    int reorths;       /* Lanczos steps given a full reorthogonalisation (reorth 2 and 3) */
} syk_krylov_stats;

/* Fill `o` with defaults for dtype dt (m = 30, tol = 1e-12 for C128 / 1e-7 for C64,
 * reorth = 0, max_substeps = 0).  With reorth = 0 on blocks served by the tiled kernel,
 * each Lanczos step is one fused apply (w = H v_j - beta v_{j-1} plus the alpha/beta sums)
 * and one normalising pass. */
void syk_krylov_default_opts(syk_dtype dt, syk_krylov_opts *o);

/* out = e^{z H_blk} v, z = z_re + i z_im, by Lanczos with restarts (the restarted Krylov
 * time evolution of supplement Sec. I.A, here with step control): up to m Lanczos steps
 * (alpha_j, beta_j reduced in double), the small exponential e^{tau z T_j} e_1 from the
 * eigendecomposition of the real symmetric tridiagonal T_j in double, a-posteriori error
 * estimate ||v|| beta_j |[e^{tau z T_j} e_1]_j|; a step ends early once the estimate
 * meets the tolerance for the remaining tau, else the largest tau that meets it is taken
 * and the propagation restarts from the result.  beta_j ~ 0 is an invariant subspace
 * (exact result).  v, out: device, n_amps = 2^L, 16-byte aligned; out == v allowed.
 * stats may be NULL.
 * SYK_FULL (n_amps = 2^(L+1)): the two halves are propagated separately (e^{zH} is block
 * diagonal), each to the tolerance relative to its own norm; the statistics are summed
 * (breakdown: either half).
 * Uses a library-owned device workspace of (m + 2) vectors, reused across calls.
 * Errors: EINVAL (also for a misaligned v or out), ENOMEM, EDEVICE, ENOTCONV (max_substeps
 * exceeded), ENUMERIC. */
syk_status syk_krylov_expm(const syk_ham *h, syk_block blk, syk_dtype dt, double z_re, double z_im,
                           const void *v, void *out, uint64_t n_amps, const syk_krylov_opts *o,
                           syk_krylov_stats *stats, void *stream);

/* ---------------------------------------------------------------- OTOC */
/* Called on the calling thread after each t point of each vector and block chain:
 * done = chain steps completed so far, total = nvec * 2 * nt. */
typedef void (*syk_progress_fn)(void *ctx, int done, int total);

typedef struct {
    int nvec;              /* Haar vectors averaged (>= 1) */
    uint64_t state_seed;   /* vector v uses syk_haar_state(N, state_seed, v, ...) */
    syk_dtype dtype;       /* state-vector precision; reductions are double either way */
    syk_krylov_opts krylov;
    int profile;           /* 1: time every apply_H launch with HIP events on `stream` */
    int layout;            /* -1: internal vector layout chosen by the planner (see
                              syk_plan_describe); r >= 0: bit rotation r (0 = standard order) */
    int autotune;          /* 1: before the first run of this handle/precision/device, time the
                              tiled apply_H variants and keep the fastest (syk_autotune) */
    syk_progress_fn progress;   /* optional (NULL = none) */
    void *progress_ctx;
    int precision_check;   /* 1: with complex64 states, evaluate F again at t = 0 and at the
                              last t with complex128 states on the same Haar vectors (the
                              complex128 default tolerance, the same m) and report the
                              deviation in stats.mp_err; needs the complex128 workspace
                              (syk_workspace_bytes with SYK_C128).  Ignored for SYK_C128. */
} syk_otoc_opts;

typedef struct {
    long long matvecs;
    long long substeps;
    double seconds;        /* wall time of the call */
    double max_err_est;    /* largest per-propagation relative error estimate */
    double apply_ms;       /* profile = 1: summed event-timed duration of apply_H launches */
    long long apply_launches;
    double mp_err;         /* precision_check = 1: error of the complex64 result against the
                              complex128 re-evaluation, max(|F_raw(0) - F_raw128(0)| / |F_raw128(0)|,
                              |F_norm(t_last) - F_norm128(t_last)|); -1 if not evaluated */
    double mp_seconds;     /* wall time of that re-evaluation (not part of `seconds`) */
} syk_otoc_stats;

/* Regularised OTOC of Eq. (2) with W = chi_i, V = chi_j (0-based; the paper uses
 * i = N-1, j = N-2), by the supplement's random-state estimator
 *   F_v(t) = <psi| e^{(it-b/8)H} W e^{-(it+b/4)H} V e^{(it-b/4)H} W e^{-(it+b/4)H} V e^{-bH/8} |psi>
 * evaluated as the sum of its U-block and D-block chains ("+ swap UD").  t: host, nt
 * non-decreasing times >= 0.  Outputs (host, nt doubles; any may be NULL):
 * F_raw[n] = mean_v Re F_v(t_n), F_imag[n] = mean_v Im F_v(t_n),
 * F_norm[n] = F_raw[n] / F_raw(t = 0) (t = 0 is evaluated if t[0] != 0).
 * Synchronises `stream`.  Errors: EINVAL (i == j, out of range, nt < 1, t decreasing or
 * negative, nvec < 1), ENOMEM, EDEVICE, ENOTCONV, ENUMERIC. */
syk_status syk_otoc(const syk_ham *h, int i, int j, double beta, const double *t, int nt,
                    const syk_otoc_opts *o, double *F_raw, double *F_norm, double *F_imag,
                    syk_otoc_stats *stats, void *stream);

/* Green function of the supplement (Sec. I, random-state estimator) for chi_n,
 *   G_v(t) = <psi| e^{(it-b/2)H} chi_n e^{-iHt} chi_n e^{-bH/2} |psi>,
 * evaluated as the sum of its U-block and D-block chains (l = e^{-itH_A} e^{-bH_A/2} psi_A and
 * r = e^{-itH_B} chi_n^{BA} e^{-bH_A/2} psi_A, both advanced incrementally in t; G_A = <l,
 * chi_n^{AB} r>).  chi_n = gamma_n / sqrt 2, so G(0) = <psi|e^{-bH}|psi> / 2 (1/2 at b = 0);
 * the paper's G_R(t) = Re G(t) / G(0) is G_norm.  n in [0, N); the paper uses n = N-1.
 * Options, outputs (G_raw = mean_v Re G_v, G_imag = mean_v Im G_v, G_norm = G_raw /
 * G_raw(t = 0)), synchronisation and errors as for syk_otoc. */
syk_status syk_green(const syk_ham *h, int n, double beta, const double *t, int nt, const syk_otoc_opts *o,
                     double *G_raw, double *G_norm, double *G_imag, syk_otoc_stats *stats, void *stream);

/* ---------------------------------------------------------------- batched OTOC */
/* Many small-N realisations and random vectors in one persistent launch: the OTOC of
 * syk_otoc for every item (W = chi_i, V = chi_j) at a common beta and t grid, nvec Haar
 * vectors each (vector v of item r uses syk_haar_state(N, state_seed, v)), complex64
 * states with double reductions and small exponential.  One workgroup runs one (item,
 * vector) job at a time, entirely on the device (Haar state, Majorana insertions, Lanczos
 * propagators with step control, overlaps), taking jobs from a device counter until none
 * is left.  The launch shape (threads per workgroup, LDS chunk, workgroups per CU) is
 * chosen by timing the eligible shapes on a sample of the batch unless `variant` >= 0.
 * Block sizes: 8 <= N/2 - 1 <= 15 (N from 18 to 32) for the shapes that serve them. */
typedef struct {
    int N;                 /* Majoranas (even) */
    double k;              /* sparsity, K = round(k N) */
    uint64_t seed;         /* realisation (syk_create_hamiltonian) */
    int i, j;              /* W = chi_i, V = chi_j, distinct, in [0, N) */
    uint64_t state_seed;
    int ensemble;          /* syk_ensemble of the realisation (0 = SYK_ENSEMBLE_EXACT_K) */
} syk_batch_item;

typedef struct {
    int nvec;              /* Haar vectors per item (>= 1) */
    double beta;
    int m;                 /* Krylov dimension, 2..60 */
    double tol;            /* per-propagation tolerance (> 0) */
    int variant;           /* launch shape, -1 = timed choice */
    int max_substeps;      /* per job over all its propagations, 0 = 20000 */
} syk_batch_opts;

typedef struct {
    long long matvecs;     /* over all jobs */
    int n_jobs, slots, variant;
    double kernel_ms;      /* the persistent launch, HIP events */
    double tuned_ms[3];    /* sample timings of shapes 0..2 (-1: not timed) */
    double seconds;        /* wall time of the call */
} syk_batch_stats;

/* F_raw, F_norm, F_imag: host, n_items x nt doubles (row r = item r; any may be NULL),
 * as syk_otoc's outputs of each item.  t: host, nt non-decreasing times >= 0.  Synchronises
 * `stream`.  Errors: EINVAL, EUNSUPPORTED (block size outside every shape), ENOMEM,
 * EDEVICE, ENOTCONV, ENUMERIC. */
syk_status syk_otoc_batch(const syk_batch_item *items, int n_items, const double *t, int nt,
                          const syk_batch_opts *o, double *F_raw, double *F_norm, double *F_imag,
                          syk_batch_stats *stats, void *stream);

/* ---------------------------------------------------------------- t*(N) and lambda_L */
/* Disorder average of the normalised OTOC of Eq. (2) over n_real realisations: realisation
 * r (0-based) is the Hamiltonian syk_create_hamiltonian_ensemble(N, 4, k, seed + r,
 * ensemble) with Haar vectors syk_haar_state(N, o->state_seed + r, v), v < o->nvec; its
 * curve is normalised by its own F(0) (the F_norm of syk_otoc), and the curves are then
 * averaged.  This averaged curve is the one whose crossing of F0 defines t*(N) (main text,
 * before Eq. (4)).  Path: the batched persistent launch of syk_otoc_batch (complex64
 * states; 18 <= N <= 32; m <= 60; profile = 0) or the single-request path of syk_otoc, one
 * realisation after the other, in o->dtype. */
typedef struct {
    int N;                 /* Majoranas (even) */
    double k;              /* sparsity (as syk_create_hamiltonian_ensemble) */
    int ensemble;          /* syk_ensemble */
    uint64_t seed;         /* realisation r uses seed + r */
    int n_real;            /* realisations (>= 1) */
    int i, j;              /* W = chi_i, V = chi_j (the paper: N-1, N-2) */
    double beta;
    int path;              /* -1: batched when it serves the request, 0: batched (EUNSUPPORTED
                              if it cannot), 1: single-request path */
} syk_ensemble_desc;

typedef struct {
    int path;              /* 0 batched, 1 single-request */
    long long matvecs;
    double seconds;
} syk_ensemble_stats;

/* t: host, nt non-decreasing times >= 0.  Outputs (host; any may be NULL): F_mean[n] and
 * F_sem[n] (nt doubles), the mean over realisations of the normalised curves and its
 * standard error (sample standard deviation / sqrt(n_real); 0 when n_real = 1); F_rows
 * (n_real x nt doubles, row r = realisation r), every normalised curve.  Options o as for
 * syk_otoc (nvec, state_seed, dtype, krylov; the batched path takes nvec, m, tol and
 * max_substeps from it).  Synchronises `stream`.  Errors: EINVAL, EUNSUPPORTED, ENOMEM,
 * EDEVICE, ENOTCONV, ENUMERIC. */
syk_status syk_otoc_ensemble(const syk_ensemble_desc *d, const double *t, int nt, const syk_otoc_opts *o,
                             double *F_mean, double *F_sem, double *F_rows, syk_ensemble_stats *stats,
                             void *stream);

/* Crossing time t* of a sampled curve (main text, before Eq. (4)): the first n >= 1 with
 * F[n] <= F0 < F[n-1], then linear interpolation between samples n-1 and n.  F_err (host,
 * nt, may be NULL) are standard errors of the samples; *tstar_err (may be NULL) receives
 * sigma_F(t*) / |dF/dt| with sigma_F interpolated linearly and the slope of the bracketing
 * segment (NaN without F_err).  A curve that never falls to F0 gives *tstar = NaN and
 * SYK_OK.  Host only.  Errors: EINVAL (nt < 2, t decreasing, non-finite F0). */
syk_status syk_crossing_time(const double *t, const double *F, const double *F_err, int nt, double F0,
                             double *tstar, double *tstar_err);

typedef enum {
    SYK_FIT_SLOPE = 0,     /* Eq. (5): 1/(N dt* / dN) = lambda + alpha_1/N + alpha_2/N^2 */
    SYK_FIT_GLOBAL = 1     /* Eq. (6): t* = gamma_0 + (log N/lambda)(1 + gamma_1/N + gamma_2/N^2) */
} syk_fit_method;

typedef struct {
    int method;            /* syk_fit_method */
    int terms;             /* bit 0: the 1/N term (alpha_1 or gamma_1), bit 1: the 1/N^2 term */
    int dN;                /* SYK_FIT_SLOPE: N is paired with N + dN (the supplement: 8) */
} syk_fit_opts;

typedef struct {
    double lambda, lambda_err;
    double coef[3], coef_err[3];   /* SLOPE: alpha_1, alpha_2, 0; GLOBAL: gamma_0, gamma_1,
                                      gamma_2 (terms left out: 0, error 0) */
    double chi2;           /* weighted residual sum of squares (unweighted without errors) */
    int n_points, dof;     /* points fitted (SLOPE: pairs), n_points - parameters */
} syk_fit_result;

/* Lyapunov exponent from crossing times t*(N) (host, n values each; N need not be sorted).
 * SYK_FIT_SLOPE: every pair (N_a, N_b = N_a + dN) gives the inverse slope
 * y = log(N_b/N_a) / (t*_b - t*_a) (a central difference in log N) at sqrt(N_a N_b), with
 * error |y| sqrt(s_a^2 + s_b^2) / |t*_b - t*_a| (supplement Sec. II.A); the pairs are fitted
 * by Eq. (5).  SYK_FIT_GLOBAL: t* is fitted by Eq. (6), solved as the linear problem in
 * (gamma_0, 1/lambda, gamma_1/lambda, gamma_2/lambda) with first-order error propagation.
 * With tstar_err (host, n, may be NULL) the fit is weighted by 1/sigma^2 and the errors are
 * the absolute ones, (A^T W A)^{-1}; without, it is unweighted and the covariance is scaled
 * by chi2/dof (errors NaN when dof = 0).  pts_N, pts_y, pts_err (host, cap entries, may be
 * NULL): the fitted points (SLOPE: N_mid, y, error; GLOBAL: N, t*, error).  Host only.
 * Errors: EINVAL (non-finite input, fewer points than parameters, dependent columns, equal
 * t* for a pair, cap below n_points). */
syk_status syk_lyapunov_fit(const double *N, const double *tstar, const double *tstar_err, int n,
                            const syk_fit_opts *o, syk_fit_result *out, double *pts_N, double *pts_y,
                            double *pts_err, int cap);

/* ---------------------------------------------------------------- request engine */
/* Serving engine: OTOC requests of mixed N, k and seed (one disorder realisation each,
 * the quantity of syk_otoc) taken as they arrive, with continuous batching: a request is
 * admitted as soon as a slot is free and its device footprint (Krylov basis, chain
 * vectors, term tables and plans) fits in the remaining budget, so requests arriving
 * while others run join them on the device.  Each slot is a host worker thread with its
 * own HIP stream on the device current at syk_engine_create; kernels of different
 * requests overlap on the GPU.  Admission is first-fit in arrival order: a request that
 * does not fit may be overtaken by smaller ones at most max_bypass times, after which
 * nothing else is admitted until it fits.  A request asking for more memory than the
 * budget runs with a lower Krylov dimension (down to its m_min); the dimension used is
 * reported.  Each result is computed with the same kernels and arithmetic as the same
 * request run alone through syk_otoc (autotune = 0, planner layout), so it does not depend
 * on what else is admitted.
 * The engine owns the Krylov state, tables and workspaces of admitted requests until they
 * finish or are cancelled; the caller owns the host arrays it passes (the t grid is copied
 * at submit). */
typedef struct syk_engine syk_engine;

typedef struct {
    uint64_t budget_bytes; /* device memory for admitted requests; 0 = 85% of free memory */
    int max_active;        /* requests running at once (one stream each); 0 = 4 */
    int max_bypass;        /* times a waiting request may be overtaken; < 0 = 8 */
} syk_engine_opts;

typedef struct {
    int N;                 /* Majoranas of this request's realisation */
    double k;              /* sparsity; K = round(k N) */
    uint64_t seed;         /* realisation seed (syk_create_hamiltonian) */
    int i, j;              /* W = chi_i, V = chi_j */
    double beta;
    const double *t;       /* host, nt non-decreasing times >= 0; copied at submit */
    int nt;
    int nvec;              /* Haar vectors (>= 1) */
    uint64_t state_seed;
    syk_dtype dtype;
    int m;                 /* Krylov dimension wanted (0 = 30) */
    int m_min;             /* lowest dimension accepted under memory pressure (0 = min(m, 8)) */
    double tol;            /* per-propagation tolerance (<= 0: the dtype's default) */
    int precision_check;   /* 1: report the complex64 result's error against complex128 in
                              stats.mp_err (as syk_otoc_opts.precision_check; the footprint then
                              holds the complex128 workspace) */
} syk_request;

typedef struct {
    uint64_t id;
    syk_status status;     /* SYK_OK, SYK_ECANCELLED or the error of the run */
    int nt;                /* entries written to each output array */
    int m_used;            /* Krylov dimension the request ran with */
    uint64_t footprint_bytes;
    double t_submit, t_start, t_end;   /* seconds since syk_engine_create */
    syk_otoc_stats stats;
} syk_result_info;

typedef struct {
    long long submitted, completed, failed, cancelled;
    int queued, active;
    uint64_t budget_bytes, bytes_in_use, peak_bytes;
    double p50_latency_s, p99_latency_s;   /* submit-to-finish over requests finished OK */
    double busy_seconds;                   /* time with at least one request running */
} syk_engine_stats;

/* Start the engine on the current HIP device.  Errors: EINVAL, EDEVICE, ENOMEM. */
syk_status syk_engine_create(const syk_engine_opts *o, syk_engine **out);

/* Queue one request; *id receives its identifier (> 0).  Errors: EINVAL (arguments as in
 * syk_create_hamiltonian and syk_otoc), ENOMEM (the footprint at m_min exceeds the
 * budget: it could never be admitted). */
syk_status syk_engine_submit(syk_engine *e, const syk_request *r, uint64_t *id);

/* Take one finished request, waiting up to wait_ms milliseconds (0 = do not wait, < 0 =
 * wait until one finishes or nothing is queued or running).  F_raw, F_norm, F_imag: host
 * arrays of cap doubles (any may be NULL), filled as by syk_otoc.  Returns SYK_EAGAIN if
 * none finished in time, SYK_EINVAL if cap is below the request's nt (the result is kept). */
syk_status syk_engine_poll(syk_engine *e, int wait_ms, syk_result_info *info, double *F_raw, double *F_norm,
                           double *F_imag, int cap);

/* Cancel a queued or running request; it finishes with SYK_ECANCELLED (a running one at
 * its next t point).  Errors: EINVAL (unknown or already finished id). */
syk_status syk_engine_cancel(syk_engine *e, uint64_t id);

syk_status syk_engine_get_stats(syk_engine *e, syk_engine_stats *st);

/* Cancel everything, join the workers, free all device memory; NULL is a no-op. */
syk_status syk_engine_destroy(syk_engine *e);

/* ---------------------------------------------------------------- spin operators */
/* General spin operators on L qubits as sums of Pauli strings c X^x Z^z (Z applied
 * first, qubit q = bit q; the <bits, coeff> operator lists of supplement Sec. I.A), with
 * the product, linear combination and adjoint computed exactly by the XOR-and-sign rule
 * (X^a Z^b)(X^c Z^d) = (-1)^{popcount(b & c)} X^{a^c} Z^{b^d}.  An operator converts to a
 * handle that syk_apply_H (either block argument) and, when Hermitian, syk_krylov_expm run
 * through the same kernels: other sparse models on the same path.  Terms are kept sorted
 * by (x, z) with equal strings merged (exact zeros dropped).  Host-only. */
typedef struct syk_op syk_op;

/* n terms (x[a], z[a], c_re[a] + i c_im[a]); c_re or c_im may be NULL (zero).  Errors:
 * EINVAL (L outside [1, 31], a string beyond qubit L-1, non-finite coefficient). */
syk_status syk_op_create(int L, size_t n, const uint64_t *x, const uint64_t *z, const double *c_re,
                         const double *c_im, syk_op **out);
syk_status syk_op_destroy(syk_op *o);                                       /* NULL is a no-op */
syk_status syk_op_product(const syk_op *a, const syk_op *b, syk_op **out);   /* a b */
/* alpha a + beta b */
syk_status syk_op_sum(const syk_op *a, const syk_op *b, double alpha_re, double alpha_im, double beta_re,
                      double beta_im, syk_op **out);
syk_status syk_op_adjoint(const syk_op *a, syk_op **out);                    /* a^dagger */
/* *n = number of terms; arrays (host, cap entries, any may be NULL) receive them. */
syk_status syk_op_get_terms(const syk_op *a, size_t cap, size_t *n, uint64_t *x, uint64_t *z, double *c_re,
                            double *c_im);
syk_status syk_op_is_hermitian(const syk_op *a, int *out);
/* A handle for syk_apply_H (N reported as 2 (L + 1), block dimension 2^L; both blocks hold
 * the operator) and, for Hermitian operators, syk_krylov_expm; syk_otoc and syk_green
 * refuse it (EUNSUPPORTED).  Errors: EINVAL (L < 2, no terms). */
syk_status syk_op_to_hamiltonian(const syk_op *a, syk_ham **out);

/* ---------------------------------------------------------------- helpers */

/* Device bytes the OTOC of one request needs (Krylov basis, chain vectors, scratch);
 * the supplement's minimum is (v+3) vectors for a Krylov dimension v.  Errors: EINVAL. */
syk_status syk_workspace_bytes(int N, int m, syk_dtype dt, int nvec, uint64_t *bytes);

/* Host-only small exponential used by syk_krylov_expm: c = e^{z T} e_1 for the real
 * symmetric tridiagonal T (diagonal alpha[0..n-1], off-diagonal beta[0..n-2]);
 * c_re, c_im: host, n doubles.  Errors: EINVAL (n < 1 or > 1024, null), ENUMERIC. */
syk_status syk_tridiag_expm(int n, const double *alpha, const double *beta, double z_re, double z_im,
                            double *c_re, double *c_im);

/* Launch plan of the tiled apply_H kernel for one block (host-only; no GPU needed).
 * Blocks of 2^L amplitudes with L >= 18 are served by the tiled kernel: output tiles of
 * 2^tile_bits amplitudes, terms grouped by partner tile (n_groups groups), tiles mapped
 * to workgroups so that the 2^res_bits tiles resident on one XCD form a coset of a
 * res_bits-dim subspace (classes_xcd = partner-tile classes modulo it, which sets the L2
 * misses) and those on the whole GPU one of a (res_bits + 3)-dim subspace (classes_gpu).
 * A workgroup holds tiles_per_wg tiles (a coset of a small subspace chosen so that their
 * partner tiles coincide as much as possible) and streams n_partners partner tiles.
 * rot is the vector layout: index bit b holds qubit (b + rot) mod L.  layout = -1 asks
 * for the planner's choice (the layout syk_otoc uses by default), layout >= 0 for that
 * rotation. */
typedef struct {
    int tiled;             /* 0: the block is served by the gather kernel; then n_groups is the
                              number of distinct x masks, each gathered once per amplitude
                              (about K / 19 for dense SYK, about K for sparse) */
    int variant;           /* compiled kernel variant in use (default or tuned) */
    int tile_bits, rot, n_groups, classes_xcd, classes_gpu, res_bits;
    int tiles_per_wg;      /* output tiles a workgroup keeps in registers */
    int n_partners;        /* partner tiles a workgroup streams (n_groups when tiles_per_wg = 1) */
    uint64_t n_tiles;
} syk_plan_desc;
syk_status syk_plan_describe(const syk_ham *h, syk_block blk, syk_dtype dt, int layout, syk_plan_desc *out);

/* Control blocks of that plan (host-only; for inspection and tests), when the variant in use
 * has record form 2: one 64-word block per partner step plus one for the last prefetch.  In
 * a block, lanes 4j .. 4j+3 (complex64; 5j .. 5j+4 for complex128) hold record j: the thread
 * bits of x | (x register bits) << 24, the thread bits of z | (register sign mask) << 24,
 * z >> tile_bits, and the coefficient (float, or the two words of a double).  Records come
 * tile by tile, real-phase before i-phase.  Lane 60 counts them (tile i: real in bits
 * 8i..8i+3, i-phase in 8i+4..8i+7).  Lane 62 counts, in the same layout, the records at the
 * head of each run that touch no register bit (register bits of x and z zero).  Lane 61 is
 * the partner offset copied during the step.  Masks are in the plan's layout (rotation rot
 * of syk_plan_describe).  out: host, cap words (NULL to query the size); *n_words receives the
 * number of words.  Errors: EINVAL, EUNSUPPORTED (block not tiled, or the variant in use has
 * no control blocks). */
syk_status syk_plan_blocks(const syk_ham *h, syk_block blk, syk_dtype dt, int layout, uint32_t *out, size_t cap,
                           size_t *n_words);

/* Schedule autotuner: time each compiled variant of the tiled apply_H kernel (tile size,
 * LDS buffering, prefetch depth; each in its planned layout) on this Hamiltonian and keep
 * the fastest for the current device and precision.  *variant receives the choice (-1 if
 * the block is not tiled); ms[v] (host, cap entries, may be NULL) the mean time of one
 * apply with variant v (-1 where skipped).  Uses a library-owned workspace of two vectors.
 * Errors: EINVAL, ENOMEM, EDEVICE. */
syk_status syk_autotune(const syk_ham *h, syk_dtype dt, int *variant, float *ms, int cap, void *stream);

/* Pin the tiled apply_H variant (0 <= variant < the number of entries syk_autotune
 * reports) for this handle, precision and the current device, in place of the default or
 * tuned one: for tests of every variant and for reproducible timings.  Host-only (without
 * a device it applies to device 0, e.g. for syk_plan_describe).  Errors: EINVAL. */
syk_status syk_select_variant(const syk_ham *h, syk_dtype dt, int variant);

/* Release the library's cached device workspaces on the current device. */
syk_status syk_release_workspace(void);

/* Identifier of the apply_H kernel revision built into this library (changes whenever the
 * kernel's memory behaviour may change; hardware-counter figures are tied to it). */
const char *syk_kernel_revision(void);

const char *syk_status_string(syk_status s);
const char *syk_last_error(void);    /* thread-local; "" if none */

#ifdef __cplusplus
}
#endif
#endif /* SYK_H */
