/*
 * scfft -- FFT fixed-point solvers for periodic two-phase conducting
 * composites on AMD Instinct MI355X (gfx950).
 *
 * The solvers follow G. W. Milton, "Substitution of subspace collections with
 * nonorthogonal subspaces to accelerate Fast Fourier Transform methods
 * applied to conducting composites":
 *
 *   SCFFT_MS      the basic Moulinec-Suquet scheme, series eq. J0-0,
 *                 reference conductivity sigma0 = (sigma1 + 1)/2 (eq. J1);
 *   SCFFT_EM      the Eyre-Milton scheme, expansion eq. J2,
 *                 sigma0 = sqrt(sigma1);
 *   SCFFT_ACC_EM  the paper's accelerated scheme: Eyre-Milton run in the
 *                 substituted Hilbert space H'' (eqs. J27-J45, expansion
 *                 eq. J43) with p set from the singularity interval
 *                 [-beta, -alpha] by eq. J24 and t(sigma1) by eq. J23;
 *   SCFFT_ACC_MS  Moulinec-Suquet run in H'' (expansion eq. J42a).
 *
 * The problem (eqs. J12-J13): on an N^d periodic voxel grid (d = 2, 3) with
 * phase map chi (1 = inclusion of conductivity sigma1, 0 = matrix of
 * conductivity sigma2 = 1) find E with <E> = e0, E - e0 curl free and
 * J = sigma E divergence free; sigma* is reported as <J>.e0/|e0|^2
 * (bilinear dot, real e0; a scalar for square/cubic symmetry, eq. J13).
 * Gamma_1 = k k^T/|k|^2 (eq. J11) is evaluated with a discrete wavevector
 * per DFT mode (SCFFT_GAMMA_*).
 *
 * Conventions for every entry point:
 *   - grids: axis 0 (x) varies fastest; voxel (x, y, z) is at
 *     x + n[0]*(y + n[1]*z); vector fields are component-major [d][N^d];
 *     the periodic cell is the unit square (cube), so a voxel is 1/n[i]
 *     wide along axis i; every n[i] must factor into 2, 3 and 5 and lie in
 *     [2, 4096], and the last axis must fit one workgroup's transform of all
 *     d components: d * n[d-1] <= 8192 in fp32 (3D: n[2] <= 2730) and
 *     <= 4096 in fp64 (2D: n[1] <= 2048; 3D: n[2] <= 1365); larger grids
 *     return SCFFT_ERR_INVALID_ARG;
 *   - every pointer documented "device" is a device address on the current
 *     HIP device, owned by the caller, and must stay valid until the call
 *     returns; "host" pointers likewise; the library never frees them;
 *   - the library owns only internal workspaces (state fields, reductions),
 *     which it caches between calls and frees in scfft_release();
 *   - all work is enqueued on options->stream (a hipStream_t, NULL = the
 *     default stream) and the calls return after synchronising that stream;
 *     calls from several host threads must use distinct streams and are
 *     otherwise not re-entrant (the workspace cache is shared);
 *   - a negative return value is an error (scfft_status); outputs are filled
 *     on SCFFT_OK, SCFFT_ERR_NOT_CONVERGED, SCFFT_ERR_DIVERGED and
 *     SCFFT_ERR_STAGNATED (with the last iterate).
 */
#ifndef SCFFT_H
#define SCFFT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { double re, im; } scfft_c64;

typedef enum {
  SCFFT_MS = 0,
  SCFFT_EM = 1,
  SCFFT_ACC_EM = 2,
  SCFFT_ACC_MS = 3
} scfft_scheme;

typedef enum {
  SCFFT_FP64 = 0, /* fp64 complex fields and FFTs */
  SCFFT_FP32 = 1  /* fp32 complex fields and FFTs; reductions, residual and
                     scheme scalars stay fp64 */
} scfft_precision;

/* Discrete reading of Gamma_1 (eq. J11), theta_j = 2 pi m_j / n_j, on the
 * unit cell (difference quotients carry 1/h_j = n_j):
 *  ROTATED  n_j = n_j sin(theta_j/2) prod_{l != j} cos(theta_l/2), the
 *           difference across a voxel averaged over the other axes; modes
 *           with n = 0 but m != 0 use n_j = n_j [m_j == n_j/2];
 *  SPECTRAL the literal wavevector (over 2 pi), m_j in (-n_j/2, n_j/2];
 *           Nyquist components are zeroed at modes that also have a
 *           non-zero non-Nyquist component;
 *  NETWORK  n_j = n_j (exp(i theta_j) - 1), the forward difference of the
 *           resistor network of section 2, used as n n^H/|n|^2.          */
typedef enum {
  SCFFT_GAMMA_ROTATED = 0,
  SCFFT_GAMMA_SPECTRAL = 1,
  SCFFT_GAMMA_NETWORK = 2
} scfft_symbol;

typedef enum {
  SCFFT_OK = 0,
  SCFFT_ERR_INVALID_ARG = -1,   /* bad size, pointer, scheme, interval ... */
  SCFFT_ERR_SLIT = -2,          /* sigma1 where the scheme's expansion has no
                                   meaning: on [-beta,-alpha] (H'' schemes),
                                   on (-inf, 0] (SCFFT_EM) */
  SCFFT_ERR_NOT_CONVERGED = -3, /* max_iter reached */
  SCFFT_ERR_DIVERGED = -4,      /* non-finite values, or the residual grew past
                                   div_factor times its running minimum */
  SCFFT_ERR_STAGNATED = -5,     /* no new residual minimum for stag_window
                                   consecutive iterations */
  SCFFT_ERR_DEVICE = -6,        /* a HIP call failed */
  SCFFT_ERR_OOM = -7            /* workspace allocation failed */
} scfft_status;

/* One solve's input. */
typedef struct {
  int d;                  /* 2 or 3 */
  int n[3];               /* grid; n[2] ignored when d = 2 */
  const uint8_t* phase;   /* device, N^d bytes: 1 = phase 1, 0 = matrix; used
                             when density is NULL */
  const double* density;  /* device, N^d doubles in [0, 1] or NULL: a graded
                             medium sigma(x) = 1 + (sigma1 - 1) rho(x); only
                             SCFFT_MS and SCFFT_EM accept it */
  scfft_c64 sigma1;       /* inclusion conductivity (sigma2 = 1) */
  double e0[3];           /* applied average field, real, not all zero */
} scfft_problem;

typedef struct {
  int scheme;             /* scfft_scheme */
  int precision;          /* scfft_precision */
  int symbol;             /* scfft_symbol */
  double alpha, beta;     /* H'' schemes: 0 < alpha < beta < inf */
  int sigma0_set;         /* MS/EM: 1 = use sigma0 below instead of the default */
  scfft_c64 sigma0;       /* reference conductivity override */
  double tol;             /* stop at the first n >= 1 with r_n <= tol, where
                             r_n = ||E^n - E^{n-1}|| / ||E^n|| over the physical
                             field; tol < 0 runs exactly max_iter iterations */
  int max_iter;           /* >= 0 */
  int check_every;        /* host reads the device status every this many
                             iterations (>= 1); does not change the result */
  int stag_window;        /* 0 disables the stagnation stop */
  double div_factor;      /* 0 disables the divergence-by-growth stop */
  void* stream;           /* hipStream_t or NULL */
} scfft_options;

/* Fills *o with the defaults: ACC_EM, FP64, ROTATED, [alpha,beta] = [1/4,4],
 * tol 1e-8, max_iter 1000, check_every 16, stag_window 20, div_factor 1e3. */
void scfft_default_options(scfft_options* o);

typedef struct {
  scfft_c64* E;           /* device [d][N^d] or NULL: physical field E^n (the
                             Q-slot of E'' for the H'' schemes) */
  scfft_c64* J;           /* device [d][N^d] or NULL: sigma(x) E^n */
  scfft_c64 sigma_star;   /* <sigma E^n>.e0/|e0|^2 */
  scfft_c64 mean_J[3];    /* <sigma E^n> */
  int iterations;         /* n of the returned iterate */
  double residual;        /* r_n (NaN when n = 0) */
  int status;             /* same as the return value */
  double* residual_history;   /* host, history_cap entries, or NULL: r_0..r_n */
  scfft_c64* sigma_history;   /* host, history_cap entries, or NULL */
  int history_cap;
  double elapsed_ms;      /* device time of the iteration loop (HIP events) */
} scfft_result;

/* Solve one problem (eqs. J12-J13) with one scheme.  A solve with
 * max_iter = m runs m + 1 passes (iterates 0..m).  The passes run as
 * replays of HIP graphs of 2^b iterations (b up to log2 min(check_every,
 * 64)), captured on opt->stream (on an internal non-blocking stream when it
 * is NULL, ordered after the caller's earlier work) and built, with the
 * plan, on the first solve of a configuration; SCFFT_NO_GRAPH launches the
 * same kernels one by one.  Plans, graphs and workspaces are cached until
 * scfft_release. */
scfft_status scfft_solve(const scfft_problem* prob, const scfft_options* opt,
                         scfft_result* res);

/* Workspace of scfft_solve_noalloc per GPU, in bytes (160 MiB). */
#define SCFFT_NOALLOC_BYTES (160u * 1024u * 1024u)

/* scfft_solve for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, semantics and results as scfft_solve, but the call
 * allocates and frees no device memory: its workspace (iterate, previous
 * field, H'' slots, partial sums, control block, max_iter + 1 history
 * entries, twiddle and symbol tables) lives in one fixed device array of
 * SCFFT_NOALLOC_BYTES inside the library, one per GPU, held from the
 * library's load until the process ends.  A problem whose workspace does
 * not fit returns SCFFT_ERR_INVALID_ARG before any device work (2048^2 fp32
 * with the accelerated scheme fits; 2048^2 fp64 and 256^3 do not).  Kernels
 * are launched one by one on opt->stream (no graph replay).  Every call on
 * one GPU uses that GPU's array and re-initialises what it reads; calls that
 * overlap on one GPU (several host threads or streams) race, and the caller
 * must serialise them.  The first call on a device also creates the two
 * HIP events that time its loop. */
scfft_status scfft_solve_noalloc(const scfft_problem* prob, const scfft_options* opt,
                                 scfft_result* res);

/* Batched sweep: nprob microstructures (grids may differ) times nsig
 * conductivities each.  sigma1s (host) holds nprob*nsig values, problem-major;
 * opts (host) holds one options struct per problem (alpha, beta may differ;
 * precision, symbol, tolerances and the stream are taken from opts[0]);
 * results (host) receives nprob*nsig entries, problem-major (their E/J
 * pointers, if set, must each hold one field).  Every solve keeps its own
 * stop status; finished solves are skipped by the remaining iterations.
 * The problems' iteration chains run as up to 4 parallel branches of one
 * replayed HIP graph (largest first onto the least loaded branch;
 * SCFFT_BRANCHES=1..4 caps the count).  prob[i].sigma1 is ignored.  Returns
 * the worst status. */
scfft_status scfft_solve_batch(int nprob, const scfft_problem* probs,
                               const scfft_options* opts, int nsig,
                               const scfft_c64* sigma1s, scfft_result* results);

/* Power-iteration estimate of the singularity interval: the spectrum of
 * Gamma_1 chi Gamma_1 on curl-free fields lies in [mu_min, mu_max], and
 * sigma*(sigma1) is singular at sigma1 = 1 - 1/mu, hence alpha = 1/mu_max - 1
 * and beta = 1/mu_min - 1 (section "Estimating the parameters alpha and
 * beta").  u_0 = e0, u_k = Gamma_1(w u_{k-1}) for k = 1..iters+1 with w = chi
 * (then w = 1 - chi), Rayleigh quotient (u, w u)/(u, u) at the last u.  fp64.
 * Outputs are host pointers (any may be NULL). */
scfft_status scfft_estimate_interval(const scfft_problem* prob, int iters,
                                     int symbol, void* stream, double* alpha,
                                     double* beta, double* mu_min,
                                     double* mu_max);

/* Lanczos process for the spectral measure behind the singularities of
 * sigma*(sigma1) (section "Estimating the parameters alpha and beta": the
 * singularities sit at sigma1 = 1 - 1/mu, mu in the support of the measure
 * of A = Gamma_1 chi Gamma_1 on E with respect to v_0 = Gamma_1 chi e0).
 * fp64 on the device with full reorthogonalisation:
 *   q_0 = v_0/|v_0|,  r = A q_j minus its components along q_0..q_j
 *   (classical Gram-Schmidt, twice), a_j = the component removed along q_j,
 *   b_{j+1} = |r|, q_{j+1} = r/b_{j+1};
 * one x pass and one Gamma pass per step; the steps + 1 basis vectors are
 * held in a device buffer allocated for the call.  prob->phase and prob->e0
 * (non-zero) are used; 1 <= steps <= 200.  a (host, steps entries) receives
 * a_0..a_{m-1}, b (host, steps entries) receives b_1..b_{m-1} in
 * b[0..m-2] and b_m, the norm of the last residual (0 when the space
 * closed), in b[m-1]; norm0 = |v_0|^2 (sum over voxels); m = number of
 * steps completed (fewer than steps when b_{j+1} < 1e-12 max(1, |a_j|), i.e.
 * the Krylov space closed).  The Gauss rule of the tridiagonal matrix
 * (a_0..a_{m-1}, b_1..b_{m-1}) gives the nodes mu_i and weights
 * norm0 * (first eigenvector component)^2; node i lies within
 * b_m |last eigenvector component| of an eigenvalue of A.
 * SCFFT_ERR_INVALID_ARG when v_0 = 0 (e0 sees no inhomogeneity). */
scfft_status scfft_lanczos(const scfft_problem* prob, int steps, int symbol,
                           void* stream, double* a, double* b, double* norm0,
                           int* m);

/* Interval [alpha, beta] from the Lanczos Gauss rule (host Jacobi
 * eigen-decomposition of the tridiagonal matrix): mu_min / mu_max are the
 * extreme nodes whose weight exceeds rel_weight times the total (1e-20
 * separates the measure from rounding: with full reorthogonalisation,
 * nodes the measure does not support carry weights of order 1e-32),
 * alpha = 1/mu_max - 1, beta = 1/mu_min - 1, and the interval for the
 * accelerated scheme follows the floating-point stability rule
 * alpha_used = min(alpha, 1/beta), beta_used = 1/alpha_used (every output
 * pointer may be NULL).  SCFFT_ERR_INVALID_ARG when no node lies inside
 * (0, 1). */
scfft_status scfft_estimate_interval_lanczos(const scfft_problem* prob, int steps,
                                             int symbol, void* stream,
                                             double rel_weight, double* alpha,
                                             double* beta, double* alpha_used,
                                             double* beta_used, double* mu_min,
                                             double* mu_max);

/* Gradient of sigma* by an adjoint solve.  Forward: SCFFT_EM (sigma0 =
 * sqrt(sigma_min sigma_max) over the medium unless opt->sigma0_set).
 * Adjoint: the transposed Eyre-Milton iteration m <- Z W m + c with
 * W = I - 2 Gamma_1, Z = (sigma - sigma0)/(sigma + sigma0),
 * c = sigma/(sigma + sigma0) e0, iterated on y = W m with the same kernels;
 * then d sigma* / d sigma(x) = 2 sigma0/(sigma + sigma0)^2 (y.P + P.e0/2) /
 * (N^d |e0|^2), P = (sigma + sigma0) E.
 * Writes (each optional): g (device, N^d) = d sigma* / d sigma(x);
 * drho (device, N^d) = (sigma1 - 1) g = d sigma* / d rho(x);
 * dsigma1 (host) = sum_x g(x) rho(x) (rho = chi for a phase map).
 * fwd/adj (host, optional) receive the two solves' reports. */
scfft_status scfft_gradient(const scfft_problem* prob, const scfft_options* opt,
                            scfft_c64* g, scfft_c64* drho, scfft_c64* dsigma1,
                            scfft_result* fwd, scfft_result* adj);

/* Full effective tensor (the anisotropic generalisation noted after
 * eq. J13): d solves of the same problem with e0 = e_1 .. e_d, run together
 * as one batch (prob->e0 is ignored).  tensor (host, d*d, row-major) receives
 * sigma*_{ij} = <J_i> for e0 = e_j; iterations (host, d entries) may be NULL.
 * Returns the worst status of the d solves. */
scfft_status scfft_effective_tensor(const scfft_problem* prob, const scfft_options* opt,
                                    scfft_c64* tensor, int* iterations);

/* Execution choices for a problem and options: the plan scfft_solve uses.
 * Unless SCFFT_TUNE=0, the first plan of a configuration (grid, precision,
 * scheme's local map, symbol, field mode) is chosen by the autotuner, which
 * times every candidate of each pass on the real kernels with the solve's
 * own coefficients (per layout: kx = 0 / n0/2 packing, padded row pitch,
 * nontemporal x-pass streams; per pass: register radix and tile width) and
 * keeps the fastest; the choice is kept for the process, and appended to the
 * file SCFFT_TUNE_CACHE names (keyed by GPU architecture), which later
 * processes read.  info (host, cap >= 10 entries) receives: [0] real-field
 * mode, [1] kx = 0 and n0/2 packed in one column (2D), [2] rows padded to
 * 128-byte lines, [3] nontemporal x-pass streams, [4] x-pass register radix
 * (0: LDS-staged mixed radix), [5] Gamma-pass register radix (0: mixed
 * radix), [6] Gamma-pass tile width, [7] 3D y-pass tile width (0 in 2D),
 * [8] 1 if the autotuner chose, 0 for the built-in rules, [9] rows per
 * x-pass workgroup; with cap >= 13 also the FFT engine of [10] the x pass,
 * [11] the Gamma pass and [12] the 3D y passes (0 in 2D): 1
 * register-resident power-of-two passes, 2 compile-time mixed-radix passes
 * (of the lengths the library instantiates, 48 ... 960: x passes and
 * strided passes, full-complex or real-field), 0 runtime-planned mixed
 * radix.
 * Environment overrides (SCFFT_XR, SCFFT_GR, SCFFT_LINE_C, SCFFT_YC,
 * SCFFT_PACK, SCFFT_PITCH, SCFFT_NT, SCFFT_R16=0, SCFFT_NO_SMOOTH) force
 * single choices over both. */
scfft_status scfft_plan_info(const scfft_problem* prob, const scfft_options* opt, int* info,
                             int cap);

/* Average device duration (ms, HIP events on opt->stream) of each kernel of
 * one iteration over `iters` iterations of the given solve configuration:
 * ms[0] real-space x pass, ms[1] Gamma pass (last axis), ms[2] forward y pass
 * (3D), ms[3] inverse y pass (3D), ms[4] status/reduction finalize.  The
 * passes run the real iteration (status checks disabled).  cap >= 5. */
scfft_status scfft_profile_passes(const scfft_problem* prob,
                                  const scfft_options* opt, int iters,
                                  double* ms, int cap);

/* Coefficients of the expansion of eqs. J5 / J7,
 *   sigma* / sqrt(t) = sum_{n >= 0} c_n z^n,  t of eq. J6,  z = (sqrt t - 1)/(sqrt t + 1),
 * for a two-phase map (prob->phase required, prob->density must be NULL;
 * prob->sigma1 is ignored: the c_n depend on the geometry, e0 and the
 * interval only).  In H'' the Eyre-Milton operator is z K with
 * K = 2 p p^T - I at phase-1 voxels and -1 on Q elsewhere (p of eq. J24), so
 * the fixed point expands in u_0 = (e0, 0, 0), u_k = W'' K u_{k-1} (W'' of
 * eq. J44) and c_0 = 1, c_k = 2 <(K u_{k-1})_Q> . e0 / |e0|^2: the accelerated
 * iteration's kernels run nterms times with z = 1 and no source term.
 * Uses opt->alpha, opt->beta (0 < alpha < beta), opt->precision,
 * opt->symbol, opt->stream; the stop rules are off.  coeffs (host) receives
 * c_0 .. c_nterms (nterms + 1 entries), 1 <= nterms <= 100000.
 * Rounding excites the zero-weight modes whose singularities (sigma1 = 0
 * and infinity) map to |z| = min(|z(t(0))|, |z(t(inf))|) < 1, so the
 * coefficients carry noise growing like that radius^-n: sums and Pade
 * approximants are reliable where |z| stays below it. */
scfft_status scfft_series_coefficients(const scfft_problem* prob,
                                       const scfft_options* opt, int nterms,
                                       scfft_c64* coeffs);

/* sigma*(sigma1) from the coefficients of scfft_series_coefficients, for
 * nsig values sigma1s (host arrays; out receives nsig values):
 * pade_m = 0: the partial sum sqrt(t) sum_{n <= nterms} c_n z^n;
 * pade_m > 0: sqrt(t) a(z)/q(z), the [L/M] Pade approximant with
 * M = pade_m, L = nterms - M (q_0 = 1; q solves the M linear conditions
 * sum_{j <= M} q_j c_{L+i-j} = 0, i = 1..M, by LU with partial pivoting).
 * Host fp64 only.  SCFFT_ERR_SLIT if a sigma1 lies on [-beta, -alpha];
 * SCFFT_ERR_INVALID_ARG for a singular Pade system or bad sizes. */
scfft_status scfft_series_evaluate(int nterms, const scfft_c64* coeffs,
                                   double alpha, double beta, int pade_m,
                                   int nsig, const scfft_c64* sigma1s,
                                   scfft_c64* out);

/* Scheme scalars (host fp64, no device use): out[] receives, as complex
 * numbers, sigma0, t (eq. J23; 0 for MS/EM), z (the expansion variable of
 * eqs. J1, J2, J42a or J4), p1, p2, p3 (eq. J24; 0 for MS/EM), E2' (eq. J21),
 * J3' (eq. J26): 8 entries. */
scfft_status scfft_scheme_scalars(int scheme, scfft_c64 sigma1, double alpha,
                                  double beta, scfft_c64* out);

/* sigma1 whose accelerated-scheme variable z (eq. J4) has the given value:
 * the inverse of the slit map t of eq. J3 at t = ((1+z)/(1-z))^2. */
scfft_c64 scfft_sigma1_from_z(double alpha, double beta, scfft_c64 z);

/* Static description of a status code. */
const char* scfft_status_string(int status);

/* Frees every cached workspace on every device. */
void scfft_release(void);

/* Library version string. */
const char* scfft_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SCFFT_H */
