/*
 * iwfpm.h - C ABI of the irrational-window-filter projection method (IWFPM)
 * Hamiltonian apply and block eigensolver for AMD gfx950 (MI355X).
 *
 * The operator (paper, Sec. 4.1): for the quasiperiodic Schroedinger problem
 *     H u = -1/2 Laplace u + v u = E u,
 * discretised on the irrational window W_{K,L} (Sec. 3.1, eq:non-tensor) and
 * moved onto the lifted grid K*_{K,L} by the index-shift map (Sec. 3.2,
 * eq:index mod, eq:inverse1-eq:inverse3), the matrix is
 *     H~ = Lambda + F V F^{-1},   F = T F*   (Sec. 3.3, eq:F),
 * with Lambda = 1/2 |2 pi P k|^2 on the true labels k = rho^{-1}(k*) and V the
 * parent potential sampled on the dual grid G_{K,L} (eq:G_KL).  F* is the
 * standard n-D DFT with the 1/N factor of the discrete inner product
 * eq:new_inner_product.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - P is d x n, row-major, float64, in the convention where the kinetic
 *    energy of mode k is 1/2 |2 pi P k|^2.  (The paper's examples carry the
 *    factor 2 pi inside P; divide it out.)  Columns 1..d form P_I, which must
 *    be invertible (Sec. 3.1); Q = P_I^{-1} P_II.
 *  - K has d entries, L has n-d entries, all >= 1 (Remark after Fig. 1).
 *  - Grid extents ext = (2L_1..2L_{n-d}, 2K_1..2K_d); N = prod(ext) is the
 *    number of degrees of freedom (Sec. 4.2, DOF).
 *  - Vectors are complex float64, interleaved (re, im), N entries each; a
 *    block of nvec vectors is column-major (vector j starts at j*N).
 *  - GRID order: entry i is the coefficient of k* where i is the row-major
 *    index of an array of shape ext, i.e. the k_II axes are slow and the k_I
 *    axes fast (k_d fastest).  WINDOW order: the same, except that along each
 *    k_I axis the entries run over the true labels k_j ascending from the
 *    slice's lower end -K_j - floor((Q k_II)_j), instead of over k*_j.
 *  - The potential is given by its parent-function Fourier modes
 *    (Sec. 4.1: V(y) = sum_m Vhat_m e^{i m.y}): n_modes integer n-vectors m
 *    (paper order: m_1..m_n) and complex coefficients Vhat (re, im pairs).
 *    V must be real: every m needs -m with the conjugate coefficient.
 *  - Every function returns an iwfpm_status.  Arguments are checked before any
 *    device work; on error nothing has been enqueued.  No function throws or
 *    aborts across the ABI.
 *  - Streams are hipStream_t passed as void*; NULL is the default stream.
 *  - The caller owns every vector buffer and the stream; the plan owns its
 *    tables and device workspace until iwfpm_destroy.  A plan is not
 *    re-entrant: calls on one plan must not overlap.
 */
#ifndef IWFPM_H
#define IWFPM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct iwfpm_plan_s* iwfpm_plan_t;
typedef struct iwfpm_batch_s* iwfpm_batch_t;

typedef enum {
    IWFPM_OK = 0,
    IWFPM_ERR_ARG = -1,            /* bad argument (sizes, NULL pointers, ranges) */
    IWFPM_ERR_SINGULAR_PI = -2,    /* P_I not invertible, or P has rank < d (Def. 2.1) */
    IWFPM_ERR_NONHERMITIAN = -3,   /* potential modes do not describe a real V */
    IWFPM_ERR_UNSUPPORTED = -4,    /* valid input outside what this library implements */
    IWFPM_ERR_ALLOC = -5,          /* device or host allocation failed */
    IWFPM_ERR_DEVICE = -6,         /* a HIP call failed */
    IWFPM_ERR_NUMERIC = -7,        /* NaN/Inf or a breakdown the solver could not recover */
    IWFPM_ERR_NOCONV = -8,         /* maxit reached; partial results are returned */
    IWFPM_ERR_WEIGHTS = -9,        /* learned preconditioner weights missing or invalid */
    IWFPM_ERR_NODEVICE = -10,      /* the plan was created host-only (device = -1) */
    IWFPM_ERR_TOO_LARGE = -11      /* input beyond iwfpm_apply_noalloc's static scratch */
} iwfpm_status;

enum { IWFPM_PREC_FP64 = 0, IWFPM_PREC_FP32 = 1 };
/* How the sheared offset q = Q k_II enters the window:
 * EXACT    k_I + q in [-K, K)               (Sec. 3.1, the method as defined)
 * ROUNDED  k_I + floor(q + 1/2) in [-K, K)  (the reading that reproduces Table 1's cond(H))
 * PM       k_I in [-K, K)                   (shear off: the projection method's rectangle) */
enum { IWFPM_WINDOW_EXACT = 0, IWFPM_WINDOW_ROUNDED = 1, IWFPM_WINDOW_PM = 2 };
enum { IWFPM_ORDER_GRID = 0, IWFPM_ORDER_WINDOW = 1 };
enum { IWFPM_SCHED_AUTO = 0, IWFPM_SCHED_FUSED = 1, IWFPM_SCHED_THREEPASS = 2 };
enum { IWFPM_PRECOND_NONE = 0, IWFPM_PRECOND_PLAIN = 1, IWFPM_PRECOND_LEARNED = 2 };

typedef struct {
    int precision;       /* IWFPM_PREC_*: arithmetic of the potential convolution.
                            FP32 keeps the kinetic term, the boundary vectors and
                            everything in the eigensolver in float64. */
    int window_variant;  /* IWFPM_WINDOW_* */
    int order;           /* IWFPM_ORDER_* */
    int device;          /* HIP device ordinal; -1 = host-only plan (geometry queries only) */
    int schedule;        /* IWFPM_SCHED_*; AUTO picks FUSED when the grid fits one workgroup */
    int split;           /* THREEPASS: number of leading grid axes in the middle pass; 0 = auto */
    int tile;            /* THREEPASS: middle-pass tile width (columns); 0 = auto */
} iwfpm_opts;

/* Fill *opts with the defaults: FP64, EXACT, GRID, device 0, AUTO, 0, 0. */
void iwfpm_default_opts(iwfpm_opts* opts);

/* Human-readable name of a status code (static storage). */
const char* iwfpm_status_string(int status);

/*
 * iwfpm_plan - Alg. 1 steps 1-2 set-up: builds K_{K,L}, K*_{K,L} and the
 * per-slice offsets of rho^{-1} (eq:inverse1-3), the kinetic tables, the
 * potential on G_{K,L} (eq:G_KL) and the FFT schedule, and uploads them to
 * the device.  The schedule is one fused kernel for grids that fit one
 * workgroup, else three passes (trailing axes, leading axes with the
 * potential, trailing axes with the kinetic term), else, when the leading
 * block fits no workgroup either (e.g. 40^3 x 10^3), five: a further pass
 * transforms the axes between the two groups before and after the middle
 * one.  Host inputs (P, K, L, modes, vhat) are copied; the caller may free
 * them on return.  opts may be NULL (defaults).  Blocking.
 * Errors: ERR_ARG (d < 1, n <= d, n > 8, K/L < 1, non-finite P or vhat),
 * ERR_UNSUPPORTED (a grid extent 2K_j or 2L_j the library has no transform
 * for, or more than 2^31 - 1 grid points), ERR_SINGULAR_PI, ERR_NONHERMITIAN,
 * ERR_DEVICE / ERR_ALLOC.
 */
int iwfpm_plan(int d, int n, const double* P, const int32_t* K, const int32_t* L,
               int n_modes, const int32_t* modes, const double* vhat,
               const iwfpm_opts* opts, iwfpm_plan_t* out);

/* Release the plan and its device memory (synchronises its device first). */
int iwfpm_destroy(iwfpm_plan_t plan);

/* Number of degrees of freedom N = (2K)^d (2L)^{n-d} (Sec. 4.2). */
int iwfpm_dof(iwfpm_plan_t plan, int64_t* N);

/* Grid extents in storage-axis order (2L_1..2L_{n-d}, 2K_1..2K_d); ext has n entries. */
int iwfpm_grid_shape(iwfpm_plan_t plan, int32_t* ext);

/* True labels k = rho^{-1}(k*) (eq:inverse1-3), paper order k_1..k_n, for every
 * vector entry in the plan's vector order.  k_out: host, N*n int32, row i = entry i. */
int iwfpm_indices(iwfpm_plan_t plan, int32_t* k_out);

/* Diagonal Lambda_i = 1/2 |2 pi P k_i|^2 (Sec. 4.1) in vector order; out: host, N float64. */
int iwfpm_kinetic(iwfpm_plan_t plan, double* out);

/* Upper bound of ||H~||_2: max Lambda + sum_m |Vhat_m|. */
int iwfpm_norm_bound(iwfpm_plan_t plan, double* out);

/*
 * iwfpm_apply - Hpsi = Lambda psi + F V F^{-1} psi (Sec. 4.1) for nvec vectors.
 * psi, hpsi: device pointers, complex float64, N x nvec column-major, in the
 * plan's vector order; they must not overlap.  Runs the window gather (T^{-1}),
 * the inverse lifted FFT, the product with V, the forward FFT and the scatter
 * T fused with the kinetic term, all on `stream` (hipStream_t).  Asynchronous:
 * returns after enqueueing.  nvec = 0 is a no-op.
 * Errors: ERR_ARG (NULL pointers, nvec < 0), ERR_NODEVICE, ERR_DEVICE.
 */
int iwfpm_apply(iwfpm_plan_t plan, const void* psi, void* hpsi, int nvec, void* stream);

/* As iwfpm_apply but forcing the convolution precision (IWFPM_PREC_*). */
int iwfpm_apply_prec(iwfpm_plan_t plan, const void* psi, void* hpsi, int nvec,
                     int precision, void* stream);

/*
 * iwfpm_apply_noalloc - iwfpm_apply for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments, result and ordering as iwfpm_apply (the
 * same kernels on the plan's precision), but the multi-pass schedules'
 * intermediate grid lives in a static device array of
 * iwfpm_noalloc_scratch_bytes() bytes (128 MiB) that each GPU the library
 * runs on holds until the process ends, instead of the plan's workspace; the
 * call allocates nothing (the first call on a device also resolves the
 * array's address there).  Vectors are applied in chunks whose intermediate
 * grids fit the array.  All calls on one GPU share its array: calls that
 * overlap in time on one GPU (other streams, other threads) race and give
 * undefined results; serialise them.
 * Errors: ERR_ARG (NULL pointers, nvec < 0, overlapping buffers),
 * ERR_NODEVICE, ERR_UNSUPPORTED, ERR_TOO_LARGE (one vector's intermediate
 * grid, N x 8 B in float32 or N x 16 B in float64, exceeds the array),
 * ERR_DEVICE.
 */
int iwfpm_apply_noalloc(iwfpm_plan_t plan, const void* psi, void* hpsi, int nvec, void* stream);

/* Size in bytes of iwfpm_apply_noalloc's static scratch array. */
int64_t iwfpm_noalloc_scratch_bytes(void);

/* The potential block alone, out = F V F^{-1} psi (Sec. 4.1), same arguments
 * as iwfpm_apply_prec (used by the learned preconditioner's convolution
 * layers). */
int iwfpm_conv(iwfpm_plan_t plan, const void* psi, void* out, int nvec, int precision, void* stream);

/*
 * iwfpm_eigenfunction - the eigenfunction in physical space (eq:int, the
 * interpolant I_{K,L} of Alg. 1's last step): for a coefficient vector U in
 * the plan's vector order,
 *     out(xi) = sum over the window of U_k exp(i 2 pi (P k) . xi)
 * (P in this library's convention, without the paper's 2 pi), at every point
 * of the tensor grid xi_j = origin[j] + step[j] * i_j, i_j = 0 .. npts[j] - 1,
 * j = 0 .. d-1 (the physical dimensions).  Sec. 4 compares eigenfunctions on
 * [-5a, 5a]^d, a = 10^(3-d), with spacing 0.1.
 * u: device, N complex float64.  origin, step: host, d float64; npts: host, d
 * int, each >= 1, product <= 2^36.  out: device, prod(npts) complex float64,
 * row-major (axis 0 slowest); it must not overlap u.  Float64 throughout:
 * phases are reduced to one turn before the sine and cosine.  Asynchronous on
 * `stream` after a one-time set-up per plan (the frequencies P k of the
 * window points, computed on the host and copied synchronously) and growth of
 * the plan's scratch (per-axis tables of up to 256 MB plus slice partials of
 * up to 512 MB), which synchronises `stream` when it reallocates.  Not
 * re-entrant per plan (shared scratch).
 * Errors: ERR_ARG (NULL pointers, npts < 1, non-finite origin or step, too
 * many points), ERR_NODEVICE / ERR_DEVICE, ERR_ALLOC.
 */
int iwfpm_eigenfunction(iwfpm_plan_t plan, const void* u, const double* origin, const double* step,
                        const int* npts, void* out, void* stream);

/*
 * Ragged batches: many plans (for example a sweep of couplings whose windows,
 * and so grid sizes, differ) applied together, Sec. 4.1's H~ psi per plan.
 * iwfpm_batch_create - B plans on one device, convolution precision
 *   IWFPM_PREC_*; use_graph != 0 captures the batch's launches (one persistent
 *   launch per pass walking a work table in device memory) into a hipGraph on
 *   the first apply and replays it afterwards.  The plans must outlive the
 *   batch and must not be used concurrently with it.
 * iwfpm_batch_apply - hpsi[i] = H~_i psi[i] for nvec[i] vectors of plan i
 *   (device pointers, same layout as iwfpm_apply; nvec[i] = 0 skips plan i).
 *   Asynchronous on `stream`; the work table is refreshed by a copy on the same
 *   stream, so consecutive applies may change pointers and counts freely.
 *   A captured graph is bound to the stream it was captured on; another
 *   stream re-captures; on the null stream the launches are issued directly.
 *   A plan may appear only once in a batch.
 * iwfpm_batch_destroy - release (synchronises the device).
 * Errors: ERR_ARG (plans on different devices, bad counts or pointers),
 * ERR_NODEVICE, ERR_UNSUPPORTED, ERR_ALLOC, ERR_DEVICE.
 */
int iwfpm_batch_create(int B, const iwfpm_plan_t* plans, int precision, int use_graph, iwfpm_batch_t* out);
int iwfpm_batch_apply(iwfpm_batch_t batch, const void* const* psi, void* const* hpsi, const int* nvec,
                      void* stream);
int iwfpm_batch_destroy(iwfpm_batch_t batch);

/*
 * iwfpm_tune - autotuner: times every feasible apply schedule of the plan on
 * its device (fused, or three-pass over every axis split x middle-pass tile
 * width x slabs per workgroup x middle-pass workgroup size (256, 512 or
 * 1024 threads); a grid that only the five-pass schedule fits
 * keeps it untimed, best_us = -1) on nvec scratch vectors with HIP events on
 * `stream`, and keeps the fastest for `precision` (IWFPM_PREC_*, or -1 for the
 * plan's).  With the environment variable IWFPM_TUNE_CACHE naming a file,
 * earlier results for the same (precision, order, potential form, d, nvec,
 * extents) are reused and new ones appended (one line per key).  best_us
 * (may be NULL) receives the best time per apply in microseconds, or -1 when
 * the cache answered.  Allocates 2 x nvec vectors of scratch; blocking.
 * iwfpm_schedule - the current schedule for `precision`: out[5] = {fused,
 * split, tile, slabs per workgroup, threads of the middle pass's workgroups
 * (of the fused kernel's when fused)}.
 * Errors: ERR_ARG, ERR_NODEVICE, ERR_UNSUPPORTED, ERR_ALLOC, ERR_DEVICE.
 */
int iwfpm_tune(iwfpm_plan_t plan, int nvec, int precision, void* stream, double* best_us);
int iwfpm_schedule(iwfpm_plan_t plan, int precision, int32_t* out);

/*
 * iwfpm_profile - start (enable = 1) or stop (0) timing the kernels of every
 * subsequent apply on this plan.  Timing uses HIP events recorded on the
 * apply's own stream before and after each kernel (fused, or passes 1-3);
 * nothing blocks while recording.  Enabling resets the totals.
 * iwfpm_profile_read - totals since the last enable: ms[4] summed kernel time
 * (fused, pass 1, pass 2, pass 3), launches[4], points[4] (grid points x
 * vectors processed).  Synchronises with the outstanding events.
 * Errors: ERR_ARG, ERR_NODEVICE, ERR_DEVICE.
 */
int iwfpm_profile(iwfpm_plan_t plan, int enable);
int iwfpm_profile_read(iwfpm_plan_t plan, double* ms, int64_t* launches, int64_t* points);

typedef struct {
    int nev;            /* eigenpairs wanted (lowest), >= 1 */
    int block;          /* LOBPCG block size m >= nev; 0 = nev + max(2, nev/4) */
    double tol;         /* target backward error eta (see iwfpm_eigs) */
    int maxit;          /* iteration limit */
    int precond;        /* IWFPM_PRECOND_* */
    uint64_t seed;      /* start block seed when x0 == NULL */
    int polish;         /* FP32 plans: 1 = finish with float64 applies once FP32 stalls */
    int arith;          /* 0 = auto (real when H~ is real symmetric and x0 == NULL),
                           1 = complex, 2 = real (requires every Vhat_m real and x0 == NULL) */
} iwfpm_eigs_opts;

typedef struct {
    int iterations;     /* LOBPCG iterations */
    int64_t matvecs;    /* single-vector applies (all precisions) */
    int converged;      /* pairs with eta <= tol at exit */
    int restarts;       /* Rayleigh-Ritz restarts without the P block */
    int fallback;       /* learned preconditioner replaced by the plain one (weights
                           that overflow, non-finite directions, or 50 iterations
                           without halving the worst backward error) */
    int polished;       /* iterations done with float64 applies on an FP32 plan */
    double t_total;     /* seconds, wall */
    double t_apply;     /* seconds in applies (device events) */
} iwfpm_stats;

void iwfpm_default_eigs_opts(iwfpm_eigs_opts* opts);

/*
 * iwfpm_eigs - lowest nev eigenpairs of H~ by block LOBPCG (Sec. 4.1: the
 * solver, with the diagonal preconditioner of eq:precond applied to
 * H~ + sigma I, sigma = max(0, sum_{m != 0} |Vhat_m| - Vhat_0) so that the
 * diagonal is positive).
 * Convergence: eta_i = ||H~ x_i - theta_i x_i|| / ((||H~||_est + |theta_i|) ||x_i||)
 * <= tol, with ||H~||_est from iwfpm_norm_bound; the final eta is always
 * evaluated with float64 applies.
 * Real-symmetric problems (every Vhat_m real, so V is even and H~ is a real
 * symmetric matrix) are solved by default in real arithmetic: real trial
 * vectors stored two per complex column, the real and imaginary halves
 * applied together; the returned eigenvectors are then real (zero imaginary
 * parts).  opts->arith chooses explicitly (iwfpm_eigs_batched likewise, real
 * when every plan is real symmetric); the learned preconditioner's training
 * solves always use complex arithmetic.
 * x0: device, N x m start block (m = block size) or NULL for a seeded random start.
 * evals, eta: host, nev float64 (eta may be NULL).  evecs: device, N x nev
 * complex float64, or NULL.  stats may be NULL.  Blocking (synchronises stream).
 * Errors: ERR_ARG, ERR_NODEVICE, ERR_NUMERIC, ERR_NOCONV (results of the last
 * iterate are still written), ERR_WEIGHTS (LEARNED without loaded weights).
 */
int iwfpm_eigs(iwfpm_plan_t plan, const iwfpm_eigs_opts* opts, const void* x0,
               double* evals, void* evecs, double* eta, iwfpm_stats* stats, void* stream);

/*
 * iwfpm_eigs_batched - lowest nev eigenpairs of B plans at once (e.g. a sweep
 * of couplings whose windows differ), by block LOBPCG run in lock step: every
 * tall operation of an iteration runs for all unconverged plans in one launch,
 * the applies in one persistent batched launch replayed from a hipGraph, and
 * each plan's small Rayleigh-Ritz problem on a host thread.  Same options,
 * convergence test and float32 -> float64 policy as iwfpm_eigs (block size at
 * most 21 here); start blocks are seeded with opts->seed + i.
 * evals, eta: host, B x nev (row i = plan i); stats: B entries or NULL.
 * Plans must be distinct and on one device.  Blocking.
 * Errors: as iwfpm_eigs; the first plan's failure status is returned
 * (ERR_NOCONV if any plan hit maxit), results are written for every plan;
 * ERR_WEIGHTS (LEARNED and a plan without a usable network).  With LEARNED,
 * each plan's directions come from its attached network (two convolutions
 * per plan and iteration) and fall back to M per plan as in iwfpm_eigs.
 */
int iwfpm_eigs_batched(int B, const iwfpm_plan_t* plans, const iwfpm_eigs_opts* opts, double* evals, double* eta,
                       iwfpm_stats* stats, void* stream);

/*
 * Host-side small dense solvers used by iwfpm_eigs's Rayleigh-Ritz step,
 * exported so that they can be checked on their own (no device needed).
 * Matrices are complex float64, column-major, interleaved (re, im), n x n.
 * iwfpm_dense_geneig - A c = w B c for Hermitian A and Hermitian positive
 *   definite B (B = NULL means the identity): Cholesky of B, reduction to a
 *   standard problem, Householder tridiagonalisation and implicit QL (cyclic
 *   Jacobi if QL does not converge).  w: n ascending eigenvalues; C: the
 *   B-orthonormal eigenvectors.  Errors: ERR_ARG (n < 1 or n > 512),
 *   ERR_NUMERIC (B not positive definite).
 * iwfpm_dense_svqb - for a Gram matrix G = V^H V (k x k) returns T (k x rank)
 *   with (V T)^H (V T) = I, dropping directions whose scaled eigenvalue is
 *   below 1e-12 of the largest.  T must hold k*k entries.
 * iwfpm_dense_heev_lowest - the Rayleigh-Ritz step's eigensolver: all n
 *   eigenvalues of the Hermitian A (w, ascending) and orthonormal
 *   eigenvectors of the nv lowest (V, n x nv), rebuilt from the stored
 *   reflectors and the recorded QL rotations for those columns only.
 *   Errors: ERR_ARG (n < 1, n > 512, nv < 0 or nv > n).
 */
int iwfpm_dense_geneig(int n, const double* A, const double* B, double* w, double* C);
int iwfpm_dense_svqb(int k, const double* G, double* T, int* rank);
int iwfpm_dense_heev_lowest(int n, int nv, const double* A, double* w, double* V);

/*
 * Learned preconditioner.  The paper preconditions LOBPCG with the diagonal
 * M of eq:precond (Sec. 4.1).  This adds a trained alternative that keeps M as
 * its starting point and its fallback:
 *     W = D0 .* R + b1 (C E + a)^H E (C E + a) R
 *       = (D0 + b1 a^2 E) .* R + 2 a b1 E .* C(E .* R) + b1 E .* C(E .* C(E .* R)),
 * with a = beta0 and b1 = max(beta1, 0), so that the two convolution layers
 * add a positive semidefinite term and W stays Hermitian positive definite,
 * with C = F V F^{-1} the potential block (the convolution of iwfpm_conv, run
 * in the plan's precision), D0 = M .* (1 + exp(o0)) / 2 (never below M/2) and
 * E = M .* exp(o1), where
 * (o0, o1) are the outputs of an MLP (IWFPM_LEARNED_FEATURES inputs, 3 hidden
 * layers of IWFPM_LEARNED_HIDDEN, exact GELU, 2 linear outputs) evaluated on
 * each kinetic-energy shell of the plan.  Shell of grid point k:
 *     s(k) = min(S - 1, floor(S sqrt(e_k / e_max))),  e_k = 1/2 |2 pi P k|^2,
 * e_max = max e_k (s = 0 everywhere when e_max = 0).  Features of shell s,
 * with c = (s + 1/2)/S, e = e_max c^2, nu = sum_{m != 0} |Vhat_m|,
 * v0 = Re Vhat_0, sigma = max(0, nu - v0), S2 = sum_{m != 0} |Vhat_m|^2,
 * h = e + v0 + sigma:
 *     f0 = c, f1 = log(1 + e)/8, f2 = e/(e + nu), f3 = log(1 + nu)/4,
 *     f4 = h^2/(h^2 + S2), f5 = nu/h, f6 = log(1 + e_max)/8,
 *     f7 = sqrt(e)/(sqrt(e) + sqrt(nu))       (0/0 read as 0).
 * Weight matrices are stored in bfloat16 (round to nearest even from the
 * float32 masters) and multiplied with float32 accumulation; biases, beta and
 * the optimiser state (Adam) are float32.  A new network reproduces M exactly
 * (last layer zero, beta = 0).
 *
 * Parameter vector (float32, iwfpm_learned_nparams entries), in order: for
 * layers l = 1..4 with (in, out) = (F, H), (H, H), (H, H), (H, 2): W_l
 * (in x out, row-major, W[i*out + o]) then b_l (out); then beta0, beta1.
 * (Where beta1 < 0 the gradient reported for it is that of its positive side.)
 *
 * Training loss of an iterate block X (m columns) given the exact lowest m
 * eigenvalues lam: with (Y, theta) the Ritz pairs of span(X), R = H~ Y - Y theta
 * and theta' the lowest m Ritz values of span([Y, W(R)]),
 *     loss = sum_j (theta'_j - lam_j) / sum_j (theta_j - lam_j),
 * the share of eigenvalue error left after one Rayleigh-Ritz step with the
 * preconditioned residuals (0 = the step finds the eigenvalues, 1 = no gain).
 * H~ is applied in float64 here (when the plan has a float64 schedule).
 * iwfpm_learned_train takes its blocks from the method's own solves: a
 * plain-preconditioned LOBPCG run per plan records the first nev columns of
 * its iterate X every `stride` iterations, and its converged eigenvalues are
 * lam (records whose columns had all converged are left out).
 */
#define IWFPM_LEARNED_FEATURES 8
#define IWFPM_LEARNED_HIDDEN 256

typedef struct iwfpm_learned_s* iwfpm_learned_t;

typedef struct {
    int device;         /* HIP device of the weights */
    int shells;         /* S, kinetic-energy shells per plan, 1..65536 */
    uint64_t seed;      /* initialisation of the hidden layers (uniform +-1/sqrt(fan_in)) */
} iwfpm_learned_opts;

typedef struct {
    int steps;          /* Adam steps */
    double lr;          /* Adam step size (beta1 0.9, beta2 0.999, eps 1e-8) */
    int nev;            /* eigenpairs of the data-producing solves (columns per sample) */
    int block;          /* their LOBPCG block size (0 = default) */
    double tol;         /* their tolerance (backward error) */
    int maxit;
    int snapshots;      /* recorded iterates per plan, 1..64 */
    int stride;         /* iterations between recorded iterates, >= 1 */
    uint64_t seed;      /* sample order and the solves' start blocks */
} iwfpm_train_opts;

void iwfpm_default_learned_opts(iwfpm_learned_opts* opts);   /* device 0, 1024 shells */
void iwfpm_default_train_opts(iwfpm_train_opts* opts);       /* 3000 steps, lr 1e-3, nev 8, tol 1e-8,
                                                                maxit 1000, 24 snapshots, stride 4 */

/* Create / destroy a network.  Destroying a network detaches it from every
 * plan it is attached to (their LEARNED solves then return ERR_WEIGHTS). */
int iwfpm_learned_create(const iwfpm_learned_opts* opts, iwfpm_learned_t* out);
int iwfpm_learned_destroy(iwfpm_learned_t net);
int iwfpm_learned_nparams(iwfpm_learned_t net, int64_t* n);
/* Copy the float32 parameters out / in (host arrays of nparams floats).
 * set: ERR_WEIGHTS if any value is not finite (the network is unchanged);
 * it also resets the optimiser state. */
int iwfpm_learned_get(iwfpm_learned_t net, float* params);
int iwfpm_learned_set(iwfpm_learned_t net, const float* params);

/* Attach net to a plan (net = NULL detaches): builds the plan's shell map and
 * features; iwfpm_eigs with IWFPM_PRECOND_LEARNED then uses it.  One network
 * may serve many plans; the plan and the net must be on one device. */
int iwfpm_learned_attach(iwfpm_plan_t plan, iwfpm_learned_t net);
/* The attached plan's shell of each vector entry (host, N int32) and the
 * shell features (host, S x IWFPM_LEARNED_FEATURES float32, row-major);
 * either may be NULL. */
int iwfpm_learned_shells(iwfpm_plan_t plan, int32_t* shell, float* features);

/* T = W(R) for nvec columns (device blocks in the plan's vector layout). */
int iwfpm_learned_forward(iwfpm_plan_t plan, const void* r, void* t, int nvec, void* stream);
/* Training loss of the iterate block x (device, nvec columns, 2 nvec <= 64)
 * with exact eigenvalues lam (host, nvec, ascending) in *loss and, if
 * grad != NULL, its gradient with respect to the parameter vector (host,
 * nparams floats; weight entries are derivatives at the bfloat16-rounded
 * weights).  No update.  Blocking.  ERR_NUMERIC when the block carries no
 * signal (dependent columns, or Ritz values already at lam). */
int iwfpm_learned_grad(iwfpm_plan_t plan, const void* x, int nvec, const double* lam, double* loss, float* grad,
                       void* stream);
/* One Adam step (step size lr) of the attached network on (x, lam); the loss
 * before the step in *loss.  A step whose loss or gradient is not finite, or
 * whose block carries no signal, is skipped (ERR_NUMERIC).  Blocking. */
int iwfpm_learned_step(iwfpm_plan_t plan, const void* x, int nvec, const double* lam, double lr, double* loss,
                       void* stream);
/* Train net on data from B plans (see above); the net is attached to each
 * plan.  loss: host, opts->steps entries or NULL.  Blocking.
 * Errors: ERR_ARG, ERR_ALLOC, ERR_DEVICE, the solves' errors (ERR_NOCONV is
 * tolerated), ERR_NUMERIC when no usable sample was recorded. */
int iwfpm_learned_train(iwfpm_learned_t net, int B, const iwfpm_plan_t* plans, const iwfpm_train_opts* opts,
                        double* loss, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* IWFPM_H */
