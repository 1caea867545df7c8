/*
 * eigseis — Laplace expected-information-gain design for 2-D seismic source
 * inversion on AMD MI355X (gfx950).  C ABI.
 *
 * Method: Long, Motamed & Tempone, "Fast Bayesian optimal experimental
 * design for seismic source inversion".  For every prior sample theta of the
 * seven source parameters the library runs one nominal and 2*7 perturbed
 * forward solves of the 2-D elastic wave equation (Section 3.3.1), forms the
 * central-difference receiver Jacobian, the Gauss-Newton Hessian H_1
 * (Theorem 2), its scaled Cholesky log-determinant (Section 3.3.3), the
 * Laplace KL estimate D^_KL (Theorem 4), and the Monte Carlo or sparse-
 * quadrature average over samples (Section 3.3.4) for each receiver design.
 *
 * Conventions (all entry points):
 *  - Return 0 on success, a negative EIG_E* code otherwise; eig_last_error()
 *    then holds a message (thread-local).  No C++ exception crosses the ABI.
 *  - Argument errors are found synchronously, before any work is enqueued.
 *    Work is enqueued on `stream` (a hipStream_t; NULL = default stream);
 *    device outputs are valid after the stream has been synchronised.
 *  - Numerical failures found on the device (a non-positive-definite
 *    Hessian, a non-finite wavefield, a time step the stability bound does
 *    not cover) are reported per sample in `status` (EIG_ENOTPD /
 *    EIG_ENONFINITE / EIG_EUNSTABLE) and poison dependent results with NaN;
 *    the other samples of the call are computed exactly as alone.
 *  - "host" pointers are read before the call returns; "device" pointers are
 *    caller-owned device memory, never freed or kept by the library after
 *    the enqueued work completes.
 *  - Units SI.  Coordinates: node (i, k) sits at x = i*h (from the left edge)
 *    and depth z = k*h; k = 0 is the traction-free surface; the nodes of the
 *    left (i = 0), right (i = nx-1) and bottom (k = nz-1) edges are rigid.
 *  - theta, in the paper's order (Section 2.1):
 *      [0] x_s  [1] z_s (depth)  [2] t_s  [3] frequency  [4] m_xx  [5] m_xz
 *      [6] m_zz
 *    For EIG_STF_GAUSS the frequency slot is omega (rad/s); for
 *    EIG_STF_GAUSS_DERIV it is f (Hz) with omega = 2 pi f.
 *  - Receiver traces: float [nsteps+1][nrec][2], level m at t_m = m*dt,
 *    component 0 = x, 1 = depth.  Level 0 is the zero initial state.
 *  - One context per host thread; calls on one context must not overlap.
 */
#ifndef EIGSEIS_H
#define EIGSEIS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EIG_NTHETA 7

/* error codes */
#define EIG_OK 0
#define EIG_EINVAL (-1)       /* invalid argument */
#define EIG_ENOMEM (-2)       /* device allocation failed */
#define EIG_EBUDGET (-3)      /* request does not fit the HBM budget */
#define EIG_ENOTPD (-4)       /* Hessian not positive definite (status) */
#define EIG_ENONFINITE (-5)   /* non-finite wavefield (status) */
#define EIG_EHIP (-6)         /* HIP runtime error */
#define EIG_EUNSUPPORTED (-7) /* valid but not supported */
#define EIG_EUNSTABLE (-8)    /* time step beyond the stability bound (status) */

/* source time functions (Section 4.1 and its time derivative) */
#define EIG_STF_GAUSS 0       /* omega/sqrt(2 pi) exp(-omega^2 (t-t_s)^2 / 2) */
#define EIG_STF_GAUSS_DERIV 1 /* d/dt of the above with omega = 2 pi f      */

/* media */
#define EIG_MEDIUM_LAYERED 0  /* rho, lam, mu arrays of [nz] (depth only) */
#define EIG_MEDIUM_NODAL 1    /* rho, lam, mu arrays of [nz][nx]          */

/* left, right and bottom edges of the grid (the top row is always the
 * traction-free surface, eq. for the free-surface condition in Section 2.1) */
#define EIG_BC_RIGID 0      /* edge nodes held at zero                        */
#define EIG_BC_ABSORBING 1  /* first-order Clayton-Engquist condition (Section
                             * 2.1 artificial boundary; Section 4.1 model)   */

/* priors */
#define EIG_PRIOR_UNIFORM 0
#define EIG_PRIOR_GAUSSIAN 1

/* noise level for jacobian_fd */
#define EIG_SIGMA_GIVEN 0        /* sigma[s] is the noise standard deviation */
#define EIG_SIGMA_NOMINAL_PEAK 1 /* sigma_s = sigma[s] * max |nominal trace| */

typedef struct eig_ctx eig_ctx;

/* Uniform grid of Section 3.3.1 (spacing h in both directions) with the
 * leapfrog time step dt and nsteps steps.  nx, nz >= 8.
 *
 * bc = EIG_BC_ABSORBING: every node of the left, right and bottom edges obeys
 * u_t = B sigma(u) n, B = -(1/rho)(n n^T/c_p + t t^T/c_s) (n outward normal,
 * t tangent, node's own rho, lambda, mu), instead of the wave equation; the
 * normal derivative is one-sided into the grid, the tangential one central
 * (one-sided at the ends of the edge, corners take their column's relation);
 * time is the centred difference of Section 3.3.1 with the node's own
 * same-component term taken at the mean of levels m+1 and m-1 (the fully
 * explicit form diverges).  Such grids always run one step per launch. */
typedef struct {
    int32_t nx, nz;
    double h, dt;
    int32_t nsteps;
    int32_t bc;  /* EIG_BC_RIGID or EIG_BC_ABSORBING */
} eig_grid;

/* Density nu and Lame parameters (lambda, mu) of the paper's stress law
 * (Section 2.1); device pointers to FP64 arrays, laid out per `kind`. */
typedef struct {
    int32_t kind;
    const double* rho;
    const double* lam;
    const double* mu;
} eig_medium;

/* Receivers on surface nodes (Section 2.1: stations coincide with grid
 * points): n distinct x-indices in 1..nx-2, host array. */
typedef struct {
    int32_t n;
    const int32_t* ix;
} eig_receivers;

/* Prior density p(theta); h(theta) = log p(theta) enters D^_KL.
 * active: bit j set = theta_j is inferred (0 means all seven).  Parameters
 * outside the mask are known: D^_KL then takes the active sub-block of H_1,
 * N_theta = the number of active parameters, and h is the prior's marginal
 * over them (uniform: the sub-box; Gaussian: the sub-mean and sub-covariance),
 * as in the reduced-parameter experiments of Sections 4.3 and 4.4. */
typedef struct {
    int32_t kind;
    double lo[EIG_NTHETA], hi[EIG_NTHETA];  /* uniform box, lo < hi */
    double mean[EIG_NTHETA];                /* gaussian mean */
    double cov[EIG_NTHETA * EIG_NTHETA];    /* gaussian covariance, SPD */
    int32_t active;                         /* bitmask of inferred parameters */
} eig_prior;

/* Create a context on HIP device `device`.  The context owns all internal
 * device workspace (wavefields, internal traces, tables) and never holds more
 * than hbm_budget_bytes of it.  Returns EIG_EINVAL for a bad device. */
int eig_ctx_create(int device, size_t hbm_budget_bytes, eig_ctx** out);
void eig_ctx_destroy(eig_ctx* ctx);
/* Message for the last error on this thread ("" if none). */
const char* eig_last_error(void);
/* Device bytes currently held by the context's workspace. */
size_t eig_ctx_workspace_bytes(const eig_ctx* ctx);
/* Stencil timing since the last reset: device time from the first to the
 * last stencil launch of every wave (HIP events on the call's stream), the
 * number of stencil launches, the grid-point updates they performed
 * (sum over solves of nx*nz per step) and their algorithmic HBM bytes (per
 * update: read u^m and u^{m-1}, write u^{m+1}, 8 bytes each; plus 12 bytes
 * of nodal coefficients for EIG_MEDIUM_NODAL).  Waits for the recorded
 * events.  Any output pointer may be NULL; reset != 0 clears the counters
 * after reading them. */
int eig_ctx_stencil_stats(eig_ctx* ctx, int32_t reset, double* ms, int64_t* launches,
                          double* updates, double* bytes);

/* Context options (take effect for later calls):
 *   "stencil_variant"  -1: choose automatically (default), else force one of
 *                      the stencil kernel variants (all give bitwise-identical
 *                      fields; they differ in tile shape and speed).  Forcing
 *                      a tiled variant also turns the resident kernels off;
 *                      forcing 21 or 22 leaves the choice among tiled kernels
 *                      automatic for grids that do not fit LDS
 *   "resident"         1 (default): a solve whose two field levels (16 nx nz
 *                      bytes), forcing window (512 B) and, for depth-only
 *                      media, coefficient table (64 nz bytes) fit the 160 KiB
 *                      of LDS one workgroup may hold, and whose edge nodes
 *                      number at most 3072, runs resident: one workgroup per
 *                      solve takes every time step in one launch (variants 21
 *                      depth-only, 22 nodal), with no field buffers in device
 *                      memory; 0: tiled kernels for every grid.  Results do
 *                      not depend on it
 *   "autotune"         1 (default): time the variants on the first steps of a
 *                      new grid class and keep the fastest; 0: use
 *                      "default_variant"
 *   "default_variant"  variant used before/without tuning
 *   "graphs"           1 (default): once a wave's variants are tuned, its time
 *                      loop is captured as a HIP graph (kernels only) and
 *                      replayed when the same wave (same descriptors at the
 *                      same device addresses) comes again; 0: direct launches.
 *                      get_option also reports "graph_captures" and
 *                      "graph_replays"
 *   "wave_cache_bytes" 201326592 (192 MiB, default): when the field buffers a
 *                      wave keeps live between launches (four per solve for
 *                      several steps per launch, else two) exceed this, the
 *                      wave runs as consecutive chunks of about this many
 *                      bytes, so that each chunk's fields stay in the
 *                      device's 256 MB last-level cache (solves grouped by
 *                      grid and length); waves where fewer than
 *                      "cache_chunk_min_solves" solves would fit are not
 *                      split.  Solves taking four steps per launch do not
 *                      count (they run as one wave through HBM).  0: never
 *                      split for the cache.  Results do not depend on it.
 *   "cache_chunk_min_solves" 16 (default): see "wave_cache_bytes"; >= 1
 *   "coef_interleave"  8 (default): in nodal media, up to this many
 *                      consecutive solves of a wave on one medium and grid
 *                      (same length) have their tiles ordered by position
 *                      first, so that the solves' tiles at one position run
 *                      together and read the medium's coefficients from L2
 *                      once; 1 keeps each solve's tiles together.  1..4096.
 *                      Results do not depend on it.
 *   "serve_cache_bytes" 201326592 (192 MiB, default): serving engines created
 *                      afterwards admit sample groups of a query one of whose
 *                      samples fits this only while the live field bytes of
 *                      all such admitted groups stay within it (groups shrink
 *                      to fit; at least one group is always admitted), and
 *                      use 16-row tiles, so their launches work in the
 *                      last-level cache; queries with larger samples, and
 *                      every query of a kind that takes four steps per
 *                      launch ("temporal_blocking" 4), are admitted by
 *                      memory alone.  0: admit whatever memory and slots
 *                      allow.  Results do not depend on it.
 *   "fused_edges"      1 (default): the two-nodes-per-lane one-step kernels
 *                      update absorbing edge nodes in extra wavefronts of
 *                      their own launch; 0: a separate edge kernel after each
 *                      launch.  Same results either way.
 *   "max_wave_solves"  0 (default): no limit; n > 0: at most n solves per
 *                      launch (n = 1 is the plain one-solve-at-a-time path)
 * EIG_EINVAL for an unknown name or value. */
int eig_ctx_set_option(eig_ctx* ctx, const char* name, int64_t value);
/* Reads an option back; "last_variant" gives the stencil variant of the most
 * recent launch.  "temporal_blocking": leapfrog steps per launch for media
 * with rigid edges, 4 (default: the tile and its halo in LDS for four steps,
 * variants 23 depth-only, 24 and 25 nodal), 2 (1 also selects 2), 3
 * (depth-only media; nodal media then take two), or 0 for one step; two to
 * four steps per launch keep four field buffers per solve.  Serving engines
 * created while it is 4 take four steps per launch for both media (variants
 * 23, 24); otherwise two for depth-only media and one for nodal media. */
int eig_ctx_get_option(const eig_ctx* ctx, const char* name, int64_t* value);

/*
 * forward_solve_batch — the parameter-to-observable map g_r(t_m; theta)
 * (Section 2.2, forward model; Section 3.3.1, full-discrete scheme) for
 * nsolve independent solves of possibly different grids and media.
 *
 *   grid, medium, rec: host arrays [nsolve]
 *   theta:     host [nsolve][7]
 *   dev_param: host [nsolve] or NULL.  -1 (or NULL): nominal solve, forcing
 *              F(theta).  j in 0..6: deviation solve driven by the FP64
 *              forcing difference F(theta + dev_step[s] e_j) - F(theta); by
 *              linearity of the discrete scheme its traces are
 *              g(theta + dev_step e_j) - g(theta).
 *   dev_step:  host [nsolve] (read only for deviation solves), nonzero.
 *   traces:    host array [nsolve] of device pointers, each float
 *              [grid.nsteps+1][rec.n][2]; fully overwritten.
 * EIG_EINVAL if the 6x6 source stencil of theta (or of theta + step e_j)
 * would touch a rigid node, a deviation step of x_s or z_s moves the source
 * out of its cell by more than one cell (the forcing window is the 7x7 union
 * of the two stencils), a receiver is off the free surface or repeated, or a
 * size is out of range.  nsolve == 0 does nothing and returns EIG_OK
 * (the arrays may then be NULL).
 */
int forward_solve_batch(eig_ctx* ctx, int32_t nsolve, const eig_grid* grid,
                        const eig_medium* medium, const double* theta,
                        const int32_t* dev_param, const double* dev_step,
                        int32_t stf_kind, const eig_receivers* rec,
                        float* const* traces, void* stream);

/*
 * jacobian_fd — for each of nsample prior samples: 1 nominal + 2*7 perturbed
 * solves, the central-difference receiver Jacobian
 *   J_j = (g(theta + d_j e_j) - g(theta - d_j e_j)) / (2 d_j),
 *   d_j = rel_step * |theta_j|,
 * formed from deviation solves (see forward_solve_batch) in FP64, and the
 * Gauss-Newton Hessian H_1 = sigma^-2 sum_{m,r,c} J^T J (Theorem 2, H_1, with
 * C_eps = sigma^2 I; Section 3.3.2, H_I with the receiver-selection Hessian).
 *
 *   grid, medium, rec: host arrays [nsample] (each sample may differ; with
 *              per_receiver != 0 all rec[s].n must be equal)
 *   theta:     host [nsample][7]; every theta_j must be nonzero
 *   sigma_mode/sigma: host [nsample]; EIG_SIGMA_GIVEN: sigma[s] > 0 is the
 *              noise std; EIG_SIGMA_NOMINAL_PEAK: sigma_s = sigma[s] times the
 *              largest |value| in sample s's nominal traces (device-side)
 *   per_receiver: 0 -> H1 device [nsample][7][7];
 *                 1 -> H1 device [nsample][nrec][7][7] (one H_1 per receiver;
 *                      their sum over receivers is the full H_1)
 *   nominal:   host array [nsample] of device pointers (float
 *              [nsteps+1][nrec][2]) or NULL
 *   J:         host array [nsample] of device pointers (double
 *              [nsteps+1][nrec][2][7]) or NULL
 *   status:    device [nsample] or NULL: 0; EIG_ENONFINITE if a trace of
 *              the sample holds a non-finite value; else EIG_EUNSTABLE if the
 *              step exceeds the sample's stability bound: with B = -dt^2
 *              rho^-1 A_h (A_h the discrete operator of Section 3.3.1 on the
 *              sample's medium), some free node's x or depth row has an
 *              absolute row sum above 4 (Gershgorin: the leapfrog step is
 *              stable when every eigenvalue of B is at most 4; this bound
 *              allows v_p dt / h up to 0.816 for v_s = v_p / sqrt 3, the exact
 *              homogeneous limit being 0.866).  A flagged sample's H_1 is NaN
 *              (its noise level is set to NaN), whether or not status is given.
 * EIG_EINVAL also when rel_step * |x_s| or rel_step * |z_s| moves the source
 * out of its cell by more than one cell (the 7x7 forcing window of a
 * deviation solve covers the nominal and the perturbed stencil only then);
 * with the paper-sized rel_step = 1e-4 this needs coordinates beyond 1e4 h.
 * nsample == 0 does nothing and returns EIG_OK (the arrays may then be NULL).
 */
int jacobian_fd(eig_ctx* ctx, int32_t nsample, const eig_grid* grid,
                const eig_medium* medium, const double* theta, double rel_step,
                int32_t stf_kind, const eig_receivers* rec, int32_t sigma_mode,
                const double* sigma, int32_t per_receiver, float* const* nominal,
                double* const* J, double* H1, int32_t* status, void* stream);

/*
 * jacobian_sensitivity — the forward-sensitivity form of the same quantity
 * (Algorithm 1, its sensitivity solves; the remark of Section 3.3.2 that H_I needs only
 * N_theta primal solves): for each sample 1 nominal solve plus, for every
 * parameter j, one solve whose forcing is dF/dtheta_j, the exact derivative of
 * the discretised point source f = S(t) M grad(delta):
 *   x_s, z_s: S(t) M grad(d delta/dx_s) from the differentiated regularised
 *             delta/delta' weights (Section 3.3.2, item 2), FP64 tables;
 *   t_0, f:   dS/dt_0, dS/df of the wavelet times M grad(delta);
 *   M_j:      S(t) E_j grad(delta) with the unit symmetric tensor E_j.
 * By linearity of the discrete solve in its forcing, each such solve's traces
 * are the column J_j itself (no step size, no truncation error), and H_1 is
 * assembled exactly as in jacobian_fd.  8 solves per sample instead of 15.
 *
 * Arguments, layouts, ownership and errors are those of jacobian_fd without
 * rel_step, except that theta entries may be zero (no relative step is
 * taken); the source's 6x6 stencil must avoid the rigid nodes.
 */
int jacobian_sensitivity(eig_ctx* ctx, int32_t nsample, const eig_grid* grid,
                         const eig_medium* medium, const double* theta, int32_t stf_kind,
                         const eig_receivers* rec, int32_t sigma_mode, const double* sigma,
                         int32_t per_receiver, float* const* nominal, double* const* J,
                         double* H1, int32_t* status, void* stream);

/*
 * nested_mc_eig — the direct double-loop sample average of the expected
 * information gain (the estimator the introduction calls prohibitively
 * expensive, compared with the Laplace method in Section 4.4).  For outer
 * samples n with model outputs g_n (data y_n = g_n + sigma e_n) and inner
 * prior samples m with outputs g_m, C_eps = sigma^2 I:
 *   logratio_n = -|e_n|^2/2 - log( (1/M) sum_m exp(-|y_n - g_m|^2 / (2 sigma^2)) )
 *   eig        = (1/N) sum_n logratio_n
 * (Gaussian normalisers cancel).  Reusing the outer samples as the inner
 * ones, as the paper does, is the caller's choice (g_inner == g_outer).
 *
 *   g_outer: device float [nouter][nobs] (e.g. traces [nt][nrec][2] per solve)
 *   noise:   device float [nouter][nobs], standard normal draws (the caller's)
 *   g_inner: device float [ninner][nobs]
 *   sigma > 0; logratio: device double [nouter]; eig: device double [1] or NULL
 * y_n in FP64 (the FP32 inputs are exact in FP64); squared distances in
 * Gram form |y|^2 + |g|^2 - 2 <y, g> on the FP64 matrix cores, which adds
 * about K 2^-53 (|y_n|^2 + |g_m|^2) / (2 sigma^2) nats of rounding to a log
 * ratio; log-sum-exp with its maximum and rescaling in FP64 and the terms
 * within 40 nats of the maximum as FP32 exponentials (at most ~3e-6 nats),
 * terms further down dropped.  Context workspace: 16 bytes per outer sample
 * per inner-range split (the inner range is split so that the launch fills
 * whole rounds of the device), 8 bytes per outer and per inner sample, and
 * FP64 copies of the y_n and g_m, k-major and padded to whole tiles:
 * 8 kpad (npad + mpad) bytes, kpad = nobs rounded up to a multiple of 16,
 * npad and mpad = nouter and ninner rounded up to multiples of 128 (1.3 GB
 * at nouter = ninner = 4e5, nobs = 204).  Errors: EIG_EINVAL for
 * non-positive sizes or sigma, NULL arrays; EIG_EBUDGET when the workspace
 * would exceed the context's budget.
 */
int nested_mc_eig(eig_ctx* ctx, int32_t nouter, int32_t ninner, int32_t nobs,
                  const float* g_outer, const float* noise, const float* g_inner,
                  double sigma, double* logratio, double* eig, void* stream);

/*
 * theorem3_eig — the O(N^-2) estimator of Theorem 3.  For each outer sample
 * (theta*_s, noise e_s): data y_s = g(theta*_s) + sigma e_s; the MAP point
 * theta^_s by Gauss-Newton from theta*_s (Theorem 1 puts it within
 * O(N^-1/2)); at theta^_s
 *   H_1 from the 7 forward-sensitivity solves (Algorithm 1),
 *   H_2 = -sum_{r,m} grad grad g o C_eps^-1 (y - g(theta^)) (Theorem 2) from one
 *         dual solve (Algorithm 1): with rigid edges the adjoint of
 *         the leapfrog scheme is the same stencil run backward in time, driven
 *         at the receivers by the residuals divided by the lumped mass
 *         h^2/2 of a surface node; its field on the 7x7 forcing window is
 *         contracted with the second derivatives of the discretised source,
 *   and the integrand
 *   -1/2 log((2 pi)^N |H^-1|) - N/2 - h(theta^) - 1/2 tr(H^-1 grad grad h),
 *   H = H_1 + H_2 - grad grad h (active parameters of the prior only; the
 *   others stay at theta*).
 * Cost per sample: 1 + 8 (iters + 1) + 1 solves; the call synchronises the
 * stream once per Gauss-Newton iteration (theta is updated on the host).
 *
 *   grid, medium, rec: host arrays [nsample]; rigid edges only
 *              (EIG_EUNSUPPORTED otherwise)
 *   theta_star: host [nsample][7]; noise: host array [nsample] of device
 *              float pointers [nsteps+1][nrec][2] (standard normal draws)
 *   sigma > 0: C_eps = sigma^2 I; prior: as for laplace_eig; w: host [nsample]
 *   iters:     Gauss-Newton steps, 0..64 (0: theta^ = theta*)
 *   theta_hat: host [nsample][7] (out); H1, H2: device [nsample][7][7] (out)
 *   val:       device [nsample] integrands; eig: device [1] (sum w_s val_s)
 *              or NULL; status: device [nsample] (EIG_ENOTPD if H is not
 *              positive definite) or NULL
 * Errors: EIG_EINVAL for bad arguments or an iterate whose source stencil
 * leaves the free nodes, EIG_ENOTPD if a Gauss-Newton system is singular.
 */
int theorem3_eig(eig_ctx* ctx, int32_t nsample, const eig_grid* grid,
                 const eig_medium* medium, const double* theta_star, int32_t stf_kind,
                 const eig_receivers* rec, const float* const* noise, double sigma,
                 const eig_prior* prior, const double* w, int32_t iters, double* theta_hat,
                 double* H1, double* H2, double* val, double* eig, int32_t* status,
                 void* stream);

/*
 * laplace_eig — Theorem 4 with the scaled Hessian of Section 3.3.3:
 *   S = sqrt(diag H_1),  H~ = S^-1 H_1 S^-1 = L L^T,
 *   log det H_1 = 2 sum log L_ii + 2 sum log S_ii,
 *   D^_KL(theta_s) = -1/2 log((2 pi)^7 |H_1^-1|) - 7/2 - h(theta_s),
 *   I = sum_s w_s D^_KL(theta_s)  (Monte Carlo or quadrature weights,
 *       Section 3.3.4), all in FP64.
 *
 *   H1:     device [nsample][7][7] (symmetric)
 *   prior:  host; theta: host [nsample][7] (needed for EIG_PRIOR_GAUSSIAN,
 *           may be NULL for EIG_PRIOR_UNIFORM); w: host [nsample]
 *   dkl:    device [nsample]; logdet: device [nsample] or NULL;
 *   eig:    device [1]; status: device [nsample] or NULL (0 or EIG_ENOTPD).
 *   A failed sample has dkl = NaN, which makes eig NaN.
 * EIG_EINVAL for nsample <= 0 (an average over no samples) or a NULL array.
 */
int laplace_eig(eig_ctx* ctx, int32_t nsample, const double* H1,
                const eig_prior* prior, const double* theta, const double* w,
                double* dkl, double* logdet, double* eig, int32_t* status,
                void* stream);

/*
 * design_eval — expected information gain of each receiver design
 * (Section 4.5: designs are receiver sets): for design d,
 *   I(d) = sum_s w_s D^_KL( sum_{c : mask[d][c] != 0} H1r[s][c] ),
 * where H1r holds one H_1 per candidate receiver (additive over receivers),
 * as produced by jacobian_fd with per_receiver = 1.
 *
 *   H1r:  device [nsample][ncand][7][7];  mask: device uint8 [ndesign][ncand]
 *   prior, theta, w: as for laplace_eig;  eig: device [ndesign]
 */
int design_eval(eig_ctx* ctx, int32_t nsample, int32_t ncand, const double* H1r,
                int32_t ndesign, const uint8_t* mask, const eig_prior* prior,
                const double* theta, const double* w, double* eig, void* stream);

/*
 * design_greedy — greedy receiver selection on the same objective: start
 * from no receivers and kmax times add the candidate c maximising
 * I(chosen + {c}); ties go to the lowest index; a candidate whose I is NaN is
 * never chosen.  The search stays on the device.
 *   order: device int32 [kmax] (chosen candidate per step, -1 once none is
 *          left); curve: device [kmax] (I after each step, NaN after -1).
 */
int design_greedy(eig_ctx* ctx, int32_t nsample, int32_t ncand,
                  const double* H1r, const eig_prior* prior, const double* theta,
                  const double* w, int32_t kmax, int32_t* order, double* curve,
                  void* stream);

/*
 * design_greedy_noalloc — design_greedy for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops and
 * harnesses that forbid hipMalloc.  It calls no hipMalloc, hipFree or other
 * allocating routine (and no memset: only kernel launches on `stream`), and
 * gives bitwise the same order and curve as design_greedy.
 *
 *   H1r:   device [nsample][ncand][7][7] (as for design_greedy)
 *   prior: host, copied into device scratch by a kernel launched on `stream`
 *   theta: DEVICE [nsample][7], needed for EIG_PRIOR_GAUSSIAN, may be NULL
 *          for EIG_PRIOR_UNIFORM
 *   w:     DEVICE [nsample] weights
 *   order, curve: device [kmax], as for design_greedy
 * Scratch: a 64 MiB static device array per GPU (held until the process
 * ends), of which a call uses about 8 * nsample * (ncand + 49) + 9 * ncand
 * bytes plus 1 KiB; EIG_EBUDGET, before any launch, if that exceeds 64 MiB.
 * Every call on one GPU shares that GPU's array: calls that overlap on one
 * GPU (different streams or host threads) race and must be serialised by
 * the caller.  The context's own workspace is not touched.
 */
int design_greedy_noalloc(eig_ctx* ctx, int32_t nsample, int32_t ncand, const double* H1r,
                          const eig_prior* prior, const double* theta, const double* w,
                          int32_t kmax, int32_t* order, double* curve, void* stream);

/*
 * noise_sigma_peak — sigma = rel * max |u| over all free surface nodes
 * (i = 1..nx-2), both components and all levels, of the nominal solve at
 * theta (usually the prior mean).  Synchronous; writes *sigma_out (host).
 */
int noise_sigma_peak(eig_ctx* ctx, const eig_grid* grid, const eig_medium* medium,
                     const double* theta, int32_t stf_kind, double rel,
                     double* sigma_out, void* stream);

/*
 * sparse_grid_gl — sparse quadrature of Section 3.3.4 for a uniform prior on
 * the box [lo, hi] (host arrays [dim]): Smolyak combination of 1-D
 * Gauss-Legendre rules with m(i) = i points over the total-degree index set
 * sum_n (i_n - 1) <= level, coincident nodes merged.  Weights sum to one and
 * may be negative.  Host-only, synchronous.
 *   nodes: host [capacity][dim]; weights: host [capacity]; *count receives
 *   the number of nodes (EIG_EINVAL, with *count set, if capacity is short).
 *   dim in 1..16, level in 0..40.
 */
int sparse_grid_gl(int32_t dim, int32_t level, const double* lo, const double* hi,
                   int32_t capacity, double* nodes, double* weights, int32_t* count);

/*
 * Serving engine (continuous batching).  A server owns an HBM arena of
 * `budget` bytes.  Submitted queries run the work of jacobian_fd (one H_1
 * per sample, per_receiver = 0) followed by laplace_eig; their samples are
 * admitted in groups of `group_samples` whenever arena memory and descriptor
 * slots are free, and every stencil launch advances all admitted solves of
 * all queries by one step, so later queries overlap earlier ones on the
 * device.  Per-sample arithmetic is independent of the batch: a query's
 * outputs are identical whether it runs alone or in a mix.
 */
typedef struct eig_server eig_server;
int eig_server_create(eig_ctx* ctx, size_t budget, int32_t group_samples,
                      eig_server** out);
void eig_server_destroy(eig_server* srv);
/* Queue a query.  Host inputs are copied.  The medium's device arrays are
 * read when the query's sample groups are admitted, later, on the stream of
 * eig_server_step; they and the device outputs are caller-owned and must stay
 * valid until eig_server_poll reports the query done:
 *   H1 device [nsample][7][7], dkl device [nsample], eig device [1],
 *   status device [nsample] or NULL (0 / EIG_ENONFINITE),
 *   chol_status device [nsample] or NULL (0 / EIG_ENOTPD).
 * sigma_mode/sigma as for jacobian_fd (one value for all samples).
 * EIG_EBUDGET if one sample's group together with the query's laplace inputs
 * does not fit the arena (any query accepted here is admitted once the server
 * is idle: groups shrink to fit); EIG_EINVAL as for jacobian_fd; *id receives
 * a handle. */
int eig_server_submit(eig_server* srv, const eig_grid* grid, const eig_medium* medium,
                      int32_t nsample, const double* theta, double rel_step,
                      int32_t stf_kind, const eig_receivers* rec, int32_t sigma_mode,
                      double sigma, const eig_prior* prior, const double* w, double* H1,
                      double* dkl, double* eig, int32_t* status, int32_t* chol_status,
                      int64_t* id);
/* Enqueue up to max_launches stencil launches on `stream`, retiring finished
 * groups (Hessian kernels, then laplace for completed queries) and admitting
 * waiting ones at segment boundaries.  *running = admitted groups left.
 * EIG_EBUDGET (with *running = 0) if queries wait and none can be admitted. */
int eig_server_step(eig_server* srv, int32_t max_launches, void* stream, int32_t* running);
/* *done = 1 once query `id`'s outputs are complete on the device (the handle
 * is then released). */
int eig_server_poll(eig_server* srv, int64_t id, int32_t* done);
/* Queries still waiting for admission of samples, and admitted groups. */
int eig_server_pending(eig_server* srv, int32_t* queued, int32_t* running);
/* Arena accounting: the budget given at creation, the bytes admitted groups
 * and query inputs hold now, and the most they ever held (never above the
 * budget).  The slot and tile tables (about 16 MiB plus 8 bytes per
 * wavefront tile) are allocated beside the arena.  Any pointer may be NULL. */
int eig_server_memory(eig_server* srv, size_t* budget, size_t* in_use, size_t* peak);

#ifdef __cplusplus
}
#endif
#endif /* EIGSEIS_H */
