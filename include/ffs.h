/*
 * ffs.h -- C ABI of the MI355X (gfx950) fast fermion sampling library.
 *
 * The library draws configurations x = (x_1..x_N) of N distinct sites out of
 * L with probability |det U[x, :]|^2 / N!  (Eq. (1)), for a caller-supplied
 * L x N matrix U with orthonormal columns (U^H U = 1).  It follows the
 * paper's fast fermion sampling algorithm: a uniformly random column order m
 * per sample (Eq. (2)), then for k = 1..N the site x_k is drawn from the
 * conditional with weight |u_y^T h|^2 over free sites y, h being normal to
 * the rows already drawn (Eq. (3), SI S-1).  The marginal of the first
 * n_keep < N particles is the same process stopped after n_keep steps (the
 * marginal-sampling paragraph after Eq. (3)).
 *
 * Conventions shared by every entry point
 *  - Positions are 0-based site indices (the paper counts 1..L) and are
 *    returned in draw order; the law is over ordered tuples (the 1/N! of
 *    Eq. (1)), so the draw order is itself a valid sample.
 *  - Randomness: Philox4x32-10 (Salmon et al., SC'11), key = (seed lo, seed
 *    hi), counter = (sample lo, sample hi, step, 0), one block per (sample,
 *    step); words 0,1 pick the column (lazy Fisher-Yates, 64-bit
 *    multiply-high), words 2,3 give a 53-bit uniform u for the inverse-CDF
 *    draw over ascending sites.  x therefore depends only on (U, seed,
 *    sample index, bulk precision) -- not on how samples are split over
 *    calls or batched.
 *  - Device pointers are HIP device (or HIP-managed) memory; host pointers
 *    are ordinary host memory.  Outputs are caller-owned.  Work is enqueued
 *    on `hip_stream` (a hipStream_t; NULL = the null stream) and outputs are
 *    valid once the caller synchronises that stream; ffs_check() reports
 *    errors found on the device by the last call on a plan.
 *  - Every entry point returns an ffs_status; no C++ exception crosses the
 *    ABI.  On failure outputs are unspecified and ffs_last_error() returns a
 *    thread-local message.
 *  - A plan is immutable after creation; calls on different streams may run
 *    concurrently (each takes its own working memory).
 */
#ifndef FFS_H
#define FFS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ffs_plan_s* ffs_plan_t;

typedef enum {
  FFS_OK = 0,
  FFS_ERR_INVALID_ARG = -1,     /* bad shape, pointer or option           */
  FFS_ERR_NOT_ORTHONORMAL = -2, /* max |U^H U - 1| above options.ortho_tol */
  FFS_ERR_OUT_OF_MEMORY = -3,   /* device allocation failed / over budget  */
  FFS_ERR_HIP = -4,             /* a HIP runtime call failed               */
  FFS_ERR_NUMERICAL = -5,       /* NaN/Inf input, zero total weight or pivot */
  FFS_ERR_UNSUPPORTED = -6      /* size or mode this library does not handle */
} ffs_status;

/* Element type of the host matrix given to ffs_plan. */
typedef enum { FFS_REAL64 = 0, FFS_COMPLEX128 = 1 } ffs_dtype;

/* Precision of the all-site weight evaluation (the 2Lk inner products per
 * step of the main-text cost count).  FP64: exact to double rounding (plain
 * path only).  FP32: float operands and accumulation on the FP32 matrix
 * cores.  SPLIT_BF16 (batched path only): U and Gamma are each split into a
 * bfloat16 head and tail (head = bf16(x), tail = bf16(x - head)) and the
 * product is formed as head*head + head*tail + tail*head on the BF16 matrix
 * cores with float32 accumulation (weights within 1e-4 relative).  In
 * both reduced modes every draw whose uniform lands within the guard
 * threshold of a CDF boundary (ffs_options: guard_scale, guard_delta) is
 * redone from float64 weights, so the drawn sites are those of a float64
 * computation. */
typedef enum {
  FFS_BULK_FP64 = 0,
  FFS_BULK_FP32 = 1,
  FFS_BULK_SPLIT_BF16 = 2
} ffs_bulk;

/* When the draws the guard flags get their float64 sites (batched path;
 * the sites are the same in every mode).  PER_STEP: in the step that drew
 * them -- a float64 product of all flagged draws of the step and a redraw
 * before the factor update absorbs the draw, two more launches per step.
 * DEFERRED: the draw keeps its float32 site and is recorded (its float64
 * Gamma and the occupancy at that step); the draw and the factor update are
 * then one launch per step, and at the end of the call every record is
 * redone in float64 with the same u.  A sample none of whose recorded
 * draws moved followed the trajectory PER_STEP would have taken; a sample
 * with a moved site (or a record that found no slot) is replayed with
 * PER_STEP resolution and its row replaced (the replay batch takes working
 * memory of its own, sized by the number of replayed samples and kept with
 * the stream's working memory; hbm_budget does not cover it).  ffs_sample and ffs_marginal
 * calls in this mode wait for the device at the end of each batch (to learn
 * whether a replay is needed), so they are not stream-asynchronous and
 * cannot be captured into a graph; the other calls always resolve per step.
 * AUTO: DEFERRED for FP32 bulk with the adaptive guard alone
 * (guard_delta unset, guard_scale <= 8), where few draws are flagged,
 * until a call of the plan needs a replay (each costs a per-step run of
 * its samples: at L = 16384, N = 512 complex about 1.7% of samples move,
 * none at L = 4096, N = 256 real); from then on PER_STEP.  PER_STEP
 * otherwise (SPLIT_BF16 or a fixed margin can flag several percent of
 * draws) and on the plain path.  The choice changes speed only. */
typedef enum {
  FFS_RESOLVE_AUTO = 0,
  FFS_RESOLVE_PER_STEP = 1,
  FFS_RESOLVE_DEFERRED = 2
} ffs_resolve;

/* Execution path.  BATCHED: samples sharing U advance step by step together
 * and the per-step weights of all samples are one L x N x S contraction on
 * the matrix cores.  PLAIN: one kernel launch per sample, all N steps fused
 * (the paper's single-sample regime). */
typedef enum { FFS_PATH_BATCHED = 0, FFS_PATH_PLAIN = 1 } ffs_path;

typedef struct {
  int32_t bulk;        /* ffs_bulk, default FFS_BULK_FP32                      */
  int32_t path;        /* ffs_path, default FFS_PATH_BATCHED                   */
  double ortho_tol;    /* default 1e-10                                        */
  double guard_delta;  /* fixed relative CDF margin of the guard (a draw is
                          flagged when u*T lies within guard_delta * T of a
                          boundary of its site's interval); default -1 =
                          none.  Set alone (guard_scale left at -1) it
                          replaces the adaptive rule below; 1 flags every
                          draw (all sites from float64 weights)              */
  int64_t max_batch;   /* samples per internal batch, default 4096             */
  size_t hbm_budget;   /* max bytes of working memory per call, 0 = unlimited  */
  int32_t overlap;     /* default 1: a batch of >= 256 samples runs as two
                          halves on two streams so that the float64 factor
                          update of one overlaps the contraction of the
                          other; 0: one stream (results are identical)       */
  int32_t resolve;     /* ffs_resolve: when flagged draws are redone from
                          float64 weights; default FFS_RESOLVE_AUTO          */
  double guard_scale;  /* adaptive guard: a draw is flagged when its margin is
                          below guard_scale * 2^-24 * sqrt(K) * sqrt(sum_b
                          B_b^2), K = N (real) or 2N (complex), B_b the
                          float64 sums of the 32-site blocks of the step's
                          weights -- the float32 CDF error scale (per-weight
                          relative error ~2^-24 sqrt(K), independent over
                          sites).  Default -1 = the bulk mode's own: 2
                          (FP32), 32 (SPLIT_BF16), 0 (FP64); 0 = off.  The
                          threshold used is the larger of the two rules     */
} ffs_options;

/* Counters of the last completed call on a plan (see ffs_check). */
typedef struct {
  int64_t draws;       /* site draws performed                                */
  int64_t flagged;     /* draws whose margin was below the guard threshold    */
  int64_t changed;     /* flagged draws whose float64 redraw moved the site
                          (DEFERRED: counted on the recorded trajectory; a
                          replayed sample's own flags and changes are added
                          again by its replay)                              */
  int32_t device_status; /* 0 or an ffs_status raised on the device          */
  int32_t reserved;
} ffs_stats_t;

/* Fill *opt with the defaults listed above.  Never fails. */
void ffs_default_options(ffs_options* opt);

/*
 * Create a plan for U (Eq. (1)): validates 1 <= N <= L, ldu >= N, finite
 * entries and max|U^H U - 1| <= ortho_tol (exact check when L*N^2 <= 2^28,
 * otherwise a randomised check ||U^H U z - z||_inf over 4 Gaussian probes),
 * then copies U to the current HIP device in the layouts the kernels use.
 *   out    : receives the plan handle (NULL on failure)
 *   U_host : host, row-major L x N; element (i, j) at U_host[i*ldu + j],
 *            double (FFS_REAL64) or interleaved (re, im) doubles
 *            (FFS_COMPLEX128).  Not retained: the caller keeps ownership.
 *   opt    : NULL for defaults
 * Errors: INVALID_ARG, NOT_ORTHONORMAL, NUMERICAL (non-finite entry),
 *         UNSUPPORTED (N > 1024, L > 65536, FP64 bulk on the batched path,
 *         SPLIT_BF16 bulk or DEFERRED resolution on the plain path),
 *         OUT_OF_MEMORY, HIP.
 */
ffs_status ffs_plan(ffs_plan_t* out, const void* U_host, int64_t L, int64_t N,
                    int64_t ldu, int32_t dtype, const ffs_options* opt);

/* As ffs_plan with U in device memory (e.g. the output of ffs_dpp_eig):
 * U is copied to the host for the checks and the layout pass, then
 * uploaded.  U_dev: device, same layout as U_host.  Same errors. */
ffs_status ffs_plan_device(ffs_plan_t* out, const void* U_dev, int64_t L, int64_t N,
                           int64_t ldu, int32_t dtype, const ffs_options* opt);

/*
 * Draw n_samples configurations (Eq. (2) with Eq. (3)'s conditionals) for
 * sample indices first_sample .. first_sample + n_samples - 1.
 *   x_dev      : device int32 [n_samples][N], 0-based sites in draw order
 *   logdet_dev : device double [n_samples] or NULL; receives
 *                sum_k log w_k(x_k) = log|det U[x, :]|^2 (the product of the
 *                squared Schur pivots of the factor update)
 *   hip_stream : hipStream_t, stream-ordered semantics (with DEFERRED
 *                resolution the call also waits for each batch's work:
 *                see ffs_resolve)
 * n_samples = 0 is a no-op.  Errors: INVALID_ARG, OUT_OF_MEMORY, HIP;
 * device-side NUMERICAL is reported by ffs_check.
 */
ffs_status ffs_sample(ffs_plan_t p, uint64_t seed, uint64_t first_sample,
                      int64_t n_samples, int32_t* x_dev, double* logdet_dev,
                      void* hip_stream);

/*
 * Marginal of the first n_keep particles (the marginal paragraph after
 * Eq. (3)): the same process stopped after n_keep steps.  Bit-identical to
 * the first n_keep columns of ffs_sample with the same arguments.
 *   n_keep : 0..N (0 is a no-op)
 *   x_dev  : device int32 [n_samples][n_keep]
 */
ffs_status ffs_marginal(ffs_plan_t p, int64_t n_keep, uint64_t seed,
                        uint64_t first_sample, int64_t n_samples,
                        int32_t* x_dev, void* hip_stream);

/*
 * Allocation-free ffs_sample, for callers that cannot allocate device memory
 * (code under stream capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, results and errors as ffs_sample on a
 * batched-path plan, bit-identical to it; the working memory comes from a
 * fixed device array of FFS_NOALLOC_SCRATCH_BYTES per GPU inside the library
 * (held until the process ends), so the call makes no hipMalloc / hipFree.
 * Samples run in batches of the largest multiple of 128 whose working memory
 * fits that array, on the caller's stream alone, with per-step resolution of
 * flagged draws whatever the plan's ffs_resolve (the call never waits for
 * the device); the memory it must start from zero is cleared by a kernel
 * (no memset node).
 *   Errors: as ffs_sample, and UNSUPPORTED for a plain-path plan or when the
 *   working memory of one 128-sample batch exceeds the array (at L = 4096
 *   that allows N up to about 330 real or 230 complex); INVALID_ARG when the
 *   current device is not the plan's.
 * Every call on one GPU shares that GPU's array and it keeps the last call's
 * contents: calls that overlap on one GPU (on two streams, or from two host
 * threads) race and must not be issued.  ffs_check on the plan reports the
 * last allocation-free call on its GPU.
 */
#define FFS_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
ffs_status ffs_sample_noalloc(ffs_plan_t p, uint64_t seed, uint64_t first_sample,
                              int64_t n_samples, int32_t* x_dev, double* logdet_dev,
                              void* hip_stream);

/*
 * Per-sample column subsets: sample s draws k distinct sites with
 * probability |det U[x, J_s]|^2 / k!, i.e. Eq. (1) with U replaced by the
 * columns J_s = cols_dev[s][0..k) of the plan's U.  This is the projection
 * stage of sampling a determinantal point process from its
 * eigendecomposition (an eigenvector subset per sample, chosen beforehand,
 * e.g. by a fixed-size selection), with every sample's conditional weights
 * still formed by one contraction over U's N columns.  The column order of
 * sample s permutes the k positions of J_s (position c is column J_s[c]),
 * so the result equals ffs_sample on a plan of U[:, J_s] with the same seed
 * and sample index.  Batched-path plans; works with FP32 and SPLIT_BF16
 * bulk.
 *   k        : 1..N
 *   cols_dev : device int32 [n_samples][k], distinct columns in [0, N)
 *   x_dev    : device int32 [n_samples][k]; logdet_dev as in ffs_sample
 * Out-of-range or repeated columns are reported by ffs_check (INVALID_ARG).
 */
ffs_status ffs_sample_subsets(ffs_plan_t p, int64_t k, const int32_t* cols_dev,
                              uint64_t seed, uint64_t first_sample,
                              int64_t n_samples, int32_t* x_dev,
                              double* logdet_dev, void* hip_stream);

/*
 * Metropolis conditional update (SI S-7), the variant for large L: the same
 * column order and float64 conditioning as ffs_sample, but x_t is drawn by
 * m_cond Metropolis iterations on the single variable x_t (target weight
 * |v_t(y)|^2, occupied sites 0, acceptance min(1, w(y)/w(c))) instead of
 * the all-site weights, so a sample costs O(m_cond N^2 + N^3), free of L.
 * The chain starts at the anchor of column m_t (the first row of largest
 * |U[., m_t]|^2, found when the plan is made); proposals are (radius > 0)
 * c + d with d uniform in [-radius, -1] u [1, radius] modulo L, or
 * (radius == 0) uniform over the L sites.  Iteration j of step t of sample s
 * draws from the Philox block (seed, s, t, 2 + j): words 0,1 the proposal
 * (multiply-high), words 2,3 the 53-bit u, accepted when u w(c) < w(y).  A
 * chain that ends on a site of weight 0 moves to the nearest free site of
 * positive weight (lower side first).  The draws are exact only as m_cond
 * grows (a Markov chain per conditional) and local moves need orbitals whose
 * weight is connected; the oracle runs the same chain.
 *   m_cond       : iterations per step (>= 0)
 *   radius       : 0 for global proposals, else the local step bound (<= L/2)
 *   x_dev        : device int32 [n_samples][N];  logdet_dev as in ffs_sample
 *   accepted_out : host, accepted proposals of the call, or NULL (non-NULL
 *                  synchronises the stream)
 * ffs_check reports the device status (NUMERICAL if a chain found no site
 * of positive weight).  Errors: INVALID_ARG, OUT_OF_MEMORY, HIP.
 */
ffs_status ffs_sample_mh(ffs_plan_t p, int32_t m_cond, int32_t radius, uint64_t seed,
                         uint64_t first_sample, int64_t n_samples, int32_t* x_dev,
                         double* logdet_dev, int64_t* accepted_out, void* hip_stream);

/* ---------------------------------------------------- DPP front end ----
 * The paper's subset-selection application (the text-summarisation part of
 * its applications section): items i = 1..L carry feature vectors b_i (the
 * rows of B, quality folded into their norms), the DPP kernel is
 * C = B B^T, and a draw first keeps each eigenvector u_j of C with
 * probability lambda_j / (lambda_j + 1), then samples the items as fermions
 * in the kept eigenvectors (Eq. (1) with U = the kept columns).  These calls
 * do the first part on the device; the second is ffs_sample_subsets on a
 * plan of all d eigenvectors (ffs_plan_device).
 */

/*
 * Eigenpairs of C = B B^T through its d x d dual B^T B (same nonzero
 * eigenvalues; u_j = B w_j / sqrt(lambda_j)), all in float64 on the device:
 * dual product, cyclic Jacobi in one workgroup, ascending order, each w_j
 * signed so that its largest-magnitude entry is positive, projection.
 *   B_dev      : device, row-major L x d float64 (d <= L, d <= 512)
 *   lambda_dev : device float64 [d], eigenvalues ascending
 *   U_dev      : device, row-major L x d float64: column j = u_j (orthonormal)
 *   W_dev      : device d x d float64 dual eigenvectors (column j = w_j), or NULL
 *   sweeps_out : host, Jacobi sweeps run, or NULL
 * Synchronises the stream.  Errors: INVALID_ARG, UNSUPPORTED (d > 512),
 * NUMERICAL (no convergence in 60 sweeps, or lambda_min <= 1e-12 lambda_max:
 * B must have full column rank), HIP.
 */
ffs_status ffs_dpp_eig(const double* B_dev, int64_t L, int64_t d, double* lambda_dev,
                       double* U_dev, double* W_dev, int32_t* sweeps_out,
                       void* hip_stream);

/*
 * Eigenvector selection of the DPP (applications section): sample
 * s = first_sample + i keeps eigenvector j when u < lambda_j / (lambda_j + 1),
 * u the 53-bit uniform of the Philox block keyed (seed, s, step = j) with
 * counter word 3 = 1 (a stream disjoint from the sampler's).
 *   lambda_dev : device float64 [d] (>= 0)
 *   cols_dev   : device int32 [n][d]: kept indices ascending, then -1
 *   sizes_dev  : device int32 [n]: number kept
 * Stream-ordered.  Errors: INVALID_ARG, UNSUPPORTED (d > 65536).
 */
ffs_status ffs_dpp_subsets(const double* lambda_dev, int64_t d, uint64_t seed,
                           uint64_t first_sample, int64_t n, int32_t* cols_dev,
                           int32_t* sizes_dev, void* hip_stream);

/*
 * Fixed-size (k-DPP) eigenvector selection: subset J, |J| = k, drawn with
 * probability prod_{j in J} lambda_j / e_k(lambda) by the elementary
 * symmetric polynomial scan (Kulesza and Taskar's DPP review): j runs from
 * d-1 down, and with l indices still to take j is kept when
 * u_j < mu_j e_{l-1}(mu_<j) / e_l(mu_<=j), mu = lambda / max(lambda), u_j the
 * uniform of the block (seed, s, step = j, word 3 = 1) as above.
 *   cols_dev : device int32 [n][k], ascending
 * Synchronises the stream (table check).  Errors: INVALID_ARG,
 * UNSUPPORTED, NUMERICAL (negative eigenvalue or e_k out of float64 range).
 */
ffs_status ffs_kdpp_subsets(const double* lambda_dev, int64_t d, int64_t k, uint64_t seed,
                            uint64_t first_sample, int64_t n, int32_t* cols_dev,
                            void* hip_stream);

/*
 * Sampling stage of the DPP with per-sample subset sizes (the output of
 * ffs_dpp_subsets): sample s = first_sample + i draws sizes[i] sites with
 * probability |det U[x, J]|^2 / |J|!, J = cols[i][0..sizes[i]), exactly as
 * ffs_sample_subsets would for that one sample with k = sizes[i] (same
 * seed, same sample index).  Samples are grouped by size on the host (the
 * sizes are read back, which synchronises the stream) and each group runs
 * as one column-subset batch keyed by its samples' own indices; the groups
 * run round-robin on hip_stream and three streams of the plan (forked from
 * and joined back into hip_stream), so the call's work is ordered on
 * hip_stream as usual; each of the four streams keeps its own column-subset
 * working memory in the plan (sized by the largest group it ran).  Calls
 * on one plan from several threads run one after another on the host.
 *   cols_dev  : device int32 [n][N] (N = the plan's column count)
 *   sizes_dev : device int32 [n], each in [0, N]
 *   x_dev     : device int32 [n][N]: the draws, then -1
 *   logdet_dev: device float64 [n] or NULL (0 for an empty subset)
 * ffs_check reports the draws, guard counters and device status of the
 * whole call.  Errors: INVALID_ARG (sizes out of range), OUT_OF_MEMORY, HIP.
 */
ffs_status ffs_sample_dpp(ffs_plan_t p, const int32_t* cols_dev, const int32_t* sizes_dev,
                          uint64_t seed, uint64_t first_sample, int64_t n_samples,
                          int32_t* x_dev, double* logdet_dev, void* hip_stream);

/* ---------------------------------------------- Slater-Jastrow reweighting
 * SI S-5, Eq. (S8): draws x of the free-fermion ensemble |psi_0(x)|^2 give
 * expectations in psi_J = J psi_0 as <O> = <J^2 o_L>_0 / <J^2>_0.  A
 * configuration is a pair (x_up[s], x_dn[s]) of rows of draws (e.g. two
 * ffs_sample calls; -1 = empty slot; distinct sites within a row).  With
 * D(x) = number of sites holding both spins and n_i = n_i,up + n_i,dn:
 *   log J^2(x) = -V D(x) - sum_{i,j} v_ij n_i n_j + extra[s]
 * (V: the Gutzwiller factor of the main text; v: the general density
 * Jastrow of SI S-5, or NULL; extra: a caller's per-sample log-weight, e.g.
 * a difference of logdet outputs, or NULL).  Observables are diagonal, so
 * o_L is their value: the site densities and the double occupancy.
 *   x_up_dev   : device int32 [n][k_up];  x_dn_dev: [n][k_dn] (k_dn = 0: spinless)
 *   vmat_dev   : device float64 [L][L] or NULL;  extra_logw_dev: [n] or NULL
 *   logw_dev   : out, device float64 [n]: log J^2(x_s) (+ extra)
 *   density_dev: out, device float64 [L]: <n_i>_J
 *   summary_dev: out, device float64 [6]: <D>_J, <D>_0, sum w, sum w^2,
 *                effective sample size (sum w)^2 / sum w^2, shift m, with
 *                w_s = exp(logw_s - m), m = max_s logw_s
 * With v and L <= 16 (k_up + k_dn) the pair term is computed as one
 * product of the per-sample site counts with v on the FP64 matrix cores
 * (samples in chunks whose counts take at most 256 MB of stream-ordered
 * working memory); otherwise from the (k_up + k_dn)^2 entries of v of each
 * configuration.  Fixed summation order (deterministic).  Synchronises the
 * stream.  Errors: INVALID_ARG (bad sizes, non-finite V, a site outside
 * [-1, L)), UNSUPPORTED (L > 65536, n > 2^24), HIP.
 */
ffs_status ffs_jastrow_estimate(const int32_t* x_up_dev, int64_t k_up,
                                const int32_t* x_dn_dev, int64_t k_dn, int64_t n_samples,
                                int64_t L, double V, const double* vmat_dev,
                                const double* extra_logw_dev, double* logw_dev,
                                double* density_dev, double* summary_dev, void* hip_stream);

/* Wait for the last call enqueued on the plan and return its device-side
 * status (FFS_OK, FFS_ERR_NUMERICAL, or FFS_ERR_INVALID_ARG for a bad column
 * subset); *stats (nullable) receives its
 * counters.  Blocks the host. */
ffs_status ffs_check(ffs_plan_t p, ffs_stats_t* stats);

/* Release the plan and its device memory (waits for its pending work). */
ffs_status ffs_destroy(ffs_plan_t p);

/* Thread-local description of the last failure on this thread. */
const char* ffs_last_error(void);

/*
 * Test hook (Eq. (3) weights): the normalised conditional w over all L sites
 * at step k (1-based) of sample `sample`, with the first k-1 sites forced to
 * prefix_host[0..k-2] (host int32) and the sample's own column order.  The
 * weights are evaluated by the plan's bulk path (batched contraction) and
 * normalised by their float64 total.  Synchronous.
 *   w_host : host double [L]
 */
ffs_status ffs_conditional(ffs_plan_t p, uint64_t seed, uint64_t sample,
                           int64_t k, const int32_t* prefix_host,
                           double* w_host);

/* Site marginals diag(U U^H) (sum = N), evaluated on the device from the
 * plan's bulk-precision copy with float64 accumulation.  Synchronous.
 *   rho_host : host double [L] */
ffs_status ffs_density(ffs_plan_t p, double* rho_host);

/*
 * Contraction tile autotuner: times every tile variant of the float32
 * contraction on the launch shapes a call of n_samples on this plan uses
 * and records the fastest for each shape (sites, contraction columns,
 * samples per launch, complex); later launches of that shape use it
 * (otherwise 128 sites x 128 columns).  The variants tile sites and samples
 * differently but reduce over K in the same order, so results are
 * bit-identical whichever is chosen.  If the environment variable
 * FFS_TUNE_FILE names a file, the table is read from it on first use and
 * rewritten after each tuning (JSON).  Synchronous.
 *   flags      : 0 = time each variant's contraction launches alone;
 *                FFS_TUNE_PIPELINE = time a short sampling call (the first
 *                32 steps of n_samples) per variant, so the choice accounts
 *                for the work that overlaps the contraction
 *   choice_out : nullable host char[32]; receives "<sites>x<columns>" (or
 *                "<sites>x<columns>k16" for a 16-wide K chunk) of the first
 *                shape's choice
 */
enum { FFS_TUNE_PIPELINE = 1 };
ffs_status ffs_autotune(ffs_plan_t p, int64_t n_samples, int32_t flags,
                        char* choice_out);

/* Record a tile choice by hand for the launch shapes of a call of n_samples
 * (tuning and test hook).  Tiles (sites x columns): 128x128, 64x128 (real
 * and complex), 128x64, 64x64 (real); kchunk: the K chunk staged through
 * LDS per barrier, 32 (0 = default) or 16 (half the LDS, so twice the
 * workgroups per CU).  The tuner reports a 16-wide choice as "SxCk16".
 * Errors: INVALID_ARG for other tiles. */
ffs_status ffs_set_tile(ffs_plan_t p, int64_t n_samples, int32_t sites,
                        int32_t cols, int32_t kchunk);

/* Kernel classes reported by ffs_kernel_times. */
typedef enum {
  FFS_K_FACTOR = 0,   /* float64 factor update + solve, one per step       */
  FFS_K_WEIGHTS = 1,  /* batched all-site weight contraction, one per step */
  FFS_K_DRAW = 2,     /* inverse-CDF draw + guard, one per step            */
  FFS_K_REPAIR = 3,   /* float64 redraw of guarded draws, one per step     */
  FFS_K_PLAIN = 4,    /* plain path, one per sample                        */
  FFS_K_FACTOR_BLOCK = 5, /* factor launches that close a 16-step block      */
  FFS_K_COUNT = 6
} ffs_kernel_class;

/* Measurement hook: when enabled (enable != 0), every kernel launch the
 * plan issues is bracketed by a pair of HIP events recorded on the same
 * stream -- except the batched contraction (FFS_K_WEIGHTS), whose pair the
 * launch itself records around its dispatch (hipExtLaunchKernelGGL), so it
 * leaves out the wait behind the stream's previous kernel.  ffs_kernel_times
 * waits for them and returns, per kernel class, the summed device time in
 * milliseconds (ms[FFS_K_COUNT], host) and the number of launches
 * (launches[FFS_K_COUNT], host, nullable), then clears the record.
 * Disabled by default; adds two events per launch. */
ffs_status ffs_set_timing(ffs_plan_t p, int32_t enable);
ffs_status ffs_kernel_times(ffs_plan_t p, double* ms, int64_t* launches);

/* Second measurement of the timed contraction launches: each records its
 * own span on the device's steady clock (the earliest start among its first
 * workgroups to the latest workgroup end), which leaves out the dispatch and
 * any wait for CUs held by other streams' kernels.  Returns the summed span
 * in milliseconds (*ms, host) and the launch count (*launches, host,
 * nullable) since the last read, then clears them.  Records at most 65536
 * launches between reads (later ones are not recorded). */
ffs_status ffs_kernel_spans(ffs_plan_t p, double* ms, int64_t* launches);

/* As ffs_set_timing, but brackets only the launches of the classes whose
 * bit (1 << class) is set in class_mask; 0 disables timing.  Fewer event
 * pairs disturb a timed run less.  Errors: INVALID_ARG for bits beyond
 * FFS_K_COUNT. */
ffs_status ffs_set_timing_classes(ffs_plan_t p, uint32_t class_mask);

/* Brackets only one launch in every `stride` launches of each timed class
 * (counted per class from this call; 1, the default, times every launch),
 * so that a long run can be sampled with few event pairs: each pair leaves
 * the GPU idle for a few microseconds around its launch.  The stamp spans
 * of ffs_kernel_spans follow the same selection.  Errors: INVALID_ARG
 * (NULL plan, stride < 1). */
ffs_status ffs_set_timing_stride(ffs_plan_t p, int32_t stride);

/* ------------------------------------------------------- grouped runs ----
 * Many instances -- each an ffs_marginal / ffs_sample call on its own plan,
 * with its own L, N, sample count and n_keep -- advance step by step in
 * lockstep: every phase of a step (contraction, draw, float64 redraw, factor
 * update) is one launch covering the work of all instances, each block
 * taking work items across instances.  Each instance's current step lives
 * in device memory and is advanced on the device, so with FFS_GROUP_GRAPH a
 * captured hipGraph of several steps is replayed until the longest instance
 * has finished (finished instances skip their items).  Results are
 * bit-identical to the separate calls.  Batched-path plans (FP32 or
 * SPLIT_BF16 bulk, resolving flagged draws per step whatever their
 * ffs_resolve) on the current device; every instance runs as one batch
 * (1 <= n_samples <= the plan's max_batch).
 *   inst  : host array [n_inst]
 *   flags : FFS_GROUP_GRAPH to replay a captured graph, 0 for direct launches
 *   stats : nullable host array [n_inst]; when given the call waits for the
 *           group and fills each instance's counters (see ffs_check)
 * Stream-ordered on hip_stream like ffs_sample (the group runs on an
 * internal stream joined to it).  Errors: INVALID_ARG, UNSUPPORTED,
 * OUT_OF_MEMORY, HIP; device-side NUMERICAL via stats[i].device_status. */
typedef struct {
  ffs_plan_t plan;
  int64_t n_keep;        /* 1..N                                            */
  uint64_t seed;
  uint64_t first_sample;
  int64_t n_samples;
  int32_t* x_dev;        /* device int32 [n_samples][n_keep]                */
  double* logdet_dev;    /* device double [n_samples] or NULL (n_keep = N)  */
} ffs_instance;

enum { FFS_GROUP_GRAPH = 1 };

ffs_status ffs_sample_group(const ffs_instance* inst, int32_t n_inst,
                            int32_t flags, ffs_stats_t* stats,
                            void* hip_stream);

/* ------------------------------------------------------------ serving ----
 * A request server: sampling requests (each an ffs_sample / ffs_marginal
 * call on some plan) are submitted from any host thread and a scheduler
 * thread admits them first fit over the queue -- as soon as there is room
 * and the request's working memory fits what is left of the HBM budget, so
 * a small request can start while a large one waits for memory.  Requests
 * that arrive while others run are admitted while those keep running, and
 * their device work overlaps.  Two execution modes:
 *   FFS_SERVE_GROUPED (default): continuous batching.  Running requests are
 *     instances of one resident group (see ffs_sample_group) that advances
 *     in rounds of `ticks` lockstep steps, one launch per phase for all of
 *     them; between rounds, finished requests retire and queued ones join
 *     (up to `capacity` at once), each at its own step.  FP32-bulk plans,
 *     n_samples <= the plan's max_batch.
 *   FFS_SERVE_STREAMS: each running request has its own stream (`slots` of
 *     them) and runs its whole step loop there.
 * Each request allocates its working memory stream-ordered at admission and
 * frees it when done; plans (U in its device layouts) stay resident.  A
 * request's result is bit-identical to the same ffs_sample / ffs_marginal
 * call made alone (the sampler's output depends only on U, seed, sample
 * index and bulk mode).  Batched-path plans on the server's device only; a
 * plan must outlive the requests that use it. */
typedef enum { FFS_SERVE_GROUPED = 0, FFS_SERVE_STREAMS = 1 } ffs_serve_mode;

typedef struct ffs_server_s* ffs_server_t;

typedef struct {
  int32_t mode;        /* ffs_serve_mode, default FFS_SERVE_GROUPED            */
  int32_t slots;       /* STREAMS: concurrent requests (streams), default 4, 1..32 */
  size_t hbm_budget;   /* bytes of request working memory admitted at once;
                          0 = half of the device memory free at creation      */
  int32_t capacity;    /* GROUPED: requests stepping together, default 128, 1..1024 */
  int32_t ticks;       /* GROUPED: lockstep steps per round, default 8, 1..256 */
} ffs_server_options;

typedef enum {
  FFS_REQ_QUEUED = 0,
  FFS_REQ_RUNNING = 1,
  FFS_REQ_DONE = 2
} ffs_request_state;

typedef struct {
  int32_t state;       /* ffs_request_state                                    */
  int32_t status;      /* ffs_status of the request, valid once DONE           */
  double t_submit;     /* seconds on the server's clock (steady, from creation) */
  double t_admit;      /* admission (slot and memory granted); 0 while queued  */
  double t_done;       /* the request's last device work finished              */
  int64_t draws;       /* n_samples * n_keep                                   */
  int64_t flagged;     /* guard statistics of the request (see ffs_check)     */
  int64_t changed;
} ffs_request_info;

void ffs_server_default_options(ffs_server_options* opt);

/* Create a server on the current HIP device.  opt: NULL for defaults.
 * Errors: INVALID_ARG, HIP, OUT_OF_MEMORY. */
ffs_status ffs_server_create(ffs_server_t* out, const ffs_server_options* opt);

/* Queue ffs_marginal(p, n_keep, seed, first_sample, n_samples, x_dev) (with
 * logdet_dev as in ffs_sample when n_keep = N; NULL otherwise) and return
 * its ticket.  x_dev: device int32 [n_samples][n_keep], written
 * asynchronously on the server's own streams, which do not wait for work
 * the caller has pending elsewhere: x_dev must be ready to be written when
 * submitted.  Valid once ffs_server_poll reports DONE.  Never blocks on the
 * device.  Errors: INVALID_ARG (bad plan, path or sizes),
 * OUT_OF_MEMORY (the request alone exceeds the budget). */
ffs_status ffs_server_submit(ffs_server_t s, ffs_plan_t p, int64_t n_keep,
                             uint64_t seed, uint64_t first_sample,
                             int64_t n_samples, int32_t* x_dev,
                             double* logdet_dev, uint64_t* ticket);

/* Wait up to timeout_ms (0 = just look, < 0 = until done) for a request and
 * fill *info (nullable).  Once a DONE state has been returned the ticket is
 * released and later polls of it fail with INVALID_ARG. */
ffs_status ffs_server_poll(ffs_server_t s, uint64_t ticket, int32_t timeout_ms,
                           ffs_request_info* info);

/* Stop admitting, wait for running requests, drop queued ones and release
 * the server's streams. */
ffs_status ffs_server_destroy(ffs_server_t s);

/* Host-side Philox block for (seed, sample, step) in the stream layout
 * above (test hook; no device work).  out: host uint32 [4]. */
void ffs_philox_words(uint64_t seed, uint64_t sample, uint32_t step,
                      uint32_t* out);

#ifdef __cplusplus
}
#endif

#endif /* FFS_H */
