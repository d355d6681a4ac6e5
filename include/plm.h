/*
 * plm.h -- C ABI of libplm, an MI355X (gfx950) implementation of asymmetric
 * l2-regularised pseudolikelihood maximisation for direct-coupling analysis
 * (asymmetric plmDCA: Ekeberg, Hartonen & Aurell, "Fast pseudolikelihood
 * maximization for direct-coupling analysis of protein structure from many
 * homologous amino-acid sequences", arXiv:1401.4832).
 *
 * The calls follow the method's rundown (sec. 3.4): reweight the alignment,
 * evaluate or minimise the N per-site objectives, then score the couplings.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Pointers named *_dev, and every array argument unless stated otherwise,
 *    are DEVICE pointers on the context's device, owned by the caller.  The
 *    library never allocates device memory; scratch space comes from a
 *    caller-provided workspace whose size the matching *_workspace_bytes call
 *    returns (any 256-byte-aligned device buffer of at least that size).
 *  - Arrays are C row-major:
 *      msa  uint8  [B][N]        symbols 0..q-1 (20 = gap for q = 21)
 *      w    double [B]           sequence weights; beff: one double
 *      h    float  [N][q]        h[r][s] = h_r(s)
 *      J    float  [N][N][q][q]  J[r][i][k][s] = J^{(r)}_{ri}(s,k): coupling of
 *                                state s at site r with state k at site i, as
 *                                seen by the site-r problem.  The self blocks
 *                                J[r][r] take no part in any result (they
 *                                must be finite: the input check covers the
 *                                whole array) and are zero on output.
 *  - Objective scale: f_r = B_eff * g_r^reg (eq. g_regdef2 multiplied by B_eff);
 *    gradients are of f_r.  Convergence tolerances are on the paper's
 *    normalised scale g_r^reg = f_r / B_eff.
 *  - lambda_J is the symmetric-model strength; the per-site problems use
 *    lambda'_J = 0.5 * lambda_J (sec. 3.4 step 1).
 *  - Supported sizes: 2 <= q <= 21, N >= 2, B >= 1, N * q <= 65535.
 *  - Calls enqueue work on the context's HIP stream and return without
 *    waiting, except plm_fit, plm_fit_batch and plm_sync, which synchronise.
 *    Errors detected on the device (a symbol >= q) are reported by the next
 *    synchronising call.  A context is not thread-safe; use one per stream.
 *  - Status codes: PLM_OK (0); PLM_W_MAXITER (+1, results written, some site
 *    stopped at the iteration cap: see its stats); negative values are errors
 *    after which outputs are unspecified.
 */
#ifndef PLM_H
#define PLM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PLM_OK 0
#define PLM_W_MAXITER 1
#define PLM_E_INVALID -1     /* null pointer, bad size, theta outside [0,1], lambda < 0 */
#define PLM_E_SYMBOL -2      /* an alignment symbol >= q (detected on the device) */
#define PLM_E_NONFINITE -3   /* a non-finite value in an input */
#define PLM_E_WORKSPACE -4   /* workspace missing, misaligned or too small */
#define PLM_E_HIP -5         /* a HIP runtime error; plm_last_error() has the text */
#define PLM_E_UNSUPPORTED -6 /* device is not gfx950, or an option not built */

/* Objective/gradient evaluation paths.  All reduce objectives and gradients
 * over sequences in FP64.  The optimiser (plm_fit and its variants) takes its
 * dot products, small matrices, objective and the gradient at the trial point
 * in FP64; the iterate and trial point are FP32 (the values the evaluation
 * kernels read), and the stored curvature pairs (s, y), the gradient kept at
 * the iterate and the search direction are FP32 unless
 * plm_fit_opts.history_fp64 asks for FP64 pairs and gradient copy.  The one-hot matrix
 * X[b][(i,k)] = [sigma_i^b = k] is exact in BF16; the MFMA paths split the
 * other operand (the couplings W_r[(i,k)][s] = J_ri(s,k) in the forward, the
 * residuals R_b(s) in the backward) into BF16 pieces and accumulate in FP32. */
#define PLM_PATH_GATHER_FP32 0 /* energies by LDS gather, coupling gradient by a symbol-sorted
                                  LDS scatter; FP32 arithmetic */
#define PLM_PATH_MFMA_BF16X2 1 /* both directions as MFMA products with hi/lo (two-piece)
                                  operands: 16 significant bits, relative error <= 2^-16 per
                                  coupling and residual (precision/speed trade-off) */
#define PLM_PATH_GATHER_MFMA_FP32 2 /* energies by LDS gather; coupling gradient as an MFMA
                                  product with three-piece residuals (24 significant bits, the
                                  FP32 significand) */
#define PLM_PATH_MFMA_FP32 3   /* both directions as MFMA products with three-piece operands */
#define PLM_PATH_GATHER_MFMA_F16X2 4 /* energies by LDS gather; coupling gradient as an MFMA
                                  product with FP16 hi/lo pieces of R * 2^12 (22 significant
                                  bits: |dR| <= 2^-22 |R|; the scaling keeps the low piece out
                                  of the FP16 subnormal range) */
#define PLM_PATH_GATHER_MFMA_I8X3 5 /* energies by LDS gather; coupling gradient as an int8 MFMA
                                  product with R in fixed point: round(R * 2^22) as three signed
                                  int8 digits (|dR| <= 2^-23, absolute; |R| <= w_b <= 1),
                                  accumulated exactly in int32; at most 2^24 - 1 sequences
                                  (PLM_E_UNSUPPORTED beyond) */
#define PLM_PATH_MFMA_I8X3 6   /* both directions as int8 MFMA products in fixed point: the
                                  gradient of path 5, and energies from each site's couplings
                                  scaled by a power of two 2^k_r with max|J_r| 2^k_r in
                                  [2^21, 2^22) and rounded (|dJ| <= 2^-22 max_i,s,k |J_ri(s,k)|),
                                  three int8 digits accumulated exactly in int32; at most
                                  2^24 - 1 sequences */
#define PLM_PATH_GATHER64_MFMA_I8X6 7 /* the precise path: energies accumulated in FP64 by the LDS
                                  gather, FP64 log-softmax and residuals; coupling gradient as two
                                  passes of the int8 MFMA product of path 5, over round(R * 2^22)
                                  and over the remainder's round((R * 2^22 - v) * 2^22), so R is
                                  carried to 2^-45 absolute and summed exactly (FP64-class
                                  results; slower than path 5; at most 2^24 - 1 sequences) */

typedef struct plm_ctx plm_ctx;

/* Create a context bound to `device` and to the HIP stream `hip_stream`
 * (a hipStream_t; NULL = the null stream).  Fails with PLM_E_UNSUPPORTED on a
 * device that is not gfx950.  The context holds host state and a few bytes of
 * pinned host memory for device-to-host status flags. */
int plm_ctx_create(plm_ctx **out, int device, void *hip_stream);
int plm_ctx_destroy(plm_ctx *ctx);
/* Text of the last error seen by this context (never NULL). */
const char *plm_last_error(const plm_ctx *ctx);
const char *plm_status_string(int status);
/* Wait for the context's stream and report deferred device-side errors. */
int plm_sync(plm_ctx *ctx);

/* ---- Reweighting (sec. 3.1, eq. inverse_weights; sec. 3.4 step 2) --------
 * m_b = #{a : id(a,b)/N >= theta} where id counts columns with equal symbols
 * (gap equal to gap counts); the row itself is counted, so m_b >= 1.
 * w_b = 1/m_b (correctly rounded FP64 division) and B_eff = sum_b w_b added in
 * index order.  Integer counting makes m, w and B_eff exactly reproducible.
 * uniform != 0 sets w_b = 1, B_eff = B (no similarity counting).
 * Outputs (device): m_out int32[B], w_out double[B], beff_out double[1].
 * No workspace. */
int plm_reweight(plm_ctx *ctx, const uint8_t *msa, int32_t B, int32_t N, int32_t q,
                 double theta, int32_t uniform, int32_t *m_out, double *w_out,
                 double *beff_out);

/* ---- Objective and gradient (sec. 3.4 step 3: eqs. g_regdef2, g_gradh2,
 * g_gradJ2), all listed sites at once ---------------------------------------
 * sites: device int32[n_sites] of distinct site indices, or NULL for all N
 * (then n_sites is ignored).  An index outside [0, N) is evaluated as site 0
 * and reported as PLM_E_INVALID by the next plm_sync.  Outputs are indexed by site; only the rows of
 * listed sites are written:
 *   f_out  double[N]          f_r = B_eff * g_r^reg
 *   gh_out float [N][q]       d f_r / d h_r(s)
 *   gJ_out float [N][N][q][q] d f_r / d J_ri(s,k) at [r][i][k][s]; zero for i == r
 * gh_out / gJ_out may be NULL to skip the gradient (with gJ_out NULL the
 * scatter kernel is not run at all).  grad_scale (device double[N], may be
 * NULL) multiplies the gradient rows of site r by grad_scale[r]: the
 * vector-Jacobian product an automatic-differentiation backward needs.  path
 * is one of PLM_PATH_*.  beff is a device pointer (as written by
 * plm_reweight). */
size_t plm_objgrad_workspace_bytes(int32_t B, int32_t N, int32_t q, int32_t path);
int plm_objgrad(plm_ctx *ctx, const uint8_t *msa, int32_t B, int32_t N, int32_t q,
                const double *w, const double *beff, const float *h, const float *J,
                double lambda_h, double lambda_J, const int32_t *sites, int32_t n_sites,
                int32_t path, void *workspace, size_t workspace_bytes,
                const double *grad_scale, double *f_out, float *gh_out, float *gJ_out);

/* ---- Objective and gradient without a workspace ----------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, serving loops, harnesses that forbid allocation.  plm_objgrad
 * (same arguments, results and stream semantics, same kernels) with its
 * scratch in a fixed device array of PLM_STATIC_SCRATCH_BYTES per GPU, which
 * the library holds from the first plm_ctx_create on that GPU until the
 * process ends; the call allocates nothing.  Problems whose
 * plm_objgrad_workspace_bytes exceeds the array are rejected with
 * PLM_E_WORKSPACE (at q = 21, 64 MiB holds N = 20 with B up to 33 700,
 * N = 40 with B up to 15 300, N = 60 with B up to 8 000).  Every call on a GPU shares that GPU's
 * array: calls ordered on one stream are safe, calls that overlap on one GPU
 * (other streams or contexts, other threads) race.  The array keeps the last
 * call's contents; an evaluation writes every scratch byte before it reads it,
 * so nothing needs clearing between calls. */
#define PLM_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
int plm_objgrad_static(plm_ctx *ctx, const uint8_t *msa, int32_t B, int32_t N, int32_t q,
                       const double *w, const double *beff, const float *h, const float *J,
                       double lambda_h, double lambda_J, const int32_t *sites, int32_t n_sites,
                       int32_t path, const double *grad_scale, double *f_out, float *gh_out,
                       float *gJ_out);

/* ---- Minimisation of every site (sec. 3.4 step 3) --------------------------
 * One limited-memory BFGS state per site, all sites advanced together on the
 * device; one replay of the captured iteration graph evaluates the trial
 * point of every active site and takes each site's line-search decision.
 * Starts from (h_io, J_io) -- zero gives the paper's cold start (sec. 6) --
 * and leaves the minimiser there.  A site stops when ||grad g_r^reg||_2 <= tol
 * (normalised scale), at max_iter, or on line-search failure. */
typedef struct {
  double lambda_h;      /* 0.01 */
  double lambda_J;      /* 0.01 (lambda'_J = lambda_J / 2) */
  double tol;           /* 1e-6 */
  int32_t max_iter;     /* per site; 2000 */
  int32_t lbfgs_m;      /* history pairs, 1..32; 10 */
  int32_t max_linesearch; /* backtracking steps before a history reset; 20 */
  int32_t path;         /* PLM_PATH_* */
  int32_t sync_every;   /* graph replays between host checks of the active count; 8 */
  int32_t use_graph;    /* 1: capture one iteration in a hipGraph; 0: eager launches */
  int32_t single_site;  /* 1: the plain path -- one site per launch, eager, no graph */
  int32_t tile_seqs;    /* forward tile rows per wave (16/32/64); 0 = default */
  int32_t site_limit;   /* single_site only: fit sites 0..site_limit-1 (0 = all) */
  int32_t timing;       /* 1: launch the iteration eagerly (no graph) with HIP events
                           between the kernels on the fit's stream, synchronise every
                           iteration, and keep the kernel times: plm_fit_last_timing */
  int32_t refine;       /* a second fit from the first one's point, to refine_tol (0: the
                           same tolerance), on another evaluation path: 0 = automatic
                           (after PLM_PATH_MFMA_I8X3, whose rounded couplings move the
                           gradient by up to about 1e-6 in norm at N = 500, refine on
                           PLM_PATH_GATHER_MFMA_I8X3, whose gradient is within the FP32
                           tolerance; after PLM_PATH_MFMA_BF16X2, whose 16-bit operands
                           leave a gradient error far above 1e-6, refine on
                           PLM_PATH_MFMA_FP32; nothing after other paths), -1 = never,
                           1 + p = always, on path p.  Site statistics and timing add both
                           fits.  With a noisy first path, give the first fit a tolerance
                           above its rounding floor (tol) and the refinement the target
                           (refine_tol).
                           plm_fit_symmetric: automatic refines after either fixed-point
                           path on PLM_PATH_GATHER64_MFMA_I8X6 (the FP32 evaluations'
                           rounding, summed over all parameters, is of the order of
                           1e-6 at N = 500). */
  int32_t n_probe;      /* plm_fit only: number of sites watched by the convergence probe
                           (0 = none).  After the start point is set up and after every
                           iteration (of the refinement fit too), the probe writes one
                           entry of probe_out: [0] the device wall clock in seconds,
                           [1] the largest max-abs difference over the watched sites
                           between the iterate (h_r, and J_r without its self block) and
                           the reference, [2 + k] that difference for watched site k.
                           probe_count (caller-zeroed) receives the entries written;
                           entries beyond probe_cap are dropped.  Meant for measuring the
                           time until a fit is within a given distance of a known
                           minimiser; it adds one small kernel per iteration. */
  double refine_tol;    /* tolerance of the refinement fit; 0 = tol */
  const int32_t *probe_sites; /* DEVICE int32[n_probe], distinct sites in [0, N) */
  const float *probe_h;       /* DEVICE float[n_probe][q] reference fields */
  const float *probe_J;       /* DEVICE float[n_probe][N][q][q] reference couplings */
  double *probe_out;          /* DEVICE double[probe_cap][2 + n_probe] */
  int32_t *probe_count;       /* DEVICE int32[1] */
  int32_t probe_cap;
  int32_t history_fp64; /* 1: the curvature pairs and the gradient kept at the iterate are stored
                           in FP64 (twice the optimiser's history traffic); 0: FP32, the
                           default (their entries are differences of gradients that carry
                           the FP32 evaluation's rounding, far above FP32 storage rounding) */
  int32_t reserved[2];
} plm_fit_opts;

/* Fill *opts with the defaults listed above. */
void plm_fit_opts_default(plm_fit_opts *opts);
/* sizeof(plm_fit_opts) as compiled into the library (a binding's layout check). */
size_t plm_fit_opts_size(void);

#define PLM_SITE_CONVERGED 0
#define PLM_SITE_MAXITER 1
#define PLM_SITE_LINESEARCH 2
#define PLM_SITE_NONFINITE 3

typedef struct {
  int32_t iterations;   /* accepted steps */
  int32_t evaluations;  /* objective+gradient evaluations */
  int32_t status;       /* PLM_SITE_* */
  int32_t pad;
  double f;             /* final g_r^reg (normalised) */
  double gnorm;         /* final ||grad g_r^reg||_2 as computed on the device */
} plm_site_stats;

/* Kernel times of the last plm_fit on this context that ran with timing = 1,
 * summed over all iterations (milliseconds, from HIP events recorded on the
 * stream the kernels run on), and the number of iterations timed. */
typedef struct {
  double forward_ms;    /* energies, log-softmax, residuals */
  double backward_ms;   /* coupling-gradient scatter */
  double lbfgs_ms;      /* line search decision, history update, two-loop recursion */
  double total_ms;      /* wall time of the fit on the device stream */
  int64_t iterations;   /* graph replays (or eager iterations) executed */
  int64_t site_evals;   /* site objective+gradient evaluations performed */
  double quant_ms;      /* the part of forward_ms spent writing the couplings' int8 digits
                           (evaluation path 6; 0 on the others) */
  /* the part of the above spent in the refinement fit (plm_fit_opts.refine) */
  double refine_forward_ms, refine_backward_ms, refine_lbfgs_ms;
  int64_t refine_iterations, refine_site_evals;
} plm_fit_timing;

int plm_fit_last_timing(const plm_ctx *ctx, plm_fit_timing *out);

/* stats_out: HOST array of N records (may be NULL). */
size_t plm_fit_workspace_bytes(int32_t B, int32_t N, int32_t q, const plm_fit_opts *opts);
int plm_fit(plm_ctx *ctx, const uint8_t *msa, int32_t B, int32_t N, int32_t q,
            const double *w, const double *beff, const plm_fit_opts *opts, void *workspace,
            size_t workspace_bytes, float *h_io, float *J_io, plm_site_stats *stats_out);

/* ---- Ragged batch of alignments --------------------------------------------
 * Every site of every alignment is minimised as in plm_fit, all alignments
 * together: each iteration is one launch per kernel over the whole batch
 * (persistent evaluation kernels draining (alignment, site, tile) work items
 * from per-XCD queues, largest alignments first), captured once in a hipGraph.
 * The alignments share q and the options; each brings its own sizes, weights
 * (plm_reweight per alignment), start point and outputs.  With the forward
 * tile size fixed (opts->tile_seqs; by default a batch takes the one its
 * largest alignment would get), results are exactly those plm_fit gives for
 * each alignment alone: same kernels, same per-item arithmetic, in any work
 * order.  descs is a HOST array; the pointers in it are device pointers
 * except stats_out (HOST, N records, may be NULL).  opts->single_site must be
 * 0.  Returns PLM_W_MAXITER if any site of any alignment hit max_iter. */
typedef struct {
  const uint8_t *msa;         /* uint8[B][N] */
  int32_t B, N;
  const double *w;            /* double[B] */
  const double *beff;         /* double[1] */
  float *h_io;                /* float[N][q] */
  float *J_io;                /* float[N][N][q][q] */
  plm_site_stats *stats_out;  /* HOST, N records, may be NULL */
} plm_msa_desc;

size_t plm_fit_batch_workspace_bytes(const plm_msa_desc *descs, int32_t n_msas, int32_t q,
                                     const plm_fit_opts *opts);
int plm_fit_batch(plm_ctx *ctx, const plm_msa_desc *descs, int32_t n_msas, int32_t q,
                  const plm_fit_opts *opts, void *workspace, size_t workspace_bytes);

/* ---- Autotuning ---------------------------------------------------------------
 * Times one all-sites objective+gradient evaluation of the batch (descs as in
 * plm_fit_batch, evaluated at each alignment's (h_io, J_io), whose diagonal
 * blocks are zeroed) for every candidate schedule: each evaluation path
 * (PLM_PATH_MFMA_BF16X2 only if fp32_only == 0) and, for the paths with the
 * LDS-gather forward, forward tiles of 16, 32 and 64 rows per wave.  Writes
 * up to max_out results, fastest first, and their number to *n_out; out[0]'s
 * path and tile_seqs are the schedule to put into plm_fit_opts.  Each time is
 * the shortest of three runs after one warm-up (HIP events on the fit's
 * stream).  Workspace: plm_fit_batch_workspace_bytes.  The choice depends on
 * the device's timing, so it is the caller's to cache (per size bucket). */
typedef struct {
  int32_t path;       /* PLM_PATH_* */
  int32_t tile_seqs;  /* forward tile rows per wave; 0 for the MFMA forward */
  double eval_ms;     /* one all-sites evaluation, forward and backward */
} plm_tune_result;

int plm_tune(plm_ctx *ctx, const plm_msa_desc *descs, int32_t n_msas, int32_t q,
             const plm_fit_opts *opts, int32_t fp32_only, void *workspace, size_t workspace_bytes,
             plm_tune_result *out, int32_t max_out, int32_t *n_out);

/* ---- Scoring (sec. 3.4 steps 4-6) ------------------------------------------
 * For every pair i != j: both estimates are moved to the Ising gauge
 * (eq. gauge_change2: subtract row and column means over all q states, add
 * the grand mean), averaged (eq. average2, the site-j estimate transposed),
 * reduced to a Frobenius norm FN_ij (eq. frob_normtrans2), and corrected by
 * the average product (eq. corr_norm2) with means over all N positions,
 * FN_ii = 0.  Outputs (device) double[N][N], symmetric, zero diagonal.
 * FP64 arithmetic on the FP32 couplings.  No workspace. */
int plm_score(plm_ctx *ctx, const float *J, int32_t N, int32_t q, double *fn_out,
              double *cfn_out);

/* ---- Symmetric pseudolikelihood maximization (eqs. npll_1, l2reg) -----------
 * The comparison method of the paper (sec. 3.2): one minimisation of
 * sum_r g_r + lambda_h sum_i ||h_i||^2 + lambda_J sum_{i<j} ||J_ij||^2 (lambda_J
 * as given, not halved) over all fields and couplings, each J_ij shared by
 * g_i and g_j.  J_io uses the layout of plm_fit and is made consistent: on
 * entry the blocks J[r][i], r < i, are the parameters (J[i][r] is overwritten
 * by their transpose, self blocks by zero); on return J[i][r] is the
 * transpose of J[r][i].  One L-BFGS over the whole vector (compact form,
 * lbfgs_m pairs, the line search of plm_fit) until ||grad||_2 <= tol;
 * stats_out (HOST, one record, may be NULL) describes the whole problem.
 * The evaluation of each trial point is the all-sites evaluation of plm_fit
 * (opts->path); every decision is taken on the device and one iteration is
 * one replay of a captured graph; opts->refine adds a second minimisation
 * from the first one's point on another path (automatic after the fixed-point
 * paths), counted in stats_out and the timing.  Returns PLM_W_MAXITER on the
 * iteration cap.  plm_fit_last_timing reports its kernel times when
 * opts->timing. */
size_t plm_fit_symmetric_workspace_bytes(int32_t B, int32_t N, int32_t q, const plm_fit_opts *opts);
int plm_fit_symmetric(plm_ctx *ctx, const uint8_t *msa, int32_t B, int32_t N, int32_t q,
                      const double *w, const double *beff, const plm_fit_opts *opts,
                      void *workspace, size_t workspace_bytes, float *h_io, float *J_io,
                      plm_site_stats *stats_out);

/* The symmetric fit with every parameter carried as a pair of FP32 words
 * (a high word and a low word; the parameter is their sum, formed in FP64,
 * about 48 significant bits), for tolerances below what FP32 storage of the
 * parameters allows: at N = 500 the rounding of h and J to FP32 alone leaves
 * ||grad|| near 3e-6.  h_lo_io [N][q] and J_lo_io [N][N][q][q] (DEVICE,
 * float) hold the low words of the start point on entry (zeros for an FP32
 * start; J_lo_io is made consistent like J_io) and of the result on return;
 * h_io, J_io hold the high words (hi = fl32(hi + lo)).  The optimiser forms
 * every iterate and trial point in FP64 and splits it; the precise path
 * (PLM_PATH_GATHER64_MFMA_I8X6, the automatic refinement of the fixed-point
 * paths) evaluates at the FP64 sums, the other paths at the high words (their
 * own rounding is far above the difference).  Both low-order pointers must be
 * given; plm_fit_symmetric is this call with both NULL.  Workspace, options,
 * statistics and errors as for plm_fit_symmetric. */
int plm_fit_symmetric_split(plm_ctx *ctx, const uint8_t *msa, int32_t B, int32_t N, int32_t q,
                            const double *w, const double *beff, const plm_fit_opts *opts,
                            void *workspace, size_t workspace_bytes, float *h_io, float *J_io,
                            float *h_lo_io, float *J_lo_io, plm_site_stats *stats_out);

/* ---- Mean-field starting guess (sec. 2, sec. 7) ------------------------------
 * Couplings from the inverse of the connected correlation matrix
 * c_ij(k,l) = f_ij(k,l) - f_i(k) f_j(l) over the states k, l < q-1 (the last
 * state, the gap, is the reference), with reweighted frequencies mixed with
 * a uniform pseudocount of weight `pseudocount` in [0, 1]:
 *   f_i = (1-p) F_i/B_eff + p/q,  f_ij = (1-p) F_ij/B_eff + p/q^2 (i != j),
 *   f_ii(k,l) = f_i(k)[k = l],  J_ij(k,l) = -(C^-1)_{(i,k),(j,l)},
 *   h_i(k) = ln(f_i(k)/f_i(q-1)) - sum_{j != i} sum_{l < q-1} J_ij(k,l) f_j(l),
 * reference-state couplings and fields zero.  Outputs (DEVICE, caller-owned):
 * h_out [N][q], J_out [N][N][q][q] in the layout of plm_fit (both estimates
 * of a pair equal, self blocks zero), usable as plm_fit's start point.  All
 * arithmetic in FP64 (frequencies summed in a fixed order; C inverted in
 * place by block Gauss-Jordan on the device), results rounded to FP32.
 * Workspace: plm_mf_init_workspace_bytes (dominated by C: (N(q-1))^2 doubles,
 * rounded up to 64-row blocks).  Synchronous on the context stream.
 * PLM_E_SYMBOL for a symbol >= q; PLM_E_NONFINITE if C is not positive
 * definite or a reference-state frequency is zero (possible only with
 * pseudocount 0 and an unused state). */
size_t plm_mf_init_workspace_bytes(int32_t B, int32_t N, int32_t q);
int plm_mf_init(plm_ctx *ctx, const uint8_t *msa, int32_t B, int32_t N, int32_t q, const double *w,
                const double *beff, double pseudocount, void *workspace, size_t workspace_bytes,
                float *h_out, float *J_out);

/* ---- Score variants (sec. 7) and contact evaluation (sec. 6) ----------------
 * The alternatives the paper tried besides the CFN score: other combinations
 * of the two Ising-gauge estimates (elementwise min or max instead of the
 * average of eq. average2), other norms (an l_p norm, the sum of |J|^p to
 * the power 1/p; the Burkoff divergence of eqs. burkoffscore1/burkoffscore2,
 * D_ij = sum P ln(P / (f_i f_j)) with P proportional to f_i(k) f_j(l)
 * exp(J*_ij(k,l)), computed on the combined Ising-gauge couplings), the gap
 * state (q-1) left out of the sums, and the average-sum correction of eq.
 * corr_normsum (S = FN - FN_i: - FN_:j + FN_::) or none instead of the APC.
 * plm_score is plm_score_ex with the defaults below. */
#define PLM_COMBINE_AVG 0
#define PLM_COMBINE_MIN 1
#define PLM_COMBINE_MAX 2
#define PLM_NORM_FROB 0
#define PLM_NORM_LP 1
#define PLM_NORM_BURKOFF 2
#define PLM_CORR_APC 0
#define PLM_CORR_NONE 1
#define PLM_CORR_ASC 2

typedef struct {
  int32_t combine;      /* PLM_COMBINE_*; default AVG */
  int32_t norm;         /* PLM_NORM_*; default FROB */
  double p;             /* exponent of PLM_NORM_LP (> 0); default 2 */
  int32_t exclude_gap;  /* 1: sums over states 0..q-2 only; default 0 */
  int32_t correction;   /* PLM_CORR_*; default APC */
  int32_t reserved[4];
} plm_score_opts;

void plm_score_opts_default(plm_score_opts *opts);

/* Reweighted single-site frequencies f_i(k) = sum_b w_b [sigma_i^b = k] / B_eff
 * (device double[N][q]), as the Burkoff score needs them.  All pointers device. */
int plm_frequencies(plm_ctx *ctx, const uint8_t *msa, int32_t B, int32_t N, int32_t q,
                    const double *w, const double *beff, double *f_out);

/* raw_out: the uncorrected pair scores, corrected_out: after the correction;
 * both device double[N][N], symmetric, zero diagonal.  freq (device
 * double[N][q], from plm_frequencies) is required for PLM_NORM_BURKOFF and
 * ignored otherwise. */
int plm_score_ex(plm_ctx *ctx, const float *J, int32_t N, int32_t q, const plm_score_opts *opts,
                 const double *freq, double *raw_out, double *corrected_out);

/* True-positive rate of the strongest predicted contacts (sec. 6): the pairs
 * i < j with j - i >= min_sep are ranked by decreasing score (ties by i, then
 * j), and tpr_out[k] is the fraction of true contacts among the k + 1 first.
 * score: device double[N][N]; contacts: device uint8[N][N] (nonzero = contact,
 * read at [i][j] for i < j).  tpr_out: HOST double[kmax]; *n_out receives the
 * number written (min(kmax, number of pairs)).  Synchronises the context's
 * stream. */
int plm_contact_tpr(plm_ctx *ctx, const double *score, int32_t N, const uint8_t *contacts,
                    int32_t min_sep, int32_t kmax, double *tpr_out, int32_t *n_out);

/* ---- Alignment ingestion (sec. 4) ------------------------------------------
 * FASTA or Stockholm text (HOST memory, len bytes) to symbol codes (HOST
 * uint8[B][N], row-major).  Inserts -- lowercase residues and "." -- are
 * removed, as for the paper's PFAM alignments.  Codes: A C D E F G H I K L M N
 * P Q R S T V W Y = 0..19, "-" = 20 (q = 21); B J O U X Z count as gaps; "*"
 * is skipped; other characters and sequences of unequal aligned length are
 * errors (PLM_E_INVALID, message in err).  Stockholm: "#" lines are
 * annotation, "//" ends the alignment, other lines are "name part", parts
 * of one name concatenated in order.  With codes_out NULL only *B_out and
 * *N_out are set; otherwise capacity must be at least B * N (else
 * PLM_E_WORKSPACE).  No context, no device. */
#define PLM_FORMAT_AUTO 0
#define PLM_FORMAT_FASTA 1
#define PLM_FORMAT_STOCKHOLM 2

int plm_parse_alignment(const char *text, size_t len, int32_t format, uint8_t *codes_out,
                        size_t capacity, int32_t *B_out, int32_t *N_out, char *err, size_t err_len);

#ifdef __cplusplus
}
#endif
#endif /* PLM_H */
