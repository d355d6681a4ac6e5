/*
 * plm_oracle.h -- plain FP64 CPU oracle for asymmetric l2-regularised
 * pseudolikelihood maximisation (asymmetric plmDCA, Ekeberg, Hartonen & Aurell,
 * arXiv:1401.4832).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists so that the tests, the smoke
 * check and the CPU-baseline leg of the benchmark can compare the GPU library
 * against an independent, slow, obviously correct implementation.  The product
 * path never links, loads or calls it.  It shares no code, header, table or
 * helper with the GPU library.
 *
 * Conventions (all arrays C row-major, host memory, caller-owned):
 *   msa   uint8[B][N], symbols 0..q-1.
 *   h     double[N][q]           h[r][s] = h_r(s)
 *   J     double[N][N][q][q]     J[r][i][k][s] = J^{(r)}_{ri}(s,k): the coupling
 *                                 between state s of site r and state k of site i
 *                                 as estimated by the site-r problem.  Blocks with
 *                                 i == r are ignored on input, zero on output.
 *   Objective scale: f_r = B_eff * g_r^reg (sec. 3.4, step 3, eq. g_regdef2); the
 *   fitted minimiser is the same on either scale.
 */
#ifndef PLM_ORACLE_H
#define PLM_ORACLE_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

/* Sec. 3.1 (eq. inverse_weights) and sec. 3.4 step 2 (eq. inverse_weights2):
 * m_b = #{a : similarity(a,b) >= theta}, similarity = (#equal columns)/N
 * computed as (double)id/(double)N; w_b = 1/m_b; B_eff = sum_b w_b summed in
 * index order.  uniform != 0 gives w_b = 1, B_eff = B.  Any output may be NULL. */
void oracle_reweight(const uint8_t *msa, int B, int N, double theta, int uniform,
                     int32_t *m_out, double *w_out, double *beff_out, int nthreads);

/* m_b for selected rows only (same definition), for alignments too large for
 * the full B x B comparison on a CPU. */
void oracle_reweight_rows(const uint8_t *msa, int B, int N, double theta,
                          const int32_t *rows, int nrows, int32_t *m_out, int nthreads);

/* Sec. 3.4 step 3: objective eq. g_regdef2 and gradient eqs. g_gradh2 /
 * g_gradJ2 for one site r, on the f = B_eff * g scale, with lambda'_J =
 * 0.5*lambda_J (step 1).  hr = h[r][q], Jr = J[r][N][q][q]; ghr, gJr receive
 * the gradient (may be NULL).  Returns f_r. */
double oracle_site_objgrad(const uint8_t *msa, int B, int N, int q, int r,
                           const double *w, double beff, const double *hr,
                           const double *Jr, double lambda_h, double lambda_J,
                           double *ghr, double *gJr);

/* The same for a list of sites, threaded over sites.  h, J are the full
 * arrays; outputs are packed per listed site: f_out[ns], gh_out[ns][q],
 * gJ_out[ns][N][q][q] (gh_out / gJ_out may be NULL). */
void oracle_objgrad(const uint8_t *msa, int B, int N, int q, const double *w,
                    double beff, const double *h, const double *J, double lambda_h,
                    double lambda_J, const int32_t *sites, int nsites, double *f_out,
                    double *gh_out, double *gJ_out, int nthreads);

/* The same from per-site slices: hr[ns][q], Jr[ns][N][q][q] hold the
 * parameters of the listed sites only (for alignments whose full J is too
 * large to hold in FP64). */
void oracle_objgrad_slices(const uint8_t *msa, int B, int N, int q, const double *w,
                           double beff, const double *hr, const double *Jr,
                           double lambda_h, double lambda_J, const int32_t *sites,
                           int nsites, double *f_out, double *gh_out, double *gJ_out,
                           int nthreads);

typedef struct {
  int m;            /* L-BFGS memory (10) */
  double tol;       /* stop when ||grad g_r^reg||_2 <= tol (normalised scale) */
  int max_iter;     /* iteration cap */
  double c1, c2;    /* strong Wolfe constants (1e-4, 0.9) */
} oracle_fit_opts;

typedef struct {
  int iterations;
  int evaluations;
  int status;       /* 0 converged, 1 iteration cap, 2 line search failed */
  double f;         /* final g_r^reg (normalised) */
  double gnorm;     /* final ||grad g_r^reg||_2 (normalised) */
} oracle_fit_stats;

/* Sec. 3.4 step 3: minimise g_r^reg from (hr_io, Jr_io) (the paper starts at
 * zero, sec. 6) by L-BFGS with a strong-Wolfe line search.  Returns status. */
int oracle_site_fit(const uint8_t *msa, int B, int N, int q, int r, const double *w,
                    double beff, double lambda_h, double lambda_J,
                    const oracle_fit_opts *opts, double *hr_io, double *Jr_io,
                    oracle_fit_stats *stats);

/* Threaded over the listed sites, each started from zero.  Outputs packed per
 * listed site: h_out[ns][q], J_out[ns][N][q][q], stats[ns]. */
void oracle_fit(const uint8_t *msa, int B, int N, int q, const double *w, double beff,
                double lambda_h, double lambda_J, const oracle_fit_opts *opts,
                const int32_t *sites, int nsites, double *h_out, double *J_out,
                oracle_fit_stats *stats, int nthreads);

/* Sec. 3.4 steps 4-6: Ising gauge (eq. gauge_change2), average of the two
 * estimates (eq. average2), Frobenius norm (eq. frob_normtrans2) and average
 * product correction (eq. corr_norm2).  fn, cfn: double[N][N], symmetric,
 * zero diagonal.  J is double (oracle_score) or float (oracle_score_f32,
 * converted exactly to double before any arithmetic). */
void oracle_score(const double *J, int N, int q, double *fn, double *cfn);
void oracle_score_f32(const float *J, int N, int q, double *fn, double *cfn);

#ifdef __cplusplus
}
#endif
#endif
