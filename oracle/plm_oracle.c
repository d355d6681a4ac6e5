/*
 * plm_oracle.c -- plain FP64 CPU oracle for asymmetric plmDCA
 * (Ekeberg, Hartonen & Aurell, arXiv:1401.4832).
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the CPU
 * baseline of the benchmark.  The GPU library never links or calls it and the
 * two share no code.  Written for a reader checking it against the paper:
 * literal loops in the order of the equations, FP64 throughout, no blocking,
 * fusion or reordering.  Threads only split independent items (rows or sites).
 *
 * Readings of points the paper leaves open (each also listed in the design
 * notes of the repository):
 *   - similarity counts equal symbols over all N columns, a gap matching a gap
 *     counting as equal (sec. 3.1 names gaps among the states); a pair is
 *     similar when (double)id/(double)N >= theta (eq. inverse_weights uses >=);
 *     the sequence itself is counted in m_b (a ranges over all of 1..B).
 *   - B_eff is summed in sequence-index order.
 *   - lambda'_J = 0.5 * lambda_J exactly (sec. 3.4 step 1).
 *   - the self block J_rr takes no part in energies, regulariser or gradient.
 *   - log-sum-exp is stabilised by subtracting the maximum.
 *   - gauge means run over all q states, gap included; APC averages use all N
 *     positions with FN_ii = 0 (denominators N and N^2); S_ii = 0.
 */
#include "plm_oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* A minimal pool: run fn(ctx, item) for item = 0..n-1 on nthreads threads.  */

typedef void (*item_fn)(void *ctx, int item);
typedef struct {
  item_fn fn;
  void *ctx;
  int n;
  int next;
  pthread_mutex_t mu;
} pool_t;

static void *pool_worker(void *arg) {
  pool_t *p = (pool_t *)arg;
  for (;;) {
    pthread_mutex_lock(&p->mu);
    int it = p->next++;
    pthread_mutex_unlock(&p->mu);
    if (it >= p->n) break;
    p->fn(p->ctx, it);
  }
  return NULL;
}

static void run_items(item_fn fn, void *ctx, int n, int nthreads) {
  if (nthreads <= 1 || n <= 1) {
    for (int i = 0; i < n; ++i) fn(ctx, i);
    return;
  }
  if (nthreads > n) nthreads = n;
  pool_t p = {fn, ctx, n, 0, PTHREAD_MUTEX_INITIALIZER};
  pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)nthreads);
  int started = 0;
  for (int t = 0; t < nthreads; ++t)
    if (pthread_create(&th[t], NULL, pool_worker, &p) == 0) ++started;
  if (started == 0) pool_worker(&p);
  for (int t = 0; t < started; ++t) pthread_join(th[t], NULL);
  free(th);
}

/* ------------------------------------------------------------------------ */
/* Reweighting: sec. 3.1, eq. inverse_weights; sec. 3.4 step 2.              */

static int similar(const uint8_t *a, const uint8_t *b, int N, double theta) {
  int id = 0;
  for (int i = 0; i < N; ++i)
    if (a[i] == b[i]) ++id;
  return ((double)id / (double)N) >= theta;
}

typedef struct {
  const uint8_t *msa;
  int B, N;
  double theta;
  const int32_t *rows;
  int32_t *m;
} rw_ctx;

static void rw_item(void *vc, int item) {
  rw_ctx *c = (rw_ctx *)vc;
  int b = c->rows ? c->rows[item] : item;
  const uint8_t *sb = c->msa + (size_t)b * c->N;
  int32_t count = 0;
  for (int a = 0; a < c->B; ++a)
    count += similar(c->msa + (size_t)a * c->N, sb, c->N, c->theta);
  c->m[item] = count;
}

void oracle_reweight(const uint8_t *msa, int B, int N, double theta, int uniform,
                     int32_t *m_out, double *w_out, double *beff_out, int nthreads) {
  int32_t *m = (int32_t *)malloc(sizeof(int32_t) * (size_t)(B > 0 ? B : 1));
  if (uniform) {
    for (int b = 0; b < B; ++b) m[b] = 1;
  } else {
    rw_ctx c = {msa, B, N, theta, NULL, m};
    run_items(rw_item, &c, B, nthreads);
  }
  double beff = 0.0;
  for (int b = 0; b < B; ++b) {
    double wb = 1.0 / (double)m[b];
    if (m_out) m_out[b] = m[b];
    if (w_out) w_out[b] = wb;
    beff += wb;
  }
  if (beff_out) *beff_out = beff;
  free(m);
}

void oracle_reweight_rows(const uint8_t *msa, int B, int N, double theta,
                          const int32_t *rows, int nrows, int32_t *m_out, int nthreads) {
  rw_ctx c = {msa, B, N, theta, rows, m_out};
  run_items(rw_item, &c, nrows, nthreads);
}

/* ------------------------------------------------------------------------ */
/* Per-site objective and gradient: sec. 3.4 step 3, eqs. g_regdef2,         */
/* g_gradh2, g_gradJ2, multiplied through by B_eff.                          */

double oracle_site_objgrad(const uint8_t *msa, int B, int N, int q, int r,
                           const double *w, double beff, const double *hr,
                           const double *Jr, double lambda_h, double lambda_J,
                           double *ghr, double *gJr) {
  const double lambda_Jp = 0.5 * lambda_J; /* step 1 */
  const size_t qq = (size_t)q * (size_t)q;
  double *E = (double *)malloc(sizeof(double) * (size_t)q);
  double *R = (double *)malloc(sizeof(double) * (size_t)q);
  if (ghr) memset(ghr, 0, sizeof(double) * (size_t)q);
  if (gJr) memset(gJr, 0, sizeof(double) * (size_t)N * qq);
  double f = 0.0;

  for (int b = 0; b < B; ++b) {
    const uint8_t *sigma = msa + (size_t)b * N;
    /* energies E(s) = h_r(s) + sum_{i != r} J_ri(s, sigma_i) (eq. condpfinal) */
    for (int s = 0; s < q; ++s) {
      double e = hr[s];
      for (int i = 0; i < N; ++i) {
        if (i == r) continue;
        e += Jr[(size_t)i * qq + (size_t)sigma[i] * q + s];
      }
      E[s] = e;
    }
    /* log of the normaliser, shifted by the maximum */
    double mx = E[0];
    for (int s = 1; s < q; ++s)
      if (E[s] > mx) mx = E[s];
    double z = 0.0;
    for (int s = 0; s < q; ++s) z += exp(E[s] - mx);
    double lse = mx + log(z);
    /* -w_b * log P(sigma_r^b | rest) */
    f += w[b] * (lse - E[sigma[r]]);
    /* w_b (P(s) - I[sigma_r = s]): the bracket of eqs. g_gradh2, g_gradJ2 with
       the sign folded in */
    for (int s = 0; s < q; ++s) {
      double P = exp(E[s] - lse);
      R[s] = w[b] * (P - (sigma[r] == s ? 1.0 : 0.0));
    }
    if (ghr)
      for (int s = 0; s < q; ++s) ghr[s] += R[s];
    if (gJr)
      for (int i = 0; i < N; ++i) {
        if (i == r) continue;
        double *row = gJr + (size_t)i * qq + (size_t)sigma[i] * q;
        for (int s = 0; s < q; ++s) row[s] += R[s];
      }
  }

  /* l2 terms of eq. g_regdef2 (times B_eff) and their derivatives */
  double hh = 0.0;
  for (int s = 0; s < q; ++s) hh += hr[s] * hr[s];
  double jj = 0.0;
  for (int i = 0; i < N; ++i) {
    if (i == r) continue;
    for (size_t e = 0; e < qq; ++e) {
      double v = Jr[(size_t)i * qq + e];
      jj += v * v;
    }
  }
  f += beff * (lambda_h * hh + lambda_Jp * jj);
  if (ghr)
    for (int s = 0; s < q; ++s) ghr[s] += 2.0 * beff * lambda_h * hr[s];
  if (gJr)
    for (int i = 0; i < N; ++i) {
      if (i == r) continue; /* the self block stays zero */
      for (size_t e = 0; e < qq; ++e)
        gJr[(size_t)i * qq + e] += 2.0 * beff * lambda_Jp * Jr[(size_t)i * qq + e];
    }
  free(E);
  free(R);
  return f;
}

typedef struct {
  const uint8_t *msa;
  int B, N, q;
  const double *w;
  double beff;
  const double *h, *J;
  double lh, lJ;
  const int32_t *sites;
  double *f, *gh, *gJ;
} og_ctx;

static void og_item(void *vc, int t) {
  og_ctx *c = (og_ctx *)vc;
  int r = c->sites[t];
  size_t qq = (size_t)c->q * c->q;
  c->f[t] = oracle_site_objgrad(c->msa, c->B, c->N, c->q, r, c->w, c->beff,
                                c->h + (size_t)r * c->q, c->J + (size_t)r * c->N * qq,
                                c->lh, c->lJ, c->gh ? c->gh + (size_t)t * c->q : NULL,
                                c->gJ ? c->gJ + (size_t)t * c->N * qq : NULL);
}

void oracle_objgrad(const uint8_t *msa, int B, int N, int q, const double *w,
                    double beff, const double *h, const double *J, double lambda_h,
                    double lambda_J, const int32_t *sites, int nsites, double *f_out,
                    double *gh_out, double *gJ_out, int nthreads) {
  og_ctx c = {msa, B, N, q, w, beff, h, J, lambda_h, lambda_J, sites, f_out, gh_out, gJ_out};
  run_items(og_item, &c, nsites, nthreads);
}

typedef struct {
  og_ctx base;
} ogs_ctx;

static void ogs_item(void *vc, int t) {
  og_ctx *c = &((ogs_ctx *)vc)->base;
  size_t qq = (size_t)c->q * c->q;
  c->f[t] = oracle_site_objgrad(c->msa, c->B, c->N, c->q, c->sites[t], c->w, c->beff,
                                c->h + (size_t)t * c->q, c->J + (size_t)t * c->N * qq,
                                c->lh, c->lJ, c->gh ? c->gh + (size_t)t * c->q : NULL,
                                c->gJ ? c->gJ + (size_t)t * c->N * qq : NULL);
}

void oracle_objgrad_slices(const uint8_t *msa, int B, int N, int q, const double *w,
                           double beff, const double *hr, const double *Jr,
                           double lambda_h, double lambda_J, const int32_t *sites,
                           int nsites, double *f_out, double *gh_out, double *gJ_out,
                           int nthreads) {
  ogs_ctx c = {{msa, B, N, q, w, beff, hr, Jr, lambda_h, lambda_J, sites, f_out, gh_out, gJ_out}};
  run_items(ogs_item, &c, nsites, nthreads);
}

/* ------------------------------------------------------------------------ */
/* Per-site minimisation (sec. 3.4 step 3; L-BFGS per sec. 5, cold start at   */
/* the origin per sec. 6).  Textbook limited-memory BFGS (two-loop recursion, */
/* initial Hessian s'y/y'y) with a line search enforcing the strong Wolfe      */
/* conditions (bracketing phase, then a zoom phase with safeguarded cubic     */
/* interpolation), on the normalised scale g = f / B_eff.                     */

typedef struct {
  const uint8_t *msa;
  int B, N, q, r;
  const double *w;
  double beff, lh, lJ;
  size_t n;         /* q + N q^2 */
  int evals;
} site_prob;

/* value and gradient of g_r^reg (normalised) at x = [h_r ; J_r] */
static double site_eval(site_prob *p, const double *x, double *g) {
  p->evals++;
  double f = oracle_site_objgrad(p->msa, p->B, p->N, p->q, p->r, p->w, p->beff, x,
                                 x + p->q, p->lh, p->lJ, g, g + p->q);
  for (size_t e = 0; e < p->n; ++e) g[e] /= p->beff;
  return f / p->beff;
}

static double dot(const double *a, const double *b, size_t n) {
  double s = 0.0;
  for (size_t e = 0; e < n; ++e) s += a[e] * b[e];
  return s;
}

/* minimiser of the cubic matching values and slopes at a and b; NAN if none */
static double cubic_step(double a, double fa, double da, double b, double fb, double db) {
  double d1 = da + db - 3.0 * (fa - fb) / (a - b);
  double disc = d1 * d1 - da * db;
  if (!(disc >= 0.0)) return NAN;
  double d2 = copysign(sqrt(disc), b - a);
  double den = db - da + 2.0 * d2;
  if (den == 0.0) return NAN;
  return b - (b - a) * (db + d2 - d1) / den;
}

/* trial point inside (lo, hi) kept away from the ends */
static double pick(double lo, double flo, double dlo, double hi, double fhi, double dhi) {
  double t = cubic_step(lo, flo, dlo, hi, fhi, dhi);
  double a = lo < hi ? lo : hi, b = lo < hi ? hi : lo;
  double margin = 0.1 * (b - a);
  if (!(t >= a + margin && t <= b - margin)) t = 0.5 * (lo + hi);
  return t;
}

typedef struct {
  double f;
  double alpha;
  int ok;
} ls_result;

/* Strong-Wolfe line search along d from (x, f0, g).  On success xt, gt hold
 * the accepted point and its gradient. */
static ls_result line_search(site_prob *p, const double *x, double f0, const double *g0,
                             const double *d, double alpha0, double c1, double c2,
                             double *xt, double *gt, double *xa, double *ga) {
  const size_t n = p->n;
  const double dphi0 = dot(g0, d, n);
  /* Round-off allowance on the value test: near the optimum the true decrease
     falls below the rounding error of f, and only the slope conditions carry
     information (the approximate Wolfe idea of Hager & Zhang, SIAM J. Optim.
     16 (2005)). */
  const double slack = 1e-13 * fabs(f0);
  ls_result res = {f0, 0.0, 0};
  double a_prev = 0.0, f_prev = f0, d_prev = dphi0;
  double a = alpha0;
  double lo = 0, flo = 0, dlo = 0, hi = 0, fhi = 0, dhi = 0;
  int zoom = 0;
  for (int it = 0; it < 40 && !zoom; ++it) {
    for (size_t e = 0; e < n; ++e) xt[e] = x[e] + a * d[e];
    double fa = site_eval(p, xt, gt);
    double da = dot(gt, d, n);
    if (fa > f0 + c1 * a * dphi0 + slack || (it > 0 && fa > f_prev + slack)) {
      lo = a_prev; flo = f_prev; dlo = d_prev; hi = a; fhi = fa; dhi = da;
      zoom = 1;
      break;
    }
    if (fabs(da) <= -c2 * dphi0) {
      res.f = fa; res.alpha = a; res.ok = 1;
      return res;
    }
    if (da >= 0.0) {
      lo = a; flo = fa; dlo = da; hi = a_prev; fhi = f_prev; dhi = d_prev;
      zoom = 1;
      break;
    }
    a_prev = a; f_prev = fa; d_prev = da;
    a = 2.0 * a;
  }
  if (!zoom) return res;
  /* zoom: lo always satisfies sufficient decrease and has the lowest value */
  int have_lo_point = 0;
  for (int it = 0; it < 60; ++it) {
    double aj = pick(lo, flo, dlo, hi, fhi, dhi);
    for (size_t e = 0; e < n; ++e) xt[e] = x[e] + aj * d[e];
    double fj = site_eval(p, xt, gt);
    double dj = dot(gt, d, n);
    if (fj > f0 + c1 * aj * dphi0 + slack || fj > flo + slack) {
      hi = aj; fhi = fj; dhi = dj;
    } else {
      if (fabs(dj) <= -c2 * dphi0) {
        res.f = fj; res.alpha = aj; res.ok = 1;
        return res;
      }
      if (dj * (hi - lo) >= 0.0) { hi = lo; fhi = flo; dhi = dlo; }
      lo = aj; flo = fj; dlo = dj;
      memcpy(xa, xt, sizeof(double) * n);
      memcpy(ga, gt, sizeof(double) * n);
      have_lo_point = 1;
    }
    if (fabs(hi - lo) <= 1e-16 * (fabs(lo) + 1e-300)) break;
  }
  /* no strong-Wolfe point found: fall back to the best sufficient-decrease point */
  if (have_lo_point && lo > 0.0) {
    memcpy(xt, xa, sizeof(double) * n);
    memcpy(gt, ga, sizeof(double) * n);
    res.f = flo; res.alpha = lo; res.ok = 1;
  }
  return res;
}

int oracle_site_fit(const uint8_t *msa, int B, int N, int q, int r, const double *w,
                    double beff, double lambda_h, double lambda_J,
                    const oracle_fit_opts *opts, double *hr_io, double *Jr_io,
                    oracle_fit_stats *stats) {
  site_prob p = {msa, B, N, q, r, w, beff, lambda_h, lambda_J,
                 (size_t)q + (size_t)N * q * q, 0};
  const size_t n = p.n;
  const int m = opts->m > 0 ? opts->m : 10;
  double *x = (double *)malloc(sizeof(double) * n);
  double *g = (double *)malloc(sizeof(double) * n);
  double *d = (double *)malloc(sizeof(double) * n);
  double *xt = (double *)malloc(sizeof(double) * n);
  double *gt = (double *)malloc(sizeof(double) * n);
  double *xa = (double *)malloc(sizeof(double) * n);
  double *ga = (double *)malloc(sizeof(double) * n);
  double *S = (double *)malloc(sizeof(double) * n * (size_t)m);
  double *Y = (double *)malloc(sizeof(double) * n * (size_t)m);
  double *rho = (double *)malloc(sizeof(double) * (size_t)m);
  double *alpha = (double *)malloc(sizeof(double) * (size_t)m);

  memcpy(x, hr_io, sizeof(double) * q);
  memcpy(x + q, Jr_io, sizeof(double) * (size_t)N * q * q);
  for (size_t e = 0; e < (size_t)q * q; ++e) x[q + (size_t)r * q * q + e] = 0.0;

  double f = site_eval(&p, x, g);
  double gnorm = sqrt(dot(g, g, n));
  int k = 0, stored = 0, head = 0, status = 1, iters = 0;
  while (iters < opts->max_iter) {
    if (gnorm <= opts->tol) { status = 0; break; }
    /* two-loop recursion: d = -H g */
    for (size_t e = 0; e < n; ++e) d[e] = -g[e];
    for (int j = 0; j < stored; ++j) {
      int idx = (head - 1 - j + m) % m;
      alpha[idx] = rho[idx] * dot(S + (size_t)idx * n, d, n);
      for (size_t e = 0; e < n; ++e) d[e] -= alpha[idx] * Y[(size_t)idx * n + e];
    }
    if (stored > 0) {
      int last = (head - 1 + m) % m;
      const double *sl = S + (size_t)last * n, *yl = Y + (size_t)last * n;
      double gamma = dot(sl, yl, n) / dot(yl, yl, n);
      for (size_t e = 0; e < n; ++e) d[e] *= gamma;
    }
    for (int j = stored - 1; j >= 0; --j) {
      int idx = (head - 1 - j + m) % m;
      double beta = rho[idx] * dot(Y + (size_t)idx * n, d, n);
      for (size_t e = 0; e < n; ++e) d[e] += (alpha[idx] - beta) * S[(size_t)idx * n + e];
    }
    if (dot(d, g, n) >= 0.0) { /* not a descent direction: restart */
      for (size_t e = 0; e < n; ++e) d[e] = -g[e];
      stored = 0;
    }
    double a0 = (k == 0 || stored == 0) ? 1.0 / gnorm : 1.0;
    if (a0 > 1.0) a0 = 1.0;
    ls_result ls = line_search(&p, x, f, g, d, a0, opts->c1, opts->c2, xt, gt, xa, ga);
    if (!ls.ok) {
      if (stored > 0) { stored = 0; continue; } /* retry once from steepest descent */
      status = 2;
      break;
    }
    /* curvature pair */
    double *sn = S + (size_t)head * n, *yn = Y + (size_t)head * n;
    for (size_t e = 0; e < n; ++e) {
      sn[e] = xt[e] - x[e];
      yn[e] = gt[e] - g[e];
    }
    double sy = dot(sn, yn, n);
    if (sy > 0.0) {
      rho[head] = 1.0 / sy;
      head = (head + 1) % m;
      if (stored < m) ++stored;
    }
    memcpy(x, xt, sizeof(double) * n);
    memcpy(g, gt, sizeof(double) * n);
    f = ls.f;
    gnorm = sqrt(dot(g, g, n));
    ++k;
    ++iters;
  }
  if (gnorm <= opts->tol) status = 0;

  memcpy(hr_io, x, sizeof(double) * q);
  memcpy(Jr_io, x + q, sizeof(double) * (size_t)N * q * q);
  if (stats) {
    stats->iterations = iters;
    stats->evaluations = p.evals;
    stats->status = status;
    stats->f = f;
    stats->gnorm = gnorm;
  }
  free(x); free(g); free(d); free(xt); free(gt); free(xa); free(ga);
  free(S); free(Y); free(rho); free(alpha);
  return status;
}

typedef struct {
  const uint8_t *msa;
  int B, N, q;
  const double *w;
  double beff, lh, lJ;
  const oracle_fit_opts *opts;
  const int32_t *sites;
  double *h, *J;
  oracle_fit_stats *st;
} fit_ctx;

static void fit_item(void *vc, int t) {
  fit_ctx *c = (fit_ctx *)vc;
  size_t qq = (size_t)c->q * c->q;
  double *hr = c->h + (size_t)t * c->q;
  double *Jr = c->J + (size_t)t * c->N * qq;
  memset(hr, 0, sizeof(double) * c->q);
  memset(Jr, 0, sizeof(double) * c->N * qq);
  oracle_site_fit(c->msa, c->B, c->N, c->q, c->sites[t], c->w, c->beff, c->lh, c->lJ,
                  c->opts, hr, Jr, c->st ? &c->st[t] : NULL);
}

void oracle_fit(const uint8_t *msa, int B, int N, int q, const double *w, double beff,
                double lambda_h, double lambda_J, const oracle_fit_opts *opts,
                const int32_t *sites, int nsites, double *h_out, double *J_out,
                oracle_fit_stats *stats, int nthreads) {
  fit_ctx c = {msa, B, N, q, w, beff, lambda_h, lambda_J, opts, sites, h_out, J_out, stats};
  run_items(fit_item, &c, nsites, nthreads);
}

/* ------------------------------------------------------------------------ */
/* Scoring: sec. 3.4 steps 4-6.                                              */

/* Both estimates of pair (i, j), i != j, as q x q matrices indexed by
 * (state of i, state of j).  The site-i estimate is J[i][j][k][s] with s the
 * state of i; the site-j estimate is J[j][i][k][s] with s the state of j, so
 * it enters transposed (the convention J_ij(k,l) = J_ji(l,k) of sec. 2). */
static void pair_estimates(const void *J, int is_f32, int N, int q, int i, int j,
                           double *Ai, double *Aj) {
  size_t qq = (size_t)q * q;
  size_t bij = ((size_t)i * N + j) * qq, bji = ((size_t)j * N + i) * qq;
  for (int a = 0; a < q; ++a)
    for (int c = 0; c < q; ++c) {
      size_t from_i = bij + (size_t)c * q + a; /* k = c (state of j), s = a */
      size_t from_j = bji + (size_t)a * q + c; /* k = a (state of i), s = c */
      if (is_f32) {
        Ai[a * q + c] = (double)((const float *)J)[from_i];
        Aj[a * q + c] = (double)((const float *)J)[from_j];
      } else {
        Ai[a * q + c] = ((const double *)J)[from_i];
        Aj[a * q + c] = ((const double *)J)[from_j];
      }
    }
}

/* eq. gauge_change2: subtract row and column means, add back the grand mean */
static void ising_gauge(const double *A, int q, double *out) {
  double grand = 0.0;
  for (int a = 0; a < q * q; ++a) grand += A[a];
  grand /= (double)(q * q);
  for (int a = 0; a < q; ++a) {
    double row = 0.0;
    for (int c = 0; c < q; ++c) row += A[a * q + c];
    row /= (double)q;
    for (int c = 0; c < q; ++c) {
      double col = 0.0;
      for (int a2 = 0; a2 < q; ++a2) col += A[a2 * q + c];
      col /= (double)q;
      out[a * q + c] = A[a * q + c] - col - row + grand;
    }
  }
}

static void score_impl(const void *J, int is_f32, int N, int q, double *fn, double *cfn) {
  size_t qq = (size_t)q * q;
  double *Ai = (double *)malloc(sizeof(double) * qq);
  double *Aj = (double *)malloc(sizeof(double) * qq);
  double *Gi = (double *)malloc(sizeof(double) * qq);
  double *Gj = (double *)malloc(sizeof(double) * qq);
  for (int i = 0; i < N; ++i) fn[(size_t)i * N + i] = 0.0;
  for (int i = 0; i < N; ++i)
    for (int j = i + 1; j < N; ++j) {
      pair_estimates(J, is_f32, N, q, i, j, Ai, Aj);
      ising_gauge(Ai, q, Gi);
      ising_gauge(Aj, q, Gj);
      double ss = 0.0;
      for (size_t e = 0; e < qq; ++e) {
        double v = 0.5 * (Gi[e] + Gj[e]); /* eq. average2 */
        ss += v * v;
      }
      double v = sqrt(ss); /* eq. frob_normtrans2 */
      fn[(size_t)i * N + j] = v;
      fn[(size_t)j * N + i] = v;
    }
  /* eq. corr_norm2: averages over positions */
  double *rowm = (double *)malloc(sizeof(double) * (size_t)N);
  double all = 0.0;
  for (int i = 0; i < N; ++i) {
    double s = 0.0;
    for (int j = 0; j < N; ++j) s += fn[(size_t)i * N + j];
    rowm[i] = s / (double)N;
    all += s;
  }
  all /= (double)N * (double)N;
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j)
      cfn[(size_t)i * N + j] =
          (i == j || all == 0.0) ? 0.0 : fn[(size_t)i * N + j] - rowm[i] * rowm[j] / all;
  free(rowm);
  free(Ai); free(Aj); free(Gi); free(Gj);
}

void oracle_score(const double *J, int N, int q, double *fn, double *cfn) {
  score_impl(J, 0, N, q, fn, cfn);
}

void oracle_score_f32(const float *J, int N, int q, double *fn, double *cfn) {
  score_impl(J, 1, N, q, fn, cfn);
}
