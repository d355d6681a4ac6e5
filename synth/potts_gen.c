/*
 * potts_gen.c -- seeded synthetic multiple-sequence alignments sampled from a
 * planted Potts model (the model of sec. 2, eq. potts_model), standing in for
 * the PFAM families used in the paper, which are not available here.
 *
 * Shared input generator for tests and benchmarks.  It holds no part of the
 * inference method (no reweighting, objective, gradient, optimiser or score);
 * it only draws model parameters and samples sequences from them.
 *
 * Random numbers: splitmix64 seeds xoshiro256** (Blackman & Vigna); normals by
 * the Box-Muller transform; categorical draws by inverse CDF on exp(E - max).
 * Every stream is keyed by (seed, stream id) so results do not depend on the
 * number of threads.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct { uint64_t s[4]; } rng_t;

static uint64_t splitmix64(uint64_t *x) {
  uint64_t z = (*x += 0x9E3779B97F4A7C15ULL);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

static void rng_seed(rng_t *r, uint64_t seed, uint64_t stream) {
  uint64_t x = seed * 0x100000001B3ULL ^ (stream + 0x632BE59BD9B4E019ULL);
  for (int k = 0; k < 4; ++k) r->s[k] = splitmix64(&x);
}

static inline uint64_t rotl(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }

static uint64_t rng_next(rng_t *r) { /* xoshiro256** */
  uint64_t *s = r->s;
  uint64_t out = rotl(s[1] * 5, 7) * 9;
  uint64_t t = s[1] << 17;
  s[2] ^= s[0];
  s[3] ^= s[1];
  s[1] ^= s[2];
  s[0] ^= s[3];
  s[2] ^= t;
  s[3] = rotl(s[3], 45);
  return out;
}

static double rng_uniform(rng_t *r) { /* [0, 1) */
  return (double)(rng_next(r) >> 11) * 0x1.0p-53;
}

static double rng_normal(rng_t *r) {
  double u1 = 1.0 - rng_uniform(r); /* (0, 1] */
  double u2 = rng_uniform(r);
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

enum { STREAM_FIELDS = 1, STREAM_PAIRS = 2, STREAM_COUPLINGS = 3, STREAM_GAPS = 4,
       STREAM_CHAIN0 = 1000 };

/* Fields h[N][q] ~ N(0, h_sd^2); npairs distinct pairs (i<j, j-i >= min_sep)
 * drawn uniformly without replacement; each planted block Jp[p][k][l] ~
 * N(0, j_sd^2) couples state k of pairs[p][0] with state l of pairs[p][1].
 * Returns the number of pairs drawn (fewer than asked if not enough exist). */
int synth_potts_model(uint64_t seed, int N, int q, int npairs, int min_sep, double h_sd,
                      double j_sd, double *h, int32_t *pairs, double *Jp) {
  rng_t r;
  rng_seed(&r, seed, STREAM_FIELDS);
  for (int e = 0; e < N * q; ++e) h[e] = h_sd * rng_normal(&r);

  int64_t neligible = 0;
  for (int i = 0; i < N; ++i)
    for (int j = i + 1; j < N; ++j)
      if (j - i >= min_sep) ++neligible;
  int32_t *cand = (int32_t *)malloc(sizeof(int32_t) * 2 * (size_t)(neligible ? neligible : 1));
  int64_t c = 0;
  for (int i = 0; i < N; ++i)
    for (int j = i + 1; j < N; ++j)
      if (j - i >= min_sep) { cand[2 * c] = i; cand[2 * c + 1] = j; ++c; }
  if (npairs > neligible) npairs = (int)neligible;
  rng_seed(&r, seed, STREAM_PAIRS);
  for (int p = 0; p < npairs; ++p) { /* partial Fisher-Yates */
    int64_t k = p + (int64_t)(rng_uniform(&r) * (double)(neligible - p));
    if (k >= neligible) k = neligible - 1;
    int32_t a = cand[2 * p], b = cand[2 * p + 1];
    cand[2 * p] = cand[2 * k]; cand[2 * p + 1] = cand[2 * k + 1];
    cand[2 * k] = a; cand[2 * k + 1] = b;
    pairs[2 * p] = cand[2 * p];
    pairs[2 * p + 1] = cand[2 * p + 1];
  }
  free(cand);
  rng_seed(&r, seed, STREAM_COUPLINGS);
  for (int64_t e = 0; e < (int64_t)npairs * q * q; ++e) Jp[e] = j_sd * rng_normal(&r);
  return npairs;
}

/* ---- Gibbs sampling ---------------------------------------------------- */

typedef struct {
  int N, q, B, nchains, burnin, thin;
  uint64_t seed;
  const double *h;
  /* sparse partner lists: for site i, entries adj_off[i]..adj_off[i+1]-1 give
     (partner j, pointer to a q x q block, transposed flag) */
  const int32_t *adj_off, *adj_j, *adj_t;
  const double *const *adj_blk;
  uint8_t *msa;
} gibbs_ctx;

static void sweep(const gibbs_ctx *g, rng_t *r, uint8_t *x, double *E) {
  const int q = g->q;
  for (int i = 0; i < g->N; ++i) {
    for (int s = 0; s < q; ++s) E[s] = g->h[(size_t)i * q + s];
    for (int a = g->adj_off[i]; a < g->adj_off[i + 1]; ++a) {
      const double *blk = g->adj_blk[a];
      int sj = x[g->adj_j[a]];
      if (g->adj_t[a]) /* block stored as (state of partner, state of i) */
        for (int s = 0; s < q; ++s) E[s] += blk[(size_t)sj * q + s];
      else
        for (int s = 0; s < q; ++s) E[s] += blk[(size_t)s * q + sj];
    }
    double mx = E[0];
    for (int s = 1; s < q; ++s) if (E[s] > mx) mx = E[s];
    double tot = 0.0;
    for (int s = 0; s < q; ++s) { E[s] = exp(E[s] - mx); tot += E[s]; }
    double u = rng_uniform(r) * tot, acc = 0.0;
    int pick = q - 1;
    for (int s = 0; s < q; ++s) { acc += E[s]; if (u < acc) { pick = s; break; } }
    x[i] = (uint8_t)pick;
  }
}

typedef struct { gibbs_ctx *g; int next; pthread_mutex_t mu; } gibbs_pool;

static void run_chain(gibbs_ctx *g, int c) {
  rng_t r;
  rng_seed(&r, g->seed, STREAM_CHAIN0 + (uint64_t)c);
  uint8_t *x = (uint8_t *)malloc((size_t)g->N);
  double *E = (double *)malloc(sizeof(double) * (size_t)g->q);
  for (int i = 0; i < g->N; ++i) {
    int s = (int)(rng_uniform(&r) * g->q);
    x[i] = (uint8_t)(s < g->q ? s : g->q - 1);
  }
  for (int t = 0; t < g->burnin; ++t) sweep(g, &r, x, E);
  for (int b = c; b < g->B; b += g->nchains) {
    for (int t = 0; t < g->thin; ++t) sweep(g, &r, x, E);
    memcpy(g->msa + (size_t)b * g->N, x, (size_t)g->N);
  }
  free(x);
  free(E);
}

static void *gibbs_worker(void *arg) {
  gibbs_pool *p = (gibbs_pool *)arg;
  for (;;) {
    pthread_mutex_lock(&p->mu);
    int c = p->next++;
    pthread_mutex_unlock(&p->mu);
    if (c >= p->g->nchains) break;
    run_chain(p->g, c);
  }
  return NULL;
}

/* Row b of msa[B][N] is the (b / nchains)-th thinned sample of chain
 * b % nchains; each chain starts uniform and runs burnin sweeps first. */
void synth_gibbs(uint64_t seed, int N, int q, const double *h, int npairs,
                 const int32_t *pairs, const double *Jp, int B, int nchains, int burnin,
                 int thin, uint8_t *msa, int nthreads) {
  int32_t *deg = (int32_t *)calloc((size_t)N + 1, sizeof(int32_t));
  for (int p = 0; p < npairs; ++p) { deg[pairs[2 * p]]++; deg[pairs[2 * p + 1]]++; }
  int32_t *off = (int32_t *)malloc(sizeof(int32_t) * ((size_t)N + 1));
  off[0] = 0;
  for (int i = 0; i < N; ++i) off[i + 1] = off[i] + deg[i];
  int32_t *fill = (int32_t *)calloc((size_t)N, sizeof(int32_t));
  size_t nadj = (size_t)off[N];
  int32_t *aj = (int32_t *)malloc(sizeof(int32_t) * (nadj ? nadj : 1));
  int32_t *at = (int32_t *)malloc(sizeof(int32_t) * (nadj ? nadj : 1));
  const double **ab = (const double **)malloc(sizeof(double *) * (nadj ? nadj : 1));
  for (int p = 0; p < npairs; ++p) {
    int i = pairs[2 * p], j = pairs[2 * p + 1];
    const double *blk = Jp + (size_t)p * q * q; /* (state of i, state of j) */
    int a = off[i] + fill[i]++;
    aj[a] = j; at[a] = 0; ab[a] = blk;
    a = off[j] + fill[j]++;
    aj[a] = i; at[a] = 1; ab[a] = blk;
  }
  gibbs_ctx g = {N, q, B, nchains, burnin, thin, seed, h, off, aj, at, ab, msa};
  gibbs_pool pool = {&g, 0, PTHREAD_MUTEX_INITIALIZER};
  if (nthreads < 1) nthreads = 1;
  if (nthreads > nchains) nthreads = nchains;
  pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)nthreads);
  int started = 0;
  for (int t = 0; t < nthreads; ++t)
    if (pthread_create(&th[t], NULL, gibbs_worker, &pool) == 0) ++started;
  if (started == 0) gibbs_worker(&pool);
  for (int t = 0; t < started; ++t) pthread_join(th[t], NULL);
  free(th); free(deg); free(off); free(fill); free(aj); free(at); free(ab);
}

/* Each cell independently replaced by `gap` with probability p. */
void synth_force_gaps(uint64_t seed, int B, int N, double p, uint8_t gap, uint8_t *msa) {
  rng_t r;
  rng_seed(&r, seed, STREAM_GAPS);
  for (size_t e = 0; e < (size_t)B * N; ++e)
    if (rng_uniform(&r) < p) msa[e] = gap;
}

/* Independent uniform draws in [0,1), for tests that need seeded noise. */
void synth_uniform(uint64_t seed, uint64_t stream, int64_t n, double *out) {
  rng_t r;
  rng_seed(&r, seed, stream);
  for (int64_t e = 0; e < n; ++e) out[e] = rng_uniform(&r);
}
