// k_lbfgs.hip -- device-resident limited-memory BFGS for all N per-site
// problems of asymmetric plmDCA (sec. 3.4 step 3; the paper minimises each
// g_r^reg by L-BFGS from the origin, secs. 5 and 6).
//
// One iteration of every active site is six launches:
//   lbfgs_eval_kernel    kLbChunks blocks per site: the regulariser and the
//                        squared gradient norm at the trial point over a
//                        contiguous range of the site's parameters (FP64
//                        partial sums; the objective's data part is the
//                        forward kernel's FP64 tile sums);
//   lbfgs_decide_kernel  one block per site: the partials added in chunk
//                        order, the line-search decision (sufficient decrease
//                        with backtracking by safeguarded quadratic
//                        interpolation) and the action the next pass takes;
//   lbfgs_update_kernel  kLbChunks blocks per site: on acceptance the
//                        candidate curvature pair (s, y) into the free history
//                        slot, the gradient kept at the iterate and the iterate
//                        itself, with the partial dot products of s, y, g and
//                        the stored pairs; otherwise the backtracking or
//                        steepest-descent trial point;
//   lbfgs_coef_kernel    one block per site: the products added in chunk
//                        order, the curvature test, the small matrices of the
//                        compact form and the coefficients of the next
//                        direction;
//   lbfgs_dir_kernel     kLbChunks blocks per site: the direction, the trial
//                        point at step 1 and partial sums of d . g;
//   lbfgs_dir_finish_kernel one block per site: the descent test.
// Every sum is formed in a fixed order (per-thread strided sums, a shuffle
// tree per wave, waves in order, chunks in order) and the partition depends
// only on the site's size, so a site's iterates do not depend on the batch
// or on the number of active sites.
//
// Arithmetic: all dot products, the small matrices, the objective and the
// gradient at the trial point are FP64.  The iterate and the trial point are
// FP32, the values the evaluation kernels read (the evaluated point and the
// stored point are the same).  The stored curvature pairs and the gradient
// kept at the iterate are FP32 by default (their entries are differences of
// gradients that carry the FP32 evaluation's rounding, far above FP32 storage
// rounding; half the bytes of this streaming code) or FP64 (HT = double,
// plm_fit_opts.history_fp64); the dot products of a stored pair are those of
// the stored values, so the compact form stays consistent with what the
// direction is formed from.  The direction is FP32 (the step along it is
// rounded to the FP32 trial point anyway).
//
// The search direction d = -H g uses the compact representation of the
// limited-memory inverse Hessian (Byrd, Nocedal and Schnabel, 1994), which
// gives the same direction as the two-loop recursion: with the n stored pairs
// in chronological order, R = upper triangle of S^T Y, D = its diagonal and
// gamma the scaling of the newest pair,
//   H g = gamma g + S q1 - gamma Y t,   R t = S^T g,
//   R^T q1 = (D + gamma Y^T Y) t - gamma Y^T g.
// S^T Y and Y^T Y are kept per site and gain one column per accepted pair, so
// an accepted step streams the history twice (one pass of dot products, one
// pass forming d) instead of the 2m passes of the two-loop recursion.  S^T g
// and Y^T g are kept per site as well and updated by the same column
// (s_j . g_new = s_j . g_old + s_j . y), so the dot-product pass needs two
// products per stored pair and no gradient.  The history has m + 1 slots, so
// that a candidate pair can be written before the curvature test decides
// whether it is kept.
#include "plm_internal.h"

namespace plm {

constexpr int kLbThreads = 256;
constexpr int kLbWaves = kLbThreads / 64;
constexpr int kGroupA = 4;  // stored pairs whose products ride on the acceptance pass
constexpr int kGroupB = 6;  // stored pairs per further pass over the chunk
constexpr int kVecMax = 4 + 2 * kGroupA > 2 * kGroupB ? 4 + 2 * kGroupA : 2 * kGroupB;  // widest block sum
constexpr int kSlotsMax = kMMax + 1;
static_assert(kLbPartW >= 4 + 2 * kMMax, "partial sums of the candidate and of every stored pair");

// the actions lbfgs_decide_kernel leaves for the update pass
enum { ACT_NONE = 0, ACT_INIT = 1, ACT_PAIR = 2, ACT_FINAL = 3, ACT_BACKTRACK = 4, ACT_STEEPEST = 5 };
// dpend: the direction the direction kernels form
enum { DIR_NONE = 0, DIR_QN = 1, DIR_STEEPEST = 2 };

// Block sums of NV per-thread FP64 values (fixed order: a shuffle tree per
// wave, then the waves in order); thread 0 gets the sums.
template <int NV>
__device__ inline void block_sum_vec(double (&v)[NV], double* red) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k)
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v[k] += __shfl_xor(v[k], o, 64);
  __syncthreads();
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < NV; ++k) red[wid * NV + k] = v[k];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double t = 0.0;
      for (int w = 0; w < kLbWaves; ++w) t += red[w * NV + k];
      v[k] = t;
    }
  __syncthreads();
}

// The site of a block of a per-site kernel (idx: position in the active list).
struct SiteOf {
  LbfgsArgs a;
  int r;
  bool ok;
  __device__ SiteOf(const BatchArgs& b, int idx) {
    ok = idx < *b.n_active;
    if (!ok) return;
    const int g = __builtin_amdgcn_readfirstlane(b.active[idx]);
    const int m = __builtin_amdgcn_readfirstlane(b.msa_of[g]);
    a = load_uniform(b.lb + m);
    r = __builtin_amdgcn_readfirstlane(g - b.site_base[m]);
  }
};

// A site's vectors, addressed by the element index e of its parameter vector
// (fields e < q, then the couplings e = q + o of its row, o = (i, k, s)).
template <typename HT>
struct Vecs {
  int q, N, P, self0, self1;
  size_t h0, j0, hs, js;  // field and coupling offsets of the site, history slot strides
  double ib, lam_h, lam_J;
  const LbfgsArgs* ap;
  __attribute__((address_space(1))) float *Xh, *XJ, *Th, *TJ, *Dh, *DJ;
  __attribute__((address_space(1))) HT *Gh, *GJ, *Sh, *SJ, *Yh, *YJ;
  const __attribute__((address_space(1))) double* gJd;
  __device__ Vecs(const LbfgsArgs& a, int r) {
    ap = &a;
    q = a.q;
    N = a.N;
    const size_t Nqq = (size_t)N * q * q;
    P = q + (int)Nqq;
    h0 = (size_t)r * q;
    j0 = (size_t)r * Nqq;
    hs = (size_t)N * q;
    js = (size_t)N * Nqq;
    self0 = q + r * q * q;
    self1 = self0 + q * q;
    ib = 1.0 / *a.beff;
    lam_h = a.lambda_h;
    lam_J = a.lambda_Jp;
    Xh = gmem_w(a.Xh); XJ = gmem_w(a.XJ); Th = gmem_w(a.Th); TJ = gmem_w(a.TJ);
    Dh = gmem_w(a.Dh); DJ = gmem_w(a.DJ);
    Gh = gmem_w((HT*)a.Gh); GJ = gmem_w((HT*)a.GJ);
    Sh = gmem_w((HT*)a.Sh); SJ = gmem_w((HT*)a.SJ); Yh = gmem_w((HT*)a.Yh); YJ = gmem_w((HT*)a.YJ);
    gJd = gmem(a.gJ);
  }
  __device__ double lam(int e) const { return e < q ? lam_h : ((e >= self0 && e < self1) ? 0.0 : lam_J); }
  __device__ float T(int e) const { return e < q ? Th[h0 + e] : TJ[j0 + (e - q)]; }
  __device__ float X(int e) const { return e < q ? Xh[h0 + e] : XJ[j0 + (e - q)]; }
  __device__ float D(int e) const { return e < q ? Dh[h0 + e] : DJ[j0 + (e - q)]; }
  __device__ HT G(int e) const { return e < q ? Gh[h0 + e] : GJ[j0 + (e - q)]; }
  __device__ __attribute__((address_space(1))) HT* Sp(int k, int e) const {
    return e < q ? Sh + k * hs + h0 + e : SJ + k * js + j0 + (e - q);
  }
  __device__ __attribute__((address_space(1))) HT* Yp(int k, int e) const {
    return e < q ? Yh + k * hs + h0 + e : YJ + k * js + j0 + (e - q);
  }
  __device__ void setX(int e, float v) const {
    if (e < q) Xh[h0 + e] = v; else XJ[j0 + (e - q)] = v;
  }
  __device__ void setG(int e, HT v) const {
    if (e < q) Gh[h0 + e] = v; else GJ[j0 + (e - q)] = v;
  }
  __device__ void setD(int e, float v) const {
    if (e < q) Dh[h0 + e] = v; else DJ[j0 + (e - q)] = v;
  }
  // the trial point, FP32; the self block stays zero
  __device__ void setT(int e, double v) const {
    const float f = (float)v;
    if (e < q) Th[h0 + e] = f; else TJ[j0 + (e - q)] = (e >= self0 && e < self1) ? 0.f : f;
  }
  // data part of the gradient at the trial point (fields: the forward's tile
  // sums, added once per evaluation by the eval pass into ghd)
  __device__ double gdata(int e, int r) const {
    return e >= q ? gJd[j0 + (e - q)] : gmem(ap->ghd)[(size_t)r * q + e];
  }
  // the forward's tile sums of field e (fixed order)
  __device__ double field_tiles(int e, int r) const {
    double t = 0.0;
#pragma unroll 8
    for (int k = 0; k < ap->tiles; ++k) t += gmem(ap->gh_part)[((size_t)k * N + r) * kSlot + e];
    return t;
  }
  // the full (normalised) gradient at the trial point
  __device__ double g(int e, int r, float t) const { return gdata(e, r) * ib + 2.0 * lam(e) * (double)t; }
  // the chunk's element range
  __device__ void chunk(int c, int& beg, int& end) const {
    const int csz = (P + kLbChunks - 1) / kLbChunks;
    beg = min(P, c * csz);
    end = min(P, beg + csz);
  }
};

__device__ inline double* site_part(const LbfgsArgs& a, int r, int chunk) {
  return a.part + ((size_t)r * kLbChunks + chunk) * kLbPartW;
}

// ---- regulariser and gradient norm at the trial point -------------------------
__global__ __launch_bounds__(kLbThreads) void lbfgs_eval_kernel(BatchArgs b) {
  __shared__ double red[kLbWaves * 3];
  const int idx = blockIdx.x / kLbChunks, chunk = blockIdx.x - idx * kLbChunks;
  const SiteOf so(b, idx);
  if (!so.ok) return;
  const LbfgsArgs& a = so.a;
  const int r = so.r;
  if (__builtin_amdgcn_readfirstlane(a.st[r].phase) == PH_DONE) return;
  const Vecs<float> v(a, r);
  int beg, end;
  v.chunk(chunk, beg, end);
  double acc[3] = {0.0, 0.0, 0.0};  // regulariser, squared gradient norm, objective data part
  const int tid = threadIdx.x;
  const int q = v.q;
  if (beg < q) {
    // the fields (the first chunk holds them all unless the site is tiny): their
    // data part is the sum of the forward's tile partials, kept for the update pass
    for (int e = beg + tid; e < min(end, q); e += kLbThreads) {
      const double gd = v.field_tiles(e, r);
      gmem_w(a.ghd)[(size_t)r * q + e] = gd;
      const float t = v.T(e);
      const double g = gd * v.ib + 2.0 * v.lam_h * (double)t;
      acc[0] += v.lam_h * (double)t * (double)t;
      acc[1] += g * g;
    }
    if (tid == 0 && chunk == 0) {
      double fd = 0.0;
#pragma unroll 8
      for (int k = 0; k < a.tiles; ++k) fd += gmem(a.f_part)[(size_t)k * a.N + r];
      acc[2] = fd;
    }
  }
  // the couplings, four per thread at a time so that their loads are in flight together
  const int cb = max(beg, q);
  constexpr int U = 4;
  for (int e0 = cb + tid; e0 < end; e0 += U * kLbThreads) {
    float t[U];
    double gd[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = min(e0 + u * kLbThreads, end - 1);
      t[u] = v.TJ[v.j0 + (e - q)];
      gd[u] = v.gJd[v.j0 + (e - q)];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = e0 + u * kLbThreads;
      if (e < end) {
        const double lo = v.lam(e);
        const double g = gd[u] * v.ib + 2.0 * lo * (double)t[u];
        acc[0] += lo * (double)t[u] * (double)t[u];
        acc[1] += g * g;
      }
    }
  }
  block_sum_vec(acc, red);
  if (threadIdx.x == 0) {
    double* p = site_part(a, r, chunk);
    p[0] = acc[0];
    p[1] = acc[1];
    p[2] = acc[2];
  }
}

// ---- the line-search decision, one block per site ------------------------------
__global__ __launch_bounds__(64) void lbfgs_decide_kernel(BatchArgs b) {
  const SiteOf so(b, blockIdx.x);
  if (!so.ok || threadIdx.x != 0) return;
  const LbfgsArgs& a = so.a;
  const int r = so.r;
  SiteState* S = a.st + r;
  const int phase = S->phase;
  if (phase == PH_DONE) return;
  double reg = 0.0, gg = 0.0, fdata = 0.0;
  for (int c = 0; c < kLbChunks; ++c) {
    const double* p = site_part(a, r, c);
    reg += p[0];
    gg += p[1];
    fdata += p[2];
  }
  const double ib = 1.0 / *a.beff;
  const double ft = fdata * ib + reg;
  const double gnt = sqrt(gg);
  const bool finite = isfinite(ft) && isfinite(gnt);

  int evals = S->evals + 1;
  int iter = S->iter, ls = S->ls_count, status = S->status, stored = S->stored;
  double f = S->f, gnorm = S->gnorm, alpha = S->alpha, gtd = S->gtd;
  int newphase = phase, act = ACT_NONE;
  if (phase == PH_INIT && !finite) {
    newphase = PH_DONE;
    status = PLM_SITE_NONFINITE;
  } else if (phase == PH_INIT || (finite && ft <= f + a.c1 * alpha * gtd + a.noise * fabs(f))) {
    // accept the trial point (the first evaluation is the start point itself);
    // sufficient decrease allows for the rounding noise of the FP32 evaluation
    const bool pair = phase != PH_INIT;
    if (pair) ++iter;
    f = ft;
    gnorm = gnt;
    ls = 0;
    if (gnorm <= a.tol) {
      newphase = PH_DONE;
      status = PLM_SITE_CONVERGED;
      act = ACT_FINAL;
    } else if (iter >= a.max_iter) {
      newphase = PH_DONE;
      status = PLM_SITE_MAXITER;
      act = ACT_FINAL;
    } else {
      newphase = PH_LS;
      if (pair) {
        act = ACT_PAIR;  // the direction follows from the curvature test (lbfgs_coef_kernel)
      } else {
        act = ACT_INIT;  // steepest descent from the start point
        stored = 0;
        gtd = -gnorm * gnorm;
        alpha = fmin(1.0, 1.0 / gnorm);
      }
    }
  } else {
    // reject: backtrack along the same direction
    ++ls;
    newphase = PH_LS;
    if (ls > a.max_ls) {
      if (stored > 0) {  // forget the history once, restart from steepest descent
        act = ACT_STEEPEST;
        ls = 0;
        stored = 0;
        gtd = -gnorm * gnorm;
        alpha = fmin(1.0, 1.0 / gnorm);
      } else {
        newphase = PH_DONE;
        status = PLM_SITE_LINESEARCH;
      }
    } else {
      // minimiser of the quadratic through f, slope gtd and f(alpha), kept in [0.1, 0.5] alpha
      double an = 0.5 * alpha;
      if (finite) {
        const double den = 2.0 * (ft - f - gtd * alpha);
        if (den > 0.0) an = -gtd * alpha * alpha / den;
        an = fmin(fmax(an, 0.1 * alpha), 0.5 * alpha);
      }
      alpha = an;
      act = ACT_BACKTRACK;
    }
  }
  S->phase = newphase;
  S->status = status;
  S->iter = iter;
  S->evals = evals;
  S->ls_count = ls;
  S->stored = stored;
  S->action = act;
  S->dpend = DIR_NONE;
  S->f = f;
  S->gnorm = gnorm;
  S->alpha = alpha;
  S->gtd = gtd;
  if (a.phase_host) a.phase_host[r] = newphase;
}

// ---- the update pass, kLbChunks blocks per site --------------------------------
template <typename HT>
__global__ __launch_bounds__(kLbThreads) void lbfgs_update_kernel(BatchArgs b) {
  __shared__ double red[kLbWaves * kVecMax];
  const int idx = blockIdx.x / kLbChunks, chunk = blockIdx.x - idx * kLbChunks;
  const SiteOf so(b, idx);
  if (!so.ok) return;
  const LbfgsArgs& a = so.a;
  const int r = so.r;
  const SiteState* S = a.st + r;
  const int act = __builtin_amdgcn_readfirstlane(S->action);
  if (act == ACT_NONE) return;
  const Vecs<HT> v(a, r);
  int beg, end;
  v.chunk(chunk, beg, end);
  const int tid = threadIdx.x;
  if (act == ACT_BACKTRACK) {
    const double alpha = S->alpha;
    for (int e = beg + tid; e < end; e += kLbThreads) v.setT(e, (double)v.X(e) + alpha * (double)v.D(e));
    return;
  }
  if (act == ACT_STEEPEST) {
    const double alpha = S->alpha;
    for (int e = beg + tid; e < end; e += kLbThreads) {
      const float d = (float)-(double)v.G(e);
      v.setD(e, d);
      v.setT(e, (double)v.X(e) + alpha * (double)d);
    }
    return;
  }
  if (act == ACT_FINAL) {  // the accepted point becomes the iterate
    for (int e = beg + tid; e < end; e += kLbThreads) v.setX(e, v.T(e));
    return;
  }
  if (act == ACT_INIT) {  // gradient and iterate at the start point, then steepest descent
    const double alpha = S->alpha;
    for (int e = beg + tid; e < end; e += kLbThreads) {
      const float t = v.T(e);
      const HT gs = (HT)v.g(e, r, t);
      v.setG(e, gs);
      v.setX(e, t);
      const float d = (float)-(double)gs;
      v.setD(e, d);
      v.setT(e, (double)t + alpha * (double)d);
    }
    return;
  }
  // ACT_PAIR: the candidate pair into the free slot `head`, the gradient and
  // the iterate at the accepted point, and the products of s, y, g with the
  // stored pairs (newest first), kGroupA pairs on this pass and kGroupB on
  // each further pass over the chunk (y re-read from the slot just written)
  const int M = a.m + 1;
  const int head = __builtin_amdgcn_readfirstlane(S->head);
  const int stored = __builtin_amdgcn_readfirstlane(S->stored);
  const int nA = min(stored, kGroupA);
  double* part = site_part(a, r, chunk);
  auto accept_pass = [&](auto na_c) {
    constexpr int NA = decltype(na_c)::value;
    int kk[NA > 0 ? NA : 1];
#pragma unroll
    for (int j = 0; j < NA; ++j) kk[j] = (head - 1 - j + 2 * M) % M;
    double acc[4 + 2 * kGroupA];
#pragma unroll
    for (int k = 0; k < 4 + 2 * kGroupA; ++k) acc[k] = 0.0;
    // two elements per thread at a time (e, e + nth), all their loads issued together
    constexpr int U = 2;
    constexpr int NA1 = NA > 0 ? NA : 1;
    for (int e0 = beg + tid; e0 < end; e0 += U * kLbThreads) {
      int ee[U];
      float t[U], x[U];
      HT gold[U], sl[U][NA1], yl[U][NA1];
      double gd[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        ee[u] = min(e0 + u * kLbThreads, end - 1);
        t[u] = v.T(ee[u]);
        x[u] = v.X(ee[u]);
        gold[u] = v.G(ee[u]);
        gd[u] = v.gdata(ee[u], r);
#pragma unroll
        for (int j = 0; j < NA; ++j) {
          sl[u][j] = *v.Sp(kk[j], ee[u]);
          yl[u][j] = *v.Yp(kk[j], ee[u]);
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (e0 + u * kLbThreads >= end) continue;
        const int e = ee[u];
        const double g = gd[u] * v.ib + 2.0 * v.lam(e) * (double)t[u];
        // stored as HT and used as stored
        const HT svs = (HT)((double)t[u] - (double)x[u]), yvs = (HT)(g - (double)gold[u]);
        *v.Sp(head, e) = svs;
        *v.Yp(head, e) = yvs;
        const double sv = svs, yv = yvs;
        acc[0] += sv * yv;
        acc[1] += yv * yv;
        acc[2] += sv * g;
        acc[3] += yv * g;
#pragma unroll
        for (int j = 0; j < NA; ++j) {
          acc[4 + 2 * j] += (double)sl[u][j] * yv;
          acc[5 + 2 * j] += (double)yl[u][j] * yv;
        }
        v.setG(e, (HT)g);
        v.setX(e, t[u]);
      }
    }
    block_sum_vec(acc, red);
    if (tid == 0)
#pragma unroll
      for (int k = 0; k < 4 + 2 * NA; ++k) part[k] = acc[k];
  };
  with_count<0, kGroupA>(nA, accept_pass);
  for (int jg = kGroupA; jg < stored; jg += kGroupB) {
    const int nB = min(kGroupB, stored - jg);
    auto pair_pass = [&](auto nb_c) {
      constexpr int NB = decltype(nb_c)::value;
      int kk[NB];
#pragma unroll
      for (int j = 0; j < NB; ++j) kk[j] = (head - 1 - (jg + j) + 2 * M) % M;
      double acc[2 * kGroupB];
#pragma unroll
      for (int k = 0; k < 2 * kGroupB; ++k) acc[k] = 0.0;
      constexpr int U = 2;
      for (int e0 = beg + tid; e0 < end; e0 += U * kLbThreads) {
        int ee[U];
        HT yh[U], sl[U][NB], yl[U][NB];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          ee[u] = min(e0 + u * kLbThreads, end - 1);
          yh[u] = *v.Yp(head, ee[u]);
#pragma unroll
          for (int j = 0; j < NB; ++j) {
            sl[u][j] = *v.Sp(kk[j], ee[u]);
            yl[u][j] = *v.Yp(kk[j], ee[u]);
          }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          if (e0 + u * kLbThreads >= end) continue;
          const double yv = (double)yh[u];
#pragma unroll
          for (int j = 0; j < NB; ++j) {
            acc[2 * j] += (double)sl[u][j] * yv;
            acc[2 * j + 1] += (double)yl[u][j] * yv;
          }
        }
      }
      block_sum_vec(acc, red);
      if (tid == 0)
#pragma unroll
        for (int k = 0; k < 2 * NB; ++k) part[4 + 2 * jg + k] = acc[k];
    };
    with_count<1, kGroupB>(nB, pair_pass);
  }
}

// ---- products, curvature test and the next direction's coefficients -------------
struct CoefShared {
  double vals[4 + 2 * kMMax];
  double Rm[kMMax * kMMax];   // S^T Y and Y^T Y of the stored pairs, chronological order
  double YYm[kMMax * kMMax];
  double cs[kMMax];           // direction coefficients of s and y, chronological order
  double cy[kMMax];
  double tv[kMMax];
  double p1[kSlotsMax];       // s_j . g and y_j . g of the stored pairs, newest first
  double p2[kSlotsMax];
  int32_t ord[kMMax];         // slots of the stored pairs, oldest first
  double gamma;               // thread 0's results, for every thread
  int32_t head, stored;
};

__global__ __launch_bounds__(256) void lbfgs_coef_kernel(BatchArgs b) {
  __shared__ CoefShared sh;
  const SiteOf so(b, blockIdx.x);
  if (!so.ok) return;
  const LbfgsArgs& a = so.a;
  const int r = so.r;
  SiteState* S = a.st + r;
  if (__builtin_amdgcn_readfirstlane(S->action) != ACT_PAIR) return;
  const int tid = threadIdx.x, nth = blockDim.x;
  const int m = a.m, M = m + 1;
  int head = __builtin_amdgcn_readfirstlane(S->head), stored = __builtin_amdgcn_readfirstlane(S->stored);
  const auto StY = gmem_w(a.small + (size_t)r * 2 * M * (M + 1));  // [M][M] s_i . y_j by slot
  const auto YtY = StY + (size_t)M * M;                             // [M][M] y_i . y_j by slot
  const auto SG = YtY + (size_t)M * M;                              // [M] s_k . G by slot
  const auto YG = SG + M;                                           // [M] y_k . G by slot
  const int nv = 4 + 2 * stored;
  for (int k = tid; k < nv; k += nth) {
    double t = 0.0;
    for (int c = 0; c < kLbChunks; ++c) t += site_part(a, r, c)[k];
    sh.vals[k] = t;
  }
  __syncthreads();
  double gamma = S->gamma;
  if (tid == 0) {
    const double sy = sh.vals[0], yy = sh.vals[1];
    // S^T g and Y^T g at the new point: the stored products moved by the
    // candidate's y (G changes by y whether or not the pair is kept)
    for (int j = 0; j < stored; ++j) {
      const int k = (head - 1 - j + 2 * M) % M;
      const double pg1 = SG[k] + sh.vals[4 + 2 * j], pg2 = YG[k] + sh.vals[5 + 2 * j];
      SG[k] = pg1;
      YG[k] = pg2;
      sh.p1[j] = pg1;
      sh.p2[j] = pg2;
    }
    if (sy > 0.0 && yy > 0.0) {
      // keep the candidate: its column of S^T Y and its row/column of Y^T Y;
      // it becomes the newest pair (index 0 of the newest-first lists)
      const int c = head;
      for (int j = 0; j < stored; ++j) {
        const int k = (head - 1 - j + 2 * M) % M;
        StY[k * M + c] = sh.vals[4 + 2 * j];
        YtY[k * M + c] = sh.vals[5 + 2 * j];
        YtY[c * M + k] = sh.vals[5 + 2 * j];
      }
      StY[c * M + c] = sy;
      YtY[c * M + c] = yy;
      for (int j = min(stored, m - 1); j > 0; --j) {
        sh.p1[j] = sh.p1[j - 1];
        sh.p2[j] = sh.p2[j - 1];
      }
      sh.p1[0] = sh.vals[2];
      sh.p2[0] = sh.vals[3];
      SG[c] = sh.vals[2];
      YG[c] = sh.vals[3];
      gamma = sy / yy;
      head = (head + 1) % M;
      if (stored < m) ++stored;
    }
    sh.gamma = gamma;
    sh.head = head;
    sh.stored = stored;
  }
  __syncthreads();
  head = __builtin_amdgcn_readfirstlane(sh.head);
  stored = __builtin_amdgcn_readfirstlane(sh.stored);
  gamma = sh.gamma;
  if (stored == 0) {
    // no pair: steepest descent from the new iterate (formed by the direction kernels)
    if (tid == 0) {
      const double gn = S->gnorm;
      S->head = head;
      S->stored = 0;
      S->gamma = gamma;
      S->gtd = -gn * gn;
      S->alpha = fmin(1.0, 1.0 / gn);
      S->dpend = DIR_STEEPEST;
    }
    return;
  }
  // the compact form over the n stored pairs, in chronological order
  const int n = stored;
  if (tid < n) sh.ord[tid] = (head - n + tid + 2 * M) % M;
  __syncthreads();
  for (int e = tid; e < n * n; e += nth) {
    const int i = e / n, j = e - i * n;
    sh.Rm[e] = i <= j ? StY[sh.ord[i] * M + sh.ord[j]] : 0.0;
    sh.YYm[e] = YtY[sh.ord[i] * M + sh.ord[j]];
  }
  __syncthreads();
  if (tid == 0) {
    // R t = S^T g (back substitution); p1, p2 are newest first
    for (int i = n - 1; i >= 0; --i) {
      double x = sh.p1[n - 1 - i];
      for (int l = i + 1; l < n; ++l) x -= sh.Rm[i * n + l] * sh.tv[l];
      sh.tv[i] = x / sh.Rm[i * n + i];
    }
    // R^T q1 = D t + gamma Y^T Y t - gamma Y^T g (forward substitution), q1 in cs
    for (int i = 0; i < n; ++i) {
      double yyt = 0.0;
      for (int l = 0; l < n; ++l) yyt += sh.YYm[i * n + l] * sh.tv[l];
      double x = sh.Rm[i * n + i] * sh.tv[i] + gamma * (yyt - sh.p2[n - 1 - i]);
      for (int l = 0; l < i; ++l) x -= sh.Rm[l * n + i] * sh.cs[l];
      sh.cs[i] = x / sh.Rm[i * n + i];
    }
    // d = -gamma g - S q1 + gamma Y t
    for (int i = 0; i < n; ++i) {
      sh.cs[i] = -sh.cs[i];
      sh.cy[i] = gamma * sh.tv[i];
    }
  }
  __syncthreads();
  DirCoef* C = a.dc + r;
  if (tid < n) {
    C->cs[tid] = sh.cs[tid];
    C->cy[tid] = sh.cy[tid];
    C->ord[tid] = sh.ord[tid];
  }
  if (tid == 0) {
    C->n = n;
    C->gamma = gamma;
    S->head = head;
    S->stored = stored;
    S->gamma = gamma;
    S->dpend = DIR_QN;
  }
}

// ---- the direction, kLbChunks blocks per site ------------------------------------
// The pending quasi-Newton direction over a contiguous range of the site's
// elements: d, the trial point X + d (step 1) and the block's partial sum of
// d . G.  A pending steepest-descent direction: d = -G and the trial point at
// the site's step.
template <typename HT>
__global__ __launch_bounds__(kLbThreads) __attribute__((amdgpu_waves_per_eu(6))) void lbfgs_dir_kernel(BatchArgs b) {
  __shared__ double cs[kMMax], cy[kMMax];
  __shared__ int32_t ord[kMMax];
  __shared__ double red[kLbWaves];
  const int idx = blockIdx.x / kLbChunks, chunk = blockIdx.x - idx * kLbChunks;
  const SiteOf so(b, idx);
  if (!so.ok) return;
  const LbfgsArgs& a = so.a;
  const int r = so.r;
  const int pend = __builtin_amdgcn_readfirstlane(a.st[r].dpend);
  if (pend == DIR_NONE) return;
  const Vecs<HT> v(a, r);
  int beg, end;
  v.chunk(chunk, beg, end);
  const int tid = threadIdx.x;
  if (pend == DIR_STEEPEST) {
    const double alpha = a.st[r].alpha;
    for (int e = beg + tid; e < end; e += kLbThreads) {
      const float d = (float)-(double)v.G(e);
      v.setD(e, d);
      v.setT(e, (double)v.X(e) + alpha * (double)d);
    }
    return;
  }
  const DirCoef* C = a.dc + r;
  const int n = __builtin_amdgcn_readfirstlane(C->n);
  const double gamma = C->gamma;
  if (tid < n) {
    cs[tid] = C->cs[tid];
    cy[tid] = C->cy[tid];
    ord[tid] = C->ord[tid];
  }
  __syncthreads();
  // four elements per thread at a time (e, e + nth, e + 2 nth, e + 3 nth),
  // so that the history loads of four elements are in flight together
  double dg = 0.0;
  constexpr int U = sizeof(HT) == 4 ? 4 : 2;
  for (int e0 = beg + tid; e0 < end; e0 += U * kLbThreads) {
    int ee[U];
    double gv[U], d[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      ee[u] = min(e0 + u * kLbThreads, end - 1);
      gv[u] = (double)v.G(ee[u]);
      d[u] = -gamma * gv[u];
    }
#pragma unroll 2
    for (int i = 0; i < n; ++i) {
      const int k = ord[i];
      const double ci = cs[i], yi = cy[i];
      double sv[U], yv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        sv[u] = (double)*v.Sp(k, ee[u]);
        yv[u] = (double)*v.Yp(k, ee[u]);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) d[u] += ci * sv[u] + yi * yv[u];
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (e0 + u * kLbThreads < end) {
        v.setD(ee[u], (float)d[u]);
        v.setT(ee[u], (double)v.X(ee[u]) + d[u]);  // trial point at alpha = 1
        dg += d[u] * gv[u];
      }
  }
  dg = block_sum_f64(dg, red);
  if (tid == 0) a.dpart[(size_t)r * kLbChunks + chunk] = dg;
}

// The descent test of every pending quasi-Newton direction (the block sums of
// d . g added in chunk order); where d is not a descent direction, steepest
// descent from the iterate with the history forgotten.
template <typename HT>
__global__ __launch_bounds__(kLbThreads) void lbfgs_dir_finish_kernel(BatchArgs b) {
  const SiteOf so(b, blockIdx.x);
  if (!so.ok) return;
  const LbfgsArgs& a = so.a;
  const int r = so.r;
  SiteState* S = a.st + r;
  const int pend = __builtin_amdgcn_readfirstlane(S->dpend);
  __syncthreads();  // every wave has read the flag before it is cleared
  if (pend == DIR_NONE) return;
  const int tid = threadIdx.x;
  if (pend == DIR_STEEPEST) {
    if (tid == 0) S->dpend = DIR_NONE;
    return;
  }
  double dg = 0.0;
  for (int c = 0; c < kLbChunks; ++c) dg += a.dpart[(size_t)r * kLbChunks + c];
  if (dg < 0.0) {
    if (tid == 0) {
      S->gtd = dg;
      S->alpha = 1.0;
      S->dpend = DIR_NONE;
    }
    return;
  }
  const double gnorm = S->gnorm;
  const double alpha = fmin(1.0, 1.0 / gnorm);
  const Vecs<HT> v(a, r);
  for (int e = tid; e < v.P; e += kLbThreads) {
    const float d = (float)-(double)v.G(e);
    v.setD(e, d);
    v.setT(e, (double)v.X(e) + alpha * (double)d);
  }
  if (tid == 0) {
    S->gtd = -gnorm * gnorm;
    S->alpha = alpha;
    S->stored = 0;
    S->dpend = DIR_NONE;
  }
}

template <typename HT>
hipError_t launch_lbfgs_t(const BatchArgs& b, int32_t nblocks, hipStream_t st) {
  hipLaunchKernelGGL(lbfgs_eval_kernel, dim3(nblocks * kLbChunks), dim3(kLbThreads), 0, st, b);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(lbfgs_decide_kernel, dim3(nblocks), dim3(64), 0, st, b);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(lbfgs_update_kernel<HT>, dim3(nblocks * kLbChunks), dim3(kLbThreads), 0, st, b);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(lbfgs_coef_kernel, dim3(nblocks), dim3(256), 0, st, b);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(lbfgs_dir_kernel<HT>, dim3(nblocks * kLbChunks), dim3(kLbThreads), 0, st, b);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(lbfgs_dir_finish_kernel<HT>, dim3(nblocks), dim3(kLbThreads), 0, st, b);
  return hipGetLastError();
}

hipError_t launch_lbfgs(const BatchArgs& b, int32_t nblocks, int32_t history_fp64, hipStream_t st) {
  return history_fp64 ? launch_lbfgs_t<double>(b, nblocks, st) : launch_lbfgs_t<float>(b, nblocks, st);
}

}  // namespace plm
