// k_sym.hip -- symmetric pseudolikelihood maximization (eqs. npll_1, l2reg):
// one minimisation of F = sum_r g_r + lambda_h sum_i ||h_i||^2 +
// lambda_J sum_{i<j} ||J_ij||^2 over all fields and couplings, each J_ij
// shared by g_i and g_j.
//
// The couplings live in the asymmetric layout J[r][i][k][s] (s the state of
// r), filled consistently: J[i][r] is J[r][i] with the state axes swapped.
// Optionally every parameter carries an FP32 low-order word (the parameter is
// hi + lo in FP64): the optimiser forms iterates and trial points in FP64 and
// stores them as such pairs, and the precise evaluation reads both words.
// The parameters are h and the blocks J[r][i], r < i.  Every iteration
// evaluates all N sites with the batch kernels (forward and gradient), then
// a fixed sequence of kernels runs one limited-memory BFGS step for the whole
// vector with every decision taken on the device (so that one iteration is
// one replay of a captured graph):
//   eval    block partial sums of the l2 term and of |grad F|^2 at the trial point
//   decide  (one block) objective, sufficient-decrease test, backtracking step
//   accept  on acceptance: gradient G, candidate pair (s, y), iterate X, and the
//           dot products of the pair and the newest stored pairs with y and g
//   group   further dot products, four stored pairs per launch
//   solve   (one block) curvature test, S^T Y / Y^T Y update, compact-form
//           coefficients of the direction (as in the per-site optimiser)
//   direct  d = -gamma g + S a + Y b, trial point X + d, partial sums of d.g
//   check   (one block) descent test, else steepest descent
//   move    steepest-descent or backtracking trial point
//   finish  (one block) counters, done flag, work tables of the next evaluation
// The gradient of a shared block is the sum of the site-r gradient and the
// transposed site-i gradient.  All sums over blocks have a fixed order.
#include "plm_internal.h"

namespace plm {

constexpr int kSymThreads = 256;
constexpr int kSymGroup = 4;
constexpr int kSymPart = 4 + 4 * kSymGroup;

enum { SD_KEEP = 0, SD_STEEPEST = 1, SD_QN = 2 };

// Visit every parameter: unit u < N is the field h_u (q entries), unit N + p
// the coupling block of pair p = (r, i), r < i (q^2 entries, with the mirror
// index of each entry).  Units are spread over the blocks, entries over the
// threads of a block.
template <class F>
__device__ inline void for_each_param(const SymArgs& a, F&& f) {
  const int q = a.q, qq = q * q, N = a.N;
  const int nunits = N + a.npairs;
  for (int u = blockIdx.x; u < nunits; u += gridDim.x) {
    if (u < N) {
      for (int s = threadIdx.x; s < q; s += blockDim.x) f(true, (size_t)u * q + s, (size_t)0);
    } else {
      const int2 pr = a.pairs[u - N];
      const size_t base = ((size_t)pr.x * N + pr.y) * qq, mbase = ((size_t)pr.y * N + pr.x) * qq;
      for (int t = threadIdx.x; t < qq; t += blockDim.x) {
        const int k = t / q, s = t - k * q;
        f(false, base + t, mbase + (size_t)s * q + k);
      }
    }
  }
}

template <int NV>
__device__ inline void block_partials(double (&v)[NV], double* red, double* out) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k)
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v[k] += __shfl_xor(v[k], o, 64);
  __syncthreads();
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < NV; ++k) red[wid * NV + k] = v[k];
  __syncthreads();
  if (threadIdx.x < NV) {
    double t = 0.0;
    for (int w = 0; w < nw; ++w) t += red[w * NV + threadIdx.x];
    out[threadIdx.x] = t;
  }
}

// Sum of base[k * stride], k < count, over one wavefront: lane l takes
// k = l, l + 64, ...; the lanes are combined in a fixed tree.  The value of
// lane 0 is the result (the other lanes may differ in the last bits).
__device__ inline double wave_sum_strided(const double* base, int count, int stride) {
  const int lane = threadIdx.x & 63;
  double t = 0.0;
  for (int k = lane; k < count; k += 64) t += base[(size_t)k * stride];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
  return t;
}

// A parameter: its FP32 high word plus, when the low words are carried, the
// low word, summed in FP64 (about 48 significant bits).
__device__ inline double pval(const float* hi, const float* lo, size_t j) {
  return lo ? (double)hi[j] + (double)lo[j] : (double)hi[j];
}
// Store v as hi = fl32(v) and, when carried, lo = fl32(v - hi).
__device__ inline void pstore(float* hi, float* lo, size_t j, double v) {
  const float h = (float)v;
  hi[j] = h;
  if (lo) lo[j] = (float)(v - (double)h);
}

// gradient of F at the trial point for one parameter (h entry or block entry)
__device__ inline double sym_grad(const SymArgs& a, bool is_h, size_t j, size_t jm, double ib) {
  if (is_h) {
    const int r = (int)(j / a.q), s = (int)(j - (size_t)r * a.q);
    double t = 0.0;
    for (int k = 0; k < a.tiles; ++k) t += a.gh_part[((size_t)k * a.N + r) * kSlot + s];
    return t * ib + 2.0 * a.lambda_h * pval(a.Th, a.Thl, j);
  }
  return (a.gJ[j] + a.gJ[jm]) * ib + 2.0 * a.lambda_J * pval(a.TJ, a.TJl, j);
}

__global__ __launch_bounds__(kSymThreads) void sym_eval_kernel(SymArgs a) {
  __shared__ double red[kSymThreads / 64 * 3];
  if (a.st->phase == PH_DONE) return;
  const double ib = 1.0 / *a.beff;
  double v[3] = {0.0, 0.0, 0.0};  // l2 term, |g|^2, data term (unnormalised)
  for_each_param(a, [&](bool is_h, size_t j, size_t jm) {
    const double t = is_h ? pval(a.Th, a.Thl, j) : pval(a.TJ, a.TJl, j);
    const double g = sym_grad(a, is_h, j, jm, ib);
    v[0] += (is_h ? a.lambda_h : a.lambda_J) * t * t;
    v[1] += g * g;
  });
  const size_t nf = (size_t)a.tiles * a.N, step = (size_t)gridDim.x * blockDim.x;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < nf; e += step) v[2] += a.f_part[e];
  block_partials(v, red, a.part + (size_t)blockIdx.x * kSymPart);
}

__global__ __launch_bounds__(kSymThreads) void sym_decide_kernel(SymArgs a) {
  __shared__ double tot[3];
  SymState* S = a.st;
  if (S->phase == PH_DONE) return;
  const int wid = threadIdx.x >> 6;
  if (wid < 3) {
    const double t = wave_sum_strided(a.part + wid, a.nblk, kSymPart);
    if ((threadIdx.x & 63) == 0) tot[wid] = t;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  const double reg = tot[0], gg = tot[1], fdata = tot[2];
  const double ft = fdata / *a.beff + reg, gnt = sqrt(gg);
  const bool finite = isfinite(ft) && isfinite(gnt);
  S->evals += 1;
  S->accept = 0;
  S->pair = 0;
  S->move = 0;
  S->dir = SD_KEEP;
  if (S->phase == PH_INIT && !finite) {
    S->phase = PH_DONE;
    S->status = PLM_SITE_NONFINITE;
  } else if (S->phase == PH_INIT ||
             (finite && ft <= S->f + a.c1 * S->alpha * S->gtd + a.noise * fabs(S->f))) {
    S->accept = 1;
    S->pair = S->phase != PH_INIT;
    if (S->phase != PH_INIT) S->iter += 1;
    S->f = ft;
    S->gnorm = gnt;
    S->ls_count = 0;
    if (gnt <= a.tol) {
      S->phase = PH_DONE;
      S->status = PLM_SITE_CONVERGED;
    } else if (S->iter >= a.max_iter) {
      S->phase = PH_DONE;
      S->status = PLM_SITE_MAXITER;
    } else {
      S->phase = PH_LS;
      S->move = 1;  // direction chosen once the pair is decided
    }
  } else {
    S->ls_count += 1;
    S->phase = PH_LS;
    if (S->ls_count > a.max_ls) {
      if (S->stored > 0) {
        S->dir = SD_STEEPEST;
        S->ls_count = 0;
        S->move = 1;
      } else {
        S->phase = PH_DONE;
        S->status = PLM_SITE_LINESEARCH;
      }
    } else {
      double an = 0.5 * S->alpha;
      if (finite) {
        const double den = 2.0 * (ft - S->f - S->gtd * S->alpha);
        if (den > 0.0) an = -S->gtd * S->alpha * S->alpha / den;
        an = fmin(fmax(an, 0.1 * S->alpha), 0.5 * S->alpha);
      }
      S->alpha = an;
      S->move = 1;
    }
  }
}

__global__ __launch_bounds__(kSymThreads) void sym_accept_kernel(SymArgs a) {
  __shared__ double red[kSymThreads / 64 * kSymPart];
  const SymState* S = a.st;
  if (!S->accept) return;
  const bool pair = S->pair;
  const int M = a.m + 1, head = __builtin_amdgcn_readfirstlane(S->head);
  const int nA = __builtin_amdgcn_readfirstlane(min(S->stored, kSymGroup));
  const double ib = 1.0 / *a.beff;
  const size_t hs = (size_t)a.N * a.q, js = (size_t)a.N * a.N * a.q * a.q;
  double v[kSymPart];
#pragma unroll
  for (int k = 0; k < kSymPart; ++k) v[k] = 0.0;
  // NA stored pairs, a compile-time count: all of a parameter's history loads
  // are issued together
  auto pass = [&](auto na_c) {
    constexpr int NA = decltype(na_c)::value;
    int kk[NA > 0 ? NA : 1];
#pragma unroll
    for (int p = 0; p < NA; ++p) kk[p] = (head - 1 - p + 2 * M) % M;
    for_each_param(a, [&](bool is_h, size_t j, size_t jm) {
      float sl[NA > 0 ? NA : 1], yl[NA > 0 ? NA : 1];
      if (pair) {
#pragma unroll
        for (int p = 0; p < NA; ++p) {
          sl[p] = (is_h ? a.Sh + (size_t)kk[p] * hs : a.SJ + (size_t)kk[p] * js)[j];
          yl[p] = (is_h ? a.Yh + (size_t)kk[p] * hs : a.YJ + (size_t)kk[p] * js)[j];
        }
      }
      double* Gp = is_h ? a.Gh + j : a.GJ + j;
      const double t = is_h ? pval(a.Th, a.Thl, j) : pval(a.TJ, a.TJl, j);
      const double x = is_h ? pval(a.Xh, a.Xhl, j) : pval(a.XJ, a.XJl, j);
      const double gold = *Gp;
      const double g = sym_grad(a, is_h, j, jm, ib);
      if (pair) {
        // the pair is stored in FP32 and its products taken from the stored values
        const float svf = (float)(t - x), yvf = (float)(g - gold);
        (is_h ? a.Sh + (size_t)head * hs : a.SJ + (size_t)head * js)[j] = svf;
        (is_h ? a.Yh + (size_t)head * hs : a.YJ + (size_t)head * js)[j] = yvf;
        const double sv = svf, yv = yvf;
        v[0] += sv * yv;
        v[1] += yv * yv;
        v[2] += sv * g;
        v[3] += yv * g;
#pragma unroll
        for (int p = 0; p < NA; ++p) {
          const double s_ = sl[p], y_ = yl[p];
          v[4 + 4 * p] += s_ * yv;
          v[5 + 4 * p] += y_ * yv;
          v[6 + 4 * p] += s_ * g;
          v[7 + 4 * p] += y_ * g;
        }
      }
      *Gp = g;
      if (is_h) {
        a.Xh[j] = a.Th[j];
        if (a.Xhl) a.Xhl[j] = a.Thl[j];
      } else {
        a.XJ[j] = a.TJ[j];
        a.XJ[jm] = a.TJ[jm];
        if (a.XJl) {
          a.XJl[j] = a.TJl[j];
          a.XJl[jm] = a.TJl[jm];
        }
      }
    });
  };
  if (pair) with_count<0, kSymGroup>(nA, pass);
  else pass(std::integral_constant<int, 0>{});
  block_partials(v, red, a.part + (size_t)blockIdx.x * kSymPart);
}

// dot products of stored pairs group*4 .. group*4+3 with the candidate y and the new g
__global__ __launch_bounds__(kSymThreads) void sym_group_kernel(SymArgs a, int32_t group) {
  __shared__ double red[kSymThreads / 64 * 4 * kSymGroup];
  const SymState* S = a.st;
  const int j0 = kSymGroup * (group + 1);  // the first kSymGroup pairs ride on the accept pass
  if (!S->accept || !S->pair || j0 >= S->stored) return;
  const int M = a.m + 1, head = __builtin_amdgcn_readfirstlane(S->head);
  const int nB = __builtin_amdgcn_readfirstlane(min(kSymGroup, S->stored - j0));
  const size_t hs = (size_t)a.N * a.q, js = (size_t)a.N * a.N * a.q * a.q;
  double v[4 * kSymGroup];
#pragma unroll
  for (int k = 0; k < 4 * kSymGroup; ++k) v[k] = 0.0;
  with_count<1, kSymGroup>(nB, [&](auto nb_c) {
    constexpr int NB = decltype(nb_c)::value;
    int kk[NB];
#pragma unroll
    for (int p = 0; p < NB; ++p) kk[p] = (head - 1 - (j0 + p) + 2 * M) % M;
    for_each_param(a, [&](bool is_h, size_t j, size_t) {
      const double g = (is_h ? a.Gh : a.GJ)[j];
      const double yv = (is_h ? a.Yh + (size_t)head * hs : a.YJ + (size_t)head * js)[j];
      float sl[NB], yl[NB];
#pragma unroll
      for (int p = 0; p < NB; ++p) {
        sl[p] = (is_h ? a.Sh + (size_t)kk[p] * hs : a.SJ + (size_t)kk[p] * js)[j];
        yl[p] = (is_h ? a.Yh + (size_t)kk[p] * hs : a.YJ + (size_t)kk[p] * js)[j];
      }
#pragma unroll
      for (int p = 0; p < NB; ++p) {
        const double s_ = sl[p], y_ = yl[p];
        v[4 * p] += s_ * yv;
        v[4 * p + 1] += y_ * yv;
        v[4 * p + 2] += s_ * g;
        v[4 * p + 3] += y_ * g;
      }
    });
  });
  block_partials(v, red, a.part + ((size_t)(1 + group) * a.nblk + blockIdx.x) * kSymPart);
}

// Curvature test, small-matrix update and the compact-form coefficients
// (block sums in parallel, the rest on one thread; n <= 32).
__global__ __launch_bounds__(kSymThreads) void sym_solve_kernel(SymArgs a) {
  __shared__ double tot[4 + 4 * kMMax];
  __shared__ double t[kMMax];
  SymState* S = a.st;
  if (!S->accept) return;
  const int m = a.m, M = m + 1;
  SymCoef* C = a.coef;
  double* StY = a.small;
  double* YtY = a.small + (size_t)M * M;
  int stored = S->stored, head = S->head;
  if (S->pair) {
    // block sums of the candidate's dot products (quantity 0..3) and of the
    // stored pairs' (4 + 4 j + k, newest first), one wavefront per quantity
    const int nq = 4 + 4 * stored;
    for (int qi = threadIdx.x >> 6; qi < nq; qi += kSymThreads / 64) {
      const double* base;
      if (qi < 4 + 4 * kSymGroup) {
        base = a.part + qi;
      } else {
        const int j = (qi - 4) >> 2, k = (qi - 4) & 3;
        const int grp = 1 + (j - kSymGroup) / kSymGroup, p = (j - kSymGroup) % kSymGroup;
        base = a.part + (size_t)grp * a.nblk * kSymPart + 4 * p + k;
      }
      const double v = wave_sum_strided(base, a.nblk, kSymPart);
      if ((threadIdx.x & 63) == 0) tot[qi] = v;
    }
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  if (S->pair) {
    for (int j = 0; j < stored; ++j) {
      C->colS[j] = tot[4 + 4 * j];
      C->colY[j] = tot[5 + 4 * j];
      C->p1[j] = tot[6 + 4 * j];
      C->p2[j] = tot[7 + 4 * j];
    }
    const double cand[4] = {tot[0], tot[1], tot[2], tot[3]};
    const double sy = cand[0], yy = cand[1];
    if (sy > 0.0 && yy > 0.0) {
      const int c = head;
      for (int j = 0; j < stored; ++j) {
        const int k = (head - 1 - j + 2 * M) % M;
        StY[k * M + c] = C->colS[j];
        YtY[k * M + c] = C->colY[j];
        YtY[c * M + k] = C->colY[j];
      }
      StY[c * M + c] = sy;
      YtY[c * M + c] = yy;
      for (int j = min(stored, m - 1); j > 0; --j) {
        C->p1[j] = C->p1[j - 1];
        C->p2[j] = C->p2[j - 1];
      }
      C->p1[0] = cand[2];
      C->p2[0] = cand[3];
      S->gamma = sy / yy;
      head = (head + 1) % M;
      if (stored < m) ++stored;
    }
  }
  S->head = head;
  S->stored = stored;
  if (S->phase == PH_DONE) return;
  if (stored == 0) {
    S->dir = SD_STEEPEST;
    return;
  }
  S->dir = SD_QN;
  const int n = stored;
  const double gamma = S->gamma;
  for (int i = 0; i < n; ++i) C->ord[i] = (head - n + i + 2 * M) % M;
  auto R = [&](int i, int j) { return StY[C->ord[i] * M + C->ord[j]]; };
  auto YY = [&](int i, int j) { return YtY[C->ord[i] * M + C->ord[j]]; };
  for (int i = n - 1; i >= 0; --i) {
    double x = C->p1[n - 1 - i];
    for (int l = i + 1; l < n; ++l) x -= R(i, l) * t[l];
    t[i] = x / R(i, i);
  }
  for (int i = 0; i < n; ++i) {
    double yyt = 0.0;
    for (int l = 0; l < n; ++l) yyt += YY(i, l) * t[l];
    double x = R(i, i) * t[i] + gamma * (yyt - C->p2[n - 1 - i]);
    for (int l = 0; l < i; ++l) x -= R(l, i) * C->cs[l];
    C->cs[i] = x / R(i, i);
  }
  for (int i = 0; i < n; ++i) {
    C->cs[i] = -C->cs[i];
    C->cy[i] = gamma * t[i];
  }
  C->n = n;
}

__global__ __launch_bounds__(kSymThreads) void sym_direct_kernel(SymArgs a) {
  __shared__ double red[kSymThreads / 64];
  __shared__ double cs[kMMax], cy[kMMax];
  __shared__ int32_t ord[kMMax];
  const SymState* S = a.st;
  if (S->dir != SD_QN || S->phase == PH_DONE) return;
  const SymCoef* C = a.coef;
  const int n = C->n;
  if (threadIdx.x < n) {
    cs[threadIdx.x] = C->cs[threadIdx.x];
    cy[threadIdx.x] = C->cy[threadIdx.x];
    ord[threadIdx.x] = C->ord[threadIdx.x];
  }
  __syncthreads();
  const double gamma = S->gamma;
  const size_t hs = (size_t)a.N * a.q, js = (size_t)a.N * a.N * a.q * a.q;
  double v[1] = {0.0};
  for_each_param(a, [&](bool is_h, size_t j, size_t jm) {
    const double g = (is_h ? a.Gh : a.GJ)[j];
    double d = -gamma * g;
    // four pairs per step, their loads issued together; the sum runs in pair order
    int i = 0;
    for (; i + 4 <= n; i += 4) {
      float sl[4], yl[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int k = ord[i + u];
        sl[u] = (is_h ? a.Sh + (size_t)k * hs : a.SJ + (size_t)k * js)[j];
        yl[u] = (is_h ? a.Yh + (size_t)k * hs : a.YJ + (size_t)k * js)[j];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) d += cs[i + u] * (double)sl[u] + cy[i + u] * (double)yl[u];
    }
    for (; i < n; ++i) {
      const int k = ord[i];
      d += cs[i] * (is_h ? a.Sh + (size_t)k * hs : a.SJ + (size_t)k * js)[j] +
           cy[i] * (is_h ? a.Yh + (size_t)k * hs : a.YJ + (size_t)k * js)[j];
    }
    (is_h ? a.Dh : a.DJ)[j] = d;
    if (is_h) {
      pstore(a.Th, a.Thl, j, pval(a.Xh, a.Xhl, j) + d);
    } else {
      const double tv = pval(a.XJ, a.XJl, j) + d;
      pstore(a.TJ, a.TJl, j, tv);
      pstore(a.TJ, a.TJl, jm, tv);
    }
    v[0] += d * g;
  });
  block_partials(v, red, a.part + (size_t)blockIdx.x * kSymPart);
}

__global__ void sym_check_kernel(SymArgs a) {
  SymState* S = a.st;
  if (S->phase == PH_DONE) return;
  const double dgw = S->dir == SD_QN ? wave_sum_strided(a.part, a.nblk, kSymPart) : 0.0;
  if (threadIdx.x != 0) return;
  if (S->dir == SD_QN) {
    const double dg = dgw;
    if (dg < 0.0) {
      S->gtd = dg;
      S->alpha = 1.0;
      S->move = 0;  // the trial point is written
      return;
    }
    S->dir = SD_STEEPEST;
  }
  if (S->dir == SD_STEEPEST) {
    S->gtd = -S->gnorm * S->gnorm;
    S->alpha = fmin(1.0, 1.0 / S->gnorm);
    S->stored = 0;
    S->move = 1;
  }
}

__global__ __launch_bounds__(kSymThreads) void sym_move_kernel(SymArgs a) {
  const SymState* S = a.st;
  if (S->phase == PH_DONE || !S->move) return;
  const bool steep = S->dir == SD_STEEPEST;
  const double alpha = S->alpha;
  for_each_param(a, [&](bool is_h, size_t j, size_t jm) {
    double* Dp = is_h ? a.Dh + j : a.DJ + j;
    if (steep) *Dp = -(is_h ? a.Gh : a.GJ)[j];
    const double d = *Dp;
    if (is_h) {
      pstore(a.Th, a.Thl, j, pval(a.Xh, a.Xhl, j) + alpha * d);
    } else {
      const double tv = pval(a.XJ, a.XJl, j) + alpha * d;
      pstore(a.TJ, a.TJl, j, tv);
      pstore(a.TJ, a.TJl, jm, tv);
    }
  });
}

// Counters, the host's done flag, and the work tables of the next
// evaluation: every site, or none once the minimisation has stopped (then the
// step flags are cleared so that further replays change nothing).
__global__ void sym_finish_kernel(SymArgs a, BatchArgs b) {
  SymState* S = a.st;
  if (threadIdx.x < 2 * kQueues) b.ctr[threadIdx.x] = 0u;
  if (threadIdx.x == 0) {
    if (S->phase == PH_DONE) {  // later replays leave every buffer alone
      S->accept = 0;
      S->pair = 0;
      S->move = 0;
      S->dir = SD_KEEP;
    }
    const int n = S->phase == PH_DONE ? 0 : a.N;
    *b.n_active = n;
    b.seg[0] = 0;
    b.seg[1] = n;
    for (int kind = 0; kind < 2; ++kind) {
      const int grp = kind_group(b, kind);
      b.item_off[kind * 2] = 0;
      b.item_off[kind * 2 + 1] = (n + grp - 1) / grp * b.nsub[kind];
    }
    if (a.done_host) *a.done_host = S->phase == PH_DONE ? 1 : 0;
  }
}

// Start point: J (and its low words) made consistent (J[i][r] = J[r][i]
// transposed, self blocks zero) in place, trial point = start point, optimiser
// state reset.
__global__ __launch_bounds__(kSymThreads) void sym_init_kernel(SymArgs a) {
  const int q = a.q, qq = q * q, N = a.N;
  for (int r = blockIdx.x; r < N; r += gridDim.x)
    for (int t = threadIdx.x; t < qq; t += blockDim.x) {
      a.XJ[((size_t)r * N + r) * qq + t] = 0.f;
      if (a.XJl) a.XJl[((size_t)r * N + r) * qq + t] = 0.f;
    }
  for_each_param(a, [&](bool is_h, size_t j, size_t jm) {
    if (is_h) {
      a.Th[j] = a.Xh[j];
      if (a.Xhl) a.Thl[j] = a.Xhl[j];
    } else {
      a.XJ[jm] = a.XJ[j];
      a.TJ[j] = a.XJ[j];
      a.TJ[jm] = a.XJ[j];
      if (a.XJl) {
        a.XJl[jm] = a.XJl[j];
        a.TJl[j] = a.XJl[j];
        a.TJl[jm] = a.XJl[j];
      }
    }
  });
  for (int r = blockIdx.x; r < N; r += gridDim.x)
    for (int t = threadIdx.x; t < qq; t += blockDim.x) {
      a.TJ[((size_t)r * N + r) * qq + t] = 0.f;
      if (a.TJl) a.TJl[((size_t)r * N + r) * qq + t] = 0.f;
    }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    SymState s;
    s.phase = PH_INIT;
    s.status = PLM_SITE_MAXITER;
    s.iter = s.evals = s.ls_count = s.head = s.stored = s.accept = s.pair = s.dir = s.move = s.pad = 0;
    s.f = s.gnorm = s.alpha = s.gtd = 0.0;
    s.gamma = 1.0;
    *a.st = s;
  }
}

hipError_t launch_sym_init(const SymArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(sym_init_kernel, dim3(a.nblk), dim3(kSymThreads), 0, st, a);
  return hipGetLastError();
}

int32_t sym_part_stride() { return kSymPart; }
int32_t sym_groups(int32_t m) { return m > kSymGroup ? (m - kSymGroup + kSymGroup - 1) / kSymGroup : 0; }

// One optimiser step after the evaluation of the trial point.
hipError_t launch_sym_step(const SymArgs& a, const BatchArgs& b, hipStream_t st) {
  hipLaunchKernelGGL(sym_eval_kernel, dim3(a.nblk), dim3(kSymThreads), 0, st, a);
  hipLaunchKernelGGL(sym_decide_kernel, dim3(1), dim3(kSymThreads), 0, st, a);
  hipLaunchKernelGGL(sym_accept_kernel, dim3(a.nblk), dim3(kSymThreads), 0, st, a);
  for (int g = 0; g < sym_groups(a.m); ++g)
    hipLaunchKernelGGL(sym_group_kernel, dim3(a.nblk), dim3(kSymThreads), 0, st, a, g);
  hipLaunchKernelGGL(sym_solve_kernel, dim3(1), dim3(kSymThreads), 0, st, a);
  hipLaunchKernelGGL(sym_direct_kernel, dim3(a.nblk), dim3(kSymThreads), 0, st, a);
  hipLaunchKernelGGL(sym_check_kernel, dim3(1), dim3(64), 0, st, a);
  hipLaunchKernelGGL(sym_move_kernel, dim3(a.nblk), dim3(kSymThreads), 0, st, a);
  hipLaunchKernelGGL(sym_finish_kernel, dim3(1), dim3(64), 0, st, a, b);
  return hipGetLastError();
}

}  // namespace plm
