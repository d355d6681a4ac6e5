// k_lbfgs.hip -- device-resident limited-memory BFGS for all N per-site
// problems of asymmetric plmDCA (sec. 3.4 step 3; the paper minimises each
// g_r^reg by L-BFGS from the origin, secs. 5 and 6).
//
// One block owns one site in the step (lbfgs_kernel).  Each launch consumes
// the evaluation of the site's trial point (objective partials from the
// forward kernel, FP64 gradient data part from the backward kernel), adds the
// l2 terms in FP64, takes the line search decision (sufficient decrease with
// backtracking by safeguarded quadratic interpolation), and on acceptance
// stores the curvature pair and computes the coefficients of the next
// direction, which lbfgs_dir_kernel forms with several blocks per site
// (writing the next trial point) and lbfgs_dir_finish_kernel tests for
// descent; backtracking and steepest-descent trial points are written by the
// step itself.  All dot products and the small matrices are
// FP64; the stored curvature pairs, the gradient kept at the iterate and the
// direction are FP32 (the gradients carry the rounding noise of the FP32
// evaluation, far above the 2^-24 relative rounding of the stored values;
// halving the stored vectors' bytes halves most of this streaming kernel's
// traffic); the gradient at the trial point and the objective are formed in
// FP64; the iterate is kept at FP32-representable values so that the
// evaluated point and the stored point are the same.
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

constexpr int kLbThreads = 512;  // two blocks per CU: every site of the benchmark alignment in one round
constexpr int kLbWaves = kLbThreads / 64;
constexpr int kGroupA = 4;  // stored pairs whose dot products ride on the acceptance pass
constexpr int kGroupB = 6;  // stored pairs per further dot-product pass (m = 10: one such pass)
constexpr int kVecMax = 4 + 2 * kGroupA > 2 * kGroupB ? 4 + 2 * kGroupA : 2 * kGroupB;  // widest block sum
constexpr int kSlotsMax = kMMax + 1;

struct LbShared {
  double red[kLbWaves * kVecMax];
  double vec[kVecMax];
  double ghd[kSlot];
  double Rm[kMMax * kMMax];   // S^T Y and Y^T Y of the stored pairs, chronological order
  double YYm[kMMax * kMMax];
  double cs[kMMax];           // direction coefficients of s and y, chronological order
  double cy[kMMax];
  double tv[kMMax];
  double p1[kSlotsMax];       // s_j . g and y_j . g of the stored pairs, newest first
  double p2[kSlotsMax];
  double colS[kSlotsMax];     // s_j . y_cand and y_j . y_cand, newest first (y_cand as stored)
  double colY[kSlotsMax];
  double cand[4];             // candidate pair: s.y, y.y, s.g, y.g
  int32_t ord[kMMax];         // slots of the stored pairs, oldest first
};

// Block sums of NV per-thread FP64 values (fixed order: a shuffle tree per
// wave, then the waves in order); every thread gets the sums.
template <int NV>
__device__ inline void block_sum_vec(double (&v)[NV], LbShared& sh) {
  static_assert(NV <= kVecMax, "block sums sized for kVecMax values");
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k)
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v[k] += __shfl_xor(v[k], o, 64);
  __syncthreads();
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < NV; ++k) sh.red[wid * NV + k] = v[k];
  __syncthreads();
  if (threadIdx.x < NV) {
    double t = 0.0;
    for (int w = 0; w < kLbWaves; ++w) t += sh.red[w * NV + threadIdx.x];
    sh.vec[threadIdx.x] = t;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = sh.vec[k];
  __syncthreads();
}

__device__ inline void lbfgs_site(const LbfgsArgs& a, int r, LbShared& sh, double* red) {
  SiteState* S = a.st + r;
  const int phase = S->phase;
  if (phase == PH_DONE) return;
  const int q = a.q, N = a.N, m = a.m, M = m + 1;  // M history slots
  const size_t Nqq = (size_t)N * q * q;
  const int P = q + (int)Nqq;
  const int tid = threadIdx.x, nth = blockDim.x;
  const double beff = *a.beff;
  const double ib = 1.0 / beff;
  const size_t h0 = (size_t)r * q, j0 = (size_t)r * Nqq;
  const int self0 = q + r * q * q, self1 = self0 + q * q;  // self block range in e
  // every buffer seen as global memory (the descriptor comes from memory, so
  // the pointers would otherwise be generic and every access a flat one)
  const auto Th = gmem_w(a.Th), TJ = gmem_w(a.TJ), Xh = gmem_w(a.Xh), XJ = gmem_w(a.XJ);
  const auto Ghp = gmem_w(a.Gh), GJp = gmem_w(a.GJ);
  const auto Dhp = gmem_w(a.Dh), DJp = gmem_w(a.DJ);
  const auto Shp = gmem_w(a.Sh), SJp = gmem_w(a.SJ), Yhp = gmem_w(a.Yh), YJp = gmem_w(a.YJ);
  const auto gJd = gmem(a.gJ);
  const auto StY = gmem_w(a.small + (size_t)r * 2 * M * (M + 1));  // [M][M] s_i . y_j by slot
  const auto YtY = StY + (size_t)M * M;                             // [M][M] y_i . y_j by slot
  const auto SG = YtY + (size_t)M * M;                              // [M] s_k . G by slot
  const auto YG = SG + M;                                           // [M] y_k . G by slot

  // ---- gather the evaluation at the trial point ----
  if (tid < q) {
    double t = 0.0;
    for (int k = 0; k < a.tiles; ++k) t += gmem(a.gh_part)[((size_t)k * N + r) * kSlot + tid];
    sh.ghd[tid] = t;
  }
  double fdata = 0.0;
  if (tid == 0)
    for (int k = 0; k < a.tiles; ++k) fdata += gmem(a.f_part)[(size_t)k * N + r];
  __syncthreads();

  const double lam_h = a.lambda_h, lam_J = a.lambda_Jp;
  auto lam = [&](int e) -> double { return e < q ? lam_h : ((e >= self0 && e < self1) ? 0.0 : lam_J); };
  auto Tv = [&](int e) -> double { return e < q ? (double)Th[h0 + e] : (double)TJ[j0 + (e - q)]; };
  auto Xv = [&](int e) -> double { return e < q ? (double)Xh[h0 + e] : (double)XJ[j0 + (e - q)]; };
  auto gtv = [&](int e) -> double {
    const double d = e < q ? sh.ghd[e] : gJd[j0 + (e - q)];
    return d * ib + 2.0 * lam(e) * Tv(e);
  };
  auto Gv = [&](int e) -> double { return e < q ? Ghp[h0 + e] : GJp[j0 + (e - q)]; };
  auto Dp = [&](int e) { return e < q ? Dhp + h0 + e : DJp + j0 + (e - q); };
  auto Gp = [&](int e) { return e < q ? Ghp + h0 + e : GJp + j0 + (e - q); };
  auto Sp = [&](int k, int e) {
    return e < q ? Shp + ((size_t)k * N) * q + h0 + e : SJp + (size_t)k * N * Nqq + j0 + (e - q);
  };
  auto Yp = [&](int k, int e) {
    return e < q ? Yhp + ((size_t)k * N) * q + h0 + e : YJp + (size_t)k * N * Nqq + j0 + (e - q);
  };
  auto storeT = [&](int e, double v) {
    const float f = (float)v;
    if (e < q) Th[h0 + e] = f; else TJ[j0 + (e - q)] = (e >= self0 && e < self1) ? 0.f : f;
  };
  auto writeT = [&](double alpha) {
    for (int e = tid; e < P; e += nth) storeT(e, Xv(e) + alpha * (double)*Dp(e));
  };

  // The element loops below visit, per thread, its field element (e = tid < q;
  // nth >= q, so there is at most one and it comes first) and then the coupling
  // elements e = q + o of the site's row in increasing order, o = e - q, the
  // order of a plain strided loop over e.  The coupling part addresses each
  // vector from a uniform (scalar) base.
  static_assert(kQMax <= kLbThreads, "at most one field element per thread");
  const int o_first = (tid < q ? tid + nth : tid) - q;  // first coupling offset of this thread
  const int nJ = (int)Nqq;
  const int sb0 = r * q * q, sb1 = sb0 + q * q;  // self block in o (no penalty, kept at zero)
  const auto TJr = TJ + j0, XJr = XJ + j0;
  const auto GJr = GJp + j0;
  const auto gJr = gJd + j0;
  const size_t slot = (size_t)N * Nqq;  // coupling entries per history slot
  auto lamJ = [&](int o) -> double { return (o >= sb0 && o < sb1) ? 0.0 : lam_J; };

  double reg = 0.0, gg = 0.0;
  if (tid < q) {
    const double t = Tv(tid), g = gtv(tid);
    reg += lam(tid) * t * t;
    gg += g * g;
  }
#pragma unroll 4
  for (int o = o_first; o < nJ; o += nth) {
    const double t = TJr[o], lo = lamJ(o);
    const double g = gJr[o] * ib + 2.0 * lo * t;
    reg += lo * t * t;
    gg += g * g;
  }
  reg = block_sum_f64(reg, red);
  gg = block_sum_f64(gg, red);
  fdata = block_sum_f64(tid == 0 ? fdata : 0.0, red);
  const double ft = fdata * ib + reg;
  const double gnt = sqrt(gg);
  const bool finite = isfinite(ft) && isfinite(gnt);

  int evals = S->evals + 1;
  int iter = S->iter, ls = S->ls_count, status = S->status;
  int head = __builtin_amdgcn_readfirstlane(S->head), stored = __builtin_amdgcn_readfirstlane(S->stored);
  double f = S->f, gnorm = S->gnorm, alpha = S->alpha, gtd = S->gtd, gamma = S->gamma;
  int newphase = phase;
  // what to do with the search direction once the decision is taken
  enum { KEEP = 0, STEEPEST = 1, QUASI_NEWTON = 2 } dir = KEEP;
  bool move = false;  // write a new trial point
  int dpend = 0;      // a quasi-Newton direction left to the direction kernels

  if (phase == PH_INIT && !finite) {
    newphase = PH_DONE;
    status = PLM_SITE_NONFINITE;
  } else if (phase == PH_INIT ||
             (finite && ft <= f + a.c1 * alpha * gtd + a.noise * fabs(f))) {
    // accept the trial point (the first evaluation is the start point itself);
    // sufficient decrease allows for the rounding noise of the FP32 evaluation.
    // One pass: gradient, candidate pair (s, y) into the free slot `head`, and
    // the dot products of the newest stored pairs with y and g.
    const bool pair = phase != PH_INIT;
    const int nA = min(stored, kGroupA);
    double acc[4 + 2 * kGroupA];
#pragma unroll
    for (int k = 0; k < 4 + 2 * kGroupA; ++k) acc[k] = 0.0;
    if (!pair) {
      // the start point: gradient and iterate only
      if (tid < q) {
        *Gp(tid) = (float)gtv(tid);
        Xh[h0 + tid] = Th[h0 + tid];
      }
      for (int o = o_first; o < nJ; o += nth) {
        const float tf = TJr[o];
        GJr[o] = (float)(gJr[o] * ib + 2.0 * lamJ(o) * (double)tf);
        XJr[o] = tf;
      }
    } else {
      // NA, the number of stored pairs in this pass, is a compile-time constant,
      // so that all of an element's history loads are issued together
      auto accept_pass = [&](auto na_c) {
        constexpr int NA = decltype(na_c)::value;
        int kk[NA > 0 ? NA : 1];
#pragma unroll
        for (int j = 0; j < NA; ++j) kk[j] = (head - 1 - j + 2 * M) % M;
        if (tid < q) {
          const int e = tid;
          const double g = gtv(e);
          // the pair is stored in FP32 and used as stored, so that its dot
          // products describe exactly the vectors the direction is formed from
          const float svf = (float)(Tv(e) - Xv(e)), yvf = (float)(g - Gv(e));
          *Sp(head, e) = svf;
          *Yp(head, e) = yvf;
          const double sv = svf, yv = yvf;
          acc[0] += sv * yv;
          acc[1] += yv * yv;
          acc[2] += sv * g;
          acc[3] += yv * g;
#pragma unroll
          for (int j = 0; j < NA; ++j) {
            acc[4 + 2 * j] += (double)*Sp(kk[j], e) * yv;
            acc[5 + 2 * j] += (double)*Yp(kk[j], e) * yv;
          }
          *Gp(e) = (float)g;
          Xh[h0 + e] = Th[h0 + e];
        }
        const auto sH = SJp + (size_t)head * slot + j0, yH = YJp + (size_t)head * slot + j0;
        std::remove_const_t<decltype(SJp)> sJ[NA > 0 ? NA : 1];
        std::remove_const_t<decltype(YJp)> yJ[NA > 0 ? NA : 1];
#pragma unroll
        for (int j = 0; j < NA; ++j) {
          sJ[j] = SJp + (size_t)kk[j] * slot + j0;
          yJ[j] = YJp + (size_t)kk[j] * slot + j0;
        }
        // one coupling element from its loaded values
        auto elem = [&](int o, float tf, float xf, double gold, double gd, const float (&sl)[NA > 0 ? NA : 1],
                        const float (&yl)[NA > 0 ? NA : 1]) {
          const double t = tf;
          const double g = gd * ib + 2.0 * lamJ(o) * t;
          const float svf = (float)(t - (double)xf), yvf = (float)(g - gold);
          sH[o] = svf;
          yH[o] = yvf;
          const double sv = svf, yv = yvf;
          acc[0] += sv * yv;
          acc[1] += yv * yv;
          acc[2] += sv * g;
          acc[3] += yv * g;
#pragma unroll
          for (int j = 0; j < NA; ++j) {
            acc[4 + 2 * j] += (double)sl[j] * yv;
            acc[5 + 2 * j] += (double)yl[j] * yv;
          }
          GJr[o] = (float)g;
          XJr[o] = tf;
        };
        for (int o = o_first; o < nJ; o += nth) {
          const float tf = TJr[o], xf = XJr[o];
          const double go = GJr[o], gd = gJr[o];
          float s0[NA > 0 ? NA : 1], y0[NA > 0 ? NA : 1];
#pragma unroll
          for (int j = 0; j < NA; ++j) {
            s0[j] = sJ[j][o];
            y0[j] = yJ[j][o];
          }
          // all of the element's loads are issued before the first use
          __builtin_amdgcn_sched_barrier(0);
          elem(o, tf, xf, go, gd, s0, y0);
        }
      };
      with_count<0, kGroupA>(nA, accept_pass);
    }
    if (pair) {
      block_sum_vec(acc, sh);
      if (tid == 0) {
#pragma unroll
        for (int k = 0; k < 4; ++k) sh.cand[k] = acc[k];
#pragma unroll
        for (int j = 0; j < kGroupA; ++j)
          if (j < nA) {
            sh.colS[j] = acc[4 + 2 * j];
            sh.colY[j] = acc[5 + 2 * j];
          }
      }
      // the older stored pairs, kGroupB at a time (y from the slot this thread
      // has just written)
      for (int jg = kGroupA; jg < stored; jg += kGroupB) {
        double bcc[2 * kGroupB];
#pragma unroll
        for (int k = 0; k < 2 * kGroupB; ++k) bcc[k] = 0.0;
        const int nB = min(kGroupB, stored - jg);
        auto pair_pass = [&](auto nb_c) {
          constexpr int NB = decltype(nb_c)::value;
          int kk[NB];
#pragma unroll
          for (int j = 0; j < NB; ++j) kk[j] = (head - 1 - (jg + j) + 2 * M) % M;
          if (tid < q) {
            const double yv = *Yp(head, tid);
#pragma unroll
            for (int j = 0; j < NB; ++j) {
              bcc[2 * j] += (double)*Sp(kk[j], tid) * yv;
              bcc[2 * j + 1] += (double)*Yp(kk[j], tid) * yv;
            }
          }
          const auto yH = YJp + (size_t)head * slot + j0;
          std::remove_const_t<decltype(SJp)> sJ[NB];
          std::remove_const_t<decltype(YJp)> yJ[NB];
#pragma unroll
          for (int j = 0; j < NB; ++j) {
            sJ[j] = SJp + (size_t)kk[j] * slot + j0;
            yJ[j] = YJp + (size_t)kk[j] * slot + j0;
          }
          for (int o = o_first; o < nJ; o += nth) {
            const float yf = yH[o];
            float sf[NB], tf[NB];
#pragma unroll
            for (int j = 0; j < NB; ++j) {
              sf[j] = sJ[j][o];
              tf[j] = yJ[j][o];
            }
            // all of the element's loads are issued before the first use
            __builtin_amdgcn_sched_barrier(0);
            const double yv = yf;
#pragma unroll
            for (int j = 0; j < NB; ++j) {
              bcc[2 * j] += (double)sf[j] * yv;
              bcc[2 * j + 1] += (double)tf[j] * yv;
            }
          }
        };
        with_count<1, kGroupB>(nB, pair_pass);
        block_sum_vec(bcc, sh);
        if (tid == 0)
#pragma unroll
          for (int j = 0; j < kGroupB; ++j)
            if (j < nB) {
              sh.colS[jg + j] = bcc[2 * j];
              sh.colY[jg + j] = bcc[2 * j + 1];
            }
      }
      __syncthreads();
      // S^T g and Y^T g at the new point: the stored products moved by the
      // candidate's y (G changes by y whether or not the pair is kept)
      if (tid == 0)
        for (int j = 0; j < stored; ++j) {
          const int k = (head - 1 - j + 2 * M) % M;
          const double pg1 = SG[k] + sh.colS[j], pg2 = YG[k] + sh.colY[j];
          SG[k] = pg1;
          YG[k] = pg2;
          sh.p1[j] = pg1;
          sh.p2[j] = pg2;
        }
      __syncthreads();
      const double sy = sh.cand[0], yy = sh.cand[1];
      if (sy > 0.0 && yy > 0.0) {
        // keep the candidate: its column of S^T Y and its row/column of Y^T Y;
        // it becomes the newest pair (index 0 of the newest-first lists)
        if (tid == 0) {
          const int c = head;
          for (int j = 0; j < stored; ++j) {
            const int k = (head - 1 - j + 2 * M) % M;
            StY[k * M + c] = sh.colS[j];
            YtY[k * M + c] = sh.colY[j];
            YtY[c * M + k] = sh.colY[j];
          }
          StY[c * M + c] = sy;
          YtY[c * M + c] = yy;
          for (int j = min(stored, m - 1); j > 0; --j) {
            sh.p1[j] = sh.p1[j - 1];
            sh.p2[j] = sh.p2[j - 1];
          }
          sh.p1[0] = sh.cand[2];
          sh.p2[0] = sh.cand[3];
          SG[c] = sh.cand[2];
          YG[c] = sh.cand[3];
        }
        gamma = sy / yy;
        head = (head + 1) % M;
        if (stored < m) ++stored;
      }
    }
    if (phase != PH_INIT) ++iter;
    f = ft;
    gnorm = gnt;
    ls = 0;
    if (gnorm <= a.tol) {
      newphase = PH_DONE;
      status = PLM_SITE_CONVERGED;
    } else if (iter >= a.max_iter) {
      newphase = PH_DONE;
      status = PLM_SITE_MAXITER;
    } else {
      newphase = PH_LS;
      dir = stored > 0 ? QUASI_NEWTON : STEEPEST;
      move = true;
    }
  } else {
    // reject: backtrack along the same direction
    ++ls;
    newphase = PH_LS;
    if (ls > a.max_ls) {
      if (stored > 0) {  // forget the history once, restart from steepest descent
        dir = STEEPEST;
        ls = 0;
        move = true;
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
      move = true;
    }
  }

  if (dir == QUASI_NEWTON) {
    // the compact form over the n stored pairs, in chronological order
    const int n = stored;
    __syncthreads();
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
    // the direction itself is formed by lbfgs_dir_kernel, several blocks per
    // site, and its descent test taken by lbfgs_dir_finish_kernel
    DirCoef* C = a.dc + r;
    if (tid < n) {
      C->cs[tid] = sh.cs[tid];
      C->cy[tid] = sh.cy[tid];
      C->ord[tid] = sh.ord[tid];
    }
    if (tid == 0) {
      C->n = n;
      C->gamma = gamma;
    }
    dpend = 1;
    move = false;
  }
  if (dir == STEEPEST) {
    __syncthreads();
    for (int e = tid; e < P; e += nth) *Dp(e) = (float)-Gv(e);
    gtd = -gnorm * gnorm;
    alpha = fmin(1.0, 1.0 / gnorm);
    stored = 0;
  }
  if (move) {
    __syncthreads();
    writeT(alpha);
  }
  __syncthreads();
  if (tid == 0) {
    S->phase = newphase;
    S->status = status;
    S->iter = iter;
    S->evals = evals;
    S->ls_count = ls;
    S->head = head;
    S->stored = stored;
    S->dpend = dpend;
    S->f = f;
    S->gnorm = gnorm;
    S->alpha = alpha;
    S->gtd = gtd;
    S->gamma = gamma;
    if (a.phase_host) a.phase_host[r] = newphase;
  }
}

// One block per active site of the batch.
// at most 128 VGPRs: two 512-thread blocks per CU
__global__ __launch_bounds__(kLbThreads) __attribute__((amdgpu_waves_per_eu(4, 4))) void lbfgs_kernel(BatchArgs b) {
  __shared__ LbShared sh;
  __shared__ double red[16];
  const int idx = blockIdx.x;
  if (idx >= *b.n_active) return;
  // site, alignment and their descriptor are block-uniform: scalar registers
  const int g = __builtin_amdgcn_readfirstlane(b.active[idx]);
  const int m = __builtin_amdgcn_readfirstlane(b.msa_of[g]);
  const LbfgsArgs a = load_uniform(b.lb + m);
  lbfgs_site(a, __builtin_amdgcn_readfirstlane(g - b.site_base[m]), sh, red);
}

// Per-site vectors of the direction kernels, addressed by the element index
// e of the site's parameter vector (fields e < q, then the couplings).
struct SiteVecs {
  int q, self0, self1;
  size_t h0, j0, hs, js;  // field and coupling offsets of the site, slot strides
  const __attribute__((address_space(1))) float *Gh, *GJ, *Xh, *XJ, *Sh, *SJ, *Yh, *YJ;
  __attribute__((address_space(1))) float *Dh, *DJ, *Th, *TJ;
  __device__ SiteVecs(const LbfgsArgs& a, int r) {
    q = a.q;
    const size_t Nqq = (size_t)a.N * a.q * a.q;
    h0 = (size_t)r * q;
    j0 = (size_t)r * Nqq;
    hs = (size_t)a.N * q;
    js = (size_t)a.N * Nqq;
    self0 = q + r * q * q;
    self1 = self0 + q * q;
    Gh = gmem(a.Gh); GJ = gmem(a.GJ); Xh = gmem(a.Xh); XJ = gmem(a.XJ);
    Sh = gmem(a.Sh); SJ = gmem(a.SJ); Yh = gmem(a.Yh); YJ = gmem(a.YJ);
    Dh = gmem_w(a.Dh); DJ = gmem_w(a.DJ); Th = gmem_w(a.Th); TJ = gmem_w(a.TJ);
  }
  __device__ double G(int e) const { return e < q ? Gh[h0 + e] : GJ[j0 + (e - q)]; }
  __device__ double X(int e) const { return e < q ? Xh[h0 + e] : XJ[j0 + (e - q)]; }
  __device__ double S(int k, int e) const { return e < q ? Sh[k * hs + h0 + e] : SJ[k * js + j0 + (e - q)]; }
  __device__ double Y(int k, int e) const { return e < q ? Yh[k * hs + h0 + e] : YJ[k * js + j0 + (e - q)]; }
  __device__ void setD(int e, float d) const {
    if (e < q) Dh[h0 + e] = d; else DJ[j0 + (e - q)] = d;
  }
  // the trial point, FP32; the self block stays zero
  __device__ void setT(int e, double v) const {
    const float f = (float)v;
    if (e < q) Th[h0 + e] = f; else TJ[j0 + (e - q)] = (e >= self0 && e < self1) ? 0.f : f;
  }
};

constexpr int kDirThreads = 256;

// The pending quasi-Newton direction of every active site, kDirChunks blocks
// per site, each over a contiguous range of the site's elements: d, the
// trial point X + d (step 1) and the block's partial sum of d . g.  The
// partition depends on the site's size only, so the sums do not depend on
// the batch.
__global__ __launch_bounds__(kDirThreads) __attribute__((amdgpu_waves_per_eu(6))) void lbfgs_dir_kernel(BatchArgs b) {
  __shared__ double cs[kMMax], cy[kMMax];
  __shared__ int32_t ord[kMMax];
  __shared__ double red[kDirThreads / 64];
  const int idx = blockIdx.x / kDirChunks, chunk = blockIdx.x - idx * kDirChunks;
  if (idx >= *b.n_active) return;
  const int g = __builtin_amdgcn_readfirstlane(b.active[idx]);
  const int m = __builtin_amdgcn_readfirstlane(b.msa_of[g]);
  const LbfgsArgs a = load_uniform(b.lb + m);
  const int r = __builtin_amdgcn_readfirstlane(g - b.site_base[m]);
  if (__builtin_amdgcn_readfirstlane(a.st[r].dpend) == 0) return;
  const DirCoef* C = a.dc + r;
  const int n = __builtin_amdgcn_readfirstlane(C->n);
  const double gamma = C->gamma;
  const int tid = threadIdx.x, nth = blockDim.x;
  if (tid < n) {
    cs[tid] = C->cs[tid];
    cy[tid] = C->cy[tid];
    ord[tid] = C->ord[tid];
  }
  __syncthreads();
  const SiteVecs v(a, r);
  const int P = a.q + a.N * a.q * a.q;
  const int csz = (P + kDirChunks - 1) / kDirChunks;
  const int e_beg = chunk * csz, e_end = min(P, e_beg + csz);
  // four elements per thread at a time (e, e + nth, e + 2 nth, e + 3 nth),
  // so that the history loads of four elements are in flight together
  double dg = 0.0;
  constexpr int U = 4;
  for (int e0 = e_beg + tid; e0 < e_end; e0 += U * nth) {
    int ee[U];
    double gv[U], d[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      ee[u] = min(e0 + u * nth, e_end - 1);
      gv[u] = v.G(ee[u]);
      d[u] = -gamma * gv[u];
    }
#pragma unroll 2
    for (int i = 0; i < n; ++i) {
      const int k = ord[i];
      const double ci = cs[i], yi = cy[i];
      double sv[U], yv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        sv[u] = v.S(k, ee[u]);
        yv[u] = v.Y(k, ee[u]);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) d[u] += ci * sv[u] + yi * yv[u];
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (e0 + u * nth < e_end) {
        v.setD(ee[u], (float)d[u]);
        v.setT(ee[u], v.X(ee[u]) + d[u]);  // trial point at alpha = 1
        dg += d[u] * gv[u];
      }
  }
  dg = block_sum_f64(dg, red);
  if (tid == 0) a.dpart[(size_t)r * kDirChunks + chunk] = dg;
}

// The descent test of every pending direction (the block sums of d . g added
// in chunk order); where d is not a descent direction, steepest descent from
// the iterate with the history forgotten.
__global__ __launch_bounds__(kDirThreads) void lbfgs_dir_finish_kernel(BatchArgs b) {
  const int idx = blockIdx.x;
  if (idx >= *b.n_active) return;
  const int g = __builtin_amdgcn_readfirstlane(b.active[idx]);
  const int m = __builtin_amdgcn_readfirstlane(b.msa_of[g]);
  const LbfgsArgs a = load_uniform(b.lb + m);
  const int r = __builtin_amdgcn_readfirstlane(g - b.site_base[m]);
  SiteState* S = a.st + r;
  const int pend = __builtin_amdgcn_readfirstlane(S->dpend);
  __syncthreads();  // every wave has read the flag before it is cleared
  if (pend == 0) return;
  double dg = 0.0;
  for (int c = 0; c < kDirChunks; ++c) dg += a.dpart[(size_t)r * kDirChunks + c];
  const int tid = threadIdx.x, nth = blockDim.x;
  if (dg < 0.0) {
    if (tid == 0) {
      S->gtd = dg;
      S->alpha = 1.0;
      S->dpend = 0;
    }
    return;
  }
  const double gnorm = S->gnorm;
  const double alpha = fmin(1.0, 1.0 / gnorm);
  const SiteVecs v(a, r);
  const int P = a.q + a.N * a.q * a.q;
  for (int e = tid; e < P; e += nth) {
    const float d = (float)-v.G(e);
    v.setD(e, d);
    v.setT(e, v.X(e) + alpha * (double)d);
  }
  if (tid == 0) {
    S->gtd = -gnorm * gnorm;
    S->alpha = alpha;
    S->stored = 0;
    S->dpend = 0;
  }
}

hipError_t launch_lbfgs(const BatchArgs& b, int32_t nblocks, hipStream_t st) {
  hipLaunchKernelGGL(lbfgs_kernel, dim3(nblocks), dim3(kLbThreads), 0, st, b);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(lbfgs_dir_kernel, dim3(nblocks * kDirChunks), dim3(kDirThreads), 0, st, b);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(lbfgs_dir_finish_kernel, dim3(nblocks), dim3(kDirThreads), 0, st, b);
  return hipGetLastError();
}

}  // namespace plm
