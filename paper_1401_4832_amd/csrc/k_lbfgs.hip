// k_lbfgs.hip -- device-resident limited-memory BFGS for all N per-site
// problems of asymmetric plmDCA (sec. 3.4 step 3; the paper minimises each
// g_r^reg by L-BFGS from the origin, secs. 5 and 6).
//
// One block owns one site.  Each launch consumes the evaluation of the site's
// trial point (objective partials from the forward kernel, FP64 gradient data
// part from the backward kernel), adds the l2 terms in FP64, takes the line
// search decision (sufficient decrease with backtracking by safeguarded
// quadratic interpolation), and on acceptance stores the curvature pair,
// runs the two-loop recursion and writes the next trial point.  All dot
// products and the history are FP64; the iterate is kept at FP32-representable
// values so that the evaluated point and the stored point are the same.
#include "plm_internal.h"

namespace plm {

__device__ inline void lbfgs_site(const LbfgsArgs& a, int r, double* red, double* ghd, double* ahist) {
  SiteState* S = a.st + r;
  const int phase = S->phase;
  if (phase == PH_DONE) return;
  const int q = a.q, N = a.N, m = a.m;
  const size_t Nqq = (size_t)N * q * q;
  const int P = q + (int)Nqq;
  const int tid = threadIdx.x, nth = blockDim.x;
  const double beff = *a.beff;
  const double ib = 1.0 / beff;
  const size_t h0 = (size_t)r * q, j0 = (size_t)r * Nqq;
  const int self0 = q + r * q * q, self1 = self0 + q * q;  // self block range in e

  // ---- gather the evaluation at the trial point ----
  if (tid < q) {
    double t = 0.0;
    for (int k = 0; k < a.tiles; ++k) t += a.gh_part[((size_t)k * N + r) * kSlot + tid];
    ghd[tid] = t;
  }
  double fdata = 0.0;
  if (tid == 0)
    for (int k = 0; k < a.tiles; ++k) fdata += a.f_part[(size_t)k * N + r];
  __syncthreads();

  const double lam_h = a.lambda_h, lam_J = a.lambda_Jp;
  auto lam = [&](int e) -> double { return e < q ? lam_h : ((e >= self0 && e < self1) ? 0.0 : lam_J); };
  auto Tv = [&](int e) -> double { return e < q ? (double)a.Th[h0 + e] : (double)a.TJ[j0 + (e - q)]; };
  auto Xv = [&](int e) -> double { return e < q ? (double)a.Xh[h0 + e] : (double)a.XJ[j0 + (e - q)]; };
  auto gtv = [&](int e) -> double {
    const double d = e < q ? ghd[e] : a.gJ[j0 + (e - q)];
    return d * ib + 2.0 * lam(e) * Tv(e);
  };
  auto Gv = [&](int e) -> double { return e < q ? a.Gh[h0 + e] : a.GJ[j0 + (e - q)]; };
  auto Dp = [&](int e) -> double* { return e < q ? a.Dh + h0 + e : a.DJ + j0 + (e - q); };
  auto Gp = [&](int e) -> double* { return e < q ? a.Gh + h0 + e : a.GJ + j0 + (e - q); };
  auto Sv = [&](int k, int e) -> double* {
    return e < q ? a.Sh + ((size_t)k * N) * q + h0 + e : a.SJ + (size_t)k * N * Nqq + j0 + (e - q);
  };
  auto Yv = [&](int k, int e) -> double* {
    return e < q ? a.Yh + ((size_t)k * N) * q + h0 + e : a.YJ + (size_t)k * N * Nqq + j0 + (e - q);
  };
  auto writeT = [&](double alpha) {
    for (int e = tid; e < P; e += nth) {
      const float v = (float)(Xv(e) + alpha * *Dp(e));
      if (e < q) a.Th[h0 + e] = v; else a.TJ[j0 + (e - q)] = (e >= self0 && e < self1) ? 0.f : v;
    }
  };

  double reg = 0.0, gg = 0.0;
  for (int e = tid; e < P; e += nth) {
    const double t = Tv(e), g = gtv(e);
    reg += lam(e) * t * t;
    gg += g * g;
  }
  reg = block_sum_f64(reg, red);
  gg = block_sum_f64(gg, red);
  fdata = block_sum_f64(tid == 0 ? fdata : 0.0, red);
  const double ft = fdata * ib + reg;
  const double gnt = sqrt(gg);
  const bool finite = isfinite(ft) && isfinite(gnt);

  int evals = S->evals + 1;
  int iter = S->iter, ls = S->ls_count, head = S->head, stored = S->stored, status = S->status;
  double f = S->f, gnorm = S->gnorm, alpha = S->alpha, gtd = S->gtd, gamma = S->gamma;
  int newphase = phase;
  // what to do with the search direction once the decision is taken
  enum { KEEP = 0, STEEPEST = 1, QUASI_NEWTON = 2 } dir = KEEP;
  bool move = false;  // write a new trial point

  if (phase == PH_INIT && !finite) {
    newphase = PH_DONE;
    status = PLM_SITE_NONFINITE;
  } else if (phase == PH_INIT ||
             (finite && ft <= f + a.c1 * alpha * gtd + a.noise * fabs(f))) {
    // accept the trial point (the first evaluation is the start point itself);
    // sufficient decrease allows for the rounding noise of the FP32 evaluation
    double sy = 0.0, yy = 0.0;
    const bool pair = (phase != PH_INIT) && m > 0;
    for (int e = tid; e < P; e += nth) {
      const double g = gtv(e);
      if (pair) {
        const double sv = Tv(e) - Xv(e), yv = g - Gv(e);
        *Sv(head, e) = sv;
        *Yv(head, e) = yv;
        sy += sv * yv;
        yy += yv * yv;
      }
      *Gp(e) = g;
      if (e < q) a.Xh[h0 + e] = a.Th[h0 + e]; else a.XJ[j0 + (e - q)] = a.TJ[j0 + (e - q)];
    }
    if (pair) {
      sy = block_sum_f64(sy, red);
      yy = block_sum_f64(yy, red);
      if (sy > 0.0 && yy > 0.0) {
        if (tid == 0) S->rho[head] = 1.0 / sy;
        gamma = sy / yy;
        head = (head + 1) % m;
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
    __syncthreads();
    // two-loop recursion d = -H g over the stored pairs, newest first
    for (int e = tid; e < P; e += nth) *Dp(e) = -Gv(e);
    for (int t = 0; t < stored; ++t) {
      const int k = (head - 1 - t + 2 * m) % m;
      double dot = 0.0;
      for (int e = tid; e < P; e += nth) dot += *Sv(k, e) * *Dp(e);
      dot = block_sum_f64(dot, red);
      const double ak = S->rho[k] * dot;
      if (tid == 0) ahist[t] = ak;
      for (int e = tid; e < P; e += nth) *Dp(e) -= ak * *Yv(k, e);
    }
    for (int e = tid; e < P; e += nth) *Dp(e) *= gamma;
    for (int t = stored - 1; t >= 0; --t) {
      const int k = (head - 1 - t + 2 * m) % m;
      double dot = 0.0;
      for (int e = tid; e < P; e += nth) dot += *Yv(k, e) * *Dp(e);
      dot = block_sum_f64(dot, red);  // its barriers also publish ahist
      const double bk = S->rho[k] * dot;
      const double ck = ahist[t] - bk;
      for (int e = tid; e < P; e += nth) *Dp(e) += ck * *Sv(k, e);
    }
    double dg = 0.0;
    for (int e = tid; e < P; e += nth) dg += *Dp(e) * Gv(e);
    dg = block_sum_f64(dg, red);
    if (dg < 0.0) {
      gtd = dg;
      alpha = 1.0;
    } else {
      dir = STEEPEST;  // not a descent direction
    }
  }
  if (dir == STEEPEST) {
    __syncthreads();
    for (int e = tid; e < P; e += nth) *Dp(e) = -Gv(e);
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
    S->f = f;
    S->gnorm = gnorm;
    S->alpha = alpha;
    S->gtd = gtd;
    S->gamma = gamma;
    if (a.phase_host) a.phase_host[r] = newphase;
  }
}

// One block per active site of the batch.
__global__ __launch_bounds__(1024) void lbfgs_kernel(BatchArgs b) {
  __shared__ double red[16];
  __shared__ double ghd[kSlot];
  __shared__ double ahist[kMMax];
  const int idx = blockIdx.x;
  if (idx >= *b.n_active) return;
  const int g = b.active[idx];
  const int m = b.msa_of[g];
  const LbfgsArgs a = load_uniform(b.lb + m);
  lbfgs_site(a, g - b.site_base[m], red, ghd, ahist);
}

hipError_t launch_lbfgs(const BatchArgs& b, int32_t nblocks, hipStream_t st) {
  hipLaunchKernelGGL(lbfgs_kernel, dim3(nblocks), dim3(1024), 0, st, b);
  return hipGetLastError();
}

}  // namespace plm
