// k_score.hip -- coupling scores of asymmetric plmDCA (sec. 3.4 steps 4-6).
//
// One wave per pair (i, j), i < j: both estimates of the pair as q x q
// matrices indexed (state of i, state of j) -- the site-i estimate is
// J[i][j][k][s] read with s the state of i, the site-j estimate J[j][i][k][s]
// with s the state of j, i.e. transposed -- each moved to the Ising gauge by
// subtracting row and column means and adding the grand mean
// (eq. gauge_change2), averaged (eq. average2) and reduced to the Frobenius
// norm (eq. frob_normtrans2).  A second pass applies the average product
// correction (eq. corr_norm2) with means over all N positions.  FP64.  The
// same kernels compute the variants the paper also tried (sec. 7): min/max
// combinations, l_p norms, the Burkoff divergence (eqs. burkoffscore1,
// burkoffscore2), the gap state left out, and the average-sum correction
// (eq. corr_normsum).
#include "plm_internal.h"

namespace plm {

// One wave per pair (i < j): both estimates to the Ising gauge, combined
// (average, elementwise min or max), reduced by the chosen norm over all
// states or over the non-gap states 0..q-2: Frobenius, l_p (sum of |J|^p to
// the power 1/p), or the Burkoff divergence sum P ln(P / (f_i f_j)) with
// P proportional to f_i(k) f_j(l) exp(J(k,l)) (computed with the largest
// exponent factored out).
__global__ __launch_bounds__(64) void pair_score_kernel(const float* __restrict__ J, int32_t N,
                                                        int32_t q, ScoreOpts o,
                                                        const double* __restrict__ freq,
                                                        double* __restrict__ raw) {
  __shared__ double A[kQMax * kQMax], Bm[kQMax * kQMax];
  __shared__ double rA[kQMax], cA[kQMax], rB[kQMax], cB[kQMax];
  const int i = blockIdx.y, j = blockIdx.x;
  if (j <= i) {
    if (j == i && threadIdx.x == 0) raw[(size_t)i * N + i] = 0.0;
    return;
  }
  const int lane = threadIdx.x, qq = q * q;
  const size_t bij = ((size_t)i * N + j) * qq, bji = ((size_t)j * N + i) * qq;
  for (int e = lane; e < qq; e += 64) {
    const int a = e / q, c = e - a * q;  // a: state of i, c: state of j
    A[e] = (double)J[bij + (size_t)c * q + a];
    Bm[e] = (double)J[bji + (size_t)a * q + c];
  }
  __syncthreads();
  if (lane < q) {
    double s1 = 0.0, s2 = 0.0, s3 = 0.0, s4 = 0.0;
    for (int c = 0; c < q; ++c) { s1 += A[lane * q + c]; s3 += Bm[lane * q + c]; }
    for (int a = 0; a < q; ++a) { s2 += A[a * q + lane]; s4 += Bm[a * q + lane]; }
    rA[lane] = s1 / q;
    cA[lane] = s2 / q;
    rB[lane] = s3 / q;
    cB[lane] = s4 / q;
  }
  __syncthreads();
  double gA = 0.0, gB = 0.0;
  for (int a = 0; a < q; ++a) { gA += rA[a]; gB += rB[a]; }
  gA /= q;
  gB /= q;
  const int qs = o.exclude_gap ? q - 1 : q;  // states summed over
  auto combined = [&](int e) {
    const int a = e / q, c = e - a * q;
    const double ga = A[e] - cA[c] - rA[a] + gA;
    const double gb = Bm[e] - cB[c] - rB[a] + gB;
    return o.combine == PLM_COMBINE_MIN ? fmin(ga, gb) : o.combine == PLM_COMBINE_MAX ? fmax(ga, gb)
                                                                                         : 0.5 * (ga + gb);
  };
  auto included = [&](int e) {
    const int a = e / q, c = e - a * q;
    return a < qs && c < qs;
  };
  double out = 0.0;
  if (o.norm == PLM_NORM_BURKOFF) {
    double mx = -INFINITY;
    for (int e = lane; e < qq; e += 64)
      if (included(e)) mx = fmax(mx, combined(e));
    for (int d = 32; d > 0; d >>= 1) mx = fmax(mx, __shfl_xor(mx, d, 64));
    double z = 0.0, zv = 0.0;
    for (int e = lane; e < qq; e += 64)
      if (included(e)) {
        const int a = e / q, c = e - a * q;
        const double v = combined(e);
        const double t = freq[(size_t)i * q + a] * freq[(size_t)j * q + c] * exp(v - mx);
        z += t;
        zv += t * v;
      }
    for (int d = 32; d > 0; d >>= 1) {
      z += __shfl_xor(z, d, 64);
      zv += __shfl_xor(zv, d, 64);
    }
    out = z > 0.0 ? zv / z - mx - log(z) : 0.0;
  } else {
    const bool lp = o.norm == PLM_NORM_LP;
    double ss = 0.0;
    for (int e = lane; e < qq; e += 64)
      if (included(e)) {
        const double v = combined(e);
        ss += lp ? pow(fabs(v), o.p) : v * v;
      }
    for (int d = 32; d > 0; d >>= 1) ss += __shfl_xor(ss, d, 64);
    out = lp ? pow(ss, 1.0 / o.p) : sqrt(ss);
  }
  if (lane == 0) {
    raw[(size_t)i * N + j] = out;
    raw[(size_t)j * N + i] = out;
  }
}

// row sums of the raw scores, parked on the diagonal of the output until the last pass
__global__ void rowsum_kernel(const double* __restrict__ fn, int32_t N, double* __restrict__ cfn) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double s = 0.0;
  for (int j = 0; j < N; ++j) s += fn[(size_t)i * N + j];
  cfn[(size_t)i * N + i] = s;
}

// Correction of the symmetric raw scores with means over all N positions:
// average product (eq. corr_norm2), average sum (eq. corr_normsum) or none;
// zero diagonal.
__global__ __launch_bounds__(1024) void correct_kernel(const double* __restrict__ fn, int32_t N,
                                                       int32_t mode, double* __restrict__ cfn) {
  __shared__ double all_s;
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < N; ++i) t += cfn[(size_t)i * N + i];
    all_s = t / ((double)N * (double)N);
  }
  __syncthreads();
  const double all = all_s;
  const size_t NN = (size_t)N * N;
  for (size_t e = threadIdx.x; e < NN; e += blockDim.x) {
    const int i = (int)(e / N), j = (int)(e - (size_t)i * N);
    if (i == j) continue;
    const double ri = cfn[(size_t)i * N + i] / (double)N, rj = cfn[(size_t)j * N + j] / (double)N;
    double v;
    if (mode == PLM_CORR_NONE) v = fn[e];
    else if (mode == PLM_CORR_ASC) v = fn[e] - ri - rj + all;
    else v = all == 0.0 ? 0.0 : fn[e] - ri * rj / all;
    cfn[e] = v;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < N; i += blockDim.x) cfn[(size_t)i * N + i] = 0.0;
}

hipError_t launch_score_ex(const float* J, int32_t N, int32_t q, const ScoreOpts& o,
                           const double* freq, double* raw, double* cor, hipStream_t st) {
  hipLaunchKernelGGL(pair_score_kernel, dim3(N, N), dim3(64), 0, st, J, N, q, o, freq, raw);
  hipLaunchKernelGGL(rowsum_kernel, dim3((N + 255) / 256), dim3(256), 0, st, raw, N, cor);
  hipLaunchKernelGGL(correct_kernel, dim3(1), dim3(1024), 0, st, raw, N, o.correction, cor);
  return hipGetLastError();
}

hipError_t launch_score(const float* J, int32_t N, int32_t q, double* fn, double* cfn,
                        hipStream_t st) {
  ScoreOpts o;
  o.combine = PLM_COMBINE_AVG;
  o.norm = PLM_NORM_FROB;
  o.p = 2.0;
  o.exclude_gap = 0;
  o.correction = PLM_CORR_APC;
  return launch_score_ex(J, N, q, o, nullptr, fn, cfn, st);
}

// Reweighted single-site frequencies f_i(k) = sum_b w_b [sigma_i^b = k] / B_eff:
// one block per column; per-thread FP64 counters in LDS, then a fixed-order
// sum over the threads.
__global__ __launch_bounds__(256) void freq_kernel(const uint8_t* __restrict__ msa, int32_t B,
                                                   int32_t N, int32_t q,
                                                   const double* __restrict__ w,
                                                   const double* __restrict__ beff,
                                                   double* __restrict__ f) {
  __shared__ double cnt[256 * kQMax];
  const int i = blockIdx.x, t = threadIdx.x;
  for (int k = 0; k < kQMax; ++k) cnt[t * kQMax + k] = 0.0;
  for (int b = t; b < B; b += 256) {
    const int k = msa[(size_t)b * N + i];
    if (k < q) cnt[t * kQMax + k] += w[b];
  }
  __syncthreads();
  if (t < q) {
    double s = 0.0;
    for (int u = 0; u < 256; ++u) s += cnt[u * kQMax + t];
    f[(size_t)i * q + t] = s / *beff;
  }
}

hipError_t launch_frequencies(const uint8_t* msa, int32_t B, int32_t N, int32_t q, const double* w,
                              const double* beff, double* f, hipStream_t st) {
  hipLaunchKernelGGL(freq_kernel, dim3(N), dim3(256), 0, st, msa, B, N, q, w, beff, f);
  return hipGetLastError();
}

}  // namespace plm
