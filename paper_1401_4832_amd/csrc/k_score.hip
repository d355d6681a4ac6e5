// k_score.hip -- coupling scores of asymmetric plmDCA (sec. 3.4 steps 4-6).
//
// One wave per pair (i, j), i < j: both estimates of the pair as q x q
// matrices indexed (state of i, state of j) -- the site-i estimate is
// J[i][j][k][s] read with s the state of i, the site-j estimate J[j][i][k][s]
// with s the state of j, i.e. transposed -- each moved to the Ising gauge by
// subtracting row and column means and adding the grand mean
// (eq. gauge_change2), averaged (eq. average2) and reduced to the Frobenius
// norm (eq. frob_normtrans2).  A second pass applies the average product
// correction (eq. corr_norm2) with means over all N positions.  FP64.
#include "plm_internal.h"

namespace plm {

__global__ __launch_bounds__(64) void fn_kernel(const float* __restrict__ J, int32_t N, int32_t q,
                                                double* __restrict__ fn) {
  __shared__ double A[kQMax * kQMax], Bm[kQMax * kQMax];
  __shared__ double rA[kQMax], cA[kQMax], rB[kQMax], cB[kQMax];
  const int i = blockIdx.y, j = blockIdx.x;
  if (j <= i) {
    if (j == i && threadIdx.x == 0) fn[(size_t)i * N + i] = 0.0;
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
  double ss = 0.0;
  for (int e = lane; e < qq; e += 64) {
    const int a = e / q, c = e - a * q;
    const double ga = A[e] - cA[c] - rA[a] + gA;
    const double gb = Bm[e] - cB[c] - rB[a] + gB;
    const double v = 0.5 * (ga + gb);
    ss += v * v;
  }
  for (int o = 32; o > 0; o >>= 1) ss += __shfl_xor(ss, o, 64);
  if (lane == 0) {
    const double v = sqrt(ss);
    fn[(size_t)i * N + j] = v;
    fn[(size_t)j * N + i] = v;
  }
}

// row sums of FN, parked on the diagonal of the output until the last pass
__global__ void rowsum_kernel(const double* __restrict__ fn, int32_t N, double* __restrict__ cfn) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double s = 0.0;
  for (int j = 0; j < N; ++j) s += fn[(size_t)i * N + j];
  cfn[(size_t)i * N + i] = s;
}

__global__ __launch_bounds__(1024) void apc_kernel(const double* __restrict__ fn, int32_t N,
                                                   double* __restrict__ cfn) {
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
    cfn[e] = all == 0.0 ? 0.0 : fn[e] - ri * rj / all;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < N; i += blockDim.x) cfn[(size_t)i * N + i] = 0.0;
}

hipError_t launch_score(const float* J, int32_t N, int32_t q, double* fn, double* cfn,
                        hipStream_t st) {
  hipLaunchKernelGGL(fn_kernel, dim3(N, N), dim3(64), 0, st, J, N, q, fn);
  hipLaunchKernelGGL(rowsum_kernel, dim3((N + 255) / 256), dim3(256), 0, st, fn, N, cfn);
  hipLaunchKernelGGL(apc_kernel, dim3(1), dim3(1024), 0, st, fn, N, cfn);
  return hipGetLastError();
}

}  // namespace plm
