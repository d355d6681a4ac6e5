// k_reweight.hip -- sequence reweighting (sec. 3.1, eq. inverse_weights;
// sec. 3.4 step 2, eq. inverse_weights2).
//
// id(a,b) = number of columns where rows a and b hold the same symbol (gap =
// gap counts).  Rows are packed four symbols per 32-bit word; for x = A ^ B a
// byte of x is zero exactly where the symbols agree, and the high bit of
// ((x & 0x7f7f7f7f) + 0x7f7f7f7f) | x marks the non-zero bytes, so one popcount
// per word counts the disagreements.  Each block compares a 64 x 64 tile of
// row pairs (upper triangle only) with integer arithmetic; counts m_b are
// integer atomics, so the result does not depend on scheduling.
#include "plm_internal.h"

namespace plm {

constexpr int kRwTile = 64;
constexpr int kRwWords = 32;  // words (4 columns each) staged per chunk

__global__ void fill_i32_kernel(int32_t* p, int32_t v, int32_t n) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) p[e] = v;
}

__global__ __launch_bounds__(256) void identity_kernel(const uint8_t* __restrict__ msa, int32_t B,
                                                       int32_t N, int32_t q, int32_t T,
                                                       int32_t ntile, int32_t* __restrict__ m,
                                                       int32_t* flag) {
  __shared__ uint32_t As[kRwTile][kRwWords + 1];
  __shared__ uint32_t Bs[kRwTile][kRwWords + 1];
  __shared__ int32_t cntA[kRwTile], cntB[kRwTile];
  // upper-triangular tile index -> (ta, tb), ta <= tb
  int64_t lin = blockIdx.x;
  int ta = 0;
  {
    int64_t rowlen = ntile;
    while (lin >= rowlen) { lin -= rowlen; ++ta; --rowlen; }
  }
  const int tb = ta + (int)lin;
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  if (tid < kRwTile) { cntA[tid] = 0; cntB[tid] = 0; }
  uint32_t nz[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) nz[u][v] = 0;
  const int W = (N + 3) / 4;
  int bad = 0;
  for (int w0 = 0; w0 < W; w0 += kRwWords) {
    __syncthreads();
    for (int e = tid; e < kRwTile * kRwWords; e += 256) {
      const int row = e / kRwWords, wd = e - row * kRwWords, word = w0 + wd;
      uint32_t va = 0, vb = 0;
      const int ra = ta * kRwTile + row, rb = tb * kRwTile + row;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int col = 4 * word + k;
        if (col < N) {
          if (ra < B) {
            const uint32_t c = msa[(size_t)ra * N + col];
            bad |= c >= (uint32_t)q;
            va |= c << (8 * k);
          }
          if (rb < B) {
            const uint32_t c = msa[(size_t)rb * N + col];
            bad |= c >= (uint32_t)q;
            vb |= c << (8 * k);
          }
        }
      }
      As[row][wd] = va;
      Bs[row][wd] = vb;
    }
    __syncthreads();
    const int nw = min(kRwWords, W - w0);
    for (int wd = 0; wd < nw; ++wd) {
      uint32_t a4[4], b4[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) a4[u] = As[ty * 4 + u][wd];
#pragma unroll
      for (int v = 0; v < 4; ++v) b4[v] = Bs[tx * 4 + v][wd];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const uint32_t x = a4[u] ^ b4[v];
          const uint32_t y = ((x & 0x7f7f7f7fu) + 0x7f7f7f7fu) | x;
          nz[u][v] += __popc(y & 0x80808080u);
        }
    }
  }
  if (bad && flag) atomicOr(flag, 1);
  // padding bytes are zero on both sides and always agree, so id = N - nz
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int la = ty * 4 + u, lb = tx * 4 + v;
      const int a = ta * kRwTile + la, b = tb * kRwTile + lb;
      if (a >= B || b >= B) continue;
      if (ta == tb && a > b) continue;
      const int id = N - (int)nz[u][v];
      if (id >= T) {
        atomicAdd(&cntA[la], 1);
        if (a != b) atomicAdd(&cntB[lb], 1);
      }
    }
  __syncthreads();
  if (tid < kRwTile) {
    const int a = ta * kRwTile + tid, b = tb * kRwTile + tid;
    if (a < B && cntA[tid]) atomicAdd(&m[a], cntA[tid]);
    if (b < B && cntB[tid]) atomicAdd(&m[b], cntB[tid]);
  }
}

// w_b = 1/m_b (IEEE division, correctly rounded) and B_eff summed in index order.
__global__ void weights_kernel(const int32_t* m, int32_t B, int32_t uniform, double* w,
                               double* beff) {
  for (int b = threadIdx.x; b < B; b += blockDim.x) w[b] = uniform ? 1.0 : 1.0 / (double)m[b];
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int b = 0; b < B; ++b) t += w[b];
    *beff = t;
  }
}

int32_t identity_threshold(int32_t N, double theta) {
  // smallest integer id with (double)id / (double)N >= theta: the comparison the
  // definition makes, evaluated once per id on the host
  for (int32_t t = 0; t <= N; ++t)
    if ((double)t / (double)N >= theta) return t;
  return N + 1;
}

hipError_t launch_reweight(const uint8_t* msa, int32_t B, int32_t N, int32_t q, double theta,
                           int32_t uniform, int32_t* m, double* w, double* beff, int32_t* flag,
                           hipStream_t st) {
  const int fb = (B + 255) / 256 < 4096 ? (B + 255) / 256 : 4096;
  hipLaunchKernelGGL(fill_i32_kernel, dim3(fb), dim3(256), 0, st, m, 0, B);
  if (!uniform) {
    const int T = identity_threshold(N, theta);
    const int ntile = (B + kRwTile - 1) / kRwTile;
    const int64_t ntri = (int64_t)ntile * (ntile + 1) / 2;
    if (ntri > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(identity_kernel, dim3((unsigned)ntri), dim3(256), 0, st, msa, B, N, q, T,
                       ntile, m, flag);
  } else {
    hipLaunchKernelGGL(fill_i32_kernel, dim3(fb), dim3(256), 0, st, m, 1, B);
  }
  hipLaunchKernelGGL(weights_kernel, dim3(1), dim3(1024), 0, st, m, B, uniform, w, beff);
  return hipGetLastError();
}

}  // namespace plm
