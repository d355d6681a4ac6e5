// k_mf.hip -- mean-field starting guess (sec. 2 and sec. 7): couplings from
// the inverse of the connected correlation matrix
//   c_ij(k,l) = f_ij(k,l) - f_i(k) f_j(l),   k, l < q - 1,
// built from reweighted frequencies mixed with a uniform pseudocount of
// weight lam (f_i = (1-lam) F_i/B_eff + lam/q, f_ij = (1-lam) F_ij/B_eff +
// lam/q^2 for i != j, f_ii(k,l) = f_i(k)[k = l]); J_ij(k,l) = -(C^-1)_(i,k),(j,l)
// with the last state (the gap) as reference, and the fields of the
// mean-field equations in that gauge,
//   h_i(k) = ln(f_i(k)/f_i(q-1)) - sum_{j != i} sum_{l < q-1} J_ij(k,l) f_j(l).
//
// Steps (all FP64, every sum in a fixed order):
//   sort    per column, a stable counting sort of the sequence indices by
//           state (one block per column)
//   single  f_i(k): the weights of one state's run summed in sorted order
//   pair    for one (i, k): the weights of the rows with state k at i,
//           histogrammed by the state of every column j; each thread owns
//           the bins of one column in LDS, so no two threads touch a bin;
//           writes row (i, k) of C
//   invert  in-place block Gauss-Jordan on the SPD matrix C (64 x 64 pivot
//           blocks, no pivoting: every pivot block is a Schur complement of
//           an SPD matrix); per pivot block: invert it, scale its row
//           panel, rank-64 update of every other tile, scale its column panel
//   output  J in the asymmetric layout J[r][i][k][s] = J_ri(s, k) (both
//           estimates equal) and the fields
#include <math.h>

#include "plm_internal.h"

namespace plm {

constexpr int kMfThreads = 256;
constexpr int kGjTile = 64;              // pivot block and tile size
constexpr int kGjLd = kGjTile + 4;       // LDS row stride of a staged tile (doubles)

// ---- sort ------------------------------------------------------------------
// order[i*B + t] = the t-th sequence (by index) among those sorted by state
// at column i; start[i*(q+1) + k] = first position of state k.  Symbols >= q
// raise bit 1 of *flag and are counted as state q - 1.
__global__ __launch_bounds__(kMfThreads) void mf_sort_kernel(const uint8_t* msa, int32_t B, int32_t N,
                                                             int32_t q, int32_t* order, int32_t* start,
                                                             int32_t* flag) {
  __shared__ int32_t cnt[kQMax][kMfThreads];
  __shared__ int32_t base[kQMax + 1];
  const int i = blockIdx.x, t = threadIdx.x;
  const int chunk = (B + kMfThreads - 1) / kMfThreads;
  const int b0 = min(B, t * chunk), b1 = min(B, b0 + chunk);
  for (int k = 0; k < q; ++k) cnt[k][t] = 0;
  bool bad = false;
  for (int b = b0; b < b1; ++b) {
    int s = msa[(size_t)b * N + i];
    if (s >= q) {
      bad = true;
      s = q - 1;
    }
    cnt[s][t] += 1;
  }
  if (bad && flag) atomicOr(flag, 1);
  __syncthreads();
  // exclusive prefix over (state, thread): state-major so that each state's
  // run is in sequence order
  if (t < q) {
    int acc = 0;
    for (int u = 0; u < kMfThreads; ++u) {
      const int c = cnt[t][u];
      cnt[t][u] = acc;
      acc += c;
    }
    base[t + 1] = acc;  // the run length of state t
  }
  __syncthreads();
  if (t == 0) {
    base[0] = 0;
    for (int k = 0; k < q; ++k) base[k + 1] += base[k];
    for (int k = 0; k <= q; ++k) start[(size_t)i * (q + 1) + k] = base[k];
  }
  __syncthreads();
  int pos[kQMax];
#pragma unroll
  for (int k = 0; k < kQMax; ++k) pos[k] = k < q ? base[k] + cnt[k][t] : 0;
  for (int b = b0; b < b1; ++b) {
    int s = msa[(size_t)b * N + i];
    if (s >= q) s = q - 1;
    int p = 0;
#pragma unroll
    for (int k = 0; k < kQMax; ++k)
      if (k == s) p = pos[k]++;
    order[(size_t)i * B + p] = b;
  }
}

// ---- single-site frequencies -------------------------------------------------
__global__ void mf_single_kernel(const int32_t* order, const int32_t* start, const double* w,
                                 const double* beff, int32_t B, int32_t N, int32_t q, double lam,
                                 double* fi) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N * q) return;
  const int i = e / q, k = e - i * q;
  const int32_t* o = order + (size_t)i * B;
  const int a = start[(size_t)i * (q + 1) + k], z = start[(size_t)i * (q + 1) + k + 1];
  double t = 0.0;
  for (int p = a; p < z; ++p) t += w[o[p]];
  fi[e] = (1.0 - lam) * t / *beff + lam / q;
}

// ---- pair frequencies -> rows of C -------------------------------------------
// Block (i, k, jb): row (i, k) of C over the columns of sites jb*256 .. +255.
// C is n_pad x n_pad row-major, n = N (q - 1), entry ((i,k), (j,l)) at
// (i (q-1) + k) * ld + j (q-1) + l.
__global__ __launch_bounds__(kMfThreads) void mf_pair_kernel(const uint8_t* msa, const int32_t* order,
                                                             const int32_t* start, const double* w,
                                                             const double* beff, const double* fi,
                                                             int32_t B, int32_t N, int32_t q, double lam,
                                                             double* C, int64_t ld) {
  __shared__ double bins[kQMax][kMfThreads];
  __shared__ int32_t rows[kMfThreads];
  __shared__ double wts[kMfThreads];
  const int i = blockIdx.x, k = blockIdx.y, t = threadIdx.x;
  const int j0 = blockIdx.z * kMfThreads, j = j0 + t;
  const int r = q - 1;
  for (int l = 0; l < q; ++l) bins[l][t] = 0.0;
  const int32_t* o = order + (size_t)i * B;
  const int a = start[(size_t)i * (q + 1) + k], z = start[(size_t)i * (q + 1) + k + 1];
  for (int c0 = a; c0 < z; c0 += kMfThreads) {
    const int nc = min(kMfThreads, z - c0);
    __syncthreads();
    if (t < nc) {
      const int b = o[c0 + t];
      rows[t] = b;
      wts[t] = w[b];
    }
    __syncthreads();
    if (j < N) {
      int c = 0;
      for (; c + 8 <= nc; c += 8) {
        uint8_t s[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) s[u] = msa[(size_t)rows[c + u] * N + j];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int su = s[u] < q ? s[u] : q - 1;
          bins[su][t] += wts[c + u];
        }
      }
      for (; c < nc; ++c) {
        const uint8_t s = msa[(size_t)rows[c] * N + j];
        bins[s < q ? s : q - 1][t] += wts[c];
      }
    }
  }
  __syncthreads();
  // row (i, k) of C over columns (j, l), j in [j0, j0 + 256), l < q - 1,
  // written contiguously
  const double ib = 1.0 / *beff, fik = fi[(size_t)i * q + k];
  const int jn = min(kMfThreads, N - j0);
  double* row = C + (size_t)(i * r + k) * ld + (size_t)j0 * r;
  for (int e = t; e < jn * r; e += kMfThreads) {
    const int jl = e / r, l = e - jl * r, jj = j0 + jl;
    const double fjl = fi[(size_t)jj * q + l];
    double v;
    if (jj == i)
      v = (l == k ? fik : 0.0) - fik * fjl;
    else
      v = (1.0 - lam) * bins[l][jl] * ib + lam / ((double)q * q) - fik * fjl;
    row[e] = v;
  }
}

// identity on the padded rows and columns [n, n_pad)
__global__ void mf_pad_kernel(double* C, int64_t ld, int32_t n, int32_t n_pad) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t npad = n_pad - n;
  if (npad <= 0) return;
  // region 1: rows [n, n_pad) x all columns; region 2: rows [0, n) x columns [n, n_pad)
  const int64_t r1 = npad * n_pad, r2 = (int64_t)n * npad;
  if (e < r1) {
    const int64_t rr = n + e / n_pad, cc = e % n_pad;
    C[rr * ld + cc] = rr == cc ? 1.0 : 0.0;
  } else if (e < r1 + r2) {
    const int64_t f = e - r1, rr = f / npad, cc = n + f % npad;
    C[rr * ld + cc] = 0.0;
  }
}

// ---- block Gauss-Jordan inversion -------------------------------------------
// Stage a 64 x 64 tile of A (row-major, leading dimension ld) in LDS.
// transposed: S[c][r] = A[r][c]; otherwise S[r][c] = A[r][c].
__device__ inline void stage_tile(const double* A, int64_t ld, int r0, int c0, double* S, bool transposed) {
  for (int e = threadIdx.x; e < kGjTile * kGjTile; e += blockDim.x) {
    const int rr = e / kGjTile, cc = e - rr * kGjTile;
    const double v = A[(size_t)(r0 + rr) * ld + c0 + cc];
    if (transposed)
      S[cc * kGjLd + rr] = v;
    else
      S[rr * kGjLd + cc] = v;
  }
}

// acc[4][4] = (X Y)[ty*4 + a][tx*4 + b] with X staged transposed (Xt[k][row])
// and Y staged plain (Y[k][col]).
__device__ inline void tile_product(const double* Xt, const double* Y, double (&acc)[4][4]) {
  const int ty = threadIdx.x >> 4, tx = threadIdx.x & 15;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
#pragma unroll 4
  for (int kk = 0; kk < kGjTile; ++kk) {
    double x[4], y[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) x[a] = Xt[kk * kGjLd + ty * 4 + a];
#pragma unroll
    for (int b = 0; b < 4; ++b) y[b] = Y[kk * kGjLd + tx * 4 + b];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] = fma(x[a], y[b], acc[a][b]);
  }
}

// Invert the pivot block in place (sweep of its 64 indices).  A pivot that
// is not positive raises bit 8 of *flag (the matrix is not positive definite).
__global__ __launch_bounds__(kMfThreads) void gj_pivot_kernel(double* A, int64_t ld, int32_t p, int32_t* flag) {
  __shared__ double M[kGjTile * kGjLd];
  __shared__ double rowk[kGjTile], colk[kGjTile];
  const int o = p * kGjTile;
  stage_tile(A, ld, o, o, M, false);
  __syncthreads();
  bool bad = false;
  for (int k = 0; k < kGjTile; ++k) {
    if (threadIdx.x < kGjTile) {
      rowk[threadIdx.x] = M[k * kGjLd + threadIdx.x];
      colk[threadIdx.x] = M[threadIdx.x * kGjLd + k];
    }
    __syncthreads();
    const double a = rowk[k];
    if (!(a > 0.0)) bad = true;
    const double ia = 1.0 / a;
    for (int e = threadIdx.x; e < kGjTile * kGjTile; e += blockDim.x) {
      const int rr = e / kGjTile, cc = e - rr * kGjTile;
      double v;
      if (rr == k && cc == k)
        v = ia;
      else if (rr == k)
        v = rowk[cc] * ia;
      else if (cc == k)
        v = -colk[rr] * ia;
      else
        v = M[rr * kGjLd + cc] - colk[rr] * rowk[cc] * ia;
      M[rr * kGjLd + cc] = v;
    }
    __syncthreads();
  }
  if (bad && threadIdx.x == 0 && flag) atomicOr(flag, 8);
  for (int e = threadIdx.x; e < kGjTile * kGjTile; e += blockDim.x) {
    const int rr = e / kGjTile, cc = e - rr * kGjTile;
    A[(size_t)(o + rr) * ld + o + cc] = M[rr * kGjLd + cc];
  }
}

// Row panel: A[p][j] <- P A[p][j] for every tile column j != p.
__global__ __launch_bounds__(kMfThreads) void gj_row_kernel(double* A, int64_t ld, int32_t p) {
  __shared__ double Pt[kGjTile * kGjLd], Y[kGjTile * kGjLd];
  const int j = blockIdx.x < (unsigned)p ? blockIdx.x : blockIdx.x + 1;
  const int o = p * kGjTile, c0 = j * kGjTile;
  stage_tile(A, ld, o, o, Pt, true);
  stage_tile(A, ld, o, c0, Y, false);
  __syncthreads();
  double acc[4][4];
  tile_product(Pt, Y, acc);
  const int ty = threadIdx.x >> 4, tx = threadIdx.x & 15;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) A[(size_t)(o + ty * 4 + a) * ld + c0 + tx * 4 + b] = acc[a][b];
}

// Update: A[i][j] <- A[i][j] - A[i][p] A[p][j] for tiles i != p, j != p
// (A[p][j] already scaled, A[i][p] not yet).
__global__ __launch_bounds__(kMfThreads) void gj_update_kernel(double* A, int64_t ld, int32_t p) {
  __shared__ double Xt[kGjTile * kGjLd], Y[kGjTile * kGjLd];
  const int i = blockIdx.y < (unsigned)p ? blockIdx.y : blockIdx.y + 1;
  const int j = blockIdx.x < (unsigned)p ? blockIdx.x : blockIdx.x + 1;
  const int o = p * kGjTile, r0 = i * kGjTile, c0 = j * kGjTile;
  stage_tile(A, ld, r0, o, Xt, true);
  stage_tile(A, ld, o, c0, Y, false);
  __syncthreads();
  double acc[4][4];
  tile_product(Xt, Y, acc);
  const int ty = threadIdx.x >> 4, tx = threadIdx.x & 15;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      double* d = A + (size_t)(r0 + ty * 4 + a) * ld + c0 + tx * 4 + b;
      *d = *d - acc[a][b];
    }
}

// Column panel: A[i][p] <- -A[i][p] P for every tile row i != p.
__global__ __launch_bounds__(kMfThreads) void gj_col_kernel(double* A, int64_t ld, int32_t p) {
  __shared__ double Xt[kGjTile * kGjLd], P[kGjTile * kGjLd];
  const int i = blockIdx.x < (unsigned)p ? blockIdx.x : blockIdx.x + 1;
  const int o = p * kGjTile, r0 = i * kGjTile;
  stage_tile(A, ld, r0, o, Xt, true);
  stage_tile(A, ld, o, o, P, false);
  __syncthreads();
  double acc[4][4];
  tile_product(Xt, P, acc);
  const int ty = threadIdx.x >> 4, tx = threadIdx.x & 15;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) A[(size_t)(r0 + ty * 4 + a) * ld + o + tx * 4 + b] = -acc[a][b];
}

// ---- output ------------------------------------------------------------------
// J[a][i][k][s] = -Cinv[(a,s),(i,k)] for s, k < q - 1 and a != i; 0 otherwise.
__global__ __launch_bounds__(kMfThreads) void mf_couplings_kernel(const double* Cinv, int64_t ld, int32_t N,
                                                                  int32_t q, float* J) {
  const int a = blockIdx.y, i = blockIdx.x, r = q - 1, qq = q * q;
  float* out = J + ((size_t)a * N + i) * qq;
  for (int e = threadIdx.x; e < qq; e += blockDim.x) {
    const int k = e / q, s = e - k * q;
    float v = 0.f;
    if (a != i && k < r && s < r) v = (float)(-Cinv[(size_t)(a * r + s) * ld + i * r + k]);
    out[e] = v;
  }
}

// h_a(s) = ln(f_a(s)/f_a(q-1)) + sum_{i != a} sum_{k < q-1} Cinv[(a,s),(i,k)] f_i(k);
// a zero reference frequency (possible only without pseudocounts) raises bit 8.
__global__ __launch_bounds__(kMfThreads) void mf_fields_kernel(const double* Cinv, int64_t ld, const double* fi,
                                                               int32_t N, int32_t q, float* h, int32_t* flag) {
  __shared__ double red[kMfThreads / 64];
  const int a = blockIdx.x, r = q - 1;
  if (threadIdx.x == 0 && !(fi[(size_t)a * q + r] > 0.0) && flag) atomicOr(flag, 8);
  for (int s = 0; s < r; ++s) {
    const double* row = Cinv + (size_t)(a * r + s) * ld;
    double t = 0.0;
    for (int e = threadIdx.x; e < N * r; e += blockDim.x) {
      const int i = e / r, k = e - i * r;
      if (i != a) t += row[e] * fi[(size_t)i * q + k];
    }
    t = block_sum_f64(t, red);
    if (threadIdx.x == 0)
      h[(size_t)a * q + s] = (float)(log(fi[(size_t)a * q + s] / fi[(size_t)a * q + r]) + t);
  }
  if (threadIdx.x == 0) h[(size_t)a * q + r] = 0.f;
}

// ---- host side -------------------------------------------------------------------
int32_t mf_tile() { return kGjTile; }

hipError_t launch_mf_frequencies(const uint8_t* msa, int32_t B, int32_t N, int32_t q, const double* w,
                                 const double* beff, double lam, int32_t* order, int32_t* start, double* fi,
                                 int32_t* flag, hipStream_t st) {
  hipLaunchKernelGGL(mf_sort_kernel, dim3(N), dim3(kMfThreads), 0, st, msa, B, N, q, order, start, flag);
  hipLaunchKernelGGL(mf_single_kernel, dim3((N * q + 255) / 256), dim3(256), 0, st, order, start, w, beff, B,
                     N, q, lam, fi);
  return hipGetLastError();
}

hipError_t launch_mf_correlation(const uint8_t* msa, const int32_t* order, const int32_t* start, const double* w,
                                 const double* beff, const double* fi, int32_t B, int32_t N, int32_t q,
                                 double lam, double* C, int32_t n_pad, hipStream_t st) {
  const int r = q - 1, n = N * r;
  hipLaunchKernelGGL(mf_pair_kernel, dim3(N, r, (N + kMfThreads - 1) / kMfThreads), dim3(kMfThreads), 0, st,
                     msa, order, start, w, beff, fi, B, N, q, lam, C, (int64_t)n_pad);
  const int64_t npad = n_pad - n;
  if (npad > 0) {
    const int64_t tot = npad * n_pad + (int64_t)n * npad;
    hipLaunchKernelGGL(mf_pad_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, C, (int64_t)n_pad,
                       n, n_pad);
  }
  return hipGetLastError();
}

hipError_t launch_mf_invert(double* C, int32_t n_pad, int32_t* flag, hipStream_t st) {
  const int nt = n_pad / kGjTile;
  const int64_t ld = n_pad;
  for (int p = 0; p < nt; ++p) {
    hipLaunchKernelGGL(gj_pivot_kernel, dim3(1), dim3(kMfThreads), 0, st, C, ld, p, flag);
    if (nt > 1) {
      hipLaunchKernelGGL(gj_row_kernel, dim3(nt - 1), dim3(kMfThreads), 0, st, C, ld, p);
      hipLaunchKernelGGL(gj_update_kernel, dim3(nt - 1, nt - 1), dim3(kMfThreads), 0, st, C, ld, p);
      hipLaunchKernelGGL(gj_col_kernel, dim3(nt - 1), dim3(kMfThreads), 0, st, C, ld, p);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_mf_output(const double* Cinv, int32_t n_pad, const double* fi, int32_t N, int32_t q, float* h,
                            float* J, int32_t* flag, hipStream_t st) {
  hipLaunchKernelGGL(mf_couplings_kernel, dim3(N, N), dim3(kMfThreads), 0, st, Cinv, (int64_t)n_pad, N, q, J);
  hipLaunchKernelGGL(mf_fields_kernel, dim3(N), dim3(kMfThreads), 0, st, Cinv, (int64_t)n_pad, fi, N, q, h, flag);
  return hipGetLastError();
}

}  // namespace plm
