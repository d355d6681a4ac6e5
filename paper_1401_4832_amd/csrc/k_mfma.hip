// k_mfma.hip -- the coupling gradient of asymmetric plmDCA (sec. 3.4 step 3,
// eq. g_gradJ2) as a one-hot matrix product on the gfx950 matrix cores.
//
// For site r, dJ_r[(i,k)][s] = sum_b X[b][(i,k)] R_b(s) with the one-hot
// X[b][(i,k)] = [sigma_i^b = k]: a product of X^T (rows (i,k), inner index b)
// with R_r (inner index b, columns s).  X^T is exact in BF16 and is generated
// in registers from the symbols; R is split into NP BF16 pieces (NP = 3 gives
// back FP32's 24-bit significand, NP = 2 the hi/lo precision path) and every
// piece is multiplied on v_mfma_f32_32x32x16_bf16 with FP32 accumulation,
// folded into FP64 every 256 rows.
//
// Fragment layouts of v_mfma_f32_32x32x16_bf16 (verified on the device): A
// lane l holds row l % 32, inner indices 8 (l / 32) + 0..7; B lane l holds
// column l % 32, the same inner indices; D lane l register j holds row
// 8 (j / 4) + 4 (l / 32) + j % 4, column l % 32.
#include "plm_internal.h"

namespace plm {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int kMWaves = 8;
constexpr int kMThreads = kMWaves * 64;
constexpr int kMRowBlocks = 4;                 // 32-row blocks per wave
constexpr int kMPos = 48;                      // columns per block: 48 * 21 <= 8 * 4 * 32 rows
constexpr int kMChunk = 256;                   // alignment rows per staged chunk (16 steps of 16)
constexpr int kMSteps = kMChunk / 16;

__device__ inline uint32_t f2bf(float f) {     // round to nearest even (finite inputs)
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return u >> 16;
}
__device__ inline float bf2f(uint32_t h) { return __uint_as_float(h << 16); }

// one-hot of 8 symbols against k: BF16 1.0 (0x3f80) where sigma == k, else 0
__device__ inline bf16x8 onehot8(uint2 s8, uint32_t kk) {
  uint32_t w[2] = {s8.x, s8.y}, r[4];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const uint32_t x = w[h] ^ kk;                                    // zero byte where equal
    const uint32_t nz = ((x & 0x7f7f7f7fu) + 0x7f7f7f7fu) | x;       // bit 7 set where not equal
    const uint32_t m = (nz & 0x80808080u) ^ 0x80808080u;             // 0x80 where equal
    // bytes (m0, 0, m1, 0) and (m2, 0, m3, 0), times 0x7f: 0x80 * 0x7f = 0x3f80
    r[2 * h] = __builtin_amdgcn_perm(0u, m, 0x0c010c00u) * 0x7fu;
    r[2 * h + 1] = __builtin_amdgcn_perm(0u, m, 0x0c030c02u) * 0x7fu;
  }
  uint4 v = make_uint4(r[0], r[1], r[2], r[3]);
  return __builtin_bit_cast(bf16x8, v);
}

template <int NP>
__global__ __launch_bounds__(kMThreads) void bwd_mfma_kernel(EvalArgs a) {
  // B fragments of the residual pieces: [piece][step][half][column][8 rows]
  __shared__ __attribute__((aligned(16))) uint16_t Bf[NP * kMSteps * 2 * 32 * 8];
  __shared__ __attribute__((aligned(16))) uint8_t sig[kMPos * kMChunk];  // [column][row] symbols
  const int idx = blockIdx.x;  // sites fastest
  const int nact = a.n_active ? *a.n_active : a.n_active_host;
  if (idx >= nact) return;
  const int r = a.sites ? a.sites[idx] : idx;
  const int q = a.q, N = a.N, qq = q * q;
  const int i0 = blockIdx.y * kMPos;
  const int npos = min(kMPos, N - i0);
  const int nrows = npos * q;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int half = lane >> 5, l32 = lane & 31;

  // this lane's A-fragment row in each of its row blocks
  int arow_col[kMRowBlocks];
  uint32_t arow_kk[kMRowBlocks];
  bool arow_ok[kMRowBlocks];
#pragma unroll
  for (int m = 0; m < kMRowBlocks; ++m) {
    const int rho = (wid * kMRowBlocks + m) * 32 + l32;
    arow_ok[m] = rho < nrows;
    const int rr = arow_ok[m] ? rho : 0;
    arow_col[m] = rr / q;
    arow_kk[m] = (uint32_t)(rr % q) * 0x01010101u;
  }
  const bool wave_live = wid * kMRowBlocks * 32 < nrows;

  for (int e = tid; e < NP * kMSteps * 2 * 32 * 8; e += kMThreads) Bf[e] = 0;
  floatx16 acc[kMRowBlocks];
  double acc64[kMRowBlocks][16];
#pragma unroll
  for (int m = 0; m < kMRowBlocks; ++m)
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      acc[m][j] = 0.f;
      acc64[m][j] = 0.0;
    }

  const float* Rr = a.R + (size_t)r * a.B3 * kSlot;
  const int nchunks = (a.B3 + kMChunk - 1) / kMChunk;
  const int c16_0 = i0 / kFwdChunk, nc16 = a.N_pad / kFwdChunk;
  for (int c = 0; c < nchunks; ++c) {
    const int bc = c * kMChunk, n = min(kMChunk, a.B3 - bc);
    __syncthreads();
    // residual pieces, transposed into the B-fragment layout (columns >= 21 stay zero)
    for (int e = tid; e < kMChunk * kSlot; e += kMThreads) {
      const int b = e / kSlot, s = e - b * kSlot;
      const float v = b < n ? Rr[(size_t)(bc + b) * kSlot + s] : 0.f;
      const int off = (((b >> 4) * 2 + ((b >> 3) & 1)) * 32 + s) * 8 + (b & 7);
      uint32_t hi = f2bf(v);
      Bf[off] = (uint16_t)hi;
      float rem = v - bf2f(hi);
#pragma unroll
      for (int p = 1; p < NP; ++p) {
        const uint32_t pc = f2bf(rem);
        Bf[p * (kMSteps * 2 * 32 * 8) + off] = (uint16_t)pc;
        rem -= bf2f(pc);
      }
    }
    // symbols of the block's columns, transposed to [column][row]
    for (int e = tid; e < kMChunk * 3; e += kMThreads) {
      const int b = e / 3, g = e - b * 3, c16 = c16_0 + g;
      uint4 v = make_uint4(0, 0, 0, 0);
      if (b < n && c16 < nc16) v = *reinterpret_cast<const uint4*>(a.msa_cm + ((size_t)c16 * a.B_pad + bc + b) * kFwdChunk);
      const uint32_t wv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int p = 0; p < 16; ++p) sig[(g * 16 + p) * kMChunk + b] = (uint8_t)(wv[p >> 2] >> (8 * (p & 3)));
    }
    __syncthreads();
    if (wave_live) {
#pragma unroll 2
      for (int t = 0; t < kMSteps; ++t) {
        bf16x8 bp[NP];
#pragma unroll
        for (int p = 0; p < NP; ++p)
          bp[p] = *reinterpret_cast<const bf16x8*>(
              &Bf[p * (kMSteps * 2 * 32 * 8) + ((t * 2 + half) * 32 + l32) * 8]);
        bf16x8 av[kMRowBlocks];
#pragma unroll
        for (int m = 0; m < kMRowBlocks; ++m) {
          const uint2 s8 = *reinterpret_cast<const uint2*>(&sig[arow_col[m] * kMChunk + t * 16 + half * 8]);
          av[m] = onehot8(s8, arow_kk[m]);
          if (!arow_ok[m]) av[m] = __builtin_bit_cast(bf16x8, make_uint4(0, 0, 0, 0));
        }
        // the row blocks are independent accumulation chains
#pragma unroll
        for (int p = 0; p < NP; ++p)
#pragma unroll
          for (int m = 0; m < kMRowBlocks; ++m)
            acc[m] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[m], bp[p], acc[m], 0, 0, 0);
      }
#pragma unroll
      for (int m = 0; m < kMRowBlocks; ++m)
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          acc64[m][j] += (double)acc[m][j];
          acc[m][j] = 0.f;
        }
    }
  }
  if (!wave_live) return;
#pragma unroll
  for (int m = 0; m < kMRowBlocks; ++m)
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int row = (wid * kMRowBlocks + m) * 32 + 8 * (j >> 2) + 4 * half + (j & 3);
      if (row < nrows && l32 < q) {
        const int i = i0 + row / q, k = row % q;
        a.gJ[((size_t)r * N + i) * qq + (size_t)k * q + l32] = (i == r) ? 0.0 : acc64[m][j];
      }
    }
}

hipError_t launch_backward_mfma(const EvalArgs& a, int32_t n_sites_grid, int32_t npieces,
                                hipStream_t st) {
  dim3 grid(n_sites_grid, (a.N + kMPos - 1) / kMPos);
  if (npieces == 3)
    hipLaunchKernelGGL(bwd_mfma_kernel<3>, grid, dim3(kMThreads), 0, st, a);
  else if (npieces == 2)
    hipLaunchKernelGGL(bwd_mfma_kernel<2>, grid, dim3(kMThreads), 0, st, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace plm
