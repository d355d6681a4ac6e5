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
// One block = one site x up to 768 rows (i,k) (36 columns at q = 21), all
// sequences, in 256-sequence chunks.  A chunk's residual pieces and symbols are
// staged in LDS (double-buffered); the global loads of chunk c+2 are issued
// before the matrix work on chunk c so that their latency is hidden.  Blocks
// are ordered so that the column blocks of one site run on one XCD and share
// its L2 copy of R_r.
//
// Fragment layouts of v_mfma_f32_32x32x16_bf16 (verified on the device): A
// lane l holds row l % 32, inner indices 8 (l / 32) + 0..7; B lane l holds
// column l % 32, the same inner indices; D lane l register j holds row
// 8 (j / 4) + 4 (l / 32) + j % 4, column l % 32.
#include <type_traits>

#include "plm_internal.h"

namespace plm {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

// FP16 pieces of the residuals are taken of R * 2^12 (|R| <= 1, so no
// overflow, and the low piece stays clear of the FP16 subnormal range); the
// FP64 sums are scaled back by 2^-12, exactly.
constexpr float kF16Scale = 4096.f;
constexpr double kF16Unscale = 1.0 / 4096.0;

constexpr int kMWaves = 8;
constexpr int kMThreads = kMWaves * 64;
constexpr int kMRB = 3;                          // 32-row blocks per wave
constexpr int kMRows = kMWaves * kMRB * 32;      // 768 rows (i,k) per block
constexpr int kMPosMax = 48;                     // alignment columns per block at most
constexpr int kMChunk = 256;                     // sequences per staged chunk
constexpr int kMSteps = kMChunk / 16;            // MFMA steps per chunk
constexpr int kSigPitch = kMChunk + 16;          // LDS bytes per column (padding spreads banks)
constexpr int kBfPiece = kMSteps * 2 * 32 * 8;   // BF16 entries of one piece of one chunk
constexpr int kRUnits = (kMChunk / 8) * kSlot;   // (8-sequence group, state) units per chunk

__host__ __device__ inline int32_t mfma_block_positions(int32_t q) {
  return kMRows / q < kMPosMax ? kMRows / q : kMPosMax;
}

__device__ inline uint32_t f2bf(float f) {  // round to nearest even (finite inputs)
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return u >> 16;
}
__device__ inline float bf2f(uint32_t h) { return __uint_as_float(h << 16); }

// One-hot of 8 symbols against k as eight 16-bit words: 2.0 where sigma == k,
// else 0 (0x4000 is 2.0 in both BF16 and FP16; the factor 2 is removed,
// exactly, when the sums are written).  Symbols and k are below 32, so the
// bytes of x = sigma ^ k are below 32 and x + 0x3f never carries out of a
// byte: bit 6 of a byte of x + 0x3f3f3f3f is clear exactly where sigma == k.
// Rows past the end use k = 31, which no symbol (< q <= 21) equals.
__device__ inline uint4 onehot8_x2(uint2 s8, uint32_t kk) {
  uint32_t w[2] = {s8.x, s8.y}, r[4];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const uint32_t nz = (w[h] ^ kk) + 0x3f3f3f3fu;
    const uint32_t m = ~nz & 0x40404040u;  // 0x40 in the bytes where sigma == k
    // bytes (0, m0, 0, m1) and (0, m2, 0, m3): words 0x4000 or 0
    r[2 * h] = __builtin_amdgcn_perm(0u, m, 0x010c000cu);
    r[2 * h + 1] = __builtin_amdgcn_perm(0u, m, 0x030c020cu);
  }
  return make_uint4(r[0], r[1], r[2], r[3]);
}

constexpr double kOneHotUnscale = 0.5;  // the one-hot value is 2

// Position-major copy of the padded alignment: msaT[i * B_pad + b].
__global__ void transpose_msa_kernel(const uint8_t* __restrict__ msa_cm, int32_t B_pad,
                                     int32_t N_pad, uint8_t* __restrict__ msaT) {
  const size_t groups = (size_t)B_pad / 16;
  const size_t total = (size_t)N_pad * groups;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int32_t i = (int32_t)(e / groups);
    const size_t b0 = (e - (size_t)i * groups) * 16;
    const uint8_t* src = msa_cm + ((size_t)(i / kFwdChunk) * B_pad + b0) * kFwdChunk + i % kFwdChunk;
    uint32_t w[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      w[t] = (uint32_t)src[(4 * t) * kFwdChunk] | ((uint32_t)src[(4 * t + 1) * kFwdChunk] << 8) |
             ((uint32_t)src[(4 * t + 2) * kFwdChunk] << 16) |
             ((uint32_t)src[(4 * t + 3) * kFwdChunk] << 24);
    }
    *reinterpret_cast<uint4*>(msaT + (size_t)i * B_pad + b0) = make_uint4(w[0], w[1], w[2], w[3]);
  }
}

hipError_t launch_transpose_msa(const uint8_t* msa_cm, int32_t B_pad, int32_t N_pad, uint8_t* msaT,
                                hipStream_t st) {
  const size_t total = (size_t)N_pad * (B_pad / 16);
  int blocks = (int)((total + 255) / 256);
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(transpose_msa_kernel, dim3(blocks), dim3(256), 0, st, msa_cm, B_pad, N_pad,
                     msaT);
  return hipGetLastError();
}

// One backward work item: site r x column block cb.  Bf: B fragments of the
// residual pieces, [buffer][piece][step][half][column][8 sequences]; sig:
// symbols of the block's columns, [buffer][column][sequence].
// F16: FP16 hi/lo pieces of R * 2^12 (v_mfma_f32_32x32x16_f16) instead of
// BF16 pieces (v_mfma_f32_32x32x16_bf16).
template <int NP, bool F16>
__device__ inline void bwd_mfma_item(const EvalArgs& a, int r, int cb, uint16_t (*Bf)[NP * kBfPiece],
                                     uint8_t (*sig)[kMPosMax * kSigPitch]) {
  const int npos_blk = mfma_block_positions(a.q);
  const int q = a.q, N = a.N, qq = q * q;
  const int i0 = cb * npos_blk;
  const int npos = min(npos_blk, N - i0);
  const int nrows = npos * q;
  const int tid = item_tid(), lane = tid & 63, wid = tid >> 6;
  const int half = lane >> 5, l32 = lane & 31;

  // this lane's A-fragment row in each of its row blocks; rows past the end
  // compare against 31, which no symbol equals, so their one-hot is zero
  int arow_off[kMRB];
  uint32_t arow_kk[kMRB];
#pragma unroll
  for (int m = 0; m < kMRB; ++m) {
    const int rho = (wid * kMRB + m) * 32 + l32;
    const bool ok = rho < nrows;
    arow_off[m] = ok ? (rho / q) * kSigPitch : 0;
    arow_kk[m] = (ok ? (uint32_t)(rho % q) : 31u) * 0x01010101u;
  }
  const bool wave_live = wid * kMRB * 32 < nrows;

  for (int e = tid; e < 2 * NP * kBfPiece / 8; e += kMThreads)
    reinterpret_cast<uint4*>(&Bf[0][0])[e] = make_uint4(0, 0, 0, 0);

  const auto Rr = gmem(a.R + (size_t)r * a.B3 * kSlot);
  const int nchunks = (a.B3 + kMChunk - 1) / kMChunk;
  const int nsig = npos_blk * (kMChunk / 16);

  float rv[2][8];
  uint4 sv[2];
  auto load = [&](int c) {
    const int bc = c * kMChunk;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int u = tid + k * kMThreads;
      const int g = u / kSlot, s = u - g * kSlot;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int row = bc + g * 8 + j;
        rv[k][j] = (u < kRUnits && row < a.B3) ? Rr[(size_t)row * kSlot + s] : 0.f;
      }
      const int e = tid + k * kMThreads;
      const int pos = e >> 4, part = e & 15;
      sv[k] = make_uint4(0, 0, 0, 0);
      if (e < nsig && i0 + pos < N)
        sv[k] = gload_u4(a.msaT + (size_t)(i0 + pos) * a.B_pad + bc + part * 16);
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int u = tid + k * kMThreads;
      if (u < kRUnits) {
        const int g = u / kSlot, s = u - g * kSlot;
        uint32_t hw[NP][4];
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
          float v0 = rv[k][2 * jj], v1 = rv[k][2 * jj + 1];
          if (F16) {
            v0 *= kF16Scale;
            v1 *= kF16Scale;
          }
#pragma unroll
          for (int p = 0; p < NP; ++p) {
            if (F16) {
              const _Float16 h0 = (_Float16)v0, h1 = (_Float16)v1;
              hw[p][jj] = (uint32_t)__builtin_bit_cast(uint16_t, h0) |
                          ((uint32_t)__builtin_bit_cast(uint16_t, h1) << 16);
              v0 -= (float)h0;
              v1 -= (float)h1;
            } else {
              const uint32_t h0 = f2bf(v0), h1 = f2bf(v1);
              hw[p][jj] = h0 | (h1 << 16);
              v0 -= bf2f(h0);
              v1 -= bf2f(h1);
            }
          }
        }
#pragma unroll
        for (int p = 0; p < NP; ++p)
          *reinterpret_cast<uint4*>(&Bf[buf][p * kBfPiece + (g * 32 + s) * 8]) =
              make_uint4(hw[p][0], hw[p][1], hw[p][2], hw[p][3]);
      }
      const int e = tid + k * kMThreads;
      if (e < nsig)
        *reinterpret_cast<uint4*>(&sig[buf][(e >> 4) * kSigPitch + (e & 15) * 16]) = sv[k];
    }
  };

  floatx16 acc[kMRB];
  double acc64[kMRB][16];
#pragma unroll
  for (int m = 0; m < kMRB; ++m)
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      acc[m][j] = 0.f;
      acc64[m][j] = 0.0;
    }

  load(0);
  __syncthreads();  // zero fill of the unused fragment columns is complete
  store(0);
  if (nchunks > 1) load(1);
  __syncthreads();
  for (int c = 0; c < nchunks; ++c) {
    const int buf = c & 1;
    if (wave_live) {
      const uint16_t* bfb = &Bf[buf][((half * 32) + l32) * 8];
      const uint8_t* sgb = &sig[buf][half * 8];
#pragma unroll 2
      for (int t = 0; t < kMSteps; ++t) {
        uint4 bp[NP];
#pragma unroll
        for (int p = 0; p < NP; ++p)
          bp[p] = *reinterpret_cast<const uint4*>(bfb + p * kBfPiece + t * (2 * 32 * 8));
        uint4 av[kMRB];
#pragma unroll
        for (int m = 0; m < kMRB; ++m)
          av[m] = onehot8_x2(*reinterpret_cast<const uint2*>(sgb + arow_off[m] + t * 16), arow_kk[m]);
        // the row blocks are independent accumulation chains
#pragma unroll
        for (int p = 0; p < NP; ++p)
#pragma unroll
          for (int m = 0; m < kMRB; ++m) {
            if (F16)
              acc[m] = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, av[m]),
                                                              __builtin_bit_cast(f16x8, bp[p]), acc[m], 0, 0, 0);
            else
              acc[m] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, av[m]),
                                                               __builtin_bit_cast(bf16x8, bp[p]), acc[m], 0, 0, 0);
          }
      }
#pragma unroll
      for (int m = 0; m < kMRB; ++m)
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          acc64[m][j] += (double)acc[m][j];
          acc[m][j] = 0.f;
        }
    }
    // the other buffer was last read before the previous barrier
    if (c + 1 < nchunks) store(buf ^ 1);
    if (c + 2 < nchunks) load(c + 2);
    __syncthreads();
  }
  if (!wave_live) return;
#pragma unroll
  for (int m = 0; m < kMRB; ++m)
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int row = (wid * kMRB + m) * 32 + 8 * (j >> 2) + 4 * half + (j & 3);
      if (row < nrows && l32 < q) {
        const int i = i0 + row / q, k = row % q;
        gmem_w(a.gJ)[((size_t)r * N + i) * qq + (size_t)k * q + l32] =
            (i == r) ? 0.0 : acc64[m][j] * (F16 ? kF16Unscale * kOneHotUnscale : kOneHotUnscale);
      }
    }
}

// ---------------------------------------------------------------- forward
// E_b(s) = h_r(s) + sum_i J_ri(s, sigma_i^b) (eq. condpfinal) as the product
// of the one-hot X[b][(i,k)] with W_r[(i,k)][s] = J_ri(s,k) (i != r), the
// couplings split into NP BF16 pieces.  One block = one site x 1024 sequences
// (8 waves x 4 row blocks of 32); the inner index runs over eight alignment
// columns per staged chunk, ordered (k-range, column, k within the range) with
// q padded to 24, so that all lanes of a step test the same k-range.  The
// log-sum-exp, objective term, residual R_b(s) and the h-gradient partials
// follow in the epilogue, in the same output buffers as the gather forward.
constexpr int kFRB = 4;                            // row blocks per wave
constexpr int kFRows = kMWaves * kFRB * 32;        // 1024 sequences per block
constexpr int kFPos = 8;                           // alignment columns per chunk
constexpr int kFGroups = kFPos * 3;                // 8-wide inner-index groups per chunk
constexpr int kFSteps = kFGroups / 2;              // 12 MFMA steps per chunk
constexpr int kFPiece = kFGroups * 32 * 8;         // BF16 entries of one piece of one chunk

int32_t mfma_forward_tile_seqs() { return kFRows; }
static_assert(kBPadUnit % kFRows == 0, "row padding covers the MFMA forward tiles");

// one-hot of sigma against the eight states kb..kb+7 (d = sigma - kb, unsigned)
__device__ inline bf16x8 onehot_range(uint32_t d) {
  const uint32_t v = (d & 1u) ? 0x3f800000u : 0x00003f80u;
  const uint32_t w = d >> 1;
  uint4 r = make_uint4(w == 0 ? v : 0u, w == 1 ? v : 0u, w == 2 ? v : 0u, w == 3 ? v : 0u);
  return __builtin_bit_cast(bf16x8, r);
}

// One forward work item: site r x sequence tile `tile`.  Wf: W fragments,
// [buffer][piece][group][column s][8 inner indices]; sgl: the tile's symbols
// for the chunk's eight columns, [buffer][sequence][column].
template <int NP>
__device__ inline void fwd_mfma_item(const EvalArgs& a, int r, int tile, uint16_t (*Wf)[NP * kFPiece],
                                     uint8_t (*sgl)[kFRows * kFPos], double* red) {
  const int q = a.q, N = a.N, qq = q * q;
  const int tid = item_tid(), lane = tid & 63, wid = tid >> 6;
  const int half = lane >> 5, l32 = lane & 31;
  const int tile0 = tile * kFRows;

  for (int e = tid; e < 2 * NP * kFPiece / 8; e += kMThreads)
    reinterpret_cast<uint4*>(&Wf[0][0])[e] = make_uint4(0, 0, 0, 0);

  const auto Jr = gmem(a.J + (size_t)r * N * qq);
  const auto msa_cm = gmem(a.msa_cm);
  const int nunits = kFGroups * q;  // (group, state) units, at most 504
  const int nchunks = (N + kFPos - 1) / kFPos;
  float wv[8];
  uint2 sv[2];
  auto load = [&](int c) {
    const int i0 = c * kFPos;
    const int u = tid;
    const int g = u / q, s = u - g * q;
    const int kg = g / kFPos, i = i0 + (g - kg * kFPos);
    const bool uok = u < nunits && i < N && i != r;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int k = kg * 8 + j;
      wv[j] = (uok && k < q) ? Jr[((size_t)i * q + k) * q + s] : 0.f;
    }
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int row = tid + t * kMThreads;
      sv[t] = gload_u2(a.msa_cm + ((size_t)(i0 / kFwdChunk) * a.B_pad + tile0 + row) * kFwdChunk +
                       (i0 % kFwdChunk));
    }
  };
  auto store = [&](int buf) {
    if (tid < nunits) {
      const int g = tid / q, s = tid - g * q;
      uint32_t hw[NP][4];
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        float v0 = wv[2 * jj], v1 = wv[2 * jj + 1];
#pragma unroll
        for (int p = 0; p < NP; ++p) {
          const uint32_t h0 = f2bf(v0), h1 = f2bf(v1);
          hw[p][jj] = h0 | (h1 << 16);
          v0 -= bf2f(h0);
          v1 -= bf2f(h1);
        }
      }
#pragma unroll
      for (int p = 0; p < NP; ++p)
        *reinterpret_cast<uint4*>(&Wf[buf][p * kFPiece + (g * 32 + s) * 8]) =
            make_uint4(hw[p][0], hw[p][1], hw[p][2], hw[p][3]);
    }
#pragma unroll
    for (int t = 0; t < 2; ++t)
      *reinterpret_cast<uint2*>(&sgl[buf][(tid + t * kMThreads) * kFPos]) = sv[t];
  };

  floatx16 acc[kFRB];
#pragma unroll
  for (int m = 0; m < kFRB; ++m)
#pragma unroll
    for (int j = 0; j < 16; ++j) acc[m][j] = 0.f;

  load(0);
  __syncthreads();
  store(0);
  if (nchunks > 1) load(1);
  __syncthreads();
  for (int c = 0; c < nchunks; ++c) {
    const int buf = c & 1;
    // this lane's eight symbols per row block; odd lanes-halves take the odd columns
    uint32_t sym[kFRB][2];
#pragma unroll
    for (int m = 0; m < kFRB; ++m) {
      const uint2 s8 = *reinterpret_cast<const uint2*>(&sgl[buf][((wid * kFRB + m) * 32 + l32) * kFPos]);
      const uint64_t v = ((uint64_t)s8.y << 32 | s8.x) >> (8 * half);
      sym[m][0] = (uint32_t)v;
      sym[m][1] = (uint32_t)(v >> 32);
    }
    const uint16_t* wfb = &Wf[buf][(half * 32 + l32) * 8];
#pragma unroll
    for (int t = 0; t < kFSteps; ++t) {
      // group 2t + half = (k-range t / 4, column 2 (t % 4) + half)
      const int kb = (t / 4) * 8;
      const int sh = 16 * (t % 4);
      bf16x8 bp[NP];
#pragma unroll
      for (int p = 0; p < NP; ++p)
        bp[p] = *reinterpret_cast<const bf16x8*>(wfb + p * kFPiece + t * (2 * 32 * 8));
      bf16x8 av[kFRB];
#pragma unroll
      for (int m = 0; m < kFRB; ++m) {
        const uint32_t sg = (sh < 32 ? sym[m][0] >> sh : sym[m][1] >> (sh - 32)) & 0xffu;
        av[m] = onehot_range(sg - (uint32_t)kb);
      }
#pragma unroll
      for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int m = 0; m < kFRB; ++m)
          acc[m] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[m], bp[p], acc[m], 0, 0, 0);
    }
    if (c + 1 < nchunks) store(buf ^ 1);
    if (c + 2 < nchunks) load(c + 2);
    __syncthreads();
  }

  // epilogue: rows of D are sequences, columns (lanes of a 32-lane half) states
  const bool col_ok = l32 < q;
  const float hv = col_ok ? a.h[r * q + l32] : 0.f;
  double facc = 0.0, ghacc = 0.0;
#pragma unroll
  for (int m = 0; m < kFRB; ++m)
#pragma unroll 4
    for (int j = 0; j < 16; ++j) {
      const int b = tile0 + (wid * kFRB + m) * 32 + 8 * (j >> 2) + 4 * half + (j & 3);
      const float e = col_ok ? acc[m][j] + hv : -INFINITY;
      float mx = e;
#pragma unroll
      for (int d = 16; d > 0; d >>= 1) mx = fmaxf(mx, __shfl_xor(mx, d, 32));
      const float ex = col_ok ? expf(e - mx) : 0.f;
      float sum = ex;
#pragma unroll
      for (int d = 16; d > 0; d >>= 1) sum += __shfl_xor(sum, d, 32);
      const float lse = mx + logf(sum);
      const int sr = msa_cm[((size_t)(r / kFwdChunk) * a.B_pad + b) * kFwdChunk + r % kFwdChunk];
      const double wb = b < a.B ? gmem(a.w)[b] : 0.0;
      const float P = ex / sum;
      const float Rv = col_ok ? (float)wb * (P - (l32 == sr ? 1.f : 0.f)) : 0.f;
      if (col_ok && l32 == sr) facc += wb * (double)(lse - e);
      ghacc += (double)Rv;
      if (col_ok && b < a.B3) gmem_w(a.R)[((size_t)r * a.B3 + b) * kSlot + l32] = Rv;
    }
  const double ftot = block_sum_f64(facc, red);
  if (tid == 0) a.f_part[(size_t)tile * N + r] = ftot;
  ghacc += __shfl_xor(ghacc, 32, 64);
  if (half == 0) red[wid * 32 + l32] = ghacc;
  __syncthreads();
  if (tid < q) {
    double t = 0.0;
    for (int w = 0; w < kMWaves; ++w) t += red[w * 32 + tid];
    a.gh_part[((size_t)tile * N + r) * kSlot + tid] = t;
  }
}

template <int NP>
__global__ __launch_bounds__(kMThreads) void fwd_mfma_kernel(BatchArgs b) {
  __shared__ __attribute__((aligned(16))) uint16_t Wf[2][NP * kFPiece];
  __shared__ __attribute__((aligned(16))) uint8_t sgl[2][kFRows * kFPos];
  __shared__ double red[kMWaves * 64];
  __shared__ int32_t item_s;
  int32_t qi = 0;
  const int32_t total = total_items(b, KIND_FWD);
  for (;;) {
    if (threadIdx.x == 0) item_s = next_item(b.ctr + KIND_FWD * kQueues, total, qi);
    __syncthreads();
    const int32_t t = __builtin_amdgcn_readfirstlane(item_s);
    if (t < 0) break;
    const Item it = decode_item(b, KIND_FWD, t);
    const EvalArgs a = load_uniform(b.ev + it.m);
    fwd_mfma_item<NP>(a, it.r, it.sub, Wf, sgl, red);
    __syncthreads();
  }
}

hipError_t launch_forward_mfma(const BatchArgs& b, int32_t npieces, int32_t nblocks, hipStream_t st) {
  if (npieces == 3)
    hipLaunchKernelGGL(fwd_mfma_kernel<3>, dim3(nblocks), dim3(kMThreads), 0, st, b);
  else if (npieces == 2)
    hipLaunchKernelGGL(fwd_mfma_kernel<2>, dim3(nblocks), dim3(kMThreads), 0, st, b);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}


template <int NP, bool F16>
__global__ __launch_bounds__(kMThreads) void bwd_mfma_kernel(BatchArgs b) {
  __shared__ __attribute__((aligned(16))) uint16_t Bf[2][NP * kBfPiece];
  __shared__ __attribute__((aligned(16))) uint8_t sig[2][kMPosMax * kSigPitch];
  __shared__ int32_t item_s;
  int32_t qi = 0;
  const int32_t total = total_items(b, KIND_BWD);
  for (;;) {
    if (threadIdx.x == 0) item_s = next_item(b.ctr + KIND_BWD * kQueues, total, qi);
    __syncthreads();
    const int32_t t = __builtin_amdgcn_readfirstlane(item_s);
    if (t < 0) break;
    const Item it = decode_item(b, KIND_BWD, t);
    const EvalArgs a = load_uniform(b.ev + it.m);
    bwd_mfma_item<NP, F16>(a, it.r, it.sub, Bf, sig);
    __syncthreads();
  }
}

// ---------------------------------------------- grouped FP16 hi/lo gradient
// The gradient of three sites at once: X^T [R_r0 | R_r1 | R_r2], the 63
// residual columns of the group filling two 32-column MFMA tiles (the single-
// site product leaves 11 of its 32 columns empty), so every one-hot A
// fragment feeds four products (two tiles x two pieces).  The residuals come
// from the forward already split (FP16 hi/lo of R * 2^12, fragment order) and
// are copied global -> LDS by the load unit (buffer loads with an LDS
// destination, 16 bytes per lane, no registers, no conversion),
// double-buffered one 256-sequence chunk ahead.  One block =
// three sites x 512 rows (i, k) (24 columns at q = 21): 8 waves x 2 row blocks
// of 32 rows; FP32 accumulators folded into FP64 every chunk, as in the
// single-site kernel, so every output is summed in the same order.
constexpr int kGWaves = 8;
constexpr int kGThreads = kGWaves * 64;
constexpr int kGRB = 2;                          // 32-row blocks per wave
constexpr int kGT = 2;                           // 32-column tiles (63 residual columns)
constexpr int kGRows = kGWaves * kGRB * 32;      // 512
constexpr int kGPosMax = 32;                     // alignment columns per block at most
// LDS stride between the sites' chunks: 21504 + 80 bytes, so that the 16-byte
// slot (address / 16 mod 8) of column c is c mod 8 within every site's run
// and the B-fragment reads of any 8 consecutive lanes hit distinct banks
constexpr int kGSiteStride = kRfChunkBytes + 80;
static_assert((kGSiteStride / 16 - kSlot) % 8 == 0 && kGSiteStride % 16 == 0, "bank-disjoint site runs");
constexpr int kGBufWords = (2 * kGSiteStride + kRfChunkBytes) / 2;  // one chunk buffer in 16-bit words

__host__ __device__ inline int32_t g3_block_positions(int32_t q) {
  return kGRows / q < kGPosMax ? kGRows / q : kGPosMax;
}

// The two chunk buffers are separate LDS arrays so that the compiler can tell
// the copy into one from the reads of the other (otherwise it waits for the
// copy before every read).
__device__ inline void g3_item(const BatchArgs& bt, const EvalArgs& a, const Item& it, uint16_t* Rf0,
                               uint16_t* Rf1, uint8_t* sig0, uint8_t* sig1) {
  const int npos_blk = g3_block_positions(a.q);
  const int q = a.q, N = a.N, qq = q * q;
  const int i0 = it.sub * npos_blk;
  const int npos = min(npos_blk, N - i0);
  const int nrows = npos * q;
  const int tid = item_tid(), lane = tid & 63, wid = tid >> 6;
  const int half = lane >> 5, l32 = lane & 31;
  const int cnt = it.cnt;
  int32_t rs[kG3Sites];
#pragma unroll
  for (int g = 0; g < kG3Sites; ++g)
    rs[g] = g < cnt ? bt.active[it.first + g] - bt.site_base[it.m] : it.r;

  int arow_off[kGRB];
  uint32_t arow_kk[kGRB];
#pragma unroll
  for (int m = 0; m < kGRB; ++m) {
    const int rho = (wid * kGRB + m) * 32 + l32;
    const bool ok = rho < nrows;
    arow_off[m] = ok ? (rho / q) * kSigPitch : 0;
    arow_kk[m] = (ok ? (uint32_t)(rho % q) : 31u) * 0x01010101u;
  }
  const bool wave_live = wid * kGRB * 32 < nrows;
  // this lane's B-fragment column in each tile: residual column 32 T + l32 =
  // (site, state); column 63 reads a valid word of site 2 and is never written out
  uint32_t boff[kGT];
#pragma unroll
  for (int T = 0; T < kGT; ++T) {
    const int col = min(32 * T + l32, 3 * kSlot - 1);
    const int g = col / kSlot, sidx = col - g * kSlot;
    boff[T] = (uint32_t)(g * kGSiteStride + half * (kSlot * 16) + sidx * 16);
  }

  const int nchunks = (a.B3 + kMChunk - 1) / kMChunk;
  const int nch_site = a.B_pad >> 8;
  const int nsig = npos_blk * (kMChunk / 16);
  // global -> LDS copy of the group's residual chunk c: 21 x 1 KB per site
  auto fetch_r = [&](int c, uint16_t* dst) {
    const int ninst = cnt * (kRfChunkBytes / 1024);
    for (int k = wid; k < ninst; k += kGWaves) {
      const int g = k / (kRfChunkBytes / 1024), part = k - g * (kRfChunkBytes / 1024);
      const int rg = g == 0 ? rs[0] : (g == 1 ? rs[1] : rs[2]);
      const char* src = reinterpret_cast<const char*>(a.R) + ((size_t)rg * nch_site + c) * kRfChunkBytes + part * 1024;
      copy16_to_lds(src, reinterpret_cast<char*>(dst) + g * kGSiteStride + part * 1024, lane);
    }
  };
  uint4 sv;
  auto load_sig = [&](int c) {
    const int bc = c * kMChunk;
    const int pos = tid >> 4, part = tid & 15;
    sv = make_uint4(0, 0, 0, 0);
    if (tid < nsig && i0 + pos < N) sv = gload_u4(a.msaT + (size_t)(i0 + pos) * a.B_pad + bc + part * 16);
  };
  auto store_sig = [&](uint8_t* dst) {
    if (tid < nsig) *reinterpret_cast<uint4*>(dst + (tid >> 4) * kSigPitch + (tid & 15) * 16) = sv;
  };

  floatx16 acc[kGRB][kGT];
  double acc64[kGRB][kGT][16];
#pragma unroll
  for (int m = 0; m < kGRB; ++m)
#pragma unroll
    for (int T = 0; T < kGT; ++T)
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        acc[m][T][j] = 0.f;
        acc64[m][T][j] = 0.0;
      }

  // chunk c from (cur, scur) while chunk c + 1 is copied into (nxt, snxt)
  auto chunk = [&](int c, const uint16_t* cur, uint16_t* nxt, const uint8_t* scur, uint8_t* snxt) {
    // the next buffers were last read before the previous barrier
    if (c + 1 < nchunks) {
      fetch_r(c + 1, nxt);
      store_sig(snxt);
    }
    if (c + 2 < nchunks) load_sig(c + 2);
    if (wave_live) {
      const char* rb = reinterpret_cast<const char*>(cur);
      const uint8_t* sgb = scur + half * 8;
      // one MFMA step; the first of a chunk starts its accumulators at zero
      auto step = [&](int t, auto first) {
        uint4 av[kGRB];
#pragma unroll
        for (int m = 0; m < kGRB; ++m)
          av[m] = onehot8_x2(*reinterpret_cast<const uint2*>(sgb + arow_off[m] + t * 16), arow_kk[m]);
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
          for (int T = 0; T < kGT; ++T) {
            const uint4 bp = *reinterpret_cast<const uint4*>(rb + boff[T] + (p * 16 + t) * (2 * kSlot * 16));
#pragma unroll
            for (int m = 0; m < kGRB; ++m) {
              floatx16 c = acc[m][T];
              if constexpr (decltype(first)::value) {
                if (p == 0) c = floatx16{};
              }
              acc[m][T] = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, av[m]),
                                                                 __builtin_bit_cast(f16x8, bp), c, 0, 0, 0);
            }
          }
      };
      step(0, std::true_type{});
#pragma unroll 3
      for (int t = 1; t < kMSteps; ++t) step(t, std::false_type{});
#pragma unroll
      for (int m = 0; m < kGRB; ++m)
#pragma unroll
        for (int T = 0; T < kGT; ++T)
#pragma unroll
          for (int j = 0; j < 16; ++j) acc64[m][T][j] += (double)acc[m][T][j];
    }
    // this wave's copies of chunk c + 1 (and the symbols of c + 2) have landed
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
  };

  fetch_r(0, Rf0);
  load_sig(0);
  store_sig(sig0);
  if (nchunks > 1) load_sig(1);
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  for (int c = 0; c < nchunks; c += 2) {
    chunk(c, Rf0, Rf1, sig0, sig1);
    if (c + 1 < nchunks) chunk(c + 1, Rf1, Rf0, sig1, sig0);
  }
  if (!wave_live) return;
#pragma unroll
  for (int T = 0; T < kGT; ++T) {
    const int col = 32 * T + l32;
    const int g = col / kSlot, sidx = col - g * kSlot;
    if (g >= cnt || sidx >= q) continue;
    const int rg = g == 0 ? rs[0] : (g == 1 ? rs[1] : rs[2]);
#pragma unroll
    for (int m = 0; m < kGRB; ++m)
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int row = (wid * kGRB + m) * 32 + 8 * (j >> 2) + 4 * half + (j & 3);
        if (row < nrows) {
          const int i = i0 + row / q, k = row % q;
          gmem_w(a.gJ)[((size_t)rg * N + i) * qq + (size_t)k * q + sidx] =
              (i == rg) ? 0.0 : acc64[m][T][j] * ((double)(1.0f / kRfScale) * kOneHotUnscale);
        }
      }
  }
}

__global__ __launch_bounds__(kGThreads) void bwd_g3_kernel(BatchArgs b) {
  __shared__ __attribute__((aligned(16))) uint16_t Rf0[kGBufWords];
  __shared__ __attribute__((aligned(16))) uint16_t Rf1[kGBufWords];
  __shared__ __attribute__((aligned(16))) uint8_t sig0[kGPosMax * kSigPitch];
  __shared__ __attribute__((aligned(16))) uint8_t sig1[kGPosMax * kSigPitch];
  __shared__ int32_t item_s;
  int32_t qi = 0;
  const int32_t total = total_items(b, KIND_BWD);
  for (;;) {
    if (threadIdx.x == 0) item_s = next_item(b.ctr + KIND_BWD * kQueues, total, qi);
    __syncthreads();
    const int32_t t = __builtin_amdgcn_readfirstlane(item_s);
    if (t < 0) break;
    const Item it = decode_item(b, KIND_BWD, t);
    const EvalArgs a = load_uniform(b.ev + it.m);
    g3_item(b, a, it, Rf0, Rf1, sig0, sig1);
    __syncthreads();
  }
}

__global__ void rfrag_tail_zero_kernel(uint4* R, int32_t N, int32_t nch_site, int32_t c0, int32_t c1,
                                       int32_t chunk16) {
  const int64_t per = (int64_t)(c1 - c0) * chunk16;
  const int64_t total = per * N;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / per, k = e - r * per;
    R[(r * nch_site + c0) * chunk16 + k] = make_uint4(0, 0, 0, 0);
  }
}

hipError_t launch_rfrag_tail_zero(float* R, int32_t N, int32_t B, int32_t B3, int32_t B_pad, int32_t chunk_bytes,
                                  hipStream_t st) {
  const int32_t c0 = B >> 8, c1 = (B3 + 255) >> 8;
  if (c0 >= c1) return hipSuccess;
  const int32_t chunk16 = chunk_bytes / 16;
  const int64_t total = (int64_t)(c1 - c0) * chunk16 * N;
  const int blocks = (int)((total + 255) / 256 < 4096 ? (total + 255) / 256 : 4096);
  hipLaunchKernelGGL(rfrag_tail_zero_kernel, dim3(blocks), dim3(256), 0, st, reinterpret_cast<uint4*>(R), N,
                     B_pad >> 8, c0, c1, chunk16);
  return hipGetLastError();
}

int32_t g3_backward_blocks_per_site(int32_t N, int32_t q) {
  const int32_t p = g3_block_positions(q);
  return (N + p - 1) / p;
}

int32_t g3_resident_blocks() {
  int per = 0;
  const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, bwd_g3_kernel, kGThreads, 0);
  return (e == hipSuccess && per > 0) ? per : 1;
}

hipError_t launch_backward_g3(const BatchArgs& b, int32_t nblocks, hipStream_t st) {
  hipLaunchKernelGGL(bwd_g3_kernel, dim3(nblocks), dim3(kGThreads), 0, st, b);
  return hipGetLastError();
}

// ------------------------------------------ grouped int8 fixed-point gradient
// The grouped product of the three-site kernel above, with the residuals as
// three signed int8 digits of round(R * 2^22) (written by the forward) on
// v_mfma_i32_32x32x32_i8: the one-hot is the byte 1, every digit plane has its
// own int32 accumulators, and integer accumulation over all sequences is exact
// (|digit| <= 128, so the sums fit for up to 2^24 sequences), so there is no
// per-chunk fold; the digit sums are combined in FP64 once at the end.
// Operand layouts (verified on the device): A lane l holds row l % 32, inner
// indices 16 (l / 32) + 0..15; B lane l column l % 32, the same inner
// indices; D as for v_mfma_f32_32x32x16_f16.
typedef int32_t i32x4 __attribute__((ext_vector_type(4)));
typedef int32_t i32x16 __attribute__((ext_vector_type(16)));
constexpr int kISteps = kMChunk / 32;                 // MFMA steps per chunk
constexpr int kISiteStride = kRiChunkBytes + 80;      // bank-disjoint site runs, as above
static_assert((kISiteStride / 16 - kSlot) % 8 == 0 && kISiteStride % 16 == 0, "bank-disjoint site runs");
constexpr int kIBufBytes = 2 * kISiteStride + kRiChunkBytes;

// One-hot of 16 symbols against k as sixteen int8 values (1 where sigma == k):
// a byte of x = sigma ^ k is below 32, so x + 0x7f keeps bit 7 clear exactly
// where x == 0 and never carries out of the byte.
__device__ inline uint4 onehot16_i8(uint4 s16, uint32_t kk) {
  uint32_t w[4] = {s16.x, s16.y, s16.z, s16.w};
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    const uint32_t y = (w[h] ^ kk) + 0x7f7f7f7fu;
    w[h] = (~y & 0x80808080u) >> 7;
  }
  return make_uint4(w[0], w[1], w[2], w[3]);
}

// The same indicator scaled by -128 (byte 0x80 where the symbol equals the
// state), in two instructions per word: 0x80808080 - (s ^ k) taken bytewise
// (no byte of s ^ k exceeds 31, so no borrow crosses a byte) is written as
// (s ^ ~k) + 0x80808081, one xor-add, and its top bits are the indicator.
// The products then sum -128 times the digits, each term in [-2^14 + 2^7,
// 2^14]: exact in int32 while a row collects fewer than 2^31 / 2^14 = 2^17
// sequences (padded counts are multiples of 3072, so at most 129 024).
constexpr int kNegSeqMax = 1 << 17;
__device__ inline uint4 onehot16_neg(uint4 s16, uint32_t nkk) {
  uint32_t w[4] = {s16.x, s16.y, s16.z, s16.w};
#pragma unroll
  for (int h = 0; h < 4; ++h) w[h] = ((w[h] ^ nkk) + 0x80808081u) & 0x80808080u;
  return make_uint4(w[0], w[1], w[2], w[3]);
}

// LO = false: the residual digits of round(R * 2^22), written to the gradient
// data part; LO = true (second pass of the precise path): the digits of the
// remainder, round((R * 2^22 - v) * 2^22), added to it scaled by 2^-44.
// NEG: the one-hot operand holds -128 for a one (alignments of fewer than
// kNegSeqMax padded sequences), and the epilogue divides it out exactly.
template <bool LO, bool NEG>
__device__ inline void i8_item(const BatchArgs& bt, const EvalArgs& a, const Item& it, int8_t* Rb0, int8_t* Rb1,
                               uint8_t* sig0, uint8_t* sig1) {
  const int npos_blk = g3_block_positions(a.q);
  const int q = a.q, N = a.N, qq = q * q;
  const int i0 = it.sub * npos_blk;
  const int npos = min(npos_blk, N - i0);
  const int nrows = npos * q;
  const int tid = item_tid(), lane = tid & 63;
  const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform: copy bookkeeping in scalars
  const int half = lane >> 5, l32 = lane & 31;
  const int cnt = it.cnt;
  int32_t rs[kG3Sites];
#pragma unroll
  for (int g = 0; g < kG3Sites; ++g)
    rs[g] = __builtin_amdgcn_readfirstlane(g < cnt ? bt.active[it.first + g] - bt.site_base[it.m] : it.r);

  int arow_off[kGRB];
  uint32_t arow_kk[kGRB];
#pragma unroll
  for (int m = 0; m < kGRB; ++m) {
    const int rho = (wid * kGRB + m) * 32 + l32;
    const bool ok = rho < nrows;
    arow_off[m] = ok ? (rho / q) * kSigPitch : 0;
    arow_kk[m] = (ok ? (uint32_t)(rho % q) : 31u) * 0x01010101u;
    if (NEG) arow_kk[m] = ~arow_kk[m];
  }
  const bool wave_live = wid * kGRB * 32 < nrows;
  uint32_t boff[kGT];
#pragma unroll
  for (int T = 0; T < kGT; ++T) {
    const int col = min(32 * T + l32, 3 * kSlot - 1);
    const int g = col / kSlot, sidx = col - g * kSlot;
    boff[T] = (uint32_t)(g * kISiteStride + half * (kSlot * 16) + sidx * 16);
  }

  const int nchunks = (a.B3 + kMChunk - 1) / kMChunk;
  const int nch_site = a.B_pad >> 8;
  const int nsig = npos_blk * (kMChunk / 16);
  // a site's chunk is 15.75 KB: 16 wave copies of 1 KB, the last one moved
  // back to end at the chunk end (it re-copies 256 bytes with the same values);
  // the LDS destination of a copy is uniform over the wave
  // with three sites, each wave's six copies are set up once per item
  static_assert(kG3Sites * 16 == 6 * kGWaves, "six copies per wave for a full group");
  const char* rsrc[6];
  uint32_t rdst[6];
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    const int k = wid + kGWaves * j;
    const int g = k >> 4, part = k & 15;
    const int off = min(part * 1024, kRiChunkBytes - 1024);
    const int rg = g == 0 ? rs[0] : (g == 1 ? rs[1] : rs[2]);
    rsrc[j] = reinterpret_cast<const char*>(a.R) + (LO ? (size_t)N * nch_site * kRiChunkBytes : 0) +
              (size_t)rg * nch_site * kRiChunkBytes + off;
    rdst[j] = (uint32_t)(g * kISiteStride + off);
  }
  auto fetch_r = [&](int c, int8_t* dst) {
    if (cnt == kG3Sites) {
#pragma unroll
      for (int j = 0; j < 6; ++j)
        copy16_to_lds(rsrc[j] + (size_t)c * kRiChunkBytes, reinterpret_cast<char*>(dst) + rdst[j], lane);
      return;
    }
    const int ninst = cnt * 16;
    for (int k = wid; k < ninst; k += kGWaves) {
      const int g = k >> 4, part = k & 15;
      const int off = min(part * 1024, kRiChunkBytes - 1024);
      const int rg = g == 0 ? rs[0] : (g == 1 ? rs[1] : rs[2]);
      const char* src = reinterpret_cast<const char*>(a.R) + (LO ? (size_t)N * nch_site * kRiChunkBytes : 0) +
                        ((size_t)rg * nch_site + c) * kRiChunkBytes + off;
      copy16_to_lds(src, reinterpret_cast<char*>(dst) + g * kISiteStride + off, lane);
    }
  };
  uint4 sv;
  auto load_sig = [&](int c) {
    const int bc = c * kMChunk;
    const int pos = tid >> 4, part = tid & 15;
    sv = make_uint4(0, 0, 0, 0);
    if (tid < nsig && i0 + pos < N) sv = gload_u4(a.msaT + (size_t)(i0 + pos) * a.B_pad + bc + part * 16);
  };
  auto store_sig = [&](uint8_t* dst) {
    if (tid < nsig) *reinterpret_cast<uint4*>(dst + (tid >> 4) * kSigPitch + (tid & 15) * 16) = sv;
  };

  i32x16 acc[3][kGRB][kGT];
#pragma unroll
  for (int d = 0; d < 3; ++d)
#pragma unroll
    for (int m = 0; m < kGRB; ++m)
#pragma unroll
      for (int T = 0; T < kGT; ++T) acc[d][m][T] = i32x16{};

  auto chunk = [&](int c, const int8_t* cur, int8_t* nxt, const uint8_t* scur, uint8_t* snxt) {
    if (c + 1 < nchunks) {
      fetch_r(c + 1, nxt);
      store_sig(snxt);
    }
    if (c + 2 < nchunks) load_sig(c + 2);
    if (wave_live) {
      const char* rb = reinterpret_cast<const char*>(cur);
      const uint8_t* sgb = scur + half * 16;
      static_assert(kGRB == 2 && kGT == 2, "two row blocks, two column tiles");
      auto ldsym = [&](int m, int t) { return *reinterpret_cast<const uint4*>(sgb + arow_off[m] + t * 32); };
      auto onehot = [&](uint4 s16, int m) {
        return NEG ? onehot16_neg(s16, arow_kk[m]) : onehot16_i8(s16, arow_kk[m]);
      };
      // row block 0's symbols are read one step ahead
      uint4 s0 = ldsym(0, 0);
#pragma unroll 2
      for (int t = 0; t < kISteps; ++t) {
        // the symbols read ahead have arrived (lgkmcnt 0; vmcnt and expcnt at
        // their maxima, so the chunk copies stay in flight)
        __builtin_amdgcn_s_waitcnt(0xc07f);
        // the six B fragments (digit, tile) of this step, each read two ahead of its use
        auto ldb = [&](int f) {
          return *reinterpret_cast<const uint4*>(rb + boff[f & 1] + ((f >> 1) * kISteps + t) * (2 * kSlot * 16));
        };
        auto prod = [&](int f, int m, const uint4& av, const uint4& bq) {
          acc[f >> 1][m][f & 1] = __builtin_amdgcn_mfma_i32_32x32x32_i8(
              __builtin_bit_cast(i32x4, av), __builtin_bit_cast(i32x4, bq), acc[f >> 1][m][f & 1], 0, 0, 0);
        };
        // issue order, fixed by scheduling fences: row block 1's symbols and the
        // first two B fragments; row block 0's one-hot operand and its first
        // product; the next symbols and the third fragment; row block 1's
        // one-hot operand; then each product pair followed by the read of the
        // fragment two ahead (an LDS wait then covers only the reads a product
        // needs)
        const uint4 s1 = ldsym(1, t);
        uint4 bq[6];
        bq[0] = ldb(0);
        bq[1] = ldb(1);
        __builtin_amdgcn_sched_barrier(0);
        const uint4 av0 = onehot(s0, 0);
        prod(0, 0, av0, bq[0]);
        __builtin_amdgcn_sched_barrier(0);
        s0 = ldsym(0, min(t + 1, kISteps - 1));
        bq[2] = ldb(2);
        __builtin_amdgcn_sched_barrier(0);
        const uint4 av1 = onehot(s1, 1);
        prod(0, 1, av1, bq[0]);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int f = 1; f < 6; ++f) {
          prod(f, 0, av0, bq[f]);
          prod(f, 1, av1, bq[f]);
          __builtin_amdgcn_sched_barrier(0);
          if (f + 2 < 6) bq[f + 2] = ldb(f + 2);
          __builtin_amdgcn_sched_barrier(0);
        }
      }
    }
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
  };

  fetch_r(0, Rb0);
  load_sig(0);
  store_sig(sig0);
  if (nchunks > 1) load_sig(1);
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  for (int c = 0; c < nchunks; c += 2) {
    chunk(c, Rb0, Rb1, sig0, sig1);
    if (c + 1 < nchunks) chunk(c + 1, Rb1, Rb0, sig1, sig0);
  }
  if (!wave_live) return;
  constexpr double kScale = (LO ? 1.0 / ((double)(1 << kRiScaleLog2) * (double)(1 << kRiScaleLog2))
                                : 1.0 / (double)(1 << kRiScaleLog2)) *
                           (NEG ? -1.0 / 128.0 : 1.0);
#pragma unroll
  for (int T = 0; T < kGT; ++T) {
    const int col = 32 * T + l32;
    const int g = col / kSlot, sidx = col - g * kSlot;
    if (g >= cnt || sidx >= q) continue;
    const int rg = g == 0 ? rs[0] : (g == 1 ? rs[1] : rs[2]);
#pragma unroll
    for (int m = 0; m < kGRB; ++m)
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int row = (wid * kGRB + m) * 32 + 8 * (j >> 2) + 4 * half + (j & 3);
        if (row < nrows) {
          const int i = i0 + row / q, k = row % q;
          // exact: every digit sum is an integer below 2^31
          const double v = (double)acc[0][m][T][j] * 65536.0 + (double)acc[1][m][T][j] * 256.0 +
                           (double)acc[2][m][T][j];
          auto out = gmem_w(a.gJ) + ((size_t)rg * N + i) * qq + (size_t)k * q + sidx;
          if (LO) {
            if (i != rg) *out += v * kScale;
          } else {
            *out = (i == rg) ? 0.0 : v * kScale;
          }
        }
      }
  }
}

template <bool LO>
__global__ __launch_bounds__(kGThreads) void bwd_i8_kernel(BatchArgs b) {
  __shared__ __attribute__((aligned(16))) int8_t Rb0[kIBufBytes];
  __shared__ __attribute__((aligned(16))) int8_t Rb1[kIBufBytes];
  __shared__ __attribute__((aligned(16))) uint8_t sig0[kGPosMax * kSigPitch];
  __shared__ __attribute__((aligned(16))) uint8_t sig1[kGPosMax * kSigPitch];
  __shared__ int32_t item_s;
  int32_t qi = 0;
  const int32_t total = total_items(b, KIND_BWD);
  for (;;) {
    if (threadIdx.x == 0) item_s = next_item(b.ctr + KIND_BWD * kQueues, total, qi);
    __syncthreads();
    const int32_t t = __builtin_amdgcn_readfirstlane(item_s);
    if (t < 0) break;
    const Item it = decode_item(b, KIND_BWD, t);
    const EvalArgs a = load_uniform(b.ev + it.m);
    if (a.B_pad < kNegSeqMax) i8_item<LO, true>(b, a, it, Rb0, Rb1, sig0, sig1);
    else i8_item<LO, false>(b, a, it, Rb0, Rb1, sig0, sig1);
    __syncthreads();
  }
}

int32_t i8_backward_blocks_per_site(int32_t N, int32_t q) { return g3_backward_blocks_per_site(N, q); }

int32_t i8_resident_blocks() {
  int per = 0;
  const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, bwd_i8_kernel<false>, kGThreads, 0);
  return (e == hipSuccess && per > 0) ? per : 1;
}

hipError_t launch_backward_i8(const BatchArgs& b, int32_t nblocks, int32_t lo, hipStream_t st) {
  if (lo) hipLaunchKernelGGL(bwd_i8_kernel<true>, dim3(nblocks), dim3(kGThreads), 0, st, b);
  else hipLaunchKernelGGL(bwd_i8_kernel<false>, dim3(nblocks), dim3(kGThreads), 0, st, b);
  return hipGetLastError();
}

int32_t mfma_backward_blocks_per_site(int32_t N, int32_t q) {
  const int32_t p = mfma_block_positions(q);
  return (N + p - 1) / p;
}

hipError_t launch_backward_mfma(const BatchArgs& b, int32_t npieces, int32_t f16, int32_t nblocks,
                                hipStream_t st) {
  if (f16 && npieces == 2)
    hipLaunchKernelGGL((bwd_mfma_kernel<2, true>), dim3(nblocks), dim3(kMThreads), 0, st, b);
  else if (!f16 && npieces == 3)
    hipLaunchKernelGGL((bwd_mfma_kernel<3, false>), dim3(nblocks), dim3(kMThreads), 0, st, b);
  else if (!f16 && npieces == 2)
    hipLaunchKernelGGL((bwd_mfma_kernel<2, false>), dim3(nblocks), dim3(kMThreads), 0, st, b);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// resident blocks per CU of the persistent MFMA kernels: kind 0 forward, 1 backward
int32_t mfma_resident_blocks(int32_t kind, int32_t npieces) {
  int per = 0;
  hipError_t e = hipErrorInvalidValue;
  if (kind == KIND_FWD)
    e = npieces == 3 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fwd_mfma_kernel<3>, kMThreads, 0)
                     : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fwd_mfma_kernel<2>, kMThreads, 0);
  else
    e = npieces == 3 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, bwd_mfma_kernel<3, false>, kMThreads, 0)
                     : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, bwd_mfma_kernel<2, true>, kMThreads, 0);
  return (e == hipSuccess && per > 0) ? per : 1;
}

}  // namespace plm
