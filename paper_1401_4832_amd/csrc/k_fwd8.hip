// k_fwd8.hip -- the energies of the pseudolikelihood (eq. condpfinal)
// E_b(s) = h_r(s) + sum_{i != r} J_ri(s, sigma_i^b) as an int8 matrix-core
// product, for three sites at once, followed by the log-softmax, objective,
// residual and field-gradient epilogue of the gather forward (sec. 3.4 step 3).
//
// Couplings in fixed point: each site's J_r is scaled by 2^k_r with
// max |J_r| 2^k_r in [2^21, 2^22) and rounded (|dJ| <= 2^-(k_r + 1) <= 2^-22 max |J_r|),
// then written as three signed int8 digits (hi 2^16 + mid 2^8 + lo), once per
// evaluation (jmax_kernel, jquant_kernel).  The product runs on the 4:2 sparse
// matrix-core instruction v_smfmac_i32_32x32x64_i8 with rows = sequences,
// columns = the 63 (site, state) pairs of the group in two 32-column tiles, and
// the inner index over position triples: a triple (3G, 3G+1, 3G+2) x 21 states
// = 63 inner indices, padded to 64 = one instruction.  The one-hot operand is
// sparse by construction: position p's states take the inner indices 21p .. 21p+20,
// so any aligned group of four holds states of at most two positions, hence at
// most two ones, which is the instruction's 4:2 format; it takes the same time
// as the dense 32x32x32 int8 product, i.e. half the matrix-core time per triple.
// A lane's operand (one sequence, inner indices [32 half, +32)) is 16 value
// bytes (a value pair per group of four) and a word of 2-bit positions; it holds
// the one of one position that lies wholly in the half and, if it lies there,
// the one of the middle position.  The coupling operand of a lane is two
// 16-byte digit fragments, inner indices [16 half, +16) and [32 + 16 half, +16).
// Each digit plane accumulates exactly in int32 (|digit| <= 128, at most
// 3 ceil(N/3) one-hot terms per output); the planes are combined and scaled
// back in FP64 once at the end.  The couplings stream through LDS four
// triples at a time (global -> LDS copies as buffer loads with an LDS
// destination, double-buffered in two separate arrays), the triples' symbols
// likewise.
#include <math.h>

#include "plm_internal.h"

namespace plm {

typedef int32_t fi32x4 __attribute__((ext_vector_type(4)));
typedef int32_t fi32x8 __attribute__((ext_vector_type(8)));
typedef int32_t fi32x16 __attribute__((ext_vector_type(16)));

constexpr int kFIWaves = 8;
constexpr int kFIThreads = kFIWaves * 64;
constexpr int kFIRB = 2;                                   // 32-sequence row blocks per wave
constexpr int kFISeqs = kFIWaves * kFIRB * 32;             // 512 sequences per item
static_assert(kFISeqs % 256 == 0, "symbol copies of 1 KB");
constexpr int kFIStageG = 4;                               // position triples per LDS stage
constexpr int kFISiteBytes = kFIStageG * kWqGroupBytes;    // 16128
// bank-disjoint site runs: column c of a tile reads 16-byte slot c mod 8
constexpr int kFISiteStride = kFISiteBytes + 80;
static_assert((kFISiteStride / 16 - kSlot) % 8 == 0 && kFISiteStride % 16 == 0, "bank-disjoint site runs");
constexpr int kFIBufBytes = 2 * kFISiteStride + kFISiteBytes;
constexpr int kFISymWords = kFIStageG * kFISeqs;
constexpr int kFIParkFloats = 3 * 32 * 24;                 // one row block of energies per wave, [site][row][24]
static_assert(4 * kFIParkFloats * 4 <= kFIBufBytes, "four waves' energies fit one buffer");
static_assert(3 * 672 <= 32 * 24 * 4, "a site's staged digits fit its park rows");
constexpr int kJexpBad = -100000;                          // non-finite coupling: energies NaN

int32_t fwd_i8_tile_seqs() { return kFISeqs; }

// ---- couplings -> digits, kJParts blocks per active site -------------------------
// jmax_kernel: block (site, part) takes the positions [part N / P, (part + 1) N / P)
// of the site's slice (the i = r block left out) and stores the largest |J| as
// float bits, or -1 when a value is not finite.
__global__ __launch_bounds__(256) void jmax_kernel(BatchArgs b) {
  __shared__ int32_t red[4];
  const int idx = blockIdx.x / kJParts, part = blockIdx.x - idx * kJParts;
  if (idx >= *b.n_active) return;
  const int g = b.active[idx];
  const int m = b.msa_of[g];
  const EvalArgs a = load_uniform(b.ev + m);
  const int r = g - b.site_base[m];
  const int N = a.N, qq = a.q * a.q;
  const auto Jr = gmem(a.J + (size_t)r * N * qq);
  const int e0 = (int)((int64_t)part * N / kJParts) * qq, e1 = (int)((int64_t)(part + 1) * N / kJParts) * qq;
  const int s0 = r * qq, s1 = s0 + qq;
  float mx = 0.f;
  int bad = 0;
  for (int e = e0 + (int)threadIdx.x; e < e1; e += 256) {
    if (e >= s0 && e < s1) continue;
    const float v = Jr[e];
    bad |= !isfinite(v);
    mx = fmaxf(mx, fabsf(v));
  }
  int32_t t = bad ? -1 : __float_as_int(mx);  // non-negative floats order as their bits
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const int32_t u = __shfl_xor(t, o, 64);
    t = (t < 0 || u < 0) ? -1 : max(t, u);
  }
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t v = red[0];
#pragma unroll
    for (int w = 1; w < 4; ++w) v = (v < 0 || red[w] < 0) ? -1 : max(v, red[w]);
    gmem_w(a.jexp + a.N)[r * kJParts + part] = v;
  }
}

// jquant_kernel: block (site, part) combines the site's partial maxima into the
// exponent k_r (part 0 stores it) and writes its share of the digit units.
__global__ __launch_bounds__(256) void jquant_kernel(BatchArgs b) {
  const int idx = blockIdx.x / kJParts, part = blockIdx.x - idx * kJParts;
  if (idx >= *b.n_active) return;
  const int g = b.active[idx];
  const int m = b.msa_of[g];
  const EvalArgs a = load_uniform(b.ev + m);
  const int r = g - b.site_base[m];
  const int q = a.q, N = a.N, qq = q * q;
  const auto Jr = gmem(a.J + (size_t)r * N * qq);
  const auto parts = gmem(a.jexp + N + (size_t)r * kJParts);
  int32_t t = 0;
#pragma unroll
  for (int p = 0; p < kJParts; ++p) {
    const int32_t u = parts[p];
    t = (t < 0 || u < 0) ? -1 : max(t, u);
  }
  const bool badsite = t < 0;
  int ex = 0;
  if (!badsite) (void)frexpf(__int_as_float(t), &ex);  // max = f 2^ex, f in [0.5, 1) (ex = 0 for 0)
  const int kexp = badsite ? kJexpBad : kRiScaleLog2 - ex;
  if (part == 0 && threadIdx.x == 0) gmem_w(a.jexp)[r] = kexp;
  const int k = badsite ? 0 : kexp;
  const int units = a.NG * 4 * kSlot;  // (triple, step, half, state)
  const int u0 = (int)((int64_t)part * units / kJParts), u1 = (int)((int64_t)(part + 1) * units / kJParts);
  auto Wq = gmem_w(a.Wq + (size_t)r * a.NG * kWqGroupBytes);
  for (int u = u0 + (int)threadIdx.x; u < u1; u += 256) {
    const int G = u / (4 * kSlot), rem = u - G * (4 * kSlot);
    const int th = rem / kSlot, sidx = rem - th * kSlot;  // th = 2 t + half
    uint32_t w[3][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}};
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int K = 16 * th + j;  // inner index within the triple
      const int p = K / kSlot, kk = K - p * kSlot;
      const int i = 3 * G + p;
      int v = 0;
      if (p < 3 && i < N && i != r && kk < q && sidx < q && !badsite)
        v = (int)rintf(ldexpf(Jr[(size_t)i * qq + kk * q + sidx], k));
      const int lo = (int)(int8_t)(v & 255);
      const int v1 = (v - lo) >> 8;
      const int mid = (int)(int8_t)(v1 & 255);
      const int hi = (v1 - mid) >> 8;
      w[0][j >> 2] |= (uint32_t)(uint8_t)hi << (8 * (j & 3));
      w[1][j >> 2] |= (uint32_t)(uint8_t)mid << (8 * (j & 3));
      w[2][j >> 2] |= (uint32_t)(uint8_t)lo << (8 * (j & 3));
    }
#pragma unroll
    for (int d = 0; d < 3; ++d)
      *reinterpret_cast<__attribute__((address_space(1))) u32x4_t*>(
          Wq + (size_t)G * kWqGroupBytes + d * (kWqGroupBytes / 3) + (th * kSlot + sidx) * 16) =
          u32x4_t{w[d][0], w[d][1], w[d][2], w[d][3]};
  }
}

// ---- symbols of position triples ---------------------------------------------
__global__ void sym3_kernel(const uint8_t* __restrict__ msa_cm, int32_t B_pad, int32_t N, int32_t NG,
                            uint32_t* __restrict__ sym3) {
  const size_t total = (size_t)NG * B_pad;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int G = (int)(e / B_pad), b = (int)(e - (size_t)G * B_pad);
    uint32_t v = 0;
#pragma unroll
    for (int p = 0; p < 3; ++p) {
      const int i = 3 * G + p;
      if (i < N) v |= (uint32_t)msa_cm[((size_t)(i >> 4) * B_pad + b) * 16 + (i & 15)] << (8 * p);
    }
    sym3[e] = v;
  }
}

hipError_t launch_sym3(const uint8_t* msa_cm, int32_t B_pad, int32_t N, int32_t NG, uint32_t* sym3, hipStream_t st) {
  const size_t total = (size_t)NG * B_pad;
  int blocks = (int)((total + 255) / 256);
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(sym3_kernel, dim3(blocks), dim3(256), 0, st, msa_cm, B_pad, N, NG, sym3);
  return hipGetLastError();
}

// 16 bytes, byte j = bit j of bits (one multiply per 4 bits)
__device__ inline uint4 spread16(uint32_t bits) {
  uint32_t w[4];
#pragma unroll
  for (int d = 0; d < 4; ++d) w[d] = (((bits >> (4 * d)) & 15u) * 0x00204081u) & 0x01010101u;
  return make_uint4(w[0], w[1], w[2], w[3]);
}

// The 4:2 sparse one-hot operand of one lane for one position triple.  s3 holds
// the triple's symbols (byte p = sigma_{3G+p}); the lane's half of the inner
// index holds the one of position shA / 8 at offset oA + sigma (always inside),
// and position 1's at oB + sigma when that lies in [0, 32).  Inner index k of
// the half is group k / 4, position k % 4: the first one takes value slot 0 of
// its group, the second slot 1 (the two may share a group, never a slot).
__device__ inline void onehot_sparse(uint32_t s3, int shA, int oA, int oB, uint4& val, uint32_t& pos) {
  const int kA = (int)((s3 >> shA) & 255u) + oA;
  const int kB0 = (int)((s3 >> 8) & 255u) + oB;
  const bool in = (uint32_t)kB0 < 32u;
  const int kB = in ? kB0 : 0;
  const uint32_t bytes = (1u << ((kA >> 1) & 0x1e)) | ((uint32_t)in << (((kB >> 1) & 0x1e) + 1));
  pos = ((uint32_t)(kA & 3) << (kA & 0x1c)) | ((uint32_t)(kB & 3) << ((kB & 0x1c) + 2));
  val = spread16(bytes);
}

// The descriptor's fields are read where they are needed (the epilogue's after
// the product loop), so that they do not occupy scalar registers across it.
__device__ inline void fwd_i8_item(const BatchArgs& bt, const EvalArgs* ea, const Item& it, int8_t* W0, int8_t* W1,
                                   uint32_t* S0, uint32_t* S1, double* red, double* wrow, uint8_t* srow) {
  const int q = load_uniform(&ea->q), N = load_uniform(&ea->N), NG = load_uniform(&ea->NG);
  const int B_pad = load_uniform(&ea->B_pad);
  const int32_t* jexp = load_uniform(&ea->jexp);
  const int8_t* Wq = load_uniform(&ea->Wq);
  const uint32_t* sym3 = load_uniform(&ea->sym3);
  const int tid = item_tid(), lane = tid & 63;
  const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform: copy bookkeeping in scalars
  const int half = lane >> 5, l32 = lane & 31;
  const int cnt = it.cnt;
  const int tile = it.sub;
  const int b0 = tile * kFISeqs;
  int32_t rs[kG3Sites];
#pragma unroll
  for (int g = 0; g < kG3Sites; ++g)
    rs[g] = __builtin_amdgcn_readfirstlane(g < cnt ? bt.active[it.first + g] - bt.site_base[it.m] : it.r);
  uint32_t boff[2];
#pragma unroll
  for (int T = 0; T < 2; ++T) {
    const int col = min(32 * T + l32, 3 * kSlot - 1);
    const int g = col / kSlot, sidx = col - g * kSlot;
    boff[T] = (uint32_t)(g * kFISiteStride + half * (kSlot * 16) + sidx * 16);
  }
  const int nst = (NG + kFIStageG - 1) / kFIStageG;

  // global -> LDS copies of stage c: the group's digits of triples 4c .. 4c+3
  // (a site's run is contiguous; the last 1 KB copy of a run is moved back to
  // end at the run's end) and the triples' symbols of the item's sequences,
  // 1 KB per copy, copy k issued by wave k mod 8.  A full stage of a full
  // group has the same copies every stage, shifted by the stage's offsets:
  // wave w copies parts w and w + 8 of each site's run and symbol part w.
  constexpr int kSymParts = kFISeqs / 256;  // 1 KB copies of a triple's symbols
  constexpr int kFullPer = (kFISiteBytes + 1023) / 1024;
  static_assert(kFullPer % kFIWaves == 0 && (kSymParts * kFIStageG) % kFIWaves == 0,
                "a full stage's copies divide evenly over the waves");
  const char* sbase[kG3Sites];
#pragma unroll
  for (int g = 0; g < kG3Sites; ++g)
    sbase[g] = reinterpret_cast<const char*>(Wq) + (size_t)rs[g] * NG * kWqGroupBytes;
  auto fetch = [&](int c, int8_t* Wd, uint32_t* Sd) {
    const int ng = min(kFIStageG, NG - c * kFIStageG);
    if (ng == kFIStageG && cnt == kG3Sites) {
#pragma unroll
      for (int g = 0; g < kG3Sites; ++g)
#pragma unroll
        for (int j = 0; j < kFullPer / kFIWaves; ++j) {
          const int off = min((wid + kFIWaves * j) * 1024, kFISiteBytes - 1024);
          copy16_to_lds(sbase[g] + (size_t)c * kFISiteBytes + off, Wd + g * kFISiteStride + off, lane);
        }
#pragma unroll
      for (int j = 0; j < kSymParts * kFIStageG / kFIWaves; ++j) {
        const int k = wid + kFIWaves * j, kg = k / kSymParts, part = k - kg * kSymParts;
        copy16_to_lds(sym3 + (size_t)(c * kFIStageG + kg) * B_pad + b0 + part * 256, Sd + kg * kFISeqs + part * 256,
                      lane);
      }
      return;
    }
    const int bytes = ng * kWqGroupBytes;
    const int per = (bytes + 1023) / 1024;
    const int ninst = cnt * per + kSymParts * ng;
    for (int k = wid; k < ninst; k += kFIWaves) {
      if (k < cnt * per) {
        const int g = k / per, part = k - g * per;
        const int off = min(part * 1024, bytes - 1024);
        const int rg = g == 0 ? rs[0] : (g == 1 ? rs[1] : rs[2]);
        const char* src = reinterpret_cast<const char*>(Wq) +
                          ((size_t)rg * NG + (size_t)c * kFIStageG) * kWqGroupBytes + off;
        copy16_to_lds(src, Wd + g * kFISiteStride + off, lane);
      } else {
        const int k2 = k - cnt * per, kg = k2 / kSymParts, part = k2 - kg * kSymParts;
        copy16_to_lds(sym3 + (size_t)(c * kFIStageG + kg) * B_pad + b0 + part * 256, Sd + kg * kFISeqs + part * 256,
                      lane);
      }
    }
  };

  fi32x16 acc[3][kFIRB][2];
#pragma unroll
  for (int d = 0; d < 3; ++d)
#pragma unroll
    for (int m = 0; m < kFIRB; ++m)
#pragma unroll
      for (int T = 0; T < 2; ++T) acc[d][m][T] = fi32x16{};

  // the lane's half of the inner index: half 0 = position 0 (offset 0) and
  // position 1's states 0..10 (offset 21); half 1 = position 2 (offset 42 - 32)
  // and position 1's states 11..20 (offset 21 - 32)
  const int shA = half ? 16 : 0, oA = half ? 2 * kSlot - 32 : 0, oB = half ? kSlot - 32 : kSlot;
  // the packed symbols of triple kg for the wave's row blocks
  auto load_s3 = [&](const uint32_t* Sc, int kg, uint32_t* s3) {
#pragma unroll
    for (int m = 0; m < kFIRB; ++m) s3[m] = Sc[kg * kFISeqs + (wid * kFIRB + m) * 32 + l32];
  };
  auto stage = [&](int c, const int8_t* Wc, const uint32_t* Sc, int8_t* Wn, uint32_t* Sn) {
    if (c + 1 < nst) fetch(c + 1, Wn, Sn);
    const int ng = min(kFIStageG, NG - c * kFIStageG);
    const char* wb = reinterpret_cast<const char*>(Wc);
    // each triple's symbols are read one triple ahead
    uint32_t s3n[kFIRB];
    load_s3(Sc, 0, s3n);
    for (int kg = 0; kg < ng; ++kg) {
      uint4 av[kFIRB];
      uint32_t ap[kFIRB];
      // the six B operands (digit, tile) of this triple, each read two ahead of
      // its use: the digit fragments of steps 0 and 1 of the lane's half
      const char* fb = wb + kg * kWqGroupBytes;
      auto ldb = [&](int f) {
        const char* p = fb + boff[f & 1] + (f >> 1) * (kWqGroupBytes / 3);
        const uint4 x = *reinterpret_cast<const uint4*>(p);
        const uint4 y = *reinterpret_cast<const uint4*>(p + 2 * kSlot * 16);
        return fi32x8{(int)x.x, (int)x.y, (int)x.z, (int)x.w, (int)y.x, (int)y.y, (int)y.z, (int)y.w};
      };
      // the symbols read one triple ahead have arrived (lgkmcnt 0, vmcnt and
      // expcnt left at their maxima, so the stage copies stay in flight): the
      // one-hot operands are then built while the first B operands are read
      __builtin_amdgcn_s_waitcnt(0xc07f);
      fi32x8 bq0 = ldb(0), bq1 = ldb(1);
#pragma unroll
      for (int m = 0; m < kFIRB; ++m) onehot_sparse(s3n[m], shA, oA, oB, av[m], ap[m]);
      load_s3(Sc, min(kg + 1, ng - 1), s3n);
#pragma unroll
      for (int f = 0; f < 6; ++f) {
        fi32x8 bq2 = bq1;
        if (f + 2 < 6) bq2 = ldb(f + 2);
#pragma unroll
        for (int m = 0; m < kFIRB; ++m)
          acc[f >> 1][m][f & 1] = __builtin_amdgcn_smfmac_i32_32x32x64_i8(
              __builtin_bit_cast(fi32x4, av[m]), bq0, acc[f >> 1][m][f & 1], (int)ap[m], 0, 0);
        bq0 = bq1;
        bq1 = bq2;
      }
      // issue order: the first two B operands, the one-hot operands and the next
      // symbols, then each pair of products followed by the reads of the B
      // operand two ahead
      __builtin_amdgcn_sched_group_barrier(0x100, 4, 0);
      __builtin_amdgcn_sched_group_barrier(0x002, 80, 0);
#pragma unroll
      for (int f = 0; f < 6; ++f) {
        __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);
        if (f == 0) __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
        if (f + 2 < 6) __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
      }
    }
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
  };

  fetch(0, W0, S0);
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  // unrolled by two so that each stage names its buffers at compile time: with
  // the buffers picked at run time the compiler cannot tell the copies' target
  // from the buffer being read and waits for the copies inside the triple loop
  for (int c = 0; c < nst; c += 2) {
    stage(c, W0, S0, W1, S1);
    if (c + 1 < nst) stage(c + 1, W1, S1, W0, S0);
  }

  // ---- epilogue: energies -> log-softmax, objective, residual digits, dh ----
  // A lane takes one (sequence, site) pair and runs over the states serially,
  // so that the log-sum-exp needs no cross-lane reductions: pass 0 takes the
  // pairs (row lane % 32, site lane / 32), pass 1 (row lane, site 2) on lanes
  // 0..31.  Energies are parked per wave as [site][row][24]; the residual
  // digits of a site are staged over its consumed park rows in the layout of
  // the gradient's fragments ([digit][16-row half][state][16 rows], 672 bytes
  // per digit and row block) and copied out 16 bytes per lane.  The field
  // gradient sums the staged digits (exact integers).  Park, weights, symbols
  // and staging are this wave's own, so the epilogue needs no block barrier.
  // An opaque zero defined here: the epilogue's LDS addresses are offset by it,
  // so that they are formed after the product loop instead of being held in
  // vector registers across it (the loop needs every register for its
  // accumulators and operands); the sites' scale exponents are loaded here for
  // the same reason.
  uint32_t zo;
  asm volatile("s_mov_b32 %0, 0" : "=s"(zo));
  W0 += zo;
  W1 += zo;
  S0 += zo;
  red = reinterpret_cast<double*>(reinterpret_cast<char*>(red) + zo);
  wrow = reinterpret_cast<double*>(reinterpret_cast<char*>(wrow) + zo);
  srow += zo;
  int32_t ks[kG3Sites];
#pragma unroll
  for (int g = 0; g < kG3Sites; ++g) ks[g] = gmem(jexp)[rs[g]];
  const int nch = B_pad >> 8;
  const float* hfield = load_uniform(&ea->h);
  const double* wts = load_uniform(&ea->w);
  const uint8_t* msa_cm = load_uniform(&ea->msa_cm);
  const int Bn = load_uniform(&ea->B);
  float* park = wid < 4 ? reinterpret_cast<float*>(W0) + wid * kFIParkFloats
                        : reinterpret_cast<float*>(W1) + (wid - 4) * kFIParkFloats;
  uint8_t* stg = reinterpret_cast<uint8_t*>(park);
  // fields of the group's sites, [site][24]; states >= q get -inf, so that
  // their energies drop out of the softmax and their residuals are exactly 0
  float* hsh = reinterpret_cast<float*>(S0);
  if (tid < 3 * 24) {
    const int g = tid / 24, ss = tid - g * 24;
    const int rg = g == 0 ? rs[0] : (g == 1 ? rs[1] : rs[2]);
    hsh[tid] = ss >= q ? -INFINITY : (g < cnt ? gmem(hfield)[rg * q + ss] : 0.f);
  }
  __syncthreads();
  double* wv = wrow + wid * 32;    // this wave's row block: weights and
  uint8_t* sv = srow + wid * 96;   // the group's own symbols, [site][row]
  const int row = lane & 31;
  double fpass[2] = {0.0, 0.0};    // objective terms of pass 0 (site lane / 32) and pass 1 (site 2)
  int32_t ghi = 0;                 // lane (site, state) < 63: digit sum of the residuals, scaled 2^22
  const int gl = lane / kSlot, sl = lane - gl * kSlot;
#pragma unroll
  for (int m = 0; m < kFIRB; ++m) {
    const int brow = b0 + (wid * kFIRB + m) * 32;
    if (lane < 32) wv[lane] = brow + lane < Bn ? gmem(wts)[brow + lane] : 0.0;
#pragma unroll
    for (int k2 = 0; k2 < 2; ++k2) {
      const int e2 = lane + 64 * k2;
      if (e2 < 96) {
        const int g2 = e2 >> 5, row2 = e2 & 31;
        const int r2 = g2 == 0 ? rs[0] : (g2 == 1 ? rs[1] : rs[2]);
        sv[e2] = gmem(msa_cm)[((size_t)(r2 / kFwdChunk) * B_pad + brow + row2) * kFwdChunk + r2 % kFwdChunk];
      }
    }
    // this row block's energies without h
#pragma unroll
    for (int T = 0; T < 2; ++T) {
      const int col = 32 * T + l32;
      const int g = col / kSlot, sc = col - g * kSlot;
      const int kg_ = g == 0 ? ks[0] : (g == 1 ? ks[1] : ks[2]);
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        // v = 65536 a0 + 256 a1 + a2 exactly: u = 256 a1 + a2 fits int32, and
        // with a0' = a0 + (u >> 16), r = u & 0xffff both FP32 operands are
        // exact, so the fma rounds v to FP32 once
        const int32_t u = acc[1][m][T][j] * 256 + acc[2][m][T][j];
        const float v = fmaf((float)(acc[0][m][T][j] + (u >> 16)), 65536.f, (float)(u & 0xffff));
        if (col < 3 * kSlot)
          park[(g * 32 + 8 * (j >> 2) + 4 * half + (j & 3)) * 24 + sc] =
              kg_ == kJexpBad ? NAN : ldexpf(v, -kg_);
      }
    }
#pragma unroll
    for (int pass = 0; pass < 2; ++pass) {
      const int g = pass == 0 ? (lane >> 5) : 2;
      if (pass == 1 && lane >= 32) continue;
      float e[24];
      const float4* pr = reinterpret_cast<const float4*>(park + (g * 32 + row) * 24);
      const float4* hr = reinterpret_cast<const float4*>(hsh + g * 24);
#pragma unroll
      for (int v4 = 0; v4 < 6; ++v4) {
        const float4 x = pr[v4], hh = hr[v4];
        e[4 * v4] = x.x + hh.x;
        e[4 * v4 + 1] = x.y + hh.y;
        e[4 * v4 + 2] = x.z + hh.z;
        e[4 * v4 + 3] = x.w + hh.w;
      }
      const int sr = sv[g * 32 + row];
      const double wb = wv[row];
      // the observed state's energy read back by index (no per-state compare
      // masks kept alive between the loops)
      const float esr = park[(g * 32 + row) * 24 + sr] + hsh[g * 24 + sr];
      float mx = -INFINITY;
#pragma unroll
      for (int st = 0; st < kSlot; ++st) mx = fmaxf(mx, e[st]);
      // exp(x) = 2^(x log2 e) on the hardware exponential; x <= 0, so no range
      // handling is needed (|x| log2 e is rounded to 2^-24 relative, i.e. the
      // probability e^x moves by at most 2^-24 |x| e^x < 2.2e-8 absolute)
      float sum = 0.f;
#pragma unroll
      for (int st = 0; st < kSlot; ++st) {
        e[st] = __builtin_amdgcn_exp2f((e[st] - mx) * 1.4426950408889634f);
        sum += e[st];
      }
      const float lse = mx + logf(sum);
      const float inv = 1.f / sum;
      fpass[pass] += wb * (double)(lse - esr);
      const float wf = (float)wb;
      // digits of round(R 2^22), R = w (P - [s = sigma_r]), into the staging of site g
      uint8_t* sg = stg + g * (32 * 24 * 4) + (row >> 4) * (kSlot * 16) + (row & 15);
#pragma unroll
      for (int st = 0; st < kSlot; ++st) {
        const float P = e[st] * inv;
        const float Rv = wf * (P - (st == sr ? 1.f : 0.f));  // P = 0 for states >= q
        const int v = (int)rintf(Rv * (float)(1 << kRiScaleLog2));
        const int lo = (int)(int8_t)(v & 255);
        const int v1 = (v - lo) >> 8;
        const int mid = (int)(int8_t)(v1 & 255);
        const int hi = (v1 - mid) >> 8;
        sg[st * 16] = (uint8_t)hi;
        sg[672 + st * 16] = (uint8_t)mid;
        sg[2 * 672 + st * 16] = (uint8_t)lo;
      }
    }
    // staged digits -> the fragment layout, 16 bytes per lane (sites of the group only)
    auto Ri = gmem_w(reinterpret_cast<int8_t*>(load_uniform(&ea->R)));
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      const int k = lane + 64 * i;  // (site, digit) segment k / 42, 16-byte part k % 42
      const int seg = k / 42, part = k - seg * 42;
      const int g = seg / 3, d = seg - g * 3;
      if (k < 9 * 42 && g < cnt) {
        const int rg = g == 0 ? rs[0] : (g == 1 ? rs[1] : rs[2]);
        const uint4 x = *reinterpret_cast<const uint4*>(stg + g * (32 * 24 * 4) + d * 672 + part * 16);
        *reinterpret_cast<__attribute__((address_space(1))) u32x4_t*>(
            Ri + rifrag_index(rg, nch, brow, 0) + (size_t)d * kRiDigitBytes + part * 16) =
            u32x4_t{x.x, x.y, x.z, x.w};
      }
    }
    // field gradient: lane (site, state) sums its 32 rows of each digit plane
    if (lane < 3 * kSlot) {
      int32_t dsum[3];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        int32_t t = 0;
#pragma unroll
        for (int h16 = 0; h16 < 2; ++h16) {
          const uint4 x = *reinterpret_cast<const uint4*>(stg + gl * (32 * 24 * 4) + d * 672 + h16 * (kSlot * 16) +
                                                          sl * 16);
          t = __builtin_amdgcn_sdot4((int)x.x, 0x01010101, t, false);
          t = __builtin_amdgcn_sdot4((int)x.y, 0x01010101, t, false);
          t = __builtin_amdgcn_sdot4((int)x.z, 0x01010101, t, false);
          t = __builtin_amdgcn_sdot4((int)x.w, 0x01010101, t, false);
        }
        dsum[d] = t;
      }
      ghi += dsum[0] * 65536 + dsum[1] * 256 + dsum[2];
    }
  }
  // objective partials: per site, a fixed-order tree over the wave's lanes, then the waves in order
  double f0 = fpass[0], f1 = fpass[1];
#pragma unroll
  for (int o = 16; o > 0; o >>= 1) {
    f0 += __shfl_xor(f0, o, 64);
    f1 += __shfl_xor(f1, o, 64);
  }
  if (lane == 0) {
    red[wid * 64] = f0;       // site 0
    red[wid * 64 + 2] = f1;   // site 2
  }
  if (lane == 32) red[wid * 64 + 1] = f0;  // site 1
  __syncthreads();
  if (tid < cnt) {
    double t = 0.0;
    for (int w = 0; w < kFIWaves; ++w) t += red[w * 64 + tid];
    const int rg = tid == 0 ? rs[0] : (tid == 1 ? rs[1] : rs[2]);
    gmem_w(load_uniform(&ea->f_part))[(size_t)tile * N + rg] = t;
  }
  __syncthreads();
  red[wid * 64 + lane] = (double)ghi;
  __syncthreads();
  if (tid < cnt * kSlot) {
    const int g = tid / kSlot, ss = tid - g * kSlot;
    double t = 0.0;
    for (int w = 0; w < kFIWaves; ++w) t += red[w * 64 + tid];
    const int rg = g == 0 ? rs[0] : (g == 1 ? rs[1] : rs[2]);
    gmem_w(load_uniform(&ea->gh_part))[((size_t)tile * N + rg) * kSlot + ss] = ss < q ? t * (1.0 / (double)(1 << kRiScaleLog2)) : 0.0;
  }
}

__global__ __launch_bounds__(kFIThreads) void fwd_i8_kernel(BatchArgs b) {
  __shared__ __attribute__((aligned(16))) int8_t W0[kFIBufBytes];
  __shared__ __attribute__((aligned(16))) int8_t W1[kFIBufBytes];
  __shared__ __attribute__((aligned(16))) uint32_t S0[kFISymWords];
  __shared__ __attribute__((aligned(16))) uint32_t S1[kFISymWords];
  __shared__ double red[kFIWaves * 64];
  __shared__ double wrow[kFIWaves * 32];
  __shared__ uint8_t srow[kFIWaves * 96];
  __shared__ int32_t item_s;
  int32_t qi = 0;
  const int32_t total = total_items(b, KIND_FWD);
  for (;;) {
    if (threadIdx.x == 0) item_s = next_item(b.ctr + KIND_FWD * kQueues, total, qi);
    __syncthreads();
    const int32_t t = __builtin_amdgcn_readfirstlane(item_s);
    if (t < 0) break;
    const Item it = decode_item(b, KIND_FWD, t);
    fwd_i8_item(b, b.ev + it.m, it, W0, W1, S0, S1, red, wrow, srow);
    __syncthreads();
  }
}

int32_t fwd_i8_resident_blocks() {
  int per = 0;
  const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fwd_i8_kernel, kFIThreads, 0);
  return (e == hipSuccess && per > 0) ? per : 1;
}

// Couplings of every active site to digits, then the energies and the rest of
// the forward.  total_sites bounds the active list (the grid of the first kernel).
hipError_t launch_jquant(const BatchArgs& b, int32_t total_sites, hipStream_t st) {
  hipLaunchKernelGGL(jmax_kernel, dim3(total_sites * kJParts), dim3(256), 0, st, b);
  hipLaunchKernelGGL(jquant_kernel, dim3(total_sites * kJParts), dim3(256), 0, st, b);
  return hipGetLastError();
}

hipError_t launch_fwd_i8(const BatchArgs& b, int32_t nblocks, hipStream_t st) {
  hipLaunchKernelGGL(fwd_i8_kernel, dim3(nblocks), dim3(kFIThreads), 0, st, b);
  return hipGetLastError();
}

}  // namespace plm
