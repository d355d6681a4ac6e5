// k_gather.hip -- FP32 gather/scatter evaluation of the per-site objective and
// gradient of asymmetric plmDCA (sec. 3.4 step 3: eqs. g_regdef2, g_gradh2,
// g_gradJ2) for many sites at once.
//
// Forward (one block = one site r x a tile of sequences): the site's coupling
// slice J_r is streamed through LDS sixteen columns at a time; each lane adds
// J_ri(s, sigma_i^b) into the energy E_b(s) of its (sequence, state) pair
// (eq. condpfinal), then a 21-lane segmented reduction gives log Z_b, the
// objective term w_b (log Z_b - E_b(sigma_r^b)) and the residual
// R_b(s) = w_b (P_b(s) - [sigma_r^b = s]), which is written to HBM.
//
// Backward (one block = one site r x 24 alignment columns, all sequences):
// dJ_ri(s,k) = sum_b [sigma_i^b = k] R_b(s).  Each wave owns three columns, so
// its read-modify-write scatter into LDS never races with another wave, and
// the three 21-lane slots of a wave write three bank-disjoint copies of each
// row.  FP32 LDS partials are folded into FP64 registers every 768 sequences.
#include "plm_internal.h"

namespace plm {

// Padded copy of the alignment in chunk-major order: symbol (b, i) at byte
// ((i / 16) * B_pad + b) * 16 + i % 16, so that the sixteen columns of a chunk
// for a run of rows are one contiguous block.  Symbols >= q raise the flag.
__global__ void pad_msa_kernel(const uint8_t* __restrict__ msa, int32_t B, int32_t N, int32_t q,
                               uint8_t* __restrict__ out, int32_t B_pad, int32_t N_pad,
                               int32_t* flag) {
  const size_t total = (size_t)B_pad * N_pad;
  const size_t per_chunk = (size_t)B_pad * kFwdChunk;
  int bad = 0;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const size_t c = e / per_chunk, rem = e - c * per_chunk;
    const int32_t b = (int32_t)(rem / kFwdChunk), i = (int32_t)(c * kFwdChunk + rem % kFwdChunk);
    uint8_t v = 0;
    if (b < B && i < N) {
      v = msa[(size_t)b * N + i];
      if (v >= q) { bad = 1; v = 0; }
    }
    out[e] = v;
  }
  if (bad && flag) atomicOr(flag, 1);
}

hipError_t launch_pad_msa(const uint8_t* msa, int32_t B, int32_t N, int32_t q, uint8_t* msa_cm,
                          int32_t B_pad, int32_t N_pad, int32_t* flag_dev, hipStream_t st) {
  const size_t total = (size_t)B_pad * N_pad;
  int blocks = (int)((total + 255) / 256);
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(pad_msa_kernel, dim3(blocks), dim3(256), 0, st, msa, B, N, q, msa_cm, B_pad,
                     N_pad, flag_dev);
  return hipGetLastError();
}

int32_t forward_tile_seqs(int32_t nb) { return kFwdWaves * kSlots * nb; }

// J chunk of the gather forward: kFwdPos columns of kQMax rows of 64 floats;
// the same LDS later parks 16 energies per lane (16 waves x 16 x 64 floats).
constexpr int kFwdPos = 8;
constexpr int kPosBytes = kQMax * kRowF * 4;  // 5376
static_assert((kFwdPos - 1) * kPosBytes + 20 * 256 + 255 < 65536, "LDS offsets fit the immediate field");
constexpr int kFwdJFloats = kFwdPos * kQMax * kRowF;
constexpr int kFwdParkFloats = kFwdWaves * 16 * 64;
// LDS floats of the forward block: the J chunk (with LO, as the FP64 sums of
// the couplings' high and low words, twice the bytes), or the parked energies
// (AT values)
template <class AT, bool LO>
constexpr int fwd_lds_floats() {
  return kFwdJFloats * (LO ? 2 : 1) > kFwdParkFloats * (int)(sizeof(AT) / 4) ? kFwdJFloats * (LO ? 2 : 1)
                                                                             : kFwdParkFloats * (int)(sizeof(AT) / 4);
}

// One forward work item: site r x sequence tile `tile` of one alignment.
// lds: J_r for kFwdPos columns, 3 copies per row, with a fixed pitch of kQMax
// rows per column so that a column's offset is a compile-time constant (and
// later the parked energies); sgl: the tile's symbols for those columns; red:
// FP64 reduction scratch.  AT is the accumulation type of the energies and of
// the log-softmax and residuals: float, or double (the precise path, whose
// residuals go out as two sets of int8 digits, rfrag = 3).  LO (with double):
// the point is h + h_lo, J + J_lo; the low words are staged and gathered like
// the high ones, and each pair is summed in FP64.
template <int NB, class AT, bool LO>
__device__ inline void fwd_item(const EvalArgs& a, int r, int tile, float* lds, uint2* sgl,
                                double* red) {
  static_assert(!LO || sizeof(AT) == 8, "low-order words only with FP64 accumulation");
  constexpr int tileSeq = kFwdWaves * kSlots * NB;
  const int q = a.q, N = a.N, qq = q * q;
  const int tid = item_tid(), lane = tid & 63, wid = tid >> 6;
  const int slot = lane / kSlot, s = lane - slot * kSlot;
  const int slotA = slot < kSlots ? slot : kSlots - 1;  // lane 63 shadows slot 2 for addressing
  const bool act = (slot < kSlots) && (s < q);
  const int tile0 = tile * tileSeq;
  const int tw = wid * (NB * kSlots) + slotA;  // tile row of row j: tw + 3j
  const int bw = tile0 + tw;

  AT E[NB];
  AT hv = act ? (AT)gmem(a.h)[r * q + s] : (AT)0;
  if (LO && act) hv += (AT)gmem(a.h_lo)[r * q + s];
#pragma unroll
  for (int j = 0; j < NB; ++j) E[j] = hv;

  const size_t Jr = (size_t)r * N * qq;
  const int nchunks = (N + kFwdPos - 1) / kFwdPos;
  const char* L = reinterpret_cast<const char*>(lds);
  // LDS byte address of row (p, sigma), this lane's word: p * kPosBytes (an
  // immediate offset) + sigma * 256 + 4 * lane, where the last two are one
  // byte permute: byte 0 = 4 * lane (< 256), byte 1 = the symbol byte
  const uint32_t lane4 = 4u * lane;
  // the next chunk's couplings and symbols travel in registers while the
  // current chunk is gathered
  constexpr int kJPer = (kFwdPos * kQMax * kQMax + kFwdThreads - 1) / kFwdThreads;
  constexpr int kSPer = (tileSeq + kFwdThreads - 1) / kFwdThreads;
  float jv[kJPer], jl[LO ? kJPer : 1];
  uint2 sv[kSPer];
  auto load = [&](int c) {
#pragma unroll
    for (int k = 0; k < kJPer; ++k) {
      const int e = tid + k * kFwdThreads;
      const int p = e / qq, rem = e - p * qq;
      const int i = c * kFwdPos + p;
      const bool in = e < kFwdPos * qq && i < N && i != r;
      jv[k] = in ? gmem(a.J)[Jr + (size_t)i * qq + rem] : 0.f;
      if (LO) jl[k] = in ? gmem(a.J_lo)[Jr + (size_t)i * qq + rem] : 0.f;
    }
#pragma unroll
    for (int k = 0; k < kSPer; ++k) {
      const int e = tid + k * kFwdThreads;
      if (e < tileSeq)
        sv[k] = gload_u2(a.msa_cm + ((size_t)(c >> 1) * a.B_pad + tile0 + e) * kFwdChunk + 8 * (c & 1));
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int k = 0; k < kJPer; ++k) {
      const int e = tid + k * kFwdThreads;
      if (e < kFwdPos * qq) {
        const int p = e / qq, rem = e - p * qq, kk = rem / q, ss = rem - kk * q;
        if (LO) {
          // the pair's exact FP64 sum (two 24-bit significands 2^24 apart fit
          // 53 bits), one 8-byte word per entry: the gather then reads one
          // word and adds once per term
          double* row = reinterpret_cast<double*>(lds) + (p * kQMax + kk) * kRowF;
          const double v = (double)jv[k] + (double)jl[k];
          row[ss] = v;
          row[ss + kSlot] = v;
          row[ss + 2 * kSlot] = v;
        } else {
          float* row = lds + (p * kQMax + kk) * kRowF;
          row[ss] = jv[k];
          row[ss + kSlot] = jv[k];
          row[ss + 2 * kSlot] = jv[k];
        }
      }
    }
#pragma unroll
    for (int k = 0; k < kSPer; ++k) {
      const int e = tid + k * kFwdThreads;
      if (e < tileSeq) sgl[e] = sv[k];
    }
  };
  load(0);
  for (int c = 0; c < nchunks; ++c) {
    __syncthreads();  // every wave is done with the previous chunk
    store();
    __syncthreads();
    if (c + 1 < nchunks) load(c + 1);
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const uint2 sg = sgl[tw + 3 * j];
      // two accumulation chains (even and odd columns)
      AT acc0 = E[j], acc1 = (AT)0;
#pragma unroll
      for (int p = 0; p < kFwdPos; ++p) {
        const uint32_t word = p < 4 ? sg.x : sg.y;
        const uint32_t addr = __builtin_amdgcn_perm(lane4, word, 0x0c0c0004u | ((uint32_t)(p & 3) << 8));
        AT v;
        if (LO) {
          // 8-byte rows: twice the float row's byte address, from a base per
          // four positions so that the offset fits the immediate field
          const char* L2 = L + (p < 4 ? 0 : 4 * 2 * kPosBytes);
          v = *reinterpret_cast<const double*>(L2 + 2 * addr + (p & 3) * 2 * kPosBytes);
        } else {
          v = (AT)*reinterpret_cast<const float*>(L + addr + p * kPosBytes);
        }
        if (p == 1) acc1 = v;
        else if (p & 1) acc1 += v;
        else acc0 += v;
      }
      E[j] = acc0 + acc1;
      // keep one row's loads in flight at a time, so rows do not pile up in registers
      __builtin_amdgcn_sched_barrier(0);
    }
  }

  // log-softmax over the 21 lanes of each slot, objective and residuals.  The
  // energies are parked in the (now free) LDS sixteen rows at a time so that
  // the per-row work below runs as a loop rather than unrolled over all rows.
  double facc = 0.0, ghacc = 0.0;
  const int sbase = slotA * kSlot;
  AT* park = reinterpret_cast<AT*>(lds) + wid * (16 * 64);  // 16 rows x 64 lanes per wave
#pragma unroll
  for (int g = 0; g < NB / 16; ++g) {
    __syncthreads();
#pragma unroll
    for (int jj = 0; jj < 16; ++jj) park[jj * 64 + lane] = E[g * 16 + jj];
    __syncthreads();
#pragma unroll 1
    for (int jj = 0; jj < 16; ++jj) {
      const int b = bw + 3 * (g * 16 + jj);
      const AT e = act ? park[jj * 64 + lane] : (AT)-INFINITY;
      AT m = e;
#pragma unroll
      for (int d = 1; d < 32; d <<= 1) {
        const AT o = __shfl_down(m, d, 64);
        if (s + d < kSlot) m = fmax(m, o);
      }
      m = __shfl(m, sbase, 64);
      const AT ex = act ? (AT)exp(e - m) : (AT)0;
      AT sum = ex;
#pragma unroll
      for (int d = 1; d < 32; d <<= 1) {
        const AT o = __shfl_down(sum, d, 64);
        if (s + d < kSlot) sum += o;
      }
      sum = __shfl(sum, sbase, 64);
      const AT lse = m + (AT)log(sum);
      const int sr = gmem(a.msa_cm)[((size_t)(r / kFwdChunk) * a.B_pad + b) * kFwdChunk + r % kFwdChunk];
      const double wb = (slot < kSlots && b < a.B) ? gmem(a.w)[b] : 0.0;
      const AT P = ex / sum;
      const AT Rv = act ? (AT)wb * (P - (s == sr ? (AT)1 : (AT)0)) : (AT)0;
      if (act && s == sr) facc += wb * (double)(lse - e);
      ghacc += (double)Rv;
      if (a.rfrag == 3) {
        // two sets of int8 digits, in the int8 gradient's fragment order for
        // every row of the tile (zero past B): v = round(R * 2^22) and, in the
        // second set, the remainder's round((R * 2^22 - v) * 2^22) -- R to
        // 2^-45 absolute; each set's integer sums are exact
        if (slot < kSlots) {
          const double x = (double)Rv * (double)(1 << kRiScaleLog2);
          const double vh = rint(x);
          const int vv[2] = {(int)vh, (int)rint((x - vh) * (double)(1 << kRiScaleLog2))};
          auto Ri = gmem_w(reinterpret_cast<int8_t*>(a.R));
          const size_t ix = rifrag_index(r, a.B_pad >> 8, b, s);
          const size_t lo_off = (size_t)a.N * (a.B_pad >> 8) * kRiChunkBytes;
#pragma unroll
          for (int z = 0; z < 2; ++z) {
            const int v = vv[z];
            const int lo = (int)(int8_t)(v & 255);
            const int v1 = (v - lo) >> 8;
            const int mid = (int)(int8_t)(v1 & 255);
            const int hi = (v1 - mid) >> 8;
            Ri[z * lo_off + ix] = (int8_t)hi;
            Ri[z * lo_off + ix + kRiDigitBytes] = (int8_t)mid;
            Ri[z * lo_off + ix + 2 * kRiDigitBytes] = (int8_t)lo;
          }
        }
      } else if (a.rfrag == 2) {
        // int8 digits of round(R * 2^22) in the int8 gradient's fragment
        // order, for every row of the tile (zero past B)
        if (slot < kSlots) {
          const int v = (int)rintf((float)Rv * (float)(1 << kRiScaleLog2));
          const int lo = (int)(int8_t)(v & 255);
          const int v1 = (v - lo) >> 8;
          const int mid = (int)(int8_t)(v1 & 255);
          const int hi = (v1 - mid) >> 8;
          auto Ri = gmem_w(reinterpret_cast<int8_t*>(a.R));
          const size_t ix = rifrag_index(r, a.B_pad >> 8, b, s);
          Ri[ix] = (int8_t)hi;
          Ri[ix + kRiDigitBytes] = (int8_t)mid;
          Ri[ix + 2 * kRiDigitBytes] = (int8_t)lo;
        }
      } else if (a.rfrag) {
        // FP16 hi/lo pieces of R * 2^12 in the grouped gradient's fragment
        // order, for every row of the tile (zero past B)
        if (slot < kSlots) {
          const float v = (float)Rv * kRfScale;
          const _Float16 hi = (_Float16)v;
          const _Float16 lo = (_Float16)(v - (float)hi);
          auto Rf = gmem_w(reinterpret_cast<uint16_t*>(a.R));
          const size_t ix = rfrag_index(r, a.B_pad >> 8, b, s);
          Rf[ix] = __builtin_bit_cast(uint16_t, hi);
          Rf[ix + kRfPieceWords] = __builtin_bit_cast(uint16_t, lo);
        }
      } else if (slot < kSlots && b < a.B3) {
        gmem_w(a.R)[((size_t)r * a.B3 + b) * kSlot + s] = (float)Rv;
      }
    }
  }
  const double ftot = block_sum_f64(facc, red);
  if (tid == 0) gmem_w(a.f_part)[(size_t)tile * N + r] = ftot;
  red[wid * 64 + lane] = (slot < kSlots) ? ghacc : 0.0;
  __syncthreads();
  if (tid < kSlot) {
    double t = 0.0;
    for (int w = 0; w < kFwdWaves; ++w)
      for (int c = 0; c < kSlots; ++c) t += red[w * 64 + c * kSlot + tid];
    gmem_w(a.gh_part)[((size_t)tile * N + r) * kSlot + tid] = t;
  }
}

// Persistent forward kernel: drains the forward work items of the batch.
template <int NB, class AT, bool LO>
__global__ __launch_bounds__(kFwdThreads) void fwd_kernel(BatchArgs b) {
  __shared__ __attribute__((aligned(16))) float lds[fwd_lds_floats<AT, LO>()];
  __shared__ uint2 sgl[kFwdWaves * kSlots * NB];
  __shared__ double red[kFwdWaves * 64];
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
    fwd_item<NB, AT, LO>(a, it.r, it.sub, lds, sgl, red);
    __syncthreads();
  }
}

// The precise path accumulates in FP64 with tiles of kFwdF64Rows rows per wave.
constexpr int kFwdF64Rows = 32;
int32_t forward_f64_tile_seqs() { return kFwdWaves * kSlots * kFwdF64Rows; }

hipError_t launch_forward(const BatchArgs& b, int32_t nb, int32_t nblocks, int32_t f64, hipStream_t st) {
  if (f64 == 2) {
    hipLaunchKernelGGL((fwd_kernel<kFwdF64Rows, double, true>), dim3(nblocks), dim3(kFwdThreads), 0, st, b);
    return hipGetLastError();
  }
  if (f64) {
    hipLaunchKernelGGL((fwd_kernel<kFwdF64Rows, double, false>), dim3(nblocks), dim3(kFwdThreads), 0, st, b);
    return hipGetLastError();
  }
  switch (nb) {
    case 16: hipLaunchKernelGGL((fwd_kernel<16, float, false>), dim3(nblocks), dim3(kFwdThreads), 0, st, b); break;
    case 32: hipLaunchKernelGGL((fwd_kernel<32, float, false>), dim3(nblocks), dim3(kFwdThreads), 0, st, b); break;
    case 64: hipLaunchKernelGGL((fwd_kernel<64, float, false>), dim3(nblocks), dim3(kFwdThreads), 0, st, b); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

int32_t forward_resident_blocks(int32_t nb, int32_t f64) {
  int per = 0;
  hipError_t e = hipErrorInvalidValue;
  if (f64) {
    e = f64 == 2
            ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fwd_kernel<kFwdF64Rows, double, true>, kFwdThreads, 0)
            : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fwd_kernel<kFwdF64Rows, double, false>, kFwdThreads,
                                                           0);
    return (e == hipSuccess && per > 0) ? per : 1;
  }
  switch (nb) {
    case 16: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fwd_kernel<16, float, false>, kFwdThreads, 0); break;
    case 32: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fwd_kernel<32, float, false>, kFwdThreads, 0); break;
    case 64: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fwd_kernel<64, float, false>, kFwdThreads, 0); break;
    default: break;
  }
  return (e == hipSuccess && per > 0) ? per : 1;
}

// Stable counting sort of each chunk's rows by their symbol at each column,
// done once per alignment.  Entry = (chunk-local row << 8) | symbol; the row
// field is then directly the byte offset of the row in the LDS residual tile
// (rows of 64 floats = 256 bytes), and the low byte the symbol.
__global__ __launch_bounds__(256) void chunk_sort_kernel(const uint8_t* __restrict__ msa_cm,
                                                         int32_t B3, int32_t B_pad, int32_t N,
                                                         int32_t q, uint16_t* __restrict__ sorted) {
  __shared__ uint16_t cnt[256][kQMax + 1];
  const int c = blockIdx.x, i = blockIdx.y * 256 + threadIdx.x;
  if (i >= N) return;
  const int b0 = c * kBwdSeqChunk, n = min(kBwdSeqChunk, B3 - b0);
  uint16_t* ct = cnt[threadIdx.x];
  for (int k = 0; k <= kQMax; ++k) ct[k] = 0;
  const uint8_t* col = msa_cm + (size_t)(i / kFwdChunk) * B_pad * kFwdChunk + i % kFwdChunk;
  for (int t = 0; t < n; ++t) ct[col[(size_t)(b0 + t) * kFwdChunk]]++;
  int run = 0;
  for (int k = 0; k < q; ++k) {
    const int v = ct[k];
    ct[k] = (uint16_t)run;
    run += v;
  }
  uint16_t* out = sorted + ((size_t)c * N + i) * kBwdSeqChunk;
  for (int t = 0; t < n; ++t) {
    const int k = col[(size_t)(b0 + t) * kFwdChunk];
    out[ct[k]++] = (uint16_t)((t << 8) | k);
  }
}

hipError_t launch_chunk_sort(const uint8_t* msa_cm, int32_t B3, int32_t B_pad, int32_t N, int32_t q,
                             uint16_t* sorted, hipStream_t st) {
  const int nchunks = (B3 + kBwdSeqChunk - 1) / kBwdSeqChunk;
  hipLaunchKernelGGL(chunk_sort_kernel, dim3(nchunks, (N + 255) / 256), dim3(256), 0, st, msa_cm,
                     B3, B_pad, N, q, sorted);
  return hipGetLastError();
}

// dJ_ri(s,k) = sum over the rows b with sigma_i^b = k of R_b(s).  Per chunk of
// 192 rows, the residual rows are staged in LDS (three bank-disjoint copies of
// each 21-float row, one per slot).  Each slot owns one column and walks the
// chunk's rows in symbol order, keeping a running FP32 sum in a register.  A
// symbol's rows are contiguous, so each group sum is final when the symbol
// changes and is stored (plain store, no read-back) into the column's slot for
// that symbol; after the chunk every lane folds its 21 slots into FP64
// registers and clears them.  No two lanes ever write the same LDS word.
// One LDS arena: residual rows first (so a row's byte offset is its address).
// Pitches chosen so that the three slots of a wave, which work on three
// consecutive columns, hit disjoint LDS banks: 200 entries (100 dwords) per
// column, and 469 = 7 * 64 + 21 floats per column of group sums.
constexpr int kEntPitch = kBwdSeqChunk + 8;
constexpr int kSegPitch = 7 * 64 + kSlot;
constexpr int kRsBytes = kBwdSeqChunk * kRowF * 4;              // 48 KB
constexpr int kEntBytes = kBwdPos * kEntPitch * 2;              // 19 KB
constexpr int kSegBytes = kBwdPos * kSegPitch * 4;              // 88 KB

// One backward work item: site r x the 48 alignment columns of block cb.
__device__ inline void bwd_item(const EvalArgs& a, int r, int cb, char* arena) {
  float* Rs = reinterpret_cast<float*>(arena);
  uint16_t* ent = reinterpret_cast<uint16_t*>(arena + kRsBytes);
  float* seg = reinterpret_cast<float*>(arena + kRsBytes + kEntBytes);
  const int q = a.q, N = a.N, qq = q * q;
  const int i0 = cb * kBwdPos;
  const int tid = item_tid(), lane = tid & 63, wid = tid >> 6;
  const int slot = lane / kSlot, s = lane - slot * kSlot;
  const int slotA = slot < kSlots ? slot : kSlots - 1;  // lane 63 shadows lane 42 and never writes
  const int pl = wid * kSlots + slotA;                   // this lane's column within the block
  const int i = i0 + pl;
  const bool writer = lane < kSlots * kSlot;
  const int npos = min(kBwdPos, N - i0);

  for (int e = tid; e < kBwdPos * kSegPitch; e += kBwdThreads) seg[e] = 0.f;
  double acc64[kQMax];
#pragma unroll
  for (int k = 0; k < kQMax; ++k) acc64[k] = 0.0;
  float* myseg = seg + pl * kSegPitch + s;                // + 21 * symbol
  const uint32_t lane_off = 4u * (uint32_t)(slotA * kSlot + s);
  const uint16_t* myent = ent + pl * kEntPitch;

  const int nchunks = (a.B3 + kBwdSeqChunk - 1) / kBwdSeqChunk;
  const auto Rr = gmem(a.R + (size_t)r * a.B3 * kSlot);
  for (int c = 0; c < nchunks; ++c) {
    const int bc = c * kBwdSeqChunk, n = min(kBwdSeqChunk, a.B3 - bc);
    __syncthreads();
    for (int e = tid; e < n * kSlot; e += kBwdThreads) {
      const int t = e / kSlot, ss = e - t * kSlot;
      const float v = Rr[(size_t)bc * kSlot + e];
      float* row = Rs + t * kRowF;
      row[ss] = v;
      row[ss + kSlot] = v;
      row[ss + 2 * kSlot] = v;
    }
    {
      constexpr int kV = kBwdSeqChunk / 8, kVP = kEntPitch / 8;   // uint4 per column: data, pitch
      const uint16_t* src = a.sorted + ((size_t)c * N + i0) * kBwdSeqChunk;
      uint4* dst = reinterpret_cast<uint4*>(ent);
      for (int e = tid; e < kBwdPos * kV; e += kBwdThreads) {
        const int col = e / kV, x = e - col * kV;
        dst[col * kVP + x] = col < npos ? gload_u4(src + 8 * (size_t)e) : make_uint4(0, 0, 0, 0);
      }
    }
    __syncthreads();
    uint32_t cur = myent[0] & 0xffu;
    float run = 0.f;
    auto rowval = [&](uint32_t e) {
      return *reinterpret_cast<const float*>(arena + ((e & 0xff00u) | lane_off));
    };
    int j = 0;
    for (; j + 8 <= n; j += 8) {
      // eight sorted entries at once; they all continue the current group
      // exactly when the last one does, since symbols ascend within the chunk
      const uint4 e8 = *reinterpret_cast<const uint4*>(myent + j);
      const uint32_t e[8] = {e8.x & 0xffffu, e8.x >> 16, e8.y & 0xffffu, e8.y >> 16,
                             e8.z & 0xffffu, e8.z >> 16, e8.w & 0xffffu, e8.w >> 16};
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = rowval(e[u]);
      if ((e[7] & 0xffu) == cur) {
        run += ((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]));
      } else {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const uint32_t sg = e[u] & 0xffu;
          if (sg != cur) {
            if (writer) myseg[cur * kQMax] = run;
            run = 0.f;
            cur = sg;
          }
          run += v[u];
        }
      }
    }
    for (; j < n; ++j) {
      const uint32_t e = myent[j];
      const uint32_t sg = e & 0xffu;
      const float v = rowval(e);
      if (sg != cur) {
        if (writer) myseg[cur * kQMax] = run;
        run = 0.f;
        cur = sg;
      }
      run += v;
    }
    if (writer) myseg[cur * kQMax] = run;
    // fold this chunk's group sums (the lane's own words) into FP64
#pragma unroll
    for (int k = 0; k < kQMax; ++k) {
      acc64[k] += (double)myseg[k * kQMax];
      if (writer) myseg[k * kQMax] = 0.f;
    }
  }
  if (writer && s < q && i < N) {
#pragma unroll
    for (int k = 0; k < kQMax; ++k)
      if (k < q) a.gJ[((size_t)r * N + i) * qq + (size_t)k * q + s] = (i == r) ? 0.0 : acc64[k];
  }
}

// Persistent backward kernel: drains the backward work items of the batch.
__global__ __launch_bounds__(kBwdThreads) void bwd_kernel(BatchArgs b) {
  __shared__ __attribute__((aligned(16))) char arena[kRsBytes + kEntBytes + kSegBytes];
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
    bwd_item(a, it.r, it.sub, arena);
    __syncthreads();
  }
}

int32_t backward_blocks_per_site(int32_t N) { return (N + kBwdPos - 1) / kBwdPos; }

int32_t backward_resident_blocks() {
  int per = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, bwd_kernel, kBwdThreads, 0);
  return (e == hipSuccess && per > 0) ? per : 1;
}

hipError_t launch_backward(const BatchArgs& b, int32_t nblocks, hipStream_t st) {
  hipLaunchKernelGGL(bwd_kernel, dim3(nblocks), dim3(kBwdThreads), 0, st, b);
  return hipGetLastError();
}

}  // namespace plm
