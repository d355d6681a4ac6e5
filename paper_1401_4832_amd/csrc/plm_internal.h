// plm_internal.h -- shared definitions of libplm's HIP sources (gfx950 only).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <type_traits>

#include "plm.h"

namespace plm {

// Lane layout of the per-site kernels: a wave64 is three 21-lane slots; slot c
// lane s works on state s of one sequence (lane 63 idles).  LDS rows hold 64
// floats: three copies of a 21-float row at offsets 0, 21, 42, so that the
// three slots of a wave, which read rows picked by three different sequences,
// always touch disjoint LDS banks.
constexpr int kSlot = 21;
constexpr int kSlots = 3;
constexpr int kRowF = 64;
constexpr int kQMax = 21;
constexpr int kMMax = 32;  // L-BFGS history cap

// Forward kernel: 8 waves, 16 alignment columns per symbol chunk.
constexpr int kFwdWaves = 8;
constexpr int kFwdThreads = kFwdWaves * 64;
// Row padding of every alignment: a multiple of every forward tile (the
// gather tiles of 16, 32 or 64 rows per wave and the 1024-row MFMA tile) and
// of the 256-row gradient chunk, so that no tile or chunk reads past it.
constexpr int kBPadUnit = 3072;
static_assert(kBPadUnit % (kFwdWaves * kSlots * 64) == 0 && kBPadUnit % 256 == 0, "row padding");
constexpr int kFwdChunk = 16;
// Backward kernel: 16 waves; the three slots of a wave own three different
// alignment columns (48 per block).  Sequences are processed in chunks of 192
// whose rows are sorted by symbol at every column (once per alignment).
constexpr int kBwdWaves = 16;
constexpr int kBwdThreads = kBwdWaves * 64;
constexpr int kBwdPos = kBwdWaves * kSlots;  // 48
constexpr int kBwdSeqChunk = 192;

// Per-site optimiser state (device).
struct SiteState {
  int32_t phase;       // 0 first evaluation pending, 1 line search, 2 done
  int32_t status;      // PLM_SITE_*
  int32_t iter;
  int32_t evals;
  int32_t ls_count;
  int32_t head;
  int32_t stored;
  int32_t dpend;       // direction pending for the direction kernels: 1 quasi-Newton (DirCoef), 2 steepest
  int32_t action;      // what the update pass does with the decision just taken
  int32_t pad2;
  double f;            // normalised objective at the current point
  double gnorm;
  double alpha;        // step of the pending trial point
  double gtd;          // g' d at the current point
  double gamma;        // initial inverse-Hessian scale
};

enum { PH_INIT = 0, PH_LS = 1, PH_DONE = 2 };

// The quasi-Newton direction d = -gamma g + sum_i (cs_i s_i + cy_i y_i) of
// one site, over its stored pairs in chronological order (slots ord), as
// computed by the L-BFGS step and formed by the direction kernels.
constexpr int kLbChunks = 32;   // blocks per site of the optimiser's passes over a site's parameters
constexpr int kLbPartW = 4 + 2 * kMMax;  // FP64 partial sums per (site, block)
struct DirCoef {
  int32_t n;
  int32_t pad;
  double gamma;
  double cs[kMMax];
  double cy[kMMax];
  int32_t ord[kMMax];
};

// Everything the evaluation kernels need about one alignment.
struct EvalArgs {
  const uint8_t* msa_cm;   // padded symbols, chunk-major: (b, i) at ((i/16)*B_pad + b)*16 + i%16
  const uint8_t* msaT;     // padded symbols, position-major: (b, i) at i*B_pad + b (MFMA paths)
  int32_t B, B3, B_pad, N, N_pad, q;
  const double* w;         // [B]
  const float* h;          // [N][q]  (trial point)
  const float* J;          // [N][N][q][q]
  float* R;                // [N][B3][21] residuals w_b (P_b(s) - [sigma_r = s])
  double* f_part;          // [tiles][N]
  double* gh_part;         // [tiles][N][21]
  double* gJ;              // [N][N][q][q] data part of d f / d J (FP64)
  int32_t tiles;
  int32_t rfrag;           // R in gradient-fragment order: 1 FP16 hi/lo pieces, 2 int8 digits, 3 two int8 digit
                           // sets (R and its remainder; the second set after N * B_pad/256 chunks; see below)
  const uint16_t* sorted;  // [nchunks][N][kBwdSeqChunk]: (row << 8) | symbol, rows sorted by symbol
  // int8 forward (path 6): couplings as fixed-point digits, symbols by position triple
  int8_t* Wq;              // [N][NG][3 digits][2 steps][2 halves][21 states][16] bytes
  int32_t* jexp;           // [N] scale exponent: digits of round(J * 2^jexp); then [N][kJParts] partial maxima
  const uint32_t* sym3;    // [NG][B_pad] symbols of positions 3G, 3G+1, 3G+2 (bytes 0..2)
  int32_t NG;              // position triples, ceil(N / 3)
  int32_t pad_;
  // low-order words of the evaluation point (the point is h + h_lo, J + J_lo,
  // summed in FP64); read only by the precise forward's low-word instance
  const float* h_lo;       // [N][q] or null
  const float* J_lo;       // [N][N][q][q] or null
};

// Residuals in gradient-fragment order (rfrag = 1): R_b(s) * kRfScale split
// into FP16 hi and lo pieces, stored per site as [chunk of 256 sequences]
// [piece][step of 16][half of 8][state 0..20][sequence 0..7] (16-bit words):
// each (chunk, site) is 21504 contiguous bytes, copied into LDS as is by the
// grouped MFMA gradient.  Covers B_pad rows per site.
constexpr float kRfScale = 4096.f;
constexpr int kRfChunk = 256;
constexpr int kRfPieceWords = 16 * 2 * kSlot * 8;          // 5376
constexpr int kRfChunkBytes = 2 * kRfPieceWords * 2;       // 21504
__device__ inline size_t rfrag_index(int32_t r, int32_t nch, int32_t b, int32_t s) {
  const size_t c = (size_t)r * nch + (b >> 8);
  return ((((c * 2) * 16 + ((b >> 4) & 15)) * 2 + ((b >> 3) & 1)) * kSlot + s) * 8 + (b & 7);
}

// Residuals as fixed-point digits (rfrag = 2): v = round(R_b(s) * 2^22) (|R| <=
// w_b <= 1, so |v| <= 2^22) written as v = hi 2^16 + mid 2^8 + lo with signed
// int8 digits, stored per site as [chunk of 256][digit][step of 32][half of
// 16][state 0..20][sequence 0..15] bytes: 16128 contiguous bytes per (chunk,
// site).  Integer accumulation of the digits is exact.
constexpr int kRiScaleLog2 = 22;
constexpr int kRiDigitBytes = 8 * 2 * kSlot * 16;           // 5376
constexpr int kRiChunkBytes = 3 * kRiDigitBytes;            // 16128
__device__ inline size_t rifrag_index(int32_t r, int32_t nch, int32_t b, int32_t s) {
  const size_t c = (size_t)r * nch + (b >> 8);
  return ((((c * 3) * 8 + ((b >> 5) & 7)) * 2 + ((b >> 4) & 1)) * kSlot + s) * 16 + (b & 15);
}


// Arguments of the optimiser kernel (one block per site).
struct LbfgsArgs {
  int32_t N, q, m, max_iter, max_ls, tiles;
  double tol, lambda_h, lambda_Jp, c1, noise;
  const double* beff;
  float* Xh;
  float* XJ;
  float* Th;
  float* TJ;
  void* Gh;    // gradient at the iterate, FP32 or FP64 (the history type)
  void* GJ;
  float* Dh;   // search direction, FP32 (the step along it is rounded to FP32 anyway)
  float* DJ;
  void* Sh;    // [m+1][N][q] history slots (one spare for the candidate pair), FP32 or FP64
  void* SJ;    // [m+1][N][N q q]
  void* Yh;
  void* YJ;
  double* small;  // per site: [m+1][m+1] S^T Y, [m+1][m+1] Y^T Y, [m+1] S^T G, [m+1] Y^T G by slot
  DirCoef* dc;    // per site: the pending direction's coefficients
  double* dpart;  // per site: [kLbChunks] partial sums of d . g
  double* part;   // per site: [kLbChunks][kLbPartW] partial sums of the passes
  double* ghd;    // per site: [q] data part of the field gradient at the trial point
  const double* f_part;   // [tiles][N]
  const double* gh_part;  // [tiles][N][21]
  const double* gJ;       // [N][N][q][q] data part
  SiteState* st;
  int32_t* phase_host;    // pinned mirror of each site's phase (nullable)
};

// Arguments of the standalone objective/gradient finalisation.
struct FinalArgs {
  int32_t N, q, tiles;
  double lambda_h, lambda_Jp;
  const double* beff;
  const float* h;
  const float* J;
  const int32_t* sites;
  const double* f_part;
  const double* gh_part;
  const double* gJ;
  const double* grad_scale;  // nullable per-site gradient multiplier
  double* f_out;
  float* gh_out;
  float* gJ_out;
};

// A batch of alignments evaluated together (a single alignment is a batch of
// one).  Sites of all alignments get global ids, alignment by alignment in the
// batch order (largest cost first); the active list keeps that order.  Each
// evaluation kernel is persistent: its blocks drain work items (alignment,
// site, tile) from kQueues queues, each a contiguous range of the item order.
constexpr int kQueues = 8;
enum { KIND_FWD = 0, KIND_BWD = 1 };

struct BatchArgs {
  const EvalArgs* ev;        // [n_msas] evaluation descriptors (device)
  const LbfgsArgs* lb;       // [n_msas] optimiser descriptors (device; fit only)
  int32_t n_msas, total_sites;
  const int32_t* site_base;  // [n_msas + 1] first global site id of each alignment
  const int32_t* msa_of;     // [total_sites] alignment of each global site
  int32_t* active;           // [total_sites] active global site ids
  int32_t* n_active;         // device count of active sites
  int32_t* seg;              // [n_msas + 1] start of each alignment's run in the active list
  int32_t* item_off;         // [2][n_msas + 1] work-item offsets (forward, backward)
  const int32_t* nsub;       // [2][n_msas] work items per site (forward tiles, backward blocks)
  uint32_t* ctr;             // [2][kQueues] queue counters, cleared when the tables are built
  int32_t bwd_group;         // sites per gradient work item (consecutive in the active list)
  int32_t fwd_group;         // sites per forward work item
};

// sites per work item of a kind
__host__ __device__ inline int32_t kind_group(const BatchArgs& b, int kind) {
  return kind == KIND_BWD ? b.bwd_group : b.fwd_group;
}

// g, r: the first site of the item; first: its position in the active list;
// cnt: the item's sites (active[first .. first + cnt), one alignment)
struct Item {
  int32_t m, g, r, sub, first, cnt;
};

// Next work item of a persistent block (call from one thread).  The block
// starts on queue blockIdx % kQueues -- under round-robin dispatch, the queue
// of its XCD, so that consecutive items of one site share that XCD's L2 --
// and moves to the following queues when its own is empty.  qi counts the
// queues finished; -1 is returned once all are empty, so every block exits.
__device__ inline int32_t next_item(uint32_t* ctr, int32_t total, int32_t& qi) {
  while (qi < kQueues) {
    const int32_t x = (int32_t)((blockIdx.x + (uint32_t)qi) % kQueues);
    const int32_t lo = (int32_t)(((int64_t)total * x) / kQueues);
    const int32_t hi = (int32_t)(((int64_t)total * (x + 1)) / kQueues);
    if (lo < hi) {
      const int32_t k = (int32_t)atomicAdd(&ctr[x], 1u);
      if (lo + k < hi) return lo + k;
    }
    ++qi;
  }
  return -1;
}

// A descriptor read by a whole block, moved into scalar registers (every
// 32-bit word through readfirstlane), so that its fields cost no VGPRs.
template <class T>
__device__ inline T load_uniform(const T* p) {
  static_assert(sizeof(T) % 4 == 0, "descriptor size");
  T out;
  const uint32_t* src = reinterpret_cast<const uint32_t*>(p);
  uint32_t* dst = reinterpret_cast<uint32_t*>(&out);
#pragma unroll
  for (int k = 0; k < (int)(sizeof(T) / 4); ++k) dst[k] = __builtin_amdgcn_readfirstlane(src[k]);
  return out;
}

// A device pointer seen as global memory (descriptors loaded from memory lose
// the address space of their pointers; global loads can then address with a
// scalar base and a 32-bit lane offset).
template <class T>
__device__ inline const __attribute__((address_space(1))) T* gmem(const T* p) {
  return (const __attribute__((address_space(1))) T*)p;
}
template <class T>
__device__ inline __attribute__((address_space(1))) T* gmem_w(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}

// f(std::integral_constant<int, n>) for a runtime n in [K, Max] (n > Max runs
// Max): loops over a uniform count become straight-line code
template <int K, int Max, class F>
__device__ inline void with_count(int n, F&& f) {
  if constexpr (K >= Max) {
    f(std::integral_constant<int, Max>{});
  } else {
    if (n == K) f(std::integral_constant<int, K>{});
    else with_count<K + 1, Max>(n, f);
  }
}

typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2_t __attribute__((ext_vector_type(2)));
__device__ inline uint4 gload_u4(const void* p) {
  const u32x4_t v = *(const __attribute__((address_space(1))) u32x4_t*)p;
  return make_uint4(v.x, v.y, v.z, v.w);
}
__device__ inline uint2 gload_u2(const void* p) {
  const u32x2_t v = *(const __attribute__((address_space(1))) u32x2_t*)p;
  return make_uint2(v.x, v.y);
}

// threadIdx.x, opaque to the optimiser: the item bodies of the persistent
// kernels derive their per-lane offsets from it, so that those are recomputed
// per item instead of being hoisted out of the item loop (where they would
// occupy registers for the whole kernel).
// A wave-uniform address held in scalar registers (so that a copy takes the
// scalar base + 32-bit lane offset form)
template <typename T>
__device__ inline const T* uniform_ptr(const T* p) {
  const uint64_t v = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return reinterpret_cast<const T*>(((uint64_t)hi << 32) | lo);
}

// Global -> LDS copy of 16 bytes per lane: lane l moves src + 16 l to
// dst + 16 l, with src and dst uniform over the wave.  It is issued as a
// buffer load with an LDS destination rather than the global form: the
// compiler's wait-count pass takes the global (FLAT-encoded) form for a
// possible LDS access, and while such a copy is in flight it waits for every
// outstanding LDS read (lgkmcnt 0) where a use needs only the older ones.
// The buffer spans 2^31 - 1 bytes from src; offsets here stay below 1 KB.
__device__ inline void copy16_to_lds(const void* src, void* dst, int lane) {
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<char*>(uniform_ptr(static_cast<const char*>(src))), (short)0, 0x7fffffff, 0x00020000);
  __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (__attribute__((address_space(3))) void*)dst, 16, lane * 16, 0, 0,
                                           0);
}

__device__ inline int item_tid() {
  int t = (int)threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

__device__ inline int32_t total_items(const BatchArgs& b, int kind) {
  return b.item_off[kind * (b.n_msas + 1) + b.n_msas];
}

__device__ inline Item decode_item(const BatchArgs& b, int kind, int32_t t) {
  const int32_t* off = b.item_off + kind * (b.n_msas + 1);
  int32_t lo = 0, hi = b.n_msas - 1;  // last alignment whose first item is <= t
  while (lo < hi) {
    const int32_t mid = (lo + hi + 1) >> 1;
    if (off[mid] <= t) lo = mid; else hi = mid - 1;
  }
  Item it;
  it.m = lo;
  const int32_t ns = b.nsub[kind * b.n_msas + lo];
  const int32_t grp = kind_group(b, kind);
  const int32_t loc = t - off[lo];
  const int32_t j = loc / ns;
  it.sub = loc - j * ns;
  it.first = b.seg[lo] + j * grp;
  it.cnt = min(grp, b.seg[lo + 1] - it.first);
  it.g = b.active[it.first];
  it.r = it.g - b.site_base[lo];
  return it;
}

// Symmetric pseudolikelihood maximization: optimiser state and arguments.
struct SymState {
  int32_t phase, status, iter, evals, ls_count, head, stored;
  int32_t accept, pair, dir, move, pad;
  double f, gnorm, alpha, gtd, gamma;
};

struct SymCoef {
  double cs[kMMax], cy[kMMax];            // direction coefficients, chronological order
  double p1[kMMax + 1], p2[kMMax + 1];    // s_j . g, y_j . g, newest first
  double colS[kMMax + 1], colY[kMMax + 1];
  int32_t ord[kMMax];
  int32_t n;
};

struct SymArgs {
  int32_t N, q, m, max_iter, max_ls, tiles, nblk, npairs;
  double tol, lambda_h, lambda_J, c1, noise;
  const double* beff;
  float *Xh, *XJ, *Th, *TJ;  // iterate (caller's h, J) and trial point, couplings mirrored
  // low-order words of the iterate (caller's) and of the trial point, or null:
  // the parameters are then hi + lo, each pair summed in FP64
  float *Xhl, *XJl, *Thl, *TJl;
  double *Gh, *GJ, *Dh, *DJ;  // full-layout vectors, blocks r < i used
  float *Sh, *SJ, *Yh, *YJ;    // curvature pairs, FP32 (used as stored)
  const double *f_part, *gh_part, *gJ;            // evaluation of the trial point
  double* part;   // block partial sums
  double* small;  // [2][m+1][m+1] S^T Y, Y^T Y by slot
  SymCoef* coef;
  SymState* st;
  const int2* pairs;  // [npairs] (r, i), r < i
  int32_t* done_host;
};

// Convergence probe of plm_fit (plm_fit_opts.n_probe): the iterate of the
// watched sites against reference values, one entry per call.
struct ProbeArgs {
  int32_t N, q, n, cap;
  const float* Xh;      // iterate [N][q], [N][N][q][q]
  const float* XJ;
  const int32_t* sites;  // [n]
  const float* ref_h;   // [n][q]
  const float* ref_J;   // [n][N][q][q]
  double* out;          // [cap][2 + n]: time (s), max over sites, per site
  int32_t* count;
  double sec_per_tick;  // of wall_clock64()
};

// Options of the pair scores (PLM_COMBINE_*, PLM_NORM_*, PLM_CORR_*).
struct ScoreOpts {
  int32_t combine, norm;
  double p;
  int32_t exclude_gap, correction;
};

// Device helpers ----------------------------------------------------------
__device__ inline double block_sum_f64(double v, double* red) {
  // deterministic: fixed shuffle tree per wave, then waves summed in order
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double t = 0.0;
  for (int k = 0; k < nw; ++k) t += red[k];
  __syncthreads();
  return t;
}

// Host-side launchers -------------------------------------------------------
// The evaluation and optimiser kernels are persistent / per-site over a batch;
// nblocks is the grid (resident blocks for the persistent kernels).
hipError_t launch_pad_msa(const uint8_t* msa, int32_t B, int32_t N, int32_t q, uint8_t* msa_cm,
                          int32_t B_pad, int32_t N_pad, int32_t* flag_dev, hipStream_t st);
hipError_t launch_transpose_msa(const uint8_t* msa_cm, int32_t B_pad, int32_t N_pad, uint8_t* msaT,
                                hipStream_t st);
hipError_t launch_chunk_sort(const uint8_t* msa_cm, int32_t B3, int32_t B_pad, int32_t N, int32_t q,
                             uint16_t* sorted, hipStream_t st);
int32_t forward_tile_seqs(int32_t nb);
// f64: 0 FP32 accumulation, 1 FP64 (the precise path), 2 FP64 reading the
// low-order words of the point as well (EvalArgs.h_lo, J_lo)
int32_t forward_resident_blocks(int32_t nb, int32_t f64);
// f64: the precise path's forward (FP64 energies, log-softmax and residuals,
// residuals out as two int8 digit sets; its own tile of forward_f64_tile_seqs rows)
hipError_t launch_forward(const BatchArgs& b, int32_t nb, int32_t nblocks, int32_t f64, hipStream_t st);
int32_t forward_f64_tile_seqs();
int32_t backward_blocks_per_site(int32_t N);
int32_t backward_resident_blocks();
hipError_t launch_backward(const BatchArgs& b, int32_t nblocks, hipStream_t st);
int32_t mfma_forward_tile_seqs();
int32_t mfma_backward_blocks_per_site(int32_t N, int32_t q);
int32_t mfma_resident_blocks(int32_t kind, int32_t npieces);
// grouped FP16 hi/lo MFMA gradient (three sites per item, R in fragment order)
constexpr int kG3Sites = 3;
int32_t g3_backward_blocks_per_site(int32_t N, int32_t q);
int32_t g3_resident_blocks();
hipError_t launch_backward_g3(const BatchArgs& b, int32_t nblocks, hipStream_t st);
// zero the fragment-order residual rows [B rounded down to 256, B3 rounded up
// to 256) of every site: the forward writes only the rows of its tiles, and the
// last gradient chunk may reach past them
hipError_t launch_rfrag_tail_zero(float* R, int32_t N, int32_t B, int32_t B3, int32_t B_pad, int32_t chunk_bytes,
                                  hipStream_t st);
// int8 fixed-point MFMA forward (three sites per item; path 6)
constexpr int kWqGroupBytes = 3 * 2 * 2 * kSlot * 16;      // 4032 per (site, position triple)
constexpr int kJParts = 16;                                 // blocks per site of the coupling quantisation
int32_t fwd_i8_tile_seqs();
int32_t fwd_i8_resident_blocks();
hipError_t launch_sym3(const uint8_t* msa_cm, int32_t B_pad, int32_t N, int32_t NG, uint32_t* sym3, hipStream_t st);
// couplings of every active site to digits (jmax_kernel, jquant_kernel), then the int8 forward
hipError_t launch_jquant(const BatchArgs& b, int32_t total_sites, hipStream_t st);
hipError_t launch_fwd_i8(const BatchArgs& b, int32_t nblocks, hipStream_t st);
// grouped int8 fixed-point MFMA gradient (three sites per item, R as digits)
int32_t i8_backward_blocks_per_site(int32_t N, int32_t q);
int32_t i8_resident_blocks();
// lo: the second pass of the precise path (the remainder digits, added in)
hipError_t launch_backward_i8(const BatchArgs& b, int32_t nblocks, int32_t lo, hipStream_t st);
hipError_t launch_forward_mfma(const BatchArgs& b, int32_t npieces, int32_t nblocks, hipStream_t st);
hipError_t launch_backward_mfma(const BatchArgs& b, int32_t npieces, int32_t f16, int32_t nblocks,
                                hipStream_t st);
hipError_t launch_lbfgs(const BatchArgs& b, int32_t nblocks, int32_t history_fp64, hipStream_t st);
hipError_t launch_compact(const BatchArgs& b, const SiteState* st_, int32_t* host_count,
                          unsigned long long* site_evals, hipStream_t st);
hipError_t launch_reset_queues(const BatchArgs& b, int32_t kind, hipStream_t st);
hipError_t launch_list_tables(const BatchArgs& b, const int32_t* list, int32_t first, int32_t n,
                              int32_t* flag, hipStream_t st);
hipError_t launch_setup_msa(const BatchArgs& b, int32_t m, const EvalArgs& e, const LbfgsArgs* l,
                            int32_t base, int32_t N, int32_t nsub_f, int32_t nsub_b,
                            unsigned long long* site_evals, hipStream_t st);
hipError_t launch_init_fit(int32_t N, int32_t q, float* Xh, float* XJ, float* Th, float* TJ,
                           SiteState* st_, int32_t* phase_host, hipStream_t st);
hipError_t launch_sym_init(const SymArgs& a, hipStream_t st);
hipError_t launch_sym_step(const SymArgs& a, const BatchArgs& b, hipStream_t st);
int32_t sym_part_stride();
int32_t sym_groups(int32_t m);

// mean-field starting guess
int32_t mf_tile();
hipError_t launch_mf_frequencies(const uint8_t* msa, int32_t B, int32_t N, int32_t q, const double* w,
                                 const double* beff, double lam, int32_t* order, int32_t* start, double* fi,
                                 int32_t* flag, hipStream_t st);
hipError_t launch_mf_correlation(const uint8_t* msa, const int32_t* order, const int32_t* start, const double* w,
                                 const double* beff, const double* fi, int32_t B, int32_t N, int32_t q,
                                 double lam, double* C, int32_t n_pad, hipStream_t st);
hipError_t launch_mf_invert(double* C, int32_t n_pad, int32_t* flag, hipStream_t st);
hipError_t launch_mf_output(const double* Cinv, int32_t n_pad, const double* fi, int32_t N, int32_t q, float* h,
                            float* J, int32_t* flag, hipStream_t st);
hipError_t launch_reweight(const uint8_t* msa, int32_t B, int32_t N, int32_t q, double theta,
                           int32_t uniform, int32_t* m_out, double* w_out, double* beff_out,
                           int32_t* flag_dev, hipStream_t st);
hipError_t launch_score(const float* J, int32_t N, int32_t q, double* fn, double* cfn, hipStream_t st);
hipError_t launch_score_ex(const float* J, int32_t N, int32_t q, const ScoreOpts& o,
                           const double* freq, double* raw, double* cor, hipStream_t st);
hipError_t launch_frequencies(const uint8_t* msa, int32_t B, int32_t N, int32_t q, const double* w,
                              const double* beff, double* f, hipStream_t st);
hipError_t launch_objgrad_final(const FinalArgs& a, int32_t nsites, hipStream_t st);
hipError_t launch_check_f32(const float* p, size_t n, int32_t* flag, hipStream_t st);
hipError_t launch_probe(const ProbeArgs& p, hipStream_t st);
hipError_t launch_check_f64(const double* p, size_t n, int32_t* flag, hipStream_t st);

}  // namespace plm
