// plm_internal.h -- shared definitions of libplm's HIP sources (gfx950 only).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

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

// Forward kernel: 16 waves, 16 alignment columns staged per LDS chunk.
constexpr int kFwdWaves = 16;
constexpr int kFwdThreads = kFwdWaves * 64;
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
  int32_t pad;
  double f;            // normalised objective at the current point
  double gnorm;
  double alpha;        // step of the pending trial point
  double gtd;          // g' d at the current point
  double gamma;        // initial inverse-Hessian scale
  double rho[kMMax];
  double ahist[kMMax];
};

enum { PH_INIT = 0, PH_LS = 1, PH_DONE = 2 };

// Everything the evaluation kernels need about one alignment.
struct EvalArgs {
  const uint8_t* msa_cm;   // padded symbols, chunk-major: (b, i) at ((i/16)*B_pad + b)*16 + i%16
  const uint8_t* msaT;     // padded symbols, position-major: (b, i) at i*B_pad + b (MFMA paths)
  int32_t B, B3, B_pad, N, N_pad, q;
  const double* w;         // [B]
  const float* h;          // [N][q]  (trial point)
  const float* J;          // [N][N][q][q]
  const int32_t* sites;    // active site list
  const int32_t* n_active; // device count (nullable: then n_active_host)
  int32_t n_active_host;
  float* R;                // [N][B3][21] residuals w_b (P_b(s) - [sigma_r = s])
  double* f_part;          // [tiles][N]
  double* gh_part;         // [tiles][N][21]
  double* gJ;              // [N][N][q][q] data part of d f / d J (FP64)
  int32_t tiles;
  const uint16_t* sorted;  // [nchunks][N][kBwdSeqChunk]: (row << 8) | symbol, rows sorted by symbol
};


// Arguments of the optimiser kernel (one block per site).
struct LbfgsArgs {
  int32_t N, q, m, max_iter, max_ls, tiles;
  double tol, lambda_h, lambda_Jp, c1, noise;
  const double* beff;
  float* Xh;
  float* XJ;
  float* Th;
  float* TJ;
  double* Gh;
  double* GJ;
  double* Dh;
  double* DJ;
  double* Sh;  // [m][N][q]
  double* SJ;  // [m][N][N q q]
  double* Yh;
  double* YJ;
  const double* f_part;   // [tiles][N]
  const double* gh_part;  // [tiles][N][21]
  const double* gJ;       // [N][N][q][q] data part
  SiteState* st;
  int32_t* phase_host;    // pinned mirror of each site's phase (nullable)
  int32_t site_offset;    // block b handles site site_offset + b
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
hipError_t launch_pad_msa(const uint8_t* msa, int32_t B, int32_t N, int32_t q, uint8_t* msa_cm,
                          int32_t B_pad, int32_t N_pad, int32_t* flag_dev, hipStream_t st);
hipError_t launch_forward(const EvalArgs& a, int32_t n_sites_grid, int32_t nb, hipStream_t st);
hipError_t launch_backward(const EvalArgs& a, int32_t n_sites_grid, hipStream_t st);
hipError_t launch_transpose_msa(const uint8_t* msa_cm, int32_t B_pad, int32_t N_pad, uint8_t* msaT,
                                hipStream_t st);
int32_t mfma_forward_tile_seqs();
hipError_t launch_forward_mfma(const EvalArgs& a, int32_t n_sites_grid, int32_t npieces,
                               hipStream_t st);
hipError_t launch_backward_mfma(const EvalArgs& a, int32_t n_sites_grid, int32_t npieces,
                                hipStream_t st);
hipError_t launch_chunk_sort(const uint8_t* msa_cm, int32_t B3, int32_t B_pad, int32_t N, int32_t q,
                             uint16_t* sorted, hipStream_t st);
int32_t forward_tile_seqs(int32_t nb);
hipError_t launch_lbfgs(const LbfgsArgs& a, int32_t nblocks, hipStream_t st);
hipError_t launch_reweight(const uint8_t* msa, int32_t B, int32_t N, int32_t q, double theta,
                           int32_t uniform, int32_t* m, double* w, double* beff, int32_t* flag,
                           hipStream_t st);
hipError_t launch_score(const float* J, int32_t N, int32_t q, double* fn, double* cfn, hipStream_t st);
hipError_t launch_objgrad_final(const FinalArgs& a, int32_t nsites, hipStream_t st);
hipError_t launch_check_f32(const float* p, size_t n, int32_t* flag, hipStream_t st);
hipError_t launch_check_f64(const double* p, size_t n, int32_t* flag, hipStream_t st);
hipError_t launch_init_fit(int32_t N, int32_t q, float* Xh, float* XJ, float* Th, float* TJ,
                           SiteState* st_, int32_t* sites, int32_t* n_active, int32_t* phase_host,
                           hipStream_t st);
hipError_t launch_compact(int32_t N, const SiteState* st_, int32_t* sites, int32_t* n_active,
                          int32_t* host_count, unsigned long long* site_evals, hipStream_t st);
hipError_t launch_zero_u64(unsigned long long* p, hipStream_t st);

}  // namespace plm
