// k_fit.hip -- small kernels around the evaluation and optimiser kernels:
// fit initialisation, active-site compaction, the standalone objective /
// gradient finalisation (adds the l2 terms of eq. g_regdef2 and their
// derivatives, eqs. g_gradh2 / g_gradJ2), and input checks.
#include <string.h>

#include "plm_internal.h"

namespace plm {

// Zero the self blocks of the start point, copy it to the trial buffers and
// reset every site's optimiser state (one alignment; st and phase_host point
// at its first site).
__global__ void init_fit_kernel(int32_t N, int32_t q, float* Xh, float* XJ, float* Th, float* TJ,
                                SiteState* st, int32_t* phase_host) {
  const int r = blockIdx.x;
  const size_t qq = (size_t)q * q, Nqq = (size_t)N * qq;
  for (size_t e = threadIdx.x; e < qq; e += blockDim.x) XJ[(size_t)r * Nqq + (size_t)r * qq + e] = 0.f;
  __syncthreads();
  for (size_t e = threadIdx.x; e < Nqq; e += blockDim.x) TJ[(size_t)r * Nqq + e] = XJ[(size_t)r * Nqq + e];
  for (int e = threadIdx.x; e < q; e += blockDim.x) Th[(size_t)r * q + e] = Xh[(size_t)r * q + e];
  if (threadIdx.x == 0) {
    SiteState s;
    s.phase = PH_INIT;
    s.status = PLM_SITE_MAXITER;
    s.iter = s.evals = s.ls_count = s.head = s.stored = s.dpend = s.action = s.pad2 = 0;
    s.f = s.gnorm = s.alpha = s.gtd = 0.0;
    s.gamma = 1.0;
    st[r] = s;
    if (phase_host) phase_host[r] = PH_INIT;
  }
}

// Work-item offsets of every alignment from the active-list runs in b.seg
// (an item covers kind_group consecutive sites of a run), and cleared queue
// counters (one block; after the runs are written).
__device__ inline void finish_tables(const BatchArgs& b) {
  __syncthreads();
  if (threadIdx.x < 2 * kQueues) b.ctr[threadIdx.x] = 0u;
  if (threadIdx.x < 2) {
    const int kind = threadIdx.x;
    int32_t* off = b.item_off + kind * (b.n_msas + 1);
    const int32_t grp = kind_group(b, kind);
    int32_t acc = 0;
    for (int m = 0; m < b.n_msas; ++m) {
      off[m] = acc;
      acc += (b.seg[m + 1] - b.seg[m] + grp - 1) / grp * b.nsub[kind * b.n_msas + m];
    }
    off[b.n_msas] = acc;
  }
}

// Active list = sites not done, in global order, with the run of each
// alignment and the work-item tables for the next evaluation; the count also
// goes to pinned host memory, and the running total of site evaluations (the
// sites active in the iteration just finished) is kept.
__global__ void compact_kernel(BatchArgs b, const SiteState* st, int32_t* host_count,
                               unsigned long long* site_evals) {
  __shared__ int32_t flags[1024];
  __shared__ int32_t base;
  if (threadIdx.x == 0) {
    if (site_evals) *site_evals += (unsigned long long)*b.n_active;
    base = 0;
  }
  __syncthreads();
  for (int g0 = 0; g0 < b.total_sites; g0 += 1024) {
    const int g = g0 + threadIdx.x;
    const int act = (g < b.total_sites && st[g].phase != PH_DONE) ? 1 : 0;
    flags[threadIdx.x] = act;
    __syncthreads();
    // inclusive scan (Hillis-Steele) over the 1024 flags
    for (int o = 1; o < 1024; o <<= 1) {
      const int v = threadIdx.x >= o ? flags[threadIdx.x - o] : 0;
      __syncthreads();
      flags[threadIdx.x] += v;
      __syncthreads();
    }
    const int excl = base + flags[threadIdx.x] - act;
    if (act) b.active[excl] = g;
    if (g < b.total_sites) {
      const int m = b.msa_of[g];
      if (g == b.site_base[m]) b.seg[m] = excl;
    }
    __syncthreads();
    if (threadIdx.x == 0) base += flags[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    *b.n_active = base;
    b.seg[b.n_msas] = base;
    if (host_count) *host_count = base;
  }
  finish_tables(b);
}

// Clear the queue counters of one kind, so that a second launch of that
// kind's persistent kernel drains the same work items again.
__global__ void reset_queues_kernel(BatchArgs b, int32_t kind) {
  if (threadIdx.x < kQueues) b.ctr[kind * kQueues + threadIdx.x] = 0u;
}

hipError_t launch_reset_queues(const BatchArgs& b, int32_t kind, hipStream_t st) {
  hipLaunchKernelGGL(reset_queues_kernel, dim3(1), dim3(64), 0, st, b, kind);
  return hipGetLastError();
}

// Tables of a one-alignment batch over an explicit site list (list[j], or
// first + j when list is null).  Site indices outside [0, N) are replaced by
// 0 and raise bit 4 of *flag.
__global__ void list_tables_kernel(BatchArgs b, const int32_t* list, int32_t first, int32_t n,
                                   int32_t* flag) {
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    int32_t v = list ? list[j] : first + j;
    if (v < 0 || v >= b.total_sites) {
      if (flag) atomicOr(flag, 4);
      v = 0;
    }
    b.active[j] = v;
  }
  if (threadIdx.x == 0) {
    *b.n_active = n;
    b.seg[0] = 0;
    b.seg[1] = n;
  }
  finish_tables(b);
}

__global__ __launch_bounds__(1024) void objgrad_final_kernel(FinalArgs a) {
  __shared__ double red[16];
  const int r = a.sites ? a.sites[blockIdx.x] : blockIdx.x;
  const int q = a.q, N = a.N;
  const size_t qq = (size_t)q * q, Nqq = (size_t)N * qq;
  const double beff = *a.beff;
  const double sc = a.grad_scale ? a.grad_scale[r] : 1.0;
  double reg = 0.0;
  for (size_t e = threadIdx.x; e < Nqq; e += blockDim.x) {
    const size_t i = e / qq;
    const double v = (double)a.J[(size_t)r * Nqq + e];
    if (i != (size_t)r) reg += a.lambda_Jp * v * v;
    if (a.gJ_out)
      a.gJ_out[(size_t)r * Nqq + e] =
          (i == (size_t)r) ? 0.f
                           : (float)(sc * (a.gJ[(size_t)r * Nqq + e] + 2.0 * beff * a.lambda_Jp * v));
  }
  if (threadIdx.x < (unsigned)q) {
    const int s = threadIdx.x;
    const double v = (double)a.h[(size_t)r * q + s];
    reg += a.lambda_h * v * v;
    if (a.gh_out) {
      double t = 0.0;
      for (int k = 0; k < a.tiles; ++k) t += a.gh_part[((size_t)k * N + r) * kSlot + s];
      a.gh_out[(size_t)r * q + s] = (float)(sc * (t + 2.0 * beff * a.lambda_h * v));
    }
  }
  reg = block_sum_f64(reg, red);
  if (threadIdx.x == 0) {
    double f = 0.0;
    for (int k = 0; k < a.tiles; ++k) f += a.f_part[(size_t)k * N + r];
    a.f_out[r] = f + beff * reg;
  }
}

hipError_t launch_objgrad_final(const FinalArgs& a, int32_t nsites, hipStream_t st) {
  hipLaunchKernelGGL(objgrad_final_kernel, dim3(nsites), dim3(1024), 0, st, a);
  return hipGetLastError();
}

template <typename T>
__global__ void nonfinite_kernel(const T* p, size_t n, int32_t* flag) {
  int bad = 0;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x)
    if (!isfinite(p[e])) bad = 1;
  if (bad) atomicOr(flag, 2);
}

hipError_t launch_check_f32(const float* p, size_t n, int32_t* flag, hipStream_t st) {
  if (n == 0) return hipSuccess;
  size_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(nonfinite_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, st, p, n, flag);
  return hipGetLastError();
}

hipError_t launch_check_f64(const double* p, size_t n, int32_t* flag, hipStream_t st) {
  if (n == 0) return hipSuccess;
  size_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(nonfinite_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, st, p, n, flag);
  return hipGetLastError();
}

// Descriptors of alignment m of a batch (one thread block; host data travels
// as kernel arguments).  lb may be absent (evaluation only).  Alignment 0 also
// clears the active count and the evaluation counter.
__global__ void setup_msa_kernel(BatchArgs b, int32_t m, EvalArgs e, LbfgsArgs l, int32_t has_l,
                                 int32_t base, int32_t N, int32_t nsub_f, int32_t nsub_b,
                                 unsigned long long* site_evals) {
  for (int j = threadIdx.x; j < N; j += blockDim.x) const_cast<int32_t*>(b.msa_of)[base + j] = m;
  if (threadIdx.x == 0) {
    const_cast<EvalArgs*>(b.ev)[m] = e;
    if (has_l) const_cast<LbfgsArgs*>(b.lb)[m] = l;
    int32_t* sb = const_cast<int32_t*>(b.site_base);
    sb[m] = base;
    if (m == b.n_msas - 1) sb[b.n_msas] = base + N;
    int32_t* ns = const_cast<int32_t*>(b.nsub);
    ns[KIND_FWD * b.n_msas + m] = nsub_f;
    ns[KIND_BWD * b.n_msas + m] = nsub_b;
    if (m == 0) {
      *b.n_active = 0;
      if (site_evals) *site_evals = 0ull;
    }
  }
}

hipError_t launch_setup_msa(const BatchArgs& b, int32_t m, const EvalArgs& e, const LbfgsArgs* l,
                            int32_t base, int32_t N, int32_t nsub_f, int32_t nsub_b,
                            unsigned long long* site_evals, hipStream_t st) {
  LbfgsArgs lz;
  if (l) lz = *l; else memset(&lz, 0, sizeof(lz));
  hipLaunchKernelGGL(setup_msa_kernel, dim3(1), dim3(256), 0, st, b, m, e, lz, l ? 1 : 0, base, N,
                     nsub_f, nsub_b, site_evals);
  return hipGetLastError();
}

hipError_t launch_init_fit(int32_t N, int32_t q, float* Xh, float* XJ, float* Th, float* TJ,
                           SiteState* st_, int32_t* phase_host, hipStream_t st) {
  hipLaunchKernelGGL(init_fit_kernel, dim3(N), dim3(1024), 0, st, N, q, Xh, XJ, Th, TJ, st_, phase_host);
  return hipGetLastError();
}

hipError_t launch_compact(const BatchArgs& b, const SiteState* st_, int32_t* host_count,
                          unsigned long long* site_evals, hipStream_t st) {
  hipLaunchKernelGGL(compact_kernel, dim3(1), dim3(1024), 0, st, b, st_, host_count, site_evals);
  return hipGetLastError();
}

hipError_t launch_list_tables(const BatchArgs& b, const int32_t* list, int32_t first, int32_t n,
                              int32_t* flag, hipStream_t st) {
  hipLaunchKernelGGL(list_tables_kernel, dim3(1), dim3(256), 0, st, b, list, first, n, flag);
  return hipGetLastError();
}


// Convergence probe: kProbeChunks blocks per watched site take the largest
// |iterate - reference| over their range of the site's fields and couplings
// (the self block left out) into entry *count of out (as float bits, an
// atomic maximum over the non-negative values, NaN above every number); then
// probe_finish_kernel writes the entry's time (device wall clock) and the
// largest of the per-site maxima and advances the count.  Entries past cap
// are dropped.
constexpr int kProbeThreads = 256;
constexpr int kProbeChunks = 32;

__device__ inline uint32_t* probe_slot(const ProbeArgs& p, int32_t idx, int k) {
  return reinterpret_cast<uint32_t*>(p.out + (size_t)idx * (2 + p.n) + 2 + k);
}

__global__ void probe_zero_kernel(ProbeArgs p) {
  const int32_t idx = *p.count;
  if (idx >= p.cap) return;
  for (int k = threadIdx.x; k < p.n; k += blockDim.x) p.out[(size_t)idx * (2 + p.n) + 2 + k] = 0.0;
}

__global__ __launch_bounds__(kProbeThreads) void probe_site_kernel(ProbeArgs p) {
  __shared__ float red[kProbeThreads / 64];
  const int k = blockIdx.x / kProbeChunks, chunk = blockIdx.x - k * kProbeChunks;
  const int32_t idx = *p.count;
  if (idx >= p.cap) return;
  const int r = p.sites[k];
  if (r < 0 || r >= p.N) {  // not a site of the alignment
    if (threadIdx.x == 0 && chunk == 0) atomicMax(probe_slot(p, idx, k), 0x7fc00000u);
    return;
  }
  const int q = p.q;
  const int Nqq = p.N * q * q, P = q + Nqq;
  const int self0 = q + r * q * q, self1 = self0 + q * q;
  const int csz = (P + kProbeChunks - 1) / kProbeChunks;
  const int beg = min(P, chunk * csz), end = min(P, beg + csz);
  const float* X = p.XJ + (size_t)r * Nqq;
  const float* R = p.ref_J + (size_t)k * Nqq;
  float mx = 0.f;
  for (int e = beg + (int)threadIdx.x; e < end; e += kProbeThreads) {
    float d;
    if (e < q) d = fabsf(p.Xh[(size_t)r * q + e] - p.ref_h[(size_t)k * q + e]);
    else d = (e >= self0 && e < self1) ? 0.f : fabsf(X[e - q] - R[e - q]);
    mx = (d != d || mx != mx) ? __builtin_nanf("") : fmaxf(mx, d);
  }
  for (int o = 32; o > 0; o >>= 1) {
    const float u = __shfl_xor(mx, o, 64);
    mx = (u != u || mx != mx) ? __builtin_nanf("") : fmaxf(mx, u);
  }
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    float t = red[0];
    for (int w = 1; w < kProbeThreads / 64; ++w) t = (red[w] != red[w] || t != t) ? __builtin_nanf("") : fmaxf(t, red[w]);
    // non-negative floats and the positive quiet NaN order as their bit patterns
    atomicMax(probe_slot(p, idx, k), t != t ? 0x7fc00000u : __float_as_uint(t));
  }
}

__global__ void probe_finish_kernel(ProbeArgs p) {
  if (threadIdx.x != 0) return;
  const int32_t idx = *p.count;
  if (idx >= p.cap) return;
  double* e = p.out + (size_t)idx * (2 + p.n);
  double mx = 0.0;
  bool bad = false;
  for (int k = 0; k < p.n; ++k) {
    const float v = __uint_as_float(*probe_slot(p, idx, k));
    e[2 + k] = (double)v;
    bad = bad || !(v == v);
    mx = fmax(mx, (double)v);
  }
  e[0] = (double)wall_clock64() * p.sec_per_tick;
  e[1] = bad ? __builtin_nan("") : mx;
  *p.count = idx + 1;
}

hipError_t launch_probe(const ProbeArgs& p, hipStream_t st) {
  if (p.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(probe_zero_kernel, dim3(1), dim3(64), 0, st, p);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(probe_site_kernel, dim3(p.n * kProbeChunks), dim3(kProbeThreads), 0, st, p);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(probe_finish_kernel, dim3(1), dim3(64), 0, st, p);
  return hipGetLastError();
}

}  // namespace plm
