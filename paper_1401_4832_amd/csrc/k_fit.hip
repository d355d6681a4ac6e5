// k_fit.hip -- small kernels around the evaluation and optimiser kernels:
// fit initialisation, active-site compaction, the standalone objective /
// gradient finalisation (adds the l2 terms of eq. g_regdef2 and their
// derivatives, eqs. g_gradh2 / g_gradJ2), and input checks.
#include "plm_internal.h"

namespace plm {

// Zero the self blocks of the start point, copy it to the trial buffers and
// reset every site's optimiser state; the active list is all sites.
__global__ void init_fit_kernel(int32_t N, int32_t q, float* Xh, float* XJ, float* Th, float* TJ,
                                SiteState* st, int32_t* sites, int32_t* n_active,
                                int32_t* phase_host) {
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
    s.iter = s.evals = s.ls_count = s.head = s.stored = s.pad = 0;
    s.f = s.gnorm = s.alpha = s.gtd = 0.0;
    s.gamma = 1.0;
    for (int k = 0; k < kMMax; ++k) s.rho[k] = s.ahist[k] = 0.0;
    st[r] = s;
    sites[r] = r;
    if (phase_host) phase_host[r] = PH_INIT;
    if (r == 0) *n_active = N;
  }
}

// Active list = sites not done, in increasing order; the count also goes to
// pinned host memory, and the running total of site evaluations is kept.
__global__ void compact_kernel(int32_t N, const SiteState* st, int32_t* sites, int32_t* n_active,
                               int32_t* host_count, unsigned long long* site_evals) {
  __shared__ int32_t flags[1024];
  __shared__ int32_t base;
  if (threadIdx.x == 0) {
    *site_evals += (unsigned long long)*n_active;  // the sites evaluated in this iteration
    base = 0;
  }
  __syncthreads();
  for (int r0 = 0; r0 < N; r0 += 1024) {
    const int r = r0 + threadIdx.x;
    const int act = (r < N && st[r].phase != PH_DONE) ? 1 : 0;
    flags[threadIdx.x] = act;
    __syncthreads();
    // inclusive scan (Hillis-Steele) over the 1024 flags
    for (int o = 1; o < 1024; o <<= 1) {
      const int v = threadIdx.x >= o ? flags[threadIdx.x - o] : 0;
      __syncthreads();
      flags[threadIdx.x] += v;
      __syncthreads();
    }
    if (act) sites[base + flags[threadIdx.x] - 1] = r;
    __syncthreads();
    if (threadIdx.x == 0) base += flags[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    *n_active = base;
    if (host_count) *host_count = base;
  }
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

hipError_t launch_init_fit(int32_t N, int32_t q, float* Xh, float* XJ, float* Th, float* TJ,
                           SiteState* st_, int32_t* sites, int32_t* n_active, int32_t* phase_host,
                           hipStream_t st) {
  hipLaunchKernelGGL(init_fit_kernel, dim3(N), dim3(1024), 0, st, N, q, Xh, XJ, Th, TJ, st_, sites,
                     n_active, phase_host);
  return hipGetLastError();
}

hipError_t launch_compact(int32_t N, const SiteState* st_, int32_t* sites, int32_t* n_active,
                          int32_t* host_count, unsigned long long* site_evals, hipStream_t st) {
  hipLaunchKernelGGL(compact_kernel, dim3(1), dim3(1024), 0, st, N, st_, sites, n_active,
                     host_count, site_evals);
  return hipGetLastError();
}

__global__ void zero_u64_kernel(unsigned long long* p) { *p = 0ull; }
hipError_t launch_zero_u64(unsigned long long* p, hipStream_t st) {
  hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(1), 0, st, p);
  return hipGetLastError();
}

}  // namespace plm
