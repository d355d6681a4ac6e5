// plm_api.hip -- host side of the C ABI declared in include/plm.h.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <vector>

#include "plm_internal.h"

using namespace plm;

struct plm_ctx {
  int device;
  hipStream_t stream;
  char err[512];
  int32_t* pin;      // pinned host words: [0] error bits, [1] active count, [2..] per-site phase
  int32_t* pin_dev;  // device view of pin
  size_t pin_words;
  hipStream_t fit_stream;  // private stream of the synchronous fit (graph capture needs one)
  hipEvent_t ev[5];        // kernel timing marks of the fit iteration
  plm_fit_timing timing;   // of the last timed fit
};

namespace {

int set_err(plm_ctx* c, int code, const char* fmt, ...) {
  if (c) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(c->err, sizeof(c->err), fmt, ap);
    va_end(ap);
  }
  return code;
}

#define HIPCHK(ctx, expr)                                                                    \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      return set_err(ctx, PLM_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));         \
  } while (0)

struct Bump {
  char* base;
  size_t off;
  template <class T>
  T* take(size_t n) {
    off = (off + 255) & ~(size_t)255;
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += n * sizeof(T);
    return p;
  }
};

size_t rup(size_t x, size_t m) { return (x + m - 1) / m * m; }

struct EvalBufs {
  uint8_t* msa_cm;
  uint8_t* msaT;
  float* R;
  double* f_part;
  double* gh_part;
  double* gJ;
  uint16_t* sorted;
  int32_t B_pad, N_pad, B3, tiles_max, nchunks;
};

void layout_eval(Bump& bp, int32_t B, int32_t N, int32_t q, EvalBufs& e) {
  e.B_pad = (int32_t)rup(B, forward_tile_seqs(64));
  e.N_pad = (int32_t)rup(N, kFwdChunk);
  e.B3 = (int32_t)rup(B, 3);
  e.tiles_max = (B + forward_tile_seqs(16) - 1) / forward_tile_seqs(16);
  e.msa_cm = bp.take<uint8_t>((size_t)e.B_pad * e.N_pad);
  e.msaT = bp.take<uint8_t>((size_t)e.B_pad * e.N_pad);
  e.R = bp.take<float>((size_t)N * e.B3 * kSlot);
  e.f_part = bp.take<double>((size_t)e.tiles_max * N);
  e.gh_part = bp.take<double>((size_t)e.tiles_max * N * kSlot);
  e.gJ = bp.take<double>((size_t)N * N * q * q);
  e.nchunks = (e.B3 + kBwdSeqChunk - 1) / kBwdSeqChunk;
  e.sorted = bp.take<uint16_t>((size_t)e.nchunks * N * kBwdSeqChunk);
}

struct FitBufs {
  EvalBufs ev;
  float *Th, *TJ;
  double *Gh, *GJ, *Dh, *DJ, *Sh, *SJ, *Yh, *YJ;
  SiteState* st;
  int32_t* sites;
  int32_t* n_active;
  unsigned long long* site_evals;
};

void layout_fit(Bump& bp, int32_t B, int32_t N, int32_t q, int32_t m, FitBufs& f) {
  layout_eval(bp, B, N, q, f.ev);
  const size_t Nq = (size_t)N * q, NNqq = (size_t)N * N * q * q;
  f.Th = bp.take<float>(Nq);
  f.TJ = bp.take<float>(NNqq);
  f.Gh = bp.take<double>(Nq);
  f.GJ = bp.take<double>(NNqq);
  f.Dh = bp.take<double>(Nq);
  f.DJ = bp.take<double>(NNqq);
  f.Sh = bp.take<double>(Nq * m);
  f.SJ = bp.take<double>(NNqq * m);
  f.Yh = bp.take<double>(Nq * m);
  f.YJ = bp.take<double>(NNqq * m);
  f.st = bp.take<SiteState>(N);
  f.sites = bp.take<int32_t>(N);
  f.n_active = bp.take<int32_t>(1);
  f.site_evals = bp.take<unsigned long long>(1);
}

int check_sizes(plm_ctx* c, int32_t B, int32_t N, int32_t q) {
  if (B < 1 || N < 2 || q < 2 || q > kQMax)
    return set_err(c, PLM_E_INVALID, "unsupported sizes B=%d N=%d q=%d (need B>=1, N>=2, 2<=q<=21)", B,
                   N, q);
  if ((int64_t)N * q > 65535) return set_err(c, PLM_E_INVALID, "N*q too large");
  return PLM_OK;
}

int check_ws(plm_ctx* c, void* ws, size_t have, size_t need) {
  if (need == 0) return PLM_OK;
  if (!ws) return set_err(c, PLM_E_WORKSPACE, "workspace is NULL (need %zu bytes)", need);
  if (((uintptr_t)ws & 255) != 0) return set_err(c, PLM_E_WORKSPACE, "workspace not 256-byte aligned");
  if (have < need) return set_err(c, PLM_E_WORKSPACE, "workspace %zu bytes < %zu needed", have, need);
  return PLM_OK;
}

int ensure_pin(plm_ctx* c, size_t words) {
  if (c->pin_words >= words) return PLM_OK;
  if (c->pin) (void)hipHostFree(c->pin);
  c->pin = nullptr;
  c->pin_words = 0;
  HIPCHK(c, hipHostMalloc((void**)&c->pin, words * sizeof(int32_t), hipHostMallocMapped));
  HIPCHK(c, hipHostGetDevicePointer((void**)&c->pin_dev, c->pin, 0));
  memset(c->pin, 0, words * sizeof(int32_t));
  c->pin_words = words;
  return PLM_OK;
}

int32_t pick_nb(int32_t B, int32_t tile_seqs) {
  if (tile_seqs == 16 || tile_seqs == 32 || tile_seqs == 64) return tile_seqs;
  if (B >= 4 * forward_tile_seqs(64)) return 64;
  if (B >= 2 * forward_tile_seqs(32)) return 32;
  return 16;
}

// Kernels of each evaluation path: 0 = LDS gather forward / sorted scatter
// backward, n > 0 = one-hot MFMA product with n BF16 pieces.
struct PathSpec {
  int fwd_np, bwd_np;
};

bool path_spec(int32_t path, PathSpec* p) {
  switch (path) {
    case PLM_PATH_GATHER_FP32: *p = {0, 0}; return true;
    case PLM_PATH_MFMA_BF16X2: *p = {2, 2}; return true;
    case PLM_PATH_GATHER_MFMA_FP32: *p = {0, 3}; return true;
    case PLM_PATH_MFMA_FP32: *p = {3, 3}; return true;
    default: return false;
  }
}

int32_t eval_tiles(const PathSpec& p, int32_t B, int32_t nb) {
  const int32_t t = p.fwd_np ? mfma_forward_tile_seqs() : forward_tile_seqs(nb);
  return (B + t - 1) / t;
}

hipError_t eval_prepare(const PathSpec& p, const EvalArgs& a, uint8_t* msaT, uint16_t* sorted,
                        hipStream_t st) {
  if (p.bwd_np) return launch_transpose_msa(a.msa_cm, a.B_pad, a.N_pad, msaT, st);
  return launch_chunk_sort(a.msa_cm, a.B3, a.B_pad, a.N, a.q, sorted, st);
}

hipError_t eval_forward(const PathSpec& p, const EvalArgs& a, int32_t n, int32_t nb, hipStream_t st) {
  return p.fwd_np ? launch_forward_mfma(a, n, p.fwd_np, st) : launch_forward(a, n, nb, st);
}

hipError_t eval_backward(const PathSpec& p, const EvalArgs& a, int32_t n, hipStream_t st) {
  return p.bwd_np ? launch_backward_mfma(a, n, p.bwd_np, st) : launch_backward(a, n, st);
}

int flags_status(plm_ctx* c) {
  const int32_t f = c->pin[0];
  if (f & 1) {
    c->pin[0] = 0;
    return set_err(c, PLM_E_SYMBOL, "alignment holds a symbol >= q");
  }
  if (f & 2) {
    c->pin[0] = 0;
    return set_err(c, PLM_E_NONFINITE, "non-finite value in an input array");
  }
  return PLM_OK;
}

}  // namespace

extern "C" {

const char* plm_status_string(int s) {
  switch (s) {
    case PLM_OK: return "ok";
    case PLM_W_MAXITER: return "some sites stopped at the iteration cap";
    case PLM_E_INVALID: return "invalid argument";
    case PLM_E_SYMBOL: return "alignment symbol out of range";
    case PLM_E_NONFINITE: return "non-finite input";
    case PLM_E_WORKSPACE: return "workspace missing or too small";
    case PLM_E_HIP: return "HIP runtime error";
    case PLM_E_UNSUPPORTED: return "unsupported device or option";
    default: return "unknown status";
  }
}

const char* plm_last_error(const plm_ctx* c) { return c ? c->err : "null context"; }

int plm_ctx_create(plm_ctx** out, int device, void* hip_stream) {
  if (!out) return PLM_E_INVALID;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return PLM_E_INVALID;
  hipDeviceProp_t p;
  if (hipGetDeviceProperties(&p, device) != hipSuccess) return PLM_E_HIP;
  if (strncmp(p.gcnArchName, "gfx950", 6) != 0) return PLM_E_UNSUPPORTED;
  plm_ctx* c = new plm_ctx();
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  c->err[0] = 0;
  c->pin = nullptr;
  c->pin_dev = nullptr;
  c->pin_words = 0;
  c->fit_stream = nullptr;
  memset(&c->timing, 0, sizeof(c->timing));
  for (int k = 0; k < 5; ++k) c->ev[k] = nullptr;
  bool ev_ok = true;
  if (hipSetDevice(device) == hipSuccess)
    for (int k = 0; k < 5; ++k) ev_ok = ev_ok && hipEventCreate(&c->ev[k]) == hipSuccess;
  if (!ev_ok || hipSetDevice(device) != hipSuccess || ensure_pin(c, 64) != PLM_OK ||
      hipStreamCreateWithFlags(&c->fit_stream, hipStreamNonBlocking) != hipSuccess) {
    if (c->pin) (void)hipHostFree(c->pin);
    delete c;
    return PLM_E_HIP;
  }
  *out = c;
  return PLM_OK;
}

int plm_ctx_destroy(plm_ctx* c) {
  if (!c) return PLM_E_INVALID;
  if (c->pin) (void)hipHostFree(c->pin);
  if (c->fit_stream) (void)hipStreamDestroy(c->fit_stream);
  for (int k = 0; k < 5; ++k)
    if (c->ev[k]) (void)hipEventDestroy(c->ev[k]);
  delete c;
  return PLM_OK;
}

int plm_sync(plm_ctx* c) {
  if (!c) return PLM_E_INVALID;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return flags_status(c);
}

int plm_reweight(plm_ctx* c, const uint8_t* msa, int32_t B, int32_t N, int32_t q, double theta,
                 int32_t uniform, int32_t* m_out, double* w_out, double* beff_out) {
  if (!c) return PLM_E_INVALID;
  if (!msa || !m_out || !w_out || !beff_out) return set_err(c, PLM_E_INVALID, "null pointer");
  int rc = check_sizes(c, B, N, q);
  if (rc) return rc;
  if (!(theta >= 0.0 && theta <= 1.0)) return set_err(c, PLM_E_INVALID, "theta outside [0,1]");
  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, launch_reweight(msa, B, N, q, theta, uniform, m_out, w_out, beff_out, c->pin_dev, c->stream));
  return PLM_OK;
}

size_t plm_objgrad_workspace_bytes(int32_t B, int32_t N, int32_t q, int32_t path) {
  (void)path;
  if (B < 1 || N < 2 || q < 2 || q > kQMax) return 0;
  Bump bp{nullptr, 0};
  EvalBufs e;
  layout_eval(bp, B, N, q, e);
  return rup(bp.off, 256);
}

int plm_objgrad(plm_ctx* c, const uint8_t* msa, int32_t B, int32_t N, int32_t q, const double* w,
                const double* beff, const float* h, const float* J, double lambda_h,
                double lambda_J, const int32_t* sites, int32_t n_sites, int32_t path, void* ws,
                size_t ws_bytes, const double* grad_scale, double* f_out, float* gh_out,
                float* gJ_out) {
  if (!c) return PLM_E_INVALID;
  if (!msa || !w || !beff || !h || !J || !f_out) return set_err(c, PLM_E_INVALID, "null pointer");
  int rc = check_sizes(c, B, N, q);
  if (rc) return rc;
  if (!(lambda_h >= 0.0) || !(lambda_J >= 0.0)) return set_err(c, PLM_E_INVALID, "negative lambda");
  PathSpec ps;
  if (!path_spec(path, &ps))
    return set_err(c, PLM_E_UNSUPPORTED, "evaluation path %d is not available", path);
  if (!sites) n_sites = N;
  if (n_sites < 1 || n_sites > N) return set_err(c, PLM_E_INVALID, "n_sites out of range");
  const size_t need = plm_objgrad_workspace_bytes(B, N, q, path);
  rc = check_ws(c, ws, ws_bytes, need);
  if (rc) return rc;
  HIPCHK(c, hipSetDevice(c->device));
  Bump bp{(char*)ws, 0};
  EvalBufs e;
  layout_eval(bp, B, N, q, e);
  HIPCHK(c, launch_check_f64(w, (size_t)B, c->pin_dev, c->stream));
  HIPCHK(c, launch_check_f32(h, (size_t)N * q, c->pin_dev, c->stream));
  HIPCHK(c, launch_check_f32(J, (size_t)N * N * q * q, c->pin_dev, c->stream));
  if (grad_scale) HIPCHK(c, launch_check_f64(grad_scale, (size_t)N, c->pin_dev, c->stream));
  HIPCHK(c, launch_pad_msa(msa, B, N, q, e.msa_cm, e.B_pad, e.N_pad, c->pin_dev, c->stream));
  const int32_t nb = pick_nb(B, 0);
  EvalArgs a;
  a.msa_cm = e.msa_cm;
  a.msaT = e.msaT;
  a.B = B; a.B3 = e.B3; a.B_pad = e.B_pad; a.N = N; a.N_pad = e.N_pad; a.q = q;
  a.w = w; a.h = h; a.J = J;
  a.sites = sites; a.n_active = nullptr; a.n_active_host = n_sites;
  a.R = e.R; a.f_part = e.f_part; a.gh_part = e.gh_part; a.gJ = e.gJ;
  a.sorted = e.sorted;
  a.tiles = eval_tiles(ps, B, nb);
  HIPCHK(c, eval_forward(ps, a, n_sites, nb, c->stream));
  if (gJ_out) {
    HIPCHK(c, eval_prepare(ps, a, e.msaT, e.sorted, c->stream));
    HIPCHK(c, eval_backward(ps, a, n_sites, c->stream));
  }
  FinalArgs fa;
  fa.N = N; fa.q = q; fa.tiles = a.tiles; fa.lambda_h = lambda_h; fa.lambda_Jp = 0.5 * lambda_J;
  fa.beff = beff; fa.h = h; fa.J = J; fa.sites = sites;
  fa.f_part = e.f_part; fa.gh_part = e.gh_part; fa.gJ = e.gJ; fa.grad_scale = grad_scale;
  fa.f_out = f_out; fa.gh_out = gh_out; fa.gJ_out = gJ_out;
  HIPCHK(c, launch_objgrad_final(fa, n_sites, c->stream));
  return PLM_OK;
}

void plm_fit_opts_default(plm_fit_opts* o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->lambda_h = 0.01;
  o->lambda_J = 0.01;
  o->tol = 1e-6;
  o->max_iter = 2000;
  o->lbfgs_m = 10;
  o->max_linesearch = 20;
  o->path = PLM_PATH_GATHER_FP32;
  o->sync_every = 8;
  o->use_graph = 1;
  o->single_site = 0;
  o->tile_seqs = 0;
  o->site_limit = 0;
  o->timing = 0;
}

size_t plm_fit_workspace_bytes(int32_t B, int32_t N, int32_t q, const plm_fit_opts* o) {
  if (B < 1 || N < 2 || q < 2 || q > kQMax || !o) return 0;
  const int m = o->lbfgs_m;
  if (m < 1 || m > kMMax) return 0;
  Bump bp{nullptr, 0};
  FitBufs f;
  layout_fit(bp, B, N, q, m, f);
  return rup(bp.off, 256);
}

int plm_fit(plm_ctx* c, const uint8_t* msa, int32_t B, int32_t N, int32_t q, const double* w,
            const double* beff, const plm_fit_opts* o, void* ws, size_t ws_bytes, float* h_io,
            float* J_io, plm_site_stats* stats_out) {
  if (!c) return PLM_E_INVALID;
  if (!msa || !w || !beff || !o || !h_io || !J_io) return set_err(c, PLM_E_INVALID, "null pointer");
  int rc = check_sizes(c, B, N, q);
  if (rc) return rc;
  if (!(o->lambda_h >= 0.0) || !(o->lambda_J >= 0.0) || !(o->tol >= 0.0) || o->max_iter < 1 ||
      o->lbfgs_m < 1 || o->lbfgs_m > kMMax || o->max_linesearch < 1)
    return set_err(c, PLM_E_INVALID, "invalid fit options");
  PathSpec ps;
  if (!path_spec(o->path, &ps))
    return set_err(c, PLM_E_UNSUPPORTED, "evaluation path %d is not available", o->path);
  const size_t need = plm_fit_workspace_bytes(B, N, q, o);
  rc = check_ws(c, ws, ws_bytes, need);
  if (rc) return rc;
  HIPCHK(c, hipSetDevice(c->device));
  rc = ensure_pin(c, 2 + (size_t)N);
  if (rc) return rc;
  int32_t* phase_host_dev = c->pin_dev + 2;
  volatile int32_t* phase_host = c->pin + 2;
  Bump bp{(char*)ws, 0};
  FitBufs f;
  layout_fit(bp, B, N, q, o->lbfgs_m, f);
  // the fit runs on the context's private stream once the caller's stream has
  // delivered its inputs, and returns after the private stream has finished
  HIPCHK(c, hipStreamSynchronize(c->stream));
  hipStream_t st = c->fit_stream;
  c->pin[1] = N;

  HIPCHK(c, launch_check_f64(w, (size_t)B, c->pin_dev, st));
  HIPCHK(c, launch_check_f32(h_io, (size_t)N * q, c->pin_dev, st));
  HIPCHK(c, launch_pad_msa(msa, B, N, q, f.ev.msa_cm, f.ev.B_pad, f.ev.N_pad, c->pin_dev, st));
  HIPCHK(c, launch_init_fit(N, q, h_io, J_io, f.Th, f.TJ, f.st, f.sites, f.n_active, phase_host_dev, st));
  HIPCHK(c, launch_check_f32(J_io, (size_t)N * N * q * q, c->pin_dev, st));
  HIPCHK(c, launch_zero_u64(f.site_evals, st));
  HIPCHK(c, hipStreamSynchronize(st));
  rc = flags_status(c);
  if (rc) return rc;

  const int32_t nb = pick_nb(B, o->tile_seqs);
  EvalArgs a;
  a.msa_cm = f.ev.msa_cm;
  a.msaT = f.ev.msaT;
  a.B = B; a.B3 = f.ev.B3; a.B_pad = f.ev.B_pad; a.N = N; a.N_pad = f.ev.N_pad; a.q = q;
  a.w = w; a.h = f.Th; a.J = f.TJ;
  a.sites = f.sites; a.n_active = f.n_active; a.n_active_host = N;
  a.R = f.ev.R; a.f_part = f.ev.f_part; a.gh_part = f.ev.gh_part; a.gJ = f.ev.gJ;
  a.sorted = f.ev.sorted;
  a.tiles = eval_tiles(ps, B, nb);
  HIPCHK(c, eval_prepare(ps, a, f.ev.msaT, f.ev.sorted, st));

  LbfgsArgs L;
  L.N = N; L.q = q; L.m = o->lbfgs_m; L.max_iter = o->max_iter; L.max_ls = o->max_linesearch;
  L.tiles = a.tiles; L.tol = o->tol; L.lambda_h = o->lambda_h; L.lambda_Jp = 0.5 * o->lambda_J;
  L.c1 = 1e-4;
  L.noise = 1e-7;  // relative rounding noise allowed in the FP32 objective
  L.beff = beff;
  L.Xh = h_io; L.XJ = J_io; L.Th = f.Th; L.TJ = f.TJ;
  L.Gh = f.Gh; L.GJ = f.GJ; L.Dh = f.Dh; L.DJ = f.DJ;
  L.Sh = f.Sh; L.SJ = f.SJ; L.Yh = f.Yh; L.YJ = f.YJ;
  L.f_part = f.ev.f_part; L.gh_part = f.ev.gh_part; L.gJ = f.ev.gJ;
  L.st = f.st; L.phase_host = phase_host_dev; L.site_offset = 0;

  const int64_t cap = (int64_t)o->max_iter * (o->max_linesearch + 2) + 16;
  if (o->single_site) {
    // the plain path: one site at a time, each launch sized for one site, the
    // host waiting for every iteration
    EvalArgs a1 = a;
    a1.n_active = nullptr;
    a1.n_active_host = 1;
    const int32_t nsites = (o->site_limit > 0 && o->site_limit < N) ? o->site_limit : N;
    for (int32_t r = 0; r < nsites; ++r) {
      a1.sites = f.sites + r;  // sites[r] == r after initialisation
      LbfgsArgs L1 = L;
      L1.site_offset = r;
      for (int64_t it = 0; it < cap; ++it) {
        HIPCHK(c, eval_forward(ps, a1, 1, nb, st));
        HIPCHK(c, eval_backward(ps, a1, 1, st));
        HIPCHK(c, launch_lbfgs(L1, 1, st));
        HIPCHK(c, hipStreamSynchronize(st));
        if (phase_host[r] == PH_DONE) break;
      }
    }
  } else {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    const bool timed = o->timing != 0;
    auto mark = [&](int k) -> hipError_t { return timed ? hipEventRecord(c->ev[k], st) : hipSuccess; };
    auto enqueue = [&]() -> hipError_t {
      hipError_t e = mark(0);
      if (e == hipSuccess) e = eval_forward(ps, a, N, nb, st);
      if (e == hipSuccess) e = mark(1);
      if (e == hipSuccess) e = eval_backward(ps, a, N, st);
      if (e == hipSuccess) e = mark(2);
      if (e == hipSuccess) e = launch_lbfgs(L, N, st);
      if (e == hipSuccess) e = mark(3);
      if (e == hipSuccess) e = launch_compact(N, f.st, f.sites, f.n_active, c->pin_dev + 1, f.site_evals, st);
      return e;
    };
    plm_fit_timing tm;
    memset(&tm, 0, sizeof(tm));
    // timing records events between the kernels, which needs eager launches
    const bool use_graph = o->use_graph && !timed;
    if (use_graph) {
      HIPCHK(c, hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
      hipError_t e = enqueue();
      hipError_t e2 = hipStreamEndCapture(st, &graph);
      if (e != hipSuccess) return set_err(c, PLM_E_HIP, "capture: %s", hipGetErrorString(e));
      HIPCHK(c, e2);
      HIPCHK(c, hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
    }
    const int every = timed ? 1 : (o->sync_every > 0 ? o->sync_every : 1);
    int64_t launched = 0;
    int err = PLM_OK;
    while (launched < cap) {
      for (int k = 0; k < every; ++k, ++launched) {
        hipError_t e = use_graph ? hipGraphLaunch(exec, st) : enqueue();
        if (e != hipSuccess) {
          err = set_err(c, PLM_E_HIP, "iteration launch: %s", hipGetErrorString(e));
          break;
        }
      }
      if (err) break;
      hipError_t e = hipStreamSynchronize(st);
      if (e != hipSuccess) {
        err = set_err(c, PLM_E_HIP, "sync: %s", hipGetErrorString(e));
        break;
      }
      if (timed) {
        float t01 = 0.f, t12 = 0.f, t23 = 0.f;
        if (hipEventElapsedTime(&t01, c->ev[0], c->ev[1]) == hipSuccess &&
            hipEventElapsedTime(&t12, c->ev[1], c->ev[2]) == hipSuccess &&
            hipEventElapsedTime(&t23, c->ev[2], c->ev[3]) == hipSuccess) {
          tm.forward_ms += t01;
          tm.backward_ms += t12;
          tm.lbfgs_ms += t23;
        } else {
          (void)hipGetLastError();  // do not leave a timing failure for the next launch check
        }
        tm.iterations += 1;
      }
      if (((volatile int32_t*)c->pin)[1] == 0) break;
    }
    if (timed) {
      unsigned long long se = 0;
      (void)hipMemcpy(&se, f.site_evals, sizeof(se), hipMemcpyDeviceToHost);
      tm.site_evals = (int64_t)se;
      tm.total_ms = tm.forward_ms + tm.backward_ms + tm.lbfgs_ms;
      c->timing = tm;
    }
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (err) return err;
  }
  HIPCHK(c, hipStreamSynchronize(st));
  rc = flags_status(c);
  if (rc) return rc;
  std::vector<SiteState> hs(N);
  HIPCHK(c, hipMemcpy(hs.data(), f.st, sizeof(SiteState) * N, hipMemcpyDeviceToHost));
  int any_max = 0;
  for (int32_t r = 0; r < N; ++r) {
    int status = hs[r].phase == PH_DONE ? hs[r].status : PLM_SITE_MAXITER;
    if (status == PLM_SITE_MAXITER) any_max = 1;
    if (stats_out) {
      stats_out[r].iterations = hs[r].iter;
      stats_out[r].evaluations = hs[r].evals;
      stats_out[r].status = status;
      stats_out[r].pad = 0;
      stats_out[r].f = hs[r].f;
      stats_out[r].gnorm = hs[r].gnorm;
    }
  }
  return any_max ? PLM_W_MAXITER : PLM_OK;
}

int plm_fit_last_timing(const plm_ctx* c, plm_fit_timing* out) {
  if (!c || !out) return PLM_E_INVALID;
  *out = c->timing;
  return PLM_OK;
}

int plm_score(plm_ctx* c, const float* J, int32_t N, int32_t q, double* fn_out, double* cfn_out) {
  if (!c) return PLM_E_INVALID;
  if (!J || !fn_out || !cfn_out) return set_err(c, PLM_E_INVALID, "null pointer");
  if (N < 2 || q < 2 || q > kQMax) return set_err(c, PLM_E_INVALID, "unsupported sizes");
  if ((int64_t)N > 65535) return set_err(c, PLM_E_INVALID, "N too large");
  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, launch_score(J, N, q, fn_out, cfn_out, c->stream));
  return PLM_OK;
}

}  // extern "C"
