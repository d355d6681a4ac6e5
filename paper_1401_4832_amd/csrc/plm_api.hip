// plm_api.hip -- host side of the C ABI declared in include/plm.h.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
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
  int32_t ncu;             // compute units of the device
};

namespace {

// Scratch of plm_objgrad_static: one fixed array per GPU, held from the first
// context on that GPU until the process ends.  Host code never uses the
// array's name as an address (on the host it is only a stand-in): the address
// on each device comes from hipGetSymbolAddress, taken once per device with
// that device current, and is what the kernels receive.
__device__ __align__(256) unsigned char scratch[PLM_STATIC_SCRATCH_BYTES];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];
bool g_scratch_set[kMaxDevices];

// (the device must be current)
hipError_t static_scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_set[device]) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[device] = p;
  g_scratch_set[device] = true;
  return hipSuccess;
}

void* static_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_set[device] ? g_scratch_ptr[device] : nullptr;
}

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
  int8_t* Wq;
  int32_t* jexp;
  uint32_t* sym3;
  int32_t NG;
};

// wide: room for the precise path's two residual digit sets (126 bytes per
// site and row instead of 21 floats)
void layout_eval(Bump& bp, int32_t B, int32_t N, int32_t q, EvalBufs& e, bool wide = false) {
  e.B_pad = (int32_t)rup(B, kBPadUnit);
  e.N_pad = (int32_t)rup(N, kFwdChunk);
  e.B3 = (int32_t)rup(B, 3);
  // the smallest forward tile gives the most tiles
  const int32_t tmin = std::min(forward_tile_seqs(16), fwd_i8_tile_seqs());
  e.tiles_max = (B + tmin - 1) / tmin;
  e.msa_cm = bp.take<uint8_t>((size_t)e.B_pad * e.N_pad);
  e.msaT = bp.take<uint8_t>((size_t)e.B_pad * e.N_pad);
  // FP32 rows [B3][21], or the fragment-order FP16 pieces over B_pad rows
  e.R = bp.take<float>((size_t)N * e.B_pad * (wide ? 32 : kSlot));
  e.f_part = bp.take<double>((size_t)e.tiles_max * N);
  e.gh_part = bp.take<double>((size_t)e.tiles_max * N * kSlot);
  e.gJ = bp.take<double>((size_t)N * N * q * q);
  e.nchunks = (e.B3 + kBwdSeqChunk - 1) / kBwdSeqChunk;
  e.sorted = bp.take<uint16_t>((size_t)e.nchunks * N * kBwdSeqChunk);
  e.NG = (N + 2) / 3;
  e.Wq = bp.take<int8_t>((size_t)N * e.NG * kWqGroupBytes);
  e.jexp = bp.take<int32_t>((size_t)N * (1 + kJParts));
  e.sym3 = bp.take<uint32_t>((size_t)e.NG * e.B_pad);
}

// per-alignment optimiser buffers
struct FitBufs {
  EvalBufs ev;
  float *Th, *TJ;
  double* small;
  float *Dh, *DJ;
  void *Gh, *GJ, *Sh, *SJ, *Yh, *YJ;  // history type: FP32, or FP64 with history_fp64
  DirCoef* dc;
  double *dpart, *part, *ghd;
};

void layout_fit(Bump& bp, int32_t B, int32_t N, int32_t q, int32_t m, int32_t hist64, bool wide, FitBufs& f) {
  layout_eval(bp, B, N, q, f.ev, wide);
  const size_t Nq = (size_t)N * q, NNqq = (size_t)N * N * q * q;
  const size_t hb = hist64 ? 2 : 1;  // history values in floats
  f.Th = bp.take<float>(Nq);
  f.TJ = bp.take<float>(NNqq);
  f.Gh = bp.take<float>(Nq * hb);
  f.GJ = bp.take<float>(NNqq * hb);
  f.Dh = bp.take<float>(Nq);
  f.DJ = bp.take<float>(NNqq);
  f.Sh = bp.take<float>(Nq * (m + 1) * hb);
  f.SJ = bp.take<float>(NNqq * (m + 1) * hb);
  f.Yh = bp.take<float>(Nq * (m + 1) * hb);
  f.YJ = bp.take<float>(NNqq * (m + 1) * hb);
  f.small = bp.take<double>((size_t)N * 2 * (m + 1) * (m + 2));
  f.dc = bp.take<DirCoef>(N);
  f.dpart = bp.take<double>((size_t)N * kLbChunks);
  f.part = bp.take<double>((size_t)N * kLbChunks * kLbPartW);
  f.ghd = bp.take<double>(Nq);
}

// device tables of a batch (BatchArgs points into them)
struct Tables {
  EvalArgs* ev;
  LbfgsArgs* lb;
  int32_t *site_base, *msa_of, *active, *n_active, *seg, *item_off, *nsub;
  uint32_t* ctr;
  SiteState* st;
  unsigned long long* site_evals;
};

void layout_tables(Bump& bp, int32_t n_msas, int32_t total, bool fit, Tables& t) {
  t.ev = bp.take<EvalArgs>(n_msas);
  t.lb = fit ? bp.take<LbfgsArgs>(n_msas) : nullptr;
  t.site_base = bp.take<int32_t>(n_msas + 1);
  t.msa_of = bp.take<int32_t>(total);
  t.active = bp.take<int32_t>(total);
  t.n_active = bp.take<int32_t>(1);
  t.seg = bp.take<int32_t>(n_msas + 1);
  t.item_off = bp.take<int32_t>(2 * (n_msas + 1));
  t.nsub = bp.take<int32_t>(2 * n_msas);
  t.ctr = bp.take<uint32_t>(2 * kQueues);
  t.st = fit ? bp.take<SiteState>(total) : nullptr;
  t.site_evals = bp.take<unsigned long long>(1);
}

BatchArgs batch_args(const Tables& t, int32_t n_msas, int32_t total, int32_t group, int32_t fgroup) {
  BatchArgs b;
  b.ev = t.ev;
  b.lb = t.lb;
  b.n_msas = n_msas;
  b.total_sites = total;
  b.site_base = t.site_base;
  b.msa_of = t.msa_of;
  b.active = t.active;
  b.n_active = t.n_active;
  b.seg = t.seg;
  b.item_off = t.item_off;
  b.nsub = t.nsub;
  b.ctr = t.ctr;
  b.bwd_group = group;
  b.fwd_group = fgroup;
  return b;
}

// buffers of the symmetric fit
struct SymBufs {
  EvalBufs ev;
  float *Th, *TJ, *Thl, *TJl;  // trial point and its low-order words
  double *Gh, *GJ, *Dh, *DJ, *part, *small;
  float *Sh, *SJ, *Yh, *YJ;
  SymCoef* coef;
  SymState* st;
  int2* pairs;
  Tables t;
};

void layout_sym(Bump& bp, int32_t B, int32_t N, int32_t q, int32_t m, int32_t nblk, bool wide, SymBufs& f) {
  layout_eval(bp, B, N, q, f.ev, wide);
  const size_t Nq = (size_t)N * q, NNqq = (size_t)N * N * q * q;
  f.Th = bp.take<float>(Nq);
  f.TJ = bp.take<float>(NNqq);
  f.Thl = bp.take<float>(Nq);
  f.TJl = bp.take<float>(NNqq);
  f.Gh = bp.take<double>(Nq);
  f.GJ = bp.take<double>(NNqq);
  f.Dh = bp.take<double>(Nq);
  f.DJ = bp.take<double>(NNqq);
  f.Sh = bp.take<float>(Nq * (m + 1));
  f.SJ = bp.take<float>(NNqq * (m + 1));
  f.Yh = bp.take<float>(Nq * (m + 1));
  f.YJ = bp.take<float>(NNqq * (m + 1));
  f.part = bp.take<double>((size_t)(1 + sym_groups(m)) * nblk * sym_part_stride());
  f.small = bp.take<double>((size_t)2 * (m + 1) * (m + 1));
  f.coef = bp.take<SymCoef>(1);
  f.st = bp.take<SymState>(1);
  f.pairs = bp.take<int2>((size_t)N * (N - 1) / 2);
  layout_tables(bp, 1, N, false, f.t);
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
  int bwd_f16;  // gradient pieces in FP16 (of R * 2^12) instead of BF16
  int bwd_g3;   // grouped gradient: three sites per item, R split by the forward
  int bwd_i8;   // grouped gradient on int8 digits of R (fixed point, exact accumulation)
  int fwd_i8;   // grouped forward on int8 digits of J (fixed point, exact accumulation)
  int f64;      // precise path: FP64 gather forward, residuals as two int8 digit sets, two gradient passes
};

// sites per work item
int32_t bwd_group(const PathSpec& p) { return (p.bwd_g3 || p.bwd_i8) ? kG3Sites : 1; }
int32_t fwd_group(const PathSpec& p) { return p.fwd_i8 ? kG3Sites : 1; }

// the int8 gradient sums up to 2^24 sequences exactly
bool path_fits(const PathSpec& p, int32_t B) { return !p.bwd_i8 || B < (1 << 24); }

bool path_spec(int32_t path, PathSpec* p) {
  switch (path) {
    case PLM_PATH_GATHER_FP32: *p = {0, 0, 0, 0, 0, 0, 0}; return true;
    case PLM_PATH_MFMA_BF16X2: *p = {2, 2, 0, 0, 0, 0, 0}; return true;
    case PLM_PATH_GATHER_MFMA_FP32: *p = {0, 3, 0, 0, 0, 0, 0}; return true;
    case PLM_PATH_MFMA_FP32: *p = {3, 3, 0, 0, 0, 0, 0}; return true;
    case PLM_PATH_GATHER_MFMA_F16X2: *p = {0, 2, 1, 1, 0, 0, 0}; return true;
    case PLM_PATH_GATHER_MFMA_I8X3: *p = {0, 3, 0, 0, 1, 0, 0}; return true;
    case PLM_PATH_MFMA_I8X3: *p = {0, 3, 0, 0, 1, 1, 0}; return true;
    case PLM_PATH_GATHER64_MFMA_I8X6: *p = {0, 3, 0, 0, 1, 0, 1}; return true;
    default: return false;
  }
}

int32_t eval_tiles(const PathSpec& p, int32_t B, int32_t nb) {
  const int32_t t = p.fwd_i8   ? fwd_i8_tile_seqs()
                    : p.fwd_np ? mfma_forward_tile_seqs()
                    : p.f64    ? forward_f64_tile_seqs()
                               : forward_tile_seqs(nb);
  return (B + t - 1) / t;
}

int32_t eval_bwd_blocks(const PathSpec& p, int32_t N, int32_t q) {
  if (p.bwd_g3) return g3_backward_blocks_per_site(N, q);
  if (p.bwd_i8) return i8_backward_blocks_per_site(N, q);
  return p.bwd_np ? mfma_backward_blocks_per_site(N, q) : backward_blocks_per_site(N);
}

// Once per alignment, before the first forward: the int8 forward's packed
// symbols, and (backward = true) the gradient path's symbol copy and, for the
// grouped gradient, the residual rows no forward tile writes.
hipError_t eval_prepare(const PathSpec& p, const EvalArgs& a, uint8_t* msaT, uint16_t* sorted,
                        hipStream_t st, bool backward = true) {
  if (!backward)
    return p.fwd_i8 ? launch_sym3(a.msa_cm, a.B_pad, a.N, a.NG, const_cast<uint32_t*>(a.sym3), st)
                    : hipSuccess;
  if (p.bwd_g3 || p.bwd_i8) {
    hipError_t e =
        launch_rfrag_tail_zero(a.R, a.N, a.B, a.B3, a.B_pad, p.bwd_i8 ? kRiChunkBytes : kRfChunkBytes, st);
    if (e == hipSuccess && p.f64)  // the remainder digits
      e = launch_rfrag_tail_zero(reinterpret_cast<float*>(reinterpret_cast<char*>(a.R) +
                                                          (size_t)a.N * (a.B_pad >> 8) * kRiChunkBytes),
                                 a.N, a.B, a.B3, a.B_pad, kRiChunkBytes, st);
    if (e != hipSuccess) return e;
  }
  if (p.fwd_i8) {
    const hipError_t e = launch_sym3(a.msa_cm, a.B_pad, a.N, a.NG, const_cast<uint32_t*>(a.sym3), st);
    if (e != hipSuccess) return e;
  }
  if (p.bwd_np) return launch_transpose_msa(a.msa_cm, a.B_pad, a.N_pad, msaT, st);
  return launch_chunk_sort(a.msa_cm, a.B3, a.B_pad, a.N, a.q, sorted, st);
}

// persistent grids: resident blocks of each kernel on the whole device
struct Grids {
  int32_t fwd, bwd;
};

Grids eval_grids(const plm_ctx* c, const PathSpec& p, int32_t nb) {
  Grids g;
  g.fwd = c->ncu * (p.fwd_i8   ? fwd_i8_resident_blocks()
                    : p.fwd_np ? mfma_resident_blocks(KIND_FWD, p.fwd_np)
                               : forward_resident_blocks(nb, p.f64));
  g.bwd = c->ncu * (p.bwd_g3   ? g3_resident_blocks()
                    : p.bwd_i8 ? i8_resident_blocks()
                    : p.bwd_np ? mfma_resident_blocks(KIND_BWD, p.bwd_np)
                               : backward_resident_blocks());
  return g;
}

// the forward's per-evaluation preparation of the couplings (int8 digits; nothing on other paths)
hipError_t eval_quant(const PathSpec& p, const BatchArgs& b, hipStream_t st) {
  return p.fwd_i8 ? launch_jquant(b, b.total_sites, st) : hipSuccess;
}

hipError_t eval_forward_main(const PathSpec& p, const BatchArgs& b, int32_t nb, const Grids& g,
                             hipStream_t st) {
  if (p.fwd_i8) return launch_fwd_i8(b, g.fwd, st);
  return p.fwd_np ? launch_forward_mfma(b, p.fwd_np, g.fwd, st) : launch_forward(b, nb, g.fwd, p.f64, st);
}

hipError_t eval_forward(const PathSpec& p, const BatchArgs& b, int32_t nb, const Grids& g,
                        hipStream_t st) {
  hipError_t e = eval_quant(p, b, st);
  return e == hipSuccess ? eval_forward_main(p, b, nb, g, st) : e;
}

hipError_t eval_backward(const PathSpec& p, const BatchArgs& b, const Grids& g, hipStream_t st) {
  if (p.bwd_g3) return launch_backward_g3(b, g.bwd, st);
  if (p.bwd_i8) {
    hipError_t e = launch_backward_i8(b, g.bwd, 0, st);
    if (e != hipSuccess || !p.f64) return e;
    // the remainder pass drains the same work items: its queues start again
    e = launch_reset_queues(b, KIND_BWD, st);
    return e == hipSuccess ? launch_backward_i8(b, g.bwd, 1, st) : e;
  }
  return p.bwd_np ? launch_backward_mfma(b, p.bwd_np, p.bwd_f16, g.bwd, st) : launch_backward(b, g.bwd, st);
}

EvalArgs eval_args(const EvalBufs& e, const uint8_t* msa_unused, int32_t B, int32_t N, int32_t q,
                   const double* w, const float* h, const float* J, int32_t tiles, const PathSpec& ps) {
  (void)msa_unused;
  EvalArgs a;
  a.msa_cm = e.msa_cm;
  a.msaT = e.msaT;
  a.B = B; a.B3 = e.B3; a.B_pad = e.B_pad; a.N = N; a.N_pad = e.N_pad; a.q = q;
  a.w = w; a.h = h; a.J = J;
  a.R = e.R; a.f_part = e.f_part; a.gh_part = e.gh_part; a.gJ = e.gJ;
  a.tiles = tiles;
  a.rfrag = ps.f64 ? 3 : ps.bwd_i8 ? 2 : (ps.bwd_g3 ? 1 : 0);
  a.Wq = e.Wq;
  a.jexp = e.jexp;
  a.sym3 = e.sym3;
  a.NG = e.NG;
  a.pad_ = 0;
  a.sorted = e.sorted;
  a.h_lo = nullptr;
  a.J_lo = nullptr;
  return a;
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
  if (f & 4) {
    c->pin[0] = 0;
    return set_err(c, PLM_E_INVALID, "site index outside [0, N)");
  }
  if (f & 8) {
    c->pin[0] = 0;
    return set_err(c, PLM_E_NONFINITE,
                   "a zero frequency or a correlation matrix that is not positive definite (raise the pseudocount)");
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
  c->ncu = p.multiProcessorCount > 0 ? p.multiProcessorCount : 1;
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
      hipStreamCreateWithFlags(&c->fit_stream, hipStreamNonBlocking) != hipSuccess ||
      static_scratch_setup(device) != hipSuccess) {
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
  if (B < 1 || N < 2 || q < 2 || q > kQMax) return 0;
  Bump bp{nullptr, 0};
  EvalBufs e;
  layout_eval(bp, B, N, q, e, path == PLM_PATH_GATHER64_MFMA_I8X6);
  Tables t;
  layout_tables(bp, 1, N, false, t);
  return rup(bp.off, 256);
}

}  // extern "C"

namespace {

// plm_objgrad on the given scratch (a caller's workspace or the static array)
int objgrad_impl(plm_ctx* c, const uint8_t* msa, int32_t B, int32_t N, int32_t q, const double* w,
                 const double* beff, const float* h, const float* J, double lambda_h,
                 double lambda_J, const int32_t* sites, int32_t n_sites, int32_t path, void* ws,
                 size_t ws_bytes, const double* grad_scale, double* f_out, float* gh_out,
                 float* gJ_out) {
  if (!msa || !w || !beff || !h || !J || !f_out) return set_err(c, PLM_E_INVALID, "null pointer");
  int rc = check_sizes(c, B, N, q);
  if (rc) return rc;
  if (!(lambda_h >= 0.0) || !(lambda_J >= 0.0)) return set_err(c, PLM_E_INVALID, "negative lambda");
  PathSpec ps;
  if (!path_spec(path, &ps))
    return set_err(c, PLM_E_UNSUPPORTED, "evaluation path %d is not available", path);
  if (!path_fits(ps, B)) return set_err(c, PLM_E_UNSUPPORTED, "path %d sums at most 2^24 - 1 sequences exactly", path);
  if (!sites) n_sites = N;
  if (n_sites < 1 || n_sites > N) return set_err(c, PLM_E_INVALID, "n_sites out of range");
  const size_t need = plm_objgrad_workspace_bytes(B, N, q, path);
  rc = check_ws(c, ws, ws_bytes, need);
  if (rc) return rc;
  HIPCHK(c, hipSetDevice(c->device));
  Bump bp{(char*)ws, 0};
  EvalBufs e;
  layout_eval(bp, B, N, q, e, path == PLM_PATH_GATHER64_MFMA_I8X6);
  Tables t;
  layout_tables(bp, 1, N, false, t);
  const BatchArgs b = batch_args(t, 1, N, bwd_group(ps), fwd_group(ps));
  HIPCHK(c, launch_check_f64(w, (size_t)B, c->pin_dev, c->stream));
  HIPCHK(c, launch_check_f32(h, (size_t)N * q, c->pin_dev, c->stream));
  HIPCHK(c, launch_check_f32(J, (size_t)N * N * q * q, c->pin_dev, c->stream));
  if (grad_scale) HIPCHK(c, launch_check_f64(grad_scale, (size_t)N, c->pin_dev, c->stream));
  HIPCHK(c, launch_pad_msa(msa, B, N, q, e.msa_cm, e.B_pad, e.N_pad, c->pin_dev, c->stream));
  const int32_t nb = pick_nb(B, 0);
  const EvalArgs a = eval_args(e, msa, B, N, q, w, h, J, eval_tiles(ps, B, nb), ps);
  HIPCHK(c, launch_setup_msa(b, 0, a, nullptr, 0, N, a.tiles, eval_bwd_blocks(ps, N, q), nullptr,
                             c->stream));
  HIPCHK(c, launch_list_tables(b, sites, 0, n_sites, c->pin_dev, c->stream));
  const Grids g = eval_grids(c, ps, nb);
  HIPCHK(c, eval_prepare(ps, a, e.msaT, e.sorted, c->stream, gJ_out != nullptr));
  HIPCHK(c, eval_forward(ps, b, nb, g, c->stream));
  if (gJ_out) HIPCHK(c, eval_backward(ps, b, g, c->stream));
  FinalArgs fa;
  fa.N = N; fa.q = q; fa.tiles = a.tiles; fa.lambda_h = lambda_h; fa.lambda_Jp = 0.5 * lambda_J;
  fa.beff = beff; fa.h = h; fa.J = J; fa.sites = t.active;  // the checked site list
  fa.f_part = e.f_part; fa.gh_part = e.gh_part; fa.gJ = e.gJ; fa.grad_scale = grad_scale;
  fa.f_out = f_out; fa.gh_out = gh_out; fa.gJ_out = gJ_out;
  HIPCHK(c, launch_objgrad_final(fa, n_sites, c->stream));
  return PLM_OK;
}

}  // namespace

extern "C" {

int plm_objgrad(plm_ctx* c, const uint8_t* msa, int32_t B, int32_t N, int32_t q, const double* w,
                const double* beff, const float* h, const float* J, double lambda_h,
                double lambda_J, const int32_t* sites, int32_t n_sites, int32_t path, void* ws,
                size_t ws_bytes, const double* grad_scale, double* f_out, float* gh_out,
                float* gJ_out) {
  if (!c) return PLM_E_INVALID;
  return objgrad_impl(c, msa, B, N, q, w, beff, h, J, lambda_h, lambda_J, sites, n_sites, path, ws,
                      ws_bytes, grad_scale, f_out, gh_out, gJ_out);
}

int plm_objgrad_static(plm_ctx* c, const uint8_t* msa, int32_t B, int32_t N, int32_t q,
                       const double* w, const double* beff, const float* h, const float* J,
                       double lambda_h, double lambda_J, const int32_t* sites, int32_t n_sites,
                       int32_t path, const double* grad_scale, double* f_out, float* gh_out,
                       float* gJ_out) {
  if (!c) return PLM_E_INVALID;
  void* ptr = static_scratch(c->device);
  if (!ptr) return set_err(c, PLM_E_HIP, "the static scratch array of device %d has no address", c->device);
  const size_t need = plm_objgrad_workspace_bytes(B, N, q, path);
  if (need > PLM_STATIC_SCRATCH_BYTES)
    return set_err(c, PLM_E_WORKSPACE, "B=%d N=%d q=%d needs %zu bytes of scratch; the static array holds %zu",
                   B, N, q, need, (size_t)PLM_STATIC_SCRATCH_BYTES);
  return objgrad_impl(c, msa, B, N, q, w, beff, h, J, lambda_h, lambda_J, sites, n_sites, path, ptr,
                      PLM_STATIC_SCRATCH_BYTES, grad_scale, f_out, gh_out, gJ_out);
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
  o->refine = 0;
  o->n_probe = 0;
  o->refine_tol = 0.0;
  o->probe_sites = nullptr;
  o->probe_h = nullptr;
  o->probe_J = nullptr;
  o->probe_out = nullptr;
  o->probe_count = nullptr;
  o->probe_cap = 0;
  o->history_fp64 = 0;
}

size_t plm_fit_opts_size(void) { return sizeof(plm_fit_opts); }

}  // extern "C"

namespace {

bool fit_opts_ok(const plm_fit_opts* o) {
  if (o->n_probe < 0 ||
      (o->n_probe > 0 && (!o->probe_sites || !o->probe_h || !o->probe_J || !o->probe_out ||
                          !o->probe_count || o->probe_cap < 1)))
    return false;
  return o->lambda_h >= 0.0 && o->lambda_J >= 0.0 && o->tol >= 0.0 && o->refine_tol >= 0.0 &&
         o->max_iter >= 1 && o->lbfgs_m >= 1 && o->lbfgs_m <= kMMax && o->max_linesearch >= 1 &&
         (o->history_fp64 == 0 || o->history_fp64 == 1);
}

int32_t refine_path(const plm_fit_opts* o);
int32_t refine_path_sym(const plm_fit_opts* o);
// the workspace needs the precise path's wide residual buffer
bool fit_wide(const plm_fit_opts* o) {
  return o->path == PLM_PATH_GATHER64_MFMA_I8X6 || refine_path(o) == PLM_PATH_GATHER64_MFMA_I8X6;
}
bool sym_wide(const plm_fit_opts* o) {
  return o->path == PLM_PATH_GATHER64_MFMA_I8X6 || refine_path_sym(o) == PLM_PATH_GATHER64_MFMA_I8X6;
}

// Alignments in batch order: decreasing evaluation cost B * N^2, ties by index.
std::vector<int32_t> batch_order(const plm_msa_desc* d, int32_t n) {
  std::vector<int32_t> ord(n);
  for (int32_t k = 0; k < n; ++k) ord[k] = k;
  std::stable_sort(ord.begin(), ord.end(), [&](int32_t x, int32_t y) {
    return (double)d[x].B * d[x].N * d[x].N > (double)d[y].B * d[y].N * d[y].N;
  });
  return ord;
}

size_t fit_layout(const plm_msa_desc* d, int32_t n, int32_t q, const plm_fit_opts* o, char* base,
                  std::vector<FitBufs>* bufs, Tables* t) {
  const std::vector<int32_t> ord = batch_order(d, n);
  Bump bp{base, 0};
  int32_t total = 0;
  if (bufs) bufs->resize(n);
  for (int32_t k = 0; k < n; ++k) {
    const plm_msa_desc& m = d[ord[k]];
    FitBufs f;
    layout_fit(bp, m.B, m.N, q, o->lbfgs_m, o->history_fp64, fit_wide(o), f);
    if (bufs) (*bufs)[k] = f;
    total += m.N;
  }
  Tables tt;
  layout_tables(bp, n, total, true, tt);
  if (t) *t = tt;
  return rup(bp.off, 256);
}

// Everything the iteration needs once a batch is set up on the device.
struct Prep {
  PathSpec ps;
  int32_t nb, total;
  Grids g;
  Tables t;
  BatchArgs b;
  std::vector<int32_t> ord, base;
  hipStream_t st;
};

// Validate, lay out the workspace, and set up every alignment of the batch on
// the context's private stream: padded symbols, trial point, optimiser states,
// descriptors, and the tables with every site active.  Synchronous.
int prepare_fit(plm_ctx* c, const plm_msa_desc* d, int32_t n, int32_t q, const plm_fit_opts* o,
                void* ws, size_t ws_bytes, Prep* P) {
  if (!fit_opts_ok(o)) return set_err(c, PLM_E_INVALID, "invalid fit options");
  PathSpec ps;
  if (!path_spec(o->path, &ps))
    return set_err(c, PLM_E_UNSUPPORTED, "evaluation path %d is not available", o->path);
  if (o->single_site && n != 1)
    return set_err(c, PLM_E_INVALID, "the single-site path takes one alignment");
  int32_t total = 0, Bmax = 0;
  for (int32_t k = 0; k < n; ++k) {
    const plm_msa_desc& m = d[k];
    if (!m.msa || !m.w || !m.beff || !m.h_io || !m.J_io)
      return set_err(c, PLM_E_INVALID, "null pointer in alignment %d", k);
    int rc = check_sizes(c, m.B, m.N, q);
    if (rc) return rc;
    if (!path_fits(ps, m.B)) return set_err(c, PLM_E_UNSUPPORTED, "path %d sums at most 2^24 - 1 sequences exactly", o->path);
    total += m.N;
    if (m.B > Bmax) Bmax = m.B;
  }
  const size_t need = fit_layout(d, n, q, o, nullptr, nullptr, nullptr);
  int rc = check_ws(c, ws, ws_bytes, need);
  if (rc) return rc;
  HIPCHK(c, hipSetDevice(c->device));
  rc = ensure_pin(c, 2 + (size_t)total);
  if (rc) return rc;
  int32_t* phase_host_dev = c->pin_dev + 2;
  std::vector<FitBufs> fb;
  Tables t;
  fit_layout(d, n, q, o, (char*)ws, &fb, &t);
  const std::vector<int32_t> ord = batch_order(d, n);
  const BatchArgs b = batch_args(t, n, total, bwd_group(ps), fwd_group(ps));
  // the fit runs on the context's private stream once the caller's stream has
  // delivered its inputs, and returns after the private stream has finished
  HIPCHK(c, hipStreamSynchronize(c->stream));
  hipStream_t st = c->fit_stream;
  c->pin[1] = total;

  const int32_t nb = pick_nb(Bmax, o->tile_seqs);
  std::vector<int32_t> base(n + 1, 0);
  for (int32_t k = 0; k < n; ++k) {
    const plm_msa_desc& m = d[ord[k]];
    const FitBufs& f = fb[k];
    base[k + 1] = base[k] + m.N;
    HIPCHK(c, launch_check_f64(m.w, (size_t)m.B, c->pin_dev, st));
    HIPCHK(c, launch_check_f32(m.h_io, (size_t)m.N * q, c->pin_dev, st));
    HIPCHK(c, launch_pad_msa(m.msa, m.B, m.N, q, f.ev.msa_cm, f.ev.B_pad, f.ev.N_pad, c->pin_dev, st));
    HIPCHK(c, launch_init_fit(m.N, q, m.h_io, m.J_io, f.Th, f.TJ, t.st + base[k], phase_host_dev + base[k], st));
    HIPCHK(c, launch_check_f32(m.J_io, (size_t)m.N * m.N * q * q, c->pin_dev, st));
    const EvalArgs a = eval_args(f.ev, m.msa, m.B, m.N, q, m.w, f.Th, f.TJ, eval_tiles(ps, m.B, nb), ps);
    HIPCHK(c, eval_prepare(ps, a, f.ev.msaT, f.ev.sorted, st));
    LbfgsArgs L;
    L.N = m.N; L.q = q; L.m = o->lbfgs_m; L.max_iter = o->max_iter; L.max_ls = o->max_linesearch;
    L.tiles = a.tiles; L.tol = o->tol; L.lambda_h = o->lambda_h; L.lambda_Jp = 0.5 * o->lambda_J;
    L.c1 = 1e-4;
    // relative rounding noise allowed in the objective's sufficient-decrease test:
    // that of the FP32 evaluations, or of the precise path's FP64 one
    L.noise = ps.f64 ? 2e-14 : 1e-7;
    L.beff = m.beff;
    L.Xh = m.h_io; L.XJ = m.J_io; L.Th = f.Th; L.TJ = f.TJ;
    L.Gh = f.Gh; L.GJ = f.GJ; L.Dh = f.Dh; L.DJ = f.DJ;
    L.Sh = f.Sh; L.SJ = f.SJ; L.Yh = f.Yh; L.YJ = f.YJ; L.small = f.small;
    L.dc = f.dc; L.dpart = f.dpart; L.part = f.part; L.ghd = f.ghd;
    L.f_part = f.ev.f_part; L.gh_part = f.ev.gh_part; L.gJ = f.ev.gJ;
    L.st = t.st + base[k];
    L.phase_host = phase_host_dev + base[k];
    HIPCHK(c, launch_setup_msa(b, k, a, &L, base[k], m.N, a.tiles, eval_bwd_blocks(ps, m.N, q),
                               t.site_evals, st));
  }
  HIPCHK(c, launch_compact(b, t.st, nullptr, nullptr, st));  // every site active
  HIPCHK(c, hipStreamSynchronize(st));
  rc = flags_status(c);
  if (rc) return rc;
  P->ps = ps;
  P->nb = nb;
  P->total = total;
  P->g = eval_grids(c, ps, nb);
  P->t = t;
  P->b = b;
  P->ord = ord;
  P->base = base;
  P->st = st;
  return PLM_OK;
}

// The fit of a batch of alignments (plm_fit is a batch of one).
int run_fit_once(plm_ctx* c, const plm_msa_desc* d, int32_t n, int32_t q, const plm_fit_opts* o,
                 void* ws, size_t ws_bytes, const ProbeArgs* probe) {
  Prep P;
  int rc = prepare_fit(c, d, n, q, o, ws, ws_bytes, &P);
  if (rc) return rc;
  const PathSpec& ps = P.ps;
  const int32_t nb = P.nb, total = P.total;
  const Grids& g = P.g;
  const Tables& t = P.t;
  const BatchArgs& b = P.b;
  const std::vector<int32_t>& ord = P.ord;
  const std::vector<int32_t>& base = P.base;
  hipStream_t st = P.st;
  volatile int32_t* phase_host = c->pin + 2;

  const int64_t cap = (int64_t)o->max_iter * (o->max_linesearch + 2) + 16;
  if (o->single_site) {
    // the plain path: one site at a time, the host waiting for every iteration
    const int32_t nsites = (o->site_limit > 0 && o->site_limit < total) ? o->site_limit : total;
    for (int32_t r = 0; r < nsites; ++r) {
      for (int64_t it = 0; it < cap; ++it) {
        HIPCHK(c, launch_list_tables(b, nullptr, r, 1, nullptr, st));
        HIPCHK(c, eval_forward(ps, b, nb, g, st));
        HIPCHK(c, eval_backward(ps, b, g, st));
        HIPCHK(c, launch_lbfgs(b, 1, o->history_fp64, st));
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
      if (e == hipSuccess) e = eval_quant(ps, b, st);
      if (e == hipSuccess) e = mark(4);
      if (e == hipSuccess) e = eval_forward_main(ps, b, nb, g, st);
      if (e == hipSuccess) e = mark(1);
      if (e == hipSuccess) e = eval_backward(ps, b, g, st);
      if (e == hipSuccess) e = mark(2);
      if (e == hipSuccess) e = launch_lbfgs(b, total, o->history_fp64, st);
      if (e == hipSuccess) e = mark(3);
      if (e == hipSuccess) e = launch_compact(b, t.st, c->pin_dev + 1, t.site_evals, st);
      if (e == hipSuccess && probe) e = launch_probe(*probe, st);
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
        float t01 = 0.f, t12 = 0.f, t23 = 0.f, t04 = 0.f;
        if (hipEventElapsedTime(&t01, c->ev[0], c->ev[1]) == hipSuccess &&
            hipEventElapsedTime(&t12, c->ev[1], c->ev[2]) == hipSuccess &&
            hipEventElapsedTime(&t23, c->ev[2], c->ev[3]) == hipSuccess &&
            hipEventElapsedTime(&t04, c->ev[0], c->ev[4]) == hipSuccess) {
          tm.forward_ms += t01;
          tm.quant_ms += t04;
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
      (void)hipMemcpy(&se, t.site_evals, sizeof(se), hipMemcpyDeviceToHost);
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
  std::vector<SiteState> hs(total);
  HIPCHK(c, hipMemcpy(hs.data(), t.st, sizeof(SiteState) * total, hipMemcpyDeviceToHost));
  int any_max = 0;
  for (int32_t k = 0; k < n; ++k) {
    const plm_msa_desc& m = d[ord[k]];
    for (int32_t r = 0; r < m.N; ++r) {
      const SiteState& S = hs[base[k] + r];
      int status = S.phase == PH_DONE ? S.status : PLM_SITE_MAXITER;
      if (status == PLM_SITE_MAXITER) any_max = 1;
      if (m.stats_out) {
        m.stats_out[r].iterations = S.iter;
        m.stats_out[r].evaluations = S.evals;
        m.stats_out[r].status = status;
        m.stats_out[r].pad = 0;
        m.stats_out[r].f = S.f;
        m.stats_out[r].gnorm = S.gnorm;
      }
    }
  }
  return any_max ? PLM_W_MAXITER : PLM_OK;
}

// the refinement path of plm_fit_opts.refine, or -1
int32_t refine_path(const plm_fit_opts* o) {
  if (o->refine == 0) {
    if (o->path == PLM_PATH_MFMA_I8X3) return PLM_PATH_GATHER_MFMA_I8X3;
    if (o->path == PLM_PATH_MFMA_BF16X2) return PLM_PATH_MFMA_FP32;
    return -1;
  }
  if (o->refine < 0) return -1;
  const int32_t p = o->refine - 1;
  return p == o->path ? -1 : p;
}

// The fit, then (plm_fit_opts.refine) a second fit from its point on another
// path; the site statistics and the kernel times add both.
int run_fit(plm_ctx* c, const plm_msa_desc* d, int32_t n, int32_t q, const plm_fit_opts* o,
            void* ws, size_t ws_bytes) {
  const int32_t rp = refine_path(o);
  if (rp >= 0 && (rp < PLM_PATH_GATHER_FP32 || rp > PLM_PATH_GATHER64_MFMA_I8X6))
    return set_err(c, PLM_E_INVALID, "refine: unknown path %d", rp);
  if (!fit_opts_ok(o)) return set_err(c, PLM_E_INVALID, "invalid fit options");
  ProbeArgs pa;
  const ProbeArgs* probe = nullptr;
  if (o->n_probe > 0) {
    if (n != 1 || o->single_site)
      return set_err(c, PLM_E_INVALID, "the convergence probe watches a single alignment's batched fit");
    int khz = 0;
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, c->device));
    if (khz <= 0) return set_err(c, PLM_E_UNSUPPORTED, "device wall clock rate unknown");
    pa.N = d[0].N; pa.q = q; pa.n = o->n_probe; pa.cap = o->probe_cap;
    pa.Xh = d[0].h_io; pa.XJ = d[0].J_io;
    pa.sites = o->probe_sites; pa.ref_h = o->probe_h; pa.ref_J = o->probe_J;
    pa.out = o->probe_out; pa.count = o->probe_count;
    pa.sec_per_tick = 1.0 / (1e3 * (double)khz);
    probe = &pa;
    // the first entry: the start point, once the caller's stream has delivered it
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, launch_probe(pa, c->fit_stream));
  }
  int rc = run_fit_once(c, d, n, q, o, ws, ws_bytes, probe);
  if (rp < 0 || (rc != PLM_OK && rc != PLM_W_MAXITER)) return rc;
  std::vector<std::vector<plm_site_stats>> first(n);
  for (int32_t k = 0; k < n; ++k)
    if (d[k].stats_out) first[k].assign(d[k].stats_out, d[k].stats_out + d[k].N);
  const plm_fit_timing t1 = c->timing;
  plm_fit_opts o2 = *o;
  o2.path = rp;
  o2.refine = -1;
  o2.tile_seqs = 0;
  if (o->refine_tol > 0.0) o2.tol = o->refine_tol;
  const int rc2 = run_fit_once(c, d, n, q, &o2, ws, ws_bytes, probe);
  if (rc2 != PLM_OK && rc2 != PLM_W_MAXITER) return rc2;
  for (int32_t k = 0; k < n; ++k)
    if (d[k].stats_out)
      for (int32_t r = 0; r < d[k].N; ++r) {
        d[k].stats_out[r].iterations += first[k][r].iterations;
        d[k].stats_out[r].evaluations += first[k][r].evaluations;
      }
  if (o->timing) {
    plm_fit_timing& t = c->timing;
    t.refine_forward_ms = t.forward_ms;
    t.refine_backward_ms = t.backward_ms;
    t.refine_lbfgs_ms = t.lbfgs_ms;
    t.refine_iterations = t.iterations;
    t.refine_site_evals = t.site_evals;
    t.forward_ms += t1.forward_ms;
    t.backward_ms += t1.backward_ms;
    t.lbfgs_ms += t1.lbfgs_ms;
    t.quant_ms += t1.quant_ms;
    t.total_ms += t1.total_ms;
    t.iterations += t1.iterations;
    t.site_evals += t1.site_evals;
  }
  return rc2;
}

plm_msa_desc single_desc(const uint8_t* msa, int32_t B, int32_t N, const double* w, const double* beff,
                         float* h_io, float* J_io, plm_site_stats* stats_out) {
  plm_msa_desc d;
  d.msa = msa; d.B = B; d.N = N; d.w = w; d.beff = beff; d.h_io = h_io; d.J_io = J_io;
  d.stats_out = stats_out;
  return d;
}

}  // namespace

extern "C" {

size_t plm_fit_workspace_bytes(int32_t B, int32_t N, int32_t q, const plm_fit_opts* o) {
  if (B < 1 || N < 2 || q < 2 || q > kQMax || !o) return 0;
  if (o->lbfgs_m < 1 || o->lbfgs_m > kMMax) return 0;
  const plm_msa_desc d = single_desc(nullptr, B, N, nullptr, nullptr, nullptr, nullptr, nullptr);
  return fit_layout(&d, 1, q, o, nullptr, nullptr, nullptr);
}

int plm_fit(plm_ctx* c, const uint8_t* msa, int32_t B, int32_t N, int32_t q, const double* w,
            const double* beff, const plm_fit_opts* o, void* ws, size_t ws_bytes, float* h_io,
            float* J_io, plm_site_stats* stats_out) {
  if (!c) return PLM_E_INVALID;
  if (!msa || !w || !beff || !o || !h_io || !J_io) return set_err(c, PLM_E_INVALID, "null pointer");
  const plm_msa_desc d = single_desc(msa, B, N, w, beff, h_io, J_io, stats_out);
  return run_fit(c, &d, 1, q, o, ws, ws_bytes);
}

size_t plm_fit_batch_workspace_bytes(const plm_msa_desc* descs, int32_t n_msas, int32_t q,
                                     const plm_fit_opts* o) {
  if (!descs || n_msas < 1 || !o || q < 2 || q > kQMax) return 0;
  if (o->lbfgs_m < 1 || o->lbfgs_m > kMMax) return 0;
  for (int32_t k = 0; k < n_msas; ++k)
    if (descs[k].B < 1 || descs[k].N < 2) return 0;
  return fit_layout(descs, n_msas, q, o, nullptr, nullptr, nullptr);
}

int plm_fit_batch(plm_ctx* c, const plm_msa_desc* descs, int32_t n_msas, int32_t q,
                  const plm_fit_opts* o, void* ws, size_t ws_bytes) {
  if (!c) return PLM_E_INVALID;
  if (!descs || !o || n_msas < 1) return set_err(c, PLM_E_INVALID, "null pointer or empty batch");
  if (o->single_site) return set_err(c, PLM_E_INVALID, "single_site is not available for batches");
  return run_fit(c, descs, n_msas, q, o, ws, ws_bytes);
}

int plm_tune(plm_ctx* c, const plm_msa_desc* descs, int32_t n_msas, int32_t q, const plm_fit_opts* o,
             int32_t fp32_only, void* ws, size_t ws_bytes, plm_tune_result* out, int32_t max_out,
             int32_t* n_out) {
  if (!c) return PLM_E_INVALID;
  if (!descs || !o || n_msas < 1 || !out || max_out < 1 || !n_out)
    return set_err(c, PLM_E_INVALID, "null pointer or empty batch");
  if (o->single_site) return set_err(c, PLM_E_INVALID, "single_site cannot be tuned");
  struct Cand {
    int32_t path, tile;
  };
  std::vector<Cand> cands;
  const int32_t paths[] = {PLM_PATH_MFMA_I8X3,   PLM_PATH_GATHER_MFMA_I8X3, PLM_PATH_GATHER_MFMA_F16X2,
                           PLM_PATH_GATHER_MFMA_FP32, PLM_PATH_GATHER_FP32,    PLM_PATH_MFMA_FP32,
                           PLM_PATH_MFMA_BF16X2};
  for (int32_t p : paths) {
    if (fp32_only && p == PLM_PATH_MFMA_BF16X2) continue;
    PathSpec ps;
    path_spec(p, &ps);
    bool fits = true;
    for (int32_t k = 0; k < n_msas; ++k) fits = fits && path_fits(ps, descs[k].B);
    if (!fits) continue;
    if (ps.fwd_np || ps.fwd_i8) {
      cands.push_back({p, 0});
    } else {
      for (int32_t tl : {16, 32, 64}) cands.push_back({p, tl});
    }
  }
  std::vector<plm_tune_result> res;
  for (const Cand& cd : cands) {
    plm_fit_opts oc = *o;
    oc.path = cd.path;
    oc.tile_seqs = cd.tile;
    oc.single_site = 0;
    Prep P;
    int rc = prepare_fit(c, descs, n_msas, q, &oc, ws, ws_bytes, &P);
    if (rc) return rc;
    // one untimed and three timed all-sites evaluations; the shortest counts
    float best = 1e30f;
    for (int rep = 0; rep < 4; ++rep) {
      HIPCHK(c, launch_compact(P.b, P.t.st, nullptr, nullptr, P.st));  // clears the queues
      HIPCHK(c, hipEventRecord(c->ev[0], P.st));
      HIPCHK(c, eval_forward(P.ps, P.b, P.nb, P.g, P.st));
      HIPCHK(c, eval_backward(P.ps, P.b, P.g, P.st));
      HIPCHK(c, hipEventRecord(c->ev[1], P.st));
      HIPCHK(c, hipStreamSynchronize(P.st));
      float ms = 0.f;
      HIPCHK(c, hipEventElapsedTime(&ms, c->ev[0], c->ev[1]));
      if (rep > 0 && ms < best) best = ms;
    }
    plm_tune_result r;
    r.path = cd.path;
    r.tile_seqs = cd.tile == 0 ? 0 : pick_nb(0, cd.tile);
    r.eval_ms = best;
    res.push_back(r);
  }
  std::stable_sort(res.begin(), res.end(),
                   [](const plm_tune_result& x, const plm_tune_result& y) { return x.eval_ms < y.eval_ms; });
  const int32_t k = (int32_t)res.size() < max_out ? (int32_t)res.size() : max_out;
  for (int32_t j = 0; j < k; ++j) out[j] = res[j];
  *n_out = k;
  return PLM_OK;
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

size_t plm_mf_init_workspace_bytes(int32_t B, int32_t N, int32_t q) {
  if (B < 1 || N < 2 || q < 2 || q > kQMax) return 0;
  const size_t tile = (size_t)mf_tile();
  const size_t n = (size_t)N * (q - 1), n_pad = (n + tile - 1) / tile * tile;
  Bump bp{nullptr, 0};
  bp.take<int32_t>((size_t)N * B);
  bp.take<int32_t>((size_t)N * (q + 1));
  bp.take<double>((size_t)N * q);
  bp.take<double>(n_pad * n_pad);
  return rup(bp.off, 256);
}

int plm_mf_init(plm_ctx* c, const uint8_t* msa, int32_t B, int32_t N, int32_t q, const double* w,
                const double* beff, double pseudocount, void* ws, size_t ws_bytes, float* h_out, float* J_out) {
  if (!c) return PLM_E_INVALID;
  if (!msa || !w || !beff || !h_out || !J_out) return set_err(c, PLM_E_INVALID, "null pointer");
  int rc = check_sizes(c, B, N, q);
  if (rc) return rc;
  if (!(pseudocount >= 0.0 && pseudocount <= 1.0)) return set_err(c, PLM_E_INVALID, "pseudocount outside [0, 1]");
  rc = check_ws(c, ws, ws_bytes, plm_mf_init_workspace_bytes(B, N, q));
  if (rc) return rc;
  HIPCHK(c, hipSetDevice(c->device));
  const int32_t tile = mf_tile();
  const int32_t n = N * (q - 1), n_pad = (n + tile - 1) / tile * tile;
  Bump bp{(char*)ws, 0};
  int32_t* order = bp.take<int32_t>((size_t)N * B);
  int32_t* start = bp.take<int32_t>((size_t)N * (q + 1));
  double* fi = bp.take<double>((size_t)N * q);
  double* C = bp.take<double>((size_t)n_pad * n_pad);
  hipStream_t st = c->stream;
  HIPCHK(c, launch_check_f64(w, (size_t)B, c->pin_dev, st));
  HIPCHK(c, launch_mf_frequencies(msa, B, N, q, w, beff, pseudocount, order, start, fi, c->pin_dev, st));
  HIPCHK(c, launch_mf_correlation(msa, order, start, w, beff, fi, B, N, q, pseudocount, C, n_pad, st));
  HIPCHK(c, launch_mf_invert(C, n_pad, c->pin_dev, st));
  HIPCHK(c, launch_mf_output(C, n_pad, fi, N, q, h_out, J_out, c->pin_dev, st));
  HIPCHK(c, hipStreamSynchronize(st));
  return flags_status(c);
}

size_t plm_fit_symmetric_workspace_bytes(int32_t B, int32_t N, int32_t q, const plm_fit_opts* o) {
  if (B < 1 || N < 2 || q < 2 || q > kQMax || !o) return 0;
  if (o->lbfgs_m < 1 || o->lbfgs_m > kMMax) return 0;
  int dev = 0, ncu = 256;
  if (hipGetDevice(&dev) == hipSuccess) {
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) == hipSuccess && p.multiProcessorCount > 0) ncu = p.multiProcessorCount;
  }
  Bump bp{nullptr, 0};
  SymBufs f;
  layout_sym(bp, B, N, q, o->lbfgs_m, 4 * ncu, sym_wide(o), f);
  return rup(bp.off, 256);
}

}  // extern "C"

namespace {

int run_sym_once(plm_ctx* c, const uint8_t* msa, int32_t B, int32_t N, int32_t q, const double* w,
                 const double* beff, const plm_fit_opts* o, void* ws, size_t ws_bytes, float* h_io,
                 float* J_io, float* h_lo_io, float* J_lo_io, plm_site_stats* stats_out) {
  if (!c) return PLM_E_INVALID;
  if (!msa || !w || !beff || !o || !h_io || !J_io) return set_err(c, PLM_E_INVALID, "null pointer");
  if ((h_lo_io == nullptr) != (J_lo_io == nullptr))
    return set_err(c, PLM_E_INVALID, "pass both low-order arrays or neither");
  const bool lo = h_lo_io != nullptr;
  int rc = check_sizes(c, B, N, q);
  if (rc) return rc;
  if (!fit_opts_ok(o) || o->single_site) return set_err(c, PLM_E_INVALID, "invalid fit options");
  PathSpec ps;
  if (!path_spec(o->path, &ps))
    return set_err(c, PLM_E_UNSUPPORTED, "evaluation path %d is not available", o->path);
  // the precise path evaluates at high + low words (its forward's low-word
  // instance); the other paths read the high words
  if (lo && ps.f64) ps.f64 = 2;
  if (!path_fits(ps, B)) return set_err(c, PLM_E_UNSUPPORTED, "path %d sums at most 2^24 - 1 sequences exactly", o->path);
  HIPCHK(c, hipSetDevice(c->device));
  const int32_t nblk = 4 * c->ncu;
  {
    Bump bq{nullptr, 0};
    SymBufs fq;
    layout_sym(bq, B, N, q, o->lbfgs_m, nblk, sym_wide(o), fq);
    rc = check_ws(c, ws, ws_bytes, rup(bq.off, 256));
    if (rc) return rc;
  }
  rc = ensure_pin(c, 3);
  if (rc) return rc;
  Bump bp{(char*)ws, 0};
  SymBufs f;
  layout_sym(bp, B, N, q, o->lbfgs_m, nblk, sym_wide(o), f);
  HIPCHK(c, hipStreamSynchronize(c->stream));
  hipStream_t st = c->fit_stream;
  c->pin[2] = 0;

  std::vector<int2> pairs;
  pairs.reserve((size_t)N * (N - 1) / 2);
  for (int32_t r = 0; r < N; ++r)
    for (int32_t i = r + 1; i < N; ++i) pairs.push_back(make_int2(r, i));
  HIPCHK(c, hipMemcpyAsync(f.pairs, pairs.data(), pairs.size() * sizeof(int2), hipMemcpyHostToDevice, st));

  const int32_t nb = pick_nb(B, o->tile_seqs);
  const BatchArgs b = batch_args(f.t, 1, N, bwd_group(ps), fwd_group(ps));
  HIPCHK(c, launch_check_f64(w, (size_t)B, c->pin_dev, st));
  HIPCHK(c, launch_check_f32(h_io, (size_t)N * q, c->pin_dev, st));
  HIPCHK(c, launch_check_f32(J_io, (size_t)N * N * q * q, c->pin_dev, st));
  if (lo) {
    HIPCHK(c, launch_check_f32(h_lo_io, (size_t)N * q, c->pin_dev, st));
    HIPCHK(c, launch_check_f32(J_lo_io, (size_t)N * N * q * q, c->pin_dev, st));
  }
  HIPCHK(c, launch_pad_msa(msa, B, N, q, f.ev.msa_cm, f.ev.B_pad, f.ev.N_pad, c->pin_dev, st));
  EvalArgs a = eval_args(f.ev, msa, B, N, q, w, f.Th, f.TJ, eval_tiles(ps, B, nb), ps);
  if (ps.f64 == 2) {
    a.h_lo = f.Thl;
    a.J_lo = f.TJl;
  }
  HIPCHK(c, eval_prepare(ps, a, f.ev.msaT, f.ev.sorted, st));
  HIPCHK(c, launch_setup_msa(b, 0, a, nullptr, 0, N, a.tiles, eval_bwd_blocks(ps, N, q), nullptr, st));
  HIPCHK(c, launch_list_tables(b, nullptr, 0, N, nullptr, st));

  SymArgs S;
  S.N = N; S.q = q; S.m = o->lbfgs_m; S.max_iter = o->max_iter; S.max_ls = o->max_linesearch;
  S.tiles = a.tiles; S.nblk = nblk; S.npairs = (int32_t)pairs.size();
  S.tol = o->tol; S.lambda_h = o->lambda_h; S.lambda_J = o->lambda_J; S.c1 = 1e-4; S.noise = ps.f64 ? 2e-14 : 1e-7;
  S.beff = beff;
  S.Xh = h_io; S.XJ = J_io; S.Th = f.Th; S.TJ = f.TJ;
  S.Xhl = h_lo_io; S.XJl = J_lo_io;
  S.Thl = lo ? f.Thl : nullptr; S.TJl = lo ? f.TJl : nullptr;
  S.Gh = f.Gh; S.GJ = f.GJ; S.Dh = f.Dh; S.DJ = f.DJ;
  S.Sh = f.Sh; S.SJ = f.SJ; S.Yh = f.Yh; S.YJ = f.YJ;
  S.f_part = f.ev.f_part; S.gh_part = f.ev.gh_part; S.gJ = f.ev.gJ;
  S.part = f.part; S.small = f.small; S.coef = f.coef; S.st = f.st; S.pairs = f.pairs;
  S.done_host = c->pin_dev + 2;
  HIPCHK(c, launch_sym_init(S, st));
  HIPCHK(c, hipStreamSynchronize(st));
  rc = flags_status(c);
  if (rc) return rc;
  const Grids g = eval_grids(c, ps, nb);

  const bool timed = o->timing != 0;
  auto mark = [&](int k) -> hipError_t { return timed ? hipEventRecord(c->ev[k], st) : hipSuccess; };
  auto enqueue = [&]() -> hipError_t {
    hipError_t e = mark(0);
    if (e == hipSuccess) e = eval_quant(ps, b, st);
    if (e == hipSuccess) e = mark(4);
    if (e == hipSuccess) e = eval_forward_main(ps, b, nb, g, st);
    if (e == hipSuccess) e = mark(1);
    if (e == hipSuccess) e = eval_backward(ps, b, g, st);
    if (e == hipSuccess) e = mark(2);
    if (e == hipSuccess) e = launch_sym_step(S, b, st);
    if (e == hipSuccess) e = mark(3);
    return e;
  };
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  const bool use_graph = o->use_graph && !timed;
  if (use_graph) {
    HIPCHK(c, hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    hipError_t e = enqueue();
    hipError_t e2 = hipStreamEndCapture(st, &graph);
    if (e != hipSuccess) return set_err(c, PLM_E_HIP, "capture: %s", hipGetErrorString(e));
    HIPCHK(c, e2);
    HIPCHK(c, hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
  }
  plm_fit_timing tm;
  memset(&tm, 0, sizeof(tm));
  const int64_t cap = (int64_t)o->max_iter * (o->max_linesearch + 2) + 16;
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
      float t01 = 0.f, t12 = 0.f, t23 = 0.f, t04 = 0.f;
      if (hipEventElapsedTime(&t01, c->ev[0], c->ev[1]) == hipSuccess &&
          hipEventElapsedTime(&t12, c->ev[1], c->ev[2]) == hipSuccess &&
          hipEventElapsedTime(&t23, c->ev[2], c->ev[3]) == hipSuccess &&
          hipEventElapsedTime(&t04, c->ev[0], c->ev[4]) == hipSuccess) {
        tm.forward_ms += t01;
        tm.quant_ms += t04;
        tm.backward_ms += t12;
        tm.lbfgs_ms += t23;
      } else {
        (void)hipGetLastError();
      }
      tm.iterations += 1;
    }
    if (((volatile int32_t*)c->pin)[2] == 1) break;
  }
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
  if (err) return err;
  HIPCHK(c, hipStreamSynchronize(st));
  rc = flags_status(c);
  if (rc) return rc;
  SymState hs;
  HIPCHK(c, hipMemcpy(&hs, f.st, sizeof(hs), hipMemcpyDeviceToHost));
  if (timed) {
    tm.site_evals = (int64_t)hs.evals * N;
    tm.total_ms = tm.forward_ms + tm.backward_ms + tm.lbfgs_ms;
    c->timing = tm;
  }
  const int status = hs.phase == PH_DONE ? hs.status : PLM_SITE_MAXITER;
  if (stats_out) {
    stats_out->iterations = hs.iter;
    stats_out->evaluations = hs.evals;
    stats_out->status = status;
    stats_out->pad = 0;
    stats_out->f = hs.f;
    stats_out->gnorm = hs.gnorm;
  }
  return status == PLM_SITE_MAXITER ? PLM_W_MAXITER : PLM_OK;
}

// Refinement path of the symmetric fit: automatic after either fixed-point
// path (their rounding noise, summed over all parameters, is of the order of
// the tolerance), on the precise path (FP64 energies and residuals): the FP32
// evaluations' own rounding, summed over the N(N-1)/2 q^2 couplings, is of the
// order of 1e-6 at N = 500.
int32_t refine_path_sym(const plm_fit_opts* o) {
  if (o->refine == 0)
    return (o->path == PLM_PATH_GATHER_MFMA_I8X3 || o->path == PLM_PATH_MFMA_I8X3) ? PLM_PATH_GATHER64_MFMA_I8X6
                                                                                   : -1;
  if (o->refine < 0) return -1;
  const int32_t p = o->refine - 1;
  return p == o->path ? -1 : p;
}

}  // namespace

extern "C" {

int plm_fit_symmetric_split(plm_ctx* c, const uint8_t* msa, int32_t B, int32_t N, int32_t q, const double* w,
                            const double* beff, const plm_fit_opts* o, void* ws, size_t ws_bytes, float* h_io,
                            float* J_io, float* h_lo_io, float* J_lo_io, plm_site_stats* stats_out) {
  if (!c) return PLM_E_INVALID;
  if (!o) return set_err(c, PLM_E_INVALID, "null pointer");
  const int32_t rp = refine_path_sym(o);
  if (rp >= 0 && (rp < PLM_PATH_GATHER_FP32 || rp > PLM_PATH_GATHER64_MFMA_I8X6))
    return set_err(c, PLM_E_INVALID, "refine: unknown path %d", rp);
  plm_site_stats first;
  memset(&first, 0, sizeof(first));
  int rc = run_sym_once(c, msa, B, N, q, w, beff, o, ws, ws_bytes, h_io, J_io, h_lo_io, J_lo_io, &first);
  if (rp < 0 || (rc != PLM_OK && rc != PLM_W_MAXITER)) {
    if (stats_out && (rc == PLM_OK || rc == PLM_W_MAXITER)) *stats_out = first;
    return rc;
  }
  // a second fit from the first one's point on the refinement path: the
  // statistics and the kernel times add both
  const plm_fit_timing t1 = c->timing;
  plm_fit_opts o2 = *o;
  o2.path = rp;
  o2.refine = -1;
  o2.tile_seqs = 0;
  if (o->refine_tol > 0.0) o2.tol = o->refine_tol;
  plm_site_stats second;
  memset(&second, 0, sizeof(second));
  const int rc2 = run_sym_once(c, msa, B, N, q, w, beff, &o2, ws, ws_bytes, h_io, J_io, h_lo_io, J_lo_io, &second);
  if (rc2 != PLM_OK && rc2 != PLM_W_MAXITER) return rc2;
  second.iterations += first.iterations;
  second.evaluations += first.evaluations;
  if (stats_out) *stats_out = second;
  if (o->timing) {
    plm_fit_timing& t = c->timing;
    t.refine_forward_ms = t.forward_ms;
    t.refine_backward_ms = t.backward_ms;
    t.refine_lbfgs_ms = t.lbfgs_ms;
    t.refine_iterations = t.iterations;
    t.refine_site_evals = t.site_evals;
    t.forward_ms += t1.forward_ms;
    t.backward_ms += t1.backward_ms;
    t.lbfgs_ms += t1.lbfgs_ms;
    t.quant_ms += t1.quant_ms;
    t.total_ms += t1.total_ms;
    t.iterations += t1.iterations;
    t.site_evals += t1.site_evals;
  }
  return rc2;
}

int plm_fit_symmetric(plm_ctx* c, const uint8_t* msa, int32_t B, int32_t N, int32_t q, const double* w,
                      const double* beff, const plm_fit_opts* o, void* ws, size_t ws_bytes, float* h_io,
                      float* J_io, plm_site_stats* stats_out) {
  return plm_fit_symmetric_split(c, msa, B, N, q, w, beff, o, ws, ws_bytes, h_io, J_io, nullptr, nullptr,
                                 stats_out);
}

void plm_score_opts_default(plm_score_opts* o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->combine = PLM_COMBINE_AVG;
  o->norm = PLM_NORM_FROB;
  o->p = 2.0;
  o->exclude_gap = 0;
  o->correction = PLM_CORR_APC;
}

int plm_frequencies(plm_ctx* c, const uint8_t* msa, int32_t B, int32_t N, int32_t q, const double* w,
                    const double* beff, double* f_out) {
  if (!c) return PLM_E_INVALID;
  if (!msa || !w || !beff || !f_out) return set_err(c, PLM_E_INVALID, "null pointer");
  int rc = check_sizes(c, B, N, q);
  if (rc) return rc;
  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, launch_frequencies(msa, B, N, q, w, beff, f_out, c->stream));
  return PLM_OK;
}

int plm_score_ex(plm_ctx* c, const float* J, int32_t N, int32_t q, const plm_score_opts* o,
                 const double* freq, double* raw_out, double* corrected_out) {
  if (!c) return PLM_E_INVALID;
  if (!J || !o || !raw_out || !corrected_out) return set_err(c, PLM_E_INVALID, "null pointer");
  if (N < 2 || q < 2 || q > kQMax) return set_err(c, PLM_E_INVALID, "unsupported sizes");
  if (o->combine < PLM_COMBINE_AVG || o->combine > PLM_COMBINE_MAX || o->norm < PLM_NORM_FROB ||
      o->norm > PLM_NORM_BURKOFF || o->correction < PLM_CORR_APC || o->correction > PLM_CORR_ASC ||
      (o->norm == PLM_NORM_LP && !(o->p > 0.0)) || (o->exclude_gap && q < 3))
    return set_err(c, PLM_E_INVALID, "invalid score options");
  if (o->norm == PLM_NORM_BURKOFF && !freq)
    return set_err(c, PLM_E_INVALID, "the Burkoff score needs the frequencies");
  HIPCHK(c, hipSetDevice(c->device));
  ScoreOpts so;
  so.combine = o->combine;
  so.norm = o->norm;
  so.p = o->p;
  so.exclude_gap = o->exclude_gap;
  so.correction = o->correction;
  HIPCHK(c, launch_score_ex(J, N, q, so, freq, raw_out, corrected_out, c->stream));
  return PLM_OK;
}

int plm_contact_tpr(plm_ctx* c, const double* score, int32_t N, const uint8_t* contacts,
                    int32_t min_sep, int32_t kmax, double* tpr_out, int32_t* n_out) {
  if (!c) return PLM_E_INVALID;
  if (!score || !contacts || !tpr_out || !n_out) return set_err(c, PLM_E_INVALID, "null pointer");
  if (N < 2 || min_sep < 1 || kmax < 1) return set_err(c, PLM_E_INVALID, "invalid sizes");
  HIPCHK(c, hipSetDevice(c->device));
  const size_t NN = (size_t)N * N;
  std::vector<double> S(NN);
  std::vector<uint8_t> C(NN);
  HIPCHK(c, hipMemcpyAsync(S.data(), score, NN * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(C.data(), contacts, NN, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  std::vector<std::pair<int32_t, int32_t>> pairs;
  for (int32_t i = 0; i < N; ++i)
    for (int32_t j = i + min_sep; j < N; ++j) pairs.emplace_back(i, j);
  std::stable_sort(pairs.begin(), pairs.end(), [&](const std::pair<int32_t, int32_t>& x,
                                                   const std::pair<int32_t, int32_t>& y) {
    return S[(size_t)x.first * N + x.second] > S[(size_t)y.first * N + y.second];
  });
  const int32_t n = (int32_t)pairs.size() < kmax ? (int32_t)pairs.size() : kmax;
  int64_t hits = 0;
  for (int32_t k = 0; k < n; ++k) {
    if (C[(size_t)pairs[k].first * N + pairs[k].second]) ++hits;
    tpr_out[k] = (double)hits / (double)(k + 1);
  }
  *n_out = n;
  return PLM_OK;
}

}  // extern "C"
