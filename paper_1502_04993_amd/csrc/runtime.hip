// glmrec runtime: contexts, device memory, the evaluation pipeline, the
// per-row ascent driver, batching and the C ABI of include/glmrec.h.
//
// One evaluation at fixed tau (the carries and dSigma are cached per tau):
//   for each time chunk of L bins:
//     kernel U   V = J x  -> W = exp(V) [Np x L], per-tile row sums of W
//     kernel V   (dL/dtau only) Y-contraction, per-tile row sums of W V
//     kernel G   per-split partials of W x^T over the chunk
//     reduce     partials -> G (FP64, fixed order, accumulated over chunks)
//   reduce row sums (FP64, fixed order); assemble L_i, dL/dmu, dL/dJ, dL/dtau.
// Nothing is accumulated with atomics, so two evaluations of the same input
// give bitwise-identical results.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstddef>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/glmrec.h"
#include "common.h"

void gemm_tiles(int prec, int tile, int* bi1, int* bt1, int* bi2, int* bj2);
int64_t ingest_scan_tmp_len(int64_t nseg);
int64_t rowpart_tmp_len(int64_t Np);

namespace {

template <typename T>
struct DBuf {
  T* p = nullptr;
  size_t n = 0;
};

struct ProfRec {
  int kind;
  hipEvent_t a, b;
};

const char* const kKindNames[] = {"ingest",       "carries",     "spike_term", "kernel_U",
                                  "kernel_V",     "kernel_G",    "reduce_G",   "assemble",
                                  "prepare",      "ascent",      "batch_U",    "batch_G",
                                  "trace_build",  "self_delay"};
enum {
  K_INGEST, K_CARRY, K_SPIKE, K_U, K_V, K_G, K_RED, K_ASM, K_PREP, K_ASC, K_BU, K_BG, K_XBUILD,
  K_SELF, K_NKIND
};

}  // namespace

struct glmr_ctx {
  glmr_config cfg{};
  int N = 0;
  int64_t B = 0;
  double dt = 0;
  int prec = 0;
  int tile = 256;
  int64_t Np = 0, Bp = 0, NS = 0, NIB = 0, L = 0;
  int bi1 = 0, bt1 = 0, bi2 = 0, bj2 = 0;
  hipStream_t st = nullptr;
  bool own_stream = false;
  std::string err;
  std::vector<void*> allocs;

  // spikes
  bool have_spikes = false;
  int64_t nspk = 0;
  int planes = 1;
  int32_t* seg_off = nullptr;
  uint16_t* seg_ent = nullptr;
  uint64_t* masks = nullptr;
  int64_t* q = nullptr;
  std::vector<int64_t> q_host;
  bool all_spiking = false;
  uint64_t raster_digest = 0;  // digest of the recorded masks (and, on the event grid, the slot times)

  // event grid (continuous time): slot start times and per-slot tables
  bool evm = false;
  double T0 = 0, T1 = 0, max_gap = 0;
  double* tslot = nullptr;  // [NS*64 + 1]
  double* evtab = nullptr;  // [5 * NS*64 + NS]: pw, ainv, left, delta, edec, asub
  float* evgl = nullptr;    // BF16: [NS*64][16] per-slot table of kernel U's interval integrals
  double max_span = 0;      // largest 64-slot span / tau of the current tables

  // transmission delays in bins (regular grid): d on j -> i (j != i), d_s on i -> i
  int64_t dly = 0, dly_s = 0;
  uint64_t* masks0 = nullptr;  // recorded raster's masks when delayed (masks is the shifted one)
  double* C0 = nullptr;        // its carries when d_s != d
  double* gpart = nullptr;     // [Bp/bt1][Np] self-delay correction of G_ii per tile
  double* gself = nullptr;     // [Np]

  // kernel
  bool have_kernel = false, have_y = false, keep_y = false;
  double tau = 0, a = 0;
  Tables* tab = nullptr;
  double* C64 = nullptr;
  double* CY64 = nullptr;
  float* C32 = nullptr;
  float* CY32 = nullptr;
  double* dsig = nullptr;
  double* dsigY = nullptr;
  // resident trace (BF16): Xtj [Bp][Np] and Xjt [Np][Bp], rebuilt per tau
  bool resident = false;
  unsigned char* Xtj = nullptr;
  unsigned char* Xjt = nullptr;
  int res_shape_u = 1, res_shape_g = 1;  // indices into res_shapes()
  int xfrag = 0;                         // BF16: Xtj, Xjt and W as MFMA fragments
  size_t x_bytes = 0;                    // bytes of each layout as allocated
  unsigned* xmax = nullptr;              // FP8: per-chunk trace maxima
  float* xscale = nullptr;               // FP8: per-chunk trace scales
  int64_t x_nchunks = 0;                 // FP8: entries of xmax / xscale
  float* jscale = nullptr;               // FP8: per-row scales of J

  // parameters (padded FP64 masters and the compute-precision copy)
  bool have_params = false;
  bool j2 = false;  // GLMR_BF16_J2: J staged as two BF16 terms (prec is PREC_BF16)
  double* J64 = nullptr;
  double* mu = nullptr;
  void* Jc = nullptr;
  double* Jr = nullptr;
  double* rowscale = nullptr;

  // evaluation workspace
  void* W = nullptr;
  void* Gp = nullptr;
  int max_splits = 0;
  double* G64 = nullptr;
  double* rowpart = nullptr;
  double* rowpartV = nullptr;
  double* rowsum = nullptr;
  double* rowsumV = nullptr;
  double* rp_tmp = nullptr;
  double* ll_rows = nullptr;
  double* gJ = nullptr;
  double* gmu = nullptr;
  double* tau_rows = nullptr;
  double* scal = nullptr;  // [4] device scalars
  double* host_scal = nullptr;

  // ascent state
  AscentArgs asc{};
  bool have_asc = false;
  bool asc_live = false;  // asc holds an ascent of the current objective that a fit can resume
  bool asc_hist = false;  // asc holds L-BFGS pairs of this recording, kernel and delays (any precision)
  int32_t* counters = nullptr;
  int32_t* host_cnt = nullptr;  // pinned copy of counters
  bool capturing = false;       // work is being captured into a graph (no profiling events)

  // profiling
  bool prof = false;
  std::vector<ProfRec> pending;
  std::vector<hipEvent_t> pool;
  double prof_ms[K_NKIND] = {};
  int64_t prof_n[K_NKIND] = {};
};

// Static scratch of the no-allocation entry point (glmr_set_kernel_noalloc):
// kScratchBytes on every device the library runs a kernel on, held until the
// process ends.  In host code `scratch` names a host-side stand-in; its device
// address comes from hipGetSymbolAddress, once per device (scratch_init), and
// only that address is passed to kernels.  Every call on a device shares that
// device's array and finds the previous call's contents in it.
constexpr size_t kScratchBytes = 256ull << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

glmr_status fail(glmr_ctx* c, glmr_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return s;
}

#define HIPCHK(c, expr)                                                                    \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail((c), GLMR_EDEVICE, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                  __LINE__);                                                               \
  } while (0)

template <typename T>
glmr_status dalloc(glmr_ctx* c, T*& p, size_t n) {
  if (p) {
    hipFree(p);
    c->allocs.erase(std::remove(c->allocs.begin(), c->allocs.end(), (void*)p), c->allocs.end());
    p = nullptr;
  }
  if (n == 0) n = 1;
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, n * sizeof(T));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(c, GLMR_ENOMEM, "hipMalloc of %zu bytes failed: %s", n * sizeof(T),
                hipGetErrorString(e));
  }
  c->allocs.push_back(q);
  p = (T*)q;
  return GLMR_OK;
}

template <typename T>
void dfree(glmr_ctx* c, T*& p) {
  if (!p) return;
  hipFree(p);
  c->allocs.erase(std::remove(c->allocs.begin(), c->allocs.end(), (void*)p), c->allocs.end());
  p = nullptr;
}

#define TRY(expr)                    \
  do {                               \
    glmr_status s_ = (expr);         \
    if (s_ != GLMR_OK) return s_;    \
  } while (0)

// Temporaries of a set-up pass come either from hipMalloc (ar == nullptr) or
// from a bump arena over the static scratch array (the no-allocation entry
// point); buffers that persist in the context must then exist already.
struct Arena {
  unsigned char* base = nullptr;
  size_t cap = 0, used = 0;
};

template <typename T>
glmr_status temp_alloc(glmr_ctx* c, Arena* ar, T*& p, size_t n) {
  if (!ar) return dalloc(c, p, n);
  const size_t at = (ar->used + 255) & ~(size_t)255;
  const size_t bytes = std::max<size_t>(n, 1) * sizeof(T);
  if (at + bytes > ar->cap)
    return fail(c, GLMR_EINVAL, "the set-up needs more than the %zu bytes of static scratch", ar->cap);
  p = (T*)(ar->base + at);
  ar->used = at + bytes;
  return GLMR_OK;
}

template <typename T>
void temp_free(glmr_ctx* c, Arena* ar, T*& p) {
  if (ar) p = nullptr;
  else dfree(c, p);
}

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};
bool g_scratch_done[kMaxDevices] = {};

// Resolve the device address of `scratch` on the current device (once).
hipError_t scratch_init(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_done[dev]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) (void)hipGetLastError();
    g_scratch_ptr[dev] = e == hipSuccess ? ptr : nullptr;
    g_scratch_err[dev] = e;
    g_scratch_done[dev] = true;
  }
  return g_scratch_err[dev];
}

template <typename T>
glmr_status persist(glmr_ctx* c, Arena* ar, T*& p, size_t n) {
  if (p) return GLMR_OK;
  if (ar)
    return fail(c, GLMR_ESTATE, "the per-tau buffers do not exist yet: call glmr_set_kernel once on this "
                                "context before glmr_set_kernel_noalloc");
  return dalloc(c, p, n);
}

hipEvent_t ev_get(glmr_ctx* c) {
  if (!c->pool.empty()) {
    hipEvent_t e = c->pool.back();
    c->pool.pop_back();
    return e;
  }
  hipEvent_t e;
  hipEventCreate(&e);
  return e;
}

struct ProfScope {
  glmr_ctx* c;
  int kind;
  hipEvent_t a = nullptr;
  ProfScope(glmr_ctx* c_, int k) : c(c_), kind(k) {
    if (c->prof && !c->capturing) {
      a = ev_get(c);
      hipEventRecord(a, c->st);
    }
  }
  ~ProfScope() {
    if (c->prof && a) {
      hipEvent_t b = ev_get(c);
      hipEventRecord(b, c->st);
      c->pending.push_back({kind, a, b});
    }
  }
};

void prof_collect(glmr_ctx* c) {
  if (c->pending.empty()) return;
  hipStreamSynchronize(c->st);
  for (auto& r : c->pending) {
    float ms = 0;
    hipEventElapsedTime(&ms, r.a, r.b);
    c->prof_ms[r.kind] += ms;
    c->prof_n[r.kind] += 1;
    c->pool.push_back(r.a);
    c->pool.push_back(r.b);
  }
  c->pending.clear();
}

int64_t rup(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

size_t in_bytes(int prec) { return prec == PREC_F64 ? 8 : prec == PREC_F32 ? 4 : prec == PREC_BF16 ? 2 : 1; }
// bytes of the staged weight copy Jc (FP32 mode stages FP32 values as FP64)
size_t jc_bytes(int prec) { return prec == PREC_F32 ? 8 : in_bytes(prec); }
// bytes of the context's Jc (two BF16 terms per weight in GLMR_BF16_J2)
size_t jc_size(const glmr_ctx* c) { return (size_t)c->Np * c->Np * jc_bytes(c->prec) * (c->j2 ? 2 : 1); }
// the public precision code of a context
int32_t public_precision(const glmr_ctx* c) { return c->j2 ? GLMR_BF16_J2 : c->prec; }

// ---------------------------------------------------------------- kernel caches
// Whether the BF16 trace is kept in HBM (see glmr_trace_mode).
bool delayed(const glmr_ctx* c) { return c->dly != 0 || c->dly_s != 0; }
bool self_delayed(const glmr_ctx* c) { return c->dly != c->dly_s; }

// The masks the contractions use: the recorded raster's shifted by d bins
// (masks0 keeps the recorded ones).  Called after the ingest and when the
// delays change.
glmr_status apply_delays(glmr_ctx* c) {
  if (!c->have_spikes && !c->masks) return GLMR_OK;
  if (!delayed(c)) {
    if (c->masks0) {
      dfree(c, c->masks);
      c->masks = c->masks0;
      c->masks0 = nullptr;
    }
    dfree(c, c->C0);
    return GLMR_OK;
  }
  const size_t nm = (size_t)c->planes * c->NS * c->Np;
  if (!c->masks0) {
    c->masks0 = c->masks;
    c->masks = nullptr;
    TRY(dalloc(c, c->masks, nm));
  }
  HIPCHK(c, launch_shift_masks(c->masks0, c->masks, c->planes, c->NS, c->Np, c->dly, c->st));
  if (!self_delayed(c)) dfree(c, c->C0);
  return GLMR_OK;
}

DelayTrace delay_trace(const glmr_ctx* c) {
  DelayTrace x{};
  x.masks = c->masks0;
  x.planes = c->planes;
  x.C = c->C0;
  x.tab = c->tab;
  x.NS = c->NS;
  x.Np = c->Np;
  return x;
}

EvSlots ev_slots(const glmr_ctx* c) {
  EvSlots e{};
  if (!c->evm || !c->evtab) return e;
  const int64_t n = c->NS * 64;
  e.pw = c->evtab;
  e.ainv = c->evtab + n;
  e.left = c->evtab + 2 * n;
  e.delta = c->evtab + 3 * n;
  e.edec = c->evtab + 4 * n;
  e.asub = c->evtab + 5 * n;
  return e;
}

// Per-slot tables of the event grid for the current tau.  A run of 64 slots
// longer than kMaxSpan tau would overflow e^{(t - t_k0)/tau}.
constexpr double kMaxSpan = 600.0;
glmr_status build_ev_tables(glmr_ctx* c, Arena* ar) {
  const int64_t n = c->NS * 64;
  TRY(persist(c, ar, c->evtab, (size_t)(5 * n + c->NS)));
  unsigned long long* ms = nullptr;
  TRY(temp_alloc(c, ar, ms, 1));
  if (ar) HIPCHK(c, launch_fill_i32((int32_t*)ms, 2, 0, c->st));  // the static scratch keeps old contents
  else HIPCHK(c, hipMemsetAsync(ms, 0, sizeof(unsigned long long), c->st));
  EvTableArgs ta{};
  ta.tslot = c->tslot;
  ta.tau = c->tau;
  ta.NS = c->NS;
  ta.pw = c->evtab;
  ta.ainv = c->evtab + n;
  ta.left = c->evtab + 2 * n;
  ta.delta = c->evtab + 3 * n;
  ta.edec = c->evtab + 4 * n;
  ta.asub = c->evtab + 5 * n;
  if (c->prec == PREC_BF16) {
    TRY(persist(c, ar, c->evgl, (size_t)(16 * n)));
    ta.gl = c->evgl;
  } else if (!ar) {
    dfree(c, c->evgl);
  }
  ta.maxspan = ms;
  HIPCHK(c, launch_ev_tables(ta, c->st));
  unsigned long long h = 0;
  HIPCHK(c, hipMemcpyAsync(&h, ms, sizeof h, hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  temp_free(c, ar, ms);
  double span = 0;
  std::memcpy(&span, &h, sizeof span);
  c->max_span = span;
  if (!(span <= kMaxSpan))
    return fail(c, GLMR_EINVAL, "64 consecutive slots span %.1f tau (at most %.0f): pass a smaller max_gap",
                span, kMaxSpan);
  return GLMR_OK;
}

bool want_resident(glmr_ctx* c) {
  if (c->evm && c->prec != PREC_BF16) return false;  // the event grid's resident trace is BF16
  if (c->prec == PREC_FP8 || c->j2) return true;  // FP8 and two-term J contractions exist only on it
  if (c->prec != PREC_BF16 || c->cfg.trace == GLMR_TRACE_RECOMPUTE) return false;
  if (c->cfg.trace == GLMR_TRACE_RESIDENT) return true;
  size_t fr = 0, tot = 0;
  if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  const size_t have = c->Xtj ? 4 * (size_t)c->Bp * c->Np : 0;  // already held
  return 4 * (size_t)c->Bp * c->Np + (4ull << 30) <= fr + have;
}

// Build (or drop) the resident trace for the current tau; needs C64 and tab.
// With an arena (no allocation) the earlier decision and buffers are kept.
glmr_status build_resident_trace(glmr_ctx* c, Arena* ar) {
  if (!ar) c->resident = want_resident(c);
  if (!c->resident) {
    if (!ar) {
      dfree(c, c->Xtj);
      dfree(c, c->Xjt);
    }
    return GLMR_OK;
  }
  const bool f8 = c->prec == PREC_FP8;
  const size_t n = (size_t)c->Bp * c->Np * (f8 ? 1 : 2);
  if (c->x_bytes != n) {
    if (ar) return fail(c, GLMR_ESTATE, "the resident trace was built for another precision: call glmr_set_kernel");
    dfree(c, c->Xtj);
    dfree(c, c->Xjt);
  }
  TRY(persist(c, ar, c->Xtj, n));
  TRY(persist(c, ar, c->Xjt, n));
  c->x_bytes = n;
  ResXArgs xa{};
  xa.C64 = c->C64;
  xa.masks = c->masks;
  xa.planes = c->planes;
  xa.tab = c->tab;
  xa.Np = c->Np;
  xa.NS = c->NS;
  xa.Bp = c->Bp;
  xa.Xtj = c->Xtj;
  xa.Xjt = c->Xjt;
  xa.xfrag = c->xfrag;
  xa.ev = ev_slots(c);
  if (f8) {
    const int64_t nchunks = (c->Bp + c->L - 1) / c->L;
    if (ar) {
      if (!c->xmax || !c->xscale || c->x_nchunks != nchunks)
        return fail(c, GLMR_ESTATE, "the FP8 trace scales do not exist for this chunking: call glmr_set_kernel");
      HIPCHK(c, launch_fill_i32((int32_t*)c->xmax, (int)nchunks, 0, c->st));
    } else {
      TRY(dalloc(c, c->xmax, (size_t)nchunks));
      TRY(dalloc(c, c->xscale, (size_t)nchunks));
      c->x_nchunks = nchunks;
      HIPCHK(c, hipMemsetAsync(c->xmax, 0, (size_t)nchunks * sizeof(unsigned), c->st));
    }
    xa.L = c->L;
    xa.xmax = c->xmax;
    xa.xscale = c->xscale;
    ProfScope ps(c, K_XBUILD);
    HIPCHK(c, launch_build_x8(xa, c->st));
    return GLMR_OK;
  }
  ProfScope ps(c, K_XBUILD);
  HIPCHK(c, launch_build_x(xa, c->st));
  return GLMR_OK;
}

// The per-tau caches: carries, resident trace, spike term.  ar != nullptr:
// the temporaries come from the static scratch and nothing is allocated (the
// spike term then takes as many time splits as the scratch holds).
glmr_status build_kernel_caches(glmr_ctx* c, bool want_y, Arena* ar = nullptr) {
  const double dt = c->dt, tau = c->tau;
  c->have_kernel = false;
  if (c->evm) {
    want_y = false;
    TRY(build_ev_tables(c, ar));
  }
  Tables h{};
  for (int m = 0; m < 64; ++m) {
    h.pw[m] = std::exp(-(double)m * dt / tau);
    h.ainv[m] = std::exp((double)(m + 1) * dt / tau);
    h.pw32[m] = (float)h.pw[m];
    h.ainv32[m] = (float)h.ainv[m];
  }
  for (int k = 0; k <= 64; ++k) h.apow[k] = std::exp(-64.0 * (double)k * dt / tau);
  TRY(persist(c, ar, c->tab, 1));
  HIPCHK(c, hipMemcpyAsync(c->tab, &h, sizeof(Tables), hipMemcpyHostToDevice, c->st));

  const size_t nc = (size_t)c->NS * c->Np;
  TRY(persist(c, ar, c->C64, nc));
  if (want_y) TRY(persist(c, ar, c->CY64, nc));
  const bool need32 = c->prec == PREC_BF16 || c->prec == PREC_FP8;
  if (need32) TRY(persist(c, ar, c->C32, nc));
  if (need32 && want_y) TRY(persist(c, ar, c->CY32, nc));
  const int64_t G = 64;
  const int64_t nseg = (c->NS + G - 1) / G;
  double *seg = nullptr, *segin = nullptr;
  TRY(temp_alloc(c, ar, seg, (size_t)nseg * c->Np * 2));
  TRY(temp_alloc(c, ar, segin, (size_t)nseg * c->Np * 2));
  CarryArgs ca{};
  ca.masks = c->masks;
  ca.planes = c->planes;
  ca.NS = c->NS;
  ca.Np = c->Np;
  ca.a = c->a;
  ca.ctau = dt / (tau * tau);
  ca.tab = c->tab;
  ca.want_y = want_y ? 1 : 0;
  ca.C64 = c->C64;
  ca.CY64 = want_y ? c->CY64 : nullptr;
  ca.C32 = need32 ? c->C32 : nullptr;
  ca.CY32 = (need32 && want_y) ? c->CY32 : nullptr;
  ca.seg = seg;
  ca.segin = segin;
  ca.G = G;
  ca.ev = ev_slots(c);
  {
    ProfScope ps(c, K_CARRY);
    HIPCHK(c, launch_carries(ca, c->st));
  }
  if (self_delayed(c)) {
    // the recorded raster's own trace, for the self-connection's delay
    TRY(persist(c, ar, c->C0, nc));
    CarryArgs c0 = ca;
    c0.masks = c->masks0;
    c0.want_y = 0;
    c0.C64 = c->C0;
    c0.CY64 = nullptr;
    c0.C32 = nullptr;
    c0.CY32 = nullptr;
    ProfScope ps(c, K_CARRY);
    HIPCHK(c, launch_carries(c0, c->st));
  }
  TRY(build_resident_trace(c, ar));

  // spike term dSigma (and dSigmaY)
  const int64_t nij = c->Np * c->Np;
  TRY(persist(c, ar, c->dsig, (size_t)nij));
  if (want_y) TRY(persist(c, ar, c->dsigY, (size_t)nij));
  int64_t pairs = c->NIB * c->NIB;
  int splits = (int)std::max<int64_t>(1, std::min<int64_t>((8192 + pairs - 1) / pairs, c->NS));
  // bound the partial buffer to ~512 MB (with the static scratch, to what it has left)
  const size_t part_cap = ar ? (ar->cap > ar->used + 256 ? ar->cap - ar->used - 256 : 0) : (512ull << 20);
  while (splits > 1 && (size_t)splits * nij * 8 * (want_y ? 2 : 1) > part_cap) splits /= 2;
  double* part = nullptr;
  // the self-delay correction reuses it for 64 time splits of Np sums
  const size_t part_n = std::max<size_t>((size_t)splits * nij * (want_y ? 2 : 1),
                                         self_delayed(c) ? 64 * (size_t)c->Np : 0);
  TRY(temp_alloc(c, ar, part, part_n));
  SpikeTermArgs sa{};
  sa.masks = c->masks;
  sa.planes = c->planes;
  sa.seg_off = c->seg_off;
  sa.seg_ent = c->seg_ent;
  sa.C64 = c->C64;
  sa.CY64 = want_y ? c->CY64 : nullptr;
  sa.tab = c->tab;
  sa.ctau = dt / (tau * tau);
  sa.NS = c->NS;
  sa.Np = c->Np;
  sa.NIB = c->NIB;
  sa.splits = splits;
  sa.part = part;
  sa.dsig = c->dsig;
  sa.dsigY = want_y ? c->dsigY : nullptr;
  sa.ev = ev_slots(c);
  {
    ProfScope ps(c, K_SPIKE);
    HIPCHK(c, launch_spike_term(sa, c->st));
  }
  if (self_delayed(c)) {
    SelfSpikeArgs ss{};
    ss.x = delay_trace(c);
    ss.seg_off = c->seg_off;
    ss.seg_ent = c->seg_ent;
    ss.NIB = c->NIB;
    ss.splits = (int)std::max<int64_t>(1, std::min<int64_t>(64, c->NS));
    ss.d = c->dly;
    ss.ds = c->dly_s;
    ss.part = part;  // splits * Np doubles fit in the spike term's partial buffer
    ss.dsig = c->dsig;
    ProfScope ps(c, K_SPIKE);
    HIPCHK(c, launch_self_spike(ss, c->st));
  }
  HIPCHK(c, hipStreamSynchronize(c->st));
  temp_free(c, ar, part);
  temp_free(c, ar, seg);
  temp_free(c, ar, segin);
  c->have_kernel = true;
  c->have_y = want_y;
  return GLMR_OK;
}

glmr_status ensure_workspace(glmr_ctx* c, bool want_grad, bool want_tau) {
  const int64_t Np = c->Np;
  const size_t wb = in_bytes(c->prec);
  if (!c->W) {
    void* p = nullptr;
    TRY(dalloc(c, (unsigned char*&)p, (size_t)Np * c->L * wb));
    c->W = p;
  }
  const int64_t ntiles_t = c->Bp / c->bt1;
  if (!c->rowpart) TRY(dalloc(c, c->rowpart, (size_t)ntiles_t * Np));
  if (want_tau && !c->rowpartV) TRY(dalloc(c, c->rowpartV, (size_t)ntiles_t * Np));
  if (!c->rowsum) TRY(dalloc(c, c->rowsum, (size_t)Np));
  if (self_delayed(c) && !c->gpart) TRY(dalloc(c, c->gpart, (size_t)ntiles_t * Np));
  if (self_delayed(c) && !c->gself) TRY(dalloc(c, c->gself, (size_t)Np));
  if (want_tau && !c->rowsumV) TRY(dalloc(c, c->rowsumV, (size_t)Np));
  if (!c->rp_tmp) TRY(dalloc(c, c->rp_tmp, (size_t)rowpart_tmp_len(Np)));
  if (!c->ll_rows) TRY(dalloc(c, c->ll_rows, (size_t)Np));
  if (!c->tau_rows) TRY(dalloc(c, c->tau_rows, (size_t)Np));
  if (!c->scal) TRY(dalloc(c, c->scal, 4));
  if (!c->host_scal) {
    HIPCHK(c, hipHostMalloc((void**)&c->host_scal, 4 * sizeof(double), hipHostMallocDefault));
  }
  if (want_grad) {
    if (!c->gmu) TRY(dalloc(c, c->gmu, (size_t)Np));
    if (!c->gJ) TRY(dalloc(c, c->gJ, (size_t)Np * Np));
    if (!c->G64) TRY(dalloc(c, c->G64, (size_t)Np * Np));
    if (!c->Gp) {
      const size_t gb = (c->prec == PREC_F64 || c->prec == PREC_F32) ? 8 : 4;
      void* p = nullptr;
      TRY(dalloc(c, (unsigned char*&)p, (size_t)c->max_splits * Np * Np * gb));
      c->Gp = p;
    }
  }
  return GLMR_OK;
}

// split length (bins) of kernel G for a chunk of Lc bins: about 2048
// workgroups over `tiles` output tiles, at most max_splits partials.  (For
// the 8-wave fragment tiles half as many splits halve the FP32 partials and
// their reduction, 0.13 ms per evaluation at 3.6e6 bins; the number of BF16
// ascent steps to the stopping test moves with such rounding changes, and in
// the one comparison made it rose from 46 to 62.)
int64_t split_len_tiles(const glmr_ctx* c, int64_t Lc, int64_t tiles) {
  int64_t want = std::max<int64_t>(1, (2048 + tiles - 1) / tiles);
  want = std::min<int64_t>(want, c->max_splits);
  // a split is a whole number of the contraction's 128-byte k steps
  const int64_t q = c->prec == PREC_FP8 ? 128 : 64;
  int64_t ks = rup((Lc + want - 1) / want, q);
  return std::max<int64_t>(ks, q);
}

int64_t split_len(const glmr_ctx* c, int64_t Lc) {
  return split_len_tiles(c, Lc, (c->Np / c->bi2) * (c->Np / c->bj2));
}

// whether shape k suits this context's trace layout and precision
bool shape_fits(const glmr_ctx* c, int k) {
  int n = 0;
  const ResShape* sh = res_shapes(&n);
  return k >= 0 && k < n && sh[k].frag == c->xfrag && (c->prec != PREC_FP8 || sh[k].fp8_ok);
}

// kernel G's tiles of shape k divide the padded neurons
bool shape_ok(const glmr_ctx* c, int k) {
  int n = 0;
  const ResShape* sh = res_shapes(&n);
  return shape_fits(c, k) && c->Np % sh[k].gi == 0 && c->Np % sh[k].gj == 0;
}

// kernel U's shapes: on the event grid only the 128-neuron tiles (the
// 256-neuron ones would need the whole LDS for the staged rows and the
// expansion table)
bool shape_ok_u(const glmr_ctx* c, int k) {
  int n = 0;
  const ResShape* sh = res_shapes(&n);
  return shape_fits(c, k) && c->Np % sh[k].ui == 0 && !(c->evm && sh[k].ui != 128);
}

// shapes worth timing for kernel U (the fragment-major shapes share one kernel U)
bool shape_tune_u(const glmr_ctx* c, int k) {
  int n = 0;
  const ResShape* sh = res_shapes(&n);
  return shape_ok_u(c, k) && sh[k].u_own;
}

ResShape res_shape(int k) {
  int n = 0;
  const ResShape* s = res_shapes(&n);
  return s[(k >= 0 && k < n) ? k : 0];
}

// Arguments of the resident-trace kernels U and G for the chunk [t0, t0 + Lc)
// with tile shape k.
ResUArgs make_u_args(glmr_ctx* c, int k, int64_t t0, int64_t Lc) {
  const ResShape su = res_shape(k);
  ResUArgs ua{};
  ua.Jc = c->Jc;
  ua.j2 = c->j2 ? 1 : 0;
  ua.Xtj = c->Xtj;
  ua.Np = c->Np;
  ua.B = c->B;
  ua.t0 = t0;
  ua.L = c->L;
  ua.n_itiles = (int)(c->Np / su.ui);
  ua.n_ttiles = (int)(Lc / GLMR_TT);
  ua.W = c->W;
  ua.rowpart = c->rowpart;
  if (c->prec == PREC_FP8) {
    ua.xscale = c->xscale + t0 / c->L;
    ua.jscale = c->jscale;
  }
  if (c->evm) {
    ua.evgl = c->evgl;
    ua.evdelta = ev_slots(c).delta;
  }
  return ua;
}

ResGArgs make_g_args(glmr_ctx* c, int k, int64_t t0, int64_t Lc) {
  const ResShape sg = res_shape(k);
  ResGArgs ga{};
  ga.W = c->W;
  ga.Xjt = c->Xjt;
  ga.Np = c->Np;
  ga.Bp = c->Bp;
  ga.t0 = t0;
  ga.L = c->L;
  ga.Lc = Lc;
  ga.n_itiles = (int)(c->Np / sg.gi);
  ga.n_jtiles = (int)(c->Np / sg.gj);
  ga.ks = split_len_tiles(c, Lc, (int64_t)ga.n_itiles * ga.n_jtiles);
  ga.n_splits = (int)((Lc + ga.ks - 1) / ga.ks);
  ga.Gp = c->Gp;
  if (c->prec == PREC_FP8) ga.xscale = c->xscale + t0 / c->L;
  return ga;
}

hipError_t launch_u_chunk(glmr_ctx* c, int k, int64_t t0, int64_t Lc) {
  return launch_res_u(k, c->prec == PREC_FP8 ? 1 : 0, make_u_args(c, k, t0, Lc), c->st);
}

hipError_t launch_g_chunk(glmr_ctx* c, int k, int64_t t0, int64_t Lc, int* n_splits) {
  const ResGArgs ga = make_g_args(c, k, t0, Lc);
  *n_splits = ga.n_splits;
  return launch_res_g(k, c->prec == PREC_FP8 ? 1 : 0, ga, c->st);
}

glmr_status eval_finish(glmr_ctx* c, bool want_grad, bool want_tau);

glmr_status eval_core(glmr_ctx* c, bool want_grad, bool want_tau) {
  TRY(ensure_workspace(c, want_grad, want_tau));
  const int64_t Np = c->Np;
  for (int64_t t0 = 0, ci = 0; t0 < c->Bp; t0 += c->L, ++ci) {
    const int64_t Lc = std::min<int64_t>(c->L, c->Bp - t0);
    Gemm1Args g1{};
    g1.Jc = c->Jc;
    g1.masks = c->masks;
    g1.planes = c->planes;
    g1.C = (c->prec == PREC_BF16 || c->prec == PREC_FP8) ? (const void*)c->C32 : (const void*)c->C64;
    g1.CY = (c->prec == PREC_BF16 || c->prec == PREC_FP8) ? (const void*)c->CY32 : (const void*)c->CY64;
    g1.tab = c->tab;
    g1.ctau = c->dt / (c->tau * c->tau);
    g1.Np = Np;
    g1.NS = c->NS;
    g1.B = c->B;
    g1.t0 = t0;
    g1.L = c->L;  // row pitch of W
    g1.n_itiles = (int)(Np / c->bi1);
    g1.n_ttiles = (int)(Lc / c->bt1);
    g1.W = c->W;
    g1.rowpart = c->rowpart;
    g1.mode = 0;
    g1.ev = ev_slots(c);
    g1.evgl = c->evgl;
    if (c->resident) {
      ProfScope ps(c, K_U);
      HIPCHK(c, launch_u_chunk(c, c->res_shape_u, t0, Lc));
    } else if (c->j2) {
      return fail(c, GLMR_EINVAL, "the two-term J runs on the resident trace only");
    } else {
      ProfScope ps(c, K_U);
      HIPCHK(c, launch_gemm1(c->prec, c->tile, g1, c->st));
    }
    if (self_delayed(c)) {
      SelfDelayArgs sd{};
      sd.x = delay_trace(c);
      sd.W = c->W;
      sd.wtype = c->prec == PREC_F64 ? 0 : (c->prec == PREC_F32 ? 1 : 2);
      sd.scaled = c->resident ? 0 : 1;
      sd.tiled = c->resident ? (c->xfrag ? 2 : 1) : 0;
      sd.Jr = c->Jr;
      sd.B = c->B;
      sd.t0 = t0;
      sd.L = c->L;
      sd.Lc = Lc;
      sd.tb = c->bt1;
      sd.d = c->dly;
      sd.ds = c->dly_s;
      sd.rowpart = c->rowpart;
      sd.gpart = c->gpart;
      ProfScope ps(c, K_SELF);
      HIPCHK(c, launch_self_delay(sd, c->st));
    }
    if (want_tau) {
      g1.mode = 1;
      g1.w_plain = c->resident ? (c->xfrag ? 2 : 1) : 0;
      g1.rowpart = c->rowpartV;
      ProfScope ps(c, K_V);
      HIPCHK(c, launch_gemm1(c->prec, c->tile, g1, c->st));
    }
    if (want_grad) {
      Gemm2Args g2{};
      g2.W = c->W;
      g2.masks = c->masks;
      g2.planes = c->planes;
      g2.C = g1.C;
      g2.tab = c->tab;
      g2.Np = Np;
      g2.NS = c->NS;
      g2.t0 = t0;
      g2.L = c->L;
      g2.Lc = Lc;
      g2.ks = split_len(c, Lc);
      g2.n_splits = (int)((Lc + g2.ks - 1) / g2.ks);
      g2.n_itiles = (int)(Np / c->bi2);
      g2.n_jtiles = (int)(Np / c->bj2);
      g2.Gp = c->Gp;
      g2.ev = ev_slots(c);
      if (c->resident) {
        ProfScope ps(c, K_G);
        HIPCHK(c, launch_g_chunk(c, c->res_shape_g, t0, Lc, &g2.n_splits));
      } else {
        ProfScope ps(c, K_G);
        HIPCHK(c, launch_gemm2(c->prec, c->tile, g2, c->st));
      }
      ProfScope ps(c, K_RED);
      HIPCHK(c, launch_gp_reduce(c->prec, c->Gp, g2.n_splits, Np, c->G64, ci == 0, c->st));
    }
  }
  return eval_finish(c, want_grad, want_tau);
}

// Row sums of the weights over all bins, then L_i, dL/dmu, dL/dJ (dL/dtau) in FP64.
glmr_status eval_finish(glmr_ctx* c, bool want_grad, bool want_tau) {
  const int64_t Np = c->Np;
  ProfScope ps(c, K_ASM);
  const int64_t ntiles_t = c->Bp / c->bt1;
  HIPCHK(c, launch_rowpart_reduce(c->rowpart, ntiles_t, Np, c->rowsum, c->rp_tmp, c->st));
  if (want_tau)
    HIPCHK(c, launch_rowpart_reduce(c->rowpartV, ntiles_t, Np, c->rowsumV, c->rp_tmp, c->st));
  if (want_grad && self_delayed(c))
    HIPCHK(c, launch_rowpart_reduce(c->gpart, ntiles_t, Np, c->gself, c->rp_tmp, c->st));
  AssembleArgs aa{};
  aa.N = c->N;
  aa.Np = Np;
  aa.dt = c->evm ? c->tau : c->dt;  // the event grid's integrals are in units of tau
  aa.q = c->q;
  aa.mu = c->mu;
  aa.Jr = c->Jr;
  aa.dsig = c->dsig;
  aa.dsigY = want_tau ? c->dsigY : nullptr;
  aa.rowsum = c->rowsum;
  aa.rowsumV = want_tau ? c->rowsumV : nullptr;
  aa.G64 = want_grad ? c->G64 : nullptr;
  aa.gself = (want_grad && self_delayed(c)) ? c->gself : nullptr;
  aa.rowscale = c->rowscale;
  aa.ll_rows = c->ll_rows;
  aa.gJ = want_grad ? c->gJ : nullptr;
  aa.gmu = want_grad ? c->gmu : nullptr;
  aa.tau_rows = want_tau ? c->tau_rows : nullptr;
  HIPCHK(c, launch_assemble(aa, c->st));
  HIPCHK(c, launch_sum_rows(c->ll_rows, c->N, c->scal, c->st));
  if (want_tau) HIPCHK(c, launch_sum_rows(c->tau_rows, c->N, c->scal + 1, c->st));
  return GLMR_OK;
}

glmr_status prepare_params(glmr_ctx* c) {
  ProfScope ps(c, K_PREP);
  if (c->prec == PREC_FP8 && !c->jscale) TRY(dalloc(c, c->jscale, (size_t)c->Np));
  HIPCHK(c, launch_prepare_params(c->prec, c->j2 ? 1 : 0, c->N, c->Np, c->J64, c->mu, c->Jc, c->Jr, c->rowscale,
                                  c->prec == PREC_FP8 ? c->jscale : nullptr, c->st));
  return GLMR_OK;
}

// tiles, chunk length and split budget of the context's precision (Np fixed)
void setup_precision(glmr_ctx* c) {
  // neuron tile of the BF16 kernels (FP64 and FP32 use 128-row tiles)
  if (c->prec != PREC_BF16 && c->prec != PREC_FP8) c->tile = 256;
  else if (c->Np % 256 != 0 || c->cfg.tile_n == 128) c->tile = 128;
  else if (c->cfg.tile_n == 256) c->tile = 256;
  else c->tile = c->N > 384 ? 256 : 128;
  gemm_tiles(c->prec, c->tile, &c->bi1, &c->bt1, &c->bi2, &c->bj2);
  // resident-trace shapes: in BF16 the fragment-major kernels (unless
  // GLMR_XFRAG=0), else the row-major ones with 256-neuron tiles when the
  // padding allows
  const char* xf = std::getenv("GLMR_XFRAG");
  c->xfrag = (c->prec == PREC_BF16 && !(xf && std::strcmp(xf, "0") == 0)) ? 1 : 0;
  if (c->xfrag) {
    // kernel G: 512-row tiles of 8 waves where the padding allows (each
    // operand byte fetched from HBM once), else 256 or 128 rows of 4 waves
    c->res_shape_u = 7;
    c->res_shape_g = (c->Np % 512 == 0) ? 10 : (c->Np % 256 == 0) ? 7 : 9;
  } else if (c->prec == PREC_FP8) {
    c->res_shape_u = c->res_shape_g = 5;
  } else {
    c->res_shape_u = c->res_shape_g = (c->Np % 256 == 0) ? 2 : 3;
    if (c->evm) c->res_shape_u = 5;  // the interval integrals: 128-neuron tiles keep kernel U unspilled
  }
  if (const char* e = std::getenv("GLMR_RES_SHAPE")) {
    int u = -1, g = -1;
    if (std::sscanf(e, "%d,%d", &u, &g) == 2 && shape_ok_u(c, u) && shape_ok(c, g)) {
      c->res_shape_u = u;
      c->res_shape_g = g;
    }
  }
  // chunk: W of at most ~4 GiB, a multiple of 4096 bins
  int64_t L = c->cfg.chunk_bins;
  if (L == 0) {
    const int64_t budget = 4ll << 30;
    L = budget / (c->Np * (int64_t)in_bytes(c->prec));
    L = std::max<int64_t>(4096, L / 4096 * 4096);
  } else {
    L = rup(L, 4096);
  }
  c->L = std::min<int64_t>(L, c->Bp);
  // partial buffer of kernel G: at most ~512 MB, at most 256 splits
  const size_t gb = c->prec == PREC_F64 ? 8 : 4;
  int64_t ms = (512ll << 20) / (int64_t)(c->Np * c->Np * gb);
  c->max_splits = (int)std::max<int64_t>(1, std::min<int64_t>(ms, 256));
}

glmr_status check_ready(glmr_ctx* c) {
  if (!c->have_spikes) return fail(c, GLMR_ESTATE, "set_spikes has not been called");
  if (!c->have_kernel) return fail(c, GLMR_ESTATE, "set_kernel has not been called");
  if (!c->have_params) return fail(c, GLMR_ESTATE, "set_params has not been called");
  return GLMR_OK;
}

hipMemcpyKind kind_to(int where) { return where == GLMR_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice; }
hipMemcpyKind kind_from(int where) { return where == GLMR_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice; }


// ------------------------------------------------------------------ ascent
glmr_status alloc_ascent(glmr_ctx* c, int m) {
  AscentArgs& a = c->asc;
  const int N = c->N, P = N + 1;
  if (c->have_asc && a.m == m) return GLMR_OK;
  a.N = N;
  a.Np = c->Np;
  a.P = P;
  a.m = m;
  const size_t np = (size_t)N * P;
  TRY(dalloc(c, a.theta, np));
  TRY(dalloc(c, a.theta_try, np));
  TRY(dalloc(c, a.g, np));
  TRY(dalloc(c, a.g_try, np));
  TRY(dalloc(c, a.d, np));
  TRY(dalloc(c, a.S, np * m));
  TRY(dalloc(c, a.Y, np * m));
  TRY(dalloc(c, a.rho, (size_t)m * N));
  TRY(dalloc(c, a.hist_len, (size_t)N));
  TRY(dalloc(c, a.hist_head, (size_t)N));
  TRY(dalloc(c, a.f, (size_t)N));
  TRY(dalloc(c, a.f_try, (size_t)N));
  TRY(dalloc(c, a.step, (size_t)N));
  TRY(dalloc(c, a.gd, (size_t)N));
  TRY(dalloc(c, a.state, (size_t)N));
  TRY(dalloc(c, a.accepted, (size_t)N));
  TRY(dalloc(c, a.eta, (size_t)N));
  TRY(dalloc(c, a.bt, (size_t)N));
  TRY(dalloc(c, a.gstep, (size_t)N));
  TRY(dalloc(c, c->counters, 4));
  if (!c->host_cnt) HIPCHK(c, hipHostMalloc((void**)&c->host_cnt, 4 * sizeof(int32_t), hipHostMallocDefault));
  c->have_asc = true;
  return GLMR_OK;
}

// evaluate at theta_src ([N][P]); gradient of f = -L into g, f into f
glmr_status eval_theta(glmr_ctx* c, const double* theta_src, double* g, double* f) {
  const AscentArgs& a = c->asc;
  HIPCHK(c, launch_pack_theta(c->N, c->Np, a.P, theta_src, c->J64, c->mu, c->st));
  TRY(prepare_params(c));
  TRY(eval_core(c, true, false));
  ProfScope ps(c, K_ASC);
  HIPCHK(c, launch_pack_grad(c->N, c->Np, a.P, c->gJ, c->gmu, c->ll_rows, g, f, c->st));
  HIPCHK(c, launch_penalty(a, theta_src, g, f, c->st));
  return GLMR_OK;
}

// Fresh ascent state: empty histories, every row active and asking for a direction.
glmr_status ascent_reset(glmr_ctx* c, bool keep_history = false) {
  AscentArgs& a = c->asc;
  if (!keep_history) {
    HIPCHK(c, launch_fill_i32(a.hist_len, c->N, 0, c->st));
    HIPCHK(c, launch_fill_i32(a.hist_head, c->N, 0, c->st));
  }
  HIPCHK(c, launch_fill_i32(a.state, c->N, 0, c->st));
  HIPCHK(c, launch_fill_i32(a.bt, c->N, 0, c->st));
  HIPCHK(c, launch_fill_i32(a.accepted, c->N, 3, c->st));
  HIPCHK(c, hipMemsetAsync(a.eta, 0, c->N * sizeof(double), c->st));
  return GLMR_OK;
}

// One asynchronous ascent step for every row: trial point, one evaluation,
// per-row Armijo test (accept, halve the step, or give up), history update
// and stopping test for accepted rows, new directions for them, and the count
// of active rows in counters[0].  Only kernel launches: it can be captured.
glmr_status ascent_step(glmr_ctx* c, double ftol, int max_bt) {
  AscentArgs& a = c->asc;
  {
    ProfScope ps(c, K_ASC);
    HIPCHK(c, launch_make_trial(a, c->st));
  }
  TRY(eval_theta(c, a.theta_try, a.g_try, a.f_try));
  ProfScope ps(c, K_ASC);
  HIPCHK(c, launch_armijo_async(a, 1e-4, max_bt, c->st));
  HIPCHK(c, launch_accept_update(a, ftol, nullptr, 1, c->st));
  HIPCHK(c, launch_lbfgs_direction(a, 1, c->st));
  HIPCHK(c, launch_count_active(a, c->counters, c->st));
  return GLMR_OK;
}

bool use_graphs() {
  const char* e = std::getenv("GLMR_NO_GRAPH");
  return !(e && e[0] == '1');
}

// A captured sequence of launches, replayed with hipGraphLaunch.
struct GraphRun {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  template <typename F>
  glmr_status capture(glmr_ctx* c, hipStream_t st, F body) {
    HIPCHK(c, hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    c->capturing = true;
    const glmr_status s1 = body();
    c->capturing = false;
    const hipError_t e = hipStreamEndCapture(st, &graph);
    if (s1 != GLMR_OK) return s1;
    if (e != hipSuccess) return fail(c, GLMR_EDEVICE, "graph capture: %s", hipGetErrorString(e));
    HIPCHK(c, hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
    return GLMR_OK;
  }
  ~GraphRun() {
    if (exec) hipGraphExecDestroy(exec);
    if (graph) hipGraphDestroy(graph);
  }
};

// the stopping threshold of a mode: below its rounding noise in L, eta cannot
// fall.  The two-term J removes BF16's J steps; L's own noise (FP32 exp and
// potentials summed in FP64) is ~1e-10 relative.
double default_ftol(const glmr_ctx* c) {
  if (c->j2) return 1e-10;
  switch (c->prec) {
    case PREC_F64: return 1e-14;
    case PREC_F32: return 1e-11;
    case PREC_BF16: return 1e-6;
    default: return 1e-4;
  }
}

glmr_status check_fit_opts(glmr_ctx* c, const glmr_fit_opts* o_in, glmr_fit_opts* o) {
  glmr_fit_defaults(o);
  if (o_in) *o = *o_in;
  if (o->max_iter < 0 || o->lbfgs_m < 1 || o->lbfgs_m > 64 || o->max_backtracks < 0 || o->ftol < 0 ||
      !(o->l1_alpha >= 0) || !(o->l1_eps >= 0) || !(o->j_max >= 0) || !(o->rate_min >= 0) ||
      !(o->rate_max >= 0) || (o->rate_min > 0 && o->rate_max > 0 && o->rate_min >= o->rate_max))
    return fail(c, GLMR_EINVAL, "bad fit options");
  if (o->resume != 0 && o->resume != 1) return fail(c, GLMR_EINVAL, "bad fit options");
  if (o->keep_history != 0 && o->keep_history != 1) return fail(c, GLMR_EINVAL, "bad fit options");
  if (!c->have_spikes || !c->have_kernel) return fail(c, GLMR_ESTATE, "set spikes and kernel first");
  if (!c->all_spiking) return fail(c, GLMR_ENOSPIKES, "some neuron has no spike: its MLE does not exist");
  if (o->resume && !c->asc_live)
    return fail(c, GLMR_ESTATE, "no ascent to resume (fit or glmr_set_state first; changing spikes, "
                                "kernel, delays, precision or parameters ends it)");
  if (o->keep_history && !o->resume && !(c->asc_hist && c->have_asc && c->asc.m == o->lbfgs_m))
    return fail(c, GLMR_ESTATE, "no L-BFGS history to keep (a fit with the same lbfgs_m first; changing "
                                "spikes, kernel or delays drops it)");
  return GLMR_OK;
}

// Starting point and a fresh ascent state (every row active, asking for a direction).
glmr_status fit_begin(glmr_ctx* c, const glmr_fit_opts& o) {
  const int N = c->N;
  const int64_t Np = c->Np;
  c->asc_live = false;
  if (!c->have_params || o.from_zero) {
    if (!c->J64) {
      std::vector<double> z((size_t)N * N, 0.0), zm(N, 0.0);
      TRY(glmr_set_params(c, z.data(), zm.data(), GLMR_HOST));
    } else {
      HIPCHK(c, hipMemsetAsync(c->J64, 0, Np * Np * sizeof(double), c->st));
      HIPCHK(c, hipMemsetAsync(c->mu, 0, Np * sizeof(double), c->st));
      c->have_params = true;
    }
  }
  if (o.warm_start_mu) {
    std::vector<double> m0(N);
    const double T = (double)c->B * c->dt;
    for (int i = 0; i < N; ++i) m0[i] = std::log((double)c->q_host[i] / T);
    HIPCHK(c, hipMemcpyAsync(c->mu, m0.data(), N * sizeof(double), hipMemcpyHostToDevice, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
  }
  TRY(alloc_ascent(c, o.lbfgs_m));
  AscentArgs& a = c->asc;
  a.alpha = o.l1_alpha;
  a.eps = o.l1_eps > 0 ? o.l1_eps : 1e-8;
  a.jmax = o.j_max > 0 ? o.j_max : 0.0;
  a.mu_lo = o.rate_min > 0 ? std::log(o.rate_min) : -INFINITY;
  a.mu_hi = o.rate_max > 0 ? std::log(o.rate_max) : INFINITY;
  HIPCHK(c, launch_unpack_theta(N, Np, a.P, c->J64, c->mu, a.theta, c->st));
  HIPCHK(c, launch_project_theta(a, a.theta, c->st));  // start inside the box
  TRY(ascent_reset(c, o.keep_history != 0));
  return GLMR_OK;
}

// Leave the context at the accepted parameters and fill the report.
glmr_status fit_end(glmr_ctx* c, int iters, int evals, double seconds, glmr_fit_report* rep) {
  const int N = c->N;
  AscentArgs& a = c->asc;
  c->asc_live = true;
  c->asc_hist = true;
  HIPCHK(c, launch_pack_theta(N, c->Np, a.P, a.theta, c->J64, c->mu, c->st));
  TRY(prepare_params(c));
  std::vector<double> f(N), eta(N);
  std::vector<int32_t> state(N);
  HIPCHK(c, hipMemcpyAsync(f.data(), a.f, N * sizeof(double), hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipMemcpyAsync(eta.data(), a.eta, N * sizeof(double), hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipMemcpyAsync(state.data(), a.state, N * sizeof(int32_t), hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  const int32_t conv = (int32_t)std::count_if(state.begin(), state.end(), [](int32_t s) { return s != 0; });
  if (rep) {
    rep->iters = iters;
    rep->evals = evals;
    double ll = 0;
    for (int i = 0; i < N; ++i) ll -= f[i];
    rep->ll = ll;
    rep->max_eta = *std::max_element(eta.begin(), eta.end());
    rep->rows_converged = conv;
    rep->seconds = seconds;
  }
  return conv < N ? GLMR_NOT_CONVERGED : GLMR_OK;
}

glmr_status fit_one(glmr_ctx* c, const glmr_fit_opts* o_in, glmr_fit_report* rep) {
  glmr_fit_opts o;
  TRY(check_fit_opts(c, o_in, &o));
  HIPCHK(c, hipSetDevice(c->cfg.device));
  auto t_start = std::chrono::steady_clock::now();
  AscentArgs& a = c->asc;
  const double ftol = o.ftol > 0 ? o.ftol : default_ftol(c);
  int evals = 0, iters = 0;
  if (o.resume) {
    // every step ends with the next directions in place: carry on from there.
    // A context restored from a checkpoint has not evaluated yet: its
    // workspace is made here, since nothing may allocate inside the capture.
    c->asc_live = false;
    TRY(ensure_workspace(c, true, false));
  } else {
    TRY(fit_begin(c, o));
    TRY(eval_theta(c, a.theta, a.g, a.f));
    ++evals;
    HIPCHK(c, launch_lbfgs_direction(a, 1, c->st));
  }
  // one ascent step, captured once into a graph and replayed
  auto step = [&]() -> glmr_status { return ascent_step(c, ftol, o.max_backtracks); };
  GraphRun gr;
  if (use_graphs()) TRY(gr.capture(c, c->st, step));
  int active = c->N;
  if (o.resume) {
    HIPCHK(c, launch_count_active(a, c->counters, c->st));
    HIPCHK(c, hipMemcpyAsync(c->host_cnt, c->counters, sizeof(int32_t), hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    active = c->host_cnt[0];
  }
  for (iters = 0; iters < o.max_iter && active > 0; ++iters) {
    if (gr.exec) HIPCHK(c, hipGraphLaunch(gr.exec, c->st));
    else TRY(step());
    ++evals;
    HIPCHK(c, hipMemcpyAsync(c->host_cnt, c->counters, sizeof(int32_t), hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    active = c->host_cnt[0];
  }
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  return fit_end(c, iters, evals, secs, rep);
}

}  // namespace

// autotuner helpers
namespace {

// mean milliseconds of `reps` launches of fn on the context's stream (after one warm-up)
template <typename F>
glmr_status time_launches(glmr_ctx* c, F fn, int reps, double* ms) {
  hipEvent_t a, b;
  HIPCHK(c, hipEventCreate(&a));
  HIPCHK(c, hipEventCreate(&b));
  glmr_status st = GLMR_OK;
  float el = 0.f;
  if (fn() != hipSuccess) st = fail(c, GLMR_EDEVICE, "autotune launch failed");
  if (st == GLMR_OK && hipEventRecord(a, c->st) != hipSuccess) st = fail(c, GLMR_EDEVICE, "event record");
  for (int r = 0; st == GLMR_OK && r < reps; ++r)
    if (fn() != hipSuccess) st = fail(c, GLMR_EDEVICE, "autotune launch failed");
  if (st == GLMR_OK && (hipEventRecord(b, c->st) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
                        hipEventElapsedTime(&el, a, b) != hipSuccess))
    st = fail(c, GLMR_EDEVICE, "event timing");
  hipEventDestroy(a);
  hipEventDestroy(b);
  *ms = el / reps;
  return st;
}

std::string tune_key(glmr_ctx* c) {
  hipDeviceProp_t prop{};
  std::string arch = "unknown";
  if (hipGetDeviceProperties(&prop, c->cfg.device) == hipSuccess) arch = prop.gcnArchName;
  for (char& ch : arch)
    if (ch == ' ') ch = '_';
  char buf[256];
  std::snprintf(buf, sizeof(buf), "%s %lld %lld %d", arch.c_str(), (long long)c->Np, (long long)c->L,
                c->prec + (c->evm ? 16 : 0));  // the event grid's kernel U differs
  return buf;
}

}  // namespace

// ---------------------------------------------------------------- batching
struct glmr_batch {
  std::vector<glmr_ctx*> ctxs;
  int dev = 0;
  hipStream_t st = nullptr;
  bool grouped = false;  // persistent launches over the recordings, one per tile shape and contraction
  // Tile shapes per recording: those the autotuner chose for its class (the
  // recordings whose padding allows 256-neuron tiles, and the rest), else the
  // context's own.  Recordings with the same pair share one launch.
  int tuned_u[2] = {-1, -1}, tuned_g[2] = {-1, -1};
  std::vector<int> rec_u, rec_g;
  struct Group {         // recordings of one chunk with the same shapes, as work queues
    int su = -1, sg = -1;
    std::vector<int> recs, nsplits;
    ResUArgs* du = nullptr;
    ResGArgs* dg = nullptr;
    int64_t *pu = nullptr, *pg = nullptr;
    int64_t tu = 0, tg = 0;
    int64_t *xu = nullptr, *xg = nullptr;  // [8][m + 1] per-XCD tile prefixes (fragment-major kernels)
    int64_t gu = 0, gg = 0;                // their launch grids
  };
  struct Chunk {         // the recordings that have time chunk ci
    std::vector<Group> groups;
  };
  std::vector<Chunk> chunks;
  int32_t** dcnt = nullptr;  // [n] each context's counters
  int32_t* dsum = nullptr;   // active rows over all recordings
  int32_t* hsum = nullptr;   // pinned
  std::vector<void*> allocs;
};

namespace {

template <typename T>
hipError_t balloc(glmr_batch* b, T*& p, size_t n) {
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, (n ? n : 1) * sizeof(T));
  if (e == hipSuccess) {
    b->allocs.push_back(q);
    p = (T*)q;
  }
  return e;
}

void free_queues(glmr_batch* b) {
  for (void* p : b->allocs) hipFree(p);
  b->allocs.clear();
  b->chunks.clear();
  b->dcnt = nullptr;
  b->dsum = nullptr;
}

// Every context works on the batch's stream while the batch runs it.
struct OnBatchStream {
  glmr_batch* b;
  std::vector<hipStream_t> old;
  explicit OnBatchStream(glmr_batch* b_) : b(b_) {
    for (glmr_ctx* c : b->ctxs) {
      hipStreamSynchronize(c->st);  // order after the context's own earlier work
      old.push_back(c->st);
      c->st = b->st;
    }
  }
  ~OnBatchStream() {
    hipStreamSynchronize(b->st);
    for (size_t r = 0; r < b->ctxs.size(); ++r) b->ctxs[r]->st = old[r];
  }
};

// shape class of a recording: 0 if its padding allows the 256-neuron tiles
int shape_class(const glmr_ctx* c) { return c->Np % 256 == 0 ? 0 : 1; }

// Work queues for the grouped launches (after every context's workspace exists).
glmr_status build_queues(glmr_batch* b) {
  glmr_ctx* c0 = b->ctxs[0];
  free_queues(b);
  const int n = (int)b->ctxs.size();
  std::vector<int32_t*> hc(n);
  for (int r = 0; r < n; ++r) {
    TRY(ensure_workspace(b->ctxs[r], true, false));
    hc[r] = b->ctxs[r]->counters;
  }
  HIPCHK(c0, balloc(b, b->dcnt, (size_t)n));
  HIPCHK(c0, balloc(b, b->dsum, 1));
  HIPCHK(c0, hipMemcpy(b->dcnt, hc.data(), n * sizeof(int32_t*), hipMemcpyHostToDevice));
  if (!b->grouped) return GLMR_OK;
  int64_t nch = 0;
  for (glmr_ctx* c : b->ctxs) nch = std::max<int64_t>(nch, (c->Bp + c->L - 1) / c->L);
  b->chunks.resize(nch);
  for (int64_t ci = 0; ci < nch; ++ci) {
    glmr_batch::Chunk& ch = b->chunks[ci];
    struct Lists {
      std::vector<ResUArgs> ua;
      std::vector<ResGArgs> ga;
      std::vector<int64_t> pu{0}, pg{0};
    };
    std::vector<Lists> lists;
    for (int r = 0; r < n; ++r) {
      glmr_ctx* c = b->ctxs[r];
      const int64_t t0 = ci * c->L;
      if (t0 >= c->Bp) continue;
      const int64_t Lc = std::min<int64_t>(c->L, c->Bp - t0);
      size_t q = 0;
      while (q < ch.groups.size() && !(ch.groups[q].su == b->rec_u[r] && ch.groups[q].sg == b->rec_g[r])) ++q;
      if (q == ch.groups.size()) {
        ch.groups.emplace_back();
        ch.groups.back().su = b->rec_u[r];
        ch.groups.back().sg = b->rec_g[r];
        lists.emplace_back();
      }
      glmr_batch::Group& gr = ch.groups[q];
      Lists& li = lists[q];
      li.ua.push_back(make_u_args(c, gr.su, t0, Lc));
      li.ga.push_back(make_g_args(c, gr.sg, t0, Lc));
      li.pu.push_back(li.pu.back() + (int64_t)li.ua.back().n_itiles * li.ua.back().n_ttiles);
      li.pg.push_back(li.pg.back() + (int64_t)li.ga.back().n_splits * li.ga.back().n_itiles * li.ga.back().n_jtiles);
      gr.recs.push_back(r);
      gr.nsplits.push_back(li.ga.back().n_splits);
    }
    for (size_t q = 0; q < ch.groups.size(); ++q) {
      glmr_batch::Group& gr = ch.groups[q];
      const Lists& li = lists[q];
      const size_t m = gr.recs.size();
      HIPCHK(c0, balloc(b, gr.du, m));
      HIPCHK(c0, balloc(b, gr.dg, m));
      HIPCHK(c0, balloc(b, gr.pu, m + 1));
      HIPCHK(c0, balloc(b, gr.pg, m + 1));
      HIPCHK(c0, hipMemcpy(gr.du, li.ua.data(), m * sizeof(ResUArgs), hipMemcpyHostToDevice));
      HIPCHK(c0, hipMemcpy(gr.dg, li.ga.data(), m * sizeof(ResGArgs), hipMemcpyHostToDevice));
      HIPCHK(c0, hipMemcpy(gr.pu, li.pu.data(), (m + 1) * sizeof(int64_t), hipMemcpyHostToDevice));
      HIPCHK(c0, hipMemcpy(gr.pg, li.pg.data(), (m + 1) * sizeof(int64_t), hipMemcpyHostToDevice));
      gr.tu = li.pu.back();
      gr.tg = li.pg.back();
      // each recording's tiles split evenly over the 8 XCDs (see ResUGroup)
      auto stripes = [&](const std::vector<int64_t>& pre, int64_t*& dst, int64_t* grid) -> glmr_status {
        std::vector<int64_t> x(8 * (m + 1), 0);
        int64_t most = 0;
        for (int xc = 0; xc < 8; ++xc) {
          for (size_t r = 0; r < m; ++r) {
            const int64_t t = pre[r + 1] - pre[r];
            x[xc * (m + 1) + r + 1] = x[xc * (m + 1) + r] + t / 8 + (xc < t % 8 ? 1 : 0);
          }
          most = std::max(most, x[xc * (m + 1) + m]);
        }
        HIPCHK(c0, balloc(b, dst, x.size()));
        HIPCHK(c0, hipMemcpy(dst, x.data(), x.size() * sizeof(int64_t), hipMemcpyHostToDevice));
        *grid = 8 * most;
        return GLMR_OK;
      };
      TRY(stripes(li.pu, gr.xu, &gr.gu));
      TRY(stripes(li.pg, gr.xg, &gr.gg));
    }
  }
  return GLMR_OK;
}

// The grouped launches of kernel U (want_u) and kernel G (want_g) over chunk ci.
glmr_status launch_chunk_groups(glmr_batch* b, size_t ci, bool want_u, bool want_g) {
  glmr_ctx* c0 = b->ctxs[0];
  const int fp8 = c0->prec == PREC_FP8 ? 1 : 0;
  for (const glmr_batch::Group& gr : b->chunks[ci].groups) {
    const int m = (int)gr.recs.size();
    if (want_u) {
      ProfScope ps(c0, K_BU);
      HIPCHK(c0, launch_res_u_group(gr.su, fp8, ResUGroup{gr.du, gr.pu, m, gr.tu, gr.xu, gr.gu}, b->st));
    }
    if (want_g) {
      ProfScope ps(c0, K_BG);
      HIPCHK(c0, launch_res_g_group(gr.sg, fp8, ResGGroup{gr.dg, gr.pg, m, gr.tg, gr.xg, gr.gg}, b->st));
    }
  }
  return GLMR_OK;
}

// L and the gradient of every recording at its current parameters.
glmr_status batch_eval_core(glmr_batch* b) {
  if (!b->grouped) {
    for (glmr_ctx* c : b->ctxs) TRY(eval_core(c, true, false));
    return GLMR_OK;
  }
  for (size_t ci = 0; ci < b->chunks.size(); ++ci) {
    TRY(launch_chunk_groups(b, ci, true, true));
    for (const glmr_batch::Group& gr : b->chunks[ci].groups)
      for (size_t q = 0; q < gr.recs.size(); ++q) {
        glmr_ctx* c = b->ctxs[gr.recs[q]];
        HIPCHK(c, launch_gp_reduce(c->prec, c->Gp, gr.nsplits[q], c->Np, c->G64, ci == 0, b->st));
      }
  }
  for (glmr_ctx* c : b->ctxs) TRY(eval_finish(c, true, false));
  return GLMR_OK;
}

glmr_status batch_eval_theta(glmr_batch* b, bool trial) {
  for (glmr_ctx* c : b->ctxs) {
    const AscentArgs& a = c->asc;
    HIPCHK(c, launch_pack_theta(c->N, c->Np, a.P, trial ? a.theta_try : a.theta, c->J64, c->mu, c->st));
    TRY(prepare_params(c));
  }
  TRY(batch_eval_core(b));
  for (glmr_ctx* c : b->ctxs) {
    const AscentArgs& a = c->asc;
    HIPCHK(c, launch_pack_grad(c->N, c->Np, a.P, c->gJ, c->gmu, c->ll_rows, trial ? a.g_try : a.g,
                               trial ? a.f_try : a.f, c->st));
    HIPCHK(c, launch_penalty(a, trial ? a.theta_try : a.theta, trial ? a.g_try : a.g, trial ? a.f_try : a.f,
                             c->st));
  }
  return GLMR_OK;
}

}  // namespace

extern "C" {

glmr_status glmr_fit(glmr_ctx* c, const glmr_fit_opts* o, glmr_fit_report* rep) {
  if (!c) return GLMR_EINVAL;
  c->err.clear();
  return fit_one(c, o, rep);
}

}  // extern "C"

// ------------------------------------------------------------ checkpoints
namespace {

// Fixed head of a checkpoint; the arrays follow in the order of state_arrays.
struct StateHead {
  char magic[8];  // "GLMRST01"
  int32_t n_neurons, time_mode;
  int64_t n_bins;
  double dt, tau;
  int64_t d, d_self;
  int32_t precision, m;  // m = 0: parameters only, no ascent
  uint64_t spikes_fp;    // FNV-1a over the spike count, the per-neuron counts q_i and the raster digest
  double alpha, eps, jmax, mu_lo, mu_hi;
};
constexpr char kStateMagic[8] = {'G', 'L', 'M', 'R', 'S', 'T', '0', '2'};
static_assert(offsetof(StateHead, precision) == 56, "the Python binding reads the precision at byte 56");

uint64_t spikes_fingerprint(const glmr_ctx* c) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](uint64_t v) {
    for (int b = 0; b < 8; ++b) {
      h ^= (v >> (8 * b)) & 0xffu;
      h *= 1099511628211ull;
    }
  };
  mix((uint64_t)c->nspk);
  for (int i = 0; i < c->N; ++i) mix((uint64_t)c->q_host[i]);
  mix(c->raster_digest);
  return h;
}

// One device array of the ascent state: pointer and byte count.
struct Span {
  void* p;
  size_t bytes;
};

std::vector<Span> state_arrays(glmr_ctx* c) {
  AscentArgs& a = c->asc;
  const size_t N = (size_t)c->N, np = N * (size_t)(c->N + 1), m = (size_t)a.m, d8 = sizeof(double),
               i4 = sizeof(int32_t);
  return {{a.theta, np * d8}, {a.theta_try, np * d8}, {a.g, np * d8},       {a.g_try, np * d8},
          {a.d, np * d8},     {a.S, np * m * d8},     {a.Y, np * m * d8},   {a.rho, m * N * d8},
          {a.f, N * d8},      {a.f_try, N * d8},      {a.step, N * d8},     {a.gd, N * d8},
          {a.eta, N * d8},    {a.gstep, N * d8},      {a.hist_len, N * i4}, {a.hist_head, N * i4},
          {a.state, N * i4},  {a.accepted, N * i4},   {a.bt, N * i4}};
}

size_t state_bytes(glmr_ctx* c, int m) {
  const size_t N = (size_t)c->N, np = N * (size_t)(c->N + 1), d8 = sizeof(double), i4 = sizeof(int32_t);
  size_t n = sizeof(StateHead) + (N * N + N) * d8;
  if (m > 0) n += (5 * np + 2 * np * (size_t)m + (size_t)m * N + 6 * N) * d8 + 5 * N * i4;
  return n;
}

}  // namespace

extern "C" {

glmr_status glmr_get_state(glmr_ctx* c, void* buf, size_t* len) {
  if (!c) return GLMR_EINVAL;
  c->err.clear();
  if (!len) return fail(c, GLMR_EINVAL, "null length");
  if (!c->have_spikes || !c->have_params) return fail(c, GLMR_ESTATE, "set spikes and parameters first");
  const int m = c->asc_live ? c->asc.m : 0;
  const size_t need = state_bytes(c, m);
  if (!buf) {
    *len = need;
    return GLMR_OK;
  }
  if (*len < need) {
    *len = need;
    return fail(c, GLMR_EINVAL, "the buffer holds %zu bytes, the state %zu", *len, need);
  }
  HIPCHK(c, hipSetDevice(c->cfg.device));
  StateHead h{};
  std::memcpy(h.magic, kStateMagic, 8);
  h.n_neurons = c->N;
  h.time_mode = c->evm ? GLMR_TIME_EVENTS : GLMR_TIME_GRID;
  h.n_bins = c->B;
  h.dt = c->dt;
  h.tau = c->tau;
  h.d = c->dly;
  h.d_self = c->dly_s;
  h.precision = public_precision(c);
  h.m = m;
  h.spikes_fp = spikes_fingerprint(c);
  h.alpha = c->asc.alpha;
  h.eps = c->asc.eps;
  h.jmax = c->asc.jmax;
  h.mu_lo = c->asc.mu_lo;
  h.mu_hi = c->asc.mu_hi;
  unsigned char* o = (unsigned char*)buf;
  std::memcpy(o, &h, sizeof h);
  o += sizeof h;
  const size_t N = (size_t)c->N;
  HIPCHK(c, hipMemcpy2DAsync(o, N * sizeof(double), c->J64, c->Np * sizeof(double), N * sizeof(double), N,
                             hipMemcpyDeviceToHost, c->st));
  o += N * N * sizeof(double);
  HIPCHK(c, hipMemcpyAsync(o, c->mu, N * sizeof(double), hipMemcpyDeviceToHost, c->st));
  o += N * sizeof(double);
  if (m > 0)
    for (const Span& s : state_arrays(c)) {
      HIPCHK(c, hipMemcpyAsync(o, s.p, s.bytes, hipMemcpyDeviceToHost, c->st));
      o += s.bytes;
    }
  HIPCHK(c, hipStreamSynchronize(c->st));
  *len = need;
  return GLMR_OK;
}

glmr_status glmr_set_state(glmr_ctx* c, const void* buf, size_t len) {
  if (!c) return GLMR_EINVAL;
  c->err.clear();
  if (!buf) return fail(c, GLMR_EINVAL, "null state");
  if (!c->have_spikes) return fail(c, GLMR_ESTATE, "set the spikes of the checkpointed recording first");
  StateHead h{};
  if (len < sizeof h) return fail(c, GLMR_EINVAL, "state too short");
  std::memcpy(&h, buf, sizeof h);
  if (std::memcmp(h.magic, kStateMagic, 8) != 0) return fail(c, GLMR_EINVAL, "not a checkpoint of this library");
  const int32_t tm = c->evm ? GLMR_TIME_EVENTS : GLMR_TIME_GRID;
  if (h.n_neurons != c->N || h.n_bins != c->B || h.time_mode != tm || h.dt != c->dt)
    return fail(c, GLMR_EINVAL, "the checkpoint is of another recording shape (N, n_bins, dt or time mode)");
  if (h.spikes_fp != spikes_fingerprint(c))
    return fail(c, GLMR_EINVAL, "the checkpoint is of other spikes (spike counts or raster differ)");
  if (h.m < 0 || h.m > 64 || len != state_bytes(c, h.m)) return fail(c, GLMR_EINVAL, "state length or history");
  if (!(h.tau > 0) || !std::isfinite(h.tau)) return fail(c, GLMR_EINVAL, "bad tau in the checkpoint");
  TRY(glmr_set_precision(c, h.precision));
  if (!c->evm && (h.d != c->dly || h.d_self != c->dly_s)) TRY(glmr_set_delays(c, h.d, h.d_self));
  if (!c->have_kernel || h.tau != c->tau) TRY(glmr_set_kernel(c, h.tau));
  const unsigned char* p = (const unsigned char*)buf + sizeof h;
  const size_t N = (size_t)c->N;
  TRY(glmr_set_params(c, (const double*)p, (const double*)(p + N * N * sizeof(double)), GLMR_HOST));
  p += (N * N + N) * sizeof(double);
  if (h.m > 0) {
    TRY(alloc_ascent(c, h.m));
    for (const Span& s : state_arrays(c)) {
      HIPCHK(c, hipMemcpyAsync(s.p, p, s.bytes, hipMemcpyHostToDevice, c->st));
      p += s.bytes;
    }
    c->asc.alpha = h.alpha;
    c->asc.eps = h.eps;
    c->asc.jmax = h.jmax;
    c->asc.mu_lo = h.mu_lo;
    c->asc.mu_hi = h.mu_hi;
    HIPCHK(c, hipStreamSynchronize(c->st));
    c->asc_live = true;
    c->asc_hist = true;
  }
  return GLMR_OK;
}

glmr_status glmr_batch_create(glmr_ctx* const* ctxs, int32_t n, glmr_batch** out) {
  if (!out) return GLMR_EINVAL;
  *out = nullptr;
  if (!ctxs || n < 1) return GLMR_EINVAL;
  for (int r = 0; r < n; ++r) {
    if (!ctxs[r]) return GLMR_EINVAL;
    if (ctxs[r]->cfg.device != ctxs[0]->cfg.device || public_precision(ctxs[r]) != public_precision(ctxs[0]))
      return GLMR_EINVAL;
    for (int q = 0; q < r; ++q)
      if (ctxs[q] == ctxs[r]) return GLMR_EINVAL;  // each recording once
  }
  if (hipSetDevice(ctxs[0]->cfg.device) != hipSuccess) return GLMR_EDEVICE;
  glmr_batch* b = new glmr_batch();
  b->ctxs.assign(ctxs, ctxs + n);
  b->dev = ctxs[0]->cfg.device;
  if (hipStreamCreate(&b->st) != hipSuccess || hipHostMalloc((void**)&b->hsum, sizeof(int32_t)) != hipSuccess) {
    if (b->st) hipStreamDestroy(b->st);
    delete b;
    return GLMR_EDEVICE;
  }
  *out = b;
  return GLMR_OK;
}

void glmr_batch_destroy(glmr_batch* b) {
  if (!b) return;
  hipSetDevice(b->dev);
  hipStreamSynchronize(b->st);
  free_queues(b);
  if (b->hsum) hipHostFree(b->hsum);
  hipStreamDestroy(b->st);
  delete b;
}

}  // extern "C"

namespace {

// Grouped mode (every recording's trace resident, one precision) and its tile
// shapes, then the work queues; the contexts must have spikes, kernel and params.
glmr_status batch_prepare(glmr_batch* b) {
  bool grouped = true;
  for (glmr_ctx* c : b->ctxs) {
    // the grouped launches take one precision for all (a context may have
    // been switched since the batch was made)
    if (public_precision(c) != public_precision(b->ctxs[0]))
      return fail(c, GLMR_ESTATE, "the batch's recordings no longer share one precision");
    TRY(check_ready(c));
    grouped = grouped && c->resident && !self_delayed(c) && !c->evm;
  }
  b->grouped = grouped;
  const size_t n = b->ctxs.size();
  b->rec_u.assign(n, -1);
  b->rec_g.assign(n, -1);
  for (size_t r = 0; r < n; ++r) {
    glmr_ctx* c = b->ctxs[r];
    const int k = shape_class(c);
    const int u = b->tuned_u[k], g = b->tuned_g[k];
    b->rec_u[r] = (u >= 0 && shape_ok_u(c, u)) ? u : c->res_shape_u;
    b->rec_g[r] = (g >= 0 && shape_ok(c, g)) ? g : c->res_shape_g;
  }
  return build_queues(b);
}

}  // namespace

extern "C" {

glmr_status glmr_batch_eval(glmr_batch* b, double* ll) {
  if (!b) return GLMR_EINVAL;
  HIPCHK(b->ctxs[0], hipSetDevice(b->dev));
  OnBatchStream on(b);
  TRY(batch_prepare(b));
  TRY(batch_eval_core(b));
  for (glmr_ctx* c : b->ctxs)
    HIPCHK(c, hipMemcpyAsync(c->host_scal, c->scal, sizeof(double), hipMemcpyDeviceToHost, b->st));
  HIPCHK(b->ctxs[0], hipStreamSynchronize(b->st));
  for (size_t r = 0; r < b->ctxs.size(); ++r) {
    if (ll) ll[r] = b->ctxs[r]->host_scal[0];
    if (!std::isfinite(b->ctxs[r]->host_scal[0]))
      return fail(b->ctxs[r], GLMR_ENONFINITE, "log-likelihood is not finite");
  }
  return GLMR_OK;
}

glmr_status glmr_batch_get_grad(glmr_batch* b, int32_t r, double* grad_J, double* grad_mu, int32_t where) {
  if (!b || r < 0 || r >= (int32_t)b->ctxs.size()) return GLMR_EINVAL;
  glmr_ctx* c = b->ctxs[r];
  if (where != GLMR_HOST && where != GLMR_DEVICE) return fail(c, GLMR_EINVAL, "bad where");
  if (!c->gJ) return fail(c, GLMR_ESTATE, "no batch evaluation yet");
  if (grad_mu) HIPCHK(c, hipMemcpyAsync(grad_mu, c->gmu, c->N * sizeof(double), kind_to(where), c->st));
  if (grad_J)
    HIPCHK(c, hipMemcpy2DAsync(grad_J, c->N * sizeof(double), c->gJ, c->Np * sizeof(double),
                               c->N * sizeof(double), c->N, kind_to(where), c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  return GLMR_OK;
}

glmr_status glmr_batch_autotune(glmr_batch* b, const char* cache_path, int32_t* shape_u, int32_t* shape_g) {
  if (!b) return GLMR_EINVAL;
  glmr_ctx* c0 = b->ctxs[0];
  HIPCHK(c0, hipSetDevice(b->dev));
  OnBatchStream on(b);
  for (int k = 0; k < 2; ++k) b->tuned_u[k] = b->tuned_g[k] = -1;
  TRY(batch_prepare(b));
  if (!b->grouped) {
    if (shape_u) *shape_u = -1;
    if (shape_g) *shape_g = -1;
    return GLMR_OK;
  }
  // key: architecture, precision, recording count and sizes
  uint64_t h = 1469598103934665603ull;
  for (glmr_ctx* c : b->ctxs) {
    for (int64_t v : {c->Np, c->Bp, c->L}) {
      h ^= (uint64_t)v;
      h *= 1099511628211ull;
    }
  }
  char kb[64];
  std::snprintf(kb, sizeof(kb), "batch%zu-%016llx", b->ctxs.size(), (unsigned long long)h);
  std::string arch = tune_key(c0);
  arch = arch.substr(0, arch.find(' '));
  const std::string key = arch + " " + kb + " " + std::to_string(c0->prec);
  bool have[2] = {false, false};
  for (glmr_ctx* c : b->ctxs) have[shape_class(c)] = true;
  auto all_ok = [&](int cls, int k, bool u) {
    for (glmr_ctx* c : b->ctxs)
      if (shape_class(c) == cls && !(u ? shape_ok_u(c, k) : shape_ok(c, k))) return false;
    return true;
  };
  auto all_tune_u = [&](int cls, int k) {
    for (glmr_ctx* c : b->ctxs)
      if (shape_class(c) == cls && !shape_tune_u(c, k)) return false;
    return true;
  };
  bool cached = false;
  if (cache_path) {
    if (FILE* f = std::fopen(cache_path, "r")) {
      char line[512];
      while (std::fgets(line, sizeof(line), f)) {
        char a[128], k2[128];
        int prec = -1, u0 = -1, g0 = -1, u1 = -1, g1 = -1;
        if (std::sscanf(line, "glmrec-tune-batch %127s %127s %d %d %d %d %d", a, k2, &prec, &u0, &g0, &u1, &g1) ==
            7) {
          const std::string kk = std::string(a) + " " + k2 + " " + std::to_string(prec);
          const int us[2] = {u0, u1}, gs[2] = {g0, g1};
          bool ok = kk == key;
          for (int c = 0; c < 2 && ok; ++c)
            if (have[c]) ok = all_ok(c, us[c], true) && all_ok(c, gs[c], false);
          if (ok) {
            for (int c = 0; c < 2; ++c) {
              b->tuned_u[c] = have[c] ? us[c] : -1;
              b->tuned_g[c] = have[c] ? gs[c] : -1;
            }
            cached = true;
          }
        }
      }
      std::fclose(f);
    }
  }
  if (!cached) {
    // one class at a time (the other at its current shapes): the time of the
    // first chunk's launches of each contraction, every group included
    int n = 0;
    (void)res_shapes(&n);
    double tu = 0, tg = 0;
    for (int cls = 0; cls < 2; ++cls) {
      if (!have[cls]) continue;
      int best_u = -1, best_g = -1;
      double bu = 1e300, bg = 1e300;
      for (int k = 0; k < n; ++k) {
        const bool oku = all_tune_u(cls, k), okg = all_ok(cls, k, false);
        if (!oku && !okg) continue;
        const int su = b->tuned_u[cls], sg = b->tuned_g[cls];
        b->tuned_u[cls] = oku ? k : su;
        b->tuned_g[cls] = okg ? k : sg;
        TRY(batch_prepare(b));
        double ms = 0;
        if (oku) {
          TRY(time_launches(c0, [&] { return launch_chunk_groups(b, 0, true, false) == GLMR_OK ? hipSuccess : hipErrorUnknown; }, 3, &ms));
          if (ms < bu) { bu = ms; best_u = k; }
        }
        if (okg) {
          TRY(time_launches(c0, [&] { return launch_chunk_groups(b, 0, false, true) == GLMR_OK ? hipSuccess : hipErrorUnknown; }, 3, &ms));
          if (ms < bg) { bg = ms; best_g = k; }
        }
        b->tuned_u[cls] = su;
        b->tuned_g[cls] = sg;
      }
      b->tuned_u[cls] = best_u;
      b->tuned_g[cls] = best_g;
      tu = bu;
      tg = bg;
    }
    if (cache_path) {
      if (FILE* f = std::fopen(cache_path, "a")) {
        std::fprintf(f, "glmrec-tune-batch %s %d %d %d %d %.4f %.4f\n", key.c_str(), b->tuned_u[0], b->tuned_g[0],
                     b->tuned_u[1], b->tuned_g[1], tu, tg);
        std::fclose(f);
      }
    }
  }
  TRY(batch_prepare(b));
  const int cls = have[0] ? 0 : 1;
  if (shape_u) *shape_u = b->tuned_u[cls];
  if (shape_g) *shape_g = b->tuned_g[cls];
  return GLMR_OK;
}

glmr_status glmr_batch_fit(glmr_batch* b, const glmr_fit_opts* o_in, glmr_fit_report* reps) {
  if (!b) return GLMR_EINVAL;
  glmr_ctx* c0 = b->ctxs[0];
  HIPCHK(c0, hipSetDevice(b->dev));
  glmr_fit_opts o;
  for (glmr_ctx* c : b->ctxs) {
    c->err.clear();
    TRY(check_fit_opts(c, o_in, &o));
    if (o.resume || o.keep_history)
      return fail(c, GLMR_EINVAL, "a batch fit starts afresh (resume each context on its own)");
  }
  auto t_start = std::chrono::steady_clock::now();
  OnBatchStream on(b);
  for (glmr_ctx* c : b->ctxs) TRY(fit_begin(c, o));
  TRY(batch_prepare(b));
  const double ftol = o.ftol > 0 ? o.ftol : default_ftol(c0);
  TRY(batch_eval_theta(b, false));
  for (glmr_ctx* c : b->ctxs) HIPCHK(c, launch_lbfgs_direction(c->asc, 1, b->st));
  // one ascent step of every recording, captured once and replayed
  auto step = [&]() -> glmr_status {
    for (glmr_ctx* c : b->ctxs) HIPCHK(c, launch_make_trial(c->asc, b->st));
    TRY(batch_eval_theta(b, true));
    for (glmr_ctx* c : b->ctxs) {
      const AscentArgs& a = c->asc;
      HIPCHK(c, launch_armijo_async(a, 1e-4, o.max_backtracks, b->st));
      HIPCHK(c, launch_accept_update(a, ftol, nullptr, 1, b->st));
      HIPCHK(c, launch_lbfgs_direction(a, 1, b->st));
      HIPCHK(c, launch_count_active(a, c->counters, b->st));
    }
    HIPCHK(c0, launch_sum_counters(b->dcnt, (int)b->ctxs.size(), b->dsum, b->st));
    return GLMR_OK;
  };
  GraphRun gr;
  if (use_graphs()) {
    auto body = [&]() -> glmr_status {
      for (glmr_ctx* c : b->ctxs) c->capturing = true;
      const glmr_status s1 = step();
      for (glmr_ctx* c : b->ctxs) c->capturing = false;
      return s1;
    };
    TRY(gr.capture(c0, b->st, body));
  }
  int iters = 0, active = 1;
  for (; iters < o.max_iter && active > 0; ++iters) {
    if (gr.exec) HIPCHK(c0, hipGraphLaunch(gr.exec, b->st));
    else TRY(step());
    HIPCHK(c0, hipMemcpyAsync(b->hsum, b->dsum, sizeof(int32_t), hipMemcpyDeviceToHost, b->st));
    HIPCHK(c0, hipStreamSynchronize(b->st));
    active = b->hsum[0];
  }
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  glmr_status worst = GLMR_OK;
  for (size_t r = 0; r < b->ctxs.size(); ++r) {
    const glmr_status s1 = fit_end(b->ctxs[r], iters, iters + 1, secs, reps ? &reps[r] : nullptr);
    if (s1 < 0) return s1;
    if (s1 == GLMR_NOT_CONVERGED) worst = s1;
  }
  return worst;
}

}  // extern "C"

namespace {
}  // namespace

// ====================================================================== C ABI
extern "C" {

const char* glmr_status_string(glmr_status s) {
  switch (s) {
    case GLMR_OK: return "ok";
    case GLMR_NOT_CONVERGED: return "not converged (iteration cap reached)";
    case GLMR_EINVAL: return "invalid argument";
    case GLMR_ENOMEM: return "out of device memory";
    case GLMR_EDEVICE: return "HIP runtime error";
    case GLMR_ENOSPIKES: return "a neuron has no spikes (its MLE does not exist)";
    case GLMR_ENONFINITE: return "non-finite likelihood";
    case GLMR_ESTATE: return "call order";
  }
  return "unknown status";
}

const char* glmr_last_error(const glmr_ctx* c) { return c ? c->err.c_str() : "null context"; }

void glmr_fit_defaults(glmr_fit_opts* o) {
  if (!o) return;
  o->max_iter = 500;
  o->ftol = 0.0;
  o->lbfgs_m = 40;  // at N = 1000, 3.6e6 bins (BF16): 46 steps to the stopping test, 82 with 10
  o->max_backtracks = 30;
  o->warm_start_mu = 0;
  o->from_zero = 0;
  o->l1_alpha = 0.0;
  o->l1_eps = 0.0;
  o->j_max = 0.0;
  o->rate_min = 0.0;
  o->rate_max = 0.0;
  o->resume = 0;
  o->keep_history = 0;
}

glmr_status glmr_create(const glmr_config* cfg, glmr_ctx** out) {
  if (!out) return GLMR_EINVAL;
  *out = nullptr;
  if (!cfg) return GLMR_EINVAL;
  if (cfg->n_neurons < 1 || cfg->n_neurons > 65536 || cfg->n_bins < 1 || !(cfg->dt > 0) ||
      !std::isfinite(cfg->dt) || cfg->chunk_bins < 0 || cfg->precision < 0 || cfg->precision > 4 ||
      !(cfg->tile_n == 0 || cfg->tile_n == 128 || cfg->tile_n == 256) || cfg->trace < 0 || cfg->trace > 2)
    return GLMR_EINVAL;
  if ((cfg->precision == GLMR_FP8 || cfg->precision == GLMR_BF16_J2) && cfg->trace == GLMR_TRACE_RECOMPUTE)
    return GLMR_EINVAL;  // FP8 and two-term J contractions exist only on the resident trace
  if (cfg->time_mode != GLMR_TIME_GRID && cfg->time_mode != GLMR_TIME_EVENTS) return GLMR_EINVAL;
  if (cfg->time_mode == GLMR_TIME_EVENTS && cfg->precision == GLMR_FP8)
    return GLMR_EINVAL;  // the event grid's contractions run in FP64, FP32 or BF16
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
    (void)hipGetLastError();
    return GLMR_EDEVICE;
  }
  if (cfg->device < 0 || cfg->device >= ndev) return GLMR_EINVAL;
  if (hipSetDevice(cfg->device) != hipSuccess) return GLMR_EDEVICE;
  // the static scratch's address on this device (used by glmr_set_kernel_noalloc;
  // a failure here is reported by that call)
  (void)scratch_init(cfg->device);
  glmr_ctx* c = new glmr_ctx();
  c->cfg = *cfg;
  c->N = cfg->n_neurons;
  c->B = cfg->n_bins;
  c->dt = cfg->dt;
  c->evm = cfg->time_mode == GLMR_TIME_EVENTS;
  c->j2 = cfg->precision == GLMR_BF16_J2;
  c->prec = c->j2 ? GLMR_BF16 : cfg->precision;
  int tile = cfg->tile_n;
  if (tile == 0) tile = ((c->prec == GLMR_BF16 || c->prec == GLMR_FP8) && c->N <= 384) ? 128 : 256;
  c->Np = rup(c->N, tile);
  c->Bp = rup(c->B, GLMR_TT);
  c->NS = c->Bp / GLMR_SUB;
  c->NIB = c->Np / GLMR_IB;
  setup_precision(c);
  if (cfg->stream) {
    c->st = (hipStream_t)cfg->stream;
  } else {
    if (hipStreamCreate(&c->st) != hipSuccess) {
      delete c;
      return GLMR_EDEVICE;
    }
    c->own_stream = true;
  }
  *out = c;
  return GLMR_OK;
}

void glmr_destroy(glmr_ctx* c) {
  if (!c) return;
  hipSetDevice(c->cfg.device);
  hipStreamSynchronize(c->st);
  for (void* p : c->allocs) hipFree(p);
  if (c->host_scal) hipHostFree(c->host_scal);
  if (c->host_cnt) hipHostFree(c->host_cnt);
  for (auto& r : c->pending) {
    hipEventDestroy(r.a);
    hipEventDestroy(r.b);
  }
  for (auto e : c->pool) hipEventDestroy(e);
  if (c->own_stream) hipStreamDestroy(c->st);
  delete c;
}

namespace {

// Spike ingest from device arrays of (bin, neuron) pairs (spike layout of the
// regular grid, or the pseudo-bins of the event grid).
glmr_status ingest_pairs(glmr_ctx* c, const int64_t* bin, const int32_t* neuron, int64_t n) {
  ProfScope ps(c, K_INGEST);
  c->asc_live = false;
  c->asc_hist = false;
  const int64_t nseg = c->NS * c->NIB;
  IngestBufs b{};
  b.n = n;
  b.N = c->N;
  b.B = c->B;
  b.NS = c->NS;
  b.NIB = c->NIB;
  b.bin = bin;
  b.neu = neuron;
  unsigned long long* bad = nullptr;
  int32_t *cnt = nullptr, *cursor = nullptr, *maxmult = nullptr;
  int64_t* scan_tmp = nullptr;
  TRY(dalloc(c, bad, 2));
  TRY(dalloc(c, cnt, (size_t)nseg + 1));
  TRY(dalloc(c, cursor, (size_t)nseg + 1));
  TRY(dalloc(c, maxmult, 1));
  TRY(dalloc(c, scan_tmp, (size_t)ingest_scan_tmp_len(nseg)));
  if (!c->seg_off) TRY(dalloc(c, c->seg_off, (size_t)nseg + 1));
  dfree(c, c->seg_ent);
  TRY(dalloc(c, c->seg_ent, (size_t)std::max<int64_t>(n, 1)));
  if (!c->q) TRY(dalloc(c, c->q, (size_t)c->Np));
  HIPCHK(c, hipMemsetAsync(bad, 0, sizeof(unsigned long long), c->st));
  HIPCHK(c, hipMemsetAsync(bad + 1, 0xff, sizeof(unsigned long long), c->st));
  HIPCHK(c, hipMemsetAsync(cnt, 0, (nseg + 1) * sizeof(int32_t), c->st));
  HIPCHK(c, hipMemsetAsync(cursor, 0, (nseg + 1) * sizeof(int32_t), c->st));
  HIPCHK(c, hipMemsetAsync(maxmult, 0, sizeof(int32_t), c->st));
  HIPCHK(c, hipMemsetAsync(c->q, 0, c->Np * sizeof(int64_t), c->st));
  b.bad = bad;
  b.cnt = cnt;
  b.off = c->seg_off;
  b.cursor = cursor;
  b.ent = c->seg_ent;
  b.q = c->q;
  b.maxmult = maxmult;
  b.scan_tmp = scan_tmp;
  c->have_spikes = false;
  c->have_kernel = false;
  unsigned long long hbad[2] = {0, 0};
  if (n > 0) HIPCHK(c, launch_ingest_count(b, c->st));
  HIPCHK(c, hipMemcpyAsync(hbad, bad, sizeof hbad, hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  if (hbad[0] > 0) return fail(c, GLMR_EINVAL, "%llu spikes out of range; first at index %llu", hbad[0], hbad[1]);
  HIPCHK(c, launch_ingest_scan(b, c->st));
  if (n > 0) HIPCHK(c, launch_ingest_scatter(b, c->st));
  HIPCHK(c, launch_ingest_sort(b, c->st));
  int32_t hmax = 0;
  HIPCHK(c, hipMemcpyAsync(&hmax, maxmult, sizeof hmax, hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  c->planes = std::max(1, (int)hmax);
  const size_t nm = (size_t)c->planes * c->NS * c->Np;
  dfree(c, c->masks);
  dfree(c, c->masks0);
  TRY(dalloc(c, c->masks, nm));
  HIPCHK(c, hipMemsetAsync(c->masks, 0, nm * sizeof(uint64_t), c->st));
  HIPCHK(c, launch_ingest_masks(b, c->masks, c->planes, c->Np, c->st));
  // digest of the recorded raster (before any delay shifts it), for checkpoints
  HIPCHK(c, hipMemsetAsync(bad, 0, 2 * sizeof(unsigned long long), c->st));
  HIPCHK(c, launch_digest_u64(c->masks, (int64_t)c->planes * c->NS, c->NS, c->Np, c->N, bad, c->st));
  if (c->evm) HIPCHK(c, launch_digest_u64((const uint64_t*)c->tslot, 1, 1, 0, c->B + 1, bad + 1, c->st));
  unsigned long long dig[2] = {0, 0};
  HIPCHK(c, hipMemcpyAsync(dig, bad, sizeof dig, hipMemcpyDeviceToHost, c->st));
  c->q_host.assign(c->Np, 0);
  HIPCHK(c, hipMemcpyAsync(c->q_host.data(), c->q, c->Np * sizeof(int64_t), hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  c->raster_digest = (uint64_t)dig[0] ^ ((uint64_t)dig[1] * 0x9E3779B97F4A7C15ull);
  dfree(c, bad);
  dfree(c, cnt);
  dfree(c, cursor);
  dfree(c, maxmult);
  dfree(c, scan_tmp);
  c->nspk = n;
  c->have_spikes = true;
  TRY(apply_delays(c));
  c->all_spiking = true;
  for (int i = 0; i < c->N; ++i)
    if (c->q_host[i] == 0) c->all_spiking = false;
  if (c->tau > 0) TRY(build_kernel_caches(c, c->keep_y));
  if (!c->all_spiking) return fail(c, GLMR_ENOSPIKES, "some neuron has no spike");
  return GLMR_OK;
}

}  // namespace

glmr_status glmr_set_spikes(glmr_ctx* c, const int64_t* bin, const int32_t* neuron, int64_t n,
                            int32_t where) {
  if (!c) return GLMR_EINVAL;
  c->err.clear();
  if (c->evm) return fail(c, GLMR_ESTATE, "an event-grid context takes glmr_set_spike_times");
  if (n < 0 || n >= (1ll << 31)) return fail(c, GLMR_EINVAL, "n_spikes must be in [0, 2^31)");
  if (n > 0 && (!bin || !neuron)) return fail(c, GLMR_EINVAL, "null spike arrays");
  if (where != GLMR_HOST && where != GLMR_DEVICE) return fail(c, GLMR_EINVAL, "bad where");
  HIPCHK(c, hipSetDevice(c->cfg.device));
  int64_t* dbin = nullptr;
  int32_t* dneu = nullptr;
  if (where == GLMR_HOST && n > 0) {
    TRY(dalloc(c, dbin, (size_t)n));
    TRY(dalloc(c, dneu, (size_t)n));
    HIPCHK(c, hipMemcpyAsync(dbin, bin, n * sizeof(int64_t), hipMemcpyHostToDevice, c->st));
    HIPCHK(c, hipMemcpyAsync(dneu, neuron, n * sizeof(int32_t), hipMemcpyHostToDevice, c->st));
    bin = dbin;
    neuron = dneu;
  }
  const glmr_status st = ingest_pairs(c, bin, neuron, n);
  HIPCHK(c, hipStreamSynchronize(c->st));
  dfree(c, dbin);
  dfree(c, dneu);
  return st;
}

glmr_status glmr_set_spike_times(glmr_ctx* c, const double* times, const int32_t* neuron, int64_t n,
                                 double T0, double T1, double max_gap, int32_t where) {
  if (!c) return GLMR_EINVAL;
  c->err.clear();
  if (!c->evm) return fail(c, GLMR_ESTATE, "a regular-grid context takes glmr_set_spikes");
  if (n < 0 || n >= (1ll << 31)) return fail(c, GLMR_EINVAL, "n_events must be in [0, 2^31)");
  if (n > 0 && (!times || !neuron)) return fail(c, GLMR_EINVAL, "null event arrays");
  if (where != GLMR_HOST && where != GLMR_DEVICE) return fail(c, GLMR_EINVAL, "bad where");
  if (!std::isfinite(T0) || !std::isfinite(T1) || !(T1 > T0)) return fail(c, GLMR_EINVAL, "need T0 < T1");
  if (std::isnan(max_gap) || std::isinf(max_gap)) return fail(c, GLMR_EINVAL, "bad max_gap");
  const double mg = ev_resolve_max_gap(n, T0, T1, max_gap);
  if (!(mg > 0) || !((T1 - T0) / mg <= 1e9)) return fail(c, GLMR_EINVAL, "max_gap too small");
  HIPCHK(c, hipSetDevice(c->cfg.device));
  c->have_spikes = false;
  c->have_kernel = false;
  double* dt_ = nullptr;
  int32_t* dn_ = nullptr;
  if (where == GLMR_HOST && n > 0) {
    TRY(dalloc(c, dt_, (size_t)n));
    TRY(dalloc(c, dn_, (size_t)n));
    HIPCHK(c, hipMemcpyAsync(dt_, times, n * sizeof(double), hipMemcpyHostToDevice, c->st));
    HIPCHK(c, hipMemcpyAsync(dn_, neuron, n * sizeof(int32_t), hipMemcpyHostToDevice, c->st));
    times = dt_;
    neuron = dn_;
  }
  EvLayoutArgs a{};
  a.n = n;
  a.times = times;
  a.neu = neuron;
  a.N = c->N;
  a.T0 = T0;
  a.T1 = T1;
  a.max_gap = mg;
  a.NS = c->NS;
  const size_t nn = (size_t)std::max<int64_t>(n, 1);
  auto cleanup = [&]() {
    (void)hipStreamSynchronize(c->st);
    dfree(c, dt_);
    dfree(c, dn_);
    dfree(c, a.bad);
    dfree(c, a.cnt);
    dfree(c, a.slot);
    dfree(c, a.scan_tmp);
    dfree(c, a.bins);
  };
  glmr_status st = GLMR_OK;
  do {
    if ((st = dalloc(c, a.bad, 2)) != GLMR_OK) break;
    if ((st = dalloc(c, a.cnt, nn)) != GLMR_OK) break;
    if ((st = dalloc(c, a.slot, nn)) != GLMR_OK) break;
    if ((st = dalloc(c, a.scan_tmp, (size_t)ev_scan_tmp_len(n))) != GLMR_OK) break;
    if ((st = dalloc(c, a.bins, nn)) != GLMR_OK) break;
    unsigned long long hbad[2] = {0, 0};
    if (hipMemsetAsync(a.bad, 0, sizeof(unsigned long long), c->st) != hipSuccess ||
        hipMemsetAsync(a.bad + 1, 0xff, sizeof(unsigned long long), c->st) != hipSuccess ||
        (n > 0 && launch_ev_check(a, c->st) != hipSuccess) ||
        hipMemcpyAsync(hbad, a.bad, sizeof hbad, hipMemcpyDeviceToHost, c->st) != hipSuccess ||
        hipStreamSynchronize(c->st) != hipSuccess) {
      st = fail(c, GLMR_EDEVICE, "event check: %s", hipGetErrorString(hipGetLastError()));
      break;
    }
    if (hbad[0] > 0) {
      st = fail(c, GLMR_EINVAL,
                "%llu events out of [T0, T1), of neuron range, or not in strictly increasing (time, neuron) "
                "order; first at index %llu", hbad[0], hbad[1]);
      break;
    }
    int64_t s_last = 0;
    double t_last = T0;
    if (launch_ev_layout(a, c->st) != hipSuccess ||
        (n > 0 && hipMemcpyAsync(&s_last, a.slot + (n - 1), sizeof s_last, hipMemcpyDeviceToHost, c->st) != hipSuccess) ||
        (n > 0 && hipMemcpyAsync(&t_last, times + (n - 1), sizeof t_last, hipMemcpyDeviceToHost, c->st) != hipSuccess) ||
        hipStreamSynchronize(c->st) != hipSuccess) {
      st = fail(c, GLMR_EDEVICE, "event layout: %s", hipGetErrorString(hipGetLastError()));
      break;
    }
    const int64_t n_tail = ev_host_slots_of_gap(T1 - t_last, mg);
    const int64_t M = s_last + n_tail;
    if (M != c->B) {
      st = fail(c, GLMR_EINVAL, "the events make %lld slots; the context has n_bins = %lld (glmr_event_slots)",
                (long long)M, (long long)c->B);
      break;
    }
    if (!c->tslot && (st = dalloc(c, c->tslot, (size_t)(c->NS * 64 + 1))) != GLMR_OK) break;
    a.tslot = c->tslot;
    if (launch_ev_place(a, s_last, t_last, n_tail, c->st) != hipSuccess) {
      st = fail(c, GLMR_EDEVICE, "event placement: %s", hipGetErrorString(hipGetLastError()));
      break;
    }
    c->T0 = T0;
    c->T1 = T1;
    c->max_gap = mg;
    st = ingest_pairs(c, a.bins, neuron, n);
  } while (false);
  cleanup();
  return st;
}

namespace {
glmr_status reject_event_grid_precision(glmr_ctx* c, int prec) {
  if (c->evm && prec == GLMR_FP8)
    return fail(c, GLMR_EINVAL, "the event grid is evaluated in FP64, FP32 or BF16");
  return GLMR_OK;
}
}  // namespace

glmr_status glmr_set_kernel(glmr_ctx* c, double tau) {
  if (!c) return GLMR_EINVAL;
  c->err.clear();
  if (!(tau > 0) || !std::isfinite(tau)) return fail(c, GLMR_EINVAL, "tau must be positive");
  if (!c->evm && tau < c->dt) return fail(c, GLMR_EINVAL, "tau must be >= dt");
  HIPCHK(c, hipSetDevice(c->cfg.device));
  c->asc_live = false;
  c->asc_hist = false;
  c->tau = tau;
  c->a = std::exp(-c->dt / tau);
  c->have_kernel = false;
  if (!c->have_spikes) return GLMR_OK;  // caches are built when the spikes arrive
  // once dL/dtau has been asked for, keep the tau-derivative caches current
  return build_kernel_caches(c, c->keep_y);
}

glmr_status glmr_set_kernel_noalloc(glmr_ctx* c, double tau) {
  if (!c) return GLMR_EINVAL;
  c->err.clear();
  if (!(tau > 0) || !std::isfinite(tau)) return fail(c, GLMR_EINVAL, "tau must be positive");
  if (!c->evm && tau < c->dt) return fail(c, GLMR_EINVAL, "tau must be >= dt");
  if (!c->have_spikes) return fail(c, GLMR_ESTATE, "set the spikes first");
  if (!c->C64 || !c->dsig || !c->tab)
    return fail(c, GLMR_ESTATE, "the per-tau buffers do not exist yet: call glmr_set_kernel once on this "
                                "context before glmr_set_kernel_noalloc");
  HIPCHK(c, hipSetDevice(c->cfg.device));
  const hipError_t se = scratch_init(c->cfg.device);
  if (se != hipSuccess)
    return fail(c, GLMR_EDEVICE, "hipGetSymbolAddress of the static scratch: %s", hipGetErrorString(se));
  // the fixed temporaries (carry segments, span maximum) and one time split
  // of the spike term must fit
  const int64_t nseg = (c->NS + 63) / 64;
  const bool wy = c->keep_y && !c->evm;
  const size_t need = 2 * ((size_t)nseg * c->Np * 2 * sizeof(double) + 256) + 512 +
                      std::max<size_t>((size_t)c->Np * c->Np * sizeof(double) * (wy ? 2 : 1),
                                       self_delayed(c) ? 64 * (size_t)c->Np * sizeof(double) : 0);
  if (need > kScratchBytes)
    return fail(c, GLMR_EINVAL, "this recording's per-tau set-up needs %zu bytes of scratch; the static "
                                "scratch holds %zu (use glmr_set_kernel)", need, kScratchBytes);
  c->asc_live = false;
  c->asc_hist = false;
  c->tau = tau;
  c->a = std::exp(-c->dt / tau);
  c->have_kernel = false;
  Arena ar;
  ar.base = (unsigned char*)g_scratch_ptr[c->cfg.device];
  ar.cap = kScratchBytes;
  return build_kernel_caches(c, c->keep_y, &ar);
}

glmr_status glmr_set_delays(glmr_ctx* c, int64_t d, int64_t d_self) {
  if (!c) return GLMR_EINVAL;
  c->err.clear();
  if (c->evm) return fail(c, GLMR_EINVAL, "delays are defined on the regular grid");
  if (d < 0 || d_self < 0 || d >= c->B || d_self >= c->B)
    return fail(c, GLMR_EINVAL, "delays must be in [0, n_bins)");
  if (d != d_self && c->prec == PREC_FP8)
    return fail(c, GLMR_EINVAL, "a self-delay other than d needs FP64, FP32 or BF16");
  HIPCHK(c, hipSetDevice(c->cfg.device));
  HIPCHK(c, hipStreamSynchronize(c->st));
  c->asc_live = false;
  c->asc_hist = false;
  c->dly = d;
  c->dly_s = d_self;
  if (!c->have_spikes) return GLMR_OK;  // applied when the spikes arrive
  c->have_kernel = false;
  TRY(apply_delays(c));
  if (c->tau > 0) TRY(build_kernel_caches(c, c->keep_y));
  return GLMR_OK;
}

glmr_status glmr_set_params(glmr_ctx* c, const double* J, const double* mu, int32_t where) {
  if (!c) return GLMR_EINVAL;
  c->err.clear();
  if (!J || !mu) return fail(c, GLMR_EINVAL, "null parameter arrays");
  if (where != GLMR_HOST && where != GLMR_DEVICE) return fail(c, GLMR_EINVAL, "bad where");
  HIPCHK(c, hipSetDevice(c->cfg.device));
  c->asc_live = false;
  const int64_t Np = c->Np;
  if (!c->J64) {
    TRY(dalloc(c, c->J64, (size_t)Np * Np));
    HIPCHK(c, hipMemsetAsync(c->J64, 0, Np * Np * sizeof(double), c->st));
    TRY(dalloc(c, c->mu, (size_t)Np));
    HIPCHK(c, hipMemsetAsync(c->mu, 0, Np * sizeof(double), c->st));
    void* p = nullptr;
    TRY(dalloc(c, (unsigned char*&)p, jc_size(c)));
    c->Jc = p;
    TRY(dalloc(c, c->Jr, (size_t)Np * Np));
    TRY(dalloc(c, c->rowscale, (size_t)Np));
  }
  HIPCHK(c, hipMemcpy2DAsync(c->J64, Np * sizeof(double), J, c->N * sizeof(double),
                             c->N * sizeof(double), c->N, kind_from(where), c->st));
  HIPCHK(c, hipMemcpyAsync(c->mu, mu, c->N * sizeof(double), kind_from(where), c->st));
  TRY(prepare_params(c));
  if (where == GLMR_HOST) HIPCHK(c, hipStreamSynchronize(c->st));
  c->have_params = true;
  return GLMR_OK;
}

glmr_status glmr_set_precision(glmr_ctx* c, int32_t precision) {
  if (!c) return GLMR_EINVAL;
  c->err.clear();
  if (precision < 0 || precision > 4)
    return fail(c, GLMR_EINVAL, "precision must be FP64, FP32, BF16, FP8 or BF16 with a two-term J");
  if ((precision == GLMR_FP8 || precision == GLMR_BF16_J2) && c->cfg.trace == GLMR_TRACE_RECOMPUTE)
    return fail(c, GLMR_EINVAL, "FP8 and the two-term J need the resident trace");
  TRY(reject_event_grid_precision(c, precision));
  if (precision == GLMR_FP8 && c->dly != c->dly_s)
    return fail(c, GLMR_EINVAL, "a self-delay other than d needs FP64, FP32 or BF16");
  const bool j2 = precision == GLMR_BF16_J2;
  const int prec = j2 ? GLMR_BF16 : precision;
  if (prec == c->prec && j2 == c->j2) return GLMR_OK;
  HIPCHK(c, hipSetDevice(c->cfg.device));
  HIPCHK(c, hipStreamSynchronize(c->st));
  c->asc_live = false;
  c->cfg.precision = precision;
  if (prec == c->prec) {
    // BF16 <-> BF16 with a two-term J: the same trace and workspace, only the
    // staged weights change (the two-term J needs the trace resident)
    c->j2 = j2;
    if (c->Jc) {
      unsigned char* jc = (unsigned char*)c->Jc;
      dfree(c, jc);
      void* p = nullptr;
      TRY(dalloc(c, (unsigned char*&)p, jc_size(c)));
      c->Jc = p;
    }
    if (j2 && c->have_kernel && !c->resident) TRY(build_kernel_caches(c, c->have_y));
    if (c->have_params) TRY(prepare_params(c));
    HIPCHK(c, hipStreamSynchronize(c->st));
    return GLMR_OK;
  }
  c->j2 = j2;
  c->prec = prec;
  setup_precision(c);
  // buffers whose size or element type depend on the precision
  unsigned char* w = (unsigned char*)c->W;
  dfree(c, w);
  c->W = nullptr;
  unsigned char* gp = (unsigned char*)c->Gp;
  dfree(c, gp);
  c->Gp = nullptr;
  dfree(c, c->rowpart);
  dfree(c, c->rowpartV);
  dfree(c, c->gpart);
  if (c->Jc) {
    unsigned char* jc = (unsigned char*)c->Jc;
    dfree(c, jc);
    void* p = nullptr;
    TRY(dalloc(c, (unsigned char*&)p, jc_size(c)));
    c->Jc = p;
  }
  if (c->have_kernel) TRY(build_kernel_caches(c, c->have_y));
  if (c->have_params) TRY(prepare_params(c));
  HIPCHK(c, hipStreamSynchronize(c->st));
  return GLMR_OK;
}

glmr_status glmr_get_params(glmr_ctx* c, double* J, double* mu, double* tau, int32_t where) {
  if (!c) return GLMR_EINVAL;
  c->err.clear();
  if (where != GLMR_HOST && where != GLMR_DEVICE) return fail(c, GLMR_EINVAL, "bad where");
  if (tau) *tau = c->tau;
  if ((J || mu) && !c->have_params) return fail(c, GLMR_ESTATE, "no parameters set");
  HIPCHK(c, hipSetDevice(c->cfg.device));
  if (J)
    HIPCHK(c, hipMemcpy2DAsync(J, c->N * sizeof(double), c->J64, c->Np * sizeof(double),
                               c->N * sizeof(double), c->N, kind_to(where), c->st));
  if (mu) HIPCHK(c, hipMemcpyAsync(mu, c->mu, c->N * sizeof(double), kind_to(where), c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  return GLMR_OK;
}

glmr_status glmr_eval(glmr_ctx* c, double* ll, double* ll_rows, double* grad_J, double* grad_mu,
                      double* grad_tau, int32_t where) {
  if (!c) return GLMR_EINVAL;
  c->err.clear();
  if (where != GLMR_HOST && where != GLMR_DEVICE) return fail(c, GLMR_EINVAL, "bad where");
  TRY(check_ready(c));
  HIPCHK(c, hipSetDevice(c->cfg.device));
  const bool want_grad = grad_J || grad_mu;
  const bool want_tau = grad_tau != nullptr;
  if (want_tau && c->j2)
    return fail(c, GLMR_EINVAL, "dL/dtau is not available with the two-term J (use GLMR_BF16)");
  if (want_tau && c->prec == PREC_FP8)
    return fail(c, GLMR_EINVAL, "dL/dtau is evaluated in FP64, FP32 or BF16, not FP8");
  if (want_tau && c->evm) return fail(c, GLMR_EINVAL, "dL/dtau is not available on the event grid");
  if (want_tau && c->dly != c->dly_s)
    return fail(c, GLMR_EINVAL, "dL/dtau needs the self-delay equal to the transmission delay");
  if (want_tau && !c->have_y) {
    c->keep_y = true;
    TRY(build_kernel_caches(c, true));
  }
  TRY(eval_core(c, want_grad, want_tau));
  if (ll_rows)
    HIPCHK(c, hipMemcpyAsync(ll_rows, c->ll_rows, c->N * sizeof(double), kind_to(where), c->st));
  if (grad_mu) HIPCHK(c, hipMemcpyAsync(grad_mu, c->gmu, c->N * sizeof(double), kind_to(where), c->st));
  if (grad_J)
    HIPCHK(c, hipMemcpy2DAsync(grad_J, c->N * sizeof(double), c->gJ, c->Np * sizeof(double),
                               c->N * sizeof(double), c->N, kind_to(where), c->st));
  HIPCHK(c, hipMemcpyAsync(c->host_scal, c->scal, 2 * sizeof(double), hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  if (ll) *ll = c->host_scal[0];
  if (grad_tau) *grad_tau = c->host_scal[1];
  if (!std::isfinite(c->host_scal[0])) return fail(c, GLMR_ENONFINITE, "log-likelihood is not finite");
  return GLMR_OK;
}

glmr_status glmr_prof_enable(glmr_ctx* c, int32_t on) {
  if (!c) return GLMR_EINVAL;
  c->prof = on != 0;
  return GLMR_OK;
}

void glmr_prof_reset(glmr_ctx* c) {
  if (!c) return;
  prof_collect(c);
  for (int k = 0; k < K_NKIND; ++k) {
    c->prof_ms[k] = 0;
    c->prof_n[k] = 0;
  }
}

int32_t glmr_prof_get(glmr_ctx* c, const char** names, double* total_ms, int64_t* launches, int32_t cap) {
  if (!c) return 0;
  prof_collect(c);
  int32_t n = 0;
  for (int k = 0; k < K_NKIND; ++k) {
    if (c->prof_n[k] == 0) continue;
    if (n < cap) {
      if (names) names[n] = kKindNames[k];
      if (total_ms) total_ms[n] = c->prof_ms[k];
      if (launches) launches[n] = c->prof_n[k];
    }
    ++n;
  }
  return n;
}

glmr_status glmr_query(const glmr_ctx* c, int64_t* n_pad, int64_t* b_pad, int64_t* chunk_bins,
                       int32_t* planes, int32_t* tile_n, int32_t* trace_resident) {
  if (!c) return GLMR_EINVAL;
  if (n_pad) *n_pad = c->Np;
  if (b_pad) *b_pad = c->Bp;
  if (chunk_bins) *chunk_bins = c->L;
  if (planes) *planes = c->planes;
  if (tile_n) *tile_n = c->tile;
  if (trace_resident) *trace_resident = c->resident ? (c->xfrag ? 2 : 1) : 0;
  return GLMR_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ autotuner


extern "C" glmr_status glmr_autotune(glmr_ctx* c, const char* cache_path, int32_t* shape_u,
                                     int32_t* shape_g) {
  if (!c) return GLMR_EINVAL;
  c->err.clear();
  TRY(check_ready(c));
  HIPCHK(c, hipSetDevice(c->cfg.device));
  if (!c->resident) {
    if (shape_u) *shape_u = -1;
    if (shape_g) *shape_g = -1;
    return GLMR_OK;  // the rebuild kernels have one shape per precision
  }
  const std::string key = tune_key(c);
  int n = 0;
  (void)res_shapes(&n);
  int best_u = -1, best_g = -1;
  if (cache_path) {
    if (FILE* f = std::fopen(cache_path, "r")) {
      char line[512];
      while (std::fgets(line, sizeof(line), f)) {
        char arch[128];
        long long np = 0, l = 0;
        int prec = -1, u = -1, g = -1;
        if (std::sscanf(line, "glmrec-tune %127s %lld %lld %d %d %d", arch, &np, &l, &prec, &u, &g) == 6) {
          char k2[256];
          std::snprintf(k2, sizeof(k2), "%s %lld %lld %d", arch, np, l, prec);
          if (key == k2 && shape_ok_u(c, u) && shape_ok(c, g)) {
            best_u = u;  // the last matching line wins
            best_g = g;
          }
        }
      }
      std::fclose(f);
    }
  }
  if (best_u < 0) {
    TRY(ensure_workspace(c, true, false));
    const int64_t Lc = std::min<int64_t>(c->L, c->Bp);
    double tu = 1e300, tg = 1e300;
    for (int k = 0; k < n; ++k) {
      double ms = 0;
      if (shape_tune_u(c, k)) {
        TRY(time_launches(c, [&] { return launch_u_chunk(c, k, 0, Lc); }, 3, &ms));
        if (ms < tu) { tu = ms; best_u = k; }
      }
      if (shape_ok(c, k)) {
        int ns = 0;
        TRY(time_launches(c, [&] { return launch_g_chunk(c, k, 0, Lc, &ns); }, 3, &ms));
        if (ms < tg) { tg = ms; best_g = k; }
      }
    }
    if (cache_path) {
      if (FILE* f = std::fopen(cache_path, "a")) {
        std::fprintf(f, "glmrec-tune %s %d %d %.4f %.4f\n", key.c_str(), best_u, best_g, tu, tg);
        std::fclose(f);
      }
    }
  }
  c->res_shape_u = best_u;
  c->res_shape_g = best_g;
  if (shape_u) *shape_u = best_u;
  if (shape_g) *shape_g = best_g;
  return GLMR_OK;
}
