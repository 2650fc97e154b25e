// Internal definitions shared by the glmrec HIP sources (gfx950 only).
//
// Device data layout (all padded, all owned by the context):
//   Np  = N rounded up to the neuron tile (128 or 256)
//   Bp  = B rounded up to 256 bins;  NS = Bp / 64 subtiles of 64 bins
//   masks[p][s][j]  uint64: bit b set if neuron j has more than p spikes in bin
//                   64*s + b (p = 0..planes-1; planes = max spikes per bin)
//   seg_off[s*NIB + ib], seg_ent[]: spikes of subtile s whose neuron lies in the
//                   64-neuron block ib (NIB = Np/64); entry = i_local | (b << 6),
//                   sorted, so a segment lists its spikes in bin order
//   C[s][j]         trace x_j at bin 64*s (the carry into subtile s)
//   CY[s][j]        d x_j / d tau at bin 64*s
//   dsig[i][j]      sum_t s_i[t] x_j[t]     (Eq. (12), parameter-free)
//   dsigY[i][j]     sum_t s_i[t] y_j[t]     (y = dx/dtau)
//   W[i][t]         exp(sum_j J_ij x_j[t]) for the bins of one time chunk
//   rowpart[tt][i]  per 256-bin tile partial sums of W (FP64)
//   Gp[k][i][j]     per split partial of sum_t W[i][t] x_j[t]
// Inside a subtile the trace is evaluated in closed form:
//   x_j[64 s + m] = a^m * (C[s][j] + sum_{b < m, spike of j in bin 64 s + b} a^-(b+1))
// On the event grid of the continuous-time likelihood the bins are the slots
// between network events and a^m, a^-(b+1), a^64 become the per-slot tables
// of EvSlots (events.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <stdint.h>

#define GLMR_SUB 64   // bins per subtile (mask word)
#define GLMR_TT 256   // bins per time tile of the likelihood kernel

// Element (i, t) of a chunk's weights W (neuron i < Np, chunk-local bin t < L):
//   layout 0  row-major [Np][L];
//   layout 1  tile-major [L / 256][Np][256] (a 256-bin tile of all rows is one block);
//   layout 2  MFMA fragments: the 32 x 16 block of neurons 32 ib .. and bins
//             16 kb .. is the 1 KB starting at byte 1024 (ib (L / 16) + kb), in
//             lane order (lane l holds neuron 32 ib + l % 32, bins 16 kb + 8 (l / 32) .. + 8).
// The resident trace's Xtj uses layout 2 of [Bp][Np] in the same way (rows t,
// columns j) when it is stored as fragments.
__host__ __device__ inline int64_t w_elem(int layout, int64_t i, int64_t t, int64_t Np, int64_t L) {
  if (layout == 1) return ((t >> 8) * Np + i) * 256 + (t & 255);
  if (layout == 2) return ((((i >> 5) * (L >> 4) + (t >> 4)) * 64 + (i & 31) + 32 * ((t >> 3) & 1)) << 3) + (t & 7);
  return i * L + t;
}
#define GLMR_IB 64    // neurons per spike-segment block

typedef __attribute__((ext_vector_type(2))) double f64x2;
typedef __attribute__((ext_vector_type(4))) double f64x4;
typedef __attribute__((ext_vector_type(4))) float f32x4;
typedef __attribute__((ext_vector_type(16))) float f32x16;
typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(8))) int i32x8;
typedef __attribute__((ext_vector_type(4))) int i32x4;

struct Tables {
  double pw[64];     // a^m
  double ainv[64];   // a^-(b+1)
  double apow[65];   // a^(64 k), k = 0..64
  float pw32[64];
  float ainv32[64];
};

// Per-slot tables of the event grid for the current tau (null pointers on the
// regular grid).  k is a slot, k0 the first slot of its subtile.
struct EvSlots {
  const double* pw;        // [NS*64] e^{-(t_k - t_k0)/tau}
  const double* ainv;      // [NS*64] e^{(t_{k+1} - t_k0)/tau}
  const double* left;      // [NS*64] e^{-(t_{k+1} - t_k0)/tau}
  const double* delta;     // [NS*64] (t_{k+1} - t_k)/tau
  const double* edec;      // [NS*64] e^{-(t_{k+1} - t_k)/tau}  (decay over slot k)
  const double* asub;      // [NS]    e^{-(t_{k0+64} - t_k0)/tau}
};

// ------------------------------------------------------------- launchers
// Every launcher enqueues on `st` and returns hipSuccess or the launch error.
struct IngestBufs {
  int64_t n;
  const int64_t* bin;
  const int32_t* neu;
  int32_t N;
  int64_t B, NS, NIB;
  unsigned long long* bad;    // [2]: count, first bad index (min)
  int32_t* cnt;               // [NS*NIB + 1]
  int32_t* off;               // [NS*NIB + 1]
  int32_t* cursor;            // [NS*NIB]
  uint16_t* ent;              // [n]
  int64_t* q;                 // [Np]
  int32_t* maxmult;           // [1]
  int64_t* scan_tmp;          // [>= nseg/1024 + 2]
};
hipError_t launch_ingest_count(const IngestBufs& b, hipStream_t st);
hipError_t launch_ingest_scan(const IngestBufs& b, hipStream_t st);
hipError_t launch_ingest_scatter(const IngestBufs& b, hipStream_t st);
hipError_t launch_ingest_sort(const IngestBufs& b, hipStream_t st);
hipError_t launch_ingest_masks(const IngestBufs& b, uint64_t* masks, int planes, int64_t Np,
                               hipStream_t st);
hipError_t launch_digest_u64(const uint64_t* p, int64_t n_outer, int64_t inner, int64_t ld, int64_t cols,
                             unsigned long long* out, hipStream_t st);

// Event grid layout (events.hip) ---------------------------------------------
struct EvLayoutArgs {
  int64_t n;                  // events
  const double* times;        // [n] sorted by (time, neuron)
  const int32_t* neu;         // [n]
  int32_t N;
  double T0, T1, max_gap;
  int64_t NS;                 // subtiles of the slot grid
  unsigned long long* bad;    // [2]: count, first bad index
  int64_t* cnt;               // [n] slots taken by event k (with the spike-free ones before it)
  int64_t* slot;              // [n] slot of event k
  int64_t* scan_tmp;          // [ev_scan_tmp_len(n)]
  int64_t* bins;              // [n] pseudo-bin of event k (slot - 1)
  double* tslot;              // [NS*64 + 1] slot start times
};
int64_t ev_scan_tmp_len(int64_t n);
hipError_t launch_ev_check(const EvLayoutArgs& a, hipStream_t st);
hipError_t launch_ev_layout(const EvLayoutArgs& a, hipStream_t st);
hipError_t launch_ev_place(const EvLayoutArgs& a, int64_t s_last, double t_last, int64_t n_tail,
                           hipStream_t st);
double ev_resolve_max_gap(int64_t n, double T0, double T1, double max_gap);
int64_t ev_host_slots_of_gap(double gap, double max_gap);
struct EvTableArgs {
  const double* tslot;
  double tau;
  int64_t NS;
  double *pw, *ainv, *left, *delta, *edec, *asub;
  float* gl;                    // [NS*64][16]: the FP32 evaluation's per-slot table (null: none)
  unsigned long long* maxspan;  // max over subtiles of the span / tau (double bits), zero on entry
};
hipError_t launch_ev_tables(const EvTableArgs& a, hipStream_t st);

struct CarryArgs {
  const uint64_t* masks;
  int planes;
  int64_t NS, Np;
  double a, ctau;          // a = exp(-dt/tau), ctau = dt / tau^2
  const Tables* tab;       // device copy
  int want_y;
  double* C64;             // [NS][Np]
  double* CY64;            // [NS][Np] (want_y)
  float* C32;              // optional fp32 copy
  float* CY32;             // optional
  double* seg;             // [nseg][Np][2] scratch
  double* segin;           // [nseg][Np][2] scratch
  int64_t G;               // subtiles per segment (64)
  EvSlots ev;              // event grid (ev.pw != null): per-slot decays, no y
};
hipError_t launch_carries(const CarryArgs& c, hipStream_t st);

struct SpikeTermArgs {
  const uint64_t* masks;
  int planes;
  const int32_t* seg_off;
  const uint16_t* seg_ent;
  const double* C64;
  const double* CY64;      // nullable: then dsigY not computed
  const Tables* tab;
  double ctau;
  int64_t NS, Np, NIB;
  int splits;              // time splits
  double* part;            // [splits][Np][Np] (and a second block for Y)
  double* dsig;            // [Np][Np]
  double* dsigY;           // [Np][Np] or null
  EvSlots ev;              // event grid: left limits at the events
};
hipError_t launch_spike_term(const SpikeTermArgs& a, hipStream_t st);

// Transmission delays (delays.hip) ---------------------------------------------
struct DelayTrace {          // the recorded (unshifted) raster's trace, FP64
  const uint64_t* masks;     // [planes][NS][Np]
  int planes;
  const double* C;           // [NS][Np] carries
  const Tables* tab;
  int64_t NS, Np;
};
hipError_t launch_shift_masks(const uint64_t* src, uint64_t* dst, int planes, int64_t NS, int64_t Np,
                              int64_t d, hipStream_t st);
struct SelfDelayArgs {
  DelayTrace x;
  void* W;                   // [Np][L] weights of the chunk (kernel U's output)
  int wtype;                 // 0 double, 1 float, 2 bf16
  int scaled;                // 1: W holds lambda a^m (rebuilt-trace kernels), 0: lambda
  int tiled;                 // W's layout (w_elem): 0 [Np][L], 1 tile-major, 2 fragments (resident trace)
  const double* Jr;          // [Np][Np] J as the contraction used it
  int64_t B, t0, L, Lc;      // bins, chunk start, W pitch, bins of the chunk
  int tb;                    // bins per row-sum tile of kernel U (128 or 256)
  int64_t d, ds;             // delays in bins
  double* rowpart;           // [Bp/tb][Np] rewritten
  double* gpart;             // [Bp/tb][Np] sum lambda Delta
};
hipError_t launch_self_delay(const SelfDelayArgs& a, hipStream_t st);
struct SelfSpikeArgs {
  DelayTrace x;
  const int32_t* seg_off;
  const uint16_t* seg_ent;
  int64_t NIB;
  int splits;
  int64_t d, ds;
  double* part;              // [splits][Np]
  double* dsig;              // [Np][Np]: the diagonal is incremented
};
hipError_t launch_self_spike(const SelfSpikeArgs& a, hipStream_t st);

// Likelihood kernels -------------------------------------------------------
enum { PREC_F64 = 0, PREC_F32 = 1, PREC_BF16 = 2, PREC_FP8 = 3 };

struct Gemm1Args {
  const void* Jc;          // [Np][Np] compute precision
  const uint64_t* masks;
  int planes;
  const void* C;           // [NS][Np] double (F64/F32) or float (BF16/FP8)
  const void* CY;          // tau mode: carries of y
  const Tables* tab;
  double ctau;
  int64_t Np, NS, B;
  int64_t t0;              // first bin of this chunk (multiple of 256)
  int64_t L;               // bins in this chunk (multiple of 256)
  int n_itiles, n_ttiles;
  void* W;                 // [Np][L]  (mode 0 writes, mode 1 reads)
  double* rowpart;         // [Bp/256][Np]  (mode 0: sum_t W; mode 1: sum_t W V)
  const float* xscale;     // FP8: per-chunk X scale (power of two); J row scale
  const float* jscale;
  int mode;                // 0: U -> W, 1: V = Y J^T -> sum W V
  int w_plain;             // mode 1: W holds exp(V) in the resident trace's layout (w_elem's
                           // layout 1 or 2) instead of exp(V) a^m ([Np][L]); 0 for the latter
  EvSlots ev;              // event grid (mode 0 only): W = H(D, delta) pw, row sums of F(D, delta)
  const float* evgl;       // event grid, BF16: [slots][16] per-slot table of the FP32 integrals
};
hipError_t launch_gemm1(int prec, int tile, const Gemm1Args& a, hipStream_t st);

struct Gemm2Args {
  const void* W;           // [Np][L]
  const uint64_t* masks;
  int planes;
  const void* C;
  const Tables* tab;
  int64_t Np, NS;
  int64_t t0, L;           // chunk start, row pitch of W
  int64_t Lc;              // bins of this chunk (<= L)
  int64_t ks;              // bins per split
  int n_splits, n_itiles, n_jtiles;
  void* Gp;                // [n_splits][Np][Np] float (double for F64)
  const float* xscale;
  const float* wscale;
  EvSlots ev;              // event grid
};
hipError_t launch_gemm2(int prec, int tile, const Gemm2Args& a, hipStream_t st);

// Resident trace (BF16): x built once per tau in two layouts -----------------
struct ResXArgs {
  const double* C64;       // [NS][Np]
  const uint64_t* masks;
  int planes;
  const Tables* tab;
  int64_t Np, NS, Bp;
  void* Xtj;               // [Bp][Np] bf16 (FP8: e4m3 bytes); MFMA fragments when xfrag
  void* Xjt;               // [Np][Bp] bf16 (FP8: e4m3 bytes)
  int xfrag;               // BF16: Xtj stored as 32 x 16 fragments (w_elem's layout 2 of [Bp][Np])
  int64_t L;               // FP8: bins per scaling chunk (the evaluation's time chunk)
  unsigned* xmax;          // FP8: [ceil(Bp / L)] chunk maxima (float bits), zero on entry
  float* xscale;           // FP8: [ceil(Bp / L)] power-of-two chunk scales
  EvSlots ev;              // event grid: per-slot decays (null on the regular grid)
};
hipError_t launch_build_x(const ResXArgs& a, hipStream_t st);
hipError_t launch_build_x8(const ResXArgs& a, hipStream_t st);

struct ResUArgs {
  const void* Jc;          // [Np][Np] bf16 ([Np][2 Np]: J_hi | J_lo when j2)
  int j2;                  // J as two BF16 terms: k runs over 2 Np, the trace repeated
  const void* Xtj;         // [Bp][Np] bf16
  int64_t Np, B;
  int64_t t0;              // first bin of this chunk
  int64_t L;               // row pitch of W (bins)
  int n_itiles, n_ttiles;  // neuron tiles, 256-bin tiles of this chunk
  void* W;                 // [Np][L] bf16: exp(V) (FP8: e5m2 bytes, exp(V) / 64)
  double* rowpart;         // [Bp/256][Np]
  const float* xscale;     // FP8: this chunk's trace scale (one value)
  const float* jscale;     // FP8: [Np] row scales of J
  const float* evgl;       // event grid: [Bp][16] per-slot table of the FP32 integrals (null on the grid)
  const double* evdelta;   // event grid: [Bp] interval lengths / tau
};
struct ResGArgs {
  const void* W;           // [Np][L] bf16
  const void* Xjt;         // [Np][Bp] bf16
  int64_t Np, Bp;
  int64_t t0, L, Lc;       // chunk start, W pitch, bins of this chunk
  int64_t ks;              // bins per split (multiple of 64)
  int n_splits, n_itiles, n_jtiles;
  void* Gp;                // [n_splits][Np][Np] float
  const float* xscale;     // FP8: this chunk's trace scale (one value)
};
struct ResShape {
  int ui;                  // kernel U: neurons per tile (x 256 bins)
  int gi, gj;              // kernel G: tile rows (i) x columns (j)
  int wgm, wgn;            // wave grid of the row-major kernels
  int fp8_ok;              // usable for FP8 operands
  int frag;                // the fragment-major kernels (trace and W as MFMA fragments, 4 waves)
  int u_own;               // kernel U differs from that of every earlier shape with the same frag
};
const ResShape* res_shapes(int* n);
// Work queue of a grouped (many-recording) launch: args[r] describes recording
// r's chunk; its tiles are k in [prefix[r], prefix[r + 1]) of [0, total).
// The fragment-major kernels take one workgroup per tile and split every
// recording's tiles evenly over the 8 XCDs (workgroup b runs on XCD b % 8):
// xprefix[x][r] (row x of 8, n + 1 entries) counts the tiles XCD x takes
// from recordings before r, and xgrid workgroups cover the largest share.
struct ResUGroup {
  const ResUArgs* args;    // device [n]
  const int64_t* prefix;   // device [n + 1]
  int n;
  int64_t total;
  const int64_t* xprefix;  // device [8][n + 1]
  int64_t xgrid;
};
struct ResGGroup {
  const ResGArgs* args;
  const int64_t* prefix;
  int n;
  int64_t total;
  const int64_t* xprefix;
  int64_t xgrid;
};
hipError_t launch_res_u_group(int shape, int fp8, const ResUGroup& q, hipStream_t st);
hipError_t launch_res_g_group(int shape, int fp8, const ResGGroup& q, hipStream_t st);
hipError_t launch_res_u(int shape, int fp8, const ResUArgs& a, hipStream_t st);
hipError_t launch_res_g(int shape, int fp8, const ResGArgs& a, hipStream_t st);

// Reductions and assembly (FP64) -------------------------------------------
hipError_t launch_gp_reduce(int prec, const void* Gp, int n_splits, int64_t Np, double* G64,
                            int first, hipStream_t st);
hipError_t launch_rowpart_reduce(const double* rowpart, int64_t n_tiles, int64_t Np, double* out,
                                 double* tmp, hipStream_t st);
struct AssembleArgs {
  int N;
  int64_t Np;
  double dt;
  const int64_t* q;
  const double* mu;       // [Np]
  const double* Jr;       // [Np][Np] parameters as used (rounded to the compute precision)
  const double* dsig;
  const double* dsigY;    // nullable
  const double* rowsum;   // sum_t W  [Np]
  const double* rowsumV;  // nullable
  const double* G64;      // nullable (no gradient)
  const double* gself;    // nullable: per-row correction of G_ii (self-delay)
  const double* rowscale; // [Np] multiplier of rowsum/G (e^mu, FP8 scales folded in)
  double* ll_rows;        // [Np]
  double* gJ;             // [Np][Np] or null
  double* gmu;            // [Np] or null
  double* tau_rows;       // [Np] or null
};
hipError_t launch_assemble(const AssembleArgs& a, hipStream_t st);
hipError_t launch_sum_rows(const double* v, int n, double* out, hipStream_t st);

// Parameter preparation
hipError_t launch_prepare_params(int prec, int j2, int N, int64_t Np, const double* J64, const double* mu,
                                 void* Jc, double* Jr, double* rowscale, float* jscale,
                                 hipStream_t st);
hipError_t launch_copy_out(const double* src, int64_t src_ld, double* dst, int rows, int cols,
                           hipStream_t st);
hipError_t launch_fp8_xscale(const void* C32, int64_t NS, int64_t Np, int64_t chunk_sub,
                             int64_t nchunks, const uint64_t* masks, int planes,
                             const Tables* tab, float* xscale, hipStream_t st);
hipError_t launch_fp8_wscale(const float* rowmax, int64_t Np, float* wscale, hipStream_t st);

// Ascent (per-row L-BFGS, FP64) --------------------------------------------
struct AscentArgs {
  int N;
  int64_t Np;
  int P;                  // parameters per row = N + 1 (mu first)
  int m;                  // history
  double* theta;          // [Np][P] current
  double* theta_try;      // [Np][P] trial
  double* g;              // [Np][P] gradient of f = -L at theta
  double* g_try;          // [Np][P]
  double* d;              // [Np][P] direction
  double* S;              // [m][Np][P]
  double* Y;              // [m][Np][P]
  double* rho;            // [m][Np]
  int32_t* hist_len;      // [Np]
  int32_t* hist_head;     // [Np]
  double* f;              // [Np] f_i = -L_i at theta
  double* f_try;          // [Np]
  double* step;           // [Np] alpha_i
  double* gd;             // [Np] g_i . d_i
  int32_t* state;         // [Np]: 0 active, 1 converged, 2 stalled
  int32_t* accepted;      // [Np]
  double* eta;            // [Np]
  int32_t* bt;            // [Np] halvings of the current line search
  double* gstep;          // [Np] g_i . (theta_try_i - theta_i) of the current trial
  // smooth epsilon-l1 penalty (alpha = 0: none) and bounds (jmax = 0: none on J)
  double alpha, eps, jmax, mu_lo, mu_hi;
};
hipError_t launch_lbfgs_direction(const AscentArgs& a, int async, hipStream_t st);
hipError_t launch_penalty(const AscentArgs& a, const double* theta, double* g, double* f, hipStream_t st);
hipError_t launch_project_theta(const AscentArgs& a, double* theta, hipStream_t st);
hipError_t launch_armijo_async(const AscentArgs& a, double c1, int max_bt, hipStream_t st);
hipError_t launch_fill_i32(int32_t* p, int n, int32_t v, hipStream_t st);
hipError_t launch_count_active(const AscentArgs& a, int32_t* counters, hipStream_t st);
hipError_t launch_sum_counters(int32_t* const* p, int n, int32_t* out, hipStream_t st);
hipError_t launch_make_trial(const AscentArgs& a, hipStream_t st);
hipError_t launch_accept_update(const AscentArgs& a, double ftol, int32_t* counters, int async,
                                hipStream_t st);
hipError_t launch_pack_theta(int N, int64_t Np, int P, const double* theta, double* J64,
                             double* mu, hipStream_t st);
hipError_t launch_pack_grad(int N, int64_t Np, int P, const double* gJ, const double* gmu,
                            const double* ll_rows, double* g, double* f, hipStream_t st);
hipError_t launch_unpack_theta(int N, int64_t Np, int P, const double* J64, const double* mu,
                               double* theta, hipStream_t st);
