// The two dense contractions of the likelihood on MFMA (gfx950).
//
//   kernel U (k_gemm1, mode 0):  V[i][t] = sum_j J[i][j] x_j[t] for a tile of
//       postsynaptic neurons i and a 256-bin tile of t; epilogue
//       W[i][t] = exp(V[i][t]) (0 for padded bins) and per-row sums of W.
//       With lambda_i[t] = e^{mu_i} W[i][t], the integral term of Eq. (7) is
//       dt e^{mu_i} sum_t W[i][t].
//   kernel V (k_gemm1, mode 1):  the same contraction with the tau-derivative
//       trace y_j[t] in place of x_j[t]; epilogue sums W[i][t] V[i][t] per row
//       (the lambda part of dL/dtau).
//   kernel G (k_gemm2):  Gp[i][j] = sum_{t in split} W[i][t] x_j[t], the
//       integral of Eq. (12) up to the factor dt e^{mu_i}, one partial per
//       time split (no atomics; reduced in a fixed order in FP64).  FP64
//       accumulation in the FP64 and FP32 modes (FP32 operands widened).
//
// The trace x never exists in HBM: each workgroup rebuilds the tile it needs
// in LDS from the spike bitmasks and the per-subtile carries, in scaled form
//   x_j[64 s + m] = a^m z_j[64 s + m],
//   z_j[64 s + m] = C[s][j] + sum_{b < m, bit b of mask(s, j)} a^-(b+1),
// one wavefront per 64-bin subtile (lane = bin m).  z is constant down the
// subtile for a column without spikes, so rebuilding it costs one rounding per
// element; the carry and mask of a column are wave-uniform scalar loads.  The
// factor a^m is applied in kernel U's epilogue (V = a^m sum_j J z) and folded
// into the weights it stores (W' = exp(V) a^m), so kernel G contracts W' with
// z: sum_t W' z = sum_t exp(V) x.
//
// Both contractions are C[m][n] = sum_k A[m][k] B[n][k] with A and B staged in
// LDS with k contiguous (rows padded by 16 bytes).  The MFMA shapes:
//   FP64 v_mfma_f64_16x16x4f64, FP32 v_mfma_f32_32x32x2f32,
//   BF16 v_mfma_f32_32x32x16_bf16.
// Each lane reads 16 contiguous bytes of k per operand and block; the k order
// inside a 16-byte group is the same for A and B, so any permutation the
// instruction applies inside the group cancels.
//
// Rounding of the rebuilt trace.  Trace values recur (a^m after every isolated
// spike), so round-to-nearest would give the same error at every occurrence and
// bias the sums; in FP32 and BF16 modes x is rounded stochastically with
// random bits r(t, j) = t*0x9E3779B9 + j*0x6C8E9CF5 (mod 2^32), a function of
// the bin and the column only, so both contractions see the identical rounded
// trace.  Rounded values are unbiased and their errors average out over t.
//
// Event grid (continuous time, FP64, FP32 and BF16 modes): the bins are the slots
// between network events, a^m and a^-(b+1) come from the per-slot tables
// (pw, ainv relative to the subtile's first slot), and kernel U's epilogue
// takes the closed forms of the interval integrals instead of exp: with
// D = pw acc the potential offset at the slot start,
//   row sums of F(D, delta) = Ei(D) - Ei(D xi)    (Eq. (10)),
//   W' = H(D, delta) pw,  H = (e^D - e^{D xi}) / D (Eq. (14)),
// so kernel G contracts W' with z into sum_k H x_j, the trace integral of
// Eq. (12) up to the factor tau e^{mu_i}.
//
// Pipelining: the J (or W) tile of the next step is fetched into registers
// and the trace tile of the next step is rebuilt into the second LDS buffer
// while the MFMAs of the current step run; one barrier per step.
#include <type_traits>

#include "common.h"
#include "evfun.h"

namespace {

template <int PREC> struct Pol;

template <> struct Pol<PREC_F64> {
  using in_t = double;
  using c_t = double;
  using w_t = double;
  using gp_t = double;
  using acc_t = f64x4;
  using frag_t = f64x2;
  static constexpr int MB = 16, EPL = 2, NACC = 4;
  __device__ static inline void mma(acc_t& c, frag_t a, frag_t b) {
    c = __builtin_amdgcn_mfma_f64_16x16x4f64(a[0], b[0], c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f64_16x16x4f64(a[1], b[1], c, 0, 0, 0);
  }
  // D layout of the 16x16x4 f64 MFMA: lane l, register r -> row l/16 + 4 r, col l%16
  __device__ static inline int row(int r, int lane) { return (lane >> 4) + 4 * r; }
  __device__ static inline int col(int lane) { return lane & 15; }
  __device__ static inline double lam(double v) { return exp(v); }
  __device__ static inline in_t cvt(double x, uint32_t) { return x; }
};

template <> struct Pol<PREC_F32> {
  using in_t = float;
  using c_t = double;  // the trace is evaluated in FP64 and rounded once
  using w_t = float;
  using gp_t = float;
  using acc_t = f32x16;
  using frag_t = f32x4;
  static constexpr int MB = 32, EPL = 4, NACC = 16;
  __device__ static inline void mma(acc_t& c, frag_t a, frag_t b) {
    c = __builtin_amdgcn_mfma_f32_32x32x2f32(a[0], b[0], c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_32x32x2f32(a[1], b[1], c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_32x32x2f32(a[2], b[2], c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_32x32x2f32(a[3], b[3], c, 0, 0, 0);
  }
  __device__ static inline int row(int r, int lane) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }
  __device__ static inline int col(int lane) { return lane & 31; }
  // exp in FP64: a biased FP32 exp would bias the integral term
  __device__ static inline double lam(float v) { return exp((double)v); }
  // stochastic rounding FP64 -> FP32 of x >= 0: add 29 random bits below the
  // FP32 mantissa, truncate
  __device__ static inline in_t cvt(double x, uint32_t r) {
    uint64_t b = (uint64_t)__double_as_longlong(x) + (uint64_t)(r >> 3);
    b &= ~((1ull << 29) - 1);
    return (float)__longlong_as_double((long long)b);
  }
};

// FP32 mode, kernel U/V: FP32 operands (J and the trace rounded to FP32)
// accumulated on the FP64 MFMA.  An FP32 accumulator absorbs the many tiny
// products of decayed traces into large partial sums, a deterministic loss
// that does not average out (2e-8 relative in L at N = 1000, measured); FP64
// accumulation keeps the likelihood within its 1e-10 target.
constexpr int PREC_F32U = 16;
template <> struct Pol<PREC_F32U> {
  using in_t = double;
  using c_t = double;
  using w_t = float;
  using gp_t = float;
  using acc_t = f64x4;
  using frag_t = f64x2;
  static constexpr int MB = 16, EPL = 2, NACC = 4;
  __device__ static inline void mma(acc_t& c, frag_t a, frag_t b) { Pol<PREC_F64>::mma(c, a, b); }
  __device__ static inline int row(int r, int lane) { return Pol<PREC_F64>::row(r, lane); }
  __device__ static inline int col(int lane) { return Pol<PREC_F64>::col(lane); }
  __device__ static inline double lam(double v) { return exp(v); }
  __device__ static inline in_t cvt(double x, uint32_t r) { return (double)Pol<PREC_F32>::cvt(x, r); }
};

// FP32 mode, kernel G: the same FP32-rounded operands (W as kernel U stored
// it, the trace rounded with the same stochastic bits) widened to FP64 in LDS
// and accumulated on the FP64 MFMA, with FP64 partials per split.  FP32
// accumulation over a split of tens of thousands of bins leaves a random-walk
// error of ~1e-5 of the lambda term, which near the maximum of L is a large
// part of the small gradient.
constexpr int PREC_F32G = 17;
template <> struct Pol<PREC_F32G> {
  using in_t = double;
  using c_t = double;
  using w_t = float;
  using gp_t = double;
  using acc_t = f64x4;
  using frag_t = f64x2;
  static constexpr int MB = 16, EPL = 2, NACC = 4;
  __device__ static inline void mma(acc_t& c, frag_t a, frag_t b) { Pol<PREC_F64>::mma(c, a, b); }
  __device__ static inline int row(int r, int lane) { return Pol<PREC_F64>::row(r, lane); }
  __device__ static inline int col(int lane) { return Pol<PREC_F64>::col(lane); }
  __device__ static inline in_t cvt(double x, uint32_t r) { return (double)Pol<PREC_F32>::cvt(x, r); }
};

template <> struct Pol<PREC_BF16> {
  using in_t = __bf16;
  using c_t = float;
  using w_t = __bf16;
  using gp_t = float;
  using acc_t = f32x16;
  using frag_t = bf16x8;
  static constexpr int MB = 32, EPL = 8, NACC = 16;
  __device__ static inline void mma(acc_t& c, frag_t a, frag_t b) {
    c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int r, int lane) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }
  __device__ static inline int col(int lane) { return lane & 31; }
  __device__ static inline float lam(float v) { return __expf(v); }
  // stochastic rounding FP32 -> BF16 (v_cvt_sr_bf16_f32)
  __device__ static inline in_t cvt(float x, uint32_t r) {
    typedef __attribute__((ext_vector_type(2))) __bf16 bf16x2;
    bf16x2 v = {};
    v = __builtin_amdgcn_cvt_sr_bf16_f32(v, x, r, false);
    return v[0];
  }
};

template <typename T> __device__ inline T tab_pw(const Tables* t, int m);
template <> __device__ inline double tab_pw<double>(const Tables* t, int m) { return t->pw[m]; }
template <> __device__ inline float tab_pw<float>(const Tables* t, int m) { return t->pw32[m]; }
template <typename T> __device__ inline T tab_ainv(const Tables* t, int b);
template <> __device__ inline double tab_ainv<double>(const Tables* t, int b) { return t->ainv[b]; }
template <> __device__ inline float tab_ainv<float>(const Tables* t, int b) { return t->ainv32[b]; }

__device__ inline int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// the per-slot factor pw as the trace arithmetic of the mode holds it
template <typename T> __device__ inline T pw_of(double pw) { return (T)pw; }

constexpr uint32_t SR_T = 0x9E3779B9u, SR_J = 0x6C8E9CF5u;

// XCD-aware block order: the hardware deals consecutive workgroups round-robin
// over the 8 XCDs; renumber so that each XCD receives a contiguous range of
// logical tiles (tiles that share an operand land on the same L2).
__device__ inline int64_t xcd_logical(int64_t bid, int64_t nblk) {
  const int64_t nx = 8;
  int64_t x = bid % nx, idx = bid / nx;
  int64_t q = nblk / nx, r = nblk % nx;
  return x * q + (x < r ? x : r) + idx;
}

// Scaled trace at lane bin m of a subtile for one column:
//   z = x / a^m = c + sum_{b < m, bit b of the masks} a^-(b+1)
// c (the carry) and mk (plane-0 mask) are wave-uniform; further planes
// (several spikes in one bin) are read here.
// On the event grid (EV) a^-(b+1) is the per-slot table eva[b] of subtile s.
template <typename T, bool EV>
__device__ inline T z_from(T c, uint64_t mk, int m, const Tables* tab, const double* __restrict__ eva,
                           const uint64_t* __restrict__ masks, int planes, int64_t NS,
                           int64_t Np, int64_t s, int64_t j) {
  T run = c;
  while (mk) {
    const int b = __builtin_ctzll(mk);
    mk &= mk - 1;
    if (b < m) run += EV ? (T)eva[b] : tab_ainv<T>(tab, b);
  }
  for (int p = 1; p < planes; ++p) {
    uint64_t mp = masks[((int64_t)p * NS + s) * Np + j];
    while (mp) {
      const int b = __builtin_ctzll(mp);
      mp &= mp - 1;
      if (b < m) run += EV ? (T)eva[b] : tab_ainv<T>(tab, b);
    }
  }
  return run;
}

// Scaled tau-derivative of the trace: y / a^m = CY + m c C + c sum_{b<m} (m-b-1) a^-(b+1)
template <typename T, typename CT>
__device__ inline T zy_at(const CT* __restrict__ C, const CT* __restrict__ CY,
                          const uint64_t* __restrict__ masks, int planes, int64_t NS, int64_t Np,
                          int64_t s, int64_t j, int m, T ctau, const Tables* tab) {
  T acc = (T)CY[s * Np + j] + (T)m * ctau * (T)C[s * Np + j];
  T inner = 0;
  for (int p = 0; p < planes; ++p) {
    uint64_t mk = masks[((int64_t)p * NS + s) * Np + j];
    while (mk) {
      const int b = __builtin_ctzll(mk);
      mk &= mk - 1;
      if (b < m) inner += (T)(m - b - 1) * tab_ainv<T>(tab, b);
    }
  }
  return acc + ctau * inner;
}

constexpr int PAD = 16;  // bytes of padding per LDS row

// ---------------------------------------------------------------- kernel U/V
// KB: bytes of k (presynaptic j) per step and LDS row
template <int PREC, int BI, int BT, int WGM, int WGN, int DB, bool EV, int KB = 128>
__global__ __launch_bounds__(WGM * WGN * 64) void k_gemm1(Gemm1Args g) {
  using P = Pol<PREC>;
  using in_t = typename P::in_t;
  using c_t = typename P::c_t;
  using w_t = typename P::w_t;
  using frag_t = typename P::frag_t;
  using acc_t = typename P::acc_t;
  using T = c_t;  // arithmetic type of the trace
  constexpr int NW = WGM * WGN;
  constexpr int NT = NW * 64;
  constexpr int BK = KB / sizeof(in_t);           // k (presynaptic j) per step
  constexpr int ROWB = BK * sizeof(in_t) + PAD;   // LDS row pitch, bytes
  constexpr int WM = BI / WGM, WN = BT / WGN;
  constexpr int WMB = WM / P::MB, WNB = WN / P::MB;
  constexpr int GROUPS = BK / P::EPL;             // 16-byte column groups per row
  constexpr int SUBS = BT / 64;
  constexpr int KC = P::EPL * (64 / P::MB);       // k per MFMA chunk
  constexpr int ABUF = BI * ROWB, BBUF = BT * ROWB;

  extern __shared__ __align__(16) unsigned char smem[];
  unsigned char* As0 = smem;                      // [DB][BI][ROWB]  J tile
  unsigned char* Bs0 = smem + DB * ABUF;          // [DB][BT][ROWB]  z tile (row = bin)
  double* red = (double*)(smem + DB * (ABUF + BBUF));  // [WGN][BI]

  const int tid = threadIdx.x, lane = tid & 63, wave = uniform(tid >> 6);
  const int wm = wave / WGN, wn = wave % WGN;
  const int64_t logical = xcd_logical(blockIdx.x, gridDim.x);
  const int itile = (int)(logical % g.n_itiles);
  const int ttile = (int)(logical / g.n_itiles);
  const int64_t i0 = (int64_t)itile * BI;
  const int64_t tl0 = (int64_t)ttile * BT;        // first bin, chunk-local
  const int64_t tt0 = g.t0 + tl0;                 // first bin, global
  const int64_t s0 = tt0 / 64;
  const in_t* __restrict__ Jc = (const in_t*)g.Jc;
  const c_t* __restrict__ C = (const c_t*)g.C;
  const c_t* __restrict__ CY = (const c_t*)g.CY;
  const T ctau = (T)g.ctau;

  acc_t acc[WMB][WNB];
#pragma unroll
  for (int a = 0; a < WMB; ++a)
#pragma unroll
    for (int b = 0; b < WNB; ++b)
#pragma unroll
      for (int r = 0; r < P::NACC; ++r) acc[a][b][r] = 0;

  constexpr int RP = BK * (int)sizeof(in_t) / 16;
  constexpr int APIECES = BI * RP;
  constexpr int APT = (APIECES + NT - 1) / NT;
  i32x4 areg[APT];
  auto load_a = [&](int64_t k0) {
#pragma unroll
    for (int q = 0; q < APT; ++q) {
      int piece = tid + q * NT;
      if (piece < APIECES) {
        int r = piece / RP, c16 = piece % RP;
        areg[q] = *(const i32x4*)((const unsigned char*)(Jc + (i0 + r) * g.Np + k0) + c16 * 16);
      }
    }
  };
  auto store_a = [&](unsigned char* As) {
#pragma unroll
    for (int q = 0; q < APT; ++q) {
      int piece = tid + q * NT;
      if (piece < APIECES) {
        int r = piece / RP, c16 = piece % RP;
        *(i32x4*)(As + r * ROWB + c16 * 16) = areg[q];
      }
    }
  };
  // rebuild the scaled trace tile z for columns [k0, k0 + BK): each wave owns
  // one subtile (lane = bin) and a share of its 16-byte column groups
  auto build_z = [&](int64_t k0, unsigned char* Bs) {
    constexpr int WPS = NW >= SUBS ? NW / SUBS : 1;  // waves per subtile
    for (int sub = wave / WPS; sub < SUBS; sub += NW / WPS) {
      const int64_t s = s0 + sub;
      const uint32_t rt = (uint32_t)(tt0 + sub * 64 + lane) * SR_T;
      for (int grp = wave % WPS; grp < GROUPS; grp += WPS) {
        const int64_t jg = k0 + grp * P::EPL;
        const c_t* __restrict__ cg = C + s * g.Np + jg;        // wave-uniform
        const uint64_t* __restrict__ mg = g.masks + s * g.Np + jg;
        in_t v[P::EPL];
        if (g.mode == 0) {
          c_t cz[P::EPL];
          uint64_t mz[P::EPL];
#pragma unroll
          for (int e = 0; e < P::EPL; ++e) { cz[e] = cg[e]; mz[e] = mg[e]; }
#pragma unroll
          for (int e = 0; e < P::EPL; ++e) {
            const int64_t j = jg + e;
            T z = cz[e];
            if (mz[e] != 0 || g.planes > 1)
              z = z_from<T, EV>(cz[e], mz[e], lane, g.tab, EV ? g.ev.ainv + s * 64 : nullptr, g.masks,
                                g.planes, g.NS, g.Np, s, j);
            v[e] = P::cvt(z, rt + (uint32_t)j * SR_J);
          }
        } else {
#pragma unroll
          for (int e = 0; e < P::EPL; ++e) {
            const int64_t j = jg + e;
            const T z = zy_at<T, c_t>(C, CY, g.masks, g.planes, g.NS, g.Np, s, j, lane, ctau, g.tab);
            v[e] = P::cvt(z, rt + (uint32_t)j * SR_J);
          }
        }
        *(frag_t*)(Bs + (sub * 64 + lane) * ROWB + grp * 16) = *(frag_t*)v;
      }
    }
  };
  auto mma_step = [&](const unsigned char* As, const unsigned char* Bs) {
#pragma unroll
    for (int kc = 0; kc < BK; kc += KC) {
      frag_t af[WMB], bfr[WNB];
      const int koff = (kc + (lane / P::MB) * P::EPL) * (int)sizeof(in_t);
#pragma unroll
      for (int a = 0; a < WMB; ++a)
        af[a] = *(const frag_t*)(As + (wm * WM + a * P::MB + lane % P::MB) * ROWB + koff);
#pragma unroll
      for (int b = 0; b < WNB; ++b)
        bfr[b] = *(const frag_t*)(Bs + (wn * WN + b * P::MB + lane % P::MB) * ROWB + koff);
#pragma unroll
      for (int a = 0; a < WMB; ++a)
#pragma unroll
        for (int b = 0; b < WNB; ++b) P::mma(acc[a][b], af[a], bfr[b]);
    }
  };

  const int nk = (int)(g.Np / BK);
  load_a(0);
  store_a(As0);
  build_z(0, Bs0);
  __syncthreads();
  for (int ks = 0; ks < nk; ++ks) {
    const int cur = (DB == 2) ? (ks & 1) : 0;
    const bool more = ks + 1 < nk;
    if (more) load_a((int64_t)(ks + 1) * BK);
    mma_step(As0 + cur * ABUF, Bs0 + cur * BBUF);
    if (DB == 2) {
      if (more) {
        build_z((int64_t)(ks + 1) * BK, Bs0 + (cur ^ 1) * BBUF);
        store_a(As0 + (cur ^ 1) * ABUF);
      }
      __syncthreads();
    } else {
      __syncthreads();
      if (more) {
        store_a(As0);
        build_z((int64_t)(ks + 1) * BK, Bs0);
      }
      __syncthreads();
    }
  }

  // epilogue, mode 0: V = a^m acc, W = exp(V) (0 for padded bins), store
  // W' = W a^m, sum W per row.  Mode 1: acc = sum_j J zy, and
  // sum_t W V_y = sum_t W' acc (the a^m factors cancel); when the weights come
  // from the resident-trace kernel U they hold W itself and take the factor a^m.  FP64 row sums, one
  // block-row at a time.
  w_t* __restrict__ W = (w_t*)g.W;
  if constexpr (EV) {
    // Event grid: the interval integrals cost far more than exp, so each wave
    // stages one 16-row block of its tile in LDS (the operand buffers are free
    // after the last barrier of the k loop) and walks it a neuron row at a
    // time, lanes over 64 consecutive slots: one table load per lane, the
    // accumulators die block by block, W stores are contiguous, and the
    // branches of the integrals follow one neuron's potential through time.
    static_assert(WN == 64, "event-grid epilogue: a wave's tile is 64 slots wide");
    using st_t = typename std::remove_reference<decltype(acc[0][0][0])>::type;  // the accumulator type
    static_assert((size_t)NW * P::MB * WN * sizeof(st_t) <= (size_t)DB * (ABUF + BBUF),
                  "event-grid epilogue: the staged blocks fit in the operand buffers");
    st_t* stage = (st_t*)smem + wave * (P::MB * WN);
    const int tl = wn * WN + lane;
    const bool valid = (tt0 + tl) < g.B;
    const double pwd = g.ev.pw[tt0 + tl];
    const double pwm = (double)pw_of<T>(pwd);  // the factor the stored W' carries
    // The lane's slot is fixed: its constants are formed once.  BF16 mode
    // takes the FP32 chain of the resident kernels (expansion coefficients,
    // quadrature and FP64 tiers from the per-slot table), the others the FP64
    // evaluation.  Padded slots have zero length: both integrals vanish.
    constexpr bool F32 = sizeof(st_t) == 4;
    glmr_ev::Slot sc{};
    float cf[16];
    if constexpr (F32) {
      const float2 de = valid ? *(const float2*)(g.evgl + (tt0 + tl) * 16) : float2{0.f, 0.f};
      glmr_ev::stage_f(de.x, de.y, cf);
    } else {
      sc = glmr_ev::slot_consts(valid ? g.ev.delta[tt0 + tl] : 0.0);
    }
#pragma unroll
    for (int a = 0; a < WMB; ++a) {
      __syncthreads();
#pragma unroll
      for (int b = 0; b < WNB; ++b)
#pragma unroll
        for (int r = 0; r < P::NACC; ++r)
          stage[P::row(r, lane) * WN + b * P::MB + P::col(lane)] = acc[a][b][r];
      __syncthreads();
#pragma unroll 2
      for (int e = 0; e < P::MB; ++e) {
        const int il = wm * WM + a * P::MB + e;
        double F, H;
        if constexpr (F32) {  // BF16 mode: FP32 potential
          const float D = (float)pwd * stage[e * WN + lane];
          float Ff, Hf;
          if (!glmr_ev::taylor_f(cf, D, &Ff, &Hf))
            glmr_ev::gl_tier_f(g.evgl + (tt0 + tl) * 16 + 8, g.ev.delta[tt0 + tl], D, &Ff, &Hf);
          F = Ff;
          H = Hf;
        } else {
          glmr_ev::interval(pwd * (double)stage[e * WN + lane], sc, &F, &H);
        }
        W[(i0 + il) * g.L + (tl0 + tl)] = (w_t)(H * pwm);
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) F += __shfl_xor(F, off, 64);
        if (lane == 0) red[wn * BI + il] = F;
      }
    }
  } else
#pragma unroll
  for (int a = 0; a < WMB; ++a) {
    double rs[P::NACC];
#pragma unroll
    for (int r = 0; r < P::NACC; ++r) rs[r] = 0.0;
#pragma unroll
    for (int b = 0; b < WNB; ++b) {
      const int tl = wn * WN + b * P::MB + P::col(lane);
      const bool valid = (tt0 + tl) < g.B;
      const T pw = tab_pw<T>(g.tab, tl & 63);
#pragma unroll
      for (int r = 0; r < P::NACC; ++r) {
        const int il = wm * WM + a * P::MB + P::row(r, lane);
        // the resident kernel U stores W tile-major or as MFMA fragments
        const int64_t tc = tl0 + tl;
        w_t* wp = W + w_elem(g.w_plain, i0 + il, tc, g.Np, g.L);
        if (g.mode == 0) {
          auto lam = P::lam(pw * acc[a][b][r]);
          if (!valid) lam = 0;
          *wp = (w_t)(lam * pw);
          rs[r] += (double)lam;
        } else {
          const double wv = g.w_plain ? (double)(*wp) * (double)pw : (double)(*wp);
          rs[r] += wv * (double)acc[a][b][r];
        }
      }
    }
    // reduce over the lanes holding the same row (the column lanes)
#pragma unroll
    for (int r = 0; r < P::NACC; ++r) {
      double v = rs[r];
#pragma unroll
      for (int off = 1; off < P::MB; off <<= 1) v += __shfl_xor(v, off, 64);
      if (P::col(lane) == 0) red[wn * BI + wm * WM + a * P::MB + P::row(r, lane)] = v;
    }
  }
  __syncthreads();
  for (int il = tid; il < BI; il += NT) {
    double v = 0.0;
#pragma unroll
    for (int q = 0; q < WGN; ++q) v += red[q * BI + il];
    g.rowpart[(tt0 / BT) * g.Np + i0 + il] = v;
  }
}

// ---------------------------------------------------------------- kernel G
template <int PREC, int BI, int BJ, int WGM, int WGN, int DB, bool EV>
__global__ __launch_bounds__(WGM * WGN * 64) void k_gemm2(Gemm2Args g) {
  using P = Pol<PREC>;
  using in_t = typename P::in_t;
  using c_t = typename P::c_t;
  using w_t = typename P::w_t;
  using frag_t = typename P::frag_t;
  using acc_t = typename P::acc_t;
  using T = c_t;
  static_assert(sizeof(w_t) == sizeof(in_t) || 2 * sizeof(w_t) == sizeof(in_t),
                "W is staged as the A operand, as is or widened to the operand type");
  constexpr bool WIDEN = sizeof(w_t) != sizeof(in_t);
  constexpr int NW = WGM * WGN;
  constexpr int NT = NW * 64;
  constexpr int BK = 64;                               // bins per step (one subtile)
  constexpr int ROWB = BK * sizeof(in_t) + PAD;
  constexpr int WM = BI / WGM, WN = BJ / WGN;
  constexpr int WMB = WM / P::MB, WNB = WN / P::MB;
  constexpr int KC = P::EPL * (64 / P::MB);
  constexpr int ABUF = BI * ROWB, BBUF = BJ * ROWB;
  constexpr int CPW = BJ / NW;  // trace columns rebuilt per wave
  constexpr int CG = 8;         // columns per scalar-load group
  static_assert(CPW % CG == 0, "column groups");

  extern __shared__ __align__(16) unsigned char smem[];
  unsigned char* As0 = smem;                 // [DB][BI][ROWB]  W' tile (row = neuron i)
  unsigned char* Bs0 = smem + DB * ABUF;     // [DB][BJ][ROWB]  z tile (row = neuron j)

  const int tid = threadIdx.x, lane = tid & 63, wave = uniform(tid >> 6);
  const int wm = wave / WGN, wn = wave % WGN;
  const int64_t logical = xcd_logical(blockIdx.x, gridDim.x);
  const int jtile = (int)(logical % g.n_jtiles);
  const int itile = (int)((logical / g.n_jtiles) % g.n_itiles);
  const int split = (int)(logical / ((int64_t)g.n_jtiles * g.n_itiles));
  const int64_t i0 = (int64_t)itile * BI, j0 = (int64_t)jtile * BJ;
  const int64_t tb = (int64_t)split * g.ks;                 // chunk-local
  const int64_t te = (tb + g.ks < g.Lc) ? tb + g.ks : g.Lc;
  const w_t* __restrict__ W = (const w_t*)g.W;
  const c_t* __restrict__ C = (const c_t*)g.C;

  acc_t acc[WMB][WNB];
#pragma unroll
  for (int a = 0; a < WMB; ++a)
#pragma unroll
    for (int b = 0; b < WNB; ++b)
#pragma unroll
      for (int r = 0; r < P::NACC; ++r) acc[a][b][r] = 0;

  constexpr int RP = BK * sizeof(w_t) / 16;    // 16-byte pieces of W per row
  constexpr int APIECES = BI * RP;
  constexpr int APT = (APIECES + NT - 1) / NT;
  i32x4 areg[APT];
  auto load_a = [&](int64_t tk) {
#pragma unroll
    for (int q = 0; q < APT; ++q) {
      int piece = tid + q * NT;
      if (piece < APIECES) {
        int r = piece / RP, c16 = piece % RP;
        areg[q] = *(const i32x4*)((const unsigned char*)(W + (i0 + r) * g.L + tk) + c16 * 16);
      }
    }
  };
  auto store_a = [&](unsigned char* As) {
#pragma unroll
    for (int q = 0; q < APT; ++q) {
      int piece = tid + q * NT;
      if (piece < APIECES) {
        int r = piece / RP, c16 = piece % RP;
        if constexpr (WIDEN) {
          const float* f = (const float*)&areg[q];
          in_t* d = (in_t*)(As + r * ROWB + c16 * 32);
          d[0] = (in_t)f[0];
          d[1] = (in_t)f[1];
          d[2] = (in_t)f[2];
          d[3] = (in_t)f[3];
        } else {
          *(i32x4*)(As + r * ROWB + c16 * 16) = areg[q];
        }
      }
    }
  };
  auto build_z = [&](int64_t tk, unsigned char* Bs) {
    const int64_t tg = g.t0 + tk;                 // global first bin of the step
    const int64_t s = tg / 64;
    const uint32_t rt = (uint32_t)(tg + lane) * SR_T;
    for (int cgi = 0; cgi < CPW; cgi += CG) {
      const int64_t jg = j0 + wave * CPW + cgi;
      const c_t* __restrict__ cg = C + s * g.Np + jg;         // wave-uniform
      const uint64_t* __restrict__ mg = g.masks + s * g.Np + jg;
      c_t cz[CG];
      uint64_t mz[CG];
#pragma unroll
      for (int e = 0; e < CG; ++e) { cz[e] = cg[e]; mz[e] = mg[e]; }
#pragma unroll
      for (int e = 0; e < CG; ++e) {
        const int64_t j = jg + e;
        T z = cz[e];
        if (mz[e] != 0 || g.planes > 1)
          z = z_from<T, EV>(cz[e], mz[e], lane, g.tab, EV ? g.ev.ainv + s * 64 : nullptr, g.masks,
                            g.planes, g.NS, g.Np, s, j);
        *(in_t*)(Bs + (wave * CPW + cgi + e) * ROWB + lane * sizeof(in_t)) =
            P::cvt(z, rt + (uint32_t)j * SR_J);
      }
    }
  };
  auto mma_step = [&](const unsigned char* As, const unsigned char* Bs) {
#pragma unroll
    for (int kc = 0; kc < BK; kc += KC) {
      frag_t af[WMB], bfr[WNB];
      const int koff = (kc + (lane / P::MB) * P::EPL) * (int)sizeof(in_t);
#pragma unroll
      for (int a = 0; a < WMB; ++a)
        af[a] = *(const frag_t*)(As + (wm * WM + a * P::MB + lane % P::MB) * ROWB + koff);
#pragma unroll
      for (int b = 0; b < WNB; ++b)
        bfr[b] = *(const frag_t*)(Bs + (wn * WN + b * P::MB + lane % P::MB) * ROWB + koff);
#pragma unroll
      for (int a = 0; a < WMB; ++a)
#pragma unroll
        for (int b = 0; b < WNB; ++b) P::mma(acc[a][b], af[a], bfr[b]);
    }
  };

  if (tb < te) {
    load_a(tb);
    store_a(As0);
    build_z(tb, Bs0);
  }
  __syncthreads();
  int it = 0;
  for (int64_t tk = tb; tk < te; tk += BK, ++it) {
    const int cur = (DB == 2) ? (it & 1) : 0;
    const bool more = tk + BK < te;
    if (more) load_a(tk + BK);
    mma_step(As0 + cur * ABUF, Bs0 + cur * BBUF);
    if (DB == 2) {
      if (more) {
        build_z(tk + BK, Bs0 + (cur ^ 1) * BBUF);
        store_a(As0 + (cur ^ 1) * ABUF);
      }
      __syncthreads();
    } else {
      __syncthreads();
      if (more) {
        store_a(As0);
        build_z(tk + BK, Bs0);
      }
      __syncthreads();
    }
  }

  using gp_t = typename P::gp_t;
  gp_t* __restrict__ Gp = (gp_t*)g.Gp + (int64_t)split * g.Np * g.Np;
#pragma unroll
  for (int a = 0; a < WMB; ++a)
#pragma unroll
    for (int b = 0; b < WNB; ++b)
#pragma unroll
      for (int r = 0; r < P::NACC; ++r) {
        const int il = wm * WM + a * P::MB + P::row(r, lane);
        const int jl = wn * WN + b * P::MB + P::col(lane);
        Gp[(i0 + il) * g.Np + j0 + jl] = (gp_t)acc[a][b][r];
      }
}

template <int PREC, int BI, int BT, int WGM, int WGN, int DB, bool EV = false, int KB = 128>
hipError_t run_gemm1(const Gemm1Args& a, hipStream_t st) {
  using P = Pol<PREC>;
  constexpr int BK = KB / sizeof(typename P::in_t);
  constexpr int ROWB = BK * sizeof(typename P::in_t) + PAD;
  size_t lds = (size_t)DB * (BI + BT) * ROWB + (size_t)WGN * BI * sizeof(double);
  auto kern = k_gemm1<PREC, BI, BT, WGM, WGN, DB, EV, KB>;
  hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  int64_t nblk = (int64_t)a.n_itiles * a.n_ttiles;
  hipLaunchKernelGGL(kern, dim3((unsigned)nblk), dim3(WGM * WGN * 64), lds, st, a);
  return hipGetLastError();
}

template <int PREC, int BI, int BJ, int WGM, int WGN, int DB, bool EV = false>
hipError_t run_gemm2(const Gemm2Args& a, hipStream_t st) {
  using P = Pol<PREC>;
  constexpr int ROWB = 64 * sizeof(typename P::in_t) + PAD;
  size_t lds = (size_t)DB * (BI + BJ) * ROWB;
  auto kern = k_gemm2<PREC, BI, BJ, WGM, WGN, DB, EV>;
  hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  int64_t nblk = (int64_t)a.n_splits * a.n_itiles * a.n_jtiles;
  hipLaunchKernelGGL(kern, dim3((unsigned)nblk), dim3(WGM * WGN * 64), lds, st, a);
  return hipGetLastError();
}

}  // namespace

// Tile shapes: BI x BT for kernel U/V, BI x BJ for kernel G.  `tile` is the
// neuron tile of the context (the padding unit of N).
hipError_t launch_gemm1(int prec, int tile, const Gemm1Args& a, hipStream_t st) {
  if (a.ev.pw) {  // event grid: FP64, FP32 and BF16 modes, likelihood kernel only
    if (a.mode != 0) return hipErrorInvalidValue;
    if (prec == PREC_F64) return run_gemm1<PREC_F64, 128, 256, 2, 4, 2, true, 128>(a, st);
    if (prec == PREC_F32) return run_gemm1<PREC_F32U, 128, 256, 2, 4, 2, true, 128>(a, st);
    if (prec == PREC_BF16) {
      if (tile == 128) return run_gemm1<PREC_BF16, 128, 256, 2, 4, 2, true>(a, st);
      return run_gemm1<PREC_BF16, 256, 256, 2, 4, 2, true>(a, st);
    }
    return hipErrorInvalidValue;
  }
  switch (prec) {
    case PREC_F64: return run_gemm1<PREC_F64, 128, 256, 2, 4, 2, false, 128>(a, st);
    case PREC_F32: return run_gemm1<PREC_F32U, 128, 256, 2, 4, 2, false, 128>(a, st);
    case PREC_BF16:
      if (tile == 128) return run_gemm1<PREC_BF16, 128, 256, 2, 4, 2>(a, st);
      return run_gemm1<PREC_BF16, 256, 256, 2, 4, 2>(a, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_gemm2(int prec, int tile, const Gemm2Args& a, hipStream_t st) {
  if (a.ev.pw) {
    if (prec == PREC_F64) return run_gemm2<PREC_F64, 128, 128, 2, 2, 1, true>(a, st);
    if (prec == PREC_F32) return run_gemm2<PREC_F32G, 128, 128, 2, 2, 1, true>(a, st);
    if (prec == PREC_BF16) {
      if (tile == 128) return run_gemm2<PREC_BF16, 128, 128, 2, 4, 2, true>(a, st);
      return run_gemm2<PREC_BF16, 256, 256, 2, 4, 2, true>(a, st);
    }
    return hipErrorInvalidValue;
  }
  switch (prec) {
    case PREC_F64: return run_gemm2<PREC_F64, 128, 128, 2, 2, 1>(a, st);
    case PREC_F32: return run_gemm2<PREC_F32G, 128, 128, 2, 2, 1>(a, st);
    case PREC_BF16:
      if (tile == 128) return run_gemm2<PREC_BF16, 128, 128, 2, 4, 2>(a, st);
      return run_gemm2<PREC_BF16, 256, 256, 2, 4, 2>(a, st);
    default: return hipErrorInvalidValue;
  }
}

// Tile sizes the runtime must respect (rows of the neuron tile, bins of the time tile).
void gemm_tiles(int prec, int tile, int* bi1, int* bt1, int* bi2, int* bj2) {
  switch (prec) {
    case PREC_F64: *bi1 = 128; *bt1 = 256; *bi2 = 128; *bj2 = 128; break;
    case PREC_F32: *bi1 = 128; *bt1 = 256; *bi2 = 128; *bj2 = 128; break;
    default:
      if (tile == 128) { *bi1 = 128; *bt1 = 256; *bi2 = 128; *bj2 = 128; }
      else { *bi1 = 256; *bt1 = 256; *bi2 = 256; *bj2 = 256; }
  }
}
