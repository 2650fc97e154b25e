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
//       time split (no atomics; reduced in a fixed order in FP64).
//
// The trace x never exists in HBM: each workgroup rebuilds the tile it needs
// in LDS from the spike bitmasks and the per-subtile carries,
//   x_j[64 s + m] = a^m (C[s][j] + sum_{b < m, bit b of mask(s, j)} a^-(b+1)),
// one wavefront per 64-bin subtile (lane = bin), so the per-column mask and
// carry are wave-uniform scalar loads.
//
// Both contractions are C[m][n] = sum_k A[m][k] B[n][k] with A and B staged in
// LDS with k contiguous (rows padded by 16 bytes).  The MFMA shapes:
//   FP64 v_mfma_f64_16x16x4f64, FP32 v_mfma_f32_32x32x2f32,
//   BF16 v_mfma_f32_32x32x16_bf16.
// Each lane reads 16 contiguous bytes of k per operand and block; the k order
// inside a 16-byte group is the same for A and B, so any permutation the
// instruction applies inside the group cancels.
#include "common.h"

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
  __device__ static inline in_t cvt(double x) { return x; }
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
  __device__ static inline in_t cvt(double x) { return (float)x; }
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
  __device__ static inline in_t cvt(float x) { return (__bf16)x; }
};

template <typename T> __device__ inline T tab_pw(const Tables* t, int m);
template <> __device__ inline double tab_pw<double>(const Tables* t, int m) { return t->pw[m]; }
template <> __device__ inline float tab_pw<float>(const Tables* t, int m) { return t->pw32[m]; }
template <typename T> __device__ inline T tab_ainv(const Tables* t, int b);
template <> __device__ inline double tab_ainv<double>(const Tables* t, int b) { return t->ainv[b]; }
template <> __device__ inline float tab_ainv<float>(const Tables* t, int b) { return t->ainv32[b]; }

__device__ inline int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// XCD-aware block order: the hardware deals consecutive workgroups round-robin
// over the 8 XCDs; renumber so that each XCD receives a contiguous range of
// logical tiles (tiles that share an operand land on the same L2).
__device__ inline int64_t xcd_logical(int64_t bid, int64_t nblk) {
  const int64_t nx = 8;
  int64_t x = bid % nx, idx = bid / nx;
  int64_t q = nblk / nx, r = nblk % nx;
  return x * q + (x < r ? x : r) + idx;
}

// Trace value at lane bin m of subtile s for column j (C: carry at the subtile
// start), from the mask bits below m.  T is the arithmetic type.
template <typename T, typename CT>
__device__ inline T trace_at(const CT* __restrict__ C, const uint64_t* __restrict__ masks,
                             int planes, int64_t NS, int64_t Np, int64_t s, int64_t j, int m,
                             T pw_m, const Tables* tab) {
  T run = (T)C[s * Np + j];
  for (int p = 0; p < planes; ++p) {
    uint64_t mk = masks[((int64_t)p * NS + s) * Np + j];
    while (mk) {
      int b = __builtin_ctzll(mk);
      mk &= mk - 1;
      if (b < m) run += tab_ainv<T>(tab, b);
    }
  }
  return pw_m * run;
}

// d x / d tau at lane bin m: a^m (CY + m c C + c sum_{b<m} (m-b-1) a^-(b+1))
template <typename T, typename CT>
__device__ inline T ytrace_at(const CT* __restrict__ C, const CT* __restrict__ CY,
                              const uint64_t* __restrict__ masks, int planes, int64_t NS,
                              int64_t Np, int64_t s, int64_t j, int m, T pw_m, T ctau,
                              const Tables* tab) {
  T acc = (T)CY[s * Np + j] + (T)m * ctau * (T)C[s * Np + j];
  T inner = 0;
  for (int p = 0; p < planes; ++p) {
    uint64_t mk = masks[((int64_t)p * NS + s) * Np + j];
    while (mk) {
      int b = __builtin_ctzll(mk);
      mk &= mk - 1;
      if (b < m) inner += (T)(m - b - 1) * tab_ainv<T>(tab, b);
    }
  }
  return pw_m * (acc + ctau * inner);
}

constexpr int PAD = 16;  // bytes of padding per LDS row

// Wave-uniform copy of lane `l`'s value (v_readlane): the carry and mask of a
// column are loaded once per step by one lane each (a coalesced vector load)
// and broadcast column by column without a memory round trip.
__device__ inline float bcast(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ inline double bcast(double v, int l) {
  const int64_t b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((int64_t)hi << 32) | (uint32_t)lo);
}
__device__ inline uint64_t bcast(uint64_t v, int l) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(v & 0xffffffffu), l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(v >> 32), l);
  return ((uint64_t)hi << 32) | lo;
}

// x at lane bin m from the column's carry c and plane-0 mask mk (uniform);
// further planes (several spikes in one bin) are read directly.
template <typename T>
__device__ inline T x_from(T c, uint64_t mk, int m, T pw_m, const Tables* tab,
                           const uint64_t* __restrict__ masks, int planes, int64_t NS,
                           int64_t Np, int64_t s, int64_t j) {
  T run = c;
  while (mk) {
    const int b = __builtin_ctzll(mk);
    mk &= mk - 1;
    if (b < m) run += tab_ainv<T>(tab, b);
  }
  for (int p = 1; p < planes; ++p) {
    uint64_t mp = masks[((int64_t)p * NS + s) * Np + j];
    while (mp) {
      const int b = __builtin_ctzll(mp);
      mp &= mp - 1;
      if (b < m) run += tab_ainv<T>(tab, b);
    }
  }
  return pw_m * run;
}

// ---------------------------------------------------------------- kernel U/V
template <int PREC, int BI, int BT, int WGM, int WGN>
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
  constexpr int BK = 128 / sizeof(in_t);          // k (presynaptic j) per step
  constexpr int ROWB = BK * sizeof(in_t) + PAD;   // LDS row pitch, bytes
  constexpr int WM = BI / WGM, WN = BT / WGN;
  constexpr int WMB = WM / P::MB, WNB = WN / P::MB;
  constexpr int GROUPS = BK / P::EPL;             // 16-byte column groups per row
  constexpr int SUBS = BT / 64;
  constexpr int KC = P::EPL * (64 / P::MB);       // k per MFMA chunk

  extern __shared__ __align__(16) unsigned char smem[];
  unsigned char* As = smem;                       // [BI][ROWB]   J tile
  unsigned char* Bs = smem + BI * ROWB;           // [BT][ROWB]   x tile (row = bin)
  double* red = (double*)(smem + (BI + BT) * ROWB);  // [WGN][BI]

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
  const T pw_m = tab_pw<T>(g.tab, lane);
  const T ctau = (T)g.ctau;

  acc_t acc[WMB][WNB];
#pragma unroll
  for (int a = 0; a < WMB; ++a)
#pragma unroll
    for (int b = 0; b < WNB; ++b)
#pragma unroll
      for (int r = 0; r < P::NACC; ++r) acc[a][b][r] = 0;

  constexpr int APIECES = BI * (BK * sizeof(in_t) / 16);
  constexpr int APT = (APIECES + NT - 1) / NT;
  i32x4 areg[APT];
  auto load_a = [&](int64_t k0) {
#pragma unroll
    for (int q = 0; q < APT; ++q) {
      int piece = tid + q * NT;
      if (piece < APIECES) {
        int r = piece / (BK * (int)sizeof(in_t) / 16), c16 = piece % (BK * (int)sizeof(in_t) / 16);
        areg[q] = *(const i32x4*)((const unsigned char*)(Jc + (i0 + r) * g.Np + k0) + c16 * 16);
      }
    }
  };
  auto store_a = [&]() {
#pragma unroll
    for (int q = 0; q < APT; ++q) {
      int piece = tid + q * NT;
      if (piece < APIECES) {
        int r = piece / (BK * (int)sizeof(in_t) / 16), c16 = piece % (BK * (int)sizeof(in_t) / 16);
        *(i32x4*)(As + r * ROWB + c16 * 16) = areg[q];
      }
    }
  };

  load_a(0);
  for (int64_t k0 = 0; k0 < g.Np; k0 += BK) {
    store_a();
    // rebuild the trace tile: each wave owns one subtile (lane = bin) and a
    // share of its 16-byte column groups
    {
      constexpr int WPS = NW >= SUBS ? NW / SUBS : 1;  // waves per subtile
      for (int sub = wave / WPS; sub < SUBS; sub += NW / WPS) {
        const int64_t s = s0 + sub;
        const int64_t jl = k0 + (lane < BK ? lane : 0);
        const c_t cv = C[s * g.Np + jl];
        const uint64_t mv = g.masks[s * g.Np + jl];
        const c_t cyv = (g.mode == 1) ? CY[s * g.Np + jl] : (c_t)0;
        for (int grp = wave % WPS; grp < GROUPS; grp += WPS) {
          in_t v[P::EPL];
#pragma unroll
          for (int e = 0; e < P::EPL; ++e) {
            const int col = grp * P::EPL + e;
            const c_t c = bcast(cv, col);
            const uint64_t mk = bcast(mv, col);
            T x;
            if (g.mode == 0) {
              x = x_from<T>(c, mk, lane, pw_m, g.tab, g.masks, g.planes, g.NS, g.Np, s, k0 + col);
            } else {
              x = ytrace_at<T, c_t>(C, CY, g.masks, g.planes, g.NS, g.Np, s, k0 + col, lane, pw_m,
                                    ctau, g.tab);
              (void)cyv;
            }
            v[e] = P::cvt(x);
          }
          *(frag_t*)(Bs + (sub * 64 + lane) * ROWB + grp * 16) = *(frag_t*)v;
        }
      }
    }
    __syncthreads();
    if (k0 + BK < g.Np) load_a(k0 + BK);  // prefetch the next J tile into registers
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
    __syncthreads();
  }

  // epilogue: W = exp(V) (mode 0) or sum W V (mode 1); per-row FP64 sums,
  // one block-row at a time
  w_t* __restrict__ W = (w_t*)g.W;
#pragma unroll
  for (int a = 0; a < WMB; ++a) {
    double rs[P::NACC];
#pragma unroll
    for (int r = 0; r < P::NACC; ++r) rs[r] = 0.0;
#pragma unroll
    for (int b = 0; b < WNB; ++b)
#pragma unroll
      for (int r = 0; r < P::NACC; ++r) {
        const int il = wm * WM + a * P::MB + P::row(r, lane);
        const int tl = wn * WN + b * P::MB + P::col(lane);
        const bool valid = (tt0 + tl) < g.B;
        w_t* wp = W + (i0 + il) * g.L + (tl0 + tl);
        if (g.mode == 0) {
          auto lam = P::lam(acc[a][b][r]);
          if (!valid) lam = 0;
          *wp = (w_t)lam;
          rs[r] += (double)lam;
        } else {
          rs[r] += (double)(*wp) * (double)acc[a][b][r];
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
template <int PREC, int BI, int BJ, int WGM, int WGN>
__global__ __launch_bounds__(WGM * WGN * 64) void k_gemm2(Gemm2Args g) {
  using P = Pol<PREC>;
  using in_t = typename P::in_t;
  using c_t = typename P::c_t;
  using w_t = typename P::w_t;
  using frag_t = typename P::frag_t;
  using acc_t = typename P::acc_t;
  using T = c_t;
  static_assert(sizeof(w_t) == sizeof(in_t), "W is staged as the A operand");
  constexpr int NW = WGM * WGN;
  constexpr int NT = NW * 64;
  constexpr int BK = 64;                               // bins per step (one subtile)
  constexpr int ROWB = BK * sizeof(in_t) + PAD;
  constexpr int WM = BI / WGM, WN = BJ / WGN;
  constexpr int WMB = WM / P::MB, WNB = WN / P::MB;
  constexpr int KC = P::EPL * (64 / P::MB);

  extern __shared__ __align__(16) unsigned char smem[];
  unsigned char* As = smem;                 // [BI][ROWB]  W tile (row = neuron i)
  unsigned char* Bs = smem + BI * ROWB;     // [BJ][ROWB]  x tile (row = neuron j)

  const int tid = threadIdx.x, lane = tid & 63, wave = uniform(tid >> 6);
  const int wm = wave / WGN, wn = wave % WGN;
  const int64_t logical = xcd_logical(blockIdx.x, gridDim.x);
  const int jtile = (int)(logical % g.n_jtiles);
  const int itile = (int)((logical / g.n_jtiles) % g.n_itiles);
  const int split = (int)(logical / ((int64_t)g.n_jtiles * g.n_itiles));
  const int64_t i0 = (int64_t)itile * BI, j0 = (int64_t)jtile * BJ;
  const int64_t tb = (int64_t)split * g.ks;                 // chunk-local
  const int64_t te = (tb + g.ks < g.L) ? tb + g.ks : g.L;
  const w_t* __restrict__ W = (const w_t*)g.W;
  const c_t* __restrict__ C = (const c_t*)g.C;
  const T pw_m = tab_pw<T>(g.tab, lane);

  acc_t acc[WMB][WNB];
#pragma unroll
  for (int a = 0; a < WMB; ++a)
#pragma unroll
    for (int b = 0; b < WNB; ++b)
#pragma unroll
      for (int r = 0; r < P::NACC; ++r) acc[a][b][r] = 0;

  constexpr int RP = BK * sizeof(in_t) / 16;   // 16-byte pieces per row
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
  auto store_a = [&]() {
#pragma unroll
    for (int q = 0; q < APT; ++q) {
      int piece = tid + q * NT;
      if (piece < APIECES) {
        int r = piece / RP, c16 = piece % RP;
        *(i32x4*)(As + r * ROWB + c16 * 16) = areg[q];
      }
    }
  };

  if (tb < te) load_a(tb);
  for (int64_t tk = tb; tk < te; tk += BK) {
    store_a();
    const int64_t s = (g.t0 + tk) / 64;
    {
      constexpr int CPW = BJ / NW;  // columns per wave (<= 64)
      static_assert(CPW <= 64, "one column per lane in the preload");
      const int64_t jw = j0 + wave * CPW;
      const int64_t jl = jw + (lane < CPW ? lane : 0);
      const c_t cv = C[s * g.Np + jl];
      const uint64_t mv = g.masks[s * g.Np + jl];
      for (int col = 0; col < CPW; ++col) {
        const T x = x_from<T>(bcast(cv, col), bcast(mv, col), lane, pw_m, g.tab, g.masks, g.planes,
                              g.NS, g.Np, s, jw + col);
        *(in_t*)(Bs + (wave * CPW + col) * ROWB + lane * sizeof(in_t)) = P::cvt(x);
      }
    }
    __syncthreads();
    if (tk + BK < te) load_a(tk + BK);
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
    __syncthreads();
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

template <int PREC, int BI, int BT, int WGM, int WGN>
hipError_t run_gemm1(const Gemm1Args& a, hipStream_t st) {
  using P = Pol<PREC>;
  constexpr int BK = 128 / sizeof(typename P::in_t);
  constexpr int ROWB = BK * sizeof(typename P::in_t) + PAD;
  size_t lds = (size_t)(BI + BT) * ROWB + (size_t)WGN * BI * sizeof(double);
  auto kern = k_gemm1<PREC, BI, BT, WGM, WGN>;
  hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  int64_t nblk = (int64_t)a.n_itiles * a.n_ttiles;
  hipLaunchKernelGGL(kern, dim3((unsigned)nblk), dim3(WGM * WGN * 64), lds, st, a);
  return hipGetLastError();
}

template <int PREC, int BI, int BJ, int WGM, int WGN>
hipError_t run_gemm2(const Gemm2Args& a, hipStream_t st) {
  using P = Pol<PREC>;
  constexpr int ROWB = 64 * sizeof(typename P::in_t) + PAD;
  size_t lds = (size_t)(BI + BJ) * ROWB;
  auto kern = k_gemm2<PREC, BI, BJ, WGM, WGN>;
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
  switch (prec) {
    case PREC_F64: return run_gemm1<PREC_F64, 128, 128, 2, 2>(a, st);
    case PREC_F32: return run_gemm1<PREC_F32, 128, 256, 2, 2>(a, st);
    case PREC_BF16:
      if (tile == 128) return run_gemm1<PREC_BF16, 128, 256, 2, 2>(a, st);
      return run_gemm1<PREC_BF16, 256, 256, 2, 2>(a, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_gemm2(int prec, int tile, const Gemm2Args& a, hipStream_t st) {
  switch (prec) {
    case PREC_F64: return run_gemm2<PREC_F64, 128, 128, 2, 2>(a, st);
    case PREC_F32: return run_gemm2<PREC_F32, 128, 128, 2, 2>(a, st);
    case PREC_BF16:
      if (tile == 128) return run_gemm2<PREC_BF16, 128, 128, 2, 2>(a, st);
      return run_gemm2<PREC_BF16, 256, 256, 2, 2>(a, st);
    default: return hipErrorInvalidValue;
  }
}

// Tile sizes the runtime must respect (rows of the neuron tile, bins of the time tile).
extern "C++" void gemm_tiles(int prec, int tile, int* bi1, int* bt1, int* bi2, int* bj2) {
  switch (prec) {
    case PREC_F64: *bi1 = 128; *bt1 = 128; *bi2 = 128; *bj2 = 128; break;
    case PREC_F32: *bi1 = 128; *bt1 = 256; *bi2 = 128; *bj2 = 128; break;
    default:
      if (tile == 128) { *bi1 = 128; *bt1 = 256; *bi2 = 128; *bj2 = 128; }
      else { *bi1 = 256; *bt1 = 256; *bi2 = 256; *bj2 = 256; }
  }
}
