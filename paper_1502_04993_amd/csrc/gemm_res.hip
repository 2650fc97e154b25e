// BF16 likelihood contractions on a resident trace (gfx950).
//
// The trace x_j[t] depends on the spikes and tau only, not on (J, mu), so
// during an ascent at fixed tau it is the same at every evaluation.  When it
// fits in HBM it is built once per tau, rounded to BF16, and kept in two
// layouts, each with the contraction index contiguous:
//   Xtj[t][j]  (pitch Np)  operand of kernel U:  V[i][t] = sum_j J[i][j] x_j[t]
//   Xjt[j][t]  (pitch Bp)  operand of kernel G:  G[i][j] = sum_t W[i][t] x_j[t]
// Both contractions are then plain "NT" products C[m][n] = sum_k A[m][k] B[n][k]
// with A and B row-major and k contiguous, run by one MFMA core
// (v_mfma_f32_32x32x16_bf16, FP32 accumulation) with LDS double buffering:
//   kernel U  A = J (bf16, rows i), B = Xtj (rows t); epilogue W = exp(V)
//             (0 for padded bins) stored as BF16 and FP64 row sums of W per
//             256-bin tile (the integral term of Eq. (7) up to dt e^{mu_i});
//   kernel G  A = W (rows i, one chunk of bins), B = Xjt (rows j); one FP32
//             partial per time split (the integral of Eq. (12) up to the same
//             factor), reduced in FP64 in a fixed order.
// Trace rounding is stochastic with the bits r(t, j) = t*0x9E3779B9 +
// j*0x6C8E9CF5, so each stored value is an unbiased estimate of x_j[t] and the
// two layouts hold the identical rounded value.
//
// FP8 (OCP formats, v_mfma_scale_f32_32x32x64_f8f6f4 with unit block scales):
//   trace  e4m3, times a power-of-two scale per time chunk, 2^floor(log2(448 /
//          max x)), rounded stochastically with the same bits r(t, j);
//   J      e4m3, times a power-of-two scale per row (set when the parameters
//          are), rounded to nearest; the likelihood is that of the rounded J;
//   W      e5m2, W' = exp(V) / 64 rounded stochastically (bits from (t, i)),
//          whose range covers exp(V) for V in about [-7, 15] without a scale.
// Scales are powers of two, so applying and removing them is exact; the row
// sums of exp(V) are taken in FP32/FP64 before W is rounded.
//
// Event grid (continuous time, BF16): the trace is built with the per-slot
// decays (x_{m+1} = e^{-delta_m} x_m + spikes) and kernel U's epilogue takes
// the interval integrals of Eq. (10), (14) in place of exp, in FP32 by the
// midpoint expansion (one exponential per potential; intervals past its
// bound by 6-point Gauss-Legendre or in FP64) from a per-slot table; W then
// holds (e^D - e^{D xi}) / D and the row sums Ei(D) - Ei(D xi).
#include <type_traits>

#include "common.h"
#include "evfun.h"

namespace {

constexpr uint32_t SR_T = 0x9E3779B9u, SR_J = 0x6C8E9CF5u;
constexpr int BK = 64;               // k per pipeline step
constexpr int ROWB = BK * 2 + 16;    // LDS row pitch in bytes (16 B pad: conflict-free b128 reads)

typedef __attribute__((ext_vector_type(2))) __bf16 bf16x2;

__device__ inline int64_t xcd_logical(int64_t bid, int64_t nblk) {
  // consecutive logical tiles land on the same XCD (and share its L2)
  const int64_t nx = 8;
  const int64_t x = bid % nx, idx = bid / nx;
  const int64_t q = nblk / nx, r = nblk % nx;
  return x * q + (x < r ? x : r) + idx;
}

// ------------------------------------------------------------------ trace build
// One workgroup per (subtile s, 64-column block): thread (jj, g) evaluates bins
// 16g .. 16g+15 of column j in FP64, from the carry C[s][j] and the spikes of
// the subtile, and rounds them to BF16.  Xjt rows are written straight from
// registers (32 contiguous bytes per thread); Xtj rows go through LDS so that
// each row of 64 columns is written as 128 contiguous bytes.
__global__ __launch_bounds__(256) void k_build_x(ResXArgs g) {
  __shared__ __align__(16) unsigned char tile[64 * ROWB];
  const int64_t njb = g.Np / 64;
  const int64_t s = blockIdx.x / njb, jb = blockIdx.x % njb;
  const int tid = threadIdx.x, jj = tid & 63, gq = tid >> 6;
  const int64_t j = jb * 64 + jj;
  const int m0 = 16 * gq;
  const double a = g.tab->pw[1];
  const bool ev = g.ev.pw != nullptr;  // event grid: per-slot decays

  // trace at bin (slot) 64 s + m0: the carry decayed, plus the spikes of the
  // subtile before m0
  double x, zs = 0.0;
  uint32_t cnt[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) cnt[e] = 0;
  x = ev ? 0.0 : g.C64[s * g.Np + j] * g.tab->pw[m0];
  for (int p = 0; p < g.planes; ++p) {
    const uint64_t mk = g.masks[((int64_t)p * g.NS + s) * g.Np + j];
    uint64_t below = (m0 == 0) ? 0ull : (mk & ((1ull << m0) - 1));
    while (below) {
      const int b = __builtin_ctzll(below);
      below &= below - 1;
      if (ev) zs += g.ev.ainv[s * 64 + b];
      else x += g.tab->pw[m0 - b - 1];
    }
    const uint32_t win = (uint32_t)((mk >> m0) & 0xffffu);
#pragma unroll
    for (int e = 0; e < 16; ++e) cnt[e] += (win >> e) & 1u;
  }
  if (ev) x = g.ev.pw[s * 64 + m0] * (g.C64[s * g.Np + j] + zs);

  // round pairs of bins to BF16; w[e/2] holds bins m0+e (low half) and m0+e+1
  uint32_t w[8];
  const uint32_t rj = (uint32_t)j * SR_J;
#pragma unroll
  for (int e = 0; e < 16; e += 2) {
    const int64_t t = s * 64 + m0 + e;
    const double a0 = ev ? g.ev.edec[t] : a;  // decay over bin (slot) t
    const double a1 = ev ? g.ev.edec[t + 1] : a;
    const float x0 = (float)x;
    x = a0 * x + (double)cnt[e];
    const float x1 = (float)x;
    x = a1 * x + (double)cnt[e + 1];
    bf16x2 p = {};
    p = __builtin_amdgcn_cvt_sr_bf16_f32(p, x0, (uint32_t)t * SR_T + rj, false);
    p = __builtin_amdgcn_cvt_sr_bf16_f32(p, x1, (uint32_t)(t + 1) * SR_T + rj, true);
    w[e / 2] = __builtin_bit_cast(uint32_t, p);
  }
  if (g.xfrag) {
    // Xjt as fragments of [Np][Bp]: bins 64 s + m0 .. + 16 of column j are
    // lanes j % 32 (first 8 bins) and j % 32 + 32 of the fragment (j / 32,
    // (64 s + m0) / 16); a wave's 64 columns fill two fragments
    i32x4* xr = (i32x4*)g.Xjt + ((j >> 5) * (g.Bp / 16) + (s * 64 + m0) / 16) * 64 + (j & 31);
    xr[0] = i32x4{(int)w[0], (int)w[1], (int)w[2], (int)w[3]};
    xr[32] = i32x4{(int)w[4], (int)w[5], (int)w[6], (int)w[7]};
  } else {
    // Xjt[j][64 s + m0 .. + 16]
    i32x4* xr = (i32x4*)((__bf16*)g.Xjt + j * g.Bp + s * 64 + m0);
    xr[0] = i32x4{(int)w[0], (int)w[1], (int)w[2], (int)w[3]};
    xr[1] = i32x4{(int)w[4], (int)w[5], (int)w[6], (int)w[7]};
  }
  // Xtj through LDS
#pragma unroll
  for (int e = 0; e < 16; ++e)
    *(uint16_t*)(tile + (m0 + e) * ROWB + jj * 2) = (uint16_t)(w[e / 2] >> (16 * (e & 1)));
  __syncthreads();
  if (g.xfrag) {
    // the 2 x 4 fragments of the 64 x 64 block, each 1 KB in lane order
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int piece = tid + q * 256, f = piece >> 6, ln = piece & 63;
      const int tbl = f >> 2, kbl = f & 3;  // 32-bin and 16-column block within the block
      const i32x4 v = *(const i32x4*)(tile + (tbl * 32 + (ln & 31)) * ROWB + (kbl * 16 + 8 * (ln >> 5)) * 2);
      const int64_t frag = (s * 2 + tbl) * (g.Np / 16) + jb * 4 + kbl;
      *(i32x4*)((unsigned char*)g.Xtj + (frag * 64 + ln) * 16) = v;
    }
    return;
  }
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int piece = tid + q * 256, row = piece >> 3, c16 = piece & 7;
    __bf16* dst = (__bf16*)g.Xtj + (s * 64 + row) * g.Np + jb * 64 + c16 * 8;
    *(i32x4*)dst = *(const i32x4*)(tile + row * ROWB + c16 * 16);
  }
}

// FP8 trace: the same FP64 values, a power-of-two scale per time chunk of L
// bins (largest with max x * scale <= 448), stochastic rounding to e4m3.
// trace_16: x at bins 16g .. 16g+15 of column j in subtile s (FP64).
__device__ inline void trace_16(const ResXArgs& g, int64_t s, int64_t j, int m0, double (&xv)[16]) {
  const double a = g.tab->pw[1];
  double x = g.C64[s * g.Np + j] * g.tab->pw[m0];
  uint32_t cnt[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) cnt[e] = 0;
  for (int p = 0; p < g.planes; ++p) {
    const uint64_t mk = g.masks[((int64_t)p * g.NS + s) * g.Np + j];
    uint64_t below = (m0 == 0) ? 0ull : (mk & ((1ull << m0) - 1));
    while (below) {
      const int b = __builtin_ctzll(below);
      below &= below - 1;
      x += g.tab->pw[m0 - b - 1];
    }
    const uint32_t win = (uint32_t)((mk >> m0) & 0xffffu);
#pragma unroll
    for (int e = 0; e < 16; ++e) cnt[e] += (win >> e) & 1u;
  }
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    xv[e] = x;
    x = a * x + (double)cnt[e];
  }
}

// per-chunk maximum of the trace (as float bits; x >= 0, so integer order is float order)
__global__ __launch_bounds__(256) void k_xmax8(ResXArgs g) {
  const int64_t njb = g.Np / 64;
  const int64_t s = blockIdx.x / njb, jb = blockIdx.x % njb;
  const int tid = threadIdx.x, jj = tid & 63, gq = tid >> 6;
  double xv[16];
  trace_16(g, s, jb * 64 + jj, 16 * gq, xv);
  float m = 0.f;
#pragma unroll
  for (int e = 0; e < 16; ++e) m = fmaxf(m, (float)xv[e]);
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
  if ((tid & 63) == 0) atomicMax(&g.xmax[(s * 64) / g.L], __float_as_uint(m));
}

__global__ void k_xscale8(ResXArgs g, int64_t nchunks) {
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= nchunks) return;
  const float amax = __uint_as_float(g.xmax[c]);
  float sc = 1.f;
  if (amax > 0.f) {
    int e = 0;
    (void)frexpf(448.f / amax, &e);  // 448 / amax = f 2^e, f in [0.5, 1)
    sc = ldexpf(1.f, e - 1);
  }
  g.xscale[c] = sc;
}

__global__ __launch_bounds__(256) void k_build_x8(ResXArgs g) {
  __shared__ __align__(16) unsigned char tile[64 * 80];
  const int64_t njb = g.Np / 64;
  const int64_t s = blockIdx.x / njb, jb = blockIdx.x % njb;
  const int tid = threadIdx.x, jj = tid & 63, gq = tid >> 6;
  const int64_t j = jb * 64 + jj;
  const int m0 = 16 * gq;
  double xv[16];
  trace_16(g, s, j, m0, xv);
  const float sc = g.xscale[(s * 64) / g.L];
  const uint32_t rj = (uint32_t)j * SR_J;
  int w[4] = {0, 0, 0, 0};
  const uint32_t rt = (uint32_t)(s * 64 + m0) * SR_T + rj;
  auto q8 = [&](int e) { return fminf((float)xv[e] * sc, 448.f); };
#pragma unroll
  for (int g4 = 0; g4 < 4; ++g4) {
    const int e = 4 * g4;
    int v = 0;
    v = __builtin_amdgcn_cvt_sr_fp8_f32(q8(e), rt + (uint32_t)e * SR_T, v, 0);
    v = __builtin_amdgcn_cvt_sr_fp8_f32(q8(e + 1), rt + (uint32_t)(e + 1) * SR_T, v, 1);
    v = __builtin_amdgcn_cvt_sr_fp8_f32(q8(e + 2), rt + (uint32_t)(e + 2) * SR_T, v, 2);
    v = __builtin_amdgcn_cvt_sr_fp8_f32(q8(e + 3), rt + (uint32_t)(e + 3) * SR_T, v, 3);
    w[g4] = v;
  }
  // Xjt[j][64 s + m0 .. + 16]
  *(i32x4*)((unsigned char*)g.Xjt + j * g.Bp + s * 64 + m0) = i32x4{w[0], w[1], w[2], w[3]};
  // Xtj through LDS (rows of 64 columns)
#pragma unroll
  for (int e = 0; e < 16; ++e) tile[(m0 + e) * 80 + jj] = (unsigned char)(w[e >> 2] >> (8 * (e & 3)));
  __syncthreads();
  const int row = tid >> 2, c16 = tid & 3;
  *(i32x4*)((unsigned char*)g.Xtj + (s * 64 + row) * g.Np + jb * 64 + c16 * 16) =
      *(const i32x4*)(tile + row * 80 + c16 * 16);
}

// ------------------------------------------------------------------ NT core
// MFMA operand formats.  Both step through k in 128-byte row slices (64 BF16
// or 128 FP8 values); a lane's fragment is LB contiguous bytes of its row at
// byte offset KC * kc + LB * (lane / 32) of the slice.
struct OpBF16 {
  static constexpr int KC = 32, LB = 16;  // bytes of k per MFMA and per lane
  using frag = bf16x8;
  __device__ static frag load(const unsigned char* p) { return *(const bf16x8*)p; }
  __device__ static void mma(f32x16& c, const frag& a, const frag& b) {
    c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
};
// FA / FB: 0 = e4m3, 1 = e5m2 (the instruction's A and B format codes)
template <int FA, int FB>
struct OpF8 {
  static constexpr int KC = 64, LB = 32;
  using frag = i32x8;
  __device__ static frag load(const unsigned char* p) {
    const i32x4 lo = *(const i32x4*)p, hi = *(const i32x4*)(p + 16);
    return frag{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
  }
  __device__ static void mma(f32x16& c, const frag& a, const frag& b) {
    c = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, FA, FB, 0, 127, 0, 127);
  }
};

template <int BM, int BN, int WGM, int WGN>
struct Nt {
  static constexpr int NT = WGM * WGN * 64;
  static constexpr int WM = BM / WGM, WN = BN / WGN;   // wave tile
  static constexpr int MB = WM / 32, NB = WN / 32;     // 32x32 blocks per wave
  static constexpr int ABUF = BM * ROWB, BBUF = BN * ROWB;
  static constexpr int APT = BM * 8 / NT, BPT = BN * 8 / NT;  // 16-byte pieces per thread and step
  static constexpr size_t LDS = 2 * (size_t)(ABUF + BBUF);
  static_assert(APT >= 1 && BPT >= 1 && BM * 8 % NT == 0 && BN * 8 % NT == 0, "tile/thread mismatch");
};

// acc[a][b] += A[m0 + wave rows][kb:ke] B[n0 + wave cols][kb:ke]^T in format Op.
// A and B point at the tile's first row; lda/ldb and the k range [kb, ke) are
// in bytes, the range a multiple of 128.  atile > 0: A is stored tile-major,
// rows of lda bytes grouped in k blocks of lda bytes that lie atile bytes
// apart (byte k of row r at A + (k / lda) atile + r lda + k % lda).  awrap > 0:
// A's k repeats with that period (byte k of row r at A + r lda + k % awrap, for
// k < 2 awrap): B then holds two k blocks against the same A.  Acc element r
// of lane l of block (a, b) is row 32a + 8(r/4) + 4(l/32) + r%4, column
// 32b + l%32 of the wave tile.
template <int BM, int BN, int WGM, int WGN, typename Op>
__device__ __forceinline__ void nt_loop(const unsigned char* __restrict__ A, int64_t lda,
                                        const unsigned char* __restrict__ Bt, int64_t ldb, int64_t kb,
                                        int64_t ke, unsigned char* smem,
                                        f32x16 (&acc)[Nt<BM, BN, WGM, WGN>::MB][Nt<BM, BN, WGM, WGN>::NB],
                                        int64_t atile = 0, int64_t awrap = 0) {
  using T = Nt<BM, BN, WGM, WGN>;
  constexpr int SB = BK * 2;  // bytes per row and step
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave / WGN, wn = wave % WGN;
  const int l32 = lane & 31, hi = lane >> 5;
  unsigned char* As0 = smem;
  unsigned char* Bs0 = smem + 2 * T::ABUF;

  i32x4 ar[T::APT], br[T::BPT];
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int q = 0; q < T::APT; ++q) {
      const int piece = tid + q * T::NT, r = piece >> 3, c = piece & 7;
      const int64_t ka = atile ? (k0 / lda) * atile + k0 % lda : (awrap && k0 >= awrap ? k0 - awrap : k0);
      ar[q] = *(const i32x4*)(A + r * lda + ka + c * 16);
    }
#pragma unroll
    for (int q = 0; q < T::BPT; ++q) {
      const int piece = tid + q * T::NT, r = piece >> 3, c = piece & 7;
      br[q] = *(const i32x4*)(Bt + r * ldb + k0 + c * 16);
    }
  };
  auto lstore = [&](int buf) {
    unsigned char* As = As0 + buf * T::ABUF;
    unsigned char* Bs = Bs0 + buf * T::BBUF;
#pragma unroll
    for (int q = 0; q < T::APT; ++q) {
      const int piece = tid + q * T::NT, r = piece >> 3, c = piece & 7;
      *(i32x4*)(As + r * ROWB + c * 16) = ar[q];
    }
#pragma unroll
    for (int q = 0; q < T::BPT; ++q) {
      const int piece = tid + q * T::NT, r = piece >> 3, c = piece & 7;
      *(i32x4*)(Bs + r * ROWB + c * 16) = br[q];
    }
  };

  const int nk = (int)((ke - kb) / SB);
  if (nk <= 0) return;
  gload(kb);
  lstore(0);
  __syncthreads();
  for (int ks = 0; ks < nk; ++ks) {
    const int cur = ks & 1;
    const bool more = ks + 1 < nk;
    if (more) gload(kb + (int64_t)(ks + 1) * SB);
    const unsigned char* As = As0 + cur * T::ABUF + (wm * T::WM + l32) * ROWB + hi * Op::LB;
    const unsigned char* Bs = Bs0 + cur * T::BBUF + (wn * T::WN + l32) * ROWB + hi * Op::LB;
#pragma unroll
    for (int kc = 0; kc < SB / Op::KC; ++kc) {
      typename Op::frag af[T::MB], bv[T::NB];
#pragma unroll
      for (int a = 0; a < T::MB; ++a) af[a] = Op::load(As + a * 32 * ROWB + kc * Op::KC);
#pragma unroll
      for (int b = 0; b < T::NB; ++b) bv[b] = Op::load(Bs + b * 32 * ROWB + kc * Op::KC);
#pragma unroll
      for (int a = 0; a < T::MB; ++a)
#pragma unroll
        for (int b = 0; b < T::NB; ++b) Op::mma(acc[a][b], af[a], bv[b]);
    }
    if (more) lstore(cur ^ 1);
    __syncthreads();
  }
}

template <int MB, int NB>
__device__ __forceinline__ void zero_acc(f32x16 (&acc)[MB][NB]) {
#pragma unroll
  for (int a = 0; a < MB; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.f;
}

// ------------------------------------------------------------------ kernel U
// tile 256 bins x BI neurons; grid n_itiles * n_ttiles (neuron tile fastest).
// The bins are the MFMA row operand (A = Xtj), the neurons the column operand
// (B = J), so a lane's accumulators hold 4 consecutive bins of one neuron per
// group: the per-neuron sums over bins are mostly in-lane (then one exchange
// between the two half-waves and one across the wave rows through LDS), and W
// is staged in LDS so that each neuron's 256 bins leave as one run.
constexpr uint32_t SR_WT = 0x85EBCA6Bu, SR_WI = 0xC2B2AE35u;  // rounding bits of the FP8 weights

// The quadrature and FP64 tiers of the interval integrals, out of line: few
// intervals leave the expansion's bound, and inlined at every one of kernel
// U's unrolled call sites this code would quadruple the kernel and its
// register demand.  F and H come back in registers (as results through
// pointers they would live in the stack, written at every call site whether
// the call is taken or not).  The quadrature tier makes no call of its own,
// so that it saves nothing on entry: where it does not apply it returns NaN
// and the caller takes the FP64 tier, a second call.  q is the slot's
// quadrature half of its table, staged in LDS with the expansion's
// coefficients.
__device__ __attribute__((noinline)) float2 ev_quad_tier(const float* q, float D) {
  float F, H;
  if (glmr_ev::gl_quad_f(q, D, &F, &H)) return float2{F, H};
  return float2{__builtin_nanf(""), 0.f};
}

__device__ __attribute__((noinline)) float2 ev_fp64_tier(const double* delta, float D) {
  float F, H;
  glmr_ev::fp64_tier_f(D, *delta, &F, &H);
  return float2{F, H};
}

__device__ __forceinline__ float2 ev_rare_tier(const float* q, const double* delta, float D) {
  float2 r = ev_quad_tier(q, D);
  if (r.x != r.x) r = ev_fp64_tier(delta, D);
  return r;
}

// floats per slot of kernel U's staged table: the expansion's 16
// coefficients, then the quadrature half of the slot's table (8: delta/2,
// the nodes, the flag)
constexpr int EVTS = 24;

// one slot's staged entries from its table in memory (zero past the last slot)
__device__ __forceinline__ void stage_slot(const float* __restrict__ evgl, int64_t t, int64_t B, float* dst) {
  float4 q0 = float4{0.f, 0.f, 0.f, 0.f}, q2 = q0, q3 = q0;
  if (t < B) {
    const float4* src = (const float4*)(evgl + t * 16);
    q0 = src[0];
    q2 = src[2];
    q3 = src[3];
  }
  // past the last slot: zero length and u = 0, so F = H = 0
  float c[16];
  glmr_ev::stage_f(q0.x, q0.y, c);
  float4* o = (float4*)dst;
#pragma unroll
  for (int v = 0; v < 4; ++v) o[v] = float4{c[4 * v], c[4 * v + 1], c[4 * v + 2], c[4 * v + 3]};
  o[4] = q2;
  o[5] = q3;
}

template <int BI, int WGM, int WGN, bool F8, bool EV = false>
__device__ __forceinline__ void res_u_tile(const ResUArgs& g, int64_t itile, int64_t ttile,
                                           unsigned char* smem) {
  constexpr int BT = GLMR_TT;
  constexpr int ES = F8 ? 1 : 2;  // bytes per element
  using T = Nt<BT, BI, WGM, WGN>;
  using Op = typename std::conditional<F8, OpF8<0, 0>, OpBF16>::type;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave / WGN, wn = wave % WGN;
  const int l32 = lane & 31, hi = lane >> 5;
  const int64_t i0 = itile * BI, tl0 = ttile * BT, tt0 = g.t0 + tl0;

  f32x16 acc[T::MB][T::NB];
  zero_acc(acc);
  // J in two BF16 terms: rows [J_hi | J_lo] of 2 Np, k over both against the same trace
  const int64_t jrow = g.Np * ES, ldj = (!F8 && g.j2) ? 2 * jrow : jrow;
  nt_loop<BT, BI, WGM, WGN, Op>((const unsigned char*)g.Xtj + tt0 * g.Np * ES, g.Np * ES,
                                (const unsigned char*)g.Jc + i0 * ldj, ldj, 0, ldj, smem, acc, 0,
                                ldj != jrow ? jrow : 0);

  // W = exp(V) (0 past the last bin); sums over the wave's bins per neuron in
  // FP32 over at most 16 MB values, FP64 beyond.  The loop ended on a barrier,
  // so its LDS is free.
  constexpr int WP = BT * ES + 16;                         // staged row pitch (bytes)
  unsigned char* wl = smem;                                // [BI][WP]
  double* red = (double*)(smem + (size_t)BI * WP);         // [WGM][BI]
  const float xs_inv = F8 ? 1.f / g.xscale[0] : 1.f;
  if constexpr (EV) {
    // Event grid: W = (e^D - e^{D xi}) / D and row sums of Ei(D) - Ei(D xi)
    // (Eq. (10), (14)) in place of exp(V).  The 16 expansion coefficients of
    // each of the tile's slots are formed once into LDS (after W's staging
    // rows and the row-sum partials); a lane reads its slot's with four
    // broadcast loads and uses them for its NB neuron blocks.  Intervals
    // outside the expansion's bound take the quadrature tier from the
    // slot's staged quadrature entries, or the FP64 tier.
    static_assert(!F8, "the event grid's resident trace is BF16");
    float* ctab = (float*)(smem + (size_t)BI * WP + (size_t)WGM * BI * sizeof(double));  // [BT][EVTS]
    for (int k = tid; k < BT; k += T::NT) stage_slot(g.evgl, tt0 + k, g.B, ctab + k * EVTS);
    __syncthreads();
    float cs[T::NB];
#pragma unroll
    for (int b = 0; b < T::NB; ++b) cs[b] = 0.f;
#pragma unroll
    for (int a = 0; a < T::MB; ++a) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int tq = wm * T::WM + a * 32 + 8 * q + 4 * hi;  // first of 4 consecutive slots
        float lam[T::NB][4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          float c[16];
          const float4* src = (const float4*)(ctab + (tq + e) * EVTS);
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const float4 w = src[v];
            c[4 * v] = w.x;
            c[4 * v + 1] = w.y;
            c[4 * v + 2] = w.z;
            c[4 * v + 3] = w.w;
          }
#pragma unroll
          for (int b = 0; b < T::NB; ++b) {
            const float D = acc[a][b][4 * q + e];
            // the expansion's F joins the sum before the branch and the
            // rare tier's inside it: no value is merged across the call,
            // which would otherwise be kept in memory around it
            float E, pf, ph;
            const bool out = !glmr_ev::taylor_parts(c, D, &E, &pf, &ph);
            cs[b] = fmaf(E, out ? 0.f : pf, cs[b]);
            float H = E * ph;
            if (out) {
              // t < B: slots past it are within the bound
              const float2 r = ev_rare_tier(ctab + (tq + e) * EVTS + 16, g.evdelta + tt0 + tq + e, D);
              cs[b] += r.x;
              H = r.y;
            }
            lam[b][e] = H;
          }
        }
#pragma unroll
        for (int b = 0; b < T::NB; ++b) {
          const int il = wn * T::WN + b * 32 + l32;
          bf16x2 p0 = {(__bf16)lam[b][0], (__bf16)lam[b][1]}, p1 = {(__bf16)lam[b][2], (__bf16)lam[b][3]};
          *(uint2*)(wl + il * WP + tq * 2) =
              uint2{__builtin_bit_cast(uint32_t, p0), __builtin_bit_cast(uint32_t, p1)};
        }
      }
    }
#pragma unroll
    for (int b = 0; b < T::NB; ++b) {
      const int il = wn * T::WN + b * 32 + l32;
      double v = (double)cs[b];
      v += __shfl_xor(v, 32, 64);
      if (hi == 0) red[wm * BI + il] = v;
    }
  } else
#pragma unroll
  for (int b = 0; b < T::NB; ++b) {
    const int il = wn * T::WN + b * 32 + l32;  // neuron within the tile
    const float vs = F8 ? xs_inv / g.jscale[i0 + il] : 1.f;  // exact: powers of two
    float cs = 0.f;
#pragma unroll
    for (int a = 0; a < T::MB; ++a) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int tq = wm * T::WM + a * 32 + 8 * q + 4 * hi;  // first of 4 consecutive bins
        float lam[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          lam[e] = __expf(acc[a][b][4 * q + e] * vs);
          if (tt0 + tq + e >= g.B) lam[e] = 0.f;
          cs += lam[e];
        }
        if constexpr (F8) {
          const uint32_t r0 = (uint32_t)(tt0 + tq) * SR_WT + (uint32_t)(i0 + il) * SR_WI;
          int wv = 0;
          wv = __builtin_amdgcn_cvt_sr_bf8_f32(lam[0] * (1.f / 64.f), r0, wv, 0);
          wv = __builtin_amdgcn_cvt_sr_bf8_f32(lam[1] * (1.f / 64.f), r0 + SR_WT, wv, 1);
          wv = __builtin_amdgcn_cvt_sr_bf8_f32(lam[2] * (1.f / 64.f), r0 + 2 * SR_WT, wv, 2);
          wv = __builtin_amdgcn_cvt_sr_bf8_f32(lam[3] * (1.f / 64.f), r0 + 3 * SR_WT, wv, 3);
          *(int*)(wl + il * WP + tq) = wv;
        } else {
          bf16x2 p0 = {(__bf16)lam[0], (__bf16)lam[1]}, p1 = {(__bf16)lam[2], (__bf16)lam[3]};
          *(uint2*)(wl + il * WP + tq * 2) =
              uint2{__builtin_bit_cast(uint32_t, p0), __builtin_bit_cast(uint32_t, p1)};
        }
      }
    }
    double v = (double)cs;
    v += __shfl_xor(v, 32, 64);
    if (hi == 0) red[wm * BI + il] = v;
  }
  __syncthreads();
  // W is tile-major over the chunk: [L / 256][Np][256] (a 256-bin tile of all
  // rows is one block), so this tile's rows leave as one contiguous run and
  // kernel G reads 512 rows of a k step from one block
  static_assert(BT == 256, "W's tiles are 256 bins");
  unsigned char* __restrict__ W = (unsigned char*)g.W + ((tl0 >> 8) * g.Np + i0) * (BT * ES);
  constexpr int CPRW = BT * ES / 16;  // 16-byte pieces per staged row
#pragma unroll 4
  for (int p = tid; p < BI * CPRW; p += T::NT) {
    const int r = p / CPRW, c = p % CPRW;
    *(i32x4*)(W + r * (BT * ES) + c * 16) = *(const i32x4*)(wl + r * WP + c * 16);
  }
  for (int il = tid; il < BI; il += T::NT) {
    double v = 0.0;
#pragma unroll
    for (int q = 0; q < WGM; ++q) v += red[q * BI + il];
    g.rowpart[(tt0 / GLMR_TT) * g.Np + i0 + il] = v;
  }
}

template <int BI, int WGM, int WGN, bool F8, bool EV = false>
__global__ __launch_bounds__(WGM * WGN * 64) void k_res_u(ResUArgs g) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int64_t logical = xcd_logical(blockIdx.x, gridDim.x);
  res_u_tile<BI, WGM, WGN, F8, EV>(g, logical % g.n_itiles, logical / g.n_itiles, smem);
}

// index r with prefix[r] <= k < prefix[r + 1] (prefix ascending, prefix[0] = 0)
__device__ inline int find_rec(const int64_t* __restrict__ prefix, int n, int64_t k) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= k) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Persistent grouped kernel U: the tiles of many recordings in one queue;
// workgroup b takes tiles b', b' + grid, ... (b' its XCD-contiguous rank), so
// neighbouring tiles of one recording share an L2.  Every workgroup leaves
// once the queue is exhausted.
template <int BI, int WGM, int WGN, bool F8>
__global__ __launch_bounds__(WGM * WGN * 64) void k_res_u_group(ResUGroup q) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int64_t rank = xcd_logical(blockIdx.x, gridDim.x);
  for (int64_t base = 0; base < q.total; base += gridDim.x) {
    const int64_t k = base + rank;
    if (k >= q.total) break;
    const int r = find_rec(q.prefix, q.n, k);
    const ResUArgs g = q.args[r];
    const int64_t local = k - q.prefix[r];
    res_u_tile<BI, WGM, WGN, F8>(g, local % g.n_itiles, local / g.n_itiles, smem);
    __syncthreads();  // the next tile reuses the LDS
  }
}

// ------------------------------------------------------------------ kernel G
// tile BM x BN of (i, j) over one split of the chunk's bins; grid
// n_splits * n_itiles * n_jtiles (column tile fastest, then row tile)
template <int BM, int BN, int WGM, int WGN, bool F8>
__device__ __forceinline__ void res_g_tile(const ResGArgs& g, int64_t logical, unsigned char* smem) {
  constexpr int ES = F8 ? 1 : 2;
  using T = Nt<BM, BN, WGM, WGN>;
  using Op = typename std::conditional<F8, OpF8<1, 0>, OpBF16>::type;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave / WGN, wn = wave % WGN;
  const int l32 = lane & 31, hi = lane >> 5;
  const int64_t jtile = logical % g.n_jtiles;
  const int64_t itile = (logical / g.n_jtiles) % g.n_itiles;
  const int64_t split = logical / ((int64_t)g.n_jtiles * g.n_itiles);
  const int64_t i0 = itile * BM, j0 = jtile * BN;
  const int64_t tb = split * g.ks;
  const int64_t te = (tb + g.ks < g.Lc) ? tb + g.ks : g.Lc;

  f32x16 acc[T::MB][T::NB];
  zero_acc(acc);
  // A = W, tile-major (rows of 256 bins, tile blocks Np rows apart)
  nt_loop<BM, BN, WGM, WGN, Op>((const unsigned char*)g.W + i0 * GLMR_TT * ES, GLMR_TT * ES,
                                (const unsigned char*)g.Xjt + (j0 * g.Bp + g.t0) * ES, g.Bp * ES, tb * ES,
                                te * ES, smem, acc, g.Np * GLMR_TT * ES);

  // FP8: the weights were stored as exp(V) / 64 and the trace times its chunk scale
  const float gs = F8 ? 64.f / g.xscale[0] : 1.f;
  float* __restrict__ Gp = (float*)g.Gp + split * g.Np * g.Np;
#pragma unroll
  for (int a = 0; a < T::MB; ++a)
#pragma unroll
    for (int b = 0; b < T::NB; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int il = wm * T::WM + a * 32 + 8 * (r >> 2) + 4 * hi + (r & 3);
        const int jl = wn * T::WN + b * 32 + l32;
        Gp[(i0 + il) * g.Np + j0 + jl] = acc[a][b][r] * gs;
      }
}

template <int BM, int BN, int WGM, int WGN, bool F8>
__global__ __launch_bounds__(WGM * WGN * 64) void k_res_g(ResGArgs g) {
  extern __shared__ __align__(16) unsigned char smem[];
  res_g_tile<BM, BN, WGM, WGN, F8>(g, xcd_logical(blockIdx.x, gridDim.x), smem);
}

// Persistent grouped kernel G (same queue discipline as kernel U's).
template <int BM, int BN, int WGM, int WGN, bool F8>
__global__ __launch_bounds__(WGM * WGN * 64) void k_res_g_group(ResGGroup q) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int64_t rank = xcd_logical(blockIdx.x, gridDim.x);
  for (int64_t base = 0; base < q.total; base += gridDim.x) {
    const int64_t k = base + rank;
    if (k >= q.total) break;
    const int r = find_rec(q.prefix, q.n, k);
    const ResGArgs g = q.args[r];
    res_g_tile<BM, BN, WGM, WGN, F8>(g, k - q.prefix[r], smem);
    __syncthreads();
  }
}

// ------------------------------------------------------------------ fragment-major kernels
// BF16 on the uniform grid, with Xtj and W stored as MFMA fragments (w_elem's
// layout 2): one operand of each contraction is read by every wave straight
// from memory into registers, one coalesced 16-byte load per lane and
// fragment, and only the other operand is staged through LDS and shared by
// the workgroup's 4 waves.  Kernel U writes W in the fragment order kernel G
// reads, exchanging half-fragments between the two half-waves
// (v_permlane32_swap) so that each lane stores 8 consecutive bins.
constexpr int FB = 128;                    // neurons per tile of the LDS-staged operand
constexpr int FLDS = 2 * FB * ROWB;        // its double buffer (bytes)

// Buffer resource over [base, base + bytes) for raw buffer loads: the wave-
// uniform base sits in scalar registers, a lane's offset in one 32-bit
// register (constant over the k loop) and the k step's offset in a scalar,
// so the loop does no 64-bit address arithmetic; reads past `bytes` return 0.
// Base and size are wave-uniform by construction; reading them from the
// first lane says so to the compiler, which otherwise wraps every load in a
// loop over distinct values when they come from memory (the grouped kernels'
// per-recording arguments).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* base, int bytes) {
  const uint64_t b = (uint64_t)base;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)b);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
  void* ub = (void*)(((uint64_t)hi << 32) | lo);
  return __builtin_amdgcn_make_buffer_rsrc(ub, (short)0, __builtin_amdgcn_readfirstlane(bytes), 0x00020000);
}

__device__ __forceinline__ f32x16 mma_bf16(const i32x4& a, const i32x4& b, const f32x16& c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                 0, 0, 0);
}

// acc[a][b] += sum over the k steps [0, nk) of Afrag(a, step) Bs(b, step)^T:
// A fragments come from ga(step, regs) into registers a step ahead; B (128 rows
// by 64 k per step) from gb(step, regs) through LDS.  BFRAG: B's 16 KB of a
// step are its 4 x 4 fragments in order (row block, k block), else 128 rows of
// 128 bytes.  Acc element r of lane l of block (a, b) is row 32 a + 8 (r / 4)
// + 4 (l / 32) + r % 4 of the wave's rows, column 32 b + l % 32 of the 128
// columns.
template <int MB, bool BFRAG, typename GA, typename GB, int NT = 256>
__device__ __forceinline__ void frag_loop(int nk, GA ga, GB gb, unsigned char* smem, f32x16 (&acc)[MB][4]) {
  constexpr int PQ = 1024 / NT;  // 16-byte pieces of B per thread and step
  const int tid = threadIdx.x, lane = tid & 63;
  const int l32 = lane & 31, hi = lane >> 5;
  i32x4 an[MB][4], bn[PQ];
  auto sb = [&](int buf) {
#pragma unroll
    for (int q = 0; q < PQ; ++q) {
      const int p = tid + NT * q, r = p >> 3, c = p & 7;
      *(i32x4*)(smem + buf * (FB * ROWB) + (BFRAG ? p * 16 : r * ROWB + c * 16)) = bn[q];
    }
  };
  if (nk <= 0) return;
  ga(0, an);
  gb(0, bn);
  sb(0);
  __syncthreads();
  for (int ks = 0; ks < nk; ++ks) {
    const int cur = ks & 1;
    const bool more = ks + 1 < nk;
    i32x4 ac[MB][4];
#pragma unroll
    for (int a = 0; a < MB; ++a)
#pragma unroll
      for (int kc = 0; kc < 4; ++kc) ac[a][kc] = an[a][kc];
    if (more) {
      gb(ks + 1, bn);
      ga(ks + 1, an);
    }
    const unsigned char* Bs = smem + cur * (FB * ROWB) + (BFRAG ? lane * 16 : l32 * ROWB + hi * 16);
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) {
      i32x4 bv[4];
#pragma unroll
      for (int b = 0; b < 4; ++b)
        bv[b] = *(const i32x4*)(Bs + (BFRAG ? (b * 4 + kc) * 1024 : b * 32 * ROWB + kc * 32));
#pragma unroll
      for (int a = 0; a < MB; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = mma_bf16(ac[a][kc], bv[b], acc[a][b]);
    }
    if (more) sb(cur ^ 1);
    __syncthreads();
  }
}

// Kernel U: tile 256 bins x 128 neurons, 4 waves of 64 bins x 128 neurons.
// A = the trace's fragments (rows t), B = J's rows i0 .. i0 + 127 (k = j, the
// two-term J's 2 Np columns against the trace repeated).  Epilogue as in
// res_u_tile: W = exp(V) (0 past the last bin) and per-neuron FP64 sums over
// the tile's bins (FP32 within a lane's 32 bins); on the event grid (EV) the
// interval integrals of Eq. (10), (14) in their place, from the tile's slot
// coefficients staged in LDS.
template <bool EV>
__device__ __forceinline__ void res_uf_tile(const ResUArgs& g, int64_t itile, int64_t ttile, unsigned char* smem) {
  constexpr int MB = 2;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int l32 = lane & 31, hi = lane >> 5;
  const int64_t i0 = itile * FB, tl0 = ttile * GLMR_TT, tt0 = g.t0 + tl0;
  const int64_t kbn = g.Np / 16;                         // 16-column blocks of a trace row block
  const int64_t ldj = (g.j2 ? 2 : 1) * g.Np * 2;         // bytes per row of J
  __amdgpu_buffer_rsrc_t xr[MB];
#pragma unroll
  for (int a = 0; a < MB; ++a)
    xr[a] = buf_rsrc((const unsigned char*)g.Xtj + ((tt0 + 64 * wave) / 32 + a) * kbn * 1024, (int)(kbn * 1024));
  const __amdgpu_buffer_rsrc_t jr = buf_rsrc((const unsigned char*)g.Jc + i0 * ldj, (int)(FB * ldj));
  auto ga = [&](int ks, i32x4 (&an)[MB][4]) {
    int kb = ks * 4;
    if (kb >= kbn) kb -= (int)kbn;  // the two-term J's second half meets the same trace
#pragma unroll
    for (int a = 0; a < MB; ++a)
#pragma unroll
      for (int kc = 0; kc < 4; ++kc)
        an[a][kc] = __builtin_amdgcn_raw_buffer_load_b128(xr[a], lane * 16 + kc * 1024, kb * 1024, 0);
  };
  auto gb = [&](int ks, i32x4 (&bn)[4]) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int p = tid + 256 * q, r = p >> 3, c = p & 7;
      bn[q] = __builtin_amdgcn_raw_buffer_load_b128(jr, r * (int)ldj + c * 16, ks * 128, 0);
    }
  };
  f32x16 acc[MB][4];
  zero_acc(acc);
  frag_loop<MB, false>((int)(ldj / 128), ga, gb, smem, acc);

  // the loop ended on a barrier: its LDS holds the per-wave sums next
  double* red = (double*)smem;  // [4][FB]
  unsigned char* __restrict__ W = (unsigned char*)g.W;
  const int64_t wkb = g.L / 16;  // 16-bin blocks of a W row block
  // W's fragment stores of one 32-bin block a of neuron block b: pk[2 q + {0, 1}]
  // hold bins 8 q + 4 hi + {0, 1}, {2, 3}.  16-bin block qp holds q = 2 qp (its
  // bins 0 .. 7) and q = 2 qp + 1 (bins 8 .. 15), and a fragment lane needs 8
  // consecutive bins: the lower half-wave gets the upper half's values of
  // q = 2 qp (bins 4 .. 7), the upper half the lower half's of q = 2 qp + 1
  // (bins 8 .. 11)
  auto store_w = [&](int a, int b, const uint32_t (&pk)[8]) {
#pragma unroll
    for (int qp = 0; qp < 2; ++qp) {
      const int q0 = 2 * qp, q1 = 2 * qp + 1;
      const auto s0 = __builtin_amdgcn_permlane32_swap(pk[2 * q0], pk[2 * q1], false, false);
      const auto s1 = __builtin_amdgcn_permlane32_swap(pk[2 * q0 + 1], pk[2 * q1 + 1], false, false);
      const i32x4 v = i32x4{(int)s0[0], (int)s1[0], (int)s0[1], (int)s1[1]};
      const int64_t kb = (tl0 + 64 * wave + 32 * a) / 16 + qp;
      *(i32x4*)(W + ((((i0 >> 5) + b) * wkb + kb) * 64 + lane) * 16) = v;
    }
  };
  if constexpr (EV) {
    // W = (e^D - e^{D xi}) / D and row sums of Ei(D) - Ei(D xi): the 16
    // expansion coefficients of each of the tile's slots are formed once into
    // LDS (after the row-sum partials); a lane reads its slot's with four
    // broadcast loads and uses them for its 4 neuron blocks.  Intervals
    // outside the expansion's bound take the quadrature tier from the
    // slot's staged quadrature entries, or the FP64 tier.
    static_assert(4 * FB * sizeof(double) + GLMR_TT * EVTS * sizeof(float) <= FLDS && GLMR_TT == 256,
                  "one slot per thread, the staged table after the row-sum partials");
    float* ctab = (float*)(smem + 4 * FB * sizeof(double));  // [GLMR_TT][EVTS]
    stage_slot(g.evgl, tt0 + tid, g.B, ctab + tid * EVTS);
    __syncthreads();
    float cs[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int a = 0; a < MB; ++a) {
      uint32_t pk[4][8];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int tq = 64 * wave + 32 * a + 8 * q + 4 * hi;  // first of the lane's 4 consecutive slots
        float lam[4][4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          float c[16];
          const float4* src = (const float4*)(ctab + (tq + e) * EVTS);
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const float4 w = src[v];
            c[4 * v] = w.x;
            c[4 * v + 1] = w.y;
            c[4 * v + 2] = w.z;
            c[4 * v + 3] = w.w;
          }
          // the expansion's F joins the sums before the branch and the rare
          // tier's inside it (no value is merged across the call, which would
          // otherwise be kept in memory around it); one branch per slot
          bool out[4];
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            float E, pf, ph;
            out[b] = !glmr_ev::taylor_parts(c, acc[a][b][4 * q + e], &E, &pf, &ph);
            cs[b] = fmaf(E, out[b] ? 0.f : pf, cs[b]);
            lam[b][e] = E * ph;
          }
          if (out[0] || out[1] || out[2] || out[3]) {
#pragma unroll
            for (int b = 0; b < 4; ++b)
              if (out[b]) {
                // t < B: slots past it are within the bound
                const float2 r = ev_rare_tier(ctab + (tq + e) * EVTS + 16, g.evdelta + tt0 + tq + e,
                                              acc[a][b][4 * q + e]);
                cs[b] += r.x;
                lam[b][e] = r.y;
              }
          }
        }
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          bf16x2 p0 = {(__bf16)lam[b][0], (__bf16)lam[b][1]}, p1 = {(__bf16)lam[b][2], (__bf16)lam[b][3]};
          pk[b][2 * q] = __builtin_bit_cast(uint32_t, p0);
          pk[b][2 * q + 1] = __builtin_bit_cast(uint32_t, p1);
        }
      }
#pragma unroll
      for (int b = 0; b < 4; ++b) store_w(a, b, pk[b]);
    }
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      double v = (double)cs[b];
      v += __shfl_xor(v, 32, 64);
      if (hi == 0) red[wave * FB + b * 32 + l32] = v;
    }
  } else {
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      float cs = 0.f;
#pragma unroll
      for (int a = 0; a < MB; ++a) {
        uint32_t pk[8];  // bins 8 q + 4 hi + {0, 1} and {2, 3} for q = 0 .. 3
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int64_t t = tt0 + 64 * wave + 32 * a + 8 * q + 4 * hi;
          float lam[4];
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            lam[e] = __expf(acc[a][b][4 * q + e]);
            if (t + e >= g.B) lam[e] = 0.f;
            cs += lam[e];
          }
          bf16x2 p0 = {(__bf16)lam[0], (__bf16)lam[1]}, p1 = {(__bf16)lam[2], (__bf16)lam[3]};
          pk[2 * q] = __builtin_bit_cast(uint32_t, p0);
          pk[2 * q + 1] = __builtin_bit_cast(uint32_t, p1);
        }
        store_w(a, b, pk);
      }
      double v = (double)cs;
      v += __shfl_xor(v, 32, 64);
      if (hi == 0) red[wave * FB + b * 32 + l32] = v;
    }
  }
  __syncthreads();
  if (tid < FB) {
    const double v = red[tid] + red[FB + tid] + red[2 * FB + tid] + red[3 * FB + tid];
    g.rowpart[(tt0 / GLMR_TT) * g.Np + i0 + tid] = v;
  }
}

// two workgroups per CU: each wave within 256 registers, so that one wave's
// loads overlap the other's MFMAs on every SIMD
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_res_uf(ResUArgs g) {
  __shared__ __align__(16) unsigned char smem[FLDS];
  const int64_t logical = xcd_logical(blockIdx.x, gridDim.x);
  res_uf_tile<false>(g, logical % g.n_itiles, logical / g.n_itiles, smem);
}

// the event grid's kernel U, also two workgroups per CU: one wave's interval
// integrals overlap the other's MFMAs
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_res_uf_ev(ResUArgs g) {
  __shared__ __align__(16) unsigned char smem[FLDS];
  const int64_t logical = xcd_logical(blockIdx.x, gridDim.x);
  res_uf_tile<true>(g, logical % g.n_itiles, logical / g.n_itiles, smem);
}

// The grouped fragment-major kernels: one workgroup per tile, each
// recording's tiles split evenly over the XCDs in contiguous runs, as a
// launch of that recording alone would place them (consecutive tiles share
// an L2; every XCD meets every recording's work in turn, so tiles of uneven
// cost stay balanced).  Workgroup b is the (b / 8)-th on XCD b % 8; its
// recording r and tile follow from that XCD's prefix row.  The recording's
// arguments are read into scalar registers (the values are the same in
// every lane).  Returns false for the workgroups past the XCD's share.
template <typename A, typename Q>
__device__ __forceinline__ bool striped_tile(const Q& q, A& g, int64_t& local) {
  const int x = (int)(blockIdx.x % 8);
  const int64_t idx = blockIdx.x / 8;
  const int64_t* __restrict__ px = q.xprefix + (int64_t)x * (q.n + 1);
  if (idx >= px[q.n]) return false;
  const int r = __builtin_amdgcn_readfirstlane(find_rec(px, q.n, idx));
  const int64_t t = q.prefix[r + 1] - q.prefix[r];
  local = x * (t / 8) + (x < t % 8 ? x : t % 8) + (idx - px[r]);
  const uint32_t* src = (const uint32_t*)(q.args + r);
  uint32_t* dst = (uint32_t*)&g;
#pragma unroll
  for (int w = 0; w < (int)(sizeof(A) / 4); ++w) dst[w] = __builtin_amdgcn_readfirstlane(src[w]);
  return true;
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_res_uf_group(ResUGroup q) {
  __shared__ __align__(16) unsigned char smem[FLDS];
  ResUArgs g;
  int64_t local;
  if (!striped_tile(q, g, local)) return;
  res_uf_tile<false>(g, local % g.n_itiles, local / g.n_itiles, smem);
}

// Kernel G: tile (32 MB NW) x 128 of (i, j) over one split of the chunk's
// bins, NW waves of 32 MB rows x 128 columns.  A = W's fragments (rows i), B =
// the fragments of Xjt's rows j0 .. j0 + 127, copied to LDS as they lie and
// shared by the NW waves.
template <int MB, int NW = 4>
__device__ __forceinline__ void res_gf_tile(const ResGArgs& g, int64_t logical, unsigned char* smem) {
  constexpr int NT = 64 * NW, PQ = 1024 / NT;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int l32 = lane & 31, hi = lane >> 5;
  const int64_t jtile = logical % g.n_jtiles;
  const int64_t itile = (logical / g.n_jtiles) % g.n_itiles;
  const int64_t split = logical / ((int64_t)g.n_jtiles * g.n_itiles);
  const int64_t i0 = itile * (NW * 32 * MB), j0 = jtile * FB;
  const int64_t tb = split * g.ks;
  const int64_t te = (tb + g.ks < g.Lc) ? tb + g.ks : g.Lc;
  const int64_t wkb = g.L / 16, xkb = g.Bp / 16;
  const int span = (int)((te - tb) / 16) * 1024;  // bytes of one row block over the split
  __amdgpu_buffer_rsrc_t wr[MB], xr[4];
#pragma unroll
  for (int a = 0; a < MB; ++a)
    wr[a] = buf_rsrc((const unsigned char*)g.W + (((i0 >> 5) + MB * wave + a) * wkb + tb / 16) * 1024, span);
#pragma unroll
  for (int q = 0; q < 4; ++q)
    xr[q] = buf_rsrc((const unsigned char*)g.Xjt + (((j0 >> 5) + q) * xkb + (g.t0 + tb) / 16) * 1024, span);
  // piece p = tid + NT q of a step's 16 KB: row block p / 256 (uniform over a
  // wave), k block p / 64 % 4, lane p % 64
  const int va = lane * 16, vb = (wave & 3) * 1024 + lane * 16;
  auto ga = [&](int ks, i32x4 (&an)[MB][4]) {
#pragma unroll
    for (int a = 0; a < MB; ++a)
#pragma unroll
      for (int kc = 0; kc < 4; ++kc) an[a][kc] = __builtin_amdgcn_raw_buffer_load_b128(wr[a], va + kc * 1024, ks * 4096, 0);
  };
  auto gb = [&](int ks, i32x4 (&bn)[PQ]) {
#pragma unroll
    for (int q = 0; q < PQ; ++q) {
      const int rb = NW == 4 ? q : 2 * q + (wave >> 2);
      bn[q] = __builtin_amdgcn_raw_buffer_load_b128(xr[rb], vb, ks * 4096, 0);
    }
  };
  f32x16 acc[MB][4];
  zero_acc(acc);
  frag_loop<MB, true, decltype(ga), decltype(gb), NT>((int)((te - tb) / 64), ga, gb, smem, acc);
  float* __restrict__ Gp = (float*)g.Gp + split * g.Np * g.Np;
#pragma unroll
  for (int a = 0; a < MB; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int64_t il = i0 + 32 * MB * wave + a * 32 + 8 * (r >> 2) + 4 * hi + (r & 3);
        Gp[il * g.Np + j0 + b * 32 + l32] = acc[a][b][r];
      }
}

template <int MB, int NW = 4>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(MB == 4 || NW == 8 ? 1 : 2))) void k_res_gf(
    ResGArgs g) {
  __shared__ __align__(16) unsigned char smem[FLDS];
  res_gf_tile<MB, NW>(g, xcd_logical(blockIdx.x, gridDim.x), smem);
}

template <int MB, int NW = 4>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(MB == 4 || NW == 8 ? 1 : 2))) void
k_res_gf_group(ResGGroup q) {
  __shared__ __align__(16) unsigned char smem[FLDS];
  ResGArgs g;
  int64_t local;
  if (!striped_tile(q, g, local)) return;
  res_gf_tile<MB, NW>(g, local, smem);
}

template <typename K>
hipError_t set_lds(K kern, size_t lds) {
  return hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

template <int BI, int WGM, int WGN, bool F8, bool EV = false>
hipError_t run_u(const ResUArgs& a, hipStream_t st) {
  using T = Nt<GLMR_TT, BI, WGM, WGN>;
  const size_t epi = (size_t)BI * (GLMR_TT * (F8 ? 1 : 2) + 16) + (size_t)WGM * BI * sizeof(double) +
                     (EV ? (size_t)GLMR_TT * EVTS * sizeof(float) : 0);
  const size_t lds = T::LDS > epi ? T::LDS : epi;
  auto kern = k_res_u<BI, WGM, WGN, F8, EV>;
  hipError_t e = set_lds(kern, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3((unsigned)((int64_t)a.n_itiles * a.n_ttiles)), dim3(T::NT), lds, st, a);
  return hipGetLastError();
}

// persistent grid: as many workgroups as fit on the device at once (at least 1)
template <typename K>
unsigned persistent_grid(K kern, int threads, size_t lds, int64_t total) {
  int dev = 0, cus = 256, occ = 1;
  if (hipGetDevice(&dev) == hipSuccess) {
    hipDeviceProp_t p{};
    if (hipGetDeviceProperties(&p, dev) == hipSuccess) cus = p.multiProcessorCount;
  }
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void*)kern, threads, lds) != hipSuccess ||
      occ < 1)
    occ = 1;
  const int64_t g = (int64_t)cus * occ;
  return (unsigned)(total < g ? (total > 0 ? total : 1) : g);
}

template <int BI, int WGM, int WGN, bool F8>
hipError_t run_u_group(const ResUGroup& q, hipStream_t st) {
  using T = Nt<GLMR_TT, BI, WGM, WGN>;
  const size_t epi = (size_t)BI * (GLMR_TT * (F8 ? 1 : 2) + 16) + (size_t)WGM * BI * sizeof(double);
  const size_t lds = T::LDS > epi ? T::LDS : epi;
  auto kern = k_res_u_group<BI, WGM, WGN, F8>;
  hipError_t e = set_lds(kern, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(persistent_grid(kern, T::NT, lds, q.total)), dim3(T::NT), lds, st, q);
  return hipGetLastError();
}

template <int BM, int BN, int WGM, int WGN, bool F8>
hipError_t run_g_group(const ResGGroup& q, hipStream_t st) {
  using T = Nt<BM, BN, WGM, WGN>;
  auto kern = k_res_g_group<BM, BN, WGM, WGN, F8>;
  hipError_t e = set_lds(kern, T::LDS);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(persistent_grid(kern, T::NT, T::LDS, q.total)), dim3(T::NT), T::LDS, st, q);
  return hipGetLastError();
}

template <int BM, int BN, int WGM, int WGN, bool F8>
hipError_t run_g(const ResGArgs& a, hipStream_t st) {
  using T = Nt<BM, BN, WGM, WGN>;
  auto kern = k_res_g<BM, BN, WGM, WGN, F8>;
  hipError_t e = set_lds(kern, T::LDS);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3((unsigned)((int64_t)a.n_splits * a.n_itiles * a.n_jtiles)),
                     dim3(T::NT), T::LDS, st, a);
  return hipGetLastError();
}

template <bool EV>
hipError_t run_uf(const ResUArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(EV ? k_res_uf_ev : k_res_uf, dim3((unsigned)((int64_t)a.n_itiles * a.n_ttiles)), dim3(256), 0,
                     st, a);
  return hipGetLastError();
}

template <int MB, int NW = 4>
hipError_t run_gf(const ResGArgs& a, hipStream_t st) {
  hipLaunchKernelGGL((k_res_gf<MB, NW>), dim3((unsigned)((int64_t)a.n_splits * a.n_itiles * a.n_jtiles)),
                     dim3(64 * NW), 0, st, a);
  return hipGetLastError();
}

template <typename Q>
hipError_t striped_grid(const Q& q, unsigned* grid) {
  if (!q.xprefix || q.xgrid < 1 || q.xgrid > (int64_t(1) << 31) / 256) return hipErrorInvalidValue;
  *grid = (unsigned)q.xgrid;
  return hipSuccess;
}

hipError_t run_uf_group(const ResUGroup& q, hipStream_t st) {
  unsigned grid = 0;
  const hipError_t e = striped_grid(q, &grid);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_res_uf_group, dim3(grid), dim3(256), 0, st, q);
  return hipGetLastError();
}

template <int MB, int NW = 4>
hipError_t run_gf_group(const ResGGroup& q, hipStream_t st) {
  unsigned grid = 0;
  const hipError_t e = striped_grid(q, &grid);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_res_gf_group<MB, NW>), dim3(grid), dim3(64 * NW), 0, st, q);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_build_x(const ResXArgs& a, hipStream_t st) {
  const int64_t blocks = a.NS * (a.Np / 64);
  hipLaunchKernelGGL(k_build_x, dim3((unsigned)blocks), dim3(256), 0, st, a);
  return hipGetLastError();
}

// FP8 trace: a.xmax must hold zeros for the ceil(Bp / L) chunks on entry.
hipError_t launch_build_x8(const ResXArgs& a, hipStream_t st) {
  const int64_t blocks = a.NS * (a.Np / 64);
  const int64_t nchunks = (a.Bp + a.L - 1) / a.L;
  hipLaunchKernelGGL(k_xmax8, dim3((unsigned)blocks), dim3(256), 0, st, a);
  hipLaunchKernelGGL(k_xscale8, dim3((unsigned)((nchunks + 255) / 256)), dim3(256), 0, st, a, nchunks);
  hipLaunchKernelGGL(k_build_x8, dim3((unsigned)blocks), dim3(256), 0, st, a);
  return hipGetLastError();
}

// Tile shapes offered to the autotuner; `shape` indexes res_shapes().
// 0 .. 6: the row-major kernels (neuron tile BM x 256 bins for U, BM x BM for
// G) with their wave grids.  The 8-wave 256-neuron tiles need more than the
// 256 registers a wave may hold at two waves per SIMD once the fragments are
// FP8 (32 bytes a lane), so FP8 skips them.  7 .. 10: the fragment-major
// kernels (BF16): one kernel U, kernel G with 256, 512 or 128 rows per tile
// of 4 waves, or 512 rows of 8 waves.
const ResShape* res_shapes(int* n) {
  static const ResShape s[] = {
      {256, 256, 256, 2, 2, 1, 0, 1}, {256, 256, 256, 2, 4, 0, 0, 1}, {256, 256, 256, 4, 2, 0, 0, 1},
      {128, 128, 128, 2, 2, 1, 0, 1}, {128, 128, 128, 1, 4, 1, 0, 1}, {128, 128, 128, 4, 2, 1, 0, 1},
      {128, 128, 128, 2, 4, 1, 0, 1}, {128, 256, 128, 4, 1, 0, 1, 1}, {128, 512, 128, 4, 1, 0, 1, 0},
      {128, 128, 128, 4, 1, 0, 1, 0}, {128, 512, 128, 8, 1, 0, 1, 0},
  };
  *n = (int)(sizeof(s) / sizeof(s[0]));
  return s;
}

template <bool F8, bool EV = false>
hipError_t res_u(int shape, const ResUArgs& a, hipStream_t st) {
  switch (shape) {
    case 0: return run_u<256, 2, 2, F8, EV>(a, st);
    case 1: return run_u<256, 2, 4, F8, EV>(a, st);
    case 2: return run_u<256, 4, 2, F8, EV>(a, st);
    case 3: return run_u<128, 2, 2, F8, EV>(a, st);
    case 4: return run_u<128, 1, 4, F8, EV>(a, st);
    case 5: return run_u<128, 4, 2, F8, EV>(a, st);
    case 6: return run_u<128, 2, 4, F8, EV>(a, st);
    case 7:
    case 8:
    case 9:
    case 10: return F8 ? hipErrorInvalidValue : run_uf<EV>(a, st);
    default: return hipErrorInvalidValue;
  }
}

template <bool F8>
hipError_t res_g(int shape, const ResGArgs& a, hipStream_t st) {
  switch (shape) {
    case 0: return run_g<256, 256, 2, 2, F8>(a, st);
    case 1: return run_g<256, 256, 2, 4, F8>(a, st);
    case 2: return run_g<256, 256, 4, 2, F8>(a, st);
    case 3: return run_g<128, 128, 2, 2, F8>(a, st);
    case 4: return run_g<128, 128, 1, 4, F8>(a, st);
    case 5: return run_g<128, 128, 4, 2, F8>(a, st);
    case 6: return run_g<128, 128, 2, 4, F8>(a, st);
    case 7: return F8 ? hipErrorInvalidValue : run_gf<2>(a, st);
    case 8: return F8 ? hipErrorInvalidValue : run_gf<4>(a, st);
    case 9: return F8 ? hipErrorInvalidValue : run_gf<1>(a, st);
    case 10: return F8 ? hipErrorInvalidValue : run_gf<2, 8>(a, st);
    default: return hipErrorInvalidValue;
  }
}

template <bool F8>
hipError_t res_u_group(int shape, const ResUGroup& q, hipStream_t st) {
  switch (shape) {
    case 0: return run_u_group<256, 2, 2, F8>(q, st);
    case 1: return run_u_group<256, 2, 4, F8>(q, st);
    case 2: return run_u_group<256, 4, 2, F8>(q, st);
    case 3: return run_u_group<128, 2, 2, F8>(q, st);
    case 4: return run_u_group<128, 1, 4, F8>(q, st);
    case 5: return run_u_group<128, 4, 2, F8>(q, st);
    case 6: return run_u_group<128, 2, 4, F8>(q, st);
    case 7:
    case 8:
    case 9:
    case 10: return F8 ? hipErrorInvalidValue : run_uf_group(q, st);
    default: return hipErrorInvalidValue;
  }
}

template <bool F8>
hipError_t res_g_group(int shape, const ResGGroup& q, hipStream_t st) {
  switch (shape) {
    case 0: return run_g_group<256, 256, 2, 2, F8>(q, st);
    case 1: return run_g_group<256, 256, 2, 4, F8>(q, st);
    case 2: return run_g_group<256, 256, 4, 2, F8>(q, st);
    case 3: return run_g_group<128, 128, 2, 2, F8>(q, st);
    case 4: return run_g_group<128, 128, 1, 4, F8>(q, st);
    case 5: return run_g_group<128, 128, 4, 2, F8>(q, st);
    case 6: return run_g_group<128, 128, 2, 4, F8>(q, st);
    case 7: return F8 ? hipErrorInvalidValue : run_gf_group<2>(q, st);
    case 8: return F8 ? hipErrorInvalidValue : run_gf_group<4>(q, st);
    case 9: return F8 ? hipErrorInvalidValue : run_gf_group<1>(q, st);
    case 10: return F8 ? hipErrorInvalidValue : run_gf_group<2, 8>(q, st);
    default: return hipErrorInvalidValue;
  }
}

// Grouped kernels U / G over many recordings (one persistent launch each).
hipError_t launch_res_u_group(int shape, int fp8, const ResUGroup& q, hipStream_t st) {
  return fp8 ? res_u_group<true>(shape, q, st) : res_u_group<false>(shape, q, st);
}

hipError_t launch_res_g_group(int shape, int fp8, const ResGGroup& q, hipStream_t st) {
  return fp8 ? res_g_group<true>(shape, q, st) : res_g_group<false>(shape, q, st);
}

// Kernel U / kernel G on the resident trace, BF16 or FP8 (fp8 != 0).
hipError_t launch_res_u(int shape, int fp8, const ResUArgs& a, hipStream_t st) {
  if (a.evgl) return fp8 ? hipErrorInvalidValue : res_u<false, true>(shape, a, st);  // event grid: BF16
  return fp8 ? res_u<true>(shape, a, st) : res_u<false>(shape, a, st);
}

hipError_t launch_res_g(int shape, int fp8, const ResGArgs& a, hipStream_t st) {
  return fp8 ? res_g<true>(shape, a, st) : res_g<false>(shape, a, st);
}
