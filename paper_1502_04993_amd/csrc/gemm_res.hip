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
#include "common.h"

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

  // round pairs of bins to BF16; w[e/2] holds bins m0+e (low half) and m0+e+1
  uint32_t w[8];
  const uint32_t rj = (uint32_t)j * SR_J;
#pragma unroll
  for (int e = 0; e < 16; e += 2) {
    const int64_t t = s * 64 + m0 + e;
    const float x0 = (float)x;
    x = a * x + (double)cnt[e];
    const float x1 = (float)x;
    x = a * x + (double)cnt[e + 1];
    bf16x2 p = {};
    p = __builtin_amdgcn_cvt_sr_bf16_f32(p, x0, (uint32_t)t * SR_T + rj, false);
    p = __builtin_amdgcn_cvt_sr_bf16_f32(p, x1, (uint32_t)(t + 1) * SR_T + rj, true);
    w[e / 2] = __builtin_bit_cast(uint32_t, p);
  }
  // Xjt[j][64 s + m0 .. + 16]
  i32x4* xr = (i32x4*)((__bf16*)g.Xjt + j * g.Bp + s * 64 + m0);
  xr[0] = i32x4{(int)w[0], (int)w[1], (int)w[2], (int)w[3]};
  xr[1] = i32x4{(int)w[4], (int)w[5], (int)w[6], (int)w[7]};
  // Xtj through LDS
#pragma unroll
  for (int e = 0; e < 16; ++e)
    *(uint16_t*)(tile + (m0 + e) * ROWB + jj * 2) = (uint16_t)(w[e / 2] >> (16 * (e & 1)));
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int piece = tid + q * 256, row = piece >> 3, c16 = piece & 7;
    __bf16* dst = (__bf16*)g.Xtj + (s * 64 + row) * g.Np + jb * 64 + c16 * 8;
    *(i32x4*)dst = *(const i32x4*)(tile + row * ROWB + c16 * 16);
  }
}

// ------------------------------------------------------------------ NT core
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

// acc[a][b] += A[m0 + wave rows][kb:ke] B[n0 + wave cols][kb:ke]^T.  A and B
// point at the tile's first row; lda/ldb are row pitches in elements; the k
// range is a multiple of BK.  Acc element r of lane l of block (a, b) is row
// 32a + 8(r/4) + 4(l/32) + r%4, column 32b + l%32 of the wave tile.
template <int BM, int BN, int WGM, int WGN>
__device__ __forceinline__ void nt_loop(const __bf16* __restrict__ A, int64_t lda,
                                        const __bf16* __restrict__ Bt, int64_t ldb, int64_t kb,
                                        int64_t ke, unsigned char* smem,
                                        f32x16 (&acc)[Nt<BM, BN, WGM, WGN>::MB][Nt<BM, BN, WGM, WGN>::NB]) {
  using T = Nt<BM, BN, WGM, WGN>;
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
      ar[q] = *(const i32x4*)(A + r * lda + k0 + c * 8);
    }
#pragma unroll
    for (int q = 0; q < T::BPT; ++q) {
      const int piece = tid + q * T::NT, r = piece >> 3, c = piece & 7;
      br[q] = *(const i32x4*)(Bt + r * ldb + k0 + c * 8);
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

  const int nk = (int)((ke - kb) / BK);
  if (nk <= 0) return;
  gload(kb);
  lstore(0);
  __syncthreads();
  for (int ks = 0; ks < nk; ++ks) {
    const int cur = ks & 1;
    const bool more = ks + 1 < nk;
    if (more) gload(kb + (int64_t)(ks + 1) * BK);
    const unsigned char* As = As0 + cur * T::ABUF + (wm * T::WM + l32) * ROWB + hi * 16;
    const unsigned char* Bs = Bs0 + cur * T::BBUF + (wn * T::WN + l32) * ROWB + hi * 16;
#pragma unroll
    for (int kc = 0; kc < BK / 16; ++kc) {
      bf16x8 af[T::MB], bv[T::NB];
#pragma unroll
      for (int a = 0; a < T::MB; ++a) af[a] = *(const bf16x8*)(As + a * 32 * ROWB + kc * 32);
#pragma unroll
      for (int b = 0; b < T::NB; ++b) bv[b] = *(const bf16x8*)(Bs + b * 32 * ROWB + kc * 32);
#pragma unroll
      for (int a = 0; a < T::MB; ++a)
#pragma unroll
        for (int b = 0; b < T::NB; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[a], bv[b], acc[a][b], 0, 0, 0);
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
// group: W is stored 8 bytes at a time and the per-neuron sums over bins are
// mostly in-lane (then one exchange between the two half-waves and one across
// the wave rows through LDS).
template <int BI, int WGM, int WGN>
__global__ __launch_bounds__(WGM * WGN * 64) void k_res_u(ResUArgs g) {
  constexpr int BT = GLMR_TT;
  using T = Nt<BT, BI, WGM, WGN>;
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave / WGN, wn = wave % WGN;
  const int l32 = lane & 31, hi = lane >> 5;
  const int64_t logical = xcd_logical(blockIdx.x, gridDim.x);
  const int64_t itile = logical % g.n_itiles, ttile = logical / g.n_itiles;
  const int64_t i0 = itile * BI, tl0 = ttile * BT, tt0 = g.t0 + tl0;

  f32x16 acc[T::MB][T::NB];
  zero_acc(acc);
  nt_loop<BT, BI, WGM, WGN>((const __bf16*)g.Xtj + tt0 * g.Np, g.Np, (const __bf16*)g.Jc + i0 * g.Np,
                            g.Np, 0, g.Np, smem, acc);

  // W = exp(V) (0 past the last bin), staged in LDS so that each neuron's 256
  // bins leave as one 512-byte run; sums over the wave's bins per neuron in
  // FP32 over at most 16 MB values, FP64 beyond.  The loop ended on a barrier,
  // so its LDS is free.
  constexpr int WP = BT * 2 + 16;                          // staged row pitch (bytes)
  unsigned char* wl = smem;                                // [BI][WP]
  double* red = (double*)(smem + (size_t)BI * WP);         // [WGM][BI]
#pragma unroll
  for (int b = 0; b < T::NB; ++b) {
    const int il = wn * T::WN + b * 32 + l32;  // neuron within the tile
    float cs = 0.f;
#pragma unroll
    for (int a = 0; a < T::MB; ++a) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int tq = wm * T::WM + a * 32 + 8 * q + 4 * hi;  // first of 4 consecutive bins
        float lam[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          lam[e] = __expf(acc[a][b][4 * q + e]);
          if (tt0 + tq + e >= g.B) lam[e] = 0.f;
          cs += lam[e];
        }
        bf16x2 p0 = {(__bf16)lam[0], (__bf16)lam[1]}, p1 = {(__bf16)lam[2], (__bf16)lam[3]};
        *(uint2*)(wl + il * WP + tq * 2) = uint2{__builtin_bit_cast(uint32_t, p0), __builtin_bit_cast(uint32_t, p1)};
      }
    }
    double v = (double)cs;
    v += __shfl_xor(v, 32, 64);
    if (hi == 0) red[wm * BI + il] = v;
  }
  __syncthreads();
  __bf16* __restrict__ W = (__bf16*)g.W;
  constexpr int CPRW = BT * 2 / 16;  // 16-byte pieces per staged row
#pragma unroll 4
  for (int p = tid; p < BI * CPRW; p += T::NT) {
    const int r = p / CPRW, c = p % CPRW;
    *(i32x4*)(W + (i0 + r) * g.L + tl0 + c * 8) = *(const i32x4*)(wl + r * WP + c * 16);
  }
  for (int il = tid; il < BI; il += T::NT) {
    double v = 0.0;
#pragma unroll
    for (int q = 0; q < WGM; ++q) v += red[q * BI + il];
    g.rowpart[(tt0 / GLMR_TT) * g.Np + i0 + il] = v;
  }
}

// ------------------------------------------------------------------ kernel G
// tile BM x BN of (i, j) over one split of the chunk's bins; grid
// n_splits * n_itiles * n_jtiles (column tile fastest, then row tile)
template <int BM, int BN, int WGM, int WGN>
__global__ __launch_bounds__(WGM * WGN * 64) void k_res_g(ResGArgs g) {
  using T = Nt<BM, BN, WGM, WGN>;
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave / WGN, wn = wave % WGN;
  const int l32 = lane & 31, hi = lane >> 5;
  const int64_t logical = xcd_logical(blockIdx.x, gridDim.x);
  const int64_t jtile = logical % g.n_jtiles;
  const int64_t itile = (logical / g.n_jtiles) % g.n_itiles;
  const int64_t split = logical / ((int64_t)g.n_jtiles * g.n_itiles);
  const int64_t i0 = itile * BM, j0 = jtile * BN;
  const int64_t tb = split * g.ks;
  const int64_t te = (tb + g.ks < g.Lc) ? tb + g.ks : g.Lc;

  f32x16 acc[T::MB][T::NB];
  zero_acc(acc);
  nt_loop<BM, BN, WGM, WGN>((const __bf16*)g.W + i0 * g.L, g.L, (const __bf16*)g.Xjt + j0 * g.Bp + g.t0,
                            g.Bp, tb, te, smem, acc);

  float* __restrict__ Gp = (float*)g.Gp + split * g.Np * g.Np;
#pragma unroll
  for (int a = 0; a < T::MB; ++a)
#pragma unroll
    for (int b = 0; b < T::NB; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int il = wm * T::WM + a * 32 + 8 * (r >> 2) + 4 * hi + (r & 3);
        const int jl = wn * T::WN + b * 32 + l32;
        Gp[(i0 + il) * g.Np + j0 + jl] = acc[a][b][r];
      }
}

template <typename K>
hipError_t set_lds(K kern, size_t lds) {
  return hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

template <int BI, int WGM, int WGN>
hipError_t run_u(const ResUArgs& a, hipStream_t st) {
  using T = Nt<GLMR_TT, BI, WGM, WGN>;
  const size_t epi = (size_t)BI * (GLMR_TT * 2 + 16) + (size_t)WGM * BI * sizeof(double);
  const size_t lds = T::LDS > epi ? T::LDS : epi;
  auto kern = k_res_u<BI, WGM, WGN>;
  hipError_t e = set_lds(kern, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3((unsigned)((int64_t)a.n_itiles * a.n_ttiles)), dim3(T::NT), lds, st, a);
  return hipGetLastError();
}

template <int BM, int BN, int WGM, int WGN>
hipError_t run_g(const ResGArgs& a, hipStream_t st) {
  using T = Nt<BM, BN, WGM, WGN>;
  auto kern = k_res_g<BM, BN, WGM, WGN>;
  hipError_t e = set_lds(kern, T::LDS);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3((unsigned)((int64_t)a.n_splits * a.n_itiles * a.n_jtiles)),
                     dim3(T::NT), T::LDS, st, a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_build_x(const ResXArgs& a, hipStream_t st) {
  const int64_t blocks = a.NS * (a.Np / 64);
  hipLaunchKernelGGL(k_build_x, dim3((unsigned)blocks), dim3(256), 0, st, a);
  return hipGetLastError();
}

// Tile shapes (neuron tile BM x 256 bins for U, BM x BM for G) and wave grids
// offered to the autotuner; `shape` indexes res_shapes().
const ResShape* res_shapes(int* n) {
  static const ResShape s[] = {
      {256, 2, 2}, {256, 2, 4}, {256, 4, 2}, {128, 2, 2}, {128, 1, 4},
  };
  *n = (int)(sizeof(s) / sizeof(s[0]));
  return s;
}

hipError_t launch_res_u(int shape, const ResUArgs& a, hipStream_t st) {
  switch (shape) {
    case 0: return run_u<256, 2, 2>(a, st);
    case 1: return run_u<256, 2, 4>(a, st);
    case 2: return run_u<256, 4, 2>(a, st);
    case 3: return run_u<128, 2, 2>(a, st);
    case 4: return run_u<128, 1, 4>(a, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_res_g(int shape, const ResGArgs& a, hipStream_t st) {
  switch (shape) {
    case 0: return run_g<256, 256, 2, 2>(a, st);
    case 1: return run_g<256, 256, 2, 4>(a, st);
    case 2: return run_g<256, 256, 4, 2>(a, st);
    case 3: return run_g<128, 128, 2, 2>(a, st);
    case 4: return run_g<128, 128, 1, 4>(a, st);
    default: return hipErrorInvalidValue;
  }
}
