// Transmission delays (Sec. 2.4, Eq. (15)) on the regular grid: every
// connection j -> i (j != i) carries the delay of d bins, the self-connection
// i -> i the delay of d_s bins.  Row i of the model sees the presynaptic spike
// trains shifted by their delays, while its own spike terms stay at the times
// the neuron fired.
//
//  * The shared trace of all rows is that of the raster shifted by d: the
//    spike-mask words are shifted by d bits across subtiles (k_shift_masks) and
//    the carries, the resident trace and both contractions use the shifted
//    masks unchanged.  The spike segments (and q) keep the recorded bins, so
//    the spike term walks the recorded spikes of i against the shifted trace.
//  * With d_s != d the self term differs: U_i[t] needs J_ii x_i[t - d_s]
//    instead of J_ii x_i[t - d].  After kernel U, k_self_delay multiplies
//    lambda_i[t] by exp(J_ii Delta_i[t]), Delta_i[t] = x_i[t - d_s] - x_i[t - d]
//    (both from the recorded raster's masks and carries, in FP64), rewrites
//    the per-tile row sums, and adds sum_t lambda_i[t] Delta_i[t] per tile,
//    which turns kernel G's G_ii = sum_t lambda_i x_i[t - d] into the
//    integral against x_i[t - d_s].  k_self_spike adds
//    sum_{spikes of i at t} Delta_i[t] to dSigma_ii once per tau.
#include <type_traits>

#include "common.h"

namespace {

// x_j[t] of the recorded raster from its masks and carries (t < 0: 0):
//   x_j[64 s + m] = a^m (C[s][j] + sum_{b < m, spike of j in bin 64 s + b} a^-(b+1))
__device__ inline double trace_at(const DelayTrace& x, int64_t j, int64_t t) {
  if (t <= 0) return 0.0;
  const int64_t s = t >> 6;
  const int m = (int)(t & 63);
  double z = x.C[s * x.Np + j];
  const uint64_t below = m ? ((1ull << m) - 1) : 0ull;
  for (int p = 0; p < x.planes; ++p) {
    uint64_t mk = x.masks[((int64_t)p * x.NS + s) * x.Np + j] & below;
    while (mk) {
      const int b = __builtin_ctzll(mk);
      mk &= mk - 1;
      z += x.tab->ainv[b];
    }
  }
  return x.tab->pw[m] * z;
}

// spikes of neuron j in bin t of the recorded raster (t < 0: none)
__device__ inline double spikes_at(const DelayTrace& x, int64_t j, int64_t t) {
  if (t < 0) return 0.0;
  const int64_t s = t >> 6;
  const int b = (int)(t & 63);
  int n = 0;
  for (int p = 0; p < x.planes; ++p) n += (int)((x.masks[((int64_t)p * x.NS + s) * x.Np + j] >> b) & 1ull);
  return (double)n;
}

// dst bit (t) = src bit (t - d): word s of dst takes words s - q and s - q - 1
// of src, d = 64 q + r
__global__ void k_shift_masks(const uint64_t* __restrict__ src, uint64_t* __restrict__ dst, int planes,
                              int64_t NS, int64_t Np, int64_t d) {
  const int64_t q = d >> 6;
  const int r = (int)(d & 63);
  const int64_t n = (int64_t)planes * NS * Np;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = k % Np;
    const int64_t ps = k / Np;
    const int64_t s = ps % NS, p = ps / NS;
    const int64_t s1 = s - q, s2 = s - q - 1;
    const uint64_t w1 = s1 >= 0 ? src[(p * NS + s1) * Np + j] : 0ull;
    const uint64_t w2 = s2 >= 0 ? src[(p * NS + s2) * Np + j] : 0ull;
    dst[k] = r ? ((w1 << r) | (w2 >> (64 - r))) : w1;
  }
}

template <typename WT>
__device__ inline double w_load(const void* W, int64_t k) {
  return (double)((const WT*)W)[k];
}
template <typename WT>
__device__ inline void w_store(void* W, int64_t k, double v) {
  ((WT*)W)[k] = (WT)v;
}

// One bin's correction: lambda_i[t] (W[k], times a^m where the rebuild
// kernels stored it so) times exp(J_ii Delta), written back; returns lambda.
template <typename WT>
__device__ inline double self_delay_bin(const SelfDelayArgs& a, int64_t k, double jd, double delta, int m) {
  // the factor in FP64, except for BF16 weights, whose rounding (2^-9) is far
  // above the FP32 exponential's error (the FP32 mode holds L to 1e-10)
  const double c = std::is_same<WT, __bf16>::value ? (double)expf((float)(jd * delta)) : exp(jd * delta);
  double lam;
  if (a.scaled) {  // the rebuild kernels store W a^m
    const double pw = a.x.tab->pw[m];
    lam = w_load<WT>(a.W, k) / pw * c;
    w_store<WT>(a.W, k, lam * pw);
  } else {
    lam = w_load<WT>(a.W, k) * c;
    w_store<WT>(a.W, k, lam);
  }
  return lam;
}

// one wave per (neuron, tile of a.tb bins of the chunk: the row-sum tile of
// kernel U); lane = tb / 64 consecutive bins
template <typename WT>
__global__ __launch_bounds__(256) void k_self_delay(SelfDelayArgs a) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t tl0 = (int64_t)blockIdx.y * a.tb;  // chunk-local first bin of the tile
  const int64_t tt0 = a.t0 + tl0;
  const double jd = a.Jr[i * a.x.Np + i];
  const int per = a.tb >> 6;
  const double dec = a.x.tab->pw[1];  // a = e^{-dt/tau}
  double s_lam = 0.0, s_gd = 0.0;
  // the lane's bins are consecutive: the two traces at its first bin, then
  // one step of the recursion x[u + 1] = a x[u] + s[u] per bin
  const int64_t tf = tt0 + lane * per;
  double xs = trace_at(a.x, i, tf - a.ds), xd = trace_at(a.x, i, tf - a.d);
  for (int e = 0; e < per; ++e) {
    const int tl = lane * per + e;
    const int64_t t = tt0 + tl;
    const double delta = xs - xd;
    xs = dec * xs + spikes_at(a.x, i, t - a.ds);
    xd = dec * xd + spikes_at(a.x, i, t - a.d);
    if (t >= a.B) continue;
    const int64_t tc = tl0 + tl;  // chunk-local bin
    const double lam = self_delay_bin<WT>(a, w_elem(a.tiled, i, tc, a.x.Np, a.L), jd, delta, tl & 63);
    s_lam += lam;
    s_gd += lam * delta;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    s_lam += __shfl_xor(s_lam, off, 64);
    s_gd += __shfl_xor(s_gd, off, 64);
  }
  if (lane == 0) {
    a.rowpart[(tt0 / a.tb) * a.x.Np + i] = s_lam;
    a.gpart[(tt0 / a.tb) * a.x.Np + i] = s_gd;
  }
}

// The same with W as MFMA fragments (layout 2, 256-bin row-sum tiles): one
// wave per (32-neuron block, 256-bin tile), lane l on neuron l % 32 of the
// block and the tile's bins 128 (l / 32) .. + 128 in order.  At each bin the
// 32 lanes of a half-wave touch one 512-byte run of W (their fragment slots),
// where a wave per neuron would touch 16-byte pieces 512 bytes apart.
template <typename WT>
__global__ __launch_bounds__(256) void k_self_delay_frag(SelfDelayArgs a) {
  const int lane = threadIdx.x & 63;
  const int64_t i = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 32 + (lane & 31);
  const int64_t tile0 = (int64_t)blockIdx.y * 256;       // chunk-local first bin of the tile
  const int64_t tl0 = tile0 + 128 * (lane >> 5);         // the lane's first bin
  const double jd = a.Jr[i * a.x.Np + i];
  const double dec = a.x.tab->pw[1];
  double s_lam = 0.0, s_gd = 0.0;
  double xs = trace_at(a.x, i, a.t0 + tl0 - a.ds), xd = trace_at(a.x, i, a.t0 + tl0 - a.d);
  for (int e = 0; e < 128; ++e) {
    const int64_t t = a.t0 + tl0 + e;
    const double delta = xs - xd;
    xs = dec * xs + spikes_at(a.x, i, t - a.ds);
    xd = dec * xd + spikes_at(a.x, i, t - a.d);
    if (t >= a.B) continue;
    const double lam = self_delay_bin<WT>(a, w_elem(2, i, tl0 + e, a.x.Np, a.L), jd, delta, (int)(t & 63));
    s_lam += lam;
    s_gd += lam * delta;
  }
  s_lam += __shfl_xor(s_lam, 32, 64);
  s_gd += __shfl_xor(s_gd, 32, 64);
  if (lane < 32) {
    const int64_t row = (a.t0 + tile0) / 256;
    a.rowpart[row * a.x.Np + i] = s_lam;
    a.gpart[row * a.x.Np + i] = s_gd;
  }
}

// dSigma_ii += sum_{spikes of i at t} Delta_i[t]: one wave per (64-neuron
// block, split of the subtiles), lane = neuron of the block; partials per split
__global__ __launch_bounds__(64) void k_self_spike(SelfSpikeArgs a) {
  const int lane = threadIdx.x;
  const int64_t ib = blockIdx.x, split = blockIdx.y;
  const int64_t per = (a.x.NS + a.splits - 1) / a.splits;
  const int64_t sb = split * per;
  const int64_t se = (sb + per < a.x.NS) ? sb + per : a.x.NS;
  const int64_t i = ib * 64 + lane;
  double acc = 0.0;
  for (int64_t s = sb; s < se; ++s) {
    const int64_t sg = s * a.NIB + ib;
    const int32_t e0 = a.seg_off[sg], e1 = a.seg_off[sg + 1];
    for (int32_t e = e0; e < e1; ++e) {
      const int v = a.seg_ent[e];
      if ((v & 63) != lane) continue;
      const int64_t t = s * 64 + (v >> 6);
      acc += trace_at(a.x, i, t - a.ds) - trace_at(a.x, i, t - a.d);
    }
  }
  a.part[split * a.x.Np + i] = acc;
}

__global__ void k_self_spike_sum(SelfSpikeArgs a) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= a.x.Np) return;
  double v = 0.0;
  for (int sp = 0; sp < a.splits; ++sp) v += a.part[sp * a.x.Np + i];
  a.dsig[i * a.x.Np + i] += v;
}

int grid_of(int64_t n) {
  int64_t g = (n + 255) / 256;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return (int)g;
}

}  // namespace

hipError_t launch_shift_masks(const uint64_t* src, uint64_t* dst, int planes, int64_t NS, int64_t Np,
                              int64_t d, hipStream_t st) {
  hipLaunchKernelGGL(k_shift_masks, dim3(grid_of((int64_t)planes * NS * Np)), dim3(256), 0, st, src, dst,
                     planes, NS, Np, d);
  return hipGetLastError();
}

hipError_t launch_self_delay(const SelfDelayArgs& a, hipStream_t st) {
  if ((a.tb != 128 && a.tb != 256) || a.Lc % a.tb) return hipErrorInvalidValue;
  if (a.tiled == 2) {
    if (a.tb != 256 || a.x.Np % 128 || a.wtype != 2 || a.scaled) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_self_delay_frag<__bf16>, dim3((unsigned)(a.x.Np / 128), (unsigned)(a.Lc / 256)), dim3(256),
                       0, st, a);
    return hipGetLastError();
  }
  dim3 grid((unsigned)(a.x.Np / 4), (unsigned)(a.Lc / a.tb));
  switch (a.wtype) {
    case 0: hipLaunchKernelGGL(k_self_delay<double>, grid, dim3(256), 0, st, a); break;
    case 1: hipLaunchKernelGGL(k_self_delay<float>, grid, dim3(256), 0, st, a); break;
    case 2: hipLaunchKernelGGL(k_self_delay<__bf16>, grid, dim3(256), 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_self_spike(const SelfSpikeArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_self_spike, dim3((unsigned)a.NIB, (unsigned)a.splits), dim3(64), 0, st, a);
  hipLaunchKernelGGL(k_self_spike_sum, dim3((unsigned)((a.x.Np + 255) / 256)), dim3(256), 0, st, a);
  return hipGetLastError();
}
