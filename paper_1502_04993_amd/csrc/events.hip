// Event grid of the continuous-time likelihood (Sec. 2.3).
//
// Between consecutive network events the potential of every neuron only
// relaxes (Eq. (8)), so the likelihood is a sum over the intervals between
// events.  The intervals are laid out as the slots of a non-uniform time
// grid: slot 0 starts at T0, slot s(k) starts at event k (k = 1..q), the last
// slot ends at T1.  An interval longer than max_gap is split by extra slots
// without a spike (splitting leaves both integrals unchanged: they are
// additive over sub-intervals); this bounds the time a run of 64 slots can
// span and with it the exponents of the per-slot decay tables below.
//
// Event k is recorded as a spike in pseudo-bin s(k) - 1, so that, exactly as
// on the regular grid, it enters the trace from the next slot on:
//   x_j[r] = sum_{events m <= r of j} e^{-(t_r - t_m)/tau}  (value right after t_r),
// and the spike ingest, carry scan and spike-term kernels of the grid apply
// unchanged once a^m and a^-(b+1) are replaced by per-slot tables relative to
// the first slot k0 of each 64-slot subtile:
//   pw[k]   = e^{-(t_k - t_k0)/tau}        (x = pw * z in the contractions)
//   ainv[k] = e^{(t_{k+1} - t_k0)/tau}     (the spike recorded at k, as seen from k0)
//   left[k] = e^{-(t_{k+1} - t_k0)/tau}    (left limit at the event of slot k + 1)
//   delta[k] = (t_{k+1} - t_k)/tau         (the interval of slot k)
//   edec[k] = e^{-delta[k]}                 (the decay over slot k)
//   asub[s] = e^{-(t_{k0+64} - t_k0)/tau}  (decay over a subtile)
// Slots past the last one have zero length (t = T1) and contribute nothing.
#include <cmath>

#include "../../include/glmrec.h"
#include "common.h"
#include "evfun.h"

namespace {

constexpr int ST = 256;  // scan block
constexpr int SPER = 8;  // elements per thread
constexpr int64_t SCH = (int64_t)ST * SPER;

__global__ void k_ev_check(EvLayoutArgs a) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < a.n;
       k += (int64_t)gridDim.x * blockDim.x) {
    const double t = a.times[k];
    const int32_t j = a.neu[k];
    bool ok = isfinite(t) && t >= a.T0 && t < a.T1 && j >= 0 && j < a.N;
    if (ok && k > 0) {
      const double tp = a.times[k - 1];
      const int32_t jp = a.neu[k - 1];
      ok = tp < t || (tp == t && jp < j);
    }
    if (!ok) {
      atomicAdd(&a.bad[0], 1ull);
      atomicMin(&a.bad[1], (unsigned long long)k);
    }
  }
}

__device__ inline int64_t slots_of_gap(double gap, double max_gap) {
  return gap > max_gap ? (int64_t)ceil(gap / max_gap) : 1;
}

__global__ void k_ev_count(EvLayoutArgs a) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < a.n;
       k += (int64_t)gridDim.x * blockDim.x) {
    const double prev = k > 0 ? a.times[k - 1] : a.T0;
    a.cnt[k] = slots_of_gap(a.times[k] - prev, a.max_gap);
  }
}

__device__ inline int64_t block_excl(int64_t v, int64_t* sh) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int off = 1; off < ST; off <<= 1) {
    const int64_t add = tid >= off ? sh[tid - off] : 0;
    __syncthreads();
    sh[tid] += add;
    __syncthreads();
  }
  const int64_t incl = sh[tid];
  __syncthreads();
  return incl - v;
}

__global__ __launch_bounds__(ST) void k_scan_blocks(const int64_t* cnt, int64_t n, int64_t* bsum) {
  __shared__ int64_t sh[ST];
  const int64_t base = (int64_t)blockIdx.x * SCH;
  int64_t v = 0;
  for (int e = 0; e < SPER; ++e) {
    const int64_t k = base + threadIdx.x * SPER + e;
    if (k < n) v += cnt[k];
  }
  const int64_t ex = block_excl(v, sh);
  if (threadIdx.x == ST - 1) bsum[blockIdx.x] = ex + v;
}

__global__ __launch_bounds__(ST) void k_scan_top(int64_t* bsum, int64_t nb) {
  __shared__ int64_t sh[ST];
  __shared__ int64_t tot;
  int64_t carry = 0;
  for (int64_t base = 0; base < nb; base += ST) {
    const int64_t k = base + threadIdx.x;
    const int64_t v = k < nb ? bsum[k] : 0;
    const int64_t ex = block_excl(v, sh);
    if (k < nb) bsum[k] = carry + ex;
    if (threadIdx.x == ST - 1) tot = ex + v;
    __syncthreads();
    carry += tot;
    __syncthreads();
  }
}

// inclusive prefix sums: slot of event k = sum_{m <= k} cnt[m]
__global__ __launch_bounds__(ST) void k_scan_apply(const int64_t* cnt, int64_t n, const int64_t* bsum,
                                                   int64_t* slot) {
  __shared__ int64_t sh[ST];
  const int64_t base = (int64_t)blockIdx.x * SCH;
  int64_t vals[SPER];
  int64_t v = 0;
  for (int e = 0; e < SPER; ++e) {
    const int64_t k = base + threadIdx.x * SPER + e;
    vals[e] = k < n ? cnt[k] : 0;
    v += vals[e];
  }
  int64_t run = block_excl(v, sh) + bsum[blockIdx.x];
  for (int e = 0; e < SPER; ++e) {
    const int64_t k = base + threadIdx.x * SPER + e;
    run += vals[e];
    if (k < n) slot[k] = run;
  }
}

// pseudo-bin of every event and the start times of its slot and of the
// spike-free slots that split the gap before it
__global__ void k_ev_place(EvLayoutArgs a) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < a.n;
       k += (int64_t)gridDim.x * blockDim.x) {
    const double t = a.times[k];
    const double prev = k > 0 ? a.times[k - 1] : a.T0;
    const int64_t s = a.slot[k];
    const int64_t nk = a.cnt[k];
    a.bins[k] = s - 1;
    a.tslot[s] = t;
    const double gap = t - prev;
    for (int64_t m = 1; m < nk; ++m) a.tslot[s - nk + m] = prev + gap * ((double)m / (double)nk);
  }
}

// slot 0, the spike-free slots after the last event, and the zero-length
// padding slots up to NS*64 (inclusive: tslot has NS*64 + 1 entries)
__global__ void k_ev_tail(EvLayoutArgs a, int64_t s_last, double t_last, int64_t n_tail) {
  const int64_t end = a.NS * 64;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx <= end;
       idx += (int64_t)gridDim.x * blockDim.x) {
    if (idx == 0) a.tslot[0] = a.T0;
    if (idx <= s_last) continue;
    const int64_t m = idx - s_last;
    a.tslot[idx] = m < n_tail ? t_last + (a.T1 - t_last) * ((double)m / (double)n_tail) : a.T1;
  }
}

__global__ void k_ev_tables(EvTableArgs a) {
  const int64_t n = a.NS * 64;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k0 = k & ~(int64_t)63;
    const double tb = a.tslot[k0], tk = a.tslot[k], tk1 = a.tslot[k + 1];
    const double r = 1.0 / a.tau;
    a.pw[k] = exp(-(tk - tb) * r);
    a.ainv[k] = exp((tk1 - tb) * r);
    a.left[k] = exp(-(tk1 - tb) * r);
    a.delta[k] = (tk1 - tk) * r;
    a.edec[k] = exp(-(tk1 - tk) * r);
    if (a.gl) {
      float o[16];
      glmr_ev::table_f((tk1 - tk) * r, o);
      float4* d = (float4*)(a.gl + k * 16);
#pragma unroll
      for (int q = 0; q < 4; ++q) d[q] = float4{o[4 * q], o[4 * q + 1], o[4 * q + 2], o[4 * q + 3]};
    }
    if (k == k0) {
      const double span = (a.tslot[k0 + 64] - tb) * r;
      a.asub[k0 / 64] = exp(-span);
      // non-negative doubles order as their bit patterns
      atomicMax(a.maxspan, (unsigned long long)__double_as_longlong(span));
    }
  }
}

int grid_of(int64_t n) {
  int64_t g = (n + 255) / 256;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return (int)g;
}

}  // namespace

int64_t ev_scan_tmp_len(int64_t n) { return (n + SCH - 1) / SCH + 2; }

hipError_t launch_ev_check(const EvLayoutArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_ev_check, dim3(grid_of(a.n)), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_ev_layout(const EvLayoutArgs& a, hipStream_t st) {
  if (a.n > 0) {
    const int64_t nb = (a.n + SCH - 1) / SCH;
    hipLaunchKernelGGL(k_ev_count, dim3(grid_of(a.n)), dim3(256), 0, st, a);
    hipLaunchKernelGGL(k_scan_blocks, dim3((unsigned)nb), dim3(ST), 0, st, a.cnt, a.n, a.scan_tmp);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(ST), 0, st, a.scan_tmp, nb);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(ST), 0, st, a.cnt, a.n, a.scan_tmp, a.slot);
  }
  return hipGetLastError();
}

hipError_t launch_ev_place(const EvLayoutArgs& a, int64_t s_last, double t_last, int64_t n_tail,
                           hipStream_t st) {
  if (a.n > 0) hipLaunchKernelGGL(k_ev_place, dim3(grid_of(a.n)), dim3(256), 0, st, a);
  hipLaunchKernelGGL(k_ev_tail, dim3(grid_of(a.NS * 64 + 1)), dim3(256), 0, st, a, s_last, t_last, n_tail);
  return hipGetLastError();
}

hipError_t launch_ev_tables(const EvTableArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_ev_tables, dim3(grid_of(a.NS * 64)), dim3(256), 0, st, a);
  return hipGetLastError();
}

// ------------------------------------------------------------ host side
double ev_resolve_max_gap(int64_t n, double T0, double T1, double max_gap) {
  return max_gap > 0 ? max_gap : 4.0 * (T1 - T0) / (double)(n + 1);
}

int64_t ev_host_slots_of_gap(double gap, double max_gap) {
  return gap > max_gap ? (int64_t)std::ceil(gap / max_gap) : 1;
}

extern "C" glmr_status glmr_event_slots(const double* times, int64_t n, double T0, double T1,
                                        double max_gap, int64_t* slots) {
  if (!slots || n < 0 || (n > 0 && !times) || !std::isfinite(T0) || !std::isfinite(T1) || !(T1 > T0) ||
      std::isnan(max_gap) || std::isinf(max_gap))
    return GLMR_EINVAL;
  const double mg = ev_resolve_max_gap(n, T0, T1, max_gap);
  if (!(mg > 0)) return GLMR_EINVAL;
  int64_t s = 0;
  double prev = T0;
  for (int64_t k = 0; k < n; ++k) {
    const double t = times[k];
    if (!std::isfinite(t) || t < prev || t >= T1 || (k == 0 && t < T0)) return GLMR_EINVAL;
    const double g = (t - prev) / mg;
    if (g > 1e9) return GLMR_EINVAL;
    s += ev_host_slots_of_gap(t - prev, mg);
    prev = t;
  }
  if ((T1 - prev) / mg > 1e9) return GLMR_EINVAL;
  s += ev_host_slots_of_gap(T1 - prev, mg);
  *slots = s;
  return GLMR_OK;
}

extern "C" void glmr_ei_interval(double D, double delta, double* F, double* H) {
  double f = 0.0, h = 0.0;
  glmr_ev::interval(D, delta, &f, &h);
  if (F) *F = f;
  if (H) *H = h;
}

extern "C" void glmr_ei_interval_f32(float D, double delta, float* F, float* H) {
  float f = 0.0f, h = 0.0f;
  glmr_ev::interval_f32(D, delta, &f, &h);
  if (F) *F = f;
  if (H) *H = h;
}
