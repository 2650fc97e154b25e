// Spike ingest: the raster S of Sec. 2.1 as (bin, neuron) pairs in any order
// becomes
//   * counts q_i,
//   * time-major segments: for subtile s (64 bins) and neuron block ib (64
//     neurons) the list of its spikes, entry = i_local | (b << 6), sorted so a
//     segment reads in bin order (deterministic regardless of input order),
//   * bitmask planes: bit b of masks[p][s][j] is set when neuron j fired more
//     than p times in bin 64 s + b.
// Validation: every pair must satisfy 0 <= bin < B and 0 <= neuron < N; the
// number of violations and the first violating index are reported.
#include <algorithm>

#include "common.h"

namespace {

__global__ void k_count(IngestBufs b) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < b.n;
       k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t t = b.bin[k];
    const int32_t i = b.neu[k];
    if (t < 0 || t >= b.B || i < 0 || i >= b.N) {
      atomicAdd(&b.bad[0], 1ull);
      atomicMin(&b.bad[1], (unsigned long long)k);
      continue;
    }
    const int64_t key = (t >> 6) * b.NIB + (i >> 6);
    atomicAdd(&b.cnt[key], 1);
    atomicAdd((unsigned long long*)&b.q[i], 1ull);
  }
}

// exclusive scan of cnt[0..n) into off[0..n], off[n] = total, in blocks of 4096
constexpr int SCAN_T = 1024, SCAN_PER = 4;
constexpr int SCAN_CH = SCAN_T * SCAN_PER;

__device__ int64_t block_exclusive_scan(int64_t v, int64_t* sh) {
  // Hillis-Steele in shared memory over SCAN_T values; returns exclusive prefix
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int off = 1; off < SCAN_T; off <<= 1) {
    int64_t add = tid >= off ? sh[tid - off] : 0;
    __syncthreads();
    sh[tid] += add;
    __syncthreads();
  }
  int64_t incl = sh[tid];
  __syncthreads();
  return incl - v;
}

__global__ __launch_bounds__(SCAN_T) void k_scan_blocks(const int32_t* cnt, int64_t n, int64_t* bsum) {
  __shared__ int64_t sh[SCAN_T];
  const int64_t base = (int64_t)blockIdx.x * SCAN_CH;
  int64_t v = 0;
  for (int e = 0; e < SCAN_PER; ++e) {
    int64_t k = base + threadIdx.x * SCAN_PER + e;
    if (k < n) v += cnt[k];
  }
  int64_t ex = block_exclusive_scan(v, sh);
  if (threadIdx.x == SCAN_T - 1) bsum[blockIdx.x] = ex + v;
}

__global__ __launch_bounds__(SCAN_T) void k_scan_top(int64_t* bsum, int64_t nb) {
  __shared__ int64_t sh[SCAN_T];
  int64_t carry = 0;
  for (int64_t base = 0; base < nb; base += SCAN_T) {
    int64_t k = base + threadIdx.x;
    int64_t v = k < nb ? bsum[k] : 0;
    int64_t ex = block_exclusive_scan(v, sh);
    if (k < nb) bsum[k] = carry + ex;
    __shared__ int64_t tot;
    if (threadIdx.x == SCAN_T - 1) tot = ex + v;
    __syncthreads();
    carry += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) bsum[nb] = carry;
}

__global__ __launch_bounds__(SCAN_T) void k_scan_apply(const int32_t* cnt, int64_t n, const int64_t* bsum,
                                                       int64_t nb, int32_t* off) {
  __shared__ int64_t sh[SCAN_T];
  const int64_t base = (int64_t)blockIdx.x * SCAN_CH;
  int64_t vals[SCAN_PER];
  int64_t v = 0;
  for (int e = 0; e < SCAN_PER; ++e) {
    int64_t k = base + threadIdx.x * SCAN_PER + e;
    vals[e] = k < n ? cnt[k] : 0;
    v += vals[e];
  }
  int64_t ex = block_exclusive_scan(v, sh) + bsum[blockIdx.x];
  for (int e = 0; e < SCAN_PER; ++e) {
    int64_t k = base + threadIdx.x * SCAN_PER + e;
    if (k < n) off[k] = (int32_t)ex;
    ex += vals[e];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) off[n] = (int32_t)bsum[nb];
}

__global__ void k_scatter(IngestBufs b) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < b.n;
       k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t t = b.bin[k];
    const int32_t i = b.neu[k];
    if (t < 0 || t >= b.B || i < 0 || i >= b.N) continue;
    const int64_t key = (t >> 6) * b.NIB + (i >> 6);
    const int32_t pos = b.off[key] + atomicAdd(&b.cursor[key], 1);
    b.ent[pos] = (uint16_t)((i & 63) | ((t & 63) << 6));
  }
}

// one thread per segment: insertion sort (segments hold tens of entries),
// then the longest run of equal entries = most spikes of one neuron in one bin
__global__ void k_sort(IngestBufs b) {
  const int64_t nseg = b.NS * b.NIB;
  for (int64_t sg = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; sg < nseg;
       sg += (int64_t)gridDim.x * blockDim.x) {
    const int32_t e0 = b.off[sg], e1 = b.off[sg + 1];
    for (int32_t k = e0 + 1; k < e1; ++k) {
      uint16_t v = b.ent[k];
      int32_t m = k - 1;
      while (m >= e0 && b.ent[m] > v) {
        b.ent[m + 1] = b.ent[m];
        --m;
      }
      b.ent[m + 1] = v;
    }
    int32_t best = e1 > e0 ? 1 : 0, run = 1;
    for (int32_t k = e0 + 1; k < e1; ++k) {
      run = (b.ent[k] == b.ent[k - 1]) ? run + 1 : 1;
      best = run > best ? run : best;
    }
    if (best > 1) atomicMax(b.maxmult, best);
  }
}

// one thread per segment: it alone owns the mask words of its 64 neurons
__global__ void k_masks(IngestBufs b, uint64_t* masks, int planes, int64_t Np) {
  const int64_t nseg = b.NS * b.NIB;
  for (int64_t sg = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; sg < nseg;
       sg += (int64_t)gridDim.x * blockDim.x) {
    const int64_t s = sg / b.NIB, ib = sg % b.NIB;
    const int32_t e0 = b.off[sg], e1 = b.off[sg + 1];
    int rank = 0;
    for (int32_t k = e0; k < e1; ++k) {
      const uint16_t v = b.ent[k];
      rank = (k > e0 && v == b.ent[k - 1]) ? rank + 1 : 0;
      const int il = v & 63, bb = v >> 6;
      if (rank < planes) {
        uint64_t* w = masks + ((int64_t)rank * b.NS + s) * Np + ib * 64 + il;
        *w |= 1ull << bb;
      }
    }
  }
}

int grid_for(int64_t n, int threads) {
  int64_t g = (n + threads - 1) / threads;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return (int)g;
}

}  // namespace

hipError_t launch_ingest_count(const IngestBufs& b, hipStream_t st) {
  hipLaunchKernelGGL(k_count, dim3(grid_for(b.n, 256)), dim3(256), 0, st, b);
  return hipGetLastError();
}

hipError_t launch_ingest_scan(const IngestBufs& b, hipStream_t st) {
  const int64_t n = b.NS * b.NIB;
  const int64_t nb = (n + SCAN_CH - 1) / SCAN_CH;
  hipLaunchKernelGGL(k_scan_blocks, dim3((unsigned)nb), dim3(SCAN_T), 0, st, b.cnt, n, b.scan_tmp);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(SCAN_T), 0, st, b.scan_tmp, nb);
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(SCAN_T), 0, st, b.cnt, n, b.scan_tmp, nb,
                     b.off);
  return hipGetLastError();
}

hipError_t launch_ingest_scatter(const IngestBufs& b, hipStream_t st) {
  hipLaunchKernelGGL(k_scatter, dim3(grid_for(b.n, 256)), dim3(256), 0, st, b);
  return hipGetLastError();
}

hipError_t launch_ingest_sort(const IngestBufs& b, hipStream_t st) {
  hipLaunchKernelGGL(k_sort, dim3(grid_for(b.NS * b.NIB, 256)), dim3(256), 0, st, b);
  return hipGetLastError();
}

hipError_t launch_ingest_masks(const IngestBufs& b, uint64_t* masks, int planes, int64_t Np,
                               hipStream_t st) {
  hipLaunchKernelGGL(k_masks, dim3(grid_for(b.NS * b.NIB, 256)), dim3(256), 0, st, b, masks, planes,
                     Np);
  return hipGetLastError();
}

// Digest of a raster for checkpoint matching, independent of the padding:
// the wrapping 64-bit sum over the nonzero words w of mix(w ^ mix(id + 1)),
// mix the splitmix64 finaliser and id the word's logical position (plane,
// subtile, neuron j < N; or the index of a plain array).  A sum does not
// depend on the order the threads add in, so the digest is deterministic;
// a changed word, or the same words at other positions, changes it except
// with probability ~2^-64.
namespace {
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// words p[(q * inner + s) * ld + j] for planes q < n_outer / inner, s < inner, j < cols;
// logical id (q, s, j)
__global__ __launch_bounds__(256) void k_digest(const uint64_t* __restrict__ p, int64_t n_outer, int64_t inner,
                                                int64_t ld, int64_t cols, unsigned long long* out) {
  uint64_t acc = 0;
  const int64_t n = n_outer * cols;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t a = k / cols, j = k % cols;
    const uint64_t w = p[a * ld + j];
    const uint64_t id = ((uint64_t)(a / inner) << 56) + ((uint64_t)(a % inner) << 20) + (uint64_t)j;
    if (w) acc += mix64(w ^ mix64(id + 1));
  }
  for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((threadIdx.x & 63) == 0) atomicAdd(out, (unsigned long long)acc);
}
}  // namespace

// Adds to *out the digest of n_outer rows of `cols` words (row pitch ld),
// row a being subtile a % inner of plane a / inner.
hipError_t launch_digest_u64(const uint64_t* p, int64_t n_outer, int64_t inner, int64_t ld, int64_t cols,
                             unsigned long long* out, hipStream_t st) {
  const int64_t n = n_outer * cols;
  const int64_t blocks = std::min<int64_t>(std::max<int64_t>((n + 255) / 256, 1), 4096);
  hipLaunchKernelGGL(k_digest, dim3((unsigned)blocks), dim3(256), 0, st, p, n_outer, inner, ld, cols, out);
  return hipGetLastError();
}

int64_t ingest_scan_tmp_len(int64_t nseg) { return (nseg + SCAN_CH - 1) / SCAN_CH + 2; }
