// Parameter-free parts of the likelihood, computed once per kernel time
// constant tau (Sec. 2.3.3 notes dSigma needs computing only once; Sec. 2.6.1
// caches everything that does not depend on theta):
//
//  * carries C[s][j] = x_j[64 s], the trace at every subtile start, and
//    CY[s][j] = dx_j/dtau at the same bins.  Over one subtile
//      C[s+1]  = A C[s] + D[s],               A = a^64,
//      CY[s+1] = A (CY[s] + 64 c C[s]) + DY[s],  c = dt / tau^2,
//    with D[s] = sum_b a^(63-b), DY[s] = c sum_b (63-b) a^(63-b) over the
//    spikes of subtile s (the grid form of Eq. (8)/(13)).  The scan runs in
//    FP64 in three passes: local segments of 64 subtiles, a sequential pass
//    over segment aggregates, and a fix-up that adds the carried-in state
//    (after k subtiles: C += A^k C_in, CY += A^k CY_in + 64 k c A^k C_in).
//
//  * On the event grid (continuous time) the same scan runs with the per-slot
//    decays of events.hip: C[s+1] = asub[s] (C[s] + sum_b ainv[64 s + b]).
//
//  * dSigma[i][j] = sum_t s_i[t] x_j[t] (Eq. (12)) and dSigmaY[i][j] =
//    sum_t s_i[t] y_j[t] in FP64, from the spike segments: one wavefront per
//    (64 presynaptic j) x (64 postsynaptic i) x time split, lane = j, walking
//    the spikes of the i-block in bin order and advancing each lane's
//    running sum over its own mask bits; accumulators in LDS; partials per
//    split reduced in a fixed order.  On the event grid the trace at a spike of
//    i is the left limit v_j(t^-) of Eq. (12): the spike recorded at slot b is
//    weighed by left[64 s + b] = e^{-(t_{b+1} - t_k0)/tau}.
#include "common.h"

namespace {

// EV: event grid, per-subtile decays; seg[...][1] then holds the product of
// the segment's subtile decays (there is no y)
template <bool EV>
__global__ void k_carry_local(CarryArgs c) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t g = blockIdx.y;
  if (j >= c.Np) return;
  const int64_t s0 = g * c.G;
  const int64_t s1 = (s0 + c.G < c.NS) ? s0 + c.G : c.NS;
  if (EV) {
    double x = 0.0, prod = 1.0;
    for (int64_t s = s0; s < s1; ++s) {
      c.C64[s * c.Np + j] = x;
      double D = 0.0;
      for (int p = 0; p < c.planes; ++p) {
        uint64_t mk = c.masks[((int64_t)p * c.NS + s) * c.Np + j];
        while (mk) {
          const int b = __builtin_ctzll(mk);
          mk &= mk - 1;
          D += c.ev.ainv[s * 64 + b];
        }
      }
      const double A = c.ev.asub[s];
      x = A * (x + D);
      prod *= A;
    }
    c.seg[(g * c.Np + j) * 2 + 0] = x;
    c.seg[(g * c.Np + j) * 2 + 1] = prod;
    return;
  }
  const double A = c.tab->apow[1];
  double x = 0.0, y = 0.0;
  for (int64_t s = s0; s < s1; ++s) {
    c.C64[s * c.Np + j] = x;
    if (c.want_y) c.CY64[s * c.Np + j] = y;
    double D = 0.0, DY = 0.0;
    for (int p = 0; p < c.planes; ++p) {
      uint64_t mk = c.masks[((int64_t)p * c.NS + s) * c.Np + j];
      while (mk) {
        int b = __builtin_ctzll(mk);
        mk &= mk - 1;
        const double w = c.tab->pw[63 - b];
        D += w;
        DY += (double)(63 - b) * w;
      }
    }
    y = A * (y + 64.0 * c.ctau * x) + c.ctau * DY;
    x = A * x + D;
  }
  c.seg[(g * c.Np + j) * 2 + 0] = x;
  c.seg[(g * c.Np + j) * 2 + 1] = y;
}

template <bool EV>
__global__ void k_carry_scan(CarryArgs c, int64_t nseg) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= c.Np) return;
  double cin = 0.0, cyin = 0.0;
  for (int64_t g = 0; g < nseg; ++g) {
    c.segin[(g * c.Np + j) * 2 + 0] = cin;
    c.segin[(g * c.Np + j) * 2 + 1] = cyin;
    if (EV) {
      cin = c.seg[(g * c.Np + j) * 2 + 1] * cin + c.seg[(g * c.Np + j) * 2 + 0];
      continue;
    }
    const int64_t s0 = g * c.G;
    const int64_t len = (s0 + c.G < c.NS) ? c.G : c.NS - s0;
    const double AG = c.tab->apow[len];
    const double xe = c.seg[(g * c.Np + j) * 2 + 0];
    const double ye = c.seg[(g * c.Np + j) * 2 + 1];
    cyin = AG * cyin + 64.0 * (double)len * c.ctau * AG * cin + ye;
    cin = AG * cin + xe;
  }
}

template <bool EV>
__global__ void k_carry_apply(CarryArgs c) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t g = blockIdx.y;
  if (j >= c.Np) return;
  const int64_t s0 = g * c.G;
  const int64_t s1 = (s0 + c.G < c.NS) ? s0 + c.G : c.NS;
  const double cin = c.segin[(g * c.Np + j) * 2 + 0];
  const double cyin = c.segin[(g * c.Np + j) * 2 + 1];
  if (EV) {
    double Ak = 1.0;  // decay from the segment start to subtile s
    for (int64_t s = s0; s < s1; ++s) {
      const double x = c.C64[s * c.Np + j] + Ak * cin;
      c.C64[s * c.Np + j] = x;
      if (c.C32) c.C32[s * c.Np + j] = (float)x;
      Ak *= c.ev.asub[s];
    }
    return;
  }
  for (int64_t s = s0; s < s1; ++s) {
    const int64_t k = s - s0;
    const double Ak = c.tab->apow[k];
    const double x = c.C64[s * c.Np + j] + Ak * cin;
    c.C64[s * c.Np + j] = x;
    if (c.C32) c.C32[s * c.Np + j] = (float)x;
    if (c.want_y) {
      const double y = c.CY64[s * c.Np + j] + Ak * cyin + 64.0 * (double)k * c.ctau * Ak * cin;
      c.CY64[s * c.Np + j] = y;
      if (c.CY32) c.CY32[s * c.Np + j] = (float)y;
    }
  }
}

// ------------------------------------------------------------ spike term
__device__ inline int lane_bcast(int v, int l) { return __builtin_amdgcn_readlane(v, l); }
__device__ inline double lane_bcast_d(double v, int l) {
  const uint64_t u = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), l);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// EV: event grid; the trace at a spike is its left limit at the event time.
// One wave per (64 columns, RB rows, time split) owns its FP64 sums in LDS
// and takes the spikes of its rows out of the 64-row block's entry lists.
// Fewer rows per wave let more waves share a SIMD and hide each other's
// latency, but every wave walks all subtiles of its split.  Measured at
// N = 1000 (3.6e6 bins; its event grid of 24.3e6 slots, about one spike per
// 64-row block and subtile): 64 / 32 / 16 / 8 rows took 39 / 29 / 24 / 28 ms
// on the grid and 100 / 78 / 84 / 159 ms on the event grid.
template <bool EV>
constexpr int spk_rows() {
  return EV ? 32 : 16;
}

template <bool WANT_Y, bool EV>
__global__ __launch_bounds__(64) void k_spike_term(SpikeTermArgs a) {
  constexpr int RB = spk_rows<EV>();
  __shared__ double acc[RB][64];
  __shared__ double accy[WANT_Y ? RB : 1][64];
  const int lane = threadIdx.x;
  const int64_t jb = blockIdx.x, ib = blockIdx.y / (64 / RB), split = blockIdx.z;
  const int h = (int)(blockIdx.y % (64 / RB));  // the wave's rows: h RB .. h RB + RB - 1 of block ib
  const int64_t j = jb * 64 + lane;
  for (int r = 0; r < RB; ++r) {
    acc[r][lane] = 0.0;
    if (WANT_Y) accy[r][lane] = 0.0;
  }
  const int64_t per = (a.NS + a.splits - 1) / a.splits;
  const int64_t sb = split * per;
  const int64_t se = (sb + per < a.NS) ? sb + per : a.NS;
  const double ctau = a.ctau;
  // The loads of a subtile (this lane's carry and mask, the event grid's
  // slot tables, the segment's first 64 entries) are issued one subtile
  // ahead, its segment bounds two ahead, so that their latency overlaps the
  // walk of the spikes before.
  struct Pre {
    int32_t e0, e1;
    double C, CY, left, ainv;
    uint64_t m0;
    int mine;
  };
  auto bounds = [&](int64_t s) {
    const int64_t sg = s * a.NIB + ib;
    return int2{a.seg_off[sg], a.seg_off[sg + 1]};
  };
  auto fetch = [&](int64_t s, int2 eb) {
    Pre p;
    p.e0 = eb.x;
    p.e1 = eb.y;
    p.C = a.C64[s * a.Np + j];
    p.CY = WANT_Y ? a.CY64[s * a.Np + j] : 0.0;
    p.m0 = a.masks[s * a.Np + j];
    p.left = EV ? a.ev.left[s * 64 + lane] : 0.0;
    p.ainv = EV ? a.ev.ainv[s * 64 + lane] : 0.0;
    p.mine = lane < eb.y - eb.x ? (int)a.seg_ent[eb.x + lane] : 0;
    return p;
  };
  // lane b holds the factors of bin b: the decay a^b and a^-(b+1) (the event
  // grid's are per subtile)
  const double pw_grid = EV ? 0.0 : a.tab->pw[lane];
  const double ainv_grid = EV ? 0.0 : a.tab->ainv[lane];
  Pre nxt{};
  int2 eb2{0, 0};
  if (sb < se) nxt = fetch(sb, bounds(sb));
  if (sb + 1 < se) eb2 = bounds(sb + 1);
  for (int64_t s = sb; s < se; ++s) {
    const Pre cur = nxt;
    if (s + 1 < se) nxt = fetch(s + 1, eb2);
    if (s + 2 < se) eb2 = bounds(s + 2);
    const int32_t e0 = cur.e0, e1 = cur.e1;
    if (e0 == e1) continue;
    // the segment's first 64 entries, one per lane (most segments have no
    // more); the wave's own (its rows) form a uniform mask, walked in order
    // (bin order within the segment).  A segment with none of the wave's
    // rows is passed before any set-up.
    int cnt = (e1 - e0 < 64) ? e1 - e0 : 64;
    int mine = cur.mine;
    uint64_t sel = __ballot(lane < cnt && ((mine & 63) / RB) == h);
    if (sel == 0 && e1 - e0 <= 64) continue;
    // this lane's column: carry and masks of subtile s
    const double C = cur.C;
    const double CY = cur.CY;
    const uint64_t m0 = cur.m0;
    // lane b holds the decay to bin (slot) b of the subtile; a spike's bin is
    // the same for the whole wave, so its factor is broadcast from that lane
    const double pw_lane = EV ? cur.left : pw_grid;
    const double ainv_lane = EV ? cur.ainv : ainv_grid;
    // This lane's column: the first four spike bins of the subtile and their
    // factors, so that the trace at a spike's bin b is C plus those below b,
    // added in bin order, with no loop or memory access.  A column with more
    // spikes in the subtile, or several spikes in one bin (more than one
    // mask plane), takes the loop over its bits instead.
    int bt[4];
    double wt[4], ut[4];
    uint64_t mm = m0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      bt[q] = mm ? __builtin_ctzll(mm) : 64;
      mm &= mm - 1;
      // every lane takes part in the exchange (a permute reads active lanes only)
      const double w = __shfl(ainv_lane, bt[q] & 63, 64);
      wt[q] = bt[q] < 64 ? w : 0.0;
      ut[q] = (double)(bt[q] + 1) * wt[q];
    }
    bool slow = mm != 0;
    for (int p = 1; p < a.planes; ++p) slow = slow || a.masks[((int64_t)p * a.NS + s) * a.Np + j] != 0;
    // the term of one spike (entry v: bin b = v >> 6, row il = v & 63) by
    // the four registered bins
    // the running sums C, C + w0, C + w0 + w1, ... of the registered bins
    // (bt is ascending: the bins below b are a prefix of them), added in the
    // order the per-spike sum would take
    const double pre1 = C + wt[0], pre2 = pre1 + wt[1], pre3 = pre2 + wt[2], pre4 = pre3 + wt[3];
    auto fast = [&, pre1, pre2, pre3, pre4](int v, double* ty) {
      const int b = v >> 6;
      double run = C, P0 = 0.0, P1 = 0.0;
      if (WANT_Y) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const bool in = bt[q] < b;
          run += in ? wt[q] : 0.0;
          P0 += in ? wt[q] : 0.0;
          P1 += in ? ut[q] : 0.0;
        }
      } else {
        run = bt[0] < b ? pre1 : C;
        run = bt[1] < b ? pre2 : run;
        run = bt[2] < b ? pre3 : run;
        run = bt[3] < b ? pre4 : run;
      }
      const double pw = lane_bcast_d(pw_lane, b);
      if (WANT_Y) *ty = pw * (CY + (double)b * ctau * C + ctau * ((double)b * P0 - P1));
      return pw * run;
    };
    const bool wave_fast = __ballot(slow) == 0;  // uniform over the wave
    for (int32_t eb = e0; eb < e1; eb += 64) {
      if (eb != e0) {
        cnt = (e1 - eb < 64) ? e1 - eb : 64;
        mine = lane < cnt ? (int)a.seg_ent[eb + lane] : 0;
        sel = __ballot(lane < cnt && ((mine & 63) / RB) == h);
      }
      auto next = [&]() {
        const int k = __builtin_ctzll(sel);
        sel &= sel - 1;
        return lane_bcast(mine, k);
      };
      if (wave_fast) {
        // four spikes at a time: their sums are independent, so their
        // instruction chains interleave; the adds keep the spikes' order
        while (__builtin_popcountll(sel) >= 4) {
          const int v0 = next(), v1 = next(), v2 = next(), v3 = next();
          double y0 = 0.0, y1 = 0.0, y2 = 0.0, y3 = 0.0;
          const double x0 = fast(v0, &y0), x1 = fast(v1, &y1), x2 = fast(v2, &y2), x3 = fast(v3, &y3);
          atomicAdd(&acc[(v0 & 63) % RB][lane], x0);
          if (WANT_Y) atomicAdd(&accy[(v0 & 63) % RB][lane], y0);
          atomicAdd(&acc[(v1 & 63) % RB][lane], x1);
          if (WANT_Y) atomicAdd(&accy[(v1 & 63) % RB][lane], y1);
          atomicAdd(&acc[(v2 & 63) % RB][lane], x2);
          if (WANT_Y) atomicAdd(&accy[(v2 & 63) % RB][lane], y2);
          atomicAdd(&acc[(v3 & 63) % RB][lane], x3);
          if (WANT_Y) atomicAdd(&accy[(v3 & 63) % RB][lane], y3);
        }
      }
      while (sel) {
        const int v = next();
        const int il = (v & 63) % RB, b = v >> 6;
        double run = C, P0 = 0.0, P1 = 0.0;
        if (!slow) {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const bool in = bt[q] < b;
            run += in ? wt[q] : 0.0;
            if (WANT_Y) {
              P0 += in ? wt[q] : 0.0;
              P1 += in ? ut[q] : 0.0;
            }
          }
        } else {
          const uint64_t below = (1ull << b) - 1;
          for (int p = 0; p < a.planes; ++p) {
            uint64_t m = (p == 0 ? m0 : a.masks[((int64_t)p * a.NS + s) * a.Np + j]) & below;
            while (m) {
              const int bb = __builtin_ctzll(m);
              m &= m - 1;
              const double w = EV ? a.ev.ainv[s * 64 + bb] : a.tab->ainv[bb];
              run += w;
              if (WANT_Y) { P0 += w; P1 += (double)(bb + 1) * w; }
            }
          }
        }
        const double pw = lane_bcast_d(pw_lane, b);
        // LDS add without return: no wait on the sum before the next spike.
        // One wave owns the block's sums and its lanes add to distinct
        // addresses, so the order of the additions is the program order.
        atomicAdd(&acc[il][lane], pw * run);
        if (WANT_Y) atomicAdd(&accy[il][lane], pw * (CY + (double)b * ctau * C + ctau * ((double)b * P0 - P1)));
      }
    }
  }
  const int64_t i0 = ib * 64 + h * RB;
  double* out = a.part + split * a.Np * a.Np;
  for (int r = 0; r < RB; ++r) out[(i0 + r) * a.Np + j] = acc[r][lane];
  if (WANT_Y) {
    double* outy = a.part + ((int64_t)a.splits + split) * a.Np * a.Np;
    for (int r = 0; r < RB; ++r) outy[(i0 + r) * a.Np + j] = accy[r][lane];
  }
}

__global__ void k_split_reduce(const double* part, int splits, int64_t n, double* out) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x) {
    double v = 0.0;
    for (int sp = 0; sp < splits; ++sp) v += part[sp * n + k];
    out[k] = v;
  }
}

}  // namespace

hipError_t launch_carries(const CarryArgs& c, hipStream_t st) {
  const int64_t nseg = (c.NS + c.G - 1) / c.G;
  dim3 grid((unsigned)((c.Np + 255) / 256), (unsigned)nseg);
  if (c.ev.pw) {
    hipLaunchKernelGGL(k_carry_local<true>, grid, dim3(256), 0, st, c);
    hipLaunchKernelGGL(k_carry_scan<true>, dim3((unsigned)((c.Np + 63) / 64)), dim3(64), 0, st, c, nseg);
    hipLaunchKernelGGL(k_carry_apply<true>, grid, dim3(256), 0, st, c);
  } else {
    hipLaunchKernelGGL(k_carry_local<false>, grid, dim3(256), 0, st, c);
    hipLaunchKernelGGL(k_carry_scan<false>, dim3((unsigned)((c.Np + 63) / 64)), dim3(64), 0, st, c, nseg);
    hipLaunchKernelGGL(k_carry_apply<false>, grid, dim3(256), 0, st, c);
  }
  return hipGetLastError();
}

hipError_t launch_spike_term(const SpikeTermArgs& a, hipStream_t st) {
  auto grid = [&](int rb) { return dim3((unsigned)a.NIB, (unsigned)(a.NIB * (64 / rb)), (unsigned)a.splits); };
  if (a.ev.pw)
    hipLaunchKernelGGL((k_spike_term<false, true>), grid(spk_rows<true>()), dim3(64), 0, st, a);
  else if (a.CY64)
    hipLaunchKernelGGL((k_spike_term<true, false>), grid(spk_rows<false>()), dim3(64), 0, st, a);
  else
    hipLaunchKernelGGL((k_spike_term<false, false>), grid(spk_rows<false>()), dim3(64), 0, st, a);
  const int64_t n = a.Np * a.Np;
  int blocks = (int)((n + 255) / 256);
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_split_reduce, dim3(blocks), dim3(256), 0, st, a.part, a.splits, n, a.dsig);
  if (a.CY64 && a.dsigY)
    hipLaunchKernelGGL(k_split_reduce, dim3(blocks), dim3(256), 0, st, a.part + a.splits * n,
                       a.splits, n, a.dsigY);
  return hipGetLastError();
}
