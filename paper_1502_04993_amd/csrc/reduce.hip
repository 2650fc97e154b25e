// FP64 reductions and assembly of the likelihood and gradient, parameter
// preparation, and the per-row L-BFGS ascent.
//
// Assembly (per postsynaptic row i, all in FP64, fixed summation order):
//   spike term    L^Sigma_i = q_i mu_i + sum_j J_ij dSigma_ij   (U is linear in
//                 theta at fixed tau, so Eq. (7)'s first term follows from the
//                 parameter-free dSigma of Eq. (12))
//   integral term L^int_i   = dt e^{mu_i} sum_t W[i][t]
//   L_i = L^Sigma_i - L^int_i,   dL/dmu_i = q_i - L^int_i   (Sec. 2.3.3)
//   dL/dJ_ij = dSigma_ij - dt e^{mu_i} G_ij
//   dL/dtau  = sum_i [ sum_j J_ij dSigmaY_ij - dt e^{mu_i} sum_t W[i][t] V[i][t] ]
//
// Ascent: every row theta_i = (mu_i, J_i.) is its own concave problem
// (Sec. 2.2); the rows run L-BFGS on f_i = -L_i side by side, each with its own
// history, step length and stopping test eta_i = |f_i^k - f_i^(k-1)| / |f_i^k|
// (the fractional-change criterion of Sec. 2.6.3).  One workgroup per row.
#include "common.h"

namespace {

constexpr int RT = 256;  // threads per row-workgroup

// fixed-order block sum of one double per thread
__device__ double block_sum(double v, double* sh) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int off = RT / 2; off > 0; off >>= 1) {
    if (tid < off) sh[tid] += sh[tid + off];
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}

// four consecutive entries a thread (16-byte loads; n is a multiple of 4),
// each summed over the splits in split order
__global__ void k_gp_reduce_f(const float* Gp, int n_splits, int64_t n, double* G, int first) {
  const int64_t n4 = n / 4;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n4;
       k += (int64_t)gridDim.x * blockDim.x) {
    double4 v = first ? double4{0.0, 0.0, 0.0, 0.0} : ((const double4*)G)[k];
    for (int s = 0; s < n_splits; ++s) {
      const float4 p = ((const float4*)(Gp + s * n))[k];
      v.x += (double)p.x;
      v.y += (double)p.y;
      v.z += (double)p.z;
      v.w += (double)p.w;
    }
    ((double4*)G)[k] = v;
  }
}
__global__ void k_gp_reduce_d(const double* Gp, int n_splits, int64_t n, double* G, int first) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x) {
    double v = first ? 0.0 : G[k];
    for (int s = 0; s < n_splits; ++s) v += Gp[s * n + k];
    G[k] = v;
  }
}

// rowpart[tile][i]: two passes, splits over tiles then a fixed-order merge
constexpr int RP_SPLITS = 64;
__global__ void k_rowpart_a(const double* rp, int64_t n_tiles, int64_t Np, double* tmp) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t sp = blockIdx.y;
  if (i >= Np) return;
  const int64_t per = (n_tiles + RP_SPLITS - 1) / RP_SPLITS;
  const int64_t t0 = sp * per, t1 = (t0 + per < n_tiles) ? t0 + per : n_tiles;
  double v = 0.0;
  for (int64_t t = t0; t < t1; ++t) v += rp[t * Np + i];
  tmp[sp * Np + i] = v;
}
__global__ void k_rowpart_b(const double* tmp, int64_t Np, double* out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= Np) return;
  double v = 0.0;
  for (int sp = 0; sp < RP_SPLITS; ++sp) v += tmp[sp * Np + i];
  out[i] = v;
}

__global__ __launch_bounds__(RT) void k_assemble(AssembleArgs a) {
  __shared__ double sh[RT];
  const int64_t i = blockIdx.x;
  const int tid = threadIdx.x;
  const double* Jr = a.Jr + i * a.Np;
  const double* ds = a.dsig + i * a.Np;
  double v = 0.0, vy = 0.0;
  for (int64_t j = tid; j < a.N; j += RT) {
    v += Jr[j] * ds[j];
    if (a.dsigY) vy += Jr[j] * a.dsigY[i * a.Np + j];
  }
  const double dot = block_sum(v, sh);
  const double doty = a.dsigY ? block_sum(vy, sh) : 0.0;
  const double sc = a.dt * a.rowscale[i];
  const double integ = sc * a.rowsum[i];
  if (tid == 0) {
    const double spike = (double)a.q[i] * a.mu[i] + dot;
    a.ll_rows[i] = spike - integ;
    if (a.gmu) a.gmu[i] = (double)a.q[i] - integ;
    if (a.tau_rows) a.tau_rows[i] = doty - (a.rowsumV ? sc * a.rowsumV[i] : 0.0);
  }
  if (a.gJ) {
    for (int64_t j = tid; j < a.Np; j += RT)
      a.gJ[i * a.Np + j] =
          (j < a.N) ? ds[j] - sc * (a.G64[i * a.Np + j] + ((a.gself && j == i) ? a.gself[i] : 0.0)) : 0.0;
  }
}

__global__ __launch_bounds__(RT) void k_sum_rows(const double* v, int n, double* out) {
  __shared__ double sh[RT];
  // Neumaier-compensated per-thread partials, then a fixed tree
  double s = 0.0, c = 0.0;
  for (int k = threadIdx.x; k < n; k += RT) {
    double x = v[k], t = s + x;
    c += (fabs(s) >= fabs(x)) ? (s - t) + x : (x - t) + s;
    s = t;
  }
  double tot = block_sum(s + c, sh);
  if (threadIdx.x == 0) out[0] = tot;
}

template <typename T> __device__ inline T to_prec(double x);
template <> __device__ inline double to_prec<double>(double x) { return x; }
template <> __device__ inline float to_prec<float>(double x) { return (float)x; }
template <> __device__ inline __bf16 to_prec<__bf16>(double x) { return (__bf16)(float)x; }

template <typename T>
__global__ void k_prepare(int N, int64_t Np, const double* J64, const double* mu, T* Jc, double* Jr,
                          double* rowscale) {
  const int64_t n = Np * Np;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = k / Np, j = k % Np;
    const double v = (i < N && j < N) ? J64[k] : 0.0;
    const T c = to_prec<T>(v);
    Jc[k] = c;
    Jr[k] = (double)c;
    if (j == 0) rowscale[i] = (i < N) ? exp(mu[i]) : 0.0;
  }
}

__global__ void k_prepare_f32u(int N, int64_t Np, const double* J64, const double* mu, double* Jc,
                               double* Jr, double* rowscale) {
  const int64_t n = Np * Np;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = k / Np, j = k % Np;
    const double v = (i < N && j < N) ? (double)(float)J64[k] : 0.0;
    Jc[k] = v;
    Jr[k] = v;
    if (j == 0) rowscale[i] = (i < N) ? exp(mu[i]) : 0.0;
  }
}

// BF16 with J in two terms: row i of Jc is [bf16(J_i.) | bf16(J_i. - bf16(J_i.))]
// (pitch 2 Np); Jr holds their exact sum, the value the likelihood is of.
__global__ void k_prepare_j2(int N, int64_t Np, const double* J64, const double* mu, __bf16* Jc, double* Jr,
                             double* rowscale) {
  const int64_t n = Np * Np;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = k / Np, j = k % Np;
    const double v = (i < N && j < N) ? J64[k] : 0.0;
    const __bf16 hi = to_prec<__bf16>(v);
    const __bf16 lo = to_prec<__bf16>(v - (double)hi);
    Jc[i * 2 * Np + j] = hi;
    Jc[i * 2 * Np + Np + j] = lo;
    Jr[k] = (double)hi + (double)lo;
    if (j == 0) rowscale[i] = (i < N) ? exp(mu[i]) : 0.0;
  }
}

// FP8: row i of J times the power-of-two scale 2^floor(log2(448 / max_j |J_ij|)),
// rounded to the nearest OCP e4m3 value; Jr holds the value actually used.
// One 256-thread block per row.
__global__ __launch_bounds__(256) void k_prepare_f8(int N, int64_t Np, const double* J64, const double* mu,
                                                    unsigned char* Jc, double* Jr, double* rowscale,
                                                    float* jscale) {
  __shared__ float red[256];
  const int64_t i = blockIdx.x;
  float m = 0.f;
  for (int64_t j = threadIdx.x; j < Np; j += 256)
    if (i < N && j < N) m = fmaxf(m, fabsf((float)J64[i * Np + j]));
  red[threadIdx.x] = m;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  const float amax = red[0];
  float sc = 1.f;
  if (amax > 0.f) {
    int e = 0;
    (void)frexpf(448.f / amax, &e);
    sc = ldexpf(1.f, e - 1);
  }
  for (int64_t j = threadIdx.x; j < Np; j += 256) {
    const float v = (i < N && j < N) ? (float)J64[i * Np + j] * sc : 0.f;
    const int q = __builtin_amdgcn_cvt_pk_fp8_f32(v, v, 0, false) & 0xff;
    Jc[i * Np + j] = (unsigned char)q;
    Jr[i * Np + j] = (double)__builtin_amdgcn_cvt_f32_fp8(q, 0) / (double)sc;
  }
  if (threadIdx.x == 0) {
    jscale[i] = sc;
    rowscale[i] = (i < N) ? exp(mu[i]) : 0.0;
  }
}

__global__ void k_copy_out(const double* src, int64_t ld, double* dst, int rows, int cols) {
  const int64_t n = (int64_t)rows * cols;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = k / cols, c = k % cols;
    dst[k] = src[r * ld + c];
  }
}

// ------------------------------------------------------------------ ascent
__global__ void k_pack_theta(int N, int64_t Np, int P, const double* theta, double* J64, double* mu) {
  const int64_t n = Np * Np;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = k / Np, j = k % Np;
    J64[k] = (i < N && j < N) ? theta[i * P + 1 + j] : 0.0;
    if (j == 0) mu[i] = (i < N) ? theta[i * P] : 0.0;
  }
}

__global__ void k_unpack_theta(int N, int64_t Np, int P, const double* J64, const double* mu,
                               double* theta) {
  const int64_t n = (int64_t)N * P;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = k / P, c = k % P;
    theta[k] = (c == 0) ? mu[i] : J64[i * Np + c - 1];
  }
}

__global__ void k_pack_grad(int N, int64_t Np, int P, const double* gJ, const double* gmu,
                            const double* ll_rows, double* g, double* f) {
  const int64_t n = (int64_t)N * P;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = k / P, c = k % P;
    g[k] = (c == 0) ? -gmu[i] : -gJ[i * Np + c - 1];
    if (c == 0) f[i] = -ll_rows[i];
  }
}

// Bounds of component c of a row (c = 0: mu, else J): [lo, hi]
__device__ inline void comp_bounds(const AscentArgs& a, int c, double* lo, double* hi) {
  if (c == 0) {
    *lo = a.mu_lo;
    *hi = a.mu_hi;
  } else if (a.jmax > 0) {
    *lo = -a.jmax;
    *hi = a.jmax;
  } else {
    *lo = -INFINITY;
    *hi = INFINITY;
  }
}

// Gradient of f = -L with the steps that would leave the box removed: a
// component at its lower bound with g > 0, or at its upper bound with g < 0,
// cannot move along -g.
__device__ inline double proj_grad(const AscentArgs& a, int c, double th, double gv) {
  double lo, hi;
  comp_bounds(a, c, &lo, &hi);
  if ((th <= lo && gv > 0.0) || (th >= hi && gv < 0.0)) return 0.0;
  return gv;
}

// f += alpha sum_{j != i} sqrt(J_ij^2 + eps), g_J += alpha J / sqrt(J^2 + eps)
// (Eq. (16)-(17); the self-connection is not penalised).  One block per row.
__global__ __launch_bounds__(RT) void k_penalty(AscentArgs a, const double* theta, double* g, double* f) {
  __shared__ double sh[RT];
  const int64_t i = blockIdx.x;
  const int P = a.P;
  const double* th = theta + i * P;
  double* gi = g + i * P;
  double v = 0.0;
  for (int c = 1 + threadIdx.x; c < P; c += RT) {
    if (c - 1 == i) continue;
    const double J = th[c], r = sqrt(J * J + a.eps);
    v += r;
    gi[c] += a.alpha * J / r;
  }
  v = block_sum(v, sh);
  if (threadIdx.x == 0) f[i] += a.alpha * v;
}

__global__ void k_project_theta(AscentArgs a, double* theta) {
  const int64_t n = (int64_t)a.N * a.P;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x) {
    double lo, hi;
    comp_bounds(a, (int)(k % a.P), &lo, &hi);
    theta[k] = fmin(fmax(theta[k], lo), hi);
  }
}

// two-loop recursion for row i (f = -L, so d is a descent direction of f)
__global__ __launch_bounds__(RT) void k_lbfgs_dir(AscentArgs a, int async) {
  __shared__ double sh[RT];
  __shared__ double alpha[64];
  const int64_t i = blockIdx.x;
  const int tid = threadIdx.x;
  const int P = a.P;
  const int64_t rs = (int64_t)a.N * P;  // history slot stride
  double* d = a.d + i * P;
  const double* g = a.g + i * P;
  if (async && a.state[i] == 0 && a.accepted[i] != 3) return;  // mid-search: keep d and step
  if (a.state[i] != 0) {
    for (int c = tid; c < P; c += RT) d[c] = 0.0;
    if (tid == 0) a.gd[i] = 0.0;
    return;
  }
  const int len = a.hist_len[i], head = a.hist_head[i];
  const double* th = a.theta + i * P;
  for (int c = tid; c < P; c += RT) d[c] = proj_grad(a, c, th[c], g[c]);
  __syncthreads();
  // newest to oldest
  for (int k = 0; k < len; ++k) {
    const int slot = (head - 1 - k + a.m) % a.m;
    const double* s = a.S + slot * rs + i * P;
    const double* y = a.Y + slot * rs + i * P;
    double v = 0.0;
    for (int c = tid; c < P; c += RT) v += s[c] * d[c];
    const double al = a.rho[slot * a.N + i] * block_sum(v, sh);
    if (tid == 0) alpha[k] = al;
    for (int c = tid; c < P; c += RT) d[c] -= al * y[c];
    __syncthreads();
  }
  double gamma;
  if (len > 0) {
    const int slot = (head - 1 + a.m) % a.m;
    const double* s = a.S + slot * rs + i * P;
    const double* y = a.Y + slot * rs + i * P;
    double sy = 0.0, yy = 0.0;
    for (int c = tid; c < P; c += RT) { sy += s[c] * y[c]; yy += y[c] * y[c]; }
    sy = block_sum(sy, sh);
    yy = block_sum(yy, sh);
    gamma = sy / yy;
  } else {
    double gg = 0.0;
    for (int c = tid; c < P; c += RT) {
      const double pg = proj_grad(a, c, th[c], g[c]);
      gg += pg * pg;
    }
    gg = block_sum(gg, sh);
    gamma = 1.0 / fmax(sqrt(gg), 1e-300);  // first step: unit length along -g
  }
  for (int c = tid; c < P; c += RT) d[c] *= gamma;
  __syncthreads();
  // oldest to newest
  for (int k = len - 1; k >= 0; --k) {
    const int slot = (head - 1 - k + a.m) % a.m;
    const double* s = a.S + slot * rs + i * P;
    const double* y = a.Y + slot * rs + i * P;
    double v = 0.0;
    for (int c = tid; c < P; c += RT) v += y[c] * d[c];
    const double be = a.rho[slot * a.N + i] * block_sum(v, sh);
    const double al = alpha[k];
    for (int c = tid; c < P; c += RT) d[c] += (al - be) * s[c];
    __syncthreads();
  }
  double gd = 0.0;
  for (int c = tid; c < P; c += RT) {
    // components held at a bound do not move
    d[c] = (proj_grad(a, c, th[c], g[c]) == 0.0 && g[c] != 0.0) ? 0.0 : -d[c];
    gd += g[c] * d[c];
  }
  gd = block_sum(gd, sh);
  if (!(gd < 0.0)) {
    // not a descent direction: drop the history, projected steepest descent of unit length
    double gg = 0.0;
    for (int c = tid; c < P; c += RT) {
      const double pg = proj_grad(a, c, th[c], g[c]);
      gg += pg * pg;
    }
    gg = block_sum(gg, sh);
    const double sc = 1.0 / fmax(sqrt(gg), 1e-300);
    for (int c = tid; c < P; c += RT) d[c] = -sc * proj_grad(a, c, th[c], g[c]);
    gd = -sqrt(gg);
    if (tid == 0) a.hist_len[i] = 0;
  }
  if (tid == 0) {
    a.gd[i] = gd;
    a.step[i] = 1.0;
    a.accepted[i] = 0;
    a.bt[i] = 0;
  }
}

// trial point of row i: theta + step d projected on the box (theta itself for
// rows that stopped), and gstep_i = g_i . (theta_try_i - theta_i), the
// first-order change the Armijo test compares with.  One block per row.
__global__ __launch_bounds__(RT) void k_make_trial(AscentArgs a) {
  __shared__ double sh[RT];
  const int64_t i = blockIdx.x;
  const int P = a.P;
  const double* th = a.theta + i * P;
  const double* d = a.d + i * P;
  const double* g = a.g + i * P;
  double* tt = a.theta_try + i * P;
  const bool move = a.state[i] == 0 && !a.accepted[i];
  const double st = a.step[i];
  double v = 0.0;
  for (int c = threadIdx.x; c < P; c += RT) {
    double x = th[c];
    if (move) {
      double lo, hi;
      comp_bounds(a, c, &lo, &hi);
      x = fmin(fmax(th[c] + st * d[c], lo), hi);
      v += g[c] * (x - th[c]);
    }
    if (move || a.state[i] != 0) tt[c] = x;
  }
  v = block_sum(v, sh);
  if (threadIdx.x == 0) a.gstep[i] = v;
}

// accept the trial, update the history, test the stopping rule.
// counters[0] += rows still active afterwards
__global__ __launch_bounds__(RT) void k_accept(AscentArgs a, double ftol, int32_t* counters, int async) {
  __shared__ double sh[RT];
  const int64_t i = blockIdx.x;
  const int tid = threadIdx.x;
  const int P = a.P;
  if (a.state[i] != 0) return;
  if (async && (a.accepted[i] == 0 || a.accepted[i] == 3)) return;  // still searching / no trial yet
  const int64_t rs = (int64_t)a.N * P;
  double* th = a.theta + i * P;
  const double* tt = a.theta_try + i * P;
  double* g = a.g + i * P;
  const double* gt = a.g_try + i * P;
  if (a.accepted[i] == 2) {
    // the line search failed: this row cannot improve at this precision
    if (tid == 0) { a.state[i] = 2; a.eta[i] = 0.0; }
    return;
  }
  const int slot = a.hist_head[i];
  double* s = a.S + slot * rs + i * P;
  double* y = a.Y + slot * rs + i * P;
  double sy = 0.0, yy = 0.0;
  for (int c = tid; c < P; c += RT) {
    const double sv = tt[c] - th[c], yv = gt[c] - g[c];
    s[c] = sv;
    y[c] = yv;
    sy += sv * yv;
    yy += yv * yv;
    th[c] = tt[c];
    g[c] = gt[c];
  }
  sy = block_sum(sy, sh);
  yy = block_sum(yy, sh);
  if (tid == 0) {
    if (sy > 1e-14 * yy && sy > 0.0) {  // curvature condition
      a.rho[slot * a.N + i] = 1.0 / sy;
      a.hist_head[i] = (slot + 1) % a.m;
      a.hist_len[i] = a.hist_len[i] < a.m ? a.hist_len[i] + 1 : a.m;
    }
    const double fo = a.f[i], fn = a.f_try[i];
    const double eta = fabs(fn - fo) / fmax(fabs(fn), 1e-300);
    a.eta[i] = eta;
    a.f[i] = fn;
    if (eta <= ftol) a.state[i] = 1;
    else if (counters) atomicAdd(&counters[0], 1);
    if (async) a.accepted[i] = 3;  // next: a new direction
  }
}

// Asynchronous per-row line search (one trial evaluation per step for every
// row; rows are independent, so each row's sequence of iterates is the same as
// with a synchronous search).  accepted: 0 searching, 1 trial accepted,
// 2 search failed, 3 direction needed.  bt: halvings of the current search.
__global__ void k_armijo_async(AscentArgs a, double c1, int max_bt) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= a.N) return;
  if (a.state[i] != 0 || a.accepted[i] != 0) return;
  const double ft = a.f_try[i];
  if (isfinite(ft) && ft <= a.f[i] + c1 * a.gstep[i]) {
    a.accepted[i] = 1;
  } else if (a.bt[i] >= max_bt) {
    a.accepted[i] = 2;
  } else {
    a.step[i] *= 0.5;
    a.bt[i] += 1;
  }
}

__global__ void k_fill_i32(int32_t* p, int n, int32_t v) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) p[k] = v;
}

// counters[0] = rows still active (state 0), by a block sum (no atomics)
__global__ __launch_bounds__(RT) void k_count_active(const AscentArgs a, int32_t* counters) {
  __shared__ double sh[RT];
  double v = 0.0;
  for (int64_t i = threadIdx.x; i < a.N; i += RT) v += (a.state[i] == 0) ? 1.0 : 0.0;
  v = block_sum(v, sh);
  if (threadIdx.x == 0) counters[0] = (int32_t)v;
}

// out[0] = sum over r of p[r][0] (active rows over many contexts), one block
__global__ __launch_bounds__(RT) void k_sum_counters(int32_t* const* p, int n, int32_t* out) {
  __shared__ double sh[RT];
  double v = 0.0;
  for (int r = threadIdx.x; r < n; r += RT) v += (double)p[r][0];
  v = block_sum(v, sh);
  if (threadIdx.x == 0) out[0] = (int32_t)v;
}

int grid_for(int64_t n, int threads) {
  int64_t g = (n + threads - 1) / threads;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return (int)g;
}

}  // namespace

hipError_t launch_gp_reduce(int prec, const void* Gp, int n_splits, int64_t Np, double* G64,
                            int first, hipStream_t st) {
  const int64_t n = Np * Np;
  if (prec == PREC_F64 || prec == PREC_F32)  // FP64 partials in both modes
    hipLaunchKernelGGL(k_gp_reduce_d, dim3(grid_for(n, 256)), dim3(256), 0, st, (const double*)Gp,
                       n_splits, n, G64, first);
  else
    hipLaunchKernelGGL(k_gp_reduce_f, dim3(grid_for(n / 4, 256)), dim3(256), 0, st, (const float*)Gp,
                       n_splits, n, G64, first);
  return hipGetLastError();
}

hipError_t launch_rowpart_reduce(const double* rowpart, int64_t n_tiles, int64_t Np, double* out,
                                 double* tmp, hipStream_t st) {
  hipLaunchKernelGGL(k_rowpart_a, dim3((unsigned)((Np + 255) / 256), RP_SPLITS), dim3(256), 0, st,
                     rowpart, n_tiles, Np, tmp);
  hipLaunchKernelGGL(k_rowpart_b, dim3((unsigned)((Np + 255) / 256)), dim3(256), 0, st, tmp, Np, out);
  return hipGetLastError();
}

int64_t rowpart_tmp_len(int64_t Np) { return RP_SPLITS * Np; }

hipError_t launch_assemble(const AssembleArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_assemble, dim3((unsigned)a.N), dim3(RT), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_sum_rows(const double* v, int n, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_sum_rows, dim3(1), dim3(RT), 0, st, v, n, out);
  return hipGetLastError();
}

hipError_t launch_prepare_params(int prec, int j2, int N, int64_t Np, const double* J64, const double* mu,
                                 void* Jc, double* Jr, double* rowscale, float* jscale,
                                 hipStream_t st) {
  const int g = grid_for(Np * Np, 256);
  switch (prec) {
    case PREC_F64:
      hipLaunchKernelGGL(k_prepare<double>, dim3(g), dim3(256), 0, st, N, Np, J64, mu, (double*)Jc, Jr,
                         rowscale);
      break;
    case PREC_F32:  // FP32 values, staged as FP64 for the FP64-accumulated contraction
      hipLaunchKernelGGL(k_prepare_f32u, dim3(g), dim3(256), 0, st, N, Np, J64, mu, (double*)Jc, Jr,
                         rowscale);
      break;
    case PREC_BF16:
      if (j2)
        hipLaunchKernelGGL(k_prepare_j2, dim3(g), dim3(256), 0, st, N, Np, J64, mu, (__bf16*)Jc, Jr,
                           rowscale);
      else
        hipLaunchKernelGGL(k_prepare<__bf16>, dim3(g), dim3(256), 0, st, N, Np, J64, mu, (__bf16*)Jc, Jr,
                           rowscale);
      break;
    case PREC_FP8:
      if (!jscale) return hipErrorInvalidValue;
      hipLaunchKernelGGL(k_prepare_f8, dim3((unsigned)Np), dim3(256), 0, st, N, Np, J64, mu,
                         (unsigned char*)Jc, Jr, rowscale, jscale);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_copy_out(const double* src, int64_t src_ld, double* dst, int rows, int cols,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_copy_out, dim3(grid_for((int64_t)rows * cols, 256)), dim3(256), 0, st, src,
                     src_ld, dst, rows, cols);
  return hipGetLastError();
}

hipError_t launch_pack_theta(int N, int64_t Np, int P, const double* theta, double* J64, double* mu,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_pack_theta, dim3(grid_for(Np * Np, 256)), dim3(256), 0, st, N, Np, P, theta,
                     J64, mu);
  return hipGetLastError();
}

hipError_t launch_unpack_theta(int N, int64_t Np, int P, const double* J64, const double* mu,
                               double* theta, hipStream_t st) {
  hipLaunchKernelGGL(k_unpack_theta, dim3(grid_for((int64_t)N * P, 256)), dim3(256), 0, st, N, Np, P,
                     J64, mu, theta);
  return hipGetLastError();
}

hipError_t launch_pack_grad(int N, int64_t Np, int P, const double* gJ, const double* gmu,
                            const double* ll_rows, double* g, double* f, hipStream_t st) {
  hipLaunchKernelGGL(k_pack_grad, dim3(grid_for((int64_t)N * P, 256)), dim3(256), 0, st, N, Np, P, gJ,
                     gmu, ll_rows, g, f);
  return hipGetLastError();
}

hipError_t launch_lbfgs_direction(const AscentArgs& a, int async, hipStream_t st) {
  hipLaunchKernelGGL(k_lbfgs_dir, dim3((unsigned)a.N), dim3(RT), 0, st, a, async);
  return hipGetLastError();
}

hipError_t launch_armijo_async(const AscentArgs& a, double c1, int max_bt, hipStream_t st) {
  hipLaunchKernelGGL(k_armijo_async, dim3((unsigned)((a.N + 255) / 256)), dim3(256), 0, st, a, c1, max_bt);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int n, int32_t v, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

hipError_t launch_sum_counters(int32_t* const* p, int n, int32_t* out, hipStream_t st) {
  hipLaunchKernelGGL(k_sum_counters, dim3(1), dim3(RT), 0, st, p, n, out);
  return hipGetLastError();
}

hipError_t launch_count_active(const AscentArgs& a, int32_t* counters, hipStream_t st) {
  hipLaunchKernelGGL(k_count_active, dim3(1), dim3(RT), 0, st, a, counters);
  return hipGetLastError();
}

hipError_t launch_make_trial(const AscentArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_make_trial, dim3((unsigned)a.N), dim3(RT), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_penalty(const AscentArgs& a, const double* theta, double* g, double* f, hipStream_t st) {
  if (!(a.alpha > 0.0)) return hipSuccess;
  hipLaunchKernelGGL(k_penalty, dim3((unsigned)a.N), dim3(RT), 0, st, a, theta, g, f);
  return hipGetLastError();
}

hipError_t launch_project_theta(const AscentArgs& a, double* theta, hipStream_t st) {
  hipLaunchKernelGGL(k_project_theta, dim3(grid_for((int64_t)a.N * a.P, 256)), dim3(256), 0, st, a, theta);
  return hipGetLastError();
}

hipError_t launch_accept_update(const AscentArgs& a, double ftol, int32_t* counters, int async,
                                hipStream_t st) {
  hipLaunchKernelGGL(k_accept, dim3((unsigned)a.N), dim3(RT), 0, st, a, ftol, counters, async);
  return hipGetLastError();
}
