/*
 * Seeded synthetic spike-raster generator (host C, OpenMP).
 *
 * This module produces INPUTS only: a ground-truth connectivity J, baseline
 * potentials mu, and the spike raster simulated from the discrete-time GLM
 * with exponential link (the data-generating process of the paper's
 * validation protocol, Fig. 2 / Sec. 3.1).  It computes no likelihood, no
 * gradient and no fit; both the FP64 oracle and the GPU library consume its
 * output.
 *
 * Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3", SC'11), a counter-based generator written here
 * from its published round function.  Every draw is addressed by
 * (seed, stream, counter), so the result does not depend on thread count.
 *
 * Simulation (grid reading of Sec. 2.2, Eq. 3-5 with delta_u = 1):
 *   trace     x_j[0] = 0,  x_j[t] = a x_j[t-1] + s_j[t-1],  a = exp(-dt/tau)
 *   potential V_i[t] = sum_j J_ij x_j[t]  (kept directly as a leaky sum)
 *   intensity lambda_i[t] = exp(mu_i + V_i[t])   [1/s]
 *   spike     s_i[t] ~ Bernoulli(min(lambda_i[t] dt, 1))
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------- Philox */
static inline void philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2],
                                 uint32_t out[4]) {
  uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int r = 0; r < 10; ++r) {
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    c0 = hi1 ^ c1 ^ k0;
    c1 = lo1;
    c2 = hi0 ^ c3 ^ k1;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* exported for the known-answer test */
void synth_philox4x32_10(const uint32_t* ctr, const uint32_t* key, uint32_t* out) {
  philox4x32_10(ctr, key, out);
}

/* stream identifiers: the key is (seed, stream) */
enum { ST_TYPES = 1, ST_CONN = 2, ST_RATES = 3, ST_SPIKES = 4, ST_SIZES = 5, ST_SYNFIRE = 6 };

typedef struct { uint32_t key[2]; uint64_t n; uint32_t buf[4]; int have; } rng_t;

static void rng_init(rng_t* r, uint64_t seed, uint32_t stream) {
  r->key[0] = (uint32_t)(seed & 0xffffffffu);
  r->key[1] = (uint32_t)(seed >> 32) ^ (stream * 0x85EBCA6Bu);
  r->n = 0; r->have = 0;
}
static uint32_t rng_u32(rng_t* r) {
  if (r->have == 0) {
    uint32_t ctr[4] = {(uint32_t)r->n, (uint32_t)(r->n >> 32), 0u, 0u};
    philox4x32_10(ctr, r->key, r->buf);
    r->n++;
    r->have = 4;
  }
  return r->buf[4 - (r->have--)];
}
/* uniform double in [0,1) with 53 random bits */
static double rng_unif(rng_t* r) {
  uint32_t a = rng_u32(r) >> 5, b = rng_u32(r) >> 6;
  return ((double)a * 67108864.0 + (double)b) * (1.0 / 9007199254740992.0);
}
/* uniform integer in [0, n) by rejection (no modulo bias) */
static uint32_t rng_below(rng_t* r, uint32_t n) {
  uint32_t lim = (uint32_t)(0x100000000ull - (0x100000000ull % n));
  for (;;) {
    uint32_t v = rng_u32(r);
    if (lim == 0 || v < lim) return v % n;
  }
}

/* ------------------------------------------------------------- networks */
/*
 * Neuron types: the first n_exc = round(f_exc * N) neurons are excitatory.
 * J is dense row-major, J[i*N + j] = weight from presynaptic j to postsynaptic i.
 */

/* Erdos-Renyi: each ordered pair i != j connected with probability p. */
void synth_net_bernoulli(int32_t N, int32_t n_exc, double p, double j_exc, double j_inh,
                         uint64_t seed, double* J) {
  rng_t r;
  rng_init(&r, seed, ST_CONN);
  for (int64_t i = 0; i < N; ++i)
    for (int64_t j = 0; j < N; ++j) {
      double u = rng_unif(&r);
      double w = 0.0;
      if (i != j && u < p) w = (j < n_exc) ? j_exc : j_inh;
      J[i * N + j] = w;
    }
}

/* Fixed in-degree: every neuron receives exactly k_exc excitatory and k_inh
 * inhibitory inputs, drawn without replacement from the other neurons. */
int synth_net_fixed_indegree(int32_t N, int32_t n_exc, int32_t k_exc, int32_t k_inh,
                             double j_exc, double j_inh, uint64_t seed, double* J) {
  int32_t n_inh = N - n_exc;
  if (k_exc > n_exc - 1 || k_inh > n_inh - 1 || k_exc < 0 || k_inh < 0) return -1;
  int32_t* pool = (int32_t*)malloc(sizeof(int32_t) * (size_t)N);
  if (!pool) return -2;
  memset(J, 0, sizeof(double) * (size_t)N * (size_t)N);
  rng_t r;
  rng_init(&r, seed, ST_CONN);
  for (int32_t i = 0; i < N; ++i) {
    /* excitatory sources: partial Fisher-Yates over E \ {i} */
    int32_t m = 0;
    for (int32_t j = 0; j < n_exc; ++j) if (j != i) pool[m++] = j;
    for (int32_t k = 0; k < k_exc; ++k) {
      uint32_t pick = k + rng_below(&r, (uint32_t)(m - k));
      int32_t t = pool[k]; pool[k] = pool[pick]; pool[pick] = t;
      J[(int64_t)i * N + pool[k]] = j_exc;
    }
    m = 0;
    for (int32_t j = n_exc; j < N; ++j) if (j != i) pool[m++] = j;
    for (int32_t k = 0; k < k_inh; ++k) {
      uint32_t pick = k + rng_below(&r, (uint32_t)(m - k));
      int32_t t = pool[k]; pool[k] = pool[pick]; pool[pick] = t;
      J[(int64_t)i * N + pool[k]] = j_inh;
    }
  }
  free(pool);
  return 0;
}

/* Synfire chain embedded in a Bernoulli background.  n_groups groups of
 * group_size excitatory neurons, drawn without replacement from the
 * excitatory population; every neuron of group g projects to every neuron of
 * group g+1 with probability p_chain and weight j_chain, overriding the
 * background weight of that pair.  group_of[i] = group index or -1. */
int synth_net_synfire(int32_t N, int32_t n_exc, double p_bg, double j_exc, double j_inh,
                      int32_t n_groups, int32_t group_size, double p_chain, double j_chain,
                      uint64_t seed, double* J, int32_t* group_of) {
  if ((int64_t)n_groups * group_size > n_exc) return -1;
  synth_net_bernoulli(N, n_exc, p_bg, j_exc, j_inh, seed, J);
  int32_t* perm = (int32_t*)malloc(sizeof(int32_t) * (size_t)n_exc);
  if (!perm) return -2;
  for (int32_t j = 0; j < n_exc; ++j) perm[j] = j;
  rng_t r;
  rng_init(&r, seed, ST_SYNFIRE);
  int32_t need = n_groups * group_size;
  for (int32_t k = 0; k < need; ++k) {
    uint32_t pick = k + rng_below(&r, (uint32_t)(n_exc - k));
    int32_t t = perm[k]; perm[k] = perm[pick]; perm[pick] = t;
  }
  for (int32_t i = 0; i < N; ++i) group_of[i] = -1;
  for (int32_t k = 0; k < need; ++k) group_of[perm[k]] = k / group_size;
  for (int32_t g = 0; g + 1 < n_groups; ++g)
    for (int32_t a = 0; a < group_size; ++a)
      for (int32_t b = 0; b < group_size; ++b) {
        int32_t pre = perm[g * group_size + a], post = perm[(g + 1) * group_size + b];
        double u = rng_unif(&r);
        if (u < p_chain) J[(int64_t)post * N + pre] = j_chain;
      }
  free(perm);
  return 0;
}

/* Base rates c_i ~ U[lo, hi] (1/s). */
void synth_rates_uniform(int32_t N, double lo, double hi, uint64_t seed, double* rate) {
  rng_t r;
  rng_init(&r, seed, ST_RATES);
  for (int32_t i = 0; i < N; ++i) rate[i] = lo + (hi - lo) * rng_unif(&r);
}

/* Draw n values uniformly from the integer range [lo, hi] (recording sizes). */
void synth_uniform_ints(int64_t n, int64_t lo, int64_t hi, uint64_t seed, uint32_t salt,
                        int64_t* out) {
  rng_t r;
  rng_init(&r, seed, ST_SIZES + 16u * salt);
  for (int64_t k = 0; k < n; ++k) out[k] = lo + (int64_t)rng_below(&r, (uint32_t)(hi - lo + 1));
}

/* ------------------------------------------------------------ simulation */
typedef struct { int64_t* bin; int32_t* neu; int64_t n, cap; } splist;

static int sp_push(splist* l, int64_t t, int32_t i) {
  if (l->n == l->cap) {
    int64_t nc = l->cap ? 2 * l->cap : 4096;
    int64_t* nb = (int64_t*)realloc(l->bin, sizeof(int64_t) * (size_t)nc);
    if (!nb) return -1;
    l->bin = nb;
    int32_t* nn = (int32_t*)realloc(l->neu, sizeof(int32_t) * (size_t)nc);
    if (!nn) return -1;
    l->neu = nn;
    l->cap = nc;
  }
  l->bin[l->n] = t; l->neu[l->n] = i; l->n++;
  return 0;
}

/* Result buffers are owned by the module until synth_take/synth_free. */
static int64_t* g_bin = NULL;
static int32_t* g_neu = NULL;
static int64_t g_n = 0;

void synth_free(void) {
  free(g_bin); free(g_neu);
  g_bin = NULL; g_neu = NULL; g_n = 0;
}

/* Copy the last simulated raster out and release it. */
void synth_take(int64_t* bin, int32_t* neu) {
  if (g_n) {
    memcpy(bin, g_bin, sizeof(int64_t) * (size_t)g_n);
    memcpy(neu, g_neu, sizeof(int32_t) * (size_t)g_n);
  }
  synth_free();
}

/*
 * Simulate B bins.  Returns the number of spikes (>= 0) or a negative error.
 * The raster is sorted by (bin, neuron).  n_threads <= 0 uses the OpenMP
 * default.  Uniform draw for (t, i): 32-bit word (i & 3) of
 * Philox(ctr = (t_lo, t_hi, i >> 2, 0), key = (seed, ST_SPIKES)).
 */
int64_t synth_simulate(int32_t N, int64_t B, double dt, double tau, const double* mu,
                       const double* J, uint64_t seed, int n_threads) {
  synth_free();
  if (N <= 0 || B <= 0 || !(dt > 0) || !(tau > 0)) return -1;
  const double a = exp(-dt / tau);
  /* outgoing adjacency (column j of J): targets and weights */
  int64_t* off = (int64_t*)calloc((size_t)N + 1, sizeof(int64_t));
  if (!off) return -2;
  for (int64_t i = 0; i < N; ++i)
    for (int64_t j = 0; j < N; ++j)
      if (J[i * N + j] != 0.0) off[j + 1]++;
  for (int32_t j = 0; j < N; ++j) off[j + 1] += off[j];
  int32_t* tgt = (int32_t*)malloc(sizeof(int32_t) * (size_t)(off[N] + 1));
  double* wgt = (double*)malloc(sizeof(double) * (size_t)(off[N] + 1));
  int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)N);
  double* V = (double*)calloc((size_t)N, sizeof(double));
  double* inp = (double*)calloc((size_t)N, sizeof(double));
  int32_t* fired = (int32_t*)malloc(sizeof(int32_t) * (size_t)N);
  if (!tgt || !wgt || !fill || !V || !inp || !fired) return -2;
  for (int32_t j = 0; j < N; ++j) fill[j] = off[j];
  for (int64_t i = 0; i < N; ++i)
    for (int64_t j = 0; j < N; ++j) {
      double w = J[i * N + j];
      if (w != 0.0) { tgt[fill[j]] = (int32_t)i; wgt[fill[j]] = w; fill[j]++; }
    }
  const double log_dt = log(dt);

  int nth = 1;
#ifdef _OPENMP
  nth = n_threads > 0 ? n_threads : omp_get_max_threads();
  if (nth > N / 16) nth = N / 16 > 0 ? N / 16 : 1;
#endif
  splist* lists = (splist*)calloc((size_t)nth, sizeof(splist));
  int32_t* nf_th = (int32_t*)calloc((size_t)nth, sizeof(int32_t));
  int32_t** fired_th = (int32_t**)calloc((size_t)nth, sizeof(int32_t*));
  int err = 0;
  int32_t n_fired = 0;

#pragma omp parallel num_threads(nth)
  {
    int th = 0;
#ifdef _OPENMP
    th = omp_get_thread_num();
#endif
    /* contiguous neuron block per thread, aligned to groups of 4 */
    int32_t per = ((N + nth - 1) / nth + 3) & ~3;
    int32_t lo = th * per, hi = lo + per;
    if (lo > N) lo = N;
    if (hi > N) hi = N;
    int32_t* my_fired = (int32_t*)malloc(sizeof(int32_t) * (size_t)(hi - lo + 1));
    fired_th[th] = my_fired;
    uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu),
                       (uint32_t)(seed >> 32) ^ (ST_SPIKES * 0x85EBCA6Bu)};
    for (int64_t t = 0; t < B; ++t) {
      /* input from the spikes of bin t-1 (the shared list from the previous step) */
      for (int32_t k = 0; k < n_fired; ++k) {
        int32_t j = fired[k];
        for (int64_t e = off[j]; e < off[j + 1]; ++e) {
          int32_t i = tgt[e];
          if (i >= lo && i < hi) inp[i] += wgt[e];
        }
      }
      int32_t nf = 0;
      uint32_t words[4];
      for (int32_t i = lo; i < hi; ++i) {
        V[i] = a * V[i] + inp[i];
        inp[i] = 0.0;
        if ((i & 3) == 0 || i == lo) {
          uint32_t ctr[4] = {(uint32_t)t, (uint32_t)((uint64_t)t >> 32), (uint32_t)(i >> 2), 0u};
          philox4x32_10(ctr, key, words);
        }
        double u = (double)words[i & 3] * (1.0 / 4294967296.0);
        double lu = mu[i] + V[i] + log_dt; /* log(lambda dt) */
        /* cheap rejection: lambda dt <= 2^(floor(lu*log2 e)+1) */
        double bound = ldexp(1.0, (int)floor(lu * 1.4426950408889634) + 1);
        if (u < bound) {
          double p = exp(lu);
          if (p > 1.0) p = 1.0;
          if (u < p) {
            my_fired[nf++] = i;
            if (sp_push(&lists[th], t, i)) err = 1;
          }
        }
      }
      nf_th[th] = nf;
#pragma omp barrier
#pragma omp single
      {
        n_fired = 0;
        for (int q = 0; q < nth; ++q) {
          memcpy(fired + n_fired, fired_th[q], sizeof(int32_t) * (size_t)nf_th[q]);
          n_fired += nf_th[q];
        }
      }
      /* implicit barrier after single */
    }
    free(my_fired);
  }

  int64_t total = 0;
  for (int q = 0; q < nth; ++q) total += lists[q].n;
  if (!err) {
    g_bin = (int64_t*)malloc(sizeof(int64_t) * (size_t)(total + 1));
    g_neu = (int32_t*)malloc(sizeof(int32_t) * (size_t)(total + 1));
    if (!g_bin || !g_neu) err = 1;
  }
  if (!err) {
    /* merge: thread blocks are ordered by neuron, each list sorted by bin */
    int64_t* pos = (int64_t*)calloc((size_t)nth, sizeof(int64_t));
    int64_t o = 0;
    for (int64_t t = 0; t < B && o < total; ++t)
      for (int q = 0; q < nth; ++q)
        while (pos[q] < lists[q].n && lists[q].bin[pos[q]] == t) {
          g_bin[o] = t; g_neu[o] = lists[q].neu[pos[q]]; ++o; ++pos[q];
        }
    free(pos);
    g_n = total;
  }
  for (int q = 0; q < nth; ++q) { free(lists[q].bin); free(lists[q].neu); }
  free(lists); free(nf_th); free(fired_th);
  free(off); free(tgt); free(wgt); free(fill); free(V); free(inp); free(fired);
  if (err) { synth_free(); return -2; }
  return total;
}
