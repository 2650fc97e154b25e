/*
 * glmrec — log-likelihood and gradient of the exponential-link point-process
 * GLM of a recurrent network, evaluated on a uniform time grid for all N
 * postsynaptic neurons at once, with per-row concave ascent, on one AMD
 * MI355X (gfx950).
 *
 * Model (Zaytsev, Morrison, Deger, arXiv:1502.04993):
 *   Sec. 2.1 Eq. (1)-(2)  L = sum_i L_i,  L_i = sum_k log lambda_i(t_ik) - int lambda_i dt
 *   Sec. 2.2 Eq. (3), (5)  U_i = mu_i + sum_j J_ij (h * s_j),  lambda_i = exp(U_i),
 *                          h(t) = H(t) exp(-t/tau); mu_i is the paper's J_i0.
 *   Sec. 2.3.3 Eq. (12)    dL_i/dJ_ij = sum_k v_ij(t_ik) - int lambda_i v_ij dt,
 *                          dL_i/dmu_i = q_i - int lambda_i dt.
 * On the grid of B bins of width dt covering [0, B dt):
 *   s_i[t]  spike count of neuron i in bin t
 *   x_j[t]  = sum_{t' < t} a^(t-t'-1) s_j[t'],  a = exp(-dt/tau)  (a spike acts on
 *             later bins only, with weight 1 in the next bin: the grid form of
 *             the recurrence Eq. (13))
 *   U_i[t]  = mu_i + sum_j J_ij x_j[t],  lambda_i[t] = exp(U_i[t])  [1/s]
 *   L_i     = sum_t s_i[t] U_i[t] - dt sum_t lambda_i[t]
 *             (the constant sum_t s_i[t] log dt is not included)
 *   dL/dJ_ij = sum_t (s_i[t] - dt lambda_i[t]) x_j[t]
 *   dL/dmu_i = q_i - dt sum_t lambda_i[t]
 *   dL/dtau  = sum_{t,i} (s_i[t] - dt lambda_i[t]) sum_j J_ij dx_j[t]/dtau
 *
 * On the event grid (continuous time, Sec. 2.3, no binning): the spikes are q
 * events (t_k, n_k) in [T0, T1); between consecutive events every potential
 * relaxes, U_i(t) = mu_i + D_ik e^{-(t - t_k)/tau} with D_ik = sum_j J_ij v_j(t_k+)
 * (Eq. (8)), so with delta_k = (t_{k+1} - t_k)/tau, xi_k = e^{-delta_k}:
 *   L_i     = sum_{k: n_k = i} U_i(t_k-) - tau e^{mu_i} sum_k [Ei(D_ik) - Ei(D_ik xi_k)]  (Eq. (7), (10))
 *   dL/dJ_ij = sum_{k: n_k = i} v_j(t_k-) - tau e^{mu_i} sum_k v_j(t_k+) (e^{D_ik} - e^{D_ik xi_k}) / D_ik
 *                                                                         (Eq. (12), (14))
 *   dL/dmu_i = q_i - tau e^{mu_i} sum_k [Ei(D_ik) - Ei(D_ik xi_k)]
 * with v_j(t) = sum_{events m of j, t_m < t} e^{-(t - t_m)/tau}; the intervals
 * run from T0 to the first event, between events, and from the last event to
 * T1.  A spike does not act on its own neuron's intensity at its own time
 * (left limit t_k-); events at equal times act in (time, neuron) order.
 * The intervals are the "bins" of a non-uniform grid of slots (n_bins of the
 * context = number of slots, from glmr_event_slots); everything else (params,
 * eval, fit, batching) is shared with the regular grid.
 *
 * Conventions shared by every entry point
 *   - Matrices are dense row-major with row = postsynaptic neuron:
 *     J[i*N + j] is the weight from presynaptic j to postsynaptic i.
 *   - `where` says whether a pointer is host memory (GLMR_HOST) or device
 *     memory of the context's device (GLMR_DEVICE).  Device pointers must be
 *     valid on the context's stream.
 *   - The library copies every input; it never keeps or frees a caller pointer.
 *     Outputs go into caller-allocated buffers of the stated size.
 *   - Every call returns a glmr_status; no exception or abort crosses this
 *     boundary.  After an error, glmr_last_error(ctx) gives a message.
 *   - A context is not thread-safe: one host thread at a time.
 *   - Work runs on the context's stream; calls that return host values
 *     synchronise that stream before returning.
 */
#ifndef GLMREC_H
#define GLMREC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GLMR_OK = 0,
  GLMR_NOT_CONVERGED = 1, /* warning: outputs valid, the iteration cap was hit */
  GLMR_EINVAL = -1,       /* bad argument (size, range, pointer, tau, ...) */
  GLMR_ENOMEM = -2,       /* device allocation failed */
  GLMR_EDEVICE = -3,      /* HIP runtime error */
  GLMR_ENOSPIKES = -4,    /* some neuron has no spike: its MLE does not exist */
  GLMR_ENONFINITE = -5,   /* the likelihood overflowed (exp of a huge potential) */
  GLMR_ESTATE = -6        /* call order: e.g. eval before set_spikes/set_kernel */
} glmr_status;

/* Arithmetic of the trace X, the weights J and the two contractions.
 * Cross-tile sums, the likelihood assembly and the ascent are FP64 in all modes. */
typedef enum {
  GLMR_FP64 = 0, /* trace, J, U, lambda in FP64; FP64 MFMA */
  GLMR_FP32 = 1, /* trace and J in FP32 (the trace rounded stochastically from
                    FP64); U accumulated on the FP64 MFMA, the gradient
                    contraction on the FP32 MFMA; exp and lambda sums in FP64 */
  GLMR_BF16 = 2, /* trace, J and lambda in BF16 (trace rounded stochastically),
                    MFMA with FP32 accumulation */
  GLMR_FP8 = 3,  /* trace, J and lambda in OCP e4m3 with power-of-two scales,
                    FP32 accumulation */
  GLMR_BF16_J2 = 4 /* GLMR_BF16 with J as the sum of two BF16 terms (its 16
                    leading significant bits): kernel U takes k over [J_hi | J_lo]
                    against the trace twice, so the likelihood is that of J to
                    ~1e-5 relative instead of BF16's 4e-3 steps, at one more pass
                    of the trace through the MFMA in kernel U.  Resident trace
                    only; no dL/dtau (GLMR_EINVAL).  Switching between GLMR_BF16
                    and GLMR_BF16_J2 keeps the trace. */
} glmr_precision;

typedef enum { GLMR_HOST = 0, GLMR_DEVICE = 1 } glmr_where;

typedef struct {
  int32_t n_neurons;   /* N >= 1 */
  int64_t n_bins;      /* B >= 1 */
  double dt;           /* bin width in seconds, > 0 */
  int64_t chunk_bins;  /* bins per time chunk of the lambda buffer; 0 = automatic.
                          Rounded up to a multiple of 4096. */
  int32_t precision;   /* glmr_precision */
  int32_t device;      /* HIP device ordinal */
  void* stream;        /* hipStream_t to run on, or NULL for the library's own stream */
  int32_t tile_n;      /* neuron tile (128 or 256); 0 = automatic */
  int32_t trace;       /* where the BF16 trace lives (glmr_trace_mode); other
                          precisions always rebuild it inside the contractions */
  int32_t time_mode;   /* glmr_time_mode: GLMR_TIME_EVENTS for continuous time
                          (then n_bins = glmr_event_slots(...), precision FP64,
                          FP32 or BF16 (the trace rebuilt inside the
                          contractions), dt is not used) */
} glmr_config;

typedef enum { GLMR_TIME_GRID = 0, GLMR_TIME_EVENTS = 1 } glmr_time_mode;

/* The trace x depends on the spikes and tau only.  GLMR_TRACE_RESIDENT builds
 * it once per tau and keeps it in HBM (4 * Bp * Np bytes: two BF16 layouts);
 * GLMR_TRACE_RECOMPUTE rebuilds its tiles from the spike bitmasks inside every
 * contraction (no storage beyond the raster).  GLMR_TRACE_AUTO keeps it
 * resident when it fits in free device memory with 4 GiB to spare. */
typedef enum { GLMR_TRACE_AUTO = 0, GLMR_TRACE_RESIDENT = 1, GLMR_TRACE_RECOMPUTE = 2 } glmr_trace_mode;

typedef struct glmr_ctx glmr_ctx;

/* Create a context; allocates nothing large until set_spikes.  *out is set to
 * NULL on failure. */
glmr_status glmr_create(const glmr_config* cfg, glmr_ctx** out);

/* Release a context and all its device memory.  NULL-safe. */
void glmr_destroy(glmr_ctx* ctx);

/* The spike raster S of Sec. 2.1: n_spikes pairs (bin[k], neuron[k]) with
 * 0 <= bin < n_bins and 0 <= neuron < n_neurons, in any order; a pair may
 * repeat (several spikes in one bin).  Both arrays live in `where` memory.
 * Builds the time-major layout on the device (spike ingest).  Invalidates
 * the kernel-dependent caches.  Returns GLMR_EINVAL on an out-of-range pair
 * (nothing is kept), GLMR_ENOSPIKES if some neuron has q_i = 0 (the raster
 * is kept; eval works, fit refuses). */
glmr_status glmr_set_spikes(glmr_ctx* ctx, const int64_t* bin, const int32_t* neuron,
                            int64_t n_spikes, int32_t where);

/* Number of slots of the event grid of q = n_events spike times (host array,
 * sorted non-decreasing, each in [T0, T1)): one slot from T0, one per event,
 * plus, for every gap between consecutive slot starts (T0, events, T1) longer
 * than max_gap, ceil(gap / max_gap) - 1 spike-free slots splitting it evenly
 * (the likelihood is additive over sub-intervals, so they change nothing but
 * bound the span of 64 consecutive slots).  max_gap <= 0 selects
 * 4 (T1 - T0) / (q + 1).  Host-only arithmetic; no device.  GLMR_EINVAL on
 * unsorted or out-of-range times or a max_gap below (T1 - T0) / 1e9. */
glmr_status glmr_event_slots(const double* times, int64_t n_events, double T0, double T1,
                             double max_gap, int64_t* slots);

/* The spikes of an event-grid context (time_mode GLMR_TIME_EVENTS): n_events
 * pairs (times[k] seconds, neuron[k]) in `where` memory, T0 <= t < T1, in
 * strictly increasing (time, neuron) order, and the same T0, T1, max_gap as
 * given to glmr_event_slots, whose slot count must equal the context's
 * n_bins.  Lays out the slots and ingests the events on the device.  Errors:
 * GLMR_EINVAL on a range or order violation or a slot-count mismatch (nothing
 * is kept), GLMR_ESTATE on a regular-grid context, GLMR_ENOSPIKES as for
 * glmr_set_spikes.  glmr_set_kernel then also fails with GLMR_EINVAL if 64
 * consecutive slots span more than 600 tau (pass a smaller max_gap). */
glmr_status glmr_set_spike_times(glmr_ctx* ctx, const double* times, const int32_t* neuron,
                                 int64_t n_events, double T0, double T1, double max_gap,
                                 int32_t where);

/* The two interval integrals of the event grid, on the host, by the same code
 * the kernels run (Eq. (10), (14)): for an interval of length delta (in units
 * of tau) starting at potential offset D,
 *   F = int_0^delta exp(D e^{-s}) ds = Ei(D) - Ei(D e^{-delta}),
 *   H = int_0^delta e^{-s} exp(D e^{-s}) ds = (e^D - e^{D e^{-delta}}) / D.
 * Either output pointer may be NULL. */
void glmr_ei_interval(double D, double delta, double* F, double* H);

/* The same integrals as the BF16 event grid's resident kernels take them, in
 * FP32 from an FP32 potential D, on the host, by the same code: the midpoint
 * expansion (Touchard polynomials to h^6, within 4e-9 relative where
 * delta max(1, |D e^{-delta/2}|) <= 0.25), else 6-point Gauss-Legendre where
 * delta <= 0.5 and |D| delta <= 1, else the FP64 evaluation rounded.  The
 * device's exponential differs from the host's by a few units of 2^-24.
 * Either output pointer may be NULL. */
void glmr_ei_interval_f32(float D, double delta, float* F, float* H);

/* Kernel time constant tau (seconds) of h(t) = H(t) exp(-t/tau), Sec. 2.2.
 * Requires dt <= tau on the regular grid.  Computes the parameter-independent parts (the trace
 * carries at every 64-bin boundary and the spike term
 * dSigma_ij = sum_t s_i[t] x_j[t] of Eq. (12), which Sec. 2.3.3 notes need
 * only be computed once). */
glmr_status glmr_set_kernel(glmr_ctx* ctx, double tau);

/* glmr_set_kernel for callers that cannot allocate device memory (code that
 * runs under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  The same per-tau set-up and the same results up to the
 * rounding order of the spike term's FP64 sums (it may take fewer time
 * splits), with no hipMalloc, hipFree or allocating library call: the
 * carries' segment sums, the spike term's partials and the event grid's span
 * maximum live in a static device array of 256 MiB (the library holds one on
 * each GPU it runs on, until the process ends); the buffers that persist in
 * the context (carries, resident trace, spike term, tables) are reused.
 * Call glmr_set_kernel once on the context first (at set-up, where
 * allocation is allowed): GLMR_ESTATE if those buffers do not exist, or were
 * made for another precision or chunking.  GLMR_EINVAL for tau as in
 * glmr_set_kernel, and when the recording's set-up needs more than the
 * static array (2 x ceil(n_bins / 4096) x n_pad x 16 bytes plus n_pad^2 x 8
 * bytes, twice that for the dL/dtau caches); nothing is changed then.  Every
 * call on a GPU uses that GPU's one array: calls on one GPU that overlap in
 * time (from several threads) race and must not be made; each call
 * synchronises the context's stream before it returns, so calls made one
 * after the other are safe. */
glmr_status glmr_set_kernel_noalloc(glmr_ctx* ctx, double tau);

/* Transmission delays of Sec. 2.4, Eq. (15), on the regular grid, in bins:
 * every connection j -> i with j != i delays by d, the self-connection
 * i -> i by d_self, 0 <= d, d_self < n_bins.  Row i then sees
 *   U_i[t] = mu_i + sum_{j != i} J_ij x_j[t - d] + J_ii x_i[t - d_self]
 * (x_j[t] = 0 for t <= 0), while its spike terms stay at the recorded bins:
 *   L_i = sum_t s_i[t] U_i[t] - dt sum_t lambda_i[t],
 *   dL/dJ_ij = sum_t (s_i[t] - dt lambda_i[t]) x_j[t - D_ij].
 * The contractions run on the raster shifted by d; d_self != d adds a
 * per-(bin, neuron) correction of the self term.  Allowed at any time
 * (rebuilds the kernel caches); (0, 0) is the undelayed model.  GLMR_EINVAL
 * on the event grid, for d_self != d in FP8, or out-of-range delays;
 * dL/dtau then requires d_self = d. */
glmr_status glmr_set_delays(glmr_ctx* ctx, int64_t d, int64_t d_self);

/* Change the arithmetic of later evaluations (glmr_precision).  Keeps the
 * spikes, the kernel and the FP64 parameters; rebuilds the precision-specific
 * buffers.  Used to finish a BF16 ascent with FP32 evaluations: BF16 rounds J
 * to 8 bits, so the BF16 likelihood is flat below that resolution and the
 * ascent stops within it of the optimum. */
glmr_status glmr_set_precision(glmr_ctx* ctx, int32_t precision);

/* Parameters theta_i = (mu_i, J_i1..J_iN) of Sec. 2.3.3: J is N*N doubles,
 * mu is N doubles (log base rates, 1/s), both in `where` memory. */
glmr_status glmr_set_params(glmr_ctx* ctx, const double* J, const double* mu, int32_t where);

/* Read back the current parameters (after set_params or fit).  Any pointer
 * may be NULL.  tau is a host pointer. */
glmr_status glmr_get_params(glmr_ctx* ctx, double* J, double* mu, double* tau, int32_t where);

/* Evaluate L (Eq. (2) on the grid) and its gradient (Eq. (12)) at the current
 * parameters.
 *   ll       host, 1 double, nullable: L
 *   ll_rows  N doubles, nullable: L_i
 *   grad_J   N*N doubles, nullable: dL/dJ_ij
 *   grad_mu  N doubles, nullable: dL/dmu_i
 *   grad_tau host, 1 double, nullable: dL/dtau (one extra contraction; regular grid only)
 * Array outputs live in `where` memory.  With grad_J and grad_mu both NULL
 * only the likelihood is computed.  GLMR_ENONFINITE if L is not finite. */
glmr_status glmr_eval(glmr_ctx* ctx, double* ll, double* ll_rows, double* grad_J,
                      double* grad_mu, double* grad_tau, int32_t where);

typedef struct {
  int32_t max_iter;       /* iteration cap (default 500) */
  double ftol;            /* per-row stop when |L_i^k - L_i^(k-1)| / |L_i^k| <= ftol
                             (Sec. 2.6.3); 0 = precision default (FP64 1e-14, FP32 1e-11,
                             BF16 1e-6, BF16 with a two-term J 1e-10, FP8 1e-4) */
  int32_t lbfgs_m;        /* history length, 1..64 (default 40; the state takes 2 m N (N+1)
                             doubles) */
  int32_t max_backtracks; /* Armijo halvings per iteration (default 30) */
  int32_t warm_start_mu;  /* 1: start mu_i at log(q_i / T) instead of the current mu */
  int32_t from_zero;      /* 1: start from J = 0, mu = 0 (overrides the current params) */
  /* Regularisation (Sec. 2.5) and bounds (Sec. 2.6.3); zeros leave them off.
   * The maximised objective becomes L_i - l1_alpha sum_{j != i}
   * sqrt(J_ij^2 + l1_eps) (Eq. (16)-(17)); parameters stay in the box
   * |J_ij| <= j_max, rate_min <= e^{mu_i} <= rate_max (trial points are
   * projected on it; components held at a bound leave the search direction). */
  double l1_alpha;        /* penalty strength, >= 0 */
  double l1_eps;          /* its smoothing epsilon (0: 1e-8) */
  double j_max;           /* bound on |J_ij| (0: none) */
  double rate_min;        /* lower bound on e^{mu_i} in 1/s (0: none) */
  double rate_max;        /* upper bound on e^{mu_i} in 1/s (0: none) */
  int32_t resume;         /* 1: continue the ascent the context holds (that of its last glmr_fit,
                             or one restored by glmr_set_state) with its histories, step sizes,
                             row status, history length, penalty and bounds; max_iter, ftol
                             and max_backtracks come from these opts, the rest is ignored.
                             A fit of a + b steps equals one of a steps resumed for b.
                             GLMR_ESTATE if there is none: changing the spikes, kernel,
                             delays, precision or parameters ends an ascent. */
  int32_t keep_history;   /* 1: a new ascent (starting point, penalty, bounds and stopping test
                             from these opts) that starts from the L-BFGS curvature pairs of
                             the context's last ascent instead of an empty history: to continue
                             an ascent in a more exact precision after glmr_set_precision (the
                             pairs are differences of the same objective's gradients, taken at
                             the other precision).  Needs the same lbfgs_m; GLMR_ESTATE if the
                             context holds no pairs (changing the spikes, kernel or delays drops
                             them; changing the precision or parameters keeps them).  Ignored
                             with resume; a batch fit refuses it. */
} glmr_fit_opts;

typedef struct {
  int32_t iters;          /* ascent steps taken (one trial evaluation each) */
  int32_t evals;          /* likelihood evaluations (steps + the initial one) */
  double ll;              /* final L (minus the penalty when l1_alpha > 0) */
  double max_eta;         /* max over rows of the last fractional change */
  int32_t rows_converged; /* rows that met ftol */
  double seconds;         /* wall time of the fit */
} glmr_fit_report;

/* Fill opts with the defaults. */
void glmr_fit_defaults(glmr_fit_opts* opts);

/* Maximise L over theta by per-row L-BFGS with a per-row Armijo line search.
 * L is separable over rows (Sec. 2.2), so every row takes its own step size,
 * searches and stops on its own: each ascent step evaluates one trial point
 * per row (all rows share the evaluation); a row whose trial fails the Armijo
 * test halves its step for the next one (at most max_backtracks times, then it
 * stops as stalled), a row whose trial passes updates its history and takes a
 * new direction.  Each row's sequence of iterates is the same as with a
 * synchronous line search.  The step is captured once in a HIP graph and
 * replayed; the host reads one counter per step.  max_iter bounds the number
 * of steps.  Stopping: the fractional change of L_i (Sec. 2.6.3) below ftol.
 * Requires q_i >= 1 for every neuron (else GLMR_ENOSPIKES).  Returns
 * GLMR_NOT_CONVERGED (a warning) if max_iter is reached.  report may be NULL. */
glmr_status glmr_fit(glmr_ctx* ctx, const glmr_fit_opts* opts, glmr_fit_report* report);

/* Checkpoint of a fit (resume support): the parameters J, mu, tau, the
 * delays, the precision and, when the context holds a resumable ascent, its
 * whole state (per-row L-BFGS histories, iterates, gradients, step sizes,
 * row status, penalty and bounds), as one flat host buffer in this machine's
 * byte order with a fixed head.  buf NULL: *len receives the size in bytes
 * (about 8 (2m + 6) N^2 with history length m, m = 40 by default).
 * Otherwise *len must hold the buffer's size; it receives the bytes
 * written (GLMR_EINVAL, with the size needed in *len, if too small).  The
 * buffer belongs to the caller.  GLMR_ESTATE before spikes and parameters. */
glmr_status glmr_get_state(glmr_ctx* ctx, void* buf, size_t* len);

/* Restore a checkpoint into a context of the same recording: same N,
 * n_bins, dt and time mode, and the same spikes (their count, the
 * per-neuron counts and a 64-bit digest of the ingested raster, which on the
 * event grid covers the slot times too, are checked; set them first,
 * GLMR_ESTATE otherwise).
 * Applies the precision, delays and tau of the checkpoint, its parameters,
 * and its ascent (glmr_fit with opts.resume = 1 then continues it).  In a
 * context created with the same configuration the resumed fit ends bit for
 * bit where the interrupted one would have; a context created in another
 * precision may pad the neurons differently (the padding is fixed at
 * creation), which regroups the sums: the same fit within that precision's
 * rounding.  GLMR_EINVAL on a buffer that is not
 * a checkpoint of this library, is truncated, or belongs to another
 * recording; the context then keeps what it had, except that a failure
 * after the checks (device errors) may leave it partly restored. */
glmr_status glmr_set_state(glmr_ctx* ctx, const void* buf, size_t len);

/* ---------------------------------------------------------------- batching
 * Many independent recordings (contexts of possibly different N and B, all
 * on one device, all in GLMR_BF16 or all in the same precision) evaluated in
 * grouped launches with a work queue over (recording, time tile, neuron
 * tile): recordings with the same tile shapes share one launch per
 * contraction (the fragment-major kernels: one workgroup per tile, each
 * recording's tiles spread evenly over the XCDs; the row-major kernels:
 * persistent workgroups walking the queue).  Each recording takes the shapes the batch autotuner chose
 * for its class (padding that allows 256-neuron tiles, or not), else its
 * context's own, so that a batch evaluation equals each context's own
 * evaluation with those shapes.  The contexts must each have had set_spikes,
 * set_kernel and set_params called.  The batch does not own the contexts;
 * they must outlive it. */
typedef struct glmr_batch glmr_batch;

glmr_status glmr_batch_create(glmr_ctx* const* ctxs, int32_t n, glmr_batch** out);
void glmr_batch_destroy(glmr_batch* b);

/* One evaluation of every recording.  ll: host array of n doubles (nullable).
 * Gradients stay inside each context (read them with glmr_eval-compatible
 * buffers through glmr_batch_get_grad). */
glmr_status glmr_batch_eval(glmr_batch* b, double* ll);

/* Copy recording r's gradient of the last batch evaluation. */
glmr_status glmr_batch_get_grad(glmr_batch* b, int32_t r, double* grad_J, double* grad_mu,
                                int32_t where);

/* Fit every recording (per-row L-BFGS as glmr_fit, all recordings advancing
 * together, each evaluation one batched launch; the per-iteration device work
 * is captured once in a HIP graph and replayed).  reports: host array of n
 * (nullable). */
glmr_status glmr_batch_fit(glmr_batch* b, const glmr_fit_opts* opts, glmr_fit_report* reports);

/* Autotuner of the grouped launches: for each class of recordings (padding
 * that allows 256-neuron tiles, and the rest) times every tile shape that all
 * its recordings allow, by the batch's first time chunk (three rounds of
 * every grouped launch of each contraction, the other class at its current
 * shapes), and keeps the fastest for later batch calls.  Reports the shapes
 * of the first class present.  Cache as in glmr_autotune (one line per
 * batch), keyed by the architecture, precision and the recordings' padded
 * sizes.  Reports -1 when the batch is not grouped (some trace not
 * resident).  Clobbers the contexts' evaluation workspaces. */
glmr_status glmr_batch_autotune(glmr_batch* b, const char* cache_path, int32_t* shape_u,
                                int32_t* shape_g);

/* ------------------------------------------------------------- diagnostics */
const char* glmr_status_string(glmr_status s);
const char* glmr_last_error(const glmr_ctx* ctx);

/* Per-kernel timing with HIP events recorded on the context's stream around
 * every launch while enabled.  glmr_prof_get fills up to `cap` entries of
 * names (static strings), total milliseconds and launch counts, and returns
 * the number of kernel kinds seen (synchronises the stream). */
glmr_status glmr_prof_enable(glmr_ctx* ctx, int32_t on);
int32_t glmr_prof_get(glmr_ctx* ctx, const char** names, double* total_ms, int64_t* launches,
                      int32_t cap);
void glmr_prof_reset(glmr_ctx* ctx);

/* Layout facts of a context (for tests and the bench): padded neuron count,
 * padded bin count, chunk bins, spike planes, neuron tile, and whether the
 * trace is resident in row-major layouts (1), resident with the trace and the
 * weights stored as MFMA fragments (2: BF16 on the uniform grid, unless the
 * environment sets GLMR_XFRAG=0 when the precision is set), or rebuilt inside
 * the contractions (0).  Any pointer may be NULL. */
glmr_status glmr_query(const glmr_ctx* ctx, int64_t* n_pad, int64_t* b_pad, int64_t* chunk_bins,
                       int32_t* planes, int32_t* tile_n, int32_t* trace_resident);

/* Autotuner: times every tile shape the library offers for the two
 * contractions that suits the context's trace layout (row-major: kernel U
 * BI neurons x 256 bins, kernel G BI x BI, several wave grids; fragments: one
 * kernel U of 128 neurons x 256 bins, kernel G of 128, 256 or 512 rows x 128)
 * on this context's own data and parameters (first time chunk, three
 * launches each) and keeps the fastest pair for later evaluations.
 * Applies to the resident BF16 trace; in other modes it changes nothing and
 * reports -1.  cache_path (nullable) is a text file of earlier results keyed
 * by GPU architecture, padded neuron count, chunk length and precision: a hit
 * skips the timing, a miss appends a line.  Kernel U's shapes give identical
 * results; kernel G's change only the grouping of its FP32 partial sums.
 * Clobbers the evaluation workspace (the next glmr_eval recomputes it). */
glmr_status glmr_autotune(glmr_ctx* ctx, const char* cache_path, int32_t* shape_u, int32_t* shape_g);

#ifdef __cplusplus
}
#endif
#endif /* GLMREC_H */
