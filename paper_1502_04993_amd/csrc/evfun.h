// Special functions of the continuous-time likelihood on the event grid
// (Sec. 2.3: between two consecutive network events the potential relaxes as
// U = mu + D e^{-s}, s = (t - t_k)/tau, so each interval's integrals have
// closed forms):
//
//   F(D, delta) = int_0^delta exp(D e^{-s}) ds = Ei(D) - Ei(D xi)      (Eq. (10))
//   H(D, delta) = int_0^delta e^{-s} exp(D e^{-s}) ds = (e^D - e^{D xi}) / D  (Eq. (14))
//
// with xi = e^{-delta}; the interval's intensity integral is tau e^{mu} F and
// its weight on the trace integral tau e^{mu} H.  Both are written for FP64
// and compiled for host and device, so the kernels' arithmetic can be checked
// on the CPU against a library exponential integral.
//
// F by branch (every branch loses at most a small constant factor of FP64
// precision):
//  * short intervals, delta max(1, |u|) <= 0.25 with u = D e^{-delta/2} (the
//    potential offset at the midpoint; nearly every interval between the
//    events of a large network): Taylor expansion of the integrand about the
//    midpoint.  With w = D e^{-s}, d/ds = -w d/dw, so the even derivatives of
//    e^w are T_2k(w) e^w with T_n the Touchard polynomials (T_n(w) =
//    sum_k S(n, k) w^k, S the Stirling numbers of the second kind), and those
//    of e^{-s} e^w are e^{-s} Q_2k(w) e^w with Q_n = T_{n+1}(w) / w; the
//    midpoint rule's moments are delta^{2k+1} / (4^k (2k+1)!).  Terms up to
//    k = 6; the first omitted one is below Bell(15) x^14 / (4^7 15!) =
//    2.4e-16 relative at x = delta max(1, |u|) = 0.25.  One exponential, no
//    loop.
//  * |D| <= 2: the series of Ei difference term by term,
//      F = delta + (1 - xi) sum_{n>=1} D^n S_n / (n n!),  S_n = 1 + xi + ... + xi^{n-1},
//    which keeps 1 - xi^n = (1 - xi) S_n exact for short intervals (no
//    cancellation between Ei(D) and Ei(D xi)); 26 terms.
//  * |D| > 2 and |D| (1 - xi) <= 1: the two Ei values nearly cancel; integrate
//    e^u / u over u in [D xi, D] (length <= 1, at least 1 away from the pole
//    at 0) by 16-point Gauss-Legendre.
//  * otherwise Ei(D) - Ei(D xi) directly.
// Ei(x): the power series gamma + ln|x| + sum x^n/(n n!) for -1 <= x <= 40
// (Abramowitz & Stegun 5.1.10), the continued fraction of E1 for x < -1
// (A&S 5.1.22, evaluated by the modified Lentz method), the asymptotic series
// e^x/x sum k!/x^k for x > 40 (A&S 5.1.51), truncated at its smallest term.
#pragma once

#include <math.h>

#if defined(__HIPCC__)
#define GLMR_HD __host__ __device__
#else
#define GLMR_HD
#endif

namespace glmr_ev {

constexpr double kEulerGamma = 0.57721566490153286061;

GLMR_HD inline double ei(double x) {
  if (x == 0.0) return -INFINITY;
  if (x < -1.0) {
    const double z = -x;
    // E1(z) = e^{-z} / (z + 1 - 1/(z + 3 - 4/(z + 5 - 9/(z + 7 - ...))))
    const double tiny = 1e-300;
    double b = z + 1.0, c = 1.0 / tiny, d = 1.0 / b, h = d;
    for (int i = 1; i < 500; ++i) {
      const double an = -(double)i * (double)i;
      b += 2.0;
      d = an * d + b;
      if (fabs(d) < tiny) d = tiny;
      c = b + an / c;
      if (fabs(c) < tiny) c = tiny;
      d = 1.0 / d;
      const double del = c * d;
      h *= del;
      if (fabs(del - 1.0) < 1e-17) break;
    }
    return -h * exp(-z);
  }
  if (x <= 40.0) {
    double term = 1.0, sum = 0.0;
    for (int n = 1; n < 400; ++n) {
      term *= x / (double)n;  // x^n / n!
      const double t = term / (double)n;
      sum += t;
      if (fabs(t) <= 1e-17 * fabs(sum)) break;
    }
    return kEulerGamma + log(fabs(x)) + sum;
  }
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 200; ++k) {
    const double next = term * (double)k / x;
    if (next > term || next < 1e-18) break;
    term = next;
    sum += term;
  }
  return exp(x) / x * sum;
}

// 16-point Gauss-Legendre nodes (positive half) and weights on [-1, 1]
GLMR_HD inline double gl16_node(int k) {
  const double v[8] = {9.50125098376374544e-02, 2.81603550779258915e-01, 4.58016777657227370e-01,
                       6.17876244402643771e-01, 7.55404408355002999e-01, 8.65631202387831755e-01,
                       9.44575023073232600e-01, 9.89400934991649939e-01};
  return v[k];
}
GLMR_HD inline double gl16_weight(int k) {
  const double v[8] = {1.89450610455068585e-01, 1.82603415044923612e-01, 1.69156519395002619e-01,
                       1.49595988816576764e-01, 1.24628971255534030e-01, 9.51585116824925914e-02,
                       6.22535239386477063e-02, 2.71524594117540374e-02};
  return v[k];
}

// Quantities of an interval that depend on its length only (a kernel lane
// keeps one slot for many neurons and computes them once).
struct Slot {
  double delta, eh, c1, c2, c3, c4, c5, c6, e1, xi;
};

GLMR_HD inline Slot slot_consts(double delta) {
  Slot q;
  q.delta = delta;
  q.eh = exp(-0.5 * delta);
  const double d2 = delta * delta;
  q.c1 = d2 * (1.0 / 24.0);
  q.c2 = d2 * d2 * (1.0 / 1920.0);
  q.c3 = d2 * d2 * d2 * (1.0 / 322560.0);
  q.c4 = d2 * d2 * d2 * d2 * (1.0 / 92897280.0);
  q.c5 = q.c4 * d2 * (1.0 / 440.0);   // delta^10 / (4^5 11!)
  q.c6 = q.c5 * d2 * (1.0 / 624.0);   // delta^12 / (4^6 13!)
  q.e1 = -expm1(-delta);  // 1 - xi, exact for short intervals
  q.xi = exp(-delta);
  return q;
}

GLMR_HD inline void interval_long(double D, const Slot& q, double* F, double* H);

// F and H of one interval of length q.delta (in units of tau) that starts with
// potential offset D; delta = 0 gives 0 for both.
GLMR_HD inline void interval(double D, const Slot& q, double* F, double* H) {
  const double delta = q.delta;
  if (!(delta > 0.0)) {
    *F = 0.0;
    *H = 0.0;
    return;
  }
  const double u = D * q.eh;
  if (delta * fmax(1.0, fabs(u)) <= 0.25) {
    const double T2 = u * (1.0 + u);
    const double T4 = u * (1.0 + u * (7.0 + u * (6.0 + u)));
    const double T6 = u * (1.0 + u * (31.0 + u * (90.0 + u * (65.0 + u * (15.0 + u)))));
    const double T8 =
        u * (1.0 + u * (127.0 + u * (966.0 + u * (1701.0 + u * (1050.0 + u * (266.0 + u * (28.0 + u)))))));
    const double Q2 = 1.0 + u * (3.0 + u);
    const double Q4 = 1.0 + u * (15.0 + u * (25.0 + u * (10.0 + u)));
    const double Q6 = 1.0 + u * (63.0 + u * (301.0 + u * (350.0 + u * (140.0 + u * (21.0 + u)))));
    const double Q8 =
        1.0 + u * (255.0 + u * (3025.0 + u * (7770.0 + u * (6951.0 + u * (2646.0 + u * (462.0 + u * (36.0 + u)))))));
    const double T10 =
        u * (1.0 + u * (511.0 + u * (9330.0 + u * (34105.0 + u * (42525.0 + u * (22827.0 + u * (5880.0 +
        u * (750.0 + u * (45.0 + u)))))))));
    const double T12 =
        u * (1.0 + u * (2047.0 + u * (86526.0 + u * (611501.0 + u * (1379400.0 + u * (1323652.0 + u * (627396.0 +
        u * (159027.0 + u * (22275.0 + u * (1705.0 + u * (66.0 + u)))))))))));
    const double Q10 =
        1.0 + u * (1023.0 + u * (28501.0 + u * (145750.0 + u * (246730.0 + u * (179487.0 + u * (63987.0 +
        u * (11880.0 + u * (1155.0 + u * (55.0 + u)))))))));
    const double Q12 =
        1.0 + u * (4095.0 + u * (261625.0 + u * (2532530.0 + u * (7508501.0 + u * (9321312.0 + u * (5715424.0 +
        u * (1899612.0 + u * (359502.0 + u * (39325.0 + u * (2431.0 + u * (78.0 + u)))))))))));
    const double g = delta * exp(u);
    *F = g * (1.0 + (q.c1 * T2 + (q.c2 * T4 + (q.c3 * T6 + (q.c4 * T8 + (q.c5 * T10 + q.c6 * T12))))));
    *H = g * q.eh * (1.0 + (q.c1 * Q2 + (q.c2 * Q4 + (q.c3 * Q6 + (q.c4 * Q8 + (q.c5 * Q10 + q.c6 * Q12))))));
    return;
  }
  interval_long(D, q, F, H);
}

// Intervals past the short-interval branch (rare between the events of a
// large network): a call, so that the kernels keep only the short branch in
// their registers.
#if defined(__HIPCC__)
__host__ __device__ __attribute__((noinline))
#endif
inline void interval_long(double D, const Slot& q, double* F, double* H) {
  const double delta = q.delta;
  const double e1 = q.e1, xi = q.xi;
  const double y = D * e1;
  *H = exp(D * xi) * e1 * (y == 0.0 ? 1.0 : expm1(y) / y);
  const double ad = fabs(D);
  if (ad <= 2.0) {
    double p = 1.0, S = 1.0, acc = 0.0;
#pragma unroll
    for (int n = 1; n <= 26; ++n) {
      p *= D * (1.0 / (double)n);            // D^n / n!
      acc += p * (1.0 / (double)n) * S;      // D^n S_n / (n n!)
      S = 1.0 + xi * S;                      // S_{n+1}
    }
    *F = delta + e1 * acc;
    return;
  }
  if (fabs(y) <= 1.0) {
    const double half = 0.5 * y, mid = D - half;  // u in [D xi, D] = mid -/+ half
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const double x = gl16_node(k) * half;
      const double u1 = mid + x, u2 = mid - x;
      acc += gl16_weight(k) * (exp(u1) / u1 + exp(u2) / u2);
    }
    *F = half * acc;
    return;
  }
  *F = ei(D) - ei(D * xi);
}

GLMR_HD inline void interval(double D, double delta, double* F, double* H) {
  interval(D, slot_consts(delta), F, H);
}

// FP32 evaluation for the BF16 mode (whose potential D is an FP32 sum of
// BF16 products), in three tiers: the midpoint expansion below; 6-point
// Gauss-Legendre in s on [0, delta],
//   F = delta/2 sum_k w_k exp(D e^{-s_k}),  H = delta/2 sum_k w_k e^{-s_k} exp(D e^{-s_k}),
// for delta <= 0.5 and |D| delta <= 1 (the integrand is entire and varies by
// at most a factor e over the interval; relative error a few units of
// 2^-24); every other interval through the FP64 evaluation.  The nodes
// e^{-s_k} depend on the interval only.
struct SlotF {
  float half;     // delta / 2 (0: empty interval)
  float e[6];     // e^{-s_k}
  float w[6];     // weights times delta / 2
  bool ok;        // delta <= 0.5
};

GLMR_HD inline SlotF slot_consts_f(const Slot& q) {
  const double xn[3] = {2.38619186083196932e-01, 6.61209386466264482e-01, 9.32469514203152050e-01};
  const double wn[3] = {4.67913934572691370e-01, 3.60761573048138939e-01, 1.71324492379169746e-01};
  SlotF f;
  const double h = 0.5 * q.delta;
  f.half = (float)h;
  f.ok = q.delta > 0.0 && q.delta <= 0.5;
  for (int k = 0; k < 3; ++k) {
    f.e[2 * k] = (float)exp(-h * (1.0 - xn[k]));
    f.e[2 * k + 1] = (float)exp(-h * (1.0 + xn[k]));
    f.w[2 * k] = f.w[2 * k + 1] = (float)(h * wn[k]);
  }
  return f;
}

// the FP64 evaluation as a call (rare in the FP32 path; kept out of its registers)
#if defined(__HIPCC__)
__host__ __device__ __attribute__((noinline))
#endif
inline void interval_call(double D, double delta, double* F, double* H) {
  interval(D, slot_consts(delta), F, H);
}

// FP32 exponential: the hardware's base-2 exponential on the device (a few
// units of 2^-24, more for |x| >> 1 through the rounding of x log2 e), the
// C library's on the host.
GLMR_HD inline float exp_f32(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __expf(x);
#else
  return expf(x);
#endif
}

// 2^x in FP32: the hardware's base-2 exponential on the device, the C
// library's on the host.
GLMR_HD inline float exp2_f32(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_exp2f(x);
#else
  return exp2f(x);
#endif
}

// The first tier of the FP32 evaluation (the resident BF16 trace): the
// midpoint expansion of the short-interval branch above, to k = 3.  With
// h = delta / 2 and u = D e^{-h},
//   F = delta e^u sum_k T_2k(u) h^2k / (2k+1)!,
//   H = delta e^{-h} e^u sum_k Q_2k(u) h^2k / (2k+1)!,   Q_n = T_{n+1} / u,
// (the Touchard generating function exp(u (e^t - 1)) = sum_n T_n(u) t^n / n!
// with t = -(s - h), odd powers of t integrating to zero).  Where
// delta max(1, |u|) <= 0.35 the first omitted terms are below
// Bell(8) 0.175^8 / 9! = 1.0e-8 (F) and Bell(9) 0.175^8 / 9! = 5.1e-8 (H)
// relative (T_n(m) <= Bell(n) m^n for m >= 1, and both sums lie within
// e^{+-0.2} of their first term, so relative means relative to the result).
// The sums are polynomials in u whose coefficients depend on the interval
// only, with delta and delta e^{-h} folded in; they are taken in
// v = u log2(e), the base-2 exponential's argument, with the coefficients of
// v^j scaled by ln(2)^j: one exponential and two degree-6 Horner evaluations
// per potential.  The 16 coefficients of an interval (stage_f):
// [0..6] F / e^u = sum_j c_j v^j, [7] e^{-h} log2(e), [8..14]
// H / e^u = sum_j c_{8+j} v^j, [15] the bound on |v| (0.35 log2(e) / delta,
// negative where delta > 0.35, so that delta max(1, |u|) <= 0.35 reads
// |v| <= [15]).
constexpr float EXP_BOUND = 0.35f;

GLMR_HD inline void stage_f(float delta, float emh, float* o) {
  const float h = 0.5f * delta;
  const float c2 = h * h * (1.0f / 6.0f);    // h^2 / 3!
  const float c4 = 0.3f * c2 * c2;           // h^4 / 5!
  const float c6 = c4 * c2 * (1.0f / 7.0f);  // h^6 / 7!
  const float dq = delta * emh;
  // ln(2)^j
  const float l1 = 0.693147180559945309f, l2 = 0.480453013918201424f, l3 = 0.333024651988929479f,
              l4 = 0.230835098583083444f, l5 = 0.160002697757141904f, l6 = 0.110905418239124928f;
  // T_0 = 1, T_2 = u + u^2, T_4 = u + 7u^2 + 6u^3 + u^4,
  // T_6 = u + 31u^2 + 90u^3 + 65u^4 + 15u^5 + u^6
  o[0] = delta;
  o[1] = l1 * (delta * (c2 + c4 + c6));
  o[2] = l2 * (delta * (c2 + 7.0f * c4 + 31.0f * c6));
  o[3] = l3 * (delta * (6.0f * c4 + 90.0f * c6));
  o[4] = l4 * (delta * (c4 + 65.0f * c6));
  o[5] = l5 * (delta * (15.0f * c6));
  o[6] = l6 * (delta * c6);
  o[7] = emh * 1.44269504088896341f;
  // Q_0 = 1, Q_2 = 1 + 3u + u^2, Q_4 = 1 + 15u + 25u^2 + 10u^3 + u^4,
  // Q_6 = 1 + 63u + 301u^2 + 350u^3 + 140u^4 + 21u^5 + u^6
  o[8] = dq * (1.0f + c2 + c4 + c6);
  o[9] = l1 * (dq * (3.0f * c2 + 15.0f * c4 + 63.0f * c6));
  o[10] = l2 * (dq * (c2 + 25.0f * c4 + 301.0f * c6));
  o[11] = l3 * (dq * (10.0f * c4 + 350.0f * c6));
  o[12] = l4 * (dq * (c4 + 140.0f * c6));
  o[13] = l5 * (dq * (21.0f * c6));
  o[14] = l6 * (dq * c6);
  o[15] = delta <= EXP_BOUND ? (delta > 0.0f ? EXP_BOUND * 1.44269504088896341f / delta : 3.0e38f) : -1.0f;
}

// The expansion from an interval's 16 coefficients in three parts,
// F = E pf and H = E ph; returns whether the interval is within its bound
// (otherwise F, H are to be taken from the next tier).
GLMR_HD inline bool taylor_parts(const float* c, float D, float* E, float* pf, float* ph) {
  const float v = D * c[7];
  *E = exp2_f32(v);
  float f = c[6], g = c[14];
#pragma unroll
  for (int k = 5; k >= 0; --k) {
    f = f * v + c[k];
    g = g * v + c[8 + k];
  }
  *pf = f;
  *ph = g;
  return fabsf(v) <= c[15];
}

// F, H by the expansion.
GLMR_HD inline bool taylor_f(const float* c, float D, float* F, float* H) {
  float E, pf, ph;
  const bool ok = taylor_parts(c, D, &E, &pf, &ph);
  *F = E * pf;
  *H = E * ph;
  return ok;
}

// The per-interval table of the FP32 evaluation, 16 floats: [0] delta,
// [1] e^{-delta/2} (the expansion), [8] delta/2, [9..14] the Gauss-Legendre
// nodes e^{-s_k}, [15] 1 where delta <= 0.5 (the quadrature), the rest 0.
GLMR_HD inline void table_f(double delta, float* o) {
  const SlotF f = slot_consts_f(slot_consts(delta));
  o[0] = (float)delta;
  o[1] = (float)exp(-0.5 * delta);
  for (int k = 2; k < 8; ++k) o[k] = 0.0f;
  o[8] = f.half;
  for (int k = 0; k < 6; ++k) o[9 + k] = f.e[k];
  o[15] = f.ok ? 1.0f : 0.0f;
}

// The second tier from the table's quadrature half q (its entries 8 .. 15:
// delta/2, the six nodes, the flag): 6-point Gauss-Legendre in FP32 where
// delta <= 0.5 and |D| delta <= 1; returns whether it applies.
GLMR_HD inline bool gl_quad_f(const float* q, float D, float* F, float* H) {
  const float half = q[0];
  if (!(q[7] != 0.0f && fabsf(D) * (2.0f * half) <= 1.0f)) return false;
  const float wn[3] = {4.67913934572691370e-01f, 3.60761573048138939e-01f, 1.71324492379169746e-01f};
  float sf = 0.0f, sh = 0.0f;
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const float v = half * wn[k >> 1] * exp_f32(D * q[1 + k]);
    sf += v;
    sh += v * q[1 + k];
  }
  *F = sf;
  *H = sh;
  return true;
}

// The third tier: the FP64 evaluation (zero for an empty interval).
GLMR_HD inline void fp64_tier_f(float D, double delta, float* F, float* H) {
  if (!(delta > 0.0)) {
    *F = 0.0f;
    *H = 0.0f;
    return;
  }
  double Fd, Hd;
  interval_call((double)D, delta, &Fd, &Hd);
  *F = (float)Fd;
  *H = (float)Hd;
}

// The second and third tiers.
GLMR_HD inline void gl_tier_f(const float* q, double delta, float D, float* F, float* H) {
  if (!gl_quad_f(q, D, F, H)) fp64_tier_f(D, delta, F, H);
}

// The whole FP32 chain for one interval, as the resident BF16 kernels take it.
GLMR_HD inline void interval_f32(float D, double delta, float* F, float* H) {
  float o[16], c[16];
  table_f(delta, o);
  stage_f(o[0], o[1], c);
  if (!taylor_f(c, D, F, H)) gl_tier_f(o + 8, delta, D, F, H);
}

}  // namespace glmr_ev
