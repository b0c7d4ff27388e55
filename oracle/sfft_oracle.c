/*
 * sfft_oracle.c -- plain, slow FP64 CPU oracle of the aliasing-filter sparse
 * FFT hot path: frequency bucketization, singleton test, phase-to-index
 * location, two-ton moment preserving solve, R-FFAST singleton estimator,
 * FFAST peeling (both schedules) and binary-tree search, as described in
 * Li, Jiang & Chen, "On Performance of Sparse Fast Fourier Transform
 * Algorithms Using the Aliasing Filter" (2020).
 *
 * TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU
 * baseline of the benchmark are its only users.  It shares no code, header,
 * table or constant with the GPU library, and nothing in it is tuned.
 *
 * Conventions (Sect. 2.1, Eq. 1-2): xhat_f = (1/N) sum_j x_j e^{-2 pi i f j/N},
 * so x_j = sum_f xhat_f e^{+2 pi i f j / N}.  Samples are taken with an
 * advance shift tau, y[m] = x[(sigma m L + tau) mod N], so that the B-point
 * DFT of y (with the 1/B of F_B) holds, in bin sigma*c mod B, the sum of
 * xhat_f e^{+2 pi i f tau/N} over f = c (mod B) -- Eq. 6 with tau -> -tau.
 * All angles are reduced to an integer modulo N (or modulo B) before any
 * trigonometric call.
 *
 * Parity status: every function below is pinned by a CPU test (aliasing
 * identity against a brute-force DFT, exact recovery of planted spectra, the
 * N=20 peeling example of Sect. 3.2, the N=64 tree example and the
 * small-support case of Sect. 3.3, Table 1 by Monte Carlo; the two-ton
 * solve by the residue structure of the tree and the N=64 example; the
 * packet-erasure schedule by the six-identification N=20 example; Kay's
 * estimator by its noiseless limit and the Cramer-Rao bound).  The paper
 * names the noisy-mode thresholds T0, T1 without values; the widths taken
 * here are pinned to the laws they imply: the zero-ton rate of noise-only
 * class vectors equals P[Gamma(n,1) <= n + zero_k sqrt(n)], the single-ton
 * rate of located tones P[Gamma(n-1,1) <= n-1 + single_k sqrt(n-1)], and
 * the noise estimate lies in the interval its order statistic implies.
 */
#include "sfft_oracle.h"

#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

static const double TWO_PI = 6.283185307179586476925286766559;

/* ------------------------------------------------------------------ */
/* SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom number
   generators", OOPSLA 2014): state advances by the golden-ratio increment,
   output is the variant-13 finaliser.                                   */
uint64_t orc_splitmix64_next(uint64_t *state) {
  uint64_t z;
  *state += 0x9E3779B97F4A7C15ULL;
  z = *state;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

static int is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

static int64_t next_pow2(int64_t v) {
  int64_t p = 1;
  while (p < v) p <<= 1;
  return p;
}

static void cfg_defaults(orc_cfg *c) {
  c->max_peel_rounds = 64;
  c->eps0 = 1e-4;
  c->eps1 = 1e-4;
  c->zero_k = 4.0;
  c->single_k = 4.0;
  c->noise_var = 0.0;
  c->window = 0;
}

int orc_set_rffast(orc_cfg *c, uint64_t seed, int32_t C, int32_t m) {
  if (c->kind != ORC_FFAST || C < 1 || C > ORC_MAX_ROUNDS || m < 2 || C * m > 64) return -1;
  uint64_t st = seed;
  c->rf_iters = C;
  c->rf_m = m;
  c->D = C * m;
  for (int i = 0; i < C; i++) c->rf_off[i] = orc_splitmix64_next(&st) % (uint64_t)c->N;
  return 0;
}

int orc_draw_starts(orc_cfg *c, uint64_t seed, int32_t count) {
  if (count < 0 || count > ORC_MAX_STARTS) return -1;
  uint64_t st = seed;
  for (int i = 0; i < c->rf_iters; i++) (void)orc_splitmix64_next(&st);
  c->n_starts = count;
  for (int i = 0; i < count; i++) c->start_f[i] = (int64_t)(orc_splitmix64_next(&st) % (uint64_t)c->N);
  return 0;
}

/* Plan of the tree (N a power of two) or of FFAST (N a product of co-prime
   prime powers, Sect. 3.2: B_i = p_i^e_i, L_i = N / B_i, ascending prime). */
int orc_config(orc_cfg *c, int64_t N, int64_t K, int32_t stages, int32_t delays,
               uint64_t seed, int32_t mode, int64_t B0, int32_t identity_round0) {
  memset(c, 0, sizeof(*c));
  cfg_defaults(c);
  if (N < 2 || K < 1 || K > N || stages < 1 || delays < 1) return -1;
  if (mode == ORC_EXACT && delays < 2) return -1;
  c->N = N;
  c->K = K;
  c->mode = mode;
  c->D = delays;
  c->R = stages;
  if (is_pow2(N)) {
    if (stages > ORC_MAX_ROUNDS) return -1;
    c->kind = ORC_TREE;
    if (B0 <= 0) {
      B0 = next_pow2(2 * K);
      if (B0 > N) B0 = N;
    }
    if (!is_pow2(B0) || B0 > N) return -1;
    c->B0 = B0;
    c->max_levels = 0;
    for (int64_t b = B0; b < N; b <<= 1) c->max_levels++;
    uint64_t st = seed;
    for (int r = 0; r < stages; r++) {
      if (r == 0 && identity_round0) {
        c->sigma[r] = 1;
        c->shift[r] = 0;
        continue;
      }
      uint64_t a = orc_splitmix64_next(&st);
      uint64_t b = orc_splitmix64_next(&st);
      c->sigma[r] = 2 * (a % (uint64_t)(N / 2)) + 1;
      c->shift[r] = b % (uint64_t)N;
    }
  } else {
    /* factor N into prime powers, in order of increasing prime */
    int64_t rest = N, f[ORC_MAX_STAGES];
    int nf = 0;
    for (int64_t p = 2; p * p <= rest; p++) {
      if (rest % p) continue;
      int64_t q = 1;
      while (rest % p == 0) { rest /= p; q *= p; }
      if (nf == ORC_MAX_STAGES) return -2;
      f[nf++] = q;
    }
    if (rest > 1) {
      if (nf == ORC_MAX_STAGES) return -2;
      f[nf++] = rest;
    }
    if (nf != stages) return -2;
    c->kind = ORC_FFAST;
    for (int j = 0; j < nf; j++) {
      c->stageB[j] = f[j];
      c->sigma[j] = 1;
      c->shift[j] = 0;
    }
  }
  return 0;
}

/* FFAST plan with explicitly chosen co-prime stage sizes. */
int orc_config_stages(orc_cfg *c, int64_t N, int64_t K, int32_t nstages,
                      const int64_t *stageB, int32_t delays, int32_t mode) {
  memset(c, 0, sizeof(*c));
  cfg_defaults(c);
  if (nstages < 1 || nstages > ORC_MAX_STAGES || delays < 1) return -1;
  if (mode == ORC_EXACT && delays < 2) return -1;
  c->N = N;
  c->K = K;
  c->mode = mode;
  c->D = delays;
  c->R = nstages;
  c->kind = ORC_FFAST;
  for (int j = 0; j < nstages; j++) {
    if (stageB[j] < 1 || N % stageB[j]) return -1;
    c->stageB[j] = stageB[j];
    c->sigma[j] = 1;
    c->shift[j] = 0;
  }
  return 0;
}

/* e^{sign * 2 pi i t / M} for an integer t already reduced modulo M */
static cplx unit(int64_t t, int64_t M, int sign) {
  double ang = TWO_PI * (double)t / (double)M;
  return cos(ang) + (double)sign * sin(ang) * I;
}

static uint64_t mulmod(uint64_t a, uint64_t b, uint64_t m) {
  return (uint64_t)(((unsigned __int128)a * b) % m);
}

static cplx load(const float *x, int64_t p) {
  return (double)x[2 * p] + (double)x[2 * p + 1] * I;
}

/* table of e^{-2 pi i k / B}, k < B */
static cplx *twiddles(int64_t B) {
  cplx *t = (cplx *)malloc(sizeof(cplx) * (size_t)B);
  for (int64_t k = 0; k < B; k++) t[k] = unit(k, B, -1);
  return t;
}

/* Eq. 5-6: bin h of F_B D_L (shift by tau) x, with permutation sigma:
   (1/B) sum_{m<B} x[(sigma m L + tau) mod N] e^{-2 pi i h m / B}. */
static cplx bin_tw(const float *x, int64_t N, int64_t B, uint64_t sigma,
                   uint64_t tau, int64_t h, const cplx *tw) {
  int64_t L = N / B;
  uint64_t step = mulmod(sigma % (uint64_t)N, (uint64_t)L, (uint64_t)N);
  uint64_t pos = tau % (uint64_t)N;
  int64_t t = 0;
  cplx acc = 0;
  for (int64_t m = 0; m < B; m++) {
    acc += load(x, (int64_t)pos) * tw[t];
    pos = (pos + step) % (uint64_t)N;
    t = (t + h) % B;
  }
  return acc / (double)B;
}

void orc_bin(const float *x, int64_t N, int64_t B, uint64_t sigma, uint64_t tau,
             int64_t h, double *out) {
  cplx *tw = twiddles(B);
  cplx v = bin_tw(x, N, B, sigma, tau, ((h % B) + B) % B, tw);
  free(tw);
  out[0] = creal(v);
  out[1] = cimag(v);
}

/* delay of FFAST measurement i: d = i, or with the R-FFAST set of Sect. 3.2
   the i-th of r_0, r_0 + 1, ..., r_1, r_1 + 2, ..., r_c + 2^c t, ...  */
static uint64_t ffast_tau(const orc_cfg *c, int i) {
  if (c->rf_iters <= 0) return (uint64_t)i;
  int it = i / c->rf_m, t = i % c->rf_m;
  return (c->rf_off[it] + ((uint64_t)t << it)) % (uint64_t)c->N;
}

/* ------------------------------------------------------------------ */
/* Singleton test of Sect. 3.2, Subproblems 1 and 2.                    */

typedef struct {
  int cls;
  int64_t f;
  cplx a;
  int64_t f2;   /* two-ton: the second position and value */
  cplx a2;
} decision;

typedef struct {
  const orc_cfg *c;
  int n;              /* measurements per class */
  int rounds;         /* rounds contributing to this class vector */
  uint64_t tau[ORC_MAX_ROUNDS * 64];
  double sref2;       /* exact mode reference power */
  double noise_var;   /* noisy mode, time domain */
} cls_ctx;

/* phase phi of a position estimate e^{2 pi i f / N} mapped to u = phi N / 2 pi
   and snapped to the lattice c + k B of class c (Subproblem 2, exact case) */
static int64_t lattice_of_phase(int64_t N, int64_t B, int64_t c, double phi) {
  int64_t L = N / B;
  if (phi < 0) phi += TWO_PI;
  double u = phi * (double)N / TWO_PI;
  double kf = floor((u - (double)c) / (double)B + 0.5);
  int64_t k = (int64_t)kf % L;
  if (k < 0) k += L;
  return k;
}

/* phase of sum over rounds and adjacent delays of Y[d+1] conj(Y[d]), with the
   advance-shift sign, snapped to the class lattice */
static int64_t snap_index(const cls_ctx *x, const cplx *Y, int64_t c, int64_t B) {
  const orc_cfg *cf = x->c;
  cplx P = 0;
  for (int r = 0; r < x->rounds; r++)
    for (int d = 0; d + 1 < cf->D; d++)
      P += Y[r * cf->D + d + 1] * conj(Y[r * cf->D + d]);
  return lattice_of_phase(cf->N, B, c, atan2(cimag(P), creal(P)));
}

/* Kay's estimator (Eq. 21-22): the angle of e^{2 pi i f g / N} from m samples
   y_t spaced g apart, as the weighted mean of the m-1 phase differences
   Delta_t = angle(y_{t+1} conj y_t) with the parabolic weights
   w_t = 3m / (2(m^2 - 1)) (1 - ((2t - m + 2) / m)^2). */
static double kay_phase(const cplx *y, int m) {
  double th = 0;
  for (int t = 0; t + 1 < m; t++) {
    cplx p = y[t + 1] * conj(y[t]);
    double u = (2.0 * t - m + 2.0) / (double)m;
    double w = 3.0 * m / (2.0 * ((double)m * m - 1.0)) * (1.0 - u * u);
    th += w * atan2(cimag(p), creal(p));
  }
  return th;
}

double orc_kay_phase(const double *y, int32_t m) { return kay_phase((const cplx *)y, m); }

/* R-FFAST singleton estimator (Sect. 3.2, Subproblem 2, general case):
   iteration c estimates the angle of e^{2 pi i 2^c f / N} from its m delays
   r_c + 2^c t and halves the interval that holds f -- angle in [0, pi): the
   lower half -- starting from [0, N); the estimate is the lattice point
   c + kB nearest to the final interval's midpoint. */
static int64_t rffast_locate(const cls_ctx *x, const cplx *Y, int64_t c, int64_t B) {
  const orc_cfg *cf = x->c;
  int64_t N = cf->N, L = N / B;
  double lo = 0.0, len = (double)N;
  for (int it = 0; it < cf->rf_iters; it++) {
    double th = kay_phase(Y + it * cf->rf_m, cf->rf_m);
    if (th < 0) th += TWO_PI;
    len *= 0.5;
    if (th >= TWO_PI / 2) lo += len;
  }
  double mid = lo + 0.5 * len;
  int64_t k = (int64_t)floor((mid - (double)c) / (double)B + 0.5) % L;
  if (k < 0) k += L;
  return k;
}

/* matched filter |sum_i Y_i e^{-2 pi i f tau_i / N}|^2 */
static double match2(const cls_ctx *x, const cplx *Y, int64_t f) {
  int64_t N = x->c->N;
  cplx g = 0;
  for (int i = 0; i < x->n; i++) {
    int64_t t = (int64_t)mulmod((uint64_t)f, x->tau[i], (uint64_t)N);
    g += Y[i] * unit(t, N, -1);
  }
  return creal(g) * creal(g) + cimag(g) * cimag(g);
}

/* Two-ton solve of a class that failed the singleton test: the moment
   preserving problem of Sect. 3.1 with a = 2 (Steps 2-3, Method 1).  Within
   round r the delays give the moments m_d = Y[r][d] = sum_j p_j z_j^d with
   z_j = e^{2 pi i f_j / N} (p_j absorbs the round's shift), so the monic
   polynomial z^2 + c1 z + c0 with roots z_0, z_1 (Eq. 12) satisfies
   c0 m_d + c1 m_{d+1} = -m_{d+2} (Eq. 14) for every d <= D-3.  The equations
   of all rounds share C = (c0, c1) and are solved together in least squares
   (one round with D = 4 is Eq. 14 itself).  The roots of Method 1 give the
   two positions, each snapped to the class lattice c + kB; the values are
   the least-squares solution of the Vandermonde system (Eq. 9, Eq. 18) over
   every measurement of the class.  Accepted when the positions differ, both
   values clear the zero-ton level and the residual passes the single-ton
   bound. */
static void two_ton(const cls_ctx *x, const cplx *Y, int64_t c, int64_t B, double T0sq,
                    double T1sq, decision *v) {
  const orc_cfg *cf = x->c;
  int64_t N = cf->N;
  int n = x->n, D = cf->D;
  cplx g00 = 0, g01 = 0, g11 = 0, h0 = 0, h1 = 0;
  for (int r = 0; r < x->rounds; r++)
    for (int d = 0; d + 2 < D; d++) {
      cplx m0 = Y[r * D + d], m1 = Y[r * D + d + 1], rhs = -Y[r * D + d + 2];
      g00 += conj(m0) * m0;
      g01 += conj(m0) * m1;
      g11 += conj(m1) * m1;
      h0 += conj(m0) * rhs;
      h1 += conj(m1) * rhs;
    }
  double det = creal(g00) * creal(g11) - (creal(g01) * creal(g01) + cimag(g01) * cimag(g01));
  if (!(det > 1e-13 * creal(g00) * creal(g11))) return;
  cplx c0 = (g11 * h0 - g01 * h1) / det;
  cplx c1 = (g00 * h1 - conj(g01) * h0) / det;
  cplx disc = csqrt(c1 * c1 - 4.0 * c0);
  cplx z0 = (-c1 - disc) / 2.0, z1 = (-c1 + disc) / 2.0;
  int64_t f0 = c + lattice_of_phase(N, B, c, carg(z0)) * B;
  int64_t f1 = c + lattice_of_phase(N, B, c, carg(z1)) * B;
  if (f0 == f1) return;
  if (f1 < f0) {
    int64_t t = f0;
    f0 = f1;
    f1 = t;
  }
  /* values: normal equations of the two columns e^{+2 pi i f_j tau_i / N} */
  cplx s01 = 0, q0 = 0, q1 = 0;
  for (int i = 0; i < n; i++) {
    cplx e0 = unit((int64_t)mulmod((uint64_t)f0, x->tau[i], (uint64_t)N), N, +1);
    cplx e1 = unit((int64_t)mulmod((uint64_t)f1, x->tau[i], (uint64_t)N), N, +1);
    s01 += conj(e0) * e1;
    q0 += conj(e0) * Y[i];
    q1 += conj(e1) * Y[i];
  }
  double nn = (double)n;
  double dv = nn * nn - (creal(s01) * creal(s01) + cimag(s01) * cimag(s01));
  if (!(dv > 1e-9 * nn * nn)) return;
  cplx a0 = (nn * q0 - s01 * q1) / dv;
  cplx a1 = (nn * q1 - conj(s01) * q0) / dv;
  if (nn * (creal(a0) * creal(a0) + cimag(a0) * cimag(a0)) <= T0sq) return;
  if (nn * (creal(a1) * creal(a1) + cimag(a1) * cimag(a1)) <= T0sq) return;
  double rho2 = 0;
  for (int i = 0; i < n; i++) {
    cplx e0 = unit((int64_t)mulmod((uint64_t)f0, x->tau[i], (uint64_t)N), N, +1);
    cplx e1 = unit((int64_t)mulmod((uint64_t)f1, x->tau[i], (uint64_t)N), N, +1);
    cplx e = Y[i] - a0 * e0 - a1 * e1;
    rho2 += creal(e) * creal(e) + cimag(e) * cimag(e);
  }
  if (!(rho2 <= T1sq)) return;
  v->cls = ORC_DOUBLE;
  v->f = f0;
  v->a = a0;
  v->f2 = f1;
  v->a2 = a1;
}

static decision classify(const cls_ctx *x, const cplx *Y, int64_t c, int64_t B) {
  const orc_cfg *cf = x->c;
  int64_t N = cf->N, L = N / B;
  int n = x->n;
  decision v;
  v.cls = ORC_ZERO;
  v.f = -1;
  v.a = 0;
  v.f2 = -1;
  v.a2 = 0;
  double E2 = 0;
  for (int i = 0; i < n; i++) E2 += creal(Y[i]) * creal(Y[i]) + cimag(Y[i]) * cimag(Y[i]);
  double T0sq, T1sq;
  if (cf->mode == ORC_EXACT) {
    T0sq = cf->eps0 * cf->eps0 * x->sref2 * (double)n;
    T1sq = cf->eps1 * cf->eps1 * E2;
  } else {
    double sb2 = x->noise_var / (double)B;
    T0sq = sb2 * ((double)n + cf->zero_k * sqrt((double)n));
    T1sq = sb2 * ((double)(n - 1) + cf->single_k * sqrt((double)(n - 1)));
  }
  if (E2 <= T0sq) return v;
  /* locate */
  int64_t k;
  if (cf->kind == ORC_FFAST && cf->rf_iters > 0) {
    k = rffast_locate(x, Y, c, B);
  } else if (cf->mode == ORC_EXACT) {
    k = snap_index(x, Y, c, B);
  } else {
    int64_t lo, cnt;
    if (cf->window > 0 && cf->D >= 2 && 2 * (int64_t)cf->window + 1 < L) {
      lo = snap_index(x, Y, c, B) - cf->window;
      cnt = 2 * (int64_t)cf->window + 1;
    } else {
      lo = 0;
      cnt = L;
    }
    double best = -1.0;
    int64_t bestk = 0;
    for (int64_t o = 0; o < cnt; o++) {
      int64_t kk = ((lo + o) % L + L) % L;
      double m2 = match2(x, Y, c + kk * B);
      if (m2 > best || (m2 == best && kk < bestk)) {
        best = m2;
        bestk = kk;
      }
    }
    k = bestk;
  }
  int64_t f = c + k * B;
  /* value: least-squares mean of the de-rotated measurements */
  cplx a = 0;
  for (int i = 0; i < n; i++) {
    int64_t t = (int64_t)mulmod((uint64_t)f, x->tau[i], (uint64_t)N);
    a += Y[i] * unit(t, N, -1);
  }
  a /= (double)n;
  double rho2 = 0;
  for (int i = 0; i < n; i++) {
    int64_t t = (int64_t)mulmod((uint64_t)f, x->tau[i], (uint64_t)N);
    cplx e = Y[i] - a * unit(t, N, +1);
    rho2 += creal(e) * creal(e) + cimag(e) * cimag(e);
  }
  v.f = f;
  v.a = a;
  v.cls = (rho2 <= T1sq) ? ORC_SINGLE : ORC_MULTI;
  if (v.cls == ORC_MULTI && cf->mpp == 2) two_ton(x, Y, c, B, T0sq, T1sq, &v);
  return v;
}

static int cmp_double(const void *a, const void *b) {
  double x = *(const double *)a, y = *(const double *)b;
  return (x > y) - (x < y);
}

/* Time-domain noise variance.  The paper names the thresholds T0, T1 of the
   general sparse case without values (Sect. 3.2, Subproblem 1); this reading
   estimates sigma^2 from the level-0 entries.  B |yhat|^2 of a bucket holding
   only noise is exponential with mean sigma^2.  A fraction phi of the entries
   is expected to be noise only (phi = mean over entries of (1 - 1/B)^K); if
   the occupied entries lie above the p-quantile, p < phi, then the p-quantile
   of all entries is the (p/phi)-quantile of the exponential:
   sigma^2 = q_p / -ln(1 - p/phi), with p = min(1/4, phi/2). */
static double estimate_noise(double *pw, int64_t cnt, double phi) {
  double p = phi / 2 < 0.25 ? phi / 2 : 0.25;
  qsort(pw, (size_t)cnt, sizeof(double), cmp_double);
  int64_t at = (int64_t)(p * (double)(cnt - 1));
  return pw[at] / -log(1.0 - p / phi);
}

static void tree_taus(const orc_cfg *c, cls_ctx *x);

/* The decision rule alone, for tests: one tree class vector Y (R*D values,
   interleaved re, im, measured with the plan's round shifts and delays) of
   class c among B buckets through the classification above (Sect. 3.2,
   Subproblems 1-2), with the given reference power (exact mode) or
   time-domain noise variance (noisy mode).  Returns the class code; *f and
   a[0..1] receive the located position and value (two-ton: the first). */
int32_t orc_classify_tree(const orc_cfg *c, const double *Y, int64_t cls, int64_t B,
                          double sref2, double noise_var, int64_t *f, double *a) {
  cls_ctx cx;
  memset(&cx, 0, sizeof(cx));
  cx.c = c;
  tree_taus(c, &cx);
  cx.sref2 = sref2;
  cx.noise_var = noise_var;
  decision v = classify(&cx, (const cplx *)Y, cls, B);
  if (f) *f = v.f;
  if (a) {
    a[0] = creal(v.a);
    a[1] = cimag(v.a);
  }
  return v.cls;
}

/* The noise estimate of the general sparse case from cnt values B |yhat|^2
   (sorted in place) with expected noise-only fraction phi. */
double orc_estimate_noise(double *pw, int64_t cnt, double phi) { return estimate_noise(pw, cnt, phi); }

/* ------------------------------------------------------------------ */
/* Found list and finalisation (goal of Sect. 2.1: K positions, K values). */

typedef struct {
  int64_t *f;
  cplx *a;
  int64_t n, cap;
} found_list;

static void found_push(found_list *L, int64_t f, cplx a) {
  if (L->n == L->cap) {
    L->cap = L->cap ? 2 * L->cap : 64;
    L->f = (int64_t *)realloc(L->f, sizeof(int64_t) * (size_t)L->cap);
    L->a = (cplx *)realloc(L->a, sizeof(cplx) * (size_t)L->cap);
  }
  L->f[L->n] = f;
  L->a[L->n] = a;
  L->n++;
}

typedef struct {
  int64_t f;
  cplx a;
  double mag2;
} entry;

static int by_mag_then_index(const void *p, const void *q) {
  const entry *a = (const entry *)p, *b = (const entry *)q;
  if (a->mag2 != b->mag2) return a->mag2 > b->mag2 ? -1 : 1;
  return (a->f > b->f) - (a->f < b->f);
}

static int by_index(const void *p, const void *q) {
  const entry *a = (const entry *)p, *b = (const entry *)q;
  return (a->f > b->f) - (a->f < b->f);
}

static int64_t finalize(const orc_cfg *c, found_list *L, int64_t *out_idx,
                        double *out_val, orc_trace *tr) {
  entry *e = (entry *)malloc(sizeof(entry) * (size_t)(L->n + 1));
  for (int64_t i = 0; i < L->n; i++) {
    e[i].f = L->f[i];
    e[i].a = L->a[i];
    e[i].mag2 = creal(L->a[i]) * creal(L->a[i]) + cimag(L->a[i]) * cimag(L->a[i]);
  }
  int64_t cnt = L->n;
  if (cnt > c->K) {
    qsort(e, (size_t)cnt, sizeof(entry), by_mag_then_index);
    cnt = c->K;
  }
  qsort(e, (size_t)cnt, sizeof(entry), by_index);
  for (int64_t i = 0; i < c->K; i++) {
    if (i < cnt) {
      out_idx[i] = e[i].f;
      out_val[2 * i] = creal(e[i].a);
      out_val[2 * i + 1] = cimag(e[i].a);
    } else {
      out_idx[i] = -1;
      out_val[2 * i] = 0;
      out_val[2 * i + 1] = 0;
    }
  }
  if (tr) {
    tr->n_found = L->n;
    for (int64_t i = 0; i < L->n && i < 4096; i++) tr->order[i] = L->f[i];
  }
  free(e);
  return cnt;
}

/* ------------------------------------------------------------------ */
/* Level-0 measurement: tree classes take bin sigma_r c mod B0 of every
   round and delay; FFAST stage j takes bin h of every delay.          */

static void tree_taus(const orc_cfg *c, cls_ctx *x) {
  x->rounds = c->R;
  x->n = c->R * c->D;
  for (int r = 0; r < c->R; r++)
    for (int d = 0; d < c->D; d++)
      x->tau[r * c->D + d] = (c->shift[r] + (uint64_t)d) % (uint64_t)c->N;
}

/* class vectors of the open classes at one tree level, by definition */
static void tree_measure(const orc_cfg *c, const float *x, int64_t B,
                         const int64_t *cls, int64_t ncls, cplx *Y) {
  cplx *tw = twiddles(B);
  int n = c->R * c->D;
  for (int64_t q = 0; q < ncls; q++)
    for (int r = 0; r < c->R; r++) {
      int64_t h = (int64_t)mulmod(c->sigma[r], (uint64_t)cls[q], (uint64_t)B);
      for (int d = 0; d < c->D; d++) {
        uint64_t tau = (c->shift[r] + (uint64_t)d) % (uint64_t)c->N;
        Y[q * n + r * c->D + d] = bin_tw(x, c->N, B, c->sigma[r], tau, h, tw);
      }
    }
  free(tw);
}

int orc_level0(const orc_cfg *c, const float *x, double *out) {
  if (c->kind == ORC_TREE) {
    int64_t B = c->B0;
    int64_t *cls = (int64_t *)malloc(sizeof(int64_t) * (size_t)B);
    for (int64_t q = 0; q < B; q++) cls[q] = q;
    tree_measure(c, x, B, cls, B, (cplx *)out);
    free(cls);
  } else {
    cplx *o = (cplx *)out;
    for (int j = 0; j < c->R; j++) {
      int64_t B = c->stageB[j];
      cplx *tw = twiddles(B);
      for (int64_t h = 0; h < B; h++)
        for (int d = 0; d < c->D; d++) o[h * c->D + d] = bin_tw(x, c->N, B, 1, ffast_tau(c, d), h, tw);
      o += B * c->D;
      free(tw);
    }
  }
  return 0;
}

/* ------------------------------------------------------------------ */
/* Binary tree search (Sect. 3.3): start at level 0 with B0 buckets, classify
   every open class, record singletons, close zero-tons and open the two
   children c, c + B of each multi-ton at the next level.             */

static int cmp_i64(const void *a, const void *b) {
  int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
  return (x > y) - (x < y);
}

static int64_t solve_tree(const orc_cfg *c, const float *x, int64_t *out_idx,
                          double *out_val, orc_trace *tr) {
  cls_ctx cx;
  memset(&cx, 0, sizeof(cx));
  cx.c = c;
  tree_taus(c, &cx);
  int n = cx.n;
  int64_t B = c->B0;
  int64_t ncls = B;
  int64_t *cls = (int64_t *)malloc(sizeof(int64_t) * (size_t)ncls);
  for (int64_t q = 0; q < ncls; q++) cls[q] = q;
  cplx *Y = (cplx *)malloc(sizeof(cplx) * (size_t)(ncls * n));
  tree_measure(c, x, B, cls, ncls, Y);
  /* reference power and noise level from all level-0 entries */
  double s = 0;
  double *pw = (double *)malloc(sizeof(double) * (size_t)(ncls * n));
  for (int64_t i = 0; i < ncls * n; i++) {
    double p = creal(Y[i]) * creal(Y[i]) + cimag(Y[i]) * cimag(Y[i]);
    s += p;
    pw[i] = p * (double)B;
  }
  cx.sref2 = s / (double)(ncls * n);
  cx.noise_var = c->noise_var > 0 ? c->noise_var
                                   : estimate_noise(pw, ncls * n, pow(1.0 - 1.0 / (double)B, (double)c->K));
  free(pw);
  int64_t samples = (int64_t)n * B;
  found_list fl = {0, 0, 0, 0};
  int partial = 0;
  int level = 0;
  for (;;) {
    int64_t L = c->N / B;
    int64_t *next = (int64_t *)malloc(sizeof(int64_t) * (size_t)(2 * ncls + 1));
    int64_t nnext = 0;
    int nz = 0, ns = 0, nm = 0, nd = 0;
    for (int64_t q = 0; q < ncls; q++) {
      decision v = classify(&cx, Y + q * n, cls[q], B);
      if (v.cls == ORC_ZERO) {
        nz++;
      } else if (v.cls == ORC_SINGLE) {
        ns++;
        found_push(&fl, v.f, v.a);
      } else if (v.cls == ORC_DOUBLE) {
        nd++;
        found_push(&fl, v.f, v.a);
        found_push(&fl, v.f2, v.a2);
      } else {
        nm++;
        if (L >= 2 && level + 1 <= c->max_levels) {
          next[nnext++] = cls[q];
          next[nnext++] = cls[q] + B;
        } else {
          partial = 1;
        }
      }
    }
    if (tr && level < ORC_MAX_LEVELS) {
      tr->n_zero[level] = nz;
      tr->n_single[level] = ns;
      tr->n_multi[level] = nm;
      tr->n_double[level] = nd;
      /* nodes of the full layer holding energy: classes found non-empty here
         plus one node for each frequency resolved at a shallower level */
      tr->occupied[level] = (int32_t)(fl.n + nm);
      tr->levels = level;
    }
    free(cls);
    free(Y);
    if (nnext == 0) {
      free(next);
      break;
    }
    qsort(next, (size_t)nnext, sizeof(int64_t), cmp_i64);
    level++;
    samples += (int64_t)n * B; /* the B odd-offset samples of each round and delay */
    B *= 2;
    cls = next;
    ncls = nnext;
    Y = (cplx *)malloc(sizeof(cplx) * (size_t)(ncls * n));
    tree_measure(c, x, B, cls, ncls, Y);
  }
  if (tr) {
    tr->samples = samples;
    tr->sref2 = cx.sref2;
    tr->noise_var = cx.noise_var;
  }
  int64_t cnt = finalize(c, &fl, out_idx, out_val, tr);
  if (tr) tr->status = partial ? ORC_PARTIAL : ORC_OK;
  free(fl.f);
  free(fl.a);
  return cnt;
}

/* ------------------------------------------------------------------ */
/* FFAST peeling decoder (Sect. 3.2, Subproblem 3, Eq. 20), in Jacobi
   rounds: identify the active buckets on the state at the start of the
   round, keep each new frequency once (lowest stage, then lowest bucket),
   subtract every new frequency from its bucket in every stage, and make
   active the buckets that changed, minus those in which a singleton was
   identified this round.  Method 1 starts with every bucket active.
   Method 2 (the packet-erasure schedule) starts with the buckets of its
   start frequencies, so that the active set of round p is the frontier of
   the depth-(2p-1) trees grown from them in lock-step, and stops once K
   frequencies are identified; if the trees die out before that, the
   buckets they never reached join the next round.                    */

static int64_t solve_ffast(const orc_cfg *c, const float *x, int64_t *out_idx,
                           double *out_val, orc_trace *tr) {
  int S = c->R, D = c->D;
  int64_t N = c->N;
  int64_t off[ORC_MAX_STAGES + 1];
  off[0] = 0;
  for (int j = 0; j < S; j++) off[j + 1] = off[j] + c->stageB[j];
  int64_t nb = off[S];
  cplx *Y = (cplx *)malloc(sizeof(cplx) * (size_t)(nb * D));
  orc_level0(c, x, (double *)Y);
  double s = 0;
  double *pw = (double *)malloc(sizeof(double) * (size_t)(nb * D));
  for (int j = 0; j < S; j++)
    for (int64_t h = 0; h < c->stageB[j]; h++)
      for (int d = 0; d < D; d++) {
        cplx v = Y[(off[j] + h) * D + d];
        double p = creal(v) * creal(v) + cimag(v) * cimag(v);
        s += p;
        pw[(off[j] + h) * D + d] = p * (double)c->stageB[j];
      }
  cls_ctx cx;
  memset(&cx, 0, sizeof(cx));
  cx.c = c;
  cx.rounds = 1;
  cx.n = D;
  for (int d = 0; d < D; d++) cx.tau[d] = ffast_tau(c, d);
  cx.sref2 = s / (double)(nb * D);
  double phi = 0;
  for (int j = 0; j < S; j++)
    phi += (double)c->stageB[j] * pow(1.0 - 1.0 / (double)c->stageB[j], (double)c->K);
  phi /= (double)nb;
  cx.noise_var = c->noise_var > 0 ? c->noise_var : estimate_noise(pw, nb * D, phi);
  free(pw);

  int *last = (int *)malloc(sizeof(int) * (size_t)nb);
  char *active = (char *)malloc((size_t)nb);
  char *modified = (char *)malloc((size_t)nb);
  char *detected = (char *)malloc((size_t)nb);
  char *seen = (char *)malloc((size_t)nb);
  int64_t *nf = (int64_t *)malloc(sizeof(int64_t) * (size_t)nb);
  cplx *na = (cplx *)malloc(sizeof(cplx) * (size_t)nb);
  /* method 1 (genie-assisted peeling) identifies every bucket in the first
     peeling; method 2 (packet-erasure schedule) starts from the d buckets of
     each start frequency -- the trees N_V^1 of its start points -- and grows
     them along the buckets that the frequencies found change */
  int schedule = c->n_starts > 0;
  for (int64_t b = 0; b < nb; b++) {
    last[b] = -1;
    active[b] = !schedule;
    seen[b] = 0;
  }
  for (int i = 0; i < c->n_starts; i++)
    for (int j = 0; j < S; j++) active[off[j] + c->start_f[i] % c->stageB[j]] = 1;
  found_list fl = {0, 0, 0, 0};
  int round = 0, partial = 0, complete = 0;
  for (;;) {
    int any = 0;
    for (int64_t b = 0; b < nb && !any; b++) any = active[b];
    if (!any && schedule && fl.n < c->K) {
      /* the trees stopped short of K frequencies: every bucket none of them
         has reached joins the next peeling */
      for (int64_t b = 0; b < nb; b++) {
        active[b] = !seen[b];
        any |= active[b];
      }
    }
    if (!any) break;
    if (round == c->max_peel_rounds) {
      partial = 1;
      break;
    }
    int nz = 0, ns = 0, nm = 0, ident = 0;
    int64_t nnew = 0;
    memset(detected, 0, (size_t)nb);
    for (int j = 0; j < S; j++)
      for (int64_t h = 0; h < c->stageB[j]; h++) {
        int64_t b = off[j] + h;
        if (!active[b]) continue;
        ident++;
        seen[b] = 1;
        decision v = classify(&cx, Y + b * D, h, c->stageB[j]);
        last[b] = v.cls;
        if (v.cls == ORC_ZERO) nz++;
        if (v.cls == ORC_MULTI) nm++;
        if (v.cls != ORC_SINGLE) continue;
        ns++;
        detected[b] = 1;
        int dup = 0;
        for (int64_t i = 0; i < fl.n && !dup; i++) dup = (fl.f[i] == v.f);
        for (int64_t i = 0; i < nnew && !dup; i++) dup = (nf[i] == v.f);
        if (!dup) {
          nf[nnew] = v.f;
          na[nnew] = v.a;
          nnew++;
        }
      }
    if (tr && round < ORC_MAX_LEVELS) {
      tr->n_zero[round] = nz;
      tr->n_single[round] = ns;
      tr->n_multi[round] = nm;
      tr->ident[round] = ident;
      tr->levels = round + 1;
    }
    round++;
    if (nnew == 0) {
      if (!schedule) break;
      memset(active, 0, (size_t)nb); /* the trees died out: fall back as above */
      continue;
    }
    memset(modified, 0, (size_t)nb);
    for (int64_t i = 0; i < nnew; i++) {
      found_push(&fl, nf[i], na[i]);
      for (int j = 0; j < S; j++) {
        int64_t b = off[j] + nf[i] % c->stageB[j];
        for (int d = 0; d < D; d++) {
          int64_t t = (int64_t)mulmod((uint64_t)nf[i], cx.tau[d], (uint64_t)N);
          Y[b * D + d] -= na[i] * unit(t, N, +1);
        }
        modified[b] = 1;
      }
    }
    for (int64_t b = 0; b < nb; b++) active[b] = modified[b] && !detected[b];
    /* the schedule ends once K frequencies are identified */
    if (schedule && fl.n >= c->K) {
      complete = 1;
      break;
    }
  }
  for (int64_t b = 0; b < nb && !partial && !complete; b++)
    if (last[b] == ORC_MULTI) partial = 1;
  if (tr) {
    int64_t tot = 0;
    for (int j = 0; j < S; j++) tot += c->stageB[j];
    tr->samples = tot * D;
    tr->sref2 = cx.sref2;
    tr->noise_var = cx.noise_var;
  }
  int64_t cnt = finalize(c, &fl, out_idx, out_val, tr);
  if (tr) tr->status = partial ? ORC_PARTIAL : ORC_OK;
  free(fl.f);
  free(fl.a);
  free(last);
  free(active);
  free(modified);
  free(detected);
  free(seen);
  free(nf);
  free(na);
  free(Y);
  return cnt;
}

int64_t orc_solve(const orc_cfg *c, const float *x, int64_t *out_idx,
                  double *out_val, orc_trace *tr) {
  if (tr) memset(tr, 0, sizeof(*tr));
  /* the two-ton solve needs the tree, exact mode and at least two moment
     equations: rounds x (delays - 2) >= 2 */
  if (c->mpp != 0 && (c->mpp != 2 || c->kind != ORC_TREE || c->mode != ORC_EXACT ||
                      c->R * (c->D - 2) < 2))
    return -1;
  if (c->kind == ORC_TREE) return solve_tree(c, x, out_idx, out_val, tr);
  return solve_ffast(c, x, out_idx, out_val, tr);
}
