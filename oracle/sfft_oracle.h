/*
 * sfft_oracle.h -- interface of the plain FP64 CPU oracle for the
 * aliasing-filter sparse FFT (Li, Jiang & Chen, "On Performance of Sparse
 * Fast Fourier Transform Algorithms Using the Aliasing Filter", 2020).
 *
 * TEST INFRASTRUCTURE ONLY.  This header, its C file and the Python wrapper
 * beside it exist to check the GPU library.  Only the test-suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load it.  It shares no
 * code, header, table or constant with the GPU library.
 */
#ifndef SFFT_ORACLE_H
#define SFFT_ORACLE_H
#include <stdint.h>

#define ORC_MAX_ROUNDS 16
#define ORC_MAX_STAGES 8
#define ORC_MAX_LEVELS 64
#define ORC_MAX_STARTS 64

enum { ORC_EXACT = 0, ORC_NOISY = 1 };
enum { ORC_TREE = 0, ORC_FFAST = 1 };
enum { ORC_ZERO = 0, ORC_SINGLE = 1, ORC_MULTI = 2, ORC_DOUBLE = 3 };
enum { ORC_OK = 0, ORC_PARTIAL = 1 };

typedef struct {
  int64_t N, K;
  int32_t kind;        /* ORC_TREE (N a power of two) or ORC_FFAST (co-prime stages) */
  int32_t mode;        /* ORC_EXACT or ORC_NOISY */
  int32_t R;           /* rounds (tree) or stages (FFAST) */
  int32_t D;           /* consecutive delays per round / stage */
  int64_t B0;          /* tree: buckets at level 0 */
  int64_t stageB[ORC_MAX_STAGES];     /* FFAST: buckets per stage */
  uint64_t sigma[ORC_MAX_ROUNDS];     /* odd permutation factor per round */
  uint64_t shift[ORC_MAX_ROUNDS];     /* random shift per round */
  int32_t max_levels;  /* tree: deepest level that may be opened */
  int32_t window;      /* noisy locator: +-window around the phase estimate, 0 = all L */
  int32_t max_peel_rounds;
  double eps0, eps1;   /* exact-mode relative thresholds */
  double zero_k, single_k;  /* noisy-mode threshold widths (in noise std units) */
  double noise_var;    /* > 0: time-domain noise variance given, else estimated */
  int32_t mpp;         /* tree, exact mode: 2 = resolve two-tons by the moment
                          preserving solve (Sect. 3.1, a_m = 2); 0 = off */
  int32_t rf_iters;    /* FFAST: C > 0 = R-FFAST delays and singleton estimator
                          (Sect. 3.2, Subproblem 2, general case): D = C * rf_m
                          delays r_c + 2^c t (c < C, t < rf_m) per stage */
  int32_t rf_m;
  uint64_t rf_off[ORC_MAX_ROUNDS];     /* r_c, SplitMix64 draws mod N */
  int32_t n_starts;    /* FFAST: 0 = every bucket in the first peeling (method 1);
                          > 0 = packet-erasure schedule (method 2) grown from the
                          buckets of these start frequencies */
  int64_t start_f[ORC_MAX_STARTS];
} orc_cfg;

typedef struct {
  int32_t status;
  int32_t levels;                      /* tree: deepest level classified; FFAST: peeling rounds */
  int32_t n_zero[ORC_MAX_LEVELS];      /* per tree level or per peeling round */
  int32_t n_single[ORC_MAX_LEVELS];
  int32_t n_multi[ORC_MAX_LEVELS];
  int32_t occupied[ORC_MAX_LEVELS];    /* tree: occupied nodes of the full layer (m_d) */
  int32_t ident[ORC_MAX_LEVELS];       /* buckets identified per peeling round */
  int64_t samples;                     /* signal samples read (with multiplicity) */
  double sref2;                        /* mean |bucket|^2 at level 0 */
  double noise_var;                    /* time-domain noise variance used */
  int64_t n_found;                     /* before the top-K cut */
  int64_t order[4096];                 /* discovery order of the first frequencies found */
  int32_t n_double[ORC_MAX_LEVELS];    /* tree: classes resolved as two-tons per level */
} orc_trace;

int orc_config(orc_cfg *c, int64_t N, int64_t K, int32_t stages, int32_t delays,
               uint64_t seed, int32_t mode, int64_t B0, int32_t identity_round0);
int orc_config_stages(orc_cfg *c, int64_t N, int64_t K, int32_t nstages,
                      const int64_t *stageB, int32_t delays, int32_t mode);
uint64_t orc_splitmix64_next(uint64_t *state);
/* start frequencies of the packet-erasure schedule: count SplitMix64 draws
   from seed, each reduced modulo N */
int orc_draw_starts(orc_cfg *c, uint64_t seed, int32_t count);
/* R-FFAST delay set of an FFAST plan: C iterations of m delays r_c + 2^c t;
   r_c are the first C SplitMix64 draws from seed (start frequencies, if any,
   are drawn after them), each mod N */
int orc_set_rffast(orc_cfg *c, uint64_t seed, int32_t C, int32_t m);
/* Kay's weighted phase-difference estimate (Eq. 21-22) from m complex
   samples (interleaved re, im); returns the angle in (-pi, pi] */
double orc_kay_phase(const double *y, int32_t m);

/* One bin of the B-point filtered spectrum of Eq. 5-6 (advance shift tau). */
void orc_bin(const float *x, int64_t N, int64_t B, uint64_t sigma, uint64_t tau,
             int64_t h, double *out_re_im);
/* Level-0 class table: out[c][i] (interleaved re,im), n = R*D (tree) or
   the per-stage tables concatenated stage by stage (FFAST). */
int orc_level0(const orc_cfg *c, const float *x, double *out);
/* The decision rule of Sect. 3.2 (Subproblems 1-2) on one tree class vector
   (n = R*D values, interleaved) of class cls among B buckets; returns the
   class code (ORC_ZERO .. ORC_DOUBLE), *f and a[2] the position and value. */
int32_t orc_classify_tree(const orc_cfg *c, const double *Y, int64_t cls, int64_t B,
                          double sref2, double noise_var, int64_t *f, double *a);
/* Noise variance estimate from cnt values B |yhat|^2 (sorted in place) and the
   expected noise-only fraction phi of the entries. */
double orc_estimate_noise(double *pw, int64_t cnt, double phi);
int64_t orc_solve(const orc_cfg *c, const float *x, int64_t *out_idx,
                  double *out_val, orc_trace *tr);
#endif
