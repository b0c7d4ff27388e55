/*
 * sfft.h -- C-ABI of the MI355X (gfx950) aliasing-filter sparse FFT library.
 *
 * Problem (Li, Jiang & Chen 2020, Sect. 2.1): given a signal x of N complex
 * samples whose spectrum xhat = F_N x (Eq. 1-2, F_N carries 1/N) is K-sparse,
 * return K frequency positions f_0..f_{K-1} and their values xhat_{f_j}.
 *
 * Method: frequency bucketization with the aliasing filter (Sect. 2.2,
 * Eq. 3-6): for every round (or stage) and every delay, subsample x with
 * stride L = N/B after a shift, take the B-point DFT, and read bucket c.
 * Reconstruction (Sect. 3.2-3.3): each bucket vector is tested as zero-ton /
 * single-ton / multi-ton; a single-ton is located from the phase of adjacent
 * delays (exact mode) or by enumeration of its L candidates (noisy mode), and
 * its value is the least-squares mean of the de-rotated measurements.  When N
 * is a product of co-prime prime powers the library runs the FFAST peeling
 * decoder (Sect. 3.2, Eq. 19-20); when N is a power of two it runs the binary
 * tree search (Sect. 3.3, Eq. 23), opening the two children c and c + B of
 * every multi-ton at the next level; optionally a multi-ton is first tried as
 * a two-ton by the moment preserving solve of Sect. 3.1.
 *
 * Conventions.  Samples use an advance shift, y[m] = x[(sigma m L + s + d)
 * mod N]; bucket c then holds sum_{f = c mod B} xhat_f e^{+2 pi i f (s+d)/N}
 * (Eq. 6 with tau -> -tau).  Values are in the 1/N scale of Eq. 2, so a tone
 * x[n] = a e^{2 pi i f n / N} is reported as a.  Signals and values are
 * interleaved complex64 (float re, float im).
 *
 * Memory.  Every pointer passed to an exec call is a DEVICE pointer (memory
 * of the current HIP device); the library never reads or writes host memory
 * through them and returns SFFT_EINVAL for a host pointer.  Buffers stay
 * owned by the caller and must stay valid until the work completes on the
 * stream.  Plans own their device tables and workspace, created on first use
 * on a device and released by sfft_destroy.  One exec may be in flight per
 * plan; concurrent solves use separate plans or one sfft_exec_batch call.
 *
 * Errors.  Functions that return a pointer return NULL on error; functions
 * that return an integer return a negative SFFT_E* code.  The last code is
 * also kept per thread (sfft_last_error).  A decoding failure is not an
 * error: the solve reports status SFFT_PARTIAL and the frequencies it found.
 */
#ifndef SFFT_H
#define SFFT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SFFT_MAX_ROUNDS 16
#define SFFT_MAX_STAGES 8
#define SFFT_MAX_PEEL_STARTS 64

/* error codes (negative returns) */
#define SFFT_OK 0
#define SFFT_EINVAL (-1)       /* bad argument: B does not divide N, K < 1, K > N,
                                  delays < 2 in exact mode, a host pointer, ... */
#define SFFT_EUNSUPPORTED (-2) /* N not factorable into `stages` co-prime parts,
                                  a size beyond the kernels' limits */
#define SFFT_ENOMEM (-3)       /* device allocation failed */
#define SFFT_EDEVICE (-4)      /* HIP runtime or kernel launch error */
#define SFFT_ETOOBIG (-5)      /* sfft_exec_noalloc: the plan's workspace exceeds
                                  the static scratch (SFFT_NOALLOC_SCRATCH_MIB) */

/* solve status (per signal) */
#define SFFT_STATUS_OK 0
#define SFFT_STATUS_PARTIAL 1  /* an unresolved multi-ton remained (decode failure,
                                  level cap or list overflow); found subset returned */

/* decoding modes */
#define SFFT_EXACT 0 /* exactly sparse: relative zero / single thresholds,
                        phase-to-index location (Sect. 3.2, Subproblem 2) */
#define SFFT_NOISY 1 /* general sparse: noise-scaled thresholds T0, T1 and
                        enumeration of the L candidates (Sect. 3.1, Method 2) */

/* signal storage (sfft_params_t.sample_format) */
#define SFFT_SAMPLES_C64 0   /* interleaved complex64 */
#define SFFT_SAMPLES_F16 1   /* packed FP16 with a per-signal scale (sfft_pack_fp16) */
#define SFFT_F16_HEADER_BYTES 16

/* plan kinds */
#define SFFT_KIND_TREE 0  /* N a power of two: binary tree search */
#define SFFT_KIND_FFAST 1 /* N a product of co-prime stages: peeling */

typedef struct sfft_plan_s *sfft_plan_t;

/* Full parameter record.  sfft_params_init fills the defaults below. */
typedef struct {
  int64_t N;               /* signal length */
  int64_t K;               /* sparsity = capacity of out_idx / out_val */
  int32_t stages;          /* FFAST: co-prime stages; tree: rounds */
  int32_t delays;          /* D consecutive delays {0..D-1} per round/stage */
  uint64_t seed;           /* SplitMix64 seed of the per-round sigma, shift */
  int32_t mode;            /* SFFT_EXACT (default) or SFFT_NOISY */
  int64_t B0;              /* tree: level-0 buckets (power of two);
                              0 = next power of two >= 2K, capped at N */
  int32_t max_levels;      /* tree: deepest level; -1 = log2(N/B0) (to L = 1) */
  int32_t window;          /* noisy: search +-window candidates around the phase
                              estimate; 0 = all L candidates */
  int32_t identity_round0; /* tree: round 0 uses sigma = 1, shift = 0 */
  int32_t nstage_B;        /* FFAST: 0 = factor N into prime powers; else the
                              number of explicit co-prime stage sizes below */
  int64_t stage_B[SFFT_MAX_STAGES];
  int32_t max_peel_rounds; /* FFAST: cap on peeling rounds (default 64) */
  int32_t jump_L;          /* tree: once a level's stride L' <= jump_L (a power of two
                              <= 128), resolve each open class's whole subtree from
                              its L' coefficients, measured by one dense pass over x;
                              every later level's class vectors are the same linear
                              functionals of x as the level-by-level gathers.
                              0 = level by level to the end (default 128) */
  double eps0;             /* exact: zero-ton if |Y|^2 <= eps0^2 sref^2 n (1e-4) */
  double eps1;             /* exact: single-ton if residual^2 <= eps1^2 |Y|^2 (1e-4) */
  double zero_k;           /* noisy: T0^2 = s_b^2 (n + zero_k sqrt(n))        (4) */
  double single_k;         /* noisy: T1^2 = s_b^2 (n-1 + single_k sqrt(n-1)) (4) */
  double noise_var;        /* noisy: time-domain noise variance; 0 = estimate */
  int32_t mpp;             /* tree, exact mode: 2 = a class that fails the single-ton
                              test is tried as a two-ton by the moment preserving
                              solve (Sect. 3.1 with a = 2: Eq. 12-14 pooled over the
                              rounds, Method 1 roots, Eq. 9 values) and closed when
                              it fits; needs rounds x (delays - 2) >= 2, else
                              SFFT_EINVAL; noisy mode or FFAST: SFFT_EUNSUPPORTED.
                              0 = off (default) */
  int32_t precision;       /* 0 (default): phase-to-index, values and residuals in FP64 on
                              FP32 buckets; 1: all in FP32 (the precision study of the
                              N = 2^24, K = 4096 workload); the two-ton solve stays
                              FP64.  Tree plans only (FFAST: SFFT_EUNSUPPORTED); other
                              values: SFFT_EINVAL */
  int32_t rf_iters;        /* FFAST: C in 1..16 selects the R-FFAST delay set and singleton
                              estimator (Sect. 3.2, Subproblem 2, general case): each stage
                              is measured at the C * rf_m delays r_c + 2^c t (c < C,
                              t < rf_m; r_c = the first C SplitMix64 draws from `seed`,
                              each mod N), replacing `delays`; a bucket's frequency is
                              found by C halvings of [0, N), halving c deciding from the
                              angle of e^{2 pi i 2^c f / N} estimated by Kay's weighted
                              phase differences (Eq. 21-22), then snapped to the bucket's
                              lattice.  Needs rf_m >= 2 and C * rf_m <= 64, else
                              SFFT_EINVAL; tree plans: SFFT_EUNSUPPORTED.  0 = off */
  int32_t rf_m;            /* R-FFAST: delays per iteration (m) */
  int32_t peel_starts;     /* FFAST: 0 = genie-assisted peeling, every bucket identified
                              in the first peeling (Sect. 3.2, Subproblem 3, method 1;
                              default).  S in 1..SFFT_MAX_PEEL_STARTS = packet-erasure
                              schedule (method 2): peeling grows from the buckets of S
                              start frequencies, one depth of their trees per round, and
                              stops once K frequencies are found; if the trees die out
                              first, the buckets they never reached join the next round.
                              Tree plans: SFFT_EUNSUPPORTED. */
  int64_t peel_start_f[SFFT_MAX_PEEL_STARTS];
                           /* the S start frequencies (each in [0, N)); all -1 (the
                              default) = S SplitMix64 draws from `seed` (after the
                              R-FFAST offsets, if any), each mod N; a mix of given
                              and -1 entries: SFFT_EINVAL */
  int32_t l1_resolve;      /* tree: 1 (default) = resolve every level-0 multi-ton at
                              level 1 from one pass over x: viewing x as B0 rows of
                              L = N/B0 samples, a B0-point DFT down each column gives
                              every class's L coefficients M_c(t) (the class's bucket
                              measured with shift t, times B0), and each class vector
                              of any later level (Sect. 3.3) is a sum of 2^d of them,
                              d levels below; taken when B0 is 512, 1024, 2048, 4096 or 8192 and
                              L >= max(32768 / B0, 16), in place of jump_L and the level-by-level
                              gathers.  0 = off; other values: SFFT_EINVAL */
  int32_t sample_format;   /* tree: SFFT_SAMPLES_C64 (default) = x holds N complex64;
                              SFFT_SAMPLES_F16 = x holds the packed FP16 form that
                              sfft_pack_fp16 writes (a 16-byte header whose first
                              float is a scale s, then N pairs (re, im) of IEEE
                              binary16, sample n = s (re + i im)): half the bytes of
                              the signal; every sum stays FP32.  FFAST plans and
                              sfft_exec_host: SFFT_EUNSUPPORTED */
  int32_t fft_tile_lg;     /* tree: log2 of the sub-FFT size of the level-0 transform
                              (the B0-point DFT of Eq. 6 taken as B0 / 2^fft_tile_lg
                              LDS-resident sub-FFTs combined by twiddles); 0 = the
                              largest that fits (2^13 / D rounded down to a power of
                              two, at most B0); else 5 .. that size's log2
                              (SFFT_EINVAL outside).  A launch-shape knob: results are
                              the same up to FP32 rounding */
  int32_t gather_unroll;   /* tree: strided sample loads each thread keeps in flight in
                              the level-0 and level gathers: 2, 4 (0 = default) or 8;
                              a batch takes the value of its first tree plan.  Results
                              are unchanged */
  int32_t col_form;        /* tree, level-1 column pass at B0 = 2048: 0 = the library's
                              choice (3 at B0 = 2048), 1 = 32 rows per thread (512-thread work-groups, a
                              32-point and a 64-point transform per column, items of 8
                              columns), 2 = 16 rows per thread (1024-thread work-groups,
                              transforms of 16, 8 and 16 points), 3 = 64 rows per thread
                              (512-thread work-groups, items of 16 columns read as
                              128-byte row segments, a 64-point and a 32-point
                              transform); other widths take form 1 (2 or 3 with another
                              B0: SFFT_EINVAL).  Results equal up to FP32 rounding */
  int32_t enum_share;      /* tree, noisy mode, levels below 0: where some class of a
                              batch has a candidate range longer than this many blocks
                              of 32 candidates, the classes of a wave that enumerate are
                              dealt to teams of lanes (a lone class gets the whole wave),
                              else each enumerates on its own lane (level 0 uses teams
                              for ranges over 64 blocks); 1 .. 64 (0 = 4, SFFT_EINVAL
                              outside).  A launch-shape knob: every candidate's
                              statistic is the same number either way, so results are
                              unchanged */
  int32_t l0_spread;       /* tree, noisy mode, level 0: lanes each class of the level-0
                              classification takes (1, 2, 4 or 8; 64 / it classes a wave),
                              the extra lanes joining the team enumeration; 0 = the
                              batch's choice: doubled from 1, up to 4, while the noisy
                              classes with ranges over enum_share blocks would fill at
                              most 8192 waves.  A batch takes the largest value its tree
                              plans fix (SFFT_EINVAL outside).  Results are unchanged */
} sfft_params_t;

/* Read-only description of a plan (what the kernels will compute). */
typedef struct {
  int64_t N, K;
  int32_t kind;            /* SFFT_KIND_TREE or SFFT_KIND_FFAST */
  int32_t mode;
  int32_t R;               /* rounds (tree) or stages (FFAST) */
  int32_t D;               /* delays */
  int64_t B0;              /* tree: level-0 buckets */
  int32_t max_levels;
  int32_t window;
  int64_t stage_B[SFFT_MAX_STAGES];   /* FFAST stage sizes */
  uint64_t sigma[SFFT_MAX_ROUNDS];    /* odd permutation factor per round */
  uint64_t shift[SFFT_MAX_ROUNDS];    /* shift per round */
  double eps0, eps1, zero_k, single_k, noise_var;
  int32_t max_peel_rounds;
  int32_t jump_L;
  int32_t found_cap;       /* device list capacities per signal */
  int32_t multi_cap;
  int32_t mpp;             /* two-ton solve (2) or off (0) */
  int32_t peel_starts;     /* FFAST schedule: start frequencies (0 = method 1) */
  int64_t peel_start_f[SFFT_MAX_PEEL_STARTS];
  int32_t rf_iters, rf_m;  /* R-FFAST delay set (rf_iters = 0: delays 0..D-1) */
  uint64_t rf_off[SFFT_MAX_ROUNDS];   /* r_c */
  int32_t precision;       /* 0: FP64 decisions, 1: FP32 */
  int32_t l1_resolve;      /* 1 when the level-1 column pass is taken */
  int32_t sample_format;   /* SFFT_SAMPLES_C64 or SFFT_SAMPLES_F16 */
  int32_t fft_tile_lg;     /* level-0 sub-FFT size in use (log2) */
  int32_t gather_unroll;   /* gather loads in flight per thread */
  int32_t col_form;        /* column-pass form in use (1, 2 or 3; 0 without the pass) */
  int32_t enum_share;      /* team enumeration above this many 32-candidate blocks */
  int32_t l0_spread;       /* level-0 lanes per class as set (0: the batch's choice) */
} sfft_plan_info_t;

/* Per-signal statistics of the last exec (host copy, see sfft_exec_stats). */
typedef struct {
  int64_t count;           /* frequencies returned */
  int32_t status;          /* SFFT_STATUS_* */
  int32_t levels;          /* tree: deepest level reached; FFAST: peeling rounds */
  int64_t samples;         /* signal samples read (with multiplicity) */
  int64_t found;           /* frequencies found before the top-K cut */
  double noise_var;        /* noise variance used (noisy mode) */
  double sref2;            /* mean level-0 bucket power */
  uint64_t level_mask;     /* tree: bit l set when level l gathered samples */
  int64_t ident;           /* FFAST: bucket identifications over all peeling rounds */
  int64_t h2d_bytes;       /* sfft_exec_host: sample bytes copied to the device */
} sfft_stats_t;

/* Defaults for (N, K, stages, delays, seed). */
void sfft_params_init(sfft_params_t *p, int64_t N, int64_t K, int32_t stages,
                      int32_t delays, uint64_t seed);

/* Plan from the problem statement; exact mode, defaults as above.  Host-only
   work (factoring, SplitMix64 draws); no device memory is touched until the
   first exec.  NULL on error (see sfft_last_error). */
sfft_plan_t sfft_plan(int64_t N, int64_t K, int32_t stages, int32_t delays, uint64_t seed);
sfft_plan_t sfft_plan_ex(const sfft_params_t *p);
int32_t sfft_plan_info(sfft_plan_t plan, sfft_plan_info_t *out);
void sfft_destroy(sfft_plan_t plan);

/* Synchronous solve on the null stream.  x: device complex64[N];
   out_idx: device int64[K]; out_val: device complex64[K].  Entries [count, K)
   are padded with index -1 and value 0.  Returns count >= 0 or SFFT_E*. */
int64_t sfft_exec(sfft_plan_t plan, const void *x, int64_t *out_idx, void *out_val);

/* Solve of a HOST-resident signal, for callers whose signals are not on the
   device: only the samples the solve reads cross to the device -- R*D*B0 at
   level 0, R*D*B' at each tree level it opens, D*sum B_j for FFAST (Sect. 2.2:
   a round costs B samples) -- instead of all N.  The samples are gathered on
   the host (up to 16 threads), copied through a pinned staging buffer and
   scattered into a device image of x on which the kernels of sfft_exec run,
   level by level: the host waits for each tree level's scheduling to learn
   whether the next level opens (one synchronisation per level).  The dense
   subtree pass is not used (it reads all of x); results otherwise follow the
   same rules as sfft_exec.  x: HOST complex64[N]; out_idx: HOST int64[K];
   out_val: HOST complex64[K] (pageable or pinned; device pointers are
   rejected with SFFT_EINVAL); stats: optional host record of the solve,
   with h2d_bytes set.  Synchronous, on an internal stream.  Returns count or
   SFFT_E*.  The plan keeps a device image of N samples and the staging
   buffers until sfft_destroy. */
int64_t sfft_exec_host(sfft_plan_t plan, const void *x, int64_t *out_idx, void *out_val,
                       sfft_stats_t *stats);

/* Asynchronous solve on `stream` (a hipStream_t; NULL = null stream).
   d_count: device int64[1], d_status: device int32[1] receive the result. */
int32_t sfft_exec_async(sfft_plan_t plan, const void *x, int64_t *out_idx, void *out_val,
                        int64_t *d_count, int32_t *d_status, void *stream);

/* Allocation-free form of sfft_exec_async, for callers that cannot allocate
   device memory (code under HIP graph capture, tight serving loops, harnesses
   that forbid hipMalloc).  It runs the same kernels on the same arguments,
   with the whole workspace -- the plan's descriptors, the level-0 buckets,
   class lists and found lists -- placed in one static device array of
   SFFT_NOALLOC_SCRATCH_MIB MiB that the library holds on every GPU it runs on
   until the process ends (the twiddle table sits in its first 64 KiB).  No
   hipMalloc, hipFree or other device allocation is made; the first call of a
   plan on a device computes the plan's workspace layout on the host, and the
   first call on a device writes the twiddle table (a synchronous copy).  Each
   call copies the plan's descriptors into the scratch on `stream`.
   x, out_idx, out_val, d_count, d_status: device pointers as for
   sfft_exec_async (d_count and d_status are required here).  A plan whose
   workspace (sfft_workspace: bytes) exceeds the scratch less 64 KiB is
   rejected with SFFT_ETOOBIG before anything is launched.  Every call on one
   GPU shares that GPU's scratch and leaves its contents behind (every value a
   call reads is written by the same call first): calls that overlap on one
   GPU -- on different streams or from different threads -- race and give
   undefined results; calls on one stream are ordered.  Returns SFFT_OK or
   SFFT_E*. */
#define SFFT_NOALLOC_SCRATCH_MIB 64
int32_t sfft_exec_noalloc(sfft_plan_t plan, const void *x, int64_t *out_idx, void *out_val,
                          int64_t *d_count, int32_t *d_status, void *stream);

/* Batched solve of n independent signals (any mix of plans, N and K) in one
   fused pipeline: one persistent level-0 launch over all signals and one
   launch per tree level, replayed from a captured HIP graph when the same
   plan list is used again.  xs[i], idx[i], vals[i] are device pointers;
   d_counts: device int64[n]; d_status: device int32[n]. */
#define SFFT_BATCH_NO_GRAPH 1 /* launch eagerly instead of replaying a graph */
int32_t sfft_exec_batch(const sfft_plan_t *plans, const void *const *xs,
                        int64_t *const *idx, void *const *vals, int64_t *d_counts,
                        int32_t *d_status, int32_t n, void *stream);
int32_t sfft_exec_batch_ex(const sfft_plan_t *plans, const void *const *xs,
                           int64_t *const *idx, void *const *vals, int64_t *d_counts,
                           int32_t *d_status, int32_t n, void *stream, int32_t flags);

/* Profiling form of sfft_exec_batch: runs the same pipeline eagerly on the
   batch's internal stream with a timing event after every kernel launch, waits
   for it, and writes the elapsed milliseconds of up to `cap` launches to ms[]
   and their kernel ids (SFFT_KERNEL_* | level << 8) to kernel[].  Returns the
   number of entries or SFFT_E*. */
#define SFFT_KERNEL_RESET 0
#define SFFT_KERNEL_LEVEL0 1        /* level-0 gather + FFT + classify (and FFAST peel) */
#define SFFT_KERNEL_SCHED 2
#define SFFT_KERNEL_EXPAND_FFT 3    /* odd-offset gather + LDS FFT, B' <= 8192 */
#define SFFT_KERNEL_EXPAND_DIRECT 4 /* odd-offset gather + per-bin partial sums */
#define SFFT_KERNEL_CHILDREN 5
#define SFFT_KERNEL_FINALIZE 6
#define SFFT_KERNEL_JUMP_PASS 7     /* dense pass: L' coefficients of each open class */
#define SFFT_KERNEL_JUMP_RESOLVE 8  /* subtree classification from the coefficients */
#define SFFT_KERNEL_COL_PASS 9      /* level-1 column DFTs: M_c(t) of every open class */
#define SFFT_KERNEL_COL_RESOLVE 10  /* classification of every later level from M_c(t) */
#define SFFT_KERNEL_COL_DEEP 11     /* classes open below half depth: an L-point FFT of the row */
int32_t sfft_exec_batch_profile(const sfft_plan_t *plans, const void *const *xs,
                                int64_t *const *idx, void *const *vals, int64_t *d_counts,
                                int32_t *d_status, int32_t n, float *ms, int32_t *kernel,
                                int32_t cap);

/* Packed FP16 form of a complex64 signal, for plans with sample_format =
   SFFT_SAMPLES_F16: out (device, SFFT_F16_HEADER_BYTES + 4 N bytes) receives
   a header whose first float is the scale s = 2^(e - 15), e the exponent with
   2^(e-1) <= m < 2^e for the largest component magnitude m of x (s = 1 when
   x = 0), so every scaled component lies below 2^15 and inside binary16's
   range whatever the signal's level; then sample n as the binary16 values of
   re / s and im / s, rounded to nearest even.  Bytes 4..15 of the header
   are scratch of the routine.  x: device complex64[N].  Asynchronous on
   `stream` (NULL = null stream).  Returns SFFT_OK or SFFT_E*. */
int32_t sfft_pack_fp16(const void *x, int64_t N, void *out, void *stream);

/* Bucketization alone (Eq. 5-6, level 0): out (device complex64) receives,
   for a tree plan, B0 class vectors of R*D values (class-major: out[c*R*D +
   r*D + d] = bucket sigma_r c mod B0 of round r, delay d); for an FFAST plan,
   the stages one after another, out[(off_j + h)*D + d].  Synchronous on the
   null stream.  Returns SFFT_OK or SFFT_E*. */
int32_t sfft_bucketize(sfft_plan_t plan, const void *x, void *out);

/* Statistics of the last exec / exec_async of `plan` (synchronises), or of
   signal i of the last sfft_exec_batch with that plan list (i < n). */
int32_t sfft_exec_stats(sfft_plan_t plan, sfft_stats_t *out);
int32_t sfft_batch_stats(const sfft_plan_t *plans, int32_t n, int32_t i, sfft_stats_t *out);

/* Device workspace of a batch, computed on the host from the plans alone (no
   device call, no allocation): the size of the one device slab that an exec
   of this plan list works in, and the element count of each arena in it --
   for admission by HBM footprint and for checking the kernels' indexing
   against what is allocated.  The workspace holds the level-0 buckets of
   Eq. 5-6, the class lists of the tree search (Sect. 3.3) and the peeling
   state (Sect. 3.2, Eq. 20).  sig (optional) receives n per-signal records.
   Returns SFFT_OK or SFFT_EINVAL. */
typedef struct {
  int64_t bytes;       /* device slab of the batch */
  int64_t y0;          /* level-0 planes, complex64 */
  int64_t fst;         /* FFAST peeling state, complex128 */
  int64_t found;       /* found-list slots (int64 position + complex128 value) */
  int64_t multi;       /* multi-ton slots per level parity */
  int64_t multi_vec;   /* class-vector entries per level parity (multi x nmax) */
  int64_t jacc;        /* dense-pass coefficients, complex128 (multi x jstride, or 0) */
  int64_t jcol;        /* column-pass rows, complex64 */
  int32_t nmax;        /* class-vector stride of the multi-ton arenas */
  int32_t jstride;     /* dense-pass coefficients per multi-ton slot */
  int32_t levels;      /* tree levels launched after level 0 */
  int32_t nsig;
} sfft_workspace_t;

typedef struct {
  int64_t y0_off, fst_off, found_off, multi_off, jcol_off;  /* element offsets */
  int32_t found_cap, multi_cap;
  int32_t n;           /* measurements per class vector */
  int32_t l1;          /* 1: takes the level-1 column pass */
  int32_t jump_L;      /* dense-pass stride in effect (0: off) */
  int32_t col_rows;    /* column-pass rows reserved (l1 only): the expected level-0
                          multi-tons x 1.5 + 64, at most multi_cap; open classes
                          beyond them leave the signal PARTIAL */
} sfft_workspace_signal_t;

int32_t sfft_workspace(const sfft_plan_t *plans, int32_t n, sfft_workspace_t *out,
                       sfft_workspace_signal_t *sig);

/* ------------------------------------------------------------ serving loop
   Continuous batching of independent solves, each the problem of Sect. 2.1,
   on the current device.  A request names a plan (created once by the caller
   and reused: plans stay resident), device pointers to its signal and outputs
   (as for sfft_exec_async) and a release time.  A scheduler thread forms a
   batch whenever one of `lanes` lanes is free and released requests wait:
   it takes them in release order while their workspaces (sfft_workspace,
   computed on the host from the plans) fit the lane's share of `hbm_bytes`
   of device memory -- admission by HBM footprint -- and launches the batched
   pipeline of sfft_exec_batch on the lane's own stream.  Lanes run at the
   same time, so requests that arrive while batches are on the device are
   admitted into the next free lane and their work overlaps with the batches
   in flight.  Each request's result equals that of sfft_exec on the same
   plan and signal.  The server owns its lanes' streams, slabs and pinned
   staging buffers (allocated at creation) and two threads per lane plus one;
   the caller owns plans and buffers, which must stay valid until the request
   is done.  Requests are numbered from 0 in submission order (tickets). */
typedef struct sfft_server_s *sfft_server_t;

typedef struct {
  int64_t hbm_bytes;   /* device memory for batch workspaces, split evenly over the
                          lanes (default 8 GiB; at least 1 MiB per lane) */
  int32_t lanes;       /* batches in flight at once, one stream each (1..8, default 2) */
  int32_t max_batch;   /* requests per batch (1..65536, default 256) */
} sfft_server_params_t;

/* Times (sfft_server_clock_ns) and outcome of one request. */
typedef struct {
  int64_t release_ns;  /* when the request became eligible for a batch */
  int64_t launch_ns;   /* when its batch was launched (0 before) */
  int64_t done_ns;     /* when its batch's completion was observed (0 before) */
  int32_t batch;       /* requests in its batch */
  int32_t lane;
  int32_t status;      /* 0 waiting or running, 1 done, < 0 the SFFT_E* its batch failed with */
  int32_t pad;
} sfft_request_t;

void sfft_server_params_init(sfft_server_params_t *p);
/* NULL on error: SFFT_EINVAL (parameters), SFFT_ENOMEM, SFFT_EDEVICE. */
sfft_server_t sfft_server_create(const sfft_server_params_t *p);
/* The server's clock (monotonic nanoseconds), for release times. */
int64_t sfft_server_clock_ns(void);
/* Queue n requests: plans[i] with device pointers xs[i], idx[i], vals[i],
   d_counts + i, d_status + i, eligible from release_ns[i] (server clock; 0 or
   a NULL array = now).  tickets (optional) receives their numbers.  A request
   whose workspace alone exceeds a lane's share is rejected with SFFT_ETOOBIG
   and nothing is queued.  Returns SFFT_OK or SFFT_E*. */
int32_t sfft_server_submit_many(sfft_server_t s, int32_t n, const sfft_plan_t *plans,
                                const void *const *xs, int64_t *const *idx, void *const *vals,
                                int64_t *d_counts, int32_t *d_status, const int64_t *release_ns,
                                int64_t *tickets);
/* One request; returns its ticket (>= 0) or SFFT_E*. */
int64_t sfft_server_submit(sfft_server_t s, sfft_plan_t plan, const void *x, int64_t *out_idx,
                           void *out_val, int64_t *d_count, int32_t *d_status, int64_t release_ns);
/* Records of tickets first .. first + n - 1. */
int32_t sfft_server_requests(sfft_server_t s, int64_t first, int32_t n, sfft_request_t *out);
/* Block until one request, or every request submitted so far, is done. */
int32_t sfft_server_wait(sfft_server_t s, int64_t ticket);
int32_t sfft_server_drain(sfft_server_t s);
/* Waits for every submitted request, then releases the server. */
void sfft_server_destroy(sfft_server_t s);

/* Release every cached batch context (graphs, workspaces). */
void sfft_release_batches(void);

int32_t sfft_last_error(void);
const char *sfft_strerror(int32_t code);

#ifdef __cplusplus
}
#endif
#endif
