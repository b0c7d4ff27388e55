// sfft_internal.h -- layouts shared by the host driver and the gfx950 kernels
// of the aliasing-filter sparse FFT library (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/sfft.h"

namespace sfft {

constexpr int kThreads = 256;        // work-group size of most kernels
constexpr int kPre = 7;              // prefix arrays of the per-level work
constexpr int kFftMax = 8192;        // largest LDS-resident pow2 FFT (64 KiB complex64)
constexpr int kLog2FftMax = 13;
constexpr int kDirectMax = 2048;     // largest non-pow2 stage (direct DFT in LDS)
constexpr int kChunk = 2048;         // samples per direct partial-sum work item
constexpr int kPerThread = kChunk / kThreads;
constexpr int kMaxD = 4;             // delays handled by the direct partial-sum kernel
constexpr int kMaxMeas = 64;         // rounds x delays per class vector
constexpr int kMaxFfastBuckets = 4096;
constexpr int kJumpMax = 128;        // largest stride L' resolved by the dense pass
constexpr int kJumpItemRows = 4096;  // rows of L' elements per dense-pass work item (large batches)
constexpr int kJumpItemRowsMin = 256; // ... and for a single signal (more work-groups per signal)
constexpr int kJumpBlockRows = 256;  // rows whose twiddles share one LDS table (VALU form)
constexpr int kJumpMfmaClasses = 16; // classes per MFMA pass (32 output rows: re, im)
constexpr int kJumpMfmaMinLg = 7;    // dense passes with L' = 128 run on the matrix cores
constexpr int kSplitMinBins = 4;     // parents from which B' > kFftMax uses split FFTs
constexpr int kColThreads = 512;     // work-group of the level-1 column pass
constexpr int kColQ = 32;            // column pass: B0 = P x 32, 32 rows per thread
constexpr int kColItemAlign = 8;     // column pass: each signal's item range padded to a multiple of this
constexpr int kColResolveCap = 128;  // open subclasses per depth of one class
constexpr int kColGroupLg = 3;      // column resolve: 2^3 lanes per class
constexpr int kColGroup = 1 << kColGroupLg;
constexpr int kColResolveAlign = 64 / kColGroup;  // ... classes a wave: each signal's range padded to it
constexpr int kColLaneDepth = 5;    // ... one lane per class-vector sum down to this depth
constexpr int kDeepNodes = 512;     // deep resolution: subtree nodes classified per round
constexpr int kDeepTw = 128;        // ... its twiddle table: L / 2^(Dz + 1) <= 8192 / 64 entries
constexpr int kEnumLaneBlocks = 64; // largest value of a plan's enum_share: noisy classes whose candidate
                                    // ranges are at most that many blocks of 32 enumerate one lane a
                                    // class, longer ones in teams of lanes
constexpr int kEnumShareDefault = 4; // ... unless the plan says otherwise
constexpr int kL0SpreadMax = 8;      // level-0 classification: at most this many lanes per class
constexpr int kL0SpreadAuto = 4;     // ... the batch's own choice: doubled up to this while the
constexpr int kL0SpreadWaves = 8192; // noisy classes fill at most this many waves (eight per SIMD)
constexpr size_t kNoAllocScratchBytes = (size_t)SFFT_NOALLOC_SCRATCH_MIB << 20;
constexpr size_t kNoAllocTwBytes = 64 * 1024;  // twiddle table at the scratch's start

// log2 of the sub-FFT size used when the D delays of a sample are held in
// LDS together (D planes of complex64 within 64 KiB)
__host__ __device__ inline int split_lg(int D) {
  return kLog2FftMax - (D <= 1 ? 0 : (D <= 2 ? 1 : 2));
}

// Static description of one signal of a batch (from its plan).
struct SigDesc {
  int64_t N, K, B0;
  int32_t log2N;          // -1 when N is not a power of two
  int32_t log2B0;
  int32_t kind, mode, R, D, n;
  int32_t max_levels, window, nstages, max_peel_rounds;
  int32_t found_cap, multi_cap;
  int32_t jump_L;
  int32_t l1;             // level-0 multi-tons resolved at level 1 from the column pass
  int32_t mpp;            // 2: two-ton moment preserving solve of multi-tons
  int32_t precision;      // 0: locate / value / residual in FP64; 1: in FP32
  int32_t fp16;           // 1: x is the packed FP16 form (header with the scale, binary16 pairs)
  int32_t col_key;        // column-pass signals: log2 B0 + 32 fp16 + 64 (16-row) / 128 (16-column form)
  int32_t col_ltc;        // column-pass signals: log2 of the columns of one item
  int32_t col_dz;         // column-pass signals: depth below which open classes go to the
                          // deep resolution (0: the column resolution goes all the way)
  int32_t l0_tile_lg;     // log2 of the level-0 sub-FFT size
  int32_t col_rows;  // column pass: rows reserved for the open level-0 classes (<= multi_cap)
  int32_t enum_lane_blocks;  // noisy enumeration below level 0: teams where ranges exceed this many 32-blocks
  int32_t rf_iters, rf_m; // FFAST R-FFAST delay set r_c + 2^c t (rf_iters = 0: delays 0..D-1)
  uint64_t rf_off[SFFT_MAX_ROUNDS];
  int32_t n_starts;       // FFAST packet-erasure schedule: start frequencies (0: method 1)
  int64_t start_f[SFFT_MAX_PEEL_STARTS];
  int64_t stageB[SFFT_MAX_STAGES];
  int64_t stageOff[SFFT_MAX_STAGES + 1];
  uint64_t shift[SFFT_MAX_ROUNDS];
  double eps0, eps1, zero_k, single_k, noise_var;
  double noise_p_den;     // -ln(1 - p/phi) of the noise estimator
  int64_t noise_at;       // rank of the p-quantile among the level-0 entries
  // offsets into the batch arenas
  int64_t y0_off;         // float2 level-0 planes (tree: n*B0; FFAST: D*sum B)
  int64_t fst_off;        // double2 FFAST state (D*sum B) + per-bucket scratch
  int64_t found_off;      // found list slots
  int64_t multi_off;      // multi-ton slots (per parity)
  int64_t jc_off;         // column-pass rows: complex64 offset of multi_cap rows of L = N/B0
};

// Per-call pointers of one signal.
struct SigIO {
  const float2 *x;
  int64_t *idx;
  float2 *val;
  int64_t *count;
  int32_t *status;
  int32_t pad[2];
};

// Per-signal device state of one exec.
struct SigState {
  int32_t found;          // appended frequencies
  int32_t multi[2];       // multi-tons per level parity
  int32_t flags;          // bit 0: unresolved multi-ton / cap; bit 1: list overflow
  int32_t levels;         // deepest tree level opened / peeling rounds
  int32_t ident;          // FFAST: bucket identifications
  int64_t samples;
  uint64_t level_mask;    // bit l set when tree level l gathered samples
  double sref2;
  double noise_var;
  double e0[SFFT_MAX_ROUNDS];  // tree: level-0 bucket power of each round (over its D planes)
};

struct Arena {
  float2 *y0;
  double2 *fst;
  int64_t *found_f;
  double2 *found_a;
  int64_t *multi_c[2];
  float2 *multi_y[2];
  double2 *multi_z[2];
  int32_t *pre;           // kPre prefix arrays of nsig+1: fft items, direct items,
                          // children, dense-pass items, subtree-resolve items,
                          // column-pass items, column-resolve items
  double2 *jacc;          // per multi-ton slot: jstride dense-pass coefficients
  float2 *jcol;           // per level-0 multi-ton slot: M_c(t), t < N/B0
  int32_t *deep_count;    // classes handed to the deep resolution (reset per run)
  int2 *deep_list;        // ... their (signal, multi-ton slot)
  uint64_t *deep_mask;    // per multi-ton slot: its open subclasses at depth col_dz + 1
  const float2 *tw;       // e^{-2 pi i k / kFftMax}, k < kFftMax
};

// e^{-2 pi i k / kFftMax}, k < kFftMax, rounded to FP32 (host computation)
void host_twiddles(float2 *out);
// device address of the current device's static scratch of sfft_exec_noalloc
// (kNoAllocScratchBytes; its first kNoAllocTwBytes hold the twiddle table)
hipError_t noalloc_scratch(int device, char **base);

// host-side kernel launchers (sfft_level0.hip, sfft_ffast.hip, sfft_tree.hip,
// sfft_jump.hip, sfft_col.hip, sfft_finalize.hip)
struct LaunchCtx {
  const SigDesc *desc;
  const SigIO *io;        // per-signal pointers in device memory (batches), or
  SigIO io1;              // null and the single signal's pointers by value
  SigState *st;
  Arena A;
  const int32_t *tree_list;
  const int32_t *ffast_list;
  const int32_t *l0_pre;   // prefix over tree_list of the rounds (level-0 FFT items)
  const int32_t *l0c_pre;  // prefix over tree_list of ceil(B0 / (256 >> l0_spread_lg)) (classify items)
  int32_t l0_items, l0c_items;
  int32_t l0_spread_lg;    // level-0 classification: log2 of the lanes per class (64 >> it classes a wave)
  int32_t any_wide_jump;   // some signal may run the dense pass on the matrix cores (L' >= 32)
  int32_t jstride;         // dense-pass coefficients per multi-ton slot (kJumpMax)
  int32_t jrows;           // rows per dense-pass work item (power of two)
  int32_t any_fp32;        // some tree signal classifies in single precision
  int32_t col_lp_mask;     // bit LP - 4 set when a signal with B0 = 2^(LP+5) takes the column pass
  int32_t col_f16_mask;    // ... for signals stored in the packed FP16 form
  int32_t col16_mask;      // bit 0 / 1: a complex64 / packed FP16 signal takes the 16-row form;
                           // bit 2 / 3: the 16-column form
  int32_t any_noisy0;      // some noisy tree signal's level-0 range exceeds its enum_share blocks, or
                           // the classes are spread over several lanes (team enumeration compiled in)
  int32_t any_noisy;       // some noisy tree signal has subtree candidate ranges longer than
                           // its enum_share blocks (team enumeration compiled in)
  int32_t any_noise_est;   // some noisy tree signal estimates its noise level (statistics launch)
  int32_t gather_u;        // gather loads in flight per thread (2, 4 or 8)
  int32_t deep_lds;        // dynamic LDS bytes of the deep resolution (largest L x 8), 0: none
  int32_t l0_lds;          // dynamic LDS bytes of the level-0 transform (largest tile x D)
  int32_t nsig, ntree, nffast;
  int32_t nmax;           // largest n = R*D of the batch (selects the template)
  int32_t max_B0;
  int32_t max_stage_B;
  int32_t max_found_cap;
};

hipError_t launch_reset(const LaunchCtx &c, hipStream_t s);
hipError_t launch_level0(const LaunchCtx &c, hipStream_t s);
hipError_t launch_ffast(const LaunchCtx &c, hipStream_t s);
hipError_t launch_sched(const LaunchCtx &c, int level, hipStream_t s);
hipError_t launch_expand_fft(const LaunchCtx &c, int level, int grid, hipStream_t s);
hipError_t launch_expand_direct(const LaunchCtx &c, int level, int grid, hipStream_t s);
hipError_t launch_children(const LaunchCtx &c, int level, int grid, hipStream_t s);
hipError_t launch_jump_pass(const LaunchCtx &c, int level, int grid, hipStream_t s);
hipError_t launch_jump_resolve(const LaunchCtx &c, int level, int grid, hipStream_t s);
hipError_t launch_col_pass(const LaunchCtx &c, int grid, hipStream_t s);
hipError_t launch_col_resolve(const LaunchCtx &c, int grid, hipStream_t s);
hipError_t launch_col_deep(const LaunchCtx &c, int grid, hipStream_t s);
hipError_t launch_finalize(const LaunchCtx &c, hipStream_t s);
// level-0 class vectors in class-major order (tree: out[c*n + i]; FFAST as stored)
hipError_t launch_export_level0(const LaunchCtx &c, void *out, hipStream_t s);
// host-gather form: write `count` packed samples of tree level `level` (or of
// the FFAST stages, level 0) to their positions in the device image of x
hipError_t launch_scatter(const SigDesc *d_desc, int level, const float2 *packed, int64_t count,
                          float2 *image, hipStream_t s);

}  // namespace sfft
