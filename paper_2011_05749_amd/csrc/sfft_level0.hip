// sfft_level0.hip -- per-signal reset, level-0 bucketization of the tree
// (gather + B0-point FFT, Eq. 5-6), level-0 statistics and classification,
// export of the level-0 table, and the host-gather scatter.
#include "sfft_device.h"

namespace sfft {

namespace {

// ---------------------------------------------------------------- kernels

__global__ void k_reset(LaunchCtx c) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s == 0 && c.deep_lds) *c.A.deep_count = 0;
  if (s >= c.nsig) return;
  SigState z;
  z.found = 0;
  z.multi[0] = 0;
  z.multi[1] = 0;
  z.flags = 0;
  z.levels = 0;
  z.ident = 0;
  z.samples = 0;
  z.level_mask = 0;
  z.sref2 = 0.0;
  z.noise_var = 0.0;
  for (int r = 0; r < SFFT_MAX_ROUNDS; r++) z.e0[r] = 0.0;
  const SigDesc &d = c.desc[s];
  if (d.kind == SFFT_KIND_TREE) {
    // level 0 reads n B0 samples; the noise level is the plan's unless the
    // level-0 statistics estimate it
    z.samples = (int64_t)d.n * d.B0;
    z.level_mask = 1ull;
    z.noise_var = d.noise_var;
  }
  c.st[s] = z;
}

// Level 0 of the tree, bucketization (Eq. 5-6): item = (signal, round r);
// the D delays of every sample are gathered together and transformed by
// P0 = B0 / Bs sub-FFTs of size Bs; with m = m' P0 + p,
//   Yhat[c] = (1/B0) sum_p e^{-2 pi i c p / B0} FFT_Bs(y[m' P0 + p])[c mod Bs],
// accumulated in the level-0 planes Y0[(r D + d) B0 + c] by this work-group
// alone (fixed order, no atomics).  The round's bucket power sum_{d, c}
// |Yhat|^2 goes to the signal's state (the zero-ton threshold's reference,
// Sect. 3.2, from the sum over rounds).
template <int U>
__global__ __launch_bounds__(kThreads) void k_level0_fft(LaunchCtx c) {
  extern __shared__ float2 lds[];
  __shared__ double red[16];
  for (int item = blockIdx.x; item < c.l0_items; item += gridDim.x) {
    const int li = find_owner(c.l0_pre, c.ntree, item);
    const int s = c.tree_list[li];
    const int r = item - c.l0_pre[li];
    const SigDesc &d = c.desc[s];
    const SigSrc src = sig_src(io_of(c, s).x, d);
    const int64_t N = d.N;
    const int lb = d.log2B0;
    const int64_t B = d.B0;
    const int64_t L = N >> lb;
    const int D = d.D;
    const int lgs = d.l0_tile_lg;
    const int64_t Bs = (int64_t)1 << lgs;
    const int P = (int)(B >> lgs);
    const float inv = 1.0f / (float)B;
    float2 *Y0 = c.A.y0 + d.y0_off + (int64_t)r * D * B;
    double psum = 0.0;  // this thread's final buckets' power, cc ascending, then d
    for (int p = 0; p < P; p++) {
      gather_delays<U>(lds, src, Bs, lgs, (uint64_t)L, (uint64_t)P, (uint64_t)p, d.shift[r],
                    (uint64_t)(N - 1), D);
      __syncthreads();
      for (int dl = 0; dl < D; dl++) fft_lds(lds + (int64_t)dl * Bs, lgs, c.A.tw);
      for (int64_t cc = threadIdx.x; cc < B; cc += blockDim.x) {
        float2 w = make_float2(inv, 0.f);
        if (p > 0) {
          const float2 u = unit_f(((uint64_t)cc * (uint64_t)p) & (uint64_t)(B - 1), (uint64_t)B);
          w = make_float2(u.x * inv, u.y * inv);
        }
        for (int dl = 0; dl < D; dl++) {
          const float2 v = cmulf(lds[(int64_t)dl * Bs + (cc & (Bs - 1))], w);
          float2 *o = Y0 + (int64_t)dl * B + cc;
          const float2 y = p == 0 ? v : make_float2(o->x + v.x, o->y + v.y);
          *o = y;
          if (p == P - 1) psum += (double)y.x * y.x + (double)y.y * y.y;
        }
      }
      __syncthreads();
    }
    const double e = block_sum_d(psum, red);
    if (threadIdx.x == 0) c.st[s].e0[r] = e;
  }
}

// Level-0 noise level of the noisy tree signals whose plan leaves it to be
// estimated: a quantile of B0 |Yhat|^2 over the signal's level-0 values
// (launched only for batches holding such a signal).
__global__ __launch_bounds__(kThreads) void k_level0_stats(LaunchCtx c) {
  __shared__ uint32_t hist[256];
  __shared__ uint32_t sel[2];
  for (int li = blockIdx.x; li < c.ntree; li += gridDim.x) {
    const int s = c.tree_list[li];
    const SigDesc &d = c.desc[s];
    if (!(d.mode == SFFT_NOISY && !(d.noise_var > 0.0))) continue;  // uniform over the work-group
    const int64_t cnt = (int64_t)d.n * d.B0;
    const float2 *Y0 = c.A.y0 + d.y0_off;
    const float q = select_kth_power(Y0, cnt, (float)d.B0, d.noise_at, hist, sel);
    if (threadIdx.x == 0) c.st[s].noise_var = (double)q / d.noise_p_den;
    __syncthreads();
  }
}

// Classification of the B0 level-0 classes (Sect. 3.2, Subproblems 1-2):
// item = (signal, 256 >> lg classes), 64 >> lg a wave on its first lanes (lg
// = l0_spread_lg: the other lanes only join the team enumeration); single-tons
// and multi-tons are compacted by wave ballot + prefix, one atomic per wave
// and list.  Registers are capped for two waves a SIMD (the instance with the
// team enumeration would otherwise take more and run one).
template <int NMAX, bool F32, bool WAVE>
__global__ __launch_bounds__(kThreads, 2) void k_level0_classify(LaunchCtx c) {
  for (int item = blockIdx.x; item < c.l0c_items; item += gridDim.x) {
    // the lists, the descriptors and the level-0 statistics are written
    // before this kernel runs: scalar loads
    const int li = find_owner(cst(c.l0c_pre), c.ntree, item);
    const int s = cst(c.tree_list)[li];
    const SigDesc &d = *(const SigDesc *)&cst(c.desc)[s];
    const int64_t B = d.B0;
    const int64_t L = d.N >> d.log2B0;
    const int n = d.n;
    const float2 *Y0 = c.A.y0 + d.y0_off;
    // mean level-0 bucket power: the rounds' sums in round order, over n B0
    double e0 = 0.0;
    for (int r = 0; r < d.R; r++) e0 += cst(c.st)[s].e0[r];
    const double sref2 = e0 / (double)((int64_t)n * B), nv = cst(c.st)[s].noise_var;
    // the signal's first item records it for the later levels and the statistics
    if (item == cst(c.l0c_pre)[li] && threadIdx.x == 0) c.st[s].sref2 = sref2;
    // 64 >> lg classes a wave, on its first lanes; the rest of the wave joins
    // the team enumeration only
    const int lg = c.l0_spread_lg;
    const int lane = threadIdx.x & 63, cpw = 64 >> lg;
    const int64_t cc = (int64_t)(item - cst(c.l0c_pre)[li]) * (kThreads >> lg) + (threadIdx.x >> 6) * cpw + lane;
    const bool valid = lane < cpw && cc < B;
    Decision v;
    v.cls = kZero;
    double2 Y[NMAX];
#pragma unroll
    for (int i = 0; i < NMAX; i++) Y[i] = make_double2(0.0, 0.0);
    if (valid) {
#pragma unroll
      for (int i = 0; i < NMAX; i++)
        if (i < n) Y[i] = to_d(Y0[(int64_t)i * B + cc]);
    }
    // every lane of the work-group takes part (the noisy enumeration may run in teams of the wave's lanes)
    v = classify<NMAX, true, F32, WAVE>(Y, d, n, d.R, cc, B, sref2, nv, valid);
    const int nf = !valid ? 0 : (v.cls == kSingle ? 1 : (v.cls == kDouble ? 2 : 0));
    const int fs = wave_append_n(&c.st[s].found, nf);
    if (nf >= 1) push_found(c, s, d, fs, v.f, v.a);
    if (nf == 2) push_found(c, s, d, fs + 1, v.f2, v.a2);
    const bool multi = valid && v.cls == kMulti;
    const bool open = multi && L >= 2 && d.max_levels >= 1;
    if (multi && !open) atomicOr(&c.st[s].flags, 1);
    const int ms = wave_append(&c.st[s].multi[0], open);
    if (open) {
      if (ms < d.multi_cap) {
        const int64_t slot = d.multi_off + ms;
        c.A.multi_c[0][slot] = cc;
#pragma unroll
        for (int i = 0; i < NMAX; i++)
          if (i < n) {
            c.A.multi_y[0][slot * c.nmax + i] = make_float2((float)Y[i].x, (float)Y[i].y);
            c.A.multi_z[0][slot * c.nmax + i] = make_double2(0.0, 0.0);
          }
        if (d.jump_L > 0 && L <= d.jump_L)
          for (int t = 0; t < L; t++) c.A.jacc[slot * c.jstride + t] = make_double2(0.0, 0.0);
      } else {
        atomicOr(&c.st[s].flags, 3);
      }
    }
  }
}

__global__ void k_export_level0(LaunchCtx c, float2 *out) {
  const SigDesc &d = c.desc[0];
  if (d.kind == SFFT_KIND_FFAST) {
    const int64_t tot = d.stageOff[d.nstages] * d.D;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < tot; i += (int64_t)gridDim.x * blockDim.x)
      out[i] = c.A.y0[d.y0_off + i];
  } else {
    const int64_t tot = (int64_t)d.n * d.B0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < tot; i += (int64_t)gridDim.x * blockDim.x) {
      const int64_t cc = i / d.n, k = i % d.n;
      out[i] = c.A.y0[d.y0_off + k * d.B0 + cc];
    }
  }
}

}  // namespace

hipError_t launch_export_level0(const LaunchCtx &c, void *out, hipStream_t s) {
  hipLaunchKernelGGL(k_export_level0, dim3(256), dim3(256), 0, s, c, (float2 *)out);
  return hipGetLastError();
}

// Host-gather form of a solve: the samples that tree level `level` (or the
// FFAST stages) read arrive packed in (round or stage, m, delay) order and
// are written to the positions the level's kernels read in the device image
// of x -- level 0: m L0 + s_r + d (m < B0); level l >= 1: the odd offsets
// m L' + L'/2 + s_r + d (m < B' = B0 2^{l-1}); FFAST stage j: m L_j + tau_d.
__global__ __launch_bounds__(kThreads) void k_scatter(const SigDesc *desc, int level,
                                                      const float2 *__restrict__ packed,
                                                      int64_t count, float2 *image) {
  const SigDesc &d = *desc;
  const uint64_t N = (uint64_t)d.N;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int dl = (int)(i % d.D);
    const int64_t rm = i / d.D;
    uint64_t pos;
    if (d.kind == SFFT_KIND_FFAST) {
      int j = 0;
      while (j + 1 < d.nstages && d.stageOff[j + 1] <= rm) j++;
      const uint64_t m = (uint64_t)(rm - d.stageOff[j]);
      pos = (m * (N / (uint64_t)d.stageB[j]) + tau_of<false>(d, dl)) % N;
    } else {
      const int lb = d.log2B0 + (level > 0 ? level - 1 : 0);
      const uint64_t Bp = (uint64_t)1 << lb, Lp = N >> lb;
      const int r = (int)(rm >> lb);
      const uint64_t m = (uint64_t)rm & (Bp - 1);
      pos = (m * Lp + (level > 0 ? (Lp >> 1) : 0) + d.shift[r] + (uint64_t)dl) & (N - 1);
    }
    image[pos] = packed[i];
  }
}

hipError_t launch_scatter(const SigDesc *d_desc, int level, const float2 *packed, int64_t count,
                          float2 *image, hipStream_t s) {
  const int64_t blocks = (count + kThreads - 1) / kThreads;
  const int grid = (int)(blocks < 8192 ? (blocks > 0 ? blocks : 1) : 8192);
  hipLaunchKernelGGL(k_scatter, dim3(grid), dim3(kThreads), 0, s, d_desc, level, packed, count, image);
  return hipGetLastError();
}

hipError_t launch_reset(const LaunchCtx &c, hipStream_t s) {
  hipLaunchKernelGGL(k_reset, dim3((c.nsig + 255) / 256), dim3(256), 0, s, c);
  return hipGetLastError();
}

hipError_t launch_level0(const LaunchCtx &c, hipStream_t s) {
  if (c.ntree > 0) {
    const size_t lds = (size_t)c.l0_lds;
    const dim3 g0(c.l0_items < 8192 ? c.l0_items : 8192), b0(kThreads);
    if (c.gather_u == 2) hipLaunchKernelGGL(k_level0_fft<2>, g0, b0, lds, s, c);
    else if (c.gather_u == 8) hipLaunchKernelGGL(k_level0_fft<8>, g0, b0, lds, s, c);
    else hipLaunchKernelGGL(k_level0_fft<4>, g0, b0, lds, s, c);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (c.any_noise_est) {
      hipLaunchKernelGGL(k_level0_stats, dim3(c.ntree < 4096 ? c.ntree : 4096), dim3(kThreads), 0, s, c);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    const int g = c.l0c_items < 8192 ? c.l0c_items : 8192;
    SFFT_LAUNCH_CLASSIFIER_W(k_level0_classify, c, c.any_noisy0 != 0, dim3(g), dim3(kThreads), 0, s, c);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (c.nffast > 0) return launch_ffast(c, s);
  return hipSuccess;
}

}  // namespace sfft
