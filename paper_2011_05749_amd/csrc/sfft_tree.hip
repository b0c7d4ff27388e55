// sfft_tree.hip -- tree levels l >= 1 gathered level by level (Sect. 3.3):
// per-level work scheduling, odd-offset gathers with their B'-point FFTs or
// per-bin partial sums (Eq. 23), and the children's classification.
#include "sfft_device.h"

namespace sfft {

namespace {

// Work of tree level `level` for every signal: prefix sums of FFT items,
// direct partial-sum items, children, dense-pass items and subtree-resolve
// items; resets this level's multi-ton count.
__global__ __launch_bounds__(1024) void k_sched(LaunchCtx c, int level) {
  __shared__ int red[16];
  const int par = (level - 1) & 1;
  const int np = c.nsig + 1;
  int carry[kPre] = {};
  for (int base = 0; base < c.nsig; base += blockDim.x) {
    const int s = base + threadIdx.x;
    int cnt[kPre] = {};
    if (s < c.nsig) {
      const SigDesc &d = c.desc[s];
      if (d.kind == SFFT_KIND_TREE && level <= d.max_levels) {
        int m = c.st[s].multi[par];
        if (m > d.multi_cap) m = d.multi_cap;
        const int lb = d.log2B0 + level - 1;
        const int64_t Bp = (int64_t)1 << lb;
        const int64_t Lp = d.N >> lb;
        if (m > 0) {
          // a dense pass over x serves a bounded number of open classes: at the
          // first stride <= jump_L it is taken when they are at most
          // kJumpMfmaClasses, one level later always
          const bool jump = d.jump_L > 0 && Lp <= d.jump_L &&
                            (m <= kJumpMfmaClasses || 2 * Lp <= d.jump_L);
          if (d.l1) {
            // level 1 of a column-pass signal: every level-0 multi-ton at once
            // items of 2^col_ltc adjacent columns, the range padded to a
            // multiple of kColItemAlign (the XCD grouping of the column pass
            // takes items in aligned groups; the padding items are skipped)
            // open classes beyond the rows reserved for them stay unresolved
            if (m > d.col_rows) {
              c.st[s].flags |= 1;
              m = d.col_rows;
            }
            const int nit = (int)(Lp >> d.col_ltc);
            cnt[5] = (nit + kColItemAlign - 1) & ~(kColItemAlign - 1);
            // the column resolution's classes, padded to whole waves of
            // 64 / kColGroup (a wave's classes then share one signal)
            cnt[6] = (m + kColResolveAlign - 1) & ~(kColResolveAlign - 1);
            c.st[s].samples += d.N;
          } else if (jump) {
            cnt[3] = (int)((Bp + c.jrows - 1) / c.jrows);
            cnt[4] = m;
            c.st[s].samples += d.N;
          } else {
            const int64_t Bsmax = (int64_t)1 << split_lg(d.D);
            if (Bp <= Bsmax || m >= kSplitMinBins) cnt[0] = d.R * (int)(Bp > Bsmax ? Bp / Bsmax : 1);
            else cnt[1] = d.R * (int)((Bp + kChunk - 1) / kChunk);
            cnt[2] = 2 * m;
            c.st[s].samples += (int64_t)d.n * Bp;
          }
          c.st[s].levels = level;
          c.st[s].level_mask |= 1ull << level;
        }
      }
      c.st[s].multi[level & 1] = 0;
    }
    for (int k = 0; k < kPre; k++) {
      int tot;
      const int ex = block_scan_excl(cnt[k], red, &tot);
      if (s < c.nsig) c.A.pre[k * np + s] = carry[k] + ex;
      carry[k] += tot;
    }
  }
  if (threadIdx.x == 0)
    for (int k = 0; k < kPre; k++) c.A.pre[k * np + c.nsig] = carry[k];
}

// Odd-offset samples of level `level` (B' = B0 2^{level-1} per round and
// delay, offset L'/2).  The parents' bins of their B'-point DFT come from P =
// B'/Bs sub-FFTs of size Bs = min(B', kFftMax) in LDS: with m = m' P + p,
//   Z[c] = sum_p e^{-2 pi i c p / B'} FFT_Bs(z[m' P + p])[c mod Bs].
// Item = (signal, round, p); the P partial bins meet in FP64 atomics.
template <int U>
__global__ __launch_bounds__(kThreads) void k_expand_fft(LaunchCtx c, int level) {
  extern __shared__ float2 lds[];
  const int par = (level - 1) & 1;
  const int32_t *pf = c.A.pre;
  const int total = pf[c.nsig];
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    const int s = find_owner(pf, c.nsig, item);
    const int rem = item - pf[s];
    const SigDesc &d = c.desc[s];
    const SigSrc src = sig_src(io_of(c, s).x, d);
    const int64_t N = d.N;
    const int lb = d.log2B0 + level - 1;
    const int64_t Bp = (int64_t)1 << lb;
    const int64_t Lp = N >> lb;
    const int D = d.D;
    const int lgs = lb < split_lg(D) ? lb : split_lg(D);
    const int64_t Bs = (int64_t)1 << lgs;
    const int P = (int)(Bp >> lgs);
    const int r = rem / P, p = rem % P;
    int m_s = c.st[s].multi[par];
    if (m_s > d.multi_cap) m_s = d.multi_cap;
    const uint64_t tau0 = (d.shift[r] + (uint64_t)(Lp >> 1)) & (uint64_t)(N - 1);
    gather_delays<U>(lds, src, Bs, lgs, (uint64_t)Lp, (uint64_t)P, (uint64_t)p, tau0, (uint64_t)(N - 1), D);
    __syncthreads();
    for (int dl = 0; dl < D; dl++) fft_lds(lds + (int64_t)dl * Bs, lgs, c.A.tw);
    for (int j = threadIdx.x; j < m_s; j += blockDim.x) {
      const int64_t slot = d.multi_off + j;
      const uint64_t cc = (uint64_t)c.A.multi_c[par][slot];
      double2 w = make_double2(1.0, 0.0);
      if (P > 1) w = unit_d((cc * (uint64_t)p) & (uint64_t)(Bp - 1), (uint64_t)Bp, -1);
      for (int dl = 0; dl < D; dl++) {
        const double2 v = cmul(to_d(lds[(int64_t)dl * Bs + (cc & (uint64_t)(Bs - 1))]), w);
        double *zz = (double *)&c.A.multi_z[par][slot * c.nmax + r * D + dl];
        if (P == 1) {
          zz[0] = v.x;
          zz[1] = v.y;
        } else {
          atomicAdd(zz, v.x);
          atomicAdd(zz + 1, v.y);
        }
      }
    }
    __syncthreads();
  }
}

// Partial DFT sums of the odd-offset samples at the parents' bins only, for
// B' > kFftMax: item = (signal, round, chunk of kChunk samples); FP64 atomics
// combine the chunks.
__global__ __launch_bounds__(kThreads) void k_expand_direct(LaunchCtx c, int level) {
  __shared__ float red[4][2 * kMaxD];
  const int par = (level - 1) & 1;
  const int32_t *pd = c.A.pre + (c.nsig + 1);
  const int total = pd[c.nsig];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    const int s = find_owner(pd, c.nsig, item);
    const int rem = item - pd[s];
    const SigDesc &d = c.desc[s];
    const SigSrc src = sig_src(io_of(c, s).x, d);
    const int64_t N = d.N;
    const int lb = d.log2B0 + level - 1;
    const int64_t Bp = (int64_t)1 << lb;
    const int64_t Lp = N >> lb;
    const int nch = (int)((Bp + kChunk - 1) / kChunk);
    const int r = rem / nch, ch = rem % nch;
    const int64_t m0 = (int64_t)ch * kChunk;
    int m_s = c.st[s].multi[par];
    if (m_s > d.multi_cap) m_s = d.multi_cap;
    const int n = d.n, D = d.D;
    const uint64_t base_tau = (d.shift[r] + (uint64_t)(Lp >> 1)) & (uint64_t)(N - 1);
    float2 z[kPerThread][kMaxD];
#pragma unroll
    for (int q = 0; q < kPerThread; q++) {
      const int64_t m = m0 + threadIdx.x + (int64_t)q * kThreads;
      const uint64_t p0 = (uint64_t)m * (uint64_t)Lp + base_tau;
#pragma unroll
      for (int dl = 0; dl < kMaxD; dl++) {
        z[q][dl] = make_float2(0.f, 0.f);
        if (dl < D && m < Bp) z[q][dl] = load_sample(src, (p0 + (uint64_t)dl) & (uint64_t)(N - 1));
      }
    }
    for (int j = 0; j < m_s; j++) {
      const int64_t slot = d.multi_off + j;
      const uint64_t cb = (uint64_t)c.A.multi_c[par][slot];
      const uint64_t msk = (uint64_t)Bp - 1;
      const double2 w0 = unit_d((cb * (uint64_t)(m0 + threadIdx.x)) & msk, (uint64_t)Bp, -1);
      const double2 ws = unit_d((cb * (uint64_t)kThreads) & msk, (uint64_t)Bp, -1);
      float2 tw = make_float2((float)w0.x, (float)w0.y);
      const float2 stp = make_float2((float)ws.x, (float)ws.y);
      float acc[2 * kMaxD];
#pragma unroll
      for (int i = 0; i < 2 * kMaxD; i++) acc[i] = 0.f;
#pragma unroll
      for (int q = 0; q < kPerThread; q++) {
#pragma unroll
        for (int dl = 0; dl < kMaxD; dl++) {
          const float2 t = cmulf(z[q][dl], tw);
          acc[2 * dl] += t.x;
          acc[2 * dl + 1] += t.y;
        }
        tw = cmulf(tw, stp);
      }
#pragma unroll
      for (int i = 0; i < 2 * kMaxD; i++) {
        float v = acc[i];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
        acc[i] = v;
      }
      if (lane == 0) {
#pragma unroll
        for (int i = 0; i < 2 * kMaxD; i++) red[w][i] = acc[i];
      }
      __syncthreads();
      if (threadIdx.x < 2 * D) {
        const int i = threadIdx.x;
        const double v = (double)red[0][i] + (double)red[1][i] + (double)red[2][i] + (double)red[3][i];
        double *zz = (double *)&c.A.multi_z[par][slot * c.nmax + r * D + (i >> 1)];
        atomicAdd(zz + (i & 1), v);
      }
      __syncthreads();
    }
  }
}

// Children of every multi-ton of level-1: Y_child = 1/2 (Y_parent +- w Z/B'),
// w = e^{-pi i c / B'} (radix-2 split of the level's transform); classify.
template <int NMAX, bool F32, bool WAVE>
__global__ __launch_bounds__(kThreads) void k_children(LaunchCtx c, int level) {
  const int par = (level - 1) & 1, cur = level & 1;
  const int32_t *pc = c.A.pre + 2 * (c.nsig + 1);
  const int total = pc[c.nsig];
  // whole work-groups step together (the noisy enumeration may run in teams of the wave's lanes)
  for (int g0 = blockIdx.x * blockDim.x; g0 < total; g0 += gridDim.x * blockDim.x) {
    const bool act = g0 + (int)threadIdx.x < total;
    const int g = act ? g0 + (int)threadIdx.x : g0;
    const int s = find_owner(pc, c.nsig, g);
    const int q = g - pc[s];
    const int j = q >> 1, side = q & 1;
    const SigDesc &d = c.desc[s];
    const int n = d.n;
    const int lb = d.log2B0 + level - 1;
    const int64_t Bp = (int64_t)1 << lb;
    const int64_t B = Bp << 1;
    const int64_t L = d.N >> (lb + 1);
    const int64_t slot = d.multi_off + j;
    const int64_t cpar = c.A.multi_c[par][slot];
    double sw, cw;
    sincospi((double)cpar / (double)Bp, &sw, &cw);
    const double wx = cw, wy = -sw;                 // e^{-pi i c / B'}
    const double sg = side ? -0.5 : 0.5;
    const double invB = 1.0 / (double)Bp;
    double2 Y[NMAX];
#pragma unroll
    for (int i = 0; i < NMAX; i++) {
      Y[i] = make_double2(0.0, 0.0);
      if (i < n) {
        const float2 p = c.A.multi_y[par][slot * c.nmax + i];
        const double2 zz = c.A.multi_z[par][slot * c.nmax + i];
        const double zx = zz.x * invB, zy = zz.y * invB;
        const double tx = wx * zx - wy * zy, ty = wx * zy + wy * zx;
        Y[i] = make_double2(0.5 * (double)p.x + sg * tx, 0.5 * (double)p.y + sg * ty);
      }
    }
    const int64_t cc = cpar + (side ? Bp : 0);
    const SigState &ss = c.st[s];
    const Decision v = classify<NMAX, true, F32, WAVE>(Y, d, n, d.R, cc, B, ss.sref2, ss.noise_var, act);
    if (!act) continue;
    if (v.cls == kSingle) {
      const int fs = atomicAdd(&c.st[s].found, 1);
      push_found(c, s, d, fs, v.f, v.a);
    } else if (v.cls == kDouble) {
      const int fs = atomicAdd(&c.st[s].found, 2);
      push_found(c, s, d, fs, v.f, v.a);
      push_found(c, s, d, fs + 1, v.f2, v.a2);
    } else if (v.cls == kMulti) {
      if (L >= 2 && level + 1 <= d.max_levels) {
        const int ms = atomicAdd(&c.st[s].multi[cur], 1);
        if (ms < d.multi_cap) {
          const int64_t sl = d.multi_off + ms;
          c.A.multi_c[cur][sl] = cc;
#pragma unroll
          for (int i = 0; i < NMAX; i++)
            if (i < n) {
              c.A.multi_y[cur][sl * c.nmax + i] = make_float2((float)Y[i].x, (float)Y[i].y);
              c.A.multi_z[cur][sl * c.nmax + i] = make_double2(0.0, 0.0);
            }
          if (d.jump_L > 0 && L <= d.jump_L)
            for (int t = 0; t < L; t++) c.A.jacc[sl * c.jstride + t] = make_double2(0.0, 0.0);
        } else {
          atomicOr(&c.st[s].flags, 3);
        }
      } else {
        atomicOr(&c.st[s].flags, 1);
      }
    }
  }
}

}  // namespace

hipError_t launch_sched(const LaunchCtx &c, int level, hipStream_t s) {
  hipLaunchKernelGGL(k_sched, dim3(1), dim3(1024), 0, s, c, level);
  return hipGetLastError();
}

hipError_t launch_expand_fft(const LaunchCtx &c, int level, int grid, hipStream_t s) {
  const size_t lds = 64 * 1024;
  if (c.gather_u == 2) hipLaunchKernelGGL(k_expand_fft<2>, dim3(grid), dim3(kThreads), lds, s, c, level);
  else if (c.gather_u == 8) hipLaunchKernelGGL(k_expand_fft<8>, dim3(grid), dim3(kThreads), lds, s, c, level);
  else hipLaunchKernelGGL(k_expand_fft<4>, dim3(grid), dim3(kThreads), lds, s, c, level);
  return hipGetLastError();
}

hipError_t launch_expand_direct(const LaunchCtx &c, int level, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_expand_direct, dim3(grid), dim3(kThreads), 0, s, c, level);
  return hipGetLastError();
}

hipError_t launch_children(const LaunchCtx &c, int level, int grid, hipStream_t s) {
  SFFT_LAUNCH_CLASSIFIER(k_children, c, dim3(grid), dim3(kThreads), 0, s, c, level);
  return hipGetLastError();
}

}  // namespace sfft
