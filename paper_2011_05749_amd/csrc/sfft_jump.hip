// sfft_jump.hip -- subtree resolution of the gathering path: one dense pass
// over x gives every open class's L' coefficients (VALU or matrix-core
// form), from which every later level's class vectors are formed.
#include "sfft_device.h"

namespace sfft {

namespace {

// Dense pass of the subtree resolution: for every open class c of level-1
// (B' buckets, stride L' <= kJumpMax) accumulate its L' coefficients
//   M_c(t) = sum_{m < B'} x[m L' + t] e^{-2 pi i c m / B'},   t < L'
// (the class's bucket at level-1 measured with shift t, times B') from one
// coalesced read of x.  All L' elements of a row m share the twiddle of the
// row, so the twiddles of a block of rows live in LDS (one entry per class
// and row) and each element costs one complex multiply-add per class.
// Item = (signal, c.jrows rows); thread tid owns t = tid mod L'.
template <int NQ>
__device__ __forceinline__ void jump_rows(const LaunchCtx &c, const SigDesc &d, const SigSrc &src,
                          int64_t row0, int nrows, int lgL, uint64_t Bp, const uint64_t *cls,
                          float2 *T, float2 (*red)[64], int64_t slot0) {
  const int Lp = 1 << lgL;
  float2 acc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; q++) acc[q] = make_float2(0.f, 0.f);
  for (int b0 = 0; b0 < nrows; b0 += kJumpBlockRows) {
    const int nb = (nrows - b0) < kJumpBlockRows ? (nrows - b0) : kJumpBlockRows;
    for (int u = threadIdx.x; u < NQ * kJumpBlockRows; u += kThreads) {
      const int q = u / kJumpBlockRows, rr = u % kJumpBlockRows;
      if (rr < nb) T[u] = unit_f((cls[q] * (uint64_t)(row0 + b0 + rr)) & (Bp - 1), Bp);
    }
    __syncthreads();
    const int ne = nb << lgL;
    const uint64_t xb = (uint64_t)(row0 + b0) << lgL;
    for (int e0 = threadIdx.x; e0 < ne; e0 += 8 * kThreads) {
      float2 v[8];
#pragma unroll
      for (int u = 0; u < 8; u++) {
        const int e = e0 + u * kThreads;
        v[u] = load_sample(src, xb + (uint64_t)(e < ne ? e : ne - 1));   // rows past nb are skipped below
      }
      // one row's twiddles live at a time: the scheduling barrier keeps the
      // compiler from hoisting every row's LDS reads (register pressure)
#pragma unroll
      for (int u = 0; u < 8; u++) {
        const int rr = (e0 + u * kThreads) >> lgL;
        if (rr < nb) {
#pragma unroll
          for (int q = 0; q < NQ; q++) cmac(acc[q], v[u], T[q * kJumpBlockRows + rr]);
        }
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    __syncthreads();
  }
  // sum the threads that share t = tid mod L', then one FP64 atomic per (class, t)
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NQ; q++) {
    float vx = acc[q].x, vy = acc[q].y;
    for (int o = Lp; o < 64; o <<= 1) {
      vx += __shfl_xor(vx, o);
      vy += __shfl_xor(vy, o);
    }
    if (lane < Lp) red[w][lane] = make_float2(vx, vy);
    __syncthreads();
    if (threadIdx.x < Lp) {
      // L' < 64: every wave holds t = lane once; L' >= 64: threads t, t + L', ...
      double sx = 0.0, sy = 0.0;
      if (Lp < 64) {
        for (int ww = 0; ww < kThreads / 64; ww++) {
          sx += (double)red[ww][threadIdx.x].x;
          sy += (double)red[ww][threadIdx.x].y;
        }
      } else {
        for (int u = threadIdx.x; u < kThreads; u += Lp) {
          sx += (double)red[u >> 6][u & 63].x;
          sy += (double)red[u >> 6][u & 63].y;
        }
      }
      double *a = (double *)&c.A.jacc[(slot0 + q) * c.jstride + threadIdx.x];
      atomicAdd(a, sx);
      atomicAdd(a + 1, sy);
    }
    __syncthreads();
  }
}

// MFMA form of the dense pass for L' = 32 NT (NT = 1, 2, 4): the coefficients
// of up to 16 classes are one complex product M (classes x L') += W (classes
// x rows) X (rows x L'), written as a real product with 32 output rows (re,
// im of each class) and K = 2 per row (re, im of x):
//   [Re M_c]   [ Re W  -Im W ] [Re X]
//   [Im M_c] = [ Im W   Re W ] [Im X]
// and fed to v_mfma_f32_32x32x2f32, one instruction per row and 32 columns.
// Lane l supplies A[l % 32][l / 32] and B[l / 32][l % 32]; accumulator
// register r of lane l holds row 8 (r / 4) + 4 (l / 32) + r % 4, column l % 32.
typedef float floatx16 __attribute__((ext_vector_type(16)));

template <int NT>
__device__ __forceinline__ void jump_rows_mfma(const LaunchCtx &c, const SigSrc &src, int64_t row0,
                               int nrows, uint64_t Bp, const uint64_t *cls /* LDS */, int nq,
                               float2 *tile /* LDS, 2 x 32 KiB */, float *red /* aliases tile */,
                               int64_t slot0) {
  constexpr int Lp = 32 * NT;
  constexpr int TR = 4096 / Lp;             // rows of a 32 KiB tile
  constexpr int PV = TR * Lp / 2 / kThreads;  // 16-byte loads per thread and tile (8)
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int m = lane & 31, k = lane >> 5;
  const int q = m >> 1, o = m & 1;
  const uint64_t cq = q < nq ? cls[q] : 0;
  // the rows of a wave are 4 apart: their twiddles differ by e^{-2 pi i 4 c_q / B'}
  const float2 st = unit_f((cq * 4u) & (Bp - 1), Bp);
  floatx16 acc[NT];
#pragma unroll
  for (int nt = 0; nt < NT; nt++)
#pragma unroll
    for (int r = 0; r < 16; r++) acc[nt][r] = 0.f;
  // tiles of TR rows stream through LDS: the 16-byte loads of tile t + 1 are
  // in flight while the MFMAs of tile t run
  typedef float f32x4 __attribute__((ext_vector_type(4)));
  typedef __attribute__((address_space(1))) const f32x4 gf4;
  gf4 *xv = (gf4 *)src.p;
  gu64 *xh = (gu64 *)src.p;  // packed FP16: two samples per 8 bytes
  const int ntiles = (nrows + TR - 1) / TR;
  f32x4 pre[PV];
  auto fetch = [&](int t) {
    const int64_t base = (row0 + (int64_t)t * TR) * (Lp / 2);
    const int64_t lim = ((int64_t)nrows - (int64_t)t * TR) * (Lp / 2);
#pragma unroll
    for (int u = 0; u < PV; u++) {
      int64_t i = threadIdx.x + (int64_t)u * kThreads;
      if (i >= lim) i = lim - 1;  // rows past the item: an in-bounds re-read, never used
      if (src.fp16) {
        const unsigned long long w = xh[base + i];
        const float2 a = half2_to_float2((unsigned)w, src.scale);
        const float2 b = half2_to_float2((unsigned)(w >> 32), src.scale);
        pre[u][0] = a.x;
        pre[u][1] = a.y;
        pre[u][2] = b.x;
        pre[u][3] = b.y;
      } else {
        pre[u] = xv[base + i];
      }
    }
  };
  auto stash = [&](int buf) {
    f32x4 *dst = (f32x4 *)(tile + (size_t)buf * TR * Lp);
#pragma unroll
    for (int u = 0; u < PV; u++) dst[threadIdx.x + u * kThreads] = pre[u];
  };
  fetch(0);
  stash(0);
  __syncthreads();
  for (int t = 0; t < ntiles; t++) {
    if (t + 1 < ntiles) fetch(t + 1);
    const float *xt = (const float *)(tile + (size_t)(t & 1) * TR * Lp);
    // lane l supplies A[l % 32][l / 32]: output row 2q + o of class q, re/im
    // o, times x's re/im k -- [Re W, -Im W; Im W, Re W] -- and B[l / 32][l % 32]
    // = (k ? Im : Re) x[row][32 nt + m], read from the tile
    float2 wv = unit_f((cq * (uint64_t)(row0 + (int64_t)t * TR + w)) & (Bp - 1), Bp);
#pragma unroll 2
    for (int j = 0; j < TR / 4; j++) {
      const int rr = w + 4 * j;
      if ((int64_t)t * TR + rr < nrows) {
        const float a = o == 0 ? (k == 0 ? wv.x : -wv.y) : (k == 0 ? wv.y : wv.x);
#pragma unroll
        for (int nt = 0; nt < NT; nt++)
          acc[nt] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, xt[(rr * Lp + nt * 32 + m) * 2 + k], acc[nt],
                                                          0, 0, 0);
      }
      wv = cmulf(wv, st);
    }
    __syncthreads();
    if (t + 1 < ntiles) stash((t + 1) & 1);
    __syncthreads();
  }
  // sum the four waves' tiles in LDS, then one FP64 atomic per (class, re|im, t)
#pragma unroll
  for (int nt = 0; nt < NT; nt++) {
#pragma unroll
    for (int r = 0; r < 16; r++) {
      const int row = 8 * (r >> 2) + 4 * k + (r & 3);
      red[(w * 32 + row) * 32 + m] = acc[nt][r];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 32 * 32; e += kThreads) {
      const int row = e >> 5, col = e & 31;
      const float v = red[row * 32 + col] + red[(32 + row) * 32 + col] +
                      red[(64 + row) * 32 + col] + red[(96 + row) * 32 + col];
      const int qq = row >> 1;
      if (qq < nq) {
        double *a = (double *)&c.A.jacc[(slot0 + qq) * c.jstride + nt * 32 + col];
        atomicAdd(a + (row & 1), (double)v);
      }
    }
    __syncthreads();
  }
}

// Dense pass, L' < 32 (VALU form, NT = 0) or L' = 32 NT for NT = 1, 2, 4
// (MFMA form): one kernel per width so that each keeps its own register
// budget; each takes the items of its width.
template <int NT>
__global__ __launch_bounds__(kThreads) void k_jump_pass(LaunchCtx c, int level) {
  constexpr bool MFMA = NT > 0;
  // VALU form: twiddle table of 16 classes x 256 rows of complex64 (32 KiB);
  // MFMA form: two 32 KiB tiles of x, whose first 16 KiB serve the
  // reduction after the row loop
  __shared__ float2 T[MFMA ? 8192 : 4096 + 512];
  __shared__ uint64_t cls[kJumpMfmaClasses];
  const int par = (level - 1) & 1;
  const int np = c.nsig + 1;
  const int32_t *pj = c.A.pre + 3 * np;
  const int total = pj[c.nsig];
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    const int s = find_owner(pj, c.nsig, item);
    const int ch = item - pj[s];
    const SigDesc &d = c.desc[s];
    const int lb = d.log2B0 + level - 1;
    const int lgL = d.log2N - lb;
    // the MFMA kernel of width NT takes L' = 32 NT (when that width runs on the
    // matrix cores); the VALU kernel every narrower width
    constexpr int kLg = NT == 1 ? 5 : (NT == 2 ? 6 : 7);
    if (MFMA ? (lgL != kLg || lgL < kJumpMfmaMinLg) : (lgL >= kJumpMfmaMinLg)) continue;
    const SigSrc src = sig_src(io_of(c, s).x, d);
    const uint64_t Bp = (uint64_t)1 << lb;
    int m_s = c.st[s].multi[par];
    if (m_s > d.multi_cap) m_s = d.multi_cap;
    const int64_t row0 = (int64_t)ch * c.jrows;
    const int nrows = (int)((int64_t)Bp - row0 < c.jrows ? (int64_t)Bp - row0 : c.jrows);
    const int G = kJumpMfmaClasses;
    for (int j0 = 0; j0 < m_s; j0 += G) {
      const int nq = (m_s - j0) < G ? (m_s - j0) : G;
      __syncthreads();
      if (threadIdx.x < G)
        cls[threadIdx.x] = (int)threadIdx.x < nq ? (uint64_t)c.A.multi_c[par][d.multi_off + j0 + threadIdx.x] : 0;
      __syncthreads();
      const int64_t slot0 = d.multi_off + j0;
      if constexpr (MFMA) {
        jump_rows_mfma<(NT > 0 ? NT : 1)>(c, src, row0, nrows, Bp, cls, nq, T, (float *)T, slot0);
      } else {
        float2 (*redv)[64] = (float2 (*)[64])(T + 4096);
        switch (nq) {
          case 1: jump_rows<1>(c, d, src, row0, nrows, lgL, Bp, cls, T, redv, slot0); break;
          case 2: jump_rows<2>(c, d, src, row0, nrows, lgL, Bp, cls, T, redv, slot0); break;
          case 3: jump_rows<3>(c, d, src, row0, nrows, lgL, Bp, cls, T, redv, slot0); break;
          case 4: jump_rows<4>(c, d, src, row0, nrows, lgL, Bp, cls, T, redv, slot0); break;
          case 5: jump_rows<5>(c, d, src, row0, nrows, lgL, Bp, cls, T, redv, slot0); break;
          case 6: jump_rows<6>(c, d, src, row0, nrows, lgL, Bp, cls, T, redv, slot0); break;
          case 7: jump_rows<7>(c, d, src, row0, nrows, lgL, Bp, cls, T, redv, slot0); break;
          case 8: jump_rows<8>(c, d, src, row0, nrows, lgL, Bp, cls, T, redv, slot0); break;
          case 9: jump_rows<9>(c, d, src, row0, nrows, lgL, Bp, cls, T, redv, slot0); break;
          case 10: jump_rows<10>(c, d, src, row0, nrows, lgL, Bp, cls, T, redv, slot0); break;
          case 11: jump_rows<11>(c, d, src, row0, nrows, lgL, Bp, cls, T, redv, slot0); break;
          case 12: jump_rows<12>(c, d, src, row0, nrows, lgL, Bp, cls, T, redv, slot0); break;
          case 13: jump_rows<13>(c, d, src, row0, nrows, lgL, Bp, cls, T, redv, slot0); break;
          case 14: jump_rows<14>(c, d, src, row0, nrows, lgL, Bp, cls, T, redv, slot0); break;
          case 15: jump_rows<15>(c, d, src, row0, nrows, lgL, Bp, cls, T, redv, slot0); break;
          default: jump_rows<16>(c, d, src, row0, nrows, lgL, Bp, cls, T, redv, slot0); break;
        }
      }
    }
  }
}

// Subtree resolution of one open class c (one work-group of kJumpMax
// threads, thread k owning frequency k at first and class k of a depth after): its L' frequencies
// f_k = c + k B' have the values xhat_{f_k} = (1/L') sum_t M_c(t)/B'
// e^{-2 pi i f_k t / N}; the class vector of any descendant class at any
// deeper level is the sum, over the frequencies it holds, of
// xhat_f e^{2 pi i f tau_i / N} -- the same linear functional of x as the
// level's gathered buckets -- so the level-by-level classification of the
// tree search (Sect. 3.3) runs on these vectors.
template <int NMAX, bool F32, bool WAVE>
__global__ __launch_bounds__(kJumpMax) void k_jump_resolve(LaunchCtx c, int level) {
  __shared__ double2 V[kJumpMax][NMAX];
  __shared__ double2 Ms[kJumpMax];
  __shared__ double2 root[kJumpMax];
  __shared__ int open_cur[kJumpMax], open_nxt[kJumpMax];
  __shared__ int any_open;
  const int par = (level - 1) & 1;
  const int np = c.nsig + 1;
  const int32_t *pr = c.A.pre + 4 * np;
  const int total = pr[c.nsig];
  const int k = threadIdx.x;
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    const int s = find_owner(pr, c.nsig, item);
    const int j = item - pr[s];
    const SigDesc &d = c.desc[s];
    const int64_t N = d.N;
    const int n = d.n;
    const int lb = d.log2B0 + level - 1;
    const int64_t Bp = (int64_t)1 << lb;
    const int Lp = (int)(N >> lb);
    const int64_t slot = d.multi_off + j;
    const int64_t cpar = c.A.multi_c[par][slot];
    const double sref2 = c.st[s].sref2, nv = c.st[s].noise_var;
    // e^{-2 pi i f_k t / N} = e^{-2 pi i c t / N} e^{-2 pi i k t / L'} (f_k = c + k B'):
    // thread t folds the first factor into M(t), the second is a root of unity
    if (k < Lp) {
      const double2 a = c.A.jacc[slot * c.jstride + k];
      const double2 b = unit_d(mod_n((uint64_t)cpar * (uint64_t)k, d), (uint64_t)N, -1);
      Ms[k] = cmul(make_double2(a.x / (double)Bp, a.y / (double)Bp), b);
      root[k] = unit_d((uint64_t)k, (uint64_t)Lp, -1);
    }
    __syncthreads();
    if (k < Lp) {
      const uint64_t f = (uint64_t)(cpar + (int64_t)k * Bp);
      double2 xh = make_double2(0.0, 0.0);
      for (int t = 0; t < Lp; t++) {
        const double2 u = cmul(Ms[t], root[(k * t) & (Lp - 1)]);
        xh.x += u.x;
        xh.y += u.y;
      }
      xh.x /= (double)Lp;
      xh.y /= (double)Lp;
      for (int i = 0; i < n; i++) V[k][i] = cmul(xh, unit_d(mod_n(f * tau_of(d, i), d), (uint64_t)N, +1));
    }
    if (k < kJumpMax) open_cur[k] = k < 2 ? 1 : 0;
    __syncthreads();
    for (int dd = 1; (1 << dd) <= Lp; dd++) {
      const int lvl = level + dd - 1;
      const int nq = 1 << dd;
      const int64_t Bd = Bp << dd;
      const int64_t Ld = N / Bd;
      if (k < kJumpMax) open_nxt[k] = 0;
      if (k == 0) any_open = 0;
      __syncthreads();
      {
        // every thread takes part (the noisy enumeration may run in teams of the wave's lanes)
        const bool act = k < nq && open_cur[k];
        double2 Y[NMAX];
#pragma unroll
        for (int i = 0; i < NMAX; i++) {
          Y[i] = make_double2(0.0, 0.0);
          if (act && i < n)
            for (int kk = k; kk < Lp; kk += nq) {
              Y[i].x += V[kk][i].x;
              Y[i].y += V[kk][i].y;
            }
        }
        const int64_t cc = cpar + (int64_t)k * Bp;
        const Decision v = classify<NMAX, true, F32, WAVE>(Y, d, n, d.R, cc, Bd, sref2, nv, act);
        if (act) {
          atomicMax(&c.st[s].levels, lvl);
          if (v.cls == kSingle) {
            const int fs = atomicAdd(&c.st[s].found, 1);
            push_found(c, s, d, fs, v.f, v.a);
          } else if (v.cls == kDouble) {
            const int fs = atomicAdd(&c.st[s].found, 2);
            push_found(c, s, d, fs, v.f, v.a);
            push_found(c, s, d, fs + 1, v.f2, v.a2);
          } else if (v.cls == kMulti) {
            if (Ld >= 2 && lvl + 1 <= d.max_levels) {
              open_nxt[k] = 1;
              open_nxt[k + nq] = 1;
              any_open = 1;
            } else {
              atomicOr(&c.st[s].flags, 1);
            }
          }
        }
      }
      __syncthreads();
      if (k < kJumpMax) open_cur[k] = open_nxt[k];
      const int more = any_open;
      __syncthreads();
      if (!more) break;
    }
    __syncthreads();
  }
}

}  // namespace

hipError_t launch_jump_pass(const LaunchCtx &c, int level, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_jump_pass<0>, dim3(grid), dim3(kThreads), 0, s, c, level);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !c.any_wide_jump) return e;
  if (5 >= kJumpMfmaMinLg) hipLaunchKernelGGL(k_jump_pass<1>, dim3(grid), dim3(kThreads), 0, s, c, level);
  if (6 >= kJumpMfmaMinLg) hipLaunchKernelGGL(k_jump_pass<2>, dim3(grid), dim3(kThreads), 0, s, c, level);
  hipLaunchKernelGGL(k_jump_pass<4>, dim3(grid), dim3(kThreads), 0, s, c, level);
  return hipGetLastError();
}

hipError_t launch_jump_resolve(const LaunchCtx &c, int level, int grid, hipStream_t s) {
  SFFT_LAUNCH_CLASSIFIER(k_jump_resolve, c, dim3(grid), dim3(kJumpMax), 0, s, c, level);
  return hipGetLastError();
}

}  // namespace sfft
