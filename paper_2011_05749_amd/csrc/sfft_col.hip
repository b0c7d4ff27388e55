// sfft_col.hip -- level-1 column pass: B0-point DFTs down the columns of x
// give every level-0 multi-ton's coefficients M_c(t) (Sect. 3.3).
#include "sfft_device.h"

namespace sfft {

namespace {

// ------------------------------------------------- level-1 column pass

// e^{-2 pi i k / 32} = cos - i sin, k < 16 (FP32-rounded constants)
__device__ __forceinline__ float w32c(int k) {
  switch (k) {
    case 1: return 9.807852507e-01f;
    case 2: return 9.238795042e-01f;
    case 3: return 8.314695954e-01f;
    case 4: return 7.071067691e-01f;
    case 5: return 5.555702448e-01f;
    case 6: return 3.826834261e-01f;
    case 7: return 1.950903237e-01f;
    case 9: return -1.950903237e-01f;
    case 10: return -3.826834261e-01f;
    case 11: return -5.555702448e-01f;
    case 12: return -7.071067691e-01f;
    case 13: return -8.314695954e-01f;
    case 14: return -9.238795042e-01f;
    case 15: return -9.807852507e-01f;
    default: return k == 0 ? 1.0f : 0.0f;
  }
}
__device__ __forceinline__ float w32s(int k) { return k <= 8 ? w32c(8 - k) : w32c(k - 8); }

// v e^{-2 pi i k / 32}; k is a compile-time constant once the caller unrolls
__device__ __forceinline__ float2 rot32(float2 v, int k) {
  if (k == 0) return v;
  if (k == 8) return make_float2(v.y, -v.x);
  const float cs = w32c(k), sn = w32s(k);
  return make_float2(fmaf(v.x, cs, v.y * sn), fmaf(v.y, cs, -v.x * sn));
}

__host__ __device__ constexpr int brev_c(int i, int lg) {
  int r = 0;
  for (int b = 0; b < lg; b++) r |= ((i >> b) & 1) << (lg - 1 - b);
  return r;
}

// In-register DFT of 2^LG <= 32 points, forward sign, no scaling: radix-2
// decimation in frequency, v[i] ends holding X[bitrev_LG(i)].
template <int LG>
__device__ __forceinline__ void dft_reg(float2 *v) {
  constexpr int n = 1 << LG;
#pragma unroll
  for (int lgs = LG - 1; lgs >= 0; lgs--) {
    const int span = 1 << lgs;
#pragma unroll
    for (int g = 0; g < n; g += 2 * span) {
#pragma unroll
      for (int j = 0; j < span; j++) {
        const float2 a = v[g + j], b = v[g + j + span];
        v[g + j] = make_float2(a.x + b.x, a.y + b.y);
        v[g + j + span] = rot32(make_float2(a.x - b.x, a.y - b.y), j * (16 >> lgs));
      }
    }
    // stage by stage: interleaving the stages would hold both halves of
    // many butterflies at once (register budget)
    __builtin_amdgcn_sched_barrier(0);
  }
}

// v of lane (this lane xor m), m in {1, 2, 4}: DPP quad permutes for 1 and 2,
// a swizzle within 32 lanes for 4
__device__ __forceinline__ float lane_xor(float v, int m) {
  const int iv = __float_as_int(v);
  if (m == 1) return __int_as_float(__builtin_amdgcn_mov_dpp(iv, 0xB1, 0xF, 0xF, false));
  if (m == 2) return __int_as_float(__builtin_amdgcn_mov_dpp(iv, 0x4E, 0xF, 0xF, false));
  return __int_as_float(__builtin_amdgcn_ds_swizzle(iv, 0x1F | (4 << 10)));
}

// Uniform values that no kernel writes while the reader runs, read through
// the constant address space so that they come in by scalar loads (which do
// not wait behind the vector loads in flight).
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(4))) T *cst(const T *p) {
  return (const __attribute__((address_space(4))) T *)p;
}

// Level-1 column pass (power-of-two N, B0 = 32 P, P = 2^LP in {16, 32, 64, 128, 256}):
// viewing x as B0 rows m of L = N/B0 samples, class c's coefficients
//   M_c(t) = sum_{m < B0} x[m L + t] e^{-2 pi i c m / B0},   t < L
// are the B0-point DFT down column t, evaluated at c.  With m = p + P q and
// c = k1 + 32 k2,
//   M_{k1 + 32 k2}(t) = sum_p e^{-2 pi i k2 p / P} e^{-2 pi i k1 p / B0}
//                       sum_q x[(p + P q) L + t] e^{-2 pi i k1 q / 32}.
// Item = (signal, TC = 512 / P adjacent columns).  Thread (t, p) loads its
// 32 rows and takes the inner DFT over q in registers; after an LDS exchange
// of the whole item, thread (t, k1, h), h < H2 = P / 32, takes the 32 values
// p = h + H2 p' of one outer DFT, a 32-point register DFT over p' and, for
// P > 32, a radix-H2 step across adjacent lanes (for P = 16, thread (t, k1)
// takes the 16-point outer DFTs of k1 and k1 + 16); the results go back to
// the LDS places the thread read.  Only the classes left open at level 0 are then
// stored (raw M_c(t), complex64, one row of L per multi-ton slot).
// One resident work-group per CU walks a contiguous range of items: the
// rows of item k + 1 are in flight while item k is transformed, and no other
// vector-memory load waits behind them (twiddles in LDS, open-class lists
// loaded ahead).  Work-groups 8 apart run on one XCD; such a pair takes the
// two items of each adjacent pair, in step, so that both read the same
// 128-byte lines through one L2.
// F16: the instance for signals stored in the packed FP16 form (binary16 rows,
// the scale applied to the stored coefficients); the other takes complex64.
template <int LP, bool F16>
__global__ __launch_bounds__(kColThreads, 2) void k_col_pass(LaunchCtx c) {
  constexpr int P = 1 << LP;
  constexpr int B0 = P * kColQ;
  constexpr int LTC = 9 - LP;          // log2 of the columns per item
  constexpr int TC = 1 << LTC;
  constexpr int LH2 = LP >= 5 ? LP - 5 : 0;  // lanes of one outer DFT: H2 = P / 32 (1 for P = 16)
  constexpr int H2 = 1 << LH2;
  // E[t][k1][p] with strides such that the writes (lanes along t, then p)
  // and the reads (lanes along h, then k1) of every 32 lanes fall on
  // distinct 8-byte bank pairs
  constexpr int SK = P + H2;           // P = 16: 17
  constexpr int ST = 32 * SK + 32 / TC;
  // e^{-2 pi i e / B0}: the whole table for B0 <= 2048, else as
  // e^{-2 pi i (64 a) / B0} e^{-2 pi i b / B0}, e = 64 a + b
  constexpr bool TW2 = B0 > 2048;
  constexpr int NTW = TW2 ? 64 + B0 / 64 : B0;
  constexpr int RL = B0 / kColThreads;  // open-list entries per thread
  static_assert(kColThreads == 512 && TC * P == kColThreads, "column pass shape");
  __shared__ float2 E[TC * ST];
  __shared__ float2 twB[NTW];
  __shared__ float2 wP[P];             // e^{-2 pi i e / P}
  __shared__ int16_t open_c[B0];
  const __attribute__((address_space(4))) int32_t *pc = cst(c.A.pre + 5 * (c.nsig + 1));
  const int npairs = pc[c.nsig] >> 1;  // every signal has an even item count
  const int nwp = gridDim.x >> 1;      // grid: a multiple of 16
  const int wp = ((blockIdx.x >> 4) << 3) + (blockIdx.x & 7), hf = (blockIdx.x >> 3) & 1;
  const int per = (npairs + nwp - 1) / nwp;
  const int ip0 = wp * per;
  const int ip1 = ip0 + per < npairs ? ip0 + per : npairs;
  if (ip0 >= ip1) return;
  const int tid = threadIdx.x;
  if (tid < P) wP[tid] = c.A.tw[tid << (kLog2FftMax - LP)];
  if (TW2) {
    if (tid < 64) twB[tid] = c.A.tw[tid << (kLog2FftMax - LP - 5)];
    else if (tid < 64 + B0 / 64) twB[tid] = c.A.tw[(tid - 64) << (kLog2FftMax - LP + 1)];
  } else {
    for (int e = tid; e < B0; e += kColThreads) twB[e] = c.A.tw[e << (kLog2FftMax - LP - 5)];
  }
  const int t = tid & (TC - 1), p = tid >> LTC;                          // loader role
  const int h = tid & (H2 - 1), k1r = (tid >> LH2) & 31, tr = tid >> (LH2 + 5);  // outer-DFT role
  typedef __attribute__((address_space(1))) const unsigned long long gq;
  float2 xn[kColQ];
  int ln[RL];
  int m_n = 0;
  // the open-class list of an item (ahead, in registers), then its rows in
  // four parts of eight, issued at three points of the previous item's work
  // so that the vector-memory queue never holds all of them at once
  typedef __attribute__((address_space(1))) const unsigned gh;
  gq *fx = nullptr;
  gh *fxh = nullptr;   // packed FP16 rows (binary16 pairs)
  float sc_n = 1.0f;   // the next item's scale (packed FP16 form)
  uint32_t foff = 0;
  int64_t frs = 0;
  bool fon = false;
  auto fetch = [&](int item, int sg) {
    const __attribute__((address_space(4))) SigDesc &ds = cst(c.desc)[sg];
    const int m = cst(c.st)[sg].multi[0];
    m_n = m > ds.multi_cap ? ds.multi_cap : m;
#pragma unroll
    for (int r = 0; r < RL; r++) {
      const int j = tid + r * kColThreads;
      ln[r] = j < m_n ? (int)c.A.multi_c[0][ds.multi_off + j] : 0;
    }
    const int64_t L = ds.N >> ds.log2B0;
    const float2 *xs = c.io ? cst(c.io)[sg].x : c.io1.x;
    const int64_t col0 = (int64_t)(item - pc[sg]) << LTC;
    if constexpr (F16) {
      fxh = (gh *)((const char *)xs + SFFT_F16_HEADER_BYTES) + col0;
      sc_n = *cst((const float *)xs);
    } else {
      fx = (gq *)xs + col0;
    }
    foff = (uint32_t)(p * L + t);  // < B0 L / 32: fits
    frs = (int64_t)P * L;
    fon = true;
  };
  auto fetch_part = [&](int part) {
    if (!fon) return;
    if constexpr (F16) {
#pragma unroll
      for (int q = 8 * part; q < 8 * part + 8; q++) xn[q] = half2_to_float2((fxh + q * frs)[foff], 1.0f);
    } else {
#pragma unroll
      for (int q = 8 * part; q < 8 * part + 8; q++) {
        const unsigned long long u = (fx + q * frs)[foff];
        xn[q] = make_float2(__uint_as_float((unsigned)u), __uint_as_float((unsigned)(u >> 32)));
      }
    }
  };
  // the stored outputs of the item held in E
  bool pend = false;
  int m_p = 0;
  int64_t L_p = 0;
  float2 *out_p = nullptr;
  float sc_p = 1.0f;   // scale of the packed FP16 form (1 for complex64)
  auto store_outputs = [&]() {
    for (int u = tid; u < (m_p << LTC); u += kColThreads) {
      const int j = u >> LTC, tt = u & (TC - 1);
      const int cc = open_c[j];
      const int k2 = cc >> 5;
      const float2 e = E[tt * ST + (cc & 31) * SK + brev_c(k2 >> 5, LH2) + H2 * (k2 & 31)];
      out_p[(int64_t)j * L_p + tt] = F16 ? make_float2(e.x * sc_p, e.y * sc_p) : e;
    }
  };
  int s = 0;
  while (2 * ip0 + hf >= pc[s + 1]) s++;
  auto is_mine = [&](int sg) { return cst(c.desc)[sg].col_key == LP + 5 + (F16 ? 32 : 0); };
  if (is_mine(s)) {
    fetch(2 * ip0 + hf, s);
    for (int part = 0; part < 4; part++) fetch_part(part);
  }
  for (int ip = ip0; ip < ip1; ip++) {
    const int item = 2 * ip + hf;
    while (item >= pc[s + 1]) s++;
    const __attribute__((address_space(4))) SigDesc &d = cst(c.desc)[s];
    const bool mine = is_mine(s);  // other widths or sample forms: another launch
    float2 v[kColQ];
#pragma unroll
    for (int q = 0; q < kColQ; q++) v[q] = xn[q];
    int lc[RL];
#pragma unroll
    for (int r = 0; r < RL; r++) lc[r] = ln[r];
    const int m_s = m_n;
    const float sc_s = sc_n;
    fon = false;
    if (ip + 1 < ip1) {
      int ns = s;
      while (item + 2 >= pc[ns + 1]) ns++;
      if (is_mine(ns)) fetch(item + 2, ns);
    }
    fetch_part(0);
    fetch_part(1);
    // the previous item's stores go out behind the loads just issued
    if (pend) store_outputs();
    pend = false;
    if (!mine) {
      for (int part = 2; part < 4; part++) fetch_part(part);
      continue;
    }
    dft_reg<5>(v);
    fetch_part(2);
    __syncthreads();  // the previous item's outputs are out of E and open_c
#pragma unroll
    for (int r = 0; r < RL; r++)
      if (tid + r * kColThreads < m_s) open_c[tid + r * kColThreads] = (int16_t)lc[r];
    // v[i] is the inner DFT at k1 = bitrev5(i); times e^{-2 pi i k1 p / B0}
#pragma unroll
    for (int i = 0; i < kColQ; i++) {
      float2 w = make_float2(1.0f, 0.0f);
      if (i > 0) {
        const int e = brev_c(i, 5) * p;  // < B0
        w = TW2 ? cmulf(twB[e & 63], twB[64 + (e >> 6)]) : twB[e];
      }
      E[t * ST + brev_c(i, 5) * SK + p] = i == 0 ? v[0] : cmulf(v[i], w);
    }
    __syncthreads();
    fetch_part(3);
    if constexpr (LP == 4) {
      // two 16-point outer DFTs per thread: k1 = tid mod 16 and k1 + 16, in place
#pragma unroll
      for (int half = 0; half < 2; half++) {
        float2 *row = E + (tid >> 4) * ST + ((tid & 15) + 16 * half) * SK;
        float2 a[16];
#pragma unroll
        for (int pp = 0; pp < 16; pp++) a[pp] = row[pp];
        dft_reg<4>(a);
#pragma unroll
        for (int i = 0; i < 16; i++) row[brev_c(i, 4)] = a[i];
      }
    } else {
      float2 *row = E + tr * ST + k1r * SK + h;
      float2 a[32];
#pragma unroll
      for (int pp = 0; pp < 32; pp++) a[pp] = row[H2 * pp];
      dft_reg<5>(a);
      if (H2 > 1) {
        // a[i] = F_h(k' = bitrev5(i)); times e^{-2 pi i k' h / P}, then the
        // H2-point DFT over h across adjacent lanes (decimation in
        // frequency): lane h ends with k2 = k' + 32 bitrev(h)
#pragma unroll
        for (int i = 1; i < 32; i++) a[i] = cmulf(a[i], wP[(brev_c(i, 5) * h) & (P - 1)]);
#pragma unroll
        for (int lhs = LH2 - 1; lhs >= 0; lhs--) {
          const int hs = 1 << lhs;
          const float sg = (h & hs) ? -1.0f : 1.0f;
          const float2 w = (h & hs) && lhs > 0 ? wP[(h & (hs - 1)) << (LP - 1 - lhs)] : make_float2(1.0f, 0.0f);
#pragma unroll
          for (int i = 0; i < 32; i++) {
            const float2 r = make_float2(fmaf(sg, a[i].x, lane_xor(a[i].x, hs)), fmaf(sg, a[i].y, lane_xor(a[i].y, hs)));
            a[i] = lhs > 0 ? cmulf(r, w) : r;
          }
        }
      }
      // back to the places this thread read: k' at h + H2 k'
#pragma unroll
      for (int i = 0; i < 32; i++) row[H2 * brev_c(i, 5)] = a[i];
    }
    __syncthreads();
    pend = true;
    m_p = m_s;
    sc_p = sc_s;
    L_p = d.N >> d.log2B0;
    out_p = c.A.jcol + d.jc_off + ((int64_t)(item - pc[s]) << LTC);
  }
  if (pend) store_outputs();
}

}  // namespace

hipError_t launch_col_pass(const LaunchCtx &c, int grid, hipStream_t s) {
  const dim3 g(grid), b(kColThreads);
  if (c.col_lp_mask & 1) hipLaunchKernelGGL((k_col_pass<4, false>), g, b, 0, s, c);
  if (c.col_lp_mask & 2) hipLaunchKernelGGL((k_col_pass<5, false>), g, b, 0, s, c);
  if (c.col_lp_mask & 4) hipLaunchKernelGGL((k_col_pass<6, false>), g, b, 0, s, c);
  if (c.col_lp_mask & 8) hipLaunchKernelGGL((k_col_pass<7, false>), g, b, 0, s, c);
  if (c.col_lp_mask & 16) hipLaunchKernelGGL((k_col_pass<8, false>), g, b, 0, s, c);
  if (c.col_f16_mask & 1) hipLaunchKernelGGL((k_col_pass<4, true>), g, b, 0, s, c);
  if (c.col_f16_mask & 2) hipLaunchKernelGGL((k_col_pass<5, true>), g, b, 0, s, c);
  if (c.col_f16_mask & 4) hipLaunchKernelGGL((k_col_pass<6, true>), g, b, 0, s, c);
  if (c.col_f16_mask & 8) hipLaunchKernelGGL((k_col_pass<7, true>), g, b, 0, s, c);
  if (c.col_f16_mask & 16) hipLaunchKernelGGL((k_col_pass<8, true>), g, b, 0, s, c);
  return hipGetLastError();
}

}  // namespace sfft
