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

// Wait until every vector-memory operation of this thread is done.  Issued at
// the top of an item, before the next item's loads go out: the item's rows
// must be in by then anyway, and the stores of run-time count that follow
// would otherwise leave the compiler only the choice of waiting for every
// outstanding load -- the prefetch of the next item included -- at the first
// use of a row, which serialises the loads and the transform.
__device__ __forceinline__ void rows_in() {
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0), the other counters untouched
  __builtin_amdgcn_sched_barrier(0);
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
  // G = max(2, 16 / TC) work-groups of one XCD (blockIdx 8 apart) take the G
  // adjacent items of a 128-byte row segment in step, so that the segment is
  // fetched once into that XCD's L2
  constexpr int LG = LTC >= 3 ? 1 : 4 - LTC;
  constexpr int G = 1 << LG;
  static_assert(G <= kColItemAlign, "item ranges are aligned to the group");
  const int npairs = pc[c.nsig] >> LG;  // every signal's item range: a multiple of kColItemAlign
  const int nwp = gridDim.x >> LG;      // grid: a multiple of 8 G
  const int wp = ((blockIdx.x >> (3 + LG)) << 3) + (blockIdx.x & 7), hf = (blockIdx.x >> 3) & (G - 1);
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
  unsigned xr[F16 ? kColQ : 1];  // packed FP16 form: the raw binary16 pairs (decoded after rows_in)
  int m_n = 0;
  // the next item's rows in four parts of eight, issued at three points of
  // the previous item's work so that the vector-memory queue never holds all
  // of them at once; its signal's open-class list is read into LDS only when
  // the signal changes (the items of one signal share it)
  typedef __attribute__((address_space(1))) const unsigned gh;
  gq *fx = nullptr;
  gh *fxh = nullptr;   // packed FP16 rows (binary16 pairs)
  float sc_n = 1.0f;   // the next item's scale (packed FP16 form)
  uint32_t foff = 0, fofb = 0;  // the lane's element and byte offsets in a row (< 2^31 bytes)
  int64_t frs = 0;
  bool fon = false;
  auto fetch = [&](int item, int sg) {
    const __attribute__((address_space(4))) SigDesc &ds = cst(c.desc)[sg];
    const int m = cst(c.st)[sg].multi[0];
    m_n = m > ds.col_rows ? ds.col_rows : m;  // col_rows <= multi_cap
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
    fofb = foff * (F16 ? 4u : 8u);
    frs = (int64_t)P * L;
    fon = true;
  };
  auto fetch_part = [&](int part) {
    if (!fon) {
      // no next item: the old values die here all the same
#pragma unroll
      for (int q = 8 * part; q < 8 * part + 8; q++) {
        xn[q] = make_float2(0.f, 0.f);
        if constexpr (F16) xr[q] = 0u;
      }
      return;
    }
    // each row's base in scalar registers (the empty asm keeps the compiler
    // from folding the lane's offset into a 64-bit vector address), the
    // lane's 32-bit byte offset apart: the loads take no vector ALU work
    typedef __attribute__((address_space(1))) const char gc;
    if constexpr (F16) {
#pragma unroll
      for (int q = 8 * part; q < 8 * part + 8; q++) {
        gc *rb = (gc *)(fxh + q * frs);
        asm volatile("" : "+s"(rb));
        xr[q] = *(gh *)(rb + fofb);
      }
    } else {
#pragma unroll
      for (int q = 8 * part; q < 8 * part + 8; q++) {
        gc *rb = (gc *)(fx + q * frs);
        asm volatile("" : "+s"(rb));
        const unsigned long long u = *(gq *)(rb + fofb);
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
  // the first group index at or after `ip` whose item this launch takes (its
  // signal in sg): other widths and sample forms, and the padding items, are
  // skipped a signal at a time (item ranges are multiples of kColItemAlign >= G)
  auto next_mine = [&](int ip, int &sg) {
    while (ip < ip1) {
      const int it = G * ip + hf;
      while (it >= pc[sg + 1]) sg++;
      const __attribute__((address_space(4))) SigDesc &ds = cst(c.desc)[sg];
      if (ds.col_key == LP + 5 + (F16 ? 32 : 0) && it - pc[sg] < (int)((ds.N >> ds.log2B0) >> LTC)) return ip;
      ip = pc[sg + 1] >> LG;
    }
    return ip1;
  };
  int s = 0, s_open = -1;  // s_open: the signal whose classes open_c holds
  int ip = next_mine(ip0, s);
  if (ip < ip1) {
    fetch(G * ip + hf, s);
    for (int part = 0; part < 4; part++) fetch_part(part);
  }
  while (ip < ip1) {
    const int item = G * ip + hf;
    const __attribute__((address_space(4))) SigDesc &d = cst(c.desc)[s];
    float2 v[kColQ];
#pragma unroll
    for (int q = 0; q < kColQ; q++) v[q] = xn[q];
    rows_in();
    if constexpr (F16) {
#pragma unroll
      for (int q = 0; q < kColQ; q++) v[q] = half2_to_float2(xr[q], 1.0f);
    }
    const int m_s = m_n;
    const float sc_s = sc_n;
    int ns = s;
    const int nip = next_mine(ip + 1, ns);
    fon = false;
    if (nip < ip1) fetch(G * nip + hf, ns);
    fetch_part(0);
    fetch_part(1);
    // the previous item's stores go out behind the loads just issued
    if (pend) store_outputs();
    pend = false;
    // the wide forms recompute their per-thread twiddle addresses in every
    // item from copies the compiler cannot hoist (held across the loop, the
    // 93 addresses would spill)
    int p_it = p, h_it = h;
    if constexpr (LP >= 7) asm volatile("" : "+v"(p_it), "+v"(h_it));
    dft_reg<5>(v);
    __syncthreads();  // the previous item's outputs are out of E and open_c
    // the third part after that barrier, not before it: the barrier would
    // wait for the last wave to issue these loads
    fetch_part(2);
    if (s != s_open) {
      // first item of another signal: its open classes (read after the
      // second barrier below, by this item's stores in the next iteration)
      s_open = s;
      for (int j = tid; j < m_s; j += kColThreads) open_c[j] = (int16_t)c.A.multi_c[0][d.multi_off + j];
    }
    // v[i] is the inner DFT at k1 = bitrev5(i); times e^{-2 pi i k1 p / B0}
#pragma unroll
    for (int i = 0; i < kColQ; i++) {
      float2 w = make_float2(1.0f, 0.0f);
      if (i > 0) {
        const int e = brev_c(i, 5) * p_it;  // < B0
        w = TW2 ? cmulf(twB[e & 63], twB[64 + (e >> 6)]) : twB[e];
      }
      E[t * ST + brev_c(i, 5) * SK + p] = i == 0 ? v[0] : cmulf(v[i], w);
      // two table reads per twiddle (B0 > 2048): keep them next to their use
      if (TW2 && (i & 7) == 7) __builtin_amdgcn_sched_barrier(0);
    }
    __syncthreads();
    // the wide forms (P >= 128) issue the last part after their outer DFT, whose
    // lane steps need the registers
    if constexpr (LP < 7) fetch_part(3);
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
        for (int i = 1; i < 32; i++) a[i] = cmulf(a[i], wP[(brev_c(i, 5) * h_it) & (P - 1)]);
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
          // stage by stage (the exchanges of several stages in flight would
          // hold both copies of the values)
          __builtin_amdgcn_sched_barrier(0);
        }
      }
      // back to the places this thread read: k' at h + H2 k'
#pragma unroll
      for (int i = 0; i < 32; i++) row[H2 * brev_c(i, 5)] = a[i];
    }
    if constexpr (LP >= 7) fetch_part(3);
    __syncthreads();
    pend = true;
    m_p = m_s;
    sc_p = sc_s;
    L_p = d.N >> d.log2B0;
    out_p = c.A.jcol + d.jc_off + ((int64_t)(item - pc[s]) << LTC);
    ip = nip;
    s = ns;
  }
  if (pend) store_outputs();
}

// Level-1 column pass, 16-row form (B0 = 2048 = 16 x 128; 1024 threads, four
// waves per SIMD).  Item = (signal, 8 adjacent columns t).  With m = p + 128 q
// (q < 16), c = k1 + 16 K, and the 128-point outer DFT split as p = p1 + 16 p2
// (p2 < 8), K = K1 + 8 K2 (K1 < 8, K2 < 16):
//   M_c(t) = sum_{p1} W16^{K2 p1} W128^{K1 p1} sum_{p2} W8^{K1 p2} Z_{k1}[p1 + 16 p2],
//   Z_{k1}[p] = W2048^{k1 p} sum_q x[(p + 128 q) L + t] W16^{k1 q}      (W_n = e^{-2 pi i / n}).
// Pass 1, thread (t, p): the 16-point DFT over q in registers, times
// W2048^{k1 p}, into LDS.  Pass 2, thread (t, k1, p1 and p1 + 8): two 8-point
// DFTs over p2 in registers, times W128^{K1 p1}, back to the same places.
// Pass 3, thread (t, k1, K1): the 16-point DFT over p1 in registers; each open
// class c = k1 + 16 K1 + 128 K2 is stored from there, the 8 lanes of its 8
// columns writing one 64-byte run.  LDS slot of (t, k1, p): t ST + k1 SK +
// (p mod 16) + 17 (p / 16), with ST = 4 mod 32 and the stride 17, so that the
// 8-byte accesses of every 32 lanes fall on distinct bank pairs in all passes.
// Persistent work-groups and the XCD pairing of the 32-row form.
template <bool F16>
__global__ __launch_bounds__(1024) void k_col_pass16(LaunchCtx c) {
  constexpr int B0 = 2048, TC = 8, LTC = 3, NT = 1024;
  constexpr int SK = 136, ST = 16 * SK + 4;
  constexpr int KEY = 11 + 64 + (F16 ? 32 : 0);
  __shared__ float2 E[TC * ST];
  __shared__ float2 tw1[B0];       // W2048^e
  __shared__ float2 tw2[128];      // W128^e
  __shared__ int16_t slot_of[B0];  // open class -> its row slot, -1 otherwise
  const __attribute__((address_space(4))) int32_t *pc = cst(c.A.pre + 5 * (c.nsig + 1));
  const int npairs = pc[c.nsig] >> 1;  // every signal's item range: a multiple of kColItemAlign
  const int nwp = gridDim.x >> 1;
  const int wp = ((blockIdx.x >> 4) << 3) + (blockIdx.x & 7), hf = (blockIdx.x >> 3) & 1;
  const int per = (npairs + nwp - 1) / nwp;
  const int ip0 = wp * per;
  const int ip1 = ip0 + per < npairs ? ip0 + per : npairs;
  if (ip0 >= ip1) return;
  const int tid = threadIdx.x;
  for (int e = tid; e < B0; e += NT) tw1[e] = c.A.tw[e << (kLog2FftMax - 11)];
  if (tid < 128) tw2[tid] = c.A.tw[tid << (kLog2FftMax - 7)];
  const int t = tid & 7;
  const int p = tid >> 3;                            // pass 1
  const int pa = (tid >> 3) & 7, kb = tid >> 6;      // pass 2: p1 in {pa, pa + 8}, k1 = kb
  const int K1c = pa, kc = kb;                       // pass 3: K1, k1
  auto slot = [](int tt, int k1, int pp) { return tt * ST + k1 * SK + (pp & 15) + 17 * (pp >> 4); };
  typedef __attribute__((address_space(1))) const unsigned long long gq;
  typedef __attribute__((address_space(1))) const unsigned gh;
  float2 xn[16];
  unsigned xr[F16 ? 16 : 1];  // packed FP16 form: the raw binary16 pairs (decoded after rows_in)
  gq *fx = nullptr;
  gh *fxh = nullptr;
  float sc_n = 1.0f;
  uint32_t foff = 0, fofb = 0;  // the lane's element and byte offsets in a row (< 2^31 bytes)
  int64_t frs = 0;
  int m_n = 0;
  bool fon = false;
  auto fetch = [&](int item, int sg) {
    const __attribute__((address_space(4))) SigDesc &ds = cst(c.desc)[sg];
    const int m = cst(c.st)[sg].multi[0];
    m_n = m > ds.col_rows ? ds.col_rows : m;  // col_rows <= multi_cap
    const int64_t L = ds.N >> 11;
    const float2 *xs = c.io ? cst(c.io)[sg].x : c.io1.x;
    const int64_t col0 = (int64_t)(item - pc[sg]) << LTC;
    if constexpr (F16) {
      fxh = (gh *)((const char *)xs + SFFT_F16_HEADER_BYTES) + col0;
      sc_n = *cst((const float *)xs);
    } else {
      fx = (gq *)xs + col0;
    }
    foff = (uint32_t)(p * L + t);  // < 128 L
    fofb = foff * (F16 ? 4u : 8u);
    frs = 128 * L;
    fon = true;
  };
  auto fetch_part = [&](int part) {
    if (!fon) {
      // no next item: the old values die here all the same
#pragma unroll
      for (int q = 8 * part; q < 8 * part + 8; q++) {
        xn[q] = make_float2(0.f, 0.f);
        if constexpr (F16) xr[q] = 0u;
      }
      return;
    }
    // each row's base in scalar registers (the empty asm keeps the compiler
    // from folding the lane's offset into a 64-bit vector address), the
    // lane's 32-bit byte offset apart: the loads take no vector ALU work
    typedef __attribute__((address_space(1))) const char gc;
    if constexpr (F16) {
#pragma unroll
      for (int q = 8 * part; q < 8 * part + 8; q++) {
        gc *rb = (gc *)(fxh + q * frs);
        asm volatile("" : "+s"(rb));
        xr[q] = *(gh *)(rb + fofb);
      }
    } else {
#pragma unroll
      for (int q = 8 * part; q < 8 * part + 8; q++) {
        gc *rb = (gc *)(fx + q * frs);
        asm volatile("" : "+s"(rb));
        const unsigned long long u = *(gq *)(rb + fofb);
        xn[q] = make_float2(__uint_as_float((unsigned)u), __uint_as_float((unsigned)(u >> 32)));
      }
    }
  };
  // the first pair index at or after `ip` whose item this launch takes (its
  // signal in sg); other widths, forms and sample types, and padding, skipped
  auto next_mine = [&](int ip, int &sg) {
    while (ip < ip1) {
      const int it = 2 * ip + hf;
      while (it >= pc[sg + 1]) sg++;
      const __attribute__((address_space(4))) SigDesc &ds = cst(c.desc)[sg];
      if (ds.col_key == KEY && it - pc[sg] < (int)((ds.N >> 11) >> LTC)) return ip;
      ip = pc[sg + 1] >> 1;
    }
    return ip1;
  };
  int s = 0, s_open = -1;  // s_open: the signal whose classes slot_of maps
  int ip = next_mine(ip0, s);
  if (ip < ip1) {
    fetch(2 * ip + hf, s);
    fetch_part(0);
    fetch_part(1);
  }
  while (ip < ip1) {
    const int item = 2 * ip + hf;
    const __attribute__((address_space(4))) SigDesc &d = cst(c.desc)[s];
    float2 v[16];
#pragma unroll
    for (int q = 0; q < 16; q++) v[q] = xn[q];
    rows_in();
    if constexpr (F16) {
#pragma unroll
      for (int q = 0; q < 16; q++) v[q] = half2_to_float2(xr[q], 1.0f);
    }
    const int m_s = m_n;
    const float sc_s = sc_n;
    int ns = s;
    const int nip = next_mine(ip + 1, ns);
    fon = false;
    if (nip < ip1) fetch(2 * nip + hf, ns);
    fetch_part(0);
    // per-thread twiddle indices recomputed in every item from copies the
    // compiler cannot hoist (held across the loop they would spill)
    int p_it = p, pa_it = pa;
    asm volatile("" : "+v"(p_it), "+v"(pa_it));
    // pass 1: v[i] = the DFT over q at k1 = bitrev4(i)
    dft_reg<4>(v);
    __syncthreads();  // the previous item's pass 3 is done with E and slot_of
#pragma unroll
    for (int i = 0; i < 16; i++) {
      const int k1 = brev_c(i, 4);
      E[slot(t, k1, p)] = i == 0 ? v[0] : cmulf(v[i], tw1[k1 * p_it]);
    }
    if (s != s_open)
      for (int j = tid; j < B0; j += NT) slot_of[j] = -1;
    fetch_part(1);
    __syncthreads();
    if (s != s_open) {
      // first item of another signal: its open classes and their row slots
      s_open = s;
      for (int j = tid; j < m_s; j += NT) slot_of[(int)c.A.multi_c[0][d.multi_off + j]] = (int16_t)j;
    }
    // pass 2: the 8-point DFTs over p2 of (t, kb, pa) and (t, kb, pa + 8)
#pragma unroll
    for (int half = 0; half < 2; half++) {
      const int p1 = pa_it + 8 * half;
      float2 a[8];
#pragma unroll
      for (int p2 = 0; p2 < 8; p2++) a[p2] = E[slot(t, kb, p1 + 16 * p2)];
      dft_reg<3>(a);
#pragma unroll
      for (int i = 0; i < 8; i++) {
        const int K1 = brev_c(i, 3);
        E[slot(t, kb, p1 + 16 * K1)] = i == 0 ? a[0] : cmulf(a[i], tw2[K1 * p1]);
      }
    }
    __syncthreads();
    // pass 3: the 16-point DFT over p1 of (t, kc, K1c); the open classes out
    float2 a[16];
#pragma unroll
    for (int p1 = 0; p1 < 16; p1++) a[p1] = E[slot(t, kc, p1 + 16 * K1c)];
    dft_reg<4>(a);
    const int64_t L = d.N >> 11;
    float2 *out = c.A.jcol + d.jc_off + ((int64_t)(item - pc[s]) << LTC) + t;
#pragma unroll
    for (int i = 0; i < 16; i++) {
      const int sl = slot_of[kc + 16 * K1c + 128 * brev_c(i, 4)];
      if (sl >= 0) out[(int64_t)sl * L] = F16 ? make_float2(a[i].x * sc_s, a[i].y * sc_s) : a[i];
    }
    ip = nip;
    s = ns;
  }
}

// e^{-2 pi i k / 64} = cos - i sin, k <= 16 (FP32-rounded constants)
__device__ __forceinline__ float w64c(int k) {
  switch (k) {
    case 0: return 1.0f;
    case 1: return 9.951847196e-01f;
    case 2: return 9.807852507e-01f;
    case 3: return 9.569403529e-01f;
    case 4: return 9.238795042e-01f;
    case 5: return 8.819212914e-01f;
    case 6: return 8.314695954e-01f;
    case 7: return 7.730104327e-01f;
    case 8: return 7.071067691e-01f;
    case 9: return 6.343932748e-01f;
    case 10: return 5.555702448e-01f;
    case 11: return 4.713967443e-01f;
    case 12: return 3.826834261e-01f;
    case 13: return 2.902846634e-01f;
    case 14: return 1.950903237e-01f;
    case 15: return 9.801714122e-02f;
    default: return 0.0f;
  }
}

// v e^{-2 pi i k / 64}, k < 32 a compile-time constant once unrolled
__device__ __forceinline__ float2 rot64(float2 v, int k) {
  if (k == 0) return v;
  if (k == 16) return make_float2(v.y, -v.x);
  const float cs = k <= 16 ? w64c(k) : -w64c(32 - k);
  const float sn = w64c(k <= 16 ? 16 - k : k - 16);
  return make_float2(fmaf(v.x, cs, v.y * sn), fmaf(v.y, cs, -v.x * sn));
}

// Level-1 column pass, 16-column form (B0 = 2048 = 32 x 64; 512 threads).
// Item = (signal, 16 adjacent columns t): every row of the item is read as one
// 128-byte segment by 16 lanes.  With m = p + 32 q (p < 32, q < 64) and
// c = k1 + 64 k2 (k1 < 64, k2 < 32):
//   M_c(t) = sum_p W32^{k2 p} W2048^{k1 p} sum_q x[(p + 32 q) L + t] W64^{k1 q}.
// Thread (t, p) takes the 64-point DFT over q in registers (a radix-2 step,
// then two 32-point DFTs: the even k1 in v[0..31], the odd in v[32..63]),
// times W2048^{k1 p}.  The exchange and the 32-point DFTs over p run in two
// halves, even k1 and then odd k1, through one LDS buffer of 16 x 32 x 32
// values; thread (t, k') of a half (k1 = 2 k' + half) stores its open classes
// from registers, 16 lanes writing one 128-byte run.  The registers a half
// frees take the next item's rows: q < 16 once the barrier after the even
// write is passed (issued just before that barrier they made the launch about
// 2 % longer, the barrier then waiting for the last wave to issue its loads),
// then a quarter after the even stores, after the odd write and after the odd
// stores; the odd k1's 32-point DFT over q runs after the even stores, so that
// the rows of two quarters are in flight meanwhile.  LDS slot of
// (t, k', p): t ST + k' SK + p, ST = 2 mod 32 and SK = 33, so that the
// 8-byte accesses of every 32 lanes fall on distinct bank pairs both ways.
// Persistent work-groups, each walking a contiguous range of items.
template <bool F16>
__global__ __launch_bounds__(512) void k_col_pass_t16(LaunchCtx c) {
  constexpr int B0 = 2048, LTC = 4, NT = 512;
  constexpr int SK = 33, ST = 32 * SK + 2;
  constexpr int KEY = 11 + 128 + (F16 ? 32 : 0);
  __shared__ float2 E[16 * ST];
  __shared__ float2 tw1[B0];       // W2048^e
  __shared__ int16_t slot_of[B0];  // open class -> its row slot, -1 otherwise
  __shared__ uint32_t omask[64];   // per k1: bit k2 set when class k1 + 64 k2 is open
  const __attribute__((address_space(4))) int32_t *pc = cst(c.A.pre + 5 * (c.nsig + 1));
  const int total = pc[c.nsig];
  const int per = (total + (int)gridDim.x - 1) / (int)gridDim.x;
  const int i0 = (int)blockIdx.x * per;
  const int i1 = i0 + per < total ? i0 + per : total;
  if (i0 >= i1) return;
  const int tid = threadIdx.x;
  for (int e = tid; e < B0; e += NT) tw1[e] = c.A.tw[e << (kLog2FftMax - 11)];
  const int t = tid & 15, p = tid >> 4;  // loads and the transform over q; (t, k' = p) over p
  typedef __attribute__((address_space(1))) const unsigned long long gq;
  typedef __attribute__((address_space(1))) const unsigned gh;
  float2 xn[64];
  unsigned xr[F16 ? 64 : 1];  // packed FP16 form: the raw binary16 pairs (decoded after rows_in)
  gq *fx = nullptr;
  gh *fxh = nullptr;
  float sc_n = 1.0f;
  uint32_t foff = 0, fofb = 0;  // the lane's element and byte offsets in a row (< 32 L x 8 <= 2^27)
  int64_t frs = 0;
  int m_n = 0;
  bool fon = false;
  auto fetch = [&](int item, int sg) {
    const __attribute__((address_space(4))) SigDesc &ds = cst(c.desc)[sg];
    const int m = cst(c.st)[sg].multi[0];
    m_n = m > ds.col_rows ? ds.col_rows : m;  // col_rows <= multi_cap
    const int64_t L = ds.N >> 11;
    const float2 *xs = c.io ? cst(c.io)[sg].x : c.io1.x;
    const int64_t col0 = (int64_t)(item - pc[sg]) << LTC;
    if constexpr (F16) {
      fxh = (gh *)((const char *)xs + SFFT_F16_HEADER_BYTES) + col0;
      sc_n = *cst((const float *)xs);
    } else {
      fx = (gq *)xs + col0;
    }
    foff = (uint32_t)(p * L + t);  // < 32 L
    fofb = foff * (F16 ? 4u : 8u);
    frs = 32 * L;
    fon = true;
  };
  // rows q in [q0, q0 + 16) of the fetched item; the loads stay where they are
  // written (hoisted into the transforms they would hold their registers longer)
  auto fetch_quarter = [&](int q0) {
    __builtin_amdgcn_sched_barrier(0);
    if (!fon) {
      // no next item: the old values die here all the same
#pragma unroll
      for (int q = q0; q < q0 + 16; q++) {
        xn[q] = make_float2(0.f, 0.f);
        if constexpr (F16) xr[q] = 0u;
      }
      return;
    }
    // each row's base in scalar registers (the empty asm keeps the compiler
    // from folding the lane's offset into a 64-bit vector address), the
    // lane's 32-bit byte offset apart: the loads take no vector ALU work
    typedef __attribute__((address_space(1))) const char gc;
    if constexpr (F16) {
#pragma unroll
      for (int q = q0; q < q0 + 16; q++) {
        gc *rb = (gc *)(fxh + q * frs);
        asm volatile("" : "+s"(rb));
        xr[q] = *(gh *)(rb + fofb);
      }
    } else {
#pragma unroll
      for (int q = q0; q < q0 + 16; q++) {
        gc *rb = (gc *)(fx + q * frs);
        asm volatile("" : "+s"(rb));
        const unsigned long long u = *(gq *)(rb + fofb);
        xn[q] = make_float2(__uint_as_float((unsigned)u), __uint_as_float((unsigned)(u >> 32)));
      }
    }
  };
  // the first item at or after `it` that this launch takes (its signal in sg):
  // other widths, forms and sample types, and the padding items, are skipped
  auto next_mine = [&](int it, int &sg) {
    while (it < i1) {
      while (it >= pc[sg + 1]) sg++;
      const __attribute__((address_space(4))) SigDesc &ds = cst(c.desc)[sg];
      if (ds.col_key == KEY && it - pc[sg] < (int)((ds.N >> 11) >> LTC)) return it;
      it = pc[sg + 1];
    }
    return i1;
  };
  int s = 0, s_open = -1;  // s_open: the signal whose classes slot_of maps
  int item = next_mine(i0, s);
  if (item < i1) {
    fetch(item, s);
    for (int q0 = 0; q0 < 64; q0 += 16) fetch_quarter(q0);
  }
  while (item < i1) {
    const __attribute__((address_space(4))) SigDesc &d = cst(c.desc)[s];
    float2 v[64];
#pragma unroll
    for (int q = 0; q < 64; q++) v[q] = xn[q];
    rows_in();
    if constexpr (F16) {
#pragma unroll
      for (int q = 0; q < 64; q++) v[q] = half2_to_float2(xr[q], 1.0f);
    }
    const int m_s = m_n;
    const float sc_s = sc_n;
    int ns = s;
    const int nx = next_mine(item + 1, ns);
    fon = false;
    if (nx < i1) fetch(nx, ns);
    int p_it = p;
    asm volatile("" : "+v"(p_it));
    // 64-point DFT over q: one radix-2 step (decimation in frequency) ...
#pragma unroll
    for (int j = 0; j < 32; j++) {
      const float2 a = v[j], b = v[j + 32];
      v[j] = make_float2(a.x + b.x, a.y + b.y);
      v[j + 32] = rot64(make_float2(a.x - b.x, a.y - b.y), j);
    }
    __builtin_amdgcn_sched_barrier(0);
    // ... then the 32-point DFT of the even k1 (v[0..31]); the odd k1's
    // (v[32..63]) waits until the even half is out, with the next item's
    // first rows in flight: v[h 32 + i] = X[k1 = 2 bitrev5(i) + h]
    dft_reg<5>(v);
    __syncthreads();  // the previous item is done with E and slot_of
#pragma unroll
    for (int i = 0; i < 32; i++) {
      const int kp = brev_c(i, 5);  // k1 = 2 kp
      E[t * ST + kp * SK + p] = i == 0 ? v[0] : cmulf(v[i], tw1[2 * kp * p_it]);
    }
    if (s != s_open) {
      for (int j = tid; j < B0; j += NT) slot_of[j] = -1;
      if (tid < 64) omask[tid] = 0u;
    }
    __syncthreads();
    if (s != s_open) {
      // first item of another signal: its open classes and their row slots
      s_open = s;
      for (int j = tid; j < m_s; j += NT) {
        const int cc = (int)c.A.multi_c[0][d.multi_off + j];
        slot_of[cc] = (int16_t)j;
        atomicOr(&omask[cc & 63], 1u << (cc >> 6));
      }
      __syncthreads();
    }
    fetch_quarter(0);
    // the item's first column in the rows of the open classes: a uniform base
    // and 32-bit offsets sl L + t < N <= 2^30
    const uint32_t L = (uint32_t)(d.N >> 11);
    float2 *out = c.A.jcol + d.jc_off + ((int64_t)(item - pc[s]) << LTC);
#pragma unroll
    for (int half = 0; half < 2; half++) {
      if (half == 1) {
        dft_reg<5>(v + 32);
        __builtin_amdgcn_sched_barrier(0);
        __syncthreads();  // the even half's reads of E are done
#pragma unroll
        for (int i = 0; i < 32; i++) {
          const int k1 = 2 * brev_c(i, 5) + 1;
          E[t * ST + brev_c(i, 5) * SK + p] = cmulf(v[32 + i], tw1[k1 * p_it]);
        }
        fetch_quarter(32);
        __syncthreads();
      }
      // the 32-point DFT over p of (t, k' = p), classes c = 2 k' + half + 64 k2,
      // split in time: the 16-point DFT of the odd p goes back to this thread's
      // own row of E, then the even p's, then X[k2] = Ev[k2] + W32^k2 Od[k2] and
      // X[k2 + 16] = Ev[k2] - W32^k2 Od[k2] are stored pair by pair (16 values
      // held at a time instead of 32)
      float2 *row = E + t * ST + p * SK;
      {
        float2 o[16];
#pragma unroll
        for (int pp = 0; pp < 16; pp++) o[pp] = row[2 * pp + 1];
        dft_reg<4>(o);
#pragma unroll
        for (int i = 0; i < 16; i++) row[2 * i + 1] = o[i];  // Od[bitrev4(i)]
      }
      float2 ev[16];
#pragma unroll
      for (int pp = 0; pp < 16; pp++) ev[pp] = row[2 * pp];
      dft_reg<4>(ev);  // ev[i] = Ev[bitrev4(i)]
      // the open classes among this thread's 32 (about one in ten): a bit test
      // each, and a slot lookup only for those
      const uint32_t om = omask[2 * p + half];
#pragma unroll
      for (int i = 0; i < 16; i++) {
        const int k2 = brev_c(i, 4);
        const float2 od = rot32(row[2 * i + 1], k2);
        const float2 x0 = make_float2(ev[i].x + od.x, ev[i].y + od.y);
        const float2 x1 = make_float2(ev[i].x - od.x, ev[i].y - od.y);
        const int cb = 2 * p + half + 64 * k2;
        if ((om >> k2) & 1u) {
          const uint32_t s0 = (uint32_t)slot_of[cb];
          out[s0 * L + (uint32_t)t] = F16 ? make_float2(x0.x * sc_s, x0.y * sc_s) : x0;
        }
        if ((om >> (k2 + 16)) & 1u) {
          const uint32_t s1 = (uint32_t)slot_of[cb + 1024];
          out[s1 * L + (uint32_t)t] = F16 ? make_float2(x1.x * sc_s, x1.y * sc_s) : x1;
        }
        // a few pairs at a time (all lookups ahead would hold their registers)
        if ((i & 3) == 3) __builtin_amdgcn_sched_barrier(0);
      }
      fetch_quarter(half == 0 ? 16 : 48);
    }
    item = nx;
    s = ns;
  }
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
  if (c.col16_mask & 1) hipLaunchKernelGGL((k_col_pass16<false>), g, dim3(1024), 0, s, c);
  if (c.col16_mask & 2) hipLaunchKernelGGL((k_col_pass16<true>), g, dim3(1024), 0, s, c);
  if (c.col16_mask & 4) hipLaunchKernelGGL((k_col_pass_t16<false>), g, dim3(512), 0, s, c);
  if (c.col16_mask & 8) hipLaunchKernelGGL((k_col_pass_t16<true>), g, dim3(512), 0, s, c);
  return hipGetLastError();
}

}  // namespace sfft
