// sfft_device.h -- device helpers shared by the gfx950 kernels of the
// aliasing-filter sparse FFT (one copy per translation unit: everything here
// is inline or in an unnamed namespace).
//
// Pipeline of one exec (any number of signals, one pass per phase):
//   k_reset        zero the per-signal state
//   k_level0_fft   (power-of-two N) per (signal, round): gather of the B0
//                  samples of every delay together (Eq. 5, advance shift),
//                  B0-point FFT in LDS (Eq. 6) as sub-FFTs of <= 8192 points
//   k_level0_stats per signal: mean bucket power, noise quantile
//   k_level0_classify per (signal, 256 classes): Sect. 3.2 Subproblems 1-2,
//                  wave-ballot compaction of single-tons and multi-tons
//   k_ffast        (co-prime N) per signal: stage DFTs and the whole peeling
//                  decoder (Sect. 3.2, Subproblem 3, Eq. 20) in one work-group
//   per tree level l >= 1 (Sect. 3.3):
//     k_sched        prefix sums of the work of every signal
//     k_expand_fft   B'-point FFT of the B' odd-offset samples (B' <= 8192)
//     k_expand_direct  partial DFT sums of the odd-offset samples at the
//                  parents' bins only (Eq. 23 evaluated per node), B' > 8192
//     k_children     child vectors 1/2 (parent +- w Z), classification
//   k_finalize     top-K by magnitude, sort by index, outputs
//
// Bucket relabeling: the GPU reads samples in natural order m = 0..B-1 at
// stride L.  A permutation sigma only relabels buckets under the aliasing
// filter (bin sigma c of the permuted transform is bin c of the natural one),
// so class c is read directly at bin c and sigma never touches the gather.
#pragma once
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "sfft_internal.h"

namespace sfft {

namespace {
constexpr int kZero = 0, kSingle = 1, kMulti = 2, kDouble = 3;

__device__ __forceinline__ float2 cmulf(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 to_d(float2 v) { return make_double2(v.x, v.y); }

// Signal reads through the global address space: a generic pointer would make
// the compiler emit flat loads, which share the wait counter of LDS accesses
// and so serialise every load behind the next LDS read.
typedef __attribute__((address_space(1))) const unsigned long long gu64;
__device__ __forceinline__ float2 ldg_at(gu64 *base, uint64_t i) {
  const unsigned long long v = base[i];
  return make_float2(__uint_as_float((unsigned)v), __uint_as_float((unsigned)(v >> 32)));
}
__device__ __forceinline__ float2 ldg(const float2 *p) { return ldg_at((gu64 *)p, 0); }

// The signal of one solve as its kernels read it: complex64 samples, or the
// packed FP16 form (a header whose first float is the scale s, then pairs of
// binary16; sample n = s (re + i im)).  The branch on the form is uniform
// over a work-group.
struct SigSrc {
  const void *p;  // sample 0
  float scale;    // 1 for complex64
  int fp16;
};
__device__ __forceinline__ SigSrc sig_src(const float2 *x, const SigDesc &d) {
  SigSrc r;
  if (d.fp16) {
    r.p = (const char *)x + SFFT_F16_HEADER_BYTES;
    r.scale = *(const float *)x;
    r.fp16 = 1;
  } else {
    r.p = x;
    r.scale = 1.0f;
    r.fp16 = 0;
  }
  return r;
}
typedef __attribute__((address_space(1))) const unsigned gu32;
// binary16 pair (re in the low half) to complex64, times s
__device__ __forceinline__ float2 half2_to_float2(unsigned v, float s) {
  const float re = __half2float(__ushort_as_half((unsigned short)(v & 0xffffu)));
  const float im = __half2float(__ushort_as_half((unsigned short)(v >> 16)));
  return make_float2(re * s, im * s);
}
__device__ __forceinline__ float2 load_sample(const SigSrc &src, uint64_t i) {
  if (src.fp16) return half2_to_float2(((gu32 *)src.p)[i], src.scale);
  return ldg_at((gu64 *)src.p, i);
}

// acc += a * b (complex, two FMAs per component)
__device__ __forceinline__ void cmac(float2 &acc, float2 a, float2 b) {
  acc.x = fmaf(a.x, b.x, acc.x);
  acc.x = fmaf(-a.y, b.y, acc.x);
  acc.y = fmaf(a.x, b.y, acc.y);
  acc.y = fmaf(a.y, b.x, acc.y);
}

// e^{sign * 2 pi i t / M}, t an exact integer already reduced modulo M
__device__ __forceinline__ double2 unit_d(uint64_t t, uint64_t M, int sign) {
  double s, c;
  sincospi(2.0 * (double)t / (double)M, &s, &c);
  return make_double2(c, sign * s);
}

__device__ __forceinline__ uint64_t mod_n(uint64_t v, const SigDesc &d) {
  return d.log2N >= 0 ? (v & (uint64_t)(d.N - 1)) : v % (uint64_t)d.N;
}

// delay of measurement i of a class vector: shift of its round + its delay;
// FFAST: delay i, or the i-th of the R-FFAST set r_c + 2^c t (Sect. 3.2)
template <bool TREE = true>
__device__ __forceinline__ uint64_t tau_of(const SigDesc &d, int i) {
  if (!TREE) {
    if (d.rf_iters <= 0) return (uint64_t)i;
    const int c = i / d.rf_m, t = i % d.rf_m;
    return (d.rf_off[c] + ((uint64_t)t << c)) % (uint64_t)d.N;
  }
  return mod_n(d.shift[i / d.D] + (uint64_t)(i % d.D), d);
}

__device__ __forceinline__ SigIO io_of(const LaunchCtx &c, int s) {
  return c.io ? c.io[s] : c.io1;
}

__device__ __forceinline__ uint32_t bitrev(uint32_t m, int lg) {
  return lg == 0 ? 0u : (__brev(m) >> (32 - lg));
}

// In-place decimation-in-time FFT of B = 2^lg complex64 values held in LDS
// in bit-reversed order; forward sign e^{-2 pi i hm / B}, no scaling.  Two
// radix-2 stages are fused per pass (radix-2^2): each thread owns four
// points at distance h = 2^{s-1}, so a pass reads and writes LDS once for two
// stages; an odd lg starts with one plain radix-2 stage.  Twiddles come from
// a table of e^{-2 pi i m / 2^lgtw} (the kFftMax-point table by default; any
// lgtw >= lg works, and its first 2^(lg-1) entries are all that are read).
__device__ void fft_lds(float2 *X, int lg, const float2 *__restrict__ tw, int lgtw = kLog2FftMax) {
  const int B = 1 << lg;
  int s = 1;
  if (lg & 1) {
    for (int t = threadIdx.x; t < (B >> 1); t += blockDim.x) {
      const float2 a = X[2 * t], b = X[2 * t + 1];
      X[2 * t] = make_float2(a.x + b.x, a.y + b.y);
      X[2 * t + 1] = make_float2(a.x - b.x, a.y - b.y);
    }
    __syncthreads();
    s = 2;
  }
  for (; s + 1 <= lg; s += 2) {
    const int h = 1 << (s - 1);
    for (int t = threadIdx.x; t < (B >> 2); t += blockDim.x) {
      const int j = t & (h - 1);
      const int i0 = ((t >> (s - 1)) << (s + 1)) + j;
      const float2 w1 = tw[j << (lgtw - s)];       // w_{2h}^j
      const float2 w2 = tw[j << (lgtw - s - 1)];   // w_{4h}^j; w_{4h}^{j+h} = -i w2
      const float2 a0 = X[i0], a1 = cmulf(X[i0 + h], w1);
      const float2 a2 = X[i0 + 2 * h], a3 = cmulf(X[i0 + 3 * h], w1);
      const float2 b0 = make_float2(a0.x + a1.x, a0.y + a1.y);
      const float2 b1 = make_float2(a0.x - a1.x, a0.y - a1.y);
      const float2 b2 = make_float2(a2.x + a3.x, a2.y + a3.y);
      const float2 b3 = make_float2(a2.x - a3.x, a2.y - a3.y);
      const float2 c2 = cmulf(b2, w2);
      const float2 t3 = cmulf(b3, w2);
      const float2 c3 = make_float2(t3.y, -t3.x);
      X[i0] = make_float2(b0.x + c2.x, b0.y + c2.y);
      X[i0 + 2 * h] = make_float2(b0.x - c2.x, b0.y - c2.y);
      X[i0 + h] = make_float2(b1.x + c3.x, b1.y + c3.y);
      X[i0 + 3 * h] = make_float2(b1.x - c3.x, b1.y - c3.y);
    }
    __syncthreads();
  }
}

// All D delays of a sample are read in the same batch of loads (adjacent
// addresses, one cache-line fill): plane dl of lds receives, in bit-reversed
// order, x[((m P + p) L + tau0 + dl) & mask] for m < Bs = 2^lg.
// U: samples (each with its D delays) whose loads a thread issues before the
// first of them is stored.
template <int U>
__device__ __forceinline__ void gather_delays(float2 *lds, const SigSrc &src, int64_t Bs,
                                              int lg, uint64_t L, uint64_t P, uint64_t p,
                                              uint64_t tau0, uint64_t mask, int D) {
  for (int64_t m0 = threadIdx.x; m0 < Bs; m0 += U * (int64_t)blockDim.x) {
    float2 v[U][kMaxD];
#pragma unroll
    for (int u = 0; u < U; u++) {
      const int64_t m = m0 + (int64_t)u * blockDim.x;
      const uint64_t mc = (uint64_t)(m < Bs ? m : Bs - 1);   // in-bounds; stored only if m < Bs
      const uint64_t base = (mc * P + p) * L + tau0;
#pragma unroll
      for (int dl = 0; dl < kMaxD; dl++)
        v[u][dl] = dl < D ? load_sample(src, (base + (uint64_t)dl) & mask) : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int u = 0; u < U; u++) {
      const int64_t m = m0 + (int64_t)u * blockDim.x;
      if (m < Bs) {
        const uint32_t br = bitrev((uint32_t)m, lg);
#pragma unroll
        for (int dl = 0; dl < kMaxD; dl++)
          if (dl < D) lds[(int64_t)dl * Bs + br] = v[u][dl];
      }
    }
  }
}

// e^{-2 pi i t / M} in FP32 for M a power of two: the ratio 2t/M is exact in
// FP32 when M <= 2^24, otherwise the angle is reduced in FP64
__device__ __forceinline__ float2 unit_f(uint64_t t, uint64_t M) {
  if (M <= (1ull << 24)) {
    float sn, cs;
    sincospif(2.0f * (float)t / (float)M, &sn, &cs);
    return make_float2(cs, -sn);
  }
  const double2 u = unit_d(t, M, -1);
  return make_float2((float)u.x, (float)u.y);
}

// wave-wide compaction: lanes with pred get consecutive slots of *counter;
// must be reached by every lane of the wave
__device__ __forceinline__ int wave_append(int32_t *counter, bool pred) {
  const unsigned long long mask = __ballot(pred);
  if (mask == 0ull) return -1;
  const int lane = __lane_id();
  const int leader = __ffsll((long long)mask) - 1;
  int base = 0;
  if (lane == leader) base = atomicAdd(counter, (int)__popcll(mask));
  base = __shfl(base, leader);
  return base + (int)__popcll(mask & ((1ull << lane) - 1ull));
}

// as wave_append, for lanes that append 0, 1 or 2 entries
__device__ __forceinline__ int wave_append_n(int32_t *counter, int cnt) {
  const unsigned long long m1 = __ballot(cnt >= 1), m2 = __ballot(cnt >= 2);
  if (m1 == 0ull) return -1;
  const int lane = __lane_id();
  const int leader = __ffsll((long long)m1) - 1;
  int base = 0;
  if (lane == leader) base = atomicAdd(counter, (int)(__popcll(m1) + __popcll(m2)));
  base = __shfl(base, leader);
  const unsigned long long below = (1ull << lane) - 1ull;
  return base + (int)(__popcll(m1 & below) + __popcll(m2 & below));
}

__device__ double block_sum_d(double v, double *red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double t = 0;
  for (int i = 0; i < (int)(blockDim.x >> 6); i++) t += red[i];
  __syncthreads();
  return t;
}

// exclusive scan of one int per thread over the work-group; returns the
// prefix, *total receives the sum
__device__ int block_scan_excl(int v, int *red, int *total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  int inc = v;
  for (int o = 1; o < 64; o <<= 1) {
    const int u = __shfl_up(inc, o);
    if (lane >= o) inc += u;
  }
  __syncthreads();
  if (lane == 63) red[w] = inc;
  __syncthreads();
  int before = 0, tot = 0;
  for (int i = 0; i < nw; i++) {
    if (i < w) before += red[i];
    tot += red[i];
  }
  __syncthreads();
  *total = tot;
  return before + inc - v;
}

// Uniform values that no kernel writes while the reader runs, read through
// the constant address space so that they come in by scalar loads (which do
// not wait behind the vector loads in flight, and which later stores cannot
// make stale, so nothing is loaded twice).
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(4))) T *cst(const T *p) {
  return (const __attribute__((address_space(4))) T *)p;
}

// index s with pre[s] <= item < pre[s+1] (pre non-decreasing, n+1 entries)
template <typename P>
__device__ __forceinline__ int find_owner(P pre, int n, int item) {
  int lo = 0, hi = n;  // pre[lo] <= item < pre[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (pre[mid] <= item) lo = mid; else hi = mid;
  }
  return lo;
}

// k-th smallest (0-based) of scale*|v|^2 over cnt complex64 values, by a
// four-pass radix select on the float bit patterns (all values >= 0).  For
// work-groups of 256 threads: each thread keeps 8 loads in flight, and the
// pass's digit is found by a scan with one histogram bin a thread.
__device__ float select_kth_power(const float2 *v, int64_t cnt, float scale, int64_t k,
                                  uint32_t *hist, uint32_t *sel) {
  static_assert(kThreads == 256, "one bin a thread");
  __shared__ int scan_red[kThreads / 64];
  const int tid = threadIdx.x;
  uint32_t prefix = 0, mask = 0;
  for (int pass = 0; pass < 4; pass++) {
    const int sh = 24 - 8 * pass;
    hist[tid] = 0;
    __syncthreads();
    for (int64_t i0 = 0; i0 < cnt; i0 += 8 * kThreads) {
      float2 y[8];
#pragma unroll
      for (int j = 0; j < 8; j++) {
        const int64_t i = i0 + j * kThreads + tid;
        y[j] = i < cnt ? v[i] : make_float2(0.f, 0.f);
      }
#pragma unroll
      for (int j = 0; j < 8; j++) {
        const int64_t i = i0 + j * kThreads + tid;
        const uint32_t key = __float_as_uint(scale * (y[j].x * y[j].x + y[j].y * y[j].y));
        if (i < cnt && (key & mask) == prefix) atomicAdd(&hist[(key >> sh) & 255u], 1u);
      }
    }
    __syncthreads();
    // the digit: the bin in which the running count passes k
    const int h = (int)hist[tid];
    int tot;
    const int before = block_scan_excl(h, scan_red, &tot);
    if ((int64_t)before <= k && k < (int64_t)before + h) {
      sel[0] = (uint32_t)tid;
      sel[1] = (uint32_t)(k - before);
    }
    __syncthreads();
    prefix |= sel[0] << sh;
    mask |= 255u << sh;
    k = sel[1];
    __syncthreads();
  }
  return __uint_as_float(prefix);
}

struct Decision {
  int cls;
  int64_t f;
  double2 a;
  int64_t f2;  // two-ton: second position and value
  double2 a2;
};

// lattice index k of class c whose position estimate has phase phi
// (u = phi N / 2 pi snapped to c + k B, Sect. 3.2 Subproblem 2)
__device__ __forceinline__ int64_t lattice_k(double phi, int64_t N, int64_t B, int64_t c) {
  const double two_pi = 6.283185307179586476925286766559;
  if (phi < 0) phi += two_pi;
  const double u = phi * (double)N / two_pi;
  const double kf = floor((u - (double)c) / (double)B + 0.5);
  const int64_t L = N / B;
  int64_t k = (int64_t)kf % L;
  if (k < 0) k += L;
  return k;
}

// principal square root of a complex number (Kahan's form, no cancellation)
__device__ __forceinline__ double2 csqrt_d(double2 z) {
  const double r = hypot(z.x, z.y);
  if (r == 0.0) return make_double2(0.0, 0.0);
  const double t = sqrt(0.5 * (r + fabs(z.x)));
  if (z.x >= 0.0) return make_double2(t, z.y / (2.0 * t));
  return make_double2(fabs(z.y) / (2.0 * t), copysign(t, z.y));
}

__device__ __forceinline__ double2 cdiv_r(double2 a, double r) { return make_double2(a.x / r, a.y / r); }
__device__ __forceinline__ double2 conj_mul(double2 a, double2 b) {  // conj(a) b
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

// Two-ton solve of a class that failed the single-ton test (Sect. 3.1, the
// moment preserving problem with a = 2).  In round r the delays are moments
// m_d = sum_j p_j z_j^d, z_j = e^{2 pi i f_j / N}; the monic z^2 + c1 z + c0
// with roots z_0, z_1 (Eq. 12) gives c0 m_d + c1 m_{d+1} = -m_{d+2} (Eq. 14)
// for d <= D-3, pooled over the rounds by 2x2 normal equations.  The roots
// (Method 1) are snapped to the class lattice; the two values solve the
// Vandermonde system of all measurements in least squares (Eq. 9).  FP64.
template <int NMAX>
__device__ __forceinline__ void two_ton(const double2 (&Y)[NMAX], const SigDesc &d, int n, int rounds,
                                     int64_t c, int64_t B, double T0sq, double T1sq, Decision &v) {
  const int D = d.D;
  const int64_t N = d.N;
  double g00 = 0.0, g11 = 0.0;
  double2 g01 = make_double2(0.0, 0.0), h0 = g01, h1 = g01;
#pragma unroll
  for (int i = 0; i + 2 < NMAX; i++) {
    if (i + 2 < n && (i % D) + 2 < D && (i / D) < rounds) {
      const double2 m0 = Y[i], m1 = Y[i + 1];
      const double2 rhs = make_double2(-Y[i + 2].x, -Y[i + 2].y);
      g00 += m0.x * m0.x + m0.y * m0.y;
      g11 += m1.x * m1.x + m1.y * m1.y;
      const double2 a = conj_mul(m0, m1), b = conj_mul(m0, rhs), e = conj_mul(m1, rhs);
      g01.x += a.x; g01.y += a.y;
      h0.x += b.x; h0.y += b.y;
      h1.x += e.x; h1.y += e.y;
    }
  }
  const double det = g00 * g11 - (g01.x * g01.x + g01.y * g01.y);
  if (!(det > 1e-13 * g00 * g11)) return;
  // C = G^{-1} h with G = [[g00, g01], [conj(g01), g11]]
  const double2 t0 = cmul(g01, h1), t1 = conj_mul(g01, h0);
  const double2 c0 = cdiv_r(make_double2(g11 * h0.x - t0.x, g11 * h0.y - t0.y), det);
  const double2 c1 = cdiv_r(make_double2(g00 * h1.x - t1.x, g00 * h1.y - t1.y), det);
  const double2 c1sq = cmul(c1, c1);
  const double2 sq = csqrt_d(make_double2(c1sq.x - 4.0 * c0.x, c1sq.y - 4.0 * c0.y));
  const double2 z0 = make_double2(0.5 * (-c1.x - sq.x), 0.5 * (-c1.y - sq.y));
  const double2 z1 = make_double2(0.5 * (-c1.x + sq.x), 0.5 * (-c1.y + sq.y));
  int64_t f0 = c + lattice_k(atan2(z0.y, z0.x), N, B, c) * B;
  int64_t f1 = c + lattice_k(atan2(z1.y, z1.x), N, B, c) * B;
  if (f0 == f1) return;
  if (f1 < f0) {
    const int64_t t = f0;
    f0 = f1;
    f1 = t;
  }
  double2 s01 = make_double2(0.0, 0.0), q0 = s01, q1 = s01;
  double E2 = 0.0;
#pragma unroll
  for (int i = 0; i < NMAX; i++) {
    if (i < n) {
      const uint64_t ti = tau_of(d, i);
      const double2 e0 = unit_d(mod_n((uint64_t)f0 * ti, d), (uint64_t)N, +1);
      const double2 e1 = unit_d(mod_n((uint64_t)f1 * ti, d), (uint64_t)N, +1);
      const double2 a = conj_mul(e0, e1), b = conj_mul(e0, Y[i]), e = conj_mul(e1, Y[i]);
      s01.x += a.x; s01.y += a.y;
      q0.x += b.x; q0.y += b.y;
      q1.x += e.x; q1.y += e.y;
      E2 += Y[i].x * Y[i].x + Y[i].y * Y[i].y;
    }
  }
  const double nn = (double)n;
  const double dv = nn * nn - (s01.x * s01.x + s01.y * s01.y);
  if (!(dv > 1e-9 * nn * nn)) return;
  const double2 u0 = cmul(s01, q1);
  const double2 u1 = conj_mul(s01, q0);
  const double2 a0 = cdiv_r(make_double2(nn * q0.x - u0.x, nn * q0.y - u0.y), dv);
  const double2 a1 = cdiv_r(make_double2(nn * q1.x - u1.x, nn * q1.y - u1.y), dv);
  if (nn * (a0.x * a0.x + a0.y * a0.y) <= T0sq) return;
  if (nn * (a1.x * a1.x + a1.y * a1.y) <= T0sq) return;
  // least-squares residual |Y - V a|^2 = |Y|^2 - Re(a^H V^H Y); its rounding
  // error (~1e-16 |Y|^2) is far below the single-ton bound eps1^2 |Y|^2
  const double rho2 = E2 - (a0.x * q0.x + a0.y * q0.y + a1.x * q1.x + a1.y * q1.y);
  if (!(rho2 <= T1sq)) return;
  v.cls = kDouble;
  v.f = f0;
  v.a = a0;
  v.f2 = f1;
  v.a2 = a1;
}

// the enumeration's per-class constants: N, its log2 (-1 when N is not a
// power of two) and the delays tau_i mod N (< N <= 2^30), read from the
// descriptor once per class rather than at every block
template <int NMAX>
struct EnumSig {
  uint64_t N;
  int lgN;
  uint32_t tau[NMAX];
};

__device__ __forceinline__ uint64_t mod_nl(uint64_t v, uint64_t N, int lgN) {
  return lgN >= 0 ? (v & (N - 1)) : v % N;
}

// e^{-2 pi i t / N} for an exact integer t < N, in FP32: from the exact FP32
// ratio 2t/N when N is a power of two up to 2^24, else through FP64
__device__ __forceinline__ float2 unit_nl(uint64_t t, uint64_t N, int lgN) {
  if (lgN >= 0 && lgN <= 24) return unit_f(t, N);
  const double2 u = unit_d(t, N, -1);
  return make_float2((float)u.x, (float)u.y);
}

// the class's constants and the step e^{-2 pi i B tau_i / N} between
// consecutive candidates c + kB
template <int NMAX, bool TREE>
__device__ __forceinline__ void enum_prep(const SigDesc &d, int n, int64_t B, EnumSig<NMAX> &es,
                                          float2 (&st)[NMAX]) {
  es.N = (uint64_t)d.N;
  es.lgN = d.log2N;
#pragma unroll
  for (int i = 0; i < NMAX; i++) es.tau[i] = i < n ? (uint32_t)tau_of<TREE>(d, i) : 0u;
#pragma unroll
  for (int i = 0; i < NMAX; i++)
    st[i] = i < n ? unit_nl(mod_nl((uint64_t)B * es.tau[i], es.N, es.lgN), es.N, es.lgN) : make_float2(0.f, 0.f);
}

// One block of the noisy-mode enumeration (Sect. 3.1, Method 2): the
// matched filter |sum_i Y_i e^{-2 pi i (c + kB) tau_i / N}| of the
// candidates k = lo + o0 + o (mod L), o < min(32, cnt - o0), in FP32 MACs
// with the twiddles anchored exactly at the block's first candidate; folds
// them into (best, bestk): the largest statistic, ties to the smaller k.
template <int NMAX>
__device__ __forceinline__ void enum_block(const float2 (&Yf)[NMAX], const float2 (&st)[NMAX], const EnumSig<NMAX> &es,
                                           int n, int64_t c, int64_t B, int64_t L, int64_t lo, int64_t cnt,
                                           int64_t o0, float &best, int64_t &bestk) {
  float2 tw[NMAX];
  const int64_t k0 = ((lo + o0) % L + L) % L;
  const uint64_t f0 = (uint64_t)(c + k0 * B);
#pragma unroll
  for (int i = 0; i < NMAX; i++)
    if (i < n) tw[i] = unit_nl(mod_nl(f0 * es.tau[i], es.N, es.lgN), es.N, es.lgN);
  const int64_t lim = (cnt - o0) < 32 ? (cnt - o0) : 32;
  for (int64_t o = 0; o < lim; o++) {
    float gx = 0.f, gy = 0.f;
#pragma unroll
    for (int i = 0; i < NMAX; i++) {
      if (i < n) {
        gx += Yf[i].x * tw[i].x - Yf[i].y * tw[i].y;
        gy += Yf[i].x * tw[i].y + Yf[i].y * tw[i].x;
        tw[i] = cmulf(tw[i], st[i]);
      }
    }
    const float m2 = gx * gx + gy * gy;
    int64_t kk = k0 + o;
    if (kk >= L) kk -= L;
    if (m2 > best || (m2 == best && kk < bestk)) {
      best = m2;
      bestk = kk;
    }
  }
}

// position of the r-th set bit of m (r < popcount(m))
__device__ __forceinline__ int nth_set_bit(unsigned long long m, int r) {
  int pos = 0;
#pragma unroll
  for (int w = 32; w >= 1; w >>= 1) {
    const int low = (int)__popcll(m & ((1ull << w) - 1ull));
    if (r >= low) {
      r -= low;
      m >>= w;
      pos += w;
    }
  }
  return pos;
}

// The enumeration of every lane whose `need` is set, by teams: the A needing
// lanes' classes are dealt, in lane order, to teams of T = 2^t adjacent lanes
// (the largest T with A T <= 64, and no larger than the longest range's block
// count); member m of a team takes its class's blocks m, m + T, ... -- the
// blocks and anchors of the one-lane loop, so every statistic is the same
// number -- and the team reduces its best candidate by a butterfly (largest
// statistic, ties to the smaller k).  T = 1 is the one-lane form, T = 64 the
// whole wave on one class.  Every lane of the wave must make the call.
template <int NMAX, bool TREE>
__device__ int64_t enum_team(bool need, const float2 (&Yf)[NMAX], const SigDesc *dp, int n, int64_t c,
                             int64_t B, int64_t lo, int64_t cnt) {
  const unsigned long long mask = __ballot(need);
  const int A = (int)__popcll(mask);
  if (A == 0) return 0;
  const int lane = __lane_id();
  if (__ballot(1) != ~0ull) {
    // not every lane present: each needing lane takes its own class
    float best = -1.0f;
    int64_t bestk = 0;
    if (need) {
      const int64_t L = dp->N / B;
      float2 st[NMAX];
      EnumSig<NMAX> es;
      enum_prep<NMAX, TREE>(*dp, n, B, es, st);
      for (int64_t o0 = 0; o0 < cnt; o0 += 32) enum_block<NMAX>(Yf, st, es, n, c, B, L, lo, cnt, o0, best, bestk);
    }
    return bestk;
  }
  // the longest range (in blocks) among the needing lanes
  int nb = need ? (int)((cnt + 31) >> 5) : 0;
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) nb = max(nb, __shfl_xor(nb, m));
  int lgT = 0;
  while ((A << (lgT + 1)) <= 64 && (1 << (lgT + 1)) <= nb) lgT++;
  const int T = 1 << lgT;
  const int r = lane >> lgT, mem = lane & (T - 1);
  const bool worker = r < A;
  const int src = worker ? nth_set_bit(mask, r) : lane;
  const SigDesc &dj = *(const SigDesc *)__shfl((unsigned long long)dp, src);
  const int nj = __shfl(n, src);
  const int64_t cj = __shfl((long long)c, src), Bj = __shfl((long long)B, src);
  const int64_t loj = __shfl((long long)lo, src), cntj = __shfl((long long)cnt, src);
  float2 Yj[NMAX];
#pragma unroll
  for (int i = 0; i < NMAX; i++) Yj[i] = make_float2(__shfl(Yf[i].x, src), __shfl(Yf[i].y, src));
  float best = -1.0f;
  int64_t bestk = 0;
  if (worker) {
    const int64_t L = dj.N / Bj;
    const int64_t nblk = (cntj + 31) >> 5;
    float2 st[NMAX];
    EnumSig<NMAX> es;
    enum_prep<NMAX, TREE>(dj, nj, Bj, es, st);
    for (int64_t b = mem; b < nblk; b += T)
      enum_block<NMAX>(Yj, st, es, nj, cj, Bj, L, loj, cntj, b << 5, best, bestk);
  }
  for (int m = 1; m < T; m <<= 1) {
    const float ob = __shfl_xor(best, m);
    const int64_t ok = __shfl_xor((long long)bestk, m);
    if (ob > best || (ob == best && ok < bestk)) {
      best = ob;
      bestk = ok;
    }
  }
  // the needing lane of rank q reads its team's first lane
  const int q = (int)__popcll(mask & ((1ull << lane) - 1ull));
  const int64_t res = __shfl((long long)bestk, (need ? q : 0) << lgT);
  return need ? res : 0;
}

// Singleton test (Sect. 3.2, Subproblems 1-2) of one class vector Y (n values,
// rounds x D layout) of class c among B buckets.
// TREE: the two-ton solve may follow (tree kernels); otherwise the R-FFAST
// estimator may locate (FFAST kernel) -- each kernel compiles only its own.
// F32: the single-precision variant of locate / value / residual is compiled
// in (batches holding a plan that asks for it).
template <int NMAX, bool TREE = true, bool F32 = false, bool WAVE = false>
__device__ Decision classify(const double2 (&Y)[NMAX], const SigDesc &d, int n, int rounds,
                            int64_t c, int64_t B, double sref2, double noise_var, bool active = true) {
  Decision v;
  v.cls = kZero;
  v.f = -1;
  v.a = make_double2(0.0, 0.0);
  v.f2 = -1;
  v.a2 = make_double2(0.0, 0.0);
  const int64_t N = d.N;
  const int64_t L = N / B;
  const int D = d.D;
  double E2 = 0.0;
#pragma unroll
  for (int i = 0; i < NMAX; i++)
    if (i < n) E2 += Y[i].x * Y[i].x + Y[i].y * Y[i].y;
  double T0sq, T1sq;
  if (d.mode == SFFT_EXACT) {
    T0sq = d.eps0 * d.eps0 * sref2 * (double)n;
    T1sq = d.eps1 * d.eps1 * E2;
  } else {
    const double sb2 = noise_var / (double)B;
    T0sq = sb2 * ((double)n + d.zero_k * sqrt((double)n));
    T1sq = sb2 * ((double)(n - 1) + d.single_k * sqrt((double)(n - 1)));
  }
  // WAVE: every lane of the wave runs to the enumeration below (which the
  // lanes share), whether its class is active and past the zero-ton test or not
  const bool go = active && !(E2 <= T0sq);
  if (!WAVE && !go) return v;

  // phase-to-index (exact-case locator, advance-shift sign)
  int64_t ksnap = 0;
  const bool rffast = !TREE && d.rf_iters > 0;
  if (!go) {
  } else if (rffast) {
    // R-FFAST estimator: iteration c estimates the angle of e^{2 pi i 2^c f / N}
    // by Kay's weighted phase differences of its m delays (Eq. 21-22) and
    // keeps the lower half of the interval holding f when it lies in [0, pi)
    const double two_pi = 6.283185307179586476925286766559;
    const int m = d.rf_m;
    double lo = 0.0, len = (double)N;
    for (int it = 0; it < d.rf_iters; it++) {
      double th = 0.0;
#pragma unroll
      for (int i = 0; i + 1 < NMAX; i++) {
        if (i / m == it && (i % m) + 1 < m) {
          const double2 a = Y[i + 1], b = Y[i];
          const double px = a.x * b.x + a.y * b.y, py = a.y * b.x - a.x * b.y;
          const double u = (2.0 * (double)(i % m) - (double)m + 2.0) / (double)m;
          const double w = 3.0 * (double)m / (2.0 * ((double)m * (double)m - 1.0)) * (1.0 - u * u);
          th += w * atan2(py, px);
        }
      }
      if (th < 0) th += two_pi;
      len *= 0.5;
      if (th >= 0.5 * two_pi) lo += len;
    }
    const double mid = lo + 0.5 * len;
    int64_t k = (int64_t)floor((mid - (double)c) / (double)B + 0.5) % L;
    if (k < 0) k += L;
    ksnap = k;
  } else if (F32 && D >= 2 && d.precision == 1) {
    // FP32 variant: pooled phase, angle and lattice snap in single precision
    float px = 0.f, py = 0.f;
#pragma unroll
    for (int i = 0; i + 1 < NMAX; i++) {
      if (i + 1 < n && (i % D) != D - 1 && (i / D) < rounds) {
        const float ax = (float)Y[i + 1].x, ay = (float)Y[i + 1].y;
        const float bx = (float)Y[i].x, by = (float)Y[i].y;
        px += ax * bx + ay * by;
        py += ay * bx - ax * by;
      }
    }
    float phi = atan2f(py, px);
    if (phi < 0.f) phi += 6.2831853071795865f;
    const float u = phi * ((float)N / 6.2831853071795865f);
    int64_t kk = (int64_t)floorf((u - (float)c) / (float)B + 0.5f) % L;
    if (kk < 0) kk += L;
    ksnap = kk;
  } else if (D >= 2) {
    double2 P = make_double2(0.0, 0.0);
#pragma unroll
    for (int i = 0; i + 1 < NMAX; i++) {
      if (i + 1 < n && (i % D) != D - 1 && (i / D) < rounds) {
        const double2 a = Y[i + 1], b = Y[i];
        P.x += a.x * b.x + a.y * b.y;
        P.y += a.y * b.x - a.x * b.y;
      }
    }
    ksnap = lattice_k(atan2(P.y, P.x), N, B, c);
  }
  int64_t k = ksnap;
  const bool enumerate = d.mode == SFFT_NOISY && !rffast;
  if (WAVE || (go && enumerate)) {
    // enumeration of the candidates c + kB (Sect. 3.1, Method 2) by the
    // matched filter |sum_i Y_i e^{-2 pi i (c + kB) tau_i / N}|, FP32 MACs,
    // twiddles re-anchored exactly every 32 candidates
    int64_t lo, cnt;
    if (d.window > 0 && D >= 2 && 2 * (int64_t)d.window + 1 < L) {
      lo = ksnap - d.window;
      cnt = 2 * (int64_t)d.window + 1;
    } else {
      lo = 0;
      cnt = L;
    }
    float2 Yf[NMAX];
#pragma unroll
    for (int i = 0; i < NMAX; i++) Yf[i] = make_float2((float)Y[i].x, (float)Y[i].y);
    if (WAVE) {
      // the wave's enumerating classes by teams of lanes (one lane each when
      // they fill the wave, the whole wave for a lone class)
      const int64_t kt = enum_team<NMAX, TREE>(go && enumerate, Yf, &d, n, c, B, lo, cnt);
      if (go && enumerate) k = kt;
    } else {
      float best = -1.0f;
      int64_t bestk = 0;
      float2 st[NMAX];
      EnumSig<NMAX> es;
      enum_prep<NMAX, TREE>(d, n, B, es, st);
      for (int64_t o0 = 0; o0 < cnt; o0 += 32) enum_block<NMAX>(Yf, st, es, n, c, B, L, lo, cnt, o0, best, bestk);
      k = bestk;
    }
  }
  if (!go) return v;
  const int64_t f = c + k * B;
  if (F32 && d.precision == 1) {
    // FP32 variant: value and residual in single precision, FP32 twiddles
    // from exact integer ratios
    float ax = 0.f, ay = 0.f;
#pragma unroll
    for (int i = 0; i < NMAX; i++) {
      if (i < n) {
        const float2 ef = unit_f(mod_n((uint64_t)f * tau_of<TREE>(d, i), d), (uint64_t)N);  // e^{-i..}
        const float yx = (float)Y[i].x, yy = (float)Y[i].y;
        ax += yx * ef.x - yy * ef.y;
        ay += yx * ef.y + yy * ef.x;
      }
    }
    ax /= (float)n;
    ay /= (float)n;
    float r2 = 0.f;
#pragma unroll
    for (int i = 0; i < NMAX; i++) {
      if (i < n) {
        const float2 ef = unit_f(mod_n((uint64_t)f * tau_of<TREE>(d, i), d), (uint64_t)N);
        // a e^{+i..} = a conj(ef)
        const float rx = ax * ef.x + ay * ef.y, ry = ay * ef.x - ax * ef.y;
        const float ex = (float)Y[i].x - rx, ey = (float)Y[i].y - ry;
        r2 += ex * ex + ey * ey;
      }
    }
    v.f = f;
    v.a = make_double2(ax, ay);
    v.cls = ((double)r2 <= T1sq) ? kSingle : kMulti;
    if (TREE && v.cls == kMulti && d.mpp == 2) two_ton<NMAX>(Y, d, n, rounds, c, B, T0sq, T1sq, v);
    return v;
  }
  // value: least-squares mean of the de-rotated measurements (FP64)
  double2 e[NMAX];
  double2 a = make_double2(0.0, 0.0);
#pragma unroll
  for (int i = 0; i < NMAX; i++) {
    if (i < n) {
      e[i] = unit_d(mod_n((uint64_t)f * tau_of<TREE>(d, i), d), (uint64_t)N, -1);
      const double2 t = cmul(Y[i], e[i]);
      a.x += t.x;
      a.y += t.y;
    }
  }
  a.x /= (double)n;
  a.y /= (double)n;
  double rho2 = 0.0;
#pragma unroll
  for (int i = 0; i < NMAX; i++) {
    if (i < n) {
      const double2 r = cmul(a, make_double2(e[i].x, -e[i].y));
      const double ex = Y[i].x - r.x, ey = Y[i].y - r.y;
      rho2 += ex * ex + ey * ey;
    }
  }
  v.f = f;
  v.a = a;
  v.cls = (rho2 <= T1sq) ? kSingle : kMulti;
  if (TREE && v.cls == kMulti && d.mpp == 2) two_ton<NMAX>(Y, d, n, rounds, c, B, T0sq, T1sq, v);
  return v;
}

__device__ __forceinline__ void push_found(const LaunchCtx &c, int s, const SigDesc &d, int slot,
                                           int64_t f, double2 a) {
  if (slot < d.found_cap) {
    c.A.found_f[d.found_off + slot] = f;
    c.A.found_a[d.found_off + slot] = a;
  } else {
    atomicOr(&c.st[s].flags, 3);
  }
}


// signal-set template bucket: n = R*D measurements per class vector
__host__ __device__ inline int nmax_bucket(int n) { return n <= 8 ? 8 : (n <= 16 ? 16 : 64); }

// Launch a classifying kernel KERNEL<NMAX, F32, WAVE> for the batch in c: its
// class-vector size, whether a signal decides in FP32, whether a signal is in
// noisy mode (the team enumeration is compiled into those instances only).
#define SFFT_LAUNCH_FW_(KERNEL, NM, f_, w_, ...)                                  \
  do {                                                                            \
    if (f_ && w_) hipLaunchKernelGGL((KERNEL<NM, true, true>), __VA_ARGS__);      \
    else if (f_) hipLaunchKernelGGL((KERNEL<NM, true, false>), __VA_ARGS__);      \
    else if (w_) hipLaunchKernelGGL((KERNEL<NM, false, true>), __VA_ARGS__);      \
    else hipLaunchKernelGGL((KERNEL<NM, false, false>), __VA_ARGS__);             \
  } while (0)
#define SFFT_LAUNCH_CLASSIFIER(KERNEL, c, ...) SFFT_LAUNCH_CLASSIFIER_W(KERNEL, c, (c).any_noisy != 0, __VA_ARGS__)
// ... with the team enumeration compiled in when `wave` holds
#define SFFT_LAUNCH_CLASSIFIER_W(KERNEL, c, wave, ...)                            \
  do {                                                                            \
    const int nm_ = nmax_bucket((c).nmax);                                        \
    const bool f_ = (c).any_fp32 != 0, w_ = (wave);                               \
    if (nm_ == 8) SFFT_LAUNCH_FW_(KERNEL, 8, f_, w_, __VA_ARGS__);                \
    else if (nm_ == 16) SFFT_LAUNCH_FW_(KERNEL, 16, f_, w_, __VA_ARGS__);         \
    else SFFT_LAUNCH_FW_(KERNEL, 64, f_, w_, __VA_ARGS__);                        \
  } while (0)

}  // namespace

}  // namespace sfft
