// sfft_kernels.hip -- gfx950 kernels of the aliasing-filter sparse FFT.
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
// the kFftMax-point table.
__device__ void fft_lds(float2 *X, int lg, const float2 *__restrict__ tw) {
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
      const float2 w1 = tw[j << (kLog2FftMax - s)];       // w_{2h}^j
      const float2 w2 = tw[j << (kLog2FftMax - s - 1)];   // w_{4h}^j; w_{4h}^{j+h} = -i w2
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
__device__ __forceinline__ void gather_delays(float2 *lds, const float2 *__restrict__ x, int64_t Bs,
                                              int lg, uint64_t L, uint64_t P, uint64_t p,
                                              uint64_t tau0, uint64_t mask, int D) {
  gu64 *xg = (gu64 *)x;
  for (int64_t m0 = threadIdx.x; m0 < Bs; m0 += 4 * (int64_t)blockDim.x) {
    float2 v[4][kMaxD];
#pragma unroll
    for (int u = 0; u < 4; u++) {
      const int64_t m = m0 + (int64_t)u * blockDim.x;
      const uint64_t mc = (uint64_t)(m < Bs ? m : Bs - 1);   // in-bounds; stored only if m < Bs
      const uint64_t base = (mc * P + p) * L + tau0;
#pragma unroll
      for (int dl = 0; dl < kMaxD; dl++)
        v[u][dl] = dl < D ? ldg_at(xg, (base + (uint64_t)dl) & mask) : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int u = 0; u < 4; u++) {
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

// index s with pre[s] <= item < pre[s+1] (pre non-decreasing, n+1 entries)
__device__ __forceinline__ int find_owner(const int32_t *pre, int n, int item) {
  int lo = 0, hi = n;  // pre[lo] <= item < pre[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (pre[mid] <= item) lo = mid; else hi = mid;
  }
  return lo;
}

// k-th smallest (0-based) of scale*|v|^2 over cnt complex64 values, by a
// four-pass radix select on the float bit patterns (all values >= 0)
__device__ float select_kth_power(const float2 *v, int64_t cnt, float scale, int64_t k,
                                  uint32_t *hist, uint32_t *sel) {
  uint32_t prefix = 0, mask = 0;
  for (int pass = 0; pass < 4; pass++) {
    const int sh = 24 - 8 * pass;
    for (int i = threadIdx.x; i < 256; i += blockDim.x) hist[i] = 0;
    __syncthreads();
    for (int64_t i = threadIdx.x; i < cnt; i += blockDim.x) {
      const float2 y = v[i];
      const float p = scale * (y.x * y.x + y.y * y.y);
      const uint32_t key = __float_as_uint(p);
      if ((key & mask) == prefix) atomicAdd(&hist[(key >> sh) & 255u], 1u);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int64_t acc = 0;
      uint32_t dsel = 255;
      for (uint32_t dg = 0; dg < 256; dg++) {
        if (acc + (int64_t)hist[dg] > k) { dsel = dg; break; }
        acc += hist[dg];
      }
      sel[0] = dsel;
      sel[1] = (uint32_t)(k - acc);
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

// Singleton test (Sect. 3.2, Subproblems 1-2) of one class vector Y (n values,
// rounds x D layout) of class c among B buckets.
// TREE: the two-ton solve may follow (tree kernels); otherwise the R-FFAST
// estimator may locate (FFAST kernel) -- each kernel compiles only its own.
// F32: the single-precision variant of locate / value / residual is compiled
// in (batches holding a plan that asks for it).
template <int NMAX, bool TREE = true, bool F32 = false>
__device__ Decision classify(const double2 (&Y)[NMAX], const SigDesc &d, int n, int rounds,
                            int64_t c, int64_t B, double sref2, double noise_var) {
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
  if (E2 <= T0sq) return v;

  // phase-to-index (exact-case locator, advance-shift sign)
  int64_t ksnap = 0;
  const bool rffast = !TREE && d.rf_iters > 0;
  if (rffast) {
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
  if (d.mode == SFFT_NOISY && !rffast) {
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
    float2 Yf[NMAX], tw[NMAX], st[NMAX];
#pragma unroll
    for (int i = 0; i < NMAX; i++) Yf[i] = make_float2((float)Y[i].x, (float)Y[i].y);
    float best = -1.0f;
    int64_t bestk = 0;
    for (int64_t o0 = 0; o0 < cnt; o0 += 32) {
      const int64_t k0 = ((lo + o0) % L + L) % L;
      const uint64_t f0 = (uint64_t)(c + k0 * B);
#pragma unroll
      for (int i = 0; i < NMAX; i++) {
        if (i < n) {
          const uint64_t ti = tau_of<TREE>(d, i);
          const double2 a = unit_d(mod_n(f0 * ti, d), (uint64_t)N, -1);
          const double2 b = unit_d(mod_n(mod_n((uint64_t)B * ti, d), d), (uint64_t)N, -1);
          tw[i] = make_float2((float)a.x, (float)a.y);
          st[i] = make_float2((float)b.x, (float)b.y);
        }
      }
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
    k = bestk;
  }
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

// ---------------------------------------------------------------- kernels

__global__ void k_reset(LaunchCtx c) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
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
  c.st[s] = z;
}

// Level 0 of the tree, bucketization (Eq. 5-6): item = (signal, round r);
// the D delays of every sample are gathered together and transformed by
// P0 = B0 / Bs sub-FFTs of size Bs; with m = m' P0 + p,
//   Yhat[c] = (1/B0) sum_p e^{-2 pi i c p / B0} FFT_Bs(y[m' P0 + p])[c mod Bs],
// accumulated in the level-0 planes Y0[(r D + d) B0 + c] by this work-group
// alone (fixed order, no atomics).
__global__ __launch_bounds__(kThreads) void k_level0_fft(LaunchCtx c) {
  extern __shared__ float2 lds[];
  for (int item = blockIdx.x; item < c.l0_items; item += gridDim.x) {
    const int li = find_owner(c.l0_pre, c.ntree, item);
    const int s = c.tree_list[li];
    const int r = item - c.l0_pre[li];
    const SigDesc &d = c.desc[s];
    const float2 *__restrict__ x = io_of(c, s).x;
    const int64_t N = d.N;
    const int lb = d.log2B0;
    const int64_t B = d.B0;
    const int64_t L = N >> lb;
    const int D = d.D;
    const int lgs = lb < split_lg(D) ? lb : split_lg(D);
    const int64_t Bs = (int64_t)1 << lgs;
    const int P = (int)(B >> lgs);
    const float inv = 1.0f / (float)B;
    float2 *Y0 = c.A.y0 + d.y0_off + (int64_t)r * D * B;
    for (int p = 0; p < P; p++) {
      gather_delays(lds, x, Bs, lgs, (uint64_t)L, (uint64_t)P, (uint64_t)p, d.shift[r],
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
          if (p == 0) *o = v;
          else *o = make_float2(o->x + v.x, o->y + v.y);
        }
      }
      __syncthreads();
    }
  }
}

// Level-0 statistics of every tree signal: mean bucket power and, in noisy
// mode, the noise variance from a quantile of B0 |Yhat|^2.
__global__ __launch_bounds__(kThreads) void k_level0_stats(LaunchCtx c) {
  __shared__ double red[16];
  __shared__ uint32_t hist[256];
  __shared__ uint32_t sel[2];
  for (int li = blockIdx.x; li < c.ntree; li += gridDim.x) {
    const int s = c.tree_list[li];
    const SigDesc &d = c.desc[s];
    const int64_t cnt = (int64_t)d.n * d.B0;
    const float2 *Y0 = c.A.y0 + d.y0_off;
    double psum = 0.0;
    for (int64_t i = threadIdx.x; i < cnt; i += blockDim.x) {
      const float2 v = Y0[i];
      psum += (double)v.x * v.x + (double)v.y * v.y;
    }
    const double sref2 = block_sum_d(psum, red) / (double)cnt;
    double nv = d.noise_var;
    if (d.mode == SFFT_NOISY && !(nv > 0.0)) {
      const float q = select_kth_power(Y0, cnt, (float)d.B0, d.noise_at, hist, sel);
      nv = (double)q / d.noise_p_den;
    }
    if (threadIdx.x == 0) {
      c.st[s].sref2 = sref2;
      c.st[s].noise_var = nv;
      c.st[s].samples = cnt;
      c.st[s].level_mask = 1ull;
      c.st[s].levels = 0;
    }
    __syncthreads();
  }
}

// Classification of the B0 level-0 classes (Sect. 3.2, Subproblems 1-2):
// item = (signal, 256 classes); single-tons and multi-tons are compacted by
// wave ballot + prefix, one atomic per wave and list.
template <int NMAX, bool F32>
__global__ __launch_bounds__(kThreads) void k_level0_classify(LaunchCtx c) {
  for (int item = blockIdx.x; item < c.l0c_items; item += gridDim.x) {
    const int li = find_owner(c.l0c_pre, c.ntree, item);
    const int s = c.tree_list[li];
    const SigDesc &d = c.desc[s];
    const int64_t B = d.B0;
    const int64_t L = d.N >> d.log2B0;
    const int n = d.n;
    const float2 *Y0 = c.A.y0 + d.y0_off;
    const double sref2 = c.st[s].sref2, nv = c.st[s].noise_var;
    const int64_t cc = (int64_t)(item - c.l0c_pre[li]) * kThreads + threadIdx.x;
    const bool valid = cc < B;
    Decision v;
    v.cls = kZero;
    double2 Y[NMAX];
#pragma unroll
    for (int i = 0; i < NMAX; i++) Y[i] = make_double2(0.0, 0.0);
    if (valid) {
#pragma unroll
      for (int i = 0; i < NMAX; i++)
        if (i < n) Y[i] = to_d(Y0[(int64_t)i * B + cc]);
      v = classify<NMAX, true, F32>(Y, d, n, d.R, cc, B, sref2, nv);
    }
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

// FFAST: one work-group per signal runs the stage DFTs and the peeling decoder.
template <int NMAX>
__global__ __launch_bounds__(kThreads) void k_ffast(LaunchCtx c) {
  extern __shared__ float2 lds[];                 // kFftMax samples
  float2 *twd = lds + kFftMax;                     // kDirectMax twiddles
  uint8_t *active = (uint8_t *)(twd + kDirectMax); // kMaxFfastBuckets each
  uint8_t *det = active + kMaxFfastBuckets;
  uint8_t *modf = det + kMaxFfastBuckets;
  uint8_t *cls = modf + kMaxFfastBuckets;
  uint8_t *isnew = cls + kMaxFfastBuckets;
  uint8_t *seen = isnew + kMaxFfastBuckets;
  __shared__ double red[16];
  __shared__ int ired[16];
  __shared__ uint32_t hist[256];
  __shared__ uint32_t sel[2];
  __shared__ int flag_any;
  for (int li = blockIdx.x; li < c.nffast; li += gridDim.x) {
    const int s = c.ffast_list[li];
    const SigDesc &d = c.desc[s];
    const float2 *__restrict__ x = io_of(c, s).x;
    const int64_t N = d.N;
    const int D = d.D;
    const int S = d.nstages;
    const int nb = (int)d.stageOff[S];
    float2 *Y0 = c.A.y0 + d.y0_off;           // complex64 copy (bucketization output)
    double2 *Yf = c.A.fst + d.fst_off;         // FP64 peeling state
    double2 *va = Yf + (int64_t)nb * D;
    int64_t *vf = (int64_t *)(va + nb);
    double psum = 0.0;
    for (int j = 0; j < S; j++) {
      const int64_t B = d.stageB[j];
      const int64_t L = N / B;
      const int lb = (B & (B - 1)) == 0 ? (31 - __clz((int)B)) : -1;
      const float inv = 1.0f / (float)B;
      if (lb < 0) {
        for (int t = threadIdx.x; t < B; t += blockDim.x) {
          const double2 w = unit_d((uint64_t)t, (uint64_t)B, -1);
          twd[t] = make_float2((float)w.x, (float)w.y);
        }
      }
      for (int dl = 0; dl < D; dl++) {
        const uint64_t tdl = tau_of<false>(d, dl);
        for (int64_t m = threadIdx.x; m < B; m += blockDim.x) {
          const uint64_t pos = ((uint64_t)m * (uint64_t)L + tdl) % (uint64_t)N;
          lds[lb >= 0 ? (int64_t)bitrev((uint32_t)m, lb) : m] = ldg(x + pos);
        }
        __syncthreads();
        float2 res[kDirectMax / kThreads];
        if (lb >= 0) {
          fft_lds(lds, lb, c.A.tw);
        } else {
          // direct B-point DFT for a stage that is not a power of two
          int q = 0;
          for (int64_t h = threadIdx.x; h < B; h += blockDim.x, q++) {
            float ax = 0.f, ay = 0.f;
            int64_t t = 0;
            for (int64_t m = 0; m < B; m++) {
              const float2 y = lds[m], w = twd[t];
              ax += y.x * w.x - y.y * w.y;
              ay += y.x * w.y + y.y * w.x;
              t += h;
              if (t >= B) t -= B;
            }
            res[q] = make_float2(ax, ay);
          }
          __syncthreads();
          q = 0;
          for (int64_t h = threadIdx.x; h < B; h += blockDim.x, q++) lds[h] = res[q];
          __syncthreads();
        }
        for (int64_t h = threadIdx.x; h < B; h += blockDim.x) {
          const float2 v = make_float2(lds[h].x * inv, lds[h].y * inv);
          const int64_t b = d.stageOff[j] + h;
          Y0[b * D + dl] = v;
          Yf[b * D + dl] = to_d(v);
          psum += (double)v.x * v.x + (double)v.y * v.y;
        }
        __syncthreads();
      }
    }
    const double sref2 = block_sum_d(psum, red) / (double)((int64_t)nb * D);
    double nv = d.noise_var;
    if (d.mode == SFFT_NOISY && !(nv > 0.0)) {
      // stage sizes differ: select on B_j |Y|^2 needs the per-entry scale, so
      // the select runs on a rescaled FP32 copy held in the FP64 state's tail
      float2 *tmp = (float2 *)(vf + nb);
      for (int b = threadIdx.x; b < nb; b += blockDim.x) {
        int j = 0;
        while (j + 1 < S && d.stageOff[j + 1] <= b) j++;
        const float sc = sqrtf((float)d.stageB[j]);
        for (int dl = 0; dl < D; dl++) {
          const float2 v = Y0[(int64_t)b * D + dl];
          tmp[(int64_t)b * D + dl] = make_float2(v.x * sc, v.y * sc);
        }
      }
      __syncthreads();
      const float q = select_kth_power(tmp, (int64_t)nb * D, 1.0f, d.noise_at, hist, sel);
      nv = (double)q / d.noise_p_den;
    }
    // method 1 activates every bucket; the packet-erasure schedule (method 2)
    // activates the buckets of its start frequencies (their depth-1 trees)
    const bool schedule = d.n_starts > 0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
      active[b] = schedule ? 0 : 1;
      cls[b] = kZero;
      seen[b] = 0;
    }
    __syncthreads();
    if (schedule)
      for (int q = threadIdx.x; q < d.n_starts * S; q += blockDim.x) {
        const int i = q / S, j = q % S;
        active[d.stageOff[j] + (int)(d.start_f[i] % d.stageB[j])] = 1;
      }
    if (threadIdx.x == 0) flag_any = 1;
    __syncthreads();
    int nfound = 0, round = 0, partial = 0, complete = 0, ident = 0;
    const int per = (nb + (int)blockDim.x - 1) / (int)blockDim.x;
    for (;;) {
      if (schedule && nfound < d.K) {
        // the trees died out short of K: the buckets never reached join in
        if (threadIdx.x == 0) flag_any = 0;
        __syncthreads();
        for (int b = threadIdx.x; b < nb; b += blockDim.x)
          if (active[b]) flag_any = 1;
        __syncthreads();
        const int live = flag_any;
        __syncthreads();
        if (!live) {
          for (int b = threadIdx.x; b < nb; b += blockDim.x) {
            active[b] = !seen[b];
            if (active[b]) flag_any = 1;
          }
        }
        __syncthreads();
      }
      if (!flag_any) break;
      if (round == d.max_peel_rounds) {
        partial = 1;
        break;
      }
      // 1. identify every active bucket on the state at the start of the round
      int nid = 0;
      for (int b = threadIdx.x; b < nb; b += blockDim.x) {
        det[b] = 0;
        if (!active[b]) continue;
        seen[b] = 1;
        nid++;
        int j = 0;
        while (j + 1 < S && d.stageOff[j + 1] <= b) j++;
        const int64_t h = b - d.stageOff[j];
        double2 Y[NMAX];
#pragma unroll
        for (int i = 0; i < NMAX; i++) Y[i] = i < D ? Yf[(int64_t)b * D + i] : make_double2(0.0, 0.0);
        const Decision v = classify<NMAX, false>(Y, d, D, 1, h, d.stageB[j], sref2, nv);
        cls[b] = (uint8_t)v.cls;
        if (v.cls == kSingle) {
          det[b] = 1;
          vf[b] = v.f;
          va[b] = v.a;
        }
      }
      __syncthreads();
      // 2. a detection is new unless an earlier bucket (stage-major order) or a
      //    previous round already found the same frequency
      for (int b = threadIdx.x; b < nb; b += blockDim.x) {
        uint8_t nw = 0;
        if (det[b]) {
          nw = 1;
          const int64_t f = vf[b];
          for (int q = 0; q < b && nw; q++)
            if (det[q] && vf[q] == f) nw = 0;
          for (int q = 0; q < nfound && nw; q++)
            if (c.A.found_f[d.found_off + q] == f) nw = 0;
        }
        isnew[b] = nw;
      }
      __syncthreads();
      // 3. append the new frequencies in bucket order (segment scan)
      int cntv = 0;
      const int b0 = threadIdx.x * per;
      for (int b = b0; b < b0 + per && b < nb; b++) cntv += isnew[b];
      int total = 0;
      int pos = block_scan_excl(cntv, ired, &total);
      for (int b = b0; b < b0 + per && b < nb; b++) {
        if (!isnew[b]) continue;
        const int slot = nfound + pos++;
        if (slot < d.found_cap) {
          c.A.found_f[d.found_off + slot] = vf[b];
          c.A.found_a[d.found_off + slot] = va[b];
        }
      }
      int nid_tot = 0;
      (void)block_scan_excl(nid, ired, &nid_tot);
      ident += nid_tot;
      __syncthreads();
      round++;
      if (total == 0) {
        if (!schedule) break;
        for (int b = threadIdx.x; b < nb; b += blockDim.x) active[b] = 0;
        if (threadIdx.x == 0) flag_any = 0;
        __syncthreads();
        continue;
      }
      int nnew = total;
      if (nfound + nnew > d.found_cap) {
        nnew = d.found_cap - nfound;
        partial = 1;
      }
      // 4. subtract every new frequency from its bucket in every stage (Eq. 20)
      for (int b = threadIdx.x; b < nb; b += blockDim.x) {
        int j = 0;
        while (j + 1 < S && d.stageOff[j + 1] <= b) j++;
        const int64_t Bj = d.stageB[j];
        const int64_t h = b - d.stageOff[j];
        uint8_t m = 0;
        for (int q = 0; q < nnew; q++) {
          const int64_t f = c.A.found_f[d.found_off + nfound + q];
          if (f % Bj != h) continue;
          const double2 a = c.A.found_a[d.found_off + nfound + q];
          for (int dl = 0; dl < D; dl++) {
            const double2 r = cmul(a, unit_d(((uint64_t)f * tau_of<false>(d, dl)) % (uint64_t)N, (uint64_t)N, +1));
            Yf[(int64_t)b * D + dl].x -= r.x;
            Yf[(int64_t)b * D + dl].y -= r.y;
          }
          m = 1;
        }
        modf[b] = m;
      }
      nfound += nnew;
      __syncthreads();
      if (threadIdx.x == 0) flag_any = 0;
      __syncthreads();
      // 5. next active set: changed buckets minus those that held a detection
      for (int b = threadIdx.x; b < nb; b += blockDim.x) {
        active[b] = modf[b] && !det[b];
        if (active[b]) flag_any = 1;
      }
      __syncthreads();
      if (partial) break;
      // the schedule ends once K frequencies are identified
      if (schedule && nfound >= d.K) {
        complete = 1;
        break;
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) flag_any = 0;
    __syncthreads();
    if (!complete)
      for (int b = threadIdx.x; b < nb; b += blockDim.x)
        if (cls[b] == kMulti) flag_any = 1;
    __syncthreads();
    if (threadIdx.x == 0) {
      c.st[s].found = nfound;
      c.st[s].flags = (partial || flag_any) ? 1 : 0;
      c.st[s].levels = round;
      c.st[s].ident = ident;
      c.st[s].samples = (int64_t)nb * D;
      c.st[s].sref2 = sref2;
      c.st[s].noise_var = nv;
    }
    __syncthreads();
  }
}

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
            cnt[5] = (int)(Lp / (kColThreads / (Bp / kColQ)));
            cnt[6] = m;
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
__global__ __launch_bounds__(kThreads) void k_expand_fft(LaunchCtx c, int level) {
  extern __shared__ float2 lds[];
  const int par = (level - 1) & 1;
  const int32_t *pf = c.A.pre;
  const int total = pf[c.nsig];
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    const int s = find_owner(pf, c.nsig, item);
    const int rem = item - pf[s];
    const SigDesc &d = c.desc[s];
    const float2 *__restrict__ x = io_of(c, s).x;
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
    gather_delays(lds, x, Bs, lgs, (uint64_t)Lp, (uint64_t)P, (uint64_t)p, tau0, (uint64_t)(N - 1), D);
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
    const float2 *__restrict__ x = io_of(c, s).x;
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
        if (dl < D && m < Bp) z[q][dl] = ldg(x + ((p0 + (uint64_t)dl) & (uint64_t)(N - 1)));
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
template <int NMAX, bool F32>
__global__ __launch_bounds__(kThreads) void k_children(LaunchCtx c, int level) {
  const int par = (level - 1) & 1, cur = level & 1;
  const int32_t *pc = c.A.pre + 2 * (c.nsig + 1);
  const int total = pc[c.nsig];
  for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < total; g += gridDim.x * blockDim.x) {
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
    const Decision v = classify<NMAX, true, F32>(Y, d, n, d.R, cc, B, ss.sref2, ss.noise_var);
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

// Dense pass of the subtree resolution: for every open class c of level-1
// (B' buckets, stride L' <= kJumpMax) accumulate its L' coefficients
//   M_c(t) = sum_{m < B'} x[m L' + t] e^{-2 pi i c m / B'},   t < L'
// (the class's bucket at level-1 measured with shift t, times B') from one
// coalesced read of x.  All L' elements of a row m share the twiddle of the
// row, so the twiddles of a block of rows live in LDS (one entry per class
// and row) and each element costs one complex multiply-add per class.
// Item = (signal, c.jrows rows); thread tid owns t = tid mod L'.
template <int NQ>
__device__ __forceinline__ void jump_rows(const LaunchCtx &c, const SigDesc &d, const float2 *__restrict__ x,
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
    const float2 *xb = x + ((row0 + b0) << lgL);
    gu64 *xg = (gu64 *)xb;
    for (int e0 = threadIdx.x; e0 < ne; e0 += 8 * kThreads) {
      float2 v[8];
#pragma unroll
      for (int u = 0; u < 8; u++) {
        const int e = e0 + u * kThreads;
        v[u] = ldg_at(xg, (uint64_t)(e < ne ? e : ne - 1));   // rows past nb are skipped below
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
__device__ __forceinline__ void jump_rows_mfma(const LaunchCtx &c, const float2 *__restrict__ x, int64_t row0,
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
  gf4 *xv = (gf4 *)x;
  const int ntiles = (nrows + TR - 1) / TR;
  f32x4 pre[PV];
  auto fetch = [&](int t) {
    const int64_t base = (row0 + (int64_t)t * TR) * (Lp / 2);
    const int64_t lim = ((int64_t)nrows - (int64_t)t * TR) * (Lp / 2);
#pragma unroll
    for (int u = 0; u < PV; u++) {
      int64_t i = threadIdx.x + (int64_t)u * kThreads;
      if (i >= lim) i = lim - 1;  // rows past the item: an in-bounds re-read, never used
      pre[u] = xv[base + i];
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
    const float2 *__restrict__ x = io_of(c, s).x;
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
        jump_rows_mfma<(NT > 0 ? NT : 1)>(c, x, row0, nrows, Bp, cls, nq, T, (float *)T, slot0);
      } else {
        float2 (*redv)[64] = (float2 (*)[64])(T + 4096);
        switch (nq) {
          case 1: jump_rows<1>(c, d, x, row0, nrows, lgL, Bp, cls, T, redv, slot0); break;
          case 2: jump_rows<2>(c, d, x, row0, nrows, lgL, Bp, cls, T, redv, slot0); break;
          case 3: jump_rows<3>(c, d, x, row0, nrows, lgL, Bp, cls, T, redv, slot0); break;
          case 4: jump_rows<4>(c, d, x, row0, nrows, lgL, Bp, cls, T, redv, slot0); break;
          case 5: jump_rows<5>(c, d, x, row0, nrows, lgL, Bp, cls, T, redv, slot0); break;
          case 6: jump_rows<6>(c, d, x, row0, nrows, lgL, Bp, cls, T, redv, slot0); break;
          case 7: jump_rows<7>(c, d, x, row0, nrows, lgL, Bp, cls, T, redv, slot0); break;
          case 8: jump_rows<8>(c, d, x, row0, nrows, lgL, Bp, cls, T, redv, slot0); break;
          case 9: jump_rows<9>(c, d, x, row0, nrows, lgL, Bp, cls, T, redv, slot0); break;
          case 10: jump_rows<10>(c, d, x, row0, nrows, lgL, Bp, cls, T, redv, slot0); break;
          case 11: jump_rows<11>(c, d, x, row0, nrows, lgL, Bp, cls, T, redv, slot0); break;
          case 12: jump_rows<12>(c, d, x, row0, nrows, lgL, Bp, cls, T, redv, slot0); break;
          case 13: jump_rows<13>(c, d, x, row0, nrows, lgL, Bp, cls, T, redv, slot0); break;
          case 14: jump_rows<14>(c, d, x, row0, nrows, lgL, Bp, cls, T, redv, slot0); break;
          case 15: jump_rows<15>(c, d, x, row0, nrows, lgL, Bp, cls, T, redv, slot0); break;
          default: jump_rows<16>(c, d, x, row0, nrows, lgL, Bp, cls, T, redv, slot0); break;
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
template <int NMAX, bool F32>
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
      if (k < nq && open_cur[k]) {
        double2 Y[NMAX];
#pragma unroll
        for (int i = 0; i < NMAX; i++) {
          Y[i] = make_double2(0.0, 0.0);
          if (i < n)
            for (int kk = k; kk < Lp; kk += nq) {
              Y[i].x += V[kk][i].x;
              Y[i].y += V[kk][i].y;
            }
        }
        const int64_t cc = cpar + (int64_t)k * Bp;
        const Decision v = classify<NMAX, true, F32>(Y, d, n, d.R, cc, Bd, sref2, nv);
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
      __syncthreads();
      if (k < kJumpMax) open_cur[k] = open_nxt[k];
      const int more = any_open;
      __syncthreads();
      if (!more) break;
    }
    __syncthreads();
  }
}

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

// Level-1 column pass (power-of-two N, B0 = 32 P, P = 2^LP in {32, 64, 128}):
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
// P > 32, a radix-H2 step across adjacent lanes; the results go back to the
// LDS places the thread read.  Only the classes left open at level 0 are then
// stored (raw M_c(t), complex64, one row of L per multi-ton slot).
// One resident work-group per CU walks a contiguous range of items: the
// rows of item k + 1 are in flight while item k is transformed, and no other
// vector-memory load waits behind them (twiddles in LDS, open-class lists
// loaded ahead).  Work-groups 8 apart run on one XCD; such a pair takes the
// two items of each adjacent pair, in step, so that both read the same
// 128-byte lines through one L2.
template <int LP>
__global__ __launch_bounds__(kColThreads, 2) void k_col_pass(LaunchCtx c) {
  constexpr int P = 1 << LP;
  constexpr int B0 = P * kColQ;
  constexpr int LTC = 9 - LP;          // log2 of the columns per item
  constexpr int TC = 1 << LTC;
  constexpr int LH2 = LP - 5;          // lanes of one outer DFT: H2 = P / 32
  constexpr int H2 = 1 << LH2;
  // E[t][k1][p] with strides such that the writes (lanes along t, then p)
  // and the reads (lanes along h, then k1) of every 32 lanes fall on
  // distinct 8-byte bank pairs
  constexpr int SK = P + H2;
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
  gq *fx = nullptr;
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
    fx = (gq *)(c.io ? cst(c.io)[sg].x : c.io1.x) + ((int64_t)(item - pc[sg]) << LTC);
    foff = (uint32_t)(p * L + t);  // < B0 L / 32: fits
    frs = (int64_t)P * L;
    fon = true;
  };
  auto fetch_part = [&](int part) {
    if (!fon) return;
#pragma unroll
    for (int q = 8 * part; q < 8 * part + 8; q++) {
      const unsigned long long u = (fx + q * frs)[foff];
      xn[q] = make_float2(__uint_as_float((unsigned)u), __uint_as_float((unsigned)(u >> 32)));
    }
  };
  // the stored outputs of the item held in E
  bool pend = false;
  int m_p = 0;
  int64_t L_p = 0;
  float2 *out_p = nullptr;
  auto store_outputs = [&]() {
    for (int u = tid; u < (m_p << LTC); u += kColThreads) {
      const int j = u >> LTC, tt = u & (TC - 1);
      const int cc = open_c[j];
      const int k2 = cc >> 5;
      out_p[(int64_t)j * L_p + tt] = E[tt * ST + (cc & 31) * SK + brev_c(k2 >> 5, LH2) + H2 * (k2 & 31)];
    }
  };
  int s = 0;
  while (2 * ip0 + hf >= pc[s + 1]) s++;
  if (cst(c.desc)[s].log2B0 == LP + 5) {
    fetch(2 * ip0 + hf, s);
    for (int part = 0; part < 4; part++) fetch_part(part);
  }
  for (int ip = ip0; ip < ip1; ip++) {
    const int item = 2 * ip + hf;
    while (item >= pc[s + 1]) s++;
    const __attribute__((address_space(4))) SigDesc &d = cst(c.desc)[s];
    const bool mine = d.log2B0 == LP + 5;  // other widths: another launch
    float2 v[kColQ];
#pragma unroll
    for (int q = 0; q < kColQ; q++) v[q] = xn[q];
    int lc[RL];
#pragma unroll
    for (int r = 0; r < RL; r++) lc[r] = ln[r];
    const int m_s = m_n;
    fon = false;
    if (ip + 1 < ip1) {
      int ns = s;
      while (item + 2 >= pc[ns + 1]) ns++;
      if (cst(c.desc)[ns].log2B0 == LP + 5) fetch(item + 2, ns);
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
    {
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
    L_p = d.N >> d.log2B0;
    out_p = c.A.jcol + d.jc_off + ((int64_t)(item - pc[s]) << LTC);
  }
  if (pend) store_outputs();
}

// acc += sum over u = u0, u0 + du, ... < nq of M[u Ld] w_u, w_u advancing by
// st per term; the loads go out CH at a time
template <int CH>
__device__ __forceinline__ void col_sum(const float2 *M, uint64_t Ld, int u0, int du, int nq, double2 w,
                                        double2 st, double2 &acc) {
  for (int ub = u0; ub < nq; ub += CH * du) {
    float2 mv[CH];
#pragma unroll
    for (int j = 0; j < CH; j++) {
      const int u = ub + j * du;
      mv[j] = u < nq ? M[(uint64_t)u * Ld] : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int j = 0; j < CH; j++) {
      acc.x += (double)mv[j].x * w.x - (double)mv[j].y * w.y;
      acc.y += (double)mv[j].x * w.y + (double)mv[j].y * w.x;
      w = cmul(w, st);
    }
  }
}

// Subtree resolution from the column pass.  Each open level-0 class c is
// served by a group of kColGroup lanes (a wave serves 64 / kColGroup classes
// side by side, so that their classifications run together).  Its subclass
// cs = c + k B0 at depth dd (level dd: B_d = B0 2^dd buckets of stride
// L_d = L / 2^dd) has, for measurement delay tau_i, the class-vector entry
//   Y_i = 1/B_d sum_{u < 2^dd} M_c(t_u) e^{-2 pi i cs (t_u - tau_i) / N},
//   t_u = (tau_i mod L_d) + u L_d,
// which is the aliasing-filter bucket of Eq. 5 at B_d buckets with its B_d
// samples grouped by the column of x they lie in: the same linear functional
// of x as the gathered bucket of that level.  Along u the twiddle advances
// by e^{-2 pi i cs L_d / N}.  Down to depth kColLaneDepth the group's lanes
// take one (subclass, measurement) sum each; deeper (2^dd terms per sum) the
// whole wave shares each sum.  Depth by depth the open subclasses are then
// classified as the tree search does (Sect. 3.3), one lane each:
// single-tons (and two-tons) are recorded, multi-tons open their children.
template <int NMAX, bool F32>
__global__ __launch_bounds__(64, 2) void k_col_resolve(LaunchCtx c) {
  constexpr int GS = kColGroup, LGS = kColGroupLg, CPW = 64 / GS, CAP = kColResolveCap;
  __shared__ double2 Ys[CPW][GS][NMAX];
  __shared__ int open_cur[CPW][CAP], open_nxt[CPW][CAP];
  __shared__ int n_nxt[CPW];
  __shared__ int deep[64];
  __shared__ int n_deep;
  const int32_t *pr = c.A.pre + 6 * (c.nsig + 1);
  const int total = pr[c.nsig];
  const int lane = threadIdx.x, g = lane >> LGS, gl = lane & (GS - 1);
  for (int base = blockIdx.x * CPW; base < total; base += gridDim.x * CPW) {
    const int item = base + g;
    const bool valid = item < total;
    const int s = valid ? find_owner(pr, c.nsig, item) : 0;
    const int jslot = valid ? item - pr[s] : 0;
    const SigDesc &d = c.desc[s];
    const uint64_t N = (uint64_t)d.N;
    const int n = valid ? d.n : 0;
    const uint64_t L = N >> d.log2B0;
    const uint64_t cpar = valid ? (uint64_t)c.A.multi_c[0][d.multi_off + jslot] : 0;
    const float2 *M = c.A.jcol + d.jc_off + (int64_t)jslot * (int64_t)L;
    const double sref2 = c.st[s].sref2, nv = c.st[s].noise_var;
    int nopen = valid ? 2 : 0;
    __syncthreads();  // the previous classes are done with the lists
    if (gl < 2) open_cur[g][gl] = gl;
    for (int dd = 1; __any(nopen > 0); dd++) {
      const int nq = 1 << dd;
      const int64_t Bd = d.B0 << dd;
      const uint64_t Ld = L >> dd;
      if (gl == 0) n_nxt[g] = 0;
      __syncthreads();
      for (int ch = 0; __any(ch * GS < nopen); ch++) {
        const int left = nopen - ch * GS;
        const int no = left < 0 ? 0 : (left < GS ? left : GS);
        if (dd <= kColLaneDepth) {
          for (int e = gl; e < no * n; e += GS) {
            const int oi = e / n, i = e - oi * n;
            const uint64_t cs = cpar + (uint64_t)open_cur[g][ch * GS + oi] * (uint64_t)d.B0;
            const uint64_t tau = tau_of(d, i);
            const uint64_t tr = tau & (Ld - 1);
            double2 w = unit_d((cs * ((tr - tau) & (N - 1))) & (N - 1), N, -1);
            const double2 st = unit_d((cs * Ld) & (N - 1), N, -1);
            double2 acc = make_double2(0.0, 0.0);
            col_sum<8>(M + tr, Ld, 0, 1, nq, w, st, acc);
            const double sc = 1.0 / (double)Bd;
            Ys[g][oi][i] = make_double2(acc.x * sc, acc.y * sc);
          }
        } else {
          // the wave's open subclasses of this chunk, one after the other;
          // 8 lanes per measurement, lane uu taking u = uu, uu + 8, ...
          if (lane == 0) n_deep = 0;
          __syncthreads();
          if (gl < no) deep[atomicAdd(&n_deep, 1)] = (g << LGS) | gl;
          __syncthreads();
          const int nd = n_deep;
          const int im = lane >> 3, uu = lane & 7;
          for (int e = 0; e < nd; e++) {
            const int ge = deep[e] >> LGS, oe = deep[e] & (GS - 1);
            const int src = ge << LGS;
            const int se = __shfl(s, src);
            const int je = __shfl(jslot, src);
            const uint64_t ce = (uint64_t)__shfl((unsigned long long)cpar, src);
            const SigDesc &de = c.desc[se];
            const uint64_t Ne = (uint64_t)de.N, Le = Ne >> de.log2B0, Lde = Le >> dd;
            const float2 *Me = c.A.jcol + de.jc_off + (int64_t)je * (int64_t)Le;
            const uint64_t cs = ce + (uint64_t)open_cur[ge][ch * GS + oe] * (uint64_t)de.B0;
            const double2 st = unit_d((cs * ((Lde << 3) & (Ne - 1))) & (Ne - 1), Ne, -1);
            for (int i0 = 0; i0 < de.n; i0 += 8) {
              const int i = i0 + im;
              double2 acc = make_double2(0.0, 0.0);
              if (i < de.n) {
                const uint64_t tau = tau_of(de, i);
                const uint64_t tr = tau & (Lde - 1);
                const uint64_t t0 = tr + (uint64_t)uu * Lde;
                double2 w = unit_d((cs * ((t0 - tau) & (Ne - 1))) & (Ne - 1), Ne, -1);
                col_sum<8>(Me + tr, Lde, uu, 8, nq, w, st, acc);
              }
              for (int o = 4; o >= 1; o >>= 1) {
                acc.x += __shfl_xor(acc.x, o);
                acc.y += __shfl_xor(acc.y, o);
              }
              if (uu == 0 && i < de.n) {
                const double sc = 1.0 / (double)((int64_t)de.B0 << dd);
                Ys[ge][oe][i] = make_double2(acc.x * sc, acc.y * sc);
              }
            }
          }
        }
        __syncthreads();
        if (gl < no) {
          const int k = open_cur[g][ch * GS + gl];
          const int64_t cs = (int64_t)cpar + (int64_t)k * d.B0;
          double2 Y[NMAX];
#pragma unroll
          for (int i = 0; i < NMAX; i++) Y[i] = i < n ? Ys[g][gl][i] : make_double2(0.0, 0.0);
          const Decision v = classify<NMAX, true, F32>(Y, d, n, d.R, cs, Bd, sref2, nv);
          atomicMax(&c.st[s].levels, dd);
          if (v.cls == kSingle) {
            const int fs = atomicAdd(&c.st[s].found, 1);
            push_found(c, s, d, fs, v.f, v.a);
          } else if (v.cls == kDouble) {
            const int fs = atomicAdd(&c.st[s].found, 2);
            push_found(c, s, d, fs, v.f, v.a);
            push_found(c, s, d, fs + 1, v.f2, v.a2);
          } else if (v.cls == kMulti) {
            if (Ld >= 2 && dd + 1 <= d.max_levels) {
              const int at = atomicAdd(&n_nxt[g], 2);
              if (at + 2 <= CAP) {
                open_nxt[g][at] = k;
                open_nxt[g][at + 1] = k + nq;
              } else {
                atomicOr(&c.st[s].flags, 1);
              }
            } else {
              atomicOr(&c.st[s].flags, 1);
            }
          }
        }
        __syncthreads();
      }
      nopen = n_nxt[g] < CAP ? n_nxt[g] : CAP;
      for (int k = gl; k < nopen; k += GS) open_cur[g][k] = open_nxt[g][k];
      __syncthreads();
    }
  }
}

// Top-K by magnitude (ties: lower index), then ascending index; padding.
__global__ __launch_bounds__(kThreads) void k_finalize(LaunchCtx c) {
  extern __shared__ uint64_t keys[];
  int32_t *ix = (int32_t *)(keys + c.max_found_cap);
  for (int s = blockIdx.x; s < c.nsig; s += gridDim.x) {
    const SigDesc &d = c.desc[s];
    const SigIO io = io_of(c, s);
    int cnt = c.st[s].found;
    if (cnt > d.found_cap) cnt = d.found_cap;
    const int K = (int)d.K;
    const int64_t *ff = c.A.found_f + d.found_off;
    const double2 *fa = c.A.found_a + d.found_off;
    int kept = cnt < K ? cnt : K;
    int P = 1;
    while (P < cnt) P <<= 1;
    if (cnt > K) {
      // sort by (magnitude descending, index ascending)
      for (int i = threadIdx.x; i < P; i += blockDim.x) {
        if (i < cnt) {
          const double2 a = fa[i];
          const double m2 = a.x * a.x + a.y * a.y;
          keys[i] = ~(uint64_t)__double_as_longlong(m2);
        } else {
          keys[i] = ~0ull;
        }
        ix[i] = i;
      }
      __syncthreads();
      for (int k = 2; k <= P; k <<= 1)
        for (int jj = k >> 1; jj > 0; jj >>= 1) {
          for (int i = threadIdx.x; i < P; i += blockDim.x) {
            const int o = i ^ jj;
            if (o > i) {
              const uint64_t ka = keys[i], kb = keys[o];
              bool gt = ka > kb;
              if (ka == kb && ix[i] < cnt && ix[o] < cnt) gt = ff[ix[i]] > ff[ix[o]];
              if (gt == ((i & k) == 0)) {
                keys[i] = kb;
                keys[o] = ka;
                const int t = ix[i];
                ix[i] = ix[o];
                ix[o] = t;
              }
            }
          }
          __syncthreads();
        }
    } else {
      for (int i = threadIdx.x; i < P; i += blockDim.x) ix[i] = i;
      __syncthreads();
    }
    // sort the kept entries by index
    int P2 = 1;
    while (P2 < kept) P2 <<= 1;
    for (int i = threadIdx.x; i < P2; i += blockDim.x) {
      keys[i] = i < kept ? (uint64_t)ff[ix[i]] : ~0ull;
      if (i >= kept) ix[i] = -1;
    }
    __syncthreads();
    for (int k = 2; k <= P2; k <<= 1)
      for (int jj = k >> 1; jj > 0; jj >>= 1) {
        for (int i = threadIdx.x; i < P2; i += blockDim.x) {
          const int o = i ^ jj;
          if (o > i) {
            const uint64_t ka = keys[i], kb = keys[o];
            if ((ka > kb) == ((i & k) == 0)) {
              keys[i] = kb;
              keys[o] = ka;
              const int t = ix[i];
              ix[i] = ix[o];
              ix[o] = t;
            }
          }
        }
        __syncthreads();
      }
    for (int i = threadIdx.x; i < K; i += blockDim.x) {
      if (i < kept) {
        io.idx[i] = ff[ix[i]];
        const double2 a = fa[ix[i]];
        io.val[i] = make_float2((float)a.x, (float)a.y);
      } else {
        io.idx[i] = -1;
        io.val[i] = make_float2(0.f, 0.f);
      }
    }
    if (threadIdx.x == 0) {
      *io.count = kept;
      *io.status = c.st[s].flags ? SFFT_STATUS_PARTIAL : SFFT_STATUS_OK;
    }
    __syncthreads();
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

static int nmax_bucket(int n) { return n <= 8 ? 8 : (n <= 16 ? 16 : 64); }

// kernels whose dynamic LDS can exceed 64 KiB declare the gfx950 maximum once
static void configure_lds() {
  static bool done = false;
  if (done) return;
  done = true;
  const int big = 160 * 1024;
  (void)hipFuncSetAttribute((const void *)k_ffast<8>, hipFuncAttributeMaxDynamicSharedMemorySize, big);
  (void)hipFuncSetAttribute((const void *)k_ffast<16>, hipFuncAttributeMaxDynamicSharedMemorySize, big);
  (void)hipFuncSetAttribute((const void *)k_ffast<64>, hipFuncAttributeMaxDynamicSharedMemorySize, big);
  (void)hipFuncSetAttribute((const void *)k_finalize, hipFuncAttributeMaxDynamicSharedMemorySize, big);
  (void)hipGetLastError();
}

hipError_t launch_reset(const LaunchCtx &c, hipStream_t s) {
  configure_lds();
  hipLaunchKernelGGL(k_reset, dim3((c.nsig + 255) / 256), dim3(256), 0, s, c);
  return hipGetLastError();
}

hipError_t launch_level0(const LaunchCtx &c, hipStream_t s) {
  const int nm = nmax_bucket(c.nmax);
  if (c.ntree > 0) {
    const size_t lds = 64 * 1024;
    hipLaunchKernelGGL(k_level0_fft, dim3(c.l0_items < 8192 ? c.l0_items : 8192), dim3(kThreads),
                       lds, s, c);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_level0_stats, dim3(c.ntree < 4096 ? c.ntree : 4096), dim3(kThreads), 0, s, c);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int g = c.l0c_items < 8192 ? c.l0c_items : 8192;
    if (c.any_fp32) {
      if (nm == 8) hipLaunchKernelGGL((k_level0_classify<8, true>), dim3(g), dim3(kThreads), 0, s, c);
      else if (nm == 16) hipLaunchKernelGGL((k_level0_classify<16, true>), dim3(g), dim3(kThreads), 0, s, c);
      else hipLaunchKernelGGL((k_level0_classify<64, true>), dim3(g), dim3(kThreads), 0, s, c);
    } else {
      if (nm == 8) hipLaunchKernelGGL((k_level0_classify<8, false>), dim3(g), dim3(kThreads), 0, s, c);
      else if (nm == 16) hipLaunchKernelGGL((k_level0_classify<16, false>), dim3(g), dim3(kThreads), 0, s, c);
      else hipLaunchKernelGGL((k_level0_classify<64, false>), dim3(g), dim3(kThreads), 0, s, c);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (c.nffast > 0) {
    const int grid = c.nffast < 4096 ? c.nffast : 4096;
    const size_t lds = sizeof(float2) * (kFftMax + kDirectMax) + 6 * kMaxFfastBuckets;
    if (nm == 8) hipLaunchKernelGGL(k_ffast<8>, dim3(grid), dim3(kThreads), lds, s, c);
    else if (nm == 16) hipLaunchKernelGGL(k_ffast<16>, dim3(grid), dim3(kThreads), lds, s, c);
    else hipLaunchKernelGGL(k_ffast<64>, dim3(grid), dim3(kThreads), lds, s, c);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_sched(const LaunchCtx &c, int level, hipStream_t s) {
  hipLaunchKernelGGL(k_sched, dim3(1), dim3(1024), 0, s, c, level);
  return hipGetLastError();
}

hipError_t launch_expand_fft(const LaunchCtx &c, int level, int grid, hipStream_t s) {
  const size_t lds = 64 * 1024;
  hipLaunchKernelGGL(k_expand_fft, dim3(grid), dim3(kThreads), lds, s, c, level);
  return hipGetLastError();
}

hipError_t launch_expand_direct(const LaunchCtx &c, int level, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_expand_direct, dim3(grid), dim3(kThreads), 0, s, c, level);
  return hipGetLastError();
}

hipError_t launch_jump_pass(const LaunchCtx &c, int level, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_jump_pass<0>, dim3(grid), dim3(kThreads), 0, s, c, level);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !c.any_wide_jump) return e;
  if (5 >= kJumpMfmaMinLg) hipLaunchKernelGGL(k_jump_pass<1>, dim3(grid), dim3(kThreads), 0, s, c, level);
  if (6 >= kJumpMfmaMinLg) hipLaunchKernelGGL(k_jump_pass<2>, dim3(grid), dim3(kThreads), 0, s, c, level);
  hipLaunchKernelGGL(k_jump_pass<4>, dim3(grid), dim3(kThreads), 0, s, c, level);
  return hipGetLastError();
}

hipError_t launch_col_pass(const LaunchCtx &c, int grid, hipStream_t s) {
  if (c.col_lp_mask & 1) hipLaunchKernelGGL(k_col_pass<5>, dim3(grid), dim3(kColThreads), 0, s, c);
  if (c.col_lp_mask & 2) hipLaunchKernelGGL(k_col_pass<6>, dim3(grid), dim3(kColThreads), 0, s, c);
  if (c.col_lp_mask & 4) hipLaunchKernelGGL(k_col_pass<7>, dim3(grid), dim3(kColThreads), 0, s, c);
  return hipGetLastError();
}

hipError_t launch_col_resolve(const LaunchCtx &c, int grid, hipStream_t s) {
  const int nm = nmax_bucket(c.nmax);
  if (c.any_fp32) {
    if (nm == 8) hipLaunchKernelGGL((k_col_resolve<8, true>), dim3(grid), dim3(64), 0, s, c);
    else if (nm == 16) hipLaunchKernelGGL((k_col_resolve<16, true>), dim3(grid), dim3(64), 0, s, c);
    else hipLaunchKernelGGL((k_col_resolve<64, true>), dim3(grid), dim3(64), 0, s, c);
  } else {
    if (nm == 8) hipLaunchKernelGGL((k_col_resolve<8, false>), dim3(grid), dim3(64), 0, s, c);
    else if (nm == 16) hipLaunchKernelGGL((k_col_resolve<16, false>), dim3(grid), dim3(64), 0, s, c);
    else hipLaunchKernelGGL((k_col_resolve<64, false>), dim3(grid), dim3(64), 0, s, c);
  }
  return hipGetLastError();
}

hipError_t launch_jump_resolve(const LaunchCtx &c, int level, int grid, hipStream_t s) {
  const int nm = nmax_bucket(c.nmax);
  if (c.any_fp32) {
    if (nm == 8) hipLaunchKernelGGL((k_jump_resolve<8, true>), dim3(grid), dim3(kJumpMax), 0, s, c, level);
    else if (nm == 16) hipLaunchKernelGGL((k_jump_resolve<16, true>), dim3(grid), dim3(kJumpMax), 0, s, c, level);
    else hipLaunchKernelGGL((k_jump_resolve<64, true>), dim3(grid), dim3(kJumpMax), 0, s, c, level);
  } else {
    if (nm == 8) hipLaunchKernelGGL((k_jump_resolve<8, false>), dim3(grid), dim3(kJumpMax), 0, s, c, level);
    else if (nm == 16) hipLaunchKernelGGL((k_jump_resolve<16, false>), dim3(grid), dim3(kJumpMax), 0, s, c, level);
    else hipLaunchKernelGGL((k_jump_resolve<64, false>), dim3(grid), dim3(kJumpMax), 0, s, c, level);
  }
  return hipGetLastError();
}

hipError_t launch_children(const LaunchCtx &c, int level, int grid, hipStream_t s) {
  const int nm = nmax_bucket(c.nmax);
  if (c.any_fp32) {
    if (nm == 8) hipLaunchKernelGGL((k_children<8, true>), dim3(grid), dim3(kThreads), 0, s, c, level);
    else if (nm == 16) hipLaunchKernelGGL((k_children<16, true>), dim3(grid), dim3(kThreads), 0, s, c, level);
    else hipLaunchKernelGGL((k_children<64, true>), dim3(grid), dim3(kThreads), 0, s, c, level);
  } else {
    if (nm == 8) hipLaunchKernelGGL((k_children<8, false>), dim3(grid), dim3(kThreads), 0, s, c, level);
    else if (nm == 16) hipLaunchKernelGGL((k_children<16, false>), dim3(grid), dim3(kThreads), 0, s, c, level);
    else hipLaunchKernelGGL((k_children<64, false>), dim3(grid), dim3(kThreads), 0, s, c, level);
  }
  return hipGetLastError();
}

hipError_t launch_finalize(const LaunchCtx &c, hipStream_t s) {
  const int grid = c.nsig < 4096 ? c.nsig : 4096;
  const size_t lds = (sizeof(uint64_t) + sizeof(int32_t)) * (size_t)c.max_found_cap;
  hipLaunchKernelGGL(k_finalize, dim3(grid), dim3(kThreads), lds, s, c);
  return hipGetLastError();
}

}  // namespace sfft
