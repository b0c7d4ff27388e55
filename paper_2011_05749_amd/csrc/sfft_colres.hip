// sfft_colres.hip -- subtree resolution of every level-0 multi-ton from the
// coefficients M_c(t) of the level-1 column pass (Sect. 3.3).
#include "sfft_device.h"

namespace sfft {

namespace {

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

// The depth-dd sums of one measurement (delay tau, tr = tau mod L_d) for the
// chunk's `no` open subclasses: its NQ = 2^dd coefficients M[tr + u L_d] are
// loaded once (all in flight together), then each subclass's sum runs over
// them in registers with the twiddle advancing term by term, in the order and
// arithmetic of col_sum; the result, over B_d, goes to Y[oi * stride].
template <int NQ>
__device__ __forceinline__ void lane_sums(const float2 *Mt, uint64_t Ld, const SigDesc &d, uint64_t N, uint64_t cpar,
                                          const int *open, int no, uint64_t tau, uint64_t tr, double sc, double2 *Y,
                                          int stride) {
  float2 mv[NQ];
#pragma unroll
  for (int u = 0; u < NQ; u++) mv[u] = Mt[(uint64_t)u * Ld];
  for (int oi = 0; oi < no; oi++) {
    const uint64_t cs = cpar + (uint64_t)open[oi] * (uint64_t)d.B0;
    double2 w = unit_d((cs * ((tr - tau) & (N - 1))) & (N - 1), N, -1);
    const double2 st = unit_d((cs * Ld) & (N - 1), N, -1);
    double2 acc = make_double2(0.0, 0.0);
#pragma unroll
    for (int u = 0; u < NQ; u++) {
      acc.x += (double)mv[u].x * w.x - (double)mv[u].y * w.y;
      acc.y += (double)mv[u].x * w.y + (double)mv[u].y * w.x;
      w = cmul(w, st);
    }
    Y[oi * stride] = make_double2(acc.x * sc, acc.y * sc);
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
template <int NMAX, bool F32, bool WAVE>
__global__ __launch_bounds__(64, 2) void k_col_resolve(LaunchCtx c) {
  constexpr int GS = kColGroup, LGS = kColGroupLg, CPW = 64 / GS, CAP = kColResolveCap;
  __shared__ double2 Ys[CPW][GS][NMAX];
  __shared__ int open_cur[CPW][CAP], open_nxt[CPW][CAP];
  __shared__ int n_nxt[CPW];
  __shared__ int deep[64];
  __shared__ int n_deep;
  __shared__ unsigned long long dmask[CPW];  // open subclasses at depth col_dz + 1
  static_assert(CPW == kColResolveAlign, "a wave's classes are one aligned group");
  const __attribute__((address_space(4))) int32_t *pr = cst(c.A.pre + 6 * (c.nsig + 1));
  const int total = pr[c.nsig];
  const int lane = threadIdx.x, g = lane >> LGS, gl = lane & (GS - 1);
  for (int base = blockIdx.x * CPW; base < total; base += gridDim.x * CPW) {
    // each signal's classes are padded to whole groups of CPW, so that the
    // wave's all belong to one signal, its descriptor read by scalar loads
    const int s = find_owner(pr, c.nsig, base);
    const SigDesc &d = *(const SigDesc *)&cst(c.desc)[s];
    const int jslot = base + g - pr[s];
    const int mcnt = cst(c.st)[s].multi[0];
    const bool valid = jslot < (mcnt < d.col_rows ? mcnt : d.col_rows);
    const uint64_t N = (uint64_t)d.N;
    const int n = valid ? d.n : 0;
    const uint64_t L = N >> d.log2B0;
    const uint64_t cpar = valid ? (uint64_t)c.A.multi_c[0][d.multi_off + jslot] : 0;
    const float2 *M = c.A.jcol + d.jc_off + (int64_t)jslot * (int64_t)L;
    const double sref2 = cst(c.st)[s].sref2, nv = cst(c.st)[s].noise_var;
    int nopen = valid ? 2 : 0;
    int deepest = 0;  // the class's deepest classified level (one atomic per class, at its end)
    __syncthreads();  // the previous classes are done with the lists
    if (gl < 2) open_cur[g][gl] = gl;
    if (gl == 0) dmask[g] = 0;
    for (int dd = 1; __any(nopen > 0); dd++) {
      if (nopen > 0) deepest = dd;
      const int nq = 1 << dd;
      const int64_t Bd = d.B0 << dd;
      const uint64_t Ld = L >> dd;
      if (gl == 0) n_nxt[g] = 0;
      __syncthreads();
      for (int ch = 0; __any(ch * GS < nopen); ch++) {
        const int left = nopen - ch * GS;
        const int no = left < 0 ? 0 : (left < GS ? left : GS);
        if (dd <= kColLaneDepth) {
          // lane gl takes measurements gl, gl + GS, ... for every open subclass
          static_assert(kColLaneDepth == 5, "lane sums are instantiated for 2 .. 32 terms");
          const double sc = 1.0 / (double)Bd;
          for (int i = gl; no > 0 && i < n; i += GS) {
            const uint64_t tau = tau_of(d, i);
            const uint64_t tr = tau & (Ld - 1);
            const int *op = &open_cur[g][ch * GS];
            double2 *yo = &Ys[g][0][i];
            switch (dd) {
              case 1: lane_sums<2>(M + tr, Ld, d, N, cpar, op, no, tau, tr, sc, yo, NMAX); break;
              case 2: lane_sums<4>(M + tr, Ld, d, N, cpar, op, no, tau, tr, sc, yo, NMAX); break;
              case 3: lane_sums<8>(M + tr, Ld, d, N, cpar, op, no, tau, tr, sc, yo, NMAX); break;
              case 4: lane_sums<16>(M + tr, Ld, d, N, cpar, op, no, tau, tr, sc, yo, NMAX); break;
              default: lane_sums<32>(M + tr, Ld, d, N, cpar, op, no, tau, tr, sc, yo, NMAX); break;
            }
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
        {
          // every lane takes part (the noisy enumeration may run in teams of the wave's lanes)
          const bool act = gl < no;
          const int k = act ? open_cur[g][ch * GS + gl] : 0;
          const int64_t cs = (int64_t)cpar + (int64_t)k * d.B0;
          double2 Y[NMAX];
#pragma unroll
          for (int i = 0; i < NMAX; i++) Y[i] = act && i < n ? Ys[g][gl][i] : make_double2(0.0, 0.0);
          const Decision v = classify<NMAX, true, F32, WAVE>(Y, d, n, d.R, cs, Bd, sref2, nv, act);
          // found entries: one reservation for the wave (its classes share a signal)
          const int nf = !act ? 0 : (v.cls == kSingle ? 1 : (v.cls == kDouble ? 2 : 0));
          const int fs = wave_append_n(&c.st[s].found, nf);
          if (nf >= 1) push_found(c, s, d, fs, v.f, v.a);
          if (nf == 2) push_found(c, s, d, fs + 1, v.f2, v.a2);
          if (act) {
            if (v.cls == kMulti) {
              if (Ld >= 2 && dd + 1 <= d.max_levels && dd == d.col_dz) {
                // the children go to the deep resolution
                atomicOr(&dmask[g], (1ull << k) | (1ull << (k + nq)));
              } else if (Ld >= 2 && dd + 1 <= d.max_levels) {
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
        }
        __syncthreads();
      }
      nopen = n_nxt[g] < CAP ? n_nxt[g] : CAP;
      for (int k = gl; k < nopen; k += GS) open_cur[g][k] = open_nxt[g][k];
      __syncthreads();
    }
    if (valid && gl == 0 && deepest > 0) atomicMax(&c.st[s].levels, deepest);
    if (valid && gl == 0 && dmask[g] != 0) {
      c.A.deep_mask[d.multi_off + jslot] = dmask[g];
      c.A.deep_list[atomicAdd(c.A.deep_count, 1)] = make_int2(s, jslot);
    }
  }
}

// Deep subtree resolution from the column pass (Sect. 3.3): the level-0
// classes that the resolution above leaves open below depth Dz = col_dz.
// The class's spectrum values Z_k = X[c + k B0], k < L, come from one L-point
// DFT of its pre-twiddled column row,
//   Z_k = sum_{t < L} M_c(t) e^{-2 pi i (c + k B0) t / N},
// and the class vector of subclass cs = c + kappa B0 at depth dd (kappa <
// 2^dd, L_d = L / 2^dd) is the same bucket value as the column sums give,
//   Y_i = 1/N e^{2 pi i cs tau_i / N} sum_{j < L_d} Z_{kappa + j 2^dd} e^{2 pi i j tau_i / L_d},
// in L_d terms instead of 2^dd.  One work-group per deep class: the row into
// LDS and its FFT; then, round by round, every node of the subtrees below the
// open subclasses -- as many levels at once as kDeepNodes nodes allow -- has
// its vector formed and is classified, all in parallel; then the round's
// levels are walked from the subtrees' roots as the tree search does
// (children of multi-tons only), a level at a time with one thread per node:
// the nodes the level-by-level search would reach are the ones that count,
// with the same vectors and so the same decisions.  Their entries take one
// reservation in the found list per round.  Multi-tons on the last level of a
// round open the next round.
template <int NMAX, bool F32, bool WAVE>
__global__ __launch_bounds__(256) void k_col_deep(LaunchCtx c) {
  constexpr int CH = 2048 / NMAX;  // nodes whose vectors are staged at once (32 KiB)
  extern __shared__ float2 Zs[];   // L values (the largest L of the batch's deep signals)
  __shared__ double2 Ys[CH][NMAX];
  __shared__ int8_t dcls[kDeepNodes], reached[kDeepNodes];
  __shared__ int64_t df[kDeepNodes], df2[kDeepNodes];
  __shared__ double2 da[kDeepNodes], da2[kDeepNodes];
  __shared__ int open_cur[kColResolveCap], open_nxt[kColResolveCap];
  __shared__ int n_cur, n_nxt;
  __shared__ int nf_round, fs_round, deepest_round;  // the walk's entries, their first slot, its deepest level
  __shared__ int16_t fslot[kDeepNodes];               // a reached node's first entry in the round's reservation
  __shared__ float2 twd[kDeepTw];  // e^{-2 pi i m / L_t}, L_t = L / 2^(Dz + 1): every sum's twiddles
  // the deep list, the descriptors and the level-0 results are written by
  // earlier kernels: scalar loads
  const int ndeep = *cst(c.A.deep_count);
  const int tid = threadIdx.x;
  for (int e = blockIdx.x; e < ndeep; e += gridDim.x) {
    const uint64_t ent = cst((const uint64_t *)c.A.deep_list)[e];  // the int2 (signal, slot)
    const int s = (int)(uint32_t)ent, jslot = (int)(uint32_t)(ent >> 32);
    const SigDesc &d = *(const SigDesc *)&cst(c.desc)[s];
    const uint64_t N = (uint64_t)d.N;
    const int lgL = d.log2N - d.log2B0;
    const int L = 1 << lgL;
    const int n = d.n;
    const uint64_t cpar = (uint64_t)cst(c.A.multi_c[0])[d.multi_off + jslot];
    const float2 *M = c.A.jcol + d.jc_off + (int64_t)jslot * L;
    const double sref2 = cst(c.st)[s].sref2, nv = cst(c.st)[s].noise_var;
    const double invN = 1.0 / (double)N;
    // deepest depth a node is classified at (a multi-ton opens children while
    // its depth is below it)
    const int dmax = d.max_levels < lgL ? d.max_levels : lgL;
    __syncthreads();  // the previous class is done with Zs, the vectors' space and the lists
    // the L-point FFT's twiddles e^{-2 pi i m / L}, m < L / 2, held in the space
    // of the class vectors (not in use before the first round)
    float2 *twf = reinterpret_cast<float2 *>(&Ys[0][0]);
    static_assert(sizeof(Ys) >= sizeof(float2) * (kFftMax / 2), "FFT twiddles fit the vectors' space");
    const int lgLt = lgL - d.col_dz - 1;  // <= 7 (L <= 8192, Dz = 5)
    static_assert(kDeepTw <= 256, "one sum twiddle a thread");
    const float2 tdv = tid < (1 << lgLt) ? c.A.tw[tid << (kLog2FftMax - lgLt)] : make_float2(0.f, 0.f);
    // the row and the FFT's twiddles, 8 + 4 values a thread in flight at once
    // (256 threads)
    for (int t0 = 0; t0 < L; t0 += 8 * 256) {
      float2 mv[8], tv[4];
#pragma unroll
      for (int j = 0; j < 8; j++) {
        const int t = t0 + j * 256 + tid;
        mv[j] = t < L ? ldg(M + t) : make_float2(0.f, 0.f);
      }
#pragma unroll
      for (int j = 0; j < 4; j++) {
        const int m = (t0 >> 1) + j * 256 + tid;
        tv[j] = m < (L >> 1) ? c.A.tw[m << (kLog2FftMax - lgL)] : make_float2(0.f, 0.f);
      }
#pragma unroll
      for (int j = 0; j < 4; j++) {
        const int m = (t0 >> 1) + j * 256 + tid;
        if (m < (L >> 1)) twf[m] = tv[j];
      }
#pragma unroll
      for (int j = 0; j < 8; j++) {
        const int t = t0 + j * 256 + tid;
        if (t < L) Zs[bitrev((uint32_t)t, lgL)] = cmulf(mv[j], unit_nl((cpar * (uint64_t)t) & (N - 1), (uint64_t)N, d.log2N));
      }
    }
    if (tid < (1 << lgLt)) twd[tid] = tdv;
    if (tid == 0) {
      const uint64_t mask = cst(c.A.deep_mask)[d.multi_off + jslot];
      int m = 0;
      for (int b = 0; b < 64; b++)
        if ((mask >> b) & 1) open_cur[m++] = b;
      n_cur = m;
    }
    __syncthreads();
    fft_lds(Zs, lgL, twf, lgL);  // Zs[k] = Z_k
    __syncthreads();             // the vectors' space is free again
    int dd = d.col_dz + 1;     // depth of the open subclasses
    int nopen = n_cur;
    while (nopen > 0) {
      // levels dd .. dd + sl - 1 this round; node l of subtree o (l = 2^r - 1 + u,
      // u < 2^r) is subclass open_cur[o] + u 2^dd at depth dd + r
      int sl = 1;
      while (dd + sl <= dmax && nopen * ((2 << sl) - 1) <= kDeepNodes) sl++;
      const int per = (1 << sl) - 1;
      const int nn = nopen * per;
      for (int q0 = 0; q0 < nn; q0 += CH) {
        const int nq = nn - q0 < CH ? nn - q0 : CH;
        // the vectors: one thread per (node, measurement)
        for (int pe = tid; pe < nq * NMAX; pe += blockDim.x) {
          const int qi = pe / NMAX, i = pe - qi * NMAX;
          if (i >= n) continue;
          const int q = q0 + qi, o = q / per, l = q - o * per;
          const int r = 31 - __clz(l + 1), u = l + 1 - (1 << r);
          const int ddn = dd + r, lgLd = lgL - ddn, Ld = 1 << lgLd;
          const int kap = open_cur[o] + (u << dd);
          const uint64_t tau = tau_of(d, i);
          const int rr = (int)(tau & (uint64_t)(Ld - 1));
          double ax = 0.0, ay = 0.0;
          for (int j = 0; j < Ld; j++) {
            const float2 z = Zs[kap + (j << ddn)];
            // e^{+2 pi i j rr / L_d}: the conjugate of e^{-2 pi i (j rr mod L_d) / L_d}
            const float2 w = twd[((j * rr) & (Ld - 1)) << (lgLt - lgLd)];
            ax += (double)z.x * w.x + (double)z.y * w.y;
            ay += (double)z.y * w.x - (double)z.x * w.y;
          }
          const uint64_t cs = cpar + (uint64_t)kap * (uint64_t)d.B0;
          const double2 w = unit_d((cs * tau) & (N - 1), N, +1);
          Ys[qi][i] = make_double2((ax * w.x - ay * w.y) * invN, (ax * w.y + ay * w.x) * invN);
        }
        __syncthreads();
        {
          // every thread classifies (the noisy enumeration may run in teams of the wave's lanes)
          const int qi = tid < nq ? tid : 0;
          const bool act = tid < nq;
          const int q = q0 + qi, o = q / per, l = q - o * per;
          const int r = 31 - __clz(l + 1), u = l + 1 - (1 << r);
          const int ddn = dd + r;
          const int64_t cs = (int64_t)cpar + (int64_t)(open_cur[o] + (u << dd)) * d.B0;
          double2 Y[NMAX];
#pragma unroll
          for (int i = 0; i < NMAX; i++) Y[i] = act && i < n ? Ys[qi][i] : make_double2(0.0, 0.0);
          const Decision v = classify<NMAX, true, F32, WAVE>(Y, d, n, d.R, cs, d.B0 << ddn, sref2, nv, act);
          if (act) {
            dcls[q] = (int8_t)v.cls;
            df[q] = v.f;
            da[q] = v.a;
            df2[q] = v.f2;
            da2[q] = v.a2;
          }
        }
        __syncthreads();
      }
      // the walk, a level at a time: node l = 2^r - 1 + u of subtree o is
      // reached when it is a root or its parent was reached as a multi-ton
      // above the deepest level
      if (tid == 0) {
        n_nxt = 0;
        nf_round = 0;
        deepest_round = 0;
      }
      __syncthreads();
      for (int r = 0; r < sl; r++) {
        const int w = 1 << r, nl = nopen << r;
        for (int e = tid; e < nl; e += blockDim.x) {
          const int o = e >> r, u = e & (w - 1);
          const int q = o * per + w - 1 + u;
          bool reach = r == 0;
          if (r > 0) {
            const int pl = o * per + (w >> 1) - 1 + (u & ((w >> 1) - 1));
            reach = reached[pl] && dcls[pl] == kMulti && dd + r - 1 < dmax;
          }
          reached[q] = reach ? 1 : 0;
          if (!reach) continue;
          const int ddn = dd + r;
          atomicMax(&deepest_round, ddn);
          const int nfq = dcls[q] == kSingle ? 1 : dcls[q] == kDouble ? 2 : 0;
          if (nfq > 0) fslot[q] = (int16_t)atomicAdd(&nf_round, nfq);
          if (dcls[q] == kMulti) {
            if (ddn >= dmax) {
              atomicOr(&c.st[s].flags, 1);
            } else if (r == sl - 1) {
              // children on the next round's first level
              const int kap = open_cur[o] + (u << dd);
              const int at = atomicAdd(&n_nxt, 2);
              if (at + 2 <= kColResolveCap) {
                open_nxt[at] = kap;
                open_nxt[at + 1] = kap + (1 << ddn);
              } else {
                atomicOr(&c.st[s].flags, 1);
              }
            }
          }
        }
        __syncthreads();
      }
      // one reservation for the round's entries, then every reached node's
      if (tid == 0) {
        if (deepest_round > 0) atomicMax(&c.st[s].levels, deepest_round);
        fs_round = nf_round > 0 ? atomicAdd(&c.st[s].found, nf_round) : 0;
      }
      __syncthreads();
      for (int q = tid; q < nn; q += blockDim.x) {
        if (!reached[q]) continue;
        const int fq = fs_round + fslot[q];
        if (dcls[q] == kSingle || dcls[q] == kDouble) push_found(c, s, d, fq, df[q], da[q]);
        if (dcls[q] == kDouble) push_found(c, s, d, fq + 1, df2[q], da2[q]);
      }
      __syncthreads();
      nopen = n_nxt < kColResolveCap ? n_nxt : kColResolveCap;
      for (int k = tid; k < nopen; k += blockDim.x) open_cur[k] = open_nxt[k];
      dd += sl;
      __syncthreads();
    }
  }
}

}  // namespace

hipError_t launch_col_resolve(const LaunchCtx &c, int grid, hipStream_t s) {
  SFFT_LAUNCH_CLASSIFIER(k_col_resolve, c, dim3(grid), dim3(64), 0, s, c);
  return hipGetLastError();
}

hipError_t launch_col_deep(const LaunchCtx &c, int grid, hipStream_t s) {
  // its subclasses' candidate ranges are short (at most L / 2^(Dz + 1)): each
  // stays with its lane, and the form without the team enumeration serves
  SFFT_LAUNCH_CLASSIFIER_W(k_col_deep, c, false, dim3(grid), dim3(256), (size_t)c.deep_lds, s, c);
  return hipGetLastError();
}

}  // namespace sfft

