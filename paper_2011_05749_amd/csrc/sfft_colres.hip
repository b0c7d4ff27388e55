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
        {
          // every lane takes part (the noisy enumeration is shared by the wave)
          const bool act = gl < no;
          const int k = act ? open_cur[g][ch * GS + gl] : 0;
          const int64_t cs = (int64_t)cpar + (int64_t)k * d.B0;
          double2 Y[NMAX];
#pragma unroll
          for (int i = 0; i < NMAX; i++) Y[i] = act && i < n ? Ys[g][gl][i] : make_double2(0.0, 0.0);
          const Decision v = classify<NMAX, true, F32, WAVE>(Y, d, n, d.R, cs, Bd, sref2, nv, act);
          if (act) {
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
        }
        __syncthreads();
      }
      nopen = n_nxt[g] < CAP ? n_nxt[g] : CAP;
      for (int k = gl; k < nopen; k += GS) open_cur[g][k] = open_nxt[g][k];
      __syncthreads();
    }
  }
}


}  // namespace

hipError_t launch_col_resolve(const LaunchCtx &c, int grid, hipStream_t s) {
  SFFT_LAUNCH_CLASSIFIER(k_col_resolve, c, dim3(grid), dim3(64), 0, s, c);
  return hipGetLastError();
}

}  // namespace sfft

