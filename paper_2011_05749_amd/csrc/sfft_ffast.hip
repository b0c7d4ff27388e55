// sfft_ffast.hip -- FFAST decoder for co-prime N: stage DFTs and the whole
// peeling decoder (Sect. 3.2, Subproblem 3, Eq. 20) in one work-group per
// signal.
#include "sfft_device.h"

namespace sfft {

namespace {

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

}  // namespace

hipError_t launch_ffast(const LaunchCtx &c, hipStream_t s) {
  static bool configured = false;
  if (!configured) {
    // dynamic LDS above 64 KiB: declare the gfx950 maximum once
    const int big = 160 * 1024;
    (void)hipFuncSetAttribute((const void *)k_ffast<8>, hipFuncAttributeMaxDynamicSharedMemorySize, big);
    (void)hipFuncSetAttribute((const void *)k_ffast<16>, hipFuncAttributeMaxDynamicSharedMemorySize, big);
    (void)hipFuncSetAttribute((const void *)k_ffast<64>, hipFuncAttributeMaxDynamicSharedMemorySize, big);
    (void)hipGetLastError();
    configured = true;
  }
  const int nm = nmax_bucket(c.nmax);
    const int grid = c.nffast < 4096 ? c.nffast : 4096;
    const size_t lds = sizeof(float2) * (kFftMax + kDirectMax) + 6 * kMaxFfastBuckets;
    if (nm == 8) hipLaunchKernelGGL(k_ffast<8>, dim3(grid), dim3(kThreads), lds, s, c);
    else if (nm == 16) hipLaunchKernelGGL(k_ffast<16>, dim3(grid), dim3(kThreads), lds, s, c);
    else hipLaunchKernelGGL(k_ffast<64>, dim3(grid), dim3(kThreads), lds, s, c);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  return hipSuccess;
}

}  // namespace sfft
