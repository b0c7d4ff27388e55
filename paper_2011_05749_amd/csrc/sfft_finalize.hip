// sfft_finalize.hip -- top-K by magnitude, ascending index, padding.
#include "sfft_device.h"

namespace sfft {

namespace {

// Top-K by magnitude (ties: lower index), then ascending index; padding.
__global__ __launch_bounds__(1024) void k_finalize(LaunchCtx c) {
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

}  // namespace

hipError_t launch_finalize(const LaunchCtx &c, hipStream_t s) {
  static bool configured = false;
  if (!configured) {
    (void)hipFuncSetAttribute((const void *)k_finalize, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    (void)hipGetLastError();
    configured = true;
  }
  const int grid = c.nsig < 4096 ? c.nsig : 4096;
  const size_t lds = (sizeof(uint64_t) + sizeof(int32_t)) * (size_t)c.max_found_cap;
  // a signal a work-group; batches that give each CU at most one signal sort
  // with 1024 threads a signal (every loop strides by the work-group size)
  const int nt = c.nsig <= 256 ? 1024 : kThreads;
  hipLaunchKernelGGL(k_finalize, dim3(grid), dim3(nt), lds, s, c);
  return hipGetLastError();
}

}  // namespace sfft
