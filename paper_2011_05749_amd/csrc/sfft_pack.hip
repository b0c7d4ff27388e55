// sfft_pack.hip -- packed FP16 form of a complex64 signal (sample_format =
// SFFT_SAMPLES_F16): a power-of-two scale from the largest component
// magnitude, then every component divided by it and rounded to binary16.
#include <hip/hip_fp16.h>

#include "sfft_internal.h"

namespace sfft {

namespace {

// header words: [0] scale (float), [1] largest |component| (float bits, as an
// unsigned for atomicMax: non-negative floats order as their bit patterns)
__global__ void k_pack_clear(unsigned *hdr) {
  if (threadIdx.x == 0) hdr[1] = 0u;
}

__global__ __launch_bounds__(256) void k_pack_absmax(const float2 *__restrict__ x, int64_t N, unsigned *hdr) {
  __shared__ float red[4];
  float m = 0.0f;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < N; i += (int64_t)gridDim.x * 256) {
    const float2 v = x[i];
    m = fmaxf(m, fmaxf(fabsf(v.x), fabsf(v.y)));
  }
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) atomicMax(hdr + 1, __float_as_uint(fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]))));
}

// s = 2^(e - 15) with 2^(e-1) <= m < 2^e: every |component| / s < 2^15
__device__ __forceinline__ float pack_scale(unsigned mbits) {
  const float m = __uint_as_float(mbits);
  if (!(m > 0.0f)) return 1.0f;
  int e = 0;
  (void)frexpf(m, &e);  // m = f 2^e, f in [0.5, 1)
  return ldexpf(1.0f, e - 15);
}

__global__ __launch_bounds__(256) void k_pack_convert(const float2 *__restrict__ x, int64_t N, unsigned *hdr) {
  const float s = pack_scale(hdr[1]);
  const float inv = 1.0f / s;  // a power of two: exact
  unsigned *out = hdr + SFFT_F16_HEADER_BYTES / 4;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < N; i += (int64_t)gridDim.x * 256) {
    const float2 v = x[i];
    const unsigned short re = __half_as_ushort(__float2half_rn(v.x * inv));
    const unsigned short im = __half_as_ushort(__float2half_rn(v.y * inv));
    out[i] = (unsigned)re | ((unsigned)im << 16);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    hdr[0] = __float_as_uint(s);
    hdr[2] = 0u;
    hdr[3] = 0u;
  }
}

bool device_ptr(const void *p) {
  hipPointerAttribute_t a;
  if (!p || hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

}  // namespace

}  // namespace sfft

extern "C" int32_t sfft_pack_fp16(const void *x, int64_t N, void *out, void *stream) {
  using namespace sfft;
  if (N < 1 || N > (int64_t(1) << 30) || !device_ptr(x) || !device_ptr(out)) return SFFT_EINVAL;
  const hipStream_t s = (hipStream_t)stream;
  unsigned *hdr = (unsigned *)out;
  const int64_t blocks = (N + 255) / 256;
  const int g1 = (int)(blocks < 1024 ? blocks : 1024), g2 = (int)(blocks < 8192 ? blocks : 8192);
  hipLaunchKernelGGL(k_pack_clear, dim3(1), dim3(64), 0, s, hdr);
  hipLaunchKernelGGL(k_pack_absmax, dim3(g1), dim3(256), 0, s, (const float2 *)x, N, hdr);
  hipLaunchKernelGGL(k_pack_convert, dim3(g2), dim3(256), 0, s, (const float2 *)x, N, hdr);
  return hipGetLastError() == hipSuccess ? SFFT_OK : SFFT_EDEVICE;
}
