// Microbenchmarks of the rates that the kernels' rooflines are set against:
// the vector FMA rate in FP32 (non-packed, as every kernel here is built)
// and FP64, the transcendental rate (v_exp_f32), the LDS FP64 atomic rate,
// and random 16-byte gathers from a buffer of a given size (the map
// interpolation's access: a buffer that fits the L2 of one XCD, or one the
// size of a map set, served by the MALL).  Diagnostics only: the docking
// path never calls them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "api_internal.h"

namespace ad {
namespace {

constexpr int kMbIters = 4096;   // dependent steps per chain
constexpr int kMbChains = 8;     // independent chains per lane
constexpr int kMbBlock = 256;

// a result the compiler cannot prove unused
template <typename T>
__device__ __forceinline__ void keep(T s, T *out) {
  if (s == (T)-1234.5) out[blockIdx.x] = s;
}

template <typename T>
__global__ __launch_bounds__(kMbBlock) void k_mb_fma(T *out, T seed) {
  T a[kMbChains];
#pragma unroll
  for (int k = 0; k < kMbChains; ++k) a[k] = seed + (T)(threadIdx.x & 7) * (T)0.001 + (T)k;
  const T m = (T)0.999, c = (T)0.001;
  for (int it = 0; it < kMbIters; ++it) {
#pragma unroll
    for (int k = 0; k < kMbChains; ++k) a[k] = fma(a[k], m, c);
  }
  T s = 0;
#pragma unroll
  for (int k = 0; k < kMbChains; ++k) s += a[k];
  keep(s, out);
}

__global__ __launch_bounds__(kMbBlock) void k_mb_exp(float *out, float seed) {
  float a[kMbChains];
#pragma unroll
  for (int k = 0; k < kMbChains; ++k) a[k] = seed + (float)(threadIdx.x & 7) * 0.001f + 0.1f * (float)k;
  for (int it = 0; it < kMbIters; ++it) {
#pragma unroll
    for (int k = 0; k < kMbChains; ++k) a[k] = __builtin_amdgcn_exp2f(-a[k]);   // stays in (0.5, 1]
  }
  float s = 0.0f;
#pragma unroll
  for (int k = 0; k < kMbChains; ++k) s += a[k];
  keep(s, out);
}

// one-wavefront work-groups, two independent ds_add_f64 streams on
// consecutive doubles (the force accumulators' conflict-free pattern)
constexpr int kMbLdsIters = 2048;
__global__ __launch_bounds__(64) void k_mb_lds(double *out) {
  __shared__ double g[256];
  for (int i = threadIdx.x; i < 256; i += 64) g[i] = 0.0;
  __syncthreads();
  const double v = 1.0 + threadIdx.x;
  for (int it = 0; it < kMbLdsIters; ++it) {
    atomicAdd(&g[threadIdx.x], v);
    atomicAdd(&g[128 + threadIdx.x], v);
  }
  __syncthreads();
  if (threadIdx.x == 0 && g[0] == -1.0) out[blockIdx.x] = g[1];
}

// kMbGathers independent 16-byte loads per lane at hashed record indices
// (n_mask + 1 records, a power of two)
constexpr int kMbGathers = 64;
__global__ __launch_bounds__(kMbBlock) void k_mb_gather(const float4 *__restrict__ buf, uint32_t n_mask, float *out) {
  const uint32_t tid = blockIdx.x * kMbBlock + threadIdx.x;
  float s = 0.0f;
#pragma unroll 8
  for (int k = 0; k < kMbGathers; ++k) {
    uint32_t h = tid * 0x9E3779B1u + (uint32_t)k * 0x85EBCA77u;
    h ^= h >> 15;
    h *= 0x2C1B3C6Du;
    h ^= h >> 12;
    const float4 r = buf[h & n_mask];
    s += (r.x + r.y) + (r.z + r.w);
  }
  keep(s, out);
}

}  // namespace
}  // namespace ad

using namespace ad;

extern "C" int ad_microbench(ad_ctx *c, int kind, size_t bytes, double *result) {
  if (!c || !result) return c ? c->fail(AD_E_INVALID, "null result") : AD_E_INVALID;
  if (kind < 0 || kind > 4) return c->fail(AD_E_INVALID, "microbenchmark kind must be 0..4");
  if (kind == 4 && (bytes < 4096 || bytes > ((size_t)1 << 34)))
    return c->fail(AD_E_INVALID, "gather buffer must be 4 KiB .. 16 GiB");
  hipSetDevice(c->device);
  int n_cu = 0;
  if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess || n_cu <= 0)
    return c->fail(AD_E_HIP, "cannot read the compute-unit count");
  const unsigned blocks = (unsigned)n_cu * 16;
  void *out = nullptr, *buf = nullptr;
  // one slot per work-group of the largest grid (blocks * 4)
  if (hipMalloc(&out, (size_t)blocks * 4 * sizeof(double)) != hipSuccess) return c->fail(AD_E_OOM, "microbenchmark");
  // gather records: the largest power of two that fits `bytes`
  uint32_t n_rec = 1;
  while ((size_t)n_rec * 2 * 16 <= bytes && n_rec < 0x80000000u) n_rec *= 2;
  if (kind == 4) {
    if (hipMalloc(&buf, (size_t)n_rec * 16) != hipSuccess) {
      hipFree(out);
      return c->fail(AD_E_OOM, "microbenchmark gather buffer");
    }
  }
  hipError_t err = buf ? hipMemsetAsync(buf, 0, (size_t)n_rec * 16, c->stream) : hipSuccess;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (err == hipSuccess) err = hipEventCreate(&e0);
  if (err == hipSuccess) err = hipEventCreate(&e1);
  float best = INFINITY;
  for (int rep = 0; rep < 4 && err == hipSuccess; ++rep) {   // the first is a warm-up
    err = hipEventRecord(e0, c->stream);
    if (err != hipSuccess) break;
    switch (kind) {
      case 0: hipLaunchKernelGGL(k_mb_fma<float>, dim3(blocks), dim3(kMbBlock), 0, c->stream, (float *)out, 0.5f); break;
      case 1: hipLaunchKernelGGL(k_mb_fma<double>, dim3(blocks), dim3(kMbBlock), 0, c->stream, (double *)out, 0.5); break;
      case 2: hipLaunchKernelGGL(k_mb_exp, dim3(blocks), dim3(kMbBlock), 0, c->stream, (float *)out, 0.5f); break;
      case 3: hipLaunchKernelGGL(k_mb_lds, dim3(blocks * 4), dim3(64), 0, c->stream, (double *)out); break;
      default:
        hipLaunchKernelGGL(k_mb_gather, dim3(blocks * 4), dim3(kMbBlock), 0, c->stream, (const float4 *)buf, n_rec - 1,
                           (float *)out);
    }
    err = hipGetLastError();
    if (err == hipSuccess) err = hipEventRecord(e1, c->stream);
    if (err == hipSuccess) err = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
    if (rep > 0) best = std::min(best, ms);
  }
  if (e0) hipEventDestroy(e0);
  if (e1) hipEventDestroy(e1);
  hipFree(out);
  if (buf) hipFree(buf);
  if (err != hipSuccess) return c->hip_fail(err, "microbenchmark");
  const double s = best * 1e-3;
  const double lanes = (double)blocks * kMbBlock;
  switch (kind) {
    case 0:
    case 1: *result = lanes * kMbChains * kMbIters * 2.0 / s; break;   // FLOP/s
    case 2: *result = lanes * kMbChains * kMbIters / s; break;         // exp2 per s
    case 3: *result = (double)blocks * 4 * 64 * 2.0 * kMbLdsIters / s; break;   // lane atomics per s
    default: *result = (double)blocks * 4 * kMbBlock * kMbGathers * 16.0 / s;   // bytes per s
  }
  return AD_OK;
}
