// Streaming-bandwidth probe: the practical HBM ceiling the stencil kernels
// are measured against, taken with the same kind of code they are (plain
// HIP loads and stores, no library copy).  A copy kernel (read + write) and
// a read-only kernel (sum) sweep one large buffer with 16-byte accesses
// per lane in a grid-stride loop over every CU.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "../../include/ep.h"

namespace {

typedef float F4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_copy4(int64_t n4, const F4* __restrict__ x,
                                               F4* __restrict__ y) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n4;
       i += stride)
    y[i] = x[i];
}

__global__ __launch_bounds__(256) void k_read4(int64_t n4, const F4* __restrict__ x,
                                               float* __restrict__ out) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  F4 a = {0.0f, 0.0f, 0.0f, 0.0f};
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n4;
       i += stride)
    a += x[i];
  float s = a.x + a.y + a.z + a.w;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  // one value per wavefront keeps the sum live; the buffer holds zeros
  if ((threadIdx.x & 63) == 0)
    out[blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)] = s;
}

}  // namespace

extern "C" EP_API ep_status ep_stream_bandwidth(int64_t bytes, int32_t reps, double* copy_gbs,
                                                double* read_gbs) {
  if (bytes < (1 << 20) || reps < 1 || !copy_gbs || !read_gbs) return EP_ERR_ARG;
  const int64_t n4 = bytes / 16;
  const size_t nb = static_cast<size_t>(n4) * 16;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return EP_ERR_HIP;
  const int grid = cus * 8;   // 8 blocks of 256 threads per CU
  void *x = nullptr, *y = nullptr, *o = nullptr;
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ep_status rc = EP_OK;
  if (hipMalloc(&x, nb) != hipSuccess || hipMalloc(&y, nb) != hipSuccess ||
      hipMalloc(&o, static_cast<size_t>(grid) * 4 * sizeof(float)) != hipSuccess) {
    (void)hipGetLastError();
    rc = EP_ERR_OOM;
  }
  if (rc == EP_OK &&
      (hipStreamCreate(&s) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
       hipEventCreate(&e1) != hipSuccess || hipMemsetAsync(x, 0, nb, s) != hipSuccess ||
       hipMemsetAsync(y, 0, nb, s) != hipSuccess))
    rc = EP_ERR_HIP;
  auto timed = [&](auto launch, double moved, double* out) {
    launch();   // warm-up
    float best = 0.0f;
    for (int r = 0; r < reps && rc == EP_OK; ++r) {
      float ms = 0.0f;
      if (hipEventRecord(e0, s) != hipSuccess) { rc = EP_ERR_HIP; break; }
      launch();
      if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        rc = EP_ERR_HIP;
        break;
      }
      if (r == 0 || ms < best) best = ms;
    }
    if (rc == EP_OK) *out = moved / (best * 1e-3) / 1e9;
  };
  if (rc == EP_OK) {
    timed([&] { k_copy4<<<grid, 256, 0, s>>>(n4, static_cast<const F4*>(x), static_cast<F4*>(y)); },
          2.0 * static_cast<double>(nb), copy_gbs);
    timed([&] { k_read4<<<grid, 256, 0, s>>>(n4, static_cast<const F4*>(x), static_cast<float*>(o)); },
          static_cast<double>(nb), read_gbs);
    if (rc == EP_OK && hipGetLastError() != hipSuccess) rc = EP_ERR_HIP;
  }
  if (s) (void)hipStreamSynchronize(s);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (s) (void)hipStreamDestroy(s);
  if (x) (void)hipFree(x);
  if (y) (void)hipFree(y);
  if (o) (void)hipFree(o);
  return rc;
}
