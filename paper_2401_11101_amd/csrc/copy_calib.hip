// Streaming copy kernels of known size, one per per-lane access width
// (4, 8, 16 bytes).  They calibrate the HBM byte counters (FETCH_SIZE,
// WRITE_SIZE) against a plain copy whose traffic is known exactly: the
// counters' request accounting depends on how a wave's accesses coalesce,
// so each width gets its own factor.  Not part of the reconstruction path.
#include <hip/hip_runtime.h>

#include <cstddef>

namespace {

template <typename T>
__global__ __launch_bounds__(256) void k_copy(const T* __restrict__ src, T* __restrict__ dst,
                                              size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

template <typename T>
int launch(const void* src, void* dst, size_t bytes, hipStream_t s) {
  const size_t n = bytes / sizeof(T);
  const unsigned blocks = 256 * 8 * 4;  // 8 waves' worth of blocks per CU, grid-stride beyond
  hipLaunchKernelGGL(k_copy<T>, dim3(blocks), dim3(256), 0, s, static_cast<const T*>(src),
                     static_cast<T*>(dst), n);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

}  // namespace

// Copies `bytes` (a multiple of `width`) from src to dst, both device
// pointers, on `stream`, with `width` = 4, 8 or 16 bytes per lane access.
// Returns 0, -1 for a bad width / size, -4 for a launch error.
extern "C" int lamino_calib_copy(const void* src, void* dst, size_t bytes, int width,
                                 void* stream) {
  if (!src || !dst || (width != 4 && width != 8 && width != 16) || bytes % width) return -1;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (width == 4) return launch<float>(src, dst, bytes, s);
  if (width == 8) return launch<float2>(src, dst, bytes, s);
  return launch<float4>(src, dst, bytes, s);
}
