// HBM copy kernels for measuring the bandwidth the chip sustains with two
// access patterns, the ceilings against which the operator's roofline
// fraction is read (HBM3E, 8 TB/s by specification):
//   pattern 0: all workgroups sweep one window of the buffer together
//     (grid-stride, four 16-byte loads in flight per thread, nontemporal
//     loads and stores) -- the pattern a stream kernel is at its best with;
//   pattern 1: workgroup b copies its own contiguous part of the buffer
//     (block-contiguous), the pattern of the fused operator, whose
//     workgroups each stream their own chunk of time slices.
#include <hip/hip_runtime.h>

#include "../../include/holstein_hmc.h"
#include "fph_internal.h"

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kNT = 512;
constexpr int kU = 4;

__global__ void __launch_bounds__(kNT)
k_copy_window(long n4, const v4f* __restrict__ in, v4f* __restrict__ out) {
  const long stride = (long)gridDim.x * kNT;
  long i = blockIdx.x * (long)kNT + threadIdx.x;
  for (; i + (kU - 1) * stride < n4; i += kU * stride) {
    v4f v[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) v[u] = __builtin_nontemporal_load(in + i + u * stride);
#pragma unroll
    for (int u = 0; u < kU; ++u) __builtin_nontemporal_store(v[u], out + i + u * stride);
  }
  for (; i < n4; i += stride) __builtin_nontemporal_store(__builtin_nontemporal_load(in + i), out + i);
}

__global__ void __launch_bounds__(kNT)
k_copy_blocks(long n4, long per, const v4f* __restrict__ in, v4f* __restrict__ out) {
  const long start = blockIdx.x * per;
  const long end = (start + per < n4) ? start + per : n4;
  long i = start + threadIdx.x;
  for (; i + (kU - 1) * kNT < end; i += kU * kNT) {
    v4f v[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) v[u] = in[i + u * kNT];
#pragma unroll
    for (int u = 0; u < kU; ++u) __builtin_nontemporal_store(v[u], out + i + u * kNT);
  }
  for (; i < end; i += kNT) __builtin_nontemporal_store(in[i], out + i);
}

}  // namespace

extern "C" int fph_hbm_copy(const void* src_dev, void* dst_dev, int64_t bytes, int32_t nblocks,
                            int32_t pattern, void* stream) {
  if (src_dev == nullptr || dst_dev == nullptr) return FPH_E_NULL;
  if ((reinterpret_cast<uintptr_t>(src_dev) | reinterpret_cast<uintptr_t>(dst_dev)) & 15)
    return FPH_E_ALIGN;
  if (bytes < 0 || bytes % 16 != 0 || (pattern != 0 && pattern != 1) || nblocks > (1 << 20))
    return FPH_E_ARG;
  if (bytes == 0) return FPH_OK;
  int dev = 0, ncu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return fph::record_hip_error(e);
  const long n4 = bytes / 16;
  const int g = nblocks > 0 ? nblocks : ncu;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (pattern == 0) {
    hipLaunchKernelGGL(k_copy_window, dim3(g), dim3(kNT), 0, s, n4,
                       static_cast<const v4f*>(src_dev), static_cast<v4f*>(dst_dev));
  } else {
    const long per = (n4 + g - 1) / g;
    hipLaunchKernelGGL(k_copy_blocks, dim3(g), dim3(kNT), 0, s, n4, per,
                       static_cast<const v4f*>(src_dev), static_cast<v4f*>(dst_dev));
  }
  e = hipGetLastError();
  return e == hipSuccess ? FPH_OK : fph::record_hip_error(e);
}
