// Device-side helpers shared by the HIP translation units (not for host code).
#pragma once
#include <hip/hip_runtime.h>

namespace hdg {

// Workgroup barrier that orders LDS accesses only: global loads issued before it
// (such as prefetched factors) stay in flight across it, where __syncthreads()
// would wait for them.  For kernels whose waves never read global memory
// written by another wave of the workgroup.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Raw buffer loads: a descriptor for one array (bounds-checked by the hardware:
// reads past num_bytes return 0), a per-lane byte offset held in one register
// for all loads and a wave-uniform byte offset per load, so a run of loads with
// different uniform offsets needs no address registers of its own.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc(const void* base, int num_bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, num_bytes, 0x00020000);
}
template <typename T>
__device__ __forceinline__ T buffer_load(__amdgpu_buffer_rsrc_t rs, int lane_bytes, int uniform_bytes);
template <>
__device__ __forceinline__ double buffer_load<double>(__amdgpu_buffer_rsrc_t rs, int lane_bytes, int uniform_bytes) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, lane_bytes, uniform_bytes, 0));
}
template <>
__device__ __forceinline__ float buffer_load<float>(__amdgpu_buffer_rsrc_t rs, int lane_bytes, int uniform_bytes) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, lane_bytes, uniform_bytes, 0));
}

}  // namespace hdg
