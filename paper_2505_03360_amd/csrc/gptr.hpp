// Device pointer helper shared by the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace bzk {

// Global-address-space pointer whose value the compiler cannot see through:
// per-pass load bases stay in the pass loop (the compiler would otherwise
// hoist every base + k*stride address out of it, 2 registers each), and the
// loads remain global (not flat) loads with immediate offsets.
#if defined(__HIP_DEVICE_COMPILE__)
template <typename T>
using gptr = const __attribute__((address_space(1))) T*;
#else
template <typename T>
using gptr = const T*;
#endif
template <typename T>
__device__ __forceinline__ gptr<T> opaque_global(const T* p) {
  asm volatile("" : "+v"(p));
  return (gptr<T>)p;
}

}  // namespace bzk
