// Global-memory pointer types for device code.  Operand pointers that a kernel reads
// from memory (pointer arrays, grouped-launch tables) are generic ("flat") pointers to
// the compiler; flat loads also count against the LDS wait counter, so an LDS wait
// would then also wait for every global load in flight.  Typed global, they compile
// to global_load / global_store.
#pragma once

#include <hip/hip_runtime.h>

#define PHIKS_GLOBAL __attribute__((address_space(1)))

namespace phiks {
template <class T> __device__ __forceinline__ PHIKS_GLOBAL T* gptr(T* p) {
  return (PHIKS_GLOBAL T*)p;
}
}  // namespace phiks
