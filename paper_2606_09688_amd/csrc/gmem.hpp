// Device-side access to global memory through explicitly global pointers.
//
// A pointer that a kernel reads from memory (a descriptor array, the argument
// structs of a launch over many problems, a per-call pointer table) has an
// unknown address space for the compiler, which then emits flat loads and
// stores.  On CDNA a flat access counts against both the vector-memory and the
// LDS/scalar wait counters, so a wait for an LDS read also waits for every
// flat load in flight (a register prefetch of the next tile, say).  Casting
// such pointers to the global address space keeps them global instructions.
#pragma once

#include <hip/hip_runtime.h>

namespace sg {

// element i of a global array, loaded / stored through a global-memory
// pointer (for pointers read from global memory, e.g. inside a descriptor)
template <class T>
__device__ __forceinline__ T gld(const T *p, long long i) {
  return ((const __attribute__((address_space(1))) T *)p)[i];
}
template <class T>
__device__ __forceinline__ void gst(T *p, long long i, T v) {
  ((__attribute__((address_space(1))) T *)p)[i] = v;
}

// typed global-memory pointers, for locals that hold such a pointer
template <class T>
using gptr = __attribute__((address_space(1))) T *;
template <class T>
__device__ __forceinline__ gptr<T> to_g(T *p) {
  return (gptr<T>)p;
}

// element i of a read-only descriptor array, read through the constant
// address space: uniform reads become scalar loads, and the pointers read
// from it are known to be global
template <class T>
__device__ __forceinline__ const T &cref(const T *p, long long i) {
  return *(const T *)((const __attribute__((address_space(4))) T *)p + i);
}

}  // namespace sg
