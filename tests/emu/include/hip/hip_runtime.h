// CPU stand-in for the few HIP device features the sliCQ kernels use, so that
// the unmodified kernel header can be compiled by g++ and run with one OS
// thread per GPU lane (std::barrier for __syncthreads). Test harness only:
// never part of the product library.
#pragma once
#include <atomic>
#include <barrier>
#include <cmath>
#include <cstdint>
#include <cstdlib>

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__

struct int2 {
  int x, y;
};

struct dim3 {
  unsigned x, y, z;
  dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};

extern thread_local dim3 threadIdx, blockIdx, blockDim, gridDim;
extern thread_local std::barrier<>* emu_barrier;

inline void __syncthreads() { emu_barrier->arrive_and_wait(); }

// The kernels read the first lane only of values that are equal on every lane
// of a wave (a wave's base thread index), so each lane's own value is the result.
inline int __builtin_amdgcn_readfirstlane(int x) { return x; }

template <class T>
inline T unsafeAtomicAdd(T* p, T v) {
  return std::atomic_ref<T>(*p).fetch_add(v);
}

// sin(pi x) and cos(pi x) (HIP's sincospi), from the C library.
inline void sincospi(double x, double* s, double* c) {
  *s = std::sin(M_PI * x);
  *c = std::cos(M_PI * x);
}
