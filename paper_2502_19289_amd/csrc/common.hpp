// Shared device-side types of the cluster-TEBD library.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace ctebd {

// Loads and stores through pointers taken from descriptors in device memory.
// The compiler cannot tell that such a pointer addresses global memory, so a
// plain access becomes a flat one, which also counts against the counter of
// outstanding LDS and scalar operations: every wait for an LDS read then waits
// for the flat loads in flight too (a prefetch issued before a slice's
// products would be waited for at its first LDS read).  These helpers access
// the same address through the global segment, which is valid because a
// descriptor pointer never addresses LDS or private memory (the two other
// apertures a flat access covers).
#define CTEBD_GLOBAL __attribute__((address_space(1)))
template <typename T>
struct gl_repr {
  using type = T;
};
template <>
struct gl_repr<float2> {
  using type = float __attribute__((ext_vector_type(2)));
};
template <>
struct gl_repr<double2> {
  using type = double __attribute__((ext_vector_type(2)));
};
template <typename T>
__device__ __forceinline__ T gld(const T* p) {
  using R = typename gl_repr<T>::type;
  const R v = *(const CTEBD_GLOBAL R*)(const void*)p;
  if constexpr (!__is_same(R, T)) {
    T r;
    r.x = v.x;
    r.y = v.y;
    return r;
  } else {
    return v;
  }
}
template <typename T>
__device__ __forceinline__ void gst(T* p, T x) {
  using R = typename gl_repr<T>::type;
  if constexpr (!__is_same(R, T)) {
    R v;
    v.x = x.x;
    v.y = x.y;
    *(CTEBD_GLOBAL R*)(void*)p = v;
  } else {
    *(CTEBD_GLOBAL T*)(void*)p = x;
  }
}

// The same pointer typed as global memory, for kernels that index plain
// scalar arrays of a descriptor.
template <typename T>
__device__ __forceinline__ const CTEBD_GLOBAL T* gp(const T* p) {
  return (const CTEBD_GLOBAL T*)p;
}
template <typename T>
__device__ __forceinline__ CTEBD_GLOBAL T* gp(T* p) {
  return (CTEBD_GLOBAL T*)p;
}

// A size that is fixed when the work is queued or read from device memory when
// the kernel runs (ranks chosen by a truncation earlier in the same step):
// value = mult * (*ptr) if ptr else mult.
struct Dim {
  int mult;
  const int* ptr;
};

__device__ __forceinline__ int dim_value(const Dim& d) { return d.ptr ? d.mult * gld(d.ptr) : d.mult; }

template <typename T>
struct cpx_of;
template <>
struct cpx_of<float> {
  using type = float2;
};
template <>
struct cpx_of<double> {
  using type = double2;
};

template <typename C>
struct real_of;
template <>
struct real_of<float2> {
  using type = float;
};
template <>
struct real_of<double2> {
  using type = double;
};

__device__ __forceinline__ double2 to_d2(float2 v) { return make_double2(v.x, v.y); }
__device__ __forceinline__ double2 to_d2(double2 v) { return v; }
template <typename C>
__device__ __forceinline__ C from_d2(double2 v);
template <>
__device__ __forceinline__ float2 from_d2<float2>(double2 v) {
  return make_float2((float)v.x, (float)v.y);
}
template <>
__device__ __forceinline__ double2 from_d2<double2>(double2 v) {
  return v;
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cmulc(double2 a, double2 b) {  // conj(a) * b
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }

// Finds the problem owning flat block index `blk` given exclusive prefix sums
// of per-problem block counts (base[0] = 0, base[nprob] = total).
__device__ __forceinline__ int find_problem(const int* base, int nprob, int blk) {
  int lo = 0, hi = nprob - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (base[mid] <= blk)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

}  // namespace ctebd
