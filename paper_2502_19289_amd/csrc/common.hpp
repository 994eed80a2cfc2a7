// Shared device-side types of the cluster-TEBD library.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace ctebd {

// A size that is fixed when the work is queued or read from device memory when
// the kernel runs (ranks chosen by a truncation earlier in the same step):
// value = mult * (*ptr) if ptr else mult.
struct Dim {
  int mult;
  const int* ptr;
};

__device__ __forceinline__ int dim_value(const Dim& d) { return d.ptr ? d.mult * (*d.ptr) : d.mult; }

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
