// 16x16x4 matrix-core (MFMA) building block shared by the complex GEMMs.
//
// Operand layout of v_mfma_{f32,f64}_16x16x4 on a 64-lane wavefront:
//   A (16x4):  lane holds A[lane % 16][lane / 16]
//   B (4x16):  lane holds B[lane / 16][lane % 16]
//   D (16x16): accumulator element r of a lane is D[row(lane, r)][lane % 16],
//              row = 4*(lane/16) + r for f32 but 4*r + lane/16 for f64
//              (both measured on gfx950)
// A complex product is split into real products sharing the fragments: four
// (CAcc: Dre += Ar Br - Ai Bi, Dim += Ar Bi + Ai Br; 8 real flops per complex
// MAC) or three (CAcc3, Gauss's form, below).
#pragma once
#include <hip/hip_runtime.h>

namespace ctebd {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T>
struct Mfma;

template <>
struct Mfma<float> {
  using acc_t = f32x4;
  __device__ __forceinline__ static acc_t zero() { return acc_t{0.f, 0.f, 0.f, 0.f}; }
  __device__ __forceinline__ static acc_t mac(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ __forceinline__ static int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

template <>
struct Mfma<double> {
  using acc_t = f64x4;
  __device__ __forceinline__ static acc_t zero() { return acc_t{0.0, 0.0, 0.0, 0.0}; }
  __device__ __forceinline__ static acc_t mac(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ __forceinline__ static int row(int lane, int r) { return 4 * r + (lane >> 4); }
};

// One complex 16x16 accumulator block.
template <typename T>
struct CAcc {
  typename Mfma<T>::acc_t re, im;
  __device__ __forceinline__ void clear() {
    re = Mfma<T>::zero();
    im = Mfma<T>::zero();
  }
  // this += a * b for one k-slice of 4 (a, b: this lane's complex fragments)
  __device__ __forceinline__ void mac(T ar, T ai, T br, T bi) {
    re = Mfma<T>::mac(ar, br, re);
    re = Mfma<T>::mac(-ai, bi, re);
    im = Mfma<T>::mac(ar, bi, im);
    im = Mfma<T>::mac(ai, br, im);
  }
};

// Complex 16x16 accumulator block with three real products per complex
// product (Gauss): P1 = sum ar br, P2 = sum ai bi, P3 = sum (ar + ai)(br + bi),
// re = P1 - P2, im = P3 - P1 - P2.  Used by all complex GEMMs (FP32 and
// FP64: contractions, Gram matrix, panel update, back-transformation): a
// quarter fewer matrix-core products; the error of an entry stays of order
// u sum |a| |b| (at most about twice the four-product bound on the
// imaginary part).
template <typename T>
struct CAcc3 {
  typename Mfma<T>::acc_t p1, p2, p3;
  __device__ __forceinline__ void clear() { p1 = p2 = p3 = Mfma<T>::zero(); }
  __device__ __forceinline__ void mac(T ar, T ai, T br, T bi) {
    p1 = Mfma<T>::mac(ar, br, p1);
    p2 = Mfma<T>::mac(ai, bi, p2);
    p3 = Mfma<T>::mac(ar + ai, br + bi, p3);
  }
};
template <typename T>
__device__ __forceinline__ T acc_re(const CAcc<T>& a, int r) { return a.re[r]; }
template <typename T>
__device__ __forceinline__ T acc_im(const CAcc<T>& a, int r) { return a.im[r]; }
template <typename T>
__device__ __forceinline__ T acc_re(const CAcc3<T>& a, int r) { return a.p1[r] - a.p2[r]; }
template <typename T>
__device__ __forceinline__ T acc_im(const CAcc3<T>& a, int r) { return a.p3[r] - a.p1[r] - a.p2[r]; }

}  // namespace ctebd
