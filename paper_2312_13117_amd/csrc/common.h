// Shared device helpers of the gfx950 kernels: complex arithmetic on interleaved
// (re, im) pairs, the 16x16x4 matrix-core wrappers, and launch checks.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define NEP_DEV __device__ __forceinline__

// ---------------------------------------------------------------- complex pairs
template <typename T> struct V2;
template <> struct V2<double> { typedef double2 t; };
template <> struct V2<float> { typedef float2 t; };
template <typename T> using c2 = typename V2<T>::t;

template <typename T> NEP_DEV c2<T> cmk(T x, T y) { c2<T> r; r.x = x; r.y = y; return r; }
template <typename T> NEP_DEV c2<T> czero() { return cmk<T>(T(0), T(0)); }
template <typename T> NEP_DEV c2<T> cadd(c2<T> a, c2<T> b) { return cmk<T>(a.x + b.x, a.y + b.y); }
template <typename T> NEP_DEV c2<T> csub(c2<T> a, c2<T> b) { return cmk<T>(a.x - b.x, a.y - b.y); }
template <typename T> NEP_DEV c2<T> cmul(c2<T> a, c2<T> b) {
  return cmk<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
template <typename T> NEP_DEV c2<T> cmulc(c2<T> a, c2<T> b) {
  return cmk<T>(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
// conj(a) * b
template <typename T> NEP_DEV c2<T> cconjmul(c2<T> a, c2<T> b) {
  return cmk<T>(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
template <typename T> NEP_DEV c2<T> cscale(c2<T> a, T s) { return cmk<T>(a.x * s, a.y * s); }
// acc - a*b
template <typename T> NEP_DEV c2<T> cfms(c2<T> acc, c2<T> a, c2<T> b) {
  return cmk<T>(acc.x - (a.x * b.x - a.y * b.y), acc.y - (a.x * b.y + a.y * b.x));
}
// acc + a*b
template <typename T> NEP_DEV c2<T> cfma(c2<T> acc, c2<T> a, c2<T> b) {
  return cmk<T>(acc.x + (a.x * b.x - a.y * b.y), acc.y + (a.x * b.y + a.y * b.x));
}
template <typename T> NEP_DEV T cabs1(c2<T> a) { return fabs(a.x) + fabs(a.y); }
template <typename T> NEP_DEV T cabs2(c2<T> a) { return a.x * a.x + a.y * a.y; }
// 1/a with scaling (Smith's method) so that |a| near the range limits does not overflow
template <typename T> NEP_DEV c2<T> crcp(c2<T> a) {
  if (fabs(a.x) >= fabs(a.y)) {
    T r = a.y / a.x, d = a.x + a.y * r;
    return cmk<T>(T(1) / d, -r / d);
  }
  T r = a.x / a.y, d = a.y + a.x * r;
  return cmk<T>(r / d, T(-1) / d);
}
template <typename T> NEP_DEV c2<T> cdiv(c2<T> a, c2<T> b) { return cmul<T>(a, crcp<T>(b)); }

template <typename D, typename S> NEP_DEV c2<D> ccast(c2<S> a) { return cmk<D>(D(a.x), D(a.y)); }

// ---------------------------------------------------------------- matrix cores
typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
template <typename T> struct AccT;
template <> struct AccT<double> { typedef d4 t; };
template <> struct AccT<float> { typedef f4 t; };
template <typename T> using acc4 = typename AccT<T>::t;

// D = A(16x4) * B(4x16) + C, wave-wide.  Operand lanes: A[l%16][l/16], B[l/16][l%16].
NEP_DEV d4 mfma16(double a, double b, d4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
NEP_DEV f4 mfma16(float a, float b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }

// Row of accumulator register r held by lane l (column is l % 16).  The two
// 16x16x4 instructions lay their results out differently: f64 interleaves the row
// groups (row l/16 + 4r), f32 keeps them blocked (row 4(l/16) + r).
template <typename T> NEP_DEV int acc_row(int lane, int r);
template <> NEP_DEV int acc_row<double>(int lane, int r) { return (lane >> 4) + 4 * r; }
template <> NEP_DEV int acc_row<float>(int lane, int r) { return 4 * (lane >> 4) + r; }

template <typename T> NEP_DEV acc4<T> acc_zero() { acc4<T> z = {T(0), T(0), T(0), T(0)}; return z; }

// ---------------------------------------------------------------- wave reductions
NEP_DEV double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
NEP_DEV float wave_sum(float v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
