// Minimal complex arithmetic for device code (interleaved re, im).
#pragma once

#include <hip/hip_runtime.h>

namespace yr {

template <typename T>
struct cplx {
  T re, im;
  __host__ __device__ cplx() : re(0), im(0) {}
  __host__ __device__ cplx(T r, T i = 0) : re(r), im(i) {}
  template <typename U>
  __host__ __device__ explicit cplx(const cplx<U>& o) : re((T)o.re), im((T)o.im) {}
};

template <typename T>
__host__ __device__ inline cplx<T> operator+(cplx<T> a, cplx<T> b) {
  return cplx<T>(a.re + b.re, a.im + b.im);
}
template <typename T>
__host__ __device__ inline cplx<T> operator-(cplx<T> a, cplx<T> b) {
  return cplx<T>(a.re - b.re, a.im - b.im);
}
template <typename T>
__host__ __device__ inline cplx<T> operator-(cplx<T> a) {
  return cplx<T>(-a.re, -a.im);
}
template <typename T>
__host__ __device__ inline cplx<T> operator*(cplx<T> a, cplx<T> b) {
  return cplx<T>(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <typename T>
__host__ __device__ inline cplx<T> operator*(T s, cplx<T> a) {
  return cplx<T>(s * a.re, s * a.im);
}
template <typename T>
__host__ __device__ inline cplx<T> operator*(cplx<T> a, T s) {
  return cplx<T>(s * a.re, s * a.im);
}
template <typename T>
__host__ __device__ inline cplx<T> conj(cplx<T> a) {
  return cplx<T>(a.re, -a.im);
}
template <typename T>
__host__ __device__ inline T norm2(cplx<T> a) {
  return a.re * a.re + a.im * a.im;
}
template <typename T>
__host__ __device__ inline cplx<T> cdiv(cplx<T> a, cplx<T> b) {
  T d = b.re * b.re + b.im * b.im;
  return cplx<T>((a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d);
}

typedef cplx<double> zd;

}  // namespace yr
