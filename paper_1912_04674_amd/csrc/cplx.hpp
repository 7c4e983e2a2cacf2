// cplx.hpp -- minimal complex arithmetic on float2 / double2 for the kernels.
#pragma once
#include <hip/hip_runtime.h>

namespace envpic {

template <class C, class R> __host__ __device__ inline C mk(R re, R im) {
  C c;
  c.x = re;
  c.y = im;
  return c;
}
template <class C> __host__ __device__ inline C cadd(C a, C b) { return mk<C>(a.x + b.x, a.y + b.y); }
template <class C> __host__ __device__ inline C csub(C a, C b) { return mk<C>(a.x - b.x, a.y - b.y); }
template <class C, class R> __host__ __device__ inline C cscale(C a, R s) { return mk<C>(a.x * s, a.y * s); }
template <class C> __host__ __device__ inline C cmul(C a, C b) {
  return mk<C>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// i * a
template <class C> __host__ __device__ inline C cmuli(C a) { return mk<C>(-a.y, a.x); }
template <class C> __host__ __device__ inline auto cnorm(C a) -> decltype(a.x) { return a.x * a.x + a.y * a.y; }
// Re[a e^{-i theta}] with (c, s) = (cos, sin)
template <class C, class R> __host__ __device__ inline R mode1_at(C a, R c, R s) { return a.x * c + a.y * s; }

}  // namespace envpic
