// Shared device/host helpers: complex arithmetic on float2/double2.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define PSFD_HD __host__ __device__ __forceinline__
#define PSFD_D __device__ __forceinline__

template <class R> struct cplx_of;
template <> struct cplx_of<float> { using type = float2; };
template <> struct cplx_of<double> { using type = double2; };
template <class T> struct real_of;
template <> struct real_of<float2> { using type = float; };
template <> struct real_of<double2> { using type = double; };

template <class T> PSFD_HD T cmake(double a, double b) {
  T r; r.x = (typename real_of<T>::type)a; r.y = (typename real_of<T>::type)b; return r;
}
template <class T> PSFD_HD T cadd(T a, T b) { a.x += b.x; a.y += b.y; return a; }
template <class T> PSFD_HD T csub(T a, T b) { a.x -= b.x; a.y -= b.y; return a; }
template <class T> PSFD_HD T cmul(T a, T b) {
  T r; r.x = a.x * b.x - a.y * b.y; r.y = a.x * b.y + a.y * b.x; return r;
}
// a * conj(b)
template <class T> PSFD_HD T cmulc(T a, T b) {
  T r; r.x = a.x * b.x + a.y * b.y; r.y = a.y * b.x - a.x * b.y; return r;
}
template <class T, class S> PSFD_HD T cscale(T a, S s) { a.x *= s; a.y *= s; return a; }
// multiply by -i (forward sign) or +i (inverse sign)
template <class T, bool INV> PSFD_HD T cmul_mi(T a) {
  T r;
  if (INV) { r.x = -a.y; r.y = a.x; } else { r.x = a.y; r.y = -a.x; }
  return r;
}
PSFD_HD double2 cdiv(double2 a, double2 b) {
  double d = b.x * b.x + b.y * b.y;
  double inv = 1.0 / d;
  double2 r; r.x = (a.x * b.x + a.y * b.y) * inv; r.y = (a.y * b.x - a.x * b.y) * inv; return r;
}
PSFD_HD double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }

PSFD_HD float2 to_f(double2 a) { return make_float2((float)a.x, (float)a.y); }
PSFD_HD double2 to_d(float2 a) { return make_double2((double)a.x, (double)a.y); }
PSFD_HD double2 to_d(double2 a) { return a; }
template <class T> PSFD_HD T from_d(double2 a);
template <> PSFD_HD float2 from_d<float2>(double2 a) { return to_f(a); }
template <> PSFD_HD double2 from_d<double2>(double2 a) { return a; }

PSFD_HD int ilog2i(int v) { int r = 0; while ((1 << r) < v) ++r; return r; }

// XCD-aware block order. The dispatcher hands workgroup hw to XCD hw mod 8, so
// the blocks one XCD receives (hw = x, x + 8, x + 16, ...) are given one
// contiguous run of logical ids: neighbouring logical blocks then share an L2
// and run at about the same time. A bijection of [0, nb) when 8 divides nb,
// the identity otherwise.
PSFD_D unsigned xcd_order(unsigned hw, unsigned nb) {
  return (nb & 7u) ? hw : (hw & 7u) * (nb >> 3) + (hw >> 3);
}
