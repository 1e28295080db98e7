// Shared device/host helpers of the chebfd library: complex element types, status plumbing.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <type_traits>

namespace chebfd {

// Interleaved complex element (re, im), the storage layout of every band block.
template <typename T> struct alignas(2 * sizeof(T)) cx { T x, y; };
using c128 = cx<double>;
using c64 = cx<float>;

template <typename T> __host__ __device__ inline cx<T> mk(T a, T b) { return cx<T>{a, b}; }
template <typename T> __host__ __device__ inline cx<T> operator+(cx<T> a, cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T> __host__ __device__ inline cx<T> operator-(cx<T> a, cx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T> __host__ __device__ inline cx<T> operator*(cx<T> a, T s) { return {a.x * s, a.y * s}; }
template <typename T> __host__ __device__ inline cx<T> cmul(cx<T> a, cx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename T> __host__ __device__ inline cx<T> cmulc(cx<T> a, cx<T> b) {
  return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename TO, typename TI> __host__ __device__ inline cx<TO> cvt(cx<TI> a) {
  return {static_cast<TO>(a.x), static_cast<TO>(a.y)};
}

// Compile-time sine/cosine of 2*pi*j/n by Taylor series after exact octant reduction of the rational
// angle; used only to fold the twiddles of the in-register DFT codelets into constants.
constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr double ct_sin_small(double x) {  // |x| <= pi/4
  double term = x, sum = x, x2 = x * x;
  for (int k = 1; k < 14; ++k) { term *= -x2 / ((2.0 * k) * (2.0 * k + 1.0)); sum += term; }
  return sum;
}
constexpr double ct_cos_small(double x) {
  double term = 1.0, sum = 1.0, x2 = x * x;
  for (int k = 1; k < 14; ++k) { term *= -x2 / ((2.0 * k - 1.0) * (2.0 * k)); sum += term; }
  return sum;
}
// returns cos(2 pi j / n) (want_sin = false) or sin(2 pi j / n)
constexpr double ct_trig(long j, long n, bool want_sin) {
  j %= n; if (j < 0) j += n;
  // angle = 2 pi j / n = (pi / 4) * (8 j / n); octant o = floor(8 j / n), remainder t = 8 j - o n
  long o = (8 * j) / n;
  long t = 8 * j - o * n;              // in [0, n)
  double a = (kPi / 4.0) * double(t) / double(n);  // in [0, pi/4)
  double s = ct_sin_small(a), c = ct_cos_small(a);
  double bs = ct_sin_small(kPi / 4.0 - a), bc = ct_cos_small(kPi / 4.0 - a);
  double cs = 0, cc = 0;  // cos / sin of the full angle
  switch (o) {
    case 0: cc = c; cs = s; break;          // [0, pi/4)
    case 1: cc = bs; cs = bc; break;        // pi/2 - (pi/4 - a)
    case 2: cc = -s; cs = c; break;         // pi/2 + a
    case 3: cc = -bc; cs = bs; break;       // pi - (pi/4 - a)
    case 4: cc = -c; cs = -s; break;        // pi + a
    case 5: cc = -bs; cs = -bc; break;      // 3pi/2 - (pi/4 - a)
    case 6: cc = s; cs = -c; break;         // 3pi/2 + a
    default: cc = bc; cs = -bs; break;      // 2pi - (pi/4 - a)
  }
  return want_sin ? cs : cc;
}

}  // namespace chebfd
