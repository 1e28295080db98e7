// Building blocks of the plane-wave FFTs: in-register DFT codelets and a two-stage line FFT on LDS.
//
// Sign convention: DIR = +1 is the unnormalised inverse transform sum_k c_k exp(+2 pi i k j / n) that
// takes sphere coefficients to real space; DIR = -1 is the forward transform. Normalisation by n^-3 is
// applied once, where the result returns to the sphere.
#pragma once
#include "common.h"

namespace chebfd {

template <int I, int N, typename F> __device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, N>(f);
  }
}

// v * W_R^(J) with W_R = exp(DIR * 2 pi i / R), J a compile-time constant
template <int R, int J, int DIR, typename T> __device__ __forceinline__ cx<T> twc(cx<T> v) {
  constexpr int j = ((J % R) + R) % R;
  if constexpr (j == 0) {
    return v;
  } else if constexpr (4 * j == R) {  // DIR * i
    return DIR > 0 ? cx<T>{-v.y, v.x} : cx<T>{v.y, -v.x};
  } else if constexpr (2 * j == R) {
    return cx<T>{-v.x, -v.y};
  } else if constexpr (4 * j == 3 * R) {  // -DIR * i
    return DIR > 0 ? cx<T>{v.y, -v.x} : cx<T>{-v.y, v.x};
  } else {
    constexpr double c = ct_trig(j, R, false);
    constexpr double s = DIR * ct_trig(j, R, true);
    const T cc = T(c), ss = T(s);
    return cx<T>{v.x * cc - v.y * ss, v.x * ss + v.y * cc};
  }
}

template <int R> struct SplitOf {  // smallest useful radix of R
  static constexpr int A = (R % 4 == 0 && R != 8) ? 4 : (R % 2 == 0 ? 2 : (R % 3 == 0 ? 3 : R));
};

// In-place DFT of length R on registers, natural order in and out.
template <int R, int DIR> struct Dft {
  template <typename T> __device__ __forceinline__ static void run(cx<T>* v) {
    if constexpr (R == 1) {
      return;
    } else if constexpr (R == 2) {
      cx<T> a = v[0], b = v[1];
      v[0] = a + b;
      v[1] = a - b;
    } else if constexpr (R == 3) {
      // X_k = sum_n x_n W3^{nk}; W3 = -1/2 + DIR i sqrt(3)/2
      const T h = T(0.5), s3 = T(DIR * 0.86602540378443864676372317075294);
      cx<T> a = v[0], b = v[1], c = v[2];
      cx<T> t1 = b + c, t2 = b - c;
      v[0] = a + t1;
      cx<T> m = {a.x - h * t1.x, a.y - h * t1.y};
      cx<T> r = {-s3 * t2.y, s3 * t2.x};  // DIR i sqrt3/2 (b - c)
      v[1] = m + r;
      v[2] = m - r;
    } else if constexpr (R == 4) {
      cx<T> a = v[0] + v[2], b = v[0] - v[2], c = v[1] + v[3], d = v[1] - v[3];
      cx<T> di = DIR > 0 ? cx<T>{-d.y, d.x} : cx<T>{d.y, -d.x};  // DIR * i * d
      v[0] = a + c;
      v[2] = a - c;
      v[1] = b + di;
      v[3] = b - di;
    } else {
      // R = A * B, n = B n1 + n2, X[k1 + A k2] = sum_n2 W_B^{n2 k2} W_R^{n2 k1} sum_n1 x[B n1 + n2] W_A^{n1 k1}
      constexpr int A = SplitOf<R>::A;
      constexpr int B = R / A;
      static_assert(A * B == R && A > 1 && B > 1, "unsupported codelet length");
      static_for<0, B>([&](auto n2c) {
        constexpr int n2 = decltype(n2c)::value;
        cx<T> y[A];
#pragma unroll
        for (int n1 = 0; n1 < A; ++n1) y[n1] = v[B * n1 + n2];
        Dft<A, DIR>::run(y);
        static_for<0, A>([&](auto k1c) {
          constexpr int k1 = decltype(k1c)::value;
          v[B * k1 + n2] = twc<R, n2 * k1, DIR>(y[k1]);
        });
      });
      cx<T> out[R];
#pragma unroll
      for (int k1 = 0; k1 < A; ++k1) {
        cx<T> z[B];
#pragma unroll
        for (int n2 = 0; n2 < B; ++n2) z[n2] = v[B * k1 + n2];
        Dft<B, DIR>::run(z);
#pragma unroll
        for (int k2 = 0; k2 < B; ++k2) out[k1 + A * k2] = z[k2];
      }
#pragma unroll
      for (int k = 0; k < R; ++k) v[k] = out[k];
    }
  }
};

// Factorisation n = N1 * N2 of the supported box sizes (both factors handled by register codelets).
template <int N> struct LineSplit;
template <> struct LineSplit<8> { static constexpr int N1 = 2, N2 = 4; };
template <> struct LineSplit<12> { static constexpr int N1 = 3, N2 = 4; };
template <> struct LineSplit<16> { static constexpr int N1 = 4, N2 = 4; };
template <> struct LineSplit<24> { static constexpr int N1 = 4, N2 = 6; };
template <> struct LineSplit<32> { static constexpr int N1 = 4, N2 = 8; };
template <> struct LineSplit<48> { static constexpr int N1 = 6, N2 = 8; };
template <> struct LineSplit<64> { static constexpr int N1 = 8, N2 = 8; };
template <> struct LineSplit<96> { static constexpr int N1 = 8, N2 = 12; };
template <> struct LineSplit<128> { static constexpr int N1 = 8, N2 = 16; };

// In-place length-N DFTs of `nlines` lines held in LDS: point e of line l at buf[l * ls + e], natural order in
// and out. The stride ls must be at least N1 * (N2 + 1): between the two register-codelet stages (N1, then
// N2, with the twiddle W_N^{n2 k1}) the line is held as N1 groups of N2 with one pad slot per group, so
// that lanes reading a group each are spread over the LDS banks. twA[k1 N2 + n2] = exp(-2 pi i n2 k1 / N)
// (read by lanes of consecutive n2), conjugated for the inverse. All threads of the block must call it.
template <int N, int DIR, typename T>
__device__ void lds_fft(cx<T>* buf, int nlines, int ls, const cx<T>* twA) {
  constexpr int N1 = LineSplit<N>::N1, N2 = LineSplit<N>::N2, PS = N2 + 1;
  const int tid = threadIdx.x, nth = blockDim.x;
  // stage 1 per (line, n2): DFT over n1 of x[N2 n1 + n2], times W_N^{n2 k1}, to group slot PS k1 + n2
  const int lines1 = nth / N2 > 0 ? nth / N2 : 1;
  for (int l0 = 0; l0 < nlines; l0 += lines1) {
    const int l1 = min(nlines, l0 + lines1);
    const bool act = tid < (l1 - l0) * N2;
    const int l = l0 + tid / N2, n2 = tid % N2;
    cx<T> v[N1];
    if (act) {
      const cx<T>* p = buf + l * ls + n2;
#pragma unroll
      for (int n1 = 0; n1 < N1; ++n1) v[n1] = p[n1 * N2];
      Dft<N1, DIR>::run(v);
#pragma unroll
      for (int k1 = 1; k1 < N1; ++k1) {
        cx<T> w = twA[k1 * N2 + n2];
        if (DIR > 0) w.y = -w.y;
        v[k1] = cmul(v[k1], w);
      }
    }
    __syncthreads();
    if (act) {
      cx<T>* p = buf + l * ls + n2;
#pragma unroll
      for (int k1 = 0; k1 < N1; ++k1) p[PS * k1] = v[k1];
    }
    __syncthreads();
  }
  // stage 2 per (line, k1): DFT over n2 of the group k1 -> X[k1 + N1 k2] (natural order)
  const int lines2 = nth / N1 > 0 ? nth / N1 : 1;
  for (int l0 = 0; l0 < nlines; l0 += lines2) {
    const int l1 = min(nlines, l0 + lines2);
    const bool act = tid < (l1 - l0) * N1;
    const int l = l0 + tid / N1, k1 = tid % N1;
    cx<T> v[N2];
    if (act) {
      const cx<T>* p = buf + l * ls + PS * k1;
#pragma unroll
      for (int n2 = 0; n2 < N2; ++n2) v[n2] = p[n2];
      Dft<N2, DIR>::run(v);
    }
    __syncthreads();
    if (act) {
      cx<T>* p = buf + l * ls + k1;
#pragma unroll
      for (int k2 = 0; k2 < N2; ++k2) p[k2 * N1] = v[k2];
    }
    __syncthreads();
  }
}

}  // namespace chebfd
