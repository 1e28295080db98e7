// Complex GEMM on CDNA4 matrix cores: four real 16x16x4 MFMAs per complex product block.
//
// Used for every O(Npw x Nprojs) contraction of the filter (projections P^H psi and back-projection
// P w, Alg. 1; the reuse trick of Sec. 5.1 leaves one of each per filter step), for the Rayleigh-Ritz
// subspace matrices Y^H H Y, Y^H S Y and the rotation Y Z (Alg. 2), and for the small projector-space
// products with P^H P and the capacitance inverse (Sec. 5.1).
#include "kernels.h"

namespace chebfd {
namespace {

template <typename T> struct Mfma;
template <> struct Mfma<double> {
  typedef double acc __attribute__((ext_vector_type(4)));
  __device__ __forceinline__ static acc run(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};
template <> struct Mfma<float> {
  typedef float acc __attribute__((ext_vector_type(4)));
  __device__ __forceinline__ static acc run(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};

constexpr int BM = 64, BN = 64, BK = 16, PAD = 2, NT = 256;

template <typename E>
__device__ __forceinline__ void epi_store(const Epi<E>& e, long m, long n, double re, double im) {
  double xr = e.alpha * re, xi = e.alpha * im;
  if (e.L) { cx<E> v = e.L[m + n * e.ldl]; xr += e.bL * double(v.x); xi += e.bL * double(v.y); }
  if (e.U) { cx<E> v = e.U[m + n * e.ldu]; xr += e.bU * double(v.x); xi += e.bU * double(v.y); }
  if (e.W) { cx<E> v = e.W[m + n * e.ldw]; xr += e.bW * double(v.x); xi += e.bW * double(v.y); }
  e.out[m + n * e.ldo] = cx<E>{E(xr), E(xi)};
}

// One 64 x 64 complex output tile per block of 4 waves; wave w owns the 32 x 32 quadrant
// (w & 1, w >> 1) as 2 x 2 MFMA blocks with separate real and imaginary accumulators.
// ROLE only separates kernel names per use (projection, back-projection, small, subspace) for profiling.
template <typename T, typename EA, typename EB, typename EO, int MODE, int ROLE>
__global__ __launch_bounds__(NT) void k_gemm(int M, int N, int K, int kchunk, const cx<EA>* __restrict__ A,
                                             long lda, const cx<EB>* __restrict__ B, long ldb, Epi<EO> epi,
                                             c128* __restrict__ part) {
  __shared__ T Ar[BK][BM + PAD], Ai[BK][BM + PAD], Br[BK][BN + PAD], Bi[BK][BN + PAD];
  using acc_t = typename Mfma<T>::acc;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
  const long m0 = long(blockIdx.x) * BM, n0 = long(blockIdx.y) * BN;
  const int kbeg = blockIdx.z * kchunk;
  const int kend = min(K, kbeg + kchunk);

  acc_t cr[2][2], ci[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) { cr[i][j][v] = T(0); ci[i][j][v] = T(0); }

  // global -> registers for one K tile (converted to the MFMA type), registers -> LDS planes
  constexpr int RA = (BM * BK) / NT, RBn = (BN * BK) / NT;
  T ra_r[RA], ra_i[RA], rb_r[RBn], rb_i[RBn];
  auto load_tile = [&](int k0) {
#pragma unroll
    for (int r = 0; r < RA; ++r) {
      const int idx = tid + r * NT;
      int kk, mm;
      if (MODE == GEMM_CN) { kk = idx % BK; mm = idx / BK; }
      else { mm = idx % BM; kk = idx / BM; }
      const long gm = m0 + mm;
      const int gk = k0 + kk;
      cx<EA> v = {EA(0), EA(0)};
      if (gm < M && gk < kend) v = (MODE == GEMM_CN) ? A[gk + gm * lda] : A[gm + long(gk) * lda];
      ra_r[r] = T(v.x);
      ra_i[r] = T(v.y);
    }
#pragma unroll
    for (int r = 0; r < RBn; ++r) {
      const int idx = tid + r * NT;
      const int kk = idx % BK, nn = idx / BK;
      const long gn = n0 + nn;
      const int gk = k0 + kk;
      cx<EB> v = {EB(0), EB(0)};
      if (gn < N && gk < kend) v = B[gk + gn * ldb];
      rb_r[r] = T(v.x);
      rb_i[r] = T(v.y);
    }
  };
  auto store_tile = [&]() {
#pragma unroll
    for (int r = 0; r < RA; ++r) {
      const int idx = tid + r * NT;
      int kk, mm;
      if (MODE == GEMM_CN) { kk = idx % BK; mm = idx / BK; }
      else { mm = idx % BM; kk = idx / BM; }
      Ar[kk][mm] = ra_r[r];
      Ai[kk][mm] = ra_i[r];
    }
#pragma unroll
    for (int r = 0; r < RBn; ++r) {
      const int idx = tid + r * NT;
      const int kk = idx % BK, nn = idx / BK;
      Br[kk][nn] = rb_r[r];
      Bi[kk][nn] = rb_i[r];
    }
  };

  if (kbeg < kend) {
    load_tile(kbeg);
    store_tile();
  }
  __syncthreads();
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    const bool more = k0 + BK < kend;
    if (more) load_tile(k0 + BK);  // in flight while this tile is multiplied
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      T ar[2], ai[2], br[2], bi[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        ar[i] = Ar[ks + lk][wm + 16 * i + li];
        ai[i] = Ai[ks + lk][wm + 16 * i + li];
        br[i] = Br[ks + lk][wn + 16 * i + li];
        bi[i] = Bi[ks + lk][wn + 16 * i + li];
      }
#pragma unroll
      for (int i = 0; i < 2; ++i) {
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          if (MODE == GEMM_CN) {  // conj(a) b
            cr[i][j] = Mfma<T>::run(ar[i], br[j], cr[i][j]);
            cr[i][j] = Mfma<T>::run(ai[i], bi[j], cr[i][j]);
            ci[i][j] = Mfma<T>::run(ar[i], bi[j], ci[i][j]);
            ci[i][j] = Mfma<T>::run(-ai[i], br[j], ci[i][j]);
          } else {  // a b
            cr[i][j] = Mfma<T>::run(ar[i], br[j], cr[i][j]);
            cr[i][j] = Mfma<T>::run(-ai[i], bi[j], cr[i][j]);
            ci[i][j] = Mfma<T>::run(ar[i], bi[j], ci[i][j]);
            ci[i][j] = Mfma<T>::run(ai[i], br[j], ci[i][j]);
          }
        }
      }
    }
    __syncthreads();
    if (more) {
      store_tile();
      __syncthreads();
    }
  }

  // accumulator v of a lane holds column li of each 16 x 16 block, row 4*lk + v for the f32 MFMA and
  // row lk + 4*v for the f64 MFMA (lane layouts of the two 16x16x4 instructions differ)
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = sizeof(T) == 8 ? lk + 4 * v : 4 * lk + v;
        const long m = m0 + wm + 16 * i + row;
        const long n = n0 + wn + 16 * j + li;
        if (m < M && n < N) {
          if (part) {
            part[(long(blockIdx.z) * N + n) * M + m] = c128{double(cr[i][j][v]), double(ci[i][j][v])};
          } else {
            epi_store(epi, m, n, double(cr[i][j][v]), double(ci[i][j][v]));
          }
        }
      }
}

template <typename EO>
__global__ __launch_bounds__(256) void k_reduce(int M, int N, int splits, const c128* __restrict__ part, Epi<EO> epi) {
  const long total = long(M) * N;
  for (long t = blockIdx.x * long(blockDim.x) + threadIdx.x; t < total; t += long(gridDim.x) * blockDim.x) {
    const long n = t / M, m = t - n * M;
    double re = 0.0, im = 0.0;
    for (int s = 0; s < splits; ++s) {
      c128 v = part[long(s) * total + t];
      re += v.x;
      im += v.y;
    }
    epi_store(epi, m, n, re, im);
  }
}

}  // namespace

int gemm_pick_splits(int M, int N, int K) {
  if (M <= 0 || N <= 0 || K <= 0) return 1;
  const long tiles = long((M + BM - 1) / BM) * ((N + BN - 1) / BN);
  const long want = 512;  // ~2 blocks per CU: enough to fill the chip, half the partial-sum traffic
  long s = (want + tiles - 1) / tiles;
  const long kblocks = (K + BK - 1) / BK;
  if (s > kblocks / 2) s = kblocks / 2;  // at least two K tiles per split
  if (s > 32) s = 32;
  if (s < 1) s = 1;
  return int(s);
}

template <typename T, typename EA, typename EB, typename EO>
hipError_t gemm(GemmMode mode, int M, int N, int K, const cx<EA>* A, long lda, const cx<EB>* B, long ldb,
                const Epi<EO>& epi, int splits, c128* part, hipStream_t st, GemmRole role) {
  if (M <= 0 || N <= 0) return hipSuccess;
  if (splits < 1) splits = 1;
  int kchunk = (K + splits - 1) / splits;
  kchunk = ((kchunk + BK - 1) / BK) * BK;
  if (kchunk < BK) kchunk = BK;
  splits = K > 0 ? (K + kchunk - 1) / kchunk : 1;
  const bool use_part = splits > 1;
  if (use_part && !part) return hipErrorInvalidValue;
  dim3 grid((M + BM - 1) / BM, (N + BN - 1) / BN, splits);
  c128* pp = use_part ? part : nullptr;
  auto launch = [&](auto modec, auto rolec) {
    constexpr int MO = decltype(modec)::value, RO = decltype(rolec)::value;
    hipLaunchKernelGGL((k_gemm<T, EA, EB, EO, MO, RO>), grid, dim3(NT), 0, st, M, N, K, kchunk, A, lda, B, ldb, epi, pp);
  };
  using CN = std::integral_constant<int, GEMM_CN>;
  using NNm = std::integral_constant<int, GEMM_NN>;
  switch (role) {
    case ROLE_PROJECT: mode == GEMM_CN ? launch(CN{}, std::integral_constant<int, 1>{}) : launch(NNm{}, std::integral_constant<int, 1>{}); break;
    case ROLE_BACKPROJECT: mode == GEMM_CN ? launch(CN{}, std::integral_constant<int, 2>{}) : launch(NNm{}, std::integral_constant<int, 2>{}); break;
    case ROLE_SUBSPACE: mode == GEMM_CN ? launch(CN{}, std::integral_constant<int, 3>{}) : launch(NNm{}, std::integral_constant<int, 3>{}); break;
    default: mode == GEMM_CN ? launch(CN{}, std::integral_constant<int, 0>{}) : launch(NNm{}, std::integral_constant<int, 0>{}); break;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !use_part) return e;
  const long total = long(M) * N;
  int blocks = int((total + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL((k_reduce<EO>), dim3(blocks), dim3(256), 0, st, M, N, splits, part, epi);
  return hipGetLastError();
}

#define INST(T, EA, EB, EO)                                                                               \
  template hipError_t gemm<T, EA, EB, EO>(GemmMode, int, int, int, const cx<EA>*, long, const cx<EB>*, long, \
                                          const Epi<EO>&, int, c128*, hipStream_t, GemmRole);
INST(double, double, double, double)
INST(float, float, float, float)
INST(float, float, double, float)
INST(float, float, float, double)
#undef INST

}  // namespace chebfd
