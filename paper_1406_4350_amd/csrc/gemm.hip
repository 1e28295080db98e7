// Complex GEMM on CDNA4 matrix cores: three (FP64) or four (FP32) real 16x16x4 MFMAs per complex product block,
// and a hi/lo split FP16 form for the projector products of the mixed-precision filter.
//
// Used for every O(Npw x Nprojs) contraction of the filter (projections P^H psi and back-projection
// P w, Alg. 1; the reuse trick of Sec. 5.1 leaves one of each per filter step), for the Rayleigh-Ritz
// subspace matrices Y^H H Y, Y^H S Y and the rotation Y Z (Alg. 2), and for the small projector-space
// products with P^H P and the capacitance inverse (Sec. 5.1).
#include <algorithm>
#include <type_traits>

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

// K tiles of 32 and rows padded by one element: measured best on the paw48 projector shapes among K tiles of 16
// and 32 and paddings of 1 to 16 (a padding of 16 puts the transposed tile stores on one bank)
constexpr int BM = 64, BN = 64, BK = 32, PAD = 1, NT = 256;

// Block placement. The hardware deals the blocks of a launch to the 8 XCDs in turn (block i to XCD i mod 8),
// each XCD with its own L2. Physical block i takes the logical item that gives each XCD one contiguous run of
// items. Items are numbered split by split; inside a split, in groups of `grp` M tiles, and inside a group with
// the M tile fastest. With grp = 8 the blocks an XCD holds at once (32 to 64) cover a square-ish patch of up to 8
// M tiles by 4 to 8 N tiles, so each slice of A and of B they read is shared by several resident blocks in the
// XCD's L2: the rule for long contractions (K >= M: projections, Gram matrices), where both operands stream
// K-long slices. With grp = 1 the N tile runs fastest and each M tile's slice of A is read once, by all N tiles
// at the same time: the rule for tall, short-K products (back-projection, rotation), whose A dwarfs B.
constexpr int kTileGroup = 8;
constexpr int kUpperTiles = -1;  // group value of the upper-triangle tile order (Hermitian products)
__host__ __device__ inline void gemm_tile_of(int i, int total, int tm, int tn, int grp, int& bx, int& by, int& bz) {
  const int q = total / 8, rem = total % 8, k = i % 8, j = i / 8;
  const int L = (k < rem ? k * (q + 1) : rem * (q + 1) + (k - rem) * q) + j;
  if (grp == kUpperTiles) {  // the tiles bx <= by of a square grid, column by column: t = by (by + 1) / 2 + bx
    const int per = tm * (tm + 1) / 2;
    bz = L / per;
    const int t = L - bz * per;
    int c = int((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while (c * (c + 1) / 2 > t) --c;
    while ((c + 1) * (c + 2) / 2 <= t) ++c;
    by = c;
    bx = t - c * (c + 1) / 2;
    return;
  }
  const int per = tm * tn;
  bz = L / per;
  const int t = L - bz * per;
  const int first = (t / (grp * tn)) * grp;
  const int gm = tm - first < grp ? tm - first : grp;  // M tiles in this group (fewer in the last)
  const int r = t - first * tn;
  bx = first + r % gm;
  by = r / gm;
}
inline int tile_group(int M, int K) { return K >= M ? kTileGroup : 1; }

template <typename E>
__device__ __forceinline__ void epi_store(const Epi<E>& e, long m, long n, double re, double im) {
  double xr = e.alpha * re, xi = e.alpha * im;
  if (e.L) { cx<E> v = e.L[m + n * e.ldl]; xr += e.bL * double(v.x); xi += e.bL * double(v.y); }
  if (e.U) { cx<E> v = e.U[m + n * e.ldu]; xr += e.bU * double(v.x); xi += e.bU * double(v.y); }
  if (e.W) { cx<E> v = e.W[m + n * e.ldw]; xr += e.bW * double(v.x); xi += e.bW * double(v.y); }
  e.out[m + n * e.ldo] = cx<E>{E(xr), e.real_only ? E(0) : E(xi)};
}

// Epilogue operands moved into the leading slots (L, then U, then W) and counted: 0, 1 or 3 slots in use, a
// second operand without a third repeated in the third slot with weight 0 (it is a finite input). The tiled
// kernels take the count as a template parameter and read every used slot without a branch.
template <typename E> int epi_slots(Epi<E>& e) {
  const cx<E>* p[3] = {e.L, e.U, e.W};
  long l[3] = {e.ldl, e.ldu, e.ldw};
  double b[3] = {e.bL, e.bU, e.bW};
  int c = 0;
  for (int s = 0; s < 3; ++s)
    if (p[s]) { p[c] = p[s]; l[c] = l[s]; b[c] = b[s]; ++c; }
  for (int s = c; s < 3; ++s) { p[s] = nullptr; l[s] = 0; b[s] = 0.0; }
  if (c == 2) { p[2] = p[1]; l[2] = l[1]; b[2] = 0.0; c = 3; }
  e.L = p[0]; e.ldl = l[0]; e.bL = b[0];
  e.U = p[1]; e.ldu = l[1]; e.bU = b[1];
  e.W = p[2]; e.ldw = l[2]; e.bW = b[2];
  return c;
}

// Epilogue of one wave's NI x NJ MFMA blocks of 16 x 16 (T accumulators, the combined real and imaginary parts in
// cr, ci; rows of accumulator v given by row_of(v); column block j scaled by scale[j]). The NE operands of block
// b + 1 are requested, at clamped in-range indices, before the stores of block b, so that every thread keeps a
// block of loads in flight instead of waiting on each element in turn.
template <int NE, int NI, int NJ, typename E, typename Acc, typename RowOf>
__device__ __forceinline__ void epi_blocks(const Epi<E>& epi, int M, int N, long mb, long nb, int li,
                                           const Acc (&cr)[NI][NJ], const Acc (&ci)[NI][NJ],
                                           const double (&scale)[NJ], RowOf row_of) {
  constexpr int NS = NE > 0 ? NE : 1, NBLK = NI * NJ;
  const cx<E>* src[3] = {epi.L, epi.U, epi.W};
  const long lds[3] = {epi.ldl, epi.ldu, epi.ldw};
  const double bet[3] = {epi.bL, epi.bU, epi.bW};
  cx<E> buf[2][NS][4];
  auto eload = [&](int b, cx<E>(&dst)[NS][4]) {
    const int i = b / NJ, j = b % NJ;
    const long n = min(nb + 16 * j + li, long(N) - 1);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const long m = min(mb + 16 * i + row_of(v), long(M) - 1);
#pragma unroll
      for (int s = 0; s < NS; ++s)
        if constexpr (NE > 0) dst[s][v] = src[s][m + n * lds[s]];
    }
  };
  if constexpr (NE > 0) eload(0, buf[0]);
#pragma unroll
  for (int b = 0; b < NBLK; ++b) {
    if constexpr (NE > 0)
      if (b + 1 < NBLK) eload(b + 1, buf[(b + 1) & 1]);
    const int i = b / NJ, j = b % NJ;
    const long n = nb + 16 * j + li;
    const double f = epi.alpha * scale[j];
    // values of all four elements first, then the guarded stores: a value computed only under the guard would
    // let the compiler move its loads there and wait on them
    cx<E> val[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      double xr = f * double(cr[i][j][v]), xi = f * double(ci[i][j][v]);
#pragma unroll
      for (int s = 0; s < NS; ++s)
        if constexpr (NE > 0) {
          xr += bet[s] * double(buf[b & 1][s][v].x);
          xi += bet[s] * double(buf[b & 1][s][v].y);
        }
      val[v] = cx<E>{E(xr), epi.real_only ? E(0) : E(xi)};
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const long m = mb + 16 * i + row_of(v);
      if (m < M && n < N) epi.out[m + n * epi.ldo] = val[v];
    }
  }
}

// One 64 x 64 complex output tile per block of 4 waves; wave w owns the 32 x 32 quadrant
// (w & 1, w >> 1) as 2 x 2 MFMA blocks. FP64 tiles take three real products per complex product
// (P1 = a_r b_r, P2 = a_i b_i, P3 = (a_r + s a_i)(b_r + b_i) with s = 1 for a b and s = -1 for conj(a) b:
// re = P1 - s P2, im = P3 - P1 - s P2), the sums formed in registers from the real and imaginary planes
// (storing them as two more LDS planes measured 9% slower); FP32 tiles keep the four-product form, whose
// rounding does not grow with the magnitude of the other component.
// ROLE only separates kernel names per use (projection, back-projection, small, subspace) for profiling.
template <typename T, typename EA, typename EB, typename EO, int MODE, int ROLE, int NE>
__global__ __launch_bounds__(NT, 2) void k_gemm(int M, int N, int K, int kchunk, const cx<EA>* __restrict__ A,
                                             long lda, const cx<EB>* __restrict__ B, long ldb, Epi<EO> epi,
                                             c128* __restrict__ part, int grp) {
  constexpr bool G3 = sizeof(T) == 8;
  __shared__ T Ar[BK][BM + PAD], Ai[BK][BM + PAD], Br[BK][BN + PAD], Bi[BK][BN + PAD];
  using acc_t = typename Mfma<T>::acc;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
  int bx, by, bz;
  gemm_tile_of(blockIdx.x, gridDim.x, (M + BM - 1) / BM, (N + BN - 1) / BN, grp, bx, by, bz);
  const long m0 = long(bx) * BM, n0 = long(by) * BN;
  const int kbeg = bz * kchunk;
  const int kend = min(K, kbeg + kchunk);

  acc_t cr[2][2], ci[2][2], c3[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) { cr[i][j][v] = T(0); ci[i][j][v] = T(0); c3[i][j][v] = T(0); }

  // global -> registers for one K tile (raw storage type, so that the loads stay in flight while the previous
  // tile is multiplied), registers -> LDS planes converted to the MFMA type
  constexpr int RA = (BM * BK) / NT, RBn = (BN * BK) / NT;
  cx<EA> va[RA];
  cx<EB> vb[RBn];
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
      va[r] = v;
    }
#pragma unroll
    for (int r = 0; r < RBn; ++r) {
      const int idx = tid + r * NT;
      const int kk = idx % BK, nn = idx / BK;
      const long gn = n0 + nn;
      const int gk = k0 + kk;
      cx<EB> v = {EB(0), EB(0)};
      if (gn < N && gk < kend) v = B[gk + gn * ldb];
      vb[r] = v;
    }
  };
  auto store_tile = [&]() {
#pragma unroll
    for (int r = 0; r < RA; ++r) {
      const int idx = tid + r * NT;
      int kk, mm;
      if (MODE == GEMM_CN) { kk = idx % BK; mm = idx / BK; }
      else { mm = idx % BM; kk = idx / BM; }
      Ar[kk][mm] = T(va[r].x);
      Ai[kk][mm] = T(va[r].y);
    }
#pragma unroll
    for (int r = 0; r < RBn; ++r) {
      const int idx = tid + r * NT;
      const int kk = idx % BK, nn = idx / BK;
      Br[kk][nn] = T(vb[r].x);
      Bi[kk][nn] = T(vb[r].y);
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
      if constexpr (G3) {
        // cr <- P1, ci <- P2, c3 <- P3
        T as[2], bs[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          as[i] = MODE == GEMM_CN ? ar[i] - ai[i] : ar[i] + ai[i];
          bs[i] = br[i] + bi[i];
        }
#pragma unroll
        for (int i = 0; i < 2; ++i) {
#pragma unroll
          for (int j = 0; j < 2; ++j) {
            cr[i][j] = Mfma<T>::run(ar[i], br[j], cr[i][j]);
            ci[i][j] = Mfma<T>::run(ai[i], bi[j], ci[i][j]);
            c3[i][j] = Mfma<T>::run(as[i], bs[j], c3[i][j]);
          }
        }
      } else {
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
    }
    __syncthreads();
    if (more) {
      store_tile();
      __syncthreads();
    }
  }

  if constexpr (G3) {
    constexpr T sg = MODE == GEMM_CN ? T(-1) : T(1);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const T p1 = cr[i][j][v], p2 = ci[i][j][v], p3 = c3[i][j][v];
          cr[i][j][v] = p1 - sg * p2;
          ci[i][j][v] = p3 - p1 - sg * p2;
        }
  }
  // accumulator v of a lane holds column li of each 16 x 16 block, row 4*lk + v for the f32 MFMA and
  // row lk + 4*v for the f64 MFMA (lane layouts of the two 16x16x4 instructions differ)
  auto row_of = [&](int v) { return sizeof(T) == 8 ? lk + 4 * v : 4 * lk + v; };
  if (part) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const long m = m0 + wm + 16 * i + row_of(v);
          const long n = n0 + wn + 16 * j + li;
          if (m < M && n < N) part[(long(bz) * N + n) * M + m] = c128{double(cr[i][j][v]), double(ci[i][j][v])};
        }
  } else {
    const double one[2] = {1.0, 1.0};
    epi_blocks<NE>(epi, M, N, m0 + wm, n0 + wn, li, cr, ci, one, row_of);
  }
}

// upper: only the elements of tiles bx <= by (the others' partials were not written)
template <typename EO>
__global__ __launch_bounds__(256) void k_reduce(int M, int N, int splits, const c128* __restrict__ part, Epi<EO> epi,
                                                int upper = 0) {
  const long total = long(M) * N;
  for (long t = blockIdx.x * long(blockDim.x) + threadIdx.x; t < total; t += long(gridDim.x) * blockDim.x) {
    const long n = t / M, m = t - n * M;
    if (upper && m / BM > n / BN) continue;
    double re = 0.0, im = 0.0;
    for (int s = 0; s < splits; ++s) {
      c128 v = part[long(s) * total + t];
      re += v.x;
      im += v.y;
    }
    epi_store(epi, m, n, re, im);
  }
}

// ---- small complex FP64 GEMM ----------------------------------------------------------------------------
// Products with at most a few hundred 16 x 16 output blocks and K of at most a thousand (the projector-space
// matrices of Sec. 5.1 and the subspace matrices of the Rayleigh-Ritz step) fill only a few dozen 64 x 64 tiles:
// the tiled kernel above then runs one wave per SIMD and needs split-K with a second reduction launch. Here one
// block of 4 waves computes one 16 x 16 output block. Wave w takes the w-th quarter of K and reads its operand
// fragments straight from global memory (a few MB that stay in L2), the next load group in flight during the
// MFMAs of the current one; the four partial blocks meet in LDS and are summed in a fixed order, so that the result does not depend on timing.
//
// Within a load group of 16 k, lane (li, lk) holds k = k0 + 4 s + lk for MFMA step s (the instruction's own k
// order): the 4 lanes of one B column (and of one A column for conj(A)^T) read 64 contiguous bytes per load.
constexpr int SKG = 16, SKMAX = 1024, SBLKMAX = 1024, SLD = 17, SW = 4;  // 8 waves per block measured slower
static_assert(SW >= 4, "the epilogue takes one thread per element of the 16 x 16 block");

template <typename EO, int MODE>
__global__ __launch_bounds__(64 * SW) void k_gemm_s(int M, int N, int K, int kchunk, const c128* __restrict__ A,
                                                long lda, const c128* __restrict__ B, long ldb, Epi<EO> epi) {
  __shared__ c128 red[SW][16 * SLD];
  using acc_t = Mfma<double>::acc;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  int bx, by, bz;
  gemm_tile_of(blockIdx.x, gridDim.x, (M + 15) / 16, (N + 15) / 16, 1, bx, by, bz);
  const long m0 = long(bx) * 16, n0 = long(by) * 16;
  // rows of A past M and columns of B past N are read clamped: they feed only output rows and columns that are
  // never stored
  const long amc = min(m0 + li, long(M) - 1), bnc = min(n0 + li, long(N) - 1);
  const c128* __restrict__ Ab = MODE == GEMM_CN ? A + amc * lda : A + amc;
  const long ask = MODE == GEMM_CN ? 1 : lda;  // A stride along k
  const c128* __restrict__ Bb = B + bnc * ldb;
  const int kb = wave * kchunk, ke = min(K, kb + kchunk);
  const int kfull = kb + (max(ke - kb, 0) / SKG) * SKG;  // end of the whole load groups

  acc_t p1, p2, p3;
#pragma unroll
  for (int v = 0; v < 4; ++v) { p1[v] = 0.0; p2[v] = 0.0; p3[v] = 0.0; }

  // whole groups load without conditions (a load under a branch would make the compiler wait for every load
  // in flight before the MFMAs); only the last partial group zeroes k >= ke by value
  c128 a0[4], b0[4], a1[4], b1[4];
  auto load = [&](int k0, c128(&a)[4], c128(&b)[4]) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int k = k0 + 4 * s + lk;
      a[s] = Ab[long(k) * ask];
      b[s] = Bb[k];
    }
  };
  auto load_tail = [&](int k0, c128(&a)[4], c128(&b)[4]) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int k = k0 + 4 * s + lk;
      const bool kok = k < ke;
      const int kc = kok ? k : ke - 1;
      const c128 va = Ab[long(kc) * ask], vb = Bb[kc];
      a[s] = kok ? va : c128{0.0, 0.0};
      b[s] = kok ? vb : c128{0.0, 0.0};
    }
  };
  // P1 = a_r b_r, P2 = a_i b_i, P3 = (a_r + s a_i)(b_r + b_i), s = -1 for conj(a) b
  auto mul = [&](const c128(&a)[4], const c128(&b)[4]) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const double as = MODE == GEMM_CN ? a[s].x - a[s].y : a[s].x + a[s].y;
      p1 = Mfma<double>::run(a[s].x, b[s].x, p1);
      p2 = Mfma<double>::run(a[s].y, b[s].y, p2);
      p3 = Mfma<double>::run(as, b[s].x + b[s].y, p3);
    }
  };
  int k0 = kb;
  if (ke - kb == 4 * SKG) {
    // exactly four whole groups (K = 256 over 4 waves, the projector-space and subspace products): every load of
    // the wave issued before the first MFMA, one memory latency instead of four
    c128 a4[4][4], b4[4][4];
#pragma unroll
    for (int g = 0; g < 4; ++g) load(kb + g * SKG, a4[g], b4[g]);
#pragma unroll
    for (int g = 0; g < 4; ++g) mul(a4[g], b4[g]);
    k0 = ke;
  }
  // otherwise the next group is always requested (clamped to the last whole group, which the final pass reads
  // twice) and rotated into place after the MFMAs of this one: a request under a condition, or one consumed only
  // past a branch, is waited for or moved by the compiler before the MFMAs
  if (k0 < kfull) load(k0, a0, b0);
  for (; k0 < kfull; k0 += SKG) {
    load(min(k0 + SKG, kfull - SKG), a1, b1);
    mul(a0, b0);
#pragma unroll
    for (int s = 0; s < 4; ++s) { a0[s] = a1[s]; b0[s] = b1[s]; }
  }
  if (k0 < ke) {
    load_tail(k0, a0, b0);
    mul(a0, b0);
  }

  // accumulator v of a lane holds row lk + 4 v, column li of the 16 x 16 block
  constexpr double sg = MODE == GEMM_CN ? -1.0 : 1.0;
#pragma unroll
  for (int v = 0; v < 4; ++v)
    red[wave][(lk + 4 * v) + SLD * li] = c128{p1[v] - sg * p2[v], p3[v] - p1[v] - sg * p2[v]};
  __syncthreads();
  if (tid < 256) {
    const int r = tid & 15, c = tid >> 4;
    double re = 0.0, im = 0.0;
#pragma unroll
    for (int w = 0; w < SW; ++w) {
      const c128 x = red[w][r + SLD * c];
      re += x.x;
      im += x.y;
    }
    const long m = m0 + r, n = n0 + c;
    if (m < M && n < N) epi_store(epi, m, n, re, im);
  }
}

// ---- FP16 hi/lo split GEMM ------------------------------------------------------------------------------
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int HBK = 32, HLD = HBK + 8;  // LDS rows of 40 halves (80 bytes): 16-byte aligned, rows spread over banks

__device__ __forceinline__ f4 mfma_h(h8 a, h8 b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0); }
// acc += x * y with x = xh + xl, y = yh + yl, dropping xl * yl
__device__ __forceinline__ f4 mul3(h8 xh, h8 xl, h8 yh, h8 yl, f4 acc) {
  acc = mfma_h(xh, yh, acc);
  acc = mfma_h(xh, yl, acc);
  return mfma_h(xl, yh, acc);
}

// FP16 tiles: TB x TB complex outputs per block (TB = 64: 4 waves, TB = 128: 8 waves), each wave a (16 NI) x 32
// sub-tile of NI x 2 MFMA blocks; the waves form a 2 x (TB / 32) grid. Every thread loads one row (A) and one column
// (B) group of 8 k per K tile of 32, so a block has 4 TB threads. The 128 tiles read each LDS fragment for twice the
// MFMA work of the 64 tiles (a 64 x 32 wave sub-tile against 32 x 32), halving the LDS traffic per product, which
// bounds the 64 tiles on the large projector products.
template <int TB> struct HTile {
  static constexpr int NI = TB / 32, NJ = 2, WM = 2, WN = TB / 32, NT = 64 * WM * WN;
  static_assert(NT == 4 * TB, "one loader row per 4 threads");
};

// The 16x16x32 FP16 MFMA takes, in lane l, row l % 16 of A and column l % 16 of B at k = 8 (l / 16) ...
// 8 (l / 16) + 7, and returns row 4 (l / 16) + v, column l % 16 in accumulator element v.
// BPRE: B arrives as pre-split planes Bp [4][brows][bld] (see split_columns) and is copied to LDS as it is.
template <int TB, typename EB, typename EO, int MODE, int ROLE, int NE, bool BPRE>
__global__ __launch_bounds__(HTile<TB>::NT) void k_gemm_h(int M, int N, int K, int kchunk,
                                                           const _Float16* __restrict__ Ap, long arows, long ald,
                                                           double ainv, const cx<EB>* __restrict__ B, long ldb,
                                                           const _Float16* __restrict__ Bp, long brows, long bld,
                                                           const float* __restrict__ bsc, Epi<EO> epi,
                                                           c128* __restrict__ part, int grp) {
  using HT = HTile<TB>;
  constexpr int NI = HT::NI, NJ = HT::NJ;
  // The 128 tiles (one block per CU) take two LDS stages: tile t is multiplied from one while tile t + 1 is
  // converted and written to the other, so the MFMAs just issued run on while the wave waits for the next tile's
  // loads, and one barrier per tile suffices. The 64 tiles keep one stage and more resident blocks.
  constexpr int NS = TB == 128 ? 2 : 1;
  __shared__ __align__(16) _Float16 As[NS][4][TB][HLD];
  __shared__ __align__(16) _Float16 Bs[NS][4][TB][HLD];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int wm = (wave % HT::WM) * 16 * NI, wn = (wave / HT::WM) * 16 * NJ;
  int bx, by, bz;
  gemm_tile_of(blockIdx.x, gridDim.x, (M + TB - 1) / TB, (N + TB - 1) / TB, grp, bx, by, bz);
  const long m0 = long(bx) * TB, n0 = long(by) * TB;
  const int kbeg = bz * kchunk;
  const int kend = min(K, kbeg + kchunk);

  f4 cr[NI][NJ], ci[NI][NJ];
#pragma unroll
  for (int i = 0; i < NI; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j) { cr[i][j] = f4{0.f, 0.f, 0.f, 0.f}; ci[i][j] = f4{0.f, 0.f, 0.f, 0.f}; }

  // loader roles: TB rows (A) / columns (B) x 4 groups of 8 k per tile, one group per thread
  const int lrow = tid >> 2, lgrp = tid & 3;
  const long gm = m0 + lrow, gn = n0 + lrow;
  const float sc = gn < N ? bsc[gn] : 1.f;
  // raw registers of one K tile (A planes as stored, B in its storage type), converted and split only when
  // written to LDS, so that the loads of the next tile stay in flight during the MFMAs of this one
  h8 ra[4], rb[4];
  cx<EB> vb[8];
  auto load_tile = [&](int k0) {
    const int kk = k0 + 8 * lgrp;
#pragma unroll
    for (int pl = 0; pl < 4; ++pl) {
      h8 v = {};
      if (gm < M) v = *reinterpret_cast<const h8*>(Ap + (pl * arows + gm) * ald + kk);  // K padded to 32: in bounds
      ra[pl] = v;
    }
    if constexpr (BPRE) {
#pragma unroll
      for (int pl = 0; pl < 4; ++pl) {
        h8 v = {};
        if (gn < N) v = *reinterpret_cast<const h8*>(Bp + (pl * brows + gn) * bld + kk);  // padded with zeros
        rb[pl] = v;
      }
    } else {
      const cx<EB>* col = B + (gn < N ? gn : 0) * ldb;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        cx<EB> v = {EB(0), EB(0)};
        if (gn < N && kk + j < kend) v = col[kk + j];
        vb[j] = v;
      }
    }
  };
  auto store_tile = [&](int sg) {
#pragma unroll
    for (int pl = 0; pl < 4; ++pl) *reinterpret_cast<h8*>(&As[sg][pl][lrow][8 * lgrp]) = ra[pl];
    if constexpr (BPRE) {
#pragma unroll
      for (int pl = 0; pl < 4; ++pl) *reinterpret_cast<h8*>(&Bs[sg][pl][lrow][8 * lgrp]) = rb[pl];
      return;
    }
    h8 rh, rl, ih, il;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const float xr = float(vb[j].x * EB(sc)), xi = float(vb[j].y * EB(sc));
      const _Float16 hr = _Float16(xr), hi = _Float16(xi);
      rh[j] = hr;
      ih[j] = hi;
      rl[j] = _Float16(xr - float(hr));
      il[j] = _Float16(xi - float(hi));
    }
    *reinterpret_cast<h8*>(&Bs[sg][0][lrow][8 * lgrp]) = rh;
    *reinterpret_cast<h8*>(&Bs[sg][1][lrow][8 * lgrp]) = rl;
    *reinterpret_cast<h8*>(&Bs[sg][2][lrow][8 * lgrp]) = ih;
    *reinterpret_cast<h8*>(&Bs[sg][3][lrow][8 * lgrp]) = il;
  };

  if (kbeg < kend) {
    load_tile(kbeg);
    store_tile(0);
  }
  __syncthreads();
  int sg = 0;
  for (int k0 = kbeg; k0 < kend; k0 += HBK) {
    const bool more = k0 + HBK < kend;
    if (more) load_tile(k0 + HBK);  // in flight while this tile is multiplied
    h8 b[NJ][4];
#pragma unroll
    for (int j = 0; j < NJ; ++j)
#pragma unroll
      for (int pl = 0; pl < 4; ++pl) b[j][pl] = *reinterpret_cast<const h8*>(&Bs[NS == 2 ? sg : 0][pl][wn + 16 * j + li][8 * lk]);
#pragma unroll
    for (int i = 0; i < NI; ++i) {
      h8 a[4];
#pragma unroll
      for (int pl = 0; pl < 4; ++pl) a[pl] = *reinterpret_cast<const h8*>(&As[NS == 2 ? sg : 0][pl][wm + 16 * i + li][8 * lk]);
      const h8 nih = -a[2], nil = -a[3];
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        cr[i][j] = mul3(a[0], a[1], b[j][0], b[j][1], cr[i][j]);
        ci[i][j] = mul3(a[0], a[1], b[j][2], b[j][3], ci[i][j]);
        if (MODE == GEMM_CN) {  // conj(a) b: re += ar br + ai bi, im += ar bi - ai br
          cr[i][j] = mul3(a[2], a[3], b[j][2], b[j][3], cr[i][j]);
          ci[i][j] = mul3(nih, nil, b[j][0], b[j][1], ci[i][j]);
        } else {  // a b: re += ar br - ai bi, im += ar bi + ai br
          cr[i][j] = mul3(nih, nil, b[j][2], b[j][3], cr[i][j]);
          ci[i][j] = mul3(a[2], a[3], b[j][0], b[j][1], ci[i][j]);
        }
      }
    }
    if constexpr (NS == 2) {
      if (more) store_tile(sg ^ 1);  // that stage was last read before the previous barrier
      __syncthreads();
      sg ^= 1;
    } else {
      __syncthreads();
      if (more) {
        store_tile(0);
        __syncthreads();
      }
    }
  }

  // column scales of the lane's columns (undo the per-band power-of-two scaling of B and the A scale)
  double fs[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const long n = n0 + wn + 16 * j + li;
    fs[j] = n < N ? ainv / double(bsc[n]) : 0.0;
  }
  auto row_of = [&](int v) { return 4 * lk + v; };
  if (part) {
#pragma unroll
    for (int i = 0; i < NI; ++i)
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        const long n = n0 + wn + 16 * j + li;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const long m = m0 + wm + 16 * i + row_of(v);
          if (m < M && n < N)
            part[(long(bz) * N + n) * M + m] = c128{fs[j] * double(cr[i][j][v]), fs[j] * double(ci[i][j][v])};
        }
      }
  } else {
    epi_blocks<NE>(epi, M, N, m0 + wm, n0 + wn, li, cr, ci, fs, row_of);
  }
}

// one 1024-thread block per column (16 waves per CU keep enough loads in flight), max over lanes by shuffles
constexpr int CST = 1024;
template <typename E>
__global__ __launch_bounds__(CST) void k_colscale(long rows, const cx<E>* __restrict__ B, long ldb, float* bsc,
                                                  double* maxout) {
  __shared__ double red[CST / 64];
  const cx<E>* col = B + long(blockIdx.x) * ldb;
  double mx = 0.0;
  for (long i = threadIdx.x; i < rows; i += blockDim.x) {
    const cx<E> v = col[i];
    mx = fmax(mx, fmax(fabs(double(v.x)), fabs(double(v.y))));
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    mx = red[0];
    for (int w = 1; w < CST / 64; ++w) mx = fmax(mx, red[w]);
    if (maxout) maxout[blockIdx.x] = mx;
    if (bsc) {
      int e = 0;
      const bool ok = mx > 0.0 && mx < 1e300;
      if (ok) (void)frexp(mx, &e);  // mx = f 2^e, f in [0.5, 1): the column is scaled to max in [2^13, 2^14)
      bsc[blockIdx.x] = ok ? ldexpf(1.f, min(kHalfTopExp - e, 126)) : 1.f;
    }
  }
}

__global__ void k_split_planes(const c128* __restrict__ X, long ldx, int ksrc, bool transpose, double scale,
                               _Float16* __restrict__ P, long prow, long pld) {
  const long total = prow * pld;
  for (long t = blockIdx.x * long(blockDim.x) + threadIdx.x; t < total; t += long(gridDim.x) * blockDim.x) {
    const long r = t / pld, k = t - r * pld;
    c128 v = {0.0, 0.0};
    if (k < ksrc) v = transpose ? X[r + k * ldx] : X[k + r * ldx];
    const double xr = v.x * scale, xi = v.y * scale;
    const _Float16 hr = _Float16(float(xr)), hi = _Float16(float(xi));
    P[t] = hr;
    P[total + t] = _Float16(float(xr - double(float(hr))));
    P[2 * total + t] = hi;
    P[3 * total + t] = _Float16(float(xi - double(float(hi))));
  }
}

template <typename E>
__global__ void k_split_columns(int K, int N, const cx<E>* __restrict__ B, long ldb, const float* __restrict__ bsc,
                                _Float16* __restrict__ P, long pld) {
  const long total = long(N) * pld;
  for (long t = blockIdx.x * long(blockDim.x) + threadIdx.x; t < total; t += long(gridDim.x) * blockDim.x) {
    const long n = t / pld, k = t - n * pld;
    cx<E> v = {E(0), E(0)};
    if (k < K) v = B[k + n * ldb];
    const E sc = E(bsc[n]);  // the same operations as the on-the-fly split in k_gemm_h
    const float xr = float(v.x * sc), xi = float(v.y * sc);
    const _Float16 hr = _Float16(xr), hi = _Float16(xi);
    P[t] = hr;
    P[total + t] = _Float16(xr - float(hr));
    P[2 * total + t] = hi;
    P[3 * total + t] = _Float16(xi - float(hi));
  }
}

}  // namespace

// Split count that minimises the rounds of resident blocks per unit of K work, ceil(tiles s / slots) / s, over
// s in [1, smax] (the smallest such s): a launch of tiles slightly above a multiple of the resident blocks
// otherwise leaves most of the GPU idle in its last round.
long quantized_splits(long tiles, long slots, long smax, long smin = 1) {
  if (smin < 1) smin = 1;
  if (smax < smin) smax = smin;
  long best = smin;
  double cost = double((tiles * smin + slots - 1) / slots) / double(smin);
  for (long s = smin + 1; s <= smax; ++s) {
    const double c = double((tiles * s + slots - 1) / slots) / double(s);
    if (c < cost - 1e-12) { cost = c; best = s; }
  }
  return best;
}

int gemm_pick_splits(int M, int N, int K) {
  if (M <= 0 || N <= 0 || K <= 0) return 1;
  const long tiles = long((M + BM - 1) / BM) * ((N + BN - 1) / BN);
  const long kblocks = (K + BK - 1) / BK;
  long smax = std::min<long>(32, kblocks / 2);  // at least two K tiles per split
  if (smax < 1) smax = 1;
  long s;
  if (tiles < 256) {
    // about one block per CU: measured on the paw48 projector shapes, the tall NN products (448 tiles) run best
    // without split-K and the 256 x 256 x 7153 reductions with 16 splits (28 and 56 slower)
    s = std::min((256 + tiles - 1) / tiles, smax);
  } else {
    // two resident blocks per CU on 256 CUs (the 3328 x 2048 x 137065 projection: 1664 tiles, 4 splits)
    s = quantized_splits(tiles, 512, std::min<long>(smax, 8));
  }
  return int(std::max<long>(s, 1));
}

template <typename T, typename EA, typename EB, typename EO>
hipError_t gemm(GemmMode mode, int M, int N, int K, const cx<EA>* A, long lda, const cx<EB>* B, long ldb,
                const Epi<EO>& epi, int splits, c128* part, hipStream_t st, GemmRole role, bool upper) {
  if (M <= 0 || N <= 0) return hipSuccess;
  if (upper && M != N) return hipErrorInvalidValue;
  if constexpr (std::is_same<T, double>::value && std::is_same<EA, double>::value && std::is_same<EB, double>::value) {
    const long blocks = long((M + 15) / 16) * ((N + 15) / 16);
    if (K <= SKMAX && blocks <= SBLKMAX) {  // splits and part are not used
      int kc = (std::max(K, 0) + SW - 1) / SW;
      kc = std::max(SKG, ((kc + SKG - 1) / SKG) * SKG);
      if (mode == GEMM_CN)
        hipLaunchKernelGGL((k_gemm_s<EO, GEMM_CN>), dim3(unsigned(blocks)), dim3(64 * SW), 0, st, M, N, K, kc, A, lda, B,
                           ldb, epi);
      else
        hipLaunchKernelGGL((k_gemm_s<EO, GEMM_NN>), dim3(unsigned(blocks)), dim3(64 * SW), 0, st, M, N, K, kc, A, lda, B,
                           ldb, epi);
      return hipGetLastError();
    }
  }
  if (splits < 1) splits = 1;
  int kchunk = (K + splits - 1) / splits;
  kchunk = ((kchunk + BK - 1) / BK) * BK;
  if (kchunk < BK) kchunk = BK;
  splits = K > 0 ? (K + kchunk - 1) / kchunk : 1;
  const bool use_part = splits > 1;
  if (use_part && !part) return hipErrorInvalidValue;
  const long tm = (M + BM - 1) / BM;
  dim3 grid(unsigned((upper ? tm * (tm + 1) / 2 : tm * ((N + BN - 1) / BN)) * splits));
  const int grp = upper ? kUpperTiles : tile_group(M, K);
  c128* pp = use_part ? part : nullptr;
  Epi<EO> en = epi;
  const int ne = epi_slots(en);
  auto launch = [&](auto modec, auto rolec) {
    constexpr int MO = decltype(modec)::value, RO = decltype(rolec)::value;
    if (ne == 0 || use_part)
      hipLaunchKernelGGL((k_gemm<T, EA, EB, EO, MO, RO, 0>), grid, dim3(NT), 0, st, M, N, K, kchunk, A, lda, B, ldb, en, pp,
                         grp);
    else if (ne == 1)
      hipLaunchKernelGGL((k_gemm<T, EA, EB, EO, MO, RO, 1>), grid, dim3(NT), 0, st, M, N, K, kchunk, A, lda, B, ldb, en, pp,
                         grp);
    else
      hipLaunchKernelGGL((k_gemm<T, EA, EB, EO, MO, RO, 3>), grid, dim3(NT), 0, st, M, N, K, kchunk, A, lda, B, ldb, en, pp,
                         grp);
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
  hipLaunchKernelGGL((k_reduce<EO>), dim3(blocks), dim3(256), 0, st, M, N, splits, part, epi, upper ? 1 : 0);
  return hipGetLastError();
}

// split count of an upper-triangle product (tm (tm + 1) / 2 tiles): the fewest rounds of 512 resident blocks per
// unit of K work, at most 8 splits and two K tiles per split
int gemm_upper_splits(int N, int K) {
  if (N <= 0 || K <= 0) return 1;
  const long tm = (N + BM - 1) / BM;
  const long kblocks = (K + BK - 1) / BK;
  const long smax = std::max<long>(1, std::min<long>(8, kblocks / 2));
  return int(quantized_splits(tm * (tm + 1) / 2, 512, smax));
}

__global__ void k_hermitian_lower(int n, c128* __restrict__ A, long lda) {
  const long total = long(n) * n;
  for (long t = blockIdx.x * long(blockDim.x) + threadIdx.x; t < total; t += long(gridDim.x) * blockDim.x) {
    const long j = t / n, i = t - j * n;
    if (i > j) {
      const c128 v = A[j + i * lda];
      A[i + j * lda] = c128{v.x, -v.y};
    }
  }
}

hipError_t hermitian_lower(int n, c128* A, long lda, hipStream_t st) {
  if (n <= 1) return hipSuccess;
  const long total = long(n) * n;
  const int blocks = int(std::min<long>((total + 255) / 256, 4096));
  hipLaunchKernelGGL(k_hermitian_lower, dim3(blocks), dim3(256), 0, st, n, A, lda);
  return hipGetLastError();
}

void gemm_block_item(int i, int total, int tm, int tn, int grp, int& bx, int& by, int& bz) {
  gemm_tile_of(i, total, tm, tn, grp, bx, by, bz);
}

// upper bound of the split counts any GEMM kernel here picks for an M x N x K product (partial-buffer sizing):
// 512 target blocks, two K tiles of 32 per split, at most 32 splits; gemm_pick_splits and gemm_h_pick_splits
// never exceed it
int gemm_split_bound(int M, int N, int K) {
  if (M <= 0 || N <= 0 || K <= 0) return 1;
  const long tiles = long((M + BM - 1) / BM) * ((N + BN - 1) / BN);
  long s = (512 + tiles - 1) / tiles;
  const long kblocks = (K + BK - 1) / BK;
  if (s > kblocks / 2) s = kblocks / 2;
  if (s > 32) s = 32;
  if (s < 1) s = 1;
  return int(std::max<long>(s, std::max(gemm_pick_splits(M, N, K), gemm_h_pick_splits(M, N, K))));
}

// Tile and split-K count of the FP16 split GEMM. The FP32 accumulators of one split sum K / splits products in
// sequence, and their rounding error grows like eps32 sqrt(K / splits): long reductions (the projections P^H x over
// all plane waves) are split into chunks of at most kHalfChunk, summed in FP64 by the reduction (at K = 57777 in one
// chunk the error set a residual floor of the mixed outer loop near 1e-5). The 128 tiles (one block of 8 waves per
// CU) are used when the launch fills at least one round of resident blocks, with the split count that wastes least
// of the last round; else the 64 tiles with about one block per CU (measured best on the paw48 shapes, where the
// 512-block target was 5% slower on the 256 x 256 x 7153 projection: twice the partial traffic).
// allow_split = false: one split (the caller bounds K).
constexpr long kHalfChunk = 4096;

void h_plan(int M, int N, int K, bool allow_split, int* tb, int* splits) {
  const long kblocks = (K + HBK - 1) / HBK;
  const long smin = allow_split ? (K + kHalfChunk - 1) / kHalfChunk : 1;
  long smax = allow_split ? std::max<long>(std::min<long>(64, kblocks / 2), smin) : 1;
  const long t128 = long((M + 127) / 128) * ((N + 127) / 128);
  // at least 16 K tiles per split of the 128 tiles, whose prologue and epilogue are long
  const long smax128 = std::max(std::min(smax, kblocks / 16), smin);
  const long s128 = quantized_splits(t128, 256, smax128, smin);
  if (t128 * s128 >= 256) {
    *tb = 128;
    *splits = int(s128);
    return;
  }
  const long tiles = long((M + 63) / 64) * ((N + 63) / 64);
  long s = (256 + tiles - 1) / tiles;
  s = std::max(std::min(s, smax), smin);
  *tb = 64;
  *splits = int(std::max<long>(s, 1));
}

int gemm_h_pick_splits(int M, int N, int K) {
  if (M <= 0 || N <= 0 || K <= 0) return 1;
  int tb = 64, s = 1;
  h_plan(M, N, K, true, &tb, &s);
  return s;
}

template <typename EB, typename EO>
hipError_t gemm_h(GemmMode mode, int M, int N, int K, const HalfPlanes& A, const cx<EB>* B, long ldb,
                  const float* bscale, const Epi<EO>& epi, int splits, c128* part, hipStream_t st, GemmRole role) {
  if (M <= 0 || N <= 0) return hipSuccess;
  if (!A.p || A.rows < M || A.ld % HBK || A.ld < ((K + HBK - 1) / HBK) * HBK) return hipErrorInvalidValue;
  int tb = 64, planned = 1;
  h_plan(M, N, K, true, &tb, &planned);
  if (splits < 1) splits = 1;
  int kchunk = (K + splits - 1) / splits;
  kchunk = ((kchunk + HBK - 1) / HBK) * HBK;
  if (kchunk < HBK) kchunk = HBK;
  splits = K > 0 ? (K + kchunk - 1) / kchunk : 1;
  const bool use_part = splits > 1;
  if (use_part && !part) return hipErrorInvalidValue;
  c128* pp = use_part ? part : nullptr;
  Epi<EO> en = epi;
  const int ne = epi_slots(en);
  const _Float16* nb16 = nullptr;
  auto launch = [&](auto tbc, auto modec, auto rolec) {
    constexpr int T = decltype(tbc)::value, MO = decltype(modec)::value, RO = decltype(rolec)::value;
    const dim3 grid(((M + T - 1) / T) * ((N + T - 1) / T) * splits), block(HTile<T>::NT);
    const int grp = tile_group(M, K);
    if (ne == 0 || use_part)
      hipLaunchKernelGGL((k_gemm_h<T, EB, EO, MO, RO, 0, false>), grid, block, 0, st, M, N, K, kchunk, A.p, A.rows,
                         A.ld, A.inv_scale, B, ldb, nb16, 0L, 0L, bscale, en, pp, grp);
    else if (ne == 1)
      hipLaunchKernelGGL((k_gemm_h<T, EB, EO, MO, RO, 1, false>), grid, block, 0, st, M, N, K, kchunk, A.p, A.rows,
                         A.ld, A.inv_scale, B, ldb, nb16, 0L, 0L, bscale, en, pp, grp);
    else
      hipLaunchKernelGGL((k_gemm_h<T, EB, EO, MO, RO, 3, false>), grid, block, 0, st, M, N, K, kchunk, A.p, A.rows,
                         A.ld, A.inv_scale, B, ldb, nb16, 0L, 0L, bscale, en, pp, grp);
  };
  using CN = std::integral_constant<int, GEMM_CN>;
  using NNm = std::integral_constant<int, GEMM_NN>;
  using R1 = std::integral_constant<int, 1>;
  using R2 = std::integral_constant<int, 2>;
  auto by_tile = [&](auto modec, auto rolec) {
    if (tb == 128) launch(std::integral_constant<int, 128>{}, modec, rolec);
    else launch(std::integral_constant<int, 64>{}, modec, rolec);
  };
  if (role == ROLE_BACKPROJECT) mode == GEMM_CN ? by_tile(CN{}, R2{}) : by_tile(NNm{}, R2{});
  else mode == GEMM_CN ? by_tile(CN{}, R1{}) : by_tile(NNm{}, R1{});
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !use_part) return e;
  const long total = long(M) * N;
  int blocks = int((total + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL((k_reduce<EO>), dim3(blocks), dim3(256), 0, st, M, N, splits, part, epi);
  return hipGetLastError();
}

template <typename E>
hipError_t split_columns_t(int K, int N, const cx<E>* B, long ldb, const float* bscale, _Float16* planes, long pld,
                           hipStream_t st) {
  if (N <= 0) return hipSuccess;
  if (K < 0 || pld < K || pld % HBK || ldb < K) return hipErrorInvalidValue;
  const long total = long(N) * pld;
  const long blocks = std::min<long>((total + 255) / 256, 65536);
  hipLaunchKernelGGL((k_split_columns<E>), dim3(unsigned(blocks)), dim3(256), 0, st, K, N, B, ldb, bscale, planes,
                     pld);
  return hipGetLastError();
}
hipError_t split_columns(int K, int N, const c128* B, long ldb, const float* bscale, _Float16* planes, long pld,
                         hipStream_t st) {
  return split_columns_t<double>(K, N, B, ldb, bscale, planes, pld, st);
}
hipError_t split_columns(int K, int N, const c64* B, long ldb, const float* bscale, _Float16* planes, long pld,
                         hipStream_t st) {
  return split_columns_t<float>(K, N, B, ldb, bscale, planes, pld, st);
}

template <typename EO>
hipError_t gemm_h_pre(GemmMode mode, int M, int N, int K, const HalfPlanes& A, const HalfPlanes& Bp,
                      const float* bscale, const Epi<EO>& epi, int splits, c128* part, hipStream_t st, GemmRole role) {
  if (M <= 0 || N <= 0) return hipSuccess;
  const long kp = ((std::max(K, 0) + HBK - 1) / HBK) * HBK;
  if (!A.p || A.rows < M || A.ld % HBK || A.ld < kp) return hipErrorInvalidValue;
  if (!Bp.p || Bp.rows != N || Bp.ld % HBK || Bp.ld < kp) return hipErrorInvalidValue;
  int tb = 64, s = 1;
  h_plan(M, N, K, splits > 1, &tb, &s);
  if (splits < 1) splits = 1;
  int kchunk = (K + splits - 1) / splits;
  kchunk = ((kchunk + HBK - 1) / HBK) * HBK;
  if (kchunk < HBK) kchunk = HBK;
  splits = K > 0 ? (K + kchunk - 1) / kchunk : 1;
  const bool use_part = splits > 1;
  if (use_part && !part) return hipErrorInvalidValue;
  Epi<EO> en = epi;
  const int ne = epi_slots(en);
  const cx<double>* nb64 = nullptr;
  c128* np = use_part ? part : nullptr;
  auto launch = [&](auto tbc, auto modec, auto rolec) {
    constexpr int T = decltype(tbc)::value, MO = decltype(modec)::value, RO = decltype(rolec)::value;
    const dim3 grid(((M + T - 1) / T) * ((N + T - 1) / T) * splits), block(HTile<T>::NT);
    const int grp = tile_group(M, K);
    if (ne == 0 || use_part)
      hipLaunchKernelGGL((k_gemm_h<T, double, EO, MO, RO, 0, true>), grid, block, 0, st, M, N, K, kchunk, A.p,
                         A.rows, A.ld, A.inv_scale, nb64, 0L, Bp.p, Bp.rows, Bp.ld, bscale, en, np, grp);
    else if (ne == 1)
      hipLaunchKernelGGL((k_gemm_h<T, double, EO, MO, RO, 1, true>), grid, block, 0, st, M, N, K, kchunk, A.p,
                         A.rows, A.ld, A.inv_scale, nb64, 0L, Bp.p, Bp.rows, Bp.ld, bscale, en, np, grp);
    else
      hipLaunchKernelGGL((k_gemm_h<T, double, EO, MO, RO, 3, true>), grid, block, 0, st, M, N, K, kchunk, A.p,
                         A.rows, A.ld, A.inv_scale, nb64, 0L, Bp.p, Bp.rows, Bp.ld, bscale, en, np, grp);
  };
  using CN = std::integral_constant<int, GEMM_CN>;
  using NNm = std::integral_constant<int, GEMM_NN>;
  using R1 = std::integral_constant<int, 1>;
  using R2 = std::integral_constant<int, 2>;
  auto by_tile = [&](auto modec, auto rolec) {
    if (tb == 128) launch(std::integral_constant<int, 128>{}, modec, rolec);
    else launch(std::integral_constant<int, 64>{}, modec, rolec);
  };
  if (role == ROLE_BACKPROJECT) mode == GEMM_CN ? by_tile(CN{}, R2{}) : by_tile(NNm{}, R2{});
  else mode == GEMM_CN ? by_tile(CN{}, R1{}) : by_tile(NNm{}, R1{});
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !use_part) return e;
  const long total = long(M) * N;
  int blocks = int((total + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL((k_reduce<EO>), dim3(blocks), dim3(256), 0, st, M, N, splits, part, epi);
  return hipGetLastError();
}

template <typename E>
hipError_t column_scales(long rows, int ncols, const cx<E>* B, long ldb, float* bscale, hipStream_t st) {
  if (ncols <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_colscale<E>), dim3(ncols), dim3(CST), 0, st, rows, B, ldb, bscale, nullptr);
  return hipGetLastError();
}

hipError_t column_maxabs(long rows, int ncols, const c128* X, long ldx, double* out, hipStream_t st) {
  if (ncols <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_colscale<double>), dim3(ncols), dim3(CST), 0, st, rows, X, ldx, nullptr, out);
  return hipGetLastError();
}

hipError_t split_planes(const c128* X, long ldx, int rows_x, int cols_x, bool transpose, double scale,
                        _Float16* planes, long prow, long pld, hipStream_t st) {
  const int ksrc = transpose ? cols_x : rows_x;
  if (prow != (transpose ? rows_x : cols_x) || pld < ksrc) return hipErrorInvalidValue;
  const long total = prow * pld;
  if (total <= 0) return hipSuccess;
  const long blocks = std::min<long>((total + 255) / 256, 65536);
  hipLaunchKernelGGL(k_split_planes, dim3(unsigned(blocks)), dim3(256), 0, st, X, ldx, ksrc, transpose, scale, planes,
                     prow, pld);
  return hipGetLastError();
}

template hipError_t gemm_h<float, float>(GemmMode, int, int, int, const HalfPlanes&, const c64*, long, const float*,
                                         const Epi<float>&, int, c128*, hipStream_t, GemmRole);
template hipError_t gemm_h<float, double>(GemmMode, int, int, int, const HalfPlanes&, const c64*, long, const float*,
                                          const Epi<double>&, int, c128*, hipStream_t, GemmRole);
template hipError_t gemm_h<double, float>(GemmMode, int, int, int, const HalfPlanes&, const c128*, long,
                                          const float*, const Epi<float>&, int, c128*, hipStream_t, GemmRole);
template hipError_t gemm_h_pre<float>(GemmMode, int, int, int, const HalfPlanes&, const HalfPlanes&, const float*,
                                       const Epi<float>&, int, c128*, hipStream_t, GemmRole);
template hipError_t gemm_h_pre<double>(GemmMode, int, int, int, const HalfPlanes&, const HalfPlanes&, const float*,
                                        const Epi<double>&, int, c128*, hipStream_t, GemmRole);
template hipError_t column_scales<float>(long, int, const c64*, long, float*, hipStream_t);
template hipError_t column_scales<double>(long, int, const c128*, long, float*, hipStream_t);

#define INST(T, EA, EB, EO)                                                                               \
  template hipError_t gemm<T, EA, EB, EO>(GemmMode, int, int, int, const cx<EA>*, long, const cx<EB>*, long, \
                                          const Epi<EO>&, int, c128*, hipStream_t, GemmRole, bool);
INST(double, double, double, double)
INST(float, float, float, float)
INST(float, float, double, float)
INST(float, float, float, double)
INST(double, float, float, double)
INST(double, float, double, float)
#undef INST

}  // namespace chebfd
