// V_loc psi by a pair of pruned 3D FFTs (Sec. 2.1, Alg. 1), fused with the kinetic diagonal.
//
// A band's sphere coefficients only touch the "disk" columns (gx, gy) with gx^2 + gy^2 <= R^2 and, in
// each z-plane, only the x-lines |gx| <= R. The box transform is therefore split into three passes:
//   column pass   : sphere -> z-lines of the disk columns, inverse FFT along z          (fft_col_inverse)
//   plane pass    : per z-plane, inverse y on the 2R+1 x-lines, then per row inverse x, multiply by
//                   V(r), forward x, keep the 2R+1 x-lines, forward y                      (fft_plane)
//   column pass   : forward FFT along z, gather the sphere, scale by n^-3, add K psi      (fft_col_forward)
// The disk-column buffer is laid out [band][z][column] so that plane passes read and write it
// contiguously and column passes stage z-lines of CPB columns in LDS.
#include <algorithm>

#include "fft.h"
#include "kernels.h"

namespace chebfd {
namespace {

constexpr int NT = 256;

// In LDS a line is kept as N1 groups of N2 points with one pad slot per group (group a starts at PS a,
// PS = N2 + 1) and an odd line stride, so that lanes walking groups and lanes walking lines both spread
// over the LDS banks.
template <int N> constexpr int group_stride() { return LineSplit<N>::N2 + 1; }
template <int N> constexpr int line_stride() { return (LineSplit<N>::N1 * group_stride<N>()) | 1; }

// columns per block of the column passes: 16 (FP64) or 32 (FP32) on the small boxes; from 96^3 up, 8 or 16 (more,
// smaller blocks: at 128^3 the FP32 passes took 43.3 / 55.1 us per 30-band launch with 32 and 36.7 / 39.6 with 16,
// the FP64 forward pass 35.7 against 34.3 us; at 48^3 the smaller blocks were slower)
template <int N, typename T> constexpr int cpb() { return N >= 96 ? (sizeof(T) == 8 ? 8 : 16) : (sizeof(T) == 8 ? 16 : 32); }

template <int N, typename T>
__global__ __launch_bounds__(NT) void k_col_inv(int ncol, const int4* __restrict__ col, const int* __restrict__ ent,
                                                const cx<T>* __restrict__ twg, const cx<T>* __restrict__ X, long ldx,
                                                cx<T>* __restrict__ colbuf) {
  constexpr int CPB = cpb<N, T>(), LS = line_stride<N>();
  __shared__ cx<T> lines[CPB * LS];
  __shared__ cx<T> twA[N];
  const int band = blockIdx.y;
  const int c0 = blockIdx.x * CPB, c1 = min(ncol, c0 + CPB), nc = c1 - c0;
  const int tid = threadIdx.x;
  for (int t = tid; t < N; t += NT) twA[t] = twg[((t % LineSplit<N>::N2) * (t / LineSplit<N>::N2)) % N];
  for (int t = tid; t < CPB * LS; t += NT) lines[t] = cx<T>{T(0), T(0)};
  __syncthreads();
  const int e0 = col[c0].z, e1 = col[c1 - 1].z + col[c1 - 1].w;
  const cx<T>* xb = X + long(band) * ldx;
  for (int e = e0 + tid; e < e1; e += NT) {
    const int code = ent[e];
    lines[((code >> 8) - c0) * LS + (code & 255)] = xb[e];
  }
  __syncthreads();
  lds_fft<N, +1, T>(lines, nc, LS, twA);
  const long cs = col_stride(ncol);
  cx<T>* out = colbuf + long(band) * N * cs;
  for (int t = tid; t < N * nc; t += NT) {
    const int z = t / nc, c = t - z * nc;
    out[long(z) * cs + c0 + c] = lines[c * LS + z];
  }
}

// Rows of the old block-synchronous x-pass, kept for the cross-density kernel of the adjoint: about one task per
// thread in the first stage, and the N = 128 double-precision plane inside 160 KB of LDS.
template <int N, typename T> constexpr int xdens_rows() {
  constexpr int N2 = LineSplit<N>::N2;
  constexpr int r = (N == 128 && sizeof(T) == 8) ? 4 : NT / N2;
  return r < N ? r : N;
}

// Inter-stage twiddles laid out for the lanes that use them: twA[k1 N2 + n2] = W_N^(n2 k1) is read by lanes of
// consecutive n2, twB[kb N1 + a] = W_N^(a kb) by lanes of consecutive a (forward sign; conjugate for inverse).
template <int N, typename T> __device__ __forceinline__ void stage_twiddles(const cx<T>* tw, cx<T>* twA, cx<T>* twB) {
  constexpr int N1 = LineSplit<N>::N1, N2 = LineSplit<N>::N2;
  for (int t = threadIdx.x; t < N; t += NT) {
    const int k1 = t / N2, n2 = t - k1 * N2;
    twA[t] = tw[(n2 * k1) % N];
    const int kb = t / N1, a = t - kb * N1;
    twB[t] = tw[(a * kb) % N];
  }
}
template <typename T> __device__ __forceinline__ cx<T> conj_if(cx<T> w, bool c) { return c ? cx<T>{w.x, -w.y} : w; }

// signed frequency of FFT index k (|result| <= (N-1)/2 for the indices the sphere uses)
template <int N> __device__ __forceinline__ int freq(int k) { return k <= (N - 1) / 2 ? k : k - N; }

// compute units of the current device (queried once per device)
int compute_units() {
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
  if (cached[dev] <= 0) {
    int cu = 0;
    if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cu <= 0) cu = 256;
    cached[dev] = cu;
  }
  return cached[dev];
}

// Orders the LDS accesses of one wave: every lane sees the LDS writes the wave issued before it. A wave's LDS
// instructions execute in order, so only the compiler has to be kept from moving accesses across it.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---- plane pass -------------------------------------------------------------------------------------------------
// One (z-plane, band) item at a time per block (a persistent grid walks the items). With N = N1 N2, every length-N
// transform is two register codelets around one exchange through LDS, and every exchange stays inside one wave:
// a wave owns whole x-lines in stages A and C and whole rows in stage B, so the only block-wide barriers are the
// three between the stages.
//   A  inverse y on the 2R+1 x-lines, read straight from the disk-column row of this plane. An x-line is kept in
//      LDS as N1 groups of N2 points, group a holding y = a + N1 b at slot b (one pad slot per group and an odd
//      line stride spread the lanes of an exchange over the banks).
//   B  per row y (dealt to the waves RPW rows at a time, each wave with its own row buffers): inverse x from the
//      2R+1 nonzero x-lines, then in registers the second inverse stage, V(r), the first forward stage; one more
//      exchange; the last forward stage writes the 2R+1 kept x-lines back in place.
//   C  forward y, written straight to the disk-column row of the output.
// Each lane keeps one task per sub-stage for the whole launch (lane -> (line or row, digit)), so its inter-stage
// twiddles are loaded once into registers: W_N^(-n2 k1) of the inverse stages (n2 = lane mod N2) and W_N^(a kb)
// of the forward ones (a = lane mod N1).
template <int N, typename T> struct PlaneCfg {
  static constexpr int N1 = LineSplit<N>::N1, N2 = LineSplit<N>::N2;
  static constexpr int PS = N2 + 1, LS = (N1 * PS) | 1;
  static constexpr int GL = 64 / N2;                 // x-lines per wave in stages A and C
  // waves per block and rows per wave and pass in stage B (at most one stage-1 task per lane). The large boxes
  // hold one block per CU (the plane of y-lines fills most of the LDS: 65 x-lines of 137 slots at N = 128), so they
  // take 8 waves, two per SIMD, where the row buffers fit; the FP64 N = 128 plane leaves room for 8 row buffers,
  // taken by 4 waves of 2 rows (more waves of fewer rows would issue the same instructions for fewer lanes). The
  // smaller boxes keep 4 waves: more blocks per CU, each an independent item, hide more latency than more waves
  // per item (6 waves at N = 48 measured 45% slower). Rows per pass: 96 = 3 x 8 x 4, 128 = 16 x 4 x 2 (FP64)
  // or 4 x 8 x 4 (FP32).
  static constexpr int NW = N == 128 ? (sizeof(T) == 8 ? 4 : 8) : (N == 96 ? 8 : 4);
  static constexpr int RPW0 = N == 128 ? (sizeof(T) == 8 ? 2 : 4) : (N == 96 ? 4 : GL);
  static constexpr int RPW = RPW0 * NW > N ? (N + NW - 1) / NW : RPW0;
  // loads one step ahead (see k_plane) where the LDS holds a single block per CU anyway; elsewhere the extra
  // registers would cost resident blocks
  static constexpr bool PF = N == 128 || (N == 96 && sizeof(T) == 8);
  static_assert(GL * N2 <= 64 && GL * N1 <= 64 && RPW <= GL, "one task per lane in every sub-stage");
};

// bytes of the y-lines and row buffers, then the x-line table at the next 16-byte boundary
template <int N, typename T> constexpr size_t plane_lines_bytes(int nx) {
  using P = PlaneCfg<N, T>;
  return ((size_t(nx + P::NW * P::RPW) * P::LS * sizeof(cx<T>)) + 15) / 16 * 16;
}
template <int N, typename T> constexpr size_t plane_lds(int nx) { return plane_lines_bytes<N, T>(nx) + size_t(nx) * 16; }

template <int N, typename T>
__global__ __launch_bounds__((64 * PlaneCfg<N, T>::NW)) void k_plane(int ncol, int rx, const int4* __restrict__ xline,
                                                                   const cx<T>* __restrict__ twg,
                                                                   const T* __restrict__ Vt,
                                                                   const cx<T>* __restrict__ cin,
                                                                   cx<T>* __restrict__ cout, int nitems) {
  using P = PlaneCfg<N, T>;
  constexpr int N1 = P::N1, N2 = P::N2, PS = P::PS, LS = P::LS, NW = P::NW, GL = P::GL, RPW = P::RPW;
  extern __shared__ unsigned char smem_raw[];
  const int nx = 2 * rx + 1;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  cx<T>* L = reinterpret_cast<cx<T>*>(smem_raw);  // [nx][LS] y-lines of the x-lines |gx| <= rx
  cx<T>* Rw = L + nx * LS + wave * RPW * LS;       // this wave's [RPW][LS] row buffers
  int4* XL = reinterpret_cast<int4*>(smem_raw + plane_lines_bytes<N, T>(nx));  // the x-line table
  const cx<T> zero = {T(0), T(0)};
  for (int t = threadIdx.x; t < nx; t += blockDim.x) XL[t] = xline[t];

  // static lane tasks: digit n2 (stage 1 of an inverse transform, stage 2 of a forward one) and digit a
  const int u2 = lane / N2, n2 = lane - u2 * N2;  // (line or row, n2 / kb)
  const int u1 = lane / N1, a1 = lane - u1 * N1;  // (line or row, k1 / a)
  cx<T> twi[N1], twf[N2];
#pragma unroll
  for (int k = 1; k < N1; ++k) {
    const cx<T> w = twg[(n2 * k) % N];
    twi[k] = cx<T>{w.x, -w.y};
  }
#pragma unroll
  for (int k = 1; k < N2; ++k) twf[k] = twg[(a1 * k) % N];
  const int ngroups = (nx + GL - 1) / GL;
  __syncthreads();

  // With PF, loads are issued one step ahead of their use and kept raw (the zero padding is selected at the use,
  // since a select right after the load would wait for it): the stage-A inputs of the next group (of the next
  // item's first group during stage C), and V(r) of the next row pass (of the first pass at the start of the item).
  // Indices past the end are clamped to valid elements whose values are never used. Without PF, each group and
  // pass loads its own inputs first.
  cx<T> araw[N1];
  int aly = 0, alz = 0;  // lowest gy and column count of the prefetched x-line
  auto load_a = [&](const cx<T>* src, int g) {
    const int xi = min(g * GL + u2, nx - 1);
    const int4 xl = XL[xi];  // {first column, lowest gy, column count, 0}
    aly = xl.y;
    alz = xl.z;
#pragma unroll
    for (int n1 = 0; n1 < N1; ++n1) {
      const int j = freq<N>(N2 * n1 + n2) - xl.y;
      araw[n1] = src[xl.x + ((j >= 0 && j < xl.z) ? j : 0)];
    }
  };
  T vr[N2];
  auto load_v = [&](const T* Vz, int y0) {
    const T* Vrow = Vz + long(min(y0 + u1, N - 1)) * N + a1;
#pragma unroll
    for (int b = 0; b < N2; ++b) vr[b] = Vrow[N1 * b];
  };
  const long cs = col_stride(ncol);
  auto item_base = [&](int item) { return long(item / N) * N * cs + long(item % N) * cs; };

  if (P::PF && int(blockIdx.x) < nitems) load_a(cin + item_base(blockIdx.x), wave);
  for (int item = blockIdx.x; item < nitems; item += gridDim.x) {
    const int z = item % N;
    const long base = item_base(item);
    const cx<T>* in = cin + base;
    cx<T>* out = cout + base;
    const T* Vz = Vt + long(z) * N * N;
    if constexpr (P::PF) load_v(Vz, wave * RPW);

    // ---- A: inverse y ----
    for (int g = wave; g < ngroups; g += NW) {
      {
        const int xi = g * GL + u2;
        const bool mine = u2 < GL && xi < nx;
        if constexpr (!P::PF) load_a(in, g);
        cx<T> v[N1];
#pragma unroll
        for (int n1 = 0; n1 < N1; ++n1) {
          const int j = freq<N>(N2 * n1 + n2) - aly;
          v[n1] = (j >= 0 && j < alz) ? araw[n1] : zero;
        }
        if constexpr (P::PF) load_a(in, min(g + NW, ngroups - 1));
        if (mine) {
          Dft<N1, +1>::run(v);
          cx<T>* p = L + xi * LS + n2;
#pragma unroll
          for (int k1 = 0; k1 < N1; ++k1) p[PS * k1] = k1 ? cmul(v[k1], twi[k1]) : v[0];
        }
      }
      wave_sync();
      {
        const int xi = g * GL + u1;
        if (u1 < GL && xi < nx) {
          cx<T>* p = L + xi * LS + PS * a1;
          cx<T> v[N2];
#pragma unroll
          for (int b = 0; b < N2; ++b) v[b] = p[b];
          Dft<N2, +1>::run(v);
#pragma unroll
          for (int b = 0; b < N2; ++b) p[b] = v[b];  // y = a1 + N1 b
        }
      }
    }
    __syncthreads();

    // ---- B: x-pass, RPW rows per wave at a time ----
    for (int y0 = wave * RPW; y0 < N; y0 += NW * RPW) {
      const int nrow = min(RPW, N - y0);
      const bool has2 = u1 < nrow;
      if constexpr (!P::PF) load_v(Vz, y0);  // requested before stage 1 so that the latency is hidden
      if (u2 < nrow) {
        const int y = y0 + u2, py = PS * (y % N1) + y / N1;
        cx<T> v[N1];
#pragma unroll
        for (int n1 = 0; n1 < N1; ++n1) {
          const int gx = freq<N>(N2 * n1 + n2);
          const bool ok = gx >= -rx && gx <= rx;
          const cx<T> x = L[(ok ? gx + rx : 0) * LS + py];
          v[n1] = ok ? x : zero;
        }
        Dft<N1, +1>::run(v);
        cx<T>* p = Rw + u2 * LS + n2;
#pragma unroll
        for (int k1 = 0; k1 < N1; ++k1) p[PS * k1] = k1 ? cmul(v[k1], twi[k1]) : v[0];
      }
      wave_sync();
      if (has2) {
        cx<T>* p = Rw + u1 * LS + PS * a1;
        cx<T> v[N2];
#pragma unroll
        for (int b = 0; b < N2; ++b) v[b] = p[b];
        Dft<N2, +1>::run(v);  // v[b] = psi(x = a1 + N1 b)
#pragma unroll
        for (int b = 0; b < N2; ++b) v[b] = cx<T>{v[b].x * vr[b], v[b].y * vr[b]};
        Dft<N2, -1>::run(v);
#pragma unroll
        for (int kb = 0; kb < N2; ++kb) p[kb] = kb ? cmul(v[kb], twf[kb]) : v[0];
      }
      if constexpr (P::PF) load_v(Vz, y0 + NW * RPW);  // the next pass (clamped past the last)
      wave_sync();
      if (u2 < nrow) {
        const int y = y0 + u2, py = PS * (y % N1) + y / N1;
        const cx<T>* p = Rw + u2 * LS + n2;  // slot kb = n2 of every group
        cx<T> v[N1];
#pragma unroll
        for (int a = 0; a < N1; ++a) v[a] = p[PS * a];
        Dft<N1, -1>::run(v);
#pragma unroll
        for (int ka = 0; ka < N1; ++ka) {
          const int gx = freq<N>(n2 + N2 * ka);
          if (gx >= -rx && gx <= rx) L[(gx + rx) * LS + py] = v[ka];
        }
      }
      wave_sync();  // the row buffers are refilled by the next pass
    }
    __syncthreads();

    // the next item's first stage-A inputs, in flight during stage C
    if constexpr (P::PF) {
      const int nxt = item + int(gridDim.x);
      load_a(cin + item_base(nxt < nitems ? nxt : item), wave);
    }

    // ---- C: forward y ----
    for (int g = wave; g < ngroups; g += NW) {
      {
        const int xi = g * GL + u1;
        if (u1 < GL && xi < nx) {
          cx<T>* p = L + xi * LS + PS * a1;
          cx<T> v[N2];
#pragma unroll
          for (int b = 0; b < N2; ++b) v[b] = p[b];
          Dft<N2, -1>::run(v);
#pragma unroll
          for (int kb = 0; kb < N2; ++kb) p[kb] = kb ? cmul(v[kb], twf[kb]) : v[0];
        }
      }
      wave_sync();
      {
        const int xi = g * GL + u2;
        if (u2 < GL && xi < nx) {
          const int4 xl = XL[xi];
          const cx<T>* p = L + xi * LS + n2;
          cx<T> v[N1];
#pragma unroll
          for (int a = 0; a < N1; ++a) v[a] = p[PS * a];
          Dft<N1, -1>::run(v);
#pragma unroll
          for (int ka = 0; ka < N1; ++ka) {
            const int j = freq<N>(n2 + N2 * ka) - xl.y;
            if (j >= 0 && j < xl.z) out[xl.x + j] = v[ka];
          }
        }
      }
    }
    __syncthreads();  // the next item overwrites the x-lines
  }
}

// ---- plane pass in two halves (FP64, N = 128) --------------------------------------------------------------------
// The whole plane of y-transformed x-lines (65 x-lines of 137 FP64 slots, 142 KB) leaves room for 8 row buffers:
// one block of 4 waves per CU, 2 rows per wave. Here the plane is processed in two halves of the y residues mod N1
// (half h holds groups a = 4h .. 4h + 3 of y = a + N1 b), 72 KB each, beside 8 waves x 4 row buffers: twice the
// waves per CU and twice the rows per wave. Per half: stage A computes the first inverse stage in full and keeps
// its four outputs of the half, then the second stage on those four groups; stage B takes the half's 64 rows
// through the full x-pass; stage C runs the first forward stage on the four groups, and the second forward stage
// (a length-8 DFT over the groups) as this half's share, sum over a in the half of x_a W8^(-a ka) =
// (-1)^(h ka) Y[ka], Y the interleaved pair of length-4 DFTs of x and of x W8^(-a). The first half stores its
// share to the output rows, the second adds its own to them (each entry stays with the same lane).
struct Half128 {
  static constexpr int N = 128, N1 = 8, N2 = 16, PS = N2 + 1, LS = (N1 * PS) | 1, G = 4;
  static constexpr int LSH = (G * PS) | 1;  // slots of one x-line of a half plane
  static constexpr int GL = 64 / N2;        // x-lines per wave and group in stages A and C
  static constexpr int NW = 8, RPW = 4;     // waves per block, rows per wave and pass in stage B
};
constexpr size_t half128_lines_bytes(int nx) {
  using H = Half128;
  return (size_t(nx) * H::LSH + size_t(H::NW) * H::RPW * H::LS + H::N) * sizeof(c128);
}
constexpr size_t half128_lds(int nx) { return half128_lines_bytes(nx) + size_t(nx) * 16; }

__global__ __launch_bounds__(64 * Half128::NW) void k_plane_half(int ncol, int rx, const int4* __restrict__ xline,
                                                                 const c128* __restrict__ twg,
                                                                 const double* __restrict__ Vt,
                                                                 const c128* __restrict__ cin,
                                                                 c128* __restrict__ cout, int nitems) {
  using H = Half128;
  using T = double;
  constexpr int N = H::N, N1 = H::N1, N2 = H::N2, PS = H::PS, LS = H::LS, LSH = H::LSH, GL = H::GL, NW = H::NW,
                RPW = H::RPW;
  extern __shared__ unsigned char smem_raw[];
  const int nx = 2 * rx + 1;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  c128* L = reinterpret_cast<c128*>(smem_raw);                // [nx][LSH] half plane
  c128* Rw = L + nx * LSH + wave * RPW * LS;                  // this wave's [RPW][LS] row buffers
  c128* TW = L + nx * LSH + NW * RPW * LS;                    // [N] twiddles W_N^k (forward sign)
  int4* XL = reinterpret_cast<int4*>(smem_raw + half128_lines_bytes(nx));
  const c128 zero = {0.0, 0.0};
  for (int t = threadIdx.x; t < nx; t += blockDim.x) XL[t] = xline[t];
  for (int t = threadIdx.x; t < N; t += blockDim.x) TW[t] = twg[t];

  const int u2 = lane / N2, n2 = lane - u2 * N2;  // (line or row, n2 / kb)
  const int u1 = lane / N1, a1 = lane - u1 * N1;  // (row, k1 / a) of stage B
  const int uq = lane / H::G, aq = lane - uq * H::G;  // (line, group within the half) of stages A2 and C1
  c128 twi[N1], twf[N2];
  twi[0] = c128{1.0, 0.0};
#pragma unroll
  for (int k = 1; k < N1; ++k) {
    const c128 w = twg[(n2 * k) % N];
    twi[k] = c128{w.x, -w.y};
  }
#pragma unroll
  for (int k = 1; k < N2; ++k) twf[k] = twg[(a1 * k) % N];
  __syncthreads();
  // The outermost x-lines (gx = -rx, rx) of a sphere of integer radius hold one column, at gy = 0: their inverse y
  // transform is that value on every y, and their one forward output (gy = 0) the sum over y. They are set and
  // summed by the last wave directly, and the others go through the transforms in groups of GL, 63 lines in 16
  // groups at 128^3 (two per wave) instead of 65 in 17 (a third round on one wave).
  const int trim = (nx >= 3 && XL[0].z == 1 && XL[0].y == 0 && XL[nx - 1].z == 1 && XL[nx - 1].y == 0) ? 1 : 0;
  const int xend = nx - trim;  // lines trim .. xend - 1 take the transforms
  const int ngroups = (xend - trim + GL - 1) / GL;
  const bool edge_wave = trim && wave == NW - 1;  // a wave with no more groups than any other
  const int et = lane >> 5, es = lane & 31;        // edge line (0: gx = -rx, 1: gx = rx) and slot of a lane
  const int exi = et ? nx - 1 : 0;

  for (int item = blockIdx.x; item < nitems; item += gridDim.x) {
    const int z = item % N;
    const long cs = col_stride(ncol);
    const long base = long(item / N) * N * cs + long(z) * cs;
    const c128* in = cin + base;
    c128* out = cout + base;
    const T* Vz = Vt + long(z) * N * N;

    for (int h = 0; h < 2; ++h) {
      // ---- A: inverse y, the half's four groups ----
      for (int g = wave; g < ngroups; g += NW) {
        {
          const int xi = trim + g * GL + u2;
          if (xi < xend) {
            const int4 xl = XL[xi];  // {first column, lowest gy, column count, 0}
            c128 v[N1];
#pragma unroll
            for (int n1 = 0; n1 < N1; ++n1) {
              const int j = freq<N>(N2 * n1 + n2) - xl.y;
              const bool ok = j >= 0 && j < xl.z;
              const c128 x = in[xl.x + (ok ? j : 0)];
              v[n1] = ok ? x : zero;
            }
            Dft<N1, +1>::run(v);
            c128* p = L + xi * LSH + n2;
            const bool hh = h != 0;
#pragma unroll
            for (int q = 0; q < H::G; ++q) {
              // the half's output k1 = q + 4h and its twiddle, selected per component (a select of whole values
              // goes through private memory)
              const c128 x = {hh ? v[q + H::G].x : v[q].x, hh ? v[q + H::G].y : v[q].y};
              const c128 w = {hh ? twi[q + H::G].x : twi[q].x, hh ? twi[q + H::G].y : twi[q].y};
              p[PS * q] = cmul(x, w);
            }
          }
        }
        wave_sync();
        {
          const int xi = trim + g * GL + uq;
          if (uq < GL && xi < xend) {
            c128* p = L + xi * LSH + PS * aq;
            c128 v[N2];
#pragma unroll
            for (int b = 0; b < N2; ++b) v[b] = p[b];
            Dft<N2, +1>::run(v);
#pragma unroll
            for (int b = 0; b < N2; ++b) p[b] = v[b];  // y = (aq + 4h) + N1 b
          }
        }
      }
      if (edge_wave) {  // the edge lines: their one value on the half's 64 slots PS q + b, two slots per lane
        const c128 c = in[XL[exi].x];
        c128* p = L + exi * LSH;
#pragma unroll
        for (int e = es; e < H::G * N2; e += 32) p[PS * (e / N2) + e % N2] = c;
      }
      __syncthreads();

      // ---- B: the half's 64 rows (row r: y = 4h + r % 4 + N1 (r / 4), slot PS (r % 4) + r / 4) ----
      for (int r0 = wave * RPW; r0 < N / 2; r0 += NW * RPW) {
        T vr[N2];
        {
          const int r = r0 + (u1 < RPW ? u1 : 0);
          const int y = H::G * h + (r % H::G) + N1 * (r / H::G);
          const T* Vrow = Vz + long(y) * N + a1;
#pragma unroll
          for (int b = 0; b < N2; ++b) vr[b] = Vrow[N1 * b];
        }
        if (u2 < RPW) {
          const int r = r0 + u2, py = PS * (r % H::G) + r / H::G;
          c128 v[N1];
#pragma unroll
          for (int n1 = 0; n1 < N1; ++n1) {
            const int gx = freq<N>(N2 * n1 + n2);
            const bool ok = gx >= -rx && gx <= rx;
            const c128 x = L[(ok ? gx + rx : 0) * LSH + py];
            v[n1] = ok ? x : zero;
          }
          Dft<N1, +1>::run(v);
          c128* p = Rw + u2 * LS + n2;
#pragma unroll
          for (int k1 = 0; k1 < N1; ++k1) p[PS * k1] = k1 ? cmul(v[k1], twi[k1]) : v[0];
        }
        wave_sync();
        if (u1 < RPW) {
          c128* p = Rw + u1 * LS + PS * a1;
          c128 v[N2];
#pragma unroll
          for (int b = 0; b < N2; ++b) v[b] = p[b];
          Dft<N2, +1>::run(v);  // v[b] = psi(x = a1 + N1 b)
#pragma unroll
          for (int b = 0; b < N2; ++b) v[b] = c128{v[b].x * vr[b], v[b].y * vr[b]};
          Dft<N2, -1>::run(v);
#pragma unroll
          for (int kb = 0; kb < N2; ++kb) p[kb] = kb ? cmul(v[kb], twf[kb]) : v[0];
        }
        wave_sync();
        if (u2 < RPW) {
          const int r = r0 + u2, py = PS * (r % H::G) + r / H::G;
          const c128* p = Rw + u2 * LS + n2;
          c128 v[N1];
#pragma unroll
          for (int a = 0; a < N1; ++a) v[a] = p[PS * a];
          Dft<N1, -1>::run(v);
#pragma unroll
          for (int ka = 0; ka < N1; ++ka) {
            const int gx = freq<N>(n2 + N2 * ka);
            if (gx >= -rx && gx <= rx) L[(gx + rx) * LSH + py] = v[ka];
          }
        }
        wave_sync();  // the row buffers are refilled by the next pass
      }
      __syncthreads();

      // ---- C: forward y, this half's share ----
      for (int g = wave; g < ngroups; g += NW) {
        {
          const int xi = trim + g * GL + uq;
          if (uq < GL && xi < xend) {
            c128* p = L + xi * LSH + PS * aq;
            const int a = aq + H::G * h;
            c128 v[N2];
#pragma unroll
            for (int b = 0; b < N2; ++b) v[b] = p[b];
            Dft<N2, -1>::run(v);
#pragma unroll
            for (int kb = 0; kb < N2; ++kb) p[kb] = kb ? cmul(v[kb], TW[(a * kb) % N]) : v[0];
          }
        }
        wave_sync();
        {
          const int xi = trim + g * GL + u2;
          if (xi < xend) {
            const int4 xl = XL[xi];
            const c128* p = L + xi * LSH + n2;
            c128 e[H::G], o[H::G];
            static_for<0, H::G>([&](auto qc) {
              constexpr int q = decltype(qc)::value;
              e[q] = p[PS * q];
              o[q] = twc<N1, q, -1>(e[q]);
            });
            Dft<H::G, -1>::run(e);  // Y[2k]
            Dft<H::G, -1>::run(o);  // Y[2k + 1]
#pragma unroll
            for (int ka = 0; ka < N1; ++ka) {
              const int j = freq<N>(n2 + N2 * ka) - xl.y;
              if (j >= 0 && j < xl.z) {
                c128 yv = (ka & 1) ? o[ka >> 1] : e[ka >> 1];
                if (h == 0) {
                  out[xl.x + j] = yv;
                } else {
                  if (ka & 1) yv = c128{-yv.x, -yv.y};
                  out[xl.x + j] = out[xl.x + j] + yv;  // this lane stored the first half's share there
                }
              }
            }
          }
        }
      }
      if (edge_wave) {  // the edge lines: the sum over the half's 64 y values, 32 lanes per line
        const c128* p = L + exi * LSH;
        c128 acc = p[PS * (es / N2) + es % N2] + p[PS * ((es + 32) / N2) + (es + 32) % N2];
#pragma unroll
        for (int o = 16; o > 0; o >>= 1) {
          acc.x += __shfl_xor(acc.x, o, 64);
          acc.y += __shfl_xor(acc.y, o, 64);
        }
        if (es == 0) {
          const int c = XL[exi].x;
          if (h == 0) out[c] = acc;
          else out[c] = out[c] + acc;  // this lane stored the first half's sum there
        }
      }
      __syncthreads();  // the next half (item) overwrites the half plane
    }
  }
}

// ---- band densities on the large boxes (N = 96, 128) ---------------------------------------------------------------
// part[chunk][z][y][x] = sum over the chunk's bands b of w_b Re(conj(a_b(r)) psi_b(r)) (cross = 1) or w_b |a_b(r)|^2
// (cross = 0). The cross term is taken as the difference of two densities, Re(conj(a) psi) =
// (|s a + psi/s|^2 - |s a - psi/s|^2) / 4 for any real s > 0 (s_b balances the two norms, so that the difference loses
// no more digits than the product would): one field at a time in real space, so that the plane of y-transformed
// x-lines (stage A of the plane pass) and the row buffers fit in LDS at the large boxes, where two planes do not. One
// block per (z-plane, band chunk), with the wave-local stages of the plane pass; the block adds each band's
// contribution into its own slice of part in global memory (zeroed first), in band order, so the sum does not depend on
// timing.
template <int N, typename T>
__global__ __launch_bounds__((64 * PlaneCfg<N, T>::NW)) void k_dens(int ncol, int rx, const int4* __restrict__ xline,
                                                                    const cx<T>* __restrict__ twg,
                                                                    const cx<T>* __restrict__ ca,
                                                                    const cx<T>* __restrict__ cb, int cross, int nband,
                                                                    int bpc, const double* __restrict__ wts,
                                                                    const double* __restrict__ sc,
                                                                    double* __restrict__ part) {
  using P = PlaneCfg<N, T>;
  constexpr int N1 = P::N1, N2 = P::N2, PS = P::PS, LS = P::LS, NW = P::NW, GL = P::GL, RPW = P::RPW;
  extern __shared__ unsigned char smem_raw[];
  const int nx = 2 * rx + 1;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  cx<T>* L = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* Rw = L + nx * LS + wave * RPW * LS;
  const cx<T> zero = {T(0), T(0)};
  const int z = blockIdx.x, chunk = blockIdx.y;
  const int b0 = chunk * bpc, b1 = min(nband, b0 + bpc);
  double* out = part + (long(chunk) * N + z) * N * N;
  for (int t = threadIdx.x; t < N * N; t += blockDim.x) out[t] = 0.0;
  __syncthreads();
  const int u2 = lane / N2, n2 = lane - u2 * N2;
  const int u1 = lane / N1, a1 = lane - u1 * N1;
  cx<T> twi[N1];
#pragma unroll
  for (int k = 1; k < N1; ++k) {
    const cx<T> w = twg[(n2 * k) % N];
    twi[k] = cx<T>{w.x, -w.y};
  }
  const int ngroups = (nx + GL - 1) / GL;
  const int npass = cross ? 2 : 1;
  for (int band = b0; band < b1; ++band) {
    const long base = long(band) * N * col_stride(ncol) + long(z) * col_stride(ncol);
    const T s = cross ? T(sc[band]) : T(1);
    const T si = cross ? T(1) / s : T(0);
    const double wt = wts ? wts[band] : 1.0;
    for (int pass = 0; pass < npass; ++pass) {
      const T sg = pass ? T(-1) : T(1);
      const double wp = cross ? (pass ? -0.25 : 0.25) * wt : wt;
      // ---- A: inverse y of u = s a + sg psi / s (u = a without cross) ----
      for (int g = wave; g < ngroups; g += NW) {
        {
          const int xi = g * GL + u2;
          if (u2 < GL && xi < nx) {
            const int4 xl = xline[xi];
            cx<T> v[N1];
#pragma unroll
            for (int n1 = 0; n1 < N1; ++n1) {
              const int j = freq<N>(N2 * n1 + n2) - xl.y;
              const bool ok = j >= 0 && j < xl.z;
              const long e = base + xl.x + (ok ? j : 0);
              const cx<T> xa = ca[e];
              const cx<T> xb = cross ? cb[e] : zero;
              const cx<T> u = {s * xa.x + sg * si * xb.x, s * xa.y + sg * si * xb.y};
              v[n1] = ok ? u : zero;
            }
            Dft<N1, +1>::run(v);
            cx<T>* p = L + xi * LS + n2;
#pragma unroll
            for (int k1 = 0; k1 < N1; ++k1) p[PS * k1] = k1 ? cmul(v[k1], twi[k1]) : v[0];
          }
        }
        wave_sync();
        {
          const int xi = g * GL + u1;
          if (u1 < GL && xi < nx) {
            cx<T>* p = L + xi * LS + PS * a1;
            cx<T> v[N2];
#pragma unroll
            for (int b = 0; b < N2; ++b) v[b] = p[b];
            Dft<N2, +1>::run(v);
#pragma unroll
            for (int b = 0; b < N2; ++b) p[b] = v[b];
          }
        }
      }
      __syncthreads();
      // ---- B: inverse x per row, then w |u(r)|^2 into this block's slice ----
      for (int y0 = wave * RPW; y0 < N; y0 += NW * RPW) {
        const int nrow = min(RPW, N - y0);
        if (u2 < nrow) {
          const int y = y0 + u2, py = PS * (y % N1) + y / N1;
          cx<T> v[N1];
#pragma unroll
          for (int n1 = 0; n1 < N1; ++n1) {
            const int gx = freq<N>(N2 * n1 + n2);
            const bool ok = gx >= -rx && gx <= rx;
            const cx<T> x = L[(ok ? gx + rx : 0) * LS + py];
            v[n1] = ok ? x : zero;
          }
          Dft<N1, +1>::run(v);
          cx<T>* p = Rw + u2 * LS + n2;
#pragma unroll
          for (int k1 = 0; k1 < N1; ++k1) p[PS * k1] = k1 ? cmul(v[k1], twi[k1]) : v[0];
        }
        wave_sync();
        if (u1 < nrow) {
          const int y = y0 + u1;
          const cx<T>* p = Rw + u1 * LS + PS * a1;
          cx<T> v[N2];
#pragma unroll
          for (int b = 0; b < N2; ++b) v[b] = p[b];
          Dft<N2, +1>::run(v);  // v[b] = u(x = a1 + N1 b, y)
          double* o = out + long(y) * N + a1;
#pragma unroll
          for (int b = 0; b < N2; ++b)
            o[N1 * b] += wp * (double(v[b].x) * double(v[b].x) + double(v[b].y) * double(v[b].y));
        }
        wave_sync();  // the row buffers are refilled by the next pass
      }
      __syncthreads();  // the next field overwrites the x-lines
    }
  }
}

// ---- cross density for the adjoint: part[chunk][z][y][x] = sum_b w_b Re(conj(a_b(r)) psi_b(r)) ----------
// Inputs are the z-transformed disk columns of both blocks (as written by the column pass). Per block: one
// z-plane and a chunk of bands; each thread keeps its (y, x) points of every row batch in FP64 registers
// across the bands of the chunk, so the band sum is in a fixed order.
template <int N, typename T> constexpr int xdens_batches() { return (N + xdens_rows<N, T>() - 1) / xdens_rows<N, T>(); }
template <int N, typename T> constexpr size_t xdens_lds(int nx) {
  return (size_t(2 * (nx + xdens_rows<N, T>())) * line_stride<N>() + 3 * N) * sizeof(cx<T>);
}

// inverse y of one x-line block (both stages), the line ends in digit-reversed order as in k_plane
template <int N, typename T>
__device__ __forceinline__ void y_inverse(const cx<T>* __restrict__ in, cx<T>* L, const int4* __restrict__ xline,
                                          const cx<T>* twA, int nx) {
  constexpr int N1 = LineSplit<N>::N1, N2 = LineSplit<N>::N2, LS = line_stride<N>(), PS = group_stride<N>();
  const int tid = threadIdx.x;
  for (int task = tid; task < nx * N2; task += NT) {
    const int xi = task / N2, n2 = task - xi * N2;
    const int4 xl = xline[xi];
    cx<T> v[N1];
#pragma unroll
    for (int n1 = 0; n1 < N1; ++n1) {
      const int j = freq<N>(N2 * n1 + n2) - xl.y;
      v[n1] = (j >= 0 && j < xl.z) ? cx<T>(in[xl.x + j]) : cx<T>{T(0), T(0)};
    }
    Dft<N1, +1>::run(v);
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) L[xi * LS + PS * k1 + n2] = k1 ? cmul(v[k1], conj_if(twA[k1 * N2 + n2], true)) : v[0];
  }
  __syncthreads();
  for (int task = tid; task < nx * N1; task += NT) {
    const int xi = task / N1, a = task - xi * N1;
    cx<T>* p = L + xi * LS + PS * a;
    cx<T> v[N2];
#pragma unroll
    for (int n2 = 0; n2 < N2; ++n2) v[n2] = p[n2];
    Dft<N2, +1>::run(v);
#pragma unroll
    for (int k2 = 0; k2 < N2; ++k2) p[k2] = v[k2];
  }
}

// first inverse-x stage of rows y0 .. y0 + nrow - 1 from the x-lines in L into the row scratch S
template <int N, typename T>
__device__ __forceinline__ void x_inverse_stage1(const cx<T>* L, cx<T>* S, const cx<T>* twA, int rx, int y0, int nrow) {
  constexpr int N1 = LineSplit<N>::N1, N2 = LineSplit<N>::N2, LS = line_stride<N>(), PS = group_stride<N>();
  for (int task = threadIdx.x; task < nrow * N2; task += NT) {
    const int yy = task / N2, n2 = task - yy * N2;
    const int y = y0 + yy, py = PS * (y % N1) + y / N1;
    cx<T> v[N1];
#pragma unroll
    for (int n1 = 0; n1 < N1; ++n1) {
      const int gx = freq<N>(N2 * n1 + n2);
      v[n1] = (gx >= -rx && gx <= rx) ? cx<T>(L[(gx + rx) * LS + py]) : cx<T>{T(0), T(0)};
    }
    Dft<N1, +1>::run(v);
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) S[yy * LS + PS * k1 + n2] = k1 ? cmul(v[k1], conj_if(twA[k1 * N2 + n2], true)) : v[0];
  }
}

template <int N, typename T>
__global__ __launch_bounds__(NT) void k_xdens(int ncol, int rx, const int4* __restrict__ xline,
                                              const cx<T>* __restrict__ twg, const cx<T>* __restrict__ ca,
                                              const cx<T>* __restrict__ cb, int nband, int bpc,
                                              const double* __restrict__ wts, double* __restrict__ part) {
  constexpr int N1 = LineSplit<N>::N1, N2 = LineSplit<N>::N2, LS = line_stride<N>(), PS = group_stride<N>();
  constexpr int RB = xdens_rows<N, T>(), NBT = xdens_batches<N, T>();
  static_assert(RB * N1 <= NT, "one second-stage task per thread and row batch");
  extern __shared__ unsigned char smem_raw[];
  const int nx = 2 * rx + 1;
  cx<T>* La = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* Lb = La + nx * LS;
  cx<T>* Sa = Lb + nx * LS;
  cx<T>* Sb = Sa + RB * LS;
  cx<T>* tw = Sb + RB * LS;
  cx<T>* twA = tw + N;
  cx<T>* twB = twA + N;
  const int z = blockIdx.x, chunk = blockIdx.y, tid = threadIdx.x;
  const int b0 = chunk * bpc, b1 = min(nband, b0 + bpc);
  for (int t = tid; t < N; t += NT) tw[t] = twg[t];
  __syncthreads();
  stage_twiddles<N, T>(tw, twA, twB);
  double acc[NBT][N2];
#pragma unroll
  for (int t = 0; t < NBT; ++t)
#pragma unroll
    for (int b = 0; b < N2; ++b) acc[t][b] = 0.0;
  const int yy = tid / N1, a = tid - (tid / N1) * N1;
  __syncthreads();
  for (int band = b0; band < b1; ++band) {
    const double wt = wts ? wts[band] : 1.0;
    const long base = long(band) * N * col_stride(ncol) + long(z) * col_stride(ncol);
    y_inverse<N, T>(ca + base, La, xline, twA, nx);
    y_inverse<N, T>(cb + base, Lb, xline, twA, nx);
    __syncthreads();
#pragma unroll
    for (int t = 0; t < NBT; ++t) {
      const int y0 = t * RB, nrow = min(RB, N - y0);
      x_inverse_stage1<N, T>(La, Sa, twA, rx, y0, nrow);
      x_inverse_stage1<N, T>(Lb, Sb, twA, rx, y0, nrow);
      __syncthreads();
      if (yy < nrow) {
        cx<T> va[N2], vb[N2];
#pragma unroll
        for (int n2 = 0; n2 < N2; ++n2) {
          va[n2] = Sa[yy * LS + PS * a + n2];
          vb[n2] = Sb[yy * LS + PS * a + n2];
        }
        Dft<N2, +1>::run(va);
        Dft<N2, +1>::run(vb);
#pragma unroll
        for (int b = 0; b < N2; ++b)
          acc[t][b] += wt * (double(va[b].x) * double(vb[b].x) + double(va[b].y) * double(vb[b].y));
      }
      __syncthreads();
    }
  }
  double* out = part + (long(chunk) * N + z) * N * N;
#pragma unroll
  for (int t = 0; t < NBT; ++t) {
    const int y0 = t * RB, nrow = min(RB, N - y0);
    if (yy < nrow) {
#pragma unroll
      for (int b = 0; b < N2; ++b) out[long(y0 + yy) * N + a + N1 * b] = acc[t][b];
    }
  }
}

// dV[x][y][z] += coef * sum_chunk part[chunk][z][y][x]
__global__ void k_xdens_reduce(int n, int nchunk, const double* __restrict__ part, double coef, double* __restrict__ dV) {
  const long total = long(n) * n * n;
  for (long t = blockIdx.x * long(blockDim.x) + threadIdx.x; t < total; t += long(gridDim.x) * blockDim.x) {
    double s = 0.0;
    for (int c = 0; c < nchunk; ++c) s += part[long(c) * total + t];
    const long x = t % n, y = (t / n) % n, z = t / (long(n) * n);
    dV[(x * n + y) * n + z] += coef * s;
  }
}

template <int N, typename T>
__global__ __launch_bounds__(NT) void k_col_fwd(int ncol, const int4* __restrict__ col, const int* __restrict__ ent,
                                                const cx<T>* __restrict__ twg, const cx<T>* __restrict__ colbuf,
                                                const cx<T>* __restrict__ X, long ldx, const T* __restrict__ kin,
                                                cx<T>* __restrict__ out, long ldo, T scale) {
  constexpr int CPB = cpb<N, T>(), LS = line_stride<N>();
  __shared__ cx<T> lines[CPB * LS];
  __shared__ cx<T> twA[N];
  const int band = blockIdx.y;
  const int c0 = blockIdx.x * CPB, c1 = min(ncol, c0 + CPB), nc = c1 - c0;
  const int tid = threadIdx.x;
  for (int t = tid; t < N; t += NT) twA[t] = twg[((t % LineSplit<N>::N2) * (t / LineSplit<N>::N2)) % N];
  const long cs = col_stride(ncol);
  const cx<T>* in = colbuf + long(band) * N * cs;
  for (int t = tid; t < N * nc; t += NT) {
    const int z = t / nc, c = t - z * nc;
    lines[c * LS + z] = in[long(z) * cs + c0 + c];
  }
  __syncthreads();
  lds_fft<N, -1, T>(lines, nc, LS, twA);
  const int e0 = col[c0].z, e1 = col[c1 - 1].z + col[c1 - 1].w;
  const cx<T>* xb = X + long(band) * ldx;
  cx<T>* ob = out + long(band) * ldo;
  for (int e = e0 + tid; e < e1; e += NT) {
    const int code = ent[e];
    const cx<T> v = lines[((code >> 8) - c0) * LS + (code & 255)];
    if (kin) {
      const cx<T> x = xb[e];
      const T k = kin[e];
      ob[e] = cx<T>{v.x * scale + k * x.x, v.y * scale + k * x.y};
    } else {
      ob[e] = cx<T>{v.x * scale, v.y * scale};
    }
  }
}

// ---- Gamma point: two real bands per complex transform --------------------------------------------------------
// Stored Gamma vectors hold sqrt(2) c_G on the half sphere (c_0 at G = 0). gmap[e] = h | (conj << 30) gives, for
// entry e of the whole sphere, the half-sphere entry h with G_e = G_h (conj = 0) or G_e = -G_h (conj = 1).
// u(G_e) = c_2j(G_e) + i c_2j+1(G_e): the inverse transform is then psi_2j(r) + i psi_2j+1(r).
template <typename T>
__global__ void k_gamma_pack(int npf, int nb, int npair, const int* __restrict__ gmap, int h0,
                             const cx<T>* __restrict__ X, long ldx, cx<T>* __restrict__ U, long ldu) {
  const long total = long(npf) * npair;
  const T r2 = T(0.70710678118654752440);
  for (long t = blockIdx.x * long(blockDim.x) + threadIdx.x; t < total; t += long(gridDim.x) * blockDim.x) {
    const int j = int(t / npf), e = int(t - long(j) * npf);
    const int code = gmap[e];
    const int h = code & 0x3fffffff;
    const bool cj = (code >> 30) & 1;
    const T s = h == h0 ? T(1) : r2;
    cx<T> v0 = X[h + long(2 * j) * ldx];
    cx<T> v1 = 2 * j + 1 < nb ? X[h + long(2 * j + 1) * ldx] : cx<T>{T(0), T(0)};
    if (cj) { v0.y = -v0.y; v1.y = -v1.y; }
    U[e + long(j) * ldu] = cx<T>{s * (v0.x - v1.y), s * (v0.y + v1.x)};
  }
}

// Separates the transformed pair: with w = W(G), m = W(-G) (pair[h] = entries of G_h and -G_h),
// band 2j gets (w + conj m) / 2, band 2j+1 gets (w - conj m) / (2i); scaled back to the stored form, plus K x.
template <typename T>
__global__ void k_gamma_split(int nh, int nb, const int2* __restrict__ pair, int h0, const cx<T>* __restrict__ W,
                              long ldw, const T* __restrict__ kin, const cx<T>* __restrict__ X, long ldx,
                              cx<T>* __restrict__ out, long ldo) {
  const long total = long(nh) * nb;
  const T sq2 = T(1.41421356237309504880);
  for (long t = blockIdx.x * long(blockDim.x) + threadIdx.x; t < total; t += long(gridDim.x) * blockDim.x) {
    const int b = int(t / nh), h = int(t - long(b) * nh);
    const int j = b >> 1;
    const int2 pe = pair[h];
    const cx<T> w = W[pe.x + long(j) * ldw], m = W[pe.y + long(j) * ldw];
    cx<T> y = (b & 1) ? cx<T>{T(0.5) * (w.y + m.y), T(-0.5) * (w.x - m.x)}
                      : cx<T>{T(0.5) * (w.x + m.x), T(0.5) * (w.y - m.y)};
    const T s = h == h0 ? T(1) : sq2;
    const cx<T> x = X[h + long(b) * ldx];
    const T k = kin[h];
    out[h + long(b) * ldo] = cx<T>{s * y.x + k * x.x, s * y.y + k * x.y};
  }
}

template <typename F> hipError_t dispatch_n(int n, F&& f) {
  switch (n) {
    case 8: return f(std::integral_constant<int, 8>{});
    case 12: return f(std::integral_constant<int, 12>{});
    case 16: return f(std::integral_constant<int, 16>{});
    case 24: return f(std::integral_constant<int, 24>{});
    case 32: return f(std::integral_constant<int, 32>{});
    case 48: return f(std::integral_constant<int, 48>{});
    case 64: return f(std::integral_constant<int, 64>{});
    case 96: return f(std::integral_constant<int, 96>{});
    case 128: return f(std::integral_constant<int, 128>{});
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

template <typename T>
hipError_t gamma_pack(int npf, int nb, const int* gmap, int h0, const cx<T>* X, long ldx, cx<T>* U, long ldu,
                      hipStream_t st) {
  const int npair = (nb + 1) / 2;
  if (npf <= 0 || nb <= 0) return hipSuccess;
  const long total = long(npf) * npair;
  const long blocks = std::min<long>((total + 255) / 256, 65536);
  hipLaunchKernelGGL((k_gamma_pack<T>), dim3(unsigned(blocks)), dim3(256), 0, st, npf, nb, npair, gmap, h0, X, ldx, U,
                     ldu);
  return hipGetLastError();
}
template <typename T>
hipError_t gamma_split(int nh, int nb, const int2* pair, int h0, const cx<T>* W, long ldw, const T* kin,
                       const cx<T>* X, long ldx, cx<T>* out, long ldo, hipStream_t st) {
  if (nh <= 0 || nb <= 0) return hipSuccess;
  const long total = long(nh) * nb;
  const long blocks = std::min<long>((total + 255) / 256, 65536);
  hipLaunchKernelGGL((k_gamma_split<T>), dim3(unsigned(blocks)), dim3(256), 0, st, nh, nb, pair, h0, W, ldw, kin, X,
                     ldx, out, ldo);
  return hipGetLastError();
}
template hipError_t gamma_pack<double>(int, int, const int*, int, const c128*, long, c128*, long, hipStream_t);
template hipError_t gamma_pack<float>(int, int, const int*, int, const c64*, long, c64*, long, hipStream_t);
template hipError_t gamma_split<double>(int, int, const int2*, int, const c128*, long, const double*, const c128*, long,
                                        c128*, long, hipStream_t);
template hipError_t gamma_split<float>(int, int, const int2*, int, const c64*, long, const float*, const c64*, long,
                                       c64*, long, hipStream_t);


template <typename T>
hipError_t fft_col_inverse(const FftGeom& g, const cx<T>* tw, const cx<T>* X, long ldx, int nb, cx<T>* colbuf,
                           hipStream_t st) {
  if (nb <= 0) return hipSuccess;
  return dispatch_n(g.n, [&](auto nc) {
    constexpr int N = decltype(nc)::value;
    dim3 grid((g.ncol + cpb<N, T>() - 1) / cpb<N, T>(), nb);
    hipLaunchKernelGGL((k_col_inv<N, T>), grid, dim3(NT), 0, st, g.ncol, g.col, g.ent, tw, X, ldx, colbuf);
    return hipGetLastError();
  });
}

hipError_t plane_half_launch(const FftGeom& g, const c128* tw, const double* Vt, const c128* cin, c128* cout, int nitems,
                             hipStream_t st) {
  const size_t lds = half128_lds(2 * g.rx + 1);
  if (lds > 160 * 1024) return hipErrorInvalidConfiguration;
  const int grid = int(std::min<long>(nitems, long(compute_units())));  // one block per CU (LDS)
  hipLaunchKernelGGL(k_plane_half, dim3(grid), dim3(64 * Half128::NW), lds, st, g.ncol, g.rx, g.xline, tw, Vt, cin,
                     cout, nitems);
  return hipGetLastError();
}
hipError_t plane_half_launch(const FftGeom&, const c64*, const float*, const c64*, c64*, int, hipStream_t) {
  return hipErrorInvalidConfiguration;  // FP32 plans keep the whole plane
}

// resident blocks of k_plane<N, T> on the device (LDS and registers): the persistent grid of the plane pass
template <int N, typename T> int plane_resident_blocks(int rx) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(&k_plane<N, T>),
                                                   64 * PlaneCfg<N, T>::NW, plane_lds<N, T>(2 * rx + 1)) != hipSuccess ||
      per_cu <= 0)
    per_cu = 1;
  return compute_units() * per_cu;
}

int fft_plane_blocks(int n, int rx, bool dbl) {
  int out = compute_units();
  (void)dispatch_n(n, [&](auto nc) {
    constexpr int N = decltype(nc)::value;
    if (N == 128 && dbl) out = compute_units();  // k_plane_half: one block per CU
    else out = dbl ? plane_resident_blocks<N, double>(rx) : plane_resident_blocks<N, float>(rx);
    return hipSuccess;
  });
  return out;
}

template <typename T>
hipError_t fft_plane(const FftGeom& g, const cx<T>* tw, const T* Vt, const cx<T>* cin, cx<T>* cout, int nb,
                     hipStream_t st) {
  if (nb <= 0) return hipSuccess;
  return dispatch_n(g.n, [&](auto nc) {
    constexpr int N = decltype(nc)::value;
    const int nitems = N * nb;
    if constexpr (N == 128 && std::is_same<T, double>::value) {  // the plane in two halves (see k_plane_half)
      return plane_half_launch(g, tw, Vt, cin, cout, nitems, st);
    } else {
      const size_t lds = plane_lds<N, T>(2 * g.rx + 1);
      if (lds > 160 * 1024) return hipErrorInvalidConfiguration;
      // a persistent grid of as many blocks as stay resident (LDS and registers), so that no block starts its share
      // of the items late and each loads its twiddles once
      constexpr int threads = 64 * PlaneCfg<N, T>::NW;
      const int grid = int(std::min<long>(nitems, long(plane_resident_blocks<N, T>(g.rx))));
      hipLaunchKernelGGL((k_plane<N, T>), dim3(grid), dim3(threads), lds, st, g.ncol, g.rx, g.xline, tw, Vt, cin,
                         cout, nitems);
      return hipGetLastError();
    }
  });
}

template <typename T>
hipError_t fft_col_forward(const FftGeom& g, const cx<T>* tw, const cx<T>* colbuf, const cx<T>* X, long ldx,
                           const T* kin, cx<T>* out, long ldo, int nb, hipStream_t st) {
  if (nb <= 0) return hipSuccess;
  const T scale = T(1.0 / (double(g.n) * g.n * g.n));
  return dispatch_n(g.n, [&](auto nc) {
    constexpr int N = decltype(nc)::value;
    dim3 grid((g.ncol + cpb<N, T>() - 1) / cpb<N, T>(), nb);
    hipLaunchKernelGGL((k_col_fwd<N, T>), grid, dim3(NT), 0, st, g.ncol, g.col, g.ent, tw, colbuf, X, ldx, kin, out,
                       ldo, scale);
    return hipGetLastError();
  });
}

size_t fft_plane_lds_bytes(int n, int rx, bool dbl) {
  size_t out = 0;
  (void)dispatch_n(n, [&](auto nc) {
    constexpr int N = decltype(nc)::value;
    if (N == 128 && dbl) out = half128_lds(2 * rx + 1);
    else out = dbl ? plane_lds<N, double>(2 * rx + 1) : plane_lds<N, float>(2 * rx + 1);
    return hipSuccess;
  });
  return out;
}

int xdens_chunks(int n, int nband) {
  int c = (1024 + n - 1) / n;
  return c < nband ? c : (nband > 0 ? nband : 1);
}

template <typename T>
hipError_t cross_density(const FftGeom& g, const cx<T>* tw, const cx<T>* ca, const cx<T>* cb, int nband,
                         const double* wts, const double* scale, double coef, double* part, double* dV,
                         hipStream_t st) {
  if (nband <= 0) return hipSuccess;
  const int nchunk = xdens_chunks(g.n, nband);
  const int bpc = (nband + nchunk - 1) / nchunk;
  hipError_t e = dispatch_n(g.n, [&](auto nc) {
    constexpr int N = decltype(nc)::value;
    if constexpr (N <= 64) {
      const size_t lds = xdens_lds<N, T>(2 * g.rx + 1);
      if (lds > 160 * 1024) return hipErrorInvalidConfiguration;
      hipLaunchKernelGGL((k_xdens<N, T>), dim3(N, nchunk), dim3(NT), lds, st, g.ncol, g.rx, g.xline, tw, ca, cb, nband,
                         bpc, wts, part);
      return hipGetLastError();
    } else {
      const size_t lds = plane_lds<N, T>(2 * g.rx + 1);
      if (lds > 160 * 1024) return hipErrorInvalidConfiguration;
      const int cross = ca != cb;
      if (cross && !scale) return hipErrorInvalidValue;
      hipLaunchKernelGGL((k_dens<N, T>), dim3(N, nchunk), dim3(64 * PlaneCfg<N, T>::NW), lds, st, g.ncol, g.rx, g.xline,
                         tw, ca, cb, cross, nband, bpc, wts, scale, part);
      return hipGetLastError();
    }
  });
  if (e != hipSuccess) return e;
  const long total = long(g.n) * g.n * g.n;
  int blocks = int((total + 255) / 256);
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_xdens_reduce, dim3(blocks), dim3(256), 0, st, g.n, nchunk, part,
                     coef / (double(g.n) * g.n * g.n), dV);
  return hipGetLastError();
}

size_t cross_density_part_doubles(int n, int nband) { return size_t(xdens_chunks(n, nband)) * n * n * n; }

size_t fft_xdens_lds_bytes(int n, int rx, bool dbl) {
  size_t out = 0;
  (void)dispatch_n(n, [&](auto nc) {
    constexpr int N = decltype(nc)::value;
    if constexpr (N <= 64) out = dbl ? xdens_lds<N, double>(2 * rx + 1) : xdens_lds<N, float>(2 * rx + 1);
    else out = dbl ? plane_lds<N, double>(2 * rx + 1) : plane_lds<N, float>(2 * rx + 1);
    return hipSuccess;
  });
  return out;
}

hipError_t fft_prepare_attributes() {
  // allow the plane kernels their full dynamic LDS (up to 160 KB on gfx950)
  hipError_t err = hipSuccess;
  auto set = [&](const void* fn) {
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) err = e;
  };
  auto each = [&](auto nc) {
    constexpr int N = decltype(nc)::value;
    if constexpr (N == 128) set(reinterpret_cast<const void*>(&k_plane_half));
    else set(reinterpret_cast<const void*>(&k_plane<N, double>));
    set(reinterpret_cast<const void*>(&k_plane<N, float>));
    if constexpr (N <= 64) {
      set(reinterpret_cast<const void*>(&k_xdens<N, double>));
      set(reinterpret_cast<const void*>(&k_xdens<N, float>));
    } else {
      set(reinterpret_cast<const void*>(&k_dens<N, double>));
      set(reinterpret_cast<const void*>(&k_dens<N, float>));
    }
    return hipSuccess;
  };
  for (int n : {8, 12, 16, 24, 32, 48, 64, 96, 128}) (void)dispatch_n(n, each);
  return err;
}

template hipError_t cross_density<double>(const FftGeom&, const c128*, const c128*, const c128*, int, const double*,
                                          const double*, double, double*, double*, hipStream_t);
template hipError_t cross_density<float>(const FftGeom&, const c64*, const c64*, const c64*, int, const double*,
                                         const double*, double, double*, double*, hipStream_t);
template hipError_t fft_col_inverse<double>(const FftGeom&, const c128*, const c128*, long, int, c128*, hipStream_t);
template hipError_t fft_col_inverse<float>(const FftGeom&, const c64*, const c64*, long, int, c64*, hipStream_t);
template hipError_t fft_plane<double>(const FftGeom&, const c128*, const double*, const c128*, c128*, int, hipStream_t);
template hipError_t fft_plane<float>(const FftGeom&, const c64*, const float*, const c64*, c64*, int, hipStream_t);
template hipError_t fft_col_forward<double>(const FftGeom&, const c128*, const c128*, const c128*, long, const double*,
                                            c128*, long, int, hipStream_t);
template hipError_t fft_col_forward<float>(const FftGeom&, const c64*, const c64*, const c64*, long, const float*,
                                           c64*, long, int, hipStream_t);

}  // namespace chebfd
