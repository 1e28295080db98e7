// Projector-space and vector kernels: block-diagonal D (Eq. 3), the capacitance matrix of the Woodbury
// inverse (Sec. 5.1), Rayleigh-Ritz preparation (Alg. 2), column dots and residual norms (Sec. 6.1).
#include <algorithm>

#include "kernels.h"

namespace chebfd {
namespace {

inline int nblocks(long work, int per = 256, int cap = 8192) {
  long b = (work + per - 1) / per;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return int(b);
}

__global__ void k_block_diag(int nproj, int nb, const int4* __restrict__ pinfo, const double* __restrict__ D,
                             const c128* __restrict__ in, long ldi, c128* __restrict__ out, long ldo) {
  const long total = long(nproj) * nb;
  for (long t = blockIdx.x * long(blockDim.x) + threadIdx.x; t < total; t += long(gridDim.x) * blockDim.x) {
    const int b = int(t / nproj), i = int(t - long(b) * nproj);
    const int4 pi = pinfo[i];  // {atom's first row, block size, block offset, 0}
    const int r = i - pi.x;
    const double* Drow = D + pi.z + long(r) * pi.y;
    const c128* col = in + long(b) * ldi + pi.x;
    double re = 0.0, im = 0.0;
    for (int j = 0; j < pi.y; ++j) {
      re += Drow[j] * col[j].x;
      im += Drow[j] * col[j].y;
    }
    out[long(b) * ldo + i] = c128{re, im};
  }
}

// One block per atom (the block of its first projector): Gauss-Jordan inverse of the atom's diagonal block of
// the Hermitian positive definite C, in LDS (block sizes up to 32), into Minv packed like D (row-major per atom).
__global__ __launch_bounds__(256) void k_block_inverse(int nproj, const int4* __restrict__ pinfo,
                                                       const c128* __restrict__ C, long ldc, c128* __restrict__ Minv,
                                                       int* __restrict__ bad) {
  __shared__ c128 a[32][33];
  __shared__ c128 x[32][33];
  const int i0 = blockIdx.x;
  const int4 pi = pinfo[i0];
  if (pi.x != i0) return;  // not the first projector of its atom
  const int n = pi.y;
  if (n > 32) {
    if (threadIdx.x == 0) bad[0] = 1;
    return;
  }
  for (int t = threadIdx.x; t < n * n; t += blockDim.x) {
    const int r = t / n, c = t - r * n;
    a[r][c] = C[(i0 + r) + long(i0 + c) * ldc];
    x[r][c] = c128{r == c ? 1.0 : 0.0, 0.0};
  }
  __syncthreads();
  for (int k = 0; k < n; ++k) {  // no pivoting: the block of an HPD matrix is HPD
    const c128 piv = a[k][k];
    const double den = piv.x * piv.x + piv.y * piv.y;
    const c128 inv = c128{piv.x / den, -piv.y / den};
    __syncthreads();
    for (int c = threadIdx.x; c < n; c += blockDim.x) {  // scale row k
      a[k][c] = cmul(a[k][c], inv);
      x[k][c] = cmul(x[k][c], inv);
    }
    __syncthreads();
    for (int t = threadIdx.x; t < n * n; t += blockDim.x) {  // eliminate column k from the other rows
      const int r = t / n, c = t - r * n;
      if (r == k) continue;
      const c128 f = a[r][k];
      if (c != k) a[r][c] = a[r][c] - cmul(f, a[k][c]);
      x[r][c] = x[r][c] - cmul(f, x[k][c]);
    }
    __syncthreads();
    for (int r = threadIdx.x; r < n; r += blockDim.x)
      if (r != k) a[r][k] = c128{0.0, 0.0};
    __syncthreads();
  }
  for (int t = threadIdx.x; t < n * n; t += blockDim.x) {
    const int r = t / n, c = t - r * n;
    Minv[pi.z + t] = x[r][c];
  }
}

// out = blockdiag(Minv) in (+ out when accumulate), complex packed blocks
__global__ void k_block_diag_c(int nproj, int nb, const int4* __restrict__ pinfo, const c128* __restrict__ M,
                               const c128* __restrict__ in, long ldi, c128* __restrict__ out, long ldo, int accumulate) {
  const long total = long(nproj) * nb;
  for (long t = blockIdx.x * long(blockDim.x) + threadIdx.x; t < total; t += long(gridDim.x) * blockDim.x) {
    const int b = int(t / nproj), i = int(t - long(b) * nproj);
    const int4 pi = pinfo[i];
    const int r = i - pi.x;
    const c128* Mrow = M + pi.z + long(r) * pi.y;
    const c128* col = in + long(b) * ldi + pi.x;
    double re = 0.0, im = 0.0;
    for (int j = 0; j < pi.y; ++j) {
      const c128 m = Mrow[j], v = col[j];
      re += m.x * v.x - m.y * v.y;
      im += m.x * v.y + m.y * v.x;
    }
    c128* o = out + long(b) * ldo + i;
    if (accumulate) { re += o->x; im += o->y; }
    *o = c128{re, im};
  }
}

// u = Q^-1 Dp - ploc (u may be ploc)
__global__ void k_overlap_rhs(int nproj, int nb, const double* __restrict__ Q, const c128* __restrict__ Dp, long ldd,
                              const c128* ploc, long ldl, c128* u, long ldu) {
  const long total = long(nproj) * nb;
  for (long t = blockIdx.x * long(blockDim.x) + threadIdx.x; t < total; t += long(gridDim.x) * blockDim.x) {
    const int b = int(t / nproj), i = int(t - long(b) * nproj);
    const c128 d = Dp[long(b) * ldd + i], l = ploc[long(b) * ldl + i];
    const double q = Q[i];
    u[long(b) * ldu + i] = c128{d.x / q - l.x, d.y / q - l.y};
  }
}

// out = s1 (Q^-1 (Dp - w) - c cur) - s2 prev (prev may be null)
__global__ void k_overlap_recur(int nproj, int nb, const double* __restrict__ Q, const c128* __restrict__ Dp, long ldd,
                                const c128* __restrict__ w, long ldw, double s1, double c, const c128* __restrict__ cur,
                                long ldc, double s2, const c128* __restrict__ prev, long ldp, c128* __restrict__ out,
                                long ldo) {
  const long total = long(nproj) * nb;
  for (long t = blockIdx.x * long(blockDim.x) + threadIdx.x; t < total; t += long(gridDim.x) * blockDim.x) {
    const int b = int(t / nproj), i = int(t - long(b) * nproj);
    const c128 d = Dp[long(b) * ldd + i], v = w[long(b) * ldw + i], x = cur[long(b) * ldc + i];
    const double q = Q[i];
    double re = s1 * ((d.x - v.x) / q - c * x.x), im = s1 * ((d.y - v.y) / q - c * x.y);
    if (prev) {
      const c128 y = prev[long(b) * ldp + i];
      re -= s2 * y.x;
      im -= s2 * y.y;
    }
    out[long(b) * ldo + i] = c128{re, im};
  }
}

__global__ void k_diag(int nproj, int nb, const double* __restrict__ d, const c128* __restrict__ in, long ldi,
                       c128* __restrict__ out, long ldo) {
  const long total = long(nproj) * nb;
  for (long t = blockIdx.x * long(blockDim.x) + threadIdx.x; t < total; t += long(gridDim.x) * blockDim.x) {
    const int b = int(t / nproj), i = int(t - long(b) * nproj);
    c128 v = in[long(b) * ldi + i];
    out[long(b) * ldo + i] = c128{d[i] * v.x, d[i] * v.y};
  }
}

template <typename E>
__global__ void k_axpbypcz(long rows, int nb, double a, const cx<E>* x, long ldx, double b, const cx<E>* y, long ldy,
                           double c, const cx<E>* z, long ldz, cx<E>* out, long ldo) {
  const long total = rows * nb;
  for (long t = blockIdx.x * long(blockDim.x) + threadIdx.x; t < total; t += long(gridDim.x) * blockDim.x) {
    const long col = t / rows, i = t - col * rows;
    double re = 0.0, im = 0.0;
    if (x) { cx<E> v = x[col * ldx + i]; re += a * double(v.x); im += a * double(v.y); }
    if (y) { cx<E> v = y[col * ldy + i]; re += b * double(v.x); im += b * double(v.y); }
    if (z) { cx<E> v = z[col * ldz + i]; re += c * double(v.x); im += c * double(v.y); }
    out[col * ldo + i] = cx<E>{E(re), E(im)};
  }
}

template <typename EO, typename EI>
__global__ void k_convert(long rows, int nb, const cx<EI>* in, long ldi, cx<EO>* out, long ldo) {
  const long total = rows * nb;
  for (long t = blockIdx.x * long(blockDim.x) + threadIdx.x; t < total; t += long(gridDim.x) * blockDim.x) {
    const long col = t / rows, i = t - col * rows;
    cx<EI> v = in[col * ldi + i];
    out[col * ldo + i] = cx<EO>{EO(v.x), EO(v.y)};
  }
}

// one block column per band; rows strided so that a wave reads consecutive coefficients
template <typename E>
__global__ void k_permute_cols(long rows, int ncols, const cx<E>* src, long lds, const int* sidx, cx<E>* dst,
                               long ldd, const int* didx) {
  const int j = blockIdx.y;
  if (j >= ncols) return;
  const cx<E>* s = src + long(sidx ? sidx[j] : j) * lds;
  cx<E>* d = dst + long(didx ? didx[j] : j) * ldd;
  for (long i = blockIdx.x * long(blockDim.x) + threadIdx.x; i < rows; i += long(gridDim.x) * blockDim.x) d[i] = s[i];
}

// LOBPCG preconditioned residuals, one block per active band a = act[j]: E = sum_g t_g |x_g|^2 / sum_g |x_g|^2,
// then W[:, j] = K(t_g / E) (HX - lambda_a SX)[:, a] with K(x) = (27 + 18x + 12x^2 + 8x^3) / (... + 16x^4).
template <typename E>
__global__ __launch_bounds__(256) void k_lobpcg_precond(long rows, const E* __restrict__ kin, const cx<E>* X,
                                                        const cx<E>* HX, const cx<E>* SX, long ld,
                                                        const double* __restrict__ lam, const int* __restrict__ act,
                                                        cx<E>* W, long ldw) {
  __shared__ double s1[256], s2[256];
  const int j = blockIdx.x, a = act[j];
  const cx<E>* x = X + long(a) * ld;
  double num = 0.0, den = 0.0;
  for (long i = threadIdx.x; i < rows; i += blockDim.x) {
    const cx<E> v = x[i];
    const double m = double(v.x) * double(v.x) + double(v.y) * double(v.y);
    num += double(kin[i]) * m;
    den += m;
  }
  s1[threadIdx.x] = num;
  s2[threadIdx.x] = den;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) { s1[threadIdx.x] += s1[threadIdx.x + k]; s2[threadIdx.x] += s2[threadIdx.x + k]; }
    __syncthreads();
  }
  const double ekin = s2[0] > 0.0 ? s1[0] / s2[0] : 1.0;
  const double l = lam[a];
  const cx<E>* h = HX + long(a) * ld;
  const cx<E>* sx = SX + long(a) * ld;
  cx<E>* w = W + long(j) * ldw;
  for (long i = threadIdx.x; i < rows; i += blockDim.x) {
    const double xx = ekin > 0.0 ? double(kin[i]) / ekin : 0.0;
    const double num4 = 27.0 + xx * (18.0 + xx * (12.0 + 8.0 * xx));
    const double K = num4 / (num4 + 16.0 * xx * xx * xx * xx);
    const cx<E> hv = h[i], sv = sx[i];
    w[i] = cx<E>{E(K * (double(hv.x) - l * double(sv.x))), E(K * (double(hv.y) - l * double(sv.y)))};
  }
}

// Z[:, j] *= 1 / sqrt(s[j]) for j < ncols
__global__ void k_scale_cols_isqrt(int n, int ncols, c128* Z, long ldz, const double* s) {
  const long total = long(n) * ncols;
  for (long t = blockIdx.x * long(blockDim.x) + threadIdx.x; t < total; t += long(gridDim.x) * blockDim.x) {
    const long j = t / n, i = t - j * n;
    const double f = 1.0 / sqrt(s[j]);
    c128 v = Z[i + j * ldz];
    Z[i + j * ldz] = c128{v.x * f, v.y * f};
  }
}

// one block per column, fixed-order tree reduction (deterministic)
template <typename E>
__global__ __launch_bounds__(256) void k_col_dots(long rows, const cx<E>* x, long ldx, const cx<E>* y, long ldy,
                                                  c128* out) {
  __shared__ double sr[256], si[256];
  const int b = blockIdx.x;
  double re = 0.0, im = 0.0;
  for (long i = threadIdx.x; i < rows; i += blockDim.x) {
    cx<E> u = x[b * ldx + i], v = y[b * ldy + i];
    re += double(u.x) * double(v.x) + double(u.y) * double(v.y);
    im += double(u.x) * double(v.y) - double(u.y) * double(v.x);
  }
  sr[threadIdx.x] = re;
  si[threadIdx.x] = im;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) { sr[threadIdx.x] += sr[threadIdx.x + s]; si[threadIdx.x] += si[threadIdx.x + s]; }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[b] = c128{sr[0], si[0]};
}

template <typename E>
__global__ __launch_bounds__(256) void k_col_resid(long rows, const cx<E>* R, long ldr, const cx<E>* U, long ldu,
                                                   const double* lam, double* out) {
  __shared__ double s[256];
  const int b = blockIdx.x;
  const double l = lam[b];
  double acc = 0.0;
  for (long i = threadIdx.x; i < rows; i += blockDim.x) {
    cx<E> r = R[b * ldr + i], u = U[b * ldu + i];
    const double dr = double(r.x) - l * double(u.x), di = double(r.y) - l * double(u.y);
    acc += dr * dr + di * di;
  }
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) s[threadIdx.x] += s[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[b] = sqrt(s[0]);
}

__global__ void k_rr_scale(int n, const c128* S, double* d, int* bad) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const double s = S[i + long(i) * n].x;
    if (!(s > 0.0) || !isfinite(s)) { bad[0] = 1; d[i] = 1.0; }
    else d[i] = 1.0 / sqrt(s);
  }
}

// lower triangle <- d_i d_j (M_ij + conj(M_ji)) / 2 for H and S; upper triangle mirrored
__global__ void k_rr_sym(int n, c128* H, c128* S, const double* d, int* bad) {
  const long total = long(n) * n;
  for (long t = blockIdx.x * long(blockDim.x) + threadIdx.x; t < total; t += long(gridDim.x) * blockDim.x) {
    const int j = int(t / n), i = int(t - long(j) * n);
    if (i < j) continue;
    const double f = d[i] * d[j];
    c128 h1 = H[i + long(j) * n], h2 = H[j + long(i) * n];
    c128 s1 = S[i + long(j) * n], s2 = S[j + long(i) * n];
    c128 h = {0.5 * f * (h1.x + h2.x), 0.5 * f * (h1.y - h2.y)};
    c128 s = {0.5 * f * (s1.x + s2.x), 0.5 * f * (s1.y - s2.y)};
    if (i == j) { h.y = 0.0; s.y = 0.0; }
    if (!isfinite(h.x) || !isfinite(h.y) || !isfinite(s.x) || !isfinite(s.y)) bad[1] = 1;
    H[i + long(j) * n] = h;
    S[i + long(j) * n] = s;
    H[j + long(i) * n] = c128{h.x, -h.y};
    S[j + long(i) * n] = c128{s.x, -s.y};
  }
}

__global__ void k_scale_rows(int n, int ncols, c128* Z, long ldz, const double* d) {
  const long total = long(n) * ncols;
  for (long t = blockIdx.x * long(blockDim.x) + threadIdx.x; t < total; t += long(gridDim.x) * blockDim.x) {
    const long j = t / n, i = t - j * n;
    c128 v = Z[i + j * ldz];
    Z[i + j * ldz] = c128{v.x * d[i], v.y * d[i]};
  }
}

__global__ void k_herm_lower(int n, c128* A, long lda) {
  const long total = long(n) * n;
  for (long t = blockIdx.x * long(blockDim.x) + threadIdx.x; t < total; t += long(gridDim.x) * blockDim.x) {
    const int j = int(t / n), i = int(t - long(j) * n);
    if (i < j) {  // upper entry (i, j) <- conj(lower (j, i))
      c128 v = A[j + long(i) * lda];
      A[i + long(j) * lda] = c128{v.x, -v.y};
    } else if (i == j) {
      A[i + long(j) * lda].y = 0.0;
    }
  }
}

__global__ void k_capacitance(int n, const c128* G, const double* q, c128* C) {
  const long total = long(n) * n;
  for (long t = blockIdx.x * long(blockDim.x) + threadIdx.x; t < total; t += long(gridDim.x) * blockDim.x) {
    const int j = int(t / n), i = int(t - long(j) * n);
    c128 v = G[t];
    if (i == j) v.x += 1.0 / q[i];
    C[t] = v;
  }
}

template <typename T>
__global__ void k_transpose_v(int n, const double* V, T* Vt) {
  const long total = long(n) * n * n;
  for (long t = blockIdx.x * long(blockDim.x) + threadIdx.x; t < total; t += long(gridDim.x) * blockDim.x) {
    const long x = t % n, y = (t / n) % n, z = t / (long(n) * n);  // output index [z][y][x]
    Vt[t] = T(V[(x * n + y) * n + z]);
  }
}

template <typename E> __global__ void k_zero(cx<E>* p, long count) {
  for (long t = blockIdx.x * long(blockDim.x) + threadIdx.x; t < count; t += long(gridDim.x) * blockDim.x)
    p[t] = cx<E>{E(0), E(0)};
}

}  // namespace

hipError_t block_diag_apply(int nproj, int nb, const int4* pinfo, const double* D, const c128* in, long ldi,
                            c128* out, long ldo, hipStream_t st) {
  if (nproj <= 0 || nb <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_block_diag, dim3(nblocks(long(nproj) * nb)), dim3(256), 0, st, nproj, nb, pinfo, D, in, ldi, out, ldo);
  return hipGetLastError();
}

hipError_t block_inverse(int nproj, const int4* pinfo, const c128* C, long ldc, c128* Minv, int* bad, hipStream_t st) {
  if (nproj <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_block_inverse, dim3(nproj), dim3(256), 0, st, nproj, pinfo, C, ldc, Minv, bad);
  return hipGetLastError();
}
hipError_t block_diag_apply_c(int nproj, int nb, const int4* pinfo, const c128* M, const c128* in, long ldi, c128* out,
                              long ldo, bool accumulate, hipStream_t st) {
  if (nproj <= 0 || nb <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_block_diag_c, dim3(nblocks(long(nproj) * nb)), dim3(256), 0, st, nproj, nb, pinfo, M, in, ldi,
                     out, ldo, accumulate ? 1 : 0);
  return hipGetLastError();
}
hipError_t overlap_rhs(int nproj, int nb, const double* Q, const c128* Dp, long ldd, const c128* ploc, long ldl,
                       c128* u, long ldu, hipStream_t st) {
  if (nproj <= 0 || nb <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_overlap_rhs, dim3(nblocks(long(nproj) * nb)), dim3(256), 0, st, nproj, nb, Q, Dp, ldd, ploc, ldl,
                     u, ldu);
  return hipGetLastError();
}
hipError_t overlap_recur(int nproj, int nb, const double* Q, const c128* Dp, long ldd, const c128* w, long ldw,
                         double s1, double c, const c128* cur, long ldc, double s2, const c128* prev, long ldp,
                         c128* out, long ldo, hipStream_t st) {
  if (nproj <= 0 || nb <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_overlap_recur, dim3(nblocks(long(nproj) * nb)), dim3(256), 0, st, nproj, nb, Q, Dp, ldd, w, ldw,
                     s1, c, cur, ldc, s2, prev, ldp, out, ldo);
  return hipGetLastError();
}
hipError_t diag_apply(int nproj, int nb, const double* d, const c128* in, long ldi, c128* out, long ldo,
                      hipStream_t st) {
  if (nproj <= 0 || nb <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_diag, dim3(nblocks(long(nproj) * nb)), dim3(256), 0, st, nproj, nb, d, in, ldi, out, ldo);
  return hipGetLastError();
}

template <typename E>
hipError_t axpbypcz(long rows, int nb, double a, const cx<E>* x, long ldx, double b, const cx<E>* y, long ldy,
                    double c, const cx<E>* z, long ldz, cx<E>* out, long ldo, hipStream_t st) {
  if (rows <= 0 || nb <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_axpbypcz<E>), dim3(nblocks(rows * nb)), dim3(256), 0, st, rows, nb, a, x, ldx, b, y, ldy, c, z,
                     ldz, out, ldo);
  return hipGetLastError();
}

template <typename EO, typename EI>
hipError_t convert_copy(long rows, int nb, const cx<EI>* in, long ldi, cx<EO>* out, long ldo, hipStream_t st) {
  if (rows <= 0 || nb <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_convert<EO, EI>), dim3(nblocks(rows * nb)), dim3(256), 0, st, rows, nb, in, ldi, out, ldo);
  return hipGetLastError();
}

template <typename E>
hipError_t permute_cols(long rows, int ncols, const cx<E>* src, long lds, const int* sidx, cx<E>* dst, long ldd,
                        const int* didx, hipStream_t st) {
  if (rows <= 0 || ncols <= 0) return hipSuccess;
  if (ncols > 65535) return hipErrorInvalidValue;
  const long bx = std::min<long>((rows + 255) / 256, 64);
  hipLaunchKernelGGL((k_permute_cols<E>), dim3(unsigned(bx), unsigned(ncols)), dim3(256), 0, st, rows, ncols, src, lds,
                     sidx, dst, ldd, didx);
  return hipGetLastError();
}

template <typename E>
hipError_t col_dots(long rows, int nb, const cx<E>* x, long ldx, const cx<E>* y, long ldy, c128* out,
                    hipStream_t st) {
  if (nb <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_col_dots<E>), dim3(nb), dim3(256), 0, st, rows, x, ldx, y, ldy, out);
  return hipGetLastError();
}

template <typename E>
hipError_t col_resid_norms(long rows, int nb, const cx<E>* R, long ldr, const cx<E>* U, long ldu,
                           const double* lam, double* out, hipStream_t st) {
  if (nb <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_col_resid<E>), dim3(nb), dim3(256), 0, st, rows, R, ldr, U, ldu, lam, out);
  return hipGetLastError();
}

template <typename E>
hipError_t lobpcg_precondition(long rows, int nact, const E* kin, const cx<E>* X, const cx<E>* HX, const cx<E>* SX,
                               long ld, const double* lam, const int* act, cx<E>* W, long ldw, hipStream_t st) {
  if (nact <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_lobpcg_precond<E>), dim3(nact), dim3(256), 0, st, rows, kin, X, HX, SX, ld, lam, act, W, ldw);
  return hipGetLastError();
}
template hipError_t lobpcg_precondition<double>(long, int, const double*, const c128*, const c128*, const c128*, long,
                                                const double*, const int*, c128*, long, hipStream_t);
template hipError_t lobpcg_precondition<float>(long, int, const float*, const c64*, const c64*, const c64*, long,
                                               const double*, const int*, c64*, long, hipStream_t);
hipError_t scale_cols_isqrt(int n, int ncols, c128* Z, long ldz, const double* s, hipStream_t st) {
  if (n <= 0 || ncols <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scale_cols_isqrt, dim3(nblocks(long(n) * ncols)), dim3(256), 0, st, n, ncols, Z, ldz, s);
  return hipGetLastError();
}

__global__ void k_real_part(long rows, int cols, const c128* A, long lda, double* R, long ldr) {
  const long total = rows * cols;
  for (long t = blockIdx.x * long(blockDim.x) + threadIdx.x; t < total; t += long(gridDim.x) * blockDim.x) {
    const long j = t / rows, i = t - j * rows;
    R[i + j * ldr] = A[i + j * lda].x;
  }
}
__global__ void k_from_real(long rows, int cols, const double* R, long ldr, c128* A, long lda) {
  const long total = rows * cols;
  for (long t = blockIdx.x * long(blockDim.x) + threadIdx.x; t < total; t += long(gridDim.x) * blockDim.x) {
    const long j = t / rows, i = t - j * rows;
    A[i + j * lda] = c128{R[i + j * ldr], 0.0};
  }
}
hipError_t real_part(long rows, int cols, const c128* A, long lda, double* R, long ldr, hipStream_t st) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_real_part, dim3(nblocks(rows * cols)), dim3(256), 0, st, rows, cols, A, lda, R, ldr);
  return hipGetLastError();
}
hipError_t complex_from_real(long rows, int cols, const double* R, long ldr, c128* A, long lda, hipStream_t st) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_from_real, dim3(nblocks(rows * cols)), dim3(256), 0, st, rows, cols, R, ldr, A, lda);
  return hipGetLastError();
}

__global__ void k_flag_nonfinite(long rows, int cols, const c128* A, long lda, int* flag) {
  const long total = rows * cols;
  for (long t = blockIdx.x * long(blockDim.x) + threadIdx.x; t < total; t += long(gridDim.x) * blockDim.x) {
    const long j = t / rows, i = t - j * rows;
    const c128 v = A[i + j * lda];
    if (!isfinite(v.x) || !isfinite(v.y)) flag[0] = 1;
  }
}
hipError_t flag_nonfinite(long rows, int cols, const c128* A, long lda, int* flag, hipStream_t st) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_flag_nonfinite, dim3(nblocks(rows * cols)), dim3(256), 0, st, rows, cols, A, lda, flag);
  return hipGetLastError();
}

__global__ void k_flag_nonfinite_real(long count, const double* x, int* flag) {
  for (long t = blockIdx.x * long(blockDim.x) + threadIdx.x; t < count; t += long(gridDim.x) * blockDim.x)
    if (!isfinite(x[t])) flag[0] = 1;
}
hipError_t flag_nonfinite_real(long count, const double* x, int* flag, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_flag_nonfinite_real, dim3(nblocks(count)), dim3(256), 0, st, count, x, flag);
  return hipGetLastError();
}

hipError_t rr_prepare(int n, c128* H, c128* S, double* d, int* bad, hipStream_t st) {
  hipLaunchKernelGGL(k_rr_scale, dim3(nblocks(n)), dim3(256), 0, st, n, S, d, bad);
  hipLaunchKernelGGL(k_rr_sym, dim3(nblocks(long(n) * n)), dim3(256), 0, st, n, H, S, d, bad);
  return hipGetLastError();
}

hipError_t scale_rows(int n, int ncols, c128* Z, long ldz, const double* d, hipStream_t st) {
  hipLaunchKernelGGL(k_scale_rows, dim3(nblocks(long(n) * ncols)), dim3(256), 0, st, n, ncols, Z, ldz, d);
  return hipGetLastError();
}

hipError_t hermitian_from_lower(int n, c128* A, long lda, hipStream_t st) {
  hipLaunchKernelGGL(k_herm_lower, dim3(nblocks(long(n) * n)), dim3(256), 0, st, n, A, lda);
  return hipGetLastError();
}

hipError_t capacitance(int n, const c128* G, const double* q, c128* C, hipStream_t st) {
  hipLaunchKernelGGL(k_capacitance, dim3(nblocks(long(n) * n)), dim3(256), 0, st, n, G, q, C);
  return hipGetLastError();
}

template <typename T> hipError_t transpose_potential(int n, const double* V, T* Vt, hipStream_t st) {
  hipLaunchKernelGGL((k_transpose_v<T>), dim3(nblocks(long(n) * n * n)), dim3(256), 0, st, n, V, Vt);
  return hipGetLastError();
}

template <typename E> hipError_t fill_zero(cx<E>* p, long count, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_zero<E>), dim3(nblocks(count)), dim3(256), 0, st, p, count);
  return hipGetLastError();
}

template hipError_t axpbypcz<double>(long, int, double, const c128*, long, double, const c128*, long, double,
                                     const c128*, long, c128*, long, hipStream_t);
template hipError_t axpbypcz<float>(long, int, double, const c64*, long, double, const c64*, long, double,
                                    const c64*, long, c64*, long, hipStream_t);
template hipError_t convert_copy<float, double>(long, int, const c128*, long, c64*, long, hipStream_t);
template hipError_t convert_copy<double, float>(long, int, const c64*, long, c128*, long, hipStream_t);
template hipError_t convert_copy<double, double>(long, int, const c128*, long, c128*, long, hipStream_t);
template hipError_t convert_copy<float, float>(long, int, const c64*, long, c64*, long, hipStream_t);
template hipError_t col_dots<double>(long, int, const c128*, long, const c128*, long, c128*, hipStream_t);
template hipError_t col_dots<float>(long, int, const c64*, long, const c64*, long, c128*, hipStream_t);
template hipError_t col_resid_norms<double>(long, int, const c128*, long, const c128*, long, const double*, double*,
                                            hipStream_t);
template hipError_t col_resid_norms<float>(long, int, const c64*, long, const c64*, long, const double*, double*,
                                           hipStream_t);
template hipError_t transpose_potential<double>(int, const double*, double*, hipStream_t);
template hipError_t transpose_potential<float>(int, const double*, float*, hipStream_t);
template hipError_t fill_zero<double>(c128*, long, hipStream_t);
template hipError_t permute_cols<double>(long, int, const c128*, long, const int*, c128*, long, const int*, hipStream_t);
template hipError_t permute_cols<float>(long, int, const c64*, long, const int*, c64*, long, const int*, hipStream_t);
template hipError_t fill_zero<float>(c64*, long, hipStream_t);

}  // namespace chebfd

namespace chebfd {
namespace {
__global__ void k_sub_scaled_cols(int rows, int nb, const c128* a, const c128* b, const double* lam, c128* out) {
  const long total = long(rows) * nb;
  for (long t = blockIdx.x * long(blockDim.x) + threadIdx.x; t < total; t += long(gridDim.x) * blockDim.x) {
    const long j = t / rows;
    const c128 u = a[t], v = b[t];
    out[t] = c128{u.x - lam[j] * v.x, u.y - lam[j] * v.y};
  }
}
__global__ void k_ratio_real(int nb, const c128* a, const c128* b, double* out) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nb; i += gridDim.x * blockDim.x) out[i] = a[i].x / b[i].x;
}
}  // namespace

hipError_t sub_scaled_cols(int rows, int nb, const c128* a, const c128* b, const double* lam, c128* out,
                           hipStream_t st) {
  if (rows <= 0 || nb <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sub_scaled_cols, dim3(nblocks(long(rows) * nb)), dim3(256), 0, st, rows, nb, a, b, lam, out);
  return hipGetLastError();
}
hipError_t ratio_real(int nb, const c128* a, const c128* b, double* out, hipStream_t st) {
  if (nb <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ratio_real, dim3(nblocks(nb)), dim3(256), 0, st, nb, a, b, out);
  return hipGetLastError();
}
}  // namespace chebfd

namespace chebfd {
namespace {
__global__ void k_block_grad(int dsize, const int2* __restrict__ dent, int nb, const c128* __restrict__ x, long ldx,
                             const c128* __restrict__ y, long ldy, const double* __restrict__ wts, double alpha,
                             double* __restrict__ out) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < dsize; e += gridDim.x * blockDim.x) {
    const int k = dent[e].x, l = dent[e].y;
    double s = 0.0;
    for (int b = 0; b < nb; ++b) {
      const c128 xk = x[b * ldx + k], xl = x[b * ldx + l], yk = y[b * ldy + k], yl = y[b * ldy + l];
      const double v = xk.x * yl.x + xk.y * yl.y + xl.x * yk.x + xl.y * yk.y;
      s += wts ? wts[b] * v : v;
    }
    out[e] += alpha * s;
  }
}
__global__ void k_weighted_adjoint(int nk, int nb, const double* w, const c128* Z, long ldz, c128* B) {
  const long total = long(nk) * nb;
  for (long t = blockIdx.x * long(blockDim.x) + threadIdx.x; t < total; t += long(gridDim.x) * blockDim.x) {
    const int j = int(t / nk), i = int(t - long(j) * nk);
    const c128 z = Z[j + i * ldz];
    B[t] = c128{w[i] * z.x, -w[i] * z.y};
  }
}
template <typename E>
__global__ void k_sub_lambda(long rows, int ncols, cx<E>* R, long ldr, const cx<E>* U, long ldu, const double* lam) {
  const long total = rows * ncols;
  for (long t = blockIdx.x * long(blockDim.x) + threadIdx.x; t < total; t += long(gridDim.x) * blockDim.x) {
    const long j = t / rows, i = t - j * rows;
    const cx<E> r = R[j * ldr + i], u = U[j * ldu + i];
    const double l = lam[j];
    R[j * ldr + i] = cx<E>{E(double(r.x) - l * double(u.x)), E(double(r.y) - l * double(u.y))};
  }
}
template <typename E> __global__ void k_zero_real(E* p, long count) {
  for (long t = blockIdx.x * long(blockDim.x) + threadIdx.x; t < count; t += long(gridDim.x) * blockDim.x) p[t] = E(0);
}
}  // namespace

hipError_t block_grad(int dsize, const int2* dent, int nb, const c128* x, long ldx, const c128* y, long ldy,
                      const double* wts, double alpha, double* out, hipStream_t st) {
  if (dsize <= 0 || nb <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_block_grad, dim3(nblocks(dsize)), dim3(256), 0, st, dsize, dent, nb, x, ldx, y, ldy, wts, alpha, out);
  return hipGetLastError();
}
hipError_t weighted_adjoint(int nk, int nb, const double* w, const c128* Z, long ldz, c128* B, hipStream_t st) {
  if (nk <= 0 || nb <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_weighted_adjoint, dim3(nblocks(long(nk) * nb)), dim3(256), 0, st, nk, nb, w, Z, ldz, B);
  return hipGetLastError();
}
template <typename E>
hipError_t sub_lambda_cols(long rows, int ncols, cx<E>* R, long ldr, const cx<E>* U, long ldu, const double* lam,
                           hipStream_t st) {
  if (rows <= 0 || ncols <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_sub_lambda<E>), dim3(nblocks(rows * ncols)), dim3(256), 0, st, rows, ncols, R, ldr, U, ldu, lam);
  return hipGetLastError();
}
template <typename E> hipError_t fill_zero_real(E* p, long count, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_zero_real<E>), dim3(nblocks(count)), dim3(256), 0, st, p, count);
  return hipGetLastError();
}
template hipError_t sub_lambda_cols<double>(long, int, c128*, long, const c128*, long, const double*, hipStream_t);
template hipError_t sub_lambda_cols<float>(long, int, c64*, long, const c64*, long, const double*, hipStream_t);
template hipError_t fill_zero_real<double>(double*, long, hipStream_t);
template hipError_t fill_zero_real<int>(int*, long, hipStream_t);
}  // namespace chebfd

// ---- warm-started refinement of the dense generalized eigenproblem (Rayleigh-Ritz) -----------------------
namespace chebfd {
namespace {
// M1 = X^H S X, M2 = X^H H X (n x n). lam_i = Re M2_ii / Re M1_ii; F_ij = (M2_ij - lam_j M1_ij) / (lam_j - lam_i)
// for i != j, F_ii = (1 - M1_ii) / 2. absF[t] = |F_t| (off-diagonal) for the convergence test; pairs closer
// than the resolution threshold get F_ij = -M1_ij / 2 and a nonzero absF if their coupling is not negligible.
// maximum that keeps a NaN (fmax would drop it)
__device__ __forceinline__ double max_nan(double a, double b) { return (a != a || b != b) ? a + b : fmax(a, b); }

__global__ __launch_bounds__(256) void k_refine_update(int n, const c128* M1, long ld1, const c128* M2, long ld2, c128* F,
                                                      double* lam, double* absF, double* bmax) {
  __shared__ double red[256];
  double mx = 0.0;
  const long total = long(n) * n;
  for (long t = blockIdx.x * long(blockDim.x) + threadIdx.x; t < total; t += long(gridDim.x) * blockDim.x) {
    const int j = int(t / n), i = int(t - long(j) * n);
    const double li = M2[i + long(i) * ld2].x / M1[i + long(i) * ld1].x;
    const double lj = M2[j + long(j) * ld2].x / M1[j + long(j) * ld1].x;
    const c128 m1 = M1[i + long(j) * ld1], m2 = M2[i + long(j) * ld2];
    if (i == j) {
      lam[i] = li;
      F[t] = c128{0.5 * (1.0 - m1.x), 0.0};
      absF[t] = 0.0;
      continue;
    }
    const double nr = m2.x - lj * m1.x, ni = m2.y - lj * m1.y;
    const double gap = lj - li;
    const double scale = fmax(1.0, fmax(fabs(li), fabs(lj)));
    if (fabs(gap) > 1e-9 * scale) {
      F[t] = c128{nr / gap, ni / gap};
      absF[t] = sqrt(nr * nr + ni * ni) / fabs(gap);
      mx = max_nan(mx, absF[t]);
    } else {
      F[t] = c128{-0.5 * m1.x, -0.5 * m1.y};
      const double cpl = sqrt(nr * nr + ni * ni);
      absF[t] = cpl > 1e-13 * scale ? 1e300 : 0.0;  // unresolvable near-degenerate coupling
      mx = max_nan(mx, absF[t]);
    }
  }
  // per-block maximum, fixed-order tree
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] = max_nan(red[threadIdx.x], red[threadIdx.x + k]);
    __syncthreads();
  }
  if (threadIdx.x == 0) bmax[blockIdx.x] = red[0];
}

// res[0] = max |M1 - I|, res[1] = max_{i != j} |M2_ij| / max(1, max_i |M2_ii|)  (one block, fixed order)
// Per-block maxima of |M1 - I|^2, of |M2_ij|^2 off the diagonal and of |M2_ii|, three per block (NaN kept)
__global__ __launch_bounds__(256) void k_refine_check(int n, const c128* M1, long ld1, const c128* M2, long ld2,
                                                     double* part) {
  __shared__ double s1[256], s2[256], s3[256];
  double a = 0.0, b = 0.0, d = 0.0;
  const long total = long(n) * n;
  for (long t = blockIdx.x * long(blockDim.x) + threadIdx.x; t < total; t += long(gridDim.x) * blockDim.x) {
    const int j = int(t / n), i = int(t - long(j) * n);
    const c128 m1 = M1[i + long(j) * ld1], m2 = M2[i + long(j) * ld2];
    const double r1 = i == j ? m1.x - 1.0 : m1.x;
    a = max_nan(a, r1 * r1 + m1.y * m1.y);
    if (i == j) d = max_nan(d, fabs(m2.x)); else b = max_nan(b, m2.x * m2.x + m2.y * m2.y);
  }
  s1[threadIdx.x] = a; s2[threadIdx.x] = b; s3[threadIdx.x] = d;
  __syncthreads();
  for (int k = blockDim.x / 2; k > 0; k >>= 1) {
    if (threadIdx.x < k) {
      s1[threadIdx.x] = max_nan(s1[threadIdx.x], s1[threadIdx.x + k]);
      s2[threadIdx.x] = max_nan(s2[threadIdx.x], s2[threadIdx.x + k]);
      s3[threadIdx.x] = max_nan(s3[threadIdx.x], s3[threadIdx.x + k]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[3 * blockIdx.x] = s1[0];
    part[3 * blockIdx.x + 1] = s2[0];
    part[3 * blockIdx.x + 2] = s3[0];
  }
}
__global__ void k_refine_check_final(int nblk, const double* part, double* res) {
  if (threadIdx.x != 0) return;
  double a = 0.0, b = 0.0, d = 0.0;
  for (int k = 0; k < nblk; ++k) {
    a = max_nan(a, part[3 * k]);
    b = max_nan(b, part[3 * k + 1]);
    d = max_nan(d, part[3 * k + 2]);
  }
  res[0] = sqrt(a);
  res[1] = sqrt(b) / fmax(1.0, d);
}

// out[0] = max of x[0..count) (one block, fixed order)
__global__ void k_identity(int n, c128* X) {
  const long total = long(n) * n;
  for (long t = blockIdx.x * long(blockDim.x) + threadIdx.x; t < total; t += long(gridDim.x) * blockDim.x) {
    const long j = t / n, i = t - j * n;
    X[t] = c128{i == j ? 1.0 : 0.0, 0.0};
  }
}

// Ascending sort of lam (n <= 2048) with its permutation, one block: element i goes to rank #{j : key_j < key_i
// or key_j = key_i and j < i}, so ties keep index order (NaN keys count as +Inf). Then ritz[k] = lam[perm[k]].
__global__ __launch_bounds__(1024) void k_sort_lam(int n, const double* lam, double* ritz, int* perm) {
  __shared__ double key[2048];
  for (int t = threadIdx.x; t < n; t += blockDim.x) key[t] = isnan(lam[t]) ? INFINITY : lam[t];
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double ki = key[i];
    int r = 0;
    for (int j = 0; j < n; ++j) r += key[j] < ki || (key[j] == ki && j < i);
    ritz[r] = lam[i];
    perm[r] = i;
  }
}

// Z[:, k] = d .* X[:, perm[k]]  (undoes the symmetric column scaling and applies the sort)
__global__ void k_permute_scale(int n, const c128* X, const int* perm, const double* d, c128* Z) {
  const long total = long(n) * n;
  for (long t = blockIdx.x * long(blockDim.x) + threadIdx.x; t < total; t += long(gridDim.x) * blockDim.x) {
    const long k = t / n, i = t - k * n;
    const c128 v = X[i + long(perm[k]) * n];
    Z[t] = c128{v.x * d[i], v.y * d[i]};
  }
}
}  // namespace

int refine_blocks(int n) { return nblocks(long(n) * n, 256, kRefineBlocksMax); }

hipError_t refine_update(int n, const c128* M1, long ld1, const c128* M2, long ld2, c128* F, double* lam, double* absF,
                         double* bmax, hipStream_t st) {
  hipLaunchKernelGGL(k_refine_update, dim3(refine_blocks(n)), dim3(256), 0, st, n, M1, ld1, M2, ld2, F, lam, absF, bmax);
  return hipGetLastError();
}
hipError_t refine_check(int n, const c128* M1, long ld1, const c128* M2, long ld2, double* part, double* res,
                        hipStream_t st) {
  const int nblk = nblocks(long(n) * n, 256, kRefineCheckBlocks);
  hipLaunchKernelGGL(k_refine_check, dim3(nblk), dim3(256), 0, st, n, M1, ld1, M2, ld2, part);
  hipLaunchKernelGGL(k_refine_check_final, dim3(1), dim3(64), 0, st, nblk, part, res);
  return hipGetLastError();
}
hipError_t identity_matrix(int n, c128* X, hipStream_t st) {
  hipLaunchKernelGGL(k_identity, dim3(nblocks(long(n) * n)), dim3(256), 0, st, n, X);
  return hipGetLastError();
}
hipError_t sort_eigen(int n, const double* lam, double* ritz, int* perm, const c128* X, const double* d, c128* Z,
                      hipStream_t st) {
  if (n > 2048) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_sort_lam, dim3(1), dim3(1024), 0, st, n, lam, ritz, perm);
  hipLaunchKernelGGL(k_permute_scale, dim3(nblocks(long(n) * n)), dim3(256), 0, st, n, X, perm, d, Z);
  return hipGetLastError();
}
}  // namespace chebfd

namespace chebfd {
namespace {
// out[j] = ||a_j - b_j|| / ||b_j|| for the columns of two projector-space blocks (one block per column, fixed-order
// tree sum, so the result does not depend on timing)
__global__ __launch_bounds__(256) void k_col_rel_diff(int rows, const c128* __restrict__ a, long lda,
                                                      const c128* __restrict__ b, long ldb, double* __restrict__ out) {
  __shared__ double sd[256], sb[256];
  const c128* ac = a + long(blockIdx.x) * lda;
  const c128* bc = b + long(blockIdx.x) * ldb;
  double d2 = 0.0, b2 = 0.0;
  for (int i = threadIdx.x; i < rows; i += 256) {
    const c128 x = ac[i], y = bc[i];
    const double dr = x.x - y.x, di = x.y - y.y;
    d2 += dr * dr + di * di;
    b2 += y.x * y.x + y.y * y.y;
  }
  sd[threadIdx.x] = d2;
  sb[threadIdx.x] = b2;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (int(threadIdx.x) < s) {
      sd[threadIdx.x] += sd[threadIdx.x + s];
      sb[threadIdx.x] += sb[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = sb[0] > 0.0 ? sqrt(sd[0] / sb[0]) : (sd[0] > 0.0 ? 1.0 : 0.0);
}
}  // namespace

hipError_t col_rel_diff(int rows, int nb, const c128* a, long lda, const c128* b, long ldb, double* out,
                        hipStream_t st) {
  if (rows <= 0 || nb <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_col_rel_diff, dim3(nb), dim3(256), 0, st, rows, a, lda, b, ldb, out);
  return hipGetLastError();
}
}  // namespace chebfd

namespace chebfd {
namespace {
// s_b = (|psi_b|^2 / |a_b|^2)^(1/4), so that |s a| = |psi / s| (1 when either is zero or not finite)
__global__ void k_balance_scales(int nb, const c128* __restrict__ aa, const c128* __restrict__ pp, double* __restrict__ s) {
  for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < nb; b += gridDim.x * blockDim.x) {
    const double x = aa[b].x, y = pp[b].x;
    const double q = (x > 0.0 && y > 0.0) ? sqrt(sqrt(y / x)) : 1.0;
    s[b] = (q > 0.0 && q < 1e300) ? q : 1.0;
  }
}
}  // namespace

hipError_t balance_scales(int nb, const c128* aa, const c128* pp, double* s, hipStream_t st) {
  if (nb <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_balance_scales, dim3(nblocks(nb)), dim3(256), 0, st, nb, aa, pp, s);
  return hipGetLastError();
}
}  // namespace chebfd
