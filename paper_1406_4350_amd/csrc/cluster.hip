// Exact solves of strongly coupled clusters inside the warm-started Rayleigh-Ritz refinement (Alg. 2, Sec. 4.2: the
// subspace eigenproblem H_Y z = lambda S_Y z).
//
// The refinement X <- X (I + F) takes first-order steps F_ij = (M2_ij - lambda_j M1_ij) / (lambda_j - lambda_i)
// in the basis of the previous Ritz vectors (M1 = X^H S' X, M2 = X^H H' X). Where Ritz values are close and
// coupled, F_ij is large and the step leaves the region where it converges. Such pairs form small clusters
// (connected components of the graph |F_ij| > tau); each cluster's pencil (M2_CC, M1_CC) is solved exactly in
// LDS by one workgroup (Cholesky of M1_CC, reduction to standard form, cyclic two-sided Jacobi rotations,
// back-substitution), and the block-diagonal Q of these eigenvectors (identity outside the clusters) rotates
// X <- X Q. The first-order steps then resume.
#include "kernels.h"

namespace chebfd {
namespace {

constexpr int CNT = 512;  // one pass over the 2 x 2 blocks and V rows of a round up to clusters of about 30
constexpr int CLD = kClusterMax + 1;  // LDS leading dimension (odd in 16-byte units)
static_assert(kClusterMax <= 64, "the Cholesky diagonal sums one term per lane of a wave");

// bits[i * W + w] bit b: |F_ij| > tau for j = 32 w + b, i != j (W = ceil(n / 32))
__global__ void k_coupling_bits(int n, const double* __restrict__ absF, double tau, unsigned* __restrict__ bits) {
  const int W = (n + 31) / 32;
  const long total = long(n) * W;
  for (long t = blockIdx.x * long(blockDim.x) + threadIdx.x; t < total; t += long(gridDim.x) * blockDim.x) {
    const int w = int(t / n), i = int(t - long(w) * n);
    unsigned word = 0;
    for (int b = 0; b < 32; ++b) {
      const int j = 32 * w + b;
      if (j < n && j != i && absF[i + long(j) * n] > tau) word |= 1u << b;
    }
    bits[long(i) * W + w] = word;
  }
}

__device__ __forceinline__ c128 conjc(c128 a) { return c128{a.x, -a.y}; }

// X <- L^-1 X for lower-triangular L (s x s, real diagonal), row by row: after row i is final, every thread
// updates its entries of the rows below
__device__ void forward_solve(const c128* L, c128* X, int s, int tid) {
  for (int i = 0; i < s; ++i) {
    const double inv = 1.0 / L[i + i * CLD].x;
    for (int j = tid; j < s; j += CNT) X[i + j * CLD] = X[i + j * CLD] * inv;
    __syncthreads();
    const int rows = s - 1 - i;
    for (int t = tid; t < rows * s; t += CNT) {
      const int j = t / rows, k = i + 1 + (t - j * rows);
      X[k + j * CLD] = X[k + j * CLD] - cmul(L[k + i * CLD], X[i + j * CLD]);
    }
    __syncthreads();
  }
}

// One cluster per workgroup: members idx[off[c] .. off[c+1]), 2 <= size <= kClusterMax. Q (ldq) must hold
// the identity outside the clusters; this kernel writes the cluster blocks. flag[0] = 1 if some M1_CC is not
// positive definite.
__global__ __launch_bounds__(CNT) void k_cluster_eig(const c128* __restrict__ M1, long ld1, const c128* __restrict__ M2,
                                                     long ld2, const int* __restrict__ idx, const int* __restrict__ off,
                                                     c128* __restrict__ Q, long ldq, int* __restrict__ flag) {
  extern __shared__ unsigned char smem_raw[];
  c128* const A = reinterpret_cast<c128*>(smem_raw);  // [s][CLD] column-major
  c128* const L = A + kClusterMax * CLD;
  c128* const V = L + kClusterMax * CLD;
  c128* const A2 = V + kClusterMax * CLD;  // second buffer of the Jacobi rounds
  double* const rot = reinterpret_cast<double*>(A2 + kClusterMax * CLD);  // [kClusterMax / 2][4]: c, s, e^{i phi}
  int* const pq = reinterpret_cast<int*>(rot + 4 * (kClusterMax / 2));      // [kClusterMax / 2][3]: p, q, on
  __shared__ int bad;
  __shared__ double sums[2 * (CNT / 64)];
  const int c0 = off[blockIdx.x], s = off[blockIdx.x + 1] - c0;
  const int tid = threadIdx.x;
  if (tid == 0) bad = 0;
  for (int t = tid; t < s * s; t += CNT) {
    const int j = t / s, i = t - j * s;
    const long gi = idx[c0 + i], gj = idx[c0 + j];
    L[i + j * CLD] = M1[gi + gj * ld1];
    A[i + j * CLD] = M2[gi + gj * ld2];
  }
  __syncthreads();

  // ---- Cholesky M1_CC = L L^H (lower, left-looking) ----
  for (int j = 0; j < s; ++j) {
    if (tid < 64) {  // d_j = M1_jj - sum_k<j |L_jk|^2: one term per lane (s <= 64), fixed-order shuffle sum
      double q = 0.0;
      if (tid < j) q = L[j + tid * CLD].x * L[j + tid * CLD].x + L[j + tid * CLD].y * L[j + tid * CLD].y;
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) q += __shfl_xor(q, o, 64);
      if (tid == 0) {
        double dj = L[j + j * CLD].x - q;
        if (!(dj > 0.0)) { bad = 1; dj = 1.0; }
        L[j + j * CLD] = c128{sqrt(dj), 0.0};
      }
    }
    __syncthreads();
    const double ljj = L[j + j * CLD].x;
    for (int i = j + 1 + tid; i < s; i += CNT) {
      c128 x = L[i + j * CLD];
      for (int k = 0; k < j; ++k) x = x - cmulc(L[i + k * CLD], L[j + k * CLD]);
      L[i + j * CLD] = x * (1.0 / ljj);
    }
    __syncthreads();
  }
  if (bad) {
    if (tid == 0) flag[0] = 1;
    return;  // uniform: bad is read after the last barrier
  }

  // ---- standard form A <- L^-1 M2 L^-H: W = L^-1 M2 (in A), V = L^-1 W^H = A_std^H, A = Hermitian part ----
  forward_solve(L, A, s, tid);
  for (int t = tid; t < s * s; t += CNT) {
    const int j = t / s, i = t - j * s;
    V[i + j * CLD] = conjc(A[j + i * CLD]);
  }
  __syncthreads();
  forward_solve(L, V, s, tid);
  for (int t = tid; t < s * s; t += CNT) {
    const int j = t / s, i = t - j * s;
    const c128 a = V[i + j * CLD], b = conjc(V[j + i * CLD]);
    A[i + j * CLD] = i == j ? c128{a.x, 0.0} : (a + b) * 0.5;
  }
  __syncthreads();
  for (int t = tid; t < s * s; t += CNT) {
    const int j = t / s, i = t - j * s;
    V[i + j * CLD] = c128{i == j ? 1.0 : 0.0, 0.0};
  }
  __syncthreads();

  // ---- cyclic Jacobi, round-robin pairs (circle method over sp = s rounded up to even players) ----
  // A round applies A <- U^H A U and V <- V U for the sp / 2 disjoint rotations of the round, all computed from
  // the round's input matrix: the update splits into independent 2 x 2 blocks (rows of one rotation, columns of
  // another) read from one buffer and written to the other. Two barriers per round: after the rotations, after
  // the update.
  const int sp = s + (s & 1), np = sp / 2;
  c128* Ac = A;
  c128* An = A2;
  for (int sweep = 0; sweep < 16; ++sweep) {
    // off-diagonal and diagonal mass (fixed-order reduction)
    double off2 = 0.0, dia2 = 0.0;
    for (int t = tid; t < s * s; t += CNT) {
      const int j = t / s, i = t - j * s;
      const c128 a = Ac[i + j * CLD];
      if (i == j) dia2 += a.x * a.x; else off2 += a.x * a.x + a.y * a.y;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) { off2 += __shfl_xor(off2, o, 64); dia2 += __shfl_xor(dia2, o, 64); }
    if ((tid & 63) == 0) { sums[2 * (tid >> 6)] = off2; sums[2 * (tid >> 6) + 1] = dia2; }
    __syncthreads();
    off2 = 0.0; dia2 = 0.0;
    for (int w = 0; w < CNT / 64; ++w) { off2 += sums[2 * w]; dia2 += sums[2 * w + 1]; }
    __syncthreads();
    // relative 1e-12 suffices: the first-order steps that follow converge quadratically from there
    if (off2 <= 1e-24 * fmax(off2 + dia2, 1e-300)) break;  // uniform
    for (int r = 0; r < sp - 1; ++r) {
      // rotation k of this round: U = [[c, s], [-s e^{-i phi}, c e^{-i phi}]] zeroing (p, q); q == s is the idle
      // player of an odd s
      if (tid < np) {
        int a, b;
        if (tid == 0) { a = sp - 1; b = r; }
        else { a = (r + tid) % (sp - 1); b = (r - tid + (sp - 1)) % (sp - 1); }
        const int p = min(a, b), q = max(a, b);
        double* R = rot + 4 * tid;
        int on = 0;
        if (q < s) {
          const c128 apq = Ac[p + q * CLD];
          const double m2 = apq.x * apq.x + apq.y * apq.y;
          const double app = Ac[p + p * CLD].x, aqq = Ac[q + q * CLD].x;
          // |a_pq| above 1e-150 and 1e-18 sqrt|a_pp a_qq| (squared comparisons)
          if (m2 > 1e-300 && m2 > 1e-36 * fabs(app * aqq)) {
            const double ri = rsqrt(m2);  // 1 / |a_pq|
            const double tau = 0.5 * (aqq - app) * ri;
            const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            const double cc = rsqrt(1.0 + t * t);
            R[0] = cc;
            R[1] = t * cc;
            R[2] = apq.x * ri;  // e^{i phi} = a_pq / |a_pq|
            R[3] = apq.y * ri;
            on = 1;
          }
        }
        pq[3 * tid] = p;
        pq[3 * tid + 1] = q;
        pq[3 * tid + 2] = on;
      }
      __syncthreads();
      for (int t = tid; t < np * np + s * np; t += CNT) {
        if (t < np * np) {
          // block rows {p, q} (rotation k), columns {p2, q2} (rotation k2); rows or columns >= s do not exist
          const int k = t / np, k2 = t - k * np;
          const int p = pq[3 * k], q = pq[3 * k + 1], p2 = pq[3 * k2], q2 = pq[3 * k2 + 1];
          const bool qr = q < s, qc = q2 < s;
          // loads at clamped in-range indices and selects of the loaded values (a conditional between two
          // lvalues would select addresses instead)
          const int qq = qr ? q : p, qq2 = qc ? q2 : p2;
          const c128 l01 = Ac[p + qq2 * CLD], l10 = Ac[qq + p2 * CLD], l11 = Ac[qq + qq2 * CLD];
          c128 b00 = Ac[p + p2 * CLD];
          c128 b01 = qc ? l01 : c128{0.0, 0.0};
          c128 b10 = qr ? l10 : c128{0.0, 0.0};
          c128 b11 = qr && qc ? l11 : c128{0.0, 0.0};
          if (pq[3 * k2 + 2]) {  // columns: B <- B U
            const double* C = rot + 4 * k2;
            const c128 em = {C[2], -C[3]};
            const c128 y0 = cmul(b01, em), y1 = cmul(b11, em);
            const c128 n00 = b00 * C[0] - y0 * C[1], n01 = b00 * C[1] + y0 * C[0];
            const c128 n10 = b10 * C[0] - y1 * C[1], n11 = b10 * C[1] + y1 * C[0];
            b00 = n00; b01 = n01; b10 = n10; b11 = n11;
          }
          if (pq[3 * k + 2]) {  // rows: B <- U^H B, U^H = [[c, -s e^{i phi}], [s, c e^{i phi}]]
            const double* R = rot + 4 * k;
            const c128 ep = {R[2], R[3]};
            const c128 y0 = cmul(ep, b10), y1 = cmul(ep, b11);
            const c128 n00 = b00 * R[0] - y0 * R[1], n10 = b00 * R[1] + y0 * R[0];
            const c128 n01 = b01 * R[0] - y1 * R[1], n11 = b01 * R[1] + y1 * R[0];
            b00 = n00; b01 = n01; b10 = n10; b11 = n11;
            if (k == k2) {  // the rotated pair: exact zeros off the diagonal, real diagonal
              b01 = c128{0.0, 0.0};
              b10 = c128{0.0, 0.0};
              b00.y = 0.0;
              b11.y = 0.0;
            }
          }
          An[p + p2 * CLD] = b00;
          if (qc) An[p + q2 * CLD] = b01;
          if (qr) An[q + p2 * CLD] = b10;
          if (qr && qc) An[q + q2 * CLD] = b11;
        } else {
          // V <- V U on columns (p, q) of rotation k, row i
          const int u = t - np * np, k = u / s, i = u - k * s;
          if (pq[3 * k + 2]) {
            const int p = pq[3 * k], q = pq[3 * k + 1];
            const double* R = rot + 4 * k;
            const c128 em = {R[2], -R[3]};
            const c128 x = V[i + p * CLD], y = cmul(V[i + q * CLD], em);
            V[i + p * CLD] = x * R[0] - y * R[1];
            V[i + q * CLD] = x * R[1] + y * R[0];
          }
        }
      }
      __syncthreads();
      c128* const tmp = Ac;
      Ac = An;
      An = tmp;
    }
  }

  // ---- Z = L^-H V, scattered into Q ----
  for (int i = s - 1; i >= 0; --i) {
    const double inv = 1.0 / L[i + i * CLD].x;
    for (int j = tid; j < s; j += CNT) V[i + j * CLD] = V[i + j * CLD] * inv;
    __syncthreads();
    for (int t = tid; t < i * s; t += CNT) {
      const int j = t / i, k = t - j * i;
      V[k + j * CLD] = V[k + j * CLD] - cmul(conjc(L[i + k * CLD]), V[i + j * CLD]);
    }
    __syncthreads();
  }
  for (int t = tid; t < s * s; t += CNT) {
    const int j = t / s, i = t - j * s;
    Q[idx[c0 + i] + long(idx[c0 + j]) * ldq] = V[i + j * CLD];
  }
}

size_t cluster_lds() {
  return size_t(4) * kClusterMax * CLD * sizeof(c128) + (kClusterMax / 2) * (4 * sizeof(double) + 3 * sizeof(int));
}

}  // namespace

hipError_t coupling_bits(int n, const double* absF, double tau, unsigned* bits, hipStream_t st) {
  const long words = long(n) * ((n + 31) / 32);
  hipLaunchKernelGGL(k_coupling_bits, dim3(int(std::min<long>((words + 255) / 256, 4096))), dim3(256), 0, st, n, absF,
                     tau, bits);
  return hipGetLastError();
}

hipError_t cluster_eig(int nclusters, const c128* M1, long ld1, const c128* M2, long ld2, const int* idx, const int* off,
                       c128* Q, long ldq, int* flag, hipStream_t st) {
  if (nclusters <= 0) return hipSuccess;
  const size_t lds = cluster_lds();
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_cluster_eig),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_cluster_eig, dim3(nclusters), dim3(CNT), lds, st, M1, ld1, M2, ld2, idx, off, Q, ldq, flag);
  return hipGetLastError();
}

}  // namespace chebfd
