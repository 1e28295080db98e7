// Exact solves of strongly coupled clusters inside the warm-started Rayleigh-Ritz refinement (Sec. 3, the
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

constexpr int CNT = 256;
constexpr int CLD = kClusterMax + 1;  // LDS leading dimension (odd in 16-byte units)

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
  double* const rot = reinterpret_cast<double*>(V + kClusterMax * CLD);  // [kClusterMax / 2][5]: c, s, cos phi, sin phi, on
  int* const pq = reinterpret_cast<int*>(rot + 5 * (kClusterMax / 2));    // [kClusterMax / 2][2]
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
    if (tid == 0) {
      double dj = L[j + j * CLD].x;
      for (int k = 0; k < j; ++k) dj -= L[j + k * CLD].x * L[j + k * CLD].x + L[j + k * CLD].y * L[j + k * CLD].y;
      if (!(dj > 0.0)) { bad = 1; dj = 1.0; }
      L[j + j * CLD] = c128{sqrt(dj), 0.0};
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
  const int sp = s + (s & 1), np = sp / 2;
  for (int sweep = 0; sweep < 16; ++sweep) {
    // off-diagonal and diagonal mass (fixed-order reduction)
    double off2 = 0.0, dia2 = 0.0;
    for (int t = tid; t < s * s; t += CNT) {
      const int j = t / s, i = t - j * s;
      const c128 a = A[i + j * CLD];
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
      if (tid < np) {
        int a, b;
        if (tid == 0) { a = sp - 1; b = r; }
        else { a = (r + tid) % (sp - 1); b = (r - tid + (sp - 1)) % (sp - 1); }
        const int p = min(a, b), q = max(a, b);
        double* R = rot + 5 * tid;
        pq[2 * tid] = p;
        pq[2 * tid + 1] = q;
        R[4] = 0.0;
        if (q < s) {
          const c128 apq = A[p + q * CLD];
          const double mag = sqrt(apq.x * apq.x + apq.y * apq.y);
          const double app = A[p + p * CLD].x, aqq = A[q + q * CLD].x;
          if (mag > 1e-300 && mag > 1e-18 * sqrt(fabs(app * aqq))) {
            const double tau = (aqq - app) / (2.0 * mag);
            const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            const double cc = 1.0 / sqrt(1.0 + t * t);
            R[0] = cc;
            R[1] = t * cc;
            R[2] = apq.x / mag;  // e^{i phi} = a_pq / |a_pq|
            R[3] = apq.y / mag;
            R[4] = 1.0;
          }
        }
      }
      __syncthreads();
      // columns: A <- A U, V <- V U with U = [[c, s], [-s e^{-i phi}, c e^{-i phi}]] on (p, q)
      for (int t = tid; t < s * np; t += CNT) {
        const int k = t / s, i = t - k * s;
        const double* R = rot + 5 * k;
        if (R[4] == 0.0) continue;
        const int p = pq[2 * k], q = pq[2 * k + 1];
        const c128 em = c128{R[2], -R[3]};
        {
          const c128 x = A[i + p * CLD], y = cmul(A[i + q * CLD], em);
          A[i + p * CLD] = x * R[0] - y * R[1];
          A[i + q * CLD] = x * R[1] + y * R[0];
        }
        {
          const c128 x = V[i + p * CLD], y = cmul(V[i + q * CLD], em);
          V[i + p * CLD] = x * R[0] - y * R[1];
          V[i + q * CLD] = x * R[1] + y * R[0];
        }
      }
      __syncthreads();
      // rows: A <- U^H A, U^H = [[c, -s e^{i phi}], [s, c e^{i phi}]]
      for (int t = tid; t < s * np; t += CNT) {
        const int k = t / s, j = t - k * s;
        const double* R = rot + 5 * k;
        if (R[4] == 0.0) continue;
        const int p = pq[2 * k], q = pq[2 * k + 1];
        const c128 ep = c128{R[2], R[3]};
        const c128 x = A[p + j * CLD], y = cmul(ep, A[q + j * CLD]);
        A[p + j * CLD] = x * R[0] - y * R[1];
        A[q + j * CLD] = x * R[1] + y * R[0];
      }
      __syncthreads();
      if (tid < np && rot[5 * tid + 4] != 0.0) {
        const int p = pq[2 * tid], q = pq[2 * tid + 1];
        A[p + q * CLD] = c128{0.0, 0.0};
        A[q + p * CLD] = c128{0.0, 0.0};
        A[p + p * CLD].y = 0.0;
        A[q + q * CLD].y = 0.0;
      }
      __syncthreads();
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
  return size_t(3) * kClusterMax * CLD * sizeof(c128) + (kClusterMax / 2) * (5 * sizeof(double) + 2 * sizeof(int));
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
