// Internal launchers of the chebfd HIP kernels (not part of the public C ABI).
#pragma once
#include "common.h"

namespace chebfd {

// Output epilogue shared by the GEMMs and the split-K reduction:
//   out = alpha * (A B) + bL * L + bU * U + bW * W      (element-wise, any of L/U/W may be null)
// `out` may alias W (the Chebyshev recurrence writes psi^i over psi^(i-2)).
template <typename E> struct Epi {
  cx<E>* out = nullptr; long ldo = 0;
  double alpha = 1.0;
  const cx<E>* L = nullptr; long ldl = 0; double bL = 0.0;
  const cx<E>* U = nullptr; long ldu = 0; double bU = 0.0;
  const cx<E>* W = nullptr; long ldw = 0; double bW = 0.0;
  bool real_only = false;  // keep the real part (inner products of real functions, Gamma point)
};

enum GemmMode { GEMM_CN = 0, GEMM_NN = 1 };
// separate kernel instances per use, so that profiles tell them apart
enum GemmRole { ROLE_SMALL = 0, ROLE_PROJECT = 1, ROLE_BACKPROJECT = 2, ROLE_SUBSPACE = 3 };

// C (M x N) = op(A) B, complex, column-major operands.
//   GEMM_CN: A stored K x M (lda), op = conjugate transpose;  GEMM_NN: A stored M x K (lda).
//   B stored K x N (ldb).
// T is the MFMA arithmetic type; EA/EB are the storage types of A and B (converted on load).
// splits > 1: K is split, FP64 partial products go to `part` (splits * M * N complex doubles) and a
// deterministic reduction applies the epilogue; splits == 1: the epilogue is applied directly.
// upper = true (M = N, a Hermitian result): only the 64 x 64 output tiles with row tile <= column tile are
// computed (the others are not written; hermitian_lower fills them), splits from gemm_upper_splits.
template <typename T, typename EA, typename EB, typename EO>
hipError_t gemm(GemmMode mode, int M, int N, int K, const cx<EA>* A, long lda, const cx<EB>* B, long ldb,
                const Epi<EO>& epi, int splits, c128* part, hipStream_t st, GemmRole role = ROLE_SMALL,
                bool upper = false);
int gemm_upper_splits(int N, int K);
// A[i][j] = conj(A[j][i]) for i > j (n x n, column-major)
hipError_t hermitian_lower(int n, c128* A, long lda, hipStream_t st);

// number of K splits the launcher would like for an (M, N, K) product on 256 CUs
int gemm_pick_splits(int M, int N, int K);

// ---- FP16 hi/lo split complex GEMM (FP32 accumulation) ---------------------------------------------------
// A is held as four FP16 planes (Re hi, Re lo, Im hi, Im lo) of sA * A, each row m holding its K values
// contiguously (row stride ld halves, a multiple of 8; K padded with zeros to a multiple of 32). sA is a power of
// two chosen so that max |sA A| is in [2^13, 2^14) (2^kHalfTopExp, near the top of the FP16 range):
// hi = fp16(sA a), lo = fp16(sA a - hi), so hi + lo carries about 22 significant bits for every entry down to
// about 2^-17 of the largest, both halves being normal FP16 numbers there. Products of such operands reach 2^28
// and their sums over K stay far inside the FP32 range of the accumulators.
constexpr int kHalfTopExp = 14;
struct HalfPlanes {
  const _Float16* p = nullptr;  // [4][rows][ld]: Re hi, Re lo, Im hi, Im lo
  long rows = 0, ld = 0;
  double inv_scale = 1.0;  // 1 / sA
};
// out (M x N) = op(A) B with op(A)[m][k] = A[m][k] (GEMM_NN) or conj(A[m][k]) (GEMM_CN, A = the conjugate-
// transposed operand stored row m = output row). B (K x N, column-major, ldb) is split on the fly after
// scaling column n by bscale[n] (a power of two, see column_scales); each product is hi*hi + hi*lo + lo*hi on
// the 16x16x32 FP16 MFMA. Splits and epilogue as for gemm().
template <typename EB, typename EO>
hipError_t gemm_h(GemmMode mode, int M, int N, int K, const HalfPlanes& A, const cx<EB>* B, long ldb,
                  const float* bscale, const Epi<EO>& epi, int splits, c128* part, hipStream_t st, GemmRole role);
// B split once, exactly as gemm_h splits it on the fly: planes [4][N][pld] of bscale[n] B[k][n] (Re hi, Re lo,
// Im hi, Im lo; zero for K <= k < pld), pld >= K a multiple of 32
hipError_t split_columns(int K, int N, const c128* B, long ldb, const float* bscale, _Float16* planes, long pld,
                         hipStream_t st);
hipError_t split_columns(int K, int N, const c64* B, long ldb, const float* bscale, _Float16* planes, long pld,
                         hipStream_t st);
// gemm_h with B given as such planes (Bp.rows = N, Bp.ld = pld, Bp.inv_scale unused); splits > 1 sums split-K
// partials in part as gemm_h does (same results as gemm_h with the same splits)
template <typename EO>
hipError_t gemm_h_pre(GemmMode mode, int M, int N, int K, const HalfPlanes& A, const HalfPlanes& Bp,
                      const float* bscale, const Epi<EO>& epi, int splits, c128* part, hipStream_t st, GemmRole role);
int gemm_h_pick_splits(int M, int N, int K);
// upper bound of both split rules, for sizing split-K partial buffers
int gemm_split_bound(int M, int N, int K);
// the work item (M tile bx, N tile by, split bz) the tiled kernels give block i of a `total`-block launch
void gemm_block_item(int i, int total, int tm, int tn, int grp, int& bx, int& by, int& bz);
// bscale[n] = 2^-e with max_k |B[k][n]| (over Re and Im) in [2^(e-1), 2^e); 1 for a zero column
template <typename E> hipError_t column_scales(long rows, int ncols, const cx<E>* B, long ldb, float* bscale,
                                               hipStream_t st);
// per-column max |Re|, |Im| of a complex128 matrix (FP64), for the global scale of the split planes
hipError_t column_maxabs(long rows, int ncols, const c128* X, long ldx, double* out, hipStream_t st);
// planes of sA * X for a complex128 X (rows_x x cols_x, ld ldx). transpose = false: plane row r = column r of X
// (k runs down X's column); transpose = true: plane row r = row r of X (k runs along X's row).
hipError_t split_planes(const c128* X, long ldx, int rows_x, int cols_x, bool transpose, double scale,
                        _Float16* planes, long prow, long pld, hipStream_t st);

// ---- FFT passes (per batch of bands) -------------------------------------------------------------------
struct FftGeom {
  int n, ncol, npw, rx;
  const int4* col;  // per column: {x-line index gx + rx, y = gy mod n, first sphere entry, length}
  const int* ent;   // per sphere entry: (column << 8) | (gz mod n)
  const int4* xline;  // per x-line xi = gx + rx: {first column, lowest gy, number of columns (consecutive gy), 0}
};
template <typename T>
hipError_t fft_col_inverse(const FftGeom& g, const cx<T>* tw, const cx<T>* X, long ldx, int nb, cx<T>* colbuf,
                           hipStream_t st);
template <typename T>
hipError_t fft_plane(const FftGeom& g, const cx<T>* tw, const T* Vt, const cx<T>* cin, cx<T>* cout, int nb,
                     hipStream_t st);
template <typename T>
hipError_t fft_col_forward(const FftGeom& g, const cx<T>* tw, const cx<T>* colbuf, const cx<T>* X, long ldx,
                           const T* kin, cx<T>* out, long ldo, int nb, hipStream_t st);
hipError_t fft_prepare_attributes();
// dV[x][y][z] += coef n^-3 sum_b w_b Re(conj(a_b(r)) psi_b(r)) for nband bands of z-transformed disk columns ca, cb
// (w = null: all weights 1); part: cross_density_part_doubles(n, nband) doubles of scratch. For n > 64 and ca != cb,
// scale[b] = (|psi_b| / |a_b|)^(1/2) balances the two fields of the polarisation form (balance_scales); else unused.
template <typename T>
hipError_t cross_density(const FftGeom& g, const cx<T>* tw, const cx<T>* ca, const cx<T>* cb, int nband,
                         const double* wts, const double* scale, double coef, double* part, double* dV,
                         hipStream_t st);
// s[b] = (pp[b].re / aa[b].re)^(1/4) from squared norms (col_dots of a with a and of psi with psi); 1 if degenerate
hipError_t balance_scales(int nb, const c128* aa, const c128* pp, double* s, hipStream_t st);
size_t cross_density_part_doubles(int n, int nband);
size_t fft_xdens_lds_bytes(int n, int rx, bool dbl);
// dynamic LDS bytes of the plane pass for box n, x-line half-width rx (0 if n unsupported)
size_t fft_plane_lds_bytes(int n, int rx, bool dbl);
// blocks of the plane pass resident on the current device at once (its persistent grid for large batches)
int fft_plane_blocks(int n, int rx, bool dbl);
// Row stride (in elements) of the disk-column buffers [band][z][column]: the column count rounded up to 16, so
// that every z-row starts on a 128-byte line (the column passes read 16 or 32 neighbouring columns of a row)
__host__ __device__ inline int col_stride(int ncol) { return (ncol + 15) & ~15; }
// Gamma point: U[:, j] = bands 2j + i 2j+1 expanded to the whole sphere (gmap: half index | conj << 30, h0 the
// half index of G = 0 or -1); out = the two bands separated from the transformed W, scaled back, + K X
template <typename T>
hipError_t gamma_pack(int npf, int nb, const int* gmap, int h0, const cx<T>* X, long ldx, cx<T>* U, long ldu,
                      hipStream_t st);
template <typename T>
hipError_t gamma_split(int nh, int nb, const int2* pair, int h0, const cx<T>* W, long ldw, const T* kin,
                       const cx<T>* X, long ldx, cx<T>* out, long ldo, hipStream_t st);

// ---- small projector-space and vector kernels -------------------------------------------------------------
// out[:, b] = blockdiag(D) in[:, b]; pinfo[i] = {first row of i's atom, block size, offset of the block in D}
hipError_t block_diag_apply(int nproj, int nb, const int4* pinfo, const double* D, const c128* in, long ldi,
                            c128* out, long ldo, hipStream_t st);
// out[i, b] = d[i] * in[i, b]
// Minv (packed like D, complex) = inverses of the atom diagonal blocks of the HPD matrix C (blocks up to 32;
// bad[0] = 1 otherwise). Preconditioner of the iterative capacitance solve (Sec. 5.1).
hipError_t block_inverse(int nproj, const int4* pinfo, const c128* C, long ldc, c128* Minv, int* bad, hipStream_t st);
// out = blockdiag(M) in (+ out if accumulate), complex packed blocks
hipError_t block_diag_apply_c(int nproj, int nb, const int4* pinfo, const c128* M, const c128* in, long ldi, c128* out,
                              long ldo, bool accumulate, hipStream_t st);
hipError_t diag_apply(int nproj, int nb, const double* d, const c128* in, long ldi, c128* out, long ldo,
                      hipStream_t st);
// Projector-space steps of the filter with an overlap (S = I + P Q P^H, Q diagonal, C = Q^-1 + P^H P):
// u = Q^-1 Dp - ploc (u may alias ploc), and out = s1 (Q^-1 (Dp - w) - c cur) - s2 prev (prev may be null)
hipError_t overlap_rhs(int nproj, int nb, const double* Q, const c128* Dp, long ldd, const c128* ploc, long ldl,
                       c128* u, long ldu, hipStream_t st);
hipError_t overlap_recur(int nproj, int nb, const double* Q, const c128* Dp, long ldd, const c128* w, long ldw,
                         double s1, double c, const c128* cur, long ldc, double s2, const c128* prev, long ldp,
                         c128* out, long ldo, hipStream_t st);
// out = a x + b y (+ c z), complex, any storage type
template <typename E>
hipError_t axpbypcz(long rows, int nb, double a, const cx<E>* x, long ldx, double b, const cx<E>* y, long ldy,
                    double c, const cx<E>* z, long ldz, cx<E>* out, long ldo, hipStream_t st);
template <typename EO, typename EI>
hipError_t convert_copy(long rows, int nb, const cx<EI>* in, long ldi, cx<EO>* out, long ldo, hipStream_t st);
// per column: out[b] = sum_i conj(x[i,b]) y[i,b]  (deterministic, FP64 accumulation)
template <typename E>
hipError_t col_dots(long rows, int nb, const cx<E>* x, long ldx, const cx<E>* y, long ldy, c128* out,
                    hipStream_t st);
// per column: out[b] = || R[:, b] - lam[b] U[:, b] ||_2
template <typename E>
hipError_t col_resid_norms(long rows, int nb, const cx<E>* R, long ldr, const cx<E>* U, long ldu,
                           const double* lam, double* out, hipStream_t st);
// H, S (n x n): symmetric scaling by 1/sqrt(S_ii), Hermitisation; writes scale d; bad[0] = 1 if some
// S_ii is not positive, bad[1] = 1 if an entry is not finite (plain stores, bad must be cleared first)
hipError_t rr_prepare(int n, c128* H, c128* S, double* d, int* bad, hipStream_t st);
// Z[i, j] *= d[i]
hipError_t scale_rows(int n, int ncols, c128* Z, long ldz, const double* d, hipStream_t st);
// full Hermitian matrix from its lower triangle
hipError_t hermitian_from_lower(int n, c128* A, long lda, hipStream_t st);
// C = diag(1/q) + G
hipError_t capacitance(int n, const c128* G, const double* q, c128* C, hipStream_t st);
// V [x][y][z] (FP64) -> Vt [z][y][x] in T
template <typename T> hipError_t transpose_potential(int n, const double* V, T* Vt, hipStream_t st);
template <typename E> hipError_t fill_zero(cx<E>* p, long count, hipStream_t st);
// dst[:, didx ? didx[j] : j] = src[:, sidx ? sidx[j] : j] for j < ncols (gather / scatter of band columns)
template <typename E>
hipError_t permute_cols(long rows, int ncols, const cx<E>* src, long lds, const int* sidx, cx<E>* dst, long ldd,
                        const int* didx, hipStream_t st);
// out[:, j] = a[:, j] - lam[j] b[:, j]  (contiguous rows x nb, complex128)
hipError_t sub_scaled_cols(int rows, int nb, const c128* a, const c128* b, const double* lam, c128* out,
                           hipStream_t st);
// out[e] += alpha sum_b w_b Re(conj(x[k,b]) y[l,b] + conj(x[l,b]) y[k,b]) for packed block entry e = (k, l)
hipError_t block_grad(int dsize, const int2* dent, int nb, const c128* x, long ldx, const c128* y, long ldy,
                      const double* wts, double alpha, double* out, hipStream_t st);
// B[i + j nk] = w_i conj(Z[j + i ldz]), i < nk, j < nb
hipError_t weighted_adjoint(int nk, int nb, const double* w, const c128* Z, long ldz, c128* B, hipStream_t st);
// R[:, i] -= lam[i] U[:, i] for i < ncols
template <typename E>
hipError_t sub_lambda_cols(long rows, int ncols, cx<E>* R, long ldr, const cx<E>* U, long ldu, const double* lam,
                           hipStream_t st);
template <typename E> hipError_t fill_zero_real(E* p, long count, hipStream_t st);
// Warm-started refinement of H X = S X Lambda (n x n, FP64): given M1 = X^H S X, M2 = X^H H X, the correction
// X <- X (I + F) with F_ij = (M2_ij - lam_j M1_ij)/(lam_j - lam_i), F_ii = (1 - M1_ii)/2, lam_i = M2_ii/M1_ii;
// absF = off-diagonal |F| (1e300 for an unresolvable near-degenerate pair); bmax[b] = the maximum of block b's
// entries (NaN if one is NaN) for b < refine_blocks(n) <= kRefineBlocksMax
constexpr int kRefineBlocksMax = 256;
int refine_blocks(int n);
hipError_t refine_update(int n, const c128* M1, long ld1, const c128* M2, long ld2, c128* F, double* lam, double* absF,
                         double* bmax, hipStream_t st);
// res[0] = max |M1 - I|, res[1] = max off-diagonal |M2| / max(1, max |diag M2|) (NaN if an entry is NaN); part
// holds 3 kRefineCheckBlocks doubles of per-block maxima
constexpr int kRefineCheckBlocks = 64;
static_assert(3 * kRefineCheckBlocks <= kRefineBlocksMax, "the block maxima of the check fit the refinement's");
hipError_t refine_check(int n, const c128* M1, long ld1, const c128* M2, long ld2, double* part, double* res,
                        hipStream_t st);
hipError_t identity_matrix(int n, c128* X, hipStream_t st);
// ascending sort of lam (n <= 2048) -> ritz, perm; Z[:, k] = d .* X[:, perm[k]]
hipError_t sort_eigen(int n, const double* lam, double* ritz, int* perm, const c128* X, const double* d, c128* Z,
                      hipStream_t st);
// LOBPCG: W[:, j] = K(t / E_kin(x_a)) (HX - lambda_a SX)[:, a], a = act[j], with the rational kinetic
// preconditioner K(x) = (27 + 18x + 12x^2 + 8x^3) / (27 + 18x + 12x^2 + 8x^3 + 16x^4)
template <typename E>
hipError_t lobpcg_precondition(long rows, int nact, const E* kin, const cx<E>* X, const cx<E>* HX, const cx<E>* SX,
                               long ld, const double* lam, const int* act, cx<E>* W, long ldw, hipStream_t st);
// R = Re A; A = R + 0 i (real symmetric eigenproblems of the Gamma point)
hipError_t real_part(long rows, int cols, const c128* A, long lda, double* R, long ldr, hipStream_t st);
hipError_t complex_from_real(long rows, int cols, const double* R, long ldr, c128* A, long lda, hipStream_t st);
// flag[0] = 1 if any entry of A (rows x cols, ld lda) is NaN or Inf (plain stores of 1, no atomics)
hipError_t flag_nonfinite(long rows, int cols, const c128* A, long lda, int* flag, hipStream_t st);
// flag[0] = 1 if any of x[0 .. count) is NaN or Inf (plain stores of 1, no atomics)
hipError_t flag_nonfinite_real(long count, const double* x, int* flag, hipStream_t st);
// Z[:, j] *= 1 / sqrt(s[j])
hipError_t scale_cols_isqrt(int n, int ncols, c128* Z, long ldz, const double* s, hipStream_t st);
// out[i] = Re a[i] / Re b[i]
hipError_t ratio_real(int nb, const c128* a, const c128* b, double* out, hipStream_t st);
// out[j] = ||a_j - b_j|| / ||b_j|| over the rows of column j (projector-space blocks, FP64)
hipError_t col_rel_diff(int rows, int nb, const c128* a, long lda, const c128* b, long ldb, double* out,
                        hipStream_t st);

// Clusters of the Rayleigh-Ritz refinement: bits[i W + w] bit b set when |F_ij| > tau, j = 32 w + b, i != j
// (W = ceil(n / 32)). cluster_eig solves each cluster's pencil (M2_CC, M1_CC), members idx[off[c] ..
// off[c+1]) with 2 <= size <= kClusterMax, and writes its eigenvectors into the block (C, C) of Q, which must
// hold the identity elsewhere; flag[0] = 1 if an M1_CC is not positive definite.
constexpr int kClusterMax = 48;
hipError_t coupling_bits(int n, const double* absF, double tau, unsigned* bits, hipStream_t st);
hipError_t cluster_eig(int nclusters, const c128* M1, long ld1, const c128* M2, long ld2, const int* idx, const int* off,
                       c128* Q, long ldq, int* flag, hipStream_t st);

}  // namespace chebfd
