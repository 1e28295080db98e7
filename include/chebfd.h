/*
 * chebfd -- Chebyshev-filtered subspace iteration for the plane-wave generalized eigenproblem
 *           H x = lambda S x  (Levitt & Torrent, "Parallel eigensolvers in plane-wave Density
 *           Functional Theory", arXiv:1406.4350), on AMD Instinct MI355X (gfx950).
 *
 * Operators (Sec. 2.1):
 *   H = K + V_loc + P D P^H      (Eq. 2, Eq. 3)   K diagonal, V_loc a multiplication by V(r) in real
 *                                                  space done with a pair of FFTs (Alg. 1), D block-
 *                                                  diagonal over atoms (real symmetric blocks)
 *   S = I + P Q P^H              (Eq. 4)           Q diagonal; S = I for norm-conserving problems
 *   S^-1 = I - P (Q^-1 + P^H P)^-1 P^H            Woodbury form (Sec. 5.1)
 * The paper writes real wavefunctions and P^T; everything here is complex Hermitian (P^H, X^H).
 *
 * FFT convention: psi(r_j) = sum_i c_i exp(+2 pi i g_i.j/n),
 *                 (V_loc psi)_i = n^-3 sum_j exp(-2 pi i g_i.j/n) V_j psi(r_j).
 *
 * Layouts: a band block X is column-major, npw rows (sphere order) by nb columns, leading dimension
 * ldx >= npw, elements interleaved complex: complex128 (double re, im) when the plan precision is
 * CHEB_FP64, complex64 (float re, im) when it is CHEB_MIXED.
 *
 * Ownership: the caller owns every device buffer -- the plan's persistent buffer, the per-call workspace,
 * inputs and outputs. Host arrays passed to cheb_plan_create are copied. After cheb_plan_create the
 * library makes no device allocation of its own; the dense eigensolver runs inside the caller's
 * workspace.
 *
 * Streams: every call enqueues its work on the given stream and returns. Exceptions, which synchronize
 * the stream before returning: cheb_plan_create, cheb_set_projectors (factorisation status),
 * cheb_rayleigh_ritz (eigensolver status), cheb_upper_bound (scalars).
 *
 * Errors: every function returns a cheb_status; argument errors are found before any launch and leave
 * buffers untouched; cheb_last_error(plan) gives the message of the last failure on that plan. A plan is
 * not thread-safe; distinct plans are independent.
 */
#ifndef CHEBFD_H
#define CHEBFD_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cheb_plan_s* cheb_plan;

typedef enum {
  CHEB_OK = 0,
  CHEB_ERR_ARG = 1,          /* invalid argument (null, size, layout, unsupported box size) */
  CHEB_ERR_HIP = 2,          /* a HIP runtime / library call failed */
  CHEB_ERR_WORKSPACE = 3,    /* workspace or persistent buffer smaller than required */
  CHEB_ERR_NOT_PD = 4,       /* a matrix that must be Hermitian positive definite is not (S_X, capacitance) */
  CHEB_ERR_EIG = 5,          /* the dense eigensolver did not converge */
  CHEB_ERR_NONFINITE = 6,    /* NaN or Inf met in a subspace matrix */
  CHEB_ERR_STATE = 7,        /* potential, projectors or D not set yet */
  CHEB_ERR_HOST = 8          /* host-side failure (host memory exhausted); any call may return it */
} cheb_status;

typedef enum { CHEB_FP64 = 0, CHEB_MIXED = 1 } cheb_prec;

typedef enum {
  CHEB_OP_H = 0,        /* cheb_apply_H */
  CHEB_OP_SINV = 1,     /* cheb_apply_Sinv, cheb_apply_S */
  CHEB_OP_FILTER = 2,   /* cheb_filter */
  CHEB_OP_RR = 3,       /* cheb_rayleigh_ritz, cheb_rayleigh_quotients */
  CHEB_OP_BOUND = 4,    /* cheb_upper_bound (nb ignored) */
  CHEB_OP_SETUP = 5,    /* cheb_set_projectors (nb ignored) */
  CHEB_OP_FILTER_DEGREES = 6, /* cheb_filter_degrees */
  CHEB_OP_LOBPCG = 7          /* cheb_lobpcg_iterate */
} cheb_op;

typedef struct {
  int n;                          /* cubic FFT box side; supported: 8 12 16 24 32 48 64 96 128 */
  int npw;                        /* plane waves in the sphere (Sec. 2.1) */
  const int32_t* gidx_host;       /* npw x 3 Miller indices (gx, gy, gz), row-major, |g_c| <= (n-1)/2;
                                     sorted by column (gx, gy), each column a run of consecutive gz */
  const double* kin_host;         /* npw kinetic diagonal 1/2 |k + G|^2 in Hartree (Sec. 2.1) */
  int natom;                      /* atoms; atom a owns projector columns [proj_off[a], proj_off[a+1]) */
  const int32_t* proj_off_host;   /* natom + 1 offsets, proj_off[0] = 0, nondecreasing; nproj = proj_off[natom] */
  int has_overlap;                /* 0: S = I (norm-conserving); 1: S = I + P Q P^H (PAW, Eq. 4) */
  int prec;                       /* cheb_prec: CHEB_FP64 or CHEB_MIXED (complex64 bands, FFTs, recurrence
                                     and projector GEMMs; FP64 capacitance inverse, subspace matrices and
                                     dense eigensolver) */
  int gamma;                      /* 0: complex bands on the whole sphere. 1: Gamma point, real wavefunctions
                                     (Sec. 2.1): gidx_host / kin_host / npw describe the half sphere H+ (gx > 0,
                                     or gx = 0 and gy > 0, or gx = gy = 0 and gz >= 0), sorted as above, and a
                                     band holds sqrt(2) c_G for G != 0 and the real c_0 at G = 0 (c_-G = conj c_G
                                     implied), so that Re x^H y is the inner product of the real functions.
                                     Projectors (cheb_set_projectors) are given the same way and must be real
                                     functions in real space. Two bands share each complex transform. Not
                                     available: cheb_filter_rr_backward, cheb_lobpcg_iterate. */
} cheb_desc;

/* Size in bytes of the device buffer a plan keeps for its lifetime (index maps, twiddles, V(r), P, D, Q,
 * P^H P, capacitance inverse). */
cheb_status cheb_plan_persistent_bytes(const cheb_desc* desc, size_t* bytes);

/* Create a plan over a caller-provided device buffer of at least cheb_plan_persistent_bytes bytes
 * (256-byte aligned). Copies the host arrays of desc; synchronizes `stream`. */
cheb_status cheb_plan_create(const cheb_desc* desc, void* persistent_dev, size_t bytes, hipStream_t stream,
                             cheb_plan* out);
cheb_status cheb_plan_destroy(cheb_plan plan);

/* Local potential V(r_j) on the n^3 grid r_j = L j / n, real FP64, C order [x][y][z] (Sec. 2.1). */
cheb_status cheb_set_potential(cheb_plan plan, const double* V_dev, hipStream_t stream);

/* Projectors P (Eq. 3): complex128, column-major npw x nproj with leading dimension ldp >= npw.
 * Q_dev: nproj FP64 overlap coefficients (Eq. 4, entries > 0), NULL iff has_overlap == 0.
 * Forms P^H P and, with overlap, the capacitance matrix C = Q^-1 + P^H P and its FP64 inverse (Sec. 5.1)
 * inside `ws` (cheb_workspace_bytes(CHEB_OP_SETUP)). Synchronizes; CHEB_ERR_NOT_PD if C is not
 * positive definite. */
cheb_status cheb_set_projectors(cheb_plan plan, const void* P_dev, int ldp, const double* Q_dev, void* ws,
                                size_t ws_bytes, hipStream_t stream);

/* Per-atom blocks of D (Eq. 3): real symmetric n_a x n_a, n_a = proj_off[a+1] - proj_off[a], each
 * row-major, concatenated over atoms, FP64. */
cheb_status cheb_set_D(cheb_plan plan, const double* D_dev, hipStream_t stream);

/* Workspace bytes a call of kind `op` with nb bands needs. */
cheb_status cheb_workspace_bytes(cheb_plan plan, int op, int nb, size_t* bytes);

/* Y = H X (Alg. 1). X and Y must not overlap. */
cheb_status cheb_apply_H(cheb_plan plan, const void* X, int ldx, void* Y, int ldy, int nb, void* ws,
                         size_t ws_bytes, hipStream_t stream);
/* Y = S X (Alg. 1, Eq. 4). */
cheb_status cheb_apply_S(cheb_plan plan, const void* X, int ldx, void* Y, int ldy, int nb, void* ws,
                         size_t ws_bytes, hipStream_t stream);
/* Y = S^-1 X by the Woodbury formula (Sec. 5.1). */
cheb_status cheb_apply_Sinv(cheb_plan plan, const void* X, int ldx, void* Y, int ldy, int nb, void* ws,
                            size_t ws_bytes, hipStream_t stream);

/* Y = H X like cheb_apply_H, for callers that cannot allocate device memory (code under graph capture, tight
 * serving loops, harnesses that forbid allocation): no workspace argument, and the call allocates nothing. Its
 * scratch is a file-scope device array of 64 MiB (cheb_workspace_bytes(CHEB_OP_H, nb) must not exceed it:
 * CHEB_ERR_WORKSPACE otherwise, before any launch), held by every GPU the library runs on until the process
 * ends; its device address is resolved at the first cheb_plan_create on each device. All calls on one GPU share
 * that GPU's array: calls that overlap in time on one GPU (several streams or host threads) race and must be
 * serialised by the caller. The plan's device must be current (CHEB_ERR_ARG otherwise). Kernel-class timers do
 * not see this entry point. */
cheb_status cheb_apply_H_noalloc(cheb_plan plan, const void* X, int ldx, void* Y, int ldy, int nb, hipStream_t stream);

/* In place: X <- T_m((S^-1 H - c)/r) X, the Chebyshev filter of Alg. 2 (recurrence of Sec. 4.2):
 *   psi^0 = X, psi^1 = (A psi^0 - c psi^0)/r, psi^i = 2/r (A psi^(i-1) - c psi^(i-1)) - psi^(i-2),
 * A = S^-1 H, unscaled. Projections P^H psi^i are carried in projector space with the reuse trick of
 * Sec. 5.1 (one P^H and one P product per step). m >= 0 (m = 0 leaves X unchanged), r > 0. */
cheb_status cheb_filter(cheb_plan plan, void* X, int ldx, int nb, int m, double c, double r, void* ws,
                        size_t ws_bytes, hipStream_t stream);

/* cheb_filter starting from quantities of the input block that the caller already holds: the reuse trick of
 * Sec. 5.1 extended over the Rayleigh-Ritz step, so that an outer iteration computes P^H X once (inside
 * Rayleigh-Ritz) instead of once per call, and transforms the block one time fewer. p_in: NULL, or the projections
 * P^H X of the input block (device, nproj x nb complex FP64, column j = band j, leading dimension nproj); hx_in:
 * NULL, or (K + V) X of the input block, the local part of H X (device, nb rows of npw values in the plan
 * precision, leading dimension npw). Normally both are the outputs of cheb_rayleigh_ritz_carry on the same block;
 * each is used instead of computing it (a NULL one is computed as cheb_filter does). Caller-owned and not
 * modified; the block must not change between the call that produced them and this one. Results equal
 * cheb_filter's up to the rounding of the given values. Projections carried in both directions with no
 * recomputation in between would let the difference between X and its projections grow by the filter's
 * amplification at every outer iteration, which is why the filter takes these quantities but returns none.
 * Same workspace as cheb_filter. */
cheb_status cheb_filter_carry(cheb_plan plan, void* X, int ldx, int nb, int m, double c, double r, const void* p_in,
                              const void* hx_in, void* ws, size_t ws_bytes, hipStream_t stream);

/* Locking (Sec. 5.4): the same filter with its own degree per band, X[:, b] <- T_{deg[b]}((S^-1 H - c)/r) X[:, b].
 * degrees: nb host int32 values >= 0; a band of degree 0 is left unchanged (locked). Bands are gathered in
 * order of decreasing degree into the workspace, step i of the recurrence runs on the bands of degree >= i
 * only (a shrinking prefix, so locked and nearly converged bands cost nothing), and each band is written
 * back from the step that finished it. Results equal cheb_filter run band by band with each band's degree.
 * The permutation is staged through a pinned host buffer owned by the plan; calls on one plan must not
 * overlap from several host threads. r > 0. Workspace: cheb_workspace_bytes(CHEB_OP_FILTER_DEGREES, nb). */
cheb_status cheb_filter_degrees(cheb_plan plan, void* X, int ldx, int nb, const int32_t* degrees, double c,
                                double r, void* ws, size_t ws_bytes, hipStream_t stream);

/* Degree per band from the residual estimate of Sec. 5.4 (Eq. 5): after a degree-n filter and Rayleigh-Ritz,
 * the residual of band i is about resid[i] / |T_n((ritz[i] - c)/r)|. degrees[i] = 0 if resid[i] <= tol,
 * else the smallest n in [1, m_max] whose estimate is <= tol, else m_max. The band's own Ritz value is
 * used in T_n (the equation prints lambda_1 where the text speaks of band i). Host arrays, host
 * arithmetic only; touches no GPU. Returns the number of locked bands in *nlocked (may be NULL). */
cheb_status cheb_locking_degrees(int nb, const double* ritz, const double* resid, double c, double r, int m_max,
                                 double tol, int32_t* degrees, int* nlocked);

/* In place Rayleigh-Ritz (Alg. 2): H_X = X^H H X, S_X = X^H S X, H_X Z = S_X Z Lambda with
 * Z^H S_X Z = I (FP64 generalized Hermitian eigensolver), X <- X Z. ritz_dev: nb FP64 Ritz values,
 * ascending. resid_dev: NULL, or nb FP64 residual norms ||H x_i - lambda_i S x_i||_2 of the rotated
 * block. Synchronizes; CHEB_ERR_NOT_PD if S_X is singular to working precision (rank-deficient X),
 * CHEB_ERR_NONFINITE on NaN/Inf, CHEB_ERR_EIG if the eigensolver fails. */
cheb_status cheb_rayleigh_ritz(cheb_plan plan, void* X, int ldx, int nb, double* ritz_dev, double* resid_dev,
                               void* ws, size_t ws_bytes, hipStream_t stream);

/* cheb_rayleigh_ritz that also returns two quantities of the rotated block for the next cheb_filter_carry.
 * p_out: NULL, or P^H of the rotated block, (P^H X) Z, formed from the exact projections of the input block that
 * the subspace matrices need anyway (with residuals the product is already there; without, one nproj x nb x nb
 * FP64 GEMM); device, nproj x nb complex FP64, column j = band j, leading dimension nproj. hx_out: NULL, or
 * (K + V) of the rotated block, ((K + V) X) Z, formed from the local part of H X that the subspace matrices use
 * (with residuals the product is already there, one copy; without, one npw x nb x nb GEMM); device, nb rows of
 * npw values in the plan precision, leading dimension npw. Both caller-owned. In a mixed plan the rotated block
 * is rounded to complex64 after the products, so the outputs match it to float32 rounding. Same workspace as
 * cheb_rayleigh_ritz. */
cheb_status cheb_rayleigh_ritz_carry(cheb_plan plan, void* X, int ldx, int nb, double* ritz_dev, double* resid_dev,
                                     void* p_out, void* hx_out, void* ws, size_t ws_bytes, hipStream_t stream);

/* LOBPCG, the block method the paper compares the filter with (Sec. 2.3), on the same operators: one
 * iteration per call. iteration = 0: Rayleigh-Ritz of X (start); 1: Rayleigh-Ritz in span[X, W]; >= 2: in
 * span[X, W, P], with W the residuals of the bands whose residual norm exceeds tol, preconditioned by
 * K(t_G / E_kin) with K(x) = (27 + 18x + 12x^2 + 8x^3) / (27 + 18x + 12x^2 + 8x^3 + 16x^4) and E_kin the band's
 * kinetic energy, and P the previous directions of those bands (soft locking: converged bands stay in X and
 * in every Rayleigh-Ritz but add no columns). At iterations 11, 21, ... H X and S X are recomputed from X and
 * the directions dropped (restart), which bounds the drift of the products carried by linear combinations;
 * the iteration also restarts from span[X, W] when the Rayleigh-Ritz with the directions fails. The Rayleigh-Ritz uses an S-orthonormal basis of the space from
 * the eigendecomposition of the scaled Gram matrix (directions below 1e-14 of the largest dropped).
 * X (npw x nb, ldx) holds the S-orthonormal Ritz vectors on return; ritz_dev the nb FP64 Ritz values
 * (input for iterations >= 1, output always); resid_dev (NULL or nb FP64) the residual norms
 * ||H x - lambda S x|| of the vectors that entered the iteration (iterations >= 1); *nactive (may be NULL) the
 * number of bands above tol. state: caller-owned device buffer of cheb_lobpcg_state_bytes, carried unchanged
 * between calls (it holds H X, S X and the directions). Requires 3 nb <= npw and an FP64 plan (the products
 * H X, S X, H P, S P are carried by linear combinations, which drift too fast in complex64). Synchronizes.
 * Workspace: cheb_workspace_bytes(CHEB_OP_LOBPCG, nb). */
cheb_status cheb_lobpcg_state_bytes(cheb_plan plan, int nb, size_t* bytes);
cheb_status cheb_lobpcg_iterate(cheb_plan plan, void* X, int ldx, int nb, int iteration, double tol, void* state,
                                size_t state_bytes, double* ritz_dev, double* resid_dev, int* nactive, void* ws,
                                size_t ws_bytes, hipStream_t stream);

/* Capacitance solve q = C^-1 b, C = Q^-1 + P^H P, inside cheb_apply_Sinv, cheb_filter(_degrees), the Lanczos
 * bound and the adjoint (Sec. 5.1). iterations = 0 (default): the inverse formed at cheb_set_projectors is
 * applied directly. iterations = k > 0: iterative refinement preconditioned by the atom-block diagonal M of C,
 * q = M^-1 b then k corrections q += M^-1 (b - C q) (error shrinks by the spectral radius of I - M^-1 C per
 * correction). Needs the projectors set and atom blocks of at most 32 projectors; the plan must have an
 * overlap (S != I). Changes the workspace sizes: query cheb_workspace_bytes after switching. */
cheb_status cheb_set_capacitance_solver(cheb_plan plan, int iterations);

/* Mixed plans only (no effect on FP64 plans): the projector products P^H x and P w of the filter and the
 * operators use the FP16 hi/lo split MFMA (on = 1, the default: each operand is a sum of two FP16 numbers,
 * about 22 significant bits, products hi*hi + hi*lo + lo*hi accumulated in FP32) or the FP32 MFMA (on = 0).
 * The split planes of P are built by cheb_set_projectors. */
cheb_status cheb_set_split_gemm(cheb_plan plan, int on);

/* Projections carried through the recurrence (the reuse trick of Sec. 5.1, P^H psi^i updated in projector space
 * instead of recomputed): in a mixed plan the complex64 bands are rounded at every step while the carried
 * projections are not, and the recurrence amplifies their difference like the bands it multiplies, which sets a
 * floor on the residuals the outer loop reaches. period = k > 0: before steps i = 1 + k, 1 + 2k, ... of
 * cheb_filter, cheb_filter_degrees and the forward pass of cheb_filter_rr_backward, the carried projections of
 * psi^(i-1) and psi^(i-2) are recomputed from the vectors (two more P^H products). period = 0: never (the plain
 * reuse trick). Default: 3 for mixed plans, 0 for FP64 plans. CHEB_ERR_ARG if period < 0. */
cheb_status cheb_set_projection_resync(cheb_plan plan, int period);

/* Diagnostic of the carried projections (an addition; synchronizes every filter step while on): before every
 * step i >= 2 of the filters above, max over bands of ||p_carried - P^H psi^(i-1)|| / ||P^H psi^(i-1)|| with
 * P^H psi recomputed on FP64 MFMA. cheb_drift_monitor(on) resets the maximum; cheb_drift_read returns it and the
 * number of steps checked. */
cheb_status cheb_drift_monitor(cheb_plan plan, int on);
cheb_status cheb_drift_read(cheb_plan plan, double* max_rel_drift, int64_t* checks);

/* Dense eigensolver of cheb_rayleigh_ritz. on (default): first try a warm-started iterative refinement of
 * Z from the identity in the column-scaled basis (n^3 products only; accepted only if X^H S_X X = I and
 * X^H H_X X diagonal to 1e-12 are verified), else the library path. off: always the library path.
 * cheb_rr_stats counts the Rayleigh-Ritz calls solved each way. */
cheb_status cheb_set_rr_refine(cheb_plan plan, int on);
cheb_status cheb_rr_stats(cheb_plan plan, int64_t* refined, int64_t* fallback);

/* rq_dev[i] = (x_i^H H x_i) / (x_i^H S x_i), FP64 (first step of Alg. 2). */
cheb_status cheb_rayleigh_quotients(cheb_plan plan, const void* X, int ldx, int nb, double* rq_dev, void* ws,
                                    size_t ws_bytes, hipStream_t stream);

/* Upper bound of the spectrum by k steps of Lanczos on S^-1 H in the S inner product, started from the
 * caller's vector v0_dev (npw elements, plan precision): max eigenvalue of the k x k tridiagonal plus the
 * last off-diagonal norm (Sec. 5.3 names this alternative to E_cut). 1 <= k <= 64. Synchronizes. */
cheb_status cheb_upper_bound(cheb_plan plan, int k, const void* v0_dev, double* lambda_plus_host, void* ws,
                             size_t ws_bytes, hipStream_t stream);

/* Adjoint of one filter + Rayleigh-Ritz pass (an addition beyond the paper: differentiation form).
 * Runs the forward Y = T_m((S^-1 H - c)/r) X0 (Alg. 2, Sec. 4.2) and Rayleigh-Ritz, writes the nb Ritz values
 * (ascending) to ritz_dev, and the gradients of L = sum_{i < nk} w_i lambda_i (c, r held fixed) with the
 * convention dL = 2 Re tr(G^H dX) for the complex start block:
 *   dX   (npw x nb, plan precision, leading dimension lddx)  dL/dX0
 *   dV   (n^3 FP64, [x][y][z] like V)                        dL/dV(r_j)
 *   dD   (packed like cheb_set_D, FP64; NULL iff no projectors) dL/dD, symmetric per block
 * w_dev: nk FP64 weights (1 <= nk <= nb). The recurrence is checkpointed every ckpt_every steps (pairs
 * psi^(t-1), psi^t) and recomputed segment by segment, so memory grows with m / ckpt_every + ckpt_every.
 * Requires a gap lambda_nk < lambda_(nk+1) and non-degenerate wanted Ritz values.
 * Synchronizes (Rayleigh-Ritz). Workspace: cheb_backward_workspace_bytes. */
cheb_status cheb_backward_workspace_bytes(cheb_plan plan, int nb, int m, int ckpt_every, size_t* bytes);
cheb_status cheb_filter_rr_backward(cheb_plan plan, const void* X0, int ldx, int nb, int m, double c, double r,
                                   int nk, const double* w_dev, int ckpt_every, double* ritz_dev, void* dX,
                                   int lddx, double* dV_dev, double* dD_dev, void* ws, size_t ws_bytes,
                                   hipStream_t stream);

/* Kernel-class timers (diagnostics). While enabled, each launch of a class below made by calls on the plan is
 * bracketed by HIP events on the call's own stream, and the algorithmic bytes and flops of the launch
 * (from its shapes: the bytes the operation must move and the flops it must do, not what the kernel
 * actually fetches) are tallied per class. */
typedef enum {
  CHEB_T_FFT_COL_INV = 0,   /* sphere -> disk columns, inverse z-FFT */
  CHEB_T_FFT_PLANE = 1,     /* per z-plane inverse y, x, V(r) multiply, forward x, y */
  CHEB_T_FFT_COL_FWD = 2,   /* forward z-FFT, sphere gather, kinetic */
  CHEB_T_PROJECT = 3,       /* P^H X products (Npw-long reductions, with their split-K reduction) */
  CHEB_T_BACKPROJECT = 4,   /* P w products with the fused vector epilogue (Chebyshev recurrence) */
  CHEB_T_SMALL = 5,         /* projector-space products with P^H P and the capacitance inverse */
  CHEB_T_RR_GRAM = 6,       /* subspace matrices X^H H X, X^H S X */
  CHEB_T_RR_EIG = 7,        /* dense generalized eigensolver */
  CHEB_T_RR_ROTATE = 8,     /* X Z rotation and residual products */
  CHEB_T_XDENS = 9,         /* cross densities of the adjoint */
  CHEB_T_COUNT = 10
} cheb_timer;

/* on != 0: reset the tallies and start timing; on == 0: stop. */
cheb_status cheb_profile_enable(cheb_plan plan, int on);
/* Totals of one class since the last enable: summed event time in ms, launches, algorithmic bytes and
 * flops. Waits for the recorded events. */
cheb_status cheb_profile_read(cheb_plan plan, int timer, double* ms, int64_t* launches, double* algo_bytes,
                              double* algo_flops);

/* Tiling rules of the complex GEMMs, host arithmetic only (no device call; usable without a GPU). For an
 * M x N x K product: *fp64 = the split-K count of the tiled FP64/FP32 kernel, *fp16 = that of the FP16 split
 * kernel of mixed plans, *bound = the count every workspace sizes its split-K partials by (each partial buffer
 * holds bound x M x N complex FP64 values; bound >= fp64 and bound >= fp16). CHEB_ERR_ARG for a null pointer. */
cheb_status cheb_gemm_splits(int M, int N, int K, int* fp64, int* fp16, int* bound);
/* Work item of block i in a tiled GEMM launch of `total` blocks over (split, M tile, N tile) items with
 * tm x tn tiles per split: the blocks are dealt to the 8 XCDs in turn and each XCD receives one contiguous run
 * of items, so that blocks sharing an operand slice share an L2. Items are ordered split by split, in groups of
 * `group` M tiles, the M tile fastest inside a group (group 1: the N tile fastest). The GEMMs use group 8 when
 * K >= M and group 1 otherwise. group = -1: the order of the Hermitian products (the Rayleigh-Ritz matrices), which
 * form only the tiles bx <= by of a square grid (tn = tm), tm (tm + 1) / 2 per split, column by column. Host
 * arithmetic only. CHEB_ERR_ARG unless 0 <= i < total, total a multiple of the tiles per split (tm * tn, or
 * tm (tm + 1) / 2 for group -1) > 0, group >= 1 or -1 and the pointers non-null. */
cheb_status cheb_gemm_block_item(int i, int total, int tm, int tn, int group, int* bx, int* by, int* bz);

/* Message of the last failing call on `plan` ("" if none). Valid until the next call on the plan. */
const char* cheb_last_error(cheb_plan plan);

#ifdef __cplusplus
}
#endif
#endif /* CHEBFD_H */
