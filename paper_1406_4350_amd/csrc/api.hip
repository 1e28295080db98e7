// C ABI of chebfd: plan set-up, operator application, Chebyshev filter, Rayleigh-Ritz, Lanczos bound.
//
// The host side here only validates arguments, carves caller-owned buffers and sequences kernels on the
// caller's stream; every arithmetic step of the path runs on the GPU.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/chebfd.h"
#include "kernels.h"

using namespace chebfd;

struct cheb_plan_s {
  int n = 0, npw = 0, ncol = 0, rx = 0, natom = 0, nproj = 0, has_overlap = 0, prec = 0;
  int gamma = 0, npf = 0, h0 = -1;  // Gamma point: FFT sphere of npf entries built from the npw half-sphere ones
  int device = 0;                   // device current at cheb_plan_create
  void* scratch = nullptr;          // device address of this device's static scratch (cheb_apply_H_noalloc)
  int* gmap = nullptr;              // per FFT-sphere entry: half index | conj << 30
  int2* gpair = nullptr;            // per half entry: FFT-sphere entries of G and -G
  std::vector<int> proj_off;
  size_t dsize = 0;  // number of doubles of the packed D blocks
  // views into the persistent buffer
  int4* col = nullptr;
  int* ent = nullptr;
  int4* xline = nullptr;
  int4* pinfo = nullptr;
  int2* dent = nullptr;  // packed D entry -> (global row, global column)
  void* tw = nullptr;
  void* kin = nullptr;
  void* Vt = nullptr;
  void* P = nullptr;
  double* D = nullptr;
  double* Q = nullptr;
  c128* G = nullptr;
  c128* Cinv = nullptr;  // C^-1, C = Q^-1 + P^H P
  c128* Cmat = nullptr;  // C itself and the inverses of its atom blocks, for the iterative solve
  c128* Minv = nullptr;
  int cap_iters = 0;     // 0: C^-1 applied directly; k > 0: k preconditioned refinement corrections
  bool cap_blocks_ok = false;  // atom blocks inverted (all of size <= 32)
  bool have_V = false, have_P = false, have_D = false;
  int fft_batch = 1;
  HalfPlanes hproj, hback;                  // mixed plans: split planes of P (set with the projectors)
  bool split_gemm = true;                   // mixed plans: FP16 hi/lo split MFMA for P^H x and P w
  bool rr_refine = true;                    // warm-started refinement before the library eigensolver
  // Projections carried through the recurrence (reuse trick) are recomputed from the vectors every `resync`
  // steps (0: never); drift_on measures ||p_carried - P^H psi|| / ||P^H psi|| before every step of the filter
  int resync = 0;
  bool drift_on = false;
  double drift_max = 0.0;
  int64_t drift_checks = 0;
  double* rr_host = nullptr;                // pinned staging of the refinement's block maxima and flag (2 slots)
  hipEvent_t rr_ev[2] = {nullptr, nullptr}; // end of the staging copy into each slot
  int64_t rr_refined = 0, rr_fallback = 0;  // how Rayleigh-Ritz steps were solved
  rocblas_handle rb = nullptr;
  // pinned staging of the band permutation of cheb_filter_degrees; lock_ev marks the end of its last copy
  int* lock_host = nullptr;
  size_t lock_cap = 0;
  hipEvent_t lock_ev = nullptr;
  std::string err;
  // kernel-class timers
  struct TimerRec { hipEvent_t a, b; int kind; };
  bool prof_on = false;
  std::vector<TimerRec> prof_pending;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_free;
  double prof_ms[CHEB_T_COUNT] = {}, prof_bytes[CHEB_T_COUNT] = {}, prof_flops[CHEB_T_COUNT] = {};
  int64_t prof_n[CHEB_T_COUNT] = {};
};

// Scratch of cheb_apply_H_noalloc, for callers that cannot allocate device memory: a file-scope device array, of
// which every GPU the library runs on holds its own copy until the process ends. Host code never passes the
// name (a host-side stand-in): the device address is resolved once per device with that device current, at the
// first cheb_plan_create on it, and kept in scratch_addr.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void* scratch_addr[kMaxDevices] = {};

// the current device's address of `scratch` (nullptr and *err set when it cannot be resolved)
void* resolve_scratch(int dev, hipError_t* err) {
  *err = hipSuccess;
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(scratch_mu);
  if (!scratch_addr[dev]) {
    void* ptr = nullptr;
    *err = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (*err != hipSuccess) return nullptr;
    scratch_addr[dev] = ptr;
  }
  return scratch_addr[dev];
}

constexpr size_t kAlign = 256;
// default period (filter steps) of the projection resynchronisation in mixed plans
constexpr int kMixedResync = 3;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Carves aligned regions from a base pointer; with base == nullptr it only measures.
struct Bump {
  char* base;
  size_t off = 0;
  explicit Bump(void* b) : base(static_cast<char*>(b)) {}
  template <typename X> X* take(size_t count) {
    size_t at = off;
    off = align_up(off + count * sizeof(X));
    return base ? reinterpret_cast<X*>(base + at) : nullptr;
  }
};

bool supported_n(int n) {
  for (int v : {8, 12, 16, 24, 32, 48, 64, 96, 128})
    if (v == n) return true;
  return false;
}

cheb_status fail(cheb_plan p, cheb_status s, const std::string& msg) {
  if (p) p->err = msg;
  return s;
}

// Every status-returning entry point is a function-try-block: a C++ exception (host memory exhausted in a
// std::vector or std::string) must not cross the C ABI, so it ends the call with CHEB_ERR_HOST instead.
cheb_status host_fail(cheb_plan p) noexcept {
  if (p) {
    try {
      p->err = "host-side failure (out of host memory or an internal exception)";
    } catch (...) {
    }
  }
  return CHEB_ERR_HOST;
}

#define HIPCHK(expr)                                                                                   \
  do {                                                                                                 \
    hipError_t e_ = (expr);                                                                            \
    if (e_ != hipSuccess) return fail(p, CHEB_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define RBCHK(expr)                                                                                    \
  do {                                                                                                 \
    rocblas_status s_ = (expr);                                                                        \
    if (s_ != rocblas_status_success)                                                                  \
      return fail(p, CHEB_ERR_HIP, std::string(#expr) + ": " + rocblas_status_to_string(s_));          \
  } while (0)

#define CHK(expr)                                                                                      \
  do {                                                                                                 \
    cheb_status s_ = (expr);                                                                           \
    if (s_ != CHEB_OK) return s_;                                                                      \
  } while (0)

size_t elem_bytes(int prec) { return prec == CHEB_MIXED ? sizeof(c64) : sizeof(c128); }

// Brackets the launches of one kernel class with events on the launching stream while profiling is on.
struct Timed {
  cheb_plan p;
  hipStream_t st;
  hipEvent_t end = nullptr;
  // count = false: a second interval of the same section (its time adds, the section's count does not)
  Timed(cheb_plan p_, hipStream_t st_, int kind, double bytes, double flops, bool count = true) : p(p_), st(st_) {
    if (!p->prof_on) return;
    std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
    if (!p->prof_free.empty()) {
      ev = p->prof_free.back();
      p->prof_free.pop_back();
    } else if (hipEventCreate(&ev.first) != hipSuccess) {
      return;
    } else if (hipEventCreate(&ev.second) != hipSuccess) {
      (void)hipEventDestroy(ev.first);
      return;
    }
    if (hipEventRecord(ev.first, st) != hipSuccess) {
      p->prof_free.push_back(ev);  // unused pair: back to the pool, released with the plan
      return;
    }
    end = ev.second;
    p->prof_pending.push_back({ev.first, ev.second, kind});
    p->prof_bytes[kind] += bytes;
    p->prof_flops[kind] += flops;
    p->prof_n[kind] += count ? 1 : 0;
  }
  ~Timed() {
    if (end) (void)hipEventRecord(end, st);
  }
};

// ---- layouts -------------------------------------------------------------------------------------------------
struct Persist {
  int4* col; int* ent; int4* xline; int4* pinfo; int2* dent; void* tw; void* kin; void* Vt; void* P; double* D; double* Q; c128* G; c128* Cinv; c128* Cmat; c128* Minv;
  _Float16* Hproj;  // mixed plans: FP16 hi/lo planes of P for P^H x (rows = projectors, k = plane waves)
  _Float16* Hback;  // and for P w (rows = plane waves, k = projectors)
  int* gmap; int2* gpair;  // Gamma point maps
  size_t bytes;
};

inline long pad32(long k) { return (k + 31) / 32 * 32; }

// Carves the persistent buffer (base == nullptr: only measures)
Persist persist_layout(void* base, int n, int npw, int npf, int ncol, int rx, int nproj, size_t dsize, int overlap,
                       int prec, int gamma) {
  Bump b(base);
  Persist l{};
  const bool mixed = prec == CHEB_MIXED;
  l.col = b.take<int4>(ncol);
  l.ent = b.take<int>(npf);
  l.xline = b.take<int4>(2 * rx + 1);
  l.pinfo = b.take<int4>(std::max(nproj, 1));
  l.dent = b.take<int2>(std::max<size_t>(dsize, 1));
  l.tw = mixed ? (void*)b.take<c64>(n) : (void*)b.take<c128>(n);
  l.kin = mixed ? (void*)b.take<float>(npw) : (void*)b.take<double>(npw);
  l.Vt = mixed ? (void*)b.take<float>(size_t(n) * n * n) : (void*)b.take<double>(size_t(n) * n * n);
  l.P = mixed ? (void*)b.take<c64>(size_t(npw) * nproj) : (void*)b.take<c128>(size_t(npw) * nproj);
  l.D = b.take<double>(std::max<size_t>(dsize, 1));
  l.Q = b.take<double>(std::max(nproj, 1));
  l.G = b.take<c128>(size_t(nproj) * nproj);
  l.Cinv = overlap ? b.take<c128>(size_t(nproj) * nproj) : nullptr;  // C^-1
  l.Cmat = overlap ? b.take<c128>(size_t(nproj) * nproj) : nullptr;
  l.Minv = overlap ? b.take<c128>(std::max<size_t>(dsize, 1)) : nullptr;
  l.Hproj = l.Hback = nullptr;
  if (mixed && nproj > 0) {
    l.Hproj = b.take<_Float16>(4 * size_t(nproj) * pad32(npw));
    l.Hback = b.take<_Float16>(4 * size_t(npw) * pad32(nproj));
  }
  l.gmap = gamma ? b.take<int>(npf) : nullptr;
  l.gpair = gamma ? b.take<int2>(npw) : nullptr;
  l.bytes = b.off;
  return l;
}

size_t persist_bytes(int n, int npw, int npf, int ncol, int rx, int nproj, size_t dsize, int overlap, int prec,
                     int gamma) {
  return persist_layout(nullptr, n, npw, npf, ncol, rx, nproj, dsize, overlap, prec, gamma).bytes;
}

// split-K partials of an M x N x K product: enough for either GEMM kernel (FP64/FP32 MFMA or FP16 split),
// whose split counts follow different rules
size_t part_elems(int M, int N, int K) {
  const int s = gemm_split_bound(M, N, K);
  return s > 1 ? size_t(s) * M * N : 0;
}
// partials of an upper-triangle (Hermitian) product, N x N x K
size_t upper_part_elems(int N, int K) {
  const int s = gemm_upper_splits(N, K);
  return s > 1 ? size_t(s) * N * N : 0;
}

// Scratch of the FFT passes: two disk-column buffers for a batch of bands.
struct FftWs { void* a; void* b; void* ga = nullptr; void* gb = nullptr; };  // ga, gb: Gamma band pairs

// Every op's workspace, carved in one place so that sizes and pointers agree.
struct Ws {
  FftWs fft{};
  void *W = nullptr, *loc = nullptr, *Ynew = nullptr, *R = nullptr;     // npw x nb, plan precision
  void *v = nullptr, *vp = nullptr, *f = nullptr, *Hv = nullptr, *Sf = nullptr;  // Lanczos vectors
  c128 *p0 = nullptr, *p1 = nullptr, *ploc = nullptr, *Dp = nullptr, *pphi = nullptr, *q = nullptr, *w = nullptr;
  c128 *Hs = nullptr, *Ss = nullptr, *part = nullptr, *dots = nullptr, *dots2 = nullptr;
  double *d = nullptr, *E = nullptr;
  int* flags = nullptr;  // [0..1] rr_prepare flags, [2] solver info
  c128 *Xa = nullptr, *Xb = nullptr, *T = nullptr, *M1 = nullptr, *M2 = nullptr, *F = nullptr;  // refinement
  c128* M1b = nullptr;  // second product buffer of the refinement (speculative step)
  double *absF = nullptr, *lam = nullptr, *res = nullptr;
  int* perm = nullptr;
  unsigned* bits = nullptr;  // coupling graph of the refinement (n x ceil(n / 32) words)
  int *cidx = nullptr, *coff = nullptr;  // its clusters: members (n), offsets (n + 1)
  double* bmax = nullptr;                // per-block maxima of |F|
  float* bsc = nullptr;  // per-band power-of-two scales of the split GEMMs
  _Float16* hb = nullptr;  // mixed plans: the back-projection's projector-space operand split into FP16 planes
  long hb_ld = 0;
  _Float16* hx = nullptr;  // mixed plans, filters: the projected bands split into FP16 planes
  long hx_ld = 0;
  c128 *cp = nullptr, *cq = nullptr, *cr = nullptr;  // iterative capacitance solve: right side, solution, residual
  c128* pfresh = nullptr;  // projections recomputed from the vectors (drift monitor)
  double* dcol = nullptr;  // per-band relative drift
  void* Xs = nullptr;   // band-sorted copy for the per-band degree filter
  int* lidx = nullptr;  // its gather / scatter indices (3 nb)
  void* solver = nullptr;
  size_t solver_bytes = 0;
  size_t total = 0;
};

int fft_batch_for(const cheb_plan_s* p, int nb) {
  const size_t per_band = size_t(p->n) * col_stride(p->ncol) * elem_bytes(p->prec);
  size_t cap = (96u << 20) / std::max<size_t>(per_band, 1);
  if (cap < 1) cap = 1;
  if (size_t(std::max(nb, 1)) <= cap) return std::max(nb, 1);
  // The plane pass takes n (z-plane, transform) items per transform on its resident blocks in rounds; of the
  // batches from cap / 2 to cap, take the one with the fewest rounds per band (the largest on a tie), so that the
  // last round of a launch does not leave blocks idle (15 bands at 128^3 FP64 are 1920 items on 256 blocks, 7.5
  // rounds; 14 are 7).
  const long R = std::max(1, fft_plane_blocks(p->n, p->rx, p->prec == CHEB_FP64));
  const int per = p->gamma ? 2 : 1;  // bands per transform
  long best = long(cap), best_rounds = 0;
  for (long b = long(cap); b >= std::max<long>(1, long(cap) / 2); --b) {
    const long items = long(p->n) * ((b + per - 1) / per);
    const long rounds = (items + R - 1) / R;
    if (b == long(cap) || rounds * best < best_rounds * b) { best = b; best_rounds = rounds; }
  }
  return int(best);
}

cheb_status solver_query(cheb_plan p, int op, int nb, size_t* bytes);

cheb_status ws_layout(cheb_plan p, int op, int nb, void* base, Ws* w) {
  Bump b(base);
  const size_t eb = elem_bytes(p->prec);
  const size_t vec = size_t(p->npw) * std::max(nb, 1) * eb;
  const int np = p->nproj;
  const size_t pp = size_t(std::max(np, 1)) * std::max(nb, 1);
  const int fb = fft_batch_for(p, nb);
  const size_t colb = size_t(fb) * p->n * col_stride(p->ncol) * eb;
  size_t part = 0;
  auto need_fft = [&]() {
    w->fft.a = b.take<char>(colb);
    w->fft.b = b.take<char>(colb);
    if (p->gamma) {  // band pairs expanded to the whole sphere, before and after the transforms
      const size_t gsz = size_t(p->npf) * ((fb + 1) / 2) * eb;
      w->fft.ga = b.take<char>(gsz);
      w->fft.gb = b.take<char>(gsz);
    }
  };
  switch (op) {
    case CHEB_OP_H:
    case CHEB_OP_SINV: {
      need_fft();
      w->p0 = b.take<c128>(pp);
      w->Dp = b.take<c128>(pp);
      part = std::max(part_elems(np, nb, p->npw), part_elems(np, nb, np));
      break;
    }
    case CHEB_OP_FILTER:
    case CHEB_OP_FILTER_DEGREES: {
      need_fft();
      w->W = b.take<char>(vec);
      w->loc = b.take<char>(vec);
      w->p0 = b.take<c128>(pp);
      w->p1 = b.take<c128>(pp);
      w->ploc = b.take<c128>(2 * pp);  // [P^H loc; D p], ld 2 nproj
      w->w = b.take<c128>(pp);
      w->pfresh = b.take<c128>(pp);
      w->dcol = b.take<double>(std::max(nb, 1));
      part = std::max({part_elems(np, nb, p->npw), part_elems(np, nb, np)});
      if (op == CHEB_OP_FILTER_DEGREES) {
        w->Xs = b.take<char>(vec);
        w->lidx = b.take<int>(3 * size_t(std::max(nb, 1)));
        // the active block shrinks step by step; split-K partials are sized for every width up to nb
        for (int k = 1; k < nb; ++k)
          part = std::max({part, part_elems(np, k, p->npw), part_elems(np, k, np)});
      }
      break;
    }
    case CHEB_OP_RR: {
      need_fft();
      w->loc = b.take<char>(vec);
      w->Ynew = b.take<char>(vec);
      w->R = b.take<char>(vec);
      w->p0 = b.take<c128>(pp);
      w->Dp = b.take<c128>(pp);
      w->q = b.take<c128>(pp);
      w->w = b.take<c128>(pp);
      w->Hs = b.take<c128>(size_t(nb) * nb);
      w->Ss = b.take<c128>(size_t(nb) * nb);
      w->dots = b.take<c128>(std::max(nb, 1));
      w->dots2 = b.take<c128>(std::max(nb, 1));
      w->d = b.take<double>(std::max(nb, 1));
      w->E = b.take<double>(std::max(nb, 1));
      w->flags = b.take<int>(4);
      {
        const size_t nn = size_t(std::max(nb, 1)) * std::max(nb, 1);
        w->Xa = b.take<c128>(nn);
        w->Xb = b.take<c128>(nn);
        w->T = b.take<c128>(2 * nn);   // [S' X; H' X], 2n x n
        w->M1 = b.take<c128>(2 * nn);  // X^H [S' X | H' X] with interleaved columns
        w->M1b = b.take<c128>(2 * nn);  // the same for the speculative step
        w->M2 = b.take<c128>(2 * nn);  // [S'; H'] stacked, 2n x n
        w->F = b.take<c128>(nn);
        w->absF = b.take<double>(nn);
        w->lam = b.take<double>(std::max(nb, 1));
        w->res = b.take<double>(4);
        w->perm = b.take<int>(std::max(nb, 1));
        w->bits = b.take<unsigned>(size_t(std::max(nb, 1)) * ((std::max(nb, 1) + 31) / 32));
        w->cidx = b.take<int>(std::max(nb, 1));
        w->coff = b.take<int>(std::max(nb, 1) + 1);
        w->bmax = b.take<double>(kRefineBlocksMax);
      }
      part = std::max({part_elems(np, nb, p->npw), part_elems(nb, nb, p->npw), part_elems(nb, nb, np),
                       part_elems(np, nb, nb), part_elems(nb, nb, nb), part_elems(2 * nb, nb, nb),
                       part_elems(nb, 2 * nb, nb), upper_part_elems(nb, p->npw), upper_part_elems(nb, np)});
      CHK(solver_query(p, CHEB_OP_RR, nb, &w->solver_bytes));
      w->solver = b.take<char>(std::max<size_t>(w->solver_bytes, 1));
      break;
    }
    case CHEB_OP_LOBPCG: {
      // operator applications on up to nb columns; Rayleigh-Ritz matrices for up to 3 nb columns
      need_fft();
      const int n3 = 3 * std::max(nb, 1);
      const size_t nn = size_t(n3) * n3;
      w->p0 = b.take<c128>(pp);
      w->Dp = b.take<c128>(pp);
      w->Hs = b.take<c128>(nn);
      w->Ss = b.take<c128>(nn);
      w->Xa = b.take<c128>(nn);
      w->Xb = b.take<c128>(nn);
      w->F = b.take<c128>(nn);
      w->d = b.take<double>(n3);
      w->lam = b.take<double>(n3);
      w->E = b.take<double>(n3);
      w->res = b.take<double>(n3);
      w->flags = b.take<int>(4);
      w->lidx = b.take<int>(n3);
      // split-K partials for every width the iteration may use (active sets shrink the blocks)
      for (int k = 1; k <= std::max(nb, 1); ++k)
        part = std::max({part, part_elems(np, k, p->npw), part_elems(np, k, np)});
      for (int k = std::max(nb, 1); k <= n3; ++k) part = std::max(part, part_elems(k, k, p->npw));
      CHK(solver_query(p, CHEB_OP_RR, n3, &w->solver_bytes));
      w->solver = b.take<char>(std::max<size_t>(w->solver_bytes, 1));
      break;
    }
    case CHEB_OP_BOUND: {
      need_fft();
      const size_t v1 = size_t(p->npw) * eb;
      w->v = b.take<char>(v1);
      w->vp = b.take<char>(v1);
      w->f = b.take<char>(v1);
      w->Hv = b.take<char>(v1);
      w->Sf = b.take<char>(v1);
      w->p0 = b.take<c128>(std::max(np, 1));
      w->Dp = b.take<c128>(std::max(np, 1));
      w->dots = b.take<c128>(2);
      part = std::max(part_elems(np, 1, p->npw), part_elems(np, 1, np));
      break;
    }
    case CHEB_OP_SETUP: {
      w->Hs = b.take<c128>(size_t(std::max(np, 1)) * std::max(np, 1));  // staging of C
      w->flags = b.take<int>(4);
      part = part_elems(np, np, p->npw);
      CHK(solver_query(p, CHEB_OP_SETUP, np, &w->solver_bytes));
      w->solver = b.take<char>(std::max<size_t>(w->solver_bytes, 1));
      break;
    }
    default:
      return fail(p, CHEB_ERR_ARG, "unknown op");
  }
  w->part = b.take<c128>(std::max<size_t>(part, 1));
  w->bsc = b.take<float>(std::max(nb, 1));
  if (p->prec == CHEB_MIXED && np > 0) {
    w->hb_ld = ((np + 31) / 32) * 32;
    w->hb = b.take<_Float16>(4 * size_t(std::max(nb, 1)) * w->hb_ld);
    if (op == CHEB_OP_FILTER || op == CHEB_OP_FILTER_DEGREES) {
      w->hx_ld = ((long(p->npw) + 31) / 32) * 32;
      w->hx = b.take<_Float16>(4 * size_t(std::max(nb, 1)) * w->hx_ld);
    }
  }
  if (p->has_overlap && p->cap_iters > 0 && op != CHEB_OP_SETUP && op != CHEB_OP_RR) {
    w->cp = b.take<c128>(pp);
    w->cq = b.take<c128>(pp);
    w->cr = b.take<c128>(pp);
  }
  w->total = b.off;
  return CHEB_OK;
}

cheb_status solver_query(cheb_plan p, int op, int n, size_t* bytes) {
  *bytes = 0;
  if (n <= 0) return CHEB_OK;
  RBCHK(rocblas_start_device_memory_size_query(p->rb));
  if (op == CHEB_OP_RR) {
    const rocblas_double_complex one = {1.0, 0.0};
    rocsolver_zpotrf(p->rb, rocblas_fill_lower, n, nullptr, n, nullptr);
    rocblas_ztrsm(p->rb, rocblas_side_left, rocblas_fill_lower, rocblas_operation_none, rocblas_diagonal_non_unit, n,
                  n, &one, nullptr, n, nullptr, n);
    rocblas_ztrsm(p->rb, rocblas_side_right, rocblas_fill_lower, rocblas_operation_conjugate_transpose,
                  rocblas_diagonal_non_unit, n, n, &one, nullptr, n, nullptr, n);
    rocblas_ztrsm(p->rb, rocblas_side_left, rocblas_fill_lower, rocblas_operation_conjugate_transpose,
                  rocblas_diagonal_non_unit, n, n, &one, nullptr, n, nullptr, n);
    rocsolver_zheevd(p->rb, rocblas_evect_original, rocblas_fill_lower, n, nullptr, n, nullptr, nullptr, nullptr);
    rocsolver_zheev(p->rb, rocblas_evect_original, rocblas_fill_lower, n, nullptr, n, nullptr, nullptr, nullptr);
    if (p->gamma) {
      const double one = 1.0;
      rocsolver_dpotrf(p->rb, rocblas_fill_lower, n, nullptr, n, nullptr);
      rocblas_dtrsm(p->rb, rocblas_side_left, rocblas_fill_lower, rocblas_operation_none, rocblas_diagonal_non_unit, n,
                    n, &one, nullptr, n, nullptr, n);
      rocblas_dtrsm(p->rb, rocblas_side_right, rocblas_fill_lower, rocblas_operation_transpose,
                    rocblas_diagonal_non_unit, n, n, &one, nullptr, n, nullptr, n);
      rocsolver_dsyevd(p->rb, rocblas_evect_original, rocblas_fill_lower, n, nullptr, n, nullptr, nullptr, nullptr);
      rocsolver_dsyev(p->rb, rocblas_evect_original, rocblas_fill_lower, n, nullptr, n, nullptr, nullptr, nullptr);
    }
  } else {
    rocsolver_zpotrf(p->rb, rocblas_fill_lower, n, nullptr, n, nullptr);
    rocsolver_zpotri(p->rb, rocblas_fill_lower, n, nullptr, n, nullptr);
  }
  size_t sz = 0;
  RBCHK(rocblas_stop_device_memory_size_query(p->rb, &sz));
  *bytes = sz;
  return CHEB_OK;
}

// Workspace of the adjoint: one filter workspace and one Rayleigh-Ritz workspace, plus checkpoints, the
// recomputed segment, the adjoint vectors and the cross-density scratch.
struct BwdWs {
  Ws fw, rr;
  FftWs fft{};
  void* colc = nullptr;
  void* F[2] = {nullptr, nullptr};
  void* bar[3] = {nullptr, nullptr, nullptr};
  void *a = nullptr, *loca = nullptr;
  std::vector<void*> ck, seg;       // 2 ncp checkpoint vectors, k - 1 segment vectors
  std::vector<c128*> ckp, segp;     // their projections
  c128* pf[2] = {nullptr, nullptr};
  c128 *pbar = nullptr, *qa = nullptr, *pa = nullptr, *Dpa = nullptr, *B = nullptr;
  double *xpart = nullptr, *norms = nullptr;
  c128* bdots = nullptr;   // squared band norms of the adjoint vectors and of psi (2 nb)
  double* bal = nullptr;   // their balancing scales (nb)
  size_t total = 0;
};

cheb_status bwd_layout(cheb_plan p, int nb, int m, int k, void* base, BwdWs* w) {
  Bump b(base);
  const size_t eb = elem_bytes(p->prec);
  const size_t vec = size_t(p->npw) * std::max(nb, 1) * eb;
  const size_t pp = size_t(std::max(p->nproj, 1)) * std::max(nb, 1);
  Ws probe;
  CHK(ws_layout(p, CHEB_OP_FILTER, nb, nullptr, &probe));
  char* fwb = b.take<char>(probe.total);
  CHK(ws_layout(p, CHEB_OP_FILTER, nb, fwb, &w->fw));
  CHK(ws_layout(p, CHEB_OP_RR, nb, nullptr, &probe));
  char* rrb = b.take<char>(probe.total);
  CHK(ws_layout(p, CHEB_OP_RR, nb, rrb, &w->rr));
  const int fb = fft_batch_for(p, nb);
  const size_t colb = size_t(fb) * p->n * col_stride(p->ncol) * eb;
  w->fft.a = b.take<char>(colb);
  w->fft.b = b.take<char>(colb);
  w->colc = b.take<char>(colb);
  for (int i = 0; i < 2; ++i) w->F[i] = b.take<char>(vec);
  for (int i = 0; i < 3; ++i) w->bar[i] = b.take<char>(vec);
  w->a = b.take<char>(vec);
  w->loca = b.take<char>(vec);
  const int ncp = (m + k - 1) / k;
  w->ck.assign(2 * ncp, nullptr);
  w->ckp.assign(2 * ncp, nullptr);
  for (int i = 0; i < 2 * ncp; ++i) { w->ck[i] = b.take<char>(vec); w->ckp[i] = b.take<c128>(pp); }
  w->seg.assign(std::max(k - 1, 0), nullptr);
  w->segp.assign(std::max(k - 1, 0), nullptr);
  for (int i = 0; i + 1 < k; ++i) { w->seg[i] = b.take<char>(vec); w->segp[i] = b.take<c128>(pp); }
  for (int i = 0; i < 2; ++i) w->pf[i] = b.take<c128>(pp);
  w->pbar = b.take<c128>(pp);
  w->qa = b.take<c128>(pp);
  w->pa = b.take<c128>(pp);
  w->Dpa = b.take<c128>(pp);
  w->B = b.take<c128>(size_t(std::max(nb, 1)) * std::max(nb, 1));
  w->xpart = b.take<double>(cross_density_part_doubles(p->n, fb));
  w->norms = b.take<double>(std::max(nb, 1));
  w->bdots = b.take<c128>(2 * size_t(std::max(nb, 1)));
  w->bal = b.take<double>(std::max(nb, 1));
  w->total = b.off;
  return CHEB_OK;
}

cheb_status check_ws(cheb_plan p, int op, int nb, void* ws, size_t wsb, Ws* w) {
  Ws probe;
  CHK(ws_layout(p, op, nb, nullptr, &probe));
  if (wsb < probe.total) return fail(p, CHEB_ERR_WORKSPACE, "workspace too small: need " + std::to_string(probe.total));
  if (!ws) return fail(p, CHEB_ERR_ARG, "workspace is null");
  if (reinterpret_cast<uintptr_t>(ws) % kAlign) return fail(p, CHEB_ERR_ARG, "workspace not 256-byte aligned");
  return ws_layout(p, op, nb, ws, w);
}

cheb_status check_ready(cheb_plan p, bool need_all = true) {
  if (!p->have_V) return fail(p, CHEB_ERR_STATE, "potential not set");
  if (need_all && p->nproj > 0 && !p->have_P) return fail(p, CHEB_ERR_STATE, "projectors not set");
  if (need_all && p->nproj > 0 && !p->have_D) return fail(p, CHEB_ERR_STATE, "D not set");
  return CHEB_OK;
}

cheb_status check_block(cheb_plan p, const void* X, int ldx, int nb, const char* name) {
  if (nb < 0) return fail(p, CHEB_ERR_ARG, std::string(name) + ": nb < 0");
  if (nb > 0 && !X) return fail(p, CHEB_ERR_ARG, std::string(name) + " is null");
  if (ldx < p->npw) return fail(p, CHEB_ERR_ARG, std::string(name) + ": leading dimension < npw");
  return CHEB_OK;
}

// ---- operator pieces, templated on the band element type --------------------------------------------------------
// Pinned host staging of index lists copied to the device (band permutations, active sets): waits for the
// previous copy out of it, grows it to at least `count` ints.
cheb_status staging(cheb_plan p, size_t count) {
  if (p->lock_ev) HIPCHK(hipEventSynchronize(p->lock_ev));
  else HIPCHK(hipEventCreateWithFlags(&p->lock_ev, hipEventDisableTiming));
  if (p->lock_cap < count) {
    if (p->lock_host) HIPCHK(hipHostFree(p->lock_host));
    p->lock_host = nullptr;
    p->lock_cap = 0;
    HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&p->lock_host), std::max<size_t>(count, 1) * sizeof(int),
                         hipHostMallocDefault));
    p->lock_cap = count;
  }
  return CHEB_OK;
}

template <typename T> struct Ops {
  using C = cx<T>;
  cheb_plan p;
  hipStream_t st;
  FftGeom geom() const { return FftGeom{p->n, p->ncol, p->npw, p->rx, p->col, p->ent, p->xline}; }
  // algorithmic flops of one band's plane pass: on each of the n z-planes, 2 (2 rx + 1) y-transforms of the
  // nonzero x-lines and 2 n x-transforms of the rows, 5 n log2 n flops per complex length-n transform, and the
  // real-space product with V(r) (2 per point)
  double plane_flops() const {
    const double n = p->n, nx = 2.0 * p->rx + 1.0;
    return n * ((2.0 * nx + 2.0 * n) * 5.0 * n * std::log2(n) + 2.0 * n * n);
  }
  const C* P() const { return static_cast<const C*>(p->P); }

  // out = (K + V_loc) X, batched over bands through the disk-column buffers
  cheb_status hloc(const C* X, long ldx, int nb, C* out, long ldo, const FftWs& fw) {
    if (p->gamma) return hloc_gamma(X, ldx, nb, out, ldo, fw);
    const int fb = fft_batch_for(p, nb);
    const FftGeom g = geom();
    const C* tw = static_cast<const C*>(p->tw);
    for (int b0 = 0; b0 < nb; b0 += fb) {
      const int cnt = std::min(fb, nb - b0);
      C* ca = static_cast<C*>(fw.a);
      C* cb = static_cast<C*>(fw.b);
      const double b = sizeof(C), colv = double(p->n) * p->ncol, npw = p->npw;
      {
        Timed t(p, st, CHEB_T_FFT_COL_INV, cnt * (npw + colv) * b, 0.0);
        HIPCHK(fft_col_inverse<T>(g, tw, X + long(b0) * ldx, ldx, cnt, ca, st));
      }
      {
        Timed t(p, st, CHEB_T_FFT_PLANE, cnt * 2.0 * colv * b, cnt * plane_flops());
        HIPCHK(fft_plane<T>(g, tw, static_cast<const T*>(p->Vt), ca, cb, cnt, st));
      }
      {
        Timed t(p, st, CHEB_T_FFT_COL_FWD, cnt * (colv + 2.0 * npw) * b, 0.0);
        HIPCHK(fft_col_forward<T>(g, tw, cb, X + long(b0) * ldx, ldx, static_cast<const T*>(p->kin),
                                  out + long(b0) * ldo, ldo, cnt, st));
      }
    }
    return CHEB_OK;
  }

  // Gamma point: bands 2j and 2j+1 go through one complex transform as psi_2j + i psi_2j+1 (both real in
  // real space, V real), then are separated from the values at G and -G.
  cheb_status hloc_gamma(const C* X, long ldx, int nb, C* out, long ldo, const FftWs& fw) {
    const int fb = fft_batch_for(p, nb);
    const FftGeom g = geom();
    const C* tw = static_cast<const C*>(p->tw);
    C* ga = static_cast<C*>(fw.ga);
    C* gb = static_cast<C*>(fw.gb);
    const long npf = p->npf;
    for (int b0 = 0; b0 < nb; b0 += fb) {
      const int cnt = std::min(fb, nb - b0), npair = (cnt + 1) / 2;
      C* ca = static_cast<C*>(fw.a);
      C* cb = static_cast<C*>(fw.b);
      const double b = sizeof(C), colv = double(p->n) * p->ncol, npw = p->npw;
      {
        Timed t(p, st, CHEB_T_FFT_COL_INV, (cnt * npw + npair * (2.0 * npf + colv)) * b, 0.0);
        HIPCHK((gamma_pack<T>(p->npf, cnt, p->gmap, p->h0, X + long(b0) * ldx, ldx, ga, npf, st)));
        HIPCHK(fft_col_inverse<T>(g, tw, ga, npf, npair, ca, st));
      }
      {
        Timed t(p, st, CHEB_T_FFT_PLANE, npair * 2.0 * colv * b, npair * plane_flops());
        HIPCHK(fft_plane<T>(g, tw, static_cast<const T*>(p->Vt), ca, cb, npair, st));
      }
      {
        Timed t(p, st, CHEB_T_FFT_COL_FWD, (npair * (colv + 2.0 * npf) + 2.0 * cnt * npw) * b, 0.0);
        HIPCHK(fft_col_forward<T>(g, tw, cb, nullptr, 0, nullptr, gb, npf, npair, st));
        HIPCHK((gamma_split<T>(p->npw, cnt, p->gpair, p->h0, gb, npf, static_cast<const T*>(p->kin),
                               X + long(b0) * ldx, ldx, out + long(b0) * ldo, ldo, st)));
      }
    }
    return CHEB_OK;
  }

  // pout (nproj x nb, c128) = P^H X. exact: FP64 MFMA whatever the plan precision (products of complex64
  // inputs are exact in FP64), for the Rayleigh-Ritz matrices of a mixed plan.
  bool use_split() const { return std::is_same<T, float>::value && p->split_gemm && p->hproj.p; }

  // pout (nproj x nb, c128) = P^H X. exact: FP64 MFMA whatever the plan precision (products of complex64
  // inputs are exact in FP64), for the Rayleigh-Ritz matrices of a mixed plan. Otherwise a mixed plan uses
  // the FP16 hi/lo split MFMA on X scaled per band by a power of two (FP32-level accuracy).
  cheb_status project(const C* X, long ldx, int nb, c128* pout, const Ws& w, bool exact = false, long ldo = 0) {
    Epi<double> e;
    e.out = pout;
    e.ldo = ldo > 0 ? ldo : p->nproj;
    e.real_only = p->gamma != 0;  // projections of real functions are real
    const double b = sizeof(C), np = p->nproj, npw = p->npw;
    Timed t(p, st, CHEB_T_PROJECT, (npw * np + npw * nb) * b + np * nb * 16.0, 8.0 * np * nb * npw);
    if (exact) {
      HIPCHK((gemm<double, T, T, double>(GEMM_CN, p->nproj, nb, p->npw, P(), p->npw, X, ldx, e,
                                         gemm_pick_splits(p->nproj, nb, p->npw), w.part, st, ROLE_PROJECT)));
    } else if (use_split()) {
      if constexpr (std::is_same<T, float>::value) {
        HIPCHK(column_scales<float>(p->npw, nb, X, ldx, w.bsc, st));
        const int splits = gemm_h_pick_splits(p->nproj, nb, p->npw);
        if (w.hx) {
          // the filters' workspaces hold the bands split once into FP16 planes (the same values the GEMM would
          // split on the fly), which the GEMM then reads as plain 16-byte rows
          HIPCHK(split_columns(p->npw, nb, X, ldx, w.bsc, w.hx, w.hx_ld, st));
          HalfPlanes xp;
          xp.p = w.hx;
          xp.rows = nb;
          xp.ld = w.hx_ld;
          HIPCHK((gemm_h_pre<double>(GEMM_CN, p->nproj, nb, p->npw, p->hproj, xp, w.bsc, e, splits, w.part, st,
                                     ROLE_PROJECT)));
        } else {
          HIPCHK((gemm_h<float, double>(GEMM_CN, p->nproj, nb, p->npw, p->hproj, X, ldx, w.bsc, e, splits, w.part,
                                        st, ROLE_PROJECT)));
        }
      }
    } else {
      HIPCHK((gemm<T, T, T, double>(GEMM_CN, p->nproj, nb, p->npw, P(), p->npw, X, ldx, e,
                                    gemm_pick_splits(p->nproj, nb, p->npw), w.part, st, ROLE_PROJECT)));
    }
    return CHEB_OK;
  }

  // out = alpha P wv + bL L (+ bU U + bW W): back-projection with the vector epilogue
  cheb_status backproject(const c128* wv, int nb, Epi<T> e, const Ws& w, long ldw = 0) {
    const double b = sizeof(C), np = p->nproj, npw = p->npw;
    const double vecs = 1.0 + (e.L ? 1 : 0) + (e.U ? 1 : 0) + (e.W ? 1 : 0);
    if (ldw <= 0) ldw = p->nproj;
    Timed t(p, st, CHEB_T_BACKPROJECT, npw * np * b + np * nb * 16.0 + vecs * npw * nb * b, 8.0 * npw * nb * np);
    if (use_split()) {
      if constexpr (std::is_same<T, float>::value) {
        // the small projector-space operand split once into FP16 planes (not once per block and K tile)
        if (!w.hb) return fail(p, CHEB_ERR_STATE, "workspace laid out without the split back-projection operand");
        HIPCHK(column_scales<double>(p->nproj, nb, wv, ldw, w.bsc, st));
        HIPCHK(split_columns(p->nproj, nb, wv, ldw, w.bsc, w.hb, w.hb_ld, st));
        HalfPlanes bp;
        bp.p = w.hb;
        bp.rows = nb;
        bp.ld = w.hb_ld;
        HIPCHK((gemm_h_pre<float>(GEMM_NN, p->npw, nb, p->nproj, p->hback, bp, w.bsc, e, 1, nullptr, st,
                                  ROLE_BACKPROJECT)));
      }
    } else {
      HIPCHK((gemm<T, T, double, T>(GEMM_NN, p->npw, nb, p->nproj, P(), p->npw, wv, ldw, e, 1, nullptr, st,
                                    ROLE_BACKPROJECT)));
    }
    return CHEB_OK;
  }

  // small projector-space product out = alpha A x (+ epilogue): A nproj x K (c128, ld lda), x K x nb (ld ldx)
  cheb_status small(const c128* A, long lda, int K, const c128* x, long ldx, int nb, Epi<double> e, c128* part) {
    const int np = p->nproj;
    const double vecs = 2.0 + (e.L ? 1 : 0) + (e.U ? 1 : 0) + (e.W ? 1 : 0);
    Timed t(p, st, CHEB_T_SMALL, double(np) * K * 16.0 + vecs * np * nb * 16.0, 8.0 * np * double(K) * nb);
    HIPCHK((gemm<double, double, double, double>(GEMM_NN, np, nb, K, A, lda, x, ldx, e, gemm_pick_splits(np, nb, K),
                                                 part, st)));
    return CHEB_OK;
  }
  cheb_status small(const c128* M, const c128* x, int nb, Epi<double> e, c128* part) {
    return small(M, p->nproj, p->nproj, x, p->nproj, nb, e, part);
  }

  // out = C^-1 b, C = Q^-1 + P^H P (Sec. 5.1): directly with the stored inverse, or by cap_iters corrections of
  // iterative refinement preconditioned by the atom-block diagonal M of C: q = M^-1 b, then r = b - C q,
  // q += M^-1 r. b and out must not overlap.
  cheb_status cinv(const c128* b, long ldb, int nb, c128* out, long ldo, const Ws& w) {
    const int np = p->nproj;
    if (p->cap_iters <= 0) {
      Epi<double> e;
      e.out = out; e.ldo = ldo;
      return small(p->Cinv, np, np, b, ldb, nb, e, w.part);
    }
    if (!w.cr) return fail(p, CHEB_ERR_STATE, "workspace laid out for the direct capacitance solve");
    HIPCHK(block_diag_apply_c(np, nb, p->pinfo, p->Minv, b, ldb, out, ldo, false, st));
    for (int k = 0; k < p->cap_iters; ++k) {
      Epi<double> e;
      e.out = w.cr; e.ldo = np; e.alpha = -1.0;
      e.L = b; e.ldl = ldb; e.bL = 1.0;
      CHK(small(p->Cmat, np, np, out, ldo, nb, e, w.part));
      HIPCHK(block_diag_apply_c(np, nb, p->pinfo, p->Minv, w.cr, np, out, ldo, true, st));
    }
    return CHEB_OK;
  }

  cheb_status apply_H(const C* X, long ldx, C* Y, long ldy, int nb, const Ws& w) {
    CHK(hloc(X, ldx, nb, Y, ldy, w.fft));
    if (p->nproj == 0) return CHEB_OK;
    CHK(project(X, ldx, nb, w.p0, w));
    HIPCHK(block_diag_apply(p->nproj, nb, p->pinfo, p->D, w.p0, p->nproj, w.Dp, p->nproj, st));
    Epi<T> e;
    e.out = Y; e.ldo = ldy; e.alpha = 1.0;
    e.L = Y; e.ldl = ldy; e.bL = 1.0;
    return backproject(w.Dp, nb, e, w);
  }

  cheb_status apply_S(const C* X, long ldx, C* Y, long ldy, int nb, const Ws& w) {
    if (!p->has_overlap || p->nproj == 0) {
      HIPCHK((convert_copy<T, T>(p->npw, nb, X, ldx, Y, ldy, st)));
      return CHEB_OK;
    }
    CHK(project(X, ldx, nb, w.p0, w));
    HIPCHK(diag_apply(p->nproj, nb, p->Q, w.p0, p->nproj, w.Dp, p->nproj, st));
    Epi<T> e;
    e.out = Y; e.ldo = ldy; e.alpha = 1.0;
    e.L = X; e.ldl = ldx; e.bL = 1.0;
    return backproject(w.Dp, nb, e, w);
  }

  cheb_status apply_Sinv(const C* X, long ldx, C* Y, long ldy, int nb, const Ws& w) {
    if (!p->has_overlap || p->nproj == 0) {
      HIPCHK((convert_copy<T, T>(p->npw, nb, X, ldx, Y, ldy, st)));
      return CHEB_OK;
    }
    CHK(project(X, ldx, nb, w.p0, w));
    CHK(cinv(w.p0, p->nproj, nb, w.Dp, p->nproj, w));
    Epi<T> e;
    e.out = Y; e.ldo = ldy; e.alpha = -1.0;
    e.L = X; e.ldl = ldx; e.bL = 1.0;
    return backproject(w.Dp, nb, e, w);
  }

  // One step of the recurrence (Alg. 2 inner loop): out = s1 (S^-1 H cur - c cur) - s2 prev, with the
  // projections p = P^H psi carried alongside (reuse trick, Sec. 5.1). out may alias prev (and pout pprev);
  // prev / pprev are unused for i = 1.
  // loc_in: (K + V) cur given by the caller (ld npw), else computed here
  cheb_status filter_step(int i, const C* cur, long ldc, const C* prev, long ldp, C* out, long ldo,
                          const c128* pcur, const c128* pprev, c128* pout, int nb, double c, double r, const Ws& w,
                          const C* loc_in = nullptr) {
    const int np = p->nproj;
    const long npw = p->npw;
    const double s1 = (i == 1 ? 1.0 : 2.0) / r;
    const double s2 = (i == 1 ? 0.0 : 1.0);
    const C* loc = loc_in;
    if (!loc) {
      C* lw = static_cast<C*>(w.loc);
      CHK(hloc(cur, ldc, nb, lw, npw, w.fft));
      loc = lw;
    }
    if (np == 0) {
      HIPCHK((axpbypcz<T>(npw, nb, s1, loc, npw, -s1 * c, cur, ldc, -s2, i == 1 ? nullptr : prev, ldp, out, ldo, st)));
      return CHEB_OK;
    }
    // projector space, stacked [p_loc; D p] (ld 2 np): p_loc = P^H loc, D p from the carried p = P^H psi.
    // With p_phi = P^H H psi = p_loc + G D p and q = C^-1 p_phi (Sec. 5.1):
    //   S^-1 H psi = loc + P w,  w = D p - q,   P^H S^-1 H psi = p_phi - G q = p_loc + G w   (reuse trick)
    // With an overlap, C = Q^-1 + G gives C^-1 G = I - C^-1 Q^-1 and G = C - Q^-1, hence
    //   w = C^-1 (Q^-1 D p - p_loc),   P^H S^-1 H psi = Q^-1 (D p - w):
    // one nproj x nproj product per step. S = I: w = D p and P^H H psi = p_loc + G D p.
    const long l2 = 2L * np;
    c128* pl = w.ploc;
    c128* dp = w.ploc + np;
    CHK(project(loc, npw, nb, pl, w, false, l2));
    HIPCHK(block_diag_apply(np, nb, p->pinfo, p->D, pcur, np, dp, l2, st));
    const c128* wv = dp;
    long ldw = l2;
    if (p->has_overlap) {
      HIPCHK(overlap_rhs(np, nb, p->Q, dp, l2, pl, l2, pl, l2, st));  // u over p_loc, which is not needed after
      CHK(cinv(pl, l2, nb, w.w, np, w));
      wv = w.w;
      ldw = np;
    }
    // psi^i = s1 (loc + P w - c psi^(i-1)) - s2 psi^(i-2)
    Epi<T> e;
    e.out = out; e.ldo = ldo; e.alpha = s1;
    e.L = loc; e.ldl = npw; e.bL = s1;
    e.U = cur; e.ldu = ldc; e.bU = -s1 * c;
    if (i > 1) { e.W = prev; e.ldw = ldp; e.bW = -s2; }
    CHK(backproject(wv, nb, e, w, ldw));
    if (p->has_overlap) {
      // p^i = s1 (Q^-1 (D p - w) - c p^(i-1)) - s2 p^(i-2)
      HIPCHK(overlap_recur(np, nb, p->Q, dp, l2, w.w, np, s1, c, pcur, np, s2, i > 1 ? pprev : nullptr, np, pout, np,
                           st));
      return CHEB_OK;
    }
    // p^i = s1 (p_loc + G w - c p^(i-1)) - s2 p^(i-2)
    Epi<double> e3;
    e3.out = pout; e3.ldo = np; e3.alpha = s1;
    e3.L = pl; e3.ldl = l2; e3.bL = s1;
    e3.U = pcur; e3.ldu = np; e3.bU = -s1 * c;
    if (i > 1) { e3.W = pprev; e3.ldw = np; e3.bW = -s2; }
    CHK(small(p->G, np, np, wv, ldw, nb, e3, w.part));
    return CHEB_OK;
  }

  // Before step i of the recurrence (cur = psi^(i-1), prev = psi^(i-2)). The reuse trick of Sec. 5.1 carries
  // p = P^H psi in projector space; with complex64 bands the carried values drift from the projections of the
  // rounded vectors, and the recurrence amplifies the drift like the bands it multiplies. With the drift monitor
  // on, the carried projections of cur are compared with P^H cur recomputed from the vector (FP64 products); at
  // the steps i = 1 + k * resync both carried projections are replaced by the projections of their vectors.
  cheb_status resync_step(int i, const C* cur, long ldc, c128* pcur, const C* prev, long ldp, c128* pprev, int nb,
                          const Ws& w) {
    const int np = p->nproj;
    if (np == 0 || nb == 0 || i < 2) return CHEB_OK;
    if (p->drift_on) {
      CHK(project(cur, ldc, nb, w.pfresh, w, true));
      HIPCHK(col_rel_diff(np, nb, pcur, np, w.pfresh, np, w.dcol, st));
      std::vector<double> h(nb);
      HIPCHK(hipMemcpyAsync(h.data(), w.dcol, nb * sizeof(double), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      for (double v : h) p->drift_max = std::isnan(v) ? v : std::max(p->drift_max, v);
      p->drift_checks += 1;
    }
    if (p->resync > 0 && (i - 1) % p->resync == 0) {
      CHK(project(cur, ldc, nb, pcur, w));
      if (i > 2) CHK(project(prev, ldp, nb, pprev, w));  // psi^0's projections are exact already
    }
    return CHEB_OK;
  }

  // Alg. 2 inner loop for the whole block. psi^i overwrites psi^(i-2); buffers alternate X, W. With pin, the
  // projections P^H X come from the caller (those the previous Rayleigh-Ritz step returned for its rotated block)
  // instead of a product over the sphere (nproj x nb, ld nproj); with hxin, so does (K + V) X (nb rows of npw),
  // which the first step then does not transform.
  cheb_status filter(C* X, long ldx, int nb, int m, double c, double r, const Ws& w, const c128* pin = nullptr,
                     const C* hxin = nullptr) {
    if (m == 0 || nb == 0) return CHEB_OK;
    const int np = p->nproj;
    const long npw = p->npw;
    C* buf[2] = {X, static_cast<C*>(w.W)};
    long ld[2] = {ldx, npw};
    c128* pb[2] = {w.p0, w.p1};
    if (np > 0) {
      if (pin) HIPCHK(hipMemcpyAsync(pb[0], pin, size_t(np) * nb * sizeof(c128), hipMemcpyDeviceToDevice, st));
      else CHK(project(X, ldx, nb, pb[0], w));
    }
    for (int i = 1; i <= m; ++i) {
      const int ci = (i - 1) & 1, oi = i & 1;
      CHK(resync_step(i, buf[ci], ld[ci], pb[ci], buf[oi], ld[oi], pb[oi], nb, w));
      CHK(filter_step(i, buf[ci], ld[ci], buf[oi], ld[oi], buf[oi], ld[oi], pb[ci], pb[oi], pb[oi], nb, c, r, w,
                      i == 1 ? hxin : nullptr));
    }
    if (m & 1) HIPCHK((convert_copy<T, T>(npw, nb, buf[1], npw, X, ldx, st)));
    return CHEB_OK;
  }

  // Per-band degrees (locking, Sec. 5.4). The bands with degree > 0 are gathered into w.Xs in order of
  // decreasing degree (idx[0, na)); step i runs the recurrence of Alg. 2 on the first active[i-1] of them,
  // a shrinking prefix, so a band's columns are never touched after its last step. psi^i lands in buffer
  // i & 1: even-degree bands are scattered back from w.Xs (idx[na, na + 2 ne): sources, then destinations),
  // odd-degree bands from w.W (the next 2 no entries).
  cheb_status filter_degrees(C* X, long ldx, const std::vector<int>& active, const int* idx, int ne, int no, double c,
                             double r, const Ws& w) {
    const long npw = p->npw;
    const int na = active.empty() ? 0 : active[0];
    if (na == 0) return CHEB_OK;
    C* buf[2] = {static_cast<C*>(w.Xs), static_cast<C*>(w.W)};
    c128* pb[2] = {w.p0, w.p1};
    HIPCHK((permute_cols<T>(npw, na, X, ldx, idx, buf[0], npw, nullptr, st)));
    if (p->nproj > 0) CHK(project(buf[0], npw, na, pb[0], w));
    for (int i = 1; i <= int(active.size()); ++i) {
      const int ci = (i - 1) & 1, oi = i & 1;
      CHK(resync_step(i, buf[ci], npw, pb[ci], buf[oi], npw, pb[oi], active[i - 1], w));
      CHK(filter_step(i, buf[ci], npw, buf[oi], npw, buf[oi], npw, pb[ci], pb[oi], pb[oi], active[i - 1], c, r, w));
    }
    const int* ev = idx + na;
    const int* od = ev + 2 * ne;
    HIPCHK((permute_cols<T>(npw, ne, buf[0], npw, ev, X, ldx, ev + ne, st)));
    HIPCHK((permute_cols<T>(npw, no, buf[1], npw, od, X, ldx, od + no, st)));
    return CHEB_OK;
  }

  // H_X = X^H H X, S_X = X^H S X into w.Hs, w.Ss; leaves loc = (K + V) X and p = P^H X in the workspace
  cheb_status subspace(const C* X, long ldx, int nb, const Ws& w) {
    const int np = p->nproj;
    const long npw = p->npw;
    C* loc = static_cast<C*>(w.loc);
    CHK(hloc(X, ldx, nb, loc, npw, w.fft));
    // the projections and their projector-space products first, so that the Gram timer below does not enclose
    // the projection's own timer
    if (np > 0) {
      CHK(project(X, ldx, nb, w.p0, w, true));
      HIPCHK(block_diag_apply(np, nb, p->pinfo, p->D, w.p0, np, w.Dp, np, st));
      if (p->has_overlap) HIPCHK(diag_apply(np, nb, p->Q, w.p0, np, w.q, np, st));
    }
    Timed t(p, st, CHEB_T_RR_GRAM, 3.0 * npw * nb * sizeof(C) + 2.0 * nb * nb * 16.0, 16.0 * npw * nb * nb);
    Epi<double> eh;
    eh.out = w.Hs; eh.ldo = nb; eh.real_only = p->gamma != 0;
    // FP64 MFMA in both precisions: with complex64 blocks the products are exact and the sums over npw
    // terms keep FP64 rounding, so the subspace matrices (and the Ritz values) are limited by the FP32
    // rounding of H X only, not by FP32 accumulation over the sphere.
    // H_X and S_X are Hermitian: the products form the tiles on and above the diagonal only (half the work), and
    // the strictly lower part is their conjugate transpose (the eigensolver reads one triangle; the refinement
    // the whole matrices)
    HIPCHK((gemm<double, T, T, double>(GEMM_CN, nb, nb, p->npw, X, ldx, loc, npw, eh,
                                       gemm_upper_splits(nb, p->npw), w.part, st, ROLE_SUBSPACE, true)));
    Epi<double> es;
    es.out = w.Ss; es.ldo = nb; es.real_only = p->gamma != 0;
    HIPCHK((gemm<double, T, T, double>(GEMM_CN, nb, nb, p->npw, X, ldx, X, ldx, es,
                                       gemm_upper_splits(nb, p->npw), w.part, st, ROLE_SUBSPACE, true)));
    if (np > 0) {
      Epi<double> e2;
      e2.out = w.Hs; e2.ldo = nb; e2.L = w.Hs; e2.ldl = nb; e2.bL = 1.0;
      HIPCHK((gemm<double, double, double, double>(GEMM_CN, nb, nb, np, w.p0, np, w.Dp, np, e2,
                                                   gemm_upper_splits(nb, np), w.part, st, ROLE_SMALL, true)));
      if (p->has_overlap) {
        Epi<double> e3;
        e3.out = w.Ss; e3.ldo = nb; e3.L = w.Ss; e3.ldl = nb; e3.bL = 1.0;
        HIPCHK((gemm<double, double, double, double>(GEMM_CN, nb, nb, np, w.p0, np, w.q, np, e3,
                                                     gemm_upper_splits(nb, np), w.part, st, ROLE_SMALL, true)));
      }
    }
    HIPCHK(hermitian_lower(nb, w.Hs, nb, st));
    HIPCHK(hermitian_lower(nb, w.Ss, nb, st));
    return CHEB_OK;
  }

  // Warm start: after the column scaling the previous Ritz vectors make Z' close to I. Generalized iterative
  // refinement X <- X (I + F) (first-order correction of X^H S' X = I, X^H H' X diagonal) converges
  // quadratically from there using only n^3 products. Where close Ritz values are strongly coupled (max |F| >
  // kClusterStep), the pairs with |F_ij| > kClusterTie are grouped into clusters whose pencils are solved
  // exactly, X <- X Q, before the first-order steps resume. The result is accepted only after an explicit
  // check of both conditions. Returns false (nothing written to ritz / Hs) when it does not converge.
  static constexpr double kClusterStep = 0.5, kClusterTie = 0.2;
  static constexpr int kRefineIters = 40, kStallWindow = 5;
  static constexpr double kRefineAccept = 1e-11;

  // connected components of the coupling graph (host union-find over the bit matrix); false if one has more
  // than kClusterMax members
  bool clusters_from_bits(int n, const std::vector<unsigned>& bits, std::vector<int>& idx, std::vector<int>& off) {
    const int W = (n + 31) / 32;
    std::vector<int> parent(n);
    for (int i = 0; i < n; ++i) parent[i] = i;
    auto find = [&](int x) {
      while (parent[x] != x) { parent[x] = parent[parent[x]]; x = parent[x]; }
      return x;
    };
    for (int i = 0; i < n; ++i)
      for (int wd = 0; wd < W; ++wd)
        for (unsigned m = bits[size_t(i) * W + wd]; m; m &= m - 1) {
          const int j = 32 * wd + __builtin_ctz(m);
          const int a = find(i), b = find(j);
          if (a != b) parent[std::max(a, b)] = std::min(a, b);
        }
    std::vector<int> count(n, 0);
    for (int i = 0; i < n; ++i) count[find(i)] += 1;
    idx.clear();
    off.assign(1, 0);
    for (int r = 0; r < n; ++r) {
      if (find(r) != r || count[r] < 2) continue;
      if (count[r] > kClusterMax) return false;
      for (int i = r; i < n; ++i)
        if (find(i) == r) idx.push_back(i);
      off.push_back(int(idx.size()));
    }
    return true;
  }

  bool rr_refine(int n, double* ritz, const Ws& w, cheb_status* st_out) {
    *st_out = CHEB_OK;
    auto hip_fail = [&](hipError_t e) { *st_out = fail(p, CHEB_ERR_HIP, std::string("refinement: ") + hipGetErrorString(e)); return false; };
    hipError_t e;
    const long n2 = 2L * n;
    c128 *X = w.Xa, *Xn = w.Xb;
    c128* HS = w.M2;  // [S'; H'] stacked: one product gives S' X and H' X together
    c128* TT = w.T;   // [S' X; H' X] (2n x n); read with ld n it is n x 2n with columns S'X_j, H'X_j interleaved
    // X^H [S'X_0, H'X_0, S'X_1, ...] in one of two buffers: X^H S' X has ld 2n at M, X^H H' X at M + n
    c128* Mbuf[2] = {w.M1, w.M1b};
    int mb = 0;
    int* cflag = w.flags + 3;  // cleared with the other flags before rr_prepare
    constexpr int kSlot = kRefineBlocksMax + 1;  // staging slot: block maxima, then the cluster flag
    if (!p->rr_host) {
      const hipError_t ea = hipHostMalloc(reinterpret_cast<void**>(&p->rr_host), 2 * kSlot * sizeof(double),
                                          hipHostMallocDefault);
      if (ea != hipSuccess) { p->rr_host = nullptr; return hip_fail(ea); }
    }
    for (hipEvent_t& ev : p->rr_ev)
      if (!ev && (e = hipEventCreateWithFlags(&ev, hipEventDisableTiming))) { ev = nullptr; return hip_fail(e); }
    double* const hst = p->rr_host;
    if ((e = convert_copy<double, double>(n, n, w.Ss, n, HS, n2, st))) return hip_fail(e);
    if ((e = convert_copy<double, double>(n, n, w.Hs, n, HS + n, n2, st))) return hip_fail(e);
    if ((e = identity_matrix(n, X, st))) return hip_fail(e);
    const c128* M1 = w.Ss;
    const c128* M2 = w.Hs;
    long ld = n;
    bool conv = false;
    std::vector<double> hist;
    std::vector<unsigned> bits;
    std::vector<int> cidx, coff;
    static const bool trace = std::getenv("CHEBFD_TRACE_RR") != nullptr;  // diagnostics: correction sizes
    const int nbm = refine_blocks(n);
    auto products = [&](const c128* Xc, c128* Mo) {
      Epi<double> e1;
      e1.out = TT; e1.ldo = n2;
      hipError_t r = gemm<double, double, double, double>(GEMM_NN, 2 * n, n, n, HS, n2, Xc, n, e1,
                                                          gemm_pick_splits(2 * n, n, n), w.part, st, ROLE_SUBSPACE);
      if (r != hipSuccess) return r;
      Epi<double> e2;
      e2.out = Mo; e2.ldo = n;
      return gemm<double, double, double, double>(GEMM_CN, n, 2 * n, n, Xc, n, TT, n, e2, gemm_pick_splits(n, 2 * n, n),
                                                  w.part, st, ROLE_SUBSPACE);
    };
    // corrections F of the X whose products are (m1, m2) and their block maxima and the cluster flag staged in
    // slot s, the slot's event recorded after the copies
    auto corrections = [&](const c128* m1, const c128* m2, long l, int s) {
      hipError_t r = refine_update(n, m1, l, m2, l, w.F, w.lam, w.absF, w.bmax, st);
      if (!r) r = hipMemcpyAsync(hst + s * kSlot, w.bmax, nbm * sizeof(double), hipMemcpyDeviceToHost, st);
      if (!r) r = hipMemcpyAsync(hst + s * kSlot + kRefineBlocksMax, cflag, sizeof(int), hipMemcpyDeviceToHost, st);
      if (!r) r = hipEventRecord(p->rr_ev[s], st);
      return r;
    };
    auto first_order = [&]() {  // Xn = X (I + F)
      Epi<double> eu;
      eu.out = Xn; eu.ldo = n; eu.L = X; eu.ldl = n; eu.bL = 1.0;
      return gemm<double, double, double, double>(GEMM_NN, n, n, n, X, n, w.F, n, eu, gemm_pick_splits(n, n, n), w.part,
                                                  st, ROLE_SUBSPACE);
    };
    // Invariant at the top of an iteration: the corrections of the current X are staged in slot `slot`.
    int slot = 0;
    if ((e = corrections(M1, M2, ld, slot))) return hip_fail(e);
    for (int it = 0; it < kRefineIters; ++it) {
      // From the second iteration on (corrections below the cluster threshold are then the rule) the first-order
      // step, its products and the next corrections are queued before this iteration's max|F| is read, so that
      // the device works while the host waits; they touch only the spare X, the other product buffer, F and the
      // other staging slot, and are dropped if the step turns out to need clusters.
      const bool spec = it > 0;
      if (spec) {
        if ((e = first_order()) || (e = products(Xn, Mbuf[mb ^ 1])) ||
            (e = corrections(Mbuf[mb ^ 1], Mbuf[mb ^ 1] + n, n2, slot ^ 1)))
          return hip_fail(e);
      }
      if ((e = hipEventSynchronize(p->rr_ev[slot]))) return hip_fail(e);
      double maxF = 0.0;
      const double* hs = hst + slot * kSlot;
      for (int b = 0; b < nbm; ++b) maxF = std::isnan(hs[b]) ? hs[b] : std::max(maxF, hs[b]);
      int bad = 0;
      std::memcpy(&bad, hs + kRefineBlocksMax, sizeof(int));
      if (trace) std::fprintf(stderr, "[rr-refine] n=%d it=%d max|F|=%.3e\n", n, it, maxF);
      if (bad || std::isnan(maxF)) return false;
      // leave when no longer converging: no halving against the best value before the last kStallWindow
      hist.push_back(maxF);
      if (int(hist.size()) > kStallWindow &&
          maxF > 0.5 * *std::min_element(hist.begin(), hist.end() - kStallWindow))
        return false;
      if (spec && maxF <= kClusterStep) {  // the queued first-order step stands
        std::swap(X, Xn);
        mb ^= 1;
        M1 = Mbuf[mb];
        M2 = Mbuf[mb] + n;
        ld = n2;
        slot ^= 1;
        if (maxF < 1e-10) { conv = true; break; }
        continue;
      }
      // the speculative step (if any) is dropped: recompute the corrections of the current X
      if (spec && (e = refine_update(n, M1, ld, M2, ld, w.F, w.lam, w.absF, w.bmax, st))) return hip_fail(e);
      bool cluster = false;
      if (maxF > kClusterStep) {
        const int W = (n + 31) / 32;
        bits.resize(size_t(n) * W);
        if ((e = coupling_bits(n, w.absF, kClusterTie, w.bits, st))) return hip_fail(e);
        if ((e = hipMemcpyAsync(bits.data(), w.bits, bits.size() * sizeof(unsigned), hipMemcpyDeviceToHost, st)))
          return hip_fail(e);
        if ((e = hipStreamSynchronize(st))) return hip_fail(e);
        if (!clusters_from_bits(n, bits, cidx, coff)) return false;
        cluster = coff.size() > 1;
        if (trace && cluster) {
          int big = 0;
          for (size_t c = 0; c + 1 < coff.size(); ++c) big = std::max(big, coff[c + 1] - coff[c]);
          std::fprintf(stderr, "[rr-refine]   %zu clusters, %zu bands, largest %d\n", coff.size() - 1, cidx.size(), big);
        }
      }
      if (cluster) {
        if ((e = hipMemcpyAsync(w.cidx, cidx.data(), cidx.size() * sizeof(int), hipMemcpyHostToDevice, st)) ||
            (e = hipMemcpyAsync(w.coff, coff.data(), coff.size() * sizeof(int), hipMemcpyHostToDevice, st)) ||
            (e = identity_matrix(n, w.F, st)) ||
            (e = cluster_eig(int(coff.size()) - 1, M1, ld, M2, ld, w.cidx, w.coff, w.F, n, cflag, st)))
          return hip_fail(e);
        // the host vectors are reused next iteration: the copies above must have left them
        if ((e = hipStreamSynchronize(st))) return hip_fail(e);
        Epi<double> eq;
        eq.out = Xn; eq.ldo = n;
        if ((e = gemm<double, double, double, double>(GEMM_NN, n, n, n, X, n, w.F, n, eq, gemm_pick_splits(n, n, n),
                                                      w.part, st, ROLE_SUBSPACE))) return hip_fail(e);
      } else {
        if (!(maxF < 1.0)) return false;  // outside the region where first-order steps converge
        if ((e = first_order())) return hip_fail(e);
      }
      std::swap(X, Xn);
      if ((e = products(X, Mbuf[mb ^ 1]))) return hip_fail(e);
      mb ^= 1;
      M1 = Mbuf[mb];
      M2 = Mbuf[mb] + n;
      ld = n2;
      if (!cluster && maxF < 1e-10) { conv = true; break; }
      slot ^= 1;
      if ((e = corrections(M1, M2, ld, slot))) return hip_fail(e);
    }
    if (!conv) return false;
    double res[2] = {1.0, 1.0};
    if ((e = refine_check(n, M1, ld, M2, ld, w.bmax, w.res, st))) return hip_fail(e);
    if ((e = hipMemcpyAsync(res, w.res, 2 * sizeof(double), hipMemcpyDeviceToHost, st))) return hip_fail(e);
    if ((e = hipStreamSynchronize(st))) return hip_fail(e);
    if (trace) std::fprintf(stderr, "[rr-refine] check |X^H S' X - I| = %.2e, off-diagonal X^H H' X = %.2e\n", res[0], res[1]);
    // acceptance: S'-orthonormal and H'-diagonal to 1e-11, about 400 n eps at n = 256 (the rounding floor of
    // the n^3 products after a dozen corrections is a few 1e-13)
    if (!(res[0] <= kRefineAccept) || !(res[1] <= kRefineAccept)) return false;
    // eigenvalues of the verified X, ascending; Z = d .* X[:, perm] replaces H_X in w.Hs
    if ((e = refine_update(n, M1, ld, M2, ld, w.F, w.lam, w.absF, w.bmax, st))) return hip_fail(e);
    if ((e = sort_eigen(n, w.lam, ritz, w.perm, X, w.d, w.Hs, st))) return hip_fail(e);
    return true;
  }

  // pout: the projections of the rotated block, (P^H X) Z with the exact P^H X (nproj x nb, ld nproj);
  // hxout: (K + V) of the rotated block, ((K + V) X) Z (nb rows of npw)
  cheb_status rayleigh_ritz(C* X, long ldx, int nb, double* ritz, double* resid, const Ws& w,
                            c128* pout = nullptr, C* hxout = nullptr) {
    const int np = p->nproj;
    const long npw = p->npw;
    CHK(subspace(X, ldx, nb, w));
    HIPCHK((fill_zero<float>(reinterpret_cast<c64*>(w.flags), 2, st)));
    HIPCHK(rr_prepare(nb, w.Hs, w.Ss, w.d, w.flags, st));
    int flags[3] = {0, 0, 0};
    HIPCHK(hipMemcpyAsync(flags, w.flags, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (flags[1]) return fail(p, CHEB_ERR_NONFINITE, "non-finite entry in the subspace matrices");
    if (flags[0]) return fail(p, CHEB_ERR_NOT_PD, "X^H S X has a non-positive diagonal (zero or non-finite column)");
    // H_X Z = S_X Z Lambda: warm-started refinement, else reduction to standard form (S' = L L^H,
    // H^ = L^-1 H' L^-H, H^ U = U Lambda, Z' = L^-H U) with the library eigensolver, FP64 throughout
    bool refined = false;
    {
      Timed t(p, st, CHEB_T_RR_EIG, 0.0, 0.0);
      if (p->rr_refine && nb <= 2048) {
        cheb_status rs_ = CHEB_OK;
        refined = rr_refine(nb, ritz, w, &rs_);
        if (rs_ != CHEB_OK) return rs_;
      }
    }
    if (refined) {
      p->rr_refined += 1;
    } else {
      p->rr_fallback += 1;
      RBCHK(rocblas_set_stream(p->rb, st));
      RBCHK(rocblas_set_workspace(p->rb, w.solver, w.solver_bytes));
      rocblas_status rs = rocblas_status_success;
      // divide and conquer, checked for non-finite vectors (returned with info 0 on some inputs whose tridiagonal
      // splits into many deflated pieces); then the QR algorithm from a copy of the standard-form matrix
      int ef[3] = {0, 0, 0};  // factorization info, eigensolver info, non-finite vectors
      auto read_flags = [&]() -> hipError_t {
        hipError_t e = hipMemcpyAsync(ef, w.flags + 2, 2 * sizeof(int), hipMemcpyDeviceToHost, st);
        if (!e) e = hipMemcpyAsync(ef + 2, w.flags, sizeof(int), hipMemcpyDeviceToHost, st);
        if (!e) e = hipStreamSynchronize(st);
        return e;
      };
      if (p->gamma) {
        // real symmetric pencil (Gamma point): real factorization and eigensolver keep Z real, so the rotated
        // bands stay real functions
        Timed t(p, st, CHEB_T_RR_EIG, 0.0, 0.0);
        double* Hr = reinterpret_cast<double*>(w.Xa);
        double* Sr = reinterpret_cast<double*>(w.Xb);
        double* Hc = reinterpret_cast<double*>(w.T);  // copy of the standard-form matrix
        HIPCHK(real_part(nb, nb, w.Hs, nb, Hr, nb, st));
        HIPCHK(real_part(nb, nb, w.Ss, nb, Sr, nb, st));
        const double one = 1.0;
        rs = rocsolver_dpotrf(p->rb, rocblas_fill_lower, nb, Sr, nb, w.flags + 2);
        if (rs == rocblas_status_success)
          rs = rocblas_dtrsm(p->rb, rocblas_side_left, rocblas_fill_lower, rocblas_operation_none,
                             rocblas_diagonal_non_unit, nb, nb, &one, Sr, nb, Hr, nb);
        if (rs == rocblas_status_success)
          rs = rocblas_dtrsm(p->rb, rocblas_side_right, rocblas_fill_lower, rocblas_operation_transpose,
                             rocblas_diagonal_non_unit, nb, nb, &one, Sr, nb, Hr, nb);
        if (rs == rocblas_status_success) {
          HIPCHK(hipMemcpyAsync(Hc, Hr, size_t(nb) * nb * sizeof(double), hipMemcpyDeviceToDevice, st));
          rs = rocsolver_dsyevd(p->rb, rocblas_evect_original, rocblas_fill_lower, nb, Hr, nb, ritz, w.E, w.flags + 3);
        }
        if (rs == rocblas_status_success) {
          HIPCHK(fill_zero_real<int>(w.flags, 1, st));
          HIPCHK(flag_nonfinite_real(long(nb) * nb, Hr, w.flags, st));
          HIPCHK(read_flags());
          if (ef[0] == 0 && (ef[1] != 0 || ef[2] != 0)) {
            HIPCHK(hipMemcpyAsync(Hr, Hc, size_t(nb) * nb * sizeof(double), hipMemcpyDeviceToDevice, st));
            rs = rocsolver_dsyev(p->rb, rocblas_evect_original, rocblas_fill_lower, nb, Hr, nb, ritz, w.E, w.flags + 3);
            if (rs == rocblas_status_success) {
              HIPCHK(fill_zero_real<int>(w.flags, 1, st));
              HIPCHK(flag_nonfinite_real(long(nb) * nb, Hr, w.flags, st));
              HIPCHK(read_flags());
            }
          }
        }
        if (rs == rocblas_status_success && ef[0] == 0)
          rs = rocblas_dtrsm(p->rb, rocblas_side_left, rocblas_fill_lower, rocblas_operation_transpose,
                             rocblas_diagonal_non_unit, nb, nb, &one, Sr, nb, Hr, nb);
        if (rs == rocblas_status_success) HIPCHK(complex_from_real(nb, nb, Hr, nb, w.Hs, nb, st));
      } else {
        Timed t(p, st, CHEB_T_RR_EIG, 0.0, 0.0);
        rocblas_double_complex* Hd = reinterpret_cast<rocblas_double_complex*>(w.Hs);
        rocblas_double_complex* Ld = reinterpret_cast<rocblas_double_complex*>(w.Ss);
        c128* Hc = w.Xa;  // copy of the standard-form matrix
        const rocblas_double_complex one = {1.0, 0.0};
        rs = rocsolver_zpotrf(p->rb, rocblas_fill_lower, nb, Ld, nb, w.flags + 2);
        if (rs == rocblas_status_success)
          rs = rocblas_ztrsm(p->rb, rocblas_side_left, rocblas_fill_lower, rocblas_operation_none,
                             rocblas_diagonal_non_unit, nb, nb, &one, Ld, nb, Hd, nb);
        if (rs == rocblas_status_success)
          rs = rocblas_ztrsm(p->rb, rocblas_side_right, rocblas_fill_lower, rocblas_operation_conjugate_transpose,
                             rocblas_diagonal_non_unit, nb, nb, &one, Ld, nb, Hd, nb);
        if (rs == rocblas_status_success) {
          HIPCHK((convert_copy<double, double>(nb, nb, w.Hs, nb, Hc, nb, st)));
          rs = rocsolver_zheevd(p->rb, rocblas_evect_original, rocblas_fill_lower, nb, Hd, nb, ritz, w.E, w.flags + 3);
        }
        if (rs == rocblas_status_success) {
          HIPCHK(fill_zero_real<int>(w.flags, 1, st));
          HIPCHK(flag_nonfinite(nb, nb, w.Hs, nb, w.flags, st));
          HIPCHK(read_flags());
          if (ef[0] == 0 && (ef[1] != 0 || ef[2] != 0)) {
            HIPCHK((convert_copy<double, double>(nb, nb, Hc, nb, w.Hs, nb, st)));
            rs = rocsolver_zheev(p->rb, rocblas_evect_original, rocblas_fill_lower, nb, Hd, nb, ritz, w.E, w.flags + 3);
            if (rs == rocblas_status_success) {
              HIPCHK(fill_zero_real<int>(w.flags, 1, st));
              HIPCHK(flag_nonfinite(nb, nb, w.Hs, nb, w.flags, st));
              HIPCHK(read_flags());
            }
          }
        }
        if (rs == rocblas_status_success && ef[0] == 0)
          rs = rocblas_ztrsm(p->rb, rocblas_side_left, rocblas_fill_lower, rocblas_operation_conjugate_transpose,
                             rocblas_diagonal_non_unit, nb, nb, &one, Ld, nb, Hd, nb);
      }
      rocblas_set_workspace(p->rb, nullptr, 0);
      if (rs != rocblas_status_success)
        return fail(p, CHEB_ERR_HIP, std::string("dense eigensolver: ") + rocblas_status_to_string(rs));
      if (ef[0] != 0) return fail(p, CHEB_ERR_NOT_PD, "X^H S X is not positive definite (rank-deficient block)");
      if (ef[1] != 0) return fail(p, CHEB_ERR_EIG, "Hermitian eigensolver did not converge");
      if (ef[2] != 0) return fail(p, CHEB_ERR_EIG, "Hermitian eigensolver returned non-finite vectors");
      // Z = diag(d) Z' undoes the symmetric column scaling
      HIPCHK(scale_rows(nb, nb, w.Hs, nb, w.d, st));
    }
    C* Ynew = static_cast<C*>(w.Ynew);
    C* R = static_cast<C*>(w.R);
    const c128* t = w.Dp;
    {
      Timed tr(p, st, CHEB_T_RR_ROTATE, (resid ? 4.0 : 2.0) * npw * nb * sizeof(C) + nb * nb * 16.0,
               (resid ? 16.0 : 8.0) * npw * nb * nb);
      // FP64 MFMA in both precisions: for complex64 bands the products of complex64 values with the FP64
      // eigenvectors are summed in FP64 and rounded once, so an ill-conditioned block (the first iterations from a
      // random start) does not lose S-orthonormality to float32 cancellation in the sums
      Epi<T> er;
      er.out = Ynew; er.ldo = npw;
      HIPCHK((gemm<double, T, double, T>(GEMM_NN, p->npw, nb, nb, X, ldx, w.Hs, nb, er, 1, nullptr, st,
                                         ROLE_SUBSPACE)));
      if (resid) {
        // H u - lambda S u = loc Z + P (D pZ - lambda Q pZ) - lambda u
        Epi<T> e1;
        e1.out = R; e1.ldo = npw;
        HIPCHK((gemm<double, T, double, T>(GEMM_NN, p->npw, nb, nb, static_cast<C*>(w.loc), npw, w.Hs, nb, e1, 1,
                                           nullptr, st, ROLE_SUBSPACE)));
        if (hxout) HIPCHK((convert_copy<T, T>(npw, nb, R, npw, hxout, npw, st)));  // before P t is added
      } else if (hxout) {
        Epi<T> e1;
        e1.out = hxout; e1.ldo = npw;
        HIPCHK((gemm<double, T, double, T>(GEMM_NN, p->npw, nb, nb, static_cast<C*>(w.loc), npw, w.Hs, nb, e1, 1,
                                           nullptr, st, ROLE_SUBSPACE)));
      }
      if (resid) {
        if (np > 0) {
          Epi<double> ez;
          ez.out = w.q; ez.ldo = np;
          HIPCHK((gemm<double, double, double, double>(GEMM_NN, np, nb, nb, w.p0, np, w.Hs, nb, ez,
                                                       gemm_pick_splits(np, nb, nb), w.part, st)));
          HIPCHK(block_diag_apply(np, nb, p->pinfo, p->D, w.q, np, w.Dp, np, st));
          if (p->has_overlap) {
            HIPCHK(diag_apply(np, nb, p->Q, w.q, np, w.w, np, st));
            HIPCHK(sub_scaled_cols(np, nb, w.Dp, w.w, ritz, w.w, st));
            t = w.w;
          }
        }
      }
    }
    if (resid && np > 0) {  // the back-projection keeps its own timer, outside the rotation's
      Epi<T> e2;
      e2.out = R; e2.ldo = npw; e2.L = R; e2.ldl = npw; e2.bL = 1.0;
      CHK(backproject(t, nb, e2, w));
    }
    Timed tr(p, st, CHEB_T_RR_ROTATE, 0.0, 0.0, false);
    if (resid) HIPCHK((col_resid_norms<T>(npw, nb, R, npw, Ynew, npw, ritz, resid, st)));
    HIPCHK((convert_copy<T, T>(npw, nb, Ynew, npw, X, ldx, st)));
    if (pout && np > 0) {  // P^H (X Z) = (P^H X) Z, already formed for the residuals
      if (resid) {
        HIPCHK(hipMemcpyAsync(pout, w.q, size_t(np) * nb * sizeof(c128), hipMemcpyDeviceToDevice, st));
      } else {
        Epi<double> ez;
        ez.out = pout; ez.ldo = np;
        HIPCHK((gemm<double, double, double, double>(GEMM_NN, np, nb, nb, w.p0, np, w.Hs, nb, ez,
                                                     gemm_pick_splits(np, nb, nb), w.part, st)));
      }
    }
    return CHEB_OK;
  }

  // ---- LOBPCG (the block method the paper compares with, Sec. 2.3) ----------------------------------------
  // Caller-owned state: V = [X | W | P] (3 nb columns), H V, S V, then the full P, H P, S P and the new X,
  // H X, S X (nb columns each); every block has leading dimension npw.
  struct LobState { C *V, *HV, *SV, *Pf, *HPf, *SPf, *tX, *tHX, *tSX; };
  LobState lob_state(void* base, int nb) const {
    C* b = static_cast<C*>(base);
    const long k = long(p->npw) * nb;
    return {b, b + 3 * k, b + 6 * k, b + 9 * k, b + 10 * k, b + 11 * k, b + 12 * k, b + 13 * k, b + 14 * k};
  }

  // Rayleigh-Ritz of (V^H H V, V^H S V) over the first n columns, in an S-orthonormal basis of span(V) taken
  // from the eigendecomposition of the diagonally scaled Gram matrix, directions with eigenvalue below
  // trunc * largest dropped (SVQB basis). Lowest nb Ritz values to lamout (device), coefficients C with
  // V C = Ritz vectors to w.F (n x nb, ld n). Synchronizes. FP64 throughout.
  cheb_status svqb_rr(const C* V, const C* HV, const C* SV, int n, int nb, double trunc, double* lamout,
                      const Ws& w) {
    const long npw = p->npw;
    {
      Timed t(p, st, CHEB_T_RR_GRAM, 3.0 * npw * n * sizeof(C) + 2.0 * n * n * 16.0, 16.0 * npw * n * n);
      Epi<double> ea;
      ea.out = w.Hs; ea.ldo = n;
      HIPCHK((gemm<double, T, T, double>(GEMM_CN, n, n, p->npw, V, npw, HV, npw, ea, gemm_pick_splits(n, n, p->npw),
                                         w.part, st, ROLE_SUBSPACE)));
      Epi<double> eb;
      eb.out = w.Ss; eb.ldo = n;
      HIPCHK((gemm<double, T, T, double>(GEMM_CN, n, n, p->npw, V, npw, SV, npw, eb, gemm_pick_splits(n, n, p->npw),
                                         w.part, st, ROLE_SUBSPACE)));
    }
    Timed t(p, st, CHEB_T_RR_EIG, 0.0, 0.0);
    HIPCHK((fill_zero<float>(reinterpret_cast<c64*>(w.flags), 2, st)));
    HIPCHK(rr_prepare(n, w.Hs, w.Ss, w.d, w.flags, st));
    CHK(heev_checked(n, w.Ss, w.Xb, w.lam, w, "scaled Gram matrix"));
    std::vector<double> sig(n);
    int flags[3] = {0, 0, 0};
    HIPCHK(hipMemcpyAsync(flags, w.flags, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(sig.data(), w.lam, n * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (flags[1]) return fail(p, CHEB_ERR_NONFINITE, "non-finite entry in the LOBPCG Gram matrices");
    if (flags[0]) return fail(p, CHEB_ERR_NOT_PD, "zero or non-finite column in the LOBPCG basis");
    int r = 0;
    for (int i = 0; i < n; ++i) r += sig[i] > trunc * sig[n - 1];
    if (r < nb) return fail(p, CHEB_ERR_NOT_PD, "LOBPCG basis of rank below the block size");
    const int k0 = n - r;
    c128* Q = w.Ss + long(k0) * n;  // kept eigenvectors, scaled to an S'-orthonormal basis
    HIPCHK(scale_cols_isqrt(n, r, Q, n, w.lam + k0, st));
    Epi<double> e1;
    e1.out = w.Xa; e1.ldo = n;
    HIPCHK((gemm<double, double, double, double>(GEMM_NN, n, r, n, w.Hs, n, Q, n, e1, 1, nullptr, st)));
    Epi<double> e2;
    e2.out = w.Xb; e2.ldo = r;
    HIPCHK((gemm<double, double, double, double>(GEMM_CN, r, r, n, Q, n, w.Xa, n, e2, 1, nullptr, st)));
    {  // which of the basis, H' Q and the projected matrix carries a NaN or Inf, if any
      HIPCHK((fill_zero<float>(reinterpret_cast<c64*>(w.flags), 2, st)));
      HIPCHK(flag_nonfinite(n, r, Q, n, w.flags, st));
      HIPCHK(flag_nonfinite(n, r, w.Xa, n, w.flags + 1, st));
      HIPCHK(flag_nonfinite(r, r, w.Xb, r, w.flags + 2, st));
      int nf[3] = {0, 0, 0};
      HIPCHK(hipMemcpyAsync(nf, w.flags, 3 * sizeof(int), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      if (nf[0] || nf[1] || nf[2])
        return fail(p, CHEB_ERR_NONFINITE, "non-finite LOBPCG " + std::string(nf[0] ? "basis" : nf[1] ? "H' Q" : "projected matrix") +
                                               " (n = " + std::to_string(n) + ", r = " + std::to_string(r) + ")");
    }
    CHK(heev_checked(r, w.Xb, w.Xa, w.res, w, "projected matrix"));
    Epi<double> e3;
    e3.out = w.F; e3.ldo = n;
    HIPCHK((gemm<double, double, double, double>(GEMM_NN, n, nb, r, Q, n, w.Xb, r, e3, 1, nullptr, st)));
    HIPCHK(scale_rows(n, nb, w.F, n, w.d, st));  // coefficients of the unscaled V
    HIPCHK(hipMemcpyAsync(lamout, w.res, nb * sizeof(double), hipMemcpyDeviceToDevice, st));
    return CHEB_OK;
  }

  // Eigendecomposition of the Hermitian n x n matrix A (ld n, lower triangle used) in place, eigenvalues to lam
  // ascending: divide and conquer, and if that reports no convergence or returns non-finite vectors (seen with
  // info 0 on scaled Gram matrices whose leading block is the identity, where the tridiagonal splits into many
  // deflated pieces) the QR algorithm from a copy of A kept in spare (n x n). Synchronizes to read the status.
  cheb_status heev_checked(int n, c128* A, c128* spare, double* lam, const Ws& w, const char* what) {
    HIPCHK((convert_copy<double, double>(n, n, A, n, spare, n, st)));
    RBCHK(rocblas_set_stream(p->rb, st));
    RBCHK(rocblas_set_workspace(p->rb, w.solver, w.solver_bytes));
    rocblas_status rs = rocsolver_zheevd(p->rb, rocblas_evect_original, rocblas_fill_lower, n,
                                         reinterpret_cast<rocblas_double_complex*>(A), n, lam, w.E, w.flags + 2);
    rocblas_set_workspace(p->rb, nullptr, 0);
    if (rs != rocblas_status_success) return fail(p, CHEB_ERR_HIP, std::string("zheevd: ") + rocblas_status_to_string(rs));
    HIPCHK((fill_zero_real<int>(w.flags + 3, 1, st)));
    HIPCHK(flag_nonfinite(n, n, A, n, w.flags + 3, st));
    int info[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(info, w.flags + 2, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (info[0] == 0 && info[1] == 0) return CHEB_OK;
    HIPCHK((convert_copy<double, double>(n, n, spare, n, A, n, st)));
    RBCHK(rocblas_set_workspace(p->rb, w.solver, w.solver_bytes));
    rs = rocsolver_zheev(p->rb, rocblas_evect_original, rocblas_fill_lower, n, reinterpret_cast<rocblas_double_complex*>(A),
                         n, lam, w.E, w.flags + 2);
    rocblas_set_workspace(p->rb, nullptr, 0);
    if (rs != rocblas_status_success) return fail(p, CHEB_ERR_HIP, std::string("zheev: ") + rocblas_status_to_string(rs));
    HIPCHK((fill_zero_real<int>(w.flags + 3, 1, st)));
    HIPCHK(flag_nonfinite(n, n, A, n, w.flags + 3, st));
    HIPCHK(hipMemcpyAsync(info, w.flags + 2, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (info[0] != 0 || info[1] != 0)
      return fail(p, CHEB_ERR_EIG, std::string("Hermitian eigensolver failed on the LOBPCG ") + what + " (n = " +
                                       std::to_string(n) + ", info " + std::to_string(info[0]) +
                                       (info[1] ? ", non-finite vectors)" : ")"));
    return CHEB_OK;
  }

  // X <- V[:, :nb] Cx + P with P = V[:, nb:n] Cr (C = [Cx; Cr] in w.F), the same combinations of H V and S V;
  // the new P, H P, S P are kept in full (nb columns) for the next iteration.
  cheb_status lob_update(const LobState& s, int n, int nb, C* X, long ldx, const Ws& w) {
    const long npw = p->npw;
    Timed t(p, st, CHEB_T_RR_ROTATE, 6.0 * npw * nb * sizeof(C) + double(n) * nb * 16.0, 3.0 * 8.0 * npw * n * nb);
    const C* src[3] = {s.V, s.HV, s.SV};
    C* pf[3] = {s.Pf, s.HPf, s.SPf};
    C* tn[3] = {s.tX, s.tHX, s.tSX};
    for (int k = 0; k < 3; ++k) {
      Epi<T> e;
      e.out = tn[k]; e.ldo = npw;
      if (n > nb) {
        Epi<T> ep;
        ep.out = pf[k]; ep.ldo = npw;
        HIPCHK((gemm<T, T, double, T>(GEMM_NN, p->npw, nb, n - nb, src[k] + long(nb) * npw, npw, w.F + nb, n, ep, 1,
                                      nullptr, st, ROLE_SUBSPACE)));
        e.L = pf[k]; e.ldl = npw; e.bL = 1.0;
      } else {
        HIPCHK((fill_zero<T>(pf[k], npw * nb, st)));
      }
      HIPCHK((gemm<T, T, double, T>(GEMM_NN, p->npw, nb, nb, src[k], npw, w.F, n, e, 1, nullptr, st, ROLE_SUBSPACE)));
    }
    HIPCHK((convert_copy<T, T>(npw, nb, s.tX, npw, s.V, npw, st)));
    HIPCHK((convert_copy<T, T>(npw, nb, s.tHX, npw, s.HV, npw, st)));
    HIPCHK((convert_copy<T, T>(npw, nb, s.tSX, npw, s.SV, npw, st)));
    HIPCHK((convert_copy<T, T>(npw, nb, s.tX, npw, X, ldx, st)));
    return CHEB_OK;
  }

  // One LOBPCG iteration. it = 0: Rayleigh-Ritz of X alone (start). it = 1: space [X, W]. it >= 2: [X, W, P].
  // W are the preconditioned residuals of the bands whose residual exceeds tol, P their previous directions.
  cheb_status lobpcg(C* X, long ldx, int nb, int it, double tol, void* state, double* ritz, double* resid,
                     int* nactive, const Ws& w) {
    const long npw = p->npw;
    const LobState s = lob_state(state, nb);
    constexpr double trunc = 1e-14;
    if (it == 0) {
      HIPCHK((convert_copy<T, T>(npw, nb, X, ldx, s.V, npw, st)));
      CHK(apply_H(s.V, npw, s.HV, npw, nb, w));
      CHK(apply_S(s.V, npw, s.SV, npw, nb, w));
      CHK(svqb_rr(s.V, s.HV, s.SV, nb, nb, trunc, ritz, w));
      CHK(lob_update(s, nb, nb, X, ldx, w));
      if (nactive) *nactive = nb;
      return CHEB_OK;
    }
    // every kRestart iterations: H X and S X recomputed from X, and no directions this iteration (bounds the
    // drift of the carried products)
    constexpr int kRestart = 10;
    const bool restart = it > 1 && (it - 1) % kRestart == 0;
    if (restart) {
      CHK(apply_H(s.V, npw, s.HV, npw, nb, w));
      CHK(apply_S(s.V, npw, s.SV, npw, nb, w));
    }
    double* res = resid ? resid : w.d;
    HIPCHK((col_resid_norms<T>(npw, nb, s.HV, npw, s.SV, npw, ritz, res, st)));
    std::vector<double> hres(nb);
    HIPCHK(hipMemcpyAsync(hres.data(), res, nb * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    CHK(staging(p, size_t(nb)));
    int nact = 0;
    for (int i = 0; i < nb; ++i)
      if (!(hres[i] <= tol)) p->lock_host[nact++] = i;
    if (nactive) *nactive = nact;
    if (nact == 0) return CHEB_OK;
    HIPCHK(hipMemcpyAsync(w.lidx, p->lock_host, nact * sizeof(int), hipMemcpyHostToDevice, st));
    HIPCHK(hipEventRecord(p->lock_ev, st));
    C* Wc = s.V + long(nb) * npw;
    HIPCHK((lobpcg_precondition<T>(npw, nact, static_cast<const T*>(p->kin), s.V, s.HV, s.SV, npw, ritz, w.lidx, Wc,
                                   npw, st)));
    CHK(apply_H(Wc, npw, s.HV + long(nb) * npw, npw, nact, w));
    CHK(apply_S(Wc, npw, s.SV + long(nb) * npw, npw, nact, w));
    int n = nb + nact;
    if (it >= 2 && !restart) {
      HIPCHK((permute_cols<T>(npw, nact, s.Pf, npw, w.lidx, s.V + long(n) * npw, npw, nullptr, st)));
      HIPCHK((permute_cols<T>(npw, nact, s.HPf, npw, w.lidx, s.HV + long(n) * npw, npw, nullptr, st)));
      HIPCHK((permute_cols<T>(npw, nact, s.SPf, npw, w.lidx, s.SV + long(n) * npw, npw, nullptr, st)));
      n += nact;
    }
    cheb_status rs = svqb_rr(s.V, s.HV, s.SV, n, nb, trunc, ritz, w);
    if (rs != CHEB_OK && n > nb + nact) {
      // the space with the directions is numerically singular: restart from [X, W] this iteration
      n = nb + nact;
      rs = svqb_rr(s.V, s.HV, s.SV, n, nb, trunc, ritz, w);
    }
    if (rs != CHEB_OK) return rs;
    return lob_update(s, n, nb, X, ldx, w);
  }

  // out = (K + V) a for a block, and dV += coef n^-3 Re sum_b conj(a_b(r)) psi_b(r) from the same column pass
  cheb_status hloc_xdens(const C* a, long lda, const C* psi, long ldp, int nb, C* out, long ldo, double coef,
                         double* dV, const BwdWs& bw) {
    const int fb = fft_batch_for(p, nb);
    const FftGeom g = geom();
    const C* tw = static_cast<const C*>(p->tw);
    C* ca = static_cast<C*>(bw.fft.a);
    C* cb = static_cast<C*>(bw.fft.b);
    C* cc = static_cast<C*>(bw.colc);
    const double b = sizeof(C), colv = double(p->n) * p->ncol, npw = p->npw;
    if (p->n > 64) {  // balancing scales of the polarisation form of the cross density
      HIPCHK((col_dots<T>(p->npw, nb, a, lda, a, lda, bw.bdots, st)));
      HIPCHK((col_dots<T>(p->npw, nb, psi, ldp, psi, ldp, bw.bdots + nb, st)));
      HIPCHK(balance_scales(nb, bw.bdots, bw.bdots + nb, bw.bal, st));
    }
    for (int b0 = 0; b0 < nb; b0 += fb) {
      const int cnt = std::min(fb, nb - b0);
      {
        Timed t(p, st, CHEB_T_FFT_COL_INV, 2.0 * cnt * (npw + colv) * b, 0.0);
        HIPCHK(fft_col_inverse<T>(g, tw, a + long(b0) * lda, lda, cnt, ca, st));
        HIPCHK(fft_col_inverse<T>(g, tw, psi + long(b0) * ldp, ldp, cnt, cc, st));
      }
      {
        Timed t(p, st, CHEB_T_FFT_PLANE, cnt * 2.0 * colv * b, cnt * plane_flops());
        HIPCHK(fft_plane<T>(g, tw, static_cast<const T*>(p->Vt), ca, cb, cnt, st));
      }
      {
        Timed t(p, st, CHEB_T_FFT_COL_FWD, cnt * (colv + 2.0 * npw) * b, 0.0);
        HIPCHK(fft_col_forward<T>(g, tw, cb, a + long(b0) * lda, lda, static_cast<const T*>(p->kin),
                                  out + long(b0) * ldo, ldo, cnt, st));
      }
      {
        Timed t(p, st, CHEB_T_XDENS, cnt * 2.0 * colv * b, 0.0);
        HIPCHK(cross_density<T>(g, tw, ca, cc, cnt, nullptr, bw.bal + b0, coef, bw.xpart, dV, st));
      }
    }
    return CHEB_OK;
  }

  // dV += n^-3 sum_i w_i |u_i(r)|^2 over the first nk bands of U (Hellmann-Feynman term)
  cheb_status density(const C* U, long ldu, int nk, const double* wts, double* dV, const BwdWs& bw) {
    const int fb = fft_batch_for(p, nk);
    const FftGeom g = geom();
    const C* tw = static_cast<const C*>(p->tw);
    C* ca = static_cast<C*>(bw.fft.a);
    for (int b0 = 0; b0 < nk; b0 += fb) {
      const int cnt = std::min(fb, nk - b0);
      HIPCHK(fft_col_inverse<T>(g, tw, U + long(b0) * ldu, ldu, cnt, ca, st));
      Timed t(p, st, CHEB_T_XDENS, cnt * double(p->n) * p->ncol * sizeof(C), 0.0);
      HIPCHK(cross_density<T>(g, tw, ca, ca, cnt, wts + b0, nullptr, 1.0, bw.xpart, dV, st));
    }
    return CHEB_OK;
  }

  // Filter + Rayleigh-Ritz forward, then the adjoint of L = sum_{i<nk} w_i lambda_i with c, r fixed.
  cheb_status backward(const C* X0, long ldx, int nb, int m, double c, double r, int nk, const double* wts, int k,
                       double* ritz, C* dX, long lddx, double* dV, double* dD, const BwdWs& bw) {
    const int np = p->nproj;
    const long npw = p->npw;
    const long nv = long(p->n) * p->n * p->n;
    HIPCHK(fill_zero_real<double>(dV, nv, st));
    if (dD && p->dsize) HIPCHK(fill_zero_real<double>(dD, long(p->dsize), st));
    C* F[2] = {static_cast<C*>(bw.F[0]), static_cast<C*>(bw.F[1])};
    const int ncp = (m + k - 1) / k;
    // ---- forward with checkpoints (psi^(t-1), psi^t) at t = 0, k, 2k, ...
    HIPCHK((convert_copy<T, T>(npw, nb, X0, ldx, F[0], npw, st)));
    if (np > 0) CHK(project(F[0], npw, nb, bw.pf[0], bw.fw));
    for (int i = 1; i <= m; ++i) {
      const int ci = (i - 1) & 1, oi = i & 1;
      CHK(resync_step(i, F[ci], npw, bw.pf[ci], F[oi], npw, bw.pf[oi], nb, bw.fw));
      if ((i - 1) % k == 0) {
        const int j = (i - 1) / k;
        HIPCHK((convert_copy<T, T>(npw, nb, F[ci], npw, static_cast<C*>(bw.ck[2 * j + 1]), npw, st)));
        if (np > 0) HIPCHK((convert_copy<double, double>(np, nb, bw.pf[ci], np, bw.ckp[2 * j + 1], np, st)));
        if (i >= 2) {
          HIPCHK((convert_copy<T, T>(npw, nb, F[oi], npw, static_cast<C*>(bw.ck[2 * j]), npw, st)));
          if (np > 0) HIPCHK((convert_copy<double, double>(np, nb, bw.pf[oi], np, bw.ckp[2 * j], np, st)));
        }
      }
      CHK(filter_step(i, F[ci], npw, F[oi], npw, F[oi], npw, bw.pf[ci], bw.pf[oi], bw.pf[oi], nb, c, r, bw.fw));
    }
    C* Y = F[m & 1];
    // ---- Rayleigh-Ritz with residual vectors: U = Y Z, R = H U - S U Lambda
    CHK(rayleigh_ritz(Y, npw, nb, ritz, bw.norms, bw.rr));
    C* R = static_cast<C*>(bw.rr.R);
    const C* U = static_cast<const C*>(bw.rr.Ynew);
    HIPCHK(sub_lambda_cols<T>(npw, nk, R, npw, U, npw, ritz, st));
    // Hellmann-Feynman terms at fixed Y
    CHK(density(U, npw, nk, wts, dV, bw));
    if (np > 0 && dD) HIPCHK(block_grad(int(p->dsize), p->dent, nk, bw.rr.q, np, bw.rr.q, np, wts, 0.5, dD, st));
    // Ybar = R_K W Z_K^H
    C* bar[3] = {static_cast<C*>(bw.bar[0]), static_cast<C*>(bw.bar[1]), static_cast<C*>(bw.bar[2])};
    HIPCHK(weighted_adjoint(nk, nb, wts, bw.rr.Hs, nb, bw.B, st));
    {
      Epi<T> e;
      e.out = bar[m % 3]; e.ldo = npw;
      HIPCHK((gemm<T, T, double, T>(GEMM_NN, p->npw, nb, nk, R, npw, bw.B, nk, e, 1, nullptr, st, ROLE_SUBSPACE)));
    }
    HIPCHK((fill_zero<T>(bar[(m - 1) % 3], npw * nb, st)));
    // ---- reverse sweep over segments, recomputing psi^(t0) .. psi^(t1-1) from each checkpoint
    std::vector<C*> seg(k);
    std::vector<c128*> segp(k);
    for (int sgm = ncp - 1; sgm >= 0; --sgm) {
      const int t0 = sgm * k, t1 = std::min(m, t0 + k);
      seg[0] = static_cast<C*>(bw.ck[2 * sgm + 1]);
      segp[0] = bw.ckp[2 * sgm + 1];
      for (int j = t0 + 1; j < t1; ++j) {
        const int idx = j - t0;
        seg[idx] = static_cast<C*>(bw.seg[idx - 1]);
        segp[idx] = bw.segp[idx - 1];
        const C* prv = idx >= 2 ? seg[idx - 2] : static_cast<const C*>(bw.ck[2 * sgm]);
        c128* pprv = idx >= 2 ? segp[idx - 2] : bw.ckp[2 * sgm];
        // the same resynchronisation as the forward pass, so that the segment is recomputed exactly
        CHK(resync_step(j, seg[idx - 1], npw, segp[idx - 1], prv, npw, pprv, nb, bw.fw));
        CHK(filter_step(j, seg[idx - 1], npw, prv, npw, seg[idx], npw, segp[idx - 1], pprv, segp[idx], nb, c, r, bw.fw));
      }
      for (int i = t1; i >= t0 + 1; --i) {
        const C* psim1 = seg[i - 1 - t0];
        const c128* pm1 = segp[i - 1 - t0];
        CHK(adjoint_step(i, bar[i % 3], bar[(i - 1) % 3], i >= 2 ? bar[(i - 2) % 3] : nullptr, psim1, pm1, nb, c, r,
                         dV, dD, bw));
      }
    }
    HIPCHK((convert_copy<T, T>(npw, nb, bar[0], npw, dX, lddx, st)));
    return CHEB_OK;
  }

  // psibar^(i-1) += s (H a - c psibar^i), psibar^(i-2) = -psibar^i, a = S^-1 psibar^i; gradient terms of step i
  cheb_status adjoint_step(int i, C* Bi, C* Bm1, C* Bm2, const C* psim1, const c128* pm1, int nb, double c, double r,
                           double* dV, double* dD, const BwdWs& bw) {
    const int np = p->nproj;
    const long npw = p->npw;
    const double si = (i == 1 ? 1.0 : 2.0) / r;
    const Ws& w = bw.fw;
    const C* a = Bi;
    const c128* pa = bw.pbar;
    if (np > 0) {
      CHK(project(Bi, npw, nb, bw.pbar, w));
      if (p->has_overlap) {
        CHK(cinv(bw.pbar, np, nb, bw.qa, np, w));
        Epi<T> ea;
        ea.out = static_cast<C*>(bw.a); ea.ldo = npw; ea.alpha = -1.0;
        ea.L = Bi; ea.ldl = npw; ea.bL = 1.0;
        CHK(backproject(bw.qa, nb, ea, w));
        a = static_cast<const C*>(bw.a);
        Epi<double> ep;
        ep.out = bw.pa; ep.ldo = np; ep.alpha = -1.0;
        ep.L = bw.pbar; ep.ldl = np; ep.bL = 1.0;
        CHK(small(p->G, bw.qa, nb, ep, w.part));
        pa = bw.pa;
      }
    }
    C* loca = static_cast<C*>(bw.loca);
    CHK(hloc_xdens(a, npw, psim1, npw, nb, loca, npw, 2.0 * si, dV, bw));
    if (np > 0) {
      HIPCHK(block_diag_apply(np, nb, p->pinfo, p->D, pa, np, bw.Dpa, np, st));
      Epi<T> e;
      e.out = Bm1; e.ldo = npw; e.alpha = si;
      e.L = loca; e.ldl = npw; e.bL = si;
      e.U = Bi; e.ldu = npw; e.bU = -si * c;
      e.W = Bm1; e.ldw = npw; e.bW = 1.0;
      CHK(backproject(bw.Dpa, nb, e, w));
      if (dD) HIPCHK(block_grad(int(p->dsize), p->dent, nb, pa, np, pm1, np, nullptr, si, dD, st));
    } else {
      HIPCHK((axpbypcz<T>(npw, nb, si, loca, npw, -si * c, Bi, npw, 1.0, Bm1, npw, Bm1, npw, st)));
    }
    if (Bm2) HIPCHK((axpbypcz<T>(npw, nb, -1.0, Bi, npw, 0.0, nullptr, 0, 0.0, nullptr, 0, Bm2, npw, st)));
    return CHEB_OK;
  }

  cheb_status rayleigh_quotients(const C* X, long ldx, int nb, double* rq, const Ws& w) {
    // reuse the RR workspace: loc <- H X, R <- S X
    C* HX = static_cast<C*>(w.loc);
    C* SX = static_cast<C*>(w.R);
    const long npw = p->npw;
    CHK(apply_H(X, ldx, HX, npw, nb, w));
    CHK(apply_S(X, ldx, SX, npw, nb, w));
    HIPCHK((col_dots<T>(npw, nb, X, ldx, HX, npw, w.dots, st)));
    HIPCHK((col_dots<T>(npw, nb, X, ldx, SX, npw, w.dots2, st)));
    HIPCHK(ratio_real(nb, w.dots, w.dots2, rq, st));
    return CHEB_OK;
  }

  cheb_status dot_host(const C* x, const C* y, const Ws& w, double* re) {
    HIPCHK((col_dots<T>(p->npw, 1, x, p->npw, y, p->npw, w.dots, st)));
    c128 h;
    HIPCHK(hipMemcpyAsync(&h, w.dots, sizeof(c128), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    *re = h.x;
    return CHEB_OK;
  }

  cheb_status upper_bound(int k, const C* v0, double* out, const Ws& w) {
    const long npw = p->npw;
    C* v = static_cast<C*>(w.v);
    C* vp = static_cast<C*>(w.vp);
    C* f = static_cast<C*>(w.f);
    C* Hv = static_cast<C*>(w.Hv);
    C* Sf = static_cast<C*>(w.Sf);
    CHK(apply_S(v0, npw, Sf, npw, 1, w));
    double nrm2 = 0.0;
    CHK(dot_host(v0, Sf, w, &nrm2));
    if (!(nrm2 > 0.0) || !std::isfinite(nrm2)) return fail(p, CHEB_ERR_ARG, "v0 has zero or non-finite S-norm");
    HIPCHK((axpbypcz<T>(npw, 1, 1.0 / std::sqrt(nrm2), v0, npw, 0.0, nullptr, 0, 0.0, nullptr, 0, v, npw, st)));
    HIPCHK((fill_zero<T>(vp, npw, st)));
    std::vector<double> alpha, beta;
    double b = 0.0;
    for (int j = 0; j < k; ++j) {
      CHK(apply_H(v, npw, Hv, npw, 1, w));
      CHK(apply_Sinv(Hv, npw, f, npw, 1, w));
      double a = 0.0;
      CHK(dot_host(v, Hv, w, &a));
      HIPCHK((axpbypcz<T>(npw, 1, 1.0, f, npw, -a, v, npw, -b, vp, npw, f, npw, st)));
      CHK(apply_S(f, npw, Sf, npw, 1, w));
      double bb = 0.0;
      CHK(dot_host(f, Sf, w, &bb));
      b = std::sqrt(std::max(bb, 0.0));
      alpha.push_back(a);
      beta.push_back(b);
      if (!(b > 0.0)) break;  // invariant subspace found: T is exact
      std::swap(v, vp);       // vp <- old v
      HIPCHK((axpbypcz<T>(npw, 1, 1.0 / b, f, npw, 0.0, nullptr, 0, 0.0, nullptr, 0, v, npw, st)));
    }
    // largest eigenvalue of the symmetric tridiagonal T (alpha, beta[0..k-2]) by Sturm-count bisection
    const int kk = int(alpha.size());
    double lo = 1e300, hi = -1e300;
    for (int i = 0; i < kk; ++i) {
      const double rad = (i > 0 ? std::fabs(beta[i - 1]) : 0.0) + (i + 1 < kk ? std::fabs(beta[i]) : 0.0);
      lo = std::min(lo, alpha[i] - rad);
      hi = std::max(hi, alpha[i] + rad);
    }
    auto count_below = [&](double x) {  // eigenvalues < x
      int cnt = 0;
      double d = 1.0;
      for (int i = 0; i < kk; ++i) {
        const double off = i > 0 ? beta[i - 1] * beta[i - 1] : 0.0;
        d = alpha[i] - x - (i > 0 ? off / d : 0.0);
        if (d == 0.0) d = -1e-300;
        if (d < 0.0) ++cnt;
      }
      return cnt;
    };
    for (int it = 0; it < 200 && hi - lo > 1e-15 * std::max(1.0, std::fabs(hi)); ++it) {
      const double mid = 0.5 * (lo + hi);
      if (count_below(mid) >= kk) hi = mid; else lo = mid;
    }
    *out = hi + beta.back();
    return CHEB_OK;
  }
};

template <typename F> cheb_status with_prec(cheb_plan p, hipStream_t st, F&& f) {
  if (p->prec == CHEB_MIXED) return f(Ops<float>{p, st});
  return f(Ops<double>{p, st});
}

}  // namespace

// ======================================= C ABI ==================================================================
extern "C" {

// The sphere of the FFTs for a Gamma plan: the half sphere plus the mirror -G of every G != 0, in the sorted
// column order; gmap / pair / h0 as kept in the plan.
struct FullSphere {
  std::vector<int32_t> g;
  std::vector<int> gmap;
  std::vector<int2> pair;
  int h0 = -1;
};

static cheb_status build_full_sphere(const cheb_desc* d, FullSphere* fs, std::string* msg) {
  struct Ent { int gx, gy, gz, h, cj; };
  const int nh = d->npw;
  std::vector<Ent> v;
  v.reserve(2 * size_t(nh));
  fs->h0 = -1;
  for (int h = 0; h < nh; ++h) {
    const int32_t* g = d->gidx_host + 3 * h;
    const bool in_half = g[0] > 0 || (g[0] == 0 && g[1] > 0) || (g[0] == 0 && g[1] == 0 && g[2] >= 0);
    if (!in_half) { *msg = "Gamma plan: entry " + std::to_string(h) + " is not in the half sphere"; return CHEB_ERR_ARG; }
    if (h > 0) {
      const int32_t* q = g - 3;
      if (!(q[0] < g[0] || (q[0] == g[0] && (q[1] < g[1] || (q[1] == g[1] && q[2] < g[2]))))) {
        *msg = "Gamma plan: half-sphere list not strictly increasing at entry " + std::to_string(h);
        return CHEB_ERR_ARG;
      }
    }
    v.push_back({g[0], g[1], g[2], h, 0});
    if (g[0] == 0 && g[1] == 0 && g[2] == 0) fs->h0 = h;
    else v.push_back({-g[0], -g[1], -g[2], h, 1});
  }
  std::sort(v.begin(), v.end(), [](const Ent& a, const Ent& b) {
    return a.gx != b.gx ? a.gx < b.gx : (a.gy != b.gy ? a.gy < b.gy : a.gz < b.gz);
  });
  fs->g.resize(3 * v.size());
  fs->gmap.resize(v.size());
  fs->pair.assign(nh, int2{-1, -1});
  for (size_t e = 0; e < v.size(); ++e) {
    fs->g[3 * e] = v[e].gx; fs->g[3 * e + 1] = v[e].gy; fs->g[3 * e + 2] = v[e].gz;
    fs->gmap[e] = v[e].h | (v[e].cj << 30);
    if (v[e].cj) fs->pair[v[e].h].y = int(e);
    else fs->pair[v[e].h].x = int(e);
  }
  if (fs->h0 >= 0) fs->pair[fs->h0].y = fs->pair[fs->h0].x;
  return CHEB_OK;
}

// Checks the descriptor; ncol, rx from the sphere of the FFTs (the whole sphere of a Gamma plan, built into fs).
static cheb_status validate_desc(const cheb_desc* d, int* ncol_out, int* rx_out, size_t* dsize_out,
                                 std::string* msg, FullSphere* fs) {
  if (!d) { *msg = "desc is null"; return CHEB_ERR_ARG; }
  if (!supported_n(d->n)) { *msg = "unsupported FFT box size " + std::to_string(d->n); return CHEB_ERR_ARG; }
  if (d->npw <= 0) { *msg = "npw must be positive"; return CHEB_ERR_ARG; }
  if (!d->gidx_host || !d->kin_host) { *msg = "gidx_host / kin_host is null"; return CHEB_ERR_ARG; }
  if (d->prec != CHEB_FP64 && d->prec != CHEB_MIXED) { *msg = "unknown precision"; return CHEB_ERR_ARG; }
  if (d->gamma != 0 && d->gamma != 1) { *msg = "gamma must be 0 or 1"; return CHEB_ERR_ARG; }
  if (d->natom < 0 || (d->natom > 0 && !d->proj_off_host)) { *msg = "bad natom / proj_off_host"; return CHEB_ERR_ARG; }
  for (int e = 0; e < d->npw; ++e)
    if (!std::isfinite(d->kin_host[e])) { *msg = "non-finite kinetic entry"; return CHEB_ERR_ARG; }
  const int32_t* G = d->gidx_host;
  int npf = d->npw;
  if (d->gamma) {
    CHK(build_full_sphere(d, fs, msg));
    G = fs->g.data();
    npf = int(fs->gmap.size());
  }
  const int hmax = (d->n - 1) / 2;
  int ncol = 0, rx = 0;
  for (int e = 0; e < npf; ++e) {
    const int32_t* g = G + 3 * e;
    for (int c = 0; c < 3; ++c)
      if (g[c] < -hmax || g[c] > hmax) { *msg = "Miller index outside the FFT box at entry " + std::to_string(e); return CHEB_ERR_ARG; }
    rx = std::max(rx, std::abs(g[0]));
    if (e == 0) { ncol = 1; continue; }
    const int32_t* h = g - 3;
    if (g[0] == h[0] && g[1] == h[1]) {
      if (g[2] != h[2] + 1) { *msg = "g-list column not a run of consecutive gz at entry " + std::to_string(e); return CHEB_ERR_ARG; }
    } else {
      if (g[0] < h[0] || (g[0] == h[0] && g[1] < h[1])) { *msg = "g-list not sorted by column (gx, gy) at entry " + std::to_string(e); return CHEB_ERR_ARG; }
      if (g[0] == h[0] && g[1] != h[1] + 1) { *msg = "columns of one gx not a run of consecutive gy at entry " + std::to_string(e); return CHEB_ERR_ARG; }
      ++ncol;
    }
  }
  if (ncol >= (1 << 22)) { *msg = "too many columns"; return CHEB_ERR_ARG; }
  if (fft_plane_lds_bytes(d->n, rx, d->prec != CHEB_MIXED) > 160 * 1024) {
    *msg = "sphere too wide in x for the plane pass in 160 KB of LDS";
    return CHEB_ERR_ARG;
  }
  size_t dsize = 0;
  if (d->natom > 0) {
    if (d->proj_off_host[0] != 0) { *msg = "proj_off[0] must be 0"; return CHEB_ERR_ARG; }
    for (int a = 0; a < d->natom; ++a) {
      const int na = d->proj_off_host[a + 1] - d->proj_off_host[a];
      if (na < 0) { *msg = "proj_off must be nondecreasing"; return CHEB_ERR_ARG; }
      dsize += size_t(na) * na;
    }
  }
  *ncol_out = ncol;
  *rx_out = rx;
  *dsize_out = dsize;
  return CHEB_OK;
}

cheb_status cheb_plan_persistent_bytes(const cheb_desc* d, size_t* bytes) try {
  if (!bytes) return CHEB_ERR_ARG;
  int ncol = 0, rx = 0;
  size_t dsize = 0;
  std::string msg;
  FullSphere fs;
  cheb_status s = validate_desc(d, &ncol, &rx, &dsize, &msg, &fs);
  if (s != CHEB_OK) return s;
  const int nproj = d->natom > 0 ? d->proj_off_host[d->natom] : 0;
  const int npf = d->gamma ? int(fs.gmap.size()) : d->npw;
  *bytes = persist_bytes(d->n, d->npw, npf, ncol, rx, nproj, dsize, d->has_overlap ? 1 : 0, d->prec, d->gamma);
  return CHEB_OK;
} catch (...) {
  return host_fail(nullptr);
}

cheb_status cheb_plan_create(const cheb_desc* d, void* persistent, size_t bytes, hipStream_t st, cheb_plan* out) try {
  if (!out) return CHEB_ERR_ARG;
  *out = nullptr;
  int ncol = 0, rx = 0;
  size_t dsize = 0;
  std::string msg;
  FullSphere fs;
  cheb_status s = validate_desc(d, &ncol, &rx, &dsize, &msg, &fs);
  if (s != CHEB_OK) { std::fprintf(stderr, "cheb_plan_create: %s\n", msg.c_str()); return s; }
  const int nproj = d->natom > 0 ? d->proj_off_host[d->natom] : 0;
  const int npf = d->gamma ? int(fs.gmap.size()) : d->npw;
  const int32_t* G = d->gamma ? fs.g.data() : d->gidx_host;  // the sphere of the FFTs
  const size_t need = persist_bytes(d->n, d->npw, npf, ncol, rx, nproj, dsize, d->has_overlap ? 1 : 0, d->prec,
                                    d->gamma);
  if (!persistent || bytes < need || reinterpret_cast<uintptr_t>(persistent) % kAlign) return CHEB_ERR_WORKSPACE;

  std::unique_ptr<cheb_plan_s> owner(new cheb_plan_s);  // handed to the caller only on success
  cheb_plan p = owner.get();
  p->n = d->n; p->npw = d->npw; p->ncol = ncol; p->rx = rx; p->natom = d->natom; p->nproj = nproj;
  p->has_overlap = d->has_overlap ? 1 : 0; p->prec = d->prec; p->dsize = dsize;
  p->gamma = d->gamma; p->npf = npf; p->h0 = fs.h0;
  p->resync = d->prec == CHEB_MIXED ? kMixedResync : 0;
  p->proj_off.assign(d->proj_off_host, d->proj_off_host + (d->natom > 0 ? d->natom + 1 : 0));
  Persist l = persist_layout(persistent, d->n, d->npw, npf, ncol, rx, nproj, dsize, p->has_overlap, d->prec, d->gamma);
  p->gmap = l.gmap; p->gpair = l.gpair;
  p->col = l.col; p->ent = l.ent; p->xline = l.xline; p->pinfo = l.pinfo; p->dent = l.dent; p->tw = l.tw; p->kin = l.kin; p->Vt = l.Vt; p->P = l.P;
  p->D = l.D; p->Q = l.Q; p->G = l.G; p->Cinv = l.Cinv; p->Cmat = l.Cmat; p->Minv = l.Minv;
  p->hproj.p = l.Hproj; p->hproj.rows = nproj; p->hproj.ld = pad32(d->npw);
  p->hback.p = l.Hback; p->hback.rows = d->npw; p->hback.ld = pad32(nproj);

  // host-side index maps
  std::vector<int4> col(ncol);
  std::vector<int> ent(npf);
  int c = -1;
  for (int e = 0; e < npf; ++e) {
    const int32_t* g = G + 3 * e;
    if (e == 0 || g[0] != g[-3] || g[1] != g[-2]) {
      ++c;
      col[c] = int4{g[0] + rx, (g[1] % d->n + d->n) % d->n, e, 0};
    }
    col[c].w += 1;
    ent[e] = (c << 8) | ((g[2] % d->n + d->n) % d->n);
  }
  // x-lines: columns sharing gx are consecutive (sorted by gy, consecutive gy checked above)
  std::vector<int4> xline(2 * rx + 1, int4{0, 0, 0, 0});
  for (int cc = 0; cc < ncol; ++cc) {
    const int32_t* g0 = G + 3 * col[cc].z;
    int4& xl = xline[g0[0] + rx];
    if (xl.z == 0) { xl.x = cc; xl.y = g0[1]; }
    xl.z += 1;
  }
  std::vector<int4> pinfo(std::max(nproj, 1), int4{0, 0, 0, 0});
  size_t doff = 0;
  std::vector<int2> dent(std::max<size_t>(dsize, 1), int2{0, 0});
  for (int a = 0; a < d->natom; ++a) {
    const int o = d->proj_off_host[a], na = d->proj_off_host[a + 1] - o;
    for (int i = 0; i < na; ++i) pinfo[o + i] = int4{o, na, int(doff), 0};
    for (int i = 0; i < na; ++i)
      for (int j = 0; j < na; ++j) dent[doff + size_t(i) * na + j] = int2{o + i, o + j};
    doff += size_t(na) * na;
  }
  const bool mixed = d->prec == CHEB_MIXED;
  std::vector<c128> tw(d->n);
  for (int j = 0; j < d->n; ++j) {
    const double a = -2.0 * M_PI * double(j) / double(d->n);
    tw[j] = c128{std::cos(a), std::sin(a)};
  }
  auto fail_hip = [&](hipError_t e, const char* what) {
    std::fprintf(stderr, "cheb_plan_create: %s: %s\n", what, hipGetErrorString(e));
    return CHEB_ERR_HIP;
  };
  // every host table exists before the first copy is issued, so that nothing thrown later frees a source
  // buffer under a copy in flight
  std::vector<c64> tw32(mixed ? d->n : 0);
  std::vector<float> kin32(mixed ? d->npw : 0);
  hipError_t e;
  if ((e = hipMemcpyAsync(p->col, col.data(), sizeof(int4) * ncol, hipMemcpyHostToDevice, st))) return fail_hip(e, "col");
  if ((e = hipMemcpyAsync(p->ent, ent.data(), sizeof(int) * npf, hipMemcpyHostToDevice, st))) return fail_hip(e, "ent");
  if (d->gamma) {
    if ((e = hipMemcpyAsync(p->gmap, fs.gmap.data(), sizeof(int) * npf, hipMemcpyHostToDevice, st))) return fail_hip(e, "gmap");
    if ((e = hipMemcpyAsync(p->gpair, fs.pair.data(), sizeof(int2) * d->npw, hipMemcpyHostToDevice, st))) return fail_hip(e, "gpair");
  }
  if ((e = hipMemcpyAsync(p->xline, xline.data(), sizeof(int4) * xline.size(), hipMemcpyHostToDevice, st))) return fail_hip(e, "xline");
  if ((e = hipMemcpyAsync(p->pinfo, pinfo.data(), sizeof(int4) * pinfo.size(), hipMemcpyHostToDevice, st))) return fail_hip(e, "pinfo");
  if ((e = hipMemcpyAsync(p->dent, dent.data(), sizeof(int2) * dent.size(), hipMemcpyHostToDevice, st))) return fail_hip(e, "dent");
  if (mixed) {
    for (int j = 0; j < d->n; ++j) tw32[j] = c64{float(tw[j].x), float(tw[j].y)};
    for (int i = 0; i < d->npw; ++i) kin32[i] = float(d->kin_host[i]);
    if ((e = hipMemcpyAsync(p->tw, tw32.data(), sizeof(c64) * d->n, hipMemcpyHostToDevice, st))) return fail_hip(e, "tw");
    if ((e = hipMemcpyAsync(p->kin, kin32.data(), sizeof(float) * d->npw, hipMemcpyHostToDevice, st))) return fail_hip(e, "kin");
    if ((e = hipStreamSynchronize(st))) return fail_hip(e, "sync");
  } else {
    if ((e = hipMemcpyAsync(p->tw, tw.data(), sizeof(c128) * d->n, hipMemcpyHostToDevice, st))) return fail_hip(e, "tw");
    if ((e = hipMemcpyAsync(p->kin, d->kin_host, sizeof(double) * d->npw, hipMemcpyHostToDevice, st))) return fail_hip(e, "kin");
    if ((e = hipStreamSynchronize(st))) return fail_hip(e, "sync");
  }
  if ((e = fft_prepare_attributes())) return fail_hip(e, "kernel attributes");
  if (rocblas_create_handle(&p->rb) != rocblas_status_success) {
    std::fprintf(stderr, "cheb_plan_create: rocblas_create_handle failed\n");
    return CHEB_ERR_HIP;
  }
  if ((e = hipGetDevice(&p->device))) return fail_hip(e, "hipGetDevice");
  // the static scratch of cheb_apply_H_noalloc on this device (a failure only disables that entry point)
  p->scratch = resolve_scratch(p->device, &e);
  *out = owner.release();
  return CHEB_OK;
} catch (...) {
  return host_fail(nullptr);
}

cheb_status cheb_plan_destroy(cheb_plan p) try {
  if (!p) return CHEB_OK;
  for (auto& r : p->prof_pending) { (void)hipEventSynchronize(r.b); (void)hipEventDestroy(r.a); (void)hipEventDestroy(r.b); }
  for (auto& r : p->prof_free) { (void)hipEventDestroy(r.first); (void)hipEventDestroy(r.second); }
  if (p->rb) rocblas_destroy_handle(p->rb);
  if (p->lock_ev) { (void)hipEventSynchronize(p->lock_ev); (void)hipEventDestroy(p->lock_ev); }
  if (p->lock_host) (void)hipHostFree(p->lock_host);
  for (hipEvent_t& ev : p->rr_ev)
    if (ev) { (void)hipEventSynchronize(ev); (void)hipEventDestroy(ev); }
  if (p->rr_host) (void)hipHostFree(p->rr_host);
  delete p;
  return CHEB_OK;
} catch (...) {
  return host_fail(nullptr);  // the plan may already be released
}

const char* cheb_last_error(cheb_plan p) { return p ? p->err.c_str() : "null plan"; }

static cheb_status prof_collect(cheb_plan p) {
  for (auto& r : p->prof_pending) {
    HIPCHK(hipEventSynchronize(r.b));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, r.a, r.b));
    p->prof_ms[r.kind] += ms;
    p->prof_free.push_back({r.a, r.b});
  }
  p->prof_pending.clear();
  return CHEB_OK;
}

cheb_status cheb_profile_enable(cheb_plan p, int on) try {
  if (!p) return CHEB_ERR_ARG;
  CHK(prof_collect(p));
  if (on) {
    for (int k = 0; k < CHEB_T_COUNT; ++k) { p->prof_ms[k] = 0; p->prof_bytes[k] = 0; p->prof_flops[k] = 0; p->prof_n[k] = 0; }
  }
  p->prof_on = on != 0;
  return CHEB_OK;
} catch (...) {
  return host_fail(p);
}

cheb_status cheb_profile_read(cheb_plan p, int timer, double* ms, int64_t* launches, double* bytes, double* flops) try {
  if (!p) return CHEB_ERR_ARG;
  if (timer < 0 || timer >= CHEB_T_COUNT) return fail(p, CHEB_ERR_ARG, "unknown timer");
  CHK(prof_collect(p));
  if (ms) *ms = p->prof_ms[timer];
  if (launches) *launches = p->prof_n[timer];
  if (bytes) *bytes = p->prof_bytes[timer];
  if (flops) *flops = p->prof_flops[timer];
  return CHEB_OK;
} catch (...) {
  return host_fail(p);
}

cheb_status cheb_set_potential(cheb_plan p, const double* V, hipStream_t st) try {
  if (!p) return CHEB_ERR_ARG;
  if (!V) return fail(p, CHEB_ERR_ARG, "V is null");
  if (p->prec == CHEB_MIXED) HIPCHK(transpose_potential<float>(p->n, V, static_cast<float*>(p->Vt), st));
  else HIPCHK(transpose_potential<double>(p->n, V, static_cast<double*>(p->Vt), st));
  p->have_V = true;
  return CHEB_OK;
} catch (...) {
  return host_fail(p);
}

cheb_status cheb_set_D(cheb_plan p, const double* D, hipStream_t st) try {
  if (!p) return CHEB_ERR_ARG;
  if (p->dsize == 0) { p->have_D = true; return CHEB_OK; }
  if (!D) return fail(p, CHEB_ERR_ARG, "D is null");
  HIPCHK(hipMemcpyAsync(p->D, D, sizeof(double) * p->dsize, hipMemcpyDeviceToDevice, st));
  p->have_D = true;
  return CHEB_OK;
} catch (...) {
  return host_fail(p);
}

cheb_status cheb_workspace_bytes(cheb_plan p, int op, int nb, size_t* bytes) try {
  if (!p || !bytes) return CHEB_ERR_ARG;
  if (nb < 0) return fail(p, CHEB_ERR_ARG, "nb < 0");
  Ws w;
  CHK(ws_layout(p, op, op == CHEB_OP_BOUND ? 1 : nb, nullptr, &w));
  *bytes = w.total;
  return CHEB_OK;
} catch (...) {
  return host_fail(p);
}

cheb_status cheb_set_projectors(cheb_plan p, const void* P, int ldp, const double* Q, void* ws, size_t wsb,
                                hipStream_t st) try {
  if (!p) return CHEB_ERR_ARG;
  const int np = p->nproj;
  if (np == 0) { p->have_P = true; return CHEB_OK; }
  if (!P) return fail(p, CHEB_ERR_ARG, "P is null");
  if (ldp < p->npw) return fail(p, CHEB_ERR_ARG, "ldp < npw");
  if (p->has_overlap && !Q) return fail(p, CHEB_ERR_ARG, "Q is null but the plan has an overlap");
  if (!p->has_overlap && Q) return fail(p, CHEB_ERR_ARG, "Q given but the plan has S = I");
  Ws w;
  CHK(check_ws(p, CHEB_OP_SETUP, np, ws, wsb, &w));
  const c128* Pd = static_cast<const c128*>(P);
  if (p->prec == CHEB_MIXED) HIPCHK((convert_copy<float, double>(p->npw, np, Pd, ldp, static_cast<c64*>(p->P), p->npw, st)));
  else HIPCHK((convert_copy<double, double>(p->npw, np, Pd, ldp, static_cast<c128*>(p->P), p->npw, st)));
  if (p->prec == CHEB_MIXED) {
    // FP16 hi/lo planes of sA P with one power-of-two scale sA taking max |P| into [2^13, 2^14), the top of the
    // FP16 range: hi and lo then stay normal numbers (22 significant bits together) down to entries about 2^-17 of
    // the largest, where a scale to [0.5, 1) leaves every entry below 2^-14 with a subnormal hi and no lo
    double* cmax = reinterpret_cast<double*>(w.Hs);
    HIPCHK(column_maxabs(p->npw, np, Pd, ldp, cmax, st));
    std::vector<double> hmax(np);
    HIPCHK(hipMemcpyAsync(hmax.data(), cmax, sizeof(double) * np, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    double mx = 0.0;
    for (double v : hmax) {
      if (!std::isfinite(v)) return fail(p, CHEB_ERR_NONFINITE, "projectors hold NaN or Inf");
      mx = std::max(mx, v);
    }
    int e = 0;
    if (mx > 0.0) (void)std::frexp(mx, &e);
    const double sA = std::ldexp(1.0, kHalfTopExp - e);
    p->hproj.inv_scale = p->hback.inv_scale = std::ldexp(1.0, e - kHalfTopExp);
    HIPCHK(split_planes(Pd, ldp, p->npw, np, false, sA, const_cast<_Float16*>(p->hproj.p), p->hproj.rows, p->hproj.ld, st));
    HIPCHK(split_planes(Pd, ldp, p->npw, np, true, sA, const_cast<_Float16*>(p->hback.p), p->hback.rows, p->hback.ld, st));
  }
  // G = P^H P in FP64 from the caller's complex128 projectors
  Epi<double> eg;
  eg.out = p->G; eg.ldo = np; eg.real_only = p->gamma != 0;
  HIPCHK((gemm<double, double, double, double>(GEMM_CN, np, np, p->npw, Pd, ldp, Pd, ldp, eg,
                                               gemm_pick_splits(np, np, p->npw), w.part, st)));
  if (p->has_overlap) {
    HIPCHK(hipMemcpyAsync(p->Q, Q, sizeof(double) * np, hipMemcpyDeviceToDevice, st));
    HIPCHK(capacitance(np, p->G, p->Q, p->Cinv, st));
    HIPCHK((convert_copy<double, double>(np, np, p->Cinv, np, p->Cmat, np, st)));
    HIPCHK((fill_zero<float>(reinterpret_cast<c64*>(w.flags), 2, st)));
    HIPCHK(block_inverse(np, p->pinfo, p->Cmat, np, p->Minv, w.flags + 2, st));
    RBCHK(rocblas_set_stream(p->rb, st));
    RBCHK(rocblas_set_workspace(p->rb, w.solver, w.solver_bytes));
    rocblas_double_complex* C = reinterpret_cast<rocblas_double_complex*>(p->Cinv);
    rocblas_status r1 = rocsolver_zpotrf(p->rb, rocblas_fill_lower, np, C, np, w.flags);
    rocblas_status r2 = r1 == rocblas_status_success ? rocsolver_zpotri(p->rb, rocblas_fill_lower, np, C, np, w.flags + 1)
                                                     : r1;
    rocblas_set_workspace(p->rb, nullptr, 0);
    if (r2 != rocblas_status_success) return fail(p, CHEB_ERR_HIP, std::string("rocsolver potrf/potri: ") + rocblas_status_to_string(r2));
    int info[4] = {0, 0, 0, 0};
    HIPCHK(hipMemcpyAsync(info, w.flags, 3 * sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (info[0] != 0 || info[1] != 0) return fail(p, CHEB_ERR_NOT_PD, "capacitance matrix Q^-1 + P^H P is not positive definite");
    p->cap_blocks_ok = info[2] == 0;
    HIPCHK(hermitian_from_lower(np, p->Cinv, np, st));
  }
  HIPCHK(hipStreamSynchronize(st));
  p->have_P = true;
  return CHEB_OK;
} catch (...) {
  return host_fail(p);
}

#define OP_PRELUDE(op, nbv)                  \
  if (!p) return CHEB_ERR_ARG;               \
  CHK(check_ready(p));                       \
  Ws w;                                      \
  if ((nbv) > 0) CHK(check_ws(p, op, nbv, ws, wsb, &w));

static cheb_status apply_common(cheb_plan p, int which, const void* X, int ldx, void* Y, int ldy, int nb, void* ws,
                                size_t wsb, hipStream_t st) {
  if (!p) return CHEB_ERR_ARG;
  CHK(check_block(p, X, ldx, nb, "X"));
  CHK(check_block(p, Y, ldy, nb, "Y"));
  if (nb == 0) return CHEB_OK;
  const size_t eb = elem_bytes(p->prec);
  const char *xa = static_cast<const char*>(X), *ya = static_cast<const char*>(Y);
  const char *xe = xa + (size_t(ldx) * (nb - 1) + p->npw) * eb, *ye = ya + (size_t(ldy) * (nb - 1) + p->npw) * eb;
  if (xa < ye && ya < xe) return fail(p, CHEB_ERR_ARG, "X and Y overlap");
  OP_PRELUDE(which == 0 ? CHEB_OP_H : CHEB_OP_SINV, nb);
  return with_prec(p, st, [&](auto ops) {
    using C = typename decltype(ops)::C;
    const C* x = static_cast<const C*>(X);
    C* y = static_cast<C*>(Y);
    if (which == 0) return ops.apply_H(x, ldx, y, ldy, nb, w);
    if (which == 1) return ops.apply_S(x, ldx, y, ldy, nb, w);
    return ops.apply_Sinv(x, ldx, y, ldy, nb, w);
  });
}

cheb_status cheb_apply_H(cheb_plan p, const void* X, int ldx, void* Y, int ldy, int nb, void* ws, size_t wsb,
                         hipStream_t st) try {
  return apply_common(p, 0, X, ldx, Y, ldy, nb, ws, wsb, st);
} catch (...) {
  return host_fail(p);
}
cheb_status cheb_apply_S(cheb_plan p, const void* X, int ldx, void* Y, int ldy, int nb, void* ws, size_t wsb,
                         hipStream_t st) try {
  return apply_common(p, 1, X, ldx, Y, ldy, nb, ws, wsb, st);
} catch (...) {
  return host_fail(p);
}
cheb_status cheb_apply_Sinv(cheb_plan p, const void* X, int ldx, void* Y, int ldy, int nb, void* ws, size_t wsb,
                            hipStream_t st) try {
  return apply_common(p, 2, X, ldx, Y, ldy, nb, ws, wsb, st);
} catch (...) {
  return host_fail(p);
}

cheb_status cheb_apply_H_noalloc(cheb_plan p, const void* X, int ldx, void* Y, int ldy, int nb, hipStream_t st) try {
  if (!p) return CHEB_ERR_ARG;
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev != p->device) return fail(p, CHEB_ERR_ARG, "cheb_apply_H_noalloc: the plan's device is not current");
  if (!p->scratch) return fail(p, CHEB_ERR_HIP, "cheb_apply_H_noalloc: the static scratch has no device address");
  if (nb < 0) return fail(p, CHEB_ERR_ARG, "nb < 0");
  Ws probe;
  CHK(ws_layout(p, CHEB_OP_H, nb, nullptr, &probe));
  if (probe.total > kNoAllocScratchBytes)
    return fail(p, CHEB_ERR_WORKSPACE, "cheb_apply_H_noalloc: " + std::to_string(nb) + " bands need " +
                                           std::to_string(probe.total) + " bytes of scratch, the static scratch holds " +
                                           std::to_string(kNoAllocScratchBytes) + "; use cheb_apply_H with a workspace");
  // no profiling events from this entry point (creating them may allocate)
  const bool prof = p->prof_on;
  p->prof_on = false;
  const cheb_status s = apply_common(p, 0, X, ldx, Y, ldy, nb, p->scratch, kNoAllocScratchBytes, st);
  p->prof_on = prof;
  return s;
} catch (...) {
  return host_fail(p);
}

cheb_status cheb_filter(cheb_plan p, void* X, int ldx, int nb, int m, double c, double r, void* ws, size_t wsb,
                        hipStream_t st) try {
  if (!p) return CHEB_ERR_ARG;
  CHK(check_block(p, X, ldx, nb, "X"));
  if (m < 0) return fail(p, CHEB_ERR_ARG, "degree m < 0");
  if (!(r > 0.0) || !std::isfinite(r) || !std::isfinite(c)) return fail(p, CHEB_ERR_ARG, "need finite c and r > 0");
  if (nb == 0 || m == 0) return CHEB_OK;
  OP_PRELUDE(CHEB_OP_FILTER, nb);
  return with_prec(p, st, [&](auto ops) {
    using C = typename decltype(ops)::C;
    return ops.filter(static_cast<C*>(X), ldx, nb, m, c, r, w);
  });
} catch (...) {
  return host_fail(p);
}

cheb_status cheb_filter_carry(cheb_plan p, void* X, int ldx, int nb, int m, double c, double r, const void* p_in,
                              const void* hx_in, void* ws, size_t wsb, hipStream_t st) try {
  if (!p) return CHEB_ERR_ARG;
  CHK(check_block(p, X, ldx, nb, "X"));
  if (m < 0) return fail(p, CHEB_ERR_ARG, "degree m < 0");
  if (!(r > 0.0) || !std::isfinite(r) || !std::isfinite(c)) return fail(p, CHEB_ERR_ARG, "need finite c and r > 0");
  if (nb == 0) return CHEB_OK;
  OP_PRELUDE(CHEB_OP_FILTER, nb);
  return with_prec(p, st, [&](auto ops) {
    using C = typename decltype(ops)::C;
    return ops.filter(static_cast<C*>(X), ldx, nb, m, c, r, w, static_cast<const c128*>(p_in),
                      static_cast<const C*>(hx_in));
  });
} catch (...) {
  return host_fail(p);
}

cheb_status cheb_filter_degrees(cheb_plan p, void* X, int ldx, int nb, const int32_t* degrees, double c, double r,
                                void* ws, size_t wsb, hipStream_t st) try {
  if (!p) return CHEB_ERR_ARG;
  CHK(check_block(p, X, ldx, nb, "X"));
  if (nb > 0 && !degrees) return fail(p, CHEB_ERR_ARG, "degrees is null");
  if (!(r > 0.0) || !std::isfinite(r) || !std::isfinite(c)) return fail(p, CHEB_ERR_ARG, "need finite c and r > 0");
  if (nb > 65535) return fail(p, CHEB_ERR_ARG, "nb > 65535");
  int m = 0;
  for (int b = 0; b < nb; ++b) {
    if (degrees[b] < 0) return fail(p, CHEB_ERR_ARG, "negative degree for band " + std::to_string(b));
    m = std::max(m, int(degrees[b]));
  }
  if (nb == 0 || m == 0) return CHEB_OK;
  OP_PRELUDE(CHEB_OP_FILTER_DEGREES, nb);
  // order of decreasing degree (stable), active counts per step, gather and scatter lists
  std::vector<int> order(nb);
  for (int b = 0; b < nb; ++b) order[b] = b;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return degrees[a] > degrees[b]; });
  std::vector<int> active(m, 0);
  int na = 0, ne = 0, no = 0;
  for (int j = 0; j < nb; ++j) {
    const int d = degrees[order[j]];
    if (d == 0) break;
    ++na;
    for (int i = 0; i < d; ++i) ++active[i];
    (d & 1 ? no : ne) += 1;
  }
  const size_t need = 3 * size_t(na);
  CHK(staging(p, need));
  int* h = p->lock_host;
  int* hev = h + na;
  int* hod = hev + 2 * ne;
  for (int j = 0, e = 0, o = 0; j < na; ++j) {
    h[j] = order[j];
    if (degrees[order[j]] & 1) { hod[o] = j; hod[no + o] = order[j]; ++o; }
    else { hev[e] = j; hev[ne + e] = order[j]; ++e; }
  }
  HIPCHK(hipMemcpyAsync(w.lidx, h, need * sizeof(int), hipMemcpyHostToDevice, st));
  HIPCHK(hipEventRecord(p->lock_ev, st));
  return with_prec(p, st, [&](auto ops) {
    using C = typename decltype(ops)::C;
    return ops.filter_degrees(static_cast<C*>(X), ldx, active, w.lidx, ne, no, c, r, w);
  });
} catch (...) {
  return host_fail(p);
}

cheb_status cheb_gemm_splits(int M, int N, int K, int* fp64, int* fp16, int* bound) try {
  if (!fp64 || !fp16 || !bound) return CHEB_ERR_ARG;
  *fp64 = gemm_pick_splits(M, N, K);
  *fp16 = gemm_h_pick_splits(M, N, K);
  *bound = gemm_split_bound(M, N, K);
  return CHEB_OK;
} catch (...) {
  return host_fail(nullptr);
}

cheb_status cheb_gemm_block_item(int i, int total, int tm, int tn, int group, int* bx, int* by, int* bz) try {
  if (!bx || !by || !bz || tm <= 0 || tn <= 0 || total <= 0 || i < 0 || i >= total) return CHEB_ERR_ARG;
  if (group == -1) {  // upper-triangle tiles of a square grid
    if (tn != tm || total % (long(tm) * (tm + 1) / 2)) return CHEB_ERR_ARG;
  } else if (group < 1 || total % (long(tm) * tn)) {
    return CHEB_ERR_ARG;
  }
  gemm_block_item(i, total, tm, tn, group, *bx, *by, *bz);
  return CHEB_OK;
} catch (...) {
  return host_fail(nullptr);
}

cheb_status cheb_locking_degrees(int nb, const double* ritz, const double* resid, double c, double r, int m_max,
                                 double tol, int32_t* degrees, int* nlocked) try {
  if (nb < 0 || m_max < 1 || !(r > 0.0) || !std::isfinite(c) || !std::isfinite(r) || !(tol >= 0.0)) return CHEB_ERR_ARG;
  if (nb > 0 && (!ritz || !resid || !degrees)) return CHEB_ERR_ARG;
  int locked = 0;
  for (int i = 0; i < nb; ++i) {
    if (!std::isfinite(resid[i]) || !std::isfinite(ritz[i])) return CHEB_ERR_ARG;
    if (resid[i] <= tol) {
      degrees[i] = 0;
      ++locked;
      continue;
    }
    // T_n(x) by its three-term recurrence; the estimate resid / |T_n(x)| (Eq. 5)
    const double x = (ritz[i] - c) / r;
    double t0 = 1.0, t1 = x;
    int deg = m_max;
    for (int n = 1; n <= m_max; ++n) {
      if (resid[i] <= tol * std::fabs(t1)) { deg = n; break; }
      const double t2 = 2.0 * x * t1 - t0;
      t0 = t1;
      t1 = t2;
    }
    degrees[i] = deg;
  }
  if (nlocked) *nlocked = locked;
  return CHEB_OK;
} catch (...) {
  return host_fail(nullptr);
}

cheb_status cheb_rayleigh_ritz(cheb_plan p, void* X, int ldx, int nb, double* ritz, double* resid, void* ws,
                               size_t wsb, hipStream_t st) try {
  if (!p) return CHEB_ERR_ARG;
  CHK(check_block(p, X, ldx, nb, "X"));
  if (nb > 0 && !ritz) return fail(p, CHEB_ERR_ARG, "ritz is null");
  if (nb == 0) return CHEB_OK;
  OP_PRELUDE(CHEB_OP_RR, nb);
  return with_prec(p, st, [&](auto ops) {
    using C = typename decltype(ops)::C;
    return ops.rayleigh_ritz(static_cast<C*>(X), ldx, nb, ritz, resid, w);
  });
} catch (...) {
  return host_fail(p);
}

cheb_status cheb_rayleigh_ritz_carry(cheb_plan p, void* X, int ldx, int nb, double* ritz, double* resid,
                                     void* p_out, void* hx_out, void* ws, size_t wsb, hipStream_t st) try {
  if (!p) return CHEB_ERR_ARG;
  CHK(check_block(p, X, ldx, nb, "X"));
  if (nb > 0 && !ritz) return fail(p, CHEB_ERR_ARG, "ritz is null");
  if (nb == 0) return CHEB_OK;
  OP_PRELUDE(CHEB_OP_RR, nb);
  return with_prec(p, st, [&](auto ops) {
    using C = typename decltype(ops)::C;
    return ops.rayleigh_ritz(static_cast<C*>(X), ldx, nb, ritz, resid, w, static_cast<c128*>(p_out),
                             static_cast<C*>(hx_out));
  });
} catch (...) {
  return host_fail(p);
}

cheb_status cheb_rayleigh_quotients(cheb_plan p, const void* X, int ldx, int nb, double* rq, void* ws, size_t wsb,
                                    hipStream_t st) try {
  if (!p) return CHEB_ERR_ARG;
  CHK(check_block(p, X, ldx, nb, "X"));
  if (nb > 0 && !rq) return fail(p, CHEB_ERR_ARG, "rq is null");
  if (nb == 0) return CHEB_OK;
  OP_PRELUDE(CHEB_OP_RR, nb);
  return with_prec(p, st, [&](auto ops) {
    using C = typename decltype(ops)::C;
    return ops.rayleigh_quotients(static_cast<const C*>(X), ldx, nb, rq, w);
  });
} catch (...) {
  return host_fail(p);
}

cheb_status cheb_upper_bound(cheb_plan p, int k, const void* v0, double* lambda_plus, void* ws, size_t wsb,
                             hipStream_t st) try {
  if (!p) return CHEB_ERR_ARG;
  if (k < 1 || k > 64) return fail(p, CHEB_ERR_ARG, "k must be in [1, 64]");
  if (!v0 || !lambda_plus) return fail(p, CHEB_ERR_ARG, "null v0 or output");
  OP_PRELUDE(CHEB_OP_BOUND, 1);
  return with_prec(p, st, [&](auto ops) {
    using C = typename decltype(ops)::C;
    return ops.upper_bound(k, static_cast<const C*>(v0), lambda_plus, w);
  });
} catch (...) {
  return host_fail(p);
}

cheb_status cheb_lobpcg_state_bytes(cheb_plan p, int nb, size_t* bytes) try {
  if (!p || !bytes) return CHEB_ERR_ARG;
  if (nb < 1) return fail(p, CHEB_ERR_ARG, "nb must be >= 1");
  *bytes = 15 * size_t(p->npw) * nb * elem_bytes(p->prec);
  return CHEB_OK;
} catch (...) {
  return host_fail(p);
}

cheb_status cheb_lobpcg_iterate(cheb_plan p, void* X, int ldx, int nb, int iteration, double tol, void* state,
                                size_t state_bytes, double* ritz_dev, double* resid_dev, int* nactive, void* ws,
                                size_t wsb, hipStream_t st) try {
  if (!p) return CHEB_ERR_ARG;
  CHK(check_ready(p));
  CHK(check_block(p, X, ldx, nb, "X"));
  if (nb < 1) return fail(p, CHEB_ERR_ARG, "nb must be >= 1");
  if (3 * nb > p->npw) return fail(p, CHEB_ERR_ARG, "3 nb must not exceed npw");
  if (p->prec != CHEB_FP64)
    return fail(p, CHEB_ERR_ARG, "LOBPCG runs on FP64 plans (its carried products drift in complex64)");
  if (p->gamma) return fail(p, CHEB_ERR_ARG, "LOBPCG is not available for Gamma plans");
  if (iteration < 0) return fail(p, CHEB_ERR_ARG, "iteration < 0");
  if (!(tol >= 0.0) || !std::isfinite(tol)) return fail(p, CHEB_ERR_ARG, "tol must be finite and >= 0");
  if (!ritz_dev) return fail(p, CHEB_ERR_ARG, "ritz is null");
  size_t need = 0;
  CHK(cheb_lobpcg_state_bytes(p, nb, &need));
  if (!state || state_bytes < need) return fail(p, CHEB_ERR_WORKSPACE, "LOBPCG state too small: need " + std::to_string(need));
  if (reinterpret_cast<uintptr_t>(state) % 16) return fail(p, CHEB_ERR_ARG, "state not 16-byte aligned");
  Ws w;
  CHK(check_ws(p, CHEB_OP_LOBPCG, nb, ws, wsb, &w));
  return with_prec(p, st, [&](auto ops) {
    using C = typename decltype(ops)::C;
    return ops.lobpcg(static_cast<C*>(X), ldx, nb, iteration, tol, state, ritz_dev, resid_dev, nactive, w);
  });
} catch (...) {
  return host_fail(p);
}

cheb_status cheb_set_capacitance_solver(cheb_plan p, int iterations) try {
  if (!p) return CHEB_ERR_ARG;
  if (iterations < 0 || iterations > 1000) return fail(p, CHEB_ERR_ARG, "iterations must be in [0, 1000]");
  if (iterations > 0 && !p->has_overlap) return fail(p, CHEB_ERR_ARG, "the plan has S = I: no capacitance matrix");
  if (iterations > 0 && p->nproj > 0 && !p->have_P) return fail(p, CHEB_ERR_STATE, "projectors not set");
  if (iterations > 0 && p->nproj > 0 && !p->cap_blocks_ok)
    return fail(p, CHEB_ERR_ARG, "atom blocks larger than 32 projectors: no block preconditioner");
  p->cap_iters = iterations;
  return CHEB_OK;
} catch (...) {
  return host_fail(p);
}

cheb_status cheb_set_split_gemm(cheb_plan p, int on) try {
  if (!p) return CHEB_ERR_ARG;
  p->split_gemm = on != 0;
  return CHEB_OK;
} catch (...) {
  return host_fail(p);
}

cheb_status cheb_set_projection_resync(cheb_plan p, int period) try {
  if (!p) return CHEB_ERR_ARG;
  if (period < 0) return fail(p, CHEB_ERR_ARG, "resync period < 0");
  p->resync = period;
  return CHEB_OK;
} catch (...) {
  return host_fail(p);
}

cheb_status cheb_drift_monitor(cheb_plan p, int on) try {
  if (!p) return CHEB_ERR_ARG;
  p->drift_on = on != 0;
  p->drift_max = 0.0;
  p->drift_checks = 0;
  return CHEB_OK;
} catch (...) {
  return host_fail(p);
}

cheb_status cheb_drift_read(cheb_plan p, double* max_rel, int64_t* checks) try {
  if (!p) return CHEB_ERR_ARG;
  if (max_rel) *max_rel = p->drift_max;
  if (checks) *checks = p->drift_checks;
  return CHEB_OK;
} catch (...) {
  return host_fail(p);
}

cheb_status cheb_set_rr_refine(cheb_plan p, int on) try {
  if (!p) return CHEB_ERR_ARG;
  p->rr_refine = on != 0;
  return CHEB_OK;
} catch (...) {
  return host_fail(p);
}

cheb_status cheb_rr_stats(cheb_plan p, int64_t* refined, int64_t* fallback) try {
  if (!p) return CHEB_ERR_ARG;
  if (refined) *refined = p->rr_refined;
  if (fallback) *fallback = p->rr_fallback;
  return CHEB_OK;
} catch (...) {
  return host_fail(p);
}

static cheb_status backward_check(cheb_plan p, int nb, int m, int k) {
  if (nb < 1) return fail(p, CHEB_ERR_ARG, "nb must be >= 1");
  if (m < 1) return fail(p, CHEB_ERR_ARG, "degree m must be >= 1");
  if (k < 1) return fail(p, CHEB_ERR_ARG, "ckpt_every must be >= 1");
  if (p->gamma) return fail(p, CHEB_ERR_ARG, "the adjoint is not available for Gamma plans");
  if (fft_xdens_lds_bytes(p->n, p->rx, p->prec != CHEB_MIXED) > 160 * 1024)
    return fail(p, CHEB_ERR_ARG, "sphere too wide in x for the cross-density pass in 160 KB of LDS");
  return CHEB_OK;
}

cheb_status cheb_backward_workspace_bytes(cheb_plan p, int nb, int m, int ckpt_every, size_t* bytes) try {
  if (!p || !bytes) return CHEB_ERR_ARG;
  CHK(backward_check(p, nb, m, ckpt_every));
  BwdWs w;
  CHK(bwd_layout(p, nb, m, ckpt_every, nullptr, &w));
  *bytes = w.total;
  return CHEB_OK;
} catch (...) {
  return host_fail(p);
}

cheb_status cheb_filter_rr_backward(cheb_plan p, const void* X0, int ldx, int nb, int m, double c, double r, int nk,
                                   const double* w_dev, int ckpt_every, double* ritz_dev, void* dX, int lddx,
                                   double* dV_dev, double* dD_dev, void* ws, size_t wsb, hipStream_t st) try {
  if (!p) return CHEB_ERR_ARG;
  CHK(check_ready(p));
  CHK(backward_check(p, nb, m, ckpt_every));
  CHK(check_block(p, X0, ldx, nb, "X0"));
  CHK(check_block(p, dX, lddx, nb, "dX"));
  if (nk < 1 || nk > nb) return fail(p, CHEB_ERR_ARG, "nk must be in [1, nb]");
  if (!w_dev || !ritz_dev || !dV_dev) return fail(p, CHEB_ERR_ARG, "null w, ritz or dV");
  if (p->dsize > 0 && !dD_dev) return fail(p, CHEB_ERR_ARG, "null dD");
  if (!(r > 0.0) || !std::isfinite(r) || !std::isfinite(c)) return fail(p, CHEB_ERR_ARG, "need finite c and r > 0");
  BwdWs probe;
  CHK(bwd_layout(p, nb, m, ckpt_every, nullptr, &probe));
  if (wsb < probe.total) return fail(p, CHEB_ERR_WORKSPACE, "workspace too small: need " + std::to_string(probe.total));
  if (!ws || reinterpret_cast<uintptr_t>(ws) % kAlign) return fail(p, CHEB_ERR_ARG, "workspace null or not 256-byte aligned");
  BwdWs w;
  CHK(bwd_layout(p, nb, m, ckpt_every, ws, &w));
  return with_prec(p, st, [&](auto ops) {
    using C = typename decltype(ops)::C;
    return ops.backward(static_cast<const C*>(X0), ldx, nb, m, c, r, nk, w_dev, ckpt_every, ritz_dev,
                        static_cast<C*>(dX), lddx, dV_dev, dD_dev, w);
  });
} catch (...) {
  return host_fail(p);
}

}  // extern "C"
