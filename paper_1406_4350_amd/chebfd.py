"""Thin Python binding of libchebfd.so (include/chebfd.h).

The methods of Plan carry the C names without their cheb_ prefix (Plan.apply_H is cheb_apply_H, and so on) and
only marshal arguments: torch tensors provide device memory and the current HIP stream, every computation runs
in the library's HIP kernels. There is no CPU
fallback: loading fails loudly when the library or a GPU is missing.

Band blocks are torch tensors of shape (nb, npw), contiguous, complex128 (CHEB_FP64) or complex64
(CHEB_MIXED): row b is band b, i.e. the column-major npw x nb block of the C ABI with ldx = npw.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libchebfd.so")

CHEB_OK, CHEB_ERR_ARG, CHEB_ERR_HIP, CHEB_ERR_WORKSPACE, CHEB_ERR_NOT_PD, CHEB_ERR_EIG, CHEB_ERR_NONFINITE, \
    CHEB_ERR_STATE, CHEB_ERR_HOST = range(9)
STATUS_NAMES = ["CHEB_OK", "CHEB_ERR_ARG", "CHEB_ERR_HIP", "CHEB_ERR_WORKSPACE", "CHEB_ERR_NOT_PD", "CHEB_ERR_EIG",
                "CHEB_ERR_NONFINITE", "CHEB_ERR_STATE", "CHEB_ERR_HOST"]
CHEB_FP64, CHEB_MIXED = 0, 1
(CHEB_OP_H, CHEB_OP_SINV, CHEB_OP_FILTER, CHEB_OP_RR, CHEB_OP_BOUND, CHEB_OP_SETUP, CHEB_OP_FILTER_DEGREES,
 CHEB_OP_LOBPCG) = range(8)

# exported symbols, as declared in include/chebfd.h
SYMBOLS = ["cheb_plan_persistent_bytes", "cheb_plan_create", "cheb_plan_destroy", "cheb_set_potential",
           "cheb_set_projectors", "cheb_set_D", "cheb_workspace_bytes", "cheb_apply_H", "cheb_apply_S",
           "cheb_apply_Sinv", "cheb_filter", "cheb_rayleigh_ritz", "cheb_rayleigh_quotients", "cheb_upper_bound",
           "cheb_profile_enable", "cheb_profile_read", "cheb_backward_workspace_bytes", "cheb_filter_rr_backward",
           "cheb_set_rr_refine", "cheb_rr_stats", "cheb_filter_degrees", "cheb_locking_degrees", "cheb_set_split_gemm",
           "cheb_set_capacitance_solver", "cheb_lobpcg_state_bytes", "cheb_lobpcg_iterate", "cheb_gemm_splits",
           "cheb_gemm_block_item", "cheb_set_projection_resync", "cheb_drift_monitor", "cheb_drift_read",
           "cheb_apply_H_noalloc", "cheb_filter_carry", "cheb_rayleigh_ritz_carry", "cheb_last_error"]
TIMERS = ["fft_col_inverse", "fft_plane", "fft_col_forward", "project", "backproject", "small", "rr_gram", "rr_eig",
          "rr_rotate", "xdens"]


class ChebError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str = ""):
        self.status = status
        name = STATUS_NAMES[status] if 0 <= status < len(STATUS_NAMES) else str(status)
        super().__init__(f"{where}: {name}" + (f": {msg}" if msg else ""))


class cheb_desc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("npw", ctypes.c_int), ("gidx_host", ctypes.c_void_p),
                ("kin_host", ctypes.c_void_p), ("natom", ctypes.c_int), ("proj_off_host", ctypes.c_void_p),
                ("has_overlap", ctypes.c_int), ("prec", ctypes.c_int), ("gamma", ctypes.c_int)]


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libchebfd.so and declare its signatures. Raises if it is missing (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_1406_4350_amd.build`")
    lib = ctypes.CDLL(path)
    vp, sz, i, d = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_double
    P = ctypes.POINTER
    sig = {
        "cheb_plan_persistent_bytes": [P(cheb_desc), P(sz)],
        "cheb_plan_create": [P(cheb_desc), vp, sz, vp, P(vp)],
        "cheb_plan_destroy": [vp],
        "cheb_set_potential": [vp, vp, vp],
        "cheb_set_projectors": [vp, vp, i, vp, vp, sz, vp],
        "cheb_set_D": [vp, vp, vp],
        "cheb_workspace_bytes": [vp, i, i, P(sz)],
        "cheb_apply_H": [vp, vp, i, vp, i, i, vp, sz, vp],
        "cheb_apply_S": [vp, vp, i, vp, i, i, vp, sz, vp],
        "cheb_apply_Sinv": [vp, vp, i, vp, i, i, vp, sz, vp],
        "cheb_filter": [vp, vp, i, i, i, d, d, vp, sz, vp],
        "cheb_rayleigh_ritz": [vp, vp, i, i, vp, vp, vp, sz, vp],
        "cheb_filter_carry": [vp, vp, i, i, i, d, d, vp, vp, vp, sz, vp],
        "cheb_rayleigh_ritz_carry": [vp, vp, i, i, vp, vp, vp, vp, vp, sz, vp],
        "cheb_rayleigh_quotients": [vp, vp, i, i, vp, vp, sz, vp],
        "cheb_upper_bound": [vp, i, vp, P(d), vp, sz, vp],
        "cheb_profile_enable": [vp, i],
        "cheb_profile_read": [vp, i, P(d), P(ctypes.c_int64), P(d), P(d)],
        "cheb_backward_workspace_bytes": [vp, i, i, i, P(sz)],
        "cheb_filter_rr_backward": [vp, vp, i, i, i, d, d, i, vp, i, vp, vp, i, vp, vp, vp, sz, vp],
        "cheb_set_rr_refine": [vp, i],
        "cheb_rr_stats": [vp, P(ctypes.c_int64), P(ctypes.c_int64)],
        "cheb_filter_degrees": [vp, vp, i, i, vp, d, d, vp, sz, vp],
        "cheb_set_split_gemm": [vp, i],
        "cheb_set_capacitance_solver": [vp, i],
        "cheb_lobpcg_state_bytes": [vp, i, P(sz)],
        "cheb_lobpcg_iterate": [vp, vp, i, i, i, d, vp, sz, vp, vp, P(i), vp, sz, vp],
        "cheb_locking_degrees": [i, vp, vp, d, d, i, d, vp, P(i)],
        "cheb_gemm_splits": [i, i, i, P(i), P(i), P(i)],
        "cheb_gemm_block_item": [i, i, i, i, i, P(i), P(i), P(i)],
        "cheb_set_projection_resync": [vp, i],
        "cheb_apply_H_noalloc": [vp, vp, i, vp, i, i, vp],
        "cheb_drift_monitor": [vp, i],
        "cheb_drift_read": [vp, P(d), P(ctypes.c_int64)],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.cheb_last_error.argtypes = [vp]
    lib.cheb_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def locking_degrees(ritz, resid, c: float, r: float, m_max: int, tol: float):
    """Degrees per band from the residual estimate of Eq. 5 (cheb_locking_degrees, host arithmetic only).
    Returns (degrees int32 array, number of locked bands)."""
    lib = load_library()
    ritz = np.ascontiguousarray(ritz, dtype=np.float64)
    resid = np.ascontiguousarray(resid, dtype=np.float64)
    if ritz.shape != resid.shape or ritz.ndim != 1:
        raise ValueError("ritz and resid must be 1-D of equal length")
    deg = np.empty(ritz.shape[0], dtype=np.int32)
    nlocked = ctypes.c_int()
    st = lib.cheb_locking_degrees(ritz.shape[0], ritz.ctypes.data, resid.ctypes.data, float(c), float(r), int(m_max),
                                  float(tol), deg.ctypes.data, ctypes.byref(nlocked))
    if st != CHEB_OK:
        raise ChebError(st, "cheb_locking_degrees")
    return deg, nlocked.value


def _ptr(t) -> int | None:
    return None if t is None else t.data_ptr()


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


class Plan:
    """A plan over one problem (sphere, box, atoms, precision); owns its persistent device buffer."""

    def __init__(self, gidx: np.ndarray, kin: np.ndarray, n: int, proj_off: np.ndarray, has_overlap: bool,
                 prec: int = CHEB_FP64, device: str = "cuda", gamma: bool = False):
        self.lib = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("chebfd needs a GPU (torch.cuda.is_available() is False)")
        self.device = torch.device(device)
        self._gidx = np.ascontiguousarray(gidx, dtype=np.int32)
        self._kin = np.ascontiguousarray(kin, dtype=np.float64)
        self._off = np.ascontiguousarray(proj_off, dtype=np.int32)
        self.n, self.npw = int(n), int(self._gidx.shape[0])
        self.natom = int(self._off.shape[0] - 1)
        self.nproj = int(self._off[-1]) if self.natom > 0 else 0
        self.prec = prec
        self.dtype = torch.complex64 if prec == CHEB_MIXED else torch.complex128
        self.gamma = bool(gamma)
        self.desc = cheb_desc(self.n, self.npw, self._gidx.ctypes.data, self._kin.ctypes.data, self.natom,
                              self._off.ctypes.data if self.natom > 0 else None, int(bool(has_overlap)), prec,
                              int(self.gamma))
        nbytes = ctypes.c_size_t()
        self._check(self.lib.cheb_plan_persistent_bytes(ctypes.byref(self.desc), ctypes.byref(nbytes)),
                    "cheb_plan_persistent_bytes", plan=False)
        self.persistent = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p()
        self._check(self.lib.cheb_plan_create(ctypes.byref(self.desc), self.persistent.data_ptr(), nbytes.value,
                                              _stream(), ctypes.byref(h)), "cheb_plan_create", plan=False)
        self.handle = h
        self._ws = {}

    # -- plumbing --------------------------------------------------------------------------------------------
    def _check(self, st: int, where: str, plan: bool = True):
        if st != CHEB_OK:
            msg = ""
            if plan and getattr(self, "handle", None):
                msg = self.lib.cheb_last_error(self.handle).decode()
            raise ChebError(st, where, msg)

    def workspace(self, op: int, nb: int) -> torch.Tensor:
        """Cached workspace for (op, nb); cheb_workspace_bytes is asked every time, since plan settings (the
        capacitance solver) change the size."""
        key = (op, nb)
        nbytes = ctypes.c_size_t()
        self._check(self.lib.cheb_workspace_bytes(self.handle, op, nb, ctypes.byref(nbytes)), "cheb_workspace_bytes")
        if key not in self._ws or self._ws[key].numel() < nbytes.value:
            self._ws[key] = torch.empty(max(nbytes.value, 256), dtype=torch.uint8, device=self.device)
        return self._ws[key]

    def lobpcg_state(self, nb: int) -> torch.Tensor:
        """Device buffer carrying H X, S X and the search directions between LOBPCG iterations."""
        nbytes = ctypes.c_size_t()
        self._check(self.lib.cheb_lobpcg_state_bytes(self.handle, int(nb), ctypes.byref(nbytes)),
                    "cheb_lobpcg_state_bytes")
        return torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)

    def lobpcg_iterate(self, X, iteration: int, tol: float, state: torch.Tensor, ritz: torch.Tensor):
        """One LOBPCG iteration in place on X (nb, npw); ritz (nb FP64, device) is read and updated.
        Returns (residual norms of the vectors that entered, number of active bands)."""
        nb, ldx = self._block(X, "X")
        res = torch.zeros(nb, dtype=torch.float64, device=self.device)
        ws = self.workspace(CHEB_OP_LOBPCG, nb)
        nact = ctypes.c_int()
        self._check(self.lib.cheb_lobpcg_iterate(self.handle, X.data_ptr(), ldx, nb, int(iteration), float(tol),
                                                 state.data_ptr(), state.numel(), ritz.data_ptr(), res.data_ptr(),
                                                 ctypes.byref(nact), ws.data_ptr(), ws.numel(), _stream()),
                    "cheb_lobpcg_iterate")
        return res, nact.value

    def set_capacitance_solver(self, iterations: int):
        """0: apply C^-1 directly (default); k > 0: k corrections of block-preconditioned iterative refinement."""
        self._check(self.lib.cheb_set_capacitance_solver(self.handle, int(iterations)), "cheb_set_capacitance_solver")

    def _block(self, X: torch.Tensor, name: str) -> tuple[int, int]:
        if X.dtype != self.dtype or X.device.type != "cuda" or X.dim() != 2 or X.shape[1] != self.npw:
            raise ValueError(f"{name}: expected a (nb, {self.npw}) {self.dtype} CUDA tensor, got {tuple(X.shape)} "
                             f"{X.dtype} on {X.device}")
        if X.stride(1) != 1:
            raise ValueError(f"{name}: rows must be contiguous")
        return X.shape[0], X.stride(0)

    def close(self):
        if getattr(self, "handle", None):
            self.lib.cheb_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass

    # -- set-up ----------------------------------------------------------------------------------------------
    def set_potential(self, V: torch.Tensor):
        V = V.to(self.device, torch.float64).contiguous()
        assert V.shape == (self.n,) * 3
        self._check(self.lib.cheb_set_potential(self.handle, V.data_ptr(), _stream()), "cheb_set_potential")
        self._V = V

    def set_projectors(self, P: torch.Tensor, Q: torch.Tensor | None):
        """P: (nproj, npw) complex128 (row j = projector j), Q: (nproj,) float64 or None."""
        P = P.to(self.device, torch.complex128).contiguous()
        Qd = None if Q is None else Q.to(self.device, torch.float64).contiguous()
        ws = self.workspace(CHEB_OP_SETUP, self.nproj)
        self._check(self.lib.cheb_set_projectors(self.handle, _ptr(P) if self.nproj else None, self.npw, _ptr(Qd),
                                                 ws.data_ptr(), ws.numel(), _stream()), "cheb_set_projectors")
        self._P, self._Q = P, Qd

    def set_D(self, D: torch.Tensor):
        D = D.to(self.device, torch.float64).contiguous()
        self._check(self.lib.cheb_set_D(self.handle, _ptr(D) if D.numel() else None, _stream()), "cheb_set_D")
        self._D = D

    # -- operations ----------------------------------------------------------------------------------------------
    def _apply(self, fn, op, X, Y):
        nb, ldx = self._block(X, "X")
        if Y is None:
            Y = torch.empty_like(X)
        _, ldy = self._block(Y, "Y")
        ws = self.workspace(op, nb)
        self._check(getattr(self.lib, fn)(self.handle, X.data_ptr(), ldx, Y.data_ptr(), ldy, nb, ws.data_ptr(),
                                          ws.numel(), _stream()), fn)
        return Y

    def apply_H(self, X, Y=None):
        return self._apply("cheb_apply_H", CHEB_OP_H, X, Y)

    def apply_H_noalloc(self, X, Y=None):
        """Y = H X through the entry point that allocates nothing (the library's static device scratch)."""
        nb, ldx = self._block(X, "X")
        if Y is None:
            Y = torch.empty_like(X)
        _, ldy = self._block(Y, "Y")
        self._check(self.lib.cheb_apply_H_noalloc(self.handle, X.data_ptr(), ldx, Y.data_ptr(), ldy, nb, _stream()),
                    "cheb_apply_H_noalloc")
        return Y

    def apply_S(self, X, Y=None):
        return self._apply("cheb_apply_S", CHEB_OP_SINV, X, Y)

    def apply_Sinv(self, X, Y=None):
        return self._apply("cheb_apply_Sinv", CHEB_OP_SINV, X, Y)

    def filter(self, X, m: int, c: float, r: float, p_in=None, hx_in=None):
        """X <- T_m((S^-1 H - c)/r) X. p_in: None, or the projections P^H X of the block (a complex128 (nb, nproj)
        device tensor, row j = band j); hx_in: None, or (K + V) X (an (nb, npw) device tensor of the plan's dtype);
        normally the p_out and hx_out of rayleigh_ritz (see cheb_filter_carry)."""
        nb, ldx = self._block(X, "X")
        ws = self.workspace(CHEB_OP_FILTER, nb)
        if p_in is None and hx_in is None:
            self._check(self.lib.cheb_filter(self.handle, X.data_ptr(), ldx, nb, int(m), float(c), float(r),
                                             ws.data_ptr(), ws.numel(), _stream()), "cheb_filter")
            return X
        self._check(self.lib.cheb_filter_carry(self.handle, X.data_ptr(), ldx, nb, int(m), float(c), float(r),
                                               self._proj(p_in, nb), self._local(hx_in, nb), ws.data_ptr(),
                                               ws.numel(), _stream()), "cheb_filter_carry")
        return X

    def projections(self, nb: int) -> torch.Tensor:
        """A device buffer for the projections of nb bands (complex128 (nb, nproj)) that rayleigh_ritz returns
        and filter takes."""
        return torch.zeros((nb, max(self.nproj, 1)), dtype=torch.complex128, device=self.device)

    def _proj(self, t, nb):
        if t is None:
            return None
        if (t.dtype != torch.complex128 or t.device.type != "cuda" or not t.is_contiguous() or t.dim() != 2
                or t.shape[0] != nb or t.shape[1] < self.nproj):
            raise ValueError(f"projections must be a contiguous complex128 ({nb}, {self.nproj}) device tensor")
        if self.nproj > 0 and t.shape[1] != self.nproj:
            raise ValueError(f"projections must have {self.nproj} columns")
        return t.data_ptr()

    def _local(self, t, nb):
        if t is None:
            return None
        if t.dtype != self.dtype or t.device.type != "cuda" or not t.is_contiguous() or tuple(t.shape) != (nb, self.npw):
            raise ValueError(f"(K + V) X must be a contiguous {self.dtype} ({nb}, {self.npw}) device tensor")
        return t.data_ptr()

    def filter_degrees(self, X, degrees, c: float, r: float):
        """Per-band degrees (locking): X[b] <- T_{degrees[b]}((S^-1 H - c)/r) X[b]; degree 0 leaves a band as is."""
        nb, ldx = self._block(X, "X")
        deg = np.ascontiguousarray(degrees, dtype=np.int32)
        if deg.shape != (nb,):
            raise ValueError(f"degrees must have shape ({nb},), got {deg.shape}")
        ws = self.workspace(CHEB_OP_FILTER_DEGREES, nb)
        self._check(self.lib.cheb_filter_degrees(self.handle, X.data_ptr(), ldx, nb, deg.ctypes.data, float(c),
                                                 float(r), ws.data_ptr(), ws.numel(), _stream()),
                    "cheb_filter_degrees")
        return X

    def rayleigh_ritz(self, X, with_residuals: bool = True, p_out=None, hx_out=None):
        """In-place Rayleigh-Ritz; returns (Ritz values, residual norms or None). p_out: None, or a complex128
        (nb, nproj) device tensor that receives the projections P^H X of the rotated block; hx_out: None, or an
        (nb, npw) device tensor of the plan's dtype that receives (K + V) X of the rotated block (see
        cheb_rayleigh_ritz_carry)."""
        nb, ldx = self._block(X, "X")
        ritz = torch.empty(nb, dtype=torch.float64, device=self.device)
        res = torch.empty(nb, dtype=torch.float64, device=self.device) if with_residuals else None
        ws = self.workspace(CHEB_OP_RR, nb)
        if p_out is None and hx_out is None:
            self._check(self.lib.cheb_rayleigh_ritz(self.handle, X.data_ptr(), ldx, nb, ritz.data_ptr(), _ptr(res),
                                                    ws.data_ptr(), ws.numel(), _stream()), "cheb_rayleigh_ritz")
        else:
            self._check(self.lib.cheb_rayleigh_ritz_carry(self.handle, X.data_ptr(), ldx, nb, ritz.data_ptr(),
                                                          _ptr(res), self._proj(p_out, nb), self._local(hx_out, nb),
                                                          ws.data_ptr(), ws.numel(), _stream()),
                        "cheb_rayleigh_ritz_carry")
        return ritz, res

    def rayleigh_quotients(self, X):
        nb, ldx = self._block(X, "X")
        rq = torch.empty(nb, dtype=torch.float64, device=self.device)
        ws = self.workspace(CHEB_OP_RR, nb)
        self._check(self.lib.cheb_rayleigh_quotients(self.handle, X.data_ptr(), ldx, nb, rq.data_ptr(),
                                                     ws.data_ptr(), ws.numel(), _stream()), "cheb_rayleigh_quotients")
        return rq

    def upper_bound(self, v0: torch.Tensor, k: int = 10) -> float:
        v0 = v0.to(self.device, self.dtype).contiguous()
        assert v0.numel() == self.npw
        ws = self.workspace(CHEB_OP_BOUND, 1)
        out = ctypes.c_double()
        self._check(self.lib.cheb_upper_bound(self.handle, int(k), v0.data_ptr(), ctypes.byref(out), ws.data_ptr(),
                                              ws.numel(), _stream()), "cheb_upper_bound")
        return out.value


    def filter_rr_backward(self, X0, m: int, c: float, r: float, w, ckpt_every: int = 3):
        """Forward filter + Rayleigh-Ritz and the adjoint of L = sum_i w_i lambda_i (lowest len(w) Ritz values).
        Returns (ritz, dX, dV, dD) with dL = 2 Re tr(dX^H dX0), dV (n, n, n) FP64, dD packed FP64."""
        nb, ldx = self._block(X0, "X0")
        w = torch.as_tensor(w, dtype=torch.float64).to(self.device).contiguous()
        nk = int(w.numel())
        nbytes = ctypes.c_size_t()
        self._check(self.lib.cheb_backward_workspace_bytes(self.handle, nb, int(m), int(ckpt_every),
                                                           ctypes.byref(nbytes)), "cheb_backward_workspace_bytes")
        key = ("bwd", nb, int(m), int(ckpt_every))
        if key not in self._ws:
            self._ws = {k: v for k, v in self._ws.items() if k[0] != "bwd"}
            self._ws[key] = torch.empty(max(nbytes.value, 256), dtype=torch.uint8, device=self.device)
        ws = self._ws[key]
        ritz = torch.empty(nb, dtype=torch.float64, device=self.device)
        dX = torch.empty_like(X0)
        dV = torch.empty((self.n,) * 3, dtype=torch.float64, device=self.device)
        dsize = int(sum((int(self._off[a + 1]) - int(self._off[a])) ** 2 for a in range(self.natom)))
        dD = torch.empty(max(dsize, 1), dtype=torch.float64, device=self.device)
        self._check(self.lib.cheb_filter_rr_backward(
            self.handle, X0.data_ptr(), ldx, nb, int(m), float(c), float(r), nk, w.data_ptr(), int(ckpt_every),
            ritz.data_ptr(), dX.data_ptr(), dX.stride(0), dV.data_ptr(), dD.data_ptr() if dsize else None,
            ws.data_ptr(), ws.numel(), _stream()), "cheb_filter_rr_backward")
        return ritz, dX, dV, dD[:dsize]

    def set_split_gemm(self, on: bool):
        """Mixed plans: FP16 hi/lo split MFMA (True, default) or FP32 MFMA (False) for the projector GEMMs."""
        self._check(self.lib.cheb_set_split_gemm(self.handle, int(bool(on))), "cheb_set_split_gemm")

    def set_projection_resync(self, period: int):
        """Recompute the carried projections P^H psi from the vectors every `period` filter steps (0: never)."""
        self._check(self.lib.cheb_set_projection_resync(self.handle, int(period)), "cheb_set_projection_resync")

    def drift_monitor(self, on: bool = True):
        """Measure the drift of the carried projections before every filter step (synchronizing diagnostic)."""
        self._check(self.lib.cheb_drift_monitor(self.handle, int(bool(on))), "cheb_drift_monitor")

    def drift_read(self) -> tuple[float, int]:
        """(largest relative drift ||p_carried - P^H psi|| / ||P^H psi|| seen, steps checked) since drift_monitor."""
        mx, n = ctypes.c_double(), ctypes.c_int64()
        self._check(self.lib.cheb_drift_read(self.handle, ctypes.byref(mx), ctypes.byref(n)), "cheb_drift_read")
        return mx.value, n.value

    def set_rr_refine(self, on: bool):
        self._check(self.lib.cheb_set_rr_refine(self.handle, int(bool(on))), "cheb_set_rr_refine")

    def rr_stats(self) -> tuple[int, int]:
        """(Rayleigh-Ritz calls solved by the warm-started refinement, calls solved by the library path)."""
        a, b = ctypes.c_int64(), ctypes.c_int64()
        self._check(self.lib.cheb_rr_stats(self.handle, ctypes.byref(a), ctypes.byref(b)), "cheb_rr_stats")
        return a.value, b.value

    def profile_enable(self, on: bool = True):
        self._check(self.lib.cheb_profile_enable(self.handle, int(bool(on))), "cheb_profile_enable")

    def profile_read(self) -> dict:
        """{timer name: dict(ms, launches, bytes, flops)} since the last profile_enable(True)."""
        out = {}
        for k, name in enumerate(TIMERS):
            ms, n, b, f = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
            self._check(self.lib.cheb_profile_read(self.handle, k, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(b),
                                                   ctypes.byref(f)), "cheb_profile_read")
            out[name] = dict(ms=ms.value, launches=n.value, bytes=b.value, flops=f.value)
        return out


def plan_from_problem(pb, prec: int = CHEB_FP64, device: str = "cuda") -> Plan:
    """Plan + potential + projectors + D for a workload.Problem, or a workload.GammaProblem (half-sphere basis,
    Gamma plan), with the inputs copied to the device."""
    gamma = hasattr(pb, "half")
    full = pb.full if gamma else pb
    plan = Plan(pb.gidx, pb.kin, pb.cfg.n, full.proj_off, full.Q is not None, prec=prec, device=device, gamma=gamma)
    plan.set_potential(torch.from_numpy(np.ascontiguousarray(full.V)))
    P = torch.from_numpy(np.ascontiguousarray(pb.P.T))  # (nproj, npw): row j = projector j
    Q = None if full.Q is None else torch.from_numpy(full.Q)
    plan.set_projectors(P, Q)
    plan.set_D(torch.from_numpy(full.D_packed))
    return plan


def to_device_block(X: np.ndarray, dtype, device="cuda") -> torch.Tensor:
    """(npw, nb) numpy block -> (nb, npw) contiguous device tensor."""
    return torch.from_numpy(np.ascontiguousarray(X.T)).to(device=device, dtype=dtype)


def to_host_block(Xt: torch.Tensor) -> np.ndarray:
    return Xt.detach().to("cpu", torch.complex128).numpy().T.copy()
