"""Seeded synthetic workloads for the plane-wave generalized eigenproblem H x = lambda S x.

The paper's test systems (a BaTiO3 cell near 7000 plane waves with 100-200 bands, a 256-atom Ti
crystal with 2048 bands, Sec. 6.1-6.2) come from PAW datasets that are not available, so this module
draws problems of the same shapes: a plane-wave sphere (Sec. 2.1), a local potential made of Gaussian
wells, Gaussian-radial projectors with real harmonics and a structure factor (the matrix P of Eq. 3),
block-diagonal D (Eq. 3) and diagonal overlap coefficients Q (Eq. 4), and a random start block.

This module holds no arithmetic of the eigensolver itself: it only draws inputs. Both the HIP path and
the CPU oracle consume what it returns, and neither is imported here.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass

import numpy as np

BASE_SEED = 14064350


@dataclass(frozen=True)
class Config:
    """Shape and draw recipe of one synthetic problem."""

    name: str
    n: int            # cubic FFT box side (grid points)
    radius: int       # sphere radius in grid units: |g| <= radius (inclusive)
    cell: float       # cubic cell side L in bohr
    lattice: str      # 'random', 'fcc', 'bcc', 'sc'
    cells: int        # conventional cells per side (ignored for 'random')
    natom: int
    channels: str     # projector composition per atom: 'sp' (4), '2s2p' (8), '2s2p1d' (13)
    overlap: bool     # True: S = I + P Q P^H (PAW); False: S = I (norm-conserving)
    nb: int           # bands
    m: int            # Chebyshev degree
    iters: int        # outer iterations used by the driver
    nk: int           # Ritz values entering the loss of the differentiation form
    seed_index: int   # seed = BASE_SEED + seed_index

    def replace(self, **kw) -> "Config":
        return dataclasses.replace(self, **kw)


CHANNELS = {"sp": 4, "2s2p": 8, "2s2p1d": 13}

# The five named workloads. Their shapes follow the paper's systems where it gives them:
# Npw ~ 7000 with 100-200 bands (Sec. 6.1), 256 atoms with 2048 bands (Sec. 6.2), 1-40 projectors
# per atom (Sec. 2.1), n_inner = 4 by default (Sec. 5.3).
CONFIGS = {c.name: c for c in (
    Config("nc16", 16, 4, 10.0, "random", 1, 2, "sp", False, 16, 4, 20, 8, 1),
    Config("paw48", 48, 12, 12.0, "fcc", 2, 32, "2s2p", True, 256, 8, 20, 128, 2),
    Config("paw96", 96, 24, 24.0, "bcc", 4, 128, "2s2p1d", True, 1024, 10, 50, 512, 3),
    Config("paw64", 64, 16, 16.0, "sc", 4, 64, "2s2p", True, 512, 8, 1, 256, 4),
    Config("paw128", 128, 32, 32.0, "fcc", 4, 256, "2s2p1d", True, 2048, 12, 3, 1024, 5),
)}

# Small problems for parity tests: several GEMM / FFT tiles and ragged tails, oracle-friendly.
SMALL = {
    "tiny_paw": Config("tiny_paw", 16, 4, 10.0, "random", 1, 3, "2s2p", True, 24, 4, 12, 12, 101),
    "mid_paw": Config("mid_paw", 24, 6, 8.0, "random", 1, 5, "2s2p1d", True, 40, 6, 8, 20, 102),
    "mid_nc": Config("mid_nc", 32, 8, 9.0, "sc", 2, 8, "2s2p", False, 70, 5, 6, 35, 103),
}


@dataclass
class Problem:
    cfg: Config
    gidx: np.ndarray      # (npw, 3) int32 Miller indices, sorted by (gx, gy) column then gz
    kin: np.ndarray       # (npw,) float64 kinetic diagonal, Hartree
    atoms: np.ndarray     # (natom, 3) positions, bohr
    V: np.ndarray         # (n, n, n) float64 local potential on r_j = L j / n, [x][y][z] C-order
    P: np.ndarray         # (npw, nproj) complex128, Fortran order (each projector contiguous)
    proj_off: np.ndarray  # (natom + 1,) int32; atom a owns projector columns [off[a], off[a+1])
    D: list               # natom real symmetric blocks (n_lmn x n_lmn)
    Q: np.ndarray | None  # (nproj,) float64 overlap coefficients, or None when S = I
    X0: np.ndarray        # (npw, nb) complex128, Fortran order
    v0: np.ndarray        # (npw,) complex128 Lanczos start vector
    w: np.ndarray         # (nk,) float64 loss weights
    dV: np.ndarray        # (ndir, n, n, n) float64 potential directions (differentiation form)

    @property
    def npw(self) -> int:
        return self.gidx.shape[0]

    @property
    def nproj(self) -> int:
        return self.P.shape[1]

    @property
    def D_packed(self) -> np.ndarray:
        """Blocks concatenated, each row-major."""
        return np.concatenate([d.ravel() for d in self.D]).astype(np.float64)


def sphere(radius: int) -> np.ndarray:
    """All integer g with |g|^2 <= radius^2, sorted lexicographically by (gx, gy, gz)."""
    r = np.arange(-radius, radius + 1)
    gx, gy, gz = np.meshgrid(r, r, r, indexing="ij")
    g = np.stack([gx.ravel(), gy.ravel(), gz.ravel()], axis=1)
    keep = (g * g).sum(axis=1) <= radius * radius
    return np.ascontiguousarray(g[keep]).astype(np.int32)  # meshgrid 'ij' order is already lexicographic


def _atoms(cfg: Config, rng: np.random.Generator) -> np.ndarray:
    L = cfg.cell
    if cfg.lattice == "random":
        return rng.uniform(0.0, L, size=(cfg.natom, 3))
    basis = {
        "sc": [(0, 0, 0)],
        "bcc": [(0, 0, 0), (0.5, 0.5, 0.5)],
        "fcc": [(0, 0, 0), (0, 0.5, 0.5), (0.5, 0, 0.5), (0.5, 0.5, 0)],
    }[cfg.lattice]
    k = cfg.cells
    a = L / k
    pos = []
    for i in range(k):
        for j in range(k):
            for l in range(k):
                for b in basis:
                    pos.append(((i + b[0]) * a, (j + b[1]) * a, (l + b[2]) * a))
    pos = np.array(pos, dtype=np.float64)
    if pos.shape[0] != cfg.natom:
        raise ValueError(f"{cfg.name}: lattice gives {pos.shape[0]} atoms, config says {cfg.natom}")
    pos += rng.uniform(-0.05, 0.05, size=pos.shape) * a
    return np.mod(pos, L)


def _potential(cfg: Config, atoms: np.ndarray, rng: np.random.Generator) -> np.ndarray:
    """Sum of Gaussian wells, one per atom, minimum-image distance in the cubic cell."""
    n, L = cfg.n, cfg.cell
    depth = rng.uniform(1.0, 3.0, size=cfg.natom)
    width = rng.uniform(0.5, 1.0, size=cfg.natom)
    x = L * np.arange(n) / n
    V = np.zeros((n, n, n))
    for a in range(cfg.natom):
        e = []
        for d in range(3):
            dx = x - atoms[a, d]
            dx -= L * np.round(dx / L)
            e.append(np.exp(-dx * dx / (2.0 * width[a] ** 2)))
        V -= depth[a] * e[0][:, None, None] * e[1][None, :, None] * e[2][None, None, :]
    return V


def _projectors(cfg: Config, gidx: np.ndarray, atoms: np.ndarray, real_space_real: bool = False):
    """Columns f_n(|G|) Y_lm(G/|G|) exp(-i G.R_a), each normalised to unit 2-norm. real_space_real: times
    (-i)^l, which makes every projector a real function in real space (P(-G) = conj P(G))."""
    L = cfg.cell
    G = (2.0 * np.pi / L) * gidx.astype(np.float64)
    G2 = (G * G).sum(axis=1)
    Gn = np.sqrt(G2)
    safe = np.where(Gn > 0, Gn, 1.0)
    u = G / safe[:, None]
    u[Gn == 0] = 0.0
    ux, uy, uz = u[:, 0], u[:, 1], u[:, 2]
    rad = [np.exp(-G2 / 4.0), np.exp(-G2 / 8.0)]
    s = np.ones_like(G2)
    p = [ux, uy, uz]
    d = [ux * uy, uy * uz, uz * ux, 0.5 * (ux * ux - uy * uy), (3.0 * uz * uz - 1.0) / (2.0 * np.sqrt(3.0))]
    d = [di if k < 4 else np.where(Gn > 0, di, 0.0) for k, di in enumerate(d)]
    shapes = {
        "sp": [rad[0] * s] + [rad[0] * c for c in p],
        "2s2p": [rad[0] * s, rad[1] * s] + [rad[0] * c for c in p] + [rad[1] * c for c in p],
        "2s2p1d": [rad[0] * s, rad[1] * s] + [rad[0] * c for c in p] + [rad[1] * c for c in p]
        + [rad[0] * c for c in d],
    }[cfg.channels]
    ells = {"sp": [0, 1, 1, 1], "2s2p": [0, 0] + [1] * 6, "2s2p1d": [0, 0] + [1] * 6 + [2] * 5}[cfg.channels]
    if real_space_real:
        shapes = [f * (-1j) ** l for f, l in zip(shapes, ells)]
    nl = len(shapes)
    npw = gidx.shape[0]
    P = np.empty((npw, cfg.natom * nl), dtype=np.complex128, order="F")
    for a in range(cfg.natom):
        sf = np.exp(-1j * (G @ atoms[a]))
        for k, f in enumerate(shapes):
            col = f * sf
            P[:, a * nl + k] = col / np.linalg.norm(col)
    off = (np.arange(cfg.natom + 1) * nl).astype(np.int32)
    return P, off


def config(cfg: Config | str) -> Config:
    """A Config, or the one named: a workload of CONFIGS or a small problem of SMALL."""
    if isinstance(cfg, Config):
        return cfg
    return CONFIGS[cfg] if cfg in CONFIGS else SMALL[cfg]


def make_problem(cfg: Config | str, nb: int | None = None, ndir: int = 0) -> Problem:
    """Draw the problem for a named workload (CONFIGS or SMALL) or a Config."""
    cfg = config(cfg)
    if nb is not None:
        cfg = cfg.replace(nb=nb)
    if cfg.n < 2 * cfg.radius + 1:
        raise ValueError("FFT box too small for the sphere")
    ss = np.random.SeedSequence(BASE_SEED + cfg.seed_index)
    kids = ss.spawn(8)  # atoms, wells, D, Q, X0, Lanczos v0, loss weights, dV directions
    rng = [np.random.Generator(np.random.PCG64(k)) for k in kids]

    gidx = sphere(cfg.radius)
    G = (2.0 * np.pi / cfg.cell) * gidx.astype(np.float64)
    kin = 0.5 * (G * G).sum(axis=1)
    atoms = _atoms(cfg, rng[0])
    V = _potential(cfg, atoms, rng[1])
    P, off = _projectors(cfg, gidx, atoms)
    nl = CHANNELS[cfg.channels]
    D = []
    for _ in range(cfg.natom):
        a = rng[2].normal(0.0, 0.5, size=(nl, nl))
        a = np.triu(a)
        D.append(a + np.triu(a, 1).T)
    Q = rng[3].uniform(0.1, 0.5, size=cfg.natom * nl) if cfg.overlap else None
    npw = gidx.shape[0]
    X0 = np.asfortranarray(rng[4].normal(size=(npw, cfg.nb)) + 1j * rng[4].normal(size=(npw, cfg.nb)))
    v0 = rng[5].normal(size=npw) + 1j * rng[5].normal(size=npw)
    w = rng[6].uniform(0.0, 1.0, size=cfg.nk)
    dV = rng[7].normal(size=(ndir, cfg.n, cfg.n, cfg.n)) if ndir else np.zeros((0, cfg.n, cfg.n, cfg.n))
    return Problem(cfg, gidx, kin, atoms, V, P, off, D, Q, X0, v0, w, dV)


def free_electron(cfg: Config | str, nb: int | None = None) -> Problem:
    """Same basis and start block, with V = 0 and no projectors (S = I)."""
    pb = make_problem(cfg, nb=nb)
    natom = pb.cfg.natom
    cfg0 = pb.cfg.replace(overlap=False)
    return Problem(cfg0, pb.gidx, pb.kin, pb.atoms, np.zeros_like(pb.V),
                   np.zeros((pb.npw, 0), dtype=np.complex128, order="F"),
                   np.zeros(natom + 1, dtype=np.int32), [np.zeros((0, 0)) for _ in range(natom)],
                   None, pb.X0, pb.v0, pb.w, pb.dV)


# --- Gamma point (real wavefunctions, Sec. 2.1) -----------------------------------------------------------------
def half_sphere_mask(gidx: np.ndarray) -> np.ndarray:
    """G in the half sphere H+: gx > 0, or gx = 0 and gy > 0, or gx = gy = 0 and gz >= 0. Every G != 0 of the
    sphere has exactly one of G, -G in H+; whole (gx, gy) columns belong to H+ except the column (0, 0)."""
    gx, gy, gz = gidx[:, 0], gidx[:, 1], gidx[:, 2]
    return (gx > 0) | ((gx == 0) & (gy > 0)) | ((gx == 0) & (gy == 0) & (gz >= 0))


@dataclass
class GammaProblem:
    """A problem with real wavefunctions: projectors real in real space, so H and S map real functions to real
    functions. Vectors are stored on the half sphere H+ as the coefficients of an orthonormal real basis:
    sqrt(2) c_G for G != 0 and the real c_0 at G = 0 (c_-G = conj c_G fills the other half). `full` is the
    same problem on the whole sphere (its X0, v0 are the expansions of the Gamma ones)."""

    full: Problem
    half: np.ndarray     # (nh,) indices of H+ in full.gidx (sphere order)
    gidx: np.ndarray     # (nh, 3)
    kin: np.ndarray      # (nh,)
    P: np.ndarray        # (nh, nproj) scaled like the vectors (Fortran order)
    X0: np.ndarray       # (nh, nb) scaled coefficients, imaginary part 0 at G = 0
    v0: np.ndarray       # (nh,)

    @property
    def npw(self) -> int:
        return self.gidx.shape[0]

    @property
    def nproj(self) -> int:
        return self.P.shape[1]

    @property
    def cfg(self) -> Config:
        return self.full.cfg


def make_gamma_problem(cfg: Config | str, nb: int | None = None) -> GammaProblem:
    """The problem of make_problem with real-space-real projectors ((-i)^l factor) and real start vectors."""
    pb = make_problem(cfg, nb=nb)
    cfg = pb.cfg
    P, off = _projectors(cfg, pb.gidx, pb.atoms, real_space_real=True)
    half = np.nonzero(half_sphere_mask(pb.gidx))[0]
    zero = np.all(pb.gidx[half] == 0, axis=1)
    scale = np.where(zero, 1.0, np.sqrt(2.0))
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(BASE_SEED + cfg.seed_index).spawn(9)[8]))
    nh = half.shape[0]
    X0 = rng.normal(size=(nh, cfg.nb)) + 1j * rng.normal(size=(nh, cfg.nb))
    X0[zero, :] = X0[zero, :].real
    v0 = rng.normal(size=nh) + 1j * rng.normal(size=nh)
    v0[zero] = v0[zero].real
    Ph = np.asfortranarray(P[half] * scale[:, None])
    # expansions of the Gamma vectors on the whole sphere, for the full problem
    pos = {tuple(g): i for i, g in enumerate(pb.gidx)}
    mirror = np.array([pos[tuple(-g)] for g in pb.gidx[half]])

    def expand(Y):
        Y = np.asarray(Y).reshape(nh, -1)
        out = np.zeros((pb.npw, Y.shape[1]), dtype=np.complex128)
        c = Y / scale[:, None]
        out[mirror] = np.conj(c)
        out[half] = c
        return out
    full = Problem(cfg, pb.gidx, pb.kin, pb.atoms, pb.V, P, off, pb.D, pb.Q, np.asfortranarray(expand(X0)),
                   expand(v0)[:, 0], pb.w, pb.dV)
    return GammaProblem(full, half, np.ascontiguousarray(pb.gidx[half]), pb.kin[half].copy(), Ph,
                        np.asfortranarray(X0), v0)
