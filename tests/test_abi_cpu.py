"""The C-ABI library loads, exports every function include/chebfd.h declares, and rejects bad descriptors
before touching the GPU (these calls make no HIP call, so they run without a GPU)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1406_4350_amd import chebfd as cf
from paper_1406_4350_amd import workload as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(cf.LIB_PATH):
        pytest.skip("libchebfd.so not built")
    return cf.load_library()


def header_functions():
    txt = open(os.path.join(ROOT, "include", "chebfd.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(cheb_[a-z_A-Z]+)\s*\(", txt)))


def test_header_symbols_exported(lib):
    names = header_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(cf.SYMBOLS)


def test_status_codes_match_header():
    txt = open(os.path.join(ROOT, "include", "chebfd.h")).read()
    body = re.search(r"typedef enum \{(.*?)\} cheb_status;", txt, flags=re.S).group(1)
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    codes = {k: int(v) for k, v in re.findall(r"(CHEB_\w+)\s*=\s*(\d+)", body)}
    assert "CHEB_ERR_HOST" in codes
    for k, v in codes.items():
        assert getattr(cf, k) == v, k
    assert cf.STATUS_NAMES == sorted(codes, key=codes.get)


def _desc(pb, n=None, gidx=None, off=None, prec=0):
    g = np.ascontiguousarray(pb.gidx if gidx is None else gidx, dtype=np.int32)
    k = np.ascontiguousarray(pb.kin[: g.shape[0]], dtype=np.float64)
    o = np.ascontiguousarray(pb.proj_off if off is None else off, dtype=np.int32)
    d = cf.cheb_desc(pb.cfg.n if n is None else n, g.shape[0], g.ctypes.data, k.ctypes.data, o.shape[0] - 1,
                     o.ctypes.data, int(pb.Q is not None), prec)
    return d, (g, k, o)


def _bytes(lib, d):
    out = ctypes.c_size_t()
    return lib.cheb_plan_persistent_bytes(ctypes.byref(d), ctypes.byref(out)), out.value


def test_valid_descriptor(lib):
    pb = wl.make_problem("tiny_paw")
    for prec in (cf.CHEB_FP64, cf.CHEB_MIXED):
        d, keep = _desc(pb, prec=prec)
        st, nbytes = _bytes(lib, d)
        assert st == cf.CHEB_OK
        # at least P, G, C^-1 and V(r) in the plan precision
        eb = 16 if prec == cf.CHEB_FP64 else 8
        assert nbytes >= pb.npw * pb.nproj * eb + 2 * 16 * pb.nproj**2 + pb.cfg.n**3 * eb // 2


def test_rejects_bad_descriptors(lib):
    pb = wl.make_problem("tiny_paw")
    d, keep = _desc(pb, n=20)
    assert _bytes(lib, d)[0] == cf.CHEB_ERR_ARG                    # unsupported box
    d, keep = _desc(pb, n=8)
    assert _bytes(lib, d)[0] == cf.CHEB_ERR_ARG                    # sphere does not fit the box
    g = pb.gidx.copy()
    g[[3, 40]] = g[[40, 3]]
    d, keep = _desc(pb, gidx=g)
    assert _bytes(lib, d)[0] == cf.CHEB_ERR_ARG                    # not column-sorted
    g = pb.gidx
    mid = next(e for e in range(1, len(g) - 1)
               if (g[e - 1, :2] == g[e, :2]).all() and (g[e + 1, :2] == g[e, :2]).all())
    g = np.delete(g, mid, axis=0)
    d, keep = _desc(pb, gidx=g)
    assert _bytes(lib, d)[0] == cf.CHEB_ERR_ARG                    # column with a gap in gz
    off = pb.proj_off.copy()
    off[1], off[2] = off[2], off[1]
    d, keep = _desc(pb, off=off)
    assert _bytes(lib, d)[0] == cf.CHEB_ERR_ARG                    # decreasing projector offsets
    d, keep = _desc(pb, prec=7)
    assert _bytes(lib, d)[0] == cf.CHEB_ERR_ARG                    # unknown precision
    out = ctypes.c_size_t()
    assert lib.cheb_plan_persistent_bytes(None, ctypes.byref(out)) == cf.CHEB_ERR_ARG


def test_create_rejects_missing_buffer(lib):
    pb = wl.make_problem("nc16")
    d, keep = _desc(pb)
    h = ctypes.c_void_p()
    assert lib.cheb_plan_create(ctypes.byref(d), None, 0, None, ctypes.byref(h)) == cf.CHEB_ERR_WORKSPACE
    assert not h.value


def test_workload_names_resolve():
    """Every workload is drawn by its name; names are unique across the full-size and the small tables."""
    assert not set(wl.CONFIGS) & set(wl.SMALL)
    for name, c in {**wl.CONFIGS, **wl.SMALL}.items():
        assert wl.config(name) is c and c.name == name
    assert wl.config(wl.CONFIGS["paw48"]) is wl.CONFIGS["paw48"]
    with pytest.raises(KeyError):
        wl.config("paw49")


def test_named_configs_validate(lib):
    """Every named workload fits the kernels' limits (LDS of the plane pass) in both precisions."""
    for cfg in wl.CONFIGS.values():
        g = wl.sphere(cfg.radius)
        kin = np.zeros(g.shape[0])
        nl = wl.CHANNELS[cfg.channels]
        off = (np.arange(cfg.natom + 1) * nl).astype(np.int32)
        for prec in (cf.CHEB_FP64, cf.CHEB_MIXED):
            d = cf.cheb_desc(cfg.n, g.shape[0], g.ctypes.data, kin.ctypes.data, cfg.natom, off.ctypes.data,
                             int(cfg.overlap), prec)
            out = ctypes.c_size_t()
            assert lib.cheb_plan_persistent_bytes(ctypes.byref(d), ctypes.byref(out)) == cf.CHEB_OK, (cfg.name, prec)


def test_locking_degrees_host_function(lib):
    """cheb_locking_degrees (host arithmetic only) picks the same degree per band as the oracle's rule
    (Eq. 5, Sec. 5.4), on random residuals spread over many decades and Ritz values inside and below the
    damped interval; and it rejects bad arguments."""
    from oracle import matfree
    rng = np.random.default_rng(7)
    nb, c, r, m, tol = 500, 3.0, 2.0, 12, 1e-7
    ritz = rng.uniform(-6.0, 5.5, nb)
    resid = 10.0 ** rng.uniform(-10, 1, nb)
    deg, nlocked = cf.locking_degrees(ritz, resid, c, r, m, tol)
    ref = matfree.locking_degrees(resid, ritz, c, r, m, tol)
    assert np.array_equal(deg, ref)
    assert nlocked == int((resid <= tol).sum()) and nlocked > 0
    assert (deg == m).sum() > 0 and ((deg > 0) & (deg < m)).sum() > 0
    with pytest.raises(cf.ChebError):
        cf.locking_degrees(ritz, resid, c, -1.0, m, tol)
    with pytest.raises(cf.ChebError):
        cf.locking_degrees(ritz, resid, c, r, 0, tol)
    bad = resid.copy()
    bad[3] = np.nan
    with pytest.raises(cf.ChebError):
        cf.locking_degrees(ritz, bad, c, r, m, tol)
    assert cf.locking_degrees(ritz[:0], resid[:0], c, r, m, tol)[0].shape == (0,)


def test_gemm_split_bound_covers_both_kernels(lib):
    """Split-K partial buffers hold bound x M x N values: the bound must cover the split count either GEMM
    kernel picks, for every shape (host arithmetic of the C ABI, no GPU). Shapes around the tile sizes (64, 16)
    and K tiles (32), the paw48 projector and subspace shapes and large K."""
    f64, f16, bd = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    mn = [1, 2, 15, 16, 17, 63, 64, 65, 127, 128, 129, 200, 255, 256, 257, 300, 448, 511, 512, 513, 1000, 2109, 7153]
    ks = [1, 2, 3, 16, 31, 32, 33, 63, 64, 65, 100, 256, 257, 1000, 1024, 1025, 2109, 7153, 20000, 137065]
    for M in mn:
        for N in mn:
            for K in ks:
                assert lib.cheb_gemm_splits(M, N, K, ctypes.byref(f64), ctypes.byref(f16), ctypes.byref(bd)) == cf.CHEB_OK
                assert 1 <= f64.value <= 32 and 1 <= f16.value <= 64, (M, N, K, f64.value, f16.value)
                # the FP16 kernel's FP32 accumulators never sum more than 4096 products of K in sequence
                assert f16.value >= -(-K // 4096), (M, N, K, f16.value)
                assert bd.value >= max(f64.value, f16.value), (M, N, K, f64.value, f16.value, bd.value)
    assert lib.cheb_gemm_splits(4, 4, 4, None, ctypes.byref(f16), ctypes.byref(bd)) == cf.CHEB_ERR_ARG


def _grouped_item(bx, by, bz, tm, tn, group=8):
    """Position of work item (split bz, M tile bx, N tile by) in the grouped order: split by split, groups of
    `group` M tiles, the M tile fastest inside a group."""
    first = (bx // group) * group
    gm = min(group, tm - first)
    return bz * tm * tn + first * tn + by * gm + (bx - first)


def test_gemm_block_item_is_a_bijection_with_one_run_per_xcd(lib):
    """Block i of a tiled GEMM launch takes work item (split, M tile, N tile) so that every item is taken once
    and the blocks dealt to each of the 8 XCDs (i mod 8) hold one contiguous run of the grouped order (groups of
    `group` M tiles, M tile fastest inside a group; group 1 is the N tile fastest), so that the blocks an XCD
    holds at once share slices of A and B (host arithmetic)."""
    bx, by, bz = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    for group in (1, 8, 3):
        for tm, tn, s in [(1, 1, 1), (1, 1, 7), (2, 3, 1), (4, 4, 16), (7, 5, 3), (112, 4, 1), (4, 4, 32), (9, 9, 2),
                          (3, 1, 13), (16, 16, 1), (26, 16, 40), (52, 32, 4), (17, 3, 2)]:
            total = tm * tn * s
            seen = {}
            for i in range(total):
                assert lib.cheb_gemm_block_item(i, total, tm, tn, group, ctypes.byref(bx), ctypes.byref(by),
                                                ctypes.byref(bz)) == 0
                assert 0 <= bx.value < tm and 0 <= by.value < tn and 0 <= bz.value < s
                seen[i] = _grouped_item(bx.value, by.value, bz.value, tm, tn, group)
            assert sorted(seen.values()) == list(range(total))
            for x in range(8):
                items = sorted(seen[i] for i in range(x, total, 8))
                assert items == list(range(items[0], items[0] + len(items))) if items else True, (tm, tn, s, x)
    # group 1 is the plain order (split, M tile, N tile) with the N tile fastest
    for i in range(7 * 5 * 3):
        lib.cheb_gemm_block_item(i, 105, 7, 5, 1, ctypes.byref(bx), ctypes.byref(by), ctypes.byref(bz))
        assert _grouped_item(bx.value, by.value, bz.value, 7, 5, 1) == (bz.value * 7 + bx.value) * 5 + by.value
    # with group 8, the first 64 items of a large split (XCD 0's first blocks) cover 8 M tiles by 8 N tiles
    tm, tn, total = 52, 32, 52 * 32 * 4
    patch = set()
    for i in range(0, 8 * 64, 8):
        lib.cheb_gemm_block_item(i, total, tm, tn, 8, ctypes.byref(bx), ctypes.byref(by), ctypes.byref(bz))
        patch.add((bx.value, by.value))
    assert {b for b, _ in patch} == set(range(8)) and {c for _, c in patch} == set(range(8))
    assert lib.cheb_gemm_block_item(5, 5, 1, 1, 1, ctypes.byref(bx), ctypes.byref(by), ctypes.byref(bz)) == cf.CHEB_ERR_ARG
    assert lib.cheb_gemm_block_item(0, 7, 2, 2, 1, ctypes.byref(bx), ctypes.byref(by), ctypes.byref(bz)) == cf.CHEB_ERR_ARG
    assert lib.cheb_gemm_block_item(0, 4, 2, 2, 0, ctypes.byref(bx), ctypes.byref(by), ctypes.byref(bz)) == cf.CHEB_ERR_ARG


def test_gemm_upper_triangle_items(lib):
    """group -1 (the Hermitian Rayleigh-Ritz products): the blocks of a launch take every tile bx <= by of a square
    tm x tm grid once per split and no tile below the diagonal, column by column inside a split, each XCD (i mod 8)
    one contiguous run (host arithmetic)."""
    bx, by, bz = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    for tm, s in [(1, 1), (1, 5), (2, 1), (3, 4), (7, 3), (32, 8), (33, 2), (64, 1), (5, 13)]:
        per = tm * (tm + 1) // 2
        total = per * s
        order = {}
        for i in range(total):
            assert lib.cheb_gemm_block_item(i, total, tm, tm, -1, ctypes.byref(bx), ctypes.byref(by),
                                            ctypes.byref(bz)) == 0
            assert 0 <= bx.value <= by.value < tm and 0 <= bz.value < s
            order[i] = bz.value * per + by.value * (by.value + 1) // 2 + bx.value
        assert sorted(order.values()) == list(range(total)), (tm, s)
        for x in range(8):
            items = sorted(order[i] for i in range(x, total, 8))
            assert not items or items == list(range(items[0], items[0] + len(items))), (tm, s, x)
    # tn must equal tm and total be a multiple of the tiles per split
    assert lib.cheb_gemm_block_item(0, 6, 3, 2, -1, ctypes.byref(bx), ctypes.byref(by), ctypes.byref(bz)) == cf.CHEB_ERR_ARG
    assert lib.cheb_gemm_block_item(0, 7, 3, 3, -1, ctypes.byref(bx), ctypes.byref(by), ctypes.byref(bz)) == cf.CHEB_ERR_ARG
    assert lib.cheb_gemm_block_item(0, 9, 3, 3, -2, ctypes.byref(bx), ctypes.byref(by), ctypes.byref(bz)) == cf.CHEB_ERR_ARG


def test_stability_factor_closed_form():
    """The driver's |T_m(x)| (the amplification logged per outer iteration, Sec. 5.3) against the oracle's closed
    form, inside and outside [-1, 1], and at the overflow guard."""
    import numpy as np

    from oracle import dense
    from paper_1406_4350_amd.driver import chebyshev_magnitude

    for m in (0, 1, 4, 8, 12):
        for x in (-3.0, -1.2, -1.0, -0.4, 0.3, 1.0, 2.5):
            ref = abs(float(dense.chebyshev_T(m, np.array([x]))[0]))
            assert abs(chebyshev_magnitude(m, x) - ref) <= 1e-12 * max(1.0, ref)
    assert chebyshev_magnitude(400, -9.0) == float("inf")
