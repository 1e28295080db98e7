"""Host logic of bench.py's roofline report (no GPU): the roofline of each timer class, the choice of the
dominant class, and the lookup of measured HBM bytes keyed by kernel, box size and source hash."""
import hashlib
import json
import os

import pytest

import bench


def _cls(ms, launches, bytes_=0.0, flops=0.0):
    return {"ms": ms, "launches": launches, "bytes": bytes_, "flops": flops}


def test_gemm_class_against_the_mfma_peak_of_its_arithmetic():
    d = _cls(ms=100.0, launches=10, flops=10 * 7.0e11)  # 7e11 flops per 10 ms launch = 70 TFLOP/s
    r = bench.class_roofline("project", d, "f64", 128)
    assert r["bound"] == "mfma" and r["mfma_dtype"] == "f64" and r["peak"] == 78.6
    assert r["achieved"] == pytest.approx(70.0)
    assert r["frac"] == pytest.approx(70.0 / 78.6)
    assert r["kernel"] == "k_gemm<double, double, double, double, 0, 1>"
    assert r["executed_frac"] == pytest.approx(0.75 * 70.0 / 78.6)  # three real products per complex one
    assert bench.class_roofline("project", d, "f32", 128)["executed_frac"] == pytest.approx(3 * 70.0 / 2500.0)
    # mixed plans: the split projector products against the FP16 MFMA peak, the Grams against FP64
    assert bench.class_roofline("project", d, "f32", 128)["peak"] == 2500.0
    assert bench.class_roofline("rr_gram", d, "f32", 128)["peak"] == 78.6


def test_fft_classes_bound_by_the_closer_roofline():
    # a column pass: bytes only, HBM bound
    col = bench.class_roofline("fft_col_inverse", _cls(ms=1.0, launches=10, bytes_=10 * 4.0e8), "f64", 96)
    assert col["bound"] == "hbm" and col["achieved"] == pytest.approx(4000.0)  # 4e8 B per 0.1 ms
    assert col["kernel"] == "k_col_inv<96, double>"
    # the plane pass: 1 % of HBM but 20 % of the FP64 vector peak -> ALU bound, with the HBM figures kept
    d = _cls(ms=1.0, launches=1, bytes_=0.08e9, flops=15.72e9)
    r = bench.class_roofline("fft_plane", d, "f64", 48)
    assert r["bound"] == "alu" and r["unit"] == "TFLOP/s"
    assert r["achieved"] == pytest.approx(15.72) and r["frac"] == pytest.approx(0.2)
    assert r["hbm"]["frac"] == pytest.approx(0.01)
    assert r["algo_per_launch"] == pytest.approx(15.72e9)
    # the other way round it stays HBM bound
    d2 = _cls(ms=1.0, launches=1, bytes_=4.0e9, flops=1.0e9)
    assert bench.class_roofline("fft_plane", d2, "f64", 48)["bound"] == "hbm"
    # the FP64 plane pass at 128^3 is the halved kernel
    assert bench.class_roofline("fft_plane", d, "f64", 128)["kernel"] == "k_plane_half"
    assert bench.class_roofline("fft_plane", d, "f32", 128)["kernel"] == "k_plane<128, float>"


def test_dominant_class_leaves_out_the_library_eigensolver():
    prof = {"project": _cls(50.0, 5, flops=5 * 1e11), "rr_eig": _cls(500.0, 2), "fft_plane": _cls(20.0, 9, 9e8),
            "small": _cls(0.0, 0)}
    r = bench.roofline(prof, "f64", 64)
    assert r["kernel_class"] == "project"
    assert set(r["by_class"]) == {"project", "fft_plane"}


def test_traffic_lookup_checks_box_size_and_source(tmp_path, monkeypatch):
    csrc = tmp_path / "paper_1406_4350_amd" / "csrc"
    csrc.mkdir(parents=True)
    (csrc / "gemm.hip").write_text("kernel source v1\n")
    sha = hashlib.sha256(b"kernel source v1\n").hexdigest()
    (tmp_path / "profiles").mkdir()
    entry = {"k": {"n": 128, "bytes_per_launch": 123.0, "source": "gemm.hip", "source_sha256": sha}}
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps(entry))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.load_traffic("k", 128) == 123.0
    assert bench.load_traffic("k", 96) is None          # another box size
    assert bench.load_traffic("other", 128) is None     # not measured
    (csrc / "gemm.hip").write_text("kernel source v2\n")
    assert bench.load_traffic("k", 128) is None         # the kernel changed since the counters were taken


def test_committed_traffic_entries_name_existing_sources():
    path = os.path.join(bench.ROOT, "profiles", "traffic.json")
    data = json.load(open(path))
    for name, ent in data.items():
        assert os.path.exists(os.path.join(bench.ROOT, "paper_1406_4350_amd", "csrc", ent["source"])), name
        assert os.path.exists(os.path.join(bench.ROOT, "profiles", ent["summary"])), name
        assert ent["bytes_per_launch"] > 0
