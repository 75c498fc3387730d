"""Host-side logic of bench.py (no GPU): kernel-name classes, the stored
counter traffic and its source digests, the host record."""
import json
import os

import pytest

import bench


@pytest.mark.parametrize("name,cls", [
    ("void dsbcg::wilson_cm_kernel<double, false, false, 512, true>(dsbcg::Geom, ...)", "wilson_stencil.f64"),
    ("void dsbcg::wilson_cm_kernel<float, true, false, 512, false>(dsbcg::Geom, ...)", "wilson_stencil.f32"),
    ("void dsbcg::ts_reg_kernel<double, 5, 2, 4>(dsbcg::TsArgs)", "block_gram_update.f64"),
    ("void dsbcg::ts_lds_kernel<float>(dsbcg::TsArgs)", "block_gram_update.f32"),
    ("void dsbcg::window_kernel<double, 1, 4, true>(dsbcg::WinArgs)", "shift_update.f64"),
    ("void dsbcg::window3_kernel<double, 2, true>(dsbcg::WinArgs)", "shift_update.f64"),
    ("void dsbcg::window3_kernel<float, 1, false>(dsbcg::WinArgs)", "shift_update.f32"),
    ("void dsbcg::transpose_kernel<double, float>(long, int, ...)", "convert"),
    ("dsbcg::link_grad_kernel(dsbcg::Geom, ...)", "link_grad"),
    ("void dsbcg::window_table3_kernel<double>(dsbcg::WinCoef, ...)", "small_algebra"),
    ("dsbcg::reduce_kernel(dsbcg::cx<double> const*, int, dsbcg::cx<double>*)", "small_algebra"),
    ("__amd_rocclr_copyBuffer", None),
])
def test_kernel_class(name, cls):
    assert bench.kernel_class(name) == cls


def test_every_class_has_sources():
    for fam, paths in bench.SOURCES.items():
        assert paths, fam
        for p in paths:
            assert os.path.exists(os.path.join(bench.ROOT, p)), p
        assert len(bench.source_digest(paths)) == 16


def test_stored_traffic_follows_the_source_digest(tmp_path, monkeypatch):
    """stored_traffic returns the counted bytes only for the digest the record
    was taken at, and None for any other or a missing class."""
    rec = {"_calibration": {"fetch_factor": 2.0, "write_factor": 1.0},
           "wilson_stencil.f64": {"bytes_per_launch": 1.25e10, "source_digest": "0123456789abcdef",
                                  "dispatches": 3}}
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.stored_traffic("wilson_stencil.f64", "0123456789abcdef") == 1.25e10
    assert bench.stored_traffic("wilson_stencil.f64", "fedcba9876543210") is None
    assert bench.stored_traffic("wilson_stencil.f32", "0123456789abcdef") is None


def test_committed_traffic_record_schema():
    with open(os.path.join(bench.ROOT, "profiles", "traffic.json")) as f:
        rec = json.load(f)
    cal = rec["_calibration"]
    assert 1.9 < cal["fetch_factor"] < 2.1 and cal["write_factor"] == 1.0
    for cls, ent in rec.items():
        if cls.startswith("_"):
            continue
        assert cls.split(".")[0] in bench.SOURCES, cls
        assert ent["bytes_per_launch"] > 0 and ent["dispatches"] > 0
        assert len(ent["source_digest"]) == 16


def test_host_info():
    info = bench.host_info()
    assert info["nproc"] >= 1 and isinstance(info["cpu"], str) and info["cpu"]
    if os.path.exists("/proc/meminfo"):
        assert info["mem_gib"] > 0
