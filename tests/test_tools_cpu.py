"""Host-side logic of the benchmark and the autotuner (CPU only)."""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_bench_traffic_record_follows_the_sources(monkeypatch):
    sys.path.insert(0, ROOT)
    import bench

    rec = bench.traffic_field(256, 3072, 10000, "mfma_i8", 3.5)
    if bench.kernel_sources_sha256() == bench.TRAFFIC["sources_sha256"]:
        assert rec["bytes"] == rec["read_bytes"] + rec["write_bytes"]
        assert os.path.exists(os.path.join(ROOT, rec["summary"]))
    # a changed kernel source invalidates the record (traffic reported as null)
    monkeypatch.setitem(bench.TRAFFIC, "sources_sha256", "0" * 64)
    assert bench.traffic_field(256, 3072, 10000, "mfma_i8", 3.5) is None
    # and the record only describes the full-band int8 workload
    assert bench.traffic_field(256, 128, 5000, "mfma_i8", 0.2) is None


def test_tuner_candidates_and_cache(tmp_path, monkeypatch):
    pytest.importorskip("torch")
    from paper_1501_05992_amd import corrx, tune

    c64, c256 = tune.candidates(64), tune.candidates(256)
    # batch: 256-input units with the default chunk, 128- and 64-input units with two chunk lengths each
    assert len(c64) == 5 * len(tune.SPLITS) and len(c256) == len(tune.SPLITS)
    assert all(c & 0xFF == corrx.CORRX_TILE_UNIT256 for c in c256)
    assert {c & 0xFF for c in c64} == {corrx.CORRX_TILE_UNIT64, corrx.CORRX_TILE_UNIT128, corrx.CORRX_TILE_UNIT256}
    assert {(c >> 8) & 0xFFFF for c in c64} == set(tune.SPLITS)
    assert {c >> 24 for c in c64} == {0, 2, 3}  # default, 128- (128-input units), 256-sample chunks (64-input)
    # corr_xmac: the 64-input unit also has 64- and 256-sample chunks
    x64 = tune.candidates(64, "xmac")
    assert len(x64) == 6 * len(tune.SPLITS) and {c >> 24 for c in x64} == {0, 1, 2, 3}
    assert corrx.tile_code(corrx.CORRX_TILE_UNIT128, 4, 128) == 2 | (4 << 8) | (2 << 24)
    d = (256, 3072, 10000, 0)
    assert tune._key(d, "mfma_i8", "xmac", "gfx950") == "gfx950|mfma_i8|xmac|N256|F3072|T10000|L0"
    assert tune._key(d, "mfma_i8", "xmac", "gfx950") != tune._key(d, "mfma_i8", "batch", "gfx950")
    path = str(tmp_path / "sub" / "tune.json")
    monkeypatch.setenv("CORRX_TUNE_CACHE", path)
    assert tune.cache_path() == path
    assert tune._load_cache(path) == {}
    data = {"gfx950|N64|F3072|T10000|L0": {"code": 257, "ms": 0.8, "times": {"257": 0.8}}}
    tune._save_cache(path, data)
    assert tune._load_cache(path) == data
    with open(path, "w") as fh:
        fh.write("{not json")
    assert tune._load_cache(path) == {}  # a corrupt cache is ignored
