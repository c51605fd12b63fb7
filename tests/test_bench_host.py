"""Host logic of bench.py: the counter records and their source hashes, the
roofline figures built from them, the tile strings and the one-GPU guard
(no GPU needed)."""
import importlib.util
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_counter_records_match_the_committed_sources(bench):
    """Every stored counter record was taken on the kernel sources in the
    tree: a record whose sources changed would report null."""
    for rec in (bench.TRAFFIC, bench.RD_TRAFFIC, bench.RENDER_VALU):
        assert bench.sources_sha256(rec["sources"]) == rec["sources_sha256"], rec["sources"]
    assert bench.measured_traffic() == bench.TRAFFIC["fetch_bytes"] + bench.TRAFFIC["write_bytes"]
    assert bench.measured_traffic(bench.RD_TRAFFIC) == \
        bench.RD_TRAFFIC["fetch_bytes"] + bench.RD_TRAFFIC["write_bytes"]


def test_stale_record_reads_null(bench):
    stale = dict(bench.TRAFFIC, sources_sha256="0" * 64)
    assert bench.measured_traffic(stale) is None


def test_render_roofline(bench, monkeypatch):
    r = bench.render_roofline(157.3e6, 0.0697)
    assert r["bound"] == "alu"
    assert r["peak"] == pytest.approx(614.4)
    rate = bench.RENDER_VALU["valu_instr"] / 0.0697e-3
    assert r["achieved"] == pytest.approx(rate / 1e9)
    assert r["frac"] == pytest.approx(rate / (256 * 4 * 2.4e9 / 4))
    assert r["hbm_frac"] == pytest.approx(157.3e6 / 0.0697e-3 / 8e12)
    assert bench.render_roofline(157.3e6, None) is None
    monkeypatch.setitem(bench.RENDER_VALU, "sources_sha256", "0" * 64)
    stale = bench.render_roofline(157.3e6, 0.0697)
    assert stale["achieved"] is None and stale["frac"] is None and stale["hbm_frac"] > 0


def test_tile_strings(bench):
    assert bench.tile_of({"wave_rows": 32, "tile_l": 128, "waves": 8, "schedule": "phase_shifted"}) == "32x128x8"
    assert bench.tile_of({"wave_rows": 32, "tile_l": 64, "waves": 8, "schedule": "pipelined"}) == "32x64x8i"
    assert bench.tile_of({"wave_rows": 64, "tile_l": 64, "waves": 4, "schedule": "pipelined"}) == "64x64x4"


def test_more_than_one_gpu_is_refused():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert "exactly one GPU" in (out.stdout + out.stderr)
