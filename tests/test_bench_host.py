"""Host-side logic of bench.py that feeds the roofline object: the counter
record of the raster's HBM traffic is reported only for the launch shape the
autotuner picked and only while the raster sources are the ones the counters
were taken on.  No GPU is needed."""
import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


SHAPES = [{"batch": b, "chunk_rows": c} for b in (128, 256) for c in (1, 2)]


@pytest.mark.parametrize("shape", SHAPES)
def test_committed_counter_records(shape):
    """Every committed per-shape record names its own shape and states its
    bytes as the calibrated counter sum; bench.py reports it exactly while
    the raster sources are those the counters were taken on."""
    with open(bench.traffic_path("fp16_g2l_split", shape)) as fh:
        rec = json.load(fh)
    assert rec["launch_shape"] == shape
    # bytes = FETCH_SIZE x fetch factor + WRITE_SIZE x write factor, KiB -> B
    cal = rec["calibration"]
    want = (rec["fetch_kib_per_dispatch"] * cal["fetch_factor"]
            + rec["write_kib_per_dispatch"] * cal["write_factor"]) * 1024
    assert rec["bytes_per_launch"] == pytest.approx(want, rel=1e-12)
    got = bench.read_traffic("fp16_g2l_split", shape)
    if rec["source_hash"] != bench.source_hash(bench.RASTER_SOURCES):
        assert got is None
        pytest.skip("raster sources changed since the counters were taken: bench.py reports "
                    "traffic null until they are taken again")
    assert got is not None and got["bytes_per_launch"] == rec["bytes_per_launch"]


def test_stale_or_other_shape_records_are_not_reported(tmp_path, monkeypatch):
    shape = {"batch": 128, "chunk_rows": 2}
    with open(bench.traffic_path("fp16_g2l_split", shape)) as fh:
        rec = json.load(fh)
    prof = tmp_path / "profiles"
    prof.mkdir()
    monkeypatch.setattr(bench, "traffic_path",
                        lambda p, s, w="fwd_1080p_1M": str(prof / f"rec_{p}_b{s['batch']}_c{s['chunk_rows']}.json"))
    # no record for the shape
    assert bench.read_traffic("fp16_g2l_split", shape) is None
    # a record taken on other sources
    stale = dict(rec, source_hash="0" * 16)
    (prof / "rec_fp16_g2l_split_b128_c2.json").write_text(json.dumps(stale))
    assert bench.read_traffic("fp16_g2l_split", shape) is None
    # a record whose shape field disagrees with the file it sits in
    other = dict(rec, launch_shape={"batch": 256, "chunk_rows": 2})
    (prof / "rec_fp16_g2l_split_b128_c2.json").write_text(json.dumps(other))
    assert bench.read_traffic("fp16_g2l_split", shape) is None
    # the matching one
    (prof / "rec_fp16_g2l_split_b128_c2.json").write_text(json.dumps(rec))
    assert bench.read_traffic("fp16_g2l_split", shape)["bytes_per_launch"] == rec["bytes_per_launch"]


def test_other_workloads_do_not_borrow_the_1080p_records():
    shape = {"batch": 128, "chunk_rows": 2}
    assert bench.read_traffic("fp16_g2l_split", shape, "fwd_4k_6M") is None


def test_more_than_one_gpu_is_refused():
    import subprocess
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
