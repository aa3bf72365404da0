"""Host-side logic of the bench and the launch-grid tuner (no GPU)."""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _counts(kb=4):
    return {"key_bytes": kb, "n_pairs": 1000, "n_cand": 1700, "n_prims": 500, "n_vox": 400, "n_fib": 10,
            "n_records": 300, "n_units": 20}


def test_byte_model_counts_each_array_once():
    c = _counts()
    # unit kernel: per record id + record + direction, per voxel key + count + w + S, per unit 32
    assert bench.kernel_bytes("unit_fib", c) == (4 + 64 + 16) * 300 + (4 + 32) * 400 + 32 * 20
    assert bench.kernel_bytes("unit_fib", _counts(8)) == (4 + 64 + 16) * 300 + (8 + 32) * 400 + 32 * 20
    # the compaction reads and writes each voxel once
    assert bench.kernel_bytes("unit_compact", c) == 2 * (4 + 32) * 400 + 24 * 20
    assert bench.kernel_bytes("no_such_kernel", c) is None


def test_flop_model_is_linear_in_candidates_and_pairs():
    c = _counts()
    f = bench.kernel_flops("unit_fib", c)
    c2 = dict(c, n_cand=2 * c["n_cand"], n_pairs=2 * c["n_pairs"])
    assert f > 0 and bench.kernel_flops("unit_fib", c2) == 2 * f


def test_traffic_is_reported_only_for_the_measured_sources(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    table = {"source_digest": bench.source_digest(),
             "kernels": {"unit_fib": {"fetch_bytes_per_launch": 100, "write_bytes_per_launch": 50}}}
    (prof / "hbm_traffic_plain_weave.json").write_text(json.dumps(table))
    # the digest covers the HIP sources of the repository; the table is read from ROOT/profiles
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "source_digest", lambda: table["source_digest"])
    assert bench.traffic_bytes("unit_fib") == 150
    assert bench.traffic_bytes("unit_compact") is None
    monkeypatch.setattr(bench, "source_digest", lambda: "0" * 16)
    assert bench.traffic_bytes("unit_fib") is None


def test_tuner_table_round_trip(tmp_path, monkeypatch):
    from paper_2604_13191_amd import autotune

    calls = []

    class FakeVx:
        TUNE_KERNELS = ("unit_fib", "unit_plan", "unit_compact", "lod_reduce", "lod_cluster")

        @staticmethod
        def set_launch_grids(g):
            calls.append(list(g))

    path = tmp_path / "grids.json"
    path.write_text(json.dumps({"device": "test", "tables": {"w": {"grids": [512, 1024, 2048, 256, 8192]}}}))
    monkeypatch.setattr(autotune, "vx", FakeVx)
    assert autotune.apply("w", str(path)) == [512, 1024, 2048, 256, 8192]
    assert calls == [[512, 1024, 2048, 256, 8192]]
    assert autotune.apply("missing", str(path)) is None
    assert autotune.apply("w", str(tmp_path / "absent.json")) is None


def test_committed_tables_are_well_formed():
    from paper_2604_13191_amd import autotune
    with open(autotune.TABLE) as f:
        t = json.load(f)
    for name, tab in t["tables"].items():
        assert len(tab["grids"]) == 5, name
        assert all(64 <= g <= 16384 for g in tab["grids"]), name
