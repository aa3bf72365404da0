"""Host-side logic of the bench and the launch-grid tuner (no GPU)."""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _counts(kb=4):
    return {"key_bytes": kb, "n_pairs": 1000, "n_cand": 1700, "n_prims": 500, "levels": [400, 60, 8, 1],
            "n_records": 300, "n_units": 20, "input_bytes": 36 * 500}


def test_byte_model_counts_each_array_once():
    c = _counts()
    # unit kernel: per primitive its direction (12), per pair emit + sort exchange + reduce read
    # (4 x 12 bytes with 32-bit keys), per leaf voxel key + count + w + S written once
    assert bench.kernel_bytes("unit_fib", c) == 12 * 500 + 4 * 12 * 1000 + (4 + 32) * 400
    c8 = _counts(8)
    assert bench.kernel_bytes("unit_tri", c8) == 12 * 500 + 4 * 16 * 1000 + (8 + 32) * 400
    # the compaction reads and writes each voxel once
    assert bench.kernel_bytes("unit_compact", c) == 2 * (4 + 32) * 400
    assert bench.kernel_bytes("no_such_kernel", c) is None


def test_step_bytes_follow_the_level_records():
    c = _counts()
    body = 36 * 500 + 12 * 500 + 4 * 12 * 1000
    # leaf: key + count + w + S (4 + 4 + 4 + 24 bytes); K = 1 above it: key + mask word + w + S
    assert bench.step_bytes(c, 1) == body + 2 * (4 + 4 + 4 + 24) * 400 + 2 * (4 + 4 + 28) * 69
    # K = 4: the one-lobe sums plus four lobes of 28 bytes each
    assert bench.step_bytes(c, 4) == body + 2 * (4 + 4 + 4 + 24) * 400 + 2 * (4 + 4 + 28 * 5) * 69


def test_traffic_is_reported_only_for_the_measured_sources(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    table = {"source_digest": bench.source_digest(),
             "kernels": {"unit_fib": {"fetch_bytes_per_launch": 100, "write_bytes_per_launch": 50}}}
    (prof / "hbm_traffic_plain_weave.json").write_text(json.dumps(table))
    # the digest covers the HIP sources of the repository; the table is read from ROOT/profiles
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "source_digest", lambda: table["source_digest"])
    assert bench.traffic_bytes("plain_weave", "unit_fib") == 150
    assert bench.traffic_bytes("plain_weave", "unit_compact") is None
    assert bench.traffic_bytes("brushed_metal", "unit_fib") is None
    monkeypatch.setattr(bench, "source_digest", lambda: "0" * 16)
    assert bench.traffic_bytes("plain_weave", "unit_fib") is None


def test_tuner_table_round_trip(tmp_path):
    from paper_2604_13191_amd import autotune
    import paper_2604_13191_amd as vx
    path = tmp_path / "tunings.json"
    t = vx.Tuning(3, 1536, (512, 1024, 2048, 256, 8192))
    path.write_text(json.dumps({"device": "test", "tables": {"w": {"tuning": t.as_dict()}}}))
    assert autotune.load("w", str(path)) == t
    assert autotune.load("missing", str(path)) is None
    assert autotune.load("w", str(tmp_path / "absent.json")) is None
    c = t.cstruct()
    assert (c.tile_bits, c.unit_budget, list(c.grids)) == (3, 1536, [512, 1024, 2048, 256, 8192])
    assert vx.Tuning.from_dict(t.as_dict()) == t and vx.Tuning.from_dict(None) is None


def test_committed_tunings_are_well_formed():
    import os
    from paper_2604_13191_amd import autotune
    if not os.path.exists(autotune.TABLE):
        return
    with open(autotune.TABLE) as f:
        t = json.load(f)
    for name, tab in t["tables"].items():
        tu = tab["tuning"]
        assert tu["tile_bits"] in (0, 2, 3, 4), name
        assert tu["unit_budget"] in (0, 1024, 1536, 2048, 3072), name
        assert len(tu["grids"]) == 5 and all(g == 0 or 64 <= g <= 16384 for g in tu["grids"]), name
        assert tab["step_ms"]["tuned"] > 0 and tab["step_ms"]["default"] > 0, name
