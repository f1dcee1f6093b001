"""Host logic of bench.py (no GPU): the driver's command line, how many time
levels one sweep launch advances, and the lookup of the committed DRAM-traffic
record, which must match the kernel source, the workload, the dtype, the
levels per launch and, for a batch, the tile assignment."""
import json

import pytest

import bench
from paper_1603_08221_amd.workloads import CONFIGS, batch_instances


def test_driver_command_line_is_accepted():
    """python bench.py --gpus 1 --steps 20 --warmup 5: any step counts, the
    timed block replays one graph of its own length."""
    a = bench.parse_args(["--gpus", "1", "--steps", "20", "--warmup", "5"])
    assert (a.gpus, a.steps, a.warmup, a.dtype) == (1, 20, 5, "f32")
    assert bench.graph_length(a.steps) == 20
    assert bench.graph_length(2000) == 100 and bench.graph_length(7) == 7
    d = bench.parse_args([])
    assert d.gpus == 1 and d.steps >= 1 and d.warmup >= 0
    for odd in (["--steps", "3", "--warmup", "1"], ["--steps", "1", "--warmup", "0"]):
        bench.parse_args(odd)  # no multiple-of-anything rule
    with pytest.raises(SystemExit):
        bench.parse_args(["--steps", "0"])


def test_more_than_one_gpu_exits_with_a_message(capsys):
    with pytest.raises(SystemExit) as e:
        bench.main(["--gpus", "2", "--steps", "20", "--warmup", "5"])
    assert e.value.code == 2
    out = json.loads(capsys.readouterr().out.strip())
    assert out["n_gpus"] == 2 and "one GPU" in out["error"]


def test_headline_table_is_the_seeded_64_member_sweep():
    ws = batch_instances()
    assert len(ws) == 64
    nodes = sum(w.nodes for w in ws)
    assert nodes > 7_000_000                      # about 1 GB of FP32 state: above the last-level cache
    assert nodes * 36 * 4 > 256 * 2 ** 20
    assert {w.ny for w in ws} <= {16, 32, 48, 64, 96, 128} and all(w.nx == 20 * w.ny for w in ws)
    assert bench.METRIC.startswith("MLUPS (both species)")


def test_levels_per_launch():
    assert bench.levels_per_launch(CONFIGS["ne_ar_64x1280"], 0) == 2  # at most 64 rows
    assert bench.levels_per_launch(CONFIGS["he_ar_512x10240"], 0) == 1
    assert bench.levels_per_launch(CONFIGS["ne_ar_64x1280"], 1) == 1  # as asked


def test_traffic_record_lookup(tmp_path, monkeypatch):
    src = bench.source_hash()
    rec = tmp_path / "traffic.txt"
    rec.write_text("# header\n"
                   f"workload=ne_ar_64x1280 dtype=f32 levels=2 source={src} bytes_per_launch=123\n"
                   f"workload=he_ar_512x10240 dtype=f32 levels=1 source=0000 bytes_per_launch=456\n"
                   f"workload=he_ar_512x10240 dtype=f32 source={src} bytes_per_launch=789\n"
                   f"workload=sweep_table_64 dtype=f32 levels=1 source={src} tiles=node,rows2 bytes_per_launch=42\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(rec))
    assert bench.measured_traffic("ne_ar_64x1280", "f32", 2) == 123
    assert bench.measured_traffic("ne_ar_64x1280", "f32", 1) is None  # other launch configuration
    assert bench.measured_traffic("ne_ar_64x1280", "f64", 2) is None
    # a record taken on another source is ignored; one without levels means one level
    assert bench.measured_traffic("he_ar_512x10240", "f32") == 789
    # a batch record holds only for the tile assignment it was taken with
    assert bench.measured_traffic("sweep_table_64", "f32", tiles="node,rows2") == 42
    assert bench.measured_traffic("sweep_table_64", "f32", tiles="node,rows4") is None


def test_source_hash_ignores_comments(tmp_path, monkeypatch):
    a, b = tmp_path / "a.hip", tmp_path / "b.hip"
    a.write_text("int f() {\n  return 1;  // one\n}\n/* block */\n")
    b.write_text("int f() {\n  return 1;\n}\n")
    monkeypatch.setattr(bench, "KERNEL_SOURCES", [str(a)])
    ha = bench.source_hash()
    monkeypatch.setattr(bench, "KERNEL_SOURCES", [str(b)])
    assert bench.source_hash() == ha
    b.write_text("int f() {\n  return 2;\n}\n")
    assert bench.source_hash() != ha


def test_named_tile_assignment_skips_the_tuner():
    """--tiles picks one of the tuner's candidates by name (for profiling runs
    that must see the assignment a traffic record was taken with)."""
    from paper_1603_08221_amd import lbsep

    t = bench.tune_table(lbsep, bench.parse_args(["--tiles", "node,rows2"]))
    assert t["name"] == "node,rows2" and set(t["rows"]) == {2} and len(t["modes"]) == 64
    with pytest.raises(SystemExit):
        bench.tune_table(lbsep, bench.parse_args(["--tiles", "no-such-assignment"]))
