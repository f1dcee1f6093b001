"""Host logic of bench.py (no GPU): how many time levels one sweep launch
advances, and the lookup of the committed DRAM-traffic record, which must
match the kernel source, the workload, the dtype, the levels per launch and,
for a batch, the tile assignment."""
import bench
from paper_1603_08221_amd.workloads import CONFIGS


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
