"""Host-side logic of the benchmark (no GPU): the byte-counter records that
give roofline.traffic count only while the sources they name are unchanged."""
import hashlib
import os
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def _record(tmp_path, kernel, form, nbytes, sources):
    items = []
    for rel in sources:
        with open(tmp_path / rel, "rb") as f:
            items.append(f"{rel}:{hashlib.sha256(f.read()).hexdigest()}")
    (tmp_path / "profiles").mkdir(exist_ok=True)
    (tmp_path / "profiles" / "k.md").write_text(
        "# summary\n\ntraffic-record: kernel=%s form=%s bytes_per_launch=%d "
        "sources=%s\n" % (kernel, form, nbytes, ",".join(items)))


def test_traffic_record_follows_its_sources(tmp_path):
    (tmp_path / "a.hip").write_text("kernel a\n")
    (tmp_path / "b.h").write_text("header b\n")
    _record(tmp_path, "spmv_px", "mixed", 1234, ["a.hip", "b.h"])
    got = bench.measured_traffic("spmv_px", "mixed", root=str(tmp_path))
    assert got == 1234.0
    # another kernel or form has no record
    assert bench.measured_traffic("spmv_px", "fp64", root=str(tmp_path)) is None
    assert bench.measured_traffic("vup_fine", "mixed", root=str(tmp_path)) is None
    # any change to a listed source voids the record
    (tmp_path / "b.h").write_text("header b, edited\n")
    assert bench.measured_traffic("spmv_px", "mixed", root=str(tmp_path)) is None
    # and so does a listed source that is gone
    (tmp_path / "b.h").write_text("header b\n")
    assert bench.measured_traffic("spmv_px", "mixed", root=str(tmp_path)) == 1234.0
    os.remove(tmp_path / "a.hip")
    assert bench.measured_traffic("spmv_px", "mixed", root=str(tmp_path)) is None


def test_traffic_record_keyed_by_workload(tmp_path):
    """A record names its workload: the lookup for one workload ignores the
    records of another (the same kernel moves other bytes at another size)."""
    (tmp_path / "a.hip").write_text("kernel a\n")
    item = "a.hip:" + hashlib.sha256(b"kernel a\n").hexdigest()
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "k.md").write_text(
        f"traffic-record: kernel=spmv_px form=mixed workload=w256 bytes_per_launch=5 sources={item}\n"
        f"traffic-record: kernel=spmv_px form=mixed workload=w640 bytes_per_launch=7 sources={item}\n")
    assert bench.measured_traffic("spmv_px", "mixed", "w640", root=str(tmp_path)) == 7.0
    assert bench.measured_traffic("spmv_px", "mixed", "w256", root=str(tmp_path)) == 5.0
    assert bench.measured_traffic("spmv_px", "mixed", "w1024", root=str(tmp_path)) is None


def test_committed_records_name_existing_sources():
    """Every record under profiles/ names sources that exist in the tree."""
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    n = 0
    for name in os.listdir(os.path.join(root, "profiles")):
        with open(os.path.join(root, "profiles", name)) as f:
            for line in f:
                if not line.startswith("traffic-record:"):
                    continue
                kv = dict(t.split("=", 1) for t in line.split()[1:])
                for item in kv["sources"].split(","):
                    rel = item.rsplit(":", 1)[0]
                    assert os.path.exists(os.path.join(root, rel)), rel
                n += 1
    assert n > 0
