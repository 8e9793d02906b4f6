"""Host logic of bench.py (no GPU): the HBM traffic it reports comes from a committed counter summary
only while that summary was taken on the current kernel sources and the same workload, and a
multi-GPU request is refused before anything touches a device."""
import json
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

BATCH_SOURCES = ("paper_1710_10569_amd/csrc/clb_device.h", "paper_1710_10569_amd/csrc/clb_inplace.h",
                 "paper_1710_10569_amd/csrc/clb_batch.hip", "paper_1710_10569_amd/build.py")
SOURCES_3D = ("paper_1710_10569_amd/csrc/clb3d.hip", "paper_1710_10569_amd/csrc/clb_device.h",
              "paper_1710_10569_amd/build.py")


def _copy_tree(tmp_path, rels):
    for rel in rels:
        dst = tmp_path / rel
        dst.parent.mkdir(parents=True, exist_ok=True)
        shutil.copyfile(os.path.join(ROOT, rel), dst)


@pytest.mark.parametrize("hash_fn,rels", [("kernel_source_hash", BATCH_SOURCES), ("kernel_source_hash_3d", SOURCES_3D)])
def test_source_hash_follows_every_kernel_source(tmp_path, monkeypatch, hash_fn, rels):
    """The hash is that of the committed sources, and a one-byte change to any of them changes it."""
    _copy_tree(tmp_path, rels)
    fn = getattr(bench, hash_fn)
    ref = fn()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert fn() == ref
    for rel in rels:
        p = tmp_path / rel
        orig = p.read_bytes()
        p.write_bytes(orig + b" ")
        assert fn() != ref, rel
        p.write_bytes(orig)
    assert fn() == ref


def test_batch_traffic_only_for_matching_sources_and_size(tmp_path, monkeypatch):
    f = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.measured_traffic(1000) is None                      # no summary
    f.write_text("not json")
    assert bench.measured_traffic(1000) is None                      # unreadable summary
    rec = {"kernel_source_hash": bench.kernel_source_hash(), "sites": 1000, "bytes_per_launch": 112345.0}
    f.write_text(json.dumps(rec))
    assert bench.measured_traffic(1000) == 112345.0
    assert bench.measured_traffic(1001) is None                      # another workload
    f.write_text(json.dumps(dict(rec, kernel_source_hash="0" * 16)))
    assert bench.measured_traffic(1000) is None                      # kernel changed since


def test_3d_traffic_only_for_matching_sources_and_size(tmp_path, monkeypatch):
    f = tmp_path / "traffic3d.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE_3D", str(f))
    assert bench.measured_traffic_3d("fp32", 1000) is None
    rec = {"kernel_source_hash": bench.kernel_source_hash_3d(), "sites": 1000,
           "precisions": {"fp32": {"bytes_per_step": 272000.0}}}
    f.write_text(json.dumps(rec))
    assert bench.measured_traffic_3d("fp32", 1000) == 272000.0
    assert bench.measured_traffic_3d("fp64", 1000) is None           # precision not measured
    assert bench.measured_traffic_3d("fp32", 999) is None
    f.write_text(json.dumps(dict(rec, kernel_source_hash="0" * 16)))
    assert bench.measured_traffic_3d("fp32", 1000) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and not r.stdout.strip()
