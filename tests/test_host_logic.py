"""Host-side logic without a GPU: the warm start's stored fallback
calibration and the bench's traffic files, which are only used while the
kernel sources they were measured on are unchanged."""
import json
import math
import os

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_stored_calibration_covers_every_schedule():
    from paper_1604_03734_amd import warmstart as W
    cal = W.load_calibration()
    assert cal is not None and cal["k"] == 100 and cal["lambda"] == W.LAM
    assert cal["streets"] == list(range(1001, 1007))
    for tau, gamma in W.SCHEDULES:
        g = W.calibrated_gap(tau, gamma, 100, cal)
        assert g is not None and math.isfinite(g) and 0.0 < g < 1.0, (tau, gamma)
        e = [x for x in cal["entries"] if abs(x["tau"] - tau) <= 1e-9 * tau and x["gamma"] == gamma][0]
        # the reference is the largest over the training streets
        assert len(e["per_street"]) == 6 and g == max(e["per_street"])
    # the accelerated schedule converges faster than the fixed one at the same tau0
    t0 = 1.0 / np.sqrt(12.0)
    assert W.calibrated_gap(t0, W.LAM, 100, cal) < W.calibrated_gap(t0, 0.0, 100, cal)


def test_calibration_lookup_misses_return_none():
    from paper_1604_03734_amd import warmstart as W
    cal = W.load_calibration()
    assert W.calibrated_gap(0.07, 0.0, 100, cal) is None          # steps not in the table
    assert W.calibrated_gap(0.05, 0.25, 100, cal) is None         # another schedule
    assert W.calibrated_gap(0.05, 0.0, 50, cal) is None           # another K
    assert W.calibrated_gap(0.05, 0.0, 100, {"k": 100, "entries": []}) is None
    assert W.calibrated_gap(0.05 * (1 + 1e-12), 0.0, 100, cal) is not None


def _traffic_files(bench):
    """(workload, storage, file) of every traffic summary, one file per
    kernel variant where the workload has several."""
    for (workload, storage), (names, srcs) in bench.TRAFFIC_FILES.items():
        for name in (names.values() if isinstance(names, dict) else [names]):
            yield workload, storage, name


def test_traffic_files_are_consistent_and_looked_up_by_digest(monkeypatch):
    """Each file's figures hang together, and the bench returns them exactly
    when the kernel sources hash to the file's digest and the kernel variant
    that ran is the one measured."""
    import bench
    for workload, storage, name in _traffic_files(bench):
        with open(os.path.join(ROOT, "profiles", name)) as f:
            t = json.load(f)
        nvox = t["voxels"]
        r = t.get("read_bytes_per_launch", t.get("read_bytes_per_iter"))
        w = t.get("write_bytes_per_launch", t.get("write_bytes_per_iter"))
        assert abs((r + w) / nvox - t["bytes_per_voxel_iter"]) < 1e-9 * t["bytes_per_voxel_iter"]
        # writes are exactly the algorithmic bytes the kernel stores
        alg_w = 20 if storage == "f32" else 10
        assert abs(w / nvox - alg_w) < 0.1, name
        assert t["bytes_per_voxel_iter"] >= t["algorithmic_bytes_per_voxel_iter"]
        monkeypatch.setattr(bench, "src_digest", lambda names=None, d=t["source_digest"]: d)
        assert bench.load_traffic(nvox, workload, storage, t["kernel_id"]) == t["bytes_per_voxel_iter"] * nvox
        # another kernel variant gives no figure, nor another block order
        assert bench.load_traffic(nvox, workload, storage, t["kernel_id"] + 1) is None
        if "layout_used" in t:
            assert bench.load_traffic(nvox, workload, storage, t["kernel_id"], t["layout_used"]) is not None
            assert bench.load_traffic(nvox, workload, storage, t["kernel_id"], t["layout_used"] ^ 1) is None


def test_traffic_is_dropped_when_the_sources_change(monkeypatch):
    import bench
    monkeypatch.setattr(bench, "src_digest", lambda names=None: "0" * 16)
    for workload, storage, name in _traffic_files(bench):
        with open(os.path.join(ROOT, "profiles", name)) as f:
            t = json.load(f)
        assert bench.load_traffic(t["voxels"], workload, storage, t["kernel_id"]) is None
