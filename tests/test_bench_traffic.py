"""bench.py's traffic bookkeeping (host only): the FETCH_SIZE / WRITE_SIZE
counters of rocprofv3 runs are scaled by a plain copy of known size, averaged
per launch, and dropped when a kernel's sources or the tuning differ."""
import csv
import importlib.util
import json
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture()
def bench(tmp_path, monkeypatch):
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    monkeypatch.setattr(b, "TRAFFIC_PATH", str(tmp_path / "traffic.json"))
    return b


def _csv(root, sub, rows):
    d = root / sub / "run"
    d.mkdir(parents=True)
    with open(d / "x_counter_collection.csv", "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writerows(rows)


def test_write_and_read_traffic(bench, tmp_path):
    pmc = tmp_path / "pmc"
    tiles = "void flood::k_flood_tiles<1>(flood::TileArgs, float const*)"
    # the copy of 1 GiB reads as 512 MiB of FETCH_SIZE (64-byte units counted as 32) and 1 GiB of WRITE_SIZE
    _csv(pmc, "pmc_copy_fetch", [[1, "__amd_rocclr_copyBuffer", "FETCH_SIZE", 524288.0]])
    _csv(pmc, "pmc_copy_write", [[1, "__amd_rocclr_copyBuffer", "WRITE_SIZE", 1048576.0]])
    _csv(pmc, "pmc_fetch", [[2, tiles, "FETCH_SIZE", 1000.0], [3, tiles, "FETCH_SIZE", 3000.0],
                            [4, "void flood::k_fps_coop<0>(int)", "FETCH_SIZE", 10.0]])
    _csv(pmc, "pmc_write", [[2, tiles, "WRITE_SIZE", 100.0], [3, tiles, "WRITE_SIZE", 300.0],
                            [4, "void flood::k_fps_coop<0>(int)", "WRITE_SIZE", 1.0]])
    tu = {"tile_lanes": 16, "cells_per_point": 1.0}
    bench.write_traffic(str(pmc), tu)
    t = json.load(open(bench.TRAFFIC_PATH))
    k = t["kernels"]["flood::k_flood_tiles<1>"]
    assert k["fetch_bytes_per_launch"] == 2000 * 1024 * 2.0
    assert k["write_bytes_per_launch"] == 200 * 1024 * 1.0
    assert k["dispatches_averaged"] == 2
    assert bench.measured_traffic("flood::k_flood_tiles<1>", dict(tu)) == 2000 * 2048 + 200 * 1024
    # another tuning, or none: the figures do not apply
    assert bench.measured_traffic("flood::k_flood_tiles<1>", {"tile_lanes": 64}) is None
    assert bench.measured_traffic("flood::k_flood_tiles<1>", None) is None
    # the landmark kernel takes no tuning
    assert bench.measured_traffic("flood::k_fps_coop<0>") == 10 * 2048 + 1024
    assert bench.measured_traffic("flood::k_flood_deep") is None


def test_traffic_dropped_when_sources_change(bench, tmp_path):
    t = {"kernels": {"flood::k_flood_deep": {"fetch_bytes_per_launch": 1.0, "write_bytes_per_launch": 2.0,
                                             "sources": ["flood.hip"], "sources_sha256": "0" * 64, "tuning": {}}}}
    json.dump(t, open(bench.TRAFFIC_PATH, "w"))
    assert bench.measured_traffic("flood::k_flood_deep", None) is None
