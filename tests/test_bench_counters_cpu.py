"""CPU: bench.py's readers of rocprofv3 counter files.  A distance round runs
the two-task kernel and then the one-wave kernel; the per-round figures sum
both kernels' dispatches and divide by the rounds (the one-wave kernel's
dispatches).  HBM bytes are scaled by what each counter reads for the 1 GiB
calibration copy."""
import csv
import json
import os

import pytest

import bench

HEADER = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]


def _write(dirpath, rows):
    os.makedirs(dirpath, exist_ok=True)
    with open(os.path.join(dirpath, "x_counter_collection.csv"), "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(HEADER)
        w.writerows(rows)


@pytest.fixture
def profdir(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "profile_file", lambda wl, kind: str(tmp_path / f"{wl}_{kind}.json"))
    return tmp_path


def test_traffic_sums_both_round_kernels(profdir):
    calib_kib = 524288.0  # FETCH_SIZE reads half of the 1 GiB copy: scale 2
    fetch = [["1", "void at::native::neg_kernel(...)", "FETCH_SIZE", str(calib_kib)]]
    write = [["1", "void at::native::neg_kernel(...)", "WRITE_SIZE", "1048576"]]
    # two rounds: pairs 100 + tasks 20 KiB, then pairs 60 + tasks 20 KiB; an unrelated kernel
    for d, (name, f, wv) in enumerate([("fl::k_ads_pairs<false>(...)", 100, 10), ("fl::k_ads_tasks<false, 1, 512u>(...)", 20, 2),
                                       ("fl::k_ads_pairs<false>(...)", 60, 6), ("fl::k_ads_tasks<false, 1, 512u>(...)", 20, 2),
                                       ("fl::k_sweep_heavy(...)", 999, 999)], start=2):
        fetch.append([str(d), name, "FETCH_SIZE", str(f)])
        write.append([str(d), name, "WRITE_SIZE", str(wv)])
    _write(str(profdir / "f"), fetch)
    _write(str(profdir / "w"), write)
    bench.write_traffic(str(profdir / "f"), str(profdir / "w"), "wl")
    out = json.load(open(profdir / "wl_traffic.json"))
    assert out["launches"] == 2
    assert out["fetch_bytes_per_launch"] == round((100 + 20 + 60 + 20) / 2 * 1024 * 2)
    assert out["write_bytes_per_launch"] == round((10 + 2 + 6 + 2) / 2 * 1024)
    assert out["kernel_source_hash"] == bench.kernel_hash()


def test_issue_sums_both_round_kernels(profdir):
    rows = []
    for d, (name, v) in enumerate([("fl::k_ads_pairs<false>(...)", 1000), ("fl::k_ads_tasks<false, 1, 512u>(...)", 200),
                                   ("fl::k_ads_tasks<false, 1, 512u>(...)", 300), ("fl::k_sweep_round(...)", 7)]):
        rows.append([str(d), name, "SQ_INSTS_VALU", str(v)])
    _write(str(profdir / "sq"), rows)
    bench.write_issue(str(profdir / "sq"), "wl")
    out = json.load(open(profdir / "wl_issue.json"))
    assert out["launches"] == 2
    assert out["sq_insts_valu_per_launch"] == (1000 + 200 + 300) // 2
