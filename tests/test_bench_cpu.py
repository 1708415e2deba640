"""Host logic of bench.py (no GPU): the measured-traffic table and its lookup,
and the refusal of multi-GPU runs."""
import argparse
import csv
import json
import os
import subprocess
import sys

import numpy as np

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _counter_csv(path, counter, rows):
    """rows: (dispatch id, kernel name, value) -> a rocprofv3-style
    counter_collection.csv (one row per dispatch and hardware instance)."""
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for d, k, v in rows:
            w.writerow({"Dispatch_Id": d, "Kernel_Name": k, "Counter_Name": counter, "Counter_Value": v})


def test_traffic_key_names_workload_precision_and_launch():
    assert bench.traffic_key("C2", "fp64", [34, 15, 43, 0]) == "C2/fp64@34,15,43"
    assert bench.traffic_key("C5/gc", "fp32", [34, 15, 128]) == "C5/gc/fp32@34,15,128"


def test_counter_summary_scaling_and_lookup(tmp_path):
    """Counters of two dispatches (each split over two hardware instances) are
    averaged per dispatch and scaled by the copy calibration: the copy moves
    COPY_BYTES each way, FETCH_SIZE reports half of it (128-byte requests
    counted as 64 bytes) and WRITE_SIZE all of it, so reads scale by 2 and
    writes by 1.  The calibration run's fill kernel (no reads, COPY_BYTES
    written) must not enter the copy's average: the default --copy-kernel
    matches the multiply kernel only."""
    kib = bench.COPY_BYTES / 1024.0
    fetch = tmp_path / "fetch.csv"
    write = tmp_path / "write.csv"
    cfetch = tmp_path / "cfetch.csv"
    cwrite = tmp_path / "cwrite.csv"
    k = "void lbm::fused_step<34, 15, PF64, false>(...)"
    _counter_csv(fetch, "FETCH_SIZE", [(1, k, 300.0), (1, k, 100.0), (2, k, 200.0), (2, k, 200.0),
                                       (3, "encode_kernel", 9e9)])
    _counter_csv(write, "WRITE_SIZE", [(1, k, 500.0), (2, k, 700.0)])
    fill = "void at::native::vectorized_elementwise_kernel<4, at::native::FillFunctor<float>, ...>"
    mul = "void at::native::vectorized_elementwise_kernel<4, at::native::AUnaryFunctor<float, float, float, " \
          "at::native::binary_internal::MulFunctor<float> >, ...>"
    _counter_csv(cfetch, "FETCH_SIZE", [(6, fill, 0.0), (7, mul, 0.5 * kib), (8, mul, 0.5 * kib)])
    _counter_csv(cwrite, "WRITE_SIZE", [(6, fill, kib), (7, mul, kib), (8, mul, kib)])
    out = tmp_path / "traffic.json"
    args = argparse.Namespace(fetch_csv=str(fetch), write_csv=str(write), copy_fetch_csv=str(cfetch),
                              copy_write_csv=str(cwrite), copy_kernel=bench.COPY_KERNEL, config="C1",
                              precision="fp64", closure="moment", tuning="18,14,8,0",
                              traffic_json=str(out))
    bench.summarize_counters(args)
    data = json.load(open(out))
    ent = data["C1/fp64@18,14,8"]
    assert abs(ent["fetch_scale"] - 2.0) < 1e-12 and ent["write_scale"] == 1.0
    expect = 400.0 * 1024 * 2.0 + 600.0 * 1024
    assert abs(ent["bytes_per_launch"] - expect) < 1e-6
    assert ent["bytes_per_update_algorithmic"] == 176
    assert abs(ent["bytes_per_update_measured"] - expect / 32768) < 1e-9
    # reported only for the same launch on the same kernel source
    tuning = {"block_x": 18, "block_y": 14, "z_chunk": 8}
    assert bench.measured_traffic("C1", "fp64", tuning, path=str(out)) == ent["bytes_per_launch"]
    assert bench.measured_traffic("C1", "fp64", dict(tuning, z_chunk=16), path=str(out)) is None
    assert bench.measured_traffic("C1", "fp32", tuning, path=str(out)) is None
    data["C1/fp64@18,14,8"]["kernel_hash"] = "0" * 16
    json.dump(data, open(out, "w"))
    assert bench.measured_traffic("C1", "fp64", tuning, path=str(out)) is None


def test_committed_traffic_entries_are_well_formed():
    """profiles/traffic.json: every entry names its launch in its key and
    holds positive, consistent byte counts.  Entries taken on an older kernel
    source are kept but not reported (bench.py reports traffic as null)."""
    data = json.load(open(bench.TRAFFIC_JSON))
    assert data
    for key, ent in data.items():
        config, rest = key.rsplit("/", 1)
        prec, launch = rest.split("@")
        assert key == bench.traffic_key(config, prec, ent["tuning"]), key
        assert ent["bytes_per_launch"] > 0 and ent["nodes"] > 0
        assert abs(ent["bytes_per_update_measured"] * ent["nodes"] - ent["bytes_per_launch"]) < 1e-3 * ent["bytes_per_launch"]
        # measured traffic cannot undercut the algorithmic minimum
        assert ent["bytes_per_update_measured"] >= ent["bytes_per_update_algorithmic"], key


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_wave_planes_counts_items_planes_and_waves():
    """34 x 15 workgroups (8 wavefronts) with 32 x 13 output columns: a
    64 x 26 x 10 box has 4 tile columns; z-chunks of 4 give items over output
    planes [0,4), [4,8), [8,10), each marching one staging plane on either
    side (6 + 6 + 4 planes) unless that side is a z wall (5 + 6 + 3)."""
    from paper_2501_00846_amd.workloads import Problem, WALL

    t = {"block_x": 34, "block_y": 15, "z_chunk": 4}
    assert bench.wave_planes([Problem(64, 26, 10)], t) == 4 * 16 * 8
    assert bench.wave_planes([Problem(64, 26, 10, bc=(0, 0, WALL))], t) == 4 * 14 * 8
    # ragged x and y: 65 columns need 3 tiles, 27 rows 3; a chunk longer than nz is nz
    t2 = {"block_x": 32, "block_y": 8, "z_chunk": 64}
    assert bench.wave_planes([Problem(65, 19, 5)], t2) == 3 * 4 * (5 + 2) * 4
    # boxes of an ensemble add up
    assert bench.wave_planes([Problem(64, 26, 10), Problem(64, 26, 10)], t) == 2 * 4 * 16 * 8


def test_alu_ceiling_and_valu_lookup(tmp_path):
    """The ALU floor is the VALU wave-instruction count over 256 CUs x 4 SIMDs
    x 2.4 GHz / 4; the committed count is scaled by wave-planes and reported
    only for the same kernel source and tile shape."""
    assert bench.VALU_ISSUE_PER_S == 614.4e9
    a = bench.alu_ceiling(614.4e9 * 1e-3, 1 << 20, 2.0)  # 1 ms of issue in a 2 ms kernel
    assert a["floor_ms"] == 1.0 and a["frac"] == 0.5
    assert a["ceiling_mlups"] == round((1 << 20) / 1e-3 / 1e6, 1)
    assert bench.alu_ceiling(None, 1, 1.0) is None
    from paper_2501_00846_amd.workloads import Problem

    probs = [Problem(64, 26, 10)]
    t = {"block_x": 34, "block_y": 15, "z_chunk": 4}
    path = tmp_path / "valu.json"
    json.dump({bench.valu_key("C9", "fp32", t): {"kernel_hash": bench.kernel_hash(),
                                                 "valu_per_wave_plane": 600.0}}, open(path, "w"))
    assert bench.valu_per_launch("C9", "fp32", probs, t, path=str(path)) == 600.0 * 4 * 16 * 8
    # another z-chunk of the same shape scales by its own wave-planes
    t8 = dict(t, z_chunk=8)
    assert bench.valu_per_launch("C9", "fp32", probs, t8, path=str(path)) == 600.0 * bench.wave_planes(probs, t8)
    assert bench.valu_per_launch("C9", "fp64", probs, t, path=str(path)) is None
    assert bench.valu_per_launch("C9", "fp32", probs, dict(t, block_x=32, block_y=8), path=str(path)) is None


def test_field_errors_are_relative_norms():
    rng = np.random.default_rng(0)
    ref = {"phi": rng.uniform(0, 1, (4, 5, 6)), "rho": rng.uniform(0.1, 1, (4, 5, 6)),
           "p": rng.normal(size=(4, 5, 6)), "u": rng.normal(size=(3, 4, 5, 6))}
    got = {k: v.copy() for k, v in ref.items()}
    got["u"][2] *= 1.001
    e = bench.field_errors(got, ref)
    assert e["phi"]["l2"] == 0 and e["ux"]["max"] == 0
    assert abs(e["uz"]["l2"] - 1e-3) < 1e-9 and abs(e["uz"]["max"] - 1e-3) < 1e-9
