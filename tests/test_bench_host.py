"""Host-side checks of the measurement tooling (no GPU): the bench refuses
more than one GPU, every kernel the bench or the profile summaries name has
an algorithmic byte count, and the counter summary scales the raw
FETCH_SIZE / WRITE_SIZE by the calibration copy."""
import csv
import json
import os
import subprocess
import sys

from paper_1510_05218_amd import profiling

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_short_name_of_rocprof_names():
    raw = ("void thiim::k_blocked<32, 16, 2, thiim::Pol64<thiim::CompactCoefs> >"
           "(thiim::Pol64<thiim::CompactCoefs>, HIP_vector_type<double, 2u> const*, "
           "HIP_vector_type<double, 2u>*, thiim::Geo, int)")
    assert profiling.short_name(raw) == "k_blocked<32,16,2,Pol64<CompactCoefs>>"
    assert profiling.short_name("thiim::k_adjoint<64, 8, thiim::AdjPol64<false> >") == \
        "k_adjoint<64,8,AdjPol64<false>>"


def test_bench_kernels_have_byte_counts():
    for key, name in bench.SWEEP_KERNEL.items():
        assert name in profiling.ALG_BYTES_PER_CELL, key
        # per-launch figure / iterations per launch = the bench's per-LUP figure
        per_lup = profiling.ALG_BYTES_PER_CELL[name] / bench.ITERS_PER_LAUNCH[key[0]]
        if key[0] != "naive":  # the naive iteration is two launches of different size
            assert per_lup == bench.BYTES_PER_LUP[key], key
    assert profiling.ALG_BYTES_PER_CELL["k_adjoint<64,8,AdjPol64<false>>"] == \
        bench.ADJ_BYTES_PER_LUP


def _counter_csv(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Value"])
        w.writeheader()
        for name, kib in rows:
            w.writerow({"Kernel_Name": name, "Counter_Value": kib})


def test_traffic_summary_scales_by_calibration_copy(tmp_path):
    n = 1000
    copy = "__amd_rocclr_copyBuffer"
    kern = "void thiim::k_fused<64, 8, thiim::CompactCoefs>(...)"
    # the counter reads the 4 GiB copy as 2x its bytes on fetch, 1x on write
    _counter_csv(tmp_path / "f.csv", [(copy, 2 * 2 ** 32 / 1024), (kern, 800.0), (kern, 1200.0)])
    _counter_csv(tmp_path / "w.csv", [(copy, 2 ** 32 / 1024), (kern, 300.0), (kern, 300.0)])
    out = profiling.traffic_summary(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), n,
                                    str(tmp_path / "t.json"), "cmd")
    assert out["fetch_counter_scale"] == 2.0 and out["write_counter_scale"] == 1.0
    k = out["kernels"]["k_fused<64,8,CompactCoefs>"]
    assert k["dispatches"] == 2
    assert k["read_bytes_per_launch"] == 1000.0 * 1024 / 2
    assert k["write_bytes_per_launch"] == 300.0 * 1024
    assert k["bytes_per_cell"] == (512000.0 + 307200.0) / n
    assert k["alg_bytes_per_cell"] == 400
    assert json.load(open(tmp_path / "t.json"))["source_hash"] == profiling.source_hash()


def test_code_balance_model_against_committed_counters():
    """The overlapped-tile code-balance model (the GPU form of the paper's
    Eq. 12) against the committed rocprofv3 counter summary of the 512^3
    sweeps: every temporally blocked sweep of the table lies within
    [0.7, 1.1] of its model (below it where ring re-reads hit in the caches,
    above it by partial cache lines), the measured bytes per update fall
    with T in FP64 compact storage, and the committed table is the one the
    generator makes from the committed summary."""
    n = 512
    m64 = profiling.code_balance(32, 16, 2, 13 * 16, 12 * 16, n, n)
    assert abs(m64 - 261.953125) < 1e-9
    path = os.path.join(ROOT, "profiles", "traffic_thiim_512cubed.json")
    md, rows = profiling.balance_table(path, n)
    got = {name: (T, model, meas) for name, _, T, _, model, meas in rows}
    assert len(got) == len(profiling.BALANCE_CASES)
    for name, (T, model, meas) in got.items():
        assert 0.7 * model <= meas <= 1.1 * model, (name, meas, model)
    assert got["k_blocked<32,16,2,Pol64<CompactCoefs>>"][2] < \
        0.6 * got["k_fused<64,8,CompactCoefs>"][2]
    assert md in open(os.path.join(ROOT, "profiles", "b_per_lup_vs_T.md")).read()
