"""Host logic of bench.py that needs no GPU: the refusal of several GPUs, the
algorithmic work its rooflines divide by, the roofline record, and the HBM
traffic file written from rocprofv3 counter CSVs (scaled by a plain copy)."""
import csv
import importlib.util
import json
import os
import subprocess
import sys

import pytest

from synth import card_c2

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_kernel_work_of_the_workload(bench):
    card = card_c2()
    # 512 traces of 2048 samples, Q = 32, a 240-sample window: 2 M Q L_h flop per trace
    flop, bound = bench.kernel_work("conv", card, 654, 8)
    assert flop == 2.0 * 512 * 2048 * 32 * 240 == 16106127360.0 and bound == "mfma"
    assert bench.kernel_work("corr", card, 654, 8) == (flop, "mfma")
    # splat: leg table (256 rows x 654 records x 16 B), image, transmittances, fine grid
    fine = 512 * 2048 * 32 * 4
    assert bench.kernel_work("splat", card, 654, 8) == (float(256 * 654 * 16 + 4 * 65536 + 4 * 256 + fine), "hbm")
    # gather: 4 MiB of one group's fine grid per launch = 16 of its 32 traces
    # (16 groups of 32): two launches per adjoint; per launch half the fine
    # grid, the leg table and transmittances, and the partial images written
    # (first launch) or read and written (second): 3 images per group in all
    assert bench.gather_launches(card, 16, 4096) == 2
    w, b = bench.kernel_work("gather", card, 654, 16, 4096)
    assert b == "hbm"
    assert w == pytest.approx((fine + 2 * (256 * 654 * 16 + 4 * 256) + 3 * 16 * 4 * 65536) / 2)
    assert 75e6 < w < 77e6
    # 16-bit storage halves the fine grid per trace: one launch of 32 traces
    assert bench.gather_launches(card, 16, 4096, elem=2) == 1
    assert bench.kernel_work("k_unknown", card, 654, 8) == (None, None)


def test_operator_roofline(bench):
    card = card_c2()
    r = bench.operator_roofline(card, 0.5e-3, 512 * 65536, 654)
    # 2 L_h flop per triple per operator, two operators
    assert r["flop_per_pair"] == 2 * 2 * 240 * 512 * 65536
    assert r["frac_of_fp32"] == pytest.approx(r["flop_per_pair"] / 0.5e-3 / 157.3e12)
    # per operator: image, traces (512 x 2048 FP32), leg table (256 rows x 654
    # records x 16 B), template (32 x 240 + 2 floats)
    per_op = 4 * 65536 + 4 * 512 * 2048 + 16 * 256 * 654 + 4 * (32 * 240 + 2)
    assert r["algorithmic_bytes_per_pair"] == 2 * per_op
    assert r["hbm_frac_at_algorithmic_bytes"] == pytest.approx(2 * per_op / 0.5e-3 / 8e12)
    assert r["hbm_frac_at_algorithmic_bytes"] < 0.01


def test_roofline_record(bench):
    card = card_c2()
    prof = {"conv": (20, 20 * 0.125)}  # 20 launches of 125 us
    r = bench.roofline("conv", prof, 2, card, 654, 8)
    assert r["bound"] == "mfma" and r["unit"] == "TFLOP/s" and r["peak"] == 157.3
    assert r["avg_launch_us"] == pytest.approx(125.0)
    assert r["achieved"] == pytest.approx(16106127360.0 / 125e-6 / 1e12)
    assert r["frac"] == pytest.approx(r["achieved"] / 157.3)
    assert r["launches_per_step"] == 10
    assert bench.roofline("gather", prof, 2, card, 654, 8) is None
    # bf16 piece products: six bf16 products per FP32 product, against the bf16 peak
    r2 = bench.roofline("conv", prof, 2, card, 654, 8, products=2)
    assert r2["peak"] == 2500.0 and r2["work_per_launch"] == 6 * 16106127360.0
    assert r2["achieved"] == pytest.approx(6 * r["achieved"])
    assert r2["fp32_equivalent_TFLOPs"] == pytest.approx(r["achieved"])
    assert r2["fp32_equivalent_frac_of_fp32_peak"] == pytest.approx(r["frac"])
    # storage in 16 bits keeps its own products
    assert bench.roofline("conv", prof, 2, card, 654, 8, elem=2, products=2)["work_per_launch"] == 16106127360.0


def _counter_csv(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for name, value in rows:
            w.writerow({"Kernel_Name": name, "Counter_Name": "X", "Counter_Value": value})


def test_traffic_file(bench, tmp_path, monkeypatch):
    # a 1 GiB copy that the counters see as 512 MiB read and 1 GiB written:
    # fetch values scale by 2, write values by 1
    _counter_csv(tmp_path / "cf.csv", [("__amd_rocclr_copyBuffer", 524288.0)] * 3)
    _counter_csv(tmp_path / "cw.csv", [("__amd_rocclr_copyBuffer", 1048576.0)] * 3)
    _counter_csv(tmp_path / "f.csv", [("void umbir::(anonymous namespace)::k_conv_mfma<32>(float const*)", 100.0),
                                      ("void umbir::(anonymous namespace)::k_conv_mfma<32>(float const*)", 300.0),
                                      ("void umbir::(anonymous namespace)::k_splat<false>(int)", 10.0),
                                      ("void umbir::(anonymous namespace)::k_corr_x3<1>(float const*)", 6.0),
                                      ("void umbir::(anonymous namespace)::k_gather_lds<false, true>(float const*)", 9.0),
                                      ("void at::native::other_kernel", 7.0)])
    _counter_csv(tmp_path / "w.csv", [("void umbir::(anonymous namespace)::k_conv_mfma<32>(float const*)", 4.0),
                                      ("void umbir::(anonymous namespace)::k_splat<false>(int)", 128.0)])
    out = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(out))
    bench.traffic_from(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), str(tmp_path / "cf.csv"),
                       str(tmp_path / "cw.csv"))
    doc = json.load(open(out))
    assert doc["source_sha256"] == bench.source_digest()
    assert doc["calibration"]["fetch_scale"] == pytest.approx(2.0)
    assert doc["calibration"]["write_scale"] == pytest.approx(1.0)
    assert sorted(doc["kernels"]) == ["conv", "corr", "gather", "splat"]  # launch names; other kernels ignored
    assert doc["kernels"]["gather"]["fetch_bytes"] == pytest.approx(9.0 * 2 * 1024)
    assert doc["kernels"]["corr"]["fetch_bytes"] == pytest.approx(6.0 * 2 * 1024)
    assert doc["kernels"]["conv"]["fetch_bytes"] == pytest.approx(200.0 * 2 * 1024)  # mean of 100 and 300 KiB
    assert doc["kernels"]["conv"]["write_bytes"] == pytest.approx(4.0 * 1024)
    assert doc["kernels"]["splat"]["write_bytes"] == pytest.approx(128.0 * 1024)
