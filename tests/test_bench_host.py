"""Host logic of bench.py (no GPU): the one-GPU contract, the steps a launch advances, the
kernel-name keys, and the rocprofv3 summary it writes and reads back (counter scaling by the
copy calibration, bytes per launch against the algorithmic ones)."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_multi_gpu_request_exits_with_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


class FakeSim:
    def __init__(self, ring, depth):
        self.ring, self.depth = ring, depth

    def fusion(self, model):
        return (self.ring, 16 if self.ring else 0)

    def fusion_depth(self, model):
        return self.depth


@pytest.mark.parametrize("ring,depth,want", [(0, 2, 1), (0, 3, 1), (8, 2, 2), (4, 3, 3), (8, 3, 3), (16, 3, 2)])
def test_launch_steps(ring, depth, want):
    # three steps per launch only with a ring of 4 or 8 rows (lbm_set_fusion_depth)
    assert bench.launch_steps(FakeSim(ring, depth), "K") == want


def test_step_kernel_keys_prefer_the_fused_kernels():
    keys = bench.step_kernel_keys("K", "f32")
    assert [k for k, _ in keys] == ["k_step3", "k_step3n", "k_step2", "k_step"]
    assert keys[0][1] == "k_step3<5, 1, "
    assert bench.step_kernel_keys("BGK", "f64")[1][1] == "k_step3n<0, 0, "
    assert bench.step_kernel_keys("BGK", "f64")[3][1] == "k_step<0, 0, "


def _write_csv(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as fh:
        fh.write(",".join(header) + "\n")
        for r in rows:
            fh.write(",".join(str(v) for v in r) + "\n")


def test_profile_summary_round_trip(tmp_path, monkeypatch):
    out = tmp_path / "run"
    prof = tmp_path / "profiles"
    monkeypatch.setattr(bench, "PROFILE_DIR", str(prof))
    n = 64
    k3 = "void (anonymous namespace)::k_step3<5, 1, 4, 64>(float const*, ...)"
    k1 = "void (anonymous namespace)::k_step<0, 1, 1>(float const*, ...)"
    _write_csv(str(out / "rp_trace" / "b_kernel_stats.csv"), ["Name", "Calls", "AverageNs", "MinNs", "MaxNs"],
               [[f'"{k3}"', 4, 3000.0, 2900.0, 3100.0], [f'"{k1}"', 2, 1000.0, 990.0, 1010.0]])
    cc = ["Kernel_Name", "Counter_Value"]
    # the calibration copy moves 1 GiB each way; FETCH_SIZE reads half of it, WRITE_SIZE all
    _write_csv(str(out / "rp_copy_fetch" / "c_counter_collection.csv"), cc, [["copyBuffer", 524288.0]])
    _write_csv(str(out / "rp_copy_write" / "c_counter_collection.csv"), cc, [["copyBuffer", 1048576.0]])
    _write_csv(str(out / "rp_fetch" / "b_counter_collection.csv"), cc,
               [[f'"{k3}"', 100.0], [f'"{k3}"', 110.0], [f'"{k1}"', 40.0]])
    _write_csv(str(out / "rp_write" / "b_counter_collection.csv"), cc, [[f'"{k3}"', 50.0], [f'"{k1}"', 30.0]])
    _write_csv(str(out / "rp_valu" / "b_counter_collection.csv"), cc, [[f'"{k3}"', 97.0]])
    # flop counters: one row per counter and dispatch; the single-step K kernel gives the
    # algorithmic flops per node update, the three-step one the executed flops (halo included)
    k1k = "void (anonymous namespace)::k_step<5, 1, 1>(float const*, ...)"
    fc = ["Kernel_Name", "Counter_Name", "Counter_Value"]
    frows = []
    for kern, (add, mul, fma, trans) in ((k3, (30, 20, 100, 3)), (k1k, (9, 6, 30, 1))):
        for c, v in zip(bench.flop_counters("f32"), (add, mul, fma, trans)):
            frows.append([f'"{kern}"', c, v * n * n / 64])
    _write_csv(str(out / "rp_flops" / "b_counter_collection.csv"), fc, frows)
    bench.profile_summary(str(out), "f32", n, bench.profile_commands("f32"))
    counters = (prof / "step_kernels_f32_dsl4096_counters.md").read_text()
    blob = json.loads(counters.split("```json", 1)[1].split("```", 1)[0])
    alg = n * n * 72
    assert blob["algorithmic_bytes"] == alg
    assert blob["scale"] == {"fetch": 2.0, "write": 1.0}
    rec = blob["per_launch"]["K"]
    assert rec["kernel"] == "k_step3"  # the three-step kernel is reported before the others
    assert rec["hbm_bytes"] == int(round(105.0 * 1024 * 2.0 + 50.0 * 1024))
    assert rec["vs_algorithmic"] == round(rec["hbm_bytes"] / alg, 4)
    assert rec["valu_busy"] == 0.97
    assert rec["flops_per_update"] == 9 + 6 + 1 + 2 * 30
    assert rec["executed_flops_per_update"] == round((30 + 20 + 3 + 2 * 100) / 3, 2)
    assert blob["per_launch"]["BGK"]["kernel"] == "k_step"
    # read back through the bench's own reader while the step sources hash as recorded
    assert bench.measured_traffic("K", "f32") == rec["hbm_bytes"]
    assert bench.measured_valu_busy("K", "f32") == 0.97
    # the roofline entry takes its bound from the counters: K is VALU-bound (0.97), so "alu" with
    # the algorithmic flops per launch over the launch time against the FP32 vector peak
    roof = bench.roofline_block("K", "f32", "k_step3", n * n, 72, 3, 10.0, 8.0, 4096)
    assert roof["bound"] == "alu" and roof["unit"] == "TFLOP/s" and roof["peak"] == 157.3
    assert roof["achieved"] == round(76 * n * n * 3 / 10e-6 / 1e12, 2)
    assert roof["frac"] == round(roof["achieved"] / 157.3, 4)
    assert roof["hbm"]["frac_at_18s_bytes_per_update"] == round(3 * roof["hbm"]["frac_at_bytes_per_launch"], 4)
    assert roof["traffic"] == rec["hbm_bytes"] and roof["limiter"] == "valu-issue"
    # BGK has no VALUBusy record: HBM bound by default, at the algorithmic bytes per launch
    roof = bench.roofline_block("BGK", "f32", "k_step", n * n, 72, 1, 10.0, 8.0, 4096)
    assert roof["bound"] == "hbm" and roof["frac"] == round(n * n * 72 / 10e-6 / 1e9 / 8000.0, 4)
    trace = (prof / "step_kernels_f32_dsl4096_trace.md").read_text()
    assert "| k_step3<K, f32> | 4 | 3.00 |" in trace
    # a summary taken from other sources is not used
    (prof / "step_kernels_f32_dsl4096_counters.md").write_text(counters.replace(blob["step_source_hash"], "0" * 16))
    assert bench.measured_traffic("K", "f32") is None


@pytest.mark.parametrize("prec", ["f32", "f64", "f16"])
def test_profiles_keyed_to_current_sources(prec):
    # the committed counter summaries were taken from the step kernels as they are now: every
    # model's record is found (the bench reports measured traffic from them only while the sources
    # hash to the recorded value), so a kernel change without new counters fails here
    for model in bench.MODEL_ORDER:
        rec = bench.counter_record(model, prec)
        assert rec is not None, (prec, model, bench.step_source_hash())
        assert rec["hbm_bytes"] > 0
