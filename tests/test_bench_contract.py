"""The benchmark script's contract, checked without a GPU: one GPU only, the
CPU-baseline leg's fields, and measured-traffic entries that name compiled
region shapes."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1303_0107_amd import inputs as I, lbm  # noqa: E402

PREC = {"f64": lbm.LBM_F64, "f32": lbm.LBM_F32, "f16": lbm.LBM_F32_S_F16,
        "bf16": lbm.LBM_F32_S_BF16}


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_cpu_baseline_fields():
    wl = I.CORRECTNESS_128x64
    out = bench.cpu_baseline(wl.types(), wl, 0.2)
    assert {"value", "unit", "cores", "kind", "sample"} <= set(out)
    assert out["unit"] == "MLUPS" and out["kind"] == "oracle"
    assert out["value"] > 0 and out["cores"] >= 1
    assert wl.name in out["sample"]
    one = out["single_thread"]
    assert one["cores"] == 1 and one["value"] > 0 and one["unit"] == "MLUPS"
    assert isinstance(out["cpu_model"], str) and out["cpu_model"]
    assert 0 < out["mflups"] < out["value"]


def test_limiter_and_measured_hbm_fields():
    roof = {}
    bench.hbm_and_limiter(roof, 8.5e6, 1.0e6, 0.0135)
    assert roof["hbm_measured_GBs"] == pytest.approx(8.5e6 / 13.5e-6 / 1e9, rel=1e-3)
    assert roof["hbm_measured_frac"] == pytest.approx(roof["hbm_measured_GBs"] / 8000, rel=1e-3)
    lim = roof["limiter"]
    assert lim["bound"] == "valu" and lim["peak"] == pytest.approx(614.4)
    assert lim["frac"] == pytest.approx(1.0e6 / 13.5e-6 / 614.4e9, rel=1e-3)
    roof = {}
    bench.hbm_and_limiter(roof, None, None, 0.0135)
    assert roof["hbm_measured_GBs"] is None and roof["limiter"] is None


def test_measured_traffic_names_compiled_shapes():
    names = set(bench.workloads())
    for (workload, prec, shape), valu in bench.MEASURED_VALU_PER_FULL_LAUNCH.items():
        assert workload in names
        assert 0 <= shape < lbm.lbm_tb_variant_count(PREC[prec])
        assert valu > 0
    for (workload, prec, shape), full in bench.MEASURED_TRAFFIC_PER_FULL_LAUNCH.items():
        assert workload in names
        assert 0 <= shape < lbm.lbm_tb_variant_count(PREC[prec])
        assert full > 0
    for table in (bench.MEASURED_TRAFFIC_PER_LAUNCH, bench.MEASURED_VALU_PER_LAUNCH):
        for (workload, prec, shape, order), per_launch in table.items():
            assert workload == bench.BATCH_WORKLOAD
            assert 0 <= shape <= lbm.lbm_tb_variant_count(PREC[prec])  # count = one step
            assert order in (0, 1)
            assert per_launch > 0


@pytest.mark.parametrize("workload", ["distributor-1024x512-L3", "channel-1024x512"])
def test_workloads_are_the_named_lattices(workload):
    wl = bench.workloads()[workload]
    t = wl.types()
    assert t.shape == (512, 1024)
    assert (t != 0).sum() > 0
