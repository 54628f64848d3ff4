"""Host checks of bench.py that need no GPU: the one-GPU contract and the
record of measured HBM traffic it reads."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    """bench.py measures one GPU: --gpus 2 exits with status 2 and says why,
    before touching a device."""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_record_is_well_formed():
    """The measured traffic of the integration kernel (rocprofv3 FETCH_SIZE /
    WRITE_SIZE, copy-calibrated) is stored per region-step with the source hash
    it belongs to; bench.py reports it only while the sources still hash to it."""
    sys.path.insert(0, ROOT)
    import bench
    with open(os.path.join(ROOT, "profiles", "traffic_uniform.json")) as f:
        t = json.load(f)
    assert t["workload"] == "uniform" and t["kernel"] == "integrate_persistent_kernel"
    assert abs(t["fetch_bytes_per_region_step"] + t["write_bytes_per_region_step"]
               - t["bytes_per_region_step"]) < 1e-9
    # at least the algorithmic bytes (4 B written + 4 B per edge read, 13.4 edges per row)
    assert t["bytes_per_region_step"] > 57.0
    assert len(t["kernel_source_sha"]) == 16 and len(bench._src_sha()) == 16
