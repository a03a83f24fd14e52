"""bench.py's contract on the CPU: one GPU only (a request for more exits with a message), and
the counter figures it reports (HBM traffic, VALU issue and barrier shares) come from
profiles/counters.json only while that file was taken on the current kernel sources."""
import json
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
REPO = os.path.dirname(HERE)
sys.path.insert(0, REPO)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(REPO, "bench.py"), "--gpus", "2"],
                       stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in r.stdout


def test_counters_are_of_the_current_kernels():
    import bench
    d = json.load(open(os.path.join(REPO, "profiles", "counters.json")))
    h = bench.kernel_source_hash()
    for name in ("rod_resident_kernel<4,2>", "rod_grid_kernel<4,2>"):
        assert d[name]["source_hash"] == h, (
            "%s: profiles/counters.json was taken on other kernel sources; profile again" % name)
    # the headline workload's figures are found
    assert bench.measured_traffic("rod_resident_kernel<4,2>", 1024, 10) is not None
    assert bench.measured_wave_shares("rod_resident_kernel<4,2>", 1024, 10) is not None
