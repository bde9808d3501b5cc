"""bench.py's host-side contract, without a GPU: the one-GPU refusal, the cluster rule it
reports, and the counter summary it reads (used only while the kernel sources and run
configuration match the ones the counters were taken with)."""
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2511_18071_amd import workload as W  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_default_cluster_rule():
    # one workgroup per 32-column tile of the finest level, at most 256
    assert bench.default_cluster(W.get("bar_513x17")) == 17
    assert bench.default_cluster(W.get("periodic_16385x33")) == 256
    assert bench.default_cluster(W.get("tiny_17x7")) == 1


def test_defaults_match_the_driver_command():
    # the driver runs `bench.py --gpus 1 --steps 20 --warmup 5`: the same as the defaults, on
    # the large single simulation
    a = bench.parse([])
    assert (a.gpus, a.steps, a.warmup, a.workload) == (1, 20, 5, "periodic_16385x33")


def test_counter_summary_is_used_only_for_its_own_configuration():
    path = bench.counters_path("periodic_16385x33")
    if not os.path.exists(path):
        path = bench.counters_path("bar_513x17")
    text = open(path).read()
    fields = dict(re.findall(r"^- ([a-z0-9-]+): `([^`]*)`", text, flags=re.M))
    wl, steps, warm, cl = fields["workload"], int(fields["steps"]), int(fields["warmup"]), int(fields["cluster"])
    got = bench.measured_traffic(wl, steps, warm, cl)
    if fields["kernel-source-sha256"] == bench.kernel_hash():
        assert got == float(fields["hbm-bytes-per-launch"])
    else:
        assert got is None
    assert bench.measured_traffic(wl, steps + 1, warm, cl) is None
    assert bench.measured_traffic(wl, steps, warm, cl + 1) is None
    assert bench.measured_traffic("periodic_65x9", steps, warm, cl) is None
