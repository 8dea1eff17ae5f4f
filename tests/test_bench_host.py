"""Host-side logic of bench.py, no GPU: the refusal of more than one GPU, the
algorithmic bytes per element that the roofline divides by the kernel time,
and the lookup of the committed counter traffic."""
import hashlib
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402  (importing it runs no GPU code)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, cwd=ROOT, timeout=300)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


@pytest.mark.parametrize("args,expected", [
    ((25, 20, 4, 8, False), 4616),         # 2-D transport p=4, per-element operators: G 4000 + c, u, u' 600 + map 16
    ((64, 96, 6, 8, True), 1560),          # 3-D transport p=3, shared operator: c, u, u' 1536 + map 24
    ((48, 16, 4, 8, True), 1168),          # 2-D diffusion p=3 (tau*), shared operator
    ((75, 20, 4, 8, False, 300), 16216),   # 2-D conv.-diff. p=4, per element, with 4 x 3 x 5^2 projection entries
    ((25, 20, 4, 4, False), 2316),         # the FP32 operators of the mixed path (map entries stay 4 bytes)
])
def test_algorithmic_bytes_per_element(args, expected):
    assert bench.algorithmic_bytes_per_element(*args) == expected


def test_counter_traffic_follows_the_source_hash_and_launch_shape():
    with open(os.path.join(ROOT, "profiles", "counters.json")) as f:
        d = json.load(f)
    assert d
    for key, rec in d.items():
        src = os.path.join(ROOT, rec.get("source", "paper_1605_03228_amd/csrc/sweep_impl.hpp"))
        with open(src, "rb") as f:
            current = hashlib.sha256(f.read()).hexdigest()[:16] == rec["source_sha16"]
        assert bench.counter_traffic(key, rec["waves"]) == (rec["traffic_bytes"] if current else None), key
        assert bench.counter_traffic(key, rec["waves"] + 100) is None, key
    assert bench.counter_traffic("no such kernel", 4) is None
