"""CPU checks of the benchmark's contract: more than one GPU is refused with
a message, the CPU-baseline leg reports what the JSON line needs, and the
HBM traffic figure is only reported for the kernel sources it was
measured on."""
import json
import os
import subprocess
import sys

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]


def test_cpu_baseline_fields():
    import bench
    h = synth.neighbour_hamiltonian(64, 23, cutoff=4.0, seed=0)
    cpu = bench.cpu_baseline(h, 16)
    assert cpu["kind"] == "oracle" and cpu["unit"] == "GFLOP/s"
    assert cpu["value"] > 0 and cpu["cores"] >= 1 and "16 of 64" in cpu["sample"]


def test_traffic_only_for_the_profiled_sources(tmp_path, monkeypatch):
    import bench
    d = json.load(open(os.path.join(ROOT, "profiles", "traffic_sign23.json")))
    got = bench.measured_traffic("sign23", d.get("graph", 0))
    if d["source_sha256"] == bench.sources_sha256():
        assert got == d["hbm_bytes_per_launch"]
    else:
        assert got is None
    # a profile taken on other sources, or with another graph mode (other
    # launches), is not reported
    prof = tmp_path / "profiles"
    prof.mkdir()
    d["graph"] = 1
    d["source_sha256"] = "0" * 64
    (prof / "traffic_sign23.json").write_text(json.dumps(d))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "sources_sha256", lambda: "f" * 64)
    assert bench.measured_traffic("sign23", 1) is None
    monkeypatch.setattr(bench, "sources_sha256", lambda: "0" * 64)
    assert bench.measured_traffic("sign23", 1) == d["hbm_bytes_per_launch"]
    assert bench.measured_traffic("sign23", 0) is None
