"""The benchmark's command line on the host: more than one GPU is refused
with a message before any device work, and the kernel-source hash that gates
the measured HBM traffic matches the committed counter summary only for the
sources it was taken on."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout.strip() == ""


def test_traffic_is_gated_by_the_kernel_sources(tmp_path, monkeypatch):
    import bench
    from paper_2011_01316_amd import binding as B
    op = B.KERNEL_SYMBOLS["linear_operator"]
    d = json.load(open(bench.PMC_FILE))
    # a summary taken on other sources gives no traffic
    other = dict(d, kernel_source_hash="0" * 16)
    f = tmp_path / "pmc.json"
    f.write_text(json.dumps(other))
    monkeypatch.setattr(bench, "PMC_FILE", str(f))
    assert bench.measured_traffic(op) is None
    # the same summary with the current hash gives its figure
    same = dict(d, kernel_source_hash=bench.kernel_source_hash())
    f.write_text(json.dumps(same))
    k = d["workloads"]["vortex64_p4"]["kernels"].get(op)
    if k is not None:
        assert bench.measured_traffic(op) == k["bytes_per_launch"]
