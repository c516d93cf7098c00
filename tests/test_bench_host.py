"""Host logic of bench.py that needs no GPU: the one-GPU contract and the guard
that reports the committed HBM-traffic figure only while the convolution
source it was measured on is unchanged."""
import hashlib
import importlib.util
import json
import os
import shutil
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SUMMARY = os.path.join("profiles", "conv_family_hbm_traffic_256x256_32rhs.md")
CONV = os.path.join("paper_2405_17696_amd", "csrc", "conv.hip")


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_traffic_figure_follows_the_convolution_source(tmp_path, monkeypatch):
    bench = load_bench()
    text = open(os.path.join(ROOT, SUMMARY)).read()
    fields = dict(line.split(": ", 1) for line in text.splitlines()
                  if line.startswith(("traffic_bytes_per_launch: ", "conv_source_sha256_16: ",
                                      "preconditioner_streams: ")))
    src = open(os.path.join(ROOT, CONV), "rb").read()
    # the committed summary was taken on the current source, in the bench's default configuration
    assert fields["conv_source_sha256_16"] == hashlib.sha256(src).hexdigest()[:16]
    streams = int(fields["preconditioner_streams"])
    assert streams == 2
    assert bench.measured_traffic(streams) == float(fields["traffic_bytes_per_launch"])
    # a launch of the other configuration covers another number of right-hand sides
    assert bench.measured_traffic(3 - streams) is None

    (tmp_path / "profiles").mkdir()
    (tmp_path / "paper_2405_17696_amd" / "csrc").mkdir(parents=True)
    shutil.copy(os.path.join(ROOT, SUMMARY), tmp_path / SUMMARY)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    (tmp_path / CONV).write_bytes(src)
    assert bench.measured_traffic(streams) == float(fields["traffic_bytes_per_launch"])
    (tmp_path / CONV).write_bytes(src + b"\n// changed\n")
    assert bench.measured_traffic(streams) is None
    (tmp_path / CONV).unlink()
    assert bench.measured_traffic(streams) is None
