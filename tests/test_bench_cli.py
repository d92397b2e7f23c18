"""bench.py host logic (CPU): the one-GPU refusal, the traffic records and their
source-hash gate, and the roofline entry built from a profile."""
import hashlib
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=60)
    assert p.returncode == 2
    assert "one GPU" in json.loads(p.stdout.strip().splitlines()[-1])["error"]


def _records(tmp_path, sha):
    f = tmp_path / "traffic.md"
    f.write_text("# t\n\ntraffic-record: class=heff_gemm1_lo kernel=gemm_bf16x3_kernel<0, 128, 128> "
                 f"bytes_per_launch=2.5e+09 sources_sha256={sha}\n\n"
                 "traffic-record: class=heff_gemm2_lo kernel=gemm_bf16x3_kernel<1, 128, 128> "
                 f"bytes_per_launch=1.5e+09 sources_sha256={sha}\n")
    return str(f)


def _sources_sha():
    h = hashlib.sha256()
    for src in bench.TRAFFIC_SOURCES:
        h.update(open(os.path.join(ROOT, src), "rb").read())
    return h.hexdigest()


def test_traffic_records_follow_the_sources(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC_FILE", _records(tmp_path, _sources_sha()))
    rec = bench.measured_traffic()
    assert rec == {"heff_gemm1_lo": ("gemm_bf16x3_kernel<0, 128, 128>", 2.5e9),
                   "heff_gemm2_lo": ("gemm_bf16x3_kernel<1, 128, 128>", 1.5e9)}
    monkeypatch.setattr(bench, "TRAFFIC_FILE", _records(tmp_path, "0" * 64))
    assert bench.measured_traffic() == {}
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.md"))
    assert bench.measured_traffic() == {}


def _run(prec, g1, g2):
    names = ["heff_gemm1", "heff_gemm2", "heff_mix", "heff_gemm1_lo", "heff_gemm2_lo", "heff_mix_lo", "convert"]
    prof = {k: (0, 0.0, 0.0) for k in names}
    sfx = "" if prec == "f64" else "_lo"
    prof["heff_gemm1" + sfx] = g1
    prof["heff_gemm2" + sfx] = g2
    return dict(prec=prec, prof=prof)


@pytest.mark.parametrize("prec", ["f64", "bf16x3"])
def test_roofline_entry(tmp_path, monkeypatch, prec):
    """The dominant stage by summed time; achieved = flops / summed time; frac = achieved / the precision's peak;
    traffic only for split-bf16 runs on the measured workload with current records."""
    monkeypatch.setattr(bench, "TRAFFIC_FILE", _records(tmp_path, _sources_sha()))
    # stage 2 dominates: 10 launches, 20 ms, 6e12 flops -> 300 TFLOP/s
    r = _run(prec, (10, 15.0, 3e12), (10, 20.0, 6e12))
    out = bench.gemm_roofline(r)
    assert out["achieved"] == pytest.approx(300.0)
    assert out["frac"] == pytest.approx(300.0 / bench.PEAK[prec], abs=1e-4)
    assert out["launches"] == 10 and out["avg_launch_ms"] == pytest.approx(2.0)
    assert "stage 2" in out["kernel"]
    if prec == "bf16x3":
        assert out["traffic"] == 1.5e9
        assert bench.gemm_roofline(r, traffic_ok=False)["traffic"] is None
    else:
        assert out["traffic"] is None

