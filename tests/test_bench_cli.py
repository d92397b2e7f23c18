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



def test_launch_gaps_from_a_trace(tmp_path, capsys):
    """The launch-gap summary of a synthetic rocprofv3 CSV pair: two overlapping kernels, a gap, a third kernel,
    inside one timed range; a kernel outside the range is ignored."""
    d = tmp_path / "trace" / "host"
    d.mkdir(parents=True)
    (d / "x_kernel_trace.csv").write_text(
        '"Kind","Kernel_Name","Start_Timestamp","End_Timestamp"\n'
        '"KERNEL_DISPATCH","a",1000,5000\n'
        '"KERNEL_DISPATCH","b",4000,6000\n'
        '"KERNEL_DISPATCH","c",8000,9000\n'
        '"KERNEL_DISPATCH","d",20000,21000\n')
    (d / "x_marker_api_trace.csv").write_text(
        '"Domain","Function","Process_Id","Start_Timestamp","End_Timestamp"\n'
        '"MARKER_CORE_API","timed:f64",1,500,10000\n')
    bench.launch_gaps(str(tmp_path / "trace"))
    r = json.loads(capsys.readouterr().out.strip().splitlines()[-1])["ranges"]
    assert len(r) == 1 and r[0]["range"] == "f64" and r[0]["kernels"] == 3
    assert r[0]["busy_share"] == round(6000 / 9500, 4)        # [1000, 6000] and [8000, 9000]
    assert r[0]["gap_share"] == round(2000 / 9500, 4)
    assert r[0]["lead_us"] == 0.5 and r[0]["tail_us"] == 1.0


def test_mfma_counters_from_a_trace(tmp_path, capsys):
    """The MFMA summary of a synthetic rocprofv3 --pmc CSV: two dispatches of one kernel, 1 ms each."""
    d = tmp_path / "pmc"
    d.mkdir()
    (d / "k_kernel_trace.csv").write_text(
        '"Dispatch_Id","Kernel_Name","Start_Timestamp","End_Timestamp"\n'
        '"1","g",0,1000000\n"2","g",2000000,3000000\n')
    rows = ['"Dispatch_Id","Kernel_Name","Counter_Name","Counter_Value"']
    for did in (1, 2):
        rows += [f'"{did}","g","SQ_INSTS_VALU_MFMA_MOPS_BF16","{1.25e15 * 1e-3 / 512}"',
                 f'"{did}","g","MfmaUtil","{40.0 + 20 * (did - 1)}"']
    (d / "k_counter_collection.csv").write_text("\n".join(rows) + "\n")
    bench.mfma_counters(str(d))
    k = json.loads(capsys.readouterr().out.strip().splitlines()[-1])["kernels"][0]
    assert k["dispatches"] == 2 and k["avg_ms"] == 1.0
    assert k["mfma_bf16_tflops"] == 1250.0 and k["mfma_bf16_peak_share"] == 0.5
    assert k["mfma_util_pct"] == 50.0


def test_counter_passes_merge_by_kernel(tmp_path, capsys):
    """Two --pmc passes over the same run (MFMA counters, then LDS counters) merge into one row per kernel; the
    percent metrics are duration-weighted and the wait counters are taken per wave cycle of their own pass."""
    def pas(name, counters):
        d = tmp_path / name
        d.mkdir()
        (d / "k_kernel_trace.csv").write_text(
            '"Dispatch_Id","Kernel_Name","Start_Timestamp","End_Timestamp"\n"1","g",0,1000000\n"2","g",0,3000000\n')
        rows = ['"Dispatch_Id","Kernel_Name","Counter_Name","Counter_Value"']
        for did in (1, 2):
            rows += [f'"{did}","g","{c}","{v[did - 1]}"' for c, v in counters.items()]
        (d / "k_counter_collection.csv").write_text("\n".join(rows) + "\n")
        return str(d)
    a = pas("a", {"SQ_INSTS_VALU_MFMA_MOPS_F64": [39.3e12 * 1e-3 / 512, 3 * 39.3e12 * 1e-3 / 512],
                  "MfmaUtil": [10.0, 30.0]})
    b = pas("b", {"LdsUtil": [20.0, 12.0], "SQ_WAIT_ANY": [10.0, 30.0], "SQ_WAVE_CYCLES": [100.0, 100.0]})
    bench.mfma_counters([a, b])
    k = json.loads(capsys.readouterr().out.strip().splitlines()[-1])["kernels"][0]
    assert k["dispatches"] == 2 and k["avg_ms"] == 2.0
    assert k["mfma_f64_tflops"] == 39.3 and k["mfma_f64_peak_share"] == 0.5
    assert k["mfma_util_pct"] == 25.0 and k["lds_util_pct"] == 14.0
    assert k["sq_wait_any_per_wave_cycle"] == 0.2


def test_traffic_summary_writes_current_records(tmp_path, capsys, monkeypatch):
    """The traffic summary of synthetic --pmc CSVs calibrates by the copy and stamps the records with the sources
    hash, so that measured_traffic() reads them back."""
    def pmc(name, counter, rows):
        d = tmp_path / name
        d.mkdir()
        lines = ['"Dispatch_Id","Kernel_Name","Counter_Name","Counter_Value"']
        lines += [f'"{i}","{k}","{counter}","{v}"' for i, (k, v) in enumerate(rows)]
        (d / "run_counter_collection.csv").write_text("\n".join(lines) + "\n")
        return str(d)
    g1, g2 = "void gemm_bf16x3_kernel<0, 128, 128>(int)", "void gemm_bf16x3_kernel<1, 128, 128>(int)"
    # the tuner's variant: the stage-1 record must come from the variant with the most dispatches
    g1p = "void idmrg::(anonymous namespace)::gemm_bf16x3_persist_kernel<0>(idmrg::GemmTask const*, int)"
    f = pmc("f", "FETCH_SIZE", [(g1, 1000.0), (g1, 1000.0), (g2, 500.0)] + [(g1p, 800.0)] * 3)
    w = pmc("w", "WRITE_SIZE", [(g1, 100.0), (g1, 100.0), (g2, 50.0)] + [(g1p, 900.0)] * 3)
    cf = pmc("cf", "FETCH_SIZE", [("copy", 131072.0)] * 3)          # factor 0.5
    cw = pmc("cw", "WRITE_SIZE", [("copy", 262144.0)] * 3)          # factor 1
    bench.traffic_summary(f, w, cf, cw)
    out = capsys.readouterr().out
    rec = tmp_path / "traffic.md"
    rec.write_text(out)
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(rec))
    t = bench.measured_traffic()
    assert t["heff_gemm1_lo"] == ("gemm_bf16x3_persist_kernel<0>", 800 * 1024 / 0.5 + 900 * 1024)
    assert t["heff_gemm2_lo"][1] == 500 * 1024 / 0.5 + 50 * 1024
