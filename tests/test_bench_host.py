"""Host logic of the benchmark and of the profile summaries (no GPU): the per-window work
counts behind the roofline fractions, the one-GPU contract of bench.py, and the rule that a
stored counter summary is used only while the kernel sources it was taken from are unchanged."""
import os
import sqlite3
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2201_06174_amd import profiling  # noqa: E402


@pytest.mark.parametrize("n,s,flops", [(8, 1, 23200), (16, 2, 334080), (16, 1, 313920)])
def test_dense_dft_count(n, s, flops):
    # 8 n^3 K + 8 n^2 K s + 4 n K s^2 with K = n/2 + 1 bins along xl (real input)
    assert bench.dense_dft_flops_per_window(n, s) == flops


@pytest.mark.parametrize("n,flops", [(8, 11520), (16, 122880)])
def test_fft_count(n, flops):
    # 2.5 N log2 N for a real-input FFT of N = n^3 points
    assert bench.algorithmic_flops_per_window(n) == flops


def test_graded_roofline():
    class W:
        n, s = 16, 2
    g = bench.graded(W, 1000, "fp32", 2.0)
    t = 334080 * 1000 / (bench.PEAK_FP32_MFMA_TFLOPS * 1e12) * 1e3
    assert g["t_roof_ms"] == round(t, 4) and g["frac"] == round(t / 2.0, 4)
    # split-BF16 executes three products of each contraction
    g3 = bench.graded(W, 1000, "split_bf16", 2.0)
    assert g3["t_roof_ms"] == round(3 * 334080 * 1000 / (bench.PEAK_BF16_MFMA_TFLOPS * 1e12) * 1e3, 4)
    peaks = {"mfma_f32": {"tflops": bench.PEAK_FP32_MFMA_TFLOPS / 2}}
    gm = bench.graded(W, 1000, "fp32", 2.0, peaks)
    assert gm["t_roof_measured_peak_ms"] == round(2 * t, 4)


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stdout


def test_stored_summaries_follow_the_sources(monkeypatch, tmp_path):
    # a summary whose digest matches the current sources is used; any other digest is ignored
    path = tmp_path / "k_project_fp32_tiny_traffic.txt"
    path.write_text("traffic_bytes_per_launch: 1234\nsource_digest: %s\n" % profiling.source_digest())
    monkeypatch.setattr(bench, "TRAFFIC_DIR", str(tmp_path))
    assert bench.stored_traffic("tiny", "fp32") == 1234.0
    monkeypatch.setattr(profiling, "source_digest", lambda *a, **k: "0" * 16)
    assert bench.stored_traffic("tiny", "fp32") is None


def test_stats_summary_lists_every_kernel(tmp_path):
    db = tmp_path / "run_results.db"
    con = sqlite3.connect(str(db))
    con.execute("create table top_kernels (name text, total_calls int, total_duration real, average real, "
                "percentage real)")
    con.execute("create table kernels (name text, grid_x int, workgroup_x int, duration real)")
    for i in range(40):
        con.execute("insert into top_kernels values (?, 1, ?, ?, 1.0)", ("k%d" % i, 100.0 - i, 100.0 - i))
        con.execute("insert into kernels values (?, 256, 64, ?)", ("k%d" % i, (100.0 - i) * 1e3))
    con.commit()
    con.close()
    md = profiling.stats_markdown(str(db), "t", "cmd", top=5)
    rows = [l for l in md.splitlines() if l.startswith("| `")]
    assert len(rows) == 40 + 5
    assert rows[0].startswith("| `k0`") and rows[40].startswith("| `k0`")


def test_oracle_section_errors_of_the_oracle_itself():
    """The bench's per-output error plumbing: a 'pipeline' holding the full-grid oracle's
    own outputs has zero error against the one-section oracle."""
    import numpy as np
    import torch
    from oracle import oracle as orc
    from paper_2201_06174_amd import synth

    shape, n, s = (20, 24, 18), 8, 2
    V, M = synth.make_volume(synth.VolumeSpec(shape, faults=[synth.centre_fault(shape)]), 5, with_mask=True)
    D, mask = synth.desired_map(M, s)

    class W:
        pass
    w = W()
    w.n, w.s, w.offsets = n, s, synth.cube_stencil(2 * s)
    o = orc.forward(V, orc.Params(n=n, s=s, offsets=w.offsets, fusion="adapt_ls", delta=1e-6, D=D, mask=mask))
    sec = bench.OracleSection(V, w, D, mask, 1e-6)

    class Pipe:
        pass
    p = Pipe()
    p.torch = torch
    p.E = torch.from_numpy(o["E"])
    p.Sm = torch.from_numpy(o["Sm"])
    p.W = torch.from_numpy(np.append(o["W"], 0.0))
    p.S = torch.from_numpy(o["S"])
    e = sec.errors(p)
    assert e["E"] == 0.0 and e["Sm"] == 0.0 and e["W"] < 1e-15 and e["S"] < 1e-15 and e["fallback"] == 0
    # a planted error in one output shows up in that output only
    p.Sm = p.Sm.clone()
    p.Sm[1, :, sec.mid, 3] *= 1.01
    e = sec.errors(p)
    assert e["Sm"] > 1e-3 and e["E"] == 0.0


def test_cpu_model_reads_proc():
    name, count = bench.cpu_model()
    assert isinstance(name, str) and count >= 0
