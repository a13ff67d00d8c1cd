"""Host-side logic of bench.py (no GPU): the algorithmic-bytes model, the probe choice, the code hash
that guards the stored traffic counters, the one-GPU contract, and that the committed throughput
and HBM-traffic summaries recompute from their own figures."""
import os
import re
import subprocess
import sys

import numpy as np
import pytest

import bench
import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_algorithmic_bytes_follow_the_method_byte_model():
    """FP32 3D: pass A 4 B per CSR entry + 130 B per particle, pass B 4 + 140, pass C 40 B per
    particle, and a damping sweep (K colour launches) 4 B per entry + 24 B per particle; the column
    (40,160,000 particles, 3,178,450,616 entries) and the 3D cantilever."""
    for n, nnz in ((40_160_000, 3_178_450_616), (1_260_000, 96_714_816)):
        ab = bench.algorithmic_bytes(3, 32, n, nnz, 27)
        assert ab["passA"] == 4 * nnz + 130 * n
        assert ab["passB"] == 4 * nnz + 140 * n
        assert ab["passC"] == 40 * n
        assert abs(27 * ab["passD"] - (4 * nnz + 24 * n)) < 1e-3
    ab = bench.algorithmic_bytes(3, 32, 1_260_000, 96_714_816, 27)
    assert round(ab["passD"] / 1e6, 2) == 15.45
    # FP64 moves more per particle in every pass, the same per entry
    a64 = bench.algorithmic_bytes(3, 64, 1_260_000, 96_714_816, 27)
    for k in ("passA", "passB", "passC", "passD"):
        assert a64[k] > ab[k]


def test_design_bytes_of_the_3d_cantilever():
    """The implementation's own byte count (FP32, D = 3): every array a pass touches once, 2-byte
    LDS slots per entry, pass D's velocities staged and written back per colour launch."""
    pb = bench.design_bytes(3, 32, 1_260_000, 96_714_816, False, 27)
    n, nnz = 1_260_000, 96_714_816
    assert pb["passA"] == n * (8 + 24 + 24 + 12 + 1 + 36 + 36 + 24) + 2 * nnz
    assert pb["passB"] == n * (8 + 24 + 36 + 24 + 1) + 2 * nnz
    assert pb["passC"] == n * (24 + 12 + 1 + 24)
    assert pb["passD"] == n * 24 + (nnz * 6 + n * 8) // 27
    assert round(pb["passD"] / 1e6, 2) == 52.11


def test_host_cpu_reports_counts():
    h = bench.host_cpu()
    assert h["nproc"] >= 1 and 1 <= h["usable"] <= h["nproc"]


def test_tip_probe_is_the_free_end_on_the_axis():
    wb = workloads.c1_cantilever_2d()
    p = bench.tip_probe(wb)
    free = wb.clamped == 0
    assert wb.clamped[p] == 0
    assert wb.X0[p, 0] == wb.X0[free, 0].max()
    mid = 0.5 * (wb.X0[free, 1].min() + wb.X0[free, 1].max())
    assert abs(wb.X0[p, 1] - mid) <= 0.5 * wb.dp + 1e-12
    wb3 = workloads.c2_cantilever_3d(nx=20, ny=5, nz=5)
    p3 = bench.tip_probe(wb3)
    assert np.allclose(wb3.X0[p3, 1:], [2.5 * wb3.dp, 2.5 * wb3.dp])


def test_code_hash_ignores_comments(tmp_path, monkeypatch):
    src = tmp_path / "paper_2103_08932_amd" / "csrc"
    src.mkdir(parents=True)
    for f in bench.KERNEL_SOURCES:
        (src / f).write_text("int f(int x) { return x + 1; }  // one\n/* block */\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h0 = bench.kernel_sources_sha256()
    (src / bench.KERNEL_SOURCES[0]).write_text("// a different comment\nint f(int x)   {\n return x + 1; }\n")
    assert bench.kernel_sources_sha256() == h0
    (src / bench.KERNEL_SOURCES[0]).write_text("int f(int x) { return x + 2; }\n")
    assert bench.kernel_sources_sha256() != h0


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def _profile(name):
    return open(os.path.join(ROOT, "profiles", name)).read().splitlines()


def test_committed_throughput_summary_reproduces_its_roofline():
    """The column's committed throughput summary recomputes: each pass's algorithmic megabytes follow
    the byte model for the body in its header, its GB/s are those bytes over the HIP-event time per
    launch, the dominant kernel is the one with the most time per step and its frac is its GB/s over
    the 8 TB/s HBM peak; the kernel trace of the same workload gives the dominant kernel's average
    launch within 5 % of the HIP-event figure."""
    lines = _profile("throughput_column3d_200x200x1000_fp32.txt")
    head = " ".join(l for l in lines if l.startswith("#"))
    m = re.search(r"([\d,]+) particles, ([\d,]+) CSR entries", head)
    n, nnz = (int(x.replace(",", "")) for x in m.groups())
    model = bench.algorithmic_bytes(3, 32, n, nnz, 27)
    rows = {}
    for l in lines:
        f = l.split()
        if len(f) == 13 and f[1] == "launches":
            rows[f[0]] = dict(launches=int(f[2]), us=float(f[4]), mb=float(f[7]), gbps=float(f[9]))
    assert {"passA", "passB", "passC", "passD"} <= set(rows)
    for p in ("passA", "passB", "passC", "passD"):
        r = rows[p]
        assert abs(r["mb"] - model[p] / 1e6) <= 0.05 + 1e-6 * r["mb"], p
        assert abs(r["gbps"] - r["mb"] / r["us"] * 1e3) <= 1.0, p
    m = re.search(r"dominant kernel (\w+): (\d+) GB/s of (\d+) \(frac ([\d.]+)\)", head)
    dom, gbps, peak, frac = m.group(1), float(m.group(2)), float(m.group(3)), float(m.group(4))
    steps = rows["passA"]["launches"]
    per_step = {p: r["us"] * r["launches"] / steps for p, r in rows.items()}
    assert dom == max(per_step, key=per_step.get)
    assert peak == 8000.0 and abs(gbps - rows[dom]["gbps"]) <= 1.0
    assert abs(frac - rows[dom]["gbps"] / peak) <= 5e-4
    trace = _profile("kernels_column3d_200x200x1000_fp32.txt")
    kname = {"passA": "k_passA<float, 3>", "passB": "k_passB<float, 3, 5>"}[dom]
    avg = [float(l[len(kname):].split()[2]) for l in trace if l.startswith(kname)]
    assert avg, kname
    assert abs(avg[0] - rows[dom]["us"]) <= 0.05 * rows[dom]["us"], (avg[0], rows[dom]["us"])


@pytest.mark.parametrize("name", ["column3d_200x200x1000", "cantilever3d_500x50x50"])
def test_committed_traffic_summary_recomputes(name):
    """The committed HBM-traffic summaries recompute: the calibration factors are a 1 GiB copy's
    bytes over the counters' readings of it, each pass's traffic is its FETCH_SIZE and WRITE_SIZE
    scaled by them (the figure bench.py reports), its ratio is traffic over the byte model's bytes
    for the body in the header."""
    lines = _profile(f"hbm_traffic_{name}_fp32.txt")
    head = " ".join(l for l in lines if l.startswith("#"))
    m = re.search(r"([\d,]+) particles, ([\d,]+) CSR entries", head)
    n, nnz = (int(x.replace(",", "")) for x in m.groups())
    model = bench.algorithmic_bytes(3, 32, n, nnz, 27)
    m = re.search(r"reads FETCH_SIZE (\d+) KiB and WRITE_SIZE (\d+) KiB per launch -> factors ([\d.]+) \(fetch\) and "
                  r"([\d.]+) \(write\)", head)
    fk, wk, ff, wf = int(m.group(1)), int(m.group(2)), float(m.group(3)), float(m.group(4))
    gib_kib = 1 << 20
    assert abs(ff - gib_kib / fk) < 5e-4 and abs(wf - gib_kib / wk) < 5e-4
    stored = {l.split()[1]: int(l.split()[2]) for l in lines if l.startswith("traffic ")}
    seen = 0
    for l in lines:
        f = l.split()
        if len(f) >= 9 and f[0] == "#" and f[1] in ("passA", "passB", "passC", "passD"):
            p = f[1]
            fetch, write, traffic_mb, alg_mb, ratio = (float(x) for x in (f[-6], f[-5], f[-4], f[-3], f[-1]))
            t = fetch * 1024 * (gib_kib / fk) + write * 1024 * (gib_kib / wk)
            assert abs(t / 1e6 - traffic_mb) <= 0.01 + 1e-5 * traffic_mb, p
            assert abs(stored[p] - t) <= 1e-5 * t + 1e4, p
            assert abs(alg_mb - model[p] / 1e6) <= 0.01 + 1e-6 * alg_mb, p
            assert abs(ratio - traffic_mb / alg_mb) <= 0.006, p
            seen += 1
    assert seen == 4
