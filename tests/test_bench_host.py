"""Host logic of the benchmark: the rocprofv3 summaries behind its roofline.

The summaries are read back by the benchmark (HBM bytes per launch for the
`traffic` field) only when they were taken on the current kernel source.  These
CPU tests feed small rocprofv3-style CSV files through the summarisers, with the
kernel names the library's step kernels carry, and check the figures and the
read-back.
"""
import csv
import os

import pytest

import bench

ODD = "void rflbm::(anonymous namespace)::step_row_kernel<0, 7, true, false, true>(rflbm::StepArgs)"
EVEN = "void rflbm::(anonymous namespace)::step_wave_kernel<0, 7, true>(rflbm::StepArgs)"
COPY = "void rflbm::(anonymous namespace)::copy_kernel(rflbm::u32x4*, rflbm::u32x4 const*, unsigned long)"
OTHER = "void rflbm::(anonymous namespace)::step_kernel<0, false, 7, true, true>(rflbm::StepArgs)"


def write_csv(path, fields, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=fields)
        w.writeheader()
        w.writerows(rows)


@pytest.fixture
def fake_root(tmp_path, monkeypatch):
    root = tmp_path / "root"
    (root / "profiles").mkdir(parents=True)
    monkeypatch.setattr(bench, "ROOT", str(root))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(root / "profiles" / "step_f32_512_traffic.txt"))
    monkeypatch.setattr(bench, "kernel_hash", lambda: "0123456789abcdef")
    return root


def test_traffic_and_trace_summaries(tmp_path, fake_root, monkeypatch):
    dims = (8, 8, 8)
    algo = 216 * 8 * 8 * 8  # bytes per launch
    out = tmp_path / "out"
    # FETCH_SIZE reads half the fetched bytes, WRITE_SIZE all written bytes (KiB)
    kib = 1024.0
    fetch = [dict(Kernel_Name=COPY, Counter_Name="FETCH_SIZE", Counter_Value=2 ** 30 / 2 / kib)]
    write = [dict(Kernel_Name=COPY, Counter_Name="WRITE_SIZE", Counter_Value=2 ** 30 / kib)]
    for name, excess in ((EVEN, 1.0), (ODD, 1.02)):
        for _ in range(3):
            fetch.append(dict(Kernel_Name=name, Counter_Name="FETCH_SIZE", Counter_Value=excess * algo / 4 / kib))
            write.append(dict(Kernel_Name=name, Counter_Name="WRITE_SIZE", Counter_Value=algo / 2 / kib))
    write_csv(str(out / "prof_fetch" / "fetch_counter_collection.csv"), ["Kernel_Name", "Counter_Name", "Counter_Value"], fetch)
    write_csv(str(out / "prof_write" / "write_counter_collection.csv"), ["Kernel_Name", "Counter_Name", "Counter_Value"], write)
    stats = [dict(Name=EVEN, Calls=35, AverageNs=4000.0, MinNs=3900, MaxNs=4100),
             dict(Name=ODD, Calls=35, AverageNs=5000.0, MinNs=4900, MaxNs=5100),
             dict(Name="void other_kernel()", Calls=1, AverageNs=1.0, MinNs=1, MaxNs=1)]
    write_csv(str(out / "prof_trace" / "trace_kernel_stats.csv"), ["Name", "Calls", "AverageNs", "MinNs", "MaxNs"], stats)

    traffic, dur = bench.summarize_profiles(str(out), dims=dims)
    assert traffic["even"] == pytest.approx(algo)
    assert traffic["odd"] == pytest.approx(algo * (1 + 0.02 / 2))
    assert dur == {"even": 4000.0, "odd": 5000.0}
    text = (fake_root / "profiles" / "step_f32_512_traffic.txt").read_text()
    assert "even_traffic_over_algorithmic = 1.0000" in text and "odd_traffic_over_algorithmic = 1.0100" in text
    trace = (fake_root / "profiles" / "step_f32_512_kernel_trace.txt").read_text()
    assert EVEN in trace and ODD in trace and "other_kernel" not in trace
    assert f"{algo / 4500e-9 / 1e9:.1f} GB/s" in trace

    # read back by the benchmark only while the kernel source is the profiled one
    assert bench.measured_traffic() == pytest.approx(algo * (1 + 0.01 / 2))
    monkeypatch.setattr(bench, "kernel_hash", lambda: "fedcba9876543210")
    assert bench.measured_traffic() is None


def test_valu_summary(tmp_path, fake_root):
    dims = (8, 8, 8)
    n = 8 * 8 * 8
    out = tmp_path / "out"
    rows = []
    for name, per_node, salu in ((EVEN, 711, 10), (ODD, 833, 20), (OTHER, 763, 30)):
        for _ in range(3):
            rows.append(dict(Kernel_Name=name, Counter_Name="SQ_INSTS_VALU", Counter_Value=per_node * n / 64))
            rows.append(dict(Kernel_Name=name, Counter_Name="SQ_INSTS_SALU", Counter_Value=salu * n / 64))
    rows.append(dict(Kernel_Name=COPY, Counter_Name="SQ_INSTS_VALU", Counter_Value=1.0))
    write_csv(str(out / "prof_valu_f32" / "valu_counter_collection.csv"), ["Kernel_Name", "Counter_Name", "Counter_Value"], rows)
    # kernel durations come from the trace summary of the same kernel source
    (fake_root / "profiles" / "step_f32_512_kernel_trace.txt").write_text(
        "# command: ...\n# kernel_source_hash = 0123456789abcdef\nName | Calls | AverageNs | MinNs | MaxNs\n"
        f"{EVEN} | 35 | 4000 | 3900 | 4100\n")
    path = bench.summarize_valu(str(out), "f32", dims=dims)
    text = open(path).read()
    # issue time: 711 n / 64 wave instructions x 2.63 cycles / (1024 SIMDs x 2.4 GHz)
    issue = 711 * n / 64 * bench.FMA_CYCLES_PER_WAVE_INSTR / (1024 * 2.4e9) * 1e3
    assert f"step_wave_kernel<0, 7, true> | 3 | 711 | 10 | {issue:.3f} | 0.004 | {100 * issue / 0.004:.1f}" in text
    assert "step_row_kernel<0, 7, true, false, true> | 3 | 833 | 20 |" in text
    assert "step_kernel<0, false, 7, true, true> | 3 | 763 | 30 |" in text
    # no duration for a kernel the trace lacks
    assert any(l.startswith("step_row_kernel") and l.endswith("| - | -") for l in text.splitlines())
    assert "copy_kernel" not in text


def test_16bit_trace_summary(tmp_path, fake_root):
    dims = (8, 8, 8)
    out = tmp_path / "out"
    even = "void rflbm::(anonymous namespace)::step_kernel<1, false, 7, false, true>(rflbm::StepArgs)"
    odd = "void rflbm::(anonymous namespace)::step_kernel<1, true, 7, false, true>(rflbm::StepArgs)"
    stats = [dict(Name=even, Calls=3, AverageNs=3000.0, MinNs=2990, MaxNs=3010),
             dict(Name=odd, Calls=3, AverageNs=3400.0, MinNs=3390, MaxNs=3410),
             dict(Name=COPY, Calls=1, AverageNs=100.0, MinNs=100, MaxNs=100)]
    write_csv(str(out / "prof_trace_f16" / "trace_kernel_stats.csv"), ["Name", "Calls", "AverageNs", "MinNs", "MaxNs"], stats)
    path = bench.summarize_trace(str(out), "f16", dims=dims)
    text = open(path).read()
    assert even in text and odd in text and "copy_kernel" not in text
    n = 8 * 8 * 8
    assert f"mean step kernel: 3200 ns -> {108 * n / 3200e-9 / 1e9:.1f} GB/s" in text
    assert f"{n / 3200e-9 / 1e6:.0f} MLUPS" in text


def test_batch_trace_summary(tmp_path, fake_root):
    out = tmp_path / "out"
    even = "void rflbm::(anonymous namespace)::batch_kernel<0, false, 7, true, false>(rflbm::BatchArgs)"
    odd = "void rflbm::(anonymous namespace)::batch_kernel<0, true, 7, true, false>(rflbm::BatchArgs)"
    stats = [dict(Name=even, Calls=30, AverageNs=800.0, MinNs=790, MaxNs=810),
             dict(Name=odd, Calls=30, AverageNs=900.0, MinNs=890, MaxNs=910),
             dict(Name="void rflbm::(anonymous namespace)::advance_step(unsigned int*)", Calls=60,
                  AverageNs=2.0, MinNs=2, MaxNs=2)]
    write_csv(str(out / "prof_batch_f32" / "trace_kernel_stats.csv"), ["Name", "Calls", "AverageNs", "MinNs", "MaxNs"], stats)
    path = bench.summarize_batch_trace(str(out), "f32", nodes=1000)
    text = open(path).read()
    assert even in text and odd in text and "advance_step" not in text
    assert f"mean batch step kernel: 850 ns -> {1000 / 850e-9 / 1e6:.0f} MLUPS" in text
