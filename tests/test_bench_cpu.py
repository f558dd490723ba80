"""Host logic of the benchmark's roofline report (no GPU): the counter summary written
from rocprofv3 CSV output, its per-candidate scaling, the VALU-issue figure read from the
SQ counter summary, the unit-busy and 4K kernel-trace summaries, and the rule that counter
figures are dropped once the kernel sources differ from the ones they were taken on."""
import csv
import os

import pytest

import bench


def write_csv(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        w.writerows(rows)


def fake_rocprof(d):
    """Kernel statistics plus FETCH_SIZE / WRITE_SIZE dispatches: a column-kernel launch of
    10 candidates (10 x 120 workgroups of 512), a row-kernel launch of 10 candidates
    (10 x 540 workgroups of 128), and the 256 MiB copy calibration."""
    write_csv(os.path.join(d, "kt", "kt_kernel_stats.csv"),
              ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs", "StdDev"],
              [["void prnu::(anonymous namespace)::k_col<1080, 512, true>(prnu::Batch, prnu::c32*)", 4,
                4000000, 1000000, 60.0, 1, 1, 0],
               ["void prnu::(anonymous namespace)::k_warp_rowfft<1920, 128, 0, false, false>(prnu::Batch)", 4,
                2000000, 500000, 40.0, 1, 1, 0]])
    head = ["Kernel_Name", "Grid_Size", "Workgroup_Size", "Counter_Name", "Counter_Value"]
    col = "void prnu::(anonymous namespace)::k_col<1080, 512, true>(prnu::Batch, prnu::c32*)"
    row = "void prnu::(anonymous namespace)::k_warp_rowfft<1920, 128, 0, false, false>(prnu::Batch)"
    write_csv(os.path.join(d, "fetch", "fetch_counter_collection.csv"), head,
              [[col, 10 * 120 * 512, 512, "FETCH_SIZE", 40000.0], [row, 10 * 540 * 128, 128, "FETCH_SIZE", 1000.0]])
    write_csv(os.path.join(d, "write", "write_counter_collection.csv"), head,
              [[col, 10 * 120 * 512, 512, "WRITE_SIZE", 10000.0], [row, 10 * 540 * 128, 128, "WRITE_SIZE", 80000.0]])
    write_csv(os.path.join(d, "copyf", "copyf_counter_collection.csv"), head,
              [["__amd_rocclr_copyBuffer", 1, 1, "FETCH_SIZE", 131072.0]])
    write_csv(os.path.join(d, "copyw", "copyw_counter_collection.csv"), head,
              [["__amd_rocclr_copyBuffer", 1, 1, "WRITE_SIZE", 262144.0]])


@pytest.fixture
def sandbox(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "PROFILE_TRAFFIC", str(tmp_path / "profiles" / "traffic_hd.txt"))
    return tmp_path


def test_profile_summary_scales_counters_per_candidate(sandbox):
    d = sandbox / "raw"
    fake_rocprof(str(d))
    bench.profile_summary(str(d), "kt-cmd", "fetch-cmd", "write-cmd", "copy-cmd")
    kv = {}
    for line in open(sandbox / "profiles" / "traffic_hd.txt"):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    # the copy of 256 MiB read as 128 MiB of FETCH_SIZE: reads scale by 2, writes by 1
    assert float(kv["fetch_factor"]) == pytest.approx(2.0)
    assert float(kv["write_factor"]) == pytest.approx(1.0)
    assert float(kv["col_product_fetch_bytes_per_candidate"]) == pytest.approx(40000 * 1024 * 2 / 10, rel=1e-6)
    assert float(kv["col_product_write_bytes_per_candidate"]) == pytest.approx(10000 * 1024 / 10, rel=1e-6)
    assert float(kv["warp_rowfft_bytes_per_candidate"]) == pytest.approx((1000 * 2 + 80000) * 1024 / 10, rel=1e-6)
    assert kv["kernel_sources_sha256_16"] == bench.kernel_source_digest()
    stats = open(sandbox / "profiles" / "kernels_hd.txt").read()
    assert "col_product | 4 | 1000.00" in stats and "warp_rowfft | 4 | 500.00" in stats
    # read back by the bench and scaled to its launch size
    per = float(kv["col_product_bytes_per_candidate"])
    assert bench.measured_traffic("col_product", 768) == round(per * 768, 1)


def test_traffic_dropped_when_the_kernels_changed(sandbox):
    os.makedirs(sandbox / "profiles")
    path = sandbox / "profiles" / "traffic_hd.txt"
    path.write_text("kernel_sources_sha256_16: 0000000000000000\ncol_product_bytes_per_candidate: 100\n")
    assert bench.measured_traffic("col_product", 10) is None
    path.write_text(f"kernel_sources_sha256_16: {bench.kernel_source_digest()}\ncol_product_bytes_per_candidate: 100\n")
    assert bench.measured_traffic("col_product", 10) == 1000.0
    assert bench.measured_traffic("band_rowifft", 10) is None
    path.unlink()
    assert bench.measured_traffic("col_product", 10) is None


def test_valu_issue_from_counter_summary(tmp_path, monkeypatch):
    path = tmp_path / "valu_hd.txt"
    monkeypatch.setattr(bench, "PROFILE_VALU", str(path))
    body = "# header\n{}\n# kernel | VALU instructions per wave | waves per candidate | VALU issue " \
           "quad-cycles per wave\ncol_product | 1000.0 | 960 | 700.0\npce | 2000.0 | 4 | 2000.0\n"
    path.write_text(body.format("kernel_sources_sha256_16: 0000000000000000"))
    assert bench.measured_valu("col_product", 10) is None  # taken on other kernels
    path.write_text(body.format(f"kernel_sources_sha256_16: {bench.kernel_source_digest()}"))
    assert bench.measured_valu("col_product", 10) == {"wave_instr": 1000.0 * 960 * 10,
                                                       "issue_quad_cycles": 700.0 * 960 * 10}
    assert bench.measured_valu("pce", 3) == {"wave_instr": 2000.0 * 4 * 3, "issue_quad_cycles": 2000.0 * 4 * 3}
    assert bench.measured_valu("band_rowifft", 10) is None
    # 1024 SIMDs, one issue quad-cycle each per 4 clocks at 2.4 GHz
    assert bench.VALU_ISSUE_PEAK == pytest.approx(614.4e9)


def test_more_than_one_gpu_is_refused_before_any_device_work():
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    p = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode != 0 and "one GPU only" in p.stdout + p.stderr
    assert p.stdout.count("{") == 0  # no JSON result line


def test_unit_summary_busy_fractions_and_readback(sandbox, monkeypatch):
    """Two counter passes of one column-kernel launch of 10 candidates: the summary's
    per-wave and per-candidate figures and busy fractions follow from the counter values,
    and the bench reads the VALU instructions back."""
    monkeypatch.setattr(bench, "PROFILE_VALU", str(sandbox / "profiles" / "valu_hd.txt"))
    d = str(sandbox / "raw")
    col = "void prnu::(anonymous namespace)::k_col<1080, 512, true>(prnu::Batch, prnu::c32*)"
    head = ["Dispatch_Id", "Kernel_Name", "Grid_Size", "Workgroup_Size", "Counter_Name", "Counter_Value"]
    g = 10 * 120 * 512
    waves = 10 * 120 * 8
    # 8 XCDs x 100,000 cycles; VALU: 1500 instructions per wave, 300 quad-cycles of them
    # issued two at a time
    write_csv(os.path.join(d, "sq", "sq_counter_collection.csv"), head,
              [[7, col, g, 512, "SQ_WAVES", waves], [7, col, g, 512, "SQ_INSTS_VALU", 1500.0 * waves],
               [7, col, g, 512, "SQ_ACTIVE_INST_VALU2", 300.0 * waves],
               [7, col, g, 512, "GRBM_GUI_ACTIVE", 800000.0]])
    write_csv(os.path.join(d, "ta", "ta_counter_collection.csv"), head,
              [[9, col, g, 512, "SQ_WAVES", waves], [9, col, g, 512, "TA_TA_BUSY", 256 * 50000.0],
               [9, col, g, 512, "TD_TD_BUSY", 256 * 75000.0], [9, col, g, 512, "SQ_LDS_BANK_CONFLICT", 12.5 * waves],
               [9, col, g, 512, "GRBM_GUI_ACTIVE", 800000.0]])
    os.makedirs(sandbox / "profiles")
    bench.unit_summary(d, bench.KERNELS_HD, ["# test"], ("sq", "ta"), "sq-cmd", "ta-cmd",
                       str(sandbox / "profiles" / "valu_hd.txt"))
    text = open(sandbox / "profiles" / "valu_hd.txt").read()
    line = [x for x in text.splitlines() if x.startswith("col_product |")][0]
    f = [x.strip() for x in line.split("|")]
    assert float(f[1]) == 1500.0 and int(f[2]) == 960
    # issue quad-cycles: 1500 - 300 per wave; busy: 1200 x 9600 waves x 4 cycles / (1024
    # SIMDs x 100,000 cycles) = 45%; 600 of the 1500 instructions went in pairs
    assert float(f[3]) == 1200.0
    assert f[4] == "45.0%" and f[5] == "40.0%"
    assert f[6] == "50.0%" and f[7] == "75.0%" and f[8] == "12.5"
    # 1200 x 960 x 4 / (1024 x 2.4 GHz) per candidate
    assert float(f[9]) == pytest.approx(1200 * 960 * 4 / (1024 * 2.4e9) * 1e6, abs=1e-3)
    assert bench.measured_valu("col_product", 768) == {"wave_instr": round(1500.0 * 960 * 768, 1),
                                                        "issue_quad_cycles": round(1200.0 * 960 * 768, 1)}


def test_uhd_kernel_summary_groups_launches_by_batch(sandbox):
    """4K kernel trace: the tuned batch's launches are summarised, the tuner's trial
    launches (another candidate count) are not mixed in."""
    d = str(sandbox / "raw")
    row = "void prnu::(anonymous namespace)::k_warp_rowfft<3840, 256, 1, false, false>(prnu::Batch)"
    col = "void prnu::(anonymous namespace)::k_col<2160, 512, true>(prnu::Batch, prnu::c32*)"
    head = ["Kernel_Name", "Grid_Size_X", "Workgroup_Size_X", "Start_Timestamp", "End_Timestamp"]
    rows = [[row, 192 * 1080 * 256, 256, 0, 2_400_000]] * 5 + [[row, 8 * 1080 * 256, 256, 0, 100_000]] * 2 + \
           [[col, 192 * 480 * 512, 512, 0, 2_880_000]] * 5
    write_csv(os.path.join(d, "uhdkt", "uhdkt_kernel_trace.csv"), head, rows)
    os.makedirs(sandbox / "profiles")
    out = str(sandbox / "profiles" / "kernels_4k_bf16.txt")
    bench.uhd_kernel_summary(d, "uhd-cmd", out)
    text = open(out).read()
    assert "warp_rowfft bf16 | 192 | 5 | 2400.0 | 12.50" in text
    assert "col_product | 192 | 5 | 2880.0 | 15.00" in text
