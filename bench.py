"""Benchmark of the EIS-inversion grid search on one MI355X.

Workload (one step): the 1080p plain search -- 30 residual frames of 1080 x 1920
(fp32, resident in HBM), each searched over the full 41 x 21 (scale, rotation) grid
with shift radius 64 against one device-resident fingerprint, followed by the
per-frame argmax and the video decision.  25,830 candidate evaluations per step
(inverse warp + FFT correlation + PCE each).

Prints one JSON line with candidates/s, the roofline of the dominant kernel
(algorithmic bytes / HIP-event duration of its launches over the timed region; the
measured HBM traffic and the VALU-issue fraction from the committed rocprofv3 counter
summaries while they match the kernel source) and the FP64 CPU oracle timed on a
bounded sample of the same workload.

    python bench.py [--steps K] [--warmup W] [--no-cpu]

Other workloads (not the headline line):

    python bench.py --workload batched     # 8 warm-started sequences of mixed sizes: serving
                                           # engine vs one synchronous search per video and vs
                                           # the plain per-frame full-grid form
    python bench.py --workload precision   # 4K frames stored in bf16: per-frame PCE error
                                           # against the FP64 oracle on the fp32 frames
    python bench.py --workload refine      # the paper's coarse-to-fine schedule on the 1080p
                                           # frames against the fixed 41 x 21 grid
    python bench.py --workload transforms  # general 8-parameter transforms vs the similarity grid
    python bench.py --workload fingerprint # Eq. (2) estimate from 64 1080p images vs the HBM peak
    python bench.py --workload cropped     # 720p frames in a 1080p fingerprint vs equal sizes
    python bench.py --workload residuals   # noise residuals (wavelet denoiser) of 64 1080p images
    python bench.py --workload serving [--rate 4] [--videos 240] [--sweep] [--small-budget-gib 4]
                                           # Poisson stream of videos: videos/s, p50/p99 latency;
                                           # saturated engine vs the synchronous forms
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "warp+xcorr+PCE candidates/sec @1080p; p50/p99 latency per video"
HBM_PEAK_GBS = 8000.0
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "traffic_hd.txt")
# the sources the search kernels are compiled from (kernels, FFT plans and passes)
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2207_14507_amd", "csrc", f) for f in
                  ("kernels.hip", "kernels.hpp", "fft_device.hpp", "fft_plans.hpp", "fft_exec.hpp")]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_digest() -> str:
    h = hashlib.sha256()
    for path in KERNEL_SOURCES:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, cands_per_launch: float):
    """HBM bytes per launch of ``kernel`` (at cands_per_launch candidates per launch) from
    the committed rocprofv3 counter summary, or None when there is none or the kernel
    source changed since it was taken."""
    if not os.path.exists(PROFILE_TRAFFIC):
        return None
    kv = {}
    for line in open(PROFILE_TRAFFIC):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_sources_sha256_16") != kernel_source_digest():
        return None
    v = kv.get(f"{kernel}_bytes_per_candidate")
    return round(float(v) * cands_per_launch, 1) if v else None


PROFILE_VALU = os.path.join(ROOT, "profiles", "valu_hd.txt")
# VALU issue slots of the chip per second: 256 CUs x 4 SIMDs, one issue quad-cycle (4
# clocks) per SIMD at a time, 2.4 GHz.  A quad-cycle issues one 64-lane VALU instruction,
# or two when both are of the dual-issue kinds (two-source fp32 and int32 forms such as
# v_add_f32, v_mul_f32 and v_add_u32; FMAs and other three-source forms issue alone).
VALU_ISSUE_PEAK = 1024 * 2.4e9 / 4


def measured_valu(kernel: str, cands_per_launch: float):
    """VALU work per launch of ``kernel`` from the committed SQ counter summary: wave
    instructions and issue quad-cycles (instructions less the quad-cycles that issued
    two), each per wave x waves per candidate x candidates; None when there is no summary
    or the kernel source changed since it was taken."""
    if not os.path.exists(PROFILE_VALU):
        return None
    digest, cols, per = None, None, {}
    want = ("VALU instructions per wave", "waves per candidate", "VALU issue quad-cycles per wave")
    for line in open(PROFILE_VALU):
        if line.startswith("# kernel |"):
            cols = [x.strip() for x in line[1:].split("|")]
        elif line.startswith("#"):
            continue
        elif line.startswith("kernel_sources_sha256_16:"):
            digest = line.split(":", 1)[1].strip()
        elif "|" in line and cols and all(w in cols for w in want):
            f = [x.strip() for x in line.split("|")]
            per[f[0]] = tuple(float(f[cols.index(w)].split()[0]) for w in want)
    if digest != kernel_source_digest() or kernel not in per:
        return None
    ipw, wpc, qpw = per[kernel]
    return {"wave_instr": round(ipw * wpc * cands_per_launch, 1),
            "issue_quad_cycles": round(qpw * wpc * cands_per_launch, 1)}


# rocprofv3 kernel names of the search kernels at 1080p -> (short name, blocks per candidate)
# (row pairs 1080/2, column strips (1920/2)/8, band row pairs (2*64 + 11 + 1)/2, one PCE
# workgroup)
KERNELS_HD = {"k_warp_rowfft<1920,": ("warp_rowfft", 540), "k_col<1080, 512, true>": ("col_product", 120),
              "k_band_rowifft<1920,": ("band_rowifft", 70), "k_pce<256>": ("pce", 1)}


# counter passes of the unit summaries (within one run's limits: SQ <= 8, TA, TD <= 2,
# GRBM <= 2 counters)
PMC_SQ = "SQ_WAVES SQ_INSTS_VALU SQ_ACTIVE_INST_VALU2 SQ_INSTS_VMEM_RD SQ_INSTS_LDS SQ_WAVE_CYCLES GRBM_GUI_ACTIVE"
PMC_TA = "SQ_WAVES SQ_LDS_BANK_CONFLICT TA_TA_BUSY TD_TD_BUSY GRBM_GUI_ACTIVE"

# the same at 4K (row pairs 2160/2, two workgroups per column strip (3840/2)/8, band row
# pairs, one PCE workgroup); the row kernel's third template argument is the frame dtype
KERNELS_UHD = {"k_warp_rowfft<3840, 256, 1,": ("warp_rowfft bf16", 1080),
               "k_warp_rowfft<3840, 256, 0,": ("warp_rowfft fp32", 1080),
               "k_col<2160, 512, true>": ("col_product", 480), "k_band_rowifft<3840,": ("band_rowifft", 70),
               "k_pce<256>": ("pce", 1)}


def _short(name: str, table=None):
    for key, v in (table or KERNELS_HD).items():
        if key.replace(" ", "") in name.replace(" ", ""):
            return v
    return None


def _csv_rows(d: str, sub: str, suffix: str):
    import csv
    path = os.path.join(d, sub, f"{sub}_{suffix}.csv")
    return list(csv.DictReader(open(path))) if os.path.exists(path) else None


def _grid_blocks(r) -> int:
    g = int(r.get("Grid_Size") or r.get("Grid_Size_X") or 0)
    w = int(r.get("Workgroup_Size") or r.get("Workgroup_Size_X") or 1)
    return g // max(1, w)


def _counters_per_kernel(d: str, sub: str, table):
    """One counter pass: each counter summed per kernel over its dispatches, and the
    candidates those dispatches covered."""
    rows = _csv_rows(d, sub, "counter_collection")
    if rows is None:
        return None
    agg, seen = {}, set()
    for r in rows:
        sh = _short(r["Kernel_Name"], table)
        if not sh:
            continue
        a = agg.setdefault(sh[0], {"_cands": 0.0})
        a[r["Counter_Name"]] = a.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
        if r["Dispatch_Id"] not in seen:
            seen.add(r["Dispatch_Id"])
            a["_cands"] += _grid_blocks(r) / sh[1]
    return agg


def unit_summary(d: str, table, head, subs, cmd_sq: str, cmd_ta: str, path: str) -> None:
    """Per-kernel VALU instructions per wave, waves per candidate and the busy fractions of
    the VALU, the vector-memory address (TA) and data (TD) units, and the LDS bank-conflict
    cycles, from two counter passes (subs = their folders under d, one rocprofv3 run each)."""
    sq = _counters_per_kernel(d, subs[0], table)
    ta = _counters_per_kernel(d, subs[1], table) or {}
    if not sq:
        return
    lines = head + [f"# command (sq): {cmd_sq}", f"# command (ta): {cmd_ta}",
                    "# GRBM_GUI_ACTIVE is summed over the 8 XCDs, so a kernel's cycles per CU are",
                    "# GRBM_GUI_ACTIVE / 8.  A SIMD issues VALU work in quad-cycles (4 clocks): one",
                    "# 64-lane instruction, or two of the dual-issue kinds (two-source fp32 and int32",
                    "# forms); SQ_ACTIVE_INST_VALU2 counts the quad-cycles that issued two.  VALU issue",
                    "# quad-cycles = SQ_INSTS_VALU - SQ_ACTIVE_INST_VALU2; VALU busy = those x 4 / (1024",
                    "# SIMDs x GRBM_GUI_ACTIVE / 8); dual share = SQ_ACTIVE_INST_VALU2 x 2 / SQ_INSTS_VALU",
                    "# (instructions issued in pairs); TA and TD busy = TA_TA_BUSY, TD_TD_BUSY / (256 CUs x",
                    "# GRBM_GUI_ACTIVE / 8), each with its own pass's GRBM_GUI_ACTIVE (ratios of counters",
                    "# taken per dispatch: a saturated unit can read slightly above 100%).",
                    "# LDS bank-conflict cycles are SQ quad-cycles (4 clocks) per wave.",
                    "# VALU-issue bound = issue quad-cycles x waves x 4 cycles / (1024 SIMDs x 2.4 GHz).",
                    f"kernel_sources_sha256_16: {kernel_source_digest()}",
                    "# kernel | VALU instructions per wave | waves per candidate | VALU issue quad-cycles per"
                    " wave | VALU busy | dual share | TA busy | TD busy | LDS bank-conflict cycles per wave"
                    " | VALU-issue bound us per candidate"]
    pct = lambda x: "-" if x is None else f"{x:.1%}"
    for k, a in sq.items():
        w, c = a.get("SQ_WAVES", 0.0), a["_cands"]
        if not w or not c:
            continue
        ipw, wpc = a.get("SQ_INSTS_VALU", 0.0) / w, w / c
        dual = a.get("SQ_ACTIVE_INST_VALU2")  # absent: no pair assumed (an upper bound)
        qpw = ipw - (dual or 0.0) / w
        g = a.get("GRBM_GUI_ACTIVE", 0.0) / 8.0
        valu = qpw * w * 4.0 / (1024 * g) if g else None
        share = "-" if dual is None or not a.get("SQ_INSTS_VALU") else f"{2.0 * dual / a['SQ_INSTS_VALU']:.1%}"
        t = ta.get(k, {})
        gt = t.get("GRBM_GUI_ACTIVE", 0.0) / 8.0
        tab = t["TA_TA_BUSY"] / (256 * gt) if gt and "TA_TA_BUSY" in t else None
        tdb = t["TD_TD_BUSY"] / (256 * gt) if gt and "TD_TD_BUSY" in t else None
        conf = f"{t['SQ_LDS_BANK_CONFLICT'] / t['SQ_WAVES']:.1f}" if t.get("SQ_WAVES") and \
            "SQ_LDS_BANK_CONFLICT" in t else "-"
        bound = qpw * w * 4.0 / (1024 * 2.4e9) / c * 1e6
        lines.append(f"{k} | {ipw:.1f} | {wpc:.0f} | {qpw:.1f} | {pct(valu)} | {share} | {pct(tab)} | {pct(tdb)}"
                     f" | {conf} | {bound:.3f}")
    open(path, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def uhd_kernel_summary(d: str, cmd: str, path: str) -> None:
    """Average launch time and time per candidate of the 4K search kernels, from the
    kernel trace of the 4K workload (bf16 frames, then the same frames in fp32)."""
    rows = _csv_rows(d, "uhdkt", "kernel_trace")
    if rows is None:
        return
    per = {}
    for r in rows:
        sh = _short(r["Kernel_Name"], KERNELS_UHD)
        if not sh:
            continue
        a = per.setdefault(sh[0], {})
        nb = _grid_blocks(r)
        cands = nb / sh[1]
        dur = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        b = a.setdefault(round(cands), [0, 0.0])
        b[0] += 1
        b[1] += dur
    lines = ["# Kernel trace of the 4K search: 16 frames of 2160 x 3840 residuals stored in bf16,",
             "# then the same frames in fp32, full 41 x 21 grid, shift radius 64; launches grouped",
             "# by candidates per launch (the tuner's trials and the tuned batch).",
             f"# command: {cmd}", f"kernel_sources_sha256_16: {kernel_source_digest()}",
             "# kernel | candidates per launch | launches | average us per launch | us per candidate"]
    for k, a in per.items():
        for c, (n, t) in sorted(a.items(), key=lambda kv: -kv[1][0] * kv[0])[:1]:
            lines.append(f"{k} | {c} | {n} | {t / n:.1f} | {t / n / max(c, 1):.2f}")
    open(path, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def profile_summary(d: str, cmd_kt: str, cmd_fetch: str, cmd_write: str, cmd_copy: str) -> None:
    """Writes profiles/kernels_hd.txt (kernel-trace statistics) and profiles/traffic_hd.txt
    (FETCH_SIZE / WRITE_SIZE per candidate, scaled by the copy calibration) from the
    rocprofv3 output under d (kt/, fetch/, write/, copyf/, copyw/)."""
    import csv

    def rows(sub, suffix):
        path = os.path.join(d, sub, f"{sub}_{suffix}.csv")
        return list(csv.DictReader(open(path)))

    lines = ["# Kernel-trace statistics of the search kernels, 1080p workload (30 frames x 861",
             "# candidates per step, tuned launch schedule read from the cache the first command writes)",
             f"# command: {cmd_kt}", "# name | calls | average us | total ms | share %"]
    for r in rows("kt", "kernel_stats"):
        sh = _short(r["Name"])
        tag = sh[0] if sh else r["Name"][:60]
        lines.append(f"{tag} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                     f"{float(r['TotalDurationNs']) / 1e6:.2f} | {float(r['Percentage']):.2f}")
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    open(os.path.join(ROOT, "profiles", "kernels_hd.txt"), "w").write("\n".join(lines) + "\n")

    def copy_factor(sub, counter, nbytes):
        vals = [float(r["Counter_Value"]) for r in rows(sub, "counter_collection")
                if r["Counter_Name"] == counter and "copyBuffer" in r["Kernel_Name"]]
        kib = sum(vals) / max(1, len(vals))
        return nbytes / (kib * 1024.0), kib

    fetch_f, fkib = copy_factor("copyf", "FETCH_SIZE", 256 << 20)
    write_f, wkib = copy_factor("copyw", "WRITE_SIZE", 256 << 20)
    per = {}
    for sub, counter, fac in (("fetch", "FETCH_SIZE", fetch_f), ("write", "WRITE_SIZE", write_f)):
        for r in rows(sub, "counter_collection"):
            sh = _short(r["Kernel_Name"])
            if not sh or r["Counter_Name"] != counter:
                continue
            blocks = int(r["Grid_Size"]) // max(1, int(r["Workgroup_Size"]))
            cands = blocks / sh[1]
            acc = per.setdefault(sh[0], {"FETCH_SIZE": [0.0, 0.0], "WRITE_SIZE": [0.0, 0.0]})[counter]
            acc[0] += float(r["Counter_Value"]) * 1024.0 * fac
            acc[1] += cands
    out = ["# HBM traffic of the search kernels at 1080p from rocprofv3 counters, per candidate.",
           f"# FETCH_SIZE command: {cmd_fetch}", f"# WRITE_SIZE command: {cmd_write}",
           f"# copy calibration command (one pass per counter): {cmd_copy}",
           f"# a 256 MiB device copy reads {fkib:.0f} KiB of FETCH_SIZE and {wkib:.0f} KiB of WRITE_SIZE",
           f"fetch_factor: {fetch_f:.4f}", f"write_factor: {write_f:.4f}",
           f"kernel_sources_sha256_16: {kernel_source_digest()}"]
    for k, v in per.items():
        fb = v["FETCH_SIZE"][0] / max(v["FETCH_SIZE"][1], 1e-9)
        wb = v["WRITE_SIZE"][0] / max(v["WRITE_SIZE"][1], 1e-9)
        out += [f"{k}_fetch_bytes_per_candidate: {fb:.0f}", f"{k}_write_bytes_per_candidate: {wb:.0f}",
                f"{k}_bytes_per_candidate: {fb + wb:.0f}"]
    open(PROFILE_TRAFFIC, "w").write("\n".join(out) + "\n")
    print("\n".join(lines + out))


def _cpu_worker(args):
    K, W, cands, radius = args
    from oracle import prnu_oracle as O
    kn = O.mean_free(K)
    return [O.evaluate_candidate(K, W, s, t, radius, kn).pce for s, t in cands]


def _cpu_warm(_):
    from oracle import prnu_oracle  # noqa: F401  (import cost outside the timed region)
    return 0


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(seq, cores: int, per_core: int = 24, single: int = 12):
    """The FP64 oracle (unchanged) on a bounded sample: cores*per_core candidates spread
    over the full grid, on frame 0, one process per core (about 10 s of wall time); and
    `single` of them in one process (one FFT thread)."""
    from concurrent.futures import ProcessPoolExecutor
    from oracle import prnu_oracle as O
    grid = O.full_grid(O.WarmOptions())
    n = min(len(grid), cores * per_core)
    cands = [grid[(i * 7) % len(grid)] for i in range(n)]
    chunks = [cands[i::cores] for i in range(cores)]
    with ProcessPoolExecutor(cores) as ex:
        list(ex.map(_cpu_warm, range(cores)))
        t0 = time.perf_counter()
        list(ex.map(_cpu_worker, [(seq.K, seq.frames[0], c, 64) for c in chunks]))
        dt = time.perf_counter() - t0
    with ProcessPoolExecutor(1) as ex:
        list(ex.map(_cpu_warm, range(1)))
        t0 = time.perf_counter()
        list(ex.map(_cpu_worker, [(seq.K, seq.frames[0], cands[:single], 64)]))
        dt1 = time.perf_counter() - t0
    return {"value": len(cands) / dt, "unit": "candidates/s", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model(), "os_cpu_count": os.cpu_count(),
            "sample": f"{len(cands)} candidates spread over the 1080p full grid (frame 0), {cores} processes "
                      f"(one FFT thread each), {dt:.1f} s wall",
            "single_process": {"value": single / dt1, "unit": "candidates/s", "cores": 1,
                               "sample": f"the first {single} of those candidates in one process, {dt1:.1f} s"}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--frames", type=int, default=30)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--host-input", action="store_true",
                    help="pass the frames as host arrays (uploaded by every call) instead of device tensors")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device copy (counter calibration for HBM traffic)")
    ap.add_argument("--workload", choices=["hd", "batched", "precision", "serving", "refine", "transforms", "fingerprint", "cropped", "residuals"], default="hd")
    ap.add_argument("--tune-cache", default=None,
                    help="launch-schedule cache file (read if present, written after tuning)")
    ap.add_argument("--profile-summary", default=None, metavar="DIR",
                    help="write profiles/kernels_hd.txt and profiles/traffic_hd.txt from rocprofv3 output in DIR")
    ap.add_argument("--rate", type=float, default=4.0, help="serving: mean arrivals per second")
    ap.add_argument("--videos", type=int, default=240, help="serving: measured videos")
    ap.add_argument("--warm-videos", type=int, default=20, help="serving: unmeasured videos first")
    ap.add_argument("--pool", type=int, default=128, help="serving: generated walk frames per fingerprint")
    ap.add_argument("--budget-gib", type=float, default=64.0, help="serving: HBM budget of the engine")
    ap.add_argument("--sweep", action="store_true", help="serving: also run arrival rates 1, 2, 3, 4 per second")
    ap.add_argument("--sweep-videos", type=int, default=40, help="serving: measured videos per sweep point")
    ap.add_argument("--small-budget-gib", type=float, default=0.0,
                    help="serving: also run the offered rate with this small HBM budget")
    ap.add_argument("--sat-videos", type=int, default=12, help="serving: videos of the saturated comparison")
    a = ap.parse_args()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(f"bench.py runs on one GPU only (asked for {a.gpus}); the search shards by video and "
              f"needs no collective, so multi-GPU figures are not produced.", file=sys.stderr)
        sys.exit(2)

    if a.profile_summary:
        d = a.profile_summary
        pre = "cd /tmp && TMPDIR=/tmp rocprofv3"
        bench = f"-- python3 /root/repo/bench.py --no-cpu --tune-cache {d}/tune.txt"
        short = f"{bench} --steps 1 --warmup 0 --frames 2"
        profile_summary(d,
                        f"{pre} --kernel-trace --stats -f csv -d {d}/kt -o kt {bench} --steps 2 --warmup 1"
                        f" (after: python3 /root/repo/bench.py --steps 1 --warmup 0 --no-cpu --tune-cache {d}/tune.txt)",
                        f"{pre} --pmc FETCH_SIZE -f csv -d {d}/fetch -o fetch {short}",
                        f"{pre} --pmc WRITE_SIZE -f csv -d {d}/write -o write {short}",
                        f"{pre} --pmc FETCH_SIZE|WRITE_SIZE -f csv -d {d}/copyf|copyw -- python3 /root/repo/bench.py --copy-calibration")
        unit_summary(d, KERNELS_HD,
                     ["# Instruction counts and unit busy fractions of the search kernels, 1080p workload",
                      "# (2 frames x 861 candidates, tuned schedule read from the cache), rocprofv3 counters",
                      "# summed over each kernel's launches."], ("sq", "ta"),
                     f"{pre} --pmc {PMC_SQ} -f csv -d {d}/sq -o sq {short}",
                     f"{pre} --pmc {PMC_TA} -f csv -d {d}/ta -o ta {short}",
                     os.path.join(ROOT, "profiles", "valu_hd.txt"))
        uhd = "-- python3 /root/repo/bench.py --workload precision --no-cpu"
        uhd_kernel_summary(d, f"{pre} --kernel-trace --stats -f csv -d {d}/uhdkt -o uhdkt {uhd}",
                           os.path.join(ROOT, "profiles", "kernels_4k_bf16.txt"))
        unit_summary(d, KERNELS_UHD,
                     ["# Instruction counts and unit busy fractions of the 4K search kernels (16 frames of",
                      "# 2160 x 3840 residuals stored in bf16, then the same frames in fp32; the tuner's",
                      "# trial launches included), rocprofv3 counters summed over each kernel's launches."],
                     ("uhdsq", "uhdta"), f"{pre} --pmc {PMC_SQ} -f csv -d {d}/uhdsq -o uhdsq {uhd}",
                     f"{pre} --pmc {PMC_TA} -f csv -d {d}/uhdta -o uhdta {uhd}",
                     os.path.join(ROOT, "profiles", "valu_4k_bf16.txt"))
        return
    import torch
    if a.copy_calibration:
        x = torch.ones(64 << 20, dtype=torch.float32, device="cuda")  # 256 MiB
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": x.numel() * 4, "copy_bytes_written": y.numel() * 4, "copies": 3}))
        return
    from paper_2207_14507_amd import prnu as P
    from paper_2207_14507_amd import synth

    if a.workload != "hd":
        import bench_workloads
        print(json.dumps(bench_workloads.run(a.workload, a, P, synth, torch, log)), flush=True)
        return

    log("generating the 1080p workload ...")
    seq = synth.hd_sequence(n_frames=a.frames)
    # device-resident frames (the measured configuration), or host arrays uploaded by
    # every call (--host-input: the transfer-inclusive rate, never the headline value)
    frames = seq.frames if a.host_input else torch.from_numpy(seq.frames).cuda()
    opts = P.make_opts(grid=(41, 0.85, 1.15, 21, -2.0, 2.0), radius=64)
    n_cand = a.frames * 41 * 21
    ctx = P.prnu_create(0, flags=int(os.environ.get("PRNU_BENCH_FLAGS", "0")), tune_cache_path=a.tune_cache)
    fp = P.prnu_open_fingerprint(ctx, torch.from_numpy(seq.K).cuda())
    torch.cuda.synchronize()
    for i in range(a.warmup):
        P.prnu_search_frames(ctx, fp, frames, opts)
        log(f"warmup step {i + 1}/{a.warmup} done")
    torch.cuda.synchronize()
    P.prnu_profile_enable(ctx, True)
    lat = []
    t0 = time.perf_counter()
    for i in range(a.steps):
        s0 = time.perf_counter()
        res, summ = P.prnu_search_frames(ctx, fp, frames, opts)
        lat.append(time.perf_counter() - s0)
        log(f"step {i + 1}/{a.steps}: {lat[-1] * 1e3:.1f} ms, mean gamma {summ.mean_pce:.1f}")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    stats = P.prnu_profile_read(ctx)
    P.prnu_profile_enable(ctx, False)
    P.prnu_close_fingerprint(ctx, fp)
    P.prnu_destroy(ctx)

    dom = max(stats, key=lambda s: s["total_ms"])
    launch_ms = dom["total_ms"] / max(1, dom["launches"])
    bytes_per_launch = dom["algo_bytes"] / max(1, dom["launches"])
    achieved = bytes_per_launch / (launch_ms * 1e-3) / 1e9
    traffic = measured_traffic(dom["name"], dom["candidates"] / max(1, dom["launches"]))
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": dom["name"],
                "launch_ms": round(launch_ms, 4), "algo_bytes_per_launch": bytes_per_launch}
    # The HBM bytes the counters saw for the same launch (FETCH_SIZE + WRITE_SIZE, copy
    # calibrated), over the same measured time: below the algorithmic figure because the
    # fingerprint strips shared by the candidates of a launch are read from cache.
    roofline["measured_frac"] = None if traffic is None else round(traffic / (launch_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
    # The same launch against the SIMDs' VALU issue slots: quad-cycles that issued VALU
    # work (from the committed SQ counters) over those the launch's measured time offers.
    valu = measured_valu(dom["name"], dom["candidates"] / max(1, dom["launches"]))
    roofline["valu_issue"] = None if valu is None else {
        "wave_instr_per_launch": valu["wave_instr"], "issue_quad_cycles_per_launch": valu["issue_quad_cycles"],
        "peak_issue_quad_cycles_per_s": VALU_ISSUE_PEAK,
        "frac": round(valu["issue_quad_cycles"] / (launch_ms * 1e-3) / VALU_ISSUE_PEAK, 4)}
    kernels = {s["name"]: {"ms_total": round(s["total_ms"], 3), "launches": s["launches"],
                           "GB/s": round(s["algo_bytes"] / max(s["total_ms"], 1e-9) / 1e6, 1)} for s in stats}
    lat_sorted = np.sort(np.array(lat))
    out = {
        "metric": METRIC,
        "value": round(n_cand * a.steps / dt, 1),
        "unit": "candidates/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(dt / a.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"1080x1920 fp32 residual frames x{a.frames} vs one fingerprint, full 41x21 "
                               f"(scale,rotation) grid, shift radius 64, 11x11 exclusion",
                   "candidates_per_step": n_cand, "frames": a.frames, "grid": [41, 21], "shift_radius": 64,
                   "frames_in": "host memory, uploaded by every call" if a.host_input else "device memory (HBM)"},
        # one step is one 30-frame video searched by a synchronous plain call; the serving
        # loop's per-video latency under Poisson arrivals is the serving workload's figure
        "step_latency_p50_s": round(float(np.percentile(lat_sorted, 50)), 4),
        "step_latency_p99_s": round(float(np.percentile(lat_sorted, 99)), 4),
        "kernels": kernels,
        "roofline": roofline,
    }
    if not a.no_cpu:
        cores = min(os.cpu_count() or 1, 16)
        log(f"timing the CPU oracle on {cores} processes ...")
        out["cpu_baseline"] = cpu_baseline(seq, cores)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
