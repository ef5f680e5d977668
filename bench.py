"""Benchmark: the convolution sweep on one MI355X, autotuned vs plain kernels.

Workload (one "step"): a 4096 x 4096 float32 image (U[0,1)) through the
separable filter and the full 2-D filter of every radius 1, 2, 3, 5, 7
(N(0,1) taps normalised to sum 1, clamp-to-edge): ten library calls, each
reading a 64 MiB image and writing a 64 MiB result.  Inputs rotate over eight
image/output pairs (1 GiB), so the 256 MB Infinity Cache cannot serve them.

value = output Gpixel/s of the autotuned step (10 x 4096^2 pixels per step).
Alongside: the plain (one pixel per thread) step, per-call Gpixel/s and % of
the binding roof (HBM 8 TB/s at 8 B/px, or the FP32 FMA rate), the roofline of
the dominant kernel, the FP64 CPU oracle on a bounded sample of the same
workload, and (unless --no-extras) the corner pipeline, the uneven half-float
batch, the filter-bank forward+backward step and the paper's own two convolution
settings (separable 4096^2 float with the constant boundary; 2-D 8192^2 unsigned
char, clamped).
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

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
FP32_FMA_PEAK_TFLOPS = 78.6    # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz, packed FP32 disabled
FP32_PACKED_PEAK_TFLOPS = 157.3
FP16_MFMA_PEAK_TFLOPS = 2500.0  # dense FP16 matrix cores, published
EXTRAS = ("corner", "batch", "bank", "paper", "tuner", "volume")
INT_DOT2_PEAK_TMACS = 78.6     # v_dot2_i32_i16: 2 int16 MACs per lane per issue, 256 CU x 64 lanes x 2.4 GHz
METRIC = "Gpixel/s & % HBM peak, autotuned vs plain kernel; fwd+bwd Gpixel/s"


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=5)
    p.add_argument("--side", type=int, default=4096)
    p.add_argument("--no-extras", action="store_true")
    p.add_argument("--no-cpu", action="store_true")
    p.add_argument("--only", default="", help="comma list of sweep call labels (sep1 ... 2d7) and extra "
                   "workloads (corner, batch, bank, paper, tuner, volume) to run; a profiling aid")
    p.add_argument("--write-traffic", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                   help="turn rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE counter_collection.csv files of a --calib-copy "
                        "run into profiles/traffic.json and exit")
    p.add_argument("--write-workload-traffic", metavar="DIR",
                   help="turn the per-workload FETCH_SIZE / WRITE_SIZE runs under DIR into profiles/traffic.json "
                        "entries and profiles/hbm_traffic_workloads.md, and exit")
    p.add_argument("--write-trace-summary", nargs=2, metavar=("TRACE_DIR", "BENCH_JSON"),
                   help="turn a rocprofv3 --kernel-trace --stats run of bench.py (its csv directory and the bench "
                        "line it printed) into profiles/kernel_trace_sweep_4096_f32.md and "
                        "profiles/kernel_trace_workloads.md, and exit")
    p.add_argument("--write-counter-summary", nargs="+", metavar="DIR",
                   help="turn rocprofv3 --pmc SQ_* runs (one counter_collection.csv per DIR) into "
                        "profiles/sq_counters.md, and exit")
    p.add_argument("--calib-copy", action="store_true",
                   help="also run three 1 GiB device-to-device copies (a known byte count for counter calibration)")
    return p.parse_args()


def flops_per_px(kind, r):
    n = 2 * r + 1
    return 4 * n if kind == "sep" else 2 * n * n


def roof_gpx(kind, r, bytes_px=8.0):
    hbm = HBM_PEAK_GBS / bytes_px
    alu = FP32_FMA_PEAK_TFLOPS * 1e3 / flops_per_px(kind, r)
    return min(hbm, alu), ("hbm" if hbm <= alu else "alu")


# kernel source files per call kind: traffic figures are valid only for the source they were taken on
KERNEL_SOURCES = {"2d": ["conv2d.hip", "conv2d_mfma.hip", "tile_stage.hpp", "corr_tile.hpp", "icl_device.hpp"],
                  "sep": ["conv_sep.hip", "sep_tile.hpp", "sep_strip.hpp", "tile_stage.hpp", "icl_device.hpp"]}


def source_hash(*names):
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_1605_06399_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def stored_traffic(kernel_key, src_files):
    """HBM bytes per launch from a committed rocprofv3 --pmc summary, if it matches today's source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            d = json.load(f)
        e = d.get(kernel_key)
        if e and e.get("source_hash") == source_hash(*src_files):
            return e["bytes_per_launch"]
    except Exception:
        pass
    return None


def kernel_variant(name):
    """(kind, radius, variant name) of a float32 sweep kernel's symbol, else None."""
    import re
    pats = [("2d", r"conv2d_pers<icl::F32, (\d+), (\d+), (\d+)>", "pers_p{1}x{2}"),
            ("2d", r"conv2d_lds<icl::F32, (\d+), (\d+), (\d+), (\d+)>", "lds_p{1}x{2}_o{3}"),
            ("2d", r"conv2d_mfma_k<icl::F32, (\d+)>", "mfma_f16x3"),
            ("sep", r"sep_pers<icl::F32, (\d+), (\d+), (\d+)>", "pers_t{1}_c{2}"),
            ("sep", r"sep_fused<icl::F32, (\d+), (\d+), (\d+)>", "fused_t{1}_c{2}"),
            ("sep", r"sep_strip<icl::F32, (\d+), (\d+)>", "strip_t{1}"),
            ("sep", r"sep_fused_img<icl::F32, (\d+), (\d+), (\d+), false>", "fused_img_t{1}_c{2}"),
            ("sep", r"sep_fused_img<icl::F32, (\d+), (\d+), (\d+), true>", "fused_img4_t{1}_c{2}"),
            ("sep", r"sep_colwalk<icl::F32, (\d+), (\d+)>", "colwalk_s{1}")]
    for kind, pat, fmt in pats:
        m = re.search(pat, name)
        if m:
            g = m.groups()
            return kind, int(g[0]), fmt.format(*g)
    return None


def calib_factors(fetch_csv, write_csv):
    """Counter scale factors from the run's three 1 GiB device-to-device copies: the copy
    dispatches whose WRITE_SIZE reads 1 GiB (the copy-ceiling copies of other sizes are left
    out), paired in dispatch order with the same dispatches of the FETCH_SIZE run."""
    import csv

    def copies(p):
        return [float(r["Counter_Value"]) for r in csv.DictReader(open(p)) if "copyBuffer" in r["Kernel_Name"]]

    cf, cw = copies(fetch_csv), copies(write_csv)
    idx = [i for i, w in enumerate(cw) if abs(w - (1 << 20)) < 0.01 * (1 << 20)]
    if len(idx) < 1 or len(cf) != len(cw):
        raise RuntimeError("calibration copies not found: run with --calib-copy")
    f = [cf[i] for i in idx]
    w = [cw[i] for i in idx]
    return (1 << 20) / (sum(f) / len(f)), (1 << 20) / (sum(w) / len(w)), f, w


def write_traffic(fetch_csv, write_csv, side=4096):
    """HBM bytes per dispatch: mean FETCH_SIZE / WRITE_SIZE (KiB) per kernel, each scaled so that the
    counter reads 1 GiB on the run's three 1 GiB device-to-device copies."""
    import collections
    import csv

    def load(p):
        agg = collections.defaultdict(list)
        for r in csv.DictReader(open(p)):
            agg[r["Kernel_Name"]].append(float(r["Counter_Value"]))
        return agg

    fe, wr = load(fetch_csv), load(write_csv)
    fcal, wcal, cf, cw = calib_factors(fetch_csv, write_csv)
    alg = 8 * side * side
    out = {"_about": "HBM bytes per dispatch from rocprofv3 --pmc FETCH_SIZE and --pmc WRITE_SIZE (KiB per "
                     "dispatch, mean over dispatches), each scaled by the factor that maps the same counter on a "
                     "1 GiB device-to-device copy to 1 GiB; source_hash covers the kernel's source files and "
                     "bench.py reports traffic only while it matches.",
           "commands": [f"rocprofv3 --pmc {ctr} --output-format csv -d {os.path.dirname(csv_path)} -o "
                        f"{os.path.basename(csv_path).split('_counter_collection')[0]} -- "
                        "python3 bench.py --steps 3 --warmup 1 --no-extras --no-cpu --calib-copy"
                        for ctr, csv_path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv))],
           "calibration": {"fetch_factor": round(fcal, 4), "write_factor": round(wcal, 4),
                           "copy_fetch_kib": [round(v, 1) for v in cf], "copy_write_kib": [round(v, 1) for v in cw]}}
    for k in fe:
        v = kernel_variant(k)
        if not v or k not in wr:
            continue
        kind, r, name = v
        f, w = float(np.mean(fe[k])), float(np.mean(wr[k]))
        b = (f * fcal + w * wcal) * 1024
        out[f"{kind}{r}:{name}"] = {"fetch_kib": round(f, 1), "write_kib": round(w, 1), "bytes_per_launch": int(b),
                                    "algorithmic_bytes": alg, "ratio": round(b / alg, 3),
                                    "source_hash": source_hash(*KERNEL_SOURCES[kind])}
    path = os.path.join(ROOT, "profiles", "traffic.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    md = [f"# HBM traffic per launch: the {side}x{side} float32 sweep, every variant the tuner times", "",
          "Commands (repository root, one MI355X), one counter per pass:", "", "```", *out["commands"],
          f"python3 bench.py --write-traffic {fetch_csv} {write_csv}", "```", "",
          f"Calibration on the same runs: three 1 GiB device-to-device copies read FETCH_SIZE = "
          f"{np.mean(cf):.0f} KiB and WRITE_SIZE = {np.mean(cw):.0f} KiB per dispatch, so FETCH_SIZE is scaled by "
          f"{fcal:.4f} and WRITE_SIZE by {wcal:.4f}.  Algorithmic bytes per launch: {alg // 2:,} B read + "
          f"{alg // 2:,} B written.  The mean is over every dispatch of the kernel in the run (the tuner's "
          "timing launches and the timed steps).", "",
          "| call:variant | FETCH_SIZE (KiB) | WRITE_SIZE (KiB) | HBM bytes / launch | / algorithmic |",
          "|---|---|---|---|---|"]
    for k, v in out.items():
        if isinstance(v, dict) and "ratio" in v:
            md.append(f"| {k} | {v['fetch_kib']:.0f} | {v['write_kib']:.0f} | {v['bytes_per_launch']:,} | "
                      f"{v['ratio']:.3f} |")
    with open(os.path.join(ROOT, "profiles", f"hbm_traffic_sweep_{side}_f32.md"), "w") as fh:
        fh.write("\n".join(md) + "\n")
    print(f"wrote {path} and profiles/hbm_traffic_sweep_{side}_f32.md")


# Kernels of the extra workloads whose HBM traffic is summarised: (workload, symbol pattern, label,
# source files, algorithmic bytes per launch).  The symbols are those of the workloads' main launches
# (the border-band launches of corners and NMS are listed by the summary as they are).
_B_PX = 273398743          # pixels of the 256-image uneven batch (seeded recipe)
_BANK = (32, 16, 1024 * 1024)
WORKLOAD_KERNELS = [
    ("batch", r"sep_batched_k<icl::(F16|BF16), (\d+)>", "walk_t{1}_{0}", ["batched.hip", "sep_tile.hpp",
     "tile_stage.hpp", "icl_device.hpp"], 4 * _B_PX),
    ("batch", r"sep_batched_strip_k<icl::(F16|BF16)>", "strip_{0}", ["batched.hip", "sep_strip.hpp",
     "icl_device.hpp"], 4 * _B_PX),
    ("batch", r"sep_batched_col_k<icl::(F16|BF16), (\d), (\d+)>", "colwalk_cx{1}_step{2}_{0}",
     ["batched.hip", "sep_colwalk.hpp", "sep_tile.hpp", "tile_stage.hpp", "icl_device.hpp"], 4 * _B_PX),
    ("corner", r"harris_(fused|stream)<(\d+), (\d+)>", "harris_{0}_t{2}", ["harris.hip", "harris_strip.hpp",
     "icl_device.hpp"], 8 * 8192 * 8192),
    ("corner", r"nms_stream<(\d+)>", "nms_stream_t{0}", ["nms.hip", "harris_strip.hpp", "icl_device.hpp"],
     5 * 8192 * 8192),
    ("corner", r"nms_stream_a<(\d+), (true|false)>", "nms_stream_a_t{0}_sm:{1}", ["nms.hip", "harris_strip.hpp",
     "icl_device.hpp"], 5 * 8192 * 8192),
    ("corner", r"corners_stream<(\d+), (\d+), 1>", "corners_stream_t{1}", ["corners.hip", "harris_strip.hpp",
     "icl_device.hpp"], 5 * 8192 * 8192),
    ("bank", r"bank_fwd_(mfma_k<4, true, \d+, (?:true|false)>|pers_k<4, true>|sse_tpre_k<4>)", "fwd_sse:{0}",
     ["bank.hip"],
     4 * (_BANK[0] * _BANK[2] + 2 * _BANK[0] * _BANK[1] * _BANK[2])),
    ("bank", r"bank_bwd_in_(pers_k|k)<4>", "bwd_input:{0}", ["bank.hip"],
     4 * (_BANK[0] * _BANK[1] * _BANK[2] + _BANK[0] * _BANK[2])),
    ("bank", r"bank_bwd_(wm_k<4, \d, (?:true|false)(?:, (?:true|false))?>|w4_k<4, \d, 16>)", "bwd_filter:{0}",
     ["bank.hip"],
     4 * (_BANK[0] * _BANK[1] * _BANK[2] + _BANK[0] * _BANK[2])),
    ("paper", r"sep_(fused|pers)<icl::F32, 2, (\d+), (\d+)>", "sep5_constant:{0}_t{1}_c{2}",
     KERNEL_SOURCES["sep"], 8 * 4096 * 4096),
    ("paper", r"u8_strip<2, (\d+), (\d+), (\d+)>", "u8_5x5:strip_p{1}_t{0}_q{2}", ["conv2d_u8.hip", "icl_device.hpp"],
     2 * 8192 * 8192),
    ("volume", r"sep3_stream<icl::F32, (\d+), (\d+)>", "sep3d_r{0}:stream_z{1}", ["conv3d.hip", "icl_device.hpp"],
     8 * 256 ** 3),
    ("volume", r"sep3_stream2<icl::F32, (\d+), (\d+), (\d+)>", "sep3d_r{0}:stream2_z{1}_h{2}",
     ["conv3d.hip", "icl_device.hpp"], 8 * 256 ** 3),
]


def write_workload_traffic(root):
    """HBM bytes per dispatch of the extra workloads' kernels from rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE
    runs of `bench.py --only <workload> --calib-copy` (one directory per workload and counter under root),
    scaled by the run's 1 GiB calibration copies; merged into profiles/traffic.json and tabulated in
    profiles/hbm_traffic_workloads.md."""
    import collections
    import csv
    import re

    def load(p):
        # per kernel, the dispatches of its largest grid (the full-size launches; a kernel that is also
        # launched on small checks or border bands has other grid sizes)
        agg = collections.defaultdict(lambda: collections.defaultdict(list))
        for r in csv.DictReader(open(p)):
            agg[r["Kernel_Name"]][int(r["Grid_Size"])].append(float(r["Counter_Value"]))
        return {k: g[max(g)] for k, g in agg.items()}

    path = os.path.join(ROOT, "profiles", "traffic.json")
    out = json.load(open(path)) if os.path.exists(path) else {}
    rows, cmds = [], []
    for wl in EXTRAS:
        fp = os.path.join(root, f"tr_{wl}_FETCH_SIZE", "tr_counter_collection.csv")
        wp = os.path.join(root, f"tr_{wl}_WRITE_SIZE", "tr_counter_collection.csv")
        if not (os.path.exists(fp) and os.path.exists(wp)):
            continue
        for ctr in ("FETCH_SIZE", "WRITE_SIZE"):
            cmds.append(f"rocprofv3 --pmc {ctr} --output-format csv -d {root}/tr_{wl}_{ctr} -o tr -- "
                        f"python3 bench.py --only {wl} --steps 4 --warmup 1 --no-cpu --calib-copy")
        fe, wr = load(fp), load(wp)
        fcal, wcal, _, _ = calib_factors(fp, wp)
        for kname in sorted(fe):
            for w2, pat, label, srcs, alg in WORKLOAD_KERNELS:
                m = re.search(pat, kname)
                if w2 != wl or not m or kname not in wr:
                    continue
                f, w = float(np.mean(fe[kname])), float(np.mean(wr[kname]))
                b = (f * fcal + w * wcal) * 1024
                key = f"{wl}:{label.format(*m.groups())}"
                out[key] = {"fetch_kib": round(f, 1), "write_kib": round(w, 1), "dispatches": len(fe[kname]),
                            "fetch_factor": round(fcal, 4), "write_factor": round(wcal, 4),
                            "bytes_per_launch": int(b), "algorithmic_bytes": alg, "ratio": round(b / alg, 3),
                            "source_hash": source_hash(*srcs)}
                rows.append((key, f, w, len(fe[kname]), int(b), alg, b / alg))
    out["_workload_commands"] = cmds
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    md = ["# HBM traffic per launch: the extra workloads' kernels", "",
          "Commands (repository root, one MI355X), one counter per pass; then "
          f"`python3 bench.py --write-workload-traffic {root}`:", "", "```", *cmds, "```", "",
          "Each counter is scaled by what it reads on the same run's three 1 GiB device-to-device copies "
          "(FETCH_SIZE reads half the copied bytes, WRITE_SIZE all of them); the mean is over a kernel's "
          "dispatches of its largest grid (the full-size launches).  Algorithmic bytes: what the call "
          "must read and write once (batch 4 B/px over 273,398,743 px; Harris 8 B/px, NMS and fused corners "
          "5 B/px at 8192^2; filter bank at 32 x 16 x 1024^2: x + t read and gy written for the fused "
          "forward+loss, gy + x (+ gx) for the adjoints; separable 5x5 8 B/px at 4096^2; unsigned char 5x5 "
          "2 B/px at 8192^2; separable 3-D 8 B/voxel at 256^3).", "",
          "| workload:kernel | dispatches | FETCH_SIZE (KiB) | WRITE_SIZE (KiB) | HBM bytes / launch | algorithmic "
          "| ratio |", "|---|---|---|---|---|---|---|"]
    for key, f, w, n, b, alg, ratio in rows:
        md.append(f"| {key} | {n} | {f:.0f} | {w:.0f} | {b:,} | {alg:,} | {ratio:.3f} |")
    with open(os.path.join(ROOT, "profiles", "hbm_traffic_workloads.md"), "w") as fh:
        fh.write("\n".join(md) + "\n")
    print(f"wrote {path} and profiles/hbm_traffic_workloads.md ({len(rows)} kernels)")


def _short_kernel(name):
    """A kernel symbol without its namespaces and parameter list."""
    import re
    n = name.replace("void ", "", 1).replace("(anonymous namespace)::", "").replace("icl::", "")
    depth, cut = 0, len(n)
    for i, ch in enumerate(n):   # the parameter list starts at the first '(' outside template brackets
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            cut = i
            break
    return re.sub(r"\s+", " ", n[:cut]).strip()


def write_trace_summary(trace_dir, bench_json, out_dir=None):
    """Kernel-trace summaries of one profiled default bench run: the sweep's calls (trace means of the
    timed dispatches beside bench.py's event means) and every kernel of the extra workloads."""
    import csv
    import glob
    line = [ln for ln in open(bench_json).read().splitlines() if ln.startswith("{")][-1]
    d = json.loads(line)
    steps = int(d["steps"])
    trace = glob.glob(os.path.join(trace_dir, "*kernel_trace.csv"))[0]
    stats = glob.glob(os.path.join(trace_dir, "*kernel_stats.csv"))[0]
    disp = [(r["Kernel_Name"], (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
            for r in csv.DictReader(open(trace))]
    tag = os.path.basename(trace).split("_kernel_trace")[0]
    prof = (f"rocprofv3 --kernel-trace --stats --output-format csv -d {trace_dir} -o {tag} -- "
            f"python3 bench.py --no-cpu > {bench_json}")
    summ = f"python3 bench.py --write-trace-summary {trace_dir} {bench_json}"
    md = ["# Kernel trace: convolution sweep 4096x4096 float32", "",
          "Commands (repository root, one MI355X):", "", "```", prof, summ, "```", "",
          f"The profiled run is the default bench (tuning, {d['warmup']} warmup and {steps} timed steps, the "
          "plain-variant steps, then the extra workloads).  bench.py times each call as one HIP-event pair "
          f"around its {steps} back-to-back launches (rotating buffers, so every launch reads its input from "
          "HBM); the timed dispatches are the first run of exactly that many consecutive dispatches of the "
          "call's kernel in the trace.  The all-dispatch mean also holds the tuner's timing launches and "
          "the later workloads' launches of the same kernel.", "",
          "| call | variant | kernel | trace mean, timed dispatches (us) | bench.py event mean (us) | "
          "trace mean, all dispatches (us) | min (us) | dispatches |", "|---|---|---|---|---|---|---|---|"]
    dom = None
    for c in d["per_call"]:
        kind, r = c["call"][:-1], int(c["call"][-1])
        sym = next((k for k, _ in disp if kernel_variant(k) == (kind, r, c["variant"])), None)
        if sym is None:
            md.append(f"| {c['call']} | {c['variant']} | (not found) | | {c['us']} | | | |")
            continue
        idx = [i for i, (k, _) in enumerate(disp) if k == sym]
        runs, cur = [], [idx[0]]
        for i in idx[1:]:
            if i == cur[-1] + 1:
                cur.append(i)
            else:
                runs.append(cur)
                cur = [i]
        runs.append(cur)
        # the timed launches: the first run of exactly `steps` consecutive dispatches (the tuner's
        # runs hold 43, the warmup's 1, and later workloads may time the same kernel again)
        timed = [rn for rn in runs if len(rn) == steps]
        tmean = float(np.mean([disp[i][1] for i in timed[0]])) if timed else float("nan")
        allt = [disp[i][1] for i in idx]
        md.append(f"| {c['call']} | {c['variant']} | `{_short_kernel(sym)}` | {tmean:.2f} | {c['us']:.2f} | "
                  f"{np.mean(allt):.2f} | {min(allt):.2f} | {len(allt)} |")
        if c["call"] == d["roofline"].get("kernel", "").split(":")[0]:
            dom = (c["call"], c["variant"], tmean, d["roofline"].get("launch_us"))
    md += ["", f"The bench line under the profiler: {d['value']} {d['unit']}, {d['ms_per_step']} ms/step."]
    if dom:
        md += ["", f"Roofline kernel ({dom[0]}:{dom[1]}): {dom[2]:.2f} us per timed dispatch in the trace against "
                   f"bench.py's event-timed {dom[3]} us per launch."]
    out_dir = out_dir or os.path.join(ROOT, "profiles")
    with open(os.path.join(out_dir, "kernel_trace_sweep_4096_f32.md"), "w") as fh:
        fh.write("\n".join(md) + "\n")
    rows = sorted(csv.DictReader(open(stats)), key=lambda r: _short_kernel(r["Name"]))
    torch_rows = [r for r in rows if r["Name"].startswith("at::") or r["Name"].startswith("void at::")]
    rows = [r for r in rows if r not in torch_rows]
    ex = d.get("extras", {})
    md = ["# Kernel trace: every kernel of the profiled default bench run", "",
          "Commands (repository root, one MI355X):", "", "```", prof, summ, "```", "",
          "bench.py times every variant of every workload (forced) beside its tuned choice, and the tuner "
          "times the candidates, so each kernel appears; the extra workloads' figures are below the table.", "",
          "| kernel | calls | mean (us) | min (us) | max (us) |", "|---|---|---|---|---|"]
    for r in rows:
        md.append(f"| `{_short_kernel(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                  f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} |")
    md += ["", f"Not listed: {sum(int(r['Calls']) for r in torch_rows)} dispatches of {len(torch_rows)} PyTorch "
           "kernels (input uploads, dtype conversions and the bench's own equality checks).",
           "", "bench.py's extra-workload figures in the profiled run:", "", "| workload | time | variant |",
           "|---|---|---|"]
    for k, v in ex.items():
        if not isinstance(v, dict):
            continue
        t = f"{v['ms']} ms" if "ms" in v else (f"{v['us']} us" if "us" in v else "")
        var = v.get("variant") or v.get("harris_variant") or ""
        if k == "filter_bank_fwd_bwd":
            var = ", ".join(f"{p}: {q['variant']} {q['ms']} ms" for p, q in v.get("phases", {}).items())
        md.append(f"| {k} | {t} | {var} |")
    with open(os.path.join(out_dir, "kernel_trace_workloads.md"), "w") as fh:
        fh.write("\n".join(md) + "\n")
    print(f"wrote kernel_trace_sweep_4096_f32.md and kernel_trace_workloads.md in {out_dir}")


# SQ counter passes (at most 8 SQ counters each) and the bench runs they profile
SQ_PASSES = {"A": "SQ_WAVES SQ_BUSY_CYCLES SQ_WAVE_CYCLES SQ_INSTS_VALU SQ_ACTIVE_INST_VALU SQ_INSTS_MFMA "
                  "SQ_VALU_MFMA_BUSY_CYCLES SQ_INSTS_SALU",
             "B": "SQ_INSTS_LDS SQ_ACTIVE_INST_LDS SQ_WAIT_INST_LDS SQ_LDS_BANK_CONFLICT SQ_WAIT_INST_ANY "
                  "SQ_INSTS_VMEM_RD SQ_INSTS_VMEM_WR SQ_WAVE_CYCLES"}
SQ_RUNS = {"sweep": "--steps 3 --warmup 1 --no-extras --no-cpu", "bank": "--only bank --steps 4 --warmup 1 --no-cpu",
           "batch": "--only batch --steps 4 --warmup 1 --no-cpu", "corner": "--only corner --steps 4 --warmup 1 --no-cpu",
           "paper": "--only paper --steps 4 --warmup 1 --no-cpu"}
SQ_KERNELS = (r"conv2d_pers<F32, [1-7], ", r"sep_(fused|pers)<F32, [1-7], ", r"bank_(fwd_mfma_k<4, true, 0, true>|"
              r"bwd_in_pers_k<4>|bwd_wm_k<4, 4, true, (?:true|false)>)", r"sep_batched_col_k<F16, 1, 64>", r"harris_stream<2, 16>",
              r"nms_stream_a<4, false>", r"corners_stream<2, 12, 1>", r"u8_strip<2, \d+, \d+, \d+>")


def write_counter_summary(dirs, out_dir=None):
    """Per-kernel SQ counter ratios from rocprofv3 --pmc passes (directories named sq{pass}_{run})."""
    import collections
    import csv
    import glob
    import re
    agg = collections.defaultdict(lambda: collections.defaultdict(list))
    for dd in dirs:
        for path in glob.glob(os.path.join(dd, "*counter_collection.csv")):
            for r in csv.DictReader(open(path)):
                k = _short_kernel(r["Kernel_Name"])
                if not any(re.search(p, k) for p in SQ_KERNELS):
                    continue
                agg[k][r["Counter_Name"]].append(float(r["Counter_Value"]))
                agg[k]["_us"].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    # one run per directory, named sq<pass>_<run> (a pass of SQ_PASSES over a run of SQ_RUNS)
    cmds = []
    for dd in dirs:
        ps, _, run = os.path.basename(os.path.normpath(dd))[2:].partition("_")
        if ps in SQ_PASSES and run in SQ_RUNS:
            cmds.append(f"rocprofv3 --pmc {SQ_PASSES[ps]} --output-format csv -d {dd} -o sq -- "
                        f"python3 bench.py {SQ_RUNS[run]}")
    md = ["# SQ counters: what the main kernels spend their time on", "", "Commands (repository root, one MI355X), one "
          "pass of at most eight SQ counters per run:", "", "```", *cmds,
          "python3 bench.py --write-counter-summary " + " ".join(dirs), "```", "",
          "Per kernel, the mean per dispatch over every dispatch of the profiled runs (the tuner's included).  "
          "Ratios: `valu/cyc` = VALU instructions x 4 / (SIMD count x kernel cycles at 2.4 GHz), the share of "
          "the vector units' issue a wave64 FP32 instruction takes at 16 lanes a cycle (over 1 where some "
          "instructions take fewer cycles, or the clock runs higher); `mfma busy` = SQ_VALU_MFMA_BUSY_CYCLES / "
          "(SIMD count x kernel cycles); `lds conflict` = bank-conflict cycles per cycle of LDS instruction "
          "activity; `lds wait`, `any wait` = SQ_WAIT_INST_LDS and SQ_WAIT_INST_ANY over SQ_WAVE_CYCLES (the "
          "share of wave time spent waiting); `lds/valu` = LDS instructions per VALU instruction.  Kernel "
          "times run longer under counter collection than in the bench.", "",
          "| kernel | us | VALU instr | valu/cyc | MFMA instr | mfma busy | LDS instr | lds/valu | lds conflict | "
          "lds wait | any wait |", "|---|---|---|---|---|---|---|---|---|---|---|"]
    simds, clk = 1024, 2.4e3   # SIMDs; cycles per us
    for k in sorted(agg):
        c = {n: float(np.mean(v)) for n, v in agg[k].items()}
        us = c["_us"]
        g = c.get
        cyc = simds * us * clk

        def ratio(a, b):
            return f"{a / b:.2f}" if a is not None and b else ""
        md.append(f"| `{k}` | {us:.1f} | {g('SQ_INSTS_VALU', 0):.3g} | {ratio(4 * g('SQ_INSTS_VALU', 0), cyc)} | "
                  f"{g('SQ_INSTS_MFMA', 0):.3g} | {ratio(g('SQ_VALU_MFMA_BUSY_CYCLES'), cyc)} | "
                  f"{g('SQ_INSTS_LDS', 0):.3g} | {ratio(g('SQ_INSTS_LDS'), g('SQ_INSTS_VALU'))} | "
                  f"{ratio(g('SQ_LDS_BANK_CONFLICT'), g('SQ_ACTIVE_INST_LDS'))} | "
                  f"{ratio(g('SQ_WAIT_INST_LDS'), g('SQ_WAVE_CYCLES'))} | "
                  f"{ratio(g('SQ_WAIT_INST_ANY'), g('SQ_WAVE_CYCLES'))} |")
    with open(os.path.join(out_dir or os.path.join(ROOT, "profiles"), "sq_counters.md"), "w") as fh:
        fh.write("\n".join(md) + "\n")
    print(f"wrote sq_counters.md in {out_dir or os.path.join(ROOT, 'profiles')} ({len(agg)} kernels)")


def main():
    a = parse()
    if a.write_counter_summary:
        write_counter_summary(a.write_counter_summary)
        return
    if a.write_trace_summary:
        write_trace_summary(*a.write_trace_summary)
        return
    if a.write_traffic:
        write_traffic(*a.write_traffic, side=a.side)
        return
    if a.write_workload_traffic:
        write_workload_traffic(a.write_workload_traffic)
        return
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}); sharding over several GPUs "
              "is a design, not part of this library.", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1605_06399_amd import binding as B, synth
    from paper_1605_06399_amd import torch_api as T

    dev = torch.device("cuda:0")
    side = a.side
    radii = synth.SWEEP_RADII
    img = synth.sweep_image(side)
    NSET = 8
    src = [torch.from_numpy(img).to(dev) for _ in range(NSET)]
    dst = [torch.empty_like(src[0]) for _ in range(NSET)]
    _, wsb = B.icl_workspace_size(B.ICL_OP_CONV_SEP, side, side)
    ws = torch.empty(wsb // 4, dtype=torch.float32, device=dev)
    taps = {}
    for r in radii:
        h, v = synth.sweep_taps_sep(r)
        taps[("sep", r)] = (torch.from_numpy(h).to(dev), torch.from_numpy(v).to(dev))
        taps[("2d", r)] = torch.from_numpy(synth.sweep_taps_2d(r)).to(dev)
    calls = [(k, r) for r in radii for k in ("sep", "2d")]
    extras = EXTRAS
    if a.only:
        keep = set(a.only.split(","))
        calls = [c for c in calls if f"{c[0]}{c[1]}" in keep]
        extras = tuple(e for e in EXTRAS if e in keep)
    if not calls:
        # profiling aid: the extra workloads alone, no sweep line
        del src, dst, ws
        torch.cuda.empty_cache()
        out = {}
        if a.calib_copy:
            out["calib_copy_bytes_each_way"] = calib_copies(torch, dev)
        out["extras"] = run_extras(torch, B, T, synth, max(3, a.steps // 2), extras)
        print(json.dumps(out), flush=True)
        return
    stream = torch.cuda.current_stream()

    def call(kind, r, k):
        if kind == "sep":
            h, v = taps[("sep", r)]
            T.conv_sep(src[k], h, v, out=dst[k], workspace=ws)
        else:
            T.conv2d(src[k], taps[("2d", r)], out=dst[k])

    # autotune every call of the sweep (outside the timed region)
    t_tune = time.perf_counter()
    for kind, r in calls:
        op = B.ICL_OP_CONV_SEP if kind == "sep" else B.ICL_OP_CONV2D
        B.check(B.icl_tune(op, B.ICL_F32, r, side, side, stream.cuda_stream), "icl_tune")
    torch.cuda.synchronize()
    t_tune = time.perf_counter() - t_tune
    chosen, arith = {}, {}
    for kind, r in calls:
        op = B.ICL_OP_CONV_SEP if kind == "sep" else B.ICL_OP_CONV2D
        vi = B.icl_selected_variant(op, B.ICL_F32, r, side, side)[1]
        chosen[f"{kind}{r}"] = B.icl_variant_name(op, vi)
        arith[f"{kind}{r}"] = B.icl_variant_arith(op, vi)

    def run(steps, warmup, label):
        """Time `steps` steps.  The calls of the steps run grouped by call (all launches of one
        call back to back, rotating buffers), so one event pair per call brackets `steps`
        launches and the per-launch mean carries no per-launch event overhead."""
        k = 0
        for _ in range(warmup):
            for kind, r in calls:
                call(kind, r, k % NSET)
                k += 1
        evs = {}
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for c in calls:
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(steps):
                call(c[0], c[1], k % NSET)
                k += 1
            e1.record(stream)
            evs[c] = (e0, e1)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        per = {c: e0.elapsed_time(e1) * 1e3 / steps for c, (e0, e1) in evs.items()}   # us per launch
        print(f"[bench] {label}: {dt * 1e3:.3f} ms/step", file=sys.stderr, flush=True)
        return dt, per

    dt_tuned, per_tuned = run(a.steps, a.warmup, "tuned")
    B.check(B.icl_force_variant(B.ICL_OP_CONV_SEP, 0))
    B.check(B.icl_force_variant(B.ICL_OP_CONV2D, 0))
    dt_plain, per_plain = run(max(2, a.steps // 4), max(1, a.warmup // 2), "plain")
    B.icl_force_variant(B.ICL_OP_CONV_SEP, -1)
    B.icl_force_variant(B.ICL_OP_CONV2D, -1)

    px = side * side
    ceiling = copy_ceiling(torch, dev)
    copy_gbs = ceiling["64MiB"]["GB_s"]     # a copy of the same bytes as one call (64 MiB in, 64 MiB out)
    per_op = []
    for kind, r in calls:
        us, usp = per_tuned[(kind, r)], per_plain[(kind, r)]
        gpx = px / (us * 1e-6) / 1e9
        roof, bound = roof_gpx(kind, r)
        if arith[f"{kind}{r}"] == "fp16x3_mfma":
            roof, bound = FP16_MFMA_PEAK_TFLOPS * 1e3 / flops_per_px(kind, r), "mfma"
        per_op.append({"call": f"{kind}{r}", "variant": chosen[f"{kind}{r}"], "arith": arith[f"{kind}{r}"],
                       "us": round(us, 2), "gpx_s": round(gpx, 1), "hbm_frac": round(gpx * 8 / HBM_PEAK_GBS, 3),
                       "copy_frac": round(gpx * 8 / copy_gbs, 3),
                       "binding_roof": bound, "roof_frac": round(gpx / roof, 3),
                       "plain_us": round(usp, 2), "speedup_vs_plain": round(usp / us, 2)})
    dom = max(calls, key=lambda c: per_tuned[c])
    kind, r = dom
    us = per_tuned[dom]
    _, bound = roof_gpx(kind, r)
    if arith[f"{kind}{r}"] == "fp16x3_mfma":
        # the matrix-core variant: FP16 MFMAs (hi/lo split) against the dense FP16 matrix peak;
        # executed = 3 products x 2 flop x 32 band columns x (2r+1) tap rows per pixel
        achieved = flops_per_px(kind, r) * px / (us * 1e-6) / 1e12
        executed = 3 * 2 * 32 * (2 * r + 1) * px
        roofline = {"bound": "mfma", "achieved": round(achieved, 2), "peak": FP16_MFMA_PEAK_TFLOPS,
                    "unit": "TFLOP/s", "frac": round(achieved / FP16_MFMA_PEAK_TFLOPS, 4),
                    "executed_flops_per_launch": executed,
                    "executed_frac": round(executed / (us * 1e-6) / 1e12 / FP16_MFMA_PEAK_TFLOPS, 3),
                    "hbm_frac": round(8.0 * px / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 3)}
    elif bound == "alu":
        achieved = flops_per_px(kind, r) * px / (us * 1e-6) / 1e12
        roofline = {"bound": "alu", "achieved": round(achieved, 2), "peak": FP32_FMA_PEAK_TFLOPS,
                    "unit": "TFLOP/s", "frac": round(achieved / FP32_FMA_PEAK_TFLOPS, 3)}
        roofline["frac_of_packed_fp32_peak"] = round(achieved / FP32_PACKED_PEAK_TFLOPS, 3)
    else:
        achieved = 8.0 * px / (us * 1e-6) / 1e9
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 3)}
    key = f"{kind}{r}:{chosen[f'{kind}{r}']}"
    roofline["traffic"] = stored_traffic(key, KERNEL_SOURCES[kind])
    roofline["kernel"] = key
    roofline["algorithmic_bytes_per_launch"] = 8 * px
    roofline["flops_per_launch"] = flops_per_px(kind, r) * px
    roofline["launch_us"] = round(us, 2)

    value = len(calls) * px / dt_tuned / 1e9
    plain_value = len(calls) * px / dt_plain / 1e9
    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "Gpixel/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": round(dt_tuned * 1e3, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"convolution sweep {side}x{side} f32: separable + full 2-D filters, "
                               f"radius {','.join(map(str, radii))}, clamp-to-edge, N(0,1) taps normalised",
                   "calls_per_step": len(calls), "pixels_per_call": px, "rotating_buffers_GiB": 2 * NSET * px * 4 / 2 ** 30},
        "plain": {"value": round(plain_value, 2), "ms_per_step": round(dt_plain * 1e3, 4),
                  "tuned_speedup": round(dt_plain / dt_tuned, 2)},
        "hbm_frac_step": round(value * 8 / HBM_PEAK_GBS, 3),
        "copy_frac_step": round(value * 8 / copy_gbs, 3),
        "math_mode": "fp32" if B.icl_get_math() == B.ICL_MATH_F32 else "fp16_split",
        "arith_per_call": sorted(set(arith.values())),
        "copy_ceiling": ceiling,
        "tune_seconds": round(t_tune, 2),
        "per_call": per_op,
        "roofline": roofline,
    }
    del src, dst, ws
    torch.cuda.empty_cache()
    if a.calib_copy:
        out["calib_copy_bytes_each_way"] = calib_copies(torch, dev)

    if not a.no_extras:
        try:
            out["extras"] = run_extras(torch, B, T, synth, max(3, a.steps // 2), extras)
        except Exception as e:  # an extra never hides the sweep's line
            out["extras"] = {"error": repr(e)}

    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(synth, radii, side)
    print(json.dumps(out), flush=True)


def calib_copies(torch, dev):
    """Three 1 GiB device-to-device copies: a known byte count that scales the traffic counters."""
    n = (1 << 30) // 4
    c_src = torch.ones(n, dtype=torch.float32, device=dev)
    c_dst = torch.empty_like(c_src)
    for _ in range(3):
        c_dst.copy_(c_src)
    torch.cuda.synchronize()
    del c_src, c_dst
    torch.cuda.empty_cache()
    return 1 << 30


def copy_ceiling(torch, dev, reps=10):
    """Achievable copy bandwidth: device-to-device copies (the runtime's copy kernel) of 64 MiB,
    256 MiB and 2 GiB, rotating over enough source/destination pairs that the 256 MB Infinity Cache
    cannot hold them (1 GiB or more in flight), events around `reps` copies each.  GB/s counts the
    bytes read plus the bytes written."""
    out = {}
    for label, nbytes, pairs in (("64MiB", 64 << 20, 8), ("256MiB", 256 << 20, 4), ("2GiB", 2 << 30, 1)):
        n = nbytes // 4
        srcs = [torch.ones(n, dtype=torch.float32, device=dev) for _ in range(pairs)]
        dsts = [torch.empty_like(srcs[0]) for _ in range(pairs)]
        for k in range(2 * pairs):
            dsts[k % pairs].copy_(srcs[k % pairs])
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for k in range(reps):
            dsts[k % pairs].copy_(srcs[k % pairs])
        e1.record()
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / reps
        out[label] = {"us": round(us, 2), "GB_s": round(2 * nbytes / (us * 1e-6) / 1e9, 1),
                      "frac_of_peak": round(2 * nbytes / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 3)}
        del srcs, dsts
        torch.cuda.empty_cache()
    return out


def _time(torch, fn, steps, warmup=2):
    for _ in range(warmup):
        fn(0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        fn(s)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def _time_graph(torch, fn, launches, reps=5):
    """Per-call seconds of `launches` calls captured once in a HIP graph and replayed `reps`
    times between events: the host-side cost of the Python front end drops out, so calls
    shorter than it are timed by the device.  fn(s) must allocate nothing and clear no memory
    (a graph must hold no memset node)."""
    for s in range(2):
        fn(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for s in range(launches):
            fn(s)
    g.replay()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    del g
    return e0.elapsed_time(e1) * 1e-3 / (reps * launches)


def run_extras(torch, B, T, synth, steps, which=EXTRAS):
    """The other workloads, timed the same way (inputs resident in HBM, events around the whole step)."""
    res = {}
    if "corner" in which:
        res.update(extra_corner(torch, B, T, synth, steps))
    if "batch" in which:
        res.update(extra_batch(torch, B, T, synth, steps))
    if "bank" in which:
        res.update(extra_bank(torch, B, T, synth, steps))
    if "paper" in which:
        res.update(extra_paper(torch, B, T, synth, steps))
    if "tuner" in which:
        res.update(extra_tuner(torch, B, T, synth, steps))
    if "volume" in which:
        res.update(extra_volume(torch, B, T, synth, steps))
    return res


def extra_volume(torch, B, T, synth, steps):
    """Separable 3-D correlation of a 256^3 float32 volume (the Image type's 3-D indexing):
    radii 1..3, every variant, 8 algorithmic B/voxel."""
    dev = torch.device("cuda:0")
    side = 256
    vol = synth.volume_uniform(7, side, side, side)
    xs = [torch.from_numpy(vol).to(dev) for _ in range(2)]
    ys = [torch.empty_like(xs[0]) for _ in range(2)]
    _, nb = B.icl_workspace_size(B.ICL_OP_CONV3D_SEP, side, side, n=side)
    ws = torch.empty(nb // 4 + 1, dtype=torch.float32, device=dev)
    res = {}
    for r in (1, 2, 3):
        tx, ty, tz = (torch.from_numpy(synth.gaussian_taps(r, max(1.0, r / 2.0))).to(dev) for _ in range(3))

        def call(s):
            T.conv3d_sep(xs[s % 2], tx, ty, tz, out=ys[s % 2], workspace=ws)

        B.check(B.icl_tune_problem(B.ICL_OP_CONV3D_SEP, B.ICL_F32, r, side, side, depth=side,
                                   stream=torch.cuda.current_stream().cuda_stream), "tune volume")
        per_variant = {}
        for v in range(B.icl_variant_count(B.ICL_OP_CONV3D_SEP)):
            B.check(B.icl_force_variant(B.ICL_OP_CONV3D_SEP, v))
            try:
                per_variant[B.icl_variant_name(B.ICL_OP_CONV3D_SEP, v)] = round(
                    _time_graph(torch, call, steps) * 1e6, 1)
            finally:
                B.icl_force_variant(B.ICL_OP_CONV3D_SEP, -1)
        dt = _time_graph(torch, call, 2 * steps)
        gvx = side ** 3 / dt / 1e9
        res[f"volume_sep3d_r{r}_256_f32"] = {
            "us": round(dt * 1e6, 2), "gvoxel_s": round(gvx, 1), "bytes_per_voxel": 8,
            "hbm_frac": round(gvx * 8 / HBM_PEAK_GBS, 3),
            "variant": B.icl_variant_name(B.ICL_OP_CONV3D_SEP, B.icl_selected_variant_problem(
                B.ICL_OP_CONV3D_SEP, B.ICL_F32, r, side, side, depth=side)[1]),
            "variants_us": per_variant}
    del xs, ys, ws
    torch.cuda.empty_cache()
    return res


def extra_tuner(torch, B, T, synth, steps):
    """Exhaustive search against the paper's model-guided search (4 sampled candidates, neural
    time model, 2 best-predicted confirmed) on the sweep's largest calls: candidates timed,
    search seconds, and the chosen variant's time measured afterwards."""
    dev = torch.device("cuda:0")
    st = torch.cuda.current_stream().cuda_stream
    img = synth.sweep_image()
    H, W = img.shape
    xs = [torch.from_numpy(img).to(dev) for _ in range(4)]
    ys = [torch.empty_like(xs[0]) for _ in range(4)]
    ws = torch.empty(B.icl_workspace_size(B.ICL_OP_CONV_SEP, W, H)[1] // 4 + 1, dtype=torch.float32, device=dev)
    res = {}
    for kind, r in (("sep", 7), ("2d", 5), ("2d", 7)):
        op = B.ICL_OP_CONV_SEP if kind == "sep" else B.ICL_OP_CONV2D
        if kind == "sep":
            h, v = (torch.from_numpy(t).to(dev) for t in synth.sweep_taps_sep(r))
            fn = lambda s: T.conv_sep(xs[s % 4], h, v, out=ys[s % 4], workspace=ws)   # noqa: E731
        else:
            w = torch.from_numpy(synth.sweep_taps_2d(r)).to(dev)
            fn = lambda s: T.conv2d(xs[s % 4], w, out=ys[s % 4])   # noqa: E731
        row = {"candidates": B.icl_variant_count(op) - 1}
        for mode in ("exhaustive", "model"):
            B.icl_tune_clear()
            t0 = time.perf_counter()
            if mode == "exhaustive":
                B.check(B.icl_tune(op, B.ICL_F32, r, W, H, st))
                timed = row["candidates"]
            else:
                stat, timed = B.icl_tune_model(op, B.ICL_F32, r, W, H, 4, 2, 2024, st)
                B.check(stat)
            torch.cuda.synchronize()
            secs = time.perf_counter() - t0
            vi = B.icl_selected_variant(op, B.ICL_F32, r, W, H)[1]
            us = _time_graph(torch, fn, 2 * steps) * 1e6
            row[mode] = {"variant": B.icl_variant_name(op, vi), "timed": timed, "search_s": round(secs, 3),
                         "us": round(us, 2)}
        row["model_vs_exhaustive_time"] = round(row["model"]["us"] / row["exhaustive"]["us"], 3)
        res[f"tuner_{kind}{r}_4096"] = row
    B.icl_tune_clear()
    del xs, ys, ws
    torch.cuda.empty_cache()
    return res


def extra_paper(torch, B, T, synth, steps):
    """The paper's two convolution benchmarks at their own settings: the separable 5x5 filter on
    a 4096^2 float image with the constant boundary (c = 0), and the full 5x5 filter on an
    8192^2 unsigned char image, clamped (int16 taps, exact integer sum, shift 12)."""
    dev = torch.device("cuda:0")
    st = torch.cuda.current_stream().cuda_stream
    res = {}
    NSET = 4
    # separable, constant boundary
    img = synth.sweep_image()
    H, W = img.shape
    xs = [torch.from_numpy(img).to(dev) for _ in range(NSET)]
    ys = [torch.empty_like(xs[0]) for _ in range(NSET)]
    h, v = synth.sweep_taps_sep(2)
    th, tv = torch.from_numpy(h).to(dev), torch.from_numpy(v).to(dev)
    ws = torch.empty(B.icl_workspace_size(B.ICL_OP_CONV_SEP, W, H)[1] // 4 + 1, dtype=torch.float32, device=dev)
    B.check(B.icl_tune(B.ICL_OP_CONV_SEP, B.ICL_F32, 2, W, H, st))

    def sep(s):
        T.conv_sep(xs[s % NSET], th, tv, out=ys[s % NSET], workspace=ws, border="constant", constant=0.0)

    dt = _time_graph(torch, sep, 4 * steps)
    per_variant = {}
    for vi in range(B.icl_variant_count(B.ICL_OP_CONV_SEP)):
        B.check(B.icl_force_variant(B.ICL_OP_CONV_SEP, vi))
        try:
            per_variant[B.icl_variant_name(B.ICL_OP_CONV_SEP, vi)] = round(_time_graph(torch, sep, 2 * steps) * 1e6,
                                                                           1)
        finally:
            B.icl_force_variant(B.ICL_OP_CONV_SEP, -1)
    gpx = H * W / dt / 1e9
    res["paper_sep5_constant_4096_f32"] = {
        "timing": "HIP graph replay of back-to-back calls over 4 rotating buffer pairs",
        "us": round(dt * 1e6, 2), "gpx_s": round(gpx, 1), "bytes_per_px": 8,
        "hbm_frac": round(gpx * 8 / HBM_PEAK_GBS, 3),
        "variant": B.icl_variant_name(B.ICL_OP_CONV_SEP, B.icl_selected_variant(B.ICL_OP_CONV_SEP, B.ICL_F32, 2, W,
                                                                                 H)[1]),
        "variants_us": per_variant}
    del xs, ys, ws
    torch.cuda.empty_cache()
    # unsigned char, clamped
    X = synth.paper_u8_image()
    H, W = X.shape
    xs = [torch.from_numpy(X).to(dev) for _ in range(NSET)]
    ys = [torch.empty_like(xs[0]) for _ in range(NSET)]
    td = torch.from_numpy(synth.u8_taps(6, 2, synth.U8_SHIFT)).to(dev)
    B.check(B.icl_tune(B.ICL_OP_CONV2D_U8, B.ICL_U8, 2, W, H, st))

    def u8(s):
        T.conv2d_u8(xs[s % NSET], td, synth.U8_SHIFT, out=ys[s % NSET])

    dt = _time_graph(torch, u8, 4 * steps)
    per_variant = {}
    for vi in range(B.icl_variant_count(B.ICL_OP_CONV2D_U8)):
        B.check(B.icl_force_variant(B.ICL_OP_CONV2D_U8, vi))
        try:
            per_variant[B.icl_variant_name(B.ICL_OP_CONV2D_U8, vi)] = round(
                _time_graph(torch, u8, steps if vi == 0 else 2 * steps, reps=2 if vi == 0 else 5) * 1e6, 1)
        finally:
            B.icl_force_variant(B.ICL_OP_CONV2D_U8, -1)
    gpx = H * W / dt / 1e9
    macs = 25 * H * W
    res["paper_conv2d5_u8_8192"] = {
        "timing": "HIP graph replay of back-to-back calls over 4 rotating buffer pairs",
        "us": round(dt * 1e6, 2), "gpx_s": round(gpx, 1), "bytes_per_px": 2,
        "hbm_frac": round(gpx * 2 / HBM_PEAK_GBS, 3),
        "int_tmac_s": round(macs / dt / 1e12, 2), "int_dot2_peak_tmac_s": INT_DOT2_PEAK_TMACS,
        "int_frac": round(macs / dt / 1e12 / INT_DOT2_PEAK_TMACS, 3),
        "variant": B.icl_variant_name(B.ICL_OP_CONV2D_U8, B.icl_selected_variant(B.ICL_OP_CONV2D_U8, B.ICL_U8, 2, W,
                                                                                   H)[1]),
        "variants_us": per_variant}
    del xs, ys
    torch.cuda.empty_cache()
    return res


def extra_corner(torch, B, T, synth, steps):
    dev = torch.device("cuda:0")
    res = {}
    # corner pipeline: Harris response + 3x3 NMS on 8192^2 (two calls: 8 + 5 algorithmic B/px)
    img = synth.corner_image()
    H, W = img.shape
    xs = [torch.from_numpy(img).to(dev) for _ in range(2)]
    Rs = [torch.empty_like(xs[0]) for _ in range(2)]
    Ms = [torch.empty((H, W), dtype=torch.uint8, device=dev) for _ in range(2)]
    g = torch.from_numpy(synth.corner_window()).to(dev)
    st = torch.cuda.current_stream().cuda_stream
    B.check(B.icl_tune(B.ICL_OP_HARRIS, B.ICL_F32, 2, W, H, st))
    B.check(B.icl_tune(B.ICL_OP_NMS, B.ICL_F32, 1, W, H, st))

    def corner(s):
        T.harris(xs[s % 2], g, 0.04, out=Rs[s % 2])
        T.nms(Rs[s % 2], 1e-3, out=Ms[s % 2])

    dt = _time(torch, corner, steps)
    gpx = H * W / dt / 1e9
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    ev[0].record()
    T.harris(xs[0], g, 0.04, out=Rs[0])
    ev[1].record()
    T.nms(Rs[0], 1e-3, out=Ms[0])
    ev[2].record()
    torch.cuda.synchronize()
    res["corner_8192"] = {"ms": round(dt * 1e3, 3), "gpx_s": round(gpx, 1), "bytes_per_px": 13,
                          "phase_ms": {"harris": round(ev[0].elapsed_time(ev[1]), 3),
                                       "nms": round(ev[1].elapsed_time(ev[2]), 3)},
                          "hbm_frac": round(gpx * 13 / HBM_PEAK_GBS, 3),
                          "harris_variant": B.icl_variant_name(B.ICL_OP_HARRIS, B.icl_selected_variant(
                              B.ICL_OP_HARRIS, B.ICL_F32, 2, W, H)[1]),
                          "corners": int(Ms[0].sum().item())}
    # every Harris variant on the same input (forced), for the record
    per_variant = {}
    ws_h = torch.empty(B.icl_workspace_size(B.ICL_OP_HARRIS, W, H)[1] // 4 + 1, dtype=torch.float32, device=dev)
    for v in range(B.icl_variant_count(B.ICL_OP_HARRIS)):
        B.check(B.icl_force_variant(B.ICL_OP_HARRIS, v))
        try:
            dv = _time(torch, lambda s: T.harris(xs[s % 2], g, 0.04, out=Rs[s % 2], workspace=ws_h), 5)
            per_variant[B.icl_variant_name(B.ICL_OP_HARRIS, v)] = round(dv * 1e3, 3)
        except Exception as e:   # a variant that does not take this input
            per_variant[B.icl_variant_name(B.ICL_OP_HARRIS, v)] = repr(e)[:60]
        finally:
            B.icl_force_variant(B.ICL_OP_HARRIS, -1)
    res["corner_8192"]["harris_variants_ms"] = per_variant
    T.harris(xs[0], g, 0.04, out=Rs[0])
    T.harris(xs[1], g, 0.04, out=Rs[1])
    nms_variants = {}
    for v in range(B.icl_variant_count(B.ICL_OP_NMS)):
        B.check(B.icl_force_variant(B.ICL_OP_NMS, v))
        try:
            dv = _time_graph(torch, lambda s: T.nms(Rs[s % 2], 1e-3, out=Ms[s % 2]), 2 * steps)
            nms_variants[B.icl_variant_name(B.ICL_OP_NMS, v)] = round(dv * 1e6, 1)
        except Exception as e:   # a variant that does not take this input
            nms_variants[B.icl_variant_name(B.ICL_OP_NMS, v)] = repr(e)[:60]
        finally:
            B.icl_force_variant(B.ICL_OP_NMS, -1)
    res["corner_8192"]["nms_variant"] = B.icl_variant_name(B.ICL_OP_NMS, B.icl_selected_variant(
        B.ICL_OP_NMS, B.ICL_F32, 1, W, H)[1])
    res["corner_8192"]["nms_variants_us"] = nms_variants
    # the same pipeline fused into one pass (icl_corners): 5 algorithmic B/px, response in registers
    B.check(B.icl_tune(B.ICL_OP_CORNERS, B.ICL_F32, 2, W, H, st))

    def fused(s):
        T.corners(xs[s % 2], g, 0.04, 1e-3, out=Ms[s % 2])

    fused_variants = {}
    for v in range(B.icl_variant_count(B.ICL_OP_CORNERS)):
        B.check(B.icl_force_variant(B.ICL_OP_CORNERS, v))
        try:
            if v == 0:   # the two-kernel variant needs the response buffer
                fn = lambda s: T.corners(xs[s % 2], g, 0.04, 1e-3, out=Ms[s % 2], resp=Rs[s % 2])   # noqa: E731
            else:
                fn = fused
            fused_variants[B.icl_variant_name(B.ICL_OP_CORNERS, v)] = round(_time_graph(torch, fn, steps) * 1e6, 1)
        finally:
            B.icl_force_variant(B.ICL_OP_CORNERS, -1)
    dtf = _time_graph(torch, fused, 2 * steps, reps=10)   # the tuned choice, after every variant has run
    gpx_f = H * W / dtf / 1e9
    dt2 = _time_graph(torch, corner, 2 * steps, reps=10)
    res["corners_fused_8192"] = {
        "timing": "HIP graph replay of back-to-back calls", "us": round(dtf * 1e6, 2), "gpx_s": round(gpx_f, 1),
        "bytes_per_px": 5, "hbm_frac": round(gpx_f * 5 / HBM_PEAK_GBS, 3),
        "two_calls_us": round(dt2 * 1e6, 2), "speedup_vs_two_calls": round(dt2 / dtf, 2),
        "variant": B.icl_variant_name(B.ICL_OP_CORNERS, B.icl_selected_variant(B.ICL_OP_CORNERS, B.ICL_F32, 2, W,
                                                                               H)[1]),
        "variants_us": fused_variants,
        "same_mask_as_two_calls_inside_strips": None}
    Mf = T.corners(xs[0], g, 0.04, 1e-3)
    T.harris(xs[0], g, 0.04, out=Rs[0])
    Mt = T.nms(Rs[0], 1e-3)
    xr = 4 + ((W - 8) // 248) * 248
    res["corners_fused_8192"]["same_mask_as_two_calls_inside_strips"] = bool(
        torch.equal(Mf[:, 8:xr - 8], Mt[:, 8:xr - 8]))
    del xs, Rs, Ms, ws_h, Mf, Mt
    torch.cuda.empty_cache()
    return res


def extra_batch(torch, B, T, synth, steps):
    dev = torch.device("cuda:0")
    res = {}
    # uneven batch: 256 images, one persistent launch replayed from a HIP graph (4 B/px half storage)
    items = synth.batch_uneven()

    def pitched(h, w, tdt):
        """h x w view with rows padded to a multiple of 256 bytes (the workload's layout)."""
        pw = -(-w * 2 // 256) * 128
        return torch.empty((h, pw), dtype=tdt, device=dev)[:, :w]

    for name, tdt in (("f16", torch.float16), ("bf16", torch.bfloat16)):
        ims, outs = [], []
        for it in items:
            x = pitched(it.height, it.width, tdt)
            x.copy_(torch.from_numpy(it.image).to(dev).to(tdt))
            ims.append(x)
            outs.append(pitched(it.height, it.width, tdt))
        taps = [torch.from_numpy(it.taps).to(dev) for it in items]
        plan = T.BatchPlan(ims, outs, taps)
        per_variant = {}
        for v in range(B.icl_variant_count(B.ICL_OP_CONV_SEP_BATCHED)):   # plain launches, forced
            B.check(B.icl_force_variant(B.ICL_OP_CONV_SEP_BATCHED, v))
            try:
                per_variant[B.icl_variant_name(B.ICL_OP_CONV_SEP_BATCHED, v)] = round(
                    _time(torch, lambda s: plan.launch(), steps) * 1e3, 3)
            finally:
                B.icl_force_variant(B.ICL_OP_CONV_SEP_BATCHED, -1)
        t0 = time.perf_counter()
        plan.tune()    # per-device choice of the walk for this plan
        tune_s = time.perf_counter() - t0
        plan.graph()   # the tuned walk, captured once and replayed
        dt = _time(torch, lambda s: plan.replay(), steps)
        gpx = plan.pixels / dt / 1e9
        res[f"batch256_{name}"] = {"ms": round(dt * 1e3, 3), "gpx_s": round(gpx, 1), "pixels": plan.pixels,
                                   "tiles": plan.tiles, "bytes_per_px": 4,
                                   "hbm_frac": round(gpx * 4 / HBM_PEAK_GBS, 3),
                                   "variant": B.icl_variant_name(B.ICL_OP_CONV_SEP_BATCHED, plan.variant()),
                                   "tune_seconds": round(tune_s, 2),
                                   "variants_ms": per_variant}
        plan.close()
        del ims, outs
    torch.cuda.empty_cache()
    return res


def extra_bank(torch, B, T, synth, steps):
    dev = torch.device("cuda:0")
    res = {}
    # differentiable filter bank training step: forward fused with the loss (gy = 2 (y - t), y never
    # stored), then the input and filter adjoints; the unfused chain (forward, loss, adjoints) beside it
    N, F, Hb, Wb, r = 32, 16, 1024, 1024, 4
    x, w, t = synth.bank_inputs()
    xt, wt, tt = torch.from_numpy(x).to(dev), torch.from_numpy(w).to(dev), torch.from_numpy(t).to(dev)
    del t
    y = torch.empty((N, F, Hb, Wb), dtype=torch.float32, device=dev)
    gy = torch.empty_like(y)
    gx = torch.empty_like(xt)
    gw = torch.empty_like(wt)
    _, nb = B.icl_workspace_size(B.ICL_OP_BANK_BWD_FILTER, Wb, Hb, N, F, r)
    wsw = torch.empty(nb // 4 + 1, dtype=torch.float32, device=dev)
    _, nb = B.icl_workspace_size(B.ICL_OP_SSE_LOSS, 1, 1)
    wsl = torch.empty(nb // 4 + 1, dtype=torch.float32, device=dev)
    _, nb = B.icl_workspace_size(B.ICL_OP_BANK_FWD_SSE, Wb, Hb, N, F, r)
    wsf = torch.empty(nb // 4 + 1, dtype=torch.float32, device=dev)
    # per-device tuning of every kernel of the step (outside the timed region)
    st = torch.cuda.current_stream().cuda_stream
    ops = {"fwd_loss": B.ICL_OP_BANK_FWD_SSE, "bwd_input": B.ICL_OP_BANK_BWD_INPUT,
           "bwd_filter": B.ICL_OP_BANK_BWD_FILTER, "fwd": B.ICL_OP_BANK_FWD}
    t0 = time.perf_counter()
    for op in ops.values():
        B.check(B.icl_tune_problem(op, B.ICL_F32, r, Wb, Hb, n=N, f=F, stream=st), "tune bank")
    torch.cuda.synchronize()
    tune_s = time.perf_counter() - t0
    sel = {k: B.icl_selected_variant_problem(op, B.ICL_F32, r, Wb, Hb, n=N, f=F)[1] for k, op in ops.items()}

    def fused(s, ev=None):
        if ev: ev[0].record()
        T.bank_fwd_sse(xt, wt, tt, workspace=wsf, gy=gy)
        if ev: ev[1].record()
        T.bank_bwd_input(gy, wt, out=gx)
        if ev: ev[2].record()
        T.bank_bwd_filter(gy, xt, r, out=gw, workspace=wsw)
        if ev: ev[3].record()

    def unfused(s, ev=None):
        if ev: ev[0].record()
        T.bank_fwd(xt, wt, out=y)
        if ev: ev[1].record()
        T.sse_loss(y, tt, workspace=wsl)
        if ev: ev[2].record()
        T.bank_bwd_input(gy, wt, out=gx)
        if ev: ev[3].record()
        T.bank_bwd_filter(gy, xt, r, out=gw, workspace=wsw)
        if ev: ev[4].record()

    def phases(fn, names):
        evs = []
        for s in range(3):
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(len(names) + 1)]
            fn(s, ev)
            evs.append(ev)
        torch.cuda.synchronize()
        return {nm: round(float(np.mean([e[i].elapsed_time(e[i + 1]) for e in evs])), 3) for i, nm in enumerate(names)}

    dt = _time(torch, fused, steps)
    ph = phases(fused, ("fwd_loss", "bwd_input", "bwd_filter"))
    dt_u = _time(torch, unfused, max(2, steps // 2))
    ph_u = phases(unfused, ("fwd", "loss", "bwd_input", "bwd_filter"))
    per_variant = {}
    for v in range(1, B.icl_variant_count(B.ICL_OP_BANK_FWD_SSE)):   # the fused kernels, plain aside
        B.check(B.icl_force_variant(B.ICL_OP_BANK_FWD_SSE, v))
        try:
            fv = _time(torch, lambda s: T.bank_fwd_sse(xt, wt, tt, workspace=wsf, gy=gy), 3)
        finally:
            B.icl_force_variant(B.ICL_OP_BANK_FWD_SSE, -1)
        per_variant[B.icl_variant_name(B.ICL_OP_BANK_FWD_SSE, v)] = round(fv * 1e3, 3)
    per_variant_w = {}
    for v in range(B.icl_variant_count(B.ICL_OP_BANK_BWD_FILTER)):
        B.check(B.icl_force_variant(B.ICL_OP_BANK_BWD_FILTER, v))
        try:
            fv = _time(torch, lambda s: T.bank_bwd_filter(gy, xt, r, out=gw, workspace=wsw), 3)
        finally:
            B.icl_force_variant(B.ICL_OP_BANK_BWD_FILTER, -1)
        per_variant_w[B.icl_variant_name(B.ICL_OP_BANK_BWD_FILTER, v)] = round(fv * 1e3, 3)
    # each phase against the peak of the unit its kernel runs on: float32 matrix instructions
    # (157.3 TFLOP/s) or float32 vector FMA (78.6, packed FMA disabled)
    flops_phase = 2 * 81 * N * F * Hb * Wb
    phases_out, roof_time = {}, 0.0
    for k in ("fwd_loss", "bwd_input", "bwd_filter"):
        ar = B.icl_variant_arith(ops[k], sel[k])
        peak = FP32_PACKED_PEAK_TFLOPS if ar == "fp32_mfma" else FP32_FMA_PEAK_TFLOPS
        tf = flops_phase / (ph[k] * 1e-3) / 1e12
        roof_time += flops_phase / (peak * 1e12)
        phases_out[k] = {"ms": ph[k], "variant": B.icl_variant_name(ops[k], sel[k]), "arith": ar,
                         "tflops": round(tf, 2), "peak_tflops": peak, "frac": round(tf / peak, 3)}
    flops = 3 * flops_phase
    res["filter_bank_fwd_bwd"] = {"ms": round(dt * 1e3, 3), "gpx_s": round(N * Hb * Wb / dt / 1e9, 2),
                                  "output_gpx_s": round(N * F * Hb * Wb / dt / 1e9, 1),
                                  "tflops": round(flops / dt / 1e12, 2),
                                  "roof_frac": round(roof_time / dt, 3),
                                  "roof_note": "time the three phases would take at the peak of the unit each "
                                               "kernel uses, over the measured step",
                                  "phases": phases_out, "tune_seconds": round(tune_s, 2),
                                  "fwd_loss_variants_ms": per_variant,
                                  "bwd_filter_variants_ms": per_variant_w,
                                  "unfused": {"ms": round(dt_u * 1e3, 3), "phase_ms": ph_u}}
    return res


def cpu_cores():
    """(threads to use, nproc, why): every core this process may run on.  A GPU job's share of the
    host is fixed by OMP_NUM_THREADS where the launcher sets it (the CPU share of one GPU)."""
    nproc = os.cpu_count() or 1
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = nproc
    omp = os.environ.get("OMP_NUM_THREADS", "")
    if omp.isdigit() and int(omp) > 0:
        return min(int(omp), avail), nproc, f"OMP_NUM_THREADS={omp} (this job's CPU share), {avail} cores in affinity"
    return avail, nproc, f"{avail} cores in affinity"


def cpu_baseline(synth, radii, side, min_seconds=10.0):
    """The FP64 oracle, as it stands, on the same step: all ten calls over the full image, rows
    split over every host thread this job may use, repeated until at least `min_seconds` (and 3
    steps) have run; then a single-thread run (median of 3) on a 256-row strip of every call."""
    from oracle import oracle
    rows = int(os.environ.get("ICL_CPU_SAMPLE_ROWS", str(side)))
    threads, nproc, why = cpu_cores()
    img = synth.sweep_image(side)[:rows].astype(np.float64)
    taps = [(synth.sweep_taps_sep(r), synth.sweep_taps_2d(r)) for r in radii]

    def step(im, nt):
        t0 = time.perf_counter()
        for (h, v), w in taps:
            oracle.conv_sep(im, h, v, nthreads=nt)
            oracle.conv2d(im, w, nthreads=nt)
        return time.perf_counter() - t0

    times = []
    while len(times) < 3 or sum(times) < min_seconds:
        times.append(step(img, threads))
        if len(times) % 5 == 1:
            print(f"[bench] cpu oracle step {len(times)}: {times[-1]:.2f} s", file=sys.stderr, flush=True)
    total = sum(times)
    px = rows * side * len(radii) * 2
    strip = min(256, rows)
    t1 = sorted(step(img[:strip], 1) for _ in range(3))[1]
    print(f"[bench] cpu oracle single thread, {strip}-row strip: {t1:.2f} s", file=sys.stderr, flush=True)
    what = "the full step" if rows == side else f"rows 0..{rows - 1} of every call (a {rows}x{side} strip)"
    return {"value": round(len(times) * px / total / 1e9, 5), "unit": "Gpixel/s", "cores": threads,
            "nproc": nproc, "cores_note": why, "kind": "oracle",
            "sample": f"{what}: {2 * len(radii)} calls on the {side}x{side} sweep image, {len(times)} steps "
                      f"in {total:.1f} s ({sorted(times)[len(times) // 2]:.2f} s median per step)",
            "single_thread": {"value": round(strip * side * len(radii) * 2 / t1 / 1e9, 6), "unit": "Gpixel/s",
                              "sample": f"rows 0..{strip - 1} of every call, median of 3 runs ({t1:.2f} s)"}}


if __name__ == "__main__":
    main()
