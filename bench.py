"""Benchmark of the differentiable bilinear point rasterizer on one MI355X.

Headline: forward + backward (through torch.autograd.Function) of 8M
synthetic points at 1920x1080 with 16 float32 features, in fragments per
second (fragments = splats the forward emits), with the HBM traffic of the
step from rocprofv3 counters.  Also reported on the same JSON line:

* per-stage timings measured with HIP events in a second set of steps
  (the markers cost time, so they stay out of the timed steps);
* the roofline figure of the dominant kernel under two byte models (the
  per-splat model, and the compulsory bytes of this design) and its counter
  traffic;
* the CPU oracle's rate on the same workload (forward and backward timed
  separately, median of 3) and the error of the GPU outputs against it;
* 1M points at 1280x720 (F=8) through the plain one-view entry points;
* 16 views of uneven size as one HIP-graph replay in bfloat16 and float32,
  against 16 sequential plain float32 calls, with the bfloat16 error of every
  output against the FP64 oracle;
* 32M points at 1080p (bfloat16, forward only): 8 poses one after another,
  and the 8 poses as one batched call over aliased views;
* the steps around the rasterizer (octree sampling, the appearance step, the
  per-point blend weight, multisampled inference, the probability update).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-batched] [--no-cpu]
                       [--no-next] [--no-extra] [--counter-run]

Profile summaries (the text files under profiles/, from rocprofv3 output):
  python bench.py --summarize-stats KERNEL_STATS_CSV TITLE COMMAND
  python bench.py --summarize-counters FETCH_COUNTER_CSV WRITE_COUNTER_CSV
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E peak
COUNTER_STEPS = 3       # steps of a --counter-run (no warm-up, nothing else but a calibration copy)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# kernel name (without template arguments) -> bench stage
KERNEL_STAGE = {
    "k_project": "project", "k_emit_count": "emit", "k_emit_write": "emit", "k_tile_emit_write": "emit",
    "k_scan_chunks": "emit", "k_radix_upsweep": "sort_upsweep", "k_scan_rows": "sort_scan",
    "k_radix_downsweep": "sort_downsweep", "k_ranges": "ranges", "k_blend_fwd": "blend_fwd",
    "k_tile_fwd": "blend_fwd", "k_blend_bwd": "blend_bwd", "k_tile_bwd": "blend_bwd",
    "k_point_reduce": "point_reduce", "k_point_reduce_q": "point_reduce", "k_fill_u32": "fill",
    "k_upload_views": "views",
    "k_order_hist": "ranges", "k_order_scan": "ranges", "k_order_place": "ranges",
}
# copies the runtime makes outside the timed steps (input upload, the counter calibration)
RUNTIME_COPY = "__amd_rocclr_copyBuffer"


def summarize_stats(path, title, cmd):
    """Markdown table of a rocprofv3 --stats kernel summary (kernel_stats.csv)."""
    import csv
    rows = list(csv.DictReader(open(path)))
    out = [f"# {title}", "", "Command (run from /tmp with TMPDIR=/tmp):", "", "```", cmd, "```", "",
           "Rasterizer kernels only.  The runtime's `" + RUNTIME_COPY + "` dispatches (the host-to-device "
           "upload of the inputs before the timed steps) are left out.", "",
           "| kernel | calls | avg us | total us | % of kernel time |", "|---|---:|---:|---:|---:|"]
    rows = [r for r in rows if not r["Name"].startswith(RUNTIME_COPY)]
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
        name = r["Name"].split("(")[0].replace("void ", "")
        out.append(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                   f"{float(r['TotalDurationNs']) / 1e3:.1f} | {100.0 * float(r['TotalDurationNs']) / tot:.1f} |")
    return "\n".join(out) + "\n"


COUNTER_CMDS = [
    "rocprofv3 --pmc FETCH_SIZE -d /root/repo/gpurun_out/pmc_fetch -o c3 --output-format csv -- "
    "python3 /root/repo/bench.py --counter-run",
    "rocprofv3 --pmc WRITE_SIZE -d /root/repo/gpurun_out/pmc_write -o c3 --output-format csv -- "
    "python3 /root/repo/bench.py --counter-run",
]
STATS_CMD = ("rocprofv3 --kernel-trace --stats -d /root/repo/gpurun_out/prof3 -o c3 --output-format csv -- "
             "python3 /root/repo/bench.py --steps 3 --warmup 1 --no-batched --no-cpu --no-next --no-extra")


def summarize_counters(fetch_csv, write_csv):
    """HBM bytes per launch of every rasterizer kernel from two rocprofv3
    counter runs (FETCH_SIZE, WRITE_SIZE; KiB per dispatch) of
    ``bench.py --counter-run`` (COUNTER_STEPS identical steps and a 1 GiB
    device copy), each scaled by what the counter reads for that copy.
    Returns (markdown summary, json record keyed by bench stage)."""
    import collections
    import csv

    def load(p):
        d = collections.defaultdict(list)
        for r in csv.DictReader(open(p)):
            d[r["Kernel_Name"].split("(")[0].replace("void ", "")].append(float(r["Counter_Value"]))
        return d

    fk, wk = load(fetch_csv), load(write_csv)
    cal_f, cal_w = max(fk[RUNTIME_COPY]), max(wk[RUNTIME_COPY])
    gib_kib = 1024.0 * 1024.0
    fs, ws = gib_kib / cal_f, gib_kib / cal_w
    rec = {"workload": "8M points, 1920x1080, F=16 float32, forward+backward", "fetch_scale": fs,
           "write_scale": ws, "calibration": "1 GiB device-to-device copy in the same runs: "
           f"FETCH_SIZE reads {cal_f:.0f} KB, WRITE_SIZE {cal_w:.0f} KB",
           "commands": COUNTER_CMDS, "steps": COUNTER_STEPS, "source_sha256": source_digest(),
           "per_launch_bytes": {}, "per_step_bytes": {}}
    lines = ["# HBM traffic per kernel launch: 8M points, 1920x1080, F=16 float32, forward+backward", "",
             "Counters from two runs (run from /tmp with TMPDIR=/tmp) of "
             f"{COUNTER_STEPS} identical steps, summarized with "
             "`python bench.py --summarize-counters <fetch csv> <write csv>`:", "", "```"] + COUNTER_CMDS + [
             "```", "", f"Calibration: a 1 GiB device copy in the same runs reads FETCH_SIZE = {cal_f:.0f} KB "
             f"and WRITE_SIZE = {cal_w:.0f} KB, so fetch counts are scaled by {fs:.3f} and write counts by "
             f"{ws:.3f}.", "", "| kernel | launches | fetch GB/launch | write GB/launch | total GB/launch |",
             "|---|---:|---:|---:|---:|"]
    per_stage = collections.defaultdict(float)
    per_stage_launch = collections.defaultdict(float)
    step_total = 0.0
    for k in sorted(fk, key=lambda k: -sum(fk[k]) / len(fk[k])):
        short = k.split("<")[0].replace("inpc::", "")
        if short not in KERNEL_STAGE:
            if k.startswith("inpc::"):
                raise ValueError(f"kernel {k} has no stage in KERNEL_STAGE")
            continue
        f = sum(fk[k]) / len(fk[k]) * fs * 1024
        w = sum(wk[k]) / len(wk[k]) * ws * 1024 if k in wk else 0.0
        lines.append(f"| `{k}` | {len(fk[k])} | {f / 1e9:.3f} | {w / 1e9:.3f} | {(f + w) / 1e9:.3f} |")
        tot = (sum(fk[k]) * fs + (sum(wk[k]) * ws if k in wk else 0.0)) * 1024
        per_stage[KERNEL_STAGE[short]] += tot / COUNTER_STEPS
        per_stage_launch[KERNEL_STAGE[short]] += f + w
        step_total += tot / COUNTER_STEPS
    # per launch: stages whose kernels run once per step (the sorts run several passes of different widths)
    rec["per_launch_bytes"] = {k: v for k, v in per_stage_launch.items()
                               if k in ("project", "blend_fwd", "blend_bwd", "point_reduce")}
    rec["per_step_bytes"] = dict(per_stage)
    rec["step_bytes"] = step_total
    lines += ["", f"Whole step (all {len(per_stage)} stages, every dispatch of the {COUNTER_STEPS} steps / "
              f"{COUNTER_STEPS}): {step_total / 1e9:.3f} GB per step.", "",
              "| stage | GB per step |", "|---|---:|"]
    for k, v in sorted(per_stage.items(), key=lambda kv: -kv[1]):
        lines.append(f"| {k} | {v / 1e9:.3f} |")
    return "\n".join(lines) + "\n", rec


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-batched", action="store_true", help="skip the 16-view batched workload")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle timing and the error reports")
    ap.add_argument("--no-next", action="store_true",
                    help="skip the timings of sampling, appearance, blend weight and multisampling")
    ap.add_argument("--no-extra", action="store_true", help="skip the 1M-point and 32M-point workloads")
    ap.add_argument("--tuning", type=int, default=-1)
    ap.add_argument("--counter-run", action="store_true",
                    help=f"run exactly {COUNTER_STEPS} headline steps and a 1 GiB device copy "
                         "(for the counter runs), nothing else")
    ap.add_argument("--summarize-stats", nargs=3, metavar=("CSV", "TITLE", "COMMAND"),
                    help="print the markdown summary of a rocprofv3 kernel_stats.csv and exit")
    ap.add_argument("--summarize-counters", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write profiles/counters_config3.md and profiles/traffic_config3.json and exit")
    return ap.parse_args()


def compulsory_bytes(N, N_vis, M, M_b, P, F, feat_bytes, zpasses, ppasses, payload_stride, E=None, n_tiles=None):
    """Compulsory bytes per step of each stage of this design (each input read
    once, each output written once).  Per-pixel lists store and sort the M
    splats; tile lists store and sort E tile entries with one range per tile
    and read each visible point's payload row (16-byte record + features,
    written by the projection).  The depth passes carry each point's anchor
    word beside its key and value, and the emission reads it in sorted order."""
    items = M if E is None else E        # list items emitted, sorted and read by the blends
    blended = M_b if E is None else E    # list items a blend reads
    R = P if E is None else n_tiles      # ranges
    row = 16 + F * feat_bytes
    payload = payload_stride * N_vis if E is not None else 0
    return {
        "project": 12 * N + 4 * N + 16 * N + 12 * N + payload,
        "sort_upsweep": zpasses * 4 * N + ppasses * 4 * items,
        "sort_downsweep": zpasses * 24 * N + ppasses * 16 * items,
        "emit": 4 * N + 8 * N + 8 * items,
        "ranges": 8 * R + 4 * items,
        "blend_fwd": 8 * R + 4 * blended + row * N_vis + (4 * F + 4 + 16) * P + 4 * M_b,
        "clear_records": 32 * N,
        "blend_bwd": 8 * R + 16 * P + 4 * blended + 4 * M_b + row * N_vis + 4 * F * P + 8 * M_b,
        "point_reduce": 16 * N + 32 * N + 4 * F * min(P, 4 * N_vis) + (4 * F + 4) * N,
    }


def per_splat_bytes(N, M, M_b, P, F, feat_bytes, pixel_bits):
    """Bytes per step of the algorithmic per-splat model: every splat is
    emitted as a (64-bit key, id) pair, sorted by one LSD radix sort of the
    full key with 8-bit digits, read once per blend with its point record
    and feature row, and reduced per point from its four corners' gradient
    rows.  Keyed by the steps of the path."""
    passes = -(-(pixel_bits + 32) // 8)
    fs = F * feat_bytes
    return {
        "project_emit": 12 * N + 8 * N + 12 * M,
        "sort": passes * 24 * M,
        "ranges": 8 * M + 4 * P,
        "blend_fwd": 4 * P + 4 * M_b + (12 + fs) * M_b + (4 * F + 8) * P,
        "blend_bwd": 12 * P + 4 * M_b + (12 + fs) * M_b + 4 * F * P + 8 * M_b + 4 * M,
        "point_reduce": 16 * N + 32 * N + 4 * 4 * F * N + 8 * N + (4 * F + 4) * N,
    }


def sort_passes(tuning_name: str, which: str, bits: int) -> int:
    """Radix passes of a sort of ``bits``-bit keys under a tuning entry (the
    library's rule for "auto" digits: fewest passes of at most 9 bits)."""
    import re
    m = re.search(which + r" sort (\d+)-bit", tuning_name)
    if m:
        d = int(m.group(1))
    else:
        p = (bits + 8) // 9
        d = max(7, -(-bits // p))
    return -(-bits // d)


def source_digest() -> str:
    """sha256 over the HIP sources, to tell whether stored counters are stale."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for p in sorted(glob.glob(os.path.join(ROOT, "paper_2403_16862_amd", "csrc", "*"))):
        h.update(open(p, "rb").read())
    return h.hexdigest()


def traffic_record():
    """The committed counter summary, or None if it is missing or the kernels
    changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "traffic_config3.json")
    if not os.path.exists(path):
        return None
    tr = json.load(open(path))
    return tr if tr.get("source_sha256") == source_digest() else None


def median(xs):
    s = sorted(xs)
    n = len(s)
    return s[n // 2] if n % 2 else 0.5 * (s[n // 2 - 1] + s[n // 2])


def event_ms(torch, fn, reps=20, warm=3):
    """Median time of fn() over reps calls, each bracketed by HIP events on
    the current stream (after warm untimed calls)."""
    for _ in range(warm):
        fn()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    torch.cuda.synchronize()
    for a, b in ev:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    return median([a.elapsed_time(b) for a, b in ev])


def grad_err(np, gpu, ref):
    """|gpu - ref| / max(|ref|, 1e-3 rms(ref)) per element."""
    ref = ref.astype(np.float64)
    rms = float(np.sqrt(np.mean(ref ** 2))) if ref.size else 0.0
    return np.abs(gpu.astype(np.float64) - ref) / np.maximum(np.abs(ref), max(1e-3 * rms, 1e-30))


def rel_err(np, gpu, ref, floor=1e-12):
    return np.abs(gpu.astype(np.float64) - ref) / np.maximum(np.abs(ref), floor)


def stat(np, e):
    e = np.asarray(e, np.float64).reshape(-1)
    if e.size == 0:
        return {"max": 0.0, "p99": 0.0}
    return {"max": float(e.max()), "p99": float(np.quantile(e, 0.99))}


def main():
    args = parse()
    if args.summarize_stats:
        print(summarize_stats(*args.summarize_stats), end="")
        return
    if args.summarize_counters:
        md, rec = summarize_counters(*args.summarize_counters)
        open(os.path.join(ROOT, "profiles", "counters_config3.md"), "w").write(md)
        json.dump(rec, open(os.path.join(ROOT, "profiles", "traffic_config3.json"), "w"), indent=1)
        print(md, end="")
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this rasterizer runs on one GPU; multi-GPU runs are not supported "
              "(use --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2403_16862_amd as pr
    import workloads

    if args.counter_run:
        args.steps, args.warmup = COUNTER_STEPS, 0

    dev = "cuda:0"
    torch.cuda.set_device(0)
    t0 = time.time()
    s = workloads.config3()
    log(f"generated config 3 in {time.time() - t0:.1f}s: N={s.n} {s.cam.width}x{s.cam.height} F={s.F}")
    x = torch.from_numpy(s.xyz).to(dev)
    f = torch.from_numpy(s.feat).to(dev).requires_grad_(True)
    o = torch.from_numpy(s.opa).to(dev).requires_grad_(True)
    g = torch.from_numpy(s.g_img).to(dev)

    def step():
        f.grad = None
        o.grad = None
        img, tf = pr.rasterize(x, f, o, s.cam, 1e-4, "save", args.tuning)
        torch.autograd.backward([img], [g])
        return img, tf

    for i in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log("warmup done")
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for a, b in ev:
        a.record()
        step()
        b.record()
    torch.cuda.synchronize()
    t_end = time.perf_counter()
    ms_per_step = (t_end - t_start) * 1e3 / args.steps
    step_ev = [a.elapsed_time(b) for a, b in ev]
    log(f"timed {args.steps} steps: {ms_per_step:.3f} ms/step (wall), median {median(step_ev):.3f} ms (events)")
    if args.counter_run:
        a_ = torch.empty(256 * 1024 * 1024, dtype=torch.float32, device=dev)
        b_ = torch.empty_like(a_)
        torch.cuda.synchronize()
        b_.copy_(a_)
        torch.cuda.synchronize()
        log("calibration copy: 1 GiB read + 1 GiB written")
        print(json.dumps({"counter_run": True, "steps": args.steps, "ms_per_step": round(ms_per_step, 4)}))
        return
    # Per-stage times from HIP events the library records around its stages, in
    # as many further steps: the markers themselves cost a few microseconds per
    # stage, so they stay out of the timed steps above.
    pr.profile_begin()
    torch.cuda.synchronize()
    t_p0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    ms_profiled = (time.perf_counter() - t_p0) * 1e3 / args.steps
    stages = pr.profile_end()
    log(f"profiled {args.steps} steps: {ms_profiled:.3f} ms/step with stage events")

    # fragment counts of this workload (deterministic; measured outside the timed region)
    _, _, st = pr.rasterize_forward(x, f.detach(), o.detach(), s.cam, 1e-4, "save", args.tuning,
                                    keep_workspace=True)
    keys, ids, nb = pr.debug_fragments(st)
    M = int(keys.shape[0])
    M_b = int(nb.astype(np.int64).sum())
    N_vis = int(np.unique(ids >> 2).size)
    items, layout = pr.state_info(st)
    del keys, ids, st
    P = s.cam.width * s.cam.height
    value = M / (ms_per_step * 1e-3)

    tn = pr.tuning_table()
    tid = args.tuning if args.tuning >= 0 else pr.lib().inpc_tuning_for(
        pr.make_views([s.cam], [0], [s.n]), 1, s.n, s.F, 0)
    zspan = int(np.float32(s.cam.far).view(np.uint32)) - int(np.float32(s.cam.near).view(np.uint32))
    zbits = max(1, zspan.bit_length())
    pbits = max(1, (P - 1).bit_length())
    zpasses = sort_passes(tn[tid], "depth", zbits)
    ps = ((16 + 4 * s.F + 63) // 64) * 64
    if layout:
        ts = 16 if layout == 5 else 8
        n_tiles = ((s.cam.width + ts - 1) // ts) * ((s.cam.height + ts - 1) // ts)
        ppasses = sort_passes(tn[tid], "pixel", max(1, (n_tiles - 1).bit_length()))
        comp = compulsory_bytes(s.n, N_vis, M, M_b, P, s.F, 4, zpasses, ppasses, ps, E=items, n_tiles=n_tiles)
    else:
        ppasses = sort_passes(tn[tid], "pixel", pbits)
        comp = compulsory_bytes(s.n, N_vis, M, M_b, P, s.F, 4, zpasses, ppasses, ps)
    alg = per_splat_bytes(s.n, M, M_b, P, s.F, 4, pbits)
    per_step = {k: (v[0] / args.steps, v[1] / args.steps) for k, v in stages.items() if v[1] > 0}
    leaf = {k: v for k, v in per_step.items() if k in comp}
    dom = max(leaf, key=lambda k: leaf[k][0])
    dom_ms = leaf[dom][0]
    launches = leaf[dom][1]
    tr = traffic_record()
    traffic = None
    if tr is not None and dom in tr.get("per_launch_bytes", {}):
        traffic = int(tr["per_launch_bytes"][dom] * launches)
    alg_dom = alg.get(dom, comp[dom])
    roofline = {
        "bound": "hbm", "kernel": dom, "launches_per_step": launches,
        "achieved": round(alg_dom / (dom_ms * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(alg_dom / (dom_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "traffic": traffic,
        "kernel_ms": round(dom_ms, 4),
        "algorithmic_bytes": int(alg_dom),
        "byte_model": "per-splat model (bytes per launch from the measured M, M_b, P, N)",
        "compulsory_bytes": int(comp[dom]),
        "compulsory_gbs": round(comp[dom] / (dom_ms * 1e-3) / 1e9, 1),
        "compulsory_frac": round(comp[dom] / (dom_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "counter_gbs": None if traffic is None else round(traffic / (dom_ms * 1e-3) / 1e9, 1),
        "counter_frac": None if traffic is None else round(traffic / (dom_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
    }
    # measured HBM rate of the stages that run one kernel per launch
    counter_gbs = {}
    if tr is not None:
        for k in ("project", "blend_fwd", "blend_bwd", "point_reduce"):
            if k in per_step and k in tr.get("per_launch_bytes", {}) and per_step[k][0] > 0:
                b = tr["per_launch_bytes"][k] * per_step[k][1]
                counter_gbs[k] = round(b / (per_step[k][0] * 1e-3) / 1e9, 1)
    hbm = {
        "per_splat_model_bytes": int(sum(alg.values())),
        "per_splat_model_gbs": round(sum(alg.values()) / (ms_per_step * 1e-3) / 1e9, 1),
        "compulsory_bytes": int(sum(comp[k] for k in leaf)),
        "compulsory_gbs": round(sum(comp[k] for k in leaf) / (ms_per_step * 1e-3) / 1e9, 1),
        "counter_bytes": None, "counter_gbs": None, "counter_frac": None,
    }
    if tr is not None and "step_bytes" in tr:
        hbm["counter_bytes"] = int(tr["step_bytes"])
        hbm["counter_gbs"] = round(tr["step_bytes"] / (ms_per_step * 1e-3) / 1e9, 1)
        hbm["counter_frac"] = round(tr["step_bytes"] / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
    result = {
        "metric": "fwd+bwd fragments/sec and HBM GB/s, 8M pts @1920x1080, batched vs plain",
        "value": round(value, 1),
        "unit": "fragments/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "8M clustered points, 1920x1080, F=16 float32, random look-at camera, "
                               "forward+backward through torch.autograd.Function",
                   "points": s.n, "width": s.cam.width, "height": s.cam.height, "features": s.F,
                   "fragments": M, "blended_fragments": M_b, "visible_points": N_vis,
                   "list_layout": "tile entries %dx%d" % ((16, 16) if layout == 5 else (8, 8)) if layout
                   else "per-pixel splat lists", "list_items": items,
                   "t_threshold": 1e-4, "tuning": tn[tid]},
        "step_ms_events": {"median": round(median(step_ev), 4), "min": round(min(step_ev), 4),
                           "max": round(max(step_ev), 4)},
        "fragments_per_s_median": round(M / (median(step_ev) * 1e-3), 1),
        "hbm": hbm,
        "counter_gbs": counter_gbs or None,
        "stages_ms_per_step": {k: round(v[0], 4) for k, v in per_step.items()},
        "ms_per_step_with_stage_events": round(ms_profiled, 4),
        "roofline": roofline,
    }

    if not args.no_cpu:
        result["cpu_baseline"], result["accuracy_f32"] = cpu_leg(pr, torch, np, s, x, f, o, step, log)

    if not args.no_next:
        # cost of the optional per-point blend weight output on the same forward
        bw = torch.empty((s.n,), dtype=torch.float32, device=dev)

        def fwd(with_bw):
            pr.rasterize_forward(x, f.detach(), o.detach(), s.cam, 1e-4, "save", args.tuning,
                                 blend_weight=bw if with_bw else None)
        result["blend_weight"] = {
            "ms_forward_without": round(event_ms(torch, lambda: fwd(False)), 4),
            "ms_forward_with": round(event_ms(torch, lambda: fwd(True)), 4),
        }
    del x, f, o, g
    torch.cuda.empty_cache()

    if not args.no_extra:
        result["plain_1m"] = bench_config2(pr, torch, np, workloads, log)

    if not args.no_batched:
        result["batched"] = bench_batched(pr, torch, np, workloads, log, with_oracle=not args.no_cpu)

    if not args.no_extra:
        result["inference_32m"] = bench_config5(pr, torch, np, workloads, log)

    if not args.no_next:
        result["pipeline"] = bench_pipeline(pr, torch, np, workloads, log)

    print(json.dumps(result), flush=True)


def cpu_leg(pr, torch, np, s, x, f, o, step, log):
    """The oracle on the headline workload: forward (splat lists + blend) and
    backward timed separately, median of 3, on the host's threads and on one
    thread (first eighth of the points); and the error of the GPU outputs of
    one step against it."""
    import oracle
    threads = oracle.num_threads()
    log(f"cpu baseline: oracle forward and backward, median of 3, {threads} threads")
    tf_, tb_ = [], []
    for _ in range(3):
        t0 = time.perf_counter()
        L = oracle.fragments(s.xyz, s.cam)
        fw = oracle.blend_forward(L, s.opa, s.feat, 1e-4)
        t1 = time.perf_counter()
        rb = oracle.blend_backward(L, s.opa, s.feat, fw["n_blended"], s.g_img)
        t2 = time.perf_counter()
        tf_.append(t1 - t0)
        tb_.append(t2 - t1)
    t_f, t_b = median(tf_), median(tb_)
    cpu = {
        "value": round(L.m / (t_f + t_b), 1), "unit": "fragments/s", "cores": threads, "kind": "oracle",
        "sample": f"whole workload (8M points, {L.m} fragments): forward {t_f:.3f} s, backward {t_b:.3f} s, "
                  "each the median of 3 runs",
        "forward_s": round(t_f, 4), "backward_s": round(t_b, 4),
    }
    # GPU outputs of one step against the oracle, the oracle held at the GPU's blend counts
    img, tf = step()
    torch.cuda.synchronize()
    gi = img.detach().reshape(-1, s.F).cpu().numpy()
    gt = tf.detach().reshape(-1).cpu().numpy()
    gf, go = f.grad.cpu().numpy(), o.grad.cpu().numpy()
    _, _, st = pr.rasterize_forward(x, f.detach(), o.detach(), s.cam, 1e-4, "save", keep_workspace=True)
    _, _, nb = pr.debug_fragments(st)
    del st
    n_gpu = nb.astype(np.int32)
    ambiguous = int(np.count_nonzero(n_gpu != fw["n_blended"]))
    if ambiguous:
        fw = oracle.blend_forward(L, s.opa, s.feat, 1e-4, n_override=n_gpu)
        rb = oracle.blend_backward(L, s.opa, s.feat, n_gpu, s.g_img)
    acc = {"reference": "FP64 oracle on the same inputs, at the GPU's blend counts",
           "ambiguous_pixels": ambiguous,
           "image_rel": stat(np, rel_err(np, gi, fw["image"])),
           "t_final_rel": stat(np, rel_err(np, gt, fw["t_final"])),
           "grad_feat": stat(np, grad_err(np, gf, rb["grad_feat"])),
           "grad_opa": stat(np, grad_err(np, go, rb["grad_opa"]))}
    del L, fw, rb
    # one thread, first eighth of the points
    oracle.set_num_threads(1)
    n1 = s.n // 8
    tf_, tb_ = [], []
    for _ in range(3):
        t0 = time.perf_counter()
        L = oracle.fragments(s.xyz[:n1], s.cam)
        fw = oracle.blend_forward(L, s.opa[:n1], s.feat[:n1], 1e-4)
        t1 = time.perf_counter()
        oracle.blend_backward(L, s.opa[:n1], s.feat[:n1], fw["n_blended"], s.g_img)
        t2 = time.perf_counter()
        tf_.append(t1 - t0)
        tb_.append(t2 - t1)
    oracle.set_num_threads(threads)
    t_f1, t_b1 = median(tf_), median(tb_)
    cpu["one_thread"] = {
        "value": round(L.m / (t_f1 + t_b1), 1), "unit": "fragments/s", "cores": 1,
        "sample": f"first {n1} points of the workload ({L.m} fragments): forward {t_f1:.3f} s, "
                  f"backward {t_b1:.3f} s, each the median of 3 runs"}
    log(f"cpu baseline: {json.dumps(cpu)}")
    log(f"accuracy f32: {json.dumps(acc)}")
    return cpu, acc


def bench_config2(pr, torch, np, workloads, log, reps=20):
    """1M points, 1280x720, F=8 float32, forward + backward through the plain
    one-view entry points, with the autotuner's choice (forward + backward)
    and with the default tuning; median of 20 event-timed steps each."""
    t0 = time.time()
    s = workloads.config2()
    log(f"generated config 2 in {time.time() - t0:.1f}s: N={s.n} {s.cam.width}x{s.cam.height} F={s.F}")
    dev = "cuda:0"
    x = torch.from_numpy(s.xyz).to(dev)
    f = torch.from_numpy(s.feat).to(dev)
    o = torch.from_numpy(s.opa).to(dev)
    g = torch.from_numpy(s.g_img).to(dev)

    tid, _ = pr.autotune(x, f, o, pr.make_views([s.cam], [0], [s.n]), g_img=g, repeats=1)

    def fb(t):
        img, tf, st = pr.rasterize_forward(x, f, o, s.cam, 1e-4, "save", t)
        pr.rasterize_backward(x, f, o, st, g)

    ms = event_ms(torch, lambda: fb(tid), reps=reps)
    ms_default = event_ms(torch, lambda: fb(0), reps=reps)
    ms_f = event_ms(torch, lambda: pr.rasterize_forward(x, f, o, s.cam, 1e-4, "save", tid), reps=reps)
    _, _, st = pr.rasterize_forward(x, f, o, s.cam, 1e-4, "save", tid, keep_workspace=True)
    M = pr.fragment_count(st)
    out = {"workload": "1M clustered points (64 clusters), 1280x720, F=8 float32, forward+backward through "
                       "inpc_rasterize_fwd / inpc_rasterize_bwd",
           "points": s.n, "fragments": M, "ms_fwd_bwd": round(ms, 4), "ms_fwd": round(ms_f, 4),
           "fragments_per_s": round(M / (ms * 1e-3), 1), "tuning": tid,
           "ms_fwd_bwd_default_tuning": round(ms_default, 4)}
    log(f"config 2: {json.dumps(out)}")
    return out


def bench_config5(pr, torch, np, workloads, log, reps=5):
    """32M points (clusters + far shell), 1920x1080, F=16 bfloat16, forward
    only (no backward state: RECOMPUTE mode keeps none): 8 poses one after
    another, and the 8 poses as one batched call whose views alias the same
    points, each with the autotuner's choice; median of 5 event-timed runs
    each."""
    t0 = time.time()
    b = workloads.config5()
    n = b.xyz.shape[0]
    log(f"generated config 5 in {time.time() - t0:.1f}s: N={n}, {len(b.cams)} poses")
    dev = "cuda:0"
    x = torch.from_numpy(b.xyz).to(dev)
    fb = torch.from_numpy(b.feat).to(dev).to(torch.bfloat16)
    o = torch.from_numpy(b.opa).to(dev)
    views = pr.make_views(b.cams, b.point_offset, b.point_count)
    # the autotuner's choice for each form (forward only)
    t_seq, _ = pr.autotune(x, fb, o, pr.make_views([b.cams[0]], [0], [n]), repeats=1)
    torch.cuda.empty_cache()
    t_bat, _ = pr.autotune(x, fb, o, views, repeats=1)
    torch.cuda.empty_cache()

    def seq():
        for cam in b.cams:
            pr.rasterize_forward(x, fb, o, cam, 1e-4, "recompute", t_seq)

    def batched():
        pr.rasterize_forward_batched(x, fb, o, views, 1e-4, "recompute", t_bat)

    ms_seq = event_ms(torch, seq, reps=reps, warm=1)
    ms_bat = event_ms(torch, batched, reps=reps, warm=1)
    _, _, st = pr.rasterize_forward_batched(x, fb, o, views, 1e-4, "save", t_bat, keep_workspace=True)
    M = pr.fragment_count(st)
    del st
    torch.cuda.empty_cache()
    out = {"workload": "32M points (95% clusters, 5% shell at radius 50-200), 1920x1080, F=16 bfloat16, "
                       "forward only, 8 poses on a circle, tau=1e-4",
           "points": n, "poses": len(b.cams), "fragments_8_poses": M,
           "ms_8_poses_sequential": round(ms_seq, 4), "ms_8_poses_batched": round(ms_bat, 4),
           "ms_per_pose_sequential": round(ms_seq / len(b.cams), 4),
           "fragments_per_s_sequential": round(M / (ms_seq * 1e-3), 1),
           "fragments_per_s_batched": round(M / (ms_bat * 1e-3), 1),
           "tuning_sequential": t_seq, "tuning_batched": t_bat}
    log(f"config 5: {json.dumps(out)}")
    return out


def bench_pipeline(pr, torch, np, workloads, log):
    """The data-parallel steps around the rasterizer, at the paper's sizes:
    8M viewpoint-specific samples from a 634k-leaf octree (training), the
    appearance step (opacity activation + degree-2 SH, 37 raw floats per
    point -> 4-D feature), rasterization with per-point blend weights, its
    backward through the appearance step, the probability update; and
    inference: 4 clouds of 8M samples without re-sampling, appearance, and
    the multisampled average, 1920x1080."""
    from workloads.octree import synthetic_octree
    dev = "cuda:0"
    t0 = time.time()
    o = synthetic_octree()
    log(f"generated octree in {time.time() - t0:.1f}s: {o.n} leaves")
    tree = pr.OctreeLeaves(torch.from_numpy(o.centre).to(dev), torch.from_numpy(o.level).to(dev),
                           torch.from_numpy(o.prob).to(dev), torch.from_numpy(o.subdiv).to(dev), o.root_size)
    cam = workloads.look_at_camera([0.3, -0.2, -2.0], [0.0, 0.0, 6.0], [0.0, -1.0, 0.0], 1920, 1080)
    n, K = 8_000_000, 4
    gen = torch.Generator(device=dev)
    gen.manual_seed(1234)

    def raw_rows(m):
        # same recipe as workloads.sh_raw, drawn on the device
        r = torch.empty((m, 37), dtype=torch.float32, device=dev)
        r[:, 0].normal_(-0.5, 1.5, generator=gen)
        r[:, 1:5].uniform_(0.0, 2.0, generator=gen)
        r[:, 5:].normal_(0.0, 0.3, generator=gen)
        return r

    out = {"leaves": o.n, "samples": n, "width": cam.width, "height": cam.height}
    # --- training-style step
    xyz, leaf, unres = pr.sample_view(tree, cam, n, seed=(1, 2), max_rounds=64)
    out["ms_sample_view_8M"] = round(event_ms(torch, lambda: pr.sample_view(tree, cam, n, seed=(1, 2)), reps=10), 4)
    out["unresolved"] = int(unres.item())
    raw = raw_rows(n).requires_grad_(True)
    views = pr.make_views([cam], [0], [n])
    out["ms_appearance_fwd_8M"] = round(
        event_ms(torch, lambda: pr.appearance_forward(xyz, raw.detach(), views), reps=10), 4)
    go = torch.randn((n,), device=dev, generator=gen)
    gf = torch.randn((n, 4), device=dev, generator=gen)
    out["ms_appearance_bwd_8M"] = round(
        event_ms(torch, lambda: pr.appearance_backward(xyz, raw.detach(), views, go, gf), reps=10), 4)
    # appearance bytes: fwd reads xyz + raw rows, writes opacity + feature; bwd reads
    # xyz, the logit, both gradients and writes the raw gradient
    ab_f, ab_b = n * (12 + 148 + 4 + 16), n * (12 + 4 + 4 + 16 + 148)
    out["appearance_gbs"] = {"fwd": round(ab_f / out["ms_appearance_fwd_8M"] / 1e6, 1),
                             "bwd": round(ab_b / out["ms_appearance_bwd_8M"] / 1e6, 1)}
    g_img = torch.randn((cam.height * cam.width, 4), device=dev, generator=gen)
    bw = torch.empty((n,), dtype=torch.float32, device=dev)

    def train_step():
        xs, lf, _ = pr.sample_view(tree, cam, n, seed=(1, 2))
        raw.grad = None
        img, tf = pr.render_sh(xs, raw, views, blend_weight=bw, blend_weight_in_backward=True)
        torch.autograd.backward([img], [g_img])
        pr.update_probabilities(tree, lf, bw)
    out["ms_train_step"] = round(event_ms(torch, train_step, reps=5), 4)
    out["ms_prob_update"] = round(event_ms(torch, lambda: pr.update_probabilities(tree, leaf, bw), reps=10), 4)
    # --- inference: 4 x 8M without re-sampling, multisampled average
    xs4 = torch.empty((K * n, 3), dtype=torch.float32, device=dev)
    lf4 = torch.empty((K * n,), dtype=torch.int32, device=dev)

    def sample4():
        for k in range(K):
            xk, lk, _ = pr.sample_view(tree, cam, n, seed=(100 + k, 2), max_rounds=0)
            xs4[k * n:(k + 1) * n] = xk
            lf4[k * n:(k + 1) * n] = lk
    sample4()
    raw4 = raw_rows(K * n)
    views4 = pr.make_views([cam] * K, [k * n for k in range(K)], [n] * K)
    out["ms_sample_4x8M"] = round(event_ms(torch, sample4, reps=3), 4)
    out["ms_appearance_4x8M"] = round(event_ms(torch, lambda: pr.appearance_forward(xs4, raw4, views4), reps=3), 4)
    o4, f4 = pr.appearance_forward(xs4, raw4, views4)
    offs = [k * n for k in range(K)]
    out["ms_multisample_raster_4x8M"] = round(
        event_ms(torch, lambda: pr.multisample(xs4, f4, o4, cam, offs, [n] * K), reps=3), 4)

    def infer():
        sample4()
        a_o, a_f = pr.appearance_forward(xs4, raw4, views4)
        pr.multisample(xs4, a_f, a_o, cam, offs, [n] * K)
    out["ms_inference_4x8M"] = round(event_ms(torch, infer, reps=3), 4)
    log(f"pipeline: {json.dumps(out)}")
    return out


def graph_ms(torch, step, reps=20):
    """Median replay time of a captured BatchedStep (event-timed replays)."""
    return event_ms(torch, step.replay, reps=reps, warm=2)


def bench_batched(pr, torch, np, workloads, log, with_oracle=True):
    """16 views, one graph replay per forward+backward: bfloat16 features and
    float32 features, against 16 sequential plain float32 calls; and the
    bfloat16 error of every output against the FP64 oracle."""
    t0 = time.time()
    b = workloads.config4()
    log(f"generated config 4 in {time.time() - t0:.1f}s: {len(b.cams)} views, {int(sum(b.point_count))} points")
    dev = "cuda:0"
    x = torch.from_numpy(b.xyz).to(dev)
    f32 = torch.from_numpy(b.feat).to(dev)
    fbf = f32.to(torch.bfloat16)
    o = torch.from_numpy(b.opa).to(dev)
    g = torch.cat([torch.from_numpy(gi.reshape(-1, b.F)) for gi in b.g_imgs]).to(dev)
    views = pr.make_views(b.cams, b.point_offset, b.point_count)
    best, _ = pr.autotune(x, fbf, o, views, g_img=g, repeats=2)
    step = pr.BatchedStep(x, fbf, o, views, g, tuning_id=best)
    step.capture()
    t_batched = graph_ms(torch, step)
    best32, _ = pr.autotune(x, f32, o, views, g_img=g, repeats=2)
    step32 = pr.BatchedStep(x, f32, o, views, g, tuning_id=best32)
    step32.capture()
    t_batched32 = graph_ms(torch, step32)
    del step32
    torch.cuda.empty_cache()
    # plain: 16 sequential FP32 single-view forward+backward calls on the same inputs
    plain = []
    offs = np.cumsum([0] + [c.width * c.height for c in b.cams])
    for v, cam in enumerate(b.cams):
        sl = slice(b.point_offset[v], b.point_offset[v] + b.point_count[v])
        plain.append((x[sl].contiguous(), f32[sl].contiguous(), o[sl].contiguous(), cam,
                      g[offs[v]:offs[v + 1]].contiguous()))

    def run_plain():
        for xv, fv, ov, cam, gv in plain:
            img, tf, st = pr.rasterize_forward(xv, fv, ov, cam, 1e-4, "save", -1)
            pr.rasterize_backward(xv, fv, ov, st, gv)

    t_plain = event_ms(torch, run_plain, reps=10, warm=2)
    M = pr.fragment_count(step.state())
    log(f"batched: bf16 {t_batched:.3f} ms (graph, tuning {best}), f32 {t_batched32:.3f} ms (graph, tuning "
        f"{best32}), plain f32 16 calls: {t_plain:.3f} ms")
    out = {"views": len(b.cams), "points": int(sum(b.point_count)), "pixels": int(offs[-1]),
           "fragments": M, "ms_batched_bf16_graph": round(t_batched, 3),
           "ms_batched_f32_graph": round(t_batched32, 3),
           "ms_plain_f32_sequential": round(t_plain, 3),
           "speedup": round(t_plain / t_batched, 3),
           "speedup_from_batching_f32": round(t_plain / t_batched32, 3),
           "speedup_from_bf16_batched": round(t_batched32 / t_batched, 3),
           "fragments_per_s_batched": round(M / (t_batched * 1e-3), 1),
           "fragments_per_s_plain": round(M / (t_plain * 1e-3), 1),
           "tuning_bf16": best, "tuning_f32": best32}
    del plain
    if with_oracle:
        out["accuracy_bf16"] = batched_accuracy(pr, torch, np, b, step, log)
    return out


def batched_accuracy(pr, torch, np, b, step, log):
    """Error of every output of the bfloat16 graph replay against the FP64
    oracle, over all 16 views (the oracle held at the GPU's blend counts):
    image against the oracle on the bfloat16-rounded features (the
    arithmetic) and on the unrounded float32 features (the storage), the
    transmittance, and both gradients against both oracles."""
    import oracle
    step.replay()
    torch.cuda.synchronize()
    _, _, nb = pr.debug_fragments(step.state())
    img, tf = step.image.cpu().numpy(), step.t_final.cpu().numpy()
    gf, go = step.grad_feat.cpu().numpy(), step.grad_opa.cpu().numpy()
    fbits = torch.from_numpy(b.feat).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    g = np.concatenate([gi.reshape(-1, b.F) for gi in b.g_imgs])
    P_v = [c.width * c.height for c in b.cams]
    pix_off = np.concatenate([[0], np.cumsum(P_v)]).astype(np.int64)
    vp_off = np.concatenate([[0], np.cumsum(b.point_count)]).astype(np.int64)
    acc = {k: [] for k in ("image_rounded_rel", "image_unrounded_abs", "t_final_rel", "grad_feat_rounded",
                           "grad_opa_rounded", "grad_feat_unrounded", "grad_opa_unrounded")}
    t0 = time.time()
    for v in range(len(b.cams)):
        sl = slice(b.point_offset[v], b.point_offset[v] + b.point_count[v])
        L = oracle.fragments(b.xyz[sl], b.cams[v])
        lo, hi = int(pix_off[v]), int(pix_off[v + 1])
        n_gpu = nb[lo:hi].astype(np.int32)
        pv = slice(int(vp_off[v]), int(vp_off[v + 1]))
        r = oracle.blend_forward(L, b.opa[sl], fbits[sl], 1e-4, n_override=n_gpu)
        acc["image_rounded_rel"].append(rel_err(np, img[lo:hi], r["image"]))
        acc["t_final_rel"].append(rel_err(np, tf[lo:hi], r["t_final"]))
        u = oracle.blend_forward(L, b.opa[sl], b.feat[sl], 1e-4, n_override=n_gpu)
        acc["image_unrounded_abs"].append(np.abs(img[lo:hi].astype(np.float64) - u["image"]))
        del r, u
        rb = oracle.blend_backward(L, b.opa[sl], fbits[sl], n_gpu, g[lo:hi])
        acc["grad_feat_rounded"].append(grad_err(np, gf[pv], rb["grad_feat"]))
        acc["grad_opa_rounded"].append(grad_err(np, go[pv], rb["grad_opa"]))
        ru = oracle.blend_backward(L, b.opa[sl], b.feat[sl], n_gpu, g[lo:hi])
        acc["grad_feat_unrounded"].append(grad_err(np, gf[pv], ru["grad_feat"]))
        acc["grad_opa_unrounded"].append(grad_err(np, go[pv], ru["grad_opa"]))
        del L, rb, ru
    out = {"reference": "FP64 oracle over all 16 views at the GPU's blend counts; images and "
                        "transmittance relative to max(|ref|, 1e-12) (unrounded image: absolute); "
                        "gradients relative to max(|ref|, 1e-3 rms(ref)) of each view"}
    for k, lst in acc.items():
        out[k] = stat(np, np.concatenate([e.reshape(-1) for e in lst]))
    log(f"accuracy bf16 (oracle {time.time() - t0:.1f}s): {json.dumps(out)}")
    return out


if __name__ == "__main__":
    main()
