"""Benchmark of the differentiable bilinear point rasterizer on one MI355X.

Headline: forward + backward (through torch.autograd.Function) of 8M
synthetic points at 1920x1080 with 16 float32 features, in fragments per
second (fragments = splats the forward emits).  Also reported on the same
JSON line: per-stage timings measured with HIP events inside the timed
steps, the roofline figure of the dominant kernel, the CPU oracle's rate on
the same workload, and the batched bfloat16 path (16 views of uneven size,
one HIP-graph replay) against 16 sequential float32 plain calls, and the
steps around the rasterizer (octree sampling, the appearance step, the
per-point blend weight, multisampled inference, the probability update).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-batched] [--no-cpu] [--no-next]

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


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# kernel name (without template arguments) -> bench stage
KERNEL_STAGE = {
    "k_project": "project", "k_emit_count": "emit", "k_emit_write": "emit", "k_tile_emit_write": "emit",
    "k_scan_chunks": "emit", "k_radix_upsweep": "sort_upsweep", "k_scan_rows": "sort_scan",
    "k_radix_downsweep": "sort_downsweep", "k_ranges": "ranges", "k_blend_fwd": "blend_fwd",
    "k_tile_fwd": "blend_fwd", "k_blend_bwd": "blend_bwd", "k_tile_bwd": "blend_bwd",
    "k_point_reduce": "point_reduce",
}


def summarize_stats(path, title, cmd):
    """Markdown table of a rocprofv3 --stats kernel summary (kernel_stats.csv)."""
    import csv
    rows = list(csv.DictReader(open(path)))
    out = [f"# {title}", "", "Command (run from /tmp with TMPDIR=/tmp):", "", "```", cmd, "```", "",
           "| kernel | calls | avg us | total us | % |", "|---|---:|---:|---:|---:|"]
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
        name = r["Name"].split("(")[0].replace("void ", "")
        out.append(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                   f"{float(r['TotalDurationNs']) / 1e3:.1f} | {float(r['Percentage']):.1f} |")
    return "\n".join(out) + "\n"


COUNTER_CMDS = [
    "rocprofv3 --pmc FETCH_SIZE -d gpurun_out/pmc_fetch -o c3 --output-format csv -- "
    "python3 bench.py --steps 2 --warmup 1 --no-batched --no-cpu --no-next --calib-copy",
    "rocprofv3 --pmc WRITE_SIZE -d gpurun_out/pmc_write -o c3 --output-format csv -- "
    "python3 bench.py --steps 2 --warmup 1 --no-batched --no-cpu --no-next --calib-copy",
]


def summarize_counters(fetch_csv, write_csv):
    """HBM bytes per launch of every rasterizer kernel from two rocprofv3
    counter runs (FETCH_SIZE, WRITE_SIZE; KiB per dispatch), each scaled by
    what the counter reads for the 1 GiB device copy of the same run.
    Returns (markdown summary, json record keyed by bench stage)."""
    import collections
    import csv

    def load(p):
        d = collections.defaultdict(list)
        for r in csv.DictReader(open(p)):
            d[r["Kernel_Name"].split("(")[0].replace("void ", "")].append(float(r["Counter_Value"]))
        return d

    fk, wk = load(fetch_csv), load(write_csv)
    cal_f, cal_w = max(fk["__amd_rocclr_copyBuffer"]), max(wk["__amd_rocclr_copyBuffer"])
    gib_kib = 1024.0 * 1024.0
    fs, ws = gib_kib / cal_f, gib_kib / cal_w
    rec = {"workload": "8M points, 1920x1080, F=16 float32, forward+backward", "fetch_scale": fs,
           "write_scale": ws, "calibration": "1 GiB device-to-device copy in the same runs: "
           f"FETCH_SIZE reads {cal_f:.0f} KB, WRITE_SIZE {cal_w:.0f} KB",
           "commands": COUNTER_CMDS, "source_sha256": source_digest(), "per_launch_bytes": {}}
    lines = ["# HBM traffic per kernel launch: 8M points, 1920x1080, F=16 float32, forward+backward", "",
             "Counters from two runs (run from /tmp with TMPDIR=/tmp), summarized with "
             "`python bench.py --summarize-counters <fetch csv> <write csv>`:", "", "```"] + COUNTER_CMDS + [
             "```", "", f"Calibration: a 1 GiB device copy in the same runs reads FETCH_SIZE = {cal_f:.0f} KB "
             f"and WRITE_SIZE = {cal_w:.0f} KB, so fetch counts are scaled by {fs:.3f} and write counts by "
             f"{ws:.3f}.", "", "| kernel | launches | fetch GB/launch | write GB/launch | total GB/launch |",
             "|---|---:|---:|---:|---:|"]
    per_stage = collections.defaultdict(float)
    for k in sorted(fk, key=lambda k: -sum(fk[k]) / len(fk[k])):
        short = k.split("<")[0].replace("inpc::", "")
        if short not in KERNEL_STAGE:
            continue
        f = sum(fk[k]) / len(fk[k]) * fs * 1024
        w = sum(wk[k]) / len(wk[k]) * ws * 1024 if k in wk else 0.0
        lines.append(f"| `{k}` | {len(fk[k])} | {f / 1e9:.3f} | {w / 1e9:.3f} | {(f + w) / 1e9:.3f} |")
        per_stage[KERNEL_STAGE[short]] += f + w
    # stages whose kernels run once per step (the sorts run several passes of different widths)
    rec["per_launch_bytes"] = {k: v for k, v in per_stage.items() if not k.startswith("sort_")}
    return "\n".join(lines) + "\n", rec


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-next", action="store_true",
                    help="skip the timings of sampling, appearance, blend weight and multisampling")
    ap.add_argument("--tuning", type=int, default=-1)
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration)")
    ap.add_argument("--summarize-stats", nargs=3, metavar=("CSV", "TITLE", "COMMAND"),
                    help="print the markdown summary of a rocprofv3 kernel_stats.csv and exit")
    ap.add_argument("--summarize-counters", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write profiles/counters_config3.md and profiles/traffic_config3.json and exit")
    return ap.parse_args()


def stage_bytes(N, N_vis, M, M_b, P, F, feat_bytes, zpasses, ppasses, E=None, n_tiles=None):
    """Compulsory bytes per step of each stage (each input read once, each
    output written once).  Per-pixel lists store and sort the M splats; tile
    lists store and sort E tile entries with one range per tile."""
    items = M if E is None else E        # list items emitted, sorted and read by the blends
    blended = M_b if E is None else E    # list items a blend reads
    R = P if E is None else n_tiles      # ranges
    return {
        "project": 12 * N + 4 * N + 16 * N + 8 * N,
        "sort_upsweep": zpasses * 4 * N + ppasses * 4 * items,
        "sort_downsweep": zpasses * 16 * N + ppasses * 16 * items,
        "emit": 4 * N + 4 * N + 16 * N_vis + 8 * items,
        "ranges": 8 * R + 4 * items,
        "blend_fwd": 8 * R + 4 * blended + (16 + F * feat_bytes) * N_vis + (4 * F + 4 + 16) * P + 4 * M_b,
        "clear_records": 32 * N,
        "blend_bwd": 8 * R + 16 * P + 4 * blended + 4 * M_b + (16 + F * feat_bytes) * N_vis + 4 * F * P + 8 * M_b,
        "point_reduce": 16 * N + 32 * N + 4 * F * min(P, 4 * N_vis) + (4 * F + 4) * N,
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


def measured_traffic(stage: str, launches: float):
    """HBM bytes per step of ``stage`` from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, calibrated with a 1 GiB copy), or None
    if the summary does not cover that stage or the kernels changed since."""
    path = os.path.join(ROOT, "profiles", "traffic_config3.json")
    if not os.path.exists(path):
        return None
    tr = json.load(open(path))
    if tr.get("source_sha256") != source_digest():
        return None
    b = tr.get("per_launch_bytes", {}).get(stage)
    return None if b is None else int(b * launches)


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

    for i in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log("warmup done")
    pr.profile_begin()
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        step()
    torch.cuda.synchronize()
    t_end = time.perf_counter()
    stages = pr.profile_end()
    ms_per_step = (t_end - t_start) * 1e3 / args.steps
    log(f"timed {args.steps} steps: {ms_per_step:.3f} ms/step")

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
    if layout:
        ts = 16 if layout == 5 else 8
        n_tiles = ((s.cam.width + ts - 1) // ts) * ((s.cam.height + ts - 1) // ts)
        ppasses = sort_passes(tn[tid], "pixel", max(1, (n_tiles - 1).bit_length()))
        model = stage_bytes(s.n, N_vis, M, M_b, P, s.F, 4, zpasses, ppasses, E=items, n_tiles=n_tiles)
    else:
        ppasses = sort_passes(tn[tid], "pixel", pbits)
        model = stage_bytes(s.n, N_vis, M, M_b, P, s.F, 4, zpasses, ppasses)
    per_step = {k: (v[0] / args.steps, v[1] / args.steps) for k, v in stages.items() if v[1] > 0}
    leaf = {k: v for k, v in per_step.items() if k in model}
    dom = max(leaf, key=lambda k: leaf[k][0])
    dom_ms = leaf[dom][0]
    launches = leaf[dom][1]
    achieved = model[dom] / (dom_ms * 1e-3) / 1e9
    total_model = sum(model[k] for k in leaf)
    traffic = measured_traffic(dom, launches)
    # measured HBM rate of the stages that run one kernel per launch
    counter_gbs = {}
    for k in ("project", "blend_fwd", "blend_bwd", "point_reduce"):
        if k in per_step:
            b = measured_traffic(k, per_step[k][1])
            if b is not None and per_step[k][0] > 0:
                counter_gbs[k] = round(b / (per_step[k][0] * 1e-3) / 1e9, 1)
    roofline = {
        "bound": "hbm", "kernel": dom, "launches_per_step": launches,
        "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "algorithmic_bytes_per_step": int(model[dom]),
        "traffic": traffic,
    }
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
        "model_gbs": round(total_model / (ms_per_step * 1e-3) / 1e9, 1),
        "counter_gbs": counter_gbs or None,
        "stages_ms_per_step": {k: round(v[0], 4) for k, v in per_step.items()},
        "roofline": roofline,
    }

    if not args.no_cpu:
        import oracle
        log("cpu baseline: oracle on the full workload (fragments + forward + backward)")
        t0 = time.perf_counter()
        L = oracle.fragments(s.xyz, s.cam)
        fw = oracle.blend_forward(L, s.opa, s.feat, 1e-4)
        oracle.blend_backward(L, s.opa, s.feat, fw["n_blended"], s.g_img)
        dt = time.perf_counter() - t0
        result["cpu_baseline"] = {
            "value": round(L.m / dt, 1), "unit": "fragments/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"whole workload once: {L.m} fragments, fwd+bwd in {dt:.2f} s",
        }
        del L, fw
        # the same on one thread, on the first eighth of the points
        threads = oracle.num_threads()
        oracle.set_num_threads(1)
        n1 = s.n // 8
        t0 = time.perf_counter()
        L = oracle.fragments(s.xyz[:n1], s.cam)
        fw = oracle.blend_forward(L, s.opa[:n1], s.feat[:n1], 1e-4)
        oracle.blend_backward(L, s.opa[:n1], s.feat[:n1], fw["n_blended"], s.g_img)
        dt1 = time.perf_counter() - t0
        oracle.set_num_threads(threads)
        result["cpu_baseline"]["one_thread"] = {
            "value": round(L.m / dt1, 1), "unit": "fragments/s", "cores": 1,
            "sample": f"first {n1} points of the workload: {L.m} fragments, fwd+bwd in {dt1:.2f} s"}
        del L, fw

    if not args.no_next:
        # cost of the optional per-point blend weight output on the same forward
        bw = torch.empty((s.n,), dtype=torch.float32, device=dev)

        def fwd(with_bw):
            pr.rasterize_forward(x, f.detach(), o.detach(), s.cam, 1e-4, "save", args.tuning,
                                 blend_weight=bw if with_bw else None)
        result["blend_weight"] = {
            "ms_forward_without": round(time_ms(torch, lambda: fwd(False)), 4),
            "ms_forward_with": round(time_ms(torch, lambda: fwd(True)), 4),
        }

    if not args.no_batched:
        result["batched"] = bench_batched(pr, torch, np, workloads, log)

    if not args.no_next:
        result["pipeline"] = bench_pipeline(pr, torch, np, workloads, log)

    if args.calib_copy:
        a = torch.empty(256 * 1024 * 1024, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log("calibration copy: 1 GiB read + 1 GiB written")
    print(json.dumps(result), flush=True)


def time_ms(torch, fn, reps=10, warm=2):
    """Mean time of fn() over reps calls, HIP events on the current stream."""
    for _ in range(warm):
        fn()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


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
    out["ms_sample_view_8M"] = round(time_ms(torch, lambda: pr.sample_view(tree, cam, n, seed=(1, 2))), 4)
    out["unresolved"] = int(unres.item())
    raw = raw_rows(n).requires_grad_(True)
    views = pr.make_views([cam], [0], [n])
    out["ms_appearance_fwd_8M"] = round(time_ms(torch, lambda: pr.appearance_forward(xyz, raw.detach(), views)), 4)
    go = torch.randn((n,), device=dev, generator=gen)
    gf = torch.randn((n, 4), device=dev, generator=gen)
    out["ms_appearance_bwd_8M"] = round(
        time_ms(torch, lambda: pr.appearance_backward(xyz, raw.detach(), views, go, gf)), 4)
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
    out["ms_train_step"] = round(time_ms(torch, train_step, reps=5), 4)
    out["ms_prob_update"] = round(time_ms(torch, lambda: pr.update_probabilities(tree, leaf, bw)), 4)
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
    out["ms_sample_4x8M"] = round(time_ms(torch, sample4, reps=3), 4)
    out["ms_appearance_4x8M"] = round(time_ms(torch, lambda: pr.appearance_forward(xs4, raw4, views4), reps=3), 4)
    o4, f4 = pr.appearance_forward(xs4, raw4, views4)
    offs = [k * n for k in range(K)]
    out["ms_multisample_raster_4x8M"] = round(
        time_ms(torch, lambda: pr.multisample(xs4, f4, o4, cam, offs, [n] * K), reps=3), 4)

    def infer():
        sample4()
        a_o, a_f = pr.appearance_forward(xs4, raw4, views4)
        pr.multisample(xs4, a_f, a_o, cam, offs, [n] * K)
    out["ms_inference_4x8M"] = round(time_ms(torch, infer, reps=3), 4)
    log(f"pipeline: {json.dumps(out)}")
    return out


def bench_batched(pr, torch, np, workloads, log, reps=5):
    """16 views, BF16 features, one graph replay vs 16 plain FP32 calls."""
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
    step = pr.BatchedStep(x, fbf, o, views, g)
    best, best_ms = pr.autotune(x, fbf, o, views, g_img=g, repeats=2)
    step = pr.BatchedStep(x, fbf, o, views, g, tuning_id=best)
    step.capture()
    for _ in range(2):
        step.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        step.replay()
    e1.record()
    torch.cuda.synchronize()
    t_batched = e0.elapsed_time(e1) / reps
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

    run_plain()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        run_plain()
    e1.record()
    torch.cuda.synchronize()
    t_plain = e0.elapsed_time(e1) / reps
    M = pr.fragment_count(step.state())
    # accuracy of the batched BF16 image vs the plain FP32 image of each view
    img32 = []
    for xv, fv, ov, cam, gv in plain:
        im, tf, st = pr.rasterize_forward(xv, fv, ov, cam, 1e-4, "save", -1)
        img32.append(im.reshape(-1, b.F))
    img32 = torch.cat(img32)
    err = (step.image - img32).abs().max().item()
    log(f"batched: {t_batched:.3f} ms (graph replay, tuning {best}), plain 16 calls: {t_plain:.3f} ms")
    return {"views": len(b.cams), "points": int(sum(b.point_count)), "pixels": int(offs[-1]),
            "fragments": M, "ms_batched_bf16_graph": round(t_batched, 3),
            "ms_plain_f32_sequential": round(t_plain, 3),
            "speedup": round(t_plain / t_batched, 3),
            "fragments_per_s_batched": round(M / (t_batched * 1e-3), 1),
            "max_abs_image_diff_bf16_vs_f32": err, "tuning": best}


if __name__ == "__main__":
    main()
