"""Benchmark: progressive critical-point classification of a 512^3 field.

One step = one pass of the whole hot path: every level of the hierarchy,
coarse (2^3) to fine (512^3), each level classified (new vertices, plus old
vertices whose polarity changed) and compacted into its ascending critical
list.  The field is resident in HBM before the timed region.

Prints one JSON line.  value = vertices of all levels / ms_per_step, in
Gvertices/s, with the steps enqueued back to back through the asynchronous
entry point; ms_per_step_sync is the same loop through the synchronous one
(the host waits for every step).  Extra keys: time_to_exact_ms (first enqueue to level-0
completion, stream events), preview F1 at 10 % of that time, the direct
level-0 rate, per-level rates, the roofline of the dominant kernel, and the
CPU oracle's rate on a bounded sample of the same workload.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOAD = "noisy512"
PMC_FILE = os.path.join(ROOT, "profiles", "classify3d_quad_level0_noisy512_traffic.txt")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2009_00083_amd", "csrc", n)
                  for n in ("classify_quad.hip", "device_util.h", "pcrit_internal.h")]


def kernel_source_hash():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch of the dominant kernel from the committed
    rocprofv3 counter summary ("key: value" lines), or None if the kernel
    sources changed since the counters were taken."""
    d = {}
    try:
        with open(PMC_FILE) as fh:
            for line in fh:
                if ":" in line and not line.startswith(("#", " ", "|")):
                    k, v = line.split(":", 1)
                    d[k.strip()] = v.strip()
    except OSError:
        return None
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    try:
        return int(float(d["hbm_bytes_per_launch"]))
    except (KeyError, ValueError):
        return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-planes", type=int, default=512,
                    help="level-0 z-planes of the oracle's timed sample")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (reference for "
                         "the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported "
              "(the method needs no collective; see DESIGN.md for how it "
              "would shard)", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_calibration:
        n = 1 << 28  # float32 elements: 1 GiB read + 1 GiB written per copy
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": 4 * n, "copies": 5}))
        return
    import fieldgen
    import paper_2009_00083_amd as pc

    dev = torch.device("cuda:0")
    f = fieldgen.config_field(WORKLOAD, device="cuda")
    shape = f.shape
    ft = torch.from_numpy(f).to(dev)
    ctx = pc.Context(0)
    levels = list(range(pc.max_level(shape), -1, -1))
    sizes = {k: int(np.prod(pc.level_dims(shape, k))) for k in levels}
    total_v = sum(sizes.values())
    cap = total_v
    codes = torch.zeros(shape, dtype=torch.uint8, device=dev)
    crit = torch.empty(cap, dtype=torch.int32, device=dev)

    def step(level_times=False):
        return pc.progressive(ft, ctx=ctx, capacity=cap, codes=codes, crit=crit,
                              level_times=level_times)

    offs_dev = torch.empty(len(levels) + 1, dtype=torch.int64, device=dev)

    def step_async():
        pc.progressive_async(ft, ctx=ctx, capacity=cap, codes=codes, crit=crit,
                             offsets=offs_dev)

    for _ in range(args.warmup):
        step()
        step_async()
    torch.cuda.synchronize()

    # timed region A: the whole hot path, steps enqueued back to back (the
    # asynchronous entry point), no events inside
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step_async()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = elapsed * 1e3 / args.steps
    value = total_v / (ms_per_step * 1e-3) / 1e9

    # region S: the synchronous entry point (host waits for every step)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r = step()
    torch.cuda.synchronize()
    ms_per_step_sync = (time.perf_counter() - t0) * 1e3 / args.steps
    assert r.status == 0
    assert np.array_equal(offs_dev.cpu().numpy(), r.offsets)

    # region T: the same steps with a completion event per launch; time to
    # exact = first kernel to level-0 completion (stream events)
    lvl_ms = []
    for _ in range(args.steps):
        lvl_ms.append(step(level_times=True).level_ms.copy())
    lvl_ms = np.array(lvl_ms)
    t_exact = float(np.median(lvl_ms[:, -1]))

    # timed region B: HIP events around the level-0 kernels (on the stream
    # they run on), for the dominant kernel's duration
    ctx.set_kernel_timing([0])
    k0 = []
    torch.cuda.synchronize()
    for _ in range(args.steps):
        step()
        a, b = ctx.kernel_ms(len(levels))
        k0.append((a[0], b[0]))
    torch.cuda.synchronize()
    k0 = np.array(k0)

    # passes with every launch timed, for the per-level breakdown (levels
    # that share a launch are timed together under the finest of them)
    ctx.set_kernel_timing(True)
    cls_ms, cmp_ms = [], []
    for _ in range(5):
        step()
        a, b = ctx.kernel_ms(len(levels))
        cls_ms.append(a)
        cmp_ms.append(b)
    ctx.set_kernel_timing(None)
    cls_ms = np.median(np.array(cls_ms), axis=0)
    cmp_ms = np.median(np.array(cmp_ms), axis=0)
    per_level = {}
    pending = []
    for k in levels:
        pending.append(k)
        c, m = float(cls_ms[k]), float(cmp_ms[k])
        if c < 0:
            continue  # shares the launch of a finer level
        nv = sum(sizes[j] for j in pending)
        e = {"vertices": nv, "classify_us": round(c * 1e3, 2),
             "compact_us": round(m * 1e3, 2),
             "gvps": round(nv / ((c + m) * 1e-3) / 1e9, 2)}
        if len(pending) > 1:
            e["levels"] = list(pending)
        per_level[str(k)] = e
        pending = []

    # dominant kernel: level-0 classification (progressive)
    k0_ms = float(np.mean(k0[:, 0]))
    alg_bytes = 5 * sizes[0]  # 4 B field read + 1 B code write per vertex
    achieved = alg_bytes / (k0_ms * 1e-3) / 1e9
    traffic = measured_traffic()

    # preview F1 at 10 % of time-to-exact (lists are deterministic, so take
    # them from one more untimed pass that also returns the codes)
    pr = pc.progressive(ft, ctx=ctx, with_crit_codes=True)
    med_lvl = np.median(lvl_ms, axis=0)
    budget = 0.1 * t_exact
    done = [i for i in range(len(levels)) if med_lvl[i] <= budget]
    exact = pr.level_list(0).cpu().numpy().view(np.uint32)
    exact_c = pr.level_codes(0).cpu().numpy()
    if done:
        i = done[-1]
        kprev = levels[i]
        prev = pr.level_list(kprev).cpu().numpy().view(np.uint32)
        prev_c = pr.level_codes(kprev).cpu().numpy()
        f1, _ = pc.preview_f1(shape, kprev, prev, prev_c, exact, exact_c)
    else:
        kprev, f1 = None, 0.0

    # old vertices whose polarity mask or absent set changed, per level
    # (a counting pass, untimed: the timed steps do not count)
    rc = pc.progressive(ft, ctx=ctx, count_reclassified=True)
    assert np.array_equal(rc.offsets, r.offsets)

    # direct level-0 pass for reference
    dcrit = torch.empty(sizes[0], dtype=torch.int32, device=dev)
    for _ in range(3):
        pc.classify(ft, 0, ctx=ctx, codes=codes, crit=dcrit)
    torch.cuda.synchronize()
    nd = max(10, args.steps // 2)
    t0 = time.perf_counter()
    for _ in range(nd):
        d = pc.classify(ft, 0, ctx=ctx, codes=codes, crit=dcrit)
    torch.cuda.synchronize()
    direct_ms = (time.perf_counter() - t0) * 1e3 / nd

    out = {
        "metric": "Gvertices/s classified at 512^3 (all levels); time-to-exact; "
                  "preview F1 @10% time",
        "value": round(value, 3),
        "unit": "Gvertices/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "ms_per_step_sync": round(ms_per_step_sync, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "progressive classification of a 512^3 float32 field "
                        "(256 Gaussians + N(0, 1e-2^2) noise, seed 3), levels "
                        "8..0 (2^3 .. 512^3), codes + ascending critical lists",
            "vertices_all_levels": total_v,
            "critical_fraction_level0": round(d.count / sizes[0], 4),
        },
        "time_to_exact_ms": round(t_exact, 4),
        "level_done_ms": {str(k): round(float(v), 4) for k, v in zip(levels, med_lvl)},
        "preview_f1_at_10pct": round(f1, 4),
        "preview_level_at_10pct": kprev,
        "direct_level0_gvps": round(sizes[0] / (direct_ms * 1e-3) / 1e9, 2),
        "direct_level0_ms": round(direct_ms, 4),
        "per_level": per_level,
        "reclassified_old_vertices": {str(k): int(v) for k, v in
                                      zip(levels, rc.reclassified)},
        "roofline": {
            "kernel": "classify3d_quad (progressive, level 0)",
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "kernel_us": round(k0_ms * 1e3, 2),
            "compact_us": round(float(np.mean(k0[:, 1])) * 1e3, 2),
            "algorithmic_bytes": alg_bytes,
        },
    }

    if not args.no_cpu_baseline:
        import oracle
        threads = min(16, os.cpu_count() or 1)
        planes = min(args.cpu_planes, shape[0])
        oracle.classify(f[:4], threads=threads)  # page in, build check
        t0 = time.perf_counter()
        res = oracle.classify(f, level=0, slow_range=(0, planes), threads=threads)
        cpu_s = time.perf_counter() - t0
        nv = planes * shape[1] * shape[2]
        out["cpu_baseline"] = {
            "value": round(nv / cpu_s / 1e9, 5),
            "unit": "Gvertices/s",
            "cores": threads,
            "kind": "oracle",
            "sample": f"level-0 classification (codes + ascending list) of "
                      f"z-planes 0..{planes - 1} of the 512^3 field "
                      f"({nv} vertices, {cpu_s:.2f} s)",
        }
        assert res.status == 0
    print(json.dumps(out))


if __name__ == "__main__":
    main()
