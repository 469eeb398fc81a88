"""Benchmark: progressive critical-point classification of a 512^3 field.

One step = one pass of the whole hot path: every level of the hierarchy,
coarse (2^3) to fine (512^3), every vertex of each level classified and the
level compacted into its ascending critical list.  The field is resident in
HBM before the timed region.

Prints one JSON line.  value = vertices of all levels / ms_per_step, in
Gvertices/s, with the steps enqueued back to back through the asynchronous
entry point; ms_per_step_sync is the same loop through the synchronous one
(the host waits for every step).  Extra keys: time_to_exact_ms (start of
the step's first kernel to level-0 completion, stream events, with the
step's kernels already queued); "preview": F1 of the preview
against the exact list at 10, 25, 50, 75 and 90 % of the plain call's time
to exact, for the
plain level order, for region-by-region refinement in region id order and
in the learned order (the order network trained, untimed, on held-out
fields), on this field and on the smooth recipe at 512^3; "batch": 200
independent fields of 33..257 samples per axis classified with shared
launches against one call per field; "order_field": the order field
(ranks by value, ties by index) and extremum lists of the bench field;
"lts_step1": the superlevel / sublevel set propagation from every maximum
and minimum of the bench field (Step 1 of the simplification, each
extremum on its own and merged at saddles, with the persistence test at two
epsilons); the
direct level-0 rate; per-level rates; the roofline of the dominant kernel; and the CPU
oracle's rate on bounded samples of the same workload (all threads of this
process's share, and one thread).
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


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


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


PREVIEW_FRACS = (0.10, 0.25, 0.50, 0.75, 0.90)
# evaluation fields (the bench field and the smooth gsin recipe at 512^3)
# and the held-out fields of the same recipes the order network trains on
EVAL_FIELDS = {"noisy512": ("noisy512", None), "gsin512": ("gsin256", None)}
TRAIN_FIELDS = [("noisy512", 13), ("gsin256", 12)]


def recipe_field(recipe, seed=None, shape=(512, 512, 512)):
    import fieldgen
    kw = dict(fieldgen.CONFIGS[recipe])
    kw["shape"] = tuple(shape)
    if seed is not None:
        kw["seed"] = seed
    return fieldgen.gaussian_field(device="cuda", **kw)


def train_order_network(pc, ctx, dev, steps=3000):
    """Trains the refinement-order network on held-out fields of both
    recipes (untimed); returns (params, first and last mean loss)."""
    import torch
    sets = []
    for recipe, seed in TRAIN_FIELDS:
        ft = torch.from_numpy(recipe_field(recipe, seed)).to(dev)
        sets.append(pc.learned_order.training_set(ft, ctx=ctx))
        del ft
    params = pc.learned_order.init_params(0, dev)
    losses = pc.learned_order.train(params, sets, steps=steps, lr=1e-2, ctx=ctx)
    return params, sets[0].level, losses


BATCH_FIELDS = 200
BATCH_AXIS = (33, 257)


def batch_measure(pc, ctx, dev, reps=10):
    """Batched classification of many independent fields against one call
    per field: 200 3D fields, every axis drawn from U{33..257} (seed 5),
    each 8 Gaussians (the small-field recipe without noise), resident on the
    GPU; every way enqueued back to back with device-side counts; the
    batched call also as a replayed HIP graph, and with the launch
    configuration the autotuner picks for this batch ('tuned')."""
    import torch
    import fieldgen
    rng = np.random.default_rng(5)
    ts = []
    for i in range(BATCH_FIELDS):
        shape = tuple(int(v) for v in rng.integers(BATCH_AXIS[0], BATCH_AXIS[1] + 1, size=3))
        f = fieldgen.gaussian_field(shape, 1000 + i, 8, device="cuda")
        ts.append(torch.from_numpy(f).to(dev))
    nv = sum(t.numel() for t in ts)
    codes = [torch.empty(t.shape, dtype=torch.uint8, device=dev) for t in ts]
    crit = torch.empty(nv, dtype=torch.int32, device=dev)
    offs = torch.empty(BATCH_FIELDS + 1, dtype=torch.int64, device=dev)
    ref = pc.classify_batch(ts, ctx=ctx, codes=codes, crit=crit)
    # one call per field into its own slice of the same list buffer
    counts = torch.empty(BATCH_FIELDS, dtype=torch.int64, device=dev)
    starts = np.concatenate([[0], np.cumsum([t.numel() for t in ts])])
    crit1 = torch.empty(nv, dtype=torch.int32, device=dev)

    def per_field():
        for i, t in enumerate(ts):
            pc.classify(t, ctx=ctx, codes=codes[i], crit=crit1[int(starts[i]):int(starts[i + 1])],
                        count_dev=counts[i:i + 1])

    def batched():
        pc.classify_batch(ts, ctx=ctx, codes=codes, crit=crit, offsets_dev=offs)

    for fn in (per_field, batched):
        fn()
    torch.cuda.synchronize()
    # the same lists both ways
    cnt = counts.cpu().numpy()
    for i in (0, BATCH_FIELDS // 2, BATCH_FIELDS - 1):
        a = ref.field_list(i)
        assert int(cnt[i]) == a.numel()
        assert torch.equal(crit1[int(starts[i]):int(starts[i]) + a.numel()], a)
    # the batched call captured once in a graph and replayed
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        batched()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        batched()
    graph.replay()
    torch.cuda.synchronize()
    assert torch.equal(offs.cpu(), torch.from_numpy(ref.offsets))
    out = {}
    for name, fn in (("per_field", per_field), ("batched", batched),
                     ("batched_graph", graph.replay)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / reps
        out[name + "_ms"] = round(ms, 3)
        out[name + "_gvps"] = round(nv / (ms * 1e-3) / 1e9, 2)
    # the launch configuration tuned on this batch (a context of its own):
    # every candidate's time, the choice, and the batched call with it
    tctx = pc.Context(0)
    choice, table, tcodes, tcrit, _ = pc.batch_autotune(ts, ctx=tctx, reps=3)
    torch.cuda.synchronize()
    n = int(ref.offsets[-1])
    assert torch.equal(tcrit[:n], ref.crit[:n])
    tcrit = tcodes = None

    def tuned():
        pc.classify_batch(ts, ctx=tctx, codes=codes, crit=crit, offsets_dev=offs)

    tuned()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        tuned()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    assert torch.equal(offs.cpu(), torch.from_numpy(ref.offsets))
    out["tuned"] = {"group": choice[0], "want_tiles": choice[1], "ms": round(ms, 3),
                    "gvps": round(nv / (ms * 1e-3) / 1e9, 2),
                    "candidates_ms": {f"{g}x{w}": round(v, 3) for (g, w), v in table.items()}}
    out.update({"fields": BATCH_FIELDS, "axis": list(BATCH_AXIS), "vertices": int(nv),
                "critical": int(ref.offsets[-1]),
                "speedup": round(out["per_field_ms"] / out["batched_ms"], 2)})
    return out


def order_measure(pc, ctx, ft, codes, reps=5):
    """Order field (ranks by value, ties by index) and extremum lists of the
    bench field; algorithmic bytes of the order field: the field read and
    the ranks written, 8 B per vertex."""
    import torch
    n = ft.numel()
    rank = torch.empty(n, dtype=torch.int32, device=ft.device)
    srt = torch.empty(n, dtype=torch.int32, device=ft.device)
    pc.order_field(ft, ctx=ctx, rank=rank, sorted_out=srt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        pc.order_field(ft, ctx=ctx, rank=rank, sorted_out=srt)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    pc.extrema(codes, ctx=ctx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        mn, mx = pc.extrema(codes, ctx=ctx)
    torch.cuda.synchronize()
    ems = (time.perf_counter() - t0) * 1e3 / reps
    gbs = 8 * n / (ms * 1e-3) / 1e9
    return {"order_field_ms": round(ms, 3), "order_field_gkeys": round(n / (ms * 1e-3) / 1e9, 2),
            "order_field_frac": round(gbs / HBM_PEAK_GBS, 4),
            "extrema_ms": round(ems, 3), "minima": int(mn.numel()), "maxima": int(mx.numel()),
            "note": "both calls wait for the stream; times include the host wait"}


def lts_measure(pc, ctx, ft, codes, reps=5):
    """LTS Step 1 on the bench field: from every maximum and every minimum,
    the propagation with the persistence test at epsilon 0.01 (about the
    noise's standard deviation) and 0.05, budget 16 vertices taken / 64
    waiting; each extremum on its own ('max', 'min') and merged at saddles
    ('merged_max', 'merged_min': the last arrival at a saddle goes on with
    every arrived component).  Inputs (order field, extremum lists) are
    computed first and not timed; the first merged call grows the scratch
    outside the timed calls."""
    import torch
    rank, _ = pc.order_field(ft, ctx=ctx)
    mn, mx = pc.extrema(codes, ctx=ctx)
    torch.cuda.synchronize()
    out = {"maxima": int(mx.numel()), "minima": int(mn.numel()), "budget": [16, 64]}
    for eps in (0.01, 0.05):
        row = {}
        for name, fn in (("", pc.lts_propagate), ("merged_", pc.lts_merged)):
            for kind, ext, up in (("max", mx, True), ("min", mn, False)):
                fn(ft, rank, ext, maxima=up, epsilon=eps, ctx=ctx)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(reps):
                    st, sd, vi = fn(ft, rank, ext, maxima=up, epsilon=eps, ctx=ctx)
                torch.cuda.synchronize()
                ms = (time.perf_counter() - t0) * 1e3 / reps
                cnt = np.bincount(st.cpu().numpy(), minlength=4)
                row[name + kind] = {"ms": round(ms, 3),
                                    "mprop_per_s": round(ext.numel() / (ms * 1e-3) / 1e6, 1),
                                    "saddle": int(cnt[0]), "persistent": int(cnt[1]),
                                    "budget": int(cnt[2]),
                                    "mean_visited": round(float(vi.float().mean().item()), 2)}
        out[f"eps_{eps}"] = row
    out["note"] = ("'max'/'min': one propagation per extremum; 'merged_*': propagations merged at "
                   "saddles (saddle = paired with a saddle, i.e. removed); times include the host wait")
    return out


def _region_of(points, shape, edge):
    nz, ny, nx = shape
    nry = -(-ny // edge)
    p = points.astype(np.int64)
    return ((p // (nx * ny)) // edge) * nry + ((p // nx) % ny) // edge


def preview_quality(pc, ctx, ft, params, reps=5, edge=64):
    """Preview F1 against the exact list at PREVIEW_FRACS of the plain
    call's time to exact (one clock for every mode): 'plain' shows the
    finest level whose list is complete; 'regional' (regions in id order),
    'learned' (regions by the network's scores) and 'ideal' (regions by
    their exact critical counts: a bound no real order reaches) show each
    region at the finest level finished there.  None where no preview
    exists yet."""
    shape = tuple(ft.shape)
    pr = pc.progressive(ft, ctx=ctx, with_crit_codes=True)
    levels = pr.levels
    lists = {k: pr.level_list(k).cpu().numpy().view(np.uint32) for k in levels}
    lcodes = {k: pr.level_codes(k).cpu().numpy() for k in levels}
    regs = {k: _region_of(lists[k], shape, edge) for k in levels}
    exact, exact_c = lists[0], lcodes[0]
    cache = {}

    def f1_levels(chosen):
        """chosen[r] = level index shown for region r (-1: none)."""
        key = chosen.tobytes()
        if key in cache:
            return cache[key]
        pts, cds, lvs = [], [], []
        for i, k in enumerate(levels):
            m = chosen[regs[k]] == i
            if m.any():
                pts.append(lists[k][m])
                cds.append(lcodes[k][m])
                lvs.append(np.full(int(m.sum()), k, np.uint8))
        if not pts:
            cache[key] = None
            return None
        f1, _ = pc.preview_f1_levels(shape, np.concatenate(pts), np.concatenate(cds),
                                     np.concatenate(lvs), exact, exact_c)
        cache[key] = round(float(f1), 4)
        return cache[key]

    nreg = pc.region_count(shape, edge)
    out = {}
    # plain: level-granular completion times of the plain progressive call
    lvl = np.median(np.array([pc.progressive(ft, ctx=ctx, level_times=True).level_ms
                              for _ in range(reps)]), axis=0)
    t_ex = clock = float(lvl[-1])
    curve = {}
    for fr in PREVIEW_FRACS:
        done = [i for i in range(len(levels)) if lvl[i] <= fr * clock]
        curve[f"{int(fr * 100)}%"] = (f1_levels(np.full(nreg, done[-1], np.int64))
                                      if done else None)
    out["plain"] = {"f1": curve, "time_to_exact_ms": round(t_ex, 4),
                    "time_to_first_preview_ms": round(float(lvl[0]), 4)}
    # an upper bound for any order: regions by their exact number of
    # level-0 critical points (known only once the exact pass has run)
    counts = np.bincount(regs[0], minlength=nreg)
    ideal_rank = np.empty(nreg, np.int32)
    ideal_rank[np.argsort(-counts, kind="stable")] = np.arange(nreg, dtype=np.int32)
    for mode in ("regional", "learned", "ideal"):
        runs = [pc.progressive_timeline(ft, edge, params=params if mode == "learned" else None,
                                        order=ideal_rank if mode == "ideal" else None,
                                        ctx=ctx) for _ in range(reps)]
        for t in runs:
            assert t.status == 0 and np.array_equal(t.offsets, pr.offsets)
        lms = np.median(np.array([t.level_ms for t in runs]), axis=0)
        rms = np.median(np.array([t.region_ms for t in runs]), axis=0)
        t_ex = float(lms[-1])
        curve = {}
        for fr in PREVIEW_FRACS:
            done = rms <= fr * clock  # [level index, region]
            idx = np.arange(len(levels))[:, None]
            chosen = np.where(done, idx, -1).max(axis=0)
            curve[f"{int(fr * 100)}%"] = f1_levels(chosen)
        out[mode] = {"f1": curve, "time_to_exact_ms": round(t_ex, 4),
                     "time_to_first_preview_ms": round(float(lms[0]), 4)}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batched many-field measurement")
    ap.add_argument("--no-preview", action="store_true",
                    help="skip the preview-quality passes (and the order "
                         "network's training)")
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
    # exact = first kernel to level-0 completion (stream events; the call
    # queues its kernels behind a short GPU wait before the start event)
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

    med_lvl = np.median(lvl_ms, axis=0)

    # preview quality (untimed passes): plain level order, regions in id
    # order, regions in the learned order, on this field and on the smooth
    # recipe at 512^3; the order network trains first on held-out fields
    previews = {}
    if not args.no_preview:
        params, flevel, losses = train_order_network(pc, ctx, dev)
        previews["order_network"] = {
            "trained_on": [f"{r} recipe, seed {sd}, 512^3" for r, sd in TRAIN_FIELDS],
            "scoring_level": flevel, "adam_steps": len(losses),
            "mean_loss_first": round(losses[0], 4), "mean_loss_last": round(losses[-1], 4)}
        for name, (recipe, seed) in EVAL_FIELDS.items():
            fe = ft if name == WORKLOAD else torch.from_numpy(recipe_field(recipe, seed)).to(dev)
            previews[name] = preview_quality(pc, ctx, fe, params)
            del fe

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
        "preview_f1_at_10pct": (previews[WORKLOAD]["plain"]["f1"]["10%"]
                                if previews else None),
        "preview": previews or None,
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

    if not args.no_batch:
        out["batch"] = batch_measure(pc, ctx, dev)
        out["order_field"] = order_measure(pc, ctx, ft, codes)
        out["lts_step1"] = lts_measure(pc, ctx, ft, codes)

    if not args.no_cpu_baseline:
        import oracle
        avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
        # the worker pool is sized to this process's share of the host
        # (OMP_NUM_THREADS when set), at most the CPUs it may run on
        share = int(os.environ.get("OMP_NUM_THREADS", avail) or avail)
        threads = max(1, min(share, avail))
        planes = min(args.cpu_planes, shape[0])
        planes1 = min(max(planes // 16, 2), shape[0])
        oracle.classify(f[:4], threads=threads)  # page in, build check
        t0 = time.perf_counter()
        res = oracle.classify(f, level=0, slow_range=(0, planes), threads=threads)
        cpu_s = time.perf_counter() - t0
        assert res.status == 0
        t0 = time.perf_counter()
        res1 = oracle.classify(f, level=0, slow_range=(0, planes1), threads=1)
        cpu1_s = time.perf_counter() - t0
        assert res1.status == 0
        nv = planes * shape[1] * shape[2]
        nv1 = planes1 * shape[1] * shape[2]
        out["cpu_baseline"] = {
            "value": round(nv / cpu_s / 1e9, 5),
            "unit": "Gvertices/s",
            "cores": threads,
            "kind": "oracle",
            "sample": f"level-0 classification (codes + ascending list) of "
                      f"z-planes 0..{planes - 1} of the 512^3 field "
                      f"({nv} vertices, {cpu_s:.2f} s on {threads} threads)",
            "value_1thread": round(nv1 / cpu1_s / 1e9, 5),
            "sample_1thread": f"z-planes 0..{planes1 - 1} ({nv1} vertices, {cpu1_s:.2f} s)",
            "cpu_model": cpu_model(),
            "cpus_visible": os.cpu_count(),
            "cpus_allowed": avail,
        }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
