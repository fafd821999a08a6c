"""Summaries of rocprofv3 output for the benchmark's kernels, and a driver
for the batched workload to run under the profiler.

    python -m paper_2307_16080_amd.profiling stats  <kernel_stats.csv>
    python -m paper_2307_16080_amd.profiling traffic <fetch_counters.csv> <write_counters.csv>
            <kernel-name-substring> <copy-bytes> <out.json> [source_hash] [tile]
    python -m paper_2307_16080_amd.profiling batched <tile> <launches>
    python -m paper_2307_16080_amd.profiling paperconv <tile> <launches>
    python -m paper_2307_16080_amd.profiling gemm <bf16|e4m3|f32|i8> <tile> <launches> [size]
    python -m paper_2307_16080_amd.profiling counters <counter_collection.csv> <kernel-name-substring>
    python -m paper_2307_16080_amd.profiling window <kernel_trace.csv> <kernel-name-substring> <first> <count>
    python -m paper_2307_16080_amd.profiling gemm-summary <dir> <source_hash> <tile> [<tile> ...]
    python -m paper_2307_16080_amd.profiling resnet <batch> <launches> [graph]
    python -m paper_2307_16080_amd.profiling lastpass <kernel_trace.csv> <dispatches per pass> [passes]
    python -m paper_2307_16080_amd.profiling convf32 <tile> <launches>
    python -m paper_2307_16080_amd.profiling convbatch <batch> <tile|default> <launches>
    python -m paper_2307_16080_amd.profiling quantize <bf16|e4m3> <launches>
    python -m paper_2307_16080_amd.profiling conv <N,C,H,W,F,KH,KW,stride,pad> <tile> <launches>

`batched` runs the 256 uneven bf16 GEMMs of the benchmark (seeded shapes and
inputs) as persistent launches, replayed from a hipGraph, with the given tile
(ten comma-separated configuration fields).

`traffic` turns the FETCH_SIZE / WRITE_SIZE counters (KiB per dispatch) of
the kernel into bytes per launch, scaled by what the same counters read for
the benchmark's plain device copy of `copy-bytes` bytes (the copy reads and
writes exactly that many bytes), and writes them as JSON.  The reference copy
is the largest copy dispatch of the run: the runtime may also move host
transfers through small staging copies of the same kernel, which are not it.
"""
import csv
import json
import sys


def _rows(path):
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def stats(path, top=12):
    rows = _rows(path)
    rows.sort(key=lambda r: -float(r.get("TotalDurationNs", 0) or 0))
    out = [f"{'calls':>7} {'avg_us':>10} {'min_us':>10} {'max_us':>10} {'pct':>6}  kernel"]
    for r in rows[:top]:
        out.append(f"{int(r['Calls']):7d} {float(r['AverageNs']) / 1e3:10.2f} {float(r['MinNs']) / 1e3:10.2f} "
                   f"{float(r['MaxNs']) / 1e3:10.2f} {float(r['Percentage']):6.2f}  {r['Name'][:150]}")
    return "\n".join(out)


def _counter_per_dispatch(path, counter, name_sub, largest=False):
    """Counter value (summed over its instances) per dispatch of kernels matching
    name_sub: the mean over those dispatches, or with largest=True the largest one."""
    per = {}
    for r in _rows(path):
        if r.get("Counter_Name") != counter or name_sub not in r.get("Kernel_Name", ""):
            continue
        d = r.get("Dispatch_Id") or r.get("Correlation_Id")
        per[d] = per.get(d, 0.0) + float(r["Counter_Value"])
    if not per:
        return None, 0
    if largest:
        return max(per.values()), len(per)
    return sum(per.values()) / len(per), len(per)


def counters(path, kernel_sub):
    """Every counter of a --pmc run, per dispatch of kernels matching
    kernel_sub: summed over the counter's instances (the largest instance for
    the GRBM_* counters, which count whole-GPU cycles), averaged over the
    dispatches."""
    per = {}
    for r in _rows(path):
        if kernel_sub not in r.get("Kernel_Name", ""):
            continue
        name = r["Counter_Name"]
        d = r.get("Dispatch_Id") or r.get("Correlation_Id")
        v = float(r["Counter_Value"])
        slot = per.setdefault(name, {})
        slot[d] = max(slot.get(d, 0.0), v) if name.startswith("GRBM_") else slot.get(d, 0.0) + v
    return {k: sum(v.values()) / len(v) for k, v in per.items()}, {k: len(v) for k, v in per.items()}


def window(trace_csv, kernel_sub, first, count):
    """Durations (us) of dispatches first .. first+count-1 (negative first counts
    from the end) of the kernels matching kernel_sub, in dispatch order."""
    rows = [r for r in _rows(trace_csv) if kernel_sub in r["Kernel_Name"]]
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    sel = rows[first:first + count] if first >= 0 else rows[len(rows) + first:len(rows) + first + count]
    return [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in sel]


def last_pass(trace_csv, count, passes=1):
    """The last `passes` runs of a sequence of `count` dispatches (the trace's
    last count * passes dispatches, in start order): per dispatch its kernel,
    duration and the gap since the previous dispatch ended, and per pass the
    kernel time summed by kernel family against first start to last end."""
    rows = sorted(_rows(trace_csv), key=lambda r: int(r["Start_Timestamp"]))
    rows = rows[len(rows) - count * passes:]
    out = []
    for p in range(passes):
        sel = rows[p * count:(p + 1) * count]
        t0, t1 = int(sel[0]["Start_Timestamp"]), max(int(r["End_Timestamp"]) for r in sel)
        fam, items, prev_end = {}, [], None
        for r in sel:
            st, en = int(r["Start_Timestamp"]), int(r["End_Timestamp"])
            name = r["Kernel_Name"].replace("(anonymous namespace)::", "").split("(")[0]
            name = name.replace("void ", "").replace("mlk::", "")
            key = name.split("<")[0]
            fam[key] = fam.get(key, 0.0) + (en - st) / 1e3
            items.append({"kernel": name[:70], "us": round((en - st) / 1e3, 2),
                          "gap_us": round((st - prev_end) / 1e3, 2) if prev_end is not None else None})
            prev_end = en
        out.append({"span_us": round((t1 - t0) / 1e3, 1), "kernel_us": round(sum(fam.values()), 1),
                    "by_family_us": {k: round(v, 1) for k, v in sorted(fam.items(), key=lambda kv: -kv[1])},
                    "dispatches": items})
    return out


def gemm_summary(root, tile, source_hash, copy_bytes=256 << 20, warmup=5, steps=20):
    """One JSON-able record for one bf16 4096^3 tile from its four rocprofv3
    runs under root: t_<tile> (kernel trace of the benchmark command), f_ and
    w_ (FETCH_SIZE / WRITE_SIZE), m_ (SQ_VALU_MFMA_BUSY_CYCLES, GRBM_GUI_ACTIVE,
    SQ_BUSY_CU_CYCLES with a kernel trace).  MFMA utilisation follows the
    profiler's own MfmaUtil definition: busy cycles / (GRBM_GUI_ACTIVE of one
    XCD x 1024 SIMDs); the CSV's GRBM_GUI_ACTIVE is summed over the 8 XCDs."""
    w = tile.split(",")
    mf = 32 if len(w) > 10 and int(w[10]) == 32 else 16
    kname = f"k_gemm_fast<1, {w[0]}, {w[1]}, {w[3]}, {w[4]}, {w[8]}, 0, {mf}>"
    every = window(f"{root}/t_{tile}/t_kernel_trace.csv", kname, 0, 1 << 30)
    timed = window(f"{root}/t_{tile}/t_kernel_trace.csv", kname, warmup, steps)
    tr = traffic(f"{root}/f_{tile}/f_counter_collection.csv", f"{root}/w_{tile}/w_counter_collection.csv", kname,
                 copy_bytes)
    cnt, _ = counters(f"{root}/m_{tile}/m_counter_collection.csv", kname)
    grbm_xcd = cnt["GRBM_GUI_ACTIVE"] / 8.0
    return {"config": [int(v) for v in w], "kernel": kname, "source_hash": source_hash,
            "trace": {"dispatches": len(every), "avg_us": round(sum(every) / len(every), 2),
                      "timed_window_avg_us": round(sum(timed) / len(timed), 2), "timed_window_min_us": round(min(timed), 2)},
            "fetch_bytes": round(tr["fetch_bytes"]), "write_bytes": round(tr["write_bytes"]),
            "bytes_per_launch": round(tr["bytes_per_launch"]),
            "mfma_busy_cycles": cnt["SQ_VALU_MFMA_BUSY_CYCLES"], "grbm_gui_active_per_xcd": round(grbm_xcd),
            "mfma_util_pct": round(100.0 * cnt["SQ_VALU_MFMA_BUSY_CYCLES"] / (grbm_xcd * 1024), 1)}


def traffic(fetch_csv, write_csv, kernel_sub, copy_bytes, copy_sub="copy"):
    f_k, nf = _counter_per_dispatch(fetch_csv, "FETCH_SIZE", kernel_sub)
    w_k, nw = _counter_per_dispatch(write_csv, "WRITE_SIZE", kernel_sub)
    f_c, _ = _counter_per_dispatch(fetch_csv, "FETCH_SIZE", copy_sub, largest=True)
    w_c, _ = _counter_per_dispatch(write_csv, "WRITE_SIZE", copy_sub, largest=True)
    if None in (f_k, w_k, f_c, w_c):
        raise SystemExit("counters missing for the kernel or the copy")
    fetch_scale = copy_bytes / f_c      # bytes per counter unit, read side
    write_scale = copy_bytes / w_c
    return {"fetch_bytes": f_k * fetch_scale, "write_bytes": w_k * write_scale,
            "bytes_per_launch": f_k * fetch_scale + w_k * write_scale,
            "raw": {"kernel_fetch_kib": f_k, "kernel_write_kib": w_k, "copy_fetch_kib": f_c,
                    "copy_write_kib": w_c, "dispatches": [nf, nw]},
            "scale": {"fetch_bytes_per_unit": fetch_scale, "write_bytes_per_unit": write_scale}}


def run_batched(tile, launches):
    import os

    import torch

    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import paper_2307_16080_amd as mlk
    from workloads import batched_inputs, batched_shapes

    shapes = batched_shapes(256, seed=0)
    probs = []
    for (a, b), (m, n, k) in zip(batched_inputs(shapes, seed=1), shapes):
        qa, _ = mlk.quantize(torch.from_numpy(a).cuda(), "bf16")
        qb, _ = mlk.quantize(torch.from_numpy(b).cuda(), "bf16")
        probs.append((qa, qb, torch.zeros(m, n, device="cuda")))
    cfg = mlk.TileConfig(*[int(v) for v in tile.split(",")])
    call = mlk.BatchedCall(probs, cfg=cfg, persistent=True, graph=True)
    for _ in range(launches):
        call()
    torch.cuda.synchronize()
    print(f"batched: {launches} persistent launches of {len(shapes)} GEMMs, tile {tile}", flush=True)


def run_conv(shape, tile, launches):
    """One bf16 convolution (normal(0, 1) inputs from seed 0, quantised to bf16
    on the GPU; y += conv) bound once with one fixed tile and called back to
    back, then the reference copy."""
    import os

    import torch

    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import paper_2307_16080_amd as mlk
    from workloads import conv_inputs

    n, c, h, w, f, kh, kw, st, pd = [int(v) for v in shape.split(",")]
    x, wt = conv_inputs(n, c, h, w, f, kh, kw, seed=0)
    xq, _ = mlk.quantize(torch.from_numpy(x).cuda(), "bf16")
    wq, _ = mlk.quantize(torch.from_numpy(wt).cuda(), "bf16")
    y = torch.zeros(n, f, (h + 2 * pd - kh) // st + 1, (w + 2 * pd - kw) // st + 1, device="cuda")
    call = mlk.ConvCall(xq, wq, y, (st, st), (pd, pd), cfg=mlk.TileConfig(*[int(v) for v in tile.split(",")]))
    for _ in range(launches):
        call()
    torch.cuda.synchronize()
    _copy_reference()
    print(f"conv {shape} bf16: {launches} calls, tile {tile}; one 256 MiB copy", flush=True)


def run_quantize(fmt, launches):
    """The benchmark's quantisation: the 4096 x 4096 float32 A operand
    (normal(0, 1), seed 0) quantised to bf16 or e4m3 into the same output
    buffers, back to back, then the reference copy."""
    import os

    import torch

    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import paper_2307_16080_amd as mlk
    from workloads import matmul_inputs

    a, _ = matmul_inputs(4096, 4096, 4096, seed=0, dist="normal")
    x = torch.from_numpy(a).cuda()
    q, s = mlk.quantize(x, fmt)
    for _ in range(launches):
        mlk.quantize(x, fmt, q=q, scale=s)
    torch.cuda.synchronize()
    _copy_reference()
    print(f"quantize {fmt} 4096x4096: {launches} calls; one 256 MiB copy", flush=True)


def run_paper_conv(tile, launches):
    """The paper's measured layer (one 1280 x 1280 image, three 3 x 3 filters,
    valid, fp32, y += conv) launched back to back with the given tile, then one
    plain 256 MiB device copy (the reference for the HBM byte counters)."""
    import os

    import torch

    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import paper_2307_16080_amd as mlk
    from workloads import conv_inputs

    x, w = conv_inputs(1, 1, 1280, 1280, 3, 3, 3, seed=0)
    xd, wd = torch.from_numpy(x).cuda(), torch.from_numpy(w).cuda()
    y = torch.zeros(1, 3, 1278, 1278, device="cuda")
    cfg = mlk.TileConfig(*[int(v) for v in tile.split(",")])
    call = mlk.ConvCall(xd, wd, y, (1, 1), (0, 0), cfg=cfg)
    for _ in range(launches):
        call()
    src = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    print(f"paper conv: {launches} launches, tile {tile}; one 256 MiB copy", flush=True)


def _copy_reference():
    """One plain 256 MiB device copy: the reference dispatch for the HBM byte counters."""
    import torch

    src = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()


def run_gemm(kind, tile, launches, size=4096):
    """The benchmark's square GEMM (C += A B, inputs seeded as the benchmark
    draws them) launched back to back with one fixed tile, then the reference
    copy.  kind: bf16 | e4m3 | f32 (size^3) or i8 (1024^3 by default)."""
    import os

    import torch

    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import paper_2307_16080_amd as mlk
    from workloads import matmul_inputs

    n = size
    A, B = matmul_inputs(n, n, n, seed=0, dist="int8" if kind == "i8" else "normal")
    Ad, Bd = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    kw = {}
    if kind == "bf16":
        a, _ = mlk.quantize(Ad, "bf16")
        b, _ = mlk.quantize(Bd, "bf16")
        C = torch.zeros(n, n, device="cuda")
    elif kind == "e4m3":
        a, sa = mlk.quantize(Ad, "e4m3")
        b, sb = mlk.quantize(Bd, "e4m3")
        kw = dict(scale_a=sa, scale_b=sb)
        C = torch.zeros(n, n, device="cuda")
    elif kind == "i8":
        a, b = Ad, Bd
        C = torch.zeros(n, n, dtype=torch.int32, device="cuda")
    else:
        a, b = Ad, Bd
        C = torch.zeros(n, n, device="cuda")
    cfg = mlk.TileConfig(*[int(v) for v in tile.split(",")])
    for _ in range(launches):
        mlk.matmul(a, b, C, cfg=cfg, **kw)
    torch.cuda.synchronize()
    _copy_reference()
    print(f"gemm {kind} {n}^3: {launches} launches, tile {tile}; one 256 MiB copy", flush=True)


def run_conv_f32(tile, launches):
    """The fp32 conv of the benchmark (1 x 64 x 56 x 56, 64 filters 3 x 3, stride
    1, pad 1, normal(0, 1) from seed 0, y += conv) bound once and called back
    to back with one fixed tile, then the reference copy."""
    import os

    import torch

    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import paper_2307_16080_amd as mlk
    from workloads import CFG_CONV_F32 as cs, conv_inputs

    x, w = conv_inputs(cs.N, cs.C, cs.H, cs.W, cs.F, cs.KH, cs.KW, seed=0)
    xd, wd = torch.from_numpy(x).cuda(), torch.from_numpy(w).cuda()
    y = torch.zeros(cs.N, cs.F, *cs.out_hw(), device="cuda")
    call = mlk.ConvCall(xd, wd, y, (cs.stride,) * 2, (cs.pad,) * 2,
                        cfg=mlk.TileConfig(*[int(v) for v in tile.split(",")]))
    for _ in range(launches):
        call()
    torch.cuda.synchronize()
    _copy_reference()
    print(f"conv f32 56x56x64: {launches} calls, tile {tile}; one 256 MiB copy", flush=True)


def run_resnet(batch, launches, graph=False):
    """The ResNet-18 conv stack (bf16, seeded inputs) at one batch size: each
    layer's tile picked as the benchmark picks it (exhaustive table, then its
    fastest entries re-timed as bound calls in graphs), then every layer of
    the stack launched `launches` times in stack order with that tile;
    with `graph`, the stack is captured once as one graph and the graph is
    replayed `launches` times (the benchmark's timing of the stack)."""
    import os

    import torch

    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import paper_2307_16080_amd as mlk
    from paper_2307_16080_amd import _lib as L
    from workloads import resnet18_conv_stack

    def graph_us(fn, n=10, replays=10):
        fn()
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            for _ in range(n):
                fn()
        g.replay()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(replays):
            g.replay()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e3 / (n * replays)

    calls = []
    for shape, count in resnet18_conv_stack(batch):
        p = mlk.conv_problem(shape.N, shape.C, shape.H, shape.W, shape.F, shape.KH, shape.KW, shape.stride,
                             shape.pad, L.MLK_BF16, L.MLK_F32)
        _, _, t = mlk.tune(p, mlk.MLK_TUNE_EXHAUSTIVE, reps=3, warmup=1, want_times=True)
        qx, _ = mlk.quantize(torch.randn(shape.N, shape.C, shape.H, shape.W, device="cuda"), "bf16")
        qw, _ = mlk.quantize(torch.randn(shape.F, shape.C, shape.KH, shape.KW, device="cuda"), "bf16")
        ho, wo = shape.out_hw()
        y = torch.zeros(shape.N, shape.F, ho, wo, device="cuda")
        # as the benchmark picks: the table's six fastest and the two fastest of
        # each conv layout, re-timed as bound calls in graphs
        cfgs = mlk.configs(p)
        ranked = [i for _, i in sorted((v, i) for i, v in enumerate(t) if v > 0)]
        order = ranked[:6]
        for lay in sorted({cfgs[i].layout for i in ranked}):
            order += [i for i in ranked if cfgs[i].layout == lay and i not in order][:2]
        cands = [mlk.ConvCall(qx, qw, y, (shape.stride,) * 2, (shape.pad,) * 2, cfg=cfgs[i]) for i in order]
        us = [graph_us(c) for c in cands]
        k = min(range(len(us)), key=lambda j: us[j])
        calls += [cands[k]] * count
        print(f"layer {shape}: tile {list(cfgs[order[k]].as_tuple())} {us[k]:.2f} us", flush=True)
    torch.cuda.synchronize()
    if graph:
        for call in calls:      # first runs (plan set-up) outside the capture
            call()
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            for call in calls:
                call()
        torch.cuda.synchronize()
        for _ in range(launches):
            g.replay()
    else:
        for _ in range(launches):
            for call in calls:
                call()
    torch.cuda.synchronize()
    print(f"resnet18 b{batch}: {launches} {'graph replays' if graph else 'passes'} over {len(calls)} layers",
          flush=True)


def run_conv_batch(batch, tile, launches):
    """The ResNet-18 stack's 19 convolutions (bf16, seeded inputs, each its own
    input and output) as one mlk.ConvBatch with the given configuration
    (eleven comma-separated fields, or "default"), run `launches` times."""
    import os

    import torch

    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import paper_2307_16080_amd as mlk
    from workloads import resnet18_conv_stack

    torch.manual_seed(0)
    convs = []
    for shape, count in resnet18_conv_stack(batch):
        ho, wo = shape.out_hw()
        for _ in range(count):
            qx, _ = mlk.quantize(torch.randn(shape.N, shape.C, shape.H, shape.W, device="cuda"), "bf16")
            qw, _ = mlk.quantize(torch.randn(shape.F, shape.C, shape.KH, shape.KW, device="cuda"), "bf16")
            convs.append((qx, qw, torch.zeros(shape.N, shape.F, ho, wo, device="cuda"), (shape.stride,) * 2,
                          (shape.pad,) * 2))
    cfg = None if tile == "default" else mlk.TileConfig(*[int(v) for v in tile.split(",")])
    cb = mlk.ConvBatch(convs, cfg=cfg)
    for _ in range(launches):
        cb()
    torch.cuda.synchronize()
    c, tasks, wgs = cb.info()
    print(f"conv batch b{batch}: {launches} runs, {list(c.as_tuple())}, {tasks} tasks on {wgs} workgroups",
          flush=True)


if __name__ == "__main__":
    if sys.argv[1] == "gemm":
        run_gemm(sys.argv[2], sys.argv[3], int(sys.argv[4]), *(int(v) for v in sys.argv[5:6]))
    elif sys.argv[1] == "convf32":
        run_conv_f32(sys.argv[2], int(sys.argv[3]))
    elif sys.argv[1] == "resnet":
        run_resnet(int(sys.argv[2]), int(sys.argv[3]), len(sys.argv) > 4 and sys.argv[4] == "graph")
    elif sys.argv[1] == "conv":
        run_conv(sys.argv[2], sys.argv[3], int(sys.argv[4]))
    elif sys.argv[1] == "quantize":
        run_quantize(sys.argv[2], int(sys.argv[3]))
    elif sys.argv[1] == "convbatch":
        run_conv_batch(int(sys.argv[2]), sys.argv[3], int(sys.argv[4]))
    elif sys.argv[1] == "batched":
        run_batched(sys.argv[2], int(sys.argv[3]))
    elif sys.argv[1] == "paperconv":
        run_paper_conv(sys.argv[2], int(sys.argv[3]))
    elif sys.argv[1] == "stats":
        print(stats(sys.argv[2]))
    elif sys.argv[1] == "gemm-summary":
        for t in sys.argv[4:]:
            print(json.dumps(gemm_summary(sys.argv[2], t, sys.argv[3])))
    elif sys.argv[1] == "counters":
        print(json.dumps(counters(sys.argv[2], sys.argv[3])))
    elif sys.argv[1] == "lastpass":
        for p in last_pass(sys.argv[2], int(sys.argv[3]), int(sys.argv[4]) if len(sys.argv) > 4 else 1):
            d = p.pop("dispatches")
            print(json.dumps(p))
            for it in d:
                print(f"  {it['us']:8.2f} us  gap {it['gap_us'] if it['gap_us'] is not None else '-':>6}  {it['kernel']}")
    elif sys.argv[1] == "window":
        d = window(sys.argv[2], sys.argv[3], int(sys.argv[4]), int(sys.argv[5]))
        print(json.dumps({"n": len(d), "avg_us": sum(d) / max(len(d), 1), "min_us": min(d), "max_us": max(d)}))
    elif sys.argv[1] == "traffic":
        t = traffic(sys.argv[2], sys.argv[3], sys.argv[4], int(sys.argv[5]))
        if len(sys.argv) > 7:
            t["source_hash"] = sys.argv[7]
        if len(sys.argv) > 8:
            t["config"] = [int(v) for v in sys.argv[8].split(",")]
        with open(sys.argv[6], "w") as f:
            json.dump(t, f, indent=1)
        print(json.dumps(t))
