#!/usr/bin/env python3
"""Throughput of the full Discrete Morse Sandwich pipeline (D0 + D1 + D2) on
one MI355X.

One step = one dms_diagram call on a 512^3 float32 field resident in HBM:
vertex order, gradient + critical cells, critical sorts, D0/D2, D1 and the
sorted pair lists in HBM. Prints ONE JSON line (rank 0) with the throughput in
Mvertices/s, the roofline of the gradient kernel (measured with HIP events on
the library's stream) and the CPU oracle timed on a bounded crop of the same
field.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

WORKLOADS = {
    "smooth512": dict(shape=(512, 512, 512), kind="gaussians", k=64, r=0.005, seed=0,
                      text="512^3 float32, 64 Gaussians + 0.5% uniform noise, seed 0"),
    "noise512": dict(shape=(512, 512, 512), kind="noise", seed=0,
                     text="512^3 float32 i.i.d. uniform noise, seed 0"),
    "smooth256": dict(shape=(256, 256, 256), kind="gaussians", k=32, r=0.01, seed=0,
                      text="256^3 float32, 32 Gaussians + 1% uniform noise, seed 0"),
    "noise256": dict(shape=(256, 256, 256), kind="noise", seed=0,
                     text="256^3 float32 i.i.d. uniform noise, seed 0"),
    # the resolution of the paper's variant curves (Sec. 9.2), for --ablation
    "smooth192": dict(shape=(192, 192, 192), kind="gaussians", k=32, r=0.01, seed=0,
                      text="192^3 float32, 32 Gaussians + 1% uniform noise, seed 0"),
    "noise192": dict(shape=(192, 192, 192), kind="noise", seed=0,
                     text="192^3 float32 i.i.d. uniform noise, seed 0"),
    # 2D grids (nz = 1) at the paper's 2D resolution, 4096^2
    "smooth4096_2d": dict(shape=(1, 4096, 4096), kind="gaussians", k=64, r=0.005, seed=0,
                          text="4096^2 float32 (2D), 64 Gaussians + 0.5% uniform noise, seed 0"),
    "noise4096_2d": dict(shape=(1, 4096, 4096), kind="noise", seed=0,
                         text="4096^2 float32 (2D) i.i.d. uniform noise, seed 0"),
}
METRIC = "Mvertices/s full D0+D1+D2 (512^3 f32), % HBM peak; served req/s + p99"
HBM_PEAK_GBS = 8000.0
# Counters of one gradient-kernel launch on smooth512 (profiles/gradient_hbm_counters_smooth512.md),
# valid for the kernel sources with this hash only: HBM bytes from FETCH_SIZE (x2 calibration) and
# WRITE_SIZE, and the VALU wave instructions issued
GRADIENT_COUNTERS = {"sources_sha256_16": "b910efd99829bc14", "workload": "smooth512",
                     "traffic_bytes": 1609068339 + 6573050368, "valu_wave_insts": 6444384616}
# VALU issue ceiling for the plain (non-packed) 32-bit integer and bit operations the gradient
# kernel runs: the fp64 vector peak, 78.6 TFLOP/s = 2 FLOP x 64 lanes per CU per clock at 256 CUs
# x 2.4 GHz, i.e. 16-lane SIMDs taking 4 cycles per wave64 instruction: one wave64 instruction
# per CU per clock. (The 157.3 TFLOP/s fp32 figure counts packed dual-lane FP32, which this
# build turns off and which integer work cannot use.)
VALU_PEAK_WINST_S = 256 * 2.4e9


def gradient_sources_hash():
    import hashlib
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2206_13932_amd", "csrc")
    h = hashlib.sha256()
    for name in ("gradient.hip", "lower_star.h", "star_tables.h", "dms_device.h"):
        with open(os.path.join(here, name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def make_field(name):
    import synthfields as sf
    w = WORKLOADS[name]
    if w["kind"] == "noise":
        return sf.noise(w["shape"], w["seed"])
    return sf.gaussians(w["shape"], w["seed"], w["k"], w["r"])


def gradient_algorithmic_bytes(V, ncrit):
    """Bytes the gradient kernel must move: read the order (4 B/vertex; the
    neighbours come from cache), write the 26 gradient byte planes, append
    critical ids + packed keys (C0: 4+4, C1, C2, C3: 4+8)."""
    return 4 * V + 26 * V + 8 * ncrit[0] + 12 * (ncrit[1] + ncrit[2] + ncrit[3])


def host_info():
    """The host CPU the CPU lines ran on: model name and usable threads."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": len(os.sched_getaffinity(0))}


def cpu_baseline(field, crop, omp_crop=128, seq_verts=1 << 18):
    """The oracle on the host: the whole pipeline, sequential, on a corner crop
    of the field; and the gradient stage (ProcessLowerStars at every vertex)
    with the vertices shared among OpenMP threads on all host threads, and
    sequentially on its first seq_verts vertices, on a larger crop."""
    import oracle
    if field.shape[0] == 1:  # 2D grid: a square corner crop with as many vertices
        side = int(round(crop ** 1.5))
        sub = field[:, :side, :side].copy()
    else:
        sub = field[:crop, :crop, :crop].copy()
    t0 = time.perf_counter()
    oracle.run(sub)
    dt = time.perf_counter() - t0
    out = {"value": round(sub.size / dt / 1e6, 4), "unit": "Mvertices/s", "cores": 1, "kind": "oracle",
           "sample": f"sequential oracle, whole pipeline on the {'x'.join(map(str, sub.shape[::-1]))} corner "
                     f"crop of the same field ({sub.size} vertices, {dt:.1f} s)",
           "host": host_info()}
    if field.shape[0] > 1:
        g = field[:omp_crop, :omp_crop, :omp_crop].copy()
        rank = oracle.vertex_order(g)
        t_omp, threads = oracle.time_gradient_omp(g.shape, rank, g.size)
        n_seq = min(seq_verts, g.size)
        t_seq = oracle.time_gradient(g.shape, rank, n_seq)
        out["gradient_stage"] = {
            "omp": {"value": round(g.size / t_omp / 1e6, 4), "unit": "Mvertices/s", "cores": threads},
            "sequential": {"value": round(n_seq / t_seq / 1e6, 4), "unit": "Mvertices/s", "cores": 1},
            "sample": f"oracle gradient stage on the {omp_crop}^3 corner crop ({g.size} vertices, {t_omp:.1f} s "
                      f"on {threads} threads); sequential on its first {n_seq} vertices ({t_seq:.1f} s)"}
    return out


def serving_bench(n_requests, rate, plain_sample, calib, sweep_n=512):
    """Continuous batching of a Poisson trace of mixed-size requests (grid
    side log-uniform in [16, 128] per axis, Gaussian mixtures + 1% noise),
    with the batch tile shapes picked by the autotuner on a calibration
    sample; the plain pipeline (one request at a time) on a sample beside."""
    import numpy as np
    import synthfields as sf
    from paper_2206_13932_amd import autotune, serving
    t = time.perf_counter()
    from concurrent.futures import ThreadPoolExecutor
    from threadpoolctl import threadpool_limits
    specs = sf.serving_requests(n_requests, seed=1000, side_range=(16, 128), k=8, noise_frac=0.01, rate=rate)
    # one BLAS thread per field, fields in parallel (numpy releases the GIL)
    with threadpool_limits(1), ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as pool:
        fields = pool.map(lambda s: sf.gaussians(s[1], s[2], 8, 0.01), specs)
        reqs = serving.make_requests(specs, fields)
    real = sum(r.host_field.numel() for r in reqs)
    print(f"[serve] {n_requests} requests ({real / 1e6:.1f} Mvertices) generated in {time.perf_counter() - t:.1f}s",
          file=sys.stderr, flush=True)
    plain = serving.run_plain(reqs[:plain_sample])
    cfg, table = autotune.autotune(reqs[:calib], rate=rate)
    chosen = 0.0
    for c, r in table:
        print(f"[serve] autotune {c}: {r:.0f} req/s", file=sys.stderr, flush=True)
        w, g = c["workers_graph"]
        if (tuple(c["cross"]), c["budget_vertices"], w, g) == (tuple(cfg.cross), cfg.budget_vertices, cfg.workers,
                                                               cfg.use_graph):
            chosen = r

    def at_rate(lam, n):
        """The first n requests with their Poisson arrivals rescaled to rate lam."""
        return [serving.Request(r.rid, r.arrival * rate / lam, r.host_field) for r in reqs[:n]]

    sweeps = {}
    server = serving.Server(cfg)
    try:
        server.warmup(reqs[:calib])
        stats = server.run_trace(reqs)
        # load sweeps: arrival rate as a fraction of the plain pipeline's capacity (one
        # request at a time) and of the server's own measured capacity
        for base_name, mu, n in (("plain", plain, sweep_n), ("server", chosen, 4 * sweep_n)):
            rows = []
            for frac in (0.5, 0.8, 0.95, 1.2):
                lam = frac * mu
                st = server.run_trace(at_rate(lam, n))
                rows.append({"rel": frac, "rate_per_s": round(lam, 1), "requests": n,
                             "req_per_s": round(st.req_per_s, 1), "p50_ms": round(st.pct(50), 2),
                             "p99_ms": round(st.pct(99), 2)})
                print(f"[serve] sweep {base_name} {rows[-1]}", file=sys.stderr, flush=True)
            sweeps[base_name] = {"mu_req_per_s": round(mu, 1), "points": rows}
    finally:
        server.close()
    b = np.array([x[1:4] for x in stats.batches], dtype=np.float64)
    out = {"requests": n_requests, "arrival_rate_per_s": rate, "req_per_s": round(stats.req_per_s, 1),
           "p50_ms": round(stats.pct(50), 2), "p99_ms": round(stats.pct(99), 2),
           "Mvertices_per_s": round(real / stats.wall_s / 1e6, 1),
           "batches": len(stats.batches), "mean_items_per_batch": round(float(b[:, 0].mean()), 1),
           "packing_efficiency": round(float(b[:, 2].sum() / b[:, 1].sum()), 3),
           "tuned": {"cross": list(cfg.cross), "budget_vertices": cfg.budget_vertices,
                     "use_graph": cfg.use_graph, "workers": cfg.workers,
                     "capacity_req_per_s": round(chosen, 1),
                     "best_capacity_req_per_s": round(max(r for _, r in table), 1)},
           "plain_req_per_s": round(plain, 1), "plain_sample": plain_sample, "sweep": sweeps}
    print(f"[serve] {out}", file=sys.stderr, flush=True)
    return out


def transfers_and_copy(ctx, f, steps=3):
    """The same diagram with the field starting in pinned host memory and the
    pair lists ending there (the PCIe copies inside the timed region), and the
    device-to-device copy rate of the GPU (a 1 GiB copy timed with HIP events),
    the practical ceiling of a streaming kernel."""
    import torch
    host = torch.from_numpy(f).pin_memory()
    outs = [None] * 3
    ms = []
    for i in range(steps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        dev = host.to("cuda", non_blocking=True)
        out = ctx.diagram(dev)
        outs = [out[d].to("cpu", non_blocking=True) for d in range(3)]
        torch.cuda.synchronize()
        if i > 0:
            ms.append((time.perf_counter() - t0) * 1e3)
    src = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    src.fill_(1.0)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 10
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    copy_ms = e0.elapsed_time(e1) / reps
    copy_gbs = 2 * src.numel() * 4 / (copy_ms / 1e3) / 1e9
    del src, dst, host, outs
    mean = sum(ms) / len(ms)
    return ({"ms_per_step": round(mean, 3), "Mvertices_per_s": round(f.size / (mean / 1e3) / 1e6, 1),
             "note": "field copied from pinned host memory and the three pair lists back, inside the timed region"},
            {"GB_per_s": round(copy_gbs, 1), "bytes_each_way": 1 << 30, "ms": round(copy_ms, 4),
             "note": "device-to-device copy of 1 GiB (read + write bytes / time), HIP events"})


def workload_bench(name, steps=2, warmup=1):
    """Another workload timed like the headline (dms_diagram on a field in HBM)."""
    import numpy as np
    import torch
    from paper_2206_13932_amd import dms
    f = make_field(name)
    field = torch.from_numpy(f).cuda()
    ctx = dms.Context(0)
    for _ in range(warmup):
        ctx.diagram(field)
    torch.cuda.synchronize()
    stages = []
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.diagram(field)
        stages.append(ctx.stage_ms())
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    st = np.mean(np.array(stages), axis=0).tolist()
    ctx.close()
    del field
    torch.cuda.empty_cache()
    return {"workload": f"{name}: {WORKLOADS[name]['text']}", "steps": steps, "ms_per_step": round(ms, 3),
            "Mvertices_per_s": round(f.size / (ms / 1e3) / 1e6, 3),
            "stage_ms": {k: round(v, 3) for k, v in zip(
                ["order", "gradient_and_counts", "critical_sort", "d0_d2", "d1", "output", "total",
                 "gradient_kernel"], st)}}


def ablation_bench(names=("smooth192", "noise192"), steps=2):
    """The variant curves of Sec. 9.2 on synthetic fields: D1 (PairCriticalSimplices)
    with and without the sandwich and with and without boundary caching, each
    checked to give the plain variant's diagrams. One context per workload (its
    buffers are sized once); the D1 stage is timed with the library's HIP events
    (milliseconds, the mean of `steps` calls after one warmup call)."""
    import numpy as np
    import torch
    from paper_2206_13932_amd import dms
    variants = {"sandwich+cache": [], "no_sandwich": [dms.OPT_D1_NO_SANDWICH], "no_cache": [dms.OPT_D1_NO_CACHE],
                "neither": [dms.OPT_D1_NO_SANDWICH, dms.OPT_D1_NO_CACHE]}
    out = {}
    for name in names:
        field = torch.from_numpy(make_field(name)).cuda()
        ctx = dms.Context(0)
        ref = None
        rows = {}
        for v, opts in variants.items():
            if v == "neither" and WORKLOADS[name]["kind"] == "noise":
                continue  # both off on noise: over the boundary storage already at 128^3
            for o in (dms.OPT_D1_NO_SANDWICH, dms.OPT_D1_NO_CACHE):
                ctx.set_option(o, 1 if o in opts else 0)
            try:
                ctx.diagram(field)
                d1, adds = [], 0
                for _ in range(steps):
                    res = ctx.diagram(field)
                    d1.append(ctx.stage_ms()[4])
                    adds = int(ctx.debug(dms.BUF_STATS, np.uint64)[6])
                pairs = [res[d].cpu().numpy() for d in range(3)]
                if ref is None:
                    ref = pairs
                same = all(np.array_equal(a, b) for a, b in zip(pairs, ref))
                rows[v] = {"d1_ms": round(float(np.mean(d1)), 2), "additions": adds, "same_diagrams": same}
            except dms.DmsError as e:
                rows[v] = {"error": str(e)}
            print(f"[bench] ablation {name} {v}: {rows[v]}", file=sys.stderr, flush=True)
        ctx.close()
        del field
        torch.cuda.empty_cache()
        out[name] = rows
    return out


def differentiation_bench(n_fields=64, side=96):
    """Forward + backward of the loss sum over D1, D2 of (death - birth)^2 on a
    batch of 96^3 fields (16 Gaussians + 2% noise)."""
    import torch
    import synthfields as sf
    from paper_2206_13932_amd import autograd, dms
    ctx = dms.Context(0)
    xs = [torch.from_numpy(sf.gaussians((side, side, side), 5000 + i, 16, 0.02)).cuda() for i in range(n_fields)]
    x = xs[0].clone().requires_grad_(True)
    autograd.d12_squared_persistence(x, ctx).backward()  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for f in xs:
        x = f.requires_grad_(True)
        autograd.d12_squared_persistence(x, ctx).backward()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.close()
    return {"fields": n_fields, "side": side, "fields_per_s": round(n_fields / dt, 1),
            "ms_per_field_fwd_bwd": round(dt * 1e3 / n_fields, 2)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="smooth512", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-crop", type=int, default=80)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=4096, help="0 skips the serving run")
    ap.add_argument("--serve-rate", type=float, default=800.0, help="Poisson arrivals per second")
    ap.add_argument("--serve-plain-sample", type=int, default=512)
    ap.add_argument("--serve-calib", type=int, default=256)
    ap.add_argument("--no-diff", action="store_true", help="skip the differentiation run")
    ap.add_argument("--no-generators", action="store_true", help="skip the 1-cycle generator export")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the transfer-inclusive run and the copy ceiling")
    ap.add_argument("--noise512", action="store_true",
                    help="add the noise512 line (off by default: one run on that field left the GPU faulted "
                         "and the cause is not found yet)")
    ap.add_argument("--ablation", action="store_true",
                    help="only the D1 variant curves (sandwich / caching on and off) on smooth192 and noise192")
    ap.add_argument("--mode", default="diagram", choices=["diagram", "gradient", "counters"],
                    help="gradient: time dms_gradient alone and a 1 GiB device copy "
                         "(the reference kernel for hardware byte counters); counters: "
                         "warmup + steps plain dms_diagram calls, then the same copy")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: the method's pipeline is built and measured on a single "
              f"MI355X (asked for --gpus {args.gpus}).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2206_13932_amd import dms

    if args.ablation:
        print(json.dumps({"mode": "ablation", "unit": "ms (D1 stage)", "curves": ablation_bench()}), flush=True)
        return

    t_gen = time.perf_counter()
    f = make_field(args.workload)
    print(f"[bench] workload={args.workload} shape={f.shape} generated in {time.perf_counter() - t_gen:.1f}s",
          file=sys.stderr, flush=True)
    V = f.size
    dev = torch.device("cuda", 0)
    field = torch.from_numpy(f).to(dev)
    ctx = dms.Context(0)
    torch.cuda.synchronize()

    if args.mode == "gradient":
        for i in range(args.warmup + args.steps):
            ncrit = ctx.gradient(field)
            torch.cuda.synchronize()
        g_ms = ctx.stage_ms()[7]
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev)  # 1 GiB
        dst = torch.empty_like(src)
        src.fill_(1.0)
        dst.copy_(src)
        torch.cuda.synchronize()
        gbytes = gradient_algorithmic_bytes(V, ncrit)
        print(json.dumps({"mode": "gradient", "workload": args.workload, "gradient_kernel_ms": round(g_ms, 4),
                          "algorithmic_bytes": int(gbytes), "n_crit": ncrit,
                          "copy_bytes_each_way": int(src.numel() * 4)}), flush=True)
        ctx.close()
        return

    if args.mode == "counters":
        for i in range(args.warmup + args.steps):
            ctx.diagram(field)
            torch.cuda.synchronize()
            print(f"[bench] diagram {i} ms={ctx.stage_ms()}", file=sys.stderr, flush=True)
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev)  # 1 GiB
        dst = torch.empty_like(src)
        src.fill_(1.0)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"mode": "counters", "workload": args.workload, "stage_ms": ctx.stage_ms(),
                          "copy_bytes_each_way": int(src.numel() * 4)}), flush=True)
        ctx.close()
        return

    for i in range(args.warmup):
        ctx.diagram(field)
        torch.cuda.synchronize()
        print(f"[bench] warmup {i} ms={ctx.stage_ms()}", file=sys.stderr, flush=True)

    grad_ms, stages = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        out = ctx.diagram(field)
        s = ctx.stage_ms()  # events were recorded on the library's stream
        grad_ms.append(s[7])
        stages.append(s)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = V / (ms_per_step / 1e3) / 1e6

    ncrit = ctx.gradient(field)  # counts for the byte model (after the timed region)
    torch.cuda.synchronize()
    nd = [int(out[d].shape[0]) for d in range(3)]
    gbytes = gradient_algorithmic_bytes(V, ncrit)
    g_avg_ms = float(np.mean(grad_ms))
    achieved = gbytes / (g_avg_ms / 1e3) / 1e9
    st = np.mean(np.array(stages), axis=0).tolist()
    print(f"[bench] stage ms (order, gradient+counts, sort, D0D2, D1, output, total, gradient kernel): "
          f"{[round(x, 3) for x in st]}", file=sys.stderr, flush=True)
    print(f"[bench] n_crit={ncrit} pairs={nd}", file=sys.stderr, flush=True)
    ctx.diagram(field)
    stats = ctx.debug(dms.BUF_STATS, np.uint64).tolist()
    print(f"[bench] work counters (D0 steps, evictions, D2 steps, evictions, D1 steps, evictions, adds, "
          f"deferrals, published, restarts): {stats[:10]}; D1 passes (columns, us): {stats[10:20]}; wide (rounds, expanded, moved): {stats[20:23]}; "
          f"wide per column (max us, sum us, max rounds, max adds, max len, n over 1 ms): {stats[23:29]}; "
          f"phases of those (window, slots, loads, sort, low merge, top merge, owner, adds, claims, refill) us: "
          f"{stats[29:39]}, rounds {stats[39]}, adds {stats[40]}; full-merge additions {stats[41]}",
          file=sys.stderr, flush=True)
    lens = (ctx.debug(dms.BUF_D1LEN, np.uint64) & 0xFFFFFF).astype(np.int64)
    if lens.size:
        q = np.percentile(lens, [50, 90, 99, 99.9, 100]).tolist()
        print(f"[bench] D1 cached boundary length p50/p90/p99/p99.9/max: {q}; columns > 1000: "
              f"{int((lens > 1000).sum())}, > 10000: {int((lens > 10000).sum())}", file=sys.stderr, flush=True)

    generators = None
    if not args.no_generators and field.shape[0] > 1:  # 3D only: 2D grids have no sandwich
        # persistent 1-cycle generators of the same diagram: the first export
        # sizes the context's working buffers, the second (after a fresh
        # diagram) is timed, from the call to the cycles in HBM
        ctx.d1_generators()
        ctx.diagram(field)
        torch.cuda.synchronize()
        tg = time.perf_counter()
        goff, gedges = ctx.d1_generators()
        torch.cuda.synchronize()
        gms = (time.perf_counter() - tg) * 1e3
        generators = {"cycles": int(goff.numel() - 1), "edges": int(gedges.numel()), "ms": round(gms, 3)}
        del goff, gedges
        print(f"[bench] generators {generators}", file=sys.stderr, flush=True)

    traffic, valu = None, None
    if (GRADIENT_COUNTERS["workload"] == args.workload
            and GRADIENT_COUNTERS["sources_sha256_16"] == gradient_sources_hash()):
        traffic = GRADIENT_COUNTERS["traffic_bytes"]
        rate = GRADIENT_COUNTERS["valu_wave_insts"] / (g_avg_ms / 1e3)
        valu = {"achieved": round(rate / 1e9, 1), "peak": VALU_PEAK_WINST_S / 1e9, "unit": "G wave-instr/s",
                "frac": round(rate / VALU_PEAK_WINST_S, 4)}
    line = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "Mvertices/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {WORKLOADS[args.workload]['text']}",
                   "n_crit": ncrit, "pairs": nd,
                   "stage_ms": {k: round(v, 3) for k, v in zip(
                       ["order", "gradient_and_counts", "critical_sort", "d0_d2", "d1", "output", "total",
                        "gradient_kernel"], st)}},
        "roofline": {"kernel": "k_gradient",
                     "note": "the kernel with an algorithmic byte and instruction count; by time the D1 workgroup "
                             "pass and the D2 tracer (dependent rounds and gathers, no algorithmic byte count) are "
                             "larger: their fetched-line rates are in profiles/pairing_kernels_counters_smooth512.md",
                     "bound": "hbm", "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "algorithmic_bytes": int(gbytes),
                     "avg_kernel_ms": round(g_avg_ms, 4), "valu_issue": valu},
    }
    if generators is not None:
        line["generators"] = generators
    if not args.no_extras:
        line["with_transfers"], line["copy_ceiling"] = transfers_and_copy(ctx, f)
        print(f"[bench] with transfers {line['with_transfers']}; copy {line['copy_ceiling']}", file=sys.stderr,
              flush=True)
    ctx.close()
    del field, out
    torch.cuda.empty_cache()
    if args.noise512 and not args.no_extras and args.workload == "smooth512":
        # the worst case for the critical-cell count (the paper's "Random"), timed like the headline
        line["noise512"] = workload_bench("noise512")
        print(f"[bench] noise512 {line['noise512']}", file=sys.stderr, flush=True)
    if args.serve_requests > 0:
        line["serving"] = serving_bench(args.serve_requests, args.serve_rate, args.serve_plain_sample,
                                        args.serve_calib)
    if not args.no_diff:
        line["differentiation"] = differentiation_bench()
        print(f"[bench] differentiation {line['differentiation']}", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(f, args.cpu_crop)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    main()
