"""Throughput of the differentiable ray marcher on one MI355X.

Default workload: 4096 primitives of 8^3 FP32 voxels on a noisy sphere (70%
of voxels transparent), 4 views of 1024x1024, step 1/512, eps_early 1e-6; one
step = culling build + forward march + MSE loss gradient + backward march
(gradients w.r.t. payloads, positions, rotations and scales).  Inputs are
seeded synthetic data resident in device memory before timing starts.

Prints one JSON line.  `value` is ray-samples (samples inside >= 1
intersected primitive, up to the early stop) per second of the whole step.
"""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Msamples/s fwd+bwd at 4096 prims, 1024² px; p50/p99 frame latency served"
HBM_PEAK_GBS = 8000.0
# algorithmic bytes per prim-sample (FP32 payload): forward gathers 8 corners x
# 16 B; backward re-gathers them and scatters 8 x 16 B of FP32 gradients
BYTES_FWD = {"f32": 128, "bf16": 64}
BYTES_BWD = {"f32": 256, "bf16": 192}
KERN_FWD, KERN_BWD = "k_march_fwd", "k_bwd_items"     # the kernels these bytes are charged to


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--size", type=int, default=1024)
    ap.add_argument("--views", type=int, default=4)
    ap.add_argument("--bf16", action="store_true", help="BF16 payload (FP32 accumulation)")
    ap.add_argument("--large", action="store_true",
                    help="the large workload instead: 32768 prims x 16^3 BF16, 2 views 2048^2, step 1/1024")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving latency run")
    ap.add_argument("--serve-requests", type=int, default=1000, help="requests per offered load")
    ap.add_argument("--cpu-rows", type=int, default=32)
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="after timing, run one plain device copy of this many MiB (reference for "
                         "rocprofv3 FETCH_SIZE/WRITE_SIZE scaling)")
    ap.add_argument("--traffic", type=str, default=os.path.join(ROOT, "profiles", "traffic.json"),
                    help="HBM bytes per launch measured by rocprofv3 counters")
    return ap.parse_args()


# ----------------------------------------------------------------------------
# CPU baseline: the oracle on a bounded sample of the same workload
# ----------------------------------------------------------------------------

def _oracle_rows(args):
    """One worker: the oracle's forward and adjoint on whole rows of view 0 of
    the benchmark workload; returns (ray-samples, prim-samples, seconds spent
    in the oracle)."""
    rows, size, views = args
    import oracle
    from paper_2103_01954_amd import scenes
    w = scenes.c2(size=size, views=views)
    cam = w.cams[0]
    rs = ps = 0
    t = 0.0
    for row in rows:
        pix = np.stack([np.full(size, row), np.arange(size)], 1)
        up = np.zeros((size, 4))
        up[:, :3] = 1.0
        t0 = time.perf_counter()
        out, _ = oracle.render_grad(w.prims, cam, w.params, up, pixels=pix)
        t += time.perf_counter() - t0
        rs += int(out["ray_samples"].sum())
        ps += int(out["prim_samples"].sum())
    return rs, ps, t


def cpu_baseline(size, views, n_rows):
    """The oracle (forward + adjoint) on n_rows evenly spaced full rows of view 0,
    one worker process per core; throughput = ray-samples / slowest worker's
    oracle time."""
    rows = [int(r) for r in np.linspace(size // (2 * n_rows), size - size // (2 * n_rows), n_rows)]
    cores = min(len(rows), len(os.sched_getaffinity(0)), 16)
    parts = [rows[i::cores] for i in range(cores)]
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        res = pool.map(_oracle_rows, [(p, size, views) for p in parts])
    wall = time.perf_counter() - t0
    rs = sum(r[0] for r in res)
    busy = max(r[2] for r in res)
    core_s = sum(r[2] for r in res)
    return {"value": rs / busy / 1e6, "unit": "Msamples/s", "cores": cores, "kind": "oracle",
            "one_core_value": rs / core_s / 1e6,
            "sample": f"FP64 NumPy oracle forward+adjoint on {len(rows)} evenly spaced full rows of view 0 "
                      f"({len(rows) * size} rays, {rs} ray-samples), rows dealt to {cores} worker processes; "
                      f"{core_s:.1f} core-s in the oracle, slowest worker {busy:.1f} s, {wall:.1f} s wall "
                      f"with process start-up"}


# ----------------------------------------------------------------------------
# GPU
# ----------------------------------------------------------------------------

def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {a.gpus}); the path shards over rays "
              "across GPUs, which this build does not launch", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2103_01954_amd import scenes
    from paper_2103_01954_amd.api import Context, DevicePrims

    if a.large:
        w = scenes.c4()
        a.bf16, a.size, a.views, a.no_cpu = True, w.cams[0].width, len(w.cams), True
        target = torch.rand((a.views, a.size, a.size, 3), device="cuda",
                            generator=torch.Generator("cuda").manual_seed(107))
        workload = (f"32768 prims x 16^3 bf16 payload (noisy sphere, 80% empty voxels), "
                    f"{a.views} views {a.size}x{a.size}, step 1/1024, eps 1e-6, build+fwd+MSE+bwd")
    else:
        w = scenes.c2(size=a.size, views=a.views)
        target = torch.from_numpy(w.extra["target"]).cuda()
    dtype = "bf16" if a.bf16 else "f32"
    if not a.large:
        workload = (f"4096 prims x 8^3 {dtype} payload (noisy sphere, 70% empty voxels), "
                    f"{a.views} views {a.size}x{a.size}, step 1/512, eps 1e-6, build+fwd+MSE+bwd")
    prims = scenes.as_bf16(w.prims) if a.bf16 and not w.prims.bf16 else w.prims
    ctx = Context(0)
    dp = DevicePrims.from_host(prims, bf16=a.bf16)
    grads = {"payload": torch.zeros(dp.payload.shape, dtype=torch.float32, device="cuda"),
             "pos": torch.zeros_like(dp.pos), "rot": torch.zeros_like(dp.rot),
             "scale": torch.zeros_like(dp.scale)}
    stream = torch.cuda.current_stream()
    n_pix = target.numel()

    def step(ev=None):
        acc = ctx.build_accel(dp, w.cams, w.params)
        if ev: ev[0].record(stream)
        rgba, aux = acc.render_fwd(dp)
        if ev: ev[1].record(stream)
        g = torch.zeros_like(rgba)
        g[..., :3] = (2.0 / n_pix) * (rgba[..., :3] - target)      # d MSE / d I
        for v in grads.values():
            v.zero_()
        if ev: ev[2].record(stream)
        acc.render_bwd(dp, aux, g, grads)
        if ev: ev[3].record(stream)
        return acc

    def note(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    for _ in range(a.warmup):
        step().destroy()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(a.steps)]
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ctx.timing_start(a.steps)      # HIP events around the march kernels themselves
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record(stream)
    last = None
    for i in range(a.steps):
        acc = step(evs[i])
        if last is not None:
            last.destroy()
        last = acc
    stop.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = start.elapsed_time(stop) / a.steps
    note(f"{a.steps} timed steps: {start.elapsed_time(stop) / a.steps:.3f} ms per step")
    ray_s, prim_s = last.counts()
    info = last.info()
    last.destroy()
    fwd_call_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in evs]))
    bwd_call_ms = float(np.mean([e[2].elapsed_time(e[3]) for e in evs]))
    fwd_ms = float(np.mean(ctx.timing_read("fwd")))
    bwd_ms = float(np.mean(ctx.timing_read("bwd")))
    ctx.timing_stop()
    value = ray_s / (ms / 1e3) / 1e6

    kern = KERN_BWD if bwd_ms >= fwd_ms else KERN_FWD
    kms = max(bwd_ms, fwd_ms)
    per = BYTES_BWD[dtype] if kern == KERN_BWD else BYTES_FWD[dtype]
    achieved = prim_s * per / (kms / 1e3) / 1e9
    traffic = None
    if os.path.exists(a.traffic):
        try:
            t = json.load(open(a.traffic))
            key = f"{kern}:{dtype}:{w.prims.n}:{a.size}x{a.views}"
            traffic = t.get(key)
        except Exception:
            traffic = None
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            # DRAM bytes per launch (rocprofv3, profiles/traffic.json) over the same kernel time
            "traffic_gbs": round(traffic / (kms / 1e3) / 1e9, 1) if traffic else None, "kernel": kern,
            "kernel_ms": round(kms, 3), "bytes_per_prim_sample": per,
            "kernel_ms_each": {KERN_FWD: round(fwd_ms, 3), KERN_BWD: round(bwd_ms, 3)},
            "call_ms": {"render_fwd": round(fwd_call_ms, 3), "render_bwd": round(bwd_call_ms, 3)},
            # the whole step (build + forward + backward) against the gather roofline of the
            # forward's and backward's bytes together: prim-samples/s x bytes / HBM peak
            "step_gather_frac": round(prim_s / (ms / 1e3) * (BYTES_FWD[dtype] + BYTES_BWD[dtype]) /
                                      (HBM_PEAK_GBS * 1e9), 4)}

    # a plain device copy: the calibration dispatch for the HBM byte counters
    # (--copy-calib-mib), and the measured copy bandwidth of this GPU
    mib = a.copy_calib_mib or 1024
    src = torch.empty(mib << 18, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 1 if a.copy_calib_mib else 5
    c0.record(stream)
    for _ in range(reps):
        dst.copy_(src)
    c1.record(stream)
    torch.cuda.synchronize()
    copy_gbs = 2.0 * (mib << 20) * reps / (c0.elapsed_time(c1) / 1e3) / 1e9
    del src, dst
    roof["measured_copy_gbs"] = round(copy_gbs, 1)

    serving = None
    if not a.no_serve:
        from paper_2103_01954_amd import serve
        note("serving: 32 GiB budget")
        serving = serve.poisson_benchmark(ctx, n_requests=a.serve_requests, seed=5)
        note("serving: 4 GiB budget")
        # the same request stream on a 4 GiB device budget (1.1 GiB of it resident
        # scenes): a 1920x1080 view of a 16384-primitive scene needs ~1.4 GB of
        # pair lists, so admission by memory makes requests wait for scratch
        small = Context(0)
        try:
            q = serve.poisson_benchmark(small, n_requests=max(a.serve_requests // 4, 50), seed=5, loads=(0.8,),
                                        budget_bytes=4 << 30)
        finally:
            small.close()
        serving["budget_4gib"] = {k: q[k] for k in ("capacity_fps", "p50_ms", "p99_ms", "failed")}
    if not a.no_cpu:
        note("oracle baseline on the host cores")
    cpu = None if a.no_cpu else cpu_baseline(a.size, a.views, a.cpu_rows)

    line = {
        "metric": METRIC, "value": round(value, 2), "unit": "Msamples/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(ms, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": dtype, "data": "synthetic",
        "config": {"workload": workload,
                   "global_batch": a.views, "rays": a.views * a.size * a.size},
        "ray_samples_per_step": ray_s, "prim_samples_per_step": prim_s,
        "mprim_samples_per_s": round(prim_s / (ms / 1e3) / 1e6, 1),
        "prims_per_sample": round(prim_s / max(ray_s, 1), 3),
        "wall_s_timed": round(wall, 3), "accel": info,
        "roofline": roof, "cpu_baseline": cpu, "serving": serving,
    }
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
