"""Client of the library's serving scheduler (mvp_serve_configure / mvp_scene_create /
mvp_submit / mvp_poll): resident scenes, continuous batching, latency stats.

The scheduling itself (admission by memory, slot streams, completion stamps)
runs in the library's host C++ thread; this module only submits requests and
reads their tickets.
"""
from __future__ import annotations

import ctypes as C
import time
from dataclasses import dataclass
from typing import List, Optional

import numpy as np
import torch

from . import _lib as L
from . import scenes
from .api import Context, DevicePrims, c_camera, c_params

STATE = {0: "queued", 1: "running", 2: "done", 3: "failed"}


class Server:
    def __init__(self, ctx: Context, budget_bytes: int = 32 << 30, slots: int = 4):
        self.ctx = ctx
        st = ctx.lib.mvp_serve_configure(ctx.handle, int(budget_bytes), int(slots))
        if st == L.MVP_ERR_BUSY:
            pass   # already configured on this context
        else:
            L.check("mvp_serve_configure", st)

    def add_scene(self, prims: DevicePrims) -> int:
        cp = prims.c_struct()
        sid = C.c_uint64()
        L.check("mvp_scene_create", self.ctx.lib.mvp_scene_create(self.ctx.handle, C.byref(cp), C.byref(sid)))
        return sid.value

    def release_scene(self, sid: int) -> int:
        return self.ctx.lib.mvp_scene_release(self.ctx.handle, C.c_uint64(sid))

    def submit(self, sid: int, cam: scenes.Camera, params: scenes.MarchParams, out: torch.Tensor) -> int:
        assert out.is_contiguous() and out.dtype == torch.float32
        assert out.numel() >= cam.width * cam.height * 4
        req = L.mvp_request(sid, c_camera(cam), c_params(params), out.data_ptr())
        t = C.c_uint64()
        L.check("mvp_submit", self.ctx.lib.mvp_submit(self.ctx.handle, C.byref(req), C.byref(t)))
        return t.value

    def poll(self, ticket: int):
        s, a, b = C.c_int32(), C.c_double(), C.c_double()
        L.check("mvp_poll", self.ctx.lib.mvp_poll(self.ctx.handle, C.c_uint64(ticket), C.byref(s), C.byref(a),
                                                  C.byref(b)))
        return s.value, a.value, b.value

    def times(self, ticket: int):
        """(t_submit, t_start, t_done) of a ticket on the library clock (mvp_clock)."""
        a, b, c = C.c_double(), C.c_double(), C.c_double()
        L.check("mvp_ticket_times", self.ctx.lib.mvp_ticket_times(self.ctx.handle, C.c_uint64(ticket), C.byref(a),
                                                                  C.byref(b), C.byref(c)))
        return a.value, b.value, c.value

    def samples(self, ticket: int):
        """(ray-samples, prim-samples) of a done ticket's forward (mvp_ticket_samples)."""
        a, b = C.c_uint64(), C.c_uint64()
        L.check("mvp_ticket_samples", self.ctx.lib.mvp_ticket_samples(self.ctx.handle, C.c_uint64(ticket),
                                                                      C.byref(a), C.byref(b)))
        return a.value, b.value

    def clock(self) -> float:
        return float(self.ctx.lib.mvp_clock())

    def wait(self, ticket: int, timeout_s: float = 60.0) -> int:
        return self.ctx.lib.mvp_wait(self.ctx.handle, C.c_uint64(ticket), float(timeout_s))

    def release(self, ticket: int):
        L.check("mvp_ticket_release", self.ctx.lib.mvp_ticket_release(self.ctx.handle, C.c_uint64(ticket)))


@dataclass
class Result:
    latency_ms: List[float]     # completion - arrival (closed loop: completion - submission)
    wall_s: float
    n: int
    failed: int
    submit_lag_ms: List[float]  # submission - arrival (the client's own delay)
    overlapped: int             # requests whose [start, done] window overlaps another's
    service_ms: List[float]     # done - start of the build (time on a slot)
    pixels: List[int]           # the request's image size
    ray_samples: List[int]      # ray-samples its forward evaluated


def _run(srv: Server, sids, reqs, params, arrivals: Optional[np.ndarray]) -> Result:
    """Submit requests at the given arrival offsets (None: all at once) and wait
    for all of them.  Latency runs from each request's scheduled arrival on the
    library's clock, so time spent on the client side counts.  Every request
    gets its own output buffer (from torch's caching allocator), so no request
    is held back for want of one."""
    n = len(reqs)
    pending = {}
    lat, lag, windows, serv, pix, rs = [], [], [], [], [], []
    failed = 0
    t0 = srv.clock()
    i = 0
    while i < n or pending:
        now = srv.clock() - t0
        while i < n and (arrivals is None or arrivals[i] <= now):
            si, cam = reqs[i]
            buf = torch.empty((cam.height, cam.width, 4), dtype=torch.float32, device="cuda")
            t = srv.submit(sids[si], cam, params, buf)
            arr = t0 + (arrivals[i] if arrivals is not None else 0.0)
            pending[t] = (buf, arr, cam.width * cam.height)
            i += 1
        for t in list(pending):
            s, _, _ = srv.poll(t)
            if s >= 2:
                _, arr, npx = pending.pop(t)
                ts, tst, td = srv.times(t)
                if s == 2:
                    lat.append((td - (arr if arrivals is not None else ts)) * 1e3)
                    lag.append((ts - arr) * 1e3)
                    windows.append((tst, td))
                    serv.append((td - tst) * 1e3)
                    pix.append(npx)
                    rs.append(srv.samples(t)[0])
                else:
                    failed += 1
                srv.release(t)
        time.sleep(0.0002)
    return Result(lat, srv.clock() - t0, n, failed, lag, count_overlapped(windows), serv, pix, rs)


def count_overlapped(windows) -> int:
    """Number of (start, done) windows that overlap at least one other window."""
    w = sorted(windows)
    hit = [False] * len(w)
    end_max, end_idx = -np.inf, -1
    for i, (a, b) in enumerate(w):
        if a < end_max:
            hit[i] = True
            hit[end_idx] = True
        if b > end_max:
            end_max, end_idx = b, i
    return int(sum(hit))


def poisson_benchmark(ctx: Context, n_requests: int = 1000, seed: int = 5, n_scenes: int = 6,
                      loads=(0.5, 0.8, 0.95), budget_bytes: int = 32 << 30, slots: int = 4,
                      scene_pick=None) -> dict:
    """Resident BF16 scenes of 256..16384 primitives and 8^3..16^3 payloads;
    requests at 256^2..1920x1080.  Measures closed-loop capacity, then an open
    Poisson stream at each of `loads` x capacity; reports p50/p99 latency
    (completion on the device - scheduled arrival, on the library clock) per
    load.  The headline p50/p99 are those at the load closest to 0.8."""
    srv = Server(ctx, budget_bytes, slots)
    specs = scenes.serving_scene_specs(seed=4, count=16)
    specs = [specs[i] for i in scene_pick] if scene_pick is not None else specs[:n_scenes]
    sids = []
    for spec in specs:
        dp = DevicePrims.from_host(scenes.serving_scene(spec), bf16=True)
        sids.append(srv.add_scene(dp))
        del dp
    params = scenes.MarchParams(1.0 / 512, 1e-6)
    reqs = scenes.serving_requests(seed, n_requests, len(sids))
    torch.cuda.synchronize()
    warm = _run(srv, sids, reqs[: min(8, n_requests)], params, None)
    closed = _run(srv, sids, reqs, params, None)
    capacity = (closed.n - closed.failed) / closed.wall_s
    pixels = sum(cam.width * cam.height for _, cam in reqs)
    per_load = []
    failed = closed.failed + warm.failed
    for i, load in enumerate(loads):
        rate = load * capacity
        gaps = np.random.default_rng(seed + 1 + i).exponential(1.0 / rate, size=n_requests)
        arrivals = np.cumsum(gaps) - gaps[0]
        opened = _run(srv, sids, reqs, params, arrivals)
        failed += opened.failed
        lat = np.array(opened.latency_ms)
        lag = np.array(opened.submit_lag_ms)
        serv = np.array(opened.service_ms)
        big = np.array(opened.pixels) == max(opened.pixels) if opened.pixels else np.zeros(0, bool)
        pct = lambda a, q: round(float(np.percentile(a, q)), 3) if a.size else None
        per_load.append({
            "load": load, "offered_fps": round(rate, 1),
            "achieved_fps": round((opened.n - opened.failed) / opened.wall_s, 1),
            "achieved_msamples_s": round(sum(opened.ray_samples) / opened.wall_s / 1e6, 1),
            "p50_ms": round(float(np.percentile(lat, 50)), 3) if lat.size else None,
            "p99_ms": round(float(np.percentile(lat, 99)), 3) if lat.size else None,
            "submit_lag_p99_ms": round(float(np.percentile(lag, 99)), 3) if lag.size else None,
            "overlapped": opened.overlapped,
            # where the tail comes from: time on a slot (build + forward) against
            # waiting, and the largest images against the rest
            "service_p50_ms": pct(serv, 50), "service_p99_ms": pct(serv, 99),
            "largest_p50_ms": pct(lat[big], 50), "largest_p99_ms": pct(lat[big], 99),
            "others_p99_ms": pct(lat[~big], 99), "largest_share": round(float(big.mean()), 3) if big.size else None,
        })
    for s in sids:
        srv.release_scene(s)
    head = min(per_load, key=lambda r: abs(r["load"] - 0.8))
    return {
        "scenes": [{"n": s[0], "m": s[1]} for s in specs],
        "requests_per_load": n_requests, "slots": slots, "budget_gib": budget_bytes / 2 ** 30,
        "capacity_fps": round(capacity, 1),
        "capacity_mpix_s": round(pixels / closed.wall_s / 1e6, 1),
        "capacity_msamples_s": round(sum(closed.ray_samples) / closed.wall_s / 1e6, 1),
        "closed_loop_p50_ms": round(float(np.percentile(closed.latency_ms, 50)), 3) if closed.latency_ms else None,
        "load": head["load"], "p50_ms": head["p50_ms"], "p99_ms": head["p99_ms"],
        "per_load": per_load, "failed": failed,
    }
