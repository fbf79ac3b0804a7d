"""Serving: resident scenes, admission by memory, continuous batching.

Each request's result must be the same rendered alone and rendered in a mix
of concurrent requests (the forward writes every pixel from one thread in a
fixed order, so equality is bit-exact), and equal to the direct render; the
BF16 served image agrees with the plain FP32 forward of the unrounded scene
within the BF16 tolerance."""
import ctypes as C

import numpy as np
import pytest
import torch

import oracle
from gpu_util import max_abs, oracle_pixels, say
from paper_2103_01954_amd import _lib as L
from paper_2103_01954_amd import scenes
from paper_2103_01954_amd.api import Context, DevicePrims
from paper_2103_01954_amd.serve import Server, count_overlapped

pytestmark = pytest.mark.gpu

PARAMS = scenes.MarchParams(1.0 / 512, 1e-6)
TOL_BF16 = 2e-3


def _scene_pool_f32():
    """FP32 scenes; the server holds their BF16 roundings (8^3, 12^3 and 16^3 payloads)."""
    return [scenes.random_box_scene(61, n=8, m=8),
            scenes.noisy_sphere_scene(62, n=256, m=8, scale=0.2, empty_frac=0.7, bf16=False),
            scenes.noisy_sphere_scene(63, n=1024, m=12, scale=0.1, empty_frac=0.7, bf16=False),
            scenes.noisy_sphere_scene(64, n=512, m=16, scale=0.12, empty_frac=0.7, bf16=False)]


def _render_direct(ctx, host, cam, bf16=True, with_counts=False):
    dp = DevicePrims.from_host(host, bf16=bf16)
    acc = ctx.build_accel(dp, [cam], PARAMS)
    rgba, _ = acc.render_fwd(dp, want_aux=False)
    torch.cuda.synchronize()
    counts = tuple(acc.counts())
    acc.destroy()
    return (rgba[0], counts) if with_counts else rgba[0]


@pytest.fixture(scope="module")
def serving():
    ctx = Context(0)
    srv = Server(ctx, budget_bytes=8 << 30, slots=4)
    f32 = _scene_pool_f32()
    hosts = [scenes.as_bf16(h) for h in f32]
    sids = [srv.add_scene(DevicePrims.from_host(h, bf16=True)) for h in hosts]
    yield ctx, srv, hosts, f32, sids
    for s in sids:
        srv.release_scene(s)
    torch.cuda.synchronize()
    ctx.close()


def test_served_bf16_against_the_fp32_forward_and_the_oracle(serving):
    ctx, srv, hosts, f32, sids = serving
    cam = scenes.look_at_camera(np.random.default_rng(70), 256, 256)
    for si in (2, 3):
        out = torch.empty((256, 256, 4), device="cuda")
        t = srv.submit(sids[si], cam, PARAMS, out)
        assert srv.wait(t, 120) == L.MVP_OK
        srv.release(t)
        served = out.cpu().numpy()
        # the same BF16 values rendered by the plain FP32 forward: only the load differs
        same = _render_direct(ctx, hosts[si], cam, bf16=False).cpu().numpy()
        e_same = max_abs(served, same)
        # the plain FP32 forward of the unrounded scene: BF16 quantisation of the payload
        plain = _render_direct(ctx, f32[si], cam, bf16=False).cpu().numpy()
        e_plain = max_abs(served, plain)
        rays = np.random.default_rng(4).choice(256 * 256, 400, replace=False)
        ref = oracle.render(hosts[si], cam, PARAMS, pixels=oracle_pixels(cam, rays))
        e_orc = max_abs(served.reshape(-1, 4)[rays], ref["rgba"])
        ref32 = oracle.render(f32[si], cam, PARAMS, pixels=oracle_pixels(cam, rays))
        e_orc32 = max_abs(plain.reshape(-1, 4)[rays], ref32["rgba"])
        say(f"scene {si} (M={hosts[si].m}): served vs FP32 forward of the same BF16 values {e_same:.2e}, "
            f"vs FP32 forward of the unrounded scene {e_plain:.2e}; served vs oracle {e_orc:.2e}, "
            f"FP32 forward vs oracle {e_orc32:.2e}")
        assert e_same <= 1e-5
        assert e_plain <= TOL_BF16
        assert e_orc <= TOL_BF16
        assert e_orc32 <= 1e-5


def test_alone_equals_mix_equals_direct(serving):
    ctx, srv, hosts, _, sids = serving
    cam_x = scenes.look_at_camera(np.random.default_rng(70), 256, 256)
    out = torch.empty((256, 256, 4), device="cuda")
    t = srv.submit(sids[2], cam_x, PARAMS, out)
    assert srv.wait(t, 120) == L.MVP_OK
    srv.release(t)
    alone = out.clone()
    assert torch.equal(alone, _render_direct(ctx, hosts[2], cam_x))
    # the same request three times inside a mix of 30 over every scene, up to 1920x1080
    reqs = scenes.serving_requests(9, 30, len(sids), resolutions=[(256, 256), (512, 512), (320, 200), (1920, 1080)])
    jobs = []
    for i, (si, cam) in enumerate(reqs):
        if i in (0, 13, 29):
            si, cam = 2, cam_x
        o = torch.empty((cam.height, cam.width, 4), device="cuda")
        jobs.append((si, cam, o, srv.submit(sids[si], cam, PARAMS, o)))
    windows, served_counts = [], []
    for si, cam, o, t in jobs:
        assert srv.wait(t, 120) == L.MVP_OK
        _, t_start, t_done = srv.times(t)
        windows.append((t_start, t_done))
        served_counts.append(srv.samples(t))
        srv.release(t)
    assert sum(1 for si, cam, _, _ in jobs if cam.width == 1920) > 0
    assert len({si for si, _, _, _ in jobs}) == len(sids)
    for (si, cam, o, _), sc in zip(jobs, served_counts):
        direct, counts = _render_direct(ctx, hosts[si], cam, with_counts=True)
        assert torch.equal(o, direct), (si, cam.width, cam.height)
        # the ray- and prim-samples the served forward reports are the direct render's
        assert sc == counts and sc[0] > 0, (si, cam.width, cam.height, sc, counts)
    for i in (0, 13, 29):
        assert torch.equal(jobs[i][2], alone)
    overlapped = count_overlapped(windows)
    say(f"mix: {overlapped} of {len(jobs)} requests overlapped another on the device")
    assert overlapped >= 2


def test_admission_under_a_tiny_budget():
    ctx = Context(0)
    srv = Server(ctx, budget_bytes=48 << 20, slots=4)
    host = scenes.noisy_sphere_scene(62, n=256, m=8, scale=0.2, empty_frac=0.7, bf16=True)
    sid = srv.add_scene(DevicePrims.from_host(host, bf16=True))
    cams = [scenes.look_at_camera(np.random.default_rng(80 + i), 256, 256) for i in range(10)]
    outs = [torch.empty((256, 256, 4), device="cuda") for _ in cams]
    tickets = [srv.submit(sid, c, PARAMS, o) for c, o in zip(cams, outs)]
    # a request whose scratch can never fit in the budget fails instead of blocking the queue
    big_cam = scenes.look_at_camera(np.random.default_rng(99), 1920, 1080)
    big_out = torch.empty((1080, 1920, 4), device="cuda")
    big = srv.submit(sid, big_cam, scenes.MarchParams(1.0 / 4096, 0.0), big_out)
    for t in tickets:
        assert srv.wait(t, 120) == L.MVP_OK
    assert srv.wait(big, 120) == L.MVP_ERR_DEVICE
    assert srv.poll(big)[0] == 3
    # a failed request has no sample counts; a done one has them
    assert srv.ctx.lib.mvp_ticket_samples(ctx.handle, C.c_uint64(big), None, None) == L.MVP_ERR_NOT_READY
    assert srv.samples(tickets[0])[0] > 0
    for c, o in zip(cams, outs):
        assert torch.equal(o, _render_direct(ctx, host, c))
    # more requests after the failure are still served
    t = srv.submit(sid, cams[1], PARAMS, outs[1])
    assert srv.wait(t, 120) == L.MVP_OK
    srv.release(t)
    # scene with pending work cannot be released; unknown tickets are rejected
    t = srv.submit(sid, cams[0], PARAMS, outs[0])
    st = srv.release_scene(sid)
    assert st in (L.MVP_ERR_BUSY, L.MVP_OK)
    if st == L.MVP_ERR_BUSY:
        srv.wait(t, 120)
        assert srv.release_scene(sid) == L.MVP_OK
    with pytest.raises(L.MVPError):
        srv.poll(123456789)
    with pytest.raises(L.MVPError):
        srv.samples(123456789)
    # scenes larger than the budget are refused
    with pytest.raises(L.MVPError):
        srv.add_scene(DevicePrims.from_host(scenes.noisy_sphere_scene(64, n=4096, m=16, scale=0.05,
                                                                      empty_frac=0.7, bf16=True), bf16=True))
    torch.cuda.synchronize()
    ctx.close()


def test_builds_that_do_not_fit_together_take_turns():
    """Under a budget that holds the scene and about one and a half 512^2
    builds, concurrent builds wait for running requests or give way to the
    oldest waiting build instead of waiting on each other; every request
    completes with the direct render's image."""
    ctx = Context(0)
    host = scenes.noisy_sphere_scene(65, n=1024, m=8, scale=0.1, empty_frac=0.7, bf16=True)
    cams = [scenes.look_at_camera(np.random.default_rng(300 + i), 512, 512) for i in range(12)]
    dp = DevicePrims.from_host(host, bf16=True)
    direct, pairs = [], 0
    for c in cams:
        acc = ctx.build_accel(dp, [c], PARAMS)
        rgba, _ = acc.render_fwd(dp, want_aux=False)
        info = acc.info()
        pairs = max(pairs, info["n_ray_pairs"] * 52 + info["n_tile_pairs"] * 20)
        torch.cuda.synchronize()
        direct.append(rgba[0].clone())
        acc.destroy()
    R, N = 512 * 512, host.n
    one_build = R * 12 + N * 100 + (R // 256) * 12 + pairs + (1 << 20)
    scene_bytes = N * 60 + N * 8 ** 3 * 4 * 2 + 1024
    srv = Server(ctx, budget_bytes=scene_bytes + int(1.5 * one_build), slots=4)
    sid = srv.add_scene(dp)
    outs = [torch.empty((512, 512, 4), device="cuda") for _ in cams]
    tickets = [srv.submit(sid, c, PARAMS, o) for c, o in zip(cams, outs)]
    windows = []
    for t in tickets:
        assert srv.wait(t, 120) == L.MVP_OK
        windows.append(srv.times(t)[1:])
        srv.release(t)
    for o, d in zip(outs, direct):
        assert torch.equal(o, d)
    say(f"budget {scene_bytes + int(1.5 * one_build)} B: {count_overlapped(windows)} of {len(cams)} overlapped")
    assert srv.release_scene(sid) == L.MVP_OK
    torch.cuda.synchronize()
    ctx.close()
