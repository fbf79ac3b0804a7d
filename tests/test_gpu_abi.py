"""Error handling and conventions of the C ABI, exercised on the device."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_2103_01954_amd import _lib as L
from paper_2103_01954_amd import scenes
from paper_2103_01954_amd.api import DevicePrims, c_camera, c_params

pytestmark = pytest.mark.gpu


def _setup(ctx):
    w = scenes.c0()
    dp = DevicePrims.from_host(w.prims)
    return w, dp


def test_invalid_arguments_are_rejected_synchronously(mvp_ctx):
    lib, h = mvp_ctx.lib, mvp_ctx.handle
    w, dp = _setup(mvp_ctx)
    cp = dp.c_struct()
    cam = (L.mvp_camera * 1)(c_camera(w.cams[0]))
    acc = C.c_void_p()
    bad = c_params(scenes.MarchParams(0.0, 1e-6))
    assert lib.mvp_build_accel(h, C.byref(cp), cam, 1, C.byref(bad), C.byref(acc), None) == L.MVP_ERR_INVALID
    assert b"step" in lib.mvp_last_error()
    bad = c_params(scenes.MarchParams(1 / 128, 1.0))
    assert lib.mvp_build_accel(h, C.byref(cp), cam, 1, C.byref(bad), C.byref(acc), None) == L.MVP_ERR_INVALID
    ok = c_params(w.params)
    assert lib.mvp_build_accel(h, C.byref(cp), cam, 0, C.byref(ok), C.byref(acc), None) == L.MVP_ERR_INVALID
    cp_bad = dp.c_struct()
    cp_bad.M = 1
    assert lib.mvp_build_accel(h, C.byref(cp_bad), cam, 1, C.byref(ok), C.byref(acc), None) == L.MVP_ERR_INVALID
    cp_bad = dp.c_struct()
    cp_bad.pos = None
    assert lib.mvp_build_accel(h, C.byref(cp_bad), cam, 1, C.byref(ok), C.byref(acc), None) == L.MVP_ERR_INVALID
    cam2 = (L.mvp_camera * 2)(c_camera(w.cams[0]), c_camera(scenes.look_at_camera(np.random.default_rng(0), 32, 32)))
    assert lib.mvp_build_accel(h, C.byref(cp), cam2, 2, C.byref(ok), C.byref(acc), None) == L.MVP_ERR_INVALID
    assert b"resolution" in lib.mvp_last_error()


def test_render_checks_against_the_structure(mvp_ctx):
    lib, h = mvp_ctx.lib, mvp_ctx.handle
    w, dp = _setup(mvp_ctx)
    acc = mvp_ctx.build_accel(dp, w.cams, w.params)
    other = DevicePrims.from_host(scenes.random_box_scene(3, n=5))
    rgba = torch.empty((1, 64, 64, 4), device="cuda")
    cp = other.c_struct()
    assert lib.mvp_render_fwd(h, acc.handle, C.byref(cp), rgba.data_ptr(), None, None) == L.MVP_ERR_INVALID
    cp = dp.c_struct()
    assert lib.mvp_render_fwd(h, acc.handle, C.byref(cp), None, None, None) == L.MVP_ERR_INVALID
    assert lib.mvp_render_bwd(h, acc.handle, C.byref(cp), None, rgba.data_ptr(), None, None, None, None,
                              None) == L.MVP_ERR_INVALID
    # misaligned payload
    cp.payload = dp.payload.data_ptr() + 4
    assert lib.mvp_render_fwd(h, acc.handle, C.byref(cp), rgba.data_ptr(), None, None) == L.MVP_ERR_INVALID
    # forward without aux is allowed
    cp = dp.c_struct()
    assert lib.mvp_render_fwd(h, acc.handle, C.byref(cp), rgba.data_ptr(), None, None) == L.MVP_OK
    torch.cuda.synchronize()
    assert lib.mvp_destroy(h) == L.MVP_ERR_BUSY   # structure still alive
    acc.destroy()


def test_gradients_accumulate_and_null_groups_are_skipped(mvp_ctx):
    w, dp = _setup(mvp_ctx)
    acc = mvp_ctx.build_accel(dp, w.cams, w.params)
    _, aux = acc.render_fwd(dp)
    g = torch.randn((1, 64, 64, 4), device="cuda", generator=torch.Generator("cuda").manual_seed(1))
    once = acc.render_bwd(dp, aux, g)
    twice = acc.render_bwd(dp, aux, g, {k: v.clone() for k, v in once.items()})
    only_pos = acc.render_bwd(dp, aux, g, {"pos": torch.zeros_like(dp.pos)})
    torch.cuda.synchronize()
    # FP32 sums: element-wise within 1e-5 of the group's largest value (the
    # backward without a payload gradient runs another work-item variant, whose
    # per-thread pose sums take the pairs in another order)
    def close(a, b):
        return (a - b).abs().max().item() <= 1e-5 * b.abs().max().item()

    for k in once:
        assert close(twice[k], 2 * once[k]), k
    assert close(only_pos["pos"], once["pos"])
    acc.destroy()


def test_stream_ordering_on_a_side_stream(mvp_ctx):
    w, dp = _setup(mvp_ctx)
    s = torch.cuda.Stream()
    ref_acc = mvp_ctx.build_accel(dp, w.cams, w.params)
    ref, _ = ref_acc.render_fwd(dp)
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        acc = mvp_ctx.build_accel(dp, w.cams, w.params, stream=s)
        out, _ = acc.render_fwd(dp, stream=s)
        acc.destroy(stream=s)
    s.synchronize()
    assert torch.equal(out, ref)
    ref_acc.destroy()


def test_repeated_builds_recycle_memory(mvp_ctx):
    w, dp = _setup(mvp_ctx)
    for _ in range(20):
        acc = mvp_ctx.build_accel(dp, w.cams, w.params)
        acc.render_fwd(dp)
        acc.destroy()
    torch.cuda.synchronize()


def test_kernel_timing_records_each_launch(mvp_ctx):
    w, dp = _setup(mvp_ctx)
    mvp_ctx.timing_start(2)
    try:
        for _ in range(3):        # the third launch of each kernel exceeds the capacity
            acc = mvp_ctx.build_accel(dp, w.cams, w.params)
            rgba, aux = acc.render_fwd(dp)
            acc.render_bwd(dp, aux, torch.ones_like(rgba))
            acc.destroy()
        fwd, bwd = mvp_ctx.timing_read("fwd"), mvp_ctx.timing_read("bwd")
    finally:
        mvp_ctx.timing_stop()
    assert len(fwd) == 2 and len(bwd) == 2
    assert all(0.0 < t < 1000.0 for t in fwd + bwd)
    ms = (C.c_float * 2)()
    n = C.c_int32()
    assert mvp_ctx.lib.mvp_timing_read(mvp_ctx.handle, 7, ms, C.byref(n)) == L.MVP_ERR_INVALID
