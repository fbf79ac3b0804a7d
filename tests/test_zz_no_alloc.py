"""The allocation-free backward (mvp_render_bwd_noalloc) through the C ABI,
against the allocating backward (mvp_render_bwd) of the same forward: two
calls in a row, a full 1024x1024 view (the entry point's maximum) and then
the 8-box 64x64 scene, which is also checked against the FP64 oracle; a
structure above the maximum is rejected without touching the outputs."""
import ctypes as C

import numpy as np
import pytest
import torch

import oracle
from gpu_util import check_grads, say
from paper_2103_01954_amd import _lib as L
from paper_2103_01954_amd import scenes
from paper_2103_01954_amd.api import DevicePrims

pytestmark = pytest.mark.gpu
GROUPS = ("payload", "pos", "rot", "scale")


def _zeros(dp):
    return {"payload": torch.zeros(dp.payload.shape, dtype=torch.float32, device="cuda"),
            "pos": torch.zeros_like(dp.pos), "rot": torch.zeros_like(dp.rot), "scale": torch.zeros_like(dp.scale)}


def _call(fn, ctx, acc, dp, aux, up, g):
    cp = dp.c_struct()
    return fn(ctx.handle, acc.handle, C.byref(cp), aux.data_ptr(), up.data_ptr(), g["payload"].data_ptr(),
              g["pos"].data_ptr(), g["rot"].data_ptr(), g["scale"].data_ptr(), None)


def _both(ctx, w, up_fn):
    """Forward, then the allocating and the allocation-free backward of the
    upstream gradient up_fn(rgba shape); returns (alloc grads, no-alloc grads)."""
    dp = DevicePrims.from_host(w.prims)
    acc = ctx.build_accel(dp, w.cams, w.params)
    rgba, aux = acc.render_fwd(dp)
    up = torch.from_numpy(up_fn(tuple(rgba.shape)).astype(np.float32)).cuda()
    g_ref, g_new = _zeros(dp), _zeros(dp)
    L.check("mvp_render_bwd", _call(ctx.lib.mvp_render_bwd, ctx, acc, dp, aux, up, g_ref))
    L.check("mvp_render_bwd_noalloc", _call(ctx.lib.mvp_render_bwd_noalloc, ctx, acc, dp, aux, up, g_new))
    torch.cuda.synchronize()
    acc.destroy()
    return ({k: v.cpu().numpy().astype(np.float64) for k, v in g_ref.items()},
            {k: v.cpu().numpy().astype(np.float64) for k, v in g_new.items()})


def _same(a, b, what):
    """The two entry points run the same kernels; only the order of the FP32
    device atomics that combine work items may differ."""
    for k in GROUPS:
        d = float(np.abs(a[k] - b[k]).max())
        m = float(np.abs(a[k]).max())
        say(f"  {what} {k}: max |noalloc - alloc| {d:.2e} (max |alloc| {m:.2e})")
        assert d <= 1e-6 * m + 1e-30, (what, k, d, m)


def test_noalloc_backward_matches_the_allocating_one_on_two_calls(mvp_ctx):
    assert L.MVP_NOALLOC_MAX_RAYS == 1024 * 1024
    say("call 1: 4096 primitives, one 1024x1024 view (the maximum)")
    w1 = scenes.c1()
    a1, b1 = _both(mvp_ctx, w1, lambda shape: np.random.default_rng(11).normal(size=shape))
    assert np.abs(a1["payload"]).max() > 0
    _same(a1, b1, "1024^2")
    say("call 2: 8 primitives, 64x64")
    w2 = scenes.c0()
    ref = oracle.render(w2.prims, w2.cams[0], w2.params)
    up = np.random.default_rng(12).normal(size=ref["rgba"].shape)
    up[ref["margin"] < 1e-4] = 0          # rays away from clamp and early-stop decisions
    a2, b2 = _both(mvp_ctx, w2, lambda shape: up.reshape(shape))
    _same(a2, b2, "64^2")
    _, gref = oracle.render_grad(w2.prims, w2.cams[0], w2.params, up)
    check_grads(b2, gref, 1e-4, GROUPS)


def test_noalloc_backward_rejects_more_rays_than_its_scratch(mvp_ctx):
    w = scenes.c0()
    dp = DevicePrims.from_host(w.prims)
    cams = [scenes.look_at_camera(np.random.default_rng(3), 1024, 1024)] * 2   # 2 x 1024^2 rays
    acc = mvp_ctx.build_accel(dp, cams, w.params)
    rgba, aux = acc.render_fwd(dp)
    up = torch.ones_like(rgba)
    g = _zeros(dp)
    st = _call(mvp_ctx.lib.mvp_render_bwd_noalloc, mvp_ctx, acc, dp, aux, up, g)
    assert st == L.MVP_ERR_INVALID
    assert b"exceed" in mvp_ctx.lib.mvp_last_error()
    torch.cuda.synchronize()
    assert all(float(v.abs().max()) == 0.0 for v in g.values())
    acc.destroy()
