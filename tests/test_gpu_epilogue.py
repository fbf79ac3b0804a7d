"""GPU parity of the opacity fade window (Sec. 3.1.3) and of the background
composite (Sec. 3.1.4), forward and backward, against the FP64 oracle, for
FP32 and BF16 payloads and for 8^3 and 16^3 payload grids (each combination
runs its own kernel instantiation)."""
import dataclasses

import numpy as np
import pytest
import torch

import oracle
from gpu_util import GROUPS, check_grads, max_abs, oracle_pixels, say
from paper_2103_01954_amd import scenes
from paper_2103_01954_amd.api import DevicePrims

pytestmark = pytest.mark.gpu


def _c0(fade, bf16):
    w = scenes.c0()
    p = w.params
    params = scenes.MarchParams(p.step, p.eps_early, fade_alpha=8.0 if fade else 0.0, fade_beta=8.0)
    prims = scenes.as_bf16(w.prims) if bf16 else w.prims
    return prims, w.cams[0], params


def _m16(fade, bf16):
    """Five large boxes with 16^3 payloads (the LDS gradient of one primitive is
    then 64 KiB of FP32 values), seen at 40x40."""
    prims = scenes.random_box_scene(91, n=5, m=16, s_lo=0.3, s_hi=0.6)
    if bf16:
        prims = scenes.as_bf16(prims)
    cam = scenes.look_at_camera(np.random.default_rng(92), 40, 40)
    params = scenes.MarchParams(1 / 256, 1e-4, fade_alpha=8.0 if fade else 0.0, fade_beta=8.0)
    return prims, cam, params


def _run(ctx, prims, cam, params, bg, seed, fwd_tol, grad_tol):
    R = cam.width * cam.height
    B = np.random.default_rng(seed).random((R, 3)).astype(np.float32) if bg else None
    ref = oracle.render(prims, cam, params, background=B)
    up = np.random.default_rng(seed + 1).normal(size=(R, 4))
    up[ref["margin"] < 1e-4] = 0
    _, gref = oracle.render_grad(prims, cam, params, up, background=B)

    dp = DevicePrims.from_host(prims)
    acc = ctx.build_accel(dp, [cam], params)
    bg_t = torch.from_numpy(B).cuda().reshape(1, cam.height, cam.width, 3) if bg else None
    rgba, aux = acc.render_fwd(dp, background=bg_t)
    g_up = torch.from_numpy(up.astype(np.float32)).cuda().reshape(1, cam.height, cam.width, 4)
    grads = acc.render_bwd(dp, aux, g_up, background=bg_t, rgba=rgba)
    torch.cuda.synchronize()
    err = max_abs(rgba.cpu().numpy().reshape(-1, 4), ref["rgba"])
    say(f"  forward max-abs {err:.2e} (gate {fwd_tol:g})")
    assert err <= fwd_tol
    keys = GROUPS + (("background",) if bg else ())
    got = {k: grads[k].cpu().numpy().astype(np.float64).reshape(gref[k].shape) for k in keys}
    check_grads(got, gref, grad_tol, keys)
    acc.destroy()


@pytest.mark.parametrize("fade,bg,bf16", [(True, False, False), (False, True, False), (True, True, False),
                                          (True, False, True), (True, True, True)],
                         ids=["fade", "background", "fade+background", "bf16+fade", "bf16+fade+background"])
def test_forward_and_backward(mvp_ctx, fade, bg, bf16):
    say(f"c0 fade={fade} bg={bg} bf16={bf16}")
    prims, cam, params = _c0(fade, bf16)
    # BF16 payloads: the oracle gets the same BF16-rounded values, FP32 accumulation on the GPU
    _run(mvp_ctx, prims, cam, params, bg, 5, 2e-3 if bf16 else 1e-5, 1e-3 if bf16 else 1e-4)


@pytest.mark.parametrize("bf16", [False, True], ids=["f32", "bf16"])
def test_fade_with_16cubed_payloads(mvp_ctx, bf16):
    """The fade window in the backward variant used for 16^3 payloads."""
    say(f"16^3 payloads with fade, bf16={bf16}")
    prims, cam, params = _m16(True, bf16)
    _run(mvp_ctx, prims, cam, params, True, 31, 2e-3 if bf16 else 1e-5, 1e-3 if bf16 else 1e-4)


def test_background_on_a_ray_subset(mvp_ctx):
    prims, cam, params = _c0(True, False)
    ids = np.random.default_rng(7).choice(cam.width * cam.height, 700, replace=False)
    B = np.random.default_rng(8).random((ids.size, 3)).astype(np.float32)
    ref = oracle.render(prims, cam, params, pixels=oracle_pixels(cam, ids), background=B)
    dp = DevicePrims.from_host(prims)
    acc = mvp_ctx.build_accel(dp, [cam], params, rays=torch.from_numpy(ids.astype(np.int64)).cuda())
    rgba, _ = acc.render_fwd(dp, background=torch.from_numpy(B).cuda())
    torch.cuda.synchronize()
    assert max_abs(rgba.cpu().numpy(), ref["rgba"]) <= 1e-5
    acc.destroy()
