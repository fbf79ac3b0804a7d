"""The per-ray pair lists built inside the forward (each workgroup builds its
tile's pairs, then marches them) against the pairs kernel of the build: the
same lists, so the forward and the backward must agree bit for bit, over the
kernel variants (FP32 and BF16 payloads, fade window, sequential combine,
16^3 payloads, ray subsets).  MVP_PAIRS_IN_FORWARD forces either path.  The
forward path is also checked against the oracle where the default choice
does not take it."""
import os

import numpy as np
import pytest
import torch

import oracle
from gpu_util import check_grads, max_abs, say
from paper_2103_01954_amd import scenes
from paper_2103_01954_amd.api import DevicePrims

pytestmark = pytest.mark.gpu
GROUPS = ("payload", "pos", "rot", "scale")


def _run(ctx, prims, cams, params, fused, rays=None, bf16=None):
    os.environ["MVP_PAIRS_IN_FORWARD"] = "1" if fused else "0"
    try:
        dp = DevicePrims.from_host(prims, bf16=bf16)
        acc = ctx.build_accel(dp, cams, params, rays=rays)
        rgba, aux = acc.render_fwd(dp)
        g = torch.zeros_like(rgba)
        g[..., :3] = 0.5 - rgba[..., :3]
        grads = acc.render_bwd(dp, aux, g)
        torch.cuda.synchronize()
        info = acc.info()
        out = {"rgba": rgba.cpu().numpy(), "aux": aux.cpu().numpy(), "pairs": info["n_ray_pairs"]}
        out.update({k: grads[k].cpu().numpy() for k in GROUPS})
        acc.destroy()
        return out
    finally:
        del os.environ["MVP_PAIRS_IN_FORWARD"]


def _same(a, b):
    assert a["pairs"] == b["pairs"]
    for k in ("rgba", "aux") + GROUPS:
        assert np.array_equal(a[k], b[k]), k


CASES = {
    "c0-f32": (lambda: scenes.c0(), {}, None),
    "c0-bf16-fade": (lambda: scenes.c0(bf16=True), {"fade_alpha": 8.0}, True),
    "c0-sequential": (lambda: scenes.c0(), {"combine": "sequential"}, None),
}


@pytest.mark.parametrize("name", list(CASES))
def test_pairs_in_the_forward_equal_the_pairs_kernel(mvp_ctx, name):
    make, over, bf16 = CASES[name]
    w = make()
    p = w.params
    params = scenes.MarchParams(p.step, p.eps_early, fade_alpha=over.get("fade_alpha", 0.0), fade_beta=8.0,
                                combine=over.get("combine", "sum"))
    say(name)
    a = _run(mvp_ctx, w.prims, w.cams, params, True, bf16=bf16)
    b = _run(mvp_ctx, w.prims, w.cams, params, False, bf16=bf16)
    _same(a, b)


def test_pairs_in_the_forward_16cubed_and_subset(mvp_ctx):
    prims = scenes.random_box_scene(91, n=5, m=16, s_lo=0.3, s_hi=0.6)
    cam = scenes.look_at_camera(np.random.default_rng(92), 40, 40)
    params = scenes.MarchParams(1 / 256, 1e-4)
    say("16^3, 40x40")
    _same(_run(mvp_ctx, prims, [cam], params, True), _run(mvp_ctx, prims, [cam], params, False))
    rays = torch.from_numpy(np.random.default_rng(93).choice(40 * 40, 500, replace=False).astype(np.int64)).cuda()
    say("16^3, 500-ray subset")
    _same(_run(mvp_ctx, prims, [cam], params, True, rays=rays), _run(mvp_ctx, prims, [cam], params, False, rays=rays))


def test_pairs_in_the_forward_against_the_oracle(mvp_ctx):
    """The fused path on its own against the FP64 oracle (forward max-abs,
    gradients by the usual gates)."""
    w = scenes.c0()
    cam = w.cams[0]
    out = _run(mvp_ctx, w.prims, [cam], w.params, True)
    ref = oracle.render(w.prims, cam, w.params)
    err = max_abs(out["rgba"].reshape(-1, 4), ref["rgba"])
    say(f"  forward max-abs {err:.3e}")
    assert err <= 1e-5
    up = np.random.default_rng(94).normal(size=ref["rgba"].shape)   # seeded upstream, never from the GPU
    up[ref["margin"] < 1e-4] = 0
    _, gref = oracle.render_grad(w.prims, cam, w.params, up)
    os.environ["MVP_PAIRS_IN_FORWARD"] = "1"
    try:
        dp = DevicePrims.from_host(w.prims)
        acc = mvp_ctx.build_accel(dp, [cam], w.params)
        _, aux = acc.render_fwd(dp)
        grads = acc.render_bwd(dp, aux, torch.from_numpy(up.reshape(1, cam.height, cam.width, 4).astype(np.float32)).cuda())
        torch.cuda.synchronize()
        got = {k: grads[k].cpu().numpy().astype(np.float64).reshape(gref[k].shape) for k in GROUPS}
        acc.destroy()
    finally:
        del os.environ["MVP_PAIRS_IN_FORWARD"]
    check_grads(got, gref, 1e-4, GROUPS)
