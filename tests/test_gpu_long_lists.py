"""Culling lists longer than the LDS sort holds (more than 4096 primitives in
one screen tile): 5000 boxes large enough to cover the whole 48x48 view, so
every tile lists nearly all of them and its list is ordered by the sort over
device memory.  A list that lost or repeated an entry would change the hit
sets and the first samples' sums, so the image and hit sets are checked
against the oracle on sampled rays."""
import time

import numpy as np
import pytest
import torch

import oracle
from gpu_util import max_abs, oracle_pixels, say
from paper_2103_01954_amd import scenes
from paper_2103_01954_amd.api import DevicePrims

pytestmark = pytest.mark.gpu


def test_tile_lists_longer_than_the_lds_sort(mvp_ctx):
    prims = scenes.random_box_scene(41, n=5000, m=2, s_lo=1.0, s_hi=2.0)
    cam = scenes.look_at_camera(np.random.default_rng(42), 48, 48, dist=6.0)
    params = scenes.MarchParams(1 / 16, 1e-6)
    dp = DevicePrims.from_host(prims)
    t0 = time.perf_counter()
    acc = mvp_ctx.build_accel(dp, [cam], params)
    rgba, _ = acc.render_fwd(dp)
    torch.cuda.synchronize()
    info = acc.info()
    say(f"  5000 boxes over 48x48: {info['n_tile_pairs']} list entries in 9 tiles, "
        f"build + forward {1e3 * (time.perf_counter() - t0):.1f} ms")
    assert info["n_tile_pairs"] > 9 * 4096
    rays = np.random.default_rng(43).choice(48 * 48, 24, replace=False)
    pix = oracle_pixels(cam, rays)
    ref = oracle.render(prims, cam, params, pixels=pix)
    err = max_abs(rgba[0].cpu().numpy().reshape(-1, 4)[rays], ref["rgba"])
    say(f"  forward max-abs {err:.3e} on {rays.size} rays")
    assert err <= 1e-5
    off, ids = acc.debug_hits(dp)
    want = oracle.hit_sets(prims, cam, params, pixels=pix)
    for r, w in zip(rays, want):
        assert np.array_equal(ids[off[r]:off[r + 1]], w)
    acc.destroy()
