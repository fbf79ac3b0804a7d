"""Forward parity of the HIP ray marcher against the FP64 CPU oracle.

Gates: hit sets bit-exact; colour and alpha within 1e-5 max-abs for FP32
payloads and within 2e-3 for BF16 payloads (the oracle is fed the same
BF16-rounded payload values)."""
import numpy as np
import pytest
import torch

import oracle
from cases import box_prims, closed_form_case, load_closed_form
from gpu_util import gpu_forward, hit_lists, max_abs, oracle_pixels, say
from paper_2103_01954_amd import scenes
from paper_2103_01954_amd.api import DevicePrims, aux_fields

pytestmark = pytest.mark.gpu

TOL_F32 = 1e-5
TOL_BF16 = 2e-3
SPEC = load_closed_form()


@pytest.mark.parametrize("case", SPEC["cases"], ids=[c["name"] for c in SPEC["cases"]])
def test_closed_form_cases(mvp_ctx, case):
    prims, cam, params = closed_form_case(SPEC, case)
    say("closed form", case["name"])
    acc, dp, rgba, aux = gpu_forward(mvp_ctx, prims, [cam], params)
    py, px = SPEC["camera"]["pixel"]
    exp = case["expected"]
    j_end, t_prev = aux_fields(aux)
    assert max_abs(rgba[0, py, px, :3], exp["I"]) <= 1e-6
    assert abs(rgba[0, py, px, 3] - exp["A"]) <= 1e-6
    assert j_end[0, py, px] == exp["j_end"]
    assert t_prev[0, py, px] == pytest.approx(exp["t_prev"], abs=1e-6)


def _compare_full(ctx, prims, cam, params, tol, bf16=None, check_hits=True):
    acc, dp, rgba, aux = gpu_forward(ctx, prims, [cam], params, bf16=bf16)
    ref = oracle.render(prims, cam, params)
    err = max_abs(rgba.reshape(-1, 4), ref["rgba"])
    say(f"  max-abs err {err:.3e} over {ref['rgba'].shape[0]} rays, "
        f"{int((ref['ray_samples'] > 0).sum())} covered")
    assert err <= tol
    if check_hits:
        off, ids = acc.debug_hits(dp)
        want = oracle.hit_sets(prims, cam, params)
        bad = [r for r, w in enumerate(want) if not np.array_equal(ids[off[r]:off[r + 1]], w)]
        assert not bad, f"{len(bad)} rays with different hit sets, first {bad[:5]}"
    rs, ps = acc.counts()
    say(f"  samples gpu {rs}/{ps} oracle {ref['ray_samples'].sum()}/{ref['prim_samples'].sum()}")
    assert abs(int(rs) - int(ref["ray_samples"].sum())) <= 1e-4 * ref["ray_samples"].sum() + 2
    assert abs(int(ps) - int(ref["prim_samples"].sum())) <= 1e-4 * ref["prim_samples"].sum() + 2
    j_end, t_prev = aux_fields(aux)
    agree = (j_end.ravel() == ref["j_end"]).mean()
    assert agree > 0.999
    acc.destroy()
    return rgba, ref


def test_c0_fp32(mvp_ctx):
    w = scenes.c0()
    say("c0 fp32")
    rgba, ref = _compare_full(mvp_ctx, w.prims, w.cams[0], w.params, TOL_F32)
    # The same image from an all-FP64 geometry (local frames, rays and sample
    # positions in FP64): the gate above compares against the canonical FP32
    # local ray; this reports what the FP32 geometry itself costs.  Rays whose
    # sample sets differ (a sample within rounding of a box face) are counted
    # apart; on the others the difference is the payload's slope times the
    # FP32 rounding of the sample position.
    f64 = oracle.render(w.prims, w.cams[0], w.params, geometry="fp64")
    same = (f64["ray_samples"] == ref["ray_samples"]) & (f64["prim_samples"] == ref["prim_samples"])
    err_all = max_abs(rgba.reshape(-1, 4), f64["rgba"])
    err_same = max_abs(rgba.reshape(-1, 4)[same], f64["rgba"][same])
    say(f"  vs all-FP64 geometry: max-abs {err_same:.3e} on {int(same.sum())} rays with the same samples, "
        f"{err_all:.3e} over all ({int((~same).sum())} rays with other sample sets)")
    assert err_same <= 1e-3


def test_c0_bf16(mvp_ctx):
    w = scenes.c0(bf16=True)          # payload values are BF16-representable
    say("c0 bf16")
    rgba, ref = _compare_full(mvp_ctx, w.prims, w.cams[0], w.params, TOL_BF16, bf16=True)
    f32 = oracle.render(scenes.c0().prims, w.cams[0], w.params)["rgba"]
    say(f"  error vs the FP32-payload oracle (quantisation): {max_abs(rgba.reshape(-1, 4), f32):.3e}")


def test_ragged_image_and_many_boxes(mvp_ctx):
    """Image size not a multiple of the 16-pixel tile; overlapping boxes."""
    prims = scenes.random_box_scene(31, n=24, m=6, s_lo=0.1, s_hi=0.5)
    cam = scenes.look_at_camera(np.random.default_rng(32), 53, 37)
    say("ragged 53x37, 24 boxes")
    _compare_full(mvp_ctx, prims, cam, scenes.MarchParams(1 / 128, 1e-6), TOL_F32)


def test_odd_step_and_near_plane(mvp_ctx):
    """Step that is not a power of two, a near distance that clips boxes, M=2."""
    prims = scenes.random_box_scene(41, n=12, m=2, s_lo=0.2, s_hi=0.6)
    cam = scenes.look_at_camera(np.random.default_rng(42), 40, 40, dist=1.6)
    say("odd step, t_near, camera inside boxes")
    _compare_full(mvp_ctx, prims, cam, scenes.MarchParams(0.0123, 1e-6, t_near=0.37), TOL_F32)


def test_large_payload_grid(mvp_ctx):
    prims = scenes.random_box_scene(51, n=4, m=16, s_lo=0.3, s_hi=0.5)
    cam = scenes.look_at_camera(np.random.default_rng(52), 48, 48)
    say("M=16")
    _compare_full(mvp_ctx, prims, cam, scenes.MarchParams(1 / 256, 1e-4), TOL_F32)


def test_empty_scene(mvp_ctx):
    w = scenes.c0()
    empty = w.prims.subset(np.zeros(0, dtype=np.int64))
    dp = DevicePrims.from_host(empty)
    acc = mvp_ctx.build_accel(dp, w.cams, w.params)
    rgba, aux = acc.render_fwd(dp)
    torch.cuda.synchronize()
    assert torch.count_nonzero(rgba).item() == 0
    j_end, t_prev = aux_fields(aux)
    assert np.all(j_end == -1)
    assert acc.counts() == (0, 0)
    acc.destroy()


def test_invariants_on_gpu(mvp_ctx):
    w = scenes.c0()
    cam, params = w.cams[0], w.params
    _, _, base, _ = gpu_forward(mvp_ctx, w.prims, [cam], params)
    perm = np.random.default_rng(3).permutation(w.prims.n)
    _, _, permuted, _ = gpu_forward(mvp_ctx, w.prims.subset(perm), [cam], params)
    say(f"permutation max diff {max_abs(permuted, base):.3e}")
    assert max_abs(permuted, base) <= 1e-6
    extra = scenes.random_box_scene(77, n=5, m=8)
    extra.payload[..., 3] = 0
    extra.pos[0] = w.prims.pos[0]
    mixed = scenes.Prims(np.concatenate([extra.pos[:2], w.prims.pos, extra.pos[2:]]),
                         np.concatenate([extra.rot[:2], w.prims.rot, extra.rot[2:]]),
                         np.concatenate([extra.scale[:2], w.prims.scale, extra.scale[2:]]),
                         np.concatenate([extra.payload[:2], w.prims.payload, extra.payload[2:]]))
    _, _, with_zero, _ = gpu_forward(mvp_ctx, mixed, [cam], params)
    say(f"transparent insertion max diff {max_abs(with_zero, base):.3e}")
    assert max_abs(with_zero, base) <= 1e-6
    pay = w.prims.payload.copy()
    pay[..., :3] = np.array([0.1, 0.55, 0.9], np.float32)
    _, _, mono, _ = gpu_forward(mvp_ctx, scenes.Prims(w.prims.pos, w.prims.rot, w.prims.scale, pay), [cam], params)
    m = mono[..., 3] > 1e-3
    ratio = mono[..., :3][m] / mono[..., 3:][m]
    assert np.abs(ratio - np.array([0.1, 0.55, 0.9], np.float32)).max() <= 1e-4


def _sample_rays(cam, n, seed, rgba_alpha=None):
    rng = np.random.default_rng(seed)
    R = cam.width * cam.height
    picks = rng.choice(R, n, replace=False)
    # a dense 16x16 block at the centre and one straddling a tile corner
    cy, cx = cam.height // 2, cam.width // 2
    block = [(y * cam.width + x) for y in range(cy - 8, cy + 8) for x in range(cx + 200, cx + 216)]
    return np.unique(np.concatenate([picks, np.array(block)]))


@pytest.mark.parametrize("bf16", [False, True], ids=["fp32", "bf16"])
def test_c1_full_size_sampled(mvp_ctx, bf16):
    """The 4096-primitive, 1024^2 workload in its benchmark launch configuration;
    the oracle checks sampled rays one by one."""
    w = scenes.c1(bf16=bf16)
    cam, params = w.cams[0], w.params
    say(f"c1 1024^2 {'bf16' if bf16 else 'fp32'}")
    acc, dp, rgba, aux = gpu_forward(mvp_ctx, w.prims, [cam], params, bf16=bf16)
    rays = _sample_rays(cam, 1500, 5)
    ref = oracle.render(w.prims, cam, params, pixels=oracle_pixels(cam, rays))
    got = rgba.reshape(-1, 4)[rays]
    err = max_abs(got, ref["rgba"])
    covered = int((ref["ray_samples"] > 0).sum())
    say(f"  {len(rays)} sampled rays, {covered} covered, max-abs err {err:.3e}")
    assert covered > 300
    assert err <= (TOL_BF16 if bf16 else TOL_F32)
    off, ids = acc.debug_hits(dp)
    want = oracle.hit_sets(w.prims, cam, params, pixels=oracle_pixels(cam, rays))
    for r, wv in zip(rays, want):
        assert np.array_equal(ids[off[r]:off[r + 1]], wv), r
    rs, ps = acc.counts()
    say(f"  whole frame: {rs} ray-samples, {ps} prim-samples, info {acc.info()}")
    acc.destroy()
