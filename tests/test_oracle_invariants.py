"""Oracle invariants and a brute-force cross-check of per-sample values.

Sec. 3.2.2: the additive accumulation of the global colour/opacity field is
independent of the order of the primitives up to the saturation point;
transparent primitives contribute nothing; a single colour composites to that
colour."""
import numpy as np
import pytest
from scipy.ndimage import map_coordinates

import oracle
from paper_2103_01954_amd import scenes


def _scene():
    w = scenes.c0()
    return w.prims, w.cams[0], w.params


def test_transparent_primitives_leave_the_image_unchanged():
    prims, cam, params = _scene()
    base = oracle.render(prims, cam, params)["rgba"]
    extra = scenes.random_box_scene(77, n=5, m=8)
    extra.payload[..., 3] = 0
    extra.pos[0] = prims.pos[0]          # one exactly on top of an existing box
    mixed = scenes.Prims(np.concatenate([extra.pos[:2], prims.pos, extra.pos[2:]]),
                         np.concatenate([extra.rot[:2], prims.rot, extra.rot[2:]]),
                         np.concatenate([extra.scale[:2], prims.scale, extra.scale[2:]]),
                         np.concatenate([extra.payload[:2], prims.payload, extra.payload[2:]]))
    out = oracle.render(mixed, cam, params)
    assert np.array_equal(out["rgba"], base)
    assert out["prim_samples"].sum() > oracle.render(prims, cam, params)["prim_samples"].sum()


def test_primitive_order_does_not_matter():
    prims, cam, params = _scene()
    base = oracle.render(prims, cam, params)
    perm = np.random.default_rng(3).permutation(prims.n)
    out = oracle.render(prims.subset(perm), cam, params)
    np.testing.assert_allclose(out["rgba"], base["rgba"], atol=1e-14)
    assert np.array_equal(out["ray_samples"], base["ray_samples"])
    h0 = oracle.hit_sets(prims, cam, params)
    h1 = oracle.hit_sets(prims.subset(perm), cam, params)
    for a, b in zip(h0, h1):
        assert sorted(perm[b].tolist()) == a.tolist()


def test_single_colour_composites_to_that_colour():
    prims, cam, params = _scene()
    pay = prims.payload.copy()
    pay[..., :3] = np.array([0.1, 0.55, 0.9], np.float32)
    out = oracle.render(scenes.Prims(prims.pos, prims.rot, prims.scale, pay), cam, params)["rgba"]
    m = out[:, 3] > 0
    assert m.sum() > 500
    np.testing.assert_allclose(out[m, :3] / out[m, 3:], np.tile([0.1, 0.55, 0.9], (m.sum(), 1)).astype(np.float32),
                               rtol=1e-12)


def test_no_primitives_gives_empty_image():
    prims, cam, params = _scene()
    out = oracle.render(prims.subset(np.zeros(0, dtype=np.int64)), cam, params)
    assert np.all(out["rgba"] == 0) and np.all(out["j_end"] == -1)


def test_alpha_is_bounded_and_clamp_is_exact():
    prims, cam, params = _scene()
    out = oracle.render(prims, cam, params)
    A = out["rgba"][:, 3]
    assert A.max() == 1.0 and A.min() >= 0
    sat = out["t_prev"] >= 0
    assert sat.sum() > 100 and np.all(A[sat] == 1.0)
    assert np.all(out["rgba"][:, :3] <= A[:, None] + 1e-12)   # colours in [0,1]


def test_per_sample_values_match_brute_force_interpolation():
    """For every processed (ray, j): sigma_j and C_j equal sums over all boxes that
    contain the sample (point-in-box in FP64), of scipy's linear interpolation
    of each payload in voxel-index coordinates."""
    prims, cam, params = _scene()
    out = oracle.render(prims, cam, params, _want_grad=True)
    _, tr, g_sig, g_col, rb, last_group = out["_internal"]
    d = out["dirs"].astype(np.float64)
    o = cam.origin.astype(np.float64)
    M = prims.m
    rays = np.nonzero(out["ray_samples"] > 0)[0][::11]
    checked = skipped = 0
    for r in rays:
        for g in range(rb[r], rb[r + 1]):
            j = tr["j"][tr["group"] == g][0]
            tau = float(np.float32(j) * np.float32(params.step))
            x = o + tau * d[r]
            sig, col = 0.0, np.zeros(3)
            ambiguous = False
            for k in range(prims.n):
                Rs = prims.rot[k].astype(np.float64) * prims.scale[k].astype(np.float64)[None, :]
                y = np.linalg.solve(Rs, x - prims.pos[k])
                if abs(np.abs(y).max() - 1) < 1e-5:
                    ambiguous = True      # within FP32 rounding of a face
                if np.abs(y).max() > 1:
                    continue
                u = (y + 1) / 2 * (M - 1)
                coords = np.array([[u[2]], [u[1]], [u[0]]])
                v = [map_coordinates(prims.payload[k, ..., c].astype(np.float64), coords, order=1)[0]
                     for c in range(4)]
                sig += v[3]
                col += v[3] * np.array(v[:3])
            if ambiguous:
                skipped += 1
                continue
            assert g_sig[g] == pytest.approx(sig, abs=5e-5)
            np.testing.assert_allclose(g_col[g], col, atol=5e-5)
            checked += 1
    assert checked > 1000 and skipped < checked / 100
