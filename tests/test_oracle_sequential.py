"""Oracle pins for the sequential combine variant (primitives of one sample
accumulated in increasing primitive id, each with its own clamp step) and
its relation to the sum rule (Sec. 3.2.2)."""
import dataclasses
import json
import os

import numpy as np
import pytest

import oracle
from cases import GOLDEN, box_prims, closed_form_camera, load_closed_form
from paper_2103_01954_amd import scenes

SPEC = load_closed_form()
with open(os.path.join(GOLDEN, "sequential_cases.json")) as f:
    SEQ = json.load(f)


def _seq(params):
    return dataclasses.replace(params, combine="sequential")


@pytest.mark.parametrize("case", SEQ["cases"], ids=[c["name"] for c in SEQ["cases"]])
def test_sequential_closed_form(case):
    prims = box_prims(case["boxes"], SPEC["M"])
    cam = closed_form_camera(SPEC)
    params = scenes.MarchParams(case["step"], case["eps"], combine="sequential")
    px, py = SPEC["camera"]["pixel"]
    out = oracle.render(prims, cam, params, pixels=[[py, px]])
    e = case["expected"]
    np.testing.assert_allclose(out["rgba"][0, :3], e["I"], rtol=0, atol=1e-15)
    assert out["rgba"][0, 3] == e["A"]
    assert out["j_end"][0] == e["j_end"] and out["t_prev"][0] == e["t_prev"]
    assert out["k_star"][0] == e["k_star"] and out["t_star"][0] == e["t_star"]


@pytest.mark.parametrize("case", SEQ["cases"], ids=[c["name"] for c in SEQ["cases"]])
def test_sequential_closed_form_gradients(case):
    prims = box_prims(case["boxes"], SPEC["M"])
    cam = closed_form_camera(SPEC)
    params = scenes.MarchParams(case["step"], case["eps"], combine="sequential")
    px, py = SPEC["camera"]["pixel"]
    _, g = oracle.render_grad(prims, cam, params, [[1.0, 0.0, 0.0, 0.0]], pixels=[[py, px]])
    e = case["expected_grad_red"]
    c1 = [k for k, b in enumerate(case["boxes"]) if b["colour"][0] == 1.0][0]
    gp = g["payload"]
    assert gp[c1, ..., 0].sum() == pytest.approx(e["colour_red_c1"], abs=1e-13)
    assert gp[c1, ..., 3].sum() == pytest.approx(e["sigma_c1_box"], abs=1e-13)
    assert gp[1 - c1, ..., 3].sum() == pytest.approx(e["sigma_c2_box"], abs=1e-13)


def _flattened_closed_form(prims, cam, params):
    """With eps = 0 the sequential rule is a clip of every (sample, primitive)
    opacity step to the budget left before it, over the steps in (sample,
    primitive id) order: I = sum_i c_i min(sigma_i dt, max(0, 1 - P_{i-1})),
    P the running sum of sigma_i dt.  Built from the per-sample primitive
    values (brute force over each ray's hit list and all samples)."""
    dt = params.step
    hits = oracle.hit_sets(prims, cam, params)
    full = oracle.render(prims, cam, dataclasses.replace(params, combine="sum"), _want_grad=True)
    _, tr, *_ = full["_internal"]
    R = len(hits)
    out = np.zeros((R, 4))
    for r in range(R):
        sel = np.nonzero(tr["ray"] == r)[0]         # sorted by (j, prim) already
        if sel.size == 0:
            continue
        s = tr["val"][sel, 3] * dt
        c = tr["val"][sel, :3]
        P = np.concatenate([[0.0], np.cumsum(s)[:-1]])
        w = np.minimum(s, np.maximum(0.0, 1.0 - P))
        out[r, :3] = (w[:, None] * c).sum(0)
        out[r, 3] = w.sum()
    return out


def test_sequential_equals_flattened_clip():
    w = scenes.c0()
    params = scenes.MarchParams(w.params.step, 0.0, combine="sequential")
    out = oracle.render(w.prims, w.cams[0], params)
    ref = _flattened_closed_form(w.prims, w.cams[0], params)
    assert (out["t_prev"] >= 0).sum() > 100
    np.testing.assert_allclose(out["rgba"], ref, rtol=0, atol=1e-12)


def test_sequential_matches_sum_rule_off_the_saturating_sample():
    w = scenes.c0()
    cam = w.cams[0]
    a = oracle.render(w.prims, cam, w.params)
    b = oracle.render(w.prims, cam, _seq(w.params))
    ok = a["margin"] > 1e-9
    assert np.array_equal(a["j_end"][ok], b["j_end"][ok])
    np.testing.assert_allclose(b["t_prev"][ok], a["t_prev"][ok], rtol=0, atol=1e-12)
    sat = a["t_prev"] >= 0
    assert sat.sum() > 100 and (~sat).sum() > 100
    np.testing.assert_allclose(b["rgba"][~sat], a["rgba"][~sat], rtol=0, atol=1e-12)
    # clamped rays: equal once the saturating sample's own contribution is
    # taken away from both (everything before it is the same additive sum)
    _, tr_a, gs, gc, _, last_a = oracle.render(w.prims, cam, w.params, _want_grad=True)["_internal"]
    differs = 0
    for r in np.nonzero(sat & ok)[0]:
        s = last_a[r]
        sel = np.nonzero(tr_a["group"] == s)[0]
        tp = a["t_prev"][r]
        sum_part = gc[s] / gs[s] * (1.0 - tp)
        sig = tr_a["val"][sel, 3] * w.params.step
        col = tr_a["val"][sel, :3]
        P = tp + np.concatenate([[0.0], np.cumsum(sig)[:-1]])
        wts = np.minimum(sig, np.maximum(0.0, 1.0 - P))
        seq_part = (wts[:, None] * col).sum(0)
        np.testing.assert_allclose(b["rgba"][r, :3] - seq_part, a["rgba"][r, :3] - sum_part, rtol=0, atol=1e-12)
        differs += int(np.abs(seq_part - sum_part).max() > 1e-6)
    assert differs > 20


def test_one_primitive_per_sample_is_the_sum_rule():
    """Disjoint boxes: every sample holds at most one primitive, so the two
    rules coincide (up to FP64 rounding), clamped rays included."""
    w = scenes.c0()
    cam = w.cams[0]
    out = oracle.render(w.prims, cam, w.params)
    single = out["prim_samples"] == out["ray_samples"]
    b = oracle.render(w.prims, cam, _seq(w.params))
    assert (single & (out["t_prev"] >= 0)).sum() > 50
    np.testing.assert_allclose(b["rgba"][single], out["rgba"][single], rtol=0, atol=1e-12)


def _fd_setup():
    w = scenes.c2_fd()
    p = w.prims
    prims = scenes.Prims(p.pos.astype(np.float64), p.rot.astype(np.float64), p.scale.astype(np.float64),
                         p.payload.astype(np.float64))
    return prims, w.cams[0], _seq(w.params)


def test_sequential_gradients_against_central_differences():
    prims, cam, params = _fd_setup()
    fwd = oracle.render(prims, cam, params, geometry="fp64")
    assert ((fwd["k_star"] >= 0) & (fwd["prim_samples"] > fwd["ray_samples"])).sum() > 5
    up = np.random.default_rng(31).normal(size=fwd["rgba"].shape)
    up[fwd["margin"] < 1e-3] = 0
    _, g = oracle.render_grad(prims, cam, params, up, geometry="fp64")

    def loss(pr):
        return float((oracle.render(pr, cam, params, geometry="fp64")["rgba"] * up).sum())

    gp = g["payload"]
    for ch in (3, 0):
        for idx in np.argsort(-np.abs(gp[..., ch]).ravel())[:3]:
            k, iz, iy, ix = np.unravel_index(idx, gp.shape[:4])
            h = 1e-3
            vals = []
            for sgn in (1, -1):
                pay = prims.payload.copy()
                pay[k, iz, iy, ix, ch] += sgn * h
                vals.append(loss(scenes.Prims(prims.pos, prims.rot, prims.scale, pay)))
            assert (vals[0] - vals[1]) / (2 * h) == pytest.approx(gp[k, iz, iy, ix, ch], rel=1e-6, abs=1e-10)
    for kind in ("pos", "scale"):
        gk = g[kind]
        k = int(np.argmax(np.abs(gk).sum(1)))
        for comp in range(3):
            h = 1e-7     # small: trilinear interpolation has kinks at cell faces
            vals = []
            for sgn in (1, -1):
                arr = getattr(prims, kind).copy()
                arr[k, comp] += sgn * h
                kw = {"pos": prims.pos, "scale": prims.scale}
                kw[kind] = arr
                vals.append(loss(scenes.Prims(kw["pos"], prims.rot, kw["scale"], prims.payload)))
            fd = (vals[0] - vals[1]) / (2 * h)
            assert fd == pytest.approx(gk[k, comp], rel=2e-5, abs=2e-5 * np.abs(gk[k]).max()), (kind, comp)
