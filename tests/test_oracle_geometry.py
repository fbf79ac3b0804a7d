"""Canonical FP32 geometry of the oracle pinned to hand cases and to an
independent point-in-box formulation (paper Sec. 3.1.2: x = R diag(s) y + t;
Sec. 3.2.1: per-ray hit lists and the domain of integration)."""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import geometry as G
from paper_2103_01954_amd import scenes

F32 = np.float32


def test_parallel_axis_inside_and_outside():
    a = np.array([[[0.5, 2.0, 0.0]], [[0.5, 1.0, 0.0]], [[0.5, 1.0000001, 0.0]]], F32)
    b = np.array([[[1.0, 0.0, 0.5]], [[1.0, 0.0, 0.5]], [[1.0, 0.0, 0.5]]], F32)
    hit, t_in, t_out = G.slab(a, b, 0.0)
    assert not hit[0, 0]                 # parallel and outside the slab
    assert hit[1, 0]                     # exactly on the face: closed box
    assert not hit[2, 0]
    assert t_in[1, 0] == 0.0 and t_out[1, 0] == F32(0.5)   # x exits at (1-0.5)/1


def test_near_clip_and_box_behind():
    # camera inside the box: t_in clipped to t_near
    a = np.array([[[0.2, -0.3, 0.1]]], F32)
    b = np.array([[[0.5, 0.25, -1.0]]], F32)
    hit, t_in, t_out = G.slab(a, b, 0.125)
    assert hit[0, 0] and t_in[0, 0] == F32(0.125)
    assert t_out[0, 0] == (F32(-1) - F32(0.1)) / F32(-1.0)
    # box entirely behind the origin
    hit, _, _ = G.slab(np.array([[[0.0, 0.0, 3.0]]], F32), np.array([[[0.0, 0.0, 1.0]]], F32), 0.0)
    assert not hit[0, 0]


def test_one_rounding_per_operation():
    """The slab bounds are fl(fl(+-1 - a)/b), not a fused or reassociated form."""
    rng = np.random.default_rng(0)
    a = rng.uniform(-30, 30, size=(1, 1000, 3)).astype(F32)
    b = rng.uniform(-30, 30, size=(1, 1000, 3)).astype(F32)
    _, t_in, t_out = G.slab(a, b, -np.inf)
    for i in range(0, 1000, 37):
        lo, hi = [], []
        for ax in range(3):
            q0 = F32(F32(-1.0) - a[0, i, ax]) / b[0, i, ax]
            q1 = F32(F32(1.0) - a[0, i, ax]) / b[0, i, ax]
            lo.append(min(q0, q1))
            hi.append(max(q0, q1))
        assert t_in[0, i] == max(lo) and t_out[0, i] == min(hi)


def test_pixel_rays_unit_and_through_pixel_centres():
    cam = scenes.look_at_camera(np.random.default_rng(1), 37, 23)
    py, px = np.meshgrid(np.arange(23), np.arange(37), indexing="ij")
    d = G.pixel_rays(cam.pix2dir, px.ravel(), py.ravel())
    assert d.dtype == F32
    e = (cam.pix2dir.astype(np.float64) @ np.stack([px.ravel() + 0.5, py.ravel() + 0.5,
                                                     np.ones(px.size)])).T
    e /= np.linalg.norm(e, axis=1, keepdims=True)
    np.testing.assert_allclose(d, e, atol=3e-7)
    np.testing.assert_allclose(np.linalg.norm(d.astype(np.float64), axis=1), 1.0, atol=3e-7)


@pytest.mark.parametrize("step", [1 / 128, 1 / 512, 0.001, 0.0123])
def test_sample_ranges_match_brute_force(step):
    """jlo = min{j : fl(j dt) >= t}, jhi = max{j : fl(j dt) <= t} by enumeration."""
    rng = np.random.default_rng(2)
    t = rng.uniform(0, 6, size=400).astype(F32)
    # add values sitting exactly on samples and one ulp either side
    on = (np.arange(40).astype(F32) * F32(7) * F32(step)).astype(F32)
    t = np.concatenate([t, on, np.nextafter(on, F32(np.inf)), np.nextafter(on, F32(-np.inf))])
    jmax = int(7 / step) + 2
    tau = np.arange(jmax).astype(F32) * F32(step)
    lo = G.first_sample_not_before(t, step)
    hi = G.last_sample_not_after(t, step)
    for i in range(t.size):
        ge = np.nonzero(tau >= t[i])[0]
        le = np.nonzero(tau <= t[i])[0]
        assert lo[i] == ge[0]
        assert hi[i] == (le[-1] if le.size else -1)


def _point_in_box(prims, k, x):
    """Independent membership: solve x = R diag(s) y + t for y (FP64)."""
    Rs = prims.rot[k].astype(np.float64) * prims.scale[k].astype(np.float64)[None, :]
    y = np.linalg.solve(Rs, (x - prims.pos[k].astype(np.float64)).T).T
    return np.abs(y).max(axis=-1)


def test_hits_and_membership_agree_with_point_in_box():
    """Every (ray, primitive, sample) the canonical geometry accepts is inside the
    box up to FP32 rounding, and every sample strictly inside is accepted."""
    w = scenes.c0()
    prims, cam, params = w.prims, w.cams[0], w.params
    out = oracle.render(prims, cam, params, _want_grad=True)
    _, tr, *_ = out["_internal"]
    d = out["dirs"].astype(np.float64)
    o = cam.origin.astype(np.float64)
    x = o[None, :] + tr["tau"][:, None] * d[tr["ray"]]
    worst_inside = 0.0
    for k in range(prims.n):
        sel = tr["prim"] == k
        if np.any(sel):
            worst_inside = max(worst_inside, _point_in_box(prims, k, x[sel]).max())
    assert worst_inside <= 1 + 1e-5
    # converse: brute force over all samples of a subset of rays
    accepted = set(zip(tr["ray"].tolist(), tr["prim"].tolist(), tr["j"].tolist()))
    rays = np.nonzero(out["ray_samples"] > 0)[0][::7]
    jmax = int(6 / params.step)
    tau = (np.arange(jmax).astype(F32) * F32(params.step)).astype(np.float64)
    n_inside = 0
    for r in rays:
        for k in range(prims.n):
            m = _point_in_box(prims, k, o[None, :] + tau[:, None] * d[r][None, :])
            for j in np.nonzero(m < 1 - 1e-5)[0]:
                assert (r, k, j) in accepted
                n_inside += 1
            for j in np.nonzero(m > 1 + 1e-5)[0]:
                assert (r, k, j) not in accepted
    assert n_inside > 1000


def test_hit_sets_match_exact_rational_slab():
    """Hit decisions equal an exact rational slab test on the same FP32 inputs,
    except for grazing rays whose exact interval is within FP32 rounding."""
    prims = scenes.random_box_scene(5, n=6, m=2)
    cam = scenes.look_at_camera(np.random.default_rng(9), 12, 12)
    params = scenes.MarchParams(1 / 64, 0.0)
    hits = oracle.hit_sets(prims, cam, params)
    py, px = np.meshgrid(np.arange(12), np.arange(12), indexing="ij")
    P = [[Fraction(float(v)) for v in row] for row in cam.pix2dir]
    o = [Fraction(float(v)) for v in cam.origin]
    disagree = 0
    for r, (yy, xx) in enumerate(zip(py.ravel(), px.ravel())):
        u, v = Fraction(int(xx)) + Fraction(1, 2), Fraction(int(yy)) + Fraction(1, 2)
        e = [P[i][0] * u + P[i][1] * v + P[i][2] for i in range(3)]
        exact = []
        for k in range(prims.n):
            Rm = [[Fraction(float(prims.rot[k, i, j])) for j in range(3)] for i in range(3)]
            s = [Fraction(float(prims.scale[k, i])) for i in range(3)]
            p = [o[m] - Fraction(float(prims.pos[k, m])) for m in range(3)]
            lo, hi = Fraction(0), None
            ok = True
            for i in range(3):   # local axis i: y_i = (R^T (x - t))_i / s_i along the ray o + lam e
                a = sum(Rm[m][i] * p[m] for m in range(3)) / s[i]
                b = sum(Rm[m][i] * e[m] for m in range(3)) / s[i]
                if b == 0:
                    ok = ok and (-1 <= a <= 1)
                    continue
                q0, q1 = (-1 - a) / b, (1 - a) / b
                lo = max(lo, min(q0, q1))
                hi = min(hi, max(q0, q1)) if hi is not None else max(q0, q1)
            if ok and (hi is None or lo <= hi):
                exact.append((k, float(hi - lo) if hi is not None else np.inf))
        got = set(hits[r].tolist())
        want = {k for k, _ in exact}
        for k in got ^ want:
            length = dict(exact).get(k, 0.0)
            assert length < 1e-5, (r, k)
            disagree += 1
    assert disagree <= 2
    assert sum(len(h) for h in hits) > 20
