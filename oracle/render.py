"""Forward ray march of the volumetric primitives in FP64 (oracle, test infrastructure).

What is computed, following the paper:

* Each primitive k holds a payload V_k of M^3 voxels with colour (3 channels)
  and opacity (1 channel) (Sec. 3.1.2).  The payload is sampled by trilinear
  interpolation (Sec. 3.2.1).  Voxel centres sit at local coordinates
  -1 + 2i/(M-1), so the box faces pass through the outer voxel centres
  ("align corners"); no padding rule is needed.
* For every pixel ray the primitives it intersects are found first, with the
  domain of integration they span; samples are only checked against that
  list (Sec. 3.2.1).  Hit tests and sample membership come from the canonical
  FP32 geometry in ``geometry.py``; the sample points are tau_j = j dt.
* Colour and opacity are accumulated front to back with the additive rule
  (Sec. 3.2.2): I = integral of V_col dT, T(t) = min(integral of V_alpha, 1),
  A = T(t_max).  With one quadrature point per step of width dt, the step
  at sample j with summed opacity density sigma_j and summed opacity-weighted
  colour C_j does
      T + sigma_j dt <= 1 :  T += sigma_j dt,  I += C_j dt
      otherwise (clamp)   :  I += (C_j / sigma_j)(1 - T),  T = 1
  and the march stops after a sample once T > 1 - eps_early (Sec. 3.2.2).
  Once the clamp is hit no later sample can change I or T, so the march also
  stops there.
* A sample inside several primitives combines them by the sum rule:
  sigma_j = sum_k sigma_kj and C_j = sum_k sigma_kj c_kj, i.e. the global
  colour/opacity field of Sec. 3.2.2.  This is what accumulating the
  primitives one after another gives up to the saturation point, and it does
  not depend on the order of the primitive list.
* Variant (``params.combine == "sequential"``): the primitives containing a
  sample are accumulated one after another in increasing primitive id, each
  with its own clamp step, as when the primitives are visited in a fixed
  traversal order instead of being merged into one field (Sec. 3.2.2 notes
  that both readings coincide up to saturation).  A sample whose summed step
  does not saturate gives exactly the sum rule; at the saturating sample the
  primitives before the clamping one k* add sigma_k c_k dt, k* adds
  c_k* (1 - T) and later ones nothing.
* Outputs per ray: I (premultiplied colour, the integral as written), A, the
  index of the last sample processed and, if the clamp was hit there, the
  value of T before it (and, for the sequential variant, the clamping
  primitive and T just before it).

Values are FP64: the local coordinate of a sample is y = a + tau b evaluated in
FP64 from the canonical FP32 local ray (a, b) of ``geometry.py`` (or from an
all-FP64 local ray with ``geometry="fp64"``, used for finite differences).
"""
from __future__ import annotations

import numpy as np

from . import geometry as G

F32 = np.float32
F64 = np.float64


# ----------------------------------------------------------------------------
# trilinear payload sampling
# ----------------------------------------------------------------------------

def trilinear(payload: np.ndarray, k: np.ndarray, y: np.ndarray, want_grad: bool = False):
    """Sample payload[k] (layout [N][iz][iy][ix][c]) at local coordinates y [n,3].

    Returns values [n,4] (FP64).  With want_grad also returns the flat voxel
    index of the 8 corners [n,8], their weights [n,8] and dvalue/dy [n,4,3]."""
    M = payload.shape[1]
    yc = np.clip(y, -1.0, 1.0)
    u = (yc + 1.0) * 0.5 * (M - 1)
    i0 = np.clip(np.floor(u), 0, M - 2).astype(np.int64)
    f = u - i0
    n = y.shape[0]
    vals = np.zeros((n, 4))
    if want_grad:
        corner_idx = np.empty((n, 8), dtype=np.int64)
        corner_w = np.empty((n, 8))
        dval = np.zeros((n, 4, 3))
    c = 0
    for dz in (0, 1):
        wz = f[:, 2] if dz else 1.0 - f[:, 2]
        sz = 1.0 if dz else -1.0
        for dy in (0, 1):
            wy = f[:, 1] if dy else 1.0 - f[:, 1]
            sy = 1.0 if dy else -1.0
            for dx in (0, 1):
                wx = f[:, 0] if dx else 1.0 - f[:, 0]
                sx = 1.0 if dx else -1.0
                iz, iy, ix = i0[:, 2] + dz, i0[:, 1] + dy, i0[:, 0] + dx
                v = payload[k, iz, iy, ix, :].astype(F64)
                w = wx * wy * wz
                vals += w[:, None] * v
                if want_grad:
                    corner_idx[:, c] = ((k * M + iz) * M + iy) * M + ix
                    corner_w[:, c] = w
                    dval[:, :, 0] += (sx * wy * wz)[:, None] * v
                    dval[:, :, 1] += (wx * sy * wz)[:, None] * v
                    dval[:, :, 2] += (wx * wy * sz)[:, None] * v
                c += 1
    if want_grad:
        dval *= 0.5 * (M - 1)          # du/dy
        return vals, corner_idx, corner_w, dval
    return vals


# ----------------------------------------------------------------------------
# ray set-up and per-(ray, primitive) intervals
# ----------------------------------------------------------------------------

def _pixels(cam, pixels):
    if pixels is None:
        py, px = np.meshgrid(np.arange(cam.height), np.arange(cam.width), indexing="ij")
        return py.reshape(-1), px.reshape(-1)
    pixels = np.asarray(pixels, dtype=np.int64).reshape(-1, 2)
    return pixels[:, 0], pixels[:, 1]


def _geometry(prims, cam, params, pixels, geometry):
    """Per ray: direction; per hit pair: ray, prim, t_in, t_out, a, b, jlo, jhi."""
    dt = F32 if geometry == "fp32" else F64
    py, px = _pixels(cam, pixels)
    d = G.pixel_rays(cam.pix2dir, px, py, dtype=dt)
    A = G.local_frame(prims.rot, prims.scale, dtype=dt)
    n = prims.n
    chunk = max(1, (1 << 21) // max(n, 1))
    out = {k: [] for k in ("ray", "prim", "t_in", "t_out", "a", "b")}
    for r0 in range(0, d.shape[0], chunk):
        dd = d[r0:r0 + chunk]
        a, b = G.local_ray(A, prims.pos, cam.origin, dd, dtype=dt)
        hit, t_in, t_out = G.slab(a, b, params.t_near, dtype=dt)
        rr, kk = np.nonzero(hit)
        out["ray"].append(rr + r0)
        out["prim"].append(kk)
        out["t_in"].append(t_in[rr, kk])
        out["t_out"].append(t_out[rr, kk])
        out["a"].append(a[rr, kk])
        out["b"].append(b[rr, kk])
    pairs = {k: (np.concatenate(v) if v else np.zeros(0)) for k, v in out.items()}
    pairs["ray"] = pairs["ray"].astype(np.int64)
    pairs["prim"] = pairs["prim"].astype(np.int64)
    if pairs["a"].size == 0:
        pairs["a"] = np.zeros((0, 3), dtype=dt)
        pairs["b"] = np.zeros((0, 3), dtype=dt)
    pairs["jlo"] = G.first_sample_not_before(pairs["t_in"].astype(dt), params.step, dtype=dt)
    pairs["jhi"] = G.last_sample_not_after(pairs["t_out"].astype(dt), params.step, dtype=dt)
    return d, A, pairs


def hit_sets(prims, cam, params, pixels=None, geometry="fp32"):
    """Sorted primitive ids hit by each ray (the slab test alone)."""
    d, _, pairs = _geometry(prims, cam, params, pixels, geometry)
    order = np.lexsort((pairs["prim"], pairs["ray"]))
    rays, prims_sorted = pairs["ray"][order], pairs["prim"][order]
    bounds = np.searchsorted(rays, np.arange(d.shape[0] + 1))
    return [prims_sorted[bounds[i]:bounds[i + 1]] for i in range(d.shape[0])]


# ----------------------------------------------------------------------------
# samples and accumulation
# ----------------------------------------------------------------------------

def _samples(prims, cam, params, pixels, geometry, want_grad):
    """Expand hit pairs into (ray, prim, j) prim-samples, evaluate the payload,
    and group them by (ray, j) in increasing j."""
    dtype = F32 if geometry == "fp32" else F64
    d, A, pairs = _geometry(prims, cam, params, pixels, geometry)
    keep = pairs["jlo"] <= pairs["jhi"]
    for key in list(pairs):
        pairs[key] = pairs[key][keep]
    cnt = pairs["jhi"] - pairs["jlo"] + 1
    tot = int(cnt.sum())
    pid = np.repeat(np.arange(cnt.size), cnt)
    first = np.cumsum(cnt) - cnt
    j = pairs["jlo"][pid] + (np.arange(tot) - first[pid])
    ray, prim = pairs["ray"][pid], pairs["prim"][pid]
    tau = G.sample_positions(j, params.step, dtype=dtype).astype(F64)
    y = pairs["a"][pid].astype(F64) + tau[:, None] * pairs["b"][pid].astype(F64)
    res = trilinear(prims.payload, prim, y, want_grad)
    vals = res[0] if want_grad else res
    order = np.lexsort((prim, j, ray))
    tr = {"ray": ray[order], "prim": prim[order], "j": j[order], "tau": tau[order],
          "y": y[order], "val": vals[order]}
    if want_grad:
        tr["corner_idx"] = res[1][order]
        tr["corner_w"] = res[2][order]
        tr["dval"] = res[3][order]
    # (ray, j) groups = ray-samples
    if tot:
        new = np.ones(tot, dtype=bool)
        new[1:] = (tr["ray"][1:] != tr["ray"][:-1]) | (tr["j"][1:] != tr["j"][:-1])
        gstart = np.nonzero(new)[0]
    else:
        gstart = np.zeros(0, dtype=np.int64)
    sig = tr["val"][:, 3]
    col = tr["val"][:, :3] * sig[:, None]
    g_sig = np.add.reduceat(sig, gstart) if tot else np.zeros(0)
    g_col = np.add.reduceat(col, gstart, axis=0) if tot else np.zeros((0, 3))
    g_ray = tr["ray"][gstart] if tot else np.zeros(0, dtype=np.int64)
    tr["group"] = np.cumsum(new) - 1 if tot else np.zeros(0, dtype=np.int64)
    ray_bounds = np.searchsorted(g_ray, np.arange(d.shape[0] + 1))
    return d, A, tr, g_sig, g_col, ray_bounds


def accumulate(sig, col, dt, eps):
    """Front-to-back additive accumulation with the clamp and early stop.

    sig[n]: summed opacity density per sample, col[n,3]: summed
    opacity-weighted colour per sample, in increasing sample order.
    Returns I, T, index of the last sample processed (-1 if none), T before
    the clamping sample (-1 if the clamp was not hit), and the smallest
    distance of a branch or stop decision from its threshold."""
    T = 0.0
    I = [0.0, 0.0, 0.0]
    last, t_prev = -1, -1.0
    margin = np.inf
    sig = sig.tolist()
    col = col.tolist()
    for i, (s, c) in enumerate(zip(sig, col)):
        step_t = s * dt
        margin = min(margin, abs(T + step_t - 1.0))
        last = i
        if T + step_t <= 1.0:
            T += step_t
            I = [I[0] + c[0] * dt, I[1] + c[1] * dt, I[2] + c[2] * dt]
        else:
            w = (1.0 - T) / s
            I = [I[0] + c[0] * w, I[1] + c[1] * w, I[2] + c[2] * w]
            t_prev, T = T, 1.0
            break
        if eps > 0:
            margin = min(margin, abs(T - (1.0 - eps)))
        if T > 1.0 - eps:
            break
    return np.array(I), T, last, t_prev, margin


def accumulate_sequential(sig, col, prim, bounds, dt, eps):
    """The sequential variant of ``accumulate``: per-primitive clamp steps in
    increasing primitive id within each sample.

    sig[n], col[n,3]: opacity density and colour (not opacity-weighted) of
    every (sample, primitive) of one ray, ordered by (sample, primitive id);
    prim[n] the primitive ids; bounds[g]..bounds[g+1] the entries of sample
    group g.  Returns I, T, index of the last group processed, T before the
    clamping group (-1 if none), margin, the clamping primitive (-1 if none)
    and T just before it."""
    T = 0.0
    I = [0.0, 0.0, 0.0]
    last, t_prev, k_star, t_star = -1, -1.0, -1, -1.0
    margin = np.inf
    sig = sig.tolist()
    col = col.tolist()
    for g in range(len(bounds) - 1):
        b0, b1 = int(bounds[g]), int(bounds[g + 1])
        last = g
        margin = min(margin, abs(T + sum(sig[b0:b1]) * dt - 1.0))
        t_group = T
        for i in range(b0, b1):
            s, c = sig[i], col[i]
            step_t = s * dt
            margin = min(margin, abs(T + step_t - 1.0))
            if T + step_t <= 1.0:
                T += step_t
                I = [I[0] + s * c[0] * dt, I[1] + s * c[1] * dt, I[2] + s * c[2] * dt]
            else:
                u = 1.0 - T
                I = [I[0] + c[0] * u, I[1] + c[1] * u, I[2] + c[2] * u]
                t_prev, k_star, t_star, T = t_group, int(prim[i]), T, 1.0
                return np.array(I), T, last, t_prev, margin, k_star, t_star
        if eps > 0:
            margin = min(margin, abs(T - (1.0 - eps)))
        if T > 1.0 - eps:
            break
    return np.array(I), T, last, t_prev, margin, k_star, t_star


def combine_mode(params):
    mode = getattr(params, "combine", "sum") or "sum"
    if mode not in ("sum", "sequential"):
        raise ValueError(f"unknown combine rule {mode!r}")
    return mode


def fade_window(M, alpha, beta):
    """Opacity fade window of Sec. 3.1.3 at the voxel centres,
    W(x, y, z) = exp(-alpha (|x|^beta + |y|^beta + |z|^beta)) with (x, y, z) the
    normalised voxel coordinates in [-1, 1]^3; returned as [iz][iy][ix] (FP64)."""
    x = -1.0 + 2.0 * np.arange(M) / (M - 1)
    p = np.abs(x) ** beta
    return np.exp(-alpha * (p[:, None, None] + p[None, :, None] + p[None, None, :]))


def windowed(prims, params):
    """Primitives whose opacity channel is multiplied by the fade window
    (identity when params.fade_alpha is 0 or absent)."""
    alpha = float(getattr(params, "fade_alpha", 0.0) or 0.0)
    if alpha == 0.0:
        return prims
    beta = float(getattr(params, "fade_beta", 8.0))
    pay = prims.payload.astype(F64)
    pay[..., 3] = pay[..., 3] * fade_window(prims.m, alpha, beta)[None]
    return type(prims)(prims.pos, prims.rot, prims.scale, pay, getattr(prims, "bf16", False))


def composite_background(rgba, background):
    """Composite the premultiplied render over a background:
    colour I + (1 - A) B, alpha A."""
    out = rgba.copy()
    out[:, :3] = rgba[:, :3] + (1.0 - rgba[:, 3:4]) * np.asarray(background, dtype=F64).reshape(-1, 3)
    return out


def render(prims, cam, params, pixels=None, geometry="fp32", _want_grad=False, background=None):
    """Render the rays of one camera (all pixels, or the (py, px) list given).

    Returns a dict with
      rgba          [R,4] FP64   premultiplied colour I and alpha A
      j_end         [R]          index j of the last sample processed (-1: none)
      t_prev        [R]          T before the clamping sample, or -1
      ray_samples   [R]          samples inside >= 1 hit primitive, up to the stop
      prim_samples  [R]          (sample, primitive) pairs up to the stop
      margin        [R]          closest distance of a clamp/stop decision to its threshold
      k_star        [R]          clamping primitive of the sequential variant, or -1
      t_star        [R]          T just before k_star (sequential variant), or -1
    """
    seq = combine_mode(params) == "sequential"
    d, A, tr, g_sig, g_col, rb = _samples(windowed(prims, params), cam, params, pixels, geometry, _want_grad)
    R = d.shape[0]
    rgba = np.zeros((R, 4))
    j_end = np.full(R, -1, dtype=np.int64)
    t_prev = np.full(R, -1.0)
    ray_samples = np.zeros(R, dtype=np.int64)
    last_group = np.full(R, -1, dtype=np.int64)
    margin = np.full(R, np.inf)
    k_star = np.full(R, -1, dtype=np.int64)
    t_star = np.full(R, -1.0)
    gfirst = np.searchsorted(tr["group"], np.arange(g_sig.size + 1))   # entries of each group
    gj = tr["j"][gfirst[:-1]] if g_sig.size else np.zeros(0)
    for r in range(R):
        g0, g1 = rb[r], rb[r + 1]
        if g0 == g1:
            continue
        if seq:
            e0, e1 = gfirst[g0], gfirst[g1]
            I, T, last, tp, mg, ks, ts = accumulate_sequential(
                tr["val"][e0:e1, 3], tr["val"][e0:e1, :3], tr["prim"][e0:e1], gfirst[g0:g1 + 1] - e0,
                float(params.step), float(params.eps_early))
            k_star[r], t_star[r] = ks, ts
        else:
            I, T, last, tp, mg = accumulate(g_sig[g0:g1], g_col[g0:g1], float(params.step),
                                            float(params.eps_early))
        rgba[r, :3] = I
        rgba[r, 3] = T
        j_end[r] = gj[g0 + last]
        t_prev[r] = tp
        ray_samples[r] = last + 1
        last_group[r] = g0 + last
        margin[r] = mg
    in_use = tr["group"] <= last_group[tr["ray"]] if tr["ray"].size else np.zeros(0, dtype=bool)
    prim_samples = np.bincount(tr["ray"][in_use], minlength=R) if R else np.zeros(0, dtype=np.int64)
    out = {"rgba": rgba, "j_end": j_end, "t_prev": t_prev, "ray_samples": ray_samples,
           "prim_samples": prim_samples, "margin": margin, "k_star": k_star, "t_star": t_star, "dirs": d}
    if background is not None:
        out["rgba_premultiplied"] = rgba
        out["rgba"] = composite_background(rgba, background)
    if _want_grad:
        out["_internal"] = (A, tr, g_sig, g_col, rb, last_group)
    return out
