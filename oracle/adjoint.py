"""FP64 gradients of the forward march (oracle, test infrastructure).

The paper trains end to end through the ray marcher and notes that the
additive accumulation rule, unlike the multiplicative one, lets the backward
pass avoid storing the full graph of per-sample operations (Sec. 3.2.2); its
details are in a supplemental document that is not available.  The adjoint
below is derived directly from the forward of ``render.py``.

Per ray, let dL/dI = g (3-vector) and dL/dA = h.  Let S be the clamping
sample if the clamp was hit (then A = 1 and T_{S-1} is the opacity before it).
Define the constant
    Tdot = h                 if the clamp was not hit,
    Tdot = -g . (C_S/sigma_S) if it was.
For every processed sample j other than S and every primitive k containing it:
    dL/dsigma_kj = dt (Tdot + g . c_kj),        dL/dc_kj = dt sigma_kj g
and at S:
    dL/dsigma_kS = (1 - T_{S-1}) g . (c_kS - C_S/sigma_S) / sigma_S,
    dL/dc_kS     = (1 - T_{S-1}) (sigma_kS / sigma_S) g.
Samples after the stop contribute nothing.  The early-stop decision and box
membership are piecewise constant and carry no gradient.

Sequential variant: if primitive k* clamps at sample S with T* the opacity
just before it, then I gains c_k*S (1 - T*) and A = 1, so
    Tdot = -g . c_k*S,
every sample before S and every primitive before k* at S take the regular
formulas above, dL/dc_k*S = (1 - T*) g, dL/dsigma_k*S = 0, and the
primitives after k* at S contribute nothing.

The channel adjoints flow to the 8 payload corners through the trilinear
weights, and to the pose through the local coordinate
y = A (x - t), A = diag(1/s) R^T, x = o + tau d:
    dL/dt = -A^T g_y,   dL/dR_mi = g_y,i (x_m - t_m) / s_i,   dL/ds_i = -g_y,i y_i / s_i
where g_y = sum over channels of (channel adjoint) * d(channel)/dy.
"""
from __future__ import annotations

import numpy as np

from .render import combine_mode, fade_window, render

F64 = np.float64


def render_grad(prims, cam, params, grad_rgba, pixels=None, geometry="fp32", background=None):
    """Forward of ``render`` plus the gradient of L = sum(grad_rgba * rgba).

    With a fade window (params.fade_alpha > 0) the payload gradient is with
    respect to the stored payload, i.e. multiplied by the window on the opacity
    channel.  With a background B [R,3] the output colour is I + (1 - A) B, so
    the upstream of I is g and the upstream of A is h - g . B; grads then also
    hold "background" = (1 - A) g.

    Returns (forward dict, grads) where grads has
      payload [N,M,M,M,4], pos [N,3], rot [N,3,3], scale [N,3]  (FP64)."""
    out = render(prims, cam, params, pixels, geometry, _want_grad=True, background=background)
    if background is not None:
        grad_rgba = np.array(grad_rgba, dtype=F64).reshape(-1, 4)
        bgr = np.asarray(background, dtype=F64).reshape(-1, 3)
        a_pm = out["rgba_premultiplied"][:, 3]
        g_bg = (1.0 - a_pm)[:, None] * grad_rgba[:, :3]
        grad_rgba[:, 3] = grad_rgba[:, 3] - np.einsum("ij,ij->i", grad_rgba[:, :3], bgr)
    A32, tr, g_sig, g_col, rb, last_group = out.pop("_internal")
    n, M = prims.n, prims.m
    gpay = np.zeros(n * M * M * M * 4)
    gpos = np.zeros((n, 3))
    grot = np.zeros((n, 3, 3))
    gscale = np.zeros((n, 3))
    grads = {"payload": gpay, "pos": gpos, "rot": grot, "scale": gscale}
    R = out["rgba"].shape[0]
    gr = np.asarray(grad_rgba, dtype=F64).reshape(R, 4)
    ntr = tr["ray"].size
    if background is not None:
        grads["background"] = g_bg
    if ntr == 0:
        grads["payload"] = gpay.reshape(n, M, M, M, 4)
        return out, grads
    dt = float(params.step)

    # per-ray constants
    seq = combine_mode(params) == "sequential"
    ray = tr["ray"]
    val = tr["val"]
    c, sig = val[:, :3], val[:, 3]
    sat = out["t_prev"] >= 0
    tdot = gr[:, 3].copy()
    cbar = np.zeros((R, 3))
    sig_s = np.ones(R)
    for r in np.nonzero(sat)[0]:
        s = last_group[r]
        if seq:
            i = np.nonzero((tr["group"] == s) & (tr["prim"] == out["k_star"][r]))[0][0]
            tdot[r] = -float(gr[r, :3] @ c[i])
        else:
            sig_s[r] = g_sig[s]
            cbar[r] = g_col[s] / g_sig[s]
            tdot[r] = -float(gr[r, :3] @ cbar[r])

    g = gr[ray, :3]
    used = tr["group"] <= last_group[ray]
    at_s = sat[ray] & (tr["group"] == last_group[ray])
    if seq:   # before the clamping primitive: regular steps
        at_s &= tr["prim"] >= out["k_star"][ray]
    regular = used & ~at_s

    adj = np.zeros((ntr, 4))
    gc_dot = np.einsum("ij,ij->i", g, c)
    adj[regular, 3] = dt * (tdot[ray][regular] + gc_dot[regular])
    adj[regular, :3] = dt * sig[regular, None] * g[regular]
    if seq:
        clamp = at_s & (tr["prim"] == out["k_star"][ray])
        adj[clamp, :3] = (1.0 - out["t_star"][ray][clamp])[:, None] * g[clamp]
    elif np.any(at_s):
        w = (1.0 - out["t_prev"][ray][at_s])
        ss = sig_s[ray][at_s]
        adj[at_s, 3] = w * np.einsum("ij,ij->i", g[at_s], c[at_s] - cbar[ray][at_s]) / ss
        adj[at_s, :3] = (w * sig[at_s] / ss)[:, None] * g[at_s]

    # payload: through the trilinear weights
    for corner in range(8):
        base = tr["corner_idx"][:, corner] * 4
        wgt = tr["corner_w"][:, corner]
        for ch in range(4):
            np.add.at(gpay, base + ch, wgt * adj[:, ch])
    grads["payload"] = gpay.reshape(n, M, M, M, 4)
    alpha = float(getattr(params, "fade_alpha", 0.0) or 0.0)
    if alpha != 0.0:
        grads["payload"][..., 3] *= fade_window(M, alpha, float(getattr(params, "fade_beta", 8.0)))[None]

    # pose: through y = diag(1/s) R^T (o + tau d - t)
    gy = np.einsum("ic,icd->id", adj, tr["dval"])                    # [ntr,3]
    k = tr["prim"]
    pos = prims.pos.astype(F64)
    rot = prims.rot.astype(F64)
    s = prims.scale.astype(F64)
    A = np.swapaxes(rot, -1, -2) / s[:, :, None]
    d = out["dirs"].astype(F64)[ray]
    xt = (np.asarray(cam.origin, dtype=F64)[None, :] - pos[k]) + tr["tau"][:, None] * d
    np.add.at(gpos, k, -np.einsum("nij,ni->nj", A[k], gy))
    np.add.at(grot, k, xt[:, :, None] * (gy / s[k])[:, None, :])
    np.add.at(gscale, k, -gy * tr["y"] / s[k])
    return out, grads
