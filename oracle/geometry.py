"""Canonical FP32 geometry of the ray marcher (oracle, test infrastructure).

The paper casts each pixel ray r(t) = o + t d (Sec. 3.2.2) against oriented
boxes: primitive k has centre t_k, rotation R_k and per-axis scale s_k that
together give its model-to-world transform (Sec. 3.1.2).  The ray marcher
first finds the primitives each ray intersects and their entry/exit distances
(t_min, t_max), then marches only against that list (Sec. 3.2.1).

Which primitives a ray hits and which fixed-step samples fall inside a box are
discrete decisions.  To make them reproducible, they are taken here in IEEE
binary32 with one rounding per written operation (no fused multiply-add, no
reassociation), in this order:

  local frame     is_i = fl(1/s_i),  A_ij = fl(R_ji * is_i)        (A = diag(1/s) R^T)
  pixel ray       e_i = fl(fl(fl(P_i0 u) + fl(P_i1 v)) + P_i2),   u = px + 1/2, v = py + 1/2
                  d_i = fl(e_i / fl(sqrt(fl(fl(e_0 e_0 + e_1 e_1)) + e_2 e_2)))
  local ray       p_m = fl(o_m - t_m)
                  a_i = fl(fl(fl(A_i0 p_0) + fl(A_i1 p_1)) + fl(A_i2 p_2)),  b_i likewise with d
  slab test       b_i == 0: inside iff -1 <= a_i <= 1 (then the axis does not bound t)
                  else q0 = fl(fl(-1 - a_i) / b_i), q1 = fl(fl(1 - a_i) / b_i)
                  t_in = max(min(q0,q1) over i, t_near), t_out = min(max(q0,q1) over i)
                  hit iff t_in <= t_out
  samples         tau_j = fl(j * dt) for integer j in [0, 2^24 - 1]
                  sample j lies in hit primitive k iff t_in <= tau_j <= t_out

(The local box is [-1,1]^3, so s is a half extent; the box is closed.)

With the numpy float32 ufuncs each arithmetic statement below is exactly one
IEEE operation.  An FP64 variant of the same steps is provided for
finite-difference tests, where the pose must be perturbed by tiny amounts.
"""
from __future__ import annotations

import numpy as np

F32 = np.float32
F64 = np.float64
J_MAX = (1 << 24) - 1   # largest sample index whose float32 value j is exact


def local_frame(rot: np.ndarray, scale: np.ndarray, dtype=F32) -> np.ndarray:
    """World-to-local linear map A_k = diag(1/s_k) R_k^T, shape [N,3,3]."""
    rot = np.asarray(rot, dtype=dtype)
    inv_s = dtype(1.0) / np.asarray(scale, dtype=dtype)                   # fl(1/s_i)
    return np.swapaxes(rot, -1, -2) * inv_s[..., :, None]                 # fl(R_ji * is_i)


def pixel_rays(pix2dir: np.ndarray, px: np.ndarray, py: np.ndarray, dtype=F32) -> np.ndarray:
    """Unit ray directions through pixel centres, shape [R,3]."""
    P = np.asarray(pix2dir, dtype=dtype)
    u = np.asarray(px).astype(dtype) + dtype(0.5)
    v = np.asarray(py).astype(dtype) + dtype(0.5)
    e = []
    for i in range(3):
        e.append(((P[i, 0] * u) + (P[i, 1] * v)) + P[i, 2])
    n2 = ((e[0] * e[0]) + (e[1] * e[1])) + (e[2] * e[2])
    nrm = np.sqrt(n2)
    return np.stack([e[0] / nrm, e[1] / nrm, e[2] / nrm], axis=-1)


def local_ray(A: np.ndarray, pos: np.ndarray, origin: np.ndarray, d: np.ndarray, dtype=F32):
    """Local-frame ray y(tau) = a + tau b for every (ray, primitive) pair.

    A [N,3,3], pos [N,3], origin [3], d [R,3] -> a, b of shape [R,N,3]."""
    A = np.asarray(A, dtype=dtype)
    pos = np.asarray(pos, dtype=dtype)
    o = np.asarray(origin, dtype=dtype)
    d = np.asarray(d, dtype=dtype)
    p = o[None, :] - pos                                                   # [N,3]  fl(o - t)
    a = np.empty((d.shape[0], pos.shape[0], 3), dtype=dtype)
    b = np.empty_like(a)
    for i in range(3):
        ai = ((A[:, i, 0] * p[:, 0]) + (A[:, i, 1] * p[:, 1])) + (A[:, i, 2] * p[:, 2])
        a[:, :, i] = ai[None, :]
        bi = ((A[None, :, i, 0] * d[:, None, 0]) + (A[None, :, i, 1] * d[:, None, 1])) \
            + (A[None, :, i, 2] * d[:, None, 2])
        b[:, :, i] = bi
    return a, b


def slab(a: np.ndarray, b: np.ndarray, t_near: float, dtype=F32):
    """Ray/box slab test in the local frame.  Returns (hit, t_in, t_out)."""
    a = np.asarray(a, dtype=dtype)
    b = np.asarray(b, dtype=dtype)
    inf = dtype(np.inf)
    t_in = np.full(a.shape[:-1], dtype(t_near), dtype=dtype)
    t_out = np.full(a.shape[:-1], inf, dtype=dtype)
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        for i in range(3):
            ai, bi = a[..., i], b[..., i]
            q0 = (dtype(-1.0) - ai) / bi
            q1 = (dtype(1.0) - ai) / bi
            parallel = bi == 0
            inside = (ai >= dtype(-1.0)) & (ai <= dtype(1.0))
            lo = np.where(parallel, np.where(inside, -inf, inf), np.minimum(q0, q1))
            hi = np.where(parallel, np.where(inside, inf, -inf), np.maximum(q0, q1))
            t_in = np.maximum(t_in, lo)
            t_out = np.minimum(t_out, hi)
    return t_in <= t_out, t_in, t_out


def sample_positions(j: np.ndarray, step: float, dtype=F32) -> np.ndarray:
    """tau_j = fl(j * dt)."""
    return np.asarray(j).astype(dtype) * dtype(step)


def first_sample_not_before(t: np.ndarray, step: float, dtype=F32) -> np.ndarray:
    """Smallest j >= 0 with tau_j >= t (J_MAX + 1 when there is none).

    Start from ceil(t/dt) in FP64 and move to the exact boundary of the
    rounded sample positions (tau_j is non-decreasing in j)."""
    t = np.asarray(t, dtype=dtype)
    with np.errstate(invalid="ignore", over="ignore"):
        q = np.ceil(t.astype(F64) / F64(dtype(step)))
    q = np.nan_to_num(q, nan=J_MAX + 1, posinf=J_MAX + 1, neginf=0)
    j = np.clip(q, 0, J_MAX + 1).astype(np.int64)
    for _ in range(4):
        back = (j > 0) & (sample_positions(j - 1, step, dtype) >= t)
        j = j - back
    for _ in range(4):
        fwd = (j <= J_MAX) & (sample_positions(j, step, dtype) < t)
        j = j + fwd
    return j


def last_sample_not_after(t: np.ndarray, step: float, dtype=F32) -> np.ndarray:
    """Largest j <= J_MAX with tau_j <= t (-1 when there is none)."""
    t = np.asarray(t, dtype=dtype)
    with np.errstate(invalid="ignore", over="ignore"):
        q = np.floor(t.astype(F64) / F64(dtype(step)))
    q = np.nan_to_num(q, nan=-1, posinf=J_MAX, neginf=-1)
    j = np.clip(q, -1, J_MAX).astype(np.int64)
    for _ in range(4):
        fwd = (j < J_MAX) & (sample_positions(j + 1, step, dtype) <= t)
        j = j + fwd
    for _ in range(4):
        back = (j >= 0) & (sample_positions(j, step, dtype) > t)
        j = j - back
    return j
