"""Primitive pose front-end in torch (differentiable; feeds the renderer's R).

The paper models each primitive's transform relative to a base frame from the
guide mesh (Sec. 3.1.2): t = t_hat + delta_t, R = delta_R R_hat,
s = s_hat + delta_s, with delta_R given as an axis-angle (Rodrigues) vector
(Sec. 3.1.2 and the motion decoder of Sec. 3.1.4).  The volume prior of
Sec. 3.3 is lambda_vol * sum_k Prod(s_k).

The renderer takes rotation matrices; these functions build them in torch so
that autograd chains the renderer's dL/dR back to the axis-angle (or
quaternion) parameters.
"""
from __future__ import annotations

import torch


def _skew(v: torch.Tensor) -> torch.Tensor:
    z = torch.zeros_like(v[..., 0])
    return torch.stack([
        torch.stack([z, -v[..., 2], v[..., 1]], -1),
        torch.stack([v[..., 2], z, -v[..., 0]], -1),
        torch.stack([-v[..., 1], v[..., 0], z], -1),
    ], -2)


def rodrigues(r: torch.Tensor) -> torch.Tensor:
    """Axis-angle vectors [...,3] -> rotation matrices [...,3,3]:
    R = I + a K + b K^2 with K = skew(r), a = sin|r|/|r|, b = (1 - cos|r|)/|r|^2
    (Taylor series near |r| = 0 keep the gradient finite)."""
    th2 = (r * r).sum(-1)
    th = torch.sqrt(th2.clamp_min(1e-30))
    small = th2 < 1e-8
    a = torch.where(small, 1.0 - th2 / 6.0, torch.sin(th) / th)
    b = torch.where(small, 0.5 - th2 / 24.0, (1.0 - torch.cos(th)) / th2.clamp_min(1e-30))
    K = _skew(r)
    eye = torch.eye(3, dtype=r.dtype, device=r.device).expand(K.shape)
    return eye + a[..., None, None] * K + b[..., None, None] * (K @ K)


def quaternion_to_matrix(q: torch.Tensor) -> torch.Tensor:
    """Quaternions (w, x, y, z) [...,4] (normalised here) -> rotation matrices."""
    q = q / q.norm(dim=-1, keepdim=True)
    w, x, y, z = q.unbind(-1)
    return torch.stack([
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)], -1),
        torch.stack([2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)], -1),
        torch.stack([2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)], -1),
    ], -2)


def compose(t_hat, R_hat, s_hat, delta_t, delta_r, delta_s):
    """Residual pose: t = t_hat + delta_t, R = Rodrigues(delta_r) R_hat, s = s_hat + delta_s."""
    return t_hat + delta_t, rodrigues(delta_r) @ R_hat, s_hat + delta_s


def volume_prior(s: torch.Tensor, lam: float = 0.01) -> torch.Tensor:
    """lambda * sum_k Prod(s_k) over the per-axis scales as passed (the renderer's
    half extents, i.e. 1/8 of the box volume each)."""
    return lam * s.prod(dim=-1).sum()
