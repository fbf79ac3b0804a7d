"""Helpers for the GPU parity tests (HIP library vs the CPU oracle)."""
import sys

import numpy as np
import torch

import oracle
from paper_2103_01954_amd.api import DevicePrims, aux_fields


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_forward(ctx, prims, cams, params, bf16=None):
    dp = DevicePrims.from_host(prims, bf16=bf16)
    acc = ctx.build_accel(dp, cams, params)
    rgba, aux = acc.render_fwd(dp)
    torch.cuda.synchronize()
    return acc, dp, rgba.cpu().numpy().astype(np.float64), aux


def hit_lists(off, ids, rays):
    return [ids[off[r]:off[r + 1]] for r in rays]


def max_abs(a, b):
    return float(np.abs(np.asarray(a, np.float64) - np.asarray(b, np.float64)).max()) if np.size(a) else 0.0


def rel_l2(a, b):
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def oracle_pixels(cam, rays):
    rays = np.asarray(rays)
    return np.stack([rays // cam.width, rays % cam.width], axis=1)
