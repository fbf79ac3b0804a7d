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


GROUPS = ("payload", "pos", "rot", "scale")


def check_grads(gpu, ref, tol, groups=GROUPS, floor=1e-2, tol_elem=None):
    """Gradient parity gates, per group (tol_elem defaults to tol):

    * relative L2 over the whole group <= tol;
    * element-wise: max |gpu - ref| <= tol_elem * max |ref|;
    * per primitive (leading axis): ||gpu_k - ref_k|| <= tol_elem * (||ref_k|| + floor * max_k ||ref_k||),
      so one wrong primitive (a misplaced corner, a lost flush, a wrong work-item
      boundary) fails even when the group norm dilutes it.  Pose groups are
      checked per primitive over all 15 pose entries together.
    Returns the worst ratios (error / allowance) for reporting."""
    te = tol if tol_elem is None else tol_elem
    worst = {}
    n = None
    pose_g, pose_r = [], []
    for k in groups:
        g = np.asarray(gpu[k], np.float64)
        r = np.asarray(ref[k], np.float64).reshape(g.shape)
        e = rel_l2(g, r)
        mref = float(np.abs(r).max()) if r.size else 0.0
        emax = float(np.abs(g - r).max()) if r.size else 0.0
        say(f"  {k}: rel-L2 {e:.2e}, max-abs {emax:.2e} (max |ref| {mref:.2e})")
        assert e <= tol, (k, "rel-L2", e)
        assert emax <= te * mref + 1e-30, (k, "max-abs", emax, mref)
        worst[k] = max(e / tol, emax / max(te * mref, 1e-300))
        if k == "payload":
            n = g.shape[0]
            dk = np.linalg.norm((g - r).reshape(n, -1), axis=1)
            rk = np.linalg.norm(r.reshape(n, -1), axis=1)
            allow = te * (rk + floor * rk.max())
            bad = np.nonzero(dk > allow)[0]
            assert bad.size == 0, ("payload per primitive", bad[:8], dk[bad[:8]], rk[bad[:8]])
            worst["payload/prim"] = float((dk / np.maximum(allow, 1e-300)).max()) if n else 0.0
        elif k in ("pos", "rot", "scale"):
            pose_g.append(g.reshape(g.shape[0], -1))
            pose_r.append(r.reshape(r.shape[0], -1))
    if pose_g:
        g = np.concatenate(pose_g, 1)
        r = np.concatenate(pose_r, 1)
        dk = np.linalg.norm(g - r, axis=1)
        rk = np.linalg.norm(r, axis=1)
        allow = te * (rk + floor * rk.max())
        bad = np.nonzero(dk > allow)[0]
        assert bad.size == 0, ("pose per primitive", bad[:8], dk[bad[:8]], rk[bad[:8]])
        worst["pose/prim"] = float((dk / np.maximum(allow, 1e-300)).max()) if g.shape[0] else 0.0
    say("  worst error / allowance: " + ", ".join(f"{k} {v:.2f}" for k, v in worst.items()))
    return worst
