"""Seeded synthetic inputs for the volumetric-primitive ray marcher.

This module only draws random numbers and packs them into the layout the
library boundary takes: primitives ``{t_k, R_k, s_k, V_k}`` (paper Sec. 3.1.2),
pinhole cameras (Sec. 4.1 calibrates pinhole cameras; rays are
``r(t) = o + t d``, Sec. 3.2.2) and the march parameters (step, early-stop
epsilon, near distance).  It contains none of the rendering arithmetic, so the
GPU path and the CPU oracle can both consume its output without sharing any
of the method's code.

The workloads mirror the paper's regime: 4096 primitives of 8^3 voxels is the
2M-voxel model of Tab. 1; 256..32768 primitives and 8^3..16^3 payloads span its
ablations.  There is no capture data here; every input is synthetic.

Layout conventions (identical to the C boundary):
  pos     [N,3]        float32  primitive centre t_k (world)
  rot     [N,3,3]      float32  row-major R_k, world-from-local: x = R diag(s) y + t
  scale   [N,3]        float32  per-axis half extent s_k of the local box [-1,1]^3
  payload [N,M,M,M,4]  float32  index [k][iz][iy][ix][c], channels (R,G,B,sigma);
                                BF16 scenes hold BF16-representable values
  camera  width, height, origin[3], pix2dir[3,3] with direction
          d ~ pix2dir @ (px + 0.5, py + 0.5, 1)
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List

import numpy as np

F32 = np.float32


@dataclass
class Prims:
    pos: np.ndarray
    rot: np.ndarray
    scale: np.ndarray
    payload: np.ndarray
    bf16: bool = False

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])

    @property
    def m(self) -> int:
        return int(self.payload.shape[1]) if self.payload.ndim == 5 else 0

    def subset(self, idx) -> "Prims":
        idx = np.asarray(idx)
        return Prims(self.pos[idx].copy(), self.rot[idx].copy(), self.scale[idx].copy(),
                     self.payload[idx].copy(), self.bf16)


@dataclass
class Camera:
    width: int
    height: int
    origin: np.ndarray
    pix2dir: np.ndarray


@dataclass
class MarchParams:
    step: float
    eps_early: float
    t_near: float = 0.0
    fade_alpha: float = 0.0     # opacity fade window (0: off; the paper uses 8)
    fade_beta: float = 8.0
    combine: str = "sum"        # "sum" (global field) or "sequential" (primitive-id order)


@dataclass
class Workload:
    name: str
    prims: Prims
    cams: List[Camera]
    params: MarchParams
    extra: dict = field(default_factory=dict)


# ----------------------------------------------------------------------------
# elementary draws
# ----------------------------------------------------------------------------

def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round float32 values to the nearest BF16 value (ties to even), returned
    as float32.  Inputs must be finite."""
    x = np.ascontiguousarray(x, dtype=F32)
    u = x.view(np.uint32)
    bias = ((u >> np.uint32(16)) & np.uint32(1)) + np.uint32(0x7FFF)
    r = (u + bias) & np.uint32(0xFFFF0000)
    return r.view(F32)


def bf16_bits(x: np.ndarray) -> np.ndarray:
    """Upper 16 bits of BF16-representable float32 values (the BF16 encoding)."""
    x = np.ascontiguousarray(x, dtype=F32)
    return (x.view(np.uint32) >> np.uint32(16)).astype(np.uint16)


def quat_to_matrix(q: np.ndarray) -> np.ndarray:
    """Unit quaternions (w,x,y,z) [N,4] -> rotation matrices [N,3,3] (float64)."""
    q = q / np.linalg.norm(q, axis=-1, keepdims=True)
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    r = np.empty((q.shape[0], 3, 3))
    r[:, 0, 0] = 1 - 2 * (y * y + z * z)
    r[:, 0, 1] = 2 * (x * y - z * w)
    r[:, 0, 2] = 2 * (x * z + y * w)
    r[:, 1, 0] = 2 * (x * y + z * w)
    r[:, 1, 1] = 1 - 2 * (x * x + z * z)
    r[:, 1, 2] = 2 * (y * z - x * w)
    r[:, 2, 0] = 2 * (x * z - y * w)
    r[:, 2, 1] = 2 * (y * z + x * w)
    r[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return r


def random_rotations(rng: np.random.Generator, n: int) -> np.ndarray:
    """Uniform random rotations from normalised Gaussian quaternions."""
    return quat_to_matrix(rng.normal(size=(n, 4)))


def tangent_frames(normals: np.ndarray, twist: np.ndarray) -> np.ndarray:
    """Rotations whose local z axis is the given unit normal, with a twist about
    it (the tangent-frame initialisation of Sec. 3.1.2)."""
    n = normals / np.linalg.norm(normals, axis=-1, keepdims=True)
    helper = np.where(np.abs(n[:, 1:2]) < 0.9, np.array([[0.0, 1.0, 0.0]]), np.array([[1.0, 0.0, 0.0]]))
    x0 = np.cross(helper, n)
    x0 /= np.linalg.norm(x0, axis=-1, keepdims=True)
    y0 = np.cross(n, x0)
    c, s = np.cos(twist)[:, None], np.sin(twist)[:, None]
    x = c * x0 + s * y0
    y = -s * x0 + c * y0
    return np.stack([x, y, n], axis=-1)  # columns are the local axes


def random_payload(rng: np.random.Generator, n: int, m: int, empty_frac: float = 0.0,
                   sigma_max: float = 4.0) -> np.ndarray:
    """RGB ~ U[0,1), sigma ~ U[0,sigma_max); a fraction of voxels gets sigma = 0."""
    pay = np.empty((n, m, m, m, 4), dtype=F32)
    pay[..., :3] = rng.random((n, m, m, m, 3), dtype=F32)
    pay[..., 3] = rng.random((n, m, m, m), dtype=F32) * F32(sigma_max)
    if empty_frac > 0:
        mask = rng.random((n, m, m, m), dtype=F32) < F32(empty_frac)
        pay[..., 3][mask] = 0
    return pay


def look_at_camera(rng: np.random.Generator, width: int, height: int, dist: float = 3.0) -> Camera:
    """Pinhole camera on a sphere of radius ``dist`` looking at the origin.

    OpenCV axes (x right, y down, z forward), focal length = width pixels,
    principal point at the image centre; pix2dir = R_cw K^-1."""
    w = rng.normal(size=3)
    w /= np.linalg.norm(w)
    pos = dist * w
    fwd = -w
    up = np.array([0.0, 1.0, 0.0]) if abs(w[1]) <= 0.99 else np.array([1.0, 0.0, 0.0])
    right = np.cross(fwd, up)
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    r_cw = np.stack([right, down, fwd], axis=1)
    f = float(width)
    k_inv = np.array([[1.0 / f, 0.0, -0.5 * width / f],
                      [0.0, 1.0 / f, -0.5 * height / f],
                      [0.0, 0.0, 1.0]])
    return Camera(width, height, pos.astype(F32), (r_cw @ k_inv).astype(F32))


def axis_camera(width: int, height: int, origin, forward_axis: int = 2, sign: float = -1.0,
                focal: float | None = None) -> Camera:
    """Camera at ``origin`` looking along +/- a world axis (used for hand-made
    closed-form scenes).  With an odd width/height the centre pixel's ray is
    exactly the viewing axis."""
    f = float(focal if focal is not None else width)
    fwd = np.zeros(3)
    fwd[forward_axis] = sign
    up = np.array([0.0, 1.0, 0.0]) if forward_axis != 1 else np.array([1.0, 0.0, 0.0])
    right = np.cross(fwd, up)
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    r_cw = np.stack([right, down, fwd], axis=1)
    k_inv = np.array([[1.0 / f, 0.0, -0.5 * width / f],
                      [0.0, 1.0 / f, -0.5 * height / f],
                      [0.0, 0.0, 1.0]])
    return Camera(width, height, np.asarray(origin, dtype=F32), (r_cw @ k_inv).astype(F32))


# ----------------------------------------------------------------------------
# scene families
# ----------------------------------------------------------------------------

def random_box_scene(seed: int, n: int = 8, m: int = 8, s_lo: float = 0.1, s_hi: float = 0.4,
                     empty_frac: float = 0.0, bf16: bool = False) -> Prims:
    """Centres U[-1,1]^3, random rotations, per-axis half extents U[s_lo,s_hi]."""
    rng = np.random.default_rng(seed)
    pos = rng.uniform(-1.0, 1.0, size=(n, 3)).astype(F32)
    rot = random_rotations(rng, n).astype(F32)
    scale = rng.uniform(s_lo, s_hi, size=(n, 3)).astype(F32)
    pay = random_payload(rng, n, m, empty_frac)
    if bf16:
        pay = bf16_round(pay)
    return Prims(pos, rot, scale, pay, bf16)


def noisy_sphere_scene(seed: int, n: int, m: int, scale: float, empty_frac: float,
                       radius: float = 0.8, bf16: bool = False) -> Prims:
    """Primitives near a noisy sphere: r(dir) = radius (1 + 0.1 mean_q a_q sin(w_q.dir + phi_q)),
    centre = r dir + N(0, 0.01^2), tangent-frame rotations with a random twist,
    half extents scale * U[0.9,1.1] per axis, sparse opacity."""
    rng = np.random.default_rng(seed)
    dirs = rng.normal(size=(n, 3))
    dirs /= np.linalg.norm(dirs, axis=-1, keepdims=True)
    omega = rng.normal(0.0, 3.0, size=(8, 3))
    amp = rng.uniform(-1.0, 1.0, size=8)
    phase = rng.uniform(0.0, 2 * np.pi, size=8)
    noise = np.mean(amp[None, :] * np.sin(dirs @ omega.T + phase[None, :]), axis=1)
    r = radius * (1.0 + 0.1 * noise)
    centres = r[:, None] * dirs + rng.normal(0.0, 0.01, size=(n, 3))
    twist = rng.uniform(0.0, 2 * np.pi, size=n)
    rot = tangent_frames(dirs, twist)
    s = scale * rng.uniform(0.9, 1.1, size=(n, 3))
    pay = random_payload(rng, n, m, empty_frac)
    if bf16:
        pay = bf16_round(pay)
    return Prims(centres.astype(F32), rot.astype(F32), s.astype(F32), pay, bf16)


def zero_outer_layers(prims: Prims, layers: int = 2) -> Prims:
    """Set opacity to zero in the outer voxel layers (finite-difference-safe
    scenes: the field and its derivative vanish near every box face)."""
    pay = prims.payload.copy()
    m = pay.shape[1]
    keep = np.zeros(m, dtype=bool)
    keep[layers:m - layers] = True
    inner = keep[:, None, None] & keep[None, :, None] & keep[None, None, :]
    pay[..., 3] *= inner[None].astype(F32)
    return Prims(prims.pos, prims.rot, prims.scale, pay, prims.bf16)


def as_bf16(prims: Prims) -> Prims:
    return Prims(prims.pos, prims.rot, prims.scale, bf16_round(prims.payload), True)


# ----------------------------------------------------------------------------
# named workloads (seeds fixed; the draw order is the code order above)
# ----------------------------------------------------------------------------

def c0(bf16: bool = False) -> Workload:
    """8 primitives of 8^3, one 64x64 view, step 1/128."""
    prims = random_box_scene(0, n=8, m=8, bf16=bf16)
    cam = look_at_camera(np.random.default_rng(100), 64, 64)
    return Workload("c0", prims, [cam], MarchParams(1.0 / 128, 1e-6))


def sphere_4096(bf16: bool = False) -> Prims:
    return noisy_sphere_scene(1, n=4096, m=8, scale=0.05, empty_frac=0.7, bf16=bf16)


def c1(bf16: bool = False, size: int = 1024) -> Workload:
    """4096 primitives of 8^3 on a noisy sphere, one 1024^2 view, step 1/512."""
    cam = look_at_camera(np.random.default_rng(101), size, size)
    return Workload("c1", sphere_4096(bf16), [cam], MarchParams(1.0 / 512, 1e-6))


def c2(size: int = 1024, views: int = 4) -> Workload:
    """The 4096-primitive scene, 4 views of 1024^2, MSE to a random target image."""
    rng = np.random.default_rng(102)
    cams = [look_at_camera(rng, size, size) for _ in range(views)]
    target = np.random.default_rng(103).random((views, size, size, 3), dtype=F32)
    return Workload("c2", sphere_4096(False), cams, MarchParams(1.0 / 512, 1e-6),
                    extra={"target": target})


def c2_fd() -> Workload:
    """16 primitives drawn like c0 with the outer two voxel layers transparent,
    one 32x32 view, step 1/128, no early stop."""
    prims = zero_outer_layers(random_box_scene(2, n=16, m=8))
    cam = look_at_camera(np.random.default_rng(104), 32, 32)
    return Workload("c2_fd", prims, [cam], MarchParams(1.0 / 128, 0.0))


def c4() -> Workload:
    """32768 primitives of 16^3 (BF16, 80% empty), 2 views of 2048^2, step 1/1024."""
    prims = noisy_sphere_scene(6, n=32768, m=16, scale=0.02, empty_frac=0.8, bf16=True)
    rng = np.random.default_rng(106)
    cams = [look_at_camera(rng, 2048, 2048) for _ in range(2)]
    return Workload("c4", prims, cams, MarchParams(1.0 / 1024, 1e-6))


SERVE_RESOLUTIONS = [(256, 256), (512, 512), (1280, 720), (1920, 1080)]


def serving_scene_specs(seed: int = 4, count: int = 16):
    """(n, m, scale, scene seed) for the resident serving pool: N = 2^U{8..14},
    M in {8,12,16}, half extent 0.05 sqrt(4096/N), BF16 payloads."""
    rng = np.random.default_rng(seed)
    specs = []
    for i in range(count):
        n = int(2 ** rng.integers(8, 15))
        m = int(rng.choice([8, 12, 16]))
        specs.append((n, m, 0.05 * float(np.sqrt(4096.0 / n)), 1000 + i))
    return specs


def serving_scene(spec) -> Prims:
    n, m, scale, seed = spec
    return noisy_sphere_scene(seed, n=n, m=m, scale=scale, empty_frac=0.7, bf16=True)


def serving_requests(seed: int, count: int, n_scenes: int, resolutions=None):
    """(scene index, camera) pairs: resolution uniform over the serving set,
    camera on the radius-3 sphere looking at the origin."""
    rng = np.random.default_rng(seed)
    res = resolutions or SERVE_RESOLUTIONS
    out = []
    for _ in range(count):
        si = int(rng.integers(0, n_scenes))
        w, h = res[int(rng.integers(0, len(res)))]
        out.append((si, look_at_camera(rng, w, h)))
    return out
