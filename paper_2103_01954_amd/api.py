"""Torch-facing wrapper of libmvp: device tensors in, device tensors out.

PyTorch supplies device memory and the current HIP stream; every step of the
rendering runs in the library's HIP kernels.  ``render`` is differentiable
with respect to positions, rotations, scales and payloads through
``MVPRender`` (a torch.autograd.Function whose backward calls the library's
adjoint kernel).
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib as L
from .scenes import Camera, MarchParams, Prims


def _stream(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


@dataclass
class DevicePrims:
    """Primitives as device tensors (layout of include/mvp.h)."""
    pos: torch.Tensor       # [N,3] float32
    rot: torch.Tensor       # [N,3,3] float32
    scale: torch.Tensor     # [N,3] float32
    payload: torch.Tensor   # [N,M,M,M,4] float32 or bfloat16

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])

    @property
    def m(self) -> int:
        return int(self.payload.shape[1])

    def c_struct(self) -> L.mvp_prims:
        for name, t in (("pos", self.pos), ("rot", self.rot), ("scale", self.scale)):
            if t.dtype != torch.float32 or not t.is_contiguous() or not t.is_cuda:
                raise ValueError(f"{name} must be a contiguous float32 CUDA tensor")
        if self.payload.dtype not in (torch.float32, torch.bfloat16) or not self.payload.is_contiguous():
            raise ValueError("payload must be a contiguous float32 or bfloat16 tensor")
        n, m = self.n, self.m
        if tuple(self.payload.shape) != (n, m, m, m, 4):
            raise ValueError(f"payload shape {tuple(self.payload.shape)} != {(n, m, m, m, 4)}")
        return L.mvp_prims(n, m, L.MVP_BF16 if self.payload.dtype == torch.bfloat16 else L.MVP_F32, 0,
                           self.pos.data_ptr(), self.rot.data_ptr(), self.scale.data_ptr(),
                           self.payload.data_ptr())

    @staticmethod
    def from_host(p: Prims, device="cuda", bf16: Optional[bool] = None) -> "DevicePrims":
        bf16 = p.bf16 if bf16 is None else bf16
        pay = torch.from_numpy(np.ascontiguousarray(p.payload, dtype=np.float32))
        pay = pay.to(device)
        if bf16:
            pay = pay.to(torch.bfloat16)   # round to nearest even (exact for BF16-representable values)
        f = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(device)
        return DevicePrims(f(p.pos), f(p.rot), f(p.scale), pay.contiguous())


def c_camera(cam: Camera) -> L.mvp_camera:
    c = L.mvp_camera()
    c.width, c.height = int(cam.width), int(cam.height)
    for i in range(3):
        c.origin[i] = float(np.float32(cam.origin[i]))
    P = np.asarray(cam.pix2dir, dtype=np.float32).reshape(9)
    for i in range(9):
        c.pix2dir[i] = float(P[i])
    return c


_COMBINE = {"sum": L.MVP_COMBINE_SUM, "sequential": L.MVP_COMBINE_SEQUENTIAL}


def c_params(p: MarchParams) -> L.mvp_march_params:
    combine = getattr(p, "combine", "sum") or "sum"
    if combine not in _COMBINE:
        raise ValueError(f"combine must be one of {sorted(_COMBINE)}, got {combine!r}")
    return L.mvp_march_params(float(p.step), float(p.eps_early), float(p.t_near),
                              float(getattr(p, "fade_alpha", 0.0)), float(getattr(p, "fade_beta", 8.0)),
                              _COMBINE[combine])


class Context:
    """A libmvp context on one HIP device."""

    def __init__(self, device: int = 0):
        self.lib = L.load()
        h = C.c_void_p()
        L.check("mvp_create", self.lib.mvp_create(int(device), C.byref(h)))
        self.handle = h
        self.device = device

    def close(self):
        if self.handle:
            L.check("mvp_destroy", self.lib.mvp_destroy(self.handle))
            self.handle = None

    def timing_start(self, capacity: int):
        """Record HIP events around the forward and backward march kernels of the
        next `capacity` launches of each (mvp_timing_start)."""
        L.check("mvp_timing_start", self.lib.mvp_timing_start(self.handle, int(capacity)))
        self._timing_cap = int(capacity)

    def timing_read(self, kernel: str):
        """Durations in ms of the recorded launches of kernel "fwd" or "bwd" (blocks)."""
        kind = {"fwd": L.MVP_KERNEL_FWD_MARCH, "bwd": L.MVP_KERNEL_BWD_MARCH}[kernel]
        buf = (C.c_float * self._timing_cap)()
        n = C.c_int32()
        L.check("mvp_timing_read", self.lib.mvp_timing_read(self.handle, kind, buf, C.byref(n)))
        return [float(buf[i]) for i in range(n.value)]

    def timing_stop(self):
        L.check("mvp_timing_stop", self.lib.mvp_timing_stop(self.handle))

    def build_accel(self, prims: DevicePrims, cams: Sequence[Camera], params: MarchParams,
                    stream=None, rays: Optional[torch.Tensor] = None) -> "Accel":
        """Culling lists and per-ray pair lists for every pixel of every view, or
        for the pixel ids in `rays` (int64 device tensor, id = (v*H + py)*W + px)."""
        arr = (L.mvp_camera * len(cams))(*[c_camera(c) for c in cams])
        cp = prims.c_struct()
        pp = c_params(params)
        h = C.c_void_p()
        if rays is None:
            L.check("mvp_build_accel", self.lib.mvp_build_accel(self.handle, C.byref(cp), arr, len(cams),
                                                                C.byref(pp), C.byref(h), _stream(stream)))
            return Accel(self, h, len(cams), cams[0].height, cams[0].width, _stream(stream))
        if rays.dtype != torch.int64 or not rays.is_cuda or rays.dim() != 1:
            raise ValueError("rays must be a 1-D int64 CUDA tensor of pixel ids")
        rays = rays.contiguous()
        L.check("mvp_build_accel_rays", self.lib.mvp_build_accel_rays(
            self.handle, C.byref(cp), arr, len(cams), C.byref(pp), rays.data_ptr(), rays.numel(), C.byref(h),
            _stream(stream)))
        return Accel(self, h, len(cams), cams[0].height, cams[0].width, _stream(stream), n_rays=rays.numel())


class Accel:
    def __init__(self, ctx: Context, handle, views: int, height: int, width: int, stream: int = 0,
                 n_rays: Optional[int] = None):
        self.ctx, self.handle = ctx, handle
        self.views, self.height, self.width = views, height, width
        self.stream = stream      # stream of the build; default for destroy
        self.n_rays = n_rays      # ray-subset size, None for full frames

    @property
    def ray_shape(self):
        return (self.views, self.height, self.width) if self.n_rays is None else (self.n_rays,)

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    def info(self) -> dict:
        i = L.mvp_accel_info()
        L.check("mvp_accel_get_info", self.ctx.lib.mvp_accel_get_info(self.handle, C.byref(i)))
        return {k: getattr(i, k) for k, _ in L.mvp_accel_info._fields_}

    def destroy(self, stream=None):
        """Release the structure once the work enqueued on ``stream`` (default:
        the stream it was built on) has finished."""
        if self.handle and self.ctx.handle:
            s = _stream(stream) if stream is not None else self.stream
            h, self.handle = self.handle, None
            L.check("mvp_accel_destroy", self.ctx.lib.mvp_accel_destroy(self.ctx.handle, h, s))

    def render_fwd(self, prims: DevicePrims, rgba: Optional[torch.Tensor] = None,
                   aux: Optional[torch.Tensor] = None, want_aux: bool = True, stream=None,
                   background: Optional[torch.Tensor] = None):
        """Forward march -> (rgba, aux).  With a background [rays,3] the colour
        is composited as I + (1 - A) B."""
        shape = self.ray_shape
        dev = prims.pos.device
        if rgba is None:
            rgba = torch.empty(shape + (4,), dtype=torch.float32, device=dev)
        if aux is None and want_aux:
            aux = torch.empty(shape, dtype=torch.int64, device=dev)   # 8-byte mvp_ray_aux per ray
        cp = prims.c_struct()
        aux_p = aux.data_ptr() if aux is not None else None
        if background is None:
            L.check("mvp_render_fwd", self.ctx.lib.mvp_render_fwd(
                self.ctx.handle, self.handle, C.byref(cp), rgba.data_ptr(), aux_p, _stream(stream)))
        else:
            bg = _check_bg(background, shape)
            L.check("mvp_render_fwd_bg", self.ctx.lib.mvp_render_fwd_bg(
                self.ctx.handle, self.handle, C.byref(cp), bg.data_ptr(), rgba.data_ptr(), aux_p, _stream(stream)))
        return rgba, aux

    def render_bwd(self, prims: DevicePrims, aux: torch.Tensor, grad_rgba: torch.Tensor,
                   grads: Optional[dict] = None, stream=None, background: Optional[torch.Tensor] = None,
                   rgba: Optional[torch.Tensor] = None) -> dict:
        """Accumulate gradients into ``grads`` (allocated as zeros if None).  For
        a composited forward pass its background and rgba; grads then also
        gets "background"."""
        dev = prims.pos.device
        if grads is None:
            grads = {"payload": torch.zeros(prims.payload.shape, dtype=torch.float32, device=dev),
                     "pos": torch.zeros_like(prims.pos), "rot": torch.zeros_like(prims.rot),
                     "scale": torch.zeros_like(prims.scale)}
            if background is not None:
                grads["background"] = torch.zeros(self.ray_shape + (3,), dtype=torch.float32, device=dev)
        g = grad_rgba.contiguous()
        cp = prims.c_struct()
        ptr = lambda k: grads[k].data_ptr() if grads.get(k) is not None else None
        if background is None:
            L.check("mvp_render_bwd", self.ctx.lib.mvp_render_bwd(
                self.ctx.handle, self.handle, C.byref(cp), aux.data_ptr(), g.data_ptr(),
                ptr("payload"), ptr("pos"), ptr("rot"), ptr("scale"), _stream(stream)))
        else:
            bg = _check_bg(background, self.ray_shape)
            assert rgba is not None, "the composited backward needs the forward's rgba"
            L.check("mvp_render_bwd_bg", self.ctx.lib.mvp_render_bwd_bg(
                self.ctx.handle, self.handle, C.byref(cp), bg.data_ptr(), rgba.contiguous().data_ptr(),
                aux.data_ptr(), g.data_ptr(), ptr("payload"), ptr("pos"), ptr("rot"), ptr("scale"),
                ptr("background"), _stream(stream)))
        return grads

    def counts(self, stream=None):
        a, b = C.c_uint64(), C.c_uint64()
        L.check("mvp_accel_counts", self.ctx.lib.mvp_accel_counts(self.ctx.handle, self.handle, C.byref(a),
                                                                  C.byref(b), _stream(stream)))
        return a.value, b.value

    LOAD_COUNT_NAMES = ("ray_samples", "prim_samples", "fwd_cells", "fwd_pair_intervals", "fwd_pair_rays",
                        "bwd_pairs_visited", "bwd_pairs_replayed", "bwd_cell_runs", "bwd_grad_flush")

    def load_counts(self, stream=None) -> dict:
        """Load counts of the latest forward and backward (mvp_accel_load_counts)."""
        buf = (C.c_uint64 * len(self.LOAD_COUNT_NAMES))()
        L.check("mvp_accel_load_counts", self.ctx.lib.mvp_accel_load_counts(self.ctx.handle, self.handle, buf,
                                                                            _stream(stream)))
        return {k: int(buf[i]) for i, k in enumerate(self.LOAD_COUNT_NAMES)}

    def debug_hits(self, prims: DevicePrims, stream=None):
        """Per-ray sorted hit sets as (offsets [R+1] int64, ids int32) numpy arrays."""
        R = int(np.prod(self.ray_shape))
        dev = prims.pos.device
        off = torch.empty(R + 1, dtype=torch.int64, device=dev)
        cap = C.c_int64(0)
        cp = prims.c_struct()
        total = C.c_int64()
        st = self.ctx.lib.mvp_debug_hits(self.ctx.handle, self.handle, C.byref(cp), off.data_ptr(), None, 0,
                                         C.byref(total), _stream(stream))
        if st not in (L.MVP_OK, L.MVP_ERR_OOM):
            L.check("mvp_debug_hits", st)
        ids = torch.empty(max(1, total.value), dtype=torch.int32, device=dev)
        cap = total.value
        L.check("mvp_debug_hits", self.ctx.lib.mvp_debug_hits(self.ctx.handle, self.handle, C.byref(cp),
                                                              off.data_ptr(), ids.data_ptr(), cap,
                                                              C.byref(total), _stream(stream)))
        return off.cpu().numpy(), ids[:total.value].cpu().numpy()


def _check_bg(bg: torch.Tensor, shape) -> torch.Tensor:
    if bg.dtype != torch.float32 or not bg.is_cuda or tuple(bg.shape) != tuple(shape) + (3,):
        raise ValueError(f"background must be a float32 CUDA tensor of shape {tuple(shape) + (3,)}")
    return bg.contiguous()


def aux_fields(aux: torch.Tensor):
    """Split the 8-byte per-ray aux into (j_end int32, t_prev float32) numpy arrays."""
    a = aux.cpu().contiguous().numpy().view(np.int32).reshape(aux.shape + (2,))
    return a[..., 0].copy(), a[..., 1].copy().view(np.float32)


class MVPRender(torch.autograd.Function):
    """rgba = render(pos, rot, scale, payload) for fixed cameras and march parameters."""

    @staticmethod
    def forward(fctx, pos, rot, scale, payload, ctx: Context, cams, params):
        prims = DevicePrims(pos.contiguous(), rot.contiguous(), scale.contiguous(), payload.contiguous())
        accel = ctx.build_accel(prims, cams, params)
        rgba, aux = accel.render_fwd(prims)
        fctx.accel = accel
        fctx.prims = prims
        fctx.save_for_backward(aux)
        fctx.payload_dtype = payload.dtype
        return rgba

    @staticmethod
    def backward(fctx, grad_rgba):
        (aux,) = fctx.saved_tensors
        accel, prims = fctx.accel, fctx.prims
        need = fctx.needs_input_grad
        dev = prims.pos.device
        grads = {
            "pos": torch.zeros_like(prims.pos) if need[0] else None,
            "rot": torch.zeros_like(prims.rot) if need[1] else None,
            "scale": torch.zeros_like(prims.scale) if need[2] else None,
            "payload": torch.zeros(prims.payload.shape, dtype=torch.float32, device=dev) if need[3] else None,
        }
        accel.render_bwd(prims, aux, grad_rgba.contiguous(), grads)
        accel.destroy()
        gp = grads["payload"]
        if gp is not None and fctx.payload_dtype != torch.float32:
            gp = gp.to(fctx.payload_dtype)
        return grads["pos"], grads["rot"], grads["scale"], gp, None, None, None


def render(ctx: Context, pos, rot, scale, payload, cams: Sequence[Camera], params: MarchParams):
    """Differentiable render of V views -> rgba [V,H,W,4] (premultiplied colour, alpha)."""
    return MVPRender.apply(pos, rot, scale, payload, ctx, list(cams), params)
