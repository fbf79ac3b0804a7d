"""CPU oracle for the volumetric-primitive ray marcher (test infrastructure).

A plain, slow, FP64 NumPy implementation of what the renderer computes,
written from the paper (Lombardi et al., "Mixture of Volumetric Primitives
for Efficient Neural Rendering", Sec. 3.1.2 and Sec. 3.2).  It exists to
check the GPU library; it is never part of the product path.  Only the test
suite, the smoke check and the CPU-baseline leg of the benchmark may import
it.  It shares no code with the HIP library: the only common module is the
seeded input generator, which holds none of the method's arithmetic.

Modules
  geometry  canonical FP32 local rays, slab test and sample ranges
            (hit sets and sample membership are decided in FP32 with a fixed
            operation order so that they are reproducible bit for bit)
  render    forward march in FP64: trilinear payload sampling, the sum rule
            for overlapping primitives, the clamped additive accumulation and
            early termination (Sec. 3.2.2)
  adjoint   FP64 gradients of the forward with respect to the payloads and the
            primitive pose and scale

Every function here is pinned by the CPU tests (closed forms, invariants,
brute force, exact rational arithmetic, finite differences); nothing is
"parity unpinned" except agreement with the authors' own renders, for which
the paper gives no numbers.
"""
from .geometry import (  # noqa: F401
    J_MAX, local_frame, pixel_rays, local_ray, slab, sample_positions,
    first_sample_not_before, last_sample_not_after,
)
from .render import render, hit_sets  # noqa: F401
from .adjoint import render_grad  # noqa: F401
