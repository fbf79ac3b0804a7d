// Internal declarations shared by the HIP translation units of libmvp.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mvp.h"

namespace mvp {

constexpr int kTile = 16;                  // screen tile edge in pixels
constexpr int kTileThreads = kTile * kTile;  // one thread per pixel of a tile
constexpr int kWave = 64;                  // CDNA wavefront width
constexpr int kStage = 256;                // culling-list entries staged in LDS per pass
constexpr int kJMax = (1 << 24) - 1;       // largest sample index with an exact float value

// Camera as the kernels see it: origin, pixel->direction matrix and its inverse
// (direction->pixel, for the conservative screen rectangles).
struct DevCam {
  float o[3];
  float P[9];
  float Pinv[9];
  int32_t W, H;
};

// Everything a kernel needs to address the per-frame structure.
struct AccelView {
  int32_t V, W, H, N, M;
  int32_t tiles_x, tiles_y;
  float step, eps, t_near;
  const DevCam *cams;          // [V]
  const float4 *xf;            // [N*3]: rows of A = diag(1/s) R^T, .w = t
  const uint64_t *tile_off;    // [V*T+1] start of each tile's culling list
  const uint32_t *tile_list;   // primitive ids
  const uint64_t *ray_off;     // [R+1] start of each ray's pair list
  const float4 *pa;            // [P] (a.xyz, jlo as bits): local ray origin, first sample
  const float4 *pb;            // [P] (b.xyz, jhi as bits): local ray direction, last sample
  const int32_t *pid;          // [P] primitive id of each pair
};

// ---- launchers (return the first HIP error) --------------------------------
hipError_t launch_zero_u32(uint32_t *p, size_t n, hipStream_t s);
hipError_t launch_zero_u64(uint64_t *p, size_t n, hipStream_t s);
// exclusive scan of n uint32 counts into n+1 uint64 offsets (scratch from scan_scratch_bytes)
size_t scan_scratch_bytes(size_t n);
hipError_t launch_scan_u32_u64(const uint32_t *in, uint64_t *out, size_t n, void *scratch, hipStream_t s);

hipError_t launch_prep(const mvp_prims &p, const AccelView &av, float4 *xf, int4 *rect,
                       uint32_t *tile_cnt, hipStream_t s);
hipError_t launch_tile_fill(const AccelView &av, const int4 *rect, uint32_t *cursor,
                            uint32_t *tile_list, hipStream_t s);
// mode 0: (ray, primitive) pairs with >= 1 sample; mode 1: every slab hit (debug)
hipError_t launch_hit_count(const AccelView &av, int mode, uint32_t *ray_cnt, hipStream_t s);
hipError_t launch_hit_emit(const AccelView &av, int mode, float4 *pa, float4 *pb, int32_t *pid,
                           hipStream_t s);

hipError_t launch_march_fwd(const AccelView &av, const mvp_prims &p, float *rgba, mvp_ray_aux *aux,
                            unsigned long long *counters, hipStream_t s);
hipError_t launch_march_bwd(const AccelView &av, const mvp_prims &p, const mvp_ray_aux *aux,
                            const float *grad_rgba, float *g_pay, float *g_pos, float *g_rot,
                            float *g_scale, hipStream_t s);

}  // namespace mvp
