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
//
// Culling lists: tile t (of V*T, view-major) owns tile_list[tile_off[t] ..
// tile_off[t+1]), primitive ids in increasing order; entry_tile[g] is the tile
// of list entry g.
// Pairs: ray r owns pairs [ray_off[r], ray_off[r+1]) sorted by (jlo, id);
// pair i is (pa[i] = (a, primitive id), pb[i] = (b, ray index),
// pj[i] = (jlo, jhi)): local ray y(t) = a + t b and its sample interval.
// entry_pairs[entry_off[g] .. entry_off[g+1]) lists the pairs formed with
// culling-list entry g (at most one per ray of the tile), in pixel order.
struct AccelView {
  int32_t V, W, H, N, M;
  int32_t tiles_x, tiles_y;
  float step, eps, t_near;
  const DevCam *cams;          // [V]
  const float4 *xf;            // [N*3]: rows of A = diag(1/s) R^T, .w = t
  const uint64_t *tile_off;    // [V*T+1]
  const uint32_t *tile_list;   // [n_tile_pairs]
  const uint32_t *entry_tile;  // [n_tile_pairs]
  const uint64_t *entry_off;   // [n_tile_pairs+1]
  const uint32_t *entry_pairs; // [n_pairs]
  const uint64_t *ray_off;     // [R+1]
  const float4 *pa;            // [n_pairs]
  const float4 *pb;            // [n_pairs]
  const int2 *pj;              // [n_pairs]
  // Ray slots.  A full frame has one slot per pixel, slot = (v*H + py)*W + px,
  // and ray_pix == tile_rays == nullptr.  A ray subset has n_slots slots;
  // ray_pix[slot] is the pixel of the slot and tile t owns the (at most 256)
  // slots tile_rays[tile_ray_off[t] .. tile_ray_off[t+1]), in increasing order.
  int64_t n_slots;
  const int64_t *ray_pix;      // [n_slots] or nullptr
  const uint64_t *tile_ray_off;  // [V*T+1] or nullptr
  const uint32_t *tile_rays;   // or nullptr
};

// Ray of thread t of the workgroup of `tile`: its slot, view and pixel.
// Returns false if the thread has no ray.
__device__ __forceinline__ bool tile_ray(const AccelView &av, int tile, int t, size_t *slot, int *v,
                                         int *px, int *py) {
  const int T = av.tiles_x * av.tiles_y;
  *v = tile / T;
  if (!av.tile_rays) {
    const int tt = tile % T;
    *px = (tt % av.tiles_x) * kTile + (t % kTile);
    *py = (tt / av.tiles_x) * kTile + (t / kTile);
    *slot = ((size_t)*v * av.H + *py) * av.W + *px;
    return *px < av.W && *py < av.H;
  }
  const uint64_t b = av.tile_ray_off[tile];
  if ((uint64_t)t >= av.tile_ray_off[tile + 1] - b) {
    *slot = 0;
    *px = *py = 0;
    return false;
  }
  *slot = av.tile_rays[b + t];
  const int64_t pix = av.ray_pix[*slot] - (int64_t)*v * av.W * av.H;
  *px = (int)(pix % av.W);
  *py = (int)(pix / av.W);
  return true;
}

// Pixel of a ray slot.
__device__ __forceinline__ void slot_pixel(const AccelView &av, size_t slot, int *v, int *px, int *py) {
  const int64_t pix = av.ray_pix ? av.ray_pix[slot] : (int64_t)slot;
  const int64_t hw = (int64_t)av.W * av.H;
  *v = (int)(pix / hw);
  const int64_t r = pix - (int64_t)*v * hw;
  *px = (int)(r % av.W);
  *py = (int)(r / av.W);
}

// ---- launchers (return the first HIP error) --------------------------------
hipError_t launch_zero_u32(uint32_t *p, size_t n, hipStream_t s);
hipError_t launch_zero_u64(uint64_t *p, size_t n, hipStream_t s);
// exclusive scan of n uint32 counts into n+1 uint64 offsets (scratch from scan_scratch_bytes)
size_t scan_scratch_bytes(size_t n);
hipError_t launch_scan_u32_u64(const uint32_t *in, uint64_t *out, size_t n, void *scratch, hipStream_t s);

hipError_t launch_prep(const mvp_prims &p, const AccelView &av, float4 *xf, int4 *rect,
                       uint32_t *tile_cnt, hipStream_t s);
hipError_t launch_tile_fill(const AccelView &av, const int4 *rect, uint32_t *cursor,
                            uint32_t *tile_list, uint32_t *entry_tile, hipStream_t s);
// sort each segment [off[i], off[i+1]) of data (n_seg segments) ascending
hipError_t launch_segment_sort(const uint64_t *off, uint32_t *data, int64_t n_seg, hipStream_t s);
// ray subsets: count the sampled rays of every tile (flag: 1 = pixel id out of
// range, 2 = more than 256 rays in a tile), then list them per tile
hipError_t launch_ray_bin(const AccelView &av, uint32_t *tile_cnt, uint32_t *flag, hipStream_t s);
hipError_t launch_ray_fill(const AccelView &av, uint32_t *cursor, uint32_t *tile_rays, hipStream_t s);
// mode 0: (ray, primitive) pairs with >= 1 sample, plus per-entry counts;
// mode 1: every slab hit (debug), entry_cnt unused
hipError_t launch_hit_count(const AccelView &av, int mode, uint32_t *ray_cnt, uint32_t *entry_cnt,
                            hipStream_t s);
// mode 0 writes the pairs to tpa/tpb/tpj (temporary, culling-list order), then
// to pa/pb/pj sorted by first sample; mode 1 writes only ids
hipError_t launch_hit_emit(const AccelView &av, int mode, float4 *tpa, float4 *tpb, int2 *tpj, float4 *pa,
                           float4 *pb, int2 *pj, uint32_t *perm, uint32_t *entry_pairs, int32_t *ids,
                           uint64_t n_pairs, hipStream_t s);

hipError_t launch_march_fwd(const AccelView &av, const mvp_prims &p, float *rgba, mvp_ray_aux *aux,
                            unsigned long long *counters, hipStream_t s);
// backward; rc is scratch of 2 floats per ray
hipError_t launch_march_bwd(const AccelView &av, const mvp_prims &p, int64_t n_entries,
                            const mvp_ray_aux *aux, const float *grad_rgba, float2 *rc, float *g_pay,
                            float *g_pos, float *g_rot, float *g_scale, hipStream_t s);

}  // namespace mvp
