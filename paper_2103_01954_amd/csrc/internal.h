// Internal declarations shared by the HIP translation units of libmvp.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mvp.h"

namespace mvp {

constexpr int kTile = 16;                  // screen tile edge in pixels
constexpr int kTileThreads = kTile * kTile;  // one thread per pixel of a tile
constexpr int kWave = 64;                  // CDNA wavefront width
constexpr int kStage = 128;                // culling-list entries staged in LDS per pass
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
// tile_off[t+1]), primitive ids ordered near to far (by an order key per view
// and primitive, then id).  Transposed: primitive k
// owns the list entries prim_entries[prim_entry_off[k] .. prim_entry_off[k+1])
// (ascending), grouped into backward work items item_off[k] .. item_off[k+1]
// of at most item_entries entries each.
// Entry frames: culling-list entry g (primitive k in the list of a tile of
// view v) has ef[3g + i] = (row i of A_k, a_i) with a = A_k (o_v - t_k), the
// local origin shared by every ray of the view; a ray's local direction is
// b = A_k d.
// Pairs: tile t reserves len(t) * R_t pair slots from pair_base[t] (len: its
// culling-list length; R_t: 256 for full frames, its number of rays for a ray
// subset), pair q of ray number i of the tile at pair_base[t] + q * R_t + i
// (so that the lanes of a wave reading or writing the q-th pairs of their
// rays touch neighbouring slots).  Ray slot r has ray_nj[r].x pairs, the q-th
// at pr[ray_seg[r] + q * R_t], sorted by first sample and then primitive id;
// pair p is pr[p] = (jlo, jhi, position in the tile's culling list, primitive
// id), and ray_nj[r].y is the ray's first sample (INT_MAX if none).  The same pairs by culling-list entry, for the backward: entry g at
// position e of tile t = ent_tile[g] lists the pairs formed with it (at most
// one per ray of the tile), in ray order, from ent_base[g] = pair_base[t] +
// e * R_t: the rays of wave w of the tile (ray numbers 64w .. 64w + 63) at
// ent_rec[ent_base[g] + 64 w .. + ent_n[4g + w]).  A record is
// (jlo | i << 24, jhi) with i the ray's number in the tile (sample indices
// stay below 2^24).
// Per-ray constants of the backward: Tdot, the clamp weight ((1 - T_{S-1}) /
// sigma_S for the sum rule, 1 - T* for the sequential combine) and the
// clamping primitive of the sequential combine (-1: none).
struct RayConst {
  float tdot, w;
  int32_t kstar, pad;
};

// Bounds on what one (ray, primitive) pair can add to any single payload
// gradient value (one voxel, one channel): at most per_sample for each of its
// replayed samples, plus clamp once if the pair holds the ray's clamping
// sample.  The backward takes the largest over the pairs of a work item to
// choose the fixed-point scale of its on-chip gradient accumulator.
struct RayBound {
  float per_sample, clamp;
};

// Scratch of one backward call over R rays: RayConst [R], RayBound [R] and
// the payload's largest colour and opacity magnitudes (2 x uint32, float bits).
__host__ __device__ constexpr size_t bwd_scratch_bytes(size_t R) {
  return ((R * sizeof(RayConst) + R * sizeof(RayBound) + 8 + 255) / 256) * 256;
}

struct AccelView {
  int32_t V, W, H, N, M;
  int32_t tiles_x, tiles_y;
  float step, eps, t_near;
  float fade_alpha, fade_beta; // opacity fade window (alpha == 0: none)
  int32_t combine;             // 0: sum rule, 1: sequential in primitive-id order
  int32_t item_entries;        // culling-list entries per backward work item
  const DevCam *cams;          // [V]
  const float4 *xf;            // [N*3]: rows of A = diag(1/s) R^T, .w = t
  const uint64_t *tile_off;    // [V*T+1]
  const uint32_t *tile_list;   // [n_tile_pairs]
  const uint64_t *prim_entry_off;  // [N+1]
  const uint32_t *prim_entries;    // [n_tile_pairs]
  const uint64_t *item_off;        // [N+1], over the primitives in the order item_prim
  const uint32_t *item_prim;       // [N] the backward's order of the primitives
  const float4 *ef;            // [3 n_tile_pairs]
  const uint64_t *pair_base;   // [V*T+1]
  const uint64_t *ray_seg;     // [R]
  const int2 *ray_nj;          // [R]
  const int4 *pr;              // [pair capacity]
  const uint64_t *ent_base;    // [n_tile_pairs]
  const uint32_t *ent_n;       // [4 n_tile_pairs]
  const uint32_t *ent_tile;    // [n_tile_pairs]
  const uint2 *ent_rec;        // [pair capacity]
  // Ray slots.  A full frame has one slot per pixel, slot = (v*H + py)*W + px,
  // and ray_pix == tile_rays == nullptr.  A ray subset has n_slots slots;
  // ray_pix[slot] is the pixel of the slot and tile t owns the (at most 256)
  // slots tile_rays[tile_ray_off[t] .. tile_ray_off[t+1]), in increasing order.
  int64_t n_slots;
  const int64_t *ray_pix;      // [n_slots] or nullptr
  const uint64_t *tile_ray_off;  // [V*T+1] or nullptr
  const uint32_t *tile_rays;   // or nullptr
};

// Where a tile's pairs go (see AccelView for the layouts).  Not restrict: the
// forward march reads them back through its AccelView after a barrier.  The
// per-entry lists (ent_*) are null for a structure built for the forward only.
struct PairsOut {
  float4 *ef;
  int4 *pr;
  uint64_t *ray_seg;
  int2 *ray_nj;
  uint64_t *ent_base;
  uint32_t *ent_n;
  uint32_t *ent_tile;
  uint2 *ent_rec;
  unsigned long long *n_pairs;
};

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own L2):
// workgroup b runs on XCD b % 8.  Launching kXcd * ceil(n / kXcd) workgroups and
// mapping b -> (b % kXcd) * per + b / kXcd gives every XCD a contiguous band of
// tiles, so neighbouring tiles (which share primitives) share an L2.  Returns
// -1 for the padding workgroups.
constexpr int kXcd = 8;
__device__ __forceinline__ int xcd_tile(int b, int n) {
  const int per = (n + kXcd - 1) / kXcd;
  const int t = (b % kXcd) * per + b / kXcd;
  return t < n ? t : -1;
}
__host__ __device__ __forceinline__ int xcd_grid(int n) { return kXcd * ((n + kXcd - 1) / kXcd); }

// Position s of the schedule -> tile index (v*T + ty*tiles_x + tx), visiting
// each view in blocks of kTileBlock x kTileBlock tiles (row-major blocks,
// row-major inside a block; edge blocks are cut to the grid).  The workgroups
// resident on one XCD at a time then cover a compact patch of the screen, whose
// primitives fit its L2 far better than a full-width stripe.
constexpr int kTileBlock = 8;
__device__ __forceinline__ int blocked_tile(int s, int tiles_x, int tiles_y) {
  const int T = tiles_x * tiles_y;
  const int v = s / T;
  const int r = s - v * T;
  const int by = r / (kTileBlock * tiles_x);
  const int rr = r - by * kTileBlock * tiles_x;
  const int hb = min(kTileBlock, tiles_y - by * kTileBlock);
  const int bx = rr / (kTileBlock * hb);
  const int q = rr - bx * kTileBlock * hb;
  const int wb = min(kTileBlock, tiles_x - bx * kTileBlock);
  return v * T + (by * kTileBlock + q / wb) * tiles_x + bx * kTileBlock + q % wb;
}

// Number of times each view's schedule is halved (first by rows, then by
// columns, alternately) so that the XCDs sharing a view get one part each:
// log2(kXcd / V) for V < kXcd views, else 0.
__host__ __device__ __forceinline__ int view_splits(int V) {
  int l = 0;
  while (l < 3 && (V << (l + 1)) <= kXcd) ++l;
  return l;
}

// The march's schedule: the view's tiles cut by `levels` halvings into
// rectangles (top before bottom, left before right), each visited in blocks as
// blocked_tile does.  With the XCDs' contiguous shares of the schedule
// (xcd_tile) each XCD then marches one compact rectangle (for two views, a
// quadrant each) rather than a full-width stripe: its block rows are shorter,
// so neighbouring block rows, which share primitives, follow each other
// sooner in the XCD's L2.
__device__ __forceinline__ int split_tile(int s, int tiles_x, int tiles_y, int levels) {
  const int T = tiles_x * tiles_y;
  const int v = s / T;
  int r = s - v * T;
  int x0 = 0, y0 = 0, w = tiles_x, h = tiles_y;
  for (int l = 0; l < levels; ++l) {
    if (!(l & 1)) {   // rows: top part first
      const int h0 = (h + 1) / 2;
      if (r < w * h0) {
        h = h0;
      } else {
        r -= w * h0;
        y0 += h0;
        h -= h0;
      }
    } else {          // columns: left part first
      const int w0 = (w + 1) / 2;
      if (r < w0 * h) {
        w = w0;
      } else {
        r -= w0 * h;
        x0 += w0;
        w -= w0;
      }
    }
  }
  const int lt = blocked_tile(r, w, h);
  return v * T + (y0 + lt / w) * tiles_x + x0 + lt % w;
}

// Ray number t (0 <= t < 256, row-major in the 16x16 tile) of `tile`: its
// slot, view and pixel.  Returns false if there is no such ray (a tile cut by
// the image border, or a ray subset with fewer rays in the tile).
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

// Canonical FP32 geometry shared by the culling kernels and the marches, so
// that both derive bit-identical pixel rays and local directions (every
// translation unit is built with -ffp-contract=off: one rounding per written
// operation).
// Unit direction of the ray through the centre of pixel (px, py).
__device__ __forceinline__ void pixel_ray(const DevCam &c, int px, int py, float d[3]) {
  const float u = (float)px + 0.5f;
  const float v = (float)py + 0.5f;
  float e[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    float t0 = c.P[3 * i + 0] * u;
    float t1 = c.P[3 * i + 1] * v;
    float t2 = t0 + t1;
    e[i] = t2 + c.P[3 * i + 2];
  }
  float s0 = e[0] * e[0];
  float s1 = e[1] * e[1];
  float s2 = e[2] * e[2];
  float n2 = (s0 + s1) + s2;
  float nrm = sqrtf(n2);
#pragma unroll
  for (int i = 0; i < 3; ++i) d[i] = e[i] / nrm;
}

// r = M v for one row (Mr0, Mr1, Mr2): fl(fl(fl(M0 v0) + fl(M1 v1)) + fl(M2 v2))
__device__ __forceinline__ float row_dot(float m0, float m1, float m2, const float v[3]) {
  float p0 = m0 * v[0];
  float p1 = m1 * v[1];
  float p2 = m2 * v[2];
  float s = p0 + p1;
  return s + p2;
}

// Sum over the lanes of a wave.
__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
  return v;
}

// Number of ray slots of a tile: 256 for full frames (rays outside the image
// included), its sampled rays for a ray subset.
__device__ __forceinline__ int tile_ray_count(const AccelView &av, int tile) {
  return av.tile_rays ? (int)(av.tile_ray_off[tile + 1] - av.tile_ray_off[tile]) : kTileThreads;
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

// Per-structure counters (uint64), written by the most recent forward (the
// first five) and backward (the last four) on the structure.
enum : int {
  kCntRaySamples = 0,   // samples inside >= 1 primitive, up to the stop
  kCntPrimSamples = 1,  // (sample, primitive) pairs: trilinear fetches
  kCntFwdCells = 2,     // forward: voxel-corner sets loaded (8 corners each)
  kCntFwdPj = 3,        // forward: pair-record loads (16 B each)
  kCntFwdPab = 4,       // forward: entry-frame loads from device memory (52 B each)
  kCntBwdVisit = 5,     // backward: pairs visited by the ordering / bound pass
  kCntBwdReplay = 6,    // backward: pairs replayed
  kCntBwdRuns = 7,      // backward: cell runs (voxel-corner sets loaded)
  kCntBwdFlush = 8,     // backward: non-zero gradient values added to device memory
  kCntPairs = 9,        // build: (ray, primitive) pairs with at least one sample
  kCntSizes = 10,       // build: culling-list entries, pair capacity, ray-subset flags (3 words)
  kNumCounters = 13
};

// ---- launchers (return the first HIP error) --------------------------------
hipError_t launch_zero_u32(uint32_t *p, size_t n, hipStream_t s);
hipError_t launch_zero_u64(uint64_t *p, size_t n, hipStream_t s);
// exclusive scan of n uint32 counts into n+1 uint64 offsets (scratch from scan_scratch_bytes)
size_t scan_scratch_bytes(size_t n);
hipError_t launch_scan_u32_u64(const uint32_t *in, uint64_t *out, size_t n, void *scratch, hipStream_t s);

// per primitive: A rows and t (xf), per view its tile rectangle (rect) and an
// order key along the view's rays (depth); counts tile entries
hipError_t launch_prep(const mvp_prims &p, const AccelView &av, float4 *xf, int4 *rect, uint32_t *depth,
                       uint32_t *tile_cnt, hipStream_t s);
hipError_t launch_tile_fill(const AccelView &av, const int4 *rect, uint32_t *cursor,
                            uint32_t *tile_list, hipStream_t s);
// transpose the culling lists (count per primitive, then place each entry
// from the rectangles), and count the backward work items of every primitive
hipError_t launch_prim_entry_count(const uint32_t *tile_list, uint64_t n, uint32_t *cnt, hipStream_t s);
hipError_t launch_prim_entry_place(const AccelView &av, const int4 *rect, uint64_t n, const uint64_t *off,
                                   uint32_t *prim_entries, hipStream_t s);
hipError_t launch_item_count(const uint64_t *prim_entry_off, const uint32_t *prim, int n_prim, int per_item,
                             uint32_t *cnt, hipStream_t s);
// the backward's order of the primitives (prim[N]) by screen position; key[N],
// bcnt[kPrimBuckets], boff[kPrimBuckets + 1] and the scan scratch are temporaries
constexpr int kPrimBuckets = 4096;
hipError_t launch_prim_order(const int4 *rect, int N, int V, int tiles_x, int tiles_y, uint32_t *key,
                             uint32_t *bcnt, uint64_t *boff, void *scan_scratch, uint32_t *prim, hipStream_t s);
int backward_item_entries(int M);   // culling-list entries per backward work item (<= 64)
// sort each segment [off[i], off[i+1]) of data (n_seg segments) ascending, or
// with depth: each tile's culling list by (depth[v N + id], id)
hipError_t launch_segment_sort(const uint64_t *off, uint32_t *data, int64_t n_seg, const uint32_t *depth, int N,
                               int tiles_per_view, hipStream_t s);
// ray subsets: count the sampled rays of every tile (flag: 1 = pixel id out of
// range, 2 = more than 256 rays in a tile), then list them per tile
hipError_t launch_ray_bin(const AccelView &av, uint32_t *tile_cnt, uint32_t *flag, hipStream_t s);
hipError_t launch_ray_fill(const AccelView &av, uint32_t *cursor, uint32_t *tile_rays, hipStream_t s);
// out[0] = *n_entries, out[1] = *capacity, out[2] = *flag (0 if flag is null)
hipError_t launch_gather_sizes(const uint64_t *n_entries, const uint64_t *capacity, const uint32_t *flag,
                               uint64_t *out, hipStream_t s);
// pair capacity of every tile: culling-list length (tile_cnt) times its rays
// (256, or tile_rays_cnt for a ray subset)
hipError_t launch_tile_capacity(const uint32_t *tile_cnt, const uint32_t *tile_rays_cnt, size_t ntile, uint32_t *cap,
                                hipStream_t s);
// the (ray, primitive) pairs of every ray, the entry frames and the per-entry
// pair lists (see AccelView); adds the number of pairs to *n_pairs
hipError_t launch_pairs(const AccelView &av, const PairsOut &o, hipStream_t s);
// debug hit sets: per ray the number of slab hits (with or without samples),
// then their primitive ids in increasing order at ids[off[ray] ..]
hipError_t launch_hit_count(const AccelView &av, uint32_t *ray_cnt, hipStream_t s);
hipError_t launch_hit_ids(const AccelView &av, const uint64_t *off, int32_t *ids, hipStream_t s);

// bg: optional background [rays,3] composited under the premultiplied colour
// build_pairs != nullptr: each workgroup first computes its tile's pairs (as
// launch_pairs does) and then marches them.
hipError_t launch_march_fwd(const AccelView &av, const mvp_prims &p, const float *bg, float *rgba,
                            mvp_ray_aux *aux, unsigned long long *counters, hipStream_t s,
                            const PairsOut *build_pairs = nullptr);
// backward; scratch holds bwd_scratch_bytes(n_slots) bytes (nothing in it needs
// to start at zero); bg/rgba/g_bg for a composited forward
hipError_t launch_march_bwd(const AccelView &av, const mvp_prims &p, int64_t n_items_max,
                            const mvp_ray_aux *aux, const float *grad_rgba, const float *bg,
                            const float *rgba, void *scratch, float *g_pay, float *g_pos, float *g_rot,
                            float *g_scale, float *g_bg, unsigned long long *counters, hipStream_t s,
                            hipEvent_t t0 = nullptr,
                            hipEvent_t t1 = nullptr);   // optional events around the per-pair kernel

}  // namespace mvp
