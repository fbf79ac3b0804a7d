// Per-frame culling and ray/primitive intervals for the primitive ray marcher.
//
// Built with -ffp-contract=off and IEEE division/square root: every written
// float operation below is exactly one binary32 operation, so the hit
// decisions and sample intervals are reproducible bit for bit.
//
// Pipeline (one frame, V views of W x H pixels, N primitives):
//   prep       per primitive: world-to-local rows A = diag(1/s) R^T (Sec. 3.1.2:
//              t, R, s are the model-to-world transform), and per view a
//              conservative rectangle of 16x16 screen tiles covering the
//              projected box; counts tile entries.
//   tile_fill  writes each primitive into the culling list of every tile of its
//              rectangle.  These lists take the role of the paper's per-frame
//              BVH (Sec. 3.2.1): a ray only looks at its tile's list.
//   pairs      per ray: slab test against every primitive of the tile's list
//              (staged in LDS), then the fixed-step sample interval [jlo, jhi]
//              inside each hit box.  The resulting per-ray list of
//              (sample interval, list position), sorted by first sample and
//              then primitive id, is the "primitives each ray intersects" and
//              their domain of integration (Sec. 3.2.1); the local ray of a
//              pair is rebuilt from its entry's frame (A, a = A (o - t)) and
//              b = A d.
#include <hip/hip_runtime.h>

#include <climits>

#include "internal.h"
#include "pairs.h"

namespace mvp {

// ---------------------------------------------------------------------------
// small utilities
// ---------------------------------------------------------------------------

__global__ void k_zero_u32(uint32_t *p, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = 0u;
}
__global__ void k_zero_u64(uint64_t *p, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = 0ull;
}

static unsigned grid_for(size_t n, unsigned block) {
  size_t g = (n + block - 1) / block;
  if (g > 65535u * 8u) g = 65535u * 8u;
  return (unsigned)(g < 1 ? 1 : g);
}

hipError_t launch_zero_u32(uint32_t *p, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_u32, dim3(grid_for(n, 256)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}
hipError_t launch_zero_u64(uint64_t *p, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_u64, dim3(grid_for(n, 256)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// exclusive scan: n counts -> n+1 offsets (the last one is the total)
// ---------------------------------------------------------------------------

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanBlock = kScanThreads * kScanItems;

__device__ inline uint64_t wave_incl_scan(uint64_t v) {
  const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    uint64_t o = __shfl_up(v, d, kWave);
    if (lane >= d) v += o;
  }
  return v;
}

// block-wide exclusive scan of one value per thread; returns the prefix, *total the sum
__device__ inline uint64_t block_excl_scan(uint64_t v, uint64_t *total) {
  __shared__ uint64_t s_wave[kScanThreads / kWave];
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  uint64_t incl = wave_incl_scan(v);
  if (lane == kWave - 1) s_wave[wave] = incl;
  __syncthreads();
  uint64_t base = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kScanThreads / kWave; ++w) {
    if (w < wave) base += s_wave[w];
    tot += s_wave[w];
  }
  __syncthreads();
  *total = tot;
  return base + incl - v;
}

template <typename T>
__global__ __launch_bounds__(kScanThreads) void k_scan_block(const T *in, size_t n, uint64_t *out,
                                                             uint64_t *partial) {
  // logical input has n+1 elements, element n reads as 0
  const size_t b0 = (size_t)blockIdx.x * kScanBlock + (size_t)threadIdx.x * kScanItems;
  uint64_t v[kScanItems];
  uint64_t sum = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    size_t idx = b0 + i;
    v[i] = idx < n ? (uint64_t)in[idx] : 0ull;
    sum += v[i];
  }
  uint64_t total;
  uint64_t pre = block_excl_scan(sum, &total);
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    size_t idx = b0 + i;
    if (idx <= n) out[idx] = pre;
    pre += v[i];
  }
  if (threadIdx.x == 0 && partial) partial[blockIdx.x] = total;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_add(uint64_t *out, size_t n1, const uint64_t *base) {
  const uint64_t add = base[blockIdx.x];
  const size_t b0 = (size_t)blockIdx.x * kScanBlock;
  for (int i = threadIdx.x; i < kScanBlock; i += kScanThreads) {
    size_t idx = b0 + i;
    if (idx < n1) out[idx] += add;
  }
}

static size_t scan_blocks(size_t n) { return (n + 1 + kScanBlock - 1) / kScanBlock; }

size_t scan_scratch_bytes(size_t n) {
  size_t bytes = 0;
  size_t nb = scan_blocks(n);
  while (nb > 1) {
    bytes += (2 * nb + 1) * sizeof(uint64_t);
    nb = scan_blocks(nb);
  }
  return bytes + 64;
}

template <typename T>
static hipError_t scan_rec(const T *in, uint64_t *out, size_t n, uint64_t *scratch, hipStream_t s) {
  size_t nb = scan_blocks(n);
  uint64_t *partial = nb > 1 ? scratch : nullptr;
  hipLaunchKernelGGL(k_scan_block<T>, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, n, out, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || nb == 1) return e;
  uint64_t *pout = scratch + nb;
  e = scan_rec<uint64_t>(partial, pout, nb, scratch + 2 * nb + 1, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), dim3(kScanThreads), 0, s, out, n + 1, pout);
  return hipGetLastError();
}

// Small scans in one workgroup of 1024 threads: each thread takes a
// contiguous run of the n+1 inputs (its loads in flight together), the run
// sums are scanned across the workgroup, then each thread reads its run again
// and writes its prefixes.  One launch instead of the three of the
// block-recursive scan; used up to 8 inputs per thread, beyond which the one
// workgroup's uncoalesced reads make it the slower of the two.
constexpr int kScanOneThreads = 1024;
constexpr int kScanOneBatch = 8;
constexpr size_t kScanOneMax = (size_t)kScanOneThreads * kScanOneBatch;

__global__ __launch_bounds__(kScanOneThreads) void k_scan_one(const uint32_t *__restrict__ in, size_t n,
                                                              uint64_t *__restrict__ out) {
  __shared__ uint64_t s_wave[kScanOneThreads / kWave];
  const size_t per = (n + 1 + kScanOneThreads - 1) / kScanOneThreads;
  const size_t b = (size_t)threadIdx.x * per, e = min(n + 1, b + per);
  uint64_t sum = 0;
  for (size_t c = b; c < e; c += kScanOneBatch) {
    uint32_t x[kScanOneBatch];
#pragma unroll
    for (int i = 0; i < kScanOneBatch; ++i) x[i] = (c + i < e && c + i < n) ? in[c + i] : 0u;
#pragma unroll
    for (int i = 0; i < kScanOneBatch; ++i) sum += x[i];
  }
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const uint64_t incl = wave_incl_scan(sum);
  if (lane == kWave - 1) s_wave[wave] = incl;
  __syncthreads();
  uint64_t pre = incl - sum;
  for (int w = 0; w < wave; ++w) pre += s_wave[w];
  for (size_t c = b; c < e; c += kScanOneBatch) {
    uint32_t x[kScanOneBatch];
#pragma unroll
    for (int i = 0; i < kScanOneBatch; ++i) x[i] = (c + i < e && c + i < n) ? in[c + i] : 0u;
#pragma unroll
    for (int i = 0; i < kScanOneBatch; ++i) {
      if (c + i < e) out[c + i] = pre;
      pre += x[i];
    }
  }
}

hipError_t launch_scan_u32_u64(const uint32_t *in, uint64_t *out, size_t n, void *scratch, hipStream_t s) {
  if (n + 1 <= kScanOneMax) {
    hipLaunchKernelGGL(k_scan_one, dim3(1), dim3(kScanOneThreads), 0, s, in, n, out);
    return hipGetLastError();
  }
  return scan_rec<uint32_t>(in, out, n, (uint64_t *)scratch, s);
}

// ---------------------------------------------------------------------------
// prep: local frames and conservative screen rectangles
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_prep(int N, const float *__restrict__ pos,
                                              const float *__restrict__ rot,
                                              const float *__restrict__ scale, AccelView av,
                                              float4 *__restrict__ xf, int4 *__restrict__ rect,
                                              uint32_t *__restrict__ depth, uint32_t *__restrict__ tile_cnt) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N) return;
  float R[9], s[3], t[3];
#pragma unroll
  for (int i = 0; i < 9; ++i) R[i] = rot[9 * (size_t)k + i];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    s[i] = scale[3 * (size_t)k + i];
    t[i] = pos[3 * (size_t)k + i];
  }
  float A[9];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    float is = 1.0f / s[i];
#pragma unroll
    for (int j = 0; j < 3; ++j) A[3 * i + j] = R[3 * j + i] * is;
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) xf[3 * (size_t)k + i] = make_float4(A[3 * i], A[3 * i + 1], A[3 * i + 2], t[i]);

  // half-extent axes of the box in world space: h_j = s_j R[:, j]
  float h[3][3];
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int m = 0; m < 3; ++m) h[j][m] = R[3 * m + j] * s[j];

  const int T = av.tiles_x * av.tiles_y;
  for (int v = 0; v < av.V; ++v) {
    const DevCam &c = av.cams[v];
    // homogeneous pixel coordinates w = Pinv (x - o) of the centre and axes
    float rel[3] = {t[0] - c.o[0], t[1] - c.o[1], t[2] - c.o[2]};
    float wc[3], wh[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      wc[i] = c.Pinv[3 * i] * rel[0] + c.Pinv[3 * i + 1] * rel[1] + c.Pinv[3 * i + 2] * rel[2];
#pragma unroll
      for (int j = 0; j < 3; ++j)
        wh[j][i] = c.Pinv[3 * i] * h[j][0] + c.Pinv[3 * i + 1] * h[j][1] + c.Pinv[3 * i + 2] * h[j][2];
    }
    float zmin = INFINITY, zmax = -INFINITY, mag = fabsf(wc[2]);
    float umin = INFINITY, umax = -INFINITY, vmin = INFINITY, vmax = -INFINITY;
#pragma unroll
    for (int cc = 0; cc < 8; ++cc) {
      const float sx = (cc & 1) ? 1.0f : -1.0f, sy = (cc & 2) ? 1.0f : -1.0f, sz = (cc & 4) ? 1.0f : -1.0f;
      float w0 = wc[0] + sx * wh[0][0] + sy * wh[1][0] + sz * wh[2][0];
      float w1 = wc[1] + sx * wh[0][1] + sy * wh[1][1] + sz * wh[2][1];
      float w2 = wc[2] + sx * wh[0][2] + sy * wh[1][2] + sz * wh[2][2];
      zmin = fminf(zmin, w2);
      zmax = fmaxf(zmax, w2);
      mag = fmaxf(mag, fabsf(w0) + fabsf(w1) + fabsf(w2));
      float iw = 1.0f / w2;
      umin = fminf(umin, w0 * iw);
      umax = fmaxf(umax, w0 * iw);
      vmin = fminf(vmin, w1 * iw);
      vmax = fmaxf(vmax, w1 * iw);
    }
    int4 r;
    const float eps = 1e-4f * mag;
    if (zmax < -eps) {
      r = make_int4(1, 1, 0, 0);                       // entirely behind the camera
    } else if (zmin <= eps) {
      r = make_int4(0, 0, av.tiles_x - 1, av.tiles_y - 1);  // straddles the camera plane
    } else {
      // pixels whose centre lies within the projected box, plus a margin
      const float lim = 1e7f;
      umin = fmaxf(umin, -lim); umax = fminf(umax, lim);
      vmin = fmaxf(vmin, -lim); vmax = fminf(vmax, lim);
      int px0 = (int)floorf(umin - 2.0f), px1 = (int)ceilf(umax + 1.0f);
      int py0 = (int)floorf(vmin - 2.0f), py1 = (int)ceilf(vmax + 1.0f);
      px0 = max(px0, 0); py0 = max(py0, 0);
      px1 = min(px1, av.W - 1); py1 = min(py1, av.H - 1);
      if (px0 > px1 || py0 > py1) r = make_int4(1, 1, 0, 0);
      else r = make_int4(px0 / kTile, py0 / kTile, px1 / kTile, py1 / kTile);
    }
    rect[(size_t)v * N + k] = r;
    // order key of the box along the rays of this view: its distance from the
    // camera less its half diagonal (a lower bound of where rays enter it),
    // as float bits mapped to an unsigned order
    const float dk = sqrtf(rel[0] * rel[0] + rel[1] * rel[1] + rel[2] * rel[2]) -
                     sqrtf(s[0] * s[0] + s[1] * s[1] + s[2] * s[2]);
    const uint32_t bits = __float_as_uint(dk);
    depth[(size_t)v * N + k] = (bits & 0x80000000u) ? ~bits : (bits | 0x80000000u);
    if (r.x <= r.z && r.y <= r.w) {
      for (int ty = r.y; ty <= r.w; ++ty)
        for (int tx = r.x; tx <= r.z; ++tx)
          atomicAdd(&tile_cnt[(size_t)v * T + (size_t)ty * av.tiles_x + tx], 1u);
    }
  }
}

hipError_t launch_prep(const mvp_prims &p, const AccelView &av, float4 *xf, int4 *rect, uint32_t *depth,
                       uint32_t *tile_cnt, hipStream_t s) {
  if (p.n_prim == 0) return hipSuccess;
  hipLaunchKernelGGL(k_prep, dim3((p.n_prim + 255) / 256), dim3(256), 0, s, p.n_prim, p.pos, p.rot,
                     p.scale, av, xf, rect, depth, tile_cnt);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_tile_fill(AccelView av, const int4 *__restrict__ rect,
                                                   uint32_t *__restrict__ cursor,
                                                   uint32_t *__restrict__ list) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)av.V * av.N) return;
  const int v = (int)(i / av.N);
  const int k = (int)(i % av.N);
  const int T = av.tiles_x * av.tiles_y;
  const int4 r = rect[i];
  for (int ty = r.y; ty <= r.w; ++ty)
    for (int tx = r.x; tx <= r.z; ++tx) {
      const size_t tile = (size_t)v * T + (size_t)ty * av.tiles_x + tx;
      const uint32_t slot = atomicAdd(&cursor[tile], 1u);
      list[av.tile_off[tile] + slot] = (uint32_t)k;
    }
}

hipError_t launch_tile_fill(const AccelView &av, const int4 *rect, uint32_t *cursor,
                            uint32_t *tile_list, hipStream_t s) {
  const size_t n = (size_t)av.V * av.N;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_tile_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, av, rect, cursor,
                     tile_list);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_prim_entry_count(const uint32_t *__restrict__ list, uint64_t n,
                                                          uint32_t *__restrict__ cnt) {
  uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (; g < n; g += stride) atomicAdd(&cnt[list[g]], 1u);
}

// Transposed lists without atomics: the entries of primitive k come from the
// tiles of its screen rectangles, view by view and row by row, so the place of
// entry g (tile (v, tx, ty), primitive k) in k's list follows from the
// rectangles alone and the lists come out ascending in g.
__global__ __launch_bounds__(256) void k_prim_entry_place(AccelView av, const int4 *__restrict__ rect, uint64_t n,
                                                          const uint64_t *__restrict__ off,
                                                          uint32_t *__restrict__ out) {
  const int T = av.tiles_x * av.tiles_y;
  uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (; g < n; g += stride) {
    // tile of entry g: last tile t with tile_off[t] <= g
    int lo = 0, hi = av.V * T - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (av.tile_off[mid] <= g) lo = mid; else hi = mid - 1;
    }
    const int v = lo / T, tt = lo - v * T, tx = tt % av.tiles_x, ty = tt / av.tiles_x;
    const uint32_t k = av.tile_list[g];
    uint64_t p = 0;
    for (int w = 0; w < v; ++w) {
      const int4 r = rect[(size_t)w * av.N + k];
      if (r.x <= r.z && r.y <= r.w) p += (uint64_t)(r.z - r.x + 1) * (uint64_t)(r.w - r.y + 1);
    }
    const int4 r = rect[(size_t)v * av.N + k];
    p += (uint64_t)(ty - r.y) * (uint64_t)(r.z - r.x + 1) + (uint64_t)(tx - r.x);
    out[off[k] + p] = (uint32_t)g;
  }
}

// Work items of the p-th primitive in the backward's order (prim[p]; the
// identity when prim is null).
__global__ __launch_bounds__(256) void k_item_count(const uint64_t *__restrict__ off, const uint32_t *__restrict__ prim,
                                                    int n, int per_item, uint32_t *__restrict__ cnt) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int k = prim ? (int)prim[p] : p;
  cnt[p] = (uint32_t)((off[k + 1] - off[k] + per_item - 1) / per_item);
}

// The backward's order of the primitives: by screen position, so that
// consecutive work items read the per-ray data of neighbouring rays.  A
// primitive's key is the Morton code (6 bits a side) of the centre of its tile
// rectangle in the first view that sees it (the last key if none does); the
// primitives are counted into the kPrimBuckets keys, and scattered by key.
// The order within a key follows the atomics and carries no meaning: the
// order only schedules the work items.
__global__ __launch_bounds__(256) void k_prim_key(const int4 *__restrict__ rect, int N, int V, int tiles_x,
                                                  int tiles_y, uint32_t *__restrict__ key,
                                                  uint32_t *__restrict__ cnt) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N) return;
  uint32_t kk = kPrimBuckets - 1;
  for (int v = 0; v < V; ++v) {
    const int4 r = rect[(size_t)v * N + k];
    if (r.x <= r.z && r.y <= r.w) {
      const uint32_t cx = (uint32_t)min(63, (int)(((int64_t)r.x + r.z) * 32 / max(tiles_x, 1)));
      const uint32_t cy = (uint32_t)min(63, (int)(((int64_t)r.y + r.w) * 32 / max(tiles_y, 1)));
      kk = 0;
      for (int b = 0; b < 6; ++b) kk |= (((cx >> b) & 1u) << (2 * b)) | (((cy >> b) & 1u) << (2 * b + 1));
      break;
    }
  }
  key[k] = kk;
  atomicAdd(&cnt[kk], 1u);
}

__global__ __launch_bounds__(256) void k_prim_scatter(const uint32_t *__restrict__ key, int N,
                                                      unsigned long long *__restrict__ boff,
                                                      uint32_t *__restrict__ prim) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < N) prim[atomicAdd(&boff[key[k]], 1ull)] = (uint32_t)k;
}

hipError_t launch_prim_order(const int4 *rect, int N, int V, int tiles_x, int tiles_y, uint32_t *key,
                             uint32_t *bcnt, uint64_t *boff, void *scan_scratch, uint32_t *prim, hipStream_t s) {
  if (N == 0) return hipSuccess;
  hipError_t e = launch_zero_u32(bcnt, kPrimBuckets, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_prim_key, dim3((N + 255) / 256), dim3(256), 0, s, rect, N, V, tiles_x, tiles_y, key, bcnt);
  e = launch_scan_u32_u64(bcnt, boff, kPrimBuckets, scan_scratch, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_prim_scatter, dim3((N + 255) / 256), dim3(256), 0, s, key, N, (unsigned long long *)boff,
                     prim);
  return hipGetLastError();
}

hipError_t launch_prim_entry_count(const uint32_t *tile_list, uint64_t n, uint32_t *cnt, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_prim_entry_count, dim3(grid_for(n, 256)), dim3(256), 0, s, tile_list, n, cnt);
  return hipGetLastError();
}

hipError_t launch_prim_entry_place(const AccelView &av, const int4 *rect, uint64_t n, const uint64_t *off,
                                   uint32_t *prim_entries, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_prim_entry_place, dim3(grid_for(n, 256)), dim3(256), 0, s, av, rect, n, off, prim_entries);
  return hipGetLastError();
}

hipError_t launch_item_count(const uint64_t *prim_entry_off, const uint32_t *prim, int n_prim, int per_item,
                             uint32_t *cnt, hipStream_t s) {
  if (n_prim == 0) return hipSuccess;
  hipLaunchKernelGGL(k_item_count, dim3((n_prim + 255) / 256), dim3(256), 0, s, prim_entry_off, prim, n_prim,
                     per_item, cnt);
  return hipGetLastError();
}

// Sort segments [off[i], off[i+1]) of 32-bit values ascending: plain values
// (depth == nullptr), or culling-list entries (primitive ids) of segment =
// tile i by (depth[v N + id], id) with v = i / tiles_per_view, so that each
// tile's list runs from near to far and a ray meets its primitives nearly in
// the order of their first samples; ties and the order itself are
// independent of the order of the fill atomics.  Bitonic sort in LDS;
// segments longer than kSortMax are sorted by the same network in device
// memory.
constexpr int kSortMax = 4096;

__device__ __forceinline__ uint64_t sort_key(uint32_t x, const uint32_t *depth, uint64_t vN) {
  return depth ? ((uint64_t)depth[vN + x] << 32) | x : (uint64_t)x;
}

__global__ __launch_bounds__(256) void k_segment_sort(const uint64_t *__restrict__ off, uint32_t *__restrict__ list,
                                                      const uint32_t *__restrict__ depth, int N, int tiles_per_view) {
  __shared__ uint64_t s[kSortMax];
  const int64_t seg = blockIdx.x;
  const uint64_t b = off[seg];
  const int64_t n = (int64_t)(off[seg + 1] - b);
  if (n < 2) return;
  const uint64_t vN = depth ? (uint64_t)(seg / tiles_per_view) * (uint64_t)N : 0;
  if (n <= kSortMax) {
    int np = 2;
    while (np < n) np <<= 1;
    for (int i = threadIdx.x; i < np; i += blockDim.x) s[i] = i < n ? sort_key(list[b + i], depth, vN) : ~0ull;
    __syncthreads();
    for (int k = 2; k <= np; k <<= 1) {
      for (int j = k >> 1; j > 0; j >>= 1) {
        for (int i = threadIdx.x; i < np; i += blockDim.x) {
          const int ixj = i ^ j;
          if (ixj > i) {
            const uint64_t x = s[i], y = s[ixj];
            const bool up = (i & k) == 0;
            if ((x > y) == up) {
              s[i] = y;
              s[ixj] = x;
            }
          }
        }
        __syncthreads();
      }
    }
    for (int i = threadIdx.x; i < n; i += blockDim.x) list[b + i] = (uint32_t)s[i];
    return;
  }
  // Longer segments: the same sort over the segment in device memory (in place,
  // keys looked up as they are compared), in the form of the bitonic network
  // whose comparators all put the smaller key first, so that the entries past
  // n act as +infinity and never move.  Each stage's comparators are
  // independent, so a thread issues several at once; a barrier separates the
  // stages (the workgroup's writes are visible to it after the barrier).
  uint32_t *a = list + b;
  int64_t np = 2;
  while (np < n) np <<= 1;
  const int64_t half = np >> 1;
  auto cmpx = [&](int64_t i, int64_t q) {
    if (q >= n) return;
    const uint32_t x = a[i], y = a[q];
    if (sort_key(x, depth, vN) > sort_key(y, depth, vN)) {
      a[i] = y;
      a[q] = x;
    }
  };
  for (int64_t k = 2; k <= np; k <<= 1) {
    const int64_t hk = k >> 1;
    for (int64_t c = threadIdx.x; c < half; c += blockDim.x) {   // flip: i against its mirror in the k-block
      const int64_t i = (c / hk) * k + (c % hk);
      cmpx(i, (i / k) * k + (k - 1 - (i % k)));
    }
    __syncthreads();
    for (int64_t j = hk >> 1; j > 0; j >>= 1) {   // half-cleaners
#pragma unroll 4
      for (int64_t c = threadIdx.x; c < half; c += blockDim.x) {
        const int64_t i = (c / j) * 2 * j + (c % j);
        cmpx(i, i + j);
      }
      __syncthreads();
    }
  }
}

hipError_t launch_segment_sort(const uint64_t *off, uint32_t *data, int64_t n_seg, const uint32_t *depth, int N,
                               int tiles_per_view, hipStream_t s) {
  if (n_seg <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_segment_sort, dim3((unsigned)n_seg), dim3(256), 0, s, off, data, depth, N, tiles_per_view);
  return hipGetLastError();
}

// Ray subsets: bin the sampled rays (pixel ids) into screen tiles.
__global__ __launch_bounds__(256) void k_ray_bin(AccelView av, uint32_t *__restrict__ tile_cnt,
                                                 uint32_t *__restrict__ flag) {
  const int64_t slot = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (slot >= av.n_slots) return;
  const int64_t pix = av.ray_pix[slot];
  if (pix < 0 || pix >= (int64_t)av.V * av.W * av.H) {
    atomicOr(flag, 1u);
    return;
  }
  const int64_t hw = (int64_t)av.W * av.H;
  const int v = (int)(pix / hw);
  const int64_t r = pix - v * hw;
  const int px = (int)(r % av.W), py = (int)(r / av.W);
  const size_t tile = (size_t)v * av.tiles_x * av.tiles_y + (size_t)(py / kTile) * av.tiles_x + px / kTile;
  if (atomicAdd(&tile_cnt[tile], 1u) >= (uint32_t)kTileThreads) atomicOr(flag, 2u);
}

__global__ __launch_bounds__(256) void k_ray_fill(AccelView av, uint32_t *__restrict__ cursor,
                                                  uint32_t *__restrict__ tile_rays) {
  const int64_t slot = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (slot >= av.n_slots) return;
  const int64_t pix = av.ray_pix[slot];
  if (pix < 0 || pix >= (int64_t)av.V * av.W * av.H) return;
  const int64_t hw = (int64_t)av.W * av.H;
  const int v = (int)(pix / hw);
  const int64_t r = pix - v * hw;
  const int px = (int)(r % av.W), py = (int)(r / av.W);
  const size_t tile = (size_t)v * av.tiles_x * av.tiles_y + (size_t)(py / kTile) * av.tiles_x + px / kTile;
  const uint32_t k = atomicAdd(&cursor[tile], 1u);
  const uint64_t pos = av.tile_ray_off[tile] + k;
  if (pos < av.tile_ray_off[tile + 1]) tile_rays[pos] = (uint32_t)slot;
}

hipError_t launch_ray_bin(const AccelView &av, uint32_t *tile_cnt, uint32_t *flag, hipStream_t s) {
  if (av.n_slots == 0) return hipSuccess;
  hipLaunchKernelGGL(k_ray_bin, dim3((unsigned)((av.n_slots + 255) / 256)), dim3(256), 0, s, av, tile_cnt, flag);
  return hipGetLastError();
}

hipError_t launch_ray_fill(const AccelView &av, uint32_t *cursor, uint32_t *tile_rays, hipStream_t s) {
  if (av.n_slots == 0) return hipSuccess;
  hipLaunchKernelGGL(k_ray_fill, dim3((unsigned)((av.n_slots + 255) / 256)), dim3(256), 0, s, av, cursor, tile_rays);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// per-ray hit lists
// ---------------------------------------------------------------------------

__global__ void k_gather_sizes(const uint64_t *__restrict__ n_entries, const uint64_t *__restrict__ capacity,
                               const uint32_t *__restrict__ flag, uint64_t *__restrict__ out) {
  if (threadIdx.x == 0) {
    out[0] = *n_entries;
    out[1] = *capacity;
    out[2] = flag ? (uint64_t)*flag : 0ull;
  }
}

hipError_t launch_gather_sizes(const uint64_t *n_entries, const uint64_t *capacity, const uint32_t *flag,
                               uint64_t *out, hipStream_t s) {
  hipLaunchKernelGGL(k_gather_sizes, dim3(1), dim3(64), 0, s, n_entries, capacity, flag, out);
  return hipGetLastError();
}

// Pair capacity of every tile: its culling-list length times its rays.
__global__ __launch_bounds__(256) void k_tile_capacity(const uint32_t *__restrict__ tile_cnt,
                                                       const uint32_t *__restrict__ tile_rays_cnt, size_t ntile,
                                                       uint32_t *__restrict__ cap) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < ntile) {   // saturated, so that a product beyond 32 bits cannot wrap to a small capacity
    const uint64_t c = (uint64_t)tile_cnt[t] * (tile_rays_cnt ? tile_rays_cnt[t] : (uint32_t)kTileThreads);
    cap[t] = c > 0xffffffffull ? 0xffffffffu : (uint32_t)c;   // integer compare (no FP64 on the device)
  }
}

hipError_t launch_tile_capacity(const uint32_t *tile_cnt, const uint32_t *tile_rays_cnt, size_t ntile, uint32_t *cap,
                                hipStream_t s) {
  if (ntile == 0) return hipSuccess;
  hipLaunchKernelGGL(k_tile_capacity, dim3((unsigned)((ntile + 255) / 256)), dim3(256), 0, s, tile_cnt,
                     tile_rays_cnt, ntile, cap);
  return hipGetLastError();
}

__global__ __launch_bounds__(kTileThreads) __attribute__((amdgpu_waves_per_eu(5))) void k_pairs(AccelView av,
                                                                                                PairsOut o) {
  tile_pairs(av, blockIdx.x, o);
}

hipError_t launch_pairs(const AccelView &av, const PairsOut &o, hipStream_t s) {
  const int ntile = av.V * av.tiles_x * av.tiles_y;
  if (ntile == 0) return hipSuccess;
  hipLaunchKernelGGL(k_pairs, dim3(ntile), dim3(kTileThreads), 0, s, av, o);
  return hipGetLastError();
}

// Debug hit sets: per ray the number of slab hits against its tile's list
// (with or without samples).
__global__ __launch_bounds__(kTileThreads) void k_hit_count(AccelView av, uint32_t *__restrict__ ray_cnt) {
  __shared__ Staged sm;
  const int tile = blockIdx.x;
  int v, px, py;
  size_t slot;
  const bool valid = tile_ray(av, tile, threadIdx.x, &slot, &v, &px, &py);
  const DevCam &cam = av.cams[v];
  float d[3];
  pixel_ray(cam, px, py, d);
  const uint64_t lb = av.tile_off[tile], le = av.tile_off[tile + 1];
  uint32_t cnt = 0;
  for (uint64_t c0 = lb; c0 < le; c0 += kStage) {
    const int n = (int)min<uint64_t>(kStage, le - c0);
    __syncthreads();
    stage_chunk(sm, av, cam, c0, n);
    __syncthreads();
    for (int e = 0; e < n; ++e) {
      float a[3], b[3];
      int jlo, jhi;
      cnt += (valid && pair_of(sm, e, d, av.t_near, av.step, 1, a, b, &jlo, &jhi)) ? 1u : 0u;
    }
  }
  if (valid) ray_cnt[slot] = cnt;
}

hipError_t launch_hit_count(const AccelView &av, uint32_t *ray_cnt, hipStream_t s) {
  const int ntile = av.V * av.tiles_x * av.tiles_y;
  if (ntile == 0) return hipSuccess;
  hipLaunchKernelGGL(k_hit_count, dim3(ntile), dim3(kTileThreads), 0, s, av, ray_cnt);
  return hipGetLastError();
}

// ... and their primitive ids in increasing order at ids[off[ray] ..] (each
// id inserted into the ray's sorted run as it is found).
__global__ __launch_bounds__(kTileThreads) void k_hit_ids(AccelView av, const uint64_t *__restrict__ off,
                                                           int32_t *__restrict__ ids) {
  __shared__ Staged sm;
  const int tile = blockIdx.x;
  int v, px, py;
  size_t slot;
  const bool valid = tile_ray(av, tile, threadIdx.x, &slot, &v, &px, &py);
  const DevCam &cam = av.cams[v];
  float d[3];
  pixel_ray(cam, px, py, d);
  const uint64_t lb = av.tile_off[tile], le = av.tile_off[tile + 1];
  const uint64_t o0 = valid ? off[slot] : 0;
  uint64_t o = o0;
  for (uint64_t c0 = lb; c0 < le; c0 += kStage) {
    const int n = (int)min<uint64_t>(kStage, le - c0);
    __syncthreads();
    stage_chunk(sm, av, cam, c0, n);
    __syncthreads();
    for (int e = 0; e < n; ++e) {
      float a[3], b[3];
      int jlo, jhi;
      if (valid && pair_of(sm, e, d, av.t_near, av.step, 1, a, b, &jlo, &jhi)) {
        const int32_t id = sm.id[e];
        uint64_t at = o++;
        while (at > o0 && ids[at - 1] > id) {
          ids[at] = ids[at - 1];
          --at;
        }
        ids[at] = id;
      }
    }
  }
}

hipError_t launch_hit_ids(const AccelView &av, const uint64_t *off, int32_t *ids, hipStream_t s) {
  const int ntile = av.V * av.tiles_x * av.tiles_y;
  if (ntile == 0) return hipSuccess;
  hipLaunchKernelGGL(k_hit_ids, dim3(ntile), dim3(kTileThreads), 0, s, av, off, ids);
  return hipGetLastError();
}

}  // namespace mvp
