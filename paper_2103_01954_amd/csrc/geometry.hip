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
//   hit_count/ per ray: slab test against every primitive of the tile's list
//   hit_emit   (staged in LDS), then the fixed-step sample interval [jlo, jhi]
//              inside each hit box.  The resulting per-ray list of
//              (primitive, local ray, sample interval), sorted by (jlo, id), is
//              the "primitives each ray intersects" and their domain of
//              integration (Sec. 3.2.1).
#include <hip/hip_runtime.h>

#include <climits>

#include "internal.h"

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

hipError_t launch_scan_u32_u64(const uint32_t *in, uint64_t *out, size_t n, void *scratch, hipStream_t s) {
  return scan_rec<uint32_t>(in, out, n, (uint64_t *)scratch, s);
}

// ---------------------------------------------------------------------------
// canonical FP32 geometry (one rounding per written operation)
// ---------------------------------------------------------------------------

// Unit direction of the ray through the centre of pixel (px, py).
__device__ inline void pixel_ray(const DevCam &c, int px, int py, float d[3]) {
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
__device__ inline float row_dot(float m0, float m1, float m2, const float v[3]) {
  float p0 = m0 * v[0];
  float p1 = m1 * v[1];
  float p2 = m2 * v[2];
  float s = p0 + p1;
  return s + p2;
}

// Slab test of the local ray y(t) = a + t b against [-1,1]^3, clipped to t >= t_near.
__device__ inline bool slab_test(const float a[3], const float b[3], float t_near, float *t_in,
                                 float *t_out) {
  float lo = t_near, hi = INFINITY;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    if (b[i] == 0.0f) {
      if (!(a[i] >= -1.0f && a[i] <= 1.0f)) return false;
    } else {
      float n0 = -1.0f - a[i];
      float n1 = 1.0f - a[i];
      float q0 = n0 / b[i];
      float q1 = n1 / b[i];
      lo = fmaxf(lo, fminf(q0, q1));
      hi = fminf(hi, fmaxf(q0, q1));
    }
  }
  *t_in = lo;
  *t_out = hi;
  return lo <= hi;
}

__device__ inline float sample_pos(int j, float dt) { return (float)j * dt; }

// smallest j >= 0 with fl(j dt) >= t (kJMax + 1 if none)
__device__ inline int first_sample_not_before(float t, float dt) {
  float q = t / dt;
  int j;
  if (!(q <= 16777216.0f)) {
    j = kJMax + 1;
  } else {
    float c = ceilf(q);
    j = c < 0.0f ? 0 : (int)c;
  }
  for (int it = 0; it < 4 && j > 0 && sample_pos(j - 1, dt) >= t; ++it) --j;
  for (int it = 0; it < 4 && j <= kJMax && sample_pos(j, dt) < t; ++it) ++j;
  return j;
}

// largest j <= kJMax with fl(j dt) <= t (-1 if none)
__device__ inline int last_sample_not_after(float t, float dt) {
  float q = t / dt;
  int j;
  if (!(q < 16777215.0f)) {
    j = (q == q) ? kJMax : -1;
  } else {
    float f = floorf(q);
    j = f < -1.0f ? -1 : (int)f;
  }
  for (int it = 0; it < 4 && j < kJMax && sample_pos(j + 1, dt) <= t; ++it) ++j;
  for (int it = 0; it < 4 && j >= 0 && sample_pos(j, dt) > t; ++it) --j;
  return j;
}

// ---------------------------------------------------------------------------
// prep: local frames and conservative screen rectangles
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_prep(int N, const float *__restrict__ pos,
                                              const float *__restrict__ rot,
                                              const float *__restrict__ scale, AccelView av,
                                              float4 *__restrict__ xf, int4 *__restrict__ rect,
                                              uint32_t *__restrict__ tile_cnt) {
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
    if (r.x <= r.z && r.y <= r.w) {
      for (int ty = r.y; ty <= r.w; ++ty)
        for (int tx = r.x; tx <= r.z; ++tx)
          atomicAdd(&tile_cnt[(size_t)v * T + (size_t)ty * av.tiles_x + tx], 1u);
    }
  }
}

hipError_t launch_prep(const mvp_prims &p, const AccelView &av, float4 *xf, int4 *rect,
                       uint32_t *tile_cnt, hipStream_t s) {
  if (p.n_prim == 0) return hipSuccess;
  hipLaunchKernelGGL(k_prep, dim3((p.n_prim + 255) / 256), dim3(256), 0, s, p.n_prim, p.pos, p.rot,
                     p.scale, av, xf, rect, tile_cnt);
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

__global__ __launch_bounds__(256) void k_prim_entry_fill(const uint32_t *__restrict__ list, uint64_t n,
                                                         const uint64_t *__restrict__ off,
                                                         uint32_t *__restrict__ cursor,
                                                         uint32_t *__restrict__ out) {
  uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (; g < n; g += stride) {
    const uint32_t k = list[g];
    const uint64_t pos = off[k] + atomicAdd(&cursor[k], 1u);
    if (pos < off[k + 1]) out[pos] = (uint32_t)g;
  }
}

__global__ __launch_bounds__(256) void k_item_count(const uint64_t *__restrict__ off, int n, int per_item,
                                                    uint32_t *__restrict__ cnt) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) cnt[k] = (uint32_t)((off[k + 1] - off[k] + per_item - 1) / per_item);
}

hipError_t launch_prim_entry_count(const uint32_t *tile_list, uint64_t n, uint32_t *cnt, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_prim_entry_count, dim3(grid_for(n, 256)), dim3(256), 0, s, tile_list, n, cnt);
  return hipGetLastError();
}

hipError_t launch_prim_entry_fill(const uint32_t *tile_list, uint64_t n, const uint64_t *off, uint32_t *cursor,
                                  uint32_t *prim_entries, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_prim_entry_fill, dim3(grid_for(n, 256)), dim3(256), 0, s, tile_list, n, off, cursor,
                     prim_entries);
  return hipGetLastError();
}

hipError_t launch_item_count(const uint64_t *prim_entry_off, int n_prim, int per_item, uint32_t *cnt,
                             hipStream_t s) {
  if (n_prim == 0) return hipSuccess;
  hipLaunchKernelGGL(k_item_count, dim3((n_prim + 255) / 256), dim3(256), 0, s, prim_entry_off, n_prim, per_item,
                     cnt);
  return hipGetLastError();
}

// Sort every tile's culling list by primitive id, so that the list order (and
// with it the order of every per-ray list and of every floating-point sum over
// a sample's primitives) does not depend on the order of the fill atomics.
// Bitonic sort in LDS; lists longer than kSortMax fall back to a heapsort by
// one thread.
constexpr int kSortMax = 4096;

__global__ __launch_bounds__(256) void k_segment_sort(const uint64_t *__restrict__ off,
                                                      uint32_t *__restrict__ list) {
  __shared__ uint32_t s[kSortMax];
  const int64_t seg = blockIdx.x;
  const uint64_t b = off[seg];
  const int64_t n = (int64_t)(off[seg + 1] - b);
  if (n < 2) return;
  if (n <= kSortMax) {
    int np = 2;
    while (np < n) np <<= 1;
    for (int i = threadIdx.x; i < np; i += blockDim.x) s[i] = i < n ? list[b + i] : 0xffffffffu;
    __syncthreads();
    for (int k = 2; k <= np; k <<= 1) {
      for (int j = k >> 1; j > 0; j >>= 1) {
        for (int i = threadIdx.x; i < np; i += blockDim.x) {
          const int ixj = i ^ j;
          if (ixj > i) {
            const uint32_t x = s[i], y = s[ixj];
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
    for (int i = threadIdx.x; i < n; i += blockDim.x) list[b + i] = s[i];
    return;
  }
  if (threadIdx.x != 0) return;
  uint32_t *a = list + b;
  auto sift = [&](int64_t root, int64_t end) {
    while (2 * root + 1 < end) {
      int64_t child = 2 * root + 1;
      if (child + 1 < end && a[child] < a[child + 1]) ++child;
      if (a[root] < a[child]) {
        const uint32_t t = a[root]; a[root] = a[child]; a[child] = t;
        root = child;
      } else {
        return;
      }
    }
  };
  for (int64_t i = n / 2; i-- > 0;) sift(i, n);
  for (int64_t end = n - 1; end > 0; --end) {
    const uint32_t t = a[0]; a[0] = a[end]; a[end] = t;
    sift(0, end);
  }
}

hipError_t launch_segment_sort(const uint64_t *off, uint32_t *data, int64_t n_seg, hipStream_t s) {
  if (n_seg <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_segment_sort, dim3((unsigned)n_seg), dim3(256), 0, s, off, data);
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

// One workgroup per screen tile, one thread per pixel.  The tile's culling
// list is staged through LDS in chunks of kStage primitives: rows of A and the
// local ray origin a = A (o - t), which is the same for every ray of a view.
struct Staged {
  float A[9][kStage];
  float a[3][kStage];
  int32_t id[kStage];
};

__device__ inline void stage_chunk(Staged &sm, const AccelView &av, const DevCam &cam, uint64_t lb,
                                   int cnt) {
  const int e = threadIdx.x;
  if (e < cnt) {
    const int k = (int)av.tile_list[lb + e];
    float A[9], t[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const float4 r = av.xf[3 * (size_t)k + i];
      A[3 * i] = r.x; A[3 * i + 1] = r.y; A[3 * i + 2] = r.z; t[i] = r.w;
    }
    float p[3];
#pragma unroll
    for (int m = 0; m < 3; ++m) p[m] = cam.o[m] - t[m];
#pragma unroll
    for (int i = 0; i < 9; ++i) sm.A[i][e] = A[i];
#pragma unroll
    for (int i = 0; i < 3; ++i) sm.a[i][e] = row_dot(A[3 * i], A[3 * i + 1], A[3 * i + 2], p);
    sm.id[e] = k;
  }
}

// Local ray, slab test and sample interval of staged entry e for direction d.
__device__ inline bool pair_of(const Staged &sm, int e, const float d[3], float t_near, float dt, int mode,
                               float a[3], float b[3], int *jlo, int *jhi) {
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    a[i] = sm.a[i][e];
    b[i] = row_dot(sm.A[3 * i][e], sm.A[3 * i + 1][e], sm.A[3 * i + 2][e], d);
  }
  float t_in, t_out;
  if (!slab_test(a, b, t_near, &t_in, &t_out)) return false;
  if (mode == 1) return true;
  *jlo = first_sample_not_before(t_in, dt);
  *jhi = last_sample_not_after(t_out, dt);
  return *jlo <= *jhi;
}


// Count kernel: per ray the number of pairs (mode 0: pairs with >= 1 sample;
// mode 1: slab hits), and in mode 0 per culling-list entry the number of the
// tile's rays that form a pair with it (entry_cnt, indexed like tile_list).
__global__ __launch_bounds__(kTileThreads) void k_hit_count(AccelView av, int mode,
                                                             uint32_t *__restrict__ ray_cnt,
                                                             uint32_t *__restrict__ entry_cnt) {
  __shared__ Staged sm;
  __shared__ uint32_t s_cnt[kTileThreads / kWave][kStage];
  const int tile = blockIdx.x;
  int v, px, py;
  size_t slot;
  const bool valid = tile_ray(av, tile, threadIdx.x, &slot, &v, &px, &py);
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
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
      const bool hit = valid && pair_of(sm, e, d, av.t_near, av.step, mode, a, b, &jlo, &jhi);
      cnt += hit ? 1u : 0u;
      if (mode == 0) {
        const unsigned long long m = __ballot(hit);
        if (lane == 0) s_cnt[wave][e] = (uint32_t)__popcll(m);
      }
    }
    if (mode == 0) {
      __syncthreads();
      if ((int)threadIdx.x < n) {
        uint32_t tot = 0;
#pragma unroll
        for (int w = 0; w < kTileThreads / kWave; ++w) tot += s_cnt[w][threadIdx.x];
        entry_cnt[c0 + threadIdx.x] = tot;
      }
    }
  }
  if (valid) ray_cnt[slot] = cnt;
}

hipError_t launch_hit_count(const AccelView &av, int mode, uint32_t *ray_cnt, uint32_t *entry_cnt,
                            hipStream_t s) {
  const int ntile = av.V * av.tiles_x * av.tiles_y;
  if (ntile == 0) return hipSuccess;
  hipLaunchKernelGGL(k_hit_count, dim3(ntile), dim3(kTileThreads), 0, s, av, mode, ray_cnt, entry_cnt);
  return hipGetLastError();
}

// Emit kernel, three passes over the tile's culling list (staged in LDS in
// chunks).  Pass 1 finds the ray's pairs (the slab tests of the count pass,
// same predicate) and keeps their first samples jlo in list order, which is
// primitive-id order.  Pass 2 ranks each pair by (jlo, list position), the
// order the forward marches them in: in LDS for lists of at most kKeys pairs
// (jlo < 2^24 in the low 24 bits, the rank in the top 8), in device memory
// (tkey/trank) for longer ones.  Pass 3 writes every pair to its ranked slot of
// the ray's segment [ray_off[ray], ray_off[ray+1]):
//   pa = (a, primitive id), pb = (b, ray index), pj = (jlo, jhi),
// and lists it under its culling-list entry (entry_pairs[entry_off[g] ..],
// pixel order) for the backward.  When the whole culling list fits one LDS
// chunk (the common case) it stays staged, and a ray with a short list
// recomputes its pairs in rank order and writes its segment front to back, so
// each output line is completed in one burst instead of piece by piece.  Mode
// 1 writes only the primitive ids of the slab hits into `ids`, in primitive-id
// order.
constexpr int kKeys = 24;

__global__ __launch_bounds__(kTileThreads) void k_hit_emit(AccelView av, int mode, int32_t *__restrict__ tkey,
                                                            uint32_t *__restrict__ trank, float4 *__restrict__ pa,
                                                            float4 *__restrict__ pb, int2 *__restrict__ pj,
                                                            uint32_t *__restrict__ entry_pairs,
                                                            int32_t *__restrict__ ids) {
  __shared__ Staged sm;
  __shared__ uint32_t s_bits[kStage / 32][kTileThreads];
  __shared__ uint32_t s_cnt[kTileThreads / kWave][kStage];
  __shared__ uint32_t s_key[kKeys][kTileThreads];
  __shared__ uint8_t s_ent[kKeys][kTileThreads];   // single-chunk lists: entry of the i-th pair
  __shared__ uint8_t s_inv[kKeys][kTileThreads];   // ... and of the pair of rank r
  const int tile = blockIdx.x;
  const int t = threadIdx.x;
  int v, px, py;
  size_t ray;
  const bool valid = tile_ray(av, tile, t, &ray, &v, &px, &py);
  const int lane = t & (kWave - 1), wave = t / kWave;
  const DevCam &cam = av.cams[v];
  float d[3];
  pixel_ray(cam, px, py, d);
  const uint64_t out0 = valid ? av.ray_off[ray] : 0;
  const int n = valid ? (int)(av.ray_off[ray + 1] - out0) : 0;   // same predicate as the count pass
  const bool in_lds = n <= kKeys;
  const uint64_t lb = av.tile_off[tile], le = av.tile_off[tile + 1];
  const bool single = le - lb <= (uint64_t)kStage;                 // the same for the whole workgroup
  const unsigned long long lt = (1ull << lane) - 1ull;
  // pass 1: first samples (or, in mode 1, primitive ids) in list order
  int i = 0;
  for (uint64_t c0 = lb; c0 < le; c0 += kStage) {
    const int nc = (int)min<uint64_t>(kStage, le - c0);
    __syncthreads();
    stage_chunk(sm, av, cam, c0, nc);
    __syncthreads();
    uint32_t word = 0;
    for (int e = 0; e < nc; ++e) {
      float a[3], b[3];
      int jlo = 0, jhi = 0;
      if (i < n && pair_of(sm, e, d, av.t_near, av.step, mode, a, b, &jlo, &jhi)) {
        if (mode != 0) {
          ids[out0 + i] = sm.id[e];
        } else if (in_lds) {
          s_key[i][t] = (uint32_t)jlo;
          s_ent[i][t] = (uint8_t)e;
        } else {
          tkey[out0 + i] = jlo;
        }
        ++i;
        word |= 1u << (e & 31);
      }
      if (single && ((e & 31) == 31 || e == nc - 1)) {
        s_bits[e >> 5][t] = word;
        word = 0;
      }
    }
  }
  if (mode != 0) return;
  // pass 2: rank of each pair by (jlo, list position), 8 pairs at a time
  for (int i0 = 0; i0 < n; i0 += 8) {
    int key[8], rank[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      key[q] = i0 + q < n ? (in_lds ? (int)(s_key[i0 + q][t] & 0xffffffu) : tkey[out0 + i0 + q]) : INT_MAX;
      rank[q] = 0;
    }
    for (int j = 0; j < n; ++j) {
      const int kj = in_lds ? (int)(s_key[j][t] & 0xffffffu) : tkey[out0 + j];
#pragma unroll
      for (int q = 0; q < 8; ++q) rank[q] += (kj < key[q] || (kj == key[q] && j < i0 + q)) ? 1 : 0;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      if (i0 + q < n) {
        if (in_lds) {
          s_key[i0 + q][t] = (uint32_t)key[q] | ((uint32_t)rank[q] << 24);
          s_inv[rank[q]][t] = s_ent[i0 + q][t];
        } else {
          trank[out0 + i0 + q] = (uint32_t)rank[q];
        }
      }
    }
  }
  // pass 3: every pair to its ranked slot, and the per-entry pair lists
  i = 0;
  for (uint64_t c0 = lb; c0 < le; c0 += kStage) {
    const int nc = (int)min<uint64_t>(kStage, le - c0);
    if (!single) {
      __syncthreads();
      stage_chunk(sm, av, cam, c0, nc);
      __syncthreads();
    }
    const int ic = i;
    if (single && in_lds) {
      // the list is still staged: recompute the pairs in rank order
      for (int r = 0; r < n; ++r) {
        const int e = s_inv[r][t];
        float a[3], b[3];
        int jlo = 0, jhi = 0;
        (void)pair_of(sm, e, d, av.t_near, av.step, mode, a, b, &jlo, &jhi);
        const uint64_t dst = out0 + r;
        pa[dst] = make_float4(a[0], a[1], a[2], __int_as_float(sm.id[e]));
        pb[dst] = make_float4(b[0], b[1], b[2], __int_as_float((int)ray));
        pj[dst] = make_int2(jlo, jhi);
      }
      i = n;
    } else {
      uint32_t word = 0;
      for (int e = 0; e < nc; ++e) {
        float a[3], b[3];
        int jlo = 0, jhi = 0;
        if (i < n && pair_of(sm, e, d, av.t_near, av.step, mode, a, b, &jlo, &jhi)) {
          const uint64_t dst = out0 + (in_lds ? (s_key[i][t] >> 24) : trank[out0 + i]);
          pa[dst] = make_float4(a[0], a[1], a[2], __int_as_float(sm.id[e]));
          pb[dst] = make_float4(b[0], b[1], b[2], __int_as_float((int)ray));
          pj[dst] = make_int2(jlo, jhi);
          ++i;
          word |= 1u << (e & 31);
        }
        if (!single && ((e & 31) == 31 || e == nc - 1)) {
          s_bits[e >> 5][t] = word;
          word = 0;
        }
      }
    }
    for (int e = 0; e < nc; ++e) {
      const bool bit = (s_bits[e >> 5][t] >> (e & 31)) & 1u;
      const unsigned long long m = __ballot(bit);
      if (lane == 0) s_cnt[wave][e] = (uint32_t)__popcll(m);
    }
    __syncthreads();
    int ii = ic;
    for (int e = 0; e < nc; ++e) {
      const bool bit = (s_bits[e >> 5][t] >> (e & 31)) & 1u;
      const unsigned long long m = __ballot(bit);
      if (bit) {
        uint32_t base = 0;
        for (int q = 0; q < wave; ++q) base += s_cnt[q][e];
        const uint64_t pos = av.entry_off[c0 + e] + base + (uint32_t)__popcll(m & lt);
        entry_pairs[pos] = (uint32_t)(out0 + (in_lds ? (s_key[ii][t] >> 24) : trank[out0 + ii]));
        ++ii;
      }
    }
  }
}

hipError_t launch_hit_emit(const AccelView &av, int mode, int32_t *tkey, uint32_t *trank, float4 *pa, float4 *pb,
                           int2 *pj, uint32_t *entry_pairs, int32_t *ids, hipStream_t s) {
  const int ntile = av.V * av.tiles_x * av.tiles_y;
  if (ntile == 0) return hipSuccess;
  hipLaunchKernelGGL(k_hit_emit, dim3(ntile), dim3(kTileThreads), 0, s, av, mode, tkey, trank, pa, pb, pj,
                     entry_pairs, ids);
  return hipGetLastError();
}

}  // namespace mvp
