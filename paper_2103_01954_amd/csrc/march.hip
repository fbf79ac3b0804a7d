// Forward and backward ray march through the per-ray primitive lists.
//
// Forward (Sec. 3.2.2): for each sample t_j = j*dt inside at least one
// primitive of the ray's list, every containing primitive is sampled
// trilinearly (Sec. 3.2.1) and the samples are combined by the sum rule
//   sigma_j = sum_k sigma_kj,   C_j = sum_k sigma_kj c_kj
// (the global colour/opacity field), then accumulated with the clamp
//   T + sigma_j dt <= 1 :  T += sigma_j dt,  I += C_j dt
//   otherwise           :  I += C_j (1 - T) / sigma_j,  T = 1   (stop)
// and the march stops once T > 1 - eps_early.  With the sequential combine
// (combine == 1) a sample whose summed step saturates is instead taken one
// primitive at a time in increasing id, each with its own clamp step: the
// primitives before the clamping one k* add sigma_k c_k dt, k* adds
// c_k* (1 - T) and the rest nothing; every other sample is the sum rule.
//
// Backward: the additive rule makes every sample's contribution independent
// of the others except through the clamp, so the backward replays each
// (ray, primitive) pair from the ray's stored final state (last sample j_end
// and, if clamped, T before the clamp) without any per-sample storage:
//   Tdot = dL/dA (unclamped)  or  -g . C_S / sigma_S (clamped at sample S)
//   dL/dsigma_kj = dt (Tdot + g . c_kj),   dL/dc_kj = dt sigma_kj g      (j < S)
//   dL/dsigma_kS = (1 - T_{S-1}) (g . c_kS + Tdot) / sigma_S
//   dL/dc_kS     = (1 - T_{S-1}) (sigma_kS / sigma_S) g
// and for the sequential combine Tdot = -g . c_k*S, the primitives before k*
// at S take the j < S formulas, dL/dc_k*S = (1 - T*) g with T* the opacity
// just before k*, and dL/dsigma_k*S = 0.
// The pairs are replayed by work items, each up to 32 or 64 culling-list
// entries (screen tile, primitive) of one primitive: channel adjoints go to
// the 8 voxel corners with the trilinear weights, accumulated in registers
// over a run of samples in one cell and then in an LDS copy of the
// primitive's gradient held in 64-bit fixed point (LDS 64-bit integer atomic
// adds run about 25 times faster than FP32 ones on gfx950, and integer sums do
// not depend on the order of the additions), which is added to device memory
// once per item; the pose gradient (through y = A (o + t d - pos)) is reduced
// over the workgroup.  The fixed-point scale of an item is chosen from a bound
// on what any one of its pairs can add to one gradient value: every single
// addend then fits 32 bits and no 64-bit sum can overflow.
//
// Built with -ffp-contract=off; fused multiply-adds are written explicitly.
#include <hip/hip_runtime.h>
#include <stdlib.h>

#include <algorithm>
#include <type_traits>
#include <climits>

#include "internal.h"
#include "pairs.h"

namespace mvp {

// Largest number of culling-list entries per backward work item (the build
// picks the number per structure, see backward_item_entries), and how the
// pairs of an item too large for the ordering buffer (below) are dealt to its
// threads.
constexpr int kItemEntries = 64;
constexpr bool kChunkedPairs = true;
// Lanes accumulate in cell coordinates mirrored by (lane mod 8), so lanes that
// flush the same cell add to different corners in each instruction.
constexpr bool kRotateFlush = true;
// The pairs of a work item are ordered by their number of samples (longest
// first) and dealt round-robin, so the lanes of a wave replay pairs of about
// the same length together; pairs without samples are dropped.
#ifndef MVP_SORT_PAIRS
#define MVP_SORT_PAIRS 1
#endif
constexpr bool kSortPairs = MVP_SORT_PAIRS;
constexpr int kLenBuckets = 64;

template <bool BF16>
struct Voxels;

template <>
struct Voxels<false> {
  static __device__ __forceinline__ float4 load(const void *p, size_t i) {
    return ((const float4 *)p)[i];
  }
};

template <>
struct Voxels<true> {
  static __device__ __forceinline__ float4 load(const void *p, size_t i) {
    const uint2 w = ((const uint2 *)p)[i];
    return make_float4(__uint_as_float(w.x << 16), __uint_as_float(w.x & 0xffff0000u),
                       __uint_as_float(w.y << 16), __uint_as_float(w.y & 0xffff0000u));
  }
};

// Position of sample tau in a primitive's voxel grid (align-corners): index of
// the lower corner of the cell and the fractional offsets.
struct Cell {
  int idx;      // (iz*M + iy)*M + ix of corner (0,0,0)
  int i[3];     // ix, iy, iz of corner (0,0,0)
  float f[3];
};

__device__ __forceinline__ Cell locate(const float4 &A, const float4 &B, float tau, int M, float hM) {
  const float y[3] = {fmaf(tau, B.x, A.x), fmaf(tau, B.y, A.y), fmaf(tau, B.z, A.z)};
  const float top = (float)(M - 2), Mf = (float)M;
  Cell c;
  float qf[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    // u is in [0, M-1] (fma(-1, hM, hM) is exactly 0), so the lower corner is
    // floor(u), except u = M-1, which belongs to the last cell with offset 1
    const float yc = fminf(fmaxf(y[i], -1.0f), 1.0f);
    const float u = fmaf(yc, hM, hM);
    qf[i] = fminf(floorf(u), top);
    c.i[i] = (int)qf[i];
    c.f[i] = u - qf[i];
  }
  // the index from the float coordinates: every term is an integer below 2^24
  // (M <= 1024), so the two fused multiply-adds are exact, and they are full
  // rate where a 32-bit integer multiply-add is not
  c.idx = (int)fmaf(fmaf(qf[2], Mf, qf[1]), Mf, qf[0]);
  return c;
}


// Deterministic in-workgroup compaction of the active pixels of a tile.
// Returns the number of active pixels; s_list receives their local indices
// in pixel order.
__device__ __forceinline__ int compact_tile(bool act, int *s_list, int *s_wave) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  const unsigned long long m = __ballot(act);
  const int pre = __popcll(m & ((1ull << lane) - 1ull));
  if (lane == 0) s_wave[wave] = __popcll(m);
  __syncthreads();
  int base = 0, total = 0;
#pragma unroll
  for (int w = 0; w < kTileThreads / kWave; ++w) {
    if (w < wave) base += s_wave[w];
    total += s_wave[w];
  }
  if (act) s_list[base + pre] = threadIdx.x;
  __syncthreads();
  return total;
}


// ---------------------------------------------------------------------------
// forward
// ---------------------------------------------------------------------------

// Trilinear RGBA from the 8 cached corners of a cell (corner q = dx + 2 dy + 4 dz):
// the 8 corner weights once, then one weighted sum per channel.
__device__ __forceinline__ float4 trilerp(const float4 (&v)[8], const Cell &c) {
  const float fx = c.f[0], fy = c.f[1], fz = c.f[2];
  const float gx = 1.0f - fx, gy = 1.0f - fy, gz = 1.0f - fz;
  const float yz[4] = {gy * gz, fy * gz, gy * fz, fy * fz};
  float4 r = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const float w = ((q & 1) ? fx : gx) * yz[q >> 1];
    r.x = fmaf(w, v[q].x, r.x);
    r.y = fmaf(w, v[q].y, r.y);
    r.z = fmaf(w, v[q].z, r.z);
    r.w = fmaf(w, v[q].w, r.w);
  }
  return r;
}

template <bool BF16>
__device__ __forceinline__ void load_corners(const void *pay, size_t b0, int M, float4 (&v)[8]) {
  const size_t MM = (size_t)M * M;
  v[0] = Voxels<BF16>::load(pay, b0);
  v[1] = Voxels<BF16>::load(pay, b0 + 1);
  v[2] = Voxels<BF16>::load(pay, b0 + M);
  v[3] = Voxels<BF16>::load(pay, b0 + M + 1);
  v[4] = Voxels<BF16>::load(pay, b0 + MM);
  v[5] = Voxels<BF16>::load(pay, b0 + MM + 1);
  v[6] = Voxels<BF16>::load(pay, b0 + MM + M);
  v[7] = Voxels<BF16>::load(pay, b0 + MM + M + 1);
}

__device__ __forceinline__ int prim_of(const float4 &A) { return __float_as_int(A.w); }

// Opacity fade window of Sec. 3.1.3 at the voxel centres of one axis,
// w(i) = exp(-alpha |x_i|^beta), x_i = -1 + 2i/(M-1); W(ix,iy,iz) = w(ix) w(iy) w(iz).
__device__ __forceinline__ void fill_fade(float *tab, int M, float alpha, float beta) {
  for (int i = threadIdx.x; i < M; i += blockDim.x) {
    const float x = fabsf(-1.0f + 2.0f * (float)i / (float)(M - 1));
    // |x|^beta (beta > 0) as exp2(beta log2 |x|), all in FP32
    const float xb = x > 0.0f ? exp2f(beta * log2f(x)) : 0.0f;
    tab[i] = expf(-alpha * xb);
  }
}

// Window of the 8 corners of a cell (corner q = dx + 2 dy + 4 dz).
__device__ __forceinline__ void corner_fade(const float *tab, const Cell &c, float (&wq)[8]) {
  const float wx[2] = {tab[c.i[0]], tab[c.i[0] + 1]};
  const float wy[2] = {tab[c.i[1]], tab[c.i[1] + 1]};
  const float wz[2] = {tab[c.i[2]], tab[c.i[2] + 1]};
#pragma unroll
  for (int q = 0; q < 8; ++q) wq[q] = wx[q & 1] * wy[(q >> 1) & 1] * wz[q >> 2];
}

// A ray's unit direction, read where it is kept (registers, or a column of
// LDS with a stride, which frees three registers in the forward march).
struct Dir {
  const float *p;
  int stride;
  __device__ __forceinline__ void get(float d[3]) const {
    d[0] = p[0];
    d[1] = p[stride];
    d[2] = p[2 * stride];
  }
};

// Where a ray finds the frames of its tile's culling-list entries: staged in
// LDS (four float4 per entry: the three rows of A with a_i in .w, then the
// primitive id as int bits in .x) or, for long lists, the entry frames in
// device memory.  local() rebuilds the pair's local ray y(t) = a + t b with
// b = A d in the build's canonical arithmetic, so sample positions and the
// pair's sample interval come from the same values.
struct Frames {
  const float4 *lds;   // [4 * list length] or nullptr
  uint64_t lb;         // first culling-list entry of the tile
  // S = 1: the frames are in LDS, S = 0: in device memory, S = -1: in LDS iff
  // lds is set.  A fixed S keeps the LDS reads LDS instructions (a pointer that
  // may point to either memory is read with flat loads, which also wait for
  // every outstanding device-memory load).
  template <int S = -1>
  __device__ __forceinline__ void local(const AccelView &av, int pos, const Dir &dir, float4 &A, float4 &B) const {
    float d[3];
    dir.get(d);
    float4 f0, f1, f2;
    int k;
    if (S == 1 || (S == -1 && lds)) {
      f0 = lds[4 * pos];
      f1 = lds[4 * pos + 1];
      f2 = lds[4 * pos + 2];
      k = __float_as_int(lds[4 * pos + 3].x);
    } else {
      const uint64_t g = lb + (uint64_t)pos;
      f0 = av.ef[3 * g];
      f1 = av.ef[3 * g + 1];
      f2 = av.ef[3 * g + 2];
      k = (int)av.tile_list[g];
    }
    A = make_float4(f0.w, f1.w, f2.w, __int_as_float(k));
    B = make_float4(row_dot(f0.x, f0.y, f0.z, d), row_dot(f1.x, f1.y, f1.z, d), row_dot(f2.x, f2.y, f2.z, d), 0.f);
  }
};

// Tile of a ray slot.
__device__ __forceinline__ int slot_tile(const AccelView &av, size_t slot) {
  int v, px, py;
  slot_pixel(av, slot, &v, &px, &py);
  return (v * av.tiles_y + py / kTile) * av.tiles_x + px / kTile;
}

// RGBA at tau of the pair with local ray (A, B) (primitive id in A.w):
// trilinear payload of its primitive (opacity times the fade window when FADE).
template <bool BF16, bool FADE>
__device__ __forceinline__ float4 sample_pair(const AccelView &av, const void *pay, const float *fade, const float4 &A,
                                              const float4 &B, float tau) {
  const int M = av.M;
  const float hM = 0.5f * (float)(M - 1);
  const Cell c = locate(A, B, tau, M, hM);
  float4 v[8];
  load_corners<BF16>(pay, (size_t)prim_of(A) * M * M * M + c.idx, M, v);
  if (FADE) {
    float wq[8];
    corner_fade(fade, c, wq);
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q].w *= wq[q];
  }
  return trilerp(v, c);
}

// Accumulated state of one ray, with its counts of samples and of loads
// (voxel-corner sets, pair records, entry frames read from device memory).
struct RayState {
  float T = 0.f, I0 = 0.f, I1 = 0.f, I2 = 0.f, t_prev = -1.0f;
  int j_end = -1;
  uint32_t n_ray = 0, n_prim = 0, n_cell = 0, n_pj = 0, n_pab = 0;
};

// One clamped additive step with the summed density sig and summed
// density-weighted colour (c0,c1,c2) of sample j.  Returns true to stop.
__device__ __forceinline__ bool composite(RayState &st, int j, float sig, float c0, float c1, float c2,
                                          float dt, float lim) {
  st.j_end = j;
  const float Tn = st.T + sig * dt;
  if (Tn <= 1.0f) {
    st.T = Tn;
    st.I0 = fmaf(c0, dt, st.I0);
    st.I1 = fmaf(c1, dt, st.I1);
    st.I2 = fmaf(c2, dt, st.I2);
    return st.T > lim;
  }
  const float w = (1.0f - st.T) / sig;
  st.I0 = fmaf(c0, w, st.I0);
  st.I1 = fmaf(c1, w, st.I1);
  st.I2 = fmaf(c2, w, st.I2);
  st.t_prev = st.T;
  st.T = 1.0f;
  return true;
}

// Among the ray's pairs [0, n) (sorted by first sample) that contain sample
// j, the one with the smallest primitive id above `after`; n if none.
__device__ __forceinline__ int next_by_id(const AccelView &av, uint32_t seg, int stride, int n, int j, int after) {
  int best = INT_MAX, bi = n;
  for (int i = 0; i < n; ++i) {
    const int4 r = av.pr[seg + i * stride];
    if (r.x > j) break;
    if (r.y < j) continue;
    if (r.w > after && r.w < best) {
      best = r.w;
      bi = i;
    }
  }
  return bi;
}

// Sequential combine at sample j, whose summed step saturates: the
// primitives containing j in increasing id, each with its own clamp step.
// Returns true to stop.
template <bool BF16, bool FADE, bool STAGED>
__device__ bool seq_sample(const AccelView &av, const Frames &fr, const void *pay, const float *fade, uint32_t seg,
                           int stride, int n, const Dir &d, int j, RayState &st) {
  const float dt = av.step;
  const float tau = (float)j * dt;
  const float T0 = st.T;
  st.j_end = j;
  int last = -1;
  for (int i = next_by_id(av, seg, stride, n, j, last); i < n; i = next_by_id(av, seg, stride, n, j, last)) {
    const int4 r = av.pr[seg + i * stride];
    float4 A, B;
    fr.template local<STAGED ? 1 : 0>(av, r.z, d, A, B);
    const float4 s = sample_pair<BF16, FADE>(av, pay, fade, A, B, tau);
    const float Tn = st.T + s.w * dt;
    if (Tn <= 1.0f) {
      st.T = Tn;
      st.I0 = fmaf(s.w * s.x, dt, st.I0);
      st.I1 = fmaf(s.w * s.y, dt, st.I1);
      st.I2 = fmaf(s.w * s.z, dt, st.I2);
    } else {
      const float u = 1.0f - st.T;
      st.I0 = fmaf(s.x, u, st.I0);
      st.I1 = fmaf(s.y, u, st.I1);
      st.I2 = fmaf(s.z, u, st.I2);
      st.t_prev = T0;
      st.T = 1.0f;
      return true;
    }
    last = r.w;
  }
  // rounding kept every per-primitive step at or below 1: an ordinary sample
  return st.T > 1.0f - av.eps;
}

// The samples J..J+kWin-1 of a ray are gathered pair by pair into per-sample
// sums held in registers (a pair's 8 voxel corners stay in registers while
// consecutive samples remain in one cell), then composited in sample order.
// The ray's pairs are sorted by (first sample, primitive id): a window visits
// only the pairs that overlap it, and the primitives of one sample are summed
// in primitive-id order within each group of pairs with the same first sample.
constexpr int kWin = 12;

// OPAQUE_J (used where the kernel also runs the pairs pass or applies the fade
// window, and is short of registers): the window start is hidden from
// loop-invariant code motion, so
// the window's sample times are recomputed for each pair instead of being held
// in about two dozen registers across the pair loop.  Same arithmetic either way.
template <bool BF16, bool FADE, bool OPAQUE_J, bool STAGED>
__device__ void march_ray(const AccelView &av, const Frames &fr, const void *pay, const float *fade, uint32_t seg,
                          int stride, int n, const Dir &d, RayState &st) {
  const float dt = av.step, lim = 1.0f - av.eps;
  const int M = av.M;
  const float hM = 0.5f * (float)(M - 1);
  const size_t M3 = (size_t)M * M * M;
  int e0 = 0;                  // pairs before e0 have ended before the window
  int4 q0 = av.pr[seg];        // record e0, kept across windows: it opens the next window's pair loop
  ++st.n_pj;
  int J = q0.x;
  while (true) {
    float as[kWin], ar[kWin], ag[kWin], ab[kWin];
    // samples of the window inside at least one primitive, and the number of
    // primitives containing each, 8 bits per sample (exact when the ray has
    // at most 255 pairs; longer lists count their prim-samples afterwards)
    uint32_t occ = 0, cp[kWin / 4] = {};
#pragma unroll
    for (int w = 0; w < kWin; ++w) as[w] = ar[w] = ag[w] = ab[w] = 0.f;
    const int J1 = J + kWin;
    int4 rn = q0;                // record i; record i + 1 is requested before pair i is marched
    for (int i = e0; i < n; ++i) {
      const int4 r = rn;
      if (r.x >= J1) break;
      if (i + 1 < n) {   // the next record is in flight while this pair is marched
        rn = av.pr[seg + (i + 1) * stride];
        ++st.n_pj;
      }
      if (r.y < J) continue;
      const int lo = max(r.x, J) - J, hi = min(r.y, J1 - 1) - J;
      occ |= ((2u << hi) - 1u) & ~((1u << lo) - 1u);
      float4 A, B;
      fr.template local<STAGED ? 1 : 0>(av, r.z, d, A, B);
      if (!STAGED) ++st.n_pab;
      const size_t kb = (size_t)prim_of(A) * M3;
      int cur = -1;
      int Jp = J;
      if (OPAQUE_J) asm volatile("" : "+v"(Jp));
      float4 v[8];
#pragma unroll
      for (int w = 0; w < kWin; ++w) {
        if (w >= lo && w <= hi) {
          const float tau = (float)(Jp + w) * dt;
          const Cell c = locate(A, B, tau, M, hM);
          if (c.idx != cur) {
            load_corners<BF16>(pay, kb + c.idx, M, v);
            ++st.n_cell;
            if (FADE) {
              float wq[8];
              corner_fade(fade, c, wq);
#pragma unroll
              for (int q = 0; q < 8; ++q) v[q].w *= wq[q];
            }
            cur = c.idx;
          }
          const float4 sv = trilerp(v, c);
          as[w] += sv.w;
          ar[w] = fmaf(sv.w, sv.x, ar[w]);
          ag[w] = fmaf(sv.w, sv.y, ag[w]);
          ab[w] = fmaf(sv.w, sv.z, ab[w]);
          cp[w / 4] += 1u << (8 * (w % 4));
        }
      }
    }
    // composite the occupied samples in order; a sample whose summed step
    // saturates under the sequential combine leaves the unrolled loop and is
    // taken primitive by primitive, then the loop resumes after it
    bool stop = false;
    int w0 = 0;
    while (!stop && w0 < kWin) {
      int wseq = kWin;
#pragma unroll
      for (int w = 0; w < kWin; ++w) {
        if (w >= w0 && !stop && wseq == kWin && ((occ >> w) & 1u)) {
          ++st.n_ray;
          st.n_prim += (cp[w / 4] >> (8 * (w % 4))) & 0xffu;
          if (av.combine && st.T + as[w] * dt > 1.0f) wseq = w;
          else stop = composite(st, J + w, as[w], ar[w], ag[w], ab[w], dt, lim);
        }
      }
      if (wseq < kWin) stop = seq_sample<BF16, FADE, STAGED>(av, fr, pay, fade, seg, stride, n, d, J + wseq, st);
      w0 = wseq + 1;
    }
    if (stop) break;
    // next occupied sample: every pair in front of e0 ends before J1, and all
    // later pairs start no earlier than e0 does
    while (q0.y < J1) {
      if (++e0 == n) break;
      q0 = av.pr[seg + e0 * stride];
      ++st.n_pj;
    }
    if (e0 == n) break;
    J = max(J1, q0.x);
  }
  if (n > 255) {   // the 8-bit per-sample counts may have wrapped: count the samples up to the last one
    uint32_t np = 0;
    for (int i = 0; i < n; ++i) {
      const int4 r = av.pr[seg + i * stride];
      np += (uint32_t)max(0, min(r.y, st.j_end) - r.x + 1);
    }
    st.n_prim = np;
  }
}

// Frames of a tile's culling list staged in LDS when the list has at most
// this many entries.
constexpr int kFrameLds = 256;

// BUILD: the workgroup first builds its tile's pairs (the pairs pass of the
// build, tile_pairs), then marches them; the records it reads back were
// written by other threads of the workgroup before the barrier.
template <bool BF16, bool FADE, bool BUILD>
__global__ __launch_bounds__(kTileThreads) __attribute__((amdgpu_waves_per_eu(3))) void k_march_fwd(
    AccelView av, const void *__restrict__ pay, const float *__restrict__ bg, float4 *__restrict__ rgba,
    mvp_ray_aux *__restrict__ aux, unsigned long long *__restrict__ counters, PairsOut po) {
  __shared__ int s_list[kTileThreads];
  __shared__ int s_wave[kTileThreads / kWave];
  __shared__ float4 s_frm[4 * kFrameLds];
  __shared__ float s_dir[3][kTileThreads];
  extern __shared__ float s_fade[];   // [M] when FADE
  const int slot = xcd_tile(blockIdx.x, av.V * av.tiles_x * av.tiles_y);
  if (slot < 0) return;
  const int tile = split_tile(slot, av.tiles_x, av.tiles_y, view_splits(av.V));
  if (BUILD) {
    tile_pairs(av, tile, po);
    __syncthreads();
  }
  if (FADE) fill_fade(s_fade, av.M, av.fade_alpha, av.fade_beta);   // visible after compact_tile's barrier
  const uint64_t lb = av.tile_off[tile], len = av.tile_off[tile + 1] - lb;
  const bool staged = len <= (uint64_t)kFrameLds;
  unsigned long long n_stage = 0;
  if (staged) {   // the tile's entry frames (visible after compact_tile's barrier)
    for (int e = threadIdx.x; e < (int)len; e += kTileThreads) {
#pragma unroll
      for (int r = 0; r < 3; ++r) s_frm[4 * e + r] = av.ef[3 * (lb + e) + r];
      s_frm[4 * e + 3] = make_float4(__int_as_float((int)av.tile_list[lb + e]), 0.f, 0.f, 0.f);
      ++n_stage;
    }
  }
  int total;
  {
    size_t ray;
    int v, px, py;
    const bool valid = tile_ray(av, tile, threadIdx.x, &ray, &v, &px, &py);
    bool act = false;
    if (valid) {
      act = av.ray_nj[ray].x > 0;
      if (!act) {
        float4 o = make_float4(0.f, 0.f, 0.f, 0.f);
        if (bg) o = make_float4(bg[3 * ray], bg[3 * ray + 1], bg[3 * ray + 2], 0.f);
        rgba[ray] = o;
        if (aux) aux[ray] = mvp_ray_aux{-1, -1.0f};
      }
    }
    total = compact_tile(act, s_list, s_wave);
  }
  RayState st;
  if ((int)threadIdx.x < total) {
    size_t ray;
    int v, px, py;
    tile_ray(av, tile, s_list[threadIdx.x], &ray, &v, &px, &py);
    float d[3];
    pixel_ray(av.cams[v], px, py, d);
#pragma unroll
    for (int i = 0; i < 3; ++i) s_dir[i][threadIdx.x] = d[i];
    const uint32_t seg = (uint32_t)av.ray_seg[ray];
    const int stride = tile_ray_count(av, tile), n = av.ray_nj[ray].x;
    const Dir dir{&s_dir[0][threadIdx.x], kTileThreads};
    if (staged) march_ray<BF16, FADE, BUILD || FADE, true>(av, Frames{s_frm, lb}, pay, s_fade, seg, stride, n, dir, st);
    else march_ray<BF16, FADE, BUILD || FADE, false>(av, Frames{nullptr, lb}, pay, s_fade, seg, stride, n, dir, st);
    if (bg) {   // composite over the background: I + (1 - A) B
      const float u = 1.0f - st.T;
      st.I0 = fmaf(u, bg[3 * ray], st.I0);
      st.I1 = fmaf(u, bg[3 * ray + 1], st.I1);
      st.I2 = fmaf(u, bg[3 * ray + 2], st.I2);
    }
    rgba[ray] = make_float4(st.I0, st.I1, st.I2, st.T);
    if (aux) aux[ray] = mvp_ray_aux{st.j_end, st.t_prev};
  }
  if (counters) {
    const unsigned long long c[5] = {wave_sum_u64(st.n_ray), wave_sum_u64(st.n_prim), wave_sum_u64(st.n_cell),
                                     wave_sum_u64(st.n_pj), wave_sum_u64(st.n_pab + n_stage)};
    if ((threadIdx.x & (kWave - 1)) == 0 && (c[3] | c[4])) {
#pragma unroll
      for (int i = 0; i < 5; ++i) atomicAdd(&counters[i], c[i]);
    }
  }
}

hipError_t launch_march_fwd(const AccelView &av, const mvp_prims &p, const float *bg, float *rgba,
                            mvp_ray_aux *aux, unsigned long long *counters, hipStream_t s,
                            const PairsOut *build_pairs) {
  const int ntile = av.V * av.tiles_x * av.tiles_y;
  if (ntile == 0) return hipSuccess;
  const bool fade = av.fade_alpha > 0.f;
  const size_t shm = fade ? (size_t)av.M * sizeof(float) : 0;
  const PairsOut po = build_pairs ? *build_pairs : PairsOut{};
#define MVP_FWD(B, F, P)                                                                                     \
  hipLaunchKernelGGL((k_march_fwd<B, F, P>), dim3(xcd_grid(ntile)), dim3(kTileThreads), shm, s, av, p.payload, \
                     bg, (float4 *)rgba, aux, counters, po)
#define MVP_FWD_P(B, F)                  \
  do {                                   \
    if (build_pairs) MVP_FWD(B, F, true); \
    else MVP_FWD(B, F, false);           \
  } while (0)
  if (p.payload_dtype == MVP_BF16) {
    if (fade) MVP_FWD_P(true, true); else MVP_FWD_P(true, false);
  } else {
    if (fade) MVP_FWD_P(false, true); else MVP_FWD_P(false, false);
  }
#undef MVP_FWD_P
#undef MVP_FWD
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// backward
// ---------------------------------------------------------------------------

// Per-ray constants of the adjoint.  Tdot is dL/dA for an unclamped ray and
// -g . C_S/sigma_S for a ray clamped at its last sample S, with the weight
// (1 - T_{S-1}) / sigma_S (recomputed here from the pairs open at S).  For
// the sequential combine the clamping primitive k* is found again by
// replaying the per-primitive steps of S from T_{S-1} with the forward's
// arithmetic; then Tdot = -g . c_k*, the weight is 1 - T* and kstar = k*.
// With a background B the output colour is I + (1 - A) B: the upstream of A
// becomes dL/dA - g . B, and dL/dB = (1 - A) g is accumulated here.
//
// Also the ray's bounds for the fixed-point accumulation (RayBound): a replayed
// sample adds to one gradient value of a corner at most its trilinear weight
// (<= 1) times dL/dsigma_k or dL/dc_k.  Away from the clamp
// |dL/dsigma_k| <= dt (|Tdot| + |g|_1 Cmax) and |dL/dc_k| <= dt sigma_max |g|_inf
// (Cmax, sigma_max: the payload's largest colour and opacity magnitudes; the
// fade window only lowers them); at the clamping sample dL/dsigma_k has the
// weight (1 - T_{S-1}) / sigma_S < dt in place of dt and the colour adjoint is
// at most |g|_inf (sum rule: (1 - T_{S-1}) sigma_k / sigma_S <= 1; sequential:
// 1 - T* <= 1).
// Rays per workgroup of k_bwd_rays (4 per thread).  Only the clamped rays
// (about one in eight on a typical frame) replay a sample; they are gathered
// in LDS first, so that the replay runs on full waves instead of on the few
// lanes of every wave whose ray clamped.
constexpr int kBwdRaysPerBlock = 1024;

template <bool BF16, bool FADE>
__global__ __launch_bounds__(256) void k_bwd_rays(AccelView av, const void *__restrict__ pay,
                                                  const mvp_ray_aux *__restrict__ aux,
                                                  const float4 *__restrict__ grad_rgba,
                                                  const float *__restrict__ bg, const float4 *__restrict__ rgba,
                                                  RayConst *__restrict__ rc, RayBound *__restrict__ rbd,
                                                  const uint32_t *__restrict__ pmax, float *__restrict__ g_bg,
                                                  size_t R) {
  extern __shared__ float s_fade[];
  __shared__ uint32_t s_clamped[kBwdRaysPerBlock];
  __shared__ int s_nc;
  if (threadIdx.x == 0) s_nc = 0;
  if (FADE) fill_fade(s_fade, av.M, av.fade_alpha, av.fade_beta);
  __syncthreads();
  const float cmax = __uint_as_float(pmax[0]), smax = __uint_as_float(pmax[1]);
  const size_t base = (size_t)blockIdx.x * kBwdRaysPerBlock;
  // dL/dA of the ray (with a background, of the composite over it)
  auto base_tdot = [&](size_t r, const float4 &g) {
    float t = g.w;
    if (bg) t -= g.x * bg[3 * r] + g.y * bg[3 * r + 1] + g.z * bg[3 * r + 2];
    return t;
  };
  auto write = [&](size_t r, const float4 &g, float tdot, float wsig, int kstar, bool clamped) {
    rc[r] = RayConst{tdot, wsig, kstar, 0};
    const float g1 = fabsf(g.x) + fabsf(g.y) + fabsf(g.z);
    const float gi = fmaxf(fabsf(g.x), fmaxf(fabsf(g.y), fabsf(g.z)));
    rbd[r] = RayBound{av.step * (fabsf(tdot) + g1 * cmax + smax * gi), clamped ? gi : 0.f};
  };
  for (int o = 0; o < kBwdRaysPerBlock; o += 256) {
    const size_t r = base + o + threadIdx.x;
    if (r >= R) break;
    const mvp_ray_aux ax = aux[r];
    const float4 g = grad_rgba[r];
    if (bg && g_bg) {
      const float u = 1.0f - rgba[r].w;
      g_bg[3 * r] += u * g.x;
      g_bg[3 * r + 1] += u * g.y;
      g_bg[3 * r + 2] += u * g.z;
    }
    if (ax.j_end >= 0 && ax.t_prev >= 0.f) s_clamped[atomicAdd(&s_nc, 1)] = (uint32_t)(o + threadIdx.x);
    else write(r, g, base_tdot(r, g), 0.f, -1, false);
  }
  __syncthreads();
  const int nc = s_nc;
  for (int ci = threadIdx.x; ci < nc; ci += blockDim.x) {
    const size_t r = base + s_clamped[ci];
    const mvp_ray_aux ax = aux[r];
    const float4 g = grad_rgba[r];
    float tdot = base_tdot(r, g), wsig = 0.f;
    int kstar = -1;
    // the ray's pairs open at its last sample, in increasing primitive id as
    // the forward visited them
    const float tau = (float)ax.j_end * av.step;
    const int tile = slot_tile(av, r);
    const Frames fr{nullptr, av.tile_off[tile]};
    int v, px, py;
    slot_pixel(av, r, &v, &px, &py);
    float d[3];
    pixel_ray(av.cams[v], px, py, d);
    const uint32_t seg = (uint32_t)av.ray_seg[r];
    const int stride = tile_ray_count(av, tile);
    const int n = av.ray_nj[r].x;
    if (av.combine) {
      float T = ax.t_prev;
      int last = -1;
      for (int i = next_by_id(av, seg, stride, n, ax.j_end, last); i < n; i = next_by_id(av, seg, stride, n, ax.j_end, last)) {
        const int4 pq = av.pr[seg + i * stride];
        float4 A, B;
        fr.local(av, pq.z, Dir{d, 1}, A, B);
        const float4 s = sample_pair<BF16, FADE>(av, pay, s_fade, A, B, tau);
        const float Tn = T + s.w * av.step;
        last = pq.w;
        if (Tn > 1.0f) {
          kstar = prim_of(A);
          tdot = -(g.x * s.x + g.y * s.y + g.z * s.z);
          wsig = 1.0f - T;
          break;
        }
        T = Tn;
      }
    } else {
      // the pairs open at S, in list order (the order the forward summed them
      // in); their records are read four at a time, so that the scan does not
      // wait for one record before asking for the next
      float sig = 0.f, c0 = 0.f, c1 = 0.f, c2 = 0.f;
      constexpr int kB = 4;
      for (int i0 = 0; i0 < n; i0 += kB) {
        int4 q[kB];
#pragma unroll
        for (int k = 0; k < kB; ++k)
          q[k] = i0 + k < n ? av.pr[seg + (i0 + k) * stride] : make_int4(INT_MAX, INT_MIN, 0, 0);
#pragma unroll
        for (int k = 0; k < kB; ++k) {
          if (q[k].x > ax.j_end || q[k].y < ax.j_end) continue;
          float4 A, B;
          fr.local(av, q[k].z, Dir{d, 1}, A, B);
          const float4 s = sample_pair<BF16, FADE>(av, pay, s_fade, A, B, tau);
          sig += s.w;
          c0 = fmaf(s.w, s.x, c0);
          c1 = fmaf(s.w, s.y, c1);
          c2 = fmaf(s.w, s.z, c2);
        }
        if (q[kB - 1].x > ax.j_end) break;   // sorted by first sample: no later pair is open
      }
      tdot = -(g.x * (c0 / sig) + g.y * (c1 / sig) + g.z * (c2 / sig));
      wsig = (1.0f - ax.t_prev) / sig;
    }
    write(r, g, tdot, wsig, kstar, !av.combine || kstar >= 0);
  }
}

// Largest colour and opacity magnitudes of the payload, as float bits in
// pmax[0] and pmax[1] (which start at zero; non-negative floats order like
// their bit patterns).
template <bool BF16>
__global__ __launch_bounds__(256) void k_payload_bound(const void *__restrict__ pay, size_t n_vox,
                                                       uint32_t *__restrict__ pmax) {
  float c = 0.f, sg = 0.f;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_vox; i += (size_t)gridDim.x * blockDim.x) {
    const float4 v = Voxels<BF16>::load(pay, i);
    c = fmaxf(c, fmaxf(fabsf(v.x), fmaxf(fabsf(v.y), fabsf(v.z))));
    sg = fmaxf(sg, fabsf(v.w));
  }
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) {
    c = fmaxf(c, __shfl_xor(c, d, kWave));
    sg = fmaxf(sg, __shfl_xor(sg, d, kWave));
  }
  // one pair of atomics per workgroup: atomics on one address are serialised
  // at the L2, so their number, not the payload read, sets this kernel's time
  __shared__ float s_c[256 / kWave], s_s[256 / kWave];
  const int wave = threadIdx.x / kWave;
  if ((threadIdx.x & (kWave - 1)) == 0) {
    s_c[wave] = c;
    s_s[wave] = sg;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 256 / kWave; ++w) {
      c = fmaxf(c, s_c[w]);
      sg = fmaxf(sg, s_s[w]);
    }
    atomicMax(&pmax[0], __float_as_uint(c));
    atomicMax(&pmax[1], __float_as_uint(sg));
  }
}

struct BwdOut {
  float *pay, *pos, *rot, *scale;
};


// The LDS copy of a primitive's payload gradient is planar: channel ch of
// voxel (ix, iy, iz) at ch * plane + ix + iy * sy + iz * sz.  A wave adds one
// channel of one corner per instruction, and the lanes working in one cell add
// to its 8 different corners (see the mirrored lanes in bwd_pair); with 64-bit
// words a bank pair is a word index mod 16, so the strides are padded until
// the 8 corner offsets {0, 1} + {0, sy} + {0, sz} fall on 8 different bank
// pairs (8^3: sy = 8, sz = 66), when the padded copy fits the LDS; otherwise
// the copy is packed (sy = M, sz = M^2, plane = M^3 + 1).
struct LdsMap {
  int sy, sz, plane;
};

__host__ __device__ inline LdsMap lds_map(int M, bool padded) {
  if (!padded) return LdsMap{M, M * M, M * M * M + 1};
  auto distinct = [](int a, int b) {   // {0, 1, a, a + 1, b, b + 1, a + b, a + b + 1} mod 16
    int seen = 0;
    const int v[8] = {0, 1, a, a + 1, b, b + 1, a + b, a + b + 1};
    for (int i = 0; i < 8; ++i) {
      const int bit = 1 << (v[i] & 15);
      if (seen & bit) return false;
      seen |= bit;
    }
    return true;
  };
  int sy = M;
  while ((sy & 15) == 0 || (sy & 15) == 1 || (sy & 15) == 15) ++sy;
  int sz = sy * M;
  while (!distinct(sy, sz)) ++sz;
  return LdsMap{sy, sz, sz * M};
}

// One addend of the fixed-point accumulator: v * scale rounded to the nearest
// integer (|v * scale| < 2^30 by the choice of scale), sign-extended to the
// 64-bit two's complement word that the LDS atomic adds.
__device__ __forceinline__ unsigned long long fixed_addend(float v, float scale) {
  return (unsigned long long)(long long)__float2int_rn(v * scale);
}

template <bool LDS_ACC, bool FADE, typename T>
__device__ __forceinline__ void flush_cell(T *dst, size_t cell, int M, const LdsMap &lm, const float (&acc)[8][4],
                                           const float (&wq)[8], unsigned slots, unsigned m, float scale) {
  // cell: LDS slot of corner (0,0,0) (LDS_ACC) or its voxel index in device memory
  const size_t sy = LDS_ACC ? (size_t)lm.sy : (size_t)M, sz = LDS_ACC ? (size_t)lm.sz : (size_t)M * M;
  const size_t plane = (size_t)lm.plane;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    if (!((slots >> q) & 1u)) continue;
    const unsigned r = (unsigned)q ^ m;
    const size_t vox = cell + (r & 1u) + ((r >> 1) & 1u) * sy + (r >> 2) * sz;
    const float a3 = FADE ? acc[q][3] * wq[q] : acc[q][3];
    if constexpr (LDS_ACC) {
      atomicAdd(dst + vox, fixed_addend(acc[q][0], scale));
      atomicAdd(dst + plane + vox, fixed_addend(acc[q][1], scale));
      atomicAdd(dst + 2 * plane + vox, fixed_addend(acc[q][2], scale));
      atomicAdd(dst + 3 * plane + vox, fixed_addend(a3, scale));
    } else {
      unsafeAtomicAdd(dst + vox * 4, acc[q][0]);
      unsafeAtomicAdd(dst + vox * 4 + 1, acc[q][1]);
      unsafeAtomicAdd(dst + vox * 4 + 2, acc[q][2]);
      unsafeAtomicAdd(dst + vox * 4 + 3, a3);
    }
  }
}

// Replay one (ray, primitive k) pair backward: channel adjoints to the 8
// voxel corners (registers while the samples stay in one cell, then gdst:
// the LDS copy of k's gradient or device memory) and the pair's pose sums
// added to P (sum G 3, then o_m G_i + d_m H_i 9; see pose_from_sums).
template <bool BF16, bool LDS_ACC, bool FADE, bool PREFETCH, typename GAcc>
__device__ __forceinline__ void bwd_pair(const AccelView &av, const float *__restrict__ rot,
                                         const float *__restrict__ scale, const void *__restrict__ pay,
                                         const mvp_ray_aux *__restrict__ aux, const float4 *__restrict__ grad_rgba,
                                         const RayConst *__restrict__ rc, const uint2 rec, uint64_t gent, int tile,
                                         int k, GAcc *gdst, const LdsMap &lm, float fxs, const float *s_fade, bool pose,
                                         float (&P)[12], uint32_t &runs) {
  const int M = av.M;
  const float hM = 0.5f * (float)(M - 1);
  const size_t M3 = (size_t)M * M * M;
  const float dt = av.step;
  const int2 jr = make_int2((int)(rec.x & 0xffffffu), (int)rec.y);
  size_t ray;
  int rv, px, py;
  (void)tile_ray(av, tile, (int)(rec.x >> 24), &ray, &rv, &px, &py);
  float d[3];
  pixel_ray(av.cams[rv], px, py, d);
  float4 A, B;   // the pair's local ray, from the frame of its culling-list entry gent
  const Frames fr{nullptr, gent};
  fr.local(av, 0, Dir{d, 1}, A, B);
  const mvp_ray_aux ax = aux[ray];
  const float4 g = grad_rgba[ray];
  const RayConst rcv = rc[ray];
  const float tdot = rcv.tdot, wsig = rcv.w;
  // sum rule: sample S uses the clamp formulas; sequential: only k* does
  // (primitives before it are ordinary steps, those after it add nothing)
  const bool clamped = ax.t_prev >= 0.f && (!av.combine || rcv.kstar >= 0);
  const bool seq = av.combine != 0;
  const int jh = min(jr.y, ax.j_end);
  const size_t kb = (size_t)k * M3;
  float G0 = 0.f, G1 = 0.f, G2 = 0.f, H0 = 0.f, H1 = 0.f, H2 = 0.f;
  float4 cv[8];
  float wq[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) wq[q] = 1.0f;
  // Into LDS, lane L works in the cell coordinates mirrored along the axes
  // named by the bits of m = L mod 8: its register slot q holds corner q ^ m,
  // so lanes of one wave that flush the same cell add to different voxels in
  // each instruction (instead of serialising on one address) at no cost in
  // register moves.  Mirroring an axis maps its offset f to 1 - f and flips
  // the sign of the derivative along it.
  const unsigned m = (LDS_ACC && kRotateFlush) ? (threadIdx.x & 7u) : 0u;
  const bool mx = m & 1u, my = (m >> 1) & 1u, mz = (m >> 2) & 1u;
  const float hMx = mx ? -hM : hM, hMy = my ? -hM : hM, hMz = mz ? -hM : hM;
  const float offx = mx ? 1.0f : 0.0f, offy = my ? 1.0f : 0.0f, offz = mz ? 1.0f : 0.0f;
  const int MMi = M * M;
  const int so0 = (mx ? 1 : 0) + (my ? M : 0) + (mz ? MMi : 0);   // slot 0's voxel offset
  const int sx = mx ? -1 : 1, sy = my ? -M : M, sz = mz ? -MMi : MMi;
  // One iteration per run of consecutive samples inside one voxel cell: the
  // corner loads before the run and the flush after it are executed by the
  // wave's lanes together (a per-sample "cell changed" branch would issue them
  // once per lane, with the other lanes masked off).
  // PREFETCH (where the registers allow it): the corners of a run are
  // requested before the previous run's flush, so that their loads are in
  // flight while the flush adds to LDS.
  auto load_cell = [&](int cell) {
    const ptrdiff_t b0 = (ptrdiff_t)(kb + cell) + so0;
#pragma unroll
    for (int q = 0; q < 8; ++q)
      cv[q] = Voxels<BF16>::load(pay, (size_t)(b0 + ((q & 1) ? sx : 0) + ((q & 2) ? sy : 0) + ((q & 4) ? sz : 0)));
  };
  int j = jr.x;
  Cell c;
  if (j <= jh) {
    c = locate(A, B, (float)j * dt, M, hM);
    if (PREFETCH) load_cell(c.idx);
  }
  while (j <= jh) {
    const int cell = c.idx;
    const int ci0 = c.i[0], ci1 = c.i[1], ci2 = c.i[2];
    ++runs;
    if (!PREFETCH) load_cell(cell);
    if (FADE) {
      const float wx[2] = {s_fade[ci0 + (mx ? 1 : 0)], s_fade[ci0 + (mx ? 0 : 1)]};
      const float wy[2] = {s_fade[ci1 + (my ? 1 : 0)], s_fade[ci1 + (my ? 0 : 1)]};
      const float wz[2] = {s_fade[ci2 + (mz ? 1 : 0)], s_fade[ci2 + (mz ? 0 : 1)]};
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        wq[q] = wx[q & 1] * wy[(q >> 1) & 1] * wz[q >> 2];
        cv[q].w *= wq[q];
      }
    }
    // The cell's field in the monomial basis: f = sum_q cf[q] m_q with m_q the
    // product of the offsets (x, y, z) named by the bits of q.  The ray's
    // upstream colour gradient g is fixed along the run, and every colour term
    // of a sample (g . rgb, the colour adjoint ws g and its position
    // derivative) involves the colours only through g . c: the run keeps
    // gcf[q] = g . cf[q][rgb] and the opacity coefficients sf[q] (the basis
    // change is linear, so gcf comes from the corners' g . c), and sums the
    // colour adjoint as g times sum_s m_q ws.
    float gcf[8], sf[8], bw[8], b3[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      gcf[q] = fmaf(g.z, cv[q].z, fmaf(g.y, cv[q].y, g.x * cv[q].x));
      sf[q] = cv[q].w;
      bw[q] = b3[q] = 0.f;
    }
#pragma unroll
    for (int bit = 1; bit < 8; bit <<= 1)
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (q & bit) {
          gcf[q] -= gcf[q ^ bit];
          sf[q] -= sf[q ^ bit];
        }
    do {
      const float tau = (float)j * dt;
      // offsets, mirrored where the lane's axis is: |0 - f| = f, |1 - f| = 1 - f
      // (0 <= f <= 1; the absolute value folds into the instructions that use it)
      const float fx = fabsf(offx - c.f[0]), fy = fabsf(offy - c.f[1]), fz = fabsf(offz - c.f[2]);
      const float mxy = fx * fy, mxz = fx * fz, myz = fy * fz, mxyz = mxy * fz;
      const float mq[8] = {1.0f, fx, fy, mxy, fz, mxz, myz, mxyz};
      float gc = gcf[0], sg = sf[0];
#pragma unroll
      for (int q = 1; q < 8; ++q) {
        gc = fmaf(mq[q], gcf[q], gc);
        sg = fmaf(mq[q], sf[q], sg);
      }
      float a3, ws;   // dL/dsigma and the factor of g in dL/d(rgb) for this prim-sample
      if (clamped && j == ax.j_end && (!seq || k >= rcv.kstar)) {
        a3 = seq ? 0.f : wsig * (gc + tdot);
        ws = seq ? (k == rcv.kstar ? wsig : 0.f) : wsig * sg;
      } else {
        a3 = dt * (tdot + gc);
        ws = dt * sg;
      }
      // adjoint of the monomial coefficients; the corners' are formed at the flush
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        bw[q] = fmaf(mq[q], ws, bw[q]);
        b3[q] = fmaf(mq[q], a3, b3[q]);
      }
      // gradient with respect to the cell offsets of the interpolant of the
      // adjoint-weighted channels: al[q] = a . cf[q], d/dx of sum al[q] m_q
      // (the factor dx/dy = hM, signed on mirrored axes, is applied to the
      // pair's sums G and H)
      float al[8];
#pragma unroll
      for (int q = 1; q < 8; ++q) al[q] = fmaf(ws, gcf[q], a3 * sf[q]);
      const float gx = fmaf(al[7], myz, fmaf(al[5], fz, fmaf(al[3], fy, al[1])));
      const float gyv = fmaf(al[7], mxz, fmaf(al[6], fz, fmaf(al[3], fx, al[2])));
      const float gz = fmaf(al[7], mxy, fmaf(al[6], fy, fmaf(al[5], fx, al[4])));
      G0 += gx;
      G1 += gyv;
      G2 += gz;
      H0 = fmaf(tau, gx, H0);
      H1 = fmaf(tau, gyv, H1);
      H2 = fmaf(tau, gz, H2);
      ++j;
      if (j > jh) break;
      c = locate(A, B, (float)j * dt, M, hM);
    } while (c.idx == cell);
    if (PREFETCH && j <= jh) load_cell(c.idx);
    // monomial adjoint -> corner adjoint (transpose of the basis change), on
    // the two sums before the colour adjoint is spread over the channels
#pragma unroll
    for (int bit = 1; bit < 8; bit <<= 1)
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (!(q & bit)) {
          bw[q] -= bw[q | bit];
          b3[q] -= b3[q | bit];
        }
    float acc[8][4];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      acc[q][0] = g.x * bw[q];
      acc[q][1] = g.y * bw[q];
      acc[q][2] = g.z * bw[q];
      acc[q][3] = b3[q];
    }
    if (gdst) {
      const size_t fc = LDS_ACC ? (size_t)((unsigned)ci0 + __umul24((unsigned)ci1, (unsigned)lm.sy) +
                                           __umul24((unsigned)ci2, (unsigned)lm.sz))
                                : (size_t)cell;
      flush_cell<LDS_ACC, FADE>(gdst, fc, M, lm, acc, wq, 0xffu, m, fxs);
    }
  }
  if (!pose) return;
  // y = A (o + tau d - t), A = diag(1/s) R^T, d the unit pixel ray.  The pose
  // gradient is linear in the pair's sums G = sum dL/dy and H = sum tau dL/dy,
  // and the primitive is the same for every pair of a work item, so the pair
  // adds only sum G (P[0..2]) and o_m G_i + d_m H_i (P[3 + 3m + i]); the
  // primitive's A, t, R and s are applied once per item (pose_from_sums).
  const DevCam &cam = av.cams[rv];
  const float G[3] = {hMx * G0, hMy * G1, hMz * G2}, H[3] = {hMx * H0, hMy * H1, hMz * H2};
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    P[i] += G[i];
#pragma unroll
    for (int m = 0; m < 3; ++m) P[3 + 3 * m + i] = fmaf(cam.o[m], G[i], fmaf(d[m], H[i], P[3 + 3 * m + i]));
  }
}

// Output i (0-2 dL/dt, 3-11 dL/dR row-major, 12-14 dL/ds) of primitive k's
// pose gradient from the sums of its pairs (bwd_pair): SG = sum G and
// S[m][i] = sum (o_m G_i + d_m H_i).  With P_mi = S[m][i] - t_m SG_i:
// dL/dt_m = -sum_i A_im SG_i, dL/dR_mi = P_mi / s_i,
// dL/ds_i = -sum_m R_mi P_mi / s_i^2.
__device__ __forceinline__ float pose_from_sums(const AccelView &av, const float *__restrict__ rot,
                                                const float *__restrict__ scale, int k, const float *sums,
                                                int i) {
  float Am[9], t[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const float4 row = av.xf[3 * (size_t)k + r];
    Am[3 * r] = row.x; Am[3 * r + 1] = row.y; Am[3 * r + 2] = row.z; t[r] = row.w;
  }
  if (i < 3) return -fmaf(Am[6 + i], sums[2], fmaf(Am[3 + i], sums[1], Am[i] * sums[0]));
  if (i < 12) {
    const int m = (i - 3) / 3, c = (i - 3) % 3;
    return (sums[i] - t[m] * sums[c]) / scale[3 * (size_t)k + c];
  }
  const int c = i - 12;
  const float sk = scale[3 * (size_t)k + c];
  float rp = 0.f;
#pragma unroll
  for (int m = 0; m < 3; ++m) rp = fmaf(rot[9 * (size_t)k + 3 * m + c], sums[3 + 3 * m + c] - t[m] * sums[c], rp);
  return -rp / (sk * sk);
}


// Samples the backward replays for the pair of entry record rec (of a
// culling-list entry of `tile`): its samples up to the ray's last.  Raises
// `bound` to the pair's bound on what it adds to any one payload gradient
// value (see RayBound), if larger.
// Maximum that propagates NaN (a non-finite bound must reach fixed_scale).
__device__ __forceinline__ float nan_max(float a, float b) {
  return (a == a && b == b) ? fmaxf(a, b) : __builtin_nanf("");
}

__device__ __forceinline__ int pair_len(const AccelView &av, const mvp_ray_aux *__restrict__ aux,
                                        const RayBound *__restrict__ rbd, const uint2 rec, int tile, float &bound) {
  const int2 jr = make_int2((int)(rec.x & 0xffffffu), (int)rec.y);
  size_t ray;
  int rv, px, py;
  (void)tile_ray(av, tile, (int)(rec.x >> 24), &ray, &rv, &px, &py);
  const int je = aux[ray].j_end;
  const int n = max(0, min(jr.y, je) - jr.x + 1);
  if (n > 0) {
    const RayBound rb = rbd[ray];
    const float b = (float)n * rb.per_sample + (jr.y >= je ? rb.clamp : 0.f);
    bound = nan_max(bound, b);
  }
  return n;
}

// Fixed-point scale of a work item none of whose pairs adds more than `bound`
// to any one gradient value.  A cell run adds part of one pair's share, so
// with the scale below every addend is under 2^29 (half of that covers the
// rounding of the run's sums) and fits 32 bits; an item has at most
// 64 entries x 256 rays = 2^14 pairs, so a 64-bit sum stays under 2^43.
// 0 for a non-finite bound (the item's gradient is then written as NaN).
__device__ __forceinline__ float fixed_scale(float bound) {
  if (!(bound < INFINITY)) return 0.0f;
  if (!(bound > 0.0f)) return 1.0f;
  int e;
  (void)frexpf(2.0f * bound, &e);   // 2 bound = m 2^e, 0.5 <= m < 1, so bound < 2^(e-1)
  return ldexpf(1.0f, min(max(30 - e, -126), 126));
}

// Length classes for ordering pairs: exact below 32 samples, then 4 wide.
__device__ __forceinline__ int len_bucket(int n) { return n < 32 ? n : min(kLenBuckets - 1, 32 + ((n - 32) >> 2)); }

// Backward, one workgroup per work item: up to kItemEntries culling-list
// entries (tile, primitive k) of one primitive.  The pairs of those entries
// (at most one per ray of each tile) are spread over the workgroup's threads;
// the payload gradient of k is accumulated in LDS (LDS_ACC, 64-bit fixed point
// with the item's scale) and added to device memory once per item, the pose
// gradient is reduced over the workgroup and added with 15 atomics.
//
// WAVES > 1 asks the compiler for that many waves per SIMD (it then keeps the
// kernel within 512 / WAVES registers, spilling a few); it is used when the
// LDS gradient leaves room for that many workgroups per CU.  THREADS is the
// workgroup size: 512 when the LDS gradient leaves room for only one
// workgroup per CU, so that the CU still runs two waves per SIMD.
template <bool BF16, bool LDS_ACC, bool FADE, int WAVES, int THREADS>
__global__ __launch_bounds__(THREADS) __attribute__((amdgpu_waves_per_eu(WAVES))) void k_bwd_items(
    AccelView av, const float *__restrict__ rot, const float *__restrict__ scale, const void *__restrict__ pay,
    const mvp_ray_aux *__restrict__ aux, const float4 *__restrict__ grad_rgba, const RayConst *__restrict__ rc,
    const RayBound *__restrict__ rbd, BwdOut out, uint32_t sort_cap, int padded,
    unsigned long long *__restrict__ counters) {
  // loads of this thread: pairs visited by the ordering / bound pass, pairs
  // replayed, their cell runs (one voxel-corner set each), and the non-zero
  // gradient values it adds to device memory at the end of an item
  uint32_t n_visit = 0, n_rep = 0, n_run = 0, n_nz = 0;
  // gradient (LDS_ACC), fade window (FADE), pair order and classes
  extern __shared__ unsigned long long s_dyn[];
  using GAcc = typename std::conditional<LDS_ACC, unsigned long long, float>::type;
  __shared__ uint32_t s_live;
  __shared__ uint32_t s_cls[kLenBuckets];
  __shared__ uint32_t s_base[2][kLenBuckets];
  __shared__ uint32_t s_wcnt[2][THREADS / kWave][kLenBuckets];
  __shared__ float s_pose[THREADS / kWave][16];
  __shared__ float s_bnd[THREADS / kWave];
  // the pairs of an item come in sub-lists, four per entry (the rays of each
  // wave of its tile): their starts in ent_rec and their prefix sums
  constexpr int kSub = 4 * kItemEntries;
  __shared__ uint64_t s_start[kSub];
  __shared__ uint32_t s_pre[kSub + 1];
  __shared__ uint32_t s_wsum[kSub / kWave];
  __shared__ uint64_t s_gent[kItemEntries];
  __shared__ int s_tile[kItemEntries];
  __shared__ int s_prim, s_pos;
  const int M = av.M;
  const size_t M3 = (size_t)M * M * M;
  const int nacc = (int)(M3 * 4);                 // gradient values of one primitive
  const LdsMap lm = lds_map(M, padded != 0);
  const int nlds = 4 * lm.plane;                  // their planar LDS copy
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const bool pose = out.pos || out.rot || out.scale;
  GAcc *s_grad = (GAcc *)s_dyn;
  float *s_fade = (float *)((char *)s_dyn + ((LDS_ACC && out.pay) ? (size_t)nlds * sizeof(GAcc) : 0));
  uint16_t *s_sort = (uint16_t *)(s_fade + (FADE ? M : 0));   // [sort_cap] pair order
  uint8_t *s_pcls = (uint8_t *)(s_sort + sort_cap);              // [sort_cap] length class of pair i
  if (FADE) {
    fill_fade(s_fade, M, av.fade_alpha, av.fade_beta);
    __syncthreads();
  }
  const uint64_t n_items = av.item_off[av.N];
  for (uint64_t it = blockIdx.x; it < n_items; it += gridDim.x) {
    if (threadIdx.x == 0) {   // primitive of the item: the p-th in item order, last p with item_off[p] <= it
      int lo = 0, hi = av.N - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (av.item_off[mid] <= it) lo = mid; else hi = mid - 1;
      }
      s_pos = lo;
      s_prim = av.item_prim ? (int)av.item_prim[lo] : lo;
    }
    __syncthreads();
    const int k = s_prim;
    const uint64_t chunk = it - av.item_off[s_pos];
    const uint64_t eb = av.prim_entry_off[k] + chunk * (uint64_t)av.item_entries;
    const int nent = (int)min<uint64_t>((uint64_t)av.item_entries, av.prim_entry_off[k + 1] - eb);
    const int nsub = 4 * nent;
    uint32_t incl = 0;
    if (threadIdx.x < kSub) {   // sub-list u = 4 q + w: entry q, wave w of its tile
      const int u = threadIdx.x, q = u >> 2, w = u & 3;
      uint32_t cnt = 0;
      if (u < nsub) {
        const uint32_t g = av.prim_entries[eb + q];
        s_start[u] = av.ent_base[g] + (uint64_t)w * kWave;
        cnt = av.ent_n[4 * (uint64_t)g + w];
        if (w == 0) {
          s_gent[q] = g;
          s_tile[q] = (int)av.ent_tile[g];
        }
      }
      incl = cnt;
#pragma unroll
      for (int d = 1; d < kWave; d <<= 1) {
        const uint32_t o = __shfl_up(incl, d, kWave);
        if (lane >= d) incl += o;
      }
      if (lane == kWave - 1) s_wsum[wave] = incl;
    }
    if (LDS_ACC && out.pay)
      for (int i = threadIdx.x; i < nlds; i += THREADS) s_grad[i] = (GAcc)0;
    __syncthreads();
    if (threadIdx.x < kSub) {   // prefix sums over the sub-lists
      uint32_t base = 0;
#pragma unroll
      for (int w = 0; w < kSub / kWave; ++w) base += w < wave ? s_wsum[w] : 0u;
      if (threadIdx.x == 0) s_pre[0] = 0;
      s_pre[threadIdx.x + 1] = base + incl;
    }
    __syncthreads();
    const uint32_t total = s_pre[nsub];
    GAcc *gdst = nullptr;
    if constexpr (LDS_ACC) {
      if (out.pay) gdst = s_grad;
    } else {
      if (out.pay) gdst = out.pay + (size_t)k * M3 * 4;
    }
    float P[12];   // the pose sums of this thread's pairs (see bwd_pair)
#pragma unroll
    for (int i = 0; i < 12; ++i) P[i] = 0.f;
    float bound = 0.f;   // largest bound of this thread's pairs, then of the item's
    float fscale = 1.0f;
    if (kSortPairs && total <= sort_cap) {
      // Counting sort of the item's pairs by length class, longest first, in a
      // fixed order (class, then round r = the r-th pair of every thread's
      // contiguous chunk, then wave, then lane), so the replay order, and with
      // it every rounding, is the same from run to run; pairs of one class that
      // are replayed together come from rays a chunk apart.  A histogram pass
      // (which also sums the pairs' bounds) and a scan give the class bases;
      // the scatter ranks each round by ballot within a wave and by per-wave
      // counts across waves (double-buffered, one barrier per round).
      const uint32_t per = (total + THREADS - 1) / THREADS;
      const uint32_t c0 = threadIdx.x * per, c1 = min(total, c0 + per);
      int q0 = 0;
      if (c0 < c1) {
        int hi = nsub - 1;
        while (q0 < hi) {
          const int mid = (q0 + hi + 1) >> 1;
          if (s_pre[mid] <= c0) q0 = mid; else hi = mid - 1;
        }
      }
      if (threadIdx.x < kLenBuckets) s_cls[threadIdx.x] = 0;
      __syncthreads();
      for (uint32_t i = c0, q = q0; i < c1; ++i) {
        while (s_pre[q + 1] <= i) ++q;
        const int n = pair_len(av, aux, rbd, av.ent_rec[s_start[q] + (i - s_pre[q])], s_tile[q >> 2], bound);
        ++n_visit;
        const int b = n > 0 ? len_bucket(n) : 0xff;
        s_pcls[i] = (uint8_t)b;
        if (n > 0) atomicAdd(&s_cls[b], 1u);
      }
#pragma unroll
      for (int d = kWave / 2; d > 0; d >>= 1) bound = nan_max(bound, __shfl_xor(bound, d, kWave));
      if (lane == 0) s_bnd[wave] = bound;
      __syncthreads();
      bound = 0.f;
#pragma unroll
      for (int w = 0; w < THREADS / kWave; ++w) bound = nan_max(bound, s_bnd[w]);
      fscale = fixed_scale(bound);
      if (wave == 0) {   // exclusive scan over the classes from the longest down
        const uint32_t c = s_cls[kLenBuckets - 1 - lane];
        uint32_t incl = c;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
          const uint32_t o = __shfl_up(incl, d, kWave);
          if (lane >= d) incl += o;
        }
        s_base[0][kLenBuckets - 1 - lane] = incl - c;
        if (lane == kWave - 1) s_live = incl;
      }
      const unsigned long long lt = (1ull << lane) - 1ull;
      for (uint32_t r = 0; r < per; ++r) {
        const int cur = r & 1;
        const uint32_t i = c0 + r;
        int b = -1;
        if (i < c1) {
          const int pb_ = s_pcls[i];
          if (pb_ != 0xff) b = pb_;
        }
        s_wcnt[cur][wave][lane] = 0;   // kLenBuckets == kWave
        uint32_t rank = 0;
        unsigned long long todo = __ballot(b >= 0);
        while (todo) {   // one class at a time: its lanes and their order
          const int src = __ffsll((long long)todo) - 1;
          const int bb = __shfl(b, src, kWave);
          const unsigned long long mm = __ballot(b == bb);
          if (b == bb) rank = (uint32_t)__popcll(mm & lt);
          if (lane == src) s_wcnt[cur][wave][bb] = (uint32_t)__popcll(mm);
          todo &= ~mm;
        }
        __syncthreads();
        if (b >= 0) {
          uint32_t pos = s_base[cur][b] + rank;
          for (int w = 0; w < wave; ++w) pos += s_wcnt[cur][w][b];
          s_sort[pos] = (uint16_t)i;
        }
        if (threadIdx.x < kLenBuckets) {
          uint32_t add = 0;
#pragma unroll
          for (int w = 0; w < THREADS / kWave; ++w) add += s_wcnt[cur][w][threadIdx.x];
          s_base[cur ^ 1][threadIdx.x] = s_base[cur][threadIdx.x] + add;
        }
      }
      __syncthreads();
      const uint32_t live = s_live;
      for (uint32_t p = threadIdx.x; p < live; p += THREADS) {
        const uint32_t i = s_sort[p];
        int q = 0, hi = nsub - 1;    // entry of flattened pair i: last q with s_pre[q] <= i
        while (q < hi) {
          const int mid = (q + hi + 1) >> 1;
          if (s_pre[mid] <= i) q = mid; else hi = mid - 1;
        }
        const uint2 rec = av.ent_rec[s_start[q] + (i - s_pre[q])];
        bwd_pair<BF16, LDS_ACC, FADE, WAVES == 1>(av, rot, scale, pay, aux, grad_rgba, rc, rec, s_gent[q >> 2], s_tile[q >> 2], k, gdst,
                                      lm, fscale, s_fade, pose, P, n_run);
        ++n_rep;
      }
    } else {
      // list order (more pairs than the ordering buffer holds).
      // kChunkedPairs: each thread replays a contiguous run of the flattened
      // pairs, so the lanes of a wave follow rays some pixels apart, which flush
      // into different voxel cells at once; otherwise pair i goes to thread
      // i mod 256 (neighbouring pixels on neighbouring lanes).
      const uint32_t per = kChunkedPairs ? (total + THREADS - 1) / THREADS : 1;
      const uint32_t stride = kChunkedPairs ? 1 : THREADS;
      const uint32_t i0 = kChunkedPairs ? threadIdx.x * per : threadIdx.x;
      const uint32_t iend = kChunkedPairs ? min(total, i0 + per) : total;
      int q0 = 0;
      if (i0 < iend) {
        int hi = nsub - 1;    // entry of flattened pair i0: last q with s_pre[q] <= i0
        while (q0 < hi) {
          const int mid = (q0 + hi + 1) >> 1;
          if (s_pre[mid] <= i0) q0 = mid; else hi = mid - 1;
        }
      }
      if (LDS_ACC && out.pay) {   // the item's bound, for the fixed-point scale
        for (uint32_t i = i0, q = q0; i < iend; i += stride) {
          while (s_pre[q + 1] <= i) ++q;
          (void)pair_len(av, aux, rbd, av.ent_rec[s_start[q] + (i - s_pre[q])], s_tile[q >> 2], bound);
          ++n_visit;
        }
#pragma unroll
        for (int d = kWave / 2; d > 0; d >>= 1) bound = nan_max(bound, __shfl_xor(bound, d, kWave));
        if (lane == 0) s_bnd[wave] = bound;
        __syncthreads();
        bound = 0.f;
#pragma unroll
        for (int w = 0; w < THREADS / kWave; ++w) bound = nan_max(bound, s_bnd[w]);
        fscale = fixed_scale(bound);
      }
      for (uint32_t i = i0, q = q0; i < iend; i += stride) {
        while (s_pre[q + 1] <= i) ++q;
        const uint2 rec = av.ent_rec[s_start[q] + (i - s_pre[q])];
        bwd_pair<BF16, LDS_ACC, FADE, WAVES == 1>(av, rot, scale, pay, aux, grad_rgba, rc, rec, s_gent[q >> 2], s_tile[q >> 2], k, gdst,
                                      lm, fscale, s_fade, pose, P, n_run);
        ++n_rep;
      }
    }
    if (pose) {
#pragma unroll
      for (int i = 0; i < 12; ++i) {
        float x = P[i];
#pragma unroll
        for (int d = kWave / 2; d > 0; d >>= 1) x += __shfl_xor(x, d, kWave);
        if (lane == 0) s_pose[wave][i] = x;
      }
    }
    __syncthreads();
    if (pose && threadIdx.x < 12) {   // the item's sums (each thread reads and writes its own column)
      float x = 0.f;
#pragma unroll
      for (int w = 0; w < THREADS / kWave; ++w) x += s_pose[w][threadIdx.x];
      s_pose[0][threadIdx.x] = x;
    }
    __syncthreads();
    if (pose && threadIdx.x < 15 && total > 0) {
      const int i = threadIdx.x;
      const float x = pose_from_sums(av, rot, scale, k, s_pose[0], i);
      if (i < 3) {
        if (out.pos) unsafeAtomicAdd(out.pos + 3 * (size_t)k + i, x);
      } else if (i < 12) {
        if (out.rot) unsafeAtomicAdd(out.rot + 9 * (size_t)k + (i - 3), x);
      } else {
        if (out.scale) unsafeAtomicAdd(out.scale + 3 * (size_t)k + (i - 12), x);
      }
    }
    if (LDS_ACC && out.pay && total > 0) {
      float *dst = out.pay + M3 * 4 * (size_t)k;
      const bool ok = fscale > 0.0f;
      const float inv = ok ? 1.0f / fscale : __builtin_nanf("");   // exact: a power of two
      for (int i = threadIdx.x; i < nacc; i += THREADS) {   // device order: voxel i/4, channel i%4
        const int vx = i >> 2, ix = vx % M, iy = (vx / M) % M, iz = vx / (M * M);
        const long long v = (long long)s_grad[(i & 3) * lm.plane + ix + iy * lm.sy + iz * lm.sz];
        if (v != 0 || !ok) {
          unsafeAtomicAdd(dst + i, (float)v * inv);
          ++n_nz;
        }
      }
    }
    __syncthreads();   // LDS is reused by the next item
  }
  if (counters) {
    const unsigned long long c[4] = {wave_sum_u64(n_visit), wave_sum_u64(n_rep), wave_sum_u64(n_run),
                                     wave_sum_u64(n_nz)};
    if (lane == 0 && (c[0] | c[1] | c[3])) {
#pragma unroll
      for (int i = 0; i < 4; ++i) atomicAdd(&counters[kCntBwdVisit + i], c[i]);
    }
  }
}

template <bool B, bool L, bool F>
static const void *bwd_items_fn(bool w3, bool wide_wg) {
  return w3 ? (const void *)k_bwd_items<B, L, F, 3, kTileThreads>
            : (wide_wg ? (const void *)k_bwd_items<B, L, F, 1, 2 * kTileThreads>
                       : (const void *)k_bwd_items<B, L, F, 1, kTileThreads>);
}

hipError_t launch_march_bwd(const AccelView &av, const mvp_prims &p, int64_t n_items_max,
                            const mvp_ray_aux *aux, const float *grad_rgba, const float *bg,
                            const float *rgba, void *scratch, float *g_pay, float *g_pos, float *g_rot,
                            float *g_scale, float *g_bg, unsigned long long *counters, hipStream_t s,
                            hipEvent_t t0, hipEvent_t t1) {
  const size_t R = (size_t)av.n_slots;
  if (counters) {
    const hipError_t ez = launch_zero_u64((uint64_t *)counters + kCntBwdVisit, 4, s);
    if (ez != hipSuccess) return ez;
  }
  if (R == 0) return hipSuccess;
  RayConst *rc = (RayConst *)scratch;
  RayBound *rbd = (RayBound *)(rc + R);
  uint32_t *pmax = (uint32_t *)(rbd + R);
  const bool bf16 = p.payload_dtype == MVP_BF16;
  const bool fade = av.fade_alpha > 0.f;
  const size_t fade_shm = fade ? (size_t)p.M * sizeof(float) : 0;
  hipError_t e = launch_zero_u32(pmax, 2, s);
  if (e != hipSuccess) return e;
  const size_t n_vox = (size_t)p.n_prim * p.M * p.M * p.M;
  if (n_vox) {
    const unsigned pg = (unsigned)std::min<size_t>((n_vox + 255) / 256, 1024);
    if (bf16)
      hipLaunchKernelGGL((k_payload_bound<true>), dim3(pg), dim3(256), 0, s, p.payload, n_vox, pmax);
    else
      hipLaunchKernelGGL((k_payload_bound<false>), dim3(pg), dim3(256), 0, s, p.payload, n_vox, pmax);
  }
  const unsigned rb = (unsigned)((R + kBwdRaysPerBlock - 1) / kBwdRaysPerBlock);
#define MVP_RAYS(B, F)                                                                                        \
  hipLaunchKernelGGL((k_bwd_rays<B, F>), dim3(rb), dim3(256), fade_shm, s, av, p.payload, aux,               \
                     (const float4 *)grad_rgba, bg, (const float4 *)rgba, rc, rbd, pmax, g_bg, R)
  if (bf16) {
    if (fade) MVP_RAYS(true, true); else MVP_RAYS(true, false);
  } else {
    if (fade) MVP_RAYS(false, true); else MVP_RAYS(false, false);
  }
#undef MVP_RAYS
  e = hipGetLastError();
  if (e != hipSuccess || p.n_prim == 0 || n_items_max == 0) return e;
  // the planar 64-bit LDS gradient, when one workgroup's copy fits a CU; its
  // padded layout unless only the packed one fits
  const size_t kStatic = 8192;   // static LDS of a 256-thread workgroup is under 8 KB (512: under 16 KB)
  auto lds_bytes = [&](bool pad) { return (size_t)lds_map(p.M, pad).plane * 4 * sizeof(unsigned long long); };
  const int padded = lds_bytes(true) + fade_shm + 2 * kStatic <= 160 * 1024 ? 1 : 0;
  const size_t lds = lds_bytes(padded != 0);
  bool in_lds = g_pay && lds + fade_shm + 2 * kStatic <= 160 * 1024;
  auto wgs_per_cu = [&](size_t grad) {
    for (int w = 3; w > 1; --w)
      if ((size_t)w * (grad + fade_shm + kStatic) <= 160 * 1024) return w;
    return 1;
  };
  // 3 waves per SIMD when 3 workgroups' LDS fits a CU; 512-thread workgroups
  // when only one does (16^3 payloads: 131 KB)
  const bool w3 = !in_lds || wgs_per_cu(lds) >= 3;
  bool wide_wg = in_lds && wgs_per_cu(lds) == 1;
  const unsigned grid = (unsigned)std::min<int64_t>(n_items_max, 1 << 20);
  BwdOut out{g_pay, g_pos, g_rot, g_scale};
  size_t shm = (in_lds ? lds : 0) + fade_shm;
  // the pair-ordering buffer takes what is left of the LDS share of a
  // workgroup at the occupancy chosen above (items with more pairs than it
  // holds keep their pairs in list order)
  uint32_t sort_cap = 0;
  if (kSortPairs) {
    const size_t wgs = w3 ? 3 : (shm + kStatic <= 80 * 1024 ? 2 : 1);
    const size_t share = 160 * 1024 / wgs - (wide_wg ? 2 * kStatic : kStatic);
    const size_t room = share > shm ? (share - shm) / (sizeof(uint16_t) + 1) : 0;
    const size_t want = (size_t)av.item_entries * kTileThreads;
    sort_cap = (uint32_t)(std::min(room, want) / kTileThreads * kTileThreads);
    shm += (size_t)sort_cap * (sizeof(uint16_t) + 1);
  }
  if (shm > 64 * 1024) {
    // allow more than the default dynamic LDS per workgroup (gfx950 has 160 KB)
    const void *fn =
        bf16 ? (in_lds ? (fade ? bwd_items_fn<true, true, true>(w3, wide_wg) : bwd_items_fn<true, true, false>(w3, wide_wg))
                       : (fade ? bwd_items_fn<true, false, true>(w3, wide_wg) : bwd_items_fn<true, false, false>(w3, wide_wg)))
             : (in_lds ? (fade ? bwd_items_fn<false, true, true>(w3, wide_wg) : bwd_items_fn<false, true, false>(w3, wide_wg))
                       : (fade ? bwd_items_fn<false, false, true>(w3, wide_wg) : bwd_items_fn<false, false, false>(w3, wide_wg)));
    if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm) != hipSuccess) {
      (void)hipGetLastError();
      in_lds = false;   // gradients straight to device memory, pairs in list order
      wide_wg = false;
      sort_cap = 0;
      shm = fade_shm;
    }
  }
  if (t0) (void)hipEventRecord(t0, s);
#define MVP_BWD(B, L, F)                                                                                        \
  do {                                                                                                          \
    if (w3)                                                                                                     \
      hipLaunchKernelGGL((k_bwd_items<B, L, F, 3, kTileThreads>), dim3(grid), dim3(kTileThreads), shm, s, av,   \
                         p.rot, p.scale, p.payload, aux, (const float4 *)grad_rgba, rc, rbd, out, sort_cap,     \
                         padded, counters);                                                                             \
    else if (wide_wg)                                                                                           \
      hipLaunchKernelGGL((k_bwd_items<B, L, F, 1, 2 * kTileThreads>), dim3(grid), dim3(2 * kTileThreads), shm, \
                         s, av, p.rot, p.scale, p.payload, aux, (const float4 *)grad_rgba, rc, rbd, out,        \
                         sort_cap, padded, counters);                                                                   \
    else                                                                                                        \
      hipLaunchKernelGGL((k_bwd_items<B, L, F, 1, kTileThreads>), dim3(grid), dim3(kTileThreads), shm, s, av,   \
                         p.rot, p.scale, p.payload, aux, (const float4 *)grad_rgba, rc, rbd, out, sort_cap,     \
                         padded, counters);                                                                             \
  } while (0)
#define MVP_BWD_F(B, F)                                  \
  do {                                                   \
    if (in_lds) MVP_BWD(B, true, F);                     \
    else MVP_BWD(B, false, F);                           \
  } while (0)
  if (bf16) {
    if (fade) MVP_BWD_F(true, true); else MVP_BWD_F(true, false);
  } else {
    if (fade) MVP_BWD_F(false, true); else MVP_BWD_F(false, false);
  }
#undef MVP_BWD_F
#undef MVP_BWD
  e = hipGetLastError();
  if (t1) (void)hipEventRecord(t1, s);
  return e;
}

// Entries per backward work item: 8^3 payloads flush small gradients, so
// shorter items (more of them) balance better; larger payloads amortise the
// per-item zeroing and flush of their LDS gradient over 64 entries.
int backward_item_entries(int M) { return M <= 8 ? 32 : kItemEntries; }

}  // namespace mvp
