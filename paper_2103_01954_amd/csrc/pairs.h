// The per-ray pair lists of one screen tile: the canonical FP32 geometry
// (slab test, sample intervals) and the per-tile pairs pass, shared by the
// build's pairs kernel and by the forward march, which can build a tile's
// pairs itself just before marching them.
//
// Built with -ffp-contract=off and IEEE division/square root: every written
// float operation below is exactly one binary32 operation, so the hit
// decisions and sample intervals are reproducible bit for bit.
#pragma once

#include <climits>

#include "internal.h"

namespace mvp {

// ---------------------------------------------------------------------------
// canonical FP32 geometry (one rounding per written operation)
// ---------------------------------------------------------------------------

// Slab test of the local ray y(t) = a + t b against [-1,1]^3, clipped to t >= t_near.
// An axis with b_i = 0 excludes the ray if a_i lies outside [-1, 1] and
// otherwise does not constrain t.  Written without branches (the quotients of
// a zero b_i are computed and discarded), so the three axes' correctly rounded
// divisions are independent and can overlap.
__device__ inline bool slab_test(const float a[3], const float b[3], float t_near, float *t_in,
                                 float *t_out) {
  float lo = t_near, hi = INFINITY;
  bool miss = false;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const float n0 = -1.0f - a[i];
    const float n1 = 1.0f - a[i];
    const float q0 = n0 / b[i];
    const float q1 = n1 / b[i];
    const bool par = b[i] == 0.0f;
    lo = par ? lo : fmaxf(lo, fminf(q0, q1));
    hi = par ? hi : fminf(hi, fmaxf(q0, q1));
    miss = miss || (par && !(a[i] >= -1.0f && a[i] <= 1.0f));
  }
  *t_in = lo;
  *t_out = hi;
  return !miss && lo <= hi;
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

// Conservative test of a pixel block against a staged entry: can the ray
// through any pixel centre of the block hit the entry's box?  The unnormalised
// directions e(u, v) = P (u, v, 1) of the block's pixel centres span the
// parallelogram of its four corner directions, so their local directions
// A e lie, componentwise, within the bounds [bl, bh] of the four corners' A e.
// A ray that hits at some t >= 0 meets, with that t, a + t bl <= 1 and
// a + t bh >= -1 on every axis (positive scaling of the direction changes no
// hit), so an empty intersection of those t-intervals excludes the whole
// block.  The bounds are widened by far more than the rounding of the per-ray
// canonical test and of this one (the box by 1e-5 (1 + max |a|), the direction
// bounds by 1e-5 |A_i|_1 max |e|), and anything non-finite never excludes.
__device__ inline bool block_may_hit(const Staged &sm, int e, const float (*E)[3], float emax) {
  float a[3], bl[3], bh[3], amax = 0.f;
  bool sane = true;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    a[i] = sm.a[i][e];
    const float A0 = sm.A[3 * i][e], A1 = sm.A[3 * i + 1][e], A2 = sm.A[3 * i + 2][e];
    float lo = INFINITY, hi = -INFINITY;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const float b = A0 * E[c][0] + A1 * E[c][1] + A2 * E[c][2];
      lo = fminf(lo, b);
      hi = fmaxf(hi, b);
    }
    const float eta = 1e-5f * (fabsf(A0) + fabsf(A1) + fabsf(A2)) * emax;
    bl[i] = lo - eta;
    bh[i] = hi + eta;
    amax = fmaxf(amax, fabsf(a[i]));
    sane = sane && fabsf(bl[i]) < 1e30f && fabsf(bh[i]) < 1e30f;
  }
  if (!(sane && amax < 1e30f)) return true;
  const float lim = 1.0f + 1e-5f * (1.0f + amax);
  float lo = 0.0f, hi = INFINITY;
  bool ok = true;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const float nu = lim - a[i];    // a + t bl <= lim
    if (bl[i] > 0.0f) hi = fminf(hi, nu * __builtin_amdgcn_rcpf(bl[i]));
    else if (bl[i] < 0.0f) lo = fmaxf(lo, nu * __builtin_amdgcn_rcpf(bl[i]));
    else ok = ok && !(nu < 0.0f);
    const float nl = -lim - a[i];   // a + t bh >= -lim
    if (bh[i] < 0.0f) hi = fminf(hi, nl * __builtin_amdgcn_rcpf(bh[i]));
    else if (bh[i] > 0.0f) lo = fmaxf(lo, nl * __builtin_amdgcn_rcpf(bh[i]));
    else ok = ok && !(nl > 0.0f);
  }
  return ok && !(lo > hi);
}

// The pairs of one screen tile, computed by a workgroup of kTileThreads
// threads, one per ray (every thread must call it: it has barriers).  The tile's
// culling list (ordered near to far) is staged through LDS in chunks of
// kStage entries; every ray runs the canonical slab test against each staged
// entry, and each pair with at least one sample is inserted into the ray's
// slots in (jlo, primitive id) order.  The list order leaves few pairs out of
// place, and those only by a few places, so the ray keeps its last kTail
// pairs sorted in registers and writes a pair to device memory once kTail
// later ones have arrived; a pair that belongs before all of those moves the
// written ones up by one.  The same pair is listed under its entry in ray
// order: the rays of each wave that hit the entry are ranked by a ballot into
// the wave's 64 slots of the entry's list (unless ent_n is null: a structure
// for the forward only).  The staging threads also write
// the entries' frames and test each entry against the pixel block of each
// wave (block_may_hit): a wave skips the entries that none of its rays can
// hit, about half of a list's entries for a wave of 16 x 4 pixels.
constexpr int kTail = 4;

__device__ __forceinline__ bool pair_before(const int4 &a, const int4 &b) {
  return a.x < b.x || (a.x == b.x && a.w < b.w);
}

__device__ inline void tile_pairs(const AccelView &av, int tile, const PairsOut &o) {
  __shared__ Staged sm;
  __shared__ float s_corner[kTileThreads / kWave][4][3];   // corner directions of each wave's pixel block
  __shared__ float s_enrm[16];
  __shared__ uint8_t s_wmask[kStage];                       // bit w: wave w may hit the entry
  const int t = threadIdx.x;
  int v, px, py;
  size_t ray;
  const bool valid = tile_ray(av, tile, t, &ray, &v, &px, &py);
  const int lane = t & (kWave - 1);
  const int wave = __builtin_amdgcn_readfirstlane(t / kWave);
  const DevCam &cam = av.cams[v];
  if (t < 16) {   // wave w's rays: rows 4w..4w+3 of the tile (a ray subset: the whole tile)
    const int T = av.tiles_x * av.tiles_y, tt = tile % T;
    const int w = t / 4, c = t % 4;
    const float u = (float)((tt % av.tiles_x) * kTile + ((c & 1) ? kTile - 1 : 0)) + 0.5f;
    constexpr int kRows = kWave / kTile;   // pixel rows per wave
    const int r0 = av.tile_rays ? 0 : w * kRows;
    const int r1 = av.tile_rays ? kTile - 1 : r0 + kRows - 1;
    const float vv = (float)((tt / av.tiles_x) * kTile + ((c & 2) ? r1 : r0)) + 0.5f;
    float nrm = 0.f;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const float x = cam.P[3 * i] * u + cam.P[3 * i + 1] * vv + cam.P[3 * i + 2];
      s_corner[w][c][i] = x;
      nrm = fmaxf(nrm, fabsf(x));
    }
    s_enrm[t] = nrm * 1.7320508f;   // bounds |e| of the corner direction
  }
  __syncthreads();
  float emax = 0.f;   // the largest over the workgroup's corner directions
#pragma unroll
  for (int q = 0; q < 16; ++q) emax = fmaxf(emax, s_enrm[q]);
  float d[3];
  pixel_ray(cam, px, py, d);
  const uint64_t lb = av.tile_off[tile], le = av.tile_off[tile + 1];
  const uint64_t len = le - lb;
  const uint64_t rays = av.tile_rays ? av.tile_ray_off[tile + 1] - av.tile_ray_off[tile] : (uint64_t)kTileThreads;
  // read once: a load inside the entry loop would wait for all of the wave's
  // earlier stores (the wait counter counts stores too)
  const uint64_t pbase = av.pair_base[tile];
  const bool lists = o.ent_n != nullptr;   // the per-entry lists (for the backward) are wanted
  const uint64_t seg = pbase + (uint64_t)t;   // pair q at seg + q * rays
  const unsigned long long lt = (1ull << lane) - 1ull;
  int nw = 0;         // pairs written to device memory, in order
  int nt = 0;         // pairs in the sorted register tail, all after the written ones
  int4 tb[kTail];
#pragma unroll
  for (int q = 0; q < kTail; ++q) tb[q] = make_int4(0, 0, 0, 0);
  int4 wl = make_int4(INT_MIN, 0, 0, INT_MIN);   // the last written pair (its key)
  for (uint64_t c0 = lb; c0 < le; c0 += kStage) {
    const int nc = (int)min<uint64_t>(kStage, le - c0);
    __syncthreads();
    stage_chunk(sm, av, cam, c0, nc);
    if (t < nc) {   // the entry's frame and where its pair list goes
      const uint64_t g = c0 + t;
#pragma unroll
      for (int r = 0; r < 3; ++r) o.ef[3 * g + r] = make_float4(sm.A[3 * r][t], sm.A[3 * r + 1][t], sm.A[3 * r + 2][t], sm.a[r][t]);
      if (lists) {
        o.ent_base[g] = pbase + (g - lb) * rays;
        o.ent_tile[g] = (uint32_t)tile;
      }
      uint32_t wm = 0;
#pragma unroll
      for (int w = 0; w < kTileThreads / kWave; ++w)
        if (block_may_hit(sm, t, s_corner[w], emax)) wm |= 1u << w;
      s_wmask[t] = (uint8_t)wm;
    }
    __syncthreads();
    for (int e = 0; e < nc; ++e) {
      const uint64_t g = c0 + e;
      if (!((__builtin_amdgcn_readfirstlane(s_wmask[e]) >> wave) & 1u)) {   // no ray of this wave can hit it
        if (lists && lane == 0) o.ent_n[4 * g + wave] = 0u;
        continue;
      }
      float a[3], b[3];
      int jlo = 0, jhi = 0;
      const bool hit = valid && pair_of(sm, e, d, av.t_near, av.step, 0, a, b, &jlo, &jhi);
      const unsigned long long m = __ballot(hit);
      if (hit) {
        const int4 rec = make_int4(jlo, jhi, (int)(g - lb), sm.id[e]);
        if (nw > 0 && pair_before(rec, wl)) {
          // before every written pair still after it: those move up by one
          int at = nw;
          while (at > 0) {
            const int4 p = o.pr[seg + (uint64_t)(at - 1) * rays];
            if (!pair_before(rec, p)) break;
            o.pr[seg + (uint64_t)at * rays] = p;
            --at;
          }
          o.pr[seg + (uint64_t)at * rays] = rec;
          ++nw;
        } else if (nt == kTail && pair_before(rec, tb[0])) {   // after the written pairs, before the tail
          o.pr[seg + (uint64_t)nw * rays] = rec;
          wl = rec;
          ++nw;
        } else {
          if (nt == kTail) {   // the tail is full: its first pair is final among the written ones
            o.pr[seg + (uint64_t)nw * rays] = tb[0];
            wl = tb[0];
            ++nw;
#pragma unroll
            for (int q = 0; q < kTail - 1; ++q) tb[q] = tb[q + 1];
            --nt;
          }
#pragma unroll
          for (int q = 0; q < kTail; ++q)
            if (q == nt) tb[q] = rec;
#pragma unroll
          for (int q = kTail - 1; q > 0; --q)   // sink the new pair to its place
            if (q <= nt && pair_before(tb[q], tb[q - 1])) {
              const int4 x = tb[q];
              tb[q] = tb[q - 1];
              tb[q - 1] = x;
            }
          ++nt;
        }
        if (lists)
          o.ent_rec[pbase + (g - lb) * rays + (uint64_t)wave * kWave + (uint32_t)__popcll(m & lt)] =
              make_uint2((uint32_t)jlo | ((uint32_t)t << 24), (uint32_t)jhi);
      }
      if (lists && lane == 0) o.ent_n[4 * g + wave] = (uint32_t)__popcll(m);
    }
  }
#pragma unroll
  for (int q = 0; q < kTail; ++q)
    if (q < nt) o.pr[seg + (uint64_t)(nw + q) * rays] = tb[q];
  const int i = nw + nt;
  if (valid) {
    o.ray_seg[ray] = seg;
    o.ray_nj[ray] = make_int2(i, i ? (nw ? o.pr[seg].x : tb[0].x) : INT_MAX);
  }
  const unsigned long long c = wave_sum_u64((unsigned long long)i);
  if (lane == 0 && c) atomicAdd(o.n_pairs, c);
}


}  // namespace mvp
