// Forward and backward ray march through the per-ray primitive lists.
//
// Forward (Sec. 3.2.2): for each sample t_j = j*dt inside at least one
// primitive of the ray's list, every containing primitive is sampled
// trilinearly (Sec. 3.2.1) and the samples are combined by the sum rule
//   sigma_j = sum_k sigma_kj,   C_j = sum_k sigma_kj c_kj
// (the global colour/opacity field), then accumulated with the clamp
//   T + sigma_j dt <= 1 :  T += sigma_j dt,  I += C_j dt
//   otherwise           :  I += C_j (1 - T) / sigma_j,  T = 1   (stop)
// and the march stops once T > 1 - eps_early.
//
// Backward: the additive rule makes every sample's contribution independent
// of the others except through the clamp, so the backward replays each ray
// from its stored final state (last sample j_end and, if clamped, T before the
// clamp) without any per-sample storage:
//   Tdot = dL/dA (unclamped)  or  -g . C_S / sigma_S (clamped at sample S)
//   dL/dsigma_kj = dt (Tdot + g . c_kj),   dL/dc_kj = dt sigma_kj g      (j < S)
//   dL/dsigma_kS = (1 - T_{S-1}) g . (c_kS - C_S/sigma_S) / sigma_S
//   dL/dc_kS     = (1 - T_{S-1}) (sigma_kS / sigma_S) g
// Channel adjoints go to the 8 payload corners with the trilinear weights
// (atomics, accumulated in registers while consecutive samples stay in one
// voxel cell) and to the pose through y = A (o + t d - pos).
//
// Built with -ffp-contract=off; fused multiply-adds are written explicitly.
#include <hip/hip_runtime.h>
#include <stdlib.h>

#include "internal.h"

namespace mvp {

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

__device__ __forceinline__ float lerpf(float a, float b, float f) { return fmaf(f, b - a, a); }

__device__ __forceinline__ float4 lerp4(float4 a, float4 b, float f) {
  return make_float4(lerpf(a.x, b.x, f), lerpf(a.y, b.y, f), lerpf(a.z, b.z, f), lerpf(a.w, b.w, f));
}

// Position of sample tau in a primitive's voxel grid (align-corners): index of
// the lower corner of the cell and the fractional offsets.
struct Cell {
  int idx;      // (iz*M + iy)*M + ix of corner (0,0,0)
  float f[3];
};

__device__ __forceinline__ Cell locate(const float4 &A, const float4 &B, float tau, int M, float hM) {
  const float y[3] = {fmaf(tau, B.x, A.x), fmaf(tau, B.y, A.y), fmaf(tau, B.z, A.z)};
  int i0[3];
  Cell c;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const float yc = fminf(fmaxf(y[i], -1.0f), 1.0f);
    const float u = fmaf(yc, hM, hM);
    int q = (int)floorf(u);
    q = min(max(q, 0), M - 2);
    i0[i] = q;
    c.f[i] = u - (float)q;
  }
  c.idx = (i0[2] * M + i0[1]) * M + i0[0];
  return c;
}

// Trilinear RGBA at a cell (lerp along x, then y, then z).
template <bool BF16>
__device__ __forceinline__ float4 trilinear(const void *pay, size_t base, int M, const Cell &c) {
  const size_t MM = (size_t)M * M;
  const float4 v000 = Voxels<BF16>::load(pay, base);
  const float4 v100 = Voxels<BF16>::load(pay, base + 1);
  const float4 v010 = Voxels<BF16>::load(pay, base + M);
  const float4 v110 = Voxels<BF16>::load(pay, base + M + 1);
  const float4 v001 = Voxels<BF16>::load(pay, base + MM);
  const float4 v101 = Voxels<BF16>::load(pay, base + MM + 1);
  const float4 v011 = Voxels<BF16>::load(pay, base + MM + M);
  const float4 v111 = Voxels<BF16>::load(pay, base + MM + M + 1);
  const float4 c00 = lerp4(v000, v100, c.f[0]);
  const float4 c10 = lerp4(v010, v110, c.f[0]);
  const float4 c01 = lerp4(v001, v101, c.f[0]);
  const float4 c11 = lerp4(v011, v111, c.f[0]);
  const float4 c0 = lerp4(c00, c10, c.f[1]);
  const float4 c1 = lerp4(c01, c11, c.f[1]);
  return lerp4(c0, c1, c.f[2]);
}

__device__ __forceinline__ int jlo_of(const float4 &A) { return __float_as_int(A.w); }
__device__ __forceinline__ int jhi_of(const float4 &B) { return __float_as_int(B.w); }

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

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
  return v;
}

// ---------------------------------------------------------------------------
// forward
// ---------------------------------------------------------------------------

// Trilinear RGBA from the 8 cached corners of a cell (corner q = dx + 2 dy + 4 dz).
__device__ __forceinline__ float4 trilerp(const float4 (&v)[8], const Cell &c) {
  const float4 c00 = lerp4(v[0], v[1], c.f[0]);
  const float4 c10 = lerp4(v[2], v[3], c.f[0]);
  const float4 c01 = lerp4(v[4], v[5], c.f[0]);
  const float4 c11 = lerp4(v[6], v[7], c.f[0]);
  const float4 c0 = lerp4(c00, c10, c.f[1]);
  const float4 c1 = lerp4(c01, c11, c.f[1]);
  return lerp4(c0, c1, c.f[2]);
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

// Accumulated state of one ray.
struct RayState {
  float T = 0.f, I0 = 0.f, I1 = 0.f, I2 = 0.f, t_prev = -1.0f;
  int j_end = -1;
  unsigned long long n_ray = 0, n_prim = 0;
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

// Sample by sample: at each sample, every open pair of the ray is evaluated.
template <bool BF16>
__device__ void march_ray_samples(const AccelView &av, const void *pay, uint64_t beg, uint64_t end, RayState &st) {
  const float dt = av.step, lim = 1.0f - av.eps;
  const int M = av.M;
  const float hM = 0.5f * (float)(M - 1);
  const size_t M3 = (size_t)M * M * M;
  uint64_t base = beg, nxt = beg;
  int j = jlo_of(av.pa[beg]);
  while (true) {
    // open every pair whose interval has started; drop finished ones in front
    while (nxt < end && jlo_of(av.pa[nxt]) <= j) ++nxt;
    while (base < nxt && jhi_of(av.pb[base]) < j) ++base;
    if (base == nxt) {
      if (nxt == end) break;
      j = jlo_of(av.pa[nxt]);   // skip empty space to the next pair
      continue;
    }
    const float tau = (float)j * dt;
    float sig = 0.f, c0 = 0.f, c1 = 0.f, c2 = 0.f;
    for (uint64_t e = base; e < nxt; ++e) {
      const float4 B = av.pb[e];
      if (jhi_of(B) < j) continue;
      const float4 A = av.pa[e];
      const Cell c = locate(A, B, tau, M, hM);
      const float4 s = trilinear<BF16>(pay, (size_t)av.pid[e] * M3 + c.idx, M, c);
      sig += s.w;
      c0 = fmaf(s.w, s.x, c0);
      c1 = fmaf(s.w, s.y, c1);
      c2 = fmaf(s.w, s.z, c2);
      ++st.n_prim;
    }
    ++st.n_ray;
    if (composite(st, j, sig, c0, c1, c2, dt, lim)) break;
    ++j;
  }
}

// Window by window: the samples J..J+kWin-1 of a ray are gathered pair by pair
// into per-sample sums held in registers (the voxel corners of a pair stay in
// registers while consecutive samples remain in one cell), then composited in
// sample order.  Same sums in the same order as sample by sample.
constexpr int kWin = 8;

template <bool BF16>
__device__ void march_ray_windows(const AccelView &av, const void *pay, uint64_t beg, uint64_t end, RayState &st) {
  const float dt = av.step, lim = 1.0f - av.eps;
  const int M = av.M;
  const float hM = 0.5f * (float)(M - 1);
  const size_t M3 = (size_t)M * M * M;
  uint64_t e0 = beg;
  int J = jlo_of(av.pa[beg]);
  while (true) {
    float as[kWin], ar[kWin], ag[kWin], ab[kWin];
    int cnt[kWin];
#pragma unroll
    for (int w = 0; w < kWin; ++w) {
      as[w] = ar[w] = ag[w] = ab[w] = 0.f;
      cnt[w] = 0;
    }
    for (uint64_t e = e0; e < end; ++e) {
      const float4 A = av.pa[e];
      const int jl = jlo_of(A);
      if (jl >= J + kWin) break;
      const float4 B = av.pb[e];
      const int jh = jhi_of(B);
      if (jh < J) continue;
      const int lo = max(jl, J) - J, hi = min(jh, J + kWin - 1) - J;
      const size_t kb = (size_t)av.pid[e] * M3;
      int cur = -1;
      float4 v[8];
#pragma unroll
      for (int w = 0; w < kWin; ++w) {
        if (w >= lo && w <= hi) {
          const float tau = (float)(J + w) * dt;
          const Cell c = locate(A, B, tau, M, hM);
          if (c.idx != cur) {
            load_corners<BF16>(pay, kb + c.idx, M, v);
            cur = c.idx;
          }
          const float4 s = trilerp(v, c);
          as[w] += s.w;
          ar[w] = fmaf(s.w, s.x, ar[w]);
          ag[w] = fmaf(s.w, s.y, ag[w]);
          ab[w] = fmaf(s.w, s.z, ab[w]);
          ++cnt[w];
        }
      }
    }
    bool stop = false;
#pragma unroll
    for (int w = 0; w < kWin; ++w) {
      if (!stop && cnt[w] > 0) {
        ++st.n_ray;
        st.n_prim += cnt[w];
        stop = composite(st, J + w, as[w], ar[w], ag[w], ab[w], dt, lim);
      }
    }
    if (stop) break;
    J += kWin;
    // the next occupied sample: pairs in front of e0 have all ended before J,
    // and every later pair starts no earlier than e0
    while (e0 < end && jhi_of(av.pb[e0]) < J) ++e0;
    if (e0 == end) break;
    J = max(J, jlo_of(av.pa[e0]));
  }
}

template <bool BF16, bool WINDOWS>
__global__ __launch_bounds__(kTileThreads) void k_march_fwd(AccelView av, const void *__restrict__ pay,
                                                             float4 *__restrict__ rgba,
                                                             mvp_ray_aux *__restrict__ aux,
                                                             unsigned long long *__restrict__ counters) {
  __shared__ int s_list[kTileThreads];
  __shared__ int s_wave[kTileThreads / kWave];
  const int T = av.tiles_x * av.tiles_y;
  const int tile = blockIdx.x;
  const int v = tile / T, tt = tile % T;
  const int tx0 = (tt % av.tiles_x) * kTile, ty0 = (tt / av.tiles_x) * kTile;

  {
    const int px = tx0 + (threadIdx.x % kTile), py = ty0 + (threadIdx.x / kTile);
    const bool valid = px < av.W && py < av.H;
    const size_t ray = ((size_t)v * av.H + py) * av.W + px;
    bool act = false;
    if (valid) {
      act = av.ray_off[ray + 1] > av.ray_off[ray];
      if (!act) {
        rgba[ray] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (aux) aux[ray] = mvp_ray_aux{-1, -1.0f};
      }
    }
    compact_tile(act, s_list, s_wave);
  }
  int total = 0;
#pragma unroll
  for (int w = 0; w < kTileThreads / kWave; ++w) total += s_wave[w];

  RayState st;
  if ((int)threadIdx.x < total) {
    const int lp = s_list[threadIdx.x];
    const int px = tx0 + (lp % kTile), py = ty0 + (lp / kTile);
    const size_t ray = ((size_t)v * av.H + py) * av.W + px;
    const uint64_t beg = av.ray_off[ray], end = av.ray_off[ray + 1];
    if (WINDOWS)
      march_ray_windows<BF16>(av, pay, beg, end, st);
    else
      march_ray_samples<BF16>(av, pay, beg, end, st);
    rgba[ray] = make_float4(st.I0, st.I1, st.I2, st.T);
    if (aux) aux[ray] = mvp_ray_aux{st.j_end, st.t_prev};
  }
  if (counters) {
    const unsigned long long nr = wave_sum_u64(st.n_ray);
    const unsigned long long np = wave_sum_u64(st.n_prim);
    if ((threadIdx.x & (kWave - 1)) == 0 && nr) {
      atomicAdd(&counters[0], nr);
      atomicAdd(&counters[1], np);
    }
  }
}

static bool fwd_windows() {
  static const bool w = [] {
    const char *e = getenv("MVP_FWD_IMPL");
    return !(e && e[0] == 's');
  }();
  return w;
}

hipError_t launch_march_fwd(const AccelView &av, const mvp_prims &p, float *rgba, mvp_ray_aux *aux,
                            unsigned long long *counters, hipStream_t s) {
  const int ntile = av.V * av.tiles_x * av.tiles_y;
  if (ntile == 0) return hipSuccess;
  const bool win = fwd_windows();
  if (p.payload_dtype == MVP_BF16) {
    if (win)
      hipLaunchKernelGGL((k_march_fwd<true, true>), dim3(ntile), dim3(kTileThreads), 0, s, av, p.payload,
                         (float4 *)rgba, aux, counters);
    else
      hipLaunchKernelGGL((k_march_fwd<true, false>), dim3(ntile), dim3(kTileThreads), 0, s, av, p.payload,
                         (float4 *)rgba, aux, counters);
  } else {
    if (win)
      hipLaunchKernelGGL((k_march_fwd<false, true>), dim3(ntile), dim3(kTileThreads), 0, s, av, p.payload,
                         (float4 *)rgba, aux, counters);
    else
      hipLaunchKernelGGL((k_march_fwd<false, false>), dim3(ntile), dim3(kTileThreads), 0, s, av, p.payload,
                         (float4 *)rgba, aux, counters);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// backward
// ---------------------------------------------------------------------------

struct BwdOut {
  float *pay, *pos, *rot, *scale;
};

__device__ __forceinline__ void flush_cell(float *g_pay, size_t base, int M, const float (&acc)[8][4]) {
  const size_t MM = (size_t)M * M;
  const size_t off[8] = {0, 1, (size_t)M, (size_t)M + 1, MM, MM + 1, MM + M, MM + M + 1};
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    float *dst = g_pay + (base + off[c]) * 4;
#pragma unroll
    for (int ch = 0; ch < 4; ++ch) unsafeAtomicAdd(dst + ch, acc[c][ch]);
  }
}

template <bool BF16>
__global__ __launch_bounds__(kTileThreads) void k_march_bwd(AccelView av, const float *__restrict__ pos,
                                                             const float *__restrict__ rot,
                                                             const float *__restrict__ scale,
                                                             const void *__restrict__ pay,
                                                             const mvp_ray_aux *__restrict__ aux,
                                                             const float4 *__restrict__ grad_rgba,
                                                             BwdOut out) {
  __shared__ int s_list[kTileThreads];
  __shared__ int s_wave[kTileThreads / kWave];
  const int T = av.tiles_x * av.tiles_y;
  const int tile = blockIdx.x;
  const int v = tile / T, tt = tile % T;
  const int tx0 = (tt % av.tiles_x) * kTile, ty0 = (tt / av.tiles_x) * kTile;
  {
    const int px = tx0 + (threadIdx.x % kTile), py = ty0 + (threadIdx.x / kTile);
    bool act = false;
    if (px < av.W && py < av.H) {
      const size_t ray = ((size_t)v * av.H + py) * av.W + px;
      const float4 g = grad_rgba[ray];
      act = aux[ray].j_end >= 0 && (g.x != 0.f || g.y != 0.f || g.z != 0.f || g.w != 0.f);
    }
    compact_tile(act, s_list, s_wave);
  }
  int total = 0;
#pragma unroll
  for (int w = 0; w < kTileThreads / kWave; ++w) total += s_wave[w];
  if ((int)threadIdx.x >= total) return;

  const int lp = s_list[threadIdx.x];
  const int px = tx0 + (lp % kTile), py = ty0 + (lp / kTile);
  const size_t ray = ((size_t)v * av.H + py) * av.W + px;
  const uint64_t beg = av.ray_off[ray], end = av.ray_off[ray + 1];
  const float4 g = grad_rgba[ray];
  const mvp_ray_aux ax = aux[ray];
  const int j_end = ax.j_end;
  const bool clamped = ax.t_prev >= 0.f;
  const float dt = av.step;
  const int M = av.M;
  const float hM = 0.5f * (float)(M - 1);
  const size_t M3 = (size_t)M * M * M;

  // per-ray constants of the adjoint
  float tdot = g.w, w_s = 0.f, sig_s = 1.f, cb0 = 0.f, cb1 = 0.f, cb2 = 0.f;
  if (clamped) {
    const float tau = (float)j_end * dt;
    float sig = 0.f, c0 = 0.f, c1 = 0.f, c2 = 0.f;
    for (uint64_t e = beg; e < end; ++e) {
      const float4 A = av.pa[e];
      if (jlo_of(A) > j_end) break;
      const float4 B = av.pb[e];
      if (jhi_of(B) < j_end) continue;
      const Cell c = locate(A, B, tau, M, hM);
      const float4 s = trilinear<BF16>(pay, (size_t)av.pid[e] * M3 + c.idx, M, c);
      sig += s.w;
      c0 = fmaf(s.w, s.x, c0);
      c1 = fmaf(s.w, s.y, c1);
      c2 = fmaf(s.w, s.z, c2);
    }
    sig_s = sig;
    cb0 = c0 / sig;
    cb1 = c1 / sig;
    cb2 = c2 / sig;
    tdot = -(g.x * cb0 + g.y * cb1 + g.z * cb2);
    w_s = 1.0f - ax.t_prev;
  }

  // ray direction for the pose chain (unit, through the pixel centre)
  const DevCam &cam = av.cams[v];
  float d[3];
  {
    const float u = (float)px + 0.5f, w = (float)py + 0.5f;
    float e[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) e[i] = cam.P[3 * i] * u + cam.P[3 * i + 1] * w + cam.P[3 * i + 2];
    const float inv = 1.0f / sqrtf(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
#pragma unroll
    for (int i = 0; i < 3; ++i) d[i] = e[i] * inv;
  }

  const size_t MM = (size_t)M * M;
  for (uint64_t e = beg; e < end; ++e) {
    const float4 A = av.pa[e];
    const int jl = jlo_of(A);
    if (jl > j_end) break;
    const float4 B = av.pb[e];
    const int jh = min(jhi_of(B), j_end);
    if (jh < jl) continue;
    const int k = av.pid[e];
    const size_t kb = (size_t)k * M3;
    float G0 = 0.f, G1 = 0.f, G2 = 0.f, H0 = 0.f, H1 = 0.f, H2 = 0.f;
    int cur = -1;
    float4 cv[8];
    float acc[8][4];
    for (int j = jl; j <= jh; ++j) {
      const float tau = (float)j * dt;
      const Cell c = locate(A, B, tau, M, hM);
      if (c.idx != cur) {
        if (cur >= 0 && out.pay) flush_cell(out.pay, kb + cur, M, acc);
        const size_t b0 = kb + c.idx;
        cv[0] = Voxels<BF16>::load(pay, b0);
        cv[1] = Voxels<BF16>::load(pay, b0 + 1);
        cv[2] = Voxels<BF16>::load(pay, b0 + M);
        cv[3] = Voxels<BF16>::load(pay, b0 + M + 1);
        cv[4] = Voxels<BF16>::load(pay, b0 + MM);
        cv[5] = Voxels<BF16>::load(pay, b0 + MM + 1);
        cv[6] = Voxels<BF16>::load(pay, b0 + MM + M);
        cv[7] = Voxels<BF16>::load(pay, b0 + MM + M + 1);
#pragma unroll
        for (int q = 0; q < 8; ++q) acc[q][0] = acc[q][1] = acc[q][2] = acc[q][3] = 0.f;
        cur = c.idx;
      }
      const float fx = c.f[0], fy = c.f[1], fz = c.f[2];
      const float wx[2] = {1.0f - fx, fx}, wy[2] = {1.0f - fy, fy}, wz[2] = {1.0f - fz, fz};
      float w[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) w[q] = wx[q & 1] * wy[(q >> 1) & 1] * wz[q >> 2];
      float r = 0.f, gg = 0.f, b = 0.f, s = 0.f;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        r = fmaf(w[q], cv[q].x, r);
        gg = fmaf(w[q], cv[q].y, gg);
        b = fmaf(w[q], cv[q].z, b);
        s = fmaf(w[q], cv[q].w, s);
      }
      float a0, a1, a2, a3;   // dL/d(r, g, b, sigma) of this prim-sample
      if (clamped && j == j_end) {
        const float gd = g.x * (r - cb0) + g.y * (gg - cb1) + g.z * (b - cb2);
        a3 = w_s * gd / sig_s;
        const float ws = w_s * s / sig_s;
        a0 = ws * g.x;
        a1 = ws * g.y;
        a2 = ws * g.z;
      } else {
        a3 = dt * (tdot + g.x * r + g.y * gg + g.z * b);
        const float ws = dt * s;
        a0 = ws * g.x;
        a1 = ws * g.y;
        a2 = ws * g.z;
      }
      float sc[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        acc[q][0] = fmaf(w[q], a0, acc[q][0]);
        acc[q][1] = fmaf(w[q], a1, acc[q][1]);
        acc[q][2] = fmaf(w[q], a2, acc[q][2]);
        acc[q][3] = fmaf(w[q], a3, acc[q][3]);
        sc[q] = a0 * cv[q].x + a1 * cv[q].y + a2 * cv[q].z + a3 * cv[q].w;
      }
      // gradient of the trilinear interpolant of sc with respect to y
      const float gx = hM * (wy[0] * wz[0] * (sc[1] - sc[0]) + wy[1] * wz[0] * (sc[3] - sc[2]) +
                             wy[0] * wz[1] * (sc[5] - sc[4]) + wy[1] * wz[1] * (sc[7] - sc[6]));
      const float gyv = hM * (wx[0] * wz[0] * (sc[2] - sc[0]) + wx[1] * wz[0] * (sc[3] - sc[1]) +
                              wx[0] * wz[1] * (sc[6] - sc[4]) + wx[1] * wz[1] * (sc[7] - sc[5]));
      const float gz = hM * (wx[0] * wy[0] * (sc[4] - sc[0]) + wx[1] * wy[0] * (sc[5] - sc[1]) +
                             wx[0] * wy[1] * (sc[6] - sc[2]) + wx[1] * wy[1] * (sc[7] - sc[3]));
      G0 += gx;
      G1 += gyv;
      G2 += gz;
      H0 = fmaf(tau, gx, H0);
      H1 = fmaf(tau, gyv, H1);
      H2 = fmaf(tau, gz, H2);
    }
    if (cur >= 0 && out.pay) flush_cell(out.pay, kb + cur, M, acc);

    // pose: y = A (o + tau d - t), A = diag(1/s) R^T
    if (out.pos || out.rot || out.scale) {
      const float G[3] = {G0, G1, G2}, H[3] = {H0, H1, H2};
      float Am[9], t[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const float4 row = av.xf[3 * (size_t)k + i];
        Am[3 * i] = row.x; Am[3 * i + 1] = row.y; Am[3 * i + 2] = row.z; t[i] = row.w;
      }
      const float p[3] = {cam.o[0] - t[0], cam.o[1] - t[1], cam.o[2] - t[2]};
      if (out.pos) {
#pragma unroll
        for (int m = 0; m < 3; ++m)
          unsafeAtomicAdd(out.pos + 3 * (size_t)k + m, -(Am[m] * G[0] + Am[3 + m] * G[1] + Am[6 + m] * G[2]));
      }
      if (out.rot || out.scale) {
        float Rm[9], s[3];
#pragma unroll
        for (int i = 0; i < 9; ++i) Rm[i] = rot[9 * (size_t)k + i];
#pragma unroll
        for (int i = 0; i < 3; ++i) s[i] = scale[3 * (size_t)k + i];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          float rp = 0.f;
#pragma unroll
          for (int m = 0; m < 3; ++m) {
            const float P = fmaf(p[m], G[i], d[m] * H[i]);
            if (out.rot) unsafeAtomicAdd(out.rot + 9 * (size_t)k + 3 * m + i, P / s[i]);
            rp = fmaf(Rm[3 * m + i], P, rp);
          }
          if (out.scale) unsafeAtomicAdd(out.scale + 3 * (size_t)k + i, -rp / (s[i] * s[i]));
        }
      }
    }
  }
  (void)pos;
}

hipError_t launch_march_bwd(const AccelView &av, const mvp_prims &p, const mvp_ray_aux *aux,
                            const float *grad_rgba, float *g_pay, float *g_pos, float *g_rot,
                            float *g_scale, hipStream_t s) {
  const int ntile = av.V * av.tiles_x * av.tiles_y;
  if (ntile == 0 || p.n_prim == 0) return hipSuccess;
  BwdOut out{g_pay, g_pos, g_rot, g_scale};
  if (p.payload_dtype == MVP_BF16)
    hipLaunchKernelGGL(k_march_bwd<true>, dim3(ntile), dim3(kTileThreads), 0, s, av, p.pos, p.rot, p.scale,
                       p.payload, aux, (const float4 *)grad_rgba, out);
  else
    hipLaunchKernelGGL(k_march_bwd<false>, dim3(ntile), dim3(kTileThreads), 0, s, av, p.pos, p.rot, p.scale,
                       p.payload, aux, (const float4 *)grad_rgba, out);
  return hipGetLastError();
}

}  // namespace mvp
