// Forward-state layout and device helpers shared by the forward and
// backward translation units.
#pragma once

#include "dv_internal.h"

namespace dv {

constexpr float F_INF = __builtin_huge_valf();
constexpr double Z_EPS_D = 1e-3;
constexpr float LOG2E = 1.4426950408889634f;
constexpr uint32_t SRC_NONE = 0x3FFu;

// Arguments of the compositing kernels (forward and backward).
struct CompArgs {
  const ViewConst* views;
  const VOConst* vo;
  int32_t n_views;
  int32_t n_oct;
  const uint32_t* tile_start;
  const uint32_t* tile_end;
  const uint32_t* tile_bgend;
  // work items: every tile's background list in 1 or more chunks
  const uint32_t* order;       // launch order -> item id
  const uint32_t* act_tile;    // (tile, actor) pair -> tile
  const uint32_t* item_tile;   // item id -> tile
  const uint32_t* item_chunk;  // item id -> chunk index in its tile
  const uint32_t* tile_nck;    // chunks per tile
  const uint32_t* tile_pbase;  // first chunk slot of a tile with nck > 1
  const uint32_t* plan_counts; // [0] items, [1] chunk slots
  float* chunk_b;          // per (chunk slot, part, pixel): first chord depth
  float4* chunk_part;      // per (chunk slot, pixel): 4 x float4 partials
  float2* chunk_tps;       // backward: per (chunk slot, pixel): T_pre, S_after
  uint32_t* item_work;     // forward: measured work per item
  // actor work items: every (tile, actor) list in 1 or more chunks; a ray
  // with one segment of the actor is composited per chunk into partials
  const uint32_t* aorder;      // launch order -> actor item id
  const uint32_t* aitem_pair;  // actor item -> (tile, actor) pair
  const uint32_t* aitem_chunk; // actor item -> chunk index
  const uint32_t* pair_nck;    // chunks per pair
  const uint32_t* pair_pbase;  // first chunk slot of a pair with nck > 1
  const uint32_t* aplan_counts;// [0] actor items, [1] chunk slots
  float4* apart;           // per (actor chunk slot, pixel): 4 x float4
  float2* atps;            // backward: per (slot, pixel): W_c, R_c
  const uint32_t* pair_val;
  const float4* rec_geo;   // vmin - camera (octree frame), h
  const float4* rec_g8a;   // corner densities 0..3
  const float4* rec_g8b;   // corner densities 4..7
  const float4* rec_cn;    // colour rgb, 1/h
  const float4* rec_nrm;   // world normal xyz, 0
  const uint64_t* rec_rect;  // covered pixels: xl | xh<<16 | yl<<32 | yh<<48
  const uint32_t* act_beg; // per global tile, n_tiles + 1
  const uint32_t* act_oct; // actor octree index per (tile, slot)
  const uint2* act_sub;    // pair sub-range per (tile, slot)
  float2* seg_se;          // per-pixel box intervals / segments
  uint32_t* seg_meta;
  float4* seg_p0;          // partial C.rgb, D
  float4* seg_p1;          // partial N.xyz, T
  float4* seg_t0;          // tail part of seg_p0 (after the rebase), else 0
  float4* seg_t1;          // tail part of seg_p1.xyz, 0
  float4* seg_bw;          // backward: T_pre, S_after, dL/dstart, dL/dend
  uint32_t* pix_nseg;
  float4* fin0;            // final C.rgb, D
  float4* fin1;            // final N.xyz, T
  float4* fin2;            // tail part of fin0 (after the rebase), else 0
  float4* fin3;            // tail part of fin1.xyz, 0
  const dv_outputs* outs;  // per view
  const dv_out_grads* gin; // per view (backward)
  float4* gr_col;          // backward per-record: dL/dc (rgb), 0
  float4* gr_nrm;          // dL/dn_world, 0
  float4* gr_g8a;          // dL/dg corners 0..3
  float4* gr_g8b;          // corners 4..7
  float* pose_grad;        // [n_views][n_actors][12] or null
  int32_t n_actors;
  int32_t K;
  float eps;
  float tau_near;
  float c;
  float inv_c;
  float bg[3];
  const float* sky;  // sky map [3][sky_h][sky_w] or null (constant bg)
  int sky_w, sky_h;
  float* sky_grad;   // dL/dsky accumulator or null
  uint32_t mask;
  unsigned long long* counters;  // work counters or null
};

// Add per-thread work counts into counters[i], counters[i+1] (one atomic
// per wave).  Called by every thread of the block.
__device__ inline void count_work(unsigned long long* counters, int i,
                                  uint32_t entries, uint32_t pieces) {
  if (!counters) return;
  unsigned long long e = entries, p = pieces;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    e += __shfl_xor(e, o, 64);
    p += __shfl_xor(p, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    atomicAdd(counters + i, e);
    atomicAdd(counters + i + 1, p);
  }
}

// Wave-level counts (wave-uniform values, added once per wave by lane 0):
// list entries a wave walked in the straight-line iteration, and those of
// them where at least one lane had a chord.
__device__ inline void count_waves(unsigned long long* counters, int i,
                                   uint32_t iters, uint32_t hits) {
  if (!counters) return;
  if ((threadIdx.x & 63) == 0) {
    atomicAdd(counters + i, (unsigned long long)iters);
    atomicAdd(counters + i + 1, (unsigned long long)hits);
  }
}

// Pixel of thread tid inside a 16x16 tile: each wave64 covers an 8x8
// quadrant, so a wave can skip list entries whose pixel rectangle misses
// its quadrant.
__device__ inline int tile_px(int tid) {
  return (((tid >> 6) & 1) << 3) | (tid & 7);
}
__device__ inline int tile_py(int tid) {
  return (((tid >> 6) >> 1) << 3) | ((tid >> 3) & 7);
}

// Entries of a staged batch (nb <= 256) whose pixel rectangle meets the
// pixel box of the wave's lanes in `lanes` (a wave ballot, e.g. of the
// lanes still compositing), as four wave-uniform 64-bit masks (bit i of
// m[c] is entry 64 c + i).  Lane l of the wave is pixel (bx + l % 8,
// by + l / 8) of the 8x8 block at (bx, by), so the box comes from scalar
// bit operations on the ballot.  Called by every lane of the wave.  An
// entry whose rectangle misses the box has no chord for any of those lanes
// (the rectangle covers every pixel the leaf's chord can reach), so
// skipping it changes nothing for them.  No lane: no entries.
__device__ inline void wave_live_masks(const uint2* rect, uint32_t nb, int bx,
                                       int by, uint64_t lanes, uint64_t m[4]) {
  if (lanes == 0) {
    m[0] = m[1] = m[2] = m[3] = 0;
    return;
  }
  uint64_t cols = lanes | (lanes >> 32);
  cols |= cols >> 16;
  cols |= cols >> 8;
  cols &= 0xFFull;
  const int x0 = bx + __builtin_ctzll(cols);
  const int x1 = bx + 63 - __builtin_clzll(cols);
  const int y0 = by + (__builtin_ctzll(lanes) >> 3);
  const int y1 = by + ((63 - __builtin_clzll(lanes)) >> 3);
  const uint32_t lane = threadIdx.x & 63;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const uint32_t r = (uint32_t)c * 64 + lane;
    bool hit = false;
    if (r < nb) {
      const uint2 rc = rect[r];
      const int xl = (int)(rc.x & 0xFFFF), xh = (int)(rc.x >> 16);
      const int yl = (int)(rc.y & 0xFFFF), yh = (int)(rc.y >> 16);
      hit = xl <= x1 && xh >= x0 && yl <= y1 && yh >= y0;
    }
    m[c] = __ballot(hit);
  }
}

// Whether the wave's selected entries (masks wm from wave_live_masks over
// the live lanes `lanes`) cover, on average, less than a quarter of the
// live-lane box: then a walk in which every lane takes only the entries
// whose rectangle holds its own pixel (lane_masks) does fewer iterations
// than the walk over the wave's union of entries.  Wave-uniform.
__device__ inline bool sparse_cover(const uint2* rect, uint32_t nb, int bx,
                                    int by, uint64_t lanes, const uint64_t m[4]) {
  if (lanes == 0) return false;
  uint64_t cols = lanes | (lanes >> 32);
  cols |= cols >> 16;
  cols |= cols >> 8;
  cols &= 0xFFull;
  const int x0 = bx + __builtin_ctzll(cols);
  const int x1 = bx + 63 - __builtin_clzll(cols);
  const int y0 = by + (__builtin_ctzll(lanes) >> 3);
  const int y1 = by + ((63 - __builtin_clzll(lanes)) >> 3);
  const uint32_t lane = threadIdx.x & 63;
  uint32_t cov = 0, n = 0;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    n += (uint32_t)__popcll(m[c]);
    if ((m[c] >> lane) & 1ull) {
      const uint2 rc = rect[c * 64 + lane];
      const int xl = max((int)(rc.x & 0xFFFF), x0), xh = min((int)(rc.x >> 16), x1);
      const int yl = max((int)(rc.y & 0xFFFF), y0), yh = min((int)(rc.y >> 16), y1);
      cov += (uint32_t)((xh - xl + 1) * (yh - yl + 1));
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) cov += __shfl_xor(cov, o, 64);
  const uint32_t box = (uint32_t)((x1 - x0 + 1) * (y1 - y0 + 1));
  return 4u * cov < n * box;
}

// Per-lane masks: of the wave's selected entries (wm), those whose
// rectangle holds the lane's own pixel (px, py).  An entry whose rectangle
// misses the pixel has no chord on the pixel's ray (the rectangle covers
// every pixel the leaf's chord can reach), so a lane that skips it walks
// the same pieces in the same order.
__device__ inline void lane_masks(const uint2* rect, const uint64_t wm[4],
                                  int px, int py, uint64_t pm[4]) {
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    uint64_t m = wm[c], out = 0;
    while (m != 0) {
      const int b = __builtin_ctzll(m);
      m &= m - 1;
      const uint2 rc = rect[c * 64 + b];
      const bool in = (int)(rc.x & 0xFFFF) <= px && px <= (int)(rc.x >> 16) &&
                      (int)(rc.y & 0xFFFF) <= py && py <= (int)(rc.y >> 16);
      out |= in ? (1ull << b) : 0ull;
    }
    pm[c] = out;
  }
}

__device__ inline int view_of_tile(const ViewConst* views, int n_views,
                                   uint32_t gt) {
  int lo = 0, hi = n_views - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (views[mid].tile_base <= gt) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ inline float3 mat3_mul(const float* M, float3 v) {
  return make_float3(
      fmaf(M[2], v.z, fmaf(M[1], v.y, M[0] * v.x)),
      fmaf(M[5], v.z, fmaf(M[4], v.y, M[3] * v.x)),
      fmaf(M[8], v.z, fmaf(M[7], v.y, M[6] * v.x)));
}

__device__ inline float fast_exp(float x) {
  return __builtin_amdgcn_exp2f(x * LOG2E);
}

// exp-linear activation (knee c): x above c, else c * exp(x/c - 1).
__device__ inline float explin(float x, float c, float inv_c) {
  return x > c ? x : c * fast_exp(fmaf(x, inv_c, -1.0f));
}
__device__ inline float explin_grad(float x, float c, float inv_c) {
  return x > c ? 1.0f : fast_exp(fmaf(x, inv_c, -1.0f));
}

// Suffix rebase.  The backward needs, per piece, the suffix S = L - P of
// everything composited after it.  Formed as a difference of running sums
// it carries an absolute FP32 error ~2^-24 |L|, which swamps the suffix of
// pieces behind an opaque surface (S ~ T |L|).  Both walks therefore split
// their running sums the first time T drops below T_REBASE (tested where
// the stop test is, on bit-identical T): the forward stores the part after
// the split (the tail) beside the totals, and the backward restarts P at 0
// against the tail total there, so deep pieces see an error ~2^-24 T_REBASE
// |L| instead.  Asset segments do the same on their own transmittance.
// Pinned staging for small per-call host tables (one buffer per host
// thread): acquire waits for the previous upload from it, release records
// an event after the upload just enqueued on s.
uint8_t* stage_acquire(size_t bytes);
dv_status stage_release(hipStream_t s);

// Heaviest-first launch order (render.hip) of n items of weight
// w[i] - (w0 ? w0[i] : 0).
dv_status launch_order_by_weight(dv_ctx* ctx, int64_t n, const uint32_t* w0,
                                 const uint32_t* w, uint32_t* order, hipStream_t s);


// Background entries per chunk: a tile whose list is longer than 1.5
// chunks is split into ceil(len / CHUNK) equal chunks, each composited by
// its own block into per-pixel partial states that are merged in order.
constexpr uint32_t CHUNK = 1024;
__host__ __device__ inline uint32_t chunks_of(uint32_t len, uint32_t chunk = CHUNK) {
  return len > chunk + chunk / 2 ? (len + chunk - 1) / chunk : 1u;
}
// Entries per chunk of an actor's list in a tile (asset walks cost more per
// entry, so their chunks are shorter).
constexpr uint32_t ACHUNK = 384;
// Entry range [cb, ce) of chunk c of nck over [beg, end).
__device__ inline void chunk_range(uint32_t beg, uint32_t end, uint32_t nck,
                                   uint32_t c, uint32_t& cb, uint32_t& ce) {
  const uint32_t len = end - beg;
  const uint32_t cs = (len + nck - 1) / nck;
  cb = min(end, beg + c * cs);
  ce = min(end, cb + cs);
}

constexpr float T_REBASE = 0.0009765625f;  // 2^-10

// alpha = 1 - exp(-tau).  For small tau the difference 1 - e cancels in
// FP32 (relative error ~6e-8 / tau), so a 4-term series is used there; the
// series' truncation error is below 2^-24 relative for tau < 2^-6.
// Both branches are evaluated and selected (no divergent branch).
__device__ inline float opacity(float tau, float e) {
  const float p = fmaf(tau, fmaf(tau, fmaf(tau, -1.0f / 24.0f, 1.0f / 6.0f),
                                 -0.5f), 1.0f);
  const float series = tau * p;
  const float direct = 1.0f - e;
  return tau < 0.015625f ? series : direct;
}

__device__ inline float lerpf(float a, float b, float t) {
  return fmaf(t, b - a, a);
}

__device__ inline float trilerp(float4 ga, float4 gb, float ux, float uy,
                                float uz) {
  float x0 = lerpf(ga.x, ga.y, ux), x1 = lerpf(ga.z, ga.w, ux);
  float x2 = lerpf(gb.x, gb.y, ux), x3 = lerpf(gb.z, gb.w, ux);
  float y0 = lerpf(x0, x1, uy), y1 = lerpf(x2, x3, uy);
  return lerpf(y0, y1, uz);
}

__device__ inline float clamp01(float x) { return fminf(fmaxf(x, 0.0f), 1.0f); }

// Slab test against an axis-aligned box [lo, hi] given relative to the ray
// origin, with precomputed reciprocal direction.
__device__ inline void slab2(float3 lo, float3 hi, float3 inv, float& t0,
                             float& t1) {
  float ax = lo.x * inv.x, bx = hi.x * inv.x;
  float ay = lo.y * inv.y, by = hi.y * inv.y;
  float az = lo.z * inv.z, bz = hi.z * inv.z;
  t0 = fmaxf(fmaxf(fminf(ax, bx), fminf(ay, by)), fminf(az, bz));
  t1 = fminf(fminf(fmaxf(ax, bx), fmaxf(ay, by)), fmaxf(az, bz));
}
// Far corner lo + h of a leaf record (the same FP32 sums wherever formed).
__device__ inline float3 leaf_hi(const float4& geo) {
  return make_float3(geo.x + geo.w, geo.y + geo.w, geo.z + geo.w);
}
// The box [lo, lo + h].
__device__ inline void slab(float3 lo, float h, float3 inv, float& t0,
                            float& t1) {
  slab2(lo, make_float3(lo.x + h, lo.y + h, lo.z + h), inv, t0, t1);
}
// Slab test of batch entry r (far corner from the batch when NORMALS is
// false, formed here otherwise: identical values).
template <bool NORMALS, class BatchT>
__device__ inline void batch_slab(const BatchT& B, uint32_t r, const float4& geo,
                                  float3 inv, float& t0, float& t1) {
  const float3 lo = make_float3(geo.x, geo.y, geo.z);
  if (NORMALS) {
    slab2(lo, leaf_hi(geo), inv, t0, t1);
  } else {
    const float4 hi = B.nrm[r];
    slab2(lo, make_float3(hi.x, hi.y, hi.z), inv, t0, t1);
  }
}

// Same, also reporting the axes that define entry and exit.
__device__ inline void slab_axes(float3 lo, float3 hi, float3 inv, float& t0,
                                 float& t1, int& a0, int& a1) {
  float ax = lo.x * inv.x, bx = hi.x * inv.x;
  float ay = lo.y * inv.y, by = hi.y * inv.y;
  float az = lo.z * inv.z, bz = hi.z * inv.z;
  float nx = fminf(ax, bx), ny = fminf(ay, by), nz = fminf(az, bz);
  float fx = fmaxf(ax, bx), fy = fmaxf(ay, by), fz = fmaxf(az, bz);
  t0 = nx; a0 = 0;
  if (ny > t0) { t0 = ny; a0 = 1; }
  if (nz > t0) { t0 = nz; a0 = 2; }
  t1 = fx; a1 = 0;
  if (fy < t1) { t1 = fy; a1 = 1; }
  if (fz < t1) { t1 = fz; a1 = 2; }
}

__device__ inline float3 safe_inv(float3 d) {
  return make_float3(1.0f / d.x, 1.0f / d.y, 1.0f / d.z);
}

// Derivatives of the optical depth of one piece.  With one sample per
// piece (KC = 1) the corner derivatives are kept factored as coef times the
// trilinear weights of (ux, uy, uz); add_corner_grads expands them.
struct PieceDer {
  float dtda, dtdb;       // d tau / d(a), d(b)
  float dg[8];            // d tau / d corner value (KC != 1)
  float coef, ux, uy, uz; // KC == 1: d tau / d g and the sample's cell coords
  float3 dx;              // sum_q d tau / d x_q
  float3 dxt;             // sum_q tau_q d tau / d x_q
};

// Optical depth of the piece [a, b] of one leaf: K-point midpoint rule of
// explin(trilinear raw density).  MODE 0: optical depth only; 1: also
// corner derivatives; 2: also geometry derivatives (samples, ends).  The
// optical depth takes the same operations in every mode, so forward and
// backward walks see bit-identical values.
// KC > 0 fixes K = KC at compile time (same arithmetic as a run-time K).
template <int MODE, int KC = 0>
__device__ inline float piece_eval(float4 geo, float4 ga, float4 gb,
                                   float inv_h, float3 d, float a, float b,
                                   int K_, float invK_, float c, float inv_c,
                                   PieceDer* o) {
  const int K = KC > 0 ? KC : K_;
  const float invK = KC > 0 ? 1.0f / (float)KC : invK_;
  const float step = (b - a) * invK;
  float sum = 0.0f, pa = 0.0f, pb = 0.0f;
  if (MODE >= 1) {
    if (KC != 1) {
#pragma unroll
      for (int m = 0; m < 8; ++m) o->dg[m] = 0.0f;
    }
    o->dx = make_float3(0, 0, 0);
    o->dxt = make_float3(0, 0, 0);
  }
  for (int q = 0; q < K; ++q) {
    const float tq = fmaf((float)q + 0.5f, step, a);
    const float ux = clamp01(fmaf(tq, d.x, -geo.x) * inv_h);
    const float uy = clamp01(fmaf(tq, d.y, -geo.y) * inv_h);
    const float uz = clamp01(fmaf(tq, d.z, -geo.z) * inv_h);
    const float g = trilerp(ga, gb, ux, uy, uz);
    // (the activation is positive, so the first sum equals the sample)
    if (q == 0) sum = explin(g, c, inv_c);
    else sum += explin(g, c, inv_c);
    if (MODE >= 1) {
      const float coef = step * explin_grad(g, c, inv_c);
      const float vx = 1.0f - ux, vy = 1.0f - uy, vz = 1.0f - uz;
      if (KC == 1) {
        o->coef = coef; o->ux = ux; o->uy = uy; o->uz = uz;
      } else {
      o->dg[0] = fmaf(coef, vx * vy * vz, o->dg[0]);
      o->dg[1] = fmaf(coef, ux * vy * vz, o->dg[1]);
      o->dg[2] = fmaf(coef, vx * uy * vz, o->dg[2]);
      o->dg[3] = fmaf(coef, ux * uy * vz, o->dg[3]);
      o->dg[4] = fmaf(coef, vx * vy * uz, o->dg[4]);
      o->dg[5] = fmaf(coef, ux * vy * uz, o->dg[5]);
      o->dg[6] = fmaf(coef, vx * uy * uz, o->dg[6]);
      o->dg[7] = fmaf(coef, ux * uy * uz, o->dg[7]);
      }
      if (MODE >= 2) {
        const float f = ((float)q + 0.5f) * invK;
        const float gx = vy * vz * (ga.y - ga.x) + uy * vz * (ga.w - ga.z) +
                         vy * uz * (gb.y - gb.x) + uy * uz * (gb.w - gb.z);
        const float gy = vx * vz * (ga.z - ga.x) + ux * vz * (ga.w - ga.y) +
                         vx * uz * (gb.z - gb.x) + ux * uz * (gb.w - gb.y);
        const float gz = vx * vy * (gb.x - ga.x) + ux * vy * (gb.y - ga.y) +
                         vx * uy * (gb.z - ga.z) + ux * uy * (gb.w - ga.w);
        const float s = coef * inv_h;
        const float3 dtdx = make_float3(s * gx, s * gy, s * gz);
        const float proj = dtdx.x * d.x + dtdx.y * d.y + dtdx.z * d.z;
        pa = fmaf(proj, 1.0f - f, pa);
        pb = fmaf(proj, f, pb);
        o->dx.x += dtdx.x; o->dx.y += dtdx.y; o->dx.z += dtdx.z;
        o->dxt.x = fmaf(tq, dtdx.x, o->dxt.x);
        o->dxt.y = fmaf(tq, dtdx.y, o->dxt.y);
        o->dxt.z = fmaf(tq, dtdx.z, o->dxt.z);
      }
    }
  }
  if (MODE >= 1) {
    o->dtda = -sum * invK + pa;
    o->dtdb = sum * invK + pb;
  }
  return sum * step;
}

// dg[m] += dtau * d tau / d corner m.
template <int KC>
__device__ inline void add_corner_grads(const PieceDer& pd, float dtau,
                                        float* dg) {
  if (KC == 1) {
    const float s = dtau * pd.coef;
    const float vx = 1.0f - pd.ux, vy = 1.0f - pd.uy, vz = 1.0f - pd.uz;
    const float s0 = s * vz, s1 = s * pd.uz;
    const float w00 = vx * vy, w10 = pd.ux * vy, w01 = vx * pd.uy,
                w11 = pd.ux * pd.uy;
    dg[0] = fmaf(s0, w00, dg[0]); dg[1] = fmaf(s0, w10, dg[1]);
    dg[2] = fmaf(s0, w01, dg[2]); dg[3] = fmaf(s0, w11, dg[3]);
    dg[4] = fmaf(s1, w00, dg[4]); dg[5] = fmaf(s1, w10, dg[5]);
    dg[6] = fmaf(s1, w01, dg[6]); dg[7] = fmaf(s1, w11, dg[7]);
  } else {
#pragma unroll
    for (int m = 0; m < 8; ++m) dg[m] = fmaf(dtau, pd.dg[m], dg[m]);
  }
}

// dg[m] = dtau * d tau / d corner m.
template <int KC>
__device__ inline void set_corner_grads(const PieceDer& pd, float dtau,
                                        float* dg) {
  if (KC == 1) {
    const float s = dtau * pd.coef;
    const float vx = 1.0f - pd.ux, vy = 1.0f - pd.uy, vz = 1.0f - pd.uz;
    const float s0 = s * vz, s1 = s * pd.uz;
    const float w00 = vx * vy, w10 = pd.ux * vy, w01 = vx * pd.uy,
                w11 = pd.ux * pd.uy;
    dg[0] = s0 * w00; dg[1] = s0 * w10; dg[2] = s0 * w01; dg[3] = s0 * w11;
    dg[4] = s1 * w00; dg[5] = s1 * w10; dg[6] = s1 * w01; dg[7] = s1 * w11;
  } else {
#pragma unroll
    for (int m = 0; m < 8; ++m) dg[m] = dtau * pd.dg[m];
  }
}

template <int KC = 0>
__device__ inline float piece_tau(float4 geo, float4 ga, float4 gb,
                                  float inv_h, float3 d, float a, float b,
                                  int K, float invK, float c, float inv_c) {
  return piece_eval<0, KC>(geo, ga, gb, inv_h, d, a, b, K, invK, c, inv_c,
                           nullptr);
}

// Pixel of thread tid in tile gt and its unit ray direction.
// Sky environment map (Sec. 3.1, Eq. 2): the unit world direction d (z up)
// maps to longitude atan2(d_y, d_x) and colatitude acos(d_z), texel (i, j)
// is centred at u = i, v = j, and the map is sampled bilinearly with
// columns wrapping in longitude and rows clamped at the poles.
struct SkyTaps {
  int o[4];    // texel offsets j * W + i in one [H][W] plane
  float w[4];  // bilinear weights
};
template <class A>
__device__ inline SkyTaps sky_taps(const A& a, float3 d) {
  const float kPi = 3.14159265358979f;
  const int W = a.sky_w, H = a.sky_h;
  const float lon = atan2f(d.y, d.x);
  // colatitude as atan2(|d_xy|, d_z), which equals acos(d_z) for a unit d
  // but stays well conditioned at the poles (acos of an FP32 d_z near 1
  // turns its rounding into ~3e-4 rad of angle)
  const float colat = atan2f(sqrtf(d.x * d.x + d.y * d.y), d.z);
  const float u = (lon + kPi) * (0.5f / kPi) * (float)W - 0.5f;
  const float v = colat * (1.0f / kPi) * (float)H - 0.5f;
  const float u0 = floorf(u), v0 = floorf(v);
  const float fu = u - u0, fv = v - v0;
  int i0 = (int)u0 % W;
  if (i0 < 0) i0 += W;
  const int i1 = i0 + 1 == W ? 0 : i0 + 1;
  const int j0 = min(max((int)v0, 0), H - 1);
  const int j1 = min(max((int)v0 + 1, 0), H - 1);
  SkyTaps t;
  t.o[0] = j0 * W + i0; t.w[0] = (1.0f - fu) * (1.0f - fv);
  t.o[1] = j0 * W + i1; t.w[1] = fu * (1.0f - fv);
  t.o[2] = j1 * W + i0; t.w[2] = (1.0f - fu) * fv;
  t.o[3] = j1 * W + i1; t.w[3] = fu * fv;
  return t;
}
// C_sky of the ray: the map's sample, or the constant colour without one.
template <class A>
__device__ inline float3 sky_colour(const A& a, float3 d) {
  if (!a.sky) return make_float3(a.bg[0], a.bg[1], a.bg[2]);
  const SkyTaps t = sky_taps(a, d);
  const size_t hw = (size_t)a.sky_w * a.sky_h;
  float3 c = make_float3(0, 0, 0);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    c.x = fmaf(t.w[k], a.sky[t.o[k]], c.x);
    c.y = fmaf(t.w[k], a.sky[hw + t.o[k]], c.y);
    c.z = fmaf(t.w[k], a.sky[2 * hw + t.o[k]], c.z);
  }
  return c;
}

struct PixSetup {
  int v;
  int px, py, bx, by;
  bool valid;
  float3 d;
  size_t pix;
};
template <class A>
__device__ inline PixSetup pixel_setup(const A& a, uint32_t gt, int tid) {
  PixSetup P;
  P.v = view_of_tile(a.views, a.n_views, gt);
  const ViewConst& V = a.views[P.v];
  const uint32_t lt = gt - V.tile_base;
  P.px = (int)(lt % V.ntx) * TILE + tile_px(tid);
  P.py = (int)(lt / V.ntx) * TILE + tile_py(tid);
  P.bx = (int)(lt % V.ntx) * TILE + (((tid >> 6) & 1) << 3);
  P.by = (int)(lt / V.ntx) * TILE + (((tid >> 6) >> 1) << 3);
  P.valid = P.px < V.w && P.py < V.h;
  const float dx = ((float)(V.x0 + P.px) + 0.5f - V.fcx) * V.inv_fx;
  const float dy = ((float)(V.y0 + P.py) + 0.5f - V.fcy) * V.inv_fy;
  float3 d = mat3_mul(V.Rc, make_float3(dx, dy, 1.0f));
  const float inv = 1.0f / sqrtf(d.x * d.x + d.y * d.y + d.z * d.z);
  P.d = make_float3(d.x * inv, d.y * inv, d.z * inv);
  P.pix = (size_t)gt * TPB + tid;
  return P;
}

// Depth boundaries of a chunked tile's background walk.  Chunk c > 0
// starts at B'_c = min over c' >= c of B_c' (B_c: entry depth of the
// pixel's first non-empty chord in chunk c, +inf if none).  Ownership
// segments starting before B'_c belong to earlier chunks (spliced by the
// chunk before, at its end), the others to chunk c or later.  Chords along
// one ray are disjoint and in depth order, so this splits the sequential
// walk exactly.  Only a pixel with segments uses them (and only its
// B_c are searched).
// B_c is searched by CB_SPLIT blocks over consecutive parts of the chunk;
// the first part (in list order) with a chord gives it.
constexpr int CB_SPLIT = 4;
// The chunked tile whose first chunk slot is sl (from the slot table of
// the plan), else 0xFFFFFFFF: kernels over chunked tiles walk the slots
// instead of launching a block per tile.
template <class A>
__device__ inline uint32_t chunked_tile_at(const A& a, const uint32_t* slot_tile,
                                           uint32_t sl) {
  const uint32_t gt = slot_tile[sl];
  return (gt != 0xFFFFFFFFu && a.tile_pbase[gt] == sl) ? gt : 0xFFFFFFFFu;
}
template <class A>
__device__ inline float chunk_first(const A& a, size_t slot, int tid) {
  const float* p = a.chunk_b + slot * CB_SPLIT * TPB + tid;
  float b = p[0];
  for (int q = 1; q < CB_SPLIT; ++q)
    if (b == F_INF) b = p[(size_t)q * TPB];
  return b;
}
template <class A>
__device__ inline void chunk_bounds(const A& a, uint32_t gt, uint32_t nck,
                                    uint32_t c, int tid, float& Bc, float& Bn) {
  Bc = -F_INF;
  Bn = F_INF;
  if (nck <= 1) return;
  const size_t pb = a.tile_pbase[gt];
  float m = F_INF;
  for (uint32_t k = nck - 1; k > c; --k) m = fminf(m, chunk_first(a, pb + k, tid));
  Bn = m;
  if (c > 0) Bc = fminf(m, chunk_first(a, pb + c, tid));
}

// Real spherical harmonics up to degree 3 (Sec. 3.1 view-dependent
// colour), orthonormal, with Y_{1,-1}, Y_{1,0}, Y_{1,1} proportional to
// y, z, x.  Coefficients are SoA [S][3][N].
__device__ inline void sh_basis(int deg, float x, float y, float z,
                                float* Y) {
  Y[0] = 0.28209479177387814f;
  if (deg < 1) return;
  Y[1] = 0.4886025119029199f * y;
  Y[2] = 0.4886025119029199f * z;
  Y[3] = 0.4886025119029199f * x;
  if (deg < 2) return;
  const float xx = x * x, yy = y * y, zz = z * z;
  Y[4] = 1.0925484305920792f * (x * y);
  Y[5] = 1.0925484305920792f * (y * z);
  Y[6] = 0.31539156525252005f * (3.0f * zz - 1.0f);
  Y[7] = 1.0925484305920792f * (x * z);
  Y[8] = 0.5462742152960396f * (xx - yy);
  if (deg < 3) return;
  Y[9] = 0.5900435899266435f * y * (3.0f * xx - yy);
  Y[10] = 2.890611442640554f * (x * y * z);
  Y[11] = 0.4570457994644658f * y * (5.0f * zz - 1.0f);
  Y[12] = 0.3731763325901154f * z * (5.0f * zz - 3.0f);
  Y[13] = 0.4570457994644658f * x * (5.0f * zz - 1.0f);
  Y[14] = 1.445305721320277f * z * (xx - yy);
  Y[15] = 0.5900435899266435f * x * (xx - 3.0f * yy);
}

// d Y_q / d(x, y, z) of the polynomials above (unit-sphere restriction is
// applied by the caller).
__device__ inline void sh_basis_grad(int deg, float x, float y, float z,
                                     float* gx, float* gy, float* gz) {
  gx[0] = gy[0] = gz[0] = 0.0f;
  if (deg < 1) return;
  const float c1 = 0.4886025119029199f;
  gx[1] = 0.0f; gy[1] = c1;  gz[1] = 0.0f;
  gx[2] = 0.0f; gy[2] = 0.0f; gz[2] = c1;
  gx[3] = c1;  gy[3] = 0.0f; gz[3] = 0.0f;
  if (deg < 2) return;
  const float a = 1.0925484305920792f, b = 0.31539156525252005f,
              c = 0.5462742152960396f;
  gx[4] = a * y; gy[4] = a * x; gz[4] = 0.0f;
  gx[5] = 0.0f;  gy[5] = a * z; gz[5] = a * y;
  gx[6] = 0.0f;  gy[6] = 0.0f;  gz[6] = 6.0f * b * z;
  gx[7] = a * z; gy[7] = 0.0f;  gz[7] = a * x;
  gx[8] = 2.0f * c * x; gy[8] = -2.0f * c * y; gz[8] = 0.0f;
  if (deg < 3) return;
  const float e = 0.5900435899266435f, f = 2.890611442640554f,
              g = 0.4570457994644658f, h = 0.3731763325901154f,
              i = 1.445305721320277f;
  const float xx = x * x, yy = y * y, zz = z * z;
  gx[9] = 6.0f * e * x * y; gy[9] = e * (3.0f * xx - 3.0f * yy); gz[9] = 0.0f;
  gx[10] = f * y * z; gy[10] = f * x * z; gz[10] = f * x * y;
  gx[11] = 0.0f; gy[11] = g * (5.0f * zz - 1.0f); gz[11] = 10.0f * g * y * z;
  gx[12] = 0.0f; gy[12] = 0.0f; gz[12] = h * (15.0f * zz - 3.0f);
  gx[13] = g * (5.0f * zz - 1.0f); gy[13] = 0.0f; gz[13] = 10.0f * g * x * z;
  gx[14] = 2.0f * i * x * z; gy[14] = -2.0f * i * y * z; gz[14] = i * (xx - yy);
  gx[15] = e * (3.0f * xx - 3.0f * yy); gy[15] = -6.0f * e * x * y; gz[15] = 0.0f;
}

// Gradient accumulators of one octree (device pointers).
struct OctGrad {
  float* corner;
  float* sh;
  float* feat;       // feature renders: dL/df of the group's first channel
  int32_t feat_nc;   // channels of the group (0: colour render)
  int32_t pad;
};

// ------------------------------------------------------------------ serving
// Device side of the serving loop (render.hip): renders whose background
// walks were left out (groups) are published into a ring; one persistent
// kernel drains their work items, merges chunked tiles, counts finished
// tiles per view and raises a request's completion flag in host memory
// when its last tile is written.
constexpr int SV_RING = 1024;    // ring entries (groups published), and the
                                 // argument blocks, one per entry
constexpr int SV_GROUPS = 16;    // group slots (forward states in flight)
constexpr int SV_FLAGS = 1024;   // request completion flags

// The drain kernel reads an entry through scalar loads (scalar cache),
// which are not kept coherent with the uploads of later groups: each entry
// fills whole 256-byte blocks of its own, so reading one group's arguments
// never brings a line of the next entry (uploaded later, perhaps while the
// kernel runs) into the cache ahead of its upload.
struct alignas(256) ServeGroup {
  CompArgs a;                    // walk arguments of the group's forward
  uint32_t* tile_ck;             // [n_tiles] chunks finished per tile
  uint32_t* view_done;           // [n_views] tiles finished per view
  const uint32_t* view_ntiles;   // [n_views]
  const uint32_t* view_flag;     // [n_views] completion flag of the request
  const unsigned long long* view_seq;  // [n_views] value the flag receives
  unsigned long long* flags;     // host-mapped [SV_FLAGS]
};

static_assert(sizeof(ServeGroup) % 256 == 0, "ring entries share cache lines");

struct ServeQueue {
  unsigned long long tail;            // groups published so far
  unsigned long long head;            // first group not known to be drained
  unsigned long long claim[SV_RING];  // (group number << 32) | items taken
  uint32_t n_items[SV_RING];
};

// Publish group number g (item count plan_counts[0]) on stream s, after the
// group's forward work and the upload of its ServeGroup into entry
// g % SV_RING of the argument ring.
dv_status launch_serve_publish(ServeQueue* q, uint64_t g,
                               const uint32_t* plan_counts, hipStream_t s);
// The persistent drain kernel: `blocks` blocks; each exits after idle_limit
// consecutive empty polls (about 3.5 us each), or when the oldest group
// with items left is numbered g_hi or above (the host keeps g_hi at most
// SV_RING / 2 above the oldest unfinished group).
dv_status launch_serve_drain(ServeQueue* q, const ServeGroup* groups,
                             bool normals, bool k1, int blocks, int idle_limit,
                             uint64_t g_hi, hipStream_t s);

// Per-pixel segment scratch: slot s of tile gt, pixel tid.
__device__ inline size_t seg_index(uint32_t slot, int tid) {
  return (size_t)slot * TPB + tid;
}

}  // namespace dv

struct dv_fwd_state {
  dv_ctx* ctx = nullptr;
  const dv_scene* scene = nullptr;
  hipStream_t stream = nullptr;
  int32_t n_views = 0, n_oct = 0, n_actors = 0;
  dv_render_opts opts{};
  std::vector<dv::ViewConst> views_h;
  std::vector<dv::VOConst> vo_h;
  std::vector<dv_view> views_in;
  int64_t n_vis = 0, n_pairs = 0, n_apairs = 0, n_tiles = 0;
  int key_bits = 0, tile_bits = 0, rank_bits = 0;
  std::vector<uint32_t> act_beg_h, act_oct_h, act_tile_h;
  std::vector<int64_t> seg_start_h;
  std::vector<int64_t> seg_pstart_h;   // starts padded to multiples of 64
  std::vector<int32_t> seg_len_h;
  std::vector<uint64_t> view_slot_h;   // first record slot per view, total last
  // host copies uploaded asynchronously by backward calls; kept until the
  // state is retired (after its stream has passed them)
  std::vector<std::vector<dv_out_grads>> grads_keep;
  std::vector<std::vector<dv::OctGrad>> og_keep;
  dv::DBuf views_d, vo_d, outs_d;
  dv::DBuf rec_geo, rec_g8a, rec_g8b, rec_cn, rec_nrm, rec_vox, rec_seg,
      rec_rect;
  dv::DBuf pair_val;
  dv::DBuf tile_start, tile_end, tile_bgend;
  dv::DBuf act_beg, act_oct, act_sub;
  dv::DBuf seg_se, seg_meta, seg_p0, seg_p1, seg_bw, pix_nseg;
  dv::DBuf fin0, fin1, fin2, fin3, seg_t0, seg_t1;
  dv::DBuf order_fwd, order_bwd, item_tile, item_chunk, item_work;
  dv::DBuf tile_nck, tile_ibase, tile_pbase, plan_counts, slot_tile;
  dv::DBuf host_tables;   // one upload: views, constants, segments, actor CSR
  // preprocess ballots and block offsets: record slot of any (view,
  // octree, leaf) item, kept for the leaf-major SH backward
  dv::DBuf pre_wmask, pre_boff, pre_wseg;
  dv::DBuf seg_pstart_d, seg_len_d;   // views into host_tables
  std::vector<std::vector<int64_t>> lstart_keep;
  dv::DBuf chunk_b, chunk_part, act_tile;
  dv::DBuf aorder, aitem_pair, aitem_chunk, pair_nck, pair_ibase, pair_pbase,
      aplan_counts, apart;
  int64_t max_aitems = 0, max_aslots = 0;
  int64_t max_items = 0, max_slots = 0;
  // walk arguments of a forward enqueued without its background walks
  dv::CompArgs ca_fwd{};
};
