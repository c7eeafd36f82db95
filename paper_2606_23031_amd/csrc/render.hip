// Forward render: per-view leaf preprocessing, record sort, tile binning,
// pair sort, tile directories and the compositing walk (Sec. 3.4, App. A,
// Alg. 1, Eq. 2).
#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstring>

#include "render.h"

namespace dv {

// ------------------------------------------------------------------ binning
// Tile rectangle of a box (contract: FP64, fixed operation order, no
// contraction).  status 0 culled, 1 rectangle, 2 whole window.
struct Rect { int status, xl, xh, yl, yh; };

__host__ __device__ inline Rect bin_box(const double A[9], const double b[3],
                                        const double lo[3], const double hi[3],
                                        double fx, double fy, double cx,
                                        double cy, int x0, int y0, int w,
                                        int h, double rnear2) {
  double X[8], Y[8], Z[8];
  bool allneg = true, anynear = false;
  double bl[3], bh[3];
  for (int m = 0; m < 8; ++m) {
    const double x = (m & 1) ? hi[0] : lo[0];
    const double y = (m & 2) ? hi[1] : lo[1];
    const double z = (m & 4) ? hi[2] : lo[2];
    X[m] = ((A[0] * x + A[1] * y) + A[2] * z) + b[0];
    Y[m] = ((A[3] * x + A[4] * y) + A[5] * z) + b[1];
    Z[m] = ((A[6] * x + A[7] * y) + A[8] * z) + b[2];
    allneg = allneg && (Z[m] <= 0.0);
    anynear = anynear || (Z[m] < Z_EPS_D);
    if (m == 0) {
      bl[0] = bh[0] = X[0]; bl[1] = bh[1] = Y[0]; bl[2] = bh[2] = Z[0];
    } else {
      bl[0] = fmin(bl[0], X[m]); bh[0] = fmax(bh[0], X[m]);
      bl[1] = fmin(bl[1], Y[m]); bh[1] = fmax(bh[1], Y[m]);
      bl[2] = fmin(bl[2], Z[m]); bh[2] = fmax(bh[2], Z[m]);
    }
  }
  Rect r;
  if (allneg) { r.status = 0; r.xl = 1; r.xh = 0; r.yl = 1; r.yh = 0; return r; }
  if (anynear) {
    double dd[3];
    for (int a = 0; a < 3; ++a) dd[a] = fmax(fmax(bl[a], 0.0), -bh[a]);
    const double dist2 = (dd[0] * dd[0] + dd[1] * dd[1]) + dd[2] * dd[2];
    if (dist2 < rnear2) {
      r.status = 2; r.xl = 0; r.xh = w - 1; r.yl = 0; r.yh = h - 1;
      return r;
    }
  }
  // projected points: corners in front of the plane Z = e, plus the
  // crossings of the edges that straddle it
  double umin = __builtin_huge_val(), umax = -__builtin_huge_val();
  double vmin = __builtin_huge_val(), vmax = -__builtin_huge_val();
  for (int m = 0; m < 8; ++m) {
    if (Z[m] >= Z_EPS_D) {
      const double u = cx + fx * (X[m] / Z[m]);
      const double v = cy + fy * (Y[m] / Z[m]);
      umin = fmin(umin, u); umax = fmax(umax, u);
      vmin = fmin(vmin, v); vmax = fmax(vmax, v);
    }
  }
  if (anynear) {
    for (int bit = 1; bit < 8; bit <<= 1) {
      for (int m = 0; m < 8; ++m) {
        if (m & bit) continue;
        const int m2 = m | bit;
        if ((Z[m] < Z_EPS_D) == (Z[m2] < Z_EPS_D)) continue;
        const double t = (Z_EPS_D - Z[m]) / (Z[m2] - Z[m]);
        const double xi = X[m] + t * (X[m2] - X[m]);
        const double yi = Y[m] + t * (Y[m2] - Y[m]);
        const double u = cx + fx * (xi / Z_EPS_D);
        const double v = cy + fy * (yi / Z_EPS_D);
        umin = fmin(umin, u); umax = fmax(umax, u);
        vmin = fmin(vmin, v); vmax = fmax(vmax, v);
      }
    }
  }
  r.status = 1;
  double lo_x = ceil(fmin(fmax(umin - 0.5625, x0 - 1.0), x0 + (double)w));
  double hi_x = floor(fmin(fmax(umax - 0.4375, x0 - 1.0), x0 + (double)w));
  double lo_y = ceil(fmin(fmax(vmin - 0.5625, y0 - 1.0), y0 + (double)h));
  double hi_y = floor(fmin(fmax(vmax - 0.4375, y0 - 1.0), y0 + (double)h));
  r.xl = (int)fmax(lo_x, (double)x0) - x0;
  r.xh = (int)fmin(hi_x, (double)(x0 + w - 1)) - x0;
  r.yl = (int)fmax(lo_y, (double)y0) - y0;
  r.yh = (int)fmin(hi_y, (double)(y0 + h - 1)) - y0;
  return r;
}

// Conservative pre-test for bin_box: true only when every box inside the
// ball of radius rad about c (octree frame) is rejected by bin_box.  The
// ball lies behind Z = 0 (all corners behind: no coverage), or it is
// farther from the camera than the near radius (the transformed corners'
// bounding box sits in the cube of half-size rad about the centre, so its
// distance is at least |X| - sqrt(3) rad) and lies behind the plane Z = e
// or outside one of the four planes through the camera that bound the
// window widened by 2 px.  Projected points then fall more than 2 px
// outside the window, where the pixel rule of bin_box leaves an empty
// rectangle; rounding of the FP64 corner arithmetic is many orders below
// that margin.  Requires fx, fy > 0; the view carries the near radius and
// the norms of the four side-plane normals (rounded up).
__host__ __device__ inline bool ball_culled(const double A[9], const double b[3],
                                            const double c[3], double rad,
                                            const ViewConst& V) {
  const double X = ((A[0] * c[0] + A[1] * c[1]) + A[2] * c[2]) + b[0];
  const double Y = ((A[3] * c[0] + A[4] * c[1]) + A[5] * c[2]) + b[1];
  const double Z = ((A[6] * c[0] + A[7] * c[1]) + A[8] * c[2]) + b[2];
  const double r = rad * (1.0 + 1e-6) + 1e-9;
  if (Z + r < 0.0) return true;
  // |X| > r_near + sqrt(3) r, compared squared (both sides positive)
  const double reach = V.rnear_m + 1.7320508075688772 * r;
  if (!((X * X + Y * Y) + Z * Z > reach * reach)) return false;
  if (Z + r < Z_EPS_D) return true;
  const double l = V.cx - (V.x0 - 2.0), rr = (V.x0 + V.w + 2.0) - V.cx;
  const double t = V.cy - (V.y0 - 2.0), bb = (V.y0 + V.h + 2.0) - V.cy;
  if (V.fx * X + l * Z + r * V.side_norm[0] < 0.0) return true;
  if (-V.fx * X + rr * Z + r * V.side_norm[1] < 0.0) return true;
  if (V.fy * Y + t * Z + r * V.side_norm[2] < 0.0) return true;
  if (-V.fy * Y + bb * Z + r * V.side_norm[3] < 0.0) return true;
  return false;
}

// Spread the low 21 bits of x to every third bit.
__device__ inline uint64_t spread3(uint64_t x) {
  x &= 0x1fffffull;
  x = (x | (x << 32)) & 0x1f00000000ffffull;
  x = (x | (x << 16)) & 0x1f0000ff0000ffull;
  x = (x | (x << 8)) & 0x100f00f00f00f00full;
  x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
  x = (x | (x << 2)) & 0x1249249249249249ull;
  return x;
}

// BSP painter's rank of a leaf (level l, index ijk, max level L) from the
// camera Q (octree frame, QBITS fixed point, clamped to [-1, 2] root
// sides).  At depth d < l the digit bit of axis a is the leaf's child bit
// XOR [Q >= the ancestor's splitting plane].  Per axis that is, in closed
// form: while the camera lies in the depth-d ancestor's slab the bit is the
// leaf's bit XOR the camera's (0 down to their first difference, 1 there);
// below it the camera is on one side of every plane, so the bits are the
// leaf's, inverted when the camera is above.  A camera outside the root
// slab is on one side of every plane.  The three l-bit strings are
// interleaved (axis a at bit 3 j + a) and placed at the top of 3 L bits.
__device__ inline uint64_t bsp_rank(const int ijk[3], int l, int L,
                                    const int64_t Q[3]) {
  if (l == 0) return 0;
  const uint32_t mask = (1u << l) - 1u;
  uint64_t r = 0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const uint32_t i = (uint32_t)ijk[a] & mask;
    uint32_t f;
    if (Q[a] < 0) {
      f = i;
    } else if (Q[a] >= (1ll << QBITS)) {
      f = ~i & mask;
    } else {
      const uint32_t qt = (uint32_t)(Q[a] >> (QBITS - l));
      const uint32_t dif = qt ^ i;
      if (dif == 0) {
        f = 0;
      } else {
        const int hb = 31 - __builtin_clz(dif);
        const uint32_t c = (qt >> hb) & 1u;
        f = (1u << hb) | ((c ? ~i : i) & ((1u << hb) - 1u));
      }
    }
    r |= spread3(f) << a;
  }
  return r << (3 * (L - l));
}

// Colour of one leaf from its SH coefficients ([S][3][N]) and the basis Y
// at the viewing direction, clamped at 0 after the +0.5 offset; all loads
// issued before the sums (same summation order as a plain loop).
template <int S>
__device__ inline void sh_colour(const float* sh, int N, int vox, const float* Y,
                                 float col[3]) {
  float c[3][S];
#pragma unroll
  for (int ch = 0; ch < 3; ++ch)
#pragma unroll
    for (int q = 0; q < S; ++q) c[ch][q] = sh[((int64_t)q * 3 + ch) * N + vox];
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) {
    float acc = 0.0f;
#pragma unroll
    for (int q = 0; q < S; ++q) acc = fmaf(Y[q], c[ch][q], acc);
    col[ch] = fmaxf(acc + 0.5f, 0.0f);
  }
}

constexpr int PAIR_PARTS = 256;
constexpr int PAIR_STRIDE = 16;   // 128 bytes between counters

struct PreArgs {
  const ViewConst* views;
  const VOConst* vo;
  const OctDev* oct;
  const int64_t* seg_start;   // padded: segments start on multiples of 64
  const uint32_t* wave_seg;   // segment of every wave of 64 items
  const int32_t* seg_len;     // leaves per segment
  uint64_t* wave_mask;        // visibility ballot per wave (pass 0 -> 1)
  int32_t n_seg;
  int32_t n_oct;
  int64_t n_items;
  int32_t rank_bits;
  uint32_t* block_count;
  // pass 0: (leaf, tile) pairs, summed into PAIR_PARTS counters (block b
  // adds to counter b % PAIR_PARTS, PAIR_STRIDE words apart) instead of one
  // word: a million blocks adding to one address serialised on it
  unsigned long long* pair_parts;
  const uint32_t* block_off;
  uint64_t* keys;
  uint32_t* vals;
  float4* s_geo;
  float4* s_g8a;
  float4* s_g8b;
  float4* s_cn;
  float4* s_nrm;
  uint32_t* s_vox;
  uint32_t* s_seg;              // (view, octree) segment of the record
  uint64_t* s_rect;
};

// Segment s fills the entries of its waves in the per-wave segment table
// (one block per segment; segments are padded to whole waves).
__global__ void k_wave_segments(const int64_t* __restrict__ pstart,
                                uint32_t* __restrict__ wave_seg) {
  const int s = blockIdx.x;
  const int64_t w0 = pstart[s] / 64, w1 = pstart[s + 1] / 64;
  for (int64_t w = w0 + threadIdx.x; w < w1; w += TPB) wave_seg[w] = (uint32_t)s;
}

// Segments (view, octree) start on multiples of 64 items, so each wave
// holds leaves of one segment: the segment search and the per-segment
// constants are wave-uniform (scalar loads).  Pass 0 stores each wave's
// visibility ballot and the block counts; pass 1 reads the ballots back,
// skips invisible waves and bins again only the visible lanes.
template <int PASS>
__global__ void __launch_bounds__(TPB) k_preprocess(PreArgs p) {
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t t0 = (int64_t)blockIdx.x * TPB + w * 64;
  const int64_t wave = (int64_t)blockIdx.x * (TPB / 64) + w;
  uint64_t m = 0;
  uint32_t woff = 0;
  if (PASS == 1) {
    const uint64_t* bm = p.wave_mask + (int64_t)blockIdx.x * (TPB / 64);
    for (int i = 0; i < w; ++i) woff += (uint32_t)__popcll(bm[i]);
    m = bm[w];
    if (!((m >> lane) & 1ull)) return;
  }
  // the wave's (view, octree) segment, from the per-wave table
  const int s = t0 < p.n_items ? (int)p.wave_seg[wave] : 0;
  const int vox = (int)(t0 - p.seg_start[s]) + lane;
  const int v = s / p.n_oct, k = s % p.n_oct;
  const ViewConst& V = p.views[v];
  const VOConst& C = p.vo[s];
  const OctDev& O = p.oct[k];
  bool vis = false;
  Rect r{0, 1, 0, 1, 0};
  int l = 0, ii = 0, jj = 0, kk = 0;
  if (t0 < p.n_items && vox < p.seg_len[s]) {
    unpack_geo(O.geo[vox], l, ii, jj, kk);
    const double h = ldexp(O.root_size, -l);
    double blo[3], bhi[3], ctr[3];
    const int ijk[3] = {ii, jj, kk};
    for (int a = 0; a < 3; ++a) {
      blo[a] = O.root_min[a] + (double)ijk[a] * h;
      bhi[a] = O.root_min[a] + (double)(ijk[a] + 1) * h;
      ctr[a] = O.root_min[a] + ((double)ijk[a] + 0.5) * h;
    }
    if (PASS == 1 || !ball_culled(C.A, C.b, ctr, 0.8660254037844386 * h, V)) {
      r = bin_box(C.A, C.b, blo, bhi, V.fx, V.fy, V.cx, V.cy, V.x0, V.y0,
                  V.w, V.h, V.rnear2);
      vis = r.status != 0 && r.xl <= r.xh && r.yl <= r.yh;
    }
  }
  if (PASS == 0) {
    __shared__ uint32_t wtot[TPB / 64];
    __shared__ uint32_t wpairs[TPB / 64];
    m = __ballot(vis);
    // tiles covered by the rectangle: the pairs this leaf emits
    uint32_t np = vis ? (uint32_t)(((r.xh >> 4) - (r.xl >> 4) + 1) *
                                   ((r.yh >> 4) - (r.yl >> 4) + 1))
                      : 0u;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) np += __shfl_xor(np, o, 64);
    if (lane == 0) {
      p.wave_mask[wave] = m;
      wtot[w] = (uint32_t)__popcll(m);
      wpairs[w] = np;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t tot = 0;
      unsigned long long pt = 0;
      for (int i = 0; i < TPB / 64; ++i) {
        tot += wtot[i];
        pt += wpairs[i];
      }
      p.block_count[blockIdx.x] = tot;
      if (pt) atomicAdd(p.pair_parts + (blockIdx.x % PAIR_PARTS) * PAIR_STRIDE, pt);
    }
    return;
  }
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const uint32_t slot = p.block_off[blockIdx.x] + woff + (uint32_t)__popcll(m & lt);
  // every load first (no store in between, so they are in flight together)
  const int N = O.n_vox;
  const float* const dens = O.dens;
  const int32_t* const cidx = O.corner_idx;
  int32_t ci[8];
#pragma unroll
  for (int c8 = 0; c8 < 8; ++c8) ci[c8] = cidx[(int64_t)c8 * N + vox];
  // leaf record in the octree frame relative to the camera
  const int ijk[3] = {ii, jj, kk};
  const double h = ldexp(O.root_size, -l);
  double rel[3];
  for (int a = 0; a < 3; ++a) rel[a] = C.rootrel[a] + (double)ijk[a] * h;
  // colour from SH at the direction camera -> leaf centre
  const double cx = rel[0] + 0.5 * h, cy = rel[1] + 0.5 * h, cz = rel[2] + 0.5 * h;
  const double rn = sqrt(cx * cx + cy * cy + cz * cz);
  const double inv_r = rn > 0 ? 1.0 / rn : 0.0;
  float Y[16];
  sh_basis(O.sh_degree, (float)(cx * inv_r), (float)(cy * inv_r),
           (float)(cz * inv_r), Y);
  float col[3];
  if (C.feat) {
    // feature render: the leaf's channels of this group in place of colour
#pragma unroll
    for (int ch = 0; ch < 3; ++ch)
      col[ch] = ch < C.feat_nc ? C.feat[(int64_t)ch * N + vox] : 0.0f;
  } else {
    switch (O.sh_degree) {
      case 0: sh_colour<1>(O.sh, N, vox, Y, col); break;
      case 1: sh_colour<4>(O.sh, N, vox, Y, col); break;
      case 2: sh_colour<9>(O.sh, N, vox, Y, col); break;
      default: sh_colour<16>(O.sh, N, vox, Y, col); break;
    }
  }
  float g[8];
#pragma unroll
  for (int c8 = 0; c8 < 8; ++c8) g[c8] = dens[ci[c8]];
  // depth rank: BSP painter's order from the quantised camera position
  const uint64_t rank = bsp_rank(ijk, l, O.max_level, C.Q);
  // normal: -grad of the trilinear field at the centre, rotated to world
  const float gx = 0.25f * ((g[1] - g[0]) + (g[3] - g[2]) + (g[5] - g[4]) + (g[7] - g[6]));
  const float gy = 0.25f * ((g[2] - g[0]) + (g[3] - g[1]) + (g[6] - g[4]) + (g[7] - g[5]));
  const float gz = 0.25f * ((g[4] - g[0]) + (g[5] - g[1]) + (g[6] - g[2]) + (g[7] - g[3]));
  const float gn = sqrtf(gx * gx + gy * gy + gz * gz);
  const float3 nl = gn > 0.0f ? make_float3(-gx / gn, -gy / gn, -gz / gn)
                              : make_float3(0.0f, 0.0f, 0.0f);
  const float3 nw = mat3_mul(C.R, nl);
  // stores
  p.keys[slot] = ((uint64_t)s << p.rank_bits) | rank;
  p.vals[slot] = slot;
  p.s_vox[slot] = (uint32_t)vox;
  p.s_seg[slot] = (uint32_t)s;
  // window-relative covered pixel bounds (inclusive), 16 bits each
  p.s_rect[slot] = (uint64_t)(uint32_t)r.xl | ((uint64_t)(uint32_t)r.xh << 16) |
                   ((uint64_t)(uint32_t)r.yl << 32) |
                   ((uint64_t)(uint32_t)r.yh << 48);
  p.s_geo[slot] = make_float4((float)rel[0], (float)rel[1], (float)rel[2],
                              (float)h);
  p.s_g8a[slot] = make_float4(g[0], g[1], g[2], g[3]);
  p.s_g8b[slot] = make_float4(g[4], g[5], g[6], g[7]);
  p.s_cn[slot] = make_float4(col[0], col[1], col[2], (float)(1.0 / h));
  p.s_nrm[slot] = make_float4(nw.x, nw.y, nw.z, 0.0f);
  (void)v;
}

// Records stay where the preprocess put them (slot order: view, octree,
// leaf; the preprocess also stores each slot's (view, octree) id).  For the
// depth-sorted order i -> slot order[i], the tile count of sorted record i.
__global__ void k_gather(int64_t n, const uint32_t* __restrict__ order,
                         const uint64_t* __restrict__ rect,
                         uint32_t* __restrict__ r_count) {
  const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (i >= n) return;
  const uint32_t sl = order[i];
  const uint64_t rc = rect[sl];
  const uint32_t tx0 = (rc & 0xFFFF) >> 4, tx1 = ((rc >> 16) & 0xFFFF) >> 4;
  const uint32_t ty0 = ((rc >> 32) & 0xFFFF) >> 4, ty1 = (rc >> 48) >> 4;
  r_count[i] = (tx1 - tx0 + 1) * (ty1 - ty0 + 1);
}

// Block b of the pair emission covers pairs [256 b, 256 b + 256); brec[b]
// is the record holding pair 256 b (each record marks the blocks whose
// first pair it holds, so every block gets exactly one).
__global__ void k_pair_block_rec(int64_t n_rec, int64_t n_pairs,
                                 const uint32_t* __restrict__ off,
                                 uint32_t* __restrict__ brec) {
  const int64_t r = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (r >= n_rec) return;
  const int64_t lo = off[r];
  const int64_t hi = r + 1 < n_rec ? (int64_t)off[r + 1] : n_pairs;
  for (int64_t b = (lo + TPB - 1) / TPB; b * TPB < hi; ++b) brec[b] = (uint32_t)r;
}

// Pair p of the depth-sorted record list: key = global tile, value = the
// record's slot (pairs come out in depth order within every tile).  Every
// record holds at least one pair (a visible leaf covers a tile), so the
// block's 256 pairs lie in records brec[b] .. brec[b] + 255: their offsets
// are staged in LDS and each thread finds its record there, instead of a
// search over all records.
__global__ void __launch_bounds__(TPB)
k_emit(int64_t n_pairs, int64_t n_rec, const uint32_t* __restrict__ off,
       const uint32_t* __restrict__ brec, const uint32_t* __restrict__ order,
       const uint64_t* __restrict__ rect, const uint32_t* __restrict__ seg,
       int n_oct, const ViewConst* __restrict__ views,
       uint32_t* __restrict__ pkey, uint32_t* __restrict__ pval) {
  __shared__ uint32_t soff[TPB];
  const int64_t p0 = (int64_t)blockIdx.x * TPB;
  const uint32_t r0 = brec[blockIdx.x];
  {
    const int64_t r = (int64_t)r0 + threadIdx.x;
    soff[threadIdx.x] = r < n_rec ? off[r] : (uint32_t)n_pairs;
  }
  __syncthreads();
  const int64_t p = p0 + threadIdx.x;
  if (p >= n_pairs) return;
  int lo = 0, hi = TPB - 1;  // the last record starting at or before p
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if ((int64_t)soff[mid] <= p) lo = mid; else hi = mid - 1;
  }
  const uint32_t sl = order[(int64_t)r0 + lo];
  const uint64_t rc = rect[sl];
  const uint32_t tx0 = (rc & 0xFFFF) >> 4, tx1 = ((rc >> 16) & 0xFFFF) >> 4;
  const uint32_t ty0 = ((rc >> 32) & 0xFFFF) >> 4;
  const uint32_t wdt = tx1 - tx0 + 1;
  const uint32_t i = (uint32_t)(p - soff[lo]);
  const ViewConst& V = views[seg[sl] / n_oct];
  pkey[p] = V.tile_base + (ty0 + i / wdt) * V.ntx + (tx0 + i % wdt);
  pval[p] = sl;
}

__global__ void k_tile_bounds(int64_t n, const uint32_t* __restrict__ key,
                              uint32_t* start, uint32_t* end) {
  const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (i >= n) return;
  const uint32_t k = key[i];
  if (i == 0 || key[i - 1] != k) start[k] = (uint32_t)i;
  if (i == n - 1 || key[i + 1] != k) end[k] = (uint32_t)(i + 1);
}

__device__ inline uint32_t first_oct_at_least(const uint32_t* pval,
                                              const uint32_t* rseg, int n_oct,
                                              uint32_t lo, uint32_t hi,
                                              uint32_t k) {
  while (lo < hi) {
    uint32_t mid = (lo + hi) >> 1;
    if (rseg[pval[mid]] % n_oct >= k) hi = mid; else lo = mid + 1;
  }
  return lo;
}

__global__ void k_tile_dir(int64_t n_tiles, const uint32_t* start,
                           const uint32_t* end, const uint32_t* pval,
                           const uint32_t* rseg, int n_oct, uint32_t* bgend) {
  const int64_t t = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (t >= n_tiles) return;
  bgend[t] = first_oct_at_least(pval, rseg, n_oct, start[t], end[t], 1);
}

__global__ void k_actor_ranges(int64_t n, const uint32_t* act_tile,
                               const uint32_t* act_oct,
                               const uint32_t* bgend, const uint32_t* end,
                               const uint32_t* pval, const uint32_t* rseg,
                               int n_oct, uint2* sub) {
  const int64_t e = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (e >= n) return;
  const uint32_t t = act_tile[e], k = act_oct[e];
  const uint32_t a = first_oct_at_least(pval, rseg, n_oct, bgend[t], end[t], k);
  const uint32_t b = first_oct_at_least(pval, rseg, n_oct, a, end[t], k + 1);
  sub[e] = make_uint2(a, b);
}

// Launch orders: heaviest work first, so long items start early and short
// ones fill the tail of the grid.  Items are bucketed by weight on a log
// scale with 8 steps per octave; the order inside a bucket (what the LDS
// atomics of the plan give, ascending ids in launch_order_by_weight)
// changes no result (items are independent).
// Up to this many lists (items) one block plans (orders) them: fewer
// launches; above it the device-wide scans and sort are faster.
constexpr int64_t PLAN_ONE_BLOCK = 32768;
__device__ inline uint32_t weight_bucket(uint32_t w) {
  if (w == 0) return 0;
  const uint32_t lz = __builtin_clz(w);
  const uint32_t mant = lz < 31 ? ((w << (lz + 1)) >> 29) : 0u;
  return (31u - lz) * 8u + mant;  // 0 .. 255
}

// Exclusive prefix sum over the 1024 threads of a block (x per thread);
// returns the thread's offset, *total receives the sum.
__device__ inline uint32_t block_scan_1024(uint32_t x, uint32_t* wsum,
                                           uint32_t* total) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  uint32_t incl = x;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(incl, o, 64);
    if (lane >= o) incl += y;
  }
  if (lane == 63) wsum[w] = incl;
  __syncthreads();
  if (tid == 0) {
    uint32_t acc = 0;
    for (int i = 0; i < 16; ++i) { const uint32_t t = wsum[i]; wsum[i] = acc; acc += t; }
    wsum[16] = acc;
  }
  __syncthreads();
  *total = wsum[16];
  return wsum[w] + incl - x;
}

// One block of 1024 threads: order items 0..n-1 by weight w[i] - (w0 ?
// w0[i] : 0), heaviest first.
__global__ void __launch_bounds__(1024) k_order_by_weight(int64_t n, const uint32_t* w0,
                                                          const uint32_t* w,
                                                          uint32_t* order) {
  __shared__ uint32_t cnt[256];
  __shared__ uint32_t off[256];
  const int tid = threadIdx.x;
  if (tid < 256) cnt[tid] = 0;
  __syncthreads();
  for (int64_t i = tid; i < n; i += 1024)
    atomicAdd(&cnt[255 - weight_bucket(w[i] - (w0 ? w0[i] : 0u))], 1u);
  __syncthreads();
  if (tid == 0) {
    uint32_t acc = 0;
    for (int b = 0; b < 256; ++b) { off[b] = acc; acc += cnt[b]; }
  }
  __syncthreads();
  for (int64_t i = tid; i < n; i += 1024)
    order[atomicAdd(&off[255 - weight_bucket(w[i] - (w0 ? w0[i] : 0u))], 1u)] = (uint32_t)i;
}

// Sort key of item i: heavier first (255 - weight bucket), value i.
__global__ void __launch_bounds__(TPB) k_weight_keys(int64_t n, const uint32_t* w0,
                                                     const uint32_t* w,
                                                     uint32_t* keys, uint32_t* vals) {
  const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (i >= n) return;
  keys[i] = 255u - weight_bucket(w[i] - (w0 ? w0[i] : 0u));
  vals[i] = (uint32_t)i;
}

// One stable 8-bit radix pass over the bucket keys (equal buckets keep
// ascending item order).
dv_status launch_order_by_weight(dv_ctx* ctx, int64_t n, const uint32_t* w0,
                                 const uint32_t* w, uint32_t* order, hipStream_t s) {
  if (n <= 0) return DV_OK;
  if (n <= PLAN_ONE_BLOCK) {
    hipLaunchKernelGGL(k_order_by_weight, dim3(1), dim3(1024), 0, s, n, w0, w, order);
    DV_TRY_HIP(hipGetLastError());
    return DV_OK;
  }
  DBuf keys, vals, kalt;
  DV_TRY(alloc_n<uint32_t>(ctx, keys, n, s));
  DV_TRY(alloc_n<uint32_t>(ctx, vals, n, s));
  DV_TRY(alloc_n<uint32_t>(ctx, kalt, n, s));
  // (a single item is its own order: written straight into order)
  hipLaunchKernelGGL(k_weight_keys, dim3(grid_for(n, TPB)), dim3(TPB), 0, s, n, w0,
                     w, keys.as<uint32_t>(), n == 1 ? order : vals.as<uint32_t>());
  DV_TRY_HIP(hipGetLastError());
  if (n == 1) return DV_OK;
  bool alt = false;
  DV_TRY(radix_sort_u32(ctx, keys.as<uint32_t>(), vals.as<uint32_t>(),
                        kalt.as<uint32_t>(), order, n, 8, s, &alt));
  return DV_OK;
}

// Work items of the compositing kernels.  Tile t's background list
// [start, bgend) becomes k = chunks_of(len) items (ids tile_ibase[t] + c)
// when its chunk slots [tile_pbase[t], + k) fit below max_slots, else one
// item; split tiles keep their partial states in those slots.  The launch
// order puts the longest chunks first.  counts[0] = items, counts[1] =
// slots reserved.  The same for the (tile, actor) lists when range is given
// (range[e] = [first, end) entries).  Device-wide: the slots each list
// wants and the items it is granted are two exclusive scans over the lists,
// and the order one stable radix pass over the items' weight buckets.
struct PlanArgs {
  int64_t n_tiles;
  const uint32_t* start;
  const uint32_t* bgend;
  const uint2* range;
  uint32_t chunk_len, max_slots;
  uint32_t* tile_nck;
  uint32_t* tile_ibase;
  uint32_t* tile_pbase;
  uint32_t* item_tile;
  uint32_t* item_chunk;
  uint32_t* order;
  uint32_t* counts;
  uint32_t* slot_tile;         // chunk slot -> its list (or null)
  int64_t max_items;           // length of order (ids past the items unused)
};

__device__ inline uint32_t plan_len(const PlanArgs& P, int64_t t) {
  return P.range ? P.range[t].y - P.range[t].x : P.bgend[t] - P.start[t];
}

// Slots wanted by list t (its chunks when it splits, else none).
__global__ void __launch_bounds__(TPB) k_plan_want(PlanArgs P, uint32_t* want) {
  const int64_t t = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (t >= P.n_tiles) return;
  const uint32_t kw = chunks_of(plan_len(P, t), P.chunk_len);
  want[t] = kw > 1 ? kw : 0u;
}

// Chunks granted: all of them when the list's slots (from the scan of the
// wanted slots) end within max_slots, else the list stays one item.
__global__ void __launch_bounds__(TPB) k_plan_grant(PlanArgs P) {
  const int64_t t = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (t >= P.n_tiles) return;
  const uint32_t kw = chunks_of(plan_len(P, t), P.chunk_len);
  const uint32_t pb = P.tile_pbase[t];
  P.tile_nck[t] = (kw > 1 && pb + kw <= P.max_slots) ? kw : 1u;
}

// Every id starts as unused (lightest key, so it sorts last).
__global__ void __launch_bounds__(TPB) k_plan_keys(int64_t n, uint32_t* keys,
                                                   uint32_t* vals) {
  const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (i >= n) return;
  keys[i] = 255u;
  vals[i] = (uint32_t)i;
}

// The items of list t (ids from the scan of the granted counts), their
// slots, and their order keys: heavier first.
__global__ void __launch_bounds__(TPB) k_plan_emit(PlanArgs P, uint32_t* keys) {
  const int64_t t = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (t >= P.n_tiles) return;
  const uint32_t len = plan_len(P, t);
  const uint32_t k = P.tile_nck[t], ib = P.tile_ibase[t], pb = P.tile_pbase[t];
  if (P.slot_tile && k > 1)
    for (uint32_t c = 0; c < k; ++c) P.slot_tile[pb + c] = (uint32_t)t;
  for (uint32_t c = 0; c < k; ++c) {
    uint32_t cb, ce;
    chunk_range(0, len, k, c, cb, ce);
    P.item_tile[ib + c] = (uint32_t)t;
    P.item_chunk[ib + c] = c;
    keys[ib + c] = 255u - weight_bucket(ce - cb);
  }
}

__global__ void k_plan_counts(PlanArgs P, const uint64_t* tot) {
  P.counts[0] = (uint32_t)tot[1];
  P.counts[1] = (uint32_t)min(tot[0], (uint64_t)P.max_slots);
}

// Small list sets: one block of 1024 threads per set (block b plans set
// b), walking the lists in rounds of 1024 consecutive ones (coalesced)
// with running totals; the order by LDS-atomic bucket offsets.
__global__ void __launch_bounds__(1024) k_plan_items(PlanArgs p0, PlanArgs p1) {
  const PlanArgs& P = blockIdx.x == 0 ? p0 : p1;
  const int64_t n_tiles = P.n_tiles;
  const uint32_t* start = P.start;
  const uint32_t* bgend = P.bgend;
  const uint2* range = P.range;
  const uint32_t chunk_len = P.chunk_len, max_slots = P.max_slots;
  uint32_t* tile_nck = P.tile_nck;
  uint32_t* tile_ibase = P.tile_ibase;
  uint32_t* tile_pbase = P.tile_pbase;
  uint32_t* item_tile = P.item_tile;
  uint32_t* item_chunk = P.item_chunk;
  uint32_t* order = P.order;
  uint32_t* counts = P.counts;
  __shared__ uint32_t wsum[17];
  __shared__ uint32_t cnt[256];
  __shared__ uint32_t off[256];
  auto list_len = [&](int64_t t) -> uint32_t {
    return range ? range[t].y - range[t].x : bgend[t] - start[t];
  };
  const int tid = threadIdx.x;
  if (tid < 256) cnt[tid] = 0;
  // rounds of 1024 consecutive lists (thread tid: list r0 + tid), running
  // totals of wanted slots and of items carried from round to round
  uint32_t pbc = 0, ibc = 0;
  for (int64_t r0 = 0; r0 < n_tiles; r0 += 1024) {
    const int64_t t = r0 + tid;
    const bool in = t < n_tiles;
    const uint32_t len = in ? list_len(t) : 0u;
    const uint32_t kw = in ? chunks_of(len, chunk_len) : 0u;
    uint32_t ts, ti;
    const uint32_t pb = pbc + block_scan_1024(kw > 1 ? kw : 0u, wsum, &ts);
    // chunks granted (a list whose slots would pass max_slots stays whole)
    const uint32_t k = (kw > 1 && pb + kw <= max_slots) ? kw : 1u;
    __syncthreads();
    const uint32_t ib = ibc + block_scan_1024(in ? k : 0u, wsum, &ti);
    if (in) {
      tile_nck[t] = k;
      tile_ibase[t] = ib;
      tile_pbase[t] = pb;
      if (P.slot_tile && k > 1)
        for (uint32_t c = 0; c < k; ++c) P.slot_tile[pb + c] = (uint32_t)t;
      for (uint32_t c = 0; c < k; ++c) {
        uint32_t cb, ce;
        chunk_range(0, len, k, c, cb, ce);
        item_tile[ib + c] = (uint32_t)t;
        item_chunk[ib + c] = c;
        atomicAdd(&cnt[255 - weight_bucket(ce - cb)], 1u);
      }
    }
    pbc += ts;
    ibc += ti;
    __syncthreads();
  }
  if (tid == 0) { counts[0] = ibc; counts[1] = min(pbc, max_slots); }
  if (tid == 0) {
    uint32_t acc = 0;
    for (int b = 0; b < 256; ++b) { off[b] = acc; acc += cnt[b]; }
  }
  __syncthreads();
  // heaviest first: items by descending weight bucket (each thread reads
  // back the lists it wrote)
  for (int64_t t = tid; t < n_tiles; t += 1024) {
    const uint32_t k = tile_nck[t], ib = tile_ibase[t];
    const uint32_t len = list_len(t);
    for (uint32_t c = 0; c < k; ++c) {
      uint32_t cb, ce;
      chunk_range(0, len, k, c, cb, ce);
      order[atomicAdd(&off[255 - weight_bucket(ce - cb)], 1u)] = ib + c;
    }
  }
}

static dv_status plan_items(dv_ctx* ctx, const PlanArgs& P, hipStream_t s) {
  const int64_t n = P.n_tiles, m = P.max_items;
  const dim3 gl(grid_for(n, TPB)), gi(grid_for(m, TPB));
  DBuf want, tot, keys, vals, kalt;
  DV_TRY(alloc_n<uint32_t>(ctx, want, n, s));
  DV_TRY(alloc_n<uint64_t>(ctx, tot, 2, s));
  DV_TRY(alloc_n<uint32_t>(ctx, keys, m, s));
  DV_TRY(alloc_n<uint32_t>(ctx, vals, m, s));
  DV_TRY(alloc_n<uint32_t>(ctx, kalt, m, s));
  hipLaunchKernelGGL(k_plan_want, gl, dim3(TPB), 0, s, P, want.as<uint32_t>());
  DV_TRY(exclusive_scan_u32(ctx, want.as<uint32_t>(), P.tile_pbase,
                            tot.as<uint64_t>(), n, s));
  hipLaunchKernelGGL(k_plan_grant, gl, dim3(TPB), 0, s, P);
  DV_TRY(exclusive_scan_u32(ctx, P.tile_nck, P.tile_ibase, tot.as<uint64_t>() + 1,
                            n, s));
  // (a single id is its own order: written straight into order)
  hipLaunchKernelGGL(k_plan_keys, gi, dim3(TPB), 0, s, m, keys.as<uint32_t>(),
                     m == 1 ? P.order : vals.as<uint32_t>());
  hipLaunchKernelGGL(k_plan_emit, gl, dim3(TPB), 0, s, P, keys.as<uint32_t>());
  hipLaunchKernelGGL(k_plan_counts, dim3(1), dim3(1), 0, s, P,
                     (const uint64_t*)tot.as<uint64_t>());
  DV_TRY_HIP(hipGetLastError());
  if (m > 1) {
    bool alt = false;
    DV_TRY(radix_sort_u32(ctx, keys.as<uint32_t>(), vals.as<uint32_t>(),
                          kalt.as<uint32_t>(), P.order, m, 8, s, &alt));
  }
  return DV_OK;
}

// ------------------------------------------------------------------ composite
struct Batch {
  float4 geo[TPB];
  float4 ga[TPB];
  float4 gb[TPB];
  float4 cn[TPB];
  float4 nrm[TPB];
  uint2 rect[TPB];
};

// NORMALS = false: the normal slot carries the leaf's far corner instead
// (see batch_slab).
template <bool NORMALS, class A>
__device__ inline void load_batch(Batch& B, const A& a, uint32_t base,
                                  uint32_t n) {
  const int tid = threadIdx.x;
  if ((uint32_t)tid < n) {
    const uint32_t r = a.pair_val[base + tid];
    const float4 geo = a.rec_geo[r];
    B.geo[tid] = geo;
    B.ga[tid] = a.rec_g8a[r];
    B.gb[tid] = a.rec_g8b[r];
    B.cn[tid] = a.rec_cn[r];
    if (NORMALS) {
      B.nrm[tid] = a.rec_nrm[r];
    } else {
      const float3 hi = leaf_hi(geo);
      B.nrm[tid] = make_float4(hi.x, hi.y, hi.z, 0.0f);
    }
    const uint64_t rc = a.rec_rect[r];
    B.rect[tid] = make_uint2((uint32_t)rc, (uint32_t)(rc >> 32));
  }
}

// Only what a slab test needs: leaf corner, far corner (in the normal
// slot, as load_batch<false> forms it) and the pixel rectangle.
template <class A>
__device__ inline void load_batch_geo(Batch& B, const A& a, uint32_t base,
                                      uint32_t n) {
  const int tid = threadIdx.x;
  if ((uint32_t)tid < n) {
    const uint32_t r = a.pair_val[base + tid];
    const float4 geo = a.rec_geo[r];
    B.geo[tid] = geo;
    const float3 hi = leaf_hi(geo);
    B.nrm[tid] = make_float4(hi.x, hi.y, hi.z, 0.0f);
    const uint64_t rc = a.rec_rect[r];
    B.rect[tid] = make_uint2((uint32_t)rc, (uint32_t)(rc >> 32));
  }
}

__device__ inline uint32_t src_code(int slot, int axis) {
  return ((uint32_t)slot << 2) | (uint32_t)axis;
}

// Build the pixel's ownership segments from the actor boxes of its tile.
// Reading for overlapping boxes: a point belongs to the lowest-index actor
// whose box contains it; the background owns the rest.
__device__ inline int build_segments(const CompArgs& a, uint32_t sbase,
                                     int n_at, uint32_t a_beg, int v,
                                     float3 d, int tid) {
  // box intervals -> slots [sbase, sbase + n_at)
  for (int j = 0; j < n_at; ++j) {
    const VOConst& C = a.vo[v * a.n_oct + a.act_oct[a_beg + j]];
    float3 dj = mat3_mul(C.Rt, d);
    float3 inv = safe_inv(dj);
    float t0, t1;
    int a0, a1;
    slab_axes(make_float3(C.boxlo[0], C.boxlo[1], C.boxlo[2]),
              make_float3(C.boxhi[0], C.boxhi[1], C.boxhi[2]), inv, t0, t1,
              a0, a1);
    uint32_t s0 = src_code(j, a0);
    if (t0 < a.tau_near) { t0 = a.tau_near; s0 = SRC_NONE; }
    uint32_t meta = s0 | (src_code(j, a1) << 10) | ((t1 > t0) ? (1u << 20) : 0u);
    a.seg_se[seg_index(sbase + j, tid)] = make_float2(t0, t1);
    a.seg_meta[seg_index(sbase + j, tid)] = meta;
  }
  // sweep over breakpoints in increasing order
  int nseg = 0;
  float cur = -F_INF;
  uint32_t cur_src = SRC_NONE;
  const uint32_t seg0 = sbase + n_at;
  for (int guard = 0; guard < 2 * n_at + 1; ++guard) {
    float nb = F_INF;
    uint32_t nb_src = SRC_NONE;
    for (int j = 0; j < n_at; ++j) {
      const uint32_t mj = a.seg_meta[seg_index(sbase + j, tid)];
      if (!(mj & (1u << 20))) continue;
      const float2 ab = a.seg_se[seg_index(sbase + j, tid)];
      if (ab.x > cur && ab.x < nb) { nb = ab.x; nb_src = mj & 0x3FF; }
      if (ab.y > cur && ab.y < nb) { nb = ab.y; nb_src = (mj >> 10) & 0x3FF; }
    }
    if (nb == F_INF) break;
    int owner = -1;
    for (int j = 0; j < n_at && cur > -F_INF; ++j) {
      const uint32_t mj = a.seg_meta[seg_index(sbase + j, tid)];
      if (!(mj & (1u << 20))) continue;
      const float2 ab = a.seg_se[seg_index(sbase + j, tid)];
      if (ab.x <= cur && cur < ab.y) { owner = j; break; }
    }
    if (owner >= 0) {
      const size_t li = seg_index(seg0 + nseg - 1, tid);
      bool extend = false;
      if (nseg > 0) {
        const uint32_t ml = a.seg_meta[li];
        extend = (int)(ml & 0xFF) == owner && a.seg_se[li].y == cur;
      }
      if (extend) {
        a.seg_se[li].y = nb;
        a.seg_meta[li] = (a.seg_meta[li] & ~(0x3FFu << 18)) | (nb_src << 18);
      } else {
        const size_t qi = seg_index(seg0 + nseg, tid);
        a.seg_se[qi] = make_float2(cur, nb);
        a.seg_meta[qi] = (uint32_t)owner | (cur_src << 8) | (nb_src << 18);
        a.seg_p0[qi] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        a.seg_p1[qi] = make_float4(0.0f, 0.0f, 0.0f, 1.0f);
        a.seg_t0[qi] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        a.seg_t1[qi] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        ++nseg;
      }
    }
    cur = nb;
    cur_src = nb_src;
  }
  return nseg;
}

// The same sweep with the box intervals in registers, for tiles of at most
// NR actor boxes: no box slot is written and read back, and the open
// segment is stored once it is complete.  Same comparisons in the same
// order, so the segments are those of build_segments.  Two instances:
// BS_REG boxes (nearly every tile) and BS_REG_BIG (a separate launch, so
// the common case keeps few registers).
constexpr int BS_REG = 8;
constexpr int BS_REG_BIG = 40;
__device__ inline void store_segment(const CompArgs& a, uint32_t q, int tid,
                                     float s, float e, uint32_t meta) {
  const size_t qi = seg_index(q, tid);
  a.seg_se[qi] = make_float2(s, e);
  a.seg_meta[qi] = meta;
  a.seg_p0[qi] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  a.seg_p1[qi] = make_float4(0.0f, 0.0f, 0.0f, 1.0f);
  a.seg_t0[qi] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  a.seg_t1[qi] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
}
template <int NR>
__device__ inline int build_segments_reg(const CompArgs& a, uint32_t seg0,
                                         int n_at, uint32_t a_beg, int v,
                                         float3 d, int tid) {
  float bs[NR], be[NR];
  uint32_t bm[NR];
#pragma unroll
  for (int j = 0; j < NR; ++j) {
    bs[j] = F_INF;
    be[j] = F_INF;
    bm[j] = 0u;  // no box: never a breakpoint, never an owner
    if (j < n_at) {
      const VOConst& C = a.vo[v * a.n_oct + a.act_oct[a_beg + j]];
      const float3 dj = mat3_mul(C.Rt, d);
      const float3 inv = safe_inv(dj);
      float t0, t1;
      int a0, a1;
      slab_axes(make_float3(C.boxlo[0], C.boxlo[1], C.boxlo[2]),
                make_float3(C.boxhi[0], C.boxhi[1], C.boxhi[2]), inv, t0, t1,
                a0, a1);
      uint32_t s0 = src_code(j, a0);
      if (t0 < a.tau_near) { t0 = a.tau_near; s0 = SRC_NONE; }
      bs[j] = t0;
      be[j] = t1;
      bm[j] = s0 | (src_code(j, a1) << 10) | ((t1 > t0) ? (1u << 20) : 0u);
    }
  }
  int nseg = 0;
  float cur = -F_INF;
  uint32_t cur_src = SRC_NONE;
  float ls = 0.0f, le = 0.0f;  // the last segment, stored when complete
  uint32_t lm = 0u;
  for (int guard = 0; guard < 2 * n_at + 1; ++guard) {
    float nb = F_INF;
    uint32_t nb_src = SRC_NONE;
#pragma unroll
    for (int j = 0; j < NR; ++j) {
      if (!(bm[j] & (1u << 20))) continue;
      if (bs[j] > cur && bs[j] < nb) { nb = bs[j]; nb_src = bm[j] & 0x3FF; }
      if (be[j] > cur && be[j] < nb) { nb = be[j]; nb_src = (bm[j] >> 10) & 0x3FF; }
    }
    if (nb == F_INF) break;
    int owner = -1;
    if (cur > -F_INF) {
      // the lowest index containing cur
#pragma unroll
      for (int j = NR - 1; j >= 0; --j)
        if ((bm[j] & (1u << 20)) && bs[j] <= cur && cur < be[j]) owner = j;
    }
    if (owner >= 0) {
      if (nseg > 0 && (int)(lm & 0xFF) == owner && le == cur) {
        le = nb;
        lm = (lm & ~(0x3FFu << 18)) | (nb_src << 18);
      } else {
        if (nseg > 0) store_segment(a, seg0 + nseg - 1, tid, ls, le, lm);
        ls = cur;
        le = nb;
        lm = (uint32_t)owner | (cur_src << 8) | (nb_src << 18);
        ++nseg;
      }
    }
    cur = nb;
    cur_src = nb_src;
  }
  if (nseg > 0) store_segment(a, seg0 + nseg - 1, tid, ls, le, lm);
  return nseg;
}

__device__ inline int next_seg_of(const CompArgs& a, uint32_t seg0, int nseg,
                                  int from, int j, int tid) {
  for (int q = from; q < nseg; ++q)
    if ((int)(a.seg_meta[seg_index(seg0 + q, tid)] & 0xFF) == j) return q;
  return nseg;
}

// Final composite with the sky behind the voxels (Eq. 2) into the outputs;
// d is the pixel's unit world ray direction.
template <class A>
__device__ inline void write_outputs(const A& a, const ViewConst& V, int v,
                                     int px, int py, float3 C3, float D,
                                     float3 N3, float T, float3 d) {
  const dv_outputs& O = a.outs[v];
  const size_t hw = (size_t)V.w * V.h, o = (size_t)py * V.w + px;
  if ((a.mask & DV_OUT_RGB) && O.rgb) {
    const float3 cs = sky_colour(a, d);
    O.rgb[o] = fmaf(T, cs.x, C3.x);
    O.rgb[hw + o] = fmaf(T, cs.y, C3.y);
    O.rgb[2 * hw + o] = fmaf(T, cs.z, C3.z);
  }
  if ((a.mask & DV_OUT_DEPTH) && O.depth) O.depth[o] = D;
  if ((a.mask & DV_OUT_NORMAL) && O.normal) {
    O.normal[o] = N3.x;
    O.normal[hw + o] = N3.y;
    O.normal[2 * hw + o] = N3.z;
  }
  if ((a.mask & DV_OUT_T) && O.T) O.T[o] = T;
}

// Forward, part 1a (tiles with actor boxes): per pixel, the ownership
// segments of the actor boxes its ray meets.
// One block per (tile, actor) pair; the block of the tile's first pair
// builds the tile's segments, the others exit (no block is spent on tiles
// without actor boxes).  A tile of more than BS_REG boxes (about one in a
// hundred) is queued in big = {count, tiles...} for k_build_segments_big.
__global__ void __launch_bounds__(TPB) k_build_segments(CompArgs a, uint32_t* big) {
  const uint32_t gt = a.act_tile[blockIdx.x];
  const uint32_t a_beg = a.act_beg[gt];
  if (blockIdx.x != a_beg) return;
  const int n_at = (int)(a.act_beg[gt + 1] - a_beg);
  const int tid = threadIdx.x;
  if (n_at > BS_REG) {
    if (tid == 0) big[1 + atomicAdd(big, 1u)] = gt;
    return;
  }
  const PixSetup P = pixel_setup(a, gt, tid);
  int nseg = 0;
  if (P.valid)
    nseg = build_segments_reg<BS_REG>(a, 3 * a_beg + n_at, n_at, a_beg, P.v, P.d, tid);
  a.pix_nseg[P.pix] = (uint32_t)nseg;
}

// The queued tiles (grid-stride over the queue): at most BS_REG_BIG boxes
// in registers, more through the box slots in memory.
__global__ void __launch_bounds__(TPB) k_build_segments_big(CompArgs a,
                                                            const uint32_t* big) {
  const uint32_t cnt = big[0];
  const int tid = threadIdx.x;
  for (uint32_t i = blockIdx.x; i < cnt; i += gridDim.x) {
    const uint32_t gt = big[1 + i];
    const uint32_t a_beg = a.act_beg[gt];
    const int n_at = (int)(a.act_beg[gt + 1] - a_beg);
    const PixSetup P = pixel_setup(a, gt, tid);
    int nseg = 0;
    if (P.valid)
      nseg = n_at <= BS_REG_BIG
                 ? build_segments_reg<BS_REG_BIG>(a, 3 * a_beg + n_at, n_at, a_beg,
                                                  P.v, P.d, tid)
                 : build_segments(a, 3 * a_beg, n_at, a_beg, P.v, P.d, tid);
    a.pix_nseg[P.pix] = (uint32_t)nseg;
  }
}

// Segments of actor j on the ray of this lane: count, first and last.
// (the loads of 8 segments in flight together)
__device__ inline int segs_of_actor(const CompArgs& a, uint32_t seg0, int nseg,
                                    int j, int tid, int& qfirst, int& qlast) {
  int nj = 0;
  qfirst = nseg;
  qlast = -1;
  for (int i0 = 0; i0 < nseg; i0 += 8) {
    uint32_t m[8];
#pragma unroll
    for (int k = 0; k < 8; ++k)
      m[k] = i0 + k < nseg ? a.seg_meta[seg_index(seg0 + i0 + k, tid)] : 0u;
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (i0 + k < nseg && (int)(m[k] & 0xFF) == j) {
        if (nj == 0) qfirst = i0 + k;
        qlast = i0 + k;
        ++nj;
      }
  }
  return nj;
}

// Forward, part 1b: one block per actor work item, a chunk of one (tile,
// actor) list: every segment of that actor on the tile's rays composited
// into a partial state (C, D, N, T) with its tail sums.  Actors are
// independent here, so they run as separate blocks; a long list is split
// into chunks for rays with a single segment of the actor (partials per
// chunk, merged by k_actor_merge), while rays with several segments of it
// (overlapping boxes) walk the whole list in chunk 0.
template <bool NORMALS, int KC>
__global__ void __launch_bounds__(TPB, NORMALS ? 4 : 5) k_actor_fwd(CompArgs a) {
  __shared__ Batch B;
  if (blockIdx.x >= a.aplan_counts[0]) return;
  const uint32_t item = a.aorder[blockIdx.x];
  const uint32_t e = a.aitem_pair[item], chunk = a.aitem_chunk[item];
  const uint32_t nck = a.pair_nck[e];
  const uint32_t gt = a.act_tile[e];
  const uint32_t a_beg = a.act_beg[gt];
  const int n_at = (int)(a.act_beg[gt + 1] - a_beg);
  const int j = (int)(e - a_beg);
  const int tid = threadIdx.x;
  const PixSetup P = pixel_setup(a, gt, tid);
  const int v = P.v, bx = P.bx, by = P.by;
  const float3 d = P.d;
  const int K = a.K;
  const float invK = 1.0f / (float)K;
  uint32_t n_test = 0, n_piece = 0;
  const uint32_t seg0 = 3 * a_beg + n_at;
  const int nseg = P.valid ? (int)a.pix_nseg[P.pix] : 0;
  int qfirst, qlast;
  const int nj = segs_of_actor(a, seg0, nseg, j, tid, qfirst, qlast);
  const bool simple = nck > 1 && nj == 1;
  bool has = nj > 0 && (nck == 1 || simple || chunk == 0);
  if (!__syncthreads_or(has)) return;
  const bool any_full = __syncthreads_or(has && nck > 1 && !simple);
  const uint2 sub = a.act_sub[e];
  uint32_t cb = sub.x, ce = sub.y;
  if (nck > 1) chunk_range(sub.x, sub.y, nck, chunk, cb, ce);
  // entries this lane walks, and the block's loop range
  const uint32_t wlo = simple ? cb : sub.x, whi = simple ? ce : sub.y;
  const uint32_t lo = any_full ? sub.x : cb, hi = any_full ? sub.y : ce;
  const VOConst& C = a.vo[v * a.n_oct + a.act_oct[e]];
  const float3 dj = mat3_mul(C.Rt, d);
  const float3 inv = safe_inv(dj);
  int q = qfirst;
  float qs = 0, qe = 0;
  // p0/p1: partial state of segment q; t0s/t1s: its tail part
  float4 p0 = make_float4(0, 0, 0, 0), p1 = make_float4(0, 0, 0, 1);
  float4 t0s = make_float4(0, 0, 0, 0);
  float3 t1s = make_float3(0, 0, 0);
  bool qdone = false;
  auto store_q = [&](int qq) {
    float4* dst;
    if (simple) {
      dst = a.apart + (((size_t)a.pair_pbase[e] + chunk) * TPB + tid) * 4;
      dst[0] = p0;
      dst[1] = p1;
      dst[2] = t0s;
      dst[3] = make_float4(t1s.x, t1s.y, t1s.z, 0.0f);
      return;
    }
    const size_t qi = seg_index(seg0 + qq, tid);
    a.seg_p0[qi] = p0;
    a.seg_p1[qi] = p1;
    a.seg_t0[qi] = t0s;
    a.seg_t1[qi] = make_float4(t1s.x, t1s.y, t1s.z, 0.0f);
  };
  if (has) {
    const float2 se = a.seg_se[seg_index(seg0 + q, tid)];
    qs = se.x; qe = se.y;
  }
  // a lane whose chord reached past its single segment is finished (fast
  // path below)
  bool fin = false;
  // once the last segment of the actor is done (T below the stop threshold)
  // the lane has nothing left in this list
  auto live = [&]() { return has && !fin && !(qdone && q == qlast); };
  // composite the piece [pa, pb) of entry r into segment q's partial state
  auto piece = [&](uint32_t r, const float4& geo, float pa, float pb) {
    const float4 cn = B.cn[r];
    const float tau = piece_tau<KC>(geo, B.ga[r], B.gb[r], cn.w, dj, pa, pb, K,
                                    invK, a.c, a.inv_c);
    const float e_ = fast_exp(-tau);
    const float wgt = p1.w * opacity(tau, e_);
    const float wt = p1.w < T_REBASE ? wgt : 0.0f;
    const float mid = 0.5f * (pa + pb);
    p0.x = fmaf(wgt, cn.x, p0.x); t0s.x = fmaf(wt, cn.x, t0s.x);
    p0.y = fmaf(wgt, cn.y, p0.y); t0s.y = fmaf(wt, cn.y, t0s.y);
    p0.z = fmaf(wgt, cn.z, p0.z); t0s.z = fmaf(wt, cn.z, t0s.z);
    p0.w = fmaf(wgt, mid, p0.w); t0s.w = fmaf(wt, mid, t0s.w);
    if (NORMALS) {
      const float4 nr = B.nrm[r];
      p1.x = fmaf(wgt, nr.x, p1.x); t1s.x = fmaf(wt, nr.x, t1s.x);
      p1.y = fmaf(wgt, nr.y, p1.y); t1s.y = fmaf(wt, nr.y, t1s.y);
      p1.z = fmaf(wgt, nr.z, p1.z); t1s.z = fmaf(wt, nr.z, t1s.z);
    }
    p1.w *= e_;
    if (p1.w < a.eps) qdone = true;
  };
  // waves in which no ray has several segments of this actor (boxes that do
  // not overlap along the ray) take a walk without segment advances: the
  // piece is the chord clipped to [qs, qe), and a chord reaching past qe
  // ends the lane (later entries lie farther along the ray)
  const bool single = __ballot(nj > 1) == 0;
  // one entry of the single-segment walk
  auto single_entry = [&](uint32_t r, uint32_t base) {
    if (live() && base + r >= wlo && base + r < whi) {
      const float4 geo = B.geo[r];
      float t0, t1;
      batch_slab<NORMALS>(B, r, geo, inv, t0, t1);
      ++n_test;
      const float pa = fmaxf(t0, qs), pb = fminf(t1, qe);
      if (pb > pa) {
        piece(r, geo, pa, pb);
        ++n_piece;
      }
      if (t1 > t0 && t1 > qs && (qe <= t0 || t1 > qe)) fin = true;
    }
  };
  for (uint32_t base = lo; base < hi; base += TPB) {
    const uint32_t nb = min((uint32_t)TPB, hi - base);
    load_batch<NORMALS>(B, a, base, nb);
    __syncthreads();
    uint64_t wm[4];
    const uint64_t lv = __ballot(live());
    wave_live_masks(B.rect, nb, bx, by, lv, wm);
    if (single && sparse_cover(B.rect, nb, bx, by, lv, wm)) {
      // entries cover few of the wave's pixels (far actors): every lane
      // walks its own entries, those whose rectangle holds its pixel
      uint64_t pm[4];
      lane_masks(B.rect, wm, P.px, P.py, pm);
      for (int c = 0; c < 4; ++c) {
        uint64_t m = pm[c];
        while (__ballot(m != 0 && live()) != 0) {
          const uint32_t r =
              m != 0 ? (uint32_t)c * 64 + (uint32_t)__builtin_ctzll(m) : 0u;
          if (m != 0) {
            m &= m - 1;
            single_entry(r, base);
          }
        }
      }
    } else {
    for (int c = 0; c < 4; ++c) {
      uint64_t m = wm[c];
      if (single) {
        while (m != 0 && __ballot(live()) != 0) {
          const uint32_t r = (uint32_t)c * 64 + (uint32_t)__builtin_ctzll(m);
          m &= m - 1;
          single_entry(r, base);
        }
        continue;
      }
      while (m != 0 && __ballot(live()) != 0) {
        const uint32_t r = (uint32_t)c * 64 + (uint32_t)__builtin_ctzll(m);
        m &= m - 1;
        if (!live() || base + r < wlo || base + r >= whi) continue;
        const float4 geo = B.geo[r];
        float t0, t1;
        batch_slab<NORMALS>(B, r, geo, inv, t0, t1);
        ++n_test;
        if (!(t1 > t0) || t1 <= qs) continue;
        while (true) {
          if (qe <= t0) {
            // segment q finished: store and move to the next one of j
            store_q(q);
            q = next_seg_of(a, seg0, nseg, q + 1, j, tid);
            if (q >= nseg) { has = false; break; }
            const float2 se = a.seg_se[seg_index(seg0 + q, tid)];
            qs = se.x; qe = se.y;
            p0 = make_float4(0, 0, 0, 0); p1 = make_float4(0, 0, 0, 1);
            t0s = make_float4(0, 0, 0, 0); t1s = make_float3(0, 0, 0);
            qdone = false;
            continue;
          }
          const float pa = fmaxf(t0, qs), pb = fminf(t1, qe);
          if (pb > pa && !qdone) {
            piece(r, geo, pa, pb);
            ++n_piece;
          }
          if (t1 > qe) {  // chord continues into a later segment of j
            qe = t0;      // forces the store-and-advance branch above
            continue;
          }
          break;
        }
      }
    }
    }
    if (!__syncthreads_or(live())) break;
  }
  if (has) store_q(q);
  count_work(a.counters, 4, n_test, n_piece);
}

// Forward, part 1c (actor lists of several chunks): per ray with a single
// segment of the actor, merge the chunk partials in order into the
// segment's state.  The segment's tail sums are per chunk (each chunk has
// its own T), so the backward takes them from the chunk partials.
__global__ void __launch_bounds__(TPB) k_actor_merge(CompArgs a) {
  const uint32_t e = blockIdx.x;
  const uint32_t nck = a.pair_nck[e];
  if (nck <= 1) return;
  const uint32_t gt = a.act_tile[e];
  const uint32_t a_beg = a.act_beg[gt];
  const int n_at = (int)(a.act_beg[gt + 1] - a_beg);
  const int tid = threadIdx.x;
  const size_t pix = (size_t)gt * TPB + tid;
  const uint32_t seg0 = 3 * a_beg + n_at;
  const int nseg = (int)a.pix_nseg[pix];
  int qfirst, qlast;
  if (segs_of_actor(a, seg0, nseg, (int)(e - a_beg), tid, qfirst, qlast) != 1) return;
  const float4* part = a.apart + ((size_t)a.pair_pbase[e] * TPB + tid) * 4;
  float4 p0 = make_float4(0, 0, 0, 0), p1 = make_float4(0, 0, 0, 1);
  for (uint32_t c = 0; c < nck; ++c) {
    const float4 c0 = part[(size_t)c * TPB * 4], c1 = part[(size_t)c * TPB * 4 + 1];
    const float T = p1.w;
    p0.x = fmaf(T, c0.x, p0.x); p0.y = fmaf(T, c0.y, p0.y);
    p0.z = fmaf(T, c0.z, p0.z); p0.w = fmaf(T, c0.w, p0.w);
    p1.x = fmaf(T, c1.x, p1.x); p1.y = fmaf(T, c1.y, p1.y);
    p1.z = fmaf(T, c1.z, p1.z);
    p1.w = T * c1.w;
  }
  const size_t qi = seg_index(seg0 + qfirst, tid);
  a.seg_p0[qi] = p0;
  a.seg_p1[qi] = p1;
  a.seg_t0[qi] = make_float4(0, 0, 0, 0);
  a.seg_t1[qi] = make_float4(0, 0, 0, 0);
}

// Forward, part 2 (chunked tiles, chunks c > 0): B_c of every pixel with
// ownership segments, the entry depth of its first non-empty chord among
// the chunk's entries (B_c only places segments between chunks, so tiles
// without actor boxes and pixels without segments skip the search and
// never read it).  The grid walks the chunk slots (slot -> list from the
// plan; each chunk in CB_SPLIT parts, one per block), so no block is spent
// on unchunked tiles; every block leaves once the slots run out.
__global__ void __launch_bounds__(TPB) k_chunk_bounds(CompArgs a,
                                                      const uint32_t* slot_tile) {
  __shared__ Batch B;
  const uint32_t part = blockIdx.x % CB_SPLIT;
  const uint32_t n_slots = a.plan_counts[1];
  const int tid = threadIdx.x;
  for (uint32_t sl = blockIdx.x / CB_SPLIT; sl < n_slots;
       sl += gridDim.x / CB_SPLIT) {
    const uint32_t gt = slot_tile[sl];
    if (gt == 0xFFFFFFFFu) continue;           // slot of no granted list
    const uint32_t c = sl - a.tile_pbase[gt];
    if (c == 0) continue;                      // chunk 0 starts at the camera
    if (a.act_beg[gt + 1] == a.act_beg[gt]) continue;   // no segments here
    const uint32_t nck = a.tile_nck[gt];
    const PixSetup P = pixel_setup(a, gt, tid);
    const float3 inv = safe_inv(P.d);
    uint32_t cb, ce;
    chunk_range(a.tile_start[gt], a.tile_bgend[gt], nck, c, cb, ce);
    {
      // this block's part of the chunk
      const uint32_t len = ce - cb;
      const uint32_t pb = cb + (uint32_t)((uint64_t)len * part / CB_SPLIT);
      ce = cb + (uint32_t)((uint64_t)len * (part + 1) / CB_SPLIT);
      cb = pb;
    }
    float Bc = F_INF;
    bool found = !P.valid || a.pix_nseg[P.pix] == 0;
    const bool all_found = __syncthreads_and(found);
    for (uint32_t base = cb; base < ce && !all_found; base += TPB) {
      const uint32_t nb = min((uint32_t)TPB, ce - base);
      load_batch_geo(B, a, base, nb);
      __syncthreads();
      uint64_t wm[4];
      wave_live_masks(B.rect, nb, P.bx, P.by, __ballot(!found), wm);
      for (int q = 0; q < 4; ++q) {
        uint64_t m = wm[q];
        // four entries per step: independent slab tests, and the first
        // chord among them in list order
        while (m != 0 && __ballot(!found) != 0) {
          uint32_t r[4];
          int nr = 0;
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            r[k] = (uint32_t)q * 64 + (uint32_t)__builtin_ctzll(m | (1ull << 63));
            if (m != 0) { m &= m - 1; ++nr; }
          }
          float h0[4];
          bool hk[4];
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const float4 geo = B.geo[r[k]];
            float t0, t1;
            batch_slab<false>(B, r[k], geo, inv, t0, t1);
            t0 = fmaxf(t0, a.tau_near);
            h0[k] = t0;
            hk[k] = k < nr && t1 > t0;
          }
          if (!found) {
#pragma unroll
            for (int k = 3; k >= 0; --k)
              if (hk[k]) Bc = h0[k];
            found = hk[0] || hk[1] || hk[2] || hk[3];
          }
        }
      }
      if (__syncthreads_and(found)) break;
    }
    a.chunk_b[((size_t)sl * CB_SPLIT + part) * TPB + tid] = Bc;
    __syncthreads();
  }
}

// Forward, part 3: the background walk of one work item (a tile, or one
// chunk of a long tile), one 256-thread block per item (each wave an 8x8
// quadrant), asset segments spliced in as the walk reaches them.  Sums are
// kept twice: over all pieces, and over the tail (pieces entered with
// T < T_REBASE), which the backward needs for its suffixes.  A tile of one
// chunk writes the outputs; a chunk writes its partial state (T starts at
// 1 in every chunk, and so does the stop test) for k_chunk_merge.
// KC = 1 fixes one sample per piece at compile time.
// The walk of one item (also run by the persistent serving kernel, which
// drains items of several renders); B and blk_work: the block's LDS.
template <bool NORMALS, int KC, class A>
__device__ __forceinline__ void composite_item(const A& a, uint32_t idx,
                                               Batch& B, uint32_t& blk_work) {
  const uint32_t item = a.order[idx];
  const uint32_t gt = a.item_tile[item], chunk = a.item_chunk[item];
  const uint32_t nck = a.tile_nck[gt];
  const int tid = threadIdx.x;
  const PixSetup P = pixel_setup(a, gt, tid);
  const int v = P.v, px = P.px, py = P.py, bx = P.bx, by = P.by;
  const bool valid = P.valid;
  const float3 d = P.d;
  const size_t pix = P.pix;
  const ViewConst& V = a.views[v];
  const int K = a.K;
  const float invK = 1.0f / (float)K;
  uint32_t n_test = 0, n_piece = 0;
  uint32_t w_test = 0, w_piece = 0;  // wave-level counts (straight-line)
  uint32_t w_iter = 0, w_hit = 0;
  const uint32_t a_beg = a.act_beg[gt];
  const int n_at = (int)(a.act_beg[gt + 1] - a_beg);
  const uint32_t seg0 = 3 * a_beg + n_at;
  const int nseg = (n_at > 0 && valid) ? (int)a.pix_nseg[pix] : 0;

  // totals C3/D/N3 and tail sums CT/DT/NT
  float3 C3 = make_float3(0, 0, 0), N3 = make_float3(0, 0, 0);
  float3 CT = make_float3(0, 0, 0), NT = make_float3(0, 0, 0);
  // an off-window lane starts below the stop threshold (a.eps > 0)
  float D = 0.0f, DT = 0.0f, T = valid ? 1.0f : 0.0f;
  auto live = [&]() { return T >= a.eps; };
  const float3 inv = safe_inv(d);
  auto add_piece = [&](uint32_t r, const float4& geo, float pa, float pb) {
    const float4 cn = B.cn[r];
    const float tau = piece_tau<KC>(geo, B.ga[r], B.gb[r], cn.w, d, pa, pb, K,
                                    invK, a.c, a.inv_c);
    const float e = fast_exp(-tau);
    const float wgt = T * opacity(tau, e);
    const float wt = T < T_REBASE ? wgt : 0.0f;
    const float mid = 0.5f * (pa + pb);
    C3.x = fmaf(wgt, cn.x, C3.x); CT.x = fmaf(wt, cn.x, CT.x);
    C3.y = fmaf(wgt, cn.y, C3.y); CT.y = fmaf(wt, cn.y, CT.y);
    C3.z = fmaf(wgt, cn.z, C3.z); CT.z = fmaf(wt, cn.z, CT.z);
    D = fmaf(wgt, mid, D); DT = fmaf(wt, mid, DT);
    if (NORMALS) {
      const float4 nr = B.nrm[r];
      N3.x = fmaf(wgt, nr.x, N3.x); NT.x = fmaf(wt, nr.x, NT.x);
      N3.y = fmaf(wgt, nr.y, N3.y); NT.y = fmaf(wt, nr.y, NT.y);
      N3.z = fmaf(wgt, nr.z, N3.z); NT.z = fmaf(wt, nr.z, NT.z);
    }
    T *= e;
  };
  uint32_t beg, bgend;
  chunk_range(a.tile_start[gt], a.tile_bgend[gt], nck, chunk, beg, bgend);
  // chunk boundaries: only to place a lane's segments between chunks
  float Bc = -F_INF, Bn = F_INF;
  if (nseg > 0) chunk_bounds(a, gt, nck, chunk, tid, Bc, Bn);
  // An entry takes the straight-line iteration (one piece per chord) when no
  // lane's chord meets a segment, which always holds for lanes without
  // segments (excl = -inf, ns = +inf); only the other entries splice.
  int qn = 0;
  while (qn < nseg && a.seg_se[seg_index(seg0 + qn, tid)].x < Bc) ++qn;
  float excl = qn > 0 ? a.seg_se[seg_index(seg0 + qn - 1, tid)].y : -F_INF;
  float ns = qn < nseg ? a.seg_se[seg_index(seg0 + qn, tid)].x : F_INF;
  auto splice = [&](int qq) {
    const size_t qi = seg_index(seg0 + qq, tid);
    const float4 q0 = a.seg_p0[qi], q1 = a.seg_p1[qi];
    const float ts = T < T_REBASE ? T : 0.0f;
    C3.x = fmaf(T, q0.x, C3.x); CT.x = fmaf(ts, q0.x, CT.x);
    C3.y = fmaf(T, q0.y, C3.y); CT.y = fmaf(ts, q0.y, CT.y);
    C3.z = fmaf(T, q0.z, C3.z); CT.z = fmaf(ts, q0.z, CT.z);
    D = fmaf(T, q0.w, D); DT = fmaf(ts, q0.w, DT);
    if (NORMALS) {
      N3.x = fmaf(T, q1.x, N3.x); NT.x = fmaf(ts, q1.x, NT.x);
      N3.y = fmaf(T, q1.y, N3.y); NT.y = fmaf(ts, q1.y, NT.y);
      N3.z = fmaf(T, q1.z, N3.z); NT.z = fmaf(ts, q1.z, NT.z);
    }
    T *= q1.w;
    excl = a.seg_se[qi].y;
  };
  for (uint32_t base = beg; base < bgend; base += TPB) {
    const uint32_t nb = min((uint32_t)TPB, bgend - base);
    load_batch<NORMALS>(B, a, base, nb);
    __syncthreads();
    uint64_t wm[4];
    wave_live_masks(B.rect, nb, bx, by, __ballot(live()), wm);
    for (int c = 0; c < 4; ++c) {
      uint64_t m = wm[c];
      while (m != 0) {
        const uint64_t lm = __ballot(live());
        if (lm == 0) break;
        const uint32_t r = (uint32_t)c * 64 + (uint32_t)__builtin_ctzll(m);
        m &= m - 1;
        const float4 geo = B.geo[r];
        float t0, t1;
        batch_slab<NORMALS>(B, r, geo, inv, t0, t1);
        t0 = fmaxf(t0, a.tau_near);
        const bool chord = live() && t1 > t0;
        // no lane's chord meets a segment: one piece [t0, t1) per chord
        const bool plain = !chord || (excl <= t0 && ns >= t1);
        if (__ballot(!plain) == 0) {
          const uint64_t hm = __ballot(chord);
          w_test += (uint32_t)__popcll(lm);
          w_piece += (uint32_t)__popcll(hm);
          ++w_iter;
          w_hit += hm != 0 ? 1u : 0u;
          // (a straight-line form with the empty piece for lanes without a
          // chord, as in the backward, is slower here)
          if (chord) add_piece(r, geo, t0, t1);
          continue;
        }
        if (!live()) continue;
        ++n_test;
        if (!(t1 > t0)) continue;
        float pa = fmaxf(t0, excl);
        while (pa < t1 && live()) {
          if (pa >= ns) {
            splice(qn);
            pa = fmaxf(pa, excl);
            ++qn;
            ns = qn < nseg ? a.seg_se[seg_index(seg0 + qn, tid)].x : F_INF;
            continue;
          }
          const float pb = fminf(t1, ns);
          add_piece(r, geo, pa, pb);
          ++n_piece;
          pa = pb;
        }
      }
    }
    if (!__syncthreads_or(live())) break;
  }
  // segments before the next chunk's boundary (all, in the last chunk)
  while (live() && qn < nseg && a.seg_se[seg_index(seg0 + qn, tid)].x < Bn) {
    splice(qn);
    ++qn;
  }
  if ((tid & 63) == 0) {
    n_test += w_test;
    n_piece += w_piece;
  }
  count_work(a.counters, 0, n_test, n_piece);
  count_waves(a.counters, 8, w_iter, w_hit);
  // measured work (slab tests + 4 per piece, at least 1), the backward's
  // schedule key
  {
    uint32_t w = n_test + 4u * n_piece + (tid == 0 ? 1u : 0u);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) w += __shfl_xor(w, o, 64);
    if (tid == 0) blk_work = 0;
    __syncthreads();
    if ((tid & 63) == 0) atomicAdd(&blk_work, w);
    __syncthreads();
    if (tid == 0) a.item_work[item] = blk_work;
  }
  if (!valid) return;
  if (nck > 1) {
    float4* part = a.chunk_part + (((size_t)a.tile_pbase[gt] + chunk) * TPB + tid) * 4;
    part[0] = make_float4(C3.x, C3.y, C3.z, D);
    part[1] = make_float4(N3.x, N3.y, N3.z, T);
    part[2] = make_float4(CT.x, CT.y, CT.z, DT);
    part[3] = make_float4(NT.x, NT.y, NT.z, 0.0f);
    return;
  }
  a.fin0[pix] = make_float4(C3.x, C3.y, C3.z, D);
  a.fin1[pix] = make_float4(N3.x, N3.y, N3.z, T);
  a.fin2[pix] = make_float4(CT.x, CT.y, CT.z, DT);
  a.fin3[pix] = make_float4(NT.x, NT.y, NT.z, 0.0f);
  write_outputs(a, V, v, px, py, C3, D, N3, T, d);
}

// Seven blocks per CU (the LDS of seven batches fits the CU's 160 KB):
// the walk gains more from the waves than it loses to the spills that the
// 72-register limit causes (six and four blocks per CU measured slower).
template <bool NORMALS, int KC>
__global__ void __launch_bounds__(TPB, 7) k_composite_fwd(CompArgs a) {
  __shared__ Batch B;
  __shared__ uint32_t blk_work;
  if (blockIdx.x >= a.plan_counts[0]) return;
  composite_item<NORMALS, KC>(a, blockIdx.x, B, blk_work);
}

// Forward, part 4 (tiles of several chunks): merge the chunk partials in
// order, C = sum_c T_<c C_c, T = prod_c T_c, and write the outputs.
template <class A>
__device__ __forceinline__ void chunk_merge_tile(const A& a, uint32_t gt) {
  const uint32_t nck = a.tile_nck[gt];
  if (nck <= 1) return;
  const int tid = threadIdx.x;
  const PixSetup P = pixel_setup(a, gt, tid);
  if (!P.valid) return;
  const ViewConst& V = a.views[P.v];
  float3 C3 = make_float3(0, 0, 0), N3 = make_float3(0, 0, 0);
  float D = 0.0f, T = 1.0f;
  const float4* part = a.chunk_part + ((size_t)a.tile_pbase[gt] * TPB + tid) * 4;
  for (uint32_t c = 0; c < nck; ++c) {
    const float4 p0 = part[(size_t)c * TPB * 4], p1 = part[(size_t)c * TPB * 4 + 1];
    C3.x = fmaf(T, p0.x, C3.x); C3.y = fmaf(T, p0.y, C3.y);
    C3.z = fmaf(T, p0.z, C3.z); D = fmaf(T, p0.w, D);
    N3.x = fmaf(T, p1.x, N3.x); N3.y = fmaf(T, p1.y, N3.y);
    N3.z = fmaf(T, p1.z, N3.z);
    T *= p1.w;
  }
  a.fin0[P.pix] = make_float4(C3.x, C3.y, C3.z, D);
  a.fin1[P.pix] = make_float4(N3.x, N3.y, N3.z, T);
  a.fin2[P.pix] = make_float4(0, 0, 0, 0);
  a.fin3[P.pix] = make_float4(0, 0, 0, 0);
  write_outputs(a, V, P.v, P.px, P.py, C3, D, N3, T, P.d);
}

// One chunked tile per slot-table hit, the grid walking the slots.
__global__ void __launch_bounds__(TPB) k_chunk_merge(CompArgs a,
                                                     const uint32_t* slot_tile) {
  const uint32_t n_slots = a.plan_counts[1];
  for (uint32_t sl = blockIdx.x; sl < n_slots; sl += gridDim.x) {
    const uint32_t gt = chunked_tile_at(a, slot_tile, sl);
    if (gt != 0xFFFFFFFFu) chunk_merge_tile(a, gt);
  }
}

// ------------------------------------------------------------------ serving
__global__ void k_serve_publish(ServeQueue* q, unsigned long long g,
                                const uint32_t* plan_counts) {
  const uint32_t e = (uint32_t)(g % SV_RING);
  q->n_items[e] = plan_counts ? plan_counts[0] : 0u;
  __hip_atomic_store(&q->claim[e], g << 32, __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
  // the entry (and, earlier in stream order, the group's buffers and its
  // argument block) before the tail that makes it visible
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __hip_atomic_store(&q->tail, g + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Persistent drain.  Thread 0 of a block takes the next item of the oldest
// published group that has items left (compare-and-swap on the group's
// claim word, which carries the group number so an entry reused by a later
// group is never taken for an earlier one); the block walks it; after the
// last chunk of a tile the block that finished it merges the chunks, and
// the block that finishes a view's last tile raises the request's flag.
// A block with nothing to take sleeps and polls again; after idle_limit
// empty polls in a row it exits, so every block ends (the host launches
// the kernel again when new groups arrive).
// Group g's arguments sit in entry g % SV_RING of `groups` and are read
// through scalar loads, which one launch may keep cached.  A launch
// therefore serves only groups below g_hi, which the host sets at most
// SV_RING / 2 above the oldest unfinished group: within one launch no
// entry is read for two different groups, and a block that reaches g_hi
// exits so that a fresh launch (fresh caches) takes the later groups.
template <bool NORMALS, int KC>
__global__ void __launch_bounds__(TPB, 4)
k_serve_drain(ServeQueue* q, const ServeGroup* __restrict__ groups,
              int idle_limit, unsigned long long g_hi) {
  __shared__ Batch B;
  __shared__ uint32_t blk_work;
  __shared__ uint32_t s_cmd, s_slot, s_idx, s_last;
  int idle = 0;
  while (true) {
    if (threadIdx.x == 0) {
      uint32_t cmd = 0;
      for (int tries = 0; tries < 16 && cmd == 0; ++tries) {
        const unsigned long long h =
            __hip_atomic_load(&q->head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned long long t =
            __hip_atomic_load(&q->tail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (h >= t) break;
        if (h >= g_hi) {
          cmd = 2;
          break;
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        const uint32_t e = (uint32_t)(h % SV_RING);
        const unsigned long long w =
            __hip_atomic_load(&q->claim[e], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if ((w >> 32) != (h & 0xFFFFFFFFull)) {
          // h was drained and its entry reused: move on
          atomicCAS(&q->head, h, h + 1);
          continue;
        }
        const uint32_t n = __hip_atomic_load(&q->n_items[e], __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t c = (uint32_t)w;
        if (c >= n) {
          atomicCAS(&q->head, h, h + 1);
          continue;
        }
        if (atomicCAS(&q->claim[e], w, w + 1) == w) {
          s_slot = e;
          s_idx = c;
          cmd = 1;
        }
      }
      if (cmd == 0 && ++idle > idle_limit) cmd = 2;
      if (cmd == 1) idle = 0;
      s_cmd = cmd;
    }
    __syncthreads();
    const uint32_t cmd = s_cmd;
    if (cmd == 2) return;
    if (cmd == 0) {
      __builtin_amdgcn_s_sleep(127);
      __syncthreads();
      continue;
    }
    // the group's tables and records were written before it was published
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    // wave-uniform: the group's arguments come through scalar loads
    const uint32_t slot = __builtin_amdgcn_readfirstlane(s_slot);
    // through the constant address space: within this launch the entry holds
    // one group's arguments only (see g_hi), so their loads can be repeated
    // instead of kept
    typedef __attribute__((address_space(4))) const ServeGroup CGroup;
    CGroup& G = ((CGroup*)groups)[slot];
    const auto& a = G.a;
    const uint32_t idx = __builtin_amdgcn_readfirstlane(s_idx);
    composite_item<NORMALS, KC>(a, idx, B, blk_work);
    const uint32_t item = a.order[idx];
    const uint32_t gt = a.item_tile[item];
    const uint32_t nck = a.tile_nck[gt];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (threadIdx.x == 0) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      s_last = nck > 1 ? (atomicAdd(G.tile_ck + gt, 1u) == nck - 1) : 1u;
    }
    __syncthreads();
    if (s_last) {
      if (nck > 1) {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        chunk_merge_tile(a, gt);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __syncthreads();
      }
      if (threadIdx.x == 0) {
        // everything this block reads of the group is read before its count
        // goes in: once a view's last tile is counted, the host may free the
        // group's buffers
        const int v = view_of_tile(a.views, a.n_views, gt);
        const uint32_t ntv = G.view_ntiles[v];
        const uint32_t fslot = G.view_flag[v];
        const unsigned long long fval = G.view_seq[v];
        unsigned long long* const flags = G.flags;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        if (atomicAdd(G.view_done + v, 1u) == ntv - 1) {
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");  // system scope
          __hip_atomic_store(flags + fslot, fval, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_SYSTEM);
        }
      }
    }
    __syncthreads();
  }
}

dv_status launch_serve_publish(ServeQueue* q, uint64_t g,
                               const uint32_t* plan_counts, hipStream_t s) {
  hipLaunchKernelGGL(k_serve_publish, dim3(1), dim3(1), 0, s, q,
                     (unsigned long long)g, plan_counts);
  DV_TRY_HIP(hipGetLastError());
  return DV_OK;
}

dv_status launch_serve_drain(ServeQueue* q, const ServeGroup* groups,
                             bool normals, bool k1, int blocks, int idle_limit,
                             uint64_t g_hi, hipStream_t s) {
  auto kern = normals ? (k1 ? k_serve_drain<true, 1> : k_serve_drain<true, 0>)
                      : (k1 ? k_serve_drain<false, 1> : k_serve_drain<false, 0>);
  hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(TPB), 0, s, q, groups,
                     idle_limit, (unsigned long long)g_hi);
  DV_TRY_HIP(hipGetLastError());
  return DV_OK;
}

// ------------------------------------------------------------------ host
static void mat_t_mul(const double Rc[9], const double Rk[9], double A[9]) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      A[i * 3 + j] = (Rc[0 * 3 + i] * Rk[0 * 3 + j] + Rc[1 * 3 + i] * Rk[1 * 3 + j]) +
                     Rc[2 * 3 + i] * Rk[2 * 3 + j];
}

static dv_status check_view(const dv_view& v) {
  if (!(v.fx > 0) || !(v.fy > 0) || !std::isfinite(v.cx) ||
      !std::isfinite(v.cy) || v.W <= 0 || v.H <= 0 || v.w <= 0 || v.h <= 0 ||
      v.x0 < 0 || v.y0 < 0 || v.x0 + v.w > v.W || v.y0 + v.h > v.H ||
      !std::isfinite(v.t)) {
    set_error("invalid view (intrinsics, size or window)");
    return DV_ERR_INVALID;
  }
  if (v.w > 16 * 65535 || v.h > 16 * 65535) {
    set_error("view window too large");
    return DV_ERR_LIMIT;
  }
  for (int i = 0; i < 12; ++i)
    if (!std::isfinite(v.c2w[i])) {
      set_error("view c2w not finite");
      return DV_ERR_INVALID;
    }
  return DV_OK;
}

}  // namespace dv

using namespace dv;

namespace dv {

// Host setup shared by dv_render and the serving loop: poses, per-view and
// per-(view, octree) constants, the preprocess segment table and the
// actor-tile lists.
dv_status setup_state(dv_fwd_state* st, const dv_scene* sc,
                      const dv_view* views, int32_t n_views,
                      const double* pose_override) {
  std::vector<int64_t>& seg_start = st->seg_start_h;
  std::vector<uint32_t>& act_tile = st->act_tile_h;
  const int n_oct = sc->n_oct;
  st->n_views = n_views;
  st->n_oct = n_oct;
  st->n_actors = n_oct - 1;
  st->views_h.resize(n_views);
  st->vo_h.resize((size_t)n_views * n_oct);
  st->views_in.assign(views, views + n_views);
  uint32_t tile_base = 0;
  for (int v = 0; v < n_views; ++v) {
    const dv_view& in = views[v];
    DV_TRY(check_view(in));
    ViewConst& V = st->views_h[v];
    std::memset(&V, 0, sizeof(V));
    V.fx = in.fx; V.fy = in.fy; V.cx = in.cx; V.cy = in.cy;
    V.inv_fx = (float)(1.0 / in.fx);
    V.inv_fy = (float)(1.0 / in.fy);
    V.fcx = (float)in.cx;
    V.fcy = (float)in.cy;
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) V.Rc[r * 3 + c] = (float)in.c2w[r * 4 + c];
    V.x0 = in.x0; V.y0 = in.y0; V.w = in.w; V.h = in.h;
    {
      // r_near^2 = (2e)^2 max over window corner pixel centres |(x, y, 1)|^2
      double m2 = 0.0;
      const int pxs[2] = {in.x0, in.x0 + in.w - 1};
      const int pys[2] = {in.y0, in.y0 + in.h - 1};
      for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
          const double x = (pxs[i] + 0.5 - in.cx) / in.fx;
          const double y = (pys[j] + 0.5 - in.cy) / in.fy;
          m2 = std::max(m2, (1.0 + x * x) + y * y);
        }
      V.rnear2 = (2.0 * Z_EPS_D) * (2.0 * Z_EPS_D) * m2;
      // for the conservative ball test: sqrt(rnear2) and |n| of the four
      // window side planes, each rounded up by a relative 1e-6
      V.rnear_m = std::sqrt(V.rnear2) * (1.0 + 1e-6) + 1e-9;
      const double l = in.cx - (in.x0 - 2.0), rr = (in.x0 + in.w + 2.0) - in.cx;
      const double t = in.cy - (in.y0 - 2.0), bb = (in.y0 + in.h + 2.0) - in.cy;
      V.side_norm[0] = std::sqrt(in.fx * in.fx + l * l) * (1.0 + 1e-6);
      V.side_norm[1] = std::sqrt(in.fx * in.fx + rr * rr) * (1.0 + 1e-6);
      V.side_norm[2] = std::sqrt(in.fy * in.fy + t * t) * (1.0 + 1e-6);
      V.side_norm[3] = std::sqrt(in.fy * in.fy + bb * bb) * (1.0 + 1e-6);
    }
    V.ntx = (in.w + TILE - 1) / TILE;
    V.nty = (in.h + TILE - 1) / TILE;
    V.tile_base = tile_base;
    const uint64_t nt = (uint64_t)V.ntx * V.nty;
    if ((uint64_t)tile_base + nt >= (1ull << 31)) {
      set_error("too many tiles");
      return DV_ERR_LIMIT;
    }
    tile_base += (uint32_t)nt;
  }
  st->n_tiles = tile_base;
  // poses and per-(view, octree) constants
  seg_start.assign((size_t)n_views * n_oct + 1, 0);
  std::vector<std::vector<uint32_t>> tile_lists;  // built below
  std::vector<std::pair<uint32_t, uint32_t>> apairs;  // (tile, octree)
  int64_t items = 0;
  for (int v = 0; v < n_views; ++v) {
    const dv_view& in = views[v];
    double Rc[9], o[3];
    for (int r = 0; r < 3; ++r) {
      for (int c = 0; c < 3; ++c) Rc[r * 3 + c] = in.c2w[r * 4 + c];
      o[r] = in.c2w[r * 4 + 3];
    }
    for (int k = 0; k < n_oct; ++k) {
      double R[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1}, p[3] = {0, 0, 0};
      int active = 1;
      if (k > 0) {
        if (pose_override) {
          const double* po = pose_override + ((size_t)v * (n_oct - 1) + (k - 1)) * 12;
          for (int i = 0; i < 9; ++i) R[i] = po[i];
          for (int i = 0; i < 3; ++i) p[i] = po[9 + i];
          for (int i = 0; i < 12; ++i)
            if (!std::isfinite(po[i])) {
              set_error("pose_override not finite (view %d actor %d)", v, k);
              return DV_ERR_INVALID;
            }
        } else {
          dv_track_desc tr;
          tr.n_keys = (int32_t)sc->trk_t[k].size();
          tr.t = sc->trk_t[k].data();
          tr.yaw = sc->trk_yaw[k].data();
          tr.trans = sc->trk_trans[k].data();
          active = dv_track_pose(&tr, in.t, R, p);
        }
      }
      VOConst& C = st->vo_h[(size_t)v * n_oct + k];
      std::memset(&C, 0, sizeof(C));
      C.active = active;
      if (st->opts.feat) {
        const int c0 = 3 * st->opts.feat_group;
        C.feat_nc = std::min(3, st->opts.feat_dim - c0);
        C.feat = st->opts.feat[k] + (size_t)c0 * sc->desc[k].n_voxels;
      }
      C.octree = k;
      C.view = v;
      mat_t_mul(Rc, R, C.A);
      const double q[3] = {p[0] - o[0], p[1] - o[1], p[2] - o[2]};
      for (int i = 0; i < 3; ++i)
        C.b[i] = (Rc[0 * 3 + i] * q[0] + Rc[1 * 3 + i] * q[1]) + Rc[2 * 3 + i] * q[2];
      const double om[3] = {o[0] - p[0], o[1] - p[1], o[2] - p[2]};
      double P[3];
      for (int j = 0; j < 3; ++j)
        P[j] = (R[0 * 3 + j] * om[0] + R[1 * 3 + j] * om[1]) + R[2 * 3 + j] * om[2];
      const dv_octree_desc& od = sc->desc[k];
      for (int a = 0; a < 3; ++a) {
        double qq = (P[a] - od.root_min[a]) / od.root_size;
        qq = std::min(std::max(qq, -1.0), 2.0);
        C.Q[a] = (int64_t)std::floor(std::ldexp(qq, QBITS));
        C.rootrel[a] = od.root_min[a] - P[a];
        C.omp[a] = (float)om[a];
      }
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
          C.Rt[i * 3 + j] = (float)R[j * 3 + i];
          C.R[i * 3 + j] = (float)R[i * 3 + j];
        }
      double blo[3], bhi[3];
      for (int a = 0; a < 3; ++a) {
        blo[a] = (k > 0 && od.has_box) ? od.box_min[a] : od.root_min[a];
        bhi[a] = (k > 0 && od.has_box) ? od.box_max[a] : od.root_min[a] + od.root_size;
        C.boxlo[a] = (float)(blo[a] - P[a]);
        C.boxhi[a] = (float)(bhi[a] - P[a]);
      }
      const size_t sidx = (size_t)v * n_oct + k;
      int64_t cnt = active ? sc->desc[k].n_voxels : 0;
      if (cnt > 0) {
        // no leaf of an octree whose root cube is culled can be binned
        const ViewConst& V = st->views_h[v];
        double ctr[3];
        for (int a = 0; a < 3; ++a) ctr[a] = od.root_min[a] + 0.5 * od.root_size;
        if (ball_culled(C.A, C.b, ctr, 0.8660254037844386 * od.root_size, V))
          cnt = 0;
      }
      seg_start[sidx + 1] = seg_start[sidx] + cnt;
      items += cnt;
      if (k > 0 && active) {
        const ViewConst& V = st->views_h[v];
        Rect r = bin_box(C.A, C.b, blo, bhi, V.fx, V.fy, V.cx, V.cy, V.x0,
                         V.y0, V.w, V.h, V.rnear2);
        if (r.status != 0 && r.xl <= r.xh && r.yl <= r.yh) {
          for (int ty = r.yl >> 4; ty <= (r.yh >> 4); ++ty)
            for (int tx = r.xl >> 4; tx <= (r.xh >> 4); ++tx)
              apairs.emplace_back(V.tile_base + ty * V.ntx + tx, k);
        }
      }
    }
  }
  (void)items;
  // actor-tile CSR (stable by tile, actors ascending within a tile)
  st->act_beg_h.assign(st->n_tiles + 1, 0);
  for (auto& pr : apairs) st->act_beg_h[pr.first + 1]++;
  for (int64_t t = 0; t < st->n_tiles; ++t) {
    if (st->act_beg_h[t + 1] > DV_MAX_TILE_ACTORS) {
      set_error("tile %lld has %u actor boxes (limit %d)", (long long)t,
                st->act_beg_h[t + 1], DV_MAX_TILE_ACTORS);
      return DV_ERR_LIMIT;
    }
    st->act_beg_h[t + 1] += st->act_beg_h[t];
  }
  st->n_apairs = (int64_t)apairs.size();
  st->act_oct_h.assign(apairs.size(), 0);
  act_tile.assign(apairs.size(), 0);
  {
    std::vector<uint32_t> fillp(st->act_beg_h.begin(), st->act_beg_h.end() - 1);
    std::stable_sort(apairs.begin(), apairs.end(),
                     [](const std::pair<uint32_t, uint32_t>& x,
                        const std::pair<uint32_t, uint32_t>& y) {
                       return x.first < y.first ||
                              (x.first == y.first && x.second < y.second);
                     });
    for (size_t e = 0; e < apairs.size(); ++e) {
      st->act_oct_h[e] = apairs[e].second;
      act_tile[e] = apairs[e].first;
    }
  }
  return DV_OK;
}

// One pinned host word per calling thread for device->host counts, so
// concurrent renders on different streams never wait for each other.
static uint64_t* pinned_words(size_t n) {
  if (Arena* ar = thread_arena()) {
    if (n * sizeof(uint64_t) > ar->pinned_cap / 2) {
      set_error("%zu count words exceed the static staging", n);
      return nullptr;
    }
    return reinterpret_cast<uint64_t*>(ar->pinned + ar->pinned_cap / 2);
  }
  static thread_local uint64_t* w = nullptr;
  static thread_local size_t cap = 0;
  if (n > cap) {
    if (w) (void)hipHostFree(w);
    w = nullptr;
    cap = 0;
    const size_t want = std::max<size_t>(n, 8);
    if (hipHostMalloc((void**)&w, want * sizeof(uint64_t), hipHostMallocDefault) !=
        hipSuccess) {
      (void)hipGetLastError();
      set_error("pinned host allocation failed");
      w = nullptr;
      return nullptr;
    }
    cap = want;
  }
  return w;
}

// Pinned staging for the per-call host tables (one per host thread).  An
// event after each upload guards reuse: the next call waits for it (a call
// normally synchronises its stream long before).
struct HostStage {
  uint8_t* p = nullptr;
  size_t cap = 0;
  hipEvent_t ev = nullptr;
  bool pending = false;
};
static HostStage& host_stage() {
  static thread_local HostStage h;
  return h;
}
uint8_t* stage_acquire(size_t bytes) {
  if (Arena* ar = thread_arena()) {
    // the call synchronises its stream after this upload, before it
    // returns, so the next call may reuse the block
    if (bytes > ar->pinned_cap / 2) {
      set_error("%zu bytes of host tables exceed the static staging", bytes);
      return nullptr;
    }
    return ar->pinned;
  }
  HostStage& h = host_stage();
  if (h.pending) {
    (void)hipEventSynchronize(h.ev);
    h.pending = false;
  }
  if (!h.ev && hipEventCreateWithFlags(&h.ev, hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    set_error("event creation failed");
    h.ev = nullptr;
    return nullptr;
  }
  if (bytes > h.cap) {
    if (h.p) (void)hipHostFree(h.p);
    h.p = nullptr;
    h.cap = 0;
    const size_t want = std::max<size_t>(bytes + bytes / 2, 1 << 16);
    if (hipHostMalloc((void**)&h.p, want, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      set_error("pinned host allocation failed");
      h.p = nullptr;
      return nullptr;
    }
    h.cap = want;
  }
  return h.p;
}
dv_status stage_release(hipStream_t s) {
  if (thread_arena()) return DV_OK;
  HostStage& h = host_stage();
  DV_TRY_HIP(hipEventRecord(h.ev, s));
  h.pending = true;
  return DV_OK;
}

// First record slot of every view (records are in slot order: view,
// octree, leaf), the record total at index n_views and the pair total (the
// sum of the preprocess's partial pair counters) at index n_views + 1.  A
// view's first item starts a wave, so its slot is the block offset plus
// the ballots of the block's earlier waves.
__global__ void k_view_slots(int n_views, int n_oct, const int64_t* pstart,
                             int64_t n_items, const uint32_t* block_off,
                             const uint64_t* wave_mask, const uint64_t* total,
                             const unsigned long long* pair_parts, uint64_t* out) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v > n_views) return;
  if (v == n_views) {
    uint64_t np = 0;
    for (int i = 0; i < PAIR_PARTS; ++i) np += pair_parts[i * PAIR_STRIDE];
    out[n_views + 1] = np;
  }
  const int64_t it = v < n_views ? pstart[(size_t)v * n_oct] : n_items;
  if (it >= n_items) { out[v] = total[0]; return; }
  const int64_t b = it / TPB;
  const int w = (int)((it / 64) % (TPB / 64));
  uint64_t sl = block_off[b];
  for (int i = 0; i < w; ++i) sl += (uint64_t)__popcll(wave_mask[b * (TPB / 64) + i]);
  out[v] = sl;
}

// Enqueue the whole forward pass on stream s.  One host synchronisation
// reads the record count (per view) and the pair count, both known after
// the first preprocess pass.
dv_status run_forward(dv_ctx* ctx, const dv_scene* sc, dv_fwd_state* st,
                      const dv_outputs* outs, hipStream_t s, bool composite) {
  const std::vector<int64_t>& seg_start = st->seg_start_h;
  const std::vector<uint32_t>& act_tile = st->act_tile_h;
  const int n_views = st->n_views, n_oct = st->n_oct;
  const dv_render_opts& op = st->opts;
  const int n_seg = n_views * n_oct;
  // item space: each segment padded to a multiple of 64 leaves
  std::vector<int64_t>& pstart = st->seg_pstart_h;
  std::vector<int32_t>& seg_len = st->seg_len_h;
  pstart.assign((size_t)n_seg + 1, 0);
  seg_len.assign((size_t)n_seg, 0);
  for (int i = 0; i < n_seg; ++i) {
    seg_len[i] = (int32_t)(seg_start[i + 1] - seg_start[i]);
    pstart[i + 1] = pstart[i] + ((seg_len[i] + 63) & ~(int64_t)63);
  }
  const int64_t n_items = pstart.back();
  // host-side tables, uploaded in one copy from pinned staging: views,
  // (view, octree) constants, output planes, padded segment starts and
  // lengths, the actor-tile CSR
  const int64_t nt = st->n_tiles, na = st->n_apairs;
  DBuf& segs_d = st->seg_pstart_d;
  DBuf& slen_d = st->seg_len_d;
  {
    const void* src[8] = {st->views_h.data(), st->vo_h.data(), outs,
                          pstart.data(), seg_len.data(), st->act_beg_h.data(),
                          st->act_oct_h.data(), act_tile.data()};
    const size_t len[8] = {sizeof(ViewConst) * n_views, sizeof(VOConst) * n_seg,
                           sizeof(dv_outputs) * n_views,
                           sizeof(int64_t) * pstart.size(), sizeof(int32_t) * n_seg,
                           4 * (size_t)(nt + 1), 4 * (size_t)na, 4 * (size_t)na};
    DBuf* dst[8] = {&st->views_d, &st->vo_d, &st->outs_d, &segs_d, &slen_d,
                    &st->act_beg, &st->act_oct, &st->act_tile};
    size_t off[8], total = 0;
    for (int i = 0; i < 8; ++i) {
      off[i] = total;
      total += (len[i] + 255) & ~(size_t)255;
    }
    DV_TRY(alloc_n<uint8_t>(ctx, st->host_tables, total, s));
    uint8_t* stage = stage_acquire(total);
    if (!stage) return DV_ERR_OOM;
    for (int i = 0; i < 8; ++i)
      if (len[i]) std::memcpy(stage + off[i], src[i], len[i]);
    DV_TRY_HIP(hipMemcpyAsync(st->host_tables.p, stage, total,
                              hipMemcpyHostToDevice, s));
    DV_TRY(stage_release(s));
    for (int i = 0; i < 8; ++i)
      dst[i]->view_of(st->host_tables.as<uint8_t>() + off[i], len[i]);
  }
  // key layout
  int seg_bits = ceil_log2((uint64_t)n_seg);
  st->rank_bits = 3 * sc->max_level_all;
  st->key_bits = st->rank_bits + seg_bits;
  if (st->key_bits > 64) {
    set_error("record key needs %d bits", st->key_bits);
    return DV_ERR_LIMIT;
  }
  st->tile_bits = ceil_log2((uint64_t)std::max<int64_t>(st->n_tiles, 2));
  // pass 0: visibility counts per block
  const unsigned nblk = grid_for(std::max<int64_t>(n_items, 1), TPB);
  DBuf bcount, total, vslot;
  DBuf& wmask = st->pre_wmask;
  DBuf& boff = st->pre_boff;
  DV_TRY(alloc_n<uint64_t>(ctx, wmask, (size_t)nblk * (TPB / 64), s));
  DV_TRY(alloc_n<uint32_t>(ctx, bcount, nblk, s));
  DV_TRY(alloc_n<uint32_t>(ctx, boff, nblk, s));
  DV_TRY(alloc_n<uint64_t>(ctx, total, 2, s));
  // first record slot per view, the record total, then the pair total
  DV_TRY(alloc_n<uint64_t>(ctx, vslot, (size_t)n_views + 2, s));
  DBuf pparts;
  DV_TRY(alloc_n<uint64_t>(ctx, pparts, (size_t)PAIR_PARTS * PAIR_STRIDE, s));
  DV_TRY(fill_u32(pparts.as<uint32_t>(), 0u, 2 * PAIR_PARTS * PAIR_STRIDE, s));
  PreArgs pa;
  std::memset(&pa, 0, sizeof(pa));
  pa.views = st->views_d.as<ViewConst>();
  pa.vo = st->vo_d.as<VOConst>();
  pa.oct = sc->oct_dev.as<OctDev>();
  pa.seg_start = segs_d.as<int64_t>();
  DBuf& wseg = st->pre_wseg;
  DV_TRY(alloc_n<uint32_t>(ctx, wseg, (size_t)std::max<int64_t>(n_items / 64, 1), s));
  if (n_items > 0) {
    hipLaunchKernelGGL(k_wave_segments, dim3((unsigned)n_seg), dim3(TPB), 0, s,
                       segs_d.as<int64_t>(), wseg.as<uint32_t>());
    DV_TRY_HIP(hipGetLastError());
  }
  pa.wave_seg = wseg.as<uint32_t>();
  pa.seg_len = slen_d.as<int32_t>();
  pa.wave_mask = wmask.as<uint64_t>();
  pa.n_seg = n_seg;
  pa.n_oct = n_oct;
  pa.n_items = n_items;
  pa.rank_bits = st->rank_bits;
  pa.block_count = bcount.as<uint32_t>();
  pa.pair_parts = reinterpret_cast<unsigned long long*>(pparts.as<uint64_t>());
  pa.block_off = boff.as<uint32_t>();
  {
    StageTimer tm(ctx, ST_PREPROCESS, s);
    if (n_items > 0)
      hipLaunchKernelGGL(k_preprocess<0>, dim3(nblk), dim3(TPB), 0, s, pa);
    else
      DV_TRY(fill_u32(bcount.as<uint32_t>(), 0, nblk, s));
    DV_TRY_HIP(hipGetLastError());
    DV_TRY(exclusive_scan_u32(ctx, bcount.as<uint32_t>(), boff.as<uint32_t>(),
                              total.as<uint64_t>(), nblk, s));
    hipLaunchKernelGGL(k_view_slots, dim3(grid_for(n_views + 1, TPB)), dim3(TPB),
                       0, s, n_views, n_oct, segs_d.as<int64_t>(), n_items,
                       boff.as<uint32_t>(), wmask.as<uint64_t>(),
                       total.as<uint64_t>(),
                       reinterpret_cast<const unsigned long long*>(pparts.as<uint64_t>()),
                       vslot.as<uint64_t>());
    DV_TRY_HIP(hipGetLastError());
  }
  uint64_t n_vis = 0, n_pairs = 0;
  {
    uint64_t* pin = pinned_words((size_t)n_views + 2);
    if (!pin) return DV_ERR_OOM;
    StageTimer tm(ctx, ST_HOST_SYNC, s);
    DV_TRY_HIP(hipMemcpyAsync(pin, vslot.p, sizeof(uint64_t) * (n_views + 2),
                              hipMemcpyDeviceToHost, s));
    DV_TRY_HIP(hipStreamSynchronize(s));
    n_vis = pin[n_views];
    n_pairs = pin[n_views + 1];
    st->view_slot_h.assign(pin, pin + n_views + 1);
  }
  st->n_vis = (int64_t)n_vis;
  if (n_vis >= 0xFFFFFFFFull) {
    set_error("%llu visible records exceed the 32-bit range",
              (unsigned long long)n_vis);
    return DV_ERR_LIMIT;
  }
  const int64_t nv = (int64_t)n_vis;
  // pass 1: records in slot order
  // the record arrays of the state, in slot order
  DBuf keys, vals, keys2, vals2;
  DV_TRY(alloc_n<uint64_t>(ctx, keys, nv, s));
  DV_TRY(alloc_n<uint32_t>(ctx, vals, nv, s));
  DV_TRY(alloc_n<uint64_t>(ctx, keys2, nv, s));
  DV_TRY(alloc_n<uint32_t>(ctx, vals2, nv, s));
  DV_TRY(alloc_n<float4>(ctx, st->rec_geo, nv, s));
  DV_TRY(alloc_n<float4>(ctx, st->rec_g8a, nv, s));
  DV_TRY(alloc_n<float4>(ctx, st->rec_g8b, nv, s));
  DV_TRY(alloc_n<float4>(ctx, st->rec_cn, nv, s));
  DV_TRY(alloc_n<float4>(ctx, st->rec_nrm, nv, s));
  DV_TRY(alloc_n<uint32_t>(ctx, st->rec_vox, nv, s));
  DV_TRY(alloc_n<uint64_t>(ctx, st->rec_rect, nv, s));
  DV_TRY(alloc_n<uint32_t>(ctx, st->rec_seg, nv, s));
  pa.keys = keys.as<uint64_t>();
  pa.vals = vals.as<uint32_t>();
  pa.s_geo = st->rec_geo.as<float4>();
  pa.s_g8a = st->rec_g8a.as<float4>();
  pa.s_g8b = st->rec_g8b.as<float4>();
  pa.s_cn = st->rec_cn.as<float4>();
  pa.s_nrm = st->rec_nrm.as<float4>();
  pa.s_vox = st->rec_vox.as<uint32_t>();
  pa.s_seg = st->rec_seg.as<uint32_t>();
  pa.s_rect = st->rec_rect.as<uint64_t>();
  {
    StageTimer tm(ctx, ST_PREPROCESS, s);
    if (n_items > 0 && nv > 0)
      hipLaunchKernelGGL(k_preprocess<1>, dim3(nblk), dim3(TPB), 0, s, pa);
    DV_TRY_HIP(hipGetLastError());
  }
  // sort records by (view, octree, rank)
  bool alt = false;
  {
    StageTimer tm(ctx, ST_SORT_RECORDS, s);
    DV_TRY(radix_sort_u64(ctx, keys.as<uint64_t>(), vals.as<uint32_t>(),
                          keys2.as<uint64_t>(), vals2.as<uint32_t>(), nv,
                          st->key_bits, s, &alt));
  }
  uint32_t* vs = alt ? vals2.as<uint32_t>() : vals.as<uint32_t>();
  // per sorted record: tile count and offset
  DBuf r_count, r_off;
  DV_TRY(alloc_n<uint32_t>(ctx, r_count, nv, s));
  DV_TRY(alloc_n<uint32_t>(ctx, r_off, nv, s));
  StageTimer tm_gather(ctx, ST_GATHER, s);
  if (nv > 0)
    hipLaunchKernelGGL(k_gather, dim3(grid_for(nv, TPB)), dim3(TPB), 0, s, nv,
                       vs, st->rec_rect.as<uint64_t>(), r_count.as<uint32_t>());
  DV_TRY_HIP(hipGetLastError());
  DV_TRY(exclusive_scan_u32(ctx, r_count.as<uint32_t>(), r_off.as<uint32_t>(),
                            total.as<uint64_t>(), nv, s));
  tm_gather.stop();
  if (n_pairs >= 0xFFFFFFFFull) {
    set_error("%llu (leaf, tile) pairs exceed the 32-bit range",
              (unsigned long long)n_pairs);
    return DV_ERR_LIMIT;
  }
  st->n_pairs = (int64_t)n_pairs;
  const int64_t np = (int64_t)n_pairs;
  keys.reset();
  keys2.reset();
  DBuf pkey, pkey2, pval2;
  DV_TRY(alloc_n<uint32_t>(ctx, pkey, np, s));
  DV_TRY(alloc_n<uint32_t>(ctx, st->pair_val, np, s));
  DV_TRY(alloc_n<uint32_t>(ctx, pkey2, np, s));
  DV_TRY(alloc_n<uint32_t>(ctx, pval2, np, s));
  StageTimer tm_emit(ctx, ST_EMIT, s);
  if (np > 0) {
    const unsigned eb = grid_for(np, TPB);
    DBuf brec;
    DV_TRY(alloc_n<uint32_t>(ctx, brec, eb, s));
    hipLaunchKernelGGL(k_pair_block_rec, dim3(grid_for(nv, TPB)), dim3(TPB), 0, s,
                       nv, np, r_off.as<uint32_t>(), brec.as<uint32_t>());
    hipLaunchKernelGGL(k_emit, dim3(eb), dim3(TPB), 0, s, np, nv,
                       r_off.as<uint32_t>(), brec.as<uint32_t>(), vs,
                       st->rec_rect.as<uint64_t>(), st->rec_seg.as<uint32_t>(),
                       n_oct, st->views_d.as<ViewConst>(), pkey.as<uint32_t>(),
                       st->pair_val.as<uint32_t>());
  }
  DV_TRY_HIP(hipGetLastError());
  tm_emit.stop();
  {
    StageTimer tm(ctx, ST_SORT_PAIRS, s);
    DV_TRY(radix_sort_u32(ctx, pkey.as<uint32_t>(), st->pair_val.as<uint32_t>(),
                          pkey2.as<uint32_t>(), pval2.as<uint32_t>(), np,
                          st->tile_bits, s, &alt));
  }
  if (alt) {
    std::swap(pkey, pkey2);
    std::swap(st->pair_val, pval2);
  }
  pkey2.reset();
  pval2.reset();
  // tile directory
  StageTimer tm_dir(ctx, ST_TILE_DIR, s);
  DV_TRY(alloc_n<uint32_t>(ctx, st->tile_start, nt, s));
  DV_TRY(alloc_n<uint32_t>(ctx, st->tile_end, nt, s));
  DV_TRY(alloc_n<uint32_t>(ctx, st->tile_bgend, nt, s));
  DV_TRY(fill_u32(st->tile_start.as<uint32_t>(), 0, nt, s));
  DV_TRY(fill_u32(st->tile_end.as<uint32_t>(), 0, nt, s));
  if (np > 0)
    hipLaunchKernelGGL(k_tile_bounds, dim3(grid_for(np, TPB)), dim3(TPB), 0, s,
                       np, pkey.as<uint32_t>(), st->tile_start.as<uint32_t>(),
                       st->tile_end.as<uint32_t>());
  hipLaunchKernelGGL(k_tile_dir, dim3(grid_for(nt, TPB)), dim3(TPB), 0, s, nt,
                     st->tile_start.as<uint32_t>(), st->tile_end.as<uint32_t>(),
                     st->pair_val.as<uint32_t>(), st->rec_seg.as<uint32_t>(),
                     n_oct, st->tile_bgend.as<uint32_t>());
  DV_TRY_HIP(hipGetLastError());
  // actor lists
  DBuf& atile = st->act_tile;
  DV_TRY(alloc_n<uint2>(ctx, st->act_sub, na, s));
  if (na > 0) {
    hipLaunchKernelGGL(k_actor_ranges, dim3(grid_for(na, TPB)), dim3(TPB), 0, s,
                       na, atile.as<uint32_t>(), st->act_oct.as<uint32_t>(),
                       st->tile_bgend.as<uint32_t>(), st->tile_end.as<uint32_t>(),
                       st->pair_val.as<uint32_t>(), st->rec_seg.as<uint32_t>(),
                       n_oct, st->act_sub.as<uint2>());
    DV_TRY_HIP(hipGetLastError());
  }
  // work items: tiles, long background lists split into chunks
  st->max_items = nt + st->n_pairs / CHUNK + 1;
  st->max_slots = 2 * (st->n_pairs / CHUNK) + 1;
  DV_TRY(alloc_n<uint32_t>(ctx, st->order_fwd, st->max_items, s));
  DV_TRY(alloc_n<uint32_t>(ctx, st->item_tile, st->max_items, s));
  DV_TRY(alloc_n<uint32_t>(ctx, st->item_chunk, st->max_items, s));
  DV_TRY(alloc_n<uint32_t>(ctx, st->item_work, st->max_items, s));
  DV_TRY(alloc_n<uint32_t>(ctx, st->tile_nck, nt, s));
  DV_TRY(alloc_n<uint32_t>(ctx, st->tile_ibase, nt, s));
  DV_TRY(alloc_n<uint32_t>(ctx, st->tile_pbase, nt, s));
  DV_TRY(alloc_n<uint32_t>(ctx, st->slot_tile, st->max_slots, s));
  DV_TRY(fill_u32(st->slot_tile.as<uint32_t>(), 0xFFFFFFFFu, st->max_slots, s));
  DV_TRY(alloc_n<uint32_t>(ctx, st->plan_counts, 2, s));
  DV_TRY(alloc_n<float>(ctx, st->chunk_b, st->max_slots * CB_SPLIT * TPB, s));
  DV_TRY(alloc_n<float4>(ctx, st->chunk_part, st->max_slots * TPB * 4, s));
  DV_TRY(fill_u32(st->item_work.as<uint32_t>(), 0u, st->max_items, s));
  // actor work items: (tile, actor) lists, long ones split into chunks
  PlanArgs plans[2];
  int n_plans = 0;
  if (na > 0) {
    st->max_aitems = na + st->n_pairs / ACHUNK + 1;
    st->max_aslots = std::min<int64_t>(2 * (st->n_pairs / ACHUNK) + 1,
                                       ((int64_t)1 << 30) / (TPB * 64));
    DV_TRY(alloc_n<uint32_t>(ctx, st->aorder, st->max_aitems, s));
    DV_TRY(alloc_n<uint32_t>(ctx, st->aitem_pair, st->max_aitems, s));
    DV_TRY(alloc_n<uint32_t>(ctx, st->aitem_chunk, st->max_aitems, s));
    DV_TRY(alloc_n<uint32_t>(ctx, st->pair_nck, na, s));
    DV_TRY(alloc_n<uint32_t>(ctx, st->pair_ibase, na, s));
    DV_TRY(alloc_n<uint32_t>(ctx, st->pair_pbase, na, s));
    DV_TRY(alloc_n<uint32_t>(ctx, st->aplan_counts, 2, s));
    DV_TRY(alloc_n<float4>(ctx, st->apart, st->max_aslots * TPB * 4, s));
    plans[n_plans++] = PlanArgs{na, nullptr, nullptr, st->act_sub.as<uint2>(), ACHUNK,
                                (uint32_t)st->max_aslots, st->pair_nck.as<uint32_t>(),
                                st->pair_ibase.as<uint32_t>(),
                                st->pair_pbase.as<uint32_t>(),
                                st->aitem_pair.as<uint32_t>(),
                                st->aitem_chunk.as<uint32_t>(),
                                st->aorder.as<uint32_t>(),
                                st->aplan_counts.as<uint32_t>(), nullptr,
                                st->max_aitems};
  }
  if (nt > 0)
    plans[n_plans++] = PlanArgs{nt, st->tile_start.as<uint32_t>(),
                                st->tile_bgend.as<uint32_t>(), nullptr, CHUNK,
                                (uint32_t)st->max_slots, st->tile_nck.as<uint32_t>(),
                                st->tile_ibase.as<uint32_t>(),
                                st->tile_pbase.as<uint32_t>(),
                                st->item_tile.as<uint32_t>(),
                                st->item_chunk.as<uint32_t>(),
                                st->order_fwd.as<uint32_t>(),
                                st->plan_counts.as<uint32_t>(),
                                st->slot_tile.as<uint32_t>(), st->max_items};
  {
    // small sets in one launch (a block each), large ones device-wide
    PlanArgs small[2];
    int n_small = 0;
    for (int i = 0; i < n_plans; ++i) {
      if (plans[i].n_tiles <= PLAN_ONE_BLOCK) small[n_small++] = plans[i];
      else DV_TRY(plan_items(ctx, plans[i], s));
    }
    if (n_small > 0) {
      hipLaunchKernelGGL(k_plan_items, dim3(n_small), dim3(1024), 0, s, small[0],
                         small[n_small - 1]);
      DV_TRY_HIP(hipGetLastError());
    }
  }
  tm_dir.stop();
  // per-pixel scratch
  const size_t nslots = (size_t)3 * na * TPB;
  DV_TRY(alloc_n<float2>(ctx, st->seg_se, nslots, s));
  DV_TRY(alloc_n<uint32_t>(ctx, st->seg_meta, nslots, s));
  DV_TRY(alloc_n<float4>(ctx, st->seg_p0, nslots, s));
  DV_TRY(alloc_n<float4>(ctx, st->seg_p1, nslots, s));
  DV_TRY(alloc_n<float4>(ctx, st->seg_t0, nslots, s));
  DV_TRY(alloc_n<float4>(ctx, st->seg_t1, nslots, s));
  DV_TRY(alloc_n<uint32_t>(ctx, st->pix_nseg, (size_t)nt * TPB, s));
  DV_TRY(alloc_n<float4>(ctx, st->fin0, (size_t)nt * TPB, s));
  DV_TRY(alloc_n<float4>(ctx, st->fin1, (size_t)nt * TPB, s));
  DV_TRY(alloc_n<float4>(ctx, st->fin2, (size_t)nt * TPB, s));
  DV_TRY(alloc_n<float4>(ctx, st->fin3, (size_t)nt * TPB, s));
  CompArgs ca;
  std::memset(&ca, 0, sizeof(ca));
  ca.views = st->views_d.as<ViewConst>();
  ca.vo = st->vo_d.as<VOConst>();
  ca.n_views = n_views;
  ca.n_oct = n_oct;
  ca.tile_start = st->tile_start.as<uint32_t>();
  ca.tile_end = st->tile_end.as<uint32_t>();
  ca.tile_bgend = st->tile_bgend.as<uint32_t>();
  ca.order = st->order_fwd.as<uint32_t>();
  ca.act_tile = st->act_tile.as<uint32_t>();
  ca.aorder = st->aorder.as<uint32_t>();
  ca.aitem_pair = st->aitem_pair.as<uint32_t>();
  ca.aitem_chunk = st->aitem_chunk.as<uint32_t>();
  ca.pair_nck = st->pair_nck.as<uint32_t>();
  ca.pair_pbase = st->pair_pbase.as<uint32_t>();
  ca.aplan_counts = st->aplan_counts.as<uint32_t>();
  ca.apart = st->apart.as<float4>();
  ca.item_tile = st->item_tile.as<uint32_t>();
  ca.item_chunk = st->item_chunk.as<uint32_t>();
  ca.tile_nck = st->tile_nck.as<uint32_t>();
  ca.tile_pbase = st->tile_pbase.as<uint32_t>();
  ca.plan_counts = st->plan_counts.as<uint32_t>();
  ca.chunk_b = st->chunk_b.as<float>();
  ca.chunk_part = st->chunk_part.as<float4>();
  ca.item_work = st->item_work.as<uint32_t>();
  ca.pair_val = st->pair_val.as<uint32_t>();
  ca.rec_geo = st->rec_geo.as<float4>();
  ca.rec_g8a = st->rec_g8a.as<float4>();
  ca.rec_g8b = st->rec_g8b.as<float4>();
  ca.rec_cn = st->rec_cn.as<float4>();
  ca.rec_nrm = st->rec_nrm.as<float4>();
  ca.rec_rect = st->rec_rect.as<uint64_t>();
  ca.act_beg = st->act_beg.as<uint32_t>();
  ca.act_oct = st->act_oct.as<uint32_t>();
  ca.act_sub = st->act_sub.as<uint2>();
  ca.seg_se = st->seg_se.as<float2>();
  ca.seg_meta = st->seg_meta.as<uint32_t>();
  ca.seg_p0 = st->seg_p0.as<float4>();
  ca.seg_p1 = st->seg_p1.as<float4>();
  ca.seg_t0 = st->seg_t0.as<float4>();
  ca.seg_t1 = st->seg_t1.as<float4>();
  ca.pix_nseg = st->pix_nseg.as<uint32_t>();
  ca.fin0 = st->fin0.as<float4>();
  ca.fin1 = st->fin1.as<float4>();
  ca.fin2 = st->fin2.as<float4>();
  ca.fin3 = st->fin3.as<float4>();
  ca.outs = st->outs_d.as<dv_outputs>();
  ca.n_actors = n_oct - 1;
  ca.K = op.K;
  // stop below eps (at least the smallest normal float: an exact walk
  // stops only where T has underflowed)
  ca.eps = std::max(op.eps_stop, FLT_MIN);
  ca.tau_near = op.tau_near;
  ca.c = op.explin_c;
  ca.inv_c = 1.0f / op.explin_c;
  for (int i = 0; i < 3; ++i) ca.bg[i] = op.bg[i];
  ca.sky = op.sky;
  ca.sky_w = op.sky_w;
  ca.sky_h = op.sky_h;
  ca.sky_grad = nullptr;
  ca.mask = op.out_mask;
  ca.counters = (ctx->prof_flags.load() & DV_PROFILE_COUNTERS) ? ctx->counters : nullptr;
  if (nt > 0) {
    const bool nrm = (op.out_mask & DV_OUT_NORMAL) != 0;
    const bool k1 = op.K == 1;
    if (st->n_apairs > 0) {
      StageTimer tm_act(ctx, ST_ACTOR_FWD, s);
      DBuf big;
      DV_TRY(alloc_n<uint32_t>(ctx, big, st->n_apairs + 1, s));
      DV_TRY(fill_u32(big.as<uint32_t>(), 0u, 1, s));
      hipLaunchKernelGGL(k_build_segments, dim3((unsigned)st->n_apairs), dim3(TPB), 0,
                         s, ca, big.as<uint32_t>());
      hipLaunchKernelGGL(k_build_segments_big,
                         dim3((unsigned)std::min<int64_t>(st->n_apairs, 256)), dim3(TPB),
                         0, s, ca, (const uint32_t*)big.as<uint32_t>());
      auto ka = nrm ? (k1 ? k_actor_fwd<true, 1> : k_actor_fwd<true, 0>)
                    : (k1 ? k_actor_fwd<false, 1> : k_actor_fwd<false, 0>);
      hipLaunchKernelGGL(ka, dim3((unsigned)st->max_aitems), dim3(TPB), 0, s, ca);
      hipLaunchKernelGGL(k_actor_merge, dim3((unsigned)st->n_apairs), dim3(TPB), 0, s, ca);
    }
    const unsigned ni = (unsigned)st->max_items;
    {
      StageTimer tm_ch(ctx, ST_OTHER, s);
      const unsigned gb = (unsigned)std::min<int64_t>(st->max_slots, 16384) * CB_SPLIT;
      hipLaunchKernelGGL(k_chunk_bounds, dim3(gb), dim3(TPB), 0, s, ca,
                         (const uint32_t*)st->slot_tile.as<uint32_t>());
    }
    if (!composite) {
      // the background walks are run by the caller (the serving kernel)
      st->ca_fwd = ca;
      DV_TRY_HIP(hipGetLastError());
      return DV_OK;
    }
    {
      StageTimer tm_comp(ctx, ST_COMPOSITE_FWD, s);
      auto kern = nrm ? (k1 ? k_composite_fwd<true, 1> : k_composite_fwd<true, 0>)
                      : (k1 ? k_composite_fwd<false, 1> : k_composite_fwd<false, 0>);
      hipLaunchKernelGGL(kern, dim3(ni), dim3(TPB), 0, s, ca);
    }
    StageTimer tm_m(ctx, ST_OTHER, s);
    hipLaunchKernelGGL(k_chunk_merge,
                       dim3((unsigned)std::min<int64_t>(st->max_slots, 16384)),
                       dim3(TPB), 0, s, ca,
                       (const uint32_t*)st->slot_tile.as<uint32_t>());
  }
  DV_TRY_HIP(hipGetLastError());
  return DV_OK;
}

void retire_state(dv_ctx* ctx, dv_fwd_state* st) {
  hipEvent_t ev = nullptr;
  if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess ||
      hipEventRecord(ev, st->stream) != hipSuccess) {
    (void)hipGetLastError();
    if (ev) hipEventDestroy(ev);
    hipStreamSynchronize(st->stream);
    delete st;
    return;
  }
  std::lock_guard<std::mutex> lk(ctx->gy_mu);
  ctx->graveyard.emplace_back(ev, st);
}

void reap_states(dv_ctx* ctx, bool wait) {
  std::vector<std::pair<hipEvent_t, dv_fwd_state*>> done;
  {
    std::lock_guard<std::mutex> lk(ctx->gy_mu);
    auto& g = ctx->graveyard;
    for (size_t i = 0; i < g.size();) {
      if (wait) hipEventSynchronize(g[i].first);
      if (hipEventQuery(g[i].first) == hipSuccess) {
        done.push_back(g[i]);
        g[i] = g.back();
        g.pop_back();
      } else {
        ++i;
      }
    }
  }
  // their work has completed: the freed blocks are idle
  IdleRelease idle;
  for (auto& pr : done) {
    hipEventDestroy(pr.first);
    delete pr.second;
  }
}

dv_status check_opts(const dv_render_opts* op) {
  if (!op || op->K < 1 || op->K > DV_MAX_K || !(op->eps_stop >= 0.0f) ||
      !(op->tau_near >= 0.0f) || !(op->explin_c > 0.0f) ||
      !std::isfinite(op->tau_near)) {
    set_error("invalid render options");
    return DV_ERR_INVALID;
  }
  if (op->sky && (op->sky_w < 1 || op->sky_h < 1 ||
                  (int64_t)op->sky_w * op->sky_h > ((int64_t)1 << 28))) {
    set_error("invalid sky map size %d x %d", op->sky_w, op->sky_h);
    return DV_ERR_INVALID;
  }
  if (op->feat && (op->feat_dim < 1 || op->feat_group < 0 ||
                   3 * (int64_t)op->feat_group >= op->feat_dim)) {
    set_error("invalid feature render: dim %d, group %d", op->feat_dim,
              op->feat_group);
    return DV_ERR_INVALID;
  }
  return DV_OK;
}

// The options a render runs with: a feature render composites over a zero
// background.
dv_render_opts effective_opts(const dv_render_opts& op) {
  dv_render_opts o = op;
  if (o.feat) {
    o.bg[0] = o.bg[1] = o.bg[2] = 0.0f;
    o.sky = nullptr;
    o.sky_w = o.sky_h = 0;
  }
  return o;
}

dv_status check_feat_ptrs(const dv_render_opts& op, const dv_scene* sc) {
  if (!op.feat) return DV_OK;
  for (int k = 0; k < sc->n_oct; ++k)
    if (!op.feat[k] && sc->desc[k].n_voxels > 0) {
      set_error("feature render: octree %d has no feature array", k);
      return DV_ERR_INVALID;
    }
  return DV_OK;
}

}  // namespace dv

extern "C" {

dv_status dv_render(dv_ctx* ctx, const dv_scene* scene, const dv_view* views,
                    int32_t n_views, const double* pose_override,
                    const dv_render_opts* opts, const dv_outputs* outs,
                    dv_fwd_state** keep, void* stream) {
  if (keep) *keep = nullptr;
  if (!ctx || !scene || !views || n_views < 1 || !outs) {
    set_error("dv_render: invalid arguments");
    return DV_ERR_INVALID;
  }
  if (ctx->poisoned) {
    set_error("dv_render: context poisoned by an earlier device error");
    return DV_ERR_DEVICE;
  }
  DV_TRY(check_opts(opts));
  DV_TRY_HIP(hipSetDevice(ctx->device));
  PoolStamp stamp_on_return(ctx);
  hipStream_t s = (hipStream_t)stream;
  std::unique_ptr<dv_fwd_state> st(new dv_fwd_state());
  st->ctx = ctx;
  st->scene = scene;
  st->stream = s;
  DV_TRY(check_feat_ptrs(*opts, scene));
  st->opts = effective_opts(*opts);
  reap_states(ctx, false);
  DV_TRY(setup_state(st.get(), scene, views, n_views, pose_override));
  dv_status rs = run_forward(ctx, scene, st.get(), outs, s, true);
  if (rs == DV_ERR_DEVICE) ctx->poisoned = true;
  if (rs != DV_OK) {
    if (rs == DV_ERR_DEVICE) return rs;
    retire_state(ctx, st.release());
    return rs;
  }
  if (keep) *keep = st.release();
  else retire_state(ctx, st.release());
  return DV_OK;
}

void dv_fwd_state_release(dv_fwd_state* state) {
  if (!state) return;
  retire_state(state->ctx, state);
}

dv_status dv_fwd_state_info(const dv_fwd_state* st, dv_state_info* info) {
  if (!st || !info) return DV_ERR_INVALID;
  info->n_views = st->n_views;
  info->n_visible = st->n_vis;
  info->n_pairs = st->n_pairs;
  info->n_actor_pairs = st->n_apairs;
  info->n_tiles = st->n_tiles;
  info->key_bits = st->key_bits;
  info->tile_bits = st->tile_bits;
  info->n_items = 0;
  info->n_chunk_slots = 0;
  if (st->n_tiles > 0) {
    uint32_t c[2] = {0, 0};
    DV_TRY_HIP(hipSetDevice(st->ctx->device));
    DV_TRY_HIP(hipStreamSynchronize(st->stream));
    DV_TRY_HIP(hipMemcpy(c, st->plan_counts.p, sizeof(c), hipMemcpyDeviceToHost));
    info->n_items = c[0];
    info->n_chunk_slots = c[1];
  }
  info->n_actor_items = 0;
  info->n_actor_chunk_slots = 0;
  if (st->n_apairs > 0) {
    uint32_t c[2] = {0, 0};
    DV_TRY_HIP(hipMemcpy(c, st->aplan_counts.p, sizeof(c), hipMemcpyDeviceToHost));
    info->n_actor_items = c[0];
    info->n_actor_chunk_slots = c[1];
  }
  return DV_OK;
}

dv_status dv_fwd_state_export_lists(const dv_fwd_state* st, int32_t view,
                                    int64_t* tile_start, int32_t* entry_oct,
                                    int32_t* entry_leaf, int64_t capacity,
                                    int64_t* actor_start, int32_t* actor_oct,
                                    int64_t actor_capacity) {
  if (!st || view < 0 || view >= st->n_views || !tile_start) {
    set_error("dv_fwd_state_export_lists: invalid arguments");
    return DV_ERR_INVALID;
  }
  DV_TRY_HIP(hipSetDevice(st->ctx->device));
  DV_TRY_HIP(hipStreamSynchronize(st->stream));
  const ViewConst& V = st->views_h[view];
  const int64_t nt = (int64_t)V.ntx * V.nty;
  std::vector<uint32_t> ts(nt), te(nt);
  if (nt > 0) {
    DV_TRY_HIP(hipMemcpy(ts.data(), st->tile_start.as<uint32_t>() + V.tile_base,
                         4 * nt, hipMemcpyDeviceToHost));
    DV_TRY_HIP(hipMemcpy(te.data(), st->tile_end.as<uint32_t>() + V.tile_base,
                         4 * nt, hipMemcpyDeviceToHost));
  }
  std::vector<uint32_t> pv(st->n_pairs), seg(st->n_vis), vox(st->n_vis);
  if (st->n_pairs > 0)
    DV_TRY_HIP(hipMemcpy(pv.data(), st->pair_val.p, 4 * st->n_pairs,
                         hipMemcpyDeviceToHost));
  if (st->n_vis > 0) {
    DV_TRY_HIP(hipMemcpy(seg.data(), st->rec_seg.p, 4 * st->n_vis,
                         hipMemcpyDeviceToHost));
    DV_TRY_HIP(hipMemcpy(vox.data(), st->rec_vox.p, 4 * st->n_vis,
                         hipMemcpyDeviceToHost));
  }
  int64_t pos = 0;
  for (int64_t t = 0; t < nt; ++t) {
    tile_start[t] = pos;
    const uint32_t b = te[t] > ts[t] ? ts[t] : 0, e = te[t] > ts[t] ? te[t] : 0;
    for (uint32_t i = b; i < e; ++i) {
      if (pos >= capacity) {
        set_error("export capacity %lld too small", (long long)capacity);
        return DV_ERR_LIMIT;
      }
      const uint32_t r = pv[i];
      if (entry_oct) entry_oct[pos] = (int32_t)(seg[r] % st->n_oct);
      if (entry_leaf) entry_leaf[pos] = (int32_t)vox[r];
      ++pos;
    }
  }
  tile_start[nt] = pos;
  if (actor_start) {
    int64_t ap = 0;
    for (int64_t t = 0; t < nt; ++t) {
      actor_start[t] = ap;
      const uint32_t b = st->act_beg_h[V.tile_base + t];
      const uint32_t e = st->act_beg_h[V.tile_base + t + 1];
      for (uint32_t i = b; i < e; ++i) {
        if (ap >= actor_capacity) {
          set_error("actor export capacity too small");
          return DV_ERR_LIMIT;
        }
        if (actor_oct) actor_oct[ap] = (int32_t)st->act_oct_h[i];
        ++ap;
      }
    }
    actor_start[nt] = ap;
  }
  return DV_OK;
}

}  // extern "C"
