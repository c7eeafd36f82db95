// Reverse pass (Sec. 3.4: gradients flow through each voxel segment).
//
// With v_i = G_C.c_i + G_D (a_i+b_i)/2 + G_N.n_i and
// L = G_C.C + G_D D + G_N.N + (G_C.bg + G_T) T_final, the derivative with
// respect to the optical depth of piece i is
//     dL/dtau_i = T_{i+1} v_i - (L - sum_{j<=i} w_j v_j),
// so the backward re-walks every pixel in forward order with identical
// FP32 arithmetic (same piece evaluation, same stop decisions) instead of
// storing per-sample state.  Asset segments were composited in the forward
// as partial states spliced into the background walk; the re-walk records
// for every spliced segment its entry transmittance T_pre and the suffix
// S_after = L - (prefix through the segment), after which each asset's
// pieces can be differentiated on their own:
//     dL/dtau_i = T_pre T_loc,i+1 v_i - (T_pre (V_q - P_loc,i) + S_after).
// Pose gradients (beyond the paper, which keeps tracks fixed) follow the
// ray in each actor frame: samples, leaf faces, box faces bounding
// segments, SH direction and the rotation of normals.
#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstring>

#include "render.h"

namespace dv {

constexpr int NACC = 14;  // per-record: dcol(3), dnrm(3), dg(8)

__device__ inline void add_axis(float3& v, int ax, float x) {
  if (ax == 0) v.x += x; else if (ax == 1) v.y += x; else v.z += x;
}
__device__ inline float get_axis(float3 v, int ax) {
  return ax == 0 ? v.x : (ax == 1 ? v.y : v.z);
}

struct BwdBatch {
  float4 geo[TPB];
  float4 ga[TPB];
  float4 gb[TPB];
  float4 cn[TPB];
  float4 nrm[TPB];
  uint2 rect[TPB];
  uint32_t rid[TPB];
  float acc[NACC][TPB];
};

// NORMALS = false: the normal slot carries the leaf's far corner instead.
template <bool NORMALS>
__device__ inline void load_bwd_batch(BwdBatch& B, const CompArgs& a,
                                      uint32_t base, uint32_t n) {
  const int tid = threadIdx.x;
  if ((uint32_t)tid < n) {
    const uint32_t r = a.pair_val[base + tid];
    const float4 geo = a.rec_geo[r];
    B.rid[tid] = r;
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

// Lane exchanges of the reduction below (gfx950).  swap32 / swap16 pair
// the two registers across lane halves / 16-lane rows so that a + b leaves
// the upper half (odd rows) with the sum of the second register and the
// lower half (even rows) with the sum of the first; dpp() reads a lane of
// the same 16-lane row.
__device__ inline float swap32_sum(float a, float b) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a),
                                                  __float_as_uint(b), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ inline float swap16_sum(float a, float b) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a),
                                                  __float_as_uint(b), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
template <int CTRL>
__device__ inline float dpp(float x) {
  return __int_as_float(
      __builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}
constexpr int DPP_ROR8 = 0x128;         // row_ror:8  -> lane ^ 8 in a row
constexpr int DPP_HALF_MIRROR = 0x141;  // lane ^ 7 within 8 lanes
constexpr int DPP_XOR2 = 0x4E;          // quad_perm [2,3,0,1]
constexpr int DPP_XOR1 = 0xB1;          // quad_perm [1,0,3,2]

// Reduce one lane-contribution set into the batch slot r.  The 14
// channels (padded to 16) are summed over the wave with a transposing
// butterfly: at each exchange a lane keeps half of its channels and adds the
// partner's copy of them (partners lane ^ 32, ^ 16, ^ 8, ^ 7, then ^ 2 and
// ^ 1 on the last channel; together they span all 64 lanes), which leaves
// lane l with the full sum of channel l >> 2; lanes with l % 4 == 0 then add
// their channel into LDS.  Cross-half and cross-row steps use the gfx950
// permlane swaps, in-row steps DPP, so no exchange goes through LDS.  Must
// be called wave-uniformly with every lane active; lanes without a hit pass
// zero contributions.
// 12-slot version of the butterfly below: 6, 3, then 2 (one pad) and 1
// values per lane; lane l ends with the wave sum of slot 6 h5 + 3 h4 + 2 h3
// + h2 (h_i: bit i of l; lanes with h3 = h2 = 1 hold the pad, 0).  Called
// wave-uniformly with every lane active.
__device__ inline float wave_sum12(float* v, int& slot, bool& pad) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int i = 0; i < 6; ++i) v[i] = swap32_sum(v[i], v[i + 6]);
#pragma unroll
  for (int i = 0; i < 3; ++i) v[i] = swap16_sum(v[i], v[i + 3]);
  v[3] = 0.0f;
  {
    const bool up = (lane & 8) != 0;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const float send = up ? v[i] : v[i + 2];
      const float keep = up ? v[i + 2] : v[i];
      v[i] = keep + dpp<DPP_ROR8>(send);
    }
  }
  {
    const bool up = (lane & 4) != 0;
    const float send = up ? v[0] : v[1];
    const float keep = up ? v[1] : v[0];
    v[0] = keep + dpp<DPP_HALF_MIRROR>(send);
  }
  v[0] += dpp<DPP_XOR2>(v[0]);
  v[0] += dpp<DPP_XOR1>(v[0]);
  slot = 6 * ((lane >> 5) & 1) + 3 * ((lane >> 4) & 1) + 2 * ((lane >> 3) & 1) +
         ((lane >> 2) & 1);
  pad = (lane & 12) == 12;
  return v[0];
}

// Without normals the 11 live channels (colour, corners) go through the
// 12-slot butterfly (slot 11 is zero).
template <bool NORMALS>
__device__ inline void accum_record(BwdBatch& B, uint32_t r, bool hit,
                                    float3 dcol, float3 dnrm,
                                    const float* dg) {
  if (__ballot(hit) == 0) return;
  const int lane = threadIdx.x & 63;
  if (!NORMALS) {
    float v[12];
    v[0] = dcol.x; v[1] = dcol.y; v[2] = dcol.z;
#pragma unroll
    for (int m = 0; m < 8; ++m) v[3 + m] = dg[m];
    v[11] = 0.0f;
    int slot;
    bool pad;
    const float x = wave_sum12(v, slot, pad);
    // slots 0-2: colour (channels 0-2), 3-10: corners (channels 6-13)
    const int ch = slot < 3 ? slot : slot + 3;
    if ((lane & 3) == 0 && !pad && slot < 11 && x != 0.0f)
      atomicAdd(&B.acc[ch][r], x);
    return;
  }
  float v[16];
  v[0] = dcol.x; v[1] = dcol.y; v[2] = dcol.z;
  v[3] = dnrm.x; v[4] = dnrm.y; v[5] = dnrm.z;
#pragma unroll
  for (int m = 0; m < 8; ++m) v[6 + m] = dg[m];
  v[14] = 0.0f;
  v[15] = 0.0f;
  // lane bit 5: channels 0-7 stay in the lower half, 8-15 in the upper
#pragma unroll
  for (int i = 0; i < 8; ++i) v[i] = swap32_sum(v[i], v[i + 8]);
  // lane bit 4 (rows)
#pragma unroll
  for (int i = 0; i < 4; ++i) v[i] = swap16_sum(v[i], v[i + 4]);
  // lane bit 3: partner lane ^ 8
  {
    const bool up = (lane & 8) != 0;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const float send = up ? v[i] : v[i + 2];
      const float keep = up ? v[i + 2] : v[i];
      v[i] = keep + dpp<DPP_ROR8>(send);
    }
  }
  // lane bit 2: partner lane ^ 7 (opposite bit 2)
  {
    const bool up = (lane & 4) != 0;
    const float send = up ? v[0] : v[1];
    const float keep = up ? v[1] : v[0];
    v[0] = keep + dpp<DPP_HALF_MIRROR>(send);
  }
  v[0] += dpp<DPP_XOR2>(v[0]);
  v[0] += dpp<DPP_XOR1>(v[0]);
  const int ch = lane >> 2;
  if ((lane & 3) == 0 && ch < NACC && v[0] != 0.0f) atomicAdd(&B.acc[ch][r], v[0]);
}

__device__ inline void flush_batch(BwdBatch& B, const CompArgs& a,
                                   uint32_t n) {
  __syncthreads();
  const int tid = threadIdx.x;
  if ((uint32_t)tid < n) {
    const uint32_t r = B.rid[tid];
    float* gc = reinterpret_cast<float*>(a.gr_col + r);
    float* gn = reinterpret_cast<float*>(a.gr_nrm + r);
    float* g0 = reinterpret_cast<float*>(a.gr_g8a + r);
    float* g1 = reinterpret_cast<float*>(a.gr_g8b + r);
#pragma unroll
    for (int c = 0; c < NACC; ++c) {
      const float x = B.acc[c][tid];
      if (x != 0.0f) {
        float* dst = c < 3 ? gc + c : (c < 6 ? gn + (c - 3)
                                             : (c < 10 ? g0 + (c - 6) : g1 + (c - 10)));
        atomicAdd(dst, x);
        B.acc[c][tid] = 0.0f;
      }
    }
  }
}

// One lane's gradients of entry r added to the batch slot (LDS atomics),
// for walks in which the lanes of a wave hold different entries.
template <bool NORMALS>
__device__ inline void lane_record(BwdBatch& B, uint32_t r, float3 dcol,
                                   float3 dnrm, const float* dg) {
  float v[NACC];
  v[0] = dcol.x; v[1] = dcol.y; v[2] = dcol.z;
  v[3] = dnrm.x; v[4] = dnrm.y; v[5] = dnrm.z;
#pragma unroll
  for (int m = 0; m < 8; ++m) v[6 + m] = dg[m];
#pragma unroll
  for (int c = 0; c < NACC; ++c)
    if ((NORMALS || c < 3 || c >= 6) && v[c] != 0.0f) atomicAdd(&B.acc[c][r], v[c]);
}

// Block-reduce 12 floats per thread and add them to dst (one atomic each).
// Called by the whole block.
__device__ inline void block_add12(float* red, const float* v12, float* dst) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  float v[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) v[c] = v12[c];
  int slot;
  bool pad;
  const float x = wave_sum12(v, slot, pad);
  __syncthreads();
  if ((lane & 3) == 0 && !pad) red[w * 12 + slot] = x;
  __syncthreads();
  if (threadIdx.x < 12) {
    float s = 0.0f;
    for (int i = 0; i < TPB / 64; ++i) s += red[i * 12 + threadIdx.x];
    if (s != 0.0f) atomicAdd(dst + threadIdx.x, s);
  }
}

// (o_k, d_k) gradients of one pixel -> (R, p) gradient row-major 9 + 3.
__device__ inline void pose12(const VOConst& C, float3 d, float3 go, float3 gd,
                              float* out) {
  const float om[3] = {C.omp[0], C.omp[1], C.omp[2]};
  const float dd[3] = {d.x, d.y, d.z};
  const float g_o[3] = {go.x, go.y, go.z}, g_d[3] = {gd.x, gd.y, gd.z};
  for (int b = 0; b < 3; ++b)
    for (int a = 0; a < 3; ++a) out[b * 3 + a] = om[b] * g_o[a] + dd[b] * g_d[a];
  for (int b = 0; b < 3; ++b)
    out[9 + b] = -(C.R[b * 3 + 0] * g_o[0] + C.R[b * 3 + 1] * g_o[1] +
                   C.R[b * 3 + 2] * g_o[2]);
}

// Upstream gradients of the pixel.
struct PixGrad {
  float3 GC, GN;
  float GD, GT;
};
template <bool NORMALS>
__device__ inline PixGrad pixel_grads(const CompArgs& a, const PixSetup& P) {
  PixGrad g;
  g.GC = make_float3(0, 0, 0);
  g.GN = make_float3(0, 0, 0);
  g.GD = 0.0f;
  g.GT = 0.0f;
  if (!P.valid) return g;
  const ViewConst& V = a.views[P.v];
  const dv_out_grads& G = a.gin[P.v];
  const size_t hw = (size_t)V.w * V.h, o = (size_t)P.py * V.w + P.px;
  if (G.rgb) g.GC = make_float3(G.rgb[o], G.rgb[hw + o], G.rgb[2 * hw + o]);
  if (G.depth) g.GD = G.depth[o];
  if (NORMALS && G.normal)
    g.GN = make_float3(G.normal[o], G.normal[hw + o], G.normal[2 * hw + o]);
  if (G.T) g.GT = G.T[o];
  return g;
}
// Upstream-weighted value of a (C.rgb, D) and (N.xyz, -) pair.
__device__ inline float gdot(const PixGrad& g, float4 c, float4 n) {
  return g.GC.x * c.x + g.GC.y * c.y + g.GC.z * c.z + g.GD * c.w +
         g.GN.x * n.x + g.GN.y * n.y + g.GN.z * n.z;
}

// Backward values of every segment of every pixel in tiles with actor
// boxes: (-1: not spliced yet, 0, 0, 0).  Only the pixel's own segments
// are ever read.
__global__ void __launch_bounds__(TPB) k_seg_bw_init(CompArgs a) {
  // one block per (tile, actor) pair; the tile's first pair does the tile
  const uint32_t gt = a.act_tile[blockIdx.x];
  const uint32_t a_beg = a.act_beg[gt];
  if (blockIdx.x != a_beg) return;
  const int n_at = (int)(a.act_beg[gt + 1] - a_beg);
  const int tid = threadIdx.x;
  const uint32_t seg0 = 3 * a_beg + n_at;
  const int nseg = (int)a.pix_nseg[(size_t)gt * TPB + tid];
  for (int q = 0; q < nseg; ++q)
    a.seg_bw[seg_index(seg0 + q, tid)] = make_float4(-1.0f, 0.0f, 0.0f, 0.0f);
}

// Backward, part 1 (tiles of several chunks): per pixel and chunk, the
// transmittance in front of the chunk and the part of L behind it,
// S_after_c = sum_{c' > c} T_<c' V_c' + T (C_bg.G_C + G_T), summed from the
// back so that no difference of large sums is formed.
template <bool NORMALS>
__device__ inline void chunk_prep_tile(const CompArgs& a, uint32_t gt) {
  const uint32_t nck = a.tile_nck[gt];
  const int tid = threadIdx.x;
  const PixSetup P = pixel_setup(a, gt, tid);
  if (!P.valid) return;
  const PixGrad g = pixel_grads<NORMALS>(a, P);
  const size_t s0 = (size_t)a.tile_pbase[gt] * TPB + tid;
  const float4* part = a.chunk_part + s0 * 4;
  float T = 1.0f;
  for (uint32_t c = 0; c < nck; ++c) {
    a.chunk_tps[s0 + (size_t)c * TPB] = make_float2(T, 0.0f);
    T *= part[(size_t)c * TPB * 4 + 1].w;
  }
  const float3 cs = sky_colour(a, P.d);
  float S = (g.GC.x * cs.x + g.GC.y * cs.y + g.GC.z * cs.z + g.GT) * T;
  for (uint32_t c = nck; c-- > 0;) {
    const size_t q = (size_t)c * TPB;
    const float Tp = a.chunk_tps[s0 + q].x;
    a.chunk_tps[s0 + q] = make_float2(Tp, S);
    const float Vc = gdot(g, part[q * 4], part[q * 4 + 1]);
    S = fmaf(Tp, Vc, S);
  }
}
template <bool NORMALS>
__global__ void __launch_bounds__(TPB) k_chunk_prep(CompArgs a,
                                                    const uint32_t* slot_tile) {
  const uint32_t n_slots = a.plan_counts[1];
  for (uint32_t sl = blockIdx.x; sl < n_slots; sl += gridDim.x) {
    const uint32_t gt = chunked_tile_at(a, slot_tile, sl);
    if (gt != 0xFFFFFFFFu) chunk_prep_tile<NORMALS>(a, gt);
  }
}

// Sky map gradient (Eq. 2): the pixel's C_sky enters C with weight
// T_final, so dL/dC_sky = T_final G_C, spread over the four bilinear taps.
// One block per tile; T_final is the product of the chunks' transmittances
// for a chunked tile. A tile's pixels fall on a few neighbouring texels, so
// the block sums its taps in LDS over its texel footprint (columns counted
// from a reference column, so the footprint may straddle the wrap) and adds
// each texel once to the map's gradient; a footprint larger than the LDS
// table adds every tap directly.
constexpr int SKY_LDS = 256;  // texels per block table
template <bool NORMALS>
__global__ void __launch_bounds__(TPB) k_sky_bwd(CompArgs a) {
  __shared__ float tab[3][SKY_LDS];
  __shared__ int box[4];  // min row, max row, min column, max column
  const uint32_t gt = blockIdx.x;
  const int tid = threadIdx.x;
  const PixSetup P = pixel_setup(a, gt, tid);
  const int W = a.sky_w, H = a.sky_h;
  const size_t hw = (size_t)W * H;
  float3 gs = make_float3(0, 0, 0);
  SkyTaps t;
  if (P.valid) {
    const PixGrad g = pixel_grads<NORMALS>(a, P);
    const uint32_t nck = a.tile_nck[gt];
    float T;
    if (nck <= 1) {
      T = a.fin1[P.pix].w;
    } else {
      const size_t s0 = (size_t)a.tile_pbase[gt] * TPB + tid;
      const float4* part = a.chunk_part + s0 * 4;
      T = 1.0f;
      for (uint32_t c = 0; c < nck; ++c) T *= part[(size_t)c * TPB * 4 + 1].w;
    }
    gs = make_float3(T * g.GC.x, T * g.GC.y, T * g.GC.z);
    t = sky_taps(a, P.d);
  }
  const bool act = gs.x != 0.0f || gs.y != 0.0f || gs.z != 0.0f;
  // reference column: the tile's centre pixel direction is not needed; any
  // fixed column works as long as every tap is counted from it
  const PixSetup Pc = pixel_setup(a, gt, 0);
  const int ref = sky_taps(a, Pc.d).o[0] % W;
  int r0 = 0, r1 = 0, c0 = 0;
  if (act) {
    r0 = t.o[0] / W;
    r1 = t.o[2] / W;
    int dc = t.o[0] % W - ref;
    if (dc < 0) dc += W;
    if (2 * dc > W) dc -= W;
    c0 = dc;
  }
  if (tid == 0) {
    box[0] = H; box[1] = -1; box[2] = W; box[3] = -W;
  }
  __syncthreads();
  if (act) {
    atomicMin(&box[0], r0);
    atomicMax(&box[1], r1);
    atomicMin(&box[2], c0);
    atomicMax(&box[3], c0 + 1);
  }
  __syncthreads();
  if (box[1] < 0) return;  // no pixel of the tile adds anything
  const int rmin = box[0], ncol = box[3] - box[2] + 1, cmin = box[2];
  const int nrow = box[1] - rmin + 1;
  if (nrow * ncol > SKY_LDS) {
    if (act) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (t.w[k] == 0.0f) continue;
        atomicAdd(a.sky_grad + t.o[k], t.w[k] * gs.x);
        atomicAdd(a.sky_grad + hw + t.o[k], t.w[k] * gs.y);
        atomicAdd(a.sky_grad + 2 * hw + t.o[k], t.w[k] * gs.z);
      }
    }
    return;
  }
  for (int i = tid; i < 3 * SKY_LDS; i += TPB) (&tab[0][0])[i] = 0.0f;
  __syncthreads();
  // taps 0/1 on row r0, 2/3 on row r1; columns c0 and c0 + 1. The lanes of
  // a wave mostly share a few texels: per texel, the wave sums its lanes'
  // values and one lane adds them to the table (the loop is wave-uniform:
  // keys come from ballots and lane reads).
  const int lane = tid & 63;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int e = act ? ((k < 2 ? r0 : r1) - rmin) * ncol + c0 + (k & 1) - cmin : -1;
    const float vx = act ? t.w[k] * gs.x : 0.0f;
    const float vy = act ? t.w[k] * gs.y : 0.0f;
    const float vz = act ? t.w[k] * gs.z : 0.0f;
    uint64_t pend = __ballot(act);
    while (pend != 0) {
      const int leader = __builtin_ctzll(pend);
      const int key = __shfl(e, leader, 64);
      const bool mine = e == key;
      pend &= ~__ballot(mine);
      float sx = mine ? vx : 0.0f, sy = mine ? vy : 0.0f, sz = mine ? vz : 0.0f;
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        sx += __shfl_xor(sx, o, 64);
        sy += __shfl_xor(sy, o, 64);
        sz += __shfl_xor(sz, o, 64);
      }
      if (lane == leader) {
        atomicAdd(&tab[0][key], sx);
        atomicAdd(&tab[1][key], sy);
        atomicAdd(&tab[2][key], sz);
      }
    }
  }
  __syncthreads();
  for (int e = tid; e < nrow * ncol; e += TPB) {
    int col = (ref + cmin + e % ncol) % W;
    if (col < 0) col += W;
    const size_t o = (size_t)(rmin + e / ncol) * W + col;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
      const float val = tab[ch][e];
      if (val != 0.0f) atomicAdd(a.sky_grad + ch * hw + o, val);
    }
  }
}

// Backward, part 2: the forward walk of one work item re-run in the same
// order with the same arithmetic (so the chunk-local T and every stop
// decision repeat bit for bit), giving for each background piece
//   dL/dtau_i = T_pre (T_{i+1} v_i - S_{i+1}) - S_after,
// where T, S are chunk-local (the suffix against the chunk's totals, or
// against its tail sums once T < T_REBASE), T_pre the transmittance in front
// of the chunk and S_after the part of L behind it (a tile of one chunk:
// T_pre = 1, S_after = its background term).  Per-record colour, normal and
// corner gradients are summed over the wave and block, then added once per
// record and batch; spliced segments get T_pre and S_after of their own for
// k_actor_bwd.
template <bool NORMALS, int KC>
__global__ void __launch_bounds__(TPB, 4) k_composite_bwd(CompArgs a) {
  __shared__ BwdBatch B;
  // the order holds every id below the grid size; ids past the item count
  // are unused
  const uint32_t item = a.order[blockIdx.x];
  if (item >= a.plan_counts[0]) return;
  const uint32_t gt = a.item_tile[item], chunk = a.item_chunk[item];
  const uint32_t nck = a.tile_nck[gt];
  const int tid = threadIdx.x;
  for (int c = 0; c < NACC; ++c) B.acc[c][tid] = 0.0f;
  const PixSetup P = pixel_setup(a, gt, tid);
  const int bx = P.bx, by = P.by;
  const bool valid = P.valid;
  const float3 d = P.d;
  const size_t pix = P.pix;
  const int K = a.K;
  const float invK = 1.0f / (float)K;
  uint32_t n_test = 0, n_piece = 0;
  uint32_t w_test = 0, w_piece = 0;  // wave-level counts (plain walk)
  uint32_t w_iter = 0, w_hit = 0;
  // upstream gradients scaled by the transmittance T_pre in front of the
  // chunk (1 for a tile of one chunk), so that
  //   dL/dtau_i = T_pre (T_{i+1} v_i - S_{i+1}) - S_after
  // becomes T_{i+1} v'_i - S'_{i+1} - S_after with v' = T_pre v
  PixGrad g = pixel_grads<NORMALS>(a, P);
  float Tpre = 1.0f, Saft = 0.0f;
  // running suffixes S' = V' - sum w v' over the chunk, and the tail's
  float S = 0.0f, ST = 0.0f;
  if (valid) {
    if (nck == 1) {
      const float4 f1 = a.fin1[pix];
      const float3 cs = sky_colour(a, P.d);
      Saft = (g.GC.x * cs.x + g.GC.y * cs.y + g.GC.z * cs.z + g.GT) * f1.w;
      S = gdot(g, a.fin0[pix], f1);
      ST = gdot(g, a.fin2[pix], a.fin3[pix]);
    } else {
      const size_t sl = ((size_t)a.tile_pbase[gt] + chunk) * TPB + tid;
      const float4* part = a.chunk_part + sl * 4;
      const float2 tps = a.chunk_tps[sl];
      Tpre = tps.x;
      Saft = tps.y;
      g.GC = make_float3(Tpre * g.GC.x, Tpre * g.GC.y, Tpre * g.GC.z);
      g.GN = make_float3(Tpre * g.GN.x, Tpre * g.GN.y, Tpre * g.GN.z);
      g.GD = Tpre * g.GD;
      S = gdot(g, part[0], part[1]);
      ST = gdot(g, part[2], part[3]);
    }
  }
  const float3 GC = g.GC, GN = g.GN;
  const float GDh = 0.5f * g.GD;  // depth of a piece: (a + b) / 2
  const uint32_t a_beg = a.act_beg[gt];
  const int n_at = (int)(a.act_beg[gt + 1] - a_beg);
  const uint32_t seg0 = 3 * a_beg + n_at;
  const int nseg = (n_at > 0 && valid) ? (int)a.pix_nseg[pix] : 0;

  // an off-window lane starts below the stop threshold (a.eps > 0)
  float T = valid ? 1.0f : 0.0f;
  auto live = [&]() { return T >= a.eps; };
  const float3 inv = safe_inv(d);
  uint32_t beg, bgend;
  chunk_range(a.tile_start[gt], a.tile_bgend[gt], nck, chunk, beg, bgend);
  // chunk boundaries: only to place a lane's segments between chunks
  float Bc = -F_INF, Bn = F_INF;
  if (nseg > 0) chunk_bounds(a, gt, nck, chunk, tid, Bc, Bn);
  auto suffix = [&]() { return T < T_REBASE ? ST : S; };
  // composite one piece of entry r and add its colour/normal/corner
  // gradients; returns dL/dtau, the piece's weight w (in the chunk) in wg
  // set: the piece's gradients replace dcol/dnrm/dg (the plain walk's one
  // piece per entry) instead of adding to them
  auto piece_grad = [&](uint32_t r, float tau, const PieceDer& pd, float pa,
                        float pb, float3& dcol, float3& dnrm, float* dg,
                        float& wg, bool set) {
    const float4 cn = B.cn[r];
    const float e = fast_exp(-tau);
    const float wgt = T * opacity(tau, e);
    const float wt = T < T_REBASE ? wgt : 0.0f;
    float vi = fmaf(GDh, pa + pb, fmaf(GC.z, cn.z, fmaf(GC.y, cn.y, GC.x * cn.x)));
    if (NORMALS) {
      const float4 nr = B.nrm[r];
      vi = fmaf(GN.z, nr.z, fmaf(GN.y, nr.y, fmaf(GN.x, nr.x, vi)));
    }
    S = fmaf(-wgt, vi, S);
    ST = fmaf(-wt, vi, ST);
    T *= e;
    const float dtau = fmaf(T, vi, -suffix()) - Saft;
    wg = wgt;
    if (set) {
      dcol = make_float3(wgt * GC.x, wgt * GC.y, wgt * GC.z);
      if (NORMALS) dnrm = make_float3(wgt * GN.x, wgt * GN.y, wgt * GN.z);
      set_corner_grads<KC>(pd, dtau, dg);
    } else {
      dcol.x += wgt * GC.x; dcol.y += wgt * GC.y; dcol.z += wgt * GC.z;
      if (NORMALS) {
        dnrm.x += wgt * GN.x; dnrm.y += wgt * GN.y; dnrm.z += wgt * GN.z;
      }
      add_corner_grads<KC>(pd, dtau, dg);
    }
    return dtau;
  };
  // waves none of whose pixels has an ownership segment take the plain
  // walk (wave-uniform), the others splice segments as they come
  const bool wseg = __ballot(nseg > 0) != 0;
  int qn = 0;
  while (qn < nseg && a.seg_se[seg_index(seg0 + qn, tid)].x < Bc) ++qn;
  float excl = qn > 0 ? a.seg_se[seg_index(seg0 + qn - 1, tid)].y : -F_INF;
  float ns = qn < nseg ? a.seg_se[seg_index(seg0 + qn, tid)].x : F_INF;
  auto splice = [&](int qq) {
    const size_t qi = seg_index(seg0 + qq, tid);
    const float4 q0 = a.seg_p0[qi], q1 = a.seg_p1[qi];
    const float Vq = gdot(g, q0, q1);
    const float Tseg = Tpre * T;
    S = fmaf(-T, Vq, S);
    ST = fmaf(T < T_REBASE ? -T : 0.0f, Vq, ST);
    T *= q1.w;
    // .x/.y only: .z (from the piece in front) and .w (from the piece
    // behind, possibly another chunk's block) are added separately
    float* bw = reinterpret_cast<float*>(a.seg_bw + qi);
    bw[0] = Tseg;
    bw[1] = suffix() + Saft;
  };
  for (uint32_t base = beg; base < bgend; base += TPB) {
    const uint32_t nb = min((uint32_t)TPB, bgend - base);
    load_bwd_batch<NORMALS>(B, a, base, nb);
    __syncthreads();
    uint64_t wm[4];
    wave_live_masks(B.rect, nb, bx, by, __ballot(live()), wm);
    for (int c = 0; c < 4; ++c) {
      uint64_t m = wm[c];
      if (!wseg) {
        // plain walk: a lane without a chord (or done) takes the empty piece
        // a = b = 0, whose tau = 0 leaves T and the sums as they are and
        // whose gradients are zero, so every lane runs the same code
        while (m != 0) {
          const uint64_t lm = __ballot(live());
          if (lm == 0) break;
          const uint32_t r = (uint32_t)c * 64 + (uint32_t)__builtin_ctzll(m);
          m &= m - 1;
          w_test += (uint32_t)__popcll(lm);
          ++w_iter;
          const float4 geo = B.geo[r];
          float t0, t1;
          batch_slab<NORMALS>(B, r, geo, inv, t0, t1);
          t0 = fmaxf(t0, a.tau_near);
          const bool hit = live() && t1 > t0;
          const uint64_t hm = __ballot(hit);
          if (hm == 0) continue;
          ++w_hit;
          w_piece += (uint32_t)__popcll(hm);
          const float pa = hit ? t0 : 0.0f, pb = hit ? t1 : 0.0f;
          PieceDer pd;
          const float tau = piece_eval<1, KC>(geo, B.ga[r], B.gb[r], B.cn[r].w,
                                              d, pa, pb, K, invK, a.c, a.inv_c,
                                              &pd);
          float3 dcol, dnrm = make_float3(0, 0, 0);
          float dg[8], wg;
          piece_grad(r, tau, pd, pa, pb, dcol, dnrm, dg, wg, true);
          accum_record<NORMALS>(B, r, hit, dcol, dnrm, dg);
        }
        continue;
      }
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
        // when no lane's chord meets a segment (nothing excluded at its
        // start, no segment starting before its end) every lane has at most
        // the one piece [t0, t1): the plain walk's straight-line code
        const bool plain = !chord || (excl <= t0 && ns >= t1);
        if (__ballot(!plain) == 0) {
          w_test += (uint32_t)__popcll(lm);
          ++w_iter;
          const uint64_t hm = __ballot(chord);
          if (hm == 0) continue;
          ++w_hit;
          w_piece += (uint32_t)__popcll(hm);
          const float pa = chord ? t0 : 0.0f, pb = chord ? t1 : 0.0f;
          PieceDer pd;
          const float tau = piece_eval<1, KC>(geo, B.ga[r], B.gb[r], B.cn[r].w,
                                              d, pa, pb, K, invK, a.c, a.inv_c,
                                              &pd);
          float3 dcol, dnrm = make_float3(0, 0, 0);
          float dg[8], wg;
          piece_grad(r, tau, pd, pa, pb, dcol, dnrm, dg, wg, true);
          accum_record<NORMALS>(B, r, chord, dcol, dnrm, dg);
          continue;
        }
        float3 dcol = make_float3(0, 0, 0), dnrm = make_float3(0, 0, 0);
        float dg[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        bool hit = false;
        if (live()) {
          ++n_test;
          if (t1 > t0) {
            float pa = fmaxf(t0, excl);
            bool a_seg = excl > t0;
            while (pa < t1 && live()) {
              if (pa >= ns) {
                const float ex = a.seg_se[seg_index(seg0 + qn, tid)].y;
                splice(qn);
                if (ex > pa) { pa = ex; a_seg = true; }
                excl = ex;
                ++qn;
                ns = qn < nseg ? a.seg_se[seg_index(seg0 + qn, tid)].x : F_INF;
                continue;
              }
              const bool b_seg = ns < t1;
              const float pb = fminf(t1, ns);
              const float inv_h = B.cn[r].w;
              PieceDer pd;
              const float tau =
                  (a_seg || b_seg)
                      ? piece_eval<2, KC>(geo, B.ga[r], B.gb[r], inv_h, d, pa, pb,
                                          K, invK, a.c, a.inv_c, &pd)
                      : piece_eval<1, KC>(geo, B.ga[r], B.gb[r], inv_h, d, pa, pb,
                                          K, invK, a.c, a.inv_c, &pd);
              ++n_piece;
              float wg;
              const float dtau =
                  piece_grad(r, tau, pd, pa, pb, dcol, dnrm, dg, wg, false);
              hit = true;
              if (a_seg && qn > 0)
                a.seg_bw[seg_index(seg0 + qn - 1, tid)].w +=
                    dtau * pd.dtda + wg * GDh;
              if (b_seg)
                a.seg_bw[seg_index(seg0 + qn, tid)].z +=
                    dtau * pd.dtdb + wg * GDh;
              pa = pb;
              a_seg = false;
            }
          }
        }
        accum_record<NORMALS>(B, r, hit, dcol, dnrm, dg);
      }
    }
    flush_batch(B, a, nb);
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
  count_work(a.counters, 2, n_test, n_piece);
  count_waves(a.counters, 10, w_iter, w_hit);
}

// Segments of actor j on the ray of this lane, in one pass over the
// lane's segments with the loads of 8 segments in flight together: their
// count and first, and the first and last of those spliced by the
// background walk (seg_bw.x >= 0; nseg and -1 when none).
__device__ inline int segs_of_actor_b(const CompArgs& a, uint32_t seg0, int nseg,
                                      int j, int tid, int& qfirst, int& sfirst,
                                      int& slast) {
  int nj = 0;
  qfirst = nseg;
  sfirst = nseg;
  slast = -1;
  for (int i0 = 0; i0 < nseg; i0 += 8) {
    bool own[8];
    float bwx[8];
#pragma unroll
    for (int k = 0; k < 8; ++k)
      own[k] = i0 + k < nseg &&
               (int)(a.seg_meta[seg_index(seg0 + i0 + k, tid)] & 0xFF) == j;
#pragma unroll
    for (int k = 0; k < 8; ++k)
      bwx[k] = own[k] ? a.seg_bw[seg_index(seg0 + i0 + k, tid)].x : -1.0f;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if (!own[k]) continue;
      if (nj == 0) qfirst = i0 + k;
      ++nj;
      if (bwx[k] >= 0.0f) {
        if (sfirst == nseg) sfirst = i0 + k;
        slast = i0 + k;
      }
    }
  }
  return nj;
}

// Backward, part 3a (actor lists of several chunks): for rays with a single
// segment of the actor, the transmittance W_c in front of chunk c inside
// the segment and the segment's part R_c behind the chunk, summed from the
// back.
template <bool NORMALS>
__global__ void __launch_bounds__(TPB) k_actor_prep(CompArgs a) {
  const uint32_t e = blockIdx.x;
  const uint32_t nck = a.pair_nck[e];
  if (nck <= 1) return;
  const uint32_t gt = a.act_tile[e];
  const uint32_t a_beg = a.act_beg[gt];
  const int n_at = (int)(a.act_beg[gt + 1] - a_beg);
  const int tid = threadIdx.x;
  const PixSetup P = pixel_setup(a, gt, tid);
  if (!P.valid) return;
  const uint32_t seg0 = 3 * a_beg + n_at;
  const int nseg = (int)a.pix_nseg[P.pix];
  int qfirst, sfirst, slast;
  if (segs_of_actor_b(a, seg0, nseg, (int)(e - a_beg), tid, qfirst, sfirst, slast) != 1)
    return;
  const PixGrad g = pixel_grads<NORMALS>(a, P);
  const size_t s0 = (size_t)a.pair_pbase[e] * TPB + tid;
  const float4* part = a.apart + s0 * 4;
  float W = 1.0f;
  for (uint32_t c = 0; c < nck; ++c) {
    a.atps[s0 + (size_t)c * TPB] = make_float2(W, 0.0f);
    W *= part[(size_t)c * TPB * 4 + 1].w;
  }
  float R = 0.0f;
  for (uint32_t c = nck; c-- > 0;) {
    const size_t q = (size_t)c * TPB;
    const float Wc = a.atps[s0 + q].x;
    a.atps[s0 + q] = make_float2(Wc, R);
    R = fmaf(Wc, gdot(g, part[q * 4], part[q * 4 + 1]), R);
  }
}

// Backward, part 3b: one block per actor work item (a chunk of one (tile,
// actor) list), after every part 2 block: pieces of the asset segments,
// with T_pre and S_after of their segment from the splice (for a chunk of a
// single-segment ray, T_pre W_c and T_pre R_c + S_after, with the chunk's
// own totals and tails); end points of segments on box faces go to the
// segment for part 4.
template <bool NORMALS, int KC>
__global__ void __launch_bounds__(TPB, 4) k_actor_bwd(CompArgs a) {
  __shared__ BwdBatch B;
  __shared__ float red[(TPB / 64) * 12];
  if (blockIdx.x >= a.aplan_counts[0]) return;
  const uint32_t item = a.aorder[blockIdx.x];
  const uint32_t e = a.aitem_pair[item], chunk = a.aitem_chunk[item];
  const uint32_t nck = a.pair_nck[e];
  const uint32_t gt = a.act_tile[e];
  const uint32_t a_beg = a.act_beg[gt];
  const int n_at = (int)(a.act_beg[gt + 1] - a_beg);
  const int jsel = (int)(e - a_beg);
  const int tid = threadIdx.x;
  for (int c = 0; c < NACC; ++c) B.acc[c][tid] = 0.0f;
  const PixSetup P = pixel_setup(a, gt, tid);
  const int v = P.v, bx = P.bx, by = P.by;
  const bool valid = P.valid;
  const float3 d = P.d;
  const int K = a.K;
  const float invK = 1.0f / (float)K;
  uint32_t n_test = 0, n_piece = 0;
  const PixGrad g = pixel_grads<NORMALS>(a, P);
  const float3 GC = g.GC, GN = g.GN;
  const float GD = g.GD;
  const uint32_t seg0 = 3 * a_beg + n_at;
  const int nseg = valid ? (int)a.pix_nseg[P.pix] : 0;

  // ---------------------------------------------------- B2: actor jsel
  for (int j = jsel; j == jsel; ++j) {
    // first and last spliced segment of slot j (once the last is done the
    // lane has nothing left in this list)
    int qf, q, qlast;
    const int nj = segs_of_actor_b(a, seg0, nseg, j, tid, qf, q, qlast);
    const bool simple = nck > 1 && nj == 1;
    bool has = q < nseg && (nck == 1 || simple || chunk == 0);
    if (!__syncthreads_or(has)) continue;
    const bool any_full = __syncthreads_or(has && nck > 1 && !simple);
    const uint32_t koct = a.act_oct[a_beg + j];
    const VOConst& C = a.vo[v * a.n_oct + koct];
    const float3 dj = mat3_mul(C.Rt, d);
    const float3 inv = safe_inv(dj);
    // Vq/Pl: segment total and prefix; VqT/PlT: their tail parts
    float qs = 0, qe = 0, Tpre = 0, Saft = 0, Vq = 0, VqT = 0, Tl = 1.0f;
    float Pl = 0.0f, PlT = 0.0f;
    bool qdone = false;
    float3 go = make_float3(0, 0, 0), gd = make_float3(0, 0, 0);
    auto load_q = [&](int qq) {
      const size_t qi = seg_index(seg0 + qq, tid);
      const float2 se = a.seg_se[qi];
      const float4 bw = a.seg_bw[qi];
      qs = se.x; qe = se.y; Tpre = bw.x; Saft = bw.y;
      if (simple) {
        // this chunk of the segment: its totals, tails and surroundings
        const size_t sl = ((size_t)a.pair_pbase[e] + chunk) * TPB + tid;
        const float4* part = a.apart + sl * 4;
        const float2 wr = a.atps[sl];
        Vq = gdot(g, part[0], part[1]);
        VqT = gdot(g, part[2], part[3]);
        Saft = fmaf(Tpre, wr.y, Saft);
        Tpre *= wr.x;
      } else {
        Vq = gdot(g, a.seg_p0[qi], a.seg_p1[qi]);
        VqT = gdot(g, a.seg_t0[qi], a.seg_t1[qi]);
      }
      Tl = 1.0f; Pl = 0.0f; PlT = 0.0f; qdone = false;
    };
    auto next_q = [&](int from) {
      for (int i = from; i < nseg; ++i) {
        const size_t qi = seg_index(seg0 + i, tid);
        if ((int)(a.seg_meta[qi] & 0xFF) == j && a.seg_bw[qi].x >= 0.0f) return i;
      }
      return nseg;
    };
    if (has) load_q(q);
    // a lane whose chord reached past its single segment is finished (fast
    // path below)
    bool fin = false;
    auto live = [&]() { return has && !fin && !(qdone && q == qlast); };
    const uint2 sub = a.act_sub[a_beg + j];
    uint32_t cb = sub.x, ce = sub.y;
    if (nck > 1) chunk_range(sub.x, sub.y, nck, chunk, cb, ce);
    // entries this lane walks, and the block's loop range
    const uint32_t wlo = simple ? cb : sub.x, whi = simple ? ce : sub.y;
    const uint32_t lo = any_full ? sub.x : cb, hi = any_full ? sub.y : ce;
    // waves in which no ray has several segments of this actor walk without
    // segment advances (as in the forward); their end-point derivatives on
    // the segment (one piece each) are kept in registers until the end
    const bool single = __ballot(nj > 1) == 0;
    float bz = 0.0f, bw_ = 0.0f;
    bool hz = false, hw = false;
    // gradients of the piece [pa, pb) of entry r in segment q (chord
    // [t0, t1) entering and leaving through axes ax0, ax1)
    // set: the gradients replace dcol/dnrm/dg (one piece per entry) rather
    // than adding to them; real = false: the empty piece a = b = 0 of a
    // lane without one (tau = 0 changes no state; dL/dtau is taken as 0, so
    // every gradient and pose term is zero)
    auto piece = [&](uint32_t r, const float4& geo, float t0, float t1, int ax0,
                     int ax1, float pa, float pb, float3& dcol, float3& dnrm,
                     float* dg, bool set, bool real) {
      const float4 cn = B.cn[r];
      PieceDer pd;
      const float tau = piece_eval<2, KC>(geo, B.ga[r], B.gb[r], cn.w, dj, pa,
                                          pb, K, invK, a.c, a.inv_c, &pd);
      n_piece += real ? 1u : 0u;
      const float e = fast_exp(-tau);
      const float wl = Tl * opacity(tau, e);
      const float4 nr = B.nrm[r];
      const float mid = 0.5f * (pa + pb);
      float vi = GC.x * cn.x + GC.y * cn.y + GC.z * cn.z + GD * mid;
      if (NORMALS) vi += GN.x * nr.x + GN.y * nr.y + GN.z * nr.z;
      const float wlt = Tl < T_REBASE ? wl : 0.0f;
      Pl = fmaf(wl, vi, Pl);
      PlT = fmaf(wlt, vi, PlT);
      Tl *= e;
      const float Sl = Tl < T_REBASE ? VqT - PlT : Vq - Pl;
      const float dtau = real ? Tpre * Tl * vi - (Tpre * Sl + Saft) : 0.0f;
      const float wt = Tpre * wl;
      if (set) {
        dcol = make_float3(wt * GC.x, wt * GC.y, wt * GC.z);
        if (NORMALS) dnrm = make_float3(wt * GN.x, wt * GN.y, wt * GN.z);
        set_corner_grads<KC>(pd, dtau, dg);
      } else {
        dcol.x += wt * GC.x; dcol.y += wt * GC.y; dcol.z += wt * GC.z;
        if (NORMALS) {
          dnrm.x += wt * GN.x; dnrm.y += wt * GN.y; dnrm.z += wt * GN.z;
        }
        add_corner_grads<KC>(pd, dtau, dg);
      }
      if (a.pose_grad) {
        go.x = fmaf(dtau, pd.dx.x, go.x);
        go.y = fmaf(dtau, pd.dx.y, go.y);
        go.z = fmaf(dtau, pd.dx.z, go.z);
        gd.x = fmaf(dtau, pd.dxt.x, gd.x);
        gd.y = fmaf(dtau, pd.dxt.y, gd.y);
        gd.z = fmaf(dtau, pd.dxt.z, gd.z);
        const float ga_ = dtau * pd.dtda + 0.5f * wt * GD;
        const float gb_ = dtau * pd.dtdb + 0.5f * wt * GD;
        if (qs > t0) {
          if (single) { bz += ga_; hz = hz || real; }
          else a.seg_bw[seg_index(seg0 + q, tid)].z += ga_;
        } else {
          // entry face on axis ax0: t = (face - o) / d, so divide by d
          // (times the reciprocal direction the slab test uses)
          const float u = real ? ga_ * get_axis(inv, ax0) : 0.0f;
          add_axis(go, ax0, -u);
          add_axis(gd, ax0, -u * pa);
        }
        if (qe < t1) {
          if (single) { bw_ += gb_; hw = hw || real; }
          else a.seg_bw[seg_index(seg0 + q, tid)].w += gb_;
        } else {
          const float u = real ? gb_ * get_axis(inv, ax1) : 0.0f;
          add_axis(go, ax1, -u);
          add_axis(gd, ax1, -u * pb);
        }
      }
      if (Tl < a.eps) qdone = true;
    };
    for (uint32_t base = lo; base < hi; base += TPB) {
      const uint32_t nb = min((uint32_t)TPB, hi - base);
      load_bwd_batch<NORMALS>(B, a, base, nb);
      __syncthreads();
      uint64_t wm[4];
      const uint64_t lv = __ballot(live());
      wave_live_masks(B.rect, nb, bx, by, lv, wm);
      if (single && sparse_cover(B.rect, nb, bx, by, lv, wm)) {
        // entries cover few of the wave's pixels (far actors): every lane
        // walks its own entries, those whose rectangle holds its pixel, and
        // adds its gradients to the entry's slot itself
        uint64_t pm[4];
        lane_masks(B.rect, wm, P.px, P.py, pm);
        for (int wc = 0; wc < 4; ++wc) {
          uint64_t m = pm[wc];
          while (__ballot(m != 0 && live()) != 0) {
            // a lane without an entry reads slot 0 (loaded) and takes the
            // empty piece
            const uint32_t r =
                m != 0 ? (uint32_t)wc * 64 + (uint32_t)__builtin_ctzll(m) : 0u;
            const bool own = m != 0;
            m &= m - 1;
            const bool act = own && live() && base + r >= wlo && base + r < whi;
            const float4 geo = B.geo[r];
            float t0, t1;
            int ax0, ax1;
            float3 hi;
            if (NORMALS) {
              hi = leaf_hi(geo);
            } else {
              const float4 h4 = B.nrm[r];
              hi = make_float3(h4.x, h4.y, h4.z);
            }
            slab_axes(make_float3(geo.x, geo.y, geo.z), hi, inv, t0, t1, ax0, ax1);
            n_test += act ? 1u : 0u;
            const float pa0 = fmaxf(t0, qs), pb0 = fminf(t1, qe);
            const bool hit = act && pb0 > pa0;
            if (act && t1 > t0 && t1 > qs && (qe <= t0 || t1 > qe)) fin = true;
            if (__ballot(hit) == 0) continue;
            const float pa = hit ? pa0 : 0.0f, pb = hit ? pb0 : 0.0f;
            float3 dcol, dnrm = make_float3(0, 0, 0);
            float dg[8];
            piece(r, geo, t0, t1, ax0, ax1, pa, pb, dcol, dnrm, dg, true, hit);
            if (hit) lane_record<NORMALS>(B, r, dcol, dnrm, dg);
          }
        }
      } else {
      for (int wc = 0; wc < 4; ++wc) {
      uint64_t m = wm[wc];
      if (single) {
        // one piece per entry at most: straight-line code, lanes without a
        // piece take the empty one
        while (m != 0 && __ballot(live()) != 0) {
          const uint32_t r = (uint32_t)wc * 64 + (uint32_t)__builtin_ctzll(m);
          m &= m - 1;
          const bool act = live() && base + r >= wlo && base + r < whi;
          const float4 geo = B.geo[r];
          float t0, t1;
          int ax0, ax1;
          float3 hi;
          if (NORMALS) {
            hi = leaf_hi(geo);
          } else {
            const float4 h4 = B.nrm[r];
            hi = make_float3(h4.x, h4.y, h4.z);
          }
          slab_axes(make_float3(geo.x, geo.y, geo.z), hi, inv, t0, t1, ax0, ax1);
          n_test += act ? 1u : 0u;
          const float pa0 = fmaxf(t0, qs), pb0 = fminf(t1, qe);
          const bool hit = act && pb0 > pa0;
          if (act && t1 > t0 && t1 > qs && (qe <= t0 || t1 > qe)) fin = true;
          if (__ballot(hit) == 0) continue;
          const float pa = hit ? pa0 : 0.0f, pb = hit ? pb0 : 0.0f;
          float3 dcol, dnrm = make_float3(0, 0, 0);
          float dg[8];
          piece(r, geo, t0, t1, ax0, ax1, pa, pb, dcol, dnrm, dg, true, hit);
          accum_record<NORMALS>(B, r, hit, dcol, dnrm, dg);
        }
        continue;
      }
      while (m != 0 && __ballot(live()) != 0) {
        const uint32_t r = (uint32_t)wc * 64 + (uint32_t)__builtin_ctzll(m);
        m &= m - 1;
        float3 dcol = make_float3(0, 0, 0), dnrm = make_float3(0, 0, 0);
        float dg[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        bool hit = false;
        if (live() && base + r >= wlo && base + r < whi) {
          const float4 geo = B.geo[r];
          float t0, t1;
          int ax0, ax1;
          float3 hi;
          if (NORMALS) {
            hi = leaf_hi(geo);
          } else {
            const float4 h4 = B.nrm[r];
            hi = make_float3(h4.x, h4.y, h4.z);
          }
          slab_axes(make_float3(geo.x, geo.y, geo.z), hi, inv, t0, t1, ax0, ax1);
          ++n_test;
          if (t1 > t0 && t1 > qs) {
            while (true) {
              if (qe <= t0) {
                q = next_q(q + 1);
                if (q >= nseg) { has = false; break; }
                load_q(q);
                continue;
              }
              const float pa = fmaxf(t0, qs), pb = fminf(t1, qe);
              if (pb > pa && !qdone) {
                piece(r, geo, t0, t1, ax0, ax1, pa, pb, dcol, dnrm, dg, false, true);
                hit = true;
              }
              if (t1 > qe) { qe = t0; continue; }
              break;
            }
          }
        }
        accum_record<NORMALS>(B, r, hit, dcol, dnrm, dg);
      }
      }
      }
      flush_batch(B, a, nb);
      if (!__syncthreads_or(live())) break;
    }
    if (hz || hw) {
      float4* sb = a.seg_bw + seg_index(seg0 + q, tid);
      if (hz) sb->z += bz;
      if (hw) sb->w += bw_;
    }
    if (a.pose_grad) {
      float p12[12];
      pose12(C, d, go, gd, p12);
      block_add12(red, p12,
                  a.pose_grad + ((size_t)v * a.n_actors + (koct - 1)) * 12);
    }
  }

  count_work(a.counters, 6, n_test, n_piece);

}

// Backward, part 4 (tiles with actor boxes, after every part 3 block): the
// box faces that bound segments, from the end-point derivatives gathered on
// the segments, into the pose gradients.
template <bool NORMALS>
__global__ void __launch_bounds__(TPB) k_box_bwd(CompArgs a) {
  __shared__ float red[(TPB / 64) * 12];
  const uint32_t gt = blockIdx.x;
  const uint32_t a_beg = a.act_beg[gt];
  const int n_at = (int)(a.act_beg[gt + 1] - a_beg);
  if (n_at == 0 || !a.pose_grad) return;
  const int tid = threadIdx.x;
  const PixSetup P = pixel_setup(a, gt, tid);
  const int v = P.v;
  const float3 d = P.d;
  const uint32_t seg0 = 3 * a_beg + n_at;
  const int nseg = P.valid ? (int)a.pix_nseg[P.pix] : 0;
  // ---------------------------------------------------- B3: box faces
  if (a.pose_grad) {
    for (int j = 0; j < n_at; ++j) {
      const uint32_t koct = a.act_oct[a_beg + j];
      const VOConst& C = a.vo[v * a.n_oct + koct];
      const float3 dj = mat3_mul(C.Rt, d);
      const float3 inv = safe_inv(dj);
      float3 go = make_float3(0, 0, 0), gd = make_float3(0, 0, 0);
      bool any = false;
      for (int q = 0; q < nseg; ++q) {
        const size_t qi = seg_index(seg0 + q, tid);
        const float4 bw = a.seg_bw[qi];
        if (bw.x < 0.0f) continue;
        const uint32_t meta = a.seg_meta[qi];
        const float2 se = a.seg_se[qi];
        const uint32_t ss = (meta >> 8) & 0x3FF, se_ = (meta >> 18) & 0x3FF;
        if (ss != SRC_NONE && (int)(ss >> 2) == j && bw.z != 0.0f) {
          const int ax = ss & 3;
          const float u = bw.z * get_axis(inv, ax);
          add_axis(go, ax, -u);
          add_axis(gd, ax, -u * se.x);
          any = true;
        }
        if (se_ != SRC_NONE && (int)(se_ >> 2) == j && bw.w != 0.0f) {
          const int ax = se_ & 3;
          const float u = bw.w * get_axis(inv, ax);
          add_axis(go, ax, -u);
          add_axis(gd, ax, -u * se.y);
          any = true;
        }
      }
      if (!__syncthreads_or(any)) continue;
      float p12[12];
      pose12(C, d, go, gd, p12);
      block_add12(red, p12,
                  a.pose_grad + ((size_t)v * a.n_actors + (koct - 1)) * 12);
    }
  }
}

// ------------------------------------------------------------------ records
// A record's normal gradient dL/dn (world) in terms of its 8 corner
// values: n = -grad/|grad| of the trilinear field at the leaf centre, so
// dL/dg_m = (s_m . dv) with dv = -(I - n n^T) R^T dL/dn / |grad| and s_m the
// corner's +-1/4 stencil.  Adds to dg; returns false (nothing added) where
// the gradient or the normal vanishes; nl: the local normal.
__device__ inline bool normal_to_corners(float4 gn, float4 ga, float4 gb,
                                         const float* R, float* dg, float* nl) {
  if (gn.x == 0.0f && gn.y == 0.0f && gn.z == 0.0f) return false;
  const float g[8] = {ga.x, ga.y, ga.z, ga.w, gb.x, gb.y, gb.z, gb.w};
  const float vx = 0.25f * ((g[1] - g[0]) + (g[3] - g[2]) + (g[5] - g[4]) + (g[7] - g[6]));
  const float vy = 0.25f * ((g[2] - g[0]) + (g[3] - g[1]) + (g[6] - g[4]) + (g[7] - g[5]));
  const float vz = 0.25f * ((g[4] - g[0]) + (g[5] - g[1]) + (g[6] - g[2]) + (g[7] - g[3]));
  const float nv = sqrtf(vx * vx + vy * vy + vz * vz);
  if (!(nv > 0.0f)) return false;
  nl[0] = -vx / nv; nl[1] = -vy / nv; nl[2] = -vz / nv;
  // dL/dn_loc = R^T dL/dn_world
  float dn[3];
  for (int a2 = 0; a2 < 3; ++a2)
    dn[a2] = R[0 * 3 + a2] * gn.x + R[1 * 3 + a2] * gn.y + R[2 * 3 + a2] * gn.z;
  const float pr = dn[0] * nl[0] + dn[1] * nl[1] + dn[2] * nl[2];
  const float dv[3] = {-(dn[0] - pr * nl[0]) / nv, -(dn[1] - pr * nl[1]) / nv,
                       -(dn[2] - pr * nl[2]) / nv};
  for (int m = 0; m < 8; ++m) {
    const float sx = (m & 1) ? 0.25f : -0.25f;
    const float sy = (m & 2) ? 0.25f : -0.25f;
    const float sz = (m & 4) ? 0.25f : -0.25f;
    dg[m] += sx * dv[0] + sy * dv[1] + sz * dv[2];
  }
  return true;
}

// SH gradient of one record, added to the [S][3][N] accumulator by plain
// read-modify-write (the caller guarantees one record per leaf and launch);
// all loads of a channel are issued before its stores.
template <int S>
__device__ inline void sh_grad_rmw(float* gsh, int N, uint32_t vox,
                                   const float* Y, const float* mc) {
  const int64_t N3 = 3 * (int64_t)N;
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) {
    if (mc[ch] == 0.0f) continue;
    float* gp = gsh + (int64_t)ch * N + vox;
    float old[S];
#pragma unroll
    for (int q = 0; q < S; ++q) old[q] = gp[q * N3];
#pragma unroll
    for (int q = 0; q < S; ++q) gp[q * N3] = old[q] + Y[q] * mc[ch];
  }
}

// SH and corner gradients, leaf-major (renders with several records per
// leaf): one thread per (octree, leaf) walks the views, finds the leaf's
// record (if the leaf was visible) from the preprocess ballots — slot =
// block offset + ballots of the block's earlier waves + lanes below in the
// wave's ballot — and sums over its records, in registers, Y(dir) dL/dc
// and the 8 corner gradients (density samples, plus the normal's terms);
// then one read-modify-write of the [S][3][N] SH accumulator, coalesced
// over consecutive leaves, and 8 corner atomics per leaf instead of per
// record.  Leaves of octree k occupy threads [lstart[k], lstart[k] + N_k),
// lstart 64-aligned, so a wave holds one octree and its lanes share every
// ballot word.
struct ShArgs {
  const int64_t* lstart;   // [n_oct + 1]
  const int64_t* pstart;   // per (view, octree): first item, 64-aligned
  const int32_t* seg_len;  // per (view, octree): leaves binned (0: none)
  const uint64_t* wmask;   // per wave of items: visibility ballot
  const uint32_t* boff;    // per block of items: first record slot
  const float4* gcol;      // per record: dL/d colour
  const float4* rcn;       // per record: colour
  const float4* rgeo;      // per record: leaf min relative to the camera, h
  const float4* gg8a;      // per record: dL/d corner values
  const float4* gg8b;
  const float4* gnrm;      // per record: dL/d normal (normals rendered)
  const float4* rg8a;      // per record: corner values
  const float4* rg8b;
  const VOConst* vo;
  const OctDev* oct;
  const OctGrad* og;
  int32_t n_oct, n_views;
  bool normals;
};

// Visibility ballots of views [v0, v0 + LB_VB) for the wave of leaves
// x0.. of octree k (0 where the leaf set is not binned in a view), and for
// each visible view the record slot of the wave's first visible lane.  The
// loads of the LB_VB views are independent, so they are in flight together
// rather than one dependent chain per view.
constexpr int LB_VB = 8;
__device__ inline void leaf_view_slots(const ShArgs& p, int k, int64_t x0, int v0,
                                       uint64_t m[LB_VB], uint32_t base[LB_VB]) {
  int64_t item0[LB_VB];
  bool ok[LB_VB];
#pragma unroll
  for (int j = 0; j < LB_VB; ++j) {
    const int v = v0 + j;
    const int sg = min(v, p.n_views - 1) * p.n_oct + k;
    ok[j] = v < p.n_views && p.seg_len[sg] != 0;
    item0[j] = p.pstart[sg] + x0;
  }
#pragma unroll
  for (int j = 0; j < LB_VB; ++j) m[j] = ok[j] ? p.wmask[item0[j] >> 6] : 0ull;
#pragma unroll
  for (int j = 0; j < LB_VB; ++j) {
    base[j] = 0;
    if (m[j] != 0) {
      const int64_t blk = item0[j] / TPB;
      const int wib = (int)((item0[j] >> 6) % (TPB / 64));
      uint32_t b = p.boff[blk];
      for (int i = 0; i < wib; ++i)
        b += (uint32_t)__popcll(p.wmask[blk * (TPB / 64) + i]);
      base[j] = b;
    }
  }
}

template <int S>
__device__ inline void sh_leaf(const ShArgs& p, int k, int64_t x0, int lane,
                               int N, int deg, float* gsh, float* gcor,
                               const int32_t* cidx) {
  const int64_t x = x0 + lane;
  const bool in = x < N;
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  float acc[3][S];
#pragma unroll
  for (int ch = 0; ch < 3; ++ch)
#pragma unroll
    for (int q = 0; q < S; ++q) acc[ch][q] = 0.0f;
  float dgs[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  bool any = false, anyc = false;
  for (int v0 = 0; v0 < p.n_views; v0 += LB_VB) {
  uint64_t mv[LB_VB];
  uint32_t bv[LB_VB];
  leaf_view_slots(p, k, x0, v0, mv, bv);
#pragma unroll
  for (int j = 0; j < LB_VB; ++j) {
    const uint64_t m = mv[j];
    if (m == 0) continue;
    const int sg = (v0 + j) * p.n_oct + k;
    if (!in || !((m >> lane) & 1ull)) continue;
    const uint32_t slot = bv[j] + (uint32_t)__popcll(m & lt);
    if (gcor) {
      const float4 a8 = p.gg8a[slot], b8 = p.gg8b[slot];
      float dg[8] = {a8.x, a8.y, a8.z, a8.w, b8.x, b8.y, b8.z, b8.w};
      float nl[3];
      if (p.normals)
        normal_to_corners(p.gnrm[slot], p.rg8a[slot], p.rg8b[slot],
                          p.vo[sg].R, dg, nl);
#pragma unroll
      for (int c8 = 0; c8 < 8; ++c8) {
        dgs[c8] += dg[c8];
        anyc = anyc || dg[c8] != 0.0f;
      }
    }
    if (!gsh) continue;
    const float4 dc = p.gcol[slot], cn = p.rcn[slot], geo = p.rgeo[slot];
    const float mc[3] = {cn.x > 0.0f ? dc.x : 0.0f, cn.y > 0.0f ? dc.y : 0.0f,
                         cn.z > 0.0f ? dc.z : 0.0f};
    if (mc[0] == 0.0f && mc[1] == 0.0f && mc[2] == 0.0f) continue;
    // direction camera -> leaf centre (octree frame)
    const float cx = geo.x + 0.5f * geo.w, cy = geo.y + 0.5f * geo.w,
                cz = geo.z + 0.5f * geo.w;
    const float rn = sqrtf(cx * cx + cy * cy + cz * cz);
    const float ir = rn > 0.0f ? 1.0f / rn : 0.0f;
    float Y[16];
    sh_basis(deg, cx * ir, cy * ir, cz * ir, Y);
#pragma unroll
    for (int ch = 0; ch < 3; ++ch)
#pragma unroll
      for (int q = 0; q < S; ++q) acc[ch][q] = fmaf(Y[q], mc[ch], acc[ch][q]);
    any = true;
  }
  }
  if (anyc) {
    int32_t ci[8];
#pragma unroll
    for (int c8 = 0; c8 < 8; ++c8) ci[c8] = cidx[(int64_t)c8 * N + x];
#pragma unroll
    for (int c8 = 0; c8 < 8; ++c8) atomicAdd(gcor + ci[c8], dgs[c8]);
  }
  if (!any) return;
  const int64_t N3 = 3 * (int64_t)N;
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) {
    float* gp = gsh + (int64_t)ch * N + x;
    float old[S];
#pragma unroll
    for (int q = 0; q < S; ++q) old[q] = gp[q * N3];
#pragma unroll
    for (int q = 0; q < S; ++q) gp[q * N3] = old[q] + acc[ch][q];
  }
}

// Feature renders, leaf-major: the leaf's colour-slot gradients summed
// over its records are its feature gradient (no basis, no clamp).
__device__ inline void feat_leaf(const ShArgs& p, int k, int64_t x0, int lane,
                                 int N, float* gf, int nc, float* gcor,
                                 const int32_t* cidx) {
  const int64_t x = x0 + lane;
  const bool in = x < N;
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  float acc[3] = {0.0f, 0.0f, 0.0f};
  float dgs[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  bool any = false, anyc = false;
  for (int v0 = 0; v0 < p.n_views; v0 += LB_VB) {
  uint64_t mv[LB_VB];
  uint32_t bv[LB_VB];
  leaf_view_slots(p, k, x0, v0, mv, bv);
#pragma unroll
  for (int j = 0; j < LB_VB; ++j) {
    const uint64_t m = mv[j];
    if (m == 0) continue;
    const int sg = (v0 + j) * p.n_oct + k;
    if (!in || !((m >> lane) & 1ull)) continue;
    const uint32_t slot = bv[j] + (uint32_t)__popcll(m & lt);
    if (gcor) {
      const float4 a8 = p.gg8a[slot], b8 = p.gg8b[slot];
      float dg[8] = {a8.x, a8.y, a8.z, a8.w, b8.x, b8.y, b8.z, b8.w};
      float nl[3];
      if (p.normals)
        normal_to_corners(p.gnrm[slot], p.rg8a[slot], p.rg8b[slot],
                          p.vo[sg].R, dg, nl);
#pragma unroll
      for (int c8 = 0; c8 < 8; ++c8) {
        dgs[c8] += dg[c8];
        anyc = anyc || dg[c8] != 0.0f;
      }
    }
    if (!gf) continue;
    const float4 dc = p.gcol[slot];
    acc[0] += dc.x;
    acc[1] += dc.y;
    acc[2] += dc.z;
    any = any || dc.x != 0.0f || dc.y != 0.0f || dc.z != 0.0f;
  }
  }
  if (anyc) {
    int32_t ci[8];
#pragma unroll
    for (int c8 = 0; c8 < 8; ++c8) ci[c8] = cidx[(int64_t)c8 * N + x];
#pragma unroll
    for (int c8 = 0; c8 < 8; ++c8) atomicAdd(gcor + ci[c8], dgs[c8]);
  }
  if (!any) return;
  float old[3];
  for (int ch = 0; ch < nc; ++ch) old[ch] = gf[(int64_t)ch * N + x];
  for (int ch = 0; ch < nc; ++ch) gf[(int64_t)ch * N + x] = old[ch] + acc[ch];
}

__global__ void __launch_bounds__(TPB) k_leaf_bwd(ShArgs p) {
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t t0 = (int64_t)blockIdx.x * TPB + w * 64;
  if (t0 >= p.lstart[p.n_oct]) return;
  int lo = 0, hi = p.n_oct - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (p.lstart[mid] <= t0) lo = mid; else hi = mid - 1;
  }
  const int k = lo;
  const OctDev& O = p.oct[k];
  float* const gsh = p.og[k].sh;
  float* const gcor = p.og[k].corner;
  float* const gf = p.og[k].feat;
  const int fnc = p.og[k].feat_nc;
  if (!gsh && !gcor && !gf) return;
  const int64_t x0 = t0 - p.lstart[k];
  const int N = O.n_vox;
  if (x0 >= N) return;
  const int32_t* const cidx = O.corner_idx;
  if (fnc > 0) {
    feat_leaf(p, k, x0, lane, N, gf, fnc, gcor, cidx);
    return;
  }
  switch (O.sh_degree) {
    case 0: sh_leaf<1>(p, k, x0, lane, N, 0, gsh, gcor, cidx); break;
    case 1: sh_leaf<4>(p, k, x0, lane, N, 1, gsh, gcor, cidx); break;
    case 2: sh_leaf<9>(p, k, x0, lane, N, 2, gsh, gcor, cidx); break;
    default: sh_leaf<16>(p, k, x0, lane, N, 3, gsh, gcor, cidx); break;
  }
}

template <bool POSE>
__global__ void __launch_bounds__(TPB)
k_record_bwd(int64_t off, int64_t n, const uint32_t* rseg, const uint32_t* rvox,
             const float4* rgeo, const float4* rcn, const float4* rg8a,
             const float4* rg8b, const float4* gcol, const float4* gnrm,
             const float4* gg8a, const float4* gg8b, const OctDev* oct,
             const OctGrad* og, const VOConst* vo, int n_oct, int n_actors,
             float* pose_grad, bool normals, bool leafmajor) {
  const int64_t i = off + (int64_t)blockIdx.x * TPB + threadIdx.x;
  float p12[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) p12[c] = 0.0f;
  uint32_t seg = 0xFFFFFFFFu;
  if (i < n) seg = rseg[i];
  // leaf-major launches add pose terms only: background records have none
  if (i < n && !(leafmajor && seg % n_oct == 0)) {
    const int k = (int)(seg % n_oct);
    const OctDev& O = oct[k];
    const OctGrad& G = og[k];
    const VOConst& C = vo[seg];
    const uint32_t vox = rvox[i];
    const int N = O.n_vox;
    const float4 dc = gcol[i];
    const float4 cn = rcn[i];
    const float4 geo = rgeo[i];
    // direction camera -> leaf centre (octree frame)
    const float cx = geo.x + 0.5f * geo.w, cy = geo.y + 0.5f * geo.w,
                cz = geo.z + 0.5f * geo.w;
    const float rn = sqrtf(cx * cx + cy * cy + cz * cz);
    const float ir = rn > 0.0f ? 1.0f / rn : 0.0f;
    const float wx = cx * ir, wy = cy * ir, wz = cz * ir;
    const bool featm = G.feat_nc > 0;
    // colour clamped at 0 (subgradient 0 there); features are not clamped
    const float mc[3] = {featm || cn.x > 0.0f ? dc.x : 0.0f,
                         featm || cn.y > 0.0f ? dc.y : 0.0f,
                         featm || cn.z > 0.0f ? dc.z : 0.0f};
    const int S = (O.sh_degree + 1) * (O.sh_degree + 1);
    float* const gsh = leafmajor ? nullptr : G.sh;
    float* const gcor = leafmajor ? nullptr : G.corner;
    const int32_t* const cidx = O.corner_idx;
    if (featm && G.feat && !leafmajor) {
      // one record per leaf in this launch: plain read-modify-write
      float old[3];
      for (int ch = 0; ch < G.feat_nc; ++ch) old[ch] = G.feat[(int64_t)ch * N + vox];
      for (int ch = 0; ch < G.feat_nc; ++ch)
        if (mc[ch] != 0.0f) G.feat[(int64_t)ch * N + vox] = old[ch] + mc[ch];
    }
    if (!featm && gsh && (mc[0] != 0.0f || mc[1] != 0.0f || mc[2] != 0.0f)) {
      float Y[16];
      sh_basis(O.sh_degree, wx, wy, wz, Y);
      // one launch covers the records of one view, where a leaf has at most
      // one record: plain read-modify-write, coalesced over consecutive leaves
      switch (O.sh_degree) {
        case 0: sh_grad_rmw<1>(gsh, N, vox, Y, mc); break;
        case 1: sh_grad_rmw<4>(gsh, N, vox, Y, mc); break;
        case 2: sh_grad_rmw<9>(gsh, N, vox, Y, mc); break;
        default: sh_grad_rmw<16>(gsh, N, vox, Y, mc); break;
      }
    }
    if (POSE && k > 0 && !featm &&
        (mc[0] != 0.0f || mc[1] != 0.0f || mc[2] != 0.0f)) {
      float gx[16], gy[16], gz[16];
      sh_basis_grad(O.sh_degree, wx, wy, wz, gx, gy, gz);
      float dw[3] = {0, 0, 0};
      for (int q = 0; q < S; ++q) {
        float s = 0.0f;
        for (int ch = 0; ch < 3; ++ch)
          s = fmaf(mc[ch], O.sh[((int64_t)q * 3 + ch) * N + vox], s);
        dw[0] = fmaf(s, gx[q], dw[0]);
        dw[1] = fmaf(s, gy[q], dw[1]);
        dw[2] = fmaf(s, gz[q], dw[2]);
      }
      // w = (c - P) / |c - P|:  dL/dP = -(I - w w^T) dw / |c - P|
      const float pr = dw[0] * wx + dw[1] * wy + dw[2] * wz;
      const float dP[3] = {-(dw[0] - pr * wx) * ir, -(dw[1] - pr * wy) * ir,
                           -(dw[2] - pr * wz) * ir};
      for (int b = 0; b < 3; ++b)
        for (int a2 = 0; a2 < 3; ++a2) p12[b * 3 + a2] += C.omp[b] * dP[a2];
      for (int b = 0; b < 3; ++b)
        p12[9 + b] -= C.R[b * 3 + 0] * dP[0] + C.R[b * 3 + 1] * dP[1] +
                      C.R[b * 3 + 2] * dP[2];
    }
    // corners: density samples plus the normal's dependence
    const float4 a8 = gg8a[i], b8 = gg8b[i];
    float dg[8] = {a8.x, a8.y, a8.z, a8.w, b8.x, b8.y, b8.z, b8.w};
    if (normals) {
      float nl[3];
      if (normal_to_corners(gnrm[i], rg8a[i], rg8b[i], C.R, dg, nl) && POSE &&
          k > 0) {
        const float4 gn = gnrm[i];
        const float gw[3] = {gn.x, gn.y, gn.z};
        for (int a2 = 0; a2 < 3; ++a2)
          for (int b = 0; b < 3; ++b) p12[a2 * 3 + b] += gw[a2] * nl[b];
      }
    }
    if (gcor && (dg[0] != 0.0f || dg[1] != 0.0f || dg[2] != 0.0f ||
                     dg[3] != 0.0f || dg[4] != 0.0f || dg[5] != 0.0f ||
                     dg[6] != 0.0f || dg[7] != 0.0f)) {
      int32_t ci[8];
#pragma unroll
      for (int m = 0; m < 8; ++m) ci[m] = cidx[(int64_t)m * N + vox];
#pragma unroll
      for (int m = 0; m < 8; ++m) atomicAdd(gcor + ci[m], dg[m]);
    }
  }
  if (!POSE) return;
  // pose: wave-reduce when the whole wave shares one (view, actor)
  const int lane = threadIdx.x & 63;
  const uint32_t s0 = __shfl(seg, 0, 64);
  const bool same = __ballot(seg != s0) == 0;
  if (same) {
    if (s0 == 0xFFFFFFFFu || (int)(s0 % n_oct) == 0) return;
    int slot;
    bool pad;
    const float x = wave_sum12(p12, slot, pad);
    if ((lane & 3) == 0 && !pad && x != 0.0f) {
      const int v = s0 / n_oct, k = s0 % n_oct;
      atomicAdd(pose_grad + ((size_t)v * n_actors + (k - 1)) * 12 + slot, x);
    }
  } else if (seg != 0xFFFFFFFFu && (int)(seg % n_oct) > 0) {
    const int v = seg / n_oct, k = seg % n_oct;
    float* dst = pose_grad + ((size_t)v * n_actors + (k - 1)) * 12;
    for (int c = 0; c < 12; ++c)
      if (p12[c] != 0.0f) atomicAdd(dst + c, p12[c]);
  }
}

}  // namespace dv

using namespace dv;

extern "C" dv_status dv_render_backward(dv_ctx* ctx, const dv_scene* scene,
                                        const dv_fwd_state* cst,
                                        const dv_out_grads* g,
                                        const dv_param_grads* acc,
                                        void* stream) {
  if (!ctx || !scene || !cst || !g || !acc || cst->scene != scene) {
    set_error("dv_render_backward: invalid arguments");
    return DV_ERR_INVALID;
  }
  if (ctx->poisoned) {
    set_error("dv_render_backward: context poisoned");
    return DV_ERR_DEVICE;
  }
  dv_fwd_state* st = const_cast<dv_fwd_state*>(cst);
  DV_TRY_HIP(hipSetDevice(ctx->device));
  PoolStamp stamp_on_return(ctx);
  reap_states(ctx, false);
  hipStream_t s = (hipStream_t)stream;
  const int64_t nv = st->n_vis, nt = st->n_tiles;
  const int n_oct = st->n_oct;
  // the normal terms of the backward (normal gradients per record, the
  // normals in the per-entry sums) run only when some view passes a normal
  // gradient; without one they are exactly zero, and the walks take the
  // kernels without normals (same forward arithmetic: the far corner the
  // slab test uses is formed from the leaf corner either way)
  bool normals = false;
  if (st->opts.out_mask & DV_OUT_NORMAL)
    for (int v = 0; v < st->n_views; ++v) normals = normals || g[v].normal != nullptr;
  // per-view upstream gradients and per-octree accumulators
  st->grads_keep.emplace_back(g, g + st->n_views);
  st->og_keep.emplace_back(n_oct);
  std::vector<OctGrad>& og = st->og_keep.back();
  for (int k = 0; k < n_oct; ++k) {
    og[k].corner = acc->octrees ? acc->octrees[k].corner : nullptr;
    og[k].sh = acc->octrees ? acc->octrees[k].sh : nullptr;
    og[k].feat = nullptr;
    og[k].feat_nc = 0;
    og[k].pad = 0;
    if (st->opts.feat) {
      // feature render: the colour gradient is the feature gradient of the
      // render's channel group; no SH term
      const int c0 = 3 * st->opts.feat_group;
      og[k].feat_nc = std::min(3, st->opts.feat_dim - c0);
      float* f = acc->octrees ? acc->octrees[k].feat : nullptr;
      og[k].feat = f ? f + (size_t)c0 * scene->desc[k].n_voxels : nullptr;
      og[k].sh = nullptr;
    }
  }
  // leaf-major thread space of the SH backward: octree k from lstart[k]
  st->lstart_keep.emplace_back((size_t)n_oct + 1, 0);
  std::vector<int64_t>& lstart = st->lstart_keep.back();
  for (int k = 0; k < n_oct; ++k)
    lstart[k + 1] = lstart[k] + ((scene->desc[k].n_voxels + 63) & ~(int64_t)63);
  // one upload: per-view gradient planes, per-octree accumulators, leaf
  // starts
  DBuf tabs, gin, ogd, lsd, gcol, gnrm, gg8a, gg8b, segbw;
  {
    const void* src[3] = {st->grads_keep.back().data(), og.data(), lstart.data()};
    const size_t len[3] = {sizeof(dv_out_grads) * st->n_views,
                           sizeof(OctGrad) * n_oct, sizeof(int64_t) * (n_oct + 1)};
    DBuf* dst[3] = {&gin, &ogd, &lsd};
    size_t off[3], total = 0;
    for (int i = 0; i < 3; ++i) {
      off[i] = total;
      total += (len[i] + 255) & ~(size_t)255;
    }
    DV_TRY(alloc_n<uint8_t>(ctx, tabs, total, s));
    uint8_t* stage = stage_acquire(total);
    if (!stage) return DV_ERR_OOM;
    for (int i = 0; i < 3; ++i) std::memcpy(stage + off[i], src[i], len[i]);
    DV_TRY_HIP(hipMemcpyAsync(tabs.p, stage, total, hipMemcpyHostToDevice, s));
    DV_TRY(stage_release(s));
    for (int i = 0; i < 3; ++i) dst[i]->view_of(tabs.as<uint8_t>() + off[i], len[i]);
  }
  // per-record gradients in one buffer (colour, corners, normal last, so a
  // render without normals clears three quarters of it)
  DBuf grec;
  DV_TRY(alloc_n<float4>(ctx, grec, 4 * (size_t)nv, s));
  gcol.view_of(grec.as<float4>(), sizeof(float4) * nv);
  gg8a.view_of(grec.as<float4>() + nv, sizeof(float4) * nv);
  gg8b.view_of(grec.as<float4>() + 2 * (size_t)nv, sizeof(float4) * nv);
  gnrm.view_of(grec.as<float4>() + 3 * (size_t)nv, sizeof(float4) * nv);
  StageTimer tm_clear(ctx, ST_BWD_CLEAR, s);
  DV_TRY(fill_f32(grec.as<float>(), 0.0f, (normals ? 16 : 12) * nv, s));
  const size_t nslots = (size_t)3 * st->n_apairs * TPB;
  DV_TRY(alloc_n<float4>(ctx, segbw, nslots, s));
  DBuf tps, atps;
  DV_TRY(alloc_n<float2>(ctx, tps, st->max_slots * TPB, s));
  DV_TRY(alloc_n<float2>(ctx, atps, st->max_aslots * TPB, s));
  CompArgs ca;
  std::memset(&ca, 0, sizeof(ca));
  ca.views = st->views_d.as<ViewConst>();
  ca.vo = st->vo_d.as<VOConst>();
  ca.n_views = st->n_views;
  ca.n_oct = n_oct;
  ca.tile_start = st->tile_start.as<uint32_t>();
  ca.tile_end = st->tile_end.as<uint32_t>();
  ca.tile_bgend = st->tile_bgend.as<uint32_t>();
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
  ca.seg_bw = segbw.as<float4>();
  ca.pix_nseg = st->pix_nseg.as<uint32_t>();
  ca.fin0 = st->fin0.as<float4>();
  ca.fin1 = st->fin1.as<float4>();
  ca.fin2 = st->fin2.as<float4>();
  ca.fin3 = st->fin3.as<float4>();
  ca.gin = gin.as<dv_out_grads>();
  ca.gr_col = gcol.as<float4>();
  ca.gr_nrm = gnrm.as<float4>();
  ca.gr_g8a = gg8a.as<float4>();
  ca.gr_g8b = gg8b.as<float4>();
  ca.pose_grad = st->n_actors > 0 ? acc->pose : nullptr;
  ca.n_actors = st->n_actors;
  const dv_render_opts& op = st->opts;
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
  ca.sky_grad = op.sky ? acc->sky : nullptr;
  ca.mask = op.out_mask;
  ca.counters = (ctx->prof_flags.load() & DV_PROFILE_COUNTERS) ? ctx->counters : nullptr;
  ca.item_tile = st->item_tile.as<uint32_t>();
  ca.item_chunk = st->item_chunk.as<uint32_t>();
  ca.tile_nck = st->tile_nck.as<uint32_t>();
  ca.tile_pbase = st->tile_pbase.as<uint32_t>();
  ca.plan_counts = st->plan_counts.as<uint32_t>();
  ca.chunk_b = st->chunk_b.as<float>();
  ca.chunk_part = st->chunk_part.as<float4>();
  ca.chunk_tps = tps.as<float2>();
  ca.atps = atps.as<float2>();
  // the same work items as the forward, ordered by the work each took there
  DV_TRY(alloc_n<uint32_t>(ctx, st->order_bwd, st->max_items, s));
  DV_TRY(launch_order_by_weight(ctx, st->max_items, nullptr, st->item_work.as<uint32_t>(),
                                st->order_bwd.as<uint32_t>(), s));
  ca.order = st->order_bwd.as<uint32_t>();
  ca.act_tile = st->act_tile.as<uint32_t>();
  ca.aorder = st->aorder.as<uint32_t>();
  ca.aitem_pair = st->aitem_pair.as<uint32_t>();
  ca.aitem_chunk = st->aitem_chunk.as<uint32_t>();
  ca.pair_nck = st->pair_nck.as<uint32_t>();
  ca.pair_pbase = st->pair_pbase.as<uint32_t>();
  ca.aplan_counts = st->aplan_counts.as<uint32_t>();
  ca.apart = st->apart.as<float4>();
  if (nt > 0) {
    const bool k1 = op.K == 1;
    if (st->n_apairs > 0)
      hipLaunchKernelGGL(k_seg_bw_init, dim3((unsigned)st->n_apairs), dim3(TPB), 0, s,
                         ca);
    auto kp = normals ? k_chunk_prep<true> : k_chunk_prep<false>;
    hipLaunchKernelGGL(kp, dim3((unsigned)std::min<int64_t>(st->max_slots, 16384)),
                       dim3(TPB), 0, s, ca,
                       (const uint32_t*)st->slot_tile.as<uint32_t>());
    tm_clear.stop();
    {
      StageTimer tm_comp(ctx, ST_COMPOSITE_BWD, s);
      auto kern = normals ? (k1 ? k_composite_bwd<true, 1> : k_composite_bwd<true, 0>)
                          : (k1 ? k_composite_bwd<false, 1> : k_composite_bwd<false, 0>);
      hipLaunchKernelGGL(kern, dim3((unsigned)st->max_items), dim3(TPB), 0, s, ca);
    }
    if (st->n_apairs > 0) {
      StageTimer tm_act(ctx, ST_ACTOR_BWD, s);
      auto kq = normals ? k_actor_prep<true> : k_actor_prep<false>;
      hipLaunchKernelGGL(kq, dim3((unsigned)st->n_apairs), dim3(TPB), 0, s, ca);
      auto ka = normals ? (k1 ? k_actor_bwd<true, 1> : k_actor_bwd<true, 0>)
                        : (k1 ? k_actor_bwd<false, 1> : k_actor_bwd<false, 0>);
      hipLaunchKernelGGL(ka, dim3((unsigned)st->max_aitems), dim3(TPB), 0, s, ca);
      if (ca.pose_grad) {
        auto kb = normals ? k_box_bwd<true> : k_box_bwd<false>;
        hipLaunchKernelGGL(kb, dim3((unsigned)nt), dim3(TPB), 0, s, ca);
      }
    }
    if (ca.sky_grad) {
      auto ks = normals ? k_sky_bwd<true> : k_sky_bwd<false>;
      hipLaunchKernelGGL(ks, dim3((unsigned)nt), dim3(TPB), 0, s, ca);
    }
    DV_TRY_HIP(hipGetLastError());
  }
  tm_clear.stop();
  StageTimer tm_rec(ctx, ST_RECORD_BWD, s);
  // leaf-major SH and corner sums when leaves carry several records on
  // average (several views), else one launch per view over its records
  const bool leafmajor = st->n_views > 1 && (double)nv >= 1.5 * (double)lstart[n_oct];
  if (nv > 0 && leafmajor) {
    if (ca.pose_grad) {
      hipLaunchKernelGGL(k_record_bwd<true>, dim3(grid_for(nv, TPB)), dim3(TPB), 0,
                         s, (int64_t)0, nv, st->rec_seg.as<uint32_t>(),
                         st->rec_vox.as<uint32_t>(), st->rec_geo.as<float4>(),
                         st->rec_cn.as<float4>(), st->rec_g8a.as<float4>(),
                         st->rec_g8b.as<float4>(), gcol.as<float4>(),
                         gnrm.as<float4>(), gg8a.as<float4>(), gg8b.as<float4>(),
                         scene->oct_dev.as<OctDev>(), ogd.as<OctGrad>(),
                         st->vo_d.as<VOConst>(), n_oct, st->n_actors,
                         ca.pose_grad, normals, true);
      DV_TRY_HIP(hipGetLastError());
    }
    ShArgs sa;
    sa.lstart = lsd.as<int64_t>();
    sa.pstart = st->seg_pstart_d.as<int64_t>();
    sa.seg_len = st->seg_len_d.as<int32_t>();
    sa.wmask = st->pre_wmask.as<uint64_t>();
    sa.boff = st->pre_boff.as<uint32_t>();
    sa.gcol = gcol.as<float4>();
    sa.rcn = st->rec_cn.as<float4>();
    sa.rgeo = st->rec_geo.as<float4>();
    sa.gg8a = gg8a.as<float4>();
    sa.gg8b = gg8b.as<float4>();
    sa.gnrm = gnrm.as<float4>();
    sa.rg8a = st->rec_g8a.as<float4>();
    sa.rg8b = st->rec_g8b.as<float4>();
    sa.vo = st->vo_d.as<VOConst>();
    sa.oct = scene->oct_dev.as<OctDev>();
    sa.og = ogd.as<OctGrad>();
    sa.n_oct = n_oct;
    sa.n_views = st->n_views;
    sa.normals = normals;
    hipLaunchKernelGGL(k_leaf_bwd, dim3(grid_for(lstart[n_oct], TPB)), dim3(TPB), 0,
                       s, sa);
    DV_TRY_HIP(hipGetLastError());
  }
  for (int v = 0; v < st->n_views && nv > 0 && !leafmajor; ++v) {
    const int64_t r0 = (int64_t)st->view_slot_h[v], r1 = (int64_t)st->view_slot_h[v + 1];
    if (r1 <= r0) continue;
    auto kr = ca.pose_grad ? k_record_bwd<true> : k_record_bwd<false>;
    hipLaunchKernelGGL(kr, dim3(grid_for(r1 - r0, TPB)), dim3(TPB), 0, s, r0, r1,
                       st->rec_seg.as<uint32_t>(), st->rec_vox.as<uint32_t>(),
                       st->rec_geo.as<float4>(), st->rec_cn.as<float4>(),
                       st->rec_g8a.as<float4>(), st->rec_g8b.as<float4>(),
                       gcol.as<float4>(), gnrm.as<float4>(), gg8a.as<float4>(),
                       gg8b.as<float4>(), scene->oct_dev.as<OctDev>(),
                       ogd.as<OctGrad>(), st->vo_d.as<VOConst>(), n_oct,
                       st->n_actors, ca.pose_grad, normals, false);
    DV_TRY_HIP(hipGetLastError());
  }
  return DV_OK;
}
