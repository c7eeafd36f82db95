// Structure kernels of the octrees: LiDAR-guided initialisation (Sec. 3.3,
// 'Initialization', background: proximity-based subdivision and the soft
// density prior of Eq. 1) and the structure edits of training (Sec. 3.1:
// adaptive pruning and progressive subdivision; Supp. 'Adaptive
// Optimization Schedule').
//
//  * Nearest point: the points are hashed into a uniform grid of cell
//    c = r_max / 2 (keys sorted with the library's radix sort, one hash
//    slot per occupied cell holding its [start, end) in the sorted order).
//    A query visits the cells in Chebyshev rings around its own cell and
//    stops after ring r once the best distance is at most r c (every point
//    in a later ring is at least r c away); past ring 3 every point is at
//    least 1.5 r_max away.  Distances are FP64, so the nearest distance is
//    exact wherever it is below r_max.
//  * Proximity flags: point-centric.  For every point and every level the
//    octree uses, the cells of that level whose box dilated by ratio * h
//    can hold the point are looked up in a hash of the leaves (level,
//    cell) and tested with the exact point-to-box distance.
//  * Edits (subdivide or prune): kept leaves compact in order, then the 8
//    children of each split leaf; the corner table is rebuilt from the
//    finest-grid integer positions of the new leaves' corners (radix sort,
//    run heads numbered in position order).  A position held by an old
//    corner keeps its value; a new one takes the parent's trilinear field.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "dv_internal.h"

namespace dv {
namespace {

constexpr uint64_t H_EMPTY = ~0ull;
constexpr uint64_t H_NONE = ~0ull;
constexpr int NN_RINGS = 3;          // rings searched around a query's cell

// ------------------------------------------------------------------ hash
// Open addressing with linear probing over 64-bit keys (never H_EMPTY);
// capacity a power of two at least twice the number of keys.
struct Hash {
  uint64_t* keys;
  uint32_t* a;
  uint32_t* b;
  uint64_t mask;
};

__device__ __forceinline__ uint64_t hmix(uint64_t k) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdull;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ull;
  k ^= k >> 33;
  return k;
}

// Slot of key, inserted if absent.
__device__ uint64_t h_insert(const Hash& h, uint64_t key) {
  uint64_t i = hmix(key) & h.mask;
  for (uint64_t n = 0; n <= h.mask; ++n) {
    const unsigned long long prev = atomicCAS(
        reinterpret_cast<unsigned long long*>(h.keys + i),
        (unsigned long long)H_EMPTY, (unsigned long long)key);
    if (prev == H_EMPTY || prev == key) return i;
    i = (i + 1) & h.mask;
  }
  return H_NONE;
}

__device__ uint64_t h_find(const Hash& h, uint64_t key) {
  uint64_t i = hmix(key) & h.mask;
  for (uint64_t n = 0; n <= h.mask; ++n) {
    const uint64_t k = h.keys[i];
    if (k == key) return i;
    if (k == H_EMPTY) return H_NONE;
    i = (i + 1) & h.mask;
  }
  return H_NONE;
}

struct HashBuf {
  DBuf keys, a, b;
  Hash h{};
};

dv_status hash_make(dv_ctx* ctx, HashBuf& hb, int64_t n_keys, bool two,
                    hipStream_t s) {
  const uint64_t cap = 1ull << ceil_log2((uint64_t)std::max<int64_t>(2 * n_keys, 64));
  DV_TRY(alloc_n<uint64_t>(ctx, hb.keys, cap, s));
  DV_TRY(alloc_n<uint32_t>(ctx, hb.a, cap, s));
  if (two) DV_TRY(alloc_n<uint32_t>(ctx, hb.b, cap, s));
  DV_TRY(fill_u32(hb.keys.as<uint32_t>(), 0xFFFFFFFFu, (int64_t)(2 * cap), s));
  hb.h.keys = hb.keys.as<uint64_t>();
  hb.h.a = hb.a.as<uint32_t>();
  hb.h.b = two ? hb.b.as<uint32_t>() : nullptr;
  hb.h.mask = cap - 1;
  return DV_OK;
}

// ------------------------------------------------------------------ readback
// Pinned words for the few counts a structure call reads back (per thread).
uint64_t* readback_words(size_t n) {
  static thread_local uint64_t* w = nullptr;
  static thread_local size_t cap = 0;
  if (n > cap) {
    if (w) (void)hipHostFree(w);
    w = nullptr;
    cap = 0;
    const size_t want = std::max<size_t>(n, 16);
    if (hipHostMalloc((void**)&w, want * sizeof(uint64_t), hipHostMallocDefault) !=
        hipSuccess) {
      (void)hipGetLastError();
      set_error("pinned host allocation failed");
      return nullptr;
    }
    cap = want;
  }
  return w;
}

dv_status read_words(const void* dev, size_t n, uint64_t* host, hipStream_t s) {
  uint64_t* pin = readback_words(n);
  if (!pin) return DV_ERR_OOM;
  DV_TRY_HIP(hipMemcpyAsync(pin, dev, n * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
  DV_TRY_HIP(hipStreamSynchronize(s));
  std::memcpy(host, pin, n * sizeof(uint64_t));
  return DV_OK;
}

__global__ void k_fill_f64(double* p, double v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * TPB)
    p[i] = v;
}

__global__ void k_fill_u8(uint8_t* p, uint8_t v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * TPB)
    p[i] = v;
}

unsigned capped_grid(int64_t n) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(grid_for(n, TPB), 8192));
}

// ------------------------------------------------------------------ points
// Bounding box of the points ([3][n] FP64) and the number of non-finite
// coordinates: per block, then one block over the block results.
// out: [0..2] min, [3..5] max (as doubles), [6] non-finite count (u64).
__global__ void __launch_bounds__(TPB)
k_bbox_part(const double* __restrict__ P, int64_t n, double* part, int nb) {
  __shared__ double smin[3][TPB], smax[3][TPB];
  __shared__ unsigned long long sbad[TPB];
  double mn[3] = {INFINITY, INFINITY, INFINITY};
  double mx[3] = {-INFINITY, -INFINITY, -INFINITY};
  unsigned long long bad = 0;
  for (int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * TPB) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double x = P[(int64_t)a * n + i];
      if (!isfinite(x)) {
        ++bad;
        continue;
      }
      mn[a] = fmin(mn[a], x);
      mx[a] = fmax(mx[a], x);
    }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    smin[a][threadIdx.x] = mn[a];
    smax[a][threadIdx.x] = mx[a];
  }
  sbad[threadIdx.x] = bad;
  __syncthreads();
  for (int o = TPB / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        smin[a][threadIdx.x] = fmin(smin[a][threadIdx.x], smin[a][threadIdx.x + o]);
        smax[a][threadIdx.x] = fmax(smax[a][threadIdx.x], smax[a][threadIdx.x + o]);
      }
      sbad[threadIdx.x] += sbad[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      part[(size_t)a * nb + blockIdx.x] = smin[a][0];
      part[(size_t)(3 + a) * nb + blockIdx.x] = smax[a][0];
    }
    reinterpret_cast<unsigned long long*>(part)[(size_t)6 * nb + blockIdx.x] = sbad[0];
  }
}

__global__ void __launch_bounds__(TPB)
k_bbox_final(const double* part, int nb, double* out) {
  __shared__ double s[6][TPB];
  __shared__ unsigned long long sb[TPB];
  double v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
  unsigned long long bad = 0;
  for (int i = threadIdx.x; i < nb; i += TPB) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      v[a] = fmin(v[a], part[(size_t)a * nb + i]);
      v[3 + a] = fmax(v[3 + a], part[(size_t)(3 + a) * nb + i]);
    }
    bad += reinterpret_cast<const unsigned long long*>(part)[(size_t)6 * nb + i];
  }
#pragma unroll
  for (int a = 0; a < 6; ++a) s[a][threadIdx.x] = v[a];
  sb[threadIdx.x] = bad;
  __syncthreads();
  for (int o = TPB / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        s[a][threadIdx.x] = fmin(s[a][threadIdx.x], s[a][threadIdx.x + o]);
        s[3 + a][threadIdx.x] = fmax(s[3 + a][threadIdx.x], s[3 + a][threadIdx.x + o]);
      }
      sb[threadIdx.x] += sb[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
#pragma unroll
    for (int a = 0; a < 6; ++a) out[a] = s[a][0];
    reinterpret_cast<unsigned long long*>(out)[6] = sb[0];
  }
}

// Grid of the points: cell (i, j, k) of side c from origin o, key
// i << 42 | j << 21 | k (each below 2^21).
struct GridDev {
  double o[3];
  double c;
  int64_t dims[3];
};

__device__ __forceinline__ uint64_t cell_key(int64_t i, int64_t j, int64_t k) {
  return ((uint64_t)i << 42) | ((uint64_t)j << 21) | (uint64_t)k;
}

__global__ void k_point_keys(const double* __restrict__ P, int64_t n, GridDev g,
                             uint64_t* keys, uint32_t* idx) {
  const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (i >= n) return;
  int64_t c[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double f = floor((P[(int64_t)a * n + i] - g.o[a]) / g.c);
    c[a] = (int64_t)fmin(fmax(f, 0.0), (double)(g.dims[a] - 1));
  }
  keys[i] = cell_key(c[0], c[1], c[2]);
  idx[i] = (uint32_t)i;
}

// After the sort: one hash slot per occupied cell with [start, end), and
// the points gathered into cell order (SoA).
__global__ void k_grid_cells(const uint64_t* __restrict__ ks,
                             const uint32_t* __restrict__ idx, int64_t n,
                             const double* __restrict__ P, Hash h,
                             double* __restrict__ Q) {
  const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (i >= n) return;
  const uint64_t k = ks[i];
  const uint32_t src = idx[i];
#pragma unroll
  for (int a = 0; a < 3; ++a) Q[(int64_t)a * n + i] = P[(int64_t)a * n + src];
  if (i == 0 || ks[i - 1] != k) {
    const uint64_t sl = h_insert(h, k);
    if (sl != H_NONE) h.a[sl] = (uint32_t)i;
  }
  if (i == n - 1 || ks[i + 1] != k) {
    const uint64_t sl = h_insert(h, k);
    if (sl != H_NONE) h.b[sl] = (uint32_t)(i + 1);
  }
}

// Exact nearest distance of every query ([3][m] FP64) that has a point
// closer than r_max; +inf otherwise (and for a non-finite query).
__global__ void __launch_bounds__(TPB)
k_nearest(const double* __restrict__ Qr, int64_t m, const double* __restrict__ S,
          int64_t n, GridDev g, Hash h, double r_max, double* __restrict__ dist) {
  const int64_t q = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (q >= m) return;
  const double x = Qr[q], y = Qr[m + q], z = Qr[2 * m + q];
  if (!(isfinite(x) && isfinite(y) && isfinite(z))) {
    dist[q] = INFINITY;
    return;
  }
  const double f[3] = {floor((x - g.o[0]) / g.c), floor((y - g.o[1]) / g.c),
                       floor((z - g.o[2]) / g.c)};
  // a query more than NN_RINGS cells outside the grid has no point within
  // r_max (the nearest cell is at least NN_RINGS c away)
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (f[a] < -(double)NN_RINGS - 1.0 || f[a] > (double)(g.dims[a] + NN_RINGS)) {
      dist[q] = INFINITY;
      return;
    }
  }
  const int64_t ci = (int64_t)f[0], cj = (int64_t)f[1], ck = (int64_t)f[2];
  double best = INFINITY;
  for (int r = 0; r <= NN_RINGS; ++r) {
    for (int dk = -r; dk <= r; ++dk) {
      const int64_t kk = ck + dk;
      if (kk < 0 || kk >= g.dims[2]) continue;
      for (int dj = -r; dj <= r; ++dj) {
        const int64_t jj = cj + dj;
        if (jj < 0 || jj >= g.dims[1]) continue;
        const bool face = (dk == -r || dk == r || dj == -r || dj == r);
        // inside the ring's shell only the two end cells of the row
        const int step = face ? 1 : (r > 0 ? 2 * r : 1);
        for (int di = -r; di <= r; di += step) {
          const int64_t ii = ci + di;
          if (ii < 0 || ii >= g.dims[0]) continue;
          const uint64_t sl = h_find(h, cell_key(ii, jj, kk));
          if (sl == H_NONE) continue;
          const uint32_t e = h.b[sl];
          for (uint32_t j = h.a[sl]; j < e; ++j) {
            const double dx = x - S[j], dy = y - S[n + j], dz = z - S[2 * n + j];
            double d2 = dx * dx + dy * dy;
            d2 = d2 + dz * dz;
            best = fmin(best, d2);
          }
        }
      }
    }
    // points of later rings are at least r c away (less a rounding margin)
    if (best < INFINITY && sqrt(best) + 1e-9 <= (double)r * g.c) break;
  }
  const double d = sqrt(best);
  dist[q] = d < r_max ? d : INFINITY;
}

struct PointGrid {
  GridDev g{};
  DBuf sorted;         // [3][n] points in cell order
  HashBuf cells;
  int64_t n = 0;
};

// Bounding box (one readback), keys, sort, cells.
dv_status build_grid(dv_ctx* ctx, const double* P, int64_t n, double c,
                     PointGrid& G, hipStream_t s) {
  G.n = n;
  if (n >= (int64_t)0xFFFFFFFFll) {
    set_error("%lld points exceed the 32-bit index range", (long long)n);
    return DV_ERR_LIMIT;
  }
  const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(grid_for(n, TPB), 1024));
  DBuf part, box;
  DV_TRY(alloc_n<double>(ctx, part, (size_t)7 * nb, s));
  DV_TRY(alloc_n<double>(ctx, box, 8, s));
  hipLaunchKernelGGL(k_bbox_part, dim3(nb), dim3(TPB), 0, s, P, n, part.as<double>(), nb);
  hipLaunchKernelGGL(k_bbox_final, dim3(1), dim3(TPB), 0, s, part.as<double>(), nb,
                     box.as<double>());
  DV_TRY_HIP(hipGetLastError());
  uint64_t w[8];
  DV_TRY(read_words(box.p, 8, w, s));
  double bb[6];
  std::memcpy(bb, w, sizeof(bb));
  if (w[6] != 0) {
    set_error("%llu point coordinates are not finite", (unsigned long long)w[6]);
    return DV_ERR_INVALID;
  }
  G.g.c = c;
  for (int a = 0; a < 3; ++a) {
    G.g.o[a] = bb[a];
    const double ext = std::floor((bb[3 + a] - bb[a]) / c) + 1.0;
    if (!(ext < (double)(1 << 21))) {
      set_error("point extent %.6g along axis %d exceeds 2^21 cells of %.6g",
                bb[3 + a] - bb[a], a, c);
      return DV_ERR_LIMIT;
    }
    G.g.dims[a] = (int64_t)ext;
  }
  DBuf k0, k1, v0, v1;
  DV_TRY(alloc_n<uint64_t>(ctx, k0, n, s));
  DV_TRY(alloc_n<uint64_t>(ctx, k1, n, s));
  DV_TRY(alloc_n<uint32_t>(ctx, v0, n, s));
  DV_TRY(alloc_n<uint32_t>(ctx, v1, n, s));
  hipLaunchKernelGGL(k_point_keys, dim3(grid_for(n, TPB)), dim3(TPB), 0, s, P, n, G.g,
                     k0.as<uint64_t>(), v0.as<uint32_t>());
  DV_TRY_HIP(hipGetLastError());
  bool alt = false;
  DV_TRY(radix_sort_u64(ctx, k0.as<uint64_t>(), v0.as<uint32_t>(), k1.as<uint64_t>(),
                        v1.as<uint32_t>(), n, 63, s, &alt));
  const uint64_t* ks = alt ? k1.as<uint64_t>() : k0.as<uint64_t>();
  const uint32_t* vs = alt ? v1.as<uint32_t>() : v0.as<uint32_t>();
  DV_TRY(hash_make(ctx, G.cells, n, true, s));
  DV_TRY(alloc_n<double>(ctx, G.sorted, (size_t)3 * n, s));
  hipLaunchKernelGGL(k_grid_cells, dim3(grid_for(n, TPB)), dim3(TPB), 0, s, ks, vs, n, P,
                     G.cells.h, G.sorted.as<double>());
  DV_TRY_HIP(hipGetLastError());
  return DV_OK;
}

dv_status nearest(dv_ctx* ctx, const double* P, int64_t n, const double* Q,
                  int64_t m, double r_max, double* dist, hipStream_t s) {
  if (m == 0) return DV_OK;
  if (n == 0) {
    hipLaunchKernelGGL(k_fill_f64, dim3(capped_grid(m)), dim3(TPB), 0, s, dist,
                       (double)INFINITY, m);
    DV_TRY_HIP(hipGetLastError());
    return DV_OK;
  }
  PointGrid G;
  DV_TRY(build_grid(ctx, P, n, 0.5 * r_max, G, s));
  hipLaunchKernelGGL(k_nearest, dim3(grid_for(m, TPB)), dim3(TPB), 0, s, Q, m,
                     G.sorted.as<double>(), n, G.g, G.cells.h, r_max, dist);
  DV_TRY_HIP(hipGetLastError());
  return DV_OK;
}

// ------------------------------------------------------------------ octree
struct LeafIn {
  int32_t n;
  int32_t max_level;
  int32_t n_corners;
  double root_min[3];
  double root_size;
  const uint8_t* level;
  const int32_t* ijk;
  const int32_t* cidx;
};

LeafIn leaf_in(const dv_octree_desc& o) {
  LeafIn L;
  L.n = o.n_voxels;
  L.max_level = o.max_level;
  L.n_corners = o.n_corners;
  for (int a = 0; a < 3; ++a) L.root_min[a] = o.root_min[a];
  L.root_size = o.root_size;
  L.level = o.level;
  L.ijk = o.ijk;
  L.cidx = o.corner_idx;
  return L;
}

dv_status check_desc(const dv_octree_desc* o, const char* who) {
  if (!o || o->n_voxels < 0 || o->max_level < 0 || o->max_level > DV_MAX_LEVEL ||
      !(o->root_size > 0) || !std::isfinite(o->root_size) ||
      !std::isfinite(o->root_min[0]) || !std::isfinite(o->root_min[1]) ||
      !std::isfinite(o->root_min[2]) ||
      (o->n_voxels > 0 && (!o->level || !o->ijk))) {
    set_error("%s: malformed octree", who);
    return DV_ERR_INVALID;
  }
  return DV_OK;
}

// Integer finest-grid position of corner m of leaf v (false: the leaf's
// level or cell is out of range).
__device__ __forceinline__ bool corner_pos(const LeafIn& L, int64_t v, int m,
                                           int64_t p[3]) {
  const int l = L.level[v];
  if (l > L.max_level) return false;
  const int64_t side = (int64_t)1 << l;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int64_t c = L.ijk[(int64_t)a * L.n + v];
    if (c < 0 || c >= side) return false;
    p[a] = (c + ((m >> a) & 1)) << (L.max_level - l);
  }
  return true;
}

// World positions of the corners ([3][Nc] FP64, root_min + pos * h_L);
// corners no leaf uses stay NaN.  err[0] counts leaves out of range.
__global__ void k_corner_world(LeafIn L, double* W, unsigned int* err) {
  const int64_t t = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (t >= (int64_t)L.n * 8) return;
  const int64_t v = t >> 3;
  const int m = (int)(t & 7);
  int64_t p[3];
  const int32_t c = L.cidx[(int64_t)m * L.n + v];
  if (!corner_pos(L, v, m, p) || c < 0 || c >= L.n_corners) {
    atomicAdd(err, 1u);
    return;
  }
  const double hL = L.root_size / (double)((int64_t)1 << L.max_level);
#pragma unroll
  for (int a = 0; a < 3; ++a)
    W[(int64_t)a * L.n_corners + c] = L.root_min[a] + (double)p[a] * hL;
}

// Eq. 1: v = v_far + (v_close - v_far) exp(-2 d^2 / s^2); d = inf -> v_far.
__global__ void k_prior(const double* __restrict__ d, int64_t n, double s,
                        double v_close, double v_far, float* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (i >= n) return;
  const double x = d[i];
  double v = v_far;
  if (x < INFINITY) v = v_far + (v_close - v_far) * exp(-2.0 * x * x / (s * s));
  out[i] = (float)v;
}

// Hash of the leaves: key level << 51 | i << 34 | j << 17 | k.
__device__ __forceinline__ uint64_t leaf_key(int64_t l, int64_t i, int64_t j, int64_t k) {
  return ((uint64_t)l << 51) | ((uint64_t)i << 34) | ((uint64_t)j << 17) | (uint64_t)k;
}

__global__ void k_leaf_hash(LeafIn L, Hash h, unsigned int* levels,
                            unsigned int* err) {
  const int64_t v = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (v >= L.n) return;
  const int l = L.level[v];
  const int64_t side = (int64_t)1 << (l <= DV_MAX_LEVEL ? l : 0);
  int64_t c[3];
  bool ok = l <= L.max_level;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    c[a] = L.ijk[(int64_t)a * L.n + v];
    ok = ok && c[a] >= 0 && c[a] < side;
  }
  if (!ok) {
    atomicAdd(err, 1u);
    return;
  }
  atomicOr(levels, 1u << l);
  const uint64_t sl = h_insert(h, leaf_key(l, c[0], c[1], c[2]));
  if (sl != H_NONE) h.a[sl] = (uint32_t)v;
}

// Proximity (the leaf's closed box within ratio * h of a point): every
// point marks the leaves it is near.  The test is written as the oracle
// writes it: lo = root_min + ijk h, hi = lo + h, q = max(lo - p, 0, p - hi)
// per axis, |q| <= ratio h.
__global__ void __launch_bounds__(TPB)
k_proximity(const double* __restrict__ P, int64_t n, LeafIn L, Hash h,
            uint32_t levels, double ratio, uint8_t* flags) {
  const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (i >= n) return;
  const double p[3] = {P[i], P[n + i], P[2 * n + i]};
  if (!(isfinite(p[0]) && isfinite(p[1]) && isfinite(p[2]))) return;
  for (int l = 0; l <= L.max_level; ++l) {
    if (!((levels >> l) & 1u)) continue;
    const double hl = L.root_size / (double)((int64_t)1 << l);
    const double tau = ratio * hl;
    const int64_t side = (int64_t)1 << l;
    int64_t lo[3], hi[3];
    bool any = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      // candidate cells; the small margin covers the rounding of the
      // division, the exact test below decides
      const double fa = floor((p[a] - tau - L.root_min[a]) / hl - 1e-6);
      const double fb = floor((p[a] + tau - L.root_min[a]) / hl + 1e-6);
      const double ca = fmax(fa, 0.0), cb = fmin(fb, (double)(side - 1));
      any = any && ca <= cb;
      lo[a] = (int64_t)ca;
      hi[a] = (int64_t)cb;
    }
    if (!any) continue;
    for (int64_t k = lo[2]; k <= hi[2]; ++k)
      for (int64_t j = lo[1]; j <= hi[1]; ++j)
        for (int64_t c = lo[0]; c <= hi[0]; ++c) {
          const uint64_t sl = h_find(h, leaf_key(l, c, j, k));
          if (sl == H_NONE) continue;
          const uint32_t v = h.a[sl];
          if (flags[v]) continue;
          const double cc[3] = {(double)c, (double)j, (double)k};
          double q2 = 0.0;
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            const double blo = L.root_min[a] + cc[a] * hl;
            const double bhi = blo + hl;
            const double qa = fmax(fmax(blo - p[a], 0.0), p[a] - bhi);
            q2 = a == 0 ? qa * qa : q2 + qa * qa;
          }
          if (sqrt(q2) <= tau) flags[v] = 1;
        }
  }
}

// ------------------------------------------------------------------ edits
// Leaf pass: kept leaves compact in order, then the children of the split
// leaves (rank r: n_keep + 8 r + m).  flags: 1 = split (subdivide) or
// keep (prune).  pre: exclusive scans of keep and split; tot[0] = n_keep.
__global__ void k_edit_leaves(LeafIn L, const uint8_t* __restrict__ flags,
                              int prune, const uint32_t* __restrict__ scan_keep,
                              const uint32_t* __restrict__ scan_split,
                              const uint64_t* __restrict__ tot, int64_t n_out,
                              uint8_t* __restrict__ lv, int32_t* __restrict__ ijk,
                              int32_t* __restrict__ src) {
  const int64_t v = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (v >= L.n) return;
  const bool f = flags[v] != 0;
  const bool kept = prune ? f : !f;
  const int l = L.level[v];
  const int32_t c0 = L.ijk[v], c1 = L.ijk[(int64_t)L.n + v], c2 = L.ijk[2 * (int64_t)L.n + v];
  if (kept) {
    const int64_t o = scan_keep[v];
    lv[o] = (uint8_t)l;
    ijk[o] = c0;
    ijk[n_out + o] = c1;
    ijk[2 * n_out + o] = c2;
    src[o] = (int32_t)v;
  } else if (!prune) {
    const int64_t base = (int64_t)tot[0] + 8 * (int64_t)scan_split[v];
    for (int m = 0; m < 8; ++m) {
      const int64_t o = base + m;
      lv[o] = (uint8_t)(l + 1);
      ijk[o] = 2 * c0 + (m & 1);
      ijk[n_out + o] = 2 * c1 + ((m >> 1) & 1);
      ijk[2 * n_out + o] = 2 * c2 + ((m >> 2) & 1);
      src[o] = (int32_t)v;
    }
  }
}

// Keep / split indicators; err[0] counts split leaves at the maximum
// level, err[1] leaves whose level, cell or corner indices are out of
// range (the later passes index with them).
__global__ void k_edit_flags(LeafIn L, const uint8_t* __restrict__ flags, int prune,
                             uint32_t* keep, uint32_t* split, unsigned int* err) {
  const int64_t v = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (v >= L.n) return;
  const bool f = flags[v] != 0;
  keep[v] = (prune ? f : !f) ? 1u : 0u;
  split[v] = (!prune && f) ? 1u : 0u;
  if (!prune && f && (int)L.level[v] >= L.max_level) atomicAdd(err, 1u);
  const int l = L.level[v];
  bool ok = l <= L.max_level;
  const int64_t side = (int64_t)1 << (ok ? l : 0);
  for (int a = 0; a < 3; ++a) {
    const int64_t c = L.ijk[(int64_t)a * L.n + v];
    ok = ok && c >= 0 && c < side;
  }
  for (int m = 0; m < 8; ++m) {
    const int32_t c = L.cidx[(int64_t)m * L.n + v];
    ok = ok && c >= 0 && c < L.n_corners;
  }
  if (!ok) atomicAdd(err + 1, 1u);
}

// Finest-grid corner keys of the new leaves, packed i << 2b | j << b | k
// with b = max_level + 1 bits (lexicographic in (i, j, k)).
__global__ void k_edit_corner_keys(const uint8_t* __restrict__ lv,
                                   const int32_t* __restrict__ ijk, int64_t n,
                                   int L, uint64_t* keys, uint32_t* vals) {
  const int64_t e = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (e >= n * 8) return;
  const int64_t v = e >> 3;
  const int m = (int)(e & 7);
  const int sh = L - lv[v];
  const int b = L + 1;
  uint64_t key = 0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const uint64_t p = ((uint64_t)ijk[(int64_t)a * n + v] + ((m >> a) & 1)) << sh;
    key = (key << b) | p;
  }
  keys[e] = key;
  vals[e] = (uint32_t)e;
}

// Keys of the old corners (same packing) into a hash: key -> old index.
__global__ void k_old_corner_hash(LeafIn L, Hash h) {
  const int64_t t = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (t >= (int64_t)L.n * 8) return;
  const int64_t v = t >> 3;
  const int m = (int)(t & 7);
  const int sh = L.max_level - L.level[v];
  const int b = L.max_level + 1;
  uint64_t key = 0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const uint64_t p = ((uint64_t)L.ijk[(int64_t)a * L.n + v] + ((m >> a) & 1)) << sh;
    key = (key << b) | p;
  }
  const uint64_t sl = h_insert(h, key);
  if (sl != H_NONE) h.a[sl] = (uint32_t)L.cidx[(int64_t)m * L.n + v];
}

__global__ void k_run_heads(const uint64_t* __restrict__ ks, int64_t n, uint32_t* head) {
  const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (i >= n) return;
  head[i] = (i == 0 || ks[i - 1] != ks[i]) ? 1u : 0u;
}

// Corner numbering and values.  Sorted entry i (value e = v * 8 + m) gets
// corner id = scan[i] + head[i] - 1; the head of a run (the smallest e of
// its position) sets the corner's value and source: the old corner at the
// position if there is one, else (a child's new corner) the parent's
// trilinear field at the corner, summed over the parent's corners in
// order in FP64, then rounded to FP32.
__global__ void k_edit_corners(const uint64_t* __restrict__ ks,
                               const uint32_t* __restrict__ es, int64_t n_e,
                               const uint32_t* __restrict__ head,
                               const uint32_t* __restrict__ scan, LeafIn L,
                               const float* __restrict__ dens, int prune,
                               const int32_t* __restrict__ src,
                               const uint64_t* __restrict__ n_keep, Hash old,
                               int64_t n_out, int32_t* __restrict__ cidx_out,
                               float* __restrict__ dens_out,
                               int32_t* __restrict__ csrc_out) {
  const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (i >= n_e) return;
  const uint32_t e = es[i];
  const int64_t v = e >> 3;
  const int m = (int)(e & 7);
  const uint32_t id = scan[i] + head[i] - 1u;
  cidx_out[(int64_t)m * n_out + v] = (int32_t)id;
  if (!head[i]) return;
  const int64_t p = src[v];
  int32_t oc = -1;
  if (prune || v < (int64_t)n_keep[0]) {
    oc = L.cidx[(int64_t)m * L.n + p];
  } else {
    const uint64_t sl = h_find(old, ks[i]);
    if (sl != H_NONE) oc = (int32_t)old.a[sl];
  }
  if (oc >= 0) {
    dens_out[id] = dens[oc];
    csrc_out[id] = oc;
    return;
  }
  const int mc = (int)((v - (int64_t)n_keep[0]) & 7);
  double u[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) u[a] = (double)(((mc >> a) & 1) + ((m >> a) & 1)) / 2.0;
  double val = 0.0;
  for (int q = 0; q < 8; ++q) {
    double w = 1.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) w *= ((q >> a) & 1) ? u[a] : 1.0 - u[a];
    val += w * (double)dens[L.cidx[(int64_t)q * L.n + p]];
  }
  dens_out[id] = (float)val;
  csrc_out[id] = -1;
}

__global__ void k_compose_src(int32_t* __restrict__ cur, const int32_t* __restrict__ prev,
                              int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (i >= n) return;
  const int32_t s = cur[i];
  cur[i] = s >= 0 ? prev[s] : -1;
}

__global__ void k_gather_sh(const float* __restrict__ sh, int64_t n_in, int rows,
                            const int32_t* __restrict__ src, int64_t n_out,
                            float* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (t >= n_out * rows) return;
  const int64_t r = t / n_out, v = t - r * n_out;
  out[t] = sh[r * n_in + src[v]];
}

__global__ void k_level_mask(const uint8_t* __restrict__ lv, int64_t n,
                             unsigned int* mask) {
  uint32_t m = 0;
  for (int64_t v = (int64_t)blockIdx.x * TPB + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * TPB)
    m |= 1u << (lv[v] & 31);
  for (int o = 32; o > 0; o >>= 1) m |= __shfl_xor(m, o, 64);
  if ((threadIdx.x & 63) == 0) atomicOr(mask, m);
}

__global__ void k_and_below(uint8_t* flags, const uint8_t* __restrict__ lv, int64_t n,
                            int max_level) {
  const int64_t v = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (v >= n) return;
  if ((int)lv[v] >= max_level) flags[v] = 0;
}

}  // namespace
}  // namespace dv

// Result of an edit (or of refinement rounds): the new leaf and corner
// tables in pool memory until dv_edit_apply copies them out.
struct dv_edit {
  dv_ctx* ctx = nullptr;
  int64_t n_leaves = 0, n_corners = 0;
  int32_t max_level = 0;
  double root_min[3] = {0, 0, 0};
  double root_size = 1;
  int32_t rounds = 0;
  // SH of the input octree (rows [S*3][n_in]), gathered by apply
  const float* sh_in = nullptr;
  int32_t sh_rows = 0;
  int64_t n_in = 0;
  dv::DBuf level, ijk, cidx, dens, leaf_src, corner_src;
};

namespace dv {
namespace {

// One edit of the octree L (densities dens) by flags: the tables land in
// E's buffers.  Synchronises the stream twice (leaf counts, corner count).
dv_status edit_once(dv_ctx* ctx, const LeafIn& L, const float* dens,
                    const uint8_t* flags, int prune, dv_edit* E, hipStream_t s) {
  const int64_t n = L.n;
  E->max_level = L.max_level;
  for (int a = 0; a < 3; ++a) E->root_min[a] = L.root_min[a];
  E->root_size = L.root_size;
  DBuf keep, split, skeep, ssplit, tots, err;
  DV_TRY(alloc_n<uint32_t>(ctx, keep, n, s));
  DV_TRY(alloc_n<uint32_t>(ctx, split, n, s));
  DV_TRY(alloc_n<uint32_t>(ctx, skeep, n, s));
  DV_TRY(alloc_n<uint32_t>(ctx, ssplit, n, s));
  DV_TRY(alloc_n<uint64_t>(ctx, tots, 4, s));
  DV_TRY(alloc_n<uint32_t>(ctx, err, 2, s));
  DV_TRY(fill_u32(tots.as<uint32_t>(), 0u, 8, s));
  DV_TRY(fill_u32(err.as<uint32_t>(), 0u, 2, s));
  if (n > 0) {
    hipLaunchKernelGGL(k_edit_flags, dim3(grid_for(n, TPB)), dim3(TPB), 0, s, L, flags,
                       prune, keep.as<uint32_t>(), split.as<uint32_t>(),
                       err.as<unsigned int>());
    DV_TRY_HIP(hipGetLastError());
    DV_TRY(exclusive_scan_u32(ctx, keep.as<uint32_t>(), skeep.as<uint32_t>(),
                              tots.as<uint64_t>(), n, s));
    DV_TRY(exclusive_scan_u32(ctx, split.as<uint32_t>(), ssplit.as<uint32_t>(),
                              tots.as<uint64_t>() + 1, n, s));
  }
  DV_TRY_HIP(hipMemcpyAsync(tots.as<uint64_t>() + 2, err.p, sizeof(uint64_t),
                            hipMemcpyDeviceToDevice, s));
  uint64_t w[3];
  DV_TRY(read_words(tots.p, 3, w, s));
  if ((uint32_t)(w[2] >> 32) != 0) {
    set_error("dv_edit: %u leaves have a level, cell or corner index out of range",
              (unsigned)(w[2] >> 32));
    return DV_ERR_RANGE;
  }
  if ((uint32_t)w[2] != 0) {
    set_error("dv_edit: %u split leaves are at the maximum level %d",
              (unsigned)(uint32_t)w[2], L.max_level);
    return DV_ERR_RANGE;
  }
  const int64_t n_keep = (int64_t)w[0], n_split = prune ? 0 : (int64_t)w[1];
  const int64_t n_out = n_keep + 8 * n_split;
  if (n_out * 8 >= (int64_t)0xFFFFFFFFll || n_out > (int64_t)INT32_MAX) {
    set_error("dv_edit: %lld leaves exceed the 32-bit index range", (long long)n_out);
    return DV_ERR_LIMIT;
  }
  E->n_leaves = n_out;
  DV_TRY(alloc_n<uint8_t>(ctx, E->level, n_out, s));
  DV_TRY(alloc_n<int32_t>(ctx, E->ijk, 3 * n_out, s));
  DV_TRY(alloc_n<int32_t>(ctx, E->leaf_src, n_out, s));
  DV_TRY(alloc_n<int32_t>(ctx, E->cidx, 8 * n_out, s));
  if (n > 0) {
    hipLaunchKernelGGL(k_edit_leaves, dim3(grid_for(n, TPB)), dim3(TPB), 0, s, L, flags,
                       prune, skeep.as<uint32_t>(), ssplit.as<uint32_t>(),
                       tots.as<uint64_t>(), n_out, E->level.as<uint8_t>(),
                       E->ijk.as<int32_t>(), E->leaf_src.as<int32_t>());
    DV_TRY_HIP(hipGetLastError());
  }
  if (n_out == 0) {
    E->n_corners = 0;
    DV_TRY(alloc_n<float>(ctx, E->dens, 1, s));
    DV_TRY(alloc_n<int32_t>(ctx, E->corner_src, 1, s));
    return DV_OK;
  }
  // corner table
  const int64_t n_e = 8 * n_out;
  DBuf k0, k1, v0, v1, head, hscan, ctot;
  DV_TRY(alloc_n<uint64_t>(ctx, k0, n_e, s));
  DV_TRY(alloc_n<uint64_t>(ctx, k1, n_e, s));
  DV_TRY(alloc_n<uint32_t>(ctx, v0, n_e, s));
  DV_TRY(alloc_n<uint32_t>(ctx, v1, n_e, s));
  DV_TRY(alloc_n<uint32_t>(ctx, head, n_e, s));
  DV_TRY(alloc_n<uint32_t>(ctx, hscan, n_e, s));
  DV_TRY(alloc_n<uint64_t>(ctx, ctot, 1, s));
  hipLaunchKernelGGL(k_edit_corner_keys, dim3(grid_for(n_e, TPB)), dim3(TPB), 0, s,
                     E->level.as<uint8_t>(), E->ijk.as<int32_t>(), n_out, L.max_level,
                     k0.as<uint64_t>(), v0.as<uint32_t>());
  DV_TRY_HIP(hipGetLastError());
  bool alt = false;
  DV_TRY(radix_sort_u64(ctx, k0.as<uint64_t>(), v0.as<uint32_t>(), k1.as<uint64_t>(),
                        v1.as<uint32_t>(), n_e, 3 * (L.max_level + 1), s, &alt));
  const uint64_t* ks = alt ? k1.as<uint64_t>() : k0.as<uint64_t>();
  const uint32_t* es = alt ? v1.as<uint32_t>() : v0.as<uint32_t>();
  hipLaunchKernelGGL(k_run_heads, dim3(grid_for(n_e, TPB)), dim3(TPB), 0, s, ks, n_e,
                     head.as<uint32_t>());
  DV_TRY_HIP(hipGetLastError());
  DV_TRY(exclusive_scan_u32(ctx, head.as<uint32_t>(), hscan.as<uint32_t>(),
                            ctot.as<uint64_t>(), n_e, s));
  HashBuf old;
  if (!prune) {
    DV_TRY(hash_make(ctx, old, 8 * n, false, s));
    if (n > 0)
      hipLaunchKernelGGL(k_old_corner_hash, dim3(grid_for(8 * n, TPB)), dim3(TPB), 0, s,
                         L, old.h);
    DV_TRY_HIP(hipGetLastError());
  }
  uint64_t nc = 0;
  DV_TRY(read_words(ctot.p, 1, &nc, s));
  E->n_corners = (int64_t)nc;
  DV_TRY(alloc_n<float>(ctx, E->dens, nc, s));
  DV_TRY(alloc_n<int32_t>(ctx, E->corner_src, nc, s));
  hipLaunchKernelGGL(k_edit_corners, dim3(grid_for(n_e, TPB)), dim3(TPB), 0, s, ks, es,
                     n_e, head.as<uint32_t>(), hscan.as<uint32_t>(), L, dens, prune,
                     E->leaf_src.as<int32_t>(), tots.as<uint64_t>(), old.h, n_out,
                     E->cidx.as<int32_t>(), E->dens.as<float>(),
                     E->corner_src.as<int32_t>());
  DV_TRY_HIP(hipGetLastError());
  return DV_OK;
}

LeafIn leaf_of_edit(const dv_edit* E) {
  LeafIn L;
  L.n = (int32_t)E->n_leaves;
  L.max_level = E->max_level;
  L.n_corners = (int32_t)E->n_corners;
  for (int a = 0; a < 3; ++a) L.root_min[a] = E->root_min[a];
  L.root_size = E->root_size;
  L.level = E->level.as<uint8_t>();
  L.ijk = E->ijk.as<int32_t>();
  L.cidx = E->cidx.as<int32_t>();
  return L;
}

// Proximity flags of octree L into flags (device [L.n]): one readback for
// the levels in use and the range errors.
dv_status proximity(dv_ctx* ctx, const LeafIn& L, const double* P, int64_t n_pts,
                    double ratio, uint8_t* flags, hipStream_t s) {
  if (L.n == 0) return DV_OK;
  hipLaunchKernelGGL(k_fill_u8, dim3(capped_grid(L.n)), dim3(TPB), 0, s, flags,
                     (uint8_t)0, (int64_t)L.n);
  HashBuf lh;
  DV_TRY(hash_make(ctx, lh, L.n, false, s));
  DBuf words;
  DV_TRY(alloc_n<uint64_t>(ctx, words, 1, s));
  DV_TRY(fill_u32(words.as<uint32_t>(), 0u, 2, s));
  hipLaunchKernelGGL(k_leaf_hash, dim3(grid_for(L.n, TPB)), dim3(TPB), 0, s, L, lh.h,
                     words.as<unsigned int>(), words.as<unsigned int>() + 1);
  DV_TRY_HIP(hipGetLastError());
  uint64_t w = 0;
  DV_TRY(read_words(words.p, 1, &w, s));
  if ((uint32_t)(w >> 32) != 0) {
    set_error("dv_proximity_flags: %u leaves have a level or cell out of range",
              (unsigned)(w >> 32));
    return DV_ERR_RANGE;
  }
  if (n_pts > 0) {
    hipLaunchKernelGGL(k_proximity, dim3(grid_for(n_pts, TPB)), dim3(TPB), 0, s, P,
                       n_pts, L, lh.h, (uint32_t)w, ratio, flags);
    DV_TRY_HIP(hipGetLastError());
  }
  return DV_OK;
}

dv_status check_points(const double* P, int64_t n, const char* who) {
  if (n < 0 || (n > 0 && !P)) {
    set_error("%s: malformed point array", who);
    return DV_ERR_INVALID;
  }
  if (n >= (int64_t)0xFFFFFFFFll) {
    set_error("%s: %lld points exceed the 32-bit index range", who, (long long)n);
    return DV_ERR_LIMIT;
  }
  return DV_OK;
}

}  // namespace
}  // namespace dv

using namespace dv;

extern "C" {

dv_status dv_nearest_distance(dv_ctx* ctx, const double* points, int64_t n_points,
                              const double* queries, int64_t n_queries,
                              double r_max, double* dist, void* stream) {
  if (!ctx || n_queries < 0 || (n_queries > 0 && (!queries || !dist)) ||
      !(r_max > 0) || !std::isfinite(r_max)) {
    set_error("dv_nearest_distance: invalid arguments");
    return DV_ERR_INVALID;
  }
  DV_TRY(check_points(points, n_points, "dv_nearest_distance"));
  DV_TRY_HIP(hipSetDevice(ctx->device));
  PoolStamp stamp_on_return(ctx);
  return nearest(ctx, points, n_points, queries, n_queries, r_max, dist,
                 (hipStream_t)stream);
}

dv_status dv_corner_prior(dv_ctx* ctx, const dv_octree_desc* octree,
                          const double* points, int64_t n_points, double s,
                          double v_close, double v_far, double r_cut,
                          float* density, void* stream) {
  DV_TRY(check_desc(octree, "dv_corner_prior"));
  if (!ctx || !(s > 0) || !std::isfinite(s) || !std::isfinite(v_close) ||
      !std::isfinite(v_far) || !(r_cut > 0) || !std::isfinite(r_cut) ||
      octree->n_corners < 0 || (octree->n_corners > 0 && !density) ||
      (octree->n_voxels > 0 && !octree->corner_idx)) {
    set_error("dv_corner_prior: invalid arguments");
    return DV_ERR_INVALID;
  }
  DV_TRY(check_points(points, n_points, "dv_corner_prior"));
  DV_TRY_HIP(hipSetDevice(ctx->device));
  PoolStamp stamp_on_return(ctx);
  hipStream_t st = (hipStream_t)stream;
  const LeafIn L = leaf_in(*octree);
  const int64_t nc = L.n_corners;
  if (nc == 0) return DV_OK;
  DBuf W, d, err;
  DV_TRY(alloc_n<double>(ctx, W, 3 * nc, st));
  DV_TRY(alloc_n<double>(ctx, d, nc, st));
  DV_TRY(alloc_n<uint64_t>(ctx, err, 1, st));
  DV_TRY(fill_u32(W.as<uint32_t>(), 0xFFFFFFFFu, 6 * nc, st));   // NaN
  DV_TRY(fill_u32(err.as<uint32_t>(), 0u, 2, st));
  if (L.n > 0) {
    hipLaunchKernelGGL(k_corner_world, dim3(grid_for(8 * (int64_t)L.n, TPB)), dim3(TPB),
                       0, st, L, W.as<double>(), err.as<unsigned int>());
    DV_TRY_HIP(hipGetLastError());
  }
  uint64_t e = 0;
  DV_TRY(read_words(err.p, 1, &e, st));
  if ((uint32_t)e != 0) {
    set_error("dv_corner_prior: %u (leaf, corner) entries out of range", (unsigned)(uint32_t)e);
    return DV_ERR_RANGE;
  }
  DV_TRY(nearest(ctx, points, n_points, W.as<double>(), nc, r_cut, d.as<double>(), st));
  hipLaunchKernelGGL(k_prior, dim3(grid_for(nc, TPB)), dim3(TPB), 0, st, d.as<double>(),
                     nc, s, v_close, v_far, density);
  DV_TRY_HIP(hipGetLastError());
  return DV_OK;
}

dv_status dv_proximity_flags(dv_ctx* ctx, const dv_octree_desc* octree,
                             const double* points, int64_t n_points, double ratio,
                             uint8_t* flags, void* stream) {
  DV_TRY(check_desc(octree, "dv_proximity_flags"));
  if (!ctx || !(ratio >= 0) || !std::isfinite(ratio) ||
      (octree->n_voxels > 0 && !flags)) {
    set_error("dv_proximity_flags: invalid arguments");
    return DV_ERR_INVALID;
  }
  DV_TRY(check_points(points, n_points, "dv_proximity_flags"));
  DV_TRY_HIP(hipSetDevice(ctx->device));
  PoolStamp stamp_on_return(ctx);
  return proximity(ctx, leaf_in(*octree), points, n_points, ratio, flags,
                   (hipStream_t)stream);
}

dv_status dv_edit_plan(dv_ctx* ctx, const dv_octree_desc* octree,
                       const uint8_t* flags, int32_t op, dv_edit** out,
                       int64_t* n_leaves, int64_t* n_corners, void* stream) {
  DV_TRY(check_desc(octree, "dv_edit_plan"));
  if (!ctx || !out || (op != DV_EDIT_SUBDIVIDE && op != DV_EDIT_PRUNE) ||
      (octree->n_voxels > 0 && (!flags || !octree->corner_idx || !octree->corner_density)) ||
      octree->sh_degree < 0 || octree->sh_degree > DV_MAX_SH_DEGREE) {
    set_error("dv_edit_plan: invalid arguments");
    return DV_ERR_INVALID;
  }
  *out = nullptr;
  DV_TRY_HIP(hipSetDevice(ctx->device));
  PoolStamp stamp_on_return(ctx);
  hipStream_t s = (hipStream_t)stream;
  std::unique_ptr<dv_edit> E(new dv_edit());
  E->ctx = ctx;
  E->sh_in = octree->sh;
  E->sh_rows = 3 * (octree->sh_degree + 1) * (octree->sh_degree + 1);
  E->n_in = octree->n_voxels;
  DV_TRY(edit_once(ctx, leaf_in(*octree), octree->corner_density, flags,
                   op == DV_EDIT_PRUNE ? 1 : 0, E.get(), s));
  E->rounds = 1;
  if (n_leaves) *n_leaves = E->n_leaves;
  if (n_corners) *n_corners = E->n_corners;
  *out = E.release();
  return DV_OK;
}

dv_status dv_refine_plan(dv_ctx* ctx, const dv_octree_desc* octree,
                         const double* points, int64_t n_points, double ratio,
                         double min_size, int32_t max_rounds, dv_edit** out,
                         int64_t* n_leaves, int64_t* n_corners, int32_t* rounds,
                         void* stream) {
  DV_TRY(check_desc(octree, "dv_refine_plan"));
  if (!ctx || !out || !(ratio >= 0) || !std::isfinite(ratio) || !(min_size > 0) ||
      max_rounds < 0 ||
      (octree->n_voxels > 0 && (!octree->corner_idx || !octree->corner_density)) ||
      octree->sh_degree < 0 || octree->sh_degree > DV_MAX_SH_DEGREE) {
    set_error("dv_refine_plan: invalid arguments");
    return DV_ERR_INVALID;
  }
  DV_TRY(check_points(points, n_points, "dv_refine_plan"));
  *out = nullptr;
  DV_TRY_HIP(hipSetDevice(ctx->device));
  PoolStamp stamp_on_return(ctx);
  hipStream_t s = (hipStream_t)stream;
  // round 0: the input itself (identity sources), copied into pool tables
  std::unique_ptr<dv_edit> cur(new dv_edit());
  cur->ctx = ctx;
  cur->sh_in = octree->sh;
  cur->sh_rows = 3 * (octree->sh_degree + 1) * (octree->sh_degree + 1);
  cur->n_in = octree->n_voxels;
  {
    const LeafIn L = leaf_in(*octree);
    DBuf keepall;
    DV_TRY(alloc_n<uint8_t>(ctx, keepall, L.n, s));
    if (L.n > 0)
      hipLaunchKernelGGL(k_fill_u8, dim3(capped_grid(L.n)), dim3(TPB), 0, s,
                         keepall.as<uint8_t>(), (uint8_t)1, (int64_t)L.n);
    // an all-keep prune renumbers the corners in position order; the
    // corner sources keep the input's numbering
    DV_TRY(edit_once(ctx, L, octree->corner_density, keepall.as<uint8_t>(), 1,
                     cur.get(), s));
  }
  int32_t done = 0;
  while (done < max_rounds && cur->n_leaves > 0) {
    const LeafIn L = leaf_of_edit(cur.get());
    // stop once the finest leaf is below min_size
    {
      DBuf mx;
      DV_TRY(alloc_n<uint64_t>(ctx, mx, 1, s));
      DV_TRY(fill_u32(mx.as<uint32_t>(), 0u, 2, s));
      hipLaunchKernelGGL(k_level_mask, dim3(capped_grid(L.n)), dim3(TPB), 0, s, L.level,
                         (int64_t)L.n, mx.as<unsigned int>());
      DV_TRY_HIP(hipGetLastError());
      uint64_t w = 0;
      DV_TRY(read_words(mx.p, 1, &w, s));
      int finest = 0;
      for (int l = 0; l <= DV_MAX_LEVEL; ++l)
        if (((uint32_t)w >> l) & 1u) finest = l;
      if (octree->root_size / (double)(1ll << finest) < min_size) break;
    }
    // leaves near a point, below the maximum level
    DBuf flags;
    DV_TRY(alloc_n<uint8_t>(ctx, flags, L.n, s));
    DV_TRY(proximity(ctx, L, points, n_points, ratio, flags.as<uint8_t>(), s));
    hipLaunchKernelGGL(k_and_below, dim3(grid_for(L.n, TPB)), dim3(TPB), 0, s,
                       flags.as<uint8_t>(), L.level, (int64_t)L.n, L.max_level);
    DV_TRY_HIP(hipGetLastError());
    std::unique_ptr<dv_edit> nxt(new dv_edit());
    nxt->ctx = ctx;
    nxt->sh_in = cur->sh_in;
    nxt->sh_rows = cur->sh_rows;
    nxt->n_in = cur->n_in;
    DV_TRY(edit_once(ctx, L, cur->dens.as<float>(), flags.as<uint8_t>(), 0, nxt.get(), s));
    if (nxt->n_leaves == cur->n_leaves) break;   // no leaf flagged
    // sources relative to the input octree
    hipLaunchKernelGGL(k_compose_src, dim3(grid_for(nxt->n_leaves, TPB)), dim3(TPB), 0, s,
                       nxt->leaf_src.as<int32_t>(), cur->leaf_src.as<int32_t>(),
                       nxt->n_leaves);
    if (nxt->n_corners > 0)
      hipLaunchKernelGGL(k_compose_src, dim3(grid_for(nxt->n_corners, TPB)), dim3(TPB), 0,
                         s, nxt->corner_src.as<int32_t>(), cur->corner_src.as<int32_t>(),
                         nxt->n_corners);
    DV_TRY_HIP(hipGetLastError());
    // the previous tables are read by the kernels just enqueued: release
    // them in stream order
    cur = std::move(nxt);
    ++done;
  }
  cur->rounds = done;
  if (n_leaves) *n_leaves = cur->n_leaves;
  if (n_corners) *n_corners = cur->n_corners;
  if (rounds) *rounds = done;
  *out = cur.release();
  return DV_OK;
}

dv_status dv_edit_apply(dv_edit* edit, const dv_edit_out* out, void* stream) {
  if (!edit || !out ||
      (edit->n_leaves > 0 && (!out->level || !out->ijk || !out->corner_idx)) ||
      (edit->n_corners > 0 && !out->corner_density) ||
      (out->sh && (!edit->sh_in || edit->sh_rows < 1))) {
    set_error("dv_edit_apply: invalid arguments");
    return DV_ERR_INVALID;
  }
  dv_ctx* ctx = edit->ctx;
  DV_TRY_HIP(hipSetDevice(ctx->device));
  PoolStamp stamp_on_return(ctx);
  hipStream_t s = (hipStream_t)stream;
  const int64_t n = edit->n_leaves, nc = edit->n_corners;
  auto cp = [&](void* dst, const DBuf& b, size_t bytes) -> dv_status {
    if (!dst || bytes == 0) return DV_OK;
    DV_TRY_HIP(hipMemcpyAsync(dst, b.p, bytes, hipMemcpyDeviceToDevice, s));
    return DV_OK;
  };
  DV_TRY(cp(out->level, edit->level, (size_t)n));
  DV_TRY(cp(out->ijk, edit->ijk, (size_t)12 * n));
  DV_TRY(cp(out->corner_idx, edit->cidx, (size_t)32 * n));
  DV_TRY(cp(out->corner_density, edit->dens, (size_t)4 * nc));
  DV_TRY(cp(out->leaf_src, edit->leaf_src, (size_t)4 * n));
  DV_TRY(cp(out->corner_src, edit->corner_src, (size_t)4 * nc));
  if (out->sh && n > 0) {
    hipLaunchKernelGGL(k_gather_sh, dim3(grid_for(n * edit->sh_rows, TPB)), dim3(TPB), 0,
                       s, edit->sh_in, edit->n_in, edit->sh_rows,
                       edit->leaf_src.as<int32_t>(), n, out->sh);
    DV_TRY_HIP(hipGetLastError());
  }
  return DV_OK;
}

void dv_edit_release(dv_edit* edit) {
  if (!edit) return;
  hipSetDevice(edit->ctx->device);
  dv_ctx* ctx = edit->ctx;
  delete edit;
  ctx->pool->stamp();
}

}  // extern "C"
