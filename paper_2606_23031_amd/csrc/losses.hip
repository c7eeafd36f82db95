// Training losses and the optimiser step (Supp. 'Optimization Details',
// Training Losses): per view
//   L = l_color ((1 - l_ssim) mean|C - C_gt| + l_ssim (1 - SSIM(C, C_gt)))
//     + l_depth mean_{D_lidar > 0} |D - D_lidar|
//     + l_normal mean_{|N_pseudo| > 0} (1 - cos(N, N_pseudo))
//     + l_sky mean_{sky} (T_final - 1)^2,
// written as the loss terms and the gradient planes of the rendered
// outputs (ready for dv_render_backward), and a fused Adam step over the
// structure-of-arrays parameters.  Everything streams: HBM-bound.
//
// SSIM: 11 x 11 Gaussian window (sigma 1.5, normalised), C1 = 0.01^2,
// C2 = 0.03^2, zero padding at the border, mean over pixels and channels.
// A first pass blurs the five moments of each 16 x 16 tile (26 x 26 input
// patch in LDS, separable), forms the per-pixel SSIM and its partials with
// respect to the blurred mean, second moment and cross moment; a second
// pass blurs those partials (the blur's adjoint is the blur: the window is
// symmetric) and combines them into dSSIM/dC.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "render.h"

namespace dv {

constexpr int LT = 16;             // output tile side
constexpr int LR = 5;              // window radius
constexpr int LP = LT + 2 * LR;    // patch side (26)
constexpr float SS_C1 = 0.0001f;
constexpr float SS_C2 = 0.0009f;

struct LossView {
  int32_t h, w;
  const float* rgb;
  const float* depth;
  const float* normal;
  const float* T;
  const float* rgb_gt;
  const float* depth_lidar;
  const float* normal_pseudo;
  const float* sky_mask;
  float* g_rgb;
  float* g_depth;
  float* g_normal;
  float* g_T;
};

// Per-block sums go to LS_SLOTS accumulators per quantity (block b adds to
// slot b % LS_SLOTS, LS_STRIDE doubles apart), summed by k_loss_finish:
// thousands of blocks adding to one word serialise on it.
constexpr int LS_SLOTS = 64;
constexpr int LS_STRIDE = 8;
// quantities: pixel counts of depth, normal, sky; sums of L1, SSIM, depth,
// normal, sky
enum { LQ_CD, LQ_CN, LQ_CS, LQ_L1, LQ_SSIM, LQ_DEP, LQ_NOR, LQ_SKY, LQ_N };

struct LossArgs {
  LossView v;
  dv_loss_weights lam;
  float win[2 * LR + 1];
  double* terms;            // [8] of this view
  double* acc;              // [LQ_N][LS_SLOTS][LS_STRIDE] of this view
  float* part;              // [3 channels][3 partials][h][w] (SSIM pass)
};

__device__ inline void acc_add(const LossArgs& a, int q, double x) {
  if (x != 0.0)
    atomicAdd(a.acc + ((size_t)q * LS_SLOTS + blockIdx.x % LS_SLOTS) * LS_STRIDE, x);
}
__device__ inline double acc_total(const double* acc, int q) {
  double s = 0.0;
  for (int i = 0; i < LS_SLOTS; ++i) s += acc[((size_t)q * LS_SLOTS + i) * LS_STRIDE];
  return s;
}

__device__ inline double block_sum(double x, double* lds) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  __syncthreads();
  if (lane == 0) lds[w] = x;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += lds[i];
  return s;
}

// Pixel counts of the sparse terms (their means' denominators).
__global__ void __launch_bounds__(TPB) k_loss_count(LossArgs a) {
  __shared__ double lds[TPB / 64];
  const int64_t n = (int64_t)a.v.h * a.v.w;
  double cd = 0, cn = 0, cs = 0;
  for (int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * TPB) {
    if (a.v.depth_lidar && a.v.depth_lidar[i] > 0.0f) cd += 1;
    if (a.v.normal_pseudo) {
      const float x = a.v.normal_pseudo[i], y = a.v.normal_pseudo[n + i],
                  z = a.v.normal_pseudo[2 * n + i];
      if (x != 0.0f || y != 0.0f || z != 0.0f) cn += 1;
    }
    if (a.v.sky_mask && a.v.sky_mask[i] > 0.0f) cs += 1;
  }
  cd = block_sum(cd, lds);
  cn = block_sum(cn, lds);
  cs = block_sum(cs, lds);
  if (threadIdx.x == 0) {
    acc_add(a, LQ_CD, cd);
    acc_add(a, LQ_CN, cn);
    acc_add(a, LQ_CS, cs);
  }
}

// Per-pixel terms: L1 colour, sparse depth, normal cosine, sky; their sums
// into terms and their gradients into the planes (the SSIM part of the
// colour gradient is added by the second SSIM pass).
__global__ void __launch_bounds__(TPB) k_loss_point(LossArgs a) {
  __shared__ double lds[TPB / 64];
  const int64_t n = (int64_t)a.v.h * a.v.w;
  __shared__ float cnt[3];
  if (threadIdx.x < 3) cnt[threadIdx.x] = (float)fmax(acc_total(a.acc, threadIdx.x), 1.0);
  __syncthreads();
  const float nd = cnt[0], nn = cnt[1], ns = cnt[2];
  const dv_loss_weights& L = a.lam;
  const float k1 = L.color * (1.0f - L.ssim) / (3.0f * (float)n);
  double s1 = 0, sd = 0, sn = 0, ss = 0;
  for (int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * TPB) {
    if (a.v.rgb && a.v.rgb_gt) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float dlt = a.v.rgb[c * n + i] - a.v.rgb_gt[c * n + i];
        s1 += fabsf(dlt);
        if (a.v.g_rgb)
          a.v.g_rgb[c * n + i] = dlt > 0.0f ? k1 : (dlt < 0.0f ? -k1 : 0.0f);
      }
    } else if (a.v.g_rgb) {
#pragma unroll
      for (int c = 0; c < 3; ++c) a.v.g_rgb[c * n + i] = 0.0f;
    }
    if (a.v.depth && a.v.depth_lidar) {
      const float dl = a.v.depth_lidar[i];
      float g = 0.0f;
      if (dl > 0.0f) {
        const float dlt = a.v.depth[i] - dl;
        sd += fabsf(dlt);
        g = (dlt > 0.0f ? L.depth : (dlt < 0.0f ? -L.depth : 0.0f)) / nd;
      }
      if (a.v.g_depth) a.v.g_depth[i] = g;
    } else if (a.v.g_depth) {
      a.v.g_depth[i] = 0.0f;
    }
    if (a.v.normal && a.v.normal_pseudo) {
      const float px = a.v.normal_pseudo[i], py = a.v.normal_pseudo[n + i],
                  pz = a.v.normal_pseudo[2 * n + i];
      float g0 = 0.0f, g1 = 0.0f, g2 = 0.0f;
      if (px != 0.0f || py != 0.0f || pz != 0.0f) {
        const float x = a.v.normal[i], y = a.v.normal[n + i], z = a.v.normal[2 * n + i];
        const float np_ = sqrtf(px * px + py * py + pz * pz);
        const float nN = sqrtf(x * x + y * y + z * z);
        const float nm = fmaxf(nN, 1e-8f);
        const float cs_ = (x * px + y * py + z * pz) / (nm * np_);
        sn += 1.0 - (double)cs_;
        // d cos / dN: (Np/|Np| - cos N/|N|) / |N|, or Np / (1e-8 |Np|)
        const float k = -L.normal / nn;
        if (nN > 1e-8f) {
          g0 = k * (px / np_ - cs_ * x / nN) / nN;
          g1 = k * (py / np_ - cs_ * y / nN) / nN;
          g2 = k * (pz / np_ - cs_ * z / nN) / nN;
        } else {
          g0 = k * px / (1e-8f * np_);
          g1 = k * py / (1e-8f * np_);
          g2 = k * pz / (1e-8f * np_);
        }
      }
      if (a.v.g_normal) {
        a.v.g_normal[i] = g0;
        a.v.g_normal[n + i] = g1;
        a.v.g_normal[2 * n + i] = g2;
      }
    } else if (a.v.g_normal) {
      a.v.g_normal[i] = 0.0f;
      a.v.g_normal[n + i] = 0.0f;
      a.v.g_normal[2 * n + i] = 0.0f;
    }
    if (a.v.T && a.v.sky_mask) {
      float g = 0.0f;
      if (a.v.sky_mask[i] > 0.0f) {
        const float dlt = a.v.T[i] - 1.0f;
        ss += (double)dlt * dlt;
        g = L.sky * 2.0f * dlt / ns;
      }
      if (a.v.g_T) a.v.g_T[i] = g;
    } else if (a.v.g_T) {
      a.v.g_T[i] = 0.0f;
    }
  }
  s1 = block_sum(s1, lds);
  sd = block_sum(sd, lds);
  sn = block_sum(sn, lds);
  ss = block_sum(ss, lds);
  if (threadIdx.x == 0) {
    acc_add(a, LQ_L1, s1);
    acc_add(a, LQ_DEP, sd);
    acc_add(a, LQ_NOR, sn);
    acc_add(a, LQ_SKY, ss);
  }
}

// Load the 26 x 26 patch of plane p around tile (tx, ty) (zero outside).
__device__ inline void load_patch(float (*dst)[LP], const float* p, int h, int w,
                                  int tx, int ty) {
  for (int i = threadIdx.x; i < LP * LP; i += TPB) {
    const int r = i / LP, c = i % LP;
    const int y = ty * LT + r - LR, x = tx * LT + c - LR;
    dst[r][c] = (y >= 0 && y < h && x >= 0 && x < w) ? p[(int64_t)y * w + x] : 0.0f;
  }
}

// SSIM pass 1: per tile and channel the five blurred moments, S, and the
// partials dS/dm_x, dS/de_xx, dS/de_xy (divided by the pixel count).
__global__ void __launch_bounds__(TPB) k_ssim_a(LossArgs a) {
  __shared__ float X[LP][LP], Y[LP][LP];
  __shared__ float H5[5][LP][LT];
  __shared__ double lds[TPB / 64];
  const int h = a.v.h, w = a.v.w;
  const int ntx = (w + LT - 1) / LT;
  const int tx = blockIdx.x % ntx, ty = blockIdx.x / ntx, c = blockIdx.y;
  const int64_t n = (int64_t)h * w;
  load_patch(X, a.v.rgb + c * n, h, w, tx, ty);
  load_patch(Y, a.v.rgb_gt + c * n, h, w, tx, ty);
  __syncthreads();
  // horizontal pass: rows of the patch, output columns
  for (int i = threadIdx.x; i < LP * LT; i += TPB) {
    const int r = i / LT, oc = i % LT;
    float mx = 0, my = 0, exx = 0, eyy = 0, exy = 0;
#pragma unroll
    for (int k = 0; k < 2 * LR + 1; ++k) {
      const float x = X[r][oc + k], y = Y[r][oc + k], g = a.win[k];
      mx = fmaf(g, x, mx);
      my = fmaf(g, y, my);
      exx = fmaf(g, x * x, exx);
      eyy = fmaf(g, y * y, eyy);
      exy = fmaf(g, x * y, exy);
    }
    H5[0][r][oc] = mx; H5[1][r][oc] = my; H5[2][r][oc] = exx;
    H5[3][r][oc] = eyy; H5[4][r][oc] = exy;
  }
  __syncthreads();
  const int orow = threadIdx.x / LT, ocol = threadIdx.x % LT;
  const int y = ty * LT + orow, x = tx * LT + ocol;
  float m[5] = {0, 0, 0, 0, 0};
#pragma unroll
  for (int k = 0; k < 2 * LR + 1; ++k) {
    const float g = a.win[k];
#pragma unroll
    for (int q = 0; q < 5; ++q) m[q] = fmaf(g, H5[q][orow + k][ocol], m[q]);
  }
  double ssum = 0.0;
  if (y < h && x < w) {
    const float mx = m[0], my = m[1];
    const float sxx = m[2] - mx * mx, syy = m[3] - my * my, sxy = m[4] - mx * my;
    const float A1 = 2.0f * mx * my + SS_C1, A2 = 2.0f * sxy + SS_C2;
    const float B1 = mx * mx + my * my + SS_C1, B2 = sxx + syy + SS_C2;
    const float S = (A1 * A2) / (B1 * B2);
    ssum = S;
    const float inv_n = 1.0f / (3.0f * (float)n);
    const float dm = (2.0f * my * (A2 - A1) / (B1 * B2) -
                      2.0f * mx * S * (1.0f / B1 - 1.0f / B2)) * inv_n;
    const float dxx = -S / B2 * inv_n;
    const float dxy = 2.0f * A1 / (B1 * B2) * inv_n;
    const int64_t o = (int64_t)y * w + x;
    a.part[(c * 3 + 0) * n + o] = dm;
    a.part[(c * 3 + 1) * n + o] = dxx;
    a.part[(c * 3 + 2) * n + o] = dxy;
  }
  ssum = block_sum(ssum, lds);
  if (threadIdx.x == 0) acc_add(a, LQ_SSIM, ssum);
}

// SSIM pass 2: dSSIM/dx = w * dm + 2 x (w * dxx) + y (w * dxy), scaled by
// -l_color l_ssim (the loss takes 1 - SSIM) and added to the colour
// gradient.
__global__ void __launch_bounds__(TPB) k_ssim_b(LossArgs a) {
  __shared__ float P[3][LP][LP];
  __shared__ float H3[3][LP][LT];
  const int h = a.v.h, w = a.v.w;
  const int ntx = (w + LT - 1) / LT;
  const int tx = blockIdx.x % ntx, ty = blockIdx.x / ntx, c = blockIdx.y;
  const int64_t n = (int64_t)h * w;
#pragma unroll
  for (int q = 0; q < 3; ++q) load_patch(P[q], a.part + (c * 3 + q) * n, h, w, tx, ty);
  __syncthreads();
  for (int i = threadIdx.x; i < LP * LT; i += TPB) {
    const int r = i / LT, oc = i % LT;
    float s[3] = {0, 0, 0};
#pragma unroll
    for (int k = 0; k < 2 * LR + 1; ++k) {
      const float g = a.win[k];
#pragma unroll
      for (int q = 0; q < 3; ++q) s[q] = fmaf(g, P[q][r][oc + k], s[q]);
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) H3[q][r][oc] = s[q];
  }
  __syncthreads();
  const int orow = threadIdx.x / LT, ocol = threadIdx.x % LT;
  const int y = ty * LT + orow, x = tx * LT + ocol;
  if (y >= h || x >= w) return;
  float b[3] = {0, 0, 0};
#pragma unroll
  for (int k = 0; k < 2 * LR + 1; ++k) {
    const float g = a.win[k];
#pragma unroll
    for (int q = 0; q < 3; ++q) b[q] = fmaf(g, H3[q][orow + k][ocol], b[q]);
  }
  const int64_t o = (int64_t)y * w + x;
  const float xv = a.v.rgb[c * n + o], yv = a.v.rgb_gt[c * n + o];
  const float d = b[0] + 2.0f * xv * b[1] + yv * b[2];
  a.v.g_rgb[c * n + o] += -a.lam.color * a.lam.ssim * d;
}

// Per view: the sums into terms [total, color, l1, ssim, depth, normal,
// sky, 0] (means and the weighted total).
__global__ void k_loss_finish(double* terms, const double* acc, int64_t n,
                              dv_loss_weights L, int has_rgb) {
  const double l1 = acc_total(acc, LQ_L1) / (3.0 * (double)n);
  const double ss = has_rgb ? acc_total(acc, LQ_SSIM) / (3.0 * (double)n) : 1.0;
  const double dep = acc_total(acc, LQ_DEP) / fmax(acc_total(acc, LQ_CD), 1.0);
  const double nor = acc_total(acc, LQ_NOR) / fmax(acc_total(acc, LQ_CN), 1.0);
  const double sky = acc_total(acc, LQ_SKY) / fmax(acc_total(acc, LQ_CS), 1.0);
  const double col = (1.0 - L.ssim) * l1 + L.ssim * (1.0 - ss);
  terms[0] = L.color * col + L.depth * dep + L.normal * nor + L.sky * sky;
  terms[1] = col;
  terms[2] = l1;
  terms[3] = ss;
  terms[4] = dep;
  terms[5] = nor;
  terms[6] = sky;
  terms[7] = 0.0;
}

// ------------------------------------------------------------------ Adam
constexpr int ADAM_CHUNK = 4096;   // elements per block; tensors start on
                                   // multiples of it in the block space
struct AdamTensor {
  float* p;
  const float* g;
  float* m;
  float* v;
  int64_t n;
  int64_t block0;                  // first block of this tensor
};

__global__ void __launch_bounds__(TPB)
k_adam(const AdamTensor* __restrict__ ts, int nt, float lr, float b1, float omb1,
       float b2, float omb2, float eps, float c1, float c2) {
  int lo = 0, hi = nt - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (ts[mid].block0 <= (int64_t)blockIdx.x) lo = mid; else hi = mid - 1;
  }
  const AdamTensor& T = ts[lo];
  const int64_t base = ((int64_t)blockIdx.x - T.block0) * ADAM_CHUNK;
#pragma unroll 4
  for (int j = 0; j < ADAM_CHUNK / TPB; ++j) {
    const int64_t i = base + (int64_t)j * TPB + threadIdx.x;
    if (i >= T.n) break;
    const float g = T.g[i];
    const float m = fmaf(b1, T.m[i], omb1 * g);
    const float v = fmaf(b2, T.v[i], omb2 * g * g);
    T.m[i] = m;
    T.v[i] = v;
    T.p[i] -= lr * (m * c1) / (sqrtf(v * c2) + eps);
  }
}

}  // namespace dv

using namespace dv;

extern "C" {

dv_status dv_loss(dv_ctx* ctx, const dv_loss_view* views, int32_t n_views,
                  const dv_loss_weights* lam, double* terms, void* stream) {
  if (!ctx || !views || n_views < 1 || !lam || !terms) {
    set_error("dv_loss: invalid arguments");
    return DV_ERR_INVALID;
  }
  DV_TRY_HIP(hipSetDevice(ctx->device));
  PoolStamp stamp_on_return(ctx);
  hipStream_t s = (hipStream_t)stream;
  // Gaussian window (sigma 1.5), normalised in double
  float win[2 * LR + 1];
  {
    double g[2 * LR + 1], sum = 0.0;
    for (int k = 0; k < 2 * LR + 1; ++k) {
      const double x = k - LR;
      g[k] = std::exp(-x * x / (2.0 * 1.5 * 1.5));
      sum += g[k];
    }
    for (int k = 0; k < 2 * LR + 1; ++k) win[k] = (float)(g[k] / sum);
  }
  DBuf accs;
  const size_t per_view = (size_t)LQ_N * LS_SLOTS * LS_STRIDE;
  DV_TRY(alloc_n<double>(ctx, accs, per_view * n_views, s));
  DV_TRY(fill_u32(accs.as<uint32_t>(), 0u, 2 * (int64_t)(per_view * n_views), s));
  for (int i = 0; i < n_views; ++i) {
    const dv_loss_view& V = views[i];
    if (V.h < 1 || V.w < 1) {
      set_error("dv_loss: view %d has an empty image", i);
      return DV_ERR_INVALID;
    }
    const bool has_rgb = V.rgb && V.rgb_gt;
    if (has_rgb && !V.g_rgb) {
      set_error("dv_loss: view %d has no colour gradient plane", i);
      return DV_ERR_INVALID;
    }
    LossArgs a;
    std::memset(&a, 0, sizeof(a));
    a.v.h = V.h; a.v.w = V.w;
    a.v.rgb = V.rgb; a.v.depth = V.depth; a.v.normal = V.normal; a.v.T = V.T;
    a.v.rgb_gt = V.rgb_gt; a.v.depth_lidar = V.depth_lidar;
    a.v.normal_pseudo = V.normal_pseudo; a.v.sky_mask = V.sky_mask;
    a.v.g_rgb = V.g_rgb; a.v.g_depth = V.g_depth; a.v.g_normal = V.g_normal;
    a.v.g_T = V.g_T;
    a.lam = *lam;
    std::memcpy(a.win, win, sizeof(win));
    a.terms = terms + 8 * (size_t)i;
    a.acc = accs.as<double>() + per_view * i;
    const int64_t n = (int64_t)V.h * V.w;
    const unsigned g = std::min<int64_t>(grid_for(n, TPB), 4096);
    hipLaunchKernelGGL(k_loss_count, dim3(g), dim3(TPB), 0, s, a);
    hipLaunchKernelGGL(k_loss_point, dim3(g), dim3(TPB), 0, s, a);
    DBuf part;
    if (has_rgb) {
      // SSIM is reported whenever the images are given; its gradient pass
      // runs only with a non-zero weight
      DV_TRY(alloc_n<float>(ctx, part, (size_t)9 * n, s));
      a.part = part.as<float>();
      const int ntx = (V.w + LT - 1) / LT, nty = (V.h + LT - 1) / LT;
      hipLaunchKernelGGL(k_ssim_a, dim3((unsigned)(ntx * nty), 3), dim3(TPB), 0, s, a);
      if (lam->ssim != 0.0f && lam->color != 0.0f)
        hipLaunchKernelGGL(k_ssim_b, dim3((unsigned)(ntx * nty), 3), dim3(TPB), 0, s, a);
    }
    hipLaunchKernelGGL(k_loss_finish, dim3(1), dim3(1), 0, s, a.terms,
                       (const double*)a.acc, n, *lam, has_rgb ? 1 : 0);
    DV_TRY_HIP(hipGetLastError());
  }
  return DV_OK;
}

dv_status dv_adam(dv_ctx* ctx, const dv_adam_param* params, int32_t n_params,
                  const dv_adam_opts* opts, void* stream) {
  if (!ctx || !params || n_params < 1 || !opts || opts->step < 1 ||
      !(opts->lr >= 0.0) || !(opts->beta1 >= 0.0 && opts->beta1 < 1.0) ||
      !(opts->beta2 >= 0.0 && opts->beta2 < 1.0) || !(opts->eps > 0.0)) {
    set_error("dv_adam: invalid arguments");
    return DV_ERR_INVALID;
  }
  DV_TRY_HIP(hipSetDevice(ctx->device));
  PoolStamp stamp_on_return(ctx);
  hipStream_t s = (hipStream_t)stream;
  std::vector<AdamTensor> ts;
  int64_t blocks = 0;
  for (int i = 0; i < n_params; ++i) {
    const dv_adam_param& P = params[i];
    if (P.n < 0 || (P.n > 0 && (!P.p || !P.g || !P.m || !P.v))) {
      set_error("dv_adam: parameter %d is malformed", i);
      return DV_ERR_INVALID;
    }
    if (P.n == 0) continue;
    ts.push_back(AdamTensor{P.p, P.g, P.m, P.v, P.n, blocks});
    blocks += (P.n + ADAM_CHUNK - 1) / ADAM_CHUNK;
  }
  if (ts.empty()) return DV_OK;
  if (blocks >= (int64_t)1 << 31) {
    set_error("dv_adam: %lld blocks exceed the grid", (long long)blocks);
    return DV_ERR_LIMIT;
  }
  const size_t bytes = sizeof(AdamTensor) * ts.size();
  DBuf tab;
  DV_TRY(alloc_n<uint8_t>(ctx, tab, bytes, s));
  uint8_t* stage = stage_acquire(bytes);
  if (!stage) return DV_ERR_OOM;
  std::memcpy(stage, ts.data(), bytes);
  DV_TRY_HIP(hipMemcpyAsync(tab.p, stage, bytes, hipMemcpyHostToDevice, s));
  DV_TRY(stage_release(s));
  // the constants are formed in double and rounded once: 1 - b in FP32
  // from a rounded b (0.999f) would be off by 5e-5 relative
  const double c1 = 1.0 / (1.0 - std::pow(opts->beta1, opts->step));
  const double c2 = 1.0 / (1.0 - std::pow(opts->beta2, opts->step));
  hipLaunchKernelGGL(k_adam, dim3((unsigned)blocks), dim3(TPB), 0, s,
                     tab.as<AdamTensor>(), (int)ts.size(), (float)opts->lr,
                     (float)opts->beta1, (float)(1.0 - opts->beta1),
                     (float)opts->beta2, (float)(1.0 - opts->beta2),
                     (float)opts->eps, (float)c1, (float)c2);
  DV_TRY_HIP(hipGetLastError());
  return DV_OK;
}

}  // extern "C"
