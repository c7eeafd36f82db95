// Scene validation and indexing (Sec. 3.1-3.2): leaf-only octrees with
// packed device geometry; actor tracks evaluated on the host in FP64.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include "dv_internal.h"

namespace dv {

// Interleave the low 21 bits of x, y, z (x lowest) into a 63-bit code.
static uint64_t spread3(uint64_t x) {
  x &= 0x1fffffull;
  x = (x | x << 32) & 0x1f00000000ffffull;
  x = (x | x << 16) & 0x1f0000ff0000ffull;
  x = (x | x << 8) & 0x100f00f00f00f00full;
  x = (x | x << 4) & 0x10c30c30c30c30c3ull;
  x = (x | x << 2) & 0x1249249249249249ull;
  return x;
}

static dv_status validate(const uint8_t* level, const int32_t* ijk,
                          const int32_t* cidx, int32_t n, int32_t max_level,
                          int32_t n_corners, int32_t sh_degree) {
  if (n < 0) { set_error("n_voxels < 0"); return DV_ERR_INVALID; }
  if (max_level < 0 || max_level > DV_MAX_LEVEL) {
    set_error("max_level %d outside [0, %d]", max_level, DV_MAX_LEVEL);
    return DV_ERR_RANGE;
  }
  if (sh_degree < 0 || sh_degree > DV_MAX_SH_DEGREE) {
    set_error("sh_degree %d outside [0, 3]", sh_degree);
    return DV_ERR_RANGE;
  }
  if (n > 0 && n_corners <= 0) {
    set_error("n_corners must be > 0");
    return DV_ERR_INVALID;
  }
  std::vector<std::pair<uint64_t, uint64_t>> span(n);
  for (int32_t v = 0; v < n; ++v) {
    int l = level[v];
    if (l > max_level) {
      set_error("leaf %d: level %d > max_level %d", v, l, max_level);
      return DV_ERR_RANGE;
    }
    uint64_t c = 0;
    for (int a = 0; a < 3; ++a) {
      int32_t x = ijk[(int64_t)a * n + v];
      if (x < 0 || x >= (1 << l)) {
        set_error("leaf %d: cell index %d outside [0, 2^%d)", v, x, l);
        return DV_ERR_RANGE;
      }
      c |= spread3((uint64_t)x << (max_level - l)) << a;
    }
    for (int m = 0; m < 8; ++m) {
      int32_t ci = cidx[(int64_t)m * n + v];
      if (ci < 0 || ci >= n_corners) {
        set_error("leaf %d corner %d: index %d outside [0, %d)", v, m, ci,
                  n_corners);
        return DV_ERR_RANGE;
      }
    }
    span[v] = {c, 1ull << (3 * (max_level - l))};
  }
  std::sort(span.begin(), span.end());
  for (int32_t v = 0; v + 1 < n; ++v) {
    if (span[v].first + span[v].second > span[v + 1].first) {
      set_error("leaves overlap (finest-level Morton code %llu)",
                (unsigned long long)span[v + 1].first);
      return DV_ERR_OVERLAP;
    }
  }
  return DV_OK;
}

}  // namespace dv

using namespace dv;

extern "C" {

dv_status dv_validate_octree_host(const uint8_t* level, const int32_t* ijk,
                                  const int32_t* corner_idx, int32_t n,
                                  int32_t max_level, int32_t n_corners,
                                  int32_t sh_degree, char* msg,
                                  int32_t msg_len) {
  if (n > 0 && (!level || !ijk || !corner_idx)) {
    set_error("NULL array");
    if (msg && msg_len > 0) snprintf(msg, msg_len, "%s", get_error());
    return DV_ERR_INVALID;
  }
  set_error("");
  dv_status st = validate(level, ijk, corner_idx, n, max_level, n_corners,
                          sh_degree);
  if (msg && msg_len > 0) snprintf(msg, msg_len, "%s", get_error());
  return st;
}

int32_t dv_track_pose(const dv_track_desc* tr, double t, double R[9],
                      double p[3]) {
  for (int i = 0; i < 9; ++i) R[i] = (i % 4 == 0) ? 1.0 : 0.0;
  p[0] = p[1] = p[2] = 0.0;
  if (!tr || tr->n_keys < 1) return 0;
  const int n = tr->n_keys;
  if (t < tr->t[0] || t > tr->t[n - 1]) return 0;
  int k = 0;  // last keyframe with t_k <= t
  while (k + 1 < n && tr->t[k + 1] <= t) ++k;
  double yaw, pp[3];
  if (k == n - 1) {
    yaw = tr->yaw[k];
    for (int a = 0; a < 3; ++a) pp[a] = tr->trans[3 * k + a];
  } else {
    double f = (t - tr->t[k]) / (tr->t[k + 1] - tr->t[k]);
    yaw = tr->yaw[k] + f * (tr->yaw[k + 1] - tr->yaw[k]);
    for (int a = 0; a < 3; ++a) {
      double p0 = tr->trans[3 * k + a], p1 = tr->trans[3 * (k + 1) + a];
      pp[a] = p0 + f * (p1 - p0);
    }
  }
  double c = std::cos(yaw), s = std::sin(yaw);
  R[0] = c; R[1] = -s; R[2] = 0.0;
  R[3] = s; R[4] = c;  R[5] = 0.0;
  R[6] = 0.0; R[7] = 0.0; R[8] = 1.0;
  p[0] = pp[0]; p[1] = pp[1]; p[2] = pp[2];
  return 1;
}

dv_status dv_build_scene(dv_ctx* ctx, const dv_octree_desc* octrees,
                         int32_t n_octrees, const dv_track_desc* tracks,
                         dv_scene** out) {
  if (!ctx || !octrees || !out || n_octrees < 1) {
    set_error("dv_build_scene: invalid arguments");
    return DV_ERR_INVALID;
  }
  if (n_octrees > DV_MAX_OCTREES) {
    set_error("dv_build_scene: %d octrees > %d", n_octrees, DV_MAX_OCTREES);
    return DV_ERR_LIMIT;
  }
  if (n_octrees > 1 && !tracks) {
    set_error("dv_build_scene: actors need tracks");
    return DV_ERR_INVALID;
  }
  *out = nullptr;
  DV_TRY_HIP(hipSetDevice(ctx->device));
  PoolStamp stamp_on_return(ctx);
  std::unique_ptr<dv_scene> sc(new dv_scene());
  sc->ctx = ctx;
  sc->n_oct = n_octrees;
  sc->desc.assign(octrees, octrees + n_octrees);
  sc->geo.resize(n_octrees);
  sc->trk_t.resize(n_octrees);
  sc->trk_yaw.resize(n_octrees);
  sc->trk_trans.resize(n_octrees);
  hipStream_t s = nullptr;
  for (int k = 0; k < n_octrees; ++k) {
    const dv_octree_desc& d = octrees[k];
    if (!(d.root_size > 0.0) || !std::isfinite(d.root_size)) {
      set_error("octree %d: root_size must be positive and finite", k);
      return DV_ERR_INVALID;
    }
    for (int a = 0; a < 3; ++a) {
      if (!std::isfinite(d.root_min[a])) {
        set_error("octree %d: root_min not finite", k);
        return DV_ERR_INVALID;
      }
    }
    if (k > 0 && d.has_box) {
      for (int a = 0; a < 3; ++a) {
        if (!(d.box_max[a] > d.box_min[a])) {
          set_error("octree %d: empty box on axis %d", k, a);
          return DV_ERR_INVALID;
        }
      }
    }
    const int32_t n = d.n_voxels;
    if (n < 0 || (n > 0 && (!d.level || !d.ijk || !d.corner_idx ||
                            !d.corner_density || !d.sh))) {
      set_error("octree %d: NULL array or negative size", k);
      return DV_ERR_INVALID;
    }
    std::vector<uint8_t> lv(n);
    std::vector<int32_t> ijk((size_t)3 * n), cidx((size_t)8 * n);
    if (n > 0) {
      DV_TRY_HIP(hipMemcpy(lv.data(), d.level, n, hipMemcpyDeviceToHost));
      DV_TRY_HIP(hipMemcpy(ijk.data(), d.ijk, (size_t)12 * n,
                           hipMemcpyDeviceToHost));
      DV_TRY_HIP(hipMemcpy(cidx.data(), d.corner_idx, (size_t)32 * n,
                           hipMemcpyDeviceToHost));
    }
    dv_status st = validate(lv.data(), ijk.data(), cidx.data(), n,
                            d.max_level, d.n_corners, d.sh_degree);
    if (st != DV_OK) {
      std::string m = get_error();
      set_error("octree %d: %s", k, m.c_str());
      return st;
    }
    std::vector<uint64_t> geo(n);
    for (int32_t v = 0; v < n; ++v)
      geo[v] = pack_geo(lv[v], ijk[v], ijk[(size_t)n + v],
                        ijk[(size_t)2 * n + v]);
    DV_TRY(alloc_n<uint64_t>(ctx, sc->geo[k], n, s));
    if (n > 0)
      DV_TRY_HIP(hipMemcpy(sc->geo[k].p, geo.data(), 8 * (size_t)n,
                           hipMemcpyHostToDevice));
    OctDev od;
    od.geo = sc->geo[k].as<uint64_t>();
    od.corner_idx = d.corner_idx;
    od.dens = d.corner_density;
    od.sh = d.sh;
    od.n_vox = n;
    od.n_corners = d.n_corners;
    od.sh_degree = d.sh_degree;
    od.max_level = d.max_level;
    for (int a = 0; a < 3; ++a) od.root_min[a] = d.root_min[a];
    od.root_size = d.root_size;
    sc->oct_host.push_back(od);
    sc->max_level_all = std::max(sc->max_level_all, d.max_level);
    sc->max_sh_degree = std::max(sc->max_sh_degree, d.sh_degree);
    sc->total_vox += n;
    if (k > 0) {
      const dv_track_desc& tr = tracks[k - 1];
      if (tr.n_keys < 1 || !tr.t || !tr.yaw || !tr.trans) {
        set_error("actor %d: empty track", k);
        return DV_ERR_INVALID;
      }
      for (int i = 0; i + 1 < tr.n_keys; ++i) {
        if (!(tr.t[i + 1] > tr.t[i])) {
          set_error("actor %d: track times not increasing", k);
          return DV_ERR_INVALID;
        }
      }
      sc->trk_t[k].assign(tr.t, tr.t + tr.n_keys);
      sc->trk_yaw[k].assign(tr.yaw, tr.yaw + tr.n_keys);
      sc->trk_trans[k].assign(tr.trans, tr.trans + 3 * tr.n_keys);
    }
  }
  DV_TRY(alloc_n<OctDev>(ctx, sc->oct_dev, n_octrees, s));
  DV_TRY_HIP(hipMemcpy(sc->oct_dev.p, sc->oct_host.data(),
                       sizeof(OctDev) * n_octrees, hipMemcpyHostToDevice));
  *out = sc.release();
  return DV_OK;
}

void dv_scene_destroy(dv_scene* scene) {
  if (!scene) return;
  hipSetDevice(scene->ctx->device);
  hipDeviceSynchronize();
  IdleRelease idle;
  delete scene;
}

}  // extern "C"
