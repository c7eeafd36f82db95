// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <cstdio>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/dv.h"

namespace dv {

// ------------------------------------------------------------------ errors
void set_error(const char* fmt, ...);
const char* get_error();

#define DV_TRY_HIP(expr)                                                    \
  do {                                                                      \
    hipError_t _e = (expr);                                                 \
    if (_e != hipSuccess) {                                                 \
      ::dv::set_error("HIP error %s at %s:%d: %s", hipGetErrorName(_e),     \
                      __FILE__, __LINE__, #expr);                           \
      return DV_ERR_DEVICE;                                                 \
    }                                                                       \
  } while (0)

#define DV_TRY(expr)                                                        \
  do {                                                                      \
    dv_status _s = (expr);                                                  \
    if (_s != DV_OK) return _s;                                             \
  } while (0)

// ------------------------------------------------------------------ memory
// Stream-aware caching pool. A freed block is reusable at once on the
// stream that freed it (stream order). For other streams it waits for a
// stamp: each library call, as it returns, records one event per stream on
// which it freed blocks (stamp()) and attaches it to those blocks, and
// another stream takes such a block once that event has completed. (An
// event recorded per free would put a marker between kernels in the queue
// for every buffer; one per call does not.) Blocks freed after their last
// use is known to be complete (IdleRelease) are reusable by any stream.
// Backing memory comes from the caller's allocator callbacks when the
// context was created with one (torch's caching allocator, say), else from
// hipMalloc; trim() hands every idle block back.
class Pool {
 public:
  Pool(int device, const dv_allocator* a) : device_(device) {
    if (a && a->alloc && a->free) {
      user_alloc_ = *a;
      has_user_alloc_ = true;
    }
  }
  ~Pool();
  void* alloc(size_t bytes, hipStream_t s);
  void release(void* p, hipStream_t s);
  // record one event on each stream that freed blocks since the last stamp
  void stamp();
  void trim();
  size_t bytes_in_use() const { return in_use_; }

 private:
  struct Block {
    void* p;
    size_t size;
    hipStream_t stream;
    hipEvent_t ev;  // stamp event, nullptr until stamped
    bool idle;      // no use pending on any stream
  };
  void drop_event(hipEvent_t ev);
  void* raw_alloc(size_t bytes, hipStream_t s);
  void raw_free(void* p, size_t bytes, hipStream_t s);
  dv_allocator user_alloc_{};
  bool has_user_alloc_ = false;
  std::mutex mu_;
  std::multimap<size_t, Block> free_;
  std::map<void*, size_t> live_;
  std::vector<hipStream_t> pending_;            // streams with unstamped frees
  std::unordered_map<hipEvent_t, int> ev_refs_;  // blocks per stamp event
  std::vector<hipEvent_t> spare_events_;
  size_t in_use_ = 0;
 public:
  size_t bytes_cached() {
    std::lock_guard<std::mutex> lk(mu_);
    size_t b = 0;
    for (auto& kv : free_) b += kv.first;
    return b;
  }
 private:
  int device_;
};

// Bump arena over caller-independent static device memory (the
// allocation-free entry point): while one is installed on a thread, every
// buffer that thread's library call asks for is carved from it (never
// freed individually), and host staging comes from its pinned block.
struct Arena {
  uint8_t* base = nullptr;      // device
  size_t cap = 0;
  size_t used = 0;
  uint8_t* pinned = nullptr;    // host, pinned: [0, cap/2) tables, rest words
  size_t pinned_cap = 0;
};
Arena* thread_arena();
struct ArenaScope {
  explicit ArenaScope(Arena* a);
  ~ArenaScope();
  ArenaScope(const ArenaScope&) = delete;
  ArenaScope& operator=(const ArenaScope&) = delete;
};

// While alive on a thread, blocks freed by that thread are marked idle: for
// buffers whose last use has been waited for.
struct IdleRelease {
  IdleRelease();
  ~IdleRelease();
};

// Owning device buffer returned to the pool on destruction.
struct DBuf {
  Pool* pool = nullptr;
  void* p = nullptr;
  size_t bytes = 0;
  hipStream_t stream = nullptr;
  DBuf() = default;
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept { *this = std::move(o); }
  DBuf& operator=(DBuf&& o) noexcept {
    reset();
    pool = o.pool; p = o.p; bytes = o.bytes; stream = o.stream;
    o.p = nullptr; o.bytes = 0;
    return *this;
  }
  ~DBuf() { reset(); }
  void reset() {
    if (p && pool) pool->release(p, stream);
    p = nullptr; bytes = 0;
  }
  template <class T> T* as() const { return reinterpret_cast<T*>(p); }
  // non-owning view of part of another buffer
  void view_of(void* q, size_t n) {
    reset();
    pool = nullptr;
    p = q;
    bytes = n;
  }
};

}  // namespace dv

struct dv_fwd_state;

namespace dv {
enum Stage {
  ST_PREPROCESS = 0, ST_SORT_RECORDS, ST_GATHER, ST_EMIT, ST_SORT_PAIRS,
  ST_TILE_DIR, ST_COMPOSITE_FWD, ST_BWD_CLEAR, ST_COMPOSITE_BWD,
  ST_RECORD_BWD, ST_HOST_SYNC, ST_OTHER, ST_ACTOR_FWD, ST_ACTOR_BWD
};
}  // namespace dv

struct dv_ctx {
  int device = 0;
  // forward states whose stream work may still be in flight; deleted once
  // their event has completed
  std::mutex gy_mu;
  std::vector<std::pair<hipEvent_t, dv_fwd_state*>> graveyard;
  std::unique_ptr<dv::Pool> pool;
  // pinned host words for device->host counters
  uint64_t* pinned = nullptr;
  std::mutex pinned_mu;
  std::atomic<bool> poisoned{false};
  int n_cu = 0;
  // profiling
  std::atomic<int> prof_flags{0};
  std::mutex prof_mu;
  struct Interval { int stage; hipEvent_t a, b; };
  std::vector<Interval> prof_pending;
  double prof_ms[DV_NUM_STAGES] = {0};
  int64_t prof_calls[DV_NUM_STAGES] = {0};
  unsigned long long* counters = nullptr;  // device [DV_NUM_COUNTERS], from the pool
  dv::DBuf counters_buf;
  // allocation-free entry point: this device's static scratch array (its
  // device address, from hipGetSymbolAddress at context creation) and a
  // pinned host block for its staging, both set up by dv_ctx_create
  uint8_t* noalloc_scratch = nullptr;
  size_t noalloc_bytes = 0;
  uint8_t* noalloc_pinned = nullptr;
  size_t noalloc_pinned_bytes = 0;
};

namespace dv {

dv_status alloc(dv_ctx* ctx, DBuf& b, size_t bytes, hipStream_t s);
// Locate this device's static scratch array of the allocation-free entry
// point and allocate its pinned staging (at context creation).
dv_status noalloc_setup(dv_ctx* ctx);
// Declared first in a library call: on return, after the call's own buffers
// are freed, stamps the blocks freed during the call.
struct PoolStamp {
  dv_ctx* ctx;
  explicit PoolStamp(dv_ctx* c) : ctx(c) {}
  ~PoolStamp() {
    if (ctx && ctx->pool) ctx->pool->stamp();
  }
  PoolStamp(const PoolStamp&) = delete;
  PoolStamp& operator=(const PoolStamp&) = delete;
};
// Defer deletion of a forward state until its stream has passed this point.
void retire_state(dv_ctx* ctx, dv_fwd_state* st);
// Delete retired states whose work has completed (all of them if wait).
void reap_states(dv_ctx* ctx, bool wait);
// Records HIP events around a stage when profiling is on.
struct StageTimer {
  dv_ctx* ctx;
  int stage;
  hipStream_t s;
  hipEvent_t a = nullptr;
  StageTimer(dv_ctx* c, int st, hipStream_t strm);
  ~StageTimer() { stop(); }
  void stop();
};

template <class T>
dv_status alloc_n(dv_ctx* ctx, DBuf& b, size_t n, hipStream_t s) {
  return alloc(ctx, b, (n ? n : 1) * sizeof(T), s);
}

// ------------------------------------------------------------------ layout
constexpr int TILE = 16;
constexpr int TPB = 256;          // threads per block (4 wave64)
constexpr float Z_EPS = 1e-3f;    // binning near-plane (R18 contract)
constexpr int QBITS = 24;         // camera quantisation for ranks

// Packed leaf geometry: i | j << 19 | k << 38 | level << 57.
__host__ __device__ inline uint64_t pack_geo(uint32_t l, uint32_t i,
                                             uint32_t j, uint32_t k) {
  return (uint64_t)i | ((uint64_t)j << 19) | ((uint64_t)k << 38) |
         ((uint64_t)l << 57);
}
__host__ __device__ inline void unpack_geo(uint64_t g, int& l, int& i, int& j,
                                           int& k) {
  i = (int)(g & 0x7FFFF);
  j = (int)((g >> 19) & 0x7FFFF);
  k = (int)((g >> 38) & 0x7FFFF);
  l = (int)(g >> 57);
}

// Device view of one octree (built once per scene).
struct OctDev {
  const uint64_t* geo;
  const int32_t* corner_idx;
  const float* dens;
  const float* sh;
  int32_t n_vox;
  int32_t n_corners;
  int32_t sh_degree;
  int32_t max_level;
  double root_min[3];
  double root_size;
};

// Per view constants.
struct ViewConst {
  double fx, fy, cx, cy;
  double rnear2;            // binning: whole-window radius^2 near the camera
  double rnear_m;           // sqrt(rnear2), rounded up (culling pre-test)
  double side_norm[4];      // |normal| of the 4 window side planes (pre-test)
  float inv_fx, inv_fy, fcx, fcy;
  float Rc[9];              // camera -> world rotation (row-major)
  int32_t x0, y0, w, h;
  int32_t ntx, nty;
  uint32_t tile_base;       // first global tile of this view
  int32_t pad;
};

// Per (view, octree) constants.
struct VOConst {
  double A[9];              // octree frame -> camera frame (binning)
  double b[3];
  double rootrel[3];        // root_min - P (camera in octree frame)
  int64_t Q[3];             // quantised camera for ranks
  float Rt[9];              // world -> octree rotation (d_k = Rt d)
  float R[9];               // octree -> world rotation (normals)
  float boxlo[3];           // box - P (actors)
  float boxhi[3];
  float omp[3];             // camera - p in world (pose gradients)
  int32_t active;
  int32_t octree;
  int32_t view;
  int32_t feat_nc;          // feature render: channels of this group (1..3)
  const float* feat;        // feature render: the group's first channel
                            // [feat_nc][N] (stride N), else null
};

}  // namespace dv

struct dv_scene {
  dv_ctx* ctx = nullptr;
  int32_t n_oct = 0;
  std::vector<dv_octree_desc> desc;
  std::vector<std::vector<double>> trk_t, trk_yaw, trk_trans;
  std::vector<dv::DBuf> geo;       // per octree packed geometry
  dv::DBuf oct_dev;                // OctDev[n_oct]
  std::vector<dv::OctDev> oct_host;
  int32_t max_level_all = 0;
  int32_t max_sh_degree = 0;
  int64_t total_vox = 0;
};

namespace dv {

// Scan: exclusive prefix sum of n uint32 counts into out (uint32), with
// the uint64 total written to *total_dev.  Temp buffers from ctx pool.
dv_status exclusive_scan_u32(dv_ctx* ctx, const uint32_t* in, uint32_t* out,
                             uint64_t* total_dev, int64_t n, hipStream_t s);

// Stable LSD radix sort of (key, value) pairs by the low `bits` bits of the
// key.  Result lands in (keys, vals) (ping-ponging through the alt arrays).
dv_status radix_sort_u64(dv_ctx* ctx, uint64_t* keys, uint32_t* vals,
                         uint64_t* keys_alt, uint32_t* vals_alt, int64_t n,
                         int bits, hipStream_t s, bool* in_alt);
dv_status radix_sort_u32(dv_ctx* ctx, uint32_t* keys, uint32_t* vals,
                         uint32_t* keys_alt, uint32_t* vals_alt, int64_t n,
                         int bits, hipStream_t s, bool* in_alt);

dv_status fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s);
dv_status fill_f32(float* p, float v, int64_t n, hipStream_t s);

inline int ceil_log2(uint64_t x) {
  int b = 0;
  while ((1ull << b) < x && b < 63) ++b;
  return b;
}

inline unsigned grid_for(int64_t n, int per_block) {
  return (unsigned)((n + per_block - 1) / per_block);
}

}  // namespace dv
