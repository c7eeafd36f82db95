// Context, error reporting, device memory pool and small fill kernels.
#include <algorithm>
#include <cstdarg>
#include <cstring>

#include "dv_internal.h"

namespace dv {

static thread_local std::string g_err;

void set_error(const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
}

const char* get_error() { return g_err.c_str(); }

static thread_local bool t_release_idle = false;

static thread_local Arena* t_arena = nullptr;
Arena* thread_arena() { return t_arena; }
ArenaScope::ArenaScope(Arena* a) { t_arena = a; }
ArenaScope::~ArenaScope() { t_arena = nullptr; }

IdleRelease::IdleRelease() { t_release_idle = true; }
IdleRelease::~IdleRelease() { t_release_idle = false; }

void* Pool::raw_alloc(size_t bytes, hipStream_t s) {
  if (has_user_alloc_)
    return user_alloc_.alloc(user_alloc_.user, bytes, device_, (void*)s);
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return p;
}

void Pool::raw_free(void* p, size_t bytes, hipStream_t s) {
  if (has_user_alloc_) {
    user_alloc_.free(user_alloc_.user, p, bytes, device_, (void*)s);
    return;
  }
  (void)hipFree(p);
}

Pool::~Pool() {
  hipSetDevice(device_);
  // the owner synchronised the device: nothing is in flight
  for (auto& kv : free_) raw_free(kv.second.p, kv.second.size, kv.second.stream);
  for (auto& kv : live_) raw_free(kv.first, kv.second, nullptr);
  for (auto& kv : ev_refs_) hipEventDestroy(kv.first);
  for (auto e : spare_events_) hipEventDestroy(e);
}

// Block sizes: powers of two from 512 B, multiples of 2 MiB from 1 MiB
// (all multiples of 512 B, the granule of torch's caching allocator, so a
// provider backed by it counts exactly the pool's bytes).
static size_t round_size(size_t b) {
  if (b < 512) return 512;
  if (b < (1u << 20)) {
    size_t r = 512;
    while (r < b) r <<= 1;
    return r;
  }
  const size_t g = 2u << 20;
  return (b + g - 1) / g * g;
}

// caller holds mu_
void Pool::drop_event(hipEvent_t ev) {
  if (!ev) return;
  auto it = ev_refs_.find(ev);
  if (it == ev_refs_.end()) return;
  if (--it->second == 0) {
    spare_events_.push_back(ev);
    ev_refs_.erase(it);
  }
}

void* Pool::alloc(size_t bytes, hipStream_t s) {
  size_t want = round_size(bytes);
  {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = free_.lower_bound(want);
    while (it != free_.end() && it->first <= 2 * want) {
      Block& b = it->second;
      if (b.idle || b.stream == s ||
          (b.ev && hipEventQuery(b.ev) == hipSuccess)) {
        void* p = b.p;
        live_[p] = b.size;
        in_use_ += b.size;
        drop_event(b.ev);
        free_.erase(it);
        return p;
      }
      ++it;
    }
  }
  void* p = raw_alloc(want, s);
  if (!p) {
    trim();
    p = raw_alloc(want, s);
    if (!p) return nullptr;
  }
  std::lock_guard<std::mutex> lk(mu_);
  live_[p] = want;
  in_use_ += want;
  return p;
}

void Pool::release(void* p, hipStream_t s) {
  std::lock_guard<std::mutex> lk(mu_);
  auto it = live_.find(p);
  if (it == live_.end()) return;
  Block b;
  b.p = p;
  b.size = it->second;
  b.stream = s;
  b.ev = nullptr;
  b.idle = t_release_idle;
  in_use_ -= b.size;
  live_.erase(it);
  free_.emplace(b.size, b);
  if (!b.idle) {
    bool seen = false;
    for (hipStream_t q : pending_) seen = seen || q == s;
    if (!seen) pending_.push_back(s);
  }
}

void Pool::stamp() {
  std::lock_guard<std::mutex> lk(mu_);
  for (hipStream_t s : pending_) {
    hipEvent_t ev = nullptr;
    if (!spare_events_.empty()) {
      ev = spare_events_.back();
      spare_events_.pop_back();
    } else if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      ev = nullptr;
    }
    if (ev && hipEventRecord(ev, s) != hipSuccess) {
      // left unstamped: such blocks are reused on their own stream only
      (void)hipGetLastError();
      spare_events_.push_back(ev);
      ev = nullptr;
    }
    if (!ev) continue;
    int n = 0;
    for (auto& kv : free_) {
      Block& b = kv.second;
      if (!b.idle && !b.ev && b.stream == s) {
        b.ev = ev;
        ++n;
      }
    }
    if (n > 0) ev_refs_[ev] += n;
    else spare_events_.push_back(ev);
  }
  pending_.clear();
}

void Pool::trim() {
  // a block's last use is enqueued before it is freed: the blocks free now
  // are unused once the device is idle (blocks freed meanwhile are kept)
  std::vector<void*> snap;
  {
    std::lock_guard<std::mutex> lk(mu_);
    for (auto& kv : free_) snap.push_back(kv.second.p);
  }
  if (hipDeviceSynchronize() != hipSuccess) (void)hipGetLastError();
  std::sort(snap.begin(), snap.end());
  std::vector<Block> gone;
  {
    std::lock_guard<std::mutex> lk(mu_);
    for (auto it = free_.begin(); it != free_.end();) {
      if (std::binary_search(snap.begin(), snap.end(), it->second.p)) {
        gone.push_back(it->second);
        drop_event(it->second.ev);
        it = free_.erase(it);
      } else {
        ++it;
      }
    }
  }
  // outside the lock: a user callback may take locks of its own
  for (const Block& b : gone) raw_free(b.p, b.size, b.stream);
}

dv_status alloc(dv_ctx* ctx, DBuf& b, size_t bytes, hipStream_t s) {
  b.reset();
  if (Arena* ar = t_arena) {
    const size_t want = (bytes + 255) & ~(size_t)255;
    if (want > ar->cap - ar->used) {
      set_error("scratch need of the call exceeds the %zu-byte static "
                "workspace (%zu bytes in use, %zu more asked)", ar->cap,
                ar->used, bytes);
      return DV_ERR_LIMIT;
    }
    b.pool = nullptr;               // carved, never returned one by one
    b.p = ar->base + ar->used;
    b.bytes = bytes;
    b.stream = s;
    ar->used += want;
    return DV_OK;
  }
  void* p = ctx->pool->alloc(bytes, s);
  if (!p) {
    set_error("device allocation of %zu bytes failed", bytes);
    return DV_ERR_OOM;
  }
  b.pool = ctx->pool.get();
  b.p = p;
  b.bytes = bytes;
  b.stream = s;
  return DV_OK;
}

__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

dv_status fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return DV_OK;
  unsigned g = grid_for(n, TPB);
  if (g > 65536) g = 65536;
  hipLaunchKernelGGL(k_fill_u32, dim3(g), dim3(TPB), 0, s, p, v, n);
  DV_TRY_HIP(hipGetLastError());
  return DV_OK;
}

dv_status fill_f32(float* p, float v, int64_t n, hipStream_t s) {
  uint32_t bits;
  std::memcpy(&bits, &v, 4);
  return fill_u32(reinterpret_cast<uint32_t*>(p), bits, n, s);
}

StageTimer::StageTimer(dv_ctx* c, int st, hipStream_t strm)
    : ctx(c), stage(st), s(strm) {
  if (!(ctx->prof_flags.load() & DV_PROFILE_EVENTS)) return;
  if (hipEventCreate(&a) != hipSuccess || hipEventRecord(a, s) != hipSuccess) {
    (void)hipGetLastError();
    a = nullptr;
  }
}

void StageTimer::stop() {
  if (!a) return;
  hipEvent_t b = nullptr;
  if (hipEventCreate(&b) != hipSuccess || hipEventRecord(b, s) != hipSuccess) {
    (void)hipGetLastError();
    a = nullptr;
    return;
  }
  std::lock_guard<std::mutex> lk(ctx->prof_mu);
  ctx->prof_pending.push_back({stage, a, b});
  a = nullptr;
}

static const char* kStageNames[DV_NUM_STAGES] = {
    "preprocess", "sort_records", "gather_scan", "emit_pairs", "sort_pairs",
    "tile_directory", "composite_fwd", "bwd_clear", "composite_bwd",
    "record_bwd", "host_sync", "other", "actor_fwd", "actor_bwd"};

}  // namespace dv

using namespace dv;

extern "C" {

const char* dv_last_error(void) { return get_error(); }

const char* dv_version(void) { return "dvox 0.1 (gfx950)"; }

dv_status dv_ctx_create(int32_t hip_device, const dv_allocator* alloc,
                        dv_ctx** out) {
  if (!out) {
    set_error("dv_ctx_create: out is NULL");
    return DV_ERR_INVALID;
  }
  *out = nullptr;
  int n = 0;
  DV_TRY_HIP(hipGetDeviceCount(&n));
  if (hip_device < 0 || hip_device >= n) {
    set_error("dv_ctx_create: device %d out of range (%d devices)",
              hip_device, n);
    return DV_ERR_INVALID;
  }
  DV_TRY_HIP(hipSetDevice(hip_device));
  auto* c = new (std::nothrow) dv_ctx();
  if (!c) return DV_ERR_OOM;
  c->device = hip_device;
  if (alloc && (!alloc->alloc || !alloc->free)) {
    delete c;
    set_error("dv_ctx_create: allocator needs both alloc and free");
    return DV_ERR_INVALID;
  }
  c->pool.reset(new Pool(hip_device, alloc));
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, hip_device) == hipSuccess)
    c->n_cu = prop.multiProcessorCount;
  if (hipHostMalloc((void**)&c->pinned, 64 * sizeof(uint64_t),
                    hipHostMallocDefault) != hipSuccess) {
    delete c;
    set_error("dv_ctx_create: pinned allocation failed");
    return DV_ERR_OOM;
  }
  {
    const dv_status rs = noalloc_setup(c);
    if (rs != DV_OK) {
      dv_ctx_destroy(c);
      return rs;
    }
  }
  *out = c;
  return DV_OK;
}

dv_status dv_ctx_set_profiling(dv_ctx* ctx, int32_t flags) {
  if (!ctx) return DV_ERR_INVALID;
  DV_TRY_HIP(hipSetDevice(ctx->device));
  if ((flags & DV_PROFILE_COUNTERS) && !ctx->counters) {
    DV_TRY(alloc_n<unsigned long long>(ctx, ctx->counters_buf, DV_NUM_COUNTERS, nullptr));
    ctx->counters = ctx->counters_buf.as<unsigned long long>();
    DV_TRY_HIP(hipMemset(ctx->counters, 0, DV_NUM_COUNTERS * sizeof(unsigned long long)));
    DV_TRY_HIP(hipDeviceSynchronize());
  }
  ctx->prof_flags = flags;
  return DV_OK;
}

dv_status dv_ctx_stage_times(dv_ctx* ctx, dv_stage_times* out, int32_t reset) {
  if (!ctx || !out) return DV_ERR_INVALID;
  DV_TRY_HIP(hipSetDevice(ctx->device));
  std::lock_guard<std::mutex> lk(ctx->prof_mu);
  for (auto& iv : ctx->prof_pending) {
    DV_TRY_HIP(hipEventSynchronize(iv.b));
    float ms = 0.0f;
    DV_TRY_HIP(hipEventElapsedTime(&ms, iv.a, iv.b));
    ctx->prof_ms[iv.stage] += ms;
    ctx->prof_calls[iv.stage] += 1;
    hipEventDestroy(iv.a);
    hipEventDestroy(iv.b);
  }
  ctx->prof_pending.clear();
  std::memset(out, 0, sizeof(*out));
  for (int i = 0; i < DV_NUM_STAGES; ++i) {
    out->ms[i] = ctx->prof_ms[i];
    out->calls[i] = ctx->prof_calls[i];
  }
  if (ctx->counters) {
    unsigned long long c[DV_NUM_COUNTERS];
    DV_TRY_HIP(hipDeviceSynchronize());
    DV_TRY_HIP(hipMemcpy(c, ctx->counters, sizeof(c), hipMemcpyDeviceToHost));
    out->entries_fwd = (int64_t)c[0];
    out->pieces_fwd = (int64_t)c[1];
    out->entries_bwd = (int64_t)c[2];
    out->pieces_bwd = (int64_t)c[3];
    out->entries_actor_fwd = (int64_t)c[4];
    out->pieces_actor_fwd = (int64_t)c[5];
    out->entries_actor_bwd = (int64_t)c[6];
    out->pieces_actor_bwd = (int64_t)c[7];
    out->wave_entries_fwd = (int64_t)c[8];
    out->wave_hits_fwd = (int64_t)c[9];
    out->wave_entries_bwd = (int64_t)c[10];
    out->wave_hits_bwd = (int64_t)c[11];
    if (reset) DV_TRY_HIP(hipMemset(ctx->counters, 0, sizeof(c)));
  }
  if (reset) {
    for (int i = 0; i < DV_NUM_STAGES; ++i) {
      ctx->prof_ms[i] = 0.0;
      ctx->prof_calls[i] = 0;
    }
  }
  return DV_OK;
}

dv_status dv_ctx_trim(dv_ctx* ctx) {
  if (!ctx) return DV_ERR_INVALID;
  DV_TRY_HIP(hipSetDevice(ctx->device));
  reap_states(ctx, true);
  ctx->pool->trim();
  return DV_OK;
}

dv_status dv_ctx_memory(dv_ctx* ctx, int64_t* in_use, int64_t* cached) {
  if (!ctx) return DV_ERR_INVALID;
  if (in_use) *in_use = (int64_t)ctx->pool->bytes_in_use();
  if (cached) *cached = (int64_t)ctx->pool->bytes_cached();
  return DV_OK;
}

const char* dv_stage_name(int32_t i) {
  if (i < 0 || i >= DV_NUM_STAGES) return "";
  return kStageNames[i];
}

void dv_ctx_destroy(dv_ctx* ctx) {
  if (!ctx) return;
  hipSetDevice(ctx->device);
  hipDeviceSynchronize();
  reap_states(ctx, true);
  {
    std::lock_guard<std::mutex> lk(ctx->prof_mu);
    for (auto& iv : ctx->prof_pending) {
      hipEventDestroy(iv.a);
      hipEventDestroy(iv.b);
    }
    ctx->prof_pending.clear();
  }
  ctx->counters = nullptr;
  {
    IdleRelease idle;
    ctx->counters_buf.reset();
  }
  ctx->pool.reset();
  if (ctx->pinned) hipHostFree(ctx->pinned);
  if (ctx->noalloc_pinned) hipHostFree(ctx->noalloc_pinned);
  delete ctx;
}

}  // extern "C"
