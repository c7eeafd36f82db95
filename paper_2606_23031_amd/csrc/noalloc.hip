// Allocation-free variant of dv_render: every per-call buffer is carved from
// a file-scope static device array of fixed size instead of the context's
// pool, and host staging comes from a pinned block set up with the context.
#include <cstring>

#include "render.h"

namespace dv {

dv_status setup_state(dv_fwd_state* st, const dv_scene* sc, const dv_view* views,
                      int32_t n_views, const double* pose_override);
dv_status run_forward(dv_ctx* ctx, const dv_scene* sc, dv_fwd_state* st,
                      const dv_outputs* outs, hipStream_t s, bool composite);
dv_status check_opts(const dv_render_opts* op);
dv_render_opts effective_opts(const dv_render_opts& op);
dv_status check_feat_ptrs(const dv_render_opts& op, const dv_scene* sc);

// The workspace: 128 MiB per GPU, held from the library's first use on that
// GPU until the process ends.  Host code must not pass this name to a
// kernel (it is a host-side stand-in); the device address comes from
// hipGetSymbolAddress, once per device, at context creation.
constexpr size_t NOALLOC_BYTES = (size_t)128 << 20;
constexpr size_t NOALLOC_PINNED_BYTES = (size_t)4 << 20;
static __device__ __align__(256) uint8_t scratch[NOALLOC_BYTES];

dv_status noalloc_setup(dv_ctx* ctx) {
  // the caller made ctx->device current
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    set_error("dv_ctx_create: locating the static workspace failed (%s)",
              hipGetErrorName(e));
    return DV_ERR_DEVICE;
  }
  ctx->noalloc_scratch = static_cast<uint8_t*>(p);
  ctx->noalloc_bytes = NOALLOC_BYTES;
  if (hipHostMalloc((void**)&ctx->noalloc_pinned, NOALLOC_PINNED_BYTES,
                    hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    ctx->noalloc_pinned = nullptr;
    set_error("dv_ctx_create: pinned staging allocation failed");
    return DV_ERR_OOM;
  }
  ctx->noalloc_pinned_bytes = NOALLOC_PINNED_BYTES;
  return DV_OK;
}

}  // namespace dv

using namespace dv;

extern "C" {

int64_t dv_noalloc_capacity(void) { return (int64_t)NOALLOC_BYTES; }

dv_status dv_render_noalloc(dv_ctx* ctx, const dv_scene* scene,
                            const dv_view* views, int32_t n_views,
                            const double* pose_override,
                            const dv_render_opts* opts, const dv_outputs* outs,
                            void* stream) {
  if (!ctx || !scene || !views || n_views < 1 || !outs) {
    set_error("dv_render_noalloc: invalid arguments");
    return DV_ERR_INVALID;
  }
  if (ctx->poisoned) {
    set_error("dv_render_noalloc: context poisoned by an earlier device error");
    return DV_ERR_DEVICE;
  }
  if (!ctx->noalloc_scratch || !ctx->noalloc_pinned) {
    set_error("dv_render_noalloc: the context has no static workspace");
    return DV_ERR_INVALID;
  }
  DV_TRY(check_opts(opts));
  DV_TRY_HIP(hipSetDevice(ctx->device));
  const hipStream_t s = (hipStream_t)stream;
  Arena ar;
  ar.base = ctx->noalloc_scratch;
  ar.cap = ctx->noalloc_bytes;
  ar.pinned = ctx->noalloc_pinned;
  ar.pinned_cap = ctx->noalloc_pinned_bytes;
  ArenaScope scope(&ar);
  // stage timers would create events: off for this call
  const int prof = ctx->prof_flags.exchange(0);
  dv_fwd_state st;
  st.ctx = ctx;
  st.scene = scene;
  st.stream = s;
  DV_TRY(check_feat_ptrs(*opts, scene));
  st.opts = effective_opts(*opts);
  dv_status rs = setup_state(&st, scene, views, n_views, pose_override);
  if (rs == DV_OK) rs = run_forward(ctx, scene, &st, outs, s, true);
  ctx->prof_flags = prof;
  if (rs == DV_ERR_DEVICE) ctx->poisoned = true;
  // the state's buffers are views into the workspace: nothing to free
  return rs;
}

}  // extern "C"
