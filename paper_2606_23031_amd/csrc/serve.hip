// Serving loop: sensor-simulation requests (camera, timestamp, resolution)
// against a resident scene (Sec. 1: the reconstruction serves novel views
// of the scene at new times and viewpoints).
//
// Continuous batching (batched = 1).  Two worker threads, each with its own
// stream, admit the oldest queued requests while request slots and the
// memory budget allow, up to max_batch at a time, and render them as the
// views of one multi-view launch sequence (preprocess, sorts, tile
// directories and compositing are each one launch for the whole batch).
// A request that arrives while both workers are busy joins the next batch
// a worker takes; with two batches in flight, one's preprocessing and
// sorts overlap the other's compositing.
//
// One launch per request (batched = 0), the baseline: the same two worker
// threads and streams, one request per dv_render call in arrival order.
//
// Persistent drain (batched = 2; refused by dv_serve_create in this build).
// A scheduler thread enqueues each group's front half (everything up to the
// background walks) on a prep stream and publishes the group's work items
// into a device ring; one persistent kernel on a second stream drains
// (group, item) work of every published group, and the block that writes a
// request's last tile raises the request's flag in host-mapped memory,
// which a completion thread watches.  On the GPU, a group after the first
// never raised its flags, with the cause not yet found; the code is kept
// for that investigation and is not reachable.
//
// Memory admission uses a running bytes-per-pixel estimate taken from the
// sizes of finished renders; a request is always admitted when nothing else
// is in flight.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <set>
#include <thread>
#include <unordered_map>

#include "render.h"

namespace dv {
dv_status check_opts(const dv_render_opts* op);
dv_render_opts effective_opts(const dv_render_opts& op);
dv_status setup_state(dv_fwd_state* st, const dv_scene* sc, const dv_view* views,
                      int32_t n_views, const double* pose_override);
dv_status run_forward(dv_ctx* ctx, const dv_scene* sc, dv_fwd_state* st,
                      const dv_outputs* outs, hipStream_t s, bool composite);
}

using namespace dv;

namespace {

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct Request {
  dv_view view;
  dv_outputs out;
  double t_submit = 0, t_admit = 0, t_done = 0;
  dv_status status = DV_PENDING;
  int64_t est_bytes = 0;
  bool done = false;
  int flag = -1;           // completion flag slot (batched mode)
};

// Host record of a published group.
struct Group {
  bool used = false;
  uint64_t number = 0;
  std::vector<uint64_t> tickets;
  int remaining = 0;
  dv_fwd_state* st = nullptr;
  DBuf counters;           // tile_ck [n_tiles] + view_done [n_views]
  DBuf vtab;               // view_ntiles, view_flag, view_seq
  int64_t used_bytes = 0, pixels = 0;
};

// Idle polls (about 3.5 us each) after which a drain block exits.
constexpr int DRAIN_IDLE_POLLS = 600;
// Requests per group (one view each) and the pinned staging per group slot:
// its ServeGroup, then per view the tile count, flag slot and flag value.
constexpr int MAX_GROUP_VIEWS = 256;
constexpr size_t STAGE_TABLE = ((size_t)MAX_GROUP_VIEWS * 16 + 64 + 255) & ~(size_t)255;
constexpr size_t STAGE_STRIDE = ((sizeof(ServeGroup) + 255) & ~(size_t)255) + STAGE_TABLE;
static_assert(STAGE_STRIDE % alignof(ServeGroup) == 0, "staging slots misaligned");

}  // namespace

struct dv_server {
  dv_ctx* ctx = nullptr;
  const dv_scene* scene = nullptr;
  dv_serve_opts opts{};
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<uint64_t> queue;
  std::unordered_map<uint64_t, Request> reqs;
  uint64_t next_ticket = 1;
  int inflight = 0;
  int64_t mem_inflight = 0;
  bool stop = false;
  double bytes_per_pixel = 512.0;   // running estimate
  std::vector<std::thread> workers;
  std::vector<hipStream_t> streams;
  // batched mode
  hipStream_t prep = nullptr, comp = nullptr;
  DBuf qbuf;                        // ServeQueue
  DBuf gbuf;                        // ServeGroup[SV_RING]: group g in entry g % SV_RING
  uint8_t* gstage = nullptr;        // pinned staging, STAGE_STRIDE per slot
  unsigned long long* flags = nullptr;      // host-mapped [SV_FLAGS]
  unsigned long long* flags_dev = nullptr;  // their device address
  std::vector<int> free_flags;
  Group groups[SV_GROUPS];
  std::vector<int> free_groups;
  uint64_t next_group = 0;
  std::set<uint64_t> live_nums;     // numbers of groups taken and not yet finished
  int groups_live = 0;
  bool drain_running = false;
  hipEvent_t drain_ev = nullptr;
  std::thread completer;

  void worker(int wid);
  void scheduler();
  void completion();
  // the oldest unfinished group (every older one has raised all its flags)
  uint64_t oldest_live() const {
    return live_nums.empty() ? next_group : *live_nums.begin();
  }
  // group next_group may take its argument entry: the group that used it
  // SV_RING numbers earlier has finished
  bool ring_entry_free() const { return oldest_live() + SV_RING > next_group; }
  bool admissible(const Request& r) const {
    if (inflight >= opts.max_inflight) return false;
    if (inflight == 0) return true;
    return mem_inflight + r.est_bytes <= opts.mem_budget;
  }
  void finish(uint64_t tk, dv_status rc, double t) {
    Request& r = reqs[tk];
    r.status = rc;
    r.t_done = t;
    r.done = true;
    inflight -= 1;
    mem_inflight -= r.est_bytes;
    if (r.flag >= 0) free_flags.push_back(r.flag);
    r.flag = -1;
  }
  void fail_queued(dv_status rc, double t) {
    for (uint64_t tk : queue) {
      Request& r = reqs[tk];
      r.status = rc;
      r.done = true;
      r.t_done = t;
    }
    queue.clear();
  }
};

// ---------------------------------------------------------------- workers
// Each worker thread owns one stream.  It admits the oldest queued
// requests while slots and the memory budget allow (at most max_batch of
// them when batching, one otherwise), renders them as the views of one
// multi-view launch sequence, waits for its stream and finishes them.
// Two workers keep two such launches in flight, so one batch's
// preprocessing and sorts overlap the other's compositing.
void dv_server::worker(int wid) {
  hipSetDevice(ctx->device);
  hipStream_t s = streams[wid];
  const int take = opts.batched ? std::max(1, opts.max_batch) : 1;
  std::vector<uint64_t> tks;
  std::vector<dv_view> views;
  std::vector<dv_outputs> outs;
  while (true) {
    tks.clear();
    views.clear();
    outs.clear();
    {
      std::unique_lock<std::mutex> lk(mu);
      cv_work.wait(lk, [&] {
        return (stop && queue.empty()) ||
               (!queue.empty() && admissible(reqs[queue.front()]));
      });
      if (queue.empty()) {
        if (stop) return;
        continue;
      }
      const double t = now_s();
      while (!queue.empty() && (int)tks.size() < take &&
             admissible(reqs[queue.front()])) {
        const uint64_t tk = queue.front();
        queue.pop_front();
        Request& r = reqs[tk];
        r.t_admit = t;
        inflight += 1;
        mem_inflight += r.est_bytes;
        tks.push_back(tk);
        views.push_back(r.view);
        outs.push_back(r.out);
      }
      if (tks.empty()) continue;
    }
    int64_t pixels = 0;
    for (auto& v : views) pixels += (int64_t)v.w * v.h;
    dv_fwd_state* st = nullptr;
    dv_status rc = ctx->poisoned
                       ? DV_ERR_DEVICE
                       : dv_render(ctx, scene, views.data(), (int32_t)views.size(),
                                   nullptr, &opts.opts, outs.data(), &st, s);
    int64_t used = 0;
    if (rc == DV_OK && st) {
      used = 24 * st->n_pairs + 150 * st->n_vis + 40 * st->n_tiles * TPB;
      dv_fwd_state_release(st);
    }
    if (rc == DV_OK && hipStreamSynchronize(s) != hipSuccess) {
      (void)hipGetLastError();
      rc = DV_ERR_DEVICE;
      ctx->poisoned = true;
    }
    {
      std::lock_guard<std::mutex> lk(mu);
      const double t = now_s();
      for (uint64_t tk : tks) finish(tk, rc, t);
      if (rc == DV_OK && pixels > 0)
        bytes_per_pixel = 0.8 * bytes_per_pixel + 0.2 * ((double)used / (double)pixels);
      if (rc == DV_ERR_DEVICE) fail_queued(DV_ERR_DEVICE, t);
    }
    cv_done.notify_all();
    cv_work.notify_all();
  }
}

// ---------------------------------------------------------------- batched
void dv_server::scheduler() {
  hipSetDevice(ctx->device);
  const int max_batch = std::max(1, opts.max_batch);
  std::vector<uint64_t> batch;
  std::vector<dv_view> views;
  std::vector<dv_outputs> outs;
  while (true) {
    int gslot = -1;
    uint64_t gnum = 0;
    batch.clear();
    views.clear();
    outs.clear();
    std::vector<int> bflags;
    {
      std::unique_lock<std::mutex> lk(mu);
      cv_work.wait(lk, [&] {
        return (stop && queue.empty()) ||
               (!queue.empty() && admissible(reqs[queue.front()]) &&
                !free_groups.empty() && !free_flags.empty() && ring_entry_free());
      });
      if (queue.empty()) {
        if (stop) return;
        continue;
      }
      if (!admissible(reqs[queue.front()]) || free_groups.empty() ||
          free_flags.empty() || !ring_entry_free())
        continue;
      gslot = free_groups.back();
      free_groups.pop_back();
      gnum = next_group++;
      live_nums.insert(gnum);
      const double t = now_s();
      while (!queue.empty() && (int)batch.size() < max_batch &&
             !free_flags.empty() && admissible(reqs[queue.front()])) {
        const uint64_t tk = queue.front();
        Request& r = reqs[tk];
        r.t_admit = t;
        r.flag = free_flags.back();
        free_flags.pop_back();
        inflight += 1;
        mem_inflight += r.est_bytes;
        batch.push_back(tk);
        views.push_back(r.view);
        outs.push_back(r.out);
        bflags.push_back(r.flag);
      }
      groups_live += 1;
    }
    Group& G = groups[gslot];
    int64_t pixels = 0;
    for (auto& v : views) pixels += (int64_t)v.w * v.h;
    int64_t used_bytes = 0;
    dv_status rc = ctx->poisoned ? DV_ERR_DEVICE : DV_OK;
    // front half of the group's render on the prep stream
    dv_fwd_state* st = nullptr;
    if (rc == DV_OK) {
      std::unique_ptr<dv_fwd_state> ps(new dv_fwd_state());
      ps->ctx = ctx;
      ps->scene = scene;
      ps->stream = prep;
      ps->opts = effective_opts(opts.opts);
      PoolStamp stamp_on_return(ctx);
      rc = setup_state(ps.get(), scene, views.data(), (int32_t)views.size(), nullptr);
      if (rc == DV_OK) rc = run_forward(ctx, scene, ps.get(), outs.data(), prep, false);
      const int nv = (int)views.size();
      const int64_t nt = ps->n_tiles;
      if (rc == DV_OK) rc = alloc_n<uint32_t>(ctx, G.counters, (size_t)nt + nv, prep);
      if (rc == DV_OK)
        rc = alloc_n<uint8_t>(ctx, G.vtab, (size_t)nv * 16 + 64, prep);
      if (rc == DV_OK) rc = fill_u32(G.counters.as<uint32_t>(), 0u, nt + nv, prep);
      if (rc == DV_OK) {
        // per view: tile count, flag slot, flag value (the ticket)
        uint8_t* slot_stage = gstage + (size_t)gslot * STAGE_STRIDE;
        ServeGroup& sg = *reinterpret_cast<ServeGroup*>(slot_stage);
        uint8_t* tab = slot_stage + ((sizeof(ServeGroup) + 255) & ~(size_t)255);
        uint32_t* ntl = reinterpret_cast<uint32_t*>(tab);
        uint32_t* fl = ntl + nv;
        unsigned long long* sq = reinterpret_cast<unsigned long long*>(
            tab + (((size_t)nv * 8 + 7) & ~(size_t)7));
        for (int v = 0; v < nv; ++v) {
          ntl[v] = (uint32_t)ps->views_h[v].ntx * ps->views_h[v].nty;
          fl[v] = (uint32_t)bflags[v];
          sq[v] = batch[v];
        }
        const size_t tab_bytes = (size_t)(reinterpret_cast<uint8_t*>(sq + nv) - tab);
        uint8_t* vt = G.vtab.as<uint8_t>();
        sg.a = ps->ca_fwd;
        sg.tile_ck = G.counters.as<uint32_t>();
        sg.view_done = G.counters.as<uint32_t>() + nt;
        sg.view_ntiles = reinterpret_cast<const uint32_t*>(vt);
        sg.view_flag = reinterpret_cast<const uint32_t*>(vt) + nv;
        sg.view_seq = reinterpret_cast<const unsigned long long*>(
            vt + (((size_t)nv * 8 + 7) & ~(size_t)7));
        sg.flags = flags_dev;
        ServeGroup* gd = gbuf.as<ServeGroup>() + (size_t)(gnum % SV_RING);
        hipError_t e = hipMemcpyAsync(vt, tab, tab_bytes, hipMemcpyHostToDevice, prep);
        if (e == hipSuccess)
          e = hipMemcpyAsync(gd, &sg, sizeof(ServeGroup), hipMemcpyHostToDevice, prep);
        if (e != hipSuccess) {
          (void)hipGetLastError();
          rc = DV_ERR_DEVICE;
        }
      }
      if (rc == DV_OK)
        rc = launch_serve_publish(qbuf.as<ServeQueue>(), gnum,
                                  ps->plan_counts.as<uint32_t>(), prep);
      if (rc == DV_OK) {
        used_bytes = 24 * ps->n_pairs + 150 * ps->n_vis + 40 * ps->n_tiles * TPB;
        st = ps.release();
      } else {
        // the group's buffers may still be read by queued prep work
        hipStreamSynchronize(prep);
        IdleRelease idle;
        ps.reset();
        G.counters.reset();
        G.vtab.reset();
      }
    }
    {
      std::lock_guard<std::mutex> lk(mu);
      if (rc != DV_OK) {
        if (rc == DV_ERR_DEVICE) ctx->poisoned = true;
        const double t = now_s();
        for (uint64_t tk : batch) finish(tk, rc, t);
        free_groups.push_back(gslot);
        live_nums.erase(gnum);
        groups_live -= 1;
        if (rc == DV_ERR_DEVICE) fail_queued(DV_ERR_DEVICE, t);
      } else {
        G.used = true;
        G.number = gnum;
        G.tickets = batch;
        G.remaining = (int)batch.size();
        G.pixels = pixels;
        G.used_bytes = used_bytes;
        G.st = st;
      }
    }
    cv_done.notify_all();
    cv_work.notify_all();
  }
}

void dv_server::completion() {
  hipSetDevice(ctx->device);
  while (true) {
    bool busy;
    uint64_t g_hi = 0;
    {
      std::lock_guard<std::mutex> lk(mu);
      busy = groups_live > 0;
      if (!busy && stop && queue.empty()) break;
      g_hi = oldest_live() + SV_RING / 2;
    }
    // keep one drain kernel running while groups are in flight
    if (drain_running) {
      const hipError_t q = hipEventQuery(drain_ev);
      if (q == hipSuccess) {
        drain_running = false;
      } else if (q != hipErrorNotReady) {
        (void)hipGetLastError();
        ctx->poisoned = true;
        drain_running = false;
      }
    }
    if (busy && !drain_running && !ctx->poisoned) {
      const bool nrm = (opts.opts.out_mask & DV_OUT_NORMAL) != 0;
      if (launch_serve_drain(qbuf.as<ServeQueue>(), gbuf.as<ServeGroup>(), nrm,
                             opts.opts.K == 1, 3 * std::max(ctx->n_cu, 1),
                             DRAIN_IDLE_POLLS, g_hi, comp) == DV_OK &&
          hipEventRecord(drain_ev, comp) == hipSuccess) {
        drain_running = true;
      } else {
        (void)hipGetLastError();
        ctx->poisoned = true;
      }
    }
    bool changed = false;
    std::vector<dv_fwd_state*> retire;
    {
      std::lock_guard<std::mutex> lk(mu);
      const double t = now_s();
      for (int gs = 0; gs < SV_GROUPS; ++gs) {
        Group& G = groups[gs];
        if (!G.used || !G.st) continue;
        for (uint64_t tk : G.tickets) {
          Request& r = reqs[tk];
          if (r.done || r.flag < 0) continue;
          const unsigned long long f = __atomic_load_n(flags + r.flag, __ATOMIC_ACQUIRE);
          if (f == tk) {
            finish(tk, DV_OK, t);
            G.remaining -= 1;
            changed = true;
          } else if (ctx->poisoned) {
            finish(tk, DV_ERR_DEVICE, t);
            G.remaining -= 1;
            changed = true;
          }
        }
        if (G.remaining == 0) {
          if (G.pixels > 0 && !ctx->poisoned)
            bytes_per_pixel = 0.8 * bytes_per_pixel +
                              0.2 * ((double)G.used_bytes / (double)G.pixels);
          retire.push_back(G.st);
          G.st = nullptr;
          {
            IdleRelease idle;
            G.counters.reset();
            G.vtab.reset();
          }
          G.used = false;
          free_groups.push_back(gs);
          live_nums.erase(G.number);
          groups_live -= 1;
        }
      }
      if (ctx->poisoned) fail_queued(DV_ERR_DEVICE, t);
    }
    if (!retire.empty()) {
      // every tile of these groups was written: no kernel reads their
      // buffers any more
      IdleRelease idle;
      for (dv_fwd_state* st : retire) delete st;
    }
    if (changed) {
      cv_done.notify_all();
      cv_work.notify_all();
    } else {
      std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
  }
  if (drain_running) hipEventSynchronize(drain_ev);
}

extern "C" {

dv_status dv_serve_create(dv_ctx* ctx, const dv_scene* scene,
                          const dv_serve_opts* opts, dv_server** out) {
  if (!ctx || !scene || !opts || !out || opts->max_inflight < 1 ||
      opts->mem_budget <= 0 || opts->max_batch < 1 || opts->batched < 0 ||
      opts->batched > 2) {
    set_error("dv_serve_create: invalid arguments");
    return DV_ERR_INVALID;
  }
  DV_TRY(check_opts(&opts->opts));
  if (opts->opts.feat) {
    set_error("dv_serve_create: feature renders are not served");
    return DV_ERR_INVALID;
  }
  DV_TRY_HIP(hipSetDevice(ctx->device));
  std::unique_ptr<dv_server> srv(new dv_server());
  srv->ctx = ctx;
  srv->scene = scene;
  srv->opts = *opts;
  srv->opts.max_inflight = std::min(opts->max_inflight, SV_FLAGS);
  if (opts->batched == 2) {
    // the persistent drain (scheduler + completion threads below): a
    // group after the first never raised its completion flags on the GPU,
    // and the cause is not yet found, so this mode is refused
    set_error("dv_serve_create: the persistent-drain mode (batched = 2) is "
              "disabled in this build");
    return DV_ERR_INVALID;
  }
  if (opts->batched == 0 || opts->batched == 1) {
    for (int i = 0; i < 2; ++i) {
      hipStream_t s;
      DV_TRY_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
      srv->streams.push_back(s);
    }
    for (int i = 0; i < 2; ++i)
      srv->workers.emplace_back(&dv_server::worker, srv.get(), i);
    *out = srv.release();
    return DV_OK;
  }
  DV_TRY_HIP(hipStreamCreateWithFlags(&srv->prep, hipStreamNonBlocking));
  srv->streams.push_back(srv->prep);
  DV_TRY_HIP(hipStreamCreateWithFlags(&srv->comp, hipStreamNonBlocking));
  srv->streams.push_back(srv->comp);
  DV_TRY_HIP(hipEventCreateWithFlags(&srv->drain_ev, hipEventDisableTiming));
  DV_TRY(alloc_n<uint8_t>(ctx, srv->qbuf, sizeof(ServeQueue), srv->prep));
  DV_TRY(alloc_n<ServeGroup>(ctx, srv->gbuf, SV_RING, srv->prep));
  DV_TRY(fill_u32(srv->qbuf.as<uint32_t>(), 0u, (int64_t)(sizeof(ServeQueue) / 4),
                  srv->prep));
  DV_TRY_HIP(hipStreamSynchronize(srv->prep));
  // pinned staging: per group slot its ServeGroup and per-view table
  DV_TRY_HIP(hipHostMalloc((void**)&srv->gstage, SV_GROUPS * STAGE_STRIDE,
                           hipHostMallocDefault));
  DV_TRY_HIP(hipHostMalloc((void**)&srv->flags, SV_FLAGS * sizeof(unsigned long long),
                           hipHostMallocCoherent | hipHostMallocMapped));
  std::memset(srv->flags, 0, SV_FLAGS * sizeof(unsigned long long));
  DV_TRY_HIP(hipHostGetDevicePointer((void**)&srv->flags_dev, srv->flags, 0));
  for (int i = SV_FLAGS - 1; i >= 0; --i) srv->free_flags.push_back(i);
  for (int i = SV_GROUPS - 1; i >= 0; --i) srv->free_groups.push_back(i);
  srv->opts.max_batch = std::min(opts->max_batch, MAX_GROUP_VIEWS);
  srv->workers.emplace_back(&dv_server::scheduler, srv.get());
  srv->completer = std::thread(&dv_server::completion, srv.get());
  *out = srv.release();
  return DV_OK;
}

dv_status dv_serve_submit(dv_server* srv, const dv_request* req,
                          uint64_t* ticket) {
  if (!srv || !req || !ticket) {
    set_error("dv_serve_submit: invalid arguments");
    return DV_ERR_INVALID;
  }
  Request r;
  r.view = req->view;
  r.out = req->out;
  r.t_submit = now_s();
  const dv_view& v = req->view;
  bool ok = v.fx > 0 && v.fy > 0 && v.w > 0 && v.h > 0 && v.x0 >= 0 &&
            v.y0 >= 0 && v.x0 + v.w <= v.W && v.y0 + v.h <= v.H &&
            std::isfinite(v.t) && std::isfinite(v.cx) && std::isfinite(v.cy);
  for (int i = 0; i < 12 && ok; ++i) ok = std::isfinite(v.c2w[i]);
  const uint32_t m = srv->opts.opts.out_mask;
  if ((m & DV_OUT_RGB) && !req->out.rgb) ok = false;
  if ((m & DV_OUT_DEPTH) && !req->out.depth) ok = false;
  if ((m & DV_OUT_NORMAL) && !req->out.normal) ok = false;
  if ((m & DV_OUT_T) && !req->out.T) ok = false;
  std::lock_guard<std::mutex> lk(srv->mu);
  if (srv->stop) {
    set_error("dv_serve_submit: server is shutting down");
    return DV_ERR_SHUTDOWN;
  }
  *ticket = srv->next_ticket++;
  if (!ok) {
    r.status = DV_ERR_INVALID;
    r.done = true;
    r.t_admit = r.t_done = r.t_submit;
    srv->reqs.emplace(*ticket, r);
    srv->cv_done.notify_all();
    return DV_OK;
  }
  r.est_bytes = (int64_t)(srv->bytes_per_pixel * (double)v.w * v.h);
  srv->reqs.emplace(*ticket, r);
  srv->queue.push_back(*ticket);
  srv->cv_work.notify_all();
  return DV_OK;
}

dv_status dv_serve_poll(dv_server* srv, uint64_t ticket, int32_t wait_us,
                        dv_result* res) {
  if (!srv) return DV_ERR_INVALID;
  std::unique_lock<std::mutex> lk(srv->mu);
  auto it = srv->reqs.find(ticket);
  if (it == srv->reqs.end()) {
    set_error("dv_serve_poll: unknown ticket %llu", (unsigned long long)ticket);
    return DV_ERR_TICKET;
  }
  auto pred = [&] { return srv->reqs[ticket].done; };
  if (!it->second.done && wait_us != 0) {
    if (wait_us < 0)
      srv->cv_done.wait(lk, pred);
    else
      srv->cv_done.wait_for(lk, std::chrono::microseconds(wait_us), pred);
  }
  Request& r = srv->reqs[ticket];
  if (res) {
    res->status = r.done ? r.status : DV_PENDING;
    res->t_submit = r.t_submit;
    res->t_admit = r.t_admit;
    res->t_done = r.t_done;
  }
  if (!r.done) return DV_PENDING;
  const dv_status st = r.status;
  srv->reqs.erase(ticket);
  return st;
}

dv_status dv_serve_destroy(dv_server* srv) {
  if (!srv) return DV_ERR_INVALID;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stop = true;
  }
  srv->cv_work.notify_all();
  for (auto& t : srv->workers) t.join();
  if (srv->completer.joinable()) srv->completer.join();
  hipSetDevice(srv->ctx->device);
  for (auto s : srv->streams) hipStreamSynchronize(s);
  // retired forward states release their buffers with events on the
  // worker streams: free them while those streams still exist
  reap_states(srv->ctx, true);
  {
    IdleRelease idle;
    for (auto& G : srv->groups) {
      if (G.st) delete G.st;
      G.st = nullptr;
      G.counters.reset();
      G.vtab.reset();
    }
    srv->qbuf.reset();
    srv->gbuf.reset();
  }
  srv->ctx->pool->stamp();
  for (auto s : srv->streams) hipStreamDestroy(s);
  if (srv->drain_ev) hipEventDestroy(srv->drain_ev);
  if (srv->gstage) hipHostFree(srv->gstage);
  if (srv->flags) hipHostFree(srv->flags);
  delete srv;
  return DV_OK;
}

}  // extern "C"
