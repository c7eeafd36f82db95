// Serving loop: sensor-simulation requests (camera, timestamp, resolution)
// against a resident scene.
//
// Continuous batching: worker threads, each with its own HIP stream, take
// the queued requests that fit the free slots and the memory budget and
// render them together in one multi-view launch; requests arriving while
// batches are on the GPU wait in the queue and are admitted by the next
// free worker, so preprocessing and sorting of one batch overlap the
// compositing of another on the device.  In per-request mode a single
// worker renders one request per launch in FIFO order.  Memory admission
// uses a running bytes-per-pixel estimate taken from the sizes of finished
// launches; a request is always admitted when nothing else is in flight.
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <thread>
#include <unordered_map>

#include "render.h"

namespace dv {
dv_status check_opts(const dv_render_opts* op);
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
};

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

  void worker(int wid);
  bool admissible(const Request& r) const {
    if (inflight >= opts.max_inflight) return false;
    if (inflight == 0) return true;
    return mem_inflight + r.est_bytes <= opts.mem_budget;
  }
};

void dv_server::worker(int wid) {
  hipSetDevice(ctx->device);
  hipStream_t s = streams[wid];
  const int max_batch = opts.batched ? std::max(1, opts.max_batch) : 1;
  std::vector<uint64_t> batch;
  std::vector<dv_view> views;
  std::vector<dv_outputs> outs;
  while (true) {
    batch.clear();
    {
      std::unique_lock<std::mutex> lk(mu);
      cv_work.wait(lk, [&] {
        return stop || (!queue.empty() && admissible(reqs[queue.front()]));
      });
      if (stop && queue.empty()) return;
      if (queue.empty()) continue;
      if (!admissible(reqs[queue.front()])) {
        // only reachable while stopping: wait for in-flight work to drain
        cv_done.wait_for(lk, std::chrono::milliseconds(1));
        continue;
      }
      const double t = now_s();
      while (!queue.empty() && (int)batch.size() < max_batch) {
        Request& r = reqs[queue.front()];
        if (!batch.empty() && !admissible(r)) break;
        if (batch.empty() && !admissible(r)) break;
        r.t_admit = t;
        inflight += 1;
        mem_inflight += r.est_bytes;
        batch.push_back(queue.front());
        queue.pop_front();
      }
      views.clear();
      outs.clear();
      for (uint64_t tk : batch) {
        views.push_back(reqs[tk].view);
        outs.push_back(reqs[tk].out);
      }
    }
    if (batch.empty()) continue;
    dv_fwd_state* st = nullptr;
    dv_status rc = ctx->poisoned ? DV_ERR_DEVICE
                                 : dv_render(ctx, scene, views.data(),
                                             (int32_t)views.size(), nullptr,
                                             &opts.opts, outs.data(), &st, s);
    int64_t used = 0, pixels = 0;
    if (rc == DV_OK && st) {
      used = 24 * st->n_pairs + 150 * st->n_vis + 40 * st->n_tiles * TPB;
      dv_fwd_state_release(st);
    }
    if (rc == DV_OK && hipStreamSynchronize(s) != hipSuccess) {
      (void)hipGetLastError();
      rc = DV_ERR_DEVICE;
      ctx->poisoned = true;
    }
    for (auto& v : views) pixels += (int64_t)v.w * v.h;
    {
      std::lock_guard<std::mutex> lk(mu);
      const double t = now_s();
      for (uint64_t tk : batch) {
        Request& r = reqs[tk];
        r.status = rc;
        r.t_done = t;
        r.done = true;
        inflight -= 1;
        mem_inflight -= r.est_bytes;
      }
      if (rc == DV_OK && pixels > 0)
        bytes_per_pixel = 0.8 * bytes_per_pixel + 0.2 * ((double)used / pixels);
      if (rc == DV_ERR_DEVICE) {
        // a device fault poisons the context: fail everything still queued
        for (uint64_t tk : queue) {
          Request& r = reqs[tk];
          r.status = DV_ERR_DEVICE;
          r.done = true;
          r.t_done = t;
        }
        queue.clear();
      }
    }
    cv_done.notify_all();
    cv_work.notify_all();
  }
}

extern "C" {

dv_status dv_serve_create(dv_ctx* ctx, const dv_scene* scene,
                          const dv_serve_opts* opts, dv_server** out) {
  if (!ctx || !scene || !opts || !out || opts->max_inflight < 1 ||
      opts->mem_budget <= 0 || opts->max_batch < 1) {
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
  const int nw = opts->batched ? 2 : 1;
  for (int i = 0; i < nw; ++i) {
    hipStream_t s;
    DV_TRY_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    srv->streams.push_back(s);
  }
  for (int i = 0; i < nw; ++i)
    srv->workers.emplace_back(&dv_server::worker, srv.get(), i);
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
  srv->cv_work.notify_one();
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
  hipSetDevice(srv->ctx->device);
  for (auto s : srv->streams) hipStreamSynchronize(s);
  // retired forward states release their buffers with events on the
  // worker streams: free them while those streams still exist
  reap_states(srv->ctx, true);
  srv->ctx->pool->stamp();
  for (auto s : srv->streams) hipStreamDestroy(s);
  delete srv;
  return DV_OK;
}

}  // extern "C"
