// Solve server with continuous batching.
//
// Requests are queued in arrival order.  A worker thread admits the head of
// the queue whenever a slot is free and its device footprint (mesh arrays +
// solver state) fits the memory budget, uploads it, and from then on every
// tick advances all live requests together: one launch per kernel family
// and (dimension, precision) group covers every request that needs that
// step, so requests that arrive while others are on the device overlap with
// them.  The host work around the device work overlaps it: while a tick's
// launches run, the worker admits the next requests (allocation, uploads,
// initial launches queued behind the tick) and copies out the results of
// the requests that finished in the previous tick (on a second stream);
// their memory is freed once the tick has ended, before the next
// admission check.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <functional>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>

#include "mesh.h"
#include "solver.h"

using namespace pfem;

namespace {
struct Req {
  int64_t id = -1;
  pfem_mesh* m = nullptr;
  std::vector<double> u0;
  bool has_u0 = false;
  pfem_solve_opts o{};
  double t_submit = 0, t_admit = -1, t_done = -1;
  int64_t solve_b = 0;   // device bytes of the solve state (charged while live)
  int64_t mesh_b = 0;    // device bytes of the mesh arrays (charged while the
                         // server holds the mesh for one or more requests)
  SlotRun slot;
  bool admitted = false, done = false, server_uploaded = false;
  bool mesh_released = false;   // complete() released the server's copy of the mesh
  std::atomic<bool> cancel{false};   // set by the client, read by the worker
  std::vector<double> u_out;
  std::vector<double> u_int;   // the solution in internal order, copied from the device
  pfem_solve_report rep{};
};
}  // namespace

struct pfem_server {
  Ctx* c = nullptr;   // own stream and descriptor ring on the caller's device
  hipStream_t side = nullptr;   // result copies that overlap the next tick
  std::vector<Req*> pending;    // finished in the last tick, results not yet copied
  int64_t budget = 0;
  int max_slots = 0;
  std::thread worker;
  std::mutex mu;
  std::condition_variable cv;
  bool stop = false;
  std::deque<Req*> queue;
  std::vector<Req*> live;
  std::map<int64_t, Req*> all;
  std::deque<int64_t> done_ids;
  std::chrono::steady_clock::time_point t0;
  int64_t bytes_in_use = 0, peak_bytes = 0, peak_live = 0;
  int64_t submitted = 0, completed = 0, steps = 0, launches = 0;
  double admit_s = 0.0, tick_s = 0.0, complete_s = 0.0;   // worker host time
  std::string worker_error;
  std::map<pfem_mesh*, int> mesh_refs;   // meshes this server uploaded: live requests on each
  // kernel timing: a mask requested by the client (-1: no change), applied
  // by the worker at its next step; counters copied out after every step
  int timing_req = -1;
  pfem_kernel_stats kstats[FAM_COUNT] = {};

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  void run();
  void admit(Req* r);
  void collect(Req* r);
  void finish(Req* r);
  void complete(Req* r);
  void retire(Req* r);
  void fail(pfem_status code, const std::string& msg);
};

void pfem_server::admit(Req* r) {
  pfem_mesh* m = r->m;
  auto it = mesh_refs.find(m);
  if (it != mesh_refs.end()) {
    ++it->second;
    r->server_uploaded = true;
  } else if (!m->uploaded) {
    mesh_upload(m, c);
    mesh_refs[m] = 1;
    r->server_uploaded = true;
  }
  slot_alloc(&r->slot, m, r->o, 65536);
  r->slot.id = r->id;
  const double* u0_int = nullptr;
  if (r->has_u0) {
    // a synchronous copy outside the library stream: it does not wait for
    // the tick that may be running there (an asynchronous copy from pageable
    // memory on that stream would)
    PFEM_HIP(hipMemcpy(r->slot.st->g64, r->u0.data(), m->n_dof() * 8, hipMemcpyHostToDevice));
    launch_permute(c, PFEM_FP64, m->dim, m->dev.perm, m->n_nodes, true, r->slot.st->g64,
                   r->slot.st->aux64);
    u0_int = r->slot.st->aux64;
  }
  slot_begin(c, &r->slot, u0_int);
  r->admitted = true;
  r->t_admit = now();
}

// Queue the copy of a finished request's solution (internal order) on the
// side stream; the caller synchronises it.  Its slot is in no tick any
// more, so the library stream does not write it.
void pfem_server::collect(Req* r) {
  if (r->slot.st == nullptr) return;
  r->u_int.resize(r->m->n_dof());
  PFEM_HIP(hipMemcpyAsync(r->u_int.data(), r->slot.st->x64, r->m->n_dof() * 8,
                          hipMemcpyDeviceToHost, side));
}

// With the copy done and the library stream drained: the caller-order
// solution, the report, and the request's device memory returned.
void pfem_server::finish(Req* r) {
  pfem_mesh* m = r->m;
  if (!r->u_int.empty()) {
    const int D = m->dim;
    r->u_out.resize(m->n_dof());
    for (int64_t n = 0; n < m->n_nodes; ++n)
      for (int i = 0; i < D; ++i) r->u_out[n * D + i] = r->u_int[(int64_t)m->perm[n] * D + i];
    std::vector<double>().swap(r->u_int);
  }
  r->rep = r->slot.rep;
  r->rep.status = r->cancel ? PFEM_E_CANCELLED : r->slot.status;
  slot_free(&r->slot);
  if (r->server_uploaded && --mesh_refs[r->m] == 0) {
    mesh_refs.erase(r->m);
    mesh_release_device(r->m);
    r->mesh_released = true;
  }
  r->u0.clear();
  r->u0.shrink_to_fit();
  r->t_done = now();
}

void pfem_server::complete(Req* r) {
  collect(r);
  PFEM_HIP(hipStreamSynchronize(side));
  PFEM_HIP(hipStreamSynchronize(c->stream));
  finish(r);
}

// With mu held: the request leaves the live set and becomes visible to
// poll/result.  Only here (and in fail()) is done set, so a client never
// sees a request the worker still touches.
void pfem_server::retire(Req* r) {
  live.erase(std::find(live.begin(), live.end(), r));
  bytes_in_use -= r->solve_b + (r->mesh_released ? r->mesh_b : 0);
  r->done = true;
  done_ids.push_back(r->id);
  ++completed;
}

// With mu held: a device or host failure ends every live request with the
// error.  Requests taken from the queue for admission are live already.
void pfem_server::fail(pfem_status code, const std::string& msg) {
  worker_error = msg;
  pending.clear();   // all of them are live: ended below
  for (Req* r : live) {
    r->rep = r->slot.rep;
    r->rep.status = code;
    r->t_done = now();
    r->done = true;
    done_ids.push_back(r->id);
    ++completed;
    try {
      slot_free(&r->slot);
      // drop the server's mesh reference, as complete() does: the caller
      // may destroy the mesh once the result is collected
      if (r->server_uploaded && --mesh_refs[r->m] == 0) {
        mesh_refs.erase(r->m);
        mesh_release_device(r->m);
      }
    } catch (...) {
    }
    r->server_uploaded = false;
  }
  live.clear();
  bytes_in_use = 0;
}

void pfem_server::run() {
  (void)hipSetDevice(c->device);
  for (;;) {
    std::vector<Req*> to_admit;
    std::vector<Req*> cancelled_live;
    {
      std::unique_lock<std::mutex> lk(mu);
      cv.wait(lk, [&] { return stop || !queue.empty() || !live.empty(); });
      if (stop) break;
      if (timing_req >= 0) {
        c->drain_timing();
        c->timing = timing_req;
        c->sample_every = 1;
        for (int f = 0; f < FAM_COUNT; ++f) {
          c->fam_seen[f] = c->fam_launches[f] = c->fam_run[f] = 0;
          c->fam_ms[f] = c->fam_alg_bytes[f] = 0.0;
          kstats[f] = pfem_kernel_stats{};
        }
        timing_req = -1;
      }
      // cancellations in the queue finish at once
      for (auto it = queue.begin(); it != queue.end();) {
        Req* r = *it;
        if (r->cancel) {
          r->rep = pfem_solve_report{};
          r->rep.status = PFEM_E_CANCELLED;
          r->t_done = now();
          r->done = true;
          done_ids.push_back(r->id);
          ++completed;
          it = queue.erase(it);
        } else {
          ++it;
        }
      }
      for (Req* r : live)   // (a finished request is collected as usual)
        if (r->cancel && !r->slot.finished) cancelled_live.push_back(r);
    }
    try {
      for (Req* r : cancelled_live) {
        complete(r);
        std::lock_guard<std::mutex> lk(mu);
        retire(r);
      }
      {
        // admission in arrival order: the head of the queue waits for a
        // slot and for memory.  Charges: the request's solve state, plus the
        // mesh arrays when the server has to upload the mesh (neither
        // resident on a context of the caller nor held for another live
        // request, nor uploaded for an earlier request of this round).  Only
        // this thread uploads or releases meshes of queued or live requests,
        // so reading their residency here is race-free.  The requests become
        // live before admission, so that a failure while admitting ends them
        // too instead of losing them.
        std::lock_guard<std::mutex> lk(mu);
        std::vector<pfem_mesh*> planned;
        while (!queue.empty() && (int64_t)live.size() < max_slots) {
          Req* r = queue.front();
          const bool upload = !r->m->uploaded && mesh_refs.count(r->m) == 0 &&
                              std::find(planned.begin(), planned.end(), r->m) == planned.end();
          const int64_t need = r->solve_b + (upload ? r->mesh_b : 0);
          if (need > budget) {   // can never fit: end it instead of blocking the queue
            queue.pop_front();
            r->rep = pfem_solve_report{};
            r->rep.status = PFEM_E_OOM;
            r->t_done = now();
            r->done = true;
            done_ids.push_back(r->id);
            ++completed;
            continue;
          }
          if (bytes_in_use + need > budget) break;
          queue.pop_front();
          if (upload) planned.push_back(r->m);
          bytes_in_use += need;
          live.push_back(r);
          to_admit.push_back(r);
        }
        peak_bytes = std::max(peak_bytes, bytes_in_use);
        peak_live = std::max<int64_t>(peak_live, (int64_t)live.size());
      }
      // this tick: the live requests that were admitted before and have not
      // finished; during it, admit the new ones and copy out the results of
      // those that finished in the last tick
      std::vector<SlotRun*> slots;
      std::vector<Req*> snapshot;
      {
        std::lock_guard<std::mutex> lk(mu);
        snapshot = live;
      }
      for (Req* r : snapshot)
        if (std::find(to_admit.begin(), to_admit.end(), r) == to_admit.end() &&
            !r->slot.finished && r->slot.st != nullptr)
          slots.push_back(&r->slot);
      std::vector<Req*> collect_now;
      collect_now.swap(pending);
      double t_overlap = 0.0;
      const std::function<void()> overlap = [&] {
        const double t0 = now();
        for (Req* r : to_admit) admit(r);
        const double t1 = now();
        for (Req* r : collect_now) collect(r);
        if (!collect_now.empty()) PFEM_HIP(hipStreamSynchronize(side));
        const double t2 = now();
        t_overlap = t2 - t0;
        std::lock_guard<std::mutex> lk(mu);
        admit_s += t1 - t0;
        complete_s += t2 - t1;
      };
      if (!slots.empty()) {
        int64_t nl = 0;
        const double t0 = now();
        engine_tick(c, slots, &nl, &overlap);
        if (c->timing != 0) c->drain_timing();   // the step ended with a stream sync
        const double dt = now() - t0 - t_overlap;
        std::lock_guard<std::mutex> lk(mu);
        tick_s += dt;
        ++steps;
        launches += nl;
        for (int f = 0; f < FAM_COUNT; ++f)
          kstats[f] = pfem_kernel_stats{c->fam_launches[f], c->fam_ms[f], c->fam_run[f],
                                        c->fam_alg_bytes[f]};
      }
      if (slots.empty()) {   // nothing to step: the overlap work alone
        overlap();
        PFEM_HIP(hipStreamSynchronize(c->stream));
      }
      // the stream has drained: return the memory of the collected requests
      for (Req* r : collect_now) {
        const double t0 = now();
        finish(r);
        const double dt = now() - t0;
        std::lock_guard<std::mutex> lk(mu);
        complete_s += dt;
        retire(r);
      }
      // finished in this tick (or at admission): collected during the next
      for (Req* r : snapshot)
        if (r->slot.finished &&
            std::find(collect_now.begin(), collect_now.end(), r) == collect_now.end())
          pending.push_back(r);
    } catch (const pfem::Error& e) {
      std::lock_guard<std::mutex> lk(mu);
      fail(e.code, e.msg);
    } catch (const std::bad_alloc&) {
      std::lock_guard<std::mutex> lk(mu);
      fail(PFEM_E_OOM, "host memory exhausted in the server worker");
    } catch (const std::exception& e) {
      std::lock_guard<std::mutex> lk(mu);
      fail(PFEM_E_DEVICE, std::string("server worker: ") + e.what());
    }
  }
}

extern "C" {

pfem_status pfem_server_create(pfem_ctx* ctx, int64_t hbm_budget_bytes, int32_t max_slots,
                               pfem_server** out) {
  try {
    require(ctx != nullptr && out != nullptr, PFEM_E_INVALID_ARG, "NULL argument");
    require(hbm_budget_bytes > 0 && max_slots > 0, PFEM_E_INVALID_ARG, "bad budget or slots");
    *out = nullptr;
    const int device = ctx->c->device;
    PFEM_HIP(hipSetDevice(device));
    pfem_server* s = new pfem_server();
    s->c = new Ctx();
    s->c->device = device;
    s->budget = hbm_budget_bytes;
    s->max_slots = max_slots;
    try {
      PFEM_HIP(hipStreamCreateWithFlags(&s->c->stream, hipStreamNonBlocking));
      s->c->own_stream = true;
      PFEM_HIP(hipStreamCreateWithFlags(&s->side, hipStreamNonBlocking));
      s->c->ring.init(16u << 20, s->c->stream);
    } catch (...) {
      ctx_unref(s->c);
      delete s;
      throw;
    }
    s->t0 = std::chrono::steady_clock::now();
    s->worker = std::thread([s] { s->run(); });
    *out = s;
    set_error("");
    return PFEM_OK;
  } catch (const pfem::Error& e) {
    set_error(e.msg);
    return e.code;
  } catch (...) {
    set_error("server creation failed");
    return PFEM_E_DEVICE;
  }
}

pfem_status pfem_server_submit(pfem_server* s, pfem_mesh* m, const double* u0,
                               const pfem_solve_opts* o, int64_t req_id) {
  try {
    require(s != nullptr && m != nullptr && o != nullptr, PFEM_E_INVALID_ARG, "NULL argument");
    require(m->finalized, PFEM_E_STATE, "mesh not finalized");
    check_solve_opts(*o);
    Req* r = new Req();
    r->id = req_id;
    r->m = m;
    r->o = *o;
    r->has_u0 = u0 != nullptr;
    if (u0) r->u0.assign(u0, u0 + m->n_dof());
    // sizes fixed at finalize; residency is decided by the worker
    r->solve_b = solve_bytes(m, o->prec, krylov_fused(*o, m),
                             o->precond == PFEM_PRECOND_TWO_LEVEL);
    r->mesh_b = mesh_device_bytes(m);
    {
      std::lock_guard<std::mutex> lk(s->mu);
      if (s->all.count(req_id)) {
        delete r;
        throw Error{PFEM_E_INVALID_ARG, "duplicate request id"};
      }
      if (r->solve_b > s->budget) {
        delete r;
        throw Error{PFEM_E_OOM, "request footprint exceeds the server budget"};
      }
      r->t_submit = s->now();
      s->all[req_id] = r;
      s->queue.push_back(r);
      ++s->submitted;
    }
    s->cv.notify_one();
    set_error("");
    return PFEM_OK;
  } catch (const pfem::Error& e) {
    set_error(e.msg);
    return e.code;
  } catch (...) {
    set_error("submit failed");
    return PFEM_E_INVALID_ARG;
  }
}

pfem_status pfem_server_poll(pfem_server* s, int64_t* done_ids, int64_t cap, int64_t* n_done) {
  if (s == nullptr || n_done == nullptr || (cap > 0 && done_ids == nullptr)) {
    set_error("NULL argument");
    return PFEM_E_INVALID_ARG;
  }
  std::lock_guard<std::mutex> lk(s->mu);
  int64_t n = 0;
  while (!s->done_ids.empty() && n < cap) {
    done_ids[n++] = s->done_ids.front();
    s->done_ids.pop_front();
  }
  *n_done = n;
  set_error("");
  return PFEM_OK;
}

pfem_status pfem_server_result(pfem_server* s, int64_t req_id, double* u_out,
                               pfem_solve_report* rep, double* t_submit, double* t_admit,
                               double* t_done) {
  if (s == nullptr) {
    set_error("NULL server");
    return PFEM_E_INVALID_ARG;
  }
  Req* r = nullptr;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(req_id);
    if (it == s->all.end()) {
      set_error("unknown request id");
      return PFEM_E_INVALID_ARG;
    }
    if (!it->second->done) {
      set_error("request not finished");
      return PFEM_E_STATE;
    }
    r = it->second;
    s->all.erase(it);
  }
  if (u_out && !r->u_out.empty()) std::copy(r->u_out.begin(), r->u_out.end(), u_out);
  if (rep) *rep = r->rep;
  if (t_submit) *t_submit = r->t_submit;
  if (t_admit) *t_admit = r->t_admit;
  if (t_done) *t_done = r->t_done;
  const pfem_status st = r->rep.status;
  delete r;
  set_error("");
  return st < 0 ? st : PFEM_OK;
}

pfem_status pfem_server_cancel(pfem_server* s, int64_t req_id) {
  if (s == nullptr) {
    set_error("NULL server");
    return PFEM_E_INVALID_ARG;
  }
  {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(req_id);
    if (it == s->all.end()) {
      set_error("unknown request id");
      return PFEM_E_INVALID_ARG;
    }
    it->second->cancel = true;
  }
  s->cv.notify_one();
  set_error("");
  return PFEM_OK;
}

pfem_status pfem_server_get_stats(pfem_server* s, pfem_server_stats* o) {
  if (s == nullptr || o == nullptr) {
    set_error("NULL argument");
    return PFEM_E_INVALID_ARG;
  }
  std::lock_guard<std::mutex> lk(s->mu);
  o->submitted = s->submitted;
  o->completed = s->completed;
  o->live = (int64_t)s->live.size();
  o->queued = (int64_t)s->queue.size();
  o->peak_live = s->peak_live;
  o->bytes_in_use = s->bytes_in_use;
  o->peak_bytes = s->peak_bytes;
  o->budget = s->budget;
  o->steps = s->steps;
  o->launches = s->launches;
  o->admit_s = s->admit_s;
  o->tick_s = s->tick_s;
  o->complete_s = s->complete_s;
  set_error("");
  return PFEM_OK;
}

pfem_status pfem_server_set_timing(pfem_server* s, int family_mask) {
  if (s == nullptr || family_mask < 0) {
    set_error("NULL server or negative mask");
    return PFEM_E_INVALID_ARG;
  }
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->timing_req = family_mask;
    for (int f = 0; f < FAM_COUNT; ++f) s->kstats[f] = pfem_kernel_stats{};
  }
  s->cv.notify_one();
  set_error("");
  return PFEM_OK;
}

pfem_status pfem_server_kernel_stats(pfem_server* s, int family, pfem_kernel_stats* out) {
  if (s == nullptr || out == nullptr || family < 0 || family >= FAM_COUNT) {
    set_error("NULL argument or bad kernel family");
    return PFEM_E_INVALID_ARG;
  }
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->kstats[family];
  set_error("");
  return PFEM_OK;
}

void pfem_server_destroy(pfem_server* s) {
  if (s == nullptr) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv.notify_all();
  if (s->worker.joinable()) s->worker.join();
  (void)hipSetDevice(s->c->device);
  (void)hipStreamSynchronize(s->c->stream);
  if (s->side != nullptr) {
    (void)hipStreamSynchronize(s->side);
    (void)hipStreamDestroy(s->side);
  }
  for (Req* r : s->live) {
    try {
      slot_free(&r->slot);
    } catch (...) {
    }
  }
  for (auto& kv : s->mesh_refs) {
    try {
      mesh_release_device(kv.first);
    } catch (...) {
    }
  }
  for (auto& kv : s->all) delete kv.second;
  ctx_unref(s->c);
  delete s;
}

}  // extern "C"
