// Host runtime pieces: error reporting, launch-descriptor ring, kernel timing.
#include <algorithm>

#include "pfem_internal.h"
#include "ring_math.h"

namespace pfem {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }
const char* last_error_cstr() { return g_last_error.c_str(); }

// ------------------------------------------------------------------ ArgRing
void ArgRing::init(size_t bytes, hipStream_t s) {
  stream_ = s;
  cap_ = bytes;
  PFEM_HIP(hipHostMalloc((void**)&host_, cap_, hipHostMallocDefault));
  PFEM_HIP(hipMalloc((void**)&dev_, cap_));
  for (int i = 0; i < kSeg; ++i) {
    PFEM_HIP(hipEventCreateWithFlags(&ev_[i], hipEventDisableTiming));
    used_[i] = false;
  }
  off_ = 0;
  seg_ = 0;
}

void ArgRing::release() {
  if (stream_ != nullptr) (void)hipStreamSynchronize(stream_);
  for (int i = 0; i < kSeg; ++i)
    if (ev_[i] != nullptr) (void)hipEventDestroy(ev_[i]);
  if (host_ != nullptr) (void)hipHostFree(host_);
  if (dev_ != nullptr) (void)hipFree(dev_);
  host_ = dev_ = nullptr;
}

void* ArgRing::put(const void* src, size_t n) {
  const size_t seg_bytes = cap_ / kSeg;
  const size_t need = (n + 255) & ~size_t(255);
  require(need <= seg_bytes, PFEM_E_INVALID_ARG,
          "launch descriptor larger than the staging segment");
  int seg = 0;
  const size_t off = ring_place(off_, need, seg_bytes, kSeg, &seg);
  if (seg != seg_) {
    // leaving seg_: everything that used it has been enqueued
    PFEM_HIP(hipEventRecord(ev_[seg_], stream_));
    used_[seg_] = true;
    if (used_[seg]) PFEM_HIP(hipEventSynchronize(ev_[seg]));
    seg_ = seg;
  }
  std::memcpy(host_ + off, src, n);
  PFEM_HIP(hipMemcpyAsync(dev_ + off, host_ + off, n, hipMemcpyHostToDevice, stream_));
  off_ = off + need;
  return dev_ + off;
}

// ---------------------------------------------------------------- context
void ctx_ref(Ctx* c) { c->refs.fetch_add(1); }

void ctx_unref(Ctx* c) {
  if (c == nullptr || c->refs.fetch_sub(1) != 1) return;
  (void)hipSetDevice(c->device);
  if (c->stream != nullptr) (void)hipStreamSynchronize(c->stream);
  c->ring.release();
  for (auto& p : c->pending) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  for (hipEvent_t e : c->event_pool) (void)hipEventDestroy(e);
  if (c->own_stream && c->stream != nullptr) (void)hipStreamDestroy(c->stream);
  delete c;
}

// ---------------------------------------------------------------- timing
void Ctx::timing_begin(int fam, hipEvent_t* a) {
  *a = nullptr;
  if (!(timing & (1 << fam))) return;
  if (fam_seen[fam]++ % sample_every != 0) return;
  if (event_pool.empty()) {
    hipEvent_t e;
    PFEM_HIP(hipEventCreate(&e));
    event_pool.push_back(e);
  }
  *a = event_pool.back();
  event_pool.pop_back();
  PFEM_HIP(hipEventRecord(*a, stream));
}

void Ctx::timing_end(int fam, hipEvent_t a) { timing_end_run(fam, a, 1); }

void Ctx::timing_begin_run(int fam, hipEvent_t* a) {
  *a = nullptr;
  if (!(timing & (1 << fam))) return;
  if (event_pool.empty()) {
    hipEvent_t e;
    PFEM_HIP(hipEventCreate(&e));
    event_pool.push_back(e);
  }
  *a = event_pool.back();
  event_pool.pop_back();
  PFEM_HIP(hipEventRecord(*a, stream));
}

void Ctx::timing_end_run(int fam, hipEvent_t a, int count) {
  if (a == nullptr) return;
  if (event_pool.empty()) {
    hipEvent_t e;
    PFEM_HIP(hipEventCreate(&e));
    event_pool.push_back(e);
  }
  hipEvent_t b = event_pool.back();
  event_pool.pop_back();
  PFEM_HIP(hipEventRecord(b, stream));
  pending.push_back({fam, a, b, cur_key, count > 1 ? 0 : cur_it, count});
  if (pending.size() > 8192 && cur_key < 0) drain_timing();
}

void Ctx::drop_noop(int64_t key, int keep) {
  std::vector<Timed> kept;
  kept.reserve(pending.size());
  for (const Timed& t : pending) {
    if (t.key == key && t.it + t.count > keep) {
      event_pool.push_back(t.a);
      event_pool.push_back(t.b);
    } else {
      kept.push_back(t);
    }
  }
  pending.swap(kept);
}

void Ctx::drain_timing() {
  for (const Timed& t : pending) {
    PFEM_HIP(hipEventSynchronize(t.b));
    float ms = 0.f;
    PFEM_HIP(hipEventElapsedTime(&ms, t.a, t.b));
    fam_ms[t.fam] += ms;
    fam_launches[t.fam] += t.count;
    event_pool.push_back(t.a);
    event_pool.push_back(t.b);
  }
  pending.clear();
}

}  // namespace pfem
