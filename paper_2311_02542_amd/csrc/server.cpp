// Serving engine of the C ABI (include/vrn.h, vrn_server_*): continuous
// batching of render requests of mixed resolutions over the resident fields
// of one context.
//
// One scheduler thread per engine makes every device call of serving:
//   * a slot is a HIP stream (default priority) with its own workspace, a
//     pinned camera buffer, its device copy and a completion event;
//   * a bucket is (field, W, H, cameras in the launch); each slot keeps, per
//     bucket, a ring of output buffers carved from one device arena, each
//     with a captured graph (camera upload from the slot's pinned buffer,
//     then the render into that buffer), so a launch is a memcpy into pinned
//     memory and one graph launch;
//   * when a slot is free the oldest pending request is taken, with the
//     single-camera requests of the same field and size queued behind it,
//     up to max_batch cameras in one launch;
//   * results are the ring buffers themselves, held until the client
//     releases the request; every buffer lives in the arena, and free
//     buffers are evicted least-recently-used when a new one does not fit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <iterator>
#include <map>
#include <mutex>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "internal.hpp"

using namespace vrn;

namespace {

constexpr uint64_t kAlign = 256;

uint64_t align_up(uint64_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// First-fit allocator over the arena; free ranges keyed by offset and
// merged with their neighbours on release.
class Arena {
 public:
  void reset(uint8_t* base, uint64_t bytes) {
    base_ = base;
    size_ = bytes;
    free_.clear();
    if (bytes) free_[0] = bytes;
  }
  uint8_t* alloc(uint64_t bytes) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      const uint64_t off = it->first, len = it->second;
      free_.erase(it);
      if (len > bytes) free_[off + bytes] = len - bytes;
      return base_ + off;
    }
    return nullptr;
  }
  void release(uint8_t* p, uint64_t bytes) {
    uint64_t off = (uint64_t)(p - base_), len = bytes;
    auto next = free_.lower_bound(off);
    if (next != free_.end() && off + len == next->first) {
      len += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        prev->second += len;
        return;
      }
    }
    free_[off] = len;
  }
  uint64_t largest() const {
    uint64_t m = 0;
    for (const auto& kv : free_) m = std::max(m, kv.second);
    return m;
  }
  uint64_t free_bytes() const {
    uint64_t m = 0;
    for (const auto& kv : free_) m += kv.second;
    return m;
  }
  uint64_t size() const { return size_; }

 private:
  uint8_t* base_ = nullptr;
  uint64_t size_ = 0;
  std::map<uint64_t, uint64_t> free_;
};

typedef std::tuple<vrn_field_id, uint32_t, uint32_t, uint32_t> Key;  // field, W, H, cameras

uint64_t rgba_bytes(uint32_t n, uint32_t W, uint32_t H) { return align_up((uint64_t)n * W * H * 16); }
uint64_t buffer_bytes(uint32_t n, uint32_t W, uint32_t H) {
  return rgba_bytes(n, W, H) + align_up((uint64_t)n * W * H * 4);
}

struct OutBuf {
  uint8_t* mem = nullptr;
  uint64_t bytes = 0;
  vrn_field_id field = 0;
  float* rgba = nullptr;
  uint32_t* ns = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int holders = 0;  // requests in flight, or finished and not released
  double last_use = 0.0;
};

struct SReq {
  uint64_t id = 0;
  vrn_field_id field = 0;
  uint32_t W = 0, H = 0, n_cams = 0;
  vrn_camera cams[kMaxCams];
  double t_arrival = 0.0, t_launch = 0.0, t_done = 0.0, deadline = 0.0;  // deadline 0: none
  uint32_t flags = 0;
  bool done = false, cancelled = false;
  int32_t status = VRN_ERR_BUSY;
  OutBuf* out = nullptr;
  uint32_t off = 0;  // first camera of this request in the buffer
};

struct SSlot {
  hipStream_t stream = nullptr;
  void* ws = nullptr;
  vrn_camera* d_cams = nullptr;
  vrn_camera* h_cams = nullptr;  // pinned
  hipEvent_t ev = nullptr;
  std::map<Key, std::vector<OutBuf*>> rings;
  std::vector<SReq*> busy;  // the launch in flight
};

}  // namespace

struct vrn_server {
  vrn_ctx* ctx = nullptr;
  int device = 0;
  vrn_server_opts opts{};
  Arena arena;
  void* arena_owned = nullptr;  // allocated by the engine when the caller gave no arena
  std::vector<SSlot> slots;
  std::mutex mu;
  std::condition_variable cv;       // wakes the scheduler: submit, release, hold, stop
  std::condition_variable done_cv;  // wakes waiters: requests finished
  std::deque<SReq*> pending;
  std::unordered_map<uint64_t, SReq*> reqs;
  uint64_t next_id = 1;
  bool hold = true;
  bool stop = false;
  std::thread th;
  hipError_t fault = hipSuccess;  // first HIP error seen in serving
  vrn_serve_stats counts{};       // event counters (launches ... failed)
};

namespace {

void note_fault(vrn_server* sv, hipError_t e) {
  if (e != hipSuccess && sv->fault == hipSuccess) sv->fault = e;
}

void free_out(vrn_server* sv, OutBuf* o) {
  if (o->exec) hipGraphExecDestroy(o->exec);
  if (o->graph) hipGraphDestroy(o->graph);
  sv->arena.release(o->mem, o->bytes);
  field_pin(sv->ctx, o->field, -1);
  delete o;
}

// A new ring buffer for key on slot, captured into a graph when the engine
// uses graphs (mu held; the slot is idle or is synchronised first).
// VRN_ERR_BUDGET when the arena has no room for it.
vrn_status new_out(vrn_server* sv, SSlot& slot, const Key& key, OutBuf** out) {
  const vrn_field_id field = std::get<0>(key);
  const uint32_t W = std::get<1>(key), H = std::get<2>(key), n = std::get<3>(key);
  const uint64_t bytes = buffer_bytes(n, W, H);
  uint8_t* mem = sv->arena.alloc(bytes);
  if (!mem) return set_error(VRN_ERR_BUDGET, "no room in the serving arena");
  vrn_status st = field_pin(sv->ctx, field, +1);
  if (st != VRN_OK) {
    sv->arena.release(mem, bytes);
    return st;
  }
  OutBuf* o = new OutBuf();
  o->mem = mem;
  o->bytes = bytes;
  o->field = field;
  o->rgba = reinterpret_cast<float*>(mem);
  o->ns = reinterpret_cast<uint32_t*>(mem + rgba_bytes(n, W, H));
  if (sv->opts.use_graphs) {
    hipError_t e = hipStreamSynchronize(slot.stream);
    if (e == hipSuccess) e = hipStreamBeginCapture(slot.stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      const hipError_t ec = hipMemcpyAsync(slot.d_cams, slot.h_cams, n * sizeof(vrn_camera),
                                           hipMemcpyHostToDevice, slot.stream);
      if (ec == hipSuccess)
        st = vrn_render_device_cams(sv->ctx, field, slot.d_cams, n, W, H, &sv->opts.render, o->rgba, o->ns,
                                    slot.ws, (uint64_t)kWsBytes, slot.stream);
      // the capture ends whatever happened inside it
      e = hipStreamEndCapture(slot.stream, &o->graph);
      if (e == hipSuccess) e = ec;
    }
    if (e == hipSuccess && st == VRN_OK) e = hipGraphInstantiate(&o->exec, o->graph, nullptr, nullptr, 0);
    if (e != hipSuccess || st != VRN_OK) {
      note_fault(sv, e);
      free_out(sv, o);
      return st != VRN_OK ? st : set_error(VRN_ERR_DEVICE, hipGetErrorString(e));
    }
    sv->counts.captures += 1;
  }
  o->last_use = now_s();
  slot.rings[key].push_back(o);
  *out = o;
  return VRN_OK;
}

// A free ring buffer for key on slot: an existing one, else a new one,
// evicting free buffers least-recently-used while the arena has no room for
// it (mu held, slot idle).  VRN_ERR_BUDGET when nothing is left to evict.
vrn_status acquire_out(vrn_server* sv, SSlot& slot, const Key& key, OutBuf** out) {
  auto it = slot.rings.find(key);
  if (it != slot.rings.end())
    for (OutBuf* o : it->second)
      if (o->holders == 0) {
        o->last_use = now_s();
        *out = o;
        return VRN_OK;
      }
  while (true) {
    const vrn_status st = new_out(sv, slot, key, out);
    if (st != VRN_ERR_BUDGET) return st;
    // a buffer without holders is in no launch in flight
    SSlot* vs = nullptr;
    Key vk;
    size_t vi = 0;
    double oldest = 0.0;
    for (SSlot& s : sv->slots)
      for (auto& kv : s.rings)
        for (size_t i = 0; i < kv.second.size(); ++i) {
          const OutBuf* o = kv.second[i];
          if (o->holders == 0 && (!vs || o->last_use < oldest)) {
            vs = &s;
            vk = kv.first;
            vi = i;
            oldest = o->last_use;
          }
        }
    if (!vs) return VRN_ERR_BUDGET;
    std::vector<OutBuf*>& ring = vs->rings[vk];
    OutBuf* victim = ring[vi];
    ring.erase(ring.begin() + (long)vi);
    if (ring.empty()) vs->rings.erase(vk);
    free_out(sv, victim);
    sv->counts.evictions += 1;
  }
}

uint64_t held_bytes(const vrn_server* sv) {
  uint64_t b = 0;
  for (const SSlot& s : sv->slots)
    for (const auto& kv : s.rings)
      for (const OutBuf* o : kv.second)
        if (o->holders > 0) b += o->bytes;
  return b;
}

// Caller notifies done_cv.
void finish(vrn_server* sv, SReq* r, int32_t status, double t) {
  r->status = status;
  r->t_done = t;
  r->done = true;
  if ((status != VRN_OK || (r->flags & VRN_SERVE_RELEASE_ON_DONE)) && r->out) {
    r->out->holders -= 1;
    r->out = nullptr;
  }
  if (status == VRN_OK) sv->counts.completed += 1;
  else sv->counts.failed += 1;
}

// 1: the batch was launched (or failed for good); 0: its output buffer does
// not fit the arena now.
int launch(vrn_server* sv, SSlot& slot, const std::vector<SReq*>& batch) {
  const SReq* r0 = batch[0];
  uint32_t n = 0;
  for (const SReq* r : batch) n += r->n_cams;
  OutBuf* o = nullptr;
  const vrn_status st = acquire_out(sv, slot, Key(r0->field, r0->W, r0->H, n), &o);
  if (st == VRN_ERR_BUDGET) return 0;
  if (st != VRN_OK) {
    const double t = now_s();
    for (SReq* r : batch) finish(sv, r, st == VRN_ERR_NOT_FOUND ? VRN_ERR_NOT_FOUND : VRN_ERR_DEVICE, t);
    sv->done_cv.notify_all();
    return 1;
  }
  // the slot is idle, so its previous camera upload has completed
  uint32_t off = 0;
  for (const SReq* r : batch) {
    std::memcpy(slot.h_cams + off, r->cams, r->n_cams * sizeof(vrn_camera));
    off += r->n_cams;
  }
  hipError_t e = hipSuccess;
  vrn_status rs = VRN_OK;
  if (o->exec) {
    e = hipGraphLaunch(o->exec, slot.stream);
  } else {
    e = hipMemcpyAsync(slot.d_cams, slot.h_cams, n * sizeof(vrn_camera), hipMemcpyHostToDevice, slot.stream);
    if (e == hipSuccess)
      rs = vrn_render_device_cams(sv->ctx, r0->field, slot.d_cams, n, r0->W, r0->H, &sv->opts.render, o->rgba,
                                  o->ns, slot.ws, (uint64_t)kWsBytes, slot.stream);
  }
  if (e == hipSuccess && rs == VRN_OK) e = hipEventRecord(slot.ev, slot.stream);
  const double t = now_s();
  if (e != hipSuccess || rs != VRN_OK) {
    note_fault(sv, e);
    for (SReq* r : batch) finish(sv, r, rs == VRN_ERR_NOT_FOUND ? VRN_ERR_NOT_FOUND : VRN_ERR_DEVICE, t);
    sv->done_cv.notify_all();
    return 1;
  }
  off = 0;
  for (SReq* r : batch) {
    r->out = o;
    r->off = off;
    r->t_launch = t;
    o->holders += 1;
    off += r->n_cams;
  }
  slot.busy = batch;
  sv->counts.launches += 1;
  if (o->exec) sv->counts.graph_launches += 1;
  sv->counts.merged_requests += batch.size() - 1;
  return 1;
}

void poll(vrn_server* sv) {
  bool any = false;
  for (SSlot& s : sv->slots) {
    if (s.busy.empty()) continue;
    const hipError_t q = hipEventQuery(s.ev);
    if (q == hipErrorNotReady) continue;
    const double t = now_s();
    note_fault(sv, q);
    for (SReq* r : s.busy) {
      int32_t st = VRN_OK;
      if (q != hipSuccess) st = VRN_ERR_DEVICE;
      else if (r->cancelled) st = VRN_ERR_CANCELLED;
      else if (r->deadline > 0.0 && t > r->deadline) st = VRN_ERR_TIMEOUT;
      finish(sv, r, st, t);
    }
    s.busy.clear();
    any = true;
  }
  if (any) sv->done_cv.notify_all();
}

// Fail queued requests whose deadline has passed (never launched).
void expire(vrn_server* sv) {
  const double t = now_s();
  bool any = false;
  for (auto it = sv->pending.begin(); it != sv->pending.end();) {
    SReq* r = *it;
    if (r->deadline > 0.0 && t > r->deadline) {
      finish(sv, r, VRN_ERR_TIMEOUT, t);
      it = sv->pending.erase(it);
      any = true;
    } else {
      ++it;
    }
  }
  if (any) sv->done_cv.notify_all();
}

// The oldest pending request plus the single-camera requests of the same
// field and size behind it, up to max_batch cameras (and no more than one
// buffer the arena could hold).
std::vector<SReq*> take_batch(vrn_server* sv) {
  std::vector<SReq*> batch;
  SReq* head = sv->pending.front();
  sv->pending.pop_front();
  batch.push_back(head);
  if (head->n_cams != 1) return batch;
  uint32_t limit = sv->opts.max_batch;
  while (limit > 1 && buffer_bytes(limit, head->W, head->H) > sv->arena.size()) --limit;
  for (auto it = sv->pending.begin(); it != sv->pending.end() && batch.size() < limit;) {
    SReq* r = *it;
    if (r->n_cams == 1 && r->field == head->field && r->W == head->W && r->H == head->H) {
      batch.push_back(r);
      it = sv->pending.erase(it);
    } else {
      ++it;
    }
  }
  return batch;
}

void requeue(vrn_server* sv, const std::vector<SReq*>& batch, size_t from) {
  for (size_t i = batch.size(); i-- > from;) sv->pending.push_front(batch[i]);
}

void loop(vrn_server* sv) {
  hipSetDevice(sv->device);
  std::unique_lock<std::mutex> lk(sv->mu);
  while (!sv->stop) {
    poll(sv);
    expire(sv);
    bool launched = false;
    if (!sv->hold && !sv->pending.empty()) {
      SSlot* free_slot = nullptr;
      size_t n_free = 0;
      for (SSlot& s : sv->slots)
        if (s.busy.empty()) {
          ++n_free;
          if (!free_slot) free_slot = &s;
        }
      if (free_slot) {
        const std::vector<SReq*> batch = take_batch(sv);
        if (launch(sv, *free_slot, batch)) {
          launched = true;
        } else if (n_free == sv->slots.size()) {
          // nothing in flight will free memory: shrink to the head request;
          // if even that does not fit it waits for held results to be
          // released, and fails only when none are held
          requeue(sv, batch, 1);
          if (launch(sv, *free_slot, {batch[0]})) {
            launched = true;
          } else if (held_bytes(sv) > 0) {
            sv->pending.push_front(batch[0]);
          } else {
            finish(sv, batch[0], VRN_ERR_BUDGET, now_s());
            sv->done_cv.notify_all();
          }
        } else {
          requeue(sv, batch, 0);
        }
      }
    }
    if (launched) continue;
    bool busy = false;
    for (const SSlot& s : sv->slots) busy = busy || !s.busy.empty();
    if (busy) {
      // renders in flight: query their events again at once
      lk.unlock();
      std::this_thread::yield();
      lk.lock();
    } else {
      // idle, held, or waiting for a held result to be released; bounded,
      // so that queued deadlines are still checked
      sv->cv.wait_for(lk, std::chrono::milliseconds(1));
    }
  }
}

bool valid_render_opts(const vrn_render_opts& o) {
  return (o.compute == VRN_F32 || o.compute == VRN_F16 || o.compute == VRN_BF16 || o.compute == VRN_F32X) &&
         o.output >= VRN_OUT_PQ &&
         o.output <= VRN_OUT_SRGB && std::isfinite(o.exposure_ev) && std::fabs(o.exposure_ev) <= 64.0f;
}

void destroy_slots(vrn_server* sv) {
  for (SSlot& s : sv->slots) {
    for (auto& kv : s.rings)
      for (OutBuf* o : kv.second) free_out(sv, o);
    s.rings.clear();
    if (s.ev) hipEventDestroy(s.ev);
    if (s.h_cams) hipHostFree(s.h_cams);
    if (s.d_cams) hipFree(s.d_cams);
    if (s.ws) hipFree(s.ws);
    if (s.stream) hipStreamDestroy(s.stream);
  }
  sv->slots.clear();
  if (sv->arena_owned) hipFree(sv->arena_owned);
  sv->arena_owned = nullptr;
}

SReq* find_req(vrn_server* sv, uint64_t id) {
  auto it = sv->reqs.find(id);
  return it == sv->reqs.end() ? nullptr : it->second;
}

std::chrono::steady_clock::time_point after(double seconds) {
  const double s = std::min(std::max(0.0, seconds), 1e6);
  return std::chrono::steady_clock::now() +
         std::chrono::duration_cast<std::chrono::steady_clock::duration>(std::chrono::duration<double>(s));
}

}  // namespace

extern "C" {

vrn_status vrn_server_create(vrn_ctx* ctx, const vrn_server_opts* opts, vrn_server** out) {
  if (!ctx || !opts || !out) return set_error(VRN_ERR_INVALID_ARG, "ctx, opts or out is NULL");
  *out = nullptr;
  if (opts->n_slots < 1 || opts->n_slots > 16) return set_error(VRN_ERR_INVALID_ARG, "n_slots must be 1..16");
  if (opts->max_batch < 1 || opts->max_batch > (uint32_t)kMaxCams)
    return set_error(VRN_ERR_INVALID_ARG, "max_batch must be 1..VRN_MAX_CAMS");
  if (opts->use_graphs != 0 && opts->use_graphs != 1)
    return set_error(VRN_ERR_INVALID_ARG, "use_graphs must be 0 or 1");
  if (!valid_render_opts(opts->render))
    return set_error(VRN_ERR_INVALID_ARG, "render options out of range (compute, output or exposure_ev)");
  const uint64_t arena_bytes = opts->arena_bytes & ~(kAlign - 1);
  if (arena_bytes < kAlign) return set_error(VRN_ERR_INVALID_ARG, "arena_bytes must be >= 256");
  if (opts->d_arena && (reinterpret_cast<uintptr_t>(opts->d_arena) & (kAlign - 1)))
    return set_error(VRN_ERR_INVALID_ARG, "d_arena must be 256-byte aligned");
  vrn_server* sv = new vrn_server();
  sv->ctx = ctx;
  sv->device = ctx_device(ctx);
  sv->opts = *opts;
  hipError_t e = hipSetDevice(sv->device);
  void* base = opts->d_arena;
  if (e == hipSuccess && !base) {
    e = hipMalloc(&sv->arena_owned, arena_bytes);
    base = sv->arena_owned;
  }
  sv->arena.reset(static_cast<uint8_t*>(base), arena_bytes);
  sv->slots.resize(opts->n_slots);
  for (SSlot& s : sv->slots) {
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipMalloc(&s.ws, kWsBytes);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&s.d_cams), kMaxCams * sizeof(vrn_camera));
    if (e == hipSuccess)
      e = hipHostMalloc(reinterpret_cast<void**>(&s.h_cams), kMaxCams * sizeof(vrn_camera), hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s.ev, hipEventDisableTiming);
    if (e == hipSuccess) e = launch_zero(s.ws, kWsBytes, s.stream);
  }
  for (SSlot& s : sv->slots)
    if (e == hipSuccess && s.stream) e = hipStreamSynchronize(s.stream);
  if (e != hipSuccess) {
    destroy_slots(sv);
    delete sv;
    return set_error(e == hipErrorOutOfMemory ? VRN_ERR_OUT_OF_MEMORY : VRN_ERR_DEVICE, hipGetErrorString(e));
  }
  sv->th = std::thread(loop, sv);
  *out = sv;
  return VRN_OK;
}

void vrn_server_destroy(vrn_server* sv) {
  if (!sv) return;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
  }
  sv->cv.notify_all();
  if (sv->th.joinable()) sv->th.join();
  hipSetDevice(sv->device);
  for (SSlot& s : sv->slots) hipStreamSynchronize(s.stream);
  destroy_slots(sv);
  for (auto& kv : sv->reqs) delete kv.second;
  delete sv;
}

vrn_status vrn_server_hold(vrn_server* sv, int hold) {
  if (!sv) return set_error(VRN_ERR_INVALID_ARG, "server is NULL");
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->hold = hold != 0;
  }
  sv->cv.notify_all();
  return VRN_OK;
}

vrn_status vrn_server_prepare(vrn_server* sv, vrn_field_id field, uint32_t n_cams, uint32_t W, uint32_t H) {
  if (!sv) return set_error(VRN_ERR_INVALID_ARG, "server is NULL");
  if (n_cams < 1 || n_cams > (uint32_t)kMaxCams || W < 1 || H < 1 || W > 16384 || H > 16384 ||
      (uint64_t)n_cams * W * H > (1ull << 31))
    return set_error(VRN_ERR_INVALID_ARG, "n_cams must be 1..16 and W, H 1..16384 (at most 2^31 pixels)");
  uint64_t fb = 0;
  vrn_status st = vrn_field_bytes(sv->ctx, field, &fb);
  if (st != VRN_OK) return st;
  std::lock_guard<std::mutex> lk(sv->mu);
  hipSetDevice(sv->device);
  const Key key(field, W, H, n_cams);
  for (SSlot& s : sv->slots) {
    auto it = s.rings.find(key);
    if (it != s.rings.end() && !it->second.empty()) continue;
    OutBuf* o = nullptr;
    if ((st = new_out(sv, s, key, &o)) != VRN_OK) return st;
  }
  return VRN_OK;
}

vrn_status vrn_server_submit(vrn_server* sv, vrn_field_id field, const vrn_camera* cams, uint32_t n_cams, uint32_t W,
                             uint32_t H, const vrn_request_opts* opts, uint64_t* id) {
  if (!sv || !id) return set_error(VRN_ERR_INVALID_ARG, "server or id is NULL");
  vrn_status st = vrn_check_cameras(cams, n_cams, W, H);
  if (st != VRN_OK) return st;
  const vrn_request_opts ro = opts ? *opts : vrn_request_opts{0.0, 0.0, 0u};
  if (!std::isfinite(ro.t_arrival)) return set_error(VRN_ERR_INVALID_ARG, "t_arrival must be finite");
  if (!std::isfinite(ro.timeout_s) || ro.timeout_s < 0.0)
    return set_error(VRN_ERR_INVALID_ARG, "timeout_s must be finite and >= 0 (0: none)");
  if (ro.flags & ~VRN_SERVE_RELEASE_ON_DONE) return set_error(VRN_ERR_INVALID_ARG, "unknown request flags");
  uint64_t fb = 0;
  if ((st = vrn_field_bytes(sv->ctx, field, &fb)) != VRN_OK) return st;
  if (buffer_bytes(n_cams, W, H) > sv->arena.size())
    return set_error(VRN_ERR_BUDGET, "the request's outputs exceed the serving arena");
  SReq* r = new SReq();
  r->field = field;
  r->W = W;
  r->H = H;
  r->n_cams = n_cams;
  std::memcpy(r->cams, cams, n_cams * sizeof(vrn_camera));
  r->flags = ro.flags;
  r->t_arrival = ro.t_arrival > 0.0 ? ro.t_arrival : now_s();
  r->deadline = ro.timeout_s > 0.0 ? r->t_arrival + ro.timeout_s : 0.0;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    r->id = sv->next_id++;
    sv->reqs[r->id] = r;
    sv->pending.push_back(r);
  }
  sv->cv.notify_all();
  *id = r->id;
  return VRN_OK;
}

vrn_status vrn_server_wait(vrn_server* sv, uint64_t id, double max_wait_s, vrn_served* out) {
  if (!sv || !out) return set_error(VRN_ERR_INVALID_ARG, "server or out is NULL");
  if (!(max_wait_s >= 0.0)) return set_error(VRN_ERR_INVALID_ARG, "max_wait_s must be >= 0");
  std::unique_lock<std::mutex> lk(sv->mu);
  SReq* r = find_req(sv, id);
  if (!r) return set_error(VRN_ERR_NOT_FOUND, "unknown or released request id");
  if (!r->done && max_wait_s > 0.0) sv->done_cv.wait_until(lk, after(max_wait_s), [r] { return r->done; });
  std::memset(out, 0, sizeof(*out));
  out->field = r->field;
  out->n_cams = r->n_cams;
  out->W = r->W;
  out->H = r->H;
  out->t_arrival = r->t_arrival;
  out->t_launch = r->t_launch;
  if (!r->done) {
    out->status = VRN_ERR_BUSY;
    return set_error(VRN_ERR_BUSY, "request not finished");
  }
  out->status = r->status;
  out->t_done = r->t_done;
  if (r->out) {
    const size_t px = (size_t)r->W * r->H;
    out->d_rgba = r->out->rgba + (size_t)r->off * px * 4;
    out->d_nsamples = r->out->ns + (size_t)r->off * px;
  }
  return VRN_OK;
}

vrn_status vrn_server_release(vrn_server* sv, uint64_t id) {
  if (!sv) return set_error(VRN_ERR_INVALID_ARG, "server is NULL");
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    SReq* r = find_req(sv, id);
    if (!r) return set_error(VRN_ERR_NOT_FOUND, "unknown or released request id");
    if (!r->done) return set_error(VRN_ERR_BUSY, "request not finished (cancel it first)");
    if (r->out) r->out->holders -= 1;
    sv->reqs.erase(id);
    delete r;
  }
  sv->cv.notify_all();
  return VRN_OK;
}

vrn_status vrn_server_cancel(vrn_server* sv, uint64_t id) {
  if (!sv) return set_error(VRN_ERR_INVALID_ARG, "server is NULL");
  std::lock_guard<std::mutex> lk(sv->mu);
  SReq* r = find_req(sv, id);
  if (!r) return set_error(VRN_ERR_NOT_FOUND, "unknown or released request id");
  if (r->done) return set_error(VRN_ERR_BUSY, "request already finished");
  r->cancelled = true;
  auto p = std::find(sv->pending.begin(), sv->pending.end(), r);
  if (p != sv->pending.end()) {
    sv->pending.erase(p);
    finish(sv, r, VRN_ERR_CANCELLED, now_s());
    sv->done_cv.notify_all();
  }
  return VRN_OK;
}

vrn_status vrn_server_drain(vrn_server* sv, double max_wait_s) {
  if (!sv) return set_error(VRN_ERR_INVALID_ARG, "server is NULL");
  const auto until = after(max_wait_s);
  std::unique_lock<std::mutex> lk(sv->mu);
  auto idle = [sv] {
    if (!sv->pending.empty()) return false;
    for (const SSlot& s : sv->slots)
      if (!s.busy.empty()) return false;
    return true;
  };
  if (!sv->done_cv.wait_until(lk, until, idle)) return set_error(VRN_ERR_BUSY, "requests still queued or running");
  return VRN_OK;
}

vrn_status vrn_server_evict(vrn_server* sv, vrn_field_id field) {
  if (!sv) return set_error(VRN_ERR_INVALID_ARG, "server is NULL");
  std::lock_guard<std::mutex> lk(sv->mu);
  bool left = false;
  for (SSlot& s : sv->slots)
    for (auto it = s.rings.begin(); it != s.rings.end();) {
      if (field != 0 && std::get<0>(it->first) != field) {
        ++it;
        continue;
      }
      std::vector<OutBuf*>& ring = it->second;
      for (size_t i = ring.size(); i-- > 0;)
        if (ring[i]->holders == 0) {
          free_out(sv, ring[i]);
          ring.erase(ring.begin() + (long)i);
          sv->counts.evictions += 1;
        }
      if (ring.empty()) {
        it = s.rings.erase(it);
      } else {
        left = true;
        ++it;
      }
    }
  return left ? set_error(VRN_ERR_BUSY, "buffers held by requests remain") : VRN_OK;
}

vrn_status vrn_server_stats(vrn_server* sv, vrn_serve_stats* out) {
  if (!sv || !out) return set_error(VRN_ERR_INVALID_ARG, "server or out is NULL");
  std::lock_guard<std::mutex> lk(sv->mu);
  *out = sv->counts;
  out->arena_bytes = sv->arena.size();
  out->used_bytes = sv->arena.size() - sv->arena.free_bytes();
  out->held_bytes = held_bytes(sv);
  out->largest_free_bytes = sv->arena.largest();
  out->pending = sv->pending.size();
  out->running = 0;
  out->buffers = 0;
  out->buckets = 0;
  for (const SSlot& s : sv->slots) {
    out->running += s.busy.size();
    for (const auto& kv : s.rings) {
      out->buffers += kv.second.size();
      out->buckets += 1;
    }
  }
  out->requests = sv->reqs.size();
  if (sv->fault != hipSuccess) return set_error(VRN_ERR_DEVICE, hipGetErrorString(sv->fault));
  return VRN_OK;
}

double vrn_server_clock(void) { return now_s(); }

}  // extern "C"
