// Serving: asynchronous event streams, continuously batched onto one context.
//
// Slices are independent (every neighbourhood lies inside its slice,
// Sec. 2.1), so slices of different streams and sensors can share one batch
// call and the result of each is the same as alone.  Every open stream keeps
// its count and pair grids resident on the device: a region of the server's
// grid arena, taken at veckm_stream_open (admission: the region must fit in
// the arena the HBM budget pays for) and reused by each of its slices (the
// encoder returns the counted voxels to zero, so the region is clean for the
// next slice).  A launcher thread packs waiting slices, at most one per
// stream, into batches while a device lane is free; each lane has its own
// event and flow buffers, so the host-to-device copy of one batch (on a copy
// stream) overlaps the kernels of the other (on the compute stream), and the
// copy of its flows back runs on a third stream.  A completer thread waits
// for each batch in order, checks its device error bits and hands the flows
// to the pollers.  A batch that reports an input error has its slices run
// again one by one, so only the offending slice gets the error.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "veckm_internal.h"

using namespace veckm;
using Clock = std::chrono::steady_clock;

namespace {

constexpr int kLanes = 2;  // batches on the device at once, each with its own buffers
constexpr int kMaxDepth = 16;

struct Slot {  // pinned host staging of one submitted slice
  veckm_event* ev = nullptr;
  float* flow = nullptr;
  bool busy = false;
};

struct Stream {
  bool open = false;
  int W = 0, H = 0, T = 0;
  int64_t max_events = 0;
  Capacity share;
  int64_t grid_at = 0, pair_at = 0;  // its resident count / pair grid region
  std::vector<Slot> slots;
  int outstanding = 0;  // submitted and not complete
  int copying = 0;      // results being copied out by veckm_poll
};

// First-fit allocator of [offset, offset + length) regions in an arena.
struct Arena {
  int64_t size = 0;
  std::vector<std::pair<int64_t, int64_t>> used;  // sorted by offset
  bool take(int64_t len, int64_t* at) {
    int64_t pos = 0;
    size_t i = 0;
    for (; i < used.size(); ++i) {
      if (used[i].first - pos >= len) break;
      pos = used[i].first + used[i].second;
    }
    if (i == used.size() && size - pos < len) return false;
    used.insert(used.begin() + (long)i, {pos, len});
    *at = pos;
    return true;
  }
  void give(int64_t at) {
    for (size_t i = 0; i < used.size(); ++i)
      if (used[i].first == at) {
        used.erase(used.begin() + (long)i);
        return;
      }
  }
};

struct Ticket {
  uint64_t id = 0;
  int sid = 0, slot = 0;
  int64_t n = 0;
  int t0 = 0, nbins = 0;
  bool solo = false;  // run alone: its batch reported an input error
  bool done = false;
  int status = VECKM_OK;
  Clock::time_point submitted, completed;
};

struct InFlight {
  std::vector<Ticket*> tickets;
  int lane = -1;
  hipEvent_t copied = nullptr, computed = nullptr, done = nullptr;
  int32_t* err = nullptr;  // pinned: the batch's device error bits
};

// What one batch can take (the grids are resident, so only the per-call
// workspaces count).
bool fits(const Capacity& used, const Capacity& need, const Capacity& cap) {
  return used.events + need.events <= cap.events && used.bricks + need.bricks <= cap.bricks &&
         used.slices + need.slices <= cap.slices;
}

void add(Capacity& a, const Capacity& b, int sign) {
  a.events += sign * b.events;
  a.voxels += sign * b.voxels;
  a.pairs += sign * b.pairs;
  a.bricks += sign * b.bricks;
  a.slices += sign * b.slices;
}

}  // namespace

struct veckm_server {
  veckm_ctx* ctx = nullptr;
  veckm_params p{};
  int device = 0;
  hipStream_t stream = nullptr;  // kernels
  hipStream_t h2d = nullptr;     // events in
  hipStream_t d2h = nullptr;     // flows out
  int depth = 1;
  Capacity cap, reserved;
  Arena grid_arena, pair_arena;  // resident stream grids (voxels, pair entries)
  veckm_event* ev_dev[kLanes] = {};
  float* flow_dev[kLanes] = {};
  bool lane_busy[kLanes] = {};
  std::vector<Stream> streams;
  // `mu` guards everything below and the stream table
  std::mutex mu;
  std::condition_variable cv_launch, cv_complete, cv_done;
  std::deque<Ticket*> pending;
  std::unordered_map<uint64_t, Ticket*> tickets;
  std::deque<InFlight> inflight;
  std::vector<InFlight> spare;  // reusable events and error words
  uint64_t next_ticket = 1;
  bool stop = false;
  bool has_mlp = false;
  std::mutex ctx_mu;  // calls on the context (which is not thread-safe)
  std::thread launcher, completer;
  std::vector<double> lat_ms;
  std::vector<int64_t> lat_sensor;  // W << 32 | H of each latency sample
  int64_t done_slices = 0, done_flows = 0, batches = 0;
  bool have_first = false;
  Clock::time_point first_submit, last_done;
};

namespace {

int take_flight(veckm_server* s, InFlight* f) {
  if (!s->spare.empty()) {
    *f = s->spare.back();
    s->spare.pop_back();
    f->tickets.clear();
    return VECKM_OK;
  }
  InFlight g;
  for (hipEvent_t* e : {&g.copied, &g.computed, &g.done})
    if (hipEventCreateWithFlags(e, hipEventDisableTiming) != hipSuccess) {
      for (hipEvent_t x : {g.copied, g.computed, g.done})
        if (x) (void)hipEventDestroy(x);
      return VECKM_E_HIP;
    }
  if (!pinned_malloc(reinterpret_cast<void**>(&g.err), sizeof(int32_t))) {
    for (hipEvent_t x : {g.copied, g.computed, g.done}) (void)hipEventDestroy(x);
    return VECKM_E_NOMEM;
  }
  *f = g;
  return VECKM_OK;
}

void drop_flight(InFlight& f) {
  for (hipEvent_t x : {f.copied, f.computed, f.done})
    if (x) (void)hipEventDestroy(x);
  if (f.err) (void)hipHostFree(f.err);
}

// Completes a ticket (caller holds mu).
void finish(veckm_server* s, Ticket* t, int status, Clock::time_point now) {
  t->done = true;
  t->status = status;
  t->completed = now;
  const Stream& st = s->streams[t->sid];
  s->streams[t->sid].outstanding -= 1;
  s->lat_ms.push_back(std::chrono::duration<double, std::milli>(now - t->submitted).count());
  s->lat_sensor.push_back((int64_t)st.W << 32 | st.H);
  s->done_slices += 1;
  s->done_flows += t->n;
  s->last_done = now;
}

// Enqueues one batch on lane f.lane: its events in on the copy stream, the
// kernels on the compute stream once they have landed, its flows out on the
// second copy stream once the kernels are done; f.done marks the end.
int enqueue(veckm_server* s, const std::vector<Ticket*>& take, InFlight& f) {
  std::lock_guard<std::mutex> g(s->ctx_mu);
  std::vector<veckm_slice> sl(take.size());
  std::vector<int64_t> at(2 * take.size());
  veckm_event* ev_dev = s->ev_dev[f.lane];
  float* flow_dev = s->flow_dev[f.lane];
  int64_t off = 0;
  for (size_t k = 0; k < take.size(); ++k) {
    const Ticket* t = take[k];
    const Stream& st = s->streams[t->sid];
    sl[k].width = st.W;
    sl[k].height = st.H;
    sl[k].t0 = t->t0;
    sl[k].nbins = t->nbins;
    sl[k].offset = off;
    sl[k].n = t->n;
    at[2 * k] = st.grid_at;
    at[2 * k + 1] = st.pair_at;
    if (t->n > 0 && hipMemcpyAsync(ev_dev + off, st.slots[t->slot].ev,
                                   (size_t)t->n * sizeof(veckm_event), hipMemcpyHostToDevice,
                                   s->h2d) != hipSuccess)
      return VECKM_E_HIP;
    off += t->n;
  }
  if (hipEventRecord(f.copied, s->h2d) != hipSuccess ||
      hipStreamWaitEvent(s->stream, f.copied, 0) != hipSuccess)
    return VECKM_E_HIP;
  int rc = flow_batch_at(s->ctx, sl.data(), (int32_t)sl.size(), at.data(), ev_dev, flow_dev,
                         s->stream);
  if (rc) return rc;
  rc = ctx_take_err(s->ctx, f.err, s->stream);
  if (rc) return rc;
  if (hipEventRecord(f.computed, s->stream) != hipSuccess ||
      hipStreamWaitEvent(s->d2h, f.computed, 0) != hipSuccess)
    return VECKM_E_HIP;
  off = 0;
  for (const Ticket* t : take) {
    const Stream& st = s->streams[t->sid];
    if (t->n > 0 && hipMemcpyAsync(st.slots[t->slot].flow, flow_dev + 2 * off,
                                   (size_t)t->n * 2 * sizeof(float), hipMemcpyDeviceToHost,
                                   s->d2h) != hipSuccess)
      return VECKM_E_HIP;
    off += t->n;
  }
  return hipEventRecord(f.done, s->d2h) == hipSuccess ? VECKM_OK : VECKM_E_HIP;
}

int free_lane(const veckm_server* s) {
  for (int l = 0; l < kLanes; ++l)
    if (!s->lane_busy[l]) return l;
  return -1;
}

void launcher_main(veckm_server* s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    s->cv_launch.wait(lk, [s] {
      return s->stop || (!s->pending.empty() && free_lane(s) >= 0);
    });
    if (s->stop) return;
    // waiting slices in submission order while they fit, at most one per
    // stream (a stream's slices share its resident grid); a slice marked
    // solo runs alone
    std::vector<Ticket*> take;
    Capacity used;
    if (s->pending.front()->solo) {
      take.push_back(s->pending.front());
      s->pending.pop_front();
    } else {
      std::vector<char> in_batch(s->streams.size(), 0);
      for (auto it = s->pending.begin(); it != s->pending.end();) {
        Ticket* t = *it;
        if (t->solo) break;
        if (in_batch[(size_t)t->sid]) {  // its stream's next slice: next batch
          ++it;
          continue;
        }
        const Stream& st = s->streams[t->sid];
        const Capacity need = slice_need(s->ctx, st.W, st.H, t->nbins, t->n);
        if (!fits(used, need, s->cap)) break;
        add(used, need, 1);
        in_batch[(size_t)t->sid] = 1;
        take.push_back(t);
        it = s->pending.erase(it);
      }
    }
    if (take.empty()) {  // cannot happen for admitted streams; never spin on it
      Ticket* t = s->pending.front();
      s->pending.pop_front();
      finish(s, t, VECKM_E_RANGE, Clock::now());
      s->cv_done.notify_all();
      continue;
    }
    InFlight f;
    int rc = take_flight(s, &f);
    f.lane = free_lane(s);
    s->lane_busy[f.lane] = true;
    lk.unlock();
    if (!rc) rc = enqueue(s, take, f);
    lk.lock();
    if (rc) {
      // whatever was enqueued must finish before the lane is reused
      (void)hipStreamSynchronize(s->h2d);
      (void)hipStreamSynchronize(s->stream);
      (void)hipStreamSynchronize(s->d2h);
      const Clock::time_point now = Clock::now();
      for (Ticket* t : take) finish(s, t, rc, now);
      s->lane_busy[f.lane] = false;
      if (f.done) s->spare.push_back(f);
      s->cv_done.notify_all();
      continue;
    }
    f.tickets = std::move(take);
    s->inflight.push_back(f);
    s->batches += 1;
    s->cv_complete.notify_one();
  }
}

void completer_main(veckm_server* s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    s->cv_complete.wait(lk, [s] { return s->stop || !s->inflight.empty(); });
    if (s->inflight.empty()) return;  // stopping, and the device is drained
    InFlight f = s->inflight.front();
    lk.unlock();
    const hipError_t e = hipEventSynchronize(f.done);
    const Clock::time_point now = Clock::now();
    lk.lock();
    s->inflight.pop_front();
    const int code = e != hipSuccess ? VECKM_E_HIP : err_code(*f.err);
    if (code != VECKM_OK && e == hipSuccess && f.tickets.size() > 1 && !s->stop) {
      // an input error in a shared batch: run its slices one by one
      for (auto it = f.tickets.rbegin(); it != f.tickets.rend(); ++it) {
        (*it)->solo = true;
        s->pending.push_front(*it);
      }
    } else {
      for (Ticket* t : f.tickets) finish(s, t, code, now);
    }
    f.tickets.clear();
    s->lane_busy[f.lane] = false;
    s->spare.push_back(f);
    s->cv_launch.notify_one();
    s->cv_done.notify_all();
  }
}

void free_slots(Stream& st) {
  for (Slot& sl : st.slots) {
    if (sl.ev) (void)hipHostFree(sl.ev);
    if (sl.flow) (void)hipHostFree(sl.flow);
  }
  st.slots.clear();
}

}  // namespace

extern "C" {

int veckm_server_create(const veckm_params* params, int64_t hbm_budget_bytes, int32_t max_streams,
                        int32_t depth, veckm_server** out) {
  if (!out) return VECKM_E_INVAL;
  *out = nullptr;
  if (!params || max_streams < 1 || depth < 1 || depth > kMaxDepth || hbm_budget_bytes <= 0)
    return VECKM_E_INVAL;
  veckm_params p = *params;
  if (p.max_slices < max_streams) p.max_slices = max_streams;
  // the resident grid arena: by default room for every stream at the
  // largest sensor and slice length
  if (p.max_voxels == 0) p.max_voxels = (int64_t)p.width * p.height * p.max_bins * max_streams;
  int rc = veckm_params_check(&p);
  if (rc) return rc;
  if (p.rt < 0) return VECKM_E_INVAL;  // batches need the temporally bounded encoder
  const int64_t ws = veckm_workspace_bytes(&p, 512);
  if (ws < 0) return (int)ws;
  const int64_t bytes =
      ws + kLanes * p.max_events * (int64_t)(sizeof(veckm_event) + 2 * sizeof(float));
  if (bytes > hbm_budget_bytes) return VECKM_E_BUDGET;
  veckm_server* s = new (std::nothrow) veckm_server();
  if (!s) return VECKM_E_NOMEM;
  s->p = p;
  s->depth = depth;
  rc = veckm_create(&p, &s->ctx);
  if (!rc && hipGetDevice(&s->device) != hipSuccess) rc = VECKM_E_HIP;
  const size_t nev = (size_t)std::max<int64_t>(p.max_events, 1);
  for (int l = 0; !rc && l < kLanes; ++l) {
    if (!dev_malloc(reinterpret_cast<void**>(&s->ev_dev[l]), nev * sizeof(veckm_event)) ||
        !dev_malloc(reinterpret_cast<void**>(&s->flow_dev[l]), nev * 2 * sizeof(float)))
      rc = VECKM_E_NOMEM;
  }
  for (hipStream_t* st : {&s->stream, &s->h2d, &s->d2h})
    if (!rc && hipStreamCreateWithFlags(st, hipStreamNonBlocking) != hipSuccess) rc = VECKM_E_HIP;
  if (rc) {
    (void)hipGetLastError();
    for (int l = 0; l < kLanes; ++l) {
      if (s->ev_dev[l]) (void)hipFree(s->ev_dev[l]);
      if (s->flow_dev[l]) (void)hipFree(s->flow_dev[l]);
    }
    for (hipStream_t st : {s->stream, s->h2d, s->d2h})
      if (st) (void)hipStreamDestroy(st);
    if (s->ctx) veckm_destroy(s->ctx);
    delete s;
    return rc;
  }
  s->cap = ctx_capacity(s->ctx);
  s->grid_arena.size = s->cap.voxels;
  s->pair_arena.size = s->cap.pairs;
  s->streams.resize((size_t)max_streams);
  s->launcher = std::thread(launcher_main, s);
  s->completer = std::thread(completer_main, s);
  *out = s;
  return VECKM_OK;
}

void veckm_server_destroy(veckm_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_launch.notify_all();
  s->cv_done.notify_all();
  s->launcher.join();  // no batch is launched after this
  s->cv_complete.notify_all();
  s->completer.join();
  for (hipStream_t st : {s->h2d, s->stream, s->d2h}) (void)hipStreamSynchronize(st);
  for (InFlight& f : s->inflight) s->spare.push_back(f);
  for (auto& kv : s->tickets) delete kv.second;
  for (InFlight& f : s->spare) drop_flight(f);
  for (Stream& st : s->streams) free_slots(st);
  for (hipStream_t st : {s->stream, s->h2d, s->d2h}) (void)hipStreamDestroy(st);
  for (int l = 0; l < kLanes; ++l) {
    (void)hipFree(s->ev_dev[l]);
    (void)hipFree(s->flow_dev[l]);
  }
  veckm_destroy(s->ctx);
  delete s;
}

int veckm_server_set_mlp(veckm_server* s, int32_t hidden, const float* W1, const float* b1,
                         const float* W2, const float* b2) {
  if (!s) return VECKM_E_INVAL;
  std::lock_guard<std::mutex> g(s->ctx_mu);
  (void)hipStreamSynchronize(s->stream);
  (void)hipStreamSynchronize(s->d2h);
  const int rc = veckm_set_mlp(s->ctx, hidden, W1, b1, W2, b2);
  if (!rc) {
    std::lock_guard<std::mutex> lk(s->mu);
    s->has_mlp = true;
  }
  return rc;
}

int veckm_stream_open(veckm_server* s, int32_t width, int32_t height, int32_t max_bins,
                      int64_t max_events, int32_t* sid) {
  if (!s || !sid) return VECKM_E_INVAL;
  if (width < 1 || height < 1 || max_bins < 1 || max_events < 1) return VECKM_E_INVAL;
  if (width > s->p.width || height > s->p.height || max_bins > s->p.max_bins ||
      max_events > s->p.max_events)
    return VECKM_E_RANGE;
  // pinned staging first (slow), then the reservation under the lock
  Stream fresh;
  fresh.slots.resize((size_t)s->depth);
  for (Slot& sl : fresh.slots) {
    if (!pinned_malloc(reinterpret_cast<void**>(&sl.ev), (size_t)max_events * sizeof(veckm_event)) ||
        !pinned_malloc(reinterpret_cast<void**>(&sl.flow), (size_t)max_events * 2 * sizeof(float))) {
      (void)hipGetLastError();
      free_slots(fresh);
      return VECKM_E_NOMEM;
    }
  }
  fresh.open = true;
  fresh.W = width;
  fresh.H = height;
  fresh.T = max_bins;
  fresh.max_events = max_events;
  fresh.share = slice_need(s->ctx, width, height, max_bins, max_events);
  std::unique_lock<std::mutex> lk(s->mu);
  int k = -1;
  for (size_t i = 0; i < s->streams.size(); ++i)
    if (!s->streams[i].open) {
      k = (int)i;
      break;
    }
  int rc = VECKM_OK;
  if (s->stop) rc = VECKM_E_STATE;
  else if (k < 0) rc = VECKM_E_AGAIN;
  else if (!fits(s->reserved, fresh.share, s->cap)) rc = VECKM_E_BUDGET;
  // the stream's resident grids
  else if (!s->grid_arena.take(fresh.share.voxels, &fresh.grid_at)) rc = VECKM_E_BUDGET;
  else if (!s->pair_arena.take(fresh.share.pairs, &fresh.pair_at)) {
    s->grid_arena.give(fresh.grid_at);
    rc = VECKM_E_BUDGET;
  }
  if (rc) {
    lk.unlock();
    free_slots(fresh);
    return rc;
  }
  add(s->reserved, fresh.share, 1);
  s->streams[(size_t)k] = std::move(fresh);
  *sid = k;
  return VECKM_OK;
}

int veckm_stream_close(veckm_server* s, int32_t sid) {
  if (!s) return VECKM_E_INVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  if (sid < 0 || sid >= (int)s->streams.size() || !s->streams[(size_t)sid].open)
    return VECKM_E_INVAL;
  Stream& st = s->streams[(size_t)sid];
  s->cv_done.wait(lk, [&] { return st.outstanding == 0 && st.copying == 0; });
  for (auto it = s->tickets.begin(); it != s->tickets.end();) {
    if (it->second->sid == sid) {
      delete it->second;
      it = s->tickets.erase(it);
    } else {
      ++it;
    }
  }
  add(s->reserved, st.share, -1);
  s->grid_arena.give(st.grid_at);
  s->pair_arena.give(st.pair_at);
  Stream gone = std::move(st);
  s->streams[(size_t)sid] = Stream();
  lk.unlock();
  free_slots(gone);
  return VECKM_OK;
}

int veckm_submit(veckm_server* s, int32_t sid, const veckm_event* events, int64_t n, int32_t t0,
                 int32_t nbins, uint64_t* ticket) {
  const Clock::time_point now = Clock::now();
  if (!s || !ticket || n < 0 || (n > 0 && !events)) return VECKM_E_INVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->stop || !s->has_mlp) return VECKM_E_STATE;
  if (sid < 0 || sid >= (int)s->streams.size() || !s->streams[(size_t)sid].open)
    return VECKM_E_INVAL;
  Stream& st = s->streams[(size_t)sid];
  if (n > st.max_events || nbins < 1 || nbins > st.T) return VECKM_E_RANGE;
  int slot = -1;
  for (size_t i = 0; i < st.slots.size(); ++i)
    if (!st.slots[i].busy) {
      slot = (int)i;
      break;
    }
  if (slot < 0) return VECKM_E_AGAIN;
  st.slots[(size_t)slot].busy = true;
  st.outstanding += 1;
  veckm_event* dst = st.slots[(size_t)slot].ev;
  Ticket* t = new (std::nothrow) Ticket();
  if (!t) {
    st.slots[(size_t)slot].busy = false;
    st.outstanding -= 1;
    return VECKM_E_NOMEM;
  }
  t->id = s->next_ticket++;
  t->sid = sid;
  t->slot = slot;
  t->n = n;
  t->t0 = t0;
  t->nbins = nbins;
  t->submitted = now;
  // copy the events without holding the lock: the slot is claimed and the
  // stream cannot close while the slice is outstanding
  lk.unlock();
  if (n > 0) std::memcpy(dst, events, (size_t)n * sizeof(veckm_event));
  lk.lock();
  if (!s->have_first) {
    s->have_first = true;
    s->first_submit = now;
  }
  s->tickets[t->id] = t;
  s->pending.push_back(t);
  *ticket = t->id;
  s->cv_launch.notify_one();
  return VECKM_OK;
}

int veckm_poll(veckm_server* s, uint64_t ticket, float* flows, int32_t timeout_us) {
  if (!s) return VECKM_E_INVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return VECKM_E_INVAL;
  Ticket* t = it->second;
  if (!t->done) {
    if (timeout_us == 0) return VECKM_E_AGAIN;
    auto ready = [&] { return t->done || s->stop; };
    if (timeout_us < 0)
      s->cv_done.wait(lk, ready);
    else
      s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready);
    if (!t->done) return VECKM_E_AGAIN;
    // the ticket may have been taken by another poller meanwhile
    it = s->tickets.find(ticket);
    if (it == s->tickets.end() || it->second != t) return VECKM_E_INVAL;
  }
  s->tickets.erase(it);
  Stream& st = s->streams[(size_t)t->sid];
  st.copying += 1;
  const float* src = st.slots[(size_t)t->slot].flow;
  lk.unlock();
  if (flows && t->n > 0 && t->status == VECKM_OK)
    std::memcpy(flows, src, (size_t)t->n * 2 * sizeof(float));
  lk.lock();
  st.slots[(size_t)t->slot].busy = false;
  st.copying -= 1;
  const int status = t->status;
  delete t;
  s->cv_done.notify_all();
  return status;
}

namespace {

int stats_of(veckm_server* s, veckm_serving_stats* out, int32_t reset, int32_t width,
             int32_t height) {
  if (!s || !out) return VECKM_E_INVAL;
  std::vector<double> lat;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    const bool all = width == 0 && height == 0;
    const int64_t key = (int64_t)width << 32 | height;
    for (size_t i = 0; i < s->lat_ms.size(); ++i)
      if (all || s->lat_sensor[i] == key) lat.push_back(s->lat_ms[i]);
    out->slices = all ? s->done_slices : (int64_t)lat.size();
    out->flows = s->done_flows;
    out->batches = s->batches;
    out->busy_s = s->have_first && s->done_slices > 0
                      ? std::chrono::duration<double>(s->last_done - s->first_submit).count()
                      : 0.0;
    if (reset) {
      s->lat_ms.clear();
      s->lat_sensor.clear();
      s->done_slices = s->done_flows = s->batches = 0;
      s->have_first = false;
    }
  }
  std::sort(lat.begin(), lat.end());
  auto pct = [&](double q) {  // nearest rank
    if (lat.empty()) return 0.0;
    const double r = std::ceil(q * (double)lat.size());
    const size_t i = (size_t)std::max(1.0, std::min(r, (double)lat.size())) - 1;
    return lat[i];
  };
  out->p50_ms = pct(0.50);
  out->p99_ms = pct(0.99);
  out->max_ms = lat.empty() ? 0.0 : lat.back();
  return VECKM_OK;
}

}  // namespace

int veckm_server_stats(veckm_server* s, veckm_serving_stats* out, int32_t reset) {
  return stats_of(s, out, reset, 0, 0);
}

int veckm_server_stats_sensor(veckm_server* s, int32_t width, int32_t height,
                              veckm_serving_stats* out) {
  if (width < 1 || height < 1) return VECKM_E_INVAL;
  return stats_of(s, out, 0, width, height);
}

}  // extern "C"
