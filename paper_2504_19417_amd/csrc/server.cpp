// Serving: asynchronous event streams, continuously batched onto one context.
//
// Slices are independent (every neighbourhood lies inside its slice,
// Sec. 2.1), so slices of different streams and sensors can share one batch
// call and the result of each is the same as alone.  A launcher thread packs
// the waiting slices into batches while fewer than kMaxInflight batches are
// on the device; a completer thread waits for each batch in order, checks its
// device error bits and hands the flows to the pollers.  A batch that reports
// an input error has its slices run again one by one, so only the offending
// slice gets the error.
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

constexpr int kMaxInflight = 2;  // batches on the device at once: one running, one queued
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
  std::vector<Slot> slots;
  int outstanding = 0;  // submitted and not complete
  int copying = 0;      // results being copied out by veckm_poll
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
  hipEvent_t done = nullptr;
  int32_t* err = nullptr;  // pinned: the batch's device error bits
};

bool fits(const Capacity& used, const Capacity& need, const Capacity& cap) {
  return used.events + need.events <= cap.events && used.voxels + need.voxels <= cap.voxels &&
         used.pairs + need.pairs <= cap.pairs && used.bricks + need.bricks <= cap.bricks &&
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
  hipStream_t stream = nullptr;
  int depth = 1;
  Capacity cap, reserved;
  veckm_event* ev_dev = nullptr;
  float* flow_dev = nullptr;
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
  if (hipEventCreateWithFlags(&g.done, hipEventDisableTiming) != hipSuccess) return VECKM_E_HIP;
  if (hipHostMalloc(reinterpret_cast<void**>(&g.err), sizeof(int32_t)) != hipSuccess) {
    (void)hipEventDestroy(g.done);
    return VECKM_E_NOMEM;
  }
  *f = g;
  return VECKM_OK;
}

// Completes a ticket (caller holds mu).
void finish(veckm_server* s, Ticket* t, int status, Clock::time_point now) {
  t->done = true;
  t->status = status;
  t->completed = now;
  s->streams[t->sid].outstanding -= 1;
  s->lat_ms.push_back(std::chrono::duration<double, std::milli>(now - t->submitted).count());
  s->done_slices += 1;
  s->done_flows += t->n;
  s->last_done = now;
}

// Copies the batch's events in, runs it, copies the flows out and records
// its completion event; all on the server's stream.
int enqueue(veckm_server* s, const std::vector<Ticket*>& take, InFlight& f) {
  std::lock_guard<std::mutex> g(s->ctx_mu);
  std::vector<veckm_slice> sl(take.size());
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
    if (t->n > 0 && hipMemcpyAsync(s->ev_dev + off, st.slots[t->slot].ev,
                                   (size_t)t->n * sizeof(veckm_event), hipMemcpyHostToDevice,
                                   s->stream) != hipSuccess)
      return VECKM_E_HIP;
    off += t->n;
  }
  int rc = veckm_flow_batch(s->ctx, sl.data(), (int32_t)sl.size(), s->ev_dev, s->flow_dev,
                            s->stream);
  if (rc) return rc;
  rc = ctx_take_err(s->ctx, f.err, s->stream);
  if (rc) return rc;
  off = 0;
  for (const Ticket* t : take) {
    const Stream& st = s->streams[t->sid];
    if (t->n > 0 && hipMemcpyAsync(st.slots[t->slot].flow, s->flow_dev + 2 * off,
                                   (size_t)t->n * 2 * sizeof(float), hipMemcpyDeviceToHost,
                                   s->stream) != hipSuccess)
      return VECKM_E_HIP;
    off += t->n;
  }
  return hipEventRecord(f.done, s->stream) == hipSuccess ? VECKM_OK : VECKM_E_HIP;
}

void launcher_main(veckm_server* s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    s->cv_launch.wait(lk, [s] {
      return s->stop || (!s->pending.empty() && (int)s->inflight.size() < kMaxInflight);
    });
    if (s->stop) return;
    // waiting slices in submission order while they fit; a slice marked
    // solo runs alone
    std::vector<Ticket*> take;
    Capacity used;
    if (s->pending.front()->solo) {
      take.push_back(s->pending.front());
      s->pending.pop_front();
    } else {
      while (!s->pending.empty() && !s->pending.front()->solo) {
        Ticket* t = s->pending.front();
        const Stream& st = s->streams[t->sid];
        const Capacity need = slice_need(s->ctx, st.W, st.H, t->nbins, t->n);
        if (!fits(used, need, s->cap)) break;
        add(used, need, 1);
        take.push_back(t);
        s->pending.pop_front();
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
    lk.unlock();
    if (!rc) rc = enqueue(s, take, f);
    lk.lock();
    if (rc) {
      const Clock::time_point now = Clock::now();
      for (Ticket* t : take) finish(s, t, rc, now);
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
  int rc = veckm_params_check(&p);
  if (rc) return rc;
  if (p.rt < 0) return VECKM_E_INVAL;  // batches need the temporally bounded encoder
  const int64_t ws = veckm_workspace_bytes(&p, 512);
  if (ws < 0) return (int)ws;
  const int64_t bytes = ws + p.max_events * (int64_t)(sizeof(veckm_event) + 2 * sizeof(float));
  if (bytes > hbm_budget_bytes) return VECKM_E_BUDGET;
  veckm_server* s = new (std::nothrow) veckm_server();
  if (!s) return VECKM_E_NOMEM;
  s->p = p;
  s->depth = depth;
  rc = veckm_create(&p, &s->ctx);
  if (!rc && hipGetDevice(&s->device) != hipSuccess) rc = VECKM_E_HIP;
  if (!rc && hipMalloc(reinterpret_cast<void**>(&s->ev_dev),
                       (size_t)std::max<int64_t>(p.max_events, 1) * sizeof(veckm_event)) != hipSuccess)
    rc = VECKM_E_NOMEM;
  if (!rc && hipMalloc(reinterpret_cast<void**>(&s->flow_dev),
                       (size_t)std::max<int64_t>(p.max_events, 1) * 2 * sizeof(float)) != hipSuccess)
    rc = VECKM_E_NOMEM;
  if (!rc && hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess)
    rc = VECKM_E_HIP;
  if (rc) {
    (void)hipGetLastError();
    if (s->ev_dev) (void)hipFree(s->ev_dev);
    if (s->flow_dev) (void)hipFree(s->flow_dev);
    if (s->ctx) veckm_destroy(s->ctx);
    delete s;
    return rc;
  }
  s->cap = ctx_capacity(s->ctx);
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
  (void)hipStreamSynchronize(s->stream);
  for (InFlight& f : s->inflight) s->spare.push_back(f);
  for (auto& kv : s->tickets) delete kv.second;
  for (InFlight& f : s->spare) {
    (void)hipEventDestroy(f.done);
    (void)hipHostFree(f.err);
  }
  for (Stream& st : s->streams) free_slots(st);
  (void)hipStreamDestroy(s->stream);
  (void)hipFree(s->ev_dev);
  (void)hipFree(s->flow_dev);
  veckm_destroy(s->ctx);
  delete s;
}

int veckm_server_set_mlp(veckm_server* s, int32_t hidden, const float* W1, const float* b1,
                         const float* W2, const float* b2) {
  if (!s) return VECKM_E_INVAL;
  std::lock_guard<std::mutex> g(s->ctx_mu);
  (void)hipStreamSynchronize(s->stream);
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
    if (hipHostMalloc(reinterpret_cast<void**>(&sl.ev), (size_t)max_events * sizeof(veckm_event)) !=
            hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&sl.flow), (size_t)max_events * 2 * sizeof(float)) !=
            hipSuccess) {
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

int veckm_server_stats(veckm_server* s, veckm_serving_stats* out, int32_t reset) {
  if (!s || !out) return VECKM_E_INVAL;
  std::vector<double> lat;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    lat = s->lat_ms;
    out->slices = s->done_slices;
    out->flows = s->done_flows;
    out->batches = s->batches;
    out->busy_s = s->have_first && s->done_slices > 0
                      ? std::chrono::duration<double>(s->last_done - s->first_submit).count()
                      : 0.0;
    if (reset) {
      s->lat_ms.clear();
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

}  // extern "C"
