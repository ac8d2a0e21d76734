// C-ABI of the veckm library: context set-up, argument validation and the
// launch sequence of one call (one slice or a batch of slices).  Every step
// of the computation runs in the HIP kernels of this library; there is no
// host fallback.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "veckm_internal.h"

using namespace veckm;

namespace {
constexpr int kRing = 8;  // slice tables of batch calls in flight per context
constexpr int64_t kMaxTotalVoxels = std::numeric_limits<int32_t>::max();

// The allocation fault hook: counts allocations since VECKM_FAULT_ALLOC last
// changed and reports whether this one is the one to fail.
std::mutex g_fault_mu;
std::string g_fault_env;
int64_t g_fault_count = 0;

bool fault_this_alloc() {
  const char* e = std::getenv("VECKM_FAULT_ALLOC");
  std::lock_guard<std::mutex> lk(g_fault_mu);
  const std::string cur = e ? e : "";
  if (cur != g_fault_env) {
    g_fault_env = cur;
    g_fault_count = 0;
  }
  const long long n = cur.empty() ? 0 : std::atoll(cur.c_str());
  if (n <= 0) return false;
  return ++g_fault_count == n;
}
}  // namespace

bool veckm::dev_malloc(void** p, size_t bytes) {
  *p = nullptr;
  if (fault_this_alloc()) return false;
  if (hipMalloc(p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return false;
  }
  return true;
}

bool veckm::pinned_malloc(void** p, size_t bytes) {
  *p = nullptr;
  if (fault_this_alloc()) return false;
  if (hipHostMalloc(p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return false;
  }
  return true;
}

struct veckm_ctx {
  veckm_params p{};
  std::vector<double> A;
  int device = 0;
  int num_cus = 0;
  EncodeTables et;                    // the tiling in use (one of `tilings`)
  std::vector<EncodeTables> tilings;  // candidate encoder tilings (same tables, other bricks)
  int tiling = 0;
  Workspace w;
  MlpWeights mw;
  bool paper = false;  // no temporal bound: the staged 2-D pooling encoder
  // sliding window (veckm_window_*): the count and pair grids are a ring of
  // max_bins planes holding bins [wend - max_bins, wend); bin t sits in plane
  // (t - tref) mod max_bins
  bool window = false;
  bool started = false;
  int32_t tref = 0;
  int64_t wend = 0;
  PaperTables pt;
  int max_slices = 1;
  std::vector<void*> allocs;
  std::vector<void*> mlp_allocs;
  uint16_t* w1_slot = nullptr;  // W1 slabs after the phase table's (fusable widths)
  // Slice tables of batch calls: pinned staging and device copies, one slot
  // per call in flight; a slot is reused once the call that used it is done.
  SliceDesc* table_host = nullptr;
  SliceDesc* table_dev = nullptr;
  hipEvent_t ring_ev[kRing] = {};
  bool ring_used[kRing] = {};
  int ring_next = 0;
  // per-stage timing
  bool prof = false;
  std::vector<hipEvent_t> ev_pool;
  struct Mark {
    int stage;
    hipEvent_t a, b;
  };
  std::vector<Mark> marks;
  size_t ev_next = 0;
};

namespace {

int device_ok(int* dev, int* cus) {
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count < 1) return VECKM_E_NODEVICE;
  if (hipGetDevice(dev) != hipSuccess) return VECKM_E_NODEVICE;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, *dev) != hipSuccess) return VECKM_E_NODEVICE;
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return VECKM_E_NODEVICE;
  *cus = prop.multiProcessorCount;
  return VECKM_OK;
}

template <typename T>
int dalloc(std::vector<void*>& list, T** out, size_t count) {
  void* p = nullptr;
  if (count == 0) count = 1;
  if (!dev_malloc(&p, count * sizeof(T))) return VECKM_E_NOMEM;
  list.push_back(p);
  *out = static_cast<T*>(p);
  return VECKM_OK;
}

int slices_of(const veckm_params* p) { return p->max_slices > 0 ? p->max_slices : 1; }

int64_t bricks_of(int W, int H, int T, const Brick& b) {
  return (int64_t)((W + b.bx - 1) / b.bx) * ((H + b.by - 1) / b.by) * ((T + b.bt - 1) / b.bt);
}

int64_t voxels_of(const veckm_params* p) {
  const int64_t per = (int64_t)p->width * p->height * p->max_bins;
  return p->max_voxels > 0 ? p->max_voxels : per * slices_of(p);
}

// Pair-grid entries: (W + 1) H T per slice, at most twice the voxels.
int64_t pair_entries_of(const veckm_params* p) {
  const int64_t per = (int64_t)(p->width + 1) * p->height * p->max_bins;
  return p->max_voxels > 0 ? 2 * p->max_voxels : per * slices_of(p);
}

struct Sizes {
  int64_t V, P, nb, ulist, lines, U, n;
};

// Workspace sizes for every tiling a context may use: the most bricks and
// the largest row list over the bricks.
Sizes sizes_for(const veckm_params* p, const std::vector<Tiling>& tl) {
  Sizes s;
  s.V = voxels_of(p);
  s.P = pair_entries_of(p);
  s.nb = 0;
  s.ulist = 0;
  s.lines = 0;
  for (const Tiling& t : tl) {
    const int64_t nb = slices_of(p) * bricks_of(p->width, p->height, p->max_bins, t.brick);
    s.nb = std::max(s.nb, nb);
    s.ulist = std::max(s.ulist, nb * t.brick.volume());
    s.lines = std::max(s.lines, nb * t.brick.by * t.brick.bt);
  }
  s.n = p->max_events;
  s.U = s.n < s.V ? s.n : s.V;
  return s;
}

// The tilings of a context made from p (the paper form numbers voxels with
// one fixed brick and has no encoder tiling to choose).
std::vector<Tiling> tilings_for(const veckm_params* p, int kp) {
  if (p->rt < 0) return {Tiling{Brick{32, 16, 8}, 2}};
  return tiling_candidates(p->rx, p->ry, p->rt, p->d, p->precision, kp);
}

int64_t bytes_for(const veckm_params* p, const std::vector<Tiling>& tl, int kp, int hidden) {
  const Sizes s = sizes_for(p, tl);
  const int na = p->precision == VECKM_FP32 ? 4 : 2;
  int64_t bytes = 0;
  if (p->rt < 0) {  // paper form: G, S grids, pixel counts, phase tables
    const int64_t V2 = (int64_t)p->width * p->height;
    bytes += 2 * 2 * (int64_t)p->d * V2 * 4 + 3 * V2 * 4 + s.U * 4;
    bytes += (int64_t)(p->max_bins + p->width + p->height) * p->d * 8;
  }
  bytes += s.V * (4 + 4 + 1);                     // count, rank, qmark
  if (p->rt >= 0) bytes += s.P * 4 + s.lines;     // pair grid, brick row flags
  bytes += s.ulist * 4;                           // ulist
  bytes += (6 * s.nb + 1) * 4;                    // brick_nq, brick_off, order
  bytes += (scan_tiles(s.nb) + 1) * kScanNV * 4;  // brick-scan partials
  bytes += s.n * (4 + 4);                         // vox, qmap
  if (p->rt >= 0) bytes += s.U * 8 + kp;          // single-row list, its box's run offsets
  bytes += s.U * 2 * p->d * 4 + s.U * 8;          // rows (fp32 size), rowflow
  bytes += (int64_t)kp * p->d * na * 2 + kp * 2;  // phase table, weights
  bytes += (int64_t)tl.size() * kp;               // run offsets (one table per tiling)
  bytes += 64 * 4 + 4 + 64 * 4;                   // plan, err, zero page
  bytes += (int64_t)kRing * slices_of(p) * (int64_t)sizeof(SliceDesc);  // slice tables
  bytes += (int64_t)hidden * (2 * p->d) * 10 + hidden * 12 + 8;  // perceptron (fp32, bf16, fp16 hi/lo W1)
  if (p->rt >= 0 && (p->d == 64 || p->d == 128))  // room for W1 after the phase table
    bytes += (int64_t)kMaxHidden * (2 * p->d) * (na / 2) * 2;
  return bytes;
}

SliceDesc describe(const veckm_ctx* c, int W, int H, int T, int t0, int64_t brick_off,
                   int64_t grid_off, int64_t pair_off, int64_t ev_off, int64_t n) {
  const Brick& b = c->et.brick;
  SliceDesc s;
  s.W = W;
  s.H = H;
  s.T = T;
  s.t0 = t0;
  s.nbx = (W + b.bx - 1) / b.bx;
  s.nby = (H + b.by - 1) / b.by;
  s.nbt = (T + b.bt - 1) / b.bt;
  s.brick_off = (int)brick_off;
  s.grid_off = grid_off;
  s.pair_off = pair_off;
  s.ev_off = (int)ev_off;
  s.n = (int)n;
  s.tshift = 0;
  return s;
}

// One slice on the context's sensor.
int single_batch(const veckm_ctx* c, const veckm_event* ev, int64_t n, int32_t t0, int32_t nbins,
                 const int32_t* queries, int64_t m, const void* out, Batch* bt) {
  if (n < 0 || m < 0) return VECKM_E_INVAL;
  if ((n > 0 && !ev) || (m > 0 && !out)) return VECKM_E_INVAL;
  if (!queries && m != n) return VECKM_E_INVAL;
  if (n > c->p.max_events || m > c->p.max_events) return VECKM_E_RANGE;
  if (nbins < 1 || nbins > c->p.max_bins) return VECKM_E_RANGE;
  const int64_t V = (int64_t)c->p.width * c->p.height * nbins;
  const int64_t P = (int64_t)(c->p.width + 1) * c->p.height * nbins;
  if (V > c->w.vmax || P > c->w.pmax) return VECKM_E_RANGE;
  bt->s0 = describe(c, c->p.width, c->p.height, nbins, t0, 0, 0, 0, 0, n);
  bt->table = nullptr;
  bt->nslices = 1;
  bt->nbricks = bt->s0.nbx * bt->s0.nby * bt->s0.nbt;
  bt->n = (int)n;
  bt->m = (int)m;
  bt->nvox = V;
  bt->npairs = P;
  bt->max_rows = (int64_t)c->p.height * nbins;
  return VECKM_OK;
}

// A batch of slices: validate and describe them (bt->table is left unset).
// Grids lie back to back, or, when `at` is given, slice k's count grid starts
// at voxel at[2k] and its pair grid at entry at[2k + 1] (regions a server
// keeps for its streams; they must not overlap).
int plan_batch(veckm_ctx* c, const veckm_slice* sl, int32_t count, const veckm_event* ev,
               const void* out, std::vector<SliceDesc>& tab, Batch* bt,
               const int64_t* at = nullptr) {
  if (!sl || count < 1 || count > c->max_slices) return VECKM_E_INVAL;
  tab.assign((size_t)count, SliceDesc{});
  int64_t evs = 0, vox = 0, prs = 0, bricks = 0, max_rows = 0, vend = 0, pend = 0;
  std::vector<std::pair<int64_t, int64_t>> vreg, preg;
  for (int k = 0; k < count; ++k) {
    const veckm_slice& s = sl[k];
    if (s.n < 0 || s.offset != evs) return VECKM_E_INVAL;
    if (s.n > c->p.max_events - evs) return VECKM_E_RANGE;
    if (s.width < 1 || s.height < 1 || s.width > c->p.width || s.height > c->p.height)
      return VECKM_E_RANGE;
    if (s.nbins < 1 || s.nbins > c->p.max_bins) return VECKM_E_RANGE;
    const int64_t V = (int64_t)s.width * s.height * s.nbins;
    const int64_t P = (int64_t)(s.width + 1) * s.height * s.nbins;
    const int64_t go = at ? at[2 * k] : vox, po = at ? at[2 * k + 1] : prs;
    if (go < 0 || po < 0) return VECKM_E_INVAL;
    tab[k] = describe(c, s.width, s.height, s.nbins, s.t0, bricks, go, po, evs, s.n);
    evs += s.n;
    vox += V;
    prs += P;
    vend = std::max(vend, go + V);
    pend = std::max(pend, po + P);
    if (at) {
      vreg.push_back({go, go + V});
      preg.push_back({po, po + P});
    }
    max_rows = std::max(max_rows, (int64_t)s.height * s.nbins);
    bricks += bricks_of(s.width, s.height, s.nbins, c->et.brick);
  }
  for (auto* reg : {&vreg, &preg}) {
    std::sort(reg->begin(), reg->end());
    for (size_t i = 1; i < reg->size(); ++i)
      if ((*reg)[i].first < (*reg)[i - 1].second) return VECKM_E_INVAL;
  }
  if (vend > c->w.vmax || pend > c->w.pmax || bricks > c->w.bmax ||
      bricks * c->et.brick.volume() > c->w.umax)
    return VECKM_E_RANGE;
  vox = vend;  // the extent the batch's grids span (cleared on failed runs)
  prs = pend;
  if (evs > 0 && (!ev || !out)) return VECKM_E_INVAL;
  bt->s0 = tab[0];
  bt->table = nullptr;
  bt->nslices = count;
  bt->nbricks = (int)bricks;
  bt->n = (int)evs;
  bt->m = (int)evs;
  bt->nvox = vox;
  bt->npairs = prs;
  bt->max_rows = max_rows;
  return VECKM_OK;
}

// A batch of slices: validate, describe, and upload the slice table through
// the next ring slot (*slot, released by release_slot after the launches).
int multi_batch(veckm_ctx* c, const veckm_slice* sl, int32_t count, const veckm_event* ev,
                const void* out, void* stream, Batch* bt, int* slot, const int64_t* at = nullptr) {
  *slot = -1;
  std::vector<SliceDesc> tab;
  const int rc = plan_batch(c, sl, count, ev, out, tab, bt, at);
  if (rc) return rc;
  const int k = c->ring_next;
  if (c->ring_used[k] && hipEventSynchronize(c->ring_ev[k]) != hipSuccess) return VECKM_E_HIP;
  c->ring_next = (k + 1) % kRing;
  SliceDesc* host = c->table_host + (size_t)k * c->max_slices;
  SliceDesc* dev = c->table_dev + (size_t)k * c->max_slices;
  std::memcpy(host, tab.data(), tab.size() * sizeof(SliceDesc));
  if (hipMemcpyAsync(dev, host, tab.size() * sizeof(SliceDesc), hipMemcpyHostToDevice,
                     (hipStream_t)stream) != hipSuccess)
    return VECKM_E_HIP;
  *slot = k;
  bt->table = dev;
  return VECKM_OK;
}

// Marks the end of the call that used ring slot `slot` on `stream`.
int release_slot(veckm_ctx* c, int slot, void* stream) {
  if (slot < 0) return VECKM_OK;
  if (hipEventRecord(c->ring_ev[slot], (hipStream_t)stream) != hipSuccess) return VECKM_E_HIP;
  c->ring_used[slot] = true;
  return VECKM_OK;
}

// Stage timing: events come from a pool made by veckm_profile_enable.
struct StageTimer {
  veckm_ctx* c;
  int stage;
  hipStream_t s;
  hipEvent_t a = nullptr, b = nullptr;
  StageTimer(veckm_ctx* c_, int stage_, void* stream)
      : c(c_), stage(stage_), s((hipStream_t)stream) {
    if (!c->prof || c->ev_next + 2 > c->ev_pool.size()) return;
    a = c->ev_pool[c->ev_next++];
    b = c->ev_pool[c->ev_next++];
    (void)hipEventRecord(a, s);
  }
  ~StageTimer() {
    if (!a) return;
    (void)hipEventRecord(b, s);
    c->marks.push_back({stage, a, b});
  }
};

// The launch sequence of one call: `emb` for encode calls, `flow` for flow
// calls, `counts` for count calls (exactly one is non-NULL), on the
// workspaces `w` (the context's own, or the allocation-free entry point's
// static ones).
int run(veckm_ctx* c, const Workspace& w, const Batch& bt, const veckm_event* ev,
        const int32_t* queries, float* emb, float* flow, void* stream,
        int32_t* counts = nullptr) {
  // a window's encode: ev holds the query events, the counts are resident
  if (bt.m == 0) return VECKM_OK;
  // rows the encoder hands to the perceptron (encodings handed out are fp32)
  // (the one-wave-per-SIMD tiling runs the perceptron itself: no rows at all)
  const bool fused = flow && !c->paper && c->mw.W1frag && encode_fusable(c->et, c->mw.hidden);
  const int rows = !flow                             ? kRowsF32
                   : fused                            ? (c->p.precision == VECKM_FP16 ? kFlowBF16
                                                                                      : kFlowHiLo16)
                   : c->p.precision == VECKM_FP16     ? kRowsBF16
                   : !mlp_rows_split(c->p.d, c->mw.hidden) ? kRowsF32
                   : c->paper                          ? kRowsSplit16
                                                      : kRowsHiLo16;
  // slice calls (not the paper form; a window's counts are resident) find
  // the count grid, the pair grid and the row flags zero and leave them
  // zero: the ranking kernel clears the flags, and after the expansion the
  // events' voxels are cleared; a call whose launches fail clears all three
  // grids densely
  const bool clear = !c->paper && !c->window;
  const int64_t nlines = (int64_t)bt.nbricks * c->et.brick.by * c->et.brick.bt;
  {
    StageTimer t(c, VECKM_STAGE_PREPARE, stream);
    const int rc = c->window ? launch_window_prepare(bt, w, ev, c->et, stream)
                             : launch_prepare(bt, w, ev, queries, c->et, !c->paper, stream);
    if (rc) {
      if (clear) (void)launch_clear_grids(bt, w, nlines, stream);
      return rc;
    }
  }
  {
    StageTimer t(c, VECKM_STAGE_ENCODE, stream);
    // the encoder writes fp32 rows unless the perceptron takes bf16 or hi/lo
    // rows, or runs inside the encoder
    const int erows = rows == kRowsBF16 || rows == kRowsHiLo16 || fused ? rows : kRowsF32;
    const int rc = c->paper ? launch_paper_encode(bt, w, c->pt, c->et.brick, erows, c->num_cus, stream)
                            : launch_encode(bt, w, c->et, erows, c->num_cus, stream,
                                            counts ? reinterpret_cast<int32_t*>(w.rowflow)
                                                   : nullptr,
                                            &c->mw);
    if (rc) {
      if (clear) (void)launch_clear_grids(bt, w, nlines, stream);
      return rc;
    }
  }
  if (flow && !fused) {
    StageTimer t(c, VECKM_STAGE_MLP, stream);
    const int rc = launch_mlp(w, c->mw, c->p.d, rows, c->num_cus, stream);
    if (rc) {
      if (clear) (void)launch_clear_grids(bt, w, nlines, stream);
      return rc;
    }
  }
  StageTimer t(c, VECKM_STAGE_EXPAND, stream);
  // (a window's queries are the query events themselves: index i is event i)
  const int32_t* q = c->window ? nullptr : queries;
  // (the flows of a dense call and its grid clear share one launch)
  const bool merged = flow && clear && !c->paper && dense_batch(bt);
  int rc = merged   ? launch_expand_flow_clear(bt, w, q, c->et.brick, flow, stream)
           : flow   ? launch_expand_flow(bt, w, q, c->et.brick, c->paper, flow, stream)
           : counts ? launch_expand_count(bt, w, q, c->et.brick, counts, stream)
                    : launch_expand_emb(bt, w, q, c->et.brick, c->paper, c->p.d, emb, stream);
  if (clear && (rc || !merged)) {
    const int rc2 = rc ? launch_clear_grids(bt, w, nlines, stream) : launch_clear_events(bt, w, stream);
    rc = rc ? rc : rc2;
  }
  return rc;
}

}  // namespace

namespace veckm {

int flow_batch_at(veckm_ctx* c, const veckm_slice* slices, int32_t count, const int64_t* at,
                  const veckm_event* events, float* flow, void* stream) {
  if (!c || c->paper || c->window || !at) return VECKM_E_INVAL;
  if (c->mw.hidden == 0) return VECKM_E_STATE;
  Batch bt;
  int slot;
  int rc = multi_batch(c, slices, count, events, flow, stream, &bt, &slot, at);
  if (rc) return rc;
  rc = run(c, c->w, bt, events, nullptr, nullptr, flow, stream);
  const int rc2 = release_slot(c, slot, stream);
  return rc ? rc : rc2;
}

Capacity ctx_capacity(const veckm_ctx* c) {
  Capacity k;
  k.events = c->p.max_events;
  k.voxels = c->w.vmax;
  k.pairs = c->w.pmax;
  k.bricks = c->w.bmax;
  k.slices = c->max_slices;
  return k;
}

Capacity slice_need(const veckm_ctx* c, int W, int H, int T, int64_t n) {
  Capacity k;
  k.events = n;
  k.voxels = (int64_t)W * H * T;
  k.pairs = (int64_t)(W + 1) * H * T;
  k.bricks = bricks_of(W, H, T, c->et.brick);
  k.slices = 1;
  return k;
}

int ctx_take_err(veckm_ctx* c, int32_t* host, void* stream) {
  return launch_take_err(c->w, host, stream);
}

int err_code(int32_t bits) {
  if (bits & kErrOverflow) return VECKM_E_OVERFLOW;
  if (bits & (kErrRange | kErrQuery)) return VECKM_E_RANGE;
  return VECKM_OK;
}

}  // namespace veckm

extern "C" {

int veckm_params_check(const veckm_params* params) {
  const int rc = check_params(params);
  if (rc) return rc;
  if (params->max_slices < 0 || params->max_voxels < 0) return VECKM_E_INVAL;
  if (voxels_of(params) > kMaxTotalVoxels) return VECKM_E_INVAL;
  return VECKM_OK;
}

int64_t veckm_workspace_bytes(const veckm_params* params, int32_t hidden) {
  const int rc = veckm_params_check(params);
  if (rc) return rc;
  if (hidden < 0) return VECKM_E_INVAL;
  const int rt_enc = params->rt < 0 ? 0 : params->rt;
  const SlotTable st = make_slots(params->rx, params->ry, rt_enc);
  return bytes_for(params, tilings_for(params, st.KP), st.KP, hidden);
}

int veckm_offset_table(const veckm_params* params, int32_t* k_count, int32_t* offsets,
                       uint16_t* phase_bits) {
  const int rc = check_params(params);
  if (rc) return rc;
  if (!k_count || params->rt < 0) return VECKM_E_INVAL;
  const OffsetTable t = make_offsets(params->rx, params->ry, params->rt);
  *k_count = t.K;
  if (offsets) std::memcpy(offsets, t.off.data(), t.off.size() * sizeof(int32_t));
  if (phase_bits) make_phase_bits(t, params->A, params->d, phase_bits);
  return VECKM_OK;
}

const char* veckm_strerror(int code) {
  switch (code) {
    case VECKM_OK: return "ok";
    case VECKM_E_INVAL: return "invalid argument";
    case VECKM_E_RANGE: return "input out of range";
    case VECKM_E_NOMEM: return "out of memory";
    case VECKM_E_BUDGET: return "memory budget exceeded";
    case VECKM_E_AGAIN: return "not ready";
    case VECKM_E_HIP: return "HIP runtime error";
    case VECKM_E_NODEVICE: return "no gfx950 device";
    case VECKM_E_OVERFLOW: return "too many events in one voxel";
    case VECKM_E_STATE: return "missing state (perceptron not set)";
    default: return "unknown error";
  }
}

int veckm_create(const veckm_params* params, veckm_ctx** out) {
  if (!out) return VECKM_E_INVAL;
  *out = nullptr;
  int rc = veckm_params_check(params);
  if (rc) return rc;
  veckm_ctx* c = new (std::nothrow) veckm_ctx();
  if (!c) return VECKM_E_NOMEM;
  rc = device_ok(&c->device, &c->num_cus);
  if (rc) {
    delete c;
    return rc;
  }
  c->p = *params;
  c->A.assign(params->A, params->A + 3 * params->d);
  c->p.A = c->A.data();
  c->max_slices = slices_of(params);
  EncodeTables& et = c->et;
  c->paper = params->rt < 0;
  // the 3-D window tables (the paper form never runs that encoder: its
  // tables are built with rt = 0 and only the brick numbering is used)
  const int rt_enc = c->paper ? 0 : params->rt;
  const SlotTable st = make_slots(params->rx, params->ry, rt_enc);
  et.K = st.K;
  et.KP = st.KP;
  et.na = params->precision == VECKM_FP32 ? 4 : 2;
  et.rx = params->rx;
  et.ry = params->ry;
  et.rt = rt_enc;
  et.d = params->d;
  const std::vector<Tiling> tl = tilings_for(params, st.KP);
  const std::vector<uint16_t> frag = make_slot_fragments(st, c->A.data(), params->d, et.na);
  const std::vector<uint16_t> wts = make_slot_weights(st);
  const Sizes s = sizes_for(params, tl);
  Workspace& w = c->w;
  uint16_t* dfrag = nullptr;
  std::vector<int32_t*> druns(tl.size(), nullptr);
  uint16_t* dwts = nullptr;
  uint32_t* dzeros = nullptr;
  float* rows = nullptr;
  rc = VECKM_OK;
  // the phase table's slabs, then room for W1 in the same slab order (the
  // fused encoder streams both through one ring: one contiguous array)
  const int nt = params->d / 16;
  const bool fusable = !c->paper && (nt == 4 || nt == 8);
  const size_t w1_room = fusable ? (size_t)(kMaxHidden / 32) * et.na * nt * 64 * 8 : 0;
  // (2 MB at least: one large page for the whole slab stream)
  const size_t frag_halves = std::max(frag.size() + w1_room, (size_t)1 << 20);
  rc = rc ? rc : dalloc(c->allocs, &dfrag, frag_halves);
  c->w1_slot = fusable && !rc ? dfrag + frag.size() : nullptr;
  for (size_t i = 0; i < tl.size(); ++i) rc = rc ? rc : dalloc(c->allocs, &druns[i], st.KP / 4);
  rc = rc ? rc : dalloc(c->allocs, &dwts, wts.size());
  rc = rc ? rc : dalloc(c->allocs, &dzeros, 64);
  rc = rc ? rc : dalloc(c->allocs, &w.count, (size_t)s.V);
  if (!c->paper) rc = rc ? rc : dalloc(c->allocs, &w.pairs, (size_t)s.P);
  if (!c->paper) rc = rc ? rc : dalloc(c->allocs, &w.lines, (size_t)s.lines);
  rc = rc ? rc : dalloc(c->allocs, &w.rank, (size_t)s.V);
  rc = rc ? rc : dalloc(c->allocs, &w.qmark, (size_t)s.V);
  rc = rc ? rc : dalloc(c->allocs, &w.ulist, (size_t)s.ulist);
  rc = rc ? rc : dalloc(c->allocs, &w.brick_nq, (size_t)s.nb);
  rc = rc ? rc : dalloc(c->allocs, &w.brick_off, (size_t)s.nb + 1);
  rc = rc ? rc : dalloc(c->allocs, &w.order, (size_t)s.nb * 4);
  rc = rc ? rc : dalloc(c->allocs, &w.scan_part, (size_t)((scan_tiles(s.nb) + 1) * kScanNV));
  int32_t* druns1 = nullptr;
  if (!c->paper) rc = rc ? rc : dalloc(c->allocs, &w.srow, (size_t)(2 * s.U));
  if (!c->paper) rc = rc ? rc : dalloc(c->allocs, &druns1, st.KP / 4);
  rc = rc ? rc : dalloc(c->allocs, &w.vox, (size_t)s.n);
  rc = rc ? rc : dalloc(c->allocs, &w.qmap, (size_t)s.n);
  rc = rc ? rc : dalloc(c->allocs, &rows, (size_t)(s.U * 2 * params->d));
  rc = rc ? rc : dalloc(c->allocs, &w.rowflow, (size_t)(s.U * 2));
  rc = rc ? rc : dalloc(c->allocs, &w.plan, 64);
  rc = rc ? rc : dalloc(c->allocs, &w.err, 1);
  rc = rc ? rc : dalloc(c->allocs, &c->table_dev, (size_t)kRing * c->max_slices);
  std::vector<float> ttab, xtab, ytab;
  float *dtt = nullptr, *dxt = nullptr, *dyt = nullptr;
  if (!rc && c->paper) {
    const int64_t V2 = (int64_t)params->width * params->height;
    const int D = params->d;
    make_paper_tables(c->A.data(), D, params->width, params->height, params->max_bins, &ttab,
                      &xtab, &ytab);
    rc = rc ? rc : dalloc(c->allocs, &w.G, (size_t)(2 * D * V2));
    rc = rc ? rc : dalloc(c->allocs, &w.S, (size_t)(2 * D * V2));
    rc = rc ? rc : dalloc(c->allocs, &w.cnt2, (size_t)V2);
    rc = rc ? rc : dalloc(c->allocs, &w.nbx, (size_t)V2);
    rc = rc ? rc : dalloc(c->allocs, &w.nbox, (size_t)V2);
    rc = rc ? rc : dalloc(c->allocs, &w.rowvox, (size_t)s.U);
    rc = rc ? rc : dalloc(c->allocs, &dtt, ttab.size());
    rc = rc ? rc : dalloc(c->allocs, &dxt, xtab.size());
    rc = rc ? rc : dalloc(c->allocs, &dyt, ytab.size());
    if (!rc && (hipMemcpy(dtt, ttab.data(), ttab.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
                hipMemcpy(dxt, xtab.data(), xtab.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
                hipMemcpy(dyt, ytab.data(), ytab.size() * 4, hipMemcpyHostToDevice) != hipSuccess))
      rc = VECKM_E_HIP;
    c->pt.ttab = dtt;
    c->pt.xtab = dxt;
    c->pt.ytab = dyt;
    c->pt.d = D;
    c->pt.rx = params->rx;
    c->pt.ry = params->ry;
  }
  if (!rc && !pinned_malloc(reinterpret_cast<void**>(&c->table_host),
                            (size_t)kRing * c->max_slices * sizeof(SliceDesc))) {
    c->table_host = nullptr;
    rc = VECKM_E_NOMEM;
  }
  for (int k = 0; !rc && k < kRing; ++k)
    if (hipEventCreateWithFlags(&c->ring_ev[k], hipEventDisableTiming) != hipSuccess) {
      c->ring_ev[k] = nullptr;
      rc = VECKM_E_HIP;
    }
  if (!rc && hipMemcpy(dfrag, frag.data(), frag.size() * 2, hipMemcpyHostToDevice) != hipSuccess)
    rc = VECKM_E_HIP;
  for (size_t i = 0; !rc && i < tl.size(); ++i) {
    const std::vector<int32_t> runs = make_run_offsets(st, tl[i].brick, params->rx, params->ry);
    if (hipMemcpy(druns[i], runs.data(), runs.size() * 4, hipMemcpyHostToDevice) != hipSuccess)
      rc = VECKM_E_HIP;
  }
  if (!rc && druns1) {  // a single voxel's count box (rows of bricks with few rows)
    const std::vector<int32_t> runs = make_run_offsets(st, Brick{1, 1, 1}, params->rx, params->ry);
    if (hipMemcpy(druns1, runs.data(), runs.size() * 4, hipMemcpyHostToDevice) != hipSuccess)
      rc = VECKM_E_HIP;
  }
  if (!rc && hipMemcpy(dwts, wts.data(), wts.size() * 2, hipMemcpyHostToDevice) != hipSuccess)
    rc = VECKM_E_HIP;
  if (!rc && hipMemset(dzeros, 0, 64 * sizeof(uint32_t)) != hipSuccess) rc = VECKM_E_HIP;
  if (!rc && hipMemset(w.err, 0, sizeof(int32_t)) != hipSuccess) rc = VECKM_E_HIP;
  if (!rc && hipMemset(w.qmark, 0, (size_t)s.V) != hipSuccess) rc = VECKM_E_HIP;
  if (!rc && hipMemset(w.count, 0, (size_t)s.V * 4) != hipSuccess) rc = VECKM_E_HIP;
  if (!rc && !c->paper &&
      (hipMemset(w.pairs, 0, (size_t)s.P * 4) != hipSuccess ||
       hipMemset(w.lines, 0, (size_t)s.lines) != hipSuccess))
    rc = VECKM_E_HIP;
  if (!rc && hipMemset(w.plan, 0, 64 * sizeof(int32_t)) != hipSuccess) rc = VECKM_E_HIP;
  if (!rc && hipDeviceSynchronize() != hipSuccess) rc = VECKM_E_HIP;
  if (rc) {
    veckm_destroy(c);
    return rc;
  }
  w.rows = rows;
  w.zeros = dzeros;
  w.vmax = s.V;
  w.pmax = s.P;
  w.nmax = s.n;
  w.bmax = s.nb;
  w.umax = s.ulist;
  et.frag = dfrag;
  et.wts = dwts;
  for (size_t i = 0; i < tl.size(); ++i) {
    EncodeTables t = et;
    t.brick = tl[i].brick;
    t.nbuf = tl[i].nbuf;
    t.layout = tl[i].layout;
    t.runs = druns[i];
    // single rows: as many single-voxel boxes as fit in the brick's box (up
    // to one 16-row tile); worth it from 8 on
    t.runs1 = druns1;
    const int vol1 = box_dwords(Brick{1, 1, 1}, params->rx, params->ry, rt_enc);
    t.rs = std::min(16, box_dwords(t.brick, params->rx, params->ry, rt_enc) / vol1);
    t.sp = druns1 && t.rs >= 8 ? kSparseBelow : 0;
    c->tilings.push_back(t);
  }
  c->et = c->tilings[0];
  c->tiling = 0;
  *out = c;
  return VECKM_OK;
}

void veckm_destroy(veckm_ctx* ctx) {
  if (!ctx) return;
  (void)hipDeviceSynchronize();
  for (void* p : ctx->allocs) (void)hipFree(p);
  for (void* p : ctx->mlp_allocs) (void)hipFree(p);
  for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
  for (hipEvent_t e : ctx->ring_ev)
    if (e) (void)hipEventDestroy(e);
  if (ctx->table_host) (void)hipHostFree(ctx->table_host);
  delete ctx;
}

int veckm_set_mlp(veckm_ctx* ctx, int32_t hidden, const float* W1, const float* b1,
                  const float* W2, const float* b2) {
  if (!ctx || !W1 || !b1 || !W2 || !b2) return VECKM_E_INVAL;
  if (hidden < 64 || hidden > kMaxHidden || hidden % 64) return VECKM_E_INVAL;
  const int K2 = 2 * ctx->p.d;
  (void)hipDeviceSynchronize();
  for (void* p : ctx->mlp_allocs) (void)hipFree(p);
  ctx->mlp_allocs.clear();
  ctx->mw = MlpWeights{};
  float *dW1 = nullptr, *db1 = nullptr, *dW2 = nullptr, *db2 = nullptr;
  uint16_t *dW1b = nullptr, *dW1h = nullptr, *dW1l = nullptr;
  int rc = VECKM_OK;
  rc = rc ? rc : dalloc(ctx->mlp_allocs, &dW1, (size_t)hidden * K2);
  rc = rc ? rc : dalloc(ctx->mlp_allocs, &dW1b, (size_t)hidden * K2);
  rc = rc ? rc : dalloc(ctx->mlp_allocs, &dW1h, (size_t)hidden * K2);
  rc = rc ? rc : dalloc(ctx->mlp_allocs, &dW1l, (size_t)hidden * K2);
  rc = rc ? rc : dalloc(ctx->mlp_allocs, &db1, (size_t)hidden);
  rc = rc ? rc : dalloc(ctx->mlp_allocs, &dW2, (size_t)2 * hidden);
  rc = rc ? rc : dalloc(ctx->mlp_allocs, &db2, 2);
  if (rc) return rc;
  std::vector<uint16_t> w1b((size_t)hidden * K2), w1h(w1b.size()), w1l(w1b.size());
  for (size_t i = 0; i < w1b.size(); ++i) w1b[i] = bf16_bits_rne(W1[i]);
  // fp16 hi/lo pair of W1 * 2^s, with s putting max |W1| * 2^s in [1, 2) so
  // that the lo parts of all but the smallest weights stay normal
  double wmax = 0.0;
  for (size_t i = 0; i < w1b.size(); ++i) wmax = std::max(wmax, std::fabs((double)W1[i]));
  int e = 0;
  if (wmax > 0.0) std::frexp(wmax, &e);  // wmax = f 2^e, f in [0.5, 1)
  const int shift = wmax > 0.0 ? 1 - e : 0;
  for (size_t i = 0; i < w1b.size(); ++i) {
    const double v = std::ldexp((double)W1[i], shift);
    w1h[i] = fp16_bits_rne(v);
    w1l[i] = fp16_bits_rne(v - fp16_to_double(w1h[i]));
  }
  if (hipMemcpy(dW1, W1, (size_t)hidden * K2 * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(dW1b, w1b.data(), w1b.size() * 2, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(dW1h, w1h.data(), w1h.size() * 2, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(dW1l, w1l.data(), w1l.size() * 2, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(db1, b1, (size_t)hidden * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(dW2, W2, (size_t)2 * hidden * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(db2, b2, 8, hipMemcpyHostToDevice) != hipSuccess)
    return VECKM_E_HIP;
  ctx->mw.hidden = hidden;
  ctx->mw.W1 = dW1;
  ctx->mw.W1b = dW1b;
  ctx->mw.W1h = dW1h;
  ctx->mw.W1l = dW1l;
  ctx->mw.unscale = (float)std::ldexp(1.0, -shift);
  ctx->mw.b1 = db1;
  ctx->mw.W2 = dW2;
  ctx->mw.b2 = db2;
  // W1 in the slab order of the encoder that runs the perceptron itself (the
  // pipelined wave layouts at D = 64 or 128), right after the phase table
  if (ctx->w1_slot) {
    const std::vector<uint16_t> wf = make_w1_fragments(W1, hidden, ctx->p.d, ctx->et.na, shift);
    if (hipMemcpy(ctx->w1_slot, wf.data(), wf.size() * 2, hipMemcpyHostToDevice) != hipSuccess) {
      ctx->mw = MlpWeights{};
      return VECKM_E_HIP;
    }
    ctx->mw.W1frag = ctx->w1_slot;
  }
  return VECKM_OK;
}

int veckm_encode(veckm_ctx* ctx, const veckm_event* events, int64_t n, int32_t t0,
                 int32_t nbins, const int32_t* queries, int64_t m, float* emb, void* stream) {
  if (!ctx || ctx->window) return VECKM_E_INVAL;
  Batch bt;
  const int rc = single_batch(ctx, events, n, t0, nbins, queries, m, emb, &bt);
  if (rc) return rc;
  return run(ctx, ctx->w, bt, events, queries, emb, nullptr, stream);
}

int veckm_flow(veckm_ctx* ctx, const veckm_event* events, int64_t n, int32_t t0,
               int32_t nbins, const int32_t* queries, int64_t m, float* flow, void* stream) {
  if (!ctx || ctx->window) return VECKM_E_INVAL;
  Batch bt;
  const int rc = single_batch(ctx, events, n, t0, nbins, queries, m, flow, &bt);
  if (rc) return rc;
  if (ctx->mw.hidden == 0) return VECKM_E_STATE;
  return run(ctx, ctx->w, bt, events, queries, nullptr, flow, stream);
}

int veckm_count(veckm_ctx* ctx, const veckm_event* events, int64_t n, int32_t t0,
                int32_t nbins, const int32_t* queries, int64_t m, int32_t* counts,
                void* stream) {
  if (!ctx || ctx->window || ctx->paper) return VECKM_E_INVAL;
  Batch bt;
  const int rc = single_batch(ctx, events, n, t0, nbins, queries, m, counts, &bt);
  if (rc) return rc;
  return run(ctx, ctx->w, bt, events, queries, nullptr, nullptr, stream, counts);
}

// ---- sliding window ------------------------------------------------------

int veckm_window_create(const veckm_params* params, veckm_ctx** out) {
  if (!out) return VECKM_E_INVAL;
  *out = nullptr;
  if (!params || params->rt < 0 || params->max_slices > 1) return VECKM_E_INVAL;
  veckm_ctx* c = nullptr;
  int rc = veckm_create(params, &c);
  if (rc) return rc;
  c->window = true;
  // an empty window: every plane of the ring holds zero counts
  const int64_t V = (int64_t)params->width * params->height * params->max_bins;
  const int64_t P = (int64_t)(params->width + 1) * params->height * params->max_bins;
  if (hipMemset(c->w.count, 0, (size_t)V * 4) != hipSuccess ||
      hipMemset(c->w.pairs, 0, (size_t)P * 4) != hipSuccess ||
      hipDeviceSynchronize() != hipSuccess) {
    veckm_destroy(c);
    return VECKM_E_HIP;
  }
  *out = c;
  return VECKM_OK;
}

int veckm_window_push(veckm_ctx* ctx, const veckm_event* events, int64_t n, int32_t t0,
                      int32_t nbins, void* stream) {
  if (!ctx || !ctx->window || n < 0 || (n > 0 && !events)) return VECKM_E_INVAL;
  if (n > ctx->p.max_events) return VECKM_E_RANGE;
  const int T = ctx->p.max_bins;
  if (nbins < 1 || nbins > T) return VECKM_E_RANGE;
  if (ctx->started && (int64_t)t0 < ctx->wend) return VECKM_E_INVAL;  // bins arrive in order
  const int32_t tref = ctx->started ? ctx->tref : t0;
  const int64_t wend0 = ctx->started ? ctx->wend : (int64_t)t0;
  const int64_t end = (int64_t)t0 + nbins;
  const int64_t b0 = end - T > wend0 ? end - T : wend0;  // bins entering the window
  const int rc = launch_window_push(ctx->w, events, n, ctx->p.width, ctx->p.height, T, t0, nbins,
                                    tref, b0, (int)(end - b0), stream);
  if (rc) return rc;
  ctx->started = true;
  ctx->tref = tref;
  ctx->wend = end;
  return VECKM_OK;
}

namespace {

int window_batch(veckm_ctx* c, const veckm_event* queries, int64_t m, const void* out,
                 Batch* bt) {
  if (!c || !c->window || m < 0 || (m > 0 && (!queries || !out))) return VECKM_E_INVAL;
  if (!c->started) return VECKM_E_STATE;
  if (m > c->p.max_events) return VECKM_E_RANGE;
  const int T = c->p.max_bins;
  const int64_t start = c->wend - T;  // may precede the first push: those planes are empty
  if (start < INT32_MIN) return VECKM_E_RANGE;
  bt->s0 = describe(c, c->p.width, c->p.height, T, (int32_t)start, 0, 0, 0, 0, m);
  bt->s0.tshift = (int)(((start - c->tref) % T + T) % T);
  bt->table = nullptr;
  bt->nslices = 1;
  bt->nbricks = bt->s0.nbx * bt->s0.nby * bt->s0.nbt;
  bt->n = (int)m;
  bt->m = (int)m;
  bt->nvox = (int64_t)c->p.width * c->p.height * T;
  bt->npairs = (int64_t)(c->p.width + 1) * c->p.height * T;
  bt->max_rows = (int64_t)c->p.height * T;
  return VECKM_OK;
}

}  // namespace

int veckm_window_encode(veckm_ctx* ctx, const veckm_event* queries, int64_t m, float* emb,
                        void* stream) {
  Batch bt;
  const int rc = window_batch(ctx, queries, m, emb, &bt);
  if (rc) return rc;
  return run(ctx, ctx->w, bt, queries, nullptr, emb, nullptr, stream);
}

int veckm_window_flow(veckm_ctx* ctx, const veckm_event* queries, int64_t m, float* flow,
                      void* stream) {
  Batch bt;
  const int rc = window_batch(ctx, queries, m, flow, &bt);
  if (rc) return rc;
  if (ctx->mw.hidden == 0) return VECKM_E_STATE;
  return run(ctx, ctx->w, bt, queries, nullptr, nullptr, flow, stream);
}

int veckm_encode_batch(veckm_ctx* ctx, const veckm_slice* slices, int32_t count,
                       const veckm_event* events, float* emb, void* stream) {
  if (!ctx || ctx->paper || ctx->window) return VECKM_E_INVAL;
  Batch bt;
  int slot;
  int rc = multi_batch(ctx, slices, count, events, emb, stream, &bt, &slot);
  if (rc) return rc;
  rc = run(ctx, ctx->w, bt, events, nullptr, emb, nullptr, stream);
  const int rc2 = release_slot(ctx, slot, stream);
  return rc ? rc : rc2;
}

int veckm_flow_batch(veckm_ctx* ctx, const veckm_slice* slices, int32_t count,
                     const veckm_event* events, float* flow, void* stream) {
  if (!ctx || ctx->paper || ctx->window) return VECKM_E_INVAL;
  if (ctx->mw.hidden == 0) return VECKM_E_STATE;
  Batch bt;
  int slot;
  int rc = multi_batch(ctx, slices, count, events, flow, stream, &bt, &slot);
  if (rc) return rc;
  rc = run(ctx, ctx->w, bt, events, nullptr, nullptr, flow, stream);
  const int rc2 = release_slot(ctx, slot, stream);
  return rc ? rc : rc2;
}

// ---- launch graphs

struct veckm_graph {
  veckm_ctx* ctx = nullptr;
  SliceDesc* table = nullptr;  // device copy of the batch's slice table
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

void veckm_graph_destroy(veckm_graph* g) {
  if (!g) return;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  if (g->table) (void)hipFree(g->table);
  delete g;
}

int veckm_graph_create(veckm_ctx* ctx, const veckm_slice* slices, int32_t count,
                       const veckm_event* events, float* out, int32_t flow, veckm_graph** g) {
  if (!g) return VECKM_E_INVAL;
  *g = nullptr;
  if (!ctx || ctx->paper || ctx->window) return VECKM_E_INVAL;
  if (flow && ctx->mw.hidden == 0) return VECKM_E_STATE;
  std::vector<SliceDesc> tab;
  Batch bt;
  int rc = plan_batch(ctx, slices, count, events, out, tab, &bt);
  if (rc) return rc;
  veckm_graph* gr = new veckm_graph;
  gr->ctx = ctx;
  if (!dev_malloc(reinterpret_cast<void**>(&gr->table), tab.size() * sizeof(SliceDesc))) {
    (void)hipGetLastError();
    gr->table = nullptr;
    veckm_graph_destroy(gr);
    return VECKM_E_NOMEM;
  }
  if (hipMemcpy(gr->table, tab.data(), tab.size() * sizeof(SliceDesc), hipMemcpyHostToDevice) !=
      hipSuccess) {
    veckm_graph_destroy(gr);
    return VECKM_E_HIP;
  }
  bt.table = gr->table;
  // capture the launch sequence on a stream of our own (stage timing off:
  // its events belong to eager calls)
  hipStream_t s = nullptr;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
    veckm_graph_destroy(gr);
    return VECKM_E_HIP;
  }
  const bool prof = ctx->prof;
  ctx->prof = false;
  rc = hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed) == hipSuccess ? VECKM_OK : VECKM_E_HIP;
  if (!rc) {
    rc = run(ctx, ctx->w, bt, events, nullptr, flow ? nullptr : out, flow ? out : nullptr, s);
    hipGraph_t graph = nullptr;
    if (hipStreamEndCapture(s, &graph) != hipSuccess && !rc) rc = VECKM_E_HIP;
    gr->graph = graph;
  }
  ctx->prof = prof;
  if (!rc && hipGraphInstantiate(&gr->exec, gr->graph, nullptr, nullptr, 0) != hipSuccess)
    rc = VECKM_E_HIP;
  (void)hipStreamDestroy(s);
  if (rc) {
    veckm_graph_destroy(gr);
    return rc;
  }
  *g = gr;
  return VECKM_OK;
}

int veckm_graph_launch(veckm_graph* g, void* stream) {
  if (!g || !g->exec) return VECKM_E_INVAL;
  return hipGraphLaunch(g->exec, (hipStream_t)stream) == hipSuccess ? VECKM_OK : VECKM_E_HIP;
}

// ---- encoder tilings and the tuner

int veckm_tiling_count(const veckm_ctx* ctx) {
  return ctx ? (int)ctx->tilings.size() : VECKM_E_INVAL;
}

int veckm_tiling_selected(const veckm_ctx* ctx) { return ctx ? ctx->tiling : VECKM_E_INVAL; }

int veckm_tiling_info(const veckm_ctx* ctx, int32_t index, int32_t* info) {
  if (!ctx || !info || index < 0 || index >= (int)ctx->tilings.size()) return VECKM_E_INVAL;
  const EncodeTables& t = ctx->tilings[(size_t)index];
  info[0] = t.brick.bx;
  info[1] = t.brick.by;
  info[2] = t.brick.bt;
  info[3] = t.nbuf;
  info[4] = t.layout;
  return VECKM_OK;
}

int veckm_tiling_select(veckm_ctx* ctx, int32_t index) {
  if (!ctx || index < 0 || index >= (int)ctx->tilings.size()) return VECKM_E_INVAL;
  ctx->et = ctx->tilings[(size_t)index];
  ctx->tiling = index;
  return VECKM_OK;
}

int veckm_tune(veckm_ctx* ctx, const veckm_slice* slices, int32_t count,
               const veckm_event* events, int32_t reps, void* stream, int32_t* chosen) {
  if (!ctx || ctx->paper || ctx->window || reps < 1 || reps > 100) return VECKM_E_INVAL;
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return VECKM_E_HIP;
  }
  // the rows the flow path would write (the epilogue differs, the work not);
  // with a perceptron set, each tiling is timed with the perceptron as a flow
  // call runs it (inside the encoder where the tiling allows, else after it)
  const bool with_mlp = ctx->mw.hidden > 0;
  const int split_rows = ctx->p.precision == VECKM_FP16 ? kRowsBF16
                         : with_mlp && mlp_rows_split(ctx->p.d, ctx->mw.hidden)
                             ? kRowsHiLo16
                             : kRowsF32;
  const int prev = ctx->tiling;
  int best = -1, rc = VECKM_OK;
  float best_ms = 0.f;
  for (int i = 0; !rc && i < (int)ctx->tilings.size(); ++i) {
    ctx->et = ctx->tilings[(size_t)i];
    const bool fused = with_mlp && ctx->mw.W1frag && encode_fusable(ctx->et, ctx->mw.hidden);
    const int rows = fused ? (ctx->p.precision == VECKM_FP16 ? kFlowBF16 : kFlowHiLo16) : split_rows;
    for (int r = 0; !rc && r <= reps; ++r) {  // one untimed run, then reps timed
      if (r == 1 && hipEventRecord(e0, s) != hipSuccess) rc = VECKM_E_HIP;
      Batch bt;
      int slot = -1;
      // (the output argument is only checked for presence; nothing is written)
      if (!rc) rc = multi_batch(ctx, slices, count, events, events, stream, &bt, &slot);
      if (!rc && bt.m > 0) {
        // (the grids return to zero as in a batch call)
        rc = launch_prepare(bt, ctx->w, events, nullptr, ctx->et, true, stream);
        if (!rc)
          rc = launch_encode(bt, ctx->w, ctx->et, rows, ctx->num_cus, stream, nullptr,
                             &ctx->mw);
        if (!rc && with_mlp && !fused)
          rc = launch_mlp(ctx->w, ctx->mw, ctx->p.d, rows, ctx->num_cus, stream);
        const int rc3 =
            rc ? launch_clear_grids(bt, ctx->w,
                                    (int64_t)bt.nbricks * ctx->et.brick.by * ctx->et.brick.bt,
                                    stream)
               : launch_clear_events(bt, ctx->w, stream);
        rc = rc ? rc : rc3;
      }
      const int rc2 = release_slot(ctx, slot, stream);
      rc = rc ? rc : rc2;
    }
    float ms = 0.f;
    if (!rc && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
      rc = VECKM_E_HIP;
    if (!rc && (best < 0 || ms < best_ms)) {
      best = i;
      best_ms = ms;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  const int pick = rc ? prev : best;
  ctx->et = ctx->tilings[(size_t)pick];
  ctx->tiling = pick;
  if (!rc && chosen) *chosen = best;
  return rc;
}

int veckm_profile_enable(veckm_ctx* ctx, int32_t enable) {
  if (!ctx) return VECKM_E_INVAL;
  ctx->prof = enable != 0;
  if (ctx->prof && ctx->ev_pool.empty()) {
    ctx->ev_pool.resize(8192);
    for (auto& e : ctx->ev_pool)
      if (hipEventCreate(&e) != hipSuccess) {
        ctx->prof = false;
        return VECKM_E_HIP;
      }
  }
  return VECKM_OK;
}

int veckm_profile_read(veckm_ctx* ctx, double* ms, int64_t* count, int32_t nstages) {
  if (!ctx || !ms || !count || nstages < 0) return VECKM_E_INVAL;
  for (int s = 0; s < nstages; ++s) {
    ms[s] = 0.0;
    count[s] = 0;
  }
  int rc = VECKM_OK;
  for (const auto& mk : ctx->marks) {
    float t = 0.f;
    if (hipEventSynchronize(mk.b) != hipSuccess ||
        hipEventElapsedTime(&t, mk.a, mk.b) != hipSuccess) {
      rc = VECKM_E_HIP;
      continue;
    }
    if (mk.stage < nstages) {
      ms[mk.stage] += t;
      count[mk.stage] += 1;
    }
  }
  ctx->marks.clear();
  ctx->ev_next = 0;
  return rc;
}

int veckm_last_rows(veckm_ctx* ctx, void* stream, int64_t* rows) {
  if (!ctx || !rows) return VECKM_E_INVAL;
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return VECKM_E_HIP;
  int32_t u = 0;
  if (hipMemcpy(&u, ctx->w.plan, 4, hipMemcpyDeviceToHost) != hipSuccess) return VECKM_E_HIP;
  *rows = u;
  return VECKM_OK;
}

// ---- allocation-free flow

}  // extern "C"

namespace {

// The per-call workspaces of veckm_flow_noalloc live in this array (one copy
// per GPU, held until the process ends).  Host code never passes its name to
// a kernel: it is a host-side stand-in; the device address comes from
// hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char scratch[VECKM_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};

// The device address of `scratch` on `device`, looked up with that device
// current on the first call for it.
int scratch_on(int device, unsigned char** out) {
  if (device < 0 || device >= kMaxScratchDevices) return VECKM_E_NODEVICE;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return VECKM_E_HIP;
    if (cur != device && hipSetDevice(device) != hipSuccess) return VECKM_E_HIP;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return VECKM_E_HIP;
    }
    g_scratch_ptr[device] = ptr;
  }
  *out = static_cast<unsigned char*>(g_scratch_ptr[device]);
  return VECKM_OK;
}

// Carves the workspaces of one slice call out of `base` (256-byte aligned
// pieces); returns the bytes needed.  With base == nullptr only sizes.
int64_t carve_noalloc(const veckm_ctx* c, const Batch& bt, unsigned char* base, Workspace* w) {
  const Brick& b = c->et.brick;
  const int64_t V = bt.nvox, P = bt.npairs, nb = bt.nbricks, n = bt.n;
  const int64_t U = n < V ? n : V;
  int64_t off = 0;
  auto take = [&](int64_t bytes) -> unsigned char* {
    unsigned char* p = base ? base + off : nullptr;
    off += (bytes + 255) / 256 * 256;
    return p;
  };
  w->count = reinterpret_cast<int32_t*>(take(V * 4));
  w->pairs = reinterpret_cast<uint32_t*>(take(P * 4));
  w->lines = take(nb * b.by * b.bt);
  w->rank = reinterpret_cast<int32_t*>(take(V * 4));
  w->qmark = nullptr;  // read only for query subsets
  w->ulist = reinterpret_cast<int32_t*>(take(nb * b.volume() * 4));
  w->brick_nq = reinterpret_cast<int32_t*>(take(nb * 4));
  w->brick_off = reinterpret_cast<int32_t*>(take((nb + 1) * 4));
  w->order = reinterpret_cast<int32_t*>(take(nb * 16));
  w->scan_part = reinterpret_cast<int32_t*>(take((scan_tiles(nb) + 1) * kScanNV * 4));
  w->srow = reinterpret_cast<int32_t*>(take(U * 8));
  w->vox = reinterpret_cast<int32_t*>(take(n * 4));
  w->qmap = nullptr;  // read only by the paper form
  w->rows = take(U * 2 * c->p.d * 4);
  w->rowflow = reinterpret_cast<float*>(take(U * 8));
  w->plan = reinterpret_cast<int32_t*>(take(64 * 4));
  w->vmax = V;
  w->pmax = P;
  w->nmax = n;
  w->bmax = nb;
  w->umax = nb * b.volume();
  return off;
}

}  // namespace

extern "C" {

int veckm_flow_noalloc(veckm_ctx* ctx, const veckm_event* events, int64_t n, int32_t t0,
                       int32_t nbins, float* flow, void* stream) {
  if (!ctx || ctx->window || ctx->paper) return VECKM_E_INVAL;
  Batch bt;
  int rc = single_batch(ctx, events, n, t0, nbins, nullptr, n, flow, &bt);
  if (rc) return rc;
  if (ctx->mw.hidden == 0) return VECKM_E_STATE;
  if (n == 0) return VECKM_OK;
  Workspace w = ctx->w;  // tables, zero page and error flag stay the context's
  if (carve_noalloc(ctx, bt, nullptr, &w) > (int64_t)VECKM_NOALLOC_SCRATCH_BYTES)
    return VECKM_E_BUDGET;
  unsigned char* base = nullptr;
  rc = scratch_on(ctx->device, &base);
  if (rc) return rc;
  carve_noalloc(ctx, bt, base, &w);
  // the array holds whatever the last call left: the count and pair grids
  // and the row flags start at zero (fill kernels, no memset)
  rc = launch_clear_grids(bt, w, bt.nbricks * (int64_t)ctx->et.brick.by * ctx->et.brick.bt,
                          stream);
  if (rc) return rc;
  return run(ctx, w, bt, events, nullptr, nullptr, flow, stream);
}

int veckm_status(veckm_ctx* ctx, void* stream) {
  if (!ctx) return VECKM_E_INVAL;
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return VECKM_E_HIP;
  int32_t bits = 0;
  if (hipMemcpy(&bits, ctx->w.err, 4, hipMemcpyDeviceToHost) != hipSuccess) return VECKM_E_HIP;
  if (bits && hipMemset(ctx->w.err, 0, 4) != hipSuccess) return VECKM_E_HIP;
  return err_code(bits);
}

}  // extern "C"
