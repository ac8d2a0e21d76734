// Internal declarations of the veckm library (not part of the C-ABI).
#pragma once

#include <cstddef>
#include <cstdint>
#include <vector>

#include "../../include/veckm.h"

namespace veckm {

// Window radius limits (the LDS count volume and the offset table must fit).
constexpr int kMaxRxy = 12;
constexpr int kMaxRt = 6;
constexpr int kKStep = 32;  // K elements per MFMA k-step (16x16x32 f16)
constexpr int kMaxSlabBuffers = 4;  // phase-table slabs the encoder keeps in LDS (2..4)

// Device-side input error bits (OR-ed into a device int).
constexpr int kErrRange = 1;     // event outside sensor / time window, or |p| != 1
constexpr int kErrQuery = 2;     // query index outside [0, n)
constexpr int kErrOverflow = 4;  // more than VECKM_MAX_VOXEL_EVENTS in a voxel

// Brick (x, y, t) that one encoder work item covers.
struct Brick {
  int bx, by, bt;
  int volume() const { return bx * by * bt; }
};

// Offsets of the half window (entry 0 is the centre), their phase table in
// the matrix-core fragment layout, and LDS deltas for a given brick.
struct OffsetTable {
  int K = 0;        // real offsets (centre + half window)
  int KP = 0;       // padded to a multiple of kKStep
  std::vector<int32_t> off;  // K x 3 (dx, dy, dt)
};

// The encoder's k-slot layout: the half window cut into runs of 4
// consecutive dx offsets (each window row padded to a multiple of 4 with
// zero-weight slots), so that every 8-slot group of an MFMA lane is two
// runs that the kernel reads with one address each.
struct SlotTable {
  int K = 0;   // real offsets
  int KP = 0;  // slots, a multiple of kKStep
  std::vector<int32_t> slot;  // KP x 4: dx, dy, dt, kind (0 pad, 1 offset, 2 centre)
};

int check_params(const veckm_params* p);
SlotTable make_slots(int rx, int ry, int rt);
// Fragment-native table over the slot layout: [ks][a][nt][lane][8] halves.
std::vector<uint16_t> make_slot_fragments(const SlotTable& t, const double* A, int d, int na);
// LDS voxel-index delta of the first slot of every run, laid out
// [ks][lane group][2].
std::vector<int32_t> make_run_offsets(const SlotTable& t, const Brick& b, int rx, int ry);
// fp16 bit patterns of the neighbour-count weight of every slot (1 for an
// offset, 1/2 for the centre, 0 for padding).
std::vector<uint16_t> make_slot_weights(const SlotTable& t);
OffsetTable make_offsets(int rx, int ry, int rt);
// FP64 phases -> fp16 bit patterns [k][j][4] = (cos hi, cos lo, sin hi, sin lo).
void make_phase_bits(const OffsetTable& t, const double* A, int d, uint16_t* out);
// false when no brick's count box fits in LDS beside two table slabs
bool choose_layout(int rx, int ry, int rt, int d, int precision, int kp, Brick* brick, int* nbuf);
// An encoder tiling: brick shape and table slabs buffered in LDS.
struct Tiling {
  Brick brick{32, 16, 8};
  int nbuf = 2;
  int layout = 0;  // encoder wave layout: 0 = 16 waves x 2 row tiles, 1 = 8 waves x 4 row tiles,
                   // 2 = 4 and 3 = 8 pipelined waves over all frequencies of their rows
};
constexpr int kMaxBrickVoxels = 8192;  // largest brick (the ranking kernel's limit)
// Work items of the encoder that hold single rows carry this bit in their
// brick field (brick numbers stay below it).
constexpr int kSparseTag = 1 << 30;
// Bricks with fewer rows than this go to the encoder row by row (each row
// with its own count box, up to 16 rows per item), when 8 or more such
// boxes fit in the LDS of the brick's box.
constexpr int kSparseBelow = 12;
std::vector<Tiling> tiling_candidates(int rx, int ry, int rt, int d, int precision, int kp);
size_t encode_lds_need(int d, int precision, int nbuf, int kp, int vol, int layout = 0);
int encode_rows_per_chunk(int d, int layout);
int encode_waves(int layout = 0);  // waves per encoder block
int lds_volume_halves(const Brick& b, int rx, int ry, int rt);
// The encoder's LDS box of a brick: the brick plus the window halo, widened
// by kRunPad columns on each side in x so that no 4-offset run of the slot
// layout ever leaves a box row.
constexpr int kRunPad = 3;
inline int box_sx(const Brick& b, int rx) { return b.bx + 2 * rx + 2 * kRunPad; }
inline int box_dwords(const Brick& b, int rx, int ry, int rt) {
  return box_sx(b, rx) * (b.by + 2 * ry) * (b.bt + 2 * rt);
}
uint16_t fp16_bits_rne(double v);
double fp16_to_double(uint16_t h);
uint16_t bf16_bits_rne(float v);

// ---------------------------------------------------------------- launches
// One slice of a call: its sensor, time window, events and its region of the
// shared grids and brick list.  Slices lie back to back in every array.
struct SliceDesc {
  int W, H, T;        // grid extent (T = nbins)
  int t0;             // time of bin 0
  int nbx, nby, nbt;  // bricks per axis
  int brick_off;      // first global brick
  int64_t grid_off;   // first voxel in the count / rank / mark grids
  int64_t pair_off;   // first entry in the pair grid (rows of W + 1 entries)
  int ev_off, n;      // events [ev_off, ev_off + n)
  int tshift;         // the count / pair grids hold bin t in plane (t + tshift) mod T (a
                      // sliding window's ring; 0 otherwise)
};

// Everything the kernels need to know about the slices of one call.
struct Batch {
  SliceDesc s0;              // the slice when nslices == 1
  const SliceDesc* table;    // device copy of all slices when nslices > 1
  int nslices;
  int nbricks;               // total bricks
  int n;                     // total events
  int m;                     // total queries
  int64_t nvox;              // total voxels
  int64_t npairs;            // total pair-grid entries (sum of (W + 1) H T)
  int64_t max_rows;          // most x rows (H T) in one slice
};

// The brick scan works on tiles of kScanTile bricks and keeps kScanNV
// partial sums per tile.
constexpr int kScanTile = 8192;
constexpr int kScanNV = 14;
inline int64_t scan_tiles(int64_t nb) { return (nb + kScanTile - 1) / kScanTile; }

struct Workspace {
  int32_t* count = nullptr;     // voxels: int32 event counts, slices back to back; all zero
                                // between slice calls (k_clear_events returns the events'
                                // voxels to zero after each call; the paper form fills it
                                // before its scatter)
  uint32_t* pairs = nullptr;    // (W + 1) H T per slice: entry x + 1 of a row holds the fp16
                                // counts of voxels x and x + 1 of that row, x in [-1, W); all
                                // zero between bounded-window slice calls, like count
  uint8_t* lines = nullptr;     // bricks x (by bt): 1 where the brick's x row holds an event;
                                // all zero between slice calls (the ranking kernel clears them)
  const uint32_t* zeros = nullptr;  // 64 zero dwords (out-of-grid reads)
  int32_t* rank = nullptr;      // voxels: brick-local rank of query voxels
  uint8_t* qmark = nullptr;     // voxels: query-voxel marks (query subsets, windows); all zero
                                // between calls (the ranking pass clears the marks it reads)
  int32_t* ulist = nullptr;     // bricks * brick volume: brick-local voxel of each rank
  int32_t* brick_nq = nullptr;  // bricks
  int32_t* brick_off = nullptr; // bricks + 1 (exclusive scan)
  int32_t* order = nullptr;     // 4 x bricks: the encoder's work list, most chunks first;
                                // per brick {brick, rows, first row, slice}
  int32_t* scan_part = nullptr; // kScanNV ints per kScanTile bricks (brick-scan partials)
  int32_t* srow = nullptr;      // 2 U: {brick, brick-local voxel} of each row of the bricks the
                                // encoder takes row by row (numbered after all other rows)
  int32_t* vox = nullptr;       // n: slice-local voxel of each event, -1 if invalid
  int32_t* qmap = nullptr;      // m: row of each query, -1 if invalid
  int32_t* rowvox = nullptr;    // U: voxel of each row (paper form only)
  void* rows = nullptr;         // U x 2D encodings (fp32 or bf16)
  float* rowflow = nullptr;     // U x 2
  int32_t* plan = nullptr;      // [0] = U, [1] = work counter, [2] = non-empty bricks
  int32_t* err = nullptr;       // error bits
  int64_t vmax = 0, pmax = 0, nmax = 0, bmax = 0, umax = 0;
  // paper form (no temporal bound) only
  float* G = nullptr;           // [D/8][H][W][8] complex: per-pixel temporal phase sums
  float* S = nullptr;           // [D/8][H][W][8] complex: window sums
  int32_t* cnt2 = nullptr;      // [H][W] events per pixel
  int32_t* nbx = nullptr;       // [H][W] x box sums of cnt2
  int32_t* nbox = nullptr;      // [H][W] window counts
};

// Phase tables of the paper form: (cos, sin) of A_t[j] t for the bins of a
// slice, of A_x[j] x over the sensor columns and of A_y[j] y over its rows
// (FP64 on the host, rounded to fp32).
struct PaperTables {
  const float* ttab = nullptr;  // [max_bins][D][cos, sin]
  const float* xtab = nullptr;  // [width][D][cos, sin]
  const float* ytab = nullptr;  // [height][D][cos, sin]
  int d = 0, rx = 0, ry = 0;
};

struct EncodeTables {
  const uint16_t* frag = nullptr;  // fragment-native phase table over the slots
  const int32_t* runs = nullptr;   // KP / 4 run byte offsets
  const int32_t* runs1 = nullptr;  // the same for the count box of a single voxel
  // bricks with fewer than sp rows (0: none) go to the encoder row by row, in
  // items of up to rs rows with a count box each
  int sp = 0, rs = 1;
  const uint16_t* wts = nullptr;   // KP slot weights (fp16)
  int K = 0, KP = 0, na = 4;
  int nbuf = 3;  // k-step slabs of the table buffered in LDS (2 to 4)
  int layout = 0;  // encoder wave layout (Tiling::layout)
  int rx = 0, ry = 0, rt = 0;
  Brick brick{32, 16, 8};
  int d = 0;
};

// Row formats the encoder writes (one row of 2D values per query voxel) and
// the perceptron forms that read them.
constexpr int kRowsF32 = 0;      // fp32 rows; perceptron on fp32 matrix cores
constexpr int kRowsBF16 = 1;     // bf16 rows; bf16 perceptron (FP16 form)
constexpr int kRowsSplit16 = 2;  // fp32 rows split into fp16 hi/lo in the perceptron (FP32 form)
constexpr int kRowsHiLo16 = 3;   // rows written as fp16 hi/lo pairs by the encoder: each group of
                                 // 4 consecutive elements is a 16-byte unit [hi x 4, lo x 4]
                                 // (FP32 form)
// The encoder runs the perceptron itself and writes one flow per row (no
// rows leave the chip): bf16 operands (FP16 form) or fp16 hi/lo operands
// (FP32 form).  Only with the one-wave-per-SIMD layout at D = 64 or 128.
constexpr int kFlowBF16 = 4;
constexpr int kFlowHiLo16 = 5;

struct MlpWeights {
  int hidden = 0;
  const float* W1 = nullptr;       // hidden x 2D fp32
  const uint16_t* W1b = nullptr;   // hidden x 2D bf16
  const uint16_t* W1h = nullptr;   // hidden x 2D fp16 hi of W1 * 2^s
  const uint16_t* W1l = nullptr;   // hidden x 2D fp16 lo of W1 * 2^s
  float unscale = 1.f;             // 2^-s
  const float* b1 = nullptr;
  const float* W2 = nullptr;       // 2 x hidden
  const float* b2 = nullptr;
  // W1 in the fused encoder's slab order (make_w1_fragments), or NULL
  const uint16_t* W1frag = nullptr;
};

// Widest perceptron hidden layer a context accepts.
constexpr int kMaxHidden = 512;

// W1 laid out as table slabs of the fused encoder (layout 2, WN = 1): slab s
// holds hidden tiles 2s and 2s + 1 (16 units each) for every 32-feature step
// kk of layer 1, fragment (t * 2 + tile, kk) as the MFMA A operand (64 lanes
// x 8 halves; t = 0 for the bf16 or fp16-hi term, 1 for the fp16-lo term of
// W1 * 2^shift).  Feature order within a step matches the encoder's
// accumulator layout (frequency tiles 2kk' and 2kk' + 1 of the real parts
// for kk < D / 32, of the imaginary parts above).
std::vector<uint16_t> make_w1_fragments(const float* W1, int hidden, int d, int na, int shift);
// Whether the encoder can run the perceptron itself for this tiling and width.
bool encode_fusable(const EncodeTables& et, int hidden);

int launch_prepare(const Batch& bt, const Workspace& w, const veckm_event* ev,
                   const int32_t* queries, const EncodeTables& et, bool pairs, void* stream);
int launch_paper_encode(const Batch& bt, const Workspace& w, const PaperTables& pt,
                        const Brick& brick, int rows, int num_cus, void* stream);
// (cos, sin) tables of the paper form, FP64 then rounded to fp32: time bins
// 0 .. max_bins - 1, columns 0 .. width - 1, rows 0 .. height - 1; each
// [coordinate][d][2].
void make_paper_tables(const double* A, int d, int width, int height, int max_bins,
                       std::vector<float>* ttab, std::vector<float>* xtab, std::vector<float>* ytab);
constexpr int kMaxPaperBins = 1024;  // bins per slice of the paper form
// rowcnt: when non-NULL, also the neighbour count of every row (int32 [U]).
int launch_encode(const Batch& bt, const Workspace& w, const EncodeTables& et, int rows,
                  int num_cus, void* stream, int32_t* rowcnt = nullptr,
                  const MlpWeights* mw = nullptr);
// Per-query outputs; use_qmap: rows from the query -> row map (paper form),
// else found from each query's voxel (`queries` as in the call, or NULL).
int launch_expand_emb(const Batch& bt, const Workspace& w, const int32_t* queries,
                      const Brick& b, bool use_qmap, int d, float* emb, void* stream);
int launch_mlp(const Workspace& w, const MlpWeights& mw, int d, int rows, int num_cus,
               void* stream);
// Whether the FP32-form perceptron runs on fp16 hi/lo operand pairs for
// this shape (W1 fragments fit in registers); else on the fp32 matrix cores.
bool mlp_rows_split(int d, int hidden);
int launch_expand_flow(const Batch& bt, const Workspace& w, const int32_t* queries,
                       const Brick& b, bool use_qmap, float* flow, void* stream);
// The flows of a dense bounded-window slice call (dense_batch) and the clear
// of its count and pair grids, in one launch (launch_expand_flow followed by
// launch_clear_events); VECKM_E_INVAL for a call that is not dense.
int launch_expand_flow_clear(const Batch& bt, const Workspace& w, const int32_t* queries,
                             const Brick& b, float* flow, void* stream);
// Per-query neighbour counts from the rows' counts (int32 [U], held in
// w.rowflow); -1 for an invalid query.
int launch_expand_count(const Batch& bt, const Workspace& w, const int32_t* queries,
                        const Brick& b, int32_t* counts, void* stream);
// Whether a bounded-window slice call is dense: its count and pair grids
// hold fewer than 30 entries per event.  Dense calls clear the two grids
// with one pass over them (about 1.5 GB/ms against about 50 M events/ms for
// per-event stores) and rank a brick per block; with 32 or more rows per
// brick on average they also take every non-empty brick whole in the
// encoder (no single rows).
inline bool dense_batch(const Batch& bt) { return bt.nvox + bt.npairs < 30 * (int64_t)bt.n; }
// After a bounded-window slice call whose launches all went through: the
// counts and pair entries of its events' voxels back to zero (the ranking
// kernel has cleared the row flags).
int launch_clear_events(const Batch& bt, const Workspace& w, void* stream);
// Dense fill of the count grid, the pair grid and `nlines` row flags (for
// workspaces whose contents are unknown).
int launch_clear_grids(const Batch& bt, const Workspace& w, int64_t nlines, void* stream);
// Copies the device error bits to `host` (pinned) and clears them, in stream order.
int launch_take_err(const Workspace& w, int32_t* host, void* stream);
// Sliding window: the bins [clear_b0, clear_b0 + clear_nb) enter the ring of
// T planes (bin b in plane (b - tref) mod T, clear_nb <= T); the events of
// bins [t0, t0 + nbins) among them are counted.  Then an encode of query
// events against the resident window (bt describes the window, tshift set).
int launch_window_push(const Workspace& w, const veckm_event* ev, int64_t n, int W, int H, int T,
                       int t0, int nbins, int tref, int64_t clear_b0, int clear_nb, void* stream);
int launch_window_prepare(const Batch& bt, const Workspace& w, const veckm_event* queries,
                          const EncodeTables& et, void* stream);

// ------------------------------------------------------------ perceptron training
// Device state of a trainer: parameters and gradients in the order W1
// [hidden][k2], b1, W2 [2][hidden], b2 (the gradient buffer has one more
// slot: the step's loss), Adam moments, layer-1 activations and their
// gradients for max_rows rows, and partial-sum buffers.
struct TrainState {
  int k2 = 0, hidden = 0;
  int64_t max_rows = 0;
  float* theta = nullptr;
  float* grad = nullptr;
  float* m1 = nullptr;
  float* m2 = nullptr;
  float* H = nullptr;
  float* dZ = nullptr;
  float* head_part = nullptr;  // head_blocks x (3 hidden + 3)
  float* w1_part = nullptr;    // max_splits x hidden x k2
  int head_blocks = 0, max_splits = 0;
};
// One step on m rows x [m][k2] (device) with targets y [m][2] (device):
// forward, loss, gradients, update (adam 0: gradient descent; 1: Adam with
// bias corrections c1, c2).  Leaves the loss in grad[n_params].
int launch_train_step(const TrainState& s, const float* x, const float* y, int64_t m, int adam,
                      float lr, float c1, float c2, void* stream);

// ------------------------------------------------- context hooks for the server
// What one call can hold, and what one slice needs of it.
struct Capacity {
  int64_t events = 0, voxels = 0, pairs = 0, bricks = 0, slices = 0;
};
Capacity ctx_capacity(const veckm_ctx* c);
// veckm_flow_batch with slice k's count grid at voxel at[2k] and its pair
// grid at entry at[2k + 1] of the context's grids (non-overlapping regions
// that stay put between calls: a server stream's resident grid).
int flow_batch_at(veckm_ctx* c, const veckm_slice* slices, int32_t count, const int64_t* at,
                  const veckm_event* events, float* flow, void* stream);
Capacity slice_need(const veckm_ctx* c, int W, int H, int T, int64_t n);
int ctx_take_err(veckm_ctx* c, int32_t* host, void* stream);
// VECKM_OK, VECKM_E_OVERFLOW or VECKM_E_RANGE for a set of device error bits.
int err_code(int32_t bits);

// ------------------------------------------------- allocation (with a test hook)
// Every device (hipMalloc) and pinned host (hipHostMalloc) allocation of the
// library goes through these.  With the environment variable
// VECKM_FAULT_ALLOC=n (n >= 1) the n-th allocation counted from the moment the
// variable took that value fails as if the device were out of memory, so the
// error paths that unwind a half-built object can be exercised; unset or 0:
// no fault.  Each returns true on success and leaves *p null on failure.
bool dev_malloc(void** p, size_t bytes);
bool pinned_malloc(void** p, size_t bytes);

}  // namespace veckm
