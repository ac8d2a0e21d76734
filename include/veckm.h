/*
 * veckm: per-event normal-flow estimation from event-camera slices on one
 * AMD Instinct MI355X (gfx950).
 *
 * The method (Yuan & Fermueller, "A Real-Time Event-Based Normal Flow
 * Estimator"): every event k of a slice is encoded by random Fourier
 * features of its centred spatio-temporal neighbourhood (Sec. 2.1, Eqn. 1;
 * Sec. 2.2.1, Eqn. 10), normalised by the neighbour count (Eqn. 17,
 * Algorithm 1 final step), and a two-layer perceptron maps the encoding to
 * a normal-flow vector (Sec. 2.1, Eqns. 5-6).  Because pixel coordinates
 * and time bins are integers, the window sum is a pooling over an integer
 * (x, y, t) grid (Sec. 2.2.2, Eqns. 14-17); this library evaluates it on
 * the GPU as a contraction of per-voxel event counts against a fixed table
 * of offset phases.
 *
 * Conventions shared by every entry point
 *   - Events are int32 tuples (x, y, t, p), 16 bytes each (veckm_event).
 *     x in [0, width), y in [0, height), t in [t0, t0 + nbins) counted in
 *     integer time bins, p in {-1, +1}.  Polarity is validated and not used
 *     by the encoder (the problem statement of Sec. 2.1 has none).
 *   - A is the frequency matrix: D rows, columns (x, y, t), FP64, applied to
 *     integer offsets.  Algorithm 1 draws X, Y, T ~ N(0, 25) and applies them
 *     to dx/delta-x, dy/delta-y, dt/delta-t: pass A[j] = (X_j/delta-x,
 *     Y_j/delta-y, T_j/delta-t).  The library does not draw it.
 *   - Encodings are float32 rows of 2D values, planar: Re emb[0..D-1], then
 *     Im emb[0..D-1].  Flows are float32 pairs (n_x, n_y).
 *   - Device pointers are hipMalloc'd (or torch CUDA tensor) memory on the
 *     context's device; host pointers are ordinary memory.  The caller owns
 *     every buffer it passes; the library owns what it allocates.
 *   - Compute calls only enqueue work on `stream` (a hipStream_t, NULL for
 *     the null stream) and return.  Results are valid once the stream has
 *     completed.  Input errors found on the device (an event out of range, a
 *     bad query index, a voxel overflow) are reported by veckm_status(); the
 *     outputs of that call are then undefined.
 *   - Return values: VECKM_OK (0) or a negative VECKM_E_* code.  Nothing
 *     throws across this boundary.  A context is not thread-safe.
 */
#ifndef VECKM_H
#define VECKM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VECKM_OK 0
#define VECKM_E_INVAL (-1)    /* NULL pointer, bad size, radius, D or precision */
#define VECKM_E_RANGE (-2)    /* event outside sensor/time window, |p| != 1, query
                                 index outside [0, n), n > max_events, nbins > max_bins */
#define VECKM_E_NOMEM (-3)    /* device or host allocation failed */
#define VECKM_E_BUDGET (-4)   /* request does not fit the memory budget */
#define VECKM_E_AGAIN (-5)    /* result not ready yet / queue full */
#define VECKM_E_HIP (-6)      /* a HIP runtime call failed */
#define VECKM_E_NODEVICE (-7) /* no usable gfx950 device */
#define VECKM_E_OVERFLOW (-8) /* more than VECKM_MAX_VOXEL_EVENTS events in one voxel */
#define VECKM_E_STATE (-9)    /* call needs state that is not set (e.g. no perceptron) */

/* Largest number of events one (x, y, t) voxel may hold in one call.  Counts
   enter the matrix cores as fp16 pair sums, exact up to 2048. */
#define VECKM_MAX_VOXEL_EVENTS 1024

/* Arithmetic of the encoder and perceptron. */
#define VECKM_FP32 0 /* offset phases carried as an fp16 hi/lo pair (22 significant
                        bits; counts are exact integers, products exact, all sums
                        in fp32); perceptron in fp32 on the matrix cores */
#define VECKM_FP16 1 /* offset phases rounded once to fp16, fp32 sums; encodings
                        handed to a bf16 x bf16 -> fp32 perceptron */

typedef struct veckm_event {
  int32_t x, y, t, p;
} veckm_event;

typedef struct veckm_params {
  int32_t width, height; /* sensor size W, H (Algorithm 1 inputs)                 */
  int32_t rx, ry;        /* spatial window radii delta-x, delta-y in pixels (Eqn. 1),
                            each in [0, 12]                                       */
  int32_t rt;            /* temporal window radius in bins, in [0, 6]: neighbours
                            also satisfy |t_k - t_q| <= rt.  -1: no temporal
                            bound, the neighbourhood of Eqn. 1 as written (the
                            whole slice in time), computed in the staged 2-D
                            form of Algorithm 1 (per-pixel temporal phase sums,
                            Eqns. 14-15; separable window sums, Eqns. 16-17), in
                            fp32 in both precisions, with max_bins <= 1024, no
                            per-voxel event limit, single-slice calls only      */
  int32_t d;             /* complex RFF dimension D: 16, 32, 48, 64, 128 or 256   */
  int32_t max_bins;      /* largest nbins accepted by a compute call               */
  int32_t precision;     /* VECKM_FP32 or VECKM_FP16                               */
  int64_t max_events;    /* largest n (and m) accepted by a compute call (all slices
                            of a batch together)                                   */
  const double* A;       /* host, d x 3 row-major, columns (x, y, t); copied       */
  int32_t max_slices;    /* largest number of slices in one batch call; 0 means 1  */
  int64_t max_voxels;    /* largest total grid volume (sum of W*H*nbins over the
                            slices) of one call; 0 means
                            width*height*max_bins*max_slices                       */
} veckm_params;

/* One slice of a batch call.  Slices are independent (every neighbourhood lies
   inside its slice, Sec. 2.1) and their events lie back to back in one array:
   slice k owns events[offset_k, offset_k + n_k) with offset_0 = 0 and
   offset_{k+1} = offset_k + n_k. */
typedef struct veckm_slice {
  int32_t width, height; /* sensor of the slice, at most the context's width, height */
  int32_t t0, nbins;     /* time window [t0, t0 + nbins), 1 <= nbins <= max_bins       */
  int64_t offset, n;     /* its events                                                 */
} veckm_slice;

typedef struct veckm_ctx veckm_ctx;

/* ---- host-only helpers (no device needed) ------------------------------ */

/* Validates a parameter block without touching the GPU.  Returns VECKM_OK or
   VECKM_E_INVAL. */
int veckm_params_check(const veckm_params* params);

/* Device bytes a context created from `params` allocates (workspaces sized
   for max_events and width x height x max_bins voxels, the phase table and a
   perceptron of `hidden` units).  Negative VECKM_E_* on bad parameters. */
int64_t veckm_workspace_bytes(const veckm_params* params, int32_t hidden);

/* The precomputed offset-phase table of Algorithm 1 (the "precomputed"
   spatial factor, here extended to (dx, dy, dt)), as the library builds it
   on the host in FP64 and rounds it for the matrix cores.  The window
   {|dx|<=rx, |dy|<=ry, |dt|<=rt} is reduced by conjugate symmetry
   (e^{-i theta} = conj e^{i theta}) to its centre plus the half with
   (dt, dy, dx) lexicographically positive: *k_count = ((2rx+1)(2ry+1)(2rt+1)
   + 1) / 2 offsets.  If `offsets` is non-NULL it receives k_count x 3 int32
   (dx, dy, dt), entry 0 being the centre.  If `phase_bits` is non-NULL it
   receives k_count x d x 4 uint16 fp16 bit patterns (cos hi, cos lo, sin hi,
   sin lo) of theta = A[j] . (dx, dy, dt), with hi = fp16(cos) rounded to
   nearest even and lo = fp16(cos - hi); the centre entry stores cos = 1/2
   (it is met twice, as +o and -o).  Returns VECKM_OK or VECKM_E_INVAL (also
   for rt = -1, whose form has no such table). */
int veckm_offset_table(const veckm_params* params, int32_t* k_count, int32_t* offsets,
                       uint16_t* phase_bits);

const char* veckm_strerror(int code);

/* ---- context ------------------------------------------------------------ */

/* Creates a context on the current HIP device: copies A, builds the phase
   table (FP64 on the host) and allocates every workspace up front, so that
   compute calls allocate nothing.  Returns VECKM_E_NODEVICE when no gfx950
   device is present, VECKM_E_NOMEM when the workspaces do not fit. */
int veckm_create(const veckm_params* params, veckm_ctx** out);

void veckm_destroy(veckm_ctx* ctx);

/* Sets the two-layer perceptron (Sec. 2.1, Eqns. 5-6):
     flow = W2 * relu(W1 * emb + b1) + b2
   W1: hidden x 2D row-major (the [Re | Im] input order above), b1: hidden,
   W2: 2 x hidden row-major, b2: 2.  Host float32, copied (and, for
   VECKM_FP16, also rounded to bf16).  hidden must be a multiple of 64, at
   most 512.  Synchronous.  Returns VECKM_E_INVAL on bad shapes. */
int veckm_set_mlp(veckm_ctx* ctx, int32_t hidden, const float* W1, const float* b1,
                  const float* W2, const float* b2);

/* Encodes the queried events of one slice (Algorithm 1 with the bounded
   window; Eqn. 10 normalised by the Eqn. 17 count).
     events  device, n events; every event must satisfy the conventions above
             with the given t0 and nbins (1 <= nbins <= max_bins).
     queries device, m event indices in [0, n), or NULL for all events (m must
             then equal n).  Duplicates are allowed.
     emb     device, m x 2D float32, row i is the encoding of event queries[i].
   Returns VECKM_E_RANGE if n, m or nbins exceed the context's limits. */
int veckm_encode(veckm_ctx* ctx, const veckm_event* events, int64_t n, int32_t t0,
                 int32_t nbins, const int32_t* queries, int64_t m, float* emb,
                 void* stream);

/* As veckm_encode, followed by the perceptron: flow is device m x 2 float32.
   Returns VECKM_E_STATE if no perceptron was set. */
int veckm_flow(veckm_ctx* ctx, const veckm_event* events, int64_t n, int32_t t0,
               int32_t nbins, const int32_t* queries, int64_t m, float* flow,
               void* stream);

/* The neighbour count of each queried event, as the encoder computes it for
   its normalisation (Eqn. 17; Algorithm 1 final step): the number of events
   k of the slice with |x_k - x_q| <= rx, |y_k - y_q| <= ry and
   |t_k - t_q| <= rt, the query itself included.  Same arguments, limits and
   errors as veckm_encode; counts is device m x int32 (-1 for a query whose
   event broke the conventions, reported by veckm_status).  The count is
   exact (integer pair sums summed exactly in fp32).  Returns VECKM_E_INVAL
   for a window or rt = -1 context. */
int veckm_count(veckm_ctx* ctx, const veckm_event* events, int64_t n, int32_t t0,
                int32_t nbins, const int32_t* queries, int64_t m, int32_t* counts,
                void* stream);

/* Batch forms: one launch sequence for `count` slices (1 <= count <=
   max_slices).  Every event of every slice is queried; outputs follow the
   event order (emb: device, total n x 2D float32; flow: device, total n x 2
   float32).  The result for each slice is bit-identical to encoding that
   slice alone.  `slices` is host memory and is copied before return.
   Returns VECKM_E_INVAL for non-contiguous slices or bad sizes, or for a
   context with rt = -1, VECKM_E_RANGE when the batch exceeds max_events,
   max_voxels or the sensor / max_bins limits. */
int veckm_encode_batch(veckm_ctx* ctx, const veckm_slice* slices, int32_t count,
                       const veckm_event* events, float* emb, void* stream);
int veckm_flow_batch(veckm_ctx* ctx, const veckm_slice* slices, int32_t count,
                     const veckm_event* events, float* flow, void* stream);

/* ---- allocation-free flow ------------------------------------------------
   For callers that cannot allocate device memory while they run (code under
   HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
   veckm_flow_noalloc computes what veckm_flow computes with queries = NULL
   (every event queried; bit-identical results), but every per-call
   workspace (count and pair grids, row flags, ranks, brick and row lists,
   rows, row flows) lives
   in one static device array of VECKM_NOALLOC_SCRATCH_BYTES that the library
   holds on each GPU it runs on until the process ends.  Only the context's
   read-only state is used (phase table, tiling, perceptron weights) and its
   device error flag (veckm_status reports input errors as usual); the
   context's own workspaces are not touched.  The call calls no hipMalloc,
   hipFree or allocating library routine (the device address of the array is
   looked up once per device, on the first call there).
     Limits: those of veckm_flow on this context, and the call's workspaces
     must fit in the array: about 16 W H nbins + (20 + 8 D) n bytes (a
     346 x 260 sensor with 25 bins and 20k events at D = 64 needs 47 MB);
     beyond that it returns VECKM_E_BUDGET and launches nothing.
     Sharing: every call on one GPU uses the same array and finds it as the
     last call left it (the count and pair grids and the row flags are
     cleared at the start of each call).
     Calls that overlap on one GPU, on any streams or contexts or threads,
     race and give undefined results: serialise them (one stream, or
     synchronise between calls).
   Returns VECKM_E_INVAL for a window or rt = -1 context, VECKM_E_STATE
   without a perceptron, VECKM_E_RANGE as veckm_flow, VECKM_E_BUDGET as
   above, VECKM_E_HIP if the array cannot be located. */
#define VECKM_NOALLOC_SCRATCH_BYTES (64ll << 20)
int veckm_flow_noalloc(veckm_ctx* ctx, const veckm_event* events, int64_t n, int32_t t0,
                       int32_t nbins, float* flow, void* stream);

/* ---- launch graphs (batch forms) ---------------------------------------
   A batch layout that repeats (the same slices, event buffer and output
   buffer on every call, as in a serving loop) can be captured once as a HIP
   graph and replayed with one launch, instead of a dozen kernel launches per
   call (launch overhead dominates small slices).  veckm_graph_create
   validates like veckm_flow_batch (flow != 0) or veckm_encode_batch
   (flow == 0), copies the slice table into device memory the graph owns,
   and captures the launch sequence for exactly these `slices`, `events` and
   `out`.  veckm_graph_launch replays it on `stream`: it reads what `events`
   holds at that time (the events may change between launches, the slice
   layout may not: every event must still satisfy its slice's window and
   sensor) and writes `out` as the batch call would, bit for bit.
     ctx      the context whose workspaces the graph uses.  Replays and other
              calls on the same context must not overlap on the device (issue
              them on one stream, or synchronise); destroy a context's graphs
              before the context.
     out      device, total n x 2 (flow) or total n x 2D (encodings) float32.
     *graph   receives the graph; release it with veckm_graph_destroy.
   Returns the batch call's errors (VECKM_E_INVAL, VECKM_E_RANGE,
   VECKM_E_STATE), VECKM_E_NOMEM, or VECKM_E_HIP if capture fails; no
   kernel runs at creation.  Device-side input errors of a replay are
   reported by veckm_status. */
typedef struct veckm_graph veckm_graph;
int veckm_graph_create(veckm_ctx* ctx, const veckm_slice* slices, int32_t count,
                       const veckm_event* events, float* out, int32_t flow,
                       veckm_graph** graph);
int veckm_graph_launch(veckm_graph* graph, void* stream);
void veckm_graph_destroy(veckm_graph* graph);

/* ---- encoder tilings and the tuner --------------------------------------
   The encoder cuts every slice into bricks of voxels and streams the phase
   table through LDS a few slabs deep (the count box of a brick and the slabs
   share the 160 KB of LDS).  A context offers a small set of tilings (brick
   shape x buffered slabs x wave layout): the largest brick that fits beside
   two slabs (as many slabs as fit), larger bricks with fewer slabs, which
   pay off where bricks hold few query voxels (sparse slices), and each of
   those with other wave layouts.  At D = 64 and 128 index 0 is a layout
   whose encoder also runs the perceptron (flow calls keep every encoding on
   the chip): the default brick in wave layout 4; elsewhere index 0 is the
   default brick in layout 0.  Encodings do not depend on the tiling (bit-identical);
   flows are bit-identical among layouts 0 and 1 and among layouts 2 to 4,
   and agree between the two groups to fp32 rounding (the perceptron's sums
   run in another order).
     veckm_tiling_count     number of tilings (>= 1), or VECKM_E_INVAL
     veckm_tiling_selected  index in use, or VECKM_E_INVAL
     veckm_tiling_info      info[0..4] = brick x, y, t sides, slabs and wave
                            layout (0: 16 waves of 2 row tiles; 1: 8 waves
                            of 4 row tiles, each table fragment feeding
                            twice the products; 2: 4 waves of 4 row tiles,
                            3: 8 waves of 2 row tiles and 4: 16 waves of
                            one row tile (D <= 128), each wave over every
                            frequency of its rows, loads pipelined within
                            the wave, one slab in flight, the perceptron
                            inside the encoder at D = 64 and 128)
                            of tiling `index` (host int32[5])
     veckm_tiling_select    use tiling `index` from the next call on
     veckm_tune             times every tiling on the given batch (as for
                            veckm_flow_batch when a perceptron is set, else
                            veckm_encode_batch: the front end, the encoder
                            and the perceptron, one untimed and `reps` timed
                            runs each, 1 <= reps
                            <= 100, HIP events on `stream`), selects the
                            fastest for the calls that follow and writes its
                            index to *chosen (may be NULL).  Synchronises
                            `stream`; writes no caller memory besides
                            *chosen.  Errors as veckm_encode_batch; VECKM_E_INVAL
                            for rt = -1 or sliding-window contexts (one
                            tiling).  Must not overlap other calls on the
                            context. */
int veckm_tiling_count(const veckm_ctx* ctx);
int veckm_tiling_selected(const veckm_ctx* ctx);
int veckm_tiling_info(const veckm_ctx* ctx, int32_t index, int32_t* info);
int veckm_tiling_select(veckm_ctx* ctx, int32_t index);
int veckm_tune(veckm_ctx* ctx, const veckm_slice* slices, int32_t count,
               const veckm_event* events, int32_t reps, void* stream, int32_t* chosen);

/* Waits for `stream`, then reports (and clears) the device-side input error
   of the calls enqueued so far: VECKM_OK, VECKM_E_RANGE or
   VECKM_E_OVERFLOW. */
int veckm_status(veckm_ctx* ctx, void* stream);

/* ---- sliding window (streaming encoder) --------------------------------- */

/* The encoder as a general-purpose per-event feature over a live event
   stream (Sec. 1: the local event encoder is offered for other event-based
   tasks; Eqn. 10 over the bounded window of Eqn. 1 with the context's rt).  A
   window context keeps the integer event counts of the last Tw =
   params->max_bins time bins of one sensor resident on the device as a ring
   over time: pushing new bins retires the oldest ones, and query events are
   encoded against every event resident in the window.  Encoding a window is
   bit-identical to veckm_encode of a slice holding the window's events with
   t0 = end - Tw and nbins = Tw.

   veckm_window_create: as veckm_create (rt >= 0; max_slices 0 or 1); the
   window starts empty.  Destroy with veckm_destroy; veckm_set_mlp and
   veckm_status apply; veckm_encode / veckm_flow and the batch calls return
   VECKM_E_INVAL on a window context. */
int veckm_window_create(const veckm_params* params, veckm_ctx** out);

/* Appends the events of bins [t0, t0 + nbins) (device, n events, every t in
   that range, 1 <= nbins <= Tw, n <= max_events).  The first push fixes the
   stream's origin; later pushes need t0 >= the previous end (skipped bins
   are empty).  The window becomes [t0 + nbins - Tw, t0 + nbins): older bins
   are retired.  Events outside the bins or the sensor are reported by
   veckm_status as VECKM_E_RANGE (and not counted), voxels over
   VECKM_MAX_VOXEL_EVENTS as VECKM_E_OVERFLOW.  Returns VECKM_E_INVAL for a
   t0 before the previous end, VECKM_E_RANGE for n or nbins out of range. */
int veckm_window_push(veckm_ctx* ctx, const veckm_event* events, int64_t n, int32_t t0,
                      int32_t nbins, void* stream);

/* Encodes m query events (device, each inside the sensor and the current
   window, else VECKM_E_RANGE via veckm_status) against the resident window:
   emb (device, m x 2D float32, planar [Re | Im]) as veckm_encode.  A query
   usually is a pushed event (then it counts itself); a query with no event in
   its neighbourhood encodes to zeros.  VECKM_E_STATE before the first push.
   veckm_window_flow adds the perceptron (flow: device, m x 2 float32;
   VECKM_E_STATE if none was set). */
int veckm_window_encode(veckm_ctx* ctx, const veckm_event* queries, int64_t m, float* emb,
                        void* stream);
int veckm_window_flow(veckm_ctx* ctx, const veckm_event* queries, int64_t m, float* flow,
                      void* stream);

/* ---- training the perceptron --------------------------------------------- */

/* Trains the two-layer perceptron (Sec. 2.1, Eqns. 5-6) on encodings with
   known normal flows.  The paper leaves its loss and sampling to its
   predecessor; the loss here is the mean over the rows of the squared error
   of the predicted 2-vector, L = (1/m) sum_r ||flow_r - target_r||^2, with
   plain gradient descent or Adam (beta1 0.9, beta2 0.999, eps 1e-8, bias
   corrected).  All arithmetic is fp32 on the device; a step is deterministic.
   The trainer keeps its own copy of the weights: read them back with
   veckm_trainer_get and hand them to veckm_set_mlp to use them. */
typedef struct veckm_trainer veckm_trainer;

/* Creates a trainer on the current HIP device for encodings of dimension
   2d and `hidden` units (a multiple of 64, at most 512), initialised with the
   host weights (layouts as veckm_set_mlp), for steps of up to max_rows rows.
   Allocates everything up front.  VECKM_E_INVAL on bad sizes, VECKM_E_NOMEM,
   VECKM_E_NODEVICE. */
int veckm_trainer_create(int32_t d, int32_t hidden, int64_t max_rows, const float* W1,
                         const float* b1, const float* W2, const float* b2, veckm_trainer** out);
void veckm_trainer_destroy(veckm_trainer* tr);

/* One step on m rows: emb device [m][2d] float32 (as veckm_encode writes
   them), target device [m][2] float32.  optimizer 0: w -= lr g; 1: Adam.
   loss: device float receiving this step's loss (before the update), or
   NULL.  Asynchronous on `stream`.  VECKM_E_RANGE if m exceeds max_rows. */
int veckm_trainer_step(veckm_trainer* tr, const float* emb, const float* target, int64_t m,
                       int32_t optimizer, float lr, float* loss, void* stream);

/* Copies the current weights to host arrays (layouts as veckm_set_mlp);
   waits for the device. */
int veckm_trainer_get(veckm_trainer* tr, float* W1, float* b1, float* W2, float* b2);

/* ---- measurement ---------------------------------------------------------- */

/* Stages of one compute call, in launch order. */
#define VECKM_STAGE_PREPARE 0 /* validate + histogram events, rank query voxels, work list */
#define VECKM_STAGE_ENCODE 1  /* the count x offset-phase contraction (one kernel; with the
                                 perceptron inside it in the fused tilings)                 */
#define VECKM_STAGE_MLP 2     /* the two-layer perceptron as its own kernel (none if fused) */
#define VECKM_STAGE_EXPAND 3  /* per-voxel rows copied out per query, grids back to zero   */
#define VECKM_NUM_STAGES 4

/* Turns per-stage timing on (1) or off (0).  While on, every compute call
   records a HIP event before and after each stage on the call's stream (no
   host synchronisation).  Events are created here, not in the compute calls.
   Returns VECKM_OK, VECKM_E_INVAL or VECKM_E_HIP. */
int veckm_profile_enable(veckm_ctx* ctx, int32_t enable);

/* Waits for the recorded events and returns, per stage, the summed device
   milliseconds (ms[s]) and the number of timed launches (count[s]) since the
   last read; then clears them.  Arrays hold `nstages` entries (at most
   VECKM_NUM_STAGES are written).  Returns VECKM_OK, VECKM_E_INVAL or
   VECKM_E_HIP. */
int veckm_profile_read(veckm_ctx* ctx, double* ms, int64_t* count, int32_t nstages);

/* Waits for `stream` and returns the number of encoder rows (distinct query
   voxels) of the last compute call enqueued on this context. */
int veckm_last_rows(veckm_ctx* ctx, void* stream, int64_t* rows);

/* ---- serving: asynchronous event streams, continuously batched -------------

   A server owns one context (sized by `params`: the largest sensor, bins and
   batch it will run), three HIP streams of its own (events in, kernels,
   flows out) and two native threads: a launcher that packs waiting slices,
   at most one per stream, into one batch call (veckm_flow_batch) whenever
   one of two device lanes is free, and a completer that waits for each
   batch, stamps its slices' completion time and wakes the pollers.  Each
   lane has its own device event and flow buffers, so the host-to-device copy
   of one batch overlaps the kernels of the other.  Slices that arrive while
   a batch runs go into the next one, so work from different streams
   overlaps on the device; a slice's result does not depend on which other
   slices share its batch (bit-identical to veckm_flow on that slice alone).

   Resident grids and admission by HBM budget: every open stream keeps its
   own count and pair grids (W*H*max_bins voxels, 8-9 bytes each) resident on
   the device for as long as it is open; each of its slices is counted into
   that region and leaves it clean for the next.  The regions come from a
   grid arena of params->max_voxels voxels (0: room for max_streams streams
   at the largest sensor and bins).  The server's device memory (the arena,
   the batch workspaces, phase table, perceptron, two lanes of event and flow
   buffers) must fit in hbm_budget_bytes at create time, and
   veckm_stream_open returns VECKM_E_BUDGET when the stream's grids do not
   fit in what is left of the arena, or when the open streams' events would
   exceed one batch (so one waiting slice of every admitted stream always
   fits into a batch).  Batches take waiting slices in submission order
   while they fit.  Closing a stream returns its grids to the arena.

   Threading: veckm_submit, veckm_poll, veckm_stream_open/close and
   veckm_server_stats(_sensor) may be called from any threads concurrently.
   veckm_server_destroy must not race with other calls on the server. */
typedef struct veckm_server veckm_server;

/* Creates a server on the current HIP device.  params->max_events,
   max_voxels and max_slices bound one batch (0 -> derived as for
   veckm_create); `max_streams` streams may be open at once, each with up to
   `depth` (1..16) submitted slices not yet polled.  Returns VECKM_E_BUDGET if
   the server's device memory exceeds hbm_budget_bytes (a positive number),
   VECKM_E_INVAL for rt = -1 (batches need the bounded window), plus the
   veckm_create errors. */
int veckm_server_create(const veckm_params* params, int64_t hbm_budget_bytes, int32_t max_streams,
                        int32_t depth, veckm_server** out);

/* Stops the threads after the batches on the device complete, then frees
   everything (results not yet polled are dropped). */
void veckm_server_destroy(veckm_server* server);

/* The perceptron, as veckm_set_mlp; call before the first submit. */
int veckm_server_set_mlp(veckm_server* server, int32_t hidden, const float* W1, const float* b1,
                         const float* W2, const float* b2);

/* Opens a stream for slices of a width x height sensor with at most
   max_bins bins and max_events events each.  *sid receives its id.
   VECKM_E_RANGE if the sensor, bins or events exceed the server's params,
   VECKM_E_BUDGET if the open streams' reservations would exceed the batch
   capacity, VECKM_E_AGAIN if max_streams are open. */
int veckm_stream_open(veckm_server* server, int32_t width, int32_t height, int32_t max_bins,
                      int64_t max_events, int32_t* sid);

/* Waits until the stream's submitted slices are complete, drops results not
   yet polled and releases its reservation. */
int veckm_stream_close(veckm_server* server, int32_t sid);

/* Submits one slice of stream `sid`: n events (host memory, copied before
   return, so the caller may reuse the buffer), time window [t0, t0 + nbins).
   Non-blocking.  *ticket identifies the slice for veckm_poll.  Every event is
   queried.  VECKM_E_AGAIN if the stream already has `depth` slices not yet
   polled; VECKM_E_RANGE if n or nbins exceed the stream's limits. */
int veckm_submit(veckm_server* server, int32_t sid, const veckm_event* events, int64_t n,
                 int32_t t0, int32_t nbins, uint64_t* ticket);

/* Waits up to timeout_us microseconds (< 0: without limit, 0: do not wait)
   for the slice `ticket`; when it is complete, copies its n x 2 float32 flows
   to `flows` (host memory, may be NULL to discard), forgets the ticket and
   returns the slice's status: VECKM_OK, or VECKM_E_RANGE / VECKM_E_OVERFLOW
   for a slice whose events broke the conventions (found on the device; the
   other slices of its batch are unaffected).  VECKM_E_AGAIN if still running,
   VECKM_E_INVAL for an unknown ticket. */
int veckm_poll(veckm_server* server, uint64_t ticket, float* flows, int32_t timeout_us);

/* Latency and throughput of the slices completed since the last reset: a
   slice's latency is the wall-clock time from its veckm_submit call to the
   completer observing its batch done (host copy of events, device work and
   the copy of flows back to host included). */
typedef struct veckm_serving_stats {
  int64_t slices;      /* completed slices                                    */
  int64_t flows;       /* their events (one flow per event)                   */
  int64_t batches;     /* batch calls launched                                */
  double p50_ms, p99_ms, max_ms;   /* slice latency percentiles               */
  double busy_s;       /* wall-clock time from the first submit to the last completion */
} veckm_serving_stats;

int veckm_server_stats(veckm_server* server, veckm_serving_stats* out, int32_t reset);

/* As veckm_server_stats (without a reset), with slices, p50, p99 and max
   over the slices of streams whose sensor is width x height only (a sensor
   class); flows, batches and busy_s are the server's totals.
   VECKM_E_INVAL for a non-positive size. */
int veckm_server_stats_sensor(veckm_server* server, int32_t width, int32_t height,
                              veckm_serving_stats* out);

#ifdef __cplusplus
}
#endif

#endif /* VECKM_H */
