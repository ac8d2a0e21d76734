// Front end of the encoder: validate and bin events into an integer
// (x, y, t) count grid per slice, rank the voxels that carry queries, and
// map queries to their voxel's row; plus the back-end expansion of
// per-voxel rows to per-query outputs.
//
// All events that share a voxel have the same offset to every neighbour, so
// the scatter of Algorithm 1 (PixelEmbed/PixelCount, Eqns. 14-15) reduces
// to an exact integer histogram; the phases are applied afterwards by the
// encoder contraction.  All queries that share a voxel get the same encoding
// (Sec. 2.1: the encoding depends on the event's position and time only), so
// the encoder computes one row per distinct query voxel and the rows are
// copied out per query.
//
// A call covers one slice or a batch of slices.  Slices are independent
// (neighbourhoods never leave a slice); each has its own sensor size, time
// window, event range and region of the shared grids, and the bricks of all
// slices form one work list.
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include "slices.h"
#include "veckm_internal.h"

namespace veckm {

__global__ void k_fill_i32(int32_t* __restrict__ p, int64_t n, int32_t v) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

// The slice of event i, for blocks whose threads take consecutive events
// i = blockIdx.x * blockDim.x + threadIdx.x: two threads find the slices of
// the block's first and last event, and the rest search only between them
// (almost always one slice).  Every thread of the block must call it.
__device__ inline SliceDesc slice_by_event_block(const Batch& bt, int i) {
  if (bt.nslices == 1) return bt.s0;
  __shared__ int ends[2];
  const int first = blockIdx.x * blockDim.x;
  const int last = min(first + (int)blockDim.x, bt.n) - 1;
  if (threadIdx.x < 2) {
    const int e = threadIdx.x ? last : first;
    int lo = 0, hi = bt.nslices - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (bt.table[mid].ev_off <= e) lo = mid; else hi = mid - 1;
    }
    ends[threadIdx.x] = lo;
  }
  __syncthreads();
  int lo = ends[0], hi = ends[1];
  const int e = min(i, bt.n - 1);
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (bt.table[mid].ev_off <= e) lo = mid; else hi = mid - 1;
  }
  return bt.table[lo];
}

// One thread per event: validate against its slice, histogram (ADD), remember
// the slice-local voxel, and mark it as a query voxel when qmark is given
// (a sliding window's query events).  With `lines` (bounded-window slice
// calls) the event also flags its brick x row: lines[gb * by * bt + lt * by +
// ly] = 1 for brick gb and brick-local row (ly, lt), so that ranking visits
// only rows that hold events (plain byte stores: every writer stores the
// same value).  Voxels over VECKM_MAX_VOXEL_EVENTS are caught where the pair
// grid is built (k_rank_lines, k_rank, or k_pairs for a sliding window),
// which reads every count once.
template <bool ADD>
__global__ void k_scatter(const int4* __restrict__ ev, Batch bt, int32_t* __restrict__ count,
                          int32_t* __restrict__ vox, int32_t* __restrict__ err,
                          uint8_t* __restrict__ qmark, Brick b, uint8_t* __restrict__ lines) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (blockIdx.x * blockDim.x >= bt.n) return;  // (whole block; launches never do this)
  const SliceDesc s = slice_by_event_block(bt, i);
  if (i >= bt.n) return;
  const int4 e = ev[i];
  const int64_t dt = (int64_t)e.z - (int64_t)s.t0;
  const bool ok = e.x >= 0 && e.x < s.W && e.y >= 0 && e.y < s.H && dt >= 0 && dt < s.T &&
                  (e.w == 1 || e.w == -1);
  if (!ok) {
    atomicOr(err, kErrRange);
    vox[i] = -1;
    return;
  }
  const int v = ((int)dt * s.H + e.y) * s.W + e.x;
  if (ADD) atomicAdd(&count[s.grid_off + v], 1);  // result unused: a no-return atomic
  if (qmark) qmark[s.grid_off + v] = 1;
  if (lines) {
    const int sx = __builtin_ctz(b.bx), sy = __builtin_ctz(b.by), st = __builtin_ctz(b.bt);
    const int gb = s.brick_off + (((int)dt >> st) * s.nby + (e.y >> sy)) * s.nbx + (e.x >> sx);
    lines[(int64_t)gb * (b.by * b.bt) + ((((int)dt & (b.bt - 1)) << sy) | (e.y & (b.by - 1)))] = 1;
  }
  vox[i] = v;
}

// A sliding window's new bins: validate each event against [t0, t0 + nbins)
// and the sensor, and count it in ring plane (t - tref) mod T.
__global__ void k_push(const int4* __restrict__ ev, int n, int W, int H, int T, int t0, int nbins,
                       int tref, int32_t* __restrict__ count, int32_t* __restrict__ err) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int4 e = ev[i];
  const int64_t dt = (int64_t)e.z - (int64_t)t0;
  const bool ok = e.x >= 0 && e.x < W && e.y >= 0 && e.y < H && dt >= 0 && dt < nbins &&
                  (e.w == 1 || e.w == -1);
  if (!ok) {
    atomicOr(err, kErrRange);
    return;
  }
  const int plane = (int)(((int64_t)e.z - tref) % T);
  atomicAdd(&count[((int64_t)plane * H + e.y) * W + e.x], 1);
}

// The encoder's view of the counts: per slice, rows of W + 1 dwords; entry
// x + 1 of a row holds the fp16 counts of voxels x and x + 1 of that x row
// (0 outside [0, W)), for x in [-1, W).  Any 4 consecutive voxels of a row
// then sit in two aligned dwords, including a run that starts at x = -1.
// Exact: counts are at most VECKM_MAX_VOXEL_EVENTS.
// The pair grid of a sliding window's new planes (slice calls build it in
// k_rank).  One wavefront per x row; blockIdx.y picks the slice, the blocks
// of a slice stride over its H T rows.
__global__ __launch_bounds__(256) void k_pairs(Batch bt, const int32_t* __restrict__ count,
                                               uint32_t* __restrict__ pairs,
                                               int32_t* __restrict__ err) {
  const SliceDesc s = bt.nslices > 1 ? bt.table[blockIdx.y] : bt.s0;
  const int lane = threadIdx.x & 63;
  const int W = s.W, nrows = s.H * s.T;
  bool bad = false;
  for (int row = blockIdx.x * 4 + (threadIdx.x >> 6); row < nrows; row += gridDim.x * 4) {
    const int32_t* c = count + s.grid_off + (int64_t)row * W;
    uint32_t* p = pairs + s.pair_off + (int64_t)row * (W + 1);
    for (int e0 = 0; e0 <= W; e0 += 256) {
      // entries e0 + 64 u + lane (entry e: voxels e - 1 and e).  The loads
      // are unconditional (addresses clamped into the row, values masked
      // afterwards), so all eight are in flight before the first wait.
      int lo[4], hi[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = e0 + 64 * u + lane;
        lo[u] = c[min(max(e - 1, 0), W - 1)];
        hi[u] = c[min(e, W - 1)];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = e0 + 64 * u + lane;
        lo[u] = e >= 1 && e <= W ? lo[u] : 0;
        hi[u] = e < W ? hi[u] : 0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = e0 + 64 * u + lane;
        bad |= hi[u] > VECKM_MAX_VOXEL_EVENTS;
        if (e <= W)
          p[e] = (uint32_t)__half_as_ushort(__float2half((float)lo[u])) |
                 ((uint32_t)__half_as_ushort(__float2half((float)hi[u])) << 16);
      }
    }
  }
  if (bad) atomicOr(err, kErrOverflow);
}

// Query subsets (one slice): mark the voxels that carry at least one query.
__global__ void k_mark(const int32_t* __restrict__ queries, Batch bt,
                       const int32_t* __restrict__ vox, uint8_t* __restrict__ qmark,
                       int32_t* __restrict__ err) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= bt.m) return;
  const int q = queries ? queries[i] : i;
  if (q < 0 || q >= bt.n) {
    atomicOr(err, kErrQuery);
    return;
  }
  const int v = vox[q];
  if (v >= 0) qmark[bt.s0.grid_off + v] = 1;
}

// One block per brick: number the brick's query voxels in (t, y, x) order
// (the paper form and sliding windows; bounded-window slice calls use
// k_rank_lines).  rank[v] gets the brick-local number, ulist[brick][number]
// the brick-local voxel index, brick_nq[brick] the total.  Wave w of the 4
// takes the w-th quarter of the brick in voxel order: a first pass keeps its
// ballots, one barrier gives every wave its offset, a second pass writes the
// numbers.  Brick sides are powers of two and a brick holds at most 256 kIt
// voxels.
template <bool ALL, int kIt>
__global__ __launch_bounds__(256) void k_rank(Batch bt, Brick b, const int32_t* __restrict__ count,
                                              uint8_t* __restrict__ qmark,
                                              int32_t* __restrict__ rank,
                                              int32_t* __restrict__ ulist,
                                              int32_t* __restrict__ brick_nq) {
  __shared__ int wave_tot[4];
  const int gb = blockIdx.x;
  const SliceDesc s = slice_by_brick(bt, gb);
  const int lb = gb - s.brick_off;
  const int bxi = lb % s.nbx, byi = (lb / s.nbx) % s.nby, bti = lb / (s.nbx * s.nby);
  const int BV = b.bx * b.by * b.bt;
  const int sx = __builtin_ctz(b.bx), sy = __builtin_ctz(b.by);
  const int per = (BV + 255) >> 8;  // iterations per wave
  const int lane = threadIdx.x & 63;
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int x0 = bxi * b.bx, y0 = byi * b.by, t0 = bti * b.bt;
  // voxel (grid index) of brick-local li, or -1 outside the slice (no
  // branches, so that the loads below are not serialised)
  auto voxel = [&](int li) -> int64_t {
    const int x = x0 + (li & (b.bx - 1)), y = y0 + ((li >> sx) & (b.by - 1)),
              t = t0 + (li >> (sx + sy));
    const bool in = li < BV && x < s.W && y < s.H && t < s.T;
    return in ? s.grid_off + ((int64_t)t * s.H + y) * s.W + x : (int64_t)-1;
  };
  // all loads first (unconditional: a voxel outside the slice reads the
  // slice's first voxel and is masked), then the ballots
  bool flag[kIt];
#pragma unroll
  for (int k = 0; k < kIt; ++k) {
    const int64_t v = k < per ? voxel((wid * per + k) * 64 + lane) : (int64_t)-1;
    const int64_t a = v >= 0 ? v : s.grid_off;
    const bool f = ALL ? count[a] > 0 : (qmark[a] != 0);
    flag[k] = v >= 0 && f;
  }
  unsigned long long bal[kIt];
  int tot = 0;
#pragma unroll
  for (int k = 0; k < kIt; ++k) {
    bal[k] = k < per ? __ballot(flag[k]) : 0ull;
    tot += __popcll(bal[k]);
  }
  if (lane == 0) wave_tot[wid] = tot;
  __syncthreads();
  int base = 0;
  for (int w = 0; w < wid; ++w) base += wave_tot[w];
  if (threadIdx.x == 0) brick_nq[gb] = wave_tot[0] + wave_tot[1] + wave_tot[2] + wave_tot[3];
  const unsigned long long below = (1ull << lane) - 1ull;
#pragma unroll
  for (int k = 0; k < kIt; ++k) {
    if (k < per) {
      if ((bal[k] >> lane) & 1ull) {
        const int li = (wid * per + k) * 64 + lane;
        const int r = base + __popcll(bal[k] & below);
        const int64_t v = voxel(li);
        rank[v] = r;
        if (!ALL) qmark[v] = 0;  // the marks are clear again for the next call
        ulist[(int64_t)gb * BV + r] = li;
      }
      base += __popcll(bal[k]);
    }
  }
}

// k_rank for bounded-window slice calls, visiting only the brick x rows
// that k_scatter flagged (`lines`).  Every other voxel of the brick has a
// zero count and no query, so it is neither loaded nor ranked.  One wave
// per brick (four bricks per block): it lists the brick's flagged rows in
// LDS, in row order, and clears their flags (the last reader; a brick
// without a flagged row only writes its zero row count).  Then it walks the
// listed rows, 64 / bx of them per step (a lane per voxel), in groups of
// kG steps: each lane issues the group's loads (its count, and the count
// beside it that the pair entries need: left of a row's first voxel, right
// of its last) before using any.  A brick's rows hold a few tens of events
// in sparse calls, so most of its rows are not visited at all and the wave
// waits on few rounds of loads.  Rows are listed in order and a row's
// voxels are consecutive lanes, so the wave numbers the query voxels in
// brick-local voxel order (as k_rank_lines4 does).  The pair grid is all
// zero between such calls (k_clear_events returns it there), so only the
// entries a flagged row touches are written: entry x of each of its voxels,
// and entry x + 1 of its last voxel in the slice (which the neighbouring
// brick may also write, with the same value: both read the final counts).
// A flagged row lies inside the slice (flags come from valid events only);
// its voxels beyond the slice's x edge are skipped.  Dynamic LDS: 4 waves x
// by x bt row numbers (uint16).
template <bool ALL>
__global__ __launch_bounds__(256) void k_rank_lines(Batch bt, Brick b,
                                                    const int32_t* __restrict__ count,
                                                    uint8_t* __restrict__ lines,
                                                    uint8_t* __restrict__ qmark,
                                                    int32_t* __restrict__ rank,
                                                    int32_t* __restrict__ ulist,
                                                    int32_t* __restrict__ brick_nq,
                                                    uint32_t* __restrict__ pairs,
                                                    int32_t* __restrict__ err) {
  constexpr int kG = 8, kU = 8;
  extern __shared__ uint16_t rl_rows[];
  const int lane = threadIdx.x & 63;
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int gb = blockIdx.x * 4 + wid;
  if (gb >= bt.nbricks) return;  // (no barriers below: each wave keeps to its own rows)
  const int NL = b.by * b.bt;
  uint16_t* rows = rl_rows + wid * NL;
  const unsigned long long below = (1ull << lane) - 1ull;
  int nr = 0;  // flagged rows (wave-uniform)
  {
    uint8_t* fl = lines + (int64_t)gb * NL;
    for (int l0 = 0; l0 < NL; l0 += 64 * kU) {
      uint8_t f[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int l = l0 + u * 64 + lane;
        f[u] = l < NL ? fl[l] : 0;
      }
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int l = l0 + u * 64 + lane;
        const unsigned long long bal = __ballot(f[u] != 0);
        if (f[u]) {
          rows[nr + __popcll(bal & below)] = (uint16_t)l;
          fl[l] = 0;
        }
        nr += __popcll(bal);
      }
    }
  }
  if (nr == 0) {
    if (lane == 0) brick_nq[gb] = 0;
    return;
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const SliceDesc s = slice_by_brick(bt, gb);  // (gb is uniform: scalar loads)
  const int lb = gb - s.brick_off;
  const int bxi = lb % s.nbx, byi = (lb / s.nbx) % s.nby, bti = lb / (s.nbx * s.nby);
  const int BV = b.bx * b.by * b.bt;
  const int sx = __builtin_ctz(b.bx), sy = __builtin_ctz(b.by);
  const int x0 = bxi * b.bx, y0 = byi * b.by, t0 = bti * b.bt;
  const int lx = lane & (b.bx - 1);  // the voxel's x within the brick (b.bx <= 64)
  const int slot = lane >> sx;       // which of the step's rows
  const int rps = 64 >> sx;          // rows per step
  const int x = x0 + lx;
  // slice-local voxel of brick-local li (slices hold fewer than 2^31 voxels)
  auto at = [&](int li) -> int {
    const int y = y0 + ((li >> sx) & (b.by - 1)), t = t0 + (li >> (sx + sy));
    return (t * s.H + y) * s.W + x;
  };
  const int32_t* cnt = count + s.grid_off;
  const bool has_left = lx == 0 && x > 0, has_right = lx == b.bx - 1 && x + 1 < s.W;
  const int steps = (nr + rps - 1) / rps;
  int base = 0;
  bool bad = false;
  for (int k0 = 0; k0 < steps; k0 += kG) {
    bool lf[kG];
    int lis[kG];
#pragma unroll
    for (int g = 0; g < kG; ++g) {
      const int j = (k0 + g) * rps + slot;
      lf[g] = j < nr && x < s.W;
      lis[g] = j < nr ? ((int)rows[j] << sx) + lx : 0;
    }
    int cv[kG], side[kG];
#pragma unroll
    for (int g = 0; g < kG; ++g) {
      const int o = at(lis[g]);
      cv[g] = lf[g] ? cnt[o] : 0;
      side[g] = lf[g] && (has_left || has_right) ? cnt[has_left ? o - 1 : o + 1] : 0;
    }
#pragma unroll
    for (int g = 0; g < kG; ++g) {
      if (k0 + g >= steps) break;  // (wave-uniform)
      const int up = __shfl_up(cv[g], 1);  // (all lanes)
      const int li = lis[g];
      bool f = false;
      if (lf[g]) {
        const int y = y0 + ((li >> sx) & (b.by - 1)), t = t0 + (li >> (sx + sy));
        const int lo = lx > 0 ? up : side[g];
        const int hi = cv[g];
        bad |= hi > VECKM_MAX_VOXEL_EVENTS;
        uint32_t* row = pairs + s.pair_off + ((int64_t)t * s.H + y) * (s.W + 1);
        row[x] = (uint32_t)__half_as_ushort(__float2half((float)lo)) |
                 ((uint32_t)__half_as_ushort(__float2half((float)hi)) << 16);
        if (lx == b.bx - 1 || x == s.W - 1) {
          const int right = x + 1 < s.W ? side[g] : 0;
          row[x + 1] = (uint32_t)__half_as_ushort(__float2half((float)hi)) |
                       ((uint32_t)__half_as_ushort(__float2half((float)right)) << 16);
        }
        f = ALL ? hi > 0 : qmark[s.grid_off + at(li)] != 0;
      }
      const unsigned long long bal = __ballot(f);
      if (f) {
        const int64_t v = s.grid_off + at(li);
        const int r = base + __popcll(bal & below);
        rank[v] = r;
        if (!ALL) qmark[v] = 0;  // the marks are clear again for the next call
        ulist[(int64_t)gb * BV + r] = li;
      }
      base += __popcll(bal);
    }
  }
  if (bad) atomicOr(err, kErrOverflow);
  if (lane == 0) brick_nq[gb] = base;
}

// k_rank_lines for dense calls (most bricks hold many rows): the same work
// with one block per brick, each of its NW waves taking an equal run of the
// brick's voxel steps, in order; the ballots of the query voxels go to LDS,
// one barrier gives every wave its offset, and a second pass writes the
// numbers.
template <bool ALL, int NW>
__global__ __launch_bounds__(NW * 64) void k_rank_lines4(Batch bt, Brick b,
                                                     const int32_t* __restrict__ count,
                                                     uint8_t* __restrict__ lines,
                                                     uint8_t* __restrict__ qmark,
                                                     int32_t* __restrict__ rank,
                                                     int32_t* __restrict__ ulist,
                                                     int32_t* __restrict__ brick_nq,
                                                     uint32_t* __restrict__ pairs,
                                                     int32_t* __restrict__ err) {
  constexpr int kG = 8;
  constexpr int kSteps = kMaxBrickVoxels / 64;
  __shared__ uint8_t sfl[kMaxBrickVoxels / 4];  // the brick's row flags (bx >= 4)
  __shared__ unsigned long long sbal[kSteps];   // query-voxel ballot of each step
  __shared__ int wave_tot[NW];
  const int gb = blockIdx.x;
  const int NL = b.by * b.bt;
  int any = 0;
  {
    uint8_t* fl = lines + (int64_t)gb * NL;
    for (int l = threadIdx.x; l < NL; l += NW * 64) {
      const uint8_t f = fl[l];
      sfl[l] = f;
      any |= f;
      if (f) fl[l] = 0;  // (the last reader: the flags are clear for the next call)
    }
  }
  if (!__syncthreads_or(any)) {
    if (threadIdx.x == 0) brick_nq[gb] = 0;
    return;
  }
  const SliceDesc s = slice_by_brick(bt, gb);
  const int lb = gb - s.brick_off;
  const int bxi = lb % s.nbx, byi = (lb / s.nbx) % s.nby, bti = lb / (s.nbx * s.nby);
  const int BV = b.bx * b.by * b.bt;
  const int sx = __builtin_ctz(b.bx), sy = __builtin_ctz(b.by);
  const int lane = threadIdx.x & 63;
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int x0 = bxi * b.bx, y0 = byi * b.by, t0 = bti * b.bt;
  const int lx = lane & (b.bx - 1);  // the voxel's x within the brick (b.bx <= 64)
  const int x = x0 + lx;
  auto at = [&](int li) -> int {
    const int y = y0 + ((li >> sx) & (b.by - 1)), t = t0 + (li >> (sx + sy));
    return (t * s.H + y) * s.W + x;
  };
  const int32_t* cnt = count + s.grid_off;
  const bool has_left = lx == 0 && x > 0, has_right = lx == b.bx - 1 && x + 1 < s.W;
  const int steps = (BV + 63) >> 6;
  const int per = (steps + NW - 1) / NW;  // steps of each wave
  const int k_lo = wid * per, k_hi = min(k_lo + per, steps);
  int tot = 0;
  bool bad = false;
  for (int k0 = k_lo; k0 < k_hi; k0 += kG) {
    bool lf[kG];
    bool anyf = false;
#pragma unroll
    for (int g = 0; g < kG; ++g) {
      const int li = (k0 + g) * 64 + lane;
      lf[g] = k0 + g < k_hi && li < BV && x < s.W && sfl[li >> sx] != 0;
      anyf |= lf[g];
    }
    if (!__ballot(anyf)) {
#pragma unroll
      for (int g = 0; g < kG; ++g)
        if (k0 + g < k_hi && lane == 0) sbal[k0 + g] = 0ull;
      continue;
    }
    int cv[kG], side[kG];
#pragma unroll
    for (int g = 0; g < kG; ++g) {
      const int o = at((k0 + g) * 64 + lane);
      cv[g] = lf[g] ? cnt[o] : 0;
      side[g] = lf[g] && (has_left || has_right) ? cnt[has_left ? o - 1 : o + 1] : 0;
    }
#pragma unroll
    for (int g = 0; g < kG; ++g) {
      const int up = __shfl_up(cv[g], 1);  // (all lanes)
      const int li = (k0 + g) * 64 + lane;
      bool f = false;
      if (lf[g]) {
        const int y = y0 + ((li >> sx) & (b.by - 1)), t = t0 + (li >> (sx + sy));
        const int lo = lx > 0 ? up : side[g];
        const int hi = cv[g];
        bad |= hi > VECKM_MAX_VOXEL_EVENTS;
        uint32_t* row = pairs + s.pair_off + ((int64_t)t * s.H + y) * (s.W + 1);
        row[x] = (uint32_t)__half_as_ushort(__float2half((float)lo)) |
                 ((uint32_t)__half_as_ushort(__float2half((float)hi)) << 16);
        if (lx == b.bx - 1 || x == s.W - 1) {
          const int right = x + 1 < s.W ? side[g] : 0;
          row[x + 1] = (uint32_t)__half_as_ushort(__float2half((float)hi)) |
                       ((uint32_t)__half_as_ushort(__float2half((float)right)) << 16);
        }
        f = ALL ? hi > 0 : qmark[s.grid_off + at(li)] != 0;
      }
      const unsigned long long bal = __ballot(f);
      if (k0 + g < k_hi && lane == 0) sbal[k0 + g] = bal;
      tot += __popcll(bal);
    }
  }
  if (bad) atomicOr(err, kErrOverflow);
  if (lane == 0) wave_tot[wid] = tot;
  __syncthreads();
  int base = 0;
  for (int w = 0; w < wid; ++w) base += wave_tot[w];
  if (threadIdx.x == 0) {
    int nq = 0;
    for (int w = 0; w < NW; ++w) nq += wave_tot[w];
    brick_nq[gb] = nq;
  }
  const unsigned long long below = (1ull << lane) - 1ull;
  for (int k = k_lo; k < k_hi; ++k) {
    const unsigned long long bal = sbal[k];
    if ((bal >> lane) & 1ull) {
      const int li = k * 64 + lane;
      const int64_t v = s.grid_off + at(li);
      const int r = base + __popcll(bal & below);
      rank[v] = r;
      if (!ALL) qmark[v] = 0;  // the marks are clear again for the next call
      ulist[(int64_t)gb * BV + r] = li;
    }
    base += __popcll(bal);
  }
}

// The count and pair grids of a dense call back to zero: one pass over both
// (cheaper than the per-event stores when the grids are small beside the
// events; see dense_batch).
__device__ inline void fill2_zero(int blk, int nblk, int32_t* __restrict__ a, int64_t na,
                                  uint32_t* __restrict__ b, int64_t nb) {
  const int64_t stride = (int64_t)nblk * blockDim.x;
  for (int64_t i = (int64_t)blk * blockDim.x + threadIdx.x; i < na + nb; i += stride) {
    if (i < na) a[i] = 0;
    else b[i - na] = 0u;
  }
}

__global__ void k_fill2_zero(int32_t* __restrict__ a, int64_t na, uint32_t* __restrict__ b,
                             int64_t nb) {
  fill2_zero(blockIdx.x, gridDim.x, a, na, b, nb);
}

// After a bounded-window slice call: every valid event's voxel count and
// the two pair entries that hold it (entries x and x + 1 of its row) back to
// zero; events that share a voxel store the same zeros.  These are all the
// non-zero entries (an entry holds the counts of voxels x - 1 and x).  The
// row flags were cleared by the ranking kernel, their last reader.
__global__ void k_clear_events(Batch bt, const int32_t* __restrict__ vox,
                               int32_t* __restrict__ count, uint32_t* __restrict__ pairs) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (blockIdx.x * blockDim.x >= bt.n) return;  // (whole block; launches never do this)
  const SliceDesc s = slice_by_event_block(bt, i);
  if (i >= bt.n) return;
  const int v = vox[i];
  if (v < 0) return;
  count[s.grid_off + v] = 0;
  const int64_t e = s.pair_off + v + v / s.W;  // entry x of row v / W
  pairs[e] = 0u;
  pairs[e + 1] = 0u;
}

// Exclusive scan of the per-brick row counts into off[] (off[nb] = total
// rows U) and the list of non-empty bricks in order[] (one record per brick:
// brick, rows, first row, slice), by size class (most encoder chunks
// first: 64 or more, 32-63, 16-31, 12-15, 8-11, then 7, 6, ..., 1 exactly;
// longest job first keeps the persistent encoder's tail short) and by brick
// number within a class.  plan[0] = U, plan[1] = 0 (the encoder's work counter),
// plan[2] = number of non-empty bricks.  Three launches: per-tile totals,
// a scan of the tile totals, then each tile places its bricks.  Within a
// tile thread t owns bricks [t kScanPer, (t + 1) kScanPer); nothing is
// counted with atomics, so order[] is the same on every call.
constexpr int kScanClasses = 12;  // kScanNV = class counts, then rows of the
constexpr int kRowsD = 12;        // bricks the encoder takes whole,
constexpr int kRowsS = 13;        // then rows of the bricks it takes as single rows
constexpr int kScanThreads = 1024, kScanPer = kScanTile / kScanThreads;
constexpr int kScanSmall = 256;  // threads of the scan of up to 2048 bricks
static_assert(kScanNV == kScanClasses + 2 && kScanTile % kScanThreads == 0, "scan tiles");

// Bricks with fewer than `sp` rows (0: none) are not the encoder's work
// items: their rows are numbered after all other rows and listed one by one
// in srow ({brick, brick-local voxel} per row), and the encoder takes them
// in items of up to `rs` rows, each row with a count box of its own.
struct SparseRows {
  int sp = 0, rs = 1, bv = 0;
  const int32_t* ulist = nullptr;
  int2* srow = nullptr;
};

__device__ inline bool sparse_brick(int q, int sp) { return q > 0 && q < sp; }

__device__ inline int chunk_class(int nq, int ch) {
  const int c = (nq + ch - 1) / ch;
  return c >= 64 ? 0 : c >= 32 ? 1 : c >= 16 ? 2 : c >= 12 ? 3 : c >= 8 ? 4 : 12 - c;
}

// The tile's counts (coalesced through LDS), this thread's class counts and
// rows in v[], their exclusive scan over the tile's threads in ex[], the
// tile totals in tot[].
template <int NT = kScanThreads>
__device__ inline void scan_tile(const int32_t* __restrict__ nq, int nb, int ch, int sp, int tile,
                                 int (&q)[kScanPer], int (&v)[kScanNV], int (&ex)[kScanNV],
                                 int (&tot)[kScanNV]) {
  constexpr int NWV = NT / 64;  // waves
  constexpr int TILE = NT * kScanPer;
  __shared__ int tq[TILE];
  __shared__ int wsum[kScanNV][NWV];
  __shared__ int ttot[kScanNV];
  const int tid = threadIdx.x, base = tile * TILE;
  const int lane = tid & 63, wid = tid >> 6;
#pragma unroll
  for (int u = 0; u < kScanPer; ++u) {
    const int i = base + u * NT + tid;
    tq[u * NT + tid] = i < nb ? nq[i] : 0;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kScanNV; ++k) v[k] = 0;
#pragma unroll
  for (int u = 0; u < kScanPer; ++u) {
    q[u] = tq[tid * kScanPer + u];
    const bool sb = sparse_brick(q[u], sp);
    v[kRowsD] += sb ? 0 : q[u];
    v[kRowsS] += sb ? q[u] : 0;
    const int c = q[u] > 0 && !sb ? chunk_class(q[u], ch) : -1;
#pragma unroll
    for (int k = 0; k < kScanClasses; ++k) v[k] += c == k;
  }
  // inclusive scans within each wave (shuffles), then over the wave totals
  int inc[kScanNV];
#pragma unroll
  for (int k = 0; k < kScanNV; ++k) inc[k] = v[k];
#pragma unroll
  for (int d = 1; d < 64; d <<= 1)
#pragma unroll
    for (int k = 0; k < kScanNV; ++k) {
      const int t = __shfl_up(inc[k], d);
      if (lane >= d) inc[k] += t;
    }
  if (lane == 63)
#pragma unroll
    for (int k = 0; k < kScanNV; ++k) wsum[k][wid] = inc[k];
  __syncthreads();
  if (wid == 0) {  // exclusive scan of the wave totals (lanes 0 .. NWV-1)
#pragma unroll
    for (int k = 0; k < kScanNV; ++k) {
      const int own = lane < NWV ? wsum[k][lane] : 0;
      int s = own;
#pragma unroll
      for (int d = 1; d < NWV; d <<= 1) {
        const int t = __shfl_up(s, d);
        if (lane >= d) s += t;
      }
      const int total = __shfl(s, NWV - 1);
      if (lane < NWV) wsum[k][lane] = s - own;
      if (lane == 0) ttot[k] = total;
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kScanNV; ++k) {
    ex[k] = wsum[k][wid] + inc[k] - v[k];
    tot[k] = ttot[k];
  }
}

__global__ __launch_bounds__(kScanThreads) void k_scan_totals(const int32_t* __restrict__ nq,
                                                              int nb, int ch, int sp,
                                                              int32_t* __restrict__ part) {
  int q[kScanPer], v[kScanNV], ex[kScanNV], tot[kScanNV];
  scan_tile(nq, nb, ch, sp, blockIdx.x, q, v, ex, tot);
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < kScanNV; ++k) part[blockIdx.x * kScanNV + k] = tot[k];
}

// One block: turns the tile totals into each tile's starting positions
// (class k of tile b starts at the class's start plus the class counts of
// tiles before b; rows likewise).
__global__ __launch_bounds__(kScanThreads) void k_scan_tiles(int ntiles, int nb, int rs,
                                                             int32_t* __restrict__ part,
                                                             int32_t* __restrict__ off,
                                                             int4* __restrict__ order,
                                                             int32_t* __restrict__ plan) {
  __shared__ int sums[kScanNV][kScanThreads];
  const int tid = threadIdx.x;
  const int per = (ntiles + kScanThreads - 1) / kScanThreads;
  const int s0 = min(tid * per, ntiles), s1 = min(s0 + per, ntiles);
  int v[kScanNV];
#pragma unroll
  for (int k = 0; k < kScanNV; ++k) {
    v[k] = 0;
    for (int i = s0; i < s1; ++i) v[k] += part[i * kScanNV + k];
    sums[k][tid] = v[k];
  }
  __syncthreads();
  for (int d = 1; d < kScanThreads; d <<= 1) {
    int add[kScanNV];
#pragma unroll
    for (int k = 0; k < kScanNV; ++k) add[k] = tid >= d ? sums[k][tid - d] : 0;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kScanNV; ++k) sums[k][tid] += add[k];
    __syncthreads();
  }
  int start[kScanNV];
  int acc = 0;
#pragma unroll
  for (int k = 0; k < kScanClasses; ++k) {
    start[k] = acc;
    acc += sums[k][kScanThreads - 1];
  }
  const int ud = sums[kRowsD][kScanThreads - 1], us = sums[kRowsS][kScanThreads - 1];
  start[kRowsD] = 0;
  start[kRowsS] = ud;  // single rows are numbered after the others
  int run[kScanNV];
#pragma unroll
  for (int k = 0; k < kScanNV; ++k) run[k] = start[k] + sums[k][tid] - v[k];
  for (int i = s0; i < s1; ++i)
#pragma unroll
    for (int k = 0; k < kScanNV; ++k) {
      const int t = part[i * kScanNV + k];
      part[i * kScanNV + k] = run[k];
      run[k] += t;
    }
  // the single-row items follow the bricks in the work list
  const int ns = (us + rs - 1) / rs;
  for (int j = tid; j < ns; j += kScanThreads)
    order[acc + j] = make_int4(kSparseTag | j, min(rs, us - j * rs), ud + j * rs, j * rs);
  if (tid == 0) {
    off[nb] = ud + us;
    plan[0] = ud + us;
    plan[1] = 0;
    plan[2] = acc + ns;
    plan[3] = ud;
  }
}

// ONE = true: the bricks fit in one tile, and this single block does the
// whole scan (part is not used; plan and off[nb] are written here).
template <bool ONE, bool SP, int NT = kScanThreads>
__global__ __launch_bounds__(NT) void k_scan_place(Batch bt,
                                                             const int32_t* __restrict__ nq,
                                                             int nb, int ch, SparseRows sr,
                                                             const int32_t* __restrict__ part,
                                                             int32_t* __restrict__ off,
                                                             int4* __restrict__ order,
                                                             int32_t* __restrict__ plan) {
  int q[kScanPer], v[kScanNV], ex[kScanNV], tot[kScanNV];
  static_assert(ONE || NT == kScanThreads, "tiles of kScanTile bricks");
  scan_tile<NT>(nq, nb, ch, SP ? sr.sp : 0, blockIdx.x, q, v, ex, tot);
  int pos[kScanNV];
  int ud;  // rows of the bricks taken whole: single rows start here
  if constexpr (ONE) {
    int start = 0;
#pragma unroll
    for (int k = 0; k < kScanClasses; ++k) {
      pos[k] = start + ex[k];
      start += tot[k];
    }
    ud = tot[kRowsD];
    pos[kRowsD] = ex[kRowsD];
    pos[kRowsS] = ud + ex[kRowsS];
    // the single-row items follow the bricks in the work list
    const int us = SP ? tot[kRowsS] : 0, ns = SP ? (us + sr.rs - 1) / sr.rs : 0;
    if constexpr (SP)
      for (int j = threadIdx.x; j < ns; j += NT)
        order[start + j] = make_int4(kSparseTag | j, min(sr.rs, us - j * sr.rs), ud + j * sr.rs,
                                     j * sr.rs);
    if (threadIdx.x == 0) {
      off[nb] = ud + us;
      plan[0] = ud + us;
      plan[1] = 0;
      plan[2] = start + ns;
      plan[3] = ud;
    }
  } else {
#pragma unroll
    for (int k = 0; k < kScanNV; ++k) pos[k] = part[blockIdx.x * kScanNV + k] + ex[k];
    ud = plan[3];
  }
  const int i0 = blockIdx.x * (NT * kScanPer) + threadIdx.x * kScanPer;
#pragma unroll
  for (int u = 0; u < kScanPer; ++u) {
    const int i = i0 + u;
    if (i >= nb) break;
    if (SP && sparse_brick(q[u], sr.sp)) {
      // its rows, one by one, among the single rows (all loads at once)
      off[i] = pos[kRowsS];
      int li[kSparseBelow - 1];
#pragma unroll
      for (int r = 0; r < kSparseBelow - 1; ++r)
        li[r] = r < q[u] ? sr.ulist[(int64_t)i * sr.bv + r] : 0;
#pragma unroll
      for (int r = 0; r < kSparseBelow - 1; ++r)
        if (r < q[u]) sr.srow[pos[kRowsS] - ud + r] = make_int2(i, li[r]);
      pos[kRowsS] += q[u];
      continue;
    }
    off[i] = pos[kRowsD];
    pos[kRowsD] += q[u];
    if (q[u] > 0) {
      const int c = chunk_class(q[u], ch);
      int p = 0;
#pragma unroll
      for (int k = 0; k < kScanClasses; ++k)
        if (c == k) p = pos[k]++;
      int sl = 0;  // the brick's slice
      if (bt.nslices > 1) {
        int hi = bt.nslices - 1;
        while (sl < hi) {
          const int mid = (sl + hi + 1) >> 1;
          if (bt.table[mid].brick_off <= i) sl = mid; else hi = mid - 1;
        }
      }
      order[p] = make_int4(i, q[u], pos[kRowsD] - q[u], sl);
    }
  }
}

// The three launches of the brick scan (part: kScanNV ints per tile).
static void launch_brick_scan(const Batch& bt, const Workspace& w, int nb, int ch,
                              const SparseRows& sr, hipStream_t s) {
  const int ntiles = nb > 0 ? (int)scan_tiles(nb) : 1;
  int4* order = reinterpret_cast<int4*>(w.order);
  if (nb <= kScanSmall * kScanPer) {  // one small block: a quarter of the issue work
    if (sr.sp > 0)
      hipLaunchKernelGGL((k_scan_place<true, true, kScanSmall>), dim3(1), dim3(kScanSmall), 0, s,
                         bt, w.brick_nq, nb, ch, sr, w.scan_part, w.brick_off, order, w.plan);
    else
      hipLaunchKernelGGL((k_scan_place<true, false, kScanSmall>), dim3(1), dim3(kScanSmall), 0,
                         s, bt, w.brick_nq, nb, ch, sr, w.scan_part, w.brick_off, order, w.plan);
    return;
  }
  if (ntiles == 1) {
    if (sr.sp > 0)
      hipLaunchKernelGGL((k_scan_place<true, true>), dim3(1), dim3(kScanThreads), 0, s, bt,
                         w.brick_nq, nb, ch, sr, w.scan_part, w.brick_off, order, w.plan);
    else
      hipLaunchKernelGGL((k_scan_place<true, false>), dim3(1), dim3(kScanThreads), 0, s, bt,
                         w.brick_nq, nb, ch, sr, w.scan_part, w.brick_off, order, w.plan);
    return;
  }
  hipLaunchKernelGGL(k_scan_totals, dim3(ntiles), dim3(kScanThreads), 0, s, w.brick_nq, nb, ch,
                     sr.sp, w.scan_part);
  hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(kScanThreads), 0, s, ntiles, nb, sr.rs,
                     w.scan_part, w.brick_off, order, w.plan);
  if (sr.sp > 0)
    hipLaunchKernelGGL((k_scan_place<false, true>), dim3(ntiles), dim3(kScanThreads), 0, s, bt,
                       w.brick_nq, nb, ch, sr, w.scan_part, w.brick_off, order, w.plan);
  else
    hipLaunchKernelGGL((k_scan_place<false, false>), dim3(ntiles), dim3(kScanThreads), 0, s, bt,
                       w.brick_nq, nb, ch, sr, w.scan_part, w.brick_off, order, w.plan);
}

// The row of slice-local voxel v (a query voxel of slice s).
__device__ inline int qmap_row(const SliceDesc& s, const Brick& b, int v,
                               const int32_t* __restrict__ rank,
                               const int32_t* __restrict__ brick_off) {
  const int x = v % s.W, y = (v / s.W) % s.H, t = v / (s.W * s.H);
  const int lb = ((t / b.bt) * s.nby + y / b.by) * s.nbx + x / b.bx;
  return brick_off[s.brick_off + lb] + rank[s.grid_off + v];
}

// One thread per query: the row of its voxel (or -1 for an invalid event).
__global__ void k_qmap(const int32_t* __restrict__ queries, Batch bt, Brick b,
                       const int32_t* __restrict__ vox, const int32_t* __restrict__ rank,
                       const int32_t* __restrict__ brick_off, int32_t* __restrict__ qmap,
                       int32_t* __restrict__ rowvox) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (!queries) {  // query i is event i: consecutive per block
    if (blockIdx.x * blockDim.x >= bt.m) return;  // (whole block; launches never do this)
    const SliceDesc s = slice_by_event_block(bt, i);
    if (i >= bt.m) return;
    const int v = vox[i];
    const int r = v < 0 ? -1 : qmap_row(s, b, v, rank, brick_off);
    qmap[i] = r;
    if (rowvox && r >= 0) rowvox[r] = v;
    return;
  }
  if (i >= bt.m) return;
  const int e = queries[i];
  if (e < 0 || e >= bt.n) {
    qmap[i] = -1;
    return;
  }
  const int v = vox[e];
  if (v < 0) {
    qmap[i] = -1;
    return;
  }
  const int r = qmap_row(slice_by_event(bt, e), b, v, rank, brick_off);
  qmap[i] = r;
  if (rowvox) rowvox[r] = v;  // every query of the voxel writes the same value
}

// One wavefront per query: copy its voxel's encoding row.
__global__ void k_expand_emb(const int32_t* __restrict__ qmap, int m,
                             const float* __restrict__ rows, int d2, float* __restrict__ out) {
  const int64_t q = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (q >= m) return;
  const int r = qmap[q];
  const float4* src = reinterpret_cast<const float4*>(rows + (int64_t)(r < 0 ? 0 : r) * d2);
  float4* dst = reinterpret_cast<float4*>(out + q * d2);
  const float nan = __builtin_nanf("");
  for (int c = lane; c < d2 / 4; c += 64) dst[c] = r >= 0 ? src[c] : make_float4(nan, nan, nan, nan);
}

__global__ void k_expand_flow(const int32_t* __restrict__ qmap, int m,
                              const float2* __restrict__ rowflow, float2* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const int r = qmap[i];
  const float nan = __builtin_nanf("");
  out[i] = r >= 0 ? rowflow[r] : make_float2(nan, nan);
}

// Output expansion without a query -> row map (all forms but the paper
// form): each query finds its row from its event's voxel, the voxel's rank
// in its brick and the brick's first row.  SUB: `queries` lists the query
// events (one slice); else query i is event i.
template <bool SUB>
__device__ inline int query_row(const int32_t* __restrict__ queries, const Batch& bt,
                                const SliceDesc& s, const Brick& b,
                                const int32_t* __restrict__ vox, const int32_t* __restrict__ rank,
                                const int32_t* __restrict__ brick_off, int i) {
  const int e = SUB ? queries[i] : i;
  if (e < 0 || e >= bt.n) return -1;  // (reported by k_mark)
  const int v = vox[e];
  return v < 0 ? -1 : qmap_row(s, b, v, rank, brick_off);
}

template <bool SUB>
__device__ inline void expand_flow_q(int blk, const int32_t* __restrict__ queries, const Batch& bt,
                                     const Brick& b, const int32_t* __restrict__ vox,
                                     const int32_t* __restrict__ rank,
                                     const int32_t* __restrict__ brick_off,
                                     const float2* __restrict__ rowflow, float2* __restrict__ out) {
  const int i = blk * blockDim.x + threadIdx.x;
  if (blk * (int)blockDim.x >= bt.m) return;  // (whole block; launches never do this)
  const SliceDesc s = SUB ? bt.s0 : slice_by_event_block(bt, i);
  if (i >= bt.m) return;
  const int r = query_row<SUB>(queries, bt, s, b, vox, rank, brick_off, i);
  const float nan = __builtin_nanf("");
  out[i] = r >= 0 ? rowflow[r] : make_float2(nan, nan);
}

template <bool SUB>
__global__ void k_expand_flow_q(const int32_t* __restrict__ queries, Batch bt, Brick b,
                                const int32_t* __restrict__ vox, const int32_t* __restrict__ rank,
                                const int32_t* __restrict__ brick_off,
                                const float2* __restrict__ rowflow, float2* __restrict__ out) {
  expand_flow_q<SUB>(blockIdx.x, queries, bt, b, vox, rank, brick_off, rowflow, out);
}

// The flows of a dense call and the clear of its count and pair grids in one
// launch: blocks [0, eb) expand, the others zero the grids (k_fill2_zero's
// work).  The expansion reads neither grid, so the two parts need no order,
// and the call saves a launch.
template <bool SUB>
__global__ void k_expand_flow_q_fill(const int32_t* __restrict__ queries, Batch bt, Brick b,
                                     const int32_t* __restrict__ vox,
                                     const int32_t* __restrict__ rank,
                                     const int32_t* __restrict__ brick_off,
                                     const float2* __restrict__ rowflow, float2* __restrict__ out,
                                     int eb, int32_t* __restrict__ count,
                                     uint32_t* __restrict__ pairs) {
  if ((int)blockIdx.x < eb)
    expand_flow_q<SUB>(blockIdx.x, queries, bt, b, vox, rank, brick_off, rowflow, out);
  else
    fill2_zero(blockIdx.x - eb, gridDim.x - eb, count, bt.nvox, pairs, bt.npairs);
}

template <bool SUB>
__global__ void k_expand_count_q(const int32_t* __restrict__ queries, Batch bt, Brick b,
                                 const int32_t* __restrict__ vox, const int32_t* __restrict__ rank,
                                 const int32_t* __restrict__ brick_off,
                                 const int32_t* __restrict__ rowcnt, int32_t* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (blockIdx.x * blockDim.x >= bt.m) return;  // (whole block; launches never do this)
  const SliceDesc s = SUB ? bt.s0 : slice_by_event_block(bt, i);
  if (i >= bt.m) return;
  const int r = query_row<SUB>(queries, bt, s, b, vox, rank, brick_off, i);
  out[i] = r >= 0 ? rowcnt[r] : -1;
}

// One wavefront per query.
template <bool SUB>
__global__ void k_expand_emb_q(const int32_t* __restrict__ queries, Batch bt, Brick b,
                               const int32_t* __restrict__ vox, const int32_t* __restrict__ rank,
                               const int32_t* __restrict__ brick_off,
                               const float* __restrict__ rows, int d2, float* __restrict__ out) {
  const int64_t q = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (q >= bt.m) return;
  const SliceDesc s = SUB ? bt.s0 : slice_by_event(bt, (int)q);
  const int r = query_row<SUB>(queries, bt, s, b, vox, rank, brick_off, (int)q);
  const float4* src = reinterpret_cast<const float4*>(rows + (int64_t)(r < 0 ? 0 : r) * d2);
  float4* dst = reinterpret_cast<float4*>(out + q * d2);
  const float nan = __builtin_nanf("");
  for (int c = lane; c < d2 / 4; c += 64) dst[c] = r >= 0 ? src[c] : make_float4(nan, nan, nan, nan);
}

static int blocks_for(int64_t n, int per) { return (int)((n + per - 1) / per); }

static int fill_grid(int64_t n) {
  int64_t b = (n + 255) / 256;
  return (int)(b < 8192 ? (b < 1 ? 1 : b) : 8192);
}

// k_pairs over nslices slices of at most max_rows x rows each: about 4096
// blocks in all (4 rows at a time per block).
static dim3 pairs_grid(int nslices, int64_t max_rows) {
  int64_t x = (4096 + nslices - 1) / nslices;
  const int64_t need = (max_rows + 3) / 4;
  x = x < need ? x : need;
  return dim3((unsigned)(x < 1 ? 1 : x), (unsigned)nslices);
}

// k_rank for every voxel with events (all) or only the marked ones; with
// `pairs` it also builds the pair grid.
static void launch_rank(const Batch& bt, const Workspace& w, const Brick& b, bool all,
                        hipStream_t s) {
  static_assert(kMaxBrickVoxels <= 8192, "k_rank holds at most 32 ballots per wave");
  const bool big = b.volume() > 4096;
  auto go = [&](auto fn) {
    hipLaunchKernelGGL(fn, dim3(bt.nbricks), dim3(256), 0, s, bt, b, w.count, w.qmark, w.rank,
                       w.ulist, w.brick_nq);
  };
  if (all)
    big ? go(k_rank<true, 32>) : go(k_rank<true, 16>);
  else
    big ? go(k_rank<false, 32>) : go(k_rank<false, 16>);
}

static void launch_rank_lines(const Batch& bt, const Workspace& w, const Brick& b, bool all,
                              hipStream_t s) {
  // dense calls: a block per brick; else a wave per brick (latency-bound
  // sparse bricks)
  auto go = [&](auto fn, unsigned blocks, size_t lds) {
    hipLaunchKernelGGL(fn, dim3(blocks), dim3(256), lds, s, bt, b, w.count, w.lines, w.qmark,
                       w.rank, w.ulist, w.brick_nq, w.pairs, w.err);
  };
  auto go8 = [&](auto fn, unsigned blocks) {
    hipLaunchKernelGGL(fn, dim3(blocks), dim3(512), 0, s, bt, b, w.count, w.lines, w.qmark,
                       w.rank, w.ulist, w.brick_nq, w.pairs, w.err);
  };
  const unsigned nb = (unsigned)bt.nbricks, nb4 = (unsigned)((bt.nbricks + 3) / 4);
  const size_t rows_lds = 4 * (size_t)b.by * b.bt * sizeof(uint16_t);  // (at most 16 KiB)
  if (dense_batch(bt)) {
    // (8 waves for the largest bricks: with a quarter of the blocks, 4 waves
    // each left the kernel latency-bound)
    if (b.volume() > 4096)
      all ? go8(k_rank_lines4<true, 8>, nb) : go8(k_rank_lines4<false, 8>, nb);
    else
      all ? go(k_rank_lines4<true, 4>, nb, 0) : go(k_rank_lines4<false, 4>, nb, 0);
  } else {
    all ? go(k_rank_lines<true>, nb4, rows_lds) : go(k_rank_lines<false>, nb4, rows_lds);
  }
}

int launch_clear_events(const Batch& bt, const Workspace& w, void* stream) {
  if (dense_batch(bt))
    hipLaunchKernelGGL(k_fill2_zero, dim3(fill_grid(bt.nvox + bt.npairs)), dim3(256), 0,
                       (hipStream_t)stream, w.count, bt.nvox, w.pairs, bt.npairs);
  else if (bt.n > 0)
    hipLaunchKernelGGL(k_clear_events, dim3(blocks_for(bt.n, 256)), dim3(256), 0,
                       (hipStream_t)stream, bt, w.vox, w.count, w.pairs);
  return hipGetLastError() == hipSuccess ? VECKM_OK : VECKM_E_HIP;
}

int launch_clear_grids(const Batch& bt, const Workspace& w, int64_t nlines, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_fill_i32, dim3(fill_grid(bt.nvox)), dim3(256), 0, s, w.count, bt.nvox, 0);
  hipLaunchKernelGGL(k_fill_i32, dim3(fill_grid(bt.npairs)), dim3(256), 0, s,
                     reinterpret_cast<int32_t*>(w.pairs), bt.npairs, 0);
  const int64_t words = (nlines + 3) / 4;
  hipLaunchKernelGGL(k_fill_i32, dim3(fill_grid(words)), dim3(256), 0, s,
                     reinterpret_cast<int32_t*>(w.lines), words, 0);
  return hipGetLastError() == hipSuccess ? VECKM_OK : VECKM_E_HIP;
}

int launch_prepare(const Batch& bt, const Workspace& w, const veckm_event* ev,
                   const int32_t* queries, const EncodeTables& et, bool pairs, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  // (a brick has at most kMaxBrickVoxels / 4 rows of flags; a step of the
  // ranking kernels holds whole rows)
  if (pairs && (et.brick.bx < 4 || et.brick.bx > 64)) return VECKM_E_INVAL;
  // slice calls (not the paper form) find the count grid, the pair grid and
  // the row flags zero: every such call returns them to zero after use (the
  // ranking kernel clears the flags, launch_clear_events the rest; all three
  // are zeroed once at context creation); the paper form clears the count
  // grid here
  if (!pairs)
    hipLaunchKernelGGL(k_fill_i32, dim3(fill_grid(bt.nvox)), dim3(256), 0, s, w.count, bt.nvox, 0);
  if (bt.n > 0)
    hipLaunchKernelGGL(k_scatter<true>, dim3(blocks_for(bt.n, 256)), dim3(256), 0, s,
                       reinterpret_cast<const int4*>(ev), bt, w.count, w.vox, w.err,
                       (uint8_t*)nullptr, et.brick, pairs ? w.lines : (uint8_t*)nullptr);
  if (queries && bt.m > 0)
    hipLaunchKernelGGL(k_mark, dim3(blocks_for(bt.m, 256)), dim3(256), 0, s, queries, bt, w.vox,
                       w.qmark, w.err);
  if (pairs)
    launch_rank_lines(bt, w, et.brick, queries == nullptr, s);
  else
    launch_rank(bt, w, et.brick, queries == nullptr, s);
  // single rows, unless every brick is likely to hold many (a dense call
  // with 32 or more rows per brick on average)
  SparseRows sr;
  if (pairs && et.sp > 0 && !(dense_batch(bt) && (int64_t)bt.m >= 32 * (int64_t)bt.nbricks)) {
    sr.sp = et.sp;
    sr.rs = et.rs;
    sr.bv = et.brick.volume();
    sr.ulist = w.ulist;
    sr.srow = reinterpret_cast<int2*>(w.srow);
  }
  launch_brick_scan(bt, w, bt.nbricks, encode_rows_per_chunk(et.d, et.layout), sr, s);
  // the paper form needs each row's voxel (and its expansion reads the query
  // -> row map); the other forms find rows as they expand
  if (!pairs && bt.m > 0)
    hipLaunchKernelGGL(k_qmap, dim3(blocks_for(bt.m, 256)), dim3(256), 0, s, queries, bt,
                       et.brick, w.vox, w.rank, w.brick_off, w.qmap, w.rowvox);
  return hipGetLastError() == hipSuccess ? VECKM_OK : VECKM_E_HIP;
}

int launch_window_push(const Workspace& w, const veckm_event* ev, int64_t n, int W, int H, int T,
                       int t0, int nbins, int tref, int64_t clear_b0, int clear_nb, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  const int64_t plane = (int64_t)W * H, pplane = (int64_t)(W + 1) * H;
  // the planes of the bins that enter the window: clear them, count the new
  // events, rebuild their pairs
  const int p0 = (int)((clear_b0 - tref) % T);
  const int first = clear_nb < T - p0 ? clear_nb : T - p0;  // planes before the ring wraps
  const int span[2][2] = {{p0, first}, {0, clear_nb - first}};
  for (const auto& sp : span)
    if (sp[1] > 0)
      hipLaunchKernelGGL(k_fill_i32, dim3(fill_grid(sp[1] * plane)), dim3(256), 0, s,
                         w.count + sp[0] * plane, sp[1] * plane, 0);
  if (n > 0)
    hipLaunchKernelGGL(k_push, dim3(blocks_for(n, 256)), dim3(256), 0, s,
                       reinterpret_cast<const int4*>(ev), (int)n, W, H, T, t0, nbins, tref,
                       w.count, w.err);
  for (const auto& sp : span)
    if (sp[1] > 0) {
      Batch pb{};
      pb.s0.W = W;
      pb.s0.H = H;
      pb.s0.T = sp[1];
      pb.nslices = 1;
      pb.npairs = sp[1] * pplane;
      hipLaunchKernelGGL(k_pairs, pairs_grid(1, (int64_t)H * sp[1]), dim3(256), 0, s, pb,
                         w.count + sp[0] * plane, w.pairs + sp[0] * pplane, w.err);
    }
  return hipGetLastError() == hipSuccess ? VECKM_OK : VECKM_E_HIP;
}

int launch_window_prepare(const Batch& bt, const Workspace& w, const veckm_event* queries,
                          const EncodeTables& et, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  if (bt.n > 0) {
    // locate the query events and mark their voxels in one pass
    hipLaunchKernelGGL(k_scatter<false>, dim3(blocks_for(bt.n, 256)), dim3(256), 0, s,
                       reinterpret_cast<const int4*>(queries), bt, w.count, w.vox, w.err, w.qmark,
                       et.brick, (uint8_t*)nullptr);
  }
  launch_rank(bt, w, et.brick, false, s);
  launch_brick_scan(bt, w, bt.nbricks, encode_rows_per_chunk(et.d, et.layout), SparseRows{}, s);
  return hipGetLastError() == hipSuccess ? VECKM_OK : VECKM_E_HIP;
}

int launch_take_err(const Workspace& w, int32_t* host, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  if (hipMemcpyAsync(host, w.err, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess)
    return VECKM_E_HIP;
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, w.err, (int64_t)1, 0);
  return hipGetLastError() == hipSuccess ? VECKM_OK : VECKM_E_HIP;
}

int launch_expand_emb(const Batch& bt, const Workspace& w, const int32_t* queries,
                      const Brick& b, bool use_qmap, int d, float* emb, void* stream) {
  if (bt.m <= 0) return VECKM_OK;
  hipStream_t s = (hipStream_t)stream;
  const dim3 grid(blocks_for((int64_t)bt.m * 64, 256));
  const float* rows = static_cast<const float*>(w.rows);
  if (use_qmap)
    hipLaunchKernelGGL(k_expand_emb, grid, dim3(256), 0, s, w.qmap, bt.m, rows, 2 * d, emb);
  else if (queries)
    hipLaunchKernelGGL(k_expand_emb_q<true>, grid, dim3(256), 0, s, queries, bt, b, w.vox, w.rank,
                       w.brick_off, rows, 2 * d, emb);
  else
    hipLaunchKernelGGL(k_expand_emb_q<false>, grid, dim3(256), 0, s, queries, bt, b, w.vox,
                       w.rank, w.brick_off, rows, 2 * d, emb);
  return hipGetLastError() == hipSuccess ? VECKM_OK : VECKM_E_HIP;
}

int launch_expand_flow(const Batch& bt, const Workspace& w, const int32_t* queries,
                       const Brick& b, bool use_qmap, float* flow, void* stream) {
  if (bt.m <= 0) return VECKM_OK;
  hipStream_t s = (hipStream_t)stream;
  const dim3 grid(blocks_for(bt.m, 256));
  const float2* rf = reinterpret_cast<const float2*>(w.rowflow);
  float2* out = reinterpret_cast<float2*>(flow);
  if (use_qmap)
    hipLaunchKernelGGL(k_expand_flow, grid, dim3(256), 0, s, w.qmap, bt.m, rf, out);
  else if (queries)
    hipLaunchKernelGGL(k_expand_flow_q<true>, grid, dim3(256), 0, s, queries, bt, b, w.vox,
                       w.rank, w.brick_off, rf, out);
  else
    hipLaunchKernelGGL(k_expand_flow_q<false>, grid, dim3(256), 0, s, queries, bt, b, w.vox,
                       w.rank, w.brick_off, rf, out);
  return hipGetLastError() == hipSuccess ? VECKM_OK : VECKM_E_HIP;
}

int launch_expand_flow_clear(const Batch& bt, const Workspace& w, const int32_t* queries,
                             const Brick& b, float* flow, void* stream) {
  if (!dense_batch(bt)) return VECKM_E_INVAL;
  const int eb = bt.m > 0 ? blocks_for(bt.m, 256) : 0;
  const dim3 grid(eb + fill_grid(bt.nvox + bt.npairs));
  const float2* rf = reinterpret_cast<const float2*>(w.rowflow);
  float2* out = reinterpret_cast<float2*>(flow);
  hipStream_t s = (hipStream_t)stream;
  if (queries)
    hipLaunchKernelGGL(k_expand_flow_q_fill<true>, grid, dim3(256), 0, s, queries, bt, b, w.vox,
                       w.rank, w.brick_off, rf, out, eb, w.count, w.pairs);
  else
    hipLaunchKernelGGL(k_expand_flow_q_fill<false>, grid, dim3(256), 0, s, queries, bt, b, w.vox,
                       w.rank, w.brick_off, rf, out, eb, w.count, w.pairs);
  return hipGetLastError() == hipSuccess ? VECKM_OK : VECKM_E_HIP;
}

int launch_expand_count(const Batch& bt, const Workspace& w, const int32_t* queries,
                        const Brick& b, int32_t* counts, void* stream) {
  if (bt.m <= 0) return VECKM_OK;
  hipStream_t s = (hipStream_t)stream;
  const dim3 grid(blocks_for(bt.m, 256));
  const int32_t* rc = reinterpret_cast<const int32_t*>(w.rowflow);
  if (queries)
    hipLaunchKernelGGL(k_expand_count_q<true>, grid, dim3(256), 0, s, queries, bt, b, w.vox,
                       w.rank, w.brick_off, rc, counts);
  else
    hipLaunchKernelGGL(k_expand_count_q<false>, grid, dim3(256), 0, s, queries, bt, b, w.vox,
                       w.rank, w.brick_off, rc, counts);
  return hipGetLastError() == hipSuccess ? VECKM_OK : VECKM_E_HIP;
}

}  // namespace veckm
