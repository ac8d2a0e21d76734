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

__global__ void k_fill_u8(uint8_t* __restrict__ p, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0;
}

// One thread per event: validate against its slice, histogram (ADD), remember
// the slice-local voxel.  Voxels over VECKM_MAX_VOXEL_EVENTS are caught by
// k_pairs, which reads every count once.
template <bool ADD>
__global__ void k_scatter(const int4* __restrict__ ev, Batch bt, int32_t* __restrict__ count,
                          int32_t* __restrict__ vox, int32_t* __restrict__ err) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= bt.n) return;
  const SliceDesc s = slice_by_event(bt, i);
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
__global__ void k_pairs(Batch bt, const int32_t* __restrict__ count, uint32_t* __restrict__ pairs,
                        int32_t* __restrict__ err) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < bt.npairs; g += stride) {
    int64_t poff = 0, voff = 0;
    int W = bt.s0.W;
    if (bt.nslices > 1) {
      int lo = 0, hi = bt.nslices - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (bt.table[mid].pair_off <= g) lo = mid; else hi = mid - 1;
      }
      poff = bt.table[lo].pair_off;
      voff = bt.table[lo].grid_off;
      W = bt.table[lo].W;
    }
    const int64_t p = g - poff;
    const int64_t row = p / (W + 1);
    const int x = (int)(p - row * (W + 1)) - 1;
    const int32_t* c = count + voff + row * W;
    const int cx = x >= 0 ? c[x] : 0;
    if (cx > VECKM_MAX_VOXEL_EVENTS) atomicOr(err, kErrOverflow);
    const uint32_t lo16 = __half_as_ushort(__float2half((float)cx));
    const uint32_t hi16 = x + 1 < W ? __half_as_ushort(__float2half((float)c[x + 1])) : 0u;
    pairs[g] = lo16 | (hi16 << 16);
  }
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

// One block per brick: number the brick's query voxels in (t, y, x) order.
// rank[v] gets the brick-local number, ulist[brick][number] the brick-local
// voxel index, brick_nq[brick] the total.
template <bool ALL>
__global__ __launch_bounds__(256) void k_rank(Batch bt, Brick b, const int32_t* __restrict__ count,
                                              const uint8_t* __restrict__ qmark,
                                              int32_t* __restrict__ rank,
                                              int32_t* __restrict__ ulist,
                                              int32_t* __restrict__ brick_nq) {
  __shared__ int wave_tot[4];
  const int gb = blockIdx.x;
  const SliceDesc s = slice_by_brick(bt, gb);
  const int lb = gb - s.brick_off;
  const int bxi = lb % s.nbx, byi = (lb / s.nbx) % s.nby, bti = lb / (s.nbx * s.nby);
  const int BV = b.bx * b.by * b.bt;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int base = 0;
  for (int it = 0; it < BV; it += 256) {
    const int li = it + threadIdx.x;
    bool flag = false;
    int64_t v = 0;
    if (li < BV) {
      const int lx = li % b.bx, ly = (li / b.bx) % b.by, lt = li / (b.bx * b.by);
      const int x = bxi * b.bx + lx, y = byi * b.by + ly, t = bti * b.bt + lt;
      if (x < s.W && y < s.H && t < s.T) {
        v = s.grid_off + (t * s.H + y) * s.W + x;
        flag = ALL ? (count[v] > 0) : (qmark[v] != 0);
      }
    }
    const unsigned long long bal = __ballot(flag);
    const int pre = __popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0) wave_tot[wid] = __popcll(bal);
    __syncthreads();
    int woff = 0;
    for (int w = 0; w < wid; ++w) woff += wave_tot[w];
    const int tot = wave_tot[0] + wave_tot[1] + wave_tot[2] + wave_tot[3];
    if (flag) {
      const int r = base + woff + pre;
      rank[v] = r;
      ulist[(int64_t)gb * BV + r] = li;
    }
    base += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) brick_nq[gb] = base;
}

// One block: exclusive scan of the per-brick row counts; plan[0] = total
// rows U, plan[1] = 0 (the encoder's work counter), plan[2] = number of
// non-empty bricks, listed in order[] with the most encoder chunks first
// (longest job first keeps the persistent encoder's tail short).
constexpr int kMaxChunkBins = 64;

__global__ __launch_bounds__(1024) void k_brick_scan(const int32_t* __restrict__ nq, int nb,
                                                     int ch, int32_t* __restrict__ off,
                                                     int32_t* __restrict__ order,
                                                     int32_t* __restrict__ plan) {
  __shared__ int sums[1024];
  __shared__ int hist[kMaxChunkBins + 1];
  const int tid = threadIdx.x;
  if (tid <= kMaxChunkBins) hist[tid] = 0;
  const int per = (nb + 1023) / 1024;
  const int s0 = min(tid * per, nb), s1 = min(s0 + per, nb);
  int local = 0;
  for (int i = s0; i < s1; ++i) local += nq[i];
  sums[tid] = local;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {
    const int v = tid >= d ? sums[tid - d] : 0;
    __syncthreads();
    sums[tid] += v;
    __syncthreads();
  }
  int run = tid ? sums[tid - 1] : 0;
  for (int i = s0; i < s1; ++i) {
    off[i] = run;
    run += nq[i];
    const int c = min((nq[i] + ch - 1) / ch, kMaxChunkBins);
    if (c > 0) atomicAdd(&hist[kMaxChunkBins - c], 1);
  }
  __syncthreads();
  if (tid == 0) {
    int acc = 0;
    for (int b = 0; b <= kMaxChunkBins; ++b) {
      const int h = hist[b];
      hist[b] = acc;
      acc += h;
    }
    off[nb] = sums[1023];
    plan[0] = sums[1023];
    plan[1] = 0;
    plan[2] = acc;
  }
  __syncthreads();
  for (int i = s0; i < s1; ++i) {
    const int c = min((nq[i] + ch - 1) / ch, kMaxChunkBins);
    if (c > 0) order[atomicAdd(&hist[kMaxChunkBins - c], 1)] = i;
  }
}

// One thread per query: the row of its voxel (or -1 for an invalid event).
__global__ void k_qmap(const int32_t* __restrict__ queries, Batch bt, Brick b,
                       const int32_t* __restrict__ vox, const int32_t* __restrict__ rank,
                       const int32_t* __restrict__ brick_off, int32_t* __restrict__ qmap,
                       int32_t* __restrict__ rowvox) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= bt.m) return;
  const int e = queries ? queries[i] : i;
  if (e < 0 || e >= bt.n) {
    qmap[i] = -1;
    return;
  }
  const int v = vox[e];
  if (v < 0) {
    qmap[i] = -1;
    return;
  }
  const SliceDesc s = slice_by_event(bt, e);
  const int x = v % s.W, y = (v / s.W) % s.H, t = v / (s.W * s.H);
  const int lb = ((t / b.bt) * s.nby + y / b.by) * s.nbx + x / b.bx;
  const int r = brick_off[s.brick_off + lb] + rank[s.grid_off + v];
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

static int blocks_for(int64_t n, int per) { return (int)((n + per - 1) / per); }

static int fill_grid(int64_t n) {
  int64_t b = (n + 255) / 256;
  return (int)(b < 8192 ? (b < 1 ? 1 : b) : 8192);
}

int launch_prepare(const Batch& bt, const Workspace& w, const veckm_event* ev,
                   const int32_t* queries, const EncodeTables& et, bool pairs, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_fill_i32, dim3(fill_grid(bt.nvox)), dim3(256), 0, s, w.count, bt.nvox, 0);
  if (queries)
    hipLaunchKernelGGL(k_fill_u8, dim3(fill_grid(bt.nvox)), dim3(256), 0, s, w.qmark, bt.nvox);
  if (bt.n > 0)
    hipLaunchKernelGGL(k_scatter<true>, dim3(blocks_for(bt.n, 256)), dim3(256), 0, s,
                       reinterpret_cast<const int4*>(ev), bt, w.count, w.vox, w.err);
  if (pairs)
    hipLaunchKernelGGL(k_pairs, dim3(fill_grid(bt.npairs)), dim3(256), 0, s, bt, w.count, w.pairs,
                       w.err);
  if (queries && bt.m > 0)
    hipLaunchKernelGGL(k_mark, dim3(blocks_for(bt.m, 256)), dim3(256), 0, s, queries, bt, w.vox,
                       w.qmark, w.err);
  if (queries)
    hipLaunchKernelGGL(k_rank<false>, dim3(bt.nbricks), dim3(256), 0, s, bt, et.brick, w.count,
                       w.qmark, w.rank, w.ulist, w.brick_nq);
  else
    hipLaunchKernelGGL(k_rank<true>, dim3(bt.nbricks), dim3(256), 0, s, bt, et.brick, w.count,
                       w.qmark, w.rank, w.ulist, w.brick_nq);
  hipLaunchKernelGGL(k_brick_scan, dim3(1), dim3(1024), 0, s, w.brick_nq, bt.nbricks,
                     encode_rows_per_chunk(et.d), w.brick_off, w.order, w.plan);
  if (bt.m > 0)
    hipLaunchKernelGGL(k_qmap, dim3(blocks_for(bt.m, 256)), dim3(256), 0, s, queries, bt,
                       et.brick, w.vox, w.rank, w.brick_off, w.qmap,
                       pairs ? nullptr : w.rowvox);
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
      pb.nslices = 1;
      pb.npairs = sp[1] * pplane;
      hipLaunchKernelGGL(k_pairs, dim3(fill_grid(pb.npairs)), dim3(256), 0, s, pb,
                         w.count + sp[0] * plane, w.pairs + sp[0] * pplane, w.err);
    }
  return hipGetLastError() == hipSuccess ? VECKM_OK : VECKM_E_HIP;
}

int launch_window_prepare(const Batch& bt, const Workspace& w, const veckm_event* queries,
                          const EncodeTables& et, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_fill_u8, dim3(fill_grid(bt.nvox)), dim3(256), 0, s, w.qmark, bt.nvox);
  if (bt.n > 0) {
    hipLaunchKernelGGL(k_scatter<false>, dim3(blocks_for(bt.n, 256)), dim3(256), 0, s,
                       reinterpret_cast<const int4*>(queries), bt, w.count, w.vox, w.err);
    hipLaunchKernelGGL(k_mark, dim3(blocks_for(bt.m, 256)), dim3(256), 0, s, nullptr, bt, w.vox,
                       w.qmark, w.err);
  }
  hipLaunchKernelGGL(k_rank<false>, dim3(bt.nbricks), dim3(256), 0, s, bt, et.brick, w.count,
                     w.qmark, w.rank, w.ulist, w.brick_nq);
  hipLaunchKernelGGL(k_brick_scan, dim3(1), dim3(1024), 0, s, w.brick_nq, bt.nbricks,
                     encode_rows_per_chunk(et.d), w.brick_off, w.order, w.plan);
  if (bt.m > 0)
    hipLaunchKernelGGL(k_qmap, dim3(blocks_for(bt.m, 256)), dim3(256), 0, s, nullptr, bt,
                       et.brick, w.vox, w.rank, w.brick_off, w.qmap, nullptr);
  return hipGetLastError() == hipSuccess ? VECKM_OK : VECKM_E_HIP;
}

int launch_take_err(const Workspace& w, int32_t* host, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  if (hipMemcpyAsync(host, w.err, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess)
    return VECKM_E_HIP;
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, w.err, (int64_t)1, 0);
  return hipGetLastError() == hipSuccess ? VECKM_OK : VECKM_E_HIP;
}

int launch_expand_emb(const Batch& bt, const Workspace& w, int d, float* emb, void* stream) {
  if (bt.m <= 0) return VECKM_OK;
  hipLaunchKernelGGL(k_expand_emb, dim3(blocks_for((int64_t)bt.m * 64, 256)), dim3(256), 0,
                     (hipStream_t)stream, w.qmap, bt.m, static_cast<const float*>(w.rows), 2 * d,
                     emb);
  return hipGetLastError() == hipSuccess ? VECKM_OK : VECKM_E_HIP;
}

int launch_expand_flow(const Batch& bt, const Workspace& w, float* flow, void* stream) {
  if (bt.m <= 0) return VECKM_OK;
  hipLaunchKernelGGL(k_expand_flow, dim3(blocks_for(bt.m, 256)), dim3(256), 0,
                     (hipStream_t)stream, w.qmap, bt.m,
                     reinterpret_cast<const float2*>(w.rowflow), reinterpret_cast<float2*>(flow));
  return hipGetLastError() == hipSuccess ? VECKM_OK : VECKM_E_HIP;
}

}  // namespace veckm
