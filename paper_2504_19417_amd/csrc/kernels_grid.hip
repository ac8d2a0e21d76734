// Front end of the encoder: validate and bin events into an integer
// (x, y, t) count grid, rank the voxels that carry queries, and map queries
// to their voxel's row; plus the back-end expansion of per-voxel rows to
// per-query outputs.
//
// All events that share a voxel have the same offset to every neighbour, so
// the scatter of Algorithm 1 (PixelEmbed/PixelCount, Eqns. 14-15) reduces
// to an exact integer histogram; the phases are applied afterwards by the
// encoder contraction.  All queries that share a voxel get the same encoding
// (Sec. 2.1: the encoding depends on the event's position and time only), so
// the encoder computes one row per distinct query voxel and the rows are
// copied out per query.
#include <hip/hip_runtime.h>

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

// One thread per event: validate, histogram, remember the voxel.
__global__ void k_scatter(const int4* __restrict__ ev, SliceGeom g, int32_t* __restrict__ count,
                          int32_t* __restrict__ vox, int32_t* __restrict__ err) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.n) return;
  const int4 e = ev[i];
  const int64_t dt = (int64_t)e.z - (int64_t)g.t0;
  const bool ok = e.x >= 0 && e.x < g.W && e.y >= 0 && e.y < g.H && dt >= 0 && dt < g.T &&
                  (e.w == 1 || e.w == -1);
  if (!ok) {
    atomicOr(err, kErrRange);
    vox[i] = -1;
    return;
  }
  const int v = ((int)dt * g.H + e.y) * g.W + e.x;
  const int old = atomicAdd(&count[v], 1);
  if (old == VECKM_MAX_VOXEL_EVENTS) atomicOr(err, kErrOverflow);
  vox[i] = v;
}

// Query subsets: mark the voxels that carry at least one query.
__global__ void k_mark(const int32_t* __restrict__ queries, SliceGeom g,
                       const int32_t* __restrict__ vox, uint8_t* __restrict__ qmark,
                       int32_t* __restrict__ err) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.m) return;
  const int q = queries[i];
  if (q < 0 || q >= g.n) {
    atomicOr(err, kErrQuery);
    return;
  }
  const int v = vox[q];
  if (v >= 0) qmark[v] = 1;
}

// One block per brick: number the brick's query voxels in (t, y, x) order.
// rank[v] gets the brick-local number, ulist[brick][number] the brick-local
// voxel index, brick_nq[brick] the total.
template <bool ALL>
__global__ __launch_bounds__(256) void k_rank(SliceGeom g, Brick b,
                                              const int32_t* __restrict__ count,
                                              const uint8_t* __restrict__ qmark,
                                              int32_t* __restrict__ rank,
                                              int32_t* __restrict__ ulist,
                                              int32_t* __restrict__ brick_nq) {
  __shared__ int wave_tot[4];
  const int bid = blockIdx.x;
  const int bxi = bid % g.nbx, byi = (bid / g.nbx) % g.nby, bti = bid / (g.nbx * g.nby);
  const int BV = b.bx * b.by * b.bt;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int base = 0;
  for (int it = 0; it < BV; it += 256) {
    const int li = it + threadIdx.x;
    bool flag = false;
    int v = 0;
    if (li < BV) {
      const int lx = li % b.bx, ly = (li / b.bx) % b.by, lt = li / (b.bx * b.by);
      const int x = bxi * b.bx + lx, y = byi * b.by + ly, t = bti * b.bt + lt;
      if (x < g.W && y < g.H && t < g.T) {
        v = (t * g.H + y) * g.W + x;
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
      ulist[(int64_t)bid * BV + r] = li;
    }
    base += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) brick_nq[bid] = base;
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
__global__ void k_qmap(const int32_t* __restrict__ queries, SliceGeom g, Brick b,
                       const int32_t* __restrict__ vox, const int32_t* __restrict__ rank,
                       const int32_t* __restrict__ brick_off, int32_t* __restrict__ qmap) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.m) return;
  const int e = queries ? queries[i] : i;
  if (e < 0 || e >= g.n) {
    qmap[i] = -1;
    return;
  }
  const int v = vox[e];
  if (v < 0) {
    qmap[i] = -1;
    return;
  }
  const int x = v % g.W, y = (v / g.W) % g.H, t = v / (g.W * g.H);
  const int bid = ((t / b.bt) * g.nby + y / b.by) * g.nbx + x / b.bx;
  qmap[i] = brick_off[bid] + rank[v];
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

int launch_prepare(const SliceGeom& g, const Workspace& w, const veckm_event* ev,
                   const int32_t* queries, const EncodeTables& et, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  const int64_t V = (int64_t)g.W * g.H * g.T;
  hipLaunchKernelGGL(k_fill_i32, dim3(fill_grid(V)), dim3(256), 0, s, w.count, V, 0);
  if (queries) hipLaunchKernelGGL(k_fill_u8, dim3(fill_grid(V)), dim3(256), 0, s, w.qmark, V);
  if (g.n > 0)
    hipLaunchKernelGGL(k_scatter, dim3(blocks_for(g.n, 256)), dim3(256), 0, s,
                       reinterpret_cast<const int4*>(ev), g, w.count, w.vox, w.err);
  if (queries && g.m > 0)
    hipLaunchKernelGGL(k_mark, dim3(blocks_for(g.m, 256)), dim3(256), 0, s, queries, g, w.vox,
                       w.qmark, w.err);
  if (queries)
    hipLaunchKernelGGL(k_rank<false>, dim3(g.nbricks), dim3(256), 0, s, g, et.brick, w.count,
                       w.qmark, w.rank, w.ulist, w.brick_nq);
  else
    hipLaunchKernelGGL(k_rank<true>, dim3(g.nbricks), dim3(256), 0, s, g, et.brick, w.count,
                       w.qmark, w.rank, w.ulist, w.brick_nq);
  hipLaunchKernelGGL(k_brick_scan, dim3(1), dim3(1024), 0, s, w.brick_nq, g.nbricks,
                     encode_rows_per_chunk(et.d), w.brick_off, w.order, w.plan);
  if (g.m > 0)
    hipLaunchKernelGGL(k_qmap, dim3(blocks_for(g.m, 256)), dim3(256), 0, s, queries, g,
                       et.brick, w.vox, w.rank, w.brick_off, w.qmap);
  return hipGetLastError() == hipSuccess ? VECKM_OK : VECKM_E_HIP;
}

int launch_expand_emb(const SliceGeom& g, const Workspace& w, int d, float* emb, void* stream) {
  if (g.m <= 0) return VECKM_OK;
  hipLaunchKernelGGL(k_expand_emb, dim3(blocks_for((int64_t)g.m * 64, 256)), dim3(256), 0,
                     (hipStream_t)stream, w.qmap, g.m, static_cast<const float*>(w.rows), 2 * d,
                     emb);
  return hipGetLastError() == hipSuccess ? VECKM_OK : VECKM_E_HIP;
}

int launch_expand_flow(const SliceGeom& g, const Workspace& w, float* flow, void* stream) {
  if (g.m <= 0) return VECKM_OK;
  hipLaunchKernelGGL(k_expand_flow, dim3(blocks_for(g.m, 256)), dim3(256), 0,
                     (hipStream_t)stream, w.qmap, g.m,
                     reinterpret_cast<const float2*>(w.rowflow), reinterpret_cast<float2*>(flow));
  return hipGetLastError() == hipSuccess ? VECKM_OK : VECKM_E_HIP;
}

}  // namespace veckm
