// The encoder of the paper's own neighbourhood (Eqn. 1 as written: every
// event of the slice within the spatial window, with no temporal bound), in
// the staged form of Algorithm 1 and Eqns. 14-17:
//
//   G_j(p)  = sum over events k at pixel p of e^{i A_t[j] t_k}    (PixelEmbed, Eqn. 14)
//   c(p)    = number of events at pixel p                          (PixelCount, Eqn. 15)
//   S_j(p)  = sum_{|dx|<=rx, |dy|<=ry} G_j(p + (dx, dy)) e^{i (A_x[j] dx + A_y[j] dy)}   (Eqn. 16)
//   N(p)    = sum_{|dx|<=rx, |dy|<=ry} c(p + (dx, dy))                                  (Eqn. 17)
//   emb_j(k) = S_j(p_k) e^{-i A_t[j] t_k} / N(p_k)                (Algorithm 1, final step)
//
// Time is in integer bins, so G is a contraction of the per-pixel bin counts
// with a temporal phase table (FP64 on the host).  The spatial factor
// e^{i(A_x dx + A_y dy)} splits into an x and a y factor, so the window sum
// is two 1-D complex passes (x, then y) over the pixel grid, each a coalesced
// sweep; N is the same separable box sum over the counts.  Events sharing a
// voxel (pixel and bin) share their encoding: rows are computed per query
// voxel and numbered like the main encoder's, so the perceptron and the
// per-query expansion are shared.
//
// Layouts: G and the x-pass result are planar ([2D][H][W]: the Re planes of
// all frequencies, then the Im planes) so that every pass reads and writes
// along x; S is pixel-major ([H][W][2D]) so that a row is one contiguous read.
#include <hip/hip_runtime.h>

#include "slices.h"
#include "veckm_internal.h"

namespace veckm {

constexpr int kTpCh = 16;  // complex channels per thread in k_tphase

__device__ inline uint16_t bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// G and c per pixel (thread per pixel and group of kTpCh frequencies).
__global__ __launch_bounds__(256) void k_tphase(int V2, int T, int D,
                                                const int32_t* __restrict__ count,
                                                const float2* __restrict__ ttab,
                                                float* __restrict__ G, int32_t* __restrict__ cnt2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const int j0 = blockIdx.y * kTpCh;
  if (p >= V2) return;
  float re[kTpCh], im[kTpCh];
#pragma unroll
  for (int jj = 0; jj < kTpCh; ++jj) re[jj] = im[jj] = 0.f;
  int n = 0;
  for (int t = 0; t < T; ++t) {
    const int c = count[(int64_t)t * V2 + p];
    if (c == 0) continue;
    n += c;
    const float cf = (float)c;
    const float2* e = ttab + (int64_t)t * D + j0;
#pragma unroll
    for (int jj = 0; jj < kTpCh; ++jj) {
      const float2 w = e[jj];
      re[jj] = fmaf(cf, w.x, re[jj]);
      im[jj] = fmaf(cf, w.y, im[jj]);
    }
  }
#pragma unroll
  for (int jj = 0; jj < kTpCh; ++jj) {
    G[(int64_t)(j0 + jj) * V2 + p] = re[jj];
    G[(int64_t)(D + j0 + jj) * V2 + p] = im[jj];
  }
  if (blockIdx.y == 0) cnt2[p] = n;
}

// x pass: Hx_j(p) = sum_dx G_j(p + dx) e^{i A_x[j] dx}, zero outside the
// image (thread per pixel, one frequency per grid row).
__global__ __launch_bounds__(256) void k_poolx(int W, int H, int D, int rx,
                                               const float* __restrict__ G,
                                               const float2* __restrict__ pxt,
                                               float* __restrict__ Hx) {
  const int64_t V2 = (int64_t)W * H;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (p >= V2) return;
  const int x = p % W;
  const float* gr = G + (int64_t)j * V2;
  const float* gi = G + (int64_t)(D + j) * V2;
  float sr = 0.f, si = 0.f;
  for (int dx = -rx; dx <= rx; ++dx) {
    if (x + dx < 0 || x + dx >= W) continue;
    const float2 w = pxt[(dx + rx) * D + j];
    const float a = gr[p + dx], b = gi[p + dx];
    sr = fmaf(a, w.x, fmaf(-b, w.y, sr));
    si = fmaf(a, w.y, fmaf(b, w.x, si));
  }
  Hx[(int64_t)j * V2 + p] = sr;
  Hx[(int64_t)(D + j) * V2 + p] = si;
}

// y pass: S_j(p) = sum_dy Hx_j(p + dy W) e^{i A_y[j] dy}.  One block per run
// of 64 pixels of an image row: each wave sweeps a quarter of the
// frequencies with lanes along x, results gather in LDS as pixel-major rows
// (row stride 2D + 1 floats: conflict-free column writes) and leave as one
// contiguous block.
__global__ __launch_bounds__(256) void k_pooly(int W, int H, int D, int ry,
                                               const float* __restrict__ Hx,
                                               const float2* __restrict__ pyt,
                                               float* __restrict__ S) {
  extern __shared__ float tile[];  // [64][2D + 1]
  const int ts = 2 * D + 1;
  const int64_t V2 = (int64_t)W * H;
  const int runs = (W + 63) / 64;
  const int y = blockIdx.x / runs, x0 = (blockIdx.x % runs) * 64;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int x = x0 + lane;
  const bool in = x < W;
  for (int j = wid; j < D; j += 4) {
    const float* hr = Hx + (int64_t)j * V2;
    const float* hi = Hx + (int64_t)(D + j) * V2;
    float sr = 0.f, si = 0.f;
    for (int dy = -ry; dy <= ry; ++dy) {
      const int yy = y + dy;
      if (!in || yy < 0 || yy >= H) continue;
      const float2 w = pyt[(dy + ry) * D + j];
      const int64_t q = (int64_t)yy * W + x;
      const float a = hr[q], b = hi[q];
      sr = fmaf(a, w.x, fmaf(-b, w.y, sr));
      si = fmaf(a, w.y, fmaf(b, w.x, si));
    }
    tile[lane * ts + j] = sr;
    tile[lane * ts + D + j] = si;
  }
  __syncthreads();
  const int np = (W - x0 < 64 ? W - x0 : 64);  // pixels of this run
  float* dst = S + ((int64_t)y * W + x0) * 2 * D;
  for (int i = threadIdx.x; i < np * 2 * D; i += blockDim.x) dst[i] = tile[(i / (2 * D)) * ts + i % (2 * D)];
}

// Box sums of the pixel counts: x pass, then y pass.
__global__ void k_boxx(int W, int H, int rx, const int32_t* __restrict__ c,
                       int32_t* __restrict__ out) {
  const int64_t V2 = (int64_t)W * H;
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= V2) return;
  const int x = (int)(p % W);
  int s = 0;
  for (int dx = -rx; dx <= rx; ++dx)
    if (x + dx >= 0 && x + dx < W) s += c[p + dx];
  out[p] = s;
}

__global__ void k_boxy(int W, int H, int ry, const int32_t* __restrict__ c,
                       int32_t* __restrict__ out) {
  const int64_t V2 = (int64_t)W * H;
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= V2) return;
  const int y = (int)(p / W);
  int s = 0;
  for (int dy = -ry; dy <= ry; ++dy)
    if (y + dy >= 0 && y + dy < H) s += c[p + (int64_t)dy * W];
  out[p] = s;
}

// One block per brick: the rows of the brick's query voxels (numbered as the
// main encoder numbers them), row = S(p) e^{-i A_t t} / N(p), lanes along
// frequencies.
template <bool BF16>
__global__ __launch_bounds__(256) void k_paper_rows(Batch bt, Brick b, int D,
                                                    const int32_t* __restrict__ ulist,
                                                    const int32_t* __restrict__ brick_nq,
                                                    const int32_t* __restrict__ brick_off,
                                                    const float* __restrict__ S,
                                                    const int32_t* __restrict__ nbox,
                                                    const float2* __restrict__ ttab,
                                                    void* __restrict__ rows) {
  const int gb = blockIdx.x;
  const int nq = brick_nq[gb];
  if (nq == 0) return;
  const SliceDesc s = slice_by_brick(bt, gb);
  const int lb = gb - s.brick_off;
  const int bxi = lb % s.nbx, byi = (lb / s.nbx) % s.nby, bti = lb / (s.nbx * s.nby);
  const int BV = b.bx * b.by * b.bt;
  const int row0 = brick_off[gb];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int r = wid; r < nq; r += 4) {
    const int li = ulist[(int64_t)gb * BV + r];
    const int x = bxi * b.bx + li % b.bx;
    const int y = byi * b.by + (li / b.bx) % b.by;
    const int t = bti * b.bt + li / (b.bx * b.by);
    const int64_t p = (int64_t)y * s.W + x;
    const float n = (float)nbox[p];
    const float* sp = S + p * 2 * D;
    const float2* e = ttab + (int64_t)t * D;
    const int64_t u = (int64_t)(row0 + r) * 2 * D;
    for (int j = lane; j < D; j += 64) {
      const float sr = sp[j], si = sp[D + j];
      const float2 w = e[j];  // multiplied by its conjugate
      const float re = fmaf(sr, w.x, si * w.y) / n;
      const float im = fmaf(si, w.x, -sr * w.y) / n;
      if constexpr (BF16) {
        uint16_t* out = static_cast<uint16_t*>(rows);
        out[u + j] = bf16_rne(re);
        out[u + D + j] = bf16_rne(im);
      } else {
        float* out = static_cast<float*>(rows);
        out[u + j] = re;
        out[u + D + j] = im;
      }
    }
  }
}

static int blocks(int64_t n, int per) { return (int)((n + per - 1) / per); }

size_t paper_pooly_lds(int d) { return (size_t)64 * (2 * d + 1) * sizeof(float); }

int launch_paper_encode(const Batch& bt, const Workspace& w, const PaperTables& pt,
                        const Brick& brick, int rows, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  const SliceDesc& sl = bt.s0;
  const int64_t V2 = (int64_t)sl.W * sl.H;
  const int D = pt.d;
  if (D % kTpCh) return VECKM_E_INVAL;
  hipLaunchKernelGGL(k_tphase, dim3(blocks(V2, 256), D / kTpCh), dim3(256), 0, s, (int)V2, sl.T, D,
                     w.count, reinterpret_cast<const float2*>(pt.ttab), w.G, w.cnt2);
  hipLaunchKernelGGL(k_poolx, dim3(blocks(V2, 256), D), dim3(256), 0, s, sl.W, sl.H, D, pt.rx,
                     w.G, reinterpret_cast<const float2*>(pt.pxt), w.Hx);
  const int runs = (sl.W + 63) / 64;
  const size_t lds = paper_pooly_lds(D);
  if (hipFuncSetAttribute(reinterpret_cast<const void*>(&k_pooly),
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return VECKM_E_HIP;
  hipLaunchKernelGGL(k_pooly, dim3(runs * sl.H), dim3(256), lds, s, sl.W, sl.H, D, pt.ry, w.Hx,
                     reinterpret_cast<const float2*>(pt.pyt), w.S);
  hipLaunchKernelGGL(k_boxx, dim3(blocks(V2, 256)), dim3(256), 0, s, sl.W, sl.H, pt.rx, w.cnt2,
                     w.nbx);
  hipLaunchKernelGGL(k_boxy, dim3(blocks(V2, 256)), dim3(256), 0, s, sl.W, sl.H, pt.ry, w.nbx,
                     w.nbox);
  if (rows == kRowsBF16)
    hipLaunchKernelGGL(k_paper_rows<true>, dim3(bt.nbricks), dim3(256), 0, s, bt, brick, D,
                       w.ulist, w.brick_nq, w.brick_off, w.S, w.nbox, reinterpret_cast<const float2*>(pt.ttab), w.rows);
  else
    hipLaunchKernelGGL(k_paper_rows<false>, dim3(bt.nbricks), dim3(256), 0, s, bt, brick, D,
                       w.ulist, w.brick_nq, w.brick_off, w.S, w.nbox, reinterpret_cast<const float2*>(pt.ttab), w.rows);
  return hipGetLastError() == hipSuccess ? VECKM_OK : VECKM_E_HIP;
}

}  // namespace veckm
