// The encoder of the paper's own neighbourhood (Eqn. 1 as written: every
// event of the slice within the spatial window, with no temporal bound), in
// the staged form of Algorithm 1 and Eqns. 14-17.  With q = (x, y) the pixel
// of the query and p = (x', y') a pixel of its window, Algorithm 1 computes
//
//   emb_j = e^{-i A_t[j] t_q} / N(q) * sum_p PixelEmbed_j(p) e^{i (A_x[j] (x' - x) + A_y[j] (y' - y))}
//
// with PixelEmbed_j(p) = sum of e^{i A_t[j] t_k} over the events at p (Eqn. 14)
// and N(q) the event count of the window (Eqns. 15, 17).  The spatial offset
// phase factors into e^{i(A_x x' + A_y y')} e^{-i(A_x x + A_y y)}, so here
//
//   G_j(p)   = e^{i (A_x[j] x' + A_y[j] y')} PixelEmbed_j(p)      (k_tphase)
//   S_j(q)   = e^{-i (A_x[j] x + A_y[j] y)}
//              * sum_{|dx|<=rx, |dy|<=ry} G_j(q + (dx, dy))        (k_pool2d: a plain box sum)
//   emb_j(q) = S_j(q) e^{-i A_t[j] t_q} / N(q)                     (k_paper_rows)
//
// which is the same sum with every term's phase taken relative to the query:
// each term still carries one rounded phase of modulus one, and the box sum
// is a direct (2r + 1)-tap sum per axis (no running sums, so no cancellation),
// but it costs two adds per tap instead of a complex multiply-add.  Time is
// in integer bins, so PixelEmbed is a contraction of the per-pixel bin counts
// with a temporal phase table.  All phase tables are FP64 on the host,
// rounded to fp32; all sums are fp32.  N is the same separable box sum over
// the counts.  Events sharing a voxel (pixel and bin) share their encoding:
// rows are computed per query voxel and numbered like the main encoder's, so
// the perceptron and the per-query expansion are shared.
#include <hip/hip_runtime.h>

#include <utility>

#include "veckm_internal.h"

namespace veckm {

constexpr int kPF = 16;       // frequencies per group of the blocked pixel grids
constexpr int kPoolW = 32;    // pixels per tile row of the window pass
constexpr int kXcds = 8;      // workgroups are dealt round-robin to the 8 XCDs (own L2 each)
constexpr int kPoolThreads = 256;
constexpr int kStageF2 = (kPoolW + 2 * kMaxRxy) * kPF;  // complex values of one staged row
constexpr int kPoolMaxTY = 128;  // output rows per column tile, at most

// Blocked pixel grids (G and S): [D / kPF][H][W][kPF] complex (re, im
// interleaved), so that one group of one pixel is one 128-byte line and one
// tile row of one group is a contiguous run.

__device__ inline uint16_t bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ inline float2 cmul(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}

// a * conj(b)
__device__ inline float2 cmulc(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, a.y * b.y), fmaf(a.y, b.x, -a.x * b.y));
}

// G per pixel: thread per (pixel, chunk of CF frequencies).  The chunks of
// one pixel run go to the same XCD (block b runs on XCD b mod 8), so they
// share the count reads in its L2.  Most voxels are empty, and the loop skips
// them.  Chunk 0 also writes the pixel's event count.
template <int CF>
__global__ __launch_bounds__(256) void k_tphase(int W, int V2, int T, int D, int npb,
                                                const int32_t* __restrict__ count,
                                                const float2* __restrict__ ttab,
                                                const float2* __restrict__ xtab,
                                                const float2* __restrict__ ytab,
                                                float4* __restrict__ G, int32_t* __restrict__ cnt2) {
  const int nc = D / CF;
  const int i = blockIdx.x / kXcds;
  const int ch = i % nc;
  const int pb = (i / nc) * kXcds + blockIdx.x % kXcds;  // pixel block
  if (pb >= npb) return;
  const int p = pb * blockDim.x + threadIdx.x;
  if (p >= V2) return;
  float re[CF], im[CF];
#pragma unroll
  for (int f = 0; f < CF; ++f) re[f] = im[f] = 0.f;
  int n = 0;
  for (int tb = 0; tb < T; tb += 8) {
    int cs[8];  // eight bins' counts fetched together
#pragma unroll
    for (int u = 0; u < 8; ++u) cs[u] = tb + u < T ? count[(int64_t)(tb + u) * V2 + p] : 0;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int c = cs[u];
      if (c == 0) continue;
      n += c;
      const float cf = (float)c;
      const float4* e = reinterpret_cast<const float4*>(ttab + (int64_t)(tb + u) * D + ch * CF);
#pragma unroll
      for (int q = 0; q < CF / 2; ++q) {
        const float4 w = e[q];  // (cos, sin) of two frequencies
        re[2 * q] = fmaf(cf, w.x, re[2 * q]);
        im[2 * q] = fmaf(cf, w.y, im[2 * q]);
        re[2 * q + 1] = fmaf(cf, w.z, re[2 * q + 1]);
        im[2 * q + 1] = fmaf(cf, w.w, im[2 * q + 1]);
      }
    }
  }
  const int x = p % W, y = p / W;
  const float2* ex = xtab + (int64_t)x * D + ch * CF;
  const float2* ey = ytab + (int64_t)y * D + ch * CF;
#pragma unroll
  for (int gg = 0; gg < CF / kPF; ++gg) {
    float4* dst = G + ((int64_t)(ch * (CF / kPF) + gg) * V2 + p) * (kPF / 2);
#pragma unroll
    for (int q = 0; q < kPF / 2; ++q) {
      const int f = gg * kPF + 2 * q;
      const float2 a = cmul(make_float2(re[f], im[f]), cmul(ex[f], ey[f]));
      const float2 b = cmul(make_float2(re[f + 1], im[f + 1]), cmul(ex[f + 1], ey[f + 1]));
      dst[q] = make_float4(a.x, a.y, b.x, b.y);
    }
  }
  if (ch == 0) cnt2[p] = n;
}

__device__ inline float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }

// The window box sum of G as an x pass and a y pass in one kernel.  A block
// owns a 64-pixel-wide column tile of TY output rows for one frequency group
// and walks down it: each step stages the next input row (with the x halo,
// zero outside the image) in LDS, takes its x sum, and keeps it in a register
// ring of the last 2 RY + 1 rows; the y sum over the ring gives one output
// row, turned back by the output pixel's conjugate spatial phase.  Thread t
// owns frequency t % 16 of pixels (t / 16) % 16 and that + 16.
template <int RY>
__global__ __launch_bounds__(kPoolThreads) void k_pool2d(int W, int H, int D, int rx, int TY,
                                                         int ng, int nxt,
                                                         const float4* __restrict__ G,
                                                         const float2* __restrict__ xtab,
                                                         const float2* __restrict__ ytab,
                                                         float2* __restrict__ S) {
  constexpr int NR = 2 * RY + 1;
  __shared__ float4 stage[2][kStageF2 / 2];
  __shared__ float2 yph[kPoolMaxTY * kPF];  // y phases of the output rows
  const int g = blockIdx.x % ng;
  const int xt = (blockIdx.x / ng) % nxt;
  const int yt = blockIdx.x / (ng * nxt);
  const int x0 = xt * kPoolW, y0 = yt * TY;
  const int y1 = min(y0 + TY, H);
  const int tid = threadIdx.x;
  const int f = tid & (kPF - 1);
  const int px = (tid >> 4) & 15;
  const int64_t V2 = (int64_t)W * H;
  const float4* Gg = G + (int64_t)g * V2 * (kPF / 2);
  float2* Sg = S + (int64_t)g * V2 * kPF;
  const int j = g * kPF + f;
  // x phases of the thread's two columns (fixed along the walk)
  const float2 cx0 = x0 + px < W ? xtab[(int64_t)(x0 + px) * D + j] : make_float2(1.f, 0.f);
  const float2 cx1 = x0 + px + 16 < W ? xtab[(int64_t)(x0 + px + 16) * D + j] : make_float2(1.f, 0.f);
  for (int i = tid; i < (y1 - y0) * kPF; i += kPoolThreads)
    yph[i] = ytab[(int64_t)(y0 + i / kPF) * D + g * kPF + i % kPF];

  // staged row: (32 + 2 rx) pixels x 8 float4; two loads per thread cover it.
  // The next row is fetched into registers while the current one is used.
  const int seg = (kPoolW + 2 * rx) * (kPF / 2);
  float4 ld[2];
  auto load_row = [&](int yi) {
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int idx = tid + k * kPoolThreads;
      const int x = x0 - rx + idx / (kPF / 2);
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (idx < seg && yi >= 0 && yi < H && x >= 0 && x < W)
        v = Gg[((int64_t)yi * W + x) * (kPF / 2) + idx % (kPF / 2)];
      ld[k] = v;
    }
  };
  // Ring of x sums: input row ybeg + i sits in slot i mod NR.  The loop below
  // is unrolled NR times, so every slot index is a constant.
  float2 h0[NR], h1[NR];
#pragma unroll
  for (int k = 0; k < NR; ++k) h0[k] = h1[k] = make_float2(0.f, 0.f);

  const int ybeg = y0 - RY, yend = y1 + RY;
  load_row(ybeg);
  for (int yb = ybeg; yb < yend; yb += NR) {
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      const int yi = yb + k;
      if (yi < yend) {  // uniform over the block
        float4* st = stage[(yi - ybeg) & 1];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const int idx = tid + q * kPoolThreads;
          if (idx < seg) st[idx] = ld[q];
        }
        __syncthreads();
        if (yi + 1 < yend) load_row(yi + 1);
        // x sum of input row yi (zero outside the image)
        float2 a0 = make_float2(0.f, 0.f), a1 = make_float2(0.f, 0.f);
        if (yi >= 0 && yi < H) {
          const float2* s2 = reinterpret_cast<const float2*>(st);
          for (int m = 0; m <= 2 * rx; ++m) {
            a0 = cadd(a0, s2[(px + m) * kPF + f]);
            a1 = cadd(a1, s2[(px + 16 + m) * kPF + f]);
          }
        }
        h0[k] = a0;
        h1[k] = a1;
        // y sum: output row yi - RY reads rows yi - 2 RY .. yi, which sit in
        // slots k + 1 .. k + NR (mod NR)
        const int yo = yi - RY;
        if (yo >= y0) {
          float2 s0 = h0[(k + 1) % NR], s1 = h1[(k + 1) % NR];
#pragma unroll
          for (int m = 1; m < NR; ++m) {
            s0 = cadd(s0, h0[(k + 1 + m) % NR]);
            s1 = cadd(s1, h1[(k + 1 + m) % NR]);
          }
          const float2 ey = yph[(yo - y0) * kPF + f];
          const int64_t row = (int64_t)yo * W;
          if (x0 + px < W) Sg[(row + x0 + px) * kPF + f] = cmulc(s0, cmul(cx0, ey));
          if (x0 + px + 16 < W) Sg[(row + x0 + px + 16) * kPF + f] = cmulc(s1, cmul(cx1, ey));
        }
      }
    }
  }
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

// The rows of the query voxels, row = S(q) e^{-i A_t t} / N(q): D / 4 lanes
// per row, each with four consecutive frequencies; every lane group takes two
// rows.  Rows past the device-side row count plan[0] are skipped.
template <bool BF16>
__global__ __launch_bounds__(256) void k_paper_rows(int W, int H, int D,
                                                    const int32_t* __restrict__ plan,
                                                    const int32_t* __restrict__ rowvox,
                                                    const float2* __restrict__ S,
                                                    const int32_t* __restrict__ nbox,
                                                    const float2* __restrict__ ttab,
                                                    void* __restrict__ rows) {
  const int U = plan[0];
  const int64_t V2 = (int64_t)W * H;
  const int L = D / 4;              // lanes per row
  const int rpw = 64 / L;           // row groups per wave
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int sub = lane / L, k = lane % L;
  if (sub >= rpw) return;
  const int groups = 4 * rpw;       // row groups per block
  const int j = 4 * k;
  const int g = j / kPF, jo = j % kPF;
  auto row = [&](int r) {
    const int v = rowvox[r];
    const int64_t p = v % V2;
    const int t = (int)(v / V2);
    const float inv = 1.f / (float)nbox[p];
    const float4* sp = reinterpret_cast<const float4*>(S + ((int64_t)g * V2 + p) * kPF + jo);
    const float4* et = reinterpret_cast<const float4*>(ttab + (int64_t)t * D + j);
    const float4 sa = sp[0], sb = sp[1];  // (re, im) of frequencies j .. j + 3
    const float4 ea = et[0], eb = et[1];
    // multiplied by the conjugate temporal phase
    const float re[4] = {fmaf(sa.x, ea.x, sa.y * ea.y) * inv, fmaf(sa.z, ea.z, sa.w * ea.w) * inv,
                         fmaf(sb.x, eb.x, sb.y * eb.y) * inv, fmaf(sb.z, eb.z, sb.w * eb.w) * inv};
    const float im[4] = {fmaf(sa.y, ea.x, -sa.x * ea.y) * inv, fmaf(sa.w, ea.z, -sa.z * ea.w) * inv,
                         fmaf(sb.y, eb.x, -sb.x * eb.y) * inv, fmaf(sb.w, eb.z, -sb.z * eb.w) * inv};
    const int64_t u = (int64_t)r * 2 * D;
    if constexpr (BF16) {
      uint16_t* out = static_cast<uint16_t*>(rows);
      const uint2 vr = make_uint2(bf16_rne(re[0]) | ((uint32_t)bf16_rne(re[1]) << 16),
                                  bf16_rne(re[2]) | ((uint32_t)bf16_rne(re[3]) << 16));
      const uint2 vi = make_uint2(bf16_rne(im[0]) | ((uint32_t)bf16_rne(im[1]) << 16),
                                  bf16_rne(im[2]) | ((uint32_t)bf16_rne(im[3]) << 16));
      *reinterpret_cast<uint2*>(out + u + j) = vr;
      *reinterpret_cast<uint2*>(out + u + D + j) = vi;
    } else {
      float* out = static_cast<float*>(rows);
      *reinterpret_cast<float4*>(out + u + j) = make_float4(re[0], re[1], re[2], re[3]);
      *reinterpret_cast<float4*>(out + u + D + j) = make_float4(im[0], im[1], im[2], im[3]);
    }
  };
  const int r0 = blockIdx.x * 2 * groups + wid * rpw + sub;
  if (r0 < U) row(r0);
  if (r0 + groups < U) row(r0 + groups);
}

static int blocks(int64_t n, int per) { return (int)((n + per - 1) / per); }

template <int RY>
static void launch_pool(int W, int H, int D, int rx, int TY, int ng, int nxt, const float4* G,
                        const float2* xtab, const float2* ytab, float2* S, hipStream_t s) {
  const int nyt = (H + TY - 1) / TY;
  hipLaunchKernelGGL(k_pool2d<RY>, dim3(ng * nxt * nyt), dim3(kPoolThreads), 0, s, W, H, D, rx,
                     TY, ng, nxt, G, xtab, ytab, S);
}

using PoolFn = void (*)(int, int, int, int, int, int, int, const float4*, const float2*,
                        const float2*, float2*, hipStream_t);

template <int... R>
static PoolFn pool_for(int ry, std::integer_sequence<int, R...>) {
  PoolFn fns[] = {&launch_pool<R>...};
  return fns[ry];
}

int launch_paper_encode(const Batch& bt, const Workspace& w, const PaperTables& pt,
                        const Brick& brick, int rows, int num_cus, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  const SliceDesc& sl = bt.s0;
  const int64_t V2 = (int64_t)sl.W * sl.H;
  const int D = pt.d;
  if (bt.nslices != 1 || D % kPF || pt.rx > kMaxRxy || pt.ry > kMaxRxy || pt.rx < 0 || pt.ry < 0)
    return VECKM_E_INVAL;
  const int ng = D / kPF;
  const float2* ttab = reinterpret_cast<const float2*>(pt.ttab);
  const float2* xtab = reinterpret_cast<const float2*>(pt.xtab);
  const float2* ytab = reinterpret_cast<const float2*>(pt.ytab);
  float4* G4 = reinterpret_cast<float4*>(w.G);
  const int npb = blocks(V2, 256);
  hipLaunchKernelGGL(k_tphase<kPF>, dim3(blocks(npb, kXcds) * kXcds * (D / kPF)), dim3(256), 0, s,
                     sl.W, (int)V2, sl.T, D, npb, w.count, ttab, xtab, ytab, G4, w.cnt2);
  // column tiles: enough blocks for about three per compute unit
  const int nxt = (sl.W + kPoolW - 1) / kPoolW;
  const int want = 3 * num_cus;
  int nyt = (want + ng * nxt - 1) / (ng * nxt);
  nyt = nyt < 1 ? 1 : (nyt > sl.H ? sl.H : nyt);
  nyt = nyt < (sl.H + kPoolMaxTY - 1) / kPoolMaxTY ? (sl.H + kPoolMaxTY - 1) / kPoolMaxTY : nyt;
  const int TY = (sl.H + nyt - 1) / nyt;
  pool_for(pt.ry, std::make_integer_sequence<int, kMaxRxy + 1>{})(
      sl.W, sl.H, D, pt.rx, TY, ng, nxt, G4, xtab, ytab, reinterpret_cast<float2*>(w.S), s);
  hipLaunchKernelGGL(k_boxx, dim3(blocks(V2, 256)), dim3(256), 0, s, sl.W, sl.H, pt.rx, w.cnt2,
                     w.nbx);
  hipLaunchKernelGGL(k_boxy, dim3(blocks(V2, 256)), dim3(256), 0, s, sl.W, sl.H, pt.ry, w.nbx,
                     w.nbox);
  // rows: at most one per query (the row count itself is on the device)
  const float2* S = reinterpret_cast<const float2*>(w.S);
  const int per_block = 2 * 4 * (64 / (D / 4));
  if (bt.m > 0) {
    if (rows == kRowsBF16)
      hipLaunchKernelGGL(k_paper_rows<true>, dim3(blocks(bt.m, per_block)), dim3(256), 0, s, sl.W,
                         sl.H, D, w.plan, w.rowvox, S, w.nbox, ttab, w.rows);
    else
      hipLaunchKernelGGL(k_paper_rows<false>, dim3(blocks(bt.m, per_block)), dim3(256), 0, s,
                         sl.W, sl.H, D, w.plan, w.rowvox, S, w.nbox, ttab, w.rows);
  }
  return hipGetLastError() == hipSuccess ? VECKM_OK : VECKM_E_HIP;
}

}  // namespace veckm
