// Training the two-layer perceptron of Sec. 2.1 (Eqns. 5-6) on encodings
// with known normal flows.  The paper delegates its loss and sampling to its
// predecessor; the loss here is our own: the mean over rows of the squared
// error of the predicted 2-vector,
//   L = (1/M) sum_r ||W2 relu(W1 x_r + b1) + b2 - y_r||^2,
// with the chain-rule gradients
//   dp_r = 2 (p_r - y_r) / M,  dW2 = sum_r dp_r h_r^T,  db2 = sum_r dp_r,
//   dz_r = (W2^T dp_r) * [z_r > 0],  dW1 = sum_r dz_r x_r^T,  db1 = sum_r dz_r,
// then plain gradient descent or Adam.  Everything is fp32; every reduction
// over rows runs in a fixed order (per-block partial sums, then a serial sum
// over blocks), so a step is deterministic.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "veckm_internal.h"

namespace veckm {

constexpr int kGemmTile = 64;
constexpr int kGemmK = 16;

// C = A B over k in this split's range (blockIdx.z), 64 x 64 output tile per
// block, 4 x 4 outputs per thread, 16-deep k slices staged in LDS.  A(i, k) =
// A[i sai + k sak], B(k, j) = B[k sbk + j sbj]; either stride of each may be
// the unit one (the staging loads follow it).  EPI 1: C[i][j] = relu(acc +
// bias[j]) (one split); EPI 0: the split's partial sums to C + split M N.
template <int EPI>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, int kchunk,
                                              const float* __restrict__ A, int64_t sai,
                                              int64_t sak, const float* __restrict__ B,
                                              int64_t sbk, int64_t sbj,
                                              const float* __restrict__ bias,
                                              float* __restrict__ C) {
  __shared__ __align__(16) float As[kGemmK][kGemmTile + 4];
  __shared__ __align__(16) float Bs[kGemmK][kGemmTile + 4];
  const int tid = threadIdx.x;
  const int i0 = blockIdx.y * kGemmTile, j0 = blockIdx.x * kGemmTile;
  const int kb = blockIdx.z * kchunk;
  const int ke = min(K, kb + kchunk);
  const int ty = tid >> 4, tx = tid & 15;
  float acc[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[r][c] = 0.f;
  const bool a_kfast = sak == 1, b_kfast = sbk == 1;
  for (int k0 = kb; k0 < ke; k0 += kGemmK) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + q * 256;  // 1024 elements of each tile
      const int ii = a_kfast ? e / kGemmK : e % kGemmTile;
      const int ka = a_kfast ? e % kGemmK : e / kGemmTile;
      const int i = i0 + ii, k = k0 + ka;
      As[ka][ii] = (i < M && k < ke) ? A[(int64_t)i * sai + (int64_t)k * sak] : 0.f;
      const int jj = b_kfast ? e / kGemmK : e % kGemmTile;
      const int kbb = b_kfast ? e % kGemmK : e / kGemmTile;
      const int j = j0 + jj, k2 = k0 + kbb;
      Bs[kbb][jj] = (j < N && k2 < ke) ? B[(int64_t)k2 * sbk + (int64_t)j * sbj] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kGemmK; ++kk) {
      const float4 a = *reinterpret_cast<const float4*>(&As[kk][ty * 4]);
      const float4 b = *reinterpret_cast<const float4*>(&Bs[kk][tx * 4]);
      const float av[4] = {a.x, a.y, a.z, a.w}, bv[4] = {b.x, b.y, b.z, b.w};
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[r][c] = fmaf(av[r], bv[c], acc[r][c]);
    }
    __syncthreads();
  }
  float* out = EPI == 1 ? C : C + (int64_t)blockIdx.z * M * N;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = i0 + ty * 4 + r;
    if (i >= M) continue;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int j = j0 + tx * 4 + c;
      if (j >= N) continue;
      float v = acc[r][c];
      if (EPI == 1) v = fmaxf(v + bias[j], 0.f);
      out[(int64_t)i * N + j] = v;
    }
  }
}

// out[c] (+)= sum over b = 0 .. nb - 1 of part[b ncols + c], in that order.
__global__ void k_sum_parts(const float* __restrict__ part, int nb, int64_t ncols,
                            float* __restrict__ out) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncols) return;
  float s = 0.f;
  for (int b = 0; b < nb; ++b) s += part[(int64_t)b * ncols + c];
  out[c] = s;
}

// Layer 2, the loss and the way back to z: one wave per row (lanes over the
// hidden units), rows strided over the grid.  Per block it leaves partial
// sums [db1 (HID) | dW2 (2 HID) | db2 (2) | loss (1)] in part[blockIdx.x]:
// the parameter order after W1, so the block sums land in place.
template <int HQ>  // hidden units per lane (hidden = 64 HQ)
__global__ __launch_bounds__(256) void k_head(int M, const float* __restrict__ Hh,
                                              const float* __restrict__ y,
                                              const float* __restrict__ W2,
                                              const float* __restrict__ b2, float inv_m,
                                              float* __restrict__ dZ, float* __restrict__ part) {
  constexpr int HID = 64 * HQ;
  constexpr int NP = 3 * HID + 3;
  __shared__ float red[4][NP];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  float w0[HQ], w1[HQ], g0[HQ], g1[HQ], gb[HQ];
#pragma unroll
  for (int q = 0; q < HQ; ++q) {
    w0[q] = W2[lane + 64 * q];
    w1[q] = W2[HID + lane + 64 * q];
    g0[q] = g1[q] = gb[q] = 0.f;
  }
  const float c0 = b2[0], c1 = b2[1];
  float d0s = 0.f, d1s = 0.f, ls = 0.f;
  const int nw = gridDim.x * 4;
  for (int r = blockIdx.x * 4 + wid; r < M; r += nw) {
    float hv[HQ];
    float p0 = 0.f, p1 = 0.f;
#pragma unroll
    for (int q = 0; q < HQ; ++q) {
      hv[q] = Hh[(int64_t)r * HID + lane + 64 * q];
      p0 = fmaf(hv[q], w0[q], p0);
      p1 = fmaf(hv[q], w1[q], p1);
    }
#pragma unroll
    for (int sh = 32; sh >= 1; sh >>= 1) {
      p0 += __shfl_xor(p0, sh);
      p1 += __shfl_xor(p1, sh);
    }
    const float e0 = p0 + c0 - y[(int64_t)r * 2], e1 = p1 + c1 - y[(int64_t)r * 2 + 1];
    const float d0 = 2.f * e0 * inv_m, d1 = 2.f * e1 * inv_m;
    d0s += d0;
    d1s += d1;
    ls = fmaf(e0, e0 * inv_m, fmaf(e1, e1 * inv_m, ls));  // the loss is a mean over rows
#pragma unroll
    for (int q = 0; q < HQ; ++q) {
      const float dz = hv[q] > 0.f ? fmaf(d0, w0[q], d1 * w1[q]) : 0.f;
      dZ[(int64_t)r * HID + lane + 64 * q] = dz;
      g0[q] = fmaf(d0, hv[q], g0[q]);
      g1[q] = fmaf(d1, hv[q], g1[q]);
      gb[q] += dz;
    }
  }
#pragma unroll
  for (int q = 0; q < HQ; ++q) {
    red[wid][lane + 64 * q] = gb[q];
    red[wid][HID + lane + 64 * q] = g0[q];
    red[wid][2 * HID + lane + 64 * q] = g1[q];
  }
  if (lane == 0) {
    red[wid][3 * HID] = d0s;
    red[wid][3 * HID + 1] = d1s;
    red[wid][3 * HID + 2] = ls;
  }
  __syncthreads();
  for (int c = threadIdx.x; c < NP; c += blockDim.x)
    part[(int64_t)blockIdx.x * NP + c] = red[0][c] + red[1][c] + red[2][c] + red[3][c];
}

// Gradient descent (adam = 0) or Adam with bias-corrected moments (c1 =
// 1 / (1 - beta1^t), c2 = 1 / (1 - beta2^t)).
__global__ void k_update(int64_t n, float* __restrict__ p, const float* __restrict__ g,
                         float* __restrict__ m, float* __restrict__ v, int adam, float lr,
                         float beta1, float beta2, float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  if (!adam) {
    p[i] -= lr * gi;
    return;
  }
  const float mi = fmaf(beta1, m[i], (1.f - beta1) * gi);
  const float vi = fmaf(beta2, v[i], (1.f - beta2) * gi * gi);
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

static int nblocks(int64_t n, int per) { return (int)((n + per - 1) / per); }

int launch_train_step(const TrainState& s, const float* x, const float* y, int64_t m, int adam,
                      float lr, float c1, float c2, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  const int K2 = s.k2, HID = s.hidden;
  float* W1 = s.theta;
  float* b1 = W1 + (int64_t)HID * K2;
  float* W2 = b1 + HID;
  float* b2 = W2 + 2 * HID;
  float* gW1 = s.grad;
  float* gb1 = gW1 + (int64_t)HID * K2;
  // forward layer 1: H = relu(X W1^T + b1)
  hipLaunchKernelGGL(k_gemm<1>, dim3(nblocks(HID, kGemmTile), nblocks(m, kGemmTile), 1),
                     dim3(256), 0, st, (int)m, HID, K2, K2, x, (int64_t)K2, (int64_t)1, W1,
                     (int64_t)1, (int64_t)K2, b1, s.H);
  // layer 2, loss, dz, and the partial sums of dW2, db1, db2, loss
  const int NP = 3 * HID + 3;
  const float inv_m = 1.f / (float)m;
  switch (HID / 64) {
#define VECKM_HEAD(Q)                                                                            \
  case Q:                                                                                        \
    hipLaunchKernelGGL(k_head<Q>, dim3(s.head_blocks), dim3(256), 0, st, (int)m, s.H, y, W2, b2, \
                       inv_m, s.dZ, s.head_part);                                                \
    break;
    VECKM_HEAD(1) VECKM_HEAD(2) VECKM_HEAD(3) VECKM_HEAD(4)
    VECKM_HEAD(5) VECKM_HEAD(6) VECKM_HEAD(7) VECKM_HEAD(8)
#undef VECKM_HEAD
    default:
      return VECKM_E_INVAL;
  }
  // head sums straight into the b1, W2, b2 gradients, then the loss slot
  hipLaunchKernelGGL(k_sum_parts, dim3(nblocks(NP, 256)), dim3(256), 0, st, s.head_part,
                     s.head_blocks, (int64_t)NP, gb1);
  // dW1 = dZ^T X, split over rows
  const int nsplit = (int)std::min<int64_t>(s.max_splits, std::max<int64_t>(1, m / 2048));
  int kchunk = (int)((m + nsplit - 1) / nsplit);
  kchunk = (kchunk + kGemmK - 1) / kGemmK * kGemmK;
  hipLaunchKernelGGL(k_gemm<0>, dim3(nblocks(K2, kGemmTile), nblocks(HID, kGemmTile), nsplit),
                     dim3(256), 0, st, HID, K2, (int)m, kchunk, s.dZ, (int64_t)1, (int64_t)HID,
                     x, (int64_t)K2, (int64_t)1, nullptr, s.w1_part);
  hipLaunchKernelGGL(k_sum_parts, dim3(nblocks((int64_t)HID * K2, 256)), dim3(256), 0, st,
                     s.w1_part, nsplit, (int64_t)HID * K2, gW1);
  // update (the loss slot after b2 is not a parameter)
  const int64_t np = (int64_t)HID * K2 + HID + 2 * HID + 2;
  hipLaunchKernelGGL(k_update, dim3(nblocks(np, 256)), dim3(256), 0, st, np, s.theta, s.grad,
                     s.m1, s.m2, adam, lr, 0.9f, 0.999f, 1e-8f, c1, c2);
  return hipGetLastError() == hipSuccess ? VECKM_OK : VECKM_E_HIP;
}

}  // namespace veckm
