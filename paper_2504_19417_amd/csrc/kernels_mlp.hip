// The two-layer perceptron of Sec. 2.1 (Eqns. 5-6) on the matrix cores:
//   flow = W2 relu(W1 x + b1) + b2,  x = [Re emb | Im emb] (2D values).
// Layer 1 is the dense contraction [rows x 2D] x [2D x hidden]; layer 2 is
// two dot products per row, done in the epilogue while the hidden values
// are still in registers (ReLU, multiply by W2, reduce across the lanes
// and waves that hold a row's hidden units).
//
// Operands stream straight from global memory into registers: each lane
// loads 16 contiguous bytes of a row of x and of a row of W1 (W1 is
// [hidden][2D], so both are contiguous along the contraction).  The
// contraction index is permuted consistently in A and B so that these
// 16-byte runs map onto the k-slots of the MFMA.
//
// One block of 4 waves handles 64 rows; wave w owns hidden units
// [w*hidden/4, (w+1)*hidden/4).  Blocks loop over row tiles (persistent);
// the row count U is read from the device, so no host synchronisation is
// needed between the encoder and the perceptron.
#include <hip/hip_runtime.h>

#include "veckm_internal.h"

namespace veckm {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

struct MlpArgs {
  const void* x;     // U x K2 (fp32 or bf16)
  const float* W1;   // hidden x K2 fp32
  const uint16_t* W1b;  // hidden x K2 bf16
  const float* b1;
  const float* W2;   // 2 x hidden
  const float* b2;
  float* out;        // U x 2
  const int32_t* plan;
  int K2;
  int hidden;
};

__device__ inline bf16x8 as_bf16x8(uint4 u) {
  bf16x8 h;
  __builtin_memcpy(&h, &u, 16);
  return h;
}

// Layer-2 epilogue shared by both precisions.  acc[mt][nt][i] is the
// pre-activation of row 16*mt + 4*(lane>>4) + i, hidden unit
// col0 + 16*nt + (lane&15).
template <int NTH>
__device__ inline void mlp_epilogue(const MlpArgs& a, floatx4 (&acc)[4][NTH], int tile, int U,
                                    float (*red)[64][2]) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int col0 = wid * NTH * 16;
  float p0[4][4], p1[4][4];
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int i = 0; i < 4; ++i) p0[mt][i] = p1[mt][i] = 0.f;
#pragma unroll
  for (int nt = 0; nt < NTH; ++nt) {
    const int c = col0 + nt * 16 + (lane & 15);
    const float bb = a.b1[c], w0 = a.W2[c], w1 = a.W2[a.hidden + c];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float h = fmaxf(acc[mt][nt][i] + bb, 0.f);
        p0[mt][i] += w0 * h;
        p1[mt][i] += w1 * h;
      }
  }
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
      for (int sh = 1; sh < 16; sh <<= 1) {
        p0[mt][i] += __shfl_xor(p0[mt][i], sh);
        p1[mt][i] += __shfl_xor(p1[mt][i], sh);
      }
      if ((lane & 15) == 0) {
        const int r = mt * 16 + 4 * (lane >> 4) + i;
        red[wid][r][0] = p0[mt][i];
        red[wid][r][1] = p1[mt][i];
      }
    }
  __syncthreads();
  if (threadIdx.x < 128) {
    const int r = threadIdx.x >> 1, o = threadIdx.x & 1;
    const int row = tile * 64 + r;
    const float v = red[0][r][o] + red[1][r][o] + red[2][r][o] + red[3][r][o] + a.b2[o];
    if (row < U) a.out[(int64_t)row * 2 + o] = v;
  }
  __syncthreads();
}

template <int NTH>
__global__ __launch_bounds__(256) void k_mlp_f32(MlpArgs a) {
  __shared__ float red[4][64][2];
  const int U = a.plan[0];
  const int ntiles = (U + 63) / 64;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const float* X = static_cast<const float*>(a.x);
  const int g = lane >> 4;
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    floatx4 acc[4][NTH];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int nt = 0; nt < NTH; ++nt) acc[mt][nt] = floatx4{0.f, 0.f, 0.f, 0.f};
    const float* xr[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      int row = tile * 64 + mt * 16 + (lane & 15);
      row = row < U ? row : U - 1;
      xr[mt] = X + (int64_t)row * a.K2 + 4 * g;
    }
    const float* wr[NTH];
#pragma unroll
    for (int nt = 0; nt < NTH; ++nt)
      wr[nt] = a.W1 + (int64_t)(wid * NTH * 16 + nt * 16 + (lane & 15)) * a.K2 + 4 * g;
    for (int kq = 0; kq < a.K2; kq += 16) {
      float4 av[4], bv[NTH];
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) av[mt] = *reinterpret_cast<const float4*>(xr[mt] + kq);
#pragma unroll
      for (int nt = 0; nt < NTH; ++nt) bv[nt] = *reinterpret_cast<const float4*>(wr[nt] + kq);
#pragma unroll
      for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int nt = 0; nt < NTH; ++nt) {
          acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[mt].x, bv[nt].x, acc[mt][nt], 0, 0, 0);
          acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[mt].y, bv[nt].y, acc[mt][nt], 0, 0, 0);
          acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[mt].z, bv[nt].z, acc[mt][nt], 0, 0, 0);
          acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[mt].w, bv[nt].w, acc[mt][nt], 0, 0, 0);
        }
    }
    mlp_epilogue<NTH>(a, acc, tile, U, red);
  }
}

template <int NTH>
__global__ __launch_bounds__(256) void k_mlp_bf16(MlpArgs a) {
  __shared__ float red[4][64][2];
  const int U = a.plan[0];
  const int ntiles = (U + 63) / 64;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const uint16_t* X = static_cast<const uint16_t*>(a.x);
  const int g = lane >> 4;
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    floatx4 acc[4][NTH];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int nt = 0; nt < NTH; ++nt) acc[mt][nt] = floatx4{0.f, 0.f, 0.f, 0.f};
    const uint16_t* xr[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      int row = tile * 64 + mt * 16 + (lane & 15);
      row = row < U ? row : U - 1;
      xr[mt] = X + (int64_t)row * a.K2 + 8 * g;
    }
    const uint16_t* wr[NTH];
#pragma unroll
    for (int nt = 0; nt < NTH; ++nt)
      wr[nt] = a.W1b + (int64_t)(wid * NTH * 16 + nt * 16 + (lane & 15)) * a.K2 + 8 * g;
    for (int kq = 0; kq < a.K2; kq += 32) {
      bf16x8 av[4], bv[NTH];
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) av[mt] = as_bf16x8(*reinterpret_cast<const uint4*>(xr[mt] + kq));
#pragma unroll
      for (int nt = 0; nt < NTH; ++nt) bv[nt] = as_bf16x8(*reinterpret_cast<const uint4*>(wr[nt] + kq));
#pragma unroll
      for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int nt = 0; nt < NTH; ++nt)
          acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[mt], bv[nt], acc[mt][nt], 0, 0, 0);
    }
    mlp_epilogue<NTH>(a, acc, tile, U, red);
  }
}

template <int NTH>
static void launch_nth(const MlpArgs& a, bool bf16, int grid, hipStream_t s) {
  if (bf16)
    hipLaunchKernelGGL(k_mlp_bf16<NTH>, dim3(grid), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(k_mlp_f32<NTH>, dim3(grid), dim3(256), 0, s, a);
}

int launch_mlp(const SliceGeom& g, const Workspace& w, const MlpWeights& mw, int d, bool bf16,
               int num_cus, void* stream) {
  (void)g;
  MlpArgs a;
  a.x = w.rows;
  a.W1 = mw.W1;
  a.W1b = mw.W1b;
  a.b1 = mw.b1;
  a.W2 = mw.W2;
  a.b2 = mw.b2;
  a.out = w.rowflow;
  a.plan = w.plan;
  a.K2 = 2 * d;
  a.hidden = mw.hidden;
  if (bf16 && (a.K2 % 32)) return VECKM_E_INVAL;
  const int grid = num_cus * 4;
  hipStream_t s = (hipStream_t)stream;
  switch (mw.hidden / 64) {
    case 1: launch_nth<1>(a, bf16, grid, s); break;
    case 2: launch_nth<2>(a, bf16, grid, s); break;
    case 3: launch_nth<3>(a, bf16, grid, s); break;
    case 4: launch_nth<4>(a, bf16, grid, s); break;
    case 5: launch_nth<5>(a, bf16, grid, s); break;
    case 6: launch_nth<6>(a, bf16, grid, s); break;
    case 7: launch_nth<7>(a, bf16, grid, s); break;
    case 8: launch_nth<8>(a, bf16, grid, s); break;
    default: return VECKM_E_INVAL;
  }
  return hipGetLastError() == hipSuccess ? VECKM_OK : VECKM_E_HIP;
}

}  // namespace veckm
