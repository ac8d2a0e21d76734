// The two-layer perceptron of Sec. 2.1 (Eqns. 5-6) on the matrix cores:
//   flow = W2 relu(W1 x + b1) + b2,  x = [Re emb | Im emb] (K2 = 2D values).
// Layer 1 is the dense contraction [hidden x K2] x [K2 x rows]; layer 2 is
// two dot products per row, done in the epilogue while the hidden values
// are still in registers (ReLU, multiply by W2, reduce across the lanes
// and waves that hold a row's hidden units).
//
// Main kernel (k_mlp_res): a block of 4 waves (one per SIMD) walks 64-row
// tiles of x; wave w owns hidden units [w hidden/4, (w+1) hidden/4) and
// keeps their W1 fragments in registers for the whole kernel.  x tiles
// stream into LDS with global->LDS copies NBUF - 1 tiles ahead of use,
// 16-byte chunks XOR-swizzled by row so that fragment reads hit distinct
// banks.  Two operand forms:
//   * bf16 rows x bf16 W1 (the FP16 form), one product;
//   * fp32 rows and W1, both carried as fp16 hi + lo pairs (the FP32 form:
//     22 significant bits per operand; rows are split as their fragments
//     are read), three products hi*hi + hi*lo + lo*hi, fp32 accumulation;
//     W1 is scaled by a power of two so that its lo parts stay normal, and
//     the sums are scaled back exactly.
// The contraction index is permuted consistently in A (W1) and B (x) so that
// each lane's operand is 16 contiguous bytes of a row of W1 and of x; with W1
// as the A operand, a lane's accumulator holds 4 consecutive hidden units of
// one row.  Fallbacks for shapes whose W1 does not fit in registers read W1
// from L2 (bf16), or run fp32 rows on the fp32 matrix cores.
//
// The row count U is read from the device, so no host synchronisation is
// needed between the encoder and the perceptron.
#include <hip/hip_runtime.h>

#include "sync.h"
#include "veckm_internal.h"

namespace veckm {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

struct MlpArgs {
  const void* x;        // U rows of K2 values, fp32 or bf16
  const float* W1;      // hidden x K2 fp32
  const uint16_t* W1b;  // hidden x K2 bf16
  const uint16_t* W1h;  // hidden x K2 fp16 hi of W1 * 2^s
  const uint16_t* W1l;  // hidden x K2 fp16 lo of W1 * 2^s
  float unscale;        // 2^-s
  const float* b1;
  const float* W2;  // 2 x hidden
  const float* b2;
  float* out;  // U x 2
  const int32_t* plan;
  int K2;
  int hidden;
};

__device__ inline bf16x8 as_bf16x8(uint4 u) {
  bf16x8 h;
  __builtin_memcpy(&h, &u, 16);
  return h;
}

__device__ inline f16x8 as_f16x8(uint4 u) {
  f16x8 h;
  __builtin_memcpy(&h, &u, 16);
  return h;
}

// s_waitcnt immediate (gfx9 encoding) waiting until at most n (<= 63) vector
// memory operations are outstanding.
constexpr int mlp_vmcnt(int n) { return (n & 15) | ((n >> 4) << 14) | (7 << 4) | (15 << 8); }
constexpr int mlp_vmcnt0() { return mlp_vmcnt(0); }

// Per-wave layer constants: b1, W2[0], W2[1] of the lane's hidden units.
template <int NTH>
struct Layer2 {
  float b[NTH], w0[NTH], w1[NTH];
  __device__ void load(const MlpArgs& a) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int nt = 0; nt < NTH; ++nt) {
      const int c = wid * NTH * 16 + nt * 16 + (lane & 15);
      b[nt] = a.b1[c];
      w0[nt] = a.W2[c];
      w1[nt] = a.W2[a.hidden + c];
    }
  }
};

// Layer-2 epilogue.  acc[mt][nt][i] is the pre-activation of row
// 16*mt + 4*(lane>>4) + i of the tile, hidden unit col0 + 16*nt + (lane&15).
template <int NTH>
__device__ inline void mlp_epilogue(const MlpArgs& a, const Layer2<NTH>& l2, floatx4 (&acc)[4][NTH],
                                    int tile, int U, float (*red)[64][2]) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  float p0[4][4], p1[4][4];
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int i = 0; i < 4; ++i) p0[mt][i] = p1[mt][i] = 0.f;
#pragma unroll
  for (int nt = 0; nt < NTH; ++nt) {
    const float bb = l2.b[nt], w0 = l2.w0[nt], w1 = l2.w1[nt];
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
  lds_barrier();
  if (threadIdx.x < 128) {
    const int r = threadIdx.x >> 1, o = threadIdx.x & 1;
    const int row = tile * 64 + r;
    const float v = red[0][r][o] + red[1][r][o] + red[2][r][o] + red[3][r][o] + a.b2[o];
    if (row < U) a.out[(int64_t)row * 2 + o] = v;
  }
}

// Starts the copy of x tile `tile` (64 rows of RB bytes) into an LDS buffer:
// LDS chunk p of row r holds global chunk p ^ (r & 15) (16-byte chunks).
// Rows past U repeat row U - 1 (their results are dropped).
template <int RB, int NW>
__device__ inline void issue_tile(const unsigned char* x, int tile, int U, uint4* buf, int wid,
                                  int lane) {
  constexpr int CPR = RB / 16;          // chunks per row
  constexpr int RPI = 64 / CPR;         // rows per wave instruction
  static_assert(64 % CPR == 0 && (64 / RPI) % NW == 0, "row size");
#pragma unroll
  for (int u = 0; u < 64 / RPI / NW; ++u) {
    const int rb = (u * NW + wid) * RPI;  // first row of this instruction
    const int r = rb + lane / CPR, p = lane % CPR;
    int row = tile * 64 + r;
    row = row < U ? row : U - 1;
    const uint4* src = reinterpret_cast<const uint4*>(x + (int64_t)row * RB) + (p ^ (r & 15));
    copy_to_lds16(src, lds_offset(buf + rb * CPR));
  }
}

// fp32: A from the LDS tile, B (W1) from L2 one k-slice ahead.
template <int NTH, int K2>
__global__ __launch_bounds__(256) void k_mlp_f32(MlpArgs a) {
  constexpr int RB = K2 * 4, CPR = RB / 16;
  extern __shared__ __align__(16) unsigned char smem_mlp[];
  uint4* tbuf = reinterpret_cast<uint4*>(smem_mlp);  // 2 x 64 rows
  __shared__ float red[4][64][2];
  const int U = a.plan[0];
  const int ntiles = (U + 63) / 64;
  Layer2<NTH> l2;
  l2.load(a);
  const int lane = threadIdx.x & 63;
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int g = lane >> 4, r16 = lane & 15;
  const unsigned char* X = static_cast<const unsigned char*>(a.x);
  const float* wr[NTH];
#pragma unroll
  for (int nt = 0; nt < NTH; ++nt)
    wr[nt] = a.W1 + (int64_t)(wid * NTH * 16 + nt * 16 + r16) * K2 + 4 * g;
  int tile = blockIdx.x;
  if (tile < ntiles) issue_tile<RB, 4>(X, tile, U, tbuf, wid, lane);
  for (int it = 0; tile < ntiles; tile += gridDim.x, ++it) {
    uint4* cur = tbuf + (it & 1) * 64 * CPR;
    const int next = tile + gridDim.x;
    __builtin_amdgcn_s_waitcnt(mlp_vmcnt0());
    lds_barrier();  // tile `tile` is in `cur`; the other buffer is free
    if (next < ntiles) issue_tile<RB, 4>(X, next, U, tbuf + ((it + 1) & 1) * 64 * CPR, wid, lane);
    floatx4 acc[4][NTH];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int nt = 0; nt < NTH; ++nt) acc[mt][nt] = floatx4{0.f, 0.f, 0.f, 0.f};
    float4 bv[NTH], bn[NTH];
#pragma unroll
    for (int nt = 0; nt < NTH; ++nt) bv[nt] = *reinterpret_cast<const float4*>(wr[nt]);
#pragma unroll 2
    for (int kq = 0; kq < K2 / 16; ++kq) {
      if (kq + 1 < K2 / 16) {
#pragma unroll
        for (int nt = 0; nt < NTH; ++nt)
          bn[nt] = *reinterpret_cast<const float4*>(wr[nt] + (kq + 1) * 16);
      }
      float4 av[4];
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) {
        const int r = mt * 16 + r16, c = kq * 4 + g;
        av[mt] = *reinterpret_cast<const float4*>(cur + r * CPR + (c ^ (r & 15)));
      }
#pragma unroll
      for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int nt = 0; nt < NTH; ++nt) {
          acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[mt].x, bv[nt].x, acc[mt][nt], 0, 0, 0);
          acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[mt].y, bv[nt].y, acc[mt][nt], 0, 0, 0);
          acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[mt].z, bv[nt].z, acc[mt][nt], 0, 0, 0);
          acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[mt].w, bv[nt].w, acc[mt][nt], 0, 0, 0);
        }
#pragma unroll
      for (int nt = 0; nt < NTH; ++nt) bv[nt] = bn[nt];
    }
    mlp_epilogue<NTH>(a, l2, acc, tile, U, red);
  }
}

// bf16 fallback (any K2 multiple of 32, any hidden): operands from L2.
template <int NTH>
__global__ __launch_bounds__(256) void k_mlp_bf16(MlpArgs a) {
  __shared__ float red[4][64][2];
  const int U = a.plan[0];
  const int ntiles = (U + 63) / 64;
  Layer2<NTH> l2;
  l2.load(a);
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
    mlp_epilogue<NTH>(a, l2, acc, tile, U, red);
    lds_barrier();
  }
}

// fp32 fallback (K2 not specialised): operands from L2.
template <int NTH>
__global__ __launch_bounds__(256) void k_mlp_f32_any(MlpArgs a) {
  __shared__ float red[4][64][2];
  const int U = a.plan[0];
  const int ntiles = (U + 63) / 64;
  Layer2<NTH> l2;
  l2.load(a);
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
    mlp_epilogue<NTH>(a, l2, acc, tile, U, red);
    lds_barrier();
  }
}

// Per-wave layer-2 constants of the lane's hidden units: unit
// w*16*NTH + 16*nt + 4*(lane>>4) + i.
template <int NTH>
struct Layer2T {
  float b[NTH][4], w0[NTH][4], w1[NTH][4];
  __device__ void load(const MlpArgs& a, int wid, int lane) {
#pragma unroll
    for (int nt = 0; nt < NTH; ++nt)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int c = wid * NTH * 16 + nt * 16 + 4 * (lane >> 4) + i;
        b[nt][i] = a.b1[c];
        w0[nt][i] = a.W2[c];
        w1[nt][i] = a.W2[a.hidden + c];
      }
  }
};

// FORM 0: bf16 rows x bf16 W1.  FORM 1: fp32 rows and W1, both as fp16 hi/lo.
// FORM 2: rows already split by the encoder (each group of 4 consecutive
// elements is a 16-byte unit [hi x 4, lo x 4]) and W1 as fp16 hi/lo.  NW
// waves per block, each owning 16 NTH hidden units.
template <int FORM, int NW, int NTH, int K2, int NBUF>
__global__ __launch_bounds__(NW * 64) void k_mlp_res(MlpArgs a) {
  constexpr int KQ = K2 / 32;
  constexpr int RB = FORM == 0 ? K2 * 2 : K2 * 4;  // bytes per row (fp32, or hi + lo halves)
  constexpr int CPR = RB / 16;                      // 16-byte chunks per row
  constexpr int TILE_U4 = 64 * CPR;
  constexpr int PFW = TILE_U4 / (NW * 64);          // copies per wave per tile
  static_assert(CPR % 16 == 0 && CPR <= 64, "row size");
  static_assert((NBUF - 2) * PFW <= 63, "copies in flight exceed the wait counter");
  extern __shared__ __align__(16) unsigned char smem_mlp[];
  uint4* tbuf = reinterpret_cast<uint4*>(smem_mlp);  // NBUF tiles of 64 rows
  __shared__ float red[NW][64][2];
  const int U = a.plan[0];
  const int ntiles = (U + 63) / 64;
  const int lane = threadIdx.x & 63;
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int g = lane >> 4, r16 = lane & 15;
  const unsigned char* X = static_cast<const unsigned char*>(a.x);
  // W1 fragments (A operand: hidden unit r16 of the tile, contraction
  // elements 32 kq + 8 g .. + 7)
  uint4 wh[KQ][NTH], wl[FORM != 0 ? KQ : 1][NTH];
#pragma unroll
  for (int nt = 0; nt < NTH; ++nt) {
    const int64_t h = wid * NTH * 16 + nt * 16 + r16;
#pragma unroll
    for (int kq = 0; kq < KQ; ++kq) {
      const uint16_t* src = (FORM == 0 ? a.W1b : a.W1h) + h * K2 + kq * 32 + 8 * g;
      wh[kq][nt] = *reinterpret_cast<const uint4*>(src);
      if constexpr (FORM != 0)
        wl[kq][nt] = *reinterpret_cast<const uint4*>(a.W1l + h * K2 + kq * 32 + 8 * g);
    }
  }
  Layer2T<NTH> l2;
  l2.load(a, wid, lane);
  const float unscale = FORM != 0 ? a.unscale : 1.f;
  const int mine = blockIdx.x < ntiles ? (ntiles - 1 - blockIdx.x) / gridDim.x + 1 : 0;
#pragma unroll
  for (int u = 0; u < NBUF - 1; ++u)
    if (u < mine)
      issue_tile<RB, NW>(X, blockIdx.x + u * gridDim.x, U, tbuf + u * TILE_U4, wid, lane);
  for (int it = 0; it < mine; ++it) {
    const int tile = blockIdx.x + it * gridDim.x;
    uint4* cur = tbuf + (it % NBUF) * TILE_U4;
    // tile `it` has landed once only the copies of the later tiles already
    // issued (at most NBUF - 2 of them) may be outstanding
    const int later = mine - 1 - it < NBUF - 2 ? mine - 1 - it : NBUF - 2;
    if (NBUF > 2 && later >= 1) {
      if (later >= 2 && NBUF > 3)
        __builtin_amdgcn_s_waitcnt(mlp_vmcnt((NBUF - 2) * PFW > 63 ? 63 : 2 * PFW));
      else
        __builtin_amdgcn_s_waitcnt(mlp_vmcnt(PFW));
    } else {
      __builtin_amdgcn_s_waitcnt(mlp_vmcnt0());
    }
    lds_barrier();  // tile `it` is in `cur`; the buffer of tile it - 1 is free
    if (it + NBUF - 1 < mine)
      issue_tile<RB, NW>(X, tile + (NBUF - 1) * gridDim.x, U,
                         tbuf + ((it + NBUF - 1) % NBUF) * TILE_U4, wid, lane);
    floatx4 acc[4][NTH];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int nt = 0; nt < NTH; ++nt) acc[mt][nt] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kq = 0; kq < KQ; ++kq) {
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) {
        const int r = mt * 16 + r16;
        if constexpr (FORM == 0) {
          const int c = kq * 4 + g;  // 8 bf16 elements per 16-byte chunk
          const uint4 xb = cur[r * CPR + (c ^ (r & 15))];
#pragma unroll
          for (int nt = 0; nt < NTH; ++nt)
            acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(wh[kq][nt]),
                                                                  as_bf16x8(xb), acc[mt][nt], 0, 0, 0);
        } else if constexpr (FORM == 2) {
          // elements 32 kq + 8 g .. + 7: two units; their hi and lo halves
          // regroup by register (no conversion)
          const int c = kq * 8 + 2 * g;
          const uint4 u0 = cur[r * CPR + (c ^ (r & 15))];
          const uint4 u1 = cur[r * CPR + ((c + 1) ^ (r & 15))];
          const f16x8 xh = as_f16x8(make_uint4(u0.x, u0.y, u1.x, u1.y));
          const f16x8 xl = as_f16x8(make_uint4(u0.z, u0.w, u1.z, u1.w));
#pragma unroll
          for (int nt = 0; nt < NTH; ++nt) {
            acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(as_f16x8(wh[kq][nt]), xh,
                                                                 acc[mt][nt], 0, 0, 0);
            acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(as_f16x8(wl[kq][nt]), xh,
                                                                 acc[mt][nt], 0, 0, 0);
            acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(as_f16x8(wh[kq][nt]), xl,
                                                                 acc[mt][nt], 0, 0, 0);
          }
        } else {
          // fp32 row elements 32 kq + 8 g .. + 7 (two chunks), split into an
          // fp16 hi + lo pair: lo = v - hi is exact in fp32, then rounded
          const int c = kq * 8 + 2 * g;
          const uint4 u0 = cur[r * CPR + (c ^ (r & 15))];
          const uint4 u1 = cur[r * CPR + ((c + 1) ^ (r & 15))];
          const float v[8] = {__uint_as_float(u0.x), __uint_as_float(u0.y), __uint_as_float(u0.z),
                              __uint_as_float(u0.w), __uint_as_float(u1.x), __uint_as_float(u1.y),
                              __uint_as_float(u1.z), __uint_as_float(u1.w)};
          f16x8 xh, xl;
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            xh[e] = (_Float16)v[e];
            xl[e] = (_Float16)(v[e] - (float)xh[e]);
          }
#pragma unroll
          for (int nt = 0; nt < NTH; ++nt) {
            acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(as_f16x8(wh[kq][nt]), xh,
                                                                 acc[mt][nt], 0, 0, 0);
            acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(as_f16x8(wl[kq][nt]), xh,
                                                                 acc[mt][nt], 0, 0, 0);
            acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(as_f16x8(wh[kq][nt]), xl,
                                                                 acc[mt][nt], 0, 0, 0);
          }
        }
      }
    }
    // layer 2: the lane holds hidden units 16 nt + 4 g + i of row 16 mt + r16
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      float p0 = 0.f, p1 = 0.f;
#pragma unroll
      for (int nt = 0; nt < NTH; ++nt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const float h = fmaxf(fmaf(acc[mt][nt][i], unscale, l2.b[nt][i]), 0.f);
          p0 = fmaf(l2.w0[nt][i], h, p0);
          p1 = fmaf(l2.w1[nt][i], h, p1);
        }
      p0 += __shfl_xor(p0, 16);
      p1 += __shfl_xor(p1, 16);
      p0 += __shfl_xor(p0, 32);
      p1 += __shfl_xor(p1, 32);
      if (g == 0) {
        red[wid][mt * 16 + r16][0] = p0;
        red[wid][mt * 16 + r16][1] = p1;
      }
    }
    lds_barrier();
    if (threadIdx.x < 128) {
      const int r = threadIdx.x >> 1, o = threadIdx.x & 1;
      const int row = tile * 64 + r;
      float v = a.b2[o];
#pragma unroll
      for (int w = 0; w < NW; ++w) v += red[w][r][o];
      if (row < U) a.out[(int64_t)row * 2 + o] = v;
    }
  }
}

// FP32 form with the split done once per tile: the fp32 tile lands in a
// staging buffer, the block splits it into fp16 hi/lo pairs in a second
// buffer (each element converted once), and the next tile's copy into the
// staging buffer overlaps the products.  Split layout per row: chunks
// [0, K2/8) hold the hi halves of elements 8c .. 8c + 7, chunks [K2/8, K2/4)
// the lo halves; chunk p of row r sits at p ^ (r & 15).
template <int NW, int NTH, int K2>
__global__ __launch_bounds__(NW * 64) void k_mlp_split(MlpArgs a) {
  constexpr int KQ = K2 / 32;
  constexpr int RB = K2 * 4;        // bytes per fp32 row (and per split row)
  constexpr int CPR = RB / 16;      // 16-byte chunks per row
  constexpr int TILE_U4 = 64 * CPR;
  constexpr int PFW = TILE_U4 / (NW * 64);
  constexpr int HALF = CPR / 2;     // first lo chunk of a split row
  static_assert(CPR % 16 == 0 && CPR <= 64, "row size");
  static_assert(PFW <= 63, "copies in flight exceed the wait counter");
  static_assert((64 * HALF) % (NW * 64) == 0, "split work per thread");
  extern __shared__ __align__(16) unsigned char smem_mlp[];
  uint4* stage = reinterpret_cast<uint4*>(smem_mlp);  // fp32 tile being copied in
  uint4* split = stage + TILE_U4;                      // the current tile as hi/lo
  __shared__ float red[NW][64][2];
  const int U = a.plan[0];
  const int ntiles = (U + 63) / 64;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int g = lane >> 4, r16 = lane & 15;
  const unsigned char* X = static_cast<const unsigned char*>(a.x);
  uint4 wh[KQ][NTH], wl[KQ][NTH];
#pragma unroll
  for (int nt = 0; nt < NTH; ++nt) {
    const int64_t h = wid * NTH * 16 + nt * 16 + r16;
#pragma unroll
    for (int kq = 0; kq < KQ; ++kq) {
      wh[kq][nt] = *reinterpret_cast<const uint4*>(a.W1h + h * K2 + kq * 32 + 8 * g);
      wl[kq][nt] = *reinterpret_cast<const uint4*>(a.W1l + h * K2 + kq * 32 + 8 * g);
    }
  }
  Layer2T<NTH> l2;
  l2.load(a, wid, lane);
  const float unscale = a.unscale;
  const int mine = blockIdx.x < ntiles ? (ntiles - 1 - blockIdx.x) / gridDim.x + 1 : 0;
  if (mine > 0) issue_tile<RB, NW>(X, blockIdx.x, U, stage, wid, lane);
  for (int it = 0; it < mine; ++it) {
    const int tile = blockIdx.x + it * gridDim.x;
    __builtin_amdgcn_s_waitcnt(mlp_vmcnt0());
    lds_barrier();  // tile `it` is in `stage`; `split` is free (previous products done)
    // ---- split: work item (row r, output chunk q) covers elements 8q .. 8q + 7
#pragma unroll
    for (int w = 0; w < 64 * HALF / (NW * 64); ++w) {
      const int item = w * NW * 64 + tid;
      const int r = item / HALF, q = item % HALF;
      const uint4 u0 = stage[r * CPR + ((2 * q) ^ (r & 15))];
      const uint4 u1 = stage[r * CPR + ((2 * q + 1) ^ (r & 15))];
      const float v[8] = {__uint_as_float(u0.x), __uint_as_float(u0.y), __uint_as_float(u0.z),
                          __uint_as_float(u0.w), __uint_as_float(u1.x), __uint_as_float(u1.y),
                          __uint_as_float(u1.z), __uint_as_float(u1.w)};
      f16x8 hi, lo;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        hi[e] = (_Float16)v[e];
        lo[e] = (_Float16)(v[e] - (float)hi[e]);
      }
      uint4 hu, lu;
      __builtin_memcpy(&hu, &hi, 16);
      __builtin_memcpy(&lu, &lo, 16);
      split[r * CPR + (q ^ (r & 15))] = hu;
      split[r * CPR + ((q + HALF) ^ (r & 15))] = lu;
    }
    lds_barrier();  // `split` holds the tile; `stage` is free
    if (it + 1 < mine) issue_tile<RB, NW>(X, tile + gridDim.x, U, stage, wid, lane);
    floatx4 acc[4][NTH];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int nt = 0; nt < NTH; ++nt) acc[mt][nt] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kq = 0; kq < KQ; ++kq) {
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) {
        const int r = mt * 16 + r16, c = kq * 4 + g;
        const f16x8 xh = as_f16x8(split[r * CPR + (c ^ (r & 15))]);
        const f16x8 xl = as_f16x8(split[r * CPR + ((c + HALF) ^ (r & 15))]);
#pragma unroll
        for (int nt = 0; nt < NTH; ++nt) {
          acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(as_f16x8(wh[kq][nt]), xh,
                                                               acc[mt][nt], 0, 0, 0);
          acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(as_f16x8(wl[kq][nt]), xh,
                                                               acc[mt][nt], 0, 0, 0);
          acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(as_f16x8(wh[kq][nt]), xl,
                                                               acc[mt][nt], 0, 0, 0);
        }
      }
    }
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      float p0 = 0.f, p1 = 0.f;
#pragma unroll
      for (int nt = 0; nt < NTH; ++nt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const float h = fmaxf(fmaf(acc[mt][nt][i], unscale, l2.b[nt][i]), 0.f);
          p0 = fmaf(l2.w0[nt][i], h, p0);
          p1 = fmaf(l2.w1[nt][i], h, p1);
        }
      p0 += __shfl_xor(p0, 16);
      p1 += __shfl_xor(p1, 16);
      p0 += __shfl_xor(p0, 32);
      p1 += __shfl_xor(p1, 32);
      if (g == 0) {
        red[wid][mt * 16 + r16][0] = p0;
        red[wid][mt * 16 + r16][1] = p1;
      }
    }
    lds_barrier();
    if (tid < 128) {
      const int r = tid >> 1, o = tid & 1;
      const int row = tile * 64 + r;
      float v = a.b2[o];
#pragma unroll
      for (int w = 0; w < NW; ++w) v += red[w][r][o];
      if (row < U) a.out[(int64_t)row * 2 + o] = v;
    }
  }
}

template <typename K>
static int launch_lds(K kern, const MlpArgs& a, size_t lds, int per_cu, int num_cus, hipStream_t s,
                      int threads) {
  if (hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return VECKM_E_HIP;
  hipLaunchKernelGGL(kern, dim3(num_cus * per_cu), dim3(threads), lds, s, a);
  return hipGetLastError() == hipSuccess ? VECKM_OK : VECKM_E_HIP;
}

// Waves per block of the register-resident perceptron: 8 (two per SIMD, so
// that one wave's conversions and LDS reads overlap the other's matrix
// operations) when the hidden units split evenly, else 4.
constexpr int kMlpWaves = 8;

template <int NTH4, int K2>
static int launch_split(const MlpArgs& a, int num_cus, hipStream_t s) {
  constexpr size_t lds = 2 * (size_t)64 * K2 * 4;
  if constexpr (kMlpWaves == 8 && NTH4 % 2 == 0)
    return launch_lds(k_mlp_split<8, NTH4 / 2, K2>, a, lds, 1, num_cus, s, 512);
  else
    return launch_lds(k_mlp_split<4, NTH4, K2>, a, lds, 1, num_cus, s, 256);
}

template <int FORM, int NTH4, int K2, int NBUF>
static int launch_res(const MlpArgs& a, int num_cus, hipStream_t s) {
  constexpr size_t lds = (size_t)NBUF * 64 * (FORM == 0 ? K2 * 2 : K2 * 4);
  if constexpr (kMlpWaves == 8 && NTH4 % 2 == 0)
    return launch_lds(k_mlp_res<FORM, 8, NTH4 / 2, K2, NBUF>, a, lds, 1, num_cus, s, 512);
  else
    return launch_lds(k_mlp_res<FORM, 4, NTH4, K2, NBUF>, a, lds, 1, num_cus, s, 256);
}

template <int NTH>
static int launch_nth(const MlpArgs& a, int rows, int num_cus, hipStream_t s) {
  if (rows == kRowsBF16) {
    // W1 of the wave's hidden units in registers when it fits
    if constexpr (NTH <= 4) {
      if (a.K2 == 256) return launch_res<0, NTH, 256, 3>(a, num_cus, s);
    }
    if constexpr (NTH <= 8) {
      if (a.K2 == 128) return launch_res<0, NTH, 128, 4>(a, num_cus, s);
    }
    hipLaunchKernelGGL(k_mlp_bf16<NTH>, dim3(num_cus * 4), dim3(256), 0, s, a);
  } else if (rows == kRowsHiLo16) {
    // shapes admitted by mlp_rows_split(); two 64-row tiles in LDS
    if constexpr (NTH <= 4) {
      if (a.K2 == 256) return launch_res<2, NTH, 256, 2>(a, num_cus, s);
    }
    if constexpr (NTH <= 6) {
      if (a.K2 == 128) return launch_res<2, NTH, 128, 2>(a, num_cus, s);
    }
    if constexpr (NTH <= 8) {
      if (a.K2 == 64) return launch_res<2, NTH, 64, 2>(a, num_cus, s);
    }
    return VECKM_E_INVAL;
  } else if (rows == kRowsSplit16) {
    // shapes admitted by mlp_rows_split()
    if constexpr (NTH <= 4) {
      if (a.K2 == 256) return launch_split<NTH, 256>(a, num_cus, s);
    }
    if constexpr (NTH <= 6) {
      if (a.K2 == 128) return launch_split<NTH, 128>(a, num_cus, s);
    }
    if constexpr (NTH <= 8) {
      if (a.K2 == 64) return launch_split<NTH, 64>(a, num_cus, s);
    }
    return VECKM_E_INVAL;
  } else {
    if (a.K2 == 256) return launch_lds(k_mlp_f32<NTH, 256>, a, 2 * 64 * 256 * 4, 1, num_cus, s, 256);
    if (a.K2 == 128) return launch_lds(k_mlp_f32<NTH, 128>, a, 2 * 64 * 128 * 4, 2, num_cus, s, 256);
    hipLaunchKernelGGL(k_mlp_f32_any<NTH>, dim3(num_cus * 4), dim3(256), 0, s, a);
  }
  return hipGetLastError() == hipSuccess ? VECKM_OK : VECKM_E_HIP;
}

bool mlp_rows_split(int d, int hidden) {
  const int k2 = 2 * d, nth = hidden / 64;
  return (k2 == 256 && nth <= 4) || (k2 == 128 && nth <= 6) || (k2 == 64 && nth <= 8);
}

int launch_mlp(const Workspace& w, const MlpWeights& mw, int d, int rows, int num_cus,
               void* stream) {
  MlpArgs a;
  a.x = w.rows;
  a.W1 = mw.W1;
  a.W1b = mw.W1b;
  a.W1h = mw.W1h;
  a.W1l = mw.W1l;
  a.unscale = mw.unscale;
  a.b1 = mw.b1;
  a.W2 = mw.W2;
  a.b2 = mw.b2;
  a.out = w.rowflow;
  a.plan = w.plan;
  a.K2 = 2 * d;
  a.hidden = mw.hidden;
  if (a.K2 % 32) return VECKM_E_INVAL;
  hipStream_t s = (hipStream_t)stream;
  switch (mw.hidden / 64) {
    case 1: return launch_nth<1>(a, rows, num_cus, s);
    case 2: return launch_nth<2>(a, rows, num_cus, s);
    case 3: return launch_nth<3>(a, rows, num_cus, s);
    case 4: return launch_nth<4>(a, rows, num_cus, s);
    case 5: return launch_nth<5>(a, rows, num_cus, s);
    case 6: return launch_nth<6>(a, rows, num_cus, s);
    case 7: return launch_nth<7>(a, rows, num_cus, s);
    case 8: return launch_nth<8>(a, rows, num_cus, s);
    default: return VECKM_E_INVAL;
  }
}

}  // namespace veckm
