// The encoder contraction on the gfx950 matrix cores.
//
// For a query voxel v and frequency j the window sum of Eqn. 16 (with the
// count of Eqn. 17), written over integer offsets o of the window B, is
//   S_j(v) = sum_{o in B} C[v + o] e^{i theta_j(o)},   N(v) = sum_{o in B} C[v + o],
// where C is the per-voxel event count (Eqns. 14-15 with every phase
// factored out) and theta_j(o) = A[j] . o.  The encoding is S_j(v) / N(v)
// (Algorithm 1, final step).  Pairing o with -o:
//   Re S_j = sum_{o in H} (C[v+o] + C[v-o]) cos theta_j(o)
//   Im S_j = sum_{o in H} (C[v+o] - C[v-o]) sin theta_j(o)
// with H the centre plus the lexicographically positive half of B (the
// centre's cos entry is 1/2 because it is counted as +o and -o).  Both are
// dense contractions of a [rows x |H|] matrix of small integers with a fixed
// [|H| x D] table, which is what the matrix cores do: counts are exact in
// fp16, the table is one fp16 term (VECKM_FP16) or an fp16 hi/lo pair
// (VECKM_FP32), products are exact and every sum is fp32.  N(v) comes from
// the same A operand against a weight column (1 per offset, 1/2 for the
// centre, 0 for padding), also exact.
//
// Work decomposition: the (x, y, t) grid is cut into bricks.  A persistent
// block takes whole bricks from a device counter, stages the brick's counts
// plus the window halo into LDS as fp16, and runs its query voxels in chunks
// of up to 128/256 rows.  The table streams through LDS one 32-offset slab
// at a time (double buffered), shared by the 4 waves of the block.  Each
// wave owns 64 rows (4 MFMA row tiles) and up to 64 frequencies.
#include <hip/hip_runtime.h>

#include "veckm_internal.h"

namespace veckm {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

struct EncArgs {
  SliceGeom g;
  Brick b;
  int rx, ry, rt;
  int K, nsteps;
  int SX, SY, ST, vol;
  int D;
  const int32_t* count;
  const int32_t* ulist;
  const int32_t* brick_nq;
  const int32_t* brick_off;
  const uint4* frag;
  const int32_t* delta;
  void* rows;
  int32_t* plan;
};

__device__ inline half8 as_half8(uint4 u) {
  half8 h;
  __builtin_memcpy(&h, &u, 16);
  return h;
}

__device__ inline uint16_t f32_to_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// Copies one k-step slab of the phase table from global memory straight into
// LDS (gfx950 global_load_lds_dwordx4: no registers, completion tracked by
// vmcnt).  Each wave moves 1 KB runs; the LDS base of a run is wave-uniform.
template <int SLAB_U4>
__device__ inline void issue_slab(const uint4* src, int, uint4* dst, int wid, int lane) {
#pragma unroll
  for (int u = 0; u < (SLAB_U4 + 255) / 256; ++u) {
    const int base = u * 256 + wid * 64;
    if (SLAB_U4 % 256 == 0 || base < SLAB_U4)
      __builtin_amdgcn_global_load_lds(src + base + lane, dst + base, 16, 0, 0);
  }
}

template <int NA, int NT>
struct EncShape {
  static constexpr int NTW = NT < 4 ? NT : 4;  // frequency tiles per wave
  static constexpr int WN = NT / NTW;           // waves across frequencies
  static constexpr int WM = 4 / WN;             // waves across rows
  static constexpr int CH = WM * 64;            // rows per chunk
  static constexpr int MT = 4;                  // 16-row tiles per wave
  static constexpr int SLAB_U4 = NA * NT * 64;  // uint4 per 32-offset slab
};

template <int NA, int NT, bool BF16OUT>
__global__ __launch_bounds__(256) void k_encode(EncArgs a) {
  using S = EncShape<NA, NT>;
  constexpr int NTW = S::NTW, WN = S::WN, CH = S::CH, MT = S::MT, SLAB_U4 = S::SLAB_U4;
  extern __shared__ __align__(16) unsigned char smem[];
  uint4* slab = reinterpret_cast<uint4*>(smem);
  int32_t* delta_l = reinterpret_cast<int32_t*>(slab + 2 * SLAB_U4);
  int32_t* rowbase = delta_l + a.nsteps * 32;
  int32_t* item = rowbase + CH;
  _Float16* vol = reinterpret_cast<_Float16*>(item + 4);

  const int tid = threadIdx.x, lane = tid & 63;
  const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wn = wid % WN, wm = wid / WN;
  const int KP = a.nsteps * 32;
  const int BV = a.b.bx * a.b.by * a.b.bt;
  const int D = a.D;
  for (int k = tid; k < KP; k += 256) delta_l[k] = a.delta[k];

  for (;;) {
    if (tid == 0) item[0] = atomicAdd(&a.plan[1], 1);
    __syncthreads();
    const int bid = item[0];
    if (bid >= a.g.nbricks) break;
    const int nq = a.brick_nq[bid];
    if (nq == 0) {
      __syncthreads();
      continue;
    }
    const int row0 = a.brick_off[bid];

    // ---- stage the brick's counts (with halo) into LDS as fp16
    {
      const int bxi = bid % a.g.nbx, byi = (bid / a.g.nbx) % a.g.nby,
                bti = bid / (a.g.nbx * a.g.nby);
      const int x0 = bxi * a.b.bx - a.rx, y0 = byi * a.b.by - a.ry, tb = bti * a.b.bt - a.rt;
      const int nrows = a.SY * a.ST;
      const int x = x0 + lane;
      const bool xin = lane < a.SX && (unsigned)x < (unsigned)a.g.W;
      for (int r0 = wid * 8; r0 < nrows; r0 += 32) {
        int cv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int rr = r0 + u;
          const int sy = rr % a.SY, st = rr / a.SY;
          const int y = y0 + sy, t = tb + st;
          cv[u] = 0;
          if (rr < nrows && xin && (unsigned)y < (unsigned)a.g.H && (unsigned)t < (unsigned)a.g.T)
            cv[u] = a.count[(t * a.g.H + y) * a.g.W + x];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int rr = r0 + u;
          if (rr < nrows && lane < a.SX) vol[rr * a.SX + lane] = (_Float16)(float)cv[u];
        }
      }
    }

    for (int c0 = 0; c0 < nq; c0 += CH) {
      // ---- LDS index of each row's voxel (padding rows reuse row c0)
      for (int r = tid; r < CH; r += 256) {
        const int rr = c0 + r < nq ? c0 + r : c0;
        const int li = a.ulist[(int64_t)bid * BV + rr];
        const int lx = li % a.b.bx, ly = (li / a.b.bx) % a.b.by, lt = li / (a.b.bx * a.b.by);
        rowbase[r] = ((lt + a.rt) * a.SY + (ly + a.ry)) * a.SX + (lx + a.rx);
      }
      issue_slab<SLAB_U4>(a.frag, 0, slab, wid, lane);
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      __syncthreads();

      int rb[MT];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) rb[mt] = rowbase[wm * 64 + mt * 16 + (lane & 15)];

      floatx4 accR[MT][NTW], accI[MT][NTW], accN[MT];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        accN[mt] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int nt = 0; nt < NTW; ++nt) {
          accR[mt][nt] = floatx4{0.f, 0.f, 0.f, 0.f};
          accI[mt][nt] = floatx4{0.f, 0.f, 0.f, 0.f};
        }
      }

      for (int ks = 0; ks < a.nsteps; ++ks) {
        const int buf = ks & 1;
        const bool more = ks + 1 < a.nsteps;
        // A operands: pair sums and differences of counts at +o / -o
        const int kg = ks * 32 + 8 * (lane >> 4);
        const int4 d0 = *reinterpret_cast<const int4*>(delta_l + kg);
        const int4 d1 = *reinterpret_cast<const int4*>(delta_l + kg + 4);
        const int dk[8] = {d0.x, d0.y, d0.z, d0.w, d1.x, d1.y, d1.z, d1.w};
        half8 aS[MT], aD[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const _Float16 p = vol[rb[mt] + dk[e]];
            const _Float16 q = vol[rb[mt] - dk[e]];
            aS[mt][e] = p + q;
            aD[mt][e] = p - q;
          }
        }
        half8 bw;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int k = kg + e;
          bw[e] = k < a.K ? (k == 0 ? (_Float16)0.5f : (_Float16)1.0f) : (_Float16)0.0f;
        }
        // B operands of this step, then start fetching the next slab into
        // the other buffer while the matrix cores work
        const uint4* sb = slab + buf * SLAB_U4;
        half8 bf[NA][NTW];
#pragma unroll
        for (int nt = 0; nt < NTW; ++nt)
#pragma unroll
          for (int q = 0; q < NA; ++q) bf[q][nt] = as_half8(sb[(q * NT + wn * NTW + nt) * 64 + lane]);
        if (more) issue_slab<SLAB_U4>(a.frag + (size_t)(ks + 1) * SLAB_U4, 0,
                                      slab + (buf ^ 1) * SLAB_U4, wid, lane);
#pragma unroll
        for (int nt = 0; nt < NTW; ++nt) {
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) {
            if constexpr (NA == 4) {
              accR[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(aS[mt], bf[0][nt], accR[mt][nt], 0, 0, 0);
              accI[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(aD[mt], bf[2][nt], accI[mt][nt], 0, 0, 0);
            } else {
              accR[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(aS[mt], bf[0][nt], accR[mt][nt], 0, 0, 0);
              accI[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(aD[mt], bf[1][nt], accI[mt][nt], 0, 0, 0);
            }
          }
        }
        if constexpr (NA == 4) {
#pragma unroll
          for (int nt = 0; nt < NTW; ++nt)
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
              accR[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(aS[mt], bf[1][nt], accR[mt][nt], 0, 0, 0);
              accI[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(aD[mt], bf[3][nt], accI[mt][nt], 0, 0, 0);
            }
        }
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
          accN[mt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(aS[mt], bw, accN[mt], 0, 0, 0);
        if (more) asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
      }

      // ---- normalise by the neighbour count and write the rows
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int r = wm * 64 + mt * 16 + 4 * (lane >> 4) + i;
          if (c0 + r >= nq) continue;
          const float cnt = accN[mt][i];
          const float rc = __builtin_amdgcn_rcpf(cnt);
          // x / cnt: reciprocal estimate plus one residual correction (exact
          // for x = cnt, so an all-ones feature still gives exactly 1)
          auto div = [cnt, rc](float x) {
            const float q = x * rc;
            return fmaf(fmaf(-q, cnt, x), rc, q);
          };
          const int64_t u = (int64_t)(row0 + c0 + r) * (2 * D);
#pragma unroll
          for (int nt = 0; nt < NTW; ++nt) {
            const int j = (wn * NTW + nt) * 16 + (lane & 15);
            const float re = div(accR[mt][nt][i]), im = div(accI[mt][nt][i]);
            if constexpr (BF16OUT) {
              uint16_t* out = static_cast<uint16_t*>(a.rows);
              out[u + j] = f32_to_bf16_rne(re);
              out[u + D + j] = f32_to_bf16_rne(im);
            } else {
              float* out = static_cast<float*>(a.rows);
              out[u + j] = re;
              out[u + D + j] = im;
            }
          }
        }
      }
    }
    __syncthreads();
  }
}

template <int NA, int NT>
static size_t encode_lds_bytes(const EncodeTables& et, int vol) {
  using S = EncShape<NA, NT>;
  return (size_t)2 * S::SLAB_U4 * 16 + (size_t)et.KP * 4 + (size_t)S::CH * 4 + 16 +
         ((size_t)vol * 2 + 15) / 16 * 16;
}

template <int NA, int NT>
static int launch_t(const EncArgs& a, const EncodeTables& et, bool bf16, int num_cus,
                    hipStream_t s) {
  const size_t lds = encode_lds_bytes<NA, NT>(et, a.vol);
  if (lds > 160 * 1024) return VECKM_E_INVAL;
  const void* fn = bf16 ? reinterpret_cast<const void*>(&k_encode<NA, NT, true>)
                        : reinterpret_cast<const void*>(&k_encode<NA, NT, false>);
  if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return VECKM_E_HIP;
  int per_cu = (int)((160 * 1024) / lds);
  per_cu = per_cu < 1 ? 1 : (per_cu > 2 ? 2 : per_cu);
  int grid = num_cus * per_cu;
  if (grid > a.g.nbricks) grid = a.g.nbricks;
  if (bf16)
    hipLaunchKernelGGL((k_encode<NA, NT, true>), dim3(grid), dim3(256), lds, s, a);
  else
    hipLaunchKernelGGL((k_encode<NA, NT, false>), dim3(grid), dim3(256), lds, s, a);
  return hipGetLastError() == hipSuccess ? VECKM_OK : VECKM_E_HIP;
}

template <int NA>
static int dispatch_nt(const EncArgs& a, const EncodeTables& et, bool bf16, int num_cus,
                       hipStream_t s) {
  switch (a.D / 16) {
    case 1: return launch_t<NA, 1>(a, et, bf16, num_cus, s);
    case 2: return launch_t<NA, 2>(a, et, bf16, num_cus, s);
    case 3: return launch_t<NA, 3>(a, et, bf16, num_cus, s);
    case 4: return launch_t<NA, 4>(a, et, bf16, num_cus, s);
    case 8: return launch_t<NA, 8>(a, et, bf16, num_cus, s);
    case 16: return launch_t<NA, 16>(a, et, bf16, num_cus, s);
    default: return VECKM_E_INVAL;
  }
}

int launch_encode(const SliceGeom& g, const Workspace& w, const EncodeTables& et,
                  bool bf16_rows, int num_cus, void* stream) {
  EncArgs a;
  a.g = g;
  a.b = et.brick;
  a.rx = et.rx;
  a.ry = et.ry;
  a.rt = et.rt;
  a.K = et.K;
  a.nsteps = et.KP / kKStep;
  a.SX = et.brick.bx + 2 * et.rx;
  a.SY = et.brick.by + 2 * et.ry;
  a.ST = et.brick.bt + 2 * et.rt;
  a.vol = a.SX * a.SY * a.ST;
  a.D = et.d;
  a.count = w.count;
  a.ulist = w.ulist;
  a.brick_nq = w.brick_nq;
  a.brick_off = w.brick_off;
  a.frag = reinterpret_cast<const uint4*>(et.frag);
  a.delta = et.delta;
  a.rows = w.rows;
  a.plan = w.plan;
  if (a.SX > 64) return VECKM_E_INVAL;  // one wavefront stages one x row
  hipStream_t s = (hipStream_t)stream;
  return et.na == 4 ? dispatch_nt<4>(a, et, bf16_rows, num_cus, s)
                    : dispatch_nt<2>(a, et, bf16_rows, num_cus, s);
}

}  // namespace veckm
