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
// (VECKM_FP32), products are exact and every sum is fp32.  N(v) is the same
// pair sums against slot weights (1 per offset, 1/2 for the centre, 0 for
// padding), summed exactly in fp32 on the vector ALU.
//
// Work decomposition: the (x, y, t) grid of every slice is cut into bricks,
// and the bricks of all slices of a call form one work list.  A persistent
// block of 16 waves (4 per SIMD) takes whole bricks from a device counter,
// copies the brick's counts plus the window halo from the pair grid into
// LDS, and runs the brick's query voxels in chunks of up to 512 rows (256
// at D = 128, 128 at D = 256).  The table streams through LDS one 32-offset
// slab per MFMA k-step, NBUF slabs deep, shared by the waves.  Each wave
// owns 2 row tiles of 16 rows and up to 64 frequencies; with four waves per
// SIMD, one wave's count gathers overlap another's matrix products.
#include <hip/hip_runtime.h>

#include "slices.h"
#include "sync.h"
#include "veckm_internal.h"

namespace veckm {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

struct EncArgs {
  Batch bt;
  Brick b;
  int rx, ry, rt;
  int K, nsteps;
  int SX, SY, ST, vol;
  int D;
  const int32_t* ulist;
  const int4* order;  // work list: {brick, rows, first row, slice}, or for single rows
                      // {kSparseTag | item, rows, first row, first entry of srow}
  const int2* srow;   // {brick, brick-local voxel} of each single row
  const int32_t* runs1;  // run offsets of a single voxel's count box
  int SX1, SY1, ST1, vol1;  // that box (x width, y and t extents, dwords)
  int lds_slices;     // slices whose descriptors are copied to LDS (0: read them from global)
  const uint4* frag;
  const int32_t* runs;
  const uint16_t* wts;
  const uint32_t* pairs;
  const uint32_t* zeros;
  void* rows;
  int32_t* plan;
  int32_t* rowcnt;  // per-row neighbour counts, or NULL
  // the perceptron, when the encoder runs it (kFlow* rows)
  const uint4* w1frag;  // hidden / 32 slabs (make_w1_fragments)
  int msteps;           // hidden / 32
  int hidden;
  float unscale;        // 2^-shift of the hi/lo W1
  const float* b1;
  const float* W2;
  const float* b2;
  float2* rowflow;      // one flow per row
};

__host__ __device__ constexpr bool fused_rows(int rows) { return rows == kFlowBF16 || rows == kFlowHiLo16; }
// LDS bytes of the perceptron's constants (b1 and both rows of W2)
__host__ __device__ constexpr size_t mlp_lds_bytes(int hidden) { return (size_t)hidden * 12; }

__device__ inline half8 as_half8(uint4 u) {
  half8 h;
  __builtin_memcpy(&h, &u, 16);
  return h;
}

// (p.lo + q.hi, p.hi + q.lo) and (p.lo - q.hi, p.hi - q.lo) on packed fp16:
// the -o run comes out of the pair layout half-swapped, and the swap is free
// (the compiler folds it into the packed add's operand selects).  Exact for
// the integer counts used here (<= 2048).
typedef _Float16 half2v __attribute__((ext_vector_type(2)));

__device__ inline uint32_t pk_sum_swapped(uint32_t p, uint32_t q) {
  half2v a, b;
  __builtin_memcpy(&a, &p, 4);
  __builtin_memcpy(&b, &q, 4);
  const half2v r = a + __builtin_shufflevector(b, b, 1, 0);
  uint32_t o;
  __builtin_memcpy(&o, &r, 4);
  return o;
}
__device__ inline uint32_t pk_diff_swapped(uint32_t p, uint32_t q) {
  half2v a, b;
  __builtin_memcpy(&a, &p, 4);
  __builtin_memcpy(&b, &q, 4);
  const half2v r = a - __builtin_shufflevector(b, b, 1, 0);
  uint32_t o;
  __builtin_memcpy(&o, &r, 4);
  return o;
}

__device__ inline uint16_t f32_to_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// s_waitcnt immediate (gfx9 encoding) waiting until at most n vector memory
// operations are outstanding; expcnt and lgkmcnt are left unconstrained.
constexpr int vmcnt_imm(int n) { return (n & 15) | ((n >> 4) << 14) | (7 << 4) | (15 << 8); }
// ... and until at most n (<= 15) LDS operations are outstanding (vmcnt and
// expcnt unconstrained).
constexpr int lgkmcnt_imm(int n) { return 15 | (3 << 14) | (7 << 4) | ((n & 15) << 8); }

// Waves per block and the most 16-frequency tiles one wave holds (layouts 0
// and 1; layout 2 holds up to 8).
constexpr int kEncWaves = 16;
constexpr int kEncMaxNtw = 4;
// 16-row tiles each wave holds per chunk.
constexpr int kEncMt = 2;
// With four slab buffers, take the k-steps in pairs: one barrier per pair.
constexpr bool kEncPairSteps = true;

// LDS byte offset of the slice descriptors (after `bytes` of everything else).
__host__ __device__ constexpr size_t slice_table_offset(size_t bytes) { return (bytes + 15) & ~size_t(15); }

// Wave layouts of the encoder block: 0 = 16 waves (4 per SIMD) of kEncMt
// row tiles each; 1 = 8 waves (2 per SIMD) of 2 kEncMt row tiles each
// (every table fragment read from LDS feeds twice the products; half the
// waves to hide latency); 2 = 4 waves (one per SIMD) of 2 kEncMt row tiles
// over up to 8 frequency tiles (128 frequencies: every count gather feeds
// all of a row's frequencies, every table fragment four row tiles; the
// accumulators take the register file's accumulation half); 3 = 8 waves of
// kEncMt row tiles and 4 = 16 waves of one row tile, each over every
// frequency of its rows (more waves to hide latency, 128 registers each).
constexpr int enc_waves(int L) {
  return L == 0 || L == 4 ? kEncWaves : L == 1 ? kEncWaves / 2 : L == 2 ? kEncWaves / 4 : kEncWaves / 2;
}
constexpr int enc_mt(int L) { return L == 4 ? kEncMt / 2 : L == 0 || L == 3 ? kEncMt : 2 * kEncMt; }
constexpr int enc_max_ntw(int L) { return L >= 2 ? 2 * kEncMaxNtw : kEncMaxNtw; }
// layouts whose k-steps are software-pipelined within each wave
constexpr bool enc_pipelined(int L) { return L >= 2; }

template <int NA, int NT, int L>
struct EncShape {
  static constexpr int NW = enc_waves(L);       // waves per block
  static constexpr int NTW = NT < enc_max_ntw(L) ? NT : enc_max_ntw(L);  // frequency tiles per wave
  static constexpr int WN = NT / NTW;           // waves across frequencies (layouts 0, 1: 2 at D = 128, 4 at D = 256)
  static constexpr int WM = NW / WN;            // waves across rows
  static constexpr int MT = enc_mt(L);          // 16-row tiles per wave
  static constexpr int CH = WM * MT * 16;       // rows per chunk
  static constexpr int SLAB_U4 = NA * NT * 64;  // uint4 per 32-slot slab
  static constexpr int PFW = SLAB_U4 / (NW * 64);  // copies per wave per slab
  static constexpr bool EVEN = SLAB_U4 % (NW * 64) == 0;
};

// Starts the copy of one k-step slab of the phase table from global memory
// straight into LDS (no registers; completion tracked by vmcnt).  Each wave
// moves 1 KB pieces.
template <int SLAB_U4, int NW>
__device__ inline void issue_slab(const uint4* src, uint4* dst, int wid, int lane) {
  const uint32_t voff = (uint32_t)lane * 16;
#pragma unroll
  for (int u = 0; u < (SLAB_U4 + NW * 64 - 1) / (NW * 64); ++u) {
    const int base = u * NW * 64 + wid * 64;
    if (SLAB_U4 % (NW * 64) == 0 || base < SLAB_U4)
      copy_to_lds16_s(src + base, voff, lds_offset(dst + base));
  }
}

// Waits until every slab copy of this wave except those of the newest
// `newer` slabs (0..2) has landed; vector memory loads complete in order.
template <int PFW>
__device__ inline void wait_slabs(int newer) {
  static_assert(2 * PFW <= 63, "copies in flight exceed the wait counter");
  if (newer >= 2)
    __builtin_amdgcn_s_waitcnt(vmcnt_imm(2 * PFW));
  else if (newer == 1)
    __builtin_amdgcn_s_waitcnt(vmcnt_imm(PFW));
  else
    __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));
}

// The count words of one k-step for MTV row tiles: for each tile, the lane's
// two +o runs (4 consecutive voxels each, two aligned pair dwords per run)
// and their -o partners.  Only the brick's count box and the run offsets are
// read, both fixed for the brick, so the next step's words can be fetched
// while the current step multiplies.
template <int MTV>
struct CountWords {
  uint32_t P[MTV > 0 ? MTV : 1][4], Q[MTV > 0 ? MTV : 1][4];
  __device__ inline void fetch(const int32_t* runs_l, const uint32_t* vol2, const int* rb, int ks,
                               int g) {
    fetch_at(*reinterpret_cast<const int2*>(runs_l + (ks * 4 + g) * 2), vol2, rb);
  }
  // the words of the two runs starting at box offsets ro.x and ro.y
  __device__ inline void fetch_at(int2 ro, const uint32_t* vol2, const int* rb) {
#pragma unroll
    for (int mt = 0; mt < MTV; ++mt) {
      const uint32_t* p0 = vol2 + (rb[mt] + ro.x);
      const uint32_t* p1 = vol2 + (rb[mt] + ro.y);
      const uint32_t* q0 = vol2 + (rb[mt] - ro.x - 3);
      const uint32_t* q1 = vol2 + (rb[mt] - ro.y - 3);
      P[mt][0] = p0[0];
      P[mt][1] = p0[2];
      P[mt][2] = p1[0];
      P[mt][3] = p1[2];
      Q[mt][0] = q0[2];
      Q[mt][1] = q0[0];
      Q[mt][2] = q1[2];
      Q[mt][3] = q1[0];
    }
  }
};

// The k-steps of one chunk for a wave that holds MTV valid 16-row tiles
// (0 <= MTV <= MT; no per-tile branches inside).  Every wave runs it: a wave
// without rows still moves its share of each slab and meets every barrier.
// On entry the first slab is in LDS and the next NBUF - 2 are in flight.
//
// The table is the MFMA A operand and the counts the B operand, so that the
// accumulator of a lane holds 4 consecutive frequencies of one row (the
// lane's row is lane & 15): the count of that row arrives in the same lane
// and the row is written with 16-byte stores.
// One k-step of the contraction for a wave with MTV valid row tiles: the
// count pair sums of its rows (gathered from the box), the table slab `sb`
// as A operand, and the exact neighbour count on the vector ALU.
template <int NA, int NT, int L, int MTV>
__device__ inline void kstep_compute(int ks, const uint4* sb, const int32_t* runs_l,
                                     const uint16_t* wts_l, const uint32_t* vol2,
                                     const int (&rb)[EncShape<NA, NT, L>::MT],
                                     floatx4 (&accR)[EncShape<NA, NT, L>::MT][EncShape<NA, NT, L>::NTW],
                                     floatx4 (&accI)[EncShape<NA, NT, L>::MT][EncShape<NA, NT, L>::NTW],
                                     float (&cnt)[EncShape<NA, NT, L>::MT], int wn, int lane) {
  using S = EncShape<NA, NT, L>;
  constexpr int NTW = S::NTW;
  const int g = lane >> 4;
  CountWords<MTV> cw;
  if constexpr (MTV > 0) {
    cw.fetch(runs_l, vol2, rb, ks, g);
    // pair sums and differences of counts at +o / -o: the -o run comes out
    // of the pair layout descending and half-swapped
    half8 cS[MTV], cD[MTV];
#pragma unroll
    for (int mt = 0; mt < MTV; ++mt) {
      uint4 s4, d4;
      s4.x = pk_sum_swapped(cw.P[mt][0], cw.Q[mt][0]);
      s4.y = pk_sum_swapped(cw.P[mt][1], cw.Q[mt][1]);
      s4.z = pk_sum_swapped(cw.P[mt][2], cw.Q[mt][2]);
      s4.w = pk_sum_swapped(cw.P[mt][3], cw.Q[mt][3]);
      d4.x = pk_diff_swapped(cw.P[mt][0], cw.Q[mt][0]);
      d4.y = pk_diff_swapped(cw.P[mt][1], cw.Q[mt][1]);
      d4.z = pk_diff_swapped(cw.P[mt][2], cw.Q[mt][2]);
      d4.w = pk_diff_swapped(cw.P[mt][3], cw.Q[mt][3]);
      cS[mt] = as_half8(s4);
      cD[mt] = as_half8(d4);
    }
    const half8 bw = *reinterpret_cast<const half8*>(wts_l + ks * 32 + 8 * g);
#pragma unroll
    for (int nt = 0; nt < NTW; ++nt) {
      half8 tf[NA];
#pragma unroll
      for (int q = 0; q < NA; ++q) tf[q] = as_half8(sb[(q * NT + wn * NTW + nt) * 64 + lane]);
#pragma unroll
      for (int mt = 0; mt < MTV; ++mt) {
        if constexpr (NA == 4) {
          accR[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(tf[0], cS[mt], accR[mt][nt], 0, 0, 0);
          accI[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(tf[2], cD[mt], accI[mt][nt], 0, 0, 0);
          accR[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(tf[1], cS[mt], accR[mt][nt], 0, 0, 0);
          accI[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(tf[3], cD[mt], accI[mt][nt], 0, 0, 0);
        } else {
          accR[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(tf[0], cS[mt], accR[mt][nt], 0, 0, 0);
          accI[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(tf[1], cD[mt], accI[mt][nt], 0, 0, 0);
        }
      }
    }
    // neighbour count: the slot weights (1, 1/2 for the centre, 0 for
    // padding) against the pair sums, exact in fp32; the lane covers its 8
    // slots of the row, the 4 lanes of a row are added after the loop
#pragma unroll
    for (int mt = 0; mt < MTV; ++mt)
#pragma unroll
      for (int e = 0; e < 4; ++e)
        cnt[mt] = __builtin_amdgcn_fdot2(half2v{bw[2 * e], bw[2 * e + 1]},
                                         half2v{cS[mt][2 * e], cS[mt][2 * e + 1]}, cnt[mt], false);
  }
}

// The k-steps of one chunk for a wave that holds MTV valid 16-row tiles
// (0 <= MTV <= MT; no per-tile branches inside).  Every wave runs it: a wave
// without rows still moves its share of each slab and meets every barrier.
// On entry the first slab is in LDS and the next NBUF - 2 are in flight.
//
// The table is the MFMA A operand and the counts the B operand, so that the
// accumulator of a lane holds 4 consecutive frequencies of one row (the
// lane's row is lane & 15): the count of that row arrives in the same lane
// and the row is written with 16-byte stores.
template <int NA, int NT, int L, int NBUF, int MTV>
__device__ inline void chunk_ksteps(int nsteps, const uint4* frag, uint4* slab,
                                    const int32_t* runs_l, const uint16_t* wts_l,
                                    const uint32_t* vol2, const int (&rb)[EncShape<NA, NT, L>::MT],
                                    floatx4 (&accR)[EncShape<NA, NT, L>::MT][EncShape<NA, NT, L>::NTW],
                                    floatx4 (&accI)[EncShape<NA, NT, L>::MT][EncShape<NA, NT, L>::NTW],
                                    float (&cnt)[EncShape<NA, NT, L>::MT], int wn, int wid,
                                    int lane) {
  using S = EncShape<NA, NT, L>;
  constexpr int NW = S::NW, SLAB_U4 = S::SLAB_U4, PFW = S::PFW;
  if constexpr (kEncPairSteps && NBUF == 4) {
    // two k-steps per barrier: the slabs of the next pair go into the two
    // buffers the previous pair used (free since the last barrier) and land
    // while this pair multiplies; on entry slabs 0 and 1 are in LDS
    for (int ks = 0; ks < nsteps; ks += 2) {
#pragma unroll
      for (int u = 2; u < 4; ++u)
        if (ks + u < nsteps)
          issue_slab<SLAB_U4, NW>(frag + (size_t)(ks + u) * SLAB_U4,
                                  slab + ((ks + u) % 4) * SLAB_U4, wid, lane);
      kstep_compute<NA, NT, L, MTV>(ks, slab + (ks % 4) * SLAB_U4, runs_l, wts_l, vol2, rb, accR,
                                 accI, cnt, wn, lane);
      if (ks + 1 < nsteps)
        kstep_compute<NA, NT, L, MTV>(ks + 1, slab + ((ks + 1) % 4) * SLAB_U4, runs_l, wts_l, vol2,
                                   rb, accR, accI, cnt, wn, lane);
      __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));  // the next pair has landed
      lds_barrier();
    }
  } else {
    constexpr int AHEAD = NBUF - 1;
    for (int ks = 0; ks < nsteps; ++ks) {
      // start the slab AHEAD steps out now, so that it lands during this
      // step: its buffer was last read in step ks - 1, before the last barrier
      if (ks + AHEAD < nsteps)
        issue_slab<SLAB_U4, NW>(frag + (size_t)(ks + AHEAD) * SLAB_U4,
                                slab + ((ks + AHEAD) % NBUF) * SLAB_U4, wid, lane);
      kstep_compute<NA, NT, L, MTV>(ks, slab + (ks % NBUF) * SLAB_U4, runs_l, wts_l, vol2, rb, accR,
                                 accI, cnt, wn, lane);
      // make sure the slab of step ks + 1 has landed (slabs ks + 2 .. ks +
      // AHEAD may stay in flight)
      const int last = ks + AHEAD < nsteps - 1 ? ks + AHEAD : nsteps - 1;  // newest slab issued
      wait_slabs<PFW>(last - ks - 1 > 0 ? last - ks - 1 : 0);
      lds_barrier();
    }
  }
}

// Dispatches on the wave's number of valid row tiles (wave-uniform).
template <int NA, int NT, int L, int NBUF, int M>
__device__ inline void chunk_ksteps_n(int mtv, int nsteps, const uint4* frag, uint4* slab,
                                      const int32_t* runs_l, const uint16_t* wts_l,
                                      const uint32_t* vol2, const int (&rb)[EncShape<NA, NT, L>::MT],
                                      floatx4 (&accR)[EncShape<NA, NT, L>::MT][EncShape<NA, NT, L>::NTW],
                                      floatx4 (&accI)[EncShape<NA, NT, L>::MT][EncShape<NA, NT, L>::NTW],
                                      float (&cnt)[EncShape<NA, NT, L>::MT], int wn, int wid,
                                      int lane) {
  if constexpr (M == 0) {
    chunk_ksteps<NA, NT, L, NBUF, 0>(nsteps, frag, slab, runs_l, wts_l, vol2, rb, accR, accI, cnt,
                                  wn, wid, lane);
  } else {
    if (mtv == M)
      chunk_ksteps<NA, NT, L, NBUF, M>(nsteps, frag, slab, runs_l, wts_l, vol2, rb, accR, accI, cnt,
                                    wn, wid, lane);
    else
      chunk_ksteps_n<NA, NT, L, NBUF, M - 1>(mtv, nsteps, frag, slab, runs_l, wts_l, vol2, rb, accR,
                                          accI, cnt, wn, wid, lane);
  }
}

// ---- layout 2: software-pipelined k-steps (one wave per SIMD) -----------
//
// With one wave per SIMD nothing else hides a wave's LDS latency, so every
// load is issued a stage ahead of its use: the count words of k-step ks + 1
// (the box is resident for the whole brick) while step ks multiplies, and the
// table fragments of frequency tile nt + kTfAhead while tile nt multiplies.
// Each accumulator still receives exactly the products of layouts 0 and 1 in
// the same order, so the results are bit-identical to theirs.
constexpr int kTfAhead = 1;  // frequency tiles of table fragments in flight

// Pair sums and differences of one k-step's count words (see kstep_compute).
template <int MTV>
__device__ inline void pair_sums(const CountWords<MTV>& cw, half8 (&cS)[MTV > 0 ? MTV : 1],
                                 half8 (&cD)[MTV > 0 ? MTV : 1]) {
#pragma unroll
  for (int mt = 0; mt < MTV; ++mt) {
    uint4 s4, d4;
    s4.x = pk_sum_swapped(cw.P[mt][0], cw.Q[mt][0]);
    s4.y = pk_sum_swapped(cw.P[mt][1], cw.Q[mt][1]);
    s4.z = pk_sum_swapped(cw.P[mt][2], cw.Q[mt][2]);
    s4.w = pk_sum_swapped(cw.P[mt][3], cw.Q[mt][3]);
    d4.x = pk_diff_swapped(cw.P[mt][0], cw.Q[mt][0]);
    d4.y = pk_diff_swapped(cw.P[mt][1], cw.Q[mt][1]);
    d4.z = pk_diff_swapped(cw.P[mt][2], cw.Q[mt][2]);
    d4.w = pk_diff_swapped(cw.P[mt][3], cw.Q[mt][3]);
    cS[mt] = as_half8(s4);
    cD[mt] = as_half8(d4);
  }
}

// What the fused perceptron needs inside a chunk (kFlow* rows).
struct FuseArgs {
  const uint4* w1frag;  // slabs of W1 fragments, after the table's k-steps
  int msteps;           // W1 slabs: two hidden tiles of 16 units each
  float unscale;
  const float* mlp_l;   // LDS: b1[hidden], W2[0][hidden], W2[1][hidden]
  int hidden;
  float b20, b21;
  float2* out;          // rowflow
  int row_first;        // row index of the chunk's first row
  int nr;               // rows in the chunk
  int wm;               // this wave's row group
};

typedef __bf16 bf16x8_e __attribute__((ext_vector_type(8)));

__device__ inline uint32_t pack_bf16x2(float a, float b) {
  return f32_to_bf16_rne(a) | ((uint32_t)f32_to_bf16_rne(b) << 16);
}

// Source of step `st` of a chunk's slab sequence: the table's k-steps, then
// (fused) the W1 slabs.
template <int SLAB_U4>
__device__ inline const uint4* step_src(const uint4* frag, const uint4* w1frag, int nsteps, int st) {
  return st < nsteps ? frag + (size_t)st * SLAB_U4 : w1frag + (size_t)(st - nsteps) * SLAB_U4;
}

template <int NA, int NT, int L, int NBUF, int MTV, bool FUSE>
__device__ inline void chunk_ksteps_p(int nsteps, const uint4* frag, uint4* slab,
                                      const int32_t* runs_l, const uint16_t* wts_l,
                                      const uint32_t* vol2, const int (&rb)[EncShape<NA, NT, L>::MT],
                                      floatx4 (&accR)[EncShape<NA, NT, L>::MT][EncShape<NA, NT, L>::NTW],
                                      floatx4 (&accI)[EncShape<NA, NT, L>::MT][EncShape<NA, NT, L>::NTW],
                                      float (&cnt)[EncShape<NA, NT, L>::MT], int wn, int wid,
                                      int lane, const FuseArgs& fz) {
  using S = EncShape<NA, NT, L>;
  constexpr int NW = S::NW, NTW = S::NTW, SLAB_U4 = S::SLAB_U4, PFW = S::PFW, WM = S::WM;
  constexpr int AHEAD = NBUF - 1;
  // (the 16-wave layout reads each tile's fragments just before its
  // products: four waves per SIMD hide the wait, and with a second set of
  // fragments its registers spill past 128)
  constexpr int TA = L == 4 ? 0 : kTfAhead < NTW ? kTfAhead : NTW - 1;
  const int g = lane >> 4;
  const int total = FUSE ? nsteps + fz.msteps : nsteps;  // slabs through the ring
  const int2* runs2 = reinterpret_cast<const int2*>(runs_l);
  static_assert(NBUF == 2, "the pipelined layout keeps one slab in flight");
  CountWords<MTV> cw;
  int2 ro_next = make_int2(0, 0);
  if constexpr (MTV > 0) {
    cw.fetch_at(runs2[g], vol2, rb);
    if (nsteps > 1) ro_next = runs2[4 + g];
  }
  for (int ks = 0; ks < nsteps; ++ks) {
    // Nothing of this wave is in flight here (with two slab buffers each step
    // ends waiting for the next slab), so this wait costs nothing; it tells
    // the compiler's wait insertion, which does not see the slab copies, that
    // loads it placed before the loop (spill reloads) are complete, instead of
    // a full wait after the copies below on every step.
    __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));
    // the slab AHEAD steps out: its buffer was last read in step ks - 1
    if (ks + AHEAD < total)
      issue_slab<SLAB_U4, NW>(step_src<SLAB_U4>(frag, fz.w1frag, nsteps, ks + AHEAD),
                              slab + ((ks + AHEAD) % NBUF) * SLAB_U4, wid, lane);
    if constexpr (MTV > 0) {
      const uint4* sb = slab + (ks % NBUF) * SLAB_U4;
      const half8 bw = *reinterpret_cast<const half8*>(wts_l + ks * 32 + 8 * g);
      half8 cS[MTV], cD[MTV];
      pair_sums<MTV>(cw, cS, cD);
      // LDS reads complete in the order they were issued (and a wait can
      // leave at most 15 of them outstanding), so the next step's count
      // words are gathered only once this step's last table fragments have
      // landed, just before the last frequency tile's products, which then
      // cover their latency; issued earlier, they would hold up every table
      // fragment behind them
      auto gather_next = [&]() {
        if (ks + 1 < nsteps) {
          cw.fetch_at(ro_next, vol2, rb);
          if (ks + 2 < nsteps) ro_next = runs2[(ks + 2) * 4 + g];
        }
      };
      // table fragments kTfAhead frequency tiles ahead of the products
      half8 tf[TA + 1][NA];
#pragma unroll
      for (int u = 0; u < TA; ++u)
#pragma unroll
        for (int q = 0; q < NA; ++q) tf[u][q] = as_half8(sb[(q * NT + wn * NTW + u) * 64 + lane]);
#pragma unroll
      for (int nt = 0; nt < NTW; ++nt) {
        if (nt + TA < NTW)
#pragma unroll
          for (int q = 0; q < NA; ++q)
            tf[(nt + TA) % (TA + 1)][q] = as_half8(sb[(q * NT + wn * NTW + nt + TA) * 64 + lane]);
        __builtin_amdgcn_sched_barrier(0);
        if (nt == NTW - 1) {
          __builtin_amdgcn_s_waitcnt(lgkmcnt_imm(0));  // the last fragments (requested a tile ago)
          gather_next();
          __builtin_amdgcn_sched_barrier(0);
        }
        const half8* t = tf[nt % (TA + 1)];
#pragma unroll
        for (int mt = 0; mt < MTV; ++mt) {
          if constexpr (NA == 4) {
            accR[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(t[0], cS[mt], accR[mt][nt], 0, 0, 0);
            accI[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(t[2], cD[mt], accI[mt][nt], 0, 0, 0);
            accR[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(t[1], cS[mt], accR[mt][nt], 0, 0, 0);
            accI[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(t[3], cD[mt], accI[mt][nt], 0, 0, 0);
          } else {
            accR[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(t[0], cS[mt], accR[mt][nt], 0, 0, 0);
            accI[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(t[1], cD[mt], accI[mt][nt], 0, 0, 0);
          }
        }
        __builtin_amdgcn_sched_barrier(0);
      }
#pragma unroll
      for (int mt = 0; mt < MTV; ++mt)
#pragma unroll
        for (int e = 0; e < 4; ++e)
          cnt[mt] = __builtin_amdgcn_fdot2(half2v{bw[2 * e], bw[2 * e + 1]},
                                           half2v{cS[mt][2 * e], cS[mt][2 * e + 1]}, cnt[mt], false);
    }
    // the slab of step ks + 1 has landed (later ones may stay in flight)
    const int last = ks + AHEAD < total - 1 ? ks + AHEAD : total - 1;
    wait_slabs<PFW>(last - ks - 1 > 0 ? last - ks - 1 : 0);
    lds_barrier();
  }
  if constexpr (FUSE) {
    // ---- the perceptron on the chunk's rows, still in registers (Sec. 2.1,
    //      Eqns. 5-6): x = [Re emb | Im emb] as the B operand of layer 1,
    //      W1 from the slabs that follow the table's, ReLU and layer 2 on the
    //      vector ALU.  The lane holds features 16 nt + 4 g + (0..3) of row
    //      lane & 15; layer-1 step kk takes frequency tiles 2kk' and 2kk' + 1
    //      (real parts for kk < NT / 2, imaginary parts above), the order the
    //      W1 fragments were laid out in.
    static_assert(S::WN == 1, "the fused perceptron needs every frequency of a row in one wave");
    constexpr int TERMS = NA / 2;
    constexpr int KK = NT;  // 32-feature steps of layer 1
    uint4 xh[MTV > 0 ? MTV : 1][KK], xl[TERMS == 2 && MTV > 0 ? MTV : 1][TERMS == 2 ? KK : 1];
    float p0[MTV > 0 ? MTV : 1], p1[MTV > 0 ? MTV : 1];
    if constexpr (MTV > 0) {
#pragma unroll
      for (int mt = 0; mt < MTV; ++mt) {
        float n = cnt[mt];
        n += __shfl_xor(n, 16);
        n += __shfl_xor(n, 32);
        const float rc = __builtin_amdgcn_rcpf(n);
        // x / n as the encoder's rows are (exact for x = n; 0 without neighbours)
        auto div = [n, rc](float x) {
          const float qq = x * rc;
          return n > 0.f ? fmaf(fmaf(-qq, n, x), rc, qq) : 0.f;
        };
#pragma unroll
        for (int kk = 0; kk < KK; ++kk) {
          const int t0 = 2 * (kk % (NT / 2));
          const floatx4 a0 = kk < NT / 2 ? accR[mt][t0] : accI[mt][t0];
          const floatx4 a1 = kk < NT / 2 ? accR[mt][t0 + 1] : accI[mt][t0 + 1];
          const float v[8] = {div(a0[0]), div(a0[1]), div(a0[2]), div(a0[3]),
                              div(a1[0]), div(a1[1]), div(a1[2]), div(a1[3])};
          if constexpr (TERMS == 2) {
            half8 h, l;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
              h[e] = (_Float16)v[e];
              l[e] = (_Float16)(v[e] - (float)h[e]);
            }
            __builtin_memcpy(&xh[mt][kk], &h, 16);
            __builtin_memcpy(&xl[mt][kk], &l, 16);
          } else {
            xh[mt][kk] = make_uint4(pack_bf16x2(v[0], v[1]), pack_bf16x2(v[2], v[3]),
                                    pack_bf16x2(v[4], v[5]), pack_bf16x2(v[6], v[7]));
          }
        }
        p0[mt] = 0.f;
        p1[mt] = 0.f;
      }
    }
    for (int ms = 0; ms < fz.msteps; ++ms) {
      const int st = nsteps + ms;
      __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));  // as in the k-steps: nothing in flight here
      if (st + AHEAD < total)
        issue_slab<SLAB_U4, NW>(step_src<SLAB_U4>(frag, fz.w1frag, nsteps, st + AHEAD),
                                slab + ((st + AHEAD) % NBUF) * SLAB_U4, wid, lane);
      if constexpr (MTV > 0) {
        const uint4* sb = slab + (st % NBUF) * SLAB_U4;
#pragma unroll
        for (int tile = 0; tile < 2; ++tile) {
          floatx4 h[MTV];
#pragma unroll
          for (int mt = 0; mt < MTV; ++mt) h[mt] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int kk = 0; kk < KK; ++kk) {
            const uint4 wh = sb[(tile * NT + kk) * 64 + lane];
            if constexpr (TERMS == 2) {
              const uint4 wl = sb[((2 + tile) * NT + kk) * 64 + lane];
#pragma unroll
              for (int mt = 0; mt < MTV; ++mt) {
                h[mt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(as_half8(wh), as_half8(xh[mt][kk]), h[mt], 0, 0, 0);
                h[mt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(as_half8(wl), as_half8(xh[mt][kk]), h[mt], 0, 0, 0);
                h[mt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(as_half8(wh), as_half8(xl[mt][kk]), h[mt], 0, 0, 0);
              }
            } else {
              bf16x8_e wb;
              __builtin_memcpy(&wb, &wh, 16);
#pragma unroll
              for (int mt = 0; mt < MTV; ++mt) {
                bf16x8_e xb;
                __builtin_memcpy(&xb, &xh[mt][kk], 16);
                h[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wb, xb, h[mt], 0, 0, 0);
              }
            }
          }
          // layer 2: the lane holds hidden units 16 (2 ms + tile) + 4 g + i
          const int u0 = (2 * ms + tile) * 16 + 4 * g;
          const float4 bb = *reinterpret_cast<const float4*>(fz.mlp_l + u0);
          const float4 wa = *reinterpret_cast<const float4*>(fz.mlp_l + fz.hidden + u0);
          const float4 wb2 = *reinterpret_cast<const float4*>(fz.mlp_l + 2 * fz.hidden + u0);
          const float bv[4] = {bb.x, bb.y, bb.z, bb.w}, w0[4] = {wa.x, wa.y, wa.z, wa.w},
                      w1[4] = {wb2.x, wb2.y, wb2.z, wb2.w};
#pragma unroll
          for (int mt = 0; mt < MTV; ++mt)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const float hv = fmaxf(fmaf(h[mt][i], fz.unscale, bv[i]), 0.f);
              p0[mt] = fmaf(w0[i], hv, p0[mt]);
              p1[mt] = fmaf(w1[i], hv, p1[mt]);
            }
        }
      }
      const int last = st + AHEAD < total - 1 ? st + AHEAD : total - 1;
      wait_slabs<PFW>(last - st - 1 > 0 ? last - st - 1 : 0);
      lds_barrier();
    }
    // ---- one flow per row: the 4 lanes of a row hold partial sums
    if constexpr (MTV > 0) {
#pragma unroll
      for (int mt = 0; mt < MTV; ++mt) {
        float f0 = p0[mt], f1 = p1[mt];
        f0 += __shfl_xor(f0, 16);
        f1 += __shfl_xor(f1, 16);
        f0 += __shfl_xor(f0, 32);
        f1 += __shfl_xor(f1, 32);
        const int r = (mt * WM + fz.wm) * 16 + (lane & 15);
        if (lane < 16 && r < fz.nr) fz.out[fz.row_first + r] = make_float2(f0 + fz.b20, f1 + fz.b21);
      }
    }
  }
}

template <int NA, int NT, int L, int NBUF, int M, bool FUSE>
__device__ inline void chunk_ksteps_pn(int mtv, int nsteps, const uint4* frag, uint4* slab,
                                       const int32_t* runs_l, const uint16_t* wts_l,
                                       const uint32_t* vol2, const int (&rb)[EncShape<NA, NT, L>::MT],
                                       floatx4 (&accR)[EncShape<NA, NT, L>::MT][EncShape<NA, NT, L>::NTW],
                                       floatx4 (&accI)[EncShape<NA, NT, L>::MT][EncShape<NA, NT, L>::NTW],
                                       float (&cnt)[EncShape<NA, NT, L>::MT], int wn, int wid,
                                       int lane, const FuseArgs& fz) {
  if constexpr (M == 0) {
    chunk_ksteps_p<NA, NT, L, NBUF, 0, FUSE>(nsteps, frag, slab, runs_l, wts_l, vol2, rb, accR, accI,
                                             cnt, wn, wid, lane, fz);
  } else {
    if (mtv == M)
      chunk_ksteps_p<NA, NT, L, NBUF, M, FUSE>(nsteps, frag, slab, runs_l, wts_l, vol2, rb, accR,
                                               accI, cnt, wn, wid, lane, fz);
    else
      chunk_ksteps_pn<NA, NT, L, NBUF, M - 1, FUSE>(mtv, nsteps, frag, slab, runs_l, wts_l, vol2, rb,
                                                    accR, accI, cnt, wn, wid, lane, fz);
  }
}

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef _Float16 half4v __attribute__((ext_vector_type(4)));

template <int NA, int NT, int L, int NBUF, int ROWS>
__global__ __launch_bounds__(enc_waves(L) * 64) void k_encode(EncArgs a) {
  using S = EncShape<NA, NT, L>;
  constexpr int NW = S::NW, NTW = S::NTW, WN = S::WN, WM = S::WM, MT = S::MT, CH = S::CH,
                SLAB_U4 = S::SLAB_U4, PFW = S::PFW;
  static_assert(NBUF == 2 || ((NBUF == 3 || NBUF == 4) && S::EVEN),
                "three or four slab buffers need slab copies split evenly over the waves");
  constexpr int AHEAD = NBUF - 1;  // slabs in flight beyond the one in use
  extern __shared__ __align__(16) unsigned char smem[];
  uint4* slab = reinterpret_cast<uint4*>(smem);
  int32_t* runs_l = reinterpret_cast<int32_t*>(slab + NBUF * SLAB_U4);
  int32_t* runs1_l = runs_l + a.nsteps * 8;
  uint16_t* wts_l = reinterpret_cast<uint16_t*>(runs1_l + a.nsteps * 8);
  int32_t* rowbase = reinterpret_cast<int32_t*>(wts_l + a.nsteps * 32);
  int32_t* item = rowbase + CH;
  // Count box as overlapping fp16 pairs: dword i holds the counts of box
  // voxels i and i + 1 of the same x row, so any run of 4 consecutive voxels
  // is two aligned dword reads.  Box rows are kRunPad voxels wider than the
  // halo on each side, so runs (padding slots included) stay inside a row.
  uint32_t* vol2 = reinterpret_cast<uint32_t*>(item + 4);
  // the perceptron's b1 and W2 (fused rows), then the slice descriptors of a
  // batch, when they fit
  constexpr bool FUSE = fused_rows(ROWS);
  static_assert(!FUSE || enc_pipelined(L), "the perceptron runs inside the pipelined layouts only");
  const size_t base_bytes = NBUF * SLAB_U4 * 16 + a.nsteps * 32 * 4 + CH * 4 + 16 + a.vol * 4;
  float* mlp_l = reinterpret_cast<float*>(smem + slice_table_offset(base_bytes));
  SliceDesc* stab = reinterpret_cast<SliceDesc*>(
      smem + slice_table_offset(base_bytes + (FUSE ? mlp_lds_bytes(a.hidden) : 0)));

  const int tid = threadIdx.x, lane = tid & 63;
  const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wn = wid % WN, wm = wid / WN;
  const int KP = a.nsteps * 32;
  const int BV = a.b.bx * a.b.by * a.b.bt;
  const int D = a.D;
  for (int k = tid; k < KP / 4; k += NW * 64) {
    runs_l[k] = a.runs[k];
    runs1_l[k] = a.runs1 ? a.runs1[k] : 0;  // (no single rows without it)
  }
  for (int k = tid; k < KP; k += NW * 64) wts_l[k] = a.wts[k];
  for (int k = tid; k < a.lds_slices * (int)(sizeof(SliceDesc) / 4); k += NW * 64)
    reinterpret_cast<int32_t*>(stab)[k] = reinterpret_cast<const int32_t*>(a.bt.table)[k];
  if constexpr (FUSE) {
    for (int k = tid; k < a.hidden; k += NW * 64) {
      mlp_l[k] = a.b1[k];
      mlp_l[a.hidden + k] = a.W2[k];
      mlp_l[2 * a.hidden + k] = a.W2[a.hidden + k];
    }
  }

  // Work items come from a shared counter, in longest-first order, one
  // brick at a time (taking the next brick ahead of time upsets the balance
  // of long jobs and measured slower on sparse batches too).  An item's
  // record holds all the brick needs; the slice descriptors are in LDS.
  int4* item4 = reinterpret_cast<int4*>(item);
  const int total = a.plan[2];
  for (;;) {
    if (tid == 0) {
      const int it = atomicAdd(&a.plan[1], 1);
      item4[0] = it < total ? a.order[it] : make_int4(-1, 0, 0, 0);
    }
    lds_barrier();
    const int4 cur = item4[0];
    const int bid = __builtin_amdgcn_readfirstlane(cur.x);
    if (bid < 0) break;
    const int nq = __builtin_amdgcn_readfirstlane(cur.y);
    const int row0 = __builtin_amdgcn_readfirstlane(cur.z);
    const int si = __builtin_amdgcn_readfirstlane(cur.w);
    const bool single = (bid & kSparseTag) != 0;  // (uniform)
    const int32_t* rl = single ? runs1_l : runs_l;

    if (single) {
      // ---- single rows (from bricks with few rows): row r gets its own count
      //      box, a single voxel's, at vol2 + r vol1; wave w copies the boxes
      //      of rows w, w + NW, ...  (rows srow[si .. si + nq))
      for (int r = wid; r < nq; r += NW) {
        const int2 e = a.srow[si + r];
        const int gb = __builtin_amdgcn_readfirstlane(e.x);
        const int li = __builtin_amdgcn_readfirstlane(e.y);
        int s_ix = 0;
        if (a.bt.nslices > 1) {
          int hi = a.bt.nslices - 1;
          while (s_ix < hi) {
            const int mid = (s_ix + hi + 1) >> 1;
            const int bo = a.lds_slices ? stab[mid].brick_off : a.bt.table[mid].brick_off;
            if (bo <= gb) s_ix = mid; else hi = mid - 1;
          }
        }
        const SliceDesc sl =
            a.bt.nslices == 1 ? a.bt.s0 : a.lds_slices ? stab[s_ix] : a.bt.table[s_ix];
        const int lb = gb - sl.brick_off;
        const int bxi = lb % sl.nbx, byi = (lb / sl.nbx) % sl.nby, bti = lb / (sl.nbx * sl.nby);
        const int vx = bxi * a.b.bx + li % a.b.bx, vy = byi * a.b.by + (li / a.b.bx) % a.b.by,
                  vt = bti * a.b.bt + li / (a.b.bx * a.b.by);
        // the box is vol1 consecutive dwords in LDS (rows of SX1): each copy
        // fills 64 of them, whatever box rows they belong to
        for (int d0 = 0; d0 < a.vol1; d0 += 64) {
          const int d = d0 + lane, rr = d / a.SX1, xi = d - rr * a.SX1;
          const int x = vx - a.rx - kRunPad + xi, y = vy - a.ry + rr % a.SY1,
                    t = vt - a.rt + rr / a.SY1;
          const bool in = x >= -1 && x < sl.W &&  // the pair grid has a column for x = -1
                          (unsigned)y < (unsigned)sl.H && (unsigned)t < (unsigned)sl.T;
          const int tp = t + sl.tshift < sl.T ? t + sl.tshift : t + sl.tshift - sl.T;
          const uint32_t* src =
              in ? a.pairs + sl.pair_off + ((int64_t)tp * sl.H + y) * (sl.W + 1) + (x + 1)
                 : a.zeros + lane;
          if (d < a.vol1) copy_to_lds4(src, lds_offset(vol2 + r * a.vol1 + d0));
        }
      }
    } else {
      // ---- the brick's count box: one global->LDS copy per box row from the
      //      pair grid (lanes outside the slice read zeros); it has landed once
      //      the first chunk's prologue wait returns
      const SliceDesc sl = a.bt.nslices == 1 ? a.bt.s0 : a.lds_slices ? stab[si] : a.bt.table[si];
      const int lb = bid - sl.brick_off;
      const int bxi = lb % sl.nbx, byi = (lb / sl.nbx) % sl.nby, bti = lb / (sl.nbx * sl.nby);
      const int x = bxi * a.b.bx - a.rx - kRunPad + lane;
      const int y0 = byi * a.b.by - a.ry, tb = bti * a.b.bt - a.rt;
      const bool xin = x >= -1 && x < sl.W;  // the pair grid has a column for x = -1
      const int nrows = a.SY * a.ST;
      int sy = wid % a.SY, st = wid / a.SY;
      for (int rr = wid; rr < nrows; rr += NW) {
        const int y = y0 + sy, t = tb + st;
        const bool in = xin && (unsigned)y < (unsigned)sl.H && (unsigned)t < (unsigned)sl.T;
        const int tp = t + sl.tshift < sl.T ? t + sl.tshift : t + sl.tshift - sl.T;  // ring plane
        const uint32_t* src =
            in ? a.pairs + sl.pair_off + ((int64_t)tp * sl.H + y) * (sl.W + 1) + (x + 1)
               : a.zeros + lane;
        if (lane < a.SX) copy_to_lds4(src, lds_offset(vol2 + rr * a.SX));
        sy += NW;
        while (sy >= a.SY) {
          sy -= a.SY;
          ++st;
        }
      }
    }

    for (int c0 = 0; c0 < nq; c0 += CH) {
      const int nr = nq - c0 < CH ? nq - c0 : CH;  // rows in this chunk
      const int ntiles = (nr + 15) / 16;          // 16-row tiles holding rows
      // ---- voxel of each row (row q*16 + l of the chunk; padding reuses row 0)
      for (int r = tid; r < CH; r += NW * 64) {
        const int rr = c0 + (r < nr ? r : 0);
        if (single) {  // the voxel at the centre of the row's own box
          rowbase[r] = rr * a.vol1 + (a.rt * a.SY1 + a.ry) * a.SX1 + (a.rx + kRunPad);
          continue;
        }
        const int li = a.ulist[(int64_t)bid * BV + rr];
        const int lx = li % a.b.bx, ly = (li / a.b.bx) % a.b.by, lt = li / (a.b.bx * a.b.by);
        rowbase[r] = ((lt + a.rt) * a.SY + (ly + a.ry)) * a.SX + (lx + a.rx + kRunPad);
      }
      // first slabs of the table
      if constexpr (kEncPairSteps && NBUF == 4 && !enc_pipelined(L)) {
        // the first pair (and the box) has landed
#pragma unroll
        for (int u = 0; u < 2; ++u)
          if (u < a.nsteps)
            issue_slab<SLAB_U4, NW>(a.frag + (size_t)u * SLAB_U4, slab + u * SLAB_U4, wid, lane);
        __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));
      } else {
        // (fused rows: the W1 slabs follow the table's in the same ring)
        const int steps = a.nsteps + (FUSE ? a.msteps : 0);
#pragma unroll
        for (int u = 0; u < AHEAD; ++u)
          if (u < steps)
            issue_slab<SLAB_U4, NW>(step_src<SLAB_U4>(a.frag, a.w1frag, a.nsteps, u),
                                    slab + u * SLAB_U4, wid, lane);
        wait_slabs<PFW>((steps < AHEAD ? steps : AHEAD) - 1);  // slab 0 (and the box) landed
      }
      lds_barrier();

      // tiles are dealt round-robin over the row waves, so a short chunk
      // spreads evenly and fully padded tiles are skipped
      int mtv = 0;
      int rb[MT];  // voxel index of each row in the volume
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        const int q = mt * WM + wm;
        if (q < ntiles) mtv = mt + 1;
        rb[mt] = rowbase[q * 16 + (lane & 15)];
      }
      mtv = __builtin_amdgcn_readfirstlane(mtv);

      floatx4 accR[MT][NTW], accI[MT][NTW];
      float cnt[MT];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        cnt[mt] = 0.f;
#pragma unroll
        for (int nt = 0; nt < NTW; ++nt) {
          accR[mt][nt] = floatx4{0.f, 0.f, 0.f, 0.f};
          accI[mt][nt] = floatx4{0.f, 0.f, 0.f, 0.f};
        }
      }
      if constexpr (enc_pipelined(L)) {
        FuseArgs fz;
        fz.w1frag = a.w1frag;
        fz.msteps = FUSE ? a.msteps : 0;
        fz.unscale = a.unscale;
        fz.mlp_l = mlp_l;
        fz.hidden = a.hidden;
        fz.b20 = FUSE ? a.b2[0] : 0.f;
        fz.b21 = FUSE ? a.b2[1] : 0.f;
        fz.out = a.rowflow;
        fz.row_first = row0 + c0;
        fz.nr = nr;
        fz.wm = wm;
        chunk_ksteps_pn<NA, NT, L, NBUF, MT, FUSE>(mtv, a.nsteps, a.frag, slab, rl, wts_l, vol2,
                                                   rb, accR, accI, cnt, wn, wid, lane, fz);
        if constexpr (FUSE) continue;  // flows written; no rows leave the chip
      } else
        chunk_ksteps_n<NA, NT, L, NBUF, MT>(mtv, a.nsteps, a.frag, slab, rl, wts_l, vol2, rb,
                                            accR, accI, cnt, wn, wid, lane);

      // ---- normalise by the neighbour count and write the rows: the lane
      //      holds frequencies 16 nt + 4 (lane >> 4) + (0..3) of row lane & 15
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        if (mt >= mtv) continue;
        const int r = (mt * WM + wm) * 16 + (lane & 15);
        // the row's count: the partial sums of its 4 lanes (exact integers)
        float n = cnt[mt];
        n += __shfl_xor(n, 16);
        n += __shfl_xor(n, 32);
        if (r >= nr) continue;
        if (a.rowcnt && wn == 0 && lane < 16) a.rowcnt[row0 + c0 + r] = (int)n;
        const float rc = __builtin_amdgcn_rcpf(n);
        // x / n: reciprocal estimate plus one residual correction (exact for
        // x = n, so an all-ones feature still gives exactly 1).  A query of a
        // sliding window can have no event in its neighbourhood (n = 0): its
        // encoding is zero.
        auto div = [n, rc](float x) {
          const float qq = x * rc;
          return n > 0.f ? fmaf(fmaf(-qq, n, x), rc, qq) : 0.f;
        };
        const int64_t u = (int64_t)(row0 + c0 + r) * (2 * D);
#pragma unroll
        for (int nt = 0; nt < NTW; ++nt) {
          const int j = (wn * NTW + nt) * 16 + 4 * (lane >> 4);
          floatx4 re, im;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            re[i] = div(accR[mt][nt][i]);
            im[i] = div(accI[mt][nt][i]);
          }
          // plain stores: a lane writes 8 or 16 bytes of a row and the other
          // lanes and frequency tiles complete its lines, which L2 merges
          // before they reach HBM (streaming stores measured 1.4-2x the
          // row bytes in HBM writes)
          if constexpr (ROWS == kRowsBF16) {
            uint16_t* out = static_cast<uint16_t*>(a.rows);
            u32x2 pr, pi;
            pr.x = f32_to_bf16_rne(re[0]) | ((uint32_t)f32_to_bf16_rne(re[1]) << 16);
            pr.y = f32_to_bf16_rne(re[2]) | ((uint32_t)f32_to_bf16_rne(re[3]) << 16);
            pi.x = f32_to_bf16_rne(im[0]) | ((uint32_t)f32_to_bf16_rne(im[1]) << 16);
            pi.y = f32_to_bf16_rne(im[2]) | ((uint32_t)f32_to_bf16_rne(im[3]) << 16);
            *reinterpret_cast<u32x2*>(out + u + j) = pr;
            *reinterpret_cast<u32x2*>(out + u + D + j) = pi;
          } else if constexpr (ROWS == kRowsHiLo16) {
            // fp16 hi = rne(v), lo = rne(v - hi) (v - hi is exact in fp32):
            // 22 significant bits in the perceptron's operands.  Each group
            // of 4 consecutive row elements becomes one 16-byte unit [hi x 4,
            // lo x 4], so a row keeps the fp32 row's size and a lane writes
            // one unit for its 4 real and one for its 4 imaginary parts.
            _Float16* out = static_cast<_Float16*>(a.rows);
            const int64_t u2 = u * 2;
            half8 ur, ui;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              ur[i] = (_Float16)re[i];
              ur[4 + i] = (_Float16)(re[i] - (float)ur[i]);
              ui[i] = (_Float16)im[i];
              ui[4 + i] = (_Float16)(im[i] - (float)ui[i]);
            }
            *reinterpret_cast<half8*>(out + u2 + 2 * j) = ur;
            *reinterpret_cast<half8*>(out + u2 + 2 * (D + j)) = ui;
          } else {
            float* out = static_cast<float*>(a.rows);
            *reinterpret_cast<floatx4*>(out + u + j) = re;
            *reinterpret_cast<floatx4*>(out + u + D + j) = im;
          }
        }
      }
    }
    lds_barrier();
  }
}

template <int NA, int NT, int L, int NBUF>
static size_t encode_lds_bytes(const EncodeTables& et, int vol) {
  using S = EncShape<NA, NT, L>;
  return (size_t)NBUF * S::SLAB_U4 * 16 + (size_t)et.KP * 2 + (size_t)et.KP * 2 +
         (size_t)S::CH * 4 + 16 + (size_t)vol * 4;
}

// Rows per chunk and LDS bytes of the encoder for a given D and wave layout
// (the host-side mirror of EncShape::CH).
static int chunk_rows(int nt, int layout) {
  const int ntw = nt < enc_max_ntw(layout) ? nt : enc_max_ntw(layout), wn = nt / ntw;
  const int wm = enc_waves(layout) / wn;
  return wm * enc_mt(layout) * 16;
}

size_t encode_lds_need(int d, int precision, int nbuf, int kp, int vol, int layout) {
  const int na = precision == VECKM_FP32 ? 4 : 2, nt = d / 16;
  return (size_t)nbuf * na * nt * 64 * 16 + (size_t)kp * 4 + (size_t)chunk_rows(nt, layout) * 4 +
         16 + (size_t)vol * 4;
}

template <int NA, int NT, int L, int NBUF, int ROWS>
static int launch_rows(const EncArgs& a, const EncodeTables& et, int num_cus, hipStream_t s) {
  constexpr bool FUSE = fused_rows(ROWS);
  size_t lds = encode_lds_bytes<NA, NT, L, NBUF>(et, a.vol);
  if (FUSE) lds = slice_table_offset(lds) + mlp_lds_bytes(a.hidden);
  if (lds > 160 * 1024) return VECKM_E_INVAL;
  // a batch's slice descriptors go to LDS when they fit beside the rest
  EncArgs b = a;
  b.lds_slices = 0;
  const size_t with_tab = slice_table_offset(lds) + (size_t)a.bt.nslices * sizeof(SliceDesc);
  if (a.bt.nslices > 1 && with_tab <= 160 * 1024) {
    b.lds_slices = a.bt.nslices;
    lds = with_tab;
  }
  const void* fn = reinterpret_cast<const void*>(&k_encode<NA, NT, L, NBUF, ROWS>);
  if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return VECKM_E_HIP;
  const int per_cu = (int)((160 * 1024) / lds);
  int grid = num_cus * (per_cu < 1 ? 1 : (per_cu > 2 ? 2 : per_cu));
  if (grid > b.bt.nbricks) grid = a.bt.nbricks;
  constexpr int threads = EncShape<NA, NT, L>::NW * 64;
  hipLaunchKernelGGL((k_encode<NA, NT, L, NBUF, ROWS>), dim3(grid), dim3(threads), lds, s, b);
  return hipGetLastError() == hipSuccess ? VECKM_OK : VECKM_E_HIP;
}

template <int NA, int NT, int L, int NBUF>
static int launch_t(const EncArgs& a, const EncodeTables& et, int rows, int num_cus,
                    hipStream_t s) {
  if (rows == kRowsHiLo16 && NA != 4) return VECKM_E_INVAL;  // hi/lo rows: the FP32 form only
  constexpr int HL = NA == 4 ? kRowsHiLo16 : kRowsF32;
  if (fused_rows(rows)) {
    // the perceptron inside the encoder: one wave holds all of a row's frequencies
    if constexpr (enc_pipelined(L) && EncShape<NA, NT, L>::WN == 1) {
      constexpr int FR = NA == 4 ? kFlowHiLo16 : kFlowBF16;
      if (rows != FR) return VECKM_E_INVAL;
      return launch_rows<NA, NT, L, NBUF, FR>(a, et, num_cus, s);
    }
    return VECKM_E_INVAL;
  }
  if (rows == kRowsBF16) return launch_rows<NA, NT, L, NBUF, kRowsBF16>(a, et, num_cus, s);
  if (rows == kRowsHiLo16) return launch_rows<NA, NT, L, NBUF, HL>(a, et, num_cus, s);
  return launch_rows<NA, NT, L, NBUF, kRowsF32>(a, et, num_cus, s);
}

static_assert(EncShape<4, 8, 0>::CH == 8 * kEncMt * 16 && EncShape<2, 16, 0>::CH == 4 * kEncMt * 16 &&
                  EncShape<4, 1, 0>::CH == 16 * kEncMt * 16 &&
                  EncShape<4, 8, 1>::CH == 4 * 2 * kEncMt * 16 &&
                  EncShape<4, 8, 2>::CH == 4 * 2 * kEncMt * 16 &&
                  EncShape<2, 16, 2>::CH == 2 * 2 * kEncMt * 16,
              "chunk_rows mirrors EncShape");

template <int NA, int NT, int L>
static int launch_nb(const EncArgs& a, const EncodeTables& et, int rows, int num_cus,
                     hipStream_t s) {
  if constexpr (enc_pipelined(L)) {  // the pipelined layouts keep one slab in flight
    if (et.nbuf != 2) return VECKM_E_INVAL;
    return launch_t<NA, NT, L, 2>(a, et, rows, num_cus, s);
  } else {
    if constexpr (EncShape<NA, NT, L>::EVEN) {
      if (et.nbuf == 4) return launch_t<NA, NT, L, 4>(a, et, rows, num_cus, s);
      if (et.nbuf == 3) return launch_t<NA, NT, L, 3>(a, et, rows, num_cus, s);
    }
    return launch_t<NA, NT, L, 2>(a, et, rows, num_cus, s);
  }
}

template <int NA, int NT>
static int launch_layout(const EncArgs& a, const EncodeTables& et, int rows, int num_cus,
                         hipStream_t s) {
  // the 8- and 4-wave layouts only where a wave holds several frequency tiles
  if constexpr (NT >= 4) {
    if (et.layout == 1) return launch_nb<NA, NT, 1>(a, et, rows, num_cus, s);
    if (et.layout == 2) return launch_nb<NA, NT, 2>(a, et, rows, num_cus, s);
    if (et.layout == 3) return launch_nb<NA, NT, 3>(a, et, rows, num_cus, s);
  }
  if constexpr (NT == 4 || NT == 8)
    if (et.layout == 4) return launch_nb<NA, NT, 4>(a, et, rows, num_cus, s);
  return launch_nb<NA, NT, 0>(a, et, rows, num_cus, s);
}

template <int NA>
static int dispatch_nt(const EncArgs& a, const EncodeTables& et, int rows, int num_cus,
                       hipStream_t s) {
  switch (a.D / 16) {
    case 1: return launch_layout<NA, 1>(a, et, rows, num_cus, s);
    case 2: return launch_layout<NA, 2>(a, et, rows, num_cus, s);
    case 3: return launch_layout<NA, 3>(a, et, rows, num_cus, s);
    case 4: return launch_layout<NA, 4>(a, et, rows, num_cus, s);
    case 8: return launch_layout<NA, 8>(a, et, rows, num_cus, s);
    case 16: return launch_layout<NA, 16>(a, et, rows, num_cus, s);
    default: return VECKM_E_INVAL;
  }
}

int encode_rows_per_chunk(int d, int layout) { return chunk_rows(d / 16, layout); }
int encode_waves(int layout) { return enc_waves(layout); }

bool encode_fusable(const EncodeTables& et, int hidden) {
  const int nt = et.d / 16;
  if (et.layout < 2 || et.layout > 4 || (nt != 4 && nt != 8) || hidden < 64 || hidden % 32)
    return false;
  const int vol = box_dwords(et.brick, et.rx, et.ry, et.rt);
  const size_t lds = slice_table_offset(encode_lds_need(et.d, et.na == 4 ? VECKM_FP32 : VECKM_FP16,
                                                        et.nbuf, et.KP, vol, et.layout)) +
                     mlp_lds_bytes(hidden);
  return lds <= 160 * 1024;
}

int launch_encode(const Batch& bt, const Workspace& w, const EncodeTables& et, int rows,
                  int num_cus, void* stream, int32_t* rowcnt, const MlpWeights* mw) {
  EncArgs a;
  a.rowcnt = rowcnt;
  a.w1frag = nullptr;
  a.msteps = 0;
  a.hidden = 0;
  a.unscale = 1.f;
  a.b1 = a.W2 = a.b2 = nullptr;
  a.rowflow = nullptr;
  if (fused_rows(rows)) {
    if (!mw || !mw->W1frag || !encode_fusable(et, mw->hidden)) return VECKM_E_INVAL;
    a.w1frag = reinterpret_cast<const uint4*>(mw->W1frag);
    a.msteps = mw->hidden / 32;
    a.hidden = mw->hidden;
    a.unscale = et.na == 4 ? mw->unscale : 1.f;  // the bf16 W1 is not scaled
    a.b1 = mw->b1;
    a.W2 = mw->W2;
    a.b2 = mw->b2;
    a.rowflow = reinterpret_cast<float2*>(w.rowflow);
  }
  a.bt = bt;
  a.b = et.brick;
  a.rx = et.rx;
  a.ry = et.ry;
  a.rt = et.rt;
  a.K = et.K;
  a.nsteps = et.KP / kKStep;
  a.SX = box_sx(et.brick, et.rx);
  a.SY = et.brick.by + 2 * et.ry;
  a.ST = et.brick.bt + 2 * et.rt;
  a.vol = a.SX * a.SY * a.ST;
  a.D = et.d;
  a.ulist = w.ulist;
  a.order = reinterpret_cast<const int4*>(w.order);
  // single rows: a single voxel's count box, rs of which fit in the brick's
  a.srow = reinterpret_cast<const int2*>(w.srow);
  a.runs1 = et.runs1;
  a.SX1 = box_sx(Brick{1, 1, 1}, et.rx);
  a.SY1 = 1 + 2 * et.ry;
  a.ST1 = 1 + 2 * et.rt;
  a.vol1 = a.SX1 * a.SY1 * a.ST1;
  a.lds_slices = 0;
  a.frag = reinterpret_cast<const uint4*>(et.frag);
  a.runs = et.runs;
  a.wts = et.wts;
  a.pairs = w.pairs;
  a.zeros = w.zeros;
  a.rows = w.rows;
  a.plan = w.plan;
  if (a.SX > 64) return VECKM_E_INVAL;  // one wavefront copies one box row
  if (et.sp > 0 && (!et.runs1 || !w.srow || a.SX1 > 64 || et.rs < 1 || et.rs > 16 ||
                    et.rs * a.vol1 > a.vol))
    return VECKM_E_INVAL;
  hipStream_t s = (hipStream_t)stream;
  return et.na == 4 ? dispatch_nt<4>(a, et, rows, num_cus, s)
                    : dispatch_nt<2>(a, et, rows, num_cus, s);
}

}  // namespace veckm
