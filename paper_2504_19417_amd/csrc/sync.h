// Work-group barrier for LDS traffic and global->LDS copies issued by hand.
//
// __syncthreads() is a release/acquire fence plus s_barrier, and the fence
// makes every wave wait for all of its outstanding global loads and stores
// (vmcnt(0)) before the barrier.  The compiler also makes every LDS read wait
// for all global->LDS copies issued with the builtin before it, since it
// cannot tell which LDS bytes a copy writes.  Kernels that keep copies of the
// next table slab or input tile in flight while they read the current one
// therefore issue the copies with the inline-asm helpers below (invisible to
// the compiler's wait insertion) and synchronise with lds_barrier(): each wave
// waits only for its own LDS operations (lgkmcnt(0)) and meets the others.
// Whoever issued a copy whose data other waves read after a barrier waits for
// it explicitly (s_waitcnt vmcnt(n), vector memory loads complete in issue
// order) before that barrier.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace veckm {

__device__ inline void lds_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// Byte offset of an LDS location (the M0 base of a global->LDS copy).
__device__ inline uint32_t lds_offset(const void* p) {
  typedef __attribute__((address_space(3))) const void* lds_cptr;
  return (uint32_t)(uintptr_t)(lds_cptr)(p);
}

// gfx950 global->LDS copies: lane i's 16 (4) bytes at `src` go to LDS byte
// lds_base + 16 i (4 i); lds_base must be wave-uniform.  The leading s_nop 4
// gives the five wait states the hardware needs between a vector-ALU write of
// a scalar register (an SGPR spill reload by v_readlane, a v_readfirstlane
// into M0) and a vector memory instruction that reads it (the M0 base, the
// scalar base address); the compiler's hazard pass does not look inside
// inline asm, so the helpers carry the wait themselves.
__device__ inline void copy_to_lds16(const void* src, uint32_t lds_base) {
  asm volatile("s_nop 4\n\tglobal_load_lds_dwordx4 %0, off"
               :: "v"(src), "{m0}"(__builtin_amdgcn_readfirstlane(lds_base)) : "memory");
}
// The same with a wave-uniform base address (scalar registers) plus the
// lane's 32-bit byte offset: no 64-bit address per copy in vector registers.
__device__ inline void copy_to_lds16_s(const void* sbase, uint32_t voff, uint32_t lds_base) {
  asm volatile("s_nop 4\n\tglobal_load_lds_dwordx4 %0, %1"
               :: "v"(voff), "s"(sbase), "{m0}"(__builtin_amdgcn_readfirstlane(lds_base)) : "memory");
}
__device__ inline void copy_to_lds4(const void* src, uint32_t lds_base) {
  asm volatile("s_nop 4\n\tglobal_load_lds_dword %0, off"
               :: "v"(src), "{m0}"(__builtin_amdgcn_readfirstlane(lds_base)) : "memory");
}

}  // namespace veckm
