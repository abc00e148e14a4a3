// Direct global-to-LDS copies on gfx950 (global_load_lds_dwordx4 and
// global_load_lds_dword), shared by
// the kernels that stage samples without passing them through registers.
//
// The copies are issued from inline assembly so that the compiler does not
// insert a wait for all outstanding copies before every LDS read (it cannot
// tell which copy feeds which read); in exchange every wait for them is
// explicit: a wave's copies are complete once vmcnt has dropped to the number
// of vector-memory operations it issued after them, and a barrier then makes
// every wave's copies visible to the workgroup.
#pragma once
#include "common.h"

namespace xc {

// Source of the time steps past the end of a channel.
static __device__ __attribute__((aligned(16))) uint32_t g_zero16[4] = {0u, 0u, 0u, 0u};

// Lane L's 16-byte granule at src goes to LDS byte address lds + 16 L (lds
// is uniform across the wave; M0 needs one wait state before the copy).  M0
// is clobbered: the kernels that use this hold nothing else in M0 (no other
// LDS-DMA, message or indexed-register instructions).
#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Winline-asm"
__device__ __forceinline__ void dma16(const void *src, uint32_t lds) {
    asm volatile("s_mov_b32 m0, %1\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, off" ::"v"(src), "s"(lds)
                 : "memory", "m0");
}
// The same with 4-byte granules: lane L's dword at src goes to lds + 4 L.
__device__ __forceinline__ void dma4(const void *src, uint32_t lds) {
    asm volatile("s_mov_b32 m0, %1\n\ts_nop 0\n\tglobal_load_lds_dword %0, off" ::"v"(src), "s"(lds)
                 : "memory", "m0");
}
#pragma clang diagnostic pop

// Workgroup barrier that the compiler may not move memory accesses across
// (the copies are invisible to it, so the plain builtin would not do).
__device__ __forceinline__ void barrier_lds() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// Wait until at most N of this wave's vector-memory operations are pending.
template <int N>
__device__ __forceinline__ void wait_vm() {
    static_assert(N >= 0 && N < 64, "vmcnt range");
    constexpr int rest = (7 << 4) | (15 << 8);   // expcnt, lgkmcnt: no wait
    __builtin_amdgcn_s_waitcnt(rest | (N & 15) | ((N >> 4) << 14));
    asm volatile("" ::: "memory");
}

// LDS byte address of a __shared__ location.
__device__ __forceinline__ uint32_t lds_addr(const void *p) {
    return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) void *)p;
}

}  // namespace xc
