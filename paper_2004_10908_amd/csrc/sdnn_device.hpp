// Device helpers shared by the forward kernel files: LDS access by absolute
// address and the asynchronous global->LDS copies of the one-row-tile kernels, the
// acquire load of a device counter, the persistent kernels' grid barrier and the
// per-layer arguments of the persistent chain.
#pragma once

#include "sdnn_internal.hpp"

namespace sdnn {

// Absolute LDS byte addresses: the row kernels declare no static LDS, so their
// dynamic LDS starts at address 0, and every LDS object is reached through a
// pointer built from its address (never as an offset into a zero-length array).
template <typename T>
using lds_ptr = T __attribute__((address_space(3)))*;
template <typename T>
__device__ __forceinline__ lds_ptr<T> lds_at(uint32_t addr) {
    return (lds_ptr<T>)(uintptr_t)addr;
}

__device__ __forceinline__ float row_lds_read(uint32_t addr) {
#if defined(__HIP_DEVICE_COMPILE__)
    return *reinterpret_cast<const float __attribute__((address_space(3)))*>(addr);
#else
    (void)addr;
    return 0.f;
#endif
}

// One 16-byte asynchronous copy per lane: global (scalar base + lane offset) ->
// LDS at M0 + 16 * lane.
__device__ __forceinline__ void row_copy16(uint64_t src, uint32_t voff, uint32_t dst) {
    uint32_t saved;
    __asm__ volatile("s_mov_b32 %0, m0\n\ts_mov_b32 m0, %2\n\tglobal_load_lds_dwordx4 %1, %3\n\ts_mov_b32 m0, %0"
                     : "=&s"(saved)
                     : "v"(voff), "s"(dst), "s"(src)
                     : "memory");
}

// One dword from src (a per-lane address) into LDS at M0 + 4 * lane.
__device__ __forceinline__ void row_copy4(const int32_t* src, uint32_t dst) {
    uint32_t saved;
    __asm__ volatile("s_mov_b32 %0, m0\n\ts_mov_b32 m0, %2\n\tglobal_load_lds_dword %1, off\n\ts_mov_b32 m0, %0"
                     : "=&s"(saved)
                     : "v"(src), "s"(dst)
                     : "memory");
}

__device__ __forceinline__ uint64_t uniform_ptr(const void* p) {
    const uint64_t v = (uint64_t)(uintptr_t)p;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | (uint64_t)lo;
}

// The persistent chains' row count of layer l: the appends to it happened before the
// grid barrier that ended layer l - 1, whose acquire fence already ordered them, so
// a relaxed load suffices (an acquiring one would invalidate the L2 once more per
// workgroup at every layer start).
__device__ __forceinline__ int ld_count(const int32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------- grid barrier
// Two-level arrive counter: workgroups arrive on one of 8 group counters
// (blockIdx % 8, the XCD a workgroup is dispatched to), the last of each group
// arrives on the root, the last at the root bumps the generation word that every
// workgroup polls.  Counters return to zero after each barrier.  Waits are
// bounded by the 100 MHz real-time counter; a time-out, or an error raised by
// any other workgroup, makes every waiter leave with `false`.
// Memory ordering: each arrival is a release (this workgroup's stores, which every
// wave has drained first, before its arrival); the last arrival of a group takes
// an acquire fence and passes the group on with a release-acquire add on the root;
// the last at the root publishes the generation with a release store.  Waiters poll
// with relaxed loads and take one acquire fence when the generation turns.  (An
// acquiring load invalidates the L2 on every poll, under the feet of the
// workgroups still finishing the layer, and a full fence per workgroup on either
// side writes the L2 back 256 times: measured 21 us per barrier against 7 us.)
// bar layout (one 128-byte line each): [g*32] group g, [8*32] root, [9*32] generation.
__device__ inline bool grid_barrier(unsigned* bar, unsigned& gen, int32_t* err, int* s_ok_ptr) {
    int& s_ok = *s_ok_ptr;
    __asm__ volatile("s_waitcnt vmcnt(0)" : : : "memory");
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned nwg = gridDim.x;
        const unsigned g = blockIdx.x & 7u;
        const unsigned ngroups = nwg < 8u ? nwg : 8u;
        const unsigned gsize = (nwg - g + 7u) / 8u;
        const unsigned target = gen + 1u;
        int ok = 1;
        const unsigned old = __hip_atomic_fetch_add(&bar[g * 32], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        if (old == gsize - 1u) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            __hip_atomic_store(&bar[g * 32], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const unsigned o2 = __hip_atomic_fetch_add(&bar[8 * 32], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
            if (o2 == ngroups - 1u) {
                __hip_atomic_store(&bar[8 * 32], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&bar[9 * 32], target, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
        while (__hip_atomic_load(&bar[9 * 32], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != target) {
            if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) { ok = 0; break; }
            if (__builtin_amdgcn_s_memrealtime() - t0 > 1000000000ull) {   // 10 s at 100 MHz
                atomicExch(err, (int32_t)DEV_BARRIER_TIMEOUT);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        gen = target;
        s_ok = ok;
    }
    __syncthreads();
    return s_ok != 0;
}

// ---------------------------------------------------------------- persistent chain arguments
// The kernel's ChainArgs (its only argument), read again from the kernel-argument
// segment through an address the compiler cannot follow, so its fields are scalar
// loads at the point of use instead of registers held across a layer's tile loop
// (in the persistent chains those were spilled and shuffled on every tile).
__device__ __forceinline__ ChainArgs reload_chain_args() {
#if defined(__HIP_DEVICE_COMPILE__)
    uint64_t p = (uint64_t)(uintptr_t)__builtin_amdgcn_kernarg_segment_ptr();
    __asm__ volatile("" : "+s"(p));
    return *(const __attribute__((address_space(4))) ChainArgs*)p;
#else
    return ChainArgs{};                                // (host pass: never called)
#endif
}

// Layer l of the persistent chain writes X_l, which is y_out when (L-1-l) is even
// and the workspace buffer otherwise, so the last layer always lands in y_out.
__device__ __forceinline__ LayerArgs chain_layer_args(const ChainArgs& c, int l, int R) {
    const int N = c.N, L = c.L;
    const size_t NK = (size_t)N * K;
    const bool out_is_y = ((L - 1 - l) & 1) == 0;
    LayerArgs a{};
    a.yin = l == 0 ? c.y0 : (out_is_y ? c.act : c.y_out);
    a.yout = out_is_y ? c.y_out : c.act;
    a.ycopy = (c.ckpt && (l + 1) % c.ckpt_every == 0 && l + 1 < L)
                  ? c.ckpt + (size_t)((l + 1) / c.ckpt_every - 1) * c.rows * N
                  : nullptr;
    a.dead_mark = (c.compaction && !out_is_y) ? -1 : 0;
    a.idx = c.idx + l * NK;
    a.w = c.w + l * NK;
    a.b = c.b + (size_t)l * N;
    a.list_in = (l == 0 || !c.compaction) ? nullptr : ((l & 1) ? c.list1 : c.list0);
    a.list_out = c.compaction ? (((l + 1) & 1) ? c.list1 : c.list0) : nullptr;
    a.cnt_in = nullptr;
    a.cnt_out = &c.cnt[l + 1];
    a.alive = c.alive;
    a.row_base = 0;
    a.nrows = R;
    a.N = N;
    a.layer = l;
    a.clamp = c.clamp;
    a.packed = c.packed;
    a.wide_words = c.wide_words;
    return a;
}

}  // namespace sdnn
