// Synchronisation between the blocks of one cooperative launch (the resident
// kernels: resident2d, resident_adj and resident_pass2d).
#pragma once

#include <stdint.h>

namespace jko {

// Synchronisation without atomics read-modify-write and without cache-wide
// fences: every value one block writes for another (a, b, the partials) is
// stored and loaded at device scope, which is coherent across the XCDs'
// separate L2s.  After a phase's stores have completed (s_waitcnt), block t
// publishes its phase count in flags[t]; before a phase that reads other
// blocks' values, a block waits until each block it reads from has published
// at least its own count.  A block only reads the tiles it depends on, so
// most phases wait on those neighbours only (each kernel keeps the relation
// symmetric, which also keeps a block from overwriting values a neighbour is
// still reading);
// at a stop-test check, block 0 waits on every block, evaluates the test
// from all partials and publishes the decision, which the others wait for.
// Each wait polls a bounded number of times; one that runs out raises the
// abort word, which every waiting block also polls, so every wave ends.

// Sync region layout (uint32 words): [0] abort, [16] decision bits of the
// last check (1 done, 2 absorb), [32] the phase count that decision belongs
// to, flags[t] at kFlag0 + kFlagStride * t.
constexpr int kDecision = 16;
constexpr int kDecisionSeq = 32;
constexpr int kFlag0 = 64;
constexpr int kFlagStride = 16;   // one 64-byte line per block

__device__ __forceinline__ uint32_t* flag_of(uint32_t* sync, int t) { return sync + kFlag0 + kFlagStride * t; }

// All stores of this block completed, then publish `count` for it.
__device__ __forceinline__ void publish(uint32_t* sync, int slot, uint32_t count) {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_store(flag_of(sync, slot), count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wait until blocks list[0 .. n) (one per thread) have published >= count.
// Returns false (in every thread) if the wait ran out or another block aborted.
__device__ __forceinline__ bool wait_for(uint32_t* sync, int n, const int* list, uint32_t count, int spin_limit) {
    int ok = 1;
    const int t = threadIdx.x;
    if (t < n) {
        const uint32_t* f = flag_of(sync, list[t]);
        for (int spins = 0; __hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < count; ++spins) {
            if ((spins & 31) == 31 &&
                __hip_atomic_load(sync, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                ok = 0;
                break;
            }
            if (spins >= spin_limit) {
                __hip_atomic_store(sync, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
    }
    return __syncthreads_and(ok) != 0;
}

// All stores of this block completed, then store `value` to `word`.
__device__ __forceinline__ void publish_word(uint32_t* word, uint32_t value) {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_store(word, value, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Thread 0 waits until `word` >= value (bounded, watching the abort word);
// false in every thread if the wait ran out or another block aborted.
__device__ __forceinline__ bool wait_word(const uint32_t* word, uint32_t value, uint32_t* sync, int spin_limit,
                                          uint32_t* shared_ok) {
    if (threadIdx.x == 0) {
        uint32_t ok = 1;
        for (int spins = 0; __hip_atomic_load(word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < value; ++spins) {
            if ((spins & 31) == 31 && __hip_atomic_load(sync, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                ok = 0;
                break;
            }
            if (spins >= spin_limit) {
                __hip_atomic_store(sync, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        *shared_ok = ok;
    }
    __syncthreads();
    return *shared_ok != 0;
}

}  // namespace jko
