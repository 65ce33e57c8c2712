// Device-side helpers shared by the gfx950 kernels of the local SpGEMM.
//
// Wave64 primitives (scans, bitonic steps over lanes), the chained-scan tile
// protocol used by every prefix sum of the path, and small atomics.  Nothing
// here is specific to one step of the method.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "internal.hpp"

namespace spg {

constexpr int kWave = 64;

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Compiler + LDS ordering point for lanes of one wave (a wave runs in
// lockstep, so only the compiler and LDS completion need fencing).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Synchronises a group of G threads: a wave-local fence when the group
// lies inside one wave, a workgroup barrier otherwise (then the group is the
// whole workgroup).
template <int G>
__device__ __forceinline__ void group_sync() {
    if constexpr (G <= kWave) {
        wave_sync();
    } else {
        __syncthreads();
    }
}

// Inclusive scan of an int over all 64 lanes with DPP moves (no LDS round
// trips): shifts by 1, 2, 4, 8 inside each row of 16 lanes, then lane 15
// of rows 0 and 2 added to rows 1 and 3, then lane 31 to rows 2 and 3.
// Lanes whose source lies outside the row read 0.  Every lane must be
// active.
__device__ __forceinline__ int wave_incl_scan_dpp(int v) {
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);  // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);  // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);  // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);  // row_shr:8
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);  // row_bcast:15
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);  // row_bcast:31
    return v;
}

// Inclusive scan over the lanes of a wave (width W, power of two <= 64).
template <int W = kWave, typename T>
__device__ __forceinline__ T wave_incl_scan(T v) {
    // 32-bit integers take the DPP scan (HIP's __popc returns unsigned int)
    if constexpr (W == kWave && (std::is_same<T, int>::value || std::is_same<T, unsigned>::value))
        return (T)wave_incl_scan_dpp((int)v);
    const int l = lane_id() & (W - 1);
#pragma unroll
    for (int d = 1; d < W; d <<= 1) {
        T o = __shfl_up(v, d, W);
        if (l >= d) v += o;
    }
    return v;
}

// The value of lane (lane ^ d).  For d = 1 and 2 (quad permutes), d = 4
// (shifts by 4 inside each row of 16 lanes, one per direction) and d = 8 (a
// rotation by 8 inside each row) DPP moves, with no LDS round trip; d = 16
// and 32 take a shuffle.  d must be a constant after unrolling (the DPP
// control is an immediate); every lane must be active.
__device__ __forceinline__ int lane_xor_i32(int v, int d) {
    if (d == 1) return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xf, 0xf, false);  // quad_perm [1,0,3,2]
    if (d == 2) return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xf, 0xf, false);  // quad_perm [2,3,0,1]
    if (d == 4) {
        const int up = __builtin_amdgcn_update_dpp(v, v, 0x104, 0xf, 0xf, false);  // row_shl:4
        const int dn = __builtin_amdgcn_update_dpp(v, v, 0x114, 0xf, 0xf, false);  // row_shr:4
        return (lane_id() & 4) ? dn : up;
    }
    if (d == 8) return __builtin_amdgcn_mov_dpp(v, 0x128, 0xf, 0xf, false);  // row_ror:8
    return __shfl_xor(v, d);
}

template <typename T>
__device__ __forceinline__ T lane_xor(T x, int d) {
    static_assert(sizeof(T) == 4 || sizeof(T) == 8, "32- or 64-bit values");
    if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(T, lane_xor_i32(__builtin_bit_cast(int, x), d));
    } else {
        const uint64_t u = __builtin_bit_cast(uint64_t, x);
        const uint32_t lo = (uint32_t)lane_xor_i32((int)(uint32_t)u, d);
        const uint32_t hi = (uint32_t)lane_xor_i32((int)(uint32_t)(u >> 32), d);
        return __builtin_bit_cast(T, ((uint64_t)hi << 32) | lo);
    }
}

// Lane 63's value, wave-uniform (a scalar register; no LDS round trip).
__device__ __forceinline__ int wave_last(int v) { return __builtin_amdgcn_readlane(v, kWave - 1); }

template <int W = kWave, typename T>
__device__ __forceinline__ T wave_sum(T v) {
    // 32-bit integers over a whole wave: the DPP scan and lane 63's total
    if constexpr (W == kWave && (std::is_same<T, int>::value || std::is_same<T, unsigned>::value))
        return (T)wave_last(wave_incl_scan_dpp((int)v));
#pragma unroll
    for (int d = W >> 1; d > 0; d >>= 1) v += __shfl_xor(v, d, W);
    return v;
}

template <int W = kWave, typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
    for (int d = W >> 1; d > 0; d >>= 1) {
        T o = __shfl_xor(v, d, W);
        v = o > v ? o : v;
    }
    return v;
}

// Number of set bits of a 64-bit lane mask below the calling lane.
__device__ __forceinline__ int lanes_below(uint64_t mask) {
    uint32_t lo = (uint32_t)mask, hi = (uint32_t)(mask >> 32);
    return __builtin_amdgcn_mbcnt_hi(hi, __builtin_amdgcn_mbcnt_lo(lo, 0u));
}

// Exclusive scan of one int value per thread over a group of G threads
// (G a power of two).  `tmp` is LDS scratch of at least G/64+1 ints when
// G > 64 (unused otherwise).  Returns the exclusive prefix; *total gets the
// group sum.  All G threads must call it.
template <int G>
__device__ __forceinline__ int group_excl_scan(int v, int *tmp, int *total) {
    if constexpr (G <= kWave) {
        int incl = wave_incl_scan<G>(v);
        *total = __shfl(incl, G - 1, G);
        return incl - v;
    } else {
        constexpr int NW = G / kWave;
        const int t = threadIdx.x;
        const int w = t / kWave;
        int incl = wave_incl_scan<kWave>(v);
        if (lane_id() == kWave - 1) tmp[w] = incl;
        __syncthreads();
        if (t < kWave) {
            int s = (t < NW) ? tmp[t] : 0;
            int si = wave_incl_scan<kWave>(s);
            if (t < NW) tmp[t] = si - s;
            if (t == kWave - 1) tmp[NW] = si;
        }
        __syncthreads();
        int res = tmp[w] + incl - v;
        *total = tmp[NW];
        __syncthreads();
        return res;
    }
}

template <int G>
__device__ __forceinline__ long long group_excl_scan64(long long v, long long *tmp,
                                                       long long *total) {
    if constexpr (G <= kWave) {
        long long incl = wave_incl_scan<G>(v);
        *total = __shfl(incl, G - 1, G);
        return incl - v;
    } else {
        constexpr int NW = G / kWave;
        const int t = threadIdx.x;
        const int w = t / kWave;
        long long incl = wave_incl_scan<kWave>(v);
        if (lane_id() == kWave - 1) tmp[w] = incl;
        __syncthreads();
        if (t < kWave) {
            long long s = (t < NW) ? tmp[t] : 0;
            long long si = wave_incl_scan<kWave>(s);
            if (t < NW) tmp[t] = si - s;
            if (t == kWave - 1) tmp[NW] = si;
        }
        __syncthreads();
        long long res = tmp[w] + incl - v;
        *total = tmp[NW];
        __syncthreads();
        return res;
    }
}

// ---------------------------------------------------------------------------
// Chained scan across workgroups (single pass, decoupled look-back).
//
// Every tile publishes one 64-bit status word: bits 62..63 hold the state
// (1 = tile aggregate, 2 = inclusive prefix), bits 0..61 the value.  A tile
// marked as a segment head publishes its inclusive prefix at once, so a
// look-back never crosses a head.  Tiles are handed out in launch order by
// an atomic ticket, so every tile a look-back waits on is already resident
// and finishes without waiting on later tiles.
// ---------------------------------------------------------------------------
constexpr uint64_t kStAgg = 1ull << 62;
constexpr uint64_t kStInc = 2ull << 62;
constexpr uint64_t kStMask = 3ull << 62;
constexpr uint64_t kValMask = ~kStMask;

// A status word carries all a look-back needs (state and value), and no
// tile reads data another tile wrote besides it: relaxed agent-scope stores
// and loads suffice (no L2 write-back per publish, no invalidation per poll;
// a release store here cost the two plan scans of an ER 65536 partition
// (16 per column, 4096 columns) about 4 us).
__device__ __forceinline__ void status_store(uint64_t *p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t status_load(uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Called by all 64 lanes of ONE wave of the tile (the same wave for the
// whole call).  Returns, in every lane, the exclusive prefix of `tile` and
// publishes its inclusive prefix.  The look-back reads 64 predecessor
// states per round trip: it sums the aggregates of the closest tiles up to
// and including the first one that already holds its inclusive prefix.
__device__ __forceinline__ long long chained_prefix(uint64_t *status, long long tile, bool head,
                                                    long long aggregate) {
    const int lane = lane_id();
    if (head) {
        if (lane == 0) status_store(&status[tile], kStInc | (uint64_t)aggregate);
        return 0;
    }
    if (lane == 0) status_store(&status[tile], kStAgg | (uint64_t)aggregate);
    long long prefix = 0;
    long long base = tile - 1;
    while (true) {
        const long long j = base - lane;
        // there is always an inclusive tile at or after index 0 (a head)
        const uint64_t s = j >= 0 ? status_load(&status[j]) : kStInc;
        const uint64_t st = s & kStMask;
        const uint64_t inc = __ballot(st == kStInc);
        const uint64_t notready = __ballot(st == 0);
        const int first = inc ? (__ffsll((unsigned long long)inc) - 1) : kWave;
        const uint64_t needed = first == kWave ? ~0ull : ((2ull << first) - 1ull);
        if (notready & needed) {
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        const long long v = lane <= first && j >= 0 ? (long long)(s & kValMask) : 0;
        prefix += wave_sum(v);
        if (first < kWave) break;
        base -= kWave;
    }
    if (lane == 0) status_store(&status[tile], kStInc | (uint64_t)(prefix + aggregate));
    return prefix;
}

// Run by every thread of one workgroup once the counters are final: copies
// the counters the host needs to `out` (pinned host memory), so no separate
// device-to-host copy is needed, then sets *ready to 1 with a system-scope
// release store: the host may read `out` as soon as it sees the flag.
__device__ __forceinline__ void publish_counters(const DevCounters *ctr, PublishedCounts *out,
                                                 unsigned int *ready) {
    const int t = threadIdx.x;
    if (t == 0)
        out->flops = __hip_atomic_load(&ctr->flops.v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else if (t == 1)
        out->nnzC = __hip_atomic_load(&ctr->nnzC, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else if (t < 2 + kNumBins)
        out->sym_count[t - 2] = __hip_atomic_load(&ctr->sym_count[t - 2].v, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT);
    else if (t < 2 + 2 * kNumBins)
        out->num_count[t - 2 - kNumBins] = __hip_atomic_load(
            &ctr->num_count[t - 2 - kNumBins].v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else if (t == 2 + 2 * kNumBins)
        out->nnz_At = __hip_atomic_load(&ctr->nnz_At, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    // wave 0 wrote every field: thread 0's system-scope release store
    // orders them before the flag
    if (t == 0) __hip_atomic_store(ready, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Called by every thread of each of `groups` workgroups of a kernel, once,
// after the workgroup's last update of the counters: the workgroup that
// finishes last publishes them.  `done` counts the finished workgroups.
__device__ __forceinline__ void publish_when_last(unsigned long long *done,
                                                  unsigned long long groups,
                                                  const DevCounters *ctr, PublishedCounts *out,
                                                  unsigned int *ready, int *lds_flag) {
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();  // this workgroup's counter updates before its ticket
        *lds_flag = atomicAdd(done, 1ull) == groups - 1;
    }
    __syncthreads();
    if (*lds_flag) {
        __threadfence();  // every other workgroup's updates are visible
        publish_counters(ctr, out, ready);
    }
}

// Takes the next tile ticket (thread 0) and broadcasts it to the workgroup.
__device__ __forceinline__ long long take_ticket(unsigned long long *counter, long long *lds_slot) {
    if (threadIdx.x == 0) *lds_slot = (long long)atomicAdd(counter, 1ull);
    __syncthreads();
    long long t = *lds_slot;
    __syncthreads();
    return t;
}

// ---------------------------------------------------------------------------
// misc
// ---------------------------------------------------------------------------
// Slot of row r in a table of T (power of two) slots: the top log2(T) bits
// of r times 2^32/phi (Knuth's multiplicative hashing), so rows that differ
// only in high bits still spread over the table.
template <int T>
__device__ __forceinline__ uint32_t hash_slot(int32_t r) {
    static_assert((T & (T - 1)) == 0 && T >= 2, "table size must be a power of two");
    constexpr int kBits = __builtin_ctz(T);
    return ((uint32_t)r * 2654435761u) >> (32 - kBits);
}

__device__ __forceinline__ void atomic_add_i64(long long *p, long long v) {
    atomicAdd(reinterpret_cast<unsigned long long *>(p), (unsigned long long)v);
}

template <typename V>
__device__ __forceinline__ void lds_atomic_add(V *p, V v) {
    atomicAdd(p, v);
}

// Work queue of a launch with fewer workgroups than items (q[0]: next item,
// q[1]: workgroups finished): every workgroup takes items in turn until
// they run out, so no compute unit idles while items are left and the long
// items do not wait behind the dispatch order.  All threads of the group
// call; s_item is LDS.
__device__ __forceinline__ int queue_take(unsigned int *q, int *s_item) {
    __syncthreads();  // every thread has read the previous item
    if (threadIdx.x == 0) *s_item = (int)atomicAdd(&q[0], 1u);
    __syncthreads();
    return *s_item;
}

// Called once by every workgroup after its last queue_take: the last one to
// leave puts the queue back to 0 for the next launch.
__device__ __forceinline__ void queue_leave(unsigned int *q) {
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(&q[1], 1u) == gridDim.x - 1) {
            atomicExch(&q[0], 0u);
            atomicExch(&q[1], 0u);
        }
    }
}

// Copies n 32-bit words with all G threads of the workgroup (between LDS
// and global memory): 16-byte accesses when both pointers allow them, with
// up to two loads in flight per thread before their stores.
template <int G>
__device__ __forceinline__ void copy_words(uint32_t *dst, const uint32_t *src, int n) {
    int head = 0;
    if ((((uintptr_t)src | (uintptr_t)dst) & 15) == 0) {
        const int n4 = n >> 2;
        const uint4 *s4 = reinterpret_cast<const uint4 *>(src);
        uint4 *d4 = reinterpret_cast<uint4 *>(dst);
        for (int i0 = threadIdx.x; i0 < n4; i0 += 2 * G) {
            uint4 t[2];
#pragma unroll
            for (int u = 0; u < 2; ++u)
                if (i0 + u * G < n4) t[u] = s4[i0 + u * G];
#pragma unroll
            for (int u = 0; u < 2; ++u)
                if (i0 + u * G < n4) d4[i0 + u * G] = t[u];
        }
        head = n4 << 2;
    }
    for (int i = head + threadIdx.x; i < n; i += G) dst[i] = src[i];
}

// Sets n 32-bit words of LDS to 0 with all G threads (16-byte stores when
// aligned).
template <int G>
__device__ __forceinline__ void zero_words(uint32_t *dst, int n) {
    int head = 0;
    if ((((uintptr_t)dst) & 15) == 0) {
        const int n4 = n >> 2;
        uint4 *d4 = reinterpret_cast<uint4 *>(dst);
        for (int i = threadIdx.x; i < n4; i += G) d4[i] = make_uint4(0u, 0u, 0u, 0u);
        head = n4 << 2;
    }
    for (int i = head + threadIdx.x; i < n; i += G) dst[i] = 0u;
}

// Position of element i of an LDS staging buffer of 32-bit words, XOR-
// swizzled by its 32-word row: when every lane of a wave writes its own run
// of consecutive elements (one run per bitmap word), runs that start a
// multiple of 32 apart would all hit one LDS bank; swizzled they spread over
// the banks.  A row of 32 elements stays a permutation of itself, so reading
// 32 consecutive elements is conflict-free too.
__device__ __forceinline__ int swz(int i) { return i ^ ((i >> 5) & 31); }

// The same for a buffer of 64-bit elements (two banks each, 16 to a row of
// banks): accumulators whose indices a wave's lanes hit 8 or 16 apart
// spread over the banks instead of piling on a few.
__device__ __forceinline__ int swz64(int i) { return i ^ ((i >> 4) & 15); }

__device__ __forceinline__ int next_pow2(int x) {
    int p = 1;
    while (p < x) p <<= 1;
    return p;
}

}  // namespace spg
