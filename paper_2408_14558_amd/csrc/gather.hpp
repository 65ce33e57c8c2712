// Gather of the selected columns of A into A~ (Alg. 1: fetch the chosen
// blocks and build A~).  On one GPU a chosen block is a contiguous range of
// A's CSC arrays, so the fetch is a device copy.  Shared by the plan kernel
// and the persistent batched kernel.
#pragma once

#include "common.hpp"

namespace spg {

constexpr int kGatherCols = 64;
constexpr int kGatherThreads = 256;
constexpr int kUnrollCopy = 8;  // a tile of hub columns (10^5 entries) in few rounds
constexpr int kUnrollTail = 4;

struct GatherStage {
    int pref[kGatherCols];
    long long src[kGatherCols];
    long long dst[kGatherCols];
    int total;
};

// Largest o in [0, N) with pref[o] <= s (pref non-decreasing, pref[0] = 0;
// N a power of two).  A fixed number of branch-free steps, so that the
// searches of a thread's several elements overlap their LDS reads.
template <int N>
__device__ __forceinline__ int find_owner(const int *pref, int s) {
    static_assert((N & (N - 1)) == 0, "N must be a power of two");
    int o = 0;
#pragma unroll
    for (int step = N / 2; step > 0; step >>= 1) o += pref[o + step] <= s ? step : 0;
    return o;
}

// One round of a thread's copy: elements e0 + u * kGatherThreads, u < U.
template <int U, typename V, bool kRows>
__device__ __forceinline__ void copy_round(int e0, int total, const GatherStage &st,
                                           const int32_t *__restrict__ Arowidx,
                                           const V *__restrict__ Avals,
                                           int32_t *__restrict__ At_rowidx,
                                           V *__restrict__ At_vals) {
    long long dp[U];
    int32_t r[U];
    V v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int e = min(e0 + u * kGatherThreads, total - 1);
        const int o = find_owner<kGatherCols>(st.pref, e);
        const int64_t off = e - st.pref[o];
        const long long sp = st.src[o] + off;
        dp[u] = st.dst[o] + off;
        if (kRows) r[u] = Arowidx[sp];
        v[u] = Avals[sp];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        if (e0 + u * kGatherThreads < total) {
            if (kRows) At_rowidx[dp[u]] = r[u];
            At_vals[dp[u]] = v[u];
        }
    }
}

// Copies the selected columns among A's columns [tile*kGatherCols,
// (tile+1)*kGatherCols) into A~.  kGatherThreads threads (the workgroup) share
// the tile's copy evenly, kUnrollCopy loads in flight per thread.
// kRows = false copies values only (new values on the planned pattern).
template <typename V, bool kRows>
__device__ __forceinline__ void gather_tile(int64_t tile, const int64_t *__restrict__ Acolptr,
                                            const int32_t *__restrict__ Arowidx,
                                            const V *__restrict__ Avals,
                                            const int32_t *__restrict__ map,
                                            const int64_t *__restrict__ At_colptr, int64_t k,
                                            int32_t *__restrict__ At_rowidx,
                                            V *__restrict__ At_vals, GatherStage &st) {
    const int tid = threadIdx.x;
    if (tid < kWave) {
        int len = 0;
        long long src = 0, dst = 0;
        const int64_t c = tile * kGatherCols + tid;
        if (tid < kGatherCols && c < k) {
            const int32_t j = map[c];
            if (j >= 0) {
                src = Acolptr[c];
                len = (int)(Acolptr[c + 1] - src);
                dst = At_colptr[j];
            }
        }
        const int incl = wave_incl_scan(len);
        if (tid < kGatherCols) {
            st.pref[tid] = incl - len;
            st.src[tid] = src;
            st.dst[tid] = dst;
        }
        if (tid == kWave - 1) st.total = incl;
    }
    __syncthreads();
    const int total = st.total;
    int e0 = tid;
    // rounds whose kUnrollCopy slots all hold an element, then rounds of
    // kUnrollTail; every slot loads (past the end: the tile's last element
    // again), so the loads carry no branches and are in flight together
    for (; e0 + (kUnrollCopy - 1) * kGatherThreads < total; e0 += kUnrollCopy * kGatherThreads)
        copy_round<kUnrollCopy, V, kRows>(e0, total, st, Arowidx, Avals, At_rowidx, At_vals);
    for (; e0 < total; e0 += kUnrollTail * kGatherThreads)
        copy_round<kUnrollTail, V, kRows>(e0, total, st, Arowidx, Avals, At_rowidx, At_vals);
    __syncthreads();
}

}  // namespace spg
