// Gather of the selected columns of A into A~ (Alg. 1: fetch the chosen
// blocks and build A~).  On one GPU a chosen block is a contiguous range of
// A's CSC arrays, so the fetch is a device copy.  Shared by the plan kernel
// and the persistent batched kernel.
#pragma once

#include "common.hpp"

namespace spg {

constexpr int kGatherCols = 64;
constexpr int kGatherThreads = 256;
constexpr int kUnrollCopy = 4;

struct GatherStage {
    int pref[kGatherCols];
    long long src[kGatherCols];
    long long dst[kGatherCols];
    int total;
};

// Largest o in [0, n) with pref[o] <= s (pref non-decreasing, pref[0] = 0).
__device__ __forceinline__ int find_owner(const int *pref, int n, int s) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pref[mid] <= s)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
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
    for (int e0 = tid; e0 < total; e0 += kUnrollCopy * kGatherThreads) {
        long long dp[kUnrollCopy];
        int32_t r[kUnrollCopy];
        V v[kUnrollCopy];
#pragma unroll
        for (int u = 0; u < kUnrollCopy; ++u) {
            const int e = e0 + u * kGatherThreads;
            if (e < total) {
                const int o = find_owner(st.pref, kGatherCols, e);
                const int64_t off = e - st.pref[o];
                const long long sp = st.src[o] + off;
                dp[u] = st.dst[o] + off;
                if (kRows) r[u] = Arowidx[sp];
                v[u] = Avals[sp];
            }
        }
#pragma unroll
        for (int u = 0; u < kUnrollCopy; ++u) {
            const int e = e0 + u * kGatherThreads;
            if (e < total) {
                if (kRows) At_rowidx[dp[u]] = r[u];
                At_vals[dp[u]] = v[u];
            }
        }
    }
    __syncthreads();
}

}  // namespace spg
