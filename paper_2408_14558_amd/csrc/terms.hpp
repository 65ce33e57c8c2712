// Enumeration of the products ("terms") a_ik * b_kj of one output column j
// of C = A~ * B_i (Gustavson's column-by-column formula): for every stored
// b_kj, the stored entries of A~'s column map[k].  Used by the symbolic,
// numeric and batched kernels.
#pragma once

#include "common.hpp"

namespace spg {

// LDS staging for one chunk of G entries of B(:,j).
template <int G, typename V>
struct EntryStage {
    int pref[G];          // exclusive prefix of the entries' term counts
    long long start[G];   // first position of the entry's column in A~
    V bv[G];              // b_kj
    int tmp[G / kWave + 2];
};

// Largest o in [0, n) with pref[o] <= s (pref non-decreasing from 0).
__device__ __forceinline__ int owner_of(const int *pref, int n, int s) {
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

// Visits every term of column j, spread evenly over the G threads of a group
// (gt = thread index inside the group).  f(p, bv) gets the position p of
// a_ik in A~ and b_kj.  All G threads must call it (it synchronises the
// group).  Terms of one chunk of G entries are handed out round-robin, so
// consecutive threads read consecutive entries of A~.
template <int G, typename V, typename F>
__device__ __forceinline__ void for_each_term(int64_t q0, int64_t q1,
                                              const int32_t *__restrict__ Browidx,
                                              const V *__restrict__ Bvals,
                                              const int32_t *__restrict__ map,
                                              const int64_t *__restrict__ At_colptr,
                                              EntryStage<G, V> *st, int gt, F &&f) {
    for (int64_t qb = q0; qb < q1; qb += G) {
        const int64_t q = qb + gt;
        int len = 0;
        long long start = 0;
        V bv = V(0);
        if (q < q1) {
            const int32_t jt = map[Browidx[q]];
            if (jt >= 0) {
                start = At_colptr[jt];
                len = (int)(At_colptr[jt + 1] - start);
                if (Bvals) bv = Bvals[q];
            }
        }
        int total;
        const int excl = group_excl_scan<G>(len, st->tmp, &total);
        st->pref[gt] = excl;
        st->start[gt] = start;
        st->bv[gt] = bv;
        group_sync<G>();
        for (int s = gt; s < total; s += G) {
            const int o = owner_of(st->pref, G, s);
            f((int64_t)(st->start[o] + (s - st->pref[o])), st->bv[o]);
        }
        group_sync<G>();
    }
}

// Same, restricted to the terms whose row lies in [r_lo, r_hi): each entry's
// sub-range is found by binary search in its (row-sorted) column of A~.
template <int G, typename V, typename F>
__device__ __forceinline__ void for_each_term_rows(int64_t q0, int64_t q1, int32_t r_lo,
                                                   int32_t r_hi,
                                                   const int32_t *__restrict__ Browidx,
                                                   const V *__restrict__ Bvals,
                                                   const int32_t *__restrict__ map,
                                                   const int64_t *__restrict__ At_colptr,
                                                   const int32_t *__restrict__ At_rowidx,
                                                   EntryStage<G, V> *st, int gt, F &&f) {
    for (int64_t qb = q0; qb < q1; qb += G) {
        const int64_t q = qb + gt;
        int len = 0;
        long long start = 0;
        V bv = V(0);
        if (q < q1) {
            const int32_t jt = map[Browidx[q]];
            if (jt >= 0) {
                int64_t lo = At_colptr[jt], hi = At_colptr[jt + 1];
                // first position with row >= r_lo
                int64_t a = lo, b = hi;
                while (a < b) {
                    const int64_t mid = (a + b) >> 1;
                    if (At_rowidx[mid] < r_lo) a = mid + 1; else b = mid;
                }
                const int64_t s0 = a;
                b = hi;
                while (a < b) {
                    const int64_t mid = (a + b) >> 1;
                    if (At_rowidx[mid] < r_hi) a = mid + 1; else b = mid;
                }
                start = s0;
                len = (int)(a - s0);
                if (Bvals) bv = Bvals[q];
            }
        }
        int total;
        const int excl = group_excl_scan<G>(len, st->tmp, &total);
        st->pref[gt] = excl;
        st->start[gt] = start;
        st->bv[gt] = bv;
        group_sync<G>();
        for (int s = gt; s < total; s += G) {
            const int o = owner_of(st->pref, G, s);
            f((int64_t)(st->start[o] + (s - st->pref[o])), st->bv[o]);
        }
        group_sync<G>();
    }
}

// The terms of a column with at most 64 of them, one per lane of a wave:
// lane s receives term s (p = its position in A~, bv = b_kj), lanes past the
// last term get p = -1.  All 64 lanes must call it.
template <typename V>
__device__ __forceinline__ void tiny_terms(int64_t q0, int64_t q1,
                                           const int32_t *__restrict__ Browidx,
                                           const V *__restrict__ Bvals,
                                           const int32_t *__restrict__ map,
                                           const int64_t *__restrict__ At_colptr, int64_t &p,
                                           V &bv) {
    const int lane = lane_id();
    p = -1;
    bv = V(0);
    int base = 0;
    for (int64_t qb = q0; qb < q1; qb += kWave) {
        const int64_t q = qb + lane;
        int len = 0;
        long long start = 0;
        V b = V(0);
        if (q < q1) {
            const int32_t jt = map[Browidx[q]];
            if (jt >= 0) {
                start = At_colptr[jt];
                len = (int)(At_colptr[jt + 1] - start);
                if (Bvals) b = Bvals[q];
            }
        }
        const int incl = wave_incl_scan(len);
        const int S = __shfl(incl, kWave - 1);
        const int s = lane - base;
        // first lane e with incl[e] > s
        int lo = 0, hi = kWave - 1;
#pragma unroll
        for (int it = 0; it < 6; ++it) {
            const int mid = (lo + hi) >> 1;
            const int v = __shfl(incl, mid);
            if (v > s) hi = mid; else lo = mid + 1;
        }
        const int e = lo;
        const int excl_e = __shfl(incl - len, e);
        const long long start_e = __shfl(start, e);
        const V b_e = __shfl(b, e);
        if (s >= 0 && s < S) {
            p = start_e + (s - excl_e);
            bv = b_e;
        }
        base += S;
    }
}

// Ascending bitonic sort of one (key, value) pair per lane across a wave.
template <typename V>
__device__ __forceinline__ void wave_sort_pairs(int &key, V &val) {
    const int l = lane_id();
#pragma unroll
    for (int kk = 2; kk <= kWave; kk <<= 1) {
#pragma unroll
        for (int jj = kk >> 1; jj > 0; jj >>= 1) {
            const int ok = __shfl_xor(key, jj);
            const V ov = __shfl_xor(val, jj);
            const bool up = (l & kk) == 0;
            const bool lower = (l & jj) == 0;
            const bool take = (lower == up) ? (ok < key) : (ok > key);
            if (take) {
                key = ok;
                val = ov;
            }
        }
    }
}

__device__ __forceinline__ void wave_sort_keys(int &key) {
    const int l = lane_id();
#pragma unroll
    for (int kk = 2; kk <= kWave; kk <<= 1) {
#pragma unroll
        for (int jj = kk >> 1; jj > 0; jj >>= 1) {
            const int ok = __shfl_xor(key, jj);
            const bool up = (l & kk) == 0;
            const bool lower = (l & jj) == 0;
            const bool take = (lower == up) ? (ok < key) : (ok > key);
            if (take) key = ok;
        }
    }
}

constexpr int kNoRow = 0x7fffffff;

}  // namespace spg
