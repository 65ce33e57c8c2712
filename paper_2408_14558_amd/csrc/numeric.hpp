// Numeric phase of C_i = A~ * B_i as device functions, one per column bin,
// so the plain per-bin kernels and the persistent batched kernel share them.
// Every function writes column j's row ids ascending at C_colptr[j] and the
// matching values (Sec. III-A, column-by-column formula).
#pragma once

#include "terms.hpp"

namespace spg {

// Everything a numeric column routine needs about one product.
template <typename V>
struct NumArgs {
    int64_t m;
    const int64_t *Bcolptr;
    const int32_t *Browidx;
    const V *Bvals;
    const int32_t *map;
    const int64_t *At_colptr;
    const int32_t *At_rowidx;
    const V *At_vals;
    const int64_t *Ccolptr;
    int32_t *Crow;
    V *Cval;
};

// --- tiny: <= 64 terms, one wave ------------------------------------------
template <typename V>
__device__ __forceinline__ void num_tiny_column(const NumArgs<V> &a, int32_t j) {
    int64_t p;
    V bv;
    tiny_terms<V>(a.Bcolptr[j], a.Bcolptr[j + 1], a.Browidx, a.Bvals, a.map, a.At_colptr, p, bv);
    int key = kNoRow;
    V val = V(0);
    if (p >= 0) {
        key = a.At_rowidx[p];
        val = a.At_vals[p] * bv;
    }
    wave_sort_pairs(key, val);
    const int lane = lane_id();
    // sum runs of equal rows (rows are sorted, so runs are contiguous)
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const int ok = __shfl_down(key, d);
        const V ov = __shfl_down(val, d);
        if (lane + d < kWave && ok == key) val += ov;
    }
    const int prev = __shfl_up(key, 1);
    const bool head = key != kNoRow && (lane == 0 || prev != key);
    const uint64_t mask = __ballot(head);
    if (head) {
        const int64_t o = a.Ccolptr[j] + lanes_below(mask);
        a.Crow[o] = key;
        a.Cval[o] = val;
    }
}

// --- hash: LDS table, compaction, bitonic sort -----------------------------
template <int T, int G, typename V>
struct NumHashLds {
    int keys[T];
    V vals[T];
    EntryStage<G, V> st;
};

// G threads (gt in [0, G)) compute column j with a table of T slots.  The
// column must hold at most T/2 distinct rows.  T == 8 * G.
template <int T, int G, typename V>
__device__ __forceinline__ void num_hash_column(const NumArgs<V> &a, int32_t j,
                                                NumHashLds<T, G, V> &L, int gt) {
    static_assert(T == 8 * G, "eight slots per thread");
    for (int s = gt; s < T; s += G) {
        L.keys[s] = -1;
        L.vals[s] = V(0);
    }
    group_sync<G>();
    for_each_term<G, V>(a.Bcolptr[j], a.Bcolptr[j + 1], a.Browidx, a.Bvals, a.map, a.At_colptr,
                        &L.st, gt, [&](int64_t p, V bv) {
                            const int32_t r = a.At_rowidx[p];
                            const V v = a.At_vals[p] * bv;
                            uint32_t h = hash_slot<T>(r);
                            while (true) {
                                const int old = atomicCAS(&L.keys[h], -1, r);
                                if (old == -1 || old == r) {
                                    lds_atomic_add(&L.vals[h], v);
                                    break;
                                }
                                h = (h + 1) & (T - 1);
                            }
                        });
    // compaction: every thread lifts its 8 slots into registers
    int kk[8];
    V vv[8];
    int c = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int s = gt + i * G;
        kk[i] = L.keys[s];
        vv[i] = L.vals[s];
        c += kk[i] != -1;
    }
    int nnz;
    const int base = group_excl_scan<G>(c, L.st.tmp, &nnz);
    group_sync<G>();
    int pos = base;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        if (kk[i] != -1) {
            L.keys[pos] = kk[i];
            L.vals[pos] = vv[i];
            ++pos;
        }
    }
    int n2 = 1;
    while (n2 < nnz) n2 <<= 1;
    for (int s = nnz + gt; s < n2; s += G) L.keys[s] = kNoRow;
    group_sync<G>();
    // bitonic sort of n2 (key, value) pairs, ascending
    for (int kk2 = 2; kk2 <= n2; kk2 <<= 1) {
        for (int jj = kk2 >> 1; jj > 0; jj >>= 1) {
            for (int i = gt; i < (n2 >> 1); i += G) {
                const int lo = ((i & ~(jj - 1)) << 1) | (i & (jj - 1));
                const int hi = lo + jj;
                const bool up = (lo & kk2) == 0;
                const int a0 = L.keys[lo], a1 = L.keys[hi];
                if ((a0 > a1) == up) {
                    L.keys[lo] = a1;
                    L.keys[hi] = a0;
                    const V t0 = L.vals[lo];
                    L.vals[lo] = L.vals[hi];
                    L.vals[hi] = t0;
                }
            }
            group_sync<G>();
        }
    }
    const int64_t o = a.Ccolptr[j];
    for (int e = gt; e < nnz; e += G) {
        a.Crow[o + e] = L.keys[e];
        a.Cval[o + e] = L.vals[e];
    }
    group_sync<G>();
}

// --- bitmap: medium columns when m is small --------------------------------
// A bitmap of all m rows plus per-word prefix counts in LDS give every row
// of the column its final position (its rank), so values are accumulated at
// that position and no sort is needed.  Two passes over the terms: rows,
// then values.  LDS (dynamic): bits[nw] u32 | wpre[nw] u16 | vals[vcap].
template <int G, typename V>
struct NumBitmapStatic {
    EntryStage<G, V> st;
    int red[G / kWave + 2];
};

template <int G, typename V>
__device__ __forceinline__ void num_bitmap_column(const NumArgs<V> &a, int32_t j, uint32_t *bits,
                                                  uint16_t *wpre, V *vals,
                                                  NumBitmapStatic<G, V> &S) {
    const int gt = threadIdx.x;
    const int nw = (int)((a.m + 31) >> 5);
    const int64_t q0 = a.Bcolptr[j], q1 = a.Bcolptr[j + 1];
    for (int i = gt; i < nw; i += G) bits[i] = 0u;
    __syncthreads();
    for_each_term<G, V>(q0, q1, a.Browidx, (const V *)nullptr, a.map, a.At_colptr, &S.st, gt,
                        [&](int64_t p, V) {
                            const int32_t r = a.At_rowidx[p];
                            atomicOr(&bits[r >> 5], 1u << (r & 31));
                        });
    const int per = (nw + G - 1) / G;
    const int w0 = gt * per, w1 = min(nw, w0 + per);
    int c = 0;
    for (int w = w0; w < w1; ++w) c += __popc(bits[w]);
    int total;
    int run = group_excl_scan<G>(c, S.red, &total);
    const int64_t o = a.Ccolptr[j];
    for (int w = w0; w < w1; ++w) {
        wpre[w] = (uint16_t)run;
        uint32_t b = bits[w];
        while (b) {
            a.Crow[o + run] = (w << 5) + __ffs(b) - 1;
            ++run;
            b &= b - 1;
        }
    }
    for (int i = gt; i < total; i += G) vals[i] = V(0);
    __syncthreads();
    for_each_term<G, V>(q0, q1, a.Browidx, a.Bvals, a.map, a.At_colptr, &S.st, gt,
                        [&](int64_t p, V bv) {
                            const int32_t r = a.At_rowidx[p];
                            const uint32_t w = bits[r >> 5];
                            const int rk = wpre[r >> 5] + __popc(w & ((1u << (r & 31)) - 1u));
                            lds_atomic_add(&vals[rk], a.At_vals[p] * bv);
                        });
    for (int i = gt; i < total; i += G) a.Cval[o + i] = vals[i];
    __syncthreads();
}

// --- dense: bitmap of all m rows + rank windows -----------------------------
// LDS layout (dynamic): bits[nw] | wpre[nw] | vals[VC]
template <typename V>
struct NumDenseStatic {
    EntryStage<kDenseThreads, V> st;
    long long red64[kDenseThreads / kWave + 2];
    int red[kDenseThreads / kWave + 2];
    int r_lo, r_hi;
};

__device__ __forceinline__ int rank_of(const uint32_t *bits, const int *wpre, int32_t r) {
    const uint32_t w = bits[r >> 5];
    return wpre[r >> 5] + __popc(w & ((1u << (r & 31)) - 1u));
}

// Row holding rank R (0 <= R < total) of the bitmap.
__device__ __forceinline__ int32_t row_of_rank(const uint32_t *bits, const int *wpre, int nw,
                                               int R) {
    int lo = 0, hi = nw - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (wpre[mid] <= R) lo = mid; else hi = mid - 1;
    }
    uint32_t w = bits[lo];
    int need = R - wpre[lo];
    while (need-- > 0) w &= w - 1;  // drop lower set bits
    return (lo << 5) + __ffs(w) - 1;
}

// kDenseThreads threads compute column j.  VC values fit in LDS at once;
// columns with more rows are done in windows of VC consecutive ranks.
template <typename V>
__device__ __forceinline__ void num_dense_column(const NumArgs<V> &a, int32_t j, uint32_t *bits,
                                                 int *wpre, V *vals, int VC,
                                                 NumDenseStatic<V> &S) {
    const int gt = threadIdx.x;
    const int nw = (int)((a.m + 31) >> 5);
    const int64_t q0 = a.Bcolptr[j], q1 = a.Bcolptr[j + 1];
    for (int i = gt; i < nw; i += kDenseThreads) bits[i] = 0u;
    __syncthreads();
    for_each_term<kDenseThreads, V>(q0, q1, a.Browidx, (const V *)nullptr, a.map, a.At_colptr,
                                    &S.st, gt, [&](int64_t p, V) {
                                        const int32_t r = a.At_rowidx[p];
                                        atomicOr(&bits[r >> 5], 1u << (r & 31));
                                    });
    // per-word exclusive prefix of set bits; each thread owns a run of words
    const int per = (nw + kDenseThreads - 1) / kDenseThreads;
    const int w0 = gt * per, w1 = min(nw, w0 + per);
    int c = 0;
    for (int w = w0; w < w1; ++w) c += __popc(bits[w]);
    int total;
    int run = group_excl_scan<kDenseThreads>(c, S.red, &total);
    const int64_t o = a.Ccolptr[j];
    for (int w = w0; w < w1; ++w) {
        wpre[w] = run;
        uint32_t b = bits[w];
        int r = run;
        while (b) {
            const int bit = __ffs(b) - 1;
            a.Crow[o + r] = (w << 5) + bit;
            ++r;
            b &= b - 1;
        }
        run = r;
    }
    __syncthreads();
    for (int w0r = 0; w0r < total; w0r += VC) {
        const int w1r = min(total, w0r + VC);
        const int cnt = w1r - w0r;
        for (int i = gt; i < cnt; i += kDenseThreads) vals[i] = V(0);
        if (gt == 0) {
            S.r_lo = row_of_rank(bits, wpre, nw, w0r);
            S.r_hi = (w1r == total) ? (int32_t)a.m : row_of_rank(bits, wpre, nw, w1r);
        }
        __syncthreads();
        auto acc = [&](int64_t p, V bv) {
            const int32_t r = a.At_rowidx[p];
            lds_atomic_add(&vals[rank_of(bits, wpre, r) - w0r], a.At_vals[p] * bv);
        };
        if (cnt == total) {
            for_each_term<kDenseThreads, V>(q0, q1, a.Browidx, a.Bvals, a.map, a.At_colptr,
                                            &S.st, gt, acc);
        } else {
            const int32_t rl = S.r_lo, rh = S.r_hi;
            for_each_term_rows<kDenseThreads, V>(q0, q1, rl, rh, a.Browidx, a.Bvals, a.map,
                                                 a.At_colptr, a.At_rowidx, &S.st, gt, acc);
        }
        for (int i = gt; i < cnt; i += kDenseThreads) a.Cval[o + w0r + i] = vals[i];
        __syncthreads();
    }
}

}  // namespace spg
