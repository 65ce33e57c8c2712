// Numeric phase of C_i = A~ * B_i as device functions, one per column bin,
// so the plain per-bin kernels and the persistent batched kernel share them.
// Every function writes column j's row ids ascending at C_colptr[j] and the
// matching values (Sec. III-A, column-by-column formula).
#pragma once

#include "terms.hpp"

namespace spg {

// Products are accumulated in LDS as doubles whatever the value type: an
// FP32 product of two FP32 values is exact in FP64, and LDS atomic adds of
// doubles run several times faster than those of floats on gfx950 (measured
// on the R-MAT 18 term stream: 4.8 against 16.4 ms).  A column's values are
// rounded to the value type once, when written.
using Acc = double;

template <typename V>
__device__ __forceinline__ Acc prod(V a, V b) {
    return (Acc)a * (Acc)b;
}

// Everything a numeric column routine needs about one product.
template <typename V>
struct NumArgs {
    int64_t m;
    const int64_t *Bcolptr;
    TermRange tr;  // per entry of B_i: its products' positions in A~
    const V *Bvals;
    const int32_t *At_rowidx;
    const V *At_vals;
    const int64_t *Ccolptr;
    int32_t *Crow;
    V *Cval;
    const int64_t *flop;  // sparse flops per column (picks the wave-sort width)
    const int32_t *Browidx;      // B_i's row ids (the split table is indexed by them)
    const int32_t *split;        // split table (windows of dense columns), see internal.hpp
    const int32_t *col_slot;     // per column: its slot in dense_bits or tiny_perm, or -1
    const uint32_t *dense_bits;  // row bitmaps kept by the symbolic phase
    const uint16_t *tiny_perm;   // sorted term order of tiny columns kept by the symbolic phase
    int32_t nblk;                // row blocks of the split table (its stride is nblk + 1)
};

// --- wave sort: <= 64*E terms, one wave, registers ---------------------------
// Terms are gathered into registers, sorted by row across the wave, equal
// rows are merged by LDS atomics at their output slot, and the column is
// written out coalesced.  s_rows/s_vals: this wave's 64*E LDS slots.
//
// kPacked (rows below 2^22): the key of a term is (row << 9) | slot, where
// slot (< 64*8) is where the term's value waits in LDS, so the sort moves one
// 32-bit word per term instead of a key and a value; after the sort every
// lane fetches its values from LDS by slot.

// q0, q1: the column's entries of B_i; o: its first output position; perm:
// its kept sort order or NULL (all loaded by the caller up front, so that
// they travel together instead of as a chain of round trips).
template <int E, typename V, bool kPacked>
__device__ __forceinline__ void num_wave_column(const NumArgs<V> &a, int64_t q0, int64_t q1,
                                                int64_t o, int *s_rows, Acc *s_vals,
                                                const uint16_t *perm) {
    static_assert(E * kWave <= (1 << kSlotBits), "slot ids need kSlotBits bits");
    const int lane = lane_id();
    uint16_t sl[E];
    if (perm) {
#pragma unroll
        for (int r = 0; r < E; ++r) sl[r] = perm[lane * E + r];  // in flight with the terms
    }
    int64_t p[E];
    V bv[E];
    wave_terms<E, V>(q0, q1, a.tr, a.Bvals, p, bv);
    int key[E];
    Acc val[E];
    if (perm) {
        // the symbolic phase kept the sorted order of the slots: rows and
        // values wait in LDS by slot and are read back in that order.  Every
        // slot loads and parks (an empty one reads A~'s entry 0, and the kept
        // order never names it), so the loads carry no branches and are in
        // flight together.
        int32_t rw[E];
        V av[E];
#pragma unroll
        for (int r = 0; r < E; ++r) {
            const int64_t q = p[r] >= 0 ? p[r] : 0;
            rw[r] = a.At_rowidx[q];
            av[r] = a.At_vals[q];
        }
#pragma unroll
        for (int r = 0; r < E; ++r) {
            const int slot = r * kWave + lane;
            s_rows[slot] = rw[r];
            s_vals[slot] = prod(av[r], bv[r]);
        }
        wave_sync();
#pragma unroll
        for (int r = 0; r < E; ++r) {
            const bool some = sl[r] != kNoSlot;
            const int at = some ? sl[r] : 0;
            const int rr = s_rows[at];
            const Acc vv = s_vals[at];
            key[r] = some ? rr : kNoRow;
            val[r] = some ? vv : Acc(0);
        }
        wave_sync();  // every slot is read before the buffers are reused below
    } else {
    // loads without branches, as above
    int32_t rw[E];
    V av[E];
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const int64_t q = p[r] >= 0 ? p[r] : 0;
        rw[r] = a.At_rowidx[q];
        av[r] = a.At_vals[q];
    }
#pragma unroll
    for (int r = 0; r < E; ++r) {
        key[r] = kNoRow;
        val[r] = Acc(0);
        const Acc v = prod(av[r], bv[r]);
        if constexpr (kPacked) {
            const int slot = r * kWave + lane;
            s_vals[slot] = v;
            if (p[r] >= 0) key[r] = (rw[r] << kSlotBits) | slot;
        } else if (p[r] >= 0) {
            key[r] = rw[r];
            val[r] = v;
        }
    }
    if constexpr (kPacked) {
        wave_sort<E, false, Acc>(key, val);
        wave_sync();
#pragma unroll
        for (int r = 0; r < E; ++r) {
            if (key[r] != kNoRow) {
                val[r] = s_vals[key[r] & ((1 << kSlotBits) - 1)];
                key[r] >>= kSlotBits;
            }
        }
        wave_sync();  // every value is read before the slots are reused below
    } else {
        wave_sort<E, true, Acc>(key, val);
    }
    }
    const int prev_last = __shfl_up(key[E - 1], 1);
    bool hd[E];
    int nh = 0;
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const int prev = r == 0 ? prev_last : key[r - 1];
        hd[r] = key[r] != kNoRow && ((r == 0 && lane == 0) || key[r] != prev);
        nh += hd[r];
    }
    const int incl = wave_incl_scan(nh);
    const int total = wave_last(incl);
    for (int e = lane; e < total; e += kWave) s_vals[e] = Acc(0);
    wave_sync();
    int run = incl - nh - 1;
#pragma unroll
    for (int r = 0; r < E; ++r) {
        if (key[r] != kNoRow) {
            if (hd[r]) {
                ++run;
                s_rows[run] = key[r];
            }
            lds_atomic_add(&s_vals[run], val[r]);
        }
    }
    wave_sync();
    for (int e = lane; e < total; e += kWave) {
        a.Crow[o + e] = s_rows[e];
        a.Cval[o + e] = (V)s_vals[e];
    }
    wave_sync();
}

// Picks the register width from the column's flops; EMAX bounds it (a
// kernel built for EMAX = 4 needs no registers for 8 terms per lane).
template <typename V, int EMAX, bool kPacked>
__device__ __forceinline__ void num_wave_dispatch(const NumArgs<V> &a, int32_t j, int *s_rows,
                                                  Acc *s_vals) {
    static_assert(EMAX == 4 || EMAX == 8, "EMAX is 4 or 8");
    // every per-column load at once
    const int64_t f = a.flop[j];
    const int slot = a.tiny_perm ? a.col_slot[j] : -1;
    const int64_t q0 = a.Bcolptr[j], q1 = a.Bcolptr[j + 1], o = a.Ccolptr[j];
    const uint16_t *perm = slot >= 0 ? a.tiny_perm + (size_t)slot * (EMAX * kWave) : nullptr;
    if (f <= kWave) num_wave_column<1, V, kPacked>(a, q0, q1, o, s_rows, s_vals, perm);
    else if (f <= 2 * kWave) num_wave_column<2, V, kPacked>(a, q0, q1, o, s_rows, s_vals, perm);
    else if (EMAX == 4 || f <= 4 * kWave)
        num_wave_column<4, V, kPacked>(a, q0, q1, o, s_rows, s_vals, perm);
    else num_wave_column<EMAX, V, kPacked>(a, q0, q1, o, s_rows, s_vals, perm);
}

// --- hash: LDS table, compaction, bitonic sort -----------------------------
template <int T, int G, typename V>
struct NumHashLds {
    int keys[T];
    Acc vals[T];
    TermStage<G, V> st;
};

// G threads (gt in [0, G)) compute column j with a table of T slots.  The
// column must hold at most T/2 distinct rows.  Each thread owns T/G slots.
template <int T, int G, typename V>
__device__ __forceinline__ void num_hash_column(const NumArgs<V> &a, int32_t j,
                                                NumHashLds<T, G, V> &L, int gt) {
    static_assert(T % G == 0 && T / G <= 16, "slots per thread");
    constexpr int SL = T / G;
    for (int s = gt; s < T; s += G) {
        L.keys[s] = -1;
        L.vals[s] = Acc(0);
    }
    group_sync<G>();
    for_each_term<G, V>(a.Bcolptr[j], a.Bcolptr[j + 1], a.tr, a.Bvals,
                        &L.st, gt,
                        [&](int64_t p) { return RowVal<V>{a.At_rowidx[p], a.At_vals[p]}; },
                        [&](const RowVal<V> &t, V bv) {
                            const int32_t r = t.r;
                            const Acc v = prod(t.v, bv);
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
    // compaction: every thread lifts its slots into registers
    int kk[SL];
    Acc vv[SL];
    int c = 0;
#pragma unroll
    for (int i = 0; i < SL; ++i) {
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
    for (int i = 0; i < SL; ++i) {
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
                    const Acc t0 = L.vals[lo];
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
        a.Cval[o + e] = (V)L.vals[e];
    }
    group_sync<G>();
}

// --- bitmap ranks -------------------------------------------------------------
// A bitmap of the column's rows in LDS (bits[nw]) gives every row its output
// position: its rank, the number of set bits before it.  wpre[w] holds the
// rank of word w's first bit, relative to its superblock of 2048 words,
// whose rank is sbase[w >> 11] (no superblocks: sbase == nullptr and ranks
// must stay below 65536).
constexpr int kSuperShift = 11;
constexpr int kMaxSuper = 16;

// Fills wpre (and sbase), stages the row ids of ranks [0, cap) in stage[]
// (LDS, int32, at swz(rank); cap a multiple of 32) and returns the number of
// set bits.  Every wave takes a
// power-of-two range of consecutive words (at most 2048 when superblocks are
// used, so every superblock starts a wave's range) and its lanes consecutive
// words, so the LDS accesses are free of bank conflicts.  All G threads
// call; ends with a group barrier.  red: G/64 + 2 ints of LDS.
template <int G>
__device__ __forceinline__ int bitmap_ranks(const uint32_t *bits, uint16_t *wpre, int *sbase,
                                            int nw, int *red, int32_t *stage, int cap) {
    constexpr int NW = G / kWave;
    const int lane = lane_id(), wv = threadIdx.x / kWave;
    int per = kWave;
    while (per * NW < nw) per <<= 1;
    const int wb = min(nw, wv * per), we = min(nw, wb + per);
    int mine = 0;
    for (int w = wb + lane; w < we; w += kWave) mine += __popc(bits[w]);
    const int wave_total = wave_sum(mine);
    int total;
    const int pre = group_excl_scan<G>(lane == 0 ? wave_total : 0, red, &total);
    const int off = __shfl(pre, 0);
    int sb = 0;
    if (sbase) {
        if (lane == 0 && wb < we && (wb & ((1 << kSuperShift) - 1)) == 0)
            sbase[wb >> kSuperShift] = off;
        __syncthreads();
        if (wb < we) sb = sbase[wb >> kSuperShift];
    }
    int run = off;
    for (int w0 = wb; w0 < we; w0 += kWave) {
        const int w = w0 + lane;
        uint32_t b = w < we ? bits[w] : 0u;
        const int c = __popc(b);
        const int incl = wave_incl_scan(c);
        int rk = run + incl - c;
        if (w < we) {
            wpre[w] = (uint16_t)(rk - sb);
            while (b && rk < cap) {
                stage[swz(rk)] = (w << 5) + __ffs(b) - 1;
                ++rk;
                b &= b - 1;
            }
        }
        run += wave_last(incl);
    }
    __syncthreads();
    return total;
}

// A kept bitmap copied from device memory into LDS with the word ranks of
// bitmap_ranks (superblock bases included) computed on the way: each wave
// takes the same range of words as there and holds them in registers, so
// the bitmap is read once instead of once for the copy and twice for the
// ranks.  G = 1024 threads and at most 8192 words (one band): at most eight
// words per lane.  All G threads call; ends with a group barrier.
template <int G>
__device__ __forceinline__ int load_bitmap_ranks(const uint32_t *__restrict__ src, uint32_t *bits,
                                                 uint16_t *wpre, int *sbase, int nw, int *red) {
    constexpr int NW = G / kWave;
    constexpr int kRegs = 8;
    static_assert(NW * kWave * kRegs >= (int)(kMaxDenseRows >> 5), "eight words per lane");
    const int lane = lane_id(), wv = threadIdx.x / kWave;
    int per = kWave;
    while (per * NW < nw) per <<= 1;
    const int wb = min(nw, wv * per), we = min(nw, wb + per);
    uint32_t wr[kRegs];
#pragma unroll
    for (int i = 0; i < kRegs; ++i) {
        const int w = wb + i * kWave + lane;
        wr[i] = w < we ? src[w] : 0u;
    }
    int mine = 0;
#pragma unroll
    for (int i = 0; i < kRegs; ++i) {
        const int w = wb + i * kWave + lane;
        if (w < we) bits[w] = wr[i];
        mine += __popc(wr[i]);
    }
    const int wave_total = wave_sum(mine);
    int total;
    const int pre = group_excl_scan<G>(lane == 0 ? wave_total : 0, red, &total);
    const int off = __shfl(pre, 0);
    if (lane == 0 && wb < we && (wb & ((1 << kSuperShift) - 1)) == 0)
        sbase[wb >> kSuperShift] = off;
    __syncthreads();
    const int sb = wb < we ? sbase[wb >> kSuperShift] : 0;
    int run = off;
#pragma unroll
    for (int i = 0; i < kRegs; ++i) {
        if (wb + i * kWave >= we) break;  // the same for the whole wave
        const int w = wb + i * kWave + lane;
        const int c = __popc(wr[i]);
        const int incl = wave_incl_scan(c);
        if (w < we) wpre[w] = (uint16_t)(run + incl - c - sb);
        run += wave_last(incl);
    }
    __syncthreads();
    return total;
}

__device__ __forceinline__ int word_rank(const uint16_t *wpre, const int *sbase, int w) {
    return (sbase ? sbase[w >> kSuperShift] : 0) + wpre[w];
}

// Writes the set rows of the bitmap in ascending order to out[0, total):
// ranks [0, cap) were staged by bitmap_ranks; later ones are staged here,
// cap at a time.  Copies are coalesced.  All G threads call; ends with a
// group barrier.
template <int G>
__device__ __forceinline__ void bitmap_rows_out(const uint32_t *bits, const uint16_t *wpre,
                                                const int *sbase, int nw, int total,
                                                int32_t *stage, int cap,
                                                int32_t *__restrict__ out) {
    for (int r0 = 0; r0 < total; r0 += cap) {
        const int r1 = min(total, r0 + cap);
        if (r0 > 0) {
            for (int w = threadIdx.x; w < nw; w += G) {
                uint32_t b = bits[w];
                if (!b) continue;
                int rk = word_rank(wpre, sbase, w);
                if (rk >= r1 || rk + __popc(b) <= r0) continue;
                while (b) {
                    if (rk >= r0 && rk < r1) stage[swz(rk - r0)] = (w << 5) + __ffs(b) - 1;
                    ++rk;
                    b &= b - 1;
                }
            }
            __syncthreads();
        }
        for (int i = threadIdx.x; i < r1 - r0; i += G) out[r0 + i] = stage[swz(i)];
        __syncthreads();
    }
}

// --- bitmap: medium columns when m is small --------------------------------
// A bitmap of all m rows plus per-word prefix counts in LDS give every row
// of the column its final position (its rank), so values are accumulated at
// that position and no sort is needed.  Two passes over the terms: rows,
// then values.  LDS (dynamic): bits[nw] u32 | wpre[nw] u16 | vals[vcap].
template <int G, typename V>
struct NumBitmapStatic {
    TermStage<G, V> st;
    int red[G / kWave + 2];
};

// Which kernel takes a medium bin of table size `table`: the LDS bitmap over
// all m rows (true) instead of the LDS hash, when the bitmap is not much
// larger than the table and fits next to the values (medium_kernel 0), or
// whenever it fits in 96 KB (medium_kernel 2; 1: always the hash).  *lds:
// the bitmap kernel's dynamic LDS bytes.
inline bool medium_uses_bitmap(int64_t m, int table, int medium_kernel, size_t vsize,
                               size_t *lds) {
    const size_t nw = (size_t)((m + 31) / 32);
    *lds = ((nw * 6 + 15) & ~(size_t)15) + (size_t)(table / 2) * vsize;
    const bool small = *lds <= 96 * 1024;
    return (medium_kernel == 0 && small && nw <= (size_t)8 * table) ||
           (medium_kernel == 2 && small);
}

template <int G, typename V>
__device__ __forceinline__ void num_bitmap_column(const NumArgs<V> &a, int32_t j, uint32_t *bits,
                                                  uint16_t *wpre, Acc *vals, int vcap,
                                                  NumBitmapStatic<G, V> &S) {
    const int gt = threadIdx.x;
    const int nw = (int)((a.m + 31) >> 5);
    const int64_t q0 = a.Bcolptr[j], q1 = a.Bcolptr[j + 1];
    zero_words<G>(bits, nw);
    __syncthreads();
    for_each_term<G, V>(q0, q1, a.tr, (const V *)nullptr, &S.st, gt,
                        [&](int64_t p) { return a.At_rowidx[p]; },
                        [&](int32_t r, V) { atomicOr(&bits[r >> 5], 1u << (r & 31)); });
    // vals holds every value of the column: as int32 slots it stages the row ids
    const int cap = vcap * (int)(sizeof(Acc) / sizeof(int32_t));
    int32_t *stage = reinterpret_cast<int32_t *>(vals);
    const int total = bitmap_ranks<G>(bits, wpre, nullptr, nw, S.red, stage, cap);
    const int64_t o = a.Ccolptr[j];
    bitmap_rows_out<G>(bits, wpre, nullptr, nw, total, stage, cap, a.Crow + o);
    for (int i = gt; i < total; i += G) vals[i] = Acc(0);
    __syncthreads();
    for_each_term<G, V>(q0, q1, a.tr, a.Bvals, &S.st, gt,
                        [&](int64_t p) { return RowVal<V>{a.At_rowidx[p], a.At_vals[p]}; },
                        [&](const RowVal<V> &t, V bv) {
                            const uint32_t w = bits[t.r >> 5];
                            const int rk = wpre[t.r >> 5] + __popc(w & ((1u << (t.r & 31)) - 1u));
                            lds_atomic_add(&vals[rk], prod(t.v, bv));
                        });
    for (int i = gt; i < total; i += G) a.Cval[o + i] = (V)vals[i];
    __syncthreads();
}

// --- dense: bitmap of all m rows + rank windows -----------------------------
// Loads in flight per lane on the long A~ columns of dense output columns:
// a wave walks pieces of this many rows of 64 terms.  Measured on the R-MAT
// scale-18 product: 3 beat 2 and 4 (numeric 13.42 against 13.64 and 13.55
// ms; window segments of a few hundred terms leave lanes of larger pieces
// idle, and the walk is bound by vector instruction issue).
#ifndef SPG_DENSE_UNROLL
#define SPG_DENSE_UNROLL 3
#endif
constexpr int kDenseUnroll = SPG_DENSE_UNROLL;
// Entries of B(:,j) staged at once by the dense kernel (its 1024 threads all
// walk the long ones).  A smaller stage leaves LDS for larger value windows,
// a larger one gives the flat short list more terms per round; measured on
// the R-MAT scale-18 product (short entries up to 64 terms): 512 beat 256 by
// 0.6 ms and 1024 by 0.5 ms of numeric time.
#ifndef SPG_DENSE_CHUNK
#define SPG_DENSE_CHUNK 512
#endif
constexpr int kDenseChunk = SPG_DENSE_CHUNK;
// LDS (dynamic): bits[nw] u32 | wpre[nw] u16 | vals[VC].  wpre holds each
// word's rank relative to its superblock of 2048 words (65536 rows), whose
// absolute rank is in sbase, so ranks above 65535 need no 32-bit table.

// Windows of one dense column computed at once (a column needing more is
// done in several batches).
constexpr int kWinBatch = 64;

template <int G, typename V>
struct NumDenseStatic {
    TermStage<kDenseChunk < G ? kDenseChunk : G, V> st;
    int red[G / kWave + 2];
    int sbase[kMaxSuper];
    int win[kWinBatch][6];  // first block, end block, first rank, end rank, first row, end row
    int nwin;
};


__device__ __forceinline__ int rank_of(const uint32_t *bits, const uint16_t *wpre,
                                       const int *sbase, int32_t r) {
    const int w = r >> 5;
    return word_rank(wpre, sbase, w) + __popc(bits[w] & ((1u << (r & 31)) - 1u));
}

// Row holding rank R (0 <= R < total) of the bitmap.
__device__ __forceinline__ int32_t row_of_rank(const uint32_t *bits, const uint16_t *wpre,
                                               const int *sbase, int nw, int R) {
    int lo = 0, hi = nw - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (word_rank(wpre, sbase, mid) <= R) lo = mid; else hi = mid - 1;
    }
    uint32_t w = bits[lo];
    int need = R - word_rank(wpre, sbase, lo);
    while (need-- > 0) w &= w - 1;  // drop lower set bits
    return (lo << 5) + __ffs(w) - 1;
}

// b_kj of term u of a batch: one value for all of a long entry's terms, or
// one per term (the flat list of short segments).
template <typename V>
__device__ __forceinline__ V pick(V b, int) { return b; }
template <typename V, int N>
__device__ __forceinline__ V pick(const V (&b)[N], int u) { return b[u]; }

// Writes the set rows (row0 + bit index) of bitmap words [wb, we) whose
// ranks lie in [r0, r0 + cnt) to out[0, cnt): every lane takes one word and stages its
// rows at their ranks in LDS (stage, cnt ints), then the group copies them
// out coalesced.  All G threads call; ends with a group barrier.
template <int G>
__device__ __forceinline__ void window_rows_out(const uint32_t *bits, const uint16_t *wpre,
                                                const int *sbase, int wb, int we, int r0, int cnt,
                                                int32_t row0, int32_t *stage,
                                                int32_t *__restrict__ out) {
    for (int w = wb + (int)threadIdx.x; w < we; w += G) {
        uint32_t b = bits[w];
        int rk = word_rank(wpre, sbase, w) - r0;
        while (b) {
            if (rk >= 0 && rk < cnt) stage[swz(rk)] = row0 + (w << 5) + __ffs(b) - 1;
            ++rk;
            b &= b - 1;
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < cnt; i += G) out[i] = stage[swz(i)];
    __syncthreads();
}

// G threads (the whole workgroup) compute column j.  The column's row
// bitmap (kept by the symbolic phase, or built here) and the rank of every
// word are held in LDS.  The column is done in windows of at most VC ranks:
// a window covers as many consecutive row blocks of the split table as fit,
// so it visits exactly the products whose rows it holds; a block with more
// than VC rows of C is split into windows of VC ranks that skip the rows
// outside.  One wave lays out the windows from the ranks at the block
// borders; per window the group writes the window's row ids, accumulates
// its values by rank in LDS and writes them.
//
// A column of more than kMaxDenseRows rows (m above 2^18) is done in bands
// of kMaxDenseRows rows, one after another: each band builds its own bitmap
// from exactly its products (its blocks of the split table) and its ranks
// follow those of the bands before it.
template <int G, typename V>
__device__ __forceinline__ void num_dense_column(const NumArgs<V> &a, int32_t j, uint32_t *bits,
                                                 uint16_t *wpre, Acc *vals, int VC,
                                                 NumDenseStatic<G, V> &S) {
    constexpr int CH = kDenseChunk < G ? kDenseChunk : G;
    constexpr int kBlockWords = (int)(kSplitRows >> 5);
    constexpr int kBandBlocks = (int)(kMaxDenseRows >> kSplitShift);
    const int gt = threadIdx.x;
    const bool banded = a.m > kMaxDenseRows;
    const int64_t q0 = a.Bcolptr[j], q1 = a.Bcolptr[j + 1];
    // a kept bitmap, if this run kept them (never for banded columns)
    const int slot = a.dense_bits && !banded ? a.col_slot[j] : -1;
    const int lane = lane_id();
    int32_t *stage = reinterpret_cast<int32_t *>(vals);
    int64_t o = a.Ccolptr[j];  // output position of the band's first rank
    // a column of at most CH entries keeps them in registers over all its
    // windows (loaded here, in flight with the bitmap's loads)
    const bool cached = q1 - q0 <= CH;
    EntryRegs<V> er;
    if (cached) er = load_entry<CH, V>(q0, q1, a.tr, a.Browidx, a.Bvals, gt);
    for (int32_t R0 = 0; R0 < a.m; R0 += (int32_t)kMaxDenseRows) {
        const int32_t R1 = (int32_t)min<int64_t>(a.m, (int64_t)R0 + kMaxDenseRows);
        const int nw = (R1 - R0 + 31) >> 5;
        const int sb0 = R0 >> kSplitShift;  // the band's first block
        int total = -1;  // set with the ranks when a kept bitmap is loaded
        if (slot >= 0) {  // the symbolic phase kept this column's row bitmap
            total = load_bitmap_ranks<G>(a.dense_bits + (size_t)slot * nw, bits, wpre, S.sbase,
                                         nw, S.red);
        } else if (!banded) {
            zero_words<G>(bits, nw);
            __syncthreads();
            for_each_term<G, V, kDenseUnroll, CH>(
                q0, q1, a.tr, (const V *)nullptr, &S.st, gt,
                [&](int64_t p) { return a.At_rowidx[p]; },
                [&](int32_t r, V) { atomicOr(&bits[r >> 5], 1u << (r & 31)); });
        } else {  // the band's products only
            zero_words<G>(bits, nw);
            __syncthreads();
            auto mark = [&](const auto &r, const auto &, const auto &, const auto &ok) {
                constexpr int N = (int)(sizeof(ok) / sizeof(ok[0]));
#pragma unroll
                for (int u = 0; u < N; ++u)
                    if (ok[u]) atomicOr(&bits[(r[u] - R0) >> 5], 1u << (r[u] & 31));
            };
            for_each_window_term<G, V, kDenseUnroll, CH, decltype(mark) &, false>(
                q0, q1, false, sb0, min(a.nblk, sb0 + kBandBlocks), a.nblk, R0, R1, a.tr,
                a.Browidx, a.split, (const V *)nullptr, a.At_rowidx, (const V *)nullptr, &S.st,
                gt, mark);
            __syncthreads();
        }
        if (total < 0) total = bitmap_ranks<G>(bits, wpre, S.sbase, nw, S.red, nullptr, 0);
        const int nblk = (nw + kBlockWords - 1) / kBlockWords;  // blocks of the band (<= 32)
        for (int w0r = 0; w0r < total;) {
            if (gt < kWave) {
                // lane b holds the rank at the start of block b (b == nblk: total)
                const int rb = lane < nblk ? word_rank(wpre, S.sbase, lane * kBlockWords)
                                           : (lane == nblk ? total : 0x7fffffff);
                int n = 0;
                int r0 = w0r;
                while (r0 < total && n < kWinBatch) {
                    // the last block starting at or before rank r0, then the
                    // last block border at most VC ranks further
                    const uint64_t m0 = __ballot(lane < nblk && rb <= r0);
                    const int b0 = 63 - __clzll((long long)m0);
                    const uint64_t m1 = __ballot(lane > b0 && lane <= nblk && rb - r0 <= VC);
                    int b1, r1;
                    if (m1) {
                        b1 = 63 - __clzll((long long)m1);
                        r1 = __shfl(rb, b1);
                    } else {  // block b0 alone holds more than VC rows of C
                        b1 = b0 + 1;
                        r1 = r0 + VC;
                    }
                    if (lane == 0) {
                        int *wd = S.win[n];
                        wd[0] = b0;
                        wd[1] = b1;
                        wd[2] = r0;
                        wd[3] = r1;
                        // rows of the window: block borders when the ranks
                        // sit on them, else the rows holding ranks r0 and r1
                        const int rb0 = word_rank(wpre, S.sbase, b0 * kBlockWords);
                        const int rb1 =
                            b1 < nblk ? word_rank(wpre, S.sbase, b1 * kBlockWords) : total;
                        wd[4] = R0 + (r0 == rb0 ? (b0 << kSplitShift)
                                                : row_of_rank(bits, wpre, S.sbase, nw, r0));
                        wd[5] = r1 == rb1
                                    ? (int)min<int64_t>((int64_t)R0 + ((int64_t)b1 << kSplitShift), R1)
                                    : R0 + row_of_rank(bits, wpre, S.sbase, nw, r1);
                    }
                    ++n;
                    r0 = r1;
                }
                if (lane == 0) S.nwin = n;
            }
            __syncthreads();
            const int nwin = S.nwin;
            for (int wi = 0; wi < nwin; ++wi) {
                const int wb0 = S.win[wi][0], wb1 = S.win[wi][1];
                const int r0 = S.win[wi][2], r1 = S.win[wi][3];
                const int32_t rlo = S.win[wi][4], rhi = S.win[wi][5];
                const int cnt = r1 - r0;
                if (slot < 0)  // kept columns have their rows written by k_dense_rows
                    window_rows_out<G>(bits, wpre, S.sbase, wb0 * kBlockWords,
                                       min(nw, wb1 * kBlockWords), r0, cnt, R0, stage,
                                       a.Crow + o + r0);
                for (int i = gt; i < cnt; i += G) vals[swz64(i)] = Acc(0);
                __syncthreads();
                const bool full = !banded && r0 == 0 && r1 == total;
                // per batch: every rank lookup's LDS reads first, then the adds
                auto add = [&](const auto &r, const auto &av, const auto &bv, const auto &ok) {
                    constexpr int N = (int)(sizeof(ok) / sizeof(ok[0]));
                    constexpr int H = N < 4 ? N : 4;  // lookups in flight per step
#pragma unroll
                    for (int h = 0; h < N; h += H) {
                        uint32_t wb[H];
                        int wr[H];
#pragma unroll
                        for (int u = 0; u < H; ++u) {
                            const int w = ((ok[h + u] ? r[h + u] : rlo) - R0) >> 5;
                            wb[u] = bits[w];
                            wr[u] = word_rank(wpre, S.sbase, w);
                        }
#pragma unroll
                        for (int u = 0; u < H; ++u) {
                            if (ok[h + u]) {
                                const int rk =
                                    wr[u] + __popc(wb[u] & ((1u << (r[h + u] & 31)) - 1u));
                                lds_atomic_add(&vals[swz64(rk - r0)],
                                               prod(av[h + u], pick(bv, h + u)));
                            }
                        }
                    }
                };
                for_each_window_term<G, V, kDenseUnroll, CH>(
                    q0, q1, full, sb0 + wb0, sb0 + wb1, a.nblk, rlo, rhi, a.tr, a.Browidx,
                    a.split, a.Bvals, a.At_rowidx, a.At_vals, &S.st, gt, add, cached, er);
                for (int i = gt; i < cnt; i += G) a.Cval[o + r0 + i] = (V)vals[swz64(i)];
                __syncthreads();
                w0r = r1;
            }
        }
        o += total;
    }
}

}  // namespace spg
