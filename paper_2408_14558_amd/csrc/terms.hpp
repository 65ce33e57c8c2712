// Enumeration of the products ("terms") a_ik * b_kj of one output column j
// of C = A~ * B_i (Gustavson's column-by-column formula): for every stored
// b_kj, the stored entries of A~'s column map[k].  Used by the symbolic,
// numeric and batched kernels.
#pragma once

#include "common.hpp"

namespace spg {

// Entries of B(:,j) whose column of A~ holds more than kShortLen entries
// are "long": a team of lanes walks them with consecutive (coalesced)
// positions.  Shorter ones are walked by the thread that loaded the entry,
// or (groups of more than one wave) as one flat list of terms over the
// group.  Measured on the R-MAT scale-18 product: 64 beat 16, 32 and 128.
constexpr int kShortLen = 64;

// Row id above every real row (row ids are below 2^31 - 1).
constexpr int kNoRow = 0x7fffffff;

// Most waves one group holds (1024 threads).
constexpr int kMaxGroupWaves = 16;

// LDS staging for one chunk of CH entries of B(:,j).
template <int CH, typename V>
struct TermStage {
    long long lstart[CH];  // long entries: first position in A~ still to visit
    long long lend[CH];    // one past the entry's last position
    V lbv[CH];             // b_kj
    int lnext[CH];         // long entries: offset (from lstart) of the next unclaimed
                           // piece; short ones: offset of the first term in the flat list
    int nlong;
    int qnext;             // next long entry to start
    int tmp[kMaxGroupWaves + 2];  // scratch for a group scan of the caller
};

constexpr int next_pow2_const(int x) {
    int p = 1;
    while (p < x) p <<= 1;
    return p;
}

// Long entries of a chunk (stage slots [0, nl)) are handed to the group's
// waves one at a time from a shared counter (qnext), and each is walked in
// pieces of U*64 consecutive terms claimed from its own counter (lnext).  A
// wave that finds no entry left to start helps on the entries that still
// have unclaimed pieces, so hub columns of A~ (power-law inputs) are spread
// over the group instead of holding one wave while the others wait.

// The next long entry to start for the calling wave (wave-uniform; the
// whole wave calls, so lane 0 is its first active lane and readfirstlane
// broadcasts the claim without an LDS round trip).
template <int CH, typename V>
__device__ __forceinline__ int claim_entry(TermStage<CH, V> *st) {
    int e = 0;
    if (lane_id() == 0) e = atomicAdd(&st->qnext, 1);
    return __builtin_amdgcn_readfirstlane(e);
}

// The offset (from lstart) of the next unclaimed piece of entry e.
template <int CH, typename V>
__device__ __forceinline__ int claim_piece(TermStage<CH, V> *st, int e, int piece) {
    int off = 0;
    if (lane_id() == 0) off = atomicAdd(&st->lnext[e], piece);
    return __builtin_amdgcn_readfirstlane(off);
}

// A long entry with unclaimed pieces before lim(e), or -1 (one LDS read per
// 64 entries); the search starts at entry `from` (a different one for every
// wave).
template <typename LIM>
__device__ __forceinline__ int entry_with_work(const int *lnext, int nl, int from, LIM &&lim) {
    const int first = nl > 0 ? from % nl : 0;
    for (int b = 0; b < nl; b += kWave) {
        int e = first + b + lane_id();
        if (e >= nl) e -= nl;  // b + lane < nl and first < nl, so e < 2 nl
        const bool left = b + lane_id() < nl && lnext[e] < lim(e);
        const uint64_t m = __ballot(left);
        if (m)
            return __builtin_amdgcn_readlane(
                e, __builtin_amdgcn_readfirstlane(__ffsll((unsigned long long)m) - 1));
    }
    return -1;
}

// Short entries of a chunk are walked as one flat list of terms spread over
// the whole group (G > 64): the entries sit in the stage's slots
// [CH - ns, CH) in entry order, lnext[s] holding the offset of the slot's
// first term in the list.  Returns the slot holding term t (0 <= t < the
// list's length): a fixed-depth search, so the U searches of a thread
// overlap.
template <int CH, typename V>
__device__ __forceinline__ int short_slot(const TermStage<CH, V> *st, int ns, int t) {
    constexpr int kTop = next_pow2_const(CH) >> 1;  // evaluated at compile time
    int lo = CH - ns;
#pragma unroll
    for (int step = kTop; step > 0; step >>= 1) {
        const int c = min(lo + step, CH - 1);  // the read stays in bounds, no branch
        lo = (lo + step < CH && st->lnext[c] <= t) ? lo + step : lo;
    }
    return lo;
}

// Terms of the flat short list taken per thread per round: a chunk holds at
// most CH * kShortLen of them, spread over G threads, so few rounds suffice.
template <int G>
constexpr int short_unroll() { return G >= 512 ? 2 : 4; }

// Scan value of one entry for the flat short list: (1 << kShortShift) | its
// length (a chunk holds at most 1024 entries of at most kShortLen terms, so
// the length sum stays at or below 2^16, below 2^kShortShift, and the count
// below 2^11: the packed sum stays below 2^28).
constexpr int kShortShift = 17;
constexpr int kShortMask = (1 << kShortShift) - 1;
static_assert(kMaxGroupWaves * kWave * kShortLen <= kShortMask, "flat short list length");
__device__ __forceinline__ int short_code(int len) {
    return len > 0 ? ((1 << kShortShift) | len) : 0;
}

// A term's row id and a_ik.
template <typename V>
struct RowVal {
    int32_t r;
    V v;
};

// Loads in flight per thread while walking terms: a walker first issues
// kUnroll independent loads (ld), then applies them (ap).
constexpr int kUnroll = 4;

// Visits every term of column j with the G threads of a group (gt = thread
// index inside the group).  For each term at position p of A~ (with b_kj =
// bv) it calls ap(ld(p), bv); ld does the global loads, ap the LDS work, so
// kUnroll loads per thread are in flight before the first use.  All G
// threads must call it (it synchronises the group).
template <int G, typename V, int U = kUnroll, int CH = G, bool kFlat = true, typename LD,
          typename AP>
__device__ __forceinline__ void for_each_term(int64_t q0, int64_t q1, TermRange tr,
                                              const V *__restrict__ Bvals,
                                              TermStage<CH, V> *st, int gt, LD &&ld, AP &&ap) {
    static_assert(CH <= G && G <= kMaxGroupWaves * kWave, "chunk and group sizes");
    using Item = decltype(ld((int64_t)0));
    constexpr int TEAM = G < kWave ? G : kWave;
    constexpr int NTEAM = G / TEAM;
    const int team = gt / TEAM, tl = gt % TEAM;
    for (int64_t qb = q0; qb < q1; qb += CH) {
        if (gt == 0) {
            st->nlong = 0;
            st->qnext = 0;
        }
        group_sync<G>();
        const int64_t q = qb + gt;
        long long start = 0;
        int len = 0;
        V bv = V(0);
        if (gt < CH && q < q1) {
            start = tr.start[q];
            len = tr.len[q];
            if (Bvals) bv = Bvals[q];
        }
        if (len > kShortLen) {
            const int slot = atomicAdd(&st->nlong, 1);
            st->lstart[slot] = start;
            st->lend[slot] = start + len;
            st->lbv[slot] = bv;
            st->lnext[slot] = 0;
        }
        if constexpr (G > kWave) {
            // short entries: one flat list of terms over the whole group, or
            // (kFlat false) each walked by the thread that loaded it
            int ns = 0, nt = 0;
            if constexpr (kFlat) {
                int tot;
                const int sp = group_excl_scan<G>(short_code(len <= kShortLen ? len : 0),
                                                  st->tmp, &tot);
                ns = tot >> kShortShift;
                nt = tot & kShortMask;
                if (len > 0 && len <= kShortLen) {
                    const int slot = CH - ns + (sp >> kShortShift);
                    st->lstart[slot] = start;
                    st->lbv[slot] = bv;
                    st->lnext[slot] = sp & kShortMask;
                }
            } else if (len <= kShortLen) {
                for (int e = 0; e < len; e += kUnroll) {
                    Item it[kUnroll];
#pragma unroll
                    for (int u = 0; u < kUnroll; ++u)
                        if (e + u < len) it[u] = ld((int64_t)(start + e + u));
#pragma unroll
                    for (int u = 0; u < kUnroll; ++u)
                        if (e + u < len) ap(it[u], bv);
                }
            }
            group_sync<G>();
            const int nl = st->nlong;
            constexpr int SU = short_unroll<G>();
            for (int t0 = 0; t0 < nt; t0 += SU * G) {
                Item it[SU];
                V b[SU];
                // threads past the list's end load its last term again (in
                // bounds, no divergent branch) and do not apply it
#pragma unroll
                for (int u = 0; u < SU; ++u) {
                    const int t = min(t0 + u * G + gt, nt - 1);
                    const int sl = short_slot<CH, V>(st, ns, t);
                    it[u] = ld((int64_t)(st->lstart[sl] + (t - st->lnext[sl])));
                    b[u] = st->lbv[sl];
                }
#pragma unroll
                for (int u = 0; u < SU; ++u)
                    if (t0 + u * G + gt < nt) ap(it[u], b[u]);
            }
            constexpr int PS = U * kWave;
            // loads without branches (lanes past the entry's end load its
            // last term again and do not apply it), and the next piece's
            // loads in flight while the current piece is applied
            auto load = [&](long long s0, int len, int off, Item (&it)[U]) {
                // the entry's first position as a scalar and 32-bit lane
                // offsets: less address arithmetic per load
                const long long sb = (long long)(
                    ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(s0 >> 32)) << 32) |
                    (uint32_t)__builtin_amdgcn_readfirstlane((int)s0));
#pragma unroll
                for (int u = 0; u < U; ++u)
                    it[u] = ld((int64_t)(sb + (uint32_t)min(off + u * kWave + tl, len - 1)));
            };
            auto walk = [&](int e) {
                const long long s0 = st->lstart[e];
                const int len = (int)(st->lend[e] - s0);
                const V b = st->lbv[e];
                int off = claim_piece<CH, V>(st, e, PS);
                if (off >= len) return;
                Item it[U];
                load(s0, len, off, it);
                while (true) {
                    const int nxt = claim_piece<CH, V>(st, e, PS);
                    Item it2[U];
                    load(s0, len, min(nxt, len - 1), it2);
#pragma unroll
                    for (int u = 0; u < U; ++u)
                        if (off + u * kWave + tl < len) ap(it[u], b);
                    if (nxt >= len) break;
                    off = nxt;
#pragma unroll
                    for (int u = 0; u < U; ++u) it[u] = it2[u];
                }
            };
            for (int e = claim_entry<CH, V>(st); e < nl; e = claim_entry<CH, V>(st)) walk(e);
            auto lim = [&](int e) { return (int)(st->lend[e] - st->lstart[e]); };
            for (int e = entry_with_work(st->lnext, nl, team, lim); e >= 0;
                 e = entry_with_work(st->lnext, nl, team, lim))
                walk(e);
        } else {
            if (len <= kShortLen) {
                for (int e = 0; e < len; e += kUnroll) {
                    Item it[kUnroll];
#pragma unroll
                    for (int u = 0; u < kUnroll; ++u)
                        if (e + u < len) it[u] = ld((int64_t)(start + e + u));
#pragma unroll
                    for (int u = 0; u < kUnroll; ++u)
                        if (e + u < len) ap(it[u], bv);
                }
            }
            group_sync<G>();
            const int nl = st->nlong;
            for (int li = team; li < nl; li += NTEAM) {
                const long long s = st->lstart[li], t = st->lend[li];
                const V b = st->lbv[li];
                for (long long e = s + tl; e < t; e += U * TEAM) {
                    Item it[U];
#pragma unroll
                    for (int u = 0; u < U; ++u)
                        if (e + u * TEAM < t) it[u] = ld((int64_t)(e + u * TEAM));
#pragma unroll
                    for (int u = 0; u < U; ++u)
                        if (e + u * TEAM < t) ap(it[u], b);
                }
            }
        }
        group_sync<G>();
    }
}

// The terms of a column with at most 64*E of them, spread over one wave:
// slot r of lane l receives term r*64 + l (p = its position in A~, bv =
// b_kj); slots past the last term get p = -1.  All 64 lanes must call it.
template <int E, typename V>
__device__ __forceinline__ void wave_terms(int64_t q0, int64_t q1, TermRange tr,
                                           const V *__restrict__ Bvals,
                                           int64_t (&p)[E], V (&bv)[E]) {
    const int lane = lane_id();
#pragma unroll
    for (int r = 0; r < E; ++r) {
        p[r] = -1;
        bv[r] = V(0);
    }
    int base = 0;
    for (int64_t qb = q0; qb < q1; qb += kWave) {
        const int64_t q = qb + lane;
        int len = 0;
        long long start = 0;
        V b = V(0);
        if (q < q1) {
            start = tr.start[q];
            len = tr.len[q];
            if (Bvals) b = Bvals[q];
        }
        const int incl = wave_incl_scan(len);
        const int S = wave_last(incl);
#pragma unroll
        for (int r = 0; r < E; ++r) {
            const int s = r * kWave + lane - base;
            // first lane e with incl[e] > s
            int lo = 0, hi = kWave - 1;
#pragma unroll
            for (int it = 0; it < 6; ++it) {
                const int mid = (lo + hi) >> 1;
                const int v = __shfl(incl, mid);
                if (v > s) hi = mid; else lo = mid + 1;
            }
            const int excl_e = __shfl(incl - len, lo);
            const long long start_e = __shfl(start, lo);
            const V b_e = __shfl(b, lo);
            if (s >= 0 && s < S) {
                p[r] = start_e + (s - excl_e);
                bv[r] = b_e;
            }
        }
        base += S;
    }
}

// Ascending bitonic sort of 64*E (key, value) pairs held by one wave; lane l
// holds elements l*E .. l*E+E-1 in slots 0..E-1.  Pairs at distance below E
// sit in one lane; the others are exchanged across lanes.
template <int E, bool kVals, typename V>
__device__ __forceinline__ void wave_sort(int (&key)[E], V (&val)[E]) {
    const int lane = lane_id();
#pragma unroll
    for (int kk = 2; kk <= kWave * E; kk <<= 1) {
#pragma unroll
        for (int jj = kk >> 1; jj > 0; jj >>= 1) {
            if (jj < E) {
#pragma unroll
                for (int r = 0; r < E; ++r) {
                    if ((r & jj) == 0) {
                        // ascending pair unless bit kk of the element index is set
                        const bool up = kk < E ? (r & kk) == 0 : ((lane * E) & kk) == 0;
                        const int a = key[r], b = key[r ^ jj];
                        const int lo = min(a, b), hi = max(a, b);
                        if constexpr (kVals) {
                            const bool sw = (a > b) == up;
                            const V va = val[r], vb = val[r ^ jj];
                            val[r] = sw ? vb : va;
                            val[r ^ jj] = sw ? va : vb;
                        }
                        key[r] = up ? lo : hi;
                        key[r ^ jj] = up ? hi : lo;
                    }
                }
            } else {
                // partner in lane ^ (jj / E); both bits depend on the lane
                // alone, so one direction serves the lane's E elements
                const int ld = jj / E;
                const bool up = ((lane * E) & kk) == 0;
                const bool lower = ((lane * E) & jj) == 0;
                const bool keep_min = lower == up;
#pragma unroll
                for (int r = 0; r < E; ++r) {
                    const int ok = lane_xor(key[r], ld);
                    if constexpr (kVals) {
                        const V ov = lane_xor(val[r], ld);
                        const bool take = keep_min ? (ok < key[r]) : (ok > key[r]);
                        val[r] = take ? ov : val[r];
                    }
                    key[r] = keep_min ? min(key[r], ok) : max(key[r], ok);
                }
            }
        }
    }
}


// Visits the terms of one window of a dense column: rows [rlo, rhi) of C,
// inside row blocks [b0, b1) of the split table (full: the whole column).
// For every entry q of B(:,j), a long column of A~ (more than kShortLen
// entries) is cut to its part in the window's blocks by the split table
// (no cut when full); a short one is taken whole.  Every term whose row lies
// in [rlo, rhi) gets ap(row, a_ik, b_kj), each exactly once: the blocks
// cover the window's rows, and rows outside it (the rest of a short column,
// the part of a block outside a window that splits it) are skipped.
// Segments of at most kShortLen terms form one flat list over the group;
// longer ones are walked by whole waves in pieces of U*64 claimed from a
// per-entry counter, with row ids and values loaded together.
// kVals = false: row ids only (values read as 0, Bvals and At_vals unused).
// What one thread of the group holds of its entry of B(:,j) across the
// windows of a column: the entry's whole A~ column (start, length), b_kj and
// the row id that indexes the split table.  A column with at most CH entries
// is staged once per column instead of once per window.
template <typename V>
struct EntryRegs {
    long long start = 0;
    int len = 0;
    int brow = 0;
    V bv = V(0);
};

// Loads thread gt's entry (q0 + gt) of a column of at most CH entries.
template <int CH, typename V, bool kVals = true>
__device__ __forceinline__ EntryRegs<V> load_entry(int64_t q0, int64_t q1, TermRange tr,
                                                   const int32_t *__restrict__ Browidx,
                                                   const V *__restrict__ Bvals, int gt) {
    EntryRegs<V> e;
    const int64_t q = q0 + gt;
    if (gt < CH && q < q1) {
        e.len = tr.len[q];
        e.start = tr.start[q];
        e.brow = Browidx[q];
        if (kVals) e.bv = Bvals[q];
    }
    return e;
}

// cached: the column has at most CH entries and every thread passes its
// entry in `er` (load_entry); otherwise the entries are loaded per chunk.
template <int G, typename V, int U, int CH, typename AP, bool kVals = true>
__device__ __forceinline__ void for_each_window_term(
    int64_t q0, int64_t q1, bool full, int b0, int b1, int nblk, int32_t rlo, int32_t rhi,
    TermRange tr, const int32_t *__restrict__ Browidx, const int32_t *__restrict__ split,
    const V *__restrict__ Bvals, const int32_t *__restrict__ At_rowidx,
    const V *__restrict__ At_vals, TermStage<CH, V> *st, int gt, AP &&ap, bool cached = false,
    const EntryRegs<V> &er = EntryRegs<V>()) {
    static_assert(G > kWave && CH <= G && G <= kMaxGroupWaves * kWave, "group and chunk sizes");
    const int team = gt / kWave, tl = lane_id();
    auto inside = [&](int32_t r) { return r >= rlo && r < rhi; };
    // applies the U terms of one lane of a piece at offset `off` of an entry
    // of `elen` terms: ap gets the whole batch, so it can issue its LDS reads
    // for all of them before it waits
    auto ap_batch = [&](int off, int elen, const int32_t (&r)[U], const V (&av)[U], V b) {
        bool ok[U];
#pragma unroll
        for (int u = 0; u < U; ++u) ok[u] = off + u * kWave + tl < elen && inside(r[u]);
        ap(r, av, b, ok);
    };
    for (int64_t qb = q0; qb < q1; qb += CH) {
        if (gt == 0) {
            st->nlong = 0;
            st->qnext = 0;
        }
        group_sync<G>();
        const int64_t q = qb + gt;
        long long start = 0;
        int len = 0;
        V bv = V(0);
        if (gt < CH && q < q1) {
            len = cached ? er.len : tr.len[q];
            if (len > 0) {
                start = cached ? er.start : tr.start[q];
                if (kVals) bv = cached ? er.bv : Bvals[q];
                if (!full && len > kShortLen) {
                    const int32_t *sp =
                        split + (int64_t)(cached ? er.brow : Browidx[q]) * (nblk + 1);
                    const int lo = b0 > 0 ? sp[b0] : 0;
                    const int hi = b1 < nblk ? sp[b1] : len;
                    start += lo;
                    len = hi - lo;
                }
            }
        }
        if (len > kShortLen) {
            const int slot = atomicAdd(&st->nlong, 1);
            st->lstart[slot] = start;
            st->lend[slot] = start + len;
            st->lbv[slot] = bv;
            st->lnext[slot] = 0;
        }
        int tot;
        const int sp = group_excl_scan<G>(short_code(len <= kShortLen ? len : 0), st->tmp, &tot);
        const int ns = tot >> kShortShift, nt = tot & kShortMask;
        if (len > 0 && len <= kShortLen) {
            const int slot = CH - ns + (sp >> kShortShift);
            st->lstart[slot] = start;
            st->lbv[slot] = bv;
            st->lnext[slot] = sp & kShortMask;
        }
        group_sync<G>();
        const int nl = st->nlong;
        constexpr int SU = short_unroll<G>();
        for (int t0 = 0; t0 < nt; t0 += SU * G) {
            int32_t r[SU];
            V av[SU], b[SU];
            // threads past the list's end load its last term again (in
            // bounds, no divergent branch) and do not apply it
#pragma unroll
            for (int u = 0; u < SU; ++u) {
                const int t = min(t0 + u * G + gt, nt - 1);
                const int sl = short_slot<CH, V>(st, ns, t);
                const long long pos = st->lstart[sl] + (t - st->lnext[sl]);
                r[u] = At_rowidx[pos];
                av[u] = kVals ? At_vals[pos] : V(0);
                b[u] = st->lbv[sl];
            }
            bool ok[SU];
#pragma unroll
            for (int u = 0; u < SU; ++u) ok[u] = t0 + u * G + gt < nt && inside(r[u]);
            ap(r, av, b, ok);
        }
        constexpr int PS = U * kWave;
        // a piece's row ids and values, loaded without branches (lanes past
        // the entry's end load its last term again and do not apply it)
        auto load = [&](long long s0, int elen, int off, int32_t (&r)[U], V (&av)[U]) {
            // the entry's first term as a scalar base and 32-bit offsets per
            // lane: one address operation per load (the walk is bound by
            // vector instruction issue)
            const long long sb =
                (long long)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(s0 >> 32))
                             << 32) |
                            (uint32_t)__builtin_amdgcn_readfirstlane((int)s0));
            const int32_t *rb = At_rowidx + sb;
            const V *vb = kVals ? At_vals + sb : nullptr;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint32_t at = (uint32_t)min(off + u * kWave + tl, elen - 1);
                r[u] = rb[at];
                av[u] = kVals ? vb[at] : V(0);
            }
        };
        // the next piece is claimed and its loads are in flight while the
        // current one is applied
        auto walk = [&](int e) {
            const long long s0 = st->lstart[e];
            const int elen = (int)(st->lend[e] - s0);
            const V b = st->lbv[e];
            int off = claim_piece<CH, V>(st, e, PS);
            if (off >= elen) return;
            int32_t r[U];
            V av[U];
            load(s0, elen, off, r, av);
            while (true) {
                const int nxt = claim_piece<CH, V>(st, e, PS);
                int32_t r2[U];
                V av2[U];
                load(s0, elen, min(nxt, elen - 1), r2, av2);
                ap_batch(off, elen, r, av, b);
                if (nxt >= elen) break;
                off = nxt;
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    r[u] = r2[u];
                    av[u] = av2[u];
                }
            }
        };
        for (int e = claim_entry<CH, V>(st); e < nl; e = claim_entry<CH, V>(st)) walk(e);
        auto lim = [&](int e) { return (int)(st->lend[e] - st->lstart[e]); };
        for (int e = entry_with_work(st->lnext, nl, team, lim); e >= 0;
             e = entry_with_work(st->lnext, nl, team, lim))
            walk(e);
        group_sync<G>();
    }
}

}  // namespace spg
