// Enumeration of the products ("terms") a_ik * b_kj of one output column j
// of C = A~ * B_i (Gustavson's column-by-column formula): for every stored
// b_kj, the stored entries of A~'s column map[k].  Used by the symbolic,
// numeric and batched kernels.
#pragma once

#include "common.hpp"

namespace spg {

// Entries of B(:,j) whose column of A~ holds more than kShortLen entries
// are "long": a team of lanes walks them with consecutive (coalesced)
// positions.  Shorter ones are walked by the thread that loaded the entry.
constexpr int kShortLen = 32;

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
    int lnext[CH];         // offset (from lstart) of the entry's next unclaimed piece
    int nlong;
    int tmp[kMaxGroupWaves + 2];  // scratch for a group scan of the caller
};

// The same plus what a windowed walk needs to resume every entry.
template <int CH, typename V>
struct TermStageCursor : TermStage<CH, V> {
    int llen[CH];  // length of the entry's column of A~
    int lq[CH];    // entry index relative to the column's first entry
    int lcut[CH];  // offset from lstart of the first term at or past the window
};

// Long entries of a chunk are dealt to the group's waves round-robin, each
// walked in pieces of U*64 consecutive terms claimed from the entry's lnext
// counter.  A wave that has finished its own entries claims pieces of the
// others, so a few very long columns of A~ (hubs of a power-law matrix) do
// not leave the other waves idle.  Stealing is tried when the chunk has at
// most kStealFactor long entries per wave (more entries balance by
// themselves).
#ifndef SPG_STEAL_FACTOR
#define SPG_STEAL_FACTOR 4
#endif
constexpr int kStealFactor = SPG_STEAL_FACTOR;

// Claims the next piece of long entry li for the calling wave: the offset of
// its first term from lstart (wave-uniform).
template <int CH, typename V>
__device__ __forceinline__ int claim_piece(TermStage<CH, V> *st, int li, int piece) {
    int off = 0;
    if (lane_id() == 0) off = atomicAdd(&st->lnext[li], piece);
    return __shfl(off, 0);
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
template <int G, typename V, int U = kUnroll, int CH = G, typename LD, typename AP>
__device__ __forceinline__ void for_each_term(int64_t q0, int64_t q1, TermRange tr,
                                              const V *__restrict__ Bvals,
                                              TermStage<CH, V> *st, int gt, LD &&ld, AP &&ap) {
    static_assert(CH <= G && G <= kMaxGroupWaves * kWave, "chunk and group sizes");
    using Item = decltype(ld((int64_t)0));
    constexpr int TEAM = G < kWave ? G : kWave;
    constexpr int NTEAM = G / TEAM;
    const int team = gt / TEAM, tl = gt % TEAM;
    for (int64_t qb = q0; qb < q1; qb += CH) {
        if (gt == 0) st->nlong = 0;
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
        } else {
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
        if constexpr (G > kWave) {
            constexpr int PS = U * kWave;
            if (gt < nl) st->lnext[gt] = 0;
            group_sync<G>();
            auto walk = [&](int li) {
                const long long s0 = st->lstart[li];
                const int len = (int)(st->lend[li] - s0);
                const V b = st->lbv[li];
                while (true) {
                    const int off = claim_piece<CH, V>(st, li, PS);
                    if (off >= len) break;
                    const long long s = s0 + off, t = s0 + min(len, off + PS);
                    Item it[U];
#pragma unroll
                    for (int u = 0; u < U; ++u)
                        if (s + u * kWave + tl < t) it[u] = ld((int64_t)(s + u * kWave + tl));
#pragma unroll
                    for (int u = 0; u < U; ++u)
                        if (s + u * kWave + tl < t) ap(it[u], b);
                }
            };
            for (int li = team; li < nl; li += NTEAM) walk(li);
            if (nl <= kStealFactor * NTEAM)
                for (int k = 1; k < nl; ++k) walk((team + k) % nl);
        } else {
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

// Visits the terms of column j whose row is below r_hi and that no earlier
// call visited: cursor[q - q0] keeps, per entry of B(:,j), how far the
// entry's column of A~ has been walked (rows ascend, so each call resumes
// where the previous one stopped).  first == true starts every cursor at 0.
// For each such term: ap(row, ldv(p), bv).  G >= 64 (long entries are
// walked by whole waves).
template <int G, typename V, int U = kUnroll, int CH = G, typename LDV, typename AP>
__device__ __forceinline__ void for_each_term_below(int64_t q0, int64_t q1, int32_t r_hi,
                                                    bool first, TermRange tr,
                                                    const V *__restrict__ Bvals,
                                                    const int32_t *__restrict__ At_rowidx,
                                                    int32_t *__restrict__ cursor,
                                                    TermStageCursor<CH, V> *st, int gt,
                                                    LDV &&ldv,
                                                    AP &&ap) {
    static_assert(G >= kWave, "teams are whole waves");
    constexpr int NTEAM = G / kWave;
    const int team = gt / kWave, tl = lane_id();
    static_assert(CH <= G && G <= kMaxGroupWaves * kWave, "chunk and group sizes");
    for (int64_t qb = q0; qb < q1; qb += CH) {
        if (gt == 0) st->nlong = 0;
        group_sync<G>();
        const int64_t q = qb + gt;
        if (gt < CH && q < q1) {
            const int len = tr.len[q];
            if (len > 0) {
                const long long c0 = tr.start[q];
                const long long end = c0 + len;
                const int rel = first ? 0 : cursor[q - q0];
                const V bv = Bvals[q];
                if (end - c0 > kShortLen) {
                    const int slot = atomicAdd(&st->nlong, 1);
                    st->lstart[slot] = c0 + rel;
                    st->lend[slot] = end;
                    st->lbv[slot] = bv;
                    st->llen[slot] = (int)(end - c0);
                    st->lq[slot] = (int)(q - q0);
                } else {
                    long long pos = c0 + rel;
                    while (pos < end) {
                        const int32_t r = At_rowidx[pos];
                        if (r >= r_hi) break;
                        ap(r, ldv((int64_t)pos), bv);
                        ++pos;
                    }
                    cursor[q - q0] = (int32_t)(pos - c0);
                }
            }
        }
        group_sync<G>();
        const int nl = st->nlong;
        constexpr int PS = U * kWave;
        if (gt < nl) {
            st->lnext[gt] = 0;
            st->lcut[gt] = (int)(st->lend[gt] - st->lstart[gt]);
        }
        group_sync<G>();
        auto walk = [&](int li) {
            const long long s0 = st->lstart[li];
            const int len = (int)(st->lend[li] - s0);
            const V b = st->lbv[li];
            while (true) {
                const int off = claim_piece<CH, V>(st, li, PS);
                // rows ascend inside an entry: once a piece has met r_hi, the
                // entry's later pieces hold nothing for this window
                if (off >= st->lcut[li]) break;
                const long long s = s0 + off, t = s0 + min(len, off + PS);
                int32_t r[U];
                V v[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const long long e = s + u * kWave + tl;
                    r[u] = e < t ? At_rowidx[e] : kNoRow;
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const long long e = s + u * kWave + tl;
                    if (r[u] < r_hi) v[u] = ldv((int64_t)e);
                }
                int cnt = 0;
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    if (r[u] < r_hi) ap(r[u], v[u], b);
                    // the positions below r_hi are a prefix of the piece
                    cnt += __popcll(__ballot(r[u] < r_hi));
                }
                if (s + cnt < t) {
                    if (tl == 0) atomicMin(&st->lcut[li], off + cnt);
                    break;
                }
            }
        };
        for (int li = team; li < nl; li += NTEAM) walk(li);
        if (nl <= kStealFactor * NTEAM)
            for (int k = 1; k < nl; ++k) walk((team + k) % nl);
        group_sync<G>();
        if (gt < nl)
            cursor[st->lq[gt]] =
                (int32_t)(st->lstart[gt] + st->lcut[gt] - (st->lend[gt] - st->llen[gt]));
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
        const int S = __shfl(incl, kWave - 1);
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
                        const int i = lane * E + r;
                        const bool up = (i & kk) == 0;
                        const int a = key[r], b = key[r ^ jj];
                        if ((a > b) == up) {
                            key[r] = b;
                            key[r ^ jj] = a;
                            if constexpr (kVals) {
                                const V t = val[r];
                                val[r] = val[r ^ jj];
                                val[r ^ jj] = t;
                            }
                        }
                    }
                }
            } else {
                const int ld = jj / E;
#pragma unroll
                for (int r = 0; r < E; ++r) {
                    const int i = lane * E + r;
                    const int ok = __shfl_xor(key[r], ld);
                    V ov = V(0);
                    if constexpr (kVals) ov = __shfl_xor(val[r], ld);
                    const bool up = (i & kk) == 0;
                    const bool lower = (i & jj) == 0;
                    const bool take = (lower == up) ? (ok < key[r]) : (ok > key[r]);
                    if (take) {
                        key[r] = ok;
                        if constexpr (kVals) val[r] = ov;
                    }
                }
            }
        }
    }
}


}  // namespace spg
