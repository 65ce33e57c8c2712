// Symbolic phase of C_i = A~ * B_i: sparse flops per output column
// (Sec. III-B), binning of columns by flops, the number of distinct rows of
// each output column (Sec. III-A, column-by-column formula; a row counts as
// soon as one product reaches it), and the exclusive scan giving C_i's
// column pointers.  The scan also bins the columns for the numeric phase.
#include "gather.hpp"
#include "terms.hpp"

namespace spg {

__device__ __forceinline__ int sym_bin_of(long long f, const Thresholds &th) {
    if (f == 0) return kBinEmpty;
    if (f <= th.tiny_max_flop) return kBinTiny;
#pragma unroll
    for (int h = 0; h < 4; ++h)
        if (th.sym_hash_max[h] > 0 && f <= th.sym_hash_max[h]) return kBinH0 + h;
    return kBinDense;
}

__device__ __forceinline__ int num_bin_of(long long f, long long nnz, const Thresholds &th) {
    if (nnz == 0) return kBinEmpty;
    if (f <= th.tiny_max_flop) return kBinTiny;
#pragma unroll
    for (int h = 0; h < 4; ++h)
        if (th.num_hash_max[h] > 0 && nnz <= th.num_hash_max[h]) return kBinH0 + h;
    return kBinDense;
}

// The calling lane's slot in bin b's workgroup-local list (LDS counters
// s_cnt; b == kBinEmpty: none, 0).  The lanes of a wave that share a bin
// take consecutive slots from one LDS atomic: lane by lane, thousands of
// columns of one bin serialise on its counter (the one-workgroup scan of the
// 4096 tiny columns of one ER 65536 partition (16 per column) spent most of
// its 9 us there).  Every lane of the wave
// calls.
__device__ __forceinline__ int wave_bin_slot(int *s_cnt, int b) {
    int pos = 0;
#pragma unroll
    for (int x = kBinEmpty + 1; x < kNumBins; ++x) {
        const uint64_t m = __ballot(b == x);
        if (m) {  // wave-uniform
            const int leader = __ffsll((unsigned long long)m) - 1;
            int base = 0;
            if (lane_id() == leader) base = atomicAdd(&s_cnt[x], __popcll(m));
            base = __shfl(base, leader);
            if (b == x) pos = base + __popcll(m & ((1ull << lane_id()) - 1ull));
        }
    }
    return pos;
}

// Appends the workgroup's columns to the per-bin lists: one global atomic
// per non-empty bin and workgroup reserves a contiguous range.
__device__ __forceinline__ void append_to_bins(int nloc, const int *s_bin, const int *s_lpos,
                                               int *s_cnt, int *s_base, int64_t j0,
                                               LineInt *__restrict__ gcount,
                                               int32_t *__restrict__ list, int64_t n) {
    // s_cnt already holds the per-bin counts of this workgroup
    if (threadIdx.x < kNumBins) {
        const int c = s_cnt[threadIdx.x];
        s_base[threadIdx.x] = c ? atomicAdd(&gcount[threadIdx.x].v, c) : 0;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nloc; i += blockDim.x) {
        const int b = s_bin[i];
        if (b != kBinEmpty) list[(int64_t)b * n + s_base[b] + s_lpos[i]] = (int32_t)(j0 + i);
    }
}

// Sparse flops of every column of B_i and its symbolic bin, and the term
// range of every entry of B_i.  Column tiles: S lanes walk one column (S
// picked from the average column length).  A column with more than 16*S
// entries (long) is left to the chunk workgroups instead: they split B_i's
// entries into chunks of kLongChunk and walk the long columns' entries in
// their chunk, so a hub column of 10^4 entries is walked by several
// workgroups at once; the chunk that completes a long column bins it.
constexpr int kFlopThreads = 256;
constexpr int64_t kLongChunk = 8192;

struct FlopArgs {
    int64_t n, nnzB;
    const int64_t *Bcolptr;
    const int32_t *Browidx;
    const int64_t *col_start;  // place in A~ of every column of A (row of B_i)
    const int32_t *col_len;
    Thresholds th;
    int64_t *tstart;
    int32_t *tlen;
    int32_t *col_slot;
    int64_t *flop;     // zero on entry (long columns add into it)
    int32_t *arrive;   // zero on entry: chunks done per long column
    int32_t *sym_bin;
    int32_t *sym_list;
    uint64_t *status;  // the colptr scan's tile states, cleared here
    int64_t nstatus;
    DevCounters *ctr;
};

// A column tile: `rounds` groups of kFlopThreads / S columns, one after
// the other, then one reservation per bin in the global lists for all of
// them.  Atomics on one address from every workgroup of a large launch
// serialise across the chip, so a launch over many columns gives each tile
// several rounds rather than running more tiles.
constexpr int kFlopTileCols = 1024;  // most columns one tile takes
template <int S>
__device__ __forceinline__ void flop_column_tile(int64_t blk, int64_t ngroups, int rounds,
                                                 const FlopArgs &a) {
    constexpr int COLS = kFlopThreads / S;
    static_assert(kFlopTileCols % COLS == 0, "whole rounds");
    static_assert(kNumBins <= 16 && kFlopTileCols < (1 << 24), "bin and position share an int");
    __shared__ int s_bl[kFlopTileCols];  // bin << 24 | place among the tile's columns of that bin
    __shared__ long long s_f[COLS];
    __shared__ int s_cnt[kNumBins];
    __shared__ int s_base[kNumBins];
    __shared__ long long s_flops;
    const int tid = threadIdx.x;
    {
        const int64_t stride = ngroups * kFlopThreads;
        for (int64_t s = blk * kFlopThreads + tid; s < a.nstatus; s += stride) a.status[s] = 0;
    }
    if (tid < kNumBins) s_cnt[tid] = 0;
    if (tid == 0) s_flops = 0;
    const int64_t jt = blk * (int64_t)rounds * COLS;
    const int ntile = (int)min<int64_t>((int64_t)rounds * COLS, a.n - jt);
    const int lc = tid / S, sub = tid % S;
    for (int rd = 0; rd * COLS < ntile; ++rd) {
        __syncthreads();  // s_f of the previous round is consumed
        const int64_t j0 = jt + (int64_t)rd * COLS;
        const int nloc = min(COLS, ntile - rd * COLS);
        long long acc = 0;
        bool is_long = false;
        if (lc < nloc) {
            const int64_t q0 = a.Bcolptr[j0 + lc], q1 = a.Bcolptr[j0 + lc + 1];
            is_long = q1 - q0 > 16 * S;
            if (!is_long) {
                // rounds of four entries per lane, loaded without branches
                // (past the end: the column's last entry again, discarded),
                // so a round's loads of one kind are in flight together
                constexpr int U = 4;
                for (int64_t qb = q0 + sub; qb < q1; qb += U * S) {
                    int32_t r[U];
#pragma unroll
                    for (int u = 0; u < U; ++u) r[u] = a.Browidx[min(qb + u * S, q1 - 1)];
                    long long st[U];
                    int len[U];
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        st[u] = a.col_start[r[u]];
                        len[u] = a.col_len[r[u]];
                    }
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const int64_t q = qb + u * S;
                        if (q < q1) {
                            a.tstart[q] = st[u];
                            a.tlen[q] = len[u];
                            acc += len[u];
                        }
                    }
                }
            }
        }
        acc = wave_sum<S>(acc);
        if (lc < nloc && sub == 0) s_f[lc] = is_long ? -1 : acc;
        __syncthreads();
        int b = kBinEmpty;
        long long fsum = 0;
        if (tid < nloc) {
            const int64_t j = j0 + tid;
            const long long f = s_f[tid];
            a.col_slot[j] = -1;
            if (f >= 0) {  // a long column is binned by the chunk that completes it
                a.flop[j] = f;
                b = sym_bin_of(f, a.th);
                a.sym_bin[j] = b;
                fsum = f;
            }
        }
        // one LDS atomic per wave for the flops total (not one per column)
        fsum = wave_sum(fsum);
        if (lane_id() == 0 && fsum) atomic_add_i64(&s_flops, fsum);
        const int slot = wave_bin_slot(s_cnt, b);
        if (tid < nloc) s_bl[rd * COLS + tid] = b != kBinEmpty ? (b << 24) | slot : kBinEmpty << 24;
    }
    __syncthreads();
    if (tid == 0 && s_flops) atomic_add_i64(&a.ctr->flops.v, s_flops);
    if (tid < kNumBins) {
        const int c = s_cnt[tid];
        s_base[tid] = c ? atomicAdd(&a.ctr->sym_count[tid].v, c) : 0;
    }
    __syncthreads();
    for (int i = tid; i < ntile; i += kFlopThreads) {
        const int b = s_bl[i] >> 24;
        if (b != kBinEmpty)
            a.sym_list[(int64_t)b * a.n + s_base[b] + (s_bl[i] & 0xFFFFFF)] = (int32_t)(jt + i);
    }
}

// Chunk c of B_i's entries, [c*kLongChunk, min((c+1)*kLongChunk, nnzB)):
// the term ranges of the long columns' entries in it and their flops.  The
// long columns met in the chunk (at most kLongList: each has more than 16
// entries, save the two cut by the chunk's ends) are listed with their part
// of the chunk, and the whole workgroup walks those parts as one flat range.
constexpr int kLongList = 512;
static_assert(kLongChunk / 17 + 2 <= kLongList, "the list holds every long column of a chunk");
template <int S>
__device__ __forceinline__ void flop_long_chunk(int64_t c, const FlopArgs &a) {
    constexpr int kColsPer = 4;   // columns per thread and batch
    constexpr int kLongUnroll = 8;
    __shared__ int64_t s_j;
    __shared__ int s_nl, s_more;
    __shared__ int32_t s_col[kLongList];
    __shared__ int64_t s_lo[kLongList];
    __shared__ int s_pre[kLongList + 1];  // prefix of the parts' lengths
    __shared__ long long s_part[kLongList];
    __shared__ int s_tmp[kFlopThreads / kWave + 1];
    const int tid = threadIdx.x, lane = lane_id();
    const int64_t e0 = c * kLongChunk, e1 = min(e0 + kLongChunk, a.nnzB);
    // the column holding entry e0 (the last j with Bcolptr[j] <= e0): a
    // 64-way search by one wave, Bcolptr[lo] <= e0 < Bcolptr[hi] throughout
    if (tid < kWave) {
        int64_t lo = 0, hi = a.n;
        while (hi - lo > 1) {
            const int64_t step = (hi - lo + kWave - 1) / kWave;
            const int64_t idx = lo + (int64_t)(lane + 1) * step;
            const bool le = idx < hi && a.Bcolptr[idx] <= e0;
            const int64_t nlo = lo + (int64_t)__popcll(__ballot(le)) * step;
            hi = min(hi, nlo + step);
            lo = nlo;
        }
        if (lane == 0) {
            s_j = lo;
            s_nl = 0;
        }
    }
    __syncthreads();
    // the long columns from there on, kColsPer * kFlopThreads at a time,
    // until one ends at or past e1 (every column before it starts below e1
    // and ends above e0, so it has entries in the chunk)
    constexpr int kBatch = kColsPer * kFlopThreads;
    for (int64_t jb = s_j;; jb += kBatch) {
        if (tid == 0) s_more = 0;
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kColsPer; ++i) {
            const int64_t j = jb + (int64_t)i * kFlopThreads + tid;
            if (j < a.n) {
                const int64_t q0 = a.Bcolptr[j], q1 = a.Bcolptr[j + 1];
                if (q0 < e1 && q1 - q0 > 16 * S) {
                    const int at = atomicAdd(&s_nl, 1);
                    s_col[at] = (int32_t)j;
                    s_lo[at] = max(q0, e0);
                    s_pre[at] = (int)(min(q1, e1) - max(q0, e0));
                }
                if (i == kColsPer - 1 && tid == kFlopThreads - 1 && q1 < e1) s_more = 1;
            }
        }
        __syncthreads();
        const bool more = s_more != 0;
        __syncthreads();
        if (!more || jb + kBatch >= a.n) break;
    }
    const int nl = s_nl;
    if (nl == 0) return;  // uniform
    // lengths -> exclusive prefix (two per thread), partial sums cleared
    int v0 = 0, v1 = 0;
    if (2 * tid < nl) v0 = s_pre[2 * tid];
    if (2 * tid + 1 < nl) v1 = s_pre[2 * tid + 1];
    int total;
    const int ex = group_excl_scan<kFlopThreads>(v0 + v1, s_tmp, &total);
    if (2 * tid < nl) {
        s_pre[2 * tid] = ex;
        s_part[2 * tid] = 0;
    }
    if (2 * tid + 1 < nl) {
        s_pre[2 * tid + 1] = ex + v0;
        s_part[2 * tid + 1] = 0;
    }
    for (int i = nl + tid; i < kLongList + 1; i += kFlopThreads) s_pre[i] = total;
    __syncthreads();
    // the flat walk: element e of the parts lies in part li, the last with
    // s_pre[li] <= e; loads without branches (past the end: the last element
    // again, discarded), so a round's loads of one kind are in flight together
    for (int eb = tid; eb < total; eb += kLongUnroll * kFlopThreads) {
        int li[kLongUnroll];
        int64_t q[kLongUnroll];
        int32_t r[kLongUnroll];
#pragma unroll
        for (int u = 0; u < kLongUnroll; ++u) {
            const int e = min(eb + u * kFlopThreads, total - 1);
            int o = 0;
#pragma unroll
            for (int step = kLongList / 2; step > 0; step >>= 1)
                o += s_pre[o + step] <= e ? step : 0;
            li[u] = o;
            q[u] = s_lo[o] + (e - s_pre[o]);
            r[u] = a.Browidx[q[u]];
        }
#pragma unroll
        for (int u = 0; u < kLongUnroll; ++u) {
            const long long st = a.col_start[r[u]];
            const int len = a.col_len[r[u]];
            if (eb + u * kFlopThreads < total) {
                a.tstart[q[u]] = st;
                a.tlen[q[u]] = len;
                if (len) atomic_add_i64(&s_part[li[u]], (long long)len);
            }
        }
    }
    __syncthreads();
    // one thread per listed column: its flops so far, then the arrival; the
    // chunk that completes a column bins it, the chunk's completed columns
    // taking one reservation per bin in the global lists
    __shared__ int s_cnt[kNumBins];
    __shared__ int s_base[kNumBins];
    __shared__ long long s_flops;
    if (tid < kNumBins) s_cnt[tid] = 0;
    if (tid == 0) s_flops = 0;
    __syncthreads();
    constexpr int kPer = kLongList / kFlopThreads;
    int mybin[kPer], mypos[kPer];
#pragma unroll
    for (int t = 0; t < kPer; ++t) {
        const int i = tid + t * kFlopThreads;
        mybin[t] = kBinEmpty;
        mypos[t] = 0;
        if (i >= nl) continue;
        const int64_t jc = s_col[i];
        const int64_t q0 = a.Bcolptr[jc], q1 = a.Bcolptr[jc + 1];
        if (s_part[i]) atomic_add_i64(reinterpret_cast<long long *>(a.flop + jc), s_part[i]);
        __threadfence();  // the flops before the arrival
        const int ncover = (int)((q1 - 1) / kLongChunk - q0 / kLongChunk + 1);
        if (atomicAdd(&a.arrive[jc], 1) == ncover - 1) {
            __threadfence();  // every chunk's flops are visible
            const long long f =
                __hip_atomic_load(a.flop + jc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const int b = sym_bin_of(f, a.th);
            a.sym_bin[jc] = b;
            if (f) atomic_add_i64(&s_flops, f);
            if (b != kBinEmpty) {
                mybin[t] = b;
                mypos[t] = atomicAdd(&s_cnt[b], 1);
            }
        }
    }
    __syncthreads();
    if (tid == 0 && s_flops) atomic_add_i64(&a.ctr->flops.v, s_flops);
    if (tid < kNumBins) {
        const int c = s_cnt[tid];
        s_base[tid] = c ? atomicAdd(&a.ctr->sym_count[tid].v, c) : 0;
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < kPer; ++t)
        if (mybin[t] != kBinEmpty)
            a.sym_list[(int64_t)mybin[t] * a.n + s_base[mybin[t]] + mypos[t]] =
                s_col[tid + t * kFlopThreads];
}

// One launch for two independent steps that both follow the selection: the
// flops and bins (column tiles, then chunk workgroups; first, since the host
// waits for their counts) and the gather tiles of A~.  Neither reads what
// the other writes, so their chains of dependent loads overlap instead of
// running one after the other.  With hout set, the last of the flop
// workgroups publishes the counters (else the early tiny symbolic launch
// does).
static_assert(kFlopThreads == kGatherThreads, "all tiles use the whole workgroup");
// Compiled for eight waves per SIMD (eight workgroups per CU, as many as
// their LDS allows), which caps the registers at 64 per lane.
constexpr int kFlopWaves = 8;
template <int S, typename V>
__global__ __launch_bounds__(kFlopThreads, kFlopWaves) void k_flop_bin_gather(
    FlopArgs a, int64_t ncols_tiles, int rounds, int64_t nchunks,
    PublishedCounts *__restrict__ hout,
    unsigned int *__restrict__ hready, int64_t k, const int64_t *__restrict__ Acolptr,
    const int32_t *__restrict__ Arowidx, const V *__restrict__ Avals,
    const int32_t *__restrict__ map, const int64_t *__restrict__ At_colptr,
    int32_t *__restrict__ At_rowidx, V *__restrict__ At_vals) {
    const int64_t blk = blockIdx.x, nflop = ncols_tiles + nchunks;
    if (blk < nflop) {
        if (blk < ncols_tiles) flop_column_tile<S>(blk, ncols_tiles, rounds, a);
        else flop_long_chunk<S>(blk - ncols_tiles, a);
        __shared__ int s_last;
        if (hout)  // NULL: the early tiny symbolic kernel publishes instead
            publish_when_last(&a.ctr->tickets[kTkFlopDone], (unsigned long long)nflop, a.ctr,
                              hout, hready, &s_last);
    } else {
        __shared__ GatherStage st;
        gather_tile<V, true>(blk - nflop, Acolptr, Arowidx, Avals, map, At_colptr, k, At_rowidx,
                             At_vals, st);
    }
}

// --- tiny bin: one wave per column, <= 64*8 terms in registers -------------
// perm (rows below kPackedRowLimit only, else NULL): the sort key of a term
// is (row << kSlotBits) | slot, and the sorted slots are kept (kNoSlot past
// the last term), so the numeric phase orders the column without sorting.
template <int E>
__device__ __forceinline__ int sym_wave_count(int64_t q0, int64_t q1, TermRange tr,
                                              const int32_t *__restrict__ At_rowidx,
                                              uint16_t *__restrict__ perm) {
    int64_t p[E];
    float bv[E];
    wave_terms<E, float>(q0, q1, tr, nullptr, p, bv);
    const int lane = lane_id();
    // loads without branches (an empty slot reads A~'s entry 0 and drops
    // it), so they are in flight together
    int32_t rw[E];
#pragma unroll
    for (int r = 0; r < E; ++r) rw[r] = At_rowidx[p[r] >= 0 ? p[r] : 0];
    int key[E];
#pragma unroll
    for (int r = 0; r < E; ++r) {
        key[r] = kNoRow;
        if (p[r] >= 0) key[r] = perm ? (rw[r] << kSlotBits) | (r * kWave + lane) : rw[r];
    }
    wave_sort<E, false, float>(key, bv);
    if (perm) {
#pragma unroll
        for (int r = 0; r < E; ++r) {
            perm[lane * E + r] =
                key[r] != kNoRow ? (uint16_t)(key[r] & ((1 << kSlotBits) - 1)) : kNoSlot;
            if (key[r] != kNoRow) key[r] >>= kSlotBits;
        }
    }
    const int prev_last = __shfl_up(key[E - 1], 1);
    int nh = 0;
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const int prev = r == 0 ? prev_last : key[r - 1];
        nh += key[r] != kNoRow && ((r == 0 && lane == 0) || key[r] != prev);
    }
    return wave_sum(nh);
}

// count_dev NULL: `count` columns, in `list` (NULL: every column is tiny).
// count_dev set (a launch before the host has the counts, sized for n
// columns plus one workgroup): the count is read there, and the list is used
// unless it holds every column; the extra last workgroup publishes the
// flops pass's counters (hout, hready) for the host.
template <int EMAX>
__global__ __launch_bounds__(256) void k_sym_tiny(const int32_t *__restrict__ list, int count,
                                                  const int *__restrict__ count_dev, int n,
                                                  const int64_t *__restrict__ Bcolptr,
                                                  TermRange tr,
                                                  const int32_t *__restrict__ At_rowidx,
                                                  const int64_t *__restrict__ flop,
                                                  int64_t *__restrict__ Ccount,
                                                  uint16_t *__restrict__ tiny_perm,
                                                  int32_t *__restrict__ col_slot,
                                                  const DevCounters *__restrict__ ctr,
                                                  PublishedCounts *__restrict__ hout,
                                                  unsigned int *__restrict__ hready) {
    if (hout && blockIdx.x == gridDim.x - 1) {  // the whole workgroup
        publish_counters(ctr, hout, hready);
        return;
    }
    const int w = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (count_dev) {
        count = *count_dev;
        if (count == n) list = nullptr;
    }
    if (w >= count) return;  // whole wave leaves together
    const int32_t j = list ? list[w] : w;  // NULL list: every column is tiny
    const int64_t q0 = Bcolptr[j], q1 = Bcolptr[j + 1], f = flop[j];
    uint16_t *perm = tiny_perm ? tiny_perm + (size_t)w * (EMAX * kWave) : nullptr;
    int c;
    if (f <= kWave) c = sym_wave_count<1>(q0, q1, tr, At_rowidx, perm);
    else if (f <= 2 * kWave) c = sym_wave_count<2>(q0, q1, tr, At_rowidx, perm);
    else if (EMAX == 4 || f <= 4 * kWave) c = sym_wave_count<4>(q0, q1, tr, At_rowidx, perm);
    else c = sym_wave_count<EMAX>(q0, q1, tr, At_rowidx, perm);
    if (lane_id() == 0) {
        Ccount[j] = c;
        if (perm) col_slot[j] = w;
    }
}

// --- hash bins: LDS open addressing (linear probing), count inserts -------
template <int T, int G>
struct SymHashLds {
    int keys[T];
    TermStage<G, float> st;
};

template <int T, int G>
__global__ __launch_bounds__(G < 256 ? 256 : G) void k_sym_hash(
    const int32_t *__restrict__ list, int count, const int64_t *__restrict__ Bcolptr,
    TermRange tr, const int32_t *__restrict__ At_rowidx, int64_t *__restrict__ Ccount) {
    constexpr int CPW = G < 256 ? 256 / G : 1;
    __shared__ SymHashLds<T, G> lds[CPW];
    const int grp = threadIdx.x / G, gt = threadIdx.x % G;
    const int w = blockIdx.x * CPW + grp;
    if (CPW == 1) {
        if (w >= count) return;  // uniform over the workgroup
    } else {
        if (w >= count) return;  // groups live inside one wave: no workgroup barrier used
    }
    SymHashLds<T, G> &L = lds[grp];
    const int32_t j = list[w];
    for (int s = gt; s < T; s += G) L.keys[s] = -1;
    group_sync<G>();
    int inserted = 0;
    for_each_term<G, float>(Bcolptr[j], Bcolptr[j + 1], tr, nullptr, &L.st,
                            gt, [&](int64_t p) { return At_rowidx[p]; },
                            [&](int32_t r, float) {
                                uint32_t h = hash_slot<T>(r);
                                while (true) {
                                    const int old = atomicCAS(&L.keys[h], -1, r);
                                    if (old == -1) {
                                        ++inserted;
                                        break;
                                    }
                                    if (old == r) break;
                                    h = (h + 1) & (T - 1);
                                }
                            });
    int total;
    if constexpr (G <= kWave) {
        total = wave_sum<G>(inserted);
    } else {
        (void)group_excl_scan<G>(inserted, L.st.tmp, &total);
    }
    if (gt == 0) Ccount[j] = total;
}

// --- dense bin: bitmap of all m rows in LDS ---------------------------------
// Row loads in flight per lane on long A~ columns.
#ifndef SPG_SYM_DENSE_UNROLL
#define SPG_SYM_DENSE_UNROLL 8
#endif
constexpr int kSymDenseUnroll = SPG_SYM_DENSE_UNROLL;
// Waves per SIMD the kernel is compiled for: eight, i.e. two workgroups of
// 1024 threads per CU (their LDS fits twice), which caps the registers at
// 64 per lane; the walk is bound by the latency of its row-id loads, so
// twice the resident waves hide more of it.
constexpr int kSymDenseWaves = 8;
struct SymDenseLds {
    TermStage<kDenseThreads, float> st;
    int red[kDenseThreads / kWave + 2];
};

__global__ __launch_bounds__(kDenseThreads, kSymDenseWaves) void k_sym_dense(
    const int32_t *__restrict__ list, int count, int64_t m, const int64_t *__restrict__ Bcolptr,
    TermRange tr, const int32_t *__restrict__ At_rowidx, int64_t *__restrict__ Ccount,
    uint32_t *__restrict__ keep_bits, int32_t *__restrict__ col_slot,
    const int32_t *__restrict__ Browidx, const int32_t *__restrict__ split, int32_t nblk,
    DevCounters *__restrict__ ctr) {
    extern __shared__ __align__(16) uint32_t s_bits[];
    __shared__ SymDenseLds L;
    __shared__ int s_item;
    unsigned int *queue = ctr->sym_dense_queue;
    const int gt = threadIdx.x;
    if (m <= kMaxDenseRows) {
        const int nw = (int)((m + 31) >> 5);
        for (int w = queue_take(queue, &s_item); w < count; w = queue_take(queue, &s_item)) {
            const int32_t j = list[w];
            zero_words<kDenseThreads>(s_bits, nw);
            __syncthreads();
            // short entries stay with their thread: a flat walk would give a
            // wave consecutive rows of one column of A~, whose bits share words
            for_each_term<kDenseThreads, float, kSymDenseUnroll, kDenseThreads, false>(
                Bcolptr[j], Bcolptr[j + 1], tr, nullptr, &L.st, gt,
                [&](int64_t p) { return At_rowidx[p]; },
                [&](int32_t r, float) {
                    // a row most products reach is set once, not once per
                    // product (an LDS read costs less than an atomic that
                    // collides with the wave's other lanes)
                    const uint32_t bit = 1u << (r & 31);
                    if (!(s_bits[r >> 5] & bit)) atomicOr(&s_bits[r >> 5], bit);
                });
            // the count, and the copy of the bitmap the numeric phase reuses,
            // from one read of each word
            uint32_t *dst = keep_bits ? keep_bits + (size_t)w * nw : nullptr;
            int c = 0;
            for (int i = gt; i < nw; i += kDenseThreads) {
                const uint32_t b = s_bits[i];
                c += __popc(b);
                if (dst) dst[i] = b;
            }
            int total;
            (void)group_excl_scan<kDenseThreads>(c, L.red, &total);
            if (gt == 0) {
                Ccount[j] = total;
                if (dst) col_slot[j] = w;
            }
        }
    } else {
        // m above 2^18: bands of kMaxDenseRows rows, each counted from
        // exactly its products (its blocks of the split table); no bitmap
        // is kept
        constexpr int kBandBlocks = (int)(kMaxDenseRows >> kSplitShift);
        for (int w = queue_take(queue, &s_item); w < count; w = queue_take(queue, &s_item)) {
            const int32_t j = list[w];
            int64_t count_j = 0;
            for (int64_t R0 = 0; R0 < m; R0 += kMaxDenseRows) {
                const int64_t R1 = min(m, R0 + kMaxDenseRows);
                const int nw = (int)((R1 - R0 + 31) >> 5);
                const int sb0 = (int)(R0 >> kSplitShift);
                zero_words<kDenseThreads>(s_bits, nw);
                __syncthreads();
                auto mark = [&](const auto &r, const auto &, const auto &, const auto &ok) {
                    constexpr int N = (int)(sizeof(ok) / sizeof(ok[0]));
#pragma unroll
                    for (int u = 0; u < N; ++u)
                        if (ok[u])
                            atomicOr(&s_bits[(r[u] - (int32_t)R0) >> 5], 1u << (r[u] & 31));
                };
                for_each_window_term<kDenseThreads, float, kSymDenseUnroll, kDenseThreads,
                                     decltype(mark) &, false>(
                    Bcolptr[j], Bcolptr[j + 1], false, sb0, min(nblk, sb0 + kBandBlocks), nblk,
                    (int32_t)R0, (int32_t)R1, tr, Browidx, split, (const float *)nullptr,
                    At_rowidx, (const float *)nullptr, &L.st, gt, mark);
                __syncthreads();
                int c = 0;
                for (int i = gt; i < nw; i += kDenseThreads) c += __popc(s_bits[i]);
                int total;
                (void)group_excl_scan<kDenseThreads>(c, L.red, &total);
                count_j += total;
                __syncthreads();  // the bitmap is cleared for the next band
            }
            if (gt == 0) {
                Ccount[j] = count_j;
                if (col_slot) col_slot[j] = -1;
            }
        }
    }
    queue_leave(queue);
}

// Exclusive scan of the per-column counts into C_i's column pointers (in
// place), numeric binning of every column, nnz(C_i) into the counters.
__global__ __launch_bounds__(kScanThreads) void k_colptr_scan(
    int64_t n, int64_t *__restrict__ Ccolptr, const int64_t *__restrict__ flop, Thresholds th,
    int32_t *__restrict__ num_bin, int32_t *__restrict__ num_list,
    uint64_t *__restrict__ status, int64_t ntiles, DevCounters *__restrict__ ctr,
    PublishedCounts *__restrict__ hout, unsigned int *__restrict__ hready) {
    __shared__ long long s_ticket;
    __shared__ long long s_tmp64[kScanThreads / kWave + 1];
    __shared__ long long s_prefix;
    __shared__ int s_bin[kScanTile];
    __shared__ int s_lpos[kScanTile];
    __shared__ int s_cnt[kNumBins];
    __shared__ int s_base[kNumBins];
    const long long t = take_ticket(&ctr->tickets[kTkColptr], &s_ticket);
    const int tid = threadIdx.x;
    if (tid < kNumBins) s_cnt[tid] = 0;
    __syncthreads();
    const int64_t j0 = t * kScanTile;
    const int nloc = (int)min<int64_t>(kScanTile, n - j0);
    // loads without branches (past the end: the tile's last column again)
    long long fl[kScanItems], cc[kScanItems];
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const int64_t j = j0 + min(tid * kScanItems + i, nloc - 1);
        fl[i] = flop[j];
        cc[i] = Ccolptr[j];
    }
    long long cnt[kScanItems];
    long long sum = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const int lc = tid * kScanItems + i;
        cnt[i] = 0;
        int b = kBinEmpty;
        if (lc < nloc) {
            const int64_t j = j0 + lc;
            cnt[i] = fl[i] == 0 ? 0 : cc[i];  // empty columns have no count
            b = num_bin_of(fl[i], cnt[i], th);
            if (b == kBinDense && th.dense_first_flop > 0 && fl[i] >= th.dense_first_flop)
                b = kBinDenseFirst;
            num_bin[j] = b;
            s_bin[lc] = b;
        }
        const int slot = wave_bin_slot(s_cnt, b);
        if (lc < nloc) s_lpos[lc] = slot;
        sum += cnt[i];
    }
    long long total;
    long long excl = group_excl_scan64<kScanThreads>(sum, s_tmp64, &total);
    if (tid < kWave) {
        const long long pre = chained_prefix(status, t, t == 0, total);
        if (tid == 0) s_prefix = pre;
    }
    __syncthreads();
    long long run = s_prefix + excl;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const int lc = tid * kScanItems + i;
        if (lc < nloc) Ccolptr[j0 + lc] = run;
        run += cnt[i];
    }
    if (t == ntiles - 1 && tid == 0) {
        Ccolptr[n] = s_prefix + total;
        ctr->nnzC = s_prefix + total;
    }
    append_to_bins(nloc, s_bin, s_lpos, s_cnt, s_base, j0, ctr->num_count, num_list, n);
    __shared__ int s_last;
    publish_when_last(&ctr->tickets[kTkColptrDone], gridDim.x, ctr, hout, hready, &s_last);
}

// The same scan and binning by one workgroup, for B_i with at most
// kSmallScanCols columns: no tile tickets, no look-back and no global atomics
// on the bin counters.  Chunks of kSmallScanThreads * kSmallScanItems
// columns follow one another, the running total and each bin's list length
// carried over; the counters the host needs are then published as by the
// tiled scan's last workgroup.
// nnz(C_i) + 1 goes to *hnnz (pinned host memory) the moment the total is
// known, so the host can return it before the rest is published.
constexpr int kSmallScanThreads = 1024;
constexpr int kSmallScanItems = 4;
static_assert(kSmallScanCols == 2 * kSmallScanThreads * kSmallScanItems, "two chunks at most");
__global__ __launch_bounds__(kSmallScanThreads) void k_colptr_scan_small(
    int64_t n, int64_t *__restrict__ Ccolptr, const int64_t *__restrict__ flop, Thresholds th,
    int32_t *__restrict__ num_bin, int32_t *__restrict__ num_list,
    DevCounters *__restrict__ ctr, PublishedCounts *__restrict__ hout,
    unsigned int *__restrict__ hready, unsigned long long *__restrict__ hnnz) {
    constexpr int CH = kSmallScanThreads * kSmallScanItems;
    __shared__ long long s_tmp64[kSmallScanThreads / kWave + 1];
    __shared__ int s_cnt[kNumBins];   // this chunk's columns per bin
    __shared__ int s_base[kNumBins];  // list entries of the earlier chunks per bin
    const int tid = threadIdx.x;
    if (tid < kNumBins) s_base[tid] = 0;
    long long carry = 0;
    for (int64_t j0 = 0; j0 < n; j0 += CH) {
        if (tid < kNumBins) s_cnt[tid] = 0;
        __syncthreads();
        // loads without branches (past the end: the last column again)
        long long fl[kSmallScanItems], cc[kSmallScanItems];
#pragma unroll
        for (int i = 0; i < kSmallScanItems; ++i) {
            const int64_t j = min(j0 + (int64_t)tid * kSmallScanItems + i, n - 1);
            fl[i] = flop[j];
            cc[i] = Ccolptr[j];
        }
        long long cnt[kSmallScanItems];
        int bin[kSmallScanItems], lpos[kSmallScanItems];
        long long sum = 0;
#pragma unroll
        for (int i = 0; i < kSmallScanItems; ++i) {
            const int64_t j = j0 + (int64_t)tid * kSmallScanItems + i;
            cnt[i] = 0;
            bin[i] = kBinEmpty;
            if (j < n) {
                const long long f = fl[i];
                cnt[i] = f == 0 ? 0 : cc[i];  // empty columns have no count
                int b = num_bin_of(f, cnt[i], th);
                if (b == kBinDense && th.dense_first_flop > 0 && f >= th.dense_first_flop)
                    b = kBinDenseFirst;
                num_bin[j] = b;
                bin[i] = b;
            }
            lpos[i] = wave_bin_slot(s_cnt, bin[i]);
            sum += cnt[i];
        }
        long long total;
        // ends with a barrier: s_cnt is complete
        long long run = carry + group_excl_scan64<kSmallScanThreads>(sum, s_tmp64, &total);
#pragma unroll
        for (int i = 0; i < kSmallScanItems; ++i) {
            const int64_t j = j0 + (int64_t)tid * kSmallScanItems + i;
            if (j < n) {
                Ccolptr[j] = run;
                if (bin[i] != kBinEmpty)
                    num_list[(int64_t)bin[i] * n + s_base[bin[i]] + lpos[i]] = (int32_t)j;
            }
            run += cnt[i];
        }
        carry += total;
        __syncthreads();  // every thread has read s_base
        if (tid < kNumBins) s_base[tid] += s_cnt[tid];
    }
    __syncthreads();
    if (tid == 0) {
        __hip_atomic_store(hnnz, (unsigned long long)carry + 1ull, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_SYSTEM);
        Ccolptr[n] = carry;
        ctr->nnzC = carry;
        hout->flops = ctr->flops.v;
        hout->nnzC = carry;
        hout->nnz_At = ctr->nnz_At;
    }
    if (tid < kNumBins) {
        ctr->num_count[tid].v = s_base[tid];
        hout->num_count[tid] = s_base[tid];
        hout->sym_count[tid] = ctr->sym_count[tid].v;
    }
    __syncthreads();
    // wave 0 wrote every host-side field: thread 0's system-scope release
    // store orders them before the flag
    if (tid == 0) __hip_atomic_store(hready, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Clears what one symbolic phase accumulates (the colptr scan's ticket and
// tile states, nnzC and the numeric bin counters), for a second symbolic
// run on one plan.  The flops and symbolic bins come from the plan.
__global__ void k_symbolic_reset(DevCounters *__restrict__ ctr, uint64_t *__restrict__ status,
                                 int64_t nstatus) {
    const int t = threadIdx.x;
    if (t == 0) {
        ctr->tickets[kTkColptr] = 0;
        ctr->tickets[kTkColptrDone] = 0;
        ctr->nnzC = 0;
    }
    if (t < kNumBins) ctr->num_count[t].v = 0;
    for (int64_t s = t; s < nstatus; s += blockDim.x) status[s] = 0;
}

// Split table: for every column c of A that is long in A~ (more than
// kShortLen entries), split[c * (nblk + 1) + b] = the number of its entries
// with row below b * kSplitRows, b = 0 .. nblk.  One wave per column; its
// lanes take the borders in turn, each by a binary search over the column's
// ascending rows.
__global__ __launch_bounds__(256) void k_split_table(int64_t k, int32_t nblk,
                                                     const int64_t *__restrict__ col_start,
                                                     const int32_t *__restrict__ col_len,
                                                     const int32_t *__restrict__ At_rowidx,
                                                     int32_t *__restrict__ split) {
    const int64_t c = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (c >= k) return;
    const int len = col_len[c];
    if (len <= kShortLen) return;
    const int32_t *rows = At_rowidx + col_start[c];
    int32_t *out = split + c * (nblk + 1);
    for (int b = lane_id(); b <= nblk; b += kWave) {
        const int64_t border = (int64_t)b << kSplitShift;
        int lo = 0, hi = len;  // first position whose row is at least the border
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (rows[mid] < border) lo = mid + 1; else hi = mid;
        }
        out[b] = lo;
    }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
int launch_split_table(Plan &p) {
    if (!p.split || p.k == 0) return SPGEMM_OK;
    hipLaunchKernelGGL(k_split_table, dim3((unsigned)((p.k + 3) / 4)), dim3(256), 0, p.stream,
                       p.k, p.nblk, p.col_start, p.col_len, p.At_rowidx, p.split);
    SPG_LAUNCHED("k_split_table");
    return SPGEMM_OK;
}

int launch_symbolic_reset(Plan &p) {
    hipLaunchKernelGGL(k_symbolic_reset, dim3(1), dim3(256), 0, p.stream, p.ctr, p.st_colptr,
                       p.n_col_tiles);
    SPG_LAUNCHED("k_symbolic_reset");
    return SPGEMM_OK;
}

template <int S, typename V>
static int flop_bin_gather_launch(Plan &p) {
    constexpr int COLS = kFlopThreads / S;
    // about kFlopTiles tiles at most: several rounds per tile beyond that.
    // Each tile takes its bins' list slots with one counter atomic per bin,
    // and those atomics on a few addresses queue behind each other: R-MAT 18
    // (262144 columns) plan + symbolic 3.50 ms at 512 tiles, 3.18 ms at 256,
    // 3.75 ms at 2048 (1024-column tiles at most; 2048- and 4096-column
    // tiles were slower again)
    constexpr int64_t kFlopTiles = 256;
    const int64_t base = (p.n + COLS - 1) / COLS;
    const int64_t want = std::max<int64_t>(1, (base + kFlopTiles - 1) / kFlopTiles);
    const int rounds = (int)std::min<int64_t>(kFlopTileCols / COLS, want);
    const int64_t ntiles = (base + rounds - 1) / rounds;
    const int64_t nchunks = p.n > 0 ? (p.nnzB + kLongChunk - 1) / kLongChunk : 0;
    const int64_t ngather = p.nnzA > 0 ? (p.k + kGatherCols - 1) / kGatherCols : 0;
    if (ntiles + nchunks + ngather == 0) return SPGEMM_OK;
    const FlopArgs a{p.n,         p.nnzB,   p.Bcolptr, p.Browidx,  p.col_start, p.col_len,
                     p.th,        p.tstart, p.tlen,    p.col_slot, p.flop,      p.arrive,
                     p.sym_bin,   p.sym_list, p.st_colptr, p.n_col_tiles, p.ctr};
    hipLaunchKernelGGL((k_flop_bin_gather<S, V>), dim3((unsigned)(ntiles + nchunks + ngather)),
                       dim3(kFlopThreads), 0, p.stream, a, ntiles, rounds, nchunks,
                       p.early_tiny ? nullptr : p.hpub_dev, p.hflags_dev + kFlagCounts, p.k,
                       p.Acolptr, p.Arowidx,
                       (const V *)p.Avals, p.map, p.At_colptr, p.At_rowidx, (V *)p.At_vals);
    SPG_LAUNCHED("k_flop_bin_gather (" + std::to_string(ntiles) + " column tiles, " +
                 std::to_string(nchunks) + " chunks, " + std::to_string(ngather) +
                 " gather tiles)");
    return SPGEMM_OK;
}

template <int S>
static int flop_bin_gather_dtype(Plan &p) {
    return p.dtype == SPGEMM_F64 ? flop_bin_gather_launch<S, double>(p)
                                 : flop_bin_gather_launch<S, float>(p);
}

int launch_flop_bin_gather(Plan &p) {
    const double avg = p.n > 0 ? (double)p.nnzB / (double)p.n : 0.0;
    if (avg <= 4.0) return flop_bin_gather_dtype<1>(p);
    if (avg <= 32.0) return flop_bin_gather_dtype<4>(p);
    return flop_bin_gather_dtype<16>(p);
}

template <int T, int G>
static int sym_hash_launch(Plan &p, int bin) {
    const int cnt = p.sym_count[bin];
    if (cnt <= 0) return SPGEMM_OK;
    constexpr int CPW = G < 256 ? 256 / G : 1;
    constexpr int threads = G < 256 ? 256 : G;
    const unsigned g = (unsigned)((cnt + CPW - 1) / CPW);
    hipLaunchKernelGGL((k_sym_hash<T, G>), dim3(g), dim3(threads), 0, p.stream,
                       p.sym_list + (int64_t)bin * p.n, cnt, p.Bcolptr, p.term_range(),
                       p.At_rowidx, p.C_colptr);
    SPG_LAUNCHED("k_sym_hash<" + std::to_string(T) + ">");
    return SPGEMM_OK;
}


// early: launched before the host has the bin counts; sized for every
// column, the count read from the device counters.
int launch_sym_tiny(Plan &p, bool early) {
    const int64_t cols = early ? p.n : p.sym_count[kBinTiny];
    if (cols <= 0) return SPGEMM_OK;
    // early: one more workgroup, which publishes the flops pass's counters
    const unsigned g = (unsigned)((cols + 3) / 4) + (early ? 1u : 0u);
    // the bin holds every column: the kernel takes column w directly
    const int32_t *list = p.sym_list + (int64_t)kBinTiny * p.n;
    if (!early && cols == p.n) list = nullptr;
    const int *count_dev = early ? &p.ctr->sym_count[kBinTiny].v : nullptr;
    PublishedCounts *hout = early ? p.hpub_dev : nullptr;
    unsigned int *hready = p.hflags_dev + kFlagCounts;
    if (p.th.tiny_max_flop <= 4 * kWave)
        hipLaunchKernelGGL(k_sym_tiny<4>, dim3(g), dim3(256), 0, p.stream, list, (int)cols,
                           count_dev, (int)p.n, p.Bcolptr, p.term_range(), p.At_rowidx, p.flop,
                           p.C_colptr, p.tiny_perm, p.col_slot, p.ctr, hout, hready);
    else
        hipLaunchKernelGGL(k_sym_tiny<8>, dim3(g), dim3(256), 0, p.stream, list, (int)cols,
                           count_dev, (int)p.n, p.Bcolptr, p.term_range(), p.At_rowidx, p.flop,
                           p.C_colptr, p.tiny_perm, p.col_slot, p.ctr, hout, hready);
    SPG_LAUNCHED(early ? "k_sym_tiny (before the counts)" : "k_sym_tiny");
    return SPGEMM_OK;
}

int launch_symbolic_bins(Plan &p, bool tiny_launched) {
    if (p.n == 0) return SPGEMM_OK;
    int rc;
    if (!tiny_launched && (rc = launch_sym_tiny(p, false))) return rc;
    if ((rc = sym_hash_launch<kSymTable[0], 64>(p, kBinH0))) return rc;
    if ((rc = sym_hash_launch<kSymTable[1], 64>(p, kBinH1))) return rc;
    if ((rc = sym_hash_launch<kSymTable[2], 256>(p, kBinH2))) return rc;
    if ((rc = sym_hash_launch<kSymTable[3], 512>(p, kBinH3))) return rc;
    if (p.sym_count[kBinDense] > 0) {
        // taller columns are counted in bands of kMaxDenseRows rows, which
        // reach A~ through the split table
        if (p.m > kMaxDenseRows && (rc = ensure_split_table(p, p.sym_count[kBinDense])))
            return rc;
        const size_t lds = (size_t)((std::min<int64_t>(p.m, kMaxDenseRows) + 31) / 32) * 4;
        const unsigned grid = resident_groups((const void *)k_sym_dense, kDenseThreads, lds,
                                              p.device, p.sym_count[kBinDense]);
        hipLaunchKernelGGL(k_sym_dense, dim3(grid), dim3(kDenseThreads), lds, p.stream,
                           p.sym_list + (int64_t)kBinDense * p.n, p.sym_count[kBinDense], p.m,
                           p.Bcolptr, p.term_range(), p.At_rowidx, p.C_colptr,
                           p.m <= kMaxDenseRows ? p.dense_bits : nullptr, p.col_slot, p.Browidx,
                           p.split, p.nblk, p.ctr);
        SPG_LAUNCHED("k_sym_dense (" + std::to_string(grid) + " workgroups)");
    }
    return SPGEMM_OK;
}

int launch_colptr_scan(Plan &p) {
    if (p.n == 0) return SPGEMM_OK;
    if (p.n <= kSmallScanCols) {
        hipLaunchKernelGGL(k_colptr_scan_small, dim3(1), dim3(kSmallScanThreads), 0, p.stream, p.n,
                           p.C_colptr, p.flop, p.th, p.num_bin, p.num_list, p.ctr, p.hpub_dev,
                           p.hflags_dev + kFlagColptr,
                           reinterpret_cast<unsigned long long *>(p.hflags_dev + kNnzSlot));
        SPG_HIP(hipGetLastError());
        return SPGEMM_OK;
    }
    hipLaunchKernelGGL(k_colptr_scan, dim3((unsigned)p.n_col_tiles), dim3(kScanThreads), 0,
                       p.stream, p.n, p.C_colptr, p.flop, p.th, p.num_bin, p.num_list,
                       p.st_colptr, p.n_col_tiles, p.ctr, p.hpub_dev,
                       p.hflags_dev + kFlagColptr);
    SPG_HIP(hipGetLastError());
    return SPGEMM_OK;
}

}  // namespace spg
