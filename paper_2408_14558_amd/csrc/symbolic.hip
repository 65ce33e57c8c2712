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

// Records where entry q of B_i finds its products in A~ (the column of A~
// that map assigns to q's row) and returns their number.
__device__ __forceinline__ int term_range(int64_t q, const int32_t *__restrict__ Browidx,
                                          const int32_t *__restrict__ map,
                                          const int64_t *__restrict__ At_colptr,
                                          int64_t *__restrict__ tstart,
                                          int32_t *__restrict__ tlen) {
    const int32_t jt = map[Browidx[q]];
    long long start = 0;
    int len = 0;
    if (jt >= 0) {
        start = At_colptr[jt];
        len = (int)(At_colptr[jt + 1] - start);
    }
    tstart[q] = start;
    tlen[q] = len;
    return len;
}

// Sparse flops of every column of B_i and its symbolic bin, and the term
// range of every entry of B_i; tile `blk` of `ngroups`.  S lanes walk
// one column (S picked from the average column length); columns with more
// than 16*S entries are walked by the whole workgroup afterwards.
constexpr int kFlopThreads = 256;
template <int S>
__device__ __forceinline__ void flop_bin_tile(
    int64_t blk, int64_t ngroups,
    int64_t n, const int64_t *__restrict__ Bcolptr, const int32_t *__restrict__ Browidx,
    const int32_t *__restrict__ map, const int64_t *__restrict__ At_colptr, Thresholds th,
    int64_t *__restrict__ tstart, int32_t *__restrict__ tlen, int32_t *__restrict__ col_slot,
    int64_t *__restrict__ flop, int32_t *__restrict__ sym_bin, int32_t *__restrict__ sym_list,
    uint64_t *__restrict__ status, int64_t nstatus, DevCounters *__restrict__ ctr,
    PublishedCounts *__restrict__ hout, unsigned int *__restrict__ hready) {
    constexpr int COLS = kFlopThreads / S;
    __shared__ int s_bin[COLS];
    __shared__ int s_lpos[COLS];
    __shared__ int s_long[COLS];
    __shared__ long long s_f[COLS];
    __shared__ int s_cnt[kNumBins];
    __shared__ int s_base[kNumBins];
    __shared__ int s_nlong;
    __shared__ long long s_flops;
    __shared__ long long s_red[kFlopThreads / kWave + 1];
    const int tid = threadIdx.x;
    {
        const int64_t stride = ngroups * kFlopThreads;
        for (int64_t s = blk * kFlopThreads + tid; s < nstatus; s += stride) status[s] = 0;
    }
    if (tid < kNumBins) s_cnt[tid] = 0;
    if (tid == 0) {
        s_flops = 0;
        s_nlong = 0;
    }
    __syncthreads();
    const int64_t j0 = blk * COLS;
    const int nloc = (int)min<int64_t>(COLS, n - j0);
    const int lc = tid / S, sub = tid % S;
    long long acc = 0;
    bool deferred = false;
    if (lc < nloc) {
        const int64_t q0 = Bcolptr[j0 + lc], q1 = Bcolptr[j0 + lc + 1];
        if (q1 - q0 <= 16 * S) {
#pragma unroll 4
            for (int64_t q = q0 + sub; q < q1; q += S) acc += term_range(q, Browidx, map, At_colptr, tstart, tlen);
        } else {
            deferred = true;
        }
    }
    acc = wave_sum<S>(acc);
    if (lc < nloc && sub == 0) {
        if (deferred) s_long[atomicAdd(&s_nlong, 1)] = lc;
        else s_f[lc] = acc;
    }
    __syncthreads();
    // long columns one after the other, each by the whole workgroup with
    // kLongUnroll entries in flight per thread: the loads of one entry
    // (row, map, A~'s pointers) depend on each other, those of different
    // entries do not
    constexpr int kLongUnroll = 8;
    const int nlong = s_nlong;
    for (int li = 0; li < nlong; ++li) {
        const int t = s_long[li];
        const int64_t q0 = Bcolptr[j0 + t], q1 = Bcolptr[j0 + t + 1];
        long long a2 = 0;
        for (int64_t qb = q0 + tid; qb < q1; qb += kLongUnroll * kFlopThreads) {
            // loads without branches (an index out of the range reads a
            // valid element and is discarded), so all of a round's loads of
            // one kind are in flight together
            int32_t jt[kLongUnroll];
#pragma unroll
            for (int u = 0; u < kLongUnroll; ++u) {
                const int64_t q = qb + (int64_t)u * kFlopThreads;
                const int32_t r = Browidx[q < q1 ? q : q1 - 1];
                jt[u] = q < q1 ? r : -1;
            }
#pragma unroll
            for (int u = 0; u < kLongUnroll; ++u) {
                const int32_t c = map[jt[u] >= 0 ? jt[u] : 0];
                jt[u] = jt[u] >= 0 ? c : -1;
            }
            long long st[kLongUnroll];
            int len[kLongUnroll];
#pragma unroll
            for (int u = 0; u < kLongUnroll; ++u) {
                const bool ok = jt[u] >= 0;
                const long long a0 = At_colptr[ok ? jt[u] : 0];
                const long long a1 = At_colptr[ok ? jt[u] + 1 : 0];
                st[u] = ok ? a0 : 0;
                len[u] = ok ? (int)(a1 - a0) : 0;
            }
#pragma unroll
            for (int u = 0; u < kLongUnroll; ++u) {
                const int64_t q = qb + (int64_t)u * kFlopThreads;
                if (q < q1) {
                    tstart[q] = st[u];
                    tlen[q] = len[u];
                    a2 += len[u];
                }
            }
        }
        long long tot;
        group_excl_scan64<kFlopThreads>(a2, s_red, &tot);
        if (tid == 0) s_f[t] = tot;
    }
    __syncthreads();
    if (tid < nloc) {
        const int64_t j = j0 + tid;
        const long long f = s_f[tid];
        flop[j] = f;
        col_slot[j] = -1;
        const int b = sym_bin_of(f, th);
        sym_bin[j] = b;
        s_bin[tid] = b;
        s_lpos[tid] = (b != kBinEmpty) ? atomicAdd(&s_cnt[b], 1) : 0;
        if (f) atomic_add_i64(&s_flops, f);
    }
    __syncthreads();
    if (tid == 0 && s_flops) atomic_add_i64(&ctr->flops.v, s_flops);
    append_to_bins(nloc, s_bin, s_lpos, s_cnt, s_base, j0, ctr->sym_count, sym_list, n);
    __shared__ int s_last;
    publish_when_last(&ctr->tickets[kTkFlopDone], (unsigned long long)ngroups, ctr, hout, hready,
                      &s_last);
}

// One launch for two independent steps that both follow the selection: the
// flop and binning tiles (first, since the host waits for their counts) and
// the gather tiles of A~.  Neither reads what the other writes, so their
// chains of dependent loads overlap instead of running one after the other.
static_assert(kFlopThreads == kGatherThreads, "both tiles use the whole workgroup");
template <int S, typename V>
__global__ __launch_bounds__(kFlopThreads) void k_flop_bin_gather(
    int64_t nflop, int64_t n, const int64_t *__restrict__ Bcolptr,
    const int32_t *__restrict__ Browidx, const int32_t *__restrict__ map,
    const int64_t *__restrict__ At_colptr, Thresholds th, int64_t *__restrict__ tstart,
    int32_t *__restrict__ tlen, int32_t *__restrict__ col_slot, int64_t *__restrict__ flop,
    int32_t *__restrict__ sym_bin, int32_t *__restrict__ sym_list, uint64_t *__restrict__ status,
    int64_t nstatus, DevCounters *__restrict__ ctr, PublishedCounts *__restrict__ hout,
    unsigned int *__restrict__ hready, int64_t k, const int64_t *__restrict__ Acolptr,
    const int32_t *__restrict__ Arowidx, const V *__restrict__ Avals,
    int32_t *__restrict__ At_rowidx, V *__restrict__ At_vals) {
    const int64_t blk = blockIdx.x;
    if (blk < nflop) {
        flop_bin_tile<S>(blk, nflop, n, Bcolptr, Browidx, map, At_colptr, th, tstart, tlen,
                         col_slot, flop, sym_bin, sym_list, status, nstatus, ctr, hout, hready);
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
    int key[E];
#pragma unroll
    for (int r = 0; r < E; ++r) {
        key[r] = kNoRow;
        if (p[r] >= 0)
            key[r] = perm ? (At_rowidx[p[r]] << kSlotBits) | (r * kWave + lane) : At_rowidx[p[r]];
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

template <int EMAX>
__global__ __launch_bounds__(256) void k_sym_tiny(const int32_t *__restrict__ list, int count,
                                                  const int64_t *__restrict__ Bcolptr,
                                                  TermRange tr,
                                                  const int32_t *__restrict__ At_rowidx,
                                                  const int64_t *__restrict__ flop,
                                                  int64_t *__restrict__ Ccount,
                                                  uint16_t *__restrict__ tiny_perm,
                                                  int32_t *__restrict__ col_slot) {
    const int w = blockIdx.x * 4 + (threadIdx.x >> 6);
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
constexpr int kSymDenseUnroll = 8;  // row loads in flight per lane on long A~ columns
struct SymDenseLds {
    TermStage<kDenseThreads, float> st;
    int red[kDenseThreads / kWave + 2];
};

__global__ __launch_bounds__(kDenseThreads) void k_sym_dense(
    const int32_t *__restrict__ list, int count, int64_t m, const int64_t *__restrict__ Bcolptr,
    TermRange tr, const int32_t *__restrict__ At_rowidx, int64_t *__restrict__ Ccount,
    uint32_t *__restrict__ keep_bits, int32_t *__restrict__ col_slot,
    DevCounters *__restrict__ ctr) {
    extern __shared__ __align__(16) uint32_t s_bits[];
    __shared__ SymDenseLds L;
    __shared__ int s_item;
    unsigned int *queue = ctr->sym_dense_queue;
    const int nw = (int)((m + 31) >> 5);
    const int gt = threadIdx.x;
    for (int w = queue_take(queue, &s_item); w < count; w = queue_take(queue, &s_item)) {
        const int32_t j = list[w];
        zero_words<kDenseThreads>(s_bits, nw);
        __syncthreads();
        // short entries stay with their thread: a flat walk would give a wave
        // consecutive rows of one column of A~, whose bits share words
        for_each_term<kDenseThreads, float, kSymDenseUnroll, kDenseThreads, false>(
            Bcolptr[j], Bcolptr[j + 1], tr, nullptr, &L.st, gt,
            [&](int64_t p) { return At_rowidx[p]; },
            [&](int32_t r, float) { atomicOr(&s_bits[r >> 5], 1u << (r & 31)); });
        int c = 0;
        for (int i = gt; i < nw; i += kDenseThreads) c += __popc(s_bits[i]);
        int total;
        (void)group_excl_scan<kDenseThreads>(c, L.red, &total);
        if (gt == 0) Ccount[j] = total;
        if (keep_bits) {  // the numeric phase reuses this bitmap
            uint32_t *dst = keep_bits + (size_t)w * nw;
            copy_words<kDenseThreads>(dst, s_bits, nw);
            if (gt == 0) col_slot[j] = w;
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
    long long cnt[kScanItems];
    long long sum = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const int lc = tid * kScanItems + i;
        cnt[i] = 0;
        if (lc < nloc) {
            const int64_t j = j0 + lc;
            cnt[i] = flop[j] == 0 ? 0 : Ccolptr[j];  // empty columns have no count
            int b = num_bin_of(flop[j], cnt[i], th);
            if (b == kBinDense && th.dense_first_flop > 0 && flop[j] >= th.dense_first_flop)
                b = kBinDenseFirst;
            num_bin[j] = b;
            s_bin[lc] = b;
            s_lpos[lc] = (b != kBinEmpty) ? atomicAdd(&s_cnt[b], 1) : 0;
        }
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

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
int launch_symbolic_reset(Plan &p) {
    hipLaunchKernelGGL(k_symbolic_reset, dim3(1), dim3(256), 0, p.stream, p.ctr, p.st_colptr,
                       p.n_col_tiles);
    SPG_LAUNCHED("k_symbolic_reset");
    return SPGEMM_OK;
}

template <int S, typename V>
static int flop_bin_gather_launch(Plan &p) {
    constexpr int COLS = kFlopThreads / S;
    const int64_t nflop = (p.n + COLS - 1) / COLS;
    const int64_t ngather = p.nnzA > 0 ? (p.k + kGatherCols - 1) / kGatherCols : 0;
    if (nflop + ngather == 0) return SPGEMM_OK;
    hipLaunchKernelGGL((k_flop_bin_gather<S, V>), dim3((unsigned)(nflop + ngather)),
                       dim3(kFlopThreads), 0, p.stream, nflop, p.n, p.Bcolptr, p.Browidx, p.map,
                       p.At_colptr, p.th, p.tstart, p.tlen, p.col_slot, p.flop, p.sym_bin,
                       p.sym_list, p.st_colptr, p.n_col_tiles, p.ctr, p.hpub_dev,
                       p.hflags_dev + kFlagCounts, p.k, p.Acolptr, p.Arowidx,
                       (const V *)p.Avals, p.At_rowidx, (V *)p.At_vals);
    SPG_LAUNCHED("k_flop_bin_gather (" + std::to_string(nflop) + " flop tiles, " +
                 std::to_string(ngather) + " gather tiles)");
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


int launch_symbolic_bins(Plan &p) {
    if (p.n == 0) return SPGEMM_OK;
    if (p.sym_count[kBinTiny] > 0) {
        const unsigned g = (unsigned)((p.sym_count[kBinTiny] + 3) / 4);
        // the bin holds every column: the kernel takes column w directly
        const int32_t *list =
            p.sym_count[kBinTiny] == p.n ? nullptr : p.sym_list + (int64_t)kBinTiny * p.n;
        if (p.th.tiny_max_flop <= 4 * kWave)
            hipLaunchKernelGGL(k_sym_tiny<4>, dim3(g), dim3(256), 0, p.stream, list,
                               p.sym_count[kBinTiny], p.Bcolptr, p.term_range(), p.At_rowidx,
                               p.flop, p.C_colptr, p.tiny_perm, p.col_slot);
        else
            hipLaunchKernelGGL(k_sym_tiny<8>, dim3(g), dim3(256), 0, p.stream, list,
                               p.sym_count[kBinTiny], p.Bcolptr, p.term_range(), p.At_rowidx,
                               p.flop, p.C_colptr, p.tiny_perm, p.col_slot);
        SPG_LAUNCHED("k_sym_tiny");
    }
    int rc;
    if ((rc = sym_hash_launch<kSymTable[0], 64>(p, kBinH0))) return rc;
    if ((rc = sym_hash_launch<kSymTable[1], 64>(p, kBinH1))) return rc;
    if ((rc = sym_hash_launch<kSymTable[2], 256>(p, kBinH2))) return rc;
    if ((rc = sym_hash_launch<kSymTable[3], 512>(p, kBinH3))) return rc;
    if (p.sym_count[kBinDense] > 0) {
        if (p.m > kMaxDenseRows)
            return fail(SPGEMM_EUNSUPPORTED,
                        "columns with more flops than the largest hash bin need m <= 262144");
        const size_t lds = (size_t)((p.m + 31) / 32) * 4;
        const unsigned grid = resident_groups((const void *)k_sym_dense, kDenseThreads, lds,
                                              p.device, p.sym_count[kBinDense]);
        hipLaunchKernelGGL(k_sym_dense, dim3(grid), dim3(kDenseThreads), lds, p.stream,
                           p.sym_list + (int64_t)kBinDense * p.n, p.sym_count[kBinDense], p.m,
                           p.Bcolptr, p.term_range(), p.At_rowidx, p.C_colptr, p.dense_bits,
                           p.col_slot, p.ctr);
        SPG_LAUNCHED("k_sym_dense (" + std::to_string(grid) + " workgroups)");
    }
    return SPGEMM_OK;
}

int launch_colptr_scan(Plan &p) {
    if (p.n == 0) return SPGEMM_OK;
    hipLaunchKernelGGL(k_colptr_scan, dim3((unsigned)p.n_col_tiles), dim3(kScanThreads), 0,
                       p.stream, p.n, p.C_colptr, p.flop, p.th, p.num_bin, p.num_list,
                       p.st_colptr, p.n_col_tiles, p.ctr, p.hpub_dev,
                       p.hflags_dev + kFlagColptr);
    SPG_HIP(hipGetLastError());
    return SPGEMM_OK;
}

}  // namespace spg
