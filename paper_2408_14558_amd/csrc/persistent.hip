// The batched numeric phase as ONE persistent launch: the numeric work of
// many planned products (the Galerkin products of an AMG setup, Sec. II-C
// and Sec. IV-B, or independent products of uneven sizes) cut into work
// items that the workgroups of a single kernel take in turn.
//
// Work items, in dependency order (products by depth; at each depth first
// every product's value gather, then its numeric columns; a product whose A~
// holds all of A reads its new A values in place and has no gather):
//   gather  tiles of 64 columns of A whose new values go into A~ (the
//           values half of Alg. 1's fetch, for a product whose A is another
//           product's C);
//   tiny    tiny columns, one wave each at a time;
//   hash h  columns of hash bin h, one LDS table per group at a time.
// Items are sized so that a product's bin gives about one item per resident
// workgroup (at least one column per group), which keeps the count of
// items, and so of completion flags and fences, small.
// An atomic ticket hands the items out in that order.  An item waits only
// for items with lower tickets (its own product's gathers before its
// numeric columns; the whole numeric phase of the product whose C it
// reads, or its A values when they are read in place), and each of those is
// held by a workgroup that is already running and itself waits only on
// lower tickets, so the launch always drains.
//
// Completion is published per item, the way the chained scans of this
// library publish their tile states: a workgroup that finishes an item makes
// its writes visible at agent scope (every wave: release fence, then the
// workgroup barrier) and thread 0 stores the item's flag with a release
// store.  A waiting workgroup reads the flags of the items it needs with
// relaxed agent-scope loads, all threads in parallel, and every wave then
// acquires at agent scope before reading their data.  No completion count
// is kept with atomic adds; atomics serve only the ticket and the exit
// count, whose returned values are used.  Every wait is bounded in time
// (wall clock): past the bound, or once another workgroup has given up, the
// workgroup stores the batch's error word and goes on, so a launch ends
// even if a flag never arrives, and the host reports the error.  The
// workgroup that leaves last clears the ticket, the exit count and the
// flags, so the next launch (or graph replay) starts clean.
//
// Numeric bins run the tiny and LDS hash column routines of the plain path
// (a medium column that the plain path would give the bitmap kernel uses
// the hash routine of its bin here; the result is the same).  Products with
// dense columns are not taken (SPGEMM_EUNSUPPORTED at batch creation).
#include <algorithm>
#include <climits>
#include <cstring>
#include <string>
#include <vector>

#include "gather.hpp"
#include "numeric.hpp"

namespace spg {

enum PKind : int32_t { kPGather = 0, kPTiny = 1, kPHash0 = 2 };  // kPHash0 + h for bin h

struct PItem {
    int32_t prod;
    int32_t kind;
    int32_t first;  // gather: tile index; numeric: first position in the bin's list
    int32_t count;  // numeric: columns of the item
};

template <typename V>
struct PProd {
    NumArgs<V> a;
    const int32_t *list[kNumBins];  // numeric bin lists of the plan
    int32_t packed;                 // tiny columns sort packed keys (m below kPackedRowLimit)
    int32_t dep_A, dep_B;           // product whose C is this A / B, or -1
    int32_t gather_first, n_gather;    // its value-gather items (consecutive tickets)
    int32_t numeric_first, n_numeric;  // its numeric items (consecutive tickets)
    int32_t publish;                   // another product of the batch reads its C
    // new values of A gathered into A~ (gather items only)
    const int64_t *Acolptr;
    const V *Avals;
    const int32_t *map;
    const int64_t *At_colptr;
    int64_t k;
    V *At_vals;
};

// Control block (u32 words): ticket, workgroups that left, error word, each
// on a 128-byte line of its own, then one completion flag per item.
constexpr int kPLine = 32;
constexpr int kPTicket = 0, kPExit = kPLine, kPError = 2 * kPLine, kPFlags = 3 * kPLine;
constexpr int kPThreads = 256;

// All threads of the workgroup: waits until the flags of items
// [first, first + count) are set.  False once `ticks` of the wall clock have
// passed or the error word is set; s_stop is LDS.
__device__ __forceinline__ bool wait_items(const unsigned *flags, int first, int count,
                                           const unsigned *err, long long ticks, int *s_stop) {
    if (count <= 0) return true;
    const unsigned long long t0 = wall_clock64();
    while (true) {
        int mine = 1;
        for (int i = threadIdx.x; i < count; i += kPThreads)
            mine &= __hip_atomic_load(&flags[first + i], __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_AGENT) != 0u;
        if (__syncthreads_and(mine)) return true;
        if (threadIdx.x == 0)
            *s_stop = (long long)(wall_clock64() - t0) > ticks ||
                      __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u;
        __syncthreads();
        if (*s_stop) return false;
        __builtin_amdgcn_s_sleep(2);
    }
}

template <typename V>
union PLds {
    struct {
        int rows[4][4 * kWave];
        Acc vals[4][4 * kWave];
    } tiny;
    NumHashLds<kNumTable[0], 32, V> h0[8];
    NumHashLds<kNumTable[1], 64, V> h1[4];
    NumHashLds<kNumTable[2], kPThreads, V> h2;
    NumHashLds<kNumTable[3], kPThreads, V> h3;
    GatherStage g;
};

template <typename V>
__global__ __launch_bounds__(kPThreads) void k_batch_persistent(const PItem *__restrict__ items,
                                                                int nitems,
                                                                const PProd<V> *__restrict__ prods,
                                                                unsigned *__restrict__ ctr,
                                                                long long wait_ticks) {
    __shared__ PLds<V> L;
    __shared__ int s_item, s_stop;
    const int tid = threadIdx.x;
    unsigned *flags = ctr + kPFlags;
    while (true) {
        __syncthreads();  // every thread is done with the previous item
        if (tid == 0) s_item = (int)atomicAdd(&ctr[kPTicket], 1u);
        __syncthreads();
        const int t = s_item;
        if (t >= nitems) break;
        const PItem it = items[t];
        const PProd<V> &P = prods[it.prod];
        // the waits (and the acquire) only where the item reads another
        // item's output
        bool ok = true, waited = false;
        if (it.kind == kPGather) {
            if (P.dep_A >= 0) {
                waited = true;
                ok = wait_items(flags, prods[P.dep_A].numeric_first, prods[P.dep_A].n_numeric,
                                ctr + kPError, wait_ticks, &s_stop);
            }
        } else {
            if (P.n_gather > 0) {
                waited = true;
                ok = wait_items(flags, P.gather_first, P.n_gather, ctr + kPError, wait_ticks,
                                &s_stop);
            } else if (P.dep_A >= 0) {  // A's new values read in place: they are dep_A's C
                waited = true;
                ok = wait_items(flags, prods[P.dep_A].numeric_first, prods[P.dep_A].n_numeric,
                                ctr + kPError, wait_ticks, &s_stop);
            }
            if (ok && P.dep_B >= 0) {
                waited = true;
                ok = wait_items(flags, prods[P.dep_B].numeric_first, prods[P.dep_B].n_numeric,
                                ctr + kPError, wait_ticks, &s_stop);
            }
        }
        if (!ok && tid == 0)
            __hip_atomic_store(&ctr[kPError], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        if (waited) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        const int end = it.first + it.count;
        if (it.kind == kPGather) {
            for (int g = it.first; g < end; ++g)  // gather_tile ends with a barrier
                gather_tile<V, false>(g, P.Acolptr, nullptr, P.Avals, P.map, P.At_colptr, P.k,
                                      nullptr, P.At_vals, L.g);
        } else if (it.kind == kPTiny) {
            // the product's arguments copied once per item, so the column
            // routines keep them in scalar registers instead of reading them
            // from the table at every use
            const NumArgs<V> a = P.a;
            const int wv = tid / kWave;
            for (int c = it.first + wv; c < end; c += kPThreads / kWave) {
                const int32_t j = P.list[kBinTiny][c];
                if (P.packed)
                    num_wave_dispatch<V, 4, true>(a, j, L.tiny.rows[wv], L.tiny.vals[wv]);
                else
                    num_wave_dispatch<V, 4, false>(a, j, L.tiny.rows[wv], L.tiny.vals[wv]);
                wave_sync();  // the wave's LDS rows are reused by its next column
            }
        } else {
            const NumArgs<V> a = P.a;  // copied once per item (see above)
            // num_hash_column ends with a barrier of its group, so a group's
            // next column may reuse its table
            const int h = it.kind - kPHash0;
            const int32_t *list = P.list[kBinH0 + h];
            if (h == 0) {
                const int grp = tid / 32;
                for (int c = it.first + grp; c < end; c += kPThreads / 32)
                    num_hash_column<kNumTable[0], 32, V>(a, list[c], L.h0[grp], tid % 32);
            } else if (h == 1) {
                const int grp = tid / kWave;
                for (int c = it.first + grp; c < end; c += kPThreads / kWave)
                    num_hash_column<kNumTable[1], 64, V>(a, list[c], L.h1[grp], tid % kWave);
            } else if (h == 2) {
                for (int c = it.first; c < end; ++c)
                    num_hash_column<kNumTable[2], kPThreads, V>(a, list[c], L.h2, tid);
            } else {
                for (int c = it.first; c < end; ++c)
                    num_hash_column<kNumTable[3], kPThreads, V>(a, list[c], L.h3, tid);
            }
        }
        // publish, where another item reads this one's output: every wave's
        // writes visible at agent scope, then the flag
        if (it.kind == kPGather || P.publish) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __syncthreads();
            if (tid == 0)
                __hip_atomic_store(&flags[t], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    // the workgroup that leaves last clears the ticket, the exit count and
    // the flags (the error word stays for the host)
    if (tid == 0) {
        __threadfence();
        s_item = atomicAdd(&ctr[kPExit], 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (s_item) {
        for (int i = tid; i < nitems; i += kPThreads)
            __hip_atomic_store(&flags[i], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (tid == 0) {
            __hip_atomic_store(&ctr[kPTicket], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&ctr[kPExit], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
// Columns an item of a numeric bin takes at least: one per group of the
// workgroup (tiny: four waves; hash bin 0: eight groups of 32; bin 1: four
// waves; bins 2 and 3: the whole workgroup).
static int per_group(int bin) {
    switch (bin) {
    case kBinTiny: return 4;
    case kBinH0: return 8;
    case kBinH1: return 4;
    default: return 1;
    }
}

// Units per item for `count` units: a multiple of `base`, about `target`
// items in all.
static int64_t item_size(int64_t count, int64_t base, int64_t target) {
    const int64_t per = (count + target - 1) / target;
    return std::max<int64_t>(base, (per + base - 1) / base * base);
}

template <typename V>
static int build_t(const std::vector<Plan *> &plans, const std::vector<spgemm_batch_io> &io,
                   const std::vector<std::vector<int>> &levels, PersistentBatch &pb) {
    const int n = (int)plans.size();
    // about one item per resident workgroup for every product's bin (the
    // fastest of 1, 2 and 8 on the AMG chain: each published item costs an
    // agent-scope release and each waiting item an acquire)
    const unsigned resident = resident_groups((const void *)k_batch_persistent<V>, kPThreads, 0,
                                              pb.device, 1LL << 30);
    const int64_t target = (int64_t)std::max(1u, resident);
    std::vector<PProd<V>> prods(n);
    std::vector<PItem> items;
    for (int t = 0; t < n; ++t) {
        Plan &p = *plans[t];
        PProd<V> &P = prods[t];
        std::memset(&P, 0, sizeof(P));
        const V *Bv = (const V *)(io[t].B_vals ? io[t].B_vals : p.Bvals);
        // new A values read in place when A~ holds all of A (nothing to gather)
        const bool in_place = io[t].A_vals && p.nnzAt_pub == p.nnzA;
        const V *Atv = (const V *)(in_place ? io[t].A_vals : p.At_vals);
        P.a = NumArgs<V>{p.m,        p.Bcolptr,    p.term_range(), Bv,        p.At_rowidx,
                         Atv,                      p.C_colptr,     io[t].C_rowidx,
                         (V *)io[t].C_vals,        p.flop,         p.Browidx, p.split,
                         p.col_slot, p.dense_bits, p.tiny_perm, p.nblk};
        for (int b = 0; b < kNumBins; ++b) P.list[b] = p.num_list + (int64_t)b * p.n;
        P.packed = p.m < kPackedRowLimit;
        P.dep_A = io[t].dep_A;
        P.dep_B = io[t].dep_B;
        if (P.dep_A >= 0) prods[P.dep_A].publish = 1;
        if (P.dep_B >= 0) prods[P.dep_B].publish = 1;
        P.Acolptr = p.Acolptr;
        P.Avals = (const V *)io[t].A_vals;
        P.map = p.map;
        P.At_colptr = p.At_colptr;
        P.k = p.k;
        P.At_vals = (V *)p.At_vals;
    }
    for (const std::vector<int> &lvl : levels) {
        for (int t : lvl) {  // value gathers of this depth
            Plan &p = *plans[t];
            if (!io[t].A_vals || p.k == 0 || p.nnzA == 0 || p.nnzAt_pub == p.nnzA) continue;
            const int64_t tiles = (p.k + kGatherCols - 1) / kGatherCols;
            const int64_t per = item_size(tiles, 1, target);
            prods[t].gather_first = (int32_t)items.size();
            for (int64_t g = 0; g < tiles; g += per)
                items.push_back(PItem{t, kPGather, (int32_t)g, (int32_t)std::min(per, tiles - g)});
            prods[t].n_gather = (int32_t)(items.size() - prods[t].gather_first);
        }
        for (int t : lvl) {  // then the numeric columns of this depth
            Plan &p = *plans[t];
            if (p.n == 0 || p.nnzC == 0) continue;
            prods[t].numeric_first = (int32_t)items.size();
            for (int b = kBinTiny; b <= kBinH3; ++b) {
                const int64_t c = p.num_count[b];
                const int64_t per = item_size(c, per_group(b), target);
                const int32_t kind = b == kBinTiny ? (int32_t)kPTiny : (int32_t)(kPHash0 + b - kBinH0);
                for (int64_t f = 0; f < c; f += per)
                    items.push_back(PItem{t, kind, (int32_t)f, (int32_t)std::min(per, c - f)});
            }
            prods[t].n_numeric = (int32_t)(items.size() - prods[t].numeric_first);
        }
    }
    if (items.size() >= (size_t)(INT32_MAX / 2)) return fail(SPGEMM_EUNSUPPORTED, "too many work items");
    pb.nitems = (int)items.size();
    pb.nprod = n;
    pb.ctr_bytes = sizeof(unsigned) * ((size_t)kPFlags + items.size());
    const size_t ib = sizeof(PItem) * std::max<size_t>(1, items.size());
    const size_t pbytes = sizeof(PProd<V>) * (size_t)n;
    SPG_HIP(hipMalloc(&pb.items, ib));
    SPG_HIP(hipMalloc(&pb.prods, pbytes));
    SPG_HIP(hipMalloc(&pb.ctr, pb.ctr_bytes));
    if (!items.empty())
        SPG_HIP(hipMemcpy(pb.items, items.data(), sizeof(PItem) * items.size(),
                          hipMemcpyHostToDevice));
    SPG_HIP(hipMemcpy(pb.prods, prods.data(), pbytes, hipMemcpyHostToDevice));
    SPG_HIP(hipMemset(pb.ctr, 0, pb.ctr_bytes));
    pb.grid = resident_groups((const void *)k_batch_persistent<V>, kPThreads, 0, pb.device,
                              std::max<long long>(1, (long long)items.size()));
    return SPGEMM_OK;
}

int persistent_build(const std::vector<Plan *> &plans, const std::vector<spgemm_batch_io> &io,
                     const std::vector<std::vector<int>> &levels, PersistentBatch &pb) {
    for (size_t t = 0; t < plans.size(); ++t) {
        const Plan &p = *plans[t];
        if (p.num_count[kBinDense] + p.num_count[kBinDenseFirst] > 0)
            return fail(SPGEMM_EUNSUPPORTED, "product " + std::to_string(t) +
                                                 " has dense columns; the single-launch batch "
                                                 "takes tiny and hash columns only");
        if (p.th.tiny_max_flop > 4 * kWave)
            return fail(SPGEMM_EUNSUPPORTED, "product " + std::to_string(t) +
                                                 ": the single-launch batch needs "
                                                 "tiny_max_flop <= 256");
    }
    SPG_HIP(hipGetDevice(&pb.device));
    // a wait bound far above any item's run time: 250 ms of the wall clock
    int khz = 0;
    SPG_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, pb.device));
    pb.wait_ticks = (long long)std::max(khz, 1000) * 250;
    pb.dtype = plans.empty() ? SPGEMM_F64 : plans[0]->dtype;
    int rc = pb.dtype == SPGEMM_F64 ? build_t<double>(plans, io, levels, pb)
                                    : build_t<float>(plans, io, levels, pb);
    if (rc) persistent_free(pb);
    return rc;
}

int persistent_launch(const PersistentBatch &pb, hipStream_t s) {
    if (pb.nitems == 0) return SPGEMM_OK;
    if (pb.dtype == SPGEMM_F64)
        hipLaunchKernelGGL(k_batch_persistent<double>, dim3(pb.grid), dim3(kPThreads), 0, s,
                           (const PItem *)pb.items, pb.nitems, (const PProd<double> *)pb.prods,
                           pb.ctr, pb.wait_ticks);
    else
        hipLaunchKernelGGL(k_batch_persistent<float>, dim3(pb.grid), dim3(kPThreads), 0, s,
                           (const PItem *)pb.items, pb.nitems, (const PProd<float> *)pb.prods,
                           pb.ctr, pb.wait_ticks);
    SPG_LAUNCHED("k_batch_persistent (" + std::to_string(pb.grid) + " workgroups, " +
                 std::to_string(pb.nitems) + " items)");
    return SPGEMM_OK;
}

int persistent_error(const PersistentBatch &pb, unsigned *err) {
    *err = 0;
    if (!pb.ctr) return SPGEMM_OK;
    SPG_HIP(hipMemcpy(err, pb.ctr + kPError, sizeof(unsigned), hipMemcpyDeviceToHost));
    if (*err) SPG_HIP(hipMemset(pb.ctr + kPError, 0, sizeof(unsigned)));
    return SPGEMM_OK;
}

void persistent_free(PersistentBatch &pb) {
    if (pb.items) (void)hipFree(pb.items);
    if (pb.prods) (void)hipFree(pb.prods);
    if (pb.ctr) (void)hipFree(pb.ctr);
    pb.items = pb.prods = nullptr;
    pb.ctr = nullptr;
    pb.nitems = 0;
}

}  // namespace spg
