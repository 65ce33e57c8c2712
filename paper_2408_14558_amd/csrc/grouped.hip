// Grouped numeric launches of the batched form (grouped.hpp): one launch per
// numeric bin and kernel over the grouped products of a dependency depth.
// Entry w of a launch's column table (built once, from the members' bin
// lists) names the member and its column, so a wave reaches its column with
// one load; the column is computed by the routine of the plain kernel
// (tiny: one wave; medium bins: the LDS hash of the bin's table, or the LDS
// bitmap over the member's m rows, as its plain numeric phase chooses).
#include <algorithm>
#include <cstring>
#include <string>

#include "grouped.hpp"
#include "numeric.hpp"

namespace spg {

template <typename V>
struct GProd {
    NumArgs<V> a;
    int32_t packed;                 // tiny columns sort packed keys (m below kPackedRowLimit)
    int32_t pad;
};

// A column table entry: the member's slot in the table of GProd (high 32
// bits) and the column of B_i (low 32 bits).
__device__ __forceinline__ int col_member(uint64_t e) { return (int)(e >> 32); }
__device__ __forceinline__ int32_t col_index(uint64_t e) { return (int32_t)(uint32_t)e; }

template <typename V>
__global__ __launch_bounds__(256) void k_num_tiny_grouped(const GProd<V> *__restrict__ prods,
                                                          const uint64_t *__restrict__ cols,
                                                          int total) {
    __shared__ int s_rows[4][4 * kWave];
    __shared__ Acc s_vals[4][4 * kWave];
    const int wv = threadIdx.x >> 6;
    const int w = blockIdx.x * 4 + wv;
    if (w >= total) return;  // the whole wave
    const uint64_t e = cols[w];
    // the member's arguments copied once (the same for the whole wave), so
    // the column routine keeps them in scalar registers instead of reading
    // them from the table at every use
    const NumArgs<V> a = prods[col_member(e)].a;
    if (prods[col_member(e)].packed)
        num_wave_dispatch<V, 4, true>(a, col_index(e), s_rows[wv], s_vals[wv]);
    else
        num_wave_dispatch<V, 4, false>(a, col_index(e), s_rows[wv], s_vals[wv]);
}

template <int T, int G, typename V>
__global__ __launch_bounds__(G < 256 ? 256 : G) void k_num_hash_grouped(
    const GProd<V> *__restrict__ prods, const uint64_t *__restrict__ cols, int total) {
    constexpr int CPW = G < 256 ? 256 / G : 1;
    __shared__ NumHashLds<T, G, V> lds[CPW];
    const int grp = threadIdx.x / G, gt = threadIdx.x % G;
    const int w = blockIdx.x * CPW + grp;
    if (w >= total) return;  // CPW > 1 only when a group sits inside one wave
    const uint64_t e = cols[w];
    const NumArgs<V> a = prods[col_member(e)].a;  // copied once (see k_num_tiny_grouped)
    num_hash_column<T, G, V>(a, col_index(e), lds[grp], gt);
}

// One column per workgroup; the dynamic LDS holds the largest member's
// bitmap, and each column lays out its own member's m rows in it.
template <int G, typename V>
__global__ __launch_bounds__(G) void k_num_bitmap_grouped(const GProd<V> *__restrict__ prods,
                                                          const uint64_t *__restrict__ cols,
                                                          int total, int vcap) {
    extern __shared__ __align__(16) unsigned char s_dyn[];
    __shared__ NumBitmapStatic<G, V> S;
    if ((int)blockIdx.x >= total) return;
    const uint64_t e = cols[blockIdx.x];
    const NumArgs<V> a = prods[col_member(e)].a;  // copied once (see k_num_tiny_grouped)
    const int nw = (int)((a.m + 31) >> 5);
    uint32_t *bits = reinterpret_cast<uint32_t *>(s_dyn);
    uint16_t *wpre = reinterpret_cast<uint16_t *>(bits + nw);
    Acc *vals = reinterpret_cast<Acc *>(s_dyn + (((size_t)nw * 6 + 15) & ~(size_t)15));
    num_bitmap_column<G, V>(a, col_index(e), bits, wpre, vals, vcap, S);
}

bool groupable(const Plan &p) {
    return p.n <= kGroupMaxCols && p.num_count[kBinDense] + p.num_count[kBinDenseFirst] == 0 &&
           p.th.tiny_max_flop <= 4 * kWave;
}

template <typename V>
static int build_t(const std::vector<Plan *> &plans, const std::vector<spgemm_batch_io> &io,
                   GroupedDepth &g) {
    const int np = (int)g.members.size();
    std::vector<GProd<V>> prods(np);
    for (int i = 0; i < np; ++i) {
        const int t = g.members[i];
        const Plan &p = *plans[t];
        GProd<V> &P = prods[i];
        std::memset(&P, 0, sizeof(P));
        const V *Bv = (const V *)(io[t].B_vals ? io[t].B_vals : p.Bvals);
        // new A values read in place when A~ holds all of A, else gathered
        // into A~ before the launch (take_new_a_values)
        const bool in_place = io[t].A_vals && p.nnzAt_pub == p.nnzA;
        const V *Atv = (const V *)(in_place ? io[t].A_vals : p.At_vals);
        P.a = NumArgs<V>{p.m,        p.Bcolptr,    p.term_range(), Bv,        p.At_rowidx,
                         Atv,                      p.C_colptr,     io[t].C_rowidx,
                         (V *)io[t].C_vals,        p.flop,         p.Browidx, p.split,
                         p.col_slot, p.dense_bits, p.tiny_perm, p.nblk};
        P.packed = p.m < kPackedRowLimit;
    }
    // the launches: tiny, then per medium bin the hash and the bitmap kernel
    // (a member's columns of a medium bin go to the kernel its plain phase
    // uses); each launch's column table lists its members' columns in order
    // every member's numeric bin lists, one copy per member (kNumBins x n)
    std::vector<std::vector<int32_t>> lists(np);
    for (int i = 0; i < np; ++i) {
        const Plan &p = *plans[g.members[i]];
        lists[i].resize((size_t)kNumBins * (size_t)p.n);
        SPG_HIP(hipMemcpy(lists[i].data(), p.num_list, sizeof(int32_t) * lists[i].size(),
                          hipMemcpyDeviceToHost));
    }
    std::vector<uint64_t> cols;
    auto add = [&](int kind, int bin, const std::vector<int> &who, size_t lds) {
        GroupedLaunch L;
        L.kind = kind;
        L.bin = bin;
        L.np = (int)who.size();
        L.lds = lds;
        L.offset = cols.size();
        for (int i : who) {
            const Plan &p = *plans[g.members[i]];
            const int64_t c = p.num_count[bin];
            const int32_t *list = lists[i].data() + (size_t)bin * (size_t)p.n;
            for (int64_t q = 0; q < c; ++q)
                cols.push_back(((uint64_t)(uint32_t)i << 32) | (uint32_t)list[q]);
            L.total += c;
        }
        if (L.total >= INT32_MAX) return fail(SPGEMM_EUNSUPPORTED, "too many grouped columns");
        if (L.total > 0) g.launches.push_back(L);
        return SPGEMM_OK;
    };
    auto with_columns = [&](int bin) {
        std::vector<int> who;
        for (int i = 0; i < np; ++i)
            if (plans[g.members[i]]->num_count[bin] > 0) who.push_back(i);
        return who;
    };
    if (int rc = add(0, kBinTiny, with_columns(kBinTiny), 0)) return rc;
    for (int b = kBinH0; b <= kBinH3; ++b) {
        std::vector<int> hash, bitmap;
        size_t lds_max = 0;
        int64_t m_max = 0;
        for (int i : with_columns(b)) {
            const Plan &p = *plans[g.members[i]];
            size_t lds = 0;
            if (medium_uses_bitmap(p.m, kNumTable[b - kBinH0], p.tun.medium_kernel, sizeof(Acc),
                                   &lds)) {
                bitmap.push_back(i);
                lds_max = std::max(lds_max, lds);
                m_max = std::max(m_max, p.m);
            } else {
                hash.push_back(i);
            }
        }
        if (int rc = add(1, b, hash, 0)) return rc;
        if (int rc = add(2, b, bitmap, lds_max)) return rc;
        if (!bitmap.empty()) g.launches.back().wide = m_max > 65536;
    }
    const size_t pbytes = sizeof(GProd<V>) * (size_t)np;
    const size_t off = (pbytes + 255) & ~(size_t)255;
    const size_t cbytes = sizeof(uint64_t) * cols.size();
    SPG_HIP(hipMalloc(&g.table, off + std::max<size_t>(cbytes, 8)));
    SPG_HIP(hipMemcpy(g.table, prods.data(), pbytes, hipMemcpyHostToDevice));
    if (cbytes)
        SPG_HIP(hipMemcpy((char *)g.table + off, cols.data(), cbytes, hipMemcpyHostToDevice));
    for (GroupedLaunch &L : g.launches) L.offset = off + sizeof(uint64_t) * L.offset;
    return SPGEMM_OK;
}

int grouped_build(const std::vector<Plan *> &plans, const std::vector<spgemm_batch_io> &io,
                  const std::vector<int> &members, GroupedDepth &g) {
    g.members = members;
    g.launches.clear();
    g.dtype = members.empty() ? SPGEMM_F64 : plans[members[0]]->dtype;
    if (members.empty()) return SPGEMM_OK;
    const int rc = g.dtype == SPGEMM_F64 ? build_t<double>(plans, io, g)
                                         : build_t<float>(plans, io, g);
    if (rc) grouped_free(g);
    return rc;
}

template <int T, int G, typename V>
static int hash_launch(const GroupedDepth &g, const GroupedLaunch &L, hipStream_t s) {
    constexpr int CPW = G < 256 ? 256 / G : 1;
    constexpr int threads = G < 256 ? 256 : G;
    const uint64_t *cols = (const uint64_t *)((const char *)g.table + L.offset);
    hipLaunchKernelGGL((k_num_hash_grouped<T, G, V>), dim3((unsigned)((L.total + CPW - 1) / CPW)),
                       dim3(threads), 0, s, (const GProd<V> *)g.table, cols, (int)L.total);
    SPG_LAUNCHED("k_num_hash_grouped<" + std::to_string(T) + "> (" + std::to_string(L.np) +
                 " products, " + std::to_string(L.total) + " columns)");
    return SPGEMM_OK;
}

template <int T, typename V>
static int bitmap_launch(const GroupedDepth &g, const GroupedLaunch &L, hipStream_t s) {
    // as the plain bitmap kernel: 512 threads for bitmaps of more than
    // 65536 rows
    constexpr int GB = T <= 512 ? 128 : 256;
    const uint64_t *cols = (const uint64_t *)((const char *)g.table + L.offset);
    if (L.wide)
        hipLaunchKernelGGL((k_num_bitmap_grouped<512, V>), dim3((unsigned)L.total), dim3(512),
                           L.lds, s, (const GProd<V> *)g.table, cols, (int)L.total, T / 2);
    else
        hipLaunchKernelGGL((k_num_bitmap_grouped<GB, V>), dim3((unsigned)L.total), dim3(GB),
                           L.lds, s, (const GProd<V> *)g.table, cols, (int)L.total, T / 2);
    SPG_LAUNCHED("k_num_bitmap_grouped (" + std::to_string(L.np) + " products, " +
                 std::to_string(L.total) + " columns)");
    return SPGEMM_OK;
}

template <typename V>
static int medium_launch(const GroupedDepth &g, const GroupedLaunch &L, hipStream_t s) {
    constexpr int T0 = kNumTable[0], T1 = kNumTable[1], T2 = kNumTable[2], T3 = kNumTable[3];
    const bool bm = L.kind == 2;
    switch (L.bin) {  // the plain path's table and group size per bin
    case kBinH0: return bm ? bitmap_launch<T0, V>(g, L, s) : hash_launch<T0, T0 / 8, V>(g, L, s);
    case kBinH1: return bm ? bitmap_launch<T1, V>(g, L, s) : hash_launch<T1, T1 / 8, V>(g, L, s);
    case kBinH2: return bm ? bitmap_launch<T2, V>(g, L, s) : hash_launch<T2, T2 / 8, V>(g, L, s);
    default: return bm ? bitmap_launch<T3, V>(g, L, s) : hash_launch<T3, T3 / 8, V>(g, L, s);
    }
}

template <typename V>
static int launch_t(const GroupedDepth &g, const std::vector<hipStream_t> &streams) {
    for (size_t k = 0; k < g.launches.size(); ++k) {
        const GroupedLaunch &L = g.launches[k];
        const hipStream_t s = streams[k % streams.size()];
        if (L.kind == 0) {
            const uint64_t *cols = (const uint64_t *)((const char *)g.table + L.offset);
            hipLaunchKernelGGL(k_num_tiny_grouped<V>, dim3((unsigned)((L.total + 3) / 4)),
                               dim3(256), 0, s, (const GProd<V> *)g.table, cols, (int)L.total);
            SPG_LAUNCHED("k_num_tiny_grouped (" + std::to_string(L.np) + " products, " +
                         std::to_string(L.total) + " columns)");
        } else if (int rc = medium_launch<V>(g, L, s)) {
            return rc;
        }
    }
    return SPGEMM_OK;
}

int grouped_launch(const GroupedDepth &g, const std::vector<hipStream_t> &streams) {
    if (g.launches.empty() || streams.empty()) return SPGEMM_OK;
    return g.dtype == SPGEMM_F64 ? launch_t<double>(g, streams) : launch_t<float>(g, streams);
}

void grouped_free(GroupedDepth &g) {
    if (g.table) (void)hipFree(g.table);
    g.table = nullptr;
    g.launches.clear();
}

}  // namespace spg
