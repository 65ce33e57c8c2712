// Numeric phase kernels: one launch per non-empty column bin.
#include "numeric.hpp"

namespace spg {

// Up to 64*EMAX terms per column: one wave per column, four columns per
// workgroup, 64*EMAX LDS slots per wave for merging equal rows.  EMAX = 4
// (tiny columns up to 256 products, the default) keeps the register file
// small enough for four waves per SIMD.
template <typename V, int EMAX, bool kPacked>
__global__ __launch_bounds__(256) void k_num_tiny(const int32_t *__restrict__ list, int count,
                                                  NumArgs<V> a) {
    __shared__ int s_rows[4][EMAX * kWave];
    __shared__ Acc s_vals[4][EMAX * kWave];
    const int wv = threadIdx.x >> 6;
    const int w = blockIdx.x * 4 + wv;
    if (w >= count) return;
    // a NULL list: every column of B_i is in this bin, column w is the w-th
    num_wave_dispatch<V, EMAX, kPacked>(a, list ? list[w] : w, s_rows[wv], s_vals[wv]);
}

template <typename V, int EMAX>
static void num_tiny_launch(const Plan &p, const int32_t *list, const NumArgs<V> &a) {
    const int cnt = p.num_count[kBinTiny];
    if (cnt == p.n) list = nullptr;  // the bin holds every column: skip the indirection
    const dim3 grid((cnt + 3) / 4);
    if (p.m < kPackedRowLimit)
        hipLaunchKernelGGL((k_num_tiny<V, EMAX, true>), grid, dim3(256), 0, p.stream, list, cnt,
                           a);
    else
        hipLaunchKernelGGL((k_num_tiny<V, EMAX, false>), grid, dim3(256), 0, p.stream, list, cnt,
                           a);
}

template <int T, int G, typename V>
__global__ __launch_bounds__(G < 256 ? 256 : G) void k_num_hash(const int32_t *__restrict__ list,
                                                                int count, NumArgs<V> a) {
    constexpr int CPW = G < 256 ? 256 / G : 1;
    __shared__ NumHashLds<T, G, V> lds[CPW];
    const int grp = threadIdx.x / G, gt = threadIdx.x % G;
    const int w = blockIdx.x * CPW + grp;
    if (w >= count) return;  // CPW > 1 only when a group sits inside one wave
    num_hash_column<T, G, V>(a, list[w], lds[grp], gt);
}

template <typename V>
__global__ __launch_bounds__(kDenseThreads) void k_num_dense(
    const int32_t *__restrict__ first, int nfirst, const int32_t *__restrict__ list, int count,
    NumArgs<V> a, int VC, DevCounters *__restrict__ ctr) {
    unsigned int *queue = ctr->num_dense_queue;
    extern __shared__ __align__(16) unsigned char s_dyn[];
    __shared__ NumDenseStatic<kDenseThreads, V> S;
    __shared__ int s_item;
    // the bitmap of one band: all m rows, or kMaxDenseRows of a taller column
    const int nw = (int)((min<int64_t>(a.m, kMaxDenseRows) + 31) >> 5);
    uint32_t *bits = reinterpret_cast<uint32_t *>(s_dyn);
    uint16_t *wpre = reinterpret_cast<uint16_t *>(bits + nw);
    Acc *vals = reinterpret_cast<Acc *>(s_dyn + (((size_t)nw * 6 + 15) & ~(size_t)15));
    // the columns with the most products (list `first`) go out first
    for (int w = queue_take(queue, &s_item); w < nfirst + count; w = queue_take(queue, &s_item))
        num_dense_column<kDenseThreads, V>(a, w < nfirst ? first[w] : list[w - nfirst], bits,
                                           wpre, vals, VC, S);
    queue_leave(queue);
}

// The order in which k_dense_rows takes the kept bitmaps: by descending
// number of rows (eight buckets per power of two), so the waves of its
// grid-stride loop get about equal shares (the columns of a power-law
// product differ by orders of magnitude, and in list order the large ones
// cluster).  One workgroup; order[i] is a position in the dense list.  Each
// wave counts, and later places, its own items (thread t takes positions t,
// t + 1024, ...) in a histogram of its own, so LDS atomics only meet inside
// a wave; the positions' columns and row counts are loaded kOrderBatch at a
// time, so their loads are in flight together.
constexpr int kOrderBuckets = 256;
constexpr int kOrderThreads = 1024;
constexpr int kOrderBatch = 8;
__global__ __launch_bounds__(kOrderThreads) void k_dense_order(int count,
                                                               const int32_t *__restrict__ list,
                                                               const int64_t *__restrict__ Ccolptr,
                                                               int32_t *__restrict__ order) {
    constexpr int NW = kOrderThreads / kWave;
    __shared__ int s_h[NW][kOrderBuckets];
    const int tid = threadIdx.x, wv = tid / kWave;
    for (int i = tid; i < NW * kOrderBuckets; i += kOrderThreads) (&s_h[0][0])[i] = 0;
    __syncthreads();
    // buckets of this thread's positions w0 + u * kOrderThreads (-1 past count)
    auto buckets = [&](int w0, int (&bk)[kOrderBatch]) {
        int32_t j[kOrderBatch];
#pragma unroll
        for (int u = 0; u < kOrderBatch; ++u) j[u] = list[min(w0 + u * kOrderThreads, count - 1)];
        long long a[kOrderBatch], z[kOrderBatch];
#pragma unroll
        for (int u = 0; u < kOrderBatch; ++u) {
            a[u] = Ccolptr[j[u]];
            z[u] = Ccolptr[j[u] + 1];
        }
#pragma unroll
        for (int u = 0; u < kOrderBatch; ++u) {
            const long long nz = z[u] - a[u];
            int b = kOrderBuckets - 1;
            if (nz > 1) {
                const int lg = 63 - __clzll((unsigned long long)nz);
                const int frac = (int)((lg >= 3 ? nz >> (lg - 3) : nz << (3 - lg)) & 7);
                b = max(0, kOrderBuckets - 1 - (lg * 8 + frac));  // more rows: lower bucket
            }
            bk[u] = w0 + u * kOrderThreads < count ? b : -1;
        }
    };
    constexpr int kStep = kOrderBatch * kOrderThreads;
    for (int w0 = tid; w0 < count; w0 += kStep) {
        int bk[kOrderBatch];
        buckets(w0, bk);
#pragma unroll
        for (int u = 0; u < kOrderBatch; ++u)
            if (bk[u] >= 0) atomicAdd(&s_h[wv][bk[u]], 1);
    }
    __syncthreads();
    // bucket-major, wave-minor exclusive scan: thread b < 256 holds bucket b
    __shared__ int s_tot[kOrderBuckets];
    if (tid < kOrderBuckets) {
        int run = 0;
        for (int v = 0; v < NW; ++v) {
            const int c = s_h[v][tid];
            s_h[v][tid] = run;
            run += c;
        }
        s_tot[tid] = run;
    }
    __syncthreads();
    if (tid == 0) {
        int run = 0;
        for (int b = 0; b < kOrderBuckets; ++b) {
            const int c = s_tot[b];
            s_tot[b] = run;
            run += c;
        }
    }
    __syncthreads();
    if (tid < kOrderBuckets)
        for (int v = 0; v < NW; ++v) s_h[v][tid] += s_tot[tid];
    __syncthreads();
    for (int w0 = tid; w0 < count; w0 += kStep) {
        int bk[kOrderBatch];
        buckets(w0, bk);
#pragma unroll
        for (int u = 0; u < kOrderBatch; ++u)
            if (bk[u] >= 0) order[atomicAdd(&s_h[wv][bk[u]], 1)] = w0 + u * kOrderThreads;
    }
}

// Row ids of the dense columns whose row bitmaps the symbolic phase kept,
// one column per wave with no workgroup barrier: the wave streams the
// column's bitmap 64 words at a time (a word per lane, kRowAhead rounds of
// loads in flight), places each round's set rows by a wave scan of the bit
// counts in its own LDS stage and writes them out coalesced, the running
// count giving the next round's first position.  The stage holds kRowStage
// rows (a round of 64 words with more set bits is placed in two halves of
// 32 words), so eight waves fit per SIMD.  Columns whose values went to a
// hash bin are skipped.  The kernel is bound by the issue of its vector
// instructions (measured: about 99 % of the SIMDs' issue cycles), so its
// loops keep their address arithmetic to a minimum.
constexpr int kRowThreads = 256;
constexpr int kRowWaves = kRowThreads / kWave;
constexpr int kRowAhead = 4;
constexpr int kRowStage = 32 * 32;  // the set bits of 32 words
__global__ __launch_bounds__(kRowThreads) void k_dense_rows(
    int count, const int32_t *__restrict__ list, const int32_t *__restrict__ order,
    const int32_t *__restrict__ num_bin, int nw, const uint32_t *__restrict__ bits,
    const int64_t *__restrict__ Ccolptr, int32_t *__restrict__ Crow) {
    __shared__ int32_t stage[kRowWaves][kRowStage];
    const int wv = threadIdx.x / kWave, lane = lane_id();
    int32_t *my = stage[wv];
    // places the set rows of `word` (word index wi, lanes' words in order)
    // at base; incl is the wave's inclusive scan of the words' bit counts and
    // n its total (wave-uniform)
    auto place = [&](uint32_t word, int wi, long long base, int incl, int n) {
        // a plain (unswizzled) stage: the kernel is bound by its vector
        // instruction count, and the address arithmetic of a swizzle cost
        // more than the bank conflicts of dense rounds
        const int wrow = (wi << 5) - 1;
        int32_t *dst = my + (incl - __popc(word));
        while (word) {
            *dst++ = wrow + __ffs(word);
            word &= word - 1;
        }
        wave_sync();
        // up to four LDS reads in flight before their stores (only the
        // reads some lane needs)
        for (int i0 = 0; i0 < n; i0 += 4 * kWave) {
            int32_t v[4] = {0, 0, 0, 0};
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int i = min(i0 + u * kWave + lane, n - 1);
                if (i0 + u * kWave < n) v[u] = my[i];
            }
            int32_t *out = Crow + base + i0 + lane;
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (i0 + u * kWave + lane < n) out[u * kWave] = v[u];
        }
        wave_sync();
    };
    for (int i = blockIdx.x * kRowWaves + wv; i < count; i += gridDim.x * kRowWaves) {
        const int w = order[i];
        const int32_t j = list[w];
        if (num_bin[j] < kBinDense) continue;  // the same for the whole wave
        long long base = Ccolptr[j];
        const uint32_t *src = bits + (size_t)w * nw;
        // kRowAhead rounds of words per step, the next step's words loaded
        // while this step's are expanded (loads without branches: past the
        // end the last word again, masked; the copies into `cur` come after
        // the work, so the wait for those loads does too)
        uint32_t cur[kRowAhead];
#pragma unroll
        for (int d = 0; d < kRowAhead; ++d) cur[d] = src[min(d * kWave + lane, nw - 1)];
        for (int s0 = 0; s0 < nw; s0 += kRowAhead * kWave) {
            uint32_t nxt[kRowAhead];
#pragma unroll
            for (int d = 0; d < kRowAhead; ++d)
                nxt[d] = src[min(s0 + (kRowAhead + d) * kWave + lane, nw - 1)];
#pragma unroll
            for (int d = 0; d < kRowAhead; ++d) {
                const int wi = s0 + d * kWave + lane;
                const uint32_t word = wi < nw ? cur[d] : 0u;
                const int incl = wave_incl_scan(__popc(word));
                const int total = wave_last(incl);
                if (total <= kRowStage) {
                    place(word, wi, base, incl, total);
                    base += total;
                } else {  // each half's 32 words hold at most kRowStage bits
                    const uint32_t lo = lane < 32 ? word : 0u, hi = lane < 32 ? 0u : word;
                    const int il = wave_incl_scan(__popc(lo));
                    const int nl = wave_last(il);
                    place(lo, wi, base, il, nl);
                    base += nl;
                    const int ih = wave_incl_scan(__popc(hi));
                    const int nh = wave_last(ih);
                    place(hi, wi, base, ih, nh);
                    base += nh;
                }
            }
#pragma unroll
            for (int d = 0; d < kRowAhead; ++d) cur[d] = nxt[d];
        }
    }
}

template <int G, typename V>
__global__ __launch_bounds__(G) void k_num_bitmap(const int32_t *__restrict__ list, int count,
                                                  NumArgs<V> a, int vcap) {
    extern __shared__ __align__(16) unsigned char s_dyn[];
    __shared__ NumBitmapStatic<G, V> S;
    if ((int)blockIdx.x >= count) return;
    const int nw = (int)((a.m + 31) >> 5);
    uint32_t *bits = reinterpret_cast<uint32_t *>(s_dyn);
    uint16_t *wpre = reinterpret_cast<uint16_t *>(bits + nw);
    Acc *vals = reinterpret_cast<Acc *>(s_dyn + (((size_t)nw * 6 + 15) & ~(size_t)15));
    num_bitmap_column<G, V>(a, list[blockIdx.x], bits, wpre, vals, vcap, S);
}

// Dynamic LDS of the dense kernel and the number of values one rank window
// holds: whatever the device's per-workgroup LDS leaves after the bitmap,
// the word ranks and the kernel's static part.
size_t dense_lds_bytes(int64_t m, size_t vsize, int lds_max, int *VC_out) {
    const size_t nw = (size_t)((m + 31) / 32);
    const size_t head = (nw * 6 + 15) & ~(size_t)15;
    const size_t stat = vsize == 8 ? sizeof(NumDenseStatic<kDenseThreads, double>)
                                   : sizeof(NumDenseStatic<kDenseThreads, float>);
    const size_t budget = (size_t)lds_max > stat + 1024 ? (size_t)lds_max - stat - 1024 : 0;
    const size_t vc_bytes = budget > head ? budget - head : 0;
    // a multiple of 16: the window's slots are swizzled in rows of 16
    const int VC = (int)std::max<size_t>(16, std::min<size_t>(vc_bytes / vsize, 1 << 20) & ~(size_t)15);
    *VC_out = VC;
    return head + (size_t)VC * vsize;
}

constexpr int64_t kBitmapWideRows = 65536;
constexpr int kBitmapWideThreads = 512;

template <int T, int G, typename V>
static int num_hash_launch(Plan &p, int bin, const NumArgs<V> &a) {
    const int cnt = p.num_count[bin];
    if (cnt <= 0) return SPGEMM_OK;
    size_t lds;
    if (medium_uses_bitmap(p.m, T, p.tun.medium_kernel, sizeof(Acc), &lds)) {
        // a bitmap of more than 65536 rows takes so much LDS that two
        // workgroups fill a CU: 512 threads each then keep 16 waves resident
        // (R-MAT 18: numeric 15.95 -> 15.4 ms; 1024 threads leave one
        // workgroup per CU and are slower)
        constexpr int GB = T <= 512 ? 128 : 256;
        if (p.m > kBitmapWideRows) {
            hipLaunchKernelGGL((k_num_bitmap<kBitmapWideThreads, V>), dim3(cnt),
                               dim3(kBitmapWideThreads), lds, p.stream,
                               p.num_list + (int64_t)bin * p.n, cnt, a, T / 2);
            SPG_LAUNCHED("k_num_bitmap<" + std::to_string(kBitmapWideThreads) + ">");
            return SPGEMM_OK;
        }
        hipLaunchKernelGGL((k_num_bitmap<GB, V>), dim3(cnt), dim3(GB), lds, p.stream,
                           p.num_list + (int64_t)bin * p.n, cnt, a, T / 2);
        SPG_LAUNCHED("k_num_bitmap<" + std::to_string(GB) + ">");
        return SPGEMM_OK;
    }
    constexpr int CPW = G < 256 ? 256 / G : 1;
    constexpr int threads = G < 256 ? 256 : G;
    const unsigned grid = (unsigned)((cnt + CPW - 1) / CPW);
    hipLaunchKernelGGL((k_num_hash<T, G, V>), dim3(grid), dim3(threads), 0, p.stream,
                       p.num_list + (int64_t)bin * p.n, cnt, a);
    SPG_LAUNCHED("k_num_hash<" + std::to_string(T) + ">");
    return SPGEMM_OK;
}

template <typename V>
static int numeric_bins_t(Plan &p, const V *Bvals, int32_t *Crow, V *Cval, const V *Atv) {
    NumArgs<V> a{p.m,         p.Bcolptr, p.term_range(), Bvals,  p.At_rowidx, Atv,
                 p.C_colptr,  Crow,      Cval,           p.flop, p.Browidx,   p.split,
                 p.col_slot,  p.dense_bits, p.tiny_perm, p.nblk};
    const int64_t n = p.n;
    auto list = [&](int bin) { return p.num_list + (int64_t)bin * n; };
    if (p.num_count[kBinTiny] > 0)
    {
        if (p.th.tiny_max_flop <= 4 * kWave)
            num_tiny_launch<V, 4>(p, list(kBinTiny), a);
        else
            num_tiny_launch<V, 8>(p, list(kBinTiny), a);
        SPG_LAUNCHED("k_num_tiny");
    }
    int rc;
    if ((rc = num_hash_launch<kNumTable[0], kNumTable[0] / 8, V>(p, kBinH0, a))) return rc;
    if ((rc = num_hash_launch<kNumTable[1], kNumTable[1] / 8, V>(p, kBinH1, a))) return rc;
    if ((rc = num_hash_launch<kNumTable[2], kNumTable[2] / 8, V>(p, kBinH2, a))) return rc;
    if ((rc = num_hash_launch<kNumTable[3], kNumTable[3] / 8, V>(p, kBinH3, a))) return rc;
    const int ndense = p.num_count[kBinDense] + p.num_count[kBinDenseFirst];
    if (ndense > 0) {
        int VC;  // a column of more than kMaxDenseRows rows is done in bands
        size_t lds = dense_lds_bytes(std::min<int64_t>(p.m, kMaxDenseRows), sizeof(Acc),
                                     p.lds_max, &VC);
        if (p.tun.dense_window > 0 && p.tun.dense_window < VC) {
            lds -= (size_t)(VC - p.tun.dense_window) * sizeof(Acc);
            VC = p.tun.dense_window;
        }
        if (p.dense_bits && p.sym_count[kBinDense] > 0) {
            const int nw = (int)((p.m + 31) / 32);
            const unsigned rg = resident_groups((const void *)k_dense_rows, kRowThreads, 0,
                                                p.device,
                                                (p.sym_count[kBinDense] + kRowWaves - 1) /
                                                    kRowWaves);
            // the order goes to the symbolic lists' dense-first slice, which
            // the symbolic phase never fills
            int32_t *order = p.sym_list + (int64_t)kBinDenseFirst * n;
            hipLaunchKernelGGL(k_dense_order, dim3(1), dim3(kOrderThreads), 0, p.stream,
                               p.sym_count[kBinDense], p.sym_list + (int64_t)kBinDense * n,
                               p.C_colptr, order);
            SPG_LAUNCHED("k_dense_order");
            hipLaunchKernelGGL(k_dense_rows, dim3(rg), dim3(kRowThreads), 0, p.stream,
                               p.sym_count[kBinDense], p.sym_list + (int64_t)kBinDense * n, order,
                               p.num_bin, nw, p.dense_bits, p.C_colptr, Crow);
            SPG_LAUNCHED("k_dense_rows");
        }
        const unsigned grid = resident_groups((const void *)k_num_dense<V>, kDenseThreads, lds,
                                              p.device, ndense);
        hipLaunchKernelGGL(k_num_dense<V>, dim3(grid), dim3(kDenseThreads), lds, p.stream,
                           list(kBinDenseFirst), p.num_count[kBinDenseFirst], list(kBinDense),
                           p.num_count[kBinDense], a, VC, p.ctr);
        SPG_LAUNCHED("k_num_dense (" + std::to_string(grid) + " workgroups, dynamic LDS " +
                     std::to_string(lds) + " B)");
    }
    SPG_HIP(hipGetLastError());
    return SPGEMM_OK;
}

int launch_numeric_bins(Plan &p, const void *Bvals, int32_t *Crow, void *Cvals,
                        const void *At_vals) {
    if (p.n == 0 || p.nnzC == 0) return SPGEMM_OK;
    const void *Atv = At_vals ? At_vals : p.At_vals;
    if (p.dtype == SPGEMM_F64)
        return numeric_bins_t<double>(p, (const double *)Bvals, Crow, (double *)Cvals,
                                      (const double *)Atv);
    return numeric_bins_t<float>(p, (const float *)Bvals, Crow, (float *)Cvals,
                                 (const float *)Atv);
}

}  // namespace spg
