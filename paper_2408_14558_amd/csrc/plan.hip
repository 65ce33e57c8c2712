// Plan-phase kernels: the gather half of the sparsity-aware 1D algorithm
// (Alg. 1: H_i, the required columns, Alg. 2's block grouping, the fetch of
// the chosen blocks and the compacted A~).  On one GPU the one-sided fetch
// of a remote block becomes a device copy of a contiguous range of A's CSC
// arrays.
#include "gather.hpp"

namespace spg {

// Clears H, the group tables, the scan states, the counters, the flops and
// arrival counts of the flops pass, and copies
// the host-written group bases and rank tiles from pinned host memory
// (up_src) to the device (up_dst), in place of a separate copy.
__global__ void k_plan_init(uint8_t *__restrict__ H, int64_t k, uint8_t *__restrict__ hit,
                            int32_t *__restrict__ gfirst, int32_t *__restrict__ glast, int64_t G,
                            uint64_t *__restrict__ status, int64_t nstatus,
                            DevCounters *__restrict__ ctr, int64_t *__restrict__ At_colptr,
                            const uint64_t *__restrict__ up_src, uint64_t *__restrict__ up_dst,
                            int64_t up_words, int64_t *__restrict__ flop,
                            int32_t *__restrict__ arrive, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t i = t0; i < up_words; i += stride) up_dst[i] = up_src[i];
    for (int64_t j = t0; j < n; j += stride) {
        flop[j] = 0;
        arrive[j] = 0;
    }
    for (int64_t i = t0; i < k; i += stride) H[i] = 0;
    for (int64_t g = t0; g < G; g += stride) {
        hit[g] = 0;
        gfirst[g] = -1;
        glast[g] = -1;
    }
    for (int64_t s = t0; s < nstatus; s += stride) status[s] = 0;
    int *w = reinterpret_cast<int *>(ctr);
    for (int64_t i = t0; i < (int64_t)(sizeof(DevCounters) / sizeof(int)); i += stride) w[i] = 0;
    if (t0 == 0) {
        At_colptr[0] = 0;
    }
}

// H_i: every row of B_i holding a stored entry (notation table; Alg. 1).
__global__ void k_mark_rows(const int32_t *__restrict__ Browidx, int64_t nnzB,
                            uint8_t *__restrict__ H) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nnzB; q += stride)
        H[Browidx[q]] = 1;
}

// Rank of every nonzero column among the nonzero columns of its partition
// (a scan segmented at partition starts), its Alg. 2 group
// g = group_base[part] + rank / b, and the group's hit flag (any column of
// the group named by H; every group of partition own_whole when that
// partition is the caller's own and is taken whole).  Also records each
// group's first and last column and counts |H|, nzc and the number of
// groups K.
__global__ __launch_bounds__(kScanThreads) void k_rank_groups(
    const int64_t *__restrict__ Acolptr, const uint8_t *__restrict__ H,
    const RankTile *__restrict__ tiles, const int64_t *__restrict__ group_base, int64_t b,
    int32_t *__restrict__ gid, uint8_t *__restrict__ hit, int32_t *__restrict__ gfirst,
    int32_t *__restrict__ glast, uint64_t *__restrict__ status, int32_t own_whole,
    DevCounters *__restrict__ ctr) {
    __shared__ long long s_ticket;
    __shared__ int s_tmp[kScanThreads / kWave + 1];
    __shared__ long long s_prefix;
    const long long t = take_ticket(&ctr->tickets[kTkRank], &s_ticket);
    const RankTile d = tiles[t];
    const int tid = threadIdx.x;
    // every item loads (past the tile's end: its last column again, not
    // counted), so the loads carry no branches and are in flight together
    int64_t a0[kScanItems], a1[kScanItems];
    int hh[kScanItems];
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const int64_t c = d.col0 + min(tid * kScanItems + i, d.ncols - 1);
        a0[i] = Acolptr[c];
        a1[i] = Acolptr[c + 1];
        hh[i] = H[c];
    }
    int nz[kScanItems];
    int cnt = 0, hcnt = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const bool in = tid * kScanItems + i < d.ncols;
        nz[i] = in && a1[i] > a0[i] ? 1 : 0;
        hcnt += in ? hh[i] : 0;
        cnt += nz[i];
    }
    int total;
    int excl = group_excl_scan<kScanThreads>(cnt, s_tmp, &total);
    if (tid < kWave) {
        const long long pre = chained_prefix(status, t, d.head != 0, total);
        if (tid == 0) s_prefix = pre;
    }
    __syncthreads();
    long long rank = s_prefix + excl;
    const long long part_last = d.last ? s_prefix + total - 1 : -1;
    const int64_t base = group_base[d.part];
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const int off = tid * kScanItems + i;
        if (off >= d.ncols) break;
        const int64_t c = d.col0 + off;
        if (nz[i]) {
            const int64_t g = base + rank / b;
            gid[c] = (int32_t)g;
            if (hh[i] || d.part == own_whole) hit[g] = 1;
            const long long r = rank % b;
            if (r == 0) gfirst[g] = (int32_t)c;
            if (r == b - 1 || rank == part_last) glast[g] = (int32_t)c;
            ++rank;
        } else {
            gid[c] = -1;
        }
    }
    // one atomic per tile and counter: thousands of workgroups' atomics on
    // one address queue behind each other
    const int hsum = wave_sum(hcnt);
    if (lane_id() == 0) s_tmp[tid / kWave] = hsum;
    __syncthreads();
    if (tid == 0) {
        int h = 0;
        for (int w = 0; w < kScanThreads / kWave; ++w) h += s_tmp[w];
        if (h) atomic_add_i64(&ctr->h_count, (long long)h);
        atomic_add_i64(&ctr->nzc, (long long)total);
        if (d.last) {
            const long long nzc_part = s_prefix + total;
            atomic_add_i64(&ctr->K, (nzc_part + b - 1) / b);
        }
    }
}

// Selection (column lies in a chosen group) and the map into A~: an
// exclusive scan of the selection, with a second scan of the selected
// columns' lengths giving A~'s column pointers (also kept per column of A in
// col_start, col_len).  Counts kt, nnz(A~) and the chosen groups M.
__global__ __launch_bounds__(kScanThreads) void k_select(
    const int64_t *__restrict__ Acolptr, int64_t k, const int32_t *__restrict__ gid,
    const uint8_t *__restrict__ hit, const int32_t *__restrict__ gfirst,
    int32_t *__restrict__ map, int32_t *__restrict__ colid, int64_t *__restrict__ At_colptr,
    int64_t *__restrict__ col_start, int32_t *__restrict__ col_len, uint64_t *__restrict__ st_cnt, uint64_t *__restrict__ st_nnz, int64_t ntiles,
    DevCounters *__restrict__ ctr) {
    __shared__ long long s_ticket;
    __shared__ int s_tmp[kScanThreads / kWave + 1];
    __shared__ long long s_tmp64[kScanThreads / kWave + 1];
    __shared__ long long s_pc, s_pn;
    const long long t = take_ticket(&ctr->tickets[kTkSelect], &s_ticket);
    const int tid = threadIdx.x;
    const int64_t c0 = t * kScanTile + (int64_t)tid * kScanItems;
    // every item loads (past the end: A's last column, a group id of -1:
    // group 0; neither counted), so the loads carry no branches and each
    // kind is in flight together
    int32_t g[kScanItems];
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) g[i] = gid[min(c0 + i, k - 1)];
    int hv[kScanItems];
    int32_t gf[kScanItems];
    int64_t a0[kScanItems], a1[kScanItems];
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const int64_t cc = min(c0 + i, k - 1);
        const int32_t gg = g[i] >= 0 ? g[i] : 0;
        hv[i] = hit[gg];
        gf[i] = gfirst[gg];
        a0[i] = Acolptr[cc];
        a1[i] = Acolptr[cc + 1];
    }
    int sel[kScanItems];
    long long len[kScanItems];
    int cnt = 0, mcnt = 0;
    long long nnz = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const int64_t c = c0 + i;
        const bool s = c < k && g[i] >= 0 && hv[i];
        sel[i] = s ? 1 : 0;
        len[i] = s ? a1[i] - a0[i] : 0;
        mcnt += s && gf[i] == (int32_t)c;
        cnt += sel[i];
        nnz += len[i];
    }
    int totc;
    long long totn;
    int exc = group_excl_scan<kScanThreads>(cnt, s_tmp, &totc);
    long long exn = group_excl_scan64<kScanThreads>(nnz, s_tmp64, &totn);
    if (tid < kWave) {
        const long long pre = chained_prefix(st_cnt, t, t == 0, totc);
        if (tid == 0) s_pc = pre;
    } else if (tid < 2 * kWave) {
        const long long pre = chained_prefix(st_nnz, t, t == 0, totn);
        if (tid == kWave) s_pn = pre;
    }
    __syncthreads();
    long long j = s_pc + exc;
    long long pos = s_pn + exn;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const int64_t c = c0 + i;
        if (c >= k) break;
        if (sel[i]) {
            map[c] = (int32_t)j;
            colid[j] = (int32_t)c;
            At_colptr[j] = pos;
            col_start[c] = pos;
            col_len[c] = (int32_t)len[i];
            ++j;
            pos += len[i];
        } else {
            map[c] = -1;
            col_start[c] = 0;
            col_len[c] = 0;
        }
    }
    // one atomic per tile (see k_rank_groups)
    const int msum = wave_sum(mcnt);
    if (lane_id() == 0) s_tmp[tid / kWave] = msum;
    __syncthreads();
    if (tid == 0) {
        int msum_tile = 0;
        for (int w = 0; w < kScanThreads / kWave; ++w) msum_tile += s_tmp[w];
        if (msum_tile) atomic_add_i64(&ctr->M, (long long)msum_tile);
    }
    if (t == ntiles - 1 && tid == 0) {
        const long long kt = s_pc + totc;
        const long long nt = s_pn + totn;
        At_colptr[kt] = nt;
        ctr->kt = kt;
        ctr->nnz_At = nt;
    }
}

template <typename V, bool kRows>
__global__ __launch_bounds__(kGatherThreads) void k_gather(const int64_t *__restrict__ Acolptr,
                                                           const int32_t *__restrict__ Arowidx,
                                                           const V *__restrict__ Avals,
                                                           const int32_t *__restrict__ map,
                                                           const int64_t *__restrict__ At_colptr,
                                                           int64_t k, int32_t *__restrict__ At_rowidx,
                                                           V *__restrict__ At_vals) {
    __shared__ GatherStage st;
    gather_tile<V, kRows>(blockIdx.x, Acolptr, Arowidx, Avals, map, At_colptr, k, At_rowidx,
                          At_vals, st);
}

// Checks the CSC invariants of a matrix: colptr[0] = 0, colptr[n] = nnz,
// non-decreasing pointers, row ids in range and strictly ascending per
// column.  Sets bit `flag` of ctr->error on a violation.
__global__ void k_validate(const int64_t *__restrict__ colptr, const int32_t *__restrict__ rowidx,
                           int64_t nrows, int64_t ncols, int64_t nnz, int flag,
                           DevCounters *__restrict__ ctr) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    bool bad = false;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t0 == 0 && (colptr[0] != 0 || colptr[ncols] != nnz)) bad = true;
    for (int64_t j = t0; j < ncols; j += stride) {
        const int64_t lo = colptr[j], hi = colptr[j + 1];
        if (hi < lo || lo < 0 || hi > nnz) {
            bad = true;
            continue;
        }
        int32_t prev = -1;
        for (int64_t p = lo; p < hi; ++p) {
            const int32_t r = rowidx[p];
            if (r <= prev || r >= nrows) {
                bad = true;
                break;
            }
            prev = r;
        }
    }
    if (bad) atomicOr(&ctr->error, flag);
}

// Writes (first, last) of every chosen group in group order (Alg. 2's R).
// A group's last column is recorded by the plan when its rank closes the
// group; a partition's final, shorter group whose last column was not seen
// by the partition's last tile is completed here by walking its columns.
__global__ __launch_bounds__(1024) void k_export_blocks(const uint8_t *__restrict__ hit,
                                                        const int32_t *__restrict__ gfirst,
                                                        const int32_t *__restrict__ glast,
                                                        const int32_t *__restrict__ gid, int64_t k,
                                                        int64_t G, int64_t *__restrict__ blocks) {
    __shared__ int s_tmp[1024 / kWave + 1];
    long long base = 0;
    for (int64_t g0 = 0; g0 < G; g0 += 1024) {
        const int64_t g = g0 + threadIdx.x;
        const int h = (g < G && hit[g]) ? 1 : 0;
        int total;
        const int excl = group_excl_scan<1024>(h, s_tmp, &total);
        if (h) {
            const int32_t first = gfirst[g];
            int32_t last = glast[g];
            if (last < 0) {
                last = first;
                for (int64_t c = first + 1; c < k; ++c) {
                    const int32_t gg = gid[c];
                    if (gg == (int32_t)g) last = (int32_t)c;
                    else if (gg != -1) break;
                }
            }
            blocks[2 * (base + excl)] = first;
            blocks[2 * (base + excl) + 1] = last;
        }
        base += total;
    }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
static inline unsigned grid_for(int64_t work, int threads, int64_t cap = 65536) {
    int64_t g = (work + threads - 1) / threads;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

int launch_validate(Plan &p) {
    hipLaunchKernelGGL(k_validate, dim3(grid_for(p.k, 256, 4096)), dim3(256), 0, p.stream,
                       p.Acolptr, p.Arowidx, p.m, p.k, p.nnzA, 1, p.ctr);
    hipLaunchKernelGGL(k_validate, dim3(grid_for(p.n, 256, 4096)), dim3(256), 0, p.stream,
                       p.Bcolptr, p.Browidx, p.k, p.n, p.nnzB, 2, p.ctr);
    SPG_HIP(hipGetLastError());
    return SPGEMM_OK;
}

int launch_plan_kernels(Plan &p) {
    const int64_t nstatus = p.n_rank_tiles + 2 * p.n_sel_tiles;
    const int64_t clear_work = std::max<int64_t>(
        std::max<int64_t>(std::max<int64_t>(p.k, p.G), std::max<int64_t>(nstatus, p.up_words)),
        p.n);
    hipLaunchKernelGGL(k_plan_init, dim3(grid_for(clear_work, 256, 2048)), dim3(256), 0, p.stream,
                       p.H, p.k, p.hit, p.gfirst, p.glast, p.G, p.st_rank, nstatus, p.ctr,
                       p.At_colptr, p.up_src, (uint64_t *)p.group_base, p.up_words, p.flop,
                       p.arrive, p.n);
    if (p.nnzB > 0)
        hipLaunchKernelGGL(k_mark_rows, dim3(grid_for(p.nnzB, 256, 8192)), dim3(256), 0, p.stream,
                           p.Browidx, p.nnzB, p.H);
    if (p.n_rank_tiles > 0)
        hipLaunchKernelGGL(k_rank_groups, dim3((unsigned)p.n_rank_tiles), dim3(kScanThreads), 0,
                           p.stream, p.Acolptr, p.H, p.rank_tiles, p.group_base, p.b, p.gid,
                           p.hit, p.gfirst, p.glast, p.st_rank,
                           p.tun.own_partition_whole ? p.tun.own_partition : -1, p.ctr);
    if (p.n_sel_tiles > 0)
        hipLaunchKernelGGL(k_select, dim3((unsigned)p.n_sel_tiles), dim3(kScanThreads), 0,
                           p.stream, p.Acolptr, p.k, p.gid, p.hit, p.gfirst, p.map, p.colid,
                           p.At_colptr, p.col_start, p.col_len, p.st_sel_cnt, p.st_sel_nnz,
                           p.n_sel_tiles, p.ctr);
    // the gather of A~ runs in one launch with the flops and bins
    // (launch_flop_bin_gather)
    SPG_HIP(hipGetLastError());
    return SPGEMM_OK;
}

int launch_gather_values(Plan &p, const void *Avals) {
    if (p.k == 0 || p.nnzA == 0) return SPGEMM_OK;
    const unsigned g = (unsigned)((p.k + kGatherCols - 1) / kGatherCols);
    if (p.dtype == SPGEMM_F64)
        hipLaunchKernelGGL((k_gather<double, false>), dim3(g), dim3(kGatherThreads), 0, p.stream,
                           p.Acolptr, p.Arowidx, (const double *)Avals, p.map, p.At_colptr, p.k,
                           p.At_rowidx, (double *)p.At_vals);
    else
        hipLaunchKernelGGL((k_gather<float, false>), dim3(g), dim3(kGatherThreads), 0, p.stream,
                           p.Acolptr, p.Arowidx, (const float *)Avals, p.map, p.At_colptr, p.k,
                           p.At_rowidx, (float *)p.At_vals);
    SPG_HIP(hipGetLastError());
    return SPGEMM_OK;
}

int launch_export_blocks(Plan &p, int64_t *blocks) {
    if (p.G == 0) return SPGEMM_OK;
    hipLaunchKernelGGL(k_export_blocks, dim3(1), dim3(1024), 0, p.stream, p.hit, p.gfirst,
                       p.glast, p.gid, p.k, p.G, blocks);
    SPG_HIP(hipGetLastError());
    return SPGEMM_OK;
}

}  // namespace spg
