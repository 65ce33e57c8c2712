// Internal declarations shared by the host side of the library and the
// kernel translation units.  Not part of the public ABI (include/spgemm.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/spgemm.h"

namespace spg {

// Bins of output columns.  The symbolic phase bins by sparse flops, the
// numeric phase by flops (tiny) and by the exact nnz of the column.
enum Bin : int {
    kBinEmpty = 0,
    kBinTiny = 1,  // flop <= tiny_max_flop (<= 512): one wave, terms in registers
    kBinH0 = 2,    // LDS hash, smallest table
    kBinH1 = 3,
    kBinH2 = 4,
    kBinH3 = 5,    // LDS hash, largest table
    kBinDense = 6, // LDS bitmap over all rows (symbolic) / rank windows (numeric)
    kBinDenseFirst = 7,  // numeric: dense columns with the most products, handed out first
    kNumBins = 8
};

// Hash-table sizes (slots, power of two) per hash bin.  A bin holds columns
// whose key count (flops for symbolic, nnz for numeric) is at most half the
// table, so probing stays short.
constexpr int kSymTable[4] = {256, 1024, 4096, 8192};
constexpr int kNumTable[4] = {256, 512, 2048, 4096};

// Rows of C one pass of a dense column holds as a bitmap in LDS (32 KiB);
// a taller column is done in bands of this many rows, one after another.
constexpr int64_t kMaxDenseRows = 1 << 18;
constexpr int kDenseThreads = 1024;

// Row blocks of the split table: the rows of C are cut into blocks of
// kSplitRows, and for every column of A~ longer than a short entry the table
// holds, per block border b, how many of the column's entries lie above row
// b * kSplitRows.  A dense output column whose values do not fit in LDS at
// once is computed in windows of whole blocks, and each window reaches
// exactly its part of every long column of A~ through the table.
constexpr int kSplitShift = 13;
constexpr int64_t kSplitRows = int64_t(1) << kSplitShift;  // 256 bitmap words

// Tiles of the chained scans.
constexpr int kScanThreads = 256;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanThreads * kScanItems;  // 1024 elements

struct RankTile {
    int64_t col0;   // first column of the tile
    int32_t ncols;  // columns in the tile (<= kScanTile)
    int32_t part;   // partition of A the tile lies in
    int32_t head;   // 1: first tile of its partition
    int32_t last;   // 1: last tile of its partition
};

// A counter alone on its 128-byte line, so atomics on different counters
// do not serialise on one cache line.
struct alignas(128) LineInt {
    int v;
    int pad[31];
};
struct alignas(128) LineI64 {
    long long v;
    long long pad[15];
};

// Counters kept in device memory; the host copies the whole block.
struct DevCounters {
    unsigned long long tickets[8];  // chained-scan tile tickets
    long long h_count;
    long long nzc;
    long long K;
    long long M;
    long long kt;
    long long nnz_At;
    long long nnzC;
    int error;  // bit 0: A malformed, bit 1: B malformed
    int pad0;
    LineI64 flops;
    LineInt sym_count[kNumBins];
    LineInt num_count[kNumBins];
    // work queues of the dense kernels: next column, workgroups finished
    // (the last workgroup of a launch puts both back to 0)
    unsigned int num_dense_queue[2];
    unsigned int sym_dense_queue[2];
};

enum PinnedFlag { kFlagCounts = 0, kFlagColptr = 1 };
// u32 index, in the same pinned block, of a 64-bit word where the
// one-workgroup scan stores nnz(C_i) + 1 as soon as it has the total, ahead
// of its other writes and of kFlagColptr (8-byte aligned).
constexpr int kNnzSlot = 16;
// B_i with at most this many columns is scanned by one workgroup.
constexpr int64_t kSmallScanCols = 8192;

// What the symbolic phase needs from the device counters, copied by the
// kernel that completes them to pinned host memory (one wave's writes).
struct PublishedCounts {
    long long flops;
    long long nnzC;
    int sym_count[kNumBins];
    int num_count[kNumBins];
    long long nnz_At;  // entries of A~ (the plan's selection, final before the flops pass)
};

enum Ticket {
    kTkRank = 0,
    kTkSelect = 1,
    kTkColptr = 2,
    kTkExport = 3,
    kTkFlopDone = 4,    // workgroups of the flops kernel that have finished
    kTkColptrDone = 5,  // tiles of the colptr scan that have finished
};

// Where the products of entry q of B_i live in A~: positions [start[q],
// start[q] + len[q]) of A~'s arrays, i.e. the column map[row of q] (len is 0
// when A~ holds no column for that row).  Filled once per symbolic phase by
// the flops kernel, so the term walkers reach A~ with one load per entry
// instead of the chain row id -> map -> column pointers.
struct TermRange {
    const int64_t *start;
    const int32_t *len;
};

// Tiny columns (at most 64*8 products) sort their products by a 32-bit key
// (row << kSlotBits) | slot when the rows fit (m below kPackedRowLimit); the
// symbolic phase keeps the sorted slots (kNoSlot past the last product).
constexpr int kSlotBits = 9;
constexpr int64_t kPackedRowLimit = int64_t(1) << (31 - kSlotBits);
constexpr uint16_t kNoSlot = 0xFFFF;

struct Thresholds {
    int tiny_max_flop;
    int sym_hash_max[4];  // flop limit per symbolic hash bin (0 = bin unused)
    int num_hash_max[4];  // nnz limit per numeric hash bin
    int dense_first_flop;  // dense columns with at least this many products: bin 7 (0 = none)
};

// ---------------------------------------------------------------------------
// host-side plan
// ---------------------------------------------------------------------------
struct Plan {
    int device = 0;
    hipStream_t stream = nullptr;
    spgemm_dtype dtype = SPGEMM_F64;
    size_t vsize = 8;
    spgemm_tuning tun{};
    Thresholds th{};

    int64_t m = 0, k = 0, n = 0, nnzA = 0, nnzB = 0;
    int64_t nnzAt_pub = -1;  // nnz(A~) as the device published it (-1: not yet read)
    const int64_t *Acolptr = nullptr;
    const int32_t *Arowidx = nullptr;
    const void *Avals = nullptr;
    const int64_t *Bcolptr = nullptr;
    const int32_t *Browidx = nullptr;
    const void *Bvals = nullptr;
    int32_t P = 1;
    int64_t b = 1;
    std::vector<int64_t> offs;

    // workspace (one pooled device block carved into arrays)
    void *ws = nullptr;
    size_t ws_bytes = 0;
    void *pinned = nullptr;  // pooled pinned host block
    size_t pinned_bytes = 0;

    uint8_t *H = nullptr;
    int32_t *gid = nullptr;
    uint8_t *hit = nullptr;
    int32_t *gfirst = nullptr;
    int32_t *glast = nullptr;
    int64_t G = 0;  // size of the group-id space
    int64_t *group_base = nullptr;  // device [P+1]
    RankTile *rank_tiles = nullptr;  // device
    int64_t n_rank_tiles = 0;
    // the host-written block [group_base .. rank_tiles] in pinned memory (a
    // device address) and its size in 8-byte words: k_plan_init copies it
    const uint64_t *up_src = nullptr;
    int64_t up_words = 0;
    int32_t *map = nullptr;
    int32_t *colid = nullptr;
    // k: where column c of A sits in A~ (first entry, length; 0, 0 when not
    // chosen), so a row of B_i finds its products with one load
    bool early_tiny = false;  // the first symbolic run launches the tiny kernel early
    int64_t *col_start = nullptr;
    int32_t *col_len = nullptr;
    int64_t *At_colptr = nullptr;
    int32_t *At_rowidx = nullptr;
    void *At_vals = nullptr;
    uint64_t *st_rank = nullptr;
    uint64_t *st_sel_cnt = nullptr;
    uint64_t *st_sel_nnz = nullptr;
    uint64_t *st_colptr = nullptr;
    int64_t n_sel_tiles = 0, n_col_tiles = 0;
    DevCounters *ctr = nullptr;

    int64_t *flop = nullptr;
    int32_t *sym_bin = nullptr;
    int32_t *num_bin = nullptr;
    int32_t *sym_list = nullptr;  // kNumBins x n
    int32_t *num_list = nullptr;  // kNumBins x n
    // split table: k x (nblk + 1) int32, rows of the columns of A that are
    // long in A~ (built once per plan, by the first run that has dense
    // columns); nblk = ceil(m / kSplitRows).  In the workspace for m up to
    // kMaxDenseRows, else a pool block (split_block) taken when needed.
    int32_t *split = nullptr;
    int32_t nblk = 0;
    bool split_ready = false;
    void *split_block = nullptr;
    size_t split_bytes = 0;
    // What the symbolic phase keeps for the numeric phase, per column: its
    // slot in dense_bits (dense columns) or in tiny_perm (tiny columns), or -1
    int32_t *col_slot = nullptr;  // n
    int32_t *arrive = nullptr;    // n: chunks of the flops pass done per long column
    void *kept = nullptr;           // pooled block holding dense_bits
    size_t kept_bytes = 0;
    void *kept_tiny = nullptr;      // pooled block holding tiny_perm
    size_t kept_tiny_bytes = 0;
    uint32_t *dense_bits = nullptr; // row bitmaps of the symbolic dense columns
    // the two above point into the no-allocation scratch array of the device
    // (spgemm_symbolic_noalloc), taken with generation scratch_gen
    bool kept_in_scratch = false;
    uint64_t scratch_gen = 0;
    uint16_t *tiny_perm = nullptr;  // sorted order of the terms of tiny columns
    int64_t *tstart = nullptr;    // nnzB: term range of every entry of B_i
    int32_t *tlen = nullptr;      // nnzB
    TermRange term_range() const { return TermRange{tstart, tlen}; }
    int lds_max = 65536;          // LDS bytes one workgroup may use on this device

    // host view of the counters (inside the pinned block) and its device
    // address, where the flops kernel and the colptr scan publish them
    DevCounters *hctr = nullptr;
    PublishedCounts *hpub = nullptr;      // pinned; written by the publishing kernels
    PublishedCounts *hpub_dev = nullptr;  // its device address
    // pinned flags the publishing kernels set once hctr holds their counters
    // (host and device addresses): kFlagCounts (flops pass), kFlagColptr (scan)
    uint32_t *hflags = nullptr;
    uint32_t *hflags_dev = nullptr;

    // symbolic results
    bool symbolic_done = false;
    // nnzC is known but the flops total and the numeric bin counts are still
    // on their way to hpub (kFlagColptr); finish_symbolic_counts collects them
    bool counts_pending = false;
    int symbolic_runs = 0;
    hipEvent_t counts_ready = nullptr;  // the plan's counters (flops, bins) reached hctr
    int64_t *C_colptr = nullptr;
    int64_t nnzC = -1;
    int64_t flops = -1;
    int sym_count[kNumBins] = {0};
    int num_count[kNumBins] = {0};
};

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
void set_error(const std::string &msg);
int fail(int code, const std::string &msg);

#define SPG_HIP(call)                                                                \
    do {                                                                             \
        hipError_t e_ = (call);                                                      \
        if (e_ != hipSuccess)                                                        \
            return ::spg::fail(SPGEMM_EHIP, std::string(#call) + ": " +              \
                                                 hipGetErrorString(e_));             \
    } while (0)

// Checks the launch just made; names the kernel in the message.
#define SPG_LAUNCHED(name)                                                           \
    do {                                                                             \
        hipError_t e_ = hipGetLastError();                                           \
        if (e_ != hipSuccess)                                                        \
            return ::spg::fail(SPGEMM_EHIP, std::string("launch of ") + (name) + ": " + \
                                                 hipGetErrorString(e_));             \
    } while (0)

// ---------------------------------------------------------------------------
// launchers (each returns SPGEMM_OK or an error code with the message set)
// ---------------------------------------------------------------------------
// Compute units of a device (queried once; 0 if unknown).
int device_cu_count(int device);
// Workgroups of `kernel` (threads each, lds bytes of dynamic LDS) that fit
// on the device at once, capped at `work` (at least 1).
unsigned resident_groups(const void *kernel, int threads, size_t lds, int device, long long work);

int launch_validate(Plan &p);
int launch_plan_kernels(Plan &p);
int launch_gather_values(Plan &p, const void *Avals);
int launch_export_blocks(Plan &p, int64_t *blocks);
int launch_flop_bin_gather(Plan &p);
// B_i with at most kEarlyTinyCols columns: the tiny symbolic kernel is
// launched before the host has the bin counts (sized for every column, the
// count read on the device), so it follows the flops pass without the
// host's round trip in between.
constexpr int64_t kEarlyTinyCols = 16384;
// Such a launch also publishes the flops pass's counters (from a workgroup
// of its own), so the flops pass ends without that round trip; set by
// spgemm_plan for the plan's first symbolic run.
int launch_sym_tiny(Plan &p, bool early);
int launch_symbolic_bins(Plan &p, bool tiny_launched);
int launch_colptr_scan(Plan &p);
int finish_symbolic_counts(Plan &p);
int launch_symbolic_reset(Plan &p);
int launch_split_table(Plan &p);
// dense_columns < 0: the numeric dense bins' count.
int ensure_split_table(Plan &p, int64_t dense_columns = -1);
// SPGEMM_ESTATE when the plan's kept symbolic data sat in the no-allocation
// scratch array and a later call has taken the array over.
int check_kept(const Plan &p);
// At_vals: A~'s values for this call (NULL: the plan's A~).
int launch_numeric_bins(Plan &p, const void *Bvals, int32_t *Crow, void *Cvals,
                        const void *At_vals = nullptr);
// New values of A for one numeric call: when A~ holds every entry of A (in
// A's order), they are A~'s values as they are and nothing is gathered
// (returns them); otherwise they are gathered into A~ (returns NULL).
int take_new_a_values(Plan &p, const void *A_vals, const void **At_vals);
int launch_backward(Plan &p, const int64_t *Ccolptr, const int32_t *Crow, const void *Avals,
                    const void *Bvals, const void *dC, void *dA, void *dB);
// The single-launch form of a batch (persistent.hip): its work items,
// per-product arguments and control block (ticket, exit count, error word,
// one completion flag per item) in device memory.
struct PersistentBatch {
    int device = 0;
    spgemm_dtype dtype = SPGEMM_F64;
    void *items = nullptr;
    void *prods = nullptr;
    unsigned *ctr = nullptr;
    size_t ctr_bytes = 0;
    int nitems = 0;
    int nprod = 0;
    unsigned grid = 1;
    long long wait_ticks = 0;  // bound of one dependency wait, in wall-clock ticks
};
int persistent_build(const std::vector<Plan *> &plans, const std::vector<spgemm_batch_io> &io,
                     const std::vector<std::vector<int>> &levels, PersistentBatch &pb);
int persistent_launch(const PersistentBatch &pb, hipStream_t s);
// The batch's error word (1: a dependency wait ran out of time); synchronises.
int persistent_error(const PersistentBatch &pb, unsigned *err);
void persistent_free(PersistentBatch &pb);

// Drops (and frees) every batch spgemm_batched keeps that names this plan.
void batch_cache_drop(const Plan *plan);

}  // namespace spg

// The opaque handle of the C ABI is the plan itself.
struct spgemm_plan_s : public spg::Plan {};
