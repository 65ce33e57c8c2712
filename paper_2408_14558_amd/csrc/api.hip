// C ABI of the local SpGEMM (include/spgemm.h): argument checks, the plan
// object and its workspace, the pooled allocator, and the order of launches.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <climits>
#include <cstring>
#include <chrono>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "internal.hpp"

namespace spg {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string t_last_error;

void set_error(const std::string &msg) { t_last_error = msg; }

int fail(int code, const std::string &msg) {
    t_last_error = msg;
    return code;
}

// ---------------------------------------------------------------------------
// pooled allocator: device workspaces and pinned host blocks are kept after a
// plan is destroyed and handed to the next plan that fits, so repeated
// plan/destroy cycles do not call hipMalloc.  A block freed on one stream
// and reused on another makes the new stream wait on an event recorded at
// the free (device), or waits on the host (pinned).
// ---------------------------------------------------------------------------
struct PoolBlock {
    void *ptr;
    size_t bytes;
    int device;
    bool pinned;
    hipEvent_t ev;
    hipStream_t stream;
};

static std::mutex g_pool_mtx;
static std::vector<PoolBlock> g_pool;
static std::vector<hipEvent_t> g_spare_events;  // recorded events come back here

// An event for pool_put: a spare one if any, else a new one.
static hipError_t take_event(hipEvent_t *ev) {
    {
        std::lock_guard<std::mutex> lk(g_pool_mtx);
        if (!g_spare_events.empty()) {
            *ev = g_spare_events.back();
            g_spare_events.pop_back();
            return hipSuccess;
        }
    }
    return hipEventCreateWithFlags(ev, hipEventDisableTiming);
}

static size_t round_block(size_t bytes, bool pinned) {
    const size_t g = pinned ? 4096 : (1 << 20);
    return (bytes + g - 1) / g * g;
}

static int pool_get(size_t bytes, bool pinned, int device, hipStream_t stream, void **out,
                    size_t *got) {
    bytes = round_block(std::max<size_t>(bytes, 1), pinned);
    {
        std::lock_guard<std::mutex> lk(g_pool_mtx);
        int best = -1;
        for (size_t i = 0; i < g_pool.size(); ++i) {
            const PoolBlock &b = g_pool[i];
            if (b.pinned != pinned || b.device != device || b.bytes < bytes ||
                b.bytes > 2 * bytes + (1 << 20))
                continue;
            if (best < 0 || b.bytes < g_pool[best].bytes) best = (int)i;
        }
        if (best >= 0) {
            PoolBlock b = g_pool[best];
            g_pool.erase(g_pool.begin() + best);
            if (pinned) {
                SPG_HIP(hipEventSynchronize(b.ev));
            } else if (b.stream != stream) {
                SPG_HIP(hipStreamWaitEvent(stream, b.ev, 0));
            }
            g_spare_events.push_back(b.ev);
            *out = b.ptr;
            *got = b.bytes;
            return SPGEMM_OK;
        }
    }
    void *p = nullptr;
    hipError_t e = pinned ? hipHostMalloc(&p, bytes, hipHostMallocDefault) : hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(SPGEMM_ENOMEM, std::string(pinned ? "hipHostMalloc" : "hipMalloc") + " of " +
                                       std::to_string(bytes) + " bytes failed: " +
                                       hipGetErrorString(e));
    }
    *out = p;
    *got = bytes;
    return SPGEMM_OK;
}

// Returns a block to the pool.  `last_use`, when given, is an event already
// recorded after the block's last use (the pool takes it over); otherwise one
// is recorded on `stream` now.
static void pool_put(void *ptr, size_t bytes, bool pinned, int device, hipStream_t stream,
                     hipEvent_t last_use = nullptr) {
    if (!ptr) return;
    if (last_use) {
        std::lock_guard<std::mutex> lk(g_pool_mtx);
        g_pool.push_back(PoolBlock{ptr, bytes, device, pinned, last_use, stream});
        return;
    }
    hipEvent_t ev = nullptr;
    if (take_event(&ev) != hipSuccess || hipEventRecord(ev, stream) != hipSuccess) {
        if (ev) (void)hipEventDestroy(ev);
        (void)hipStreamSynchronize(stream);
        if (pinned) (void)hipHostFree(ptr); else (void)hipFree(ptr);
        return;
    }
    std::lock_guard<std::mutex> lk(g_pool_mtx);
    g_pool.push_back(PoolBlock{ptr, bytes, device, pinned, ev, stream});
}

static int pool_trim() {
    std::vector<PoolBlock> blocks;
    std::vector<hipEvent_t> spare;
    {
        std::lock_guard<std::mutex> lk(g_pool_mtx);
        blocks.swap(g_pool);
        spare.swap(g_spare_events);
    }
    for (hipEvent_t e : spare) (void)hipEventDestroy(e);
    for (auto &b : blocks) {
        (void)hipEventSynchronize(b.ev);
        (void)hipEventDestroy(b.ev);
        if (b.pinned) (void)hipHostFree(b.ptr); else (void)hipFree(b.ptr);
    }
    return SPGEMM_OK;
}

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
// Waits until a publishing kernel has set pinned flag f (its counters are in
// hctr by then): spins on the flag for up to kSpinMicros, because a blocking
// wait adds the host's wake-up latency to every small product, then falls
// back to block(), which also reports launch errors.
constexpr int kSpinMicros = 500;

template <typename F>
static hipError_t wait_flag(Plan &p, int f, F &&block) {
    const auto t0 = std::chrono::steady_clock::now();
    for (unsigned i = 0;; ++i) {
        if (__atomic_load_n(p.hflags + f, __ATOMIC_ACQUIRE)) return hipSuccess;
        if ((i & 255u) == 255u &&
            std::chrono::steady_clock::now() - t0 > std::chrono::microseconds(kSpinMicros))
            break;
        __builtin_ia32_pause();
    }
    return block();
}

// Compute units of a device (queried once); 0 if the query fails.
int device_cu_count(int device) {
    static std::mutex mtx;
    static std::vector<int> cache;
    std::lock_guard<std::mutex> lk(mtx);
    if (device < 0) return 0;
    if ((size_t)device >= cache.size()) cache.resize(device + 1, 0);
    if (cache[device] == 0 &&
        hipDeviceGetAttribute(&cache[device], hipDeviceAttributeMultiprocessorCount, device) !=
            hipSuccess)
        cache[device] = 0;
    return cache[device];
}

unsigned resident_groups(const void *kernel, int threads, size_t lds, int device,
                         long long work) {
    // the occupancy query costs tens of microseconds of host time: asked once
    // per kernel, block size, LDS size and device
    static std::mutex mtx;
    static std::map<std::tuple<const void *, int, size_t, int>, int> cache;
    int per_cu = 0;
    {
        std::lock_guard<std::mutex> lk(mtx);
        const auto key = std::make_tuple(kernel, threads, lds, device);
        auto it = cache.find(key);
        if (it != cache.end()) {
            per_cu = it->second;
        } else {
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, lds) !=
                hipSuccess) {
                (void)hipGetLastError();
                per_cu = 0;
            }
            cache[key] = per_cu;
        }
    }
    const long long cus = device_cu_count(device);
    long long g = (long long)std::max(per_cu, 1) * (cus > 0 ? cus : 256);
    g = std::min(g, work);
    return (unsigned)std::max(g, 1LL);
}

// LDS bytes one workgroup may use, per device (queried once).
static int device_lds_max(int device, int *out) {
    static std::mutex mtx;
    static std::vector<int> cache;
    std::lock_guard<std::mutex> lk(mtx);
    if (device < 0) return 1;
    if ((size_t)device >= cache.size()) cache.resize(device + 1, 0);
    if (cache[device] == 0 &&
        hipDeviceGetAttribute(&cache[device], hipDeviceAttributeMaxSharedMemoryPerBlock, device) !=
            hipSuccess) {
        cache[device] = 0;
        return 1;
    }
    *out = cache[device];
    return 0;
}
struct Carver {
    size_t off = 0;
    template <typename T>
    size_t take(int64_t count) {
        off = (off + 255) & ~(size_t)255;
        const size_t at = off;
        off += (size_t)std::max<int64_t>(count, 0) * sizeof(T);
        return at;
    }
};

static int check_csc(const spgemm_csc *M, const char *name) {
    if (!M) return fail(SPGEMM_EINVAL, std::string(name) + " is NULL");
    if (M->nrows < 0 || M->ncols < 0 || M->nnz < 0)
        return fail(SPGEMM_EINVAL, std::string(name) + " has a negative size");
    if (M->nrows >= (1ll << 31) || M->ncols >= (1ll << 31))
        return fail(SPGEMM_EINVAL, std::string(name) + " dimensions must be below 2^31");
    if (!M->colptr) return fail(SPGEMM_EINVAL, std::string(name) + "->colptr is NULL");
    if (M->nnz > 0 && !M->rowidx) return fail(SPGEMM_EINVAL, std::string(name) + "->rowidx is NULL");
    if (M->nnz > 0 && M->nrows == 0)
        return fail(SPGEMM_EINVAL, std::string(name) + " stores entries but has no rows");
    return SPGEMM_OK;
}

static void thresholds_from(const spgemm_tuning &t, Thresholds &th) {
    // hash bin h holds keys up to half its table; a bin is used only above
    // the previous bin's limit and never above the tuned maximum
    th.tiny_max_flop = t.tiny_max_flop;
    int prev = t.tiny_max_flop;
    for (int h = 0; h < 4; ++h) {
        const int lim = kSymTable[h] / 2;
        if (prev >= t.hash_max_flop) {
            th.sym_hash_max[h] = 0;
        } else {
            th.sym_hash_max[h] = std::min(lim, t.hash_max_flop);
            prev = th.sym_hash_max[h];
        }
    }
    prev = 0;
    for (int h = 0; h < 4; ++h) {
        const int lim = kNumTable[h] / 2;
        if (prev >= t.hash_max_nnz) {
            th.num_hash_max[h] = 0;
        } else {
            th.num_hash_max[h] = std::min(lim, t.hash_max_nnz);
            prev = th.num_hash_max[h];
        }
    }
    th.dense_first_flop = t.dense_first_flop;
}

static int check_tuning(const spgemm_tuning &t) {
    if (t.tiny_max_flop < 0 || t.tiny_max_flop > 512)
        return fail(SPGEMM_EINVAL, "tiny_max_flop must lie in [0, 512]");
    if (t.hash_max_flop < 0 || t.hash_max_flop > kSymTable[3] / 2)
        return fail(SPGEMM_EINVAL, "hash_max_flop must lie in [0, 4096]");
    if (t.hash_max_nnz < 0 || t.hash_max_nnz > kNumTable[3] / 2)
        return fail(SPGEMM_EINVAL, "hash_max_nnz must lie in [0, 2048]");
    if (t.workspace_limit < 0) return fail(SPGEMM_EINVAL, "workspace_limit must be >= 0");
    if (t.dense_window != 0 && (t.dense_window < 32 || (t.dense_window & (t.dense_window - 1))))
        return fail(SPGEMM_EINVAL, "dense_window must be 0 or a power of two >= 32");
    if (t.medium_kernel < 0 || t.medium_kernel > 2)
        return fail(SPGEMM_EINVAL, "medium_kernel must be 0, 1 or 2");
    if (t.batch_streams < 0 || t.batch_streams > 8)
        return fail(SPGEMM_EINVAL, "batch_streams must lie in [0, 8]");
    if (t.dense_first_flop < 0) return fail(SPGEMM_EINVAL, "dense_first_flop must be >= 0");
    if (t.reserved != 0) return fail(SPGEMM_EINVAL, "reserved tuning fields must be 0");
    return SPGEMM_OK;
}

// Room for what the symbolic phase keeps for the numeric phase, in two
// pooled blocks: the sorted product order of each tiny column (the numeric
// phase does not sort again) and the row bitmap of each dense column (the
// numeric phase loads it instead of walking the products again).  Optional:
// a part that is too large, above workspace_limit, or not allocatable is left
// out and the numeric phase recomputes it.
constexpr size_t kDenseBitsMax = size_t(8) << 30;

// Makes *block hold at least `need` bytes (keeping it when it does); false
// when it cannot.
static bool reserve_block(Plan &p, void **block, size_t *bytes, size_t need) {
    if (*bytes >= need) return true;
    pool_put(*block, *bytes, false, p.device, p.stream);
    *block = nullptr;
    *bytes = 0;
    void *ptr = nullptr;
    size_t got = 0;
    if (pool_get(need, false, p.device, p.stream, &ptr, &got) != SPGEMM_OK) {
        (void)hipGetLastError();
        return false;
    }
    *block = ptr;
    *bytes = got;
    return true;
}

static size_t kept_limit(const Plan &p) {
    return p.tun.workspace_limit > 0 ? (size_t)p.tun.workspace_limit : SIZE_MAX;
}

// Tiny part for `cols` tiny columns: the kernels' 64*EMAX product slots, 2
// bytes each.
static void reserve_tiny(Plan &p, int64_t cols) {
    const size_t slots = p.th.tiny_max_flop <= 256 ? 256 : 512;
    size_t tiny = p.m < kPackedRowLimit ? (size_t)cols * slots * 2 : 0;
    if (tiny > kDenseBitsMax || p.ws_bytes + tiny > kept_limit(p)) tiny = 0;
    p.tiny_perm = nullptr;
    if (tiny && reserve_block(p, &p.kept_tiny, &p.kept_tiny_bytes, tiny))
        p.tiny_perm = (uint16_t *)p.kept_tiny;
}

// Bytes of the kept row bitmaps of the dense columns.
static size_t dense_part_bytes(const Plan &p) {
    if (p.m > kMaxDenseRows) return 0;  // banded columns rebuild their bitmaps
    const size_t nw = (size_t)((p.m + 31) / 32);
    return (size_t)p.sym_count[kBinDense] * nw * sizeof(uint32_t);
}

static void reserve_dense(Plan &p) {
    size_t dense = dense_part_bytes(p);
    const size_t tiny = p.tiny_perm ? p.kept_tiny_bytes : 0;
    if (dense > kDenseBitsMax || p.ws_bytes + tiny + dense > kept_limit(p)) dense = 0;
    p.dense_bits = nullptr;
    if (dense && reserve_block(p, &p.kept, &p.kept_bytes, dense)) p.dense_bits = (uint32_t *)p.kept;
}

static int sync_counters(Plan &p) {
    SPG_HIP(hipMemcpyAsync(p.hctr, p.ctr, sizeof(DevCounters), hipMemcpyDeviceToHost, p.stream));
    SPG_HIP(hipStreamSynchronize(p.stream));
    return SPGEMM_OK;
}

// ---------------------------------------------------------------------------
// The no-allocation symbolic phase (spgemm_symbolic_noalloc) keeps what the
// symbolic phase hands to the numeric phase (the tiny columns' sort orders,
// the dense columns' row bitmaps) in this array instead of pooled blocks.
// Each device holds its own copy at its own address, taken once per device
// with hipGetSymbolAddress; host code uses that address, never the name.
// The array belongs to the last plan that ran spgemm_symbolic_noalloc on the
// device (generation counter per device).
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static std::mutex g_scratch_mtx;
static std::vector<void *> g_scratch_ptr;     // per device
static std::vector<uint64_t> g_scratch_gen;   // per device: the current owner's generation

// Address of this device's array (the plan's device must be current) and a
// new generation for the caller, who owns the array from now on.
static int scratch_take(int device, void **ptr, uint64_t *gen) {
    int cur = -1;
    SPG_HIP(hipGetDevice(&cur));
    if (cur != device)
        return fail(SPGEMM_EINVAL, "the plan's device must be the current device");
    std::lock_guard<std::mutex> lk(g_scratch_mtx);
    if ((size_t)device >= g_scratch_ptr.size()) {
        g_scratch_ptr.resize(device + 1, nullptr);
        g_scratch_gen.resize(device + 1, 0);
    }
    if (!g_scratch_ptr[device]) {
        void *addr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&addr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !addr) {
            (void)hipGetLastError();
            return fail(SPGEMM_EHIP, std::string("hipGetSymbolAddress(scratch): ") +
                                         hipGetErrorString(e));
        }
        g_scratch_ptr[device] = addr;
    }
    *ptr = g_scratch_ptr[device];
    *gen = ++g_scratch_gen[device];
    return SPGEMM_OK;
}

// The plan's kept data lives in the device array and a later
// spgemm_symbolic_noalloc on the device has taken the array over.
static bool scratch_lost(const Plan &p) {
    if (!p.kept_in_scratch) return false;
    std::lock_guard<std::mutex> lk(g_scratch_mtx);
    return (size_t)p.device >= g_scratch_gen.size() || g_scratch_gen[p.device] != p.scratch_gen;
}

int check_kept(const Plan &p) {
    if (scratch_lost(p))
        return fail(SPGEMM_ESTATE, "this plan's symbolic data sat in the no-allocation scratch, "
                                   "which a later spgemm_symbolic_noalloc on the device has "
                                   "taken over: run the symbolic phase again");
    return SPGEMM_OK;
}

// Bytes of the tiny part for `cols` tiny columns (the kernels' 64*EMAX
// product slots, 2 bytes each); 0 when the rows are too wide to pack.
static size_t tiny_part_bytes(const Plan &p, int64_t cols) {
    const size_t slots = p.th.tiny_max_flop <= 256 ? 256 : 512;
    return p.m < kPackedRowLimit ? (size_t)cols * slots * 2 : 0;
}


// The flops total and the numeric bin counts of a symbolic run that returned
// nnz(C_i) early (one-workgroup scan): waits for the scan's flag and reads
// them from the pinned block.
static size_t split_table_bytes(const Plan &p) {
    return sizeof(int32_t) * (size_t)p.k * (size_t)(p.nblk + 1);
}

// Windows of dense columns reach A~ through the split table, which depends
// on the patterns only: built once per plan, by the first run that has dense
// columns (numeric or batch; for m above 2^18 already the symbolic run, whose
// bands need it, and the table is then taken from the pool).
int ensure_split_table(Plan &p, int64_t dense_columns) {
    if (dense_columns < 0) dense_columns = p.num_count[kBinDense] + p.num_count[kBinDenseFirst];
    if (p.split_ready || dense_columns == 0 || p.nblk <= 1 || p.k == 0) return SPGEMM_OK;
    if (!p.split) {
        const size_t need = split_table_bytes(p);
        if (!reserve_block(p, &p.split_block, &p.split_bytes, need))
            return fail(SPGEMM_ENOMEM, "split table of " + std::to_string(need) + " bytes");
        p.split = (int32_t *)p.split_block;
    }
    if (int rc = launch_split_table(p)) return rc;
    p.split_ready = true;
    return SPGEMM_OK;
}

int take_new_a_values(Plan &p, const void *A_vals, const void **At_vals) {
    *At_vals = nullptr;
    if (!A_vals) return SPGEMM_OK;
    // every nonzero column chosen: A~'s entries are A's, in A's order
    if (p.nnzAt_pub == p.nnzA) {
        *At_vals = A_vals;
        return SPGEMM_OK;
    }
    return launch_gather_values(p, A_vals);
}

int finish_symbolic_counts(Plan &p) {
    if (!p.counts_pending) return SPGEMM_OK;
    SPG_HIP(wait_flag(p, kFlagColptr, [&] { return hipStreamSynchronize(p.stream); }));
    // the fallback synchronised the stream the scan ran on (spgemm_plan_set_stream
    // finishes the counts before it switches): the flag must be set by now
    if (!__atomic_load_n(p.hflags + kFlagColptr, __ATOMIC_ACQUIRE))
        return fail(SPGEMM_EHIP, "the symbolic scan's counts were not published");
    p.flops = p.hpub->flops;
    for (int b = 0; b < kNumBins; ++b) p.num_count[b] = p.hpub->num_count[b];
    p.nnzAt_pub = p.hpub->nnz_At;
    p.counts_pending = false;
    return SPGEMM_OK;
}

}  // namespace spg

using namespace spg;


extern "C" {

const char *spgemm_last_error(void) { return spg::t_last_error.c_str(); }

const char *spgemm_version(void) { return "spgemm-mi355x 0.1 (gfx950)"; }

// SPGEMM_<FIELD> environment variables override the built-in defaults
// (an unparsable value is ignored; the plan validates ranges).
static void env_override(const char *name, int32_t *field) {
    const char *v = std::getenv(name);
    if (!v || !*v) return;
    char *end = nullptr;
    const long long x = std::strtoll(v, &end, 10);
    if (end && *end == '\0' && x >= INT32_MIN && x <= INT32_MAX) *field = (int32_t)x;
}

int spgemm_default_tuning(spgemm_tuning *t) {
    if (!t) return fail(SPGEMM_EINVAL, "tuning is NULL");
    std::memset(t, 0, sizeof(*t));
    t->tiny_max_flop = 256;
    t->hash_max_flop = 4096;
    t->hash_max_nnz = 2048;
    t->dense_window = 0;
    t->medium_kernel = 0;
    t->batch_streams = 0;
    t->batch_form = 0;
    t->dense_first_flop = 1 << 18;
    t->reserved = 0;
    t->validate = 0;
    t->own_partition = -1;
    t->own_partition_whole = 0;
    t->workspace_limit = 0;
    env_override("SPGEMM_TINY_MAX_FLOP", &t->tiny_max_flop);
    env_override("SPGEMM_HASH_MAX_FLOP", &t->hash_max_flop);
    env_override("SPGEMM_HASH_MAX_NNZ", &t->hash_max_nnz);
    env_override("SPGEMM_DENSE_WINDOW", &t->dense_window);
    env_override("SPGEMM_DENSE_FIRST_FLOP", &t->dense_first_flop);
    env_override("SPGEMM_MEDIUM_KERNEL", &t->medium_kernel);
    env_override("SPGEMM_BATCH_STREAMS", &t->batch_streams);
    env_override("SPGEMM_VALIDATE", &t->validate);
    if (const char *v = std::getenv("SPGEMM_WORKSPACE_LIMIT"); v && *v) {
        char *end = nullptr;
        const long long x = std::strtoll(v, &end, 10);
        if (end && *end == '\0') t->workspace_limit = x;
    }
    return SPGEMM_OK;
}

int spgemm_pool_trim(void) { return pool_trim(); }

int spgemm_plan(const spgemm_csc *A, const spgemm_csc *Bi, spgemm_dtype dtype,
                const int64_t *offs, int32_t P, int64_t block_size, const spgemm_tuning *tuning,
                void *stream, spgemm_plan_t *out) {
    (void)hipGetLastError();  // drop errors left by other code on this thread
    if (!out) return fail(SPGEMM_EINVAL, "out is NULL");
    *out = nullptr;
    int rc;
    if ((rc = check_csc(A, "A")) || (rc = check_csc(Bi, "Bi"))) return rc;
    if (dtype != SPGEMM_F32 && dtype != SPGEMM_F64)
        return fail(SPGEMM_EUNSUPPORTED, "dtype must be SPGEMM_F32 or SPGEMM_F64");
    if (A->ncols != Bi->nrows)
        return fail(SPGEMM_EINVAL, "A has " + std::to_string(A->ncols) + " columns but Bi has " +
                                       std::to_string(Bi->nrows) + " rows");
    if (P < 1) return fail(SPGEMM_EINVAL, "P must be >= 1");
    if (block_size < 1) return fail(SPGEMM_EINVAL, "block_size must be >= 1");
    if (!offs) return fail(SPGEMM_EINVAL, "a_part_offsets is NULL");
    if (offs[0] != 0 || offs[P] != A->ncols)
        return fail(SPGEMM_EINVAL, "a_part_offsets must start at 0 and end at A->ncols");
    for (int r = 0; r < P; ++r)
        if (offs[r + 1] < offs[r]) return fail(SPGEMM_EINVAL, "a_part_offsets must not decrease");
    spgemm_tuning tun;
    spgemm_default_tuning(&tun);
    if (tuning) tun = *tuning;
    if ((rc = check_tuning(tun))) return rc;
    if (tun.own_partition_whole && (tun.own_partition < 0 || tun.own_partition >= P))
        return fail(SPGEMM_EINVAL, "own_partition_whole needs own_partition in [0, P)");

    auto *p = new (std::nothrow) spgemm_plan_s();
    if (!p) return fail(SPGEMM_ENOMEM, "plan allocation failed");
    Plan &pl = *p;
    if (hipGetDevice(&pl.device) != hipSuccess || device_lds_max(pl.device, &pl.lds_max)) {
        delete p;
        return fail(SPGEMM_EHIP, "hipGetDevice / hipDeviceGetAttribute failed");
    }
    pl.stream = (hipStream_t)stream;
    pl.dtype = dtype;
    pl.vsize = dtype == SPGEMM_F64 ? 8 : 4;
    pl.tun = tun;
    thresholds_from(tun, pl.th);
    pl.m = A->nrows;
    pl.k = A->ncols;
    pl.n = Bi->ncols;
    pl.nnzA = A->nnz;
    pl.nnzB = Bi->nnz;
    pl.Acolptr = A->colptr;
    pl.Arowidx = A->rowidx;
    pl.Avals = A->vals;
    pl.Bcolptr = Bi->colptr;
    pl.Browidx = Bi->rowidx;
    pl.Bvals = Bi->vals;
    pl.P = P;
    pl.b = block_size;
    pl.offs.assign(offs, offs + P + 1);

    // group-id space and rank tiles
    std::vector<int64_t> gbase(P + 1, 0);
    std::vector<RankTile> tiles;
    for (int r = 0; r < P; ++r) {
        const int64_t kr = offs[r + 1] - offs[r];
        gbase[r + 1] = gbase[r] + (kr + block_size - 1) / block_size;
        const int64_t nt = (kr + kScanTile - 1) / kScanTile;
        for (int64_t t = 0; t < nt; ++t) {
            RankTile d;
            d.col0 = offs[r] + t * kScanTile;
            d.ncols = (int32_t)std::min<int64_t>(kScanTile, kr - t * kScanTile);
            d.part = r;
            d.head = t == 0;
            d.last = t == nt - 1;
            tiles.push_back(d);
        }
    }
    pl.G = gbase[P];
    if (pl.G >= (1ll << 31)) {
        delete p;
        return fail(SPGEMM_EINVAL, "too many groups for int32 group ids");
    }
    pl.n_rank_tiles = (int64_t)tiles.size();
    pl.n_sel_tiles = (pl.k + kScanTile - 1) / kScanTile;
    pl.n_col_tiles = (pl.n + kScanTile - 1) / kScanTile;

    Carver cv;
    const size_t o_H = cv.take<uint8_t>(pl.k);
    const size_t o_gid = cv.take<int32_t>(pl.k);
    const size_t o_hit = cv.take<uint8_t>(pl.G);
    const size_t o_gfirst = cv.take<int32_t>(pl.G);
    const size_t o_glast = cv.take<int32_t>(pl.G);
    const size_t o_gbase = cv.take<int64_t>(P + 1);
    const size_t o_tiles = cv.take<RankTile>(pl.n_rank_tiles);
    // the upload copies [group_base .. tiles] as one block: same relative layout
    const size_t up_gap = o_tiles - o_gbase;
    const size_t o_map = cv.take<int32_t>(pl.k);
    const size_t o_colid = cv.take<int32_t>(pl.k);
    const size_t o_cst = cv.take<int64_t>(pl.k);
    const size_t o_cln = cv.take<int32_t>(pl.k);
    const size_t o_Atc = cv.take<int64_t>(pl.k + 1);
    const size_t o_Atr = cv.take<int32_t>(pl.nnzA);
    const size_t o_Atv = cv.take<uint8_t>(pl.nnzA * (int64_t)pl.vsize);
    const size_t o_st = cv.take<uint64_t>(pl.n_rank_tiles + 2 * pl.n_sel_tiles);
    const size_t o_stc = cv.take<uint64_t>(pl.n_col_tiles);
    const size_t o_ctr = cv.take<DevCounters>(1);
    const size_t o_flop = cv.take<int64_t>(pl.n);
    const size_t o_sbin = cv.take<int32_t>(pl.n);
    const size_t o_nbin = cv.take<int32_t>(pl.n);
    const size_t o_slist = cv.take<int32_t>(kNumBins * pl.n);
    const size_t o_nlist = cv.take<int32_t>(kNumBins * pl.n);
    pl.nblk = (int32_t)((pl.m + kSplitRows - 1) / kSplitRows);
    // the table of a plan of at most 2^18 rows sits in the workspace; a
    // taller one is taken from the pool when a symbolic run first meets a
    // dense column
    const bool split_in_ws = pl.nblk > 1 && pl.m <= kMaxDenseRows;
    const size_t o_split = cv.take<int32_t>(split_in_ws ? pl.k * (pl.nblk + 1) : 0);
    const size_t o_tst = cv.take<int64_t>(pl.nnzB);
    const size_t o_dsl = cv.take<int32_t>(pl.n);
    const size_t o_arr = cv.take<int32_t>(pl.n);
    const size_t o_tln = cv.take<int32_t>(pl.nnzB);
    const size_t ws_bytes = cv.off;
    if (tun.workspace_limit > 0 && (int64_t)ws_bytes > tun.workspace_limit) {
        delete p;
        return fail(SPGEMM_ENOMEM, "plan needs " + std::to_string(ws_bytes) +
                                       " bytes of workspace, above workspace_limit");
    }
    Carver ch;
    const size_t h_ctr = ch.take<DevCounters>(1);
    const size_t h_flags = ch.take<uint32_t>(32);
    const size_t h_pub = ch.take<PublishedCounts>(1);
    const size_t h_gbase = ch.take<int64_t>(P + 1);
    const size_t h_tiles = h_gbase + up_gap;
    const size_t pinned_bytes = h_tiles + sizeof(RankTile) * (size_t)pl.n_rank_tiles;

    if ((rc = pool_get(ws_bytes, false, pl.device, pl.stream, &pl.ws, &pl.ws_bytes))) {
        delete p;
        return rc;
    }
    if ((rc = pool_get(pinned_bytes, true, pl.device, pl.stream, &pl.pinned, &pl.pinned_bytes))) {
        pool_put(pl.ws, pl.ws_bytes, false, pl.device, pl.stream);
        delete p;
        return rc;
    }
    char *w = (char *)pl.ws;
    pl.H = (uint8_t *)(w + o_H);
    pl.gid = (int32_t *)(w + o_gid);
    pl.hit = (uint8_t *)(w + o_hit);
    pl.gfirst = (int32_t *)(w + o_gfirst);
    pl.glast = (int32_t *)(w + o_glast);
    pl.group_base = (int64_t *)(w + o_gbase);
    pl.rank_tiles = (RankTile *)(w + o_tiles);
    pl.map = (int32_t *)(w + o_map);
    pl.colid = (int32_t *)(w + o_colid);
    pl.col_start = (int64_t *)(w + o_cst);
    pl.col_len = (int32_t *)(w + o_cln);
    pl.At_colptr = (int64_t *)(w + o_Atc);
    pl.At_rowidx = (int32_t *)(w + o_Atr);
    pl.At_vals = (void *)(w + o_Atv);
    pl.st_rank = (uint64_t *)(w + o_st);
    pl.st_sel_cnt = pl.st_rank + pl.n_rank_tiles;
    pl.st_sel_nnz = pl.st_sel_cnt + pl.n_sel_tiles;
    pl.st_colptr = (uint64_t *)(w + o_stc);
    pl.ctr = (DevCounters *)(w + o_ctr);
    pl.flop = (int64_t *)(w + o_flop);
    pl.sym_bin = (int32_t *)(w + o_sbin);
    pl.num_bin = (int32_t *)(w + o_nbin);
    pl.sym_list = (int32_t *)(w + o_slist);
    pl.num_list = (int32_t *)(w + o_nlist);
    pl.split = split_in_ws ? (int32_t *)(w + o_split) : nullptr;
    pl.tstart = (int64_t *)(w + o_tst);
    pl.col_slot = (int32_t *)(w + o_dsl);
    pl.arrive = (int32_t *)(w + o_arr);
    pl.tlen = (int32_t *)(w + o_tln);
    char *h = (char *)pl.pinned;
    pl.hctr = (DevCounters *)(h + h_ctr);
    {
        void *dev = nullptr;
        if (hipHostGetDevicePointer(&dev, pl.pinned, 0) != hipSuccess) {
            (void)hipGetLastError();
            pool_put(pl.ws, pl.ws_bytes, false, pl.device, pl.stream);
            pool_put(pl.pinned, pl.pinned_bytes, true, pl.device, pl.stream);
            delete p;
            return fail(SPGEMM_EHIP, "hipHostGetDevicePointer failed");
        }
        pl.hpub = (PublishedCounts *)(h + h_pub);
        pl.hpub_dev = (PublishedCounts *)((char *)dev + h_pub);
        pl.hflags = (uint32_t *)(h + h_flags);
        pl.hflags_dev = (uint32_t *)((char *)dev + h_flags);
        // group bases and rank tiles sit at the same offsets in both blocks:
        // k_plan_init copies them as one block of 8-byte words
        pl.up_src = (const uint64_t *)((char *)dev + h_gbase);
        pl.up_words = (int64_t)(((h_tiles - h_gbase) + sizeof(RankTile) * tiles.size()) / 8);
    }
    std::memcpy(h + h_gbase, gbase.data(), sizeof(int64_t) * (P + 1));
    if (!tiles.empty()) std::memcpy(h + h_tiles, tiles.data(), sizeof(RankTile) * tiles.size());

    auto cleanup = [&](int code) {
        (void)hipStreamSynchronize(pl.stream);
        pool_put(pl.ws, pl.ws_bytes, false, pl.device, pl.stream);
        pool_put(pl.pinned, pl.pinned_bytes, true, pl.device, pl.stream);
        delete p;
        return code;
    };
    static_assert(sizeof(RankTile) % 8 == 0 && sizeof(int64_t) == 8, "upload in 8-byte words");
    hipError_t e = hipSuccess;
    if (tun.validate) {
        e = hipMemsetAsync(pl.ctr, 0, sizeof(DevCounters), pl.stream);
        if (e != hipSuccess) return cleanup(fail(SPGEMM_EHIP, hipGetErrorString(e)));
        if ((rc = launch_validate(pl))) return cleanup(rc);
        if ((rc = sync_counters(pl))) return cleanup(rc);
        if (pl.hctr->error & 1) return cleanup(fail(SPGEMM_EINVAL, "A is not a valid CSC matrix "
                                                                   "(pointers or sorted unique rows)"));
        if (pl.hctr->error & 2) return cleanup(fail(SPGEMM_EINVAL, "Bi is not a valid CSC matrix "
                                                                   "(pointers or sorted unique rows)"));
    }
    if ((rc = launch_plan_kernels(pl))) return cleanup(rc);
    // sparse flops, term ranges and symbolic bins depend on the patterns
    // only: computed here, in one launch with the gather of A~, with their
    // counts on their way to the host by the time spgemm_symbolic needs them
    if (pl.n > 0) __atomic_store_n(pl.hflags + kFlagCounts, 0u, __ATOMIC_RELEASE);
    // the first symbolic run launches the tiny kernel before it has the
    // counts, and that launch publishes them
    pl.early_tiny = pl.n > 0 && pl.n <= kEarlyTinyCols && pl.th.tiny_max_flop > 0;
    if ((rc = launch_flop_bin_gather(pl))) return cleanup(rc);
    if (pl.n > 0) {
        e = take_event(&pl.counts_ready);
        if (e == hipSuccess) e = hipEventRecord(pl.counts_ready, pl.stream);
        if (e != hipSuccess)
            return cleanup(fail(SPGEMM_EHIP, std::string("plan counters: ") + hipGetErrorString(e)));
    }
    *out = p;
    return SPGEMM_OK;
}

int spgemm_plan_set_stream(spgemm_plan_t plan, void *stream) {
    (void)hipGetLastError();
    if (!plan) return fail(SPGEMM_EINVAL, "plan is NULL");
    Plan &p = *plan;
    const hipStream_t next = (hipStream_t)stream;
    if (next == p.stream) return SPGEMM_OK;
    // counts a symbolic phase publishes on the old stream are read before
    // the switch (their fallback wait synchronises the stream they ran on),
    // and the new stream's work starts after the old stream's
    if (int rc = finish_symbolic_counts(p)) return rc;
    hipEvent_t ev = nullptr;
    SPG_HIP(take_event(&ev));
    hipError_t e = hipEventRecord(ev, p.stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(next, ev, 0);
    {
        std::lock_guard<std::mutex> lk(g_pool_mtx);
        g_spare_events.push_back(ev);  // reusable once recorded again
    }
    if (e != hipSuccess) return fail(SPGEMM_EHIP, std::string("set_stream: ") + hipGetErrorString(e));
    p.stream = next;
    return SPGEMM_OK;
}

int spgemm_plan_stats(spgemm_plan_t plan, spgemm_stats *s) {
    if (!plan || !s) return fail(SPGEMM_EINVAL, "plan or stats is NULL");
    Plan &p = *plan;
    int rc = finish_symbolic_counts(p);
    if (rc) return rc;
    rc = sync_counters(p);
    if (rc) return rc;
    const DevCounters &c = *p.hctr;
    std::memset(s, 0, sizeof(*s));
    s->m = p.m;
    s->k = p.k;
    s->n = p.n;
    s->nnz_A = p.nnzA;
    s->nnz_B = p.nnzB;
    s->h_count = c.h_count;
    s->nzc_A = c.nzc;
    s->K = c.K;
    s->M = c.M;
    s->kt = c.kt;
    s->nnz_At = c.nnz_At;
    s->cv_memA = p.nnzA > 0 ? (double)c.nnz_At / (double)p.nnzA : 0.0;
    s->flops = p.symbolic_done ? p.flops : -1;
    s->nnz_C = p.symbolic_done ? p.nnzC : -1;
    for (int b = 0; b < kNumBins; ++b) {
        s->sym_bins[b] = p.symbolic_done ? p.sym_count[b] : 0;
        s->num_bins[b] = p.symbolic_done ? p.num_count[b] : 0;
    }
    return SPGEMM_OK;
}

int spgemm_plan_export(spgemm_plan_t plan, uint8_t *H, int32_t *map, int64_t *At_colptr,
                       int32_t *At_rowidx, void *At_vals, int64_t *blocks) {
    (void)hipGetLastError();  // drop errors left by other code on this thread
    if (!plan) return fail(SPGEMM_EINVAL, "plan is NULL");
    Plan &p = *plan;
    int rc = sync_counters(p);
    if (rc) return rc;
    const int64_t kt = p.hctr->kt, nt = p.hctr->nnz_At;
    if (H && p.k) SPG_HIP(hipMemcpyAsync(H, p.H, p.k, hipMemcpyDeviceToDevice, p.stream));
    if (map && p.k)
        SPG_HIP(hipMemcpyAsync(map, p.map, 4 * p.k, hipMemcpyDeviceToDevice, p.stream));
    if (At_colptr)
        SPG_HIP(hipMemcpyAsync(At_colptr, p.At_colptr, 8 * (kt + 1), hipMemcpyDeviceToDevice,
                               p.stream));
    if (At_rowidx && nt)
        SPG_HIP(hipMemcpyAsync(At_rowidx, p.At_rowidx, 4 * nt, hipMemcpyDeviceToDevice, p.stream));
    if (At_vals && nt)
        SPG_HIP(hipMemcpyAsync(At_vals, p.At_vals, p.vsize * nt, hipMemcpyDeviceToDevice,
                               p.stream));
    if (blocks && (rc = launch_export_blocks(p, blocks))) return rc;
    return SPGEMM_OK;
}

int spgemm_plan_export_bins(spgemm_plan_t plan, int64_t *flop, int32_t *sym_bin,
                            int32_t *num_bin) {
    (void)hipGetLastError();  // drop errors left by other code on this thread
    if (!plan) return fail(SPGEMM_EINVAL, "plan is NULL");
    Plan &p = *plan;
    if (!p.symbolic_done) return fail(SPGEMM_ESTATE, "spgemm_symbolic has not run on this plan");
    if (p.n == 0) return SPGEMM_OK;
    if (flop) SPG_HIP(hipMemcpyAsync(flop, p.flop, 8 * p.n, hipMemcpyDeviceToDevice, p.stream));
    if (sym_bin)
        SPG_HIP(hipMemcpyAsync(sym_bin, p.sym_bin, 4 * p.n, hipMemcpyDeviceToDevice, p.stream));
    if (num_bin)
        SPG_HIP(hipMemcpyAsync(num_bin, p.num_bin, 4 * p.n, hipMemcpyDeviceToDevice, p.stream));
    return SPGEMM_OK;
}

// The symbolic phase.  noalloc: what is kept for the numeric phase goes to
// the device's scratch array (nothing is allocated; SPGEMM_ENOMEM when it
// does not fit) instead of pooled blocks.
static int symbolic_impl(spgemm_plan_t plan, int64_t *C_colptr, int64_t *nnzC, bool noalloc) {
    (void)hipGetLastError();  // drop errors left by other code on this thread
    if (!plan) return fail(SPGEMM_EINVAL, "plan is NULL");
    if (!C_colptr || !nnzC) return fail(SPGEMM_EINVAL, "C_colptr and nnzC must not be NULL");
    Plan &p = *plan;
    int rc;
    // a previous run's late publish must land before the flags are reset
    if ((rc = finish_symbolic_counts(p))) return rc;
    p.C_colptr = C_colptr;
    p.symbolic_done = false;
    p.kept_in_scratch = false;
    p.tiny_perm = nullptr;
    p.dense_bits = nullptr;
    unsigned char *sbuf = nullptr;
    if (noalloc && p.n > 0) {
        void *addr = nullptr;
        if ((rc = scratch_take(p.device, &addr, &p.scratch_gen))) return rc;
        sbuf = (unsigned char *)addr;
        p.kept_in_scratch = true;
    }
    // the tiny part at the start of the array, the dense part after it
    auto scratch_tiny = [&](int64_t cols) {
        const size_t t = tiny_part_bytes(p, cols);
        p.tiny_perm = t ? (uint16_t *)sbuf : nullptr;
        return t;
    };
    size_t tiny_bytes = 0;
    if (p.n == 0) {
        SPG_HIP(hipMemsetAsync(C_colptr, 0, sizeof(int64_t), p.stream));
        p.nnzC = 0;
        p.flops = 0;
        for (int b = 0; b < kNumBins; ++b) p.sym_count[b] = p.num_count[b] = 0;
        p.symbolic_done = true;
        *nnzC = 0;
        return SPGEMM_OK;
    }
    // flops and symbolic bins came with the plan; a later run clears what the
    // previous symbolic run accumulated
    bool early = false;
    if (p.symbolic_runs++ == 0) {
        early = p.early_tiny;
        if (early) {
            if (noalloc) {
                // sized for every column (the counts are not known yet): at
                // most kEarlyTinyCols columns of 1 KiB, well inside the array
                tiny_bytes = scratch_tiny(p.n);
            } else {
                reserve_tiny(p, p.n);
            }
            if ((rc = launch_sym_tiny(p, true))) return rc;  // publishes the counts
        }
        SPG_HIP(wait_flag(p, kFlagCounts, [&] {
            return early ? hipStreamSynchronize(p.stream) : hipEventSynchronize(p.counts_ready);
        }));
        for (int b = 0; b < kNumBins; ++b) p.sym_count[b] = p.hpub->sym_count[b];
        p.nnzAt_pub = p.hpub->nnz_At;
    } else if ((rc = launch_symbolic_reset(p))) {
        return rc;
    }
    if (noalloc) {
        if (!early) tiny_bytes = scratch_tiny(p.sym_count[kBinTiny]);
        const size_t at = (tiny_bytes + 255) & ~(size_t)255;
        const size_t dense = dense_part_bytes(p);
        if (at + dense > kScratchBytes)
            return fail(SPGEMM_ENOMEM,
                        "spgemm_symbolic_noalloc needs " + std::to_string(at + dense) +
                            " bytes of scratch for the kept sort orders and row bitmaps, above its " +
                            std::to_string(kScratchBytes) + " bytes; use spgemm_symbolic");
        p.dense_bits = dense ? (uint32_t *)(sbuf + at) : nullptr;
        // the bands of a tall plan's dense columns need the split table,
        // which this entry point cannot allocate
        if (p.m > kMaxDenseRows && p.sym_count[kBinDense] > 0 && !p.split)
            return fail(SPGEMM_ENOMEM,
                        "a plan of more than 262144 rows with dense columns needs its split "
                        "table (" + std::to_string(split_table_bytes(p)) +
                            " bytes), which one spgemm_symbolic run builds first");
    } else {
        if (!early) reserve_tiny(p, p.sym_count[kBinTiny]);
        reserve_dense(p);
    }
    if ((rc = launch_symbolic_bins(p, early))) return rc;
    __atomic_store_n(p.hflags + kFlagColptr, 0u, __ATOMIC_RELEASE);
    // the one-workgroup scan stores nnz(C_i) + 1 ahead of the rest: return
    // it as soon as it lands and collect the rest when it is needed
    uint64_t *hnnz = reinterpret_cast<uint64_t *>(p.hflags + kNnzSlot);
    const bool small = p.n <= kSmallScanCols;
    if (small) __atomic_store_n(hnnz, (uint64_t)0, __ATOMIC_RELEASE);
    if ((rc = launch_colptr_scan(p))) return rc;  // publishes its counters to hpub
    if (small) {
        const auto t0 = std::chrono::steady_clock::now();
        uint64_t v = 0;
        for (unsigned i = 0; (v = __atomic_load_n(hnnz, __ATOMIC_ACQUIRE)) == 0; ++i) {
            if ((i & 255u) == 255u &&
                std::chrono::steady_clock::now() - t0 > std::chrono::microseconds(kSpinMicros)) {
                SPG_HIP(hipStreamSynchronize(p.stream));
                v = __atomic_load_n(hnnz, __ATOMIC_ACQUIRE);
                break;
            }
            __builtin_ia32_pause();
        }
        if (v == 0) return fail(SPGEMM_EHIP, "the column-pointer scan did not report nnz(C_i)");
        p.nnzC = (int64_t)(v - 1);
        p.counts_pending = true;
    } else {
        SPG_HIP(wait_flag(p, kFlagColptr, [&] { return hipStreamSynchronize(p.stream); }));
        p.nnzC = p.hpub->nnzC;
        p.flops = p.hpub->flops;
        for (int b = 0; b < kNumBins; ++b) p.num_count[b] = p.hpub->num_count[b];
        p.counts_pending = false;
    }
    p.symbolic_done = true;
    *nnzC = p.nnzC;
    return SPGEMM_OK;
}

int spgemm_symbolic(spgemm_plan_t plan, int64_t *C_colptr, int64_t *nnzC) {
    return symbolic_impl(plan, C_colptr, nnzC, false);
}

int spgemm_symbolic_noalloc(spgemm_plan_t plan, int64_t *C_colptr, int64_t *nnzC) {
    return symbolic_impl(plan, C_colptr, nnzC, true);
}

int spgemm_numeric(spgemm_plan_t plan, const void *A_vals, const void *Bi_vals,
                   int32_t *C_rowidx, void *C_vals) {
    (void)hipGetLastError();  // drop errors left by other code on this thread
    if (!plan) return fail(SPGEMM_EINVAL, "plan is NULL");
    Plan &p = *plan;
    if (!p.symbolic_done) return fail(SPGEMM_ESTATE, "spgemm_numeric needs spgemm_symbolic first");
    int rc0;
    if ((rc0 = check_kept(p)) || (rc0 = finish_symbolic_counts(p))) return rc0;
    if (p.nnzC > 0 && (!C_rowidx || !C_vals))
        return fail(SPGEMM_EINVAL, "C_rowidx and C_vals must not be NULL");
    const void *Bv = Bi_vals ? Bi_vals : p.Bvals;
    if (p.nnzC > 0 && !Bv) return fail(SPGEMM_EINVAL, "no values for B_i");
    if (!A_vals && !p.Avals && p.nnzC > 0) return fail(SPGEMM_EINVAL, "no values for A");
    int rc;
    const void *Atv = nullptr;
    if ((rc = take_new_a_values(p, A_vals, &Atv))) return rc;
    if ((rc = ensure_split_table(p))) return rc;
    return launch_numeric_bins(p, Bv, C_rowidx, C_vals, Atv);
}

int spgemm_backward(spgemm_plan_t plan, const int64_t *C_colptr, const int32_t *C_rowidx,
                    const void *A_vals, const void *Bi_vals, const void *dC_vals, void *dA_vals,
                    void *dB_vals) {
    (void)hipGetLastError();  // drop errors left by other code on this thread
    if (!plan) return fail(SPGEMM_EINVAL, "plan is NULL");
    Plan &p = *plan;
    if (!p.symbolic_done) return fail(SPGEMM_ESTATE, "spgemm_backward needs spgemm_symbolic first");
    int rc0;
    if ((rc0 = check_kept(p)) || (rc0 = finish_symbolic_counts(p))) return rc0;
    if (!dA_vals && !dB_vals) return SPGEMM_OK;
    const void *Av = A_vals ? A_vals : p.Avals;
    const void *Bv = Bi_vals ? Bi_vals : p.Bvals;
    if (!C_colptr) return fail(SPGEMM_EINVAL, "C_colptr is NULL");
    if (p.nnzC > 0 && (!C_rowidx || !dC_vals))
        return fail(SPGEMM_EINVAL, "C_rowidx and dC_vals must not be NULL");
    if ((p.nnzA > 0 && !Av) || (p.nnzB > 0 && !Bv))
        return fail(SPGEMM_EINVAL, "backward needs the values of A and B_i");
    return launch_backward(p, C_colptr, C_rowidx, Av, Bv, dC_vals, dA_vals, dB_vals);
}

int spgemm_plan_destroy(spgemm_plan_t plan) {
    if (!plan) return SPGEMM_OK;
    Plan &p = *plan;
    // the scan's publish into the pinned block lands before the block is reused
    (void)finish_symbolic_counts(p);
    batch_cache_drop(plan);
    pool_put(p.ws, p.ws_bytes, false, p.device, p.stream);
    // the pinned block's last device-side use is the counters copy that
    // counts_ready follows (later copies were waited for on the host)
    pool_put(p.pinned, p.pinned_bytes, true, p.device, p.stream, p.counts_ready);
    pool_put(p.kept, p.kept_bytes, false, p.device, p.stream);
    pool_put(p.kept_tiny, p.kept_tiny_bytes, false, p.device, p.stream);
    pool_put(p.split_block, p.split_bytes, false, p.device, p.stream);
    delete plan;
    return SPGEMM_OK;
}

}  // extern "C"
