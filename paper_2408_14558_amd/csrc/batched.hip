// Batched numeric phase: the numeric work of many planned products (uneven
// sizes, optionally chained like the two products of every AMG Galerkin
// level) issued as one dependency DAG of the per-bin kernels, optionally
// captured once into a hipGraph and replayed; or, with
// tuning.batch_form = 1, as one persistent launch (persistent.hip).
//
// Products are ordered by dependency depth (a product's depth is one more
// than the deepest product it reads).  Products of one depth are
// independent.  With batch_form = 0, the depth's products without dense
// columns (at least two of them) share one launch per numeric bin and
// kernel (grouped.hip), after their value gathers; the depth's other
// products are spread round-robin over side streams forked from the
// caller's stream and joined back before the next depth starts, each running
// exactly the kernels of its plain spgemm_numeric call (value gather of A~
// when new A values are given, then one launch per non-empty numeric bin).
// batch_form = 2 runs every product that way.  A depth never starts before
// the products it reads have finished.
#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "grouped.hpp"

using namespace spg;

namespace {

constexpr int kMaxBatchStreams = 8;
constexpr int kDefaultBatchStreams = 4;

}  // namespace

struct spgemm_batch_s {
    int device = 0;
    spgemm_dtype dtype = SPGEMM_F64;
    std::vector<spgemm_plan_t> plans;
    std::vector<spgemm_batch_io> io;
    std::vector<std::vector<int>> levels;  // product indices per depth
    std::vector<hipStream_t> side;         // default priority, non-blocking
    std::vector<hipEvent_t> fork, join;    // one fork event, one join event per side stream
    int64_t launches = 0;                  // kernels one run enqueues
    std::vector<GroupedDepth> groups;      // per depth: its grouped products (np = 0: none)
    bool persistent = false;               // one persistent launch per run
    PersistentBatch pb;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

// Whether product t gathers new A values into A~ before its numeric phase.
static bool gathers_values(const Plan &p, const spgemm_batch_io &io) {
    return io.A_vals && p.k > 0 && p.nnzA > 0 && p.nnzAt_pub != p.nnzA;
}

// Kernels product t enqueues per run (for spgemm_batch_info).
static int64_t product_launches(const Plan &p, const spgemm_batch_io &io) {
    int64_t n = gathers_values(p, io) ? 1 : 0;
    if (p.n == 0 || p.nnzC == 0) return n;
    for (int bin = kBinTiny; bin < kBinDense; ++bin) n += p.num_count[bin] > 0;
    n += p.num_count[kBinDense] + p.num_count[kBinDenseFirst] > 0;  // one launch serves both
    return n;
}

// Enqueues product t on stream s: the plan's kernels run on s for this call
// only (the plan's own stream is restored afterwards).
static int run_product(spgemm_batch_s &b, int t, hipStream_t s) {
    Plan &p = *b.plans[t];
    const spgemm_batch_io &io = b.io[t];
    const hipStream_t keep = p.stream;
    p.stream = s;
    const void *Atv = nullptr;
    int rc = take_new_a_values(p, io.A_vals, &Atv);
    if (!rc)
        rc = launch_numeric_bins(p, io.B_vals ? io.B_vals : p.Bvals, io.C_rowidx, io.C_vals, Atv);
    p.stream = keep;
    return rc;
}

// Enqueues the value gathers of a depth's grouped products on s.
static int grouped_gathers(spgemm_batch_s &b, const GroupedDepth &g, hipStream_t s) {
    for (int t : g.members) {
        Plan &p = *b.plans[t];
        if (!gathers_values(p, b.io[t])) continue;
        const hipStream_t keep = p.stream;
        p.stream = s;
        const int rc = launch_gather_values(p, b.io[t].A_vals);
        p.stream = keep;
        if (rc) return rc;
    }
    return SPGEMM_OK;
}

// Enqueues the whole DAG on s (eagerly, or into a capture that s is in).
// At a depth, the grouped products' value gathers go first on s; then the
// other products and the grouped launches share s and the side streams.
static int enqueue_dag(spgemm_batch_s &b, hipStream_t s) {
    if (b.persistent) return persistent_launch(b.pb, s);
    for (size_t d = 0; d < b.levels.size(); ++d) {
        const std::vector<int> &lvl = b.levels[d];
        const GroupedDepth &g = b.groups[d];
        std::vector<int> rest;  // products that run their own kernels
        for (int t : lvl)
            if (std::find(g.members.begin(), g.members.end(), t) == g.members.end())
                rest.push_back(t);
        if (int rc = grouped_gathers(b, g, s)) return rc;
        const size_t jobs = rest.size() + g.launches.size();
        const int width = std::min<int>((int)b.side.size(), (int)jobs - 1);
        if (width <= 0) {
            if (int rc = grouped_launch(g, {s})) return rc;
            for (int t : rest)
                if (int rc = run_product(b, t, s)) return rc;
            continue;
        }
        SPG_HIP(hipEventRecord(b.fork[0], s));
        for (int i = 0; i < width; ++i) SPG_HIP(hipStreamWaitEvent(b.side[i], b.fork[0], 0));
        // s and the side streams in turn: the grouped launches first, then
        // the other products
        std::vector<hipStream_t> all(1, s);
        all.insert(all.end(), b.side.begin(), b.side.begin() + width);
        if (int rc = grouped_launch(g, all)) return rc;
        for (size_t u = 0; u < rest.size(); ++u)
            if (int rc = run_product(b, rest[u], all[(g.launches.size() + u) % all.size()]))
                return rc;
        for (int i = 0; i < width; ++i) {
            SPG_HIP(hipEventRecord(b.join[i], b.side[i]));
            SPG_HIP(hipStreamWaitEvent(s, b.join[i], 0));
        }
    }
    return SPGEMM_OK;
}

static void release(spgemm_batch_s *b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (hipEvent_t e : b->fork) (void)hipEventDestroy(e);
    for (hipEvent_t e : b->join) (void)hipEventDestroy(e);
    for (hipStream_t st : b->side) (void)hipStreamDestroy(st);
    for (GroupedDepth &g : b->groups) grouped_free(g);
    persistent_free(b->pb);
    delete b;
}

// The batches spgemm_batched builds for itself, one per distinct (plans, io)
// table, so a capture (mode 1) and its replays (mode 2) meet the same graph.
// A batch is dropped when one of its plans is destroyed.
namespace {
struct CachedBatch {
    std::vector<spgemm_plan_t> plans;
    std::vector<spgemm_batch_io> io;
    spgemm_batch_t batch;
};
std::mutex g_cache_mtx;
std::vector<CachedBatch> g_cache;

bool same_io(const spgemm_batch_io &a, const spgemm_batch_io &b) {
    return a.A_vals == b.A_vals && a.B_vals == b.B_vals && a.C_rowidx == b.C_rowidx &&
           a.C_vals == b.C_vals && a.dep_A == b.dep_A && a.dep_B == b.dep_B;
}
}  // namespace

namespace spg {
void batch_cache_drop(const Plan *plan) {
    std::vector<spgemm_batch_t> gone;
    {
        std::lock_guard<std::mutex> lk(g_cache_mtx);
        for (size_t i = 0; i < g_cache.size();) {
            const auto &pl = g_cache[i].plans;
            if (std::find(pl.begin(), pl.end(), plan) != pl.end()) {
                gone.push_back(g_cache[i].batch);
                g_cache.erase(g_cache.begin() + i);
            } else {
                ++i;
            }
        }
    }
    for (spgemm_batch_t b : gone) {
        (void)hipDeviceSynchronize();
        release(b);
    }
}
}  // namespace spg

extern "C" {

int spgemm_batch_create(int32_t count, const spgemm_plan_t *plans, const spgemm_batch_io *io,
                        const spgemm_tuning *tuning, spgemm_batch_t *out) {
    (void)hipGetLastError();
    if (!out) return fail(SPGEMM_EINVAL, "out is NULL");
    *out = nullptr;
    if (count < 1 || !plans || !io) return fail(SPGEMM_EINVAL, "need count >= 1, plans and io");
    spgemm_tuning tun;
    spgemm_default_tuning(&tun);
    if (tuning) tun = *tuning;
    if (tun.batch_form < 0 || tun.batch_form > 2)
        return fail(SPGEMM_EINVAL, "batch_form must be 0, 1 or 2");
    if (tun.batch_streams < 0 || tun.batch_streams > kMaxBatchStreams)
        return fail(SPGEMM_EINVAL, "batch_streams must be in 0..8");
    const spgemm_dtype dt = plans[0] ? plans[0]->dtype : SPGEMM_F64;
    std::vector<int> depth(count, 0);
    for (int t = 0; t < count; ++t) {
        const spgemm_plan_t p = plans[t];
        const std::string who = "product " + std::to_string(t);
        if (!p) return fail(SPGEMM_EINVAL, who + ": plan is NULL");
        if (!p->symbolic_done) return fail(SPGEMM_ESTATE, who + " has not run symbolic");
        if (int rc = check_kept(*p)) return rc;
        if (int rc = finish_symbolic_counts(*p)) return rc;
        if (int rc = ensure_split_table(*p)) return rc;  // on the plan's stream, before the sync
        if (p->dtype != dt) return fail(SPGEMM_EINVAL, "plans must share one dtype");
        for (int u = 0; u < t; ++u)
            if (plans[u] == p)
                return fail(SPGEMM_EINVAL, who + " repeats the plan of product " + std::to_string(u));
        if (io[t].dep_A >= t || io[t].dep_B >= t || io[t].dep_A < -1 || io[t].dep_B < -1)
            return fail(SPGEMM_EINVAL, "dependencies must point to lower indices");
        if (p->nnzC > 0 && (!io[t].C_rowidx || !io[t].C_vals))
            return fail(SPGEMM_EINVAL, who + " has no C buffers");
        if (p->nnzC > 0 && !io[t].B_vals && !p->Bvals)
            return fail(SPGEMM_EINVAL, who + " has no B values");
        if (p->nnzC > 0 && !io[t].A_vals && !p->Avals)
            return fail(SPGEMM_EINVAL, who + " has no A values");
        if (io[t].dep_A >= 0 && !io[t].A_vals)
            return fail(SPGEMM_EINVAL, "a product whose A is another product's C needs A_vals");
        if (io[t].dep_B >= 0 && !io[t].B_vals)
            return fail(SPGEMM_EINVAL, "a product whose B is another product's C needs B_vals");
        if (io[t].dep_A >= 0) depth[t] = std::max(depth[t], depth[io[t].dep_A] + 1);
        if (io[t].dep_B >= 0) depth[t] = std::max(depth[t], depth[io[t].dep_B] + 1);
    }
    auto *b = new (std::nothrow) spgemm_batch_s();
    if (!b) return fail(SPGEMM_ENOMEM, "batch allocation failed");
    b->dtype = dt;
    b->plans.assign(plans, plans + count);
    b->io.assign(io, io + count);
    const int levels = *std::max_element(depth.begin(), depth.end()) + 1;
    b->levels.resize(levels);
    for (int t = 0; t < count; ++t) {
        b->levels[depth[t]].push_back(t);
        b->launches += product_launches(*plans[t], io[t]);
    }
    hipError_t e = hipGetDevice(&b->device);
    // the products' symbolic phases (bin lists, counts) ran on the plans'
    // streams: finished before any table is built from them
    for (int t = 0; t < count && e == hipSuccess; ++t) e = hipStreamSynchronize(plans[t]->stream);
    if (e == hipSuccess && tun.batch_form == 1) {
        std::vector<Plan *> pv(plans, plans + count);
        std::vector<spgemm_batch_io> iov(io, io + count);
        if (int rc = persistent_build(pv, iov, b->levels, b->pb)) {
            release(b);
            return rc;
        }
        b->persistent = true;
        b->launches = b->pb.nitems > 0 ? 1 : 0;
        *out = b;
        return SPGEMM_OK;
    }
    // grouped launches: at each depth, the products without dense columns,
    // when there are at least two
    b->groups.resize(b->levels.size());
    if (e == hipSuccess && tun.batch_form == 0) {
        std::vector<Plan *> pv(plans, plans + count);
        std::vector<spgemm_batch_io> iov(io, io + count);
        for (size_t d = 0; d < b->levels.size(); ++d) {
            std::vector<int> members;
            for (int t : b->levels[d]) {
                const Plan &p = *plans[t];
                if (p.n > 0 && p.nnzC > 0 && groupable(p)) members.push_back(t);
            }
            if (members.size() < 2) continue;
            if (int rc = grouped_build(pv, iov, members, b->groups[d])) {
                release(b);
                return rc;
            }
            for (int t : members) b->launches -= product_launches(*plans[t], io[t]);
            for (int t : members) b->launches += gathers_values(*plans[t], io[t]) ? 1 : 0;
            b->launches += (int64_t)b->groups[d].launches.size();
        }
    }
    // side streams: one fewer than the most jobs of a depth (products that
    // run their own kernels, and grouped launches), s taking one of them
    size_t widest = 0;
    for (size_t d = 0; d < b->levels.size(); ++d)
        widest = std::max(widest, b->levels[d].size() - b->groups[d].members.size() +
                                      b->groups[d].launches.size());
    const int nside = (int)std::min<size_t>(
        widest > 1 ? widest - 1 : 0, tun.batch_streams ? tun.batch_streams : kDefaultBatchStreams);
    for (int i = 0; i < nside && e == hipSuccess; ++i) {
        hipStream_t st = nullptr;
        hipEvent_t ev = nullptr;
        e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (e == hipSuccess) b->side.push_back(st);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e == hipSuccess) b->join.push_back(ev);
    }
    if (e == hipSuccess && nside > 0) {
        hipEvent_t ev = nullptr;
        e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e == hipSuccess) b->fork.push_back(ev);
    }
    if (e != hipSuccess) {
        release(b);
        return fail(SPGEMM_EHIP, std::string("batch set-up: ") + hipGetErrorString(e));
    }
    *out = b;
    return SPGEMM_OK;
}

int spgemm_batch_run(spgemm_batch_t b, int32_t mode, void *stream) {
    (void)hipGetLastError();
    if (!b) return fail(SPGEMM_EINVAL, "batch is NULL");
    hipStream_t s = (hipStream_t)stream;
    if (mode == 0) return enqueue_dag(*b, s);
    if (mode == 1) {
        if (b->exec) {
            SPG_HIP(hipGraphExecDestroy(b->exec));
            b->exec = nullptr;
        }
        if (b->graph) {
            SPG_HIP(hipGraphDestroy(b->graph));
            b->graph = nullptr;
        }
        SPG_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        const int rc = enqueue_dag(*b, s);
        hipGraph_t g = nullptr;
        const hipError_t ee = hipStreamEndCapture(s, &g);
        if (rc) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (ee != hipSuccess)
            return fail(SPGEMM_EHIP, std::string("end capture: ") + hipGetErrorString(ee));
        b->graph = g;
        SPG_HIP(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0));
        SPG_HIP(hipGraphLaunch(b->exec, s));
        return SPGEMM_OK;
    }
    if (mode == 2) {
        if (!b->exec) return fail(SPGEMM_ESTATE, "replay needs a captured graph (mode 1) first");
        SPG_HIP(hipGraphLaunch(b->exec, s));
        return SPGEMM_OK;
    }
    return fail(SPGEMM_EINVAL, "mode must be 0, 1 or 2");
}

int spgemm_batched(int32_t count, const spgemm_plan_t *plans, const spgemm_batch_io *io,
                   int32_t mode, void *stream) {
    (void)hipGetLastError();
    if (count < 1 || !plans || !io) return fail(SPGEMM_EINVAL, "need count >= 1, plans and io");
    if (mode < 0 || mode > 2) return fail(SPGEMM_EINVAL, "mode must be 0, 1 or 2");
    spgemm_batch_t b = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_cache_mtx);
        for (const CachedBatch &c : g_cache) {
            if ((int32_t)c.plans.size() != count) continue;
            bool same = true;
            for (int32_t t = 0; t < count && same; ++t)
                same = c.plans[t] == plans[t] && same_io(c.io[t], io[t]);
            if (same) {
                b = c.batch;
                break;
            }
        }
        if (!b) {
            if (mode == 2)
                return fail(SPGEMM_ESTATE, "replay needs a capture (mode 1) of the same table first");
            // the batch fields (side streams, persistent launch) come from
            // the first plan's tuning, which the autotuner fills
            spgemm_tuning tun;
            spgemm_default_tuning(&tun);
            if (plans[0]) {
                tun.batch_streams = plans[0]->tun.batch_streams;
                tun.batch_form = plans[0]->tun.batch_form;
            }
            if (int rc = spgemm_batch_create(count, plans, io, &tun, &b)) return rc;
            g_cache.push_back(CachedBatch{std::vector<spgemm_plan_t>(plans, plans + count),
                                          std::vector<spgemm_batch_io>(io, io + count), b});
        }
    }
    return spgemm_batch_run(b, mode, stream);
}

int spgemm_batch_info(spgemm_batch_t b, int64_t *streams, int64_t *launches) {
    if (!b) return fail(SPGEMM_EINVAL, "batch is NULL");
    if (streams) *streams = (int64_t)b->side.size();
    if (launches) *launches = b->launches;
    return SPGEMM_OK;
}

int spgemm_batch_check(spgemm_batch_t b) {
    (void)hipGetLastError();
    if (!b) return fail(SPGEMM_EINVAL, "batch is NULL");
    SPG_HIP(hipDeviceSynchronize());
    if (b->persistent) {
        unsigned err = 0;
        if (int rc = persistent_error(b->pb, &err)) return rc;
        if (err)
            return fail(SPGEMM_EHIP, "a dependency wait of the persistent batch ran out of time; "
                                     "its outputs are not valid (the error is cleared)");
    }
    return SPGEMM_OK;
}

int spgemm_batch_destroy(spgemm_batch_t b) {
    if (!b) return SPGEMM_OK;
    (void)hipDeviceSynchronize();
    release(b);
    return SPGEMM_OK;
}

}  // extern "C"
