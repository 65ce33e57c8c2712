// Grouped numeric launches of the batched form: at one dependency depth, the
// tiny columns of all products that have no dense columns go to ONE launch,
// and so do the columns of each medium bin that the plain path gives to one
// kernel (LDS hash, or LDS bitmap over all rows), instead of one launch per
// product and bin.  Products of one depth are independent, so the grouped
// launches need no waits inside; a depth of many small products then fills
// the device with a few launches.
#pragma once

#include <vector>

#include "internal.hpp"

namespace spg {

// One grouped launch: columns of bin `bin` over `np` of the depth's members.
struct GroupedLaunch {
    int kind = 0;          // 0 tiny, 1 LDS hash, 2 LDS bitmap
    int bin = 0;
    int np = 0;            // members with columns in this launch
    int64_t total = 0;     // columns
    size_t lds = 0;        // bitmap: dynamic LDS bytes (the largest member's)
    bool wide = false;     // bitmap: a member has more than 65536 rows (512 threads)
    size_t offset = 0;     // byte offset of its column table in the table block
};

// One depth's grouped products and their device tables.
struct GroupedDepth {
    std::vector<int> members;            // product indices (host)
    spgemm_dtype dtype = SPGEMM_F64;
    std::vector<GroupedLaunch> launches;  // in launch order
    void *table = nullptr;               // device: per member its numeric arguments, then
                                         // each launch's column table (member
                                         // slot << 32 | column of B_i, one entry per column)
};

// A product the grouped launches take: at most kGroupMaxCols columns (a
// larger product fills its own launches, which then run beside the grouped
// ones on side streams; measured: 64 ER products of 1e3-5e4 columns ran
// 12 % slower all grouped than all separate, while 256 and 1024 products of
// up to 2000 columns ran 5x and 12x faster grouped), no dense columns, and
// tiny columns of at most 256 products.
constexpr int64_t kGroupMaxCols = 4096;
bool groupable(const Plan &p);

// Builds the device tables for `members` (counts final, bin lists written),
// choosing per member and medium bin the kernel its plain numeric phase
// uses.  New A values are read in place or gathered into A~ exactly as
// spgemm_numeric does; the caller enqueues the value gathers before
// grouped_launch.
int grouped_build(const std::vector<Plan *> &plans, const std::vector<spgemm_batch_io> &io,
                  const std::vector<int> &members, GroupedDepth &g);

// Enqueues the depth's grouped launches, launch k on streams[k % size]
// (independent launches: tiny columns beside the medium bins).
int grouped_launch(const GroupedDepth &g, const std::vector<hipStream_t> &streams);

void grouped_free(GroupedDepth &g);

}  // namespace spg
