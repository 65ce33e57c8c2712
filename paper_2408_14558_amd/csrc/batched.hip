// placeholder, replaced below
#include "internal.hpp"
using namespace spg;
extern "C" {
int spgemm_batch_create(int32_t, const spgemm_plan_t *, const spgemm_batch_io *,
                        const spgemm_tuning *, spgemm_batch_t *) {
    return fail(SPGEMM_EUNSUPPORTED, "batched not built");
}
int spgemm_batched(spgemm_batch_t, int32_t, void *) { return SPGEMM_EUNSUPPORTED; }
int spgemm_batch_info(spgemm_batch_t, int64_t *, int64_t *) { return SPGEMM_EUNSUPPORTED; }
int spgemm_batch_destroy(spgemm_batch_t) { return SPGEMM_OK; }
}
