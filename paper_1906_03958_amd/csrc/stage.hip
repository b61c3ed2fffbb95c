// stage.hip -- per-stage launches for large shared networks (placeholder
// until the MFMA stage kernel lands).
#include "stage.h"

struct StageBatch {
    int dummy;
};

psst_status stage_integrate_single(psst_network *, float *, const psst_stimulus *, float, int64_t,
                                   int64_t, const psst_record *, void *)
{
    return PSST_ERR_UNSUPPORTED;
}
psst_status stage_batch_create(psst_network *, int32_t, StageBatch **out)
{
    *out = nullptr;
    return PSST_ERR_UNSUPPORTED;
}
void stage_batch_free(StageBatch *sb) { delete sb; }
const char *stage_batch_describe(const StageBatch *) { return ""; }
psst_status stage_batch_integrate(StageBatch *, float *, const psst_stimulus *, float, int64_t,
                                  int64_t, const psst_record *, float *, int32_t, void *)
{
    return PSST_ERR_UNSUPPORTED;
}
psst_status stage_batch_poll(StageBatch *, void *) { return PSST_ERR_UNSUPPORTED; }
