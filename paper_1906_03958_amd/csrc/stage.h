// stage.h -- per-stage kernels for networks too large for one workgroup:
// every RK4 stage is one launch over the whole chip, the synaptic product a
// float32 MFMA GEMM over the trials of a shared network.
#pragma once

#include "../../include/psst.h"
#include "kernels.h"

struct StageBatch;

psst_status stage_integrate_single(psst_network *net, float *state, const psst_stimulus *stim,
                                   float dt, int64_t n_steps, int64_t step0,
                                   const psst_record *rec, void *stream);
psst_status stage_batch_create(psst_network *net, int32_t n_trials, StageBatch **out);
void stage_batch_free(StageBatch *sb);
const char *stage_batch_describe(const StageBatch *sb);
psst_status stage_batch_integrate(StageBatch *sb, float *states, const psst_stimulus *stim,
                                  float dt, int64_t n_steps, int64_t step0,
                                  const psst_record *rec, float *ckpt, int32_t K, void *stream);
psst_status stage_batch_poll(StageBatch *sb, void *stream);
