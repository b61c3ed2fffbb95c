// stage.h -- per-stage path for networks too large for one workgroup: each
// RK4 stage is one launch over the whole chip whose synaptic product is a
// float32 matrix-core GEMM over the trials of a shared network
// ("Circumventing memory constraints", item 1: synaptic coupling as a matrix
// multiplication), with the per-neuron right-hand side and the RK4 update
// fused into the GEMM epilogue.
#pragma once

#include "runtime.h"

// Device layout of a large network: conductances row-major [Mp][Kp] (post
// row i, presynaptic column k) in nS, the presynaptic axis cut into padded
// blocks: cholinergic PN columns [0, ka), fast-GABA LN columns [ka, ka + kg),
// slow-GABA LN columns [ka + kg, Kp).  Padding rows and columns are zero.
//
// Sparse storage keeps, instead of G, the synapses themselves grouped by
// (64-row block rb, 128-column tile kt, row r of the block): bucket
// (rb * ntl + kt) * 64 + r holds row 64 rb + r's synapses in tile kt, by
// ascending column -- sp_off[bucket] .. sp_off[bucket + 1] - 1 index sp_col
// (the column within the tile; read by in-place updates only) and sp_val
// (nS); sp_mask[4 bucket .. 4 bucket + 3] has bit c set for each column c of
// the tile the bucket holds, so a synapse's place in its bucket is the count
// of set bits below its column.
struct StageNet {
    float *G = nullptr;
    int n = 0, n_pn = 0, Mp = 0, Kp = 0, ka = 0, kg = 0, kb = 0;
    bool gabab = false;
    bool sparse = false;
    int32_t *sp_off = nullptr;
    uint8_t *sp_col = nullptr;
    float *sp_val = nullptr;
    uint32_t *sp_mask = nullptr;   // per bucket: which of the tile's 128 columns it holds
    int64_t nnz = 0;
};

// Build the layout on the device from the (validated) pathways: dense, or
// (sparse = true) the synapse buckets.
psst_status stage_net_create(psst_network *net, const psst_pathway *paths, int32_t np,
                             bool sparse = false);
void stage_net_free(StageNet *sn);

// The one-trial stage batch of a large network (for psst_integrate).
psst_status stage_single_prepare(psst_network *net);
psst_status stage_integrate_single(psst_network *net, float *state, const psst_stimulus *stim,
                                   float dt, int64_t n_steps, int64_t step0,
                                   const psst_record *rec, void *stream);
// n_trials trials of net; st_stride > 0 and st_off place them inside a larger
// batch's state, stimulus and record arrays (plane stride, first trial's
// offset: trial b's neuron i at st_off + b * n + i).
psst_status stage_batch_create(psst_network *net, int32_t n_trials, StageBatch **out,
                               int64_t st_stride = 0, int64_t st_off = 0);
// The batch's non-finite flag (the caller's, or its own when flag is NULL).
void stage_batch_use_flag(StageBatch *sb, int32_t *flag);
void stage_batch_free(StageBatch *sb);
const char *stage_batch_describe(const StageBatch *sb);
psst_status stage_batch_integrate(StageBatch *sb, float *states, const psst_stimulus *stim,
                                  float dt, int64_t n_steps, int64_t step0,
                                  const psst_record *rec, float *ckpt, int32_t K, void *stream);
psst_status stage_batch_poll(StageBatch *sb, void *stream);
// Bytes of the conductances one stage launch reads (the padded matrix once
// per tile of trials, or the synapse buckets).
int64_t stage_batch_matrix_bytes(const StageBatch *sb);
// Switch between classical RK4 (gen = false) and a generic explicit method;
// the step graph is rebuilt on the next call.
void stage_batch_set_method(StageBatch *sb, bool gen, const psst::Tab &tab);
