// runtime.h -- library-internal handle types and error helpers shared by the
// host files of the runtime.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <functional>
#include <string>
#include <vector>

#include "../../include/psst.h"
#include "kernels.h"

namespace psst {
// Record a thread-local error message and return the status.
psst_status fail(psst_status s, const char *fmt, ...);
}  // namespace psst

#define HIPCHK(call)                                                              \
    do {                                                                          \
        hipError_t e_ = (call);                                                   \
        if (e_ != hipSuccess)                                                     \
            return psst::fail(e_ == hipErrorOutOfMemory ? PSST_ERR_OUT_OF_MEMORY  \
                                                        : PSST_ERR_DEVICE,        \
                              "%s failed: %s", #call, hipGetErrorString(e_));     \
    } while (0)

struct StageNet;
struct StageBatch;
struct AdjWork;
struct StreamBufs;
void stream_bufs_free(StreamBufs *s);

using psst::InstDesc;
using psst::WGArgs;

namespace psst {
// Arguments of the in-place conductance update (network.hip): values in the
// gradient layout scattered into each storage the network keeps (NULL
// pointers: that storage is absent, or those values are left as they are).
struct NetUpdateArgs {
    const float *g;                 // [entries] pathway blocks, or NULL
    const float *g_na, *g_k, *g_l;  // [n] each, or NULL
    const int64_t *paths;           // [n_paths][6]: type, pre0, pre1, post0, post1, offset
    const uint32_t *present_bits;   // bit e: entry e is a synapse (NULL: all are)
    int64_t entries;
    int32_t n_paths, n, n_pn, ld;
    float *gt, *gtb;                // dense transposed matrices
    float *sp_val;                  // sparse rows and each entry's slot (-1: absent)
    const int32_t *sp_slot;
    float *stage_G;                 // per-stage layout [Mp x Kp]
    int64_t stage_Kp, stage_ka, stage_kg;
    const int32_t *bk_off;          // per-stage sparse layout: synapse buckets
    const uint8_t *bk_col;
    float *bk_val;
    float *prm;                     // [NPRM][ld]
};
}  // namespace psst
psst_status network_update_launch(const psst::NetUpdateArgs &a, hipStream_t s);

struct PathInfo {
    int32_t type, pre0, pre1, post0, post1;
    int64_t grad_off;   // offset of this block in a grad_g copy
};

struct psst_network {
    int device = 0;
    int32_t n = 0, n_pn = 0, ld = 0;
    bool gabab = false;
    float area = 0.f;
    double cg = 0, ci = 0;
    std::vector<PathInfo> paths;
    int64_t grad_entries = 0;
    // device
    float *d_gt = nullptr, *d_gtb = nullptr, *d_prm = nullptr, *d_kin = nullptr;
    uint8_t *d_maskt = nullptr;     // fast/slow mask transposed like gt (1 = synapse)
    int64_t *d_paths = nullptr;     // [n_paths][6] pathway table for gradient scatter
    InstDesc desc{};
    InstDesc *d_desc = nullptr;
    int32_t *d_order = nullptr;
    int32_t *d_flag = nullptr;
    // host copies used for gradient scatter and sizing
    std::vector<float> h_kin;
    int64_t g_floats = 0;           // n * ld (+ n_ln * ld)
    int nch = 0;                    // column chunks of the synaptic sums
    // per-stage path (networks too large for one workgroup)
    StageNet *stage = nullptr;
    StageBatch *single = nullptr;   // one-trial stage batch for psst_integrate
    // method: classical RK4 unless gen (then the explicit tableau tab)
    bool gen = false;
    psst::Tab tab{};
    // sparse storage (per-instance path): ELL rows of synapses
    bool sparse = false;
    int32_t *d_spcol = nullptr;
    float *d_spval = nullptr;
    // in-place updates: each gradient-layout entry's sparse slot, and which
    // entries are synapses (NULL when every pathway is dense)
    int32_t *d_spslot = nullptr;
    uint32_t *d_gbits = nullptr;
};


struct Group {
    std::vector<int32_t> order;     // instance indices, largest first
    int32_t *d_order = nullptr;
    int max_n = 0, max_ld = 0;
    int bs = 0, npt = 0;
    int slots = 0;                  // register slots for conductance columns (0: none)
    size_t lds = 0;                 // dynamic LDS of the launch
    bool lg = false;                // lane-group kernel (every instance eligible)
};

struct psst_batch {
    std::vector<psst_network *> nets;
    int32_t n = 0;
    int64_t nt = 0;
    std::vector<int64_t> offsets;
    InstDesc *d_desc = nullptr;
    std::vector<Group> groups;
    int32_t *d_flag = nullptr;
    bool shared = false;            // every instance is the same network
    bool stage_path = false;        // large shared network: per-stage kernels
    StageBatch *stage = nullptr;
    // ragged batches with networks above the per-instance limit: each run of
    // consecutive instances of one such network is a per-stage sub-batch
    // placed in the batch's arrays; the other instances take the groups
    std::vector<StageBatch *> subs;
    std::string describe_groups;    // the launch groups' part of describe
    std::string describe;
    // graph of the persistent launches
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<hipGraphNode_t> nodes;
    std::vector<WGArgs> node_args;
    AdjWork *adj = nullptr;         // adjoint workspace, sized on first use
    // direct launches (no graph): groups after the first run on streams of
    // their own, forked from and joined to the caller's stream by events
    std::vector<hipStream_t> aux;
    std::vector<hipEvent_t> aux_done;
    hipEvent_t aux_fork = nullptr;
    Group lean;                     // every instance on a kernel without conductances
                                    // in LDS (the adjoint's recomputation beside its
                                    // reverse sweep), made on first use
    StreamBufs *strm = nullptr;     // streaming buffers, sized on first use
    bool gen = false;               // method: classical RK4 unless gen
    psst::Tab tab{};
};


// Launch a per-instance batch's kernels directly on a stream (no graph).
psst_status batch_launch_direct(psst_batch *b, float *states, const psst_stimulus *stim, float dt,
                                int64_t n_steps, int64_t step0, const psst_record *rec,
                                void *stream);

// Forward recomputation for the adjoint: n_steps steps of every instance of a
// batch from global step step0, the state read from ckpt_row (not stored
// back), each step's stage inputs and synaptic sums written to stash
// (instance b at stash + b * stash_stride, K steps per block).
typedef std::function<psst_status(const float *ckpt_row, int64_t step0, int64_t n_steps,
                                  double *stash, int64_t stash_stride, int32_t K,
                                  hipStream_t stream)>
    RecomputeFn;

// Discrete adjoint over a batch of per-instance networks (adjoint.hip).
// lean (optional): a recomputation needing at most lean_lds bytes of LDS per
// workgroup; with it, and two segments or more, a segment's recomputation
// runs beside the previous segment's reverse sweep (same results).
psst_status adjoint_run(const std::vector<psst_network *> &nets, const InstDesc *d_desc,
                        int64_t nt, AdjWork **work, const RecomputeFn &recompute,
                        const float *ckpt, int32_t K, const psst_stimulus *stim, float dt,
                        int64_t n_steps, int64_t step0, const float *dLdV, float *grad_g,
                        float *gna, float *gk, float *gl, int32_t per_instance, int32_t *flag,
                        size_t lds_max, bool gen, const psst::Tab &tab, void *stream,
                        const RecomputeFn *lean = nullptr, size_t lean_lds = 0);
void adjoint_free(AdjWork *w);
// The same with the workspace in the library's per-device scratch array
// (no allocation); sizes beyond its capacity are refused.
psst_status adjoint_run_noalloc(const std::vector<psst_network *> &nets, const InstDesc *d_desc,
                                int64_t nt, const RecomputeFn &recompute, const float *ckpt,
                                int32_t K, const psst_stimulus *stim, float dt, int64_t n_steps,
                                int64_t step0, const float *dLdV, float *grad_g, float *gna,
                                float *gk, float *gl, int32_t per_instance, int32_t *flag,
                                size_t lds_max, bool gen, const psst::Tab &tab, void *stream);
