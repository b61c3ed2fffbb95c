// kernels.h -- launch arguments shared by the host runtime and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hh_device.h"

namespace psst {

struct StimDev {
    const float *i_const;       // [n_total] nA or null
    const int32_t *pulse_ptr;   // [n_total + 1] or null
    const int64_t *on_step, *off_step;
    const float *amp;           // nA
};

struct RecDev {
    float *v_out;               // [capacity x n_total] or null
    int64_t stride, capacity;
    int32_t *spike_count;       // [n_total] or null
    float *spike_t;             // [n_total x spike_cap]
    int32_t spike_cap;
};

// Explicit Runge-Kutta tableau (stages <= 4, a strictly lower triangular)
// for the kernels' generic step; classical RK4 has kernels of its own.
struct Tab {
    int32_t s;
    double a[4][4];
    double b[4];
};

// Arguments of the persistent per-instance kernel (one workgroup integrates
// one instance for all steps of the call).
struct WGArgs {
    const InstDesc *desc;       // [n_instances]
    const int32_t *order;       // launch-local block -> instance index
    float *state;               // packed [14][n_total]
    int64_t nt;                 // n_total
    StimDev stim;
    RecDev rec;
    double dt;
    int64_t n_steps, step0;
    float *ckpt;                // [ceil(n_steps / K)][14 * n_total] or null
    int32_t K;
    int64_t lds_bytes;          // dynamic LDS of the launch; instances whose
                                // conductances fit keep them in LDS
    int32_t *flag;              // set to 1 when a state turns non-finite
    Tab tab;                    // method of the generic-step variants
    // recomputation for the adjoint: the initial state comes from state_in
    // (when not null) and is not stored back when store_state is 0; each
    // step's stage inputs and synaptic sums go to stash (when not null):
    // instance b's block at stash + b * stash_stride, laid out as the
    // adjoint's workspace (stage inputs [stash_K][4][NVAR][ld], then sums
    // [stash_K][4][3][ld], ld the instance's padded size)
    const float *state_in;
    int32_t store_state;
    double *stash;
    int64_t stash_stride;
    int32_t stash_K;
};

typedef void (*wg_kernel_t)(WGArgs);

// Kernel variant: threads per workgroup, neurons per thread, whether it
// runs the generic tableau step (else classical RK4), and whether it is the
// lane-group kernel (every instance of its launches must be eligible).
struct WGVariant {
    int bs, npt;
    bool gen;
    bool lg;
    const void *fn;
    int slots;                  // float4 register slots per thread for
                                // conductance columns (0: none)
};

// All compiled variants (terminated by fn == nullptr).
const WGVariant *wg_variants();
const void *init_kernel();

// Column chunk width of the synaptic sums (fixed summation structure).
constexpr int kChunkWidth = 64;

// Leading columns of every conductance chunk that a workgroup keeps in LDS
// for a whole launch: what its dynamic LDS (lds_bytes) leaves beside the two
// float64 activation vectors and the nch float64 partial-sum rows of ld
// entries, in whole columns of every chunk, at most the chunk width (all
// columns when the instance has no dense chunks).  The kernels' set-up and
// the host's byte accounting both use it.
__host__ __device__ inline int resident_columns(int64_t lds_bytes, int ld, int nch)
{
    const int64_t room = lds_bytes - (int64_t)sizeof(double) * (2 + nch) * ld;
    const int64_t per_col = (int64_t)sizeof(float) * nch * ld;
    const int64_t R = per_col == 0 ? kChunkWidth : (room > 0 ? room / per_col : 0);
    return (int)(R < kChunkWidth ? R : kChunkWidth);
}

// Register columns: a kernel variant with S float4 register slots per thread
// keeps, for instances that stream part of their conductances, the leading
// columns of each chunk of the thread's column group in registers -- XC
// columns (four rows each) of each of its KC chunks, XC = S / KC rounded
// down to a multiple of kRegBatch (so that no batch of kRegBatch slots spans
// two chunks), KC at most kMaxRegChunks.
constexpr int kMaxRegChunks = 8;
constexpr int kRegBatch = 4;

// On-chip columns of every conductance chunk for a workgroup of bs threads
// of a variant with `slots` register slots per thread (0: none): an instance
// that fits the LDS alone keeps every column there (*R = kChunkWidth, *XR =
// 0); otherwise, when each column group (ld / 4 threads, four rows each)
// takes KC <= kMaxRegChunks chunks, the first *XR columns of every chunk
// (slots / KC rounded down to a multiple of kRegBatch) sit in registers and
// the next *R in LDS; the rest streams every stage.  *KC = 0 when no
// register columns are used.  The kernels' set-up and the host's byte
// accounting both use it.
__host__ __device__ inline void wg_residency(int64_t lds_bytes, int ld, int nch, int bs, int slots,
                                             int *R, int *XR, int *KC)
{
    const int R0 = resident_columns(lds_bytes, ld, nch);
    *R = R0;
    *XR = 0;
    *KC = 0;
    if (R0 >= kChunkWidth || slots <= 0 || nch == 0 || ld < 4) return;
    const int ncg = bs / (ld / 4);
    if (ncg <= 0) return;
    const int kc = (nch + ncg - 1) / ncg;
    if (kc > kMaxRegChunks) return;
    int xr = slots / kc / kRegBatch * kRegBatch;
    if (xr > kChunkWidth) xr = kChunkWidth;
    if (xr <= 0) return;
    *XR = xr;
    *KC = kc;
    *R = R0 < kChunkWidth - xr ? R0 : kChunkWidth - xr;
}

// Column chunks of an instance: cholinergic, fast-GABA and slow-GABA columns.
__host__ __device__ inline int n_chunks(int n, int n_pn, bool gabab)
{
    const int na = (n_pn + kChunkWidth - 1) / kChunkWidth;
    const int ng = (n - n_pn + kChunkWidth - 1) / kChunkWidth;
    return na + ng + (gabab ? ng : 0);
}

// LDS bytes one instance needs: two float64 activation vectors and n_chunks
// float64 partial-sum rows of ld entries, plus (G in LDS) its conductance
// floats n * ld (+ n_ln * ld with slow GABA).
inline size_t wg_lds_bytes(bool glds, int ld, int n_chunks, int64_t g_floats)
{
    return sizeof(double) * (2 + (size_t)n_chunks) * (size_t)ld +
           sizeof(float) * (glds ? (size_t)g_floats : 0);
}

// Lane-group kernel (256 threads): networks of at most kLGRows neurons with
// dense storage and at most 4 column chunks keep every conductance in
// registers, two (chunk, row) pairs of 64 columns per lane (the variant's
// "neurons per thread" field holds that count); the LDS holds only the
// activations, in one slot of kLGSlot doubles per chunk (64 used; the 2 extra
// stagger the slots' LDS banks), two sets alternating by stage.
constexpr int kLGRows = 128;
constexpr int kLGPairs = 2;
constexpr int kLGSlot = 66;
constexpr int kLGThreads = 256;
constexpr int64_t kLGLdsBytes = (int64_t)sizeof(double) * 2 * 4 * kLGSlot;

// Whether an instance can take the lane-group kernel (flags as in InstDesc).
__host__ __device__ inline bool lg_eligible(int n, int n_pn, int flags)
{
    if (flags & (DESC_NOSYN | DESC_SPARSE)) return false;
    if (n > kLGRows) return false;
    return n_chunks(n, n_pn, (flags & DESC_GABAB) != 0) <= 4;
}

struct InitArgs {
    const InstDesc *desc;
    int32_t n_inst;
    const float *v0;
    float *state;
    int64_t nt;
};

}  // namespace psst
