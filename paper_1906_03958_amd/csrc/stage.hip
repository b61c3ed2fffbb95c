// stage.hip -- one launch per Runge-Kutta stage for large shared networks.
//
// Stage q of step g (paper, "Brain simulations as computational graphs": RK4;
// "Circumventing memory constraints", item 1: the synaptic update as a
// matrix multiplication):
//   A[i][b] = sum_k G[i][k] X_q[b][k]      float32 GEMM on the matrix cores,
//                                          one accumulator set per synapse class;
//                                          each 32-column float32 sum is added
//                                          to float64 totals
//   f = rhs(Y_q, cg * A, I(g))             float64, fused epilogue
//   acc += w_q f; Y_{q+1} = y + c_{q+1} dt f; X_{q+1} = x(Y_{q+1})
// and at q = 3 the combine y <- y + dt/6 acc, spikes and records.  A generic
// explicit method (template flag) takes its stage count, a and b from a
// tableau instead.
//
// GEMM tiling: a workgroup (8 wavefronts, 4 x 2, for NTILE = 64) owns 64
// postsynaptic rows x NTILE trials over the whole presynaptic axis, so each
// conductance is read from HBM once per stage.  Tiles of 128 presynaptic
// columns are staged through LDS (double-buffered) with the next tile loaded
// into registers -- 64 KiB in flight per workgroup -- while the current one
// feeds v_mfma_f32_16x16x4f32; the next tile's LDS stores follow the current
// tile's last products, so they overlap the matrix cores' work in flight,
// and one barrier per tile separates the buffers' writers and readers.  Within a 16-column group, lane l at sub-step
// s takes column 4 (l / 16) + s, so each lane reads its four A and four B
// values with one 16-byte LDS load; the column order of the sum is fixed, so
// results are deterministic.  A float32 running sum over all K columns would
// carry a rounding error growing with K (16384 here); each sum of two
// 16-column groups therefore starts from zero on the matrix cores (eight
// chained products of four columns) and is added in float64, so float32
// rounding acts on 32-term sums of non-negative products only.
//
// Between launches the per-(neuron, trial) stage input Y and accumulator acc
// live in a float64 workspace; activations X are double-buffered float32.
#include <algorithm>
#include <cstdio>
#include <cstring>

#include "stage.h"

using namespace psst;

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int KT = 128;       // presynaptic columns per LDS tile
constexpr int MT = 64;        // postsynaptic rows per workgroup
constexpr int LDK = KT + 4;   // LDS row stride in floats
// 16-column groups per float32 matrix-core sum: each sum of 32 columns starts
// from zero and is added to the float64 totals
constexpr int kFoldGroups = 2;
static_assert((KT / 16) % kFoldGroups == 0, "a fold never spans two tiles");

// Dynamic LDS of a stage launch with NTILE trials per workgroup, in floats:
// the double-buffered G and X tiles during the products, then the float64
// totals of the three synapse classes for the epilogue (same memory).
constexpr size_t tile_floats(int ntile) { return 2 * (size_t)(MT + ntile) * LDK; }
constexpr size_t acc_floats(int ntile) { return 2 * 3 * (size_t)MT * (ntile + 1); }
constexpr size_t stage_lds_floats(int ntile)
{
    return tile_floats(ntile) > acc_floats(ntile) ? tile_floats(ntile) : acc_floats(ntile);
}
constexpr int NVS = NVAR;

struct StageFixed {
    const float *G;
    const int32_t *sp_off;    // sparse storage: synapse buckets (stage.h)
    const uint8_t *sp_col;
    const float *sp_val;
    const uint32_t *sp_mask;
    int Kp, ka, kg;           // K blocks [0,ka) ACh, [ka,ka+kg) fast GABA, [ka+kg,Kp) slow GABA
    float *X0, *X1;           // [Bp][Kp] activations (double-buffered by stage launch)
    double *Yw, *accw;        // [NVAR][nt] stage input and RK4 accumulator
    double *P2, *P3;          // generic method: partial inputs of stages 2, 3
    Tab tab;                  // generic method (stages, a, b)
    const float *prm;         // [NPRM][ld]
    const float *kin;
    int ld, n, n_pn, B, Bp;
    int64_t nt;               // B * n (workspace planes)
    // the caller's state, stimulus and record arrays: plane stride and the
    // first trial's offset (B * n and 0, unless the trials are one run of
    // instances inside a larger batch)
    int64_t st_stride, st_off;
    int gabab;
    double cg, ci;
};

struct StageCtl {
    float *state;
    StimDev stim;
    RecDev rec;
    double dt;
    int64_t step0, g;
    int32_t *flag;
};

__device__ __forceinline__ int k_fast(const StageFixed &fx, int i)
{
    return i < fx.n_pn ? i : fx.ka + (i - fx.n_pn);
}

__device__ __forceinline__ void write_x(const StageFixed &fx, float *X, int b, int i,
                                        const double *Y, const Kin &K)
{
    float *xr = X + (int64_t)b * fx.Kp;
    xr[k_fast(fx, i)] = (float)Y[YS];
    if (fx.gabab && i >= fx.n_pn) xr[fx.ka + fx.kg + (i - fx.n_pn)] = (float)gabab_act(Y[YG], K);
}

// Per call: publish the call's control block, then the stage-0 activations
// from the carried state (stage 0 reads its input from the state itself).
__global__ __launch_bounds__(256) void stage_prologue(StageFixed fx, StageCtl c, StageCtl *dctl)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) *dctl = c;
    const Kin K = load_kin(fx.kin);
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < fx.nt;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int b = (int)(p / fx.n), i = (int)(p % fx.n);
        const int64_t so = fx.st_off + p;
        double y[NVS];
#pragma unroll
        for (int v = 0; v < NVS; ++v)
            y[v] = (double)c.state[(2 * v) * fx.st_stride + so] +
                   (double)c.state[(2 * v + 1) * fx.st_stride + so];
        write_x(fx, fx.X0, b, i, y, K);
    }
}

__global__ void stage_advance(StageCtl *dctl) { dctl->g += 1; }

// Global -> register part of the tile pipeline.  The conductances are read
// once per stage and exceed the caches, so they are loaded non-temporally and
// leave L2 and the infinity cache to the activations and the workspace.
template <int GV, int XVT, int RPP>
__device__ __forceinline__ void tile_load(floatx4 (&rg)[GV], floatx4 (&rx)[XVT], const float *G,
                                          const float *X, int Kp, int m0, int n0, int lr, int lk,
                                          int k0)
{
#pragma unroll
    for (int u = 0; u < GV; ++u)
        rg[u] = __builtin_nontemporal_load(
            reinterpret_cast<const floatx4 *>(G + (int64_t)(m0 + lr + RPP * u) * Kp + k0 + lk));
#pragma unroll
    for (int u = 0; u < XVT; ++u)
        rx[u] = *reinterpret_cast<const floatx4 *>(X + (int64_t)(n0 + lr + RPP * u) * Kp + k0 + lk);
}

// The fused epilogue of a stage launch: right-hand side and Runge-Kutta
// bookkeeping per (neuron, trial) of the workgroup's MT x NTILE block, from
// the synaptic sums of the three classes in sA [3][MT][NTILE + 1] (LDS).
template <int NTILE, int NTH, bool GEN>
__device__ __forceinline__ void stage_epilogue(const StageFixed &fx,
                                               const StageCtl *__restrict__ dctl, int q,
                                               const double *sA, float *Xn, int m0, int n0,
                                               int tid)
{
    const Kin K = load_kin(fx.kin);
    const StageCtl c = *dctl;
    const double dt = c.dt;
    const int64_t g = c.g;
    const int64_t nt = fx.nt, ST = fx.st_stride;
    bool bad = false;
    // without slow GABA the r, G planes have zero derivative: they are neither
    // read nor written (the state keeps them as they are)
    const int nv = fx.gabab ? NVS : YR;
    for (int p = tid; p < MT * NTILE; p += NTH) {
        const int il = p % MT, bl = p / MT;
        const int i = m0 + il, b = n0 + bl;
        if (i >= fx.n || b >= fx.B) continue;
        const int64_t gi = (int64_t)b * fx.n + i;   // workspace index
        const int64_t so = fx.st_off + gi;           // state, stimulus, records
        // y: the step's start state; Y: this stage's input (y itself at stage
        // 0); a: the weighted sum of the earlier stages' derivatives.  The
        // generic method keeps, per variable, B = sum_r b_r k_r in accw and
        // in the slot of each later stage m the partial input
        // sum_r a_mr k_r, replaced by the input y + dt * sum itself once
        // stage m - 1 has added the last term.
        auto slot = [&](int m) { return m == 1 ? fx.Yw : (m == 2 ? fx.P2 : fx.P3); };
        const int last = GEN ? fx.tab.s - 1 : 3;
        double Y[NVS], a[NVS], y[NVS];
#pragma unroll
        for (int v = 0; v < NVS; ++v) {
            y[v] = v < nv ? (double)c.state[(2 * v) * ST + so] + (double)c.state[(2 * v + 1) * ST + so]
                          : 0.0;
            Y[v] = (q == 0 || v >= nv) ? y[v] : slot(GEN ? q : 1)[v * nt + gi];
            a[v] = (q == 0 || v >= nv) ? 0.0 : fx.accw[v * nt + gi];
        }
        Prm P = load_prm(fx.prm, fx.ld, i);
        double I = c.stim.i_const ? (double)c.stim.i_const[so] : 0.0;
        if (c.stim.pulse_ptr)
            for (int k = c.stim.pulse_ptr[so]; k < c.stim.pulse_ptr[so + 1]; ++k)
                if (c.stim.on_step[k] <= g && g < c.stim.off_step[k]) I += (double)c.stim.amp[k];
        const double sa = sA[(0 * MT + il) * (NTILE + 1) + bl];
        const double sg = sA[(1 * MT + il) * (NTILE + 1) + bl];
        const double sb = sA[(2 * MT + il) * (NTILE + 1) + bl];
        double f[NVS];
        hh_rhs(Y, P, K, fx.cg * sa, fx.cg * sg, fx.cg * sb, fx.ci * I, i >= fx.n_pn,
               fx.gabab != 0, f);
        double yn[NVS];                       // the step's result (last stage)
        if constexpr (GEN) {
#pragma unroll
            for (int v = 0; v < NVS; ++v) a[v] += fx.tab.b[q] * f[v];
            if (q < last) {
#pragma unroll
                for (int v = 0; v < NVS; ++v) {
                    for (int m = q + 1; m <= last; ++m) {
                        const double pm = (q == 0 || v >= nv ? 0.0 : slot(m)[v * nt + gi]) +
                                          fx.tab.a[m][q] * f[v];
                        const double val = m == q + 1 ? y[v] + dt * pm : pm;
                        if (m == q + 1) Y[v] = val;
                        if (v < nv) slot(m)[v * nt + gi] = val;
                    }
                    if (v < nv) fx.accw[v * nt + gi] = a[v];
                }
                write_x(fx, Xn, b, i, Y, K);
            } else {
#pragma unroll
                for (int v = 0; v < NVS; ++v) yn[v] = y[v] + dt * a[v];
            }
        } else {
            const double w = (q == 0 || q == 3) ? 1.0 : 2.0;
#pragma unroll
            for (int v = 0; v < NVS; ++v) a[v] += w * f[v];
            if (q < 3) {
                const double cq = (q == 2) ? dt : 0.5 * dt;
#pragma unroll
                for (int v = 0; v < NVS; ++v) {
                    Y[v] = y[v] + cq * f[v];
                    if (v < nv) {
                        fx.Yw[v * nt + gi] = Y[v];
                        fx.accw[v * nt + gi] = a[v];
                    }
                }
                write_x(fx, Xn, b, i, Y, K);
            } else {
#pragma unroll
                for (int v = 0; v < NVS; ++v) yn[v] = y[v] + (dt / 6.0) * a[v];
            }
        }
        if (q == last) {
            const double vold = y[YV];
            double chk = 0.0;
#pragma unroll
            for (int v = 0; v < NVS; ++v) {
                if (v >= nv) continue;
                float hi, lo;
                y[v] = split_store(yn[v], hi, lo);
                c.state[(2 * v) * ST + so] = hi;
                c.state[(2 * v + 1) * ST + so] = lo;
                chk += y[v];
            }
            bad |= !finite_d(chk);
            write_x(fx, Xn, b, i, y, K);
            const double vnew = y[YV];
            if (c.rec.spike_count && vold < 0.0 && vnew >= 0.0) {
                const int32_t cnt = c.rec.spike_count[so];
                if (cnt < c.rec.spike_cap)
                    c.rec.spike_t[so * c.rec.spike_cap + cnt] =
                        (float)(((double)g + (0.0 - vold) / (vnew - vold)) * dt);
                c.rec.spike_count[so] = cnt + 1;
            }
            if (c.rec.v_out && c.rec.stride > 0 && (g + 1) % c.rec.stride == 0) {
                const int64_t row = (g + 1) / c.rec.stride - c.step0 / c.rec.stride - 1;
                if (row < c.rec.capacity) c.rec.v_out[row * ST + so] = (float)vnew;
            }
        }
    }
    if (bad) atomicOr(c.flag, 1);
}

// One workgroup per CU (its LDS tiles take most of the CU's LDS); WR x WC
// wavefronts, each owning BR x BC blocks of 16 x 16 outputs.
// SP: sparse storage -- each conductance tile is built in LDS from the row
// block's synapse buckets (zeros elsewhere) instead of being loaded dense, so
// the products, and the results, are those of dense storage bit for bit
// while HBM carries only the synapses.
template <int WR, int WC, int BR, int BC, bool GEN, bool SP = false>
__global__ __launch_bounds__(64 * WR * WC) __attribute__((amdgpu_waves_per_eu(WR * WC / 4, WR * WC / 4))) void stage_kernel(StageFixed fx, const StageCtl *__restrict__ dctl,
                                                    int q)
{
    constexpr int NTILE = WC * BC * 16;
    constexpr int NTH = 64 * WR * WC;           // threads per workgroup
    static_assert(WR * BR * 16 == MT, "tile rows");
    extern __shared__ float smem[];                 // stage_lds_floats(NTILE) floats
    float *sG = smem;                       // [2][MT * LDK]
    float *sX = smem + 2 * MT * LDK;        // [2][NTILE * LDK]

    const int m0 = blockIdx.x * MT, n0 = blockIdx.y * NTILE;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave / WC, wc = wave % WC;
    // activations alternate between the two buffers at every stage launch of
    // the call (the prologue fills X0 for the first): the launch's position
    // is (step - first step) * stages + q, whatever the method's stage count
    const int64_t k_launch = (dctl->g - dctl->step0) * (GEN ? fx.tab.s : 4) + q;
    const float *X = (k_launch & 1) ? fx.X1 : fx.X0;
    float *Xn = (k_launch & 1) ? fx.X0 : fx.X1;

    double acc[3][BR][BC][4];
#pragma unroll
    for (int t = 0; t < 3; ++t)
#pragma unroll
        for (int br = 0; br < BR; ++br)
#pragma unroll
            for (int bc = 0; bc < BC; ++bc)
#pragma unroll
                for (int r = 0; r < 4; ++r) acc[t][br][bc][r] = 0.0;

    // tile loaders: a G tile is MT x KT floats = 8 float4 per thread, an X
    // tile NTILE x KT floats = NTILE / 8 float4 per thread; the next tile is
    // loaded into registers while the current one feeds the matrix cores
    constexpr int K4 = KT / 4;                 // float4 per tile row
    constexpr int RPP = NTH / K4;              // rows per pass of the workgroup
    constexpr int GV = MT / RPP;               // G float4 per thread
    constexpr int XVT = NTILE / RPP;           // X float4 per thread
    const int lr = tid / K4, lk = (tid % K4) * 4;
#pragma unroll
    for (int blk = 0; blk < 3; ++blk) {
        const int kbeg = blk == 0 ? 0 : (blk == 1 ? fx.ka : fx.ka + fx.kg);
        const int kend = blk == 0 ? fx.ka : (blk == 1 ? fx.ka + fx.kg : fx.Kp);
        const int ntile = (kend - kbeg) / KT;
        if (ntile == 0) continue;
        floatx4 rg[SP ? 1 : GV], rx[XVT];
        // sparse source: thread tid builds row sr of the tile, columns
        // [sk SW, (sk + 1) SW) -- zeros, then its synapses there.  The row's
        // bucket mask and start (loaded a tile ahead) give the segment's
        // synapses: they follow the bucket's start by the number of set bits
        // below the segment, in column order; the first SPV of them are
        // loaded a tile ahead like the dense rows (at p = 0.1 a 16-column
        // segment holds more about once in 2,000), the rest when the tile is
        // built
        constexpr int SEG = NTH / MT, SW = KT / SEG, SPV = SW == 32 ? 8 : 6;
        static_assert(SW == 16 || SW == 32, "segment of a mask word or half a word");
        const int sr = tid / SEG, sk = tid % SEG;
        uint32_t nmask[4] = {0u, 0u, 0u, 0u};
        int nb0 = 0;                        // the next tile's bucket
        uint32_t seg = 0;                   // the loaded tile's segment bits
        int sbase = 0;                      // its first synapse
        float spv[SP ? SPV : 1];
        auto sp_bucket = [&](int kt) {      // kt: tile on the whole K axis
            const int64_t bk = ((int64_t)blockIdx.x * (fx.Kp / KT) + kt) * MT + sr;
            const uint4 m = *reinterpret_cast<const uint4 *>(fx.sp_mask + 4 * bk);
            nmask[0] = m.x, nmask[1] = m.y, nmask[2] = m.z, nmask[3] = m.w;
            nb0 = fx.sp_off[bk];
        };
        auto sp_load = [&](int kt_next) {
            const int w = (sk * SW) / 32, sh = (sk * SW) % 32;
            int below = 0;
#pragma unroll
            for (int i = 0; i < 4; ++i) below += i < w ? __builtin_popcount(nmask[i]) : 0;
            uint32_t mw = nmask[0];
#pragma unroll
            for (int i = 1; i < 4; ++i) mw = i == w ? nmask[i] : mw;
            below += __builtin_popcount(sh ? mw & ((1u << sh) - 1u) : 0u);
            seg = SW == 32 ? mw : (mw >> sh) & 0xFFFFu;
            sbase = nb0 + below;
            const int cnt = __builtin_popcount(seg);
#pragma unroll
            for (int u = 0; u < SPV; ++u) spv[u] = fx.sp_val[u < cnt ? sbase + u : nb0];
            sp_bucket(kt_next);
        };
        auto tile_store = [&](int t) {
            float *g = sG + (t & 1) * MT * LDK;
            float *x = sX + (t & 1) * NTILE * LDK;
            if constexpr (SP) {
                float *row = g + sr * LDK + sk * SW;
                // zeros, 16 bytes at a time; the start is rotated by the
                // segment's place so the segments of a row begin in
                // different banks
#pragma unroll
                for (int j = 0; j < SW / 4; ++j) {
                    const int c = ((j + sk * SW / 64) % (SW / 4)) * 4;
                    *reinterpret_cast<floatx4 *>(row + c) = floatx4{0.f, 0.f, 0.f, 0.f};
                }
                uint32_t m = seg;
#pragma unroll
                for (int k = 0; k < SPV; ++k)
                    if (m) {
                        row[__builtin_ctz(m)] = spv[k];
                        m &= m - 1u;
                    }
                for (int u = SPV; m; ++u, m &= m - 1u)      // the rare long segments
                    row[__builtin_ctz(m)] = fx.sp_val[sbase + u];
            } else {
#pragma unroll
                for (int u = 0; u < GV; ++u)
                    *reinterpret_cast<floatx4 *>(g + (lr + RPP * u) * LDK + lk) = rg[u];
            }
#pragma unroll
            for (int u = 0; u < XVT; ++u)
                *reinterpret_cast<floatx4 *>(x + (lr + RPP * u) * LDK + lk) = rx[u];
        };
        // load tile t of this block (at column kbeg + t KT) into registers
        auto load_tile = [&](int t) {
            if constexpr (SP) {
                sp_load(kbeg / KT + min(t + 1, ntile - 1));
#pragma unroll
                for (int u = 0; u < XVT; ++u)
                    rx[u] = *reinterpret_cast<const floatx4 *>(
                        X + (int64_t)(n0 + lr + RPP * u) * fx.Kp + kbeg + t * KT + lk);
            } else {
                tile_load<GV, XVT, RPP>(rg, rx, fx.G, X, fx.Kp, m0, n0, lr, lk, kbeg + t * KT);
            }
        };
        // tile t + 1 is loaded into registers while tile t feeds the matrix
        // cores, and stored to the other LDS buffer right after tile t's last
        // products are issued (its stores overlap them) and before the one
        // barrier per tile; the last tile is loaded and stored once more past
        // the end (in bounds, never read), so every iteration is the same
        const auto last = [&](int t) { return min(t, ntile - 1); };
        if constexpr (SP) sp_bucket(kbeg / KT);
        load_tile(0);
        __syncthreads();     // previous users of the tile buffers are done
        tile_store(0);
        load_tile(last(1));
        __syncthreads();
        for (int t = 0; t < ntile; ++t) {
            const float *g = sG + (t & 1) * MT * LDK;
            const float *x = sX + (t & 1) * NTILE * LDK;
            // ask the scheduler to interleave the LDS operand reads of the next
            // sub-step with the matrix-core instructions of the current one
            // instead of grouping every read ahead of its products
            // (single-wave small-GEMM strategy)
            __builtin_amdgcn_iglp_opt(1);
            floatx4 tacc[BR][BC];
#pragma unroll
            for (int kk = 0; kk < KT / 16; ++kk) {
                if (kk % kFoldGroups == 0) {
#pragma unroll
                    for (int br = 0; br < BR; ++br)
#pragma unroll
                        for (int bc = 0; bc < BC; ++bc) tacc[br][bc] = floatx4{0.f, 0.f, 0.f, 0.f};
                }
                floatx4 a[BR], bv[BC];
                const int kq = kk * 16 + 4 * (lane >> 4);
#pragma unroll
                for (int br = 0; br < BR; ++br) {
                    const int row = (wr * BR + br) * 16 + (lane & 15);
                    a[br] = *reinterpret_cast<const floatx4 *>(g + row * LDK + kq);
                }
#pragma unroll
                for (int bc = 0; bc < BC; ++bc) {
                    const int col = (wc * BC + bc) * 16 + (lane & 15);
                    bv[bc] = *reinterpret_cast<const floatx4 *>(x + col * LDK + kq);
                }
#pragma unroll
                for (int s = 0; s < 4; ++s)
#pragma unroll
                    for (int br = 0; br < BR; ++br)
#pragma unroll
                        for (int bc = 0; bc < BC; ++bc)
                            tacc[br][bc] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                                a[br][s], bv[bc][s], tacc[br][bc], 0, 0, 0);
                if (kk % kFoldGroups == kFoldGroups - 1) {
#pragma unroll
                    for (int br = 0; br < BR; ++br)
#pragma unroll
                        for (int bc = 0; bc < BC; ++bc)
#pragma unroll
                            for (int r = 0; r < 4; ++r)
                                acc[blk][br][bc][r] += (double)tacc[br][bc][r];
                }
            }
            // the other buffer was last read before the previous barrier
            tile_store(t + 1);
            load_tile(last(t + 2));
            __syncthreads();
        }
    }
    __syncthreads();
    // accumulators to LDS: lane holds rows 4 (lane / 16) + r, column lane % 16
    double *sA = reinterpret_cast<double *>(smem);   // [3][MT][NTILE + 1]
#pragma unroll
    for (int t = 0; t < 3; ++t)
#pragma unroll
        for (int br = 0; br < BR; ++br)
#pragma unroll
            for (int bc = 0; bc < BC; ++bc)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int m = (wr * BR + br) * 16 + 4 * (lane >> 4) + r;
                    const int nn = (wc * BC + bc) * 16 + (lane & 15);
                    sA[(t * MT + m) * (NTILE + 1) + nn] = acc[t][br][bc][r];
                }
    __syncthreads();

    stage_epilogue<NTILE, NTH, GEN>(fx, dctl, q, sA, Xn, m0, n0, tid);
}

}  // namespace

struct StageBatch {
    psst_network *net = nullptr;
    int B = 0, Bp = 0, ntile = 0;
    StageFixed fx{};
    StageCtl *d_ctl = nullptr;
    int32_t *d_flag = nullptr;
    bool own_flag = true;             // d_flag allocated by the batch
    float *X = nullptr;
    double *work = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int q_arg[4] = {0, 1, 2, 3};
    bool gen = false;                 // generic explicit method (fx.tab)
    std::string desc;
};

static int round_up(int x, int m) { return (x + m - 1) / m * m; }

// The synapse buckets of a sparse large network (layout in stage.h).
static psst_status stage_net_sparse(StageNet *sn, const psst_network *net,
                                    const psst_pathway *paths, int32_t np)
{
    const int ntl = sn->Kp / KT, nrb = sn->Mp / MT;
    const int64_t nb = (int64_t)nrb * ntl * 64;
    auto column = [&](const psst_pathway &w, int j) {
        return w.type == PSST_SYN_ACH ? j
                                      : (w.type == PSST_SYN_GABA_A ? sn->ka + (j - net->n_pn)
                                                                   : sn->ka + sn->kg + (j - net->n_pn));
    };
    auto bucket = [&](int i, int k) { return ((int64_t)(i / MT) * ntl + k / KT) * MT + i % MT; };
    std::vector<int64_t> off(nb + 1, 0);
    for (int q = 0; q < np; ++q) {
        const psst_pathway &w = paths[q];
        const int npre = w.pre_end - w.pre_begin;
        for (int i = w.post_begin; i < w.post_end; ++i)
            for (int j = w.pre_begin; j < w.pre_end; ++j) {
                const int64_t e = (int64_t)(i - w.post_begin) * npre + (j - w.pre_begin);
                if (!w.mask || w.mask[e]) ++off[bucket(i, column(w, j)) + 1];
            }
    }
    for (int64_t b = 0; b < nb; ++b) off[b + 1] += off[b];
    const int64_t nnz = off[nb];
    if (nnz >= ((int64_t)1 << 31))
        return fail(PSST_ERR_UNSUPPORTED, "%lld synapses exceed the sparse layout's 2^31",
                    (long long)nnz);
    // one entry more than the synapses: a kernel's read at the start of an
    // empty last bucket stays in bounds (its value is never used)
    std::vector<uint8_t> col((size_t)nnz + 1, 0);
    std::vector<float> val((size_t)nnz + 1, 0.f);
    std::vector<int64_t> pos(off.begin(), off.end() - 1);
    for (int q = 0; q < np; ++q) {
        const psst_pathway &w = paths[q];
        const int npre = w.pre_end - w.pre_begin;
        for (int i = w.post_begin; i < w.post_end; ++i)
            for (int j = w.pre_begin; j < w.pre_end; ++j) {
                const int64_t e = (int64_t)(i - w.post_begin) * npre + (j - w.pre_begin);
                if (w.mask && !w.mask[e]) continue;
                const int k = column(w, j);
                const int64_t p = pos[bucket(i, k)]++;
                col[p] = (uint8_t)(k % KT);
                val[p] = w.g_nS[e];
            }
    }
    // ascending columns within each bucket (pathways of one class may come
    // in any order; no column repeats, pathways of a type do not overlap)
    std::vector<std::pair<uint8_t, float>> tmp;
    for (int64_t b = 0; b < nb; ++b) {
        const int64_t b0 = off[b], b1 = off[b + 1];
        tmp.clear();
        for (int64_t p = b0; p < b1; ++p) tmp.push_back({col[p], val[p]});
        std::sort(tmp.begin(), tmp.end(),
                  [](const std::pair<uint8_t, float> &x, const std::pair<uint8_t, float> &y) {
                      return x.first < y.first;
                  });
        for (int64_t p = b0; p < b1; ++p) {
            col[p] = tmp[p - b0].first;
            val[p] = tmp[p - b0].second;
        }
    }
    std::vector<uint32_t> mask((size_t)nb * 4, 0u);
    for (int64_t b = 0; b < nb; ++b)
        for (int64_t p = off[b]; p < off[b + 1]; ++p) mask[4 * b + col[p] / 32] |= 1u << (col[p] % 32);
    std::vector<int32_t> off32(off.begin(), off.end());
    hipError_t e = hipMalloc(&sn->sp_off, sizeof(int32_t) * off32.size());
    if (e == hipSuccess)
        e = hipMemcpy(sn->sp_off, off32.data(), sizeof(int32_t) * off32.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc(&sn->sp_col, col.size());
    if (e == hipSuccess) e = hipMemcpy(sn->sp_col, col.data(), col.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc(&sn->sp_val, sizeof(float) * val.size());
    if (e == hipSuccess)
        e = hipMemcpy(sn->sp_val, val.data(), sizeof(float) * val.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc(&sn->sp_mask, sizeof(uint32_t) * mask.size());
    if (e == hipSuccess)
        e = hipMemcpy(sn->sp_mask, mask.data(), sizeof(uint32_t) * mask.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess)
        return fail(e == hipErrorOutOfMemory ? PSST_ERR_OUT_OF_MEMORY : PSST_ERR_DEVICE,
                    "sparse stage layout upload failed: %s", hipGetErrorString(e));
    sn->sparse = true;
    sn->nnz = nnz;
    return PSST_OK;
}

psst_status stage_net_create(psst_network *net, const psst_pathway *paths, int32_t np,
                             bool sparse)
{
    StageNet *sn = new StageNet();
    sn->n = net->n;
    sn->n_pn = net->n_pn;
    sn->gabab = net->gabab;
    const int n_ln = net->n - net->n_pn;
    sn->Mp = round_up(net->n, MT);
    sn->ka = round_up(net->n_pn, KT);
    sn->kg = round_up(n_ln, KT);
    sn->kb = net->gabab ? round_up(n_ln, KT) : 0;
    sn->Kp = sn->ka + sn->kg + sn->kb;
    if (sparse) {
        psst_status st = stage_net_sparse(sn, net, paths, np);
        if (st != PSST_OK) {
            stage_net_free(sn);
            return st;
        }
        net->stage = sn;
        return PSST_OK;
    }
    std::vector<float> G((size_t)sn->Mp * sn->Kp, 0.f);
    for (int q = 0; q < np; ++q) {
        const psst_pathway &w = paths[q];
        const int npre = w.pre_end - w.pre_begin;
        for (int i = w.post_begin; i < w.post_end; ++i) {
            float *row = G.data() + (size_t)i * sn->Kp;
            const float *src = w.g_nS + (size_t)(i - w.post_begin) * npre;
            const uint8_t *msk = w.mask ? w.mask + (size_t)(i - w.post_begin) * npre : nullptr;
            for (int j = w.pre_begin; j < w.pre_end; ++j) {
                int k;
                if (w.type == PSST_SYN_ACH) k = j;
                else if (w.type == PSST_SYN_GABA_A) k = sn->ka + (j - net->n_pn);
                else k = sn->ka + sn->kg + (j - net->n_pn);
                const int e = j - w.pre_begin;
                row[k] = (!msk || msk[e]) ? src[e] : 0.f;
            }
        }
    }
    hipError_t e = hipMalloc(&sn->G, sizeof(float) * G.size());
    if (e == hipSuccess)
        e = hipMemcpy(sn->G, G.data(), sizeof(float) * G.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        stage_net_free(sn);
        return fail(e == hipErrorOutOfMemory ? PSST_ERR_OUT_OF_MEMORY : PSST_ERR_DEVICE,
                    "stage layout upload failed: %s", hipGetErrorString(e));
    }
    net->stage = sn;
    return PSST_OK;
}

void stage_net_free(StageNet *sn)
{
    if (!sn) return;
    (void)hipFree(sn->G);
    (void)hipFree(sn->sp_off);
    (void)hipFree(sn->sp_col);
    (void)hipFree(sn->sp_val);
    (void)hipFree(sn->sp_mask);
    delete sn;
}

psst_status stage_batch_create(psst_network *net, int32_t n_trials, StageBatch **out,
                               int64_t st_stride, int64_t st_off)
{
    *out = nullptr;
    if (!net->stage) return fail(PSST_ERR_UNSUPPORTED, "network has no per-stage layout");
    StageNet *sn = net->stage;
    StageBatch *sb = new StageBatch();
    sb->net = net;
    sb->B = n_trials;
    sb->ntile = n_trials <= 16 ? 16 : 64;
    sb->Bp = round_up(n_trials, sb->ntile);
    const int64_t nt = (int64_t)n_trials * net->n;
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t x) { if (e == hipSuccess) e = x; };
    chk(hipMalloc(&sb->X, sizeof(float) * 2 * (size_t)sb->Bp * sn->Kp));
    chk(hipMemset(sb->X, 0, sizeof(float) * 2 * (size_t)sb->Bp * sn->Kp));
    // four float64 planes per (variable, neuron, trial): classical RK4 uses
    // the first two (stage input, accumulator), a generic method all four
    chk(hipMalloc(&sb->work, sizeof(double) * 4 * NVAR * (size_t)nt));
    chk(hipMalloc(&sb->d_ctl, sizeof(StageCtl)));
    chk(hipMalloc(&sb->d_flag, sizeof(int32_t)));
    chk(hipMemset(sb->d_flag, 0, sizeof(int32_t)));
    if (e != hipSuccess) {
        stage_batch_free(sb);
        return fail(e == hipErrorOutOfMemory ? PSST_ERR_OUT_OF_MEMORY : PSST_ERR_DEVICE,
                    "stage batch allocation failed: %s", hipGetErrorString(e));
    }
    StageFixed &fx = sb->fx;
    fx.G = sn->G;
    fx.sp_off = sn->sp_off;
    fx.sp_col = sn->sp_col;
    fx.sp_val = sn->sp_val;
    fx.sp_mask = sn->sp_mask;
    fx.Kp = sn->Kp;
    fx.ka = sn->ka;
    fx.kg = sn->kg;
    fx.X0 = sb->X;
    fx.X1 = sb->X + (size_t)sb->Bp * sn->Kp;
    fx.Yw = sb->work;
    fx.accw = sb->work + (size_t)NVAR * nt;
    fx.P2 = sb->work + 2 * (size_t)NVAR * nt;
    fx.P3 = sb->work + 3 * (size_t)NVAR * nt;
    fx.prm = net->d_prm;
    fx.kin = net->d_kin;
    fx.ld = net->ld;
    fx.n = net->n;
    fx.n_pn = net->n_pn;
    fx.B = n_trials;
    fx.Bp = sb->Bp;
    fx.nt = nt;
    fx.st_stride = st_stride > 0 ? st_stride : nt;
    fx.st_off = st_off;
    fx.gabab = net->gabab ? 1 : 0;
    fx.cg = net->cg;
    fx.ci = net->ci;
    stage_batch_set_method(sb, net->gen, net->tab);
    *out = sb;
    return PSST_OK;
}

void stage_batch_set_method(StageBatch *sb, bool gen, const Tab &tab)
{
    if (sb->exec) {
        // the graph's kernel and stage count change: build it on the next call
        (void)hipGraphExecDestroy(sb->exec);
        (void)hipGraphDestroy(sb->graph);
        sb->exec = nullptr;
        sb->graph = nullptr;
    }
    sb->gen = gen;
    sb->fx.tab = gen ? tab : Tab{};
    const StageNet *sn = sb->net->stage;
    char buf[256];
    if (sn->sparse)
        snprintf(buf, sizeof buf,
                 "[per-stage sparse: fp32 MFMA GEMM on tiles built from %lld synapses, %d rows x "
                 "%d trials (tile 64 x %d), K %d, %d launches per step]",
                 (long long)sn->nnz, sn->Mp, sb->Bp, sb->ntile, sn->Kp, gen ? tab.s : 4);
    else
        snprintf(buf, sizeof buf,
                 "[per-stage fp32 MFMA GEMM: %d rows x %d trials (tile 64 x %d), K %d, %d launches "
                 "per step]",
                 sn->Mp, sb->Bp, sb->ntile, sn->Kp, gen ? tab.s : 4);
    sb->desc = buf;
}

void stage_batch_free(StageBatch *sb)
{
    if (!sb) return;
    if (sb->exec) (void)hipGraphExecDestroy(sb->exec);
    if (sb->graph) (void)hipGraphDestroy(sb->graph);
    (void)hipFree(sb->X);
    (void)hipFree(sb->work);
    (void)hipFree(sb->d_ctl);
    if (sb->own_flag) (void)hipFree(sb->d_flag);
    delete sb;
}

const char *stage_batch_describe(const StageBatch *sb) { return sb ? sb->desc.c_str() : ""; }

void stage_batch_use_flag(StageBatch *sb, int32_t *flag)
{
    if (sb->own_flag) (void)hipFree(sb->d_flag);
    sb->d_flag = flag;
    sb->own_flag = false;
}

// Each workgroup column (one tile of trials) reads the whole padded matrix
// once per stage launch; sparse storage: every synapse's value and every
// bucket's start and column mask.
int64_t stage_batch_matrix_bytes(const StageBatch *sb)
{
    const StageNet *sn = sb->net->stage;
    if (sn->sparse)
        return ((int64_t)sizeof(float) * sn->nnz +
                (int64_t)(sizeof(int32_t) + 4 * sizeof(uint32_t)) * sn->Mp / MT * (sn->Kp / KT) *
                    MT) *
               (sb->Bp / sb->ntile);
    return (int64_t)sizeof(float) * sn->Mp * sn->Kp * (sb->Bp / sb->ntile);
}

static const void *stage_fn(int ntile, bool gen, bool sparse)
{
    if (sparse) {
        if (gen)
            return ntile == 16 ? (const void *)stage_kernel<4, 1, 1, 1, true, true>
                               : (const void *)stage_kernel<4, 2, 1, 2, true, true>;
        return ntile == 16 ? (const void *)stage_kernel<4, 1, 1, 1, false, true>
                           : (const void *)stage_kernel<4, 2, 1, 2, false, true>;
    }
    if (gen)
        return ntile == 16 ? (const void *)stage_kernel<4, 1, 1, 1, true>
                           : (const void *)stage_kernel<4, 2, 1, 2, true>;
    return ntile == 16 ? (const void *)stage_kernel<4, 1, 1, 1, false>
                       : (const void *)stage_kernel<4, 2, 1, 2, false>;
}

static int stage_threads(int ntile) { return ntile == 16 ? 256 : 512; }

static size_t stage_lds_bytes(int ntile) { return sizeof(float) * stage_lds_floats(ntile); }

// One step as a graph: its stages (4 for RK4) then the step-counter advance.
static psst_status build_graph(StageBatch *sb)
{
    const size_t lds = stage_lds_bytes(sb->ntile);
    const void *fn = stage_fn(sb->ntile, sb->gen, sb->net->stage->sparse);
    HIPCHK(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    HIPCHK(hipGraphCreate(&sb->graph, 0));
    hipGraphNode_t prev = nullptr;
    const dim3 grid(sb->net->stage->Mp / MT, sb->Bp / sb->ntile);
    const int stages = sb->gen ? sb->fx.tab.s : 4;
    for (int q = 0; q < stages; ++q) {
        void *kp[] = {&sb->fx, &sb->d_ctl, &sb->q_arg[q]};
        hipKernelNodeParams p{};
        p.func = const_cast<void *>(fn);
        p.gridDim = grid;
        p.blockDim = dim3(stage_threads(sb->ntile));
        p.sharedMemBytes = (unsigned)lds;
        p.kernelParams = kp;
        p.extra = nullptr;
        hipGraphNode_t node;
        HIPCHK(hipGraphAddKernelNode(&node, sb->graph, prev ? &prev : nullptr, prev ? 1 : 0, &p));
        prev = node;
    }
    void *kp[] = {&sb->d_ctl};
    hipKernelNodeParams p{};
    p.func = (void *)stage_advance;
    p.gridDim = dim3(1);
    p.blockDim = dim3(1);
    p.kernelParams = kp;
    hipGraphNode_t node;
    HIPCHK(hipGraphAddKernelNode(&node, sb->graph, &prev, 1, &p));
    HIPCHK(hipGraphInstantiate(&sb->exec, sb->graph, nullptr, nullptr, 0));
    return PSST_OK;
}

psst_status stage_batch_integrate(StageBatch *sb, float *states, const psst_stimulus *stim,
                                  float dt, int64_t n_steps, int64_t step0,
                                  const psst_record *rec, float *ckpt, int32_t K, void *stream)
{
    (void)K;
    if (ckpt) return fail(PSST_ERR_UNSUPPORTED, "checkpoints are not supported on the per-stage path");
    if (n_steps == 0) return PSST_OK;
    hipStream_t s = (hipStream_t)stream;
    if (!sb->exec) {
        psst_status st = build_graph(sb);
        if (st != PSST_OK) return st;
    }
    StageCtl c{};
    c.state = states;
    if (stim) {
        c.stim.i_const = stim->i_const_nA;
        c.stim.pulse_ptr = stim->pulse_ptr;
        c.stim.on_step = stim->on_step;
        c.stim.off_step = stim->off_step;
        c.stim.amp = stim->amp_nA;
    }
    if (rec) {
        c.rec.v_out = rec->v_out;
        c.rec.stride = rec->stride;
        c.rec.capacity = rec->capacity;
        c.rec.spike_count = rec->spike_count;
        c.rec.spike_t = rec->spike_t_ms;
        c.rec.spike_cap = rec->spike_cap;
    }
    c.dt = (double)dt;
    c.step0 = step0;
    c.g = step0;
    c.flag = sb->d_flag;
    void *args[] = {&sb->fx, &c, &sb->d_ctl};
    HIPCHK(hipLaunchKernel((const void *)stage_prologue, dim3(1024), dim3(256), args, 0, s));
    for (int64_t k = 0; k < n_steps; ++k) HIPCHK(hipGraphLaunch(sb->exec, s));
    return PSST_OK;
}

psst_status stage_batch_poll(StageBatch *sb, void *stream)
{
    HIPCHK(hipStreamSynchronize((hipStream_t)stream));
    int32_t f = 0;
    HIPCHK(hipMemcpy(&f, sb->d_flag, sizeof f, hipMemcpyDeviceToHost));
    if (f) {
        int32_t z = 0;
        HIPCHK(hipMemcpy(sb->d_flag, &z, sizeof z, hipMemcpyHostToDevice));
        return fail(PSST_ERR_NONFINITE, "a state variable became non-finite");
    }
    return PSST_OK;
}

psst_status stage_single_prepare(psst_network *net)
{
    if (net->single) return PSST_OK;
    psst_status st = stage_batch_create(net, 1, &net->single);
    if (st != PSST_OK) return st;
    net->single->fx.B = 1;
    // the network's own non-finite flag is the one its poll reads
    (void)hipFree(net->single->d_flag);
    net->single->d_flag = nullptr;
    return PSST_OK;
}

psst_status stage_integrate_single(psst_network *net, float *state, const psst_stimulus *stim,
                                   float dt, int64_t n_steps, int64_t step0,
                                   const psst_record *rec, void *stream)
{
    psst_status st0 = stage_single_prepare(net);     // made at network creation
    if (st0 != PSST_OK) return st0;
    StageBatch *sb = net->single;
    const int32_t *saved = sb->d_flag;
    sb->d_flag = net->d_flag;
    psst_status st = stage_batch_integrate(sb, state, stim, dt, n_steps, step0, rec, nullptr, 0,
                                           stream);
    sb->d_flag = const_cast<int32_t *>(saved);
    return st;
}
