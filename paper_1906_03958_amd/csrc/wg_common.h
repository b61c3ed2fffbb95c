// wg_common.h -- device code shared by the per-instance forward kernel and
// the adjoint kernel: the fixed summation structure of the synaptic
// products and the LDS layout of one instance.  The adjoint's forward
// recomputation uses exactly these routines, so it reproduces the forward
// trajectory bit for bit.
#pragma once

#include "kernels.h"

namespace psst {

// Fixed summation structure of the synaptic products: columns are cut into
// chunks of CW consecutive presynaptic neurons (cholinergic columns, then
// fast-GABA columns, then the slow-GABA matrix); each chunk's partial sum runs
// in column order and the partials are added in chunk order.  Every launch
// shape follows this structure, so results are bitwise independent of it.
constexpr int CW = kChunkWidth;

struct Chunks {
    int na, ng, nb;    // chunks over the ACh columns, fast-GABA columns, slow matrix
};

__device__ inline Chunks chunks_of(int n, int n_pn, bool gabab)
{
    Chunks c;
    c.na = (n_pn + CW - 1) / CW;
    c.ng = (n - n_pn + CW - 1) / CW;
    c.nb = gabab ? c.ng : 0;
    return c;
}

// Partial sums of one chunk for rows 4 r4 .. 4 r4 + 3.  Columns go in
// batches of U: all U loads are issued before the first is consumed, so each
// wavefront keeps U 16-byte loads in flight.  Past the chunk end the row
// index is clamped and the activation taken as 0, which adds exact zeros and
// leaves the column-order sum unchanged.
template <int U>
__device__ __forceinline__ void chunk_rows4(const float *G, int ld, const double *x, int j0,
                                            int j1, int r4, double &s0, double &s1, double &s2,
                                            double &s3)
{
    const float4 *G4 = reinterpret_cast<const float4 *>(G);
    const int q = ld >> 2;
    s0 = s1 = s2 = s3 = 0.0;
    for (int j = j0; j < j1; j += U) {
        float4 g[U];
        double xv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int jj = min(j + u, j1 - 1);
            g[u] = G4[(int64_t)jj * q + r4];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) xv[u] = (j + u < j1) ? x[j + u] : 0.0;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            s0 = fma((double)g[u].x, xv[u], s0);
            s1 = fma((double)g[u].y, xv[u], s1);
            s2 = fma((double)g[u].z, xv[u], s2);
            s3 = fma((double)g[u].w, xv[u], s3);
        }
    }
}

// One stage's chunk partials: column group cg takes chunks cg, cg + NCG, ...
__device__ __forceinline__ void stage_partials(const float *G, const float *GB, int ld,
                                               const double *xf, const double *xb,
                                               double *part, const Chunks &ch, int n, int n_pn,
                                               int cg, int NCG, int r4)
{
    const int nch = ch.na + ch.ng + ch.nb;
    for (int c = cg; c < nch; c += NCG) {
        const float *M;
        const double *X;
        int j0, j1;
        if (c < ch.na) {
            M = G; X = xf; j0 = c * CW; j1 = min(j0 + CW, n_pn);
        } else if (c < ch.na + ch.ng) {
            M = G; X = xf; j0 = n_pn + (c - ch.na) * CW; j1 = min(j0 + CW, n);
        } else {
            M = GB; X = xb; j0 = (c - ch.na - ch.ng) * CW; j1 = min(j0 + CW, n - n_pn);
        }
        double s0, s1, s2, s3;
        chunk_rows4<8>(M, ld, X, j0, j1, r4, s0, s1, s2, s3);
        double *pc = part + (size_t)c * ld + 4 * r4;
        pc[0] = s0; pc[1] = s1; pc[2] = s2; pc[3] = s3;
    }
}

// LDS layout of one instance: activations xf[ld], xb[ld], chunk partials
// [nch][ld] (float64), then -- when the whole instance fits the launch's LDS
// allocation -- its conductances gt[n][ld] and gtb[n_ln][ld] (float32).
__device__ __forceinline__ size_t inst_lds_bytes(int n, int n_ln, int ld, int nch, bool gabab,
                                                 bool with_g)
{
    size_t b = sizeof(double) * (size_t)(2 + nch) * ld;
    if (with_g) b += sizeof(float) * ((size_t)n * ld + (gabab ? (size_t)n_ln * ld : 0));
    return b;
}


// Injected current (nA) of one neuron at global step g: constant part plus
// the pulses p0 .. p1-1 that are on (zero-order hold over the step).
__device__ __forceinline__ double stim_nA(const StimDev &s, double Ic, int32_t p0, int32_t p1,
                                          int64_t g)
{
    double I = Ic;
    for (int p = p0; p < p1; ++p)
        if (s.on_step[p] <= g && g < s.off_step[p]) I += (double)s.amp[p];
    return I;
}

// Per-workgroup view of one instance for the synaptic sums.
struct WGSyn {
    const float *gt, *gtb;     // conductances in global memory
    const float *gl;           // LDS copy (gt rows then gtb rows) when glds
    double *xf, *xb, *part;    // LDS activations and chunk partials
    Chunks ch;
    int n, n_pn, ld, nch, NCG, r4, cg;
    bool glds, gabab;
};

// Synaptic sums (nS) at stage input Y for the calling thread's neurons
// i = tid + k * BS: write the activations, sync, form the chunk partials, sync,
// add the partials in chunk order.  Every thread of the workgroup must call.
template <int BS, int NPT>
__device__ __forceinline__ void syn_sums(const WGSyn &w, const Kin &K, const double (&Y)[NPT][NVAR],
                                         double (&sa)[NPT], double (&sg)[NPT], double (&sb)[NPT])
{
    const int tid = threadIdx.x;
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
        const int i = tid + k * BS;
        if (i < w.n) {
            w.xf[i] = Y[k][YS];
            if (w.gabab && i >= w.n_pn) w.xb[i - w.n_pn] = gabab_act(Y[k][YG], K);
        }
    }
    __syncthreads();
    if (w.cg < w.NCG) {
        if (w.glds)
            stage_partials(w.gl, w.gl + (int64_t)w.n * w.ld, w.ld, w.xf, w.xb, w.part, w.ch, w.n,
                           w.n_pn, w.cg, w.NCG, w.r4);
        else
            stage_partials(w.gt, w.gtb, w.ld, w.xf, w.xb, w.part, w.ch, w.n, w.n_pn, w.cg, w.NCG,
                           w.r4);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
        const int i = tid + k * BS;
        const int ir = i < w.n ? i : 0;
        double a = 0.0, g = 0.0, b = 0.0;
        for (int c = 0; c < w.ch.na; ++c) a += w.part[(size_t)c * w.ld + ir];
        for (int c = w.ch.na; c < w.ch.na + w.ch.ng; ++c) g += w.part[(size_t)c * w.ld + ir];
        for (int c = w.ch.na + w.ch.ng; c < w.nch; ++c) b += w.part[(size_t)c * w.ld + ir];
        sa[k] = a;
        sg[k] = g;
        sb[k] = b;
    }
}

__device__ __forceinline__ Prm prm_of(const float (&pr)[NPRM])
{
    Prm P;
    P.C = pr[P_CM];  P.gNa = pr[P_GNA]; P.gK = pr[P_GK]; P.gL = pr[P_GL];
    P.ENa = pr[P_ENA]; P.EK = pr[P_EK]; P.EL = pr[P_EL];
    return P;
}

// Optional record of a step's stage inputs Y_q and synaptic sums (nS), for
// the adjoint: sY[(q * NVAR + v) * ld + i], sS[(q * 3 + t) * ld + i].
struct StageStash {
    double *sY, *sS;
    int ld;
};

// One RK4 step of the calling thread's neurons, y updated in place and
// rounded to its stored float32 pair.  Iu: injected current (uA/cm^2).
template <int BS, int NPT>
__device__ __forceinline__ void rk4_step_wg(const WGSyn &w, const Kin &K, double cgf,
                                            const float (&pr)[NPT][NPRM], const double (&Iu)[NPT],
                                            double dt, double (&y)[NPT][NVAR],
                                            const StageStash *stash)
{
    const int tid = threadIdx.x;
    double acc[NPT][NVAR];
    double Y[NPT][NVAR];
#pragma unroll
    for (int k = 0; k < NPT; ++k)
#pragma unroll
        for (int v = 0; v < NVAR; ++v) {
            acc[k][v] = 0.0;
            Y[k][v] = y[k][v];
        }
#pragma unroll 1
    for (int q = 0; q < 4; ++q) {
        double sa[NPT], sg[NPT], sb[NPT];
        syn_sums<BS, NPT>(w, K, Y, sa, sg, sb);
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            if (k * BS >= w.n) continue;
            const int i = tid + k * BS;
            if (stash && i < w.n) {
#pragma unroll
                for (int v = 0; v < NVAR; ++v) stash->sY[(q * NVAR + v) * stash->ld + i] = Y[k][v];
                stash->sS[(q * 3 + 0) * stash->ld + i] = sa[k];
                stash->sS[(q * 3 + 1) * stash->ld + i] = sg[k];
                stash->sS[(q * 3 + 2) * stash->ld + i] = sb[k];
            }
            double f[NVAR];
            hh_rhs(Y[k], prm_of(pr[k]), K, cgf * sa[k], cgf * sg[k], cgf * sb[k], Iu[k],
                   i >= w.n_pn, w.gabab, f);
            const double wq = (q == 0 || q == 3) ? 1.0 : 2.0;
            const double c = (q == 2) ? dt : 0.5 * dt;
#pragma unroll
            for (int v = 0; v < NVAR; ++v) {
                acc[k][v] += wq * f[v];
                if (q < 3) Y[k][v] = y[k][v] + c * f[v];
            }
        }
    }
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
        if (tid + k * BS >= w.n) continue;
#pragma unroll
        for (int v = 0; v < NVAR; ++v) {
            float hi, lo;
            y[k][v] = split_store(y[k][v] + (dt / 6.0) * acc[k][v], hi, lo);
        }
    }
}

// Set up the workgroup's view of instance d: LDS carve-up and, when the
// whole instance fits the launch's LDS allocation, the conductance copy.
template <int BS>
__device__ __forceinline__ WGSyn wg_setup(const InstDesc &d, double *lds_d, int64_t lds_bytes)
{
    WGSyn w;
    w.n = d.n;
    w.n_pn = d.n_pn;
    w.ld = d.ld;
    w.gabab = (d.flags & DESC_GABAB) != 0;
    w.ch = chunks_of(d.n, d.n_pn, w.gabab);
    w.nch = w.ch.na + w.ch.ng + w.ch.nb;
    w.xf = lds_d;
    w.xb = lds_d + d.ld;
    w.part = lds_d + 2 * d.ld;
    float *gl = reinterpret_cast<float *>(w.part + (size_t)w.nch * d.ld);
    w.gl = gl;
    w.gt = d.gt;
    w.gtb = d.gtb;
    const int n_ln = d.n - d.n_pn;
    w.glds = inst_lds_bytes(d.n, n_ln, d.ld, w.nch, w.gabab, true) <= (size_t)lds_bytes;
    const int tid = threadIdx.x;
    if (w.glds) {
        const int64_t nf4 = (int64_t)d.n * d.ld / 4;
        const float4 *src = reinterpret_cast<const float4 *>(d.gt);
        float4 *dst = reinterpret_cast<float4 *>(gl);
        for (int64_t e = tid; e < nf4; e += BS) dst[e] = src[e];
        if (w.gabab) {
            const int64_t nb4 = (int64_t)n_ln * d.ld / 4;
            const float4 *srcb = reinterpret_cast<const float4 *>(d.gtb);
            for (int64_t e = tid; e < nb4; e += BS) dst[nf4 + e] = srcb[e];
        }
    }
    const int RQ = d.ld >> 2;
    w.NCG = BS / RQ;
    w.r4 = tid % RQ;
    w.cg = tid / RQ;
    return w;
}

}  // namespace psst
