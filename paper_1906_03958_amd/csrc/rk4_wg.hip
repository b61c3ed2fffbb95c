// rk4_wg.hip -- persistent RK4 kernel: one workgroup integrates one network
// instance through every step of the call, its state held in registers.
//
// Per step (paper, "Brain simulations as computational graphs": RK4 with four
// evaluations of f; vectorised per-neuron equations) and per stage:
//   1. stage input Y = y + c_q dt k_{q-1} (registers, float64);
//   2. presynaptic activations x_j (float64) into an LDS vector;
//   3. synaptic products sum_j g_ij x_j ("Circumventing memory constraints",
//      item 1: the synaptic update is a matrix-vector product) with the
//      transposed conductance matrix read row by row: a thread owns four
//      consecutive postsynaptic rows and one column chunk, reads
//      gt[j * ld + 4 r .. 4 r + 3] as one 16-byte load per column (a
//      wavefront load covers up to 1 KiB) and x_j as an LDS broadcast, so
//      each column group keeps several KiB of loads in flight; G comes from
//      LDS when it fits, else from L2/MALL/HBM.  G stays float32 (the given values); each product is
//      widened and summed in float64 -- float32 sums over a few hundred
//      synapses drift past 1e-3 mV within 50 ms, and on this chip a float64
//      FMA issues at the float32 rate, so the LDS-fed loop stays bound by LDS
//      bandwidth and the HBM-fed loop by HBM;
//   4. per-neuron right-hand side (float64) and RK4 accumulation.
// Then the combine y <- y + dt/6 (k1 + 2 k2 + 2 k3 + k4), stored as a float32
// pair, spike detection and recording.  Two barriers per stage (activations
// written; chunk partials written).
//
// Instance b's arithmetic does not depend on the workgroup size, on the other
// instances or on where its conductances live: the products are summed in
// column order j = 0, 1, ... with one float64 fma each, so every variant gives
// bitwise the same trajectory.
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

template <int BS, int NPT>
__global__ __launch_bounds__(BS) void rk4_wg_kernel(WGArgs a)
{
    extern __shared__ double lds_d[];
    const int32_t b = a.order[blockIdx.x];
    const InstDesc d = a.desc[b];
    const int n = d.n, n_pn = d.n_pn, ld = d.ld;
    const int n_ln = n - n_pn;
    const bool gabab = (d.flags & DESC_GABAB) != 0;
    const int tid = threadIdx.x;
    const Chunks ch = chunks_of(n, n_pn, gabab);
    const int nch = ch.na + ch.ng + ch.nb;
    double *xf = lds_d;                  // [ld] fast activations (s_j)
    double *xb = lds_d + ld;             // [ld] slow activations (G^n / (G^n + K_d))
    double *part = lds_d + 2 * ld;       // [nch][ld] chunk partial sums
    float *gl = reinterpret_cast<float *>(part + (size_t)nch * ld);

    // conductances in LDS when the instance fits this launch's allocation
    const bool glds = inst_lds_bytes(n, n_ln, ld, nch, gabab, true) <= a.lds_bytes;
    if (glds) {
        const int64_t nf4 = (int64_t)n * ld / 4;
        const float4 *src = reinterpret_cast<const float4 *>(d.gt);
        float4 *dst = reinterpret_cast<float4 *>(gl);
        for (int64_t e = tid; e < nf4; e += BS) dst[e] = src[e];
        if (gabab) {
            const int64_t nb4 = (int64_t)n_ln * ld / 4;
            const float4 *srcb = reinterpret_cast<const float4 *>(d.gtb);
            for (int64_t e = tid; e < nb4; e += BS) dst[nf4 + e] = srcb[e];
        }
    }

    // matvec thread mapping: row quad r4, column group cg
    const int RQ = ld >> 2;
    const int NCG = BS / RQ;
    const int r4 = tid % RQ;
    const int cg = tid / RQ;

    const Kin K = load_kin(d.kin);
    const double dt = a.dt;
    const int64_t NT = a.nt;

    bool own[NPT];
    double y[NPT][NVAR];
    float pr[NPT][NPRM];
    double Ic[NPT];       // constant injected current, nA
    int32_t p0[NPT], p1[NPT];
    int32_t nspk[NPT];
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
        const int i = tid + k * BS;
        own[k] = i < n;
        const int ic = own[k] ? i : 0;
        const int64_t gi = d.off + ic;
#pragma unroll
        for (int v = 0; v < NVAR; ++v)
            y[k][v] = (double)a.state[(2 * v) * NT + gi] + (double)a.state[(2 * v + 1) * NT + gi];
#pragma unroll
        for (int p = 0; p < NPRM; ++p) pr[k][p] = d.prm[p * ld + ic];
        Ic[k] = a.stim.i_const ? (double)a.stim.i_const[gi] : 0.0;
        p0[k] = a.stim.pulse_ptr ? a.stim.pulse_ptr[gi] : 0;
        p1[k] = a.stim.pulse_ptr ? a.stim.pulse_ptr[gi + 1] : 0;
        nspk[k] = (a.rec.spike_count && own[k]) ? a.rec.spike_count[gi] : 0;
    }

    const int64_t stride = a.rec.stride > 0 ? a.rec.stride : 0;
    int64_t next_rec = (a.rec.v_out && stride) ? (a.step0 / stride + 1) * stride : -1;
    int64_t rec_row = 0;
    int64_t next_ck = a.ckpt ? 0 : -1;
    int64_t ck_row = 0;
    bool bad = false;

    for (int64_t st = 0; st < a.n_steps; ++st) {
        const int64_t g = a.step0 + st;
        if (st == next_ck) {
            float *cp = a.ckpt + ck_row * (14 * NT);
#pragma unroll
            for (int k = 0; k < NPT; ++k) {
                if (!own[k]) continue;
                const int64_t gi = d.off + tid + k * BS;
#pragma unroll
                for (int v = 0; v < NVAR; ++v) {
                    float hi, lo;
                    split_store(y[k][v], hi, lo);
                    cp[(2 * v) * NT + gi] = hi;
                    cp[(2 * v + 1) * NT + gi] = lo;
                }
            }
            ck_row++;
            next_ck += a.K;
        }
        double Iu[NPT];
        double acc[NPT][NVAR];
        double Y[NPT][NVAR];
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            double I = Ic[k];
            for (int p = p0[k]; p < p1[k]; ++p)
                if (a.stim.on_step[p] <= g && g < a.stim.off_step[p]) I += (double)a.stim.amp[p];
            Iu[k] = d.ci * I;
#pragma unroll
            for (int v = 0; v < NVAR; ++v) {
                acc[k][v] = 0.0;
                Y[k][v] = y[k][v];
            }
        }
#pragma unroll 1
        for (int q = 0; q < 4; ++q) {
#pragma unroll
            for (int k = 0; k < NPT; ++k) {
                const int i = tid + k * BS;
                if (own[k]) {
                    xf[i] = Y[k][YS];
                    if (gabab && i >= n_pn) xb[i - n_pn] = gabab_act(Y[k][YG], K);
                }
            }
            __syncthreads();
            if (cg < NCG) {
                if (glds)
                    stage_partials(gl, gl + (int64_t)n * ld, ld, xf, xb, part, ch, n, n_pn, cg,
                                   NCG, r4);
                else
                    stage_partials(d.gt, d.gtb, ld, xf, xb, part, ch, n, n_pn, cg, NCG, r4);
            }
            __syncthreads();
#pragma unroll
            for (int k = 0; k < NPT; ++k) {
                if (k * BS >= n) continue;
                const int i = tid + k * BS;
                const int ir = own[k] ? i : 0;
                double sa = 0.0, sg = 0.0, sb = 0.0;
                for (int c = 0; c < ch.na; ++c) sa += part[(size_t)c * ld + ir];
                for (int c = ch.na; c < ch.na + ch.ng; ++c) sg += part[(size_t)c * ld + ir];
                for (int c = ch.na + ch.ng; c < nch; ++c) sb += part[(size_t)c * ld + ir];
                Prm P;
                P.C = pr[k][P_CM];  P.gNa = pr[k][P_GNA]; P.gK = pr[k][P_GK];
                P.gL = pr[k][P_GL]; P.ENa = pr[k][P_ENA]; P.EK = pr[k][P_EK];
                P.EL = pr[k][P_EL];
                double f[NVAR];
                hh_rhs(Y[k], P, K, d.cg * sa, d.cg * sg, d.cg * sb, Iu[k], i >= n_pn, gabab, f);
                const double w = (q == 0 || q == 3) ? 1.0 : 2.0;
                const double c = (q == 2) ? dt : 0.5 * dt;
#pragma unroll
                for (int v = 0; v < NVAR; ++v) {
                    acc[k][v] += w * f[v];
                    if (q < 3) Y[k][v] = y[k][v] + c * f[v];
                }
            }
        }
        // combine, spikes, records
        const bool do_rec = (g + 1 == next_rec);
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            if (!own[k]) continue;
            const int64_t gi = d.off + tid + k * BS;
            const double vold = y[k][YV];
            double chk = 0.0;
#pragma unroll
            for (int v = 0; v < NVAR; ++v) {
                float hi, lo;
                y[k][v] = split_store(y[k][v] + (dt / 6.0) * acc[k][v], hi, lo);
                chk += y[k][v];
            }
            bad |= !finite_d(chk);
            const double vnew = y[k][YV];
            if (a.rec.spike_count && vold < 0.0 && vnew >= 0.0) {
                if (nspk[k] < a.rec.spike_cap)
                    a.rec.spike_t[gi * a.rec.spike_cap + nspk[k]] =
                        (float)(((double)g + (0.0 - vold) / (vnew - vold)) * dt);
                nspk[k]++;
            }
            if (do_rec && rec_row < a.rec.capacity)
                a.rec.v_out[rec_row * NT + gi] = (float)vnew;
        }
        if (do_rec) {
            rec_row++;
            next_rec += stride;
        }
    }
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
        if (!own[k]) continue;
        const int64_t gi = d.off + tid + k * BS;
#pragma unroll
        for (int v = 0; v < NVAR; ++v) {
            float hi, lo;
            split_store(y[k][v], hi, lo);
            a.state[(2 * v) * NT + gi] = hi;
            a.state[(2 * v + 1) * NT + gi] = lo;
        }
        if (a.rec.spike_count) a.rec.spike_count[gi] = nspk[k];
    }
    if (bad) atomicOr(a.flag, 1);
}

// Initial state: V = v0, gates at steady state, synaptic variables 0.
__global__ __launch_bounds__(256) void init_state_kernel(InitArgs a)
{
    const InstDesc d = a.desc[blockIdx.x];
    for (int i = threadIdx.x; i < d.n; i += blockDim.x) {
        const int64_t gi = d.off + i;
        const double V = (double)a.v0[gi];
        const Rates r = hh_rates(V);
        double y[NVAR] = {V, r.am / (r.am + r.bm), r.ah / (r.ah + r.bh), r.an / (r.an + r.bn),
                          0.0, 0.0, 0.0};
#pragma unroll
        for (int v = 0; v < NVAR; ++v) {
            float hi, lo;
            split_store(y[v], hi, lo);
            a.state[(2 * v) * a.nt + gi] = hi;
            a.state[(2 * v + 1) * a.nt + gi] = lo;
        }
    }
}

#define WGV(BS, NPT) {BS, NPT, (const void *)rk4_wg_kernel<BS, NPT>}

static const WGVariant kVariants[] = {
    WGV(64, 1), WGV(128, 1), WGV(128, 2), WGV(256, 1), WGV(256, 2), WGV(256, 4), WGV(512, 1),
    {0, 0, nullptr},
};

const WGVariant *wg_variants() { return kVariants; }
const void *init_kernel() { return (const void *)init_state_kernel; }

}  // namespace psst
