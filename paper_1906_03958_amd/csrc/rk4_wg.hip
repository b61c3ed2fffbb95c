// rk4_wg.hip -- persistent RK4 kernel: one workgroup integrates one network
// instance through every step of the call, its state held in registers.
//
// Per step (paper, "Brain simulations as computational graphs": RK4 with four
// evaluations of f; vectorised per-neuron equations) and per stage:
//   1. stage input Y = y + c_q dt k_{q-1} (registers, float64);
//   2. presynaptic activations x_j (float64) into a double-buffered LDS vector;
//   3. synaptic products sum_j g_ij x_j ("Circumventing memory constraints",
//      item 1: the synaptic update is a matrix-vector product) with the
//      transposed conductance matrix read row by row: thread i reads
//      gt[j * ld + i], so each wavefront load is 256 contiguous bytes and x_j
//      is an LDS broadcast; G comes from LDS when it fits, else from
//      L2/MALL/HBM.  G stays float32 (the given values); each product is
//      widened and summed in float64 -- float32 sums over a few hundred
//      synapses drift past 1e-3 mV within 50 ms, and on this chip a float64
//      FMA issues at the float32 rate, so the LDS-fed loop stays bound by LDS
//      bandwidth and the HBM-fed loop by HBM;
//   4. per-neuron right-hand side (float64) and RK4 accumulation.
// Then the combine y <- y + dt/6 (k1 + 2 k2 + 2 k3 + k4), stored as a float32
// pair, spike detection and recording.  One barrier per stage.
//
// Instance b's arithmetic does not depend on the workgroup size, on the other
// instances or on where its conductances live: the products are summed in
// column order j = 0, 1, ... with one float64 fma each, so every variant gives
// bitwise the same trajectory.
#include "kernels.h"

namespace psst {

template <int BS, int NPT, bool GLDS>
__global__ __launch_bounds__(BS) void rk4_wg_kernel(WGArgs a)
{
    extern __shared__ float lds[];
    const int32_t b = a.order[blockIdx.x];
    const InstDesc d = a.desc[b];
    const int n = d.n, n_pn = d.n_pn, ld = d.ld;
    const int n_ln = n - n_pn;
    const bool gabab = (d.flags & DESC_GABAB) != 0;
    const int tid = threadIdx.x;
    const int LX = a.lds_ld;
    double *xf = reinterpret_cast<double *>(lds);   // [2][LX] fast activations (s_j)
    double *xb = xf + 2 * LX;                       // [2][LX] slow activations

    const float *G = d.gt;
    const float *GB = d.gtb;
    if (GLDS) {
        float *gl = lds + 8 * LX;
        const int64_t nf = (int64_t)n * ld;
        for (int64_t e = tid; e < nf; e += BS) gl[e] = d.gt[e];
        if (gabab) {
            const int64_t nb = (int64_t)n_ln * ld;
            for (int64_t e = tid; e < nb; e += BS) gl[nf + e] = d.gtb[e];
        }
        G = gl;
        GB = gl + nf;
    }

    const Kin K = load_kin(d.kin);
    const double dt = a.dt;
    const int64_t NT = a.nt;

    int ik[NPT];          // matvec row (clamped inside the padded row)
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
        ik[k] = i < ld ? i : ld - 1;
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
    bool bad = false;

    for (int64_t st = 0; st < a.n_steps; ++st) {
        const int64_t g = a.step0 + st;
        if (a.ckpt && (st % a.K) == 0) {
            float *cp = a.ckpt + (st / a.K) * (14 * NT);
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
            double *xfq = xf + (q & 1) * LX;
            double *xbq = xb + (q & 1) * LX;
#pragma unroll
            for (int k = 0; k < NPT; ++k) {
                const int i = tid + k * BS;
                if (own[k]) {
                    xfq[i] = Y[k][YS];
                    if (gabab && i >= n_pn) xbq[i - n_pn] = gabab_act(Y[k][YG], K);
                }
            }
            __syncthreads();
            double sa[NPT], sg[NPT], sb[NPT];
#pragma unroll
            for (int k = 0; k < NPT; ++k) { sa[k] = 0.0; sg[k] = 0.0; sb[k] = 0.0; }
#pragma unroll 4
            for (int j = 0; j < n_pn; ++j) {
                const double x = xfq[j];
                const float *row = G + (int64_t)j * ld;
#pragma unroll
                for (int k = 0; k < NPT; ++k)
                    if (k * BS < n) sa[k] = fma((double)row[ik[k]], x, sa[k]);
            }
#pragma unroll 4
            for (int j = n_pn; j < n; ++j) {
                const double x = xfq[j];
                const float *row = G + (int64_t)j * ld;
#pragma unroll
                for (int k = 0; k < NPT; ++k)
                    if (k * BS < n) sg[k] = fma((double)row[ik[k]], x, sg[k]);
            }
            if (gabab) {
#pragma unroll 4
                for (int j = 0; j < n_ln; ++j) {
                    const double x = xbq[j];
                    const float *row = GB + (int64_t)j * ld;
#pragma unroll
                    for (int k = 0; k < NPT; ++k)
                        if (k * BS < n) sb[k] = fma((double)row[ik[k]], x, sb[k]);
                }
            }
#pragma unroll
            for (int k = 0; k < NPT; ++k) {
                if (k * BS >= n) continue;
                const int i = tid + k * BS;
                Prm P;
                P.C = pr[k][P_CM];  P.gNa = pr[k][P_GNA]; P.gK = pr[k][P_GK];
                P.gL = pr[k][P_GL]; P.ENa = pr[k][P_ENA]; P.EK = pr[k][P_EK];
                P.EL = pr[k][P_EL];
                double f[NVAR];
                hh_rhs(Y[k], P, K, d.cg * sa[k], d.cg * sg[k], d.cg * sb[k], Iu[k],
                       i >= n_pn, gabab, f);
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

#define WGV(BS, NPT, GL) {BS, NPT, GL, (const void *)rk4_wg_kernel<BS, NPT, GL>}

static const WGVariant kVariants[] = {
    WGV(64, 1, false),  WGV(64, 1, true),
    WGV(128, 1, false), WGV(128, 1, true),
    WGV(128, 2, false), WGV(128, 2, true),
    WGV(256, 1, false), WGV(256, 1, true),
    WGV(256, 2, false), WGV(256, 2, true),
    WGV(256, 4, false), WGV(256, 4, true),
    WGV(512, 1, false), WGV(512, 1, true),
    {0, 0, false, nullptr},
};

const WGVariant *wg_variants() { return kVariants; }
const void *init_kernel() { return (const void *)init_state_kernel; }

}  // namespace psst
