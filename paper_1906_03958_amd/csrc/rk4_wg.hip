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
#include "wg_common.h"

namespace psst {

template <int BS, int NPT, bool GEN>
__global__ __launch_bounds__(BS) void rk4_wg_kernel(WGArgs a)
{
    extern __shared__ double lds_d[];
    const int32_t b = a.order[blockIdx.x];
    const InstDesc d = a.desc[b];
    const WGSyn w = wg_setup<BS>(d, lds_d, a.lds_bytes);
    const int tid = threadIdx.x;
    const int n = d.n, ld = d.ld;
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
        double Iu[NPT], vold[NPT];
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            Iu[k] = d.ci * stim_nA(a.stim, Ic[k], p0[k], p1[k], g);
            vold[k] = y[k][YV];
        }
        if constexpr (GEN)
            rk_step_wg_tab<BS, NPT>(w, K, d.cg, pr, Iu, dt, y, nullptr, a.tab);
        else
            rk4_step_wg<BS, NPT>(w, K, d.cg, pr, Iu, dt, y, nullptr);
        // spikes, records
        const bool do_rec = (g + 1 == next_rec);
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            if (!own[k]) continue;
            const int64_t gi = d.off + tid + k * BS;
            double chk = 0.0;
#pragma unroll
            for (int v = 0; v < NVAR; ++v) chk += y[k][v];
            bad |= !finite_d(chk);
            const double vnew = y[k][YV];
            if (a.rec.spike_count && vold[k] < 0.0 && vnew >= 0.0) {
                if (nspk[k] < a.rec.spike_cap)
                    a.rec.spike_t[gi * a.rec.spike_cap + nspk[k]] =
                        (float)(((double)g + (0.0 - vold[k]) / (vnew - vold[k])) * dt);
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

#define WGV(BS, NPT) {BS, NPT, false, (const void *)rk4_wg_kernel<BS, NPT, false>}
#define WGG(BS, NPT) {BS, NPT, true, (const void *)rk4_wg_kernel<BS, NPT, true>}

static const WGVariant kVariants[] = {
    WGV(64, 1), WGV(128, 1), WGV(128, 2), WGV(256, 1), WGV(256, 2), WGV(256, 4), WGV(512, 1),
    WGG(64, 1), WGG(128, 1), WGG(128, 2), WGG(256, 1), WGG(256, 2), WGG(256, 4), WGG(512, 1),
    {0, 0, false, nullptr},
};

const WGVariant *wg_variants() { return kVariants; }
const void *init_kernel() { return (const void *)init_state_kernel; }

}  // namespace psst
