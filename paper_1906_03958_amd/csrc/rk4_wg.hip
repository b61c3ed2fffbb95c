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

// The integration loop of one instance for every step of the call: state
// in registers, stimulus at each step's start (zero-order hold), spikes and
// records after each step, checkpoints before each K-th step, state stored at
// the end.  Slot k of the calling thread is neuron nid(k); own(k) says
// whether this thread carries that neuron (loads, stores, records); step(Iu,
// y) advances every slot by one step and is called by every thread.
template <int NPT, typename Nid, typename Own, typename Step>
__device__ __forceinline__ void integrate_loop(const WGArgs &a, const InstDesc &d, Nid &&nid,
                                               Own &&own_of, Step &&step)
{
    const int n = d.n, ld = d.ld;
    const int64_t NT = a.nt;
    const float *sin = a.state_in ? a.state_in : a.state;
    bool own[NPT];
    double y[NPT][NVAR];
    float pr[NPT][NPRM];
    double Ic[NPT];       // constant injected current, nA
    int32_t p0[NPT], p1[NPT];
    int32_t nspk[NPT];
    StimCache sc[NPT];
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
        sc[k].I = 0.0;
        sc[k].next = -1;
        const int i = nid(k);
        own[k] = own_of(k);
        const int ic = (own[k] && i < n) ? i : 0;
        const int64_t gi = d.off + ic;
#pragma unroll
        for (int v = 0; v < NVAR; ++v)
            y[k][v] = (double)sin[(2 * v) * NT + gi] + (double)sin[(2 * v + 1) * NT + gi];
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
                const int64_t gi = d.off + nid(k);
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
            Iu[k] = d.ci * stim_nA_cached(a.stim, Ic[k], p0[k], p1[k], g, sc[k]);
            vold[k] = y[k][YV];
        }
        StageStash stash;
        if (a.stash) {
            double *base = a.stash + (int64_t)a.order[blockIdx.x] * a.stash_stride;
            stash.sY = base + st * 4 * NVAR * ld;
            stash.sS = base + (int64_t)a.stash_K * 4 * NVAR * ld + st * 12 * ld;
            stash.ld = ld;
        }
        step(pr, Iu, y, a.stash ? &stash : nullptr);
        // spikes, records
        const bool do_rec = (g + 1 == next_rec);
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            if (!own[k]) continue;
            const int64_t gi = d.off + nid(k);
            double chk = 0.0;
#pragma unroll
            for (int v = 0; v < NVAR; ++v) chk += y[k][v];
            bad |= !finite_d(chk);
            const double vnew = y[k][YV];
            if (a.rec.spike_count && vold[k] < 0.0 && vnew >= 0.0) {
                if (nspk[k] < a.rec.spike_cap)
                    a.rec.spike_t[gi * a.rec.spike_cap + nspk[k]] =
                        (float)(((double)g + (0.0 - vold[k]) / (vnew - vold[k])) * a.dt);
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
        const int64_t gi = d.off + nid(k);
        if (a.store_state) {
#pragma unroll
            for (int v = 0; v < NVAR; ++v) {
                float hi, lo;
                split_store(y[k][v], hi, lo);
                a.state[(2 * v) * NT + gi] = hi;
                a.state[(2 * v + 1) * NT + gi] = lo;
            }
        }
        if (a.rec.spike_count) a.rec.spike_count[gi] = nspk[k];
    }
    if (bad) atomicOr(a.flag, 1);
}

// A double moved between the lanes of each quad (four consecutive lanes):
// lane q of the quad receives the value of lane (q + D) mod 4 (DPP quad
// permutation, no LDS traffic).
template <int D>
__device__ __forceinline__ double quad_rotate(double v)
{
    constexpr int ctrl = ((0 + D) & 3) | (((1 + D) & 3) << 2) | (((2 + D) & 3) << 4) |
                         (((3 + D) & 3) << 6);
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffLL), ctrl, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), ctrl, 0xf, 0xf, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Lane-group mapping (small dense networks, kLGThreads = 256 threads, one
// wavefront per SIMD so that a lane has room for its conductances): lane
// 4 r + c of wavefront w takes the pairs (chunk c, row i_k = 64 k + 16 w +
// r), k < RPL row blocks, and keeps their 64 conductances each in registers
// for the whole launch (zeros past the chunk's last column); lane 4 r + k
// owns neuron i_k (k < RPL).  Per stage the owners write their activations
// into the chunk slots of one of two LDS slot sets (alternating by stage, so
// a wavefront that runs ahead writes the other set), one barrier, each lane
// sums its pairs in column order -- the fma sequence of every other mapping,
// the zero columns adding exact zeros -- and each owner collects its row's
// partials from the other lanes of its quad (three quad permutations: at
// distance d the source lane offers the partial of row block (c' - d) mod 4)
// and adds them in chunk order, per synapse class.  An LN owner of a network
// with slow GABA forms the next stage's slow activation as soon as the stage
// update has its input, beside the rest of the right-hand side.
template <bool GEN, int RPL>
__device__ __forceinline__ void lg_integrate(const WGArgs &a, const InstDesc &d, double *lds)
{
    static_assert(RPL >= 1 && RPL <= 4, "row blocks are owned by quad lanes 0 .. RPL-1");
    const int tid = threadIdx.x, lane = tid & 63;
    const int cl = lane & 3, r = lane >> 2;
    const int row0 = (tid >> 6) * 16 + r;
    const int n = d.n, n_pn = d.n_pn, ld = d.ld;
    const bool gabab = (d.flags & DESC_GABAB) != 0;
    const Chunks ch = chunks_of(n, n_pn, gabab);
    const int nch = ch.na + ch.ng + ch.nb;
    const Kin K = load_kin(d.kin);
    int mat = 0, j0 = 0, j1 = 0;
    if (cl < nch) chunk_range(ch, n, n_pn, cl, mat, j0, j1);
    const int wc = j1 - j0;               // columns of this lane's chunk (0: no chunk)
    float g[RPL][CW];
#pragma unroll
    for (int k = 0; k < RPL; ++k) {
        const int i = row0 + 64 * k;
        const bool pair = wc > 0 && i < n;
        // every address is inside the matrix (row j0 + min(u, wc - 1), or
        // entry 0 for a lane without a pair); the value is kept only for the
        // chunk's own columns
        const float *M = (mat ? d.gtb : d.gt) + (pair ? i : 0);
#pragma unroll
        for (int u = 0; u < CW; ++u) {
            const int64_t jj = pair ? (int64_t)(j0 + min(u, wc - 1)) * ld : 0;
            const float v = M[jj];
            g[k][u] = (pair && u < wc) ? v : 0.f;
        }
    }
    const int me = row0 + 64 * cl;        // the neuron this lane owns when cl < RPL
    const bool owner = cl < RPL && me < n;
    const bool slow_owner = owner && gabab && me >= n_pn;
    double xb_next = 0.0;                 // slow activation of the next stage input
    bool xb_ready = false;
    // both slot sets start at zero: columns past a chunk's end stay 0
    for (int e = tid; e < 2 * 4 * kLGSlot; e += kLGThreads) lds[e] = 0.0;
    __syncthreads();
    int parity = 0;
    RateSet rs_pre;                       // the owner's factors, formed in syn
    auto syn = [&](const double (&Y)[1][NVAR], double (&sa)[1], double (&sg)[1],
                   double (&sb)[1]) {
        double *S = lds + parity * 4 * kLGSlot;
        parity ^= 1;
        if (owner) {
            const bool ln = me >= n_pn;
            const int c = ln ? ch.na + (me - n_pn) / CW : me / CW;
            const int u = ln ? (me - n_pn) % CW : me % CW;
            S[c * kLGSlot + u] = Y[0][YS];
            if (slow_owner)
                S[(ch.na + ch.ng + (me - n_pn) / CW) * kLGSlot + u] =
                    xb_ready ? xb_next : gabab_act(Y[0][YG], K);
        }
        xb_ready = false;
        // the owner's voltage-dependent factors for this stage's right-hand
        // side (they need only its V), formed before the barrier, where a
        // wavefront that arrives early would otherwise wait (measured: 120
        // neurons 10.8 -> 10.4 us per step; formed after the barrier 11.1)
        rs_pre = rate_set(Y[0][YV], K, me >= n_pn, me >= n_pn && gabab);
        __syncthreads();
        // the partial sums as one straight-line block: a lane whose chunk is
        // narrower than 64 columns, or that has none, holds g = 0 there and
        // its activation slots past the chunk's end hold 0, so the extra
        // columns add exact zeros (every lane of a wavefront runs all of them
        // anyway, its lanes' chunks differing)
        double p[RPL];
#pragma unroll
        for (int k = 0; k < RPL; ++k) p[k] = 0.0;
        {
            lds_double *X = (lds_double *)(S + (cl < nch ? cl : 0) * kLGSlot);
#pragma unroll
            for (int u0 = 0; u0 < CW; u0 += 8) {
                double xv[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) xv[u] = X[u0 + u];
#pragma unroll
                for (int u = 0; u < 8; ++u)
#pragma unroll
                    for (int k = 0; k < RPL; ++k) p[k] = fma((double)g[k][u0 + u], xv[u], p[k]);
            }
        }
        // pd[dd] = partial of chunk (cl + dd) mod 4 for this lane's row block cl:
        // the quad lane dd places further offers its partial of row block
        // (its c - dd) mod 4
        double offer[4];
#pragma unroll
        for (int dd = 0; dd < 4; ++dd) {
            const int kk = (cl - dd) & 3;
            double o = 0.0;
#pragma unroll
            for (int k = 0; k < RPL; ++k) o = kk == k ? p[k] : o;
            offer[dd] = o;
        }
        const double pd[4] = {offer[0], quad_rotate<1>(offer[1]), quad_rotate<2>(offer[2]),
                              quad_rotate<3>(offer[3])};
        double ta = 0.0, tg = 0.0, tb = 0.0;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int dd = (c - cl) & 3;
            double v = pd[0];
#pragma unroll
            for (int e = 1; e < 4; ++e) v = dd == e ? pd[e] : v;
            if (c < ch.na) ta += v;
            else if (c < ch.na + ch.ng) tg += v;
            else if (c < nch) tb += v;
        }
        sa[0] = ta;
        sg[0] = tg;
        sb[0] = tb;
    };
    auto post = [&](int, const double (&Yn)[NVAR]) {
        if (slow_owner) {
            xb_next = gabab_act(Yn[YG], K);
            xb_ready = true;
        }
    };
    const Slots sl{n, n_pn, gabab};
    auto nid = [&](int) { return me; };
    auto own = [&](int) { return owner; };
    const double dt = a.dt;
    integrate_loop<1>(a, d, nid, own,
                      [&](const float (&pr)[1][NPRM], const double (&Iu)[1], double (&y)[1][NVAR],
                          const StageStash *stash) {
                          auto rates = [&](int, const double (&)[NVAR], const Kin &, bool,
                                           bool) { return rs_pre; };
                          if constexpr (GEN)
                              rk_step_core_tab<1>(sl, syn, nid, own, K, d.cg, pr, Iu, dt, y,
                                                  stash, a.tab, post, rates);
                          else
                              rk4_step_core<1>(sl, syn, nid, own, K, d.cg, pr, Iu, dt, y, stash,
                                               post, rates);
                      });
}

// S > 0: the variant keeps conductance columns in S float4 register slots per
// thread for instances that stream part of their conductances (the register
// file of a one-wavefront-per-SIMD workgroup beside its LDS).
template <int BS, int NPT, bool GEN, int S = 0>
__global__ __launch_bounds__(BS) void rk4_wg_kernel(WGArgs a)
{
    extern __shared__ double lds_d[];
    const int32_t b = a.order[blockIdx.x];
    const InstDesc d = a.desc[b];
    const WGSyn w = wg_setup<BS>(d, lds_d, a.lds_bytes, S);
    RegCols<S> rc;
    if constexpr (S > 0) load_regcols<S>(rr_view(w), rc);
    const int tid = threadIdx.x;
    const Kin K = load_kin(d.kin);
    const double dt = a.dt;
    integrate_loop<NPT>(
        a, d, [&](int k) { return tid + k * BS; }, [&](int k) { return tid + k * BS < d.n; },
        [&](const float (&pr)[NPT][NPRM], const double (&Iu)[NPT], double (&y)[NPT][NVAR],
            const StageStash *stash) {
            if constexpr (GEN)
                rk_step_wg_tab<BS, NPT, S>(w, K, d.cg, pr, Iu, dt, y, stash, a.tab, &rc);
            else
                rk4_step_wg<BS, NPT, S>(w, K, d.cg, pr, Iu, dt, y, stash, &rc);
        });
}

// The lane-group mapping as a kernel of its own (its registers hold the
// conductances; the other mappings' register budget stays unchanged): every
// instance of the launch must be eligible.
template <bool GEN, int RPL>
__global__ __launch_bounds__(kLGThreads) void rk4_lg_kernel(WGArgs a)
{
    extern __shared__ double lds_d[];
    const int32_t b = a.order[blockIdx.x];
    const InstDesc d = a.desc[b];
    lg_integrate<GEN, RPL>(a, d, lds_d);
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

#define WGV(BS, NPT) {BS, NPT, false, false, (const void *)rk4_wg_kernel<BS, NPT, false>, 0}
#define WGG(BS, NPT) {BS, NPT, true, false, (const void *)rk4_wg_kernel<BS, NPT, true>, 0}
#define WGR(BS, NPT, S) {BS, NPT, false, false, (const void *)rk4_wg_kernel<BS, NPT, false, S>, S}

static const WGVariant kVariants[] = {
    WGV(64, 1), WGV(128, 1), WGV(128, 2), WGV(256, 1), WGV(256, 2), WGV(256, 4), WGV(512, 1),
    WGG(64, 1), WGG(128, 1), WGG(128, 2), WGG(256, 1), WGG(256, 2), WGG(256, 4), WGG(512, 1),
    WGR(256, 2, 48), WGR(256, 2, 32),
    {kLGThreads, 2, false, true, (const void *)rk4_lg_kernel<false, 2>, 0},
    {kLGThreads, 2, true, true, (const void *)rk4_lg_kernel<true, 2>, 0},
    {0, 0, false, false, nullptr, 0},
};

const WGVariant *wg_variants() { return kVariants; }
const void *init_kernel() { return (const void *)init_state_kernel; }

}  // namespace psst
