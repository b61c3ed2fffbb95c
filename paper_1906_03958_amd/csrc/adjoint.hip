// adjoint.hip -- discrete adjoint of the RK4 map for batches of
// per-instance networks: gradients of a loss of the recorded potentials with
// respect to the synaptic conductances g_ij and the intrinsic g_Na, g_K, g_L.
//
// The paper integrates with RK4 ("Brain simulations as computational graphs")
// but says nothing about gradients; this differentiates the discrete step
// y_{n+1} = y_n + dt/6 (k1 + 2 k2 + 2 k3 + k4) exactly (discretise, then
// differentiate), so the result matches finite differences of the forward
// map.  With lam = dL/dy_{n+1}:
//   kbar_q = dt b_q lam + dt c_{q+1} u_{q+1},  u_q = J(Y_q)^T kbar_q  (q = 3..0)
//   dL/dy_n = lam + u_0 + u_1 + u_2 + u_3 (+ dL/dV_n injected from the loss)
//   dL/dtheta += sum_q (df/dtheta)(Y_q)^T kbar_q.
//
// One workgroup per instance.  The forward trajectory is rebuilt segment by
// segment from checkpoints taken every K steps: the segment's K steps are
// recomputed with the forward kernel's own routines (bitwise the forward
// trajectory) and each step's four stage inputs and synaptic sums are kept in
// a float64 workspace; each reverse step then walks its stages backwards.
// J^T has an elementwise part per neuron and a presynaptic part
// sum_i g_ij q(i) -- a transposed product, four lanes per presynaptic row,
// each summing one residue class of i in index order.  dL/dg_ij = sum over
// steps and stages of q(i) x_j is a contraction over the segment's 4K stage
// records, formed once per segment in float64 (on the float64 matrix cores
// when the LDS allows) and folded into a float32 (value, compensation) pair
// per entry; per-neuron gradients likewise.  A generic explicit method
// (general tableau) runs the same scheme with its own a and b.
#include <cstdlib>
#include <cstring>
#include <mutex>

#include "runtime.h"
#include "wg_common.h"

using namespace psst;

namespace {

struct AdjArgs {
    const InstDesc *desc;
    const float *ckpt;          // [ceil(n_steps / K)][14][nt]
    int32_t K;
    int64_t nt;
    StimDev stim;
    double dt;
    int64_t n_steps, step0;
    const float *dLdV;          // [n_steps][nt]
    double *ws;                 // per-instance workspace, ws_stride doubles each
    int64_t ws_stride;
    float *gacc;                // per-instance compensated pairs, gacc_stride floats each
    int64_t gacc_stride;
    int64_t lds_bytes;
    int32_t *flag;
    Tab tab;                    // method of the generic-step variants
    int32_t mode;               // 0 default, 1 per-step LDS accumulation of dL/dg
    double *adj_state;          // per instance [NVAR][ld]: lam between segment launches
    int64_t adj_stride;
    int64_t seg;                // the segment this launch handles
    int32_t first;              // 1: the first launch of the call (the last segment)
};

// workspace layout of one instance (doubles), ld = padded neuron count
struct WsLayout {
    double *sY;   // [K][4][NVAR][ld] stage inputs of every step of the segment
    double *sS;   // [K][4][3][ld]    their synaptic sums (nS)
    double *Qs;   // [4K][3][ld]      q of each (step, stage)
    double *Xs;   // [4K][2][ld]      activations x_s (all rows), x_B (LN rows)
};

__host__ __device__ inline int64_t ws_doubles(int ld, int K)
{
    return (int64_t)ld * K * (4LL * NVAR + 12 + 12 + 8);
}

__device__ inline WsLayout ws_layout(double *base, int ld, int K)
{
    WsLayout w;
    w.sY = base;
    w.sS = w.sY + 4LL * NVAR * K * ld;
    w.Qs = w.sS + 12LL * K * ld;
    w.Xs = w.Qs + 12LL * K * ld;
    return w;
}

// gradient accumulators of one instance: three sections of float32 pairs
// (value plane then compensation plane): fast [n][ld], slow [n_ln][ld],
// per-neuron [3][ld]
__host__ __device__ inline int64_t gacc_floats(int n, int n_ln, int ld)
{
    return 2LL * ((int64_t)n * ld + (int64_t)n_ln * ld + 3LL * ld);
}

__device__ inline void comp_add(float *hi, float *lo, double v)
{
    const double s = (double)*hi + (double)*lo + v;
    float h, l;
    split_store(s, h, l);
    *hi = h;
    *lo = l;
}

// sum_i row[i] q[i] over i < n: four interleaved partial sums (i mod 4),
// each in index order, added as (s0 + s1) + (s2 + s3); row holds ld >= n
// floats, zero padded, and q is finite up to ld.
template <typename V4>
__device__ __forceinline__ double row_dot(V4 *row, const double *q, int n)
{
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    const int n4 = (n + 3) >> 2;
#pragma unroll 4
    for (int k = 0; k < n4; ++k) {
        const v4f g = row[k];
        const int i0 = 4 * k;
        s0 = fma((double)g.x, q[i0], s0);
        s1 = fma((double)g.y, q[i0 + 1], s1);
        s2 = fma((double)g.z, q[i0 + 2], s2);
        s3 = fma((double)g.w, q[i0 + 3], s3);
    }
    return (s0 + s1) + (s2 + s3);
}

typedef double dbl4 __attribute__((ext_vector_type(4)));

// dL/dg of one segment on the matrix cores: for each synapse class the
// product X^T Q over the segment's T stage records (rows j presynaptic,
// columns i postsynaptic; x_j and q(i) as stashed by the reverse sweep), added
// to the compensated accumulators.  Records go through LDS TT at a time; a
// wavefront owns a strip of one 16-row tile by kStripTiles 16-column tiles
// (v_mfma_f64_16x16x4f64: A lane l = X[row l%16][rec l/16], B lane l =
// Q[rec l/16][col l%16], D lane l item r = [row 4r + l/16][col l%16]).
constexpr int kStripTiles = 4;     // 16-column tiles per wavefront strip
template <int BS>
__device__ void contract_mma(const WsLayout &W, int T, int n, int n_pn, int n_ln, bool gabab,
                             int ld, double *lds, int64_t room, float *gacc, int64_t half,
                             int64_t sec_f)
{
    constexpr int NW = BS / 64;
    constexpr int SPW = BS >= 512 ? 2 : 4;     // strips per wavefront and pass
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int rt0 = (n_pn + 15) / 16, rt1 = (n_ln + 15) / 16, rt2 = gabab ? rt1 : 0;
    const int CT = (n + 15) / 16;
    const int CS = (CT + kStripTiles - 1) / kStripTiles;
    const int strips = (rt0 + rt1 + rt2) * CS;
    int TT = (int)(room / (5LL * ld)) & ~3;
    TT = TT > 64 ? 64 : TT;
    // explicit address spaces: global loads may then pass LDS stores
    typedef double d2v __attribute__((ext_vector_type(2)));
    typedef __attribute__((address_space(1))) const d2v gdbl2;
    typedef __attribute__((address_space(3))) d2v ldbl2;
    typedef __attribute__((address_space(3))) const double ldbl;
    ldbl *sx = (ldbl *)lds;                          // [TT][2][ld]
    ldbl *sq = (ldbl *)(lds + (int64_t)TT * 2 * ld);   // [TT][3][ld]
    // each pass over the records serves NW * SPW strips: a wavefront keeps the
    // accumulators of SPW strips, so a record block is staged once per pass
    for (int g0 = 0; g0 < strips; g0 += NW * SPW) {
        int ty[SPW], trow[SPW], c0[SPW];
        bool act[SPW];
        dbl4 acc[SPW][kStripTiles];
#pragma unroll
        for (int sp = 0; sp < SPW; ++sp) {
            const int sidx = g0 + sp * NW + wave;
            act[sp] = sidx < strips;
            ty[sp] = 0;
            trow[sp] = 0;
            c0[sp] = 0;
            if (act[sp]) {
                const int rt = sidx / CS;
                c0[sp] = (sidx % CS) * kStripTiles;
                if (rt < rt0) {
                    trow[sp] = rt * 16;
                } else if (rt < rt0 + rt1) {
                    ty[sp] = 1;
                    trow[sp] = n_pn + (rt - rt0) * 16;
                } else {
                    ty[sp] = 2;
                    trow[sp] = (rt - rt0 - rt1) * 16;
                }
            }
#pragma unroll
            for (int c = 0; c < kStripTiles; ++c) acc[sp][c] = dbl4{0.0, 0.0, 0.0, 0.0};
        }
        for (int t0 = 0; t0 < T; t0 += TT) {
            const int tn = T - t0 < TT ? T - t0 : TT;
            __syncthreads();                   // previous block consumed
            // stage records t0 .. t0 + tn - 1: the x and q blocks of these
            // records are contiguous in the workspace and in LDS, so this is a
            // flat copy with SU loads in flight per thread.  Entries never
            // written (columns past n, slow x past n_ln) are copied too but
            // never used: the operand reads below mask them.
            {
                constexpr int SU = 8;
                const int nx2 = tn * ld;                 // double2 of the x block
                const int ntot = nx2 + tn * 3 * ld / 2;  // plus the q block
                gdbl2 *gx = (gdbl2 *)(W.Xs + (int64_t)t0 * 2 * ld);
                gdbl2 *gq = (gdbl2 *)(W.Qs + (int64_t)t0 * 3 * ld);
                ldbl2 *lx = (ldbl2 *)lds;
                ldbl2 *lq = (ldbl2 *)(lds + (int64_t)TT * 2 * ld);
                // indices past the block are clamped to its last pair: those
                // lanes load and store that pair's own value again, so every
                // access is in bounds and no branch keeps a load from issuing
                for (int e0 = tid; e0 < ntot; e0 += SU * BS) {
                    d2v v[SU];
#pragma unroll
                    for (int u = 0; u < SU; ++u) {
                        const int e = e0 + u * BS < ntot ? e0 + u * BS : ntot - 1;
                        v[u] = e < nx2 ? gx[e] : gq[e - nx2];
                    }
#pragma unroll
                    for (int u = 0; u < SU; ++u) {
                        const int e = e0 + u * BS < ntot ? e0 + u * BS : ntot - 1;
                        ldbl2 *dst = e < nx2 ? lx + e : lq + (e - nx2);
                        *dst = v[u];
                    }
                }
            }
            __syncthreads();
            // T = 4 L, so every block holds whole groups of four records
#pragma unroll
            for (int sp = 0; sp < SPW; ++sp) {
                if (!act[sp]) continue;
                const int row = trow[sp] + (lane & 15);
                const int row_end = ty[sp] == 0 ? n_pn : (ty[sp] == 1 ? n : n_ln);
                const int xs = ty[sp] == 2 ? 1 : 0;
                for (int k0 = 0; k0 < tn; k0 += 4) {
                    const int rk = k0 + (lane >> 4);
                    const double av = row < row_end ? sx[(rk * 2 + xs) * ld + row] : 0.0;
#pragma unroll
                    for (int c = 0; c < kStripTiles; ++c) {
                        const int col = (c0[sp] + c) * 16 + (lane & 15);
                        const double bv = col < n ? sq[(rk * 3 + ty[sp]) * ld + col] : 0.0;
                        acc[sp][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[sp][c], 0, 0, 0);
                    }
                }
            }
        }
#pragma unroll
        for (int sp = 0; sp < SPW; ++sp) {
            if (!act[sp]) continue;
            const int row_end = ty[sp] == 0 ? n_pn : (ty[sp] == 1 ? n : n_ln);
#pragma unroll
            for (int c = 0; c < kStripTiles; ++c) {
                const int col = (c0[sp] + c) * 16 + (lane & 15);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = trow[sp] + 4 * r + (lane >> 4);
                    if (row < row_end && col < n) {
                        const int64_t e = (ty[sp] == 2 ? sec_f : 0) + (int64_t)row * ld + col;
                        comp_add(gacc + e, gacc + half + e, acc[sp][c][r]);
                    }
                }
                // one tile at a time: keeps the scheduler from hoisting every
                // tile's accumulator loads (and their addresses) at once
                __asm__ volatile("" ::: "memory");
            }
        }
    }
}

// One residue class of row_dot, for four lanes sharing a row: lane k of the
// group sums row[i] q[i] over i = k, k + 4, ... below 4 ceil(n / 4) in index
// order; the group then forms (s0 + s1) + (s2 + s3), so the result equals
// row_dot's bit for bit.  Every lane of the wavefront must call (shuffles).
template <typename F>
__device__ __forceinline__ double row_dot_quad(F *row, const double *q, int n, int k, bool on)
{
    typedef __attribute__((address_space(3))) const double lds_dbl;
    lds_dbl *Q = (lds_dbl *)q;
    double s = 0.0;
    if (on) {
        const int n4 = (n + 3) >> 2;
        int m = 0;
        for (; m + 8 <= n4; m += 8) {
            float g[8];
            double x[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) g[u] = row[4 * (m + u) + k];
#pragma unroll
            for (int u = 0; u < 8; ++u) x[u] = Q[4 * (m + u) + k];
#pragma unroll
            for (int u = 0; u < 8; ++u) s = fma((double)g[u], x[u], s);
        }
        for (; m < n4; ++m) s = fma((double)row[4 * m + k], Q[4 * m + k], s);
    }
    const double p = s + __shfl_xor(s, 1);       // s0 + s1 on lanes 0, 1; s2 + s3 on 2, 3
    return p + __shfl_xor(p, 2);
}

// How one instance's reverse sweep uses the LDS: lacc -- the step's stage
// records and the dL/dg accumulator as float32 (value, compensation) planes in
// LDS, updated every step (only when asked for, PSST_ADJ_MODE=lacc, and when
// it fits); otherwise the records go to the workspace for the segment's
// contraction kernel.  staged -- one step's stage data (40 doubles per
// neuron) staged through LDS: when the whole conductance matrix still fits
// beside it, or, when the matrix does not fit anyway, when the staging takes
// at most half of the LDS.
struct AdjModes {
    bool lacc, staged;
    int rows;                   // presynaptic rows of the conductance matrices
};

__device__ inline AdjModes adj_modes(const InstDesc &d, int64_t lds_bytes, int mode)
{
    const int n = d.n, ld = d.ld, n_ln = d.n - d.n_pn;
    const bool gb_net = (d.flags & DESC_GABAB) != 0;
    AdjModes m;
    m.rows = (d.flags & DESC_NOSYN) ? 0 : n + (gb_net ? n_ln : 0);
    const Chunks ch0 = chunks_of(n, d.n_pn, gb_net);
    const int nch = ch0.na + ch0.ng + ch0.nb;
    const int64_t fwd_min = (int64_t)sizeof(double) * (2 + nch) * ld;
    const int64_t lacc_bytes = (int64_t)sizeof(double) * (5 + 20) * ld +
                               (int64_t)sizeof(float) * 2 * m.rows * ld;
    const int64_t res_bytes = (int64_t)sizeof(float) * nch * CW * ld;
    const int64_t base5 = (int64_t)sizeof(double) * 5 * ld;
    const int64_t stage_b = (int64_t)sizeof(double) * 40 * ld;
    m.lacc = mode == 1 && m.rows > 0 && lacc_bytes + fwd_min <= lds_bytes;
    const bool res_fits = base5 + fwd_min + res_bytes <= lds_bytes;
    m.staged = !m.lacc && (res_fits ? base5 + stage_b + fwd_min + res_bytes <= lds_bytes
                                    : 2 * (base5 + stage_b) <= lds_bytes);
    return m;
}

// The reverse sweep over one segment (a.seg) of every instance, one
// workgroup per instance: the stage inputs and synaptic sums of the
// segment's steps are in the workspace (written by the forward kernels'
// recomputation); lam and the per-neuron gradient partials carry over from
// the previous launch through adj_state.  Per step, stages last to first:
// the elementwise VJP, the presynaptic term sum_i g_ij q(i) (four lanes per
// presynaptic row, each summing one residue class of i in index order), and
// lam <- lam + sum_q u_q + dL/dV.  The q and x vectors of every (step, stage)
// go to the workspace for the contraction kernel (or, lacc, into the LDS
// accumulator).
template <int BS, bool GEN>
__global__ __launch_bounds__(BS) void adjoint_reverse_kernel(AdjArgs a)
{
    constexpr int NPT = 1;
    extern __shared__ double lds_d[];
    const int b = blockIdx.x;
    const InstDesc d = a.desc[b];
    const int n = d.n, n_pn = d.n_pn, ld = d.ld, n_ln = d.n - d.n_pn;
    const int tid = threadIdx.x;
    // LDS: q vectors [3][ld] and transposed products [2][ld]; then, lacc, the
    // step's four stage records [4][5][ld] and the gradient accumulator
    // [2][rows][ld] float32, or a staging area for one step's stage data
    // [40][ld]; then the conductance view with as many columns as remain.
    const AdjModes md = adj_modes(d, a.lds_bytes, a.mode);
    const bool lacc = md.lacc, staged = md.staged;
    const int rows = md.rows;
    const int64_t lacc_bytes = (int64_t)sizeof(double) * (5 + 20) * ld +
                               (int64_t)sizeof(float) * 2 * rows * ld;
    double *qb = lds_d;
    double *tb = lds_d + 3 * ld;
    double *recs = lds_d + 5 * ld;                         // lacc: [4][5][ld]
    float *gls = reinterpret_cast<float *>(lds_d + 25 * ld);  // lacc: [2][rows][ld]
    const int64_t stage_d = 40LL * ld;
    double *stg = lds_d + 5 * ld;
    const int64_t used_b = lacc ? lacc_bytes
                                : (int64_t)sizeof(double) * (5 * ld + (staged ? stage_d : 0));
    const WGSyn w = wg_setup<BS>(d, lds_d + used_b / sizeof(double), a.lds_bytes - used_b);
    const bool gabab = w.gabab;
    const Kin K = load_kin(d.kin);
    const double dt = a.dt;
    const int64_t NT = a.nt;
    const int KK = a.K;
    const WsLayout W = ws_layout(a.ws + (int64_t)b * a.ws_stride, ld, KK);
    float *gacc = a.gacc + (int64_t)b * a.gacc_stride;
    const int64_t sec_f = (int64_t)n * ld, sec_b = (int64_t)n_ln * ld, sec_p = 3LL * ld;
    const int64_t half = sec_f + sec_b + sec_p;     // value plane size
    double *ast = a.adj_state + (int64_t)b * a.adj_stride;
    if (a.first)
        for (int64_t e = tid; e < 2 * half; e += BS) gacc[e] = 0.f;
    for (int e = tid; e < 3 * ld; e += BS) qb[e] = 0.0;   // padding entries stay 0
    if (lacc) {
        for (int e = tid; e < 20 * ld; e += BS) recs[e] = 0.0;
        // the accumulator continues from the previous launch's
        for (int64_t e = tid; e < (int64_t)rows * ld; e += BS) {
            gls[e] = a.first ? 0.f : gacc[e];
            gls[(int64_t)rows * ld + e] = a.first ? 0.f : gacc[half + e];
        }
    }
    __syncthreads();
    const int i = tid;                               // the thread's neuron (NPT = 1)
    const bool own = i < n;
    const int ic = own ? i : 0;
    const int64_t gi = d.off + ic;
    const bool is_ln = ic >= n_pn;
    float pr[NPT][NPRM];
#pragma unroll
    for (int p = 0; p < NPRM; ++p) pr[0][p] = d.prm[p * ld + ic];
    const Prm P = prm_of(pr[0]);

    double lam[NVAR];
    double pg[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int v = 0; v < NVAR; ++v) lam[v] = (a.first || !own) ? 0.0 : ast[(int64_t)v * ld + i];
    const double bq[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
    const double cq[4] = {0.0, 0.5, 0.5, 1.0};

    const int64_t seg = a.seg;
    const int64_t s0 = seg * KK;
    const int L = (int)((a.n_steps - s0) < KK ? (a.n_steps - s0) : KK);
    // ---- reverse steps
    for (int s = L - 1; s >= 0; --s) {
        const int64_t ls = s0 + s;                 // local step index
        if (own) lam[YV] += (double)a.dLdV[ls * NT + gi];
        const double *sYs = W.sY + (int64_t)s * 4 * NVAR * ld;
        const double *sSs = W.sS + (int64_t)s * 12 * ld;
        if (staged) {
            // each thread moves its own neuron's 40 values (the same
            // thread reads them back, so no barrier is needed)
            if (own) {
                double tmp[40];
#pragma unroll
                for (int e = 0; e < 28; ++e) tmp[e] = sYs[(int64_t)e * ld + i];
#pragma unroll
                for (int e = 0; e < 12; ++e) tmp[28 + e] = sSs[(int64_t)e * ld + i];
#pragma unroll
                for (int e = 0; e < 40; ++e) stg[(int64_t)e * ld + i] = tmp[e];
            }
            sYs = stg;
            sSs = stg + 28 * ld;
        }
        double un[NVAR], usum[NVAR];
        double uh[GEN ? 4 : 1][NVAR];      // generic method: u of the later stages
        constexpr int kStageUnroll = GEN ? 4 : 1;
#pragma unroll
        for (int v = 0; v < NVAR; ++v) {
            un[v] = 0.0;
            usum[v] = 0.0;
        }
        // classical RK4: kbar_q = dt b_q lam + dt c_{q+1} u_{q+1}; a generic
        // tableau: kbar_q = dt b_q lam + dt sum_{r>q} a_rq u_r (stages last
        // to first, unrolled so the u_r stay in registers)
#pragma unroll kStageUnroll
        for (int q = 3; q >= 0; --q) {
            if (GEN && q >= a.tab.s) {
                // a stage the method lacks: its records enter the segment
                // contraction as zeros (the workspace keeps older contents)
                if (!lacc && own) {
                    const int64_t rz = (ls - s0) * 4 + q;
#pragma unroll
                    for (int t = 0; t < 3; ++t) W.Qs[(rz * 3 + t) * ld + i] = 0.0;
                    W.Xs[(rz * 2 + 0) * ld + i] = 0.0;
                    if (gabab && is_ln) W.Xs[(rz * 2 + 1) * ld + (i - n_pn)] = 0.0;
                }
                continue;
            }
            double Yq[NVAR], kb[NVAR], u[NVAR], qq[3], dg[3];
#pragma unroll
            for (int v = 0; v < NVAR; ++v) {
                Yq[v] = own ? sYs[(q * NVAR + v) * ld + i] : 0.0;
                if constexpr (GEN) {
                    double t = dt * a.tab.b[q] * lam[v];
#pragma unroll
                    for (int r = q + 1; r < 4; ++r)
                        if (r < a.tab.s) t += dt * a.tab.a[r][q] * uh[r][v];
                    kb[v] = t;
                } else {
                    kb[v] = dt * bq[q] * lam[v] + (q < 3 ? dt * cq[q + 1] * un[v] : 0.0);
                }
            }
            if (!own) Yq[YM] = Yq[YH] = Yq[YN] = 0.5;   // keep idle lanes finite
            const double sa = own ? sSs[(q * 3 + 0) * ld + i] : 0.0;
            const double sg = own ? sSs[(q * 3 + 1) * ld + i] : 0.0;
            const double sbv = own ? sSs[(q * 3 + 2) * ld + i] : 0.0;
            hh_vjp(Yq, P, K, d.cg, d.cg * sa, d.cg * sg, d.cg * sbv, kb, is_ln, gabab, u, qq,
                   dg);
            const int64_t rec = ls - s0;           // stage record within the segment
            double *qv0 = lacc ? recs + q * 5 * ld : qb;  // this stage's q vectors
            if (own) {
                pg[0] += dg[0];
                pg[1] += dg[1];
                pg[2] += dg[2];
#pragma unroll
                for (int t = 0; t < 3; ++t) qv0[t * ld + i] = qq[t];
                if (lacc) {
                    recs[(q * 5 + 3) * ld + i] = Yq[YS];
                    if (gabab && is_ln) recs[(q * 5 + 4) * ld + (i - n_pn)] = gabab_act(Yq[YG], K);
                } else {
#pragma unroll
                    for (int t = 0; t < 3; ++t) W.Qs[((rec * 4 + q) * 3 + t) * ld + i] = qq[t];
                    W.Xs[((rec * 4 + q) * 2 + 0) * ld + i] = Yq[YS];
                    if (gabab && is_ln)
                        W.Xs[((rec * 4 + q) * 2 + 1) * ld + (i - n_pn)] = gabab_act(Yq[YG], K);
                }
            }
            __syncthreads();
            // presynaptic terms: t_j = sum_i g_ij q_type(j)(i), four lanes per
            // presynaptic row j (row j of the transposed matrix is contiguous)
            for (int r0 = 0; r0 < rows; r0 += BS / 4) {
                const int r = r0 + (tid >> 2);
                const bool on = r < rows;
                const int rr = on ? r : 0;
                const bool slow = rr >= n;
                const int jr = slow ? rr - n : rr;
                const double *qv = qv0 + (slow ? 2 : (jr < n_pn ? 0 : 1)) * ld;
                double acc;
                // rows of the transposed matrix: from LDS when the dense
                // layout is resident there, else from global memory (also
                // for sparse storage, whose LDS holds the forward's rows)
                if (w.R >= CW && !w.sparse)
                    acc = row_dot_quad((lds_float *)lds_row(w, slow ? 1 : 0, jr), qv, n,
                                       tid & 3, on);
                else
                    acc = row_dot_quad((global_float *)((slow ? d.gtb : d.gt) + (int64_t)jr * ld),
                                       qv, n, tid & 3, on);
                if (on && (tid & 3) == 0) tb[(slow ? ld : 0) + jr] = acc;
            }
            __syncthreads();
            if (own && rows > 0) {
                u[YS] += tb[i];
                if (gabab && is_ln) u[YG] += tb[ld + (i - n_pn)] * gabab_act_d(Yq[YG], K);
            }
#pragma unroll
            for (int v = 0; v < NVAR; ++v) {
                un[v] = u[v];
                if constexpr (GEN) uh[q][v] = u[v];
                usum[v] += u[v];
            }
        }
#pragma unroll
        for (int v = 0; v < NVAR; ++v) lam[v] += usum[v];
        if (lacc) {
            // dL/dg_ij += sum over this step's stages of q(i) x_j: float64
            // sum of the four products, then one compensated add per entry
            __syncthreads();
            const int q4 = ld >> 2;
            const int RG = BS / q4;
            const int i4 = tid % q4, rg = tid / q4;
            if (rg < RG) {
                int cur_t = -1;
                double qv[4][4];
                for (int r = rg; r < rows; r += RG) {
                    const bool slow = r >= n;
                    const int j = slow ? r - n : r;
                    const int t = slow ? 2 : (j < n_pn ? 0 : 1);
                    if (t != cur_t) {
                        cur_t = t;
#pragma unroll
                        for (int q = 0; q < 4; ++q)
#pragma unroll
                            for (int c = 0; c < 4; ++c) qv[q][c] = recs[(q * 5 + t) * ld + 4 * i4 + c];
                    }
                    double v[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const double x = recs[(q * 5 + (slow ? 4 : 3)) * ld + j];
#pragma unroll
                        for (int c = 0; c < 4; ++c) v[c] = fma(qv[q][c], x, v[c]);
                    }
                    float *hp = gls + (int64_t)r * ld + 4 * i4;
                    float *lp = gls + (int64_t)(rows + r) * ld + 4 * i4;
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        float h, l;
                        split_store((double)hp[c] + (double)lp[c] + v[c], h, l);
                        hp[c] = h;
                        lp[c] = l;
                    }
                }
            }
            __syncthreads();
        }
    }
    // the per-neuron gradients of the segment into their accumulators
    if (own) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int64_t e = sec_f + sec_b + (int64_t)k * ld + i;
            comp_add(gacc + e, gacc + half + e, pg[k]);
        }
    }
    if (lacc) {
        __syncthreads();
        // value plane -> gacc[0 .. rows*ld), compensation plane -> gacc[half ..]
        for (int64_t e = tid; e < (int64_t)rows * ld; e += BS) {
            gacc[e] = gls[e];
            gacc[half + e] = gls[(int64_t)rows * ld + e];
        }
    }
    if (own) {
#pragma unroll
        for (int v = 0; v < NVAR; ++v) ast[(int64_t)v * ld + i] = lam[v];
    }
    if (seg == 0) {
        double chk = 0.0;
#pragma unroll
        for (int v = 0; v < NVAR; ++v) chk += lam[v];
        if (own && !finite_d(chk)) atomicOr(a.flag, 1);
    }
}

// dL/dg over one segment (a.seg) of every instance: for each synapse class
// the product X^T Q over the segment's 4L stage records on the float64
// matrix cores, added to the compensated accumulators (instances whose
// reverse sweep accumulated in LDS, and networks without synapses, have
// nothing to add).
template <int BS>
__global__ __launch_bounds__(BS) void adjoint_contract_kernel(AdjArgs a)
{
    extern __shared__ double lds_d[];
    const int b = blockIdx.x;
    const InstDesc d = a.desc[b];
    const AdjModes md = adj_modes(d, a.lds_bytes, a.mode);
    if (md.lacc || md.rows == 0) return;
    const int n = d.n, n_pn = d.n_pn, ld = d.ld, n_ln = d.n - d.n_pn;
    const bool gabab = (d.flags & DESC_GABAB) != 0;
    const int KK = a.K;
    const WsLayout W = ws_layout(a.ws + (int64_t)b * a.ws_stride, ld, KK);
    float *gacc = a.gacc + (int64_t)b * a.gacc_stride;
    const int64_t sec_f = (int64_t)n * ld, sec_b = (int64_t)n_ln * ld;
    const int64_t half = sec_f + sec_b + 3LL * ld;
    const int64_t s0 = a.seg * KK;
    const int L = (int)((a.n_steps - s0) < KK ? (a.n_steps - s0) : KK);
    contract_mma<BS>(W, 4 * L, n, n_pn, n_ln, gabab, ld, lds_d,
                     a.lds_bytes / (int64_t)sizeof(double), gacc, half, sec_f);
}

// Scatter the accumulators into the caller's layout: per instance (grid.x =
// instance) or summed over instances in instance order (grid.x = 1).
struct FinArgs {
    const InstDesc *desc;
    int32_t n_inst;
    const float *gacc;
    int64_t gacc_stride;
    const int64_t *goff;        // per instance offset into grad_g (per-instance mode)
    float *grad_g, *gna, *gk, *gl;
    int32_t per_instance;
};

__global__ __launch_bounds__(256) void adjoint_finalize(FinArgs f)
{
    const int b0 = f.per_instance ? blockIdx.x : 0;
    const int nb = f.per_instance ? 1 : f.n_inst;
    const InstDesc d = f.desc[b0];
    const int n = d.n, ld = d.ld, n_ln = d.n - d.n_pn;
    const int64_t sec_f = (int64_t)n * ld, sec_b = (int64_t)n_ln * ld;
    const int64_t half = sec_f + sec_b + 3LL * ld;
    auto total = [&](int64_t e) {
        double s = 0.0;
        for (int b = b0; b < b0 + nb; ++b) {
            const float *g = f.gacc + (int64_t)b * f.gacc_stride;
            s += (double)g[e] + (double)g[half + e];
        }
        return (float)s;
    };
    float *out = f.grad_g + (f.per_instance ? f.goff[b0] : 0);
    for (int p = 0; p < d.n_paths; ++p) {
        const int64_t *pi = d.paths + 6 * p;
        const int type = (int)pi[0], pre0 = (int)pi[1], pre1 = (int)pi[2];
        const int post0 = (int)pi[3], post1 = (int)pi[4];
        const int64_t go = pi[5];
        const int npre = pre1 - pre0;
        const int64_t cnt = (int64_t)(post1 - post0) * npre;
        for (int64_t e = threadIdx.x; e < cnt; e += blockDim.x) {
            const int ii = post0 + (int)(e / npre), j = pre0 + (int)(e % npre);
            const int64_t slot = type == T_GABA_B ? sec_f + (int64_t)(j - d.n_pn) * ld + ii
                                                  : (int64_t)j * ld + ii;
            out[go + e] = d.maskt[slot] ? total(slot) : 0.f;
        }
    }
    const int64_t noff = f.per_instance ? d.off : 0;
    for (int ii = threadIdx.x; ii < n; ii += blockDim.x) {
        f.gna[noff + ii] = total(sec_f + sec_b + 0LL * ld + ii);
        f.gk[noff + ii] = total(sec_f + sec_b + 1LL * ld + ii);
        f.gl[noff + ii] = total(sec_f + sec_b + 2LL * ld + ii);
    }
}

}  // namespace

// ---------------------------------------------------------------------------

struct AdjWork {
    double *ws = nullptr;
    size_t ws_bytes = 0;
    double *ws2 = nullptr;          // second stage-record buffer (pipelined calls)
    size_t ws2_bytes = 0;
    float *gacc = nullptr;
    size_t gacc_bytes = 0;
    int64_t *goff = nullptr;
    double *astate = nullptr;
    size_t astate_bytes = 0;
    // pipelined calls: the recomputation's stream and the events that order
    // it against the caller's stream
    hipStream_t aux = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    hipEvent_t ev_rec[2] = {nullptr, nullptr}, ev_con[2] = {nullptr, nullptr};
};

static psst_status ensure(void **p, size_t *have, size_t need)
{
    if (*have >= need) return PSST_OK;
    (void)hipFree(*p);
    *p = nullptr;
    *have = 0;
    HIPCHK(hipMalloc(p, need));
    *have = need;
    return PSST_OK;
}

static const void *adj_fn(int bs, bool gen)
{
    switch (bs) {
    case 64: return gen ? (const void *)adjoint_reverse_kernel<64, true> : (const void *)adjoint_reverse_kernel<64, false>;
    case 128: return gen ? (const void *)adjoint_reverse_kernel<128, true> : (const void *)adjoint_reverse_kernel<128, false>;
    case 256: return gen ? (const void *)adjoint_reverse_kernel<256, true> : (const void *)adjoint_reverse_kernel<256, false>;
    case 512: return gen ? (const void *)adjoint_reverse_kernel<512, true> : (const void *)adjoint_reverse_kernel<512, false>;
    }
    return nullptr;
}

static const void *contract_fn(int bs)
{
    switch (bs) {
    case 64: return (const void *)adjoint_contract_kernel<64>;
    case 128: return (const void *)adjoint_contract_kernel<128>;
    case 256: return (const void *)adjoint_contract_kernel<256>;
    case 512: return (const void *)adjoint_contract_kernel<512>;
    }
    return nullptr;
}

// Exclusive prefix sum of the instances' gradient-block sizes: goff[b] =
// offset of instance b's blocks in a per-instance grad_g (one workgroup).
__global__ __launch_bounds__(256) void grad_offsets_kernel(const InstDesc *desc, int32_t n,
                                                           int64_t *goff)
{
    __shared__ int64_t part[256];
    const int t = threadIdx.x;
    const int per = (n + 255) / 256;
    const int b0 = min(n, t * per), b1 = min(n, b0 + per);
    int64_t s = 0;
    for (int b = b0; b < b1; ++b) s += desc[b].grad_entries;
    part[t] = s;
    __syncthreads();
    if (t == 0) {
        int64_t run = 0;
        for (int k = 0; k < 256; ++k) {
            const int64_t v = part[k];
            part[k] = run;
            run += v;
        }
    }
    __syncthreads();
    int64_t run = part[t];
    for (int b = b0; b < b1; ++b) {
        goff[b] = run;
        run += desc[b].grad_entries;
    }
}

// Zero fill (the accumulators of a call with no steps).
__global__ __launch_bounds__(256) void fill_zero_kernel(float *p, int64_t count)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
         e += (int64_t)gridDim.x * blockDim.x)
        p[e] = 0.f;
}

// Launch shape, LDS and workspace strides of one adjoint call.
struct AdjPlan {
    int bs = 0;
    size_t lds = 0;
    int64_t wstride = 0;     // doubles of stage records per instance
    int64_t gstride = 0;     // floats of gradient accumulators per instance
    int64_t astride = 0;     // doubles of carried adjoint state per instance
    const void *fn = nullptr;
    const void *fn_con = nullptr;
};

static psst_status adjoint_plan(const std::vector<psst_network *> &nets, int32_t K,
                                size_t lds_max, bool gen, AdjPlan *p)
{
    int max_n = 0, max_ld = 0;
    int64_t gstride = 0;
    for (auto *q : nets) {
        max_n = std::max(max_n, q->n);
        max_ld = std::max(max_ld, q->ld);
        gstride = std::max(gstride, gacc_floats(q->n, q->n - q->n_pn, q->ld));
    }
    if (max_n > 512)
        return fail(PSST_ERR_UNSUPPORTED, "the adjoint takes networks of at most 512 neurons");
    // 256 threads even for small networks: the spare threads shorten the
    // synaptic products and the gradient update (measured 10 % faster at 120)
    int bs = max_n <= 256 ? 256 : 512;
    if (const char *e = std::getenv("PSST_ADJ_BS")) {     // launch-shape override
        const int v = std::atoi(e);
        if (adj_fn(v, gen) && v >= max_n) bs = v;
    }
    if (4 * bs < max_ld) return fail(PSST_ERR_UNSUPPORTED, "no adjoint launch shape for n=%d", max_n);
    // LDS: q and product vectors, the forward view, and G when it fits
    size_t need = 0;
    for (auto *q : nets) {
        const size_t base = sizeof(double) * 5 * q->ld + wg_lds_bytes(false, q->ld, q->nch, 0);
        need = std::max(need, base);
    }
    if (need > lds_max) return fail(PSST_ERR_UNSUPPORTED, "adjoint LDS buffers exceed the LDS");
    p->bs = bs;
    p->lds = lds_max;     // the rest holds conductance columns
    p->wstride = ws_doubles(max_ld, K);
    p->gstride = gstride;
    p->astride = (int64_t)NVAR * max_ld;
    p->fn = adj_fn(bs, gen);
    p->fn_con = contract_fn(bs);
    return PSST_OK;
}

// The adjoint of one call, all on stream: per segment, last to first, the
// forward kernels' recomputation of the segment (stage records into ws),
// the reverse sweep over it and the contraction of its records into the
// accumulators; then the finalize kernel.  Without steps the accumulators
// are zeroed.  ws, gacc, goff (per-instance gradient offsets) and astate
// (carried lam) are device buffers sized by the plan.
static psst_status adjoint_launch(const AdjPlan &P, int32_t n, const InstDesc *d_desc, int64_t nt,
                                  double *ws, float *gacc, const int64_t *goff, double *astate,
                                  const RecomputeFn &recompute, const float *ckpt, int32_t K,
                                  const psst_stimulus *stim, float dt, int64_t n_steps,
                                  int64_t step0, const float *dLdV, float *grad_g, float *gna,
                                  float *gk, float *gl, int32_t per_instance, int32_t *flag,
                                  const Tab &tab, hipStream_t st)
{
    if (P.lds > 65536) {
        HIPCHK(hipFuncSetAttribute(P.fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)P.lds));
        HIPCHK(hipFuncSetAttribute(P.fn_con, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)P.lds));
    }
    AdjArgs a{};
    a.desc = d_desc;
    a.ckpt = ckpt;
    a.K = K;
    a.nt = nt;
    if (stim) {
        a.stim.i_const = stim->i_const_nA;
        a.stim.pulse_ptr = stim->pulse_ptr;
        a.stim.on_step = stim->on_step;
        a.stim.off_step = stim->off_step;
        a.stim.amp = stim->amp_nA;
    }
    a.dt = (double)dt;
    a.n_steps = n_steps;
    a.step0 = step0;
    a.dLdV = dLdV;
    a.ws = ws;
    a.ws_stride = P.wstride;
    a.gacc = gacc;
    a.gacc_stride = P.gstride;
    a.lds_bytes = (int64_t)P.lds;
    a.flag = flag;
    a.tab = tab;
    a.adj_state = astate;
    a.adj_stride = P.astride;
    // PSST_ADJ_MODE=lacc keeps dL/dg in the per-step LDS accumulator where it
    // fits (comparison runs)
    if (const char *e = std::getenv("PSST_ADJ_MODE")) a.mode = std::strcmp(e, "lacc") == 0 ? 1 : 0;
    if (n_steps > 0) {
        const int64_t nseg = (n_steps + K - 1) / K;
        for (int64_t seg = nseg - 1; seg >= 0; --seg) {
            const int64_t s0 = seg * K;
            const int64_t L = std::min<int64_t>(K, n_steps - s0);
            psst_status s = recompute(ckpt + seg * 14 * nt, step0 + s0, L, ws, P.wstride, K, st);
            if (s != PSST_OK) return s;
            a.seg = seg;
            a.first = seg == nseg - 1;
            void *args[] = {&a};
            HIPCHK(hipLaunchKernel(P.fn, dim3(n), dim3(P.bs), args, P.lds, st));
            HIPCHK(hipLaunchKernel(P.fn_con, dim3(n), dim3(P.bs), args, P.lds, st));
        }
    } else {
        const int64_t cnt = P.gstride * n;
        const unsigned blocks = (unsigned)std::min<int64_t>((cnt + 255) / 256, 4096);
        fill_zero_kernel<<<dim3(blocks > 0 ? blocks : 1), dim3(256), 0, st>>>(gacc, cnt);
        HIPCHK(hipGetLastError());
    }
    FinArgs f{};
    f.desc = d_desc;
    f.n_inst = n;
    f.gacc = gacc;
    f.gacc_stride = P.gstride;
    f.goff = goff;
    f.grad_g = grad_g;
    f.gna = gna;
    f.gk = gk;
    f.gl = gl;
    f.per_instance = per_instance;
    void *fargs[] = {&f};
    HIPCHK(hipLaunchKernel((const void *)adjoint_finalize, dim3(per_instance ? n : 1), dim3(256),
                           fargs, 0, st));
    return PSST_OK;
}

// The same call with segment s - 1's recomputation (on the work's own
// stream, from the lean recomputation: a launch that needs little LDS) beside
// segment s's reverse sweep (on the caller's stream, with the LDS the
// recomputation leaves): stage records alternate between two workspaces by
// segment parity; the reverse sweep of a segment waits for its
// recomputation, and a recomputation waits for the contraction that last
// read its workspace.  The same kernels' arithmetic as adjoint_launch.
static psst_status adjoint_launch_pipe(const AdjPlan &P, int32_t n, const InstDesc *d_desc,
                                       int64_t nt, AdjWork *W, const RecomputeFn &recompute,
                                       const float *ckpt, int32_t K, const psst_stimulus *stim,
                                       float dt, int64_t n_steps, int64_t step0,
                                       const float *dLdV, float *grad_g, float *gna, float *gk,
                                       float *gl, int32_t per_instance, int32_t *flag,
                                       const Tab &tab, hipStream_t st)
{
    if (P.lds > 65536) {
        HIPCHK(hipFuncSetAttribute(P.fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)P.lds));
        HIPCHK(hipFuncSetAttribute(P.fn_con, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)P.lds));
    }
    AdjArgs a{};
    a.desc = d_desc;
    a.ckpt = ckpt;
    a.K = K;
    a.nt = nt;
    if (stim) {
        a.stim.i_const = stim->i_const_nA;
        a.stim.pulse_ptr = stim->pulse_ptr;
        a.stim.on_step = stim->on_step;
        a.stim.off_step = stim->off_step;
        a.stim.amp = stim->amp_nA;
    }
    a.dt = (double)dt;
    a.n_steps = n_steps;
    a.step0 = step0;
    a.dLdV = dLdV;
    a.ws_stride = P.wstride;
    a.gacc = W->gacc;
    a.gacc_stride = P.gstride;
    a.lds_bytes = (int64_t)P.lds;
    a.flag = flag;
    a.tab = tab;
    a.adj_state = W->astate;
    a.adj_stride = P.astride;
    if (const char *e = std::getenv("PSST_ADJ_MODE")) a.mode = std::strcmp(e, "lacc") == 0 ? 1 : 0;
    double *wsb[2] = {W->ws, W->ws2};
    hipStream_t aux = W->aux;
    HIPCHK(hipEventRecord(W->ev_fork, st));
    HIPCHK(hipStreamWaitEvent(aux, W->ev_fork, 0));
    const int64_t nseg = (n_steps + K - 1) / K;
    for (int64_t seg = nseg - 1; seg >= 0; --seg) {
        const int par = (int)(seg & 1);
        const int64_t s0 = seg * K;
        const int64_t L = std::min<int64_t>(K, n_steps - s0);
        // recomputation of seg into wsb[par], after the contraction of seg + 2
        if (seg + 2 <= nseg - 1) HIPCHK(hipStreamWaitEvent(aux, W->ev_con[par], 0));
        psst_status s =
            recompute(ckpt + seg * 14 * nt, step0 + s0, L, wsb[par], P.wstride, K, aux);
        if (s != PSST_OK) return s;
        HIPCHK(hipEventRecord(W->ev_rec[par], aux));
        // reverse sweep and contraction of seg on the caller's stream
        HIPCHK(hipStreamWaitEvent(st, W->ev_rec[par], 0));
        a.ws = wsb[par];
        a.seg = seg;
        a.first = seg == nseg - 1;
        void *args[] = {&a};
        HIPCHK(hipLaunchKernel(P.fn, dim3(n), dim3(P.bs), args, P.lds, st));
        HIPCHK(hipLaunchKernel(P.fn_con, dim3(n), dim3(P.bs), args, P.lds, st));
        HIPCHK(hipEventRecord(W->ev_con[par], st));
    }
    HIPCHK(hipEventRecord(W->ev_join, aux));
    HIPCHK(hipStreamWaitEvent(st, W->ev_join, 0));
    FinArgs f{};
    f.desc = d_desc;
    f.n_inst = n;
    f.gacc = W->gacc;
    f.gacc_stride = P.gstride;
    f.goff = W->goff;
    f.grad_g = grad_g;
    f.gna = gna;
    f.gk = gk;
    f.gl = gl;
    f.per_instance = per_instance;
    void *fargs[] = {&f};
    HIPCHK(hipLaunchKernel((const void *)adjoint_finalize, dim3(per_instance ? n : 1), dim3(256),
                           fargs, 0, st));
    return PSST_OK;
}

psst_status adjoint_run(const std::vector<psst_network *> &nets, const InstDesc *d_desc,
                        int64_t nt, AdjWork **work, const RecomputeFn &recompute,
                        const float *ckpt, int32_t K, const psst_stimulus *stim, float dt,
                        int64_t n_steps, int64_t step0, const float *dLdV, float *grad_g,
                        float *gna, float *gk, float *gl, int32_t per_instance, int32_t *flag,
                        size_t lds_max, bool gen, const Tab &tab, void *stream,
                        const RecomputeFn *lean, size_t lean_lds)
{
    const int32_t n = (int32_t)nets.size();
    AdjPlan P;
    psst_status s = adjoint_plan(nets, K, lds_max, gen, &P);
    if (s != PSST_OK) return s;
    if (!*work) *work = new AdjWork();
    AdjWork *W = *work;
    // pipelined when a lean recomputation is offered, the call has two
    // segments or more and the reverse sweep's buffers fit the LDS the
    // recomputation leaves (PSST_ADJ_PIPE=0: one stream, as adjoint_launch)
    const char *pe = std::getenv("PSST_ADJ_PIPE");
    const bool pipe_ok = lean && !(pe && pe[0] == '0') && n_steps > K && lean_lds < lds_max;
    AdjPlan PP;
    bool pipe = false;
    if (pipe_ok && adjoint_plan(nets, K, lds_max - lean_lds, gen, &PP) == PSST_OK) pipe = true;
    if ((s = ensure((void **)&W->ws, &W->ws_bytes, sizeof(double) * P.wstride * n)) != PSST_OK)
        return s;
    if (pipe) {
        if ((s = ensure((void **)&W->ws2, &W->ws2_bytes, sizeof(double) * P.wstride * n)) !=
            PSST_OK)
            return s;
        if (!W->aux) {
            HIPCHK(hipStreamCreateWithFlags(&W->aux, hipStreamNonBlocking));
            HIPCHK(hipEventCreateWithFlags(&W->ev_fork, hipEventDisableTiming));
            HIPCHK(hipEventCreateWithFlags(&W->ev_join, hipEventDisableTiming));
            for (int k = 0; k < 2; ++k) {
                HIPCHK(hipEventCreateWithFlags(&W->ev_rec[k], hipEventDisableTiming));
                HIPCHK(hipEventCreateWithFlags(&W->ev_con[k], hipEventDisableTiming));
            }
        }
    }
    if ((s = ensure((void **)&W->gacc, &W->gacc_bytes, sizeof(float) * P.gstride * n)) != PSST_OK)
        return s;
    if ((s = ensure((void **)&W->astate, &W->astate_bytes, sizeof(double) * P.astride * n)) !=
        PSST_OK)
        return s;
    if (!W->goff) HIPCHK(hipMalloc(&W->goff, sizeof(int64_t) * n));
    hipStream_t st = (hipStream_t)stream;
    grad_offsets_kernel<<<dim3(1), dim3(256), 0, st>>>(d_desc, n, W->goff);
    HIPCHK(hipGetLastError());
    if (pipe)
        return adjoint_launch_pipe(PP, n, d_desc, nt, W, *lean, ckpt, K, stim, dt, n_steps, step0,
                                   dLdV, grad_g, gna, gk, gl, per_instance, flag, tab, st);
    return adjoint_launch(P, n, d_desc, nt, W->ws, W->gacc, W->goff, W->astate, recompute, ckpt,
                          K, stim, dt, n_steps, step0, dLdV, grad_g, gna, gk, gl, per_instance,
                          flag, tab, st);
}

// ---------------------------------------------------------------------------
// The adjoint without allocation (psst_adjoint_noalloc): the stage records,
// gradient accumulators and gradient offsets live in one file-scope device
// array of kAdjScratchBytes, one copy per device, shared by every call on
// that device (the last call's contents stay; calls that overlap on one
// device race).  Its device address is looked up once per device with the
// device current and kept; kernels are handed that address, never the
// array's host-side name.
// ---------------------------------------------------------------------------

static constexpr int64_t kAdjScratchBytes = 64LL << 20;
static __device__ __align__(256) unsigned char scratch[kAdjScratchBytes];

static constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices] = {};

static psst_status scratch_on_device(void **out)
{
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices)
        return fail(PSST_ERR_UNSUPPORTED, "device %d beyond the %d devices of the scratch table",
                    dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(PSST_ERR_DEVICE, "no device address for the adjoint scratch array");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return PSST_OK;
}

static int64_t align256(int64_t x) { return (x + 255) & ~(int64_t)255; }

psst_status adjoint_run_noalloc(const std::vector<psst_network *> &nets, const InstDesc *d_desc,
                                int64_t nt, const RecomputeFn &recompute, const float *ckpt,
                                int32_t K, const psst_stimulus *stim, float dt, int64_t n_steps,
                                int64_t step0, const float *dLdV, float *grad_g, float *gna,
                                float *gk, float *gl, int32_t per_instance, int32_t *flag,
                                size_t lds_max, bool gen, const Tab &tab, void *stream)
{
    const int32_t n = (int32_t)nets.size();
    AdjPlan P;
    psst_status s = adjoint_plan(nets, K, lds_max, gen, &P);
    if (s != PSST_OK) return s;
    const int64_t ws_b = align256((int64_t)sizeof(double) * P.wstride * n);
    const int64_t ga_b = align256((int64_t)sizeof(float) * P.gstride * n);
    const int64_t as_b = align256((int64_t)sizeof(double) * P.astride * n);
    const int64_t go_b = align256((int64_t)sizeof(int64_t) * n);
    if (ws_b + ga_b + as_b + go_b > kAdjScratchBytes)
        return fail(PSST_ERR_INVALID_ARGUMENT,
                    "psst_adjoint_noalloc needs %lld bytes of scratch (stage records %lld, "
                    "accumulators %lld, carried state %lld, offsets %lld) for %d instances at "
                    "K=%d; its maximum is %lld: use a smaller K or fewer instances, or "
                    "psst_adjoint",
                    (long long)(ws_b + ga_b + as_b + go_b), (long long)ws_b, (long long)ga_b,
                    (long long)as_b, (long long)go_b, n, K, (long long)kAdjScratchBytes);
    void *base = nullptr;
    if ((s = scratch_on_device(&base)) != PSST_OK) return s;
    unsigned char *b8 = static_cast<unsigned char *>(base);
    double *ws = reinterpret_cast<double *>(b8);
    float *gacc = reinterpret_cast<float *>(b8 + ws_b);
    double *astate = reinterpret_cast<double *>(b8 + ws_b + ga_b);
    int64_t *goff = reinterpret_cast<int64_t *>(b8 + ws_b + ga_b + as_b);
    hipStream_t st = (hipStream_t)stream;
    grad_offsets_kernel<<<dim3(1), dim3(256), 0, st>>>(d_desc, n, goff);
    HIPCHK(hipGetLastError());
    return adjoint_launch(P, n, d_desc, nt, ws, gacc, goff, astate, recompute, ckpt, K, stim, dt,
                          n_steps, step0, dLdV, grad_g, gna, gk, gl, per_instance, flag, tab, st);
}

void adjoint_free(AdjWork *w)
{
    if (!w) return;
    if (w->aux) {
        (void)hipStreamSynchronize(w->aux);
        (void)hipStreamDestroy(w->aux);
    }
    for (hipEvent_t e : {w->ev_fork, w->ev_join, w->ev_rec[0], w->ev_rec[1], w->ev_con[0],
                         w->ev_con[1]})
        if (e) (void)hipEventDestroy(e);
    (void)hipFree(w->ws2);
    (void)hipFree(w->ws);
    (void)hipFree(w->gacc);
    (void)hipFree(w->goff);
    (void)hipFree(w->astate);
    delete w;
}
