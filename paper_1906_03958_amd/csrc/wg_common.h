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

// Partial sums over columns [ja, jb) of one chunk for rows 4 r4 .. 4 r4 + 3,
// added to s0..s3.  Row jj of the matrix is at G + (jj - row0) * ld.  Columns
// go in batches of U: all U loads are issued before the first is consumed, so
// each wavefront keeps U 16-byte loads in flight.  In the last, partial batch
// the row index is clamped and the activation taken as 0, which adds exact
// zeros and leaves the column-order sum unchanged.
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) const v4f global_float4;
typedef __attribute__((address_space(3))) const v4f lds_float4;
typedef __attribute__((address_space(3))) const double lds_double;
typedef __attribute__((address_space(3))) const float lds_float;
typedef __attribute__((address_space(1))) const float global_float;

template <int U, typename V4>
__device__ __forceinline__ void chunk_rows4(V4 *G4, int row0, int ld, const double *x, int ja,
                                            int jb, int r4, double &s0, double &s1, double &s2,
                                            double &s3)
{
    lds_double *X = (lds_double *)x;
    const int64_t q = ld >> 2;
    V4 *p = G4 + (ja - row0) * q + r4;
    int j = ja;
    for (; j + U <= jb; j += U, p += U * q) {
        v4f g[U];
        double xv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) g[u] = p[u * q];
#pragma unroll
        for (int u = 0; u < U; ++u) xv[u] = X[j + u];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            s0 = fma((double)g[u].x, xv[u], s0);
            s1 = fma((double)g[u].y, xv[u], s1);
            s2 = fma((double)g[u].z, xv[u], s2);
            s3 = fma((double)g[u].w, xv[u], s3);
        }
    }
    if (j < jb) {
        const int last = jb - 1 - j;
        v4f g[U];
        double xv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) g[u] = p[min(u, last) * q];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const double xx = X[j + min(u, last)];
            xv[u] = u <= last ? xx : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            s0 = fma((double)g[u].x, xv[u], s0);
            s1 = fma((double)g[u].y, xv[u], s1);
            s2 = fma((double)g[u].z, xv[u], s2);
            s3 = fma((double)g[u].w, xv[u], s3);
        }
    }
}

// Column range and source of chunk c: matrix 0 = fast (rows = presynaptic
// index), 1 = slow (rows = LN index); [j0, j1) in that matrix's row numbers
// and in the matching activation vector.
__device__ __forceinline__ void chunk_range(const Chunks &ch, int n, int n_pn, int c, int &mat,
                                            int &j0, int &j1)
{
    if (c < ch.na) {
        mat = 0; j0 = c * CW; j1 = min(j0 + CW, n_pn);
    } else if (c < ch.na + ch.ng) {
        mat = 0; j0 = n_pn + (c - ch.na) * CW; j1 = min(j0 + CW, n);
    } else {
        mat = 1; j0 = (c - ch.na - ch.ng) * CW; j1 = min(j0 + CW, n - n_pn);
    }
}

// One stage's chunk partials: column group cg takes chunks cg, cg + NCG, ...
// The first R columns of every chunk are read from the LDS copy (chunk c's
// rows at gl + c * R * ld), the rest from global memory.
__device__ __forceinline__ void stage_partials(const float *G, const float *GB, const float *gl,
                                               int R, int ld, const double *xf, const double *xb,
                                               double *part, const Chunks &ch, int n, int n_pn,
                                               int cg, int NCG, int r4)
{
    const int nch = ch.na + ch.ng + ch.nb;
    for (int c = cg; c < nch; c += NCG) {
        int mat, j0, j1;
        chunk_range(ch, n, n_pn, c, mat, j0, j1);
        const float *M = mat ? GB : G;
        const double *X = mat ? xb : xf;
        const int jr = min(j1, j0 + R);
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
        if (jr > j0)
            chunk_rows4<8>((lds_float4 *)(gl + (int64_t)c * R * ld), j0, ld, X, j0, jr, r4, s0,
                           s1, s2, s3);
        if (j1 > jr)
            chunk_rows4<8>((global_float4 *)M, 0, ld, X, jr, j1, r4, s0, s1, s2, s3);
        double *pc = part + (size_t)c * ld + 4 * r4;
        pc[0] = s0; pc[1] = s1; pc[2] = s2; pc[3] = s3;
    }
}

// One stage's chunk partials when the whole instance is in LDS: a thread
// takes one (chunk, postsynaptic row) pair at a time and sums that row over
// the chunk's columns -- the same column-order fma sequence (batches of U
// with clamped extra columns adding exact zeros) as the four-row form above,
// spread over rows x chunks threads instead of rows / 4 x chunks, so the
// sequential chain per stage is one chunk of one row.
template <int U>
__device__ __forceinline__ void stage_partials_lds(const float *gl, int ld, const double *xf,
                                                   const double *xb, double *part,
                                                   const Chunks &ch, int n, int n_pn, int tid,
                                                   int nthreads)
{
    const int nch = ch.na + ch.ng + ch.nb;
    for (int t = tid; t < nch * n; t += nthreads) {
        const int c = t / n, i = t - c * n;
        int mat, j0, j1;
        chunk_range(ch, n, n_pn, c, mat, j0, j1);
        lds_float *M = (lds_float *)(gl + (int64_t)c * CW * ld + i);
        lds_double *X = (lds_double *)(mat ? xb : xf);
        double s = 0.0;
        int j = j0;
        for (; j + U <= j1; j += U, M += U * ld) {
            float g[U];
            double xv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) g[u] = M[u * ld];
#pragma unroll
            for (int u = 0; u < U; ++u) xv[u] = X[j + u];
#pragma unroll
            for (int u = 0; u < U; ++u) s = fma((double)g[u], xv[u], s);
        }
        if (j < j1) {
            const int last = j1 - 1 - j;
            float g[U];
            double xv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) g[u] = M[min(u, last) * ld];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const double xx = X[j + min(u, last)];
                xv[u] = u <= last ? xx : 0.0;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) s = fma((double)g[u], xv[u], s);
        }
        part[(size_t)c * ld + i] = s;
    }
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

// The same current for steps taken in increasing order: the set of pulses
// that are on changes only at a pulse's on or off step, so the sum (formed as
// stim_nA forms it, in pulse order) is kept with the first step at which the
// set changes next, and the pulse table is read again only there.  Start
// with next = -1.
struct StimCache {
    double I;
    int64_t next;
};

__device__ __forceinline__ double stim_nA_cached(const StimDev &s, double Ic, int32_t p0,
                                                 int32_t p1, int64_t g, StimCache &c)
{
    if (g >= c.next) {
        double I = Ic;
        int64_t nx = INT64_MAX;
        for (int p = p0; p < p1; ++p) {
            const int64_t on = s.on_step[p], off = s.off_step[p];
            if (on <= g && g < off) I += (double)s.amp[p];
            if (on > g) nx = min(nx, on);
            else if (off > g) nx = min(nx, off);
        }
        c.I = I;
        c.next = nx;
    }
    return c.I;
}

// Sum of the chunk partials c0 .. c1-1 of one row (stride ld), added in
// chunk order starting from 0; loads go four at a time.
__device__ __forceinline__ double chunk_total(lds_double *P, int ld, int c0, int c1)
{
    double t = 0.0;
    int c = c0;
    for (; c + 4 <= c1; c += 4) {
        const double p0 = P[(c + 0) * ld], p1 = P[(c + 1) * ld];
        const double p2 = P[(c + 2) * ld], p3 = P[(c + 3) * ld];
        t += p0;
        t += p1;
        t += p2;
        t += p3;
    }
    for (; c < c1; ++c) t += P[c * ld];
    return t;
}

// Per-workgroup view of one instance for the synaptic sums.
struct WGSyn {
    const float *gt, *gtb;     // conductances in global memory
    const float *gl;           // LDS copy: the first R rows of every chunk
    double *xf, *xb, *part;    // LDS activations and chunk partials
    Chunks ch;
    int n, n_pn, ld, nch, NCG, r4, cg;
    int R;                     // LDS columns per chunk (CW = whole matrix in LDS)
    int XR;                    // register columns per chunk, before the LDS ones
    int KC;                    // chunks per column group when XR > 0 (else 0)
    bool gabab;
    bool sparse;               // conductances in sparse rows (sp_col, sp_val)
    bool sp_lds;               // ... copied to LDS for the launch
    const int32_t *sp_col;
    const float *sp_val;
    int sp_kf, sp_kb;
};

// Sparse rows: postsynaptic row i's synapses e = k0 .. k1-1 (sorted by
// presynaptic column, padded with the last column and g = 0), entry e at
// e * ld + i.  The products are summed in the fixed structure of the dense
// form -- each 64-column chunk's partial in column order from 0, partials
// added in chunk order, class by class -- and an absent synapse adds an exact
// zero there, so the totals equal the dense ones bit for bit.  split: first
// column of the second class (n_pn for the fast matrix; past every column for
// the slow matrix, one class).
template <int U, int AS>
__device__ __forceinline__ void sparse_row(const int32_t *col, const float *val, int ld, int i,
                                           int k0, int k1, const double *x, int split,
                                           double &t0, double &t1)
{
    typedef __attribute__((address_space(AS))) const int32_t gint;
    typedef __attribute__((address_space(AS))) const float gflt;
    gint *C = (gint *)col;
    gflt *G = (gflt *)val;
    lds_double *X = (lds_double *)x;
    double cur = 0.0;
    int key = -1;                  // chunk of the running partial (class 1 keys offset)
    for (int e = k0; e < k1; e += U) {
        int j[U];
        float g[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int ee = min(e + u, k1 - 1);
            j[u] = C[(int64_t)ee * ld + i];
            g[u] = G[(int64_t)ee * ld + i];
        }
        double xv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) xv[u] = X[j[u]];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (e + u >= k1) break;
            const int kk = j[u] < split ? j[u] / CW : (1 << 24) + (j[u] - split) / CW;
            if (kk != key) {
                if (key >= 0) {
                    if (key < (1 << 24)) t0 += cur;
                    else t1 += cur;
                }
                cur = 0.0;
                key = kk;
            }
            cur = fma((double)g[u], xv[u], cur);
        }
    }
    if (key >= 0) {
        if (key < (1 << 24)) t0 += cur;
        else t1 += cur;
    }
}

// Conductance columns a thread keeps in registers for a whole launch: S
// float4 slots; with KC chunks per column group (chunk cg + k NCG, k < KC)
// and XC columns per chunk (a multiple of kRegBatch, XC KC <= S), slot
// k XC + u holds column j0 + u of chunk k's four rows (zeros past the chunk's
// end and in unused slots).  The slot index is a compile-time constant
// wherever a slot is touched, so the slots stay in registers whatever KC is.
// S = 0: none.
template <int S>
struct RegCols {
    v4f g[S];
};
template <>
struct RegCols<0> {
};

// The pointers and sizes the register-column routines use, passed as values
// (selecting between fields of the per-workgroup struct would make the
// compiler address that struct in memory and lose the pointers' address
// spaces).
struct RRView {
    const float *gt, *gtb, *gl;
    const double *xf, *xb;
    double *part;
    Chunks ch;
    int n, n_pn, ld, nch, NCG, cg, r4, R, XR, KC;
};

__device__ __forceinline__ RRView rr_view(const WGSyn &w)
{
    return RRView{w.gt,  w.gtb,  w.gl,  w.xf,  w.xb,  w.part, w.ch, w.n,  w.n_pn,
                  w.ld,  w.nch,  w.NCG, w.cg,  w.r4,  w.R,    w.XR, w.KC};
}

template <int S>
__device__ __forceinline__ void load_regcols(const RRView v, RegCols<S> &rc)
{
    if (v.KC == 0) {            // no register columns (the matrices may not exist)
#pragma unroll
        for (int sl = 0; sl < S; ++sl) rc.g[sl] = v4f{0.f, 0.f, 0.f, 0.f};
        return;
    }
    const int64_t q = v.ld >> 2;
    const int XC = v.XR;
    global_float4 *Gf = (global_float4 *)v.gt + v.r4;
    global_float4 *Gb = (global_float4 *)(v.gtb ? v.gtb : v.gt) + v.r4;
#pragma unroll
    for (int sl = 0; sl < S; ++sl) {
        const int k = sl / XC, u = sl - k * XC;
        const int c = v.cg + k * v.NCG;
        const bool valid = k < v.KC && v.cg < v.NCG && c < v.nch;
        int mat = 0, j0 = 0, j1 = 0;
        if (valid) chunk_range(v.ch, v.n, v.n_pn, c, mat, j0, j1);
        const bool in = valid && j0 + u < j1;
        const int64_t e = in ? (int64_t)(j0 + u) * q : 0;
        const v4f val = mat ? Gb[e] : Gf[e];
        rc.g[sl] = in ? val : v4f{0.f, 0.f, 0.f, 0.f};
    }
}

// One stage's chunk partials with register columns (v.KC > 0): per chunk k of
// the thread's column group, its register columns (the batches of kRegBatch
// slots among k XC .. k XC + XC - 1; a column past the chunk's end has g = 0
// and adds an exact zero, its activation read from the chunk's last column),
// then its LDS columns, then the streamed rest -- the column-order fma
// sequence of stage_partials.
template <int S, int UG = 8>
__device__ __forceinline__ void stage_partials_rr(const RRView v, const RegCols<S> &rc)
{
    constexpr int B = kRegBatch;
    static_assert(S % B == 0, "slots come in whole batches");
    const int XC = v.XR;
#pragma unroll 1
    for (int k = 0; k < v.KC; ++k) {
        const int c = v.cg + k * v.NCG;
        if (c >= v.nch) break;
        int mat, j0, j1;
        chunk_range(v.ch, v.n, v.n_pn, c, mat, j0, j1);
        const float *M = mat ? v.gtb : v.gt;
        const double *Xd = mat ? v.xb : v.xf;
        lds_double *X = (lds_double *)Xd;
        const int s_lo = k * XC, s_hi = s_lo + XC;    // this chunk's slots
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll
        for (int b0 = 0; b0 < S; b0 += B) {
            if (b0 < s_lo || b0 >= s_hi) continue;     // uniform: batch of another chunk
            double xv[B];
#pragma unroll
            for (int u = 0; u < B; ++u) xv[u] = X[min(j0 + (b0 - s_lo) + u, j1 - 1)];
#pragma unroll
            for (int u = 0; u < B; ++u) {
                // an empty asm makes each stage use the float32 values
                // afresh: otherwise their float64 widening is hoisted out of
                // the time loop and takes twice the registers
                v4f g = rc.g[b0 + u];
                asm volatile("" : "+v"(g));
                s0 = fma((double)g.x, xv[u], s0);
                s1 = fma((double)g.y, xv[u], s1);
                s2 = fma((double)g.z, xv[u], s2);
                s3 = fma((double)g.w, xv[u], s3);
            }
        }
        const int ja = min(j1, j0 + XC);
        const int jr = min(j1, ja + v.R);
        if (jr > ja)
            chunk_rows4<8>((lds_float4 *)(v.gl + (int64_t)c * v.R * v.ld), ja, v.ld, Xd, ja, jr,
                           v.r4, s0, s1, s2, s3);
        if (j1 > jr)
            chunk_rows4<UG>((global_float4 *)M, 0, v.ld, Xd, jr, j1, v.r4, s0, s1, s2, s3);
        typedef __attribute__((address_space(3))) double lds_double_w;
        lds_double_w *pc = (lds_double_w *)(v.part + (size_t)c * v.ld + 4 * v.r4);
        pc[0] = s0; pc[1] = s1; pc[2] = s2; pc[3] = s3;
    }
}

// Synaptic sums (nS) at stage input Y for the calling thread's neurons
// i = tid + k * BS: write the activations, sync, form the chunk partials, sync,
// add the partials in chunk order.  Every thread of the workgroup must call.
template <int BS, int NPT, int S = 0>
__device__ __forceinline__ void syn_sums(const WGSyn &w, const Kin &K, const double (&Y)[NPT][NVAR],
                                         double (&sa)[NPT], double (&sg)[NPT], double (&sb)[NPT],
                                         const RegCols<S> *rc = nullptr)
{
    const int tid = threadIdx.x;
    if (w.sparse) {
        // activations, barrier, each thread its own rows, barrier (the
        // activations are rewritten at the next stage)
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            const int i = tid + k * BS;
            if (i < w.n) {
                w.xf[i] = Y[k][YS];
                if (w.gabab && i >= w.n_pn) w.xb[i - w.n_pn] = gabab_act(Y[k][YG], K);
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            const int i = tid + k * BS;
            double a = 0.0, g = 0.0, b = 0.0, unused = 0.0;
            if (i < w.n) {
                if (w.sp_lds) {
                    sparse_row<8, 3>(w.sp_col, w.sp_val, w.ld, i, 0, w.sp_kf, w.xf, w.n_pn, a, g);
                    if (w.sp_kb > 0)
                        sparse_row<8, 3>(w.sp_col, w.sp_val, w.ld, i, w.sp_kf, w.sp_kf + w.sp_kb,
                                         w.xb, 1 << 30, b, unused);
                } else {
                    sparse_row<8, 1>(w.sp_col, w.sp_val, w.ld, i, 0, w.sp_kf, w.xf, w.n_pn, a, g);
                    if (w.sp_kb > 0)
                        sparse_row<8, 1>(w.sp_col, w.sp_val, w.ld, i, w.sp_kf, w.sp_kf + w.sp_kb,
                                         w.xb, 1 << 30, b, unused);
                }
            }
            sa[k] = a;
            sg[k] = g;
            sb[k] = b;
        }
        __syncthreads();
        return;
    }
    if (w.nch == 0) {      // no synapses (uniform over the workgroup: no barriers)
#pragma unroll
        for (int k = 0; k < NPT; ++k) sa[k] = sg[k] = sb[k] = 0.0;
        return;
    }
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
        const int i = tid + k * BS;
        if (i < w.n) {
            w.xf[i] = Y[k][YS];
            if (w.gabab && i >= w.n_pn) w.xb[i - w.n_pn] = gabab_act(Y[k][YG], K);
        }
    }
    __syncthreads();
    if (w.R == CW) {
        stage_partials_lds<8>(w.gl, w.ld, w.xf, w.xb, w.part, w.ch, w.n, w.n_pn, tid, BS);
    } else if (w.cg < w.NCG) {
        bool done = false;
        if constexpr (S > 0) {
            if (w.KC > 0) {
                stage_partials_rr<S, S >= 48 ? 8 : 16>(rr_view(w), *rc);
                done = true;
            }
        }
        if (!done)
            stage_partials(w.gt, w.gtb, w.gl, w.R, w.ld, w.xf, w.xb, w.part, w.ch, w.n, w.n_pn,
                           w.cg, w.NCG, w.r4);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
        const int i = tid + k * BS;
        const int ir = i < w.n ? i : 0;
        lds_double *P = (lds_double *)w.part + ir;
        sa[k] = chunk_total(P, w.ld, 0, w.ch.na);
        sg[k] = chunk_total(P, w.ld, w.ch.na, w.ch.na + w.ch.ng);
        sb[k] = chunk_total(P, w.ld, w.ch.na + w.ch.ng, w.nch);
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

// The calling thread's neuron slots for one step: slot k holds neuron
// idx(k) of the instance (a neuron when below n); live(k) false skips the
// slot's per-neuron work (uniform over the workgroup for the per-instance
// mappings, per lane for the lane-group one).  syn(Y, sa, sg, sb) forms the
// synaptic sums of every slot from the stage inputs; every thread calls it.
struct Slots {
    int n, n_pn;
    bool gabab;
};

// One RK4 step of the calling thread's neurons, y updated in place and
// rounded to its stored float32 pair.  Iu: injected current (uA/cm^2).
// post(k, Y) (optional) sees every slot's next stage input -- after each
// stage's update, and the step's result after the combine -- in the basic
// block that formed it, so work that only depends on it (the lane-group
// kernel's slow-GABA activation) can overlap the right-hand side.
struct NoPost {
    __device__ void operator()(int, const double (&)[NVAR]) const {}
};

// The voltage-dependent factors of slot k's right-hand side at its stage
// input; a kernel that formed them earlier returns those (same values).
struct RatesHere {
    __device__ RateSet operator()(int, const double (&Yk)[NVAR], const Kin &K, bool is_ln,
                                  bool gabab) const
    {
        return rate_set(Yk[YV], K, is_ln, is_ln && gabab);
    }
};

template <int NPT, typename Syn, typename Idx, typename Live, typename Post = NoPost,
          typename RS = RatesHere>
__device__ __forceinline__ void rk4_step_core(const Slots &sl, Syn &&syn, Idx &&idx, Live &&live,
                                              const Kin &K, double cgf,
                                              const float (&pr)[NPT][NPRM],
                                              const double (&Iu)[NPT], double dt,
                                              double (&y)[NPT][NVAR], const StageStash *stash,
                                              Post &&post = Post(), RS &&rates = RS())
{
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
        syn(Y, sa, sg, sb);
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            if (!live(k)) continue;
            const int i = idx(k);
            if (stash && i < sl.n) {
#pragma unroll
                for (int v = 0; v < NVAR; ++v) stash->sY[(q * NVAR + v) * stash->ld + i] = Y[k][v];
                stash->sS[(q * 3 + 0) * stash->ld + i] = sa[k];
                stash->sS[(q * 3 + 1) * stash->ld + i] = sg[k];
                stash->sS[(q * 3 + 2) * stash->ld + i] = sb[k];
            }
            double f[NVAR];
            hh_rhs_rs(Y[k], prm_of(pr[k]), K, cgf * sa[k], cgf * sg[k], cgf * sb[k], Iu[k],
                      i >= sl.n_pn, sl.gabab, rates(k, Y[k], K, i >= sl.n_pn, sl.gabab), f);
            const double wq = (q == 0 || q == 3) ? 1.0 : 2.0;
            const double c = (q == 2) ? dt : 0.5 * dt;
#pragma unroll
            for (int v = 0; v < NVAR; ++v) {
                acc[k][v] += wq * f[v];
                if (q < 3) Y[k][v] = y[k][v] + c * f[v];
            }
            if (q < 3) post(k, Y[k]);
            // one neuron's right-hand side at a time: interleaving several
            // would multiply the temporaries held at once
            if constexpr (NPT > 1) __builtin_amdgcn_sched_barrier(0);
        }
    }
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
        if (idx(k) >= sl.n || !live(k)) continue;
#pragma unroll
        for (int v = 0; v < NVAR; ++v) {
            float hi, lo;
            y[k][v] = split_store(y[k][v] + (dt / 6.0) * acc[k][v], hi, lo);
        }
        post(k, y[k]);
    }
}

// One step of the explicit method T (1 to 4 stages) for the calling thread's
// neurons: stage inputs Y_q = y + dt sum_{r<q} a_qr k_r (the sum over r in
// order, from 0), k_q = f(Y_q), then y <- y + dt sum_q b_q k_q rounded to its
// stored float32 pair.  The stage loop is unrolled so the earlier k stay in
// registers; T.s is the same for the whole workgroup, so the barriers inside
// the synaptic sums are reached by every thread.
template <int NPT, typename Syn, typename Idx, typename Live, typename Post = NoPost,
          typename RS = RatesHere>
__device__ __forceinline__ void rk_step_core_tab(const Slots &sl, Syn &&syn, Idx &&idx,
                                                 Live &&live, const Kin &K, double cgf,
                                                 const float (&pr)[NPT][NPRM],
                                                 const double (&Iu)[NPT], double dt,
                                                 double (&y)[NPT][NVAR], const StageStash *stash,
                                                 const Tab &T, Post &&post = Post(),
                                                 RS &&rates = RS())
{
    double inc[NPT][NVAR];
    double kq[3][NPT][NVAR];
    double Y[NPT][NVAR];
#pragma unroll
    for (int k = 0; k < NPT; ++k)
#pragma unroll
        for (int v = 0; v < NVAR; ++v) {
            inc[k][v] = 0.0;
            Y[k][v] = y[k][v];
        }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (q >= T.s) break;
        if (q > 0) {
#pragma unroll
            for (int k = 0; k < NPT; ++k)
#pragma unroll
                for (int v = 0; v < NVAR; ++v) {
                    double acc = 0.0;
#pragma unroll
                    for (int r = 0; r < q; ++r) acc += T.a[q][r] * kq[r][k][v];
                    Y[k][v] = y[k][v] + dt * acc;
                }
#pragma unroll
            for (int k = 0; k < NPT; ++k)
                if (live(k)) post(k, Y[k]);
        }
        double sa[NPT], sg[NPT], sb[NPT];
        syn(Y, sa, sg, sb);
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            if (!live(k)) continue;
            const int i = idx(k);
            if (stash && i < sl.n) {
#pragma unroll
                for (int v = 0; v < NVAR; ++v) stash->sY[(q * NVAR + v) * stash->ld + i] = Y[k][v];
                stash->sS[(q * 3 + 0) * stash->ld + i] = sa[k];
                stash->sS[(q * 3 + 1) * stash->ld + i] = sg[k];
                stash->sS[(q * 3 + 2) * stash->ld + i] = sb[k];
            }
            double f[NVAR];
            hh_rhs_rs(Y[k], prm_of(pr[k]), K, cgf * sa[k], cgf * sg[k], cgf * sb[k], Iu[k],
                      i >= sl.n_pn, sl.gabab, rates(k, Y[k], K, i >= sl.n_pn, sl.gabab), f);
#pragma unroll
            for (int v = 0; v < NVAR; ++v) {
                inc[k][v] += T.b[q] * f[v];
                if (q < 3) kq[q][k][v] = f[v];
            }
        }
    }
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
        if (idx(k) >= sl.n || !live(k)) continue;
#pragma unroll
        for (int v = 0; v < NVAR; ++v) {
            float hi, lo;
            y[k][v] = split_store(y[k][v] + dt * inc[k][v], hi, lo);
        }
        post(k, y[k]);
    }
}

// The per-instance mappings: slot k of thread tid is neuron tid + k BS.
template <int BS, int NPT, int S = 0>
__device__ __forceinline__ void rk4_step_wg(const WGSyn &w, const Kin &K, double cgf,
                                            const float (&pr)[NPT][NPRM], const double (&Iu)[NPT],
                                            double dt, double (&y)[NPT][NVAR],
                                            const StageStash *stash,
                                            const RegCols<S> *rc = nullptr)
{
    const int tid = threadIdx.x;
    rk4_step_core<NPT>(
        Slots{w.n, w.n_pn, w.gabab},
        [&](const double (&Y)[NPT][NVAR], double (&sa)[NPT], double (&sg)[NPT],
            double (&sb)[NPT]) { syn_sums<BS, NPT, S>(w, K, Y, sa, sg, sb, rc); },
        [&](int k) { return tid + k * BS; }, [&](int k) { return k * BS < w.n; }, K, cgf, pr,
        Iu, dt, y, stash);
}

template <int BS, int NPT, int S = 0>
__device__ __forceinline__ void rk_step_wg_tab(const WGSyn &w, const Kin &K, double cgf,
                                               const float (&pr)[NPT][NPRM],
                                               const double (&Iu)[NPT], double dt,
                                               double (&y)[NPT][NVAR], const StageStash *stash,
                                               const Tab &T,
                                               const RegCols<S> *rc = nullptr)
{
    const int tid = threadIdx.x;
    rk_step_core_tab<NPT>(
        Slots{w.n, w.n_pn, w.gabab},
        [&](const double (&Y)[NPT][NVAR], double (&sa)[NPT], double (&sg)[NPT],
            double (&sb)[NPT]) { syn_sums<BS, NPT, S>(w, K, Y, sa, sg, sb, rc); },
        [&](int k) { return tid + k * BS; }, [&](int k) { return k * BS < w.n; }, K, cgf, pr,
        Iu, dt, y, stash, T);
}

// Set up the workgroup's view of instance d: LDS carve-up and the resident
// part of the conductances -- as many leading columns of every chunk as the
// launch's LDS allocation leaves room for (all of them when the instance fits).
template <int BS>
__device__ __forceinline__ WGSyn wg_setup(const InstDesc &d, double *lds_d, int64_t lds_bytes,
                                          int slots = 0)
{
    WGSyn w;
    w.n = d.n;
    w.n_pn = d.n_pn;
    w.ld = d.ld;
    w.gabab = (d.flags & DESC_GABAB) != 0;
    w.sparse = (d.flags & DESC_SPARSE) != 0;
    w.sp_col = d.sp_col;
    w.sp_val = d.sp_val;
    w.sp_kf = d.sp_kf;
    w.sp_kb = d.sp_kb;
    w.ch = (d.flags & (DESC_NOSYN | DESC_SPARSE)) ? Chunks{0, 0, 0}
                                                  : chunks_of(d.n, d.n_pn, w.gabab);
    w.nch = w.ch.na + w.ch.ng + w.ch.nb;
    w.xf = lds_d;
    w.xb = lds_d + d.ld;
    w.part = lds_d + 2 * d.ld;
    float *gl = reinterpret_cast<float *>(w.part + (size_t)w.nch * d.ld);
    w.gl = gl;
    w.gt = d.gt;
    w.gtb = d.gtb;
    const int64_t room = lds_bytes - (int64_t)sizeof(double) * (2 + w.nch) * d.ld;
    // sparse rows: the whole ELL (columns then values) into LDS when it fits
    w.sp_lds = false;
    if (w.sparse) {
        const int64_t ents = (int64_t)(d.sp_kf + d.sp_kb) * d.ld;
        if (8 * ents <= room) {
            int32_t *lc = reinterpret_cast<int32_t *>(gl);
            float *lv = reinterpret_cast<float *>(lc + ents);
            for (int64_t e = threadIdx.x; e < ents; e += BS) {
                lc[e] = d.sp_col[e];
                lv[e] = d.sp_val[e];
            }
            w.sp_col = lc;
            w.sp_val = lv;
            w.sp_lds = true;
        }
    }
    wg_residency(lds_bytes, d.ld, w.nch, BS, slots, &w.R, &w.XR, &w.KC);
    const int tid = threadIdx.x;
    if (w.R > 0) {
        const int q = d.ld >> 2;
        for (int c = 0; c < w.nch; ++c) {
            int mat, j0, j1;
            chunk_range(w.ch, d.n, d.n_pn, c, mat, j0, j1);
            const int jl = min(j1, j0 + w.XR);      // first LDS column of the chunk
            const int rows = min(j1, jl + w.R) - jl;
            const float4 *src = reinterpret_cast<const float4 *>((mat ? d.gtb : d.gt) +
                                                                 (int64_t)jl * d.ld);
            float4 *dst = reinterpret_cast<float4 *>(gl + (int64_t)c * w.R * d.ld);
            for (int e = tid; e < rows * q; e += BS) dst[e] = src[e];
        }
    }
    const int RQ = d.ld >> 2;
    w.NCG = BS / RQ;
    w.r4 = tid % RQ;
    w.cg = tid / RQ;
    return w;
}

// Row j of matrix mat (0 fast, 1 slow) in the LDS copy, when the whole
// instance is resident (R == CW).
__device__ __forceinline__ const float *lds_row(const WGSyn &w, int mat, int j)
{
    const int c = mat ? w.ch.na + w.ch.ng + j / CW
                      : (j < w.n_pn ? j / CW : w.ch.na + (j - w.n_pn) / CW);
    const int j0 = mat ? (j / CW) * CW : (j < w.n_pn ? (j / CW) * CW : w.n_pn + ((j - w.n_pn) / CW) * CW);
    return w.gl + ((int64_t)c * w.R + (j - j0)) * w.ld;
}

}  // namespace psst
