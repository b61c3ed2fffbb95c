// hh_device.h -- per-neuron Hodgkin-Huxley right-hand side on the GPU.
//
// State of neuron i (paper, "Brain simulations as computational graphs",
// vectorisation paragraph: X = [V, m, n, h] with per-neuron parameters
// C_m, g_K, ..., E_L): V, m, h, n, plus its outgoing transmitter gate s and,
// for local neurons of networks with slow GABA, the G-protein pair r, G.
//
// Everything here runs in float64: the per-neuron work is a few hundred
// operations per stage, negligible next to the synaptic products, and float64
// keeps the trajectory within 1e-3 mV of an exact-arithmetic solution for the
// first 50 ms (float32 rate functions alone would not).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace psst {

enum { YV = 0, YM = 1, YH = 2, YN = 3, YS = 4, YR = 5, YG = 6, NVAR = 7 };
enum { K_ALPHA = 0, K_BETA, K_EREV, K_VP, K_KP, K_R1, K_R2, K_R3, K_R4, K_KD, K_HILL, NKIN = 11 };
enum { P_CM = 0, P_GNA, P_GK, P_GL, P_ENA, P_EK, P_EL, NPRM = 7 };
enum { T_ACH = 0, T_GABA_A = 1, T_GABA_B = 2 };

// Instance descriptor: one network copy inside a launch.
struct InstDesc {
    const float *gt;    // fast conductances, transposed: gt[j * ld + i] = g(pre j -> post i), nS
    const float *gtb;   // slow-GABA conductances, transposed: gtb[(j - n_pn) * ld + i]; null if none
    const float *prm;   // [NPRM][ld] per-neuron parameters
    const float *kin;   // [3][NKIN] synapse kinetics
    int64_t off;        // first neuron of this instance in the packed arrays
    int32_t n, n_pn, ld, flags;   // flags bit 0: has slow GABA
    double cg, ci;      // nS -> mS/cm^2 and nA -> uA/cm^2 for this network's area
    const int64_t *paths;     // [n_paths][6]: type, pre0, pre1, post0, post1, grad offset
    const uint8_t *maskt;     // synapse mask laid out like gt (then gtb)
    int32_t n_paths;
    int64_t grad_entries;     // entries of one copy of the pathway blocks
    // sparse storage (flag DESC_SPARSE): per postsynaptic row i, its synapses
    // sorted by presynaptic index in ELL form, entry e at e * ld + i: the
    // fast matrix (columns 0..n-1) in entries [0, sp_kf), the slow matrix
    // (columns = LN index) in [sp_kf, sp_kf + sp_kb); short rows are padded
    // with their last column and g = 0
    const int32_t *sp_col;
    const float *sp_val;
    int32_t sp_kf, sp_kb;
};

// flags: bit 0 the network has slow GABA; bit 1 it has no synapses at all
// (the synaptic products are skipped, every synaptic sum is 0); bit 2 its
// conductances are stored sparse (sp_col, sp_val)
enum { DESC_GABAB = 1, DESC_NOSYN = 2, DESC_SPARSE = 4 };

// Synapse kinetics widened to float64.
struct Kin {
    double a_ach, b_ach, vp_ach, kp_ach, e_ach;
    double a_ga, b_ga, vp_ga, kp_ga, e_ga;
    double r1, r2, r3, r4, kd, vp_gb, kp_gb, e_gb;
    int hill;
};

__device__ inline Kin load_kin(const float *k)
{
    Kin q;
    q.a_ach = k[T_ACH * NKIN + K_ALPHA];  q.b_ach = k[T_ACH * NKIN + K_BETA];
    q.vp_ach = k[T_ACH * NKIN + K_VP];    q.kp_ach = k[T_ACH * NKIN + K_KP];
    q.e_ach = k[T_ACH * NKIN + K_EREV];
    q.a_ga = k[T_GABA_A * NKIN + K_ALPHA]; q.b_ga = k[T_GABA_A * NKIN + K_BETA];
    q.vp_ga = k[T_GABA_A * NKIN + K_VP];   q.kp_ga = k[T_GABA_A * NKIN + K_KP];
    q.e_ga = k[T_GABA_A * NKIN + K_EREV];
    q.r1 = k[T_GABA_B * NKIN + K_R1]; q.r2 = k[T_GABA_B * NKIN + K_R2];
    q.r3 = k[T_GABA_B * NKIN + K_R3]; q.r4 = k[T_GABA_B * NKIN + K_R4];
    q.kd = k[T_GABA_B * NKIN + K_KD];
    q.vp_gb = k[T_GABA_B * NKIN + K_VP]; q.kp_gb = k[T_GABA_B * NKIN + K_KP];
    q.e_gb = k[T_GABA_B * NKIN + K_EREV];
    q.hill = (int)k[T_GABA_B * NKIN + K_HILL];
    return q;
}

struct Prm {
    double C, gNa, gK, gL, ENa, EK, EL;
};

__device__ inline Prm load_prm(const float *p, int ld, int i)
{
    Prm q;
    q.C = p[P_CM * ld + i];   q.gNa = p[P_GNA * ld + i]; q.gK = p[P_GK * ld + i];
    q.gL = p[P_GL * ld + i];  q.ENa = p[P_ENA * ld + i]; q.EK = p[P_EK * ld + i];
    q.EL = p[P_EL * ld + i];
    return q;
}

// u / (1 - exp(-u)) from u and emu = exp(-u), extended by continuity
// (value 1) at u = 0; near 0 the series 1 + u/2 + u^2/12 - u^4/720 +
// u^6/30240 (Bernoulli numbers) replaces the cancelling quotient.
__device__ inline double exprel_from(double u, double emu)
{
    if (fabs(u) < 5e-2)
        return 1.0 + u * (0.5 + u * ((1.0 / 12.0) +
                                     u * u * ((-1.0 / 720.0) + u * u * (1.0 / 30240.0))));
    return u / (1.0 - emu);
}

// d/du of exprel, from u and exp(-u); series 1/2 + u/6 - u^3/180 + u^5/5040
// near 0.
__device__ inline double exprel_d_from(double u, double emu)
{
    if (fabs(u) < 5e-2)
        return 0.5 + u * ((1.0 / 6.0) + u * u * ((-1.0 / 180.0) + u * u * (1.0 / 5040.0)));
    const double d = 1.0 - emu;
    return (d - u * emu) / (d * d);
}

struct Rates {
    double am, bm, ah, bh, an, bn;
    double um, em, un, en;   // argument u and exp(-u) of the two exprel terms
};

// Hodgkin & Huxley 1952 rate functions, -65 mV convention, ms^-1.  With
// z = V + 65, every exponential of V in them is a power of E = exp(-z/720):
// exp(-z/80) = E^9, exp(-z/40) = E^18, exp(-z/20) = E^36, exp(-z/18) = E^40,
// exp(-z/10) = E^72, and exp(-(V+40)/10), exp(-(V+55)/10), exp(-(V+35)/10)
// are exp(-z/10) times e^2.5, e, e^3.  One exponential and eight products
// replace seven exponentials; the powers carry a relative error of a few
// tens of ulp (about 1e-14).
__device__ inline Rates hh_rates(double V)
{
    constexpr double kE1 = 2.718281828459045;      // e
    constexpr double kE25 = 12.182493960703473;    // e^2.5
    constexpr double kE3 = 20.085536923187668;     // e^3
    const double z = V + 65.0;
    const double e1 = exp(z * (-1.0 / 720.0));
    const double e2 = e1 * e1, e4 = e2 * e2, e8 = e4 * e4;
    const double e80 = e8 * e1;        // exp(-z / 80)
    const double e40 = e80 * e80;      // exp(-z / 40)
    const double e20 = e40 * e40;      // exp(-z / 20)
    const double e18 = e20 * e4;       // exp(-z / 18)
    const double e10 = e20 * e20;      // exp(-z / 10)
    Rates r;
    r.um = (V + 40.0) * 0.1;
    r.em = e10 * kE25;
    r.un = (V + 55.0) * 0.1;
    r.en = e10 * kE1;
    r.am = exprel_from(r.um, r.em);
    r.bm = 4.0 * e18;
    r.ah = 0.07 * e20;
    r.bh = 1.0 / (1.0 + e10 * kE3);
    r.an = 0.1 * exprel_from(r.un, r.en);
    r.bn = 0.125 * e80;
    return r;
}

__device__ inline double release(double V, double vp, double kp)
{
    return 1.0 / (1.0 + exp(-(V - vp) / kp));
}

// Release of a neuron's own transmitter (cholinergic for PN, fast GABA for
// LN rows) and, for LN rows with slow GABA, the slow-GABA release: one
// release evaluation each, the second reusing the first when the two share
// V_p and K_p (the same function of the same arguments, so the same value).
__device__ inline void releases(double V, const Kin &K, bool is_ln, bool slow, double &T,
                                double &TB)
{
    const double vp = is_ln ? K.vp_ga : K.vp_ach;
    const double kp = is_ln ? K.kp_ga : K.kp_ach;
    T = release(V, vp, kp);
    TB = T;
    if (slow && !(K.vp_gb == vp && K.kp_gb == kp)) TB = release(V, K.vp_gb, K.kp_gb);
}

__device__ inline double ipow(double x, int n)
{
    double p = 1.0;
    for (int i = 0; i < n; ++i) p *= x;
    return p;
}

// Slow-GABA activation x = G^n / (G^n + K_d).
__device__ inline double gabab_act(double G, const Kin &k)
{
    double gn = ipow(G, k.hill);
    return gn / (gn + k.kd);
}

__device__ inline double gabab_act_d(double G, const Kin &k)
{
    double gn = ipow(G, k.hill);
    double den = gn + k.kd;
    return k.hill * k.kd * ipow(G, k.hill - 1) / (den * den);
}

// The voltage-dependent factors of one neuron's right-hand side: the gate
// rates and the transmitter release(s) at V.
struct RateSet {
    Rates r;
    double T, TB;
};

__device__ inline RateSet rate_set(double V, const Kin &K, bool is_ln, bool slow)
{
    RateSet rs;
    rs.r = hh_rates(V);
    releases(V, K, is_ln, slow, rs.T, rs.TB);
    return rs;
}

// f(Y) for one neuron with its voltage-dependent factors rs = rate_set(Y[YV],
// K, is_ln, is_ln && gabab) already formed (a kernel may form them early, to
// overlap them with other work).  gs_* are the synaptic conductance sums
// already in mS/cm^2 (cg * sum_j g_ij x_j); Iu is the injected current in
// uA/cm^2.
__device__ inline void hh_rhs_rs(const double Y[NVAR], const Prm &P, const Kin &K,
                                 double gs_ach, double gs_ga, double gs_gb, double Iu,
                                 bool is_ln, bool gabab, const RateSet &rs, double f[NVAR])
{
    const double V = Y[YV], m = Y[YM], h = Y[YH], n = Y[YN], s = Y[YS];
    const Rates &r = rs.r;
    const double m3h = m * m * m * h;
    const double n4 = (n * n) * (n * n);
    const double Iion = P.gNa * m3h * (V - P.ENa) + P.gK * n4 * (V - P.EK) + P.gL * (V - P.EL);
    const double Isyn = (V - K.e_ach) * gs_ach + (V - K.e_ga) * gs_ga + (V - K.e_gb) * gs_gb;
    f[YV] = (Iu - Iion - Isyn) / P.C;
    f[YM] = r.am * (1.0 - m) - r.bm * m;
    f[YH] = r.ah * (1.0 - h) - r.bh * h;
    f[YN] = r.an * (1.0 - n) - r.bn * n;
    const double a = is_ln ? K.a_ga : K.a_ach;
    const double b = is_ln ? K.b_ga : K.b_ach;
    const double T = rs.T, TB = rs.TB;
    f[YS] = a * T * (1.0 - s) - b * s;
    if (is_ln && gabab) {
        f[YR] = K.r1 * TB * (1.0 - Y[YR]) - K.r2 * Y[YR];
        f[YG] = K.r3 * Y[YR] - K.r4 * Y[YG];
    } else {
        f[YR] = 0.0;
        f[YG] = 0.0;
    }
}

// f(Y) for one neuron (hh_rhs_rs with the factors formed here).
__device__ inline void hh_rhs(const double Y[NVAR], const Prm &P, const Kin &K,
                              double gs_ach, double gs_ga, double gs_gb, double Iu,
                              bool is_ln, bool gabab, double f[NVAR])
{
    hh_rhs_rs(Y, P, K, gs_ach, gs_ga, gs_gb, Iu, is_ln, gabab,
              rate_set(Y[YV], K, is_ln, is_ln && gabab), f);
}

// Vector-Jacobian product of hh_rhs at Y with cotangent w (dL/df): the
// elementwise part of u = J(Y)^T w, the synaptic weights q_t = dL/dI-share
// of each synapse class (q_t = w_V * (-(V - E_t) * cg / C), so that
// dL/dg_ij = q_t(i) * x_j and the presynaptic term is sum_i g_ij q_t(i)), and
// the per-neuron conductance cotangents dg = (dL/dg_Na, dL/dg_K, dL/dg_L).
// The synaptic terms u_s += sum_i g_ij q(i), u_G += (...) dx/dG are added by
// the caller, which holds the conductance matrix.
__device__ inline void hh_vjp(const double Y[NVAR], const Prm &P, const Kin &K, double cgf,
                              double gs_ach, double gs_ga, double gs_gb, const double w[NVAR],
                              bool is_ln, bool gabab, double u[NVAR], double q[3], double dg[3])
{
    const double V = Y[YV], m = Y[YM], h = Y[YH], n = Y[YN], s = Y[YS];
    const Rates r = hh_rates(V);
    // derivatives of the rates in V
    const double dam = exprel_d_from(r.um, r.em) * 0.1;
    const double dbm = -r.bm * (1.0 / 18.0);
    const double dah = -r.ah * 0.05;
    const double dbh = r.bh * (1.0 - r.bh) * 0.1;
    const double dan = 0.1 * exprel_d_from(r.un, r.en) * 0.1;
    const double dbn = -r.bn * 0.0125;
    const double invC = 1.0 / P.C;
    const double m2h = m * m * h, m3 = m * m * m, n3 = n * n * n;
    const double wV = w[YV];
    const double gtot = P.gNa * m3 * h + P.gK * n3 * n + P.gL + gs_ach + gs_ga + gs_gb;
    double uV = -wV * gtot * invC;
    uV += w[YM] * (dam * (1.0 - m) - dbm * m);
    uV += w[YH] * (dah * (1.0 - h) - dbh * h);
    uV += w[YN] * (dan * (1.0 - n) - dbn * n);
    const double al = is_ln ? K.a_ga : K.a_ach;
    const double be = is_ln ? K.b_ga : K.b_ach;
    const double kp = is_ln ? K.kp_ga : K.kp_ach;
    double T, TB;
    releases(V, K, is_ln, is_ln && gabab, T, TB);
    uV += w[YS] * al * (T * (1.0 - T) / kp) * (1.0 - s);
    u[YS] = -w[YS] * (al * T + be);
    if (is_ln && gabab) {
        const double rr = Y[YR];
        uV += w[YR] * K.r1 * (TB * (1.0 - TB) / K.kp_gb) * (1.0 - rr);
        u[YR] = -w[YR] * (K.r1 * TB + K.r2) + w[YG] * K.r3;
        u[YG] = -w[YG] * K.r4;
    } else {
        u[YR] = 0.0;
        u[YG] = 0.0;
    }
    u[YV] = uV;
    const double dENa = V - P.ENa, dEK = V - P.EK;
    u[YM] = -wV * 3.0 * P.gNa * m2h * dENa * invC - w[YM] * (r.am + r.bm);
    u[YH] = -wV * P.gNa * m3 * dENa * invC - w[YH] * (r.ah + r.bh);
    u[YN] = -wV * 4.0 * P.gK * n3 * dEK * invC - w[YN] * (r.an + r.bn);
    dg[0] = -wV * m3 * h * dENa * invC;
    dg[1] = -wV * n3 * n * dEK * invC;
    dg[2] = -wV * (V - P.EL) * invC;
    q[0] = -wV * (V - K.e_ach) * cgf * invC;
    q[1] = -wV * (V - K.e_ga) * cgf * invC;
    q[2] = -wV * (V - K.e_gb) * cgf * invC;
}

// Store a float64 value as a float32 pair (value, compensation); returns the
// exact float64 sum of the pair, which becomes the carried state.
__device__ inline double split_store(double y, float &hi, float &lo)
{
    hi = (float)y;
    lo = (float)(y - (double)hi);
    return (double)hi + (double)lo;
}

__device__ inline bool finite_d(double x)
{
    return !(x != x) && fabs(x) <= 1.7976931348623157e308;
}

}  // namespace psst
