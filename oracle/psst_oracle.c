/*
 * psst_oracle.c -- plain, slow FP64 reference for fixed-step RK4 integration
 * of coupled Hodgkin-Huxley networks, and its discrete adjoint.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the HIP library; the two meet only in the
 * seeded float32 inputs produced by the workload generator.
 *
 * What it computes (paper sections cited; the paper prints no rate functions
 * or synapse equations, so those follow the readings listed beside them):
 *
 *  - the initial value problem dy/dt = f(y, t), y(t0) = y0 ("Brain
 *    simulations as computational graphs", equation of the IVP);
 *  - the classical fourth-order Runge-Kutta step, local error O(dt^5) (same
 *    section, RK4 paragraph), iterated as a scan whose output rows are the
 *    states after each step, without the initial value (the tf.scan
 *    cumulative-sum example prints [6 8 11 15 20 26] for initializer 5);
 *  - per-neuron state [V, m, h, n] in structure-of-arrays form with per-neuron
 *    parameter vectors C_m, g_Na, g_K, g_L, E_Na, E_K, E_L (vectorisation
 *    paragraph); rate functions: Hodgkin & Huxley 1952, -65 mV convention;
 *  - synaptic currents summed over a dense n x n conductance matrix per
 *    synapse type ("Circumventing memory constraints", item 1), with a
 *    first-order gate s_j per presynaptic neuron for cholinergic and fast-GABA
 *    synapses and a two-variable (r, G) G-protein scheme for slow GABA;
 *  - every step in float64, no compensation, no reassociation.
 *
 * State layout: y[var * n + i], var = V, m, h, n, s, r, G (7 planes; the
 * slow-GABA pair r, G exists only for LN rows of networks that have a slow-GABA
 * pathway, and stays constant otherwise).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { YV = 0, YM = 1, YH = 2, YN = 3, YS = 4, YR = 5, YG = 6, NVAR = 7 };
enum { T_ACH = 0, T_GABA_A = 1, T_GABA_B = 2 };
enum { K_ALPHA = 0, K_BETA, K_EREV, K_VP, K_KP, K_R1, K_R2, K_R3, K_R4, K_KD,
       K_HILL, NKIN };
enum { P_CM = 0, P_GNA, P_GK, P_GL, P_ENA, P_EK, P_EL, NPRM };

/* Network description (all float64, already widened from float32). */
typedef struct {
    int32_t n, n_pn;
    const double *prm;      /* [NPRM][n] */
    int32_t n_path;
    const int32_t *pinfo;   /* [n_path][5]: type, pre0, pre1, post0, post1 */
    const double *g;        /* packed pathway blocks, each [post x pre], nS */
    const double *kin;      /* [3][NKIN] */
    double area_cm2;
} or_net;

/* Injected current, nA: constant + per-neuron pulses (CSR by neuron). */
typedef struct {
    const double *i_const;  /* [n] */
    const int32_t *pulse_ptr;   /* [n+1] or NULL */
    const int64_t *on_step, *off_step;
    const double *amp;
} or_stim;

/* ---------------------------------------------------------------------- */
/* Rate functions                                                          */
/* ---------------------------------------------------------------------- */

/* u / (1 - exp(-u)), continuously extended by 1 at u = 0. */
double or_exprel(double u)
{
    if (fabs(u) < 1e-6)
        return 1.0 + u / 2.0 + u * u / 12.0;
    return u / (-expm1(-u));
}

/* derivative of or_exprel */
double or_exprel_d(double u)
{
    if (fabs(u) < 1e-4)
        return 0.5 + u / 6.0 - u * u * u / 180.0;
    double e = exp(-u);
    double d = -expm1(-u);
    return (d - u * e) / (d * d);
}

/* alpha/beta of m, h, n at membrane potential V (mV); ms^-1. */
void or_rates(double V, double r[6])
{
    r[0] = or_exprel((V + 40.0) / 10.0);              /* alpha_m */
    r[1] = 4.0 * exp(-(V + 65.0) / 18.0);             /* beta_m  */
    r[2] = 0.07 * exp(-(V + 65.0) / 20.0);            /* alpha_h */
    r[3] = 1.0 / (1.0 + exp(-(V + 35.0) / 10.0));     /* beta_h  */
    r[4] = 0.1 * or_exprel((V + 55.0) / 10.0);        /* alpha_n */
    r[5] = 0.125 * exp(-(V + 65.0) / 80.0);           /* beta_n  */
}

/* d/dV of the six rates */
static void rates_d(double V, const double r[6], double d[6])
{
    d[0] = or_exprel_d((V + 40.0) / 10.0) / 10.0;
    d[1] = -r[1] / 18.0;
    d[2] = -r[2] / 20.0;
    d[3] = r[3] * (1.0 - r[3]) / 10.0;
    d[4] = 0.1 * or_exprel_d((V + 55.0) / 10.0) / 10.0;
    d[5] = -r[5] / 80.0;
}

/* transmitter release: sigmoid of the presynaptic potential */
static double release(double V, const double *k)
{
    return 1.0 / (1.0 + exp(-(V - k[K_VP]) / k[K_KP]));
}

static double ipow(double x, int n)
{
    double p = 1.0;
    for (int i = 0; i < n; ++i) p *= x;
    return p;
}

/* slow-GABA activation x = G^n / (G^n + K_d) */
static double gabab_act(double G, const double *k)
{
    double gn = ipow(G, (int)k[K_HILL]);
    return gn / (gn + k[K_KD]);
}

static double gabab_act_d(double G, const double *k)
{
    int n = (int)k[K_HILL];
    double gn = ipow(G, n);
    double den = gn + k[K_KD];
    return n * k[K_KD] * ipow(G, n - 1) / (den * den);
}

/* kinetics row used by the outgoing synapse of neuron i (cell type) */
static const double *own_kin(const or_net *net, int i)
{
    return net->kin + (i < net->n_pn ? T_ACH : T_GABA_A) * NKIN;
}

static int has_slow_gaba(const or_net *net)
{
    for (int p = 0; p < net->n_path; ++p)
        if (net->pinfo[5 * p] == T_GABA_B) return 1;
    return 0;
}

static int64_t path_offset(const or_net *net, int p)
{
    int64_t off = 0;
    for (int q = 0; q < p; ++q) {
        const int32_t *pi = net->pinfo + 5 * q;
        off += (int64_t)(pi[4] - pi[3]) * (pi[2] - pi[1]);
    }
    return off;
}

/* presynaptic activation of neuron j for synapse type t */
static double activation(const or_net *net, const double *y, int t, int j)
{
    int n = net->n;
    if (t == T_GABA_B) return gabab_act(y[YG * n + j], net->kin + T_GABA_B * NKIN);
    return y[YS * n + j];
}

/* ---------------------------------------------------------------------- */
/* Stimulus                                                                */
/* ---------------------------------------------------------------------- */

static double stim_nA(const or_stim *st, int i, int64_t g)
{
    double I = st->i_const ? st->i_const[i] : 0.0;
    if (st->pulse_ptr) {
        for (int k = st->pulse_ptr[i]; k < st->pulse_ptr[i + 1]; ++k)
            if (st->on_step[k] <= g && g < st->off_step[k]) I += st->amp[k];
    }
    return I;
}

/* ---------------------------------------------------------------------- */
/* Right-hand side f(y), with I held over the step                        */
/* ---------------------------------------------------------------------- */

/* syn[p][i]: sum_j g^p_ij x^p_j in nS for the post rows of pathway p */
static void synaptic_sums(const or_net *net, const double *y, double *A)
{
    int n = net->n;
    memset(A, 0, sizeof(double) * 3 * n);   /* A[type][i] */
    int64_t off = 0;
    for (int p = 0; p < net->n_path; ++p) {
        const int32_t *pi = net->pinfo + 5 * p;
        int t = pi[0], pre0 = pi[1], pre1 = pi[2], post0 = pi[3], post1 = pi[4];
        int npre = pre1 - pre0;
        const double *g = net->g + off;
        for (int i = post0; i < post1; ++i) {
            double acc = 0.0;
            for (int j = pre0; j < pre1; ++j)
                acc += g[(int64_t)(i - post0) * npre + (j - pre0)] * activation(net, y, t, j);
            A[t * n + i] += acc;
        }
        off += (int64_t)(post1 - post0) * npre;
    }
}

void or_rhs(const or_net *net, const double *y, const double *I_nA, double *f)
{
    int n = net->n;
    double cg = 1e-6 / net->area_cm2;   /* nS -> mS/cm^2 */
    double ci = 1e-3 / net->area_cm2;   /* nA -> uA/cm^2 */
    double *A = (double *)malloc(sizeof(double) * 3 * n);
    synaptic_sums(net, y, A);
    const double *kb = net->kin + T_GABA_B * NKIN;
    int gb = has_slow_gaba(net);
    for (int i = 0; i < n; ++i) {
        double V = y[YV * n + i], m = y[YM * n + i], h = y[YH * n + i];
        double nn = y[YN * n + i], s = y[YS * n + i];
        double r = y[YR * n + i], G = y[YG * n + i];
        const double *P = net->prm;
        double C = P[P_CM * n + i];
        double INa = P[P_GNA * n + i] * m * m * m * h * (V - P[P_ENA * n + i]);
        double IK = P[P_GK * n + i] * nn * nn * nn * nn * (V - P[P_EK * n + i]);
        double IL = P[P_GL * n + i] * (V - P[P_EL * n + i]);
        double Isyn = 0.0;
        for (int t = 0; t < 3; ++t)
            Isyn += (V - net->kin[t * NKIN + K_EREV]) * cg * A[t * n + i];
        double rt[6];
        or_rates(V, rt);
        f[YV * n + i] = (ci * I_nA[i] - INa - IK - IL - Isyn) / C;
        f[YM * n + i] = rt[0] * (1.0 - m) - rt[1] * m;
        f[YH * n + i] = rt[2] * (1.0 - h) - rt[3] * h;
        f[YN * n + i] = rt[4] * (1.0 - nn) - rt[5] * nn;
        const double *k = own_kin(net, i);
        double T = release(V, k);
        f[YS * n + i] = k[K_ALPHA] * T * (1.0 - s) - k[K_BETA] * s;
        if (gb && i >= net->n_pn) {
            double TB = release(V, kb);
            f[YR * n + i] = kb[K_R1] * TB * (1.0 - r) - kb[K_R2] * r;
            f[YG * n + i] = kb[K_R3] * r - kb[K_R4] * G;
        } else {
            f[YR * n + i] = 0.0;
            f[YG * n + i] = 0.0;
        }
    }
    free(A);
}

/* gates at steady state for V0; synaptic variables at zero */
void or_init(const or_net *net, const double *v0, double *y)
{
    int n = net->n;
    memset(y, 0, sizeof(double) * NVAR * n);
    for (int i = 0; i < n; ++i) {
        double rt[6];
        or_rates(v0[i], rt);
        y[YV * n + i] = v0[i];
        y[YM * n + i] = rt[0] / (rt[0] + rt[1]);
        y[YH * n + i] = rt[2] / (rt[2] + rt[3]);
        y[YN * n + i] = rt[4] / (rt[4] + rt[5]);
    }
}

/* ---------------------------------------------------------------------- */
/* RK4 scan                                                                */
/* ---------------------------------------------------------------------- */

/* Butcher tableau of an explicit method with up to 4 stages.  RK4 is
 * c = (0, 1/2, 1/2, 1), a_{s,s-1} = c_s, b = (1, 2, 2, 1)/6; forward Euler is
 * one stage with b = (1). */
typedef struct { int stages; double a[4][4]; double b[4]; } tableau;

static tableau rk4_tab(void)
{
    tableau t;
    memset(&t, 0, sizeof t);
    t.stages = 4;
    t.a[1][0] = 0.5; t.a[2][1] = 0.5; t.a[3][2] = 1.0;
    t.b[0] = 1.0 / 6.0; t.b[1] = 2.0 / 6.0; t.b[2] = 2.0 / 6.0; t.b[3] = 1.0 / 6.0;
    return t;
}

static tableau euler_tab(void)
{
    tableau t;
    memset(&t, 0, sizeof t);
    t.stages = 1;
    t.b[0] = 1.0;
    return t;
}

/* One explicit Runge-Kutta step y <- y + dt sum_s b_s k_s. */
static void rk_step(const or_net *net, const tableau *tb, double *y,
                    const double *I, double dt, double *work)
{
    int W = NVAR * net->n;
    double *k = work;            /* [4][W] */
    double *Y = work + 4 * W;    /* [W] */
    for (int s = 0; s < tb->stages; ++s) {
        for (int w = 0; w < W; ++w) {
            double v = y[w];
            for (int q = 0; q < s; ++q) v += dt * tb->a[s][q] * k[q * W + w];
            Y[w] = v;
        }
        or_rhs(net, Y, I, k + s * W);
    }
    for (int w = 0; w < W; ++w) {
        double inc = 0.0;
        for (int s = 0; s < tb->stages; ++s) inc += tb->b[s] * k[s * W + w];
        y[w] += dt * inc;
    }
}

static int integrate_tab(const or_net *net, const tableau *tb, double *y,
                         const or_stim *st, double dt, int64_t n_steps,
                         int64_t step0, int64_t rec_stride, int64_t rec_cap,
                         double *v_out, int32_t spike_cap, int32_t *spike_count,
                         double *spike_t)
{
    int n = net->n;
    int W = NVAR * n;
    double *work = (double *)malloc(sizeof(double) * 5 * W);
    double *I = (double *)malloc(sizeof(double) * n);
    double *vold = (double *)malloc(sizeof(double) * n);
    int64_t rows = 0;
    for (int64_t s = 0; s < n_steps; ++s) {
        int64_t g = step0 + s;    /* global index of the step's start t_g */
        for (int i = 0; i < n; ++i) I[i] = stim_nA(st, i, g);
        memcpy(vold, y, sizeof(double) * n);
        rk_step(net, tb, y, I, dt, work);
        if (spike_count) {
            for (int i = 0; i < n; ++i) {
                double a = vold[i], b = y[YV * n + i];
                if (a < 0.0 && b >= 0.0) {
                    int32_t c = spike_count[i];
                    if (c < spike_cap && spike_t)
                        spike_t[(int64_t)i * spike_cap + c] = ((double)g + (0.0 - a) / (b - a)) * dt;
                    spike_count[i] = c + 1;
                }
            }
        }
        if (v_out && rec_stride > 0 && (g + 1) % rec_stride == 0) {
            if (rows < rec_cap)
                memcpy(v_out + rows * n, y, sizeof(double) * n);
            rows++;
        }
    }
    free(work); free(I); free(vold);
    return 0;
}

int or_integrate(const or_net *net, double *y, const or_stim *st, double dt,
                 int64_t n_steps, int64_t step0, int64_t rec_stride,
                 int64_t rec_cap, double *v_out, int32_t spike_cap,
                 int32_t *spike_count, double *spike_t)
{
    tableau tb = rk4_tab();
    return integrate_tab(net, &tb, y, st, dt, n_steps, step0, rec_stride,
                         rec_cap, v_out, spike_cap, spike_count, spike_t);
}

/* Any explicit tableau of up to 4 stages: a is 4 x 4 row-major (only
 * a[s][q], q < s, is read), b has 4 entries. */
int or_integrate_tab(const or_net *net, double *y, const or_stim *st, double dt,
                     int64_t n_steps, int64_t step0, int64_t rec_stride,
                     int64_t rec_cap, double *v_out, int32_t spike_cap,
                     int32_t *spike_count, double *spike_t, int32_t stages,
                     const double *a, const double *b)
{
    tableau tb;
    memset(&tb, 0, sizeof tb);
    if (stages < 1 || stages > 4) return -1;
    tb.stages = stages;
    for (int i = 0; i < stages; ++i) {
        for (int q = 0; q < i; ++q) tb.a[i][q] = a[4 * i + q];
        tb.b[i] = b[i];
    }
    return integrate_tab(net, &tb, y, st, dt, n_steps, step0, rec_stride,
                         rec_cap, v_out, spike_cap, spike_count, spike_t);
}

int or_integrate_euler(const or_net *net, double *y, const or_stim *st,
                       double dt, int64_t n_steps, int64_t step0,
                       int64_t rec_stride, int64_t rec_cap, double *v_out)
{
    tableau tb = euler_tab();
    return integrate_tab(net, &tb, y, st, dt, n_steps, step0, rec_stride,
                         rec_cap, v_out, 0, NULL, NULL);
}

/* ---------------------------------------------------------------------- */
/* Per-synapse form: one gate s_ij per synapse (the n x n arrangement of    */
/* synaptic variables), first-order types only.  Used to check that the     */
/* per-presynaptic gate s_j is the same dynamics: ds_ij/dt depends only on  */
/* V_j and s_ij, so equal initial values stay equal.                        */
/* ---------------------------------------------------------------------- */

int or_integrate_persyn(const or_net *net, double *y, const or_stim *st,
                        double dt, int64_t n_steps, int64_t step0,
                        double *v_out)
{
    int n = net->n;
    double cg = 1e-6 / net->area_cm2, ci = 1e-3 / net->area_cm2;
    for (int p = 0; p < net->n_path; ++p)
        if (net->pinfo[5 * p] == T_GABA_B) return -1;
    int64_t ng = path_offset(net, net->n_path);
    int64_t W = 4 * (int64_t)n + ng;     /* V, m, h, n then one s per entry */
    double *z = (double *)calloc(W, sizeof(double));
    double *k = (double *)malloc(sizeof(double) * 4 * W);
    double *Z = (double *)malloc(sizeof(double) * W);
    double *I = (double *)malloc(sizeof(double) * n);
    memcpy(z, y, sizeof(double) * 4 * n);
    for (int p = 0, off = 0; p < net->n_path; ++p) {   /* s_ij(0) = s_j(0) */
        const int32_t *pi = net->pinfo + 5 * p;
        for (int i = pi[3]; i < pi[4]; ++i)
            for (int j = pi[1]; j < pi[2]; ++j)
                z[4 * n + off + (i - pi[3]) * (pi[2] - pi[1]) + (j - pi[1])] = y[YS * n + j];
        off += (pi[4] - pi[3]) * (pi[2] - pi[1]);
    }
    const double cs[4] = {0.0, 0.5, 0.5, 1.0};
    const double bw[4] = {1.0 / 6, 2.0 / 6, 2.0 / 6, 1.0 / 6};
    for (int64_t s = 0; s < n_steps; ++s) {
        int64_t gidx = step0 + s;
        for (int i = 0; i < n; ++i) I[i] = stim_nA(st, i, gidx);
        for (int st_ = 0; st_ < 4; ++st_) {
            for (int64_t w = 0; w < W; ++w)
                Z[w] = z[w] + (st_ ? dt * cs[st_] * k[(st_ - 1) * W + w] : 0.0);
            double *f = k + st_ * W;
            for (int i = 0; i < n; ++i) {
                double V = Z[i], m = Z[n + i], h = Z[2 * n + i], nn = Z[3 * n + i];
                const double *P = net->prm;
                double rt[6];
                or_rates(V, rt);
                double Isyn = 0.0;
                int64_t off = 0;
                for (int p = 0; p < net->n_path; ++p) {
                    const int32_t *pi = net->pinfo + 5 * p;
                    int npre = pi[2] - pi[1];
                    if (i >= pi[3] && i < pi[4]) {
                        double acc = 0.0;
                        for (int j = pi[1]; j < pi[2]; ++j) {
                            int64_t e = off + (int64_t)(i - pi[3]) * npre + (j - pi[1]);
                            acc += net->g[e] * Z[4 * n + e];
                        }
                        Isyn += (V - net->kin[pi[0] * NKIN + K_EREV]) * cg * acc;
                    }
                    off += (int64_t)(pi[4] - pi[3]) * npre;
                }
                f[i] = (ci * I[i] - P[P_GNA * n + i] * m * m * m * h * (V - P[P_ENA * n + i])
                        - P[P_GK * n + i] * nn * nn * nn * nn * (V - P[P_EK * n + i])
                        - P[P_GL * n + i] * (V - P[P_EL * n + i]) - Isyn) / P[P_CM * n + i];
                f[n + i] = rt[0] * (1 - m) - rt[1] * m;
                f[2 * n + i] = rt[2] * (1 - h) - rt[3] * h;
                f[3 * n + i] = rt[4] * (1 - nn) - rt[5] * nn;
            }
            int64_t off = 0;
            for (int p = 0; p < net->n_path; ++p) {
                const int32_t *pi = net->pinfo + 5 * p;
                const double *kk = net->kin + pi[0] * NKIN;
                for (int i = pi[3]; i < pi[4]; ++i)
                    for (int j = pi[1]; j < pi[2]; ++j) {
                        int64_t e = off + (int64_t)(i - pi[3]) * (pi[2] - pi[1]) + (j - pi[1]);
                        double T = release(Z[j], kk);
                        double sij = Z[4 * n + e];
                        f[4 * n + e] = kk[K_ALPHA] * T * (1 - sij) - kk[K_BETA] * sij;
                    }
                off += (int64_t)(pi[4] - pi[3]) * (pi[2] - pi[1]);
            }
        }
        for (int64_t w = 0; w < W; ++w)
            z[w] += dt * (bw[0] * k[w] + bw[1] * k[W + w] + bw[2] * k[2 * W + w] + bw[3] * k[3 * W + w]);
        if (v_out) memcpy(v_out + s * n, z, sizeof(double) * n);
    }
    memcpy(y, z, sizeof(double) * 4 * n);
    free(z); free(k); free(Z); free(I);
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Discrete adjoint of the RK4 map                                         */
/* ---------------------------------------------------------------------- */
/*
 * Loss L depends on the recorded potentials V_n (n = 1..n_steps, the state
 * after step n); dLdV[(n-1) * n_neurons + i] = dL/dV_{n,i}.  The gradient is
 * that of the discrete forward map (differentiate the RK4 recursion), so it
 * agrees with finite differences of or_integrate to O(h^2).
 *
 * VJP of f at Y with cotangent w: u = J(Y)^T w, and parameter cotangents
 * accumulated into gg (pathway blocks, nS), gna/gk/gl (mS/cm^2).
 */
static void rhs_vjp(const or_net *net, const double *Y, const double *w,
                    double *u, double *gg, double *gna, double *gk, double *gl)
{
    int n = net->n;
    double cg = 1e-6 / net->area_cm2;
    const double *P = net->prm;
    const double *kb = net->kin + T_GABA_B * NKIN;
    double *A = (double *)malloc(sizeof(double) * 3 * n);
    double *q = (double *)malloc(sizeof(double) * 3 * n);  /* dI_syn weights */
    synaptic_sums(net, Y, A);
    int gb = has_slow_gaba(net);
    memset(u, 0, sizeof(double) * NVAR * n);
    for (int i = 0; i < n; ++i) {
        double V = Y[YV * n + i], m = Y[YM * n + i], h = Y[YH * n + i];
        double nn = Y[YN * n + i], s = Y[YS * n + i], r = Y[YR * n + i];
        double C = P[P_CM * n + i];
        double wV = w[YV * n + i];
        double rt[6], rd[6];
        or_rates(V, rt);
        rates_d(V, rt, rd);
        double gsum = P[P_GNA * n + i] * m * m * m * h + P[P_GK * n + i] * nn * nn * nn * nn
                      + P[P_GL * n + i];
        for (int t = 0; t < 3; ++t) gsum += cg * A[t * n + i];
        double uV = wV * (-gsum / C);
        uV += w[YM * n + i] * (rd[0] * (1 - m) - rd[1] * m);
        uV += w[YH * n + i] * (rd[2] * (1 - h) - rd[3] * h);
        uV += w[YN * n + i] * (rd[4] * (1 - nn) - rd[5] * nn);
        const double *k = own_kin(net, i);
        double T = release(V, k);
        uV += w[YS * n + i] * k[K_ALPHA] * (T * (1 - T) / k[K_KP]) * (1 - s);
        u[YS * n + i] += w[YS * n + i] * (-(k[K_ALPHA] * T + k[K_BETA]));
        if (gb && i >= net->n_pn) {
            double TB = release(V, kb);
            uV += w[YR * n + i] * kb[K_R1] * (TB * (1 - TB) / kb[K_KP]) * (1 - r);
            u[YR * n + i] += w[YR * n + i] * (-(kb[K_R1] * TB + kb[K_R2])) + w[YG * n + i] * kb[K_R3];
            u[YG * n + i] += w[YG * n + i] * (-kb[K_R4]);
        }
        u[YV * n + i] += uV;
        double ENa = P[P_ENA * n + i], EK = P[P_EK * n + i];
        u[YM * n + i] += wV * (-3.0 * P[P_GNA * n + i] * m * m * h * (V - ENa) / C)
                         - w[YM * n + i] * (rt[0] + rt[1]);
        u[YH * n + i] += wV * (-P[P_GNA * n + i] * m * m * m * (V - ENa) / C)
                         - w[YH * n + i] * (rt[2] + rt[3]);
        u[YN * n + i] += wV * (-4.0 * P[P_GK * n + i] * nn * nn * nn * (V - EK) / C)
                         - w[YN * n + i] * (rt[4] + rt[5]);
        gna[i] += wV * (-m * m * m * h * (V - ENa) / C);
        gk[i] += wV * (-nn * nn * nn * nn * (V - EK) / C);
        gl[i] += wV * (-(V - P[P_EL * n + i]) / C);
        for (int t = 0; t < 3; ++t)
            q[t * n + i] = wV * (-(V - net->kin[t * NKIN + K_EREV]) * cg / C);
    }
    int64_t off = 0;
    for (int p = 0; p < net->n_path; ++p) {
        const int32_t *pi = net->pinfo + 5 * p;
        int t = pi[0], pre0 = pi[1], pre1 = pi[2], post0 = pi[3], post1 = pi[4];
        int npre = pre1 - pre0;
        const double *g = net->g + off;
        for (int i = post0; i < post1; ++i)
            for (int j = pre0; j < pre1; ++j) {
                int64_t e = (int64_t)(i - post0) * npre + (j - pre0);
                double x = activation(net, Y, t, j);
                gg[off + e] += q[t * n + i] * x;
                double dx = (t == T_GABA_B) ? gabab_act_d(Y[YG * n + j], kb) : 1.0;
                u[(t == T_GABA_B ? YG : YS) * n + j] += q[t * n + i] * g[e] * dx;
            }
        off += (int64_t)(post1 - post0) * npre;
    }
    free(A); free(q);
}

int or_adjoint(const or_net *net, const double *y0, const or_stim *st,
               double dt, int64_t n_steps, int64_t step0, const double *dLdV,
               double *grad_g, double *grad_gna, double *grad_gk,
               double *grad_gl, double *lambda0)
{
    int n = net->n;
    int64_t W = NVAR * (int64_t)n;
    int64_t ng = path_offset(net, net->n_path);
    double *traj = (double *)malloc(sizeof(double) * W * (n_steps > 0 ? n_steps : 1));
    double *work = (double *)malloc(sizeof(double) * 5 * W);
    double *I = (double *)malloc(sizeof(double) * n);
    double *y = (double *)malloc(sizeof(double) * W);
    tableau tb = rk4_tab();
    memcpy(y, y0, sizeof(double) * W);
    for (int64_t s = 0; s < n_steps; ++s) {       /* forward, keep y_n */
        memcpy(traj + s * W, y, sizeof(double) * W);
        for (int i = 0; i < n; ++i) I[i] = stim_nA(st, i, step0 + s);
        rk_step(net, &tb, y, I, dt, work);
    }
    memset(grad_g, 0, sizeof(double) * (ng > 0 ? ng : 1));
    memset(grad_gna, 0, sizeof(double) * n);
    memset(grad_gk, 0, sizeof(double) * n);
    memset(grad_gl, 0, sizeof(double) * n);
    double *lam = (double *)calloc(W, sizeof(double));
    double *Ys = (double *)malloc(sizeof(double) * 4 * W);  /* stage states */
    double *k = (double *)malloc(sizeof(double) * 4 * W);
    double *kb = (double *)malloc(sizeof(double) * W);      /* k-bar of a stage */
    double *u = (double *)malloc(sizeof(double) * 4 * W);
    const double c[4] = {0.0, 0.5, 0.5, 1.0};
    const double b[4] = {1.0 / 6, 2.0 / 6, 2.0 / 6, 1.0 / 6};
    for (int64_t s = n_steps - 1; s >= 0; --s) {
        for (int i = 0; i < n; ++i) lam[YV * n + i] += dLdV[s * n + i];
        const double *yn = traj + s * W;
        for (int i = 0; i < n; ++i) I[i] = stim_nA(st, i, step0 + s);
        for (int q = 0; q < 4; ++q) {             /* recompute the stages */
            for (int64_t w = 0; w < W; ++w)
                Ys[q * W + w] = yn[w] + (q ? dt * c[q] * k[(q - 1) * W + w] : 0.0);
            or_rhs(net, Ys + q * W, I, k + q * W);
        }
        /* Y_{q} = y + dt c_q k_{q-1};  y' = y + dt sum b_q k_q.
         * kbar_q = dt b_q lam' + dt c_{q+1} u_{q+1}, u_q = J(Y_q)^T kbar_q. */
        for (int q = 3; q >= 0; --q) {
            for (int64_t w = 0; w < W; ++w)
                kb[w] = dt * b[q] * lam[w] + (q < 3 ? dt * c[q + 1] * u[(q + 1) * W + w] : 0.0);
            rhs_vjp(net, Ys + q * W, kb, u + q * W, grad_g, grad_gna, grad_gk, grad_gl);
        }
        for (int64_t w = 0; w < W; ++w)
            lam[w] += u[w] + u[W + w] + u[2 * W + w] + u[3 * W + w];
    }
    if (lambda0) memcpy(lambda0, lam, sizeof(double) * W);
    free(traj); free(work); free(I); free(y); free(lam); free(Ys); free(k);
    free(kb); free(u);
    return 0;
}

/*
 * Discrete adjoint of any explicit tableau (up to 4 stages).  Stage inputs
 * Y_s = y + dt sum_{q<s} a_{sq} k_q, k_s = f(Y_s), y' = y + dt sum_s b_s k_s.
 * With lam = dL/dy', going through the stages last to first:
 *   kbar_s = dt b_s lam + dt sum_{r>s} a_{rs} u_r,   u_s = J(Y_s)^T kbar_s,
 * and dL/dy = lam + sum_s u_s; parameter cotangents collect
 * (df/dtheta)(Y_s)^T kbar_s.  For RK4 (a_{s,s-1} = c_s only) this is the
 * recursion of or_adjoint above.
 */
int or_adjoint_tab(const or_net *net, const double *y0, const or_stim *st,
                   double dt, int64_t n_steps, int64_t step0, const double *dLdV,
                   double *grad_g, double *grad_gna, double *grad_gk,
                   double *grad_gl, double *lambda0, int32_t stages,
                   const double *a, const double *b)
{
    if (stages < 1 || stages > 4) return -1;
    tableau tb;
    memset(&tb, 0, sizeof tb);
    tb.stages = stages;
    for (int i = 0; i < stages; ++i) {
        for (int q = 0; q < i; ++q) tb.a[i][q] = a[4 * i + q];
        tb.b[i] = b[i];
    }
    int n = net->n;
    int64_t W = NVAR * (int64_t)n;
    int64_t ng = path_offset(net, net->n_path);
    double *traj = (double *)malloc(sizeof(double) * W * (n_steps > 0 ? n_steps : 1));
    double *work = (double *)malloc(sizeof(double) * 5 * W);
    double *I = (double *)malloc(sizeof(double) * n);
    double *y = (double *)malloc(sizeof(double) * W);
    memcpy(y, y0, sizeof(double) * W);
    for (int64_t s = 0; s < n_steps; ++s) {
        memcpy(traj + s * W, y, sizeof(double) * W);
        for (int i = 0; i < n; ++i) I[i] = stim_nA(st, i, step0 + s);
        rk_step(net, &tb, y, I, dt, work);
    }
    memset(grad_g, 0, sizeof(double) * (ng > 0 ? ng : 1));
    memset(grad_gna, 0, sizeof(double) * n);
    memset(grad_gk, 0, sizeof(double) * n);
    memset(grad_gl, 0, sizeof(double) * n);
    double *lam = (double *)calloc(W, sizeof(double));
    double *Ys = (double *)malloc(sizeof(double) * 4 * W);
    double *k = (double *)malloc(sizeof(double) * 4 * W);
    double *kb = (double *)malloc(sizeof(double) * W);
    double *u = (double *)malloc(sizeof(double) * 4 * W);
    for (int64_t s = n_steps - 1; s >= 0; --s) {
        for (int i = 0; i < n; ++i) lam[YV * n + i] += dLdV[s * n + i];
        const double *yn = traj + s * W;
        for (int i = 0; i < n; ++i) I[i] = stim_nA(st, i, step0 + s);
        for (int q = 0; q < stages; ++q) {
            for (int64_t w = 0; w < W; ++w) {
                double v = yn[w];
                for (int r = 0; r < q; ++r) v += dt * tb.a[q][r] * k[r * W + w];
                Ys[q * W + w] = v;
            }
            or_rhs(net, Ys + q * W, I, k + q * W);
        }
        for (int q = stages - 1; q >= 0; --q) {
            for (int64_t w = 0; w < W; ++w) {
                double v = dt * tb.b[q] * lam[w];
                for (int r = q + 1; r < stages; ++r) v += dt * tb.a[r][q] * u[r * W + w];
                kb[w] = v;
            }
            rhs_vjp(net, Ys + q * W, kb, u + q * W, grad_g, grad_gna, grad_gk, grad_gl);
        }
        for (int64_t w = 0; w < W; ++w)
            for (int q = 0; q < stages; ++q) lam[w] += u[q * W + w];
    }
    if (lambda0) memcpy(lambda0, lam, sizeof(double) * W);
    free(traj); free(work); free(I); free(y); free(lam); free(Ys); free(k);
    free(kb); free(u);
    return 0;
}

/* Jacobian-transpose of one RK4 step applied to a cotangent: lam_in is
 * dL/dy_{n+1}, result is dL/dy_n (no parameter gradients kept).  Used by the
 * transpose identity test <J v, w> = <v, J^T w>. */
int or_step_vjp(const or_net *net, const double *yn, const double *I,
                double dt, const double *lam_in, double *lam_out)
{
    int n = net->n;
    int64_t W = NVAR * (int64_t)n;
    int64_t ng = path_offset(net, net->n_path);
    double *Ys = (double *)malloc(sizeof(double) * 4 * W);
    double *k = (double *)malloc(sizeof(double) * 4 * W);
    double *kb = (double *)malloc(sizeof(double) * W);
    double *u = (double *)malloc(sizeof(double) * 4 * W);
    double *gg = (double *)calloc(ng > 0 ? ng : 1, sizeof(double));
    double *g3 = (double *)calloc(3 * n, sizeof(double));
    const double c[4] = {0.0, 0.5, 0.5, 1.0};
    const double b[4] = {1.0 / 6, 2.0 / 6, 2.0 / 6, 1.0 / 6};
    for (int q = 0; q < 4; ++q) {
        for (int64_t w = 0; w < W; ++w)
            Ys[q * W + w] = yn[w] + (q ? dt * c[q] * k[(q - 1) * W + w] : 0.0);
        or_rhs(net, Ys + q * W, I, k + q * W);
    }
    for (int q = 3; q >= 0; --q) {
        for (int64_t w = 0; w < W; ++w)
            kb[w] = dt * b[q] * lam_in[w] + (q < 3 ? dt * c[q + 1] * u[(q + 1) * W + w] : 0.0);
        rhs_vjp(net, Ys + q * W, kb, u + q * W, gg, g3, g3 + n, g3 + 2 * n);
    }
    for (int64_t w = 0; w < W; ++w)
        lam_out[w] = lam_in[w] + u[w] + u[W + w] + u[2 * W + w] + u[3 * W + w];
    free(Ys); free(k); free(kb); free(u); free(gg); free(g3);
    return 0;
}
