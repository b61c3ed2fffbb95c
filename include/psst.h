/*
 * psst.h -- C ABI of the MI355X (gfx950) engine for fixed-step fourth-order
 * Runge-Kutta integration of coupled Hodgkin-Huxley networks.
 *
 * The calls follow the paper's statement of the problem (Mohanta & Assisi,
 * "Parallel scalable simulations of biological neural networks using
 * TensorFlow"):
 *   - an initial value problem dy/dt = f(y, t), y(t0) = y0, integrated with
 *     the classical RK4 step ("Brain simulations as computational graphs",
 *     IVP equation and the RK4 paragraph);
 *   - a scan of that step over a time grid whose output rows are the states
 *     after each step, the initial value excluded (same section, the tf.scan
 *     cumulative-sum example);
 *   - per-neuron state [V, m, h, n] and per-neuron parameter vectors
 *     C_m, g_Na, g_K, g_L, E_Na, E_K, E_L in structure-of-arrays form (same
 *     section, vectorisation paragraph);
 *   - synaptic coupling as dense n x n conductance matrices per synapse type
 *     ("Circumventing memory constraints", item 1);
 *   - long runs split into successive batches of steps that resume from the
 *     carried state (same section, item 2).
 *
 * Conventions
 *   - Every call returns psst_status; no C++ exception crosses the ABI.  On
 *     failure psst_last_error() returns a thread-local description.
 *   - Arguments are validated on the host before any device call; invalid
 *     arguments never reach the GPU.
 *   - Ownership: handles (psst_network, psst_batch) and their device copies of
 *     parameters and conductances belong to the library.  State, stimulus,
 *     record, checkpoint and gradient buffers belong to the caller (device
 *     memory, e.g. from torch tensors); the library never frees them.
 *   - create/destroy/poll calls are synchronous; integrate and adjoint calls
 *     are asynchronous on the caller's HIP stream (NULL = default stream).
 *   - Environment variables, for comparisons and tests (defaults are the
 *     library's own choices): PSST_TUNE=0 and PSST_WG_SHAPE (batch and
 *     psst_integrate launch shapes, see there), PSST_LDS_G=0 (conductances
 *     never held in LDS: always streamed), PSST_LG=0 (small dense networks
 *     -- at most 128 neurons and 4 column chunks of 64 -- take the
 *     LDS-resident kernels instead of the one holding their conductances in
 *     registers; both give the same bits), PSST_RR=0 (the batch tuner never
 *     picks a variant holding leading conductance columns of larger
 *     networks in registers; same bits), PSST_ADJ_MODE=lacc|mma (how the
 *     adjoint accumulates dL/dg), PSST_ADJ_BS=64|128|256|512 (adjoint
 *     workgroup size, when it covers the batch's largest network),
 *     PSST_ADJ_PIPE=0 (the adjoint's recomputation on the caller's stream,
 *     not beside the reverse sweep on a second one; same bits),
 *     PSST_TUNE_FILE (path of the tuning table, default tuning/<arch>.txt
 *     beside the library), PSST_TUNE_WRITE=1 (a batch tuned on creation
 *     writes its choices to that table), PSST_TUNE_LOG=1 (the tuner prints
 *     its timings to stderr).
 *   - A handle holds per-handle device state (control blocks, graphs,
 *     workspaces, error flags): calls on one network or batch must be issued
 *     from one host thread at a time and on one stream, or the caller orders
 *     them; different handles are independent.
 *   - Units: mV, ms, nS (synaptic g), nA (injected current), uF/cm^2, mS/cm^2
 *     (intrinsic g).  With membrane area A (cm^2), 1 nS = 1e-6/A mS/cm^2 and
 *     1 nA = 1e-3/A uA/cm^2.
 *
 * Numerics: conductances are kept as the float32 values given; the
 * per-neuron right-hand side (rate functions, currents, gating ODEs), the RK4
 * stage arithmetic and the synaptic sums sum_j g_ij x_j run in float64 (each
 * product of a float32 g and a float64 activation is exact before the sum);
 * each state variable is stored as a float32 pair (value, compensation) whose
 * sum is the state after every step, rounded to 48 significant bits.  Large
 * shared networks on the per-stage path (more than 1024 neurons) take float32
 * activations and the synaptic sums from a float32 matrix-core GEMM: float32
 * sums over groups of 32 presynaptic columns, the group sums added in
 * float64 (with dense or sparse storage alike).
 */
#ifndef PSST_H
#define PSST_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PSST_OK = 0,
    PSST_ERR_INVALID_ARGUMENT = 1,  /* a pointer, size, range or value is invalid */
    PSST_ERR_OUT_OF_MEMORY = 2,     /* a device or host allocation failed */
    PSST_ERR_DEVICE = 3,            /* no usable gfx950 device, or a HIP call failed */
    PSST_ERR_NONFINITE = 4,         /* a state variable became NaN or infinite */
    PSST_ERR_UNSUPPORTED = 5        /* valid request the library does not implement */
} psst_status;

/* Thread-local text describing the last failure of a call on this thread. */
const char *psst_last_error(void);

/* Library version string. */
const char *psst_version(void);

/* Number of visible HIP devices (0 when none); never fails. */
int32_t psst_device_count(void);

/* ------------------------------------------------------------------------ */
/* Networks                                                                  */
/* ------------------------------------------------------------------------ */

typedef struct psst_network psst_network;   /* opaque, library-owned */
typedef struct psst_batch psst_batch;       /* opaque, library-owned */

typedef enum { PSST_SYN_ACH = 0, PSST_SYN_GABA_A = 1, PSST_SYN_GABA_B = 2 } psst_syn_type;

/* Per-neuron parameter vectors (host pointers, length n_neurons each).
 * Neurons [0, n_pn) are projection neurons (PN, cholinergic output),
 * [n_pn, n) local neurons (LN, GABAergic output). */
typedef struct {
    const float *C_m, *g_Na, *g_K, *g_L;    /* uF/cm^2, mS/cm^2 */
    const float *E_Na, *E_K, *E_L;          /* mV */
    int32_t n_pn;
    float area_cm2;                         /* > 0 */
} psst_neuron_params;

/* One dense masked block of synapses of one type: g_nS[(i - post_begin) *
 * (pre_end - pre_begin) + (j - pre_begin)] is the conductance from
 * presynaptic j to postsynaptic i (row-major [post x pre], host memory).
 * Cholinergic blocks must have their presynaptic range inside the PN rows,
 * GABA blocks inside the LN rows; blocks of one type must not overlap.
 * mask (same shape, or NULL = all present): entries with mask == 0 are no
 * synapse; their g is ignored and their gradient is 0. */
typedef struct {
    int32_t type;                           /* psst_syn_type */
    int32_t pre_begin, pre_end, post_begin, post_end;
    const float *g_nS;
    const uint8_t *mask;
} psst_pathway;

/* Synapse kinetics per type (index = psst_syn_type).
 * Release T(V_pre) = 1 / (1 + exp(-(V_pre - V_p) / K_p)).
 * ACh, GABA_A: ds/dt = alpha T (1 - s) - beta s, activation x = s.
 * GABA_B:      dr/dt = r1 T (1 - r) - r2 r, dG/dt = r3 r - r4 G,
 *              activation x = G^n / (G^n + K_d), n = hill_n (integer 1..8).
 * Current onto i: sum over types of (V_i - E_rev) * sum_j g_ij x_j. */
typedef struct {
    float alpha, beta, E_rev, V_p, K_p;
    float r1, r2, r3, r4, K_d, hill_n;
} psst_kinetics;

/* Build a network and upload its parameters and conductance matrices to the
 * current HIP device.  All pointers are host pointers and are only read
 * during the call.  n_neurons in [1, 1 << 20]; n_pathways in [0, 64].
 * Errors: INVALID_ARGUMENT (checked before any device call), DEVICE,
 * OUT_OF_MEMORY. */
psst_status psst_network_create(const psst_neuron_params *params, int32_t n_neurons,
                                const psst_pathway *pathways, int32_t n_pathways,
                                const psst_kinetics kinetics[3], psst_network **out);
psst_status psst_network_destroy(psst_network *net);

/* Storage of the conductance matrices ("Circumventing memory constraints",
 * item 1: sparse matrices where connectivity is low).  DENSE keeps every
 * [post x pre] entry (zeros included) and reads each once per stage.
 * SPARSE, on the per-instance path (at most 1024 neurons), keeps per
 * postsynaptic neuron its present synapses sorted by presynaptic index, so a
 * stage reads 8 bytes per synapse instead of 4 bytes per matrix entry; both
 * sum the products in the same fixed order (64-column chunks in column
 * order, partials in chunk order; absent synapses add exact zeros), so the
 * two give the same trajectory bit for bit.  SPARSE above 1024 neurons (the
 * per-stage path, networks shared by trials) keeps the synapses grouped by
 * postsynaptic row and 128-column tile (a float32 value per synapse; per row
 * and tile a start offset and a 128-bit column mask, 20 bytes), read once
 * per stage and tile of 64 trials; each stage builds the dense conductance
 * tiles from them in LDS and feeds the same matrix-core products as DENSE,
 * so the two give the same trajectory bit for bit: SPARSE saves HBM, not
 * time.  AUTO picks SPARSE when at most a quarter of the pathway entries are
 * synapses, and above 1024 neurons only when the dense per-stage matrix
 * would take more than 16 GiB. */
typedef enum {
    PSST_STORAGE_AUTO = 0,
    PSST_STORAGE_DENSE = 1,
    PSST_STORAGE_SPARSE = 2
} psst_storage;

/* psst_network_create with a storage choice (psst_network_create = AUTO).
 * A sparse
 * network of at most 512 neurons (the adjoint's limit) also keeps the dense
 * transposed matrices and the synapse mask on the device (5 bytes per
 * matrix entry) for psst_adjoint's transposed products and gradient mask;
 * its forward reads only the sparse rows, and its adjoint equals that of the
 * same network stored dense bit for bit. */
psst_status psst_network_create_storage(const psst_neuron_params *params, int32_t n_neurons,
                                        const psst_pathway *pathways, int32_t n_pathways,
                                        const psst_kinetics kinetics[3], int32_t storage,
                                        psst_network **out);

/* State layout: 7 variables (V, m, h, n, s, r, G) x 2 float32 words (value,
 * compensation), plane-major: word (2 * var + c) * n_total + i.  n_words =
 * 14 * n_neurons for a network.  s is the neuron's own outgoing transmitter
 * gate (ACh for PN, fast GABA for LN); r, G are the slow-GABA pair of LN rows
 * (zero and unused for PN rows or networks without slow GABA). */
psst_status psst_state_layout(const psst_network *net, int64_t *n_words, int32_t *n_vars);

/* Initial state from v0 (device, [n] mV): gates at their steady state for
 * v0, synaptic variables 0, compensation words 0.  state: device
 * [n_words] float32, written.  Asynchronous on stream. */
psst_status psst_state_init(const psst_network *net, const float *v0, float *state,
                            void *hip_stream);

/* Injected current (device pointers, nA), indexed by neuron (packed over all
 * instances for a batch: n_total entries): i_const (or NULL = 0) plus
 * pulses; neuron k owns pulses pulse_ptr[k] .. pulse_ptr[k+1]-1 (pulse_ptr
 * NULL = no pulses), each on during global steps on_step <= g < off_step.
 * The current is held constant over each step (zero-order hold). */
typedef struct {
    const float *i_const_nA;
    const int32_t *pulse_ptr;
    const int64_t *on_step, *off_step;
    const float *amp_nA;
} psst_stimulus;

/* Recording (device pointers; any member may be NULL/0 to skip it).
 * v_out [capacity x n_total] float32: row r holds V of every neuron after
 * global step g + 1 = (step0 / stride + 1 + r) * stride, i.e. every stride-th
 * state after the call's first step (the initial state is not a row); rows
 * beyond capacity are dropped.
 * spike_count [n_total] int32 (in/out, incremented) and spike_t_ms
 * [n_total x spike_cap] float32: upward crossings of 0 mV, V_g < 0 <= V_g+1,
 * at time (g + (0 - V_g) / (V_g+1 - V_g)) * dt; spikes beyond spike_cap are
 * counted but not stored. */
typedef struct {
    float *v_out;
    int64_t stride, capacity;
    int32_t *spike_count;
    float *spike_t_ms;
    int32_t spike_cap;
} psst_record;

/* Integrate one network (the plain one-network-per-launch form; the RK4 step
 * of "Brain simulations as computational graphs" iterated as a scan over the
 * time grid, long runs resumed batch by batch per "Circumventing memory
 * constraints", item 2): n_steps steps of the network's method (classical RK4 unless
 * psst_network_set_tableau says otherwise) of size dt_ms from global step
 * index step0 (time t = step0 * dt), state in/out.  Calling it with
 * (n1, step0) then (n2, step0 + n1) gives bitwise the same state and records
 * as one call with n1 + n2.  stim, rec may be NULL.  n_steps >= 0, dt_ms > 0
 * and finite, step0 >= 0.  A network of at most 1024 neurons runs as one
 * persistent workgroup (its shape follows the network; the environment
 * variable PSST_WG_SHAPE="<threads>x<neurons per thread>" overrides it);
 * larger ones take the per-stage path with one trial (its workspace is
 * allocated by psst_network_create).  Errors: INVALID_ARGUMENT, DEVICE.
 * Non-finite states are reported by psst_network_poll. */
psst_status psst_integrate(psst_network *net, float *state, const psst_stimulus *stim,
                           float dt_ms, int64_t n_steps, int64_t step0,
                           const psst_record *rec, void *hip_stream);

/* Synchronize the stream and report (then clear) the non-finite flag set by
 * earlier integrate calls on this network: PSST_OK or PSST_ERR_NONFINITE. */
psst_status psst_network_poll(psst_network *net, void *hip_stream);

/* ------------------------------------------------------------------------ */
/* Batches: many independent instances in one launch                         */
/* ------------------------------------------------------------------------ */

/* Batch of n instances, integrated side by side like the independent ODEs of
 * the paper's Fig. 2b runtime comparison ("Motivation"), with the per-neuron
 * equations vectorised across all of them ("Brain simulations as
 * computational graphs", vectorisation paragraph); nets[b] may repeat
 * (trials of one network share its device conductances).  The batch keeps references: the networks must
 * outlive it.  Instance b owns neurons [off_b, off_b + n_b) of every packed
 * array, off_b = sum of the sizes of instances before b.  Instances are
 * grouped into launches by size class (neurons up to 192, 256, 320, 384,
 * 448, 512, 1024; small dense networks on their own kernel); creation tunes
 * each class's kernel variant -- threads per workgroup, neurons per thread,
 * conductance columns held in registers -- on the device (timing a few short
 * candidate runs) and merges neighbouring classes that choose the same
 * variant, unless the environment variable PSST_TUNE=0 (one launch, default
 * shape) or PSST_WG_SHAPE="<threads>x<neurons per thread>[r<register
 * slots>]" names the variant to use.  A class's choice is kept for the
 * process per (device architecture, size class, method, storage, slow GABA
 * present) and reused by later batches.  Networks above 1024 neurons take
 * the per-stage path: a batch whose instances all share one such network is
 * one per-stage launch sequence over its trials; in any other batch each run
 * of consecutive instances of one such network is a per-stage sub-batch of
 * its own (its trials side by side), run after the other instances' launches
 * on the same stream, in the same packed arrays.  Checkpoints and the
 * adjoint are not available for batches with per-stage instances
 * (UNSUPPORTED).  n in [1, 1 << 20]. */
psst_status psst_batch_create(psst_network *const *nets, int32_t n, psst_batch **out);
psst_status psst_batch_destroy(psst_batch *batch);

/* n_total = total neurons, n_words = 14 * n_total; offsets (host, may be
 * NULL) receives n + 1 neuron offsets. */
psst_status psst_batch_layout(const psst_batch *batch, int64_t *n_total, int64_t *n_words,
                              int64_t *offsets);

/* Packed initial state for every instance from v0 [n_total] (device). */
psst_status psst_batch_state_init(const psst_batch *batch, const float *v0, float *states,
                                  void *hip_stream);

/* Integrate every instance of the batch by n_steps (the RK4 scan of "Brain
 * simulations as computational graphs" for all instances in one launch; same
 * semantics as psst_integrate per instance; instance results are bitwise independent of
 * the batch's order and composition).  states, stim, rec are packed over
 * n_total neurons.  checkpoints: NULL, or device [n_steps / K + 1 x n_words]
 * float32 receiving the state before global steps step0 + c K (c = 0, 1,
 * ...), for psst_adjoint.  Submitted as one graph launch (plus the
 * per-stage sub-batches' step graphs, if any). */
psst_status psst_integrate_batch(psst_batch *batch, float *states, const psst_stimulus *stim,
                                 float dt_ms, int64_t n_steps, int64_t step0,
                                 const psst_record *rec, float *checkpoints, int32_t K,
                                 void *hip_stream);

psst_status psst_batch_poll(psst_batch *batch, void *hip_stream);

/* Text description of the tuned launch shape (for logs and benchmarks). */
psst_status psst_batch_describe(const psst_batch *batch, char *buf, int32_t buf_len);

/* Conductance bytes a forward launch of the batch reads, by the library's
 * own placement of the matrices (for roofline accounting; "Circumventing
 * memory constraints", item 1: the synaptic update is a product with the
 * conductance matrices, so these bytes are its operand traffic):
 * resident_bytes are read once per launch (the leading columns of every
 * conductance chunk kept in registers and LDS for the whole launch, an
 * instance's whole sparse rows, or a small network's whole matrices held in
 * registers),
 * streamed_bytes once per stage evaluation (the rest; on the
 * per-stage path of a large shared network, its whole padded matrix, or
 * with sparse storage every synapse value and every bucket's start and
 * column mask).  Trials
 * that share one network count once per workgroup that reads it.  Either
 * pointer may be NULL.  Synchronous, no device call. */
psst_status psst_batch_conductance_bytes(const psst_batch *batch, int64_t *resident_bytes,
                                         int64_t *streamed_bytes);

/* ------------------------------------------------------------------------ */
/* Discrete adjoint                                                          */
/* ------------------------------------------------------------------------ */

/* Gradients of a loss of the recorded potentials with respect to the synaptic
 * and intrinsic conductances, by reverse differentiation of the RK4 map (or
 * of the batch's explicit method, psst_batch_set_tableau).  Networks of at
 * most 512 neurons on the per-instance path, dense or sparse storage.
 * checkpoints: as written by psst_integrate_batch(..., K) for the same
 * stimulus, dt, n_steps and step0.  dL_dV: device [n_steps x n_total],
 * row k = dL/dV after global step step0 + k + 1.
 * grad_g: device, per instance the pathway blocks of its network in pathway
 * order, each [post x pre] (nS^-1 units of L), zero where there is no synapse;
 * grad_gNa, grad_gK, grad_gL: device per-neuron gradients (per mS/cm^2).
 * per_instance = 1: outputs are per instance (grad_g packed instance after
 * instance, per-neuron arrays [n_total]); per_instance = 0: all instances
 * must share one network and outputs hold the sum over instances
 * (grad_g [network's blocks], per-neuron arrays [n]).  Sums over time and
 * instances use compensated float32.  Outputs are overwritten.  The
 * batch's adjoint workspace (per instance K steps of stage records, float64)
 * is allocated on the first call and grown when a later call needs more;
 * calls that fit it allocate nothing.
 * Errors: INVALID_ARGUMENT, UNSUPPORTED, DEVICE, OUT_OF_MEMORY. */
psst_status psst_adjoint(psst_batch *batch, const float *checkpoints, int32_t K,
                         const psst_stimulus *stim, float dt_ms, int64_t n_steps,
                         int64_t step0, const float *dL_dV, float *grad_g, float *grad_gNa,
                         float *grad_gK, float *grad_gL, int32_t per_instance,
                         void *hip_stream);

/* psst_adjoint for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same arguments, kernels and results (bit for bit), but the stage
 * records, gradient accumulators and per-instance gradient offsets live in a
 * 64 MiB device array of the library (one per device, reserved when the
 * library's code loads on that device and held until the process ends)
 * instead of the batch's workspace.  The call allocates nothing, copies
 * nothing from the host and does not synchronize; it enqueues its kernels on
 * the stream.  It needs 8 * 60 * ld * K bytes of stage records per instance
 * (ld = the largest network's neuron count rounded up to 4), the largest
 * over the batch's networks of 8 * (n + n_LN + 3) * ld bytes of accumulators
 * per instance, and 8 bytes per instance, each part rounded up to 256 bytes: a request above 64 MiB is refused with
 * PSST_ERR_INVALID_ARGUMENT before any device call (use a smaller K, fewer
 * instances, or psst_adjoint).  Every call on a device shares that device's
 * array and leaves its contents behind: calls that overlap on one device
 * (different streams, or host threads) race and must be ordered by the
 * caller.  Errors: INVALID_ARGUMENT, UNSUPPORTED, DEVICE. */
psst_status psst_adjoint_noalloc(psst_batch *batch, const float *checkpoints, int32_t K,
                                 const psst_stimulus *stim, float dt_ms, int64_t n_steps,
                                 int64_t step0, const float *dL_dV, float *grad_g,
                                 float *grad_gNa, float *grad_gK, float *grad_gL,
                                 int32_t per_instance, void *hip_stream);

/* Number of float32 gradient entries one copy of the network's pathway blocks
 * occupies in grad_g. */
psst_status psst_network_grad_size(const psst_network *net, int64_t *n_entries);

/* New values of the parameters psst_adjoint differentiates, written into the
 * network's device storage where it lies, so that a descent loop keeps one
 * network and its batches instead of creating them again at every step (the
 * network is a computational graph built once and then evaluated with new
 * values, "Brain simulations as computational graphs"; the graph is fixed
 * before it runs, "Circumventing memory constraints", item 3).
 *   g: device [psst_network_grad_size] float32 in grad_g's layout (the
 *     pathway blocks in pathway order, each [post x pre] row-major), or NULL
 *     to keep the synaptic values; entries where the network has no synapse
 *     (mask 0 at creation) are ignored and stay zero;
 *   g_Na, g_K, g_L: device [n] float32 each (mS/cm^2), or NULL to keep.
 * Sizes, pathways, masks and storage stay those given to
 * psst_network_create; every storage the network keeps (dense, sparse rows,
 * the per-stage layout) is rewritten, so later integrate and adjoint calls
 * on the network, and on batches created from it before or after, use the
 * new values, bit for bit as a network created with them would.
 * Asynchronous: one kernel on hip_stream; allocates nothing and copies
 * nothing from the host.  Work on other streams that reads the network must
 * be ordered with it by the caller.  Values are not checked: non-finite ones
 * give non-finite states, which the polls report.
 * Errors: INVALID_ARGUMENT (NULL network), DEVICE. */
psst_status psst_network_update(psst_network *net, const float *g, const float *g_Na,
                                const float *g_K, const float *g_L, void *hip_stream);

/* ------------------------------------------------------------------------ */
/* Long runs streamed to host memory                                        */
/* ------------------------------------------------------------------------ */

/* psst_integrate_batch over n_steps in chunks of chunk_steps, the records of
 * every chunk drained to host memory while the next chunk integrates (the
 * paper's batches of time steps whose solution is moved off the device,
 * "Circumventing memory constraints", item 2): two device record buffers and
 * two pinned host staging buffers alternate; the GPU integrates chunk c + 1
 * on the caller's stream while chunk c is copied out on a second stream and
 * then into the caller's arrays by the host.  Device memory is bounded by two
 * chunks, whatever n_steps.
 *   host_v: host [n_steps / rec_stride][n_total] floats, V after every
 *     rec_stride-th step (rows as in psst_record), or NULL;
 *   host_spike_count: host [n_total] int32, spikes of the whole run (added to
 *     the values it holds), or NULL; host_spike_t: host
 *     [n_total][spike_cap] ms, each neuron's times appended after its
 *     existing count, those beyond spike_cap dropped (counted).
 * rec_stride must divide chunk_steps, and step0 must be a multiple of it.
 * Returns when every record is in host memory (the call is synchronous);
 * states holds the state after the last step.  Batches of a large shared
 * network (per-stage path) stream the same way.  Errors: INVALID_ARGUMENT,
 * OUT_OF_MEMORY, DEVICE, NONFINITE (checked once at the end). */
psst_status psst_integrate_batch_streamed(psst_batch *batch, float *states,
                                          const psst_stimulus *stim, float dt_ms,
                                          int64_t n_steps, int64_t step0, int64_t chunk_steps,
                                          int64_t rec_stride, float *host_v,
                                          int32_t *host_spike_count, float *host_spike_t,
                                          int32_t spike_cap, void *hip_stream);

/* ------------------------------------------------------------------------ */
/* Explicit Runge-Kutta tableaux                                             */
/* ------------------------------------------------------------------------ */

/* An explicit Runge-Kutta method of 1 to 4 stages, the family the classical
 * RK4 step belongs to ("Brain simulations as computational graphs", RK4
 * paragraph; the same section's IVP equation): stage inputs
 * Y_s = y + dt sum_{q<s} a[s][q] k_q, k_s = f(Y_s) with the injected current
 * held at t_n, and y' = y + dt sum_s b[s] k_s.  a must be strictly lower
 * triangular (a[s][q] = 0 for q >= s), and every a and b entry of an unused
 * stage (s >= stages) must be 0; all entries finite. */
typedef struct {
    int32_t stages;        /* 1..4 */
    double a[4][4];        /* a[s][q]: weight of k_q in stage s's input */
    double b[4];           /* weight of k_s in the step */
} psst_tableau;

/* Set the method used by psst_integrate on this network and inherited by
 * batches created from it afterwards.  NULL restores classical RK4; a tableau
 * equal to classical RK4 (a[1][0] = a[2][1] = 1/2, a[3][2] = 1,
 * b = 1/6, 1/3, 1/3, 1/6) is treated as NULL (same kernels, same bits).
 * Networks on the per-stage path (more than 1024 neurons) take one launch
 * per stage of the method.  Synchronous; errors: INVALID_ARGUMENT for a NULL
 * network or a tableau that breaks the rules above. */
psst_status psst_network_set_tableau(psst_network *net, const psst_tableau *tab);

/* The same for a batch: its integrate and adjoint calls use this method.
 * psst_batch_create takes the method of its networks, which must all agree
 * (else INVALID_ARGUMENT).  The adjoint needs a per-instance batch (the
 * per-stage path of a large network has none). */
psst_status psst_batch_set_tableau(psst_batch *batch, const psst_tableau *tab);

#ifdef __cplusplus
}
#endif

#endif /* PSST_H */
