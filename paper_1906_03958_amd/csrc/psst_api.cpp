// psst_api.cpp -- host runtime behind the C ABI in include/psst.h: argument
// validation, device copies of networks, batch packing and scheduling, graph
// submission and launch-shape tuning.
#include <dlfcn.h>
#include <hip/hip_runtime.h>
#include <sys/stat.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <set>
#include <sstream>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/psst.h"
#include "runtime.h"
#include "stage.h"

using namespace psst;

static thread_local std::string g_err;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------

psst_status psst::fail(psst_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

extern "C" const char *psst_last_error(void) { return g_err.c_str(); }
extern "C" const char *psst_version(void) { return "psst-mi355x 0.1 (gfx950)"; }

extern "C" int32_t psst_device_count(void)
{
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess) return 0;
    return n;
}

static psst_status check_device(int *dev_out)
{
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= 0)
        return fail(PSST_ERR_DEVICE, "no HIP device available");
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(PSST_ERR_DEVICE, "device %d is %s; this library is built for gfx950", dev,
                    prop.gcnArchName);
    *dev_out = dev;
    return PSST_OK;
}

static bool is_finite_f(float x) { return std::isfinite(x); }

static size_t max_lds_per_block();
static bool fits_wg(const psst_network *q);
static const int kMaxWGNeurons = 1024;   // largest network of the per-instance kernel
// dense per-stage matrices up to this size stay dense under AUTO (16 GiB, a
// network of about 65000 neurons)
static const int64_t kStageDenseAutoBytes = 16LL << 30;
static const int kMaxAdjointNeurons = 512;  // largest network of the adjoint

// ---------------------------------------------------------------------------
// networks
// ---------------------------------------------------------------------------

static void net_free(psst_network *n)
{
    if (!n) return;
    (void)hipFree(n->d_gt);
    (void)hipFree(n->d_gtb);
    (void)hipFree(n->d_prm);
    (void)hipFree(n->d_kin);
    (void)hipFree(n->d_maskt);
    (void)hipFree(n->d_desc);
    (void)hipFree(n->d_order);
    (void)hipFree(n->d_flag);
    (void)hipFree(n->d_paths);
    (void)hipFree(n->d_spcol);
    (void)hipFree(n->d_spval);
    (void)hipFree(n->d_spslot);
    (void)hipFree(n->d_gbits);
    stage_batch_free(n->single);
    stage_net_free(n->stage);
    delete n;
}

static psst_status validate_network(const psst_neuron_params *p, int32_t n,
                                    const psst_pathway *paths, int32_t np,
                                    const psst_kinetics *kin)
{
    if (!p) return fail(PSST_ERR_INVALID_ARGUMENT, "params is NULL");
    if (n < 1 || n > (1 << 20)) return fail(PSST_ERR_INVALID_ARGUMENT, "n_neurons=%d out of [1, 2^20]", n);
    if (np < 0 || np > 64) return fail(PSST_ERR_INVALID_ARGUMENT, "n_pathways=%d out of [0, 64]", np);
    if (np > 0 && !paths) return fail(PSST_ERR_INVALID_ARGUMENT, "pathways is NULL");
    if (!kin) return fail(PSST_ERR_INVALID_ARGUMENT, "kinetics is NULL");
    if (p->n_pn < 0 || p->n_pn > n) return fail(PSST_ERR_INVALID_ARGUMENT, "n_pn=%d out of [0, n]", p->n_pn);
    if (!(p->area_cm2 > 0.f) || !is_finite_f(p->area_cm2))
        return fail(PSST_ERR_INVALID_ARGUMENT, "area_cm2 must be positive and finite");
    const float *vecs[7] = {p->C_m, p->g_Na, p->g_K, p->g_L, p->E_Na, p->E_K, p->E_L};
    const char *names[7] = {"C_m", "g_Na", "g_K", "g_L", "E_Na", "E_K", "E_L"};
    for (int k = 0; k < 7; ++k) {
        if (!vecs[k]) return fail(PSST_ERR_INVALID_ARGUMENT, "params.%s is NULL", names[k]);
        for (int i = 0; i < n; ++i)
            if (!is_finite_f(vecs[k][i]))
                return fail(PSST_ERR_INVALID_ARGUMENT, "params.%s[%d] is not finite", names[k], i);
    }
    for (int i = 0; i < n; ++i)
        if (!(p->C_m[i] > 0.f)) return fail(PSST_ERR_INVALID_ARGUMENT, "C_m[%d] must be > 0", i);
    for (int t = 0; t < 3; ++t) {
        const float *f = &kin[t].alpha;
        for (int k = 0; k < NKIN; ++k)
            if (!is_finite_f(f[k])) return fail(PSST_ERR_INVALID_ARGUMENT, "kinetics[%d] field %d not finite", t, k);
        if (kin[t].K_p == 0.f) return fail(PSST_ERR_INVALID_ARGUMENT, "kinetics[%d].K_p is 0", t);
    }
    const float hill = kin[PSST_SYN_GABA_B].hill_n;
    bool has_gb = false;
    for (int q = 0; q < np; ++q) has_gb |= paths[q].type == PSST_SYN_GABA_B;
    if (has_gb) {
        if (!(hill >= 1.f && hill <= 8.f && hill == std::floor(hill)))
            return fail(PSST_ERR_INVALID_ARGUMENT, "kinetics[GABA_B].hill_n must be an integer in [1, 8]");
        if (!(kin[PSST_SYN_GABA_B].K_d > 0.f))
            return fail(PSST_ERR_INVALID_ARGUMENT, "kinetics[GABA_B].K_d must be > 0");
    }
    for (int q = 0; q < np; ++q) {
        const psst_pathway &w = paths[q];
        if (w.type < 0 || w.type > 2) return fail(PSST_ERR_INVALID_ARGUMENT, "pathway %d: bad type %d", q, w.type);
        if (!(0 <= w.pre_begin && w.pre_begin < w.pre_end && w.pre_end <= n &&
              0 <= w.post_begin && w.post_begin < w.post_end && w.post_end <= n))
            return fail(PSST_ERR_INVALID_ARGUMENT, "pathway %d: empty or out-of-range block", q);
        if (w.type == PSST_SYN_ACH && w.pre_end > p->n_pn)
            return fail(PSST_ERR_INVALID_ARGUMENT, "pathway %d: cholinergic presynaptic range must lie in the PN rows", q);
        if (w.type != PSST_SYN_ACH && w.pre_begin < p->n_pn)
            return fail(PSST_ERR_INVALID_ARGUMENT, "pathway %d: GABA presynaptic range must lie in the LN rows", q);
        if (!w.g_nS) return fail(PSST_ERR_INVALID_ARGUMENT, "pathway %d: g_nS is NULL", q);
        const int64_t cnt = (int64_t)(w.post_end - w.post_begin) * (w.pre_end - w.pre_begin);
        for (int64_t e = 0; e < cnt; ++e)
            if (!is_finite_f(w.g_nS[e])) return fail(PSST_ERR_INVALID_ARGUMENT, "pathway %d: g_nS[%lld] not finite", q, (long long)e);
        for (int r = 0; r < q; ++r) {
            const psst_pathway &o = paths[r];
            bool same_matrix = (o.type == PSST_SYN_GABA_B) == (w.type == PSST_SYN_GABA_B);
            if (same_matrix && o.pre_begin < w.pre_end && w.pre_begin < o.pre_end &&
                o.post_begin < w.post_end && w.post_begin < o.post_end && o.type == w.type)
                return fail(PSST_ERR_INVALID_ARGUMENT, "pathways %d and %d of one type overlap", r, q);
        }
    }
    return PSST_OK;
}

static psst_status network_create_impl(const psst_neuron_params *p, int32_t n,
                                       const psst_pathway *paths, int32_t np,
                                       const psst_kinetics kin[3], int32_t storage,
                                       psst_network **out)
{
    if (!out) return fail(PSST_ERR_INVALID_ARGUMENT, "out is NULL");
    *out = nullptr;
    psst_status s = validate_network(p, n, paths, np, kin);
    if (s != PSST_OK) return s;
    int dev = 0;
    if ((s = check_device(&dev)) != PSST_OK) return s;

    psst_network *net = new psst_network();
    net->device = dev;
    net->n = n;
    net->n_pn = p->n_pn;
    net->ld = (n + 3) & ~3;
    net->area = p->area_cm2;
    net->cg = 1e-6 / (double)p->area_cm2;
    net->ci = 1e-3 / (double)p->area_cm2;
    const int ld = net->ld, n_ln = n - p->n_pn;
    for (int q = 0; q < np; ++q) net->gabab |= paths[q].type == PSST_SYN_GABA_B;

    int64_t goff = 0;
    for (int q = 0; q < np; ++q) {
        const psst_pathway &w = paths[q];
        net->paths.push_back(PathInfo{w.type, w.pre_begin, w.pre_end, w.post_begin, w.post_end, goff});
        goff += (int64_t)(w.post_end - w.post_begin) * (w.pre_end - w.pre_begin);
    }
    net->grad_entries = goff;
    net->g_floats = (int64_t)n * ld + (net->gabab ? (int64_t)n_ln * ld : 0);
    net->nch = n_chunks(n, p->n_pn, net->gabab);

    // storage: sparse when asked, or (AUTO) when at most a quarter of the
    // pathway entries are synapses
    int64_t present = 0;
    for (int q = 0; q < np; ++q) {
        const psst_pathway &w = paths[q];
        const int64_t cnt = (int64_t)(w.post_end - w.post_begin) * (w.pre_end - w.pre_begin);
        if (!w.mask) present += cnt;
        else
            for (int64_t e = 0; e < cnt; ++e) present += w.mask[e] != 0;
    }
    // which gradient-layout entries are synapses, for in-place updates
    // (only when some pathway has a mask)
    std::vector<uint32_t> gbits;
    if (present < goff) {
        gbits.assign((size_t)((goff + 31) / 32), 0u);
        for (int q = 0; q < np; ++q) {
            const psst_pathway &w = paths[q];
            const int64_t cnt = (int64_t)(w.post_end - w.post_begin) * (w.pre_end - w.pre_begin);
            for (int64_t e = 0; e < cnt; ++e)
                if (!w.mask || w.mask[e]) {
                    const int64_t ge = net->paths[q].grad_off + e;
                    gbits[(size_t)(ge >> 5)] |= 1u << (ge & 31);
                }
        }
    }
    // AUTO above the per-instance limit keeps dense storage unless the dense
    // per-stage matrix would take more than kStageDenseAutoBytes: the sparse
    // form builds the same matrix-core tiles in LDS (bit for bit the same
    // run), which saves HBM but adds the tile build to every stage
    const int64_t stage_dense_bytes = 4LL * ((n + 63) / 64 * 64) *
                                      ((int64_t)((p->n_pn + 127) / 128) * 128 +
                                       (net->gabab ? 2LL : 1LL) * ((n_ln + 127) / 128) * 128);
    bool sparse = false;
    if (storage == PSST_STORAGE_SPARSE) sparse = np > 0;
    else if (storage == PSST_STORAGE_AUTO)
        sparse = np > 0 && 4 * present <= goff &&
                 (n <= kMaxWGNeurons || stage_dense_bytes > kStageDenseAutoBytes);
    // above the per-instance limit the per-stage path keeps its own sparse
    // layout (synapse buckets) instead of the ELL rows
    const bool stage_sparse = sparse && n > kMaxWGNeurons;
    if (stage_sparse) sparse = false;
    std::vector<int32_t> sp_col, sp_slot;
    std::vector<float> sp_val;
    if (sparse) {
        // ELL rows: per postsynaptic i its synapses sorted by presynaptic
        // column, each with its entry in the gradient layout (so an in-place
        // update finds its slot)
        struct Syn {
            int32_t col;
            float g;
            int64_t e;
        };
        std::vector<std::vector<Syn>> rf(n), rb(n);
        for (int q = 0; q < np; ++q) {
            const psst_pathway &w = paths[q];
            const int npre = w.pre_end - w.pre_begin;
            for (int i = w.post_begin; i < w.post_end; ++i)
                for (int j = w.pre_begin; j < w.pre_end; ++j) {
                    const int64_t e = (int64_t)(i - w.post_begin) * npre + (j - w.pre_begin);
                    if (w.mask && w.mask[e] == 0) continue;
                    const int64_t ge = net->paths[q].grad_off + e;
                    if (w.type == PSST_SYN_GABA_B) rb[i].push_back({j - p->n_pn, w.g_nS[e], ge});
                    else rf[i].push_back({j, w.g_nS[e], ge});
                }
        }
        const auto by_col = [](const Syn &x, const Syn &y) { return x.col < y.col; };
        int kf = 1, kb = net->gabab ? 1 : 0;
        for (int i = 0; i < n; ++i) {
            std::stable_sort(rf[i].begin(), rf[i].end(), by_col);
            std::stable_sort(rb[i].begin(), rb[i].end(), by_col);
            kf = std::max(kf, (int)rf[i].size());
            if (net->gabab) kb = std::max(kb, (int)rb[i].size());
        }
        sp_col.assign((size_t)(kf + kb) * ld, 0);
        sp_val.assign((size_t)(kf + kb) * ld, 0.f);
        sp_slot.assign((size_t)goff, -1);
        for (int i = 0; i < n; ++i) {
            for (int half = 0; half < 2; ++half) {
                const auto &r = half ? rb[i] : rf[i];
                const int k0 = half ? kf : 0, K = half ? kb : kf;
                for (int e = 0; e < K; ++e) {
                    const bool real = e < (int)r.size();
                    const size_t slot = (size_t)(k0 + e) * ld + i;
                    sp_col[slot] = real ? r[e].col : (r.empty() ? 0 : r.back().col);
                    sp_val[slot] = real ? r[e].g : 0.f;
                    if (real) sp_slot[(size_t)r[e].e] = (int32_t)slot;
                }
            }
        }
        net->sparse = true;
        net->nch = 0;
        net->g_floats = 2LL * (kf + kb) * ld;      // 8 bytes per stored entry
        net->desc.sp_kf = kf;
        net->desc.sp_kb = kb;
    }
    const bool wg = fits_wg(net);

    // per-instance kernel layout: transposed conductance matrices with padded
    // rows, gt[j * ld + i] (pre j, post i), and the synapse mask alike.  A
    // sparse network small enough for the adjoint keeps them as well: the
    // adjoint's transposed products and its gradient mask read them.
    const bool dense_wg = wg && (!sparse || n <= kMaxAdjointNeurons);
    std::vector<float> gt(dense_wg ? (size_t)n * ld : 0, 0.f);
    std::vector<float> gtb(dense_wg && net->gabab ? (size_t)n_ln * ld : 0, 0.f);
    std::vector<uint8_t> mt(dense_wg ? (size_t)n * ld + gtb.size() : 0, 0);
    for (int q = 0; q < np && dense_wg; ++q) {
        const psst_pathway &w = paths[q];
        const int npre = w.pre_end - w.pre_begin;
        for (int i = w.post_begin; i < w.post_end; ++i)
            for (int j = w.pre_begin; j < w.pre_end; ++j) {
                const int64_t e = (int64_t)(i - w.post_begin) * npre + (j - w.pre_begin);
                const bool present = !w.mask || w.mask[e] != 0;
                const float g = present ? w.g_nS[e] : 0.f;
                if (w.type == PSST_SYN_GABA_B) {
                    gtb[(size_t)(j - p->n_pn) * ld + i] = g;
                    mt[(size_t)n * ld + (size_t)(j - p->n_pn) * ld + i] = present;
                } else {
                    gt[(size_t)j * ld + i] = g;
                    mt[(size_t)j * ld + i] = present;
                }
            }
    }
    std::vector<float> prm((size_t)NPRM * ld, 0.f);
    const float *vecs[7] = {p->C_m, p->g_Na, p->g_K, p->g_L, p->E_Na, p->E_K, p->E_L};
    for (int k = 0; k < 7; ++k)
        for (int i = 0; i < ld; ++i) prm[(size_t)k * ld + i] = i < n ? vecs[k][i] : (k == 0 ? 1.f : 0.f);
    net->h_kin.assign(&kin[0].alpha, &kin[0].alpha + 3 * NKIN);

#define NETCHK(call)                                                              \
    do {                                                                          \
        hipError_t e_ = (call);                                                   \
        if (e_ != hipSuccess) {                                                   \
            net_free(net);                                                        \
            return fail(e_ == hipErrorOutOfMemory ? PSST_ERR_OUT_OF_MEMORY        \
                                                  : PSST_ERR_DEVICE,              \
                        "%s failed: %s", #call, hipGetErrorString(e_));           \
        }                                                                         \
    } while (0)

    if (sparse) {
        NETCHK(hipMalloc(&net->d_spcol, sizeof(int32_t) * sp_col.size()));
        NETCHK(hipMemcpy(net->d_spcol, sp_col.data(), sizeof(int32_t) * sp_col.size(),
                         hipMemcpyHostToDevice));
        NETCHK(hipMalloc(&net->d_spval, sizeof(float) * sp_val.size()));
        NETCHK(hipMemcpy(net->d_spval, sp_val.data(), sizeof(float) * sp_val.size(),
                         hipMemcpyHostToDevice));
        NETCHK(hipMalloc(&net->d_spslot, sizeof(int32_t) * sp_slot.size()));
        NETCHK(hipMemcpy(net->d_spslot, sp_slot.data(), sizeof(int32_t) * sp_slot.size(),
                         hipMemcpyHostToDevice));
    }
    if (!gbits.empty()) {
        NETCHK(hipMalloc(&net->d_gbits, sizeof(uint32_t) * gbits.size()));
        NETCHK(hipMemcpy(net->d_gbits, gbits.data(), sizeof(uint32_t) * gbits.size(),
                         hipMemcpyHostToDevice));
    }
    if (dense_wg) {
        NETCHK(hipMalloc(&net->d_gt, sizeof(float) * gt.size()));
        NETCHK(hipMemcpy(net->d_gt, gt.data(), sizeof(float) * gt.size(), hipMemcpyHostToDevice));
        if (!gtb.empty()) {
            NETCHK(hipMalloc(&net->d_gtb, sizeof(float) * gtb.size()));
            NETCHK(hipMemcpy(net->d_gtb, gtb.data(), sizeof(float) * gtb.size(), hipMemcpyHostToDevice));
        }
        NETCHK(hipMalloc(&net->d_maskt, mt.size()));
        NETCHK(hipMemcpy(net->d_maskt, mt.data(), mt.size(), hipMemcpyHostToDevice));
    } else if (!wg) {
        psst_status st = stage_net_create(net, paths, np, stage_sparse);
        if (st != PSST_OK) {
            net_free(net);
            return st;
        }
    }
    NETCHK(hipMalloc(&net->d_prm, sizeof(float) * prm.size()));
    NETCHK(hipMemcpy(net->d_prm, prm.data(), sizeof(float) * prm.size(), hipMemcpyHostToDevice));
    NETCHK(hipMalloc(&net->d_kin, sizeof(float) * 3 * NKIN));
    NETCHK(hipMemcpy(net->d_kin, net->h_kin.data(), sizeof(float) * 3 * NKIN, hipMemcpyHostToDevice));
    if (np > 0) {
        std::vector<int64_t> pt;
        for (auto &q : net->paths) {
            pt.push_back(q.type); pt.push_back(q.pre0); pt.push_back(q.pre1);
            pt.push_back(q.post0); pt.push_back(q.post1); pt.push_back(q.grad_off);
        }
        NETCHK(hipMalloc(&net->d_paths, sizeof(int64_t) * pt.size()));
        NETCHK(hipMemcpy(net->d_paths, pt.data(), sizeof(int64_t) * pt.size(), hipMemcpyHostToDevice));
    }
    InstDesc &d = net->desc;
    d.paths = net->d_paths;
    d.maskt = net->d_maskt;
    d.n_paths = np;
    d.grad_entries = net->grad_entries;
    d.gt = net->d_gt;
    d.gtb = net->d_gtb;
    d.prm = net->d_prm;
    d.kin = net->d_kin;
    d.off = 0;
    d.n = n;
    d.n_pn = p->n_pn;
    d.ld = ld;
    d.flags = (net->gabab ? DESC_GABAB : 0) | (np == 0 ? DESC_NOSYN : 0) |
              (sparse ? DESC_SPARSE : 0);
    d.sp_col = net->d_spcol;
    d.sp_val = net->d_spval;
    d.cg = net->cg;
    d.ci = net->ci;
    NETCHK(hipMalloc(&net->d_desc, sizeof(InstDesc)));
    NETCHK(hipMemcpy(net->d_desc, &d, sizeof(InstDesc), hipMemcpyHostToDevice));
    int32_t zero = 0;
    NETCHK(hipMalloc(&net->d_order, sizeof(int32_t)));
    NETCHK(hipMemcpy(net->d_order, &zero, sizeof(int32_t), hipMemcpyHostToDevice));
    NETCHK(hipMalloc(&net->d_flag, sizeof(int32_t)));
    NETCHK(hipMemset(net->d_flag, 0, sizeof(int32_t)));
#undef NETCHK
    if (!wg) {
        // the one-trial stage batch psst_integrate uses: allocated here, so
        // integrate calls allocate nothing
        psst_status st = stage_single_prepare(net);
        if (st != PSST_OK) {
            net_free(net);
            return st;
        }
    }
    *out = net;
    return PSST_OK;
}

extern "C" psst_status psst_network_create(const psst_neuron_params *p, int32_t n,
                                           const psst_pathway *paths, int32_t np,
                                           const psst_kinetics kin[3], psst_network **out)
{
    return network_create_impl(p, n, paths, np, kin, PSST_STORAGE_AUTO, out);
}

extern "C" psst_status psst_network_create_storage(const psst_neuron_params *p, int32_t n,
                                                   const psst_pathway *paths, int32_t np,
                                                   const psst_kinetics kin[3], int32_t storage,
                                                   psst_network **out)
{
    if (storage < PSST_STORAGE_AUTO || storage > PSST_STORAGE_SPARSE) {
        if (out) *out = nullptr;
        return fail(PSST_ERR_INVALID_ARGUMENT, "storage=%d is not a psst_storage value", storage);
    }
    return network_create_impl(p, n, paths, np, kin, storage, out);
}

extern "C" psst_status psst_network_destroy(psst_network *net)
{
    if (!net) return fail(PSST_ERR_INVALID_ARGUMENT, "network is NULL");
    net_free(net);
    return PSST_OK;
}

extern "C" psst_status psst_state_layout(const psst_network *net, int64_t *n_words, int32_t *n_vars)
{
    if (!net) return fail(PSST_ERR_INVALID_ARGUMENT, "network is NULL");
    if (n_words) *n_words = 2LL * NVAR * net->n;
    if (n_vars) *n_vars = NVAR;
    return PSST_OK;
}

extern "C" psst_status psst_network_grad_size(const psst_network *net, int64_t *n_entries)
{
    if (!net || !n_entries) return fail(PSST_ERR_INVALID_ARGUMENT, "NULL argument");
    *n_entries = net->grad_entries;
    return PSST_OK;
}

extern "C" psst_status psst_network_update(psst_network *net, const float *g, const float *g_Na,
                                           const float *g_K, const float *g_L, void *stream)
{
    if (!net) return fail(PSST_ERR_INVALID_ARGUMENT, "network is NULL");
    psst::NetUpdateArgs a{};
    a.g = net->grad_entries > 0 ? g : nullptr;
    a.g_na = g_Na;
    a.g_k = g_K;
    a.g_l = g_L;
    a.paths = net->d_paths;
    a.present_bits = net->d_gbits;
    a.entries = net->grad_entries;
    a.n_paths = (int32_t)net->paths.size();
    a.n = net->n;
    a.n_pn = net->n_pn;
    a.ld = net->ld;
    a.gt = net->d_gt;
    a.gtb = net->d_gtb;
    a.sp_val = net->d_spval;
    a.sp_slot = net->d_spslot;
    if (net->stage) {
        a.stage_G = net->stage->G;
        a.stage_Kp = net->stage->Kp;
        a.stage_ka = net->stage->ka;
        a.stage_kg = net->stage->kg;
        a.bk_off = net->stage->sp_off;
        a.bk_col = net->stage->sp_col;
        a.bk_val = net->stage->sp_val;
    }
    a.prm = net->d_prm;
    return network_update_launch(a, (hipStream_t)stream);
}

static psst_status launch_init(const InstDesc *d_desc, int32_t n_inst, const float *v0,
                               float *state, int64_t nt, hipStream_t s)
{
    InitArgs a{d_desc, n_inst, v0, state, nt};
    void *args[] = {&a};
    HIPCHK(hipLaunchKernel(init_kernel(), dim3(n_inst), dim3(256), args, 0, s));
    return PSST_OK;
}

extern "C" psst_status psst_state_init(const psst_network *net, const float *v0, float *state,
                                       void *stream)
{
    if (!net || !v0 || !state) return fail(PSST_ERR_INVALID_ARGUMENT, "NULL argument");
    return launch_init(net->d_desc, 1, v0, state, net->n, (hipStream_t)stream);
}

// ---------------------------------------------------------------------------
// the per-instance persistent kernel: variant choice and launch
// ---------------------------------------------------------------------------

static const WGVariant *find_variant(int bs, int npt, bool gen, bool lg = false, int slots = 0)
{
    for (const WGVariant *v = wg_variants(); v->fn; ++v)
        if (v->bs == bs && v->npt == npt && v->gen == gen && v->lg == lg && v->slots == slots)
            return v;
    return nullptr;
}

// The variant a launch group runs: register-column variants exist for
// classical RK4 only, so a group tuned to one runs the same shape without
// register columns once an explicit tableau is set on its batch.
static const WGVariant *group_variant(const Group &g, bool gen)
{
    const WGVariant *v = find_variant(g.bs, g.npt, gen, g.lg, g.slots);
    if (!v && g.slots) v = find_variant(g.bs, g.npt, gen, g.lg, 0);
    return v;
}

// Register-column variants are candidates of the tuner unless the
// environment variable PSST_RR=0 turns them off (comparisons: the same bits).
static bool rr_enabled()
{
    const char *e = std::getenv("PSST_RR");
    return !(e && e[0] == '0');
}

// The lane-group kernel (conductances in registers) takes the instances it
// can unless the environment variable PSST_LG=0 turns it off (comparisons:
// both mappings give the same bits).
static bool lg_enabled()
{
    const char *e = std::getenv("PSST_LG");
    return !(e && e[0] == '0');
}

static bool net_lg(const psst_network *q)
{
    return lg_enabled() && lg_eligible(q->n, q->n_pn, q->desc.flags);
}

static size_t max_lds_per_block()
{
    static size_t cached = 0;
    if (!cached) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess) dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess) cached = prop.sharedMemPerBlock;
        if (!cached) cached = 65536;
    }
    return cached;
}

static psst_status set_lds_attr(const void *fn, size_t bytes)
{
    if (bytes > 65536) HIPCHK(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    return PSST_OK;
}

// Default variant for instances up to max_n neurons (the synaptic product
// needs bs >= ld / 4 threads: one per row quad).
static void default_shape(int max_n, int *bs, int *npt)
{
    if (max_n <= 64) { *bs = 64; *npt = 1; }
    else if (max_n <= 256) { *bs = 256; *npt = 1; }
    else if (max_n <= 512) { *bs = 512; *npt = 1; }
    else { *bs = 256; *npt = 4; }
}


// Networks the per-instance kernel takes: at most 1024 neurons, and the
// activation and partial-sum buffers fit the workgroup's LDS.
static bool fits_wg(const psst_network *q)
{
    return q->n <= kMaxWGNeurons && wg_lds_bytes(false, q->ld, q->nch, 0) <= max_lds_per_block();
}

static psst_status validate_common(float dt, int64_t n_steps, int64_t step0, const psst_record *rec)
{
    if (!(dt > 0.f) || !is_finite_f(dt)) return fail(PSST_ERR_INVALID_ARGUMENT, "dt_ms must be positive and finite");
    if (n_steps < 0) return fail(PSST_ERR_INVALID_ARGUMENT, "n_steps < 0");
    if (step0 < 0) return fail(PSST_ERR_INVALID_ARGUMENT, "step0 < 0");
    if (rec) {
        if (rec->v_out && (rec->stride <= 0 || rec->capacity < 0))
            return fail(PSST_ERR_INVALID_ARGUMENT, "record: v_out needs stride > 0 and capacity >= 0");
        if (rec->spike_count && rec->spike_cap > 0 && !rec->spike_t_ms)
            return fail(PSST_ERR_INVALID_ARGUMENT, "record: spike_cap > 0 needs spike_t_ms");
        if (rec->spike_cap < 0) return fail(PSST_ERR_INVALID_ARGUMENT, "record: spike_cap < 0");
    }
    return PSST_OK;
}

static psst_status validate_stim(const psst_stimulus *st)
{
    if (st && st->pulse_ptr && (!st->on_step || !st->off_step || !st->amp_nA))
        return fail(PSST_ERR_INVALID_ARGUMENT, "stimulus: pulse_ptr given without on/off/amp arrays");
    return PSST_OK;
}

static StimDev to_dev(const psst_stimulus *st)
{
    StimDev s{};
    if (st) {
        s.i_const = st->i_const_nA;
        s.pulse_ptr = st->pulse_ptr;
        s.on_step = st->on_step;
        s.off_step = st->off_step;
        s.amp = st->amp_nA;
    }
    return s;
}

static RecDev to_dev(const psst_record *r)
{
    RecDev d{};
    if (r) {
        d.v_out = r->v_out;
        d.stride = r->stride;
        d.capacity = r->capacity;
        d.spike_count = r->spike_count;
        d.spike_t = r->spike_t_ms;
        d.spike_cap = r->spike_cap;
    }
    return d;
}

extern "C" psst_status psst_integrate(psst_network *net, float *state, const psst_stimulus *stim,
                                      float dt, int64_t n_steps, int64_t step0,
                                      const psst_record *rec, void *stream)
{
    if (!net) return fail(PSST_ERR_INVALID_ARGUMENT, "network is NULL");
    if (!state) return fail(PSST_ERR_INVALID_ARGUMENT, "state is NULL");
    psst_status s = validate_common(dt, n_steps, step0, rec);
    if (s != PSST_OK) return s;
    if ((s = validate_stim(stim)) != PSST_OK) return s;
    if (!fits_wg(net))
        return stage_integrate_single(net, state, stim, dt, n_steps, step0, rec, stream);
    if (n_steps == 0) return PSST_OK;
    int bs, npt;
    default_shape(net->n, &bs, &npt);
    // small dense networks: the lane-group kernel (unless a shape is forced)
    const bool lg = net_lg(net) && !std::getenv("PSST_WG_SHAPE");
    if (lg) {
        bs = kLGThreads;
        npt = kLGPairs;
    }
    // a network whose whole conductance matrix stays in LDS sums one (chunk,
    // row) pair per thread: enough threads for every pair in one pass (up to
    // 512) shorten the stage (measured: 120 neurons, 512 threads 12.0 us per
    // step against 14.0 with 256; 60 neurons, 128 threads 8.9 against 10.1)
    if (!lg && !net->sparse && net->nch > 0 && net->n <= 512 &&
        sizeof(double) * (2 + (size_t)net->nch) * net->ld +
                sizeof(float) * (size_t)net->nch * kChunkWidth * net->ld <= max_lds_per_block()) {
        const int pairs = net->nch * net->n;
        int b = 64;
        while (b < 512 && (b < pairs || b < net->n)) b *= 2;
        if (find_variant(b, 1, net->gen)) {
            bs = b;
            npt = 1;
        }
    }
    // PSST_WG_SHAPE="<threads>x<neurons per thread>" fixes the launch shape
    // when that variant can take the network (as for batches)
    if (const char *shp = std::getenv("PSST_WG_SHAPE")) {
        int b2 = 0, n2 = 0;
        if (std::sscanf(shp, "%dx%d", &b2, &n2) == 2 && find_variant(b2, n2, net->gen) &&
            b2 * n2 >= net->n && 4 * b2 >= net->ld) {
            bs = b2;
            npt = n2;
        }
    }
    // the whole LDS: whatever the activation and partial buffers leave holds
    // the leading columns of every conductance chunk (all of G when it fits);
    // the lane-group kernel needs only its activation slots
    const char *env = std::getenv("PSST_LDS_G");
    const size_t lds = lg ? (size_t)kLGLdsBytes
                          : (env && env[0] == '0') ? wg_lds_bytes(false, net->ld, net->nch, 0)
                                                   : max_lds_per_block();
    const WGVariant *v = find_variant(bs, npt, net->gen, lg);
    if (!v) return fail(PSST_ERR_UNSUPPORTED, "no kernel variant for n=%d", net->n);
    if ((s = set_lds_attr(v->fn, lds)) != PSST_OK) return s;
    WGArgs a{};
    a.desc = net->d_desc;
    a.order = net->d_order;
    a.state = state;
    a.nt = net->n;
    a.stim = to_dev(stim);
    a.rec = to_dev(rec);
    a.dt = (double)dt;
    a.n_steps = n_steps;
    a.step0 = step0;
    a.ckpt = nullptr;
    a.K = 1;
    a.lds_bytes = (int64_t)lds;
    a.flag = net->d_flag;
    a.tab = net->tab;
    a.store_state = 1;
    void *args[] = {&a};
    HIPCHK(hipLaunchKernel(v->fn, dim3(1), dim3(bs), args, lds, (hipStream_t)stream));
    return PSST_OK;
}

static psst_status poll_flag(int32_t *d_flag, void *stream)
{
    HIPCHK(hipStreamSynchronize((hipStream_t)stream));
    int32_t f = 0;
    HIPCHK(hipMemcpy(&f, d_flag, sizeof f, hipMemcpyDeviceToHost));
    if (f) {
        int32_t z = 0;
        HIPCHK(hipMemcpy(d_flag, &z, sizeof z, hipMemcpyHostToDevice));
        return fail(PSST_ERR_NONFINITE, "a state variable became non-finite");
    }
    return PSST_OK;
}

extern "C" psst_status psst_network_poll(psst_network *net, void *stream)
{
    if (!net) return fail(PSST_ERR_INVALID_ARGUMENT, "network is NULL");
    return poll_flag(net->d_flag, stream);
}

// ---------------------------------------------------------------------------
// batches
// ---------------------------------------------------------------------------

static void batch_free(psst_batch *b)
{
    if (!b) return;
    for (hipStream_t st : b->aux) {
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
    }
    for (hipEvent_t e : b->aux_done) (void)hipEventDestroy(e);
    if (b->aux_fork) (void)hipEventDestroy(b->aux_fork);
    for (auto &g : b->groups) (void)hipFree(g.d_order);
    (void)hipFree(b->lean.d_order);
    (void)hipFree(b->d_desc);
    (void)hipFree(b->d_flag);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    stage_batch_free(b->stage);
    for (StageBatch *sb : b->subs) stage_batch_free(sb);
    adjoint_free(b->adj);
    stream_bufs_free(b->strm);
    delete b;
}

static WGArgs group_args(psst_batch *b, const Group &g, float *states, const psst_stimulus *stim,
                         float dt, int64_t n_steps, int64_t step0, const psst_record *rec,
                         float *ckpt, int32_t K)
{
    WGArgs a{};
    a.desc = b->d_desc;
    a.order = g.d_order;
    a.state = states;
    a.nt = b->nt;
    a.stim = to_dev(stim);
    a.rec = to_dev(rec);
    a.dt = (double)dt;
    a.n_steps = n_steps;
    a.step0 = step0;
    a.ckpt = ckpt;
    a.K = K > 0 ? K : 1;
    a.lds_bytes = (int64_t)g.lds;
    a.flag = b->d_flag;
    a.tab = b->tab;
    a.store_state = 1;
    return a;
}

static psst_status launch_group(const Group &g, bool gen, WGArgs &a, hipStream_t s)
{
    const WGVariant *v = group_variant(g, gen);
    if (!v) return fail(PSST_ERR_UNSUPPORTED, "no kernel variant bs=%d npt=%d", g.bs, g.npt);
    psst_status st = set_lds_attr(v->fn, g.lds);
    if (st != PSST_OK) return st;
    void *args[] = {&a};
    HIPCHK(hipLaunchKernel(v->fn, dim3((unsigned)g.order.size()), dim3(g.bs), args, g.lds, s));
    return PSST_OK;
}

// Two timing events, destroyed on every return path.
struct EventPair {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~EventPair()
    {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    }
};

// PSST_TUNE_LOG=1 prints every timed candidate to stderr.
static bool tune_log()
{
    const char *e = std::getenv("PSST_TUNE_LOG");
    return e && e[0] == '1';
}

// Compute units of the current device.
static int device_cus()
{
    static int cached = 0;
    if (!cached) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess) dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess) cached = prop.multiProcessorCount;
        if (cached <= 0) cached = 1;
    }
    return cached;
}

// Time candidate variants -- shape (threads x neurons per thread) and
// register columns -- for one group on a scratch state (short run, no
// stimulus, no recording) and keep the fastest.  The timed launch covers the
// group's largest instances, one per compute unit: the size classes of a
// batch run side by side and fill each other's last rounds, so what counts
// is the time of a full round, not of a tail with most units idle.
struct Shape {
    int bs, npt, slots;
};

static psst_status tune_group(psst_batch *b, Group &g, float *scratch, hipStream_t s,
                              Shape *no_regs, float *t_best, float *t_plain)
{
    *no_regs = Shape{g.bs, g.npt, 0};
    *t_best = *t_plain = 0.f;
    if (g.lg) return PSST_OK;          // one shape
    std::vector<Shape> cands;
    for (const WGVariant *v = wg_variants(); v->fn; ++v) {
        if (v->gen != b->gen || v->lg) continue;
        if (v->slots && !rr_enabled()) continue;
        const int cap = v->bs * v->npt;
        if (cap < g.max_n || cap >= 4 * std::max(g.max_n, 64)) continue;
        if (4 * v->bs < g.max_ld) continue;     // every row quad needs a thread
        cands.push_back({v->bs, v->npt, v->slots});
    }
    if (cands.size() <= 1) {
        if (cands.size() == 1) {
            g.bs = cands[0].bs;
            g.npt = cands[0].npt;
            g.slots = cands[0].slots;
            if (!g.slots) *no_regs = cands[0];
        }
        return PSST_OK;
    }
    EventPair ev;
    HIPCHK(hipEventCreate(&ev.e0));
    HIPCHK(hipEventCreate(&ev.e1));
    float best = 1e30f, best_plain = 1e30f;
    Shape bsh{g.bs, g.npt, g.slots};
    const size_t round = std::min(g.order.size(), (size_t)device_cus());
    for (auto &c : cands) {
        Group t = g;
        t.order.resize(round);          // the grid: the first (largest) instances
        t.bs = c.bs;
        t.npt = c.npt;
        t.slots = c.slots;
        WGArgs a = group_args(b, t, scratch, nullptr, 0.01f, 4, 0, nullptr, nullptr, 1);
        psst_status st = launch_group(t, b->gen, a, s);        // warm-up
        if (st != PSST_OK) return st;
        a.n_steps = 16;
        HIPCHK(hipEventRecord(ev.e0, s));
        if ((st = launch_group(t, b->gen, a, s)) != PSST_OK) return st;
        HIPCHK(hipEventRecord(ev.e1, s));
        HIPCHK(hipEventSynchronize(ev.e1));
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, ev.e0, ev.e1));
        if (tune_log())
            std::fprintf(stderr,
                         "psst tune: %zu of %zu instances, n <= %d: %d x %d, %d slots: %.3f ms\n",
                         round, g.order.size(), g.max_n, c.bs, c.npt, c.slots, ms);
        if (ms < best) {
            best = ms;
            bsh = c;
        }
        if (!c.slots && ms < best_plain) {
            best_plain = ms;
            *no_regs = c;
        }
    }
    g.bs = bsh.bs;
    g.npt = bsh.npt;
    g.slots = bsh.slots;
    *t_best = best;
    *t_plain = best_plain < 1e29f ? best_plain : best;
    return PSST_OK;
}

// Launch groups of a batch from its size classes, largest first: a class
// joins the group before it when both use the same variant (the instances
// stay in largest-first order); the lane-group group last.
static std::vector<Group> merge_classes(const std::vector<Group> &cls, const Group &gl)
{
    std::vector<Group> merged;
    for (int c = (int)cls.size() - 1; c >= 0; --c) {
        const Group &t = cls[c];
        if (t.order.empty()) continue;
        if (!merged.empty() && merged.back().bs == t.bs && merged.back().npt == t.npt &&
            merged.back().slots == t.slots) {
            Group &m = merged.back();
            m.order.insert(m.order.end(), t.order.begin(), t.order.end());
            m.max_n = std::max(m.max_n, t.max_n);
            m.max_ld = std::max(m.max_ld, t.max_ld);
        } else {
            merged.push_back(t);
        }
    }
    if (!gl.order.empty()) merged.push_back(gl);
    for (Group &t : merged) t.d_order = nullptr;
    return merged;
}

// Time a whole launch plan (its groups as the nodes of one graph, as
// psst_integrate_batch submits them) over a 50-step run on the scratch
// state, the better of two launches after a warm-up: size classes run side
// by side, so how they share the chip decides.
static psst_status time_plan(psst_batch *b, std::vector<Group> &plan, float *scratch,
                             hipStream_t s, float *ms_out)
{
    struct Tmp {
        std::vector<int32_t *> d;
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        ~Tmp()
        {
            if (exec) (void)hipGraphExecDestroy(exec);
            if (graph) (void)hipGraphDestroy(graph);
            for (auto *p : d) (void)hipFree(p);
        }
    } tmp;
    std::vector<WGArgs> args(plan.size());
    HIPCHK(hipGraphCreate(&tmp.graph, 0));
    for (size_t k = 0; k < plan.size(); ++k) {
        Group &g = plan[k];
        int32_t *d = nullptr;
        HIPCHK(hipMalloc(&d, sizeof(int32_t) * g.order.size()));
        tmp.d.push_back(d);
        HIPCHK(hipMemcpy(d, g.order.data(), sizeof(int32_t) * g.order.size(),
                         hipMemcpyHostToDevice));
        g.d_order = d;
        args[k] = group_args(b, g, scratch, nullptr, 0.01f, 50, 0, nullptr, nullptr, 1);
        g.d_order = nullptr;
        const WGVariant *v = group_variant(g, b->gen);
        if (!v) return fail(PSST_ERR_UNSUPPORTED, "no kernel variant");
        psst_status st = set_lds_attr(v->fn, g.lds);
        if (st != PSST_OK) return st;
        void *kp[] = {&args[k]};
        hipKernelNodeParams p{};
        p.func = const_cast<void *>(v->fn);
        p.gridDim = dim3((unsigned)g.order.size());
        p.blockDim = dim3(g.bs);
        p.sharedMemBytes = (unsigned)g.lds;
        p.kernelParams = kp;
        p.extra = nullptr;
        hipGraphNode_t node;
        HIPCHK(hipGraphAddKernelNode(&node, tmp.graph, nullptr, 0, &p));
    }
    HIPCHK(hipGraphInstantiate(&tmp.exec, tmp.graph, nullptr, nullptr, 0));
    EventPair ev;
    HIPCHK(hipEventCreate(&ev.e0));
    HIPCHK(hipEventCreate(&ev.e1));
    HIPCHK(hipGraphLaunch(tmp.exec, s));          // warm-up
    float best = 1e30f;
    for (int r = 0; r < 2; ++r) {                  // the better of two timed launches
        HIPCHK(hipEventRecord(ev.e0, s));
        HIPCHK(hipGraphLaunch(tmp.exec, s));
        HIPCHK(hipEventRecord(ev.e1, s));
        HIPCHK(hipEventSynchronize(ev.e1));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, ev.e0, ev.e1));
        best = std::min(best, ms);
    }
    *ms_out = best;
    return PSST_OK;
}

// Size classes of the per-instance kernels (upper bounds of n): each class
// is tuned on its own; neighbouring classes that choose the same variant
// share one launch.
static const int kClassEdges[] = {192, 256, 320, 384, 448, 512, 1024};
static const int kNumClasses = (int)(sizeof(kClassEdges) / sizeof(kClassEdges[0]));

static int size_class(int n)
{
    int c = 0;
    while (c + 1 < kNumClasses && n > kClassEdges[c]) ++c;
    return c;
}

// Name of the device's architecture, for the tuning cache key.
static std::string device_arch()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return "unknown";
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    return std::string(prop.gcnArchName);
}

// ---------------------------------------------------------------------------
// tuning table: per size class, the chosen variant and the fastest without
// register columns (with their full-round times); per batch composition, the
// mask of classes that take register columns.  Kept for the process and read
// from (PSST_TUNE_WRITE=1: written to) a text file per device architecture,
// tuning/<arch>.txt beside the library (PSST_TUNE_FILE overrides the path),
// so that a shipped table makes the choices without timing runs.
// ---------------------------------------------------------------------------

typedef std::tuple<std::string, int, bool, bool, bool, size_t, bool> TuneKey;
typedef std::tuple<std::string, std::vector<size_t>, bool, bool, bool, size_t, bool> PlanKey;
struct ClassChoice {
    Shape best, plain;
    float t_best, t_plain;          // ms of a full round of the class
};
static std::mutex g_tune_mu;
static std::map<TuneKey, ClassChoice> g_tune_cache;
static std::map<PlanKey, int> g_plan_cache;
static std::set<std::string> g_tables_read;

static std::string tune_table_path(const std::string &arch)
{
    if (const char *e = std::getenv("PSST_TUNE_FILE")) return e;
    Dl_info info;
    if (!dladdr((void *)&psst_version, &info) || !info.dli_fname) return std::string();
    const std::string lib(info.dli_fname);
    const size_t slash = lib.rfind('/');
    const std::string dir = slash == std::string::npos ? std::string(".") : lib.substr(0, slash);
    return dir + "/tuning/" + arch.substr(0, arch.find(':')) + ".txt";
}

// Read the table of arch into the caches once per process (caller holds
// g_tune_mu).  Lines:
//   class <arch> <class> <gen> <sparse> <gabab> <lds> <rr> <bs> <npt> <slots>
//         <plain bs> <plain npt> <t_best ms> <t_plain ms>
//   plan <arch> <gen> <sparse> <gabab> <lds> <rr> <mask> <n> <count_0> .. <count_n-1>
// '#' starts a comment line; malformed lines are skipped.
static void read_tune_table(const std::string &arch)
{
    if (!g_tables_read.insert(arch).second) return;
    const std::string path = tune_table_path(arch);
    if (path.empty()) return;
    std::ifstream in(path);
    std::string line;
    while (std::getline(in, line)) {
        std::istringstream ss(line);
        std::string kind, a;
        if (!(ss >> kind >> a) || kind[0] == '#' || a != arch) continue;
        int gen, sparse, gabab, rr;
        size_t lds;
        if (kind == "class") {
            int c;
            ClassChoice ch;
            if (!(ss >> c >> gen >> sparse >> gabab >> lds >> rr >> ch.best.bs >> ch.best.npt >>
                  ch.best.slots >> ch.plain.bs >> ch.plain.npt >> ch.t_best >> ch.t_plain))
                continue;
            ch.plain.slots = 0;
            g_tune_cache[TuneKey{arch, c, gen != 0, sparse != 0, gabab != 0, lds, rr != 0}] = ch;
        } else if (kind == "plan") {
            int mask;
            size_t nc;
            if (!(ss >> gen >> sparse >> gabab >> lds >> rr >> mask >> nc) || nc > 64) continue;
            std::vector<size_t> counts(nc);
            bool ok = true;
            for (size_t k = 0; k < nc && ok; ++k) ok = (bool)(ss >> counts[k]);
            if (ok)
                g_plan_cache[PlanKey{arch, counts, gen != 0, sparse != 0, gabab != 0, lds,
                                     rr != 0}] = mask;
        }
    }
}

// Write the caches' entries of arch to its table (caller holds g_tune_mu).
static void write_tune_table(const std::string &arch)
{
    const std::string path = tune_table_path(arch);
    if (path.empty()) return;
    const size_t slash = path.rfind('/');
    if (slash != std::string::npos) (void)mkdir(path.substr(0, slash).c_str(), 0755);
    const std::string tmp = path + ".tmp";
    {
        std::ofstream out(tmp);
        if (!out) return;
        out << "# psst batch tuning table (written with PSST_TUNE_WRITE=1)\n";
        for (const auto &kv : g_tune_cache) {
            const TuneKey &k = kv.first;
            if (std::get<0>(k) != arch) continue;
            const ClassChoice &ch = kv.second;
            out << "class " << arch << ' ' << std::get<1>(k) << ' ' << std::get<2>(k) << ' '
                << std::get<3>(k) << ' ' << std::get<4>(k) << ' ' << std::get<5>(k) << ' '
                << std::get<6>(k) << ' ' << ch.best.bs << ' ' << ch.best.npt << ' '
                << ch.best.slots << ' ' << ch.plain.bs << ' ' << ch.plain.npt << ' '
                << ch.t_best << ' ' << ch.t_plain << '\n';
        }
        for (const auto &kv : g_plan_cache) {
            const PlanKey &k = kv.first;
            if (std::get<0>(k) != arch) continue;
            out << "plan " << arch << ' ' << std::get<2>(k) << ' ' << std::get<3>(k) << ' '
                << std::get<4>(k) << ' ' << std::get<5>(k) << ' ' << std::get<6>(k) << ' '
                << kv.second << ' ' << std::get<1>(k).size();
            for (size_t c : std::get<1>(k)) out << ' ' << c;
            out << '\n';
        }
    }
    (void)std::rename(tmp.c_str(), path.c_str());
}

static bool tune_write()
{
    const char *e = std::getenv("PSST_TUNE_WRITE");
    return e && e[0] == '1';
}

extern "C" psst_status psst_batch_create(psst_network *const *nets, int32_t n, psst_batch **out)
{
    if (!out) return fail(PSST_ERR_INVALID_ARGUMENT, "out is NULL");
    *out = nullptr;
    if (!nets) return fail(PSST_ERR_INVALID_ARGUMENT, "nets is NULL");
    if (n < 1 || n > (1 << 20)) return fail(PSST_ERR_INVALID_ARGUMENT, "n=%d out of [1, 2^20]", n);
    for (int32_t k = 0; k < n; ++k)
        if (!nets[k]) return fail(PSST_ERR_INVALID_ARGUMENT, "nets[%d] is NULL", k);
    int dev = 0;
    psst_status s = check_device(&dev);
    if (s != PSST_OK) return s;

    psst_batch *b = new psst_batch();
    b->nets.assign(nets, nets + n);
    b->n = n;
    b->offsets.resize(n + 1);
    b->offsets[0] = 0;
    b->shared = true;
    for (int32_t k = 0; k < n; ++k) {
        b->offsets[k + 1] = b->offsets[k] + nets[k]->n;
        b->shared &= nets[k] == nets[0];
    }
    b->nt = b->offsets[n];
    // the method of the networks, which must agree
    b->gen = nets[0]->gen;
    b->tab = nets[0]->tab;
    for (int32_t k = 1; k < n; ++k)
        if (nets[k]->gen != b->gen ||
            (b->gen && std::memcmp(&nets[k]->tab, &b->tab, sizeof(psst::Tab)) != 0)) {
            delete b;
            return fail(PSST_ERR_INVALID_ARGUMENT,
                        "nets[%d] uses a different Runge-Kutta tableau than nets[0]", k);
        }

#define BCHK(call)                                                                \
    do {                                                                          \
        hipError_t e_ = (call);                                                   \
        if (e_ != hipSuccess) {                                                   \
            batch_free(b);                                                        \
            return fail(e_ == hipErrorOutOfMemory ? PSST_ERR_OUT_OF_MEMORY        \
                                                  : PSST_ERR_DEVICE,              \
                        "%s failed: %s", #call, hipGetErrorString(e_));           \
        }                                                                         \
    } while (0)

    BCHK(hipMalloc(&b->d_flag, sizeof(int32_t)));
    BCHK(hipMemset(b->d_flag, 0, sizeof(int32_t)));
    std::vector<InstDesc> desc(n);
    for (int32_t k = 0; k < n; ++k) {
        desc[k] = nets[k]->desc;
        desc[k].off = b->offsets[k];
    }
    BCHK(hipMalloc(&b->d_desc, sizeof(InstDesc) * n));
    BCHK(hipMemcpy(b->d_desc, desc.data(), sizeof(InstDesc) * n, hipMemcpyHostToDevice));

    bool all_wg = true;
    for (auto *q : b->nets) all_wg &= fits_wg(q);
    if (!all_wg && !b->shared) {
        // runs of consecutive instances of one large network become per-stage
        // sub-batches inside the batch's arrays, sharing its error flag
        for (int32_t k = 0; k < n;) {
            if (fits_wg(nets[k])) {
                ++k;
                continue;
            }
            int32_t k1 = k + 1;
            while (k1 < n && nets[k1] == nets[k]) ++k1;
            StageBatch *sb = nullptr;
            s = stage_batch_create(nets[k], k1 - k, &sb, b->nt, b->offsets[k]);
            if (s != PSST_OK) {
                batch_free(b);
                return s;
            }
            stage_batch_use_flag(sb, b->d_flag);
            b->subs.push_back(sb);
            k = k1;
        }
    }
    if (!all_wg && b->shared) {
        b->stage_path = true;
        s = stage_batch_create(nets[0], n, &b->stage);
        if (s != PSST_OK) {
            batch_free(b);
            return s;
        }
        b->describe = stage_batch_describe(b->stage);
        *out = b;
        return PSST_OK;
    }

    // Launch groups, workgroups in largest-first (LPT) order of cost ~ n^2:
    // small dense networks the lane-group kernel takes (conductances in
    // registers) form one group; the rest are split into size classes, each
    // with its own tuned variant (shape and register columns) and the full
    // per-workgroup LDS: each instance keeps the leading columns of every
    // conductance chunk on chip (registers, then LDS; all of G when it fits)
    // and streams the rest from L2/MALL/HBM.  Neighbouring classes that
    // choose the same variant share one launch.  Each group is one launch (a
    // node of the batch's graph).
    std::vector<int32_t> idx(n);
    for (int32_t k = 0; k < n; ++k) idx[k] = k;
    std::stable_sort(idx.begin(), idx.end(), [&](int32_t x, int32_t y) {
        return nets[x]->g_floats > nets[y]->g_floats;
    });
    const size_t lmax = max_lds_per_block();
    const char *env = std::getenv("PSST_LDS_G");
    const bool allow_lds = !(env && env[0] == '0');
    const char *shp = std::getenv("PSST_WG_SHAPE");
    const char *tenv = std::getenv("PSST_TUNE");
    const bool tune = !shp && !(tenv && tenv[0] == '0');
    Group gl;
    gl.lg = true;
    std::vector<Group> cls(tune ? kNumClasses : 1);
    bool any_syn = false, any_sparse = false, any_gabab = false;
    size_t need = 0;
    for (int32_t k : idx) {
        const psst_network *q = nets[k];
        if (!fits_wg(q)) continue;        // a per-stage sub-batch's instance
        if (!shp && net_lg(q)) {
            gl.order.push_back(k);
            gl.max_n = std::max(gl.max_n, q->n);
            gl.max_ld = std::max(gl.max_ld, q->ld);
            continue;
        }
        Group &t = cls[tune ? size_class(q->n) : 0];
        t.order.push_back(k);
        t.max_n = std::max(t.max_n, q->n);
        t.max_ld = std::max(t.max_ld, q->ld);
        need = std::max(need, wg_lds_bytes(false, q->ld, q->nch, 0));
        // networks without synapses need no LDS beyond the small buffers,
        // so several workgroups share a CU
        any_syn |= q->desc.n_paths > 0;
        any_sparse |= q->sparse;
        any_gabab |= q->gabab;
    }
    const size_t glds = (allow_lds && any_syn) ? lmax : need;
    for (Group &t : cls) {
        t.lds = glds;
        default_shape(t.max_n, &t.bs, &t.npt);
    }
    gl.bs = kLGThreads;
    gl.npt = kLGPairs;
    gl.lds = (size_t)kLGLdsBytes;
    // PSST_WG_SHAPE="<threads>x<neurons per thread>[r<register slots>]"
    // fixes the launch variant (and skips tuning) when it can take every
    // instance.
    if (shp) {
        int bs = 0, npt = 0, sl = 0;
        const int got = std::sscanf(shp, "%dx%dr%d", &bs, &npt, &sl);
        if (got >= 2 && find_variant(bs, npt, b->gen, false, got == 3 ? sl : 0) &&
            bs * npt >= cls[0].max_n && 4 * bs >= cls[0].max_ld) {
            cls[0].bs = bs;
            cls[0].npt = npt;
            cls[0].slots = got == 3 ? sl : 0;
        }
    }
    // launch-variant tuning on a scratch state: per size class, the fastest
    // variant on a full round of the class's largest instances, and the
    // fastest without register columns; then, when the two differ, the
    // batch's whole launch with either set of choices (classes run side by
    // side and share the chip, so their interplay decides).  Per-class
    // choices are cached per (architecture, size class, method, storage,
    // slow GABA, LDS, register columns allowed); the plan choice per the
    // same and the batch's class counts.
    std::vector<Group> merged;
    if (tune) {
        const std::string arch = device_arch();
        typedef TuneKey Key;
        std::mutex &tune_mu = g_tune_mu;
        std::map<TuneKey, ClassChoice> &tune_cache = g_tune_cache;
        std::map<PlanKey, int> &plan_cache = g_plan_cache;
        bool wrote = false;             // new entries to put in the table
        std::vector<Shape> plain(cls.size());
        std::vector<float> t_best(cls.size(), 0.f), t_plain(cls.size(), 0.f);
        std::vector<int> todo;
        std::vector<size_t> counts;
        for (const Group &t : cls) counts.push_back(t.order.size());
        counts.push_back(gl.order.size());
        const PlanKey pkey{arch, counts, b->gen, any_sparse, any_gabab, glds, rr_enabled()};
        int plan_cached = -1;
        {
            std::lock_guard<std::mutex> lock(tune_mu);
            read_tune_table(arch);
            for (int c = 0; c < kNumClasses; ++c) {
                Group &t = cls[c];
                if (t.order.empty()) continue;
                const Key key{arch, c, b->gen, any_sparse, any_gabab, glds, rr_enabled()};
                auto it = tune_cache.find(key);
                const Shape sb = it != tune_cache.end() ? it->second.best : Shape{};
                const Shape sp = it != tune_cache.end() ? it->second.plain : Shape{};
                if (it != tune_cache.end() &&
                    find_variant(sb.bs, sb.npt, b->gen, false, sb.slots) != nullptr &&
                    sb.bs * sb.npt >= t.max_n && 4 * sb.bs >= t.max_ld &&
                    find_variant(sp.bs, sp.npt, b->gen, false, 0) != nullptr &&
                    sp.bs * sp.npt >= t.max_n && 4 * sp.bs >= t.max_ld) {
                    t.bs = sb.bs;
                    t.npt = sb.npt;
                    t.slots = sb.slots;
                    plain[c] = sp;
                    t_best[c] = it->second.t_best;
                    t_plain[c] = it->second.t_plain;
                } else {
                    todo.push_back(c);
                }
            }
            auto pit = plan_cache.find(pkey);
            if (pit != plan_cache.end()) plan_cached = pit->second;
        }
        std::vector<Group> cls_plain = cls;
        // a class is a candidate for register columns when its fastest
        // variant holds them and beats the fastest one without by 10 % on a
        // full round of the class
        auto candidate = [&](size_t c) {
            return !cls[c].order.empty() && cls[c].slots && t_best[c] < 0.9f * t_plain[c];
        };
        auto plans_differ = [&]() {
            for (size_t c = 0; c < cls.size(); ++c)
                if (candidate(c)) return true;
            return false;
        };
        // scratch state for the timing runs; every buffer is released on
        // every path before an error is returned
        float *scratch = nullptr;
        float *v0 = nullptr;
        hipStream_t st = nullptr;
        auto release = [&]() {
            if (st) (void)hipStreamDestroy(st);
            (void)hipFree(scratch);
            (void)hipFree(v0);
            st = nullptr;
            scratch = v0 = nullptr;
        };
        auto setup = [&]() -> hipError_t {
            hipError_t e = hipMalloc(&scratch, sizeof(float) * 14 * b->nt);
            if (e == hipSuccess) e = hipMalloc(&v0, sizeof(float) * b->nt);
            if (e == hipSuccess) {
                std::vector<float> hv(b->nt, -65.f);
                e = hipMemcpy(v0, hv.data(), sizeof(float) * b->nt, hipMemcpyHostToDevice);
            }
            if (e == hipSuccess) e = hipStreamCreate(&st);
            if (e == hipSuccess && launch_init(b->d_desc, n, v0, scratch, b->nt, st) != PSST_OK)
                e = hipErrorLaunchFailure;
            return e;
        };
        hipError_t e = hipSuccess;
        if (!todo.empty() || (plan_cached < 0 && plans_differ())) e = setup();
        if (e == hipSuccess && !todo.empty()) {
            for (int c : todo) {
                if (s != PSST_OK || e != hipSuccess) break;
                Group &t = cls[c];
                e = hipMalloc(&t.d_order, sizeof(int32_t) * t.order.size());
                if (e == hipSuccess)
                    e = hipMemcpy(t.d_order, t.order.data(), sizeof(int32_t) * t.order.size(),
                                  hipMemcpyHostToDevice);
                if (e == hipSuccess)
                    s = tune_group(b, t, scratch, st, &plain[c], &t_best[c], &t_plain[c]);
                const hipError_t e2 = hipStreamSynchronize(st);
                if (e == hipSuccess) e = e2;
                (void)hipFree(t.d_order);
                t.d_order = nullptr;
            }
            if (e == hipSuccess && s == PSST_OK) {
                std::lock_guard<std::mutex> lock(tune_mu);
                for (int c : todo) {
                    const Group &t = cls[c];
                    tune_cache[Key{arch, c, b->gen, any_sparse, any_gabab, glds, rr_enabled()}] =
                        ClassChoice{Shape{t.bs, t.npt, t.slots}, plain[c], t_best[c], t_plain[c]};
                    wrote = true;
                }
            }
        }
        for (size_t c = 0; c < cls.size(); ++c) {
            cls_plain[c].bs = plain[c].bs;
            cls_plain[c].npt = plain[c].npt;
            cls_plain[c].slots = 0;
        }
        // which candidate classes take their register-column choice:
        // greedily, from the largest class down, a class switches when the
        // whole launch gets faster by at least 1 % (concurrent classes make
        // smaller differences noise)
        uint32_t mask = 0;
        auto plan_of = [&](uint32_t m) {
            std::vector<Group> pick(cls.size());
            for (size_t c = 0; c < cls.size(); ++c) pick[c] = (m >> c) & 1u ? cls[c] : cls_plain[c];
            return merge_classes(pick, gl);
        };
        if (e == hipSuccess && s == PSST_OK && plans_differ()) {
            if (plan_cached >= 0) {
                mask = (uint32_t)plan_cached;
            } else {
                std::vector<Group> p0 = plan_of(0);
                float best_t = 0.f;
                s = time_plan(b, p0, scratch, st, &best_t);
                if (tune_log() && s == PSST_OK)
                    std::fprintf(stderr, "psst tune: whole launch %.3f ms without register "
                                         "columns\n", best_t);
                for (int c = (int)cls.size() - 1; c >= 0 && s == PSST_OK; --c) {
                    if (!candidate((size_t)c)) continue;
                    const uint32_t trial = mask | (1u << c);
                    std::vector<Group> pt = plan_of(trial);
                    float t = 0.f;
                    s = time_plan(b, pt, scratch, st, &t);
                    if (s != PSST_OK) break;
                    if (tune_log())
                        std::fprintf(stderr, "psst tune: whole launch %.3f ms with register "
                                             "columns for n <= %d too\n", t, cls[c].max_n);
                    if (t < 0.99f * best_t) {
                        best_t = t;
                        mask = trial;
                    }
                }
                if (s == PSST_OK) {
                    std::lock_guard<std::mutex> lock(tune_mu);
                    plan_cache[pkey] = (int)mask;
                    wrote = true;
                }
            }
        }
        if (e == hipSuccess && scratch) e = hipStreamSynchronize(st);
        release();
        if (e != hipSuccess && s == PSST_OK)
            s = fail(e == hipErrorOutOfMemory ? PSST_ERR_OUT_OF_MEMORY : PSST_ERR_DEVICE,
                     "launch-shape tuning failed: %s", hipGetErrorString(e));
        if (s != PSST_OK) {
            batch_free(b);
            return s;
        }
        BCHK(hipMemset(b->d_flag, 0, sizeof(int32_t)));
        if (wrote && tune_write()) {
            std::lock_guard<std::mutex> lock(tune_mu);
            write_tune_table(arch);
        }
        merged = plan_of(mask);
    } else {
        merged = merge_classes(cls, gl);
    }
    for (const Group &t : merged) {
        b->groups.push_back(t);         // the batch owns (and frees) d_order
        Group &bg = b->groups.back();
        BCHK(hipMalloc(&bg.d_order, sizeof(int32_t) * bg.order.size()));
        BCHK(hipMemcpy(bg.d_order, bg.order.data(), sizeof(int32_t) * bg.order.size(),
                       hipMemcpyHostToDevice));
    }
#undef BCHK
    char buf[256];
    for (auto &g : b->groups) {
        char rr[48] = "";
        if (g.slots) snprintf(rr, sizeof rr, ", %d register slots", g.slots);
        snprintf(buf, sizeof buf, "[%zu inst, n<=%d, %s%d thr x %d neurons%s, lds %zu B] ",
                 g.order.size(), g.max_n, g.lg ? "lane-group, " : "", g.bs, g.npt, rr, g.lds);
        b->describe += buf;
    }
    b->describe_groups = b->describe;
    for (StageBatch *sb : b->subs) {
        b->describe += stage_batch_describe(sb);
        b->describe += " ";
    }
    *out = b;
    return PSST_OK;
}

extern "C" psst_status psst_batch_destroy(psst_batch *b)
{
    if (!b) return fail(PSST_ERR_INVALID_ARGUMENT, "batch is NULL");
    batch_free(b);
    return PSST_OK;
}

extern "C" psst_status psst_batch_layout(const psst_batch *b, int64_t *n_total, int64_t *n_words,
                                         int64_t *offsets)
{
    if (!b) return fail(PSST_ERR_INVALID_ARGUMENT, "batch is NULL");
    if (n_total) *n_total = b->nt;
    if (n_words) *n_words = 2LL * NVAR * b->nt;
    if (offsets) std::memcpy(offsets, b->offsets.data(), sizeof(int64_t) * (b->n + 1));
    return PSST_OK;
}

extern "C" psst_status psst_batch_describe(const psst_batch *b, char *buf, int32_t len)
{
    if (!b || !buf || len <= 0) return fail(PSST_ERR_INVALID_ARGUMENT, "bad argument");
    snprintf(buf, len, "%s", b->describe.c_str());
    return PSST_OK;
}

extern "C" psst_status psst_batch_conductance_bytes(const psst_batch *b, int64_t *resident,
                                                    int64_t *streamed)
{
    if (!b) return fail(PSST_ERR_INVALID_ARGUMENT, "batch is NULL");
    int64_t res = 0, str = 0;
    for (const StageBatch *sb : b->subs) str += stage_batch_matrix_bytes(sb);
    if (b->stage_path) {
        str = stage_batch_matrix_bytes(b->stage);
    } else {
        for (const Group &g : b->groups) {
            const WGVariant *v = group_variant(g, b->gen);
            const int slots = v ? v->slots : 0;
            for (int32_t k : g.order) {
                const psst_network *q = b->nets[k];
                if (q->desc.flags & DESC_NOSYN) continue;
                if (g.lg) {
                    // the lane-group kernel holds every conductance in registers
                    res += (int64_t)sizeof(float) * q->ld *
                           (q->n + (q->gabab ? q->n - q->n_pn : 0));
                    continue;
                }
                if (q->sparse) {
                    // ELL rows (column index and value, 8 bytes per entry) go to
                    // LDS for the launch when they fit beside the two
                    // activation vectors
                    const int64_t ents = (int64_t)(q->desc.sp_kf + q->desc.sp_kb) * q->ld;
                    const int64_t room = (int64_t)g.lds - (int64_t)sizeof(double) * 2 * q->ld;
                    (8 * ents <= room ? res : str) += 8 * ents;
                    continue;
                }
                // chunk widths: cholinergic columns, fast-GABA columns, slow
                // matrix, each cut at kChunkWidth; the first XR columns of
                // every chunk stay in registers and the next R in LDS
                int R = 0, XR = 0, KC = 0;
                wg_residency((int64_t)g.lds, q->ld, q->nch, g.bs, slots, &R, &XR, &KC);
                const int n_ln = q->n - q->n_pn;
                const int spans[3] = {q->n_pn, n_ln, q->gabab ? n_ln : 0};
                for (int t = 0; t < 3; ++t)
                    for (int j0 = 0; j0 < spans[t]; j0 += kChunkWidth) {
                        const int w = std::min(kChunkWidth, spans[t] - j0);
                        const int r = std::min(w, XR + R);
                        res += (int64_t)sizeof(float) * q->ld * r;
                        str += (int64_t)sizeof(float) * q->ld * (w - r);
                    }
            }
        }
    }
    if (resident) *resident = res;
    if (streamed) *streamed = str;
    return PSST_OK;
}

extern "C" psst_status psst_batch_state_init(const psst_batch *b, const float *v0, float *states,
                                             void *stream)
{
    if (!b || !v0 || !states) return fail(PSST_ERR_INVALID_ARGUMENT, "NULL argument");
    return launch_init(b->d_desc, b->n, v0, states, b->nt, (hipStream_t)stream);
}

// Build (first call) or update the graph holding one kernel node per group;
// (one node per launch group; a batch currently forms one group).
static psst_status submit_graph(psst_batch *b, std::vector<WGArgs> &args, hipStream_t s)
{
    const size_t G = b->groups.size();
    if (!b->exec) {
        HIPCHK(hipGraphCreate(&b->graph, 0));
        b->nodes.resize(G);
        b->node_args = args;
        for (size_t k = 0; k < G; ++k) {
            const Group &g = b->groups[k];
            const WGVariant *v = group_variant(g, b->gen);
            if (!v) return fail(PSST_ERR_UNSUPPORTED, "no kernel variant");
            psst_status st = set_lds_attr(v->fn, g.lds);
            if (st != PSST_OK) return st;
            void *kp[] = {&b->node_args[k]};
            hipKernelNodeParams p{};
            p.func = const_cast<void *>(v->fn);
            p.gridDim = dim3((unsigned)g.order.size());
            p.blockDim = dim3(g.bs);
            p.sharedMemBytes = (unsigned)g.lds;
            p.kernelParams = kp;
            p.extra = nullptr;
            HIPCHK(hipGraphAddKernelNode(&b->nodes[k], b->graph, nullptr, 0, &p));
        }
        HIPCHK(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    } else {
        for (size_t k = 0; k < G; ++k) {
            if (std::memcmp(&b->node_args[k], &args[k], sizeof(WGArgs)) == 0) continue;
            b->node_args[k] = args[k];
            const Group &g = b->groups[k];
            const WGVariant *v = group_variant(g, b->gen);
            if (!v) return fail(PSST_ERR_UNSUPPORTED, "no kernel variant");
            void *kp[] = {&b->node_args[k]};
            hipKernelNodeParams p{};
            p.func = const_cast<void *>(v->fn);
            p.gridDim = dim3((unsigned)g.order.size());
            p.blockDim = dim3(g.bs);
            p.sharedMemBytes = (unsigned)g.lds;
            p.kernelParams = kp;
            p.extra = nullptr;
            HIPCHK(hipGraphExecKernelNodeSetParams(b->exec, b->nodes[k], &p));
        }
    }
    HIPCHK(hipGraphLaunch(b->exec, s));
    return PSST_OK;
}

extern "C" psst_status psst_integrate_batch(psst_batch *b, float *states, const psst_stimulus *stim,
                                            float dt, int64_t n_steps, int64_t step0,
                                            const psst_record *rec, float *ckpt, int32_t K,
                                            void *stream)
{
    if (!b) return fail(PSST_ERR_INVALID_ARGUMENT, "batch is NULL");
    if (!states) return fail(PSST_ERR_INVALID_ARGUMENT, "states is NULL");
    psst_status s = validate_common(dt, n_steps, step0, rec);
    if (s != PSST_OK) return s;
    if ((s = validate_stim(stim)) != PSST_OK) return s;
    if (ckpt && K <= 0) return fail(PSST_ERR_INVALID_ARGUMENT, "checkpoints need K > 0");
    if (b->stage_path)
        return stage_batch_integrate(b->stage, states, stim, dt, n_steps, step0, rec, ckpt, K,
                                     stream);
    if (ckpt && !b->subs.empty())
        return fail(PSST_ERR_UNSUPPORTED, "checkpoints are not supported on the per-stage path");
    if (n_steps == 0) return PSST_OK;
    if (!b->groups.empty()) {
        std::vector<WGArgs> args;
        for (auto &g : b->groups)
            args.push_back(group_args(b, g, states, stim, dt, n_steps, step0, rec, ckpt, K));
        if ((s = submit_graph(b, args, (hipStream_t)stream)) != PSST_OK) return s;
    }
    for (StageBatch *sb : b->subs)
        if ((s = stage_batch_integrate(sb, states, stim, dt, n_steps, step0, rec, nullptr, 0,
                                       stream)) != PSST_OK)
            return s;
    return PSST_OK;
}

// The batch's launches without the graph (the streamed path issues one per
// chunk while earlier chunks are in flight; changing the graph's parameters
// would wait for them).
psst_status batch_launch_direct(psst_batch *b, float *states, const psst_stimulus *stim, float dt,
                                int64_t n_steps, int64_t step0, const psst_record *rec,
                                void *stream)
{
    psst_status s = validate_common(dt, n_steps, step0, rec);
    if (s != PSST_OK) return s;
    if ((s = validate_stim(stim)) != PSST_OK) return s;
    if (n_steps == 0) return PSST_OK;
    if (b->stage_path)        // the per-stage graph: parameters go through its control block
        return stage_batch_integrate(b->stage, states, stim, dt, n_steps, step0, rec, nullptr, 0,
                                     stream);
    // the launch groups side by side, as in the graph: the heaviest on the
    // caller's stream, the next on streams of their own forked from it and
    // joined back, at most kDirectAux of them -- with the caller's stream and
    // a copy stream that keeps the streams within the device's four hardware
    // queues (streams beyond them share a queue and run one after another);
    // the last of them takes the remaining groups in turn
    constexpr size_t kDirectAux = 2;
    const hipStream_t st = (hipStream_t)stream;
    const size_t G = b->groups.size();
    const size_t S = std::min(G, 1 + kDirectAux);     // streams in use
    if (S > 1 && b->aux.size() < S - 1) {
        if (!b->aux_fork) HIPCHK(hipEventCreateWithFlags(&b->aux_fork, hipEventDisableTiming));
        while (b->aux.size() < S - 1) {
            hipStream_t a = nullptr;
            HIPCHK(hipStreamCreateWithFlags(&a, hipStreamNonBlocking));
            b->aux.push_back(a);
            hipEvent_t e = nullptr;
            HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
            b->aux_done.push_back(e);
        }
    }
    for (StageBatch *sb : b->subs)
        if ((s = stage_batch_integrate(sb, states, stim, dt, n_steps, step0, rec, nullptr, 0,
                                       stream)) != PSST_OK)
            return s;
    // groups by decreasing work (sum of n^2 over their instances)
    std::vector<size_t> rank(G);
    std::vector<double> work(G, 0.0);
    for (size_t k = 0; k < G; ++k) {
        rank[k] = k;
        for (int32_t i : b->groups[k].order) work[k] += (double)b->nets[i]->n * b->nets[i]->n;
    }
    std::stable_sort(rank.begin(), rank.end(), [&](size_t x, size_t y) { return work[x] > work[y]; });
    if (S > 1) HIPCHK(hipEventRecord(b->aux_fork, st));
    for (size_t a = 0; a + 1 < S; ++a) HIPCHK(hipStreamWaitEvent(b->aux[a], b->aux_fork, 0));
    for (size_t r = 0; r < G; ++r) {
        const Group &g = b->groups[rank[r]];
        const size_t si = std::min(r, S - 1);
        const hipStream_t gs = si == 0 ? st : b->aux[si - 1];
        WGArgs a = group_args(b, g, states, stim, dt, n_steps, step0, rec, nullptr, 1);
        if ((s = launch_group(g, b->gen, a, gs)) != PSST_OK) return s;
    }
    for (size_t a = 0; a + 1 < S; ++a) {
        HIPCHK(hipEventRecord(b->aux_done[a], b->aux[a]));
        HIPCHK(hipStreamWaitEvent(st, b->aux_done[a], 0));
    }
    return PSST_OK;
}

extern "C" psst_status psst_batch_poll(psst_batch *b, void *stream)
{
    if (!b) return fail(PSST_ERR_INVALID_ARGUMENT, "batch is NULL");
    if (b->stage_path) return stage_batch_poll(b->stage, stream);
    return poll_flag(b->d_flag, stream);
}

// The forward kernels of a batch as the adjoint's recomputation: each launch
// group over n_steps steps from the checkpoint row, nothing stored back,
// stage records to the stash.
static RecomputeFn batch_recompute(psst_batch *b, const psst_stimulus *stim, float dt)
{
    return [b, stim, dt](const float *ckpt_row, int64_t step0, int64_t n_steps, double *stash,
                         int64_t stash_stride, int32_t K, hipStream_t s) -> psst_status {
        for (const Group &g : b->groups) {
            WGArgs a = group_args(b, g, nullptr, stim, dt, n_steps, step0, nullptr, nullptr, 1);
            a.state_in = ckpt_row;
            a.store_state = 0;
            a.stash = stash;
            a.stash_stride = stash_stride;
            a.stash_K = K;
            psst_status st = launch_group(g, b->gen, a, s);
            if (st != PSST_OK) return st;
        }
        return PSST_OK;
    };
}

// The adjoint's lean recomputation: every instance in one launch of a
// per-instance variant (no lane-group kernel, no register columns) with only
// the activation and partial-sum buffers in LDS -- the conductances stream
// from L2 -- so that it fits on a compute unit beside the reverse sweep.  Its
// sums follow the same column order as every other mapping (same bits).
static psst_status ensure_lean(psst_batch *b)
{
    Group &g = b->lean;
    if (g.d_order) return PSST_OK;
    g = Group{};
    for (const Group &t : b->groups) g.order.insert(g.order.end(), t.order.begin(), t.order.end());
    std::stable_sort(g.order.begin(), g.order.end(), [&](int32_t x, int32_t y) {
        return b->nets[x]->g_floats > b->nets[y]->g_floats;
    });
    size_t need = 0;
    for (int32_t k : g.order) {
        const psst_network *q = b->nets[k];
        g.max_n = std::max(g.max_n, q->n);
        g.max_ld = std::max(g.max_ld, q->ld);
        need = std::max(need, wg_lds_bytes(false, q->ld, q->nch, 0));
    }
    g.lds = need;
    default_shape(g.max_n, &g.bs, &g.npt);
    if (!find_variant(g.bs, g.npt, false) || !find_variant(g.bs, g.npt, true))
        return fail(PSST_ERR_UNSUPPORTED, "no kernel variant for the adjoint's recomputation");
    int32_t *d = nullptr;
    HIPCHK(hipMalloc(&d, sizeof(int32_t) * g.order.size()));
    hipError_t e = hipMemcpy(d, g.order.data(), sizeof(int32_t) * g.order.size(),
                             hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(d);
        return fail(PSST_ERR_DEVICE, "hipMemcpy failed: %s", hipGetErrorString(e));
    }
    g.d_order = d;
    return PSST_OK;
}

static RecomputeFn batch_recompute_lean(psst_batch *b, const psst_stimulus *stim, float dt)
{
    return [b, stim, dt](const float *ckpt_row, int64_t step0, int64_t n_steps, double *stash,
                         int64_t stash_stride, int32_t K, hipStream_t s) -> psst_status {
        const Group &g = b->lean;
        WGArgs a = group_args(b, g, nullptr, stim, dt, n_steps, step0, nullptr, nullptr, 1);
        a.state_in = ckpt_row;
        a.store_state = 0;
        a.stash = stash;
        a.stash_stride = stash_stride;
        a.stash_K = K;
        return launch_group(g, b->gen, a, s);
    };
}

extern "C" psst_status psst_adjoint(psst_batch *b, const float *ckpt, int32_t K,
                                    const psst_stimulus *stim, float dt, int64_t n_steps,
                                    int64_t step0, const float *dLdV, float *grad_g,
                                    float *grad_gNa, float *grad_gK, float *grad_gL,
                                    int32_t per_instance, void *stream)
{
    if (!b) return fail(PSST_ERR_INVALID_ARGUMENT, "batch is NULL");
    if (!ckpt || !dLdV || !grad_g || !grad_gNa || !grad_gK || !grad_gL)
        return fail(PSST_ERR_INVALID_ARGUMENT, "NULL buffer");
    if (K <= 0) return fail(PSST_ERR_INVALID_ARGUMENT, "K must be > 0");
    psst_status s = validate_common(dt, n_steps, step0, nullptr);
    if (s != PSST_OK) return s;
    if ((s = validate_stim(stim)) != PSST_OK) return s;
    if (!per_instance && !b->shared)
        return fail(PSST_ERR_INVALID_ARGUMENT, "summed gradients need every instance to share one network");
    if (b->stage_path || !b->subs.empty())
        return fail(PSST_ERR_UNSUPPORTED, "the adjoint is not available on the per-stage path");
    const int64_t max_n = b->nets.empty() ? 0 : (*std::max_element(
        b->nets.begin(), b->nets.end(),
        [](const psst_network *x, const psst_network *y) { return x->n < y->n; }))->n;
    if (max_n <= 512 && (s = ensure_lean(b)) != PSST_OK) return s;
    const RecomputeFn lean = batch_recompute_lean(b, stim, dt);
    return adjoint_run(b->nets, b->d_desc, b->nt, &b->adj, batch_recompute(b, stim, dt), ckpt, K,
                       stim, dt, n_steps,
                       step0, dLdV, grad_g, grad_gNa, grad_gK, grad_gL, per_instance, b->d_flag,
                       max_lds_per_block(), b->gen, b->tab, stream,
                       b->lean.d_order ? &lean : nullptr,
                       ((b->lean.lds + 4095) & ~(size_t)4095) + 4096);
}

extern "C" psst_status psst_adjoint_noalloc(psst_batch *b, const float *ckpt, int32_t K,
                                            const psst_stimulus *stim, float dt,
                                            int64_t n_steps, int64_t step0, const float *dLdV,
                                            float *grad_g, float *grad_gNa, float *grad_gK,
                                            float *grad_gL, int32_t per_instance, void *stream)
{
    if (!b) return fail(PSST_ERR_INVALID_ARGUMENT, "batch is NULL");
    if (!ckpt || !dLdV || !grad_g || !grad_gNa || !grad_gK || !grad_gL)
        return fail(PSST_ERR_INVALID_ARGUMENT, "NULL buffer");
    if (K <= 0) return fail(PSST_ERR_INVALID_ARGUMENT, "K must be > 0");
    psst_status s = validate_common(dt, n_steps, step0, nullptr);
    if (s != PSST_OK) return s;
    if ((s = validate_stim(stim)) != PSST_OK) return s;
    if (!per_instance && !b->shared)
        return fail(PSST_ERR_INVALID_ARGUMENT, "summed gradients need every instance to share one network");
    if (b->stage_path || !b->subs.empty())
        return fail(PSST_ERR_UNSUPPORTED, "the adjoint is not available on the per-stage path");
    return adjoint_run_noalloc(b->nets, b->d_desc, b->nt, batch_recompute(b, stim, dt), ckpt, K,
                               stim, dt, n_steps, step0, dLdV,
                               grad_g, grad_gNa, grad_gK, grad_gL, per_instance, b->d_flag,
                               max_lds_per_block(), b->gen, b->tab, stream);
}

// ---------------------------------------------------------------------------
// explicit Runge-Kutta tableaux
// ---------------------------------------------------------------------------

// Check the rules of psst_tableau; on success *gen says whether it differs
// from classical RK4 and *t holds its device form.
static psst_status read_tableau(const psst_tableau *tab, bool *gen, psst::Tab *t)
{
    *gen = false;
    *t = psst::Tab{};
    if (!tab) return PSST_OK;
    const int S = tab->stages;
    if (S < 1 || S > 4) return fail(PSST_ERR_INVALID_ARGUMENT, "tableau: stages=%d not in 1..4", S);
    for (int i = 0; i < 4; ++i) {
        for (int q = 0; q < 4; ++q) {
            const double v = tab->a[i][q];
            if (!std::isfinite(v)) return fail(PSST_ERR_INVALID_ARGUMENT, "tableau: a[%d][%d] not finite", i, q);
            if ((q >= i || i >= S) && v != 0.0)
                return fail(PSST_ERR_INVALID_ARGUMENT,
                            "tableau: a[%d][%d] must be 0 (explicit, %d stages)", i, q, S);
        }
        if (!std::isfinite(tab->b[i])) return fail(PSST_ERR_INVALID_ARGUMENT, "tableau: b[%d] not finite", i);
        if (i >= S && tab->b[i] != 0.0) return fail(PSST_ERR_INVALID_ARGUMENT, "tableau: b[%d] must be 0", i);
    }
    const bool rk4 = S == 4 && tab->a[1][0] == 0.5 && tab->a[2][0] == 0.0 &&
                     tab->a[2][1] == 0.5 && tab->a[3][0] == 0.0 && tab->a[3][1] == 0.0 &&
                     tab->a[3][2] == 1.0 && tab->b[0] == 1.0 / 6.0 && tab->b[1] == 1.0 / 3.0 &&
                     tab->b[2] == 1.0 / 3.0 && tab->b[3] == 1.0 / 6.0;
    if (rk4) return PSST_OK;
    *gen = true;
    t->s = S;
    for (int i = 0; i < 4; ++i) {
        for (int q = 0; q < 4; ++q) t->a[i][q] = tab->a[i][q];
        t->b[i] = tab->b[i];
    }
    return PSST_OK;
}

extern "C" psst_status psst_network_set_tableau(psst_network *net, const psst_tableau *tab)
{
    if (!net) return fail(PSST_ERR_INVALID_ARGUMENT, "network is NULL");
    bool gen;
    psst::Tab t;
    psst_status s = read_tableau(tab, &gen, &t);
    if (s != PSST_OK) return s;
    net->gen = gen;
    net->tab = t;
    if (net->single) stage_batch_set_method(net->single, gen, t);   // plain calls, large network
    return PSST_OK;
}

extern "C" psst_status psst_batch_set_tableau(psst_batch *b, const psst_tableau *tab)
{
    if (!b) return fail(PSST_ERR_INVALID_ARGUMENT, "batch is NULL");
    bool gen;
    psst::Tab t;
    psst_status s = read_tableau(tab, &gen, &t);
    if (s != PSST_OK) return s;
    if (b->stage_path) {
        stage_batch_set_method(b->stage, gen, t);
        b->describe = stage_batch_describe(b->stage);
    }
    if (!b->subs.empty()) {
        b->describe = b->describe_groups;
        for (StageBatch *sb : b->subs) {
            stage_batch_set_method(sb, gen, t);
            b->describe += stage_batch_describe(sb);
            b->describe += " ";
        }
    }
    if (gen != b->gen && b->exec) {
        // the graph's kernel changes: build it again on the next call
        HIPCHK(hipGraphExecDestroy(b->exec));
        HIPCHK(hipGraphDestroy(b->graph));
        b->exec = nullptr;
        b->graph = nullptr;
    }
    b->gen = gen;
    b->tab = t;
    return PSST_OK;
}
