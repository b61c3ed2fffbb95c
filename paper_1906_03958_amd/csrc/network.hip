// network.hip -- in-place update of a network's conductances.
//
// The gradient of the method's adjoint ("Brain simulations as computational
// graphs": gradients of a loss of the simulated traces by backpropagation
// through the unrolled RK4 steps) is taken with respect to the synaptic
// conductance blocks and the intrinsic conductances g_Na, g_K, g_L.  A
// descent step changes only those values, so the network's device storage
// is rewritten where it lies instead of being built again from host arrays:
// one launch scatters the pathway blocks (gradient layout: block after block
// in pathway order, each [post x pre] row-major) into every storage the
// network keeps --
//   dense per-instance storage   gt[j * ld + i] (fast GABA and ACh) and
//                                gtb[(j - n_pn) * ld + i] (slow GABA);
//   sparse rows                  val[slot(e)] for the entry's ELL slot;
//   per-stage layout             G[i * Kp + k(type, j)], or the synapse
//                                buckets of its sparse form;
// absent synapses (mask 0) keep their zero, and the intrinsic vectors go to
// rows g_Na, g_K, g_L of the parameter table.

#include <hip/hip_runtime.h>

#include "runtime.h"

namespace {

__global__ __launch_bounds__(256) void network_update_kernel(psst::NetUpdateArgs a)
{
    const int64_t total = a.entries + 3LL * a.n;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        if (e >= a.entries) {
            const int64_t r = e - a.entries;
            const int k = (int)(r / a.n), i = (int)(r % a.n);
            const float *src = k == 0 ? a.g_na : (k == 1 ? a.g_k : a.g_l);
            if (src) a.prm[(int64_t)(1 + k) * a.ld + i] = src[i];
            continue;
        }
        if (!a.g) continue;
        int q = 0;
        while (q + 1 < a.n_paths && a.paths[6 * (q + 1) + 5] <= e) ++q;
        const int64_t *w = a.paths + 6 * q;
        const int type = (int)w[0];
        const int64_t npre = w[2] - w[1], r = e - w[5];
        const int i = (int)(w[3] + r / npre), j = (int)(w[1] + r % npre);
        const bool present = !a.present_bits || ((a.present_bits[e >> 5] >> (e & 31)) & 1u);
        const float v = present ? a.g[e] : 0.f;
        if (a.gt) {
            if (type == PSST_SYN_GABA_B) a.gtb[(int64_t)(j - a.n_pn) * a.ld + i] = v;
            else a.gt[(int64_t)j * a.ld + i] = v;
        }
        if (a.sp_val) {
            const int32_t slot = a.sp_slot[e];
            if (slot >= 0) a.sp_val[slot] = v;
        }
        if (a.stage_G || a.bk_val) {
            const int64_t k = type == PSST_SYN_ACH ? j
                              : (type == PSST_SYN_GABA_A ? a.stage_ka + (j - a.n_pn)
                                                         : a.stage_ka + a.stage_kg + (j - a.n_pn));
            if (a.stage_G) a.stage_G[(int64_t)i * a.stage_Kp + k] = v;
            if (a.bk_val && present) {
                // the synapse's bucket (64-row block, 128-column tile, row)
                // holds ascending columns: binary search
                const int64_t ntl = a.stage_Kp / 128;
                const int64_t bk = ((int64_t)(i / 64) * ntl + k / 128) * 64 + i % 64;
                int lo = a.bk_off[bk], hi = a.bk_off[bk + 1];
                const int c = (int)(k % 128);
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (a.bk_col[mid] < c) lo = mid + 1;
                    else hi = mid;
                }
                if (lo < a.bk_off[bk + 1] && a.bk_col[lo] == c) a.bk_val[lo] = v;
            }
        }
    }
}

}  // namespace

psst_status network_update_launch(const psst::NetUpdateArgs &a, hipStream_t s)
{
    const int64_t total = a.entries + 3LL * a.n;
    if (total == 0) return PSST_OK;
    const int64_t blocks = std::min<int64_t>((total + 255) / 256, 8192);
    hipLaunchKernelGGL(network_update_kernel, dim3((unsigned)blocks), dim3(256), 0, s, a);
    HIPCHK(hipGetLastError());
    return PSST_OK;
}
