// streaming.cpp -- long batched runs with their records drained to host
// memory chunk by chunk (psst_integrate_batch_streamed): two device record
// buffers and two pinned staging buffers alternate so that the copy-out of
// one chunk overlaps the integration of the next.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <thread>
#include <vector>

#include "runtime.h"

using psst::fail;

namespace {

struct Side {                        // one of the two alternating buffer sets
    float *d_v = nullptr, *h_v = nullptr;
    int32_t *d_cnt = nullptr, *h_cnt = nullptr;
    float *d_spk = nullptr, *h_spk = nullptr;
    size_t v_bytes = 0, cnt_bytes = 0, spk_bytes = 0;   // allocated sizes
    hipEvent_t computed = nullptr, copied = nullptr;
    int64_t chunk = -1;              // chunk whose records it holds (-1: none)
    int64_t rows = 0;
};

// device and pinned host buffers of one batch, kept between calls and grown
// on demand (pinning host memory costs far more than a chunk's copy)
static psst_status grow(void **d, void **h, size_t *have, size_t need)
{
    if (need <= *have) return PSST_OK;
    (void)hipFree(*d);
    (void)hipHostFree(*h);
    *d = nullptr;
    *h = nullptr;
    *have = 0;
    HIPCHK(hipMalloc(d, need));
    HIPCHK(hipHostMalloc(h, need, hipHostMallocDefault));
    *have = need;
    return PSST_OK;
}

// staging -> caller copy of a chunk's trace: one thread moves a few GB/s, a
// chunk of the 1.1 M-neuron batch is ~0.4 GB, so large copies are split over
// several threads to stay shorter than the next chunk's integration
static void host_copy(void *dst, const void *src, size_t bytes)
{
    constexpr size_t kMinPart = size_t(16) << 20;
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const size_t parts = std::min<size_t>(std::min(8u, hw), std::max<size_t>(1, bytes / kMinPart));
    if (parts <= 1) {
        std::memcpy(dst, src, bytes);
        return;
    }
    const size_t step = (bytes / parts + 4095) & ~size_t(4095);
    std::vector<std::thread> pool;
    for (size_t k = 1; k < parts; ++k) {
        const size_t off = k * step;
        if (off >= bytes) break;
        const size_t len = std::min(step, bytes - off);
        pool.emplace_back([=] { std::memcpy((char *)dst + off, (const char *)src + off, len); });
    }
    std::memcpy(dst, src, std::min(step, bytes));
    for (auto &t : pool) t.join();
}

}  // namespace

struct StreamBufs {
    Side side[2];
    hipStream_t copy = nullptr;
    ~StreamBufs()
    {
        if (copy) {
            (void)hipStreamSynchronize(copy);
            (void)hipStreamDestroy(copy);
        }
        for (Side &s : side) {
            (void)hipFree(s.d_v);
            (void)hipFree(s.d_cnt);
            (void)hipFree(s.d_spk);
            (void)hipHostFree(s.h_v);
            (void)hipHostFree(s.h_cnt);
            (void)hipHostFree(s.h_spk);
            if (s.computed) (void)hipEventDestroy(s.computed);
            if (s.copied) (void)hipEventDestroy(s.copied);
        }
    }
};

void stream_bufs_free(StreamBufs *s) { delete s; }

extern "C" psst_status psst_integrate_batch_streamed(psst_batch *b, float *states,
                                                     const psst_stimulus *stim, float dt,
                                                     int64_t n_steps, int64_t step0,
                                                     int64_t chunk, int64_t stride, float *host_v,
                                                     int32_t *host_cnt, float *host_spk,
                                                     int32_t cap, void *stream)
{
    if (!b) return fail(PSST_ERR_INVALID_ARGUMENT, "batch is NULL");
    if (!states) return fail(PSST_ERR_INVALID_ARGUMENT, "states is NULL");
    if (n_steps < 0 || step0 < 0) return fail(PSST_ERR_INVALID_ARGUMENT, "n_steps and step0 must be >= 0");
    if (chunk <= 0) return fail(PSST_ERR_INVALID_ARGUMENT, "chunk_steps must be > 0");
    if (host_v && (stride <= 0 || chunk % stride != 0 || step0 % stride != 0))
        return fail(PSST_ERR_INVALID_ARGUMENT,
                    "rec_stride must be > 0 and divide chunk_steps and step0");
    if (host_cnt && cap < 0) return fail(PSST_ERR_INVALID_ARGUMENT, "spike_cap < 0");
    if (host_cnt && cap > 0 && !host_spk)
        return fail(PSST_ERR_INVALID_ARGUMENT, "spike_cap > 0 needs host_spike_t");
    if (n_steps == 0) return PSST_OK;
    const int64_t nt = b->nt;
    const int64_t rows_max = host_v ? chunk / stride : 0;
    const hipStream_t cs = (hipStream_t)stream;

    if (!b->strm) b->strm = new StreamBufs();
    StreamBufs &S = *b->strm;
    // non-blocking: the caller's stream may be the null stream, which would
    // otherwise wait for every copy
    if (!S.copy) HIPCHK(hipStreamCreateWithFlags(&S.copy, hipStreamNonBlocking));
    psst_status st = PSST_OK;
    for (Side &s : S.side) {
        if (host_v && (st = grow((void **)&s.d_v, (void **)&s.h_v, &s.v_bytes,
                                 sizeof(float) * rows_max * nt)) != PSST_OK)
            return st;
        if (host_cnt && (st = grow((void **)&s.d_cnt, (void **)&s.h_cnt, &s.cnt_bytes,
                                   sizeof(int32_t) * nt)) != PSST_OK)
            return st;
        if (host_cnt && cap > 0 && (st = grow((void **)&s.d_spk, (void **)&s.h_spk, &s.spk_bytes,
                                              sizeof(float) * nt * cap)) != PSST_OK)
            return st;
        if (!s.computed) HIPCHK(hipEventCreateWithFlags(&s.computed, hipEventDisableTiming));
        if (!s.copied) HIPCHK(hipEventCreateWithFlags(&s.copied, hipEventDisableTiming));
        s.chunk = -1;
    }

    // host side of one finished chunk: staging -> the caller's arrays
    auto drain = [&](Side &s, int64_t c_done, int64_t rows) -> psst_status {
        if (c_done < 0) return PSST_OK;
        HIPCHK(hipEventSynchronize(s.copied));
        if (host_v && rows > 0)
            host_copy(host_v + (c_done * chunk / stride) * nt, s.h_v, sizeof(float) * rows * nt);
        if (host_cnt) {
            for (int64_t i = 0; i < nt; ++i) {
                const int32_t k = s.h_cnt[i];
                if (k <= 0) continue;
                const int32_t base = host_cnt[i];
                for (int32_t m = 0; m < k && m < cap && base + m < cap; ++m)
                    host_spk[i * cap + base + m] = s.h_spk[i * cap + m];
                host_cnt[i] = base + k;
            }
        }
        return PSST_OK;
    };

    // chunk c: its integration is queued first (after the copy-out of chunk
    // c - 2, which used the same device buffers, on the device side), then
    // the host drains chunk c - 2 while chunk c integrates, then chunk c's
    // copy-out is queued behind its integration
    const int64_t n_chunks = (n_steps + chunk - 1) / chunk;
    for (int64_t c = 0; c < n_chunks && st == PSST_OK; ++c) {
        Side &s = S.side[c & 1];
        const int64_t prev = s.chunk, prev_rows = s.rows;
        if (prev >= 0) HIPCHK(hipStreamWaitEvent(cs, s.copied, 0));
        const int64_t len = std::min(chunk, n_steps - c * chunk);
        const int64_t s0 = step0 + c * chunk;
        const int64_t rows = host_v ? (s0 + len) / stride - s0 / stride : 0;
        if (host_cnt) HIPCHK(hipMemsetAsync(s.d_cnt, 0, sizeof(int32_t) * nt, cs));
        psst_record rec{};
        rec.v_out = host_v ? s.d_v : nullptr;
        rec.stride = host_v ? stride : 0;
        rec.capacity = rows;
        rec.spike_count = host_cnt ? s.d_cnt : nullptr;
        rec.spike_t_ms = host_cnt && cap > 0 ? s.d_spk : nullptr;
        rec.spike_cap = host_cnt ? cap : 0;
        if ((st = batch_launch_direct(b, states, stim, dt, len, s0, &rec, stream)) != PSST_OK)
            break;
        HIPCHK(hipEventRecord(s.computed, cs));
        if ((st = drain(s, prev, prev_rows)) != PSST_OK) break;   // chunk c - 2's records
        s.chunk = -1;
        HIPCHK(hipStreamWaitEvent(S.copy, s.computed, 0));
        if (host_v && rows > 0)
            HIPCHK(hipMemcpyAsync(s.h_v, s.d_v, sizeof(float) * rows * nt,
                                  hipMemcpyDeviceToHost, S.copy));
        if (host_cnt) {
            HIPCHK(hipMemcpyAsync(s.h_cnt, s.d_cnt, sizeof(int32_t) * nt, hipMemcpyDeviceToHost,
                                  S.copy));
            if (cap > 0)
                HIPCHK(hipMemcpyAsync(s.h_spk, s.d_spk, sizeof(float) * nt * cap,
                                      hipMemcpyDeviceToHost, S.copy));
        }
        HIPCHK(hipEventRecord(s.copied, S.copy));
        s.chunk = c;
        s.rows = rows;
    }
    // the last two chunks, in order
    for (int64_t c = std::max<int64_t>(0, n_chunks - 2); c < n_chunks && st == PSST_OK; ++c) {
        Side &s = S.side[c & 1];
        st = drain(s, s.chunk, s.rows);
        s.chunk = -1;
    }
    if (st != PSST_OK) {
        (void)hipStreamSynchronize(cs);
        (void)hipStreamSynchronize(S.copy);   // no copy into the staging buffers outlives the call
        return st;
    }
    return psst_batch_poll(b, stream);
}
