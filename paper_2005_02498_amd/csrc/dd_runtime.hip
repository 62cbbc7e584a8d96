// Host runtime of libdd.so: error reporting, per-device workspace, the
// Gauss-Legendre rule, version/validation switches.
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <mutex>
#include <vector>

#include "dd_common.h"

namespace dd {

namespace {
thread_local char g_msg[1024] = "";
std::atomic<int> g_validate{1};
std::mutex g_ws_mu;
std::vector<Workspace *> g_ws;   // indexed by device ordinal

// event timing of the all-pairs kernel
std::atomic<int> g_timing{0};
std::vector<hipEvent_t> g_ev;    // start/stop pairs, reused
size_t g_ev_used = 0;            // events recorded since the last reset
}  // namespace

bool timing_on() { return g_timing.load() != 0; }

static hipEvent_t next_event()
{
    if (g_ev_used >= g_ev.size()) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        g_ev.push_back(e);
    }
    return g_ev[g_ev_used++];
}

void timing_begin(hipStream_t st, bool capturing)
{
    if (!timing_on() || capturing) return;
    if (g_ev_used % 2) return;   // unmatched begin: ignore
    hipEvent_t e = next_event();
    if (e) (void)hipEventRecord(e, st);
}

void timing_end(hipStream_t st, bool capturing)
{
    if (!timing_on() || capturing) return;
    if (g_ev_used % 2 == 0) return;
    hipEvent_t e = next_event();
    if (e) (void)hipEventRecord(e, st);
    else --g_ev_used;   // drop the unmatched start
}

int set_error(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_msg, sizeof g_msg, fmt, ap);
    va_end(ap);
    return code;
}

void clear_error() { g_msg[0] = 0; }

bool validation_on() { return g_validate.load() != 0; }

int workspace(Workspace **out)
{
    int dev = 0;
    DD_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_ws_mu);
    if ((int)g_ws.size() <= dev) g_ws.resize(dev + 1, nullptr);
    if (!g_ws[dev]) {
        Workspace *w = new Workspace();
        w->device = dev;
        if (hipMalloc(&w->flags_dev, 256) != hipSuccess) {
            delete w;
            return set_error(DD_ENOMEM, "hipMalloc of the flag word failed");
        }
        w->near_count = (unsigned long long *)((char *)w->flags_dev + 128);
        if (hipMemset(w->flags_dev, 0, 256) != hipSuccess) {
            (void)hipFree(w->flags_dev);
            delete w;
            return set_error(DD_EHIP, "hipMemset of the flag word failed");
        }
        if (hipHostMalloc(&w->flags_host, 256, hipHostMallocDefault) != hipSuccess) {
            (void)hipFree(w->flags_dev);
            delete w;
            return set_error(DD_ENOMEM, "hipHostMalloc of the flag mirror failed");
        }
        g_ws[dev] = w;
    }
    *out = g_ws[dev];
    return DD_OK;
}

int ensure(Workspace *ws, Slot s, size_t bytes, void **out)
{
    if (bytes == 0) bytes = 256;
    if (ws->cap[s] < bytes) {
        size_t want = bytes + bytes / 4;
        want = (want + 255) & ~size_t(255);
        if (ws->ptr[s]) {
            // an earlier call may still be reading it
            DD_HIP(hipDeviceSynchronize());
            DD_HIP(hipFree(ws->ptr[s]));
            ws->ptr[s] = nullptr;
            ws->cap[s] = 0;
        }
        if (hipMalloc(&ws->ptr[s], want) != hipSuccess) {
            (void)hipGetLastError();
            ws->ptr[s] = nullptr;
            return set_error(DD_ENOMEM, "hipMalloc(%zu bytes) for workspace slot %d failed", want, (int)s);
        }
        ws->cap[s] = want;
    }
    *out = ws->ptr[s];
    return DD_OK;
}

void drop_graphs(Workspace *ws)
{
    if (ws->graphs.empty()) return;
    (void)hipDeviceSynchronize();
    for (auto &g : ws->graphs)
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    ws->graphs.clear();
}

}  // namespace dd

extern "C" {

const char *dd_last_error(void) { return dd::g_msg; }

int dd_version(void) { return 1 * 10000 + 0 * 100 + 0; }

int dd_set_validation(int on) { return dd::g_validate.exchange(on ? 1 : 0); }

int dd_timing_enable(int on) { return dd::g_timing.exchange(on ? 1 : 0); }

int dd_timing_read(double *kernel_ms, int64_t *launches, int64_t *near_evals, int64_t *quad_evals,
                   int reset)
{
    dd::clear_error();
    double total = 0.0;
    size_t pairs = dd::g_ev_used / 2;
    for (size_t k = 0; k < pairs; ++k) {
        hipEvent_t a = dd::g_ev[2 * k], b = dd::g_ev[2 * k + 1];
        if (hipEventSynchronize(b) != hipSuccess) return dd::set_error(DD_EHIP, "hipEventSynchronize failed");
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return dd::set_error(DD_EHIP, "hipEventElapsedTime failed");
        total += ms;
    }
    if (kernel_ms) *kernel_ms = total;
    if (launches) *launches = (int64_t)pairs;
    dd::Workspace *ws = nullptr;
    int rc = dd::workspace(&ws);
    if (rc) return rc;
    unsigned long long cnt[2] = {0, 0};
    if (hipDeviceSynchronize() != hipSuccess) return dd::set_error(DD_EHIP, "hipDeviceSynchronize failed");
    if (hipMemcpy(cnt, ws->near_count, sizeof cnt, hipMemcpyDeviceToHost) != hipSuccess)
        return dd::set_error(DD_EHIP, "reading the band counters failed");
    if (near_evals) *near_evals = (int64_t)cnt[0];
    if (quad_evals) *quad_evals = (int64_t)cnt[1];
    if (reset) {
        dd::g_ev_used = 0;
        if (hipMemset(ws->near_count, 0, sizeof cnt) != hipSuccess)
            return dd::set_error(DD_EHIP, "clearing the near-pair counter failed");
        if (hipDeviceSynchronize() != hipSuccess) return dd::set_error(DD_EHIP, "hipDeviceSynchronize failed");
    }
    return DD_OK;
}

int dd_shutdown(void)
{
    std::lock_guard<std::mutex> lk(dd::g_ws_mu);
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess) cur = 0;
    for (auto *&w : dd::g_ws) {
        if (!w) continue;
        (void)hipSetDevice(w->device);
        (void)hipDeviceSynchronize();
        dd::drop_graphs(w);
        for (int s = 0; s < dd::WS_NSLOTS; ++s)
            if (w->ptr[s]) (void)hipFree(w->ptr[s]);
        if (w->flags_dev) (void)hipFree(w->flags_dev);
        if (w->flags_host) (void)hipHostFree(w->flags_host);
        if (w->capture_stream) (void)hipStreamDestroy(w->capture_stream);
        if (w->near_ev) (void)hipEventDestroy(w->near_ev);
        delete w;
        w = nullptr;
    }
    (void)hipSetDevice(cur);
    return DD_OK;
}

}  // extern "C"
