// Process-wide kernel timing with HIP events (qc_timing_enable / _read).
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "qc.h"
#include "qc_internal.h"

namespace {

struct Record {
    int stage;
    hipEvent_t start, stop;
};

std::mutex g_mu;
bool g_on = false;
thread_local bool t_off = false;   // this thread's timers are switched off
std::vector<Record> g_records;
std::vector<hipEvent_t> g_pool;

hipEvent_t take_event()
{
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

void clear_records()
{
    for (auto &r : g_records) {
        (void)hipEventSynchronize(r.stop);
        g_pool.push_back(r.start);
        g_pool.push_back(r.stop);
    }
    g_records.clear();
}

bool capturing(hipStream_t s)
{
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess) return true;
    return cs != hipStreamCaptureStatusNone;
}

}  // namespace

namespace qc {

StageTimer::StageTimer(int stage, hipStream_t stream) : stage_(stage), stream_(stream)
{
    if (t_off) return;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_on || capturing(stream)) return;
    hipEvent_t a = take_event(), b = take_event();
    if (!a || !b) return;
    if (hipEventRecord(a, stream) != hipSuccess) return;
    start_ = a;
    stop_ = b;
}

StageTimer::~StageTimer()
{
    if (!start_) return;
    std::lock_guard<std::mutex> lk(g_mu);
    if (hipEventRecord((hipEvent_t)stop_, stream_) == hipSuccess)
        g_records.push_back(Record{stage_, (hipEvent_t)start_, (hipEvent_t)stop_});
}

StageTimingOff::StageTimingOff() : prev_(t_off) { t_off = true; }
StageTimingOff::~StageTimingOff() { t_off = prev_; }

}  // namespace qc

extern "C" {

qc_status qc_timing_enable(int32_t on)
{
    std::lock_guard<std::mutex> lk(g_mu);
    clear_records();
    g_on = on != 0;
    return QC_OK;
}

qc_status qc_timing_read(int32_t stage, double *total_ms, int64_t *launches)
{
    if (stage < 0 || stage >= QC_N_STAGES) return QC_E_INVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    double total = 0.0;
    int64_t count = 0;
    for (auto &r : g_records) {
        if (r.stage != stage) continue;
        if (hipEventSynchronize(r.stop) != hipSuccess) return QC_E_DEVICE;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.start, r.stop) != hipSuccess) return QC_E_DEVICE;
        total += ms;
        ++count;
    }
    if (total_ms) *total_ms = total;
    if (launches) *launches = count;
    return QC_OK;
}

}  // extern "C"
