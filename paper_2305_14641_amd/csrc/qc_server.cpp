// Serving form (include/qc_server.h): admission by device-memory footprint
// into a fixed arena (oldest first, with a bounded bypass of a request that
// does not fit), `max_slots` worker threads each driving its own HIP stream,
// so requests that arrive while others run are admitted as soon as a slot and
// memory are free and their GPU work overlaps. Queued requests can time out
// or be cancelled; a failed request releases its region and slot.
#include <hip/hip_runtime.h>
#include <string.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "qc_handle.h"
#include "qc_server.h"

using namespace qc;

namespace {

double mono_now()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// First-fit allocator over [0, size) with coalescing frees.
class Arena {
  public:
    void reset(size_t size)
    {
        free_.clear();
        free_[0] = size;
    }
    bool alloc(size_t bytes, size_t *off)
    {
        bytes = align256(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t start = it->first + bytes;
                free_.erase(it);
                if (rest) free_[start] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = align256(bytes);
        auto it = free_.emplace(off, bytes).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }

  private:
    std::map<size_t, size_t> free_;
};

struct Request {
    int64_t id = 0;
    int32_t n = 0;
    std::vector<int32_t> row_ptr, col;
    std::vector<double> sigmas;
    int64_t footprint = 0;
    size_t offset = 0;
    qc_status status = QC_OK;
    bool admitted = false, done = false;
    int32_t bypassed = 0;             // times younger requests were admitted before it
    int32_t dmax = -1, slot = -1;
    double t_submit = 0, t_admit = 0, t_done = 0;
    std::vector<int32_t> labels;
    std::vector<float> psi, v;
};

}  // namespace

struct qc_server_s {
    qc_server_opts opts{};
    char *d_arena = nullptr;
    Arena arena;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request *> queue;
    std::map<int64_t, Request *> all;
    std::vector<std::thread> workers;
    std::vector<hipStream_t> streams;
    int64_t next_id = 1;
    bool stop = false;
    int64_t bytes_in_flight = 0, peak_bytes = 0;
    int32_t in_flight = 0, peak_requests = 0;
    int device = 0;
};

namespace {

qc_status run_request(qc_server s, Request *r, int slot, void **stage, size_t *stage_bytes)
{
    hipStream_t st = s->streams[slot];
    void *stream = (void *)st;
    const int S = (int)r->sigmas.size();
    const int n = r->n;
    qc_graph g = nullptr;
    QC_TRY(create_graph(n, (int64_t)r->col.size(), r->row_ptr.data(), r->col.data(), 0, st,
                        s->d_arena + r->offset, (size_t)r->footprint, &g));
    // On every exit the slot's stream is drained before the handle (and then
    // its arena region) is released, so no kernel can still write into it.
    struct Guard {
        qc_graph g;
        hipStream_t st;
        ~Guard()
        {
            (void)hipStreamSynchronize(st);
            destroy(g, false);
        }
    } guard{g, st};
    int32_t *d_labels = nullptr;
    QC_TRY(galloc(g, &d_labels, (size_t)S * n));
    QC_TRY(qc_distances(g, nullptr, &r->dmax, stream));
    QC_TRY(qc_potential(g, r->sigmas.data(), S, nullptr, nullptr, QC_PREC_FP64ACC, stream));
    for (int k = 0; k < S; ++k)
        QC_TRY(qc_ggd_labels(g, k, s->opts.tie_mode, d_labels + (size_t)k * n, stream));
    const size_t lab_bytes = (size_t)S * n * sizeof(int32_t);
    const size_t pot_bytes = s->opts.want_potentials ? (size_t)S * n * sizeof(float) : 0;
    // the resident V keeps its sigmas interleaved in groups (v_index)
    const size_t v_bytes = s->opts.want_potentials ? (size_t)v_floats(n, S) * sizeof(float) : 0;
    const size_t need = lab_bytes + pot_bytes + v_bytes;
    if (*stage_bytes < need) {
        if (*stage) (void)hipHostFree(*stage);
        *stage = nullptr;
        *stage_bytes = 0;
        QC_HIP(hipHostMalloc(stage, need, hipHostMallocDefault));
        *stage_bytes = need;
    }
    char *h = (char *)*stage;
    QC_HIP(hipMemcpyAsync(h, d_labels, lab_bytes, hipMemcpyDeviceToHost, st));
    if (pot_bytes) {
        QC_HIP(hipMemcpyAsync(h + lab_bytes, g->d_psi, pot_bytes, hipMemcpyDeviceToHost, st));
        QC_HIP(hipMemcpyAsync(h + lab_bytes + pot_bytes, g->d_v, v_bytes, hipMemcpyDeviceToHost, st));
    }
    QC_HIP(hipStreamSynchronize(st));
    r->labels.assign((int32_t *)h, (int32_t *)(h + lab_bytes));
    if (pot_bytes) {
        r->psi.assign((float *)(h + lab_bytes), (float *)(h + lab_bytes + pot_bytes));
        const float *hv = (const float *)(h + lab_bytes + pot_bytes);
        r->v.resize((size_t)S * n);
        for (int k = 0; k < S; ++k)
            for (int32_t i = 0; i < n; ++i) r->v[(size_t)k * n + i] = hv[v_index(n, k, i)];
    }
    return QC_OK;
}

// Complete the queued requests whose admission deadline has passed (the
// caller holds s->mu).
void expire_locked(qc_server s, double now)
{
    if (s->opts.queue_timeout_s <= 0) return;
    bool any = false;
    for (auto it = s->queue.begin(); it != s->queue.end();) {
        Request *r = *it;
        if (now - r->t_submit >= s->opts.queue_timeout_s) {
            r->status = QC_E_TIMEOUT;
            r->t_done = now;
            r->done = true;
            it = s->queue.erase(it);
            any = true;
        } else {
            ++it;
        }
    }
    if (any) s->cv_done.notify_all();
}

// The next request to admit, its arena region carved (the caller holds
// s->mu): the oldest queued request that fits, where a request that does not
// fit may be passed by younger ones at most max_bypass times.
Request *admit_locked(qc_server s)
{
    for (auto it = s->queue.begin(); it != s->queue.end(); ++it) {
        Request *r = *it;
        size_t off = 0;
        if (s->arena.alloc((size_t)r->footprint, &off)) {
            r->offset = off;
            r->admitted = true;
            for (auto jt = s->queue.begin(); jt != it; ++jt) (*jt)->bypassed += 1;
            s->queue.erase(it);
            return r;
        }
        if (r->bypassed >= s->opts.max_bypass) break;   // nothing may pass it now
    }
    return nullptr;
}

void worker(qc_server s, int slot)
{
    (void)hipSetDevice(s->device);
    void *stage = nullptr;
    size_t stage_bytes = 0;
    for (;;) {
        Request *r = nullptr;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            for (;;) {
                expire_locked(s, mono_now());
                if (!s->queue.empty()) {
                    if ((r = admit_locked(s))) break;
                } else if (s->stop) {
                    break;
                }
                if (s->opts.queue_timeout_s > 0 && !s->queue.empty()) {
                    // wake at the oldest queued request's deadline at the latest
                    const double left =
                        s->queue.front()->t_submit + s->opts.queue_timeout_s - mono_now();
                    s->cv_work.wait_for(lk, std::chrono::duration<double>(left > 0 ? left : 0.0));
                } else {
                    s->cv_work.wait(lk);
                }
            }
            if (!r) break;
            r->t_admit = mono_now();
            r->slot = slot;
            s->bytes_in_flight += align256((size_t)r->footprint);
            s->in_flight += 1;
            if (s->bytes_in_flight > s->peak_bytes) s->peak_bytes = s->bytes_in_flight;
            if (s->in_flight > s->peak_requests) s->peak_requests = s->in_flight;
        }
        const qc_status st = run_request(s, r, slot, &stage, &stage_bytes);
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->arena.release(r->offset, (size_t)r->footprint);
            s->bytes_in_flight -= align256((size_t)r->footprint);
            s->in_flight -= 1;
            r->status = st;
            r->t_done = mono_now();
            r->done = true;
        }
        s->cv_done.notify_all();
        s->cv_work.notify_all();
    }
    if (stage) (void)hipHostFree(stage);
}

}  // namespace

extern "C" {

int64_t qc_request_footprint(int32_t n, int64_t nnz, int32_t n_sigmas)
{
    return handle_footprint(n, nnz, n_sigmas, true, true);
}

qc_status qc_server_create(const qc_server_opts *opts, qc_server *out)
{
    if (!opts || !out) return QC_E_INVAL;
    if (opts->max_slots < 1 || opts->max_slots > 64 || opts->hbm_budget_bytes <= 0 ||
        opts->tie_mode > QC_TIE_MERGE || !(opts->queue_timeout_s >= 0) ||
        opts->queue_timeout_s > 1e9 || opts->max_bypass < 0 || opts->max_bypass > 1000000)
        return QC_E_INVAL;
    int dev = 0;
    QC_TRY(check_device(&dev));
    qc_server s = new qc_server_s();
    s->opts = *opts;
    s->device = dev;
    {
        const qc_status a = device_malloc((void **)&s->d_arena, (size_t)opts->hbm_budget_bytes);
        if (a != QC_OK) {
            delete s;
            return a;
        }
    }
    s->arena.reset((size_t)opts->hbm_budget_bytes);
    for (int k = 0; k < opts->max_slots; ++k) {
        hipStream_t st = nullptr;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            for (auto x : s->streams) (void)hipStreamDestroy(x);
            device_free(s->d_arena);
            delete s;
            return QC_E_DEVICE;
        }
        s->streams.push_back(st);
    }
    for (int k = 0; k < opts->max_slots; ++k) s->workers.emplace_back(worker, s, k);
    *out = s;
    return QC_OK;
}

qc_status qc_server_submit(qc_server s, int32_t n, int64_t nnz, const int32_t *row_ptr,
                           const int32_t *col_idx, const double *sigmas, int32_t n_sigmas,
                           int64_t *id_out)
{
    if (!s || !id_out) return QC_E_INVAL;
    QC_TRY(validate_sigmas(sigmas, n_sigmas));
    Request *r = new Request();
    qc_status st = validate_csr(n, nnz, row_ptr, col_idx, false, r->row_ptr, r->col);
    if (st != QC_OK) {
        delete r;
        return st;
    }
    r->n = n;
    r->sigmas.assign(sigmas, sigmas + n_sigmas);
    r->footprint = qc_request_footprint(n, nnz, n_sigmas);
    if (r->footprint > s->opts.hbm_budget_bytes) {
        delete r;
        return QC_E_BUSY;
    }
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) {
            delete r;
            return QC_E_STATE;
        }
        r->id = s->next_id++;
        r->t_submit = mono_now();
        s->all[r->id] = r;
        s->queue.push_back(r);
        *id_out = r->id;
    }
    s->cv_work.notify_all();
    return QC_OK;
}

qc_status qc_server_poll(qc_server s, int64_t id, int32_t *done_out)
{
    if (!s || !done_out) return QC_E_INVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    expire_locked(s, mono_now());
    auto it = s->all.find(id);
    if (it == s->all.end()) return QC_E_INVAL;
    *done_out = it->second->done ? 1 : 0;
    return QC_OK;
}

qc_status qc_server_wait(qc_server s, int64_t id, int32_t *labels_out, float *psi_out,
                         float *v_out, qc_request_info *info)
{
    if (!s) return QC_E_INVAL;
    Request *r = nullptr;
    {
        std::unique_lock<std::mutex> lk(s->mu);
        auto it = s->all.find(id);
        if (it == s->all.end()) return QC_E_INVAL;
        r = it->second;
        while (!r->done) {
            if (s->opts.queue_timeout_s > 0 && !r->admitted) {
                // every worker may be busy: expire the request here at its deadline
                const double left = r->t_submit + s->opts.queue_timeout_s - mono_now();
                s->cv_done.wait_for(lk, std::chrono::duration<double>(left > 0 ? left : 0.0));
                expire_locked(s, mono_now());
            } else {
                s->cv_done.wait(lk);
            }
        }
        s->all.erase(it);
    }
    const size_t cells = r->sigmas.size() * (size_t)r->n;
    if (labels_out && r->labels.size() == cells) memcpy(labels_out, r->labels.data(), cells * 4);
    if (psi_out && r->psi.size() == cells) memcpy(psi_out, r->psi.data(), cells * 4);
    if (v_out && r->v.size() == cells) memcpy(v_out, r->v.data(), cells * 4);
    if (info) {
        info->id = r->id;
        info->t_submit = r->t_submit;
        info->t_admit = r->t_admit;
        info->t_done = r->t_done;
        info->footprint_bytes = r->footprint;
        info->n = r->n;
        info->n_sigmas = (int32_t)r->sigmas.size();
        info->dmax = r->dmax;
        info->slot = r->slot;
        info->status = r->status;
    }
    const qc_status st = r->status;
    delete r;
    return st;
}

qc_status qc_server_cancel(qc_server s, int64_t id)
{
    if (!s) return QC_E_INVAL;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->all.find(id);
        if (it == s->all.end()) return QC_E_INVAL;
        Request *r = it->second;
        if (r->done) return QC_E_STATE;
        if (r->admitted) return QC_E_BUSY;
        for (auto q = s->queue.begin(); q != s->queue.end(); ++q) {
            if (*q == r) {
                s->queue.erase(q);
                break;
            }
        }
        r->status = QC_E_CANCELLED;
        r->t_done = mono_now();
        r->done = true;
    }
    s->cv_done.notify_all();
    s->cv_work.notify_all();   // a request it blocked may fit now
    return QC_OK;
}

qc_status qc_server_stats(qc_server s, int64_t *peak_bytes_out, int32_t *peak_requests_out)
{
    if (!s) return QC_E_INVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    if (peak_bytes_out) *peak_bytes_out = s->peak_bytes;
    if (peak_requests_out) *peak_requests_out = s->peak_requests;
    return QC_OK;
}

qc_status qc_server_destroy(qc_server s)
{
    if (!s) return QC_E_INVAL;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    for (auto &t : s->workers) t.join();
    for (auto st : s->streams) (void)hipStreamDestroy(st);
    device_free(s->d_arena);
    for (auto &kv : s->all) delete kv.second;
    delete s;
    return QC_OK;
}

}  // extern "C"
