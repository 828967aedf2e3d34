// Served form: a request loop over the clustering library.
//
// Requests (device rows, eps, minPts, device label array) wait in one FIFO
// queue.  Worker threads, each with its own context and HIP stream, take the
// next requests as a batch whenever they are free: consecutive requests of
// d <= 4 go together through one batched launch sequence per dimension, a
// request of larger d runs alone through the plain path.  A worker admits a
// batch only while the estimated device footprint of all running batches
// stays within the budget (an idle server always admits one request), so
// requests that arrive while others run are admitted as workers and memory
// free up, and the work of different workers overlaps on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include "hca.h"

namespace {

double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct Request {
    const int32_t *pts;
    int64_t n;
    int32_t d;
    double eps;
    int32_t min_pts;
    int32_t *labels;
    uint64_t tag;
    size_t bytes;
    double est_ms;              // estimated device time alone
    hipEvent_t ready;           // recorded on the caller's stream at submission, or null
};

struct Done {
    uint64_t tag;
    int32_t status;
    double t_done;
};

constexpr int32_t kBatchDimMax = 4;

// Device bytes one request needs while it runs (workspace estimate).
size_t footprint(int64_t n, int32_t d)
{
    uint64_t dirs = 1;
    for (int k = 0; k < std::min(d, 4); k++) dirs *= 3;
    // + 72 B for the neighbours recorded by core marking, and for lists (d >= 3)
    // up to 256 B of prefix-range table
    uint64_t per_point = 256 + 72 + 8ull * (dirs - 1) + 16ull * (uint64_t)d + (d >= 3 ? 264 + 256 : 0);
    if (d > 8) per_point += 12ull * (((uint64_t)d + 3) & ~3ull);      // padded rows and group boxes
    return (size_t)((uint64_t)n * per_point + (1ull << 20));
}

// Estimated device time of a request alone (ms), from its rows and axes:
// the per-point costs measured for the launch sequence on one MI355X (about
// 0.4 ns per point for up to two axes, 2.7 for three, 5.6 for four, more
// with search groups), used only to bound how much work one batch gathers.
double estimate_ms(int64_t n, int32_t d)
{
    const double ns_per_pt = d <= 2 ? 0.4 : d == 3 ? 2.7 : d == 4 ? 5.6 : d <= 8 ? 12.0 : 200.0;
    return 0.02 + (double)n * ns_per_pt * 1e-6;
}

}  // namespace

struct hca_server {
    int device = 0;
    size_t budget = 0;
    int32_t max_batch = 64;
    double batch_ms = 4.0;      // a batch stops growing past this much estimated device time
    std::vector<hca_ctx *> ctx;
    std::vector<hipStream_t> streams;
    std::vector<std::thread> workers;
    std::mutex mu;
    std::condition_variable cv_work, cv_idle;
    std::deque<Request> queue;
    std::vector<Done> done;
    std::vector<hipEvent_t> spare_events;   // recorded-and-waited events for reuse
    size_t in_flight = 0;
    int active = 0;
    bool stop = false;

    void run_worker(int w);
};

void hca_server::run_worker(int w)
{
    (void)hipSetDevice(device);
    hca_ctx *c = ctx[w];
    std::vector<Request> batch;
    std::vector<int64_t> rows;
    std::vector<int32_t> dims, mps;
    std::vector<double> eps;
    while (true) {
        batch.clear();
        {
            std::unique_lock<std::mutex> lk(mu);
            cv_work.wait(lk, [&] {
                if (stop && queue.empty()) return true;
                if (queue.empty()) return false;
                return in_flight == 0 || in_flight + queue.front().bytes <= budget;
            });
            if (queue.empty()) return;                       // stopping, nothing left
            // the front request, then (if it can be batched) the requests of
            // d <= 4 behind it while they fit
            size_t bytes = 0;
            double est = 0;
            const bool batchable = queue.front().d <= kBatchDimMax;
            while (!queue.empty() && (int32_t)batch.size() < max_batch) {
                const Request &r = queue.front();
                if (!batch.empty() && (!batchable || r.d > kBatchDimMax)) break;
                if (!batch.empty() && in_flight + bytes + r.bytes > budget) break;
                // small requests are not held behind large ones: a batch
                // takes requests only while its estimated time stays short
                if (!batch.empty() && est + r.est_ms > batch_ms) break;
                est += r.est_ms;
                bytes += r.bytes;
                batch.push_back(r);
                queue.pop_front();
            }
            in_flight += bytes;
            active++;
        }
        // run the batch on this worker's stream, after the work its requests'
        // callers queued before submitting them
        for (const Request &r : batch)
            if (r.ready) (void)hipStreamWaitEvent(streams[w], r.ready, 0);
        std::vector<int32_t> status(batch.size(), HCA_OK);
        if (batch.size() == 1 && batch[0].d > kBatchDimMax) {
            const Request &r = batch[0];
            status[0] = hca_cluster(c, r.pts, r.n, r.d, r.eps, r.min_pts, r.labels);
        } else {
            // one batched call over the requests' own arrays
            const int32_t nb = (int32_t)batch.size();
            std::vector<const int32_t *> src(nb);
            std::vector<int32_t *> dst(nb);
            rows.assign(nb, 0);
            dims.assign(nb, 0);
            eps.assign(nb, 0.0);
            mps.assign(nb, 0);
            for (int32_t i = 0; i < nb; i++) {
                src[i] = batch[i].pts;
                dst[i] = batch[i].labels;
                rows[i] = batch[i].n;
                dims[i] = batch[i].d;
                eps[i] = batch[i].eps;
                mps[i] = batch[i].min_pts;
            }
            hca_status st = hca_cluster_sets(c, src.data(), dst.data(), nb, rows.data(), dims.data(), eps.data(),
                                             mps.data());
            if (st != HCA_OK) {
                // find out which request failed: each one alone
                for (int32_t i = 0; i < nb; i++)
                    status[i] = hca_cluster_sets(c, &src[i], &dst[i], 1, &rows[i], &dims[i], &eps[i], &mps[i]);
            }
        }
        const double t = now_s();
        {
            std::lock_guard<std::mutex> lk(mu);
            size_t bytes = 0;
            for (size_t i = 0; i < batch.size(); i++) {
                bytes += batch[i].bytes;
                done.push_back({batch[i].tag, status[i], t});
                // the clustering call synchronised the stream that waited on it
                if (batch[i].ready) spare_events.push_back(batch[i].ready);
            }
            in_flight -= bytes;
            active--;
        }
        cv_work.notify_all();
        cv_idle.notify_all();
    }
}

extern "C" {

double hca_clock(void) { return now_s(); }

hca_status hca_server_create(hca_server **out, int32_t device, int32_t workers, int64_t budget_bytes,
                             int32_t max_batch)
{
    if (!out || workers < 1 || workers > 16 || budget_bytes <= 0 || max_batch < 1) return HCA_E_INVAL;
    *out = nullptr;
    hca_server *srv = new (std::nothrow) hca_server();
    if (!srv) return HCA_E_NOMEM;
    srv->device = device;
    srv->budget = (size_t)budget_bytes;
    srv->max_batch = max_batch;
    if (hipSetDevice(device) != hipSuccess) {
        delete srv;
        return HCA_E_DEVICE;
    }
    for (int32_t w = 0; w < workers; w++) {
        hca_ctx *c = nullptr;
        hipStream_t s = nullptr;
        hca_status st = hca_create(&c, device);
        if (st == HCA_OK && hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) st = HCA_E_DEVICE;
        if (st != HCA_OK) {
            if (c) hca_destroy(c);
            for (size_t i = 0; i < srv->ctx.size(); i++) {
                hca_destroy(srv->ctx[i]);
                (void)hipStreamDestroy(srv->streams[i]);
            }
            delete srv;
            return st;
        }
        hca_set_stream(c, s);
        srv->ctx.push_back(c);
        srv->streams.push_back(s);
    }
    for (int32_t w = 0; w < workers; w++) srv->workers.emplace_back(&hca_server::run_worker, srv, w);
    *out = srv;
    return HCA_OK;
}

hca_status hca_server_submit(hca_server *srv, const int32_t *points, int64_t n, int32_t d, double eps,
                             int32_t min_pts, int32_t *labels, uint64_t tag, void *after_stream)
{
    if (!srv || n < 0 || d < 1 || d > 64 || min_pts < 1 || !(eps > 0.0)) return HCA_E_INVAL;
    if (n > 0 && (!points || !labels)) return HCA_E_INVAL;
    hipEvent_t ev = nullptr;
    {
        {
            std::lock_guard<std::mutex> lk(srv->mu);
            if (!srv->spare_events.empty()) {
                ev = srv->spare_events.back();
                srv->spare_events.pop_back();
            }
        }
        if (!ev && hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) return HCA_E_DEVICE;
        if (hipEventRecord(ev, (hipStream_t)after_stream) != hipSuccess) {
            (void)hipEventDestroy(ev);
            return HCA_E_DEVICE;
        }
    }
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        if (srv->stop) {
            if (ev) srv->spare_events.push_back(ev);
            return HCA_E_INVAL;
        }
        srv->queue.push_back({points, n, d, eps, min_pts, labels, tag, footprint(n, d), estimate_ms(n, d), ev});
    }
    srv->cv_work.notify_one();
    return HCA_OK;
}

hca_status hca_server_set_batch_time(hca_server *srv, double ms)
{
    if (!srv || !(ms > 0.0) || !std::isfinite(ms)) return HCA_E_INVAL;
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->batch_ms = ms;
    return HCA_OK;
}

int32_t hca_server_poll(hca_server *srv, uint64_t *tags, int32_t *status, double *t_done, int32_t max)
{
    if (!srv || max <= 0 || !tags || !status || !t_done) return 0;
    std::lock_guard<std::mutex> lk(srv->mu);
    const int32_t k = (int32_t)std::min<size_t>(srv->done.size(), (size_t)max);
    for (int32_t i = 0; i < k; i++) {
        tags[i] = srv->done[i].tag;
        status[i] = srv->done[i].status;
        t_done[i] = srv->done[i].t_done;
    }
    srv->done.erase(srv->done.begin(), srv->done.begin() + k);
    return k;
}

hca_status hca_server_drain(hca_server *srv)
{
    if (!srv) return HCA_E_INVAL;
    std::unique_lock<std::mutex> lk(srv->mu);
    srv->cv_idle.wait(lk, [&] { return srv->queue.empty() && srv->active == 0; });
    return HCA_OK;
}

void hca_server_destroy(hca_server *srv)
{
    if (!srv) return;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
    }
    srv->cv_work.notify_all();
    for (auto &t : srv->workers) t.join();
    (void)hipSetDevice(srv->device);
    for (size_t i = 0; i < srv->ctx.size(); i++) {
        hca_destroy(srv->ctx[i]);
        (void)hipStreamDestroy(srv->streams[i]);
    }
    for (hipEvent_t e : srv->spare_events) (void)hipEventDestroy(e);
    delete srv;
}

}  // extern "C"
