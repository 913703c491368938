// Serving loop: PDQ queries (Sec. 3; the server's Answer step, Alg. 7) answered as
// they arrive, by continuous batching over resident keys, database and diagonals.
//
// One host thread owns the device side. Requests wait in a FIFO queue. Whenever a
// lane (a stream with its own pre-reserved workspace and staging area) is free, the
// thread admits the oldest waiting requests into a batch while the batch's exact
// workspace footprint (batch_shape) fits the lane and the batch holds at most
// max_batch queries, and enqueues the batch's phases (compress_many) on the lane's
// stream. With several lanes a new batch starts while earlier ones are still on the
// device, so requests that arrive meanwhile overlap with them instead of queueing
// behind the whole batch. A batch's completion is seen through an event; its
// requests then move to the done queue with host timestamps (CLOCK_MONOTONIC).
#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <thread>

#include "compress.h"

namespace hc {

static int64_t now_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct ServerReq {
    uint64_t id = 0;
    QueryRun run;
    hc_server_result res{};
    hipEvent_t ready = nullptr;  // recorded on the submitter's stream after ct_v was produced
    ~ServerReq() {
        if (ready) (void)hipEventDestroy(ready);
    }
};

struct ServerLane {
    Lane lane;
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
    hc_status status = HC_OK;
    std::vector<ServerReq*> reqs;
};

}  // namespace hc

struct hc_server {
    hc_context* c = nullptr;
    const hc_gk* gk = nullptr;
    const hc_db* db = nullptr;
    uint32_t comp_level = 0, out_level = 0;
    size_t lane_bytes = 0;
    uint32_t max_batch = 1;
    std::vector<std::unique_ptr<hc::ServerLane>> lanes;
    std::mutex mu;
    std::condition_variable wake, done_cv;
    std::deque<hc::ServerReq*> pending, done;
    bool stop = false;
    uint64_t next_id = 1;
    hc_server_stats stats{};
    std::thread th;

    void loop();
    hc_status launch(hc::ServerLane& ln, std::vector<hc::ServerReq*>& batch);
};

using namespace hc;

hc_status hc_server::launch(ServerLane& ln, std::vector<ServerReq*>& batch) {
    std::vector<QueryRun> runs;
    runs.reserve(batch.size());
    for (ServerReq* r : batch) runs.push_back(r->run);
    const int64_t t = now_ns();
    // the batch reads each ct_v only after the work its submitter queued before it
    hc_status s = HC_OK;
    for (ServerReq* r : batch)
        if (r->ready && hipStreamWaitEvent(ln.stream, r->ready, 0) != hipSuccess) s = HC_EDEVICE;
    if (s == HC_OK) s = compress_many(*c, ln.lane, gk, db, runs, ln.stream);
    for (size_t i = 0; i < batch.size(); i++) {
        batch[i]->res.start_ns = t;
        batch[i]->res.batch_size = (uint32_t)batch.size();
        if (s == HC_OK) fill_info(runs[i], &batch[i]->res.info);
    }
    if (hipEventRecord(ln.done, ln.stream) != hipSuccess && s == HC_OK) s = HC_EDEVICE;
    return s;
}

void hc_server::loop() {
    (void)hipSetDevice(c->device);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        bool progressed = false, any_busy = false;
        // completions
        for (auto& lp : lanes) {
            ServerLane& ln = *lp;
            if (!ln.busy) continue;
            const hipError_t q = hipEventQuery(ln.done);
            if (q == hipErrorNotReady) {
                any_busy = true;
                continue;
            }
            const int64_t t = now_ns();
            for (ServerReq* r : ln.reqs) {
                r->res.done_ns = t;
                r->res.status = (q == hipSuccess) ? ln.status : HC_EDEVICE;
                done.push_back(r);
                stats.completed++;
            }
            ln.reqs.clear();
            ln.busy = false;
            progressed = true;
        }
        if (progressed) done_cv.notify_all();
        // admissions: the oldest waiting requests while the batch fits one lane
        for (auto& lp : lanes) {
            ServerLane& ln = *lp;
            if (ln.busy || pending.empty()) continue;
            std::vector<ServerReq*> batch;
            std::vector<QueryRun> trial;
            while (!pending.empty() && batch.size() < max_batch) {
                trial.push_back(pending.front()->run);
                BatchShape shape;
                if (batch_shape(*c, gk, db, trial, shape) != HC_OK || shape.total > lane_bytes) {
                    trial.pop_back();
                    break;
                }
                batch.push_back(pending.front());
                pending.pop_front();
            }
            if (batch.empty()) {  // cannot happen: submit admits only queries that fit alone
                ServerReq* r = pending.front();
                pending.pop_front();
                r->res.status = HC_ENOMEM;
                r->res.done_ns = now_ns();
                done.push_back(r);
                stats.completed++;
                done_cv.notify_all();
                continue;
            }
            ln.reqs = batch;
            ln.busy = true;
            uint32_t nb = 0;
            for (auto& o : lanes) nb += o->busy ? 1 : 0;
            stats.batches++;
            if (batch.size() > stats.max_batch_seen) stats.max_batch_seen = (uint32_t)batch.size();
            if (nb > stats.max_lanes_busy) stats.max_lanes_busy = nb;
            lk.unlock();
            ln.status = launch(ln, ln.reqs);
            lk.lock();
            any_busy = true;
            progressed = true;
        }
        if (stop && pending.empty()) {
            bool idle = true;
            for (auto& lp : lanes) idle = idle && !lp->busy;
            if (idle) break;
        }
        if (!progressed) {
            // poll the device while batches run; otherwise sleep until a submission
            if (any_busy)
                wake.wait_for(lk, std::chrono::microseconds(50));
            else
                wake.wait_for(lk, std::chrono::milliseconds(20));
        }
    }
}

extern "C" hc_status hc_server_create(hc_context* cp, const hc_gk* gk, const hc_db* db, uint32_t comp_level,
                                      uint32_t out_level, uint64_t lane_bytes, uint32_t lanes, uint32_t max_batch,
                                      hc_server** out) {
    if (!cp || !gk || !out || lanes < 1 || lanes > 4 || max_batch < 1 || lane_bytes < (1u << 20))
        return HC_EINVAL;
    *out = nullptr;
    Ctx& c = *cp;
    HC_CHECK(hipSetDevice(c.device));
    std::unique_ptr<hc_server> s(new hc_server());
    s->c = cp;
    s->gk = gk;
    s->db = db;
    s->comp_level = comp_level;
    s->out_level = out_level;
    s->lane_bytes = lane_bytes;
    s->max_batch = max_batch;
    // tables that compressions build on first use, built now (their construction
    // synchronises the device)
    for (uint32_t sv = 1; sv <= (uint32_t)c.nh; sv *= 2) {
        const uint64_t* m = nullptr;
        hc_status st = prefix_mask(c, sv, &m);
        if (st != HC_OK) return st;
    }
    for (uint32_t i = 0; i < lanes; i++) {
        std::unique_ptr<ServerLane> ln(new ServerLane());
        hc_status st = ln->lane.init((size_t)8 << 20);
        if (st == HC_OK) st = ln->lane.ws.reserve(lane_bytes);
        if (st != HC_OK) {
            ln->lane.release();
            for (auto& o : s->lanes) o->lane.release();
            return HC_ENOMEM;
        }
        HC_CHECK(hipStreamCreateWithFlags(&ln->stream, hipStreamNonBlocking));
        HC_CHECK(hipEventCreateWithFlags(&ln->done, hipEventDisableTiming));
        s->lanes.push_back(std::move(ln));
    }
    HC_CHECK(hipDeviceSynchronize());
    hc_server* raw = s.release();
    raw->th = std::thread([raw]() { raw->loop(); });
    *out = raw;
    return HC_OK;
}

extern "C" hc_status hc_server_submit(hc_server* s, const uint64_t* ct_v, uint64_t N, uint32_t t_bound,
                                      uint64_t* ct_out, hipStream_t stream, uint64_t* id_out) {
    if (!s || !ct_v || !ct_out) return HC_EINVAL;
    std::unique_ptr<ServerReq> r(new ServerReq());
    hc_status st =
        make_plan(*s->c, N, s->db ? s->db->ncol : 0, t_bound, s->comp_level, s->out_level, r->run.pl);
    if (st != HC_OK) return st;
    r->run.ct_v = ct_v;
    r->run.ct_out = ct_out;
    {
        std::vector<QueryRun> one{r->run};
        BatchShape shape;
        st = batch_shape(*s->c, s->gk, s->db, one, shape);
        if (st != HC_OK) return st;
        if (shape.total > s->lane_bytes) return HC_ENOMEM;
    }
    HC_CHECK(hipSetDevice(s->c->device));
    HC_CHECK(hipEventCreateWithFlags(&r->ready, hipEventDisableTiming));
    HC_CHECK(hipEventRecord(r->ready, stream));
    std::lock_guard<std::mutex> g(s->mu);
    if (s->stop) return HC_EINVAL;
    r->id = s->next_id++;
    r->res.id = r->id;
    r->res.submit_ns = now_ns();
    if (id_out) *id_out = r->id;
    s->pending.push_back(r.release());
    s->stats.submitted++;
    s->wake.notify_all();
    return HC_OK;
}

extern "C" hc_status hc_server_poll(hc_server* s, hc_server_result* out, uint32_t cap, uint32_t* count,
                                    double timeout_ms) {
    if (!s || !count || (cap && !out)) return HC_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->done.empty() && timeout_ms > 0)
        s->done_cv.wait_for(lk, std::chrono::microseconds((int64_t)(timeout_ms * 1000.0)),
                            [s]() { return !s->done.empty(); });
    uint32_t k = 0;
    while (k < cap && !s->done.empty()) {
        ServerReq* r = s->done.front();
        s->done.pop_front();
        out[k++] = r->res;
        delete r;
    }
    *count = k;
    return HC_OK;
}

extern "C" hc_status hc_server_stats_get(hc_server* s, hc_server_stats* out) {
    if (!s || !out) return HC_EINVAL;
    std::lock_guard<std::mutex> g(s->mu);
    *out = s->stats;
    return HC_OK;
}

extern "C" void hc_server_destroy(hc_server* s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
        s->wake.notify_all();
    }
    if (s->th.joinable()) s->th.join();
    (void)hipSetDevice(s->c->device);
    for (auto& lp : s->lanes) {
        (void)hipStreamSynchronize(lp->stream);
        (void)hipEventDestroy(lp->done);
        (void)hipStreamDestroy(lp->stream);
        lp->lane.release();
    }
    for (ServerReq* r : s->done) delete r;
    for (ServerReq* r : s->pending) delete r;
    delete s;
}
