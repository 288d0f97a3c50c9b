// Serving runtime of libflowroi (host C++, part of flowroi.hip's
// translation unit): HBM-budget admission of camera streams, continuous
// batching of arriving frames into steps, and completion time-stamping.
//
// Threads: the caller's (open/submit/poll/drain), one scheduler that forms
// and issues steps, one completion thread that waits for steps in issue
// order. All shared state is under Server::mu; only the scheduler touches
// stream contexts and HIP streams after a stream is open.
#pragma once

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <thread>

namespace {

double now_seconds()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct SrvFrame {
    const void *host;
    int64_t pitch;
    float *flow;
    uint8_t *mask;
    uint64_t tag;
    double t_arrival;
};

struct SrvStream {
    bool open = false;
    bool closing = false;
    roi_stream_ctx *ctx = nullptr;
    uint8_t *slot[2] = {nullptr, nullptr}; // device copies of the last two frames
    int next_slot = 0;
    int cstream = 0;                       // compute stream this stream always runs on
    int inflight = 0;                      // frames in issued, unfinished steps
    std::deque<SrvFrame> queue;
};

struct SrvStep {
    std::vector<int> ids;
    std::vector<SrvFrame> frames;
    std::vector<int32_t> status;
    std::vector<hipEvent_t> done; // one per compute stream used
    std::vector<hipEvent_t> aux;  // fork/join events of the step's shared grids
};

constexpr int SRV_COMPUTE_STREAMS = 4;

struct Server {
    roi_server_config cfg{};
    size_t stream_bytes = 0, frame_bytes = 0, used = 0;
    int device = 0;
    std::vector<SrvStream> streams;
    hipStream_t copy_s = nullptr;
    hipStream_t comp_s[SRV_COMPUTE_STREAMS] = {};
    std::vector<hipEvent_t> ev_pool;
    std::mutex ev_mu; // guards ev_pool (issue() runs without mu)
    std::mutex mu;
    std::condition_variable cv_sched, cv_done, cv_drain;
    std::deque<SrvStep *> inflight;
    std::deque<roi_server_result> results;
    int64_t submitted = 0, completed = 0;
    roi_status error = ROI_OK;
    bool stop = false;
    std::thread sched, comp;
    int rr = 0;

    hipEvent_t get_event()
    {
        std::lock_guard<std::mutex> g(ev_mu);
        if (!ev_pool.empty()) {
            hipEvent_t e = ev_pool.back();
            ev_pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        hipEventCreateWithFlags(&e, hipEventDisableTiming);
        return e;
    }

    bool ready_locked() const
    {
        for (const SrvStream &s : streams)
            if (s.open && !s.queue.empty() && s.inflight < 2) return true;
        return false;
    }

    void scheduler()
    {
        hipSetDevice(device);
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            cv_sched.wait(lk, [&] {
                return stop || (ready_locked() && (int)inflight.size() < cfg.max_inflight);
            });
            if (stop && !ready_locked()) break;
            if ((int)inflight.size() >= cfg.max_inflight) continue;
            // at most one frame per stream, oldest arrival first
            std::vector<std::pair<double, int>> cand;
            for (int i = 0; i < (int)streams.size(); ++i) {
                const SrvStream &s = streams[i];
                if (s.open && !s.queue.empty() && s.inflight < 2) cand.emplace_back(s.queue.front().t_arrival, i);
            }
            std::sort(cand.begin(), cand.end());
            if ((int)cand.size() > cfg.max_batch) cand.resize(cfg.max_batch);
            SrvStep *st = new SrvStep();
            for (auto &c : cand) {
                SrvStream &s = streams[c.second];
                st->ids.push_back(c.second);
                st->frames.push_back(s.queue.front());
                s.queue.pop_front();
                s.inflight += 1;
            }
            lk.unlock();
            issue(*st);
            lk.lock();
            inflight.push_back(st);
            cv_done.notify_one();
        }
    }

    // Copies the step's frames to their device slots and runs the step's
    // pushes: each stream's own work on its compute stream, the coarse-level
    // updates of all of them in shared grids on compute stream 0; records one
    // completion event per compute stream used.
    void issue(SrvStep &st)
    {
        const size_t es = dtype_bytes(cfg.dtype);
        const int n = (int)st.ids.size();
        std::vector<const void *> dev(n);
        st.status.assign(n, ROI_OK);
        for (int i = 0; i < n; ++i) {
            SrvStream &s = streams[st.ids[i]];
            uint8_t *slot = s.slot[s.next_slot];
            s.next_slot ^= 1;
            dev[i] = slot;
            const SrvFrame &f = st.frames[i];
            if (hipMemcpy2DAsync(slot, (size_t)cfg.w * es, f.host, (size_t)f.pitch * es, (size_t)cfg.w * es, cfg.h,
                                 hipMemcpyHostToDevice, copy_s) != hipSuccess)
                st.status[i] = ROI_EDEVICE;
        }
        hipEvent_t copied = get_event();
        hipEventRecord(copied, copy_s);
        bool used_cs[SRV_COMPUTE_STREAMS] = {};
        for (int i = 0; i < n; ++i) used_cs[streams[st.ids[i]].cstream] = true;
        for (int k = 0; k < SRV_COMPUTE_STREAMS; ++k)
            if (used_cs[k]) hipStreamWaitEvent(comp_s[k], copied, 0);
        {
            std::vector<int> idx;
            std::vector<roi_stream_ctx *> cs;
            std::vector<const void *> fr;
            std::vector<int64_t> pitch;
            std::vector<float *> fl;
            std::vector<uint8_t *> mk;
            std::vector<hipStream_t> ss;
            for (int i = 0; i < n; ++i) {
                if (st.status[i] != ROI_OK) continue;
                SrvStream &s = streams[st.ids[i]];
                idx.push_back(i);
                cs.push_back(s.ctx);
                fr.push_back(dev[i]);
                pitch.push_back(cfg.w);
                fl.push_back(st.frames[i].flow);
                mk.push_back(st.frames[i].mask);
                ss.push_back(comp_s[s.cstream]);
            }
            if (!idx.empty()) {
                hipEvent_t evs[2 * SRV_FORK_MAX];
                for (hipEvent_t &e : evs) {
                    e = get_event();
                    st.aux.push_back(e);
                }
                std::vector<int32_t> sub(idx.size(), ROI_OK);
                const roi_status r = stream_push_batch((int)idx.size(), cs.data(), fr.data(), pitch.data(), fl.data(),
                                                       mk.data(), sub.data(), ss.data(), comp_s[0], evs);
                for (size_t k = 0; k < idx.size(); ++k) st.status[idx[k]] = r != ROI_OK ? r : sub[k];
                used_cs[0] = true; // the shared grids ran there
            }
        }
        for (int k = 0; k < SRV_COMPUTE_STREAMS; ++k) {
            if (!used_cs[k]) continue;
            hipEvent_t e = get_event();
            hipEventRecord(e, comp_s[k]);
            st.done.push_back(e);
        }
        st.done.push_back(copied);
    }

    void completer()
    {
        hipSetDevice(device);
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            cv_done.wait(lk, [&] { return !inflight.empty() || (stop && inflight.empty()); });
            if (inflight.empty()) break;
            SrvStep *st = inflight.front();
            lk.unlock();
            roi_status err = ROI_OK;
            for (hipEvent_t e : st->done)
                if (hipEventSynchronize(e) != hipSuccess) err = ROI_EDEVICE;
            const double t = now_seconds();
            lk.lock();
            inflight.pop_front();
            for (size_t i = 0; i < st->ids.size(); ++i) {
                SrvStream &s = streams[st->ids[i]];
                s.inflight -= 1;
                roi_server_result r{};
                r.tag = st->frames[i].tag;
                r.stream = st->ids[i];
                r.status = err != ROI_OK ? err : st->status[i];
                r.t_arrival = st->frames[i].t_arrival;
                r.t_done = t;
                r.batch = (int32_t)st->ids.size();
                results.push_back(r);
                if (r.status < 0 && error == ROI_OK) error = (roi_status)r.status;
                completed += 1;
            }
            {
                std::lock_guard<std::mutex> g(ev_mu);
                for (hipEvent_t e : st->done) ev_pool.push_back(e);
                for (hipEvent_t e : st->aux) ev_pool.push_back(e);
            }
            delete st;
            cv_sched.notify_one();
            cv_drain.notify_all();
        }
    }
};

bool server_config_ok(const roi_server_config *c)
{
    if (!c) return false;
    if (roi_validate(c->h, c->w, c->dtype, &c->params) != ROI_OK || c->h < 1 || c->w < 1) return false;
    if (c->max_streams < 1 || c->max_streams > 256 || c->max_batch < 1 || c->max_batch > 256) return false;
    if (c->max_inflight < 1 || c->max_inflight > 4 || c->queue_depth < 1 || c->queue_depth > 64) return false;
    return true;
}

} // namespace

extern "C" {

size_t roi_server_stream_bytes(const roi_server_config *cfg)
{
    if (!server_config_ok(cfg)) return 0;
    const size_t fb = align_up((size_t)cfg->h * cfg->w * dtype_bytes(cfg->dtype), ALIGN);
    return roi_stream_state_bytes(cfg->h, cfg->w, cfg->dtype, &cfg->params) + 2 * fb;
}

roi_status roi_server_create(const roi_server_config *cfg, void **out_srv)
{
    if (!out_srv) return ROI_EINVAL;
    *out_srv = nullptr;
    if (!server_config_ok(cfg)) return ROI_EINVAL;
    Server *sv = new Server();
    sv->cfg = *cfg;
    sv->frame_bytes = align_up((size_t)cfg->h * cfg->w * dtype_bytes(cfg->dtype), ALIGN);
    sv->stream_bytes = roi_server_stream_bytes(cfg);
    sv->streams.resize(cfg->max_streams);
    hipGetDevice(&sv->device);
    bool ok = hipStreamCreateWithFlags(&sv->copy_s, hipStreamNonBlocking) == hipSuccess;
    for (int k = 0; k < SRV_COMPUTE_STREAMS && ok; ++k)
        ok = hipStreamCreateWithFlags(&sv->comp_s[k], hipStreamNonBlocking) == hipSuccess;
    if (!ok) {
        delete sv;
        return ROI_EDEVICE;
    }
    sv->sched = std::thread([sv] { sv->scheduler(); });
    sv->comp = std::thread([sv] { sv->completer(); });
    *out_srv = sv;
    return ROI_OK;
}

roi_status roi_server_open_stream(void *srv, int32_t *out_id)
{
    if (!srv || !out_id) return ROI_EINVAL;
    Server *sv = (Server *)srv;
    std::unique_lock<std::mutex> lk(sv->mu);
    int id = -1;
    for (int i = 0; i < (int)sv->streams.size(); ++i)
        if (!sv->streams[i].open && !sv->streams[i].closing) {
            id = i;
            break;
        }
    if (id < 0 || sv->used + sv->stream_bytes > sv->cfg.hbm_budget) return ROI_ENOMEM;
    sv->used += sv->stream_bytes; // reserve before allocating outside the lock
    lk.unlock();
    hipSetDevice(sv->device);
    SrvStream fresh;
    roi_status st = roi_stream_create(sv->cfg.h, sv->cfg.w, sv->cfg.dtype, &sv->cfg.params, (void **)&fresh.ctx);
    if (st == ROI_OK && (hipMalloc((void **)&fresh.slot[0], sv->frame_bytes) != hipSuccess ||
                         hipMalloc((void **)&fresh.slot[1], sv->frame_bytes) != hipSuccess))
        st = ROI_ENOMEM;
    lk.lock();
    if (st != ROI_OK) {
        sv->used -= sv->stream_bytes;
        lk.unlock();
        if (fresh.ctx) roi_stream_destroy(fresh.ctx);
        if (fresh.slot[0]) hipFree(fresh.slot[0]);
        if (fresh.slot[1]) hipFree(fresh.slot[1]);
        return st;
    }
    SrvStream &s = sv->streams[id];
    s.ctx = fresh.ctx;
    s.slot[0] = fresh.slot[0];
    s.slot[1] = fresh.slot[1];
    s.next_slot = 0;
    s.cstream = (sv->rr++) % SRV_COMPUTE_STREAMS;
    s.inflight = 0;
    s.queue.clear();
    s.closing = false;
    s.open = true;
    *out_id = id;
    return ROI_OK;
}

roi_status roi_server_close_stream(void *srv, int32_t id)
{
    if (!srv) return ROI_EINVAL;
    Server *sv = (Server *)srv;
    std::unique_lock<std::mutex> lk(sv->mu);
    if (id < 0 || id >= (int)sv->streams.size() || !sv->streams[id].open) return ROI_EINVAL;
    SrvStream &s = sv->streams[id];
    s.closing = true;
    sv->cv_drain.wait(lk, [&] { return (s.queue.empty() && s.inflight == 0) || sv->error != ROI_OK; });
    s.open = false;
    roi_stream_ctx *ctx = s.ctx;
    uint8_t *a = s.slot[0], *b = s.slot[1];
    s.ctx = nullptr;
    s.slot[0] = s.slot[1] = nullptr;
    s.queue.clear();
    lk.unlock();
    roi_stream_destroy(ctx);
    hipFree(a);
    hipFree(b);
    lk.lock();
    sv->used -= sv->stream_bytes;
    s.closing = false;
    return ROI_OK;
}

roi_status roi_server_submit(void *srv, int32_t id, const void *host_frame, int64_t pitch, float *flow,
                             uint8_t *mask, uint64_t tag)
{
    if (!srv || !host_frame || !flow) return ROI_EINVAL;
    Server *sv = (Server *)srv;
    if (pitch < sv->cfg.w) return ROI_EINVAL;
    std::lock_guard<std::mutex> lk(sv->mu);
    if (id < 0 || id >= (int)sv->streams.size() || !sv->streams[id].open || sv->streams[id].closing)
        return ROI_EINVAL;
    SrvStream &s = sv->streams[id];
    if ((int)s.queue.size() >= sv->cfg.queue_depth) return ROI_ENOMEM;
    s.queue.push_back({host_frame, pitch, flow, mask, tag, now_seconds()});
    sv->submitted += 1;
    sv->cv_sched.notify_one();
    return ROI_OK;
}

int32_t roi_server_poll(void *srv, roi_server_result *out, int32_t max)
{
    if (!srv || !out || max < 1) return 0;
    Server *sv = (Server *)srv;
    std::lock_guard<std::mutex> lk(sv->mu);
    int n = 0;
    while (n < max && !sv->results.empty()) {
        out[n++] = sv->results.front();
        sv->results.pop_front();
    }
    return n;
}

roi_status roi_server_drain(void *srv)
{
    if (!srv) return ROI_EINVAL;
    Server *sv = (Server *)srv;
    std::unique_lock<std::mutex> lk(sv->mu);
    sv->cv_drain.wait(lk, [&] { return sv->completed == sv->submitted || sv->error != ROI_OK; });
    return sv->error;
}

void roi_server_destroy(void *srv)
{
    if (!srv) return;
    Server *sv = (Server *)srv;
    roi_server_drain(srv);
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
        for (SrvStream &s : sv->streams) s.queue.clear();
    }
    sv->cv_sched.notify_all();
    sv->cv_done.notify_all();
    sv->sched.join();
    sv->comp.join();
    hipSetDevice(sv->device);
    hipStreamSynchronize(sv->copy_s);
    for (int k = 0; k < SRV_COMPUTE_STREAMS; ++k) hipStreamSynchronize(sv->comp_s[k]);
    for (SrvStream &s : sv->streams) {
        if (s.ctx) roi_stream_destroy(s.ctx);
        if (s.slot[0]) hipFree(s.slot[0]);
        if (s.slot[1]) hipFree(s.slot[1]);
    }
    for (hipEvent_t e : sv->ev_pool) hipEventDestroy(e);
    hipStreamDestroy(sv->copy_s);
    for (int k = 0; k < SRV_COMPUTE_STREAMS; ++k) hipStreamDestroy(sv->comp_s[k]);
    delete sv;
}

} // extern "C"
