// Serving engine: continuous batching of per-projection solves for many
// patient streams on one GPU (pcr_server_* in include/pcr.h).
//
// A worker thread owns `max_slots` slots, each a HIP stream plus the device
// scratch of one solve in flight.  Queued requests take free slots in arrival
// order (one solve per stream at a time, because each solve warm-starts from
// the stream's previous result).  Every slot runs the same resumable solver
// state machine as pcr_reconstruct_from_projection; the worker polls the
// slots' events and, whenever a slot's line-search trial has finished, feeds
// its moments and immediately enqueues the slot's next trial, so solves of
// different sizes overlap on the device without a global step barrier.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "host.h"

using namespace pcr;

namespace {

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Stream {
    int id = 0;
    pcr_grid grid{};
    pcr_model model{};
    double scale[8];
    pcr_dtype f0_dtype = PCR_F32;
    DevBuf f0, mean, U;
    pcr_solve_opts opts{};
    double w[8];
    // last results and their submit times (history for the predicted warm start)
    double hist_w[3][8];
    double hist_t[3];
    int nhist = 0;
    double mu_last = 0;   // step size the stream's last solve ended with
    bool active = false;
    bool removing = false;
    size_t bytes = 0;
    size_t scratch = 0;
    int queued = 0;
    Support sup;
};

struct Request {
    int64_t id;
    int sid;
    const void* y;
    pcr_geom geom;
    double t_submit;
};

struct Slot {
    hipStream_t s = nullptr;
    hipEvent_t ev = nullptr;
    Scratch sc;
    bool busy = false;
    bool pending = false;   // an evaluation is enqueued
    double t_enq = 0;
    Request req{};
    Stream* st = nullptr;
    Evaluator E{};
    SolveSM sm;
    double t_start = 0;
    double w0[8];
    double mu0 = 0;
};

// Bytes of slot scratch a stream's solves need (fused image + partials +
// moments; partials bounded for detectors up to 2048 x 2048).
size_t slot_scratch_bytes(const pcr_grid& g, int K)
{
    size_t cells = (size_t)(g.n[0] + 3) * (g.n[1] + 3) * (g.n[2] + 3);
    return cells * channels_for(K + 1) * 4 + ((size_t)8 << 20);
}

}  // namespace

struct pcr_server {
    pcr_server_opts o{};
    int device = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::map<int, std::unique_ptr<Stream>> streams;
    int next_sid = 0;
    std::deque<Request> queue;
    int64_t next_req = 0;
    std::deque<pcr_result> results;
    std::vector<std::unique_ptr<Slot>> slots;
    size_t stream_bytes = 0, max_scratch = 0;
    std::thread worker;
    bool stop = false;
    int busy = 0;

    void run();
    bool start_slot(Slot& sl);
    void finish_slot(Slot& sl, pcr_status err);
    size_t footprint(size_t extra_stream, size_t scratch) const
    {
        return stream_bytes + extra_stream + (size_t)o.max_slots * std::max(max_scratch, scratch);
    }
};

static pcr_result base_result(const Request& r, int K)
{
    pcr_result res;
    std::memset(&res, 0, sizeof res);
    res.req_id = r.id;
    res.stream_id = r.sid;
    res.K = K;
    res.t_submit_s = r.t_submit;
    return res;
}

// Binds a slot's evaluator to its request and enqueues the first projection.
bool pcr_server::start_slot(Slot& sl)
{
    Stream* st = sl.st;
    sl.E = Evaluator{&st->grid, &st->model, st->f0_dtype, PCR_F32, st->f0.p, &sl.sc, sl.s};
    sl.E.sup = &st->sup;
    sl.E.image_f16 = o.image_f16 != 0;
    sl.t_start = now_s();
    for (int k = 0; k < 8; ++k) sl.w0[k] = k < st->model.K ? st->w[k] : 0.0;
    if (o.predict_order > 0 && st->nhist >= 2) {
        double wh[3 * 8], th[3];
        const int K = st->model.K;
        for (int i = 0; i < st->nhist; ++i) {
            th[i] = st->hist_t[i];
            for (int k = 0; k < K; ++k) wh[i * K + k] = st->hist_w[i][k];
        }
        double wp[8];
        if (pcr_predict_w(wh, th, st->nhist, K, sl.req.t_submit, o.predict_order, wp) == PCR_OK)
            for (int k = 0; k < K; ++k) sl.w0[k] = wp[k];
    }
    pcr_status e = sl.E.prepare(sl.req.y, sl.req.geom, PCR_GRAD_FUSED);
    if (e == PCR_OK) {
        pcr_solve_opts so = st->opts;
        if (o.chain_step && st->mu_last > 0) so.mu0 = st->mu_last;
        sl.mu0 = so.mu0;
        sl.sm.begin(st->model.K, so, st->model.scale ? st->scale : nullptr, sl.w0);
        e = sl.E.enqueue_eval(sl.sm.eval_w());
    }
    if (e == PCR_OK && hipEventRecord(sl.ev, sl.s) != hipSuccess) e = PCR_EDEVICE;
    if (e != PCR_OK) {
        finish_slot(sl, e);
        return false;
    }
    sl.pending = true;
    sl.t_enq = now_s();
    return true;
}

void pcr_server::finish_slot(Slot& sl, pcr_status err)
{
    Stream* st = sl.st;
    pcr_result res = base_result(sl.req, st->model.K);
    res.t_start_s = sl.t_start;
    for (int k = 0; k < 8; ++k) res.w0[k] = sl.w0[k];
    res.fp_status = PCR_OK;
    if (err == PCR_OK) {
        res.status = sl.sm.status;
        res.iterations = sl.sm.iters;
        res.trials = sl.sm.trials;
        res.J = sl.sm.J;
        res.ab[0] = sl.sm.a;
        res.ab[1] = sl.sm.b;
        res.mu0 = sl.mu0;
        res.mu = sl.sm.mu;
        for (int k = 0; k < st->model.K; ++k) res.w[k] = sl.sm.w[k];
        if (st->opts.localize && (res.status == PCR_OK || res.status == PCR_ENOCONV)) {
            int32_t it = 0;
            res.fp_status = pcr_localize_tumor(&st->grid, &st->model, sl.sm.w, st->opts.p_ref_mm,
                                               st->opts.fp_tol_mm, st->opts.fp_max_iter, res.tumor_mm,
                                               &it, sl.s);
        }
    } else {
        res.status = err;
    }
    res.t_done_s = now_s();
    std::lock_guard<std::mutex> lk(mu);
    if (err == PCR_OK && (res.status == PCR_OK || res.status == PCR_ENOCONV)) {
        for (int k = 0; k < st->model.K; ++k) st->w[k] = res.w[k];
        st->mu_last = sl.sm.mu;
        if (st->nhist == 3) {
            for (int i = 0; i < 2; ++i) {
                st->hist_t[i] = st->hist_t[i + 1];
                for (int k = 0; k < 8; ++k) st->hist_w[i][k] = st->hist_w[i + 1][k];
            }
            st->nhist = 2;
        }
        st->hist_t[st->nhist] = sl.req.t_submit;
        for (int k = 0; k < 8; ++k) st->hist_w[st->nhist][k] = res.w[k];
        ++st->nhist;
    }
    st->active = false;
    sl.busy = false;
    sl.pending = false;
    sl.st = nullptr;
    --busy;
    results.push_back(res);
    cv_done.notify_all();
    cv_work.notify_all();
}

void pcr_server::run()
{
    (void)hipSetDevice(device);
    for (;;) {
        std::vector<Slot*> fresh;
        {
            std::unique_lock<std::mutex> lk(mu);
            if (busy == 0 && queue.empty()) {
                if (stop) break;
                cv_work.wait_for(lk, std::chrono::milliseconds(20));
                continue;
            }
            // admission: free slots take the oldest requests of idle streams
            for (auto& sp : slots) {
                if (sp->busy) continue;
                auto it = std::find_if(queue.begin(), queue.end(), [&](const Request& r) {
                    auto s = streams.find(r.sid);
                    return s != streams.end() && !s->second->active;
                });
                if (it == queue.end()) break;
                Stream* st = streams[it->sid].get();
                st->active = true;
                st->queued--;
                sp->busy = true;
                sp->req = *it;
                sp->st = st;
                ++busy;
                queue.erase(it);
                fresh.push_back(sp.get());
            }
        }
        for (Slot* sl : fresh) start_slot(*sl);
        // progress every slot whose trial has finished
        bool progressed = false;
        Slot* oldest = nullptr;
        for (auto& sp : slots) {
            Slot& sl = *sp;
            if (!sl.busy || !sl.pending) continue;
            hipError_t q = hipEventQuery(sl.ev);
            if (q == hipErrorNotReady) {
                if (!oldest || sl.t_enq < oldest->t_enq) oldest = &sl;
                continue;
            }
            progressed = true;
            sl.pending = false;
            if (q != hipSuccess) {
                finish_slot(sl, fail(PCR_EDEVICE, "serving slot: %s", hipGetErrorString(q)));
                continue;
            }
            Moments mo;
            sl.E.collect(mo);
            auto no_grad = [](const double*, double, double, double*) { return PCR_EINVAL; };
            pcr_status e = sl.sm.feed(mo, no_grad);
            if (e != PCR_OK || sl.sm.done()) {
                finish_slot(sl, e);
                continue;
            }
            e = sl.E.enqueue_eval(sl.sm.eval_w());
            if (e == PCR_OK && hipEventRecord(sl.ev, sl.s) != hipSuccess) e = PCR_EDEVICE;
            if (e != PCR_OK) {
                finish_slot(sl, e);
                continue;
            }
            sl.pending = true;
            sl.t_enq = now_s();
        }
        if (!progressed && oldest) (void)hipEventSynchronize(oldest->ev);
    }
}

extern "C" {

pcr_status pcr_server_create(const pcr_server_opts* opts, pcr_server** out)
{
    if (!opts || !out) return fail(PCR_EINVAL, "NULL argument");
    *out = nullptr;
    if (opts->max_slots < 1 || opts->max_slots > 64) return fail(PCR_EINVAL, "max_slots must be in 1..64");
    if (opts->predict_order < 0 || opts->predict_order > 2) return fail(PCR_EINVAL, "predict_order must be 0..2");
    if (opts->hbm_budget_bytes == 0) return fail(PCR_EINVAL, "hbm_budget_bytes must be > 0");
    auto S = std::make_unique<pcr_server>();
    S->o = *opts;
    HIP_TRY(hipGetDevice(&S->device));
    for (int i = 0; i < opts->max_slots; ++i) {
        auto sl = std::make_unique<Slot>();
        HIP_TRY(hipStreamCreateWithFlags(&sl->s, hipStreamNonBlocking));
        HIP_TRY(hipEventCreateWithFlags(&sl->ev, hipEventDisableTiming));
        sl->sc.device = S->device;
        S->slots.push_back(std::move(sl));
    }
    pcr_server* raw = S.release();
    raw->worker = std::thread([raw] { raw->run(); });
    *out = raw;
    return PCR_OK;
}

void pcr_server_destroy(pcr_server* S)
{
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
        S->queue.clear();
        for (auto& kv : S->streams) kv.second->queued = 0;
    }
    S->cv_work.notify_all();
    if (S->worker.joinable()) S->worker.join();
    (void)hipSetDevice(S->device);
    (void)hipDeviceSynchronize();
    for (auto& sl : S->slots) {
        sl->sc.release();
        if (sl->ev) (void)hipEventDestroy(sl->ev);
        if (sl->s) (void)hipStreamDestroy(sl->s);
    }
    for (auto& kv : S->streams) {
        kv.second->f0.release();
        kv.second->mean.release();
        kv.second->U.release();
    }
    delete S;
}

pcr_status pcr_server_add_stream(pcr_server* S, const pcr_grid* grid, const pcr_model* model,
                                 pcr_dtype f0_dtype, const void* f0_dev, const pcr_solve_opts* opts,
                                 const double* w0, int32_t* stream_id)
{
    if (!S || !stream_id) return fail(PCR_EINVAL, "NULL argument");
    PCR_TRY(check_grid(grid));
    PCR_TRY(check_model(model));
    PCR_TRY(check_storage(f0_dtype));
    PCR_TRY(check_opts(opts));
    PCR_TRY(check_finite(w0, model->K, "w0"));
    if (!f0_dev) return fail(PCR_EINVAL, "f0_dev is NULL");
    if (opts->grad_mode != PCR_GRAD_FUSED) return fail(PCR_EINVAL, "serving uses the fused gradient");
    const int K = model->K;
    if ((double)(grid->n[0] + 3) * (grid->n[1] + 3) * (grid->n[2] + 3) * channels_for(K + 1) * 4 >= 2147483648.0)
        return fail(PCR_EINVAL, "padded multi-channel image exceeds 2 GiB (32-bit offsets)");
    auto st = std::make_unique<Stream>();
    st->grid = *grid;
    st->f0_dtype = f0_dtype;
    st->opts = *opts;
    for (int k = 0; k < 8; ++k) {
        st->scale[k] = (model->scale && k < K) ? model->scale[k] : 1.0;
        st->w[k] = k < K ? w0[k] : 0.0;
    }
    const size_t N = (size_t)grid->n[0] * grid->n[1] * grid->n[2];
    const size_t es = dtype_size(model->storage);
    st->bytes = model_bytes(*grid, K, model->storage, f0_dtype);
    st->scratch = slot_scratch_bytes(*grid, K);
    {
        std::lock_guard<std::mutex> lk(S->mu);
        size_t need = S->footprint(st->bytes, st->scratch);
        if (need > S->o.hbm_budget_bytes)
            return fail(PCR_EBUSY, "admission refused: %.3g GB needed, budget %.3g GB", need * 1e-9,
                        S->o.hbm_budget_bytes * 1e-9);
        // reserve before allocating so concurrent admissions see it
        S->stream_bytes += st->bytes;
        S->max_scratch = std::max(S->max_scratch, st->scratch);
    }
    auto unreserve = [&](pcr_status e) {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stream_bytes -= st->bytes;
        return e;
    };
    pcr_status e = st->f0.ensure(N * dtype_size(f0_dtype), S->device, nullptr);
    if (e == PCR_OK) e = st->mean.ensure(3 * N * es, S->device, nullptr);
    if (e == PCR_OK) e = st->U.ensure((size_t)K * 3 * N * es, S->device, nullptr);
    if (e != PCR_OK) return unreserve(e);
    hipError_t he = hipMemcpy(st->f0.p, f0_dev, N * dtype_size(f0_dtype), hipMemcpyDeviceToDevice);
    if (he == hipSuccess) he = hipMemcpy(st->mean.p, model->mean, 3 * N * es, hipMemcpyDeviceToDevice);
    if (he == hipSuccess) he = hipMemcpy(st->U.p, model->U, (size_t)K * 3 * N * es, hipMemcpyDeviceToDevice);
    if (he != hipSuccess) return unreserve(fail(PCR_EDEVICE, "stream copy: %s", hipGetErrorString(he)));
    st->model.K = K;
    st->model.storage = model->storage;
    st->model.mean = st->mean.p;
    st->model.U = st->U.p;
    st->model.scale = model->scale ? st->scale : nullptr;
    e = compute_support(st->grid, st->model, st->f0_dtype, st->f0.p, S->device, nullptr, &st->sup);
    if (e != PCR_OK) return unreserve(e);
    std::lock_guard<std::mutex> lk(S->mu);
    st->id = S->next_sid++;
    *stream_id = st->id;
    S->streams[st->id] = std::move(st);
    return PCR_OK;
}

pcr_status pcr_server_remove_stream(pcr_server* S, int32_t sid)
{
    if (!S) return fail(PCR_EINVAL, "NULL server");
    std::unique_ptr<Stream> st;
    {
        std::unique_lock<std::mutex> lk(S->mu);
        auto it = S->streams.find(sid);
        if (it == S->streams.end()) return fail(PCR_EINVAL, "unknown stream %d", sid);
        Stream* p = it->second.get();
        p->removing = true;
        for (auto q = S->queue.begin(); q != S->queue.end();) {
            if (q->sid == sid) {
                pcr_result r = base_result(*q, p->model.K);
                r.status = PCR_EBUSY;
                r.t_done_s = now_s();
                S->results.push_back(r);
                q = S->queue.erase(q);
            } else {
                ++q;
            }
        }
        p->queued = 0;
        S->cv_done.wait(lk, [&] { return !p->active; });
        st = std::move(it->second);
        S->streams.erase(it);
        S->stream_bytes -= st->bytes;
    }
    st->f0.release();
    st->mean.release();
    st->U.release();
    return PCR_OK;
}

pcr_status pcr_server_submit(pcr_server* S, int32_t sid, const void* y_dev, const pcr_geom* geom,
                             int64_t* req_id)
{
    if (!S || !y_dev) return fail(PCR_EINVAL, "NULL argument");
    PCR_TRY(check_geom(geom));
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->streams.find(sid);
    if (it == S->streams.end() || it->second->removing) return fail(PCR_EINVAL, "unknown stream %d", sid);
    Stream* st = it->second.get();
    if (S->o.drop_stale && st->queued > 0) {
        for (auto q = S->queue.begin(); q != S->queue.end(); ++q) {
            if (q->sid != sid) continue;
            pcr_result r = base_result(*q, st->model.K);
            r.status = PCR_EBUSY;
            r.t_done_s = now_s();
            S->results.push_back(r);
            S->queue.erase(q);
            st->queued--;
            break;
        }
    }
    Request r{S->next_req++, sid, y_dev, *geom, now_s()};
    S->queue.push_back(r);
    st->queued++;
    if (req_id) *req_id = r.id;
    S->cv_work.notify_all();
    S->cv_done.notify_all();
    return PCR_OK;
}

pcr_status pcr_server_poll(pcr_server* S, pcr_result* out, int32_t max, int32_t* n, int32_t wait_ms)
{
    if (!S || !n || (max > 0 && !out)) return fail(PCR_EINVAL, "NULL argument");
    std::unique_lock<std::mutex> lk(S->mu);
    if (S->results.empty() && wait_ms > 0)
        S->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), [&] { return !S->results.empty(); });
    int k = 0;
    while (k < max && !S->results.empty()) {
        out[k++] = S->results.front();
        S->results.pop_front();
    }
    *n = k;
    return PCR_OK;
}

pcr_status pcr_server_drain(pcr_server* S, int32_t timeout_ms)
{
    if (!S) return fail(PCR_EINVAL, "NULL server");
    std::unique_lock<std::mutex> lk(S->mu);
    auto idle = [&] { return S->queue.empty() && S->busy == 0; };
    if (timeout_ms < 0) {
        S->cv_done.wait(lk, idle);
        return PCR_OK;
    }
    if (!S->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), idle))
        return fail(PCR_EBUSY, "drain timed out");
    return PCR_OK;
}

pcr_status pcr_server_get_w(pcr_server* S, int32_t sid, double* w_out)
{
    if (!S || !w_out) return fail(PCR_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->streams.find(sid);
    if (it == S->streams.end()) return fail(PCR_EINVAL, "unknown stream %d", sid);
    for (int k = 0; k < it->second->model.K; ++k) w_out[k] = it->second->w[k];
    return PCR_OK;
}

pcr_status pcr_server_set_w(pcr_server* S, int32_t sid, const double* w)
{
    if (!S) return fail(PCR_EINVAL, "NULL server");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->streams.find(sid);
    if (it == S->streams.end()) return fail(PCR_EINVAL, "unknown stream %d", sid);
    PCR_TRY(check_finite(w, it->second->model.K, "w"));
    if (it->second->active) return fail(PCR_EBUSY, "stream %d has a solve in flight", sid);
    for (int k = 0; k < it->second->model.K; ++k) it->second->w[k] = w[k];
    it->second->nhist = 0;
    it->second->mu_last = 0;
    return PCR_OK;
}

size_t pcr_server_device_bytes(const pcr_server* S)
{
    if (!S) return 0;
    auto* s = const_cast<pcr_server*>(S);
    std::lock_guard<std::mutex> lk(s->mu);
    size_t b = s->stream_bytes;
    for (auto& sl : s->slots) b += sl->sc.device_bytes();
    return b;
}

}  // extern "C"
