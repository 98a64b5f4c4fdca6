// Serving engine: continuous batching of per-projection solves for many
// patient streams on one GPU (pcr_server_* in include/pcr.h).
//
// The scheduling policies (admission, the request queue, warm starts, stream
// removal, result delivery) live in scheduler.h, free of device code.  This file
// is the HIP executor they drive: `max_slots` slots, each a HIP stream plus
// the device scratch of one solve in flight.  Every slot runs the same
// resumable solver state machine as pcr_reconstruct_from_projection; the
// worker polls the slots' events and, whenever a slot's line-search trial has
// finished, feeds its moments and immediately enqueues the slot's next trial,
// so solves of different sizes overlap on the device without a global step
// barrier.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <memory>
#include <mutex>
#include <vector>

#include "host.h"
#include "scheduler.h"

using namespace pcr;

namespace {

// A stream's device data: server-owned copies of its reference image and
// model, its solve options and its support box.
struct StreamDev {
    pcr_grid grid{};
    pcr_model model{};
    double scale[8];
    pcr_dtype f0_dtype = PCR_F32;
    DevBuf f0, mean, U;
    pcr_solve_opts opts{};
    Support sup;

    void release()
    {
        f0.release();
        mean.release();
        U.release();
        sup.release();
    }
};

struct Slot {
    hipStream_t s = nullptr;
    hipEvent_t ev = nullptr;
    Scratch sc;
    bool pending = false;     // an evaluation is enqueued
    pcr_status err = PCR_OK;  // a failure to start, reported by the next advance()
    double mu0 = 0;           // first trial step of the solve (0: the default rule)
    double step0 = 0;         // first trial distance (when mu0 is 0)
    StreamDev* st = nullptr;
    Evaluator E{};
    SolveSM sm;
};

size_t fused_image_bytes(const pcr_grid& g, int K)
{
    size_t cells = (size_t)(g.n[0] + 3) * (g.n[1] + 3) * (g.n[2] + 3);
    return cells * channels_for(K + 1) * 4;
}

// Bytes of slot scratch a stream's solves need (fused image + partials +
// moments; partials bounded for detectors up to 2048 x 2048).
size_t slot_scratch_bytes(const pcr_grid& g, int K)
{
    return fused_image_bytes(g, K) + ((size_t)8 << 20);
}

struct HipExec {
    int device = 0;
    bool image_f16 = false;
    std::vector<std::unique_ptr<Slot>> slots;
    std::mutex smu;   // guards streams and max_image
    std::map<int, std::unique_ptr<StreamDev>> streams;
    size_t max_image = 0;   // largest fused image (FP32 cells) of an admitted stream

    bool start(int slot, const sched::Request& r, int sid, const double* w0, double mu0, double move);
    int advance(int slot, pcr_result* res);
    void wait_any();
    void forget_stream(int sid);
};

// Binds a slot's evaluator to its request and enqueues the first projection.
bool HipExec::start(int slot, const sched::Request& r, int sid, const double* w0, double mu0,
                    double move)
{
    Slot& sl = *slots[slot];
    sl.pending = false;
    sl.err = PCR_OK;
    sl.mu0 = 0;
    {
        std::lock_guard<std::mutex> lk(smu);
        auto it = streams.find(sid);
        sl.st = it == streams.end() ? nullptr : it->second.get();
        // size the slot's fused image once for the largest admitted stream,
        // so that streams of other sizes do not reallocate it in the loop
        sl.sc.volc_floor = max_image;
    }
    if (!sl.st) {
        sl.err = fail(PCR_EINVAL, "serving slot: stream %d has no device data", sid);
        return false;
    }
    StreamDev* st = sl.st;
    sl.E = Evaluator{&st->grid, &st->model, st->f0_dtype, PCR_F32, st->f0.p, &sl.sc, sl.s};
    sl.E.sup = &st->sup;
    sl.E.image_f16 = image_f16;
    pcr_status e = sl.E.prepare(r.y, r.geom, PCR_GRAD_FUSED);
    if (e == PCR_OK) {
        pcr_solve_opts so = st->opts;
        if (mu0 > 0) so.mu0 = mu0;
        if (move >= 0) so.step0 = std::min(std::max(move, 1e-3 * so.step0), so.step0);
        sl.mu0 = so.mu0;
        sl.step0 = so.mu0 > 0 ? 0.0 : so.step0;
        sl.sm.begin(st->model.K, so, st->model.scale ? st->scale : nullptr, w0);
        e = sl.E.enqueue_eval(sl.sm.eval_w());
    }
    if (e == PCR_OK && hipEventRecord(sl.ev, sl.s) != hipSuccess) e = PCR_EDEVICE;
    if (e != PCR_OK) {
        sl.err = e;
        return false;
    }
    sl.pending = true;
    return true;
}

// Whether the slot's last evaluation has published its moments.
static bool published(const Slot& sl)
{
    const unsigned long long* done = (const unsigned long long*)(sl.sc.host.p + kDoneSlot);
    return __atomic_load_n(done, __ATOMIC_ACQUIRE) == sl.sc.seq;
}

int HipExec::advance(int slot, pcr_result* res)
{
    Slot& sl = *slots[slot];
    if (sl.err != PCR_OK) {
        res->status = sl.err;
        sl.err = PCR_OK;
        return 2;
    }
    if (!sl.pending) return 0;
    if (!published(sl)) {
        const hipError_t q = hipEventQuery(sl.ev);
        if (q == hipErrorNotReady) return 0;
        sl.pending = false;
        if (q != hipSuccess) {
            res->status = fail(PCR_EDEVICE, "serving slot: %s", hipGetErrorString(q));
            return 2;
        }
        if (!published(sl)) {
            res->status = fail(PCR_EDEVICE, "serving slot: evaluation finished without publishing");
            return 2;
        }
    }
    sl.pending = false;
    Moments mo;
    sl.E.collect(mo);
    auto no_grad = [](const double*, double, double, double*) { return PCR_EINVAL; };
    pcr_status e = sl.sm.feed(mo, no_grad);
    if (e == PCR_OK && !sl.sm.done()) {
        e = sl.E.enqueue_eval(sl.sm.eval_w());
        if (e == PCR_OK && hipEventRecord(sl.ev, sl.s) != hipSuccess) e = PCR_EDEVICE;
        if (e == PCR_OK) {
            sl.pending = true;
            return 1;
        }
    }
    if (e != PCR_OK) {
        res->status = e;
        return 2;
    }
    // the solve is done: its result, then the tumour position
    const StreamDev* st = sl.st;
    res->status = sl.sm.status;
    res->iterations = sl.sm.iters;
    res->trials = sl.sm.trials;
    res->J = sl.sm.J;
    res->ab[0] = sl.sm.a;
    res->ab[1] = sl.sm.b;
    res->mu0 = sl.mu0;
    res->step0 = sl.step0;
    res->mu = sl.sm.mu;
    res->samples = sl.sm.samples;
    for (int k = 0; k < st->model.K; ++k) res->w[k] = sl.sm.w[k];
    res->fp_status = PCR_OK;
    if (st->opts.localize && (res->status == PCR_OK || res->status == PCR_ENOCONV)) {
        int32_t it = 0;
        res->fp_status = pcr_localize_tumor(&st->grid, &st->model, sl.sm.w, st->opts.p_ref_mm,
                                            st->opts.fp_tol_mm, st->opts.fp_max_iter, res->tumor_mm,
                                            &it, sl.s);
    }
    return 2;
}

// Spins until some pending slot has published its moments, or (checked now
// and then) some slot's stream has finished or failed; returns at once when
// nothing is pending.
void HipExec::wait_any()
{
    for (unsigned long n = 1;; ++n) {
        bool any = false;
        for (auto& sp : slots) {
            if (!sp->pending) continue;
            any = true;
            if (published(*sp)) return;
        }
        if (!any) return;
        if ((n & 1023) == 0)
            for (auto& sp : slots)
                if (sp->pending && hipEventQuery(sp->ev) != hipErrorNotReady) return;
        __builtin_ia32_pause();
    }
}

void HipExec::forget_stream(int sid)
{
    std::unique_ptr<StreamDev> st;
    {
        std::lock_guard<std::mutex> lk(smu);
        auto it = streams.find(sid);
        if (it == streams.end()) return;
        st = std::move(it->second);
        streams.erase(it);
    }
    st->release();
}

sched::Options core_options(const pcr_server_opts& o)
{
    sched::Options c;
    c.budget = o.hbm_budget_bytes;
    c.slots = o.max_slots;
    c.drop_stale = o.drop_stale != 0;
    c.predict_order = o.predict_order;
    c.chain_step = o.chain_step != 0;
    c.carry_move = o.carry_move != 0;
    return c;
}

}  // namespace

struct pcr_server {
    pcr_server_opts o{};
    HipExec ex;
    std::unique_ptr<sched::Core<HipExec>> core;   // destroyed before ex
};

extern "C" {

pcr_status pcr_server_create(const pcr_server_opts* opts, pcr_server** out)
{
    if (!opts || !out) return fail(PCR_EINVAL, "NULL argument");
    *out = nullptr;
    if (opts->max_slots < 1 || opts->max_slots > 64) return fail(PCR_EINVAL, "max_slots must be in 1..64");
    if (opts->predict_order < 0 || opts->predict_order > 2) return fail(PCR_EINVAL, "predict_order must be 0..2");
    if (opts->hbm_budget_bytes == 0) return fail(PCR_EINVAL, "hbm_budget_bytes must be > 0");
    if (opts->chain_step && opts->carry_move)
        return fail(PCR_EINVAL, "chain_step and carry_move are alternatives: set one");
    auto S = std::make_unique<pcr_server>();
    S->o = *opts;
    HIP_TRY(hipGetDevice(&S->ex.device));
    S->ex.image_f16 = opts->image_f16 != 0;
    for (int i = 0; i < opts->max_slots; ++i) {
        auto sl = std::make_unique<Slot>();
        HIP_TRY(hipStreamCreateWithFlags(&sl->s, hipStreamNonBlocking));
        HIP_TRY(hipEventCreateWithFlags(&sl->ev, hipEventDisableTiming));
        sl->sc.device = S->ex.device;
        S->ex.slots.push_back(std::move(sl));
    }
    S->core = std::make_unique<sched::Core<HipExec>>(core_options(*opts), S->ex);
    const int dev = S->ex.device;
    S->core->start_worker_on([dev] { (void)hipSetDevice(dev); });
    *out = S.release();
    return PCR_OK;
}

void pcr_server_destroy(pcr_server* S)
{
    if (!S) return;
    S->core->stop();
    (void)hipSetDevice(S->ex.device);
    (void)hipDeviceSynchronize();
    for (auto& sl : S->ex.slots) {
        sl->sc.release();
        if (sl->ev) (void)hipEventDestroy(sl->ev);
        if (sl->s) (void)hipStreamDestroy(sl->s);
    }
    for (auto& kv : S->ex.streams) kv.second->release();
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
    PCR_TRY(check_march_image(*grid, channels_for(K + 1), PCR_F32));
    const size_t bytes = model_bytes(*grid, K, model->storage, f0_dtype);
    const size_t scratch = slot_scratch_bytes(*grid, K);
    // reserve before allocating, so that concurrent admissions see it
    const int sid = S->core->reserve_stream(K, bytes, scratch, w0);
    if (sid < 0)
        return fail(PCR_EBUSY, "admission refused: %.3g GB needed, budget %.3g GB",
                    S->core->footprint(bytes, scratch) * 1e-9, S->o.hbm_budget_bytes * 1e-9);
    auto unreserve = [&](pcr_status e) {
        S->core->unreserve_stream(sid);
        return e;
    };
    auto st = std::make_unique<StreamDev>();
    st->grid = *grid;
    st->f0_dtype = f0_dtype;
    st->opts = *opts;
    for (int k = 0; k < 8; ++k) st->scale[k] = (model->scale && k < K) ? model->scale[k] : 1.0;
    const size_t N = (size_t)grid->n[0] * grid->n[1] * grid->n[2];
    const size_t es = dtype_size(model->storage);
    pcr_status e = st->f0.ensure(N * dtype_size(f0_dtype), S->ex.device, nullptr);
    if (e == PCR_OK) e = st->mean.ensure(3 * N * es, S->ex.device, nullptr);
    if (e == PCR_OK) e = st->U.ensure((size_t)K * 3 * N * es, S->ex.device, nullptr);
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
    e = compute_support(st->grid, st->model, st->f0_dtype, st->f0.p, S->ex.device, nullptr, &st->sup);
    if (e != PCR_OK) return unreserve(e);
    {
        std::lock_guard<std::mutex> lk(S->ex.smu);
        S->ex.max_image = std::max(S->ex.max_image, fused_image_bytes(*grid, K));
        S->ex.streams[sid] = std::move(st);
    }
    S->core->commit_stream(sid);
    *stream_id = sid;
    return PCR_OK;
}

pcr_status pcr_server_remove_stream(pcr_server* S, int32_t sid)
{
    if (!S) return fail(PCR_EINVAL, "NULL server");
    if (S->core->remove_stream(sid) != PCR_OK) return fail(PCR_EINVAL, "unknown stream %d", sid);
    return PCR_OK;
}

pcr_status pcr_server_submit(pcr_server* S, int32_t sid, const void* y_dev, const pcr_geom* geom,
                             int64_t* req_id)
{
    if (!S || !y_dev) return fail(PCR_EINVAL, "NULL argument");
    PCR_TRY(check_geom(geom));
    if (S->core->submit(sid, y_dev, *geom, req_id) != PCR_OK) return fail(PCR_EINVAL, "unknown stream %d", sid);
    return PCR_OK;
}

pcr_status pcr_server_poll(pcr_server* S, pcr_result* out, int32_t max, int32_t* n, int32_t wait_ms)
{
    if (!S || !n || (max > 0 && !out)) return fail(PCR_EINVAL, "NULL argument");
    *n = S->core->poll(out, max, wait_ms);
    return PCR_OK;
}

pcr_status pcr_server_drain(pcr_server* S, int32_t timeout_ms)
{
    if (!S) return fail(PCR_EINVAL, "NULL server");
    if (!S->core->drain(timeout_ms)) return fail(PCR_EBUSY, "drain timed out");
    return PCR_OK;
}

pcr_status pcr_server_get_w(pcr_server* S, int32_t sid, double* w_out)
{
    if (!S || !w_out) return fail(PCR_EINVAL, "NULL argument");
    if (S->core->get_w(sid, w_out) != PCR_OK) return fail(PCR_EINVAL, "unknown stream %d", sid);
    return PCR_OK;
}

pcr_status pcr_server_set_w(pcr_server* S, int32_t sid, const double* w)
{
    if (!S) return fail(PCR_EINVAL, "NULL server");
    const int K = S->core->stream_K(sid);
    if (K < 0) return fail(PCR_EINVAL, "unknown stream %d", sid);
    PCR_TRY(check_finite(w, K, "w"));
    const pcr_status e = S->core->set_w(sid, w);
    if (e == PCR_EBUSY) return fail(PCR_EBUSY, "stream %d has a solve in flight", sid);
    if (e != PCR_OK) return fail(PCR_EINVAL, "unknown stream %d", sid);
    return PCR_OK;
}

size_t pcr_server_device_bytes(const pcr_server* S)
{
    if (!S) return 0;
    size_t b = S->core->stream_bytes();
    for (auto& sl : S->ex.slots) b += sl->sc.device_bytes();
    return b;
}

}  // extern "C"
