// Request scheduling of the serving engine (pcr_server_* in include/pcr.h),
// free of device code: admission by memory footprint, the request queue
// (stale-frame dropping, one solve per stream at a time, oldest first),
// slot assignment, warm starts (the stream's last result, or its
// extrapolation in time), step-size carry-over, stream removal and result
// delivery.  The device work of a solve is delegated to an executor, so the
// same policies run with the HIP executor in serve.hip and with stand-in
// executors in CPU tests.
//
// Executor interface (duck-typed):
//   bool start(int slot, const Request& r, int sid, const double* w0, double mu0,
//              double move);
//       begin a solve in `slot` (mu0 > 0: its first trial's step size; move
//       >= 0: the distance the stream's previous solve moved w, from which
//       the first trial's distance is set); false if it could not start (the
//       executor then reports the failure from the next advance()).
//   int advance(int slot, pcr_result* res);
//       0: nothing new; 1: progressed, still running; 2: finished, `res`
//       holds status, iterations, trials, w, ab, J, tumour, mu0, mu (the
//       scheduler fills the ids, K, times and w0).
//   void wait_any();
//       block until some slot's pending work may have completed.
//   void forget_stream(int sid);   the stream's device data may be freed.
#pragma once

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "pcr.h"

namespace pcr {
namespace sched {

inline double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Value at t_next of the polynomial of degree d = min(order, n - 1) through
// the last d + 1 points (t_hist[i], w_hist[i][.]) (Lagrange form); inputs
// already validated.
inline void extrapolate_w(const double* w_hist, const double* t_hist, int n, int K, double t_next,
                          int order, double* w_out)
{
    const int d = std::min(order, n - 1);
    const int first = n - 1 - d;
    for (int k = 0; k < K; ++k) w_out[k] = 0.0;
    for (int i = first; i < n; ++i) {
        double L = 1.0;
        for (int j = first; j < n; ++j)
            if (j != i) L *= (t_next - t_hist[j]) / (t_hist[i] - t_hist[j]);
        for (int k = 0; k < K; ++k) w_out[k] += L * w_hist[i * K + k];
    }
}

struct Request {
    int64_t id;
    int sid;
    const void* y;
    pcr_geom geom;
    double t_submit;
};

struct StreamState {
    int K = 0;
    bool active = false;     // a solve of this stream is in a slot
    bool removing = false;
    int queued = 0;
    double w[8] = {0};       // warm start: the last result
    double hist_w[3][8];     // last results and their submit times
    double hist_t[3];
    int nhist = 0;
    double mu_last = 0;      // step size the last solve ended with
    double move_last = -1;   // distance the last solve moved w (< 0: none yet)
    size_t bytes = 0;        // device bytes of the stream's own data
    size_t scratch = 0;      // slot scratch its solves need
};

struct Options {
    size_t budget = 0;
    int slots = 1;
    bool drop_stale = true;
    int predict_order = 0;
    bool chain_step = false;
    bool carry_move = false;
};

template <class Exec>
class Core {
  public:
    Core(const Options& o, Exec& e)
        : o_(o), ex_(e), slot_busy_(o.slots, 0), slot_sid_(o.slots, -1), slot_req_(o.slots),
          slot_w0_(o.slots, std::vector<double>(8, 0.0)), slot_t_start_(o.slots, 0.0)
    {
    }
    ~Core() { stop(); }

    // Starts the worker thread; `init` runs on it first (e.g. to bind the
    // device).
    void start_worker_on(std::function<void()> init)
    {
        worker_ = std::thread([this, init] {
            if (init) init();
            run();
        });
    }
    // Stops the worker after the solves in flight; queued requests are dropped.
    void stop()
    {
        {
            std::lock_guard<std::mutex> lk(mu_);
            if (stopping_) return;
            stopping_ = true;
            queue_.clear();
            for (auto& kv : streams_) kv.second.queued = 0;
        }
        cv_work_.notify_all();
        if (worker_.joinable()) worker_.join();
    }

    // Bytes the server would hold with one more stream of `bytes` own data
    // whose solves need `scratch` bytes per slot.
    size_t footprint(size_t bytes, size_t scratch) const
    {
        return stream_bytes_ + bytes + (size_t)o_.slots * std::max(max_scratch_, scratch);
    }
    // Admission by footprint: reserves the stream's bytes and returns its id,
    // or -1 (nothing reserved) when the budget would be exceeded.
    int reserve_stream(int K, size_t bytes, size_t scratch, const double* w0)
    {
        std::lock_guard<std::mutex> lk(mu_);
        if (footprint(bytes, scratch) > o_.budget) return -1;
        const int sid = next_sid_++;
        StreamState st;
        st.K = K;
        st.bytes = bytes;
        st.scratch = scratch;
        st.removing = true;   // not submittable until committed
        for (int k = 0; k < 8; ++k) st.w[k] = k < K ? w0[k] : 0.0;
        streams_[sid] = st;
        stream_bytes_ += bytes;
        max_scratch_ = std::max(max_scratch_, scratch);
        return sid;
    }
    void commit_stream(int sid)
    {
        std::lock_guard<std::mutex> lk(mu_);
        streams_[sid].removing = false;
    }
    void unreserve_stream(int sid)
    {
        std::lock_guard<std::mutex> lk(mu_);
        auto it = streams_.find(sid);
        if (it == streams_.end()) return;
        stream_bytes_ -= it->second.bytes;
        streams_.erase(it);
    }
    size_t max_scratch() const
    {
        std::lock_guard<std::mutex> lk(mu_);
        return max_scratch_;
    }
    size_t stream_bytes() const
    {
        std::lock_guard<std::mutex> lk(mu_);
        return stream_bytes_;
    }

    // Queues a request; with drop_stale a queued (not started) request of
    // the same stream is answered PCR_EBUSY and replaced.
    pcr_status submit(int sid, const void* y, const pcr_geom& geom, int64_t* req_id)
    {
        std::lock_guard<std::mutex> lk(mu_);
        auto it = streams_.find(sid);
        if (it == streams_.end() || it->second.removing || stopping_) return PCR_EINVAL;
        StreamState& st = it->second;
        if (o_.drop_stale && st.queued > 0) {
            for (auto q = queue_.begin(); q != queue_.end(); ++q) {
                if (q->sid != sid) continue;
                push_dropped(*q, st.K);
                queue_.erase(q);
                st.queued--;
                break;
            }
        }
        Request r{next_req_++, sid, y, geom, now_s()};
        queue_.push_back(r);
        st.queued++;
        if (req_id) *req_id = r.id;
        cv_work_.notify_all();
        cv_done_.notify_all();
        return PCR_OK;
    }

    // Removes a stream: its queued requests are answered PCR_EBUSY, an
    // in-flight solve finishes first.
    pcr_status remove_stream(int sid)
    {
        std::unique_lock<std::mutex> lk(mu_);
        auto it = streams_.find(sid);
        if (it == streams_.end() || it->second.removing) return PCR_EINVAL;
        it->second.removing = true;
        for (auto q = queue_.begin(); q != queue_.end();) {
            if (q->sid == sid) {
                push_dropped(*q, it->second.K);
                q = queue_.erase(q);
            } else {
                ++q;
            }
        }
        it->second.queued = 0;
        cv_done_.wait(lk, [&] { return !streams_[sid].active; });
        stream_bytes_ -= streams_[sid].bytes;
        streams_.erase(sid);
        lk.unlock();
        ex_.forget_stream(sid);
        return PCR_OK;
    }

    int poll(pcr_result* out, int max, int wait_ms)
    {
        std::unique_lock<std::mutex> lk(mu_);
        if (results_.empty() && wait_ms > 0)
            cv_done_.wait_for(lk, std::chrono::milliseconds(wait_ms), [&] { return !results_.empty(); });
        int k = 0;
        while (k < max && !results_.empty()) {
            out[k++] = results_.front();
            results_.pop_front();
        }
        return k;
    }

    // Waits until the queue is empty and no solve is in flight; false on
    // timeout (timeout_ms >= 0).
    bool drain(int timeout_ms)
    {
        std::unique_lock<std::mutex> lk(mu_);
        auto idle = [&] { return queue_.empty() && busy_ == 0; };
        if (timeout_ms < 0) {
            cv_done_.wait(lk, idle);
            return true;
        }
        return cv_done_.wait_for(lk, std::chrono::milliseconds(timeout_ms), idle);
    }

    pcr_status get_w(int sid, double* w) const
    {
        std::lock_guard<std::mutex> lk(mu_);
        auto it = streams_.find(sid);
        if (it == streams_.end()) return PCR_EINVAL;
        for (int k = 0; k < it->second.K; ++k) w[k] = it->second.w[k];
        return PCR_OK;
    }
    // Replaces the warm start; forgets the history and the carried step.
    pcr_status set_w(int sid, const double* w)
    {
        std::lock_guard<std::mutex> lk(mu_);
        auto it = streams_.find(sid);
        if (it == streams_.end()) return PCR_EINVAL;
        if (it->second.active) return PCR_EBUSY;
        for (int k = 0; k < it->second.K; ++k) it->second.w[k] = w[k];
        it->second.nhist = 0;
        it->second.mu_last = 0;
        it->second.move_last = -1;
        return PCR_OK;
    }
    int stream_K(int sid) const
    {
        std::lock_guard<std::mutex> lk(mu_);
        auto it = streams_.find(sid);
        return it == streams_.end() ? -1 : it->second.K;
    }

  private:
    void push_dropped(const Request& r, int K)
    {
        pcr_result res;
        std::memset(&res, 0, sizeof res);
        res.req_id = r.id;
        res.stream_id = r.sid;
        res.K = K;
        res.status = PCR_EBUSY;
        res.t_submit_s = r.t_submit;
        res.t_done_s = now_s();
        results_.push_back(res);
    }

    // Predicted warm start: the stream's last results extrapolated to the
    // request's submit time; kept at the last result unless the history's
    // times increase strictly and the prediction is finite.
    void predict(const StreamState& st, double t_next, double* w0) const
    {
        for (int i = 1; i < st.nhist; ++i)
            if (!(st.hist_t[i] > st.hist_t[i - 1])) return;
        double wh[3 * 8], wp[8];
        for (int i = 0; i < st.nhist; ++i)
            for (int k = 0; k < st.K; ++k) wh[i * st.K + k] = st.hist_w[i][k];
        extrapolate_w(wh, st.hist_t, st.nhist, st.K, t_next, o_.predict_order, wp);
        for (int k = 0; k < st.K; ++k)
            if (!std::isfinite(wp[k])) return;
        for (int k = 0; k < st.K; ++k) w0[k] = wp[k];
    }

    struct Fresh {
        int slot;
        Request req;
        double w0[8];
        double mu0;
        double move;
    };

    // Under the lock: free slots take the oldest queued requests of idle
    // streams; the warm start is fixed here from the stream's state.
    void dispatch(std::vector<Fresh>& fresh)
    {
        for (int s = 0; s < o_.slots; ++s) {
            if (slot_busy_[s]) continue;
            auto it = std::find_if(queue_.begin(), queue_.end(), [&](const Request& r) {
                auto q = streams_.find(r.sid);
                return q != streams_.end() && !q->second.active;
            });
            if (it == queue_.end()) break;
            StreamState& st = streams_[it->sid];
            Fresh f;
            f.slot = s;
            f.req = *it;
            for (int k = 0; k < 8; ++k) f.w0[k] = st.w[k];
            if (o_.predict_order > 0 && st.nhist >= 2) predict(st, it->t_submit, f.w0);
            f.mu0 = (o_.chain_step && st.mu_last > 0) ? st.mu_last : 0.0;
            f.move = o_.carry_move ? st.move_last : -1.0;
            st.active = true;
            st.queued--;
            slot_busy_[s] = 1;
            slot_sid_[s] = it->sid;
            slot_req_[s] = *it;
            slot_w0_[s] = std::vector<double>(f.w0, f.w0 + 8);
            slot_t_start_[s] = now_s();
            ++busy_;
            queue_.erase(it);
            fresh.push_back(f);
        }
    }

    // A slot's solve ended (res from the executor, or a failure to start).
    void complete(int s, pcr_result res)
    {
        std::lock_guard<std::mutex> lk(mu_);
        const Request& r = slot_req_[s];
        StreamState& st = streams_[slot_sid_[s]];
        res.req_id = r.id;
        res.stream_id = r.sid;
        res.K = st.K;
        res.t_submit_s = r.t_submit;
        res.t_start_s = slot_t_start_[s];
        res.t_done_s = now_s();
        for (int k = 0; k < 8; ++k) res.w0[k] = k < st.K ? slot_w0_[s][k] : 0.0;
        if (res.status == PCR_OK || res.status == PCR_ENOCONV) {
            double m2 = 0.0;
            for (int k = 0; k < st.K; ++k) {
                const double d = res.w[k] - slot_w0_[s][k];
                m2 += d * d;
            }
            for (int k = 0; k < st.K; ++k) st.w[k] = res.w[k];
            st.mu_last = res.mu;
            st.move_last = std::sqrt(m2);
            if (st.nhist == 3) {
                for (int i = 0; i < 2; ++i) {
                    st.hist_t[i] = st.hist_t[i + 1];
                    for (int k = 0; k < 8; ++k) st.hist_w[i][k] = st.hist_w[i + 1][k];
                }
                st.nhist = 2;
            }
            st.hist_t[st.nhist] = r.t_submit;
            for (int k = 0; k < 8; ++k) st.hist_w[st.nhist][k] = res.w[k];
            ++st.nhist;
        }
        st.active = false;
        slot_busy_[s] = 0;
        slot_sid_[s] = -1;
        --busy_;
        results_.push_back(res);
        cv_done_.notify_all();
        cv_work_.notify_all();
    }

    void run()
    {
        std::vector<Fresh> fresh;
        for (;;) {
            fresh.clear();
            {
                std::unique_lock<std::mutex> lk(mu_);
                if (busy_ == 0 && queue_.empty()) {
                    if (stopping_) break;
                    cv_work_.wait_for(lk, std::chrono::milliseconds(20));
                    continue;
                }
                dispatch(fresh);
            }
            for (const Fresh& f : fresh) {
                if (!ex_.start(f.slot, f.req, f.req.sid, f.w0, f.mu0, f.move)) {
                    pcr_result res;
                    std::memset(&res, 0, sizeof res);
                    if (ex_.advance(f.slot, &res) != 2) res.status = PCR_EDEVICE;
                    complete(f.slot, res);
                }
            }
            bool progressed = false;
            for (int s = 0; s < o_.slots; ++s) {
                {
                    std::lock_guard<std::mutex> lk(mu_);
                    if (!slot_busy_[s]) continue;
                }
                pcr_result res;
                std::memset(&res, 0, sizeof res);
                const int a = ex_.advance(s, &res);
                if (a == 0) continue;
                progressed = true;
                if (a == 2) complete(s, res);
            }
            if (!progressed) ex_.wait_any();
        }
    }

    Options o_;
    Exec& ex_;
    mutable std::mutex mu_;
    std::condition_variable cv_work_, cv_done_;
    std::map<int, StreamState> streams_;
    int next_sid_ = 0;
    std::deque<Request> queue_;
    int64_t next_req_ = 0;
    std::deque<pcr_result> results_;
    std::vector<int> slot_busy_, slot_sid_;
    std::vector<Request> slot_req_;
    std::vector<std::vector<double>> slot_w0_;
    std::vector<double> slot_t_start_;
    size_t stream_bytes_ = 0, max_scratch_ = 0;
    int busy_ = 0;
    bool stopping_ = false;
    std::thread worker_;
};

}  // namespace sched
}  // namespace pcr
