// CPU test of the serving scheduler (paper_1004_0014_amd/csrc/scheduler.h)
// with a stand-in executor: admission by footprint, one solve per stream in
// arrival order, slot reuse, stale-frame dropping, failure isolation, stream
// removal with a solve in flight, warm starts (last result, extrapolation in
// time) and the carried step size.  Built and run by test_sched_cpu.py;
// exits nonzero on the first failed check.
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <thread>
#include <vector>

#include "scheduler.h"

using pcr::sched::Core;
using pcr::sched::Options;
using pcr::sched::Request;

#define CHECK(c)                                                              \
    do {                                                                      \
        if (!(c)) {                                                           \
            std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__,       \
                         __LINE__, #c);                                       \
            std::exit(1);                                                     \
        }                                                                     \
    } while (0)

// What a request's "projection" holds for the stand-in solver: the result
// it converges to, how many advances it takes, and how it fails.
struct Frame {
    double w[8];
    double mu = 0.25;
    int steps = 3;
    int fail = 0;   // 1: fails to start; 2: fails while running
};

struct StartCall {
    int slot, sid;
    int64_t req;
    double w0[8];
    double mu0;
    double move;
};

struct FakeExec {
    struct S {
        bool on = false, err = false;
        int left = 0, sid = -1;
        const Frame* f = nullptr;
        double mu0 = 0;
    };
    std::vector<S> slots;
    std::mutex m;
    std::vector<StartCall> starts;
    std::vector<int> forgotten;
    std::atomic<bool> gate{true};   // advances happen only while open
    std::atomic<int> in_flight{0}, max_in_flight{0};
    bool overlap_seen = false;      // two slots ran one stream at once

    explicit FakeExec(int n) : slots(n) {}

    bool start(int slot, const Request& r, int sid, const double* w0, double mu0, double move)
    {
        std::lock_guard<std::mutex> lk(m);
        S& s = slots[slot];
        CHECK(!s.on);
        for (const S& o : slots)
            if (o.on && o.sid == sid) overlap_seen = true;
        StartCall c{slot, sid, r.id, {0}, mu0, move};
        for (int k = 0; k < 8; ++k) c.w0[k] = w0[k];
        starts.push_back(c);
        s.f = static_cast<const Frame*>(r.y);
        s.sid = sid;
        s.mu0 = mu0;
        s.left = s.f->steps;
        if (s.f->fail == 1) {
            s.err = true;
            return false;
        }
        s.on = true;
        const int n = ++in_flight;
        int mx = max_in_flight.load();
        while (n > mx && !max_in_flight.compare_exchange_weak(mx, n)) {
        }
        return true;
    }
    int advance(int slot, pcr_result* res)
    {
        std::lock_guard<std::mutex> lk(m);
        S& s = slots[slot];
        if (s.err) {
            s.err = false;
            res->status = PCR_EINVAL;
            return 2;
        }
        if (!s.on || !gate.load()) return 0;
        if (--s.left > 0) return 1;
        s.on = false;
        --in_flight;
        if (s.f->fail == 2) {
            res->status = PCR_EDEVICE;
            return 2;
        }
        res->status = PCR_OK;
        res->iterations = s.f->steps;
        for (int k = 0; k < 8; ++k) res->w[k] = s.f->w[k];
        res->mu0 = s.mu0;
        res->mu = s.f->mu;
        return 2;
    }
    void wait_any() { std::this_thread::sleep_for(std::chrono::microseconds(200)); }
    void forget_stream(int sid)
    {
        std::lock_guard<std::mutex> lk(m);
        for (const S& o : slots) CHECK(!(o.on && o.sid == sid));
        forgotten.push_back(sid);
    }
    std::vector<StartCall> calls()
    {
        std::lock_guard<std::mutex> lk(m);
        return starts;
    }
};

struct Server {
    FakeExec ex;
    Core<FakeExec> core;
    Server(const Options& o) : ex(o.slots), core(o, ex) { core.start_worker_on(nullptr); }
};

Options opts(int slots, bool drop_stale = false, int order = 0, bool chain = false)
{
    Options o;
    o.budget = 1000;
    o.slots = slots;
    o.drop_stale = drop_stale;
    o.predict_order = order;
    o.chain_step = chain;
    return o;
}

int add(Core<FakeExec>& c, int K, const double* w0, size_t bytes = 10, size_t scratch = 10)
{
    const int sid = c.reserve_stream(K, bytes, scratch, w0);
    CHECK(sid >= 0);
    c.commit_stream(sid);
    return sid;
}

std::vector<pcr_result> collect(Core<FakeExec>& c, int n)
{
    std::vector<pcr_result> out(n);
    int got = 0;
    for (int tries = 0; got < n && tries < 2000; ++tries) got += c.poll(out.data() + got, n - got, 5);
    CHECK(got == n);
    return out;
}

const pcr_result& by_req(const std::vector<pcr_result>& v, int64_t id)
{
    for (const pcr_result& r : v)
        if (r.req_id == id) return r;
    std::fprintf(stderr, "request %lld has no result\n", (long long)id);
    std::exit(1);
}

pcr_geom geom0()
{
    pcr_geom g{};
    g.angle_rad = 0.3;
    return g;
}

void test_extrapolate()
{
    // order 2 through three samples of a quadratic reproduces it exactly;
    // order 1 uses the last two points; order 0 (or one point) the last value
    const double t[3] = {0.5, 1.0, 2.5};
    double wh[3 * 2];
    auto q = [](double x, int k) { return k == 0 ? 1 + 2 * x - 3 * x * x : -0.5 * x * x + 4; };
    for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 2; ++k) wh[i * 2 + k] = q(t[i], k);
    double w[2];
    pcr::sched::extrapolate_w(wh, t, 3, 2, 3.25, 2, w);
    for (int k = 0; k < 2; ++k) CHECK(std::fabs(w[k] - q(3.25, k)) < 1e-12 * (1 + std::fabs(q(3.25, k))));
    pcr::sched::extrapolate_w(wh, t, 3, 2, 3.25, 1, w);
    for (int k = 0; k < 2; ++k) {
        const double lin = wh[2 + k] + (wh[4 + k] - wh[2 + k]) * (3.25 - 1.0) / (2.5 - 1.0);
        CHECK(std::fabs(w[k] - lin) < 1e-12 * (1 + std::fabs(lin)));
    }
    pcr::sched::extrapolate_w(wh, t, 3, 2, 3.25, 0, w);
    for (int k = 0; k < 2; ++k) CHECK(w[k] == wh[4 + k]);
    pcr::sched::extrapolate_w(wh, t, 1, 2, 3.25, 2, w);
    for (int k = 0; k < 2; ++k) CHECK(w[k] == wh[k]);
}

void test_admission()
{
    FakeExec ex(4);
    Core<FakeExec> c(opts(4), ex);   // budget 1000, 4 slots
    const double w0[1] = {0};
    // footprint: stream bytes + slots x the largest per-slot scratch
    CHECK(c.footprint(100, 50) == 100 + 4 * 50);
    const int a = c.reserve_stream(1, 100, 50, w0);
    CHECK(a >= 0);
    CHECK(c.stream_bytes() == 100);
    CHECK(c.footprint(0, 0) == 100 + 4 * 50);
    // a larger scratch raises every slot's share
    CHECK(c.reserve_stream(1, 100, 201, w0) == -1);   // 200 + 4 x 201 > 1000
    CHECK(c.stream_bytes() == 100);
    const int b = c.reserve_stream(1, 600, 50, w0);  // 700 + 200 = 900
    CHECK(b >= 0 && b != a);
    CHECK(c.reserve_stream(1, 101, 50, w0) == -1);   // 1001
    // an uncommitted stream takes no requests
    Frame f;
    int64_t id;
    CHECK(c.submit(b, &f, geom0(), &id) == PCR_EINVAL);
    c.unreserve_stream(b);
    CHECK(c.stream_bytes() == 100);
    CHECK(c.reserve_stream(1, 101, 50, w0) >= 0);
    CHECK(c.stream_K(a) == 1 && c.stream_K(12345) == -1);
}

void test_order_and_warm_start()
{
    // two slots; stream A gets three frames, stream B one; A's solves run one
    // at a time in arrival order, each starting from the previous result
    Server s(opts(2));
    const double wa[2] = {0.5, -0.5}, wb[2] = {3, 4};
    const int A = add(s.core, 2, wa), B = add(s.core, 2, wb);
    s.ex.gate = false;
    Frame fa[3], fb;
    for (int i = 0; i < 3; ++i) {
        fa[i].w[0] = i + 1;
        fa[i].w[1] = -(i + 1);
        fa[i].steps = 2 + i;
    }
    fb.w[0] = 7;
    fb.w[1] = 8;
    int64_t ra[3], rb;
    for (int i = 0; i < 3; ++i) CHECK(s.core.submit(A, &fa[i], geom0(), &ra[i]) == PCR_OK);
    CHECK(s.core.submit(B, &fb, geom0(), &rb) == PCR_OK);
    // with the gate closed both slots fill: A's first frame and B's frame
    for (int t = 0; t < 1000 && s.ex.calls().size() < 2; ++t) std::this_thread::sleep_for(std::chrono::milliseconds(1));
    CHECK(s.ex.calls().size() == 2);
    CHECK(s.core.drain(20) == false);   // solves held in flight
    s.ex.gate = true;
    CHECK(s.core.drain(5000));
    auto res = collect(s.core, 4);
    auto calls = s.ex.calls();
    CHECK(calls.size() == 4);
    CHECK(!s.ex.overlap_seen);
    CHECK(s.ex.max_in_flight.load() <= 2);
    // A's requests started in submit order
    std::vector<int64_t> a_order;
    for (const StartCall& c : calls)
        if (c.sid == A) a_order.push_back(c.req);
    CHECK(a_order.size() == 3 && a_order[0] == ra[0] && a_order[1] == ra[1] && a_order[2] == ra[2]);
    // warm starts: the stream's initial w, then each previous result
    for (int i = 0; i < 3; ++i) {
        const pcr_result& r = by_req(res, ra[i]);
        CHECK(r.status == PCR_OK && r.stream_id == A && r.K == 2);
        CHECK(r.w[0] == fa[i].w[0] && r.w[1] == fa[i].w[1]);
        const double* want = i == 0 ? wa : fa[i - 1].w;
        CHECK(r.w0[0] == want[0] && r.w0[1] == want[1]);
        CHECK(r.t_submit_s <= r.t_start_s && r.t_start_s <= r.t_done_s);
        CHECK(r.mu0 == 0.0);   // no carried step without chain_step
    }
    const pcr_result& r = by_req(res, rb);
    CHECK(r.w0[0] == 3 && r.w0[1] == 4 && r.w[0] == 7);
    double w[2];
    CHECK(s.core.get_w(A, w) == PCR_OK && w[0] == 3 && w[1] == -3);
}

void test_slot_reuse()
{
    // 12 single-frame streams through 3 slots
    Server s(opts(3));
    const double z[1] = {0};
    std::vector<int> ids;
    std::vector<Frame> f(12);
    std::vector<int64_t> rq(12);
    for (int i = 0; i < 12; ++i) {
        ids.push_back(add(s.core, 1, z));
        f[i].w[0] = 10 + i;
        f[i].steps = 1 + i % 4;
    }
    for (int i = 0; i < 12; ++i) CHECK(s.core.submit(ids[i], &f[i], geom0(), &rq[i]) == PCR_OK);
    CHECK(s.core.drain(5000));
    auto res = collect(s.core, 12);
    CHECK(s.ex.max_in_flight.load() <= 3);
    for (int i = 0; i < 12; ++i) {
        const pcr_result& r = by_req(res, rq[i]);
        CHECK(r.status == PCR_OK && r.stream_id == ids[i] && r.w[0] == 10 + i);
    }
    for (const StartCall& c : s.ex.calls()) CHECK(c.slot >= 0 && c.slot < 3);
}

void test_drop_stale()
{
    // frame 1 in flight, frame 2 queued; frame 3 replaces frame 2, which is
    // answered PCR_EBUSY; frame 3 then starts from frame 1's result
    Server s(opts(1, true));
    const double z[1] = {0};
    const int A = add(s.core, 1, z);
    s.ex.gate = false;
    Frame f[3];
    for (int i = 0; i < 3; ++i) f[i].w[0] = i + 1;
    int64_t r[3];
    CHECK(s.core.submit(A, &f[0], geom0(), &r[0]) == PCR_OK);
    for (int t = 0; t < 1000 && s.ex.calls().empty(); ++t) std::this_thread::sleep_for(std::chrono::milliseconds(1));
    CHECK(s.ex.calls().size() == 1);
    CHECK(s.core.submit(A, &f[1], geom0(), &r[1]) == PCR_OK);
    CHECK(s.core.submit(A, &f[2], geom0(), &r[2]) == PCR_OK);
    pcr_result d;
    CHECK(s.core.poll(&d, 1, 1000) == 1);   // the drop is answered at once
    CHECK(d.req_id == r[1] && d.status == PCR_EBUSY && d.stream_id == A);
    s.ex.gate = true;
    CHECK(s.core.drain(5000));
    auto res = collect(s.core, 2);
    CHECK(by_req(res, r[0]).w[0] == 1);
    CHECK(by_req(res, r[2]).w0[0] == 1 && by_req(res, r[2]).w[0] == 3);
    CHECK(s.ex.calls().size() == 2);
}

void test_failures()
{
    // a solve that fails to start and one that fails while running are
    // reported with their status; the stream's warm start stays the last
    // good result and other streams are unaffected
    Server s(opts(2));
    const double z[1] = {0};
    const int A = add(s.core, 1, z), B = add(s.core, 1, z);
    Frame ok1, bad1, bad2, ok2, fb;
    ok1.w[0] = 5;
    bad1.fail = 1;
    bad1.w[0] = 99;
    bad2.fail = 2;
    bad2.w[0] = 98;
    ok2.w[0] = 6;
    fb.w[0] = 1;
    int64_t r[4], rb;
    CHECK(s.core.submit(A, &ok1, geom0(), &r[0]) == PCR_OK);
    CHECK(s.core.submit(A, &bad1, geom0(), &r[1]) == PCR_OK);
    CHECK(s.core.submit(A, &bad2, geom0(), &r[2]) == PCR_OK);
    CHECK(s.core.submit(A, &ok2, geom0(), &r[3]) == PCR_OK);
    CHECK(s.core.submit(B, &fb, geom0(), &rb) == PCR_OK);
    CHECK(s.core.drain(5000));
    auto res = collect(s.core, 5);
    CHECK(by_req(res, r[0]).status == PCR_OK);
    CHECK(by_req(res, r[1]).status == PCR_EINVAL);
    CHECK(by_req(res, r[2]).status == PCR_EDEVICE);
    CHECK(by_req(res, r[3]).status == PCR_OK);
    CHECK(by_req(res, r[3]).w0[0] == 5);   // failures did not move the warm start
    CHECK(by_req(res, rb).status == PCR_OK && by_req(res, rb).w[0] == 1);
    double w;
    CHECK(s.core.get_w(A, &w) == PCR_OK && w == 6);
}

void test_remove()
{
    // removal waits for the solve in flight, answers the queued request
    // PCR_EBUSY, releases the stream's bytes and tells the executor after
    // the solve has ended
    Server s(opts(1));
    const double z[1] = {0};
    const int A = add(s.core, 1, z, 100, 10), B = add(s.core, 1, z, 50, 10);
    CHECK(s.core.stream_bytes() == 150);
    s.ex.gate = false;
    Frame f[2];
    int64_t r[2];
    CHECK(s.core.submit(A, &f[0], geom0(), &r[0]) == PCR_OK);
    for (int t = 0; t < 1000 && s.ex.calls().empty(); ++t) std::this_thread::sleep_for(std::chrono::milliseconds(1));
    CHECK(s.core.submit(A, &f[1], geom0(), &r[1]) == PCR_OK);
    std::atomic<bool> removed{false};
    std::thread t([&] {
        CHECK(s.core.remove_stream(A) == PCR_OK);
        removed = true;
    });
    std::this_thread::sleep_for(std::chrono::milliseconds(50));
    CHECK(!removed.load());   // the in-flight solve holds it
    {
        std::lock_guard<std::mutex> lk(s.ex.m);
        CHECK(s.ex.forgotten.empty());
    }
    s.ex.gate = true;
    t.join();
    CHECK(removed.load());
    auto res = collect(s.core, 2);
    CHECK(by_req(res, r[0]).status == PCR_OK);
    CHECK(by_req(res, r[1]).status == PCR_EBUSY);
    {
        std::lock_guard<std::mutex> lk(s.ex.m);
        CHECK(s.ex.forgotten.size() == 1 && s.ex.forgotten[0] == A);
    }
    CHECK(s.core.stream_bytes() == 50);
    int64_t id;
    CHECK(s.core.submit(A, &f[0], geom0(), &id) == PCR_EINVAL);
    CHECK(s.core.remove_stream(A) == PCR_EINVAL);
    CHECK(s.core.get_w(A, nullptr) == PCR_EINVAL);
    CHECK(s.core.submit(B, &f[0], geom0(), &id) == PCR_OK);
    CHECK(s.core.drain(5000));
}

void test_predict_and_chain()
{
    // order 1: the third solve starts from the line through the first two
    // results at their submit times; chain_step: each solve's first trial
    // step is the step the previous one ended with; set_w forgets both
    Server s(opts(1, false, 1, true));
    const double z[2] = {0, 0};
    const int A = add(s.core, 2, z);
    Frame f[4];
    for (int i = 0; i < 4; ++i) {
        f[i].w[0] = 1.0 + 2.0 * i;
        f[i].w[1] = -3.0 * i;
        f[i].mu = 0.5 / (i + 1);
    }
    int64_t r[4];
    for (int i = 0; i < 3; ++i) {
        CHECK(s.core.submit(A, &f[i], geom0(), &r[i]) == PCR_OK);
        CHECK(s.core.drain(5000));
        std::this_thread::sleep_for(std::chrono::milliseconds(2));
    }
    auto res = collect(s.core, 3);
    const pcr_result &p0 = by_req(res, r[0]), &p1 = by_req(res, r[1]), &p2 = by_req(res, r[2]);
    // one point of history: the last result
    CHECK(p1.w0[0] == f[0].w[0] && p1.w0[1] == f[0].w[1]);
    for (int k = 0; k < 2; ++k) {
        const double lin = p1.w[k] + (p1.w[k] - p0.w[k]) * (p2.t_submit_s - p1.t_submit_s) /
                                         (p1.t_submit_s - p0.t_submit_s);
        CHECK(std::fabs(p2.w0[k] - lin) <= 1e-9 * (1 + std::fabs(lin)));
    }
    CHECK(p0.mu0 == 0.0 && p1.mu0 == f[0].mu && p2.mu0 == f[1].mu);
    const double wn[2] = {9, 9};
    CHECK(s.core.set_w(A, wn) == PCR_OK);
    CHECK(s.core.submit(A, &f[3], geom0(), &r[3]) == PCR_OK);
    CHECK(s.core.drain(5000));
    auto r3 = collect(s.core, 1);
    CHECK(r3[0].w0[0] == 9 && r3[0].w0[1] == 9 && r3[0].mu0 == 0.0);
}

void test_carry_move()
{
    // carry_move: each solve starts with the distance the stream's previous
    // solve moved w (none before the first, and none after set_w)
    Options o = opts(1);
    o.carry_move = true;
    Server s(o);
    const double z[2] = {0, 0};
    const int A = add(s.core, 2, z);
    Frame f[4];
    for (int i = 0; i < 4; ++i) {
        f[i].w[0] = 3.0 * i + 1.0;
        f[i].w[1] = 4.0 * i * i;
    }
    int64_t r[4];
    for (int i = 0; i < 3; ++i) {
        CHECK(s.core.submit(A, &f[i], geom0(), &r[i]) == PCR_OK);
        CHECK(s.core.drain(5000));
    }
    auto c = s.ex.calls();
    CHECK(c.size() == 3);
    CHECK(c[0].move < 0);
    // solve 0 moved w from (0, 0) to (1, 0); solve 1 from (1, 0) to (4, 4)
    CHECK(std::fabs(c[1].move - 1.0) <= 1e-12);
    CHECK(std::fabs(c[2].move - 5.0) <= 1e-12);
    for (const auto& k : c) CHECK(k.mu0 == 0.0);
    collect(s.core, 3);
    const double wn[2] = {9, 9};
    CHECK(s.core.set_w(A, wn) == PCR_OK);
    CHECK(s.core.submit(A, &f[3], geom0(), &r[3]) == PCR_OK);
    CHECK(s.core.drain(5000));
    CHECK(s.ex.calls().back().move < 0);
}

void test_set_w_busy_and_stop()
{
    Server s(opts(1));
    const double z[1] = {0};
    const int A = add(s.core, 1, z);
    s.ex.gate = false;
    Frame f[3];
    int64_t r;
    for (int i = 0; i < 3; ++i) CHECK(s.core.submit(A, &f[i], geom0(), &r) == PCR_OK);
    for (int t = 0; t < 1000 && s.ex.calls().empty(); ++t) std::this_thread::sleep_for(std::chrono::milliseconds(1));
    const double w[1] = {1};
    CHECK(s.core.set_w(A, w) == PCR_EBUSY);
    s.ex.gate = true;
    // stop with requests queued: the solve in flight ends, the queue is dropped
    s.core.stop();
    CHECK(s.ex.in_flight.load() == 0);
    CHECK(s.core.submit(A, &f[0], geom0(), &r) == PCR_EINVAL);
}

int main()
{
    test_extrapolate();
    test_carry_move();
    test_admission();
    test_order_and_warm_start();
    test_slot_reuse();
    test_drop_stale();
    test_failures();
    test_remove();
    test_predict_and_chain();
    test_set_w_busy_and_stop();
    std::printf("scheduler: all checks passed\n");
    return 0;
}
