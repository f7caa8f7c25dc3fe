// Host-only checks of the serving core (paper_2104_03186_amd/csrc/lqt_serve.hpp):
// the pool's range allocator and the admission of requests into batches,
// driven by a fake device.  Built by tests/test_serve_host.py with the
// address and undefined-behaviour sanitizers; exits non-zero on the first
// failed check.
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include <set>
#include <vector>

#include "lqt_serve.hpp"

static int g_checks = 0;
#define CHECK(cond)                                                              \
    do {                                                                         \
        ++g_checks;                                                              \
        if (!(cond)) {                                                           \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
            std::exit(1);                                                        \
        }                                                                        \
    } while (0)

// A fake device: a batch's workspace is the sum of its requests' bytes plus a
// fixed table; batches finish when the test says so.
struct FakeOps {
    std::map<size_t, size_t> bytes;      // handle -> bytes alone (without the table)
    std::map<size_t, int> final_status;  // handle -> status reported by the "device"
    std::set<size_t> fail_launch;        // handles whose batch launch fails
    std::set<int> fail_query;            // slots whose completion query fails
    struct Run {
        bool busy = false, done = false;
        std::vector<size_t> req;
        size_t off = 0, len = 0;
    };
    std::vector<Run> run;
    std::vector<std::vector<size_t>> launched;  // every batch, in launch order
    static constexpr size_t kTable = 64;

    struct Acc {
        const FakeOps* ops;
        size_t sum = 0;
        int count = 0;
        void add(size_t h) {
            sum += ops->bytes.at(h);
            ++count;
        }
        size_t total() const { return sum + (count ? kTable : 0); }
    };
    Acc acc() { return Acc{this}; }
    int launch(int slot, const size_t* req, size_t count, size_t off, size_t len) {
        CHECK(slot >= 0 && slot < (int)run.size());
        CHECK(!run[slot].busy);
        std::vector<size_t> r(req, req + count);
        for (size_t h : r)
            if (fail_launch.count(h)) return LQT_EHIP;
        run[slot] = Run{true, false, r, off, len};
        launched.push_back(r);
        return LQT_OK;
    }
    int query(int slot) {
        if (fail_query.count(slot)) return -1;
        if (!run[slot].done) return 0;
        statuses = run[slot].req;  // what status() reports until the next launch on any slot
        run[slot] = Run{};         // the core retires the batch: the slot is free again
        return 1;
    }
    std::vector<size_t> statuses;  // requests of the batch being retired
    int status(int, size_t i) {
        CHECK(i < statuses.size());
        return final_status.count(statuses[i]) ? final_status[statuses[i]] : 0;
    }
    void drain(int slot) { run[slot] = Run{}; }
    void finish_all() {
        for (Run& r : run)
            if (r.busy) r.done = true;
    }
    void clear_done() {
        for (Run& r : run)
            if (r.done) r = Run{};
    }
};

using Core = lqt::ServeCore<FakeOps>;

static void test_range_pool() {
    lqt::RangePool p;
    p.reset(1000);
    size_t a, b, c;
    CHECK(p.take(100, a) && a == 0);
    CHECK(p.take(200, b) && b == 100);
    CHECK(p.take(300, c) && c == 300);
    CHECK(p.largest() == 400 && p.in_use() == 600);
    p.give(b, 200);
    CHECK(p.largest() == 400);
    size_t d;
    CHECK(p.take(150, d) && d == 100);  // first fit
    p.give(a, 100);
    p.give(d, 150);
    p.give(c, 300);
    CHECK(p.in_use() == 0 && p.free_ranges().size() == 1 && p.largest() == 1000);  // coalesced
    CHECK(!p.take(1001, a));
    // random sequences against a byte map
    std::mt19937_64 rng(7);
    p.reset(4096);
    std::vector<char> used(4096, 0);
    std::vector<std::pair<size_t, size_t>> held;
    for (int it = 0; it < 20000; ++it) {
        if (held.empty() || (rng() % 3)) {
            const size_t len = 1 + rng() % 300;
            size_t off;
            if (p.take(len, off)) {
                CHECK(off + len <= 4096);
                for (size_t i = off; i < off + len; ++i) {
                    CHECK(!used[i]);
                    used[i] = 1;
                }
                held.push_back({off, len});
            } else {
                CHECK(p.largest() < len);
            }
        } else {
            const size_t k = rng() % held.size();
            for (size_t i = held[k].first; i < held[k].first + held[k].second; ++i) used[i] = 0;
            p.give(held[k].first, held[k].second);
            held.erase(held.begin() + (long)k);
        }
        size_t inuse = 0;
        for (auto& h : held) inuse += h.second;
        CHECK(p.in_use() == inuse);
    }
    for (auto& h : held) p.give(h.first, h.second);
    CHECK(p.in_use() == 0 && p.free_ranges().size() == 1);
}

static Core make_core(FakeOps& ops, size_t pool, int max_batch = 8, int max_inflight = 1000) {
    Core c;
    c.init(pool, {0, 0, 1, 1}, max_batch, max_inflight);
    ops.run.assign(4, FakeOps::Run{});
    return c;
}

static void test_fifo_and_completion() {
    FakeOps ops;
    Core core = make_core(ops, 1 << 20, 4);
    for (size_t h = 1; h <= 20; ++h) {
        ops.bytes[h] = 100;
        CHECK(core.submit(h, (int)(h % 2), 100 + FakeOps::kTable, h) == LQT_OK);
    }
    std::vector<size_t> order[2];
    for (int round = 0; round < 20 && !core.idle(); ++round) {
        CHECK(core.pump(ops) == LQT_OK);
        ops.finish_all();
        CHECK(core.pump(ops) == LQT_OK);
        ops.clear_done();
    }
    CHECK(core.idle());
    for (auto& b : ops.launched) {
        CHECK(!b.empty() && b.size() <= 4);
        for (size_t h : b) order[h % 2].push_back(h);
    }
    for (int l = 0; l < 2; ++l) {  // each lane launched in FIFO order, each request once
        CHECK(order[l].size() == 10);
        for (size_t i = 1; i < order[l].size(); ++i) CHECK(order[l][i] > order[l][i - 1]);
    }
    for (size_t h = 1; h <= 20; ++h) {
        int st = -1;
        CHECK(core.poll(h, st) && st == LQT_OK);
        CHECK(!core.known(h));
    }
    int st = 0;
    CHECK(core.poll(999, st) && st == LQT_EINVAL);
    CHECK(core.pool().in_use() == 0);
}

static void test_memory_admission_and_codes() {
    FakeOps ops;
    Core core = make_core(ops, 1000, 8, 5);
    ops.bytes[1] = 600;
    ops.bytes[2] = 600;
    ops.bytes[3] = 100;
    CHECK(core.submit(1, 0, 664, 1) == LQT_OK);
    CHECK(core.submit(2, 0, 664, 2) == LQT_OK);
    CHECK(core.submit(3, 0, 164, 3) == LQT_OK);
    CHECK(core.submit(9, 0, 2000, 9) == LQT_ENOMEM);
    CHECK(core.pump(ops) == LQT_OK);
    CHECK(ops.launched.size() == 1 && ops.launched[0] == std::vector<size_t>({1}));  // 2 waits: no overtaking by 3
    CHECK(core.pending(2) && core.pending(3));
    ops.bytes[4] = 10;
    ops.bytes[5] = 10;
    CHECK(core.submit(4, 0, 74, 4) == LQT_OK);
    CHECK(core.submit(5, 0, 74, 5) == LQT_OK);
    CHECK(core.submit(6, 0, 74, 6) == LQT_EBUSY);  // five queued or running
    ops.finish_all();
    CHECK(core.pump(ops) == LQT_OK);  // 1 retires, 2..5 fit now
    int st = -1;
    CHECK(core.poll(1, st) && st == LQT_OK);
    CHECK(ops.launched.size() == 2 && ops.launched[1] == std::vector<size_t>({2, 3, 4, 5}));
    ops.finish_all();
    CHECK(core.pump(ops) == LQT_OK);
    ops.clear_done();
    CHECK(core.idle() && core.pool().in_use() == 0);
}

static void test_lane_isolation_and_no_starvation() {
    // a long request that needs most of the pool must not be starved by a
    // stream of short ones; short requests are never batched with long ones
    FakeOps ops;
    Core core = make_core(ops, 10000, 8);
    size_t h = 1;
    ops.bytes[h] = 100;
    CHECK(core.submit(h, 1, 164, h) == LQT_OK);  // a long request runs
    ++h;
    CHECK(core.pump(ops) == LQT_OK);
    const size_t big = h++;
    ops.bytes[big] = 9000;
    CHECK(core.submit(big, 1, 9064, big) == LQT_OK);  // the next long one needs almost everything
    bool big_launched = false;
    for (int round = 0; round < 200 && !big_launched; ++round) {
        for (int k = 0; k < 3; ++k, ++h) {  // steady short traffic
            ops.bytes[h] = 500;
            CHECK(core.submit(h, 0, 564, h) == LQT_OK);
        }
        CHECK(core.pump(ops) == LQT_OK);
        for (auto& b : ops.launched)
            for (size_t x : b) big_launched = big_launched || x == big;
        ops.finish_all();
        CHECK(core.pump(ops) == LQT_OK);
        ops.clear_done();
    }
    CHECK(big_launched);
    for (auto& b : ops.launched) {
        bool has_long = false, has_short = false;
        for (size_t x : b) (x == 1 || x == big ? has_long : has_short) = true;
        CHECK(!(has_long && has_short));
    }
}

static void test_failures() {
    FakeOps ops;
    Core core = make_core(ops, 100000, 3);
    for (size_t h = 1; h <= 6; ++h) {
        ops.bytes[h] = 50;
        CHECK(core.submit(h, 0, 114, h) == LQT_OK);
    }
    ops.fail_launch.insert(2);  // the batch {1, 2, 3} fails to launch
    ops.final_status[5] = LQT_ENOTPD;
    CHECK(core.pump(ops) == LQT_EHIP);
    int st = -1;
    for (size_t h = 1; h <= 3; ++h) CHECK(core.poll(h, st) && st == LQT_EHIP);
    CHECK(core.pool().in_use() > 0);  // {4, 5, 6} launched on the other short slot
    ops.finish_all();
    CHECK(core.pump(ops) == LQT_OK);
    ops.clear_done();
    CHECK(core.poll(4, st) && st == LQT_OK);
    CHECK(core.poll(5, st) && st == LQT_ENOTPD);  // per-request status from the device
    CHECK(core.poll(6, st) && st == LQT_OK);
    CHECK(core.pool().in_use() == 0);
    // a batch whose completion query fails: its requests fail, its range returns
    ops.bytes[7] = 50;
    CHECK(core.submit(7, 1, 114, 7) == LQT_OK);
    CHECK(core.pump(ops) == LQT_OK);
    ops.fail_query.insert(2);
    CHECK(core.pump(ops) == LQT_EHIP);
    CHECK(core.poll(7, st) && st == LQT_EHIP);
    CHECK(core.pool().in_use() == 0 && core.idle());
}

static void test_random_stress() {
    std::mt19937_64 rng(11);
    FakeOps ops;
    Core core = make_core(ops, 50000, 16, 200);
    std::map<uint64_t, bool> outstanding;
    uint64_t next = 1;
    size_t completed = 0;
    for (int it = 0; it < 20000; ++it) {
        const int act = (int)(rng() % 4);
        if (act < 2) {
            const size_t b = 1 + rng() % 8000;
            ops.bytes[next] = b;
            const int code = core.submit(next, (int)(rng() % 2), b + FakeOps::kTable, next);
            if (code == LQT_OK) outstanding[next] = true;
            else CHECK(code == LQT_EBUSY);
            ++next;
        } else if (act == 2) {
            for (auto& r : ops.run)
                if (r.busy && (rng() % 2)) r.done = true;
        }
        CHECK(core.pump(ops) == LQT_OK);
        ops.clear_done();
        size_t busy_len = 0;
        for (auto& r : ops.run)
            if (r.busy) busy_len += r.len;
        CHECK(core.pool().in_use() == busy_len);
        for (auto it2 = outstanding.begin(); it2 != outstanding.end();) {
            int st = -1;
            if (core.poll(it2->first, st)) {
                CHECK(st == LQT_OK);
                ++completed;
                it2 = outstanding.erase(it2);
            } else {
                ++it2;
            }
        }
    }
    for (int round = 0; round < 1000 && !outstanding.empty(); ++round) {
        ops.finish_all();
        CHECK(core.pump(ops) == LQT_OK);
        ops.clear_done();
        for (auto it2 = outstanding.begin(); it2 != outstanding.end();) {
            int st = -1;
            if (core.poll(it2->first, st)) {
                ++completed;
                it2 = outstanding.erase(it2);
            } else {
                ++it2;
            }
        }
    }
    CHECK(outstanding.empty() && core.idle() && core.pool().in_use() == 0);
    CHECK(completed > 1000);
}

int main() {
    test_range_pool();
    test_fifo_and_completion();
    test_memory_admission_and_codes();
    test_lane_isolation_and_no_starvation();
    test_failures();
    test_random_stress();
    std::printf("serve host checks passed: %d\n", g_checks);
    return 0;
}
