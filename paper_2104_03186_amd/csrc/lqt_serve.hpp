// Host logic of the continuous-batching serving interface, free of HIP: the
// range allocator of the device pool and the admission of queued requests
// into batches on the serving streams ("slots").  The runtime supplies the
// device side through an operations object; the same logic is built and
// checked on the host alone (under the address and undefined-behaviour
// sanitizers) with a fake device.
//
// Requests wait in one FIFO per lane; lane 0 takes short solves, lane 1 long
// ones, and every slot belongs to one lane, so a short request never waits
// for a long one to finish in its batch.  Whenever a slot is idle, the longest
// prefix of its lane's queue whose workspace fits one free range of the pool
// (at most max_batch requests) becomes a batch on that slot.  Nothing
// overtakes a lane's head; a head that waits for memory is protected: another
// lane launches only batches that leave a free range the waiting head fits.
// Running batches always finish and return their ranges, so every head is
// eventually launched.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <algorithm>
#include <deque>
#include <map>
#include <unordered_map>
#include <vector>

#include "../../include/lqt.h"

namespace lqt {

// First-fit allocator of ranges of [0, size) with a coalescing free list.
class RangePool {
public:
    void reset(size_t size) {
        free_.clear();
        size_ = size;
        in_use_ = 0;
        if (size) free_[0] = size;
    }
    bool take(size_t len, size_t& off) { return take_from(free_, len, off) && (in_use_ += len, true); }
    void give(size_t off, size_t len) {
        in_use_ -= len;
        give_to(free_, off, len);
    }
    size_t largest() const { return largest_of(free_); }
    // largest free range left if `len` were taken now
    size_t largest_after(size_t len) const {
        std::map<size_t, size_t> f = free_;
        size_t off = 0;
        if (!take_from(f, len, off)) return 0;
        return largest_of(f);
    }
    size_t size() const { return size_; }
    size_t in_use() const { return in_use_; }
    const std::map<size_t, size_t>& free_ranges() const { return free_; }

private:
    static bool take_from(std::map<size_t, size_t>& f, size_t len, size_t& off) {
        if (len == 0) len = 1;
        for (auto it = f.begin(); it != f.end(); ++it) {
            if (it->second >= len) {
                off = it->first;
                const size_t rest = it->second - len;
                f.erase(it);
                if (rest) f[off + len] = rest;
                return true;
            }
        }
        return false;
    }
    static void give_to(std::map<size_t, size_t>& f, size_t off, size_t len) {
        if (len == 0) len = 1;
        auto it = f.emplace(off, len).first;
        auto nx = std::next(it);
        if (nx != f.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            f.erase(nx);
        }
        if (it != f.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                f.erase(it);
            }
        }
    }
    static size_t largest_of(const std::map<size_t, size_t>& f) {
        size_t b = 0;
        for (auto& kv : f) b = std::max(b, kv.second);
        return b;
    }
    std::map<size_t, size_t> free_;
    size_t size_ = 0, in_use_ = 0;
};

struct ServeCounters {
    int64_t submitted = 0, completed = 0, batches = 0;
    int32_t running_batches = 0, max_running_batches = 0, max_batch = 0;
    size_t pool_peak = 0;
};

// Ops (the device side) provides:
//   Ops::Acc acc()                                        an empty batch-size accumulator:
//                                                         acc.add(handle), acc.total() (copyable)
//   int    launch(int slot, const size_t* req, size_t count, size_t off, size_t len)
//                                                         enqueue; lqt_status
//   int    query(int slot)                                1 done, 0 running, < 0 failed
//   int    status(int slot, size_t i)                     final status of the slot's i-th request
//   void   drain(int slot)                                wait for everything enqueued on the slot
// where a request is identified by the handle given to submit.
template <class Ops>
class ServeCore {
public:
    static constexpr int kLanes = 2;

    // slot_lanes[s]: lane of slot s (every lane needs a slot)
    void init(size_t pool_bytes, const std::vector<int>& slot_lanes, int max_batch, int max_inflight) {
        pool_.reset(pool_bytes);
        slots_.assign(slot_lanes.size(), Slot{});
        for (size_t s = 0; s < slot_lanes.size(); ++s) slots_[s].lane = slot_lanes[s];
        max_batch_ = max_batch;
        max_inflight_ = max_inflight;
    }

    // Queue a request of `bytes` workspace alone on `lane`; handle: the
    // caller's identifier of its payload.  LQT_ENOMEM: it can never fit the
    // pool; LQT_EBUSY: max_inflight requests are queued or running.
    int submit(uint64_t ticket, int lane, size_t bytes, size_t handle) {
        if (bytes > pool_.size()) return LQT_ENOMEM;
        if (live_ >= (size_t)max_inflight_) return LQT_EBUSY;
        if (lane < 0 || lane >= kLanes) lane = kLanes - 1;
        queue_[lane].push_back(Req{ticket, bytes, handle});
        state_[ticket] = -1;
        ++live_;
        cnt_.submitted += 1;
        return LQT_OK;
    }

    // Retire finished batches, then launch queued requests on idle slots.
    // Returns LQT_OK, or the first failure (the requests of a failed batch
    // take that status; its range is returned after its slot is drained).
    int pump(Ops& ops) {
        int err = LQT_OK;
        for (size_t s = 0; s < slots_.size(); ++s) {
            Slot& sl = slots_[s];
            if (!sl.busy) continue;
            const int q = ops.query((int)s);
            if (q == 0) continue;
            if (q < 0) {
                ops.drain((int)s);
                retire(ops, (int)s, LQT_EHIP);
                if (err == LQT_OK) err = LQT_EHIP;
            } else {
                retire(ops, (int)s, -1);
            }
        }
        bool waiting[kLanes] = {false, false};  // lane head waits for pool memory
        size_t need[kLanes] = {0, 0};
        for (int l = 0; l < kLanes; ++l)
            if (!queue_[l].empty() && queue_[l].front().bytes > pool_.largest()) {
                waiting[l] = true;
                need[l] = queue_[l].front().bytes;
            }
        for (size_t s = 0; s < slots_.size(); ++s) {
            Slot& sl = slots_[s];
            const int l = sl.lane;
            if (sl.busy || queue_[l].empty() || waiting[l]) continue;
            // longest prefix whose batch fits the largest free range
            const size_t room = pool_.largest();
            std::vector<size_t> ids;
            typename Ops::Acc acc = ops.acc();
            for (size_t k = 0; k < queue_[l].size() && (int)ids.size() < max_batch_; ++k) {
                typename Ops::Acc t = acc;
                t.add(queue_[l][k].handle);
                if (t.total() > room) break;
                acc = t;
                ids.push_back(queue_[l][k].handle);
            }
            const size_t bytes = acc.total();
            if (ids.empty()) {
                waiting[l] = true;
                need[l] = queue_[l].front().bytes;
                continue;
            }
            // leave room for the waiting heads of the other lanes
            bool hurts = false;
            for (int o = 0; o < kLanes; ++o)
                if (o != l && waiting[o] && pool_.largest_after(bytes) < need[o]) hurts = true;
            if (hurts) continue;
            size_t off = 0;
            if (!pool_.take(bytes, off)) continue;
            sl.busy = true;
            sl.off = off;
            sl.len = bytes;
            sl.tickets.clear();
            for (size_t k = 0; k < ids.size(); ++k) sl.tickets.push_back(queue_[l][k].ticket);
            queue_[l].erase(queue_[l].begin(), queue_[l].begin() + (ptrdiff_t)ids.size());
            cnt_.batches += 1;
            cnt_.running_batches += 1;
            cnt_.max_running_batches = std::max(cnt_.max_running_batches, cnt_.running_batches);
            cnt_.max_batch = std::max(cnt_.max_batch, (int32_t)ids.size());
            cnt_.pool_peak = std::max(cnt_.pool_peak, pool_.in_use());
            const int st = ops.launch((int)s, ids.data(), ids.size(), off, bytes);
            if (st != LQT_OK) {
                ops.drain((int)s);
                retire(ops, (int)s, st);
                if (err == LQT_OK) err = st;
            }
        }
        return err;
    }

    // false while the request is queued or running; then true with its status
    // (the ticket is forgotten).  Unknown ticket: true with LQT_EINVAL.
    bool poll(uint64_t ticket, int& status) {
        auto it = state_.find(ticket);
        if (it == state_.end()) {
            status = LQT_EINVAL;
            return true;
        }
        if (it->second < 0) return false;
        status = it->second;
        state_.erase(it);
        return true;
    }
    bool known(uint64_t ticket) const { return state_.count(ticket) != 0; }
    bool pending(uint64_t ticket) const {
        auto it = state_.find(ticket);
        return it != state_.end() && it->second < 0;
    }

    int busy_slot() const {  // a slot with a batch in flight, or -1
        for (size_t s = 0; s < slots_.size(); ++s)
            if (slots_[s].busy) return (int)s;
        return -1;
    }
    bool idle() const { return live_ == 0; }
    int32_t queued() const { return (int32_t)(queue_[0].size() + queue_[1].size()); }
    const ServeCounters& counters() const { return cnt_; }
    const RangePool& pool() const { return pool_; }
    size_t live() const { return live_; }

private:
    struct Req {
        uint64_t ticket;
        size_t bytes, handle;
    };
    struct Slot {
        int lane = 0;
        bool busy = false;
        size_t off = 0, len = 0;
        std::vector<uint64_t> tickets;
    };

    // code < 0: each request's own status from the device, else `code` for all
    void retire(Ops& ops, int s, int code) {
        Slot& sl = slots_[s];
        for (size_t i = 0; i < sl.tickets.size(); ++i) state_[sl.tickets[i]] = code < 0 ? ops.status(s, i) : code;
        live_ -= sl.tickets.size();
        cnt_.completed += (int64_t)sl.tickets.size();
        cnt_.running_batches -= 1;
        pool_.give(sl.off, sl.len);
        sl.tickets.clear();
        sl.busy = false;
    }

    RangePool pool_;
    std::vector<Slot> slots_;
    std::deque<Req> queue_[kLanes];
    std::unordered_map<uint64_t, int> state_;  // -1 queued or running, else the final status
    size_t live_ = 0;
    int max_batch_ = 1, max_inflight_ = 1;
    ServeCounters cnt_;
};

}  // namespace lqt
