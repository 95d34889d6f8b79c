// Request admission of the serving loop (host only, no device calls): a
// FIFO queue of requests with their scratch footprint (an upper bound of
// what their launch uses), and a scratch pool of `budget` bytes that every
// launched batch takes one contiguous region of.  The pool is the server's
// whole device scratch, so the budget bounds what is allocated, not only
// what is counted.
//
// Rules:
//   - a request larger than the budget, or one more than max_queue queued
//     requests, is refused at submission;
//   - a batch takes queued requests in arrival order, among the first
//     skip_ahead, while their summed footprint fits the largest free region
//     of the pool; a request that does not fit is passed over, and counts
//     it; once a request has been passed over max_skips times, nothing
//     behind it is admitted until it is (so it waits at most until the
//     batches in flight finish: with the pool empty every request fits);
//   - with a hold time, a partial batch (fewer than max_batch queued) waits
//     until its oldest request is that old, unless flushing;
//   - a queued request may be cancelled, and one still queued at its
//     deadline expires.
// Everything is a pure function of the calls and the clock values passed
// in, so the order of admission is deterministic.
#pragma once
#include <stdint.h>

#include <algorithm>
#include <deque>
#include <map>
#include <vector>

namespace habmi {

struct AdmReq {
    uint64_t ticket = 0;
    uint64_t bytes = 0;        // scratch footprint (upper bound)
    uint64_t submit_ns = 0;
    uint64_t deadline_ns = 0;  // 0: none
    uint32_t skipped = 0;      // batches that passed it over
};

class Admission {
public:
    enum Submit { kQueued = 0, kTooBig = 1, kQueueFull = 2 };

    struct Batch {
        std::vector<AdmReq> reqs;
        uint64_t offset = 0, size = 0;   // region of the pool
    };

    Admission(uint64_t budget, uint32_t max_queue, uint32_t max_batch, uint32_t skip_ahead,
              uint32_t max_skips)
        : budget_(budget), max_queue_(max_queue), max_batch_(std::max<uint32_t>(max_batch, 1)),
          skip_ahead_(std::max<uint32_t>(skip_ahead, 1)), max_skips_(max_skips)
    {
        if (budget_) free_[0] = budget_;
    }

    uint64_t budget() const { return budget_; }
    size_t queued() const { return q_.size(); }
    uint64_t in_use() const { return in_use_; }

    Submit submit(const AdmReq &r)
    {
        if (r.bytes > budget_) return kTooBig;
        if (q_.size() >= max_queue_) return kQueueFull;
        q_.push_back(r);
        q_.back().skipped = 0;
        return kQueued;
    }

    // Remove a queued request; false if it is not queued (launched, done or
    // unknown).
    bool cancel(uint64_t ticket)
    {
        for (auto it = q_.begin(); it != q_.end(); ++it)
            if (it->ticket == ticket) {
                q_.erase(it);
                return true;
            }
        return false;
    }

    // Remove the queued requests whose deadline is at or before `now`,
    // appending their tickets to `out` in queue order.
    void expire(uint64_t now, std::vector<uint64_t> &out)
    {
        for (auto it = q_.begin(); it != q_.end();) {
            if (it->deadline_ns && it->deadline_ns <= now) {
                out.push_back(it->ticket);
                it = q_.erase(it);
            } else {
                ++it;
            }
        }
    }

    uint64_t largest_free() const
    {
        uint64_t m = 0;
        for (const auto &f : free_) m = std::max(m, f.second);
        return m;
    }

    // The next batch, its region taken from the pool; false when nothing
    // can start now (empty queue, holding, or nothing fits until a region
    // is released).
    bool next(uint64_t now, uint64_t hold_ns, bool flushing, Batch &b)
    {
        b.reqs.clear();
        b.offset = b.size = 0;
        if (q_.empty()) return false;
        if (hold_ns && !flushing && q_.size() < max_batch_ && now - q_.front().submit_ns < hold_ns)
            return false;
        const uint64_t room = largest_free();
        uint64_t total = 0;
        uint32_t scanned = 0;
        std::vector<size_t> take, passed;
        for (size_t i = 0; i < q_.size() && take.size() < max_batch_ && scanned < skip_ahead_; ++i, ++scanned) {
            const AdmReq &r = q_[i];
            if (total + r.bytes <= room) {
                total += r.bytes;
                take.push_back(i);
            } else {
                // passed over; one passed over too often stops the scan
                if (r.skipped >= max_skips_) break;
                passed.push_back(i);
            }
        }
        if (take.empty()) return false;
        // only a batch that launches passes anyone over
        for (size_t i : passed)
            if (i < take.back()) ++q_[i].skipped;
        // first fit: the lowest region that holds the batch
        auto it = free_.begin();
        while (it != free_.end() && it->second < total) ++it;
        if (it == free_.end()) return false;   // unreachable: total <= room
        b.offset = it->first;
        b.size = total;
        const uint64_t rest = it->second - total, rest_off = it->first + total;
        free_.erase(it);
        if (rest) free_[rest_off] = rest;
        in_use_ += total;
        for (size_t k = take.size(); k-- > 0;) {
            b.reqs.push_back(q_[take[k]]);
            q_.erase(q_.begin() + (std::ptrdiff_t)take[k]);
        }
        std::reverse(b.reqs.begin(), b.reqs.end());
        return true;
    }

    // Return a batch's region to the pool (merging neighbours).
    void release(uint64_t offset, uint64_t size)
    {
        if (!size) return;
        in_use_ -= size;
        auto nx = free_.lower_bound(offset);
        uint64_t off = offset, sz = size;
        if (nx != free_.begin()) {
            auto pv = std::prev(nx);
            if (pv->first + pv->second == off) {
                off = pv->first;
                sz += pv->second;
                free_.erase(pv);
            }
        }
        if (nx != free_.end() && off + sz == nx->first) {
            sz += nx->second;
            free_.erase(nx);
        }
        free_[off] = sz;
    }

private:
    uint64_t budget_;
    uint32_t max_queue_, max_batch_, skip_ahead_, max_skips_;
    std::deque<AdmReq> q_;
    std::map<uint64_t, uint64_t> free_;   // offset -> size of each free region
    uint64_t in_use_ = 0;
};

}  // namespace habmi
