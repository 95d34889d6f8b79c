// Checks of the serving loop's admission rules (csrc/admission.h) with a
// fake clock and budget, on the CPU.  Built by tests/test_admission_host.py
// with AddressSanitizer and UndefinedBehaviorSanitizer; prints "ok" and
// exits 0 when every check holds.
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <map>
#include <random>
#include <set>
#include <vector>

#include "admission.h"

using habmi::AdmReq;
using habmi::Admission;

static int failures = 0;
#define CHECK(c)                                                          \
    do {                                                                  \
        if (!(c)) {                                                       \
            fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
            ++failures;                                                   \
        }                                                                 \
    } while (0)

static AdmReq req(uint64_t t, uint64_t bytes, uint64_t now, uint64_t deadline = 0)
{
    AdmReq r;
    r.ticket = t;
    r.bytes = bytes;
    r.submit_ns = now;
    r.deadline_ns = deadline;
    return r;
}

static std::vector<uint64_t> tickets(const Admission::Batch &b)
{
    std::vector<uint64_t> v;
    for (const auto &r : b.reqs) v.push_back(r.ticket);
    return v;
}

// Submission limits, arrival order, batch size cap, region placement.
static void basics()
{
    Admission a(1000, 4, 3, 64, 8);
    CHECK(a.submit(req(1, 1001, 0)) == Admission::kTooBig);
    for (uint64_t t = 1; t <= 4; ++t) CHECK(a.submit(req(t, 100, t)) == Admission::kQueued);
    CHECK(a.submit(req(5, 100, 5)) == Admission::kQueueFull);
    Admission::Batch b;
    CHECK(a.next(10, 0, false, b));
    CHECK((tickets(b) == std::vector<uint64_t>{1, 2, 3}));
    CHECK(b.offset == 0 && b.size == 300);
    Admission::Batch c, none;
    CHECK(a.next(10, 0, false, c));
    CHECK((tickets(c) == std::vector<uint64_t>{4}));
    CHECK(c.offset == 300 && c.size == 100);
    CHECK(a.in_use() == 400 && a.queued() == 0);
    CHECK(!a.next(10, 0, false, none));
    a.release(b.offset, b.size);
    a.release(c.offset, c.size);
    CHECK(a.in_use() == 0 && a.largest_free() == 1000);
}

// A request that does not fit is passed over by smaller ones, at most
// max_skips times; then it blocks everything behind it until it fits.
static void no_starvation()
{
    const uint32_t max_skips = 3;
    Admission a(1000, 1000, 1, 64, max_skips);
    uint64_t now = 0, next_ticket = 2;
    // a batch of 600 is in flight, then a 900 arrives, then a stream of 100s
    CHECK(a.submit(req(1, 600, now)) == Admission::kQueued);
    Admission::Batch big;
    CHECK(a.next(now, 0, false, big) && big.reqs[0].ticket == 1);
    CHECK(a.submit(req(1000, 900, ++now)) == Admission::kQueued);
    std::vector<Admission::Batch> inflight;
    int passes = 0;
    bool admitted = false;
    for (int round = 0; round < 100 && !admitted; ++round) {
        CHECK(a.submit(req(next_ticket++, 100, ++now)) == Admission::kQueued);
        Admission::Batch b;
        while (a.next(now, 0, false, b)) {
            if (b.reqs[0].ticket == 1000) admitted = true;
            else if (!admitted) ++passes;   // a batch launched past the big request
            inflight.push_back(b);
        }
        // small batches finish right away; the big first batch finishes late
        for (auto &x : inflight) a.release(x.offset, x.size);
        inflight.clear();
        if (round == 20) a.release(big.offset, big.size);
    }
    CHECK(admitted);
    CHECK(passes <= (int)max_skips);
}

// Cancel and expiry remove queued requests only, in queue order.
static void cancel_and_expiry()
{
    Admission a(1000, 100, 8, 64, 8);
    CHECK(a.submit(req(1, 100, 0, 50)) == Admission::kQueued);
    CHECK(a.submit(req(2, 100, 0, 0)) == Admission::kQueued);
    CHECK(a.submit(req(3, 100, 0, 20)) == Admission::kQueued);
    CHECK(a.cancel(2));
    CHECK(!a.cancel(2));
    std::vector<uint64_t> gone;
    a.expire(19, gone);
    CHECK(gone.empty());
    a.expire(20, gone);
    CHECK((gone == std::vector<uint64_t>{3}));
    Admission::Batch b;
    CHECK(a.next(21, 0, false, b) && tickets(b) == std::vector<uint64_t>{1});
    CHECK(!a.cancel(1));   // launched: not cancellable
    gone.clear();
    a.expire(1000, gone);
    CHECK(gone.empty());
}

// A partial batch waits for the hold time unless flushing or full.
static void hold()
{
    Admission a(1000, 100, 2, 64, 8);
    CHECK(a.submit(req(1, 10, 100)) == Admission::kQueued);
    Admission::Batch b;
    CHECK(!a.next(150, 100, false, b));
    CHECK(a.next(150, 100, true, b) && b.reqs.size() == 1);
    CHECK(a.submit(req(2, 10, 200)) == Admission::kQueued);
    CHECK(a.submit(req(3, 10, 201)) == Admission::kQueued);
    CHECK(a.next(202, 100, false, b) && b.reqs.size() == 2);   // full: no hold
    CHECK(a.submit(req(4, 10, 300)) == Admission::kQueued);
    CHECK(!a.next(399, 100, false, b));
    CHECK(a.next(400, 100, false, b));
}

// Random arrivals, completions, cancels and deadlines: regions of the
// batches in flight never overlap and stay inside the budget; every
// request ends exactly once (launched, cancelled or expired); two runs
// with the same seed admit the same batches.
static std::vector<std::vector<uint64_t>> simulate(uint32_t seed, bool check)
{
    std::mt19937_64 rng(seed);
    const uint64_t budget = 1 << 20;
    Admission a(budget, 512, 16, 32, 4);
    std::vector<Admission::Batch> inflight;
    std::vector<std::vector<uint64_t>> log;
    std::set<uint64_t> open, ended;
    uint64_t now = 0, t = 1;
    for (int step = 0; step < 20000; ++step) {
        now += 1 + rng() % 50;
        if (rng() % 3 == 0) {
            const uint64_t bytes = 1 + (rng() % 8 == 0 ? rng() % budget : rng() % (budget / 16));
            const uint64_t dl = rng() % 4 == 0 ? now + rng() % 2000 : 0;
            if (a.submit(req(t, bytes, now, dl)) == Admission::kQueued) open.insert(t);
            ++t;
        }
        if (rng() % 17 == 0 && !open.empty()) {
            auto it = open.begin();
            std::advance(it, (long)(rng() % open.size()));
            const uint64_t k = *it;
            if (a.cancel(k)) {
                open.erase(k);
                CHECK(ended.insert(k).second);
            }
        }
        std::vector<uint64_t> gone;
        a.expire(now, gone);
        for (uint64_t k : gone) {
            CHECK(open.erase(k) == 1);
            CHECK(ended.insert(k).second);
        }
        Admission::Batch b;
        while (inflight.size() < 4 && a.next(now, 100, false, b)) {
            if (check) {
                CHECK(b.offset + b.size <= budget);
                for (const auto &x : inflight)
                    CHECK(b.offset + b.size <= x.offset || x.offset + x.size <= b.offset);
                uint64_t sum = 0;
                for (const auto &r : b.reqs) sum += r.bytes;
                CHECK(sum == b.size);
            }
            for (const auto &r : b.reqs) {
                CHECK(open.erase(r.ticket) == 1);
                CHECK(ended.insert(r.ticket).second);
            }
            log.push_back(tickets(b));
            inflight.push_back(b);
        }
        if (!inflight.empty() && rng() % 4 == 0) {
            const size_t k = rng() % inflight.size();
            a.release(inflight[k].offset, inflight[k].size);
            inflight.erase(inflight.begin() + (long)k);
        }
        uint64_t used = 0;
        for (const auto &x : inflight) used += x.size;
        if (check) CHECK(used == a.in_use() && used <= budget);
    }
    return log;
}

int main()
{
    basics();
    no_starvation();
    cancel_and_expiry();
    hold();
    const auto l1 = simulate(7, true);
    const auto l2 = simulate(7, false);
    CHECK(l1 == l2);
    CHECK(l1.size() > 1000);
    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("ok\n");
    return 0;
}
