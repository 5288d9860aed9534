// Host check of the serving policy (queue, arena, admission, batching) against a
// fake executor that finishes batches in random order.  Exit status 0 = pass.
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <map>
#include <random>
#include <set>
#include <vector>

#include "sk_sched.hpp"

static int failures = 0;
#define CHECK(c)                                                         \
    do {                                                                 \
        if (!(c)) {                                                      \
            fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
            ++failures;                                                  \
        }                                                                \
    } while (0)

static void arena_cases() {
    sk::Arena a(4096);
    CHECK(a.capacity() == 4096);
    const int64_t x = a.alloc(1000), y = a.alloc(1000), z = a.alloc(1000);
    CHECK(x == 0 && y == 1024 && z == 2048);
    CHECK(a.alloc(2000) == -1);             // 1024 left
    a.free(y);
    CHECK(a.largest_free() == 1024);
    a.free(x);                              // merges with y's range
    CHECK(a.largest_free() == 2048);
    CHECK(a.alloc(2000) == 0);              // first fit reuses the merged range
    a.free(0);
    a.free(z);
    CHECK(a.in_use() == 0 && a.largest_free() == 4096);
    CHECK(a.alloc(0) == 0 && a.in_use() == 0);
    a.free(12345);                          // unknown offset: ignored
    CHECK(a.in_use() == 0);
}

static void admission_cases() {
    // budget 10 KiB, 2 slots, batches of 2
    sk::Scheduler s(10240, 2, 2, 4);
    sk::ReqInfo big{8192, 1}, small{1024, 1}, other{1024, 2};
    CHECK(s.submit({20000, 1}, 0) == -1);   // larger than the whole budget
    const int64_t a = s.submit(big, 0), b = s.submit(big, 0), c = s.submit(small, 0);
    CHECK(a == 1 && b == 2 && c == 3);
    auto bs = s.admit(1);
    // a fits; b does not (memory) and c must not overtake it
    CHECK(bs.size() == 1 && bs[0].reqs.size() == 1 && bs[0].reqs[0] == a);
    sk::Req r;
    CHECK(s.get(c, &r) && r.state == sk::kQueued);
    CHECK(s.submit(other, 1) == 4);
    CHECK(s.submit(other, 1) == 5);
    CHECK(s.submit(other, 1) == -2);        // queue (4) full
    CHECK(s.cancel(4) && !s.cancel(4) && !s.cancel(a));
    s.finish_batch(bs[0].id, true, 2);
    CHECK(s.get(a, &r) && r.state == sk::kDone && r.t_done == 2);
    bs = s.admit(3);
    // b and c admitted (2 slots); 5 waits for a slot
    CHECK(bs.size() == 1 && bs[0].reqs == std::vector<int64_t>({b, c}));
    CHECK(s.stats().running == 2 && s.stats().bytes_in_use == 9216);
    s.finish_batch(bs[0].id, false, 4);
    CHECK(s.get(b, &r) && r.state == sk::kFailed);
    bs = s.admit(5);
    CHECK(bs.size() == 1 && bs[0].reqs[0] == 5 && bs[0].tile_class == 2);
    s.finish_batch(bs[0].id, true, 6);
    const sk::SchedStats st = s.stats();
    CHECK(st.completed == 2 && st.failed == 2 && st.cancelled == 1 && st.rejected == 2);
    CHECK(st.bytes_in_use == 0 && st.running == 0 && st.queued == 0);
    CHECK(s.forget(a) && !s.get(a, &r) && !s.forget(a) && s.get(5, &r));
    CHECK(s.submit(small, 7) == 6 && !s.forget(6));   // queued: kept
}

static void grouped_admission_cases() {
    // 4 slots; admissions wait until 3 are free
    sk::Scheduler s(1 << 20, 4, 4, 64);
    for (int i = 0; i < 8; ++i) CHECK(s.submit({1024, 1}, 0) == i + 1);
    auto b1 = s.admit(1, 3);
    CHECK(b1.size() == 1 && b1[0].reqs.size() == 4);   // all 4 free: admit 4
    CHECK(s.admit(2, 3).empty());                        // none free
    s.finish_batch(b1[0].id, true, 3);
    auto b2 = s.admit(4, 9);                             // threshold capped at the slot count
    CHECK(b2.size() == 1 && b2[0].reqs == std::vector<int64_t>({5, 6, 7, 8}));
}

static void random_run(uint32_t seed) {
    std::mt19937 rng(seed);
    const size_t budget = 1 << 20;
    const int slots = 1 + rng() % 8, maxb = 1 + rng() % 5;
    sk::Scheduler s(budget, slots, maxb, 64);
    std::map<int64_t, std::pair<int64_t, size_t>> live;   // id -> (offset, bytes)
    std::map<int64_t, std::vector<int64_t>> inflight;
    std::vector<int64_t> submitted, admitted_order;
    std::set<int64_t> cancelled;
    double now = 0;
    int to_submit = 400;
    while (to_submit > 0 || !inflight.empty() || s.stats().queued > 0) {
        now += 1;
        const int op = rng() % 4;
        if (op == 0 && to_submit > 0) {
            sk::ReqInfo in{(size_t)(rng() % 3 == 0 ? 0 : 1 + rng() % (budget / 3)), (int)(rng() % 3)};
            const int64_t id = s.submit(in, now);
            if (id > 0) {
                submitted.push_back(id);
                --to_submit;
            }
        } else if (op == 1 && !submitted.empty() && rng() % 8 == 0) {
            const int64_t id = submitted[rng() % submitted.size()];
            sk::Req r;
            const bool was_queued = s.get(id, &r) && r.state == sk::kQueued;
            CHECK(s.cancel(id) == was_queued);
            if (was_queued) cancelled.insert(id);
        } else if (op == 2) {
            std::vector<int64_t> this_call;   // batches group by class: sort the call's ids
            const int min_free = (int)(rng() % 3 == 0 ? 1 + rng() % slots : 1);
            for (const sk::Batch& b : s.admit(now, min_free)) {
                CHECK(!b.reqs.empty() && (int)b.reqs.size() <= maxb);
                for (int64_t id : b.reqs) {
                    sk::Req r;
                    CHECK(s.get(id, &r) && r.state == sk::kRunning && r.batch == b.id);
                    CHECK(r.info.tile_class == b.tile_class);
                    if (r.arena_offset >= 0) {
                        // no overlap with any live range, inside the budget
                        const int64_t lo = r.arena_offset, hi = lo + (int64_t)r.info.footprint;
                        CHECK(hi <= (int64_t)budget);
                        for (auto& kv : live)
                            CHECK(hi <= kv.second.first ||
                                  lo >= kv.second.first + (int64_t)kv.second.second);
                        live[id] = {lo, r.info.footprint};
                    }
                    this_call.push_back(id);
                }
                inflight[b.id] = b.reqs;
            }
            std::sort(this_call.begin(), this_call.end());
            admitted_order.insert(admitted_order.end(), this_call.begin(), this_call.end());
            CHECK(s.stats().running <= slots);
            CHECK(s.stats().bytes_in_use <= budget);
        } else if (op == 3 && !inflight.empty()) {
            auto it = inflight.begin();
            std::advance(it, rng() % inflight.size());
            s.finish_batch(it->first, rng() % 10 != 0, now);
            for (int64_t id : it->second) live.erase(id);
            inflight.erase(it);
        }
    }
    // FIFO: each admission takes a prefix of the queue, so the admitted ids are the
    // submitted ones, minus the cancelled, in order
    std::vector<int64_t> expect;
    for (int64_t id : submitted)
        if (!cancelled.count(id)) expect.push_back(id);
    CHECK(admitted_order == expect);
    const sk::SchedStats st = s.stats();
    CHECK(st.completed + st.failed + st.cancelled == (int64_t)submitted.size());
    CHECK(st.bytes_in_use == 0 && st.running == 0 && st.peak_bytes_in_use <= budget);
    CHECK(st.max_running <= slots);
}

int main() {
    arena_cases();
    admission_cases();
    grouped_admission_cases();
    for (uint32_t seed = 1; seed <= 200; ++seed) random_run(seed);
    if (failures) {
        fprintf(stderr, "%d check(s) failed\n", failures);
        return 1;
    }
    printf("scheduler checks passed\n");
    return 0;
}
