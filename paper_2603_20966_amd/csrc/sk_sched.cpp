// Serving policy: first-fit arena, FIFO admission by memory footprint and
// in-flight slots, batching by tile class.  Host-only C++.
#include "sk_sched.hpp"

#include <algorithm>

namespace sk {

namespace {
constexpr size_t kGranule = 256;
size_t round_up(size_t b) { return (b + kGranule - 1) / kGranule * kGranule; }
}  // namespace

Arena::Arena(size_t capacity) : capacity_(capacity / kGranule * kGranule) {
    if (capacity_ > 0) free_[0] = capacity_;
}

int64_t Arena::alloc(size_t bytes) {
    if (bytes == 0) return 0;
    const size_t need = round_up(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
        if (it->second < need) continue;
        const size_t off = it->first;
        const size_t left = it->second - need;
        free_.erase(it);
        if (left > 0) free_[off + need] = left;
        used_[off] = need;
        in_use_ += need;
        return (int64_t)off;
    }
    return -1;
}

void Arena::free(int64_t offset) {
    auto u = used_.find((size_t)offset);
    if (offset < 0 || u == used_.end()) return;
    size_t off = u->first, size = u->second;
    used_.erase(u);
    in_use_ -= size;
    // merge with the free neighbours
    auto next = free_.lower_bound(off);
    if (next != free_.end() && off + size == next->first) {
        size += next->second;
        next = free_.erase(next);
    }
    if (next != free_.begin()) {
        auto prev = std::prev(next);
        if (prev->first + prev->second == off) {
            prev->second += size;
            return;
        }
    }
    free_[off] = size;
}

size_t Arena::largest_free() const {
    size_t best = 0;
    for (const auto& f : free_) best = std::max(best, f.second);
    return best;
}

Scheduler::Scheduler(size_t budget_bytes, int max_running, int max_batch, int max_queue)
    : arena_(budget_bytes),
      max_running_(std::max(1, max_running)),
      max_batch_(std::max(1, max_batch)),
      max_queue_(std::max(1, max_queue)) {}

int64_t Scheduler::submit(const ReqInfo& info, double now) {
    if (round_up(info.footprint) > arena_.capacity()) {
        ++st_.rejected;
        return -1;
    }
    if ((int64_t)queue_.size() >= max_queue_) {
        ++st_.rejected;
        return -2;
    }
    Req r;
    r.id = next_id_++;
    r.info = info;
    r.t_submit = now;
    reqs_[r.id] = r;
    queue_.push_back(r.id);
    ++st_.submitted;
    ++st_.queued;
    return r.id;
}

std::vector<Batch> Scheduler::admit(double now, int min_free) {
    std::vector<Req*> admitted;
    if (max_running_ - st_.running < std::min(std::max(1, min_free), max_running_)) return {};
    while (!queue_.empty() && st_.running < max_running_) {
        Req& r = reqs_[queue_.front()];
        int64_t off = 0;
        if (r.info.footprint > 0) {
            off = arena_.alloc(r.info.footprint);
            if (off < 0) break;   // wait for memory: no request overtakes the head
        }
        queue_.pop_front();
        r.arena_offset = r.info.footprint > 0 ? off : -1;
        r.state = kRunning;
        r.t_start = now;
        admitted.push_back(&r);
        --st_.queued;
        ++st_.running;
        ++st_.admitted;
    }
    st_.bytes_in_use = arena_.in_use();
    st_.peak_bytes_in_use = std::max(st_.peak_bytes_in_use, st_.bytes_in_use);
    st_.max_running = std::max(st_.max_running, st_.running);

    // group by tile class, keeping admission order inside each class
    std::vector<Batch> out;
    std::vector<bool> taken(admitted.size(), false);
    for (size_t i = 0; i < admitted.size(); ++i) {
        if (taken[i]) continue;
        Batch cur;
        cur.tile_class = admitted[i]->info.tile_class;
        for (size_t j = i; j < admitted.size(); ++j) {
            if (taken[j] || admitted[j]->info.tile_class != cur.tile_class) continue;
            if ((int)cur.reqs.size() == max_batch_) {
                out.push_back(cur);
                cur.reqs.clear();
            }
            cur.reqs.push_back(admitted[j]->id);
            taken[j] = true;
        }
        out.push_back(cur);
    }
    for (auto& b : out) {
        b.id = next_batch_++;
        for (int64_t id : b.reqs) reqs_[id].batch = b.id;
        batches_[b.id] = b.reqs;
        ++st_.batches;
    }
    return out;
}

void Scheduler::finish_batch(int64_t batch, bool ok, double now) {
    auto it = batches_.find(batch);
    if (it == batches_.end()) return;
    for (int64_t id : it->second) {
        Req& r = reqs_[id];
        if (r.state != kRunning) continue;
        if (r.arena_offset >= 0) arena_.free(r.arena_offset);
        r.arena_offset = -1;
        r.state = ok ? kDone : kFailed;
        r.t_done = now;
        --st_.running;
        if (ok) ++st_.completed;
        else ++st_.failed;
    }
    batches_.erase(it);
    st_.bytes_in_use = arena_.in_use();
}

bool Scheduler::cancel(int64_t id) {
    auto it = reqs_.find(id);
    if (it == reqs_.end() || it->second.state != kQueued) return false;
    queue_.erase(std::find(queue_.begin(), queue_.end(), id));
    it->second.state = kCancelled;
    --st_.queued;
    ++st_.cancelled;
    return true;
}

bool Scheduler::get(int64_t id, Req* out) const {
    auto it = reqs_.find(id);
    if (it == reqs_.end()) return false;
    *out = it->second;
    return true;
}

bool Scheduler::forget(int64_t id) {
    auto it = reqs_.find(id);
    if (it == reqs_.end() || it->second.state < kDone) return false;
    reqs_.erase(it);
    return true;
}

SchedStats Scheduler::stats() const { return st_; }

}  // namespace sk
