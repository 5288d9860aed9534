// Serving policy for sketch requests: a FIFO queue, a first-fit allocator over
// a fixed device-memory budget, admission by memory footprint and in-flight
// slots, and batching of admitted requests by tile class.  Pure C++ (no HIP):
// the executor that launches batches is behind a small interface, so the
// policy is tested on the host with a fake executor.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <deque>
#include <map>
#include <vector>

namespace sk {

// First-fit allocator over [0, capacity) with 256-byte granules.
class Arena {
public:
    explicit Arena(size_t capacity);
    // Offset of a free range of at least `bytes`, or -1.  bytes == 0 -> 0 (no range).
    int64_t alloc(size_t bytes);
    void free(int64_t offset);
    size_t capacity() const { return capacity_; }
    size_t in_use() const { return in_use_; }
    size_t largest_free() const;

private:
    size_t capacity_;
    size_t in_use_ = 0;
    std::map<size_t, size_t> free_;   // offset -> size
    std::map<size_t, size_t> used_;   // offset -> size
};

enum ReqState : int { kQueued = 0, kRunning = 1, kDone = 2, kFailed = 3, kCancelled = 4 };

// What the policy needs to know about a request.
struct ReqInfo {
    size_t footprint = 0;   // device bytes the server must hold while it runs
    int tile_class = 0;     // requests of one class can share a launch
};

struct Req {
    int64_t id = 0;
    ReqInfo info;
    int state = kQueued;
    int64_t arena_offset = -1;
    int64_t batch = -1;
    double t_submit = 0, t_start = 0, t_done = 0;
};

struct Batch {
    int64_t id = 0;
    int tile_class = 0;
    std::vector<int64_t> reqs;   // request ids in admission order
};

struct SchedStats {
    int64_t submitted = 0, admitted = 0, completed = 0, failed = 0, cancelled = 0, rejected = 0;
    int64_t batches = 0, queued = 0, running = 0;
    size_t bytes_in_use = 0, peak_bytes_in_use = 0;
    int64_t max_running = 0;
};

class Scheduler {
public:
    Scheduler(size_t budget_bytes, int max_running, int max_batch, int max_queue);

    // Queue a request; returns its id (>= 1), or -1 if its footprint exceeds the
    // whole budget, or -2 if the queue is full.
    int64_t submit(const ReqInfo& info, double now);
    // Admit queued requests in FIFO order while slots and memory allow (stops at
    // the first that does not fit: no overtaking), and group them into batches
    // of at most max_batch requests of one tile class.  Nothing is admitted
    // unless at least min_free slots are free (so that, under load, admissions
    // come in groups that form batches).
    std::vector<Batch> admit(double now, int min_free = 1);
    int max_running() const { return max_running_; }
    // A batch handed out by admit() finished (ok) or failed: its requests leave
    // the running set and free their memory.
    void finish_batch(int64_t batch, bool ok, double now);
    // Cancel a request that is still queued; false otherwise.
    bool cancel(int64_t id);
    // Copy of a request's record; false for an unknown id.
    bool get(int64_t id, Req* out) const;
    // Forget a finished (done, failed or cancelled) request; false otherwise.
    bool forget(int64_t id);
    SchedStats stats() const;

private:
    Arena arena_;
    int max_running_, max_batch_, max_queue_;
    int64_t next_id_ = 1, next_batch_ = 1;
    std::deque<int64_t> queue_;
    std::map<int64_t, Req> reqs_;
    std::map<int64_t, std::vector<int64_t>> batches_;
    SchedStats st_;
};

}  // namespace sk
