// Admission control and tick formation of the request server.
//
// Host-only C++ (no HIP): the same policy object runs inside the HIP server
// (wall clock, ticks executed by the device) and inside the simulated-clock
// entry point that tests the policy on the CPU.
//
// Life of a request: Pending (waiting for memory) -> Admitted (its output
// buffer reserved in the arena) -> Launched (part of a tick) -> Done
// (results readable) -> released by the client, which frees its memory.
// Admission is strict FIFO: the oldest pending request is admitted first and
// a request that does not fit blocks the ones behind it, so no request
// starves.  A tick takes admitted requests in order up to a draw and a
// triangle limit (always at least one) and is formed only while fewer than
// `max_inflight` ticks are queued on the device: under load, requests that
// arrive while ticks run accumulate and the next tick carries all of them
// (continuous batching).
#pragma once

#include <algorithm>
#include <cstdint>
#include <deque>
#include <iterator>
#include <map>
#include <unordered_map>
#include <vector>

namespace vr {
namespace sched {

// First-fit allocator over [0, capacity) in 256-byte granules.  Free blocks
// are kept by offset and merged with their neighbours on release.
class Arena {
  public:
    static constexpr uint64_t kGranule = 256;
    explicit Arena(uint64_t capacity = 0) { reset(capacity); }

    static uint64_t round_up(uint64_t b) { return (std::max<uint64_t>(b, 1) + kGranule - 1) & ~(kGranule - 1); }

    void reset(uint64_t capacity) {
        cap_ = capacity & ~(kGranule - 1);
        free_.clear();
        if (cap_) free_[0] = cap_;
        used_ = peak_ = 0;
    }

    bool alloc(uint64_t bytes, uint64_t *off) {
        bytes = round_up(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const uint64_t at = it->first + bytes, rest = it->second - bytes;
            free_.erase(it);
            if (rest) free_[at] = rest;
            used_ += bytes;
            peak_ = std::max(peak_, used_);
            return true;
        }
        return false;
    }

    void release(uint64_t off, uint64_t bytes) {
        bytes = round_up(bytes);
        used_ -= bytes;
        uint64_t start = off, len = bytes;
        auto next = free_.lower_bound(off);
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                start = prev->first;
                len += prev->second;
                free_.erase(prev);
            }
        }
        if (next != free_.end() && off + bytes == next->first) {
            len += next->second;
            free_.erase(next);
        }
        free_[start] = len;
    }

    uint64_t capacity() const { return cap_; }
    uint64_t used() const { return used_; }
    uint64_t peak() const { return peak_; }
    size_t free_blocks() const { return free_.size(); }

  private:
    uint64_t cap_ = 0, used_ = 0, peak_ = 0;
    std::map<uint64_t, uint64_t> free_;
};

enum class State : uint8_t { Pending, Admitted, Launched, Done };

// Status codes carried by jobs (values of vr_status).
constexpr int kOk = 0, kArg = 1, kCapacity = 3, kBusy = 6, kCancelled = 7;

struct Job {
    uint64_t ticket = 0, user = 0;
    uint64_t bytes = 0;   // arena reservation
    uint64_t tris = 0;    // work size, for the tick limit
    uint64_t off = 0;
    bool has_mem = false;
    State state = State::Pending;
    int status = kOk;
    uint32_t tick = 0;
    double t_submit = 0, t_admit = -1, t_launch = -1, t_done = -1;
};

struct Policy {
    uint64_t budget = 0;
    uint32_t max_inflight = 2;
    uint32_t max_tick_draws = 1024;
    uint64_t max_tick_tris = 0;   // 0: no limit
};

struct Counts {
    uint64_t submitted = 0, completed = 0, cancelled = 0, rejected = 0, ticks = 0;
    uint64_t max_pending = 0, max_tick_draws = 0, admission_blocked = 0;
};

class Scheduler {
  public:
    explicit Scheduler(const Policy &p) : p_(p), arena_(p.budget) {}

    const Policy &policy() const { return p_; }
    const Arena &arena() const { return arena_; }
    const Counts &counts() const { return n_; }
    size_t pending() const { return pending_.size(); }
    size_t admitted() const { return admitted_.size(); }
    size_t inflight() const { return inflight_.size(); }
    bool idle() const { return pending_.empty() && admitted_.empty() && inflight_.empty(); }

    Job *find(uint64_t ticket) {
        auto it = jobs_.find(ticket);
        return it == jobs_.end() ? nullptr : &it->second;
    }

    // A request larger than the whole budget can never be admitted: rejected.
    int submit(uint64_t user, uint64_t bytes, uint64_t tris, double now, uint64_t *ticket) {
        if (Arena::round_up(bytes) > arena_.capacity()) {
            ++n_.rejected;
            return kCapacity;
        }
        Job j;
        j.ticket = next_ticket_++;
        j.user = user;
        j.bytes = bytes;
        j.tris = tris;
        j.t_submit = now;
        jobs_[j.ticket] = j;
        pending_.push_back(j.ticket);
        ++n_.submitted;
        n_.max_pending = std::max<uint64_t>(n_.max_pending, pending_.size());
        *ticket = j.ticket;
        return kOk;
    }

    // Pending and admitted (not yet launched) jobs end as cancelled; a
    // launched or finished job cannot be cancelled.
    int cancel(uint64_t ticket, double now) {
        Job *j = find(ticket);
        if (!j) return kArg;
        if (j->state == State::Launched || j->state == State::Done) return kBusy;
        auto &q = j->state == State::Pending ? pending_ : admitted_;
        q.erase(std::find(q.begin(), q.end(), ticket));
        if (j->has_mem) {
            arena_.release(j->off, j->bytes);
            j->has_mem = false;
        }
        j->state = State::Done;
        j->status = kCancelled;
        j->t_done = now;
        ++n_.cancelled;
        return kOk;
    }

    // Moves pending jobs into memory in submission order; returns how many.
    size_t admit(double now) {
        size_t k = 0;
        while (!pending_.empty()) {
            Job &j = jobs_[pending_.front()];
            if (!arena_.alloc(j.bytes, &j.off)) {
                ++n_.admission_blocked;
                break;
            }
            j.has_mem = true;
            j.state = State::Admitted;
            j.t_admit = now;
            admitted_.push_back(j.ticket);
            pending_.pop_front();
            ++k;
        }
        return k;
    }

    // Forms the next tick if a device slot is free.
    bool next_tick(double now, std::vector<uint64_t> &out, uint32_t *tick_id) {
        out.clear();
        if (admitted_.empty() || inflight_.size() >= p_.max_inflight) return false;
        uint64_t tris = 0;
        while (!admitted_.empty() && out.size() < p_.max_tick_draws) {
            Job &j = jobs_[admitted_.front()];
            if (!out.empty() && p_.max_tick_tris && tris + j.tris > p_.max_tick_tris) break;
            tris += j.tris;
            j.state = State::Launched;
            j.t_launch = now;
            j.tick = next_tick_;
            out.push_back(j.ticket);
            admitted_.pop_front();
        }
        *tick_id = next_tick_++;
        inflight_.push_back({*tick_id, out});
        ++n_.ticks;
        n_.max_tick_draws = std::max<uint64_t>(n_.max_tick_draws, out.size());
        return true;
    }

    // The oldest in-flight tick has finished; its jobs end with `status`
    // unless set_status was called for them before.
    void retire_oldest(double now, int status) {
        if (inflight_.empty()) return;
        for (uint64_t t : inflight_.front().second) {
            Job &j = jobs_[t];
            j.state = State::Done;
            if (j.status == kOk) j.status = status;
            j.t_done = now;
            ++n_.completed;
        }
        inflight_.pop_front();
    }

    uint32_t oldest_tick() const { return inflight_.empty() ? 0u : inflight_.front().first; }
    const std::vector<uint64_t> &oldest_jobs() const { return inflight_.front().second; }

    // The client is done with a finished job: its memory is freed and the
    // job forgotten.
    int release(uint64_t ticket) {
        Job *j = find(ticket);
        if (!j) return kArg;
        if (j->state != State::Done) return kBusy;
        if (j->has_mem) arena_.release(j->off, j->bytes);
        jobs_.erase(ticket);
        return kOk;
    }

    // Cancels everything not yet launched (shutdown).
    std::vector<uint64_t> cancel_all(double now) {
        std::vector<uint64_t> out(pending_.begin(), pending_.end());
        out.insert(out.end(), admitted_.begin(), admitted_.end());
        for (uint64_t t : out) cancel(t, now);
        return out;
    }

  private:
    Policy p_;
    Arena arena_;
    std::unordered_map<uint64_t, Job> jobs_;
    std::deque<uint64_t> pending_, admitted_;
    std::deque<std::pair<uint32_t, std::vector<uint64_t>>> inflight_;
    uint64_t next_ticket_ = 1;
    uint32_t next_tick_ = 0;
    Counts n_;
};

}  // namespace sched
}  // namespace vr
