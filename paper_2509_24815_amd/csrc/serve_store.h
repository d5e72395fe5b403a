// Request store and scratch accounting of the serving loop (host-only C++,
// no HIP): tickets are handed out in submission order; a request's words are
// dropped once they are copied into a batch, and its result once the caller
// releases its ticket, so a long-running server holds only the requests that
// are queued, in flight, or done and not yet released.
#pragma once

#include <cstdint>
#include <deque>
#include <utility>
#include <vector>

namespace seismic {

struct ServeRequest {
    std::vector<uint32_t> words;  // emptied at admission
    double not_before = 0.0;      // server clock (s): earliest admission
    double arrival = 0.0;         // max(submit time, not_before)
    double done_at = 0.0;
    bool done = false;
    std::vector<uint32_t> ids;    // k results once done
    std::vector<float> scores;
};

class RequestStore {
  public:
    // Ticket of the next submission.
    uint64_t end() const { return base_ + q_.size(); }
    // First ticket still held (tickets below it were released).
    uint64_t base() const { return base_; }
    uint64_t held() const { return q_.size(); }
    uint64_t completed() const { return completed_; }
    uint64_t next_admit() const { return next_admit_; }

    uint64_t submit(ServeRequest&& r) {
        q_.push_back(std::move(r));
        return end() - 1;
    }
    // nullptr for a released or unknown ticket.
    ServeRequest* get(uint64_t t) { return t >= base_ && t < end() ? &q_[t - base_] : nullptr; }
    const ServeRequest* get(uint64_t t) const { return t >= base_ && t < end() ? &q_[t - base_] : nullptr; }
    double last_not_before() const { return q_.empty() ? last_nb_ : q_.back().not_before; }

    bool has_pending() const { return next_admit_ < end(); }
    ServeRequest& pending() { return q_[next_admit_ - base_]; }
    // The pending request went into a batch: its words are no longer needed.
    uint64_t admit() {
        std::vector<uint32_t>().swap(pending().words);
        return next_admit_++;
    }
    void deliver(uint64_t t, const uint32_t* ids, const float* scores, uint32_t k, double at) {
        ServeRequest& r = q_[t - base_];
        r.ids.assign(ids, ids + k);
        r.scores.assign(scores, scores + k);
        r.done_at = at;
        r.done = true;
        ++completed_;
    }
    // Drop the results of every ticket below end_ticket.  Stops at the first
    // ticket that is not done yet; returns the first ticket still held.
    uint64_t release(uint64_t end_ticket) {
        while (base_ < end_ticket && !q_.empty() && q_.front().done) {
            last_nb_ = q_.front().not_before;
            q_.pop_front();
            ++base_;
        }
        if (q_.empty()) q_.shrink_to_fit();
        return base_;
    }

  private:
    std::deque<ServeRequest> q_;
    uint64_t base_ = 0, next_admit_ = 0, completed_ = 0;
    double last_nb_ = 0.0;
};

// Device scratch an in-flight query holds, in bytes: its words (4 per
// nonzero), its result row (8 per result), its top-k state (8 per result),
// and its block-order buffers (8 bytes for each block of its longest
// possible cut: cut lists times the index's largest block count per list).
inline uint64_t query_scratch_bytes(uint32_t nnz, uint32_t k, uint32_t cut_lists, uint32_t max_list_blocks) {
    return 4ull * nnz + 16ull * k + 8ull * cut_lists * max_list_blocks;
}

// Admission budget shared by every slot of a server.  budget = 0: no limit
// beyond the slots.  inject > 0: that many reservations fail as if the
// budget were held (a host-forced failure; their queries wait).
class ScratchBudget {
  public:
    ScratchBudget(uint64_t budget, uint64_t inject) : budget_(budget), inject_(inject) {}
    bool reserve(uint64_t bytes) {
        if (inject_) {
            --inject_;
            ++failed_;
            return false;
        }
        if (budget_ && used_ + bytes > budget_) {
            ++failed_;
            return false;
        }
        used_ += bytes;
        if (used_ > peak_) peak_ = used_;
        return true;
    }
    void release(uint64_t bytes) { used_ -= bytes; }
    uint64_t used() const { return used_; }
    uint64_t peak() const { return peak_; }
    uint64_t failed() const { return failed_; }
    uint64_t budget() const { return budget_; }

  private:
    uint64_t budget_, inject_, used_ = 0, peak_ = 0, failed_ = 0;
};

}  // namespace seismic
