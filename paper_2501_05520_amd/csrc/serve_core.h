// Request scheduler of the serving loop (host only, no HIP): the analogue of the
// inference server of Section 2.3 (clients send requests, the server batches them
// and runs them on its coprocessor) and of the concurrent model instances of
// Section 4.2.1.
//
// Requests enter a FIFO queue once admitted by memory: each request carries an
// estimate of the device and staging memory it will hold, and submission waits
// (or is refused, when the estimate alone exceeds the budget) until the in-flight
// total fits the budget.  Each of n_slots workers owns an executor slot (on the
// GPU: a context, a stream and staging buffers); whenever a slot is free it takes
// the queued requests in arrival order, up to max_batch_events events and
// max_batch_hits spacepoints, and runs them as one batch.  Requests that arrive
// while batches are running join the next batch a slot forms, so work of
// different batches overlaps on the device (continuous batching at launch-sequence
// granularity).  A request whose deadline passes before it is batched completes
// with TRK_SERVE_EXPIRED.  Destruction drains: queued requests are run, then the
// workers stop.
//
// The executor is a template parameter: Exec::run(slot, batch) must fill every
// request's labels, info and status.
#pragma once
#include <stdint.h>
#include <string.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

namespace trk_serve {

enum { SERVE_OK = 0, SERVE_INVAL = -1, SERVE_CAPACITY = -3, SERVE_EXPIRED = -7, SERVE_SHUTDOWN = -8 };

typedef std::chrono::steady_clock Clock;

struct Request {
  int64_t id = 0;
  int64_t n = 0;                    // spacepoints
  std::vector<float> x;             // [n][3], copied at submission
  std::vector<int32_t> labels;      // [n], filled by the executor
  int64_t counts[5] = {0, 0, 0, 0, 0};  // n_hits, n_cand, n_filt, n_kept, n_saturated
  float stage_ms[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  uint64_t mem = 0;                 // admission estimate (bytes)
  int status = SERVE_OK;
  bool done = false;
  Clock::time_point t_submit, t_start, t_done, deadline;
  bool has_deadline = false;
};

struct Stats {
  int64_t submitted = 0, completed = 0, rejected = 0, expired = 0, batches = 0, batched_events = 0;
  int64_t admitted_at_once = 0, waited_for_memory = 0;
  uint64_t inflight_bytes = 0, peak_inflight_bytes = 0;
};

template <class Exec>
class Server {
 public:
  Server(Exec* exec, int n_slots, int max_batch_events, int64_t max_batch_hits, uint64_t mem_budget,
         uint64_t bytes_per_hit, uint64_t bytes_per_request)
      : exec_(exec), max_events_(max_batch_events), max_hits_(max_batch_hits), budget_(mem_budget),
        per_hit_(bytes_per_hit), per_req_(bytes_per_request) {
    for (int s = 0; s < n_slots; ++s) workers_.emplace_back([this, s] { worker(s); });
  }

  ~Server() { shutdown(); }

  // Admits a request (copying x) and returns its ticket in *ticket.  Blocks while the
  // memory budget is full.  deadline_ms <= 0: no deadline.
  int submit(const float* x, int64_t n, double deadline_ms, int64_t* ticket) {
    if (!ticket || n < 0 || (n > 0 && !x)) return SERVE_INVAL;
    if (n > max_hits_) return SERVE_CAPACITY;
    std::unique_ptr<Request> r(new Request());
    r->n = n;
    r->x.assign(x, x + 3 * n);
    r->mem = per_req_ + per_hit_ * (uint64_t)n;
    r->t_submit = Clock::now();
    if (deadline_ms > 0) {
      r->has_deadline = true;
      r->deadline = r->t_submit + std::chrono::duration_cast<Clock::duration>(
                                      std::chrono::duration<double, std::milli>(deadline_ms));
    }
    std::unique_lock<std::mutex> lk(mu_);
    if (stop_ || draining_) return SERVE_SHUTDOWN;
    if (r->mem > budget_) {
      ++stats_.rejected;
      return SERVE_CAPACITY;
    }
    ++stats_.submitted;
    if (stats_.inflight_bytes + r->mem <= budget_) {
      ++stats_.admitted_at_once;
    } else {
      ++stats_.waited_for_memory;
      mem_cv_.wait(lk, [&] { return stop_ || draining_ || stats_.inflight_bytes + r->mem <= budget_; });
      if (stop_ || draining_) return SERVE_SHUTDOWN;
    }
    stats_.inflight_bytes += r->mem;
    if (stats_.inflight_bytes > stats_.peak_inflight_bytes) stats_.peak_inflight_bytes = stats_.inflight_bytes;
    r->id = next_id_++;
    *ticket = r->id;
    Request* raw = r.get();
    table_[r->id] = std::move(r);
    queue_.push_back(raw);
    work_cv_.notify_one();
    return SERVE_OK;
  }

  // Waits for a request, copies its labels (n ints) and counts out, and forgets it.
  int wait(int64_t ticket, int32_t* labels, int64_t* counts5, float* stage_ms8, double* latency_ms) {
    std::unique_lock<std::mutex> lk(mu_);
    auto it = table_.find(ticket);
    if (it == table_.end()) return SERVE_INVAL;
    Request* r = it->second.get();
    done_cv_.wait(lk, [&] { return r->done; });
    std::unique_ptr<Request> own = std::move(it->second);
    table_.erase(it);
    lk.unlock();
    if (labels && own->status == SERVE_OK && own->n > 0)
      memcpy(labels, own->labels.data(), sizeof(int32_t) * own->n);
    if (counts5) memcpy(counts5, own->counts, sizeof(own->counts));
    if (stage_ms8) memcpy(stage_ms8, own->stage_ms, sizeof(own->stage_ms));
    if (latency_ms) latency_ms[0] = std::chrono::duration<double, std::milli>(own->t_done - own->t_submit).count();
    return own->status;
  }

  Stats stats() {
    std::lock_guard<std::mutex> lk(mu_);
    return stats_;
  }

  void shutdown() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      if (stop_ && workers_.empty()) return;
      draining_ = true;
    }
    work_cv_.notify_all();
    mem_cv_.notify_all();
    for (auto& t : workers_) t.join();
    workers_.clear();
    std::lock_guard<std::mutex> lk(mu_);
    stop_ = true;
  }

 private:
  void complete(Request* r, int status) {
    r->status = status;
    r->t_done = Clock::now();
    r->done = true;
    stats_.inflight_bytes -= r->mem;
    if (status == SERVE_EXPIRED) ++stats_.expired;
    ++stats_.completed;
  }

  void worker(int slot) {
    std::vector<Request*> batch;
    while (true) {
      batch.clear();
      {
        std::unique_lock<std::mutex> lk(mu_);
        work_cv_.wait(lk, [&] { return draining_ || !queue_.empty(); });
        if (queue_.empty() && draining_) return;
        int64_t hits = 0;
        const Clock::time_point now = Clock::now();
        bool freed = false;
        while (!queue_.empty() && (int)batch.size() < max_events_) {
          Request* r = queue_.front();
          if (r->has_deadline && now > r->deadline) {
            queue_.pop_front();
            complete(r, SERVE_EXPIRED);
            freed = true;
            continue;
          }
          if (!batch.empty() && hits + r->n > max_hits_) break;
          queue_.pop_front();
          hits += r->n;
          r->t_start = now;
          batch.push_back(r);
        }
        if (freed) {
          done_cv_.notify_all();
          mem_cv_.notify_all();
        }
        if (!queue_.empty()) work_cv_.notify_one();
        if (batch.empty()) continue;
        ++stats_.batches;
        stats_.batched_events += (int64_t)batch.size();
      }
      const int rc = exec_->run(slot, batch);
      {
        std::lock_guard<std::mutex> lk(mu_);
        for (Request* r : batch) complete(r, rc == 0 ? r->status : rc);
      }
      done_cv_.notify_all();
      mem_cv_.notify_all();
    }
  }

  Exec* exec_;
  const int max_events_;
  const int64_t max_hits_;
  const uint64_t budget_, per_hit_, per_req_;
  std::mutex mu_;
  std::condition_variable work_cv_, done_cv_, mem_cv_;
  std::deque<Request*> queue_;
  std::unordered_map<int64_t, std::unique_ptr<Request>> table_;
  std::vector<std::thread> workers_;
  Stats stats_;
  int64_t next_id_ = 1;
  bool draining_ = false, stop_ = false;
};

}  // namespace trk_serve
