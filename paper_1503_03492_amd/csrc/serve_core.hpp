// serve_core.hpp -- continuous-batching scheduler of the projection server.
//
// Plain C++17 (threads, no HIP): the device work sits behind `Backend`, so
// the scheduling logic -- tickets, a bounded FIFO queue, admission by memory
// footprint, retirement, failure propagation -- is the same code whether the
// backend runs HIP kernels or (in the CPU test harness) a stand-in.
//
// One scheduler thread owns the backend.  It admits queued requests while a
// slot is free and their footprint fits the budget, runs one sweep over all
// admitted requests, and retires the ones the backend reports finished.
// Requests that arrive while others are running join at the next sweep:
// that is the continuous batching.  submit() and poll() may be called from
// any thread.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "smre.h"

namespace smre_serve {

inline double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct Request {
  uint64_t ticket = 0;
  int H = 0, W = 0;
  std::vector<float> in;        // host copy of the input (taken at submit)
  std::vector<int32_t> sides;
  std::vector<double> r2;
  double tol = 0;
  int max_sweeps = 0;
  size_t footprint = 0;         // device bytes while admitted
  std::vector<float> out;       // result, filled at retirement
  smre_report rep{};
  int status = SMRE_PENDING;    // PENDING until retired
  int failed_alone = 0;         // set by retire: this request's result is bad (its status)
  double t_submit = 0, t_admit = 0, t_done = 0;
  int slot = -1;
};

// What the scheduler needs from a device.
class Backend {
 public:
  virtual ~Backend() {}
  virtual int slots() const = 0;                      // requests on the device at once
  virtual size_t budget() const = 0;                  // device bytes for requests
  virtual size_t footprint(const Request& r) const = 0;
  // Set up request r in slot s (copy input, zero state).  SMRE_ENOMEM means
  // "not now" (fragmentation); other errors fail the request.
  virtual int admit(Request& r, int s) = 0;
  // One sweep over all admitted slots; appends the slots found finished.
  // An error fails the whole server.
  virtual int step(std::vector<int>& finished) = 0;
  // Copy the result of slot s into r (out, rep) and free the slot.  An error
  // return fails the whole server; a failure of this request alone is
  // reported through r.failed_alone.
  virtual int retire(Request& r, int s) = 0;
};

struct Stats {
  int64_t submitted = 0, completed = 0, rejected = 0, failed = 0;
  int64_t active = 0, queued = 0, sweeps = 0;
  size_t bytes_in_use = 0;
  int64_t peak_active = 0;     // most requests on the device at once
  int64_t joined_running = 0;  // admissions while other requests were mid-solve
};

class Server {
 public:
  Server(std::unique_ptr<Backend> be, int queue_cap)
      : be_(std::move(be)), queue_cap_(queue_cap), slot_req_(be_->slots(), nullptr) {
    worker_ = std::thread([this] { loop(); });
  }
  ~Server() {
    {
      std::lock_guard<std::mutex> g(mu_);
      stop_ = true;
    }
    cv_.notify_all();
    worker_.join();
  }

  int submit(const float* x, int H, int W, const smre_params* p, uint64_t* ticket) {
    if (!x || !p || !ticket || H < 1 || W < 1 || !p->sides || !p->radius2 || p->n_sides < 1)
      return SMRE_EINVAL;
    auto r = std::make_shared<Request>();
    r->H = H;
    r->W = W;
    r->sides.assign(p->sides, p->sides + p->n_sides);
    r->r2.assign(p->radius2, p->radius2 + p->n_sides);
    r->tol = p->tol;
    r->max_sweeps = p->max_sweeps;
    for (int k = 0; k < p->n_sides; ++k)
      if (r->sides[k] < 1 || r->sides[k] > H || r->sides[k] > W || !(r->r2[k] > 0))
        return SMRE_EINVAL;
    if (p->max_sweeps < 1) return SMRE_EINVAL;
    r->footprint = be_->footprint(*r);
    if (r->footprint == 0) return SMRE_EINVAL;
    if (r->footprint > be_->budget()) {
      std::lock_guard<std::mutex> g(mu_);
      stats_.rejected++;
      return SMRE_ETOOBIG;
    }
    r->in.assign(x, x + (size_t)H * W);
    for (float v : r->in)
      if (!(v - v == 0.0f)) return SMRE_ENONFINITE;
    {
      std::lock_guard<std::mutex> g(mu_);
      if (failed_) return failed_;
      if ((int)queue_.size() >= queue_cap_) {
        stats_.rejected++;
        return SMRE_EBUSY;
      }
      r->ticket = ++next_ticket_;
      r->t_submit = now_s();
      tickets_[r->ticket] = r;
      queue_.push_back(r);
      stats_.submitted++;
      *ticket = r->ticket;
    }
    cv_.notify_all();
    return SMRE_OK;
  }

  // OK / NOT_CONVERGED with the result copied out (ticket released), PENDING,
  // or an error (ticket released).
  int poll(uint64_t ticket, float* out, size_t out_elems, smre_report* rep, double* latency) {
    std::lock_guard<std::mutex> g(mu_);
    auto it = tickets_.find(ticket);
    if (it == tickets_.end()) return SMRE_EUNKNOWN_TICKET;
    Request& r = *it->second;
    if (r.status == SMRE_PENDING) return SMRE_PENDING;
    const int st = r.status;
    if (st >= 0) {
      if (!out || out_elems < r.out.size()) return SMRE_EINVAL;
      std::memcpy(out, r.out.data(), r.out.size() * sizeof(float));
      if (rep) *rep = r.rep;
    }
    if (latency) *latency = r.t_done - r.t_submit;
    tickets_.erase(it);
    return st;
  }

  Stats stats() {
    std::lock_guard<std::mutex> g(mu_);
    Stats s = stats_;
    s.queued = (int64_t)queue_.size();
    s.bytes_in_use = used_;
    return s;
  }

 private:
  void finish(Request& r, int status) {  // with mu_ held
    r.status = status;
    r.t_done = now_s();
    if (status >= 0) stats_.completed++;
    else stats_.failed++;
  }

  void fail_all(int code) {  // with mu_ held
    failed_ = code;
    for (auto& r : queue_) finish(*r, code);
    queue_.clear();
    for (auto& p : slot_req_)
      if (p) {
        finish(*p, code);
        p = nullptr;
      }
    stats_.active = 0;
  }

  void loop() {
    std::vector<int> fin;
    for (;;) {
      {
        std::unique_lock<std::mutex> lk(mu_);
        cv_.wait(lk, [this] { return stop_ || (!failed_ && (active_ > 0 || !queue_.empty())); });
        if (stop_) {
          fail_all(SMRE_ECANCELLED);
          return;
        }
        // admission, FIFO: the head waits until it fits
        while (!queue_.empty()) {
          auto r = queue_.front();
          int s = -1;
          for (int k = 0; k < (int)slot_req_.size(); ++k)
            if (!slot_req_[k]) {
              s = k;
              break;
            }
          if (s < 0 || used_ + r->footprint > be_->budget()) break;
          lk.unlock();
          const int rc = be_->admit(*r, s);
          lk.lock();
          if (rc == SMRE_ENOMEM && active_ > 0) break;  // fragmented: wait for a retirement
          queue_.pop_front();
          if (rc != SMRE_OK) {
            finish(*r, rc == SMRE_ENOMEM ? SMRE_ETOOBIG : rc);
            if (rc == SMRE_EDEVICE) {
              fail_all(rc);
              break;
            }
            continue;
          }
          r->slot = s;
          r->t_admit = now_s();
          slot_req_[s] = r;
          used_ += r->footprint;
          if (active_ > 0) stats_.joined_running++;
          ++active_;
          stats_.active = active_;
          if (active_ > stats_.peak_active) stats_.peak_active = active_;
        }
        if (active_ == 0 || failed_) continue;
      }
      fin.clear();
      const int rc = be_->step(fin);
      std::lock_guard<std::mutex> g(mu_);
      stats_.sweeps++;
      if (rc < 0) {
        fail_all(rc);
        active_ = 0;
        used_ = 0;
        continue;
      }
      for (int s : fin) {
        auto r = slot_req_[s];
        if (!r) continue;
        const int rr = be_->retire(*r, s);
        if (rr < 0) {
          finish(*r, rr);
          fail_all(rr);
          active_ = 0;
          used_ = 0;
          break;
        }
        finish(*r, r->failed_alone ? r->failed_alone
                                   : r->rep.converged || r->tol <= 0 ? SMRE_OK
                                                                     : SMRE_NOT_CONVERGED);
        slot_req_[s] = nullptr;
        used_ -= r->footprint;
        --active_;
        stats_.active = active_;
      }
    }
  }

  std::unique_ptr<Backend> be_;
  int queue_cap_;
  std::mutex mu_;
  std::condition_variable cv_;
  std::deque<std::shared_ptr<Request>> queue_;
  std::map<uint64_t, std::shared_ptr<Request>> tickets_;
  std::vector<std::shared_ptr<Request>> slot_req_;
  uint64_t next_ticket_ = 0;
  size_t used_ = 0;
  int active_ = 0;
  int failed_ = 0;
  bool stop_ = false;
  Stats stats_;
  std::thread worker_;
};

}  // namespace smre_serve
