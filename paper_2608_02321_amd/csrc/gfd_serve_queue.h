// Request queue of the serving form (gfd_server_*), apart from the device
// work: submitted requests wait in arrival order; a free worker takes every
// waiting request while its batch stays within a GFD count and a byte
// estimate; a worker publishes its batch's results under the queue's one
// mutex, and each finished request goes to exactly one waiter, who then owns
// it.  Plain C++ with no device calls, so that a host-only build can run its
// locking under ThreadSanitizer.
#pragma once

#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "gfd.h"

namespace gfd {

inline int64_t serve_now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

struct ServerReq {
  uint64_t id = 0;
  std::vector<gfd_spec> specs;
  std::vector<gfd_result> res;
  std::vector<int32_t> viol;  // first-K tuples of every GFD of the request
  int64_t est_bytes = 0;      // estimated device bytes of its jobs
  gfd_request_info info{};
  int32_t status = GFD_OK;
  std::string err;
  bool done = false;
  bool claimed = false;  // a waiter holds it
};

struct ServeQueue {
  enum Status { OK = 0, STOPPING, UNKNOWN, CLAIMED, TIMEOUT };

  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<ServerReq*> queue;
  std::unordered_map<uint64_t, ServerReq*> reqs;  // submitted, not yet handed to a waiter
  uint64_t next_id = 1, next_batch = 1;
  bool stop = false;

  ServeQueue() = default;
  ServeQueue(const ServeQueue&) = delete;
  ServeQueue& operator=(const ServeQueue&) = delete;
  // requests nobody waited for; the workers have been joined
  ~ServeQueue() {
    for (auto& kv : reqs) delete kv.second;
  }

  // Queues r (the queue owns it from here) and gives it the next id.
  Status submit(ServerReq* r, uint64_t* id) {
    {
      std::lock_guard<std::mutex> lk(mu);
      if (stop) return STOPPING;
      r->id = next_id++;
      r->info.submit_ns = serve_now_ns();
      reqs[r->id] = r;
      queue.push_back(r);
      *id = r->id;
    }
    cv_work.notify_one();
    return OK;
  }

  // Worker side: waits for requests, then takes those waiting in arrival
  // order while the batch stays within max_gfds GFDs and max_bytes estimated
  // bytes (the first request always).  False once the queue stops and is
  // empty.
  bool take(int64_t max_gfds, int64_t max_bytes, std::vector<ServerReq*>& batch, uint64_t& batch_id) {
    batch.clear();
    std::unique_lock<std::mutex> lk(mu);
    cv_work.wait(lk, [&] { return stop || !queue.empty(); });
    if (queue.empty()) return false;
    int64_t n = 0, bytes = 0;
    while (!queue.empty()) {
      ServerReq* r = queue.front();
      const int64_t rn = (int64_t)r->specs.size();
      if (!batch.empty() && (n + rn > max_gfds || bytes + r->est_bytes > max_bytes)) break;
      batch.push_back(r);
      queue.pop_front();
      n += rn;
      bytes += r->est_bytes;
    }
    batch_id = next_batch++;
    return true;
  }

  // Worker side: fill(b, r) writes the results of request b of the batch
  // under the lock; the requests are then finished and their waiters woken.
  template <class Fill>
  void publish(const std::vector<ServerReq*>& batch, Fill fill) {
    {
      std::lock_guard<std::mutex> lk(mu);
      for (size_t b = 0; b < batch.size(); b++) {
        fill(b, *batch[b]);
        batch[b]->done = true;
      }
    }
    cv_done.notify_all();
  }

  // Client side: waits for request id (timeout_ms < 0: without limit).  On
  // OK the request has left the queue and the caller owns (and deletes) it;
  // on TIMEOUT another wait may follow.
  Status wait(uint64_t id, int32_t timeout_ms, ServerReq*& out) {
    out = nullptr;
    std::unique_lock<std::mutex> lk(mu);
    auto it = reqs.find(id);
    if (it == reqs.end()) return UNKNOWN;
    ServerReq* r = it->second;
    // one waiter at a time: a second one would find the request freed
    if (r->claimed) return CLAIMED;
    r->claimed = true;
    auto ready = [&] { return r->done; };
    if (timeout_ms < 0) {
      cv_done.wait(lk, ready);
    } else if (!cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready)) {
      r->claimed = false;
      return TIMEOUT;
    }
    reqs.erase(id);  // by id: the map may have changed while waiting
    out = r;
    return OK;
  }

  // No more submissions; the workers finish what is queued and return.
  void shutdown() {
    {
      std::lock_guard<std::mutex> lk(mu);
      stop = true;
    }
    cv_work.notify_all();
  }
};

}  // namespace gfd
