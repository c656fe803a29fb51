"""The serving form's request queue under ThreadSanitizer (no GPU).

The queue (csrc/gfd_serve_queue.h) is the serving form's whole shared state:
arrival-order queue, request map, ids, the done/claimed flags and the two
condition variables.  It is built here for the host with -fsanitize=thread
into a program that drives it as gfd_server_* does: three workers take
batches within a GFD and a byte limit and publish results from a stand-in
validator; four client threads submit and wait (blocking, with time-outs,
and a second waiter racing the first for the same request); requests nobody
waits for are freed at shutdown; a submit after shutdown is refused.  The
run must end cleanly, with every result equal to what the stand-in computed
for that request alone, every batch within its limits, and no report."""
import os
import subprocess

import pytest

from paper_2608_02321_amd import build as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SRC = r"""
#include "gfd_serve_queue.h"
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <memory>
#include <random>
#include <thread>

using gfd::ServeQueue;
using gfd::ServerReq;

static uint64_t expect(const gfd_spec& s) {  // what the stand-in validator answers
  return (uint64_t)s.num_vertices * 1000u + (uint64_t)s.vertex_labels[0];
}
static std::atomic<int> failures{0};
static void fail(const char* what, unsigned long long a) {
  std::fprintf(stderr, "FAIL %s %llu\n", what, a);
  failures++;
}

int main() {
  constexpr int WORKERS = 3, CLIENTS = 4, PER_CLIENT = 400, MAX_GFDS = 6;
  constexpr int64_t MAX_BYTES = 1000;
  ServeQueue q;
  std::atomic<int> served{0};
  std::vector<std::thread> workers;
  for (int w = 0; w < WORKERS; w++)
    workers.emplace_back([&, w] {
      std::mt19937 rng(100 + w);
      std::vector<ServerReq*> batch;
      uint64_t bid = 0;
      while (q.take(MAX_GFDS, MAX_BYTES, batch, bid)) {
        int64_t gfds = 0, bytes = 0;
        for (ServerReq* r : batch) {
          gfds += (int64_t)r->specs.size();
          bytes += r->est_bytes;
        }
        if (batch.empty()) fail("empty batch", bid);
        if (batch.size() > 1 && (gfds > MAX_GFDS || bytes > MAX_BYTES)) fail("batch over its limits", bid);
        // the device work, outside the lock: reads only the batch's requests
        std::vector<std::vector<uint64_t>> out(batch.size());
        for (size_t b = 0; b < batch.size(); b++)
          for (const gfd_spec& s : batch[b]->specs) out[b].push_back(expect(s));
        std::this_thread::sleep_for(std::chrono::microseconds(rng() % 300));
        q.publish(batch, [&](size_t b, ServerReq& r) {
          for (size_t i = 0; i < r.specs.size(); i++) r.res[i].match_count = out[b][i];
          r.status = GFD_OK;
          r.info.batch_id = bid;
          r.info.batch_gfds = (int32_t)gfds;
          r.info.batch_requests = (int32_t)batch.size();
          r.info.worker = w;
        });
        served += (int)batch.size();
      }
    });
  std::vector<std::thread> clients;
  for (int c = 0; c < CLIENTS; c++)
    clients.emplace_back([&, c] {
      std::mt19937 rng(7 + c);
      for (int j = 0; j < PER_CLIENT; j++) {
        auto r = std::make_unique<ServerReq>();
        const int n = 1 + (int)(rng() % 4);
        for (int i = 0; i < n; i++) {
          gfd_spec s{};
          s.num_vertices = 2 + (int32_t)(rng() % 7);
          s.vertex_labels[0] = (int32_t)(rng() % 100);
          r->specs.push_back(s);
        }
        r->res.resize(n);
        r->est_bytes = (int64_t)(rng() % 600);
        const std::vector<gfd_spec> specs = r->specs;
        uint64_t id = 0;
        if (q.submit(r.get(), &id) != ServeQueue::OK) { fail("submit", j); return; }
        r.release();
        if (j % 10 == 9) continue;  // never waited for: freed at shutdown
        ServerReq* got = nullptr;
        ServeQueue::Status st;
        if (j % 3 == 0) {
          st = q.wait(id, -1, got);
        } else if (j % 3 == 1) {
          while ((st = q.wait(id, 1, got)) == ServeQueue::TIMEOUT) {}
        } else {
          // a second waiter races this one for the same request: exactly one
          // of them gets it; the other sees it claimed or already gone
          ServerReq* other = nullptr;
          ServeQueue::Status ost = ServeQueue::OK;
          std::thread t([&] { ost = q.wait(id, -1, other); });
          do st = q.wait(id, 0, got); while (st == ServeQueue::TIMEOUT);
          t.join();
          if ((st == ServeQueue::OK) == (ost == ServeQueue::OK)) fail("two waiters, one request", id);
          if (st != ServeQueue::OK) {
            st = ost;
            got = other;
          }
        }
        if (st != ServeQueue::OK || !got) { fail("wait", id); continue; }
        if (got->id != id || !got->done || got->specs.size() != specs.size()) fail("request", id);
        for (size_t i = 0; i < specs.size(); i++)
          if (got->res[i].match_count != expect(specs[i])) fail("result", id);
        ServerReq* again = nullptr;
        if (q.wait(id, 0, again) != ServeQueue::UNKNOWN) fail("waited twice", id);
        delete got;
      }
    });
  for (auto& t : clients) t.join();
  q.shutdown();
  for (auto& t : workers) t.join();
  ServerReq late;
  uint64_t id = 0;
  if (q.submit(&late, &id) != ServeQueue::STOPPING) fail("submit after shutdown", id);
  if (served.load() != CLIENTS * PER_CLIENT) fail("served", (unsigned long long)served.load());
  if (!q.queue.empty()) fail("queue left", q.queue.size());
  std::printf("served %d requests, %d failures\n", served.load(), failures.load());
  return failures.load() ? 1 : 0;
}
"""


# clang's ThreadSanitizer: the one of GCC 11 does not intercept
# pthread_cond_clockwait, which libstdc++'s timed waits call, and then reports
# a double lock at the next wait on that mutex
CLANG = os.path.join(os.path.dirname(os.path.realpath(B.HIPCC)), "..", "llvm", "bin", "clang++")


def test_serve_queue_under_tsan(tmp_path):
    if not os.path.exists(CLANG):
        pytest.skip("clang++ not available")
    src, exe = tmp_path / "serve_queue.cpp", tmp_path / "serve_queue"
    src.write_text(SRC)
    r = subprocess.run([CLANG, "-std=c++17", "-O1", "-g", "-fsanitize=thread", "-pthread",
                        f"-I{os.path.join(ROOT, 'include')}", f"-I{B.CSRC}", str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1:second_deadlock_stack=1")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0 and "ThreadSanitizer" not in r.stderr, (r.stdout + r.stderr)[-4000:]
    assert "served 1600 requests, 0 failures" in r.stdout, r.stdout
