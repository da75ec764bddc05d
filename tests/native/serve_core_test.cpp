// CPU test of the serving scheduler (serve_core.h) with a sleeping test double
// as executor: admission by memory, batching limits, deadlines, draining on
// shutdown, many client threads.  Built and run under ThreadSanitizer and
// AddressSanitizer by tests/test_serve_core.py.
#include <stdio.h>
#include <stdlib.h>

#include <atomic>
#include <chrono>
#include <random>
#include <thread>
#include <vector>

#include "../../paper_2501_05520_amd/csrc/serve_core.h"

using namespace trk_serve;

static int failures = 0;
#define CHECK(c)                                                        \
  do {                                                                  \
    if (!(c)) {                                                         \
      fprintf(stderr, "CHECK failed at line %d: %s\n", __LINE__, #c);   \
      ++failures;                                                       \
    }                                                                   \
  } while (0)

struct SleepExec {
  int max_events, us_per_batch;
  int64_t max_hits;
  std::atomic<int> running{0}, max_running{0}, bad_batches{0};
  int run(int, std::vector<Request*>& batch) {
    const int now = ++running;
    int prev = max_running.load();
    while (now > prev && !max_running.compare_exchange_weak(prev, now)) {}
    int64_t hits = 0;
    for (Request* r : batch) hits += r->n;
    if ((int)batch.size() > max_events || (batch.size() > 1 && hits > max_hits)) ++bad_batches;
    std::this_thread::sleep_for(std::chrono::microseconds(us_per_batch));
    for (Request* r : batch) {
      r->labels.resize(r->n);
      // label = the first coordinate of each hit, so the caller can check routing
      for (int64_t i = 0; i < r->n; ++i) r->labels[i] = (int32_t)r->x[3 * i];
      r->counts[0] = r->n;
      r->status = SERVE_OK;
    }
    --running;
    return 0;
  }
};

static std::vector<float> make_x(int64_t n, int tag) {
  std::vector<float> x(3 * n);
  for (int64_t i = 0; i < n; ++i) {
    x[3 * i] = (float)(tag * 1000 + (i % 1000));
    x[3 * i + 1] = 0.f;
    x[3 * i + 2] = 0.f;
  }
  return x;
}

static void many_clients() {
  SleepExec ex{8, 200, 2000};
  Server<SleepExec> srv(&ex, 3, 8, 2000, 1ull << 40, 16, 64);
  std::atomic<int> bad{0};
  std::vector<std::thread> th;
  for (int c = 0; c < 32; ++c)
    th.emplace_back([&, c] {
      std::mt19937 rng(c);
      for (int k = 0; k < 40; ++k) {
        const int64_t n = 1 + rng() % 1000;
        const int tag = c * 100 + k;
        auto x = make_x(n, tag % 2000);
        int64_t t = 0;
        if (srv.submit(x.data(), n, 0.0, &t) != SERVE_OK) { ++bad; continue; }
        std::vector<int32_t> lab(n);
        int64_t counts[5];
        double lat = 0;
        if (srv.wait(t, lab.data(), counts, nullptr, &lat) != SERVE_OK) ++bad;
        for (int64_t i = 0; i < n; ++i)
          if (lab[i] != (int32_t)x[3 * i]) { ++bad; break; }
        if (counts[0] != n || lat < 0) ++bad;
      }
    });
  for (auto& t : th) t.join();
  Stats st = srv.stats();
  CHECK(bad == 0);
  CHECK(st.submitted == 32 * 40 && st.completed == 32 * 40);
  CHECK(st.batched_events == 32 * 40);
  CHECK(st.batches < st.batched_events);      // batching happened
  CHECK(ex.bad_batches == 0);
  CHECK(ex.max_running > 1);                  // slots overlapped
  CHECK(st.inflight_bytes == 0);
}

static void memory_admission() {
  // batches of 50 ms and a start gate: all eight submissions land while the first
  // admitted requests still hold the budget, however the threads are scheduled
  SleepExec ex{4, 50000, 100000};
  const uint64_t per_hit = 100, per_req = 0, budget = 3 * 100 * per_hit;  // three 100-hit requests
  Server<SleepExec> srv(&ex, 1, 4, 100000, budget, per_hit, per_req);
  std::vector<std::thread> th;
  std::atomic<int> bad{0}, ready{0};
  for (int c = 0; c < 8; ++c)
    th.emplace_back([&, c] {
      auto x = make_x(100, c);
      ++ready;
      while (ready.load() < 8) std::this_thread::yield();
      int64_t t;
      if (srv.submit(x.data(), 100, 0.0, &t) != SERVE_OK) { ++bad; return; }
      std::vector<int32_t> lab(100);
      if (srv.wait(t, lab.data(), nullptr, nullptr, nullptr) != SERVE_OK) ++bad;
    });
  for (auto& t : th) t.join();
  Stats st = srv.stats();
  CHECK(bad == 0);
  CHECK(st.waited_for_memory > 0);
  CHECK(st.peak_inflight_bytes <= budget);
  CHECK(st.completed == 8);
  // a request whose estimate alone exceeds the budget is refused
  auto big = make_x(400, 1);
  int64_t t;
  CHECK(srv.submit(big.data(), 400, 0.0, &t) == SERVE_CAPACITY);
  CHECK(srv.stats().rejected == 1);
  // and one beyond the batch limit too
  Server<SleepExec> srv2(&ex, 1, 4, 50, 1ull << 30, 1, 1);
  CHECK(srv2.submit(big.data(), 400, 0.0, &t) == SERVE_CAPACITY);
  CHECK(srv2.submit(nullptr, 5, 0.0, &t) == SERVE_INVAL);
}

static void deadlines() {
  SleepExec ex{1, 30000, 100000};   // one event per batch, 30 ms each, one slot
  Server<SleepExec> srv(&ex, 1, 1, 100000, 1ull << 30, 1, 1);
  std::vector<int64_t> tickets;
  for (int k = 0; k < 10; ++k) {
    auto x = make_x(10, k);
    int64_t t;
    CHECK(srv.submit(x.data(), 10, 5.0, &t) == SERVE_OK);
    tickets.push_back(t);
  }
  int ok = 0, expired = 0;
  for (int64_t t : tickets) {
    std::vector<int32_t> lab(10);
    const int rc = srv.wait(t, lab.data(), nullptr, nullptr, nullptr);
    ok += rc == SERVE_OK;
    expired += rc == SERVE_EXPIRED;
  }
  CHECK(ok >= 1 && expired >= 5 && ok + expired == 10);
  CHECK(srv.stats().expired == expired);
  CHECK(srv.stats().inflight_bytes == 0);
}

static void drain_on_shutdown() {
  SleepExec ex{4, 1000, 100000};
  std::vector<int64_t> tickets;
  auto* srv = new Server<SleepExec>(&ex, 2, 4, 100000, 1ull << 30, 1, 1);
  for (int k = 0; k < 50; ++k) {
    auto x = make_x(20, k);
    int64_t t;
    CHECK(srv->submit(x.data(), 20, 0.0, &t) == SERVE_OK);
    tickets.push_back(t);
  }
  srv->shutdown();                       // runs everything admitted
  Stats st = srv->stats();
  CHECK(st.completed == 50);
  int64_t t;
  auto x = make_x(5, 0);
  CHECK(srv->submit(x.data(), 5, 0.0, &t) == SERVE_SHUTDOWN);
  for (int64_t tk : tickets) CHECK(srv->wait(tk, nullptr, nullptr, nullptr, nullptr) == SERVE_OK);
  CHECK(srv->wait(tickets[0], nullptr, nullptr, nullptr, nullptr) == SERVE_INVAL);  // released
  delete srv;
}

int main() {
  many_clients();
  memory_admission();
  deadlines();
  drain_on_shutdown();
  if (failures) {
    fprintf(stderr, "%d check(s) failed\n", failures);
    return 1;
  }
  printf("serve_core: all checks passed\n");
  return 0;
}
