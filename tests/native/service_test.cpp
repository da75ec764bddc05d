// CPU test of the socket front end (service_core.h) over the serving scheduler
// (serve_core.h) with a sleeping test double as executor: many client
// connections with requests of random sizes, protocol errors, shutdown with open
// connections.  Built and run under ThreadSanitizer and AddressSanitizer by
// tests/test_service.py; with --serve it listens on a free port (printed on the
// first line of stdout) until stdin closes, for the Python client's test.
#include <arpa/inet.h>
#include <netinet/in.h>
#include <stdio.h>
#include <string.h>
#include <sys/socket.h>
#include <unistd.h>

#include <atomic>
#include <chrono>
#include <random>
#include <thread>
#include <vector>

#include "../../paper_2501_05520_amd/csrc/serve_core.h"
#include "../../paper_2501_05520_amd/csrc/service_core.h"

using namespace trk_serve;
using namespace trk_net;

static std::atomic<int> failures{0};
#define CHECK(c)                                                        \
  do {                                                                  \
    if (!(c)) {                                                         \
      fprintf(stderr, "CHECK failed at line %d: %s\n", __LINE__, #c);   \
      ++failures;                                                       \
    }                                                                   \
  } while (0)

// label of hit i = its first coordinate, so a client can check routing
struct SleepExec {
  int run(int, std::vector<Request*>& batch) {
    std::this_thread::sleep_for(std::chrono::microseconds(300));
    for (Request* r : batch) {
      r->labels.resize(r->n);
      for (int64_t i = 0; i < r->n; ++i) r->labels[i] = (int32_t)r->x[3 * i];
      r->counts[0] = r->n;
      r->status = SERVE_OK;
    }
    return 0;
  }
};

struct SchedBackend {
  Server<SleepExec>* s;
  int submit(const float* x, int64_t n, double d, int64_t* t) { return s->submit(x, n, d, t); }
  int wait(int64_t t, int32_t* l, int64_t* c, float* st, double* lat) { return s->wait(t, l, c, st, lat); }
};

static int connect_to(int port) {
  const int fd = socket(AF_INET, SOCK_STREAM, 0);
  sockaddr_in a{};
  a.sin_family = AF_INET;
  a.sin_port = htons((uint16_t)port);
  inet_pton(AF_INET, "127.0.0.1", &a.sin_addr);
  if (connect(fd, (sockaddr*)&a, sizeof(a))) {
    close(fd);
    return -1;
  }
  return fd;
}

// one request; returns the status (-100 on a transport failure)
static int request(int fd, const std::vector<float>& x, std::vector<int32_t>& labels, int64_t* n_hits,
                   uint32_t magic = REQ_MAGIC, int64_t n_override = -2) {
  ReqHeader q{magic, 0, n_override == -2 ? (int64_t)(x.size() / 3) : n_override, 0.0};
  if (!write_all(fd, &q, sizeof(q))) return -100;
  if (n_override == -2 && !x.empty() && !write_all(fd, x.data(), x.size() * sizeof(float))) return -100;
  RespHeader r;
  if (!read_all(fd, &r, sizeof(r)) || r.magic != RESP_MAGIC) return -100;
  if (n_hits) *n_hits = r.counts[0];
  if (r.status == 0) {
    labels.resize((size_t)r.n);
    if (r.n > 0 && !read_all(fd, labels.data(), labels.size() * sizeof(int32_t))) return -100;
  }
  return r.status;
}

static std::vector<float> make_x(int64_t n, int tag) {
  std::vector<float> x(3 * n);
  for (int64_t i = 0; i < n; ++i) x[3 * i] = (float)(tag * 1000 + (i % 1000));
  return x;
}

static void clients_and_errors(Service<SchedBackend>& svc, int port) {
  std::vector<std::thread> th;
  std::atomic<int> bad{0};
  for (int c = 0; c < 16; ++c)
    th.emplace_back([&, c] {
      const int fd = connect_to(port);
      if (fd < 0) { ++bad; return; }
      std::mt19937 rng(c);
      for (int k = 0; k < 25; ++k) {
        const int64_t n = rng() % 500;   // includes empty requests
        const auto x = make_x(n, (c * 25 + k) % 2000);
        std::vector<int32_t> lab;
        int64_t nh = -1;
        if (request(fd, x, lab, &nh) != 0 || nh != n || (int64_t)lab.size() != n) { ++bad; continue; }
        for (int64_t i = 0; i < n; ++i)
          if (lab[i] != (int32_t)x[3 * i]) { ++bad; break; }
      }
      close(fd);
    });
  for (auto& t : th) t.join();
  CHECK(bad == 0);
  CHECK(svc.served() == 16 * 25);
  // protocol errors: status -1, then the service closes the connection
  std::vector<int32_t> lab;
  int fd = connect_to(port);
  CHECK(request(fd, make_x(4, 1), lab, nullptr, 0xdeadbeef) == -1);
  char b;
  CHECK(recv(fd, &b, 1, 0) == 0);
  close(fd);
  fd = connect_to(port);
  CHECK(request(fd, {}, lab, nullptr, REQ_MAGIC, 100000) == -1);   // beyond max_hits
  close(fd);
  fd = connect_to(port);
  CHECK(request(fd, {}, lab, nullptr, REQ_MAGIC, -5) == -1);
  close(fd);
}

int main(int argc, char** argv) {
  SleepExec ex;
  Server<SleepExec> sched(&ex, 2, 8, 4000, 1ull << 40, 16, 64);
  SchedBackend be{&sched};
  Service<SchedBackend> svc(&be, 4000);
  int port = 0;
  if (svc.start("127.0.0.1", 0, &port) != 0 || port <= 0) {
    fprintf(stderr, "cannot listen\n");
    return 1;
  }
  if (argc > 1 && !strcmp(argv[1], "--serve")) {
    printf("%d\n", port);
    fflush(stdout);
    char buf[64];
    while (fread(buf, 1, sizeof(buf), stdin) > 0) {}
    svc.stop();
    return 0;
  }
  clients_and_errors(svc, port);
  // shutdown with a connection still open and idle
  const int idle = connect_to(port);
  CHECK(idle >= 0);
  std::this_thread::sleep_for(std::chrono::milliseconds(100));
  svc.stop();
  if (idle >= 0) close(idle);
  sched.shutdown();
  if (failures == 0) printf("all checks passed\n");
  return failures == 0 ? 0 : 1;
}
