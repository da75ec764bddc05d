// Out-of-process front end of the serving loop (host only, no HIP): clients
// send events over stream sockets and get the labels back, the analogue of the
// inference server's network protocol (Section 2.3: clients send requests to a
// server that runs them on its coprocessor; Section 4 measures what the transfer
// adds to the latency).  One thread per connection; the requests of a connection
// are served in order, different connections concurrently (they meet in the
// backend's scheduler, which batches them).
//
// Wire format, little-endian, a fixed header then its payload:
//   request : u32 magic 0x5154524B, u32 reserved (0), i64 n, f64 deadline_ms, f32 x[n][3]
//   response: u32 magic 0x5254524B, i32 status, i64 n, f64 latency_ms,
//             i64 counts[5] (hits, candidate, filtered, kept edges, saturated points),
//             f32 stage_ms[8], then i32 labels[n] when status == 0
// latency_ms is the backend's, from submission to completion.  A request with a
// bad magic, n < 0 or n > max_hits gets a response with status -1 (TRK_E_INVAL)
// and no labels, and the connection is closed.
//
// Backend interface:
//   int submit(const float* x, int64_t n, double deadline_ms, int64_t* ticket);
//   int wait(int64_t ticket, int32_t* labels, int64_t* counts5, float* stage8, double* latency_ms);
#pragma once
#include <arpa/inet.h>
#include <netinet/in.h>
#include <netinet/tcp.h>
#include <poll.h>
#include <stdint.h>
#include <string.h>
#include <sys/socket.h>
#include <unistd.h>

#include <atomic>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

namespace trk_net {

constexpr uint32_t REQ_MAGIC = 0x5154524B;
constexpr uint32_t RESP_MAGIC = 0x5254524B;

struct ReqHeader {
  uint32_t magic, reserved;
  int64_t n;
  double deadline_ms;
};
struct RespHeader {
  uint32_t magic;
  int32_t status;
  int64_t n;
  double latency_ms;
  int64_t counts[5];
  float stage_ms[8];
};
static_assert(sizeof(ReqHeader) == 24, "request header layout");
static_assert(sizeof(RespHeader) == 96, "response header layout");

inline bool read_all(int fd, void* p, size_t n) {
  char* c = (char*)p;
  while (n > 0) {
    const ssize_t r = recv(fd, c, n, 0);
    if (r <= 0) return false;
    c += r;
    n -= (size_t)r;
  }
  return true;
}

inline bool write_all(int fd, const void* p, size_t n) {
  const char* c = (const char*)p;
  while (n > 0) {
    const ssize_t r = send(fd, c, n, MSG_NOSIGNAL);
    if (r <= 0) return false;
    c += r;
    n -= (size_t)r;
  }
  return true;
}

template <class Backend>
class Service {
 public:
  Service(Backend* backend, int64_t max_hits) : be_(backend), max_hits_(max_hits) {}
  ~Service() { stop(); }

  // Listens on host:port (port 0: any free port, written to *bound_port);
  // returns 0, or -1 when the address cannot be bound.
  int start(const char* host, int port, int* bound_port) {
    lfd_ = socket(AF_INET, SOCK_STREAM, 0);
    if (lfd_ < 0) return -1;
    const int one = 1;
    setsockopt(lfd_, SOL_SOCKET, SO_REUSEADDR, &one, sizeof(one));
    sockaddr_in a{};
    a.sin_family = AF_INET;
    a.sin_port = htons((uint16_t)port);
    if (inet_pton(AF_INET, host ? host : "127.0.0.1", &a.sin_addr) != 1 || bind(lfd_, (sockaddr*)&a, sizeof(a)) ||
        listen(lfd_, 128)) {
      close(lfd_);
      lfd_ = -1;
      return -1;
    }
    socklen_t len = sizeof(a);
    getsockname(lfd_, (sockaddr*)&a, &len);
    if (bound_port) *bound_port = ntohs(a.sin_port);
    acceptor_ = std::thread([this] { accept_loop(); });
    return 0;
  }

  // Stops accepting, ends every connection (a request being served completes
  // first) and joins the threads.  Idempotent.
  void stop() {
    if (stopping_.exchange(true)) return;
    if (acceptor_.joinable()) acceptor_.join();
    if (lfd_ >= 0) close(lfd_);
    lfd_ = -1;
    std::vector<std::shared_ptr<Conn>> conns;
    {
      std::lock_guard<std::mutex> g(mu_);
      conns = conns_;
    }
    for (auto& c : conns) {
      std::lock_guard<std::mutex> g(c->mu);
      if (c->fd >= 0) shutdown(c->fd, SHUT_RDWR);
    }
    for (auto& c : conns)
      if (c->th.joinable()) c->th.join();
  }

  int64_t served() const { return served_.load(); }

 private:
  struct Conn {
    std::mutex mu;
    int fd = -1;
    std::thread th;
  };

  void accept_loop() {
    while (!stopping_.load()) {
      pollfd p{lfd_, POLLIN, 0};
      if (poll(&p, 1, 50) <= 0 || !(p.revents & POLLIN)) continue;
      const int fd = accept(lfd_, nullptr, nullptr);
      if (fd < 0) continue;
      const int one = 1;
      setsockopt(fd, IPPROTO_TCP, TCP_NODELAY, &one, sizeof(one));
      auto c = std::make_shared<Conn>();
      c->fd = fd;
      std::lock_guard<std::mutex> g(mu_);
      if (stopping_.load()) {
        close(fd);
        break;
      }
      conns_.push_back(c);
      c->th = std::thread([this, c] { serve(c); });
    }
  }

  void serve(std::shared_ptr<Conn> c) {
    const int fd = c->fd;
    std::vector<float> x;
    std::vector<int32_t> labels;
    while (true) {
      ReqHeader q;
      if (!read_all(fd, &q, sizeof(q))) break;
      RespHeader r{};
      r.magic = RESP_MAGIC;
      r.n = q.n;
      if (q.magic != REQ_MAGIC || q.n < 0 || q.n > max_hits_) {
        r.status = -1;
        write_all(fd, &r, sizeof(r));
        // close gracefully: end our side, then discard what the client still sends
        // (for at most about a second), so that the response is not lost to a reset
        shutdown(fd, SHUT_WR);
        char sink[4096];
        for (int k = 0; k < 20 && !stopping_.load(); ++k) {
          pollfd p{fd, POLLIN, 0};
          if (poll(&p, 1, 50) > 0 && recv(fd, sink, sizeof(sink), 0) <= 0) break;
        }
        break;
      }
      x.resize((size_t)q.n * 3);
      if (q.n > 0 && !read_all(fd, x.data(), x.size() * sizeof(float))) break;
      int64_t ticket = 0;
      r.status = be_->submit(x.data(), q.n, q.deadline_ms, &ticket);
      if (r.status == 0) {
        labels.resize((size_t)q.n);
        r.status = be_->wait(ticket, labels.data(), r.counts, r.stage_ms, &r.latency_ms);
      }
      if (!write_all(fd, &r, sizeof(r))) break;
      if (r.status == 0 && q.n > 0 && !write_all(fd, labels.data(), labels.size() * sizeof(int32_t))) break;
      ++served_;
    }
    std::lock_guard<std::mutex> g(c->mu);
    close(c->fd);
    c->fd = -1;
  }

  Backend* be_;
  int64_t max_hits_;
  int lfd_ = -1;
  std::atomic<bool> stopping_{false};
  std::atomic<int64_t> served_{0};
  std::thread acceptor_;
  std::mutex mu_;
  std::vector<std::shared_ptr<Conn>> conns_;
};

}  // namespace trk_net
