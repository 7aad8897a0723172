// mi_server.cpp -- continuous-batching request loop (include/mi_server.h).
//
// One host thread per server.  Requests wait in a FIFO; whenever a slot (a
// HIP stream) is free the loop admits waiting requests that fit the HBM
// budget next to what is already running and launches them on that slot.
// Batches on different slots run concurrently on the device.
//
// Batch formation uses a cost estimate per request (pair updates at a
// sustained rate plus a launch floor), so that small requests are never tied
// to a large one:
//   - a large request (estimate >= kLargeUs) runs alone, as a plain launch;
//   - consecutive small requests are launched together until their summed
//     estimate reaches kBatchCapUs: up to kPlainBatch of them as plain
//     launches back to back, each completing on its own event, more as one
//     persistent launch that completes as a whole;
//   - with two or more slots, slot 0 runs the large requests, one at a time
//     and first come first served (alone a large request already fills the
//     device; two at once only share it), and the other slots run the small
//     batches; while the head of the queue is a large request waiting for
//     slot 0, small requests behind it may start first.
// Admission against the budget stays first come, first served: a request
// that does not fit waits, and nothing behind it overtakes it.
// While work is in flight the loop polls its events, yielding the CPU between
// polls (a timed wait would oversleep by tens of microseconds).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "mi.h"
#include "mi_host.hpp"
#include "mi_server.h"

namespace {

using Clock = std::chrono::steady_clock;

enum ReqState { kWaiting = 0, kRunning = 1, kDone = 2 };

struct Req {
  mi_problem p;
  size_t bytes = 0;
  double est_us = 0.0;
  Clock::time_point t_submit, t_done;
  int state = kWaiting;
  mi_status status = MI_OK;
};

// Requests launched together on one slot.  A batch of plain launches has one
// event per request (each completes on its own, in stream order); a
// persistent batch has one event for all.
struct Batch {
  std::vector<uint64_t> tickets;
  std::vector<size_t> req_bytes;
  std::vector<hipEvent_t> evs;
  size_t ndone = 0;
  int slot = -1;
  size_t bytes = 0;
  bool large = false;
};

constexpr int kMaxBatch = 256;          // requests launched together at most
constexpr int kPlainBatch = 8;          // batches up to this size run as plain launches
constexpr double kLargeUs = 250.0;      // estimate from which a request runs alone
constexpr double kBatchCapUs = 400.0;   // summed estimate of one batch of small requests

}  // namespace

struct mi_server {
  int dev = 0;
  size_t budget = 0;
  int nslots = 0;
  size_t max_queue = 0;
  std::vector<hipStream_t> streams;
  std::vector<char> slot_busy;
  std::vector<hipEvent_t> free_events;

  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<uint64_t> waiting;
  std::unordered_map<uint64_t, Req> reqs;
  std::vector<Batch> running;
  size_t in_flight = 0;
  uint64_t next_ticket = 1;
  bool stop = false;
  mi_server_stats stats{};
  std::thread th;

  void loop();
  void finish_ticket(Batch& b, size_t k, mi_status st, Clock::time_point now);
  void release_batch(Batch& b);
};

namespace {

// Device memory a request holds while it is admitted.
size_t request_bytes(const mi_problem& p, int64_t ldx) {
  size_t b = (size_t)p.m * (size_t)ldx;
  if (p.out) b += (size_t)p.n * (size_t)p.n * sizeof(float);
  if (p.pairs) b += (size_t)p.pairs_capacity * sizeof(mi_pair) + sizeof(unsigned long long);
  if (p.n11_out) b += (size_t)p.n * (size_t)p.n * sizeof(int32_t);
  if (p.colsum_out) b += (size_t)p.n * sizeof(int32_t);
  if (p.n > 0) {
    const int cfg = p.tile == MI_TILE_256 ? 1 : 0;
    mi::Plan pl = mi::make_plan(p.m, p.n, p.tile == 0 ? (p.n >= 1536 ? 1 : 0) : cfg, 2);
    b += mi::workspace_bytes(pl);  // the most any plan of this shape uses
    if (mi::converts_to_fp4(&p))    // the FP4 copy of X (an unaligned X needs no repack then)
      b += (size_t)p.m * (size_t)mi::packed_pitch((p.n + 1) / 2);
    else if (!mi::is_aligned(p.X, ldx))
      b += (size_t)p.m * (size_t)mi::packed_pitch(p.n);
  }
  return b;
}

double seconds(Clock::duration d) { return std::chrono::duration<double>(d).count(); }

// Device time of a request alone, in microseconds: a launch floor, the pair
// updates m n (n+1) / 2 at a sustained 1e15 per second, and the n^2 FP32
// output at 4 TB/s.  Only the ratio between requests matters for batching.
double estimate_us(const mi_problem& p) {
  const double n = (double)p.n, m = (double)p.m;
  return 10.0 + m * n * (n + 1.0) / 2.0 / 1.0e9 + 4.0 * n * n / 4.0e6;
}

}  // namespace

void mi_server::finish_ticket(Batch& b, size_t k, mi_status st, Clock::time_point now) {
  auto it = reqs.find(b.tickets[k]);
  if (it != reqs.end()) {
    it->second.state = kDone;
    it->second.status = st;
    it->second.t_done = now;
  }
  stats.completed++;
  in_flight -= b.req_bytes[k];
  stats.bytes_in_flight = in_flight;
}

void mi_server::release_batch(Batch& b) {
  slot_busy[b.slot] = 0;
  for (hipEvent_t ev : b.evs) free_events.push_back(ev);
  b.evs.clear();
}

void mi_server::loop() {
  (void)hipSetDevice(dev);
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    bool progressed = false;
    // 1. Completed requests (in stream order within a batch).
    const auto now = Clock::now();
    for (size_t i = 0; i < running.size();) {
      Batch& b = running[i];
      const bool one_event = b.evs.size() == 1 && b.tickets.size() > 1;
      while (b.ndone < b.tickets.size()) {
        const hipError_t e = hipEventQuery(one_event ? b.evs[0] : b.evs[b.ndone]);
        if (e == hipErrorNotReady) break;
        const mi_status st = e == hipSuccess ? MI_OK : MI_ERR_DEVICE;
        if (one_event) {
          for (size_t k = b.ndone; k < b.tickets.size(); ++k) finish_ticket(b, k, st, now);
          b.ndone = b.tickets.size();
        } else {
          finish_ticket(b, b.ndone++, st, now);
        }
        progressed = true;
      }
      if (b.ndone == b.tickets.size()) {
        release_batch(b);
        running.erase(running.begin() + i);
      } else {
        ++i;
      }
    }
    if (progressed) cv_done.notify_all();

    // 2. Admission onto one free slot (see the policy at the top of this file).
    // With two or more slots, slot 0 runs large requests and the others
    // batches of small ones; with one slot it runs both.
    const bool split = nslots >= 2;
    int small_slot = -1;
    for (int s = split ? 1 : 0; s < nslots && small_slot < 0; ++s)
      if (!slot_busy[s]) small_slot = s;
    const bool large_free = !slot_busy[0];
    if (!waiting.empty() && (large_free || small_slot >= 0)) {
      Batch b;
      std::vector<mi_problem> probs;
      auto take = [&](std::deque<uint64_t>::iterator it) {
        Req& r = reqs[*it];
        b.bytes += r.bytes;
        b.req_bytes.push_back(r.bytes);
        b.tickets.push_back(*it);
        probs.push_back(r.p);
        r.state = kRunning;
        return waiting.erase(it);
      };
      auto it = waiting.begin();
      const Req& head = reqs[*it];
      const bool head_large = head.est_us >= kLargeUs;
      if (head_large && large_free) {
        if (in_flight + head.bytes <= budget) {  // else it waits for budget, and nothing overtakes it
          take(it);
          b.large = true;
          b.slot = 0;
        }
      } else if (small_slot >= 0 && (!head_large || split)) {
        // Small requests from the head on; a large head waiting for its slot
        // is passed over, any other request that is large or over budget
        // ends the batch.
        b.slot = small_slot;
        double cost = 0.0;
        if (head_large) ++it;
        while (it != waiting.end() && (int)probs.size() < kMaxBatch) {
          const Req& r = reqs[*it];
          if (r.est_us >= kLargeUs) break;
          if (in_flight + b.bytes + r.bytes > budget) break;
          if (!probs.empty() && cost + r.est_us > kBatchCapUs) break;
          cost += r.est_us;
          it = take(it);
        }
      }
      if (!probs.empty()) {
        const int slot = b.slot;
        slot_busy[slot] = 1;
        in_flight += b.bytes;
        stats.bytes_in_flight = in_flight;
        stats.max_bytes_in_flight = std::max(stats.max_bytes_in_flight, in_flight);
        size_t nrun = 0;
        for (auto& rb : running) nrun += rb.tickets.size();
        stats.max_in_flight = std::max<uint64_t>(stats.max_in_flight, nrun + probs.size());
        stats.batches++;
        // A few requests run as plain launches back to back on the slot's
        // stream (no work-list upload), each with its own completion event;
        // more run as one persistent launch.
        const bool plain = (int)probs.size() <= kPlainBatch;
        const size_t nev = plain ? probs.size() : 1;
        mi_status rc = MI_OK;
        while (free_events.size() < nev && rc == MI_OK) {
          hipEvent_t ev = nullptr;
          if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess)
            free_events.push_back(ev);
          else
            rc = MI_ERR_DEVICE;
        }
        for (size_t q = 0; q < nev && rc == MI_OK; ++q) {
          b.evs.push_back(free_events.back());
          free_events.pop_back();
        }
        hipStream_t st = streams[slot];
        size_t launched = 0;  // requests whose launch and event were issued
        lk.unlock();  // launches may allocate; clients can keep submitting
        if (rc == MI_OK) {
          if (plain) {
            for (; launched < probs.size(); ++launched) {
              rc = mi::run_one(&probs[launched], st, 0);
              if (rc == MI_OK && hipEventRecord(b.evs[launched], st) != hipSuccess) rc = MI_ERR_DEVICE;
              if (rc != MI_OK) break;
            }
          } else {
            rc = mi::run_batched(probs.data(), (int64_t)probs.size(), st, MI_BATCH_PERSISTENT);
            if (rc == MI_OK && hipEventRecord(b.evs[0], st) != hipSuccess) rc = MI_ERR_DEVICE;
            if (rc == MI_OK) launched = probs.size();
          }
        }
        lk.lock();
        if (rc == MI_OK) {
          running.push_back(std::move(b));
        } else {
          // Requests launched before the failure complete normally; the
          // failed one and those after it report the error.
          (void)hipStreamSynchronize(st);
          const auto t = Clock::now();
          for (size_t k = 0; k < b.tickets.size(); ++k) finish_ticket(b, k, k < launched ? MI_OK : rc, t);
          release_batch(b);
          cv_done.notify_all();
        }
        progressed = true;
      }
    }

    if (stop && waiting.empty() && running.empty()) break;
    if (!progressed) {
      if (running.empty()) {
        cv_work.wait_for(lk, std::chrono::milliseconds(2));
      } else {
        // Work in flight: poll its events again soon.  A timed wait can
        // oversleep by tens of microseconds, so release the lock and yield.
        lk.unlock();
        std::this_thread::yield();
        lk.lock();
      }
    }
  }
}

extern "C" {

mi_status mi_server_create(mi_server** server, size_t hbm_budget_bytes, int32_t max_slots, int32_t max_queue) {
  mi::clear_error();
  if (!server) return mi::fail(MI_ERR_INVALID_ARG, "server is NULL");
  *server = nullptr;
  if (hbm_budget_bytes == 0) return mi::fail(MI_ERR_INVALID_ARG, "budget must be > 0");
  if (max_slots < 1 || max_slots > 64) return mi::fail(MI_ERR_INVALID_ARG, "max_slots must be in 1..64");
  if (max_queue < 0) return mi::fail(MI_ERR_INVALID_ARG, "max_queue must be >= 0");
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  mi_server* s = new mi_server();
  s->dev = dev;
  s->budget = hbm_budget_bytes;
  s->nslots = max_slots;
  s->max_queue = max_queue == 0 ? 65536 : (size_t)max_queue;
  s->slot_busy.assign(max_slots, 0);
  for (int i = 0; i < max_slots; ++i) {
    hipStream_t st = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e != hipSuccess) {
      for (auto x : s->streams) (void)hipStreamDestroy(x);
      delete s;
      return mi::fail(MI_ERR_DEVICE, "hipStreamCreateWithFlags: %s", hipGetErrorString(e));
    }
    s->streams.push_back(st);
  }
  s->th = std::thread([s] { s->loop(); });
  *server = s;
  return MI_OK;
}

mi_status mi_server_submit(mi_server* s, const mi_problem* p, uint64_t* ticket) {
  mi::clear_error();
  if (!s || !ticket) return mi::fail(MI_ERR_INVALID_ARG, "server and ticket must be non-NULL");
  int64_t ldx = 0;
  mi_status st = mi::check_problem(p, &ldx);
  if (st != MI_OK) return st;
  if (p->validate) return mi::fail(MI_ERR_INVALID_ARG, "validate is not supported by the server");
  if (p->algo != MI_ALGO_DENSE) return mi::fail(MI_ERR_INVALID_ARG, "the server takes only the dense algorithm");
  if (p->packed) return mi::fail(MI_ERR_INVALID_ARG, "the server takes only the byte layout");
  Req r;
  r.p = *p;
  r.bytes = request_bytes(*p, ldx);
  r.est_us = estimate_us(*p);
  r.t_submit = Clock::now();
  std::lock_guard<std::mutex> lk(s->mu);
  if (r.bytes > s->budget) {
    s->stats.rejected++;
    return mi::fail(MI_ERR_BUDGET, "request needs %zu bytes, budget is %zu", r.bytes, s->budget);
  }
  if (s->waiting.size() >= s->max_queue) {
    s->stats.rejected++;
    return mi::fail(MI_ERR_QUEUE_FULL, "queue holds %zu waiting requests", s->waiting.size());
  }
  if (s->stop) return mi::fail(MI_ERR_INVALID_ARG, "server is shutting down");
  const uint64_t t = s->next_ticket++;
  s->reqs.emplace(t, r);
  s->waiting.push_back(t);
  s->stats.submitted++;
  *ticket = t;
  s->cv_work.notify_one();
  return MI_OK;
}

mi_status mi_server_poll(mi_server* s, uint64_t ticket) {
  mi::clear_error();
  if (!s) return mi::fail(MI_ERR_INVALID_ARG, "server is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return mi::fail(MI_ERR_UNKNOWN_TICKET, "unknown ticket %llu", (unsigned long long)ticket);
  return it->second.state == kDone ? MI_OK : MI_ERR_NOT_READY;
}

mi_status mi_server_wait(mi_server* s, uint64_t ticket, double timeout_s, double* latency_s) {
  mi::clear_error();
  if (!s) return mi::fail(MI_ERR_INVALID_ARG, "server is NULL");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return mi::fail(MI_ERR_UNKNOWN_TICKET, "unknown ticket %llu", (unsigned long long)ticket);
  const auto deadline = Clock::now() + std::chrono::duration_cast<Clock::duration>(std::chrono::duration<double>(
                                           timeout_s > 0 ? timeout_s : 1e9));
  while (it->second.state != kDone) {
    if (s->cv_done.wait_until(lk, deadline) == std::cv_status::timeout && it->second.state != kDone)
      return mi::fail(MI_ERR_TIMEOUT, "ticket %llu not finished", (unsigned long long)ticket);
    it = s->reqs.find(ticket);
  }
  const Req r = it->second;
  s->reqs.erase(it);
  if (latency_s) *latency_s = seconds(r.t_done - r.t_submit);
  if (r.status != MI_OK) return mi::fail(r.status, "request %llu failed on the device", (unsigned long long)ticket);
  return MI_OK;
}

mi_status mi_server_get_stats(mi_server* s, mi_server_stats* out) {
  mi::clear_error();
  if (!s || !out) return mi::fail(MI_ERR_INVALID_ARG, "server and stats must be non-NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->stats;
  return MI_OK;
}

mi_status mi_server_destroy(mi_server* s) {
  mi::clear_error();
  if (!s) return mi::fail(MI_ERR_INVALID_ARG, "server is NULL");
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  if (s->th.joinable()) s->th.join();
  for (auto st : s->streams) {
    (void)hipStreamSynchronize(st);
    mi::release_stream_resources(st);
    (void)hipStreamDestroy(st);
  }
  for (auto ev : s->free_events) (void)hipEventDestroy(ev);
  delete s;
  return MI_OK;
}

}  // extern "C"
