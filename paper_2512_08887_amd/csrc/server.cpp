// Continuous-batching block server over resident plans (fbst_server_* in
// include/fbst.h).
//
// Requests (plan, x, beams) are queued by any thread.  One scheduler thread
// owns the device side: whenever one of its launch streams is idle it takes
// the oldest queued request, gathers up to max_batch queued requests of the
// same plan (in arrival order), reserves their workspace from the server's
// budget (admission by memory: a launch starts only when its workspace fits),
// and launches the whole path for that batch with per-block input/output
// pointers.  Launches on different streams overlap on the GPU; requests that
// arrive while others run join the next launch boundary.  A launch's
// completion (polled with a stream event) releases its workspace and reports
// each request's submit / launch / completion times.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <list>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "kernels.h"
#include "plan.h"

namespace {

using clk = std::chrono::steady_clock;

struct Request {
  const fbst_plan* plan;
  const void* x;
  void* beams;
  unsigned long long tag;
  double submit_us;
};

struct Launch {
  int stream = -1;
  hipEvent_t done = nullptr;
  size_t ws_off = 0, ws_len = 0;
  double start_us = 0;
  std::vector<Request> reqs;
};

// First-fit allocator over [0, size) with 256-byte granules.
class RangeAlloc {
 public:
  explicit RangeAlloc(size_t size) { free_.push_back({0, size}); }
  bool alloc(size_t len, size_t* off) {
    len = (len + 255) & ~static_cast<size_t>(255);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= len) {
        *off = it->first;
        it->first += len;
        it->second -= len;
        if (it->second == 0) free_.erase(it);
        return true;
      }
    }
    return false;
  }
  size_t largest() const {
    size_t m = 0;
    for (const auto& r : free_) m = std::max(m, r.second);
    return m;
  }
  void release(size_t off, size_t len) {
    len = (len + 255) & ~static_cast<size_t>(255);
    auto it = free_.begin();
    while (it != free_.end() && it->first < off) ++it;
    it = free_.insert(it, {off, len});
    // merge with the next and previous ranges
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }

 private:
  std::list<std::pair<size_t, size_t>> free_;
};

}  // namespace

struct fbst_server {
  int device = 0;
  int max_batch = 16;
  size_t ws_size = 0;
  void* ws = nullptr;
  std::vector<hipStream_t> streams;
  std::vector<bool> busy;
  RangeAlloc* pool = nullptr;
  clk::time_point t0;

  std::mutex mu;
  std::condition_variable cv, idle_cv;
  std::deque<Request> queue;
  std::vector<fbst_completion> done;
  std::vector<Launch> inflight;
  bool stop = false;
  int staging = 0;          // launches taken off the queue but not yet in flight
  std::string error;
  std::thread worker;

  bool idle() const { return queue.empty() && inflight.empty() && staging == 0; }

  double now_us() const {
    return std::chrono::duration<double, std::micro>(clk::now() - t0).count();
  }

  void complete(Launch& l, int status, double t) {
    for (const Request& r : l.reqs) {
      fbst_completion c{};
      c.tag = r.tag;
      c.status = status;
      c.submit_us = r.submit_us;
      c.start_us = l.start_us;
      c.done_us = t;
      c.batch = static_cast<int>(l.reqs.size());
      done.push_back(c);
    }
  }

  // One scheduling round; called with mu held.  Returns true if it did anything.
  bool step(std::unique_lock<std::mutex>& lk) {
    bool acted = false;
    // retire finished launches
    for (size_t i = 0; i < inflight.size();) {
      Launch& l = inflight[i];
      const hipError_t q = hipEventQuery(l.done);
      if (q == hipErrorNotReady) {
        ++i;
        continue;
      }
      const double t = now_us();
      complete(l, q == hipSuccess ? FBST_OK : FBST_E_DEVICE, t);
      pool->release(l.ws_off, l.ws_len);
      busy[l.stream] = false;
      (void)hipEventDestroy(l.done);
      inflight.erase(inflight.begin() + static_cast<long>(i));
      acted = true;
    }
    // start launches on idle streams
    while (!queue.empty()) {
      int s = -1;
      for (size_t i = 0; i < busy.size(); ++i)
        if (!busy[i]) {
          s = static_cast<int>(i);
          break;
        }
      if (s < 0) break;
      const fbst_plan* plan = queue.front().plan;
      // workspace of n blocks: n per + fixed (fixed: the split float64 stage 2's scratch)
      const size_t per = plan->ws_bytes_per_block, fixed = plan->ws_fixed_bytes;
      // gather same-plan requests in arrival order
      std::vector<size_t> pick;
      for (size_t i = 0; i < queue.size() && static_cast<int>(pick.size()) < max_batch; ++i)
        if (queue[i].plan == plan) pick.push_back(i);
      size_t off = 0;
      // as many of them as the largest free workspace range holds
      const size_t room = pool->largest();
      int n = room < fixed ? 0
                           : static_cast<int>(std::min<size_t>(
                                 pick.size(), per ? (room - fixed) / per : pick.size()));
      while (n > 0 && !pool->alloc(per * static_cast<size_t>(n) + fixed, &off)) --n;
      if (n == 0) {
        if (inflight.empty()) {
          // the budget cannot hold even one block of this plan: fail the request
          Launch l;
          l.reqs.push_back(queue.front());
          l.start_us = now_us();
          complete(l, FBST_E_NOMEM, l.start_us);
          queue.pop_front();
          acted = true;
          continue;
        }
        break;   // wait for workspace to be released
      }
      pick.resize(static_cast<size_t>(n));
      Launch l;
      l.stream = s;
      l.ws_off = off;
      l.ws_len = per * static_cast<size_t>(n) + fixed;
      fbst::InPtrs xs{};
      fbst::OutPtrs outs{};
      for (int i = 0; i < n; ++i) {
        const Request& r = queue[pick[static_cast<size_t>(i)]];
        xs.p[i] = r.x;
        outs.p[i] = r.beams;
        l.reqs.push_back(r);
      }
      for (int i = n - 1; i >= 0; --i) queue.erase(queue.begin() + static_cast<long>(pick[static_cast<size_t>(i)]));
      ++staging;
      lk.unlock();   // launching does not touch the queue
      l.start_us = now_us();
      hipError_t e = fbst::run_blocks(plan, n, xs, outs, static_cast<unsigned char*>(ws) + off,
                                      streams[static_cast<size_t>(s)]);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&l.done, hipEventDisableTiming);
      if (e == hipSuccess) e = hipEventRecord(l.done, streams[static_cast<size_t>(s)]);
      lk.lock();
      --staging;
      if (e != hipSuccess) {
        error = std::string("launch failed: ") + hipGetErrorString(e);
        if (l.done) (void)hipEventDestroy(l.done);
        complete(l, FBST_E_DEVICE, now_us());
        pool->release(l.ws_off, l.ws_len);
      } else {
        busy[static_cast<size_t>(s)] = true;
        inflight.push_back(std::move(l));
      }
      acted = true;
    }
    if (idle()) idle_cv.notify_all();
    return acted;
  }

  void run() {
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    while (!stop) {
      const bool acted = step(lk);
      if (!acted) {
        if (inflight.empty())
          cv.wait_for(lk, std::chrono::milliseconds(5));
        else {
          lk.unlock();
          std::this_thread::sleep_for(std::chrono::microseconds(5));
          lk.lock();
        }
      }
    }
    // requests never launched are reported as cancelled
    for (const Request& r : queue) {
      Launch l;
      l.reqs.push_back(r);
      l.start_us = now_us();
      complete(l, FBST_E_INVALID, l.start_us);
    }
    queue.clear();
    // drain what is still running before the streams go away
    while (!inflight.empty()) {
      step(lk);
      lk.unlock();
      std::this_thread::sleep_for(std::chrono::microseconds(20));
      lk.lock();
    }
  }
};

namespace {
fbst_status sfail(fbst_status st, const std::string& m) {
  fbst::set_last_error(m);
  return st;
}
}  // namespace

extern "C" {

fbst_status fbst_server_create(const fbst_server_options* opt, fbst_server** out) {
  if (!out) return sfail(FBST_E_INVALID, "out is NULL");
  *out = nullptr;
  fbst_server_options o{};
  o.workspace_bytes = static_cast<size_t>(1) << 30;
  o.streams = 4;
  o.max_batch = 16;
  o.device = -1;
  if (opt) o = *opt;
  if (o.workspace_bytes == 0 || o.streams < 1 || o.streams > 16 || o.max_batch < 1 ||
      o.max_batch > fbst::MAX_LAUNCH_BLOCKS)
    return sfail(FBST_E_INVALID, "need workspace_bytes > 0, 1 <= streams <= 16, 1 <= max_batch <= FBST_MAX_LAUNCH_BLOCKS");
  fbst_server* s = new (std::nothrow) fbst_server();
  if (!s) return sfail(FBST_E_NOMEM, "host allocation failed");
  hipError_t e = hipSuccess;
  if (o.device >= 0) e = hipSetDevice(o.device);
  if (e == hipSuccess) e = hipGetDevice(&s->device);
  if (e == hipSuccess) e = hipMalloc(&s->ws, o.workspace_bytes);
  if (e != hipSuccess) {
    delete s;
    (void)hipGetLastError();
    return sfail(FBST_E_NOMEM, std::string("server workspace allocation failed: ") + hipGetErrorString(e));
  }
  s->ws_size = o.workspace_bytes;
  s->max_batch = o.max_batch;
  s->pool = new RangeAlloc(o.workspace_bytes);
  s->streams.resize(static_cast<size_t>(o.streams));
  s->busy.assign(static_cast<size_t>(o.streams), false);
  for (auto& st : s->streams) {
    e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e != hipSuccess) {
      for (auto& q : s->streams)
        if (q) (void)hipStreamDestroy(q);
      (void)hipFree(s->ws);
      delete s->pool;
      delete s;
      return sfail(FBST_E_DEVICE, std::string("stream creation failed: ") + hipGetErrorString(e));
    }
  }
  s->t0 = clk::now();
  s->worker = std::thread([s] { s->run(); });
  *out = s;
  return FBST_OK;
}

fbst_status fbst_server_submit(fbst_server* s, const fbst_plan* plan, const void* x, void* beams,
                               unsigned long long tag) {
  if (!s || !plan || !x || !beams) return sfail(FBST_E_INVALID, "server, plan, x and beams must not be NULL");
  if (plan->host_only || !plan->dev) return sfail(FBST_E_INVALID, "plan was created host-only");
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return sfail(FBST_E_INVALID, "server is shutting down");
    s->queue.push_back(Request{plan, x, beams, tag, s->now_us()});
  }
  s->cv.notify_one();
  return FBST_OK;
}

int fbst_server_poll(fbst_server* s, fbst_completion* out, int max) {
  if (!s || (!out && max > 0) || max < 0) return FBST_E_INVALID;
  std::lock_guard<std::mutex> lk(s->mu);
  const int n = std::min(max, static_cast<int>(s->done.size()));
  for (int i = 0; i < n; ++i) out[i] = s->done[static_cast<size_t>(i)];
  s->done.erase(s->done.begin(), s->done.begin() + n);
  return n;
}

fbst_status fbst_server_drain(fbst_server* s, double timeout_s) {
  if (!s) return sfail(FBST_E_INVALID, "server is NULL");
  std::unique_lock<std::mutex> lk(s->mu);
  const auto pred = [s] { return s->idle(); };
  if (timeout_s <= 0) {
    s->idle_cv.wait(lk, pred);
    return FBST_OK;
  }
  if (!s->idle_cv.wait_for(lk, std::chrono::duration<double>(timeout_s), pred))
    return sfail(FBST_E_DEVICE, "drain timed out");
  return FBST_OK;
}

double fbst_server_clock_us(const fbst_server* s) { return s ? s->now_us() : 0.0; }

void fbst_server_destroy(fbst_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv.notify_all();
  if (s->worker.joinable()) s->worker.join();
  for (auto& st : s->streams) (void)hipStreamDestroy(st);
  (void)hipFree(s->ws);
  delete s->pool;
  delete s;
}

}  // extern "C"
