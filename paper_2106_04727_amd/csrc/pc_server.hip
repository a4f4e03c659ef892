// Serving layer of libparchain.so (declared in include/parchain.h): many
// clustering requests of uneven n, d and linkage on one device.
//
// A server owns `slots` workers. Each worker has its own context (device
// workspace) and HIP stream, so the rounds of the requests it runs overlap on
// the GPU with those of the other workers. Device bytes are accounted per
// slot: an idle slot counts what its context keeps from earlier requests, a
// busy slot its request's reservation (at least that). A waiting request is
// admitted when a worker is free and the reservation it adds (its footprint,
// initially the workspace model of pc_hac_workspace_bytes, less what the
// slot already holds) fits into what is left of the HBM budget; requests
// are taken in arrival order, a later one that fits may start before an
// earlier one that does not (first fit), and a request passed over kMaxBypass
// times stops any further overtaking until it starts. While a request runs,
// its slot's context may not hold more than the reservation; a request that
// needs more (its candidate records grow with the data) stops, goes back to
// the head of the queue with twice the reservation, and runs again when that
// fits (it fails with PC_ERR_OUT_OF_MEMORY once the reservation would exceed
// the whole budget). The computation of a request is pc_hac's, on the same
// inputs, so its rows do not depend on what else runs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/parchain.h"

namespace pc {
size_t context_bytes(const pc_context *c);
void context_trim(pc_context *c);
void context_set_budget(pc_context *c, size_t bytes);
bool context_over_budget(const pc_context *c);
int context_device(const pc_context *c);
void set_error(const char *msg);  // the text pc_last_error() returns on this thread
}  // namespace pc

namespace {

constexpr int kMaxBypass = 16;  // overtakes a waiting request tolerates

enum JobState { kQueued = 0, kRunning = 1, kDone = 2, kCancelled = 3 };

struct Job {
  uint64_t ticket = 0;
  const float *points = nullptr;
  int64_t n = 0;
  int32_t d = 0, linkage = 0;
  pc_options opt{};
  bool has_opt = false;
  pc_merge *out = nullptr;
  uint64_t model = 0;  // pc_hac_workspace_bytes of the request
  uint64_t bytes = 0;  // its reservation (the model, doubled at each requeue)
  int requeues = 0;
  int state = kQueued;
  int slot = -1;
  int bypassed = 0;
  pc_status result = PC_OK;
  double t_submit = 0, t_start = 0, t_done = 0;
  pc_stats stats{};
  std::string error;
};

pc_status sfail(pc_status st, const char *msg) {
  pc::set_error(msg);
  return st;
}

}  // namespace

struct pc_server {
  int device = 0;
  int slots = 4;
  uint64_t budget = 0;
  double fake_us = 0.0;
  double fake_growth = 1.0;  // test mode: a request's device need is model x this
  std::chrono::steady_clock::time_point t0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Job *> queue;
  std::unordered_map<uint64_t, Job *> jobs;
  uint64_t next_ticket = 1;
  std::vector<std::thread> workers;
  std::vector<pc_context *> ctxs;
  std::vector<hipStream_t> streams;
  bool stop = false;
  // in_use = sum over slots of max(held, reserved)
  std::vector<uint64_t> held;      // per slot: bytes its context keeps between requests
  std::vector<uint64_t> reserved;  // per slot: the running request's reservation (0 if idle)
  uint64_t in_use = 0, peak_bytes = 0;
  int running = 0, peak_running = 0;
  int64_t submitted = 0, completed = 0, rejected = 0, cancelled = 0, failed = 0, requeued = 0;

  double now_ms() const {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }

  // bytes a request adds when it starts on `slot`
  uint64_t extra(const Job *j, int slot) const {
    return j->bytes > held[slot] ? j->bytes - held[slot] : 0;
  }

  // first waiting request that fits on `slot`, honouring the overtaking
  // limit; caller holds mu
  Job *pick(int slot) {
    for (size_t i = 0; i < queue.size(); ++i) {
      Job *j = queue[i];
      if (extra(j, slot) <= budget - in_use) {
        for (size_t k = 0; k < i; ++k) ++queue[k]->bypassed;
        queue.erase(queue.begin() + (long)i);
        return j;
      }
      if (j->bypassed >= kMaxBypass) return nullptr;  // nobody may overtake it any more
    }
    return nullptr;
  }

  void work(int slot) {
    if (fake_us <= 0.0) hipSetDevice(device);
    for (;;) {
      Job *j = nullptr;
      uint64_t resv = 0;
      {
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
          if (stop) return;
          j = pick(slot);
          if (j) break;
          if (!queue.empty() && held[slot] > 0) {
            // a waiting request does not fit: this idle slot gives back what
            // its context keeps (the other idle slots do the same on waking)
            in_use -= held[slot];
            held[slot] = 0;
            if (fake_us <= 0.0) pc::context_trim(ctxs[slot]);
            cv_work.notify_all();
            continue;
          }
          cv_work.wait(lk);
        }
        j->state = kRunning;
        j->slot = slot;
        if (j->requeues == 0) j->t_start = now_ms();
        resv = std::max(j->bytes, held[slot]);
        in_use += resv - held[slot];
        reserved[slot] = resv;
        peak_bytes = std::max(peak_bytes, in_use);
        ++running;
        peak_running = std::max(peak_running, running);
      }
      pc_status st = PC_OK;
      bool over = false;
      uint64_t keep = 0;
      if (fake_us > 0.0) {
        // host-only test mode: occupy the slot for a time proportional to n;
        // the request needs model x fake_growth bytes
        const uint64_t need = (uint64_t)((double)j->model * fake_growth);
        if (need > resv) {
          over = true;
          st = PC_ERR_OUT_OF_MEMORY;
          keep = held[slot];
        } else {
          std::this_thread::sleep_for(std::chrono::duration<double, std::micro>(fake_us * (double)j->n / 1000.0));
          for (int64_t r = 0; r + 1 < j->n; ++r) j->out[r] = pc_merge{0, 0, 0.0, 0};
          keep = std::max(need, held[slot]);
        }
      } else {
        j->stats.struct_size = sizeof(pc_stats);
        pc::context_set_budget(ctxs[slot], resv);
        st = pc_hac(ctxs[slot], j->points, j->n, j->d, 0, j->linkage, j->has_opt ? &j->opt : nullptr, j->out, 0,
                    (void *)streams[slot], &j->stats);
        over = st == PC_ERR_OUT_OF_MEMORY && pc::context_over_budget(ctxs[slot]);
        if (st != PC_OK) j->error = pc_last_error();
        keep = pc::context_bytes(ctxs[slot]);
      }
      // keep the slot within its share of the budget
      if (keep > budget / (uint64_t)slots) {
        if (fake_us <= 0.0) pc::context_trim(ctxs[slot]);
        keep = 0;
      }
      {
        std::lock_guard<std::mutex> lk(mu);
        in_use = in_use - resv + keep;
        held[slot] = keep;
        reserved[slot] = 0;
        --running;
        if (over && j->bytes < budget) {
          // needs more than it reserved: back to the head of the queue
          j->bytes = std::min<uint64_t>(2 * resv, budget);
          ++j->requeues;
          ++requeued;
          j->state = kQueued;
          j->slot = -1;
          j->error.clear();
          queue.push_front(j);
        } else {
          j->result = st;
          j->state = kDone;
          j->t_done = now_ms();
          ++completed;
          if (st != PC_OK) ++failed;
        }
      }
      cv_done.notify_all();
      cv_work.notify_all();
    }
  }
};

extern "C" {

pc_status pc_server_create(pc_context *ctx, const pc_server_options *opt, pc_server **out) {
  if (!out) return sfail(PC_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (opt && opt->struct_size < sizeof(pc_server_options))
    return sfail(PC_ERR_INVALID_ARG, "pc_server_options.struct_size too small");
  pc_server *s = new (std::nothrow) pc_server();
  if (!s) return sfail(PC_ERR_OUT_OF_MEMORY, "host allocation failed");
  s->t0 = std::chrono::steady_clock::now();
  s->slots = opt && opt->slots > 0 ? opt->slots : 4;
  if (s->slots > 64) {
    delete s;
    return sfail(PC_ERR_INVALID_ARG, "at most 64 slots");
  }
  s->fake_us = opt ? opt->fake_us_per_kpoint : 0.0;
  s->fake_growth = opt && opt->fake_growth > 0.0 ? opt->fake_growth : 1.0;
  s->budget = opt ? opt->hbm_budget_bytes : 0;
  s->held.assign((size_t)s->slots, 0);
  s->reserved.assign((size_t)s->slots, 0);
  if (s->fake_us > 0.0) {
    if (!s->budget) s->budget = 1ull << 30;
  } else {
    int dev = ctx ? pc::context_device(ctx) : -1;
    if (dev < 0 && hipGetDevice(&dev) != hipSuccess) {
      delete s;
      return sfail(PC_ERR_DEVICE, "hipGetDevice failed");
    }
    s->device = dev;
    if (hipSetDevice(dev) != hipSuccess) {
      delete s;
      return sfail(PC_ERR_INVALID_ARG, "hipSetDevice failed");
    }
    if (!s->budget) {
      size_t fr = 0, tot = 0;
      if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
        delete s;
        return sfail(PC_ERR_DEVICE, "hipMemGetInfo failed");
      }
      s->budget = (uint64_t)(0.8 * (double)fr);
    }
    for (int i = 0; i < s->slots; ++i) {
      pc_context *c = nullptr;
      pc_status st = pc_context_create(dev, 0, &c);
      hipStream_t hs = nullptr;
      if (st == PC_OK && hipStreamCreateWithFlags(&hs, hipStreamNonBlocking) != hipSuccess) st = PC_ERR_DEVICE;
      if (st != PC_OK) {
        if (c) pc_context_destroy(c);
        for (pc_context *x : s->ctxs) pc_context_destroy(x);
        for (hipStream_t x : s->streams) hipStreamDestroy(x);
        delete s;
        return sfail(st, "slot setup failed");
      }
      s->ctxs.push_back(c);
      s->streams.push_back(hs);
    }
  }
  for (int i = 0; i < s->slots; ++i) s->workers.emplace_back([s, i] { s->work(i); });
  *out = s;
  pc::set_error("");
  return PC_OK;
}

pc_status pc_server_submit(pc_server *s, const float *points, int64_t n, int32_t d, int32_t linkage,
                           const pc_options *opt, pc_merge *out, uint64_t *ticket) {
  if (!s || !points || !ticket || (n > 1 && !out)) return sfail(PC_ERR_INVALID_ARG, "NULL argument");
  *ticket = 0;
  if (opt && opt->struct_size < sizeof(pc_options)) return sfail(PC_ERR_INVALID_ARG, "pc_options.struct_size too small");
  const size_t bytes = pc_hac_workspace_bytes(n, d, linkage, opt);
  if (!bytes) return sfail(PC_ERR_INVALID_ARG, "bad n, d or linkage");
  Job *j = new (std::nothrow) Job();
  if (!j) return sfail(PC_ERR_OUT_OF_MEMORY, "host allocation failed");
  j->points = points;
  j->n = n;
  j->d = d;
  j->linkage = linkage;
  if (opt) {
    j->opt = *opt;
    j->has_opt = true;
  }
  j->out = out;
  j->model = bytes;
  j->bytes = bytes;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    ++s->submitted;
    if (bytes > s->budget) {
      ++s->rejected;
      delete j;
      return sfail(PC_ERR_OUT_OF_MEMORY, "request footprint exceeds the server's HBM budget");
    }
    j->ticket = s->next_ticket++;
    j->t_submit = s->now_ms();
    s->jobs[j->ticket] = j;
    s->queue.push_back(j);
    *ticket = j->ticket;
  }
  s->cv_work.notify_one();
  pc::set_error("");
  return PC_OK;
}

static void fill_info(const Job *j, pc_request_info *info) {
  if (!info) return;
  info->status = j->state == kCancelled ? PC_ERR_CANCELLED : j->result;
  info->state = j->state;
  info->slot = j->slot;
  info->footprint_bytes = j->bytes;
  info->t_submit_ms = j->t_submit;
  info->t_start_ms = j->t_start;
  info->t_done_ms = j->t_done;
  info->stats = j->stats;
  const size_t m = std::min(j->error.size(), sizeof(info->error) - 1);
  std::copy(j->error.begin(), j->error.begin() + (long)m, info->error);
  info->error[m] = 0;
}

pc_status pc_server_poll(pc_server *s, uint64_t ticket, int *done, pc_status *result, pc_stats *stats) {
  if (!s) return sfail(PC_ERR_INVALID_ARG, "server is NULL");
  if (stats && stats->struct_size < sizeof(pc_stats))
    return sfail(PC_ERR_INVALID_ARG, "pc_stats.struct_size too small");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->jobs.find(ticket);
  if (it == s->jobs.end()) return sfail(PC_ERR_INVALID_ARG, "unknown ticket");
  const Job *j = it->second;
  const bool fin = j->state == kDone || j->state == kCancelled;
  if (done) *done = fin ? 1 : 0;
  if (result) *result = !fin ? PC_ERR_BUSY : (j->state == kCancelled ? PC_ERR_CANCELLED : j->result);
  if (stats && fin) {
    const uint32_t size = stats->struct_size;
    *stats = j->stats;
    stats->struct_size = size;
  }
  return PC_OK;
}

pc_status pc_server_query(pc_server *s, uint64_t ticket, pc_request_info *info) {
  if (!s) return sfail(PC_ERR_INVALID_ARG, "server is NULL");
  if (info && info->struct_size < sizeof(pc_request_info))
    return sfail(PC_ERR_INVALID_ARG, "pc_request_info.struct_size too small");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->jobs.find(ticket);
  if (it == s->jobs.end()) return sfail(PC_ERR_INVALID_ARG, "unknown ticket");
  fill_info(it->second, info);
  return PC_OK;
}

pc_status pc_server_wait(pc_server *s, uint64_t ticket, double timeout_ms, pc_request_info *info) {
  if (!s) return sfail(PC_ERR_INVALID_ARG, "server is NULL");
  if (info && info->struct_size < sizeof(pc_request_info))
    return sfail(PC_ERR_INVALID_ARG, "pc_request_info.struct_size too small");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->jobs.find(ticket);
  if (it == s->jobs.end()) return sfail(PC_ERR_INVALID_ARG, "unknown ticket");
  Job *j = it->second;
  auto finished = [j] { return j->state == kDone || j->state == kCancelled; };
  if (timeout_ms < 0) {
    s->cv_done.wait(lk, finished);
  } else if (!s->cv_done.wait_for(lk, std::chrono::duration<double, std::milli>(timeout_ms), finished)) {
    fill_info(j, info);
    return sfail(PC_ERR_BUSY, "timed out");
  }
  fill_info(j, info);
  return PC_OK;
}

pc_status pc_server_cancel(pc_server *s, uint64_t ticket) {
  if (!s) return sfail(PC_ERR_INVALID_ARG, "server is NULL");
  {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->jobs.find(ticket);
    if (it == s->jobs.end()) return sfail(PC_ERR_INVALID_ARG, "unknown ticket");
    Job *j = it->second;
    if (j->state == kRunning) return sfail(PC_ERR_BUSY, "request is running");
    if (j->state == kQueued) {
      s->queue.erase(std::find(s->queue.begin(), s->queue.end(), j));
      j->state = kCancelled;
      j->t_done = s->now_ms();
      ++s->cancelled;
    }
  }
  s->cv_done.notify_all();
  s->cv_work.notify_all();
  return PC_OK;
}

pc_status pc_server_release(pc_server *s, uint64_t ticket) {
  if (!s) return sfail(PC_ERR_INVALID_ARG, "server is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->jobs.find(ticket);
  if (it == s->jobs.end()) return sfail(PC_ERR_INVALID_ARG, "unknown ticket");
  Job *j = it->second;
  if (j->state == kQueued || j->state == kRunning) return sfail(PC_ERR_BUSY, "request not finished");
  s->jobs.erase(it);
  delete j;
  return PC_OK;
}

pc_status pc_server_get_stats(pc_server *s, pc_server_stats *st) {
  if (!s || !st) return sfail(PC_ERR_INVALID_ARG, "NULL argument");
  if (st->struct_size < sizeof(pc_server_stats)) return sfail(PC_ERR_INVALID_ARG, "pc_server_stats.struct_size too small");
  std::lock_guard<std::mutex> lk(s->mu);
  st->submitted = s->submitted;
  st->completed = s->completed;
  st->rejected = s->rejected;
  st->cancelled = s->cancelled;
  st->failed = s->failed;
  st->running = s->running;
  st->queued = (int32_t)s->queue.size();
  st->peak_running = s->peak_running;
  st->slots = s->slots;
  st->budget_bytes = s->budget;
  st->bytes_in_use = s->in_use;
  st->peak_bytes_in_use = s->peak_bytes;
  if (st->struct_size >= sizeof(pc_server_stats)) st->requeued = s->requeued;
  return PC_OK;
}

void pc_server_destroy(pc_server *s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    for (Job *j : s->queue) {
      j->state = kCancelled;
      ++s->cancelled;
    }
    s->queue.clear();
    s->stop = true;
  }
  s->cv_work.notify_all();
  s->cv_done.notify_all();
  for (std::thread &t : s->workers) t.join();  // running requests finish first
  for (pc_context *c : s->ctxs) pc_context_destroy(c);
  for (hipStream_t x : s->streams) hipStreamDestroy(x);
  for (auto &kv : s->jobs) delete kv.second;
  delete s;
}

}  // extern "C"
