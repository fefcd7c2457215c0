// Serving loop of libdisthist: a scheduler thread that admits histogram jobs
// by free slots and HBM budget (one stream per slot) and paces their
// pair-kernel launches onto the device, each from the admitted job with the
// least work left, so a job that arrives while a huge one runs is computed
// at the huge job's next launch boundary.
#include "disthist.h"
#include "dh_internal.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

namespace {

using Clock = std::chrono::steady_clock;

// pairs per pair-kernel launch of a served job (about 8-11 ms of binary32
// work on MI355X). Shorter launches cut the wait of a small job behind a
// large one but pay every workgroup's histogram flush once per launch
// (2^33 pairs: median latency 3 ms instead of 7 ms, 99th percentile and
// one-at-a-time latencies 12-15 % higher on the serving trace).
constexpr int64_t kServeLaunchPairs = int64_t{3} << 33;
// pair-kernel work on the device at once (at least one launch): one launch
// at a time, so a newly admitted job waits for the running one only; the
// device idles for one scheduling step between launches (two in flight
// measured no faster)
constexpr uint64_t kInflightPairs = static_cast<uint64_t>(kServeLaunchPairs);

double seconds_since(Clock::time_point t0, Clock::time_point t1) {
  return std::chrono::duration<double>(t1 - t0).count();
}

struct Job {
  int64_t id = 0;
  std::vector<double> coords;
  std::vector<int64_t> offsets;
  int32_t box_type = 0;
  double box[9] = {};
  bool has_box = false;
  double r_max = 0;
  int32_t n_bins = 0;
  int32_t precision = 0;
  int32_t n_hist = 0;
  int64_t n = 0;
  int64_t need = 0;  // device footprint while running
  double work = 0;   // pairs, the order of admission and of launches
  int status = DH_JOB_QUEUED;
  int slot = -1;
  Clock::time_point t_submit, t_admit, t_done;
  std::vector<uint64_t> out, oor;
};

struct Slot {
  dh_ctx *ctx = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  double *d_in = nullptr;
  size_t in_cap = 0;
  uint64_t *d_out = nullptr;
  size_t out_cap = 0;
  uint64_t *d_oor = nullptr;
  size_t oor_cap = 0;
  double *h_in = nullptr;
  size_t h_in_cap = 0;
  uint64_t *h_out = nullptr;
  size_t h_out_cap = 0;
  uint64_t *h_oor = nullptr;
  size_t h_oor_cap = 0;
  Job *job = nullptr;
  // scheduler thread only: the job's launches are still being paced
  // (stepping), or its closing copies and `done` are enqueued (closing)
  bool stepping = false, closing = false;
  uint64_t left = 0;  // pairs of the launches not issued yet
};

// a pair-kernel launch on the device and the event recorded after it
struct InFlight {
  hipEvent_t ev;
  uint64_t pairs;
};

int grow_device(void **p, size_t *cap, size_t need) {
  if (need <= *cap) return DH_OK;
  if (*p) (void)hipFree(*p);
  *p = nullptr;
  *cap = 0;
  const size_t want = std::max(need, static_cast<size_t>(1) << 20);
  if (hipMalloc(p, want) != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return DH_ENOMEM;
  }
  *cap = want;
  return DH_OK;
}

int grow_pinned(void **p, size_t *cap, size_t need) {
  if (need <= *cap) return DH_OK;
  if (*p) (void)hipHostFree(*p);
  *p = nullptr;
  *cap = 0;
  const size_t want = std::max(need, static_cast<size_t>(1) << 20);
  if (hipHostMalloc(p, want, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return DH_ENOMEM;
  }
  *cap = want;
  return DH_OK;
}

}  // namespace

struct dh_server {
  int32_t device = 0;
  int64_t budget = 0;
  double head_wait_limit = 1.0;
  std::atomic<int32_t> policy{DH_SCHED_SHORTEST};
  std::vector<Slot> slots;
  // scheduler thread only
  std::deque<InFlight> inflight;
  uint64_t inflight_pairs = 0;
  std::vector<hipEvent_t> event_pool;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Job *> queue;
  std::map<int64_t, std::unique_ptr<Job>> jobs;
  int64_t next_id = 1;
  int64_t used = 0;
  bool stop = false;
  std::thread worker;
  // statistics
  int64_t n_submitted = 0, n_completed = 0, n_failed = 0, max_running = 0, peak_used = 0;
  int64_t running = 0;
};

extern "C" int32_t dh_sched_select(const int64_t *need_bytes, const double *waited_s,
                                   const double *work, int32_t n_queued, int64_t free_bytes,
                                   int32_t free_slots, double head_wait_limit_s,
                                   int32_t *admit) {
  if (!need_bytes || !waited_s || !admit || n_queued <= 0 || free_slots <= 0) return 0;
  int32_t n = 0;
  auto take = [&](int32_t q) {
    admit[n++] = q;
    free_bytes -= need_bytes[q];
    --free_slots;
  };
  // jobs past the wait limit first, oldest first: one that does not fit
  // stops all admissions, so the memory that running jobs free goes to it
  std::vector<int32_t> rest;
  for (int32_t q = 0; q < n_queued; ++q) {
    if (waited_s[q] >= head_wait_limit_s) {
      if (free_slots == 0) break;
      if (need_bytes[q] > free_bytes) {
        std::sort(admit, admit + n);
        return n;
      }
      take(q);
    } else {
      rest.push_back(q);
    }
  }
  // then the others, least work first (arrival order without work), each
  // if it fits (backfill)
  if (work)
    std::stable_sort(rest.begin(), rest.end(),
                     [&](int32_t x, int32_t y) { return work[x] < work[y]; });
  for (int32_t q : rest) {
    if (free_slots == 0) break;
    if (need_bytes[q] <= free_bytes) take(q);
  }
  std::sort(admit, admit + n);
  return n;
}

namespace {

// Starts one admitted job on its slot (scheduler thread). Returns a status;
// on failure nothing is left running on the slot.
int start_job(dh_server *s, Slot &sl, Job &j) {
  const size_t in_b = static_cast<size_t>(std::max<int64_t>(1, j.n)) * 3 * sizeof(double);
  const size_t out_b = static_cast<size_t>(j.n_hist) * j.n_bins * sizeof(uint64_t);
  const size_t oor_b = static_cast<size_t>(j.n_hist) * sizeof(uint64_t);
  int rc = grow_device(reinterpret_cast<void **>(&sl.d_in), &sl.in_cap, in_b);
  if (!rc) rc = grow_device(reinterpret_cast<void **>(&sl.d_out), &sl.out_cap, out_b);
  if (!rc) rc = grow_device(reinterpret_cast<void **>(&sl.d_oor), &sl.oor_cap, oor_b);
  if (!rc) rc = grow_pinned(reinterpret_cast<void **>(&sl.h_in), &sl.h_in_cap, in_b);
  if (!rc) rc = grow_pinned(reinterpret_cast<void **>(&sl.h_out), &sl.h_out_cap, out_b);
  if (!rc) rc = grow_pinned(reinterpret_cast<void **>(&sl.h_oor), &sl.h_oor_cap, oor_b);
  if (rc) return rc;
  if (j.n > 0) {
    std::memcpy(sl.h_in, j.coords.data(), static_cast<size_t>(j.n) * 3 * sizeof(double));
    if (hipMemcpyAsync(sl.d_in, sl.h_in, static_cast<size_t>(j.n) * 3 * sizeof(double),
                       hipMemcpyHostToDevice, sl.stream) != hipSuccess)
      return DH_EDEVICE;
  }
  // staging and zeroing now; the pair-kernel launches wait for dispatch()
  rc = dh::histo_job(sl.ctx, sl.stream, sl.d_in, j.offsets.data(),
                     static_cast<int32_t>(j.offsets.size() - 1), j.box_type,
                     j.has_box ? j.box : nullptr, j.r_max, j.n_bins, j.precision, sl.d_out,
                     sl.d_oor, false, nullptr, true);
  if (rc) return rc;
  sl.stepping = true;
  sl.closing = false;
  sl.left = static_cast<uint64_t>(j.work);
  (void)s;
  return DH_OK;
}

// Enqueues the copies of a job's results and its completion event.
int close_job(Slot &sl) {
  const Job &j = *sl.job;
  const size_t out_b = static_cast<size_t>(j.n_hist) * j.n_bins * sizeof(uint64_t);
  const size_t oor_b = static_cast<size_t>(j.n_hist) * sizeof(uint64_t);
  if (hipMemcpyAsync(sl.h_out, sl.d_out, out_b, hipMemcpyDeviceToHost, sl.stream) != hipSuccess ||
      hipMemcpyAsync(sl.h_oor, sl.d_oor, oor_b, hipMemcpyDeviceToHost, sl.stream) != hipSuccess ||
      hipEventRecord(sl.done, sl.stream) != hipSuccess)
    return DH_EDEVICE;
  sl.stepping = false;
  sl.closing = true;
  return DH_OK;
}

void finish_job(dh_server *s, Slot &sl, Job &j, int status) {
  j.t_done = Clock::now();
  if (status == DH_OK) {
    const size_t out_n = static_cast<size_t>(j.n_hist) * j.n_bins;
    j.out.assign(sl.h_out, sl.h_out + out_n);
    j.oor.assign(sl.h_oor, sl.h_oor + j.n_hist);
    ++s->n_completed;
  } else {
    ++s->n_failed;
  }
  j.status = status;
  j.coords.clear();
  j.coords.shrink_to_fit();
  s->used -= j.need;
  --s->running;
  sl.job = nullptr;
  sl.stepping = sl.closing = false;
  sl.left = 0;
}

// true when slot a's job goes before slot b's: least work left first
// (shortest remaining work), or the earliest submitted under arrival order
bool goes_first(const dh_server *s, const Slot &a, const Slot &b) {
  if (s->policy == DH_SCHED_SHORTEST && a.left != b.left) return a.left < b.left;
  return a.job->id < b.job->id;
}

// Retires finished launches, then issues held launches while the pairs on
// the device stay within kInflightPairs (one launch at least), each from the
// job that goes first; a job with none left gets its closing step, copies
// and completion event. Scheduler thread, outside the lock.
void dispatch(dh_server *s) {
  for (auto it = s->inflight.begin(); it != s->inflight.end();) {
    const hipError_t e = hipEventQuery(it->ev);
    if (e == hipErrorNotReady) {
      ++it;
      continue;
    }
    if (e != hipSuccess) (void)hipGetLastError();  // the job's `done` reports it
    s->inflight_pairs -= it->pairs;
    s->event_pool.push_back(it->ev);
    it = s->inflight.erase(it);
  }
  while (true) {
    Slot *best = nullptr;
    for (Slot &sl : s->slots)
      if (sl.stepping && (!best || goes_first(s, sl, *best))) best = &sl;
    if (!best) return;
    const uint64_t next = dh::stepped_next_pairs(best->ctx);
    if (next > 0 && !s->inflight.empty() && s->inflight_pairs + next > kInflightPairs) return;
    uint64_t left = 0;
    bool done = false;
    int rc = dh::step_job(best->ctx, best->stream, &left, &done);
    best->left = left;
    if (!rc && !done) {
      hipEvent_t ev = nullptr;
      if (!s->event_pool.empty()) {
        ev = s->event_pool.back();
        s->event_pool.pop_back();
      } else if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
        ev = nullptr;
      }
      if (ev && hipEventRecord(ev, best->stream) == hipSuccess) {
        s->inflight.push_back({ev, next});
        s->inflight_pairs += next;
      } else {
        if (ev) s->event_pool.push_back(ev);
        rc = DH_EDEVICE;
      }
    }
    if (!rc && done) rc = close_job(*best);
    if (rc) {
      (void)hipStreamSynchronize(best->stream);
      (void)hipGetLastError();
      std::lock_guard<std::mutex> lk(s->mu);
      finish_job(s, *best, *best->job, rc);
      s->cv_done.notify_all();
    }
  }
}

void scheduler(dh_server *s) {
  if (hipSetDevice(s->device) != hipSuccess) (void)hipGetLastError();
  std::vector<int64_t> need;
  std::vector<double> waited, work;
  std::vector<int32_t> admit;
  while (true) {
    std::vector<std::pair<Slot *, Job *>> to_start;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      // completions
      bool any_done = false;
      for (Slot &sl : s->slots) {
        if (!sl.job || !sl.closing) continue;
        const hipError_t e = hipEventQuery(sl.done);
        if (e == hipErrorNotReady) continue;
        finish_job(s, sl, *sl.job, e == hipSuccess ? DH_OK : DH_EDEVICE);
        if (e != hipSuccess) (void)hipGetLastError();
        any_done = true;
      }
      if (any_done) s->cv_done.notify_all();
      if (s->stop && s->running == 0) break;
      // admissions
      int32_t free_slots = 0;
      for (Slot &sl : s->slots) free_slots += sl.job ? 0 : 1;
      if (!s->stop && free_slots > 0 && !s->queue.empty()) {
        const Clock::time_point now = Clock::now();
        need.clear();
        waited.clear();
        work.clear();
        for (Job *j : s->queue) {
          need.push_back(j->need);
          waited.push_back(seconds_since(j->t_submit, now));
          work.push_back(j->work);
        }
        admit.assign(s->queue.size(), 0);
        const int32_t n = dh_sched_select(need.data(), waited.data(),
                                          s->policy == DH_SCHED_SHORTEST ? work.data() : nullptr,
                                          static_cast<int32_t>(need.size()), s->budget - s->used,
                                          free_slots, s->head_wait_limit, admit.data());
        std::vector<Job *> chosen;
        for (int32_t k = n - 1; k >= 0; --k) {
          chosen.push_back(s->queue[admit[k]]);
          s->queue.erase(s->queue.begin() + admit[k]);
        }
        std::reverse(chosen.begin(), chosen.end());
        size_t next_slot = 0;
        for (Job *j : chosen) {
          while (s->slots[next_slot].job) ++next_slot;
          Slot &sl = s->slots[next_slot];
          sl.job = j;
          j->slot = static_cast<int>(next_slot);
          j->status = DH_JOB_RUNNING;
          j->t_admit = now;
          s->used += j->need;
          ++s->running;
          s->peak_used = std::max(s->peak_used, s->used);
          s->max_running = std::max(s->max_running, s->running);
          to_start.emplace_back(&sl, j);
        }
      }
      if (to_start.empty() && s->running == 0) {
        if (s->stop) break;
        s->cv_work.wait(lk, [&] { return s->stop || !s->queue.empty(); });
        continue;
      }
    }
    // device work outside the lock (only this thread touches the device)
    for (auto &sj : to_start) {
      const int rc = start_job(s, *sj.first, *sj.second);
      if (rc) {
        (void)hipStreamSynchronize(sj.first->stream);
        (void)hipGetLastError();
        std::lock_guard<std::mutex> lk(s->mu);
        finish_job(s, *sj.first, *sj.second, rc);
        s->cv_done.notify_all();
      }
    }
    dispatch(s);
    if (to_start.empty()) std::this_thread::sleep_for(std::chrono::microseconds(20));
  }
}

void release_slot(Slot &sl) {
  if (sl.d_in) (void)hipFree(sl.d_in);
  if (sl.d_out) (void)hipFree(sl.d_out);
  if (sl.d_oor) (void)hipFree(sl.d_oor);
  if (sl.h_in) (void)hipHostFree(sl.h_in);
  if (sl.h_out) (void)hipHostFree(sl.h_out);
  if (sl.h_oor) (void)hipHostFree(sl.h_oor);
  if (sl.done) (void)hipEventDestroy(sl.done);
  if (sl.stream) (void)hipStreamDestroy(sl.stream);
  if (sl.ctx) dh_ctx_destroy(sl.ctx);
  sl = Slot();
}

}  // namespace

extern "C" {

int dh_server_create(int32_t device, int64_t hbm_budget_bytes, int32_t max_inflight,
                     double head_wait_limit_s, dh_server **out) {
  if (!out) return DH_EINVAL;
  *out = nullptr;
  if (hbm_budget_bytes <= 0 || max_inflight < 1 || max_inflight > 16) return DH_EINVAL;
  std::unique_ptr<dh_server> s(new (std::nothrow) dh_server);
  if (!s) return DH_ENOMEM;
  s->device = device;
  s->budget = hbm_budget_bytes;
  s->head_wait_limit = head_wait_limit_s < 0 ? 1.0 : head_wait_limit_s;
  s->slots.resize(max_inflight);
  for (Slot &sl : s->slots) {
    int rc = dh_ctx_create(device, &sl.ctx);
    // bounded launches: a job that arrives while a huge one runs waits for
    // one launch of the huge job (about 10 ms), not for all of it
    if (!rc) rc = dh_ctx_set_launch_pairs(sl.ctx, kServeLaunchPairs);
    if (!rc && (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
                hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess))
      rc = DH_EDEVICE;
    if (rc) {
      (void)hipGetLastError();
      for (Slot &x : s->slots) release_slot(x);
      return rc;
    }
  }
  s->worker = std::thread(scheduler, s.get());
  *out = s.release();
  return DH_OK;
}

int dh_server_submit(dh_server *s, const double *coords, const int64_t *offsets,
                     int32_t n_species, int32_t box_type, const double *box, double r_max,
                     int32_t n_bins, int32_t precision, int64_t *job_id) {
  if (!s || !job_id) return DH_EINVAL;
  int rc = dh_check_args(coords, offsets, n_species, box_type, box, r_max, n_bins, precision);
  if (rc) return rc;
  const int64_t n = offsets[n_species];
  if (n > 0 && !coords) return DH_EINVAL;
  auto j = std::make_unique<Job>();
  j->n = n;
  j->n_hist = n_species * (n_species + 1) / 2;
  j->work = 0.5 * static_cast<double>(n) * static_cast<double>(n > 0 ? n - 1 : 0);
  j->need = static_cast<int64_t>(std::max<int64_t>(1, n) * 3 * sizeof(double) +
                                 static_cast<size_t>(j->n_hist) * n_bins * sizeof(uint64_t) +
                                 dh::job_scratch_bytes(n, j->n_hist, n_bins, precision,
                                                       kServeLaunchPairs));
  if (j->need > s->budget) return DH_EBUDGET;
  j->coords.assign(coords, coords + 3 * n);
  j->offsets.assign(offsets, offsets + n_species + 1);
  j->box_type = box_type;
  j->has_box = box_type != DH_BOX_NONE && box != nullptr;
  if (j->has_box) std::memcpy(j->box, box, sizeof j->box);
  j->r_max = r_max;
  j->n_bins = n_bins;
  j->precision = precision;
  j->t_submit = Clock::now();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    j->id = s->next_id++;
    *job_id = j->id;
    s->queue.push_back(j.get());
    s->jobs[j->id] = std::move(j);
    ++s->n_submitted;
  }
  s->cv_work.notify_all();
  return DH_OK;
}

int dh_server_set_policy(dh_server *s, int32_t policy) {
  if (!s || (policy != DH_SCHED_SHORTEST && policy != DH_SCHED_ARRIVAL)) return DH_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  s->policy = policy;
  return DH_OK;
}

int dh_server_status(dh_server *s, int64_t job_id) {
  if (!s) return DH_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->jobs.find(job_id);
  if (it == s->jobs.end()) return DH_EINVAL;
  return it->second->status;
}

int dh_server_wait(dh_server *s, int64_t job_id, uint64_t *out, uint64_t *out_of_range,
                   double *times) {
  if (!s) return DH_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->jobs.find(job_id);
  if (it == s->jobs.end()) return DH_EINVAL;
  Job *j = it->second.get();
  s->cv_done.wait(lk, [&] { return j->status <= DH_JOB_DONE; });
  const int status = j->status;
  if (status == DH_OK) {
    if (out) std::memcpy(out, j->out.data(), j->out.size() * sizeof(uint64_t));
    if (out_of_range) std::memcpy(out_of_range, j->oor.data(), j->oor.size() * sizeof(uint64_t));
  }
  if (times) {
    times[0] = seconds_since(j->t_submit, j->t_admit);
    times[1] = seconds_since(j->t_admit, j->t_done);
    times[2] = seconds_since(j->t_submit, j->t_done);
  }
  s->jobs.erase(it);
  return status;
}

int dh_server_stats(const dh_server *s, int64_t *stats) {
  if (!s || !stats) return DH_EINVAL;
  dh_server *m = const_cast<dh_server *>(s);
  std::lock_guard<std::mutex> lk(m->mu);
  stats[0] = s->n_submitted;
  stats[1] = s->n_completed;
  stats[2] = s->n_failed;
  stats[3] = s->max_running;
  stats[4] = s->peak_used;
  stats[5] = s->budget;
  return DH_OK;
}

void dh_server_destroy(dh_server *s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    for (Job *j : s->queue) j->status = DH_EINVAL;
    s->queue.clear();
  }
  s->cv_work.notify_all();
  s->cv_done.notify_all();
  if (s->worker.joinable()) s->worker.join();
  if (hipSetDevice(s->device) == hipSuccess) (void)hipDeviceSynchronize();
  for (Slot &sl : s->slots) release_slot(sl);
  for (const InFlight &f : s->inflight) (void)hipEventDestroy(f.ev);
  for (hipEvent_t ev : s->event_pool) (void)hipEventDestroy(ev);
  (void)hipGetLastError();
  delete s;
}

}  // extern "C"
