// Serving loop of libdisthist with continuous batching.
//
// Jobs are admitted by free slots and HBM budget (dh_sched_select). An
// admitted job's frame is copied, staged and zeroed on a setup stream and
// stays resident in its slot; its work list is kept on the host. The
// scheduler thread then builds every pair-kernel launch from the work items
// of all ready jobs that share a kernel variant (precision, minimum-image
// kind, accumulation mode and launch shape), in policy order, up to a fixed
// amount of work per launch: a job admitted while others run joins the next
// launch, and the launch packs the small jobs together with pieces of the
// large ones. Each slot's frame constants sit at the slot's index of one
// device table, so items of different frames share a launch as they do in
// a batch. When a launch carries the last items of a job, a copy stream
// waits for that launch and copies the job's results out.
//
// The paper's engine (Sec. 3.3) feeds frames from a producer to workers that
// each take a frame at a time; here the unit of work handed to the device is
// a work item, so several frames are computed by one launch.
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
using dh::FrameParams;
using dh::LaunchPlan;
using dh::WorkItem;

// Pairs per pair-kernel launch, about 10 ms of binary32 work on MI355X: a
// new job waits for the launches in flight (at most two) before its items
// are on the device.
constexpr uint64_t kLaunchPairs = uint64_t{3} << 33;
constexpr int kLaunchesInFlight = 2;
constexpr int kRegions = kLaunchesInFlight + 1;
// work items of one launch at most (32 bytes each); the tail refinement
// splits up to one grid of items into four pieces each
constexpr int64_t kMaxItemsPerLaunch = int64_t{1} << 16;
constexpr int kItemsPerWg = 8;

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
  int64_t need = 0;  // device footprint while resident
  double work = 0;   // pairs: the order of admission
  int status = DH_JOB_QUEUED;
  int slot = -1;
  Clock::time_point t_submit, t_admit, t_done;
  std::vector<uint64_t> out, oor;
  // scheduler thread only, once admitted
  int kind = 0;
  LaunchPlan plan{};
  std::vector<WorkItem> items;
  size_t next_item = 0;
  uint64_t left = 0;     // pairs of the items not issued yet
  bool ready = false;    // frame staged and zeroed on the device
  bool closing = false;  // last items issued, result copies enqueued
};

struct Slot {
  Job *job = nullptr;
  hipEvent_t setup = nullptr, done = nullptr;
  double *d_in = nullptr;
  size_t in_cap = 0;
  void *d_staged = nullptr;
  size_t staged_cap = 0;
  uint64_t *d_out = nullptr;
  size_t out_cap = 0;
  uint64_t *d_oor = nullptr;
  size_t oor_cap = 0;
  uint64_t *d_pairs = nullptr;
  size_t pairs_cap = 0;
  void *d_keys = nullptr;  // sort keys of a spatially sorted frame
  size_t keys_cap = 0;
  double *h_in = nullptr;
  size_t h_in_cap = 0;
  uint64_t *h_out = nullptr;
  size_t h_out_cap = 0;
  uint64_t *h_oor = nullptr;
  size_t h_oor_cap = 0;
  uint64_t *h_pairs = nullptr;
  size_t h_pairs_cap = 0;
};

// Device work list of one launch (items, then its work counter) and the
// pinned copy it is uploaded from; reused once the launch has finished.
struct Region {
  WorkItem *d_items = nullptr;
  WorkItem *h_items = nullptr;
  hipEvent_t ev = nullptr;
  bool busy = false;
};

int grow_device(void **p, size_t *cap, size_t need) {
  if (need <= *cap) return DH_OK;
  if (*p) (void)hipFree(*p);
  *p = nullptr;
  *cap = 0;
  size_t want = size_t{1} << 20;
  while (want < need) want <<= 1;
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
  size_t want = size_t{1} << 16;
  while (want < need) want <<= 1;
  if (hipHostMalloc(p, want, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return DH_ENOMEM;
  }
  *cap = want;
  return DH_OK;
}

size_t region_bytes() {
  return static_cast<size_t>(kMaxItemsPerLaunch) * sizeof(WorkItem) + 256;
}

}  // namespace

struct dh_server {
  int32_t device = 0;
  int64_t budget = 0;
  double head_wait_limit = 1.0;
  int n_cu = 0;
  size_t lds_per_block = 0;
  std::atomic<int32_t> policy{DH_SCHED_SHORTEST};
  std::vector<Slot> slots;
  // scheduler thread only
  hipStream_t compute = nullptr, setup = nullptr, copy = nullptr;
  FrameParams *d_frames = nullptr;   // one entry per slot
  FrameParams *h_frames = nullptr;   // pinned staging of the entries
  Region regions[kRegions];
  std::deque<int> inflight;          // regions of launches in flight, oldest first
  std::vector<WorkItem> launch_items;
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
  std::atomic<int64_t> n_launches{0}, max_jobs_per_launch{0}, shared_launches{0};
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

// Device bytes a job holds while resident: its coordinates, the staged copy
// (and the sort keys of a spatially sorted frame), histograms, out-of-range
// and pair counts. Large frames that may be staged in spatial order are
// counted as if sorted, an upper bound that needs no cell geometry.
int64_t job_footprint(int64_t n, int32_t n_hist, int32_t n_bins, int32_t precision,
                      int32_t box_type) {
  const int64_t pts = std::max<int64_t>(1, n);
  const bool may_sort = (box_type == DH_BOX_TRICLINIC ||
                         (box_type == DH_BOX_ORTHO && precision == DH_FP64)) &&
                        n >= dh::kSortMinPoints;
  return pts * 3 * static_cast<int64_t>(sizeof(double)) +
         pts * (precision == DH_FP64 || may_sort ? 32 : 16) +
         (may_sort ? dh::sort_keys_count(n) * 8 : 0) +
         static_cast<int64_t>(n_hist) * n_bins * static_cast<int64_t>(sizeof(uint64_t)) +
         2 * static_cast<int64_t>(n_hist) * static_cast<int64_t>(sizeof(uint64_t));
}

// j-range of one item: about kItemsPerWg items per workgroup of a launch's
// share of the job, in whole j-tiles (the host planner's rule, applied to
// at most one launch of work).
int64_t serve_jchunk(const LaunchPlan &p, uint64_t work) {
  const uint64_t bi = static_cast<uint64_t>(p.cfg.threads) * p.cfg.r;
  const uint64_t w = std::min<uint64_t>(work, kLaunchPairs);
  uint64_t jc = w / (static_cast<uint64_t>(std::max(1, p.grid)) * kItemsPerWg * bi + 1);
  jc = (jc + p.cfg.tj - 1) / p.cfg.tj * p.cfg.tj;
  jc = std::max<uint64_t>(jc, p.cfg.tj);
  jc = std::min<uint64_t>(jc, 64ull * p.cfg.tj);
  return static_cast<int64_t>(jc);
}

uint64_t item_pairs(const WorkItem &w) {
  return static_cast<uint64_t>(w.i1 - w.i0) * static_cast<uint64_t>(w.j1 - w.j0);
}

// Splits the last `grid` items of a launch into pieces of about a quarter of
// their j-range (whole j-tiles; diagonal items stay whole), so workgroups
// finish close together.
void refine_tail(std::vector<WorkItem> &items, int grid, int tj) {
  const size_t n = items.size();
  const size_t tail = std::min<size_t>(n, static_cast<size_t>(std::max(grid, 0)));
  if (tail == 0) return;
  std::vector<WorkItem> last(items.end() - static_cast<std::ptrdiff_t>(tail), items.end());
  items.resize(n - tail);
  for (const WorkItem &w : last) {
    const int32_t len = w.j1 - w.j0;
    const int32_t piece = std::max<int32_t>(tj, (len / 4 + tj - 1) / tj * tj);
    if ((w.flags & dh::kItemDiag) || len <= piece) {
      items.push_back(w);
      continue;
    }
    for (int32_t j = w.j0; j < w.j1; j += piece) {
      WorkItem p = w;
      p.j0 = j;
      p.j1 = std::min(j + piece, w.j1);
      items.push_back(p);
    }
  }
}

// Enqueues one admitted job's setup on the setup stream: input copy, frame
// constants into the slot's table entry, pair counts, staging and zeroing;
// plans its work items on the host. Scheduler thread.
int start_job(dh_server *s, int slot_idx) {
  Slot &sl = s->slots[static_cast<size_t>(slot_idx)];
  Job &j = *sl.job;
  const int32_t k = static_cast<int32_t>(j.offsets.size() - 1);
  const size_t pts = static_cast<size_t>(std::max<int64_t>(1, j.n));
  const size_t in_b = pts * 3 * sizeof(double);
  FrameParams fp;
  j.kind = dh::staged_kind(
      dh::frame_constants(j.box_type, j.has_box ? j.box : nullptr, j.r_max, j.n_bins, fp),
      j.precision, fp.L, j.n);
  fp.box = j.kind;
  const size_t staged_b = pts * dh::staged_point_bytes(j.precision, j.kind);
  const size_t out_b = static_cast<size_t>(j.n_hist) * j.n_bins * sizeof(uint64_t);
  const size_t h_b = static_cast<size_t>(j.n_hist) * sizeof(uint64_t);
  int rc = grow_device(reinterpret_cast<void **>(&sl.d_in), &sl.in_cap, in_b);
  if (!rc) rc = grow_device(&sl.d_staged, &sl.staged_cap, staged_b);
  if (!rc) rc = grow_device(reinterpret_cast<void **>(&sl.d_out), &sl.out_cap, out_b);
  if (!rc) rc = grow_device(reinterpret_cast<void **>(&sl.d_oor), &sl.oor_cap, h_b);
  if (!rc) rc = grow_device(reinterpret_cast<void **>(&sl.d_pairs), &sl.pairs_cap, h_b);
  if (!rc) rc = grow_pinned(reinterpret_cast<void **>(&sl.h_in), &sl.h_in_cap, in_b);
  if (!rc) rc = grow_pinned(reinterpret_cast<void **>(&sl.h_out), &sl.h_out_cap, out_b);
  if (!rc) rc = grow_pinned(reinterpret_cast<void **>(&sl.h_oor), &sl.h_oor_cap, h_b);
  if (!rc) rc = grow_pinned(reinterpret_cast<void **>(&sl.h_pairs), &sl.h_pairs_cap, h_b);
  if (!rc && j.kind == dh::kBoxTricSorted)
    rc = grow_device(&sl.d_keys, &sl.keys_cap,
                     static_cast<size_t>(dh::sort_keys_count(j.n)) * sizeof(uint64_t));
  if (rc) return rc;
  uint64_t total = 0;
  for (int32_t h = 0; h < j.n_hist; ++h) {
    sl.h_pairs[h] = dh::hist_rows(j.offsets.data(), k, h).pairs;
    total += sl.h_pairs[h];
  }
  // one workgroup size per accumulation mode, so that frames of one kind
  // and mode can share a launch: 512 threads with one LDS histogram (two or
  // more workgroups per CU), 1024 with bin windows (one per CU)
  const LaunchPlan probe = dh::default_launch(s->n_cu, s->lds_per_block, j.precision, fp, total);
  const int threads = probe.mode == dh::kModeSweep ? 1024 : 512;
  j.plan = dh::serve_launch(s->n_cu, s->lds_per_block, j.precision, fp, total, threads);
  fp.coords = sl.d_staged;
  fp.out = sl.d_out;
  fp.win = j.plan.win;
  fp.n_sweeps = j.plan.n_sweeps;
  fp.noclamp = j.plan.noclamp ? 1 : 0;
  const bool oor_flush = j.plan.mode != dh::kModeGlobal;
  fp.oor = oor_flush ? sl.d_oor : nullptr;
  fp.oor_by_flush = oor_flush ? 1 : 0;
  fp.searched = nullptr;
  s->h_frames[slot_idx] = fp;

  // items of every histogram and bin window; the frame is the slot index
  const int64_t bi = static_cast<int64_t>(j.plan.cfg.threads) * j.plan.cfg.r;
  const int64_t jc = serve_jchunk(j.plan, total * static_cast<uint64_t>(j.plan.n_sweeps));
  j.items.clear();
  for (int32_t h = 0; h < j.n_hist; ++h) {
    const dh::HistRows r = dh::hist_rows(j.offsets.data(), k, h);
    const int64_t nr = dh::hist_row_count(r, bi);
    for (int32_t sw = 0; sw < j.plan.n_sweeps; ++sw)
      for (int64_t row = 0; row < nr; ++row) {
        const size_t at = j.items.size();
        j.items.resize(at + static_cast<size_t>(dh::row_item_count(r, row, bi, jc)));
        dh::emit_row(r, h, sw, row, bi, jc, j.items.data() + at);
      }
  }
  j.left = 0;
  for (WorkItem &w : j.items) {
    w.frame = slot_idx;
    j.left += item_pairs(w);
  }
  j.next_item = 0;
  j.ready = false;
  j.closing = false;

  if (j.n > 0) {
    std::memcpy(sl.h_in, j.coords.data(), static_cast<size_t>(j.n) * 3 * sizeof(double));
    if (hipMemcpyAsync(sl.d_in, sl.h_in, static_cast<size_t>(j.n) * 3 * sizeof(double),
                       hipMemcpyHostToDevice, s->setup) != hipSuccess)
      return DH_EDEVICE;
  }
  if (hipMemcpyAsync(s->d_frames + slot_idx, s->h_frames + slot_idx, sizeof(FrameParams),
                     hipMemcpyHostToDevice, s->setup) != hipSuccess ||
      hipMemcpyAsync(sl.d_pairs, sl.h_pairs, h_b, hipMemcpyHostToDevice, s->setup) !=
          hipSuccess)
    return DH_EDEVICE;
  const hipError_t staged =
      j.kind == dh::kBoxTricSorted
          ? dh::launch_stage_sorted(j.precision, sl.d_in, sl.d_staged, j.n, j.offsets.data(), k, fp,
                                    static_cast<uint64_t *>(sl.d_keys), s->setup)
          : dh::launch_stage(j.precision, j.kind, sl.d_in, sl.d_staged, j.n, fp, s->setup);
  if (staged != hipSuccess ||
      dh::launch_zero(sl.d_out, static_cast<int64_t>(j.n_hist) * j.n_bins, nullptr, 0, fp.oor,
                      sl.d_pairs, j.n_hist, s->setup) != hipSuccess ||
      hipEventRecord(sl.setup, s->setup) != hipSuccess)
    return DH_EDEVICE;
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
  j.items.clear();
  j.items.shrink_to_fit();
  s->used -= j.need;
  --s->running;
  sl.job = nullptr;
}

// Launch class of a job: jobs of one class can share a pair-kernel launch.
bool same_class(const Job &a, const Job &b) {
  return a.precision == b.precision && a.kind == b.kind && a.plan.mode == b.plan.mode &&
         a.plan.cfg.threads == b.plan.cfg.threads && a.plan.cfg.r == b.plan.cfg.r &&
         a.plan.cfg.copies == b.plan.cfg.copies && a.plan.cfg.tj == b.plan.cfg.tj;
}

bool goes_first(const dh_server *s, const Job &a, const Job &b) {
  if (s->policy == DH_SCHED_SHORTEST && a.left != b.left) return a.left < b.left;
  return a.id < b.id;
}

// Enqueues the closing steps of a job whose last items went into the launch
// of region `reg`: the global-atomic mode's out-of-range pass on the compute
// stream, then the result copies on the copy stream once that launch is done.
int close_job(dh_server *s, Slot &sl, hipEvent_t launch_done) {
  Job &j = *sl.job;
  const size_t out_b = static_cast<size_t>(j.n_hist) * j.n_bins * sizeof(uint64_t);
  const size_t h_b = static_cast<size_t>(j.n_hist) * sizeof(uint64_t);
  if (hipStreamWaitEvent(s->copy, launch_done, 0) != hipSuccess ||
      hipMemcpyAsync(sl.h_out, sl.d_out, out_b, hipMemcpyDeviceToHost, s->copy) != hipSuccess ||
      hipMemcpyAsync(sl.h_oor, sl.d_oor, h_b, hipMemcpyDeviceToHost, s->copy) != hipSuccess ||
      hipEventRecord(sl.done, s->copy) != hipSuccess)
    return DH_EDEVICE;
  j.closing = true;
  return DH_OK;
}

void fail_slot(dh_server *s, Slot &sl, int rc) {
  (void)hipDeviceSynchronize();
  (void)hipGetLastError();
  std::lock_guard<std::mutex> lk(s->mu);
  if (sl.job) finish_job(s, sl, *sl.job, rc);
  s->cv_done.notify_all();
}

// Builds and enqueues one launch from the ready jobs; false when no work is
// ready or no region is free.
bool issue_launch(dh_server *s) {
  int reg = -1;
  for (int r = 0; r < kRegions; ++r)
    if (!s->regions[r].busy) {
      reg = r;
      break;
    }
  if (reg < 0) return false;
  std::vector<int> cand;
  for (size_t q = 0; q < s->slots.size(); ++q) {
    const Job *j = s->slots[q].job;
    if (j && j->ready && !j->closing && j->next_item < j->items.size())
      cand.push_back(static_cast<int>(q));
  }
  if (cand.empty()) return false;
  std::stable_sort(cand.begin(), cand.end(), [&](int a, int b) {
    return goes_first(s, *s->slots[static_cast<size_t>(a)].job,
                      *s->slots[static_cast<size_t>(b)].job);
  });
  const Job &top = *s->slots[static_cast<size_t>(cand[0])].job;
  std::vector<WorkItem> &list = s->launch_items;
  list.clear();
  uint64_t pairs = 0;
  int grid = top.plan.grid, stride = 0;
  size_t lds = 0;
  std::vector<int> members, finished;
  const int64_t cap = kMaxItemsPerLaunch - 3 * static_cast<int64_t>(s->n_cu) * 16;
  for (int q : cand) {
    Job &j = *s->slots[static_cast<size_t>(q)].job;
    if (!same_class(top, j)) continue;
    if (pairs >= kLaunchPairs || static_cast<int64_t>(list.size()) >= cap) break;
    const size_t first = j.next_item;
    while (j.next_item < j.items.size() && pairs < kLaunchPairs &&
           static_cast<int64_t>(list.size()) < cap) {
      const WorkItem &w = j.items[j.next_item++];
      pairs += item_pairs(w);
      j.left -= item_pairs(w);
      list.push_back(w);
    }
    if (j.next_item == first) continue;
    members.push_back(q);
    grid = std::min(grid, j.plan.grid);
    stride = std::max(stride, j.plan.stride);
    lds = std::max(lds, j.plan.lds);
    if (j.next_item == j.items.size()) finished.push_back(q);
  }
  grid = std::max(1, std::min<int>(grid, static_cast<int>(list.size())));
  refine_tail(list, grid, top.plan.cfg.tj);
  Region &R = s->regions[reg];
  std::memcpy(R.h_items, list.data(), list.size() * sizeof(WorkItem));
  int32_t *h_counter = reinterpret_cast<int32_t *>(R.h_items + kMaxItemsPerLaunch);
  *h_counter = 0;
  hipError_t e = hipMemcpyAsync(R.d_items, R.h_items, list.size() * sizeof(WorkItem),
                                hipMemcpyHostToDevice, s->compute);
  if (e == hipSuccess)
    e = hipMemcpyAsync(R.d_items + kMaxItemsPerLaunch, h_counter, sizeof(int32_t),
                       hipMemcpyHostToDevice, s->compute);
  dh::PairKernelArgs a;
  a.frames = s->d_frames;
  a.items = R.d_items;
  a.counter = reinterpret_cast<int32_t *>(R.d_items + kMaxItemsPerLaunch);
  a.n_items = static_cast<int32_t>(list.size());
  a.copies = top.plan.cfg.copies;
  a.stride = stride;
  a.tj = top.plan.cfg.tj;
  if (e == hipSuccess)
    e = dh::launch_pairs(top.precision, top.kind, top.plan.mode, top.plan.cfg, a, grid, lds,
                         s->compute);
  // the global-atomic mode counts out-of-range pairs after the last launch
  for (int q : finished) {
    Slot &sl = s->slots[static_cast<size_t>(q)];
    if (e == hipSuccess && sl.job->plan.mode == dh::kModeGlobal)
      e = dh::launch_oor(sl.d_out, sl.job->n_hist, sl.job->n_bins, sl.d_pairs, sl.d_oor,
                         s->compute);
  }
  if (e == hipSuccess) e = hipEventRecord(R.ev, s->compute);
  if (e != hipSuccess) {
    for (int q : members) fail_slot(s, s->slots[static_cast<size_t>(q)], DH_EDEVICE);
    return false;
  }
  R.busy = true;
  s->inflight.push_back(reg);
  ++s->n_launches;
  if (members.size() > 1) ++s->shared_launches;
  if (static_cast<int64_t>(members.size()) > s->max_jobs_per_launch)
    s->max_jobs_per_launch = static_cast<int64_t>(members.size());
  for (int q : finished) {
    const int rc = close_job(s, s->slots[static_cast<size_t>(q)], R.ev);
    if (rc) fail_slot(s, s->slots[static_cast<size_t>(q)], rc);
  }
  return true;
}

void scheduler(dh_server *s) {
  if (hipSetDevice(s->device) != hipSuccess) (void)hipGetLastError();
  std::vector<int64_t> need;
  std::vector<double> waited, work;
  std::vector<int32_t> admit;
  while (true) {
    std::vector<int> to_start;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      // completions
      bool any_done = false;
      for (Slot &sl : s->slots) {
        if (!sl.job || !sl.job->closing) continue;
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
        for (int32_t q = n - 1; q >= 0; --q) {
          chosen.push_back(s->queue[static_cast<size_t>(admit[q])]);
          s->queue.erase(s->queue.begin() + admit[q]);
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
          to_start.push_back(static_cast<int>(next_slot));
        }
      }
      if (to_start.empty() && s->running == 0) {
        if (s->stop) break;
        s->cv_work.wait(lk, [&] { return s->stop || !s->queue.empty(); });
        continue;
      }
    }
    // device work outside the lock (only this thread touches the device)
    for (int q : to_start) {
      const int rc = start_job(s, q);
      if (rc) fail_slot(s, s->slots[static_cast<size_t>(q)], rc);
    }
    for (Slot &sl : s->slots) {
      if (!sl.job || sl.job->ready) continue;
      const hipError_t e = hipEventQuery(sl.setup);
      if (e == hipErrorNotReady) continue;
      if (e != hipSuccess) {
        fail_slot(s, sl, DH_EDEVICE);
        continue;
      }
      sl.job->ready = true;
      // a job without pairs has nothing to launch: its results are ready
      if (sl.job->items.empty()) {
        const size_t out_b = static_cast<size_t>(sl.job->n_hist) * sl.job->n_bins * 8;
        const size_t h_b = static_cast<size_t>(sl.job->n_hist) * 8;
        if (hipMemcpyAsync(sl.h_out, sl.d_out, out_b, hipMemcpyDeviceToHost, s->copy) !=
                hipSuccess ||
            hipMemcpyAsync(sl.h_oor, sl.d_oor, h_b, hipMemcpyDeviceToHost, s->copy) !=
                hipSuccess ||
            hipEventRecord(sl.done, s->copy) != hipSuccess)
          fail_slot(s, sl, DH_EDEVICE);
        else
          sl.job->closing = true;
      }
    }
    // retire finished launches, then keep up to kLaunchesInFlight on the device
    while (!s->inflight.empty()) {
      Region &R = s->regions[s->inflight.front()];
      const hipError_t e = hipEventQuery(R.ev);
      if (e == hipErrorNotReady) break;
      if (e != hipSuccess) (void)hipGetLastError();  // the jobs' `done` report it
      R.busy = false;
      s->inflight.pop_front();
    }
    while (static_cast<int>(s->inflight.size()) < kLaunchesInFlight && issue_launch(s)) {
    }
    std::this_thread::sleep_for(std::chrono::microseconds(20));
  }
}

void release(dh_server *s) {
  for (Slot &sl : s->slots) {
    void *dev[] = {sl.d_in, sl.d_staged, sl.d_out, sl.d_oor, sl.d_pairs, sl.d_keys};
    for (void *p : dev)
      if (p) (void)hipFree(p);
    void *host[] = {sl.h_in, sl.h_out, sl.h_oor, sl.h_pairs};
    for (void *p : host)
      if (p) (void)hipHostFree(p);
    if (sl.setup) (void)hipEventDestroy(sl.setup);
    if (sl.done) (void)hipEventDestroy(sl.done);
    sl = Slot();
  }
  for (Region &R : s->regions) {
    if (R.d_items) (void)hipFree(R.d_items);
    if (R.h_items) (void)hipHostFree(R.h_items);
    if (R.ev) (void)hipEventDestroy(R.ev);
    R = Region();
  }
  if (s->d_frames) (void)hipFree(s->d_frames);
  if (s->h_frames) (void)hipHostFree(s->h_frames);
  for (hipStream_t st : {s->compute, s->setup, s->copy})
    if (st) (void)hipStreamDestroy(st);
  (void)hipGetLastError();
}

}  // namespace

extern "C" {

int dh_server_create(int32_t device, int64_t hbm_budget_bytes, int32_t max_inflight,
                     double head_wait_limit_s, dh_server **out) {
  if (!out) return DH_EINVAL;
  *out = nullptr;
  if (hbm_budget_bytes <= 0 || max_inflight < 1 || max_inflight > 64) return DH_EINVAL;
  std::unique_ptr<dh_server> s(new (std::nothrow) dh_server);
  if (!s) return DH_ENOMEM;
  s->device = device;
  s->budget = hbm_budget_bytes;
  s->head_wait_limit = head_wait_limit_s < 0 ? 1.0 : head_wait_limit_s;
  s->slots.resize(static_cast<size_t>(max_inflight));
  int n_cu = 0, lds = 0;
  bool ok = hipSetDevice(device) == hipSuccess &&
            hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, device) ==
                hipSuccess &&
            hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) ==
                hipSuccess;
  s->n_cu = n_cu;
  s->lds_per_block = static_cast<size_t>(lds);
  for (hipStream_t *st : {&s->compute, &s->setup, &s->copy})
    ok = ok && hipStreamCreateWithFlags(st, hipStreamNonBlocking) == hipSuccess;
  ok = ok && hipMalloc(&s->d_frames, sizeof(FrameParams) * s->slots.size()) == hipSuccess &&
       hipHostMalloc(&s->h_frames, sizeof(FrameParams) * s->slots.size(),
                     hipHostMallocDefault) == hipSuccess;
  for (Slot &sl : s->slots)
    ok = ok && hipEventCreateWithFlags(&sl.setup, hipEventDisableTiming) == hipSuccess &&
         hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) == hipSuccess;
  for (Region &R : s->regions)
    ok = ok && hipMalloc(&R.d_items, region_bytes()) == hipSuccess &&
         hipHostMalloc(&R.h_items, region_bytes(), hipHostMallocDefault) == hipSuccess &&
         hipEventCreateWithFlags(&R.ev, hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    release(s.get());
    return DH_EDEVICE;
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
  j->need = job_footprint(n, j->n_hist, n_bins, precision, box_type);
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

int dh_server_launch_stats(const dh_server *s, int64_t *launches, int64_t *shared_launches,
                           int64_t *max_jobs_per_launch) {
  if (!s || !launches || !shared_launches || !max_jobs_per_launch) return DH_EINVAL;
  *launches = s->n_launches.load();
  *shared_launches = s->shared_launches.load();
  *max_jobs_per_launch = s->max_jobs_per_launch.load();
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
  release(s);
  delete s;
}

}  // extern "C"
