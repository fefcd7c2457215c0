// Trajectory engine of libdisthist: frames of a trajectory file are read by a
// host thread into pinned buffers, copied to the device on a copy stream
// while the previous frame is histogrammed on a compute stream, and summed
// over consecutive intervals of frames (the paper's engine sums histograms
// over frame intervals in its writer, Sec. 3.3 and Sec. 4.4). Every finished
// interval is appended to a results file, which is also the checkpoint: a
// later call with the same parameters skips the intervals already there.
//
// Hybrid mode (the paper's CPU and GPU workers side by side, Sec. 3.3 and
// Table 4): a CPU worker thread runs the library's CPU kernel on whole
// frames taken from the end of the current interval, while the GPU takes
// them from the start; the interval's record adds both. The CPU takes a
// frame only if its measured time per frame is below the GPU's time for the
// frames still unclaimed besides it, so it never holds an interval back by
// more than about one GPU frame (DH_HYBRID_GREEDY lifts that rule).
#include "disthist.h"
#include "dh_internal.h"

#include <fcntl.h>
#include <sys/stat.h>
#include <unistd.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <mutex>
#include <thread>
#include <vector>

namespace {

constexpr char kTrajMagic[8] = {'D', 'H', 'T', 'R', 'A', 'J', '0', '1'};
constexpr char kResMagic[8] = {'D', 'H', 'R', 'E', 'S', '0', '0', '1'};
constexpr int64_t kTrajHeader = 64;
constexpr int64_t kResHeader = 128;

// FNV-1a over the bytes of the parameters a results file belongs to.
uint64_t fnv(uint64_t h, const void *p, size_t n) {
  const unsigned char *b = static_cast<const unsigned char *>(p);
  for (size_t k = 0; k < n; ++k) {
    h ^= b[k];
    h *= 1099511628211ull;
  }
  return h;
}

bool read_all(int fd, void *buf, size_t n, int64_t off) {
  char *p = static_cast<char *>(buf);
  while (n > 0) {
    const ssize_t r = pread(fd, p, n, off);
    if (r <= 0) return false;
    p += r;
    n -= static_cast<size_t>(r);
    off += r;
  }
  return true;
}

bool write_all(int fd, const void *buf, size_t n) {
  const char *p = static_cast<const char *>(buf);
  while (n > 0) {
    const ssize_t r = write(fd, p, n);
    if (r <= 0) return false;
    p += r;
    n -= static_cast<size_t>(r);
  }
  return true;
}

struct ResHeader {
  char magic[8];
  uint64_t params;  // hash of everything below and of the species offsets
  int64_t frame_begin, frame_end, interval;
  int32_t n_species, n_bins, precision, box_type;
  double r_max;
  int64_t n_points, traj_frames;
  char pad[kResHeader - 8 - 8 - 24 - 16 - 8 - 16];
};
static_assert(sizeof(ResHeader) == kResHeader, "results header size");

// Claims of the current interval's frames: the GPU takes [lo, ...) from the
// start, the CPU worker (lo, hi] from the end.
struct Hybrid {
  std::mutex mu;
  std::condition_variable cv;
  int64_t lo = 0, hi = 0;  // unclaimed frames [lo, hi)
  bool open = false;       // the current interval takes claims
  bool busy = false;       // the CPU worker is computing a frame
  bool quit = false;
  bool greedy = false;
  std::vector<uint64_t> sum;  // CPU frames' histograms of the interval
  std::vector<uint64_t> pairs;  // and their pair counts per histogram
  int64_t frames = 0, total_frames = 0;
  double gpu_s = 0.0, cpu_s = 0.0;  // seconds per frame (running estimates)
  int rc = DH_OK;
  // worth a CPU frame: the GPU stays busy longer with the other frames
  bool cpu_takes() const {
    if (hi <= lo) return false;
    if (greedy) return true;
    return cpu_s > 0.0 && gpu_s > 0.0 && cpu_s < static_cast<double>(hi - lo - 1) * gpu_s;
  }
};

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

}  // namespace

struct dh_traj {
  int fd = -1;
  int64_t n_frames = 0, n_points = 0;
  int32_t box_type = 0;
  int64_t frame_bytes = 0;  // 9 box doubles + 3 N coordinates
};

extern "C" {

int dh_traj_open(const char *path, dh_traj **out) {
  if (!path || !out) return DH_EINVAL;
  *out = nullptr;
  const int fd = open(path, O_RDONLY);
  if (fd < 0) return DH_EINVAL;
  char hdr[kTrajHeader];
  struct stat st;
  int64_t nf = 0, np = 0;
  int32_t bt = 0;
  bool ok = read_all(fd, hdr, sizeof hdr, 0) && std::memcmp(hdr, kTrajMagic, 8) == 0 &&
            fstat(fd, &st) == 0;
  if (ok) {
    std::memcpy(&nf, hdr + 8, 8);
    std::memcpy(&np, hdr + 16, 8);
    std::memcpy(&bt, hdr + 24, 4);
    ok = nf >= 0 && np >= 0 && np <= (int64_t{1} << 31) - 1 && bt >= DH_BOX_NONE &&
         bt <= DH_BOX_TRICLINIC &&
         st.st_size == kTrajHeader + nf * (72 + 24 * np);
  }
  if (!ok) {
    close(fd);
    return DH_EINVAL;
  }
  dh_traj *t = new (std::nothrow) dh_traj;
  if (!t) {
    close(fd);
    return DH_ENOMEM;
  }
  t->fd = fd;
  t->n_frames = nf;
  t->n_points = np;
  t->box_type = bt;
  t->frame_bytes = 72 + 24 * np;
  *out = t;
  return DH_OK;
}

int dh_traj_info(const dh_traj *t, int64_t *n_frames, int64_t *n_points, int32_t *box_type) {
  if (!t) return DH_EINVAL;
  if (n_frames) *n_frames = t->n_frames;
  if (n_points) *n_points = t->n_points;
  if (box_type) *box_type = t->box_type;
  return DH_OK;
}

void dh_traj_close(dh_traj *t) {
  if (!t) return;
  if (t->fd >= 0) close(t->fd);
  delete t;
}

int dh_traj_histo(dh_ctx *ctx, dh_traj *t, const int64_t *offsets, int32_t n_species,
                  double r_max, int32_t n_bins, int32_t precision, int64_t frame_begin,
                  int64_t frame_end, int64_t interval, const char *results_path,
                  int64_t max_intervals, int64_t *intervals_done) {
  return dh_traj_histo_hybrid(ctx, t, offsets, n_species, r_max, n_bins, precision, frame_begin,
                              frame_end, interval, results_path, max_intervals, 0, 0,
                              intervals_done, nullptr);
}

int dh_traj_histo_hybrid(dh_ctx *ctx, dh_traj *t, const int64_t *offsets, int32_t n_species,
                         double r_max, int32_t n_bins, int32_t precision, int64_t frame_begin,
                         int64_t frame_end, int64_t interval, const char *results_path,
                         int64_t max_intervals, int32_t cpu_threads, int32_t flags,
                         int64_t *intervals_done, int64_t *cpu_frames) {
  if (cpu_frames) *cpu_frames = 0;
  if (!ctx || !t || !offsets || !results_path || interval < 1 || max_intervals < 0 ||
      frame_begin < 0 || frame_end < frame_begin || frame_end > t->n_frames || cpu_threads < 0 ||
      (flags & ~DH_HYBRID_GREEDY) != 0)
    return DH_EINVAL;
  if (n_species < 1 || n_species > 64 || offsets[0] != 0 || offsets[n_species] != t->n_points)
    return DH_EINVAL;
  // everything but the per-frame boxes (checked frame by frame below)
  const int arc = dh_check_args(nullptr, offsets, n_species, DH_BOX_NONE, nullptr, r_max, n_bins,
                                precision);
  if (arc) return arc;
  // each frame's box and the other arguments are validated as the frame is
  // processed (an invalid frame stops the run before its interval is written)
  const int32_t n_hist = n_species * (n_species + 1) / 2;
  const int64_t n_int = (frame_end - frame_begin + interval - 1) / interval;
  const size_t hist_words = static_cast<size_t>(n_hist) * n_bins;
  const size_t rec_bytes = (hist_words + n_hist + 1) * sizeof(uint64_t);

  // results file: header, then one record per finished interval
  ResHeader want;
  std::memset(&want, 0, sizeof want);
  std::memcpy(want.magic, kResMagic, 8);
  want.frame_begin = frame_begin;
  want.frame_end = frame_end;
  want.interval = interval;
  want.n_species = n_species;
  want.n_bins = n_bins;
  want.precision = precision;
  want.box_type = t->box_type;
  want.r_max = r_max;
  want.n_points = t->n_points;
  want.traj_frames = t->n_frames;
  uint64_t h = fnv(1469598103934665603ull, &want.frame_begin, sizeof want - 16);
  want.params = fnv(h, offsets, sizeof(int64_t) * (n_species + 1));

  const int rfd = open(results_path, O_RDWR | O_CREAT, 0644);
  if (rfd < 0) return DH_EINVAL;
  struct stat rst;
  if (fstat(rfd, &rst) != 0) {
    close(rfd);
    return DH_EINVAL;
  }
  int64_t done = 0;
  if (rst.st_size == 0) {
    if (!write_all(rfd, &want, sizeof want)) {
      close(rfd);
      return DH_EINVAL;
    }
  } else {
    ResHeader have;
    if (!read_all(rfd, &have, sizeof have, 0) ||
        std::memcmp(&have, &want, sizeof want) != 0) {
      close(rfd);
      return DH_EINVAL;  // another run's results, or not a results file
    }
    // complete records only: a partial last record (interrupted write) is
    // cut off and its interval recomputed
    done = std::min<int64_t>(n_int, (rst.st_size - kResHeader) / static_cast<int64_t>(rec_bytes));
    if (ftruncate(rfd, kResHeader + done * static_cast<int64_t>(rec_bytes)) != 0) {
      close(rfd);
      return DH_EINVAL;
    }
  }
  if (lseek(rfd, kResHeader + done * static_cast<int64_t>(rec_bytes), SEEK_SET) < 0) {
    close(rfd);
    return DH_EINVAL;
  }
  int64_t last = n_int;
  if (max_intervals > 0) last = std::min(n_int, done + max_intervals);
  if (done >= last) {
    if (intervals_done) *intervals_done = done;
    close(rfd);
    return DH_OK;
  }

  int rc = DH_OK;
  if (hipSetDevice(dh::ctx_device(ctx)) != hipSuccess) rc = DH_EDEVICE;
  const int64_t f0 = frame_begin + done * interval;
  const int64_t f1 = std::min(frame_end, frame_begin + last * interval);

  // device and pinned buffers: two frame slots each
  constexpr int kSlots = 2;
  double *d_in[kSlots] = {nullptr, nullptr};
  double *h_in[kSlots] = {nullptr, nullptr};
  uint64_t *d_out = nullptr, *h_out = nullptr;
  hipStream_t s_copy = nullptr, s_comp = nullptr;
  hipEvent_t copied[kSlots] = {}, consumed[kSlots] = {}, out_ready = nullptr;
  const size_t fbytes = static_cast<size_t>(t->frame_bytes);
  for (int k = 0; k < kSlots && !rc; ++k) {
    if (hipMalloc(&d_in[k], std::max<size_t>(fbytes, 8)) != hipSuccess ||
        hipHostMalloc(&h_in[k], std::max<size_t>(fbytes, 8), hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&copied[k], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&consumed[k], hipEventDisableTiming) != hipSuccess)
      rc = DH_ENOMEM;
  }
  if (!rc && (hipMalloc(&d_out, hist_words * 8) != hipSuccess ||
              hipHostMalloc(&h_out, hist_words * 8, hipHostMallocDefault) != hipSuccess))
    rc = DH_ENOMEM;
  if (!rc && (hipStreamCreateWithFlags(&s_copy, hipStreamNonBlocking) != hipSuccess ||
              hipStreamCreateWithFlags(&s_comp, hipStreamNonBlocking) != hipSuccess ||
              hipEventCreateWithFlags(&out_ready, hipEventDisableTiming) != hipSuccess))
    rc = DH_EDEVICE;

  // reader thread: fills host slot k with frame f once the copy of the frame
  // that used the slot before has completed
  std::mutex mu;
  std::condition_variable cv;
  std::vector<int> filled(kSlots, -1);  // frame index held by a host slot
  std::vector<bool> free_slot(kSlots, true);
  bool reader_failed = false, stop = false;
  std::thread reader;
  if (!rc) {
    reader = std::thread([&] {
      for (int64_t f = f0; f < f1; ++f) {
        const int k = static_cast<int>((f - f0) % kSlots);
        {
          std::unique_lock<std::mutex> lk(mu);
          cv.wait(lk, [&] { return free_slot[k] || stop; });
          if (stop) return;
          free_slot[k] = false;
        }
        const bool ok = read_all(t->fd, h_in[k], fbytes, kTrajHeader + f * t->frame_bytes);
        {
          std::lock_guard<std::mutex> lk(mu);
          if (!ok) reader_failed = true;
          filled[k] = static_cast<int>(f - f0);
        }
        cv.notify_all();
        if (!ok) return;
      }
    });
  }

  // CPU worker: whole frames from the end of the open interval
  Hybrid hy;
  hy.greedy = (flags & DH_HYBRID_GREEDY) != 0;
  hy.sum.assign(hist_words, 0);
  hy.pairs.assign(n_hist, 0);
  std::thread cpu;
  if (!rc && cpu_threads > 0) {
    cpu = std::thread([&] {
      std::vector<double> frame(static_cast<size_t>(t->frame_bytes / 8));
      std::vector<uint64_t> out(hist_words), oor(n_hist);
      while (true) {
        int64_t f;
        {
          std::unique_lock<std::mutex> lk(hy.mu);
          hy.cv.wait(lk, [&] { return hy.quit || (hy.open && hy.cpu_takes()); });
          if (hy.quit) return;
          f = --hy.hi;
          hy.busy = true;
        }
        const double t0 = now_s();
        int frc = read_all(t->fd, frame.data(), fbytes, kTrajHeader + f * t->frame_bytes)
                      ? DH_OK
                      : DH_EINVAL;
        if (!frc)
          frc = dh_cpu_histo(frame.data() + 9, offsets, n_species, t->box_type,
                             t->box_type == DH_BOX_NONE ? nullptr : frame.data(), r_max, n_bins,
                             precision, cpu_threads, out.data(), oor.data());
        const double dt = now_s() - t0;
        {
          std::lock_guard<std::mutex> lk(hy.mu);
          if (frc) {
            hy.rc = frc;
          } else {
            for (size_t q = 0; q < hist_words; ++q) hy.sum[q] += out[q];
            for (int hh = 0; hh < n_hist; ++hh) {
              uint64_t in_range = 0;
              for (int32_t b = 0; b < n_bins; ++b) in_range += out[static_cast<size_t>(hh) * n_bins + b];
              hy.pairs[hh] += in_range + oor[hh];
            }
            ++hy.frames;
            ++hy.total_frames;
          }
          hy.cpu_s = hy.cpu_s > 0.0 ? 0.5 * (hy.cpu_s + dt) : dt;
          hy.busy = false;
        }
        hy.cv.notify_all();
      }
    });
  }
  // before the first CPU frame its time per frame is unknown: assume 2e8
  // pairs per second per thread, a low rate for the CPU kernel
  {
    uint64_t fp_pairs = 0;
    for (int32_t hh = 0; hh < n_hist; ++hh) fp_pairs += dh::hist_rows(offsets, n_species, hh).pairs;
    hy.cpu_s = cpu_threads > 0 ? static_cast<double>(fp_pairs) / (2e8 * cpu_threads) : 0.0;
  }

  std::vector<uint64_t> rec(hist_words + n_hist + 1);
  std::vector<uint64_t> pairs(n_hist);
  int64_t cur_interval = done;
  int64_t frames_in = 0;
  std::vector<uint64_t> hist_pairs(n_hist, 0);
  double t_prev = 0.0;  // when the GPU took its previous frame
  for (int64_t f = f0; f < f1 && !rc; ++f) {
    const int k = static_cast<int>((f - f0) % kSlots);
    const int64_t int_begin = frame_begin + cur_interval * interval;
    const int64_t int_end = std::min(frame_end, int_begin + interval);
    if (f == int_begin) {
      // open the interval for claims
      std::lock_guard<std::mutex> lk(hy.mu);
      hy.lo = int_begin;
      hy.hi = int_end;
      hy.open = cpu_threads > 0;
      hy.frames = 0;
      std::fill(hy.sum.begin(), hy.sum.end(), 0);
      std::fill(hy.pairs.begin(), hy.pairs.end(), 0);
    }
    if (cpu_threads > 0) hy.cv.notify_all();
    {
      std::unique_lock<std::mutex> lk(mu);
      cv.wait(lk, [&] { return filled[k] == static_cast<int>(f - f0) || reader_failed; });
      if (reader_failed && filled[k] != static_cast<int>(f - f0)) {
        rc = DH_EINVAL;
        break;
      }
    }
    bool cpu_frame = false;
    {
      std::lock_guard<std::mutex> lk(hy.mu);
      if (f >= hy.hi) {
        cpu_frame = true;  // taken by the CPU worker
      } else {
        hy.lo = f + 1;
        const double now = now_s();
        if (t_prev > 0.0 && f > int_begin)
          hy.gpu_s = hy.gpu_s > 0.0 ? 0.5 * (hy.gpu_s + (now - t_prev)) : now - t_prev;
        t_prev = now;
      }
    }
    if (cpu_frame) {
      // the reader's copy of this frame is not needed
      {
        std::lock_guard<std::mutex> lk(mu);
        free_slot[k] = true;
      }
      cv.notify_all();
    } else {
    // the device slot must be free: the compute of its previous frame is done
    if (hipStreamWaitEvent(s_copy, consumed[k], 0) != hipSuccess) {
      rc = DH_EDEVICE;
      break;
    }
    if (hipMemcpyAsync(d_in[k], h_in[k], fbytes, hipMemcpyHostToDevice, s_copy) != hipSuccess ||
        hipEventRecord(copied[k], s_copy) != hipSuccess) {
      rc = DH_EDEVICE;
      break;
    }
    // the host slot is reusable once its copy has completed
    if (hipEventSynchronize(copied[k]) != hipSuccess) {
      rc = DH_EDEVICE;
      break;
    }
    double box[9];
    std::memcpy(box, h_in[k], sizeof box);
    {
      std::lock_guard<std::mutex> lk(mu);
      free_slot[k] = true;
    }
    cv.notify_all();
    if (hipStreamWaitEvent(s_comp, copied[k], 0) != hipSuccess) {
      rc = DH_EDEVICE;
      break;
    }
    const bool first = frames_in == 0;
    // zero the interval's sums by a kernel on the compute stream
    if (first) {
      rc = dh::zero_u64(d_out, static_cast<int64_t>(hist_words), s_comp);
      if (rc) break;
    }
    uint64_t total = 0;
    rc = dh::histo_job(ctx, s_comp, d_in[k] + 9, offsets, n_species, t->box_type,
                       t->box_type == DH_BOX_NONE ? nullptr : box, r_max, n_bins, precision,
                       d_out, nullptr, true, &total);
    if (rc) break;
    if (hipEventRecord(consumed[k], s_comp) != hipSuccess) {
      rc = DH_EDEVICE;
      break;
    }
    // per-histogram pair counts of this frame (for the out-of-range counts)
    for (int s = 0, hh = 0; s < n_species; ++s, ++hh) {
      const uint64_t a = static_cast<uint64_t>(offsets[s + 1] - offsets[s]);
      hist_pairs[hh] += a * (a > 0 ? a - 1 : 0) / 2;
    }
    for (int s = 0, hh = n_species; s < n_species; ++s)
      for (int u = s + 1; u < n_species; ++u, ++hh)
        hist_pairs[hh] += static_cast<uint64_t>(offsets[s + 1] - offsets[s]) *
                          static_cast<uint64_t>(offsets[u + 1] - offsets[u]);
    ++frames_in;
    }  // GPU frame
    if (f + 1 == int_end) {
      // interval finished: close it to claims, wait for the CPU worker's
      // frame, copy the GPU sums out, add the CPU sums, append the record
      int64_t cpu_n = 0;
      {
        std::unique_lock<std::mutex> lk(hy.mu);
        hy.open = false;
        hy.cv.wait(lk, [&] { return !hy.busy; });
        if (hy.rc) rc = hy.rc;
        cpu_n = hy.frames;
        for (int hh = 0; hh < n_hist; ++hh) hist_pairs[hh] += hy.pairs[hh];
      }
      if (rc) break;
      if (frames_in == 0) {
        // every frame of the interval ran on the CPU: the device sums were
        // never zeroed for it
        rc = dh::zero_u64(d_out, static_cast<int64_t>(hist_words), s_comp);
        if (rc) break;
      }
      if (hipMemcpyAsync(h_out, d_out, hist_words * 8, hipMemcpyDeviceToHost, s_comp) !=
              hipSuccess ||
          hipEventRecord(out_ready, s_comp) != hipSuccess ||
          hipEventSynchronize(out_ready) != hipSuccess) {
        rc = DH_EDEVICE;
        break;
      }
      for (size_t q = 0; q < hist_words; ++q) h_out[q] += hy.sum[q];
      frames_in += cpu_n;
      std::memcpy(rec.data(), h_out, hist_words * 8);
      for (int hh = 0; hh < n_hist; ++hh) {
        uint64_t in_range = 0;
        for (int32_t b = 0; b < n_bins; ++b) in_range += h_out[static_cast<size_t>(hh) * n_bins + b];
        rec[hist_words + hh] = hist_pairs[hh] - in_range;
      }
      rec[hist_words + n_hist] = static_cast<uint64_t>(frames_in);
      if (!write_all(rfd, rec.data(), rec_bytes) || fsync(rfd) != 0) {
        rc = DH_EINVAL;
        break;
      }
      ++cur_interval;
      frames_in = 0;
      std::fill(hist_pairs.begin(), hist_pairs.end(), 0);
    }
  }
  if (reader.joinable()) {
    {
      std::lock_guard<std::mutex> lk(mu);
      stop = true;
    }
    cv.notify_all();
    reader.join();
  }
  if (cpu.joinable()) {
    {
      std::lock_guard<std::mutex> lk(hy.mu);
      hy.quit = true;
    }
    hy.cv.notify_all();
    cpu.join();
  }
  if (cpu_frames) *cpu_frames = hy.total_frames;
  if (s_comp) (void)hipStreamSynchronize(s_comp);
  if (s_copy) (void)hipStreamSynchronize(s_copy);
  for (int k = 0; k < kSlots; ++k) {
    if (d_in[k]) (void)hipFree(d_in[k]);
    if (h_in[k]) (void)hipHostFree(h_in[k]);
    if (copied[k]) (void)hipEventDestroy(copied[k]);
    if (consumed[k]) (void)hipEventDestroy(consumed[k]);
  }
  if (d_out) (void)hipFree(d_out);
  if (h_out) (void)hipHostFree(h_out);
  if (out_ready) (void)hipEventDestroy(out_ready);
  if (s_copy) (void)hipStreamDestroy(s_copy);
  if (s_comp) (void)hipStreamDestroy(s_comp);
  (void)hipGetLastError();
  close(rfd);
  if (intervals_done) *intervals_done = cur_interval;
  return rc;
}

}  // extern "C"
