// dh_histo_noalloc: the single-frame histogram of dh_histo_async without any
// allocation, for callers that cannot allocate device memory (work under
// HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
//
// Everything a call needs beyond the caller's input and output lives in one
// file-scope device array, `scratch`: the frame constants, the pairs per
// histogram, the work counters, the work list and the staged coordinates.
// The host computes the frame constants and the launch shape (built-in
// defaults, no tuning) and passes them as kernel arguments; a one-workgroup
// planner kernel writes the constants and the work list into the scratch
// with the same row cutting as the host planner (hist_rows / emit_row), so
// no host buffer is copied and no pinned memory is needed. Then the library's
// own staging, zeroing and pair kernels run on the scratch.
//
// Every call on a device shares that device's array: calls that overlap on
// one device (on different streams, or from several host threads) race and
// must be serialised by the caller. The planner clears the work counters on
// every call.
#include "dh_internal.h"
#include "disthist.h"

#include <algorithm>
#include <mutex>

namespace dh {
namespace {

// Largest frame: staged coordinates take 16 bytes per point in binary32 and
// 32 in binary64, so 48 MiB holds about 1.4 million binary64 points (2.9
// million binary32) together with their work list; frames staged in spatial
// order (see staged_kind) take 32 bytes per point plus 8 bytes of sort keys
// per point rounded up to a power of two (about 1.0 million points).
constexpr size_t kScratchBytes = size_t{48} << 20;
constexpr int kMaxDevices = 64;
constexpr int kPlanThreads = 1024;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

struct DeviceSlot {
  bool ready = false;
  unsigned char *ptr = nullptr;  // device address of this device's scratch
  int n_cu = 0;
  size_t lds = 0;
};

std::mutex g_slots_mu;
DeviceSlot g_slots[kMaxDevices];

// The scratch address on the current device, found once per device (each
// device holds its own copy of the array at its own address).
int device_slot(DeviceSlot &out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return thread_fail(DH_EDEVICE, "no current HIP device");
  }
  if (dev < 0 || dev >= kMaxDevices) return thread_fail(DH_EDEVICE, "device %d", dev);
  std::lock_guard<std::mutex> lock(g_slots_mu);
  DeviceSlot &s = g_slots[dev];
  if (!s.ready) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) {
      (void)hipGetLastError();
      return thread_fail(DH_EDEVICE, "hipGetSymbolAddress of the scratch array: %s",
                         hipGetErrorString(e));
    }
    int n_cu = 0, lds = 0;
    if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) !=
            hipSuccess) {
      (void)hipGetLastError();
      return thread_fail(DH_EDEVICE, "device attributes of device %d", dev);
    }
    s.ptr = static_cast<unsigned char *>(p);
    s.n_cu = n_cu;
    s.lds = static_cast<size_t>(lds);
    s.ready = true;
  }
  out = s;
  return DH_OK;
}

constexpr int kMaxSpeciesNA = 64;

struct PlanArgs {
  int64_t off[kMaxSpeciesNA + 1];
  int32_t k;
  int32_t n_sweeps;
  int32_t n_counters;
  int64_t bi, jc;
  int64_t n_items;  // items the host counted: the list is never written past it
  FrameParams *fp_dst;
  uint64_t *pairs;
  int32_t *counters;
  WorkItem *items;
};

// One workgroup: frame constants, pairs per histogram, cleared counters, and
// the work list grouped by (histogram, bin window) as the host plan groups it.
__global__ __launch_bounds__(kPlanThreads) void noalloc_plan_kernel(FrameParams fp, PlanArgs a) {
  __shared__ int64_t off[kMaxSpeciesNA + 1];
  __shared__ int64_t scan[kPlanThreads];
  const int tid = threadIdx.x;
  for (int s = tid; s <= a.k; s += blockDim.x) off[s] = a.off[s];
  if (tid == 0) *a.fp_dst = fp;
  for (int c = tid; c < a.n_counters; c += blockDim.x) a.counters[c] = 0;
  __syncthreads();
  const int32_t n_hist = a.k * (a.k + 1) / 2;
  for (int h = tid; h < n_hist; h += blockDim.x) a.pairs[h] = hist_rows(off, a.k, h).pairs;
  int64_t base = 0;
  for (int32_t h = 0; h < n_hist; ++h) {
    const HistRows r = hist_rows(off, a.k, h);
    const int64_t nr = hist_row_count(r, a.bi);
    for (int32_t sw = 0; sw < a.n_sweeps; ++sw) {
      for (int64_t r0 = 0; r0 < nr; r0 += blockDim.x) {
        const int64_t row = r0 + tid;
        const int64_t cnt = row < nr ? row_item_count(r, row, a.bi, a.jc) : 0;
        scan[tid] = cnt;
        __syncthreads();
        for (int o = 1; o < static_cast<int>(blockDim.x); o <<= 1) {
          const int64_t v = tid >= o ? scan[tid - o] : 0;
          __syncthreads();
          scan[tid] += v;
          __syncthreads();
        }
        const int64_t at = base + scan[tid] - cnt;
        if (cnt > 0 && at + cnt <= a.n_items) emit_row(r, h, sw, row, a.bi, a.jc, a.items + at);
        base += scan[blockDim.x - 1];
        __syncthreads();
      }
    }
  }
}

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

}  // namespace
}  // namespace dh

using namespace dh;

extern "C" int dh_histo_noalloc(dh_stream stream, const double *d_coords,
                                const int64_t *offsets, int32_t n_species, int32_t box_type,
                                const double *box, double r_max, int32_t n_bins,
                                int32_t precision, uint64_t *d_out, uint64_t *d_out_of_range) {
  int rc = dh_check_args(nullptr, offsets, n_species, box_type, box, r_max, n_bins, precision);
  if (rc) return thread_fail(rc, "invalid arguments");
  const int64_t n = offsets[n_species];
  if (!d_out || (n > 0 && !d_coords)) return thread_fail(DH_EINVAL, "null device pointer");
  const size_t coord_bytes = precision == DH_FP64 ? 32 : 16;
  // the staged copy alone must fit; checked before any device call
  if (static_cast<size_t>(n) * coord_bytes > kScratchBytes)
    return thread_fail(DH_EINVAL,
                       "%lld points need %zu bytes of staged coordinates; the allocation-free "
                       "entry point has %zu bytes of scratch",
                       static_cast<long long>(n), static_cast<size_t>(n) * coord_bytes,
                       kScratchBytes);
  DeviceSlot dev;
  rc = device_slot(dev);
  if (rc) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);

  FrameParams fp;
  const int kind =
      staged_kind(frame_constants(box_type, box, r_max, n_bins, fp), precision, fp.L, n);
  fp.box = kind;
  const size_t point_bytes = staged_point_bytes(precision, kind);
  const size_t keys_bytes =
      kind == kBoxTricSorted ? static_cast<size_t>(sort_keys_count(n)) * sizeof(uint64_t) : 0;
  const int32_t n_hist = n_species * (n_species + 1) / 2;
  uint64_t total = 0;
  for (int32_t h = 0; h < n_hist; ++h) total += hist_rows(offsets, n_species, h).pairs;
  const LaunchPlan L = default_launch(dev.n_cu, dev.lds, precision, fp, total);
  const int64_t bi = static_cast<int64_t>(L.cfg.threads) * L.cfg.r;
  const int64_t jc = L.cfg.jchunk;
  int64_t n_items = 0;
  for (int32_t h = 0; h < n_hist; ++h) {
    const HistRows r = hist_rows(offsets, n_species, h);
    const int64_t nr = hist_row_count(r, bi);
    for (int64_t row = 0; row < nr; ++row) n_items += row_item_count(r, row, bi, jc);
  }
  n_items *= L.n_sweeps;

  // scratch layout: constants | pairs | counters (work counter, then the
  // 8-byte image-search count) | work list | sort keys (spatially sorted
  // frames) | staged coordinates
  const size_t off_fp = 0;
  const size_t off_pairs = align256(off_fp + sizeof(FrameParams));
  const size_t off_counters = align256(off_pairs + static_cast<size_t>(n_hist) * sizeof(uint64_t));
  const int32_t n_counters = 6;
  const size_t off_items = align256(off_counters + n_counters * sizeof(int32_t));
  const size_t off_keys = align256(off_items + static_cast<size_t>(n_items) * sizeof(WorkItem));
  const size_t off_staged = align256(off_keys + keys_bytes);
  const size_t need = off_staged + std::max<size_t>(1, static_cast<size_t>(n)) * point_bytes;
  if (need > kScratchBytes)
    return thread_fail(DH_EINVAL,
                       "the frame needs %zu bytes of scratch (%lld points, %lld work items); the "
                       "allocation-free entry point has %zu",
                       need, static_cast<long long>(n), static_cast<long long>(n_items),
                       kScratchBytes);
  unsigned char *base = dev.ptr;
  int32_t *counters = reinterpret_cast<int32_t *>(base + off_counters);
  fp.coords = base + off_staged;
  fp.out = d_out;
  fp.win = L.win;
  fp.n_sweeps = L.n_sweeps;
  fp.noclamp = L.noclamp ? 1 : 0;
  const bool oor_flush = d_out_of_range != nullptr && L.mode != kModeGlobal;
  fp.oor = oor_flush ? d_out_of_range : nullptr;
  fp.oor_by_flush = oor_flush ? 1 : 0;
  fp.searched = kind == kBoxTricSearch ? reinterpret_cast<unsigned long long *>(counters + 2)
                                       : nullptr;

  PlanArgs pa;
  for (int s = 0; s <= n_species; ++s) pa.off[s] = offsets[s];
  for (int s = n_species + 1; s <= kMaxSpeciesNA; ++s) pa.off[s] = offsets[n_species];
  pa.k = n_species;
  pa.n_sweeps = L.n_sweeps;
  pa.n_counters = n_counters;
  pa.bi = bi;
  pa.jc = jc;
  pa.n_items = n_items;
  pa.fp_dst = reinterpret_cast<FrameParams *>(base + off_fp);
  pa.pairs = reinterpret_cast<uint64_t *>(base + off_pairs);
  pa.counters = counters;
  pa.items = reinterpret_cast<WorkItem *>(base + off_items);
  noalloc_plan_kernel<<<1, kPlanThreads, 0, st>>>(fp, pa);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess)
    e = kind == kBoxTricSorted
            ? launch_stage_sorted(precision, d_coords, base + off_staged, n, offsets, n_species, fp,
                                  reinterpret_cast<uint64_t *>(base + off_keys), st)
            : launch_stage(precision, kind, d_coords, base + off_staged, n, fp, st);
  // the counters were cleared by the planner: none passed here
  if (e == hipSuccess)
    e = launch_zero(d_out, static_cast<int64_t>(n_hist) * n_bins, nullptr, 0, fp.oor, pa.pairs,
                    n_hist, st);
  if (e == hipSuccess && n_items > 0) {
    PairKernelArgs a;
    a.frames = pa.fp_dst;
    a.items = pa.items;
    a.counter = counters;
    a.n_items = static_cast<int32_t>(n_items);
    a.copies = L.cfg.copies;
    a.stride = L.stride;
    a.tj = L.cfg.tj;
    const int grid = std::max(1, std::min<int>(L.grid, a.n_items));
    e = launch_pairs(precision, kind, L.mode, L.cfg, a, grid, L.lds, st);
  }
  if (e == hipSuccess && d_out_of_range && !oor_flush)
    e = launch_oor(d_out, n_hist, n_bins, pa.pairs, d_out_of_range, st);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return thread_fail(DH_EDEVICE, "launch failed: %s", hipGetErrorString(e));
  }
  return DH_OK;
}
