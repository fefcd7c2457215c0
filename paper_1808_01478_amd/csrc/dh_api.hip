// Host side of libdisthist: argument validation, frame constants, the work
// planner, device contexts and the C entry points declared in disthist.h.
#include "disthist.h"
#include "dh_internal.h"

#include <algorithm>
#include <array>
#include <fstream>
#include <sstream>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

using namespace dh;

struct dh_ctx {
  int device = 0;
  int n_cu = 0;
  size_t lds_per_block = 0;
  hipStream_t own_stream = nullptr;
  void *d_staged = nullptr;
  size_t staged_cap = 0;
  void *d_keys = nullptr;  // sort keys of spatially sorted frames
  size_t keys_cap = 0;
  void *d_blob = nullptr;
  size_t blob_cap = 0;
  void *h_blob = nullptr;
  size_t hblob_cap = 0;
  hipEvent_t blob_evt = nullptr;
  bool blob_pending = false;
  // bytes of the last work blob uploaded to d_blob (its counters excepted):
  // an identical plan is not uploaded again
  std::vector<char> blob_last;
  double *d_in = nullptr;
  size_t in_cap = 0;
  uint64_t *d_out = nullptr;
  size_t out_cap = 0;
  // device memory budget of the context's scratch and its live batches
  // (0: none), and the device bytes those batches hold
  size_t budget = 0;
  size_t batch_bytes = 0;
  std::string last_error;
  std::mutex mu;
  std::string arch;
  // launch tuning (see dh_ctx_set_tuning)
  int tune_mode = 0;
  std::string tune_path;
  std::map<std::string, std::array<int32_t, 8>> tune_cache;   // launch knobs per bucket
  bool forced = false;
  std::array<int32_t, 8> forced_knobs{};
  std::array<int32_t, 13> last_config{};
  // pairs per pair-kernel launch at most (0: one launch per frame)
  uint64_t launch_pairs = 0;
  // stepped job: pair-kernel launches held back for dh::step_job, then the
  // closing out-of-range pass (global-atomic launches only; LDS launches
  // count out-of-range pairs in their flushes)
  struct HeldLaunch {
    int precision, kind, mode;
    KernelConfig cfg;
    PairKernelArgs args;
    int grid;
    size_t lds;
    uint64_t pairs;
  };
  bool hold = false;
  std::vector<HeldLaunch> held;
  size_t held_next = 0;
  uint64_t held_left = 0;
  bool held_oor = false;
  uint64_t *oor_hist = nullptr, *oor_out = nullptr;
  int32_t oor_n_hist = 0, oor_n_bins = 0;
  const uint64_t *oor_pairs = nullptr;
  // kernel timing: event pairs recorded around pair-kernel launches
  bool profile = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_events;
  size_t prof_used = 0;
  // image-search pair counter of the last single-frame call (in the work
  // blob), null when that call ran no image search
  unsigned long long *searched_dev = nullptr;
};

struct dh_batch {
  struct Group {
    int kind = 0;
    int mode = kModeLds;
    KernelConfig cfg{};
    int stride = 0, grid = 0;
    size_t lds = 0;
    size_t item_begin = 0, item_count = 0;
  };
  dh_ctx *ctx = nullptr;
  int precision = 0;
  int32_t n_frames = 0;
  int64_t max_points = 0, max_words = 0;
  int32_t max_hist = 0;
  bool any_oor = false;
  void *d_staged = nullptr;
  void *d_blob = nullptr;
  size_t budget_bytes = 0;  // device bytes counted against the context's budget
  size_t off_frames = 0, off_items = 0, off_counters = 0;
  std::vector<Group> groups;
  // spatially sorted frames (staged by their own sort, not the batched
  // staging kernel): frame index, input, staged copy, species offsets
  struct Sorted {
    int32_t frame;
    const double *d_in;
    void *staged;
    std::vector<int64_t> offsets;
    FrameParams fp;
  };
  std::vector<Sorted> sorted;
  void *d_keys = nullptr;
  int64_t n_items = 0;
  double total_pairs = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

constexpr int32_t kMaxSpecies = 64;
constexpr int32_t kMaxBins = 1 << 24;
// binary32 bins come from t + (2^23 - 1/2), exact for t < 2^22
constexpr int32_t kMaxBins32 = 1 << 22;
constexpr int64_t kMaxN = 2147483647LL;

// message of the last failure that had no context to hold it (a fixed
// buffer: recording an error allocates nothing)
thread_local char t_last_error[512];

int fail(dh_ctx *ctx, int code, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(t_last_error, sizeof t_last_error, fmt, ap);
  va_end(ap);
  if (ctx) ctx->last_error = t_last_error;
  return code;
}

#define DH_HIP(ctx, call)                                                              \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail((ctx), DH_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_));   \
  } while (0)

bool box_ok(int32_t box_type, const double *box) {
  if (box_type == DH_BOX_NONE) return true;
  if (box_type != DH_BOX_ORTHO && box_type != DH_BOX_TRICLINIC) return false;
  if (!box) return false;
  for (int k = 0; k < 9; ++k)
    if (!std::isfinite(box[k])) return false;
  const double ax = box[0], ay = box[1], az = box[2];
  const double bx = box[3], by = box[4], bz = box[5];
  const double cx = box[6], cy = box[7], cz = box[8];
  if (!(ax > 0 && by > 0 && cz > 0)) return false;
  if (ay != 0 || az != 0 || bz != 0) return false;
  if (box_type == DH_BOX_ORTHO) return bx == 0 && cx == 0 && cy == 0;
  // reduced triclinic cell
  return std::fabs(bx) <= 0.5 * ax && std::fabs(cx) <= 0.5 * ax && std::fabs(cy) <= 0.5 * by;
}

int check(const double *coords, const int64_t *offsets, int32_t n_species, int32_t box_type,
          const double *box, double r_max, int32_t n_bins, int32_t precision) {
  if (!offsets || n_species < 1 || n_species > kMaxSpecies) return DH_EINVAL;
  if (offsets[0] != 0) return DH_EINVAL;
  for (int s = 0; s < n_species; ++s)
    if (offsets[s + 1] < offsets[s]) return DH_EINVAL;
  const int64_t n = offsets[n_species];
  if (n > kMaxN) return DH_EINVAL;
  if (!(r_max > 0) || !std::isfinite(r_max)) return DH_EINVAL;
  if (n_bins < 1 || n_bins > kMaxBins) return DH_EINVAL;
  if (precision != DH_FP32 && precision != DH_FP64) return DH_EINVAL;
  if (precision == DH_FP32 && n_bins > kMaxBins32) return DH_EINVAL;
  if (!box_ok(box_type, box)) return DH_EINVAL;
  if (coords)
    for (int64_t i = 0; i < 3 * n; ++i)
      if (!std::isfinite(coords[i])) return DH_EINVAL;
  return DH_OK;
}

// smallest face-to-face width of a lower-triangular cell
double min_width_tri(double ax, double bx, double by, double cx, double cy, double cz) {
  const double vol = ax * by * cz;
  const double wc = cz;
  const double wb = vol / (ax * std::sqrt(cy * cy + cz * cz));
  const double bc0 = by * cz, bc1 = -bx * cz, bc2 = bx * cy - by * cx;
  const double wa = vol / std::sqrt(bc0 * bc0 + bc1 * bc1 + bc2 * bc2);
  return std::min(wa, std::min(wb, wc));
}

// The images of the 27-image search that can be nearer than a reduced
// vector d, for each octant of d's fractional coordinates f = B^-1 d. An
// image d + S (S = B n) is nearer iff g(f) = 2 (B f).S + |S|^2 < 0, linear in
// f, so over the box of an octant ([-e, 1/2 + e] along a non-negative
// component, [-1/2 - e, e] along a negative one) it is least at a vertex. An
// image is left out of the octant's list when g exceeds a margin at every
// vertex: then its q exceeds the reduced vector's own q by more than the
// rounding of either, so the minimum over the list is the minimum over all
// 27, bit for bit (ties, g = 0 on a face of the box, stay in the list). The
// kernel assigns a vector to an octant only when its computed fractional
// coordinates lie within e/2 of the box, else to the full list, as it does
// for octants with more than kOctCap images.
// The uncapped image list of every octant (shift indices, ascending).
void octant_lists(const FrameParams &fp, int (&list)[8][kShifts], int (&len)[8]) {
  const double B[3][3] = {{fp.ax, 0.0, 0.0}, {fp.bx, fp.by, 0.0}, {fp.cx, fp.cy, fp.cz}};
  const double size = std::fabs(fp.ax) + std::fabs(fp.bx) + std::fabs(fp.by) +
                      std::fabs(fp.cx) + std::fabs(fp.cy) + std::fabs(fp.cz);
  const double margin = std::ldexp(size * size, -30);
  const double e = kOctSlack;
  for (int o = 0; o < 8; ++o) {
    len[o] = 0;
    for (int m = 0; m < kShifts; ++m) {
      if (m == kZeroShift) continue;
      const double *S = fp.shift64[m];
      const double s2 = S[0] * S[0] + S[1] * S[1] + S[2] * S[2];
      double gmin = 0.0;
      for (int v = 0; v < 8; ++v) {
        double f[3];
        for (int k = 0; k < 3; ++k) {
          const bool neg = (o >> k) & 1;
          const bool hi = (v >> k) & 1;
          f[k] = neg ? (hi ? e : -0.5 - e) : (hi ? 0.5 + e : -e);
        }
        double dot = 0.0;
        for (int c = 0; c < 3; ++c) {
          const double bf = f[0] * B[0][c] + f[1] * B[1][c] + f[2] * B[2][c];
          dot += bf * S[c];
        }
        const double gv = 2.0 * dot + s2;
        gmin = v == 0 ? gv : std::min(gmin, gv);
      }
      if (!(gmin > margin)) list[o][len[o]++] = m;
    }
  }
}

void octant_images(FrameParams &fp) {
  int list[8][kShifts], len[8];
  octant_lists(fp, list, len);
  fp.oct_full = 0;
  int longest = 0;
  for (int o = 0; o < 8; ++o) {
    int n = len[o];
    if (n > kOctCap) {
      fp.oct_full |= static_cast<uint8_t>(1u << o);
      n = 0;
    }
    longest = std::max(longest, n);
    for (int k = 0; k < kOctCap; ++k)
      fp.oct_shift[o][k] = static_cast<uint8_t>(k < n ? list[o][k] : kZeroShift);
  }
  fp.oct_n = static_cast<uint8_t>(longest);
}

// Canonical constants of a frame (binary64), plus their binary32 images.
int frame_consts(int32_t box_type, const double *box, double r_max, int32_t n_bins,
                 FrameParams &fp) {
  std::memset(&fp, 0, sizeof fp);
  fp.n_bins = n_bins;
  fp.s = static_cast<double>(n_bins) / r_max;
  fp.s32 = static_cast<float>(fp.s);
  int kind = kBoxNone;
  if (box_type != DH_BOX_NONE) {
    fp.ax = box[0]; fp.bx = box[3]; fp.by = box[4];
    fp.cx = box[6]; fp.cy = box[7]; fp.cz = box[8];
    fp.L[0] = fp.ax; fp.L[1] = fp.by; fp.L[2] = fp.cz;
    for (int c = 0; c < 3; ++c) fp.iL[c] = 1.0 / fp.L[c];
    fp.h11 = 1.0 / fp.ax;
    fp.h22 = 1.0 / fp.by;
    fp.h33 = 1.0 / fp.cz;
    fp.h12 = -fp.bx / (fp.ax * fp.by);
    fp.h23 = -fp.cy / (fp.by * fp.cz);
    fp.h13 = (fp.bx * fp.cy - fp.by * fp.cx) / (fp.ax * fp.by * fp.cz);
    int m = 0;
    for (int i = -1; i <= 1; ++i)
      for (int j = -1; j <= 1; ++j)
        for (int k = -1; k <= 1; ++k, ++m) {
          fp.shift64[m][0] = static_cast<double>(i) * fp.ax + static_cast<double>(j) * fp.bx +
                             static_cast<double>(k) * fp.cx;
          fp.shift64[m][1] = static_cast<double>(j) * fp.by + static_cast<double>(k) * fp.cy;
          fp.shift64[m][2] = static_cast<double>(k) * fp.cz;
        }
    if (box_type == DH_BOX_ORTHO) {
      kind = kBoxOrtho;
    } else {
      const double w = min_width_tri(fp.ax, fp.bx, fp.by, fp.cx, fp.cy, fp.cz);
      kind = (2.0 * r_max >= w * (1.0 - 1e-9)) ? kBoxTricSearch : kBoxTric;
    }
    constexpr double kTwo32 = 4294967296.0;
    for (int c = 0; c < 3; ++c) fp.k32[c] = static_cast<float>(fp.L[c] * fp.s / kTwo32);
    if (fp.L[0] > 0)
      for (int c = 0; c < 2; ++c)
        fp.ryz32[c] = static_cast<float>((fp.L[c + 1] / fp.L[0]) * (fp.L[c + 1] / fp.L[0]));
    const double B[6] = {fp.ax, fp.bx, fp.by, fp.cx, fp.cy, fp.cz};
    for (int c = 0; c < 6; ++c) fp.Bk[c] = static_cast<float>(B[c] * fp.s / kTwo32);
    for (int c = 0; c < 6; ++c) fp.cell32[c] = static_cast<float>(B[c]);
    const double H[6] = {fp.h11, fp.h12, fp.h13, fp.h22, fp.h23, fp.h33};
    for (int c = 0; c < 6; ++c) fp.hinv32[c] = static_cast<float>(H[c]);
    for (int q = 0; q < 64; ++q) {
      float f[3];
      for (int k = 0; k < 3; ++k) f[k] = static_cast<float>((q >> k & 1) - (q >> (3 + k) & 1));
      const float *b = fp.cell32;
      fp.gshift32[q][0] = (f[0] * b[0] + f[1] * b[1]) + f[2] * b[3];
      fp.gshift32[q][1] = f[1] * b[2] + f[2] * b[4];
      fp.gshift32[q][2] = f[2] * b[5];
      fp.gshift32[q][3] = 0.f;
    }
    if (fp.ax > 0)
      for (int c = 0; c < 5; ++c) fp.Bn[c] = static_cast<float>(B[c + 1] / fp.ax);
    for (int q = 0; q < kShifts; ++q)
      for (int c = 0; c < 3; ++c) fp.shift32[q][c] = static_cast<float>(fp.shift64[q][c] * fp.s);
    // A reduced vector shorter than half the shortest lattice vector lambda
    // is the nearest image: every other image is at least lambda - |d| away.
    // The margin 1e-6 puts the decision far above the rounding of q.
    double lambda2 = 0.0;
    for (int q = 0; q < kShifts; ++q) {
      const double *v = fp.shift64[q];
      const double l2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
      if (l2 > 0.0 && (lambda2 == 0.0 || l2 < lambda2)) lambda2 = l2;
    }
    fp.qskip64 = 0.25 * lambda2 * (1.0 - 1e-6);
    fp.qskip32 = static_cast<float>(0.25 * lambda2 * fp.s * fp.s * (1.0 - 4e-6));
    octant_images(fp);
  }
  fp.box = kind;
  return kind;
}

// Upper bound of t = r * s over all pairs of a periodic frame (the minimum
// image is at most the longest half-diagonal of the cell); 0 without a box.
double t_bound(const FrameParams &fp) {
  if (fp.box == kBoxNone) return 0.0;
  double best = 0.0;
  for (int sa = -1; sa <= 1; sa += 2)
    for (int sb = -1; sb <= 1; sb += 2)
      for (int sc = -1; sc <= 1; sc += 2) {
        const double vx = 0.5 * (sa * fp.ax + sb * fp.bx + sc * fp.cx);
        const double vy = 0.5 * (sb * fp.by + sc * fp.cy);
        const double vz = 0.5 * (sc * fp.cz);
        best = std::max(best, std::sqrt(vx * vx + vy * vy + vz * vz));
      }
  return best * fp.s;
}

struct Launch {
  KernelConfig cfg;
  int mode = kModeLds;
  int win = 0, n_sweeps = 1, stride = 0, grid = 0;
  bool noclamp = false;
  size_t lds = 0;
};

size_t coord_bytes(int precision) { return precision == DH_FP64 ? 32 : 16; }

// LDS of the image-search rings (one per wave), the table of the shift
// vectors (per-octant lists and all 27) and the padding before them.
size_t search_queue_bytes(int precision, int threads, int r) {
  return 32 + (static_cast<size_t>(threads / 64) * queue_cap(r) + kSearchTable) *
                  coord_bytes(precision);
}

// Smallest work item (pairs) when a frame is split into bounded launches.
constexpr int64_t kMinItemPairs = int64_t{1} << 21;

// Launch shape for one frame (heuristic defaults).
// Launch knobs. Every choice yields identical counts; they only change speed.
constexpr int kNumKnobs = 8;

// Bin windows from which the global-atomic kernel replaces LDS windows when
// no tuned shape says otherwise. Measured on MI355X (100k points, periodic
// cube, half the pairs in range): a binary32 window pass costs about 1.75 ms
// and a binary64 one about 5.5 ms, while uint64 global atomics run at about
// 2.4e10 per second whatever the bin count, so global atomics pay off from
// about 63 windows (binary32) and 20 windows (binary64).
constexpr int32_t kWideDefault32 = 60;
constexpr int32_t kWideDefault64 = 20;

struct Knobs {
  int32_t r = 4;             // i-particles per lane: 4 or 8
  int32_t copies = 1;        // interleaved LDS copies: 1, 2 or 4
  int32_t tj = 256;          // j-tile length: 128 or 256
  int32_t noclamp = 1;       // allow unclamped interior blocks
  int32_t occ_cap = 0;       // workgroups per CU at most (0: as many as fit)
  int32_t items_per_wg = 8;  // work items per workgroup (sets the j-chunk)
  // workgroup size: 256, 512 or 1024; 0 = the smallest that gives every
  // SIMD at least four waves within the LDS limit on workgroups per CU
  int32_t threads = 0;
  // global-atomic kernel when the LDS plan needs at least this many bin
  // windows (0: never, 1: always)
  int32_t wide = kWideDefault32;
  std::array<int32_t, kNumKnobs> pack() const {
    return {r, copies, tj, noclamp, occ_cap, items_per_wg, threads, wide};
  }
  static Knobs unpack(const std::array<int32_t, kNumKnobs> &v) {
    Knobs k;
    k.r = v[0]; k.copies = v[1]; k.tj = v[2]; k.noclamp = v[3]; k.occ_cap = v[4];
    k.items_per_wg = v[5]; k.threads = v[6]; k.wide = v[7];
    return k;
  }
  bool valid() const {
    return (r == 4 || r == 8) && (copies == 1 || copies == 2 || copies == 4) &&
           (tj == 128 || tj == 256) && (noclamp == 0 || noclamp == 1) && occ_cap >= 0 &&
           occ_cap <= 16 && items_per_wg >= 1 && items_per_wg <= 64 &&
           (threads == 0 || threads == 256 || threads == 512 || threads == 1024) && wide >= 0 &&
           wide <= 65536;
  }
};

Knobs default_knobs(int precision) {
  Knobs k;
  if (precision == DH_FP64) {
    k.r = 4;
    k.tj = 128;
    k.wide = kWideDefault64;
  }
  return k;
}

// Base kernel configuration and LDS budget of a precision and knob set.
struct BaseConfig {
  KernelConfig cfg;
  size_t tile_bytes;
  int64_t win_max;  // widest bin window that fits the LDS budget
  int occ_cap;
  int items_per_wg;
  bool noclamp;
};

BaseConfig base_config(size_t lds_per_block, int precision, const Knobs &k, int kind) {
  BaseConfig b;
  KernelConfig &c = b.cfg;
  // the image-search kernels are built for at most 256 threads; "auto" is
  // resolved by resolve_threads once the LDS size is known
  c.threads = kind == kBoxTricSearch ? 256 : (k.threads ? k.threads : 256);
  c.r = k.r;
  c.copies = k.copies;
  c.tj = k.tj;
  c.wg_per_cu = k.occ_cap;
  c.jchunk = c.tj;
  // two j-tiles, plus one entry of pad: the look-ahead read of j may touch
  // the entry just past the second tile
  b.tile_bytes = (2 * static_cast<size_t>(c.tj) + 1) * staged_point_bytes(precision, kind);
  if (kind == kBoxTricSorted) b.tile_bytes += kSortedBoxBytes;
  // the search kernels keep their queues after the histogram; counting them
  // with the tiles leaves the histogram budget below them
  if (kind == kBoxTricSearch) b.tile_bytes += search_queue_bytes(precision, c.threads, c.r);
  const size_t budget = std::min<size_t>(lds_per_block, 160 * 1024) - b.tile_bytes - 256;
  b.win_max = static_cast<int64_t>(budget / 4 / c.copies) - kDump;
  b.occ_cap = k.occ_cap;
  b.items_per_wg = k.items_per_wg;
  const char *env = std::getenv("DH_NOCLAMP");
  b.noclamp = k.noclamp && !(env && env[0] == '0');
  return b;
}

int32_t jchunk_for(const KernelConfig &c, int grid, uint64_t work, int items_per_wg) {
  const uint64_t bi = static_cast<uint64_t>(c.threads) * c.r;
  uint64_t jc = work / (static_cast<uint64_t>(grid) * items_per_wg * bi + 1);
  jc = (jc + c.tj - 1) / c.tj * c.tj;
  jc = std::max<uint64_t>(jc, c.tj);
  jc = std::min<uint64_t>(jc, 64ull * c.tj);
  return static_cast<int32_t>(jc);
}

// Workgroup size "auto": the LDS histogram caps the workgroups per CU, so
// take the smallest workgroup that still gives each of the 4 SIMDs at least
// four waves (measured on MI355X: 256 threads when several workgroups fit,
// 512 with two per CU, 1024 with one).
void resolve_threads(int precision, int kind, int mode, const Knobs &k, size_t lds,
                     KernelConfig &cfg) {
  if (k.threads != 0 || kind == kBoxTricSearch) return;
  for (int th : {256, 512}) {
    KernelConfig c = cfg;
    c.threads = th;
    if (pairs_occupancy(precision, kind, mode, c, lds) * (th / 64) >= 16) {
      cfg.threads = th;
      return;
    }
  }
  cfg.threads = 1024;
}

int grid_for_config(int n_cu, int precision, int kind, int mode, const BaseConfig &b,
                    size_t lds, const KernelConfig &cfg) {
  int occ = pairs_occupancy(precision, kind, mode, cfg, lds);
  if (b.occ_cap > 0) occ = std::min(occ, b.occ_cap);
  return n_cu * std::max(1, occ);
}

// Launch shape for one frame on a device with n_cu compute units and
// lds_per_block bytes of LDS per workgroup.
Launch choose_launch(int n_cu, size_t lds_per_block, int precision, const FrameParams &fp,
                     uint64_t total_pairs, const Knobs &k) {
  Launch L;
  const BaseConfig b = base_config(lds_per_block, precision, k, fp.box);
  L.cfg = b.cfg;
  const int32_t n_bins = fp.n_bins;
  if (n_bins <= b.win_max) {
    L.n_sweeps = 1;
    L.win = n_bins;
  } else {
    L.n_sweeps = static_cast<int>((n_bins + b.win_max - 1) / b.win_max);
    L.win = (n_bins + L.n_sweeps - 1) / L.n_sweeps;
  }
  if (k.wide > 0 && L.n_sweeps >= k.wide) {
    // one pass, uint64 atomics into the output; LDS holds the j-tiles only
    L.mode = kModeGlobal;
    L.n_sweeps = 1;
    L.win = n_bins;
    L.stride = 0;
    L.lds = b.tile_bytes;
    resolve_threads(precision, fp.box, L.mode, k, L.lds, L.cfg);
    L.grid = grid_for_config(n_cu, precision, fp.box, L.mode, b, L.lds, L.cfg);
    L.cfg.jchunk = jchunk_for(L.cfg, L.grid, total_pairs, b.items_per_wg);
    return L;
  }
  L.mode = L.n_sweeps > 1 ? kModeSweep : kModeLds;
  L.stride = L.win + kDump;
  // Without clamping, every t of a periodic frame must index a slot below the
  // stride: slots = floor(bound * (1 + 1e-4)) + 2 covers the rounding of the
  // minimum image and of the distance.
  L.noclamp = false;
  const double tb = t_bound(fp);
  if (b.noclamp && L.n_sweeps == 1 && tb > 0) {
    const int64_t slots = static_cast<int64_t>(tb * (1.0 + 1e-4)) + 2;
    if (slots <= b.win_max + kDump) {
      L.noclamp = true;
      L.stride = static_cast<int>(std::max<int64_t>(L.stride, slots));
    }
  }
  L.lds = b.tile_bytes + static_cast<size_t>(L.cfg.copies) * L.stride * 4;
  resolve_threads(precision, fp.box, L.mode, k, L.lds, L.cfg);
  L.grid = grid_for_config(n_cu, precision, fp.box, L.mode, b, L.lds, L.cfg);
  L.cfg.jchunk = jchunk_for(L.cfg, L.grid, total_pairs * static_cast<uint64_t>(L.n_sweeps),
                            b.items_per_wg);
  return L;
}

Launch choose_launch(const dh_ctx *ctx, int precision, const FrameParams &fp,
                     uint64_t total_pairs, const Knobs &k) {
  return choose_launch(ctx->n_cu, ctx->lds_per_block, precision, fp, total_pairs, k);
}

// Work items of one frame, grouped by (histogram, sweep); the rows and items
// of each histogram as hist_rows / emit_row cut them (shared with the
// device-side planner).
void plan_frame(int32_t frame, const int64_t *off, int32_t k, const Launch &L,
                std::vector<WorkItem> &items, std::vector<uint64_t> &pairs) {
  const int64_t bi = static_cast<int64_t>(L.cfg.threads) * L.cfg.r;
  const int64_t jc = L.cfg.jchunk;
  const int32_t n_hist = k * (k + 1) / 2;
  for (int32_t h = 0; h < n_hist; ++h) {
    const HistRows r = hist_rows(off, k, h);
    pairs.push_back(r.pairs);
    const size_t first = items.size();
    const int64_t nr = hist_row_count(r, bi);
    for (int64_t b = 0; b < nr; ++b) {
      const size_t at = items.size();
      items.resize(at + static_cast<size_t>(row_item_count(r, b, bi, jc)));
      emit_row(r, h, 0, b, bi, jc, items.data() + at);
    }
    const size_t last = items.size();
    for (size_t q = first; q < last; ++q) items[q].frame = frame;
    // replicate for every bin window, keeping items grouped by (h, sweep)
    for (int32_t sw = 1; sw < L.n_sweeps; ++sw)
      for (size_t q = first; q < last; ++q) {
        WorkItem w = items[q];
        w.sweep = sw;
        items.push_back(w);
      }
  }
}

// Splits the last `grid` items of a work list (the ones workgroups take
// when the rest is done) into pieces of about a quarter of their j-range,
// in whole j-tiles, so that the workgroups finish close together instead of
// idling for up to one full item. Diagonal items stay whole; the grouping
// by (histogram, window) is kept.
void refine_tail(std::vector<WorkItem> &items, int grid, int tj) {
  const size_t n = items.size();
  const size_t tail = std::min<size_t>(n, static_cast<size_t>(std::max(grid, 0)));
  if (tail == 0) return;
  std::vector<WorkItem> out(items.begin(), items.end() - static_cast<std::ptrdiff_t>(tail));
  out.reserve(n + 3 * tail);
  for (size_t q = n - tail; q < n; ++q) {
    const WorkItem &w = items[q];
    const int32_t len = w.j1 - w.j0;
    const int32_t piece = std::max<int32_t>(tj, (len / 4 + tj - 1) / tj * tj);
    if ((w.flags & kItemDiag) || len <= piece) {
      out.push_back(w);
      continue;
    }
    for (int32_t j = w.j0; j < w.j1; j += piece) {
      WorkItem p = w;
      p.j0 = j;
      p.j1 = std::min(j + piece, w.j1);
      out.push_back(p);
    }
  }
  items.swap(out);
}

int ensure_device(dh_ctx *ctx, void **ptr, size_t *cap, size_t need) {
  if (need <= *cap) return DH_OK;
  size_t want = std::max(need, *cap + *cap / 2);
  if (ctx->budget) {
    // checked before the old buffer goes, so a refused call leaves the
    // context as it was; the growth slack is cut to what the budget leaves
    const size_t others = ctx_device_bytes(ctx) - *cap + ctx->batch_bytes;
    if (others > ctx->budget || need > ctx->budget - others)
      return fail(ctx, DH_EBUDGET,
                  "%zu bytes of device scratch needed beside the %zu held; budget %zu bytes",
                  need, others, ctx->budget);
    want = std::min(want, ctx->budget - others);
  }
  if (*ptr) {
    DH_HIP(ctx, hipDeviceSynchronize());
    DH_HIP(ctx, hipFree(*ptr));
    *ptr = nullptr;
    *cap = 0;
  }
  if (hipMalloc(ptr, want) != hipSuccess) {
    (void)hipGetLastError();
    *ptr = nullptr;
    return fail(ctx, DH_ENOMEM, "hipMalloc of %zu bytes failed", want);
  }
  *cap = want;
  return DH_OK;
}

int ensure_pinned(dh_ctx *ctx, size_t need) {
  if (need <= ctx->hblob_cap) return DH_OK;
  if (ctx->blob_pending) {
    DH_HIP(ctx, hipEventSynchronize(ctx->blob_evt));
    ctx->blob_pending = false;
  }
  if (ctx->h_blob) DH_HIP(ctx, hipHostFree(ctx->h_blob));
  ctx->h_blob = nullptr;
  ctx->hblob_cap = 0;
  size_t want = std::max(need, static_cast<size_t>(1) << 16);
  if (hipHostMalloc(&ctx->h_blob, want, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    ctx->h_blob = nullptr;
    return fail(ctx, DH_ENOMEM, "hipHostMalloc of %zu bytes failed", want);
  }
  ctx->hblob_cap = want;
  return DH_OK;
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Uploads frames | items | pairs | counter through the pinned staging buffer.
struct BlobLayout {
  size_t frames = 0, items = 0, pairs = 0, counter = 0, total = 0;
};

BlobLayout blob_layout(size_t n_frames, size_t n_items, size_t n_pairs, size_t n_counters = 1) {
  BlobLayout b;
  b.frames = 0;
  b.items = align_up(b.frames + n_frames * sizeof(FrameParams), 256);
  b.pairs = align_up(b.items + n_items * sizeof(WorkItem), 256);
  b.counter = align_up(b.pairs + n_pairs * sizeof(uint64_t), 256);
  b.total = b.counter + align_up(std::max<size_t>(1, n_counters) * sizeof(int32_t), 256);
  return b;
}

// Uploads frames, items and pair counts with zeroed work counters. With
// reuse set, a blob identical to the one already on the device (same plan,
// same buffers) is not uploaded again; the caller then zeroes the counters.
int upload_blob(dh_ctx *ctx, hipStream_t st, const BlobLayout &lay,
                const std::vector<FrameParams> &frames, const std::vector<WorkItem> &items,
                const std::vector<uint64_t> &pairs, bool reuse = false) {
  std::vector<char> next(lay.counter, 0);
  if (!frames.empty()) std::memcpy(next.data() + lay.frames, frames.data(), frames.size() * sizeof(FrameParams));
  if (!items.empty()) std::memcpy(next.data() + lay.items, items.data(), items.size() * sizeof(WorkItem));
  if (!pairs.empty()) std::memcpy(next.data() + lay.pairs, pairs.data(), pairs.size() * sizeof(uint64_t));
  if (reuse && ctx->d_blob && ctx->blob_cap >= lay.total && next == ctx->blob_last) return DH_OK;
  ctx->blob_last.clear();
  int rc = ensure_pinned(ctx, lay.total);
  if (rc) return rc;
  rc = ensure_device(ctx, &ctx->d_blob, &ctx->blob_cap, lay.total);
  if (rc) return rc;
  if (ctx->blob_pending) {
    DH_HIP(ctx, hipEventSynchronize(ctx->blob_evt));
    ctx->blob_pending = false;
  }
  char *h = static_cast<char *>(ctx->h_blob);
  std::memcpy(h, next.data(), next.size());
  std::memset(h + lay.counter, 0, lay.total - lay.counter);
  DH_HIP(ctx, hipMemcpyAsync(ctx->d_blob, h, lay.total, hipMemcpyHostToDevice, st));
  DH_HIP(ctx, hipEventRecord(ctx->blob_evt, st));
  ctx->blob_pending = true;
  ctx->blob_last.swap(next);
  return DH_OK;
}

int load_tune_cache(dh_ctx *ctx);

int ctx_init(dh_ctx *ctx, int32_t device) {
  int n = 0;
  DH_HIP(ctx, hipGetDeviceCount(&n));
  if (device < 0 || device >= n) return fail(ctx, DH_EINVAL, "device %d of %d", device, n);
  ctx->device = device;
  DH_HIP(ctx, hipSetDevice(device));
  hipDeviceProp_t prop;
  DH_HIP(ctx, hipGetDeviceProperties(&prop, device));
  ctx->n_cu = prop.multiProcessorCount;
  ctx->arch = prop.gcnArchName;
  ctx->arch = ctx->arch.substr(0, ctx->arch.find(':'));
  if (const char *m = std::getenv("DH_TUNE")) ctx->tune_mode = std::atoi(m);
  if (ctx->tune_mode < DH_TUNE_OFF || ctx->tune_mode > DH_TUNE_ON) ctx->tune_mode = DH_TUNE_OFF;
  if (const char *pth = std::getenv("DH_TUNE_CACHE")) {
    ctx->tune_path = pth;
    int rc = load_tune_cache(ctx);
    if (rc) return rc;
  }
  ctx->lds_per_block = prop.sharedMemPerBlock;
  DH_HIP(ctx, hipEventCreateWithFlags(&ctx->blob_evt, hipEventDisableTiming));
  DH_HIP(ctx, hipStreamCreateWithFlags(&ctx->own_stream, hipStreamNonBlocking));
  return DH_OK;
}

// One single-frame histogram call, prepared on the host.
struct FrameJob {
  const double *d_coords = nullptr;
  const int64_t *offsets = nullptr;
  int32_t n_species = 0;
  int precision = 0;
  int kind = 0;
  FrameParams fp{};
  uint64_t total = 0;
  uint64_t *d_out = nullptr;
  uint64_t *d_oor = nullptr;
  bool accumulate = false;  // add into d_out instead of overwriting it
};

// Stages a frame's coordinates into the context's scratch (spatially sorted
// frames: the sort keys in the context's key buffer).
int stage_job(dh_ctx *ctx, hipStream_t st, const FrameJob &job, const FrameParams &fp) {
  const int64_t n = job.offsets[job.n_species];
  if (job.kind == kBoxTricSorted) {
    int rc = ensure_device(ctx, &ctx->d_keys, &ctx->keys_cap,
                           static_cast<size_t>(sort_keys_count(n)) * sizeof(uint64_t));
    if (rc) return rc;
    DH_HIP(ctx, launch_stage_sorted(job.precision, job.d_coords, ctx->d_staged, n, job.offsets, job.n_species,
                                    fp, static_cast<uint64_t *>(ctx->d_keys), st));
    return DH_OK;
  }
  DH_HIP(ctx, launch_stage(job.precision, job.kind, job.d_coords, ctx->d_staged, n, fp, st));
  return DH_OK;
}

// Plans and enqueues one frame with the given knobs: stage (optional), zero,
// pair kernel (between e0 and e1 when given), out-of-range counts.
int run_frame(dh_ctx *ctx, hipStream_t st, const FrameJob &job, const Knobs &k, bool stage,
              hipEvent_t e0, hipEvent_t e1) {
  FrameParams fp = job.fp;
  const int64_t n = job.offsets[job.n_species];
  const int32_t n_hist = job.n_species * (job.n_species + 1) / 2;
  Launch L = choose_launch(ctx, job.precision, fp, job.total, k);
  fp.win = L.win;
  fp.n_sweeps = L.n_sweeps;
  fp.noclamp = L.noclamp ? 1 : 0;
  // bounded launches: size the items for one launch's share of the work,
  // then cut the list wherever the running pair count reaches the limit
  const uint64_t work = job.total * static_cast<uint64_t>(L.n_sweeps);
  const uint64_t limit = ctx->launch_pairs;
  if (limit > 0 && work > limit) {
    // items of at least kMinItemPairs keep the work list of a huge frame small
    const int64_t bi = static_cast<int64_t>(L.cfg.threads) * L.cfg.r;
    const int64_t min_jc = (kMinItemPairs / bi + L.cfg.tj - 1) / L.cfg.tj * L.cfg.tj;
    L.cfg.jchunk = std::max<int32_t>(jchunk_for(L.cfg, L.grid, limit, k.items_per_wg),
                                     static_cast<int32_t>(std::min<int64_t>(min_jc, 64 * L.cfg.tj)));
  }
  std::vector<WorkItem> items;
  std::vector<uint64_t> pairs;
  plan_frame(0, job.offsets, job.n_species, L, items, pairs);
  std::vector<size_t> cuts(1, 0);
  if (limit > 0 && work > limit) {
    uint64_t acc = 0;
    for (size_t q = 0; q < items.size(); ++q) {
      acc += static_cast<uint64_t>(items[q].i1 - items[q].i0) *
             static_cast<uint64_t>(items[q].j1 - items[q].j0);
      if (acc >= limit && q + 1 < items.size()) {
        cuts.push_back(q + 1);
        acc = 0;
      }
    }
  }
  cuts.push_back(items.size());
  // every launch drains its own list: refine the tail of each
  {
    std::vector<WorkItem> all, seg;
    std::vector<size_t> at(1, 0);
    for (size_t c = 0; c + 1 < cuts.size(); ++c) {
      seg.assign(items.begin() + static_cast<std::ptrdiff_t>(cuts[c]),
                 items.begin() + static_cast<std::ptrdiff_t>(cuts[c + 1]));
      refine_tail(seg, L.grid, L.cfg.tj);
      all.insert(all.end(), seg.begin(), seg.end());
      at.push_back(all.size());
    }
    items.swap(all);
    cuts.swap(at);
  }
  const size_t n_launches = cuts.size() - 1;
  fp.coords = ctx->d_staged;
  fp.out = job.d_out;
  // with LDS histograms the flushes count the out-of-range pairs: oor starts
  // at the pair count (zero kernel) and every flush subtracts its counts
  const bool oor_flush = job.d_oor && L.mode != kModeGlobal;
  fp.oor = oor_flush ? job.d_oor : nullptr;
  fp.oor_by_flush = oor_flush ? 1 : 0;
  // counters: one work counter per launch, then (8-byte aligned) the counts
  // of image-searched pairs and of the images evaluated for them; the upload
  // or the zero kernel clears them all
  const size_t n_work_counters = (n_launches + 1) / 2 * 2;
  const size_t n_counters = n_work_counters + 4;
  const BlobLayout lay = blob_layout(1, items.size(), pairs.size(), n_counters);
  // the counter's device address goes into the frame constants, so the blob
  // is allocated before they are uploaded (a new allocation is never taken
  // for an unchanged plan)
  if (lay.total > ctx->blob_cap) ctx->blob_last.clear();
  {
    int rc0 = ensure_device(ctx, &ctx->d_blob, &ctx->blob_cap, lay.total);
    if (rc0) return rc0;
  }
  fp.searched = job.kind == kBoxTricSearch && !job.accumulate
                    ? reinterpret_cast<unsigned long long *>(
                          static_cast<char *>(ctx->d_blob) + lay.counter +
                          n_work_counters * sizeof(int32_t))
                    : nullptr;
  ctx->searched_dev = fp.searched;
  std::vector<FrameParams> frames(1, fp);
  // an unchanged plan is reused when the zero kernel below resets the counters
  int rc = upload_blob(ctx, st, lay, frames, items, pairs, !job.accumulate);
  if (rc) return rc;
  char *db = static_cast<char *>(ctx->d_blob);
  if (stage) {
    const int rc_stage = stage_job(ctx, st, job, fp);
    if (rc_stage) return rc_stage;
  }
  if (!job.accumulate)
    DH_HIP(ctx, launch_zero(job.d_out, static_cast<int64_t>(n_hist) * fp.n_bins,
                            reinterpret_cast<int32_t *>(db + lay.counter),
                            static_cast<int32_t>(n_counters), fp.oor,
                            reinterpret_cast<const uint64_t *>(db + lay.pairs), n_hist, st));
  const int grid = std::max(1, std::min<int>(L.grid, static_cast<int>(items.size())));
  if (ctx->hold) {
    ctx->held.clear();
    ctx->held_next = 0;
    ctx->held_left = 0;
  }
  if (e0) DH_HIP(ctx, hipEventRecord(e0, st));
  for (size_t c = 0; c < n_launches && !items.empty(); ++c) {
    // every launch has its own work counter (zeroed by the upload or, for a
    // reused blob, by the zero kernel)
    PairKernelArgs a;
    a.frames = reinterpret_cast<const FrameParams *>(db + lay.frames);
    a.items = reinterpret_cast<const WorkItem *>(db + lay.items) + cuts[c];
    a.counter = reinterpret_cast<int32_t *>(db + lay.counter) + c;
    a.n_items = static_cast<int32_t>(cuts[c + 1] - cuts[c]);
    a.copies = L.cfg.copies;
    a.stride = L.stride;
    a.tj = L.cfg.tj;
    const int g = std::max(1, std::min(grid, a.n_items));
    if (ctx->hold) {
      uint64_t p = 0;
      for (size_t q = cuts[c]; q < cuts[c + 1]; ++q)
        p += static_cast<uint64_t>(items[q].i1 - items[q].i0) *
             static_cast<uint64_t>(items[q].j1 - items[q].j0);
      ctx->held.push_back({job.precision, job.kind, L.mode, L.cfg, a, g, L.lds, p});
      ctx->held_left += p;
      continue;
    }
    DH_HIP(ctx, launch_pairs(job.precision, job.kind, L.mode, L.cfg, a, g, L.lds, st));
  }
  if (e1) DH_HIP(ctx, hipEventRecord(e1, st));
  if (ctx->hold) {
    ctx->held_oor = job.d_oor != nullptr && !oor_flush;
    ctx->oor_hist = job.d_out;
    ctx->oor_n_hist = n_hist;
    ctx->oor_n_bins = fp.n_bins;
    ctx->oor_pairs = reinterpret_cast<const uint64_t *>(db + lay.pairs);
    ctx->oor_out = job.d_oor;
  } else if (job.d_oor && !oor_flush) {
    DH_HIP(ctx, launch_oor(job.d_out, n_hist, fp.n_bins,
                           reinterpret_cast<const uint64_t *>(db + lay.pairs), job.d_oor, st));
  }
  const std::array<int32_t, kNumKnobs> kp = k.pack();
  for (int q = 0; q < kNumKnobs; ++q) ctx->last_config[q] = kp[q];
  ctx->last_config[6] = L.cfg.threads;  // the workgroup size actually launched
  ctx->last_config[8] = items.empty() ? 0 : grid;
  ctx->last_config[9] = static_cast<int32_t>(L.lds);
  ctx->last_config[10] = L.n_sweeps;
  ctx->last_config[11] = static_cast<int32_t>(items.size());
  ctx->last_config[12] = L.mode;
  return DH_OK;
}

int ilog2_ceil(uint64_t v) {
  int e = 0;
  while ((1ull << e) < v) ++e;
  return e;
}

// Cache bucket of a frame: architecture, precision, minimum-image kind,
// ceil(log2 n_bins), ceil(log2 N), species (capped at 4).
std::string tune_key(const dh_ctx *ctx, const FrameJob &job) {
  char buf[160];
  snprintf(buf, sizeof buf, "%s|p%d|b%d|nb%d|n%d|k%d", ctx->arch.c_str(), job.precision, job.kind,
           ilog2_ceil(static_cast<uint64_t>(job.fp.n_bins)),
           ilog2_ceil(static_cast<uint64_t>(std::max<int64_t>(1, job.offsets[job.n_species]))),
           std::min(job.n_species, 4));
  return buf;
}

int save_tune_cache(dh_ctx *ctx) {
  if (ctx->tune_path.empty()) return DH_OK;
  std::ostringstream o;
  o << "{\"version\": 3, \"knobs\": [\"r\", \"copies\", \"tj\", \"noclamp\", \"occ_cap\", "
       "\"items_per_wg\", \"threads\", \"wide\"], \"entries\": {";
  bool first = true;
  for (const auto &kv : ctx->tune_cache) {
    o << (first ? "\n  " : ",\n  ") << '"' << kv.first << "\": [";
    for (int q = 0; q < kNumKnobs; ++q) o << (q ? ", " : "") << kv.second[q];
    o << ']';
    first = false;
  }
  o << "\n}}\n";
  const std::string tmp = ctx->tune_path + ".tmp";
  {
    std::ofstream f(tmp);
    if (!f) return fail(ctx, DH_EINVAL, "cannot write %s", tmp.c_str());
    f << o.str();
  }
  if (std::rename(tmp.c_str(), ctx->tune_path.c_str()) != 0)
    return fail(ctx, DH_EINVAL, "cannot replace %s", ctx->tune_path.c_str());
  return DH_OK;
}

// Reads entries written by save_tune_cache ("key": [kNumKnobs integers]);
// entries of another length or with invalid knobs are skipped.
int load_tune_cache(dh_ctx *ctx) {
  std::ifstream f(ctx->tune_path);
  if (!f) return DH_OK;  // no cache yet
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string t = ss.str();
  size_t pos = t.find("\"entries\"");
  if (pos != std::string::npos) pos = t.find('{', pos);
  if (pos == std::string::npos) return fail(ctx, DH_EINVAL, "malformed tuning cache");
  while (true) {
    const size_t q0 = t.find('"', pos + 1);
    if (q0 == std::string::npos) break;
    const size_t q1 = t.find('"', q0 + 1);
    if (q1 == std::string::npos) break;
    const size_t lb = t.find('[', q1);
    if (lb == std::string::npos) break;
    const size_t rb = t.find(']', lb);
    if (rb == std::string::npos) break;
    const std::string key = t.substr(q0 + 1, q1 - q0 - 1);
    std::array<int32_t, kNumKnobs> v{};
    std::istringstream in(t.substr(lb + 1, rb - lb - 1));
    int q = 0;
    std::string tok;
    try {
      while (q < kNumKnobs && std::getline(in, tok, ','))
      v[q++] = static_cast<int32_t>(std::stol(tok));
    } catch (...) {
      return fail(ctx, DH_EINVAL, "malformed tuning cache entry %s", key.c_str());
    }
    if (q == kNumKnobs && Knobs::unpack(v).valid()) ctx->tune_cache[key] = v;
    pos = rb;
  }
  return DH_OK;
}

// Times the pair kernel of candidate knob sets on this frame (coordinate
// descent from the defaults, one knob at a time) and keeps the fastest.
// Every candidate computes the same counts.
int tune_frame(dh_ctx *ctx, hipStream_t st, const FrameJob &job, const std::string &key,
               Knobs &best) {
  const int64_t n = job.offsets[job.n_species];
  FrameParams fp = job.fp;
  fp.coords = ctx->d_staged;
  (void)n;
  {
    const int rc_stage = stage_job(ctx, st, job, fp);
    if (rc_stage) return rc_stage;
  }
  hipEvent_t e0, e1;
  DH_HIP(ctx, hipEventCreate(&e0));
  DH_HIP(ctx, hipEventCreate(&e1));
  auto time_of = [&](const Knobs &k, float *ms) -> int {
    float bestms = 1e30f;
    for (int rep = 0; rep < 2; ++rep) {
      int rc = run_frame(ctx, st, job, k, false, e0, e1);
      if (rc) return rc;
      DH_HIP(ctx, hipEventSynchronize(e1));
      float v = 0.f;
      DH_HIP(ctx, hipEventElapsedTime(&v, e0, e1));
      bestms = std::min(bestms, v);
    }
    *ms = bestms;
    return DH_OK;
  };
  best = default_knobs(job.precision);
  // LDS bin windows against global atomics, only where the histogram needs
  // more than one window: 0 keeps the windows, 1 always takes global atomics
  std::vector<int32_t> wide_choices;
  {
    Knobs k0 = best;
    k0.wide = 0;
    if (choose_launch(ctx, job.precision, job.fp, job.total, k0).n_sweeps > 1) {
      best.wide = 0;
      wide_choices = {1};
    }
  }
  float best_ms = 0.f;
  int rc = time_of(best, &best_ms);
  auto consider = [&](const Knobs &cand) {
    float ms = 0.f;
    rc = time_of(cand, &ms);
    if (!rc && ms < best_ms * 0.99f) {
      best = cand;
      best_ms = ms;
    }
  };
  for (int32_t v : wide_choices) {
    Knobs cand = best;
    cand.wide = v;
    if (!rc) consider(cand);
  }
  // i-particles per lane and workgroup size together: they trade registers
  // against waves per SIMD, and the best pair is often not reached one knob
  // at a time
  {
    const Knobs base = best;
    for (int32_t r : {4, 8})
      for (int32_t th : {256, 512, 1024}) {
        Knobs cand = base;
        cand.r = r;
        cand.threads = th;
        if (!rc && (cand.r != base.r || cand.threads != base.threads)) consider(cand);
      }
  }
  const std::vector<std::vector<int32_t>> choices = {
      {0, 1},            // noclamp
      {1, 2, 4},         // copies
      {0, 1, 2, 3},      // occ_cap
      {4, 8, 16},        // items_per_wg
      {128, 256},        // tj
  };
  const int order[5] = {3, 1, 4, 5, 2};  // knob index in pack() order
  for (int d = 0; d < 5 && !rc; ++d) {
    const int q = order[d];
    for (int32_t v : choices[d]) {
      std::array<int32_t, kNumKnobs> kp = best.pack();
      if (kp[q] == v) continue;
      kp[q] = v;
      const Knobs cand = Knobs::unpack(kp);
      float ms = 0.f;
      rc = time_of(cand, &ms);
      if (rc) break;
      if (ms < best_ms * 0.99f) {
        best = cand;
        best_ms = ms;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  ctx->tune_cache[key] = best.pack();
  return save_tune_cache(ctx);
}

std::mutex g_default_mu;
std::map<int, dh_ctx *> g_default;

}  // namespace

namespace dh {

int ctx_device(const dh_ctx *ctx) { return ctx->device; }

LaunchPlan default_launch(int n_cu, size_t lds_per_block, int precision, const FrameParams &fp,
                          uint64_t total_pairs) {
  const Launch L = choose_launch(n_cu, lds_per_block, precision, fp, total_pairs,
                                 default_knobs(precision));
  LaunchPlan p;
  p.cfg = L.cfg;
  p.mode = L.mode;
  p.win = L.win;
  p.n_sweeps = L.n_sweeps;
  p.stride = L.stride;
  p.grid = L.grid;
  p.noclamp = L.noclamp;
  p.lds = L.lds;
  return p;
}

LaunchPlan serve_launch(int n_cu, size_t lds_per_block, int precision, const FrameParams &fp,
                        uint64_t total_pairs, int threads) {
  Knobs k = default_knobs(precision);
  k.threads = threads;
  const Launch L = choose_launch(n_cu, lds_per_block, precision, fp, total_pairs, k);
  LaunchPlan p;
  p.cfg = L.cfg;
  p.mode = L.mode;
  p.win = L.win;
  p.n_sweeps = L.n_sweeps;
  p.stride = L.stride;
  p.grid = L.grid;
  p.noclamp = L.noclamp;
  p.lds = L.lds;
  return p;
}

int thread_fail(int code, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(t_last_error, sizeof t_last_error, fmt, ap);
  va_end(ap);
  return code;
}

int frame_constants(int32_t box_type, const double *box, double r_max, int32_t n_bins,
                    FrameParams &fp) {
  return frame_consts(box_type, box, r_max, n_bins, fp);
}

int zero_u64(uint64_t *p, int64_t n, hipStream_t st) {
  return launch_zero(p, n, nullptr, 0, nullptr, nullptr, 0, st) == hipSuccess ? DH_OK
                                                                           : DH_EDEVICE;
}

size_t ctx_device_bytes(const dh_ctx *ctx) {
  return ctx->staged_cap + ctx->blob_cap + ctx->in_cap + ctx->out_cap + ctx->keys_cap;
}

void ctx_release_scratch(dh_ctx *ctx) {
  if (hipSetDevice(ctx->device) != hipSuccess) return;
  void **bufs[5] = {&ctx->d_staged, &ctx->d_blob, reinterpret_cast<void **>(&ctx->d_in),
                    reinterpret_cast<void **>(&ctx->d_out), &ctx->d_keys};
  size_t *caps[5] = {&ctx->staged_cap, &ctx->blob_cap, &ctx->in_cap, &ctx->out_cap,
                     &ctx->keys_cap};
  for (int k = 0; k < 5; ++k) {
    if (*bufs[k]) (void)hipFree(*bufs[k]);
    *bufs[k] = nullptr;
    *caps[k] = 0;
  }
  ctx->blob_last.clear();
  (void)hipGetLastError();
}

size_t job_scratch_bytes(int64_t n_points, int32_t n_hist, int32_t n_bins, int32_t precision,
                         int64_t launch_pairs) {
  // staged coordinates plus the work blob (frame constants, pair counts and
  // work items: a few MB, plus one item per kMinItemPairs pairs of every bin
  // window when the frame runs as bounded launches, and the tail pieces of
  // every launch, at most three more items per workgroup of a grid of at
  // most 2,048; at least 9,000 bins fit one window, and beyond 64 windows
  // the global-atomic mode needs one pass)
  const uint64_t n = static_cast<uint64_t>(std::max<int64_t>(1, n_points));
  const uint64_t windows = std::min<uint64_t>(64, (static_cast<uint64_t>(n_bins) + 8999) / 9000);
  const uint64_t work = n * (n - 1) / 2 * windows;
  const uint64_t launches =
      launch_pairs > 0 ? work / static_cast<uint64_t>(launch_pairs) + 1 : 1;
  return static_cast<size_t>(n) * coord_bytes(precision) + (4u << 20) +
         static_cast<size_t>(n_hist) * 8 +
         static_cast<size_t>(work / kMinItemPairs + launches * 3 * 2048) * sizeof(WorkItem);
}

}  // namespace dh

// The launch sequence of a batch: stage, zero, one persistent pair kernel per
// class of frames, out-of-range counts. Recorded once into a graph, or issued
// directly.
static int dh_batch_launch_direct(dh_batch *b, hipStream_t st) {
  dh_ctx *ctx = b->ctx;
  char *db = static_cast<char *>(b->d_blob);
  const FrameParams *d_frames = reinterpret_cast<const FrameParams *>(db + b->off_frames);
  int32_t *counters = reinterpret_cast<int32_t *>(db + b->off_counters);
  DH_HIP(ctx, launch_stage_batch(b->precision, d_frames, b->n_frames, b->max_points, st));
  // spatially sorted frames one after the other (one key buffer)
  for (const dh_batch::Sorted &q : b->sorted)
    DH_HIP(ctx, launch_stage_sorted(b->precision, q.d_in, q.staged, q.fp.n_points, q.offsets.data(),
                                    static_cast<int32_t>(q.offsets.size() - 1), q.fp,
                                    static_cast<uint64_t *>(b->d_keys), st));
  DH_HIP(ctx, launch_zero_batch(d_frames, b->n_frames, b->max_words, counters,
                                static_cast<int32_t>(b->groups.size()), st));
  for (size_t k = 0; k < b->groups.size(); ++k) {
    const dh_batch::Group &g = b->groups[k];
    if (g.item_count == 0) continue;
    PairKernelArgs a;
    a.frames = d_frames;
    a.items = reinterpret_cast<const WorkItem *>(db + b->off_items) + g.item_begin;
    a.counter = counters + k;
    a.n_items = static_cast<int32_t>(g.item_count);
    a.copies = g.cfg.copies;
    a.stride = g.stride;
    a.tj = g.cfg.tj;
    const int grid = std::max(1, std::min<int>(g.grid, a.n_items));
    DH_HIP(ctx, launch_pairs(b->precision, g.kind, g.mode, g.cfg, a, grid, g.lds, st));
  }
  if (b->any_oor) DH_HIP(ctx, launch_oor_batch(d_frames, b->n_frames, b->max_hist, st));
  return DH_OK;
}

extern "C" {

const char *dh_version(void) { return "0.1.0"; }

const char *dh_strerror(int code) {
  switch (code) {
    case DH_OK: return "success";
    case DH_EINVAL: return "invalid argument";
    case DH_ENOMEM: return "out of memory";
    case DH_EDEVICE: return "device error";
    case DH_EBUDGET: return "memory budget exceeded";
    case DH_EUNSUPPORTED: return "unsupported";
    default: return "unknown error";
  }
}

int dh_check_args(const double *coords, const int64_t *offsets, int32_t n_species,
                  int32_t box_type, const double *box, double r_max, int32_t n_bins,
                  int32_t precision) {
  return check(coords, offsets, n_species, box_type, box, r_max, n_bins, precision);
}

int dh_search_images(const double *box, int32_t *lists, int32_t *counts, int32_t *full_mask) {
  if (!box || !lists || !counts || !full_mask) return DH_EINVAL;
  if (!box_ok(DH_BOX_TRICLINIC, box)) return DH_EINVAL;  // the rules of a histogram call
  FrameParams fp;
  frame_consts(DH_BOX_TRICLINIC, box, 1.0, 1, fp);
  int list[8][kShifts], len[8];
  octant_lists(fp, list, len);
  for (int o = 0; o < 8; ++o) {
    counts[o] = len[o];
    for (int k = 0; k < kShifts - 1; ++k)
      lists[o * (kShifts - 1) + k] = k < len[o] ? list[o][k] : kZeroShift;
  }
  *full_mask = fp.oct_full;
  return DH_OK;
}

int dh_ctx_create(int32_t device, int64_t hbm_budget_bytes, dh_ctx **out) {
  if (!out) return DH_EINVAL;
  *out = nullptr;
  if (hbm_budget_bytes < 0) return DH_EINVAL;
  dh_ctx *ctx = new (std::nothrow) dh_ctx;
  if (!ctx) return DH_ENOMEM;
  ctx->budget = static_cast<size_t>(hbm_budget_bytes);
  int rc = ctx_init(ctx, device);
  if (rc) {
    dh_ctx_destroy(ctx);
    return rc;
  }
  *out = ctx;
  return DH_OK;
}

void dh_ctx_destroy(dh_ctx *ctx) {
  if (!ctx) return;
  if (hipSetDevice(ctx->device) == hipSuccess) {
    (void)hipDeviceSynchronize();
    if (ctx->d_staged) (void)hipFree(ctx->d_staged);
    if (ctx->d_keys) (void)hipFree(ctx->d_keys);
    if (ctx->d_blob) (void)hipFree(ctx->d_blob);
    if (ctx->d_in) (void)hipFree(ctx->d_in);
    if (ctx->d_out) (void)hipFree(ctx->d_out);
    if (ctx->h_blob) (void)hipHostFree(ctx->h_blob);
    if (ctx->blob_evt) (void)hipEventDestroy(ctx->blob_evt);
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->own_stream);
    for (auto &ev : ctx->prof_events) {
      (void)hipEventDestroy(ev.first);
      (void)hipEventDestroy(ev.second);
    }
  }
  (void)hipGetLastError();
  delete ctx;
}

const char *dh_ctx_last_error(const dh_ctx *ctx) {
  return ctx ? ctx->last_error.c_str() : t_last_error;
}

int dh_histo_async(dh_ctx *ctx, dh_stream stream, const double *d_coords, const int64_t *offsets,
                   int32_t n_species, int32_t box_type, const double *box, double r_max,
                   int32_t n_bins, int32_t precision, uint64_t *d_out, uint64_t *d_out_of_range) {
  return dh::histo_job(ctx, static_cast<hipStream_t>(stream), d_coords, offsets, n_species,
                       box_type, box, r_max, n_bins, precision, d_out, d_out_of_range, false,
                       nullptr);
}

}  // extern "C"

namespace dh {

int histo_job(dh_ctx *ctx, hipStream_t stream, const double *d_coords, const int64_t *offsets,
              int32_t n_species, int32_t box_type, const double *box, double r_max,
              int32_t n_bins, int32_t precision, uint64_t *d_out, uint64_t *d_out_of_range,
              bool accumulate, uint64_t *total_pairs, bool stepped) {
  if (!ctx) return DH_EINVAL;
  int rc = check(nullptr, offsets, n_species, box_type, box, r_max, n_bins, precision);
  if (rc) return fail(ctx, rc, "invalid arguments");
  const int64_t n = offsets[n_species];
  if (!d_out || (n > 0 && !d_coords)) return fail(ctx, DH_EINVAL, "null device pointer");
  hipStream_t st = static_cast<hipStream_t>(stream);
  DH_HIP(ctx, hipSetDevice(ctx->device));

  FrameJob job;
  job.d_coords = d_coords;
  job.offsets = offsets;
  job.n_species = n_species;
  job.precision = precision;
  job.d_out = d_out;
  job.d_oor = accumulate ? nullptr : d_out_of_range;
  job.accumulate = accumulate;
  job.kind = staged_kind(frame_consts(box_type, box, r_max, n_bins, job.fp), precision,
                         job.fp.L, n);
  job.fp.box = job.kind;
  for (int s = 0; s < n_species; ++s) {
    const uint64_t a = static_cast<uint64_t>(offsets[s + 1] - offsets[s]);
    job.total += a * (a > 0 ? a - 1 : 0) / 2;
    for (int t = s + 1; t < n_species; ++t)
      job.total += a * static_cast<uint64_t>(offsets[t + 1] - offsets[t]);
  }
  rc = ensure_device(ctx, &ctx->d_staged, &ctx->staged_cap,
                     std::max<size_t>(1, static_cast<size_t>(n)) *
                         staged_point_bytes(precision, job.kind));
  if (rc) return rc;

  Knobs k = default_knobs(precision);
  const std::string key = tune_key(ctx, job);
  if (ctx->forced) {
    k = Knobs::unpack(ctx->forced_knobs);
  } else if (ctx->tune_mode != DH_TUNE_OFF) {
    auto it = ctx->tune_cache.find(key);
    if (it != ctx->tune_cache.end()) {
      k = Knobs::unpack(it->second);
    } else if (ctx->tune_mode == DH_TUNE_ON && job.total > 0 && !accumulate && !stepped) {
      // (tuning overwrites the output, so accumulating calls never tune;
      // nor do stepped jobs, whose launches someone else paces)
      rc = tune_frame(ctx, st, job, key, k);
      if (rc) return rc;
    }
  }
  if (total_pairs) *total_pairs = job.total;

  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (stepped) {
    ctx->hold = true;
    rc = run_frame(ctx, st, job, k, true, nullptr, nullptr);
    ctx->hold = false;
    if (rc) ctx->held.clear();
    return rc;
  }
  if (ctx->profile) {
    if (ctx->prof_used == ctx->prof_events.size()) {
      hipEvent_t x, y;
      DH_HIP(ctx, hipEventCreate(&x));
      DH_HIP(ctx, hipEventCreate(&y));
      ctx->prof_events.emplace_back(x, y);
    }
    e0 = ctx->prof_events[ctx->prof_used].first;
    e1 = ctx->prof_events[ctx->prof_used].second;
    ++ctx->prof_used;
  }
  return run_frame(ctx, st, job, k, true, e0, e1);
}

int step_job(dh_ctx *ctx, hipStream_t st, uint64_t *pairs_left, bool *done) {
  *done = false;
  if (ctx->held_next < ctx->held.size()) {
    const dh_ctx::HeldLaunch &h = ctx->held[ctx->held_next++];
    ctx->held_left -= h.pairs;
    DH_HIP(ctx, launch_pairs(h.precision, h.kind, h.mode, h.cfg, h.args, h.grid, h.lds, st));
  } else {
    if (ctx->held_oor)
      DH_HIP(ctx, launch_oor(ctx->oor_hist, ctx->oor_n_hist, ctx->oor_n_bins, ctx->oor_pairs,
                             ctx->oor_out, st));
    ctx->held.clear();
    ctx->held_next = 0;
    ctx->held_oor = false;
    *done = true;
  }
  *pairs_left = ctx->held_left;
  return DH_OK;
}

uint64_t stepped_next_pairs(const dh_ctx *ctx) {
  return ctx->held_next < ctx->held.size() ? ctx->held[ctx->held_next].pairs : 0;
}

}  // namespace dh

extern "C" {

int dh_histo(const double *coords, const int64_t *offsets, int32_t n_species, int32_t box_type,
             const double *box, double r_max, int32_t n_bins, int32_t precision, uint64_t *out) {
  int rc = check(coords, offsets, n_species, box_type, box, r_max, n_bins, precision);
  if (rc) return rc;
  if (!out) return DH_EINVAL;
  const int64_t n = offsets[n_species];
  if (n > 0 && !coords) return DH_EINVAL;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return DH_EDEVICE;
  }
  dh_ctx *ctx = nullptr;
  {
    std::lock_guard<std::mutex> g(g_default_mu);
    auto it = g_default.find(dev);
    if (it == g_default.end()) {
      rc = dh_ctx_create(dev, 0, &ctx);
      if (rc) return rc;
      g_default[dev] = ctx;
    } else {
      ctx = it->second;
    }
  }
  std::lock_guard<std::mutex> g(ctx->mu);
  const int32_t n_hist = n_species * (n_species + 1) / 2;
  const size_t out_bytes = static_cast<size_t>(n_hist) * n_bins * sizeof(uint64_t);
  rc = ensure_device(ctx, reinterpret_cast<void **>(&ctx->d_in), &ctx->in_cap,
                     std::max<size_t>(1, static_cast<size_t>(n)) * 3 * sizeof(double));
  if (rc) return rc;
  rc = ensure_device(ctx, reinterpret_cast<void **>(&ctx->d_out), &ctx->out_cap, out_bytes);
  if (rc) return rc;
  hipStream_t st = ctx->own_stream;
  if (n > 0)
    DH_HIP(ctx, hipMemcpyAsync(ctx->d_in, coords, static_cast<size_t>(n) * 3 * sizeof(double),
                               hipMemcpyHostToDevice, st));
  rc = dh_histo_async(ctx, st, ctx->d_in, offsets, n_species, box_type, box, r_max, n_bins,
                      precision, ctx->d_out, nullptr);
  if (rc) return rc;
  DH_HIP(ctx, hipMemcpyAsync(out, ctx->d_out, out_bytes, hipMemcpyDeviceToHost, st));
  DH_HIP(ctx, hipStreamSynchronize(st));
  return DH_OK;
}

int dh_pair_t_async(dh_ctx *ctx, dh_stream stream, const double *d_coords, int64_t n,
                    int32_t box_type, const double *box, double r_max, int32_t n_bins,
                    int32_t precision, const int32_t *d_pi, const int32_t *d_pj, int64_t n_pairs,
                    double *d_t) {
  if (!ctx) return DH_EINVAL;
  const int64_t off[2] = {0, n};
  if (n < 1) return fail(ctx, DH_EINVAL, "n < 1");
  int rc = check(nullptr, off, 1, box_type, box, r_max, n_bins, precision);
  if (rc) return fail(ctx, rc, "invalid arguments");
  if (!d_coords || (n_pairs > 0 && (!d_pi || !d_pj || !d_t)) || n_pairs < 0)
    return fail(ctx, DH_EINVAL, "null device pointer");
  hipStream_t st = static_cast<hipStream_t>(stream);
  DH_HIP(ctx, hipSetDevice(ctx->device));
  FrameParams fp;
  int kind = frame_consts(box_type, box, r_max, n_bins, fp);
  if (precision == DH_FP32 && kind == kBoxOrtho && fp.L[0] == fp.L[1] && fp.L[1] == fp.L[2])
    fp.box = kind = kBoxCube;
  fp.win = n_bins;
  fp.n_sweeps = 1;
  rc = ensure_device(ctx, &ctx->d_staged, &ctx->staged_cap,
                     static_cast<size_t>(n) * coord_bytes(precision));
  if (rc) return rc;
  fp.coords = ctx->d_staged;
  const BlobLayout lay = blob_layout(1, 0, 0);
  rc = upload_blob(ctx, st, lay, std::vector<FrameParams>(1, fp), {}, {});
  if (rc) return rc;
  DH_HIP(ctx, launch_stage(precision, kind, d_coords, ctx->d_staged, n, fp, st));
  DH_HIP(ctx, launch_pair_t(precision, kind, static_cast<const FrameParams *>(ctx->d_blob), d_pi,
                            d_pj, n_pairs, static_cast<int32_t>(n), d_t, st));
  return DH_OK;
}

int dh_batch_create(dh_ctx *ctx, const dh_frame_desc *frames, int32_t n_frames, int32_t precision,
                    int32_t flags, dh_batch **out) {
  if (!ctx || !out) return DH_EINVAL;
  *out = nullptr;
  if (!frames || n_frames < 1 || n_frames > 65535)
    return fail(ctx, DH_EINVAL, "n_frames must be in 1..65535");
  if (precision != DH_FP32 && precision != DH_FP64) return fail(ctx, DH_EINVAL, "precision");
  struct FrameInfo {
    FrameParams fp;
    int mode = kModeLds;
    bool noclamp_ok = false;
    int64_t slots = 0;
    uint64_t pairs = 0;
    std::vector<int64_t> offsets;
    std::vector<uint64_t> hist_pairs;
  };
  std::vector<FrameInfo> info(n_frames);
  const Knobs bk = ctx->forced ? Knobs::unpack(ctx->forced_knobs) : default_knobs(precision);
  const BaseConfig base = base_config(ctx->lds_per_block, precision, bk, kBoxNone);
  for (int32_t f = 0; f < n_frames; ++f) {
    const dh_frame_desc &d = frames[f];
    int rc = check(nullptr, d.offsets, d.n_species, d.box_type, d.box, d.r_max, d.n_bins,
                   precision);
    if (rc) return fail(ctx, rc, "frame %d: invalid arguments", f);
    const int64_t n = d.offsets[d.n_species];
    if (!d.d_out || (n > 0 && !d.d_coords)) return fail(ctx, DH_EINVAL, "frame %d: null pointer", f);
    FrameInfo &fi = info[f];
    const int kind =
        staged_kind(frame_consts(d.box_type, d.box, d.r_max, d.n_bins, fi.fp), precision,
                    fi.fp.L, n);
    fi.fp.box = kind;
    fi.offsets.assign(d.offsets, d.offsets + d.n_species + 1);
    // the bin window that fits beside this kind's j-tiles
    const BaseConfig fbase = base_config(ctx->lds_per_block, precision, bk, kind);
    if (d.n_bins <= fbase.win_max) {
      fi.fp.win = d.n_bins;
      fi.fp.n_sweeps = 1;
    } else {
      fi.fp.n_sweeps = static_cast<int32_t>((d.n_bins + fbase.win_max - 1) / fbase.win_max);
      fi.fp.win = (d.n_bins + fi.fp.n_sweeps - 1) / fi.fp.n_sweeps;
      fi.mode = kModeSweep;
    }
    if (bk.wide > 0 && fi.fp.n_sweeps >= bk.wide) {
      fi.mode = kModeGlobal;
      fi.fp.win = d.n_bins;
      fi.fp.n_sweeps = 1;
    }
    const double tb = t_bound(fi.fp);
    if (fbase.noclamp && fi.mode == kModeLds && tb > 0) {
      fi.slots = static_cast<int64_t>(tb * (1.0 + 1e-4)) + 2;
      fi.noclamp_ok = fi.slots <= fbase.win_max + kDump;
    }
    fi.fp.n_points = n;
    fi.fp.n_hist = d.n_species * (d.n_species + 1) / 2;
    fi.fp.in = d.d_coords;
    fi.fp.out = d.d_out;
    fi.fp.oor = d.d_out_of_range;
  }

  dh_batch *b = new (std::nothrow) dh_batch;
  if (!b) return DH_ENOMEM;
  b->ctx = ctx;
  b->precision = precision;
  b->n_frames = n_frames;
  auto bail = [&](int rc) {
    dh_batch_destroy(b);
    return rc;
  };
  if (hipSetDevice(ctx->device) != hipSuccess) return bail(fail(ctx, DH_EDEVICE, "hipSetDevice"));

  // classes of frames that share one persistent launch
  std::map<std::pair<int, int>, std::vector<int32_t>> classes;
  for (int32_t f = 0; f < n_frames; ++f)
    classes[{info[f].fp.box, info[f].mode}].push_back(f);

  std::vector<WorkItem> items;
  std::vector<uint64_t> pairs;
  std::vector<size_t> pairs_base(n_frames, 0);
  for (auto &kv : classes) {
    std::vector<int32_t> &fs = kv.second;
    dh_batch::Group g;
    g.kind = kv.first.first;
    g.mode = kv.first.second;
    const BaseConfig gbase = base_config(ctx->lds_per_block, precision, bk, g.kind);
    g.cfg = gbase.cfg;
    int64_t stride = 0;
    uint64_t work = 0;
    for (int32_t f : fs) {
      FrameInfo &fi = info[f];
      if (g.mode != kModeGlobal) {
        int64_t need = fi.fp.win + kDump;
        if (fi.noclamp_ok) need = std::max<int64_t>(need, fi.slots);
        stride = std::max(stride, need);
      }
      for (int s = 0; s < frames[f].n_species; ++s) {
        const uint64_t a = static_cast<uint64_t>(fi.offsets[s + 1] - fi.offsets[s]);
        fi.pairs += a * (a > 0 ? a - 1 : 0) / 2;
        for (int t = s + 1; t < frames[f].n_species; ++t)
          fi.pairs += a * static_cast<uint64_t>(fi.offsets[t + 1] - fi.offsets[t]);
      }
      work += fi.pairs * static_cast<uint64_t>(fi.fp.n_sweeps);
    }
    for (int32_t f : fs) info[f].fp.noclamp = (info[f].noclamp_ok && info[f].slots <= stride) ? 1 : 0;
    g.stride = static_cast<int>(stride);
    g.lds = gbase.tile_bytes + static_cast<size_t>(g.cfg.copies) * g.stride * 4;
    resolve_threads(precision, g.kind, g.mode, bk, g.lds, g.cfg);
    g.grid = grid_for_config(ctx->n_cu, precision, g.kind, g.mode, gbase, g.lds, g.cfg);
    g.cfg.jchunk = jchunk_for(g.cfg, g.grid, work, gbase.items_per_wg);
    // large frames first: the tail of the work list is made of small items
    std::stable_sort(fs.begin(), fs.end(),
                     [&](int32_t x, int32_t y) { return info[x].pairs > info[y].pairs; });
    g.item_begin = items.size();
    Launch L;
    L.cfg = g.cfg;
    for (int32_t f : fs) {
      L.n_sweeps = info[f].fp.n_sweeps;
      pairs_base[f] = pairs.size();
      plan_frame(f, info[f].offsets.data(), frames[f].n_species, L, items, pairs);
    }
    g.item_count = items.size() - g.item_begin;
    b->groups.push_back(g);
    b->total_pairs += static_cast<double>(work);
  }
  b->n_items = static_cast<int64_t>(items.size());

  // staged coordinates
  std::vector<size_t> staged_off(n_frames);
  size_t staged_bytes = 0;
  for (int32_t f = 0; f < n_frames; ++f) {
    staged_off[f] = staged_bytes;
    staged_bytes += align_up(std::max<int64_t>(1, info[f].fp.n_points) *
                                 staged_point_bytes(precision, info[f].fp.box),
                             256);
    b->max_points = std::max(b->max_points, info[f].fp.n_points);
    b->max_words = std::max(b->max_words, static_cast<int64_t>(info[f].fp.n_hist) * frames[f].n_bins);
    b->max_hist = std::max(b->max_hist, info[f].fp.n_hist);
    b->any_oor = b->any_oor || frames[f].d_out_of_range != nullptr;
  }
  // blob: frames | items | pairs | counters
  b->off_frames = 0;
  b->off_items = align_up(n_frames * sizeof(FrameParams), 256);
  const size_t off_pairs = align_up(b->off_items + items.size() * sizeof(WorkItem), 256);
  b->off_counters = align_up(off_pairs + pairs.size() * sizeof(uint64_t), 256);
  const size_t blob_bytes = b->off_counters + align_up(b->groups.size() * sizeof(int32_t), 256);
  int64_t max_sorted = 0;
  for (int32_t f = 0; f < n_frames; ++f)
    if (info[f].fp.box == kBoxTricSorted) max_sorted = std::max(max_sorted, info[f].fp.n_points);
  const size_t keys_bytes =
      max_sorted > 0 ? static_cast<size_t>(sort_keys_count(max_sorted)) * 8 : 0;
  // the batch's buffers count against the context's budget while it lives
  const size_t own = staged_bytes + blob_bytes + keys_bytes;
  if (ctx->budget) {
    const size_t held = ctx_device_bytes(ctx) + ctx->batch_bytes;
    if (held > ctx->budget || own > ctx->budget - held)
      return bail(fail(ctx, DH_EBUDGET,
                       "the batch needs %zu bytes of device memory beside the %zu held; "
                       "budget %zu bytes",
                       own, held, ctx->budget));
  }
  if (hipMalloc(&b->d_staged, staged_bytes) != hipSuccess) {
    (void)hipGetLastError();
    b->d_staged = nullptr;
    return bail(fail(ctx, DH_ENOMEM, "hipMalloc of %zu bytes failed", staged_bytes));
  }
  if (hipMalloc(&b->d_blob, blob_bytes) != hipSuccess) {
    (void)hipGetLastError();
    b->d_blob = nullptr;
    return bail(fail(ctx, DH_ENOMEM, "hipMalloc of %zu bytes failed", blob_bytes));
  }
  char *db = static_cast<char *>(b->d_blob);
  std::vector<char> host(blob_bytes, 0);
  for (int32_t f = 0; f < n_frames; ++f) {
    FrameParams fp = info[f].fp;
    fp.coords = static_cast<char *>(b->d_staged) + staged_off[f];
    fp.pairs = reinterpret_cast<const uint64_t *>(db + off_pairs) + pairs_base[f];
    std::memcpy(host.data() + b->off_frames + f * sizeof(FrameParams), &fp, sizeof fp);
    if (fp.box == kBoxTricSorted)
      b->sorted.push_back({f, frames[f].d_coords, const_cast<void *>(fp.coords),
                           info[f].offsets, fp});
  }
  if (keys_bytes > 0 && hipMalloc(&b->d_keys, keys_bytes) != hipSuccess) {
    (void)hipGetLastError();
    b->d_keys = nullptr;
    return bail(fail(ctx, DH_ENOMEM, "hipMalloc of the sort keys failed"));
  }
  b->budget_bytes = own;
  ctx->batch_bytes += own;
  if (!items.empty())
    std::memcpy(host.data() + b->off_items, items.data(), items.size() * sizeof(WorkItem));
  if (!pairs.empty())
    std::memcpy(host.data() + off_pairs, pairs.data(), pairs.size() * sizeof(uint64_t));
  if (hipMemcpy(b->d_blob, host.data(), blob_bytes, hipMemcpyHostToDevice) != hipSuccess)
    return bail(fail(ctx, DH_EDEVICE, "hipMemcpy of the batch plan failed"));

  if (flags & DH_BATCH_GRAPH) {
    hipStream_t cs = nullptr;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess)
      return bail(fail(ctx, DH_EDEVICE, "hipStreamCreate failed"));
    int rc = DH_OK;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      rc = fail(ctx, DH_EDEVICE, "hipStreamBeginCapture failed");
    } else {
      int erc = dh_batch_launch_direct(b, cs);
      hipGraph_t graph = nullptr;
      hipError_t e = hipStreamEndCapture(cs, &graph);
      if (erc) rc = erc;
      else if (e != hipSuccess) rc = fail(ctx, DH_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
      b->graph = graph;
      if (!rc && hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess)
        rc = fail(ctx, DH_EDEVICE, "hipGraphInstantiate failed");
    }
    (void)hipStreamDestroy(cs);
    (void)hipGetLastError();
    if (rc) return bail(rc);
  }
  *out = b;
  return DH_OK;
}

int dh_batch_launch(dh_batch *b, dh_stream stream) {
  if (!b) return DH_EINVAL;
  dh_ctx *ctx = b->ctx;
  DH_HIP(ctx, hipSetDevice(ctx->device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (b->exec) {
    DH_HIP(ctx, hipGraphLaunch(b->exec, st));
    return DH_OK;
  }
  return dh_batch_launch_direct(b, st);
}

int dh_batch_info(const dh_batch *b, int64_t *n_items, int32_t *n_launches, double *total_pairs) {
  if (!b) return DH_EINVAL;
  if (n_items) *n_items = b->n_items;
  if (n_launches) *n_launches = static_cast<int32_t>(b->groups.size());
  if (total_pairs) *total_pairs = b->total_pairs;
  return DH_OK;
}

void dh_batch_destroy(dh_batch *b) {
  if (!b) return;
  if (b->ctx && hipSetDevice(b->ctx->device) == hipSuccess) {
    (void)hipDeviceSynchronize();
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->d_staged) (void)hipFree(b->d_staged);
    if (b->d_blob) (void)hipFree(b->d_blob);
    if (b->d_keys) (void)hipFree(b->d_keys);
  }
  if (b->ctx) b->ctx->batch_bytes -= b->budget_bytes;
  (void)hipGetLastError();
  delete b;
}

int dh_ctx_set_tuning(dh_ctx *ctx, int32_t mode, const char *cache_path) {
  if (!ctx || mode < DH_TUNE_OFF || mode > DH_TUNE_ON) return DH_EINVAL;
  ctx->tune_mode = mode;
  if (cache_path) {
    ctx->tune_path = cache_path;
    return load_tune_cache(ctx);
  }
  return DH_OK;
}

int dh_ctx_set_config(dh_ctx *ctx, const int32_t *knobs) {
  if (!ctx) return DH_EINVAL;
  if (!knobs) {
    ctx->forced = false;
    return DH_OK;
  }
  std::array<int32_t, kNumKnobs> v;
  for (int q = 0; q < kNumKnobs; ++q) v[q] = knobs[q];
  if (!Knobs::unpack(v).valid()) return fail(ctx, DH_EINVAL, "invalid launch knobs");
  ctx->forced = true;
  ctx->forced_knobs = v;
  return DH_OK;
}

int dh_ctx_last_config(const dh_ctx *ctx, int32_t *out) {
  if (!ctx || !out) return DH_EINVAL;
  for (int q = 0; q < 13; ++q) out[q] = ctx->last_config[q];
  return DH_OK;
}

int dh_ctx_set_launch_pairs(dh_ctx *ctx, int64_t max_pairs) {
  if (!ctx || max_pairs < 0) return DH_EINVAL;
  if (max_pairs > 0 && max_pairs < (int64_t{1} << 24))
    return fail(ctx, DH_EINVAL, "max_pairs must be 0 or at least 2^24");
  ctx->launch_pairs = static_cast<uint64_t>(max_pairs);
  return DH_OK;
}

int dh_ctx_searched_pairs(dh_ctx *ctx, uint64_t *searched) {
  if (!ctx || !searched) return DH_EINVAL;
  *searched = 0;
  if (!ctx->searched_dev) return DH_OK;
  DH_HIP(ctx, hipSetDevice(ctx->device));
  unsigned long long v = 0;
  DH_HIP(ctx, hipMemcpy(&v, ctx->searched_dev, sizeof v, hipMemcpyDeviceToHost));
  *searched = v;
  return DH_OK;
}

int dh_ctx_searched_images(dh_ctx *ctx, uint64_t *images) {
  if (!ctx || !images) return DH_EINVAL;
  *images = 0;
  if (!ctx->searched_dev) return DH_OK;
  DH_HIP(ctx, hipSetDevice(ctx->device));
  unsigned long long v = 0;
  DH_HIP(ctx, hipMemcpy(&v, ctx->searched_dev + 1, sizeof v, hipMemcpyDeviceToHost));
  *images = v;
  return DH_OK;
}

int dh_ctx_profile(dh_ctx *ctx, int32_t enable) {
  if (!ctx) return DH_EINVAL;
  ctx->profile = enable != 0;
  ctx->prof_used = 0;
  return DH_OK;
}

int dh_ctx_profile_read(dh_ctx *ctx, double *kernel_ms, int64_t *launches) {
  if (!ctx || !kernel_ms || !launches) return DH_EINVAL;
  DH_HIP(ctx, hipSetDevice(ctx->device));
  double total = 0.0;
  for (size_t k = 0; k < ctx->prof_used; ++k) {
    DH_HIP(ctx, hipEventSynchronize(ctx->prof_events[k].second));
    float ms = 0.f;
    DH_HIP(ctx, hipEventElapsedTime(&ms, ctx->prof_events[k].first, ctx->prof_events[k].second));
    total += ms;
  }
  *kernel_ms = total;
  *launches = static_cast<int64_t>(ctx->prof_used);
  ctx->prof_used = 0;
  return DH_OK;
}

}  // extern "C"
