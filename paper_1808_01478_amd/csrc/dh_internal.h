// Internal types shared by the host planner and the gfx950 kernels of
// libdisthist. Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace dh {

enum BoxKind : int32_t {
  kBoxNone = 0,
  kBoxOrtho = 1,
  kBoxTric = 2,        // Eq. 5 reduction only (r_max below half the smallest width)
  kBoxTricSearch = 3,  // Eq. 5 reduction, then the 27 neighbouring images
  kBoxCube = 4,        // binary32 only: orthorhombic cell with equal edges
  // Eq. 5 reduction only, points spatially sorted within each species at
  // staging (frames of at least kSortMinPoints; see staged_kind)
  kBoxTricSorted = 5,
};

// Largest species count of a frame (the staging kernels take the offsets by
// value).
constexpr int kMaxSpeciesStage = 64;
// frames with at least this many points may be staged in spatial order
// (kBoxTricSorted, see staged_kind)
constexpr int64_t kSortMinPoints = int64_t{1} << 16;

// The minimum-image kind the kernels use for a frame: the geometric kind of
// frame_constants, with large frames staged in spatial order (triclinic
// frames in both precisions; orthorhombic ones in binary64, where the sorted
// kernel with a diagonal cell matrix gives the orthorhombic sequence's
// counts bit for bit) and the binary32 special case of equal orthorhombic
// edges.
inline int staged_kind(int kind, int precision, const double L[3], int64_t n_points) {
  if (n_points >= kSortMinPoints &&
      (kind == kBoxTric || (kind == kBoxOrtho && precision != 0)))
    return kBoxTricSorted;
  if (precision != 0) return kind;
  if (kind == kBoxOrtho && L[0] == L[1] && L[1] == L[2]) return kBoxCube;
  return kind;
}

// Bytes per staged point (binary64 double4; binary32 float4, two of them
// for spatially sorted frames) and the sort workspace of a frame.
inline size_t staged_point_bytes(int precision, int kind) {
  return precision != 0 ? 32 : (kind == kBoxTricSorted ? 32 : 16);
}
inline int64_t sort_keys_count(int64_t n) {
  int64_t p = 2048;
  while (p < n) p <<= 1;
  return p;
}

// How a pair kernel accumulates its counts.
enum HistMode : int32_t {
  kModeLds = 0,     // the whole histogram in LDS sub-histograms
  kModeSweep = 1,   // LDS sub-histograms of one bin window per item
  kModeGlobal = 2,  // uint64 atomics straight into the output (wide histograms)
};

// WorkItem::flags
constexpr int32_t kItemDiag = 1;  // i- and j-range are the same block: count j > i only
constexpr int32_t kItemFull = 2;  // every lane holds a valid i-particle

constexpr int kShifts = 27;
// index of the zero shift (i = j = k = 0) in the shift tables
constexpr int kZeroShift = 13;
// the image search keeps at most kOctCap images per octant of a reduced
// vector (octants that need more search all 27)
constexpr int kOctCap = 12;
// the search's LDS table: 8 octant rows of kOctCap shift vectors, then the
// 27 shift vectors (the full list)
constexpr int kSearchTable = 8 * kOctCap + kShifts;
// slack e of the octant boxes in fractional coordinates (see octant_images)
constexpr double kOctSlack = 0x1p-30;
constexpr int kDump = 64;  // per-lane discard slots after the bin window
// Per-wave LDS ring of reduced vectors waiting for the 27-image search: the
// wave searches 64 of them as soon as 64 are queued, after each slice of
// pairs, so a slice adds at most 64 on top of fewer than 64 (the same for
// every number of slices r).
constexpr int queue_cap(int /* slices per lane */) { return 128; }

// Constants of one frame, computed once on the host.
//
// binary64 members follow the canonical op sequence: s = n_bins / r_max,
// iL = 1 / L, and the inverse of the upper-triangular cell matrix
//   h11 = 1/ax, h22 = 1/by, h33 = 1/cz, h12 = -bx/(ax*by),
//   h23 = -cy/(by*cz), h13 = (bx*cy - by*cx)/(ax*by*cz),
// with shifts S = i*a + j*b + k*c for i, j, k in {-1, 0, 1}.
//
// binary32 members serve the reduced-precision path. Without a box the
// coordinates are staged pre-scaled by s. With a periodic cell they are
// staged as 32-bit fixed-point fractional coordinates u = 2^32 * (f mod 1),
// f = B^-1 x: the wrapped difference u_j - u_i read as a signed integer is
// 2^32 * (f_j - f_i - nint(f_j - f_i)), the reduced vector of Eq. 5 in
// fractional form, and the cell matrix scaled by s / 2^32 maps it to t units.
struct FrameParams {
  const void *coords;  // staged float4 / double4 [N] (device)
  uint64_t *out;       // [H][n_bins] (device)
  const double *in;    // caller's binary64 [N][3] (device)
  uint64_t *oor;       // caller's out-of-range counts [H] or null (device)
  const uint64_t *pairs;  // pairs per histogram [H] (device)
  int64_t n_points;
  int32_t n_hist;
  int32_t oor_by_flush;  // 1: oor starts at pairs and every flush subtracts its counts
  int32_t n_bins;
  int32_t box;         // BoxKind
  int32_t win;         // bin window of one sweep (<= n_bins)
  int32_t n_sweeps;
  double s;
  double L[3], iL[3];
  double ax, bx, by, cx, cy, cz;
  double h11, h12, h13, h22, h23, h33;
  double shift64[kShifts][3];
  float k32[3];        // orthorhombic: L_c * s / 2^32 (cube: k32[0])
  float ryz32[2];      // orthorhombic: (L_y / L_x)^2, (L_z / L_x)^2
  float Bk[6];         // ax bx by cx cy cz, times s / 2^32
  float Bn[5];         // bx by cx cy cz divided by ax
  float shift32[kShifts][3];  // image shifts times s
  int32_t noclamp;     // 1: every t of a full block fits below `stride` slots
  float qskip32;       // binary32 q (t units) below which no image is nearer
  double qskip64;      // binary64 q below which the reduced vector is nearest
  // image search: pairs that went through the image search are added to
  // searched[0], the images evaluated for them to searched[1] (device,
  // 8-byte aligned) unless null
  unsigned long long *searched;
  // spatially sorted binary32 frames: the cell rows (ax bx by cx cy cz), the
  // entries of B^-1 (h11 h12 h13 h22 h23 h33) and s = n_bins / r_max,
  // rounded to binary32
  float cell32[6];
  float hinv32[6];
  float s32;
  // spatially sorted binary32 frames: the lattice shift B n for the wraps
  // n_k = +1 (bit k of q), -1 (bit 3 + k) or 0, in binary32 as
  // (n_a a_x + n_b b_x) + n_c c_x, n_b b_y + n_c c_y, n_c c_z (w unused)
  alignas(16) float gshift32[64][4];
  // image search: for each octant of a reduced vector's fractional
  // coordinates (bit k set when component k is negative) the images that
  // can be nearer than the vector itself, as indices into the shift tables
  // padded with the zero shift (kZeroShift); oct_full bit o when octant o
  // needs more than kOctCap images (it searches all 27); oct_n the longest
  // of the other lists
  uint8_t oct_shift[8][kOctCap];
  uint8_t oct_full;
  uint8_t oct_n;
};

// LDS of a spatially sorted frame's pair kernel besides its two j-tiles:
// the bounding boxes of the tiles' groups of 64 points (two tiles, at most
// four groups each, eight words per box: 32-bit fixed-point fractions in
// binary32, binary64 fractions in binary64)
constexpr size_t kSortedBoxBytes = 2 * 4 * 8 * sizeof(double);

// One unit of work: particles [i0, i1) of the frame against [j0, j1), for
// histogram `hist`, bin window `sweep`; flags: kItemDiag, kItemFull.
struct WorkItem {
  int32_t frame, hist, sweep, flags;
  int32_t i0, i1, j0, j1;
};

struct PairKernelArgs {
  const FrameParams *frames;
  const WorkItem *items;
  int32_t *counter;  // dynamic work counter, zero before launch
  int32_t n_items;
  int32_t copies;    // interleaved LDS sub-histogram copies (1, 2 or 4)
  int32_t stride;    // slots per copy (>= win + kDump of every frame); 0 in kModeGlobal
  int32_t tj;        // j-tile length staged through LDS
};

// Kernel configuration (chosen per launch by the tuner).
struct KernelConfig {
  int32_t threads;   // workgroup size: 256, 512 or 1024
  int32_t r;         // i-particles per lane (4 or 8)
  int32_t copies;    // interleaved sub-histogram copies (1, 2, 4)
  int32_t tj;        // j-tile length (<= threads)
  int32_t jchunk;    // j-range of one work item (multiple of tj)
  int32_t wg_per_cu; // 0 = as many as fit
};

// Species pair (s, t) of histogram h among k species, in the library order:
// (0,0), (1,1), ..., (k-1,k-1), then (s,t) for s < t lexicographically.
__host__ __device__ inline void hist_pair(int32_t k, int32_t h, int32_t &s, int32_t &t) {
  s = t = h;
  if (h < k) return;
  int32_t idx = h - k;
  for (s = 0; s < k; ++s) {
    const int32_t m = k - 1 - s;
    if (idx < m) {
      t = s + 1 + idx;
      return;
    }
    idx -= m;
  }
}

// How the work list of one histogram is cut (the host planner and the
// device planner of the allocation-free entry point emit the same items):
// rows are blocks of bi particles in the lanes; an intra-species row has a
// diagonal item (when its block holds at least two particles) followed by
// j-chunks of at most jc particles from the end of its block to the end of
// the species; a cross-species row puts the larger species in the lanes and
// streams the smaller one in j-chunks.
struct HistRows {
  int64_t lane0, lane1;  // particles in the lanes
  int64_t str0, str1;    // particles streamed as j (cross-species)
  bool intra;
  uint64_t pairs;        // pairs of the histogram
};

__host__ __device__ inline HistRows hist_rows(const int64_t *off, int32_t k, int32_t h) {
  int32_t s, t;
  hist_pair(k, h, s, t);
  HistRows r;
  const int64_t ns = off[s + 1] - off[s], nt = off[t + 1] - off[t];
  r.intra = s == t;
  if (r.intra) {
    r.lane0 = r.str0 = off[s];
    r.lane1 = r.str1 = off[s + 1];
    r.pairs = static_cast<uint64_t>(ns) * static_cast<uint64_t>(ns > 0 ? ns - 1 : 0) / 2;
  } else {
    const int32_t si = ns >= nt ? s : t, sj = ns >= nt ? t : s;
    r.lane0 = off[si]; r.lane1 = off[si + 1];
    r.str0 = off[sj]; r.str1 = off[sj + 1];
    r.pairs = static_cast<uint64_t>(ns) * static_cast<uint64_t>(nt);
  }
  return r;
}

__host__ __device__ inline int64_t hist_row_count(const HistRows &r, int64_t bi) {
  return (r.lane1 - r.lane0 + bi - 1) / bi;
}

__host__ __device__ inline int64_t row_item_count(const HistRows &r, int64_t row, int64_t bi,
                                                  int64_t jc) {
  const int64_t b0 = r.lane0 + row * bi;
  const int64_t b1 = b0 + bi < r.lane1 ? b0 + bi : r.lane1;
  if (r.intra) return (b1 - b0 >= 2 ? 1 : 0) + (r.lane1 - b1 + jc - 1) / jc;
  return (r.str1 - r.str0 + jc - 1) / jc;
}

// Writes the items of one row (for bin window `sweep`) from dst on; returns
// how many. Flags as in WorkItem.
__host__ __device__ inline int64_t emit_row(const HistRows &r, int32_t h, int32_t sweep,
                                            int64_t row, int64_t bi, int64_t jc,
                                            WorkItem *dst) {
  const int64_t b0 = r.lane0 + row * bi;
  const int64_t b1 = b0 + bi < r.lane1 ? b0 + bi : r.lane1;
  const int32_t full = b1 - b0 == bi ? kItemFull : 0;
  int64_t n = 0;
  auto put = [&](int64_t j0, int64_t j1, int32_t diag) {
    WorkItem w;
    w.frame = 0; w.hist = h; w.sweep = sweep; w.flags = diag | full;
    w.i0 = static_cast<int32_t>(b0); w.i1 = static_cast<int32_t>(b1);
    w.j0 = static_cast<int32_t>(j0); w.j1 = static_cast<int32_t>(j1);
    dst[n++] = w;
  };
  if (r.intra) {
    if (b1 - b0 >= 2) put(b0, b1, kItemDiag);
    for (int64_t j = b1; j < r.lane1; j += jc) put(j, j + jc < r.lane1 ? j + jc : r.lane1, 0);
  } else {
    for (int64_t j = r.str0; j < r.str1; j += jc) put(j, j + jc < r.str1 ? j + jc : r.str1, 0);
  }
  return n;
}

// host-side launchers (dh_kernels.hip)
// Staging of a kBoxTricSorted frame: the points of every species in Morton
// order of their wrapped fractional coordinates (keys: a workspace of
// sort_keys_count(n) words); binary32: two float4 per point in `out`,
// binary64: the input coordinates as one double4 per point.
hipError_t launch_stage_sorted(int precision, const double *in, void *out, int64_t n,
                               const int64_t *offsets, int32_t n_species, const FrameParams &fp,
                               uint64_t *keys, hipStream_t st);
hipError_t launch_stage(int precision, int box_kind, const double *in, void *out, int64_t n,
                        const FrameParams &fp, hipStream_t st);
// zeroes out[n_words] and counters[n_counters]; with oor, sets oor[h] =
// pairs[h] for h < n_hist (the flushes then subtract the in-range counts)
hipError_t launch_zero(uint64_t *out, int64_t n_words, int32_t *counters, int32_t n_counters,
                       uint64_t *oor, const uint64_t *pairs, int32_t n_hist, hipStream_t st);
hipError_t launch_pairs(int precision, int box_kind, int mode, const KernelConfig &cfg,
                        const PairKernelArgs &args, int grid, size_t lds_bytes, hipStream_t st);
hipError_t launch_oor(const uint64_t *hist, int32_t n_hist, int32_t n_bins, const uint64_t *pairs,
                      uint64_t *oor, hipStream_t st);
// batched staging / zeroing / out-of-range over a device table of frames
hipError_t launch_stage_batch(int precision, const FrameParams *d_frames, int32_t n_frames,
                              int64_t max_points, hipStream_t st);
hipError_t launch_zero_batch(const FrameParams *d_frames, int32_t n_frames, int64_t max_words,
                             int32_t *counters, int32_t n_counters, hipStream_t st);
hipError_t launch_oor_batch(const FrameParams *d_frames, int32_t n_frames, int32_t max_hist,
                            hipStream_t st);
hipError_t launch_pair_t(int precision, int box_kind, const FrameParams *d_fp, const int32_t *pi,
                         const int32_t *pj, int64_t n_pairs, int32_t n, double *t,
                         hipStream_t st);
// Occupancy of the pair kernel (workgroups per CU) for a config and LDS size.
int pairs_occupancy(int precision, int box_kind, int mode, const KernelConfig &cfg,
                    size_t lds_bytes);

}  // namespace dh

struct dh_ctx;
namespace dh {
// device bytes held by a context's scratch (staged coordinates, work blob)
size_t ctx_device_bytes(const dh_ctx *ctx);
// frees a context's scratch (the context must be idle); it regrows on use
void ctx_release_scratch(dh_ctx *ctx);
// device footprint of a single-frame job besides the caller's buffers
// (launch_pairs: the bounded launch size the job runs with, 0 = one launch)
size_t job_scratch_bytes(int64_t n_points, int32_t n_hist, int32_t n_bins, int32_t precision,
                         int64_t launch_pairs);
// binary64 constants of a frame (s, inverse cell, shifts, box kind; returns
// the kind: none, ortho, triclinic, triclinic with image search)
int frame_constants(int32_t box_type, const double *box, double r_max, int32_t n_bins,
                    FrameParams &fp);
// device ordinal of a context
int ctx_device(const dh_ctx *ctx);
// The launch shape a frame gets with the built-in default knobs (no tuning
// cache) on a device with n_cu compute units and lds_per_block bytes of LDS
// per workgroup; fp comes from frame_constants (box kind, n_bins).
struct LaunchPlan {
  KernelConfig cfg;
  int32_t mode, win, n_sweeps, stride, grid;
  bool noclamp;
  size_t lds;
};
LaunchPlan default_launch(int n_cu, size_t lds_per_block, int precision, const FrameParams &fp,
                          uint64_t total_pairs);
// The same with a given workgroup size (0 = automatic): launches that mix
// frames need one shape for all of them.
LaunchPlan serve_launch(int n_cu, size_t lds_per_block, int precision, const FrameParams &fp,
                        uint64_t total_pairs, int threads);
// Records the message of a failure that has no context (read back by
// dh_ctx_last_error(NULL); a fixed thread-local buffer, so it allocates
// nothing) and returns code.
int thread_fail(int code, const char *fmt, ...);
// zeroes n words with a kernel on stream st (never a memset node in graphs)
int zero_u64(uint64_t *p, int64_t n, hipStream_t st);
// dh_histo_async with an accumulate option: when set, the frame's counts are
// added into d_out (not zeroed first) and no out-of-range counts are written;
// total_pairs (optional) receives the frame's pair count.
int histo_job(dh_ctx *ctx, hipStream_t stream, const double *d_coords, const int64_t *offsets,
              int32_t n_species, int32_t box_type, const double *box, double r_max,
              int32_t n_bins, int32_t precision, uint64_t *d_out, uint64_t *d_out_of_range,
              bool accumulate, uint64_t *total_pairs, bool stepped = false);
// A stepped job (histo_job with stepped set) enqueues staging and zeroing
// only and holds its pair-kernel launches back in the context; step_job
// enqueues the next one on st, or, when none is left, the closing
// out-of-range pass if the job needs one (*done then becomes true). *pairs_left receives the
// pairs of the launches still held back. The context runs nothing else
// until the job is done.
int step_job(dh_ctx *ctx, hipStream_t st, uint64_t *pairs_left, bool *done);
// pairs of a stepped job's next held-back launch (0: the closing pass is next)
uint64_t stepped_next_pairs(const dh_ctx *ctx);
}  // namespace dh
