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
};

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
constexpr int kDump = 64;  // per-lane discard slots after the bin window
// Per-wave LDS ring of reduced vectors waiting for the 27-image search:
// one j adds at most 64 per i-particle of a lane (R) on top of fewer than 64.
constexpr int queue_cap(int r) { return 64 * (r + 1); }

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
};

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

// host-side launchers (dh_kernels.hip)
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
